// column1d.h -- the complete 1D lattice update of one spatial site, held
// by one lane (gfx950): used by the single-lattice and the batched passes.
#pragma once

#include "device_common.h"

namespace lat {

// The whole 1D update of one site x (one lane): pull the velocity column,
// nsub x [drift, diffusion] in registers, store.  alpha = dt_s u(x) /
// (dv tau_p) is the drift of the zero-velocity cell in cell widths.  Plane
// j starts pitch elements after plane j-1 (pitch >= nx).
template <typename T, int CAP, bool KOREN>
__device__ __forceinline__ void column1d(const T* __restrict__ fin,
                                         T* __restrict__ fout, int x, int nx,
                                         int pitch, int nv, int h,
                                         int step_mod,
                                         int init_off, int nsub, T alpha,
                                         T beta, T D) {
  // ---- 1. pull streaming: source site of cell j is (x - shift*(j-h)) mod nx
  T c[CAP];
  int xs = x + init_off;  // (x + shift*h) mod nx
  if (xs >= nx) xs -= nx;
#pragma unroll
  for (int j = 0; j < CAP; ++j) {
    if (j < nv) {
      c[j] = fin[(size_t)j * pitch + xs];
      xs -= step_mod;
      if (xs < 0) xs += nx;
    } else {
      c[j] = T(0);
    }
  }

  for (int sub = 0; sub < nsub; ++sub) {
    // ---- 2a. drift: split fluxes g+ = max(nu,0) c, g- = min(nu,0) c with
    // nu_j = alpha - beta*(j-h).  Faces k = 1..nv-1 (cells k-1 | k) are
    // visited in order with a sliding window of g values, and cell k-1 is
    // updated as soon as its right face is known; faces 0 and nv carry no
    // flux, cells past nv are empty.
    T gpm2 = T(0), gpm1, gpk, gmm1, gmk, gmp1;
    {
      const T nu0 = alpha - beta * (T)(0 - h);
      gpm1 = pos(nu0) * c[0];
      gmm1 = neg(nu0) * c[0];
      const T nu1 = alpha - beta * (T)(1 - h);
      gpk = pos(nu1) * c[1];
      gmk = neg(nu1) * c[1];
    }
    T Fprev = T(0);  // face k-1
#pragma unroll
    for (int k = 1; k <= CAP; ++k) {
      T cnext = T(0);
      if (k + 1 < CAP) cnext = c[k + 1];
      const T nun = alpha - beta * (T)(k + 1 - h);
      gmp1 = neg(nun) * cnext;
      const T gpn = pos(nun) * cnext;
      T fl = gpm1 + gmk;
      if (KOREN)
        fl += koren(gpk - gpm1, gpm1 - gpm2) + koren(gmm1 - gmk, gmk - gmp1);
      fl = (k < nv) ? fl : T(0);  // face nv and beyond: zero flux
      c[k - 1] = c[k - 1] - (fl - Fprev);
      Fprev = fl;
      gpm2 = gpm1;
      gpm1 = gpk;
      gpk = gpn;
      gmm1 = gmk;
      gmk = gmp1;
    }

    // ---- 2b. diffusion: face flux D (c_{k-1} - c_k), k = 1..nv-1
    T dprev = T(0);
    T cprev = c[0];
#pragma unroll
    for (int k = 1; k <= CAP; ++k) {
      const T ck = k < CAP ? c[k] : T(0);
      const T del = (k < nv) ? (cprev - ck) : T(0);
      c[k - 1] = cprev + D * (dprev - del);
      dprev = del;
      cprev = ck;
    }
  }

  // ---- 3. store
#pragma unroll
  for (int j = 0; j < CAP; ++j)
    if (j < nv) fout[(size_t)j * pitch + x] = c[j];
}


}  // namespace lat
