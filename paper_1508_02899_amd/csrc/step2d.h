// step2d.h -- fused streaming + collision pass for 2D lattices (gfx950).
//
// Layout: f[jy*NV + jx][y][x], x fastest.  One wavefront owns S = 64/P
// consecutive sites of one spatial row y; each site's vx axis is split over
// P lanes ("parts"), part p holding the W = ceil(NV/P) slots jx = p*W + i.
// The kernel streams over the vy index (rows jy = 0..NV-1), carrying a few
// rows of state in registers, so that every state element is read once and
// written once per pass and every load/store is a coalesced run of S
// consecutive sites of one velocity plane:
//
//   for each row t = jy:
//     load row t, pulled from the source sites (x - s(jx-h), y - s(t-h))
//       [Sec. 2 exact streaming];
//     A_x: drift along vx inside the row (split upwind fluxes, Koren
//       correction; 2 halo cells per side from the neighbouring parts);
//     A_y: drift along vy, streamed: face t-1 is complete once row t is in,
//       giving the A_y output of row t-2;
//     D_x: diffusion along vx on that row (1 halo cell per side);
//     D_y: diffusion along vy, streamed, giving the final row t-3;
//     store row t-3.
//
// The per-site order A_x, A_y, D_x, D_y is the paper's "force, then
// diffusion" split by velocity axis.  Zero flux through the outer faces of
// the velocity square; cells outside it are empty for the limiter.
#pragma once

#include "device_common.h"
#include "lattice_internal.h"

namespace lat {

template <typename T, int NV, int P, bool KOREN>
__global__ __launch_bounds__(256) void k_step2d(
    const T* __restrict__ fin, T* __restrict__ fout, const T* __restrict__ u,
    const int* __restrict__ flag, int nx, int ny, int xstep, int xoff0,
    int ystep, int yoff0, T alpha_scale, T beta, T D, int ntx, int ntiles,
    int nblocks) {
  constexpr int W = (NV + P - 1) / P;  // slots per lane
  constexpr int S = 64 / P;            // sites per wavefront
  constexpr int H = (NV - 1) / 2;
  constexpr int FB = NV - (P - 1) * W;  // slot of face NV in the last part
  static_assert(FB >= 1 && FB <= W, "bad split");

  if (*flag != 0) return;
  const int lane = (int)threadIdx.x & 63;
  const int tile = xcd_remap(blockIdx.x, nblocks) * 4 + ((int)threadIdx.x >> 6);
  if (tile >= ntiles) return;  // whole wavefront idle
  const int p = lane / S;
  const int y = tile / ntx;
  int x = (tile - y * ntx) * S + (lane - p * S);
  const bool active = x < nx;
  if (!active) x = nx - 1;  // duplicate a real site; never stored
  const bool first = p == 0, last = p == P - 1;
  const int lane_l = lane - S, lane_r = lane + S;

  const size_t nxy = (size_t)nx * (size_t)ny;
  const size_t rowpitch = (size_t)NV * nxy;  // elements between vy rows
  const T ax = u[(size_t)y * nx + x] * alpha_scale;
  const T ay = u[nxy + (size_t)y * nx + x] * alpha_scale;

  // element offset of slot i inside one vy row: plane jx, site (y', xs_i);
  // xs_i = (x - shift*(jx - H)) mod nx
  uint32_t koff[W];
  {
    int xs = x + xoff0;  // jx = 0: (x + shift*H) mod nx
    if (xs >= nx) xs -= nx;
    for (int k = 0; k < p * W; ++k) {  // advance to jx = p*W
      xs -= xstep;
      if (xs < 0) xs += nx;
    }
#pragma unroll
    for (int i = 0; i < W; ++i) {
      koff[i] = (uint32_t)((size_t)(p * W + i) * nxy + (size_t)xs);
      xs -= xstep;
      if (xs < 0) xs += nx;
    }
  }
  bool valid[W];
#pragma unroll
  for (int i = 0; i < W; ++i) valid[i] = (p * W + i) < NV;

  // vx drift of slot i (i = -2 .. W+1 at index i+2), cell widths per step
  T nxp[W + 4], nxm[W + 4];
#pragma unroll
  for (int i = 0; i < W + 4; ++i) {
    const T nu = ax - beta * (T)(p * W + i - 2 - H);
    nxp[i] = pos(nu);
    nxm[i] = neg(nu);
  }

  // streamed vy state (per slot): g+ / g- of the previous row and their
  // last differences, the previous face's g+ flux, the running A_y output
  // accumulator and the previous x-passed row; then the D_y state.
  T gp1[W], dpp1[W], gm1[W], em1[W], Fp1[W], acc2[W], c1[W], a3[W], del3[W];
#pragma unroll
  for (int i = 0; i < W; ++i) {
    gp1[i] = dpp1[i] = gm1[i] = em1[i] = Fp1[i] = acc2[i] = c1[i] = a3[i] =
        del3[i] = T(0);
  }

  int ys = y + yoff0;  // row t = 0 comes from (y + shift*H) mod ny
  if (ys >= ny) ys -= ny;
  const T* frow = fin;
  T* orow = fout + (size_t)y * nx + x;

#pragma unroll 1
  for (int t = 0; t < NV + 3; ++t) {
    T q[W];  // row t after A_x
    if (t < NV) {
      // ---- load row t (pull streaming) ------------------------------------
      const T* src = frow + (size_t)ys * nx;
      T c[W];
#pragma unroll
      for (int i = 0; i < W; ++i) c[i] = valid[i] ? src[koff[i]] : T(0);
      frow += rowpitch;
      ys -= ystep;
      if (ys < 0) ys += ny;

      // ---- A_x: halos c_{-2}, c_{-1}, c_W, c_{W+1} from neighbour parts ---
      T cc[W + 4];
#pragma unroll
      for (int i = 0; i < W; ++i) cc[i + 2] = c[i];
      if (P > 1) {
        T l2 = lane_read(c[W - 2 >= 0 ? W - 2 : 0], lane_l);
        T l1 = lane_read(c[W - 1], lane_l);
        T r0 = lane_read(c[0], lane_r);
        T r1 = lane_read(c[W > 1 ? 1 : 0], lane_r);
        cc[0] = first ? T(0) : (W >= 2 ? l2 : T(0));
        cc[1] = first ? T(0) : l1;
        cc[W + 2] = last ? T(0) : r0;
        cc[W + 3] = last ? T(0) : (W >= 2 ? r1 : T(0));
      } else {
        cc[0] = cc[1] = cc[W + 2] = cc[W + 3] = T(0);
      }
      T gp[W + 4], gm[W + 4];
#pragma unroll
      for (int i = 0; i < W + 4; ++i) {
        gp[i] = nxp[i] * cc[i];
        gm[i] = nxm[i] * cc[i];
      }
      T F[W + 1];  // face f between slots f-1 and f (f = 0..W)
#pragma unroll
      for (int f = 0; f <= W; ++f) {
        // slot f-1 -> index f+1
        T fl = gp[f + 1] + gm[f + 2];
        if (KOREN)
          fl += koren(gp[f + 2] - gp[f + 1], gp[f + 1] - gp[f]) +
                koren(gm[f + 1] - gm[f + 2], gm[f + 2] - gm[f + 3]);
        if (f == 0) fl = first ? T(0) : fl;
        if (f >= FB) fl = last ? T(0) : fl;
        F[f] = fl;
      }
#pragma unroll
      for (int i = 0; i < W; ++i) q[i] = c[i] - (F[i + 1] - F[i]);
    } else {
#pragma unroll
      for (int i = 0; i < W; ++i) q[i] = T(0);
    }

    // ---- A_y (streamed): face t for g+, face t-1 for g- ------------------
    const T nu = ay - beta * (T)(t - H);
    const T nyp = pos(nu), nym = neg(nu);
    const bool fpv = t >= 1 && t <= NV - 1;
    const bool fmv = t >= 2 && t <= NV;
    T a[W];
#pragma unroll
    for (int i = 0; i < W; ++i) {
      const T gpv = nyp * q[i], gmv = nym * q[i];
      const T dpp = gpv - gp1[i];
      T Fp = gp1[i];
      if (KOREN) Fp += koren(dpp, dpp1[i]);
      Fp = fpv ? Fp : T(0);
      const T em = gm1[i] - gmv;
      T Fm = gm1[i];
      if (KOREN) Fm += koren(em1[i], em);
      Fm = fmv ? Fm : T(0);
      const T Fface = Fp1[i] + Fm;  // total flux through face t-1
      a[i] = acc2[i] - Fface;       // A_y output of row t-2
      acc2[i] = c1[i] + Fface;
      c1[i] = q[i];
      Fp1[i] = Fp;
      gp1[i] = gpv;
      dpp1[i] = dpp;
      gm1[i] = gmv;
      em1[i] = em;
    }

    if (t >= 2) {
      // ---- D_x on row t-2 (halos a_{-1}, a_W) ------------------------------
      T al = T(0), ar = T(0);
      if (P > 1) {
        al = lane_read(a[W - 1], lane_l);
        ar = lane_read(a[0], lane_r);
        al = first ? T(0) : al;
        ar = last ? T(0) : ar;
      }
      T dx[W + 1];  // a_{f-1} - a_f across face f
#pragma unroll
      for (int f = 0; f <= W; ++f) {
        const T left = f == 0 ? al : a[f - 1];
        const T right = f == W ? ar : a[f];
        T d = left - right;
        if (f == 0) d = first ? T(0) : d;
        if (f >= FB) d = last ? T(0) : d;
        dx[f] = d;
      }
      T b[W];
#pragma unroll
      for (int i = 0; i < W; ++i) b[i] = a[i] + D * (dx[i] - dx[i + 1]);

      // ---- D_y (streamed) and store row t-3 ------------------------------
      const int r = t - 2;  // row of b
      const bool dv = r >= 1 && r <= NV - 1;
#pragma unroll
      for (int i = 0; i < W; ++i) {
        const T del = dv ? a3[i] - b[i] : T(0);
        if (r >= 1 && active && valid[i])
          orow[(size_t)(r - 1) * rowpitch + (size_t)(p * W + i) * nxy] =
              a3[i] + D * (del3[i] - del);
        a3[i] = b[i];
        del3[i] = del;
      }
    }
  }
}

template <typename T, int NV, int P>
hipError_t launch_step2d_nv(const StepArgs& a, hipStream_t s) {
  constexpr int S = 64 / P;
  const int nx = (int)a.nx, ny = (int)a.ny;
  const int H = (NV - 1) / 2;
  const int ntx = (nx + S - 1) / S;
  const int ntiles = ntx * ny;
  const int nblocks = (ntiles + 3) / 4;
  const int xstep = a.shift % nx;
  const int xoff0 = (int)(((int64_t)a.shift * H) % nx);
  const int ystep = a.shift % ny;
  const int yoff0 = (int)(((int64_t)a.shift * H) % ny);
  const T as = (T)a.alpha_scale, be = (T)a.beta, D = (T)a.D;
  if (a.koren)
    hipLaunchKernelGGL((k_step2d<T, NV, P, true>), dim3(nblocks), dim3(256), 0,
                       s, (const T*)a.fin, (T*)a.fout, (const T*)a.u, a.flag,
                       nx, ny, xstep, xoff0, ystep, yoff0, as, be, D, ntx,
                       ntiles, nblocks);
  else
    hipLaunchKernelGGL((k_step2d<T, NV, P, false>), dim3(nblocks), dim3(256),
                       0, s, (const T*)a.fin, (T*)a.fout, (const T*)a.u,
                       a.flag, nx, ny, xstep, xoff0, ystep, yoff0, as, be, D,
                       ntx, ntiles, nblocks);
  return hipGetLastError();
}

}  // namespace lat
