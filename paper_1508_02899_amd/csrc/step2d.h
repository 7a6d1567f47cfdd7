// step2d.h -- fused streaming + collision pass for 2D lattices (gfx950).
//
// Layout: f[jy*NV + jx][y][x], x fastest.  One wavefront owns S = 64/P
// consecutive sites of one spatial row y.  Each site's vx axis is split
// over P lanes ("parts") that overlap by one cell: part p holds the
// W = (NV-1)/P + 1 cells jx = p*(W-1) + i, i = 0..W-1, so the last cell of
// part p is the first cell of part p+1 (both lanes compute it from the same
// inputs with the same operations, hence bit-identical values) and no lane
// holds cells outside the velocity square.
//
// The kernel streams over the vy index (rows jy = 0..NV-1), carrying a few
// rows of state in registers, so that every state element is read once and
// written once per pass and every load/store instruction moves S
// consecutive sites of P velocity planes:
//
//   for each row t = jy (the load of row t+1 is issued before row t is
//   processed):
//     load row t, pulled from the source sites (x - s(jx-h), y - s(t-h))
//       [Sec. 2 exact streaming];
//     A_x: drift along vx inside the row (split upwind fluxes, Koren
//       correction; 2 halo cells per side from the neighbouring parts);
//     A_y: drift along vy, streamed: face t-1 is complete once row t is in,
//       which gives the A_y output of row t-2;
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

// Streamed vy state of one lane (per cell i of its vx slice): g+ / g- of the
// previous row and their last differences, the previous face's g+ flux, the
// A_y accumulator of row t-2, the previous A_x output row, then the D_y
// state (previous D_x output row and its face difference).
template <typename T, int W>
struct YState {
  T gp1[W], dpp1[W], gm1[W], em1[W], Fp1[W], acc2[W], c1[W], a3[W], del3[W];
};

template <typename T, int NV, int P, bool KOREN>
struct Step2D {
  static constexpr int W = (NV - 1) / P + 1;  // cells per lane
  static constexpr int S = 64 / P;            // sites per wavefront
  static constexpr int H = (NV - 1) / 2;
  static_assert((NV - 1) % P == 0, "parts must tile the velocity axis");
  static_assert(P == 1 || W >= 3, "halo needs 3 cells per part");

  // One row t: c holds row t after streaming (when t < NV).  Reads state
  // `in`, writes state `out`; stores the finished row t-3 when t >= 3.
  __device__ __forceinline__ static void row(
      const int t, const T (&c)[W], const YState<T, W>& in,
      YState<T, W>& out, const T (&nxp)[W + 4], const T (&nxm)[W + 4],
      const T ay, const T beta, const T D, const bool first, const bool last,
      const int lane_l, const int lane_r, T* __restrict__ obase,
      const size_t rowpitch, const uint32_t slot_bytes,
      const uint32_t lane_off, const bool store_ok) {
    T q[W];  // row t after A_x (zero past the last row)
    if (t < NV) {
      T cc[W + 4];  // cells -2 .. W+1 of this lane's slice
#pragma unroll
      for (int i = 0; i < W; ++i) cc[i + 2] = c[i];
      if (P > 1) {
        const T l2 = lane_read(c[W - 3], lane_l);
        const T l1 = lane_read(c[W - 2], lane_l);
        const T r0 = lane_read(c[1], lane_r);
        const T r1 = lane_read(c[2], lane_r);
        cc[0] = first ? T(0) : l2;
        cc[1] = first ? T(0) : l1;
        cc[W + 2] = last ? T(0) : r0;
        cc[W + 3] = last ? T(0) : r1;
      } else {
        cc[0] = cc[1] = cc[W + 2] = cc[W + 3] = T(0);
      }
      T gp[W + 4], gm[W + 4];
#pragma unroll
      for (int i = 0; i < W + 4; ++i) {
        gp[i] = nxp[i] * cc[i];
        gm[i] = nxm[i] * cc[i];
      }
      T F[W + 1];  // face f between cells f-1 and f of the slice
#pragma unroll
      for (int f = 0; f <= W; ++f) {
        T fl = gp[f + 1] + gm[f + 2];
        if (KOREN)
          fl += koren(gp[f + 2] - gp[f + 1], gp[f + 1] - gp[f]) +
                koren(gm[f + 1] - gm[f + 2], gm[f + 2] - gm[f + 3]);
        if (f == 0) fl = first ? T(0) : fl;  // face 0 of the velocity square
        if (f == W) fl = last ? T(0) : fl;   // face NV
        F[f] = fl;
      }
#pragma unroll
      for (int i = 0; i < W; ++i) q[i] = c[i] - (F[i + 1] - F[i]);
    } else {
#pragma unroll
      for (int i = 0; i < W; ++i) q[i] = T(0);
    }

    // ---- A_y (streamed): g+ flux of face t, g- flux of face t-1 ----------
    const T nu = ay - beta * (T)(t - H);
    const T nyp = pos(nu), nym = neg(nu);
    const bool fpv = t >= 1 && t <= NV - 1;
    const bool fmv = t >= 2 && t <= NV;
    T a[W];
#pragma unroll
    for (int i = 0; i < W; ++i) {
      const T gpv = nyp * q[i], gmv = nym * q[i];
      const T dpp = gpv - in.gp1[i];
      T Fp = in.gp1[i];
      if (KOREN) Fp += koren(dpp, in.dpp1[i]);
      Fp = fpv ? Fp : T(0);
      const T em = in.gm1[i] - gmv;
      T Fm = in.gm1[i];
      if (KOREN) Fm += koren(in.em1[i], em);
      Fm = fmv ? Fm : T(0);
      const T Fface = in.Fp1[i] + Fm;  // total flux through face t-1
      a[i] = in.acc2[i] - Fface;       // A_y output of row t-2
      out.acc2[i] = in.c1[i] + Fface;
      out.c1[i] = q[i];
      out.Fp1[i] = Fp;
      out.gp1[i] = gpv;
      out.dpp1[i] = dpp;
      out.gm1[i] = gmv;
      out.em1[i] = em;
    }

    if (t >= 2) {
      // ---- D_x on row t-2 (halos a_{-1}, a_W) ------------------------------
      T al = T(0), ar = T(0);
      if (P > 1) {
        al = lane_read(a[W - 2], lane_l);
        ar = lane_read(a[1], lane_r);
        al = first ? T(0) : al;
        ar = last ? T(0) : ar;
      }
      T dxf[W + 1];  // a_{f-1} - a_f across face f
#pragma unroll
      for (int f = 0; f <= W; ++f) {
        const T left = f == 0 ? al : a[f - 1];
        const T right = f == W ? ar : a[f];
        T d = left - right;
        if (f == 0) d = first ? T(0) : d;
        if (f == W) d = last ? T(0) : d;
        dxf[f] = d;
      }
      // ---- D_y (streamed) and store row t-3 ------------------------------
      const int r = t - 2;  // row of b
      const bool dv = r >= 1 && r <= NV - 1;
      T* orow = obase + (size_t)(r - 1) * rowpitch;
#pragma unroll
      for (int i = 0; i < W; ++i) {
        const T b = a[i] + D * (dxf[i] - dxf[i + 1]);
        const T del = dv ? in.a3[i] - b : T(0);
        if (r >= 1 && store_ok)
          *(T*)((char*)orow + (size_t)(i * slot_bytes) + lane_off) =
              in.a3[i] + D * (in.del3[i] - del);
        out.a3[i] = b;
        out.del3[i] = del;
      }
    } else {
#pragma unroll
      for (int i = 0; i < W; ++i) {
        out.a3[i] = in.a3[i];
        out.del3[i] = in.del3[i];
      }
    }
  }
};

// INTERIOR: every source site of the tile lies inside [0, nx) without
// wrapping, so all cells of a row load from one uniform base plus one
// per-lane offset (plus a uniform per-cell stride); otherwise each cell
// keeps its own wrapped offset.
template <typename T, int NV, int P, bool KOREN, bool INTERIOR>
__device__ __forceinline__ void step2d_tile(
    const T* __restrict__ fin, T* __restrict__ fout, const T* __restrict__ u,
    int nx, int ny, int shift, int xstep, int xoff0, int ystep, int yoff0,
    T alpha_scale, T beta, T D, int x0, int y) {
  using K = Step2D<T, NV, P, KOREN>;
  constexpr int W = K::W, S = K::S, H = K::H;
  const int lane = (int)threadIdx.x & 63;
  const int p = lane / S;
  const int sl = lane - p * S;
  int x = x0 + sl;
  const bool active = x < nx;
  if (!active) x = nx - 1;  // duplicate a real site; never stored
  const bool first = p == 0, last = p == P - 1;
  const int lane_l = lane - S, lane_r = lane + S;
  const int jx0 = p * (W - 1);  // first vx cell of this lane

  const size_t nxy = (size_t)nx * (size_t)ny;
  const size_t rowpitch = (size_t)NV * nxy;  // elements between vy rows
  const T ax = u[(size_t)y * nx + x] * alpha_scale;
  const T ay = u[nxy + (size_t)y * nx + x] * alpha_scale;

  // vx drift of cells -2 .. W+1 (index + 2), cell widths per step
  T nxp[W + 4], nxm[W + 4];
#pragma unroll
  for (int i = 0; i < W + 4; ++i) {
    const T nu = ax - beta * (T)(jx0 + i - 2 - H);
    nxp[i] = pos(nu);
    nxm[i] = neg(nu);
  }

  // load offsets (bytes) of the W cells inside one vy row
  uint32_t koff[INTERIOR ? 1 : W];
  uint32_t cell_stride = 0;  // INTERIOR: bytes between consecutive cells
  if (INTERIOR) {
    // cell jx of site x comes from x - shift*(jx - H) = x0 + shift*H + sl
    //   - shift*jx, i.e. element jx*(nxy - shift) + (x0 + shift*H) + sl
    koff[0] = (uint32_t)(((size_t)jx0 * (nxy - shift) + (size_t)sl) *
                         sizeof(T));
    cell_stride = (uint32_t)((nxy - shift) * sizeof(T));
  } else {
    int xs = x + xoff0;  // jx = 0: (x + shift*H) mod nx
    if (xs >= nx) xs -= nx;
    for (int k = 0; k < jx0; ++k) {
      xs -= xstep;
      if (xs < 0) xs += nx;
    }
#pragma unroll
    for (int i = 0; i < (INTERIOR ? 1 : W); ++i) {
      koff[i] = (uint32_t)(((size_t)(jx0 + i) * nxy + (size_t)xs) * sizeof(T));
      xs -= xstep;
      if (xs < 0) xs += nx;
    }
  }
  const uint32_t slot_bytes = (uint32_t)(nxy * sizeof(T));
  const uint32_t store_lane = (uint32_t)(((size_t)jx0 * nxy + sl) * sizeof(T));
  T* obase = fout + (size_t)y * nx + x0;
  const T* fbase = INTERIOR ? fin + x0 + (size_t)shift * H : fin;

  auto load_row = [&](int t, int ys, T (&c)[W]) {
    const char* src = (const char*)(fbase + (size_t)t * rowpitch +
                                    (size_t)ys * nx);
#pragma unroll
    for (int i = 0; i < W; ++i) {
      if (INTERIOR)
        c[i] = *(const T*)(src + (size_t)(i * cell_stride) + koff[0]);
      else
        c[i] = *(const T*)(src + koff[i]);
    }
  };

  YState<T, W> s0, s1;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    s0.gp1[i] = s0.dpp1[i] = s0.gm1[i] = s0.em1[i] = s0.Fp1[i] =
        s0.acc2[i] = s0.c1[i] = s0.a3[i] = s0.del3[i] = T(0);
  }

  int ys = y + yoff0;  // row t = 0 comes from (y + shift*H) mod ny
  if (ys >= ny) ys -= ny;
  auto next_ys = [&](int v) {
    v -= ystep;
    return v < 0 ? v + ny : v;
  };

  T bufA[W], bufB[W];
  load_row(0, ys, bufA);
  ys = next_ys(ys);
  int t = 0;
#pragma unroll 1
  for (; t + 1 < NV + 3; t += 2) {
    if (t + 1 < NV) {
      load_row(t + 1, ys, bufB);
      ys = next_ys(ys);
    }
    K::row(t, bufA, s0, s1, nxp, nxm, ay, beta, D, first, last, lane_l,
           lane_r, obase, rowpitch, slot_bytes, store_lane, INTERIOR || active);
    if (t + 2 < NV) {
      load_row(t + 2, ys, bufA);
      ys = next_ys(ys);
    }
    K::row(t + 1, bufB, s1, s0, nxp, nxm, ay, beta, D, first, last, lane_l,
           lane_r, obase, rowpitch, slot_bytes, store_lane, INTERIOR || active);
  }
  if (t < NV + 3)
    K::row(t, bufA, s0, s1, nxp, nxm, ay, beta, D, first, last, lane_l,
           lane_r, obase, rowpitch, slot_bytes, store_lane, INTERIOR || active);
}

template <typename T, int NV, int P, bool KOREN>
__global__ __launch_bounds__(256) void k_step2d(
    const T* __restrict__ fin, T* __restrict__ fout, const T* __restrict__ u,
    const int* __restrict__ flag, int nx, int ny, int shift, int xstep,
    int xoff0, int ystep, int yoff0, T alpha_scale, T beta, T D, int ntx,
    int ntiles, int nblocks) {
  constexpr int S = 64 / P;
  constexpr int H = (NV - 1) / 2;
  if (*flag != 0) return;
  // tile index is uniform per wavefront; keep it (and all row bases) in
  // scalar registers
  const int tile = __builtin_amdgcn_readfirstlane(
      xcd_remap(blockIdx.x, nblocks) * 4 + ((int)threadIdx.x >> 6));
  if (tile >= ntiles) return;  // whole wavefront idle
  const int y = tile / ntx;
  const int x0 = (tile - y * ntx) * S;
  const bool interior = x0 + S <= nx && x0 - shift * H >= 0 &&
                        x0 + S - 1 + shift * H <= nx - 1;
  if (interior)
    step2d_tile<T, NV, P, KOREN, true>(fin, fout, u, nx, ny, shift, xstep,
                                       xoff0, ystep, yoff0, alpha_scale, beta,
                                       D, x0, y);
  else
    step2d_tile<T, NV, P, KOREN, false>(fin, fout, u, nx, ny, shift, xstep,
                                        xoff0, ystep, yoff0, alpha_scale,
                                        beta, D, x0, y);
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
                       nx, ny, a.shift, xstep, xoff0, ystep, yoff0, as, be, D,
                       ntx, ntiles, nblocks);
  else
    hipLaunchKernelGGL((k_step2d<T, NV, P, false>), dim3(nblocks), dim3(256),
                       0, s, (const T*)a.fin, (T*)a.fout, (const T*)a.u,
                       a.flag, nx, ny, a.shift, xstep, xoff0, ystep, yoff0, as,
                       be, D, ntx, ntiles, nblocks);
  return hipGetLastError();
}

}  // namespace lat
