// parts1d.h -- the split-column 1D update of one tile of consecutive
// sites (gfx950), shared by the single-lattice pass (step1d_parts.hip) and
// the batched pass (batch1d.hip).
//
// Each site's velocity column is split over P lanes that overlap by one
// cell, as the parts of the 2D pass: part p holds the W = (NV-1)/P + 1
// cells j = p(W-1) + i, i = 0..W-1 (both copies of a shared cell are
// computed from the same inputs with the same operations, hence
// bit-identical).  One workgroup of WGW wavefronts owns a tile of
// G = WGW S consecutive sites (S = 64/P per wavefront):
//   1. pull streaming (Sec. 2): the workgroup loads velocity plane j of its
//      G sites from the source sites x - s(j-h) (consecutive addresses, one
//      wrap at most) and writes it to an LDS tile [NV][G];
//   2. each lane reads its W cells and runs nsub x [drift, diffusion]
//      (Eq. 5 force at cell centres, split upwind fluxes with the Koren
//      correction, zero flux through the outer faces; Eq. 4 diffusion
//      fluxes), with the halo cells and the end faces of a part taken
//      from the neighbouring parts by lane exchange;
//   3. the finished cells go back to the LDS tile and the workgroup stores
//      plane by plane, G consecutive sites per plane.
// Each state element is read once and written once per pass.
#pragma once

#include "device_common.h"

namespace lat {

template <typename T, int NV, int P, int WGW>
struct Parts1D {
  static constexpr int W = (NV - 1) / P + 1;  // cells per lane
  static constexpr int S = 64 / P;            // sites per wavefront
  static constexpr int G = WGW * S;           // sites per workgroup
  static constexpr int H = (NV - 1) / 2;
  static constexpr int K = (NV + P - 1) / P;  // planes per thread (1, 4)
  static constexpr int DW = sizeof(T) / 4;    // dwords per element
  static_assert((NV - 1) % P == 0, "parts must tile the velocity axis");
  static_assert(W >= 3, "the halo exchange needs 3 cells per part");
  // LDS layout: plane j at j STRIDE + (j / (W-1)) SKEW elements.  The P
  // parts of a wavefront read rows p(W-1) + i of S consecutive columns; the
  // padding of a plane is the smallest that puts the 64 lanes of one read in
  // distinct banks.  Where no padding can (parts W-1 = 16 planes apart: a
  // plane offset times 16 reaches only 4 of the 8 bank groups that 8 parts
  // need), a skew per block of W-1 planes separates the parts instead.
  static constexpr bool banks_ok(int pd, int sk) {
    bool used[64] = {};
    for (int p = 0; p < P; ++p)
      for (int sl = 0; sl < S; ++sl)
        for (int d = 0; d < DW; ++d) {
          const int bank = ((p * (W - 1) * (G + pd) + p * sk + sl) * DW + d) % 64;
          if (used[bank]) return false;
          used[bank] = true;
        }
    return true;
  }
  static constexpr int pad() {
    if (P * S * DW > 64) return 0;  // two or more elements per bank anyway
    for (int pd = 0; pd < 64; ++pd)
      if (banks_ok(pd, 0)) return pd;
    return 0;
  }
  static constexpr int skew() {
    if (P * S * DW > 64 || banks_ok(pad(), 0)) return 0;
    for (int sk = 1; sk < 64; ++sk)
      if (banks_ok(0, sk)) return sk;
    return 0;
  }
  static constexpr int STRIDE = G + pad();  // elements per LDS plane
  static constexpr int SKEW = skew();       // elements per block of W-1 planes
  static constexpr int SIZE = NV * STRIDE + P * SKEW;  // tile elements
  // offset of plane j in the tile
  __device__ __forceinline__ static constexpr int row(int j) {
    return j * STRIDE + (SKEW ? (j / (W - 1)) * SKEW : 0);
  }
};

// Parts and wavefronts per workgroup for each compiled velocity lattice
// (timed on configuration-2-like lattices: P in {4, 8, 16} and 2-8
// wavefronts per workgroup were within 10 %; these were the best).
template <typename T, int NV>
struct PartsShape;
template <> struct PartsShape<float, 17> { static constexpr int P = 4, WGW = 4; };
template <> struct PartsShape<float, 33> { static constexpr int P = 4, WGW = 4; };
template <> struct PartsShape<float, 65> { static constexpr int P = 8, WGW = 4; };
template <> struct PartsShape<float, 129> { static constexpr int P = 8, WGW = 4; };
template <> struct PartsShape<double, 17> { static constexpr int P = 4, WGW = 4; };
template <> struct PartsShape<double, 33> { static constexpr int P = 4, WGW = 4; };
template <> struct PartsShape<double, 65> { static constexpr int P = 8, WGW = 4; };

// The phases of the update of the tile of sites x0 .. x0+G-1 of one
// lattice [NV][nx] by one workgroup (every thread of the workgroup calls
// each phase; the tile is SIZE elements of LDS).  The loads and
// stores move whole planes: thread (fj0, fs) = (tid / G, tid % G) moves
// planes fj0 + P k, k < K, of site fs (the workgroup has 64 WGW = P G
// threads).  No implicit multiply-add contraction anywhere: the fused
// multiply-adds are written out, so that a site's bits do not depend on
// scheduling.
template <typename T, int NV, int P, int WGW>
struct Parts1DTile {
  using C = Parts1D<T, NV, P, WGW>;
  static constexpr int W = C::W, S = C::S, G = C::G, H = C::H, K = C::K;
  static constexpr int STRIDE = C::STRIDE, SKEW = C::SKEW, SIZE = C::SIZE;

  // 1a. pull streaming: plane j of site x comes from (x - s(j-h)) mod nx;
  // jump = (P s) mod nx, step_mod = s mod nx, init_off = (s h) mod nx;
  // plane j starts pitch elements after plane j-1 (pitch >= nx).
  // idle: the same loads (so that the memory-counter waits after them stay
  // exact) all from the first element of fin; r is not used then.
  __device__ __forceinline__ static void load(const T* __restrict__ fin,
                                              int nx, int pitch, int x0,
                                              int step_mod, int init_off,
                                              int jump, T (&r)[K],
                                              bool idle = false) {
    const int tid = (int)threadIdx.x;
    const int fj0 = tid / G;
    const int fs = tid - fj0 * G;
    const int fx = min(x0 + fs, nx - 1);  // past the end: a real site
    // (s h - s fj0) mod nx by fj0 < P wrapped subtractions (no division)
    int xs = init_off;
    for (int q = 0; q < fj0; ++q) {
      xs -= step_mod;
      if (xs < 0) xs += nx;
    }
    xs += fx;  // both below nx
    if (xs >= nx) xs -= nx;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = fj0 + P * k;
      const size_t e = idle ? 0 : (size_t)j * pitch + xs;
      r[k] = (k < K - 1 || j < NV) ? fin[e] : T(0);
      xs -= jump;
      if (xs < 0) xs += nx;
    }
  }

  // 1b. the loaded planes into the LDS tile
  __device__ __forceinline__ static void put(T* __restrict__ tile,
                                             const T (&r)[K]) {
    const int tid = (int)threadIdx.x;
    const int fj0 = tid / G;
    const int fs = tid - fj0 * G;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = fj0 + P * k;
      if (k < K - 1 || j < NV) tile[C::row(j) + fs] = r[k];
    }
  }

  // Site of this lane in the tile: lane (p, sl) of wavefront w holds cells
  // p(W-1) .. p(W-1)+W-1 of site w S + sl.
  __device__ __forceinline__ static int lane_site() {
    const int lane = (int)threadIdx.x & 63;
    return ((int)threadIdx.x >> 6) * S + (lane - (lane / S) * S);
  }

  // 2a. drift of the zero-velocity cell of this lane's site, alpha =
  // dt_s u(x) / (dv tau_p) (u: the lattice's flow slice)
  __device__ __forceinline__ static T alpha_at(const T* __restrict__ u,
                                               int nx, int x0,
                                               T alpha_scale) {
    return u[min(x0 + lane_site(), nx - 1)] * alpha_scale;
  }

  // 2b. nsub x [drift, diffusion] on every column of the tile, in place.
  // A site's column belongs to one wavefront, so no other wavefront
  // touches it (no barrier needed between the read and the write-back).
  template <bool KOREN>
  __device__ __forceinline__ static void collide(T* __restrict__ tile,
                                                 T alpha, int nsub, T beta,
                                                 T D) {
#pragma clang fp contract(off)
    const int lane = (int)threadIdx.x & 63;
    const int p = lane / S;
    const bool first = p == 0, last = p == P - 1;
    const int lane_l = lane - S, lane_r = lane + S;
    const int j0 = p * (W - 1);
    T* col = tile + j0 * STRIDE + p * SKEW + lane_site();  // = row(j0 + i)
    // for i < W-1; the part's last cell lies in the next block

    T nup[W + 2], num[W + 2];  // split coefficients of cells -1 .. W
#pragma unroll
    for (int i = 0; i < W + 2; ++i) {
      const T nu = fma_t(-beta, (T)(j0 + i - 1 - H), alpha);
      nup[i] = pos(nu);
      num[i] = neg(nu);
    }
    T c[W];
#pragma unroll
    for (int i = 0; i < W - 1; ++i) c[i] = col[i * STRIDE];
    c[W - 1] = col[(W - 1) * STRIDE + SKEW];

#pragma unroll 1
    for (int sub = 0; sub < nsub; ++sub) {
      // drift: cells -1 .. W (the outer cells from the neighbouring parts,
      // empty past the ends of the velocity axis)
      T gp[W + 2], gm[W + 2];
      {
        const T l1 = lane_read(c[W - 2], lane_l);
        const T r0 = lane_read(c[1], lane_r);
        const T cl = first ? T(0) : l1;
        const T cr = last ? T(0) : r0;
        gp[0] = nup[0] * cl;
        gm[0] = num[0] * cl;
#pragma unroll
        for (int i = 0; i < W; ++i) {
          gp[i + 1] = nup[i + 1] * c[i];
          gm[i + 1] = num[i + 1] * c[i];
        }
        gp[W + 1] = nup[W + 1] * cr;
        gm[W + 1] = num[W + 1] * cr;
      }
      // face f lies between cells f-1 and f; inner faces 1..W-1 here, face
      // 0 is the left part's face W-1 and face W the right part's face 1
      // (or closed at the ends of the velocity axis)
      T F[W + 1];
#pragma unroll
      for (int f = 1; f < W; ++f) {
        T fl = gp[f] + gm[f + 1];
        if (KOREN)
          fl += koren(gp[f + 1] - gp[f], gp[f] - gp[f - 1]) +
                koren(gm[f] - gm[f + 1], gm[f + 1] - gm[f + 2]);
        F[f] = fl;
      }
      {
        const T fl = lane_read(F[W - 1], lane_l);
        const T fr = lane_read(F[1], lane_r);
        F[0] = first ? T(0) : fl;
        F[W] = last ? T(0) : fr;
      }
      T q[W];
#pragma unroll
      for (int i = 0; i < W; ++i) q[i] = c[i] - (F[i + 1] - F[i]);

      // diffusion: face difference q_{f-1} - q_f, zero at the outer faces
      const T al = lane_read(q[W - 2], lane_l);
      const T ar = lane_read(q[1], lane_r);
      T df[W + 1];
#pragma unroll
      for (int f = 0; f <= W; ++f) {
        const T left = f == 0 ? al : q[f - 1];
        const T right = f == W ? ar : q[f];
        T d = left - right;
        if (f == 0) d = first ? T(0) : d;
        if (f == W) d = last ? T(0) : d;
        df[f] = d;
      }
#pragma unroll
      for (int i = 0; i < W; ++i) c[i] = fma_t(D, df[i] - df[i + 1], q[i]);
    }
#pragma unroll
    for (int i = 0; i < W - 1; ++i) col[i * STRIDE] = c[i];
    if (last) col[(W - 1) * STRIDE + SKEW] = c[W - 1];
  }

  // 3. plane-by-plane stores of the finished tile; NT: non-temporal stores
  // (for a launch whose output is too large to be found in the caches by
  // the next one; a compile-time choice: a run-time branch between the two
  // stores of one address is merged into one ordinary store)
  template <bool NT = false>
  __device__ __forceinline__ static void store(const T* __restrict__ tile,
                                               T* __restrict__ fout, int nx,
                                               int pitch, int x0) {
    const int tid = (int)threadIdx.x;
    const int fj0 = tid / G;
    const int fs = tid - fj0 * G;
    const int ox = x0 + fs;
    if (ox < nx) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int j = fj0 + P * k;
        if (k < K - 1 || j < NV) {
          T* const q = &fout[(size_t)j * pitch + ox];
          if constexpr (NT)
            __builtin_nontemporal_store(tile[C::row(j) + fs], q);
          else
            *q = tile[C::row(j) + fs];
        }
      }
    }
  }
};

// The whole update of one tile: load, put, barrier, collide, barrier,
// store.  A caller that reuses the tile synchronises again before the
// next put.
template <typename T, int NV, int P, int WGW, bool KOREN>
__device__ __forceinline__ void parts1d_tile(
    const T* __restrict__ fin, T* __restrict__ fout, const T* __restrict__ u,
    T* __restrict__ tile, int nx, int pitch, int x0, int step_mod,
    int init_off, int jump, int nsub, T alpha_scale, T beta, T D) {
  using PT = Parts1DTile<T, NV, P, WGW>;
  T r[PT::K];
  PT::load(fin, nx, pitch, x0, step_mod, init_off, jump, r);
  PT::put(tile, r);
  __syncthreads();
  const T alpha = PT::alpha_at(u, nx, x0, alpha_scale);
  PT::template collide<KOREN>(tile, alpha, nsub, beta, D);
  __syncthreads();
  PT::store(tile, fout, nx, pitch, x0);
}

}  // namespace lat
