// step2d.h -- fused streaming + collision pass for 2D lattices (gfx950).
//
// Layout: f[jy*NV + jx][y][x], x fastest, velocity planes `pitch` elements
// apart (pitch >= nx*ny; padding keeps the planes that one row of the
// pass touches together off the same HBM channels).  One wavefront owns
// S = 64/P consecutive sites of one spatial row y.  Each site's vx axis is split
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
//       correction; 1 halo cell per side from the neighbouring parts, and
//       the two end faces of a part taken from its neighbours);
//     A_y: drift along vy, streamed: face t-1 is complete once row t is in,
//       which gives the A_y output of row t-2;
//     D_x: diffusion along vx on that row (1 halo cell per side);
//     D_y: diffusion along vy, streamed, giving the final row t-3;
//     store row t-3.
//
// Addressing: each row's base and the per-cell stride are wave-uniform
// (scalar registers), the per-lane part is one 32-bit VGPR offset (every
// byte offset inside a vy row stays below 2^32 - 1; the host checks this).  Rows 3..NV-1 run in a loop without the row-range selects
// of the first and last rows.
//
// The per-site order A_x, A_y, D_x, D_y is the paper's "force, then
// diffusion" split by velocity axis.  Zero flux through the outer faces of
// the velocity square; cells outside it are empty for the limiter.
#pragma once

#include <type_traits>

#include "device_common.h"
#include "lattice_internal.h"

// No implicit multiply-add contraction in this file: interior and edge tiles
// are separate instantiations, and a site must get the same bits in either
// (the result is invariant under translation of the lattice).  Fused
// multiply-adds are written out where they are meant.
#pragma clang fp contract(off)

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
  // STEADY: 3 <= t < NV, where every row-range condition below holds, so
  // the steady loop carries no selects for them.  MODE (steady rows only):
  // which split half of the vy drift to skip, see A_y below (0: none, 1: g-,
  // 2: g+, 3: decided on this row).
  // emit(i, v) receives cell i of the finished row t-3.
  template <bool STEADY, int MODE, typename Emit>
  __device__ __forceinline__ static void row(
      const int t, const T (&c)[W], YState<T, W>& st,
      const T (&nxp)[W + 2], const T (&nxm)[W + 2],
      const T ay, const T beta, const T D, const bool first, const bool last,
      const int lane_l, const int lane_r, Emit&& emit) {
    T q[W];  // row t after A_x (zero past the last row)
    if (STEADY || t < NV) {
      T cc[W + 2];  // cells -1 .. W of this lane's slice
#pragma unroll
      for (int i = 0; i < W; ++i) cc[i + 1] = c[i];
      if (P > 1) {
        const T l1 = lane_read(c[W - 2], lane_l);
        const T r0 = lane_read(c[1], lane_r);
        cc[0] = first ? T(0) : l1;
        cc[W + 1] = last ? T(0) : r0;
      } else {
        cc[0] = cc[W + 1] = T(0);
      }
      T gp[W + 2], gm[W + 2];
#pragma unroll
      for (int i = 0; i < W + 2; ++i) {
        gp[i] = nxp[i] * cc[i];
        gm[i] = nxm[i] * cc[i];
      }
      // face f lies between cells f-1 and f; this lane computes the inner
      // faces 1..W-1.  Face 0 is the left part's face W-1 and face W the
      // right part's face 1 (same inputs, same operations), or closed at
      // the ends of the velocity axis.
      T F[W + 1];
#pragma unroll
      for (int f = 1; f < W; ++f) {
        T fl = gp[f] + gm[f + 1];
        if (KOREN) {
          fl += koren(gp[f + 1] - gp[f], gp[f] - gp[f - 1]) +
                koren(gm[f] - gm[f + 1], gm[f + 1] - gm[f + 2]);
        }
        F[f] = fl;
      }
      if (P > 1) {
        const T fl = lane_read(F[W - 1], lane_l);
        const T fr = lane_read(F[1], lane_r);
        F[0] = first ? T(0) : fl;
        F[W] = last ? T(0) : fr;
      } else {
        F[0] = F[W] = T(0);
      }
#pragma unroll
      for (int i = 0; i < W; ++i) q[i] = c[i] - (F[i + 1] - F[i]);
    } else {
#pragma unroll
      for (int i = 0; i < W; ++i) q[i] = T(0);
    }

    // ---- A_y (streamed): g+ flux of face t, g- flux of face t-1 ----------
    const T nu = fma_t(-beta, (T)(t - H), ay);
    const T nyp = pos(nu), nym = neg(nu);
    const bool fpv = STEADY || (t >= 1 && t <= NV - 1);
    const bool fmv = STEADY || (t >= 2 && t <= NV);
    T a[W];
    // The streamed state is updated in place (each cell's old values are
    // read before they are replaced).  With beta >= 0 the vy drift falls
    // along the rows, so a split half that is zero on every lane of the
    // wavefront stays zero: once nu(t) >= 0 everywhere, g- of rows t-2..t is
    // zero and so is its flux through face t-1, and its state (gm1, em1)
    // already holds zeros; once nu(t-1) <= 0 everywhere, the g+ flux of
    // face t is zero, gp1 already holds zero, and dpp1 is not read again
    // (later rows skip g+ as well; the rows past the last plane force that
    // flux to zero).  Steady rows may skip such a half: M = 1 skips g-,
    // M = 2 skips g+, M = 0 computes both.  The caller guarantees the
    // condition of a skip it asks for (MODE 1 or 2) or leaves it to this row
    // (MODE 3).  The results differ from the full computation at most in the
    // sign of a zero.
    auto ay_cells = [&](auto mode) {
      constexpr int M = decltype(mode)::value;
#pragma unroll
      for (int i = 0; i < W; ++i) {
        T Fface = st.Fp1[i];  // g+ flux of face t-1 (previous row)
        if (M != 2) {
          const T gpv = nyp * q[i];
          const T dpp = gpv - st.gp1[i];
          T Fp = st.gp1[i];
          if (KOREN) Fp += koren(dpp, st.dpp1[i]);
          if (!STEADY) Fp = fpv ? Fp : T(0);
          st.Fp1[i] = Fp;
          st.gp1[i] = gpv;
          st.dpp1[i] = dpp;
        } else {
          st.Fp1[i] = T(0);
        }
        if (M != 1) {
          const T gmv = nym * q[i];
          const T em = st.gm1[i] - gmv;
          T Fm = st.gm1[i];
          if (KOREN) Fm += koren(st.em1[i], em);
          if (!STEADY) Fm = fmv ? Fm : T(0);
          Fface = Fface + Fm;  // total flux through face t-1
          st.gm1[i] = gmv;
          st.em1[i] = em;
        }
        a[i] = st.acc2[i] - Fface;  // A_y output of row t-2
        st.acc2[i] = st.c1[i] + Fface;
        st.c1[i] = q[i];
      }
    };
    static_assert(STEADY || MODE == 0, "edge rows compute both halves");
    if constexpr (MODE == 3) {
      if (beta >= T(0) && __all(nu >= T(0))) {
        ay_cells(std::integral_constant<int, 1>());
      } else {
        const T nu_prev = fma_t(-beta, (T)(t - 1 - H), ay);
        if (beta >= T(0) && __all(nu_prev <= T(0)))
          ay_cells(std::integral_constant<int, 2>());
        else
          ay_cells(std::integral_constant<int, 0>());
      }
    } else {
      ay_cells(std::integral_constant<int, MODE>());
    }

    if (STEADY || t >= 2) {
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
      // ---- D_y (streamed), giving row t-3 ----------------------------------
      const int r = t - 2;  // row of b
      const bool dv = STEADY || (r >= 1 && r <= NV - 1);
#pragma unroll
      for (int i = 0; i < W; ++i) {
        const T b = fma_t(D, dxf[i] - dxf[i + 1], a[i]);
        const T del = dv ? st.a3[i] - b : T(0);
        if (STEADY || r >= 1) emit(i, fma_t(D, st.del3[i] - del, st.a3[i]));
        st.a3[i] = b;
        st.del3[i] = del;
      }
    }
  }
};

// Output staging of a workgroup (P > 1).  The WGW wavefronts of a
// workgroup own G = WGW S consecutive sites of one spatial row; a
// wavefront's direct stores would write S-site pieces of P planes per
// instruction.  Instead each finished row goes to LDS and the workgroup
// stores it plane by plane, 64 consecutive elements per store instruction
// (and G consecutive elements per plane per round).  The plane stride is
// padded so that the P parts of a wavefront write to disjoint LDS banks.
template <typename T, int NV, int P, int WGW>
struct OutStage {
  static constexpr int S = 64 / P;
  static constexpr int G = WGW * S;        // sites per workgroup
  static constexpr int W = (NV - 1) / P + 1;
  static constexpr int DW = sizeof(T) / 4;  // dwords per element
  static constexpr int pad() {
    for (int pd = 0; pd < 64; ++pd) {
      bool used[64] = {};
      bool ok = true;
      for (int p = 0; p < P && ok; ++p)
        for (int sl = 0; sl < S && ok; ++sl)
          for (int d = 0; d < DW && ok; ++d) {
            const int bank =
                ((p * (W - 1) * (G + pd) + sl) * DW + d) % 64;
            if (used[bank]) ok = false;
            used[bank] = true;
          }
      if (ok || P * S * DW > 64) return pd;
    }
    return 0;
  }
  static constexpr int STRIDE = G + pad();      // elements per plane
  static constexpr int SIZE = NV * STRIDE;      // elements per buffer
  static constexpr int K = (NV + P - 1) / P;    // stores per thread per row
};

// Wavefronts per workgroup: wider workgroups make each stored plane run
// longer (measured on the row-streaming copy pattern: 128 consecutive
// sites per workgroup beat 64) at the cost of a barrier over more waves.
template <typename T, int NV, int P>
constexpr int step2d_wgw() {
  // FP32 lanes of 9 cells or fewer (nv <= 33 in 4 parts, nv = 65 in 8)
  // fit 8 waves per workgroup; longer slices need more than the registers
  // a wave may hold there
  return sizeof(T) == 4 && ((P == 4 && NV <= 33) || (P == 8 && NV == 65))
             ? 8
             : 4;
}

// INTERIOR: every source site of the tile lies inside [0, nx) without
// wrapping, so all cells of a row load from one uniform base plus one
// per-lane offset (plus a uniform per-cell stride); otherwise each cell
// keeps its own wrapped offset.
template <typename T, int NV, int P, bool KOREN, bool INTERIOR, int WGW,
          bool NT>
__device__ __forceinline__ void step2d_tile(
    const T* __restrict__ fin, T* __restrict__ fout, const T* __restrict__ u,
    T* __restrict__ stage, int nx, int ny, size_t pitch, int shift, int xstep,
    int xoff0, int ystep, int yoff0, T alpha_scale, T beta, T D, int xg, int w,
    int y) {
  using K = Step2D<T, NV, P, KOREN>;
  using O = OutStage<T, NV, P, WGW>;
  constexpr int W = K::W, S = K::S, H = K::H, G = O::G;
  const int lane = (int)threadIdx.x & 63;
  const int p = lane / S;
  const int sl = lane - p * S;
  const int x0 = xg * G + w * S;  // first site of this wavefront
  int x = x0 + sl;
  const bool active = x < nx;
  if (!active) x = nx - 1;  // duplicate a real site; never stored
  const bool first = p == 0, last = p == P - 1;
  const int lane_l = lane - S, lane_r = lane + S;
  const int jx0 = p * (W - 1);  // first vx cell of this lane

  const size_t nxy = (size_t)nx * (size_t)ny;   // one u component
  const size_t rowpitch = (size_t)NV * pitch;  // elements between vy rows
  const T ax = u[(size_t)y * nx + x] * alpha_scale;
  const T ay = u[nxy + (size_t)y * nx + x] * alpha_scale;

  // vx drift of cells -1 .. W (index + 1), cell widths per step
  T nxp[W + 2], nxm[W + 2];
#pragma unroll
  for (int i = 0; i < W + 2; ++i) {
    const T nu = fma_t(-beta, (T)(jx0 + i - 1 - H), ax);
    nxp[i] = pos(nu);
    nxm[i] = neg(nu);
  }

  // byte offsets of the W cells of one vy row from the row's base
  uint32_t koff[INTERIOR ? 1 : W];
  uint32_t cell_stride = 0;  // INTERIOR: bytes between consecutive cells
  if (INTERIOR) {
    // cell jx of site x comes from x - shift*(jx - H) = x0 + shift*H + sl
    //   - shift*jx, i.e. element jx*(pitch - shift) + (x0 + shift*H) + sl
    koff[0] = (uint32_t)(((size_t)jx0 * (pitch - shift) + (size_t)sl) *
                         sizeof(T));
    cell_stride = (uint32_t)((pitch - shift) * sizeof(T));
  } else {
    int xs = x + xoff0;  // jx = 0: (x + shift*H) mod nx
    if (xs >= nx) xs -= nx;
    for (int k = 0; k < jx0; ++k) {
      xs -= xstep;
      if (xs < 0) xs += nx;
    }
#pragma unroll
    for (int i = 0; i < (INTERIOR ? 1 : W); ++i) {
      koff[i] = (uint32_t)(((size_t)(jx0 + i) * pitch + (size_t)xs) *
                           sizeof(T));
      xs -= xstep;
      if (xs < 0) xs += nx;
    }
  }
  const uint32_t slot_bytes = (uint32_t)(pitch * sizeof(T));
  const T* fbase = INTERIOR ? fin + x0 + (size_t)shift * H : fin;

  auto load_row = [&](int t, int ys, T (&c)[W]) {
    const T* src = fbase + (size_t)t * rowpitch + (size_t)ys * nx;
    // a fresh copy of the lane offset per row: the loads then take the
    // scalar base + 32-bit offset form (the offset itself, held from
    // before the row loop, would be widened to 64 bits once and every
    // load would pay a 64-bit vector add)
    uint32_t lo = koff[0];
    if (INTERIOR) asm volatile("" : "+v"(lo));
#pragma unroll
    for (int i = 0; i < W; ++i)
      c[i] = INTERIOR ? row_load(src, (uint32_t)i * cell_stride, lo)
                      : row_load(src, 0u, koff[i]);
  };

  // Output of row t (the finished row t-3).  P == 1: a wavefront already
  // stores 64 consecutive sites per instruction.  P > 1: cells go to the
  // LDS buffer of t's parity; flush() then stores the workgroup's row.
  // Lanes past the end of the spatial row hold a duplicate of site nx-1
  // (same inputs, same operations, so the same bits) and store it there:
  // every store is unconditional, which keeps the memory-counter waits
  // exact.
  // P == 1: offsets from the start of spatial row y (x is the clamped site,
  // so the offset is never negative, also for wavefronts past the end)
  const uint32_t store_lane =
      (uint32_t)(((size_t)jx0 * pitch + (size_t)x) * sizeof(T));
  T* const orow0 = fout + (size_t)y * nx;
  T* const sbase = stage + jx0 * O::STRIDE + w * S + sl;  // P > 1
  const int tid = (int)threadIdx.x;
  // flush: thread tid stores plane fj0 + P k, site fs of the workgroup
  const int fj0 = G >= 64 ? __builtin_amdgcn_readfirstlane(tid / G) : tid / G;
  const int fs = tid - (tid / G) * G;
  const int fx = min(xg * G + fs, nx - 1);
  const uint32_t flane =
      (uint32_t)(((size_t)fj0 * pitch + (size_t)(fx - xg * G)) * sizeof(T));
  T* const frow0 = fout + (size_t)y * nx + (size_t)xg * G;
  auto flush = [&](int t) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    // the staged row leaves at raised wave priority: the workgroup's waves
    // issue their stores ahead of the neighbouring workgroups' arithmetic
    // (measured: about 1 % shorter passes)
    __builtin_amdgcn_s_setprio(3);
    const T* sb = stage + (t & 1) * O::SIZE + fj0 * O::STRIDE + fs;
    T* orow = frow0 + (size_t)(t - 3) * rowpitch;
    uint32_t fl = flane;  // per row, as for the loads
    asm volatile("" : "+v"(fl));
    constexpr int KL = O::K - 1;  // the last round covers planes < NV only
    T v[O::K];  // all LDS reads first, then the stores
#pragma unroll
    for (int k = 0; k < KL; ++k) v[k] = sb[k * P * O::STRIDE];
    const bool last_in = fj0 + P * KL < NV;
    v[KL] = last_in ? sb[KL * P * O::STRIDE] : T(0);
#pragma unroll
    for (int k = 0; k < KL; ++k)
      row_store<NT>(orow, (uint32_t)(k * P) * slot_bytes, fl, v[k]);
    __builtin_amdgcn_s_setprio(0);
    row_store_if<NT>(orow, (uint32_t)(KL * P) * slot_bytes, fl, v[KL],
                 last_in);
  };
  // kind: -1 for an edge row, else the steady row's skip mode
  auto run_row = [&](auto kind, int t, const T (&c)[W], YState<T, W>& st) {
    constexpr int KIND = decltype(kind)::value;
    constexpr bool STEADY = KIND >= 0;
    constexpr int MODE = STEADY ? KIND : 0;
    if (P == 1) {
      T* orow = orow0 + (size_t)(t - 3) * rowpitch;
      K::template row<STEADY, MODE>(
          t, c, st, nxp, nxm, ay, beta, D, first, last, lane_l,
          lane_r, [&](int i, T v) {
            row_store<NT>(orow, (uint32_t)i * slot_bytes, store_lane, v);
          });
    } else {
      T* sb = sbase + (t & 1) * O::SIZE;
      K::template row<STEADY, MODE>(
          t, c, st, nxp, nxm, ay, beta, D, first, last, lane_l,
          lane_r, [&](int i, T v) { sb[i * O::STRIDE] = v; });
      if (STEADY || t >= 3) flush(t);
    }
  };
  using edge_t = std::integral_constant<int, -1>;

  YState<T, W> st;
#pragma unroll
  for (int i = 0; i < W; ++i) {
    st.gp1[i] = st.dpp1[i] = st.gm1[i] = st.em1[i] = st.Fp1[i] =
        st.acc2[i] = st.c1[i] = st.a3[i] = st.del3[i] = T(0);
  }

  int ys = y + yoff0;  // row t = 0 comes from (y + shift*H) mod ny
  if (ys >= ny) ys -= ny;
  auto next_ys = [&](int v) {
    v -= ystep;
    return __builtin_amdgcn_readfirstlane(v < 0 ? v + ny : v);
  };

  // rows 0..2 fill the streamed state; rows 3..NV-1 are the steady part
  // (NV - 3 rows, an even count, processed in pairs); rows NV..NV+2 drain
  // it.  Row t+1 is loaded before row t is processed.  The first and the
  // last steady pair are peeled so that the loop bodies issue the same
  // loads and stores on every trip and on entry: the memory counter waits
  // then only ever wait for the row about to be used, never for the
  // stores issued after it.  The pairs between them run in three loops,
  // one per skip mode of the vy drift (the drift falls along the rows:
  // first g- is zero on every lane, then neither half, then g+), so that
  // each loop keeps its state in the same registers from trip to trip.
  T bufA[W], bufB[W];
  load_row(0, ys, bufA);
  ys = next_ys(ys);
  load_row(1, ys, bufB);
  ys = next_ys(ys);
  run_row(edge_t(), 0, bufA, st);
  load_row(2, ys, bufA);
  ys = next_ys(ys);
  run_row(edge_t(), 1, bufB, st);
  if (NV > 3) {
    load_row(3, ys, bufB);
    ys = next_ys(ys);
  }
  run_row(edge_t(), 2, bufA, st);
  // steady pair (t, t+1): row t is in bufB
  auto pair = [&](auto mode, int t, bool load2) {
    load_row(t + 1, ys, bufA);
    ys = next_ys(ys);
    run_row(mode, t, bufB, st);
    if (load2) {
      load_row(t + 2, ys, bufB);
      ys = next_ys(ys);
    }
    run_row(mode, t + 1, bufA, st);
  };
  using pick_t = std::integral_constant<int, 3>;
  // g- of rows t and t+1 is zero on every lane (the drift is >= 0 through
  // row t+1); g+ of faces t and t+1 is zero (the drift is <= 0 from row t-1)
  auto skip_gm = [&](int t) {
    return beta >= T(0) && __all(fma_t(-beta, (T)(t + 1 - H), ay) >= T(0));
  };
  auto skip_gp = [&](int t) {
    return beta >= T(0) && __all(fma_t(-beta, (T)(t - 1 - H), ay) <= T(0));
  };
  if (NV >= 7) {
    pair(std::integral_constant<int, 0>(), 3, true);
    int t = 5;
#pragma unroll 1
    for (; t <= NV - 4 && skip_gm(t); t += 2)
      pair(std::integral_constant<int, 1>(), t, true);
#pragma unroll 1
    for (; t <= NV - 4 && !skip_gp(t); t += 2)
      pair(std::integral_constant<int, 0>(), t, true);
#pragma unroll 1
    for (; t <= NV - 4; t += 2)
      pair(std::integral_constant<int, 2>(), t, true);
    pair(std::integral_constant<int, 0>(), NV - 2, false);
  } else if (NV == 5) {
    pair(pick_t(), 3, false);
  }
  run_row(edge_t(), NV, bufB, st);
  run_row(edge_t(), NV + 1, bufB, st);
  run_row(edge_t(), NV + 2, bufB, st);
}

// XCD x receives its blocks in rounds of g (the tiles of one
// spatial row), and round r of XCD x is logical row 8 r + x, so that each
// spatial row's tiles (which share the cache lines at their edges) run in
// one L2 while the workgroups running at any moment cover one band of
// consecutive rows, i.e. one stretch of memory per velocity plane instead
// of one per XCD.  Blocks past the last full round of the 8 XCDs take the
// contiguous ranges of xcd_remap.  A bijection of [0, n) for every g >= 1.
__device__ __forceinline__ int xcd_rows(int b, int n, int g) {
  const int full = n / (8 * g) * (8 * g);
  if (b >= full) return full + xcd_remap(b - full, n - full);
  const int xcd = b & 7, k = b >> 3;
  const int r = k / g;
  return (r * 8 + xcd) * g + (k - r * g);
}

// One workgroup = WGW wavefronts = G consecutive sites of spatial row y.  All
// run the same row sequence (the staged stores synchronise them once
// per row), so none may leave early; wavefronts past the end of the row
// compute on duplicated sites and store nothing.
template <typename T, int NV, int P, bool KOREN, bool NT,
          int WGW = step2d_wgw<T, NV, P>()>
__global__ __launch_bounds__(64 * WGW) void k_step2d(
    const T* __restrict__ fin, T* __restrict__ fout, const T* __restrict__ u,
    const int* __restrict__ flag, int nx, int ny, int64_t pitch, int shift,
    int xstep, int xoff0, int ystep, int yoff0, T alpha_scale, T beta, T D,
    int ngx, int nblocks) {
  using O = OutStage<T, NV, P, WGW>;
  constexpr int S = 64 / P;
  constexpr int H = (NV - 1) / 2;
  __shared__ T stage[P > 1 ? 2 * O::SIZE : 1];
  if (*flag != 0) return;  // uniform over the grid
  // whole rows of tiles per XCD, rows interleaved over the XCDs: the tiles
  // of a row, which read the same cache lines at their edges, meet in one
  // L2, and the rows in flight are consecutive (measured on 512^2 x 33^2:
  // 427 us per pass against 445 us with one contiguous range of rows per
  // XCD, whose eight bands of rows are far apart in every plane, and the
  // same time but 1.245x the HBM reads in plain dispatch order)
  const int b = xcd_rows(blockIdx.x, nblocks, ngx);
  const int y = b / ngx;
  const int xg = b - y * ngx;
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int x0 = xg * O::G + w * S;
  const bool interior = x0 + S <= nx && x0 - shift * H >= 0 &&
                        x0 + S - 1 + shift * H <= nx - 1;
  if (interior)
    step2d_tile<T, NV, P, KOREN, true, WGW, NT>(
        fin, fout, u, stage, nx, ny, (size_t)pitch, shift, xstep, xoff0,
        ystep, yoff0, alpha_scale, beta, D, xg, w, y);
  else
    step2d_tile<T, NV, P, KOREN, false, WGW, NT>(
        fin, fout, u, stage, nx, ny, (size_t)pitch, shift, xstep, xoff0,
        ystep, yoff0, alpha_scale, beta, D, xg, w, y);
}

template <typename T, int NV, int P>
hipError_t launch_step2d_nv(const StepArgs& a, hipStream_t s) {
  constexpr int WGW = step2d_wgw<T, NV, P>();
  constexpr int G = OutStage<T, NV, P, WGW>::G;
  if (!step2d_offsets_fit(NV, a.pitch, sizeof(T)) || a.pitch < a.nx * a.ny)
    return hipErrorNotSupported;
  const int nx = (int)a.nx, ny = (int)a.ny;
  const int H = (NV - 1) / 2;
  const int ngx = (nx + G - 1) / G;
  const int64_t nb = (int64_t)ngx * ny;
  if (nb > 0x7FFFFFFF) return hipErrorInvalidValue;
  const int nblocks = (int)nb;
  const int xstep = a.shift % nx;
  const int xoff0 = (int)(((int64_t)a.shift * H) % nx);
  const int ystep = a.shift % ny;
  const int yoff0 = (int)(((int64_t)a.shift * H) % ny);
  const T as = (T)a.alpha_scale, be = (T)a.beta, D = (T)a.D;
  // non-temporal stores when the state is larger than the 256 MB
  // memory-side cache (the next pass cannot find it there anyway)
  const bool nt = (uint64_t)NV * NV * (uint64_t)a.pitch * sizeof(T) >
                  (256ull << 20);
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(nblocks), dim3(64 * WGW), 0, s,
                       (const T*)a.fin, (T*)a.fout, (const T*)a.u, a.flag, nx,
                       ny, a.pitch, a.shift, xstep, xoff0, ystep, yoff0, as,
                       be, D, ngx, nblocks);
  };
  if (a.koren) {
    if (nt)
      go(k_step2d<T, NV, P, true, true>);
    else
      go(k_step2d<T, NV, P, true, false>);
  } else {
    if (nt)
      go(k_step2d<T, NV, P, false, true>);
    else
      go(k_step2d<T, NV, P, false, false>);
  }
  return hipGetLastError();
}

}  // namespace lat
