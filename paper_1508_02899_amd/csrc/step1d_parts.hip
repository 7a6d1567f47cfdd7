// step1d_parts.hip -- fused streaming + collision pass for 1D lattices with
// each site's velocity column split over P lanes (gfx950).
//
// The one-lane-per-site pass (step1d.hip) gives nx lanes: a short lattice
// (a few thousand to tens of thousands of sites) then leaves most of the
// chip idle.  Here P lanes share a column, as the parts of the 2D pass do:
// part p holds the W = (NV-1)/P + 1 cells j = p(W-1) + i, i = 0..W-1, and
// neighbouring parts overlap by one cell (both compute it from the same
// inputs with the same operations, so the copies are bit-identical).
//
// One workgroup of WGW wavefronts owns G = WGW S consecutive sites
// (S = 64/P per wavefront):
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
#include <type_traits>

#include "device_common.h"
#include "lattice_internal.h"

// No implicit multiply-add contraction: the fused multiply-adds are written
// out, so that a site's bits do not depend on how the compiler schedules it.
#pragma clang fp contract(off)

namespace lat {
namespace {

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
  // LDS padding: the P parts of a wavefront read rows p(W-1) + i of S
  // consecutive columns; pick the smallest padding that puts the 64 lanes
  // of one read in distinct banks.
  static constexpr int pad() {
    for (int pd = 0; pd < 64; ++pd) {
      bool used[64] = {};
      bool ok = true;
      for (int p = 0; p < P && ok; ++p)
        for (int sl = 0; sl < S && ok; ++sl)
          for (int d = 0; d < DW && ok; ++d) {
            const int bank = ((p * (W - 1) * (G + pd) + sl) * DW + d) % 64;
            if (used[bank]) ok = false;
            used[bank] = true;
          }
      if (ok || P * S * DW > 64) return pd;
    }
    return 0;
  }
  static constexpr int STRIDE = G + pad();  // elements per LDS plane
};

template <typename T, int NV, int P, int WGW, bool KOREN>
__global__ __launch_bounds__(64 * WGW) void k_step1d_parts(
    const T* __restrict__ fin, T* __restrict__ fout, const T* __restrict__ u,
    const int* __restrict__ flag, int nx, int step_mod, int init_off,
    int jump, int nsub, T alpha_scale, T beta, T D, int nblocks) {
  using C = Parts1D<T, NV, P, WGW>;
  constexpr int W = C::W, S = C::S, G = C::G, H = C::H, K = C::K;
  constexpr int STRIDE = C::STRIDE;
  __shared__ T tile[NV * STRIDE];
  if (*flag != 0) return;  // uniform over the grid
  const int xg = xcd_remap(blockIdx.x, nblocks);
  const int tid = (int)threadIdx.x;

  // ---- 1. pull streaming into the tile: thread (fj0, fs) moves planes
  // fj0 + P k of site fs (the workgroup has 64 WGW = P G threads)
  const int fj0 = tid / G;
  const int fs = tid - fj0 * G;
  const int fx = min(xg * G + fs, nx - 1);  // past the end: a real site
  {
    // source site of plane j: (fx + s h - s j) mod nx
    int xs = (int)(((int64_t)fx + init_off - (int64_t)fj0 * step_mod) % nx);
    if (xs < 0) xs += nx;
    T r[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = fj0 + P * k;
      r[k] = (k < K - 1 || j < NV) ? fin[(size_t)j * nx + xs] : T(0);
      xs -= jump;  // jump = (P s) mod nx
      if (xs < 0) xs += nx;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = fj0 + P * k;
      if (k < K - 1 || j < NV) tile[j * STRIDE + fs] = r[k];
    }
  }
  __syncthreads();

  // ---- 2. collision on the lanes' slices
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int p = lane / S;
  const int sl = lane - p * S;
  const int site = w * S + sl;
  const int x = min(xg * G + site, nx - 1);
  const bool first = p == 0, last = p == P - 1;
  const int lane_l = lane - S, lane_r = lane + S;
  const int j0 = p * (W - 1);
  T* col = tile + j0 * STRIDE + site;

  const T alpha = u[x] * alpha_scale;
  T nup[W + 2], num[W + 2];  // split coefficients of cells -1 .. W
#pragma unroll
  for (int i = 0; i < W + 2; ++i) {
    const T nu = fma_t(-beta, (T)(j0 + i - 1 - H), alpha);
    nup[i] = pos(nu);
    num[i] = neg(nu);
  }
  T c[W];
#pragma unroll
  for (int i = 0; i < W; ++i) c[i] = col[i * STRIDE];

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
    // face f lies between cells f-1 and f; inner faces 1..W-1 here, face 0
    // is the left part's face W-1 and face W the right part's face 1 (or
    // closed at the ends of the velocity axis)
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

  // ---- 3. back to the tile (a site's column belongs to one wavefront, so
  // no other wavefront reads these cells), then plane-by-plane stores
#pragma unroll
  for (int i = 0; i < W - 1; ++i) col[i * STRIDE] = c[i];
  if (last) col[(W - 1) * STRIDE] = c[W - 1];
  __syncthreads();
  const int ox = xg * G + fs;
  if (ox < nx) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int j = fj0 + P * k;
      if (k < K - 1 || j < NV) fout[(size_t)j * nx + ox] = tile[j * STRIDE + fs];
    }
  }
}

// Parts and wavefronts per workgroup for each compiled velocity lattice.
template <typename T, int NV>
struct PartsShape;
template <> struct PartsShape<float, 17> { static constexpr int P = 4, WGW = 4; };
template <> struct PartsShape<float, 33> { static constexpr int P = 4, WGW = 4; };
template <> struct PartsShape<float, 65> { static constexpr int P = 8, WGW = 4; };
template <> struct PartsShape<float, 129> { static constexpr int P = 8, WGW = 4; };
template <> struct PartsShape<double, 17> { static constexpr int P = 4, WGW = 4; };
template <> struct PartsShape<double, 33> { static constexpr int P = 4, WGW = 4; };
template <> struct PartsShape<double, 65> { static constexpr int P = 8, WGW = 4; };

template <typename T, int NV>
hipError_t launch_nv(const StepArgs& a, hipStream_t s) {
  constexpr int P = PartsShape<T, NV>::P, WGW = PartsShape<T, NV>::WGW;
  constexpr int G = Parts1D<T, NV, P, WGW>::G;
  const int nx = (int)a.nx;
  const int nblocks = (nx + G - 1) / G;
  const int h = (NV - 1) / 2;
  const int step_mod = a.shift % nx;
  const int init_off = (int)(((int64_t)a.shift * h) % nx);
  const int jump = (int)(((int64_t)P * step_mod) % nx);
  const T as = (T)a.alpha_scale, be = (T)a.beta, D = (T)a.D;
  if (a.koren)
    hipLaunchKernelGGL((k_step1d_parts<T, NV, P, WGW, true>), dim3(nblocks),
                       dim3(64 * WGW), 0, s, (const T*)a.fin, (T*)a.fout,
                       (const T*)a.u, a.flag, nx, step_mod, init_off, jump,
                       a.nsub_inline, as, be, D, nblocks);
  else
    hipLaunchKernelGGL((k_step1d_parts<T, NV, P, WGW, false>), dim3(nblocks),
                       dim3(64 * WGW), 0, s, (const T*)a.fin, (T*)a.fout,
                       (const T*)a.u, a.flag, nx, step_mod, init_off, jump,
                       a.nsub_inline, as, be, D, nblocks);
  return hipGetLastError();
}

}  // namespace

bool step1d_parts_supported(int nv, int f64) {
  return nv == 17 || nv == 33 || nv == 65 || (nv == 129 && !f64);
}

hipError_t launch_step1d_parts(const StepArgs& a, hipStream_t s) {
  if (!step1d_parts_supported(a.nv, a.f64) || a.nx < 1 ||
      a.nx > 0x7FFFFFFF)
    return hipErrorInvalidValue;
  if (a.f64) {
    switch (a.nv) {
      case 17: return launch_nv<double, 17>(a, s);
      case 33: return launch_nv<double, 33>(a, s);
      default: return launch_nv<double, 65>(a, s);
    }
  }
  switch (a.nv) {
    case 17: return launch_nv<float, 17>(a, s);
    case 33: return launch_nv<float, 33>(a, s);
    case 65: return launch_nv<float, 65>(a, s);
    default: return launch_nv<float, 129>(a, s);
  }
}

}  // namespace lat
