// batch1d.hip -- kernels of the batched 1D form: many independent
// realizations (each its own nx, nv, dt, tau_p, kappa and flow) in one
// packed state buffer, advanced by persistent kernels that walk a list of
// (member, tile) work items.  The per-site update is column1d (one lane per
// site) or, for a class whose members all have nv equal to the class
// capacity, the split-column tile of parts1d.h -- exactly the updates of
// the single-lattice passes.
#include "batch_internal.h"
#include "column1d.h"
#include "parts1d.h"

namespace lat {
namespace {

template <int CAP, bool KOREN>
__global__ __launch_bounds__(256) void k_batch1d(
    const float* __restrict__ fin, float* __restrict__ fout,
    const float* __restrict__ u, const BatchMember* __restrict__ mem,
    const BatchTile* __restrict__ tiles, int ntiles,
    const int* __restrict__ mflag, const int* __restrict__ step_base,
    int local_step) {
  const int step = *step_base + local_step;
  // grid-stride walk over this class's work items (persistent when the
  // grid is smaller than the work list)
  for (int w = blockIdx.x; w < ntiles; w += gridDim.x) {
    const BatchTile tl = tiles[w];
    if (mflag[tl.member] != 0) continue;  // frozen member
    const BatchMember m = mem[tl.member];
    const int x = tl.x0 + (int)threadIdx.x;
    if (x >= m.nx) continue;
    const int sl = m.u_hold > 0 ? step / m.u_hold : 0;
    const float ux = u[m.u_off + (int64_t)sl * m.nx + x];
    column1d<float, CAP, KOREN>(fin + m.f_off, fout + m.f_off, x, m.nx, m.nv,
                                m.h, m.step_mod, m.init_off, m.nsub,
                                ux * m.alpha_scale, m.beta, m.D);
  }
}

// Parts and wavefronts per workgroup of the batched split-column tiles
// (timed on configuration 4's classes: nv = 65 prefers longer columns per
// lane and nv = 129 wider workgroups here than on a single short lattice).
template <int NV>
struct BatchShape {
  static constexpr int P = PartsShape<float, NV>::P;
  static constexpr int WGW = PartsShape<float, NV>::WGW;
};
template <>
struct BatchShape<65> {
  static constexpr int P = 4, WGW = 4;
};
template <>
struct BatchShape<129> {
  static constexpr int P = 8, WGW = 8;
};

template <int NV>
constexpr int parts_threads() {
  return 64 * BatchShape<NV>::WGW;
}

// Split-column form: work items are tiles of G sites of one member (all
// members of the class have nv == NV).  Software-pipelined over the work
// items of a workgroup: the loads of the next tile are issued before the
// current tile's columns are updated, so that they overlap its collision
// and its stores.
template <int NV, bool KOREN, bool NT>
__global__ __launch_bounds__(parts_threads<NV>()) void k_batch1d_parts(
    const float* __restrict__ fin, float* __restrict__ fout,
    const float* __restrict__ u, const BatchMember* __restrict__ mem,
    const BatchTile* __restrict__ tiles, int ntiles,
    const int* __restrict__ mflag, const int* __restrict__ step_base,
    int local_step) {
  constexpr int P = BatchShape<NV>::P, WGW = BatchShape<NV>::WGW;
  using PT = Parts1DTile<float, NV, P, WGW>;
  __shared__ float tile[PT::SIZE];
  const int step = *step_base + local_step;
  // next work item of this workgroup at or after w, skipping frozen
  // members (uniform over the workgroup)
  auto next = [&](int w) {
    while (w < ntiles && mflag[tiles[w].member] != 0) w += gridDim.x;
    return w;
  };
  auto issue = [&](int w, float (&r)[PT::K], bool idle) {
    const BatchTile tl = tiles[w];
    const BatchMember m = mem[tl.member];
    int jump = 0;  // (P s) mod nx, no division
    for (int q = 0; q < P; ++q) {
      jump += m.step_mod;
      if (jump >= m.nx) jump -= m.nx;
    }
    PT::load(fin + m.f_off, m.nx, tl.x0, m.step_mod, m.init_off, jump, r,
             idle);
  };
  float r[PT::K];
  int w = next((int)blockIdx.x);
  if (w < ntiles) issue(w, r, false);
  while (w < ntiles) {
    const BatchTile tl = tiles[w];
    const BatchMember m = mem[tl.member];
    PT::put(tile, r);
    const int sl = m.u_hold > 0 ? step / m.u_hold : 0;
    // the flow value first: the memory counter is in order, and the
    // collision must not wait for the loads of the next tile
    const float alpha = PT::alpha_at(u + m.u_off + (int64_t)sl * m.nx, m.nx,
                                     tl.x0, m.alpha_scale);
    __syncthreads();
    const int wn = next(w + (int)gridDim.x);
    // in flight during the update below (unconditional, so that the
    // counter waits stay exact; past the last item: idle loads of one
    // element of this member)
    issue(wn < ntiles ? wn : w, r, wn >= ntiles);
    PT::template collide<KOREN>(tile, alpha, m.nsub, m.beta, m.D);
    __syncthreads();
    PT::template store<NT>(tile, fout + m.f_off, m.nx, tl.x0);
    __syncthreads();  // the tile is refilled for the next work item
    w = wn;
  }
}

// Per member: flag |= 1 if one of the slices the call uses has |u| past the
// member's drift bound or non-finite.  Grid (chunks, members): the
// workgroups of one member share its slices grid-stride.
__global__ __launch_bounds__(256) void k_batch_cfl(
    const float* __restrict__ u, const BatchMember* __restrict__ mem,
    int64_t nsteps, int strict, int* __restrict__ mflag) {
  const BatchMember m = mem[blockIdx.y];
  if (!(m.umax_ok < 3.0e38f)) return;  // no drag: no drift bound
  const int64_t need = m.u_hold > 0 ? (nsteps + m.u_hold - 1) / m.u_hold : 1;
  const int64_t n = need * m.nx;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    float a = u[m.u_off + i];
    a = a < 0.f ? -a : a;
    bad |= strict ? !(a < m.umax_ok) : !(a <= m.umax_ok);
  }
  if (__any(bad) && ((int)threadIdx.x & 63) == 0)
    atomicOr(&mflag[blockIdx.y], 1);
}

// FP64 sum of one velocity plane of one member per workgroup.
__global__ __launch_bounds__(256) void k_batch_plane_sums(
    const float* __restrict__ f, const BatchPlane* __restrict__ planes,
    double* __restrict__ out) {
  __shared__ double sh[256];
  const BatchPlane pl = planes[blockIdx.x];
  const float* p = f + pl.off;
  double acc = 0.0;
  for (int i = threadIdx.x; i < pl.nx; i += 256) acc += (double)p[i];
  const int t = (int)threadIdx.x;
  sh[t] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) sh[t] += sh[t + w];
    __syncthreads();
  }
  if (t == 0) out[blockIdx.x] = sh[0];
}

// Per member: combine its plane sums (fixed order) into
// {M, P, Q, variance} with weights dx dv and velocities (j - h) dv.
__global__ void k_batch_moments_final(const double* __restrict__ ps,
                                      const BatchMember* __restrict__ mem,
                                      int count, double* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= count) return;
  const BatchMember m = mem[r];
  double M = 0, P = 0, Q = 0;
  for (int j = 0; j < m.nv; ++j) {
    const double s = ps[m.plane0 + j];
    const double v = (double)(j - m.h) * m.dv;
    M += s;
    P += s * v;
    Q += s * v * v;
  }
  const double w = m.dx * m.dv;
  out[6 * r + 0] = w * M;
  out[6 * r + 1] = w * P;
  out[6 * r + 2] = w * Q;
  out[6 * r + 3] = Q / M - (P / M) * (P / M);
  out[6 * r + 4] = 0.0;
  out[6 * r + 5] = 0.0;
}

__global__ void k_set_int(int* p, int v) { *p = v; }
__global__ void k_add_int(int* p, int v) { *p += v; }
__global__ void k_clear_ints(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

template <int CAP>
hipError_t launch_cap(const BatchLaunch& a, hipStream_t s) {
  if (a.koren)
    hipLaunchKernelGGL((k_batch1d<CAP, true>), dim3(a.grid), dim3(a.block), 0,
                       s, a.fin, a.fout, a.u, a.mem, a.tiles, a.ntiles,
                       a.mflag, a.step_base, a.local_step);
  else
    hipLaunchKernelGGL((k_batch1d<CAP, false>), dim3(a.grid), dim3(a.block),
                       0, s, a.fin, a.fout, a.u, a.mem, a.tiles, a.ntiles,
                       a.mflag, a.step_base, a.local_step);
  return hipGetLastError();
}

template <int NV>
hipError_t launch_parts(const BatchLaunch& a, hipStream_t s) {
  constexpr int WGW = BatchShape<NV>::WGW;
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(a.grid), dim3(64 * WGW), 0, s, a.fin,
                       a.fout, a.u, a.mem, a.tiles, a.ntiles, a.mflag,
                       a.step_base, a.local_step);
  };
  if (a.koren) {
    if (a.nt)
      go(k_batch1d_parts<NV, true, true>);
    else
      go(k_batch1d_parts<NV, true, false>);
  } else {
    if (a.nt)
      go(k_batch1d_parts<NV, false, true>);
    else
      go(k_batch1d_parts<NV, false, false>);
  }
  return hipGetLastError();
}

}  // namespace

namespace {
template <int NV>
constexpr int batch_g() {
  return Parts1D<float, NV, BatchShape<NV>::P, BatchShape<NV>::WGW>::G;
}
}  // namespace

int batch_parts_sites(int cap) {
  switch (cap) {
    case 17: return batch_g<17>();
    case 33: return batch_g<33>();
    case 65: return batch_g<65>();
    case 129: return batch_g<129>();
    default: return 0;
  }
}

hipError_t launch_batch1d(const BatchLaunch& a, hipStream_t s) {
  if (a.block == 0) {  // split-column tiles
    switch (a.cap) {
      case 17: return launch_parts<17>(a, s);
      case 33: return launch_parts<33>(a, s);
      case 65: return launch_parts<65>(a, s);
      case 129: return launch_parts<129>(a, s);
      default: return hipErrorInvalidValue;
    }
  }
  switch (a.cap) {
    case 9: return launch_cap<9>(a, s);
    case 17: return launch_cap<17>(a, s);
    case 33: return launch_cap<33>(a, s);
    case 65: return launch_cap<65>(a, s);
    case 129: return launch_cap<129>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batch_cfl(const float* u, const BatchMember* mem, int count,
                            int64_t nsteps, int64_t max_values, int strict,
                            int* mflag, hipStream_t s) {
  if (count < 1 || count > 65535) return hipErrorInvalidValue;
  // about 16 values per thread for the largest member, at most 4096
  // workgroups per member
  int64_t chunks = (max_values + 256 * 16 - 1) / (256 * 16);
  chunks = chunks < 1 ? 1 : (chunks > 4096 ? 4096 : chunks);
  hipLaunchKernelGGL(k_batch_cfl, dim3((unsigned)chunks, (unsigned)count),
                     dim3(256), 0, s, u, mem, nsteps, strict, mflag);
  return hipGetLastError();
}

hipError_t launch_batch_moments(const float* f, const BatchPlane* planes,
                                int nplanes, const BatchMember* mem, int count,
                                double* plane_sums, double* out,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_batch_plane_sums, dim3(nplanes), dim3(256), 0, s, f,
                     planes, plane_sums);
  hipLaunchKernelGGL(k_batch_moments_final, dim3((count + 63) / 64), dim3(64),
                     0, s, plane_sums, mem, count, out);
  return hipGetLastError();
}

hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_add_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_add_int, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_clear_ints(int* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear_ints, dim3((n + 255) / 256), dim3(256), 0, s, p,
                     n);
  return hipGetLastError();
}

}  // namespace lat
