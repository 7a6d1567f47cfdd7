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
    column1d<float, CAP, KOREN>(fin + m.f_off, fout + m.f_off, x, m.nx,
                                m.pitch, m.nv,
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
    PT::load(fin + m.f_off, m.nx, m.pitch, tl.x0, m.step_mod, m.init_off,
             jump, r, idle);
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
    PT::template store<NT>(tile, fout + m.f_off, m.nx, m.pitch, tl.x0);
    __syncthreads();  // the tile is refilled for the next work item
    w = wn;
  }
}

// ---------------------------------------------------------------------
// Resident multi-step form: one launch advances every member by all the
// steps of a call.  The members are split among the XCDs (the chip's
// accelerator dies, each with its own L2 cache shared by its compute
// units); every tile of a member, at every step, is updated by a
// workgroup of the member's XCD.  Each XCD has a work counter over its
// (step, tile) items, numbered step-major with the tiles of one step
// listed member by member; its workgroups take chunks from it.  The
// chunks come in blocks of `stride` (1 or 2): a block covers stride x
// chunk consecutive items, and its chunk r holds items r, r + stride,
// r + 2 stride, ... of them, so that the workgroups sharing a block work on
// neighbouring tiles at the same time (fewer places in memory at once;
// 5 % shorter steps on configuration 4 with stride 2, longer with 4 or
// more, where a member's step is spread over too many workgroups that then
// wait for each other).  A member's tile of step t > 0 starts once the member's counter
// of finished tiles shows all of its step t-1 tiles done: the pull
// streaming of step t reads any of them, and they have finished reading the
// buffer that step t writes.  Because producer and consumer share one L2,
// a finished tile is published by waiting for the workgroup's stores to
// reach the L2 before counting it (no L2 write-back, which publishing to
// another XCD's L2 would need on every tile: measured 15x slower), and
// consumed after invalidating the compute unit's L1.
// Deadlock freedom: a workgroup publishes its finished items before it
// ever waits, works its chunk's items in increasing order, and only waits
// on smaller items (of the previous step).  Take the smallest unfinished
// item u: if its chunk is held, the holder is at u and u's items are all
// finished, so it proceeds.  If not, every chunk of an earlier block is
// finished (its items are all below u), so a workgroup holding one of them
// moves on to the next chunk; only the other chunks of u's block (at most
// stride - 1) can be held by waiting workgroups, so with at least stride
// workgroups running on the XCD one of them takes u's chunk.  (A launch
// that runs fewer ends at the bounded waits with ETIMEOUT.)  Every
// class uses eight wavefronts per workgroup so that one kernel serves all
// of them (split-column tiles of parts1d.h).
template <int NV>
struct ResidentShape;
template <> struct ResidentShape<17> { static constexpr int P = 4; };
template <> struct ResidentShape<33> { static constexpr int P = 4; };
template <> struct ResidentShape<65> { static constexpr int P = 4; };
template <> struct ResidentShape<129> { static constexpr int P = 8; };
constexpr int kResW = 8;  // wavefronts per workgroup
template <int NV>
using ResTile = Parts1DTile<float, NV, ResidentShape<NV>::P, kResW>;
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kResLds = cmax(cmax(ResTile<17>::SIZE, ResTile<33>::SIZE),
                             cmax(ResTile<65>::SIZE, ResTile<129>::SIZE));

// Tiles x0, x0 + G, ..., x0 + (n-1) G of member m at one step, software
// pipelined: the loads of the next tile are in flight while the current
// one is updated and stored (as in the per-step split-column kernel).
// Every thread of the workgroup calls it; the tile LDS is free on return.
template <int NV, bool KOREN>
__device__ __forceinline__ void resident_run(float* tile,
                                             const float* __restrict__ fin,
                                             float* __restrict__ fout,
                                             const float* __restrict__ u,
                                             const BatchMember& m, int x0,
                                             int n, int slice, int stride) {
  constexpr int P = ResidentShape<NV>::P;
  using PT = ResTile<NV>;
  int jump = 0;  // (P s) mod nx, no division
  for (int q = 0; q < P; ++q) {
    jump += m.step_mod;
    if (jump >= m.nx) jump -= m.nx;
  }
  const float* const src = fin + m.f_off;
  float* const dst = fout + m.f_off;
  const float* const us = u + m.u_off + (int64_t)slice * m.nx;
  float r[PT::K];
  PT::load(src, m.nx, m.pitch, x0, m.step_mod, m.init_off, jump, r);
  const int hop = stride * PT::G;
  for (int q = 0; q < n; ++q) {
    const int xq = x0 + q * hop;
    PT::put(tile, r);
    // the flow value first: the memory counter is in order, and the
    // collision must not wait for the next tile's loads
    const float alpha = PT::alpha_at(us, m.nx, xq, m.alpha_scale);
    __syncthreads();
    // unconditional, so that the counter waits stay exact (past the last
    // tile: idle loads of one element)
    PT::load(src, m.nx, m.pitch, q + 1 < n ? xq + hop : xq, m.step_mod,
             m.init_off, jump, r, q + 1 >= n);
    PT::template collide<KOREN>(tile, alpha, m.nsub, m.beta, m.D);
    __syncthreads();
    PT::store(tile, dst, m.nx, m.pitch, xq);
    __syncthreads();
  }
}

template <bool KOREN>
__device__ __forceinline__ void resident_dispatch(
    float* tile, const float* __restrict__ fin, float* __restrict__ fout,
    const float* __restrict__ u, const BatchMember& m, int x0, int n,
    int slice, int stride) {
  switch (m.nv) {
    case 17: resident_run<17, KOREN>(tile, fin, fout, u, m, x0, n, slice, stride); break;
    case 33: resident_run<33, KOREN>(tile, fin, fout, u, m, x0, n, slice, stride); break;
    case 65: resident_run<65, KOREN>(tile, fin, fout, u, m, x0, n, slice, stride); break;
    default: resident_run<129, KOREN>(tile, fin, fout, u, m, x0, n, slice, stride); break;
  }
}

__device__ __forceinline__ int resident_g(int nv) {
  switch (nv) {
    case 17: return ResTile<17>::G;
    case 33: return ResTile<33>::G;
    case 65: return ResTile<65>::G;
    default: return ResTile<129>::G;
  }
}

// The XCD this workgroup runs on (hardware register XCC_ID, bits 0..3).
__device__ __forceinline__ int xcc_id() {
  return (int)__builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & 15;
}

// This wavefront's stores have reached the L2 (vector memory counter at
// zero; also a compiler barrier, so no store is scheduled after it).
__device__ __forceinline__ void stores_in_l2() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// Later loads of this wavefront see what other compute units of the XCD
// wrote to the L2 before the counter it polled: the device-scope acquire
// invalidates the compute unit's L1 (a workgroup-scope invalidate is a
// no-op when a workgroup's wavefronts share one L1).
__device__ __forceinline__ void drop_l1() {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// b0 holds the state before local step 0; step t reads b0 (t even) or b1
// and writes the other.  XCD x owns tiles[goff[x] .. goff[x+1]), one
// step's items; its counter is sync[kResQStride x].  sync[kResAbort] is
// the abort flag, sync[kResDone + m] member m's finished tiles; all zero at
// launch.  A wait that polls more than wait_limit times (or any wait when
// wait_limit < 0) raises the abort flag and ends the workgroup; the others
// end at their next wait or when their queue runs out.
template <bool KOREN>
__global__ __launch_bounds__(64 * kResW) void k_batch_resident(
    float* __restrict__ b0, float* __restrict__ b1,
    const float* __restrict__ u, const BatchMember* __restrict__ mem,
    const BatchTile* __restrict__ tiles, const int* __restrict__ goff,
    int nxcd, const int* __restrict__ mtiles, const int* __restrict__ mflag,
    int step0, int nsteps, int chunk, int* __restrict__ sync,
    int wait_limit, int stride) {
  __shared__ float tile[kResLds];
  __shared__ int s_base[2];
  __shared__ int s_go;
  const int tid = (int)threadIdx.x;
  const int x = xcc_id();
  if (x >= nxcd) return;
  const int g0 = goff[x], T = goff[x + 1] - g0;
  if (T == 0) return;
  const int total = T * nsteps;  // the host keeps it below 2^31 - grid chunk
  int* const queue = sync + kResQStride * x;
  int* const abort_flag = sync + kResAbort;
  int* const done = sync + kResDone;
  if (tid == 0)
    s_base[0] = __hip_atomic_fetch_add(queue, chunk, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  int slot = 0;
  int cur_m = -1, cur_t = -1, pend = 0;  // run of same member and step
  bool stop = false;
  // publish the finished tiles of the current run
  auto flush = [&]() {
    if (pend == 0) return;
    stores_in_l2();
    __syncthreads();
    if (tid == 0)
      __hip_atomic_fetch_add(&done[cur_m], pend, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    pend = 0;
  };
  while (!stop) {
    const int cidx = s_base[slot] / chunk;
    const int blk = cidx / stride;
    const int first = blk * stride * chunk + (cidx - blk * stride);
    if (first >= total) break;
    // the next chunk's number travels while this one is worked on
    if (tid == 0)
      s_base[slot ^ 1] = __hip_atomic_fetch_add(queue, chunk,
                                                __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    // the chunk's items first, first + stride, ...: runs of tiles of one
    // member at one step, stride tiles apart
    for (int j = 0; j < chunk;) {
      const int i = first + j * stride;
      if (i >= total) break;
      const int t = i / T;
      const BatchTile tl = tiles[g0 + (i - t * T)];
      const BatchMember m = mem[tl.member];
      const int k = tl.x0 / resident_g(m.nv);
      int n = (mtiles[tl.member] - k + stride - 1) / stride;
      if (n > chunk - j) n = chunk - j;
      const int rest = (total - i + stride - 1) / stride;
      if (n > rest) n = rest;
      j += n;
      if (mflag[tl.member] != 0) continue;  // frozen members do nothing
      if (tl.member != cur_m || t != cur_t) {
        flush();
        cur_m = tl.member;
        cur_t = t;
        if (t > 0) {
          if (tid == 0) {
            const int need = t * mtiles[tl.member];
            int polls = 0, ok = 1;
            while (__hip_atomic_load(&done[tl.member], __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT) < need) {
              if (wait_limit < 0 || ++polls > wait_limit ||
                  __hip_atomic_load(abort_flag, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT) != 0) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
              }
              __builtin_amdgcn_s_sleep(2);
            }
            s_go = ok;
          }
          __syncthreads();
          if (!s_go) {
            stop = true;
            break;
          }
          drop_l1();
        }
      }
      float* const fin = (t & 1) ? b1 : b0;
      float* const fout = (t & 1) ? b0 : b1;
      const int sl = m.u_hold > 0 ? (step0 + t) / m.u_hold : 0;
      resident_dispatch<KOREN>(tile, fin, fout, u, m, tl.x0, n, sl, stride);
      pend += n;
    }
    __syncthreads();  // s_base[slot ^ 1] is written
    slot ^= 1;
  }
  if (!stop) flush();
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
__global__ void k_or_int(const int* src, int* dst) { *dst |= *src; }
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

int batch_resident_sites(int cap) {
  switch (cap) {
    case 17: return ResTile<17>::G;
    case 33: return ResTile<33>::G;
    case 65: return ResTile<65>::G;
    case 129: return ResTile<129>::G;
    default: return 0;
  }
}

int batch_resident_threads() { return 64 * kResW; }

hipError_t batch_resident_occupancy(int koren, int* blocks_per_cu) {
  return koren ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                     blocks_per_cu, k_batch_resident<true>, 64 * kResW, 0)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                     blocks_per_cu, k_batch_resident<false>, 64 * kResW, 0);
}

hipError_t launch_batch_resident(const ResidentLaunch& a, hipStream_t s) {
  auto go = [&](auto kernel) {
    hipLaunchKernelGGL(kernel, dim3(a.grid), dim3(64 * kResW), 0, s, a.b0,
                       a.b1, a.u, a.mem, a.tiles, a.goff, a.nxcd, a.mtiles,
                       a.mflag, a.step0, a.nsteps, a.chunk, a.sync,
                       a.wait_limit, a.stride);
  };
  if (a.koren)
    go(k_batch_resident<true>);
  else
    go(k_batch_resident<false>);
  return hipGetLastError();
}

// After a resident launch: every XCD with items must have handed all of
// them out (a workgroup ran there); otherwise the launch did not complete
// and the abort flag is raised.
__global__ void k_resident_check(int* sync, const int* goff, int nxcd,
                                 int nsteps) {
  for (int x = 0; x < nxcd; ++x) {
    const int64_t need = (int64_t)(goff[x + 1] - goff[x]) * nsteps;
    if (need > 0 && (int64_t)sync[kResQStride * x] < need)
      sync[kResAbort] = 1;
  }
}

hipError_t launch_resident_check(int* sync, const int* goff, int nxcd,
                                 int nsteps, hipStream_t s) {
  hipLaunchKernelGGL(k_resident_check, dim3(1), dim3(1), 0, s, sync, goff,
                     nxcd, nsteps);
  return hipGetLastError();
}

__global__ void k_xcc_probe(int* out) {
  if (threadIdx.x == 0) out[blockIdx.x] = xcc_id();
}

hipError_t launch_xcc_probe(int* out, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k_xcc_probe, dim3(nblocks), dim3(64), 0, s, out);
  return hipGetLastError();
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

hipError_t launch_or_int(const int* src, int* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_or_int, dim3(1), dim3(1), 0, s, src, dst);
  return hipGetLastError();
}

hipError_t launch_clear_ints(int* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear_ints, dim3((n + 255) / 256), dim3(256), 0, s, p,
                     n);
  return hipGetLastError();
}

}  // namespace lat
