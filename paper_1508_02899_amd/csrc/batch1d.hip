// batch1d.hip -- kernels of the batched 1D form: many independent
// realizations (each its own nx, nv, dt, tau_p, kappa and flow) in one
// packed state buffer, advanced by persistent kernels that walk a list of
// (member, tile) work items.  The per-site update is column1d, exactly the
// single-lattice pass.
#include "batch_internal.h"
#include "column1d.h"

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

// Per member: flag |= 1 if one of the slices the call uses has |u| past the
// member's drift bound or non-finite.  One workgroup per member.
__global__ __launch_bounds__(256) void k_batch_cfl(
    const float* __restrict__ u, const BatchMember* __restrict__ mem,
    int64_t nsteps, int strict, int* __restrict__ mflag) {
  const BatchMember m = mem[blockIdx.x];
  if (!(m.umax_ok < 3.0e38f)) return;  // no drag: no drift bound
  const int64_t need = m.u_hold > 0 ? (nsteps + m.u_hold - 1) / m.u_hold : 1;
  const int64_t n = need * m.nx;
  bool bad = false;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    float a = u[m.u_off + i];
    a = a < 0.f ? -a : a;
    bad |= strict ? !(a < m.umax_ok) : !(a <= m.umax_ok);
  }
  if (__any(bad) && ((int)threadIdx.x & 63) == 0) atomicOr(&mflag[blockIdx.x], 1);
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

}  // namespace

hipError_t launch_batch1d(const BatchLaunch& a, hipStream_t s) {
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
                            int64_t nsteps, int strict, int* mflag,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_batch_cfl, dim3(count), dim3(256), 0, s, u, mem, nsteps,
                     strict, mflag);
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
