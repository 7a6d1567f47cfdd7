// observables.hip -- coarse-grained density statistics (gfx950).
//
// rho_r on non-overlapping tilings with boxes of r = 2^k lattice spacings
// per direction (the paper's coarse-grained density of Sec. 3.2, tiled
// rather than sliding): the box mass m_b is the sum of the site densities
// inside, rho_r = (m_b / M) * N_b so that <rho_r> = 1, and
//   <rho_r^2> = N_b * sum_b m_b^2 / M^2.
// Level k + 1 box masses are the sums of 2^dim level-k boxes, so each level
// reads the previous one.  All sums are FP64 in a fixed order.
#include "device_common.h"
#include "lattice_internal.h"

namespace lat {
namespace {

constexpr int kObsBlock = 256;
constexpr int kMaxLevels = kRhoMaxLevels;

__device__ void block_sum2(double& a, double& b, double* sa, double* sb) {
  const int t = (int)threadIdx.x;
  sa[t] = a;
  sb[t] = b;
  __syncthreads();
#pragma unroll
  for (int w = kObsBlock / 2; w > 0; w >>= 1) {
    if (t < w) {
      sa[t] = sa[t] + sa[t + w];
      sb[t] = sb[t] + sb[t + w];
    }
    __syncthreads();
  }
  a = sa[0];
  b = sb[0];
  __syncthreads();
}

// One thread per output box.  mode 0: boxes are the input cells themselves
// (level 0); mode 1: 2 x 2 children (2D), mode 2: 2 children (1D).
// partial[2 * block] = sum m, partial[2 * block + 1] = sum m^2.
__global__ __launch_bounds__(kObsBlock) void k_tile_level(
    const double* __restrict__ m_in, int64_t nx_out, int64_t ny_out,
    int mode, double* __restrict__ m_out, double* __restrict__ partial) {
  __shared__ double sa[kObsBlock], sb[kObsBlock];
  const int64_t n = nx_out * ny_out;
  const int64_t i = (int64_t)blockIdx.x * kObsBlock + threadIdx.x;
  double m = 0.0;
  if (i < n) {
    if (mode == 0) {
      m = m_in[i];
    } else if (mode == 2) {
      m = m_in[2 * i] + m_in[2 * i + 1];
    } else {
      const int64_t y = i / nx_out, x = i - y * nx_out;
      const int64_t nx_in = 2 * nx_out;
      const double* r0 = m_in + (2 * y) * nx_in + 2 * x;
      const double* r1 = r0 + nx_in;
      m = (r0[0] + r0[1]) + (r1[0] + r1[1]);
    }
    if (m_out) m_out[i] = m;
  }
  double s1 = m, s2 = m * m;
  block_sum2(s1, s2, sa, sb);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s1;
    partial[2 * blockIdx.x + 1] = s2;
  }
}

struct LevelMeta {
  int64_t off[kMaxLevels], nblk[kMaxLevels], nbox[kMaxLevels];
};

// One block per level: fixed-order sum of that level's partials, then
// out[k] = N_b * sum m^2 / (sum m)^2.
__global__ __launch_bounds__(kObsBlock) void k_tile_final(
    const double* __restrict__ partial, LevelMeta meta,
    double* __restrict__ out) {
  __shared__ double sa[kObsBlock], sb[kObsBlock];
  const int k = blockIdx.x;
  const double* p = partial + 2 * meta.off[k];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t j = threadIdx.x; j < meta.nblk[k]; j += kObsBlock) {
    s1 += p[2 * j];
    s2 += p[2 * j + 1];
  }
  block_sum2(s1, s2, sa, sb);
  if (threadIdx.x == 0) out[k] = (double)meta.nbox[k] * s2 / (s1 * s1);
}

}  // namespace

int64_t rho_r2_partials(int dim, int64_t nx, int64_t ny, int levels) {
  int64_t cx = nx, cy = dim == 2 ? ny : 1, total = 0;
  for (int k = 0; k < levels; ++k) {
    if (k > 0) {
      cx /= 2;
      if (dim == 2) cy /= 2;
    }
    total += (cx * cy + kObsBlock - 1) / kObsBlock;
  }
  return total;
}

hipError_t launch_rho_r2(const double* rho, int dim, int64_t nx, int64_t ny,
                         int levels, double* work, double* partial,
                         double* out, hipStream_t s) {
  // work: every level's box masses after level 0 (fewer than the sites);
  // partial: 2 doubles per block of every level (rho_r2_partials blocks).
  LevelMeta meta;
  const double* in = rho;
  double* w = work;
  int64_t cx = nx, cy = dim == 2 ? ny : 1, poff = 0;
  for (int k = 0; k < levels; ++k) {
    if (k > 0) {
      cx /= 2;
      if (dim == 2) cy /= 2;
    }
    const int64_t n = cx * cy;
    const int64_t nb = (n + kObsBlock - 1) / kObsBlock;
    const int mode = k == 0 ? 0 : (dim == 2 ? 1 : 2);
    double* o = k == 0 ? nullptr : w;
    hipLaunchKernelGGL(k_tile_level, dim3((unsigned)nb), dim3(kObsBlock), 0, s,
                       k == 0 ? rho : in, cx, cy, mode, o, partial + 2 * poff);
    meta.off[k] = poff;
    meta.nblk[k] = nb;
    meta.nbox[k] = n;
    poff += nb;
    if (k > 0) {
      in = o;
      w += n;
    }
  }
  hipLaunchKernelGGL(k_tile_final, dim3(levels), dim3(kObsBlock), 0, s,
                     partial, meta, out);
  return hipGetLastError();
}

}  // namespace lat
