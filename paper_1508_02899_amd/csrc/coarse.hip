// coarse.hip -- coarse velocity lattice with a learned face-flux correction
// (gfx950): fine -> coarse restriction, minimum-norm flux targets for
// training, the network's training kernels (FP32) and its matrix-core
// (bf16 MFMA, FP32 accumulation) inference fused with the conservative
// correction of the coarse state.
//
// The coarse lattice keeps dx and dt and takes every 4th fine velocity
// (velocity stride 4), so its streaming stays an exact integer shift
// (Sec. 2: dx = dv dt).  After each coarse step (stream, drift, diffusion),
// every interior velocity face of every site gets a correction flux
//   G = sign * m_s * y,
// y being the network's output for the face's 8 features (the 5-cell
// stencil of the face, ordered from its upwind side and divided by the
// stencil mass m_s; |face drift| in cells per step; ln St; 0), limited to
// a quarter of the donor cell's mass (so no cell can go negative), and the
// state is updated by f -= div G (mass is conserved exactly).
#include <math.h>

#include "coarse_internal.h"
#include "device_common.h"
#include "lattice_internal.h"

namespace lat {
namespace {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) {
  return __uint_as_float((uint32_t)b << 16);
}
__device__ __forceinline__ float qbf(float f) { return bf2f(f2bf(f)); }

// GELU, tanh form (Hendrycks & Gimpel 2016), and its derivative, written
// with the identity 0.5 (1 + tanh(y)) = 1 / (1 + exp(-2y)): one exponential
// and one approximate reciprocal (1 ulp) per value, no division.  For very
// negative z, exp overflows to +inf and the reciprocal gives 0 (gelu -> -0).
// The argument -2 log2(e) y with y = a z (1 + c z^2) is formed as
// z (K1 + K2 z^2): one multiply-add and one multiply.
__device__ __forceinline__ float gelu_sig(float z, float z2) {
  constexpr float a = 0.7978845608028654f, c = 0.044715f;
  constexpr float K1 = -2.0f * 1.4426950408889634f * a;  // -2 log2(e) a
  constexpr float K2 = K1 * c;
  return __builtin_amdgcn_rcpf(
      1.0f + __builtin_amdgcn_exp2f(z * __builtin_fmaf(K2, z2, K1)));
}
__device__ __forceinline__ float gelu(float z) {
  return z * gelu_sig(z, z * z);
}
__device__ __forceinline__ float gelu_d(float z, float* dg) {
  const float a = 0.7978845608028654f, c = 0.044715f;
  const float z2 = z * z;
  const float sg = gelu_sig(z, z2);
  *dg = sg + 2.0f * z * sg * (1.0f - sg) * a * __builtin_fmaf(3.0f * c, z2, 1.0f);
  return z * sg;
}

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
// Four floats to bf16, round to nearest even: two packed hardware
// conversions (v_cvt_pk_bf16_f32), the same rounding as f2bf.
typedef __bf16 bf16x2h __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d) {
  const f32x2 lo = {a, b}, hi = {c, d};
  const u32x2 w = {
      __builtin_bit_cast(unsigned, __builtin_convertvector(lo, bf16x2h)),
      __builtin_bit_cast(unsigned, __builtin_convertvector(hi, bf16x2h))};
  return __builtin_bit_cast(bf16x4, w);
}

// The network in matrix-core form.  16 inputs (faces) per wavefront pass;
// each layer is computed transposed, D = W^T X^T, so that the 16x16x16
// MFMA result layout (lane l: rows 4(l/16)+i, column l%16) is exactly the
// B-operand layout of the next layer (lane l: k = 4(l/16)+i, column l%16).
struct MlpRegs {
  bf16x4 a1[4];      // W1^T tiles (units 16u.., features)
  bf16x4 a2[4][4];   // W2^T tiles [unit tile][k step]
  bf16x4 a3[4];      // w3 as row 0 of a 16-row A operand, per k step
  float b1[4][4], b2[4][4];  // biases of this lane's D rows
  float b3;
};

__device__ void load_mlp(MlpRegs& R, const float* __restrict__ P,
                         const uint16_t* __restrict__ wq) {
  const int l = (int)threadIdx.x & 63;
  const int col = l & 15, ks = l >> 4;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 4 * ks + i, unit = 16 * u + col;
      R.a1[u][i] = k < kNF ? (short)wq[kOffW1 + k * kNH + unit] : (short)0;
    }
#pragma unroll
    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int k = 16 * kk + 4 * ks + i, unit = 16 * u + col;
        R.a2[u][kk][i] = (short)wq[kOffW2 + k * kNH + unit];
      }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      R.b1[u][i] = P[kOffB1 + 16 * u + 4 * ks + i];
      R.b2[u][i] = P[kOffB2 + 16 * u + 4 * ks + i];
    }
  }
#pragma unroll
  for (int kk = 0; kk < 4; ++kk)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      R.a3[kk][i] = col == 0 ? (short)wq[kOffW3 + 16 * kk + 4 * ks + i]
                             : (short)0;
  R.b3 = P[kOffB3];
}

// x = this lane's 4 features (k = 4(l/16)+i of input column l%16; zero for
// l >= 32).  Returns the output of column l%16 in lanes 0..15.
// The biases enter as the accumulator inputs of the first matrix-core
// step of each layer.
__device__ __forceinline__ float mlp_forward(const MlpRegs& R, bf16x4 x) {
  bf16x4 h1[4], h2[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const f32x4 b = {R.b1[u][0], R.b1[u][1], R.b1[u][2], R.b1[u][3]};
    const f32x4 d = mfma16(R.a1[u], x, b);
    h1[u] = pack4(gelu(d[0]), gelu(d[1]), gelu(d[2]), gelu(d[3]));
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    f32x4 d = {R.b2[u][0], R.b2[u][1], R.b2[u][2], R.b2[u][3]};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) d = mfma16(R.a2[u][kk], h1[kk], d);
    h2[u] = pack4(gelu(d[0]), gelu(d[1]), gelu(d[2]), gelu(d[3]));
  }
  f32x4 y = {R.b3, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) y = mfma16(R.a3[kk], h2[kk], y);
  return y[0];
}

// The same network with the layer biases read from LDS (b1s, b2s: the 64
// biases of each hidden layer, 16-byte aligned): a kernel that keeps the
// weights in registers for its whole run frees the 32 bias registers.
__device__ __forceinline__ float mlp_forward_lds(const MlpRegs& R,
                                                 const float* b1s,
                                                 const float* b2s, bf16x4 x) {
  const int ks = ((int)threadIdx.x & 63) >> 4;
  bf16x4 h1[4], h2[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const f32x4 b = *(const f32x4*)(b1s + 16 * u + 4 * ks);
    const f32x4 d = mfma16(R.a1[u], x, b);
    h1[u] = pack4(gelu(d[0]), gelu(d[1]), gelu(d[2]), gelu(d[3]));
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    f32x4 d = *(const f32x4*)(b2s + 16 * u + 4 * ks);
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) d = mfma16(R.a2[u][kk], h1[kk], d);
    h2[u] = pack4(gelu(d[0]), gelu(d[1]), gelu(d[2]), gelu(d[3]));
  }
  f32x4 y = {R.b3, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) y = mfma16(R.a3[kk], h2[kk], y);
  return y[0];
}

// -------------------------------------------------------------- restriction
// Coarse cell J spans fine centres 4J-2..4J+2: fine cells 4J-1..4J+1 count
// fully, 4J+-2 half (tensor product in 2D); densities scale by 1/4 per axis.
__global__ __launch_bounds__(256) void k_restrict2d(const float* __restrict__ ff,
                                                    float* __restrict__ fc,
                                                    int64_t sites, int nvf) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= sites) return;
  const int nvc = (nvf - 1) / 4 + 1;
  const int J = blockIdx.y, Jy = J / nvc, Jx = J - Jy * nvc;
  float acc = 0.f;
  for (int oy = -2; oy <= 2; ++oy) {
    const int jy = 4 * Jy + oy;
    if (jy < 0 || jy >= nvf) continue;
    const float wy = (oy == -2 || oy == 2) ? 0.5f : 1.f;
    for (int ox = -2; ox <= 2; ++ox) {
      const int jx = 4 * Jx + ox;
      if (jx < 0 || jx >= nvf) continue;
      const float wx = (ox == -2 || ox == 2) ? 0.5f : 1.f;
      acc += wy * wx * ff[(size_t)(jy * nvf + jx) * sites + s];
    }
  }
  fc[(size_t)J * sites + s] = acc * (1.f / 16.f);
}

__global__ __launch_bounds__(256) void k_restrict1d(const float* __restrict__ ff,
                                                    float* __restrict__ fc,
                                                    int64_t sites, int nvf) {
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= sites) return;
  const int J = blockIdx.y;
  float acc = 0.f;
  for (int o = -2; o <= 2; ++o) {
    const int j = 4 * J + o;
    if (j < 0 || j >= nvf) continue;
    acc += ((o == -2 || o == 2) ? 0.5f : 1.f) * ff[(size_t)j * sites + s];
  }
  fc[(size_t)J * sites + s] = acc * 0.25f;
}

// ---------------------------------------------------------- face features
// Features of interior face k (cells k-1 | k) of one velocity line of a
// site; line(i) returns the density of cell i (0 outside the line).
template <typename LINE>
__device__ __forceinline__ void face_feat(LINE line, int nv, int k, float u,
                                          const CoarseGeom& g, float* st,
                                          float* ms, float* sg, float* anu) {
  const int h = (nv - 1) / 2;
  const float vface = ((float)k - 0.5f - (float)h) * g.dv;
  const float nu = g.nu_scale * (u - vface);
  const bool up = nu >= 0.f;
  float m = 0.f;
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const int c = up ? k - 3 + i : k + 2 - i;
    const float v = (c >= 0 && c < nv) ? line(c) : 0.f;
    st[i] = v;
    m += v;
  }
  *ms = m;
  *sg = up ? 1.f : -1.f;
  *anu = up ? nu : -nu;
}

// ---------------------------------------------------------- flux targets
// One workgroup per listed site.  r = f_true - f_pred; the face fluxes with
// -div G = r of least norm are G = D^T psi with (D D^T) psi = -r, D D^T
// being the Neumann Laplacian of the velocity square, diagonal in the
// cosine (DCT-II) basis with eigenvalues lam_kx + lam_ky,
// lam_k = 4 sin^2(pi k / (2 nv)).
constexpr float kMinStencilMass = 1e-30f;  // 1 / m_s stays finite above

template <int NV>
__global__ __launch_bounds__(320) void k_flux_samples(
    CoarseGeom g, const float* __restrict__ fp, const float* __restrict__ ft,
    const float* __restrict__ u, const int32_t* __restrict__ sites,
    float* __restrict__ X, float* __restrict__ T, float* __restrict__ Wt) {
  constexpr int N2 = NV * NV;
  constexpr int NFACE = 2 * NV * (NV - 1);
  __shared__ float cs[NV][NV];
  __shared__ float lam[NV];
  __shared__ float r[N2], a[N2], pred[N2];
  const int tid = (int)threadIdx.x, bd = (int)blockDim.x;
  const int64_t S = (int64_t)g.nx * g.ny;
  const int site = sites[blockIdx.x];
  for (int i = tid; i < N2; i += bd) {
    const int k = i / NV, j = i - k * NV;
    const float ck = k == 0 ? sqrtf(1.0f / NV) : sqrtf(2.0f / NV);
    cs[k][j] = ck * cospif((float)k * ((float)j + 0.5f) / (float)NV);
    const float p = fp[(size_t)i * S + site];
    pred[i] = p;
    r[i] = ft[(size_t)i * S + site] - p;
  }
  for (int k = tid; k < NV; k += bd) {
    const float sk = sinpif((float)k / (2.0f * NV));
    lam[k] = 4.0f * sk * sk;
  }
  __shared__ float msite;
  __syncthreads();
  if (tid == 0) {  // site mass, in a fixed order
    float m = 0.f;
    for (int i = 0; i < N2; ++i) m += pred[i];
    msite = m;
  }
  // forward transform along x, then y
  for (int i = tid; i < N2; i += bd) {
    const int jy = i / NV, kx = i - jy * NV;
    float s = 0.f;
    for (int jx = 0; jx < NV; ++jx) s += cs[kx][jx] * r[jy * NV + jx];
    a[i] = s;
  }
  __syncthreads();
  for (int i = tid; i < N2; i += bd) {
    const int ky = i / NV, kx = i - ky * NV;
    float s = 0.f;
    for (int jy = 0; jy < NV; ++jy) s += cs[ky][jy] * a[jy * NV + kx];
    const float den = lam[kx] + lam[ky];
    r[i] = (i == 0) ? 0.f : -s / den;  // psi in the cosine basis
  }
  __syncthreads();
  // inverse transform along y, then x
  for (int i = tid; i < N2; i += bd) {
    const int jy = i / NV, kx = i - jy * NV;
    float s = 0.f;
    for (int ky = 0; ky < NV; ++ky) s += cs[ky][jy] * r[ky * NV + kx];
    a[i] = s;
  }
  __syncthreads();
  for (int i = tid; i < N2; i += bd) {
    const int jy = i / NV, jx = i - jy * NV;
    float s = 0.f;
    for (int kx = 0; kx < NV; ++kx) s += cs[kx][jx] * a[jy * NV + kx];
    r[i] = s;  // psi
  }
  __syncthreads();
  const float ux = u[site], uy = u[S + site];
  const size_t base = (size_t)blockIdx.x * NFACE;
  for (int f = tid; f < NFACE; f += bd) {
    float st[5], ms, sg, anu, G;
    if (f < NV * (NV - 1)) {  // x-face (row jy, face k)
      const int jy = f / (NV - 1), k = f - jy * (NV - 1) + 1;
      auto line = [&](int c) { return pred[jy * NV + c]; };
      face_feat(line, NV, k, ux, g, st, &ms, &sg, &anu);
      G = r[jy * NV + k - 1] - r[jy * NV + k];
    } else {  // y-face (face k, column jx)
      const int q = f - NV * (NV - 1);
      const int k = q / NV + 1, jx = q - (k - 1) * NV;
      auto line = [&](int c) { return pred[c * NV + jx]; };
      face_feat(line, NV, k, uy, g, st, &ms, &sg, &anu);
      G = r[(k - 1) * NV + jx] - r[k * NV + jx];
    }
    // faces with (next to) no mass in the stencil carry no sample weight
    const bool use = ms > kMinStencilMass && ms >= g.line_eps * msite;
    const float inv = use ? 1.0f / ms : 0.f;
    float* x = X + (base + f) * kNF;
#pragma unroll
    for (int i = 0; i < 5; ++i) x[i] = st[i] * inv;
    x[5] = anu;
    x[6] = g.log_st;
    x[7] = 0.f;
    T[base + f] = use ? sg * G * inv : 0.f;
    Wt[base + f] = use ? ms : 0.f;
  }
}

// ------------------------------------------------- natural flux targets
// The collision of one site's velocity square c[NV][NV] (row jy, column jx)
// held in LDS, with the face fluxes of every sub-operation summed into
// Fx[jy][face 0..NV] and Fy[face 0..NV][jx]: the sub-steps of the lattice
// pass (drift along vx, along vy, diffusion along vx, along vy; force at
// cell centres, split fluxes with the Koren correction, outer faces
// closed), so that c_after = c_before - div F.  tmp: NV (NV+1) floats.
struct CollideCoef {
  float ax, ay;  // drift of the zero-velocity cell, per axis (cells)
  float beta, D;
  int nsub, koren;
};

template <int NV>
__device__ void collide_record(float* __restrict__ c, float* __restrict__ tmp,
                               float* __restrict__ Fx, float* __restrict__ Fy,
                               const CollideCoef& p) {
  constexpr int H = (NV - 1) / 2, NF = NV * (NV + 1);
  const int tid = (int)threadIdx.x, bd = (int)blockDim.x;
  for (int i = tid; i < NF; i += bd) Fx[i] = Fy[i] = 0.f;
  __syncthreads();
  for (int sub = 0; sub < p.nsub; ++sub) {
    for (int pass = 0; pass < 4; ++pass) {
      const bool xa = (pass & 1) == 0, drift = pass < 2;
      const float al = xa ? p.ax : p.ay;
      for (int q = tid; q < NF; q += bd) {  // face k of line a
        const int a = q / (NV + 1), k = q - a * (NV + 1);
        auto cell = [&](int i) {
          return (i < 0 || i >= NV) ? 0.f : c[xa ? a * NV + i : i * NV + a];
        };
        auto nu = [&](int i) {
          return __builtin_fmaf(-p.beta, (float)(i - H), al);
        };
        auto gp = [&](int i) { return pos(nu(i)) * cell(i); };
        auto gm = [&](int i) { return neg(nu(i)) * cell(i); };
        float fl = 0.f;
        if (k >= 1 && k <= NV - 1) {
          if (drift) {
            float fp = gp(k - 1), fm = gm(k);
            if (p.koren) {
              fp += koren(gp(k) - gp(k - 1), gp(k - 1) - gp(k - 2));
              fm += koren(gm(k - 1) - gm(k), gm(k) - gm(k + 1));
            }
            fl = fp + fm;
          } else {
            fl = p.D * (cell(k - 1) - cell(k));
          }
        }
        tmp[q] = fl;
      }
      __syncthreads();
      for (int q = tid; q < NV * NV; q += bd) {
        const int a = q / NV, i = q - a * NV;
        c[xa ? a * NV + i : i * NV + a] -=
            tmp[a * (NV + 1) + i + 1] - tmp[a * (NV + 1) + i];
      }
      for (int q = tid; q < NF; q += bd) {
        const int a = q / (NV + 1), k = q - a * (NV + 1);
        if (xa)
          Fx[a * (NV + 1) + k] += tmp[q];
        else
          Fy[k * NV + a] += tmp[q];
      }
      __syncthreads();
    }
  }
}

// Stride-4 restriction weight of fine offset o = j - 4J (|o| <= 2), with the
// density factor 1/4 of the 4x wider coarse cell.
__device__ __forceinline__ float rweight(int o) {
  return (o == -2 || o == 2) ? 0.125f : 0.25f;
}

// One workgroup per listed site.  From the streamed fine state g (before
// its collision) of the site: the fine collision with its face fluxes F,
// the coarse face fluxes they imply under the restriction R
// (div_c G = R div F: coarse face k takes the fine faces 4k-2 and 4k-1 on
// either side of the shared fine cell 4k-2, (F_{4k-2} + F_{4k-1}) / 8 per
// fine line, lines combined with R across the other axis), minus the face
// fluxes of the coarse collision of R g: the target fluxes T with
// pred - div T = R (C_f g), pred = C_c (R g).  Features and weights from
// pred, as in k_flux_samples.
template <int NVF, int NVC>
__global__ __launch_bounds__(256) void k_flux_samples_nat(
    CoarseGeom g, CollideCoef cf, CollideCoef cc, float alpha_f,
    float alpha_c, const float* __restrict__ ff, const float* __restrict__ fp,
    const float* __restrict__ u, const int32_t* __restrict__ sites,
    float* __restrict__ X, float* __restrict__ T, float* __restrict__ Wt) {
  static_assert(NVF == 4 * (NVC - 1) + 1, "stride-4 lattices");
  constexpr int NFF = NVF * (NVF + 1), NFC = NVC * (NVC + 1);
  constexpr int NFACE = 2 * NVC * (NVC - 1);
  __shared__ float c[NVF * NVF], tmp[NFF], Fx[NFF], Fy[NFF];
  __shared__ float rc[NVC * NVC], pred[NVC * NVC];
  __shared__ float tx[NVC * (NVC + 1)], ty[(NVC + 1) * NVC];
  __shared__ float msite;
  const int tid = (int)threadIdx.x, bd = (int)blockDim.x;
  const int64_t S = (int64_t)g.nx * g.ny;
  const int site = sites[blockIdx.x];
  const float ux = u[site], uy = u[S + site];
  for (int i = tid; i < NVF * NVF; i += bd) c[i] = ff[(size_t)i * S + site];
  for (int i = tid; i < NVC * NVC; i += bd) pred[i] = fp[(size_t)i * S + site];
  __syncthreads();
  // R g (before the fine collision changes c)
  for (int q = tid; q < NVC * NVC; q += bd) {
    const int Jy = q / NVC, Jx = q - Jy * NVC;
    float acc = 0.f;
    for (int oy = -2; oy <= 2; ++oy) {
      const int jy = 4 * Jy + oy;
      if (jy < 0 || jy >= NVF) continue;
      for (int ox = -2; ox <= 2; ++ox) {
        const int jx = 4 * Jx + ox;
        if (jx < 0 || jx >= NVF) continue;
        acc += rweight(oy) * rweight(ox) * c[jy * NVF + jx];
      }
    }
    rc[q] = acc;
  }
  if (tid == 0) {  // site mass of pred, in a fixed order
    float m = 0.f;
    for (int i = 0; i < NVC * NVC; ++i) m += pred[i];
    msite = m;
  }
  CollideCoef pf = cf;
  pf.ax = ux * alpha_f;
  pf.ay = uy * alpha_f;
  collide_record<NVF>(c, tmp, Fx, Fy, pf);
  // natural coarse fluxes of the fine collision
  for (int q = tid; q < NFC; q += bd) {
    const int a = q / (NVC + 1), k = q - a * (NVC + 1);  // line a, face k
    float gx = 0.f, gy = 0.f;
    if (k >= 1 && k <= NVC - 1) {
      for (int o = -2; o <= 2; ++o) {
        const int j = 4 * a + o;
        if (j < 0 || j >= NVF) continue;
        const float wgt = rweight(o) * 0.125f;
        gx += wgt * (Fx[j * (NVF + 1) + 4 * k - 2] + Fx[j * (NVF + 1) + 4 * k - 1]);
        gy += wgt * (Fy[(4 * k - 2) * NVF + j] + Fy[(4 * k - 1) * NVF + j]);
      }
    }
    tx[a * (NVC + 1) + k] = gx;  // x-faces of row a
    ty[k * NVC + a] = gy;        // y-faces of column a
  }
  __syncthreads();
  // minus the coarse collision's own fluxes (Fx, Fy and tmp reused)
  CollideCoef pc = cc;
  pc.ax = ux * alpha_c;
  pc.ay = uy * alpha_c;
  collide_record<NVC>(rc, tmp, Fx, Fy, pc);
  const size_t base = (size_t)blockIdx.x * NFACE;
  for (int f = tid; f < NFACE; f += bd) {
    float st[5], ms, sg, anu, G;
    if (f < NVC * (NVC - 1)) {  // x-face (row jy, face k)
      const int jy = f / (NVC - 1), k = f - jy * (NVC - 1) + 1;
      auto line = [&](int cc2) { return pred[jy * NVC + cc2]; };
      face_feat(line, NVC, k, ux, g, st, &ms, &sg, &anu);
      G = tx[jy * (NVC + 1) + k] - Fx[jy * (NVC + 1) + k];
    } else {  // y-face (face k, column jx)
      const int q = f - NVC * (NVC - 1);
      const int k = q / NVC + 1, jx = q - (k - 1) * NVC;
      auto line = [&](int cc2) { return pred[cc2 * NVC + jx]; };
      face_feat(line, NVC, k, uy, g, st, &ms, &sg, &anu);
      G = ty[k * NVC + jx] - Fy[k * NVC + jx];
    }
    const bool use = ms > kMinStencilMass && ms >= g.line_eps * msite;
    const float inv = use ? 1.0f / ms : 0.f;
    float* x = X + (base + f) * kNF;
#pragma unroll
    for (int i = 0; i < 5; ++i) x[i] = st[i] * inv;
    x[5] = anu;
    x[6] = g.log_st;
    x[7] = 0.f;
    T[base + f] = use ? sg * G * inv : 0.f;
    Wt[base + f] = use ? ms : 0.f;
  }
}

// --------------------------------------------------------------- training
// Gradients of L = sum_i w_i (y_i - t_i)^2 / sum_i w_i, weights and layer
// inputs rounded to bf16 as in the matrix-core forward (the rounding passed
// straight through).  One wavefront per block walks its share of samples
// 64 at a time: per-sample activations in LDS, then every lane accumulates
// its own parameters (p = lane + 64 m) over the 64 samples.
constexpr int kOwn = (kNParams + 63) / 64;  // 76 parameters per lane

__global__ __launch_bounds__(64) void k_mlp_grad(
    const float* __restrict__ P, const float* __restrict__ X,
    const float* __restrict__ T, const float* __restrict__ Wt, int64_t n,
    float inv_wsum, float* __restrict__ partial, int nblocks) {
  __shared__ float w1[kNF * kNH], b1[kNH], w2[kNH * kNH], b2[kNH], w3[kNH];
  __shared__ float sx[64][kNF + 1];
  __shared__ float sh1[64][kNH + 1], sh2[64][kNH + 1];
  __shared__ float sd1[64][kNH + 1], sd2[64][kNH + 1];
  __shared__ float sdy[64];
  __shared__ float sl[64];
  __shared__ float sacc[kOwn][64];  // this block's gradient, lane-owned
  const int tid = (int)threadIdx.x;
  for (int m = 0; m < kOwn; ++m) sacc[m][tid] = 0.f;
  for (int i = tid; i < kNF * kNH; i += 64) w1[i] = qbf(P[kOffW1 + i]);
  for (int i = tid; i < kNH * kNH; i += 64) w2[i] = qbf(P[kOffW2 + i]);
  for (int i = tid; i < kNH; i += 64) {
    b1[i] = P[kOffB1 + i];
    b2[i] = P[kOffB2 + i];
    w3[i] = qbf(P[kOffW3 + i]);
  }
  const float b3 = P[kOffB3];
  __syncthreads();
  float lsum = 0.f;
  const int64_t lo = n * blockIdx.x / nblocks, hi = n * (blockIdx.x + 1) / nblocks;
  for (int64_t base = lo; base < hi; base += 64) {
    const int64_t i = base + tid;
    const bool valid = i < hi;
    float x[kNF];
#pragma unroll
    for (int k = 0; k < kNF; ++k) x[k] = valid ? qbf(X[i * kNF + k]) : 0.f;
    const float t = valid ? T[i] : 0.f, w = valid ? Wt[i] : 0.f;
    // forward
    float z2[kNH];
#pragma unroll
    for (int j = 0; j < kNH; ++j) z2[j] = b2[j];
    for (int j = 0; j < kNH; ++j) {
      float z = b1[j];
#pragma unroll
      for (int k = 0; k < kNF; ++k) z += x[k] * w1[k * kNH + j];
      float dg;
      const float h = qbf(gelu_d(z, &dg));
      sh1[tid][j] = h;
      sd1[tid][j] = dg;  // gelu'(z1), replaced by dz1 below
#pragma unroll
      for (int q = 0; q < kNH; ++q) z2[q] += h * w2[j * kNH + q];
    }
    float y = b3;
    float dz2[kNH];
#pragma unroll
    for (int j = 0; j < kNH; ++j) {
      float dg;
      const float h = qbf(gelu_d(z2[j], &dg));
      sh2[tid][j] = h;
      y += h * w3[j];
      dz2[j] = dg;
    }
    const float e = y - t;
    lsum += w * e * e * inv_wsum;
    const float dy = 2.0f * w * e * inv_wsum;
    sdy[tid] = dy;
#pragma unroll
    for (int j = 0; j < kNH; ++j) {
      dz2[j] *= dy * w3[j];
      sd2[tid][j] = dz2[j];
    }
    for (int j = 0; j < kNH; ++j) {
      float dh = 0.f;
#pragma unroll
      for (int q = 0; q < kNH; ++q) dh += dz2[q] * w2[j * kNH + q];
      sd1[tid][j] = dh * sd1[tid][j];
    }
#pragma unroll
    for (int k = 0; k < kNF; ++k) sx[tid][k] = x[k];
    __syncthreads();
    // accumulate this lane's parameters over the 64 samples
    for (int m = 0; m < kOwn; ++m) {
      const int p = tid + 64 * m;
      float s = 0.f;
      if (p < kOffB1) {  // W1[k][j]
        const int k = p / kNH, j = p - k * kNH;
        for (int b = 0; b < 64; ++b) s += sx[b][k] * sd1[b][j];
      } else if (p < kOffW2) {  // b1[j]
        const int j = p - kOffB1;
        for (int b = 0; b < 64; ++b) s += sd1[b][j];
      } else if (p < kOffB2) {  // W2[i][j]
        const int q = p - kOffW2, ii = q / kNH, j = q - ii * kNH;
        for (int b = 0; b < 64; ++b) s += sh1[b][ii] * sd2[b][j];
      } else if (p < kOffW3) {  // b2[j]
        const int j = p - kOffB2;
        for (int b = 0; b < 64; ++b) s += sd2[b][j];
      } else if (p < kOffB3) {  // w3[j]
        const int j = p - kOffW3;
        for (int b = 0; b < 64; ++b) s += sh2[b][j] * sdy[b];
      } else if (p == kOffB3) {
        for (int b = 0; b < 64; ++b) s += sdy[b];
      }
      sacc[m][tid] += s;
    }
    __syncthreads();
  }
  float* out = partial + (size_t)blockIdx.x * (kNParams + 1);
  for (int m = 0; m < kOwn; ++m) {
    const int p = tid + 64 * m;
    if (p < kNParams) out[p] = sacc[m][tid];
  }
  sl[tid] = lsum;
  __syncthreads();
  if (tid == 0) {
    float s = 0.f;
    for (int b = 0; b < 64; ++b) s += sl[b];
    out[kNParams] = s;
  }
}

__global__ __launch_bounds__(256) void k_grad_reduce(const float* __restrict__ partial,
                                                     int nblocks,
                                                     float* __restrict__ grad,
                                                     float* __restrict__ loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p > kNParams) return;
  float s = 0.f;
  for (int b = 0; b < nblocks; ++b) s += partial[(size_t)b * (kNParams + 1) + p];
  if (p < kNParams)
    grad[p] = s;
  else
    loss[0] = s;
}

// Adam (Kingma & Ba 2015).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ P,
                                              float* __restrict__ m,
                                              float* __restrict__ v,
                                              const float* __restrict__ g,
                                              int step, float lr, float b1,
                                              float b2, float eps) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= kNParams) return;
  const float gi = g[p];
  const float mi = b1 * m[p] + (1.f - b1) * gi;
  const float vi = b2 * v[p] + (1.f - b2) * gi * gi;
  m[p] = mi;
  v[p] = vi;
  const float mh = mi / (1.f - powf(b1, (float)step));
  const float vh = vi / (1.f - powf(b2, (float)step));
  P[p] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ __launch_bounds__(256) void k_pack_bf16(const float* __restrict__ P,
                                                   uint16_t* __restrict__ wq) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < kNParams) wq[p] = f2bf(P[p]);
}

// ------------------------------------------------------ network forward
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ P,
                                                     const uint16_t* __restrict__ wq,
                                                     const float* __restrict__ X,
                                                     int64_t n,
                                                     float* __restrict__ Y) {
  MlpRegs R;
  load_mlp(R, P, wq);
  const int l = (int)threadIdx.x & 63;
  const int64_t chunk = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6));
  const int64_t i = chunk * 16 + (l & 15);
  const int ks = l >> 4;
  float f[4] = {0.f, 0.f, 0.f, 0.f};
  if (ks < 2 && i < n)
#pragma unroll
    for (int q = 0; q < 4; ++q) f[q] = X[i * kNF + 4 * ks + q];
  const float y = mlp_forward(R, pack4(f[0], f[1], f[2], f[3]));
  if (l < 16 && i < n) Y[i] = y;
}

// ---------------------------------------------------- fused correction
// 17^2 coarse velocities.  A workgroup loads a tile of TS sites (coalesced,
// all 289 planes) into LDS; each wavefront corrects its sites one at a
// time: the interior faces whose 5-cell stencil holds at least line_eps of
// the site's mass (the faces the network is trained on) are gathered into
// a queue (ballot + prefix count), the queue goes through the matrix cores
// 16 faces per pass, the limited fluxes update the site's cells; the tile
// is stored back.
constexpr int kNVC = 17;
constexpr int kTS = 32;

// interior face id -> (axis, line, face): x-faces (line = row Jy, face k
// between columns k-1 | k) first, then y-faces (line = column Jx)
__device__ __forceinline__ void face_of(int fid, int* axis, int* a, int* k) {
  constexpr int NFX = kNVC * (kNVC - 1);
  const int ax = fid >= NFX;
  const int r = fid - ax * NFX;
  *axis = ax;
  *a = r / (kNVC - 1);
  *k = r - *a * (kNVC - 1) + 1;
}

// Three wavefronts per SIMD: the registers are capped at 168 (the weights
// stay in registers, the biases come from LDS) and three workgroups' LDS
// fit in a CU; the per-site steps are latency-bound, so the third
// wavefront pays (measured: 13 % shorter passes than at two).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
void k_mlp_correct17(
    CoarseGeom g, const float* __restrict__ P, const uint16_t* __restrict__ wq,
    float* __restrict__ f, const float* __restrict__ u,
    const int* __restrict__ flag) {
  constexpr int NV = kNVC, N2 = NV * NV;
  constexpr int NFACE = 2 * NV * (NV - 1);
  __shared__ float tile[N2][kTS + 1];
  __shared__ float gx[4][NV][NV + 1];  // x-face fluxes [row][face 0..NV]
  __shared__ float gy[4][NV + 1][NV];  // y-face fluxes [face 0..NV][col]
  __shared__ uint16_t queue[4][NFACE];
  __shared__ float us[2][kTS];  // flow at the tile's sites
  __shared__ __align__(16) float bsh[2][kNH];  // hidden-layer biases
  if (*flag != 0) return;
  const int tid = (int)threadIdx.x, l = tid & 63, w = tid >> 6;
  const int64_t S = (int64_t)g.nx * g.ny;
  const int64_t s0 = (int64_t)blockIdx.x * kTS;
  const int nts = (int)((S - s0) < kTS ? (S - s0) : kTS);
  // every load of a thread is issued before the first LDS write, so the
  // tile costs one memory latency, not one per element.  Thread tid moves
  // site ls of planes lj, lj + JP, ...; loads past the tile's end read
  // plane 0 of a valid site instead and are dropped
  constexpr int JP = 256 / kTS, NL = (N2 + JP - 1) / JP;
  static_assert(256 % kTS == 0, "whole planes per pass");
  const int ls = tid % kTS, lj = tid / kTS;
  const bool lsv = ls < nts;
  const float* const fsite = f + s0 + (lsv ? ls : 0);
  const size_t pstride = (size_t)JP * (size_t)S;
  {
    float v[NL];
    const float* p = fsite + (size_t)lj * (size_t)S;
#pragma unroll
    for (int it = 0; it < NL; ++it) {
      v[it] = *(lj + JP * it < N2 ? p : fsite);
      p += pstride;
    }
    if (tid < 2 * kTS) {
      const int c = tid / kTS, s = tid - c * kTS;
      us[c][s] = s < nts ? u[c * S + s0 + s] : 0.f;
    }
#pragma unroll
    for (int it = 0; it < NL; ++it) {
      const int J = lj + JP * it;
      if (J < N2) tile[J][ls] = lsv ? v[it] : 0.f;
    }
  }
  if (tid < 2 * kNH)
    bsh[tid / kNH][tid % kNH] = P[(tid < kNH ? kOffB1 : kOffB2) + tid % kNH];
  MlpRegs R;
  load_mlp(R, P, wq);
  __syncthreads();
  const int col = l & 15, ks = l >> 4;
  for (int s = w; s < nts; s += 4) {
    const float ux = us[0][s], uy = us[1][s];
    // a face's line as a base and a stride into the tile, so that x- and
    // y-faces in one pass of 16 take the same instructions
    // (24-bit index products: full-rate multiplies)
    const float* const tcol = &tile[0][s];
    auto feat = [&](int fid, float* st, float* ms, float* sg, float* anu) {
      int axis, a, k;
      face_of(fid, &axis, &a, &k);
      const int boff = __umul24(axis == 0 ? a * NV : a, kTS + 1);
      const int soff = axis == 0 ? kTS + 1 : NV * (kTS + 1);
      auto ln = [&](int c) { return tcol[boff + __umul24(c, soff)]; };
      face_feat(ln, NV, k, axis == 0 ? ux : uy, g, st, ms, sg, anu);
    };
    // the faces that get a correction: lanes 0..NV-1 take the rows (x-faces),
    // lanes 32..32+NV-1 the columns (y-faces) of the site; each keeps the
    // prefix sums of its line in registers (Pf[c] = sum of the cells < c)
    // and takes a face's stencil mass from two of them; the site mass sums
    // the row masses in row order
    const bool rl = l < NV, cl = l >= 32 && l < 32 + NV;
    const int la = rl ? l : (cl ? l - 32 : 0);
    float Pf[NV + 1];
    Pf[0] = 0.f;
    {
      const float* lp = &tile[rl ? la * NV : la][s];
      const int lstep = (rl ? 1 : NV) * (kTS + 1);
#pragma unroll
      for (int j = 0; j < NV; ++j) Pf[j + 1] = Pf[j] + lp[j * lstep];
    }
    float M = 0.f;
#pragma unroll
    for (int j = 0; j < NV; ++j)
      M += __int_as_float(
          __builtin_amdgcn_readlane(__float_as_int(Pf[NV]), j));
    const float thr = g.line_eps * M;
    const float uax = rl ? ux : uy;
    const int fbase = (cl ? NV * (NV - 1) : 0) + la * (NV - 1) - 1;
    constexpr int H = (NV - 1) / 2;
    int nq = 0;
#pragma unroll
    for (int k = 1; k < NV; ++k) {
      const float vface = ((float)k - 0.5f - (float)H) * g.dv;
      const float nu = g.nu_scale * (uax - vface);
      // stencil cells lo..lo+4 (lo = k-3 upwind from below, else k-2),
      // clipped to the line
      const float ms = nu >= 0.f
                           ? Pf[k + 2 < NV ? k + 2 : NV] - Pf[k - 3 > 0 ? k - 3 : 0]
                           : Pf[k + 3 < NV ? k + 3 : NV] - Pf[k - 2 > 0 ? k - 2 : 0];
      const bool use = (rl || cl) && ms > kMinStencilMass && ms >= thr;
      const uint64_t b = __ballot(use);
      // lanes below this one with a face (v_mbcnt)
      const int before = (int)__builtin_amdgcn_mbcnt_hi(
          (uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
      if (use) queue[w][nq + before] = (uint16_t)(fbase + k);
      nq += __popcll(b);
    }
    for (int i = l; i < NV * (NV + 1); i += 64) {
      (&gx[w][0][0])[i] = 0.f;
      (&gy[w][0][0])[i] = 0.f;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    for (int c0 = 0; c0 < nq; c0 += 16) {
      const int e = c0 + col;
      const bool live = e < nq;
      const int fid = live ? (int)queue[w][e] : 0;
      float st[5], ms, sg, anu;
      feat(fid, st, &ms, &sg, &anu);
      // 1/m_s to 1 ulp (the features are rounded to bf16 next)
      const float inv = ms > 0.f ? __builtin_amdgcn_rcpf(ms) : 0.f;
      bf16x4 x;
      if (ks == 0 && live)
        x = pack4(st[0] * inv, st[1] * inv, st[2] * inv, st[3] * inv);
      else if (ks == 1 && live)
        x = pack4(st[4] * inv, anu, g.log_st, 0.f);
      else
        x = pack4(0.f, 0.f, 0.f, 0.f);
      const float y = mlp_forward_lds(R, bsh[0], bsh[1], x);
      if (l < 16 && live) {
        int axis, a, k;
        face_of(fid, &axis, &a, &k);
        float G = sg * ms * y;
        const int boff = __umul24(axis == 0 ? a * NV : a, kTS + 1);
        const int soff = axis == 0 ? kTS + 1 : NV * (kTS + 1);
        const float donor = tcol[boff + __umul24(G > 0.f ? k - 1 : k, soff)];
        const float cap = 0.25f * donor;
        G = G > cap ? cap : (G < -cap ? -cap : G);
        *(axis == 0 ? &gx[w][a][k] : &gy[w][k][a]) = G;
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
#pragma unroll
    for (int it = 0; it < (N2 + 63) / 64; ++it) {
      const int J = l + 64 * it;
      if (J < N2) {
        const int jy = J / NV, jx = J - jy * NV;
        tile[J][s] -= (gx[w][jy][jx + 1] - gx[w][jy][jx]) +
                      (gy[w][jy + 1][jx] - gy[w][jy][jx]);
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  }
  __syncthreads();
  {
    float v[NL];
#pragma unroll
    for (int it = 0; it < NL; ++it) {
      const int J = lj + JP * it;
      v[it] = J < N2 ? tile[J][ls] : 0.f;
    }
    float* p = f + s0 + ls + (size_t)lj * (size_t)S;
#pragma unroll
    for (int it = 0; it < NL; ++it) {
      if (lsv && lj + JP * it < N2) *p = v[it];
      p += pstride;
    }
  }
}

}  // namespace

hipError_t launch_restrict(int dim, int64_t sites, int nv_fine,
                           const float* ff, float* fc, hipStream_t s) {
  if ((nv_fine - 1) % 4 || nv_fine < 5) return hipErrorInvalidValue;
  const int nvc = (nv_fine - 1) / 4 + 1;
  const int gx = (int)((sites + 255) / 256);
  if (dim == 1)
    hipLaunchKernelGGL(k_restrict1d, dim3(gx, nvc), dim3(256), 0, s, ff, fc,
                       sites, nv_fine);
  else
    hipLaunchKernelGGL(k_restrict2d, dim3(gx, nvc * nvc), dim3(256), 0, s, ff,
                       fc, sites, nv_fine);
  return hipGetLastError();
}

hipError_t launch_flux_samples(const CoarseGeom& g, const float* f_pred,
                               const float* f_true, const float* u,
                               const int32_t* sites, int nsites, float* X,
                               float* t, float* w, hipStream_t s) {
  if (g.nv != kNVC || nsites < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_flux_samples<kNVC>, dim3(nsites), dim3(320), 0, s, g,
                     f_pred, f_true, u, sites, X, t, w);
  return hipGetLastError();
}

hipError_t launch_flux_samples_natural(
    const CoarseGeom& g, const NaturalCoef& nc, const float* f_fine,
    const float* f_pred, const float* u, const int32_t* sites, int nsites,
    float* X, float* t, float* w, hipStream_t s) {
  if (g.nv != kNVC || nc.nv_fine != 4 * (kNVC - 1) + 1 || nsites < 1)
    return hipErrorInvalidValue;
  CollideCoef cf{0.f, 0.f, nc.beta_f, nc.D_f, nc.nsub_f, nc.koren_f};
  CollideCoef cc{0.f, 0.f, nc.beta_c, nc.D_c, nc.nsub_c, nc.koren_c};
  hipLaunchKernelGGL((k_flux_samples_nat<4 * (kNVC - 1) + 1, kNVC>),
                     dim3(nsites), dim3(256), 0, s, g, cf, cc, nc.alpha_f,
                     nc.alpha_c, f_fine, f_pred, u, sites, X, t, w);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* params, const float* X,
                           const float* t, const float* w, int64_t n,
                           double wsum, float* partial, int nblocks,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_grad, dim3(nblocks), dim3(64), 0, s, params, X, t,
                     w, n, (float)(1.0 / wsum), partial, nblocks);
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const float* partial, int nblocks, float* grad,
                              float* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_reduce, dim3((kNParams + 1 + 255) / 256),
                     dim3(256), 0, s, partial, nblocks, grad, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* params, float* m, float* v, const float* grad,
                       int step, float lr, float b1, float b2, float eps,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((kNParams + 255) / 256), dim3(256), 0, s,
                     params, m, v, grad, step, lr, b1, b2, eps);
  return hipGetLastError();
}

hipError_t launch_pack_bf16(const float* params, uint16_t* wq, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_bf16, dim3((kNParams + 255) / 256), dim3(256), 0,
                     s, params, wq);
  return hipGetLastError();
}

hipError_t launch_mlp_correct(const CoarseGeom& g, const float* params,
                              const uint16_t* wq, float* f, const float* u,
                              const int* flag, hipStream_t s) {
  if (g.nv != kNVC) return hipErrorInvalidValue;
  const int64_t S = (int64_t)g.nx * g.ny;
  const int grid = (int)((S + kTS - 1) / kTS);
  hipLaunchKernelGGL(k_mlp_correct17, dim3(grid), dim3(256), 0, s, g, params,
                     wq, f, u, flag);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* params, const uint16_t* wq,
                              const float* X, int64_t n, float* y,
                              hipStream_t s) {
  const int64_t chunks = (n + 15) / 16;
  const int grid = (int)((chunks + 3) / 4);
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(256), 0, s, params, wq, X,
                     n, y);
  return hipGetLastError();
}

}  // namespace lat
