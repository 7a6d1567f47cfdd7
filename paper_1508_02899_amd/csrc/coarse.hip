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

// 16x16x32 bf16 matrix-core product (gfx950), FP32 accumulation: A lane l
// holds row l%16, K indices 8(l/16)+i; B lane l holds column l%16, the
// same K indices; the result lane l holds rows 4(l/16)+r of column l%16.
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mfma32(s16x8 a, s16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(
      __builtin_bit_cast(bf16x8v, a), __builtin_bit_cast(bf16x8v, b), c, 0, 0,
      0);
}
// K index i (0..7) of K step kk for lane group g -> unit of the 64-wide
// hidden layer (two stacked output tiles, see above)
__device__ __forceinline__ int kunit(int kk, int g, int i) {
  return 32 * kk + (i < 4 ? 4 * g + i : 16 + 4 * g + (i - 4));
}
__device__ __forceinline__ short bfs(float f) { return (short)f2bf(f); }
// two stacked 16-row output tiles as one 16x16x32 K operand
__device__ __forceinline__ s16x8 cat8(bf16x4 p, bf16x4 q) {
  return s16x8{p[0], p[1], p[2], p[3], q[0], q[1], q[2], q[3]};
}

// The network in matrix-core form.  16 inputs (faces) per wavefront pass;
// each layer is computed transposed, D = W^T X^T.  Layer 1 (K = 8
// features) is a 16x16x16 product whose B operand is the input; the 64
// hidden units of a layer come out as four 16x16 tiles (lane l: rows
// 4(l/16)+r of column l%16), and two of them (units u and u+16 of a 32-unit
// K step) are the B operand of a 16x16x32 product when its K index
// 8(l/16)+i names unit kunit(kk, l/16, i); the weight operands are loaded
// in that K order.
struct MlpRegs {
  bf16x4 a1[4];      // W1^T tiles (units 16u.., features)
  s16x8 a2[4][2];    // W2^T tiles [unit tile][K step of 32 units]
  s16x8 a3[2];       // w3 as row 0 of a 16-row A operand, per K step
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
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int i = 0; i < 8; ++i)
        R.a2[u][kk][i] =
            (short)wq[kOffW2 + kunit(kk, ks, i) * kNH + 16 * u + col];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      R.b1[u][i] = P[kOffB1 + 16 * u + 4 * ks + i];
      R.b2[u][i] = P[kOffB2 + 16 * u + 4 * ks + i];
    }
  }
#pragma unroll
  for (int kk = 0; kk < 2; ++kk)
#pragma unroll
    for (int i = 0; i < 8; ++i)
      R.a3[kk][i] =
          col == 0 ? (short)wq[kOffW3 + kunit(kk, ks, i)] : (short)0;
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
    for (int kk = 0; kk < 2; ++kk)
      d = mfma32(R.a2[u][kk], cat8(h1[2 * kk], h1[2 * kk + 1]), d);
    h2[u] = pack4(gelu(d[0]), gelu(d[1]), gelu(d[2]), gelu(d[3]));
  }
  f32x4 y = {R.b3, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kk = 0; kk < 2; ++kk)
    y = mfma32(R.a3[kk], cat8(h2[2 * kk], h2[2 * kk + 1]), y);
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
    for (int kk = 0; kk < 2; ++kk)
      d = mfma32(R.a2[u][kk], cat8(h1[2 * kk], h1[2 * kk + 1]), d);
    h2[u] = pack4(gelu(d[0]), gelu(d[1]), gelu(d[2]), gelu(d[3]));
  }
  f32x4 y = {R.b3, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kk = 0; kk < 2; ++kk)
    y = mfma32(R.a3[kk], cat8(h2[2 * kk], h2[2 * kk + 1]), y);
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
// straight through).
// ---------------------------------------------------- training, matrix cores
// The same gradients on the matrix cores (gfx950 v_mfma_f32_16x16x32_bf16,
// FP32 accumulation).  Every product pairs an operand that is a bf16 value
// by definition of the network (the rounded weights, layer inputs and
// activations) with one that is FP32 in the definition (the backward
// signals dz); the latter enters as two bf16 operands, hi = bf16(dz) and
// lo = bf16(dz - hi), i.e. about 16 significant bits, so the products match
// the FP32 arithmetic of the definition to ~2^-17 relative.
//
// A wavefront takes 32 samples at a time (two 16-sample column tiles).  The
// forward and the backward-data products run transposed (units x samples,
// as in the inference kernel): the 16x16 output tile of one layer, lane l
// holding rows 4(l/16)+r, r < 4, of column l%16, is the B operand of the
// next product once two tiles (rows u and u+16 of a 32-row K step) are
// read as K indices 8(l/16)+i, i < 8 -- the weight operand is loaded in the
// same K order.  The weight gradients sum over the samples (K = the 32
// samples of the step): the activations and signals go through a
// per-wavefront LDS transpose ([unit][sample], bf16).  Each wavefront writes
// one row of per-parameter sums (then the block order reduction).

constexpr int kGS = 32;                 // samples per wavefront step
constexpr int kGP = kGS + 8;            // LDS row pitch (bf16), 80 bytes
constexpr int kGWaves = 4;              // wavefronts per block
// per wavefront: H1 / (X^T, 16 rows) and the hi / lo signals, [row][sample]
constexpr int kGLds = (kNH + kNH + kNH + 16) * kGP;

__global__ __launch_bounds__(64 * kGWaves) void k_mlp_grad_mfma(
    const float* __restrict__ P, const float* __restrict__ X,
    const float* __restrict__ T, const float* __restrict__ Wt, int64_t n,
    float inv_wsum, float* __restrict__ partial, int nrows) {
  __shared__ __attribute__((aligned(16))) short lds[kGWaves * kGLds];
  const int wv = (int)threadIdx.x >> 6;
  const int row = (int)blockIdx.x * kGWaves + wv;  // partial row of this wave
  if (row >= nrows) return;  // wave-uniform; no block barrier below
  short* sH = lds + wv * kGLds;           // [64][kGP]: h1, later unused
  short* sHi = sH + kNH * kGP;            // [64][kGP]: dz2 hi, then dz1 hi
  short* sLo = sHi + kNH * kGP;           // [64][kGP]: dz2 lo, then dz1 lo
  short* sX = sLo + kNH * kGP;            // [16][kGP]: x^T, row 8 = ones
  const int l = (int)threadIdx.x & 63;
  const int c = l & 15, g = l >> 4;

  // ---- weights (bf16 as the network defines them) and biases
  bf16x4 a1[4];          // W1^T, K = features 4g + r
  s16x8 a2[4][2];        // W2^T: rows = output units, K = input units
  s16x8 a2t[4][2];       // W2:   rows = input units,  K = output units
  float w3q[4][4], b1r[4][4], b2r[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 4 * g + r;
      a1[u][r] = k < kNF ? bfs(P[kOffW1 + k * kNH + 16 * u + c]) : (short)0;
      const int unit = 16 * u + 4 * g + r;
      w3q[u][r] = qbf(P[kOffW3 + unit]);
      b1r[u][r] = P[kOffB1 + unit];
      b2r[u][r] = P[kOffB2 + unit];
    }
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int ku = kunit(kk, g, i);
        a2[u][kk][i] = bfs(P[kOffW2 + ku * kNH + 16 * u + c]);
        a2t[u][kk][i] = bfs(P[kOffW2 + (16 * u + c) * kNH + ku]);
      }
  }
  const float b3 = P[kOffB3];
  // rows 8..15 of x^T: ones (row 8, for the b1 gradient) and zeros
  for (int i = l; i < 8 * kGP; i += 64)
    sX[8 * kGP + i] = (i < kGP) ? bfs(1.0f) : (short)0;

  f32x4 gW2[4][4], gW1[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    gW1[a] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 4; ++b) gW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  float gb2[4][4] = {}, gw3[4][4] = {};
  float gb3 = 0.f, lsum = 0.f;

  const int64_t lo = n * row / nrows, hi = n * (row + 1) / nrows;
  for (int64_t s0 = lo; s0 < hi; s0 += kGS) {
    // ---- inputs of the two column tiles (sample s0 + 16 t + c)
    bf16x4 xb[2];
    float tt[2], ww[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int64_t i = s0 + 16 * t + c;
      const bool ok = i < hi;
      float xf[4] = {0.f, 0.f, 0.f, 0.f};
      if (ok && g < 2)
#pragma unroll
        for (int r = 0; r < 4; ++r) xf[r] = X[i * kNF + 4 * g + r];
      tt[t] = ok ? T[i] : 0.f;
      ww[t] = ok ? Wt[i] : 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        xb[t][r] = bfs(xf[r]);
        if (g < 2) sX[(4 * g + r) * kGP + 16 * t + c] = xb[t][r];
      }
    }
    // ---- layer 1 (K = 8 features, 16x16x16) and GELU
    float gd1[4][2][4];
    bf16x4 h1[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const f32x4 b = {b1r[u][0], b1r[u][1], b1r[u][2], b1r[u][3]};
        const f32x4 z = mfma16(a1[u], xb[t], b);
        float h[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float dg;
          h[r] = gelu_d(z[r], &dg);
          gd1[u][t][r] = dg;
        }
        h1[u][t] = pack4(h[0], h[1], h[2], h[3]);
#pragma unroll
        for (int r = 0; r < 4; ++r)
          sH[(16 * u + 4 * g + r) * kGP + 16 * t + c] = h1[u][t][r];
      }
    // ---- layer 2 (K = 64, 16x16x32) and GELU
    float gd2[4][2][4], h2[4][2][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        f32x4 z = {b2r[m][0], b2r[m][1], b2r[m][2], b2r[m][3]};
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
          z = mfma32(a2[m][kk], cat8(h1[2 * kk][t], h1[2 * kk + 1][t]), z);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float dg;
          h2[m][t][r] = qbf(gelu_d(z[r], &dg));
          gd2[m][t][r] = dg;
        }
      }
    // ---- output, loss, dy (each sample's four lane groups agree)
    float dy[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      float part = 0.f;
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) part += h2[m][t][r] * w3q[m][r];
      part += __shfl_xor(part, 16);
      part += __shfl_xor(part, 32);
      const float y = b3 + part;
      const float e = y - tt[t];
      if (g == 0) {
        lsum += ww[t] * e * e * inv_wsum;
      }
      dy[t] = 2.0f * ww[t] * e * inv_wsum;
      if (g == 0) gb3 += dy[t];
    }
    // ---- backward through layer 3 and the second GELU
    s16x8 dhi[4][2], dlo[4][2];  // dz2 as K operands: [K step][t] below
    float dz2[4][2][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float d = w3q[m][r] * dy[t] * gd2[m][t][r];
          dz2[m][t][r] = d;
          gb2[m][r] += d;
          gw3[m][r] += h2[m][t][r] * dy[t];
          const short hs = bfs(d);
          const short ls = bfs(d - bf2f((uint16_t)hs));
          sHi[(16 * m + 4 * g + r) * kGP + 16 * t + c] = hs;
          sLo[(16 * m + 4 * g + r) * kGP + 16 * t + c] = ls;
        }
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float d = dz2[2 * kk + (i >> 2)][t][i & 3];
          const short hs = bfs(d);
          dhi[kk][t][i] = hs;
          dlo[kk][t][i] = bfs(d - bf2f((uint16_t)hs));
        }
    // ---- weight gradient of layer 2: sum over the 32 samples
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const s16x8 ah = *(const s16x8*)(sH + (16 * a + c) * kGP + 8 * g);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const s16x8 bh = *(const s16x8*)(sHi + (16 * b + c) * kGP + 8 * g);
        const s16x8 bl = *(const s16x8*)(sLo + (16 * b + c) * kGP + 8 * g);
        gW2[a][b] = mfma32(ah, bh, gW2[a][b]);
        gW2[a][b] = mfma32(ah, bl, gW2[a][b]);
      }
    }
    // ---- backward through layer 2 (K = 64 output units) and the first GELU
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        f32x4 dh = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
          dh = mfma32(a2t[m][kk], dhi[kk][t], dh);
          dh = mfma32(a2t[m][kk], dlo[kk][t], dh);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float d = dh[r] * gd1[m][t][r];
          const short hs = bfs(d);
          sHi[(16 * m + 4 * g + r) * kGP + 16 * t + c] = hs;
          sLo[(16 * m + 4 * g + r) * kGP + 16 * t + c] =
              bfs(d - bf2f((uint16_t)hs));
        }
      }
    // ---- weight gradient of layer 1 (rows: 8 features, ones, zeros)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    {
      const s16x8 ax = *(const s16x8*)(sX + c * kGP + 8 * g);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const s16x8 bh = *(const s16x8*)(sHi + (16 * b + c) * kGP + 8 * g);
        const s16x8 bl = *(const s16x8*)(sLo + (16 * b + c) * kGP + 8 * g);
        gW1[b] = mfma32(ax, bh, gW1[b]);
        gW1[b] = mfma32(ax, bl, gW1[b]);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
  }

  // ---- this wavefront's row of per-parameter sums
  float* out = partial + (size_t)row * (kNParams + 1);
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 4 * g + r, j = 16 * b + c;
      if (k < kNF) out[kOffW1 + k * kNH + j] = gW1[b][r];
      if (k == kNF) out[kOffB1 + j] = gW1[b][r];   // the ones row
#pragma unroll
      for (int a = 0; a < 4; ++a)
        out[kOffW2 + (16 * a + 4 * g + r) * kNH + j] = gW2[a][b][r];
    }
  // per-unit sums over the 16 sample lanes of each lane group
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float sb = gb2[m][r], sw = gw3[m][r];
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) {
        sb += __shfl_xor(sb, o);
        sw += __shfl_xor(sw, o);
      }
      if (c == 0) {
        out[kOffB2 + 16 * m + 4 * g + r] = sb;
        out[kOffW3 + 16 * m + 4 * g + r] = sw;
      }
    }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    gb3 += __shfl_xor(gb3, o);
    lsum += __shfl_xor(lsum, o);
  }
  if (l == 0) {
    out[kOffB3] = gb3;
    out[kNParams] = lsum;
  }
}

// Sum of the partial rows, fixed order: a block takes 64 consecutive
// entries (coalesced row reads); its eight wavefronts sum rows q, q+8, ...
// (q = wavefront) and the eight sums are added pairwise in a fixed order.
// With adam_step > 0 the Adam update (Kingma & Ba 2015) of those
// parameters follows at once.
constexpr int kRedWaves = 8;
__global__ __launch_bounds__(64 * kRedWaves) void k_grad_reduce(
    const float* __restrict__ partial, int nrows, float* __restrict__ grad,
    float* __restrict__ loss, float* __restrict__ P, float* __restrict__ m,
    float* __restrict__ v, int adam_step, float lr, float b1, float b2,
    float eps) {
  __shared__ float sh[kRedWaves][64];
  const int q = (int)threadIdx.x >> 6, j = (int)threadIdx.x & 63;
  const int p = (int)blockIdx.x * 64 + j;
  float s = 0.f;
  if (p <= kNParams) {
    // the loads of eight rows in flight together, added in row order
    const float* col = partial + p;
    const size_t rs = (size_t)kRedWaves * (kNParams + 1);
    int r = q;
    for (; r + 7 * kRedWaves < nrows; r += 8 * kRedWaves) {
      float v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = col[(size_t)r * (kNParams + 1) + k * rs];
#pragma unroll
      for (int k = 0; k < 8; ++k) s += v[k];
    }
    for (; r < nrows; r += kRedWaves) s += col[(size_t)r * (kNParams + 1)];
  }
  sh[q][j] = s;
  __syncthreads();
  if (q != 0 || p > kNParams) return;
  const float gi = ((sh[0][j] + sh[1][j]) + (sh[2][j] + sh[3][j])) +
                   ((sh[4][j] + sh[5][j]) + (sh[6][j] + sh[7][j]));
  if (p == kNParams) {
    loss[0] = gi;
    return;
  }
  grad[p] = gi;
  if (adam_step > 0) {
    const float mi = b1 * m[p] + (1.f - b1) * gi;
    const float vi = b2 * v[p] + (1.f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    const float mh = mi / (1.f - powf(b1, (float)adam_step));
    const float vh = vi / (1.f - powf(b2, (float)adam_step));
    P[p] -= lr * mh / (sqrtf(vh) + eps);
  }
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

// one 32-sample step per wavefront at least: a minibatch of 8192 samples
// is then 256 wavefronts (64 workgroups), 19.5 us; with two steps per
// wavefront the grid halves and the pass takes 25.5 us, more than the
// summation of the extra partial rows saves
int mlp_grad_rows(int64_t n, int max_rows) {
  int64_t r = (n + kGS - 1) / kGS;
  if (r > max_rows) r = max_rows;
  return r < 1 ? 1 : (int)r;
}

hipError_t launch_mlp_grad_mfma(const float* params, const float* X,
                                const float* t, const float* w, int64_t n,
                                double wsum, float* partial, int nrows,
                                hipStream_t s) {
  const int blocks = (nrows + kGWaves - 1) / kGWaves;
  hipLaunchKernelGGL(k_mlp_grad_mfma, dim3(blocks), dim3(64 * kGWaves), 0, s,
                     params, X, t, w, n, (float)(1.0 / wsum), partial, nrows);
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const float* partial, int nrows, float* grad,
                              float* loss, hipStream_t s) {
  hipLaunchKernelGGL(k_grad_reduce, dim3((kNParams + 1 + 63) / 64),
                     dim3(64 * kRedWaves), 0, s, partial, nrows, grad, loss,
                     (float*)nullptr,
                     (float*)nullptr, (float*)nullptr, 0, 0.f, 0.f, 0.f, 0.f);
  return hipGetLastError();
}

hipError_t launch_grad_reduce_adam(const float* partial, int nrows,
                                   float* grad, float* loss, float* params,
                                   float* m, float* v, int step, float lr,
                                   float b1, float b2, float eps,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_grad_reduce, dim3((kNParams + 1 + 63) / 64),
                     dim3(64 * kRedWaves), 0, s, partial, nrows, grad, loss,
                     params, m, v, step, lr, b1, b2, eps);
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
