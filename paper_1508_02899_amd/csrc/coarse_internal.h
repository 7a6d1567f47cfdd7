// coarse_internal.h -- launch interface of the coarse-velocity-lattice form
// with the learned face-flux correction (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lat {

// Parameter packing of the correction network (FP32 master copy):
//   W1[8][64], b1[64], W2[64][64], b2[64], w3[64], b3
constexpr int kNF = 8;    // input features (7 used + 1 zero pad)
constexpr int kNH = 64;   // hidden width
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kNF * kNH;
constexpr int kOffW2 = kOffB1 + kNH;
constexpr int kOffB2 = kOffW2 + kNH * kNH;
constexpr int kOffW3 = kOffB2 + kNH;
constexpr int kOffB3 = kOffW3 + kNH;
constexpr int kNParams = kOffB3 + 1;  // 4801

// Geometry of a coarse 2D lattice seen by the correction / sampling kernels.
struct CoarseGeom {
  int nx, ny, nv;
  float dv;       // coarse velocity spacing
  float nu_scale; // dt / (tau_p dv): face drift per unit of (u - v_face)
  float log_st;   // ln St
  float line_eps; // lines with less than line_eps x site mass are skipped
};

hipError_t launch_restrict(int dim, int64_t sites, int nv_fine,
                           const float* ff, float* fc, hipStream_t s);

// Training samples of the face-flux correction at the listed sites:
// residual r = f_true - f_pred, minimum-norm face fluxes G with
// -div G = r, features of every interior face from f_pred and u.
// Outputs per site (2 nv (nv-1) faces): X[face][8], t[face], w[face].
hipError_t launch_flux_samples(const CoarseGeom& g, const float* f_pred,
                               const float* f_true, const float* u,
                               const int32_t* sites, int nsites, float* X,
                               float* t, float* w, hipStream_t s);

// Collision coefficients of a fine lattice and of its stride-4 coarse
// lattice for the natural-flux training targets: alpha = dt_s / (dv tau_p)
// (times u: drift of the zero-velocity cell), beta = dt_s / tau_p,
// D = kappa dt_s / dv^2, nsub sub-steps, Koren (1) or upwind (0).
struct NaturalCoef {
  int nv_fine;
  float alpha_f, beta_f, D_f;
  int nsub_f, koren_f;
  float alpha_c, beta_c, D_c;
  int nsub_c, koren_c;
};

// Training samples with natural targets: from the streamed fine state
// f_fine (before its collision; [nv_f^2][ny][nx]) and pred = the coarse
// collision of its restriction ([nv_c^2][ny][nx]), per listed site and
// interior coarse face: the coarse fluxes implied by the fine collision's
// face fluxes under the restriction, minus the coarse collision's fluxes.
// Same outputs as launch_flux_samples.
hipError_t launch_flux_samples_natural(
    const CoarseGeom& g, const NaturalCoef& nc, const float* f_fine,
    const float* f_pred, const float* u, const int32_t* sites, int nsites,
    float* X, float* t, float* w, hipStream_t s);

// Per-wavefront partial sums of the loss gradient (matrix cores): nrows
// rows of kNParams + 1 floats (gradient, then the row's loss sum), one per
// wavefront; mlp_grad_rows gives the row count for n samples (at most
// max_rows).
int mlp_grad_rows(int64_t n, int max_rows);
hipError_t launch_mlp_grad_mfma(const float* params, const float* X,
                                const float* t, const float* w, int64_t n,
                                double wsum, float* partial, int nrows,
                                hipStream_t s);
// Sum of the partial rows in a fixed order into grad[kNParams] and loss[0];
// the _adam form then applies one Adam step (step >= 1) to params.
hipError_t launch_grad_reduce_adam(const float* partial, int nrows,
                                   float* grad, float* loss, float* params,
                                   float* m, float* v, int step, float lr,
                                   float b1, float b2, float eps,
                                   hipStream_t s);
hipError_t launch_grad_reduce(const float* partial, int nrows, float* grad,
                              float* loss, hipStream_t s);
// bf16 copies of the weights for the matrix-core forward pass.
hipError_t launch_pack_bf16(const float* params, uint16_t* wq, hipStream_t s);

// In-place learned correction of a coarse 2D state f[nv*nv][ny][nx]
// (nv = 17): per site, per velocity line, the network's face fluxes,
// limited to a quarter of the donor cell, applied conservatively.
hipError_t launch_mlp_correct(const CoarseGeom& g, const float* params,
                              const uint16_t* wq, float* f, const float* u,
                              const int* flag, hipStream_t s);
// Forward pass only (network outputs for X[n][8]) -- for checks.
hipError_t launch_mlp_forward(const float* params, const uint16_t* wq,
                              const float* X, int64_t n, float* y,
                              hipStream_t s);

}  // namespace lat
