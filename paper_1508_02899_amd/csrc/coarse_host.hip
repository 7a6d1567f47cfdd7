// coarse_host.hip -- C ABI of the coarse velocity lattice with the learned
// face-flux correction: restriction, training samples, the network's
// parameters, gradients, Adam training loop and forward pass.
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "../../include/lattice.h"
#include "coarse_internal.h"
#include "lattice_internal.h"
#include "lattice_struct.h"

struct lattice_mlp {
  hipStream_t stream = nullptr;
  float* params = nullptr;    // FP32 master copy (kNParams)
  uint16_t* wq = nullptr;     // bf16 copy for the matrix-core forward
  float* grad = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  float* loss = nullptr;      // 1 float
  float* partial = nullptr;   // nblocks x (kNParams + 1)
  int max_blocks = 256;
  int adam_t = 0;
  float* host_loss = nullptr;  // pinned
};

namespace {

hipError_t mlp_sync_bf16(lattice_mlp_t* M) {
  return lat::launch_pack_bf16(M->params, M->wq, M->stream);
}

// sum of w[0..n) on the device (one-off, synchronous)
hipError_t device_sum(const float* w, int64_t n, hipStream_t s, double* out) {
  std::vector<float> h((size_t)n);
  hipError_t e = hipMemcpyAsync(h.data(), w, sizeof(float) * n,
                                hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return e;
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  double acc = 0.0;
  for (float x : h) acc += x;
  *out = acc;
  return hipSuccess;
}


}  // namespace

extern "C" {

int lattice_restrict(int32_t dim, int64_t sites, int32_t nv_fine,
                     const float* f_fine, float* f_coarse, void* stream) {
  if ((dim != 1 && dim != 2) || sites < 1 || nv_fine < 5 ||
      (nv_fine - 1) % 4 || !f_fine || !f_coarse)
    return LATTICE_EINVAL;
  if (lat::launch_restrict(dim, sites, nv_fine, f_fine, f_coarse,
                           (hipStream_t)stream) != hipSuccess)
    return LATTICE_EHIP;
  return LATTICE_OK;
}

int lattice_mlp_create(void* stream, lattice_mlp_t** out) {
  if (!out) return LATTICE_EINVAL;
  *out = nullptr;
  lattice_mlp_t* M = new (std::nothrow) lattice_mlp;
  if (!M) return LATTICE_ENOMEM;
  M->stream = (hipStream_t)stream;
  const size_t np = lat::kNParams;
  if (hipMalloc(&M->params, sizeof(float) * np) != hipSuccess ||
      hipMalloc(&M->wq, sizeof(uint16_t) * np) != hipSuccess ||
      hipMalloc(&M->grad, sizeof(float) * np) != hipSuccess ||
      hipMalloc(&M->m, sizeof(float) * np) != hipSuccess ||
      hipMalloc(&M->v, sizeof(float) * np) != hipSuccess ||
      hipMalloc(&M->loss, sizeof(float)) != hipSuccess ||
      hipMalloc(&M->partial,
                sizeof(float) * (np + 1) * M->max_blocks) != hipSuccess ||
      hipHostMalloc((void**)&M->host_loss, sizeof(float),
                    hipHostMallocDefault) != hipSuccess) {
    lattice_mlp_destroy(M);
    return LATTICE_ENOMEM;
  }
  std::vector<float> zero(np, 0.f);
  if (hipMemcpy(M->params, zero.data(), sizeof(float) * np,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(M->m, zero.data(), sizeof(float) * np,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(M->v, zero.data(), sizeof(float) * np,
                hipMemcpyHostToDevice) != hipSuccess ||
      mlp_sync_bf16(M) != hipSuccess ||
      hipStreamSynchronize(M->stream) != hipSuccess) {
    lattice_mlp_destroy(M);
    return LATTICE_EHIP;
  }
  *out = M;
  return LATTICE_OK;
}

int lattice_mlp_set_params(lattice_mlp_t* M, const float* host_params) {
  if (!M || !host_params) return LATTICE_EINVAL;
  if (hipMemcpyAsync(M->params, host_params, sizeof(float) * lat::kNParams,
                     hipMemcpyHostToDevice, M->stream) != hipSuccess ||
      mlp_sync_bf16(M) != hipSuccess ||
      hipStreamSynchronize(M->stream) != hipSuccess)
    return LATTICE_EHIP;
  M->adam_t = 0;
  std::vector<float> zero(lat::kNParams, 0.f);
  if (hipMemcpy(M->m, zero.data(), sizeof(float) * lat::kNParams,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(M->v, zero.data(), sizeof(float) * lat::kNParams,
                hipMemcpyHostToDevice) != hipSuccess)
    return LATTICE_EHIP;
  return LATTICE_OK;
}

int lattice_mlp_get_params(lattice_mlp_t* M, float* host_params) {
  if (!M || !host_params) return LATTICE_EINVAL;
  if (hipMemcpyAsync(host_params, M->params, sizeof(float) * lat::kNParams,
                     hipMemcpyDeviceToHost, M->stream) != hipSuccess ||
      hipStreamSynchronize(M->stream) != hipSuccess)
    return LATTICE_EHIP;
  return LATTICE_OK;
}

int lattice_mlp_samples(lattice_t* L, double dt, double tau_p, double St,
                        double rel_eps, const float* f_pred, const float* f_true,
                        const float* u, const int32_t* sites, int64_t nsites,
                        float* X, float* t, float* w) {
  if (!L || !f_pred || !f_true || !u || !sites || !X || !t || !w ||
      nsites < 1 || nsites > (1 << 30) || !(dt > 0) || !(tau_p > 0) ||
      !(St > 0) || !(rel_eps >= 0) || !(rel_eps < 1))
    return LATTICE_EINVAL;
  const lattice_desc& d = L->d;
  if (d.dim != 2 || d.nv != 17 || d.dtype != LATTICE_F32 ||
      L->pitch != L->sites)  // the network kernels read contiguous states
    return LATTICE_ENOTSUP;
  lat::CoarseGeom g;
  g.nx = (int)d.nx;
  g.ny = (int)d.ny;
  g.nv = d.nv;
  const double dv = d.vstride * d.dx / dt;
  g.dv = (float)dv;
  g.nu_scale = (float)(dt / (tau_p * dv));
  g.log_st = (float)log(St);
  g.line_eps = (float)rel_eps;
  if (lat::launch_flux_samples(g, f_pred, f_true, u, sites, (int)nsites, X, t,
                               w, L->stream) != hipSuccess)
    return LATTICE_EHIP;
  return LATTICE_OK;
}

int lattice_mlp_samples_natural(const lattice_t* fine, lattice_t* L,
                                double dt, double tau_p, double kappa,
                                double St, double rel_eps,
                                const float* f_fine, const float* f_pred,
                                const float* u, const int32_t* sites,
                                int64_t nsites, float* X, float* t, float* w) {
  if (!fine || !L || !f_fine || !f_pred || !u || !sites || !X || !t || !w ||
      nsites < 1 || nsites > (1 << 30) || !(dt > 0) || !isfinite(dt) ||
      !(tau_p > 0) || !isfinite(tau_p) || !(kappa >= 0) ||
      !isfinite(kappa) || !(St > 0) || !(rel_eps >= 0) || !(rel_eps < 1))
    return LATTICE_EINVAL;
  const lattice_desc& d = L->d;
  const lattice_desc& e = fine->d;
  if (d.dim != 2 || d.nv != 17 || d.dtype != LATTICE_F32 || e.dim != 2 ||
      e.nv != 65 || e.dtype != LATTICE_F32 || L->pitch != L->sites ||
      fine->pitch != fine->sites)  // the network kernels read contiguous states
    return LATTICE_ENOTSUP;
  if (e.nx != d.nx || e.ny != d.ny || e.dx != d.dx ||
      d.vstride != 4 * e.vstride)
    return LATTICE_EINVAL;  // not the stride-4 coarse lattice of `fine`
  const double dvc = d.vstride * d.dx / dt, dvf = e.vstride * e.dx / dt;
  lat::CoarseGeom g;
  g.nx = (int)d.nx;
  g.ny = (int)d.ny;
  g.nv = d.nv;
  g.dv = (float)dvc;
  g.nu_scale = (float)(dt / (tau_p * dvc));
  g.log_st = (float)log(St);
  g.line_eps = (float)rel_eps;
  lat::NaturalCoef nc;
  nc.nv_fine = e.nv;
  const double dtf = dt / e.nsub, dtc = dt / d.nsub;
  nc.alpha_f = (float)(dtf / (dvf * tau_p));
  nc.beta_f = (float)(dtf / tau_p);
  nc.D_f = (float)(kappa * dtf / (dvf * dvf));
  nc.nsub_f = e.nsub;
  nc.koren_f = e.scheme == LATTICE_KOREN;
  nc.alpha_c = (float)(dtc / (dvc * tau_p));
  nc.beta_c = (float)(dtc / tau_p);
  nc.D_c = (float)(kappa * dtc / (dvc * dvc));
  nc.nsub_c = d.nsub;
  nc.koren_c = d.scheme == LATTICE_KOREN;
  if (lat::launch_flux_samples_natural(g, nc, f_fine, f_pred, u, sites,
                                       (int)nsites, X, t, w,
                                       L->stream) != hipSuccess)
    return LATTICE_EHIP;
  return LATTICE_OK;
}

int lattice_mlp_grad(lattice_mlp_t* M, const float* X, const float* t,
                     const float* w, int64_t n, float* grad, double* loss) {
  if (!M || !X || !t || !w || n < 1) return LATTICE_EINVAL;
  double ws = 0.0;
  if (device_sum(w, n, M->stream, &ws) != hipSuccess) return LATTICE_EHIP;
  if (!(ws > 0)) return LATTICE_EINVAL;
  const int nr = lat::mlp_grad_rows(n, M->max_blocks);
  if (lat::launch_mlp_grad_mfma(M->params, X, t, w, n, ws, M->partial, nr,
                                M->stream) != hipSuccess ||
      lat::launch_grad_reduce(M->partial, nr, M->grad, M->loss, M->stream) !=
          hipSuccess)
    return LATTICE_EHIP;
  if (grad && hipMemcpyAsync(grad, M->grad, sizeof(float) * lat::kNParams,
                             hipMemcpyDeviceToDevice, M->stream) != hipSuccess)
    return LATTICE_EHIP;
  if (hipMemcpyAsync(M->host_loss, M->loss, sizeof(float),
                     hipMemcpyDeviceToHost, M->stream) != hipSuccess ||
      hipStreamSynchronize(M->stream) != hipSuccess)
    return LATTICE_EHIP;
  if (loss) *loss = *M->host_loss;
  return LATTICE_OK;
}

int lattice_mlp_train(lattice_mlp_t* M, const float* X, const float* t,
                      const float* w, int64_t n, int64_t batch, int64_t steps,
                      double lr, double* final_loss) {
  if (!M || !X || !t || !w || n < 1 || batch < 1 || steps < 0 ||
      !(lr > 0))
    return LATTICE_EINVAL;
  if (batch > n) batch = n;
  double ws = 0.0;
  if (device_sum(w, n, M->stream, &ws) != hipSuccess) return LATTICE_EHIP;
  if (!(ws > 0)) return LATTICE_EINVAL;
  // loss of a minibatch = sum w e^2 / (batch * mean w)
  const double norm = (double)batch * (ws / (double)n);
  const int64_t nwin = n / batch;  // whole windows of the (shuffled) data
  for (int64_t k = 0; k < steps; ++k) {
    const int64_t off = (k % (nwin > 0 ? nwin : 1)) * batch;
    const int nr = lat::mlp_grad_rows(batch, M->max_blocks);
    if (lat::launch_mlp_grad_mfma(M->params, X + off * lat::kNF, t + off,
                                  w + off, batch, norm, M->partial, nr,
                                  M->stream) != hipSuccess ||
        lat::launch_grad_reduce_adam(M->partial, nr, M->grad, M->loss,
                                     M->params, M->m, M->v, ++M->adam_t,
                                     (float)lr, 0.9f, 0.999f, 1e-8f,
                                     M->stream) != hipSuccess)
      return LATTICE_EHIP;
  }
  if (mlp_sync_bf16(M) != hipSuccess) return LATTICE_EHIP;
  if (hipMemcpyAsync(M->host_loss, M->loss, sizeof(float),
                     hipMemcpyDeviceToHost, M->stream) != hipSuccess ||
      hipStreamSynchronize(M->stream) != hipSuccess)
    return LATTICE_EHIP;
  if (final_loss) *final_loss = *M->host_loss;
  return LATTICE_OK;
}

int lattice_mlp_forward(lattice_mlp_t* M, const float* X, int64_t n,
                        float* y) {
  if (!M || !X || !y || n < 1) return LATTICE_EINVAL;
  if (lat::launch_mlp_forward(M->params, M->wq, X, n, y, M->stream) !=
      hipSuccess)
    return LATTICE_EHIP;
  return LATTICE_OK;
}

int lattice_mlp_attach(lattice_t* L, lattice_mlp_t* M, double St,
                       double line_eps) {
  if (!L) return LATTICE_EINVAL;
  if (!M) {
    L->mlp = nullptr;
    return LATTICE_OK;
  }
  if (L->d.dim != 2 || L->d.nv != 17 || L->d.dtype != LATTICE_F32 ||
      L->pitch != L->sites)
    return LATTICE_ENOTSUP;
  if (!(St > 0) || !(line_eps >= 0)) return LATTICE_EINVAL;
  L->mlp = M;
  L->mlp_St = St;
  L->mlp_eps = line_eps;
  return LATTICE_OK;
}

int lattice_mlp_destroy(lattice_mlp_t* M) {
  if (!M) return LATTICE_OK;
  (void)hipStreamSynchronize(M->stream);
  if (M->params) (void)hipFree(M->params);
  if (M->wq) (void)hipFree(M->wq);
  if (M->grad) (void)hipFree(M->grad);
  if (M->m) (void)hipFree(M->m);
  if (M->v) (void)hipFree(M->v);
  if (M->loss) (void)hipFree(M->loss);
  if (M->partial) (void)hipFree(M->partial);
  if (M->host_loss) (void)hipHostFree(M->host_loss);
  delete M;
  return LATTICE_OK;
}

}  // extern "C"

// Used by lattice_step: the correction pass after every step when a model
// is attached to a coarse 2D lattice.
namespace lat {
hipError_t apply_mlp(lattice_t* L, void* f, const void* u, double dt,
                     double tau_p) {
  lattice_mlp_t* M = L->mlp;
  CoarseGeom g;
  g.nx = (int)L->d.nx;
  g.ny = (int)L->d.ny;
  g.nv = L->d.nv;
  const double dv = L->d.vstride * L->d.dx / dt;
  g.dv = (float)dv;
  g.nu_scale = isfinite(tau_p) ? (float)(dt / (tau_p * dv)) : 0.f;
  g.log_st = (float)log(L->mlp_St);
  g.line_eps = (float)L->mlp_eps;
  return launch_mlp_correct(g, M->params, M->wq, (float*)f, (const float*)u,
                            L->flag, L->stream);
}
}  // namespace lat
