// lattice_host.hip -- C ABI of the phase-space lattice library: argument
// validation, velocity geometry, stability checks, buffer ownership and the
// launch sequence of one lattice_step call.  All arithmetic on the state
// happens in the kernels (step1d.hip, step2d*.hip, aux_kernels.hip).
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "../../include/lattice.h"
#include "lattice_internal.h"
#include "lattice_struct.h"


namespace {

int set_err(lattice_t* L, int code, const char* fmt, ...) {
  if (L) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(L->msg, sizeof(L->msg), fmt, ap);
    va_end(ap);
  }
  return code;
}

int hip_err(lattice_t* L, hipError_t e, const char* where) {
  return set_err(L, LATTICE_EHIP, "%s: %s", where, hipGetErrorString(e));
}

#define HIPCHK(L, expr)                            \
  do {                                             \
    hipError_t e_ = (expr);                        \
    if (e_ != hipSuccess) return hip_err(L, e_, #expr); \
  } while (0)

bool bad_desc(const lattice_desc* d) {
  if (!d) return true;
  if (d->dim != 1 && d->dim != 2) return true;
  if (d->nx < 1 || (d->dim == 2 && d->ny < 1)) return true;
  if (d->nv < 3 || (d->nv % 2) == 0) return true;
  if (d->vstride < 1) return true;
  if (!(d->dx > 0.0) || !isfinite(d->dx)) return true;
  if (d->scheme != LATTICE_UPWIND && d->scheme != LATTICE_KOREN) return true;
  if (d->dtype != LATTICE_F32 && d->dtype != LATTICE_F64) return true;
  if (d->nsub < 1 || d->u_hold < 0) return true;
  const double elem = d->dtype == LATTICE_F64 ? 8.0 : 4.0;
  const double ny = d->dim == 2 ? (double)d->ny : 1.0;
  const double sites = (double)d->nx * ny;
  if (d->nx >= 2147483647 || ny >= 2147483647) return true;
  if (d->plane_pitch < 0) return true;
  if (d->plane_pitch != 0 && (double)d->plane_pitch < sites) return true;
  if (d->dim == 1 && d->plane_pitch != 0 && d->plane_pitch != d->nx)
    return true;
  const double pitch = d->plane_pitch ? (double)d->plane_pitch : sites;
  const double row = pitch * (d->dim == 2 ? (double)d->nv : 1.0) * elem;
  const double total = pitch * pow((double)d->nv, d->dim) * elem;
  if (row >= 2147483648.0 || total >= 1099511627776.0) return true;
  return false;
}

// Element pitch between velocity planes of a valid descriptor.
int64_t plane_pitch_of(const lattice_desc& d) {
  const int64_t sites = d.nx * (d.dim == 2 ? d.ny : 1);
  return d.plane_pitch ? d.plane_pitch : sites;
}

// Drift bound of Eq. 3 for the scheme: strict CFL < 1 for upwind; CFL <= 1/2
// for the Koren-limited fluxes (outflow of a cell is at most twice its
// upwind value, so 2*CFL <= 1 keeps every cell non-negative).
double cfl_bound(int scheme) { return scheme == LATTICE_KOREN ? 0.5 : 1.0; }

hipError_t record_pair(lattice_t* L, bool stop) {
  if (!L->prof) return hipSuccess;
  if (!stop) {
    if (L->ev_used + 2 > L->ev.size()) {
      for (int k = 0; k < 64; ++k) {
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        L->ev.push_back(e);
      }
    }
    return hipEventRecord(L->ev[L->ev_used], L->stream);
  }
  hipError_t r = hipEventRecord(L->ev[L->ev_used + 1], L->stream);
  L->ev_used += 2;
  return r;
}

// Fold recorded event pairs into the totals (stream must be idle).
hipError_t prof_drain(lattice_t* L) {
  for (size_t k = 0; k + 1 < L->ev_used; k += 2) {
    float ms = 0.f;
    hipError_t r = hipEventElapsedTime(&ms, L->ev[k], L->ev[k + 1]);
    if (r != hipSuccess) return r;
    L->prof_ms += ms;
    L->prof_launches += 1;
  }
  L->ev_used = 0;
  return hipSuccess;
}

}  // namespace

extern "C" {

int lattice_desc_default(lattice_desc* d) {
  if (!d) return LATTICE_EINVAL;
  memset(d, 0, sizeof(*d));
  d->dim = 1;
  d->nx = 1;
  d->ny = 1;
  d->nv = 33;
  d->vstride = 1;
  d->dx = 1.0;
  d->scheme = LATTICE_KOREN;
  d->dtype = LATTICE_F32;
  d->nsub = 1;
  d->u_hold = 0;
  d->stream = nullptr;
  return LATTICE_OK;
}

int lattice_plane_pitch(const lattice_desc* d, int64_t* pitch) {
  if (!pitch) return LATTICE_EINVAL;
  if (!d) return LATTICE_EINVAL;
  lattice_desc c = *d;
  c.plane_pitch = 0;
  if (bad_desc(&c)) return LATTICE_EINVAL;
  const int64_t sites = c.nx * (c.dim == 2 ? c.ny : 1);
  const int64_t elem = c.dtype == LATTICE_F64 ? 8 : 4;
  int64_t p = sites;
  // 64 elements (256 B in FP32) after every plane whose size is a multiple
  // of 64 KiB: the copy of the step's access pattern at 512^2 x 33^2 runs
  // about 9 % faster with any pad of 32..192 elements, and 64 keeps every
  // plane 256-byte aligned
  if (c.dim == 2 && (sites * elem) % 65536 == 0) p = sites + 64;
  c.plane_pitch = p;
  if (bad_desc(&c)) p = sites;  // the padded row would pass the limits
  *pitch = p;
  return LATTICE_OK;
}

int lattice_velocity(const lattice_desc* d, double dt, double* dv,
                     double* vmax) {
  if (bad_desc(d) || !(dt > 0.0) || !isfinite(dt) || !dv || !vmax)
    return LATTICE_EINVAL;
  *dv = (double)d->vstride * d->dx / dt;
  *vmax = (double)((d->nv - 1) / 2) * (*dv);
  return LATTICE_OK;
}

int lattice_init(const lattice_desc* d, lattice_t** out) {
  if (!out) return LATTICE_EINVAL;
  *out = nullptr;
  if (bad_desc(d)) return LATTICE_EINVAL;
  if (d->dim == 1 && !lat::step1d_supported(d->nv, d->dtype == LATTICE_F64))
    return LATTICE_ENOTSUP;
  if (d->dim == 2 && !lat::step2d_supported(d->nv, d->dtype == LATTICE_F64))
    return LATTICE_ENOTSUP;

  lattice_t* L = new (std::nothrow) lattice;
  if (!L) return LATTICE_ENOMEM;
  L->d = *d;
  if (L->d.dim == 1) L->d.ny = 1;
  L->msg[0] = 0;
  L->sites = L->d.nx * L->d.ny;
  L->nplanes = L->d.dim == 1 ? L->d.nv : (int64_t)L->d.nv * L->d.nv;
  L->cells = L->sites * L->nplanes;
  L->pitch = plane_pitch_of(L->d);
  L->span = (L->nplanes - 1) * L->pitch + L->sites;
  L->elem = L->d.dtype == LATTICE_F64 ? 8 : 4;
  L->stream = (hipStream_t)L->d.stream;
  hipError_t e = hipMalloc(&L->scratch, (size_t)L->span * L->elem);
  if (e != hipSuccess) {
    delete L;
    return e == hipErrorOutOfMemory ? LATTICE_ENOMEM : LATTICE_EHIP;
  }
  if (hipMalloc(&L->flag, sizeof(int)) != hipSuccess ||
      hipMalloc(&L->plane_sums, sizeof(double) * (size_t)L->nplanes) !=
          hipSuccess ||
      hipMalloc(&L->red, sizeof(double) * 8) != hipSuccess ||
      hipHostMalloc((void**)&L->host_red, sizeof(double) * 8,
                    hipHostMallocDefault) != hipSuccess) {
    lattice_destroy(L);
    return LATTICE_ENOMEM;
  }
  if (lat::launch_clear_flag(L->flag, L->stream) != hipSuccess ||
      hipStreamSynchronize(L->stream) != hipSuccess) {
    lattice_destroy(L);
    return LATTICE_EHIP;
  }
  *out = L;
  return LATTICE_OK;
}

// Host-side checks and derived parameters of one call of nsteps steps
// (shared by the handle's entry points and the no-allocation step).
struct CallPlan {
  lat::StepArgs a;         // per-pass arguments (fin/fout/u/shift set later)
  int64_t slice_len = 0;   // elements of one u slice
  int64_t used = 0;        // u slices the device check reads
  double umax_ok = 0.0;    // |u| bound of Eq. 3 for this call
  int64_t passes_per_step = 1;
  int64_t passes = 0;
};

static int plan_call(const lattice_desc& d, int64_t sites, size_t elem,
                     void* f, const void* u, int64_t n_u_slices, double tau_p,
                     double kappa, double dt, int64_t nsteps, CallPlan* p,
                     char* msg, size_t msglen) {
  auto fail = [&](int code, const char* fmt, auto... args) {
    if (msg) snprintf(msg, msglen, fmt, args...);
    return code;
  };
  if (!f || !u) return fail(LATTICE_EINVAL, "%s", "f or u is NULL");
  if (((uintptr_t)f % elem) || ((uintptr_t)u % elem))
    return fail(LATTICE_EINVAL, "%s", "misaligned f or u");
  if (!(dt > 0.0) || !isfinite(dt))
    return fail(LATTICE_EINVAL, "%s", "dt must be > 0");
  if (!(tau_p > 0.0)) return fail(LATTICE_EINVAL, "%s", "tau_p must be > 0");
  if (!(kappa >= 0.0) || !isfinite(kappa))
    return fail(LATTICE_EINVAL, "%s", "kappa must be >= 0");
  if (nsteps < 0) return fail(LATTICE_EINVAL, "%s", "nsteps < 0");
  const int64_t need =
      d.u_hold > 0 ? (nsteps + d.u_hold - 1) / d.u_hold : 1;
  if (n_u_slices < need || n_u_slices < 1)
    return fail(LATTICE_EINVAL, "u holds %lld slices, call needs %lld",
                (long long)n_u_slices, (long long)need);
  if (nsteps == 0) return LATTICE_OK;  // a no-op; nothing else is checked

  const double dv = (double)d.vstride * d.dx / dt;
  const int h = (d.nv - 1) / 2;
  const double vmax = h * dv;
  const double dts = dt / d.nsub;
  const double Dn = kappa * dts / (dv * dv);
  if (!(Dn < 0.5))
    return fail(LATTICE_EDIFF, "kappa dt_s/dv^2 = %g >= 1/2", Dn);
  const bool drag = isfinite(tau_p);
  const double bound = cfl_bound(d.scheme);
  if (drag) {
    // (dt_s/dv)(|u| + Vmax)/tau_p within bound  <=>  |u| within umax_ok
    p->umax_ok = bound * tau_p * dv / dts - vmax;
    const double cfl0 = (dts / dv) * vmax / tau_p;
    if (p->umax_ok < 0.0 || (d.scheme == LATTICE_UPWIND && !(cfl0 < 1.0)))
      return fail(LATTICE_ECFL, "Vmax alone gives CFL %g", cfl0);
  }
  p->slice_len = (int64_t)d.dim * sites;
  p->used = drag ? need : 0;
  // per step, 1D does everything in one pass (nsub inline); 2D does one
  // streaming pass plus (nsub - 1) collision-only passes.
  p->passes_per_step = d.dim == 1 ? 1 : d.nsub;
  p->passes = nsteps * p->passes_per_step;
  lat::StepArgs& a = p->a;
  a.nx = d.nx;
  a.ny = d.ny;
  a.pitch = plane_pitch_of(d);
  a.nv = d.nv;
  a.alpha_scale = drag ? dts / (dv * tau_p) : 0.0;
  a.beta = drag ? dts / tau_p : 0.0;
  a.D = Dn;
  a.koren = d.scheme == LATTICE_KOREN;
  a.f64 = d.dtype == LATTICE_F64;
  a.nsub_inline = d.dim == 1 ? d.nsub : 1;
  return LATTICE_OK;
}

// The launch sequence of one call: the device CFL check of the u slices the
// call reads, the passes ping-ponging between f and twin (with one copy of
// f into twin first when the number of passes is odd, so that the result
// lands in f), and after every streaming step the learned correction when L
// has one attached.  L (optional) supplies profiling and the correction.
static int run_call(const lattice_desc& d, CallPlan& p, void* f,
                    const void* u, int64_t nsteps, void* twin, int* flag,
                    int64_t state_bytes, size_t elem, hipStream_t st,
                    bool stream, lattice_t* L, double tau_p, double dt,
                    const char** where, hipError_t* herr) {
  auto chk = [&](hipError_t e, const char* w) {
    if (e != hipSuccess) {
      *where = w;
      *herr = e;
      return false;
    }
    return true;
  };
  if (p.used > 0 &&
      !chk(lat::launch_cfl_check(u, p.used * p.slice_len, p.umax_ok,
                                 d.scheme == LATTICE_UPWIND ? 1 : 0,
                                 d.dtype == LATTICE_F64, flag, st),
           "cfl check launch"))
    return LATTICE_EHIP;
  void* bufs[2];
  if (p.passes % 2 == 0) {
    bufs[0] = f;
    bufs[1] = twin;
  } else {
    if (!chk(lat::launch_copy(twin, f, state_bytes, st), "state copy"))
      return LATTICE_EHIP;
    bufs[0] = twin;
    bufs[1] = f;
  }
  lat::StepArgs& a = p.a;
  a.flag = flag;
  int64_t k = 0;
  for (int64_t s = 0; s < nsteps; ++s) {
    const int64_t sl = d.u_hold > 0 ? s / d.u_hold : 0;
    a.u = (const char*)u + (size_t)(sl * p.slice_len) * elem;
    for (int64_t ps = 0; ps < p.passes_per_step; ++ps, ++k) {
      a.fin = bufs[k & 1];
      a.fout = bufs[(k + 1) & 1];
      a.shift = (ps == 0 && stream) ? d.vstride : 0;
      if (L && !chk(record_pair(L, false), "event record")) return LATTICE_EHIP;
      hipError_t e = d.dim == 1 ? lat::launch_step1d(a, st)
                                : lat::launch_step2d(a, st);
      if (!chk(e, "step kernel launch")) return LATTICE_EHIP;
      if (L && !chk(record_pair(L, true), "event record")) return LATTICE_EHIP;
    }
    if (L && L->mlp && stream &&  // learned face-flux correction (coarse)
        !chk(lat::apply_mlp(L, bufs[k & 1], a.u, dt, tau_p),
             "correction launch"))
      return LATTICE_EHIP;
  }
  return LATTICE_OK;
}

// One call of nsteps steps; stream == false leaves out the streaming (every
// pass has shift 0) and the learned correction: the collision part alone.
static int advance(lattice_t* L, void* f, const void* u, int64_t n_u_slices,
                   double tau_p, double kappa, double dt, int64_t nsteps,
                   bool stream) {
  if (!L) return LATTICE_EINVAL;
  L->msg[0] = 0;
  CallPlan p;
  int rc = plan_call(L->d, L->sites, L->elem, f, u, n_u_slices, tau_p, kappa,
                     dt, nsteps, &p, L->msg, sizeof(L->msg));
  if (rc != LATTICE_OK || nsteps == 0) return rc;
  const char* where = "";
  hipError_t e = hipSuccess;
  rc = run_call(L->d, p, f, u, nsteps, L->scratch, L->flag,
                L->span * (int64_t)L->elem, L->elem, L->stream, stream, L,
                tau_p, dt, &where, &e);
  if (rc == LATTICE_EHIP) return hip_err(L, e, where);
  return rc;
}

int lattice_step(lattice_t* L, void* f, const void* u, int64_t n_u_slices,
                 double tau_p, double kappa, double dt, int64_t nsteps) {
  return advance(L, f, u, n_u_slices, tau_p, kappa, dt, nsteps, true);
}

int lattice_collide(lattice_t* L, void* f, const void* u, int64_t n_u_slices,
                    double tau_p, double kappa, double dt, int64_t nsteps) {
  return advance(L, f, u, n_u_slices, tau_p, kappa, dt, nsteps, false);
}

}  // extern "C"

// ---- the step entry point that allocates nothing ---------------------------
namespace {

// Scratch of lattice_step_noalloc on every GPU the library runs on: the
// sticky flag word at offset 0, the ping-pong twin of the state from offset
// 256.  In host code the name stands for the host-side shadow, not for the
// device memory: kernels and copies get the address hipGetSymbolAddress
// returns for the current device (noalloc_scratch()).
__device__ __align__(256) unsigned char scratch[LATTICE_NOALLOC_MAX_BYTES +
                                                256];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
unsigned char* g_noalloc_ptr[kMaxDevices] = {};

// Device address of this device's scratch (looked up once per device, with
// that device current).  nullptr on failure.
unsigned char* noalloc_scratch(hipError_t* err) {
  int dev = 0;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    *err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_noalloc_ptr[dev] = (unsigned char*)ptr;
  }
  return g_noalloc_ptr[dev];
}

}  // namespace

extern "C" {

int lattice_step_noalloc(const lattice_desc* d, void* f, const void* u,
                         int64_t n_u_slices, double tau_p, double kappa,
                         double dt, int64_t nsteps, int32_t* status) {
  if (bad_desc(d)) return LATTICE_EINVAL;
  lattice_desc dd = *d;
  if (dd.dim == 1) dd.ny = 1;
  if (dd.dim == 1 && !lat::step1d_supported(dd.nv, dd.dtype == LATTICE_F64))
    return LATTICE_ENOTSUP;
  if (dd.dim == 2 && !lat::step2d_supported(dd.nv, dd.dtype == LATTICE_F64))
    return LATTICE_ENOTSUP;
  if (status && ((uintptr_t)status % sizeof(int32_t)))
    return LATTICE_EINVAL;
  const int64_t sites = dd.nx * dd.ny;
  const int64_t nplanes = dd.dim == 1 ? dd.nv : (int64_t)dd.nv * dd.nv;
  const int64_t span = (nplanes - 1) * plane_pitch_of(dd) + sites;
  const size_t elem = dd.dtype == LATTICE_F64 ? 8 : 4;
  if ((uint64_t)span * elem > (uint64_t)LATTICE_NOALLOC_MAX_BYTES)
    return LATTICE_ETOOBIG;
  CallPlan p;
  int rc = plan_call(dd, sites, elem, f, u, n_u_slices, tau_p, kappa, dt,
                     nsteps, &p, nullptr, 0);
  if (rc != LATTICE_OK) return rc;
  hipError_t e = hipSuccess;
  unsigned char* base = noalloc_scratch(&e);
  if (!base) return LATTICE_EHIP;
  int* flag = (int*)base;
  void* twin = base + 256;
  const hipStream_t st = (hipStream_t)dd.stream;
  // the flag starts at zero on every call (the array keeps the last call's
  // contents); cleared by a kernel so that the call can be captured
  if (lat::launch_clear_flag(flag, st) != hipSuccess) return LATTICE_EHIP;
  if (nsteps > 0) {
    const char* where = "";
    rc = run_call(dd, p, f, u, nsteps, twin, flag, span * (int64_t)elem,
                  elem, st, true, nullptr, tau_p, dt, &where, &e);
    if (rc != LATTICE_OK) return rc;
  }
  if (status && lat::launch_flag_out(flag, status, st) != hipSuccess)
    return LATTICE_EHIP;
  return LATTICE_OK;
}

// Report a set sticky flag (whose value the host has already read) and
// queue its clearing: stream order makes every later call see it cleared.
static int report_flag(lattice_t* L, int h) {
  if (!h) return LATTICE_OK;
  hipError_t e = lat::launch_clear_flag(L->flag, L->stream);
  if (e != hipSuccess) return hip_err(L, e, "flag clear");
  return set_err(L, LATTICE_ECFL,
                 "drift CFL bound (Eq. 3) violated or non-finite u");
}

// Wait for the stream and read the flag: one copy into pinned memory.
static int read_flag(lattice_t* L) {
  int* h = (int*)(L->host_red + 7);
  hipError_t e = hipMemcpyAsync(h, L->flag, sizeof(int),
                                hipMemcpyDeviceToHost, L->stream);
  if (e != hipSuccess) return hip_err(L, e, "flag copy");
  e = hipStreamSynchronize(L->stream);
  if (e != hipSuccess) return hip_err(L, e, "stream sync");
  return report_flag(L, *h);
}

int lattice_moments(lattice_t* L, const void* f, double dt,
                    lattice_moments_t* out) {
  if (!L) return LATTICE_EINVAL;
  L->msg[0] = 0;
  if (!f || !out || !(dt > 0.0) || !isfinite(dt))
    return set_err(L, LATTICE_EINVAL, "bad moments arguments");
  const lattice_desc& d = L->d;
  const double dv = (double)d.vstride * d.dx / dt;
  const double w = d.dim == 1 ? d.dx * dv : d.dx * d.dx * dv * dv;
  // the moments and the sticky flag come back in one copy (red[6] holds
  // the flag) with one wait
  HIPCHK(L, lat::launch_moments(f, L->sites, L->pitch, d.nv, d.dim,
                                d.dtype == LATTICE_F64, w, dv, L->plane_sums,
                                L->flag, L->red, L->stream));
  HIPCHK(L, hipMemcpyAsync(L->host_red, L->red, sizeof(double) * 7,
                           hipMemcpyDeviceToHost, L->stream));
  HIPCHK(L, hipStreamSynchronize(L->stream));
  const double* r = L->host_red;
  memset(out, 0, sizeof(*out));
  out->mass = r[0];
  out->momentum[0] = r[1];
  out->second_moment[0] = r[3];
  if (d.dim == 2) {
    out->momentum[1] = r[2];
    out->second_moment[1] = r[4];
  }
  out->variance = r[5];
  int nonfinite = 0;
  for (int i = 0; i < 6; ++i) nonfinite |= !isfinite(r[i]);
  out->nonfinite = nonfinite;
  int rc = report_flag(L, r[6] != 0.0);
  if (rc != LATTICE_OK) return rc;
  if (nonfinite)
    return set_err(L, LATTICE_ENONFINITE, "moments are not finite");
  return LATTICE_OK;
}

int lattice_density(lattice_t* L, const void* f, double dt, double* rho) {
  if (!L) return LATTICE_EINVAL;
  L->msg[0] = 0;
  if (!f || !rho || !(dt > 0.0) || !isfinite(dt))
    return set_err(L, LATTICE_EINVAL, "bad density arguments");
  const lattice_desc& d = L->d;
  const double dv = (double)d.vstride * d.dx / dt;
  const double dvd = d.dim == 1 ? dv : dv * dv;
  HIPCHK(L, lat::launch_density(f, L->sites, L->pitch, (int)L->nplanes,
                                d.dtype == LATTICE_F64, dvd, rho, L->stream));
  return LATTICE_OK;
}

int lattice_rho_r2(lattice_t* L, const double* rho, int levels, double* out) {
  if (!L) return LATTICE_EINVAL;
  L->msg[0] = 0;
  const lattice_desc& d = L->d;
  if (!rho || !out || levels < 1 || levels > lat::kRhoMaxLevels)
    return set_err(L, LATTICE_EINVAL, "bad rho_r2 arguments");
  const int64_t tile = (int64_t)1 << (levels - 1);
  if (d.nx % tile != 0 || (d.dim == 2 && d.ny % tile != 0))
    return set_err(L, LATTICE_EINVAL,
                   "nx (and ny) must be multiples of 2^(levels-1)");
  const int64_t npart = lat::rho_r2_partials(d.dim, d.nx, d.ny, levels);
  double* work = nullptr;
  if (hipMalloc(&work, sizeof(double) * (size_t)(L->sites + 2 * npart +
                                                 levels)) != hipSuccess)
    return set_err(L, LATTICE_ENOMEM, "rho_r2 workspace");
  double* partial = work + L->sites;
  double* dout = partial + 2 * npart;
  hipError_t e = lat::launch_rho_r2(rho, d.dim, d.nx, d.ny, levels, work,
                                    partial, dout, L->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, dout, sizeof(double) * levels,
                       hipMemcpyDeviceToHost, L->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
  (void)hipFree(work);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_err(L, LATTICE_EHIP, hipGetErrorString(e));
  }
  for (int k = 0; k < levels; ++k)
    if (!isfinite(out[k]))
      return set_err(L, LATTICE_ENONFINITE, "rho_r2 not finite");
  return LATTICE_OK;
}

int lattice_rho_r2_error(const double* a, const double* b, int levels,
                         double dx, double* err) {
  if (!a || !b || !err || levels < 1 || levels > lat::kRhoMaxLevels ||
      !(dx > 0.0) || !isfinite(dx))
    return LATTICE_EINVAL;
  double num = 0.0, den = 0.0, r = dx;
  for (int k = 0; k < levels; ++k, r *= 2.0) {
    const double w = r * r;  // r dr on the grid r_k = 2^k dx
    num += w * fabs(a[k] - b[k]);
    den += w * fabs(b[k]);
  }
  *err = num / den;
  if (!(den > 0.0) || !isfinite(*err)) return LATTICE_ENONFINITE;
  return LATTICE_OK;
}

int lattice_stability(lattice_t* L, const void* u, int64_t n_u_slices,
                      double tau_p, double kappa, double dt, double* out) {
  if (!L) return LATTICE_EINVAL;
  L->msg[0] = 0;
  if (!u || !out || n_u_slices < 1 || !(dt > 0.0) || !(tau_p > 0.0) ||
      !(kappa >= 0.0))
    return set_err(L, LATTICE_EINVAL, "bad stability arguments");
  const lattice_desc& d = L->d;
  const double dv = (double)d.vstride * d.dx / dt;
  const double vmax = ((d.nv - 1) / 2) * dv;
  const double dts = dt / d.nsub;
  HIPCHK(L, lat::launch_absmax(u, n_u_slices * d.dim * L->sites,
                               d.dtype == LATTICE_F64, L->red, L->stream));
  HIPCHK(L, hipMemcpyAsync(L->host_red, L->red, sizeof(double),
                           hipMemcpyDeviceToHost, L->stream));
  HIPCHK(L, hipStreamSynchronize(L->stream));
  const double umax = L->host_red[0];
  out[0] = (dts / dv) * (umax + vmax) / tau_p;
  out[1] = kappa * dts / (dv * dv);
  return LATTICE_OK;
}

int lattice_copy_state(lattice_t* L, void* dst, const void* src) {
  if (!L) return LATTICE_EINVAL;
  if (!dst || !src) return set_err(L, LATTICE_EINVAL, "NULL pointer");
  HIPCHK(L, lat::launch_copy(dst, src, L->span * (int64_t)L->elem,
                             L->stream));
  return LATTICE_OK;
}

int lattice_sync(lattice_t* L) {
  if (!L) return LATTICE_EINVAL;
  L->msg[0] = 0;
  HIPCHK(L, hipStreamSynchronize(L->stream));
  return read_flag(L);
}

int lattice_profile(lattice_t* L, int enable) {
  if (!L) return LATTICE_EINVAL;
  HIPCHK(L, hipStreamSynchronize(L->stream));
  L->ev_used = 0;
  L->prof_ms = 0.0;
  L->prof_launches = 0;
  L->prof = enable != 0;
  return LATTICE_OK;
}

int lattice_profile_read(lattice_t* L, double* total_ms, int64_t* launches) {
  if (!L || !total_ms || !launches) return LATTICE_EINVAL;
  HIPCHK(L, hipStreamSynchronize(L->stream));
  HIPCHK(L, prof_drain(L));
  *total_ms = L->prof_ms;
  *launches = L->prof_launches;
  return LATTICE_OK;
}

int lattice_destroy(lattice_t* L) {
  if (!L) return LATTICE_OK;
  int rc = LATTICE_OK;
  if (hipStreamSynchronize(L->stream) != hipSuccess) rc = LATTICE_EHIP;
  if (L->scratch) (void)hipFree(L->scratch);
  if (L->flag) (void)hipFree(L->flag);
  if (L->plane_sums) (void)hipFree(L->plane_sums);
  if (L->red) (void)hipFree(L->red);
  if (L->host_red) (void)hipHostFree(L->host_red);
  for (hipEvent_t e : L->ev) (void)hipEventDestroy(e);
  delete L;
  return rc;
}

const char* lattice_strerror(int code) {
  switch (code) {
    case LATTICE_OK: return "ok";
    case LATTICE_EINVAL: return "invalid argument";
    case LATTICE_ECFL: return "drift CFL condition (Eq. 3) violated";
    case LATTICE_EDIFF: return "diffusion stability kappa dt/dv^2 < 1/2 violated";
    case LATTICE_EHIP: return "HIP runtime error";
    case LATTICE_ENOMEM: return "out of device memory";
    case LATTICE_ENONFINITE: return "non-finite moments";
    case LATTICE_ENOTSUP: return "no kernel compiled for this lattice";
    case LATTICE_ETOOBIG:
      return "state larger than the static scratch of lattice_step_noalloc";
    case LATTICE_ETIMEOUT:
      return "resident batched launch gave up waiting for a member's step";
    default: return "unknown error";
  }
}

const char* lattice_last_error(const lattice_t* L) { return L ? L->msg : ""; }

}  // extern "C"
