/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of the phase-space
 * lattice update of Laenen, Krstulovic & Bec, "A lattice model for the
 * Eulerian description of heavy particle suspensions" (arXiv:1508.02899).
 * It exists so that tests, the smoke check and the benchmark's CPU baseline
 * can check the GPU library against an independent statement of the method.
 * The product path never calls it; it shares no code, header or constant
 * with the GPU library.
 *
 * What it computes (Sec. 2 of the paper, "Description of the method"):
 *   phase space is cut into (2d)-dimensional cells; f is piecewise constant;
 *   velocities sit on a lattice v_j = (j - h) dv, h = (nv-1)/2, with
 *   dx = s * dv * dt (s = 1 in the paper) so that advection is an exact
 *   shift by s*(j-h) cells; each time step applies, one after the other,
 *     S  exact lattice streaming,
 *     A  finite-volume Stokes drift (u - v)/tau_p across velocity faces
 *        (Eq. 5 gives the force; Eq. 3 its stability bound),
 *     D  finite-volume velocity diffusion kappa d_v^2 f (Eq. 4 bound),
 *   with zero flux through the outer faces of the velocity domain.
 *
 * Readings of points the paper leaves open:
 *   - drift sign follows the particle equation (Eq. 5): mass drifts toward u;
 *   - dv = 2 Vmax / (nv - 1): cell centres span [-Vmax, Vmax] (Sec. 3.2 and
 *     the caption of Fig. 14 fix this; Sec. 2 prints 2 Vmax / nv);
 *   - the drift is evaluated at cell centres and split into its positive and
 *     negative parts (flux-vector splitting); the face flux is the upwind
 *     value of each part, optionally corrected by the Koren limiter
 *     psi(theta) = max(0, min(1, 1/3 + theta/6, theta)) of Hundsdorfer et al.
 *     (1995), with cells outside the velocity domain holding zero mass;
 *   - forward Euler in time; in 2D each operator is split by velocity axis:
 *     A_x, A_y, then D_x, D_y;
 *   - u is sampled at the destination site of the streaming, at the start
 *     of the step; step s of a call uses slice s / u_hold (slice 0 when
 *     u_hold == 0);
 *   - nsub optional collide sub-steps (A and D repeated with dt/nsub) per
 *     streaming step; nsub = 1 is the paper's scheme.
 *
 * Layouts (plain C arrays, row-major):
 *   f[jv][y][x] with jv = jy*nv + jx in 2D (jv = j in 1D, ny = 1), x fastest;
 *   u[slice][component][y][x].
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_UPWIND 0
#define ORC_KOREN 1

/* Positive modulo for periodic spatial indices. */
static long wrap(long i, long n) {
  long r = i % n;
  return r < 0 ? r + n : r;
}

/* Koren limiter in ratio form (Hundsdorfer et al. 1995, cited in Sec. 2):
 * the correction added to the upwind face value is psi(theta) * dp, where
 * dp is the difference toward the downwind cell, dm the difference on the
 * upwind side, theta = dm / dp and
 *   psi(theta) = max(0, min(1, 1/3 + theta/6, theta)).
 * When dp == 0 there is nothing to correct. */
static double koren_correction(double dp, double dm) {
  if (dp == 0.0) return 0.0;
  double theta = dm / dp;
  double psi = 1.0;
  double third_order = 1.0 / 3.0 + theta / 6.0;
  if (third_order < psi) psi = third_order;
  if (theta < psi) psi = theta;
  if (psi < 0.0) psi = 0.0;
  return psi * dp;
}

/*
 * Drift along one velocity line (Sec. 2, force step): c[0..nv-1] holds the
 * masses of the cells of one velocity line at one site; nu[j] is the drift
 * of cell j in cell widths per (sub-)step, nu_j = dt_s (u - v_j) / (tau_p dv).
 * Each cell's outgoing mass rate is split into g+ = max(nu,0) c (moving to
 * larger j) and g- = min(nu,0) c (moving to smaller j).  The flux through
 * face k (between cells k-1 and k), k = 1..nv-1, is the upwind value of
 * each part plus, for the Koren scheme, the limited correction; faces 0 and
 * nv carry no flux (zero-flux velocity boundary).  Cells outside [0, nv)
 * count as empty when the limiter looks past the boundary.
 */
void orc_drift_line(double* c, int nv, const double* nu, int scheme) {
  double* gp = (double*)calloc((size_t)nv + 4, sizeof(double));
  double* gm = (double*)calloc((size_t)nv + 4, sizeof(double));
  double* F = (double*)calloc((size_t)nv + 1, sizeof(double));
  /* index shift by 2 so that gp[-2..nv+1] are addressable */
  double* P = gp + 2;
  double* M = gm + 2;
  for (int j = 0; j < nv; ++j) {
    P[j] = (nu[j] > 0.0 ? nu[j] : 0.0) * c[j];
    M[j] = (nu[j] < 0.0 ? nu[j] : 0.0) * c[j];
  }
  for (int k = 1; k <= nv - 1; ++k) {
    double fp = P[k - 1];
    double fm = M[k];
    if (scheme == ORC_KOREN) {
      fp += koren_correction(P[k] - P[k - 1], P[k - 1] - P[k - 2]);
      fm += koren_correction(M[k - 1] - M[k], M[k] - M[k + 1]);
    }
    F[k] = fp + fm;
  }
  F[0] = 0.0;
  F[nv] = 0.0;
  for (int j = 0; j < nv; ++j) c[j] = c[j] - (F[j + 1] - F[j]);
  free(gp);
  free(gm);
  free(F);
}

/*
 * Diffusion along one velocity line (Sec. 2, diffusion step, Eq. 4): the
 * flux through face k is the finite difference -D (c_k - c_{k-1}) with
 * D = kappa dt_s / dv^2, for k = 1..nv-1; faces 0 and nv carry no flux.
 */
void orc_diffuse_line(double* c, int nv, double D) {
  double* F = (double*)calloc((size_t)nv + 1, sizeof(double));
  for (int k = 1; k <= nv - 1; ++k) F[k] = -D * (c[k] - c[k - 1]);
  for (int j = 0; j < nv; ++j) c[j] = c[j] - (F[j + 1] - F[j]);
  free(F);
}

/*
 * Exact lattice streaming (Sec. 2, advection step): with dx = s dv dt the
 * mass of velocity index j moves by n_j = s (j - h) cells per component in
 * one step, periodically in space.  Pull form: g(x) = f(x - n_j).
 */
void orc_stream(int dim, long nx, long ny, int nv, int s, const double* f,
                double* g) {
  long h = (nv - 1) / 2;
  long sites = nx * ny;
  if (dim == 1) {
#pragma omp parallel for schedule(static)
    for (long j = 0; j < nv; ++j)
      for (long x = 0; x < nx; ++x)
        g[j * nx + x] = f[j * nx + wrap(x - s * (j - h), nx)];
  } else {
#pragma omp parallel for schedule(static)
    for (long jy = 0; jy < nv; ++jy)
      for (long jx = 0; jx < nv; ++jx) {
        long jv = jy * nv + jx;
        for (long y = 0; y < ny; ++y)
          for (long x = 0; x < nx; ++x) {
            long xs = wrap(x - s * (jx - h), nx);
            long ys = wrap(y - s * (jy - h), ny);
            g[jv * sites + y * nx + x] = f[jv * sites + ys * nx + xs];
          }
      }
  }
}

/*
 * Force then diffusion at every site (Sec. 2, operator splitting), with the
 * velocity dt_s = dt/nsub and the u slice given.  In 1D: A then D on the
 * velocity line.  In 2D: A along vx on every vy row, A along vy on every vx
 * column, then D along vx, then D along vy.
 */
static void collide(int dim, long nx, long ny, int nv, double dv, int scheme,
                    double* g, const double* u, double tau_p, double kappa,
                    double dts) {
  long h = (nv - 1) / 2;
  long sites = nx * ny;
  double D = kappa * dts / (dv * dv);
  /* Sites are independent.  A build with OpenMP (used only to time the
   * CPU baseline) spreads them over threads, each with its own line
   * buffers; the plain build runs the same loop on one thread.  The
   * arithmetic of a site does not depend on the thread that runs it. */
#pragma omp parallel
  {
  double* line = (double*)malloc(sizeof(double) * (size_t)nv);
  double* nu = (double*)malloc(sizeof(double) * (size_t)nv);
#pragma omp for schedule(static)
  for (long site = 0; site < sites; ++site) {
    if (dim == 1) {
      for (int j = 0; j < nv; ++j) {
        double vj = (double)(j - h) * dv;
        nu[j] = dts * (u[site] - vj) / (tau_p * dv);
        line[j] = g[(long)j * sites + site];
      }
      orc_drift_line(line, nv, nu, scheme);
      orc_diffuse_line(line, nv, D);
      for (int j = 0; j < nv; ++j) g[(long)j * sites + site] = line[j];
    } else {
      const double ux = u[site];
      const double uy = u[sites + site];
      /* A_x: every row of fixed jy, along jx */
      for (int jx = 0; jx < nv; ++jx)
        nu[jx] = dts * (ux - (double)(jx - h) * dv) / (tau_p * dv);
      for (int jy = 0; jy < nv; ++jy) {
        for (int jx = 0; jx < nv; ++jx)
          line[jx] = g[((long)jy * nv + jx) * sites + site];
        orc_drift_line(line, nv, nu, scheme);
        for (int jx = 0; jx < nv; ++jx)
          g[((long)jy * nv + jx) * sites + site] = line[jx];
      }
      /* A_y: every column of fixed jx, along jy */
      for (int jy = 0; jy < nv; ++jy)
        nu[jy] = dts * (uy - (double)(jy - h) * dv) / (tau_p * dv);
      for (int jx = 0; jx < nv; ++jx) {
        for (int jy = 0; jy < nv; ++jy)
          line[jy] = g[((long)jy * nv + jx) * sites + site];
        orc_drift_line(line, nv, nu, scheme);
        for (int jy = 0; jy < nv; ++jy)
          g[((long)jy * nv + jx) * sites + site] = line[jy];
      }
      /* D_x */
      for (int jy = 0; jy < nv; ++jy) {
        for (int jx = 0; jx < nv; ++jx)
          line[jx] = g[((long)jy * nv + jx) * sites + site];
        orc_diffuse_line(line, nv, D);
        for (int jx = 0; jx < nv; ++jx)
          g[((long)jy * nv + jx) * sites + site] = line[jx];
      }
      /* D_y */
      for (int jx = 0; jx < nv; ++jx) {
        for (int jy = 0; jy < nv; ++jy)
          line[jy] = g[((long)jy * nv + jx) * sites + site];
        orc_diffuse_line(line, nv, D);
        for (int jy = 0; jy < nv; ++jy)
          g[((long)jy * nv + jx) * sites + site] = line[jy];
      }
    }
  }
  free(line);
  free(nu);
  }
}

/*
 * nsteps full time steps, in place on f.  dv = s dx / dt (Sec. 2: dx = dv dt
 * for s = 1).  Returns 0, or -1 on bad arguments / allocation failure.
 */
int orc_step(int dim, long nx, long ny, int nv, int s, double dx, int scheme,
             int nsub, long u_hold, double* f, const double* u,
             long n_u_slices, double tau_p, double kappa, double dt,
             long nsteps) {
  if ((dim != 1 && dim != 2) || nx < 1 || ny < 1 || nv < 3 || nv % 2 == 0 ||
      s < 1 || dx <= 0.0 || dt <= 0.0 || nsub < 1 || nsteps < 0 ||
      n_u_slices < 1 || !(tau_p > 0.0) || kappa < 0.0)
    return -1;
  if (dim == 1) ny = 1;
  long cells = nx * ny;
  for (int d = 0; d < dim; ++d) cells *= nv;
  double dv = (double)s * dx / dt;
  double dts = dt / (double)nsub;
  double* g = (double*)malloc(sizeof(double) * (size_t)cells);
  if (!g) return -1;
  long slice_len = (long)dim * nx * ny;
  for (long step = 0; step < nsteps; ++step) {
    long sl = u_hold > 0 ? step / u_hold : 0;
    if (sl >= n_u_slices) {
      free(g);
      return -1;
    }
    const double* us = u + sl * slice_len;
    orc_stream(dim, nx, ny, nv, s, f, g);
    for (int k = 0; k < nsub; ++k)
      collide(dim, nx, ny, nv, dv, scheme, g, us, tau_p, kappa, dts);
    memcpy(f, g, sizeof(double) * (size_t)cells);
  }
  free(g);
  return 0;
}

/*
 * Conservation moments of f (mass normalisation of Sec. 3.2 and its first
 * two velocity moments): with w = dx^d dv^d,
 *   out[0]        = M   = w sum f
 *   out[1 + k]    = P_k = w sum f v_k          (k < dim)
 *   out[1+dim+k]  = Q_k = w sum f v_k^2
 *   out[1+2 dim]  = sum_k Q_k / M - |P / M|^2  (velocity variance)
 */
void orc_moments(int dim, long nx, long ny, int nv, int s, double dx,
                 double dt, const double* f, double* out) {
  if (dim == 1) ny = 1;
  long h = (nv - 1) / 2;
  long sites = nx * ny;
  double dv = (double)s * dx / dt;
  double w = dim == 1 ? dx * dv : dx * dx * dv * dv;
  double M = 0.0, P[2] = {0.0, 0.0}, Q[2] = {0.0, 0.0};
  long nplanes = dim == 1 ? nv : (long)nv * nv;
  for (long jv = 0; jv < nplanes; ++jv) {
    double vx = (double)((dim == 1 ? jv : jv % nv) - h) * dv;
    double vy = dim == 2 ? (double)(jv / nv - h) * dv : 0.0;
    for (long i = 0; i < sites; ++i) {
      double m = f[jv * sites + i];
      M += m;
      P[0] += m * vx;
      Q[0] += m * vx * vx;
      if (dim == 2) {
        P[1] += m * vy;
        Q[1] += m * vy * vy;
      }
    }
  }
  out[0] = w * M;
  double var = 0.0;
  for (int k = 0; k < dim; ++k) {
    out[1 + k] = w * P[k];
    out[1 + dim + k] = w * Q[k];
    var += Q[k] / M - (P[k] / M) * (P[k] / M);
  }
  out[1 + 2 * dim] = var;
}

/*
 * Stability numbers for one call (Eqs. 3 and 4).  The force per unit mass is
 * (u - v)/tau_p, so its largest magnitude per component over the sampled
 * sites and the velocity lattice is (max|u_k| + Vmax)/tau_p with
 * Vmax = h dv.  out[0] = CFL = (dt_s/dv) max_k (max|u_k| + Vmax)/tau_p,
 * out[1] = kappa dt_s / dv^2.
 */
void orc_stability(int dim, long nx, long ny, int nv, int s, double dx,
                   int nsub, const double* u, long n_u_slices, double tau_p,
                   double kappa, double dt, double* out) {
  if (dim == 1) ny = 1;
  double dv = (double)s * dx / dt;
  double dts = dt / (double)nsub;
  double vmax = (double)((nv - 1) / 2) * dv;
  long n = (long)dim * nx * ny * n_u_slices;
  double umax = 0.0;
  for (long i = 0; i < n; ++i) {
    double a = fabs(u[i]);
    if (a > umax) umax = a;
  }
  out[0] = (dts / dv) * (umax + vmax) / tau_p;
  out[1] = kappa * dts / (dv * dv);
}
