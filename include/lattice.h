/*
 * lattice.h -- C ABI of the MI355X phase-space lattice library.
 *
 * The library advances the position/velocity phase-space density f(x, v, t)
 * of diffusive heavy inertial particles with the lattice method of
 * F. Laenen, G. Krstulovic, J. Bec, "A lattice model for the Eulerian
 * description of heavy particle suspensions" (arXiv:1508.02899):
 *
 *   - phase space is cut into (2d)-dimensional cells on which f is piecewise
 *     constant (Sec. 2);
 *   - velocities sit on a lattice v_j = (j - h) dv, j = 0..nv-1,
 *     h = (nv-1)/2, with dv = vstride * dx / dt, so that the mass of velocity
 *     index j moves by exactly vstride*(j-h) cells per step (Sec. 2: dx = dv
 *     dt, vstride = 1);  Vmax = h dv, i.e. dv = 2 Vmax / (nv - 1) (Sec. 3.2,
 *     Fig. 14 caption);
 *   - one time step is exact streaming, then the Stokes drift
 *     (u(x,t) - v)/tau_p of Eq. 5 as finite-volume fluxes across velocity
 *     faces (first-order upwind or Koren-limited), then velocity diffusion
 *     kappa d_v^2 f as finite-difference face fluxes (Sec. 2, Eqs. 3-5), with
 *     zero flux through the outer faces of the velocity domain.
 *
 * Everything runs in HIP kernels for gfx950 on the stream bound to the
 * handle.  State is FP32 (or FP64); the conservation moments are reduced in
 * FP64 on the GPU.
 *
 * Conventions for every function:
 *   - return 0 on success, a negative LATTICE_E* code on failure; nothing
 *     throws across the ABI;
 *   - "device" pointers are HIP device allocations (e.g. torch tensors on
 *     cuda:0), "host" pointers are ordinary memory;
 *   - a handle is not thread-safe; distinct handles are independent.
 */
#ifndef LATTICE_H
#define LATTICE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lattice lattice_t;

/* state / flow element type */
enum { LATTICE_F32 = 0, LATTICE_F64 = 1 };

/* drift scheme (Sec. 2): first-order upwind, or the Koren flux limiter
 * psi(theta) = max(0, min(1, 1/3 + theta/6, theta)) (Hundsdorfer et al.
 * 1995) applied to the upwind-split drift fluxes. */
enum { LATTICE_UPWIND = 0, LATTICE_KOREN = 1 };

/* error codes */
enum {
  LATTICE_OK = 0,
  LATTICE_EINVAL = -1,     /* bad argument (see each function) */
  LATTICE_ECFL = -2,       /* drift CFL of Eq. 3 violated (see lattice_step) */
  LATTICE_EDIFF = -3,      /* kappa dt_s / dv^2 >= 1/2 (Eq. 4) */
  LATTICE_EHIP = -4,       /* HIP runtime error; lattice_last_error explains */
  LATTICE_ENOMEM = -5,     /* device allocation failed */
  LATTICE_ENONFINITE = -6, /* moments are NaN or Inf */
  LATTICE_ENOTSUP = -7,    /* valid but not compiled in (2D nv, see below) */
  LATTICE_ETOOBIG = -8,    /* state too large for lattice_step_noalloc */
  LATTICE_ETIMEOUT = -9    /* a resident batched launch gave up waiting */
};

/*
 * Lattice description.  Layouts (x fastest):
 *   f : nv^dim velocity planes, plane jv = jy*nv + jx in 2D (jv = j in 1D,
 *       ny = 1); each plane is [ny][nx] contiguous dtype elements and plane
 *       jv starts plane_pitch*jv elements after plane 0 (plane_pitch = 0
 *       means nx*ny: the whole state is contiguous [nv^dim][ny][nx]).  The
 *       plane_pitch - nx*ny elements after each plane are never read as
 *       state and never written in f (whole-state copies may carry them
 *       through the library's own buffers);
 *   u : [slices][dim][ny][nx]  fluid velocity components, contiguous, dtype
 *       elements.
 * Why a pitch: when the plane size is a multiple of a large power of two
 * (512 x 512 FP32 sites: 1 MiB), the same site of the velocity planes that
 * one step touches together falls on the same HBM channels; a few hundred
 * bytes of padding per plane spreads them (lattice_plane_pitch).
 * Limits: nx*ny*nv^dim*sizeof(dtype) < 2^40 and
 * nv^(dim-1)*plane_pitch*sizeof(dtype) < 2^31 (one row of velocity planes).
 * Compiled velocity lattices: 1D any odd nv in [3, 129] (FP32) or [3, 65]
 * (FP64); 2D odd nv in [3, 21], 25, 33, 65 (FP32) and 3, 5, 9, 17, 33
 * (FP64).  Other odd nv >= 3 give LATTICE_ENOTSUP.
 */
typedef struct {
  int32_t dim;     /* 1 or 2 */
  int64_t nx, ny;  /* spatial sites per direction; ny is ignored (1) in 1D */
  int32_t nv;      /* velocities per component: odd, >= 3 (paper: 2^n + 1) */
  int32_t vstride; /* cells moved per velocity index per step; 1 = paper */
  double dx;       /* spatial spacing (> 0) */
  int32_t scheme;  /* LATTICE_UPWIND or LATTICE_KOREN */
  int32_t dtype;   /* LATTICE_F32 or LATTICE_F64 */
  int32_t nsub;    /* drift+diffusion sub-steps per streaming step (>= 1);
                      1 = the paper's scheme */
  int64_t u_hold;  /* steps per u slice within one lattice_step call;
                      0 = a single slice for the whole call */
  void* stream;    /* hipStream_t to run on; NULL = the default stream */
  int64_t plane_pitch; /* elements from one velocity plane of f to the next;
                          0 = nx*ny (contiguous); else >= nx*ny.  1D: 0 or
                          nx only */
} lattice_desc;

/* Moments of f (Sec. 3.2 mass normalisation and its velocity moments):
 * with w = dx^d dv^d,  mass = w sum f,  momentum[k] = w sum f v_k,
 * second_moment[k] = w sum f v_k^2,
 * variance = sum_k second_moment[k]/mass - |momentum/mass|^2.
 * Components k >= dim are 0.  nonfinite = 1 if any sum is NaN/Inf. */
typedef struct {
  double mass;
  double momentum[2];
  double second_moment[2];
  double variance;
  int32_t nonfinite;
} lattice_moments_t;

/* Fill *d with defaults: dim 1, nx 1, ny 1, nv 33, vstride 1, dx 1, Koren,
 * FP32, nsub 1, u_hold 0, default stream, plane_pitch 0 (contiguous).
 * EINVAL if d is NULL. */
int lattice_desc_default(lattice_desc* d);

/* The plane pitch this library recommends for the lattice *d (its
 * plane_pitch field is ignored): nx*ny, or, when one plane of the state
 * spans a multiple of 64 KiB, nx*ny plus 64 elements, which keeps the
 * velocity planes that one step reads and writes together off the same HBM
 * channels.  1D lattices: nx.  Host-only; EINVAL on a bad descriptor. */
int lattice_plane_pitch(const lattice_desc* d, int64_t* pitch);

/* Velocity geometry for a time step dt: *dv = vstride dx / dt,
 * *vmax = h dv.  Host-only; EINVAL on a bad descriptor or dt <= 0. */
int lattice_velocity(const lattice_desc* d, double dt, double* dv,
                     double* vmax);

/*
 * Validate *d and create a handle that owns a device scratch buffer of the
 * state's size (the ping-pong twin of f) plus small reduction buffers.
 * EINVAL: dim not 1/2, nx/ny < 1, nv even or < 3, vstride < 1, dx <= 0,
 * scheme/dtype unknown, nsub < 1, u_hold < 0, plane_pitch negative, below
 * nx*ny or (1D) other than nx, out NULL, sizes past the limits; ENOTSUP:
 * 2D nv without a compiled kernel; ENOMEM; EHIP.  The scratch twin has the
 * same plane pitch as f.
 */
int lattice_init(const lattice_desc* d, lattice_t** out);

/*
 * Advance f (device, in/out, layout above) by nsteps time steps of length
 * dt.  Step s of the call applies: exact pull streaming (Sec. 2), then nsub
 * times [drift (Eq. 5 force at cell centres, upwind or Koren fluxes), then
 * diffusion (finite-difference fluxes)] with dt_s = dt/nsub; in 2D each of
 * drift and diffusion is split by velocity axis (vx then vy).  The flow is
 * sampled at the destination site of the streaming from slice
 * s / u_hold of u (slice 0 if u_hold == 0).
 *
 * u (device, read-only) holds n_u_slices slices; the call needs
 * ceil(nsteps/u_hold) of them (1 if u_hold == 0), else EINVAL.  tau_p may be
 * +INFINITY (no drag: drift exactly zero); kappa may be 0 (no diffusion).
 *
 * Checked on the host, returned immediately: EINVAL (NULL f/u, misaligned
 * pointers, dt <= 0 or NaN, tau_p <= 0 or NaN, kappa < 0 or NaN,
 * nsteps < 0), EDIFF (kappa dt_s/dv^2 >= 1/2, Eq. 4), ECFL when Vmax alone
 * already violates the drift bound.  Checked on the device: the drift CFL
 * of Eq. 3, (dt_s/dv) (max|u_k| + Vmax)/tau_p, must be < 1 (upwind) or
 * <= 1/2 (Koren, the positivity bound of the limited scheme), and u must be
 * finite; a violation sets a sticky flag that turns every later step into a
 * no-op (f keeps the state before the call) until the next lattice_sync or
 * lattice_moments reports LATTICE_ECFL and clears it.
 *
 * Asynchronous: kernels are queued on the handle's stream and the call
 * returns without waiting.  f and u must stay valid until the stream has
 * passed the call.  The result always ends in f (the library ping-pongs
 * with its scratch buffer and copies once when nsteps is odd).
 */
int lattice_step(lattice_t* L, void* f, const void* u, int64_t n_u_slices,
                 double tau_p, double kappa, double dt, int64_t nsteps);

/*
 * The collision part of lattice_step alone: the same nsub sub-steps of
 * drift and diffusion (Sec. 2 operator splitting) with the streaming left
 * out, and no learned correction.  Same arguments, checks and semantics as
 * lattice_step.  A step equals streaming followed by this.  Used to build
 * velocity-space training targets for the coarse lattice.
 */
int lattice_collide(lattice_t* L, void* f, const void* u, int64_t n_u_slices,
                    double tau_p, double kappa, double dt, int64_t nsteps);

/*
 * lattice_step without a handle and without any allocation, for callers
 * that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  *d describes the lattice
 * as for lattice_init (its stream field selects the stream); f, u,
 * n_u_slices, tau_p, kappa, dt, nsteps and the host-side checks (EINVAL,
 * EDIFF, ECFL, ENOTSUP) are those of lattice_step, and the launch sequence
 * is the same, with the same kernels, so the result is bit-identical.
 *
 * Scratch: the state's ping-pong twin and the CFL flag live in one static
 * device array of LATTICE_NOALLOC_MAX_BYTES (+256) bytes that each GPU the
 * library runs on holds until the process ends; a state larger than that
 * returns LATTICE_ETOOBIG.  The first call on a device looks the array's
 * address up (hipGetSymbolAddress, no allocation); make that first call
 * outside any graph capture.  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (on different streams, or from
 * different threads) race and must not be issued.
 *
 * status (device int32, optional): receives, in stream order at the end of
 * the call, 0 when every step ran, nonzero when the device check of Eq. 3
 * (or finiteness of u) failed, in which case every step of the call was a
 * no-op (f keeps its state).  Asynchronous; returns without waiting.
 */
#define LATTICE_NOALLOC_MAX_BYTES (64ll << 20)
int lattice_step_noalloc(const lattice_desc* d, void* f, const void* u,
                         int64_t n_u_slices, double tau_p, double kappa,
                         double dt, int64_t nsteps, int32_t* status);

/*
 * FP64 moments of f (device, read-only) for time step dt (which fixes dv),
 * reduced on the GPU in a fixed order (deterministic) into *out (host).
 * Synchronous: waits for the stream.  Returns ECFL if the sticky CFL flag
 * was set by an earlier lattice_step (and clears it), ENONFINITE if a sum
 * is not finite (out is filled in both cases), EINVAL, EHIP.
 */
int lattice_moments(lattice_t* L, const void* f, double dt,
                    lattice_moments_t* out);

/*
 * Spatial density rho(x) = dv^dim sum_j f(x, v_j) (the velocity integral
 * of f, Sec. 3.2) into rho (device, [ny][nx] FP64).  Asynchronous.
 * EINVAL on NULL pointers or dt <= 0.
 */
int lattice_density(lattice_t* L, const void* f, double dt, double* rho);

/*
 * Second moment of the coarse-grained density (Sec. 3.1 defines rho_r as
 * the mass in a window of size r; Sec. 3.2 evaluates it on a tiling of
 * boxes of size r; Sec. 4.2.1 studies <rho_r^2> against r).  Tilings with
 * boxes of r = 2^k lattice spacings per direction, k = 0..levels-1, of
 * the density rho (device, [ny][nx] FP64, e.g. from lattice_density):
 *   out[k] = <rho_r^2> = N_b sum_b m_b^2 / (sum_b m_b)^2,
 * m_b the density summed over box b, N_b the number of boxes (so that
 * <rho_r> = 1).  out: host, levels doubles.  nx (and ny in 2D) must be
 * multiples of 2^(levels-1); levels <= 32.  FP64 sums in a fixed order
 * (bit-reproducible).  Synchronous; allocates a temporary device
 * workspace.  EINVAL, ENOMEM, ENONFINITE (zero or non-finite mass), EHIP.
 */
int lattice_rho_r2(lattice_t* L, const double* rho, int levels, double* out);

/*
 * Distance-averaged relative error of <rho_r^2> (Sec. 4.2.1, Eqs. 14-15:
 * the r dr average over the scales of |<rho_r^2>_A - <rho_r^2>_B| relative
 * to that of <rho_r^2>_B), on the tiling scales r_k = 2^k dx of
 * lattice_rho_r2 (k = 0..levels-1): with weights r_k dr_k = r_k^2 on that
 * log-spaced grid,
 *   *err = sum_k r_k^2 |a[k] - b[k]| / sum_k r_k^2 |b[k]|.
 * a, b: host, levels doubles (e.g. two lattice_rho_r2 outputs).  Host-only.
 * EINVAL on NULL pointers, levels outside [1, 32], dx <= 0; ENONFINITE
 * when the denominator is zero or a value is not finite.
 */
int lattice_rho_r2_error(const double* a, const double* b, int levels,
                         double dx, double* err);

/*
 * Eulerian first-order structure function of the particle velocity (Eq. 11,
 * Sec. 3.1; its scaling exponent is studied in Secs. 3.2 and 4.2.1):
 *   S1(r) = <sum_{j,j'} f(x,v_j) f(x+r,v_j') |v_j - v_j'|>_x
 *           / <sum_{j,j'} f(x,v_j) f(x+r,v_j')>_x
 * for the nr separations r[k] (host, int32, in lattice sites, >= 0;
 * periodic).  1D: r along x.  2D: |v - v'| is the Euclidean distance on the
 * velocity square; the estimate is the mean of the separations r e_x and
 * r e_y.  out: host, nr doubles.  FP64 correlation sums in a fixed order;
 * in 2D the velocity-space product runs as one GEMM (rocBLAS) in the state
 * dtype.  Synchronous; allocates a temporary device workspace of one state
 * plus (2D) an nv^2 x nv^2 matrix.  EINVAL, ENOMEM, ENONFINITE, EHIP.
 */
int lattice_s1(lattice_t* L, const void* f, double dt, int32_t nr,
               const int32_t* r, double* out);

/*
 * Carrier-flow synthesis on the device from Fourier mode tables (the random
 * Fourier flows of Sec. 3 and the streamfunction flows of Sec. 4; Eq. 7
 * gives the Ornstein-Uhlenbeck time law of the amplitudes, which the host
 * draws): the mode amplitudes of n_slices time slices in, u slices in the
 * layout lattice_step reads out.  Asynchronous on the handle's stream.
 *
 * 1D (dim 1): coef = device FP32 [n_slices][nmodes][2] = (a_k, b_k) for
 *   k = 1..nmodes; u[s][0][ix] = sum_k a_k cos(2 pi k ix/nx)
 *   + b_k sin(2 pi k ix/nx) in the lattice dtype.  EINVAL.
 * 2D (dim 2): coef = device FP32 [n_slices][2 kmax + 1][kmax + 1][2], the
 *   complex streamfunction amplitudes c(ky, kx) for ky = -kmax..kmax (row
 *   ky + kmax), kx = 0..kmax; psi(ix, iy) = sum Re(c e^{2 pi i (kx ix/nx +
 *   ky iy/ny)}), u[s][0] = d psi/dy, u[s][1] = -d psi/dx with the site
 *   spacing dx of the lattice (domain nx dx by ny dx).  Two separable passes
 *   (along x, then along y) through a stream-ordered temporary of
 *   2 (2 kmax + 1) nx n_slices complex values.  1 <= kmax <= 64,
 *   2 kmax < nx, ny; n_slices, ny <= 65535.  EINVAL, EHIP.
 */
int lattice_flow1d_modes(lattice_t* L, int32_t nmodes, const float* coef,
                         int64_t n_slices, void* u);
int lattice_flow2d_modes(lattice_t* L, int32_t kmax, const float* coef,
                         int64_t n_slices, void* u);

/*
 * Largest drift CFL number of Eq. 3 and the diffusion number of Eq. 4 for
 * the given u slices (device) and parameters: out[0] = (dt_s/dv)
 * (max|u_k| + Vmax)/tau_p, out[1] = kappa dt_s/dv^2 (out host, 2 doubles).
 * The max|u| reduction runs on the GPU.  Synchronous.  EINVAL, EHIP.
 */
int lattice_stability(lattice_t* L, const void* u, int64_t n_u_slices,
                      double tau_p, double kappa, double dt, double* out);

/* Copy a state-sized array (device to device) with the library's copy
 * kernel on the handle's stream.  Asynchronous.  EINVAL on NULL. */
int lattice_copy_state(lattice_t* L, void* dst, const void* src);

/* Wait for the stream; report LATTICE_ECFL (and clear the flag) if a CFL
 * violation was flagged since the last report, or EHIP. */
int lattice_sync(lattice_t* L);

/* Per-launch timing of the streaming/collision kernels with HIP events on
 * the handle's stream.  enable != 0 starts recording (and resets the
 * totals); lattice_profile_read waits for the stream and returns the summed
 * kernel time in milliseconds and the number of timed launches. */
int lattice_profile(lattice_t* L, int enable);
int lattice_profile_read(lattice_t* L, double* total_ms, int64_t* launches);

/* Release the handle and its device buffers (waits for the stream).
 * NULL is accepted. */
int lattice_destroy(lattice_t* L);

/* Static description of an error code. */
const char* lattice_strerror(int code);

/* Last detailed error message of the handle (e.g. the HIP error string),
 * or "" ; valid until the next call on the handle. */
const char* lattice_last_error(const lattice_t* L);


/* ===================================================================== *
 * Batched 1D lattices: many independent realizations (each with its own
 * grid size, velocity lattice, time step, Stokes number, diffusivity and
 * flow) advanced together.  Every member follows exactly the single-lattice
 * update of lattice_step (Sec. 2, Eqs. 3-5), FP32 state.
 *
 * Packed layouts (device, FP32): member m's state occupies
 * f[f_off[m] .. f_off[m] + nv_m*pitch_m) in the layout [nv_m][pitch_m],
 * of which elements 0 .. nx_m-1 of each velocity plane are the lattice's
 * cells and the rest padding that no kernel reads or writes; pitch_m is
 * nx_m rounded up to a multiple of 64, so that every plane starts on a
 * 256-byte boundary.  Its flow occupies u[u_off[m] .. u_off[m] +
 * n_u_slices_m*nx_m) as [slices][nx_m].  Offsets and pitches are assigned
 * by lattice_batch_init in member order (lattice_batch_layout,
 * lattice_batch_plane_pitch).
 *
 * Two schedules (lattice_batch_schedule).  Per step (the default): one
 * lattice_batch_step call queues, per time step, one persistent kernel per
 * velocity-capacity class (members with nv <= 9, 17, 33, 65, 129); the
 * classes run on parallel streams (they touch disjoint memory).  With
 * use_graph != 0 the per-step launches are captured once into a HIP graph
 * of graph_steps steps and replayed.  Resident: one kernel advances every
 * member by all the steps of the call, with a per-member step barrier on
 * device counters instead of a launch boundary per step.
 * ===================================================================== */
typedef struct lattice_batch lattice_batch_t;

typedef struct {
  int64_t nx;          /* sites (>= 1) */
  int32_t nv;          /* odd, 3..129 */
  double dx;           /* spatial spacing (> 0) */
  double dt;           /* time step (> 0); dv = vstride dx / dt */
  double tau_p;        /* > 0, may be +INFINITY */
  double kappa;        /* >= 0; kappa dt / dv^2 < 1/2 (Eq. 4) */
  int64_t u_hold;      /* steps per u slice; 0 = one slice */
  int64_t n_u_slices;  /* slices stored for this member (>= 1) */
} lattice_member_desc;

/* Validate count members (1 <= count <= 65535; all must satisfy Eq. 4 and
 * have Vmax alone within the drift bound) and allocate the packed scratch
 * state, the
 * member table, the work lists and reduction buffers.  EINVAL, EDIFF, ECFL,
 * ENOMEM, EHIP.  scheme: LATTICE_UPWIND / LATTICE_KOREN; stream: hipStream_t
 * or NULL. */
int lattice_batch_init(const lattice_member_desc* members, int32_t count,
                       int32_t scheme, int32_t vstride, void* stream,
                       lattice_batch_t** out);

/* Packed offsets (host arrays of count elements, may be NULL) and the
 * element counts of the packed state (padding included) and flow
 * buffers. */
int lattice_batch_layout(const lattice_batch_t* B, int64_t* f_off,
                         int64_t* u_off, int64_t* total_cells,
                         int64_t* total_u);

/* Plane pitch of every member (host array of count elements, may be NULL)
 * and the number of lattice cells of the batch (sum of nv_m nx_m; may be
 * NULL).  EINVAL. */
int lattice_batch_plane_pitch(const lattice_batch_t* B, int64_t* pitch,
                              int64_t* cells);

/* Work decomposition of one capacity class (cap = 9, 17, 33, 65 or 129):
 * block = lanes (= sites) per tile (64, 128 or 256), one lane per site with
 * its whole velocity column, or 0 = split-column tiles (each column over
 * several lanes, a tile of consecutive sites staged through LDS; only for
 * cap 17, 33, 65 or 129 and only when every member of the class has
 * nv == cap); grid_per_cu = resident workgroups per compute unit of the
 * persistent launch (1..16, or 0 = one workgroup per tile, not
 * persistent).  Chosen by the autotuner; defaults 256 / 0.  EINVAL (the
 * class keeps its previous decomposition). */
int lattice_batch_tune(lattice_batch_t* B, int32_t cap, int32_t block,
                       int32_t grid_per_cu);

enum { LATTICE_BATCH_PER_STEP = 0, LATTICE_BATCH_RESIDENT = 1 };

/* Schedule of lattice_batch_step.  LATTICE_BATCH_PER_STEP (default): as
 * described above.  LATTICE_BATCH_RESIDENT: each call is one launch (per
 * 2^31 work items) of a kernel that advances every member by all the
 * steps.  The members are split among the chip's XCDs (balanced by cells;
 * each XCD is one L2 cache domain), and all the tiles of a member, at
 * every step, are updated on its XCD: workgroups take chunks of `chunk`
 * (step, tile) items from their XCD's device work counter, in step order
 * (the tiles of one step member by member; split-column tiles, 128 sites
 * for nv 17, 33, 65 and 64 for nv 129), two chunks at a time interleaved
 * (one holds the even, the other the odd items of their 2 x chunk), so
 * that two workgroups work on neighbouring tiles.  A member's tile of step t > 0
 * starts once the member's device counter of finished tiles shows all of
 * its step t-1 tiles done (they wrote what the pull streaming of step t
 * reads, and have read the buffer that step t writes): a barrier per
 * member, none across the grid, so members of different sizes and
 * velocity lattices overlap.  Finished tiles are published through the
 * shared L2 of the XCD (stores complete before the count; the reader's L1
 * dropped before loading).  A workgroup publishes its finished tiles
 * before it waits and only waits on smaller items, so the queues drain as
 * long as two of the launch's workgroups run at once on each XCD (the
 * grid always holds at least that many; a device shared with other work
 * that leaves fewer ends in the bounded waits below); a launch that leaves
 * items of some XCD untaken (no workgroup ran there) is reported like a
 * time-out.
 * Every member's nv must be 17, 33, 65 or 129 (else ENOTSUP; the schedule
 * is unchanged); use_graph and graph_steps of lattice_batch_step are then
 * ignored, and the per-class decompositions of lattice_batch_tune are not
 * used.  grid_per_cu: resident workgroups per compute unit (1..16, 0 = as
 * many as fit); chunk: items per counter fetch (1..64, 0 = 4).
 * wait_limit: polls (each about a microsecond) after which a waiting
 * workgroup gives up; the launch then ends early, the state is undefined
 * and lattice_batch_sync returns ETIMEOUT; 0 = 2^22; a negative value makes
 * every wait give up at once (to exercise that path).  EINVAL, ENOTSUP,
 * EHIP. */
int lattice_batch_schedule(lattice_batch_t* B, int32_t mode,
                           int32_t grid_per_cu, int32_t chunk,
                           int64_t wait_limit);

/* Advance every member by nsteps (asynchronous).  u must hold, for each
 * member, ceil(nsteps/u_hold) slices (1 if u_hold == 0).  The drift CFL of
 * Eq. 3 is checked on the device per member; a violating member is frozen
 * (its steps are no-ops) and reported by lattice_batch_sync.  use_graph:
 * 0 = eager launches, else replay a HIP graph of graph_steps (even) steps.
 * EINVAL, EHIP. */
int lattice_batch_step(lattice_batch_t* B, float* f, const float* u,
                       int64_t nsteps, int32_t use_graph,
                       int32_t graph_steps);

/* FP64 moments per member into out[count][6] = {mass, momentum,
 * second moment, variance, 0, 0} (host), reduced on the GPU in a fixed
 * order.  Synchronous.  EINVAL, EHIP. */
int lattice_batch_moments(lattice_batch_t* B, const float* f, double* out);

/* Wait; return ETIMEOUT if a resident launch gave up waiting since the
 * last report (cleared), else ECFL if some member was frozen since the last
 * report (its flag is copied to member_flags[count] when that is not NULL,
 * and cleared), else 0 / EHIP. */
int lattice_batch_sync(lattice_batch_t* B, int32_t* member_flags);

/* Last detailed error message of the batch handle, or "". */
const char* lattice_batch_last_error(const lattice_batch_t* B);

int lattice_batch_destroy(lattice_batch_t* B);

/* ===================================================================== *
 * Coarse velocity lattice with a learned face-flux correction (2D, FP32).
 *
 * A coarse lattice keeps dx and dt and takes every 4th velocity of a fine
 * one (vstride 4, nv_c = (nv_f - 1)/4 + 1, dv_c = 4 dv_f), so its streaming
 * stays exact (Sec. 2).  With a network attached (lattice_mlp_attach), every
 * lattice_step time step of a 2D nv = 17 FP32 lattice is followed by a
 * correction: for each site and each interior velocity face whose 5-cell
 * stencil holds at least line_eps of the site's mass (the faces the
 * training samples of lattice_mlp_samples keep), the network maps the
 * face's 8 features [5-cell stencil from the upwind side / its mass m_s,
 * |face drift| in cells per step, ln St, 0] to y; the face flux
 * sign * m_s * y, limited to a quarter of the donor cell's mass, updates the
 * state conservatively (f -= div G; mass exact, f >= 0 kept).
 * Network: 8 -> 64 -> 64 -> 1, GELU (tanh form), bf16 weights and inputs on
 * the matrix cores with FP32 accumulation.  Parameters are packed as
 * W1[8][64], b1[64], W2[64][64], b2[64], w3[64], b3 (4801 floats).
 * ===================================================================== */
typedef struct lattice_mlp lattice_mlp_t;

/* Mass-conservative restriction of a fine state (nv_fine = 4k + 1
 * velocities per axis, [nv_f^dim][sites]) to the coarse lattice
 * ([nv_c^dim][sites]): coarse cell J spans fine centres 4J-2..4J+2, the
 * fine cells 4J+-2 being shared half/half.  Device pointers, asynchronous
 * on stream.  EINVAL, EHIP. */
int lattice_restrict(int32_t dim, int64_t sites, int32_t nv_fine,
                     const float* f_fine, float* f_coarse, void* stream);

/* Create a network (parameters zero) whose kernels run on stream. */
int lattice_mlp_create(void* stream, lattice_mlp_t** out);
/* Copy 4801 FP32 parameters from / to host memory (resets Adam). */
int lattice_mlp_set_params(lattice_mlp_t* M, const float* host_params);
int lattice_mlp_get_params(lattice_mlp_t* M, float* host_params);

/* Training samples at nsites listed sites (device int32) of the coarse
 * lattice L (2D, nv 17, FP32): with f_pred = one plain coarse step of the
 * restricted fine state and f_true = the restricted fine state one step
 * later (both device [289][ny][nx]), the residual r = f_true - f_pred is
 * written as the face fluxes of least norm with -div G = r, and for every
 * interior face (x-faces (row, k) then y-faces (k, column); 544 per site)
 * X[8] = features of f_pred, t = sign * G / m_s, w = m_s.  Faces whose
 * stencil mass m_s is below rel_eps times the site mass (0 <= rel_eps < 1)
 * or below 1e-30 get w = 0, t = 0 and zero stencil features.  Device
 * outputs.  Asynchronous.  EINVAL, ENOTSUP, EHIP. */
int lattice_mlp_samples(lattice_t* L, double dt, double tau_p, double St,
                        double rel_eps,
                        const float* f_pred, const float* f_true,
                        const float* u, const int32_t* sites, int64_t nsites,
                        float* X, float* t, float* w);

/* Training samples with natural flux targets at nsites listed sites of the
 * coarse lattice L (2D, nv 17, FP32) of the fine lattice `fine` (2D, nv 65,
 * FP32, same sites and dx, vstride 4x smaller).  f_fine = the fine state
 * after streaming, before its collision ([65^2][ny][nx]); f_pred = the
 * coarse collision (lattice_collide of L) of its restriction
 * ([17^2][ny][nx]); u the flow slice [2][ny][nx]; all device.  Per site the
 * fine collision (fine's nsub and scheme, coefficients of Eqs. 4, 5 with
 * tau_p, kappa, dt) is repeated with its face fluxes F recorded; the
 * target fluxes are the coarse fluxes implied by F under the restriction
 * R (div_c G = R div F) minus the face fluxes of the coarse collision of
 * R f_fine (L's nsub and scheme), so that f_pred - div T = R (fine
 * collision of f_fine).  X, t, w as in lattice_mlp_samples (features and
 * weights from f_pred; the same face rule with rel_eps).  These targets
 * are face-local (the fine fluxes near the face), unlike the least-norm
 * ones.  Asynchronous on L's stream.  EINVAL, ENOTSUP, EHIP. */
int lattice_mlp_samples_natural(const lattice_t* fine, lattice_t* L,
                                double dt, double tau_p, double kappa,
                                double St, double rel_eps,
                                const float* f_fine, const float* f_pred,
                                const float* u, const int32_t* sites,
                                int64_t nsites, float* X, float* t, float* w);

/* Gradient of L = sum w (y - t)^2 / sum w over n samples (device X[n][8],
 * t, w) into grad (device, 4801 floats, may be NULL) and *loss (host);
 * weights and layer inputs rounded to bf16 as in the forward pass.
 * Synchronous.  EINVAL, EHIP. */
int lattice_mlp_grad(lattice_mlp_t* M, const float* X, const float* t,
                     const float* w, int64_t n, float* grad, double* loss);

/* steps Adam steps (lr, beta 0.9/0.999, eps 1e-8) on consecutive
 * minibatches of batch samples (the data should be shuffled); *final_loss =
 * loss of the last minibatch.  Synchronous.  EINVAL, EHIP. */
int lattice_mlp_train(lattice_mlp_t* M, const float* X, const float* t,
                      const float* w, int64_t n, int64_t batch, int64_t steps,
                      double lr, double* final_loss);

/* Network outputs y[n] for inputs X[n][8] (device), matrix-core path.
 * Asynchronous.  EINVAL, EHIP. */
int lattice_mlp_forward(lattice_mlp_t* M, const float* X, int64_t n,
                        float* y);

/* Attach (M != NULL) or detach (M == NULL) the correction to a coarse 2D
 * lattice (nv 17, FP32); St and line_eps enter as described above.
 * EINVAL, ENOTSUP. */
int lattice_mlp_attach(lattice_t* L, lattice_mlp_t* M, double St,
                       double line_eps);

int lattice_mlp_destroy(lattice_mlp_t* M);

#ifdef __cplusplus
}
#endif

#endif /* LATTICE_H */
