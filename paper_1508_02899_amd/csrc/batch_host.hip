// batch_host.hip -- C ABI of the batched 1D form: packing of many
// independent realizations, per-member coefficients and checks, work lists
// per velocity-capacity class, eager or HIP-graph launch sequences.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/lattice.h"
#include "batch_internal.h"
#include "lattice_internal.h"

namespace {

constexpr int kNumCls = 5;
constexpr int kCaps[kNumCls] = {9, 17, 33, 65, 129};
constexpr int kSide = 3;  // parallel streams for the classes beyond the first
constexpr int64_t kPlaneAlign = 64;  // elements: planes on 256-byte boundaries

struct Cls {
  int cap = 0;
  int block = 256;  // sites per tile, one lane each; 0 = split-column tiles
  int gpc = 0;  // resident workgroups per CU (0: one per tile)
  std::vector<int> members;
  int64_t bytes = 0;  // the class's state, bytes
  lat::BatchTile* d_tiles = nullptr;
  int ntiles = 0;
  int grid = 0;
};

}  // namespace

struct lattice_batch {
  int count = 0, scheme = 0, vstride = 1;
  std::vector<lattice_member_desc> desc;
  std::vector<lat::BatchMember> mem;
  int64_t total_cells = 0, total_u = 0;  // packed elements (padding included)
  int64_t cells = 0;                      // lattice cells
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;  // private stream the HIP graph is captured on
  hipStream_t side[kSide] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kSide] = {};
  lat::BatchMember* d_mem = nullptr;
  int* d_flag = nullptr;  // per member
  int* d_base = nullptr;  // step index of local step 0
  float* scratch = nullptr;
  lat::BatchPlane* d_planes = nullptr;
  int nplanes = 0;
  double* d_psums = nullptr;
  double* d_out = nullptr;
  double* h_out = nullptr;
  Cls cls[kNumCls];
  int ncu = 256;
  hipGraphExec_t gexec = nullptr;
  const void *g_a = nullptr, *g_b = nullptr, *g_u = nullptr;
  int g_steps = 0;
  // resident multi-step schedule
  int mode = LATTICE_BATCH_PER_STEP;
  int r_grid = 0;
  int wait_limit = 1 << 22;
  lat::BatchTile* d_rtiles = nullptr;  // one step's items, XCD by XCD
  int r_span = 0;            // most items of one XCD per step
  int r_nxcd = 0;
  int r_chunk = 4;
  int* d_goff = nullptr;     // XCD x owns d_rtiles[goff[x] .. goff[x+1])
  int* d_rmtiles = nullptr;  // tiles per member
  int* d_sync = nullptr;     // work counters, abort flag, done per member
  int* d_aborted = nullptr;  // some chunk gave up since the last sync
  char msg[512];
};

namespace {

int berr(lattice_batch_t* B, int code, const char* fmt, ...) {
  if (B) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(B->msg, sizeof(B->msg), fmt, ap);
    va_end(ap);
  }
  return code;
}

#define BCHK(B, expr)                                                     \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess)                                                 \
      return berr(B, LATTICE_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

int cap_class(int nv) {
  for (int c = 0; c < kNumCls; ++c)
    if (nv <= kCaps[c]) return c;
  return -1;
}

hipError_t build_tiles(lattice_batch_t* B, Cls& c) {
  std::vector<lat::BatchTile> t;
  const int sites = c.block > 0 ? c.block : lat::batch_parts_sites(c.cap);
  if (sites <= 0) return hipErrorInvalidValue;
  for (int m : c.members)
    for (int64_t x0 = 0; x0 < B->desc[m].nx; x0 += sites)
      t.push_back({m, (int32_t)x0});
  if (c.d_tiles) (void)hipFree(c.d_tiles);
  c.d_tiles = nullptr;
  c.ntiles = (int)t.size();
  if (t.empty()) return hipSuccess;
  hipError_t e = hipMalloc(&c.d_tiles, sizeof(lat::BatchTile) * t.size());
  if (e != hipSuccess) return e;
  e = hipMemcpy(c.d_tiles, t.data(), sizeof(lat::BatchTile) * t.size(),
                hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  const int64_t persistent = (int64_t)B->ncu * c.gpc;
  c.grid = (c.gpc == 0 || persistent >= c.ntiles) ? c.ntiles : (int)persistent;
  return hipSuccess;
}

// Queue n steps (local indices first..first+n-1) of every class, classes on
// parallel streams (they touch disjoint memory), buffers alternating from
// parity p0.  The first non-empty class runs on the main stream.
hipError_t enqueue_steps(lattice_batch_t* B, hipStream_t main,
                         float* const bufs[2], const float* u, int first,
                         int64_t n, int p0) {
  hipStream_t cs[kNumCls] = {};
  int nside = 0, ne = 0;
  for (int c = 0; c < kNumCls; ++c) {
    if (B->cls[c].ntiles == 0) continue;
    if (ne == 0) {
      cs[c] = main;
    } else {
      const int i = (ne - 1) % kSide;
      cs[c] = B->side[i];
      if (i + 1 > nside) nside = i + 1;
    }
    ++ne;
  }
  hipError_t e = hipSuccess;
  if (nside > 0) {
    e = hipEventRecord(B->ev_fork, main);
    if (e != hipSuccess) return e;
    for (int i = 0; i < nside; ++i) {
      e = hipStreamWaitEvent(B->side[i], B->ev_fork, 0);
      if (e != hipSuccess) return e;
    }
  }
  for (int64_t k = 0; k < n; ++k) {
    for (int c = 0; c < kNumCls; ++c) {
      Cls& cl = B->cls[c];
      if (cl.ntiles == 0) continue;
      lat::BatchLaunch a;
      a.cap = cl.cap;
      a.koren = B->scheme == LATTICE_KOREN;
      a.block = cl.block;
      a.grid = cl.grid;
      a.fin = bufs[(p0 + k) & 1];
      a.fout = bufs[(p0 + k + 1) & 1];
      a.u = u;
      a.mem = B->d_mem;
      a.tiles = cl.d_tiles;
      a.ntiles = cl.ntiles;
      a.mflag = B->d_flag;
      a.step_base = B->d_base;
      a.local_step = first + (int)k;
      // a class that writes more than 128 MB per step: measured on 256
      // lattices (the nv = 129 class, 191 MB) 4 % faster steps with
      // non-temporal stores, slower for the smaller classes, whose states
      // the next step still finds in the caches
      a.nt = cl.bytes > (int64_t)(128ll << 20);
      e = lat::launch_batch1d(a, cs[c]);
      if (e != hipSuccess) return e;
    }
  }
  for (int i = 0; i < nside; ++i) {
    e = hipEventRecord(B->ev_join[i], B->side[i]);
    if (e != hipSuccess) return e;
    e = hipStreamWaitEvent(main, B->ev_join[i], 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

int lattice_batch_destroy(lattice_batch_t* B);

int lattice_batch_init(const lattice_member_desc* members, int32_t count,
                       int32_t scheme, int32_t vstride, void* stream,
                       lattice_batch_t** out) {
  if (!out) return LATTICE_EINVAL;
  *out = nullptr;
  if (!members || count < 1 || count > 65535 || vstride < 1 ||
      (scheme != LATTICE_UPWIND && scheme != LATTICE_KOREN))
    return LATTICE_EINVAL;
  lattice_batch_t* B = new (std::nothrow) lattice_batch;
  if (!B) return LATTICE_ENOMEM;
  B->msg[0] = 0;
  B->count = count;
  B->scheme = scheme;
  B->vstride = vstride;
  B->stream = (hipStream_t)stream;
  B->desc.assign(members, members + count);
  B->mem.resize(count);
  const double bound = scheme == LATTICE_KOREN ? 0.5 : 1.0;
  std::vector<lat::BatchPlane> planes;
  int64_t foff = 0, uoff = 0;
  for (int r = 0; r < count; ++r) {
    const lattice_member_desc& d = members[r];
    if (d.nx < 1 || d.nx >= (1LL << 30) || d.nv < 3 || d.nv > 129 ||
        (d.nv % 2) == 0 || !(d.dx > 0) || !(d.dt > 0) || !(d.tau_p > 0) ||
        !(d.kappa >= 0) || !isfinite(d.kappa) || d.u_hold < 0 ||
        d.n_u_slices < 1) {
      delete B;
      return LATTICE_EINVAL;
    }
    const int h = (d.nv - 1) / 2;
    const double dv = vstride * d.dx / d.dt;
    const double Dn = d.kappa * d.dt / (dv * dv);
    if (!(Dn < 0.5)) {
      delete B;
      return LATTICE_EDIFF;
    }
    lat::BatchMember& m = B->mem[r];
    m.f_off = foff;
    m.u_off = uoff;
    m.nx = (int32_t)d.nx;
    m.nv = d.nv;
    m.h = h;
    m.step_mod = (int32_t)(vstride % d.nx);
    m.init_off = (int32_t)(((int64_t)vstride * h) % d.nx);
    m.nsub = 1;
    m.u_hold = (int32_t)d.u_hold;
    m.plane0 = (int32_t)planes.size();
    // planes start on 256-byte boundaries: a tile's rows then never share
    // a cache line with another tile's (measured: without, the kernels
    // write 1.16x the state, the partial lines written back twice)
    const int64_t pitch = (d.nx + kPlaneAlign - 1) / kPlaneAlign * kPlaneAlign;
    m.pitch = (int32_t)pitch;
    const bool drag = isfinite(d.tau_p);
    m.alpha_scale = drag ? (float)(d.dt / (dv * d.tau_p)) : 0.f;
    m.beta = drag ? (float)(d.dt / d.tau_p) : 0.f;
    m.D = (float)Dn;
    if (drag) {
      const double ok = bound * d.tau_p * dv / d.dt - h * dv;
      const double cfl0 = (d.dt / dv) * h * dv / d.tau_p;
      if (ok < 0 || (scheme == LATTICE_UPWIND && !(cfl0 < 1.0))) {
        delete B;
        return LATTICE_ECFL;
      }
      m.umax_ok = (float)ok;
    } else {
      m.umax_ok = INFINITY;
    }
    m.dx = d.dx;
    m.dv = dv;
    for (int j = 0; j < d.nv; ++j)
      planes.push_back({foff + (int64_t)j * pitch, (int32_t)d.nx, 0});
    foff += (int64_t)d.nv * pitch;
    B->cells += (int64_t)d.nv * d.nx;
    uoff += d.n_u_slices * d.nx;
    B->cls[cap_class(d.nv)].members.push_back(r);
    B->cls[cap_class(d.nv)].bytes += d.nx * d.nv * (int64_t)sizeof(float);
  }
  B->total_cells = foff;
  B->total_u = uoff;
  B->nplanes = (int)planes.size();
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&B->ncu, hipDeviceAttributeMultiprocessorCount,
                            dev) != hipSuccess) {
    delete B;
    return LATTICE_EHIP;
  }
  int rc = LATTICE_OK;
  do {
    if (hipMalloc(&B->d_mem, sizeof(lat::BatchMember) * count) != hipSuccess ||
        hipMalloc(&B->d_flag, sizeof(int) * count) != hipSuccess ||
        hipMalloc(&B->d_base, sizeof(int)) != hipSuccess ||
        hipMalloc(&B->scratch, sizeof(float) * (size_t)foff) != hipSuccess ||
        hipMalloc(&B->d_planes, sizeof(lat::BatchPlane) * planes.size()) !=
            hipSuccess ||
        hipMalloc(&B->d_psums, sizeof(double) * planes.size()) != hipSuccess ||
        hipMalloc(&B->d_out, sizeof(double) * 6 * count) != hipSuccess ||
        hipHostMalloc((void**)&B->h_out, sizeof(double) * 6 * count,
                      hipHostMallocDefault) != hipSuccess) {
      rc = LATTICE_ENOMEM;
      break;
    }
    if (hipMemcpy(B->d_mem, B->mem.data(), sizeof(lat::BatchMember) * count,
                  hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(B->d_planes, planes.data(),
                  sizeof(lat::BatchPlane) * planes.size(),
                  hipMemcpyHostToDevice) != hipSuccess) {
      rc = LATTICE_EHIP;
      break;
    }
    if (hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) !=
        hipSuccess) {
      rc = LATTICE_EHIP;
      break;
    }
    for (int i = 0; i < kSide; ++i)
      if (hipStreamCreateWithFlags(&B->side[i], hipStreamNonBlocking) !=
              hipSuccess ||
          hipEventCreateWithFlags(&B->ev_join[i], hipEventDisableTiming) !=
              hipSuccess) {
        rc = LATTICE_EHIP;
        break;
      }
    if (rc) break;
    if (hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming) !=
        hipSuccess) {
      rc = LATTICE_EHIP;
      break;
    }
    for (int c = 0; c < kNumCls; ++c) {
      B->cls[c].cap = kCaps[c];
      if (build_tiles(B, B->cls[c]) != hipSuccess) {
        rc = LATTICE_EHIP;
        break;
      }
    }
    if (rc) break;
    if (lat::launch_clear_ints(B->d_flag, count, B->stream) != hipSuccess ||
        hipStreamSynchronize(B->stream) != hipSuccess)
      rc = LATTICE_EHIP;
  } while (0);
  if (rc != LATTICE_OK) {
    lattice_batch_destroy(B);
    return rc;
  }
  *out = B;
  return LATTICE_OK;
}

int lattice_batch_layout(const lattice_batch_t* B, int64_t* f_off,
                         int64_t* u_off, int64_t* total_cells,
                         int64_t* total_u) {
  if (!B) return LATTICE_EINVAL;
  for (int r = 0; r < B->count; ++r) {
    if (f_off) f_off[r] = B->mem[r].f_off;
    if (u_off) u_off[r] = B->mem[r].u_off;
  }
  if (total_cells) *total_cells = B->total_cells;
  if (total_u) *total_u = B->total_u;
  return LATTICE_OK;
}

int lattice_batch_plane_pitch(const lattice_batch_t* B, int64_t* pitch,
                              int64_t* cells) {
  if (!B) return LATTICE_EINVAL;
  for (int r = 0; r < B->count; ++r)
    if (pitch) pitch[r] = B->mem[r].pitch;
  if (cells) *cells = B->cells;
  return LATTICE_OK;
}

int lattice_batch_tune(lattice_batch_t* B, int32_t cap, int32_t block,
                       int32_t grid_per_cu) {
  if (!B) return LATTICE_EINVAL;
  if (block != 0 && block != 64 && block != 128 && block != 256)
    return berr(B, LATTICE_EINVAL, "block must be 0, 64, 128 or 256");
  if (grid_per_cu < 0 || grid_per_cu > 16)
    return berr(B, LATTICE_EINVAL, "grid_per_cu must be 0..16");
  int c = -1;
  for (int i = 0; i < kNumCls; ++i)
    if (kCaps[i] == cap) c = i;
  if (c < 0) return berr(B, LATTICE_EINVAL, "unknown capacity %d", cap);
  if (block == 0) {
    if (lat::batch_parts_sites(cap) == 0)
      return berr(B, LATTICE_EINVAL,
                  "no split-column kernel for capacity %d", cap);
    for (int m : B->cls[c].members)
      if (B->desc[m].nv != cap)
        return berr(B, LATTICE_EINVAL,
                    "split-column tiles need nv == %d for every member of "
                    "the class (member %d has %d)", cap, m, B->desc[m].nv);
  }
  BCHK(B, hipStreamSynchronize(B->stream));
  B->cls[c].block = block;
  B->cls[c].gpc = grid_per_cu;
  BCHK(B, build_tiles(B, B->cls[c]));
  if (B->gexec) {  // work lists changed: the captured graph is stale
    (void)hipGraphExecDestroy(B->gexec);
    B->gexec = nullptr;
  }
  return LATTICE_OK;
}

int lattice_batch_schedule(lattice_batch_t* B, int32_t mode,
                           int32_t grid_per_cu, int32_t chunk,
                           int64_t wait_limit) {
  if (!B) return LATTICE_EINVAL;
  B->msg[0] = 0;
  if (mode != LATTICE_BATCH_PER_STEP && mode != LATTICE_BATCH_RESIDENT)
    return berr(B, LATTICE_EINVAL, "unknown schedule %d", mode);
  if (grid_per_cu < 0 || grid_per_cu > 16)
    return berr(B, LATTICE_EINVAL, "grid_per_cu must be 0..16");
  if (chunk < 0 || chunk > 64)
    return berr(B, LATTICE_EINVAL, "chunk must be 0..64");
  if (wait_limit >= (1LL << 31))
    return berr(B, LATTICE_EINVAL, "wait_limit must be below 2^31");
  if (mode == LATTICE_BATCH_PER_STEP) {
    B->mode = mode;
    return LATTICE_OK;
  }
  for (int r = 0; r < B->count; ++r) {
    const int nv = B->desc[r].nv;
    if (lat::batch_resident_sites(nv) == 0)
      return berr(B, LATTICE_ENOTSUP,
                  "resident schedule: member %d has nv %d (needs 17, 33, 65 "
                  "or 129)", r, nv);
  }
  BCHK(B, hipStreamSynchronize(B->stream));
  int occ = 0;
  BCHK(B, lat::batch_resident_occupancy(B->scheme == LATTICE_KOREN, &occ));
  if (occ < 1)
    return berr(B, LATTICE_ENOTSUP, "resident kernel does not fit a CU");
  const int gpc = grid_per_cu == 0 ? occ : grid_per_cu;
  // which XCDs the workgroups of a launch land on: every id below the
  // count must appear (a probe of many workgroups)
  int nxcd = 0;
  {
    const int nb = 8 * B->ncu;
    int* d_ids = nullptr;
    BCHK(B, hipMalloc(&d_ids, sizeof(int) * nb));
    std::vector<int> ids(nb);
    hipError_t e = lat::launch_xcc_probe(d_ids, nb, B->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    if (e == hipSuccess)
      e = hipMemcpy(ids.data(), d_ids, sizeof(int) * nb,
                    hipMemcpyDeviceToHost);
    (void)hipFree(d_ids);
    BCHK(B, e);
    bool seen[lat::kResMaxXcd] = {};
    for (int v : ids) {
      if (v < 0 || v >= lat::kResMaxXcd)
        return berr(B, LATTICE_ENOTSUP, "unexpected XCD id %d", v);
      seen[v] = true;
      if (v + 1 > nxcd) nxcd = v + 1;
    }
    for (int v = 0; v < nxcd; ++v)
      if (!seen[v])
        return berr(B, LATTICE_ENOTSUP, "no workgroup landed on XCD %d", v);
  }
  // members to XCDs: largest first, each to the least loaded XCD (cells)
  std::vector<int> order(B->count), owner(B->count);
  for (int r = 0; r < B->count; ++r) order[r] = r;
  auto cells = [&](int r) { return B->desc[r].nx * (int64_t)B->desc[r].nv; };
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    return cells(a) != cells(b) ? cells(a) > cells(b) : a < b;
  });
  std::vector<int64_t> load(nxcd, 0);
  for (int r : order) {
    int best = 0;
    for (int x = 1; x < nxcd; ++x)
      if (load[x] < load[best]) best = x;
    owner[r] = best;
    load[best] += cells(r);
  }
  std::vector<lat::BatchTile> t;
  std::vector<int> goff(nxcd + 1, 0), per(B->count);
  int span = 1;
  for (int x = 0; x < nxcd; ++x) {
    goff[x] = (int)t.size();
    for (int r = 0; r < B->count; ++r) {
      if (owner[r] != x) continue;
      const int g = lat::batch_resident_sites(B->desc[r].nv);
      for (int64_t x0 = 0; x0 < B->desc[r].nx; x0 += g)
        t.push_back({r, (int32_t)x0});
      per[r] = (int)((B->desc[r].nx + g - 1) / g);
    }
    if ((int)t.size() - goff[x] > span) span = (int)t.size() - goff[x];
  }
  goff[nxcd] = (int)t.size();
  if ((int64_t)t.size() > (1 << 24))
    return berr(B, LATTICE_ENOTSUP, "resident schedule: too many tiles");
  if (B->d_rtiles) (void)hipFree(B->d_rtiles);
  B->d_rtiles = nullptr;
  BCHK(B, hipMalloc(&B->d_rtiles, sizeof(lat::BatchTile) * t.size()));
  BCHK(B, hipMemcpy(B->d_rtiles, t.data(), sizeof(lat::BatchTile) * t.size(),
                    hipMemcpyHostToDevice));
  if (!B->d_goff)
    BCHK(B, hipMalloc(&B->d_goff, sizeof(int) * (lat::kResMaxXcd + 1)));
  BCHK(B, hipMemcpy(B->d_goff, goff.data(), sizeof(int) * (nxcd + 1),
                    hipMemcpyHostToDevice));
  if (!B->d_rmtiles) BCHK(B, hipMalloc(&B->d_rmtiles, sizeof(int) * B->count));
  BCHK(B, hipMemcpy(B->d_rmtiles, per.data(), sizeof(int) * B->count,
                    hipMemcpyHostToDevice));
  if (!B->d_sync)
    BCHK(B, hipMalloc(&B->d_sync, sizeof(int) * (lat::kResDone + B->count)));
  if (!B->d_aborted) {
    BCHK(B, hipMalloc(&B->d_aborted, sizeof(int)));
    BCHK(B, lat::launch_clear_ints(B->d_aborted, 1, B->stream));
    BCHK(B, hipStreamSynchronize(B->stream));
  }
  B->r_span = span;
  B->r_nxcd = nxcd;
  B->r_chunk = chunk == 0 ? 4 : chunk;
  B->r_grid = gpc * B->ncu;
  B->wait_limit = wait_limit < 0 ? -1
                  : wait_limit == 0 ? (1 << 22) : (int)wait_limit;
  B->mode = mode;
  return LATTICE_OK;
}

int lattice_batch_step(lattice_batch_t* B, float* f, const float* u,
                       int64_t nsteps, int32_t use_graph,
                       int32_t graph_steps) {
  if (!B) return LATTICE_EINVAL;
  B->msg[0] = 0;
  if (!f || !u) return berr(B, LATTICE_EINVAL, "NULL f or u");
  if (((uintptr_t)f % 4) || ((uintptr_t)u % 4))
    return berr(B, LATTICE_EINVAL, "misaligned f or u");
  if (nsteps < 0 || nsteps >= (1LL << 30))
    return berr(B, LATTICE_EINVAL, "bad nsteps");
  if (use_graph && (graph_steps < 2 || (graph_steps % 2)))
    return berr(B, LATTICE_EINVAL, "graph_steps must be even and >= 2");
  for (int r = 0; r < B->count; ++r) {
    const lattice_member_desc& d = B->desc[r];
    const int64_t need = d.u_hold > 0 ? (nsteps + d.u_hold - 1) / d.u_hold : 1;
    if (d.n_u_slices < need)
      return berr(B, LATTICE_EINVAL, "member %d: %lld u slices, needs %lld", r,
                  (long long)d.n_u_slices, (long long)need);
  }
  if (nsteps == 0) return LATTICE_OK;
  int64_t max_values = 1;
  for (int r = 0; r < B->count; ++r) {
    const lattice_member_desc& d = B->desc[r];
    const int64_t need = d.u_hold > 0 ? (nsteps + d.u_hold - 1) / d.u_hold : 1;
    if (need * d.nx > max_values) max_values = need * d.nx;
  }
  BCHK(B, lat::launch_batch_cfl(u, B->d_mem, B->count, nsteps, max_values,
                                B->scheme == LATTICE_UPWIND, B->d_flag,
                                B->stream));
  BCHK(B, lat::launch_set_int(B->d_base, 0, B->stream));
  float* bufs[2];
  if (nsteps % 2) {
    BCHK(B, lat::launch_copy(B->scratch, f, B->total_cells * 4, B->stream));
    bufs[0] = B->scratch;
    bufs[1] = f;
  } else {
    bufs[0] = f;
    bufs[1] = B->scratch;
  }
  if (B->mode == LATTICE_BATCH_RESIDENT) {
    // chunks of steps whose items stay countable in 32 bits
    const int64_t per =
        ((int64_t)0x7fffffff - 2 * (int64_t)B->r_grid * B->r_chunk) /
        B->r_span;
    for (int64_t s0 = 0; s0 < nsteps;) {
      const int64_t n = nsteps - s0 < per ? nsteps - s0 : per;
      BCHK(B, lat::launch_clear_ints(B->d_sync, lat::kResDone + B->count,
                                     B->stream));
      lat::ResidentLaunch a;
      a.koren = B->scheme == LATTICE_KOREN;
      a.grid = B->r_grid;
      a.b0 = bufs[s0 & 1];
      a.b1 = bufs[(s0 & 1) ^ 1];
      a.u = u;
      a.mem = B->d_mem;
      a.tiles = B->d_rtiles;
      a.goff = B->d_goff;
      a.nxcd = B->r_nxcd;
      a.mtiles = B->d_rmtiles;
      a.mflag = B->d_flag;
      a.step0 = (int)s0;
      a.nsteps = (int)n;
      a.chunk = B->r_chunk;
      // pairs of workgroups share their chunks' items (item stride 2):
      // 5 % shorter steps on configuration 4 than one chunk per
      // workgroup; needs two co-resident workgroups per XCD, which the
      // grid gives unless it holds fewer than two per XCD
      a.stride = B->r_grid / B->r_nxcd >= 2 ? 2 : 1;
      a.sync = B->d_sync;
      a.wait_limit = B->wait_limit;
      BCHK(B, lat::launch_batch_resident(a, B->stream));
      BCHK(B, lat::launch_resident_check(B->d_sync, B->d_goff, B->r_nxcd,
                                         (int)n, B->stream));
      // the abort flag of this launch is kept for lattice_batch_sync
      BCHK(B, lat::launch_or_int(B->d_sync + lat::kResAbort, B->d_aborted,
                                 B->stream));
      s0 += n;
    }
    return LATTICE_OK;
  }
  int64_t done = 0;
  if (use_graph && nsteps >= graph_steps) {
    if (!B->gexec || B->g_a != bufs[0] || B->g_b != bufs[1] || B->g_u != u ||
        B->g_steps != graph_steps) {
      if (B->gexec) {
        BCHK(B, hipGraphExecDestroy(B->gexec));
        B->gexec = nullptr;
      }
      // capture on the private stream (the caller's stream may be the
      // legacy default stream, which cannot be captured); the graph is
      // then launched on the caller's stream
      hipGraph_t g = nullptr;
      BCHK(B, hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
      hipError_t e = enqueue_steps(B, B->cap, bufs, u, 0, graph_steps, 0);
      if (e == hipSuccess) e = lat::launch_add_int(B->d_base, graph_steps,
                                                   B->cap);
      hipError_t e2 = hipStreamEndCapture(B->cap, &g);
      if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return berr(B, LATTICE_EHIP, "graph capture: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
      }
      e = hipGraphInstantiate(&B->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return berr(B, LATTICE_EHIP, "graph instantiate: %s",
                    hipGetErrorString(e));
      }
      B->g_a = bufs[0];
      B->g_b = bufs[1];
      B->g_u = u;
      B->g_steps = graph_steps;
    }
    const int64_t reps = nsteps / graph_steps;
    for (int64_t r = 0; r < reps; ++r)
      BCHK(B, hipGraphLaunch(B->gexec, B->stream));
    done = reps * graph_steps;
  }
  if (done < nsteps)
    BCHK(B, enqueue_steps(B, B->stream, bufs, u, 0, nsteps - done,
                          (int)(done & 1)));
  return LATTICE_OK;
}

int lattice_batch_moments(lattice_batch_t* B, const float* f, double* out) {
  if (!B || !f || !out) return LATTICE_EINVAL;
  BCHK(B, lat::launch_batch_moments(f, B->d_planes, B->nplanes, B->d_mem,
                                    B->count, B->d_psums, B->d_out,
                                    B->stream));
  BCHK(B, hipMemcpyAsync(B->h_out, B->d_out, sizeof(double) * 6 * B->count,
                         hipMemcpyDeviceToHost, B->stream));
  BCHK(B, hipStreamSynchronize(B->stream));
  memcpy(out, B->h_out, sizeof(double) * 6 * B->count);
  return LATTICE_OK;
}

int lattice_batch_sync(lattice_batch_t* B, int32_t* member_flags) {
  if (!B) return LATTICE_EINVAL;
  BCHK(B, hipStreamSynchronize(B->stream));
  if (B->d_aborted) {
    int ab = 0;
    BCHK(B, hipMemcpy(&ab, B->d_aborted, sizeof(int), hipMemcpyDeviceToHost));
    if (ab) {
      BCHK(B, lat::launch_clear_ints(B->d_aborted, 1, B->stream));
      BCHK(B, hipStreamSynchronize(B->stream));
      return berr(B, LATTICE_ETIMEOUT,
                  "resident schedule: a workgroup waited past the wait "
                  "limit for a member's previous step; the state is "
                  "undefined");
    }
  }
  std::vector<int> fl(B->count);
  BCHK(B, hipMemcpy(fl.data(), B->d_flag, sizeof(int) * B->count,
                    hipMemcpyDeviceToHost));
  int any = 0;
  for (int r = 0; r < B->count; ++r) {
    any |= fl[r] != 0;
    if (member_flags) member_flags[r] = fl[r];
  }
  if (any) {
    BCHK(B, lat::launch_clear_ints(B->d_flag, B->count, B->stream));
    BCHK(B, hipStreamSynchronize(B->stream));
    return berr(B, LATTICE_ECFL, "a member violated the drift CFL bound");
  }
  return LATTICE_OK;
}

const char* lattice_batch_last_error(const lattice_batch_t* B) {
  return B ? B->msg : "";
}

int lattice_batch_destroy(lattice_batch_t* B) {
  if (!B) return LATTICE_OK;
  (void)hipStreamSynchronize(B->stream);
  if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
  for (int c = 0; c < kNumCls; ++c)
    if (B->cls[c].d_tiles) (void)hipFree(B->cls[c].d_tiles);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  for (int i = 0; i < kSide; ++i) {
    if (B->side[i]) (void)hipStreamDestroy(B->side[i]);
    if (B->ev_join[i]) (void)hipEventDestroy(B->ev_join[i]);
  }
  if (B->ev_fork) (void)hipEventDestroy(B->ev_fork);
  if (B->d_rtiles) (void)hipFree(B->d_rtiles);
  if (B->d_goff) (void)hipFree(B->d_goff);
  if (B->d_rmtiles) (void)hipFree(B->d_rmtiles);
  if (B->d_sync) (void)hipFree(B->d_sync);
  if (B->d_aborted) (void)hipFree(B->d_aborted);
  if (B->d_mem) (void)hipFree(B->d_mem);
  if (B->d_flag) (void)hipFree(B->d_flag);
  if (B->d_base) (void)hipFree(B->d_base);
  if (B->scratch) (void)hipFree(B->scratch);
  if (B->d_planes) (void)hipFree(B->d_planes);
  if (B->d_psums) (void)hipFree(B->d_psums);
  if (B->d_out) (void)hipFree(B->d_out);
  if (B->h_out) (void)hipHostFree(B->h_out);
  delete B;
  return LATTICE_OK;
}

}  // extern "C"
