// batch_internal.h -- device tables and launch interface of the batched 1D
// form (many independent realizations in one packed buffer).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lat {

// One realization, as the kernels see it.
struct BatchMember {
  int64_t f_off;      // element offset of its state [nv][pitch]
  int64_t u_off;      // element offset of its flow slices [slices][nx]
  int32_t nx, nv, h;
  int32_t step_mod;   // vstride mod nx
  int32_t init_off;   // (vstride*h) mod nx
  int32_t nsub;       // collision sub-steps per step
  int32_t u_hold;     // steps per flow slice (0 = one slice)
  int32_t plane0;     // index of its first velocity plane in plane tables
  int32_t pitch;      // elements from one velocity plane to the next
  float alpha_scale;  // dt_s / (dv tau_p)
  float beta;         // dt_s / tau_p
  float D;            // kappa dt_s / dv^2
  float umax_ok;      // largest |u| within the drift bound (inf: no drag)
  double dx, dv;      // geometry (moments)
};

// One work item: sites x0 .. x0+block-1 of one member.
struct BatchTile {
  int32_t member, x0;
};

// One velocity plane of one member (moments).
struct BatchPlane {
  int64_t off;
  int32_t nx, pad;
};

struct BatchLaunch {
  int cap;   // velocity capacity class of the kernel (9..129)
  int koren;
  int block;  // sites per tile, one lane each; 0 = split-column tiles
  int grid;
  const float* fin;
  float* fout;
  const float* u;
  const BatchMember* mem;
  const BatchTile* tiles;
  int ntiles;
  const int* mflag;
  const int* step_base;
  int local_step;
  int nt;  // split-column tiles: non-temporal stores
};

hipError_t launch_batch1d(const BatchLaunch& a, hipStream_t s);

// The resident multi-step kernel (all classes, split-column tiles).
// Layout of its synchronisation words (ints, zero at launch): the work
// counter of XCD x at kResQStride x (x < kResMaxXcd, one 128-byte line
// each), the abort flag at kResAbort, member m's finished tiles at
// kResDone + m.
constexpr int kResQStride = 32, kResMaxXcd = 16;
constexpr int kResAbort = kResQStride * kResMaxXcd;
constexpr int kResDone = kResAbort + kResQStride;
struct ResidentLaunch {
  int koren;
  int grid;
  float* b0;  // state before local step 0
  float* b1;
  const float* u;
  const BatchMember* mem;
  const BatchTile* tiles;  // one step's items, XCD by XCD, member by member
  const int* goff;         // XCD x owns tiles[goff[x] .. goff[x+1])
  int nxcd;
  const int* mtiles;  // tiles per member
  const int* mflag;
  int step0;   // step index of local step 0 within the call (flow slices)
  int nsteps;  // (largest goff span) * nsteps + grid * chunk < 2^31
  int chunk;   // items per work-counter fetch
  int stride;  // chunks of a block of `stride` interleave their items
  int* sync;
  int wait_limit;
};
hipError_t launch_batch_resident(const ResidentLaunch& a, hipStream_t s);
// Sites per tile of a capacity class in the resident kernel (0: none).
int batch_resident_sites(int cap);
int batch_resident_threads();
hipError_t batch_resident_occupancy(int koren, int* blocks_per_cu);
// Raise the abort flag if some XCD did not hand out all of its items.
hipError_t launch_resident_check(int* sync, const int* goff, int nxcd,
                                 int nsteps, hipStream_t s);
// out[b] = XCD of workgroup b, for nblocks workgroups.
hipError_t launch_xcc_probe(int* out, int nblocks, hipStream_t s);
// Sites per split-column tile of a capacity class (0: no split-column
// kernel for it).
int batch_parts_sites(int cap);
// max_values: the largest number of flow values one member's check reads
// (slices used x nx), to size the grid.
hipError_t launch_batch_cfl(const float* u, const BatchMember* mem, int count,
                            int64_t nsteps, int64_t max_values, int strict,
                            int* mflag, hipStream_t s);
hipError_t launch_batch_moments(const float* f, const BatchPlane* planes,
                                int nplanes, const BatchMember* mem, int count,
                                double* plane_sums, double* out,
                                hipStream_t s);
hipError_t launch_set_int(int* p, int v, hipStream_t s);
hipError_t launch_add_int(int* p, int v, hipStream_t s);
hipError_t launch_clear_ints(int* p, int n, hipStream_t s);
hipError_t launch_or_int(const int* src, int* dst, hipStream_t s);

}  // namespace lat
