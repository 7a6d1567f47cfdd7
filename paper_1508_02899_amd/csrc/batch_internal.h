// batch_internal.h -- device tables and launch interface of the batched 1D
// form (many independent realizations in one packed buffer).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lat {

// One realization, as the kernels see it.
struct BatchMember {
  int64_t f_off;      // element offset of its state [nv][nx]
  int64_t u_off;      // element offset of its flow slices [slices][nx]
  int32_t nx, nv, h;
  int32_t step_mod;   // vstride mod nx
  int32_t init_off;   // (vstride*h) mod nx
  int32_t nsub;       // collision sub-steps per step
  int32_t u_hold;     // steps per flow slice (0 = one slice)
  int32_t plane0;     // index of its first velocity plane in plane tables
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

}  // namespace lat
