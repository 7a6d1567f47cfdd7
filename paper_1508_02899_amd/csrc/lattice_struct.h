// lattice_struct.h -- the single-lattice handle shared by the host files.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/lattice.h"

struct lattice {
  lattice_desc d;
  int64_t sites;    // nx * ny
  int64_t nplanes;  // nv^dim
  int64_t cells;    // sites * nplanes
  int64_t pitch;    // elements from one velocity plane to the next (>= sites)
  int64_t span;     // elements from the first to the last state element
                    // + 1: (nplanes - 1) * pitch + sites
  size_t elem;      // sizeof state element
  hipStream_t stream;
  void* scratch = nullptr;      // state-sized ping-pong twin
  int* flag = nullptr;          // sticky CFL / finiteness flag (device)
  double* plane_sums = nullptr; // nplanes doubles
  double* red = nullptr;        // 8 doubles: moments / absmax
  double* host_red = nullptr;   // pinned mirror of red
  char msg[512];
  // profiling
  bool prof = false;
  std::vector<hipEvent_t> ev;   // pairs (start, stop)
  size_t ev_used = 0;
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
  // learned face-flux correction applied after every step (coarse 2D)
  lattice_mlp_t* mlp = nullptr;
  double mlp_St = 1.0, mlp_eps = 0.0;
};

namespace lat {
// learned correction pass (coarse_host.hip)
hipError_t apply_mlp(lattice_t* L, void* f, const void* u, double dt,
                     double tau_p);
}  // namespace lat
