// Forward path used by mpm_step when no gradient is recorded.
#pragma once
#include <hip/hip_runtime.h>
#include "mpm_internal.h"

namespace mpm {

struct FastPath {
  char* ws;
  int n_grid, n_scenes, N;
  float4* mmv;     // dense grid (m, mv), shared with the plain path
  float4* vgrid;   // dense grid velocity
  bool valid;      // internal state mirrors the user state
};

size_t fast_workspace_bytes(int n_grid, int n_scenes, int N);
int fast_init(FastPath& f, char* ws, int n_grid, int n_scenes, int N, hipStream_t s);
void fast_bind_grid(FastPath& f, float4* mmv, float4* vgrid);
void fast_invalidate(FastPath& f);
int fast_run(FastPath& f, const StepParams& P, const PState& user, int t0, int n, const double* pose, const float* act,
             hipStream_t s, KernelTimer* timer);
void fast_destroy(FastPath& f);

}  // namespace mpm
