// Forward path used by mpm_step when no gradient is recorded (plain kernels).
#include "mpm_fast.h"

namespace mpm {

size_t fast_workspace_bytes(int, int, int) { return 0; }

int fast_init(FastPath& f, char* ws, int n_grid, int n_scenes, int N, hipStream_t) {
  f.ws = ws; f.n_grid = n_grid; f.n_scenes = n_scenes; f.N = N; f.valid = false;
  f.mmv = nullptr; f.vgrid = nullptr;
  return 0;
}
void fast_bind_grid(FastPath& f, float4* mmv, float4* vgrid) { f.mmv = mmv; f.vgrid = vgrid; }
void fast_invalidate(FastPath& f) { f.valid = false; }
void fast_destroy(FastPath&) {}

int fast_run(FastPath& f, const StepParams& P, const PState& user, int t0, int n, const double* pose, const float* act,
             hipStream_t s, KernelTimer* timer) {
  size_t nodes = (size_t)f.n_grid * f.n_grid * f.n_grid * f.n_scenes;
  for (int t = t0; t < t0 + n; t++) {
    launch_zero(f.mmv, nodes * sizeof(float4), s);
    timer->begin(s);
    launch_p2g_plain(user, P, f.mmv, s);
    timer->end(s);
    launch_grid_plain(P, f.mmv, f.vgrid, pose + (size_t)t * f.n_scenes * POSE_DOUBLES, act + (size_t)t * f.n_scenes * 6, s);
    launch_g2p_plain(user, user, P, f.vgrid, s);
  }
  return 0;
}

}  // namespace mpm
