// Internal structures shared by the HIP kernels and the C ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <vector>

namespace mpm {

enum { KIND_ELASTIC = 0, KIND_LIQUID = 1, KIND_SAND = 2, KIND_VONMISES = 3, KIND_BOX = 4, KIND_RIGID = 5 };
enum { ERR_OUTSIDE = 1, ERR_NONFINITE = 2, ERR_SAND_SIGMA = 4, ERR_TILE = 8 };

// Per-material constants as the kernels use them (alpha, kappa precomputed).
struct MatDev {
  int kind;
  float mu, lam, eta;
  float alpha, kappa, coh;
  float vol, mass;
  float yrad;          // von Mises return radius in log strain, yield / (2 mu)
  float box_lo, box_hi; // Box yield: singular values clamped to [box_lo, box_hi]
};

// Particle state, structure of arrays: component k of particle p at ptr[k*N + p].
struct PState {
  float* x;   // 3
  float* v;   // 3
  float* C;   // 9
  float* F;   // 9
  float* J;   // 1
  int N;
};

// Floats per particle in a packed state buffer (x, v, C, F, J).
constexpr int STATE_FLOATS = 25;

__host__ __device__ inline PState packed_state(float* base, int N) {
  PState s;
  s.x = base;
  s.v = base + 3 * (size_t)N;
  s.C = base + 6 * (size_t)N;
  s.F = base + 15 * (size_t)N;
  s.J = base + 24 * (size_t)N;
  s.N = N;
  return s;
}

struct StepParams {
  int n_grid, n_scenes, n_particles, bound;
  float dx, inv_dx, dt;
  float grav[3];
  float band, friction;
  const MatDev* mats;      // [n_materials]
  const uint8_t* mat;      // [N] material index
  const int* pscene;       // [N] scene index
  const float* cyl_radius; // [n_scenes]
  int* err;                // device error word
};

// Pose history entry: c (3), R (9) in FP64.
constexpr int POSE_DOUBLES = 12;
// Per-step, per-scene local adjoint accumulators:
// u (3), w (3), c (3), axis a = R e_y (3).
constexpr int ACC_DOUBLES = 12;

// Optional per-launch timing of one kernel with HIP events on its stream.
struct KernelTimer {
  bool on = false;
  const char* name = "";
  hipEvent_t ev[2 * 4096];
  int created = 0;
  int used = 0;
  double total_ms = 0.0;
  long long launches = 0;
  void begin(hipStream_t s) {
    if (!on || used >= 4096) return;
    if (used >= created) {
      hipEventCreate(&ev[2 * used]);
      hipEventCreate(&ev[2 * used + 1]);
      created = used + 1;
    }
    hipEventRecord(ev[2 * used], s);
  }
  void end(hipStream_t s) {
    if (!on || used >= 4096) return;
    hipEventRecord(ev[2 * used + 1], s);
    used++;
  }
  // event pairs owned elsewhere (a captured graph, or a call's temporaries
  // with owned = true), read at the next collect()
  std::vector<hipEvent_t> ext;
  std::vector<char> ext_owned;
  void adopt(const std::vector<hipEvent_t>& pairs, int n_pairs, bool owned = false) {
    for (int i = 0; i < n_pairs && 2 * i + 1 < (int)pairs.size(); i++) {
      ext.push_back(pairs[2 * i]);
      ext.push_back(pairs[2 * i + 1]);
      ext_owned.push_back(owned ? 1 : 0);
    }
  }
  // after the stream has been synchronised; a failed query is skipped and
  // its error cleared so that it does not surface at an unrelated call
  void collect() {
    for (int i = 0; i < used; i++) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) == hipSuccess) { total_ms += ms; launches++; }
      else (void)hipGetLastError();
    }
    used = 0;
    for (size_t i = 0; 2 * i + 1 < ext.size(); i++) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ext[2 * i], ext[2 * i + 1]) == hipSuccess) { total_ms += ms; launches++; }
      else (void)hipGetLastError();
      if (ext_owned[i]) { hipEventDestroy(ext[2 * i]); hipEventDestroy(ext[2 * i + 1]); }
    }
    ext.clear();
    ext_owned.clear();
  }
  void destroy() {
    for (int i = 0; i < created; i++) { hipEventDestroy(ev[2 * i]); hipEventDestroy(ev[2 * i + 1]); }
    created = 0;
  }
};

// ---- launch wrappers (mpm_kernels.hip) ----
void launch_pose(int n_scenes, int t0, int n, float dt, const float* act, double* pose, hipStream_t s);
void launch_zero(void* p, size_t bytes, hipStream_t s);   // fills floor(bytes / 16) 16-byte words
void launch_p2g_plain(const PState& st, const StepParams& P, float4* mmv, hipStream_t s);
void launch_grid_plain(const StepParams& P, const float4* mmv, float4* vgrid, const double* pose_t,
                       const float* act_t, hipStream_t s);
void launch_g2p_plain(const PState& in, const PState& out, const StepParams& P, const float4* vgrid, hipStream_t s);

void launch_g2p_adj_plain(const PState& st, const PState& bar_next, const PState& bar, const StepParams& P,
                          const float4* vgrid, float4* vbar_grid, hipStream_t s);
void launch_grid_adj_plain(const StepParams& P, const float4* mmv, const float4* vbar_grid, float4* mmv_bar,
                           const double* pose_t, const float* act_t, double* acc_t, hipStream_t s);
void launch_p2g_adj_plain(const PState& st, const PState& bar, const StepParams& P, const float4* mmv_bar,
                          hipStream_t s);
void launch_pose_adj(int n_scenes, int T, float dt, const float* act, const double* pose, const double* acc,
                     float* grad_act, hipStream_t s);

// blob loss: scratch holds 2 + 2 LOSS_SLOTS doubles, zeroed by the caller
constexpr int LOSS_SLOTS = 128;
void launch_loss_blob(const StepParams& P, const PState& st, float mx, float my, float mz, float sigma,
                      double* scratch, float* loss, float* gx, hipStream_t s);
void launch_copy_state(const PState& src, const PState& dst, hipStream_t s);
void launch_scene_index(const int64_t* offs_dev, int n_scenes, int N, int* pscene, hipStream_t s);

}  // namespace mpm
