/*
 * mpm.h -- C ABI of the MI355X MLS-MPM step and its adjoint.
 *
 * The library advances the particle-grid time step of FluidEngine's
 * MLS-MPM solver (FluidLab, section 3.2: particle-to-grid transfer with the
 * material stress, grid operations with boundary conditions and SDF contact,
 * grid-to-particle transfer) on one GPU, and runs the same steps backwards to
 * give gradients of a loss with respect to the manipulator actions (section
 * 3.3 and Appendix A: hand-written SVD gradients and gradient checkpointing).
 * The calls follow the paper's statement of the problem (section 4.2): an MDP
 * whose transition is the simulator, a particle state of positions and
 * velocities (plus the internal C, F, J of MLS-MPM), a 6-vector action of
 * end-effector translational and angular velocity per step, and gradients
 * through long horizons.
 *
 * Conventions
 *  - Unit cube domain, n_grid nodes per axis at x_i = i*dx, dx = 1/n_grid,
 *    y axis up.  All particle arrays are FP32, structure-of-arrays, length N
 *    per component: x[3][N], v[3][N], C[9][N], F[9][N] (row-major 3x3,
 *    component a*3+b), J[N], mat[N] (uint8 index into the material table).
 *  - Liquids carry J only (F is ignored and left unchanged); solids carry F
 *    (J is ignored and left unchanged).
 *  - Device pointers are HIP device memory on the current device.  Host
 *    pointers are read during the call only.
 *  - Every call returns an mpm_status; nothing throws across the ABI.
 *
 * Ownership and memory
 *  - The caller owns all device memory: the particle state, the actions, the
 *    gradients and one workspace of mpm_workspace_bytes() bytes.  The library
 *    allocates no device memory; it borrows the pointers for the lifetime of
 *    the context and never frees them.  mpm_create allocates a small host
 *    struct; mpm_destroy frees it.
 *  - All work is enqueued on the stream given to mpm_create.  mpm_step,
 *    mpm_step_backward and mpm_loss_blob end with one read of the device
 *    error word (the only host synchronisation) and return MPM_EDOMAIN if a
 *    kernel flagged a particle leaving the grid, a non-finite value or a
 *    non-positive sand singular value.
 *  - A context must not be used from two host threads at once.
 */
#ifndef MPM355_MPM_H
#define MPM355_MPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MPM_OK = 0,
  MPM_EINVAL = -1,      /* bad size, NULL pointer or out-of-range parameter */
  MPM_EWORKSPACE = -2,  /* workspace smaller than mpm_workspace_bytes() */
  MPM_EHIP = -3,        /* HIP runtime failure (launch, copy, sync) */
  MPM_EDOMAIN = -4,     /* a kernel flagged an invalid simulation state */
  MPM_ESTATE = -5       /* call out of order: no state, no actions, no recorded forward */
} mpm_status;

typedef enum {
  MPM_ELASTIC_FCR = 0,  /* fixed-corotated elastic solid (the paper's corotated model) */
  MPM_LIQUID_J = 1,     /* liquid: J-based pressure + Newtonian viscosity (F reset, section 3.2) */
  MPM_SAND_DP = 2       /* Hencky elasticity + Drucker-Prager projection (Klar et al. 2016) */
} mpm_material_kind;

/* Error bits of the device error word (returned by mpm_last_error_bits). */
enum {
  MPM_ERR_OUTSIDE = 1,     /* a particle stencil left the grid */
  MPM_ERR_NONFINITE = 2,   /* a non-finite particle value */
  MPM_ERR_SAND_SIGMA = 4,  /* a sand singular value <= 0 */
  MPM_ERR_TILE = 8         /* a particle moved farther than the kernels' tiles allow (CFL > 1) */
};

typedef struct mpm_ctx mpm_ctx;

/* One particle group (typically one box of particles).  Table 4 of the
 * paper gives mu, lambda and rho; p_vol = V_box / N_box and p_mass = rho p_vol
 * are the initial particle volume and mass. */
typedef struct {
  int32_t kind;          /* mpm_material_kind */
  float mu, lambda;      /* Lame parameters */
  float viscosity;       /* liquids: Newtonian eta */
  float friction_deg;    /* sand: Drucker-Prager friction angle (degrees) */
  float cohesion;        /* sand: apex shift in log-strain */
  float p_vol, p_mass;
} mpm_material;

/* Particle state: SoA device pointers, see Conventions.  mat may be NULL in
 * gradient structs. */
typedef struct {
  float* x;
  float* v;
  float* C;
  float* F;
  float* J;
  const uint8_t* mat;
} mpm_state;

/* Scene description.  All pointers are host pointers, copied by mpm_create. */
typedef struct {
  int32_t n_grid;            /* nodes per axis, 8..1024 */
  float dt;                  /* step size (one MPM substep) */
  float gravity[3];
  int32_t bound;             /* slip-wall band in nodes (3) */
  int32_t n_particles;       /* N >= 1 */
  int32_t n_materials;       /* 1..256 */
  const mpm_material* materials;
  int32_t n_scenes;          /* independent scenes in one launch, >= 1 */
  const int64_t* scene_offsets; /* n_scenes+1 particle offsets; NULL when n_scenes == 1 */
  const float* cyl_radius;   /* [n_scenes]; <= 0 disables the cylinder of that scene */
  const float* cyl_pos0;     /* [n_scenes][3] axis point at t = 0 */
  const float* cyl_rot0;     /* [n_scenes][9] orientation at t = 0 (axis = R e_y) */
  float contact_band;        /* contact threshold epsilon, in cells (3) */
  float contact_friction;    /* Coulomb coefficient (0.5) */
  int32_t horizon;           /* maximum number of steps between mpm_set_state calls */
  int32_t ckpt_every;        /* checkpoint period k for the backward (16) */
  int32_t requires_grad;     /* record checkpoints during mpm_step */
} mpm_desc;

/* Bytes of device workspace needed for this description (0 on bad input). */
size_t mpm_workspace_bytes(const mpm_desc* d);

/* Create a context on the current device.  workspace_dev must hold at least
 * mpm_workspace_bytes(d) bytes, 256-byte aligned.  stream is a hipStream_t
 * (NULL = the default stream). */
int mpm_create(const mpm_desc* d, void* workspace_dev, size_t ws_bytes, void* stream, mpm_ctx** out);

/* Borrow the particle state arrays (device) and reset the clock to t = 0,
 * with the cylinder at its initial pose.  mpm_step advances these arrays in
 * place. */
int mpm_set_state(mpm_ctx* c, const mpm_state* st);

/* Copy n steps of actions (device, [n][n_scenes][6]: ux uy uz wx wy wz in
 * the world frame) to steps t0..t0+n-1. */
int mpm_set_actions(mpm_ctx* c, int32_t t0, int32_t n, const float* actions_dev);

/* Advance n_steps steps from the current clock t, applying actions t..t+n-1.
 * The state at a step boundary is the state after grid-to-particle transfer.
 * Records checkpoints every ckpt_every steps when requires_grad is set. */
int mpm_step(mpm_ctx* c, int32_t n_steps);

/* Reverse-mode gradient of the steps 0..t-1 recorded since mpm_set_state.
 * grad_T holds dL/d(state at t) (x and v required, C/F/J may be NULL = 0);
 * grad_actions_dev receives dL/d(actions) [t][n_scenes][6]; grad_0, if not
 * NULL, receives dL/d(state at 0) (x, v, C, F, J).  Does not change the
 * forward state. */
int mpm_step_backward(mpm_ctx* c, const mpm_state* grad_T, float* grad_actions_dev, mpm_state* grad_0);

/* Blob loss of the liquid particles of the current state:
 * L = mean_liquid |x_p - mu_g|^2 + 3 sigma_g^2 (expected squared distance to a
 * Gaussian N(mu_g, sigma_g^2 I)).  loss_dev receives one float; if grad_out
 * is not NULL its x array receives dL/dx (zero for non-liquid particles). */
int mpm_loss_blob(mpm_ctx* c, const float mu_g[3], float sigma_g, float* loss_dev, mpm_state* grad_out);

/* Current clock (number of steps since mpm_set_state). */
int mpm_clock(const mpm_ctx* c, int32_t* t_out);

/* Error bits (MPM_ERR_*) seen by the last call that returned MPM_EDOMAIN. */
int mpm_last_error_bits(const mpm_ctx* c, int32_t* bits_out);

/* Measurement: when enabled, every launch of the step's dominant kernel
 * (the particle kernel that carries the transfer traffic) is bracketed by
 * HIP events on the context's stream; elapsed times are summed when a call
 * synchronises.  mpm_timing_read returns the accumulated time, the number of
 * timed launches and the kernel's name, and resets the counters. */
int mpm_timing_enable(mpm_ctx* c, int32_t enable);
int mpm_timing_read(mpm_ctx* c, double* total_ms, int64_t* launches, char* name, int32_t name_len);

/* Launch-shape and mode options of the forward path (mpm_step without
 * requires_grad).  Defaults: graph 0, particle workgroup 256 threads, 2048
 * particle workgroups, 2048 grid workgroups. */
enum {
  MPM_OPT_GRAPH = 1,          /* 1: capture each call shape in a HIP graph and replay it */
  MPM_OPT_PART_THREADS = 2,   /* 128 or 256 threads per particle workgroup */
  MPM_OPT_PART_WGS = 3,       /* particle workgroups per launch (persistent, 64..65536) */
  MPM_OPT_GRID_WGS = 4        /* grid-update workgroups per launch (64..65536) */
};
int mpm_set_option(mpm_ctx* c, int32_t key, int32_t value);
int mpm_get_option(const mpm_ctx* c, int32_t key, int32_t* value);

/* Autotuner: times n_steps of the forward path from the current state (the
 * state and the clock are left unchanged; actions t..t+n_steps-1 must be
 * set) for every launch shape in a fixed candidate set, keeps the fastest
 * and returns it in best[4] = {part_threads, part_wgs, grid_wgs,
 * microseconds per step}. */
int mpm_autotune(mpm_ctx* c, int32_t n_steps, int32_t* best);

/* Free the host context (not the borrowed device memory). */
int mpm_destroy(mpm_ctx* c);

/* Static text for a status code. */
const char* mpm_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* MPM355_MPM_H */
