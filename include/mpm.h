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
  MPM_SAND_DP = 2,      /* Hencky elasticity + Drucker-Prager projection (Klar et al. 2016) */
  MPM_PLASTIC_VM = 3,   /* Hencky elasticity + von Mises projection in log strain: the
                           non-Newtonian ice cream of section 3.2 */
  MPM_PLASTIC_BOX = 4,  /* corotated elasticity + Box yield (singular values of F clamped to
                           [1 - theta_c, 1 + theta_s]): the plastic material of section 3.2 */
  MPM_RIGID = 5         /* rigid body represented by particles (section 3.2), one body per
                           material: see "Rigid bodies" below */
} mpm_material_kind;

/* Rigid bodies.  The particles of a material of kind MPM_RIGID form one body.
 * Each step they first take the G2P update of a corotated elastic solid;
 * then the body's rigid transformation is found by shape matching and
 * imposed: with rest offsets r_p (the particle positions at mpm_set_state
 * about their mass-weighted centroid, kept for the life of the state), the
 * centroid c and velocity v_cm of the updated particles, the rotation R of
 * the polar decomposition of sum m (x - c) r^T and the angular velocity
 * w = R I_rest^-1 R^T L from the angular momentum L about c, every particle
 * is set to x = c + R r, v = v_cm + w x (R r), C = [w]x, F = R.  Linear and
 * angular momentum are kept.  The rest offsets are constants of the body:
 * gradients do not flow into them.  A body whose particles do not span 3-D
 * space (singular rest inertia) makes mpm_set_state return MPM_EINVAL.
 * Scenes with rigid bodies step unfused (the projection needs the whole body
 * between G2P and the next P2G): MPM_OPT_GRAPH and the kernel timer do not
 * apply to them, and sample logging and the learned closure are refused
 * (MPM_ESTATE).  Give each body of each batched scene its own material. */

/* Error bits of the device error word (returned by mpm_last_error_bits). */
enum {
  MPM_ERR_OUTSIDE = 1,     /* a particle stencil left the grid */
  MPM_ERR_NONFINITE = 2,   /* a non-finite particle value */
  MPM_ERR_SAND_SIGMA = 4,  /* a sand, von Mises or Box-yield singular value <= 0 */
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
  float yield_stress;    /* von Mises: yield stress; the return radius in log strain is
                            yield_stress / (2 mu) */
  float theta_c, theta_s; /* Box yield: critical compression (0 <= theta_c < 1) and stretch */
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
  int32_t ckpt_every;        /* checkpoint period k for the backward (16); 0 = keep a block-sorted
                                 record of every step during the forward, so that the backward
                                 recomputes nothing (tiled adjoint, no rigid bodies; the workspace
                                 then holds horizon records of about 113 B per particle plus
                                 2 x 1 KB per grid block) */
  int32_t requires_grad;     /* record checkpoints during mpm_step */
} mpm_desc;

/* Bytes of device workspace needed for this description (0 on bad input):
 * the sorted particle buffers and block grid of the step (section 3.2) and,
 * with requires_grad, the checkpoints and segment records of the adjoint
 * (Appendix A). */
size_t mpm_workspace_bytes(const mpm_desc* d);

/* Create a context on the current device for the scene d: the simulator of
 * section 3.2 with the materials of Table 4 (Appendix B.1) and the
 * end-effector of section 4.2.  workspace_dev must hold at least
 * mpm_workspace_bytes(d) bytes, 256-byte aligned (else MPM_EWORKSPACE; a bad
 * description gives MPM_EINVAL).  stream is a hipStream_t (NULL = the
 * default stream).  *out receives the host context. */
int mpm_create(const mpm_desc* d, void* workspace_dev, size_t ws_bytes, void* stream, mpm_ctx** out);

/* Borrow the particle state arrays (device) and reset the clock to t = 0,
 * with the cylinder at its initial pose.  The state is the MDP state of
 * section 4.2 (particle positions and velocities) plus the internal C, F, J
 * that MLS-MPM carries (section 3.2).  mpm_step advances these arrays in
 * place.  Rigid bodies take their rest shapes from this state.  NULL
 * pointers give MPM_EINVAL. */
int mpm_set_state(mpm_ctx* c, const mpm_state* st);

/* Copy n steps of actions (device, [n][n_scenes][6]: ux uy uz wx wy wz in
 * the world frame) to steps t0..t0+n-1.  The action space of section 4.2:
 * the end-effector's translational and angular velocity, one 6-vector per
 * step.  A range outside [0, horizon) gives MPM_EINVAL. */
int mpm_set_actions(mpm_ctx* c, int32_t t0, int32_t n, const float* actions_dev);

/* Advance n_steps steps from the current clock t, applying actions t..t+n-1:
 * the transition function of section 4.2, one MLS-MPM substep each
 * (section 3.2: particle-to-grid transfer with the material stress, grid
 * update with gravity, slip walls and the soft contact of section 5.1,
 * grid-to-particle transfer updating v, C, F or J and x).  The state at a
 * step boundary is the state after grid-to-particle transfer.  Records
 * checkpoints every ckpt_every steps when requires_grad is set (Appendix A).
 * MPM_ESTATE without a state or with an action of the range unset;
 * MPM_EDOMAIN when a kernel flags an invalid state (MPM_ERR_* bits). */
int mpm_step(mpm_ctx* c, int32_t n_steps);

/* Reverse-mode gradient of the steps 0..t-1 recorded since mpm_set_state:
 * the differentiable simulation of section 3.3 and Appendix A (hand-written
 * gradients of the SVD-based stresses and projections, checkpoints every
 * ckpt_every steps recomputed segment by segment).
 * grad_T holds dL/d(state at t) (x and v required, C/F/J may be NULL = 0);
 * grad_actions_dev receives dL/d(actions) [t][n_scenes][6]; grad_0, if not
 * NULL, receives dL/d(state at 0) (x, v, C, F, J).  Does not change the
 * forward state. */
int mpm_step_backward(mpm_ctx* c, const mpm_state* grad_T, float* grad_actions_dev, mpm_state* grad_0);

/* Blob loss of the liquid particles of the current state (a particle-
 * distribution loss in the spirit of Appendix B.2's task losses):
 * L = mean_liquid |x_p - mu_g|^2 + 3 sigma_g^2 (expected squared distance to a
 * Gaussian N(mu_g, sigma_g^2 I)).  loss_dev receives one float; if grad_out
 * is not NULL its x array receives dL/dx (zero for non-liquid particles). */
int mpm_loss_blob(mpm_ctx* c, const float mu_g[3], float sigma_g, float* loss_dev, mpm_state* grad_out);

/* Current clock (number of steps since mpm_set_state, the MDP's time step
 * index of section 4.2). */
int mpm_clock(const mpm_ctx* c, int32_t* t_out);

/* Error bits (MPM_ERR_*) seen by the last call that returned MPM_EDOMAIN.
 * Invalid states are reported, never clamped. */
int mpm_last_error_bits(const mpm_ctx* c, int32_t* bits_out);

/* Measurement: when enabled, every launch of the step's dominant kernel
 * (the particle kernel that carries the transfer traffic) is bracketed by
 * HIP events on the context's stream; elapsed times are summed when a call
 * synchronises.  mpm_timing_read returns the accumulated time, the number of
 * timed launches and the kernel's name, and resets the counters.  While
 * timing is enabled, calls run without graph capture (MPM_OPT_GRAPH is
 * ignored) so that the events bracket the launches themselves. */
int mpm_timing_enable(mpm_ctx* c, int32_t enable);
int mpm_timing_read(mpm_ctx* c, double* total_ms, int64_t* launches, char* name, int32_t name_len);

/* Launch-shape and mode options.  Defaults: graph 0, particle workgroup 256
 * threads, 2048 particle workgroups, 2048 grid workgroups, tiled adjoint.
 * MPM_OPT_ADJOINT selects how requires_grad contexts step and differentiate:
 * 0 = the tiled path (forward on the tiled path, checkpoint segments
 * recomputed on block-sorted states, tiled adjoint kernels); 1 = the plain
 * path (one particle per thread with global atomics on a dense grid, for
 * both the forward and the adjoint).  Both record the same checkpoints. */
enum {
  MPM_OPT_GRAPH = 1,          /* 1: capture each call shape in a HIP graph and replay it (forward calls
                                 without rigid bodies, including those that keep every step's record;
                                 tiled backward calls without rigid bodies) */
  MPM_OPT_PART_THREADS = 2,   /* 128, 256 or 512 threads per particle workgroup */
  MPM_OPT_PART_WGS = 3,       /* particle workgroups per launch (persistent, 64..65536) */
  MPM_OPT_GRID_WGS = 4,       /* grid-update workgroups per launch (64..65536) */
  MPM_OPT_ADJOINT = 5,        /* 0: tiled (default), 1: plain */
  MPM_OPT_N_KEYS = 6,         /* read only: grid blocks of the context (rows of a sort snapshot list) */
  MPM_OPT_SHARE_CHUNKS = 7    /* a block holding more than this many chunks (of MPM_OPT_PART_THREADS
                                 particles) is shared by two particle workgroups; 0 = never; default 2 */
};
int mpm_set_option(mpm_ctx* c, int32_t key, int32_t value);
int mpm_get_option(const mpm_ctx* c, int32_t key, int32_t* value);

/* Integer outputs of the block sort that orders the particles for the
 * step's transfers (section 3.2's particle-grid transfers, run on particles
 * grouped by 4^3-node grid block), for checking it.  which = 0: sorts the
 * state set by mpm_set_state (the import that starts every mpm_step) and
 * writes the user indices of the sorted particles (id_dev, N uint32), their
 * block keys (key_dev, N uint32) and the occupied-block list (list_dev,
 * MPM_OPT_N_KEYS rows of int32 {key, offset, count, 0}; *n_list_out rows
 * are valid, in no particular order).  which = 2: the same, with the rows in
 * increasing key order (the order the adjoint's recompute lists the blocks
 * in).  which = 1: writes the user indices
 * of the sorted buffer the last forward mpm_step call left (key_dev,
 * list_dev and n_list_out unused, may be NULL; MPM_ESTATE if no such call).
 * A block key is (scene << 3 kb) | the Morton interleave of the block
 * coordinates (x bits above y bits above z bits), kb the bits per axis of
 * ceil(n_grid / 4).  Device arrays are caller-owned; the call synchronises. */
int mpm_sort_snapshot(mpm_ctx* c, int32_t which, uint32_t* id_dev, uint32_t* key_dev, int32_t* list_dev,
                      int32_t* n_list_out);

/* Autotuner: times n_steps of the forward path from the current state (the
 * state and the clock are left unchanged; actions t..t+n_steps-1 must be
 * set) for every launch shape in a fixed candidate set (particles per
 * chunk, workgroup counts, and the chunk count above which a block is
 * shared by two workgroups), keeps the fastest and returns it in best[5] =
 * {part_threads, part_wgs, grid_wgs, microseconds per step, share_chunks}. */
int mpm_autotune(mpm_ctx* c, int32_t n_steps, int32_t* best);

/* ---- learned closure of the Drucker-Prager cone return (sand) ----------
 * Not part of the paper, whose sand and plastic models use exact return
 * maps (section 3.2): an extension that replaces the cone case of the
 * Drucker-Prager projection (Klar et al. 2016) by a small network, judged
 * by the exact projection.
 * A 6 -> 64 -> 64 -> 3 MLP (ReLU; BF16 weights, FP32 accumulation on the
 * matrix cores) maps (log singular values of the trial F sorted descending,
 * alpha, c, kappa) to the projected log singular values.  It is trained on
 * samples logged from the simulator's own exact projections.  The state
 * buffer (device, caller-owned, mpm_mlp_state_bytes()) holds the FP32 master
 * weights, the Adam moments and the inference copy. */

/* Log every exact cone-case projection of sand particles during mpm_step:
 * records of 9 floats (log sigma_tr[3], alpha, c, kappa, projected[3]) are
 * appended to buf_dev (capacity records) and *count_dev (device uint64) is
 * advanced (it may exceed the capacity; records beyond it are dropped).
 * buf_dev == NULL stops logging.  Returns MPM_ESTATE with an active closure,
 * with rigid bodies, and in a requires_grad context with ckpt_every == 0
 * (that context's forward keeps each step's record and runs no logging). */
int mpm_log_samples(mpm_ctx* c, float* buf_dev, uint64_t capacity, uint64_t* count_dev);

/* Use the trained MLP (mlp_state_dev; NULL disables) for the cone case of
 * the sand projection in mpm_step.  A prediction whose yield residual
 * |f(eps)| + |tr eps - tr eps_tr| exceeds residual_tol falls back to the
 * exact return.  Forward only: a requires_grad context returns MPM_ESTATE
 * (its adjoint differentiates the exact return). */
int mpm_set_closure(mpm_ctx* c, const void* mlp_state_dev, float residual_tol);

/* Counts of closure predictions accepted and fallen back since the last read
 * (reads reset them). */
int mpm_closure_stats(mpm_ctx* c, uint64_t* accepted, uint64_t* fallback);

size_t mpm_mlp_state_bytes(void);
/* Scratch (device) for mpm_mlp_train / mpm_mlp_grad with this batch size. */
size_t mpm_mlp_scratch_bytes(int32_t batch);
/* Initialise: normalisation statistics from the n logged records in
 * samples_dev, weights from init_params (host, MLP parameter vector of 4803
 * floats W1 b1 W2 b2 W3 b3, row-major [out][in]) or, if NULL, a seeded
 * He-uniform draw; zero Adam moments. */
int mpm_mlp_init(void* state_dev, const float* samples_dev, int64_t n, const float* init_params, uint64_t seed,
                 void* stream);
/* Train with Adam (lr; beta 0.9/0.999) on the n records, `epochs` passes of
 * batches of `batch` records starting at a seeded offset; loss_hist_host
 * (may be NULL) receives the mean batch loss of each epoch. */
int mpm_mlp_train(void* state_dev, const float* samples_dev, int64_t n, int32_t batch, int32_t epochs, float lr,
                  uint64_t seed, void* scratch_dev, double* loss_hist_host, void* stream);
/* Loss (host) and parameter gradient (device, 4803 floats) on the first
 * min(n, batch) records, without updating the weights. */
int mpm_mlp_grad(void* state_dev, const float* samples_dev, int64_t n, int32_t batch, void* scratch_dev,
                 float* grad_out_dev, double* loss_out_host, void* stream);
/* mpm_mlp_grad for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the per-sample scratch is a static device array of the library, sized for
 * MPM_MLP_NOALLOC_MAX_BATCH records (2.2 MB, held by each device the
 * library runs on until the process ends), instead of a caller buffer.
 * min(n, batch) above the maximum returns MPM_EWORKSPACE and does nothing.
 * The call allocates nothing.  Every call on one device shares that
 * device's scratch (each call writes all of it that it reads): calls that
 * overlap on one device, from several streams or host threads, race. */
#define MPM_MLP_NOALLOC_MAX_BATCH 2048
int mpm_mlp_grad_noalloc(void* state_dev, const float* samples_dev, int64_t n, int32_t batch, float* grad_out_dev,
                         double* loss_out_host, void* stream);
/* Outputs (n x 3) for n records of 9 floats (only the 6 inputs are read). */
int mpm_mlp_predict(const void* state_dev, const float* records_dev, int64_t n, float* y_dev, void* stream);
/* Copy the FP32 parameter vector and/or the inference blob to the host. */
int mpm_mlp_params(const void* state_dev, float* params_host, void* blob_host, void* stream);

/* Free the host context (not the borrowed device memory). */
int mpm_destroy(mpm_ctx* c);

/* Static text for a status code. */
const char* mpm_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* MPM355_MPM_H */
