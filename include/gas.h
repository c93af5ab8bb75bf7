/*
 * gas.h -- C ABI of the MI355X gas step (incompressible advection-projection)
 * and its adjoint.
 *
 * FluidEngine simulates gas (smoke, air) as an incompressible fluid on a
 * Cartesian grid with the advection-projection scheme of Stam 1999 (FluidLab
 * section 3.2, "Gas"), carrying a velocity field and advected quantities such
 * as temperature and smoke density (section 3.1), with a hand-written
 * gradient of the projection (section 3.3).  One step here:
 *   1. semi-Lagrangian advection of the velocity and the scalars by the
 *      velocity of the step's start (trilinear interpolation at the point
 *      traced back for one step; back-traces that leave a grid sample its
 *      boundary);
 *   2. the agent's emitter (the air conditioner of the air-circulation task,
 *      section 4.1) at its pose of the step: every grid value moves towards
 *      its source value by chi(x) = kappa exp(-|x - c|^2 / (2 sigma^2)):
 *      velocities towards emit_speed * R e_y, scalars towards src[];
 *   3. buoyancy on the interior y-faces: v += dt beta (T - t_amb), T (scalar
 *      0) averaged over the two cells the face separates;
 *   4. closed walls: zero normal velocity on the domain's boundary faces;
 *   5. the exact projection onto divergence-free fields (pressure Poisson
 *      equation with Neumann walls, solved spectrally by DCT-II transforms
 *      along the three axes, or by multigrid V-cycles).
 * The emitter pose follows the 6-vector action of section 4.2 like the MPM
 * manipulator: c_{t+1} = c_t + dt u_t, R_{t+1} = exp(dt [w_t]x) R_t.
 *
 * Grid and layout.  nx x ny x nz cells of size h; domain [0, nx h] x
 * [0, ny h] x [0, nz h].  Staggered (MAC) velocities, FP32, row-major with z
 * fastest: u[(i*ny + j)*nz + k] on x-faces (i in [0, nx]), v[(i*(ny+1) + j)*nz
 * + k] on y-faces, w[(i*ny + j)*(nz+1) + k] on z-faces; scalars
 * s[q][(i*ny + j)*nz + k], q < n_scalars, at cell centres; scalar 0 is the
 * temperature.
 *
 * Memory and errors follow mpm.h: the caller owns every device buffer (the
 * state, actions, gradients and one workspace of gas_workspace_bytes()
 * bytes, 256-byte aligned); the library allocates no device memory; all work
 * goes on the stream given to gas_create; calls return an mpm_status.
 * Back-traces that leave a grid are clamped, so a gas step never leaves
 * its domain; non-finite values are reported (gas_last_error_bits).
 */
#ifndef MPM355_GAS_H
#define MPM355_GAS_H

#include "mpm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gas_ctx gas_ctx;

typedef struct {
  int32_t nx, ny, nz;        /* cells per axis: multiples of 4 in [8, 1024]; for the multigrid
                                solver, halving while every axis is even must reach at most
                                4096 cells */
  float h;                   /* cell size */
  float dt;
  float buoyancy, t_amb;     /* beta and the ambient temperature */
  int32_t n_scalars;         /* 1..4 */
  const float* src;          /* [n_scalars] emitter source values (host) */
  float emit_sigma, emit_kappa, emit_speed;   /* sigma > 0, 0 <= kappa <= 1 */
  float emit_pos0[3], emit_rot0[9];           /* emitter pose at t = 0 */
  int32_t horizon;           /* maximum number of steps between gas_set_state calls */
  int32_t ckpt_every;        /* checkpoint period for the backward */
  int32_t requires_grad;     /* record checkpoints during gas_step */
  int32_t mg_cycles;         /* multigrid V-cycles per pressure solve (1..64; 6 reach the FP32
                                residual floor, about 3e-5, on 128^3) */
  int32_t pressure_solver;   /* 0: spectral (exact: DCT-II axis transforms diagonalise the
                                Neumann Laplacian of the closed box; default);
                                1: multigrid V-cycles */
} gas_desc;

typedef struct {
  float* u;
  float* v;
  float* w;
  float* s;                  /* n_scalars consecutive cell arrays */
} gas_state;

/* Bytes of device workspace for this description (0 on bad input). */
size_t gas_workspace_bytes(const gas_desc* d);

/* Create a context on the current device (stream: hipStream_t, NULL = default). */
int gas_create(const gas_desc* d, void* workspace_dev, size_t ws_bytes, void* stream, gas_ctx** out);

/* Borrow the state arrays (device) and reset the clock and the emitter pose.
 * gas_step advects these arrays in place. */
int gas_set_state(gas_ctx* c, const gas_state* st);

/* Copy n steps of actions (device, [n][6]) to steps t0..t0+n-1. */
int gas_set_actions(gas_ctx* c, int32_t t0, int32_t n, const float* actions_dev);

/* Advance n_steps steps from the current clock. */
int gas_step(gas_ctx* c, int32_t n_steps);

/* Reverse-mode gradient of the steps 0..t-1 since gas_set_state (requires_grad).
 * grad_T: dL/d(state at t) (u, v, w required; s may be NULL = 0);
 * grad_actions_dev: dL/d(actions) [t][6]; grad_0 (may be NULL): dL/d(state at 0).
 * The adjoint of the projection is the projection of the adjoint (the
 * projector is self-adjoint on fields with closed walls). */
int gas_step_backward(gas_ctx* c, const gas_state* grad_T, float* grad_actions_dev, gas_state* grad_0);

/* Sensor loss of the air-circulation task: L = sum_m |T(cell_m) - target_m|
 * over n sensors (cells_dev: flat cell indices, device int32; targets_dev:
 * device floats).  loss_dev receives one float; if grad_out is not NULL its
 * arrays are cleared and its s[0] receives dL/dT (sign of the error). */
int gas_sensor_loss(gas_ctx* c, int32_t n, const int32_t* cells_dev, const float* targets_dev, float* loss_dev,
                    gas_state* grad_out);

/* Relative residual |f - A psi| / |f| of the last pressure solve, computed
 * when stats are enabled (one extra reduction per solve). */
int gas_enable_stats(gas_ctx* c, int32_t enable);
int gas_solver_residual(gas_ctx* c, double* rel_residual);

/* Measurement: time launches of the step's dominant kernels with HIP events
 * and read the sums: advection (advect_*), and as smooth_* the six axis
 * transforms of each spectral solve (one event pair around them, counted as
 * six launches) or every finest-level smoothing sweep of the multigrid
 * solver. */
int gas_timing_enable(gas_ctx* c, int32_t enable);
int gas_timing_read(gas_ctx* c, double* advect_ms, int64_t* advect_launches, double* smooth_ms,
                    int64_t* smooth_launches);

/* gas_step and gas_step_backward end with one read of a device error word
 * and return MPM_EDOMAIN when a kernel wrote a non-finite velocity, scalar
 * or adjoint velocity (MPM_ERR_NONFINITE); the bits of the last such call: */
int gas_last_error_bits(const gas_ctx* c, int32_t* bits_out);

int gas_clock(const gas_ctx* c, int32_t* t_out);
int gas_destroy(gas_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* MPM355_GAS_H */
