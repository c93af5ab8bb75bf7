// Rigid bodies represented by particles (FluidLab section 3.2): a body's
// particles take the G2P update of an elastic (corotated) solid, then the
// object-level rigid transformation is computed from them and imposed.
//
// Shape matching per body, with rest offsets r_p taken from the body's
// particles at mpm_set_state (about their mass-weighted centroid):
//   c = sum m x' / M,  v_cm = sum m v' / M,
//   A = sum m (x' - c) r^T,  R = rotation of the polar decomposition of A,
//   L = sum m (x' - c) x (v' - v_cm),  w = R I_rest^-1 R^T L,
//   x = c + R r,  v = v_cm + w x (R r),  C = [w]x,  F = R.
// The sums are taken in FP64 as sum m x', sum m v', sum m x' r^T and
// sum m x' x v' and centred afterwards.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "mpm_internal.h"
#include "mpm_fast.h"

namespace mpm {

constexpr int RIGID_ACC = 18;   // FP64 sums per body (forward and adjoint share the slots)
// Each wavefront adds its per-body sums into one of RIGID_SLOTS copies of the
// accumulators (by wavefront index), so that the FP64 atomics of a large body
// do not all queue on the same 18 addresses; the solve adds the copies up.
constexpr int RIGID_SLOTS = 128;
constexpr int RIGID_REC = 48;   // FP64 record of one step's projection per body

// Record layout (doubles): c 0, v_cm 3, R 6, w 15, L 18, z = I^-1 R^T L 21,
// the signed SVD of A / |A|: U 24, s 33, V 36, and |A| at 45.
enum { RR_C = 0, RR_VCM = 3, RR_R = 6, RR_W = 15, RR_L = 18, RR_Z = 21, RR_U = 24, RR_S = 33, RR_V = 36, RR_NRM = 45 };

// Static constants of a body (set at mpm_set_state).
struct RigidBody {
  double M;         // total mass
  double Sr[3];     // sum m r of the stored FP32 rest offsets (zero up to rounding)
  double Iinv[9];   // inverse rest inertia about the centroid
};

// Per-body terms of the adjoint of the projection, applied per particle:
// with x', v' the G2P output (before the projection),
//   xbar' = m (a + Abar r + (v' - v_cm) x Lbar),  vbar' = m (b + Lbar x (x' - c)),
// and zero adjoints for the overwritten C' and F'.
struct RigidAdjTerms {
  float a[3], Ab[9], Lb[3], b[3], c[3], vcm[3];
};

struct RigidCtx {
  int n_bodies;
  const int* body_of;       // [256] material index -> body (-1: not a rigid material)
  float* rest;              // [3][N] rest offsets, by user particle index
  RigidBody* bodies;        // [n_bodies]
  double* acc;              // [RIGID_SLOTS][n_bodies][RIGID_ACC]
  double* rec;              // [n_rec][n_bodies][RIGID_REC]
  RigidAdjTerms* adj;       // [n_bodies]
  double* rest_acc;         // [n_bodies][16] set-up sums
  int* status;              // set-up status (0 ok, 1 singular rest inertia)
};

// Particle rows for the rigid kernels: a state (user order, or a packed
// buffer of a sorted order), its material indices, and the user index of
// each row (NULL = the row is the user index).
struct RigidRows {
  PState st;
  const uint8_t* mat;
  const uint32_t* id;
};

// Set-up: rest offsets and per-body constants from the state x (user order).
void rigid_setup(const RigidCtx& R, const StepParams& P, const PState& user, hipStream_t s);
// Forward: sums over the G2P output, body solve (writes record slot `rec`),
// and the projection of the body particles of `rows` (in place).
void rigid_forward(const RigidCtx& R, const StepParams& P, const RigidRows& rows, double* rec, bool project,
                   hipStream_t s);
// Adjoint of the projection of one step.  abar_next: the adjoint of the
// projected state (packed 25 x N, row map[j] for row j of `rows`, map NULL =
// same rows); rows: the state s_t that the step started from; its G2P is
// recomputed from vgrid (block layout of the tiled path when g is given,
// dense layout otherwise).  Rewrites the x, v, C, F rows of the rigid
// particles of abar_next in place into the adjoint of the G2P output.
void rigid_adjoint(const RigidCtx& R, const StepParams& P, const RigidRows& rows, const uint32_t* map,
                   float* abar_next, const double* rec, const float4* vgrid, const FastGeom* g, hipStream_t s);

}  // namespace mpm
