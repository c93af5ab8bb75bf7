// Rigid bodies from particles (FluidLab section 3.2): set-up of the rest
// shapes, the per-step shape-matching projection and its adjoint.  The
// per-body sums are reduced per wavefront (one FP64 atomic per body present
// in the wavefront and per component); the body solves run one thread per
// body.
#include <hip/hip_runtime.h>
#include <math.h>
#include "mpm_rigid.h"
#include "mpm_blocks.h"
#include "mpm_math.h"
#include "mpm_phys.h"

namespace mpm {

namespace {

inline unsigned nblk(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

// Adds each lane's K values into base[body * stride + q] for the lanes with
// body >= 0: per distinct body of the wavefront, a shuffle sum and one atomic
// per component.  Every lane of the wavefront must call it.
template <int K>
__device__ void body_reduce(int body, const double* v, double* base, int stride) {
  const int lane = __lane_id();
  unsigned long long pending = __ballot(body >= 0);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int b = __shfl(body, leader);
    const bool mine = body == b;
    pending &= ~__ballot(mine);
#pragma unroll
    for (int q = 0; q < K; q++) {
      double x = mine ? v[q] : 0.0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
      if (lane == leader) atomicAdd(base + (size_t)b * stride + q, x);
    }
  }
}

// The accumulator copy this wavefront adds into.
__device__ inline double* wave_slot(double* acc, int n_bodies) {
  const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  return acc + (size_t)(wave % RIGID_SLOTS) * n_bodies * RIGID_ACC;
}

// Sum of the RIGID_SLOTS copies of body b's accumulators into tot (in lane 0
// of the calling wavefront, which must be the whole workgroup); the copies
// are cleared for the next use.
__device__ void gather_slots(double* acc, int n_bodies, int b, double* tot) {
  const int lane = threadIdx.x;
#pragma unroll
  for (int q = 0; q < RIGID_ACC; q++) tot[q] = 0.0;
  for (int sl = lane; sl < RIGID_SLOTS; sl += 64) {
    double* S = acc + ((size_t)sl * n_bodies + b) * RIGID_ACC;
#pragma unroll
    for (int q = 0; q < RIGID_ACC; q++) { tot[q] += S[q]; S[q] = 0.0; }
  }
#pragma unroll
  for (int q = 0; q < RIGID_ACC; q++)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) tot[q] += __shfl_xor(tot[q], off);
}

MPM_DI void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

MPM_DI int row_body(const RigidRows& rows, const int* body_of, int j, int N, uint32_t& pid) {
  if (j >= N) return -1;
  const int b = body_of[rows.mat[j]];
  pid = rows.id ? rows.id[j] : (uint32_t)j;
  if (pid >= (uint32_t)N) return -1;
  return b;
}

// ---- set-up ---------------------------------------------------------------
// rest_acc per body: [0] sum m, [1..3] sum m x, [4..6] sum m r, [7..15] the
// rest inertia sum m (|r|^2 I - r r^T)
__global__ __launch_bounds__(256) void k_rigid_rest_sum(PState u, const uint8_t* __restrict__ mat,
                                                        const int* __restrict__ body_of, const MatDev* __restrict__ mats,
                                                        double* __restrict__ rest_acc) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = u.N;
  const int b = j < N ? body_of[mat[j]] : -1;
  double v[4] = {0, 0, 0, 0};
  if (b >= 0) {
    const double m = (double)mats[mat[j]].mass;
    v[0] = m;
#pragma unroll
    for (int a = 0; a < 3; a++) v[1 + a] = m * (double)u.x[a * N + j];
  }
  body_reduce<4>(b, v, rest_acc, 16);
}

__global__ __launch_bounds__(256) void k_rigid_rest(PState u, const uint8_t* __restrict__ mat,
                                                    const int* __restrict__ body_of, const MatDev* __restrict__ mats,
                                                    double* __restrict__ rest_acc, float* __restrict__ rest) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = u.N;
  const int b = j < N ? body_of[mat[j]] : -1;
  double v[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (b >= 0) {
    const double* S = rest_acc + (size_t)b * 16;
    const double m = (double)mats[mat[j]].mass;
    double r[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      const float rf = (float)((double)u.x[a * N + j] - S[1 + a] / S[0]);
      rest[a * (size_t)N + j] = rf;
      r[a] = (double)rf;
    }
    const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
#pragma unroll
    for (int a = 0; a < 3; a++) v[a] = m * r[a];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int c = 0; c < 3; c++) v[3 + a * 3 + c] = m * ((a == c ? rr : 0.0) - r[a] * r[c]);
  }
  body_reduce<12>(b, v, rest_acc + 4, 16);
}

__global__ void k_rigid_init(int n_bodies, const double* __restrict__ rest_acc, RigidBody* __restrict__ bodies,
                             int* __restrict__ status) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_bodies) return;
  const double* S = rest_acc + (size_t)b * 16;
  RigidBody B;
  B.M = S[0];
#pragma unroll
  for (int a = 0; a < 3; a++) B.Sr[a] = S[4 + a];
  const double* I = S + 7;
  double K[9];
  cof3(I, K);
  const double det = I[0] * K[0] + I[1] * K[1] + I[2] * K[2];
  const double tr = I[0] + I[4] + I[8];
  // a body whose particles do not span 3-D space has no rotation to match
  const bool ok = B.M > 0.0 && tr > 0.0 && det > 1e-9 * tr * tr * tr;
#pragma unroll
  for (int k = 0; k < 9; k++) B.Iinv[k] = ok ? K[k] / det : 0.0;   // I symmetric: inverse = cof / det
  bodies[b] = B;
  if (!ok) atomicOr(status, 1);
}

// ---- forward --------------------------------------------------------------
// acc per body: [0..2] sum m x', [3..5] sum m v', [6..14] sum m x' r^T,
// [15..17] sum m x' x v'
__global__ __launch_bounds__(256) void k_rigid_sum(RigidRows rows, int n_bodies, const int* __restrict__ body_of,
                                                   const MatDev* __restrict__ mats, const float* __restrict__ rest,
                                                   double* __restrict__ acc) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = rows.st.N;
  uint32_t pid = 0;
  const int b = row_body(rows, body_of, j, N, pid);
  double v[RIGID_ACC];
#pragma unroll
  for (int q = 0; q < RIGID_ACC; q++) v[q] = 0.0;
  if (b >= 0) {
    const double m = (double)mats[rows.mat[j]].mass;
    double x[3], vv[3], r[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      x[a] = (double)rows.st.x[a * (size_t)N + j];
      vv[a] = (double)rows.st.v[a * (size_t)N + j];
      r[a] = (double)rest[a * (size_t)N + pid];
    }
#pragma unroll
    for (int a = 0; a < 3; a++) { v[a] = m * x[a]; v[3 + a] = m * vv[a]; }
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int c = 0; c < 3; c++) v[6 + a * 3 + c] = m * x[a] * r[c];
    double xv[3];
    cross3(x, vv, xv);
#pragma unroll
    for (int a = 0; a < 3; a++) v[15 + a] = m * xv[a];
  }
  body_reduce<RIGID_ACC>(b, v, wave_slot(acc, n_bodies), RIGID_ACC);
}

// one wavefront per body
__global__ __launch_bounds__(64) void k_rigid_solve(int n_bodies, const RigidBody* __restrict__ bodies,
                                                    double* __restrict__ acc, double* __restrict__ rec) {
  const int b = blockIdx.x;
  double S[RIGID_ACC];
  gather_slots(acc, n_bodies, b, S);
  if (threadIdx.x != 0) return;
  double* O = rec + (size_t)b * RIGID_REC;
  const RigidBody B = bodies[b];
  const double iM = 1.0 / B.M;
  double c[3], vcm[3], A[9], L[3];
#pragma unroll
  for (int a = 0; a < 3; a++) { c[a] = S[a] * iM; vcm[a] = S[3 + a] * iM; }
  // A = sum m (x' - c) r^T = sum m x' r^T - c (sum m r)^T
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int k = 0; k < 3; k++) A[a * 3 + k] = S[6 + a * 3 + k] - c[a] * B.Sr[k];
  // L = sum m (x' - c) x (v' - v_cm) = sum m x' x v' - M c x v_cm
  double cv[3];
  cross3(c, vcm, cv);
#pragma unroll
  for (int a = 0; a < 3; a++) L[a] = S[15 + a] - B.M * cv[a];
  // polar rotation of A from the signed SVD of A / |A| (scale-free)
  double nrm = 0.0;
#pragma unroll
  for (int k = 0; k < 9; k++) nrm += A[k] * A[k];
  nrm = sqrt(nrm);
  const double inrm = nrm > 0.0 ? 1.0 / nrm : 0.0;
  double An[9], U[9], s[3], V[9], R[9];
#pragma unroll
  for (int k = 0; k < 9; k++) An[k] = A[k] * inrm;
  svd3(An, U, s, V);
  matmul_nt(U, V, R);
  // w = R I^-1 R^T L
  double u[3], z[3], w[3];
#pragma unroll
  for (int i = 0; i < 3; i++) u[i] = R[i] * L[0] + R[3 + i] * L[1] + R[6 + i] * L[2];
#pragma unroll
  for (int i = 0; i < 3; i++) z[i] = B.Iinv[i * 3] * u[0] + B.Iinv[i * 3 + 1] * u[1] + B.Iinv[i * 3 + 2] * u[2];
#pragma unroll
  for (int i = 0; i < 3; i++) w[i] = R[i * 3] * z[0] + R[i * 3 + 1] * z[1] + R[i * 3 + 2] * z[2];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    O[RR_C + a] = c[a]; O[RR_VCM + a] = vcm[a]; O[RR_W + a] = w[a]; O[RR_L + a] = L[a]; O[RR_Z + a] = z[a];
    O[RR_S + a] = s[a];
  }
#pragma unroll
  for (int k = 0; k < 9; k++) { O[RR_R + k] = R[k]; O[RR_U + k] = U[k]; O[RR_V + k] = V[k]; }
  O[RR_NRM] = nrm;
}

__global__ __launch_bounds__(256) void k_rigid_project(RigidRows rows, const int* __restrict__ body_of,
                                                       const float* __restrict__ rest, const double* __restrict__ rec) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = rows.st.N;
  uint32_t pid = 0;
  const int b = row_body(rows, body_of, j, N, pid);
  if (b < 0) return;
  const double* O = rec + (size_t)b * RIGID_REC;
  double r[3], q[3], wq[3];
#pragma unroll
  for (int a = 0; a < 3; a++) r[a] = (double)rest[a * (size_t)N + pid];
#pragma unroll
  for (int a = 0; a < 3; a++) q[a] = O[RR_R + a * 3] * r[0] + O[RR_R + a * 3 + 1] * r[1] + O[RR_R + a * 3 + 2] * r[2];
  cross3(O + RR_W, q, wq);
  const PState& st = rows.st;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    st.x[a * (size_t)N + j] = (float)(O[RR_C + a] + q[a]);
    st.v[a * (size_t)N + j] = (float)(O[RR_VCM + a] + wq[a]);
  }
  const double* w = O + RR_W;
  const double W[9] = {0.0, -w[2], w[1], w[2], 0.0, -w[0], -w[1], w[0], 0.0};
#pragma unroll
  for (int k = 0; k < 9; k++) {
    st.C[k * (size_t)N + j] = (float)W[k];
    st.F[k * (size_t)N + j] = (float)O[RR_R + k];
  }
}

// ---- adjoint --------------------------------------------------------------
// acc per body: [0..2] sum xbar, [3..5] sum vbar, [6..8] wbar, [9..17] Rbar,
// where per particle (q = R r): wbar_p = q x vbar + vee(Cbar - Cbar^T) and
// Rbar_p = (xbar + vbar x w) r^T + Fbar.
__global__ __launch_bounds__(256) void k_rigid_adj_sum(RigidRows rows, int n_bodies, const uint32_t* __restrict__ map,
                                                       const float* __restrict__ abar, const int* __restrict__ body_of,
                                                       const float* __restrict__ rest, const double* __restrict__ rec,
                                                       double* __restrict__ acc) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = rows.st.N;
  uint32_t pid = 0;
  int b = row_body(rows, body_of, j, N, pid);
  const uint32_t jn = (b >= 0 && map) ? map[j] : (uint32_t)j;
  if (jn >= (uint32_t)N) b = -1;
  double v[RIGID_ACC];
#pragma unroll
  for (int q = 0; q < RIGID_ACC; q++) v[q] = 0.0;
  if (b >= 0) {
    const double* O = rec + (size_t)b * RIGID_REC;
    double r[3], q[3], xb[3], vb[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      r[a] = (double)rest[a * (size_t)N + pid];
      xb[a] = (double)abar[a * (size_t)N + jn];
      vb[a] = (double)abar[(3 + a) * (size_t)N + jn];
    }
#pragma unroll
    for (int a = 0; a < 3; a++) q[a] = O[RR_R + a * 3] * r[0] + O[RR_R + a * 3 + 1] * r[1] + O[RR_R + a * 3 + 2] * r[2];
    double Cb[9];
#pragma unroll
    for (int k = 0; k < 9; k++) Cb[k] = (double)abar[(6 + k) * (size_t)N + jn];
    double qv[3], vw[3];
    cross3(q, vb, qv);
    cross3(vb, O + RR_W, vw);
    v[0] = xb[0]; v[1] = xb[1]; v[2] = xb[2];
    v[3] = vb[0]; v[4] = vb[1]; v[5] = vb[2];
    v[6] = qv[0] + Cb[7] - Cb[5];
    v[7] = qv[1] + Cb[2] - Cb[6];
    v[8] = qv[2] + Cb[3] - Cb[1];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int c = 0; c < 3; c++)
        v[9 + a * 3 + c] = (xb[a] + vw[a]) * r[c] + (double)abar[(15 + a * 3 + c) * (size_t)N + jn];
  }
  body_reduce<RIGID_ACC>(b, v, wave_slot(acc, n_bodies), RIGID_ACC);
}

// one wavefront per body
__global__ __launch_bounds__(64) void k_rigid_adj_solve(int n_bodies, const RigidBody* __restrict__ bodies,
                                                        double* __restrict__ acc, const double* __restrict__ rec,
                                                        RigidAdjTerms* __restrict__ out) {
  const int b = blockIdx.x;
  double S[RIGID_ACC];
  gather_slots(acc, n_bodies, b, S);
  if (threadIdx.x != 0) return;
  const double* O = rec + (size_t)b * RIGID_REC;
  const RigidBody B = bodies[b];
  const double* R = O + RR_R;
  const double* z = O + RR_Z;
  const double* L = O + RR_L;
  double Rb[9], wb[3];
#pragma unroll
  for (int a = 0; a < 3; a++) wb[a] = S[6 + a];
#pragma unroll
  for (int k = 0; k < 9; k++) Rb[k] = S[9 + k];
  // w = R z, z = I^-1 u, u = R^T L
  double zb[3], ub[3], Lb[3];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int k = 0; k < 3; k++) Rb[a * 3 + k] += wb[a] * z[k];
#pragma unroll
  for (int k = 0; k < 3; k++) zb[k] = R[k] * wb[0] + R[3 + k] * wb[1] + R[6 + k] * wb[2];
#pragma unroll
  for (int k = 0; k < 3; k++) ub[k] = B.Iinv[k] * zb[0] + B.Iinv[3 + k] * zb[1] + B.Iinv[6 + k] * zb[2];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int k = 0; k < 3; k++) Rb[a * 3 + k] += L[a] * ub[k];
#pragma unroll
  for (int a = 0; a < 3; a++) Lb[a] = R[a * 3] * ub[0] + R[a * 3 + 1] * ub[1] + R[a * 3 + 2] * ub[2];
  // adjoint of the polar rotation: the isotropic map with g = 1 on the
  // singular values of A (those of A / |A| times |A|)
  const double nrm = O[RR_NRM];
  const double s[3] = {O[RR_S] * nrm, O[RR_S + 1] * nrm, O[RR_S + 2] * nrm};
  const double g[3] = {1.0, 1.0, 1.0};
  const double zero9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double Ab[9];
  iso_adjoint(O + RR_U, s, O + RR_V, g, zero9, zero9, Rb, Ab);
  RigidAdjTerms T;
  const double iM = 1.0 / B.M;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    const double AS = Ab[a * 3] * B.Sr[0] + Ab[a * 3 + 1] * B.Sr[1] + Ab[a * 3 + 2] * B.Sr[2];
    T.a[a] = (float)((S[a] - AS) * iM);
    T.b[a] = (float)(S[3 + a] * iM);
    T.Lb[a] = (float)Lb[a];
    T.c[a] = (float)O[RR_C + a];
    T.vcm[a] = (float)O[RR_VCM + a];
  }
#pragma unroll
  for (int k = 0; k < 9; k++) T.Ab[k] = (float)Ab[k];
  out[b] = T;
}

// Recompute v' of the rigid rows (G2P of the state s_t from the step's grid
// velocities) and replace their adjoint rows by the adjoint of the G2P output.
template <bool BLOCK>
__global__ __launch_bounds__(256) void k_rigid_adj_apply(RigidRows rows, const uint32_t* __restrict__ map,
                                                         float* __restrict__ abar, const int* __restrict__ body_of,
                                                         const MatDev* __restrict__ mats, const float* __restrict__ rest,
                                                         const RigidAdjTerms* __restrict__ terms,
                                                         const float4* __restrict__ vgrid, StepParams P, FastGeom g) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = rows.st.N;
  uint32_t pid = 0;
  const int b = row_body(rows, body_of, j, N, pid);
  if (b < 0) return;
  const uint32_t jn = map ? map[j] : (uint32_t)j;
  if (jn >= (uint32_t)N) return;
  float x[3];
#pragma unroll
  for (int a = 0; a < 3; a++) x[a] = rows.st.x[a * (size_t)N + j];
  Stencil S;
  if (!stencil_setup(x, P, S)) return;   // flagged by the step's other kernels
  const int sc = P.pscene[pid];
  const int n = P.n_grid;
  float vn[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int jj = 0; jj < 3; jj++)
#pragma unroll
      for (int k = 0; k < 3; k++) {
        const float w = S.w[0][i] * S.w[1][jj] * S.w[2][k];
        const int gx = S.base[0] + i, gy = S.base[1] + jj, gz = S.base[2] + k;
        size_t node;
        if (BLOCK) node = (size_t)block_key(g, sc, gx >> 2, gy >> 2, gz >> 2) * 64 + (((gx & 3) << 4) | ((gy & 3) << 2) | (gz & 3));
        else node = (size_t)sc * n * n * n + ((size_t)gx * n + gy) * n + gz;
        const float4 gv = vgrid[node];
        vn[0] += w * gv.x;
        vn[1] += w * gv.y;
        vn[2] += w * gv.z;
      }
  const RigidAdjTerms T = terms[b];
  const float m = mats[rows.mat[j]].mass;
  float r[3], dx[3], dv[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    r[a] = rest[a * (size_t)N + pid];
    dx[a] = x[a] + P.dt * vn[a] - T.c[a];
    dv[a] = vn[a] - T.vcm[a];
  }
  const float xb[3] = {m * (T.a[0] + T.Ab[0] * r[0] + T.Ab[1] * r[1] + T.Ab[2] * r[2] + dv[1] * T.Lb[2] - dv[2] * T.Lb[1]),
                       m * (T.a[1] + T.Ab[3] * r[0] + T.Ab[4] * r[1] + T.Ab[5] * r[2] + dv[2] * T.Lb[0] - dv[0] * T.Lb[2]),
                       m * (T.a[2] + T.Ab[6] * r[0] + T.Ab[7] * r[1] + T.Ab[8] * r[2] + dv[0] * T.Lb[1] - dv[1] * T.Lb[0])};
  const float vb[3] = {m * (T.b[0] + T.Lb[1] * dx[2] - T.Lb[2] * dx[1]),
                       m * (T.b[1] + T.Lb[2] * dx[0] - T.Lb[0] * dx[2]),
                       m * (T.b[2] + T.Lb[0] * dx[1] - T.Lb[1] * dx[0])};
#pragma unroll
  for (int a = 0; a < 3; a++) {
    abar[a * (size_t)N + jn] = xb[a];
    abar[(3 + a) * (size_t)N + jn] = vb[a];
  }
#pragma unroll
  for (int k = 0; k < 18; k++) abar[(6 + k) * (size_t)N + jn] = 0.f;
}

}  // namespace

void rigid_setup(const RigidCtx& R, const StepParams& P, const PState& user, hipStream_t s) {
  const int N = user.N;
  launch_zero(R.rest_acc, (size_t)R.n_bodies * 16 * sizeof(double), s);
  launch_zero(R.status, 64, s);   // (the status slot is 64 bytes; the fill works in 16-byte units)
  launch_zero(R.acc, (size_t)RIGID_SLOTS * R.n_bodies * RIGID_ACC * sizeof(double), s);
  k_rigid_rest_sum<<<nblk(N, 256), 256, 0, s>>>(user, P.mat, R.body_of, P.mats, R.rest_acc);
  k_rigid_rest<<<nblk(N, 256), 256, 0, s>>>(user, P.mat, R.body_of, P.mats, R.rest_acc, R.rest);
  k_rigid_init<<<nblk(R.n_bodies, 64), 64, 0, s>>>(R.n_bodies, R.rest_acc, R.bodies, R.status);
}

void rigid_forward(const RigidCtx& R, const StepParams& P, const RigidRows& rows, double* rec, bool project,
                   hipStream_t s) {
  const int N = rows.st.N;
  k_rigid_sum<<<nblk(N, 256), 256, 0, s>>>(rows, R.n_bodies, R.body_of, P.mats, R.rest, R.acc);
  k_rigid_solve<<<R.n_bodies, 64, 0, s>>>(R.n_bodies, R.bodies, R.acc, rec);
  if (project) k_rigid_project<<<nblk(N, 256), 256, 0, s>>>(rows, R.body_of, R.rest, rec);
}

void rigid_adjoint(const RigidCtx& R, const StepParams& P, const RigidRows& rows, const uint32_t* map,
                   float* abar_next, const double* rec, const float4* vgrid, const FastGeom* g, hipStream_t s) {
  const int N = rows.st.N;
  k_rigid_adj_sum<<<nblk(N, 256), 256, 0, s>>>(rows, R.n_bodies, map, abar_next, R.body_of, R.rest, rec, R.acc);
  k_rigid_adj_solve<<<R.n_bodies, 64, 0, s>>>(R.n_bodies, R.bodies, R.acc, rec, R.adj);
  if (g)
    k_rigid_adj_apply<true><<<nblk(N, 256), 256, 0, s>>>(rows, map, abar_next, R.body_of, P.mats, R.rest, R.adj,
                                                         vgrid, P, *g);
  else
    k_rigid_adj_apply<false><<<nblk(N, 256), 256, 0, s>>>(rows, map, abar_next, R.body_of, P.mats, R.rest, R.adj,
                                                          vgrid, P, FastGeom{});
}

}  // namespace mpm
