// MLS-MPM step kernels for gfx950: the plain one-particle-per-thread path
// (global atomics, dense grid) used for the adjoint and as the reference
// point for the tiled forward path.
//
// Method (FluidLab, section 3.2, MLS-MPM of Hu et al. 2018):
//   P2G   A_p = -dt V_p (4/dx^2) tau_p + m_p C_p
//         m_i += w m_p ;  mv_i += w (m_p v_p + A_p (x_i - x_p))
//   grid  v = mv/m + dt g ; soft cylinder contact (section 5.1) ; slip walls
//   G2P   v' = sum w v_i ; C' = (4/dx^2) sum w v_i (x_i - x_p)^T ; x' = x + dt v'
//         F_tr = (I + dt C') F ; elastic F' = F_tr ; liquid J' = J det(I + dt C') ;
//         sand F' = U exp(P_DP(log s)) V^T.
#include <hip/hip_runtime.h>
#include <math.h>
#include "mpm_internal.h"
#include "mpm_math.h"
#include "mpm_phys.h"

namespace mpm {

// ---------------------------------------------------------------------------
// Manipulator pose: c_{t+1} = c_t + dt u_t ; R_{t+1} = exp(dt [w_t]x) R_t
// ---------------------------------------------------------------------------
// Poses of steps t0 + 1 .. t0 + n of every scene (one workgroup per scene):
// c_{t+1} = c_t + dt u_t and R_{t+1} = E_t R_t with E_t = exp(dt [w_t]x).
// Chunks of POSE_NT steps: every thread forms its step's E_t, then
// inclusive prefix products (later steps on the left) and prefix sums by
// doubling in LDS, applied to the pose carried in from the previous chunk.
constexpr int POSE_NT = 256;
__global__ __launch_bounds__(POSE_NT) void k_pose(int n_scenes, int t0, int n, float dt, const float* __restrict__ act,
                                                  double* __restrict__ pose) {
  __shared__ double sP[2][POSE_NT][12];   // {prefix product (9), prefix sum of dt u (3)}
  __shared__ double s_carry[12];          // pose at the chunk's start: c (3), R (9)
  const int s = blockIdx.x, tid = threadIdx.x;
  if (s >= n_scenes) return;
  if (tid < 12) s_carry[tid] = pose[((size_t)t0 * n_scenes + s) * POSE_DOUBLES + tid];
  for (int ch = 0; ch < n; ch += POSE_NT) {
    const int m = min(POSE_NT, n - ch);
    double v[12];
    if (tid < m) {
      const float* a = act + ((size_t)(t0 + ch + tid) * n_scenes + s) * 6;
      const double th[3] = {dt * (double)a[3], dt * (double)a[4], dt * (double)a[5]};
      rodrigues(th, v);
#pragma unroll
      for (int k = 0; k < 3; k++) v[9 + k] = dt * (double)a[k];
    } else {
#pragma unroll
      for (int k = 0; k < 12; k++) v[k] = (k % 4 == 0 && k < 9) ? 1.0 : 0.0;
    }
    int buf = 0;
#pragma unroll
    for (int k = 0; k < 12; k++) sP[0][tid][k] = v[k];
    __syncthreads();
    for (int off = 1; off < POSE_NT; off <<= 1) {
      if (tid >= off) {
        const double* L = sP[buf][tid - off];
        double w[12];
        matmul(v, L, w);   // (steps tid - 2 off + 1 .. tid) = (later block) (earlier block)
#pragma unroll
        for (int k = 0; k < 3; k++) w[9 + k] = v[9 + k] + L[9 + k];
#pragma unroll
        for (int k = 0; k < 12; k++) v[k] = w[k];
      }
      buf ^= 1;
#pragma unroll
      for (int k = 0; k < 12; k++) sP[buf][tid][k] = v[k];
      __syncthreads();
    }
    if (tid < m) {
      double* Q = pose + ((size_t)(t0 + ch + tid + 1) * n_scenes + s) * POSE_DOUBLES;
#pragma unroll
      for (int k = 0; k < 3; k++) Q[k] = s_carry[k] + v[9 + k];
      matmul(v, s_carry + 3, Q + 3);
    }
    __syncthreads();
    if (tid == m - 1) {
      double c1[3], R1[9];
#pragma unroll
      for (int k = 0; k < 3; k++) c1[k] = s_carry[k] + v[9 + k];
      matmul(v, s_carry + 3, R1);
#pragma unroll
      for (int k = 0; k < 3; k++) s_carry[k] = c1[k];
#pragma unroll
      for (int k = 0; k < 9; k++) s_carry[3 + k] = R1[k];
    }
    __syncthreads();
  }
}

__global__ void k_zero(float4* p, size_t n4) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  size_t st = (size_t)gridDim.x * blockDim.x;
  for (; i < n4; i += st) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// ---------------------------------------------------------------------------
// P2G, one particle per thread, global float atomics into a dense grid
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_p2g_plain(PState st, StepParams P, float4* __restrict__ mmv) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= st.N) return;
  const int N = st.N;
  float x[3] = {st.x[p], st.x[N + p], st.x[2 * N + p]};
  Stencil S;
  if (!stencil_setup(x, P, S)) { atomicOr(P.err, ERR_OUTSIDE); return; }
  const MatDev& M = P.mats[P.mat[p]];
  float v[3] = {st.v[p], st.v[N + p], st.v[2 * N + p]};
  float C[9], F[9];
#pragma unroll
  for (int k = 0; k < 9; k++) C[k] = st.C[k * N + p];
  float tau[9];
  if (M.kind == KIND_LIQUID) {
    stress_liquid(st.J[p], C, M, tau);
  } else {
#pragma unroll
    for (int k = 0; k < 9; k++) F[k] = st.F[k * N + p];
    if (!stress_solid(F, M, tau)) atomicOr(P.err, ERR_SAND_SIGMA);
  }
  float A[9];
  const float sc = -P.dt * M.vol * 4.f * P.inv_dx * P.inv_dx;
#pragma unroll
  for (int k = 0; k < 9; k++) A[k] = sc * tau[k] + M.mass * C[k];
  const float mvp[3] = {M.mass * v[0], M.mass * v[1], M.mass * v[2]};
  const int n = P.n_grid;
  const size_t sbase = (size_t)P.pscene[p] * n * n * n;
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++)
#pragma unroll
      for (int k = 0; k < 3; k++) {
        float w = S.w[0][i] * S.w[1][j] * S.w[2][k];
        float d0 = (i - S.f[0]) * P.dx, d1 = (j - S.f[1]) * P.dx, d2 = (k - S.f[2]) * P.dx;
        size_t node = sbase + ((size_t)(S.base[0] + i) * n + (S.base[1] + j)) * n + (S.base[2] + k);
        float4* g = mmv + node;
        atomicAdd(&g->x, w * (mvp[0] + A[0] * d0 + A[1] * d1 + A[2] * d2));
        atomicAdd(&g->y, w * (mvp[1] + A[3] * d0 + A[4] * d1 + A[5] * d2));
        atomicAdd(&g->z, w * (mvp[2] + A[6] * d0 + A[7] * d1 + A[8] * d2));
        atomicAdd(&g->w, w * M.mass);
      }
}

// ---------------------------------------------------------------------------
// Grid update on the dense grid: normalise, gravity, contact, walls
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_grid_plain(StepParams P, const float4* __restrict__ mmv, float4* __restrict__ vgrid,
                                                    const double* __restrict__ pose_t, const float* __restrict__ act_t) {
  const int n = P.n_grid;
  const size_t nn = (size_t)n * n * n;
  size_t node = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (node >= nn * P.n_scenes) return;
  float4 g = mmv[node];
  if (!(g.w > 0.f)) { vgrid[node] = make_float4(0.f, 0.f, 0.f, 0.f); return; }
  int s = (int)(node / nn);
  size_t loc = node - (size_t)s * nn;
  int idx[3] = {(int)(loc / ((size_t)n * n)), (int)((loc / n) % n), (int)(loc % n)};
  float vg[3];
  grid_node_forward(P, s, idx, g, pose_t, act_t, vg, nullptr);
  vgrid[node] = make_float4(vg[0], vg[1], vg[2], g.w);
}

// ---------------------------------------------------------------------------
// G2P, one particle per thread
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_g2p_plain(PState in, PState out, StepParams P, const float4* __restrict__ vgrid) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= in.N) return;
  const int N = in.N;
  float x[3] = {in.x[p], in.x[N + p], in.x[2 * N + p]};
  Stencil S;
  if (!stencil_setup(x, P, S)) { atomicOr(P.err, ERR_OUTSIDE); return; }
  const int n = P.n_grid;
  const size_t sbase = (size_t)P.pscene[p] * n * n * n;
  float vn[3] = {0, 0, 0}, B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++)
#pragma unroll
      for (int k = 0; k < 3; k++) {
        float w = S.w[0][i] * S.w[1][j] * S.w[2][k];
        float d[3] = {(i - S.f[0]) * P.dx, (j - S.f[1]) * P.dx, (k - S.f[2]) * P.dx};
        size_t node = sbase + ((size_t)(S.base[0] + i) * n + (S.base[1] + j)) * n + (S.base[2] + k);
        float4 g = vgrid[node];
        float gv[3] = {g.x, g.y, g.z};
#pragma unroll
        for (int a = 0; a < 3; a++) {
          vn[a] += w * gv[a];
#pragma unroll
          for (int b = 0; b < 3; b++) B[a * 3 + b] += w * gv[a] * d[b];
        }
      }
  const MatDev& M = P.mats[P.mat[p]];
  ParticleUpdate U;
  particle_update(x, vn, B, M, P, in, p, U);
  if (!U.ok_sigma) atomicOr(P.err, ERR_SAND_SIGMA);
  if (!U.finite) atomicOr(P.err, ERR_NONFINITE);
#pragma unroll
  for (int a = 0; a < 3; a++) { out.x[a * N + p] = U.x[a]; out.v[a * N + p] = vn[a]; }
#pragma unroll
  for (int k = 0; k < 9; k++) out.C[k * N + p] = U.C[k];
  if (M.kind == KIND_LIQUID) {
    out.J[p] = U.J;
    if (out.F != in.F) {
#pragma unroll
      for (int k = 0; k < 9; k++) out.F[k * N + p] = in.F[k * N + p];
    }
  } else {
#pragma unroll
    for (int k = 0; k < 9; k++) out.F[k * N + p] = U.F[k];
    if (out.J != in.J) out.J[p] = in.J[p];
  }
}

// ---------------------------------------------------------------------------
// Adjoint of G2P: scatter vbar_i to the grid, partial xbar, Fbar, Jbar.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_g2p_adj_plain(PState st, PState bn, PState bo, StepParams P,
                                                       const float4* __restrict__ vgrid, float4* __restrict__ vbar) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= st.N) return;
  const int N = st.N;
  float x[3] = {st.x[p], st.x[N + p], st.x[2 * N + p]};
  Stencil S;
  if (!stencil_setup(x, P, S)) { atomicOr(P.err, ERR_OUTSIDE); return; }
  const int n = P.n_grid;
  const size_t sbase = (size_t)P.pscene[p] * n * n * n;
  // forward gather (recompute)
  float vn[3] = {0, 0, 0}, B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++)
#pragma unroll
      for (int k = 0; k < 3; k++) {
        float w = S.w[0][i] * S.w[1][j] * S.w[2][k];
        float d[3] = {(i - S.f[0]) * P.dx, (j - S.f[1]) * P.dx, (k - S.f[2]) * P.dx};
        size_t node = sbase + ((size_t)(S.base[0] + i) * n + (S.base[1] + j)) * n + (S.base[2] + k);
        float4 g = vgrid[node];
        float gv[3] = {g.x, g.y, g.z};
#pragma unroll
        for (int a = 0; a < 3; a++) {
          vn[a] += w * gv[a];
#pragma unroll
          for (int b = 0; b < 3; b++) B[a * 3 + b] += w * gv[a] * d[b];
        }
      }
  const MatDev& M = P.mats[P.mat[p]];
  // adjoint of the particle update -> vbar' (total), Bbar, xbar (direct), F/J bar
  float xb[3], vb[3], Cb[9], Fb[9], Jb;
#pragma unroll
  for (int a = 0; a < 3; a++) { xb[a] = bn.x[a * N + p]; vb[a] = bn.v[a * N + p]; }
#pragma unroll
  for (int k = 0; k < 9; k++) { Cb[k] = bn.C[k * N + p]; Fb[k] = bn.F[k * N + p]; }
  Jb = bn.J[p];
  float vbt[3], Bb[9], Fbo[9], Jbo;
  particle_update_adjoint(x, vn, B, M, P, st, p, xb, vb, Cb, Fb, Jb, vbt, Bb, Fbo, Jbo);
  // scatter to grid and weight/position gradients
  float xo[3] = {xb[0], xb[1], xb[2]};
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++)
#pragma unroll
      for (int k = 0; k < 3; k++) {
        float w = S.w[0][i] * S.w[1][j] * S.w[2][k];
        float d[3] = {(i - S.f[0]) * P.dx, (j - S.f[1]) * P.dx, (k - S.f[2]) * P.dx};
        size_t node = sbase + ((size_t)(S.base[0] + i) * n + (S.base[1] + j)) * n + (S.base[2] + k);
        float4 g = vgrid[node];
        float gv[3] = {g.x, g.y, g.z};
        float Bd[3], BTv[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
          Bd[a] = Bb[a * 3] * d[0] + Bb[a * 3 + 1] * d[1] + Bb[a * 3 + 2] * d[2];
          BTv[a] = Bb[a] * gv[0] + Bb[3 + a] * gv[1] + Bb[6 + a] * gv[2];
        }
        float4* gb = vbar + node;
        atomicAdd(&gb->x, w * (vbt[0] + Bd[0]));
        atomicAdd(&gb->y, w * (vbt[1] + Bd[1]));
        atomicAdd(&gb->z, w * (vbt[2] + Bd[2]));
        float Wb = gv[0] * (vbt[0] + Bd[0]) + gv[1] * (vbt[1] + Bd[1]) + gv[2] * (vbt[2] + Bd[2]);
        float gw[3];
        S.grad_w(i, j, k, P.inv_dx, gw);
#pragma unroll
        for (int a = 0; a < 3; a++) xo[a] += Wb * gw[a] - w * BTv[a];
      }
#pragma unroll
  for (int a = 0; a < 3; a++) { bo.x[a * N + p] = xo[a]; bo.v[a * N + p] = 0.f; }
#pragma unroll
  for (int k = 0; k < 9; k++) { bo.C[k * N + p] = 0.f; bo.F[k * N + p] = Fbo[k]; }
  bo.J[p] = Jbo;
}

// ---------------------------------------------------------------------------
// Adjoint of the grid update: (m, mv)bar per node, action / pose partials
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_grid_adj_plain(StepParams P, const float4* __restrict__ mmv,
                                                        const float4* __restrict__ vbar, float4* __restrict__ mmv_bar,
                                                        const double* __restrict__ pose_t, const float* __restrict__ act_t,
                                                        double* __restrict__ acc_t) {
  const int n = P.n_grid;
  const size_t nn = (size_t)n * n * n;
  size_t node = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  bool valid = node < nn * P.n_scenes;
  float loc_acc[ACC_DOUBLES];
#pragma unroll
  for (int q = 0; q < ACC_DOUBLES; q++) loc_acc[q] = 0.f;
  int s = 0;
  if (valid) {
    float4 g = mmv[node];
    s = (int)(node / nn);
    if (g.w > 0.f) {
      size_t loc = node - (size_t)s * nn;
      int idx[3] = {(int)(loc / ((size_t)n * n)), (int)((loc / n) % n), (int)(loc % n)};
      float4 vb4 = vbar[node];
      float vb[3] = {vb4.x, vb4.y, vb4.z};
      float mb, mvb[3];
      grid_node_adjoint(P, s, idx, g, pose_t, act_t, vb, mb, mvb, loc_acc);
      mmv_bar[node] = make_float4(mvb[0], mvb[1], mvb[2], mb);
    } else {
      mmv_bar[node] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  // one scene per wave is not guaranteed: reduce per lane group of equal scene
  // by plain double atomics on the lanes that hold a contribution
  bool any = false;
#pragma unroll
  for (int q = 0; q < ACC_DOUBLES; q++) any |= (loc_acc[q] != 0.f);
  if (any) {
    double* dst = acc_t + (size_t)s * ACC_DOUBLES;
#pragma unroll
    for (int q = 0; q < ACC_DOUBLES; q++)
      if (loc_acc[q] != 0.f) atomicAdd(dst + q, (double)loc_acc[q]);
  }
}

// ---------------------------------------------------------------------------
// Adjoint of P2G: gather (m, mv)bar -> vbar, Cbar, xbar, taubar -> F/J/C bar
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_p2g_adj_plain(PState st, PState bo, StepParams P, const float4* __restrict__ mmvb) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= st.N) return;
  const int N = st.N;
  float x[3] = {st.x[p], st.x[N + p], st.x[2 * N + p]};
  Stencil S;
  if (!stencil_setup(x, P, S)) { atomicOr(P.err, ERR_OUTSIDE); return; }
  const MatDev& M = P.mats[P.mat[p]];
  float v[3] = {st.v[p], st.v[N + p], st.v[2 * N + p]};
  float C[9], F[9];
#pragma unroll
  for (int k = 0; k < 9; k++) C[k] = st.C[k * N + p];
  float tau[9];
  float Jv = st.J[p];
  if (M.kind == KIND_LIQUID) {
    stress_liquid(Jv, C, M, tau);
  } else {
#pragma unroll
    for (int k = 0; k < 9; k++) F[k] = st.F[k * N + p];
    stress_solid(F, M, tau);
  }
  float A[9];
  const float sc = -P.dt * M.vol * 4.f * P.inv_dx * P.inv_dx;
#pragma unroll
  for (int k = 0; k < 9; k++) A[k] = sc * tau[k] + M.mass * C[k];
  const float mvp[3] = {M.mass * v[0], M.mass * v[1], M.mass * v[2]};
  const int n = P.n_grid;
  const size_t sbase = (size_t)P.pscene[p] * n * n * n;
  float vb[3] = {0, 0, 0}, Ab[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, xb[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++)
#pragma unroll
      for (int k = 0; k < 3; k++) {
        float w = S.w[0][i] * S.w[1][j] * S.w[2][k];
        float d[3] = {(i - S.f[0]) * P.dx, (j - S.f[1]) * P.dx, (k - S.f[2]) * P.dx};
        size_t node = sbase + ((size_t)(S.base[0] + i) * n + (S.base[1] + j)) * n + (S.base[2] + k);
        float4 gb4 = mmvb[node];
        float gb[3] = {gb4.x, gb4.y, gb4.z};
        float mom[3];
#pragma unroll
        for (int a = 0; a < 3; a++) mom[a] = mvp[a] + A[a * 3] * d[0] + A[a * 3 + 1] * d[1] + A[a * 3 + 2] * d[2];
        float Wb = gb4.w * M.mass + gb[0] * mom[0] + gb[1] * mom[1] + gb[2] * mom[2];
        float gw[3];
        S.grad_w(i, j, k, P.inv_dx, gw);
#pragma unroll
        for (int a = 0; a < 3; a++) {
          vb[a] += w * M.mass * gb[a];
#pragma unroll
          for (int b = 0; b < 3; b++) Ab[a * 3 + b] += w * gb[a] * d[b];
          float ATg = A[a] * gb[0] + A[3 + a] * gb[1] + A[6 + a] * gb[2];
          xb[a] += Wb * gw[a] - w * ATg;
        }
      }
  float taub[9];
#pragma unroll
  for (int k = 0; k < 9; k++) taub[k] = sc * Ab[k];
  float Cb[9];
#pragma unroll
  for (int k = 0; k < 9; k++) Cb[k] = M.mass * Ab[k];
  float Fb[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  float Jb = 0.f;
  if (M.kind == KIND_LIQUID) {
    stress_liquid_adjoint(Jv, C, M, taub, Jb, Cb);
  } else {
    stress_solid_adjoint(F, M, taub, Fb);
  }
#pragma unroll
  for (int a = 0; a < 3; a++) { bo.x[a * N + p] += xb[a]; bo.v[a * N + p] += vb[a]; }
#pragma unroll
  for (int k = 0; k < 9; k++) { bo.C[k * N + p] += Cb[k]; bo.F[k * N + p] += Fb[k]; }
  bo.J[p] += Jb;
}

// ---------------------------------------------------------------------------
// Pose adjoint: backpropagate the per-step local partials through
// c_{t+1} = c_t + dt u_t and R_{t+1} = exp(dt [w_t]x) R_t.
// ---------------------------------------------------------------------------
// One workgroup per scene, in chunks of PADJ_NT steps from the last: the
// step rotations E_t are formed in parallel, one thread then runs the
// recursion of the pose adjoints (Rbar_t = E_t^T Rbar_{t+1} + abar e_y^T,
// cbar_t = cbar_{t+1} + local), keeping the values that enter every step,
// and the action adjoints of all steps are formed in parallel from them.
constexpr int PADJ_NT = 128;
__global__ __launch_bounds__(PADJ_NT) void k_pose_adj(int n_scenes, int T, float dt, const float* __restrict__ act,
                                                      const double* __restrict__ pose, const double* __restrict__ acc,
                                                      float* __restrict__ grad_act) {
  __shared__ double sE[PADJ_NT][9], sRb[PADJ_NT][9], scb[PADJ_NT][3], sA[PADJ_NT][6];
  __shared__ double s_Rb[9], s_cb[3];   // the adjoints entering the chunk's last step
  const int s = blockIdx.x, tid = threadIdx.x;
  if (s >= n_scenes) return;
  if (tid < 9) s_Rb[tid] = 0.0;
  if (tid < 3) s_cb[tid] = 0.0;
  for (int hi = T; hi > 0; hi -= PADJ_NT) {
    const int lo = hi > PADJ_NT ? hi - PADJ_NT : 0, m = hi - lo;
    if (tid < m) {
      const int t = lo + tid;
      const float* a = act + ((size_t)t * n_scenes + s) * 6;
      const double th[3] = {dt * (double)a[3], dt * (double)a[4], dt * (double)a[5]};
      rodrigues(th, sE[tid]);
      const double* A = acc + ((size_t)t * n_scenes + s) * ACC_DOUBLES;
      for (int k = 0; k < 6; k++) sA[tid][k] = A[6 + k];
    }
    __syncthreads();
    if (tid == 0) {
      double Rb[9], cb[3];
      for (int k = 0; k < 9; k++) Rb[k] = s_Rb[k];
      for (int k = 0; k < 3; k++) cb[k] = s_cb[k];
      for (int i = m - 1; i >= 0; i--) {
        for (int k = 0; k < 9; k++) sRb[i][k] = Rb[k];
        for (int k = 0; k < 3; k++) { scb[i][k] = cb[k]; cb[k] += sA[i][k]; }
        double Rn[9];
        matmul_tn(sE[i], Rb, Rn);
        for (int k = 0; k < 9; k++) Rb[k] = Rn[k];
        for (int k = 0; k < 3; k++) Rb[k * 3 + 1] += sA[i][3 + k];
      }
      for (int k = 0; k < 9; k++) s_Rb[k] = Rb[k];
      for (int k = 0; k < 3; k++) s_cb[k] = cb[k];
    }
    __syncthreads();
    if (tid < m) {
      const int t = lo + tid;
      const float* a = act + ((size_t)t * n_scenes + s) * 6;
      const double th[3] = {dt * (double)a[3], dt * (double)a[4], dt * (double)a[5]};
      const double* A = acc + ((size_t)t * n_scenes + s) * ACC_DOUBLES;
      const double* Rt = pose + ((size_t)t * n_scenes + s) * POSE_DOUBLES + 3;
      // Ebar = Rbar_{t+1} R_t^T ; m = vee(Ebar E^T) ; thbar = J_l(th)^T m
      double Eb[9], T1[9];
      matmul_nt(sRb[tid], Rt, Eb);
      matmul_nt(Eb, sE[tid], T1);
      const double mv[3] = {T1[7] - T1[5], T1[2] - T1[6], T1[3] - T1[1]};
      double thb[3];
      left_jacobian_T(th, mv, thb);
      float* g = grad_act + ((size_t)t * n_scenes + s) * 6;
      for (int k = 0; k < 3; k++) g[k] = (float)(A[k] + dt * scb[tid][k]);
      for (int k = 0; k < 3; k++) g[3 + k] = (float)(A[3 + k] + dt * thb[k]);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Blob loss over liquid particles
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_loss_sum(StepParams P, PState st, float mx, float my, float mz, double* scratch) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  double sq = 0.0, cnt = 0.0;
  if (p < st.N && P.mats[P.mat[p]].kind == KIND_LIQUID) {
    const int N = st.N;
    double d0 = st.x[p] - mx, d1 = st.x[N + p] - my, d2 = st.x[2 * N + p] - mz;
    sq = d0 * d0 + d1 * d1 + d2 * d2;
    cnt = 1.0;
  }
  for (int off = 32; off > 0; off >>= 1) {
    sq += __shfl_xor(sq, off);
    cnt += __shfl_xor(cnt, off);
  }
  // one FP64 atomic pair per wavefront, into one of LOSS_SLOTS copies (by
  // wavefront index) so that the atomics do not queue on one address
  if ((threadIdx.x & 63) == 0 && cnt > 0) {
    const int w = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6) % LOSS_SLOTS;
    atomicAdd(scratch + 2 + 2 * w, sq);
    atomicAdd(scratch + 3 + 2 * w, cnt);
  }
}

// sums the copies into scratch[0] (squared distances) and scratch[1] (count)
__global__ __launch_bounds__(64) void k_loss_final(double* scratch, float sigma, float* loss) {
  double sq = 0.0, cnt = 0.0;
  for (int w = threadIdx.x; w < LOSS_SLOTS; w += 64) { sq += scratch[2 + 2 * w]; cnt += scratch[3 + 2 * w]; }
  for (int off = 32; off > 0; off >>= 1) {
    sq += __shfl_xor(sq, off);
    cnt += __shfl_xor(cnt, off);
  }
  if (threadIdx.x == 0) {
    scratch[0] = sq;
    scratch[1] = cnt;
    loss[0] = (float)((cnt > 0 ? sq / cnt : 0.0) + 3.0 * (double)sigma * sigma);
  }
}

__global__ __launch_bounds__(256) void k_loss_grad(StepParams P, PState st, float mx, float my, float mz,
                                                   const double* scratch, float* gx) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= st.N) return;
  const int N = st.N;
  double cnt = scratch[1];
  bool liq = P.mats[P.mat[p]].kind == KIND_LIQUID && cnt > 0;
  float sc = liq ? (float)(2.0 / cnt) : 0.f;
  gx[p] = sc * (st.x[p] - mx);
  gx[N + p] = sc * (st.x[N + p] - my);
  gx[2 * N + p] = sc * (st.x[2 * N + p] - mz);
}

__global__ void k_copy_state(PState a, PState b) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= a.N) return;
  const int N = a.N;
  for (int k = 0; k < 3; k++) { b.x[k * N + p] = a.x[k * N + p]; b.v[k * N + p] = a.v[k * N + p]; }
  for (int k = 0; k < 9; k++) { b.C[k * N + p] = a.C[k * N + p]; b.F[k * N + p] = a.F[k * N + p]; }
  b.J[p] = a.J[p];
}

__global__ void k_scene_index(const int64_t* offs, int n_scenes, int N, int* pscene) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  int lo = 0, hi = n_scenes - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= p) lo = mid; else hi = mid - 1;
  }
  pscene[p] = lo;
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
static inline unsigned blocks_for(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

void launch_pose(int n_scenes, int t0, int n, float dt, const float* act, double* pose, hipStream_t s) {
  if (n > 0) k_pose<<<n_scenes, POSE_NT, 0, s>>>(n_scenes, t0, n, dt, act, pose);
}
void launch_zero(void* p, size_t bytes, hipStream_t s) {
  size_t n4 = bytes / 16;
  unsigned nb = (unsigned)(n4 / 256 + 1);
  if (nb > 8192) nb = 8192;
  k_zero<<<nb, 256, 0, s>>>((float4*)p, n4);
}
void launch_p2g_plain(const PState& st, const StepParams& P, float4* mmv, hipStream_t s) {
  k_p2g_plain<<<blocks_for(st.N, 256), 256, 0, s>>>(st, P, mmv);
}
void launch_grid_plain(const StepParams& P, const float4* mmv, float4* vgrid, const double* pose_t, const float* act_t,
                       hipStream_t s) {
  size_t nodes = (size_t)P.n_grid * P.n_grid * P.n_grid * P.n_scenes;
  k_grid_plain<<<blocks_for(nodes, 256), 256, 0, s>>>(P, mmv, vgrid, pose_t, act_t);
}
void launch_g2p_plain(const PState& in, const PState& out, const StepParams& P, const float4* vgrid, hipStream_t s) {
  k_g2p_plain<<<blocks_for(in.N, 256), 256, 0, s>>>(in, out, P, vgrid);
}
void launch_g2p_adj_plain(const PState& st, const PState& bar_next, const PState& bar, const StepParams& P,
                          const float4* vgrid, float4* vbar_grid, hipStream_t s) {
  k_g2p_adj_plain<<<blocks_for(st.N, 256), 256, 0, s>>>(st, bar_next, bar, P, vgrid, vbar_grid);
}
void launch_grid_adj_plain(const StepParams& P, const float4* mmv, const float4* vbar_grid, float4* mmv_bar,
                           const double* pose_t, const float* act_t, double* acc_t, hipStream_t s) {
  size_t nodes = (size_t)P.n_grid * P.n_grid * P.n_grid * P.n_scenes;
  k_grid_adj_plain<<<blocks_for(nodes, 256), 256, 0, s>>>(P, mmv, vbar_grid, mmv_bar, pose_t, act_t, acc_t);
}
void launch_p2g_adj_plain(const PState& st, const PState& bar, const StepParams& P, const float4* mmv_bar, hipStream_t s) {
  k_p2g_adj_plain<<<blocks_for(st.N, 256), 256, 0, s>>>(st, bar, P, mmv_bar);
}
void launch_pose_adj(int n_scenes, int T, float dt, const float* act, const double* pose, const double* acc,
                     float* grad_act, hipStream_t s) {
  if (T > 0) k_pose_adj<<<n_scenes, PADJ_NT, 0, s>>>(n_scenes, T, dt, act, pose, acc, grad_act);
}
void launch_loss_blob(const StepParams& P, const PState& st, float mx, float my, float mz, float sigma,
                      double* scratch, float* loss, float* gx, hipStream_t s) {
  k_loss_sum<<<blocks_for(st.N, 256), 256, 0, s>>>(P, st, mx, my, mz, scratch);
  k_loss_final<<<1, 64, 0, s>>>(scratch, sigma, loss);
  if (gx) k_loss_grad<<<blocks_for(st.N, 256), 256, 0, s>>>(P, st, mx, my, mz, scratch, gx);
}
void launch_copy_state(const PState& src, const PState& dst, hipStream_t s) {
  k_copy_state<<<blocks_for(src.N, 256), 256, 0, s>>>(src, dst);
}
void launch_scene_index(const int64_t* offs_dev, int n_scenes, int N, int* pscene, hipStream_t s) {
  k_scene_index<<<blocks_for(N, 256), 256, 0, s>>>(offs_dev, n_scenes, N, pscene);
}

}  // namespace mpm
