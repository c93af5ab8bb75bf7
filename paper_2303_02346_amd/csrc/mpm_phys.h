// Per-particle and per-node physics of the MLS-MPM step and their adjoints,
// shared by the plain and the tiled kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include "mpm_internal.h"
#include "mpm_math.h"

namespace mpm {

// ---------------------------------------------------------------------------
// Quadratic B-spline stencil: base = floor(x/dx - 1/2), f = x/dx - base,
// w0 = (3/2 - f)^2/2, w1 = 3/4 - (f - 1)^2, w2 = (f - 1/2)^2/2.
// ---------------------------------------------------------------------------
struct Stencil {
  int base[3];
  float f[3];
  float w[3][3];   // [axis][node]
  float dw[3][3];  // d w / d f
  MPM_DI void grad_w(int i, int j, int k, float inv_dx, float* g) const {
    g[0] = dw[0][i] * w[1][j] * w[2][k] * inv_dx;
    g[1] = w[0][i] * dw[1][j] * w[2][k] * inv_dx;
    g[2] = w[0][i] * w[1][j] * dw[2][k] * inv_dx;
  }
};

MPM_DI bool stencil_setup(const float* x, const StepParams& P, Stencil& S) {
  bool ok = true;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    float X = x[a] * P.inv_dx;
    if (!(X >= 0.5f && X < (float)(P.n_grid - 2) + 0.5f)) ok = false;   // also rejects NaN
    float b = floorf(X - 0.5f);
    S.base[a] = (int)b;
    float f = X - b;
    S.f[a] = f;
    S.w[a][0] = 0.5f * (1.5f - f) * (1.5f - f);
    S.w[a][1] = 0.75f - (f - 1.f) * (f - 1.f);
    S.w[a][2] = 0.5f * (f - 0.5f) * (f - 0.5f);
    S.dw[a][0] = f - 1.5f;
    S.dw[a][1] = -2.f * (f - 1.f);
    S.dw[a][2] = f - 0.5f;
  }
  if (ok) {
#pragma unroll
    for (int a = 0; a < 3; a++) ok = ok && S.base[a] >= 0 && S.base[a] + 2 <= P.n_grid - 1;
  }
  return ok;
}

// ---------------------------------------------------------------------------
// Constitutive models (Kirchhoff stress tau = P F^T)
// ---------------------------------------------------------------------------
// Liquid: tau = lam J (J - 1) I + eta J (C + C^T)
MPM_DI void stress_liquid(float J, const float* C, const MatDev& M, float* tau) {
  float pr = M.lam * J * (J - 1.f);
  float e = M.eta * J;
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) tau[a * 3 + b] = e * (C[a * 3 + b] + C[b * 3 + a]) + (a == b ? pr : 0.f);
}

MPM_DI void stress_liquid_adjoint(float J, const float* C, const MatDev& M, const float* taub, float& Jb, float* Cb) {
  float tr = taub[0] + taub[4] + taub[8];
  float cc = 0.f;
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) cc += taub[a * 3 + b] * (C[a * 3 + b] + C[b * 3 + a]);
  Jb += M.lam * (2.f * J - 1.f) * tr + M.eta * cc;
  float e = M.eta * J;
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) Cb[a * 3 + b] += e * (taub[a * 3 + b] + taub[b * 3 + a]);
}

// Solids, FP64 inside: fixed corotated tau = 2 mu (F - R) F^T + lam J (J-1) I
// with R = U V^T; Hencky tau = U diag(2 mu eps + lam tr eps) U^T, eps = log s.
// Returns false when a sand singular value is not positive.
// Solids with the corotated stress (elastic, Box-yield plastic and the
// particles of rigid bodies); the other solids (sand, von Mises) use Hencky.
MPM_DI bool corotated_kind(int kind) { return kind == KIND_ELASTIC || kind == KIND_BOX || kind == KIND_RIGID; }
// Solids whose G2P update is the plain elastic F' = (I + dt C') F (a rigid
// body's particles too: the rigid projection that follows replaces F).
MPM_DI bool elastic_update_kind(int kind) { return kind == KIND_ELASTIC || kind == KIND_RIGID; }

// Hencky Kirchhoff stress U diag(2 mu eps + lam tr eps) U^T.
template <typename T> MPM_DI void hencky_tau(const T* U, const T* e, const MatDev& M, float* tau) {
  const T tr = e[0] + e[1] + e[2];
  T h[3];
#pragma unroll
  for (int a = 0; a < 3; a++) h[a] = T(2) * (T)M.mu * e[a] + (T)M.lam * tr;
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++)
      tau[i * 3 + j] = (float)(U[i * 3] * h[0] * U[j * 3] + U[i * 3 + 1] * h[1] * U[j * 3 + 1] + U[i * 3 + 2] * h[2] * U[j * 3 + 2]);
}

// The stress from a given signed SVD F = U diag(s) V^T of the copy F (in the
// precision T of the SVD).
template <typename T>
MPM_DI bool stress_solid_usv(const T* F, const T* U, const T* s, const T* V, const MatDev& M, float* tau) {
  if (corotated_kind(M.kind)) {
    T R[9], D[9], Tm[9];
    matmul_nt(U, V, R);
#pragma unroll
    for (int k = 0; k < 9; k++) D[k] = F[k] - R[k];
    matmul_nt(D, F, Tm);
    const T J = s[0] * s[1] * s[2];
    const T pr = (T)M.lam * J * (J - T(1));
    const T m2 = T(2) * (T)M.mu;
#pragma unroll
    for (int k = 0; k < 9; k++) tau[k] = (float)(m2 * Tm[k] + ((k % 4 == 0) ? pr : T(0)));
    return true;
  }
  const bool ok = s[2] > T(0);
  T e[3];
#pragma unroll
  for (int a = 0; a < 3; a++) e[a] = ok ? t_log(s[a]) : T(0);
  hencky_tau(U, e, M, tau);
  return ok;
}

MPM_DI bool stress_solid(const float* Ff, const MatDev& M, float* tau) {
  double F[9], U[9], s[3], V[9];
#pragma unroll
  for (int k = 0; k < 9; k++) F[k] = (double)Ff[k];
  svd3(F, U, s, V);
  return stress_solid_usv(F, U, s, V, M, tau);
}

// The solid stress with an FP32 SVD, redone in FP64 when F is
// ill-conditioned (s2 < s0/4) or the FP32 sweeps do not converge.
// Returns false when a Hencky solid has a singular value that is not positive.
MPM_DI bool stress_solid_fast(const float* Ff, const MatDev& M, float* tau) {
  float U[9], s[3], V[9];
  const bool conv = svd3(Ff, U, s, V);
  if (!conv || !(s[2] > 0.25f * s[0])) return stress_solid(Ff, M, tau);
  if (corotated_kind(M.kind)) {
    float R[9], D[9], T[9];
    matmul_nt(U, V, R);
#pragma unroll
    for (int k = 0; k < 9; k++) D[k] = Ff[k] - R[k];
    matmul_nt(D, Ff, T);
    const float J = s[0] * s[1] * s[2];
    const float pr = M.lam * J * (J - 1.f), m2 = 2.f * M.mu;
#pragma unroll
    for (int k = 0; k < 9; k++) tau[k] = m2 * T[k] + ((k % 4 == 0) ? pr : 0.f);
    return true;
  }
  float e[3];
#pragma unroll
  for (int a = 0; a < 3; a++) e[a] = logf(s[a]);
  hencky_tau(U, e, M, tau);
  return true;
}

// Adjoint of the solid stress, from a given signed SVD of the copy F (in the
// precision T of the SVD).
template <typename T>
MPM_DI void stress_solid_adjoint_usv(const T* F, const T* U, const T* s, const T* V, const MatDev& M,
                                     const float* taubf, float* Fbf) {
  T tb[9];
#pragma unroll
  for (int k = 0; k < 9; k++) tb[k] = (T)taubf[k];
  T Fb[9];
  if (corotated_kind(M.kind)) {
    T R[9], D[9], T1[9], T2[9], Rb[9];
    matmul_nt(U, V, R);
#pragma unroll
    for (int k = 0; k < 9; k++) D[k] = F[k] - R[k];
    const T m2 = T(2) * (T)M.mu;
    matmul(tb, F, T1);      // taub F
    matmul_tn(tb, D, T2);   // taub^T (F - R)
#pragma unroll
    for (int k = 0; k < 9; k++) { Fb[k] = m2 * (T1[k] + T2[k]); Rb[k] = -m2 * T1[k]; }
    // polar rotation: g = 1, dg = 0, divided differences 0
    const T g[3] = {T(1), T(1), T(1)};
    const T dg[9] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
    T Fr[9];
    iso_adjoint(U, s, V, g, dg, dg, Rb, Fr);
    const T J = s[0] * s[1] * s[2];
    T K[9];
    cof3(F, K);
    const T jb = (T)M.lam * (T(2) * J - T(1)) * (tb[0] + tb[4] + tb[8]);
#pragma unroll
    for (int k = 0; k < 9; k++) Fb[k] += Fr[k] + jb * K[k];
  } else {
    T e[3], g[3], dg[9], sdd[9];
    const bool ok = s[2] > T(0);
#pragma unroll
    for (int a = 0; a < 3; a++) e[a] = ok ? t_log(s[a]) : T(0);
    const T tr = e[0] + e[1] + e[2];
    const T mu = (T)M.mu, lam = (T)M.lam;
    T h[3], is[3];
#pragma unroll
    for (int a = 0; a < 3; a++) { is[a] = t_div(T(1), s[a]); h[a] = T(2) * mu * e[a] + lam * tr; g[a] = h[a] * is[a]; }
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int k = 0; k < 3; k++)
        dg[i * 3 + k] = (T(2) * mu * T(i == k) + lam) * is[k] * is[i] - (i == k ? h[i] * is[i] * is[i] : T(0));
    // (log s_i - log s_j)/(s_i - s_j) is symmetric: one evaluation per pair
    const T L01 = log_divdiff(s[0], s[1]), L02 = log_divdiff(s[0], s[2]), L12 = log_divdiff(s[1], s[2]);
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int j = 0; j < 3; j++) {
        if (i == j) { sdd[i * 3 + j] = T(0); continue; }
        const T L = (i + j == 1) ? L01 : ((i + j == 2) ? L02 : L12);
        sdd[i * 3 + j] = (T(2) * mu * (s[j] * L - e[j]) - lam * tr) * is[i] * is[j];
      }
    T Pm[9], Pb[9], T1[9], Fr[9];
    usv(U, g, V, Pm);
    matmul(tb, F, Pb);        // Pbar = taub F
    matmul_tn(tb, Pm, T1);    // taub^T P
    iso_adjoint(U, s, V, g, dg, sdd, Pb, Fr);
#pragma unroll
    for (int k = 0; k < 9; k++) Fb[k] = T1[k] + Fr[k];
  }
#pragma unroll
  for (int k = 0; k < 9; k++) Fbf[k] = (float)Fb[k];
}

MPM_DI void stress_solid_adjoint(const float* Ff, const MatDev& M, const float* taubf, float* Fbf) {
  double F[9], U[9], s[3], V[9];
#pragma unroll
  for (int k = 0; k < 9; k++) F[k] = (double)Ff[k];
  svd3(F, U, s, V);
  stress_solid_adjoint_usv(F, U, s, V, M, taubf, Fbf);
}

// ---------------------------------------------------------------------------
// Drucker-Prager return map in log-strain (Klar et al. 2016), FP64.
// case 0 inside, 1 apex, 2 cone.
// ---------------------------------------------------------------------------
// Result of a return map in log strain.  In the flowing case (cse 2) the
// map is eps' = t/3 1 + k0 + beta |dev| nh - k1 t nh with nh = dev/|dev|, so
// its Jacobian is 11^T/3 - k1 nh 1^T + beta (I - nh nh^T - 11^T/3) and
// eps'_i - eps'_j = beta (eps_i - eps_j).
template <typename T> struct DPInfoT {
  int cse;            // 0 inside, 1 apex (Drucker-Prager only), 2 flowing
  T t, ndev, beta, k1;
  T nh[3];
};
using DPInfo = DPInfoT<double>;

template <typename T> MPM_DI void dp_project(const T* e, const MatDev& M, T* ep, DPInfoT<T>& I) {
  T c = M.coh;
  T es[3] = {e[0] - c, e[1] - c, e[2] - c};
  T t = es[0] + es[1] + es[2];
  T dev[3] = {es[0] - t / T(3), es[1] - t / T(3), es[2] - t / T(3)};
  T nd = t_sqrt(dev[0] * dev[0] + dev[1] * dev[1] + dev[2] * dev[2]);
  T ka = (T)M.kappa * (T)M.alpha;
  T dg = nd + ka * t;
  I.t = t; I.ndev = nd;
  if (t > T(0)) {
    I.cse = 1; I.beta = T(0);
#pragma unroll
    for (int a = 0; a < 3; a++) { ep[a] = c; I.nh[a] = T(0); }
  } else if (dg <= T(0)) {
    I.cse = 0; I.beta = T(1);
#pragma unroll
    for (int a = 0; a < 3; a++) { ep[a] = e[a]; I.nh[a] = T(0); }
  } else {
    I.cse = 2;
    const T ind = t_div(T(1), nd);
#pragma unroll
    for (int a = 0; a < 3; a++) { I.nh[a] = dev[a] * ind; ep[a] = es[a] - dg * I.nh[a] + c; }
    I.beta = -ka * t * ind;
  }
  I.k1 = ka;
}

// Von Mises return (section 3.2, non-Newtonian liquid): |dev| <= r inside,
// else the deviatoric part is scaled back to radius r, the trace kept.
template <typename T> MPM_DI void vm_project(const T* e, const MatDev& M, T* ep, DPInfoT<T>& I) {
  const T t = e[0] + e[1] + e[2];
  const T dev[3] = {e[0] - t / T(3), e[1] - t / T(3), e[2] - t / T(3)};
  const T nd = t_sqrt(dev[0] * dev[0] + dev[1] * dev[1] + dev[2] * dev[2]);
  const T r = (T)M.yrad;
  I.t = t; I.ndev = nd; I.k1 = T(0);
  if (nd <= r) {
    I.cse = 0; I.beta = T(1);
#pragma unroll
    for (int a = 0; a < 3; a++) { ep[a] = e[a]; I.nh[a] = T(0); }
  } else {
    I.cse = 2;
    const T ind = t_div(T(1), nd);
    I.beta = r * ind;
#pragma unroll
    for (int a = 0; a < 3; a++) { I.nh[a] = dev[a] * ind; ep[a] = t * (T(1) / T(3)) + r * I.nh[a]; }
  }
}

// Box yield (section 3.2's plastic material, Stomakhin et al. 2013): the
// singular values clamped to [box_lo, box_hi]; returns whether any changed.
template <typename T> MPM_DI bool box_clamp(const T* s, const MatDev& M, T* g) {
  bool changed = false;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    g[a] = fmin(fmax(s[a], (T)M.box_lo), (T)M.box_hi);
    changed |= g[a] != s[a];
  }
  return changed;
}

// The return map of a plastic material (sand or von Mises).
template <typename T> MPM_DI void plastic_project(const T* e, const MatDev& M, T* ep, DPInfoT<T>& I) {
  if (M.kind == KIND_VONMISES) vm_project(e, M, ep, I);
  else dp_project(e, M, ep, I);
}

// ---------------------------------------------------------------------------
// G2P update of a plastic solid (sand, von Mises, Box yield) in precision T:
// the trial F_tr = Md F, its signed SVD, the return map, F' and, for the
// Hencky kinds, the Kirchhoff stress of F' from the same SVD.
// ---------------------------------------------------------------------------
enum { PLASTIC_OK = 0, PLASTIC_SIGMA = 1, PLASTIC_RETRY = 2 };

template <typename T> struct PlasticStep {
  T U[9], V[9];     // SVD of F_tr
  T e[3], ep[3];    // trial and returned log singular values (Hencky kinds)
  int cse;          // return-map case (0 inside, 1 apex, 2 flowing)
};

// In FP32 the SVD comes from F_tr^T F_tr, whose rounding costs the smallest
// singular value eps (s0/s2)^2 of relative accuracy; a trial state with
// s2 < s0/4 (relative error above 16 eps) or an unconverged sweep returns
// PLASTIC_RETRY without output so that the caller redoes it in FP64.
// PLASTIC_SIGMA: a singular value is not positive (F' = F_tr, no stress).
template <typename T, bool TAU>
MPM_DI int plastic_step(const float* Md, const float* Fin, const MatDev& M, float* Fo, float* tau, PlasticStep<T>& R) {
  constexpr bool dbl = sizeof(T) == 8;
  T Ft[9], s[3];
  {
    T Mdd[9], Fd[9];
#pragma unroll
    for (int k = 0; k < 9; k++) { Mdd[k] = (T)Md[k]; Fd[k] = (T)Fin[k]; }
    matmul(Mdd, Fd, Ft);
  }
  const bool conv = svd3(Ft, R.U, s, R.V);
  if (!dbl && (!conv || !(s[2] > T(0.25) * s[0]))) return PLASTIC_RETRY;
  R.cse = 0;
  if (!(s[2] > T(0))) {
#pragma unroll
    for (int k = 0; k < 9; k++) Fo[k] = (float)Ft[k];
    return PLASTIC_SIGMA;
  }
  if (M.kind == KIND_BOX) {
    T gg[3], Fn[9];
    const bool clamped = box_clamp(s, M, gg);
    if (clamped) usv(R.U, gg, R.V, Fn);
#pragma unroll
    for (int k = 0; k < 9; k++) Fo[k] = (float)(clamped ? Fn[k] : Ft[k]);
    return PLASTIC_OK;
  }
#pragma unroll
  for (int a = 0; a < 3; a++) R.e[a] = t_log(s[a]);
  DPInfoT<T> I;
  plastic_project(R.e, M, R.ep, I);
  R.cse = I.cse;
  if (I.cse == 0) {
#pragma unroll
    for (int k = 0; k < 9; k++) Fo[k] = (float)Ft[k];
  } else {
    T gg[3], Fn[9];
#pragma unroll
    for (int a = 0; a < 3; a++) gg[a] = t_exp(R.ep[a]);
    usv(R.U, gg, R.V, Fn);
#pragma unroll
    for (int k = 0; k < 9; k++) Fo[k] = (float)Fn[k];
  }
  if (TAU) hencky_tau(R.U, R.ep, M, tau);
  return PLASTIC_OK;
}

// ---------------------------------------------------------------------------
// Particle update after the G2P gather (vn = sum w v_i, B = sum w v_i d^T)
// ---------------------------------------------------------------------------
struct ParticleUpdate {
  float x[3], C[9], F[9], J;
  bool ok_sigma, finite;
};

MPM_DI void particle_update(const float* x, const float* vn, const float* B, const MatDev& M, const StepParams& P,
                            const PState& in, int p, ParticleUpdate& U) {
  const int N = in.N;
  const float d4 = 4.f * P.inv_dx * P.inv_dx;
  U.ok_sigma = true;
#pragma unroll
  for (int k = 0; k < 9; k++) U.C[k] = d4 * B[k];
#pragma unroll
  for (int a = 0; a < 3; a++) U.x[a] = x[a] + P.dt * vn[a];
  bool fin = isfinite(U.x[0]) && isfinite(U.x[1]) && isfinite(U.x[2]) && isfinite(vn[0]) && isfinite(vn[1]) && isfinite(vn[2]);
  float Md[9];
#pragma unroll
  for (int k = 0; k < 9; k++) Md[k] = P.dt * U.C[k] + ((k % 4 == 0) ? 1.f : 0.f);
  if (M.kind == KIND_LIQUID) {
    U.J = in.J[p] * det3(Md);
    fin = fin && isfinite(U.J);
  } else {
    float F[9];
#pragma unroll
    for (int k = 0; k < 9; k++) F[k] = in.F[k * N + p];
    if (elastic_update_kind(M.kind)) {
      matmul(Md, F, U.F);
    } else {
      double Mdd[9], Fd[9], Ft[9], Uu[9], s[3], V[9];
#pragma unroll
      for (int k = 0; k < 9; k++) { Mdd[k] = Md[k]; Fd[k] = F[k]; }
      matmul(Mdd, Fd, Ft);
      svd3(Ft, Uu, s, V);
      if (!(s[2] > 0.0)) {
        U.ok_sigma = false;
#pragma unroll
        for (int k = 0; k < 9; k++) U.F[k] = (float)Ft[k];
      } else if (M.kind == KIND_BOX) {
        double g[3], Fo[9];
        bool clamped = box_clamp(s, M, g);
        if (clamped) usv(Uu, g, V, Fo);
#pragma unroll
        for (int k = 0; k < 9; k++) U.F[k] = (float)(clamped ? Fo[k] : Ft[k]);
      } else {
        double e[3] = {log(s[0]), log(s[1]), log(s[2])}, ep[3], g[3], Fo[9];
        DPInfo I;
        plastic_project(e, M, ep, I);
        if (I.cse == 0) {
#pragma unroll
          for (int k = 0; k < 9; k++) U.F[k] = (float)Ft[k];
        } else {
#pragma unroll
          for (int a = 0; a < 3; a++) g[a] = exp(ep[a]);
          usv(Uu, g, V, Fo);
#pragma unroll
          for (int k = 0; k < 9; k++) U.F[k] = (float)Fo[k];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 9; k++) fin = fin && isfinite(U.F[k]);
  }
#pragma unroll
  for (int k = 0; k < 9; k++) fin = fin && isfinite(U.C[k]);
  U.finite = fin;
}

// Adjoint of the plastic update F' = Phi(F_tr), F_tr = Md F, of a Box-yield,
// sand or von Mises solid: Ftb = dL/dF_tr from Fb = dL/dF', through the
// isotropic-map derivative of the return map, in precision T.  In FP32 an
// ill-conditioned trial state (s2 < s0/4) or an unconverged sweep returns
// false without output, for the caller to redo it in FP64.
template <typename T>
MPM_DI bool plastic_adjoint(const float* Md, const float* F, const MatDev& M, const float* Fb, float* Ftb) {
  constexpr bool dbl = sizeof(T) == 8;
  T Ft[9], Uu[9], s[3], V[9];
  {
    T Mdd[9], Fd[9];
#pragma unroll
    for (int k = 0; k < 9; k++) { Mdd[k] = (T)Md[k]; Fd[k] = (T)F[k]; }
    matmul(Mdd, Fd, Ft);
  }
  const bool conv = svd3(Ft, Uu, s, V);
  if (!dbl && (!conv || !(s[2] > T(0.25) * s[0]))) return false;
  T e[3], ep[3];
  const bool ok = s[2] > T(0);
#pragma unroll
  for (int a = 0; a < 3; a++) e[a] = ok ? t_log(s[a]) : T(0);
  DPInfoT<T> I;
  if (M.kind == KIND_BOX) {
    // clamp: dg = diag(inside), divided differences (g_i - g_j)/(s_i - s_j)
    T g[3], dg[9], sdd[9], Pb[9], Fr[9];
    const bool clamped = ok && box_clamp(s, M, g);
    if (!clamped) {
#pragma unroll
      for (int k = 0; k < 9; k++) Ftb[k] = Fb[k];
    } else {
#pragma unroll
      for (int i = 0; i < 3; i++)
#pragma unroll
        for (int k = 0; k < 3; k++) dg[i * 3 + k] = (i == k && g[i] == s[i]) ? T(1) : T(0);
      const T tiny = dbl ? T(1e-12) : T(1e-6);
#pragma unroll
      for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
          const T d = s[i] - s[j];
          sdd[i * 3 + j] = (i == j) ? T(0) : (t_abs(d) > tiny ? t_div(g[i] - g[j], d) : dg[i * 3 + i]);
        }
#pragma unroll
      for (int k = 0; k < 9; k++) Pb[k] = (T)Fb[k];
      iso_adjoint(Uu, s, V, g, dg, sdd, Pb, Fr);
#pragma unroll
      for (int k = 0; k < 9; k++) Ftb[k] = (float)Fr[k];
    }
    return true;
  }
  plastic_project(e, M, ep, I);
  if (!ok || I.cse == 0) {
#pragma unroll
    for (int k = 0; k < 9; k++) Ftb[k] = Fb[k];
    return true;
  }
  T g[3], dg[9], sdd[9], Pb[9], Fr[9];
#pragma unroll
  for (int a = 0; a < 3; a++) g[a] = t_exp(ep[a]);
  if (I.cse == 1) {
#pragma unroll
    for (int k = 0; k < 9; k++) { dg[k] = T(0); sdd[k] = T(0); }
  } else {
    const T is[3] = {t_div(T(1), s[0]), t_div(T(1), s[1]), t_div(T(1), s[2])};
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int k = 0; k < 3; k++) {
        const T Jik = T(1) / T(3) - I.k1 * I.nh[i] + I.beta * ((i == k ? T(1) : T(0)) - I.nh[i] * I.nh[k] - T(1) / T(3));
        dg[i * 3 + k] = g[i] * Jik * is[k];
      }
    // exp(ep_j - e_j) = g_j / s_j; the ratios of a pair share their expm1s
    T r01, r10, r02, r20, r12, r21;
    expm1_ratio_pair(I.beta, e[0] - e[1], r01, r10);
    expm1_ratio_pair(I.beta, e[0] - e[2], r02, r20);
    expm1_ratio_pair(I.beta, e[1] - e[2], r12, r21);
    const T q[3] = {g[0] * is[0], g[1] * is[1], g[2] * is[2]};
    sdd[0] = sdd[4] = sdd[8] = T(0);
    sdd[1] = q[1] * r01; sdd[3] = q[0] * r10;
    sdd[2] = q[2] * r02; sdd[6] = q[0] * r20;
    sdd[5] = q[2] * r12; sdd[7] = q[1] * r21;
  }
#pragma unroll
  for (int k = 0; k < 9; k++) Pb[k] = (T)Fb[k];
  iso_adjoint(Uu, s, V, g, dg, sdd, Pb, Fr);
#pragma unroll
  for (int k = 0; k < 9; k++) Ftb[k] = (float)Fr[k];
  return true;
}

// Adjoint of particle_update.  Inputs: the output adjoints (xb, vb, Cb, Fb,
// Jb).  Outputs: vbt = adjoint of vn, Bb = adjoint of B, Fbo/Jbo = adjoint of
// the input F/J.  The direct x term (x' = x + ...) is left to the caller.
// PREC selects the precision of the plastic-return adjoint: ADJ_AUTO takes
// the FP32 adjoint and redoes an ill-conditioned one in FP64; ADJ_FP32
// returns false, with nothing written, where the FP32 adjoint is
// ill-conditioned (the caller redoes the particle with ADJ_FP64); ADJ_FP64
// takes the FP64 adjoint.  Returns true otherwise.
enum { ADJ_AUTO = 0, ADJ_FP32 = 1, ADJ_FP64 = 2 };
template <int PREC = ADJ_AUTO>
MPM_DI bool particle_update_adjoint(const float* x, const float* vn, const float* B, const MatDev& M, const StepParams& P,
                                    const PState& in, int p, const float* xb, const float* vb, const float* Cb,
                                    const float* Fb, float Jb, float* vbt, float* Bb, float* Fbo, float& Jbo) {
  const int N = in.N;
  const float d4 = 4.f * P.inv_dx * P.inv_dx;
#pragma unroll
  for (int a = 0; a < 3; a++) vbt[a] = vb[a] + P.dt * xb[a];
  float Cn[9], Md[9], Cbt[9];
#pragma unroll
  for (int k = 0; k < 9; k++) {
    Cn[k] = d4 * B[k];
    Md[k] = P.dt * Cn[k] + ((k % 4 == 0) ? 1.f : 0.f);
    Cbt[k] = Cb[k];
  }
  if (M.kind == KIND_LIQUID) {
    float J = in.J[p];
    float dM = det3(Md);
    Jbo = Jb * dM;
    float K[9];
    cof3(Md, K);
#pragma unroll
    for (int k = 0; k < 9; k++) { Cbt[k] += Jb * J * P.dt * K[k]; Fbo[k] = Fb[k]; }
  } else {
    Jbo = Jb;
    float F[9], Ftb[9];
#pragma unroll
    for (int k = 0; k < 9; k++) F[k] = in.F[k * N + p];
    if (elastic_update_kind(M.kind)) {
#pragma unroll
      for (int k = 0; k < 9; k++) Ftb[k] = Fb[k];
    } else {
      if (PREC == ADJ_FP64) plastic_adjoint<double>(Md, F, M, Fb, Ftb);
      else if (!plastic_adjoint<float>(Md, F, M, Fb, Ftb)) {
        if (PREC == ADJ_FP32) return false;
        plastic_adjoint<double>(Md, F, M, Fb, Ftb);
      }
    }
    // F_tr = Md F : Cbar += dt Ftb F^T ; Fbar = Md^T Ftb
    float T1[9];
    matmul_nt(Ftb, F, T1);
#pragma unroll
    for (int k = 0; k < 9; k++) Cbt[k] += P.dt * T1[k];
    matmul_tn(Md, Ftb, Fbo);
  }
#pragma unroll
  for (int k = 0; k < 9; k++) Bb[k] = d4 * Cbt[k];
  return true;
}

// ---------------------------------------------------------------------------
// Grid node update: v = mv/m + dt g ; soft cylinder contact ; slip walls
// ---------------------------------------------------------------------------
MPM_DI void rodrigues(const double* th, double* E) {
  double t2 = th[0] * th[0] + th[1] * th[1] + th[2] * th[2];
  double t = sqrt(t2);
  double a, b;   // sin t / t, (1 - cos t)/t^2
  if (t < 1e-4) { a = 1.0 - t2 / 6.0 + t2 * t2 / 120.0; b = 0.5 - t2 / 24.0 + t2 * t2 / 720.0; }
  else { a = sin(t) / t; b = (1.0 - cos(t)) / t2; }
  double K[9] = {0, -th[2], th[1], th[2], 0, -th[0], -th[1], th[0], 0};
  double K2[9];
  matmul(K, K, K2);
#pragma unroll
  for (int k = 0; k < 9; k++) E[k] = ((k % 4 == 0) ? 1.0 : 0.0) + a * K[k] + b * K2[k];
}

// out = J_l(th)^T m with J_l = I + (1 - cos t)/t^2 [th]x + (t - sin t)/t^3 [th]x^2
MPM_DI void left_jacobian_T(const double* th, const double* m, double* out) {
  double t2 = th[0] * th[0] + th[1] * th[1] + th[2] * th[2];
  double t = sqrt(t2);
  double a, b;
  if (t < 1e-4) { a = 0.5 - t2 / 24.0 + t2 * t2 / 720.0; b = 1.0 / 6.0 - t2 / 120.0 + t2 * t2 / 5040.0; }
  else { a = (1.0 - cos(t)) / t2; b = (t - sin(t)) / (t2 * t); }
  // [th]x^T = -[th]x ; ([th]x^2)^T = [th]x^2
  double c1[3] = {th[1] * m[2] - th[2] * m[1], th[2] * m[0] - th[0] * m[2], th[0] * m[1] - th[1] * m[0]};  // th x m
  double c2[3] = {th[1] * c1[2] - th[2] * c1[1], th[2] * c1[0] - th[0] * c1[2], th[0] * c1[1] - th[1] * c1[0]};  // th x (th x m)
#pragma unroll
  for (int k = 0; k < 3; k++) out[k] = m[k] - a * c1[k] + b * c2[k];
}

struct ContactGeom {
  float c[3], a[3], ex[3], u[3], w[3], radius;
};

MPM_DI void load_contact(const StepParams& P, int s, const double* pose_t, const float* act_t, ContactGeom& G) {
  const double* Q = pose_t + (size_t)s * POSE_DOUBLES;
  const float* A = act_t + (size_t)s * 6;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    G.c[k] = (float)Q[k];
    G.a[k] = (float)Q[3 + k * 3 + 1];
    G.ex[k] = (float)Q[3 + k * 3 + 0];
    G.u[k] = A[k];
    G.w[k] = A[3 + k];
  }
  G.radius = P.cyl_radius[s];
}

MPM_DI void cross3(const float* a, const float* b, float* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Soft contact of a node velocity v (in/out) at node position xi.
MPM_DI void contact_forward(const StepParams& P, const ContactGeom& G, const float* xi, float* v) {
  float r[3] = {xi[0] - G.c[0], xi[1] - G.c[1], xi[2] - G.c[2]};
  float sa = r[0] * G.a[0] + r[1] * G.a[1] + r[2] * G.a[2];
  float rp[3] = {r[0] - sa * G.a[0], r[1] - sa * G.a[1], r[2] - sa * G.a[2]};
  float dist = sqrtf(rp[0] * rp[0] + rp[1] * rp[1] + rp[2] * rp[2]);
  float d = dist - G.radius;
  if (!(d < P.band * P.dx)) return;
  float nrm[3];
  if (dist > 0.f) { nrm[0] = rp[0] / dist; nrm[1] = rp[1] / dist; nrm[2] = rp[2] / dist; }
  else { nrm[0] = G.ex[0]; nrm[1] = G.ex[1]; nrm[2] = G.ex[2]; }
  float wr[3];
  cross3(G.w, r, wr);
  float vco[3] = {G.u[0] + wr[0], G.u[1] + wr[1], G.u[2] + wr[2]};
  float vrel[3] = {v[0] - vco[0], v[1] - vco[1], v[2] - vco[2]};
  float vn = vrel[0] * nrm[0] + vrel[1] * nrm[1] + vrel[2] * nrm[2];
  float vc[3] = {v[0], v[1], v[2]};
  if (vn < 0.f) {
    float vt[3] = {vrel[0] - vn * nrm[0], vrel[1] - vn * nrm[1], vrel[2] - vn * nrm[2]};
    float tn = sqrtf(vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2]);
    if (tn <= -P.friction * vn) {
      vc[0] = vco[0]; vc[1] = vco[1]; vc[2] = vco[2];
    } else {
      float k = 1.f + P.friction * vn / tn;
#pragma unroll
      for (int q = 0; q < 3; q++) vc[q] = k * vt[q] + vco[q];
    }
  }
  float al = fminf(expf(-d * P.inv_dx), 1.f);
#pragma unroll
  for (int q = 0; q < 3; q++) v[q] = al * vc[q] + (1.f - al) * v[q];
}

// Adjoint of contact_forward.  v0 is the input velocity, ob the adjoint of the
// output; returns v0b and accumulates the collider partials into acc:
// u (0..2), w (3..5), c (6..8), axis a (9..11).
MPM_DI void contact_adjoint(const StepParams& P, const ContactGeom& G, const float* xi, const float* v0, const float* ob,
                            float* v0b, float* acc) {
  float r[3] = {xi[0] - G.c[0], xi[1] - G.c[1], xi[2] - G.c[2]};
  float sa = r[0] * G.a[0] + r[1] * G.a[1] + r[2] * G.a[2];
  float rp[3] = {r[0] - sa * G.a[0], r[1] - sa * G.a[1], r[2] - sa * G.a[2]};
  float dist = sqrtf(rp[0] * rp[0] + rp[1] * rp[1] + rp[2] * rp[2]);
  float d = dist - G.radius;
#pragma unroll
  for (int q = 0; q < 3; q++) v0b[q] = ob[q];
  if (!(d < P.band * P.dx)) return;
  bool on_axis = !(dist > 0.f);
  float nrm[3];
  if (!on_axis) { nrm[0] = rp[0] / dist; nrm[1] = rp[1] / dist; nrm[2] = rp[2] / dist; }
  else { nrm[0] = G.ex[0]; nrm[1] = G.ex[1]; nrm[2] = G.ex[2]; }
  float wr[3];
  cross3(G.w, r, wr);
  float vco[3] = {G.u[0] + wr[0], G.u[1] + wr[1], G.u[2] + wr[2]};
  float vrel[3] = {v0[0] - vco[0], v0[1] - vco[1], v0[2] - vco[2]};
  float vn = vrel[0] * nrm[0] + vrel[1] * nrm[1] + vrel[2] * nrm[2];
  float vc[3] = {v0[0], v0[1], v0[2]};
  float vt[3] = {0, 0, 0}, tn = 0.f, kf = 0.f;
  bool approach = vn < 0.f, stick = false;
  if (approach) {
#pragma unroll
    for (int q = 0; q < 3; q++) vt[q] = vrel[q] - vn * nrm[q];
    tn = sqrtf(vt[0] * vt[0] + vt[1] * vt[1] + vt[2] * vt[2]);
    stick = tn <= -P.friction * vn;
    if (stick) {
#pragma unroll
      for (int q = 0; q < 3; q++) vc[q] = vco[q];
    } else {
      kf = 1.f + P.friction * vn / tn;
#pragma unroll
      for (int q = 0; q < 3; q++) vc[q] = kf * vt[q] + vco[q];
    }
  }
  float ar = expf(-d * P.inv_dx);
  float al = fminf(ar, 1.f);
  // out = al vc + (1 - al) v0
  float vcb[3], alb = 0.f;
#pragma unroll
  for (int q = 0; q < 3; q++) {
    vcb[q] = al * ob[q];
    v0b[q] = (1.f - al) * ob[q];
    alb += ob[q] * (vc[q] - v0[q]);
  }
  float db = (ar < 1.f) ? -alb * ar * P.inv_dx : 0.f;
  float vcob[3] = {0, 0, 0}, nrmb[3] = {0, 0, 0};
  if (approach) {
#pragma unroll
    for (int q = 0; q < 3; q++) vcob[q] = vcb[q];
    if (!stick) {
      float tdot = vt[0] * vcb[0] + vt[1] * vcb[1] + vt[2] * vcb[2];
      float vtb[3];
      float coef = P.friction * vn * tdot / (tn * tn * tn);
#pragma unroll
      for (int q = 0; q < 3; q++) vtb[q] = kf * vcb[q] - coef * vt[q];
      float vnb = P.friction * tdot / tn;
      vnb -= vtb[0] * nrm[0] + vtb[1] * nrm[1] + vtb[2] * nrm[2];
      float vrelb[3];
#pragma unroll
      for (int q = 0; q < 3; q++) {
        nrmb[q] = -vn * vtb[q] + vnb * vrel[q];
        vrelb[q] = vtb[q] + vnb * nrm[q];
        v0b[q] += vrelb[q];
        vcob[q] -= vrelb[q];
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < 3; q++) v0b[q] += vcb[q];
  }
  // vco = u + w x r
  float wb[3], rb[3];
  cross3(r, vcob, wb);
  cross3(vcob, G.w, rb);
  // nrm = rp/dist ; d = dist - radius
  float rpb[3] = {0, 0, 0};
  if (!on_axis) {
    float nn = nrmb[0] * nrm[0] + nrmb[1] * nrm[1] + nrmb[2] * nrm[2];
#pragma unroll
    for (int q = 0; q < 3; q++) rpb[q] = (nrmb[q] - nn * nrm[q]) / dist + db * nrm[q];
  }
  // rp = r - (r.a) a
  float ra = rpb[0] * G.a[0] + rpb[1] * G.a[1] + rpb[2] * G.a[2];
  float ab[3];
#pragma unroll
  for (int q = 0; q < 3; q++) {
    rb[q] += rpb[q] - ra * G.a[q];
    ab[q] = -sa * rpb[q] - ra * r[q];
  }
#pragma unroll
  for (int q = 0; q < 3; q++) {
    acc[q] += vcob[q];
    acc[3 + q] += wb[q];
    acc[6 + q] -= rb[q];
    acc[9 + q] += ab[q];
  }
}

MPM_DI void grid_node_forward(const StepParams& P, int s, const int* idx, float4 g, const double* pose_t,
                              const float* act_t, float* v, void*) {
  float inv_m = 1.f / g.w;
  v[0] = g.x * inv_m + P.dt * P.grav[0];
  v[1] = g.y * inv_m + P.dt * P.grav[1];
  v[2] = g.z * inv_m + P.dt * P.grav[2];
  if (P.cyl_radius[s] > 0.f) {
    ContactGeom G;
    load_contact(P, s, pose_t, act_t, G);
    float xi[3] = {idx[0] * P.dx, idx[1] * P.dx, idx[2] * P.dx};
    contact_forward(P, G, xi, v);
  }
  const int n = P.n_grid;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    if (idx[a] < P.bound && v[a] < 0.f) v[a] = 0.f;
    if (idx[a] > n - 1 - P.bound && v[a] > 0.f) v[a] = 0.f;
  }
}

MPM_DI void grid_node_adjoint(const StepParams& P, int s, const int* idx, float4 g, const double* pose_t,
                              const float* act_t, const float* vb, float& mb, float* mvb, float* acc) {
  float inv_m = 1.f / g.w;
  float v0[3] = {g.x * inv_m + P.dt * P.grav[0], g.y * inv_m + P.dt * P.grav[1], g.z * inv_m + P.dt * P.grav[2]};
  float v1[3] = {v0[0], v0[1], v0[2]};
  bool cyl = P.cyl_radius[s] > 0.f;
  ContactGeom G;
  float xi[3] = {idx[0] * P.dx, idx[1] * P.dx, idx[2] * P.dx};
  if (cyl) {
    load_contact(P, s, pose_t, act_t, G);
    contact_forward(P, G, xi, v1);
  }
  const int n = P.n_grid;
  float ob[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    bool z = (idx[a] < P.bound && v1[a] < 0.f) || (idx[a] > n - 1 - P.bound && v1[a] > 0.f);
    ob[a] = z ? 0.f : vb[a];
  }
  float v0b[3] = {ob[0], ob[1], ob[2]};
  if (cyl) contact_adjoint(P, G, xi, v0, ob, v0b, acc);
  // v0 = mv/m + dt g
#pragma unroll
  for (int a = 0; a < 3; a++) mvb[a] = v0b[a] * inv_m;
  mb = -(v0b[0] * g.x + v0b[1] * g.y + v0b[2] * g.z) * inv_m * inv_m;
}

}  // namespace mpm
