// Device math for the MLS-MPM kernels: 3x3 helpers, an FP64 signed SVD and
// the isotropic-function derivatives used by the constitutive adjoints.
//
// Matrices are row-major arrays of 9 (element a*3+b).
#pragma once
#include <hip/hip_runtime.h>

namespace mpm {

#define MPM_DI __device__ __forceinline__

template <typename T> MPM_DI void mat_eye(T* A) {
#pragma unroll
  for (int i = 0; i < 9; i++) A[i] = (i % 4 == 0) ? T(1) : T(0);
}

// C = A B
template <typename T> MPM_DI void matmul(const T* A, const T* B, T* C) {
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) C[i * 3 + j] = A[i * 3] * B[j] + A[i * 3 + 1] * B[3 + j] + A[i * 3 + 2] * B[6 + j];
}
// C = A B^T
template <typename T> MPM_DI void matmul_nt(const T* A, const T* B, T* C) {
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) C[i * 3 + j] = A[i * 3] * B[j * 3] + A[i * 3 + 1] * B[j * 3 + 1] + A[i * 3 + 2] * B[j * 3 + 2];
}
// C = A^T B
template <typename T> MPM_DI void matmul_tn(const T* A, const T* B, T* C) {
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) C[i * 3 + j] = A[i] * B[j] + A[3 + i] * B[3 + j] + A[6 + i] * B[6 + j];
}
template <typename T> MPM_DI T det3(const T* A) {
  return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) + A[2] * (A[3] * A[7] - A[4] * A[6]);
}
// cofactor matrix: cof(A) = det(A) A^{-T}
template <typename T> MPM_DI void cof3(const T* A, T* K) {
  K[0] = A[4] * A[8] - A[5] * A[7];
  K[1] = A[5] * A[6] - A[3] * A[8];
  K[2] = A[3] * A[7] - A[4] * A[6];
  K[3] = A[2] * A[7] - A[1] * A[8];
  K[4] = A[0] * A[8] - A[2] * A[6];
  K[5] = A[1] * A[6] - A[0] * A[7];
  K[6] = A[1] * A[5] - A[2] * A[4];
  K[7] = A[2] * A[3] - A[0] * A[5];
  K[8] = A[0] * A[4] - A[1] * A[3];
}

// Precision helpers: the FP32 versions use the hardware reciprocal, square
// root and reciprocal square root (about 1 ulp; no denormal inputs arise).
MPM_DI double t_rsqrt(double x) { return rsqrt(x); }
MPM_DI float t_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
MPM_DI double t_sqrt(double x) { return sqrt(x); }
MPM_DI float t_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
MPM_DI double t_div(double a, double b) { return a / b; }
MPM_DI float t_div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
MPM_DI double t_abs(double x) { return fabs(x); }
MPM_DI float t_abs(float x) { return fabsf(x); }
MPM_DI double t_log(double x) { return log(x); }
MPM_DI float t_log(float x) { return logf(x); }
MPM_DI double t_exp(double x) { return exp(x); }
MPM_DI float t_exp(float x) { return expf(x); }

// ---------------------------------------------------------------------------
// Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations (Golub and
// Van Loan, "Matrix Computations", section 8.5): A <- J^T A J, V <- V J.
// ---------------------------------------------------------------------------
template <typename T> MPM_DI void jacobi_rotate(T* A, T* V, int p, int q) {
  T apq = A[p * 3 + q];
  if (apq == T(0)) return;
  T app = A[p * 3 + p], aqq = A[q * 3 + q];
  // t = tan(theta) of the smaller rotation angle: with d = aqq - app and
  // e = 2 apq, t = sign(d) e / (|d| + sqrt(d^2 + e^2)) (one division, one
  // square root); c = 1/sqrt(1 + t^2) keeps c^2 + s^2 = 1 for whatever t
  const T d = aqq - app, e = T(2) * apq;
  T t = t_div(d >= T(0) ? e : -e, t_abs(d) + t_sqrt(d * d + e * e));
  T c = t_rsqrt(T(1) + t * t);
  T s = t * c;
  A[p * 3 + p] = app - t * apq;
  A[q * 3 + q] = aqq + t * apq;
  A[p * 3 + q] = T(0);
  A[q * 3 + p] = T(0);
  int r = 3 - p - q;
  T arp = A[r * 3 + p], arq = A[r * 3 + q];
  T nrp = c * arp - s * arq, nrq = s * arp + c * arq;
  A[r * 3 + p] = nrp; A[p * 3 + r] = nrp;
  A[r * 3 + q] = nrq; A[q * 3 + r] = nrq;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    T vp = V[k * 3 + p], vq = V[k * 3 + q];
    V[k * 3 + p] = c * vp - s * vq;
    V[k * 3 + q] = s * vp + c * vq;
  }
}

// Signed SVD F = U diag(s) V^T with U, V in SO(3), s0 >= s1 >= |s2|, and the
// sign of det F carried by s2.  V and s^2 come from the eigen-decomposition
// of F^T F; U from the columns of F V (Gram-Schmidt, u2 = u0 x u1).
// In FP64 the sweeps stop once the off-diagonal part is below 1e-12 of the
// diagonal (eigenvalues then exact to about 1e-24 relative where separated,
// 1e-12 where they nearly coincide).  In FP32 they stop at 1e-7, the
// rounding level, within at most 6 sweeps.  Returns whether that happened.
template <typename T> MPM_DI bool svd3(const T* F, T* U, T* s, T* V) {
  constexpr bool dbl = sizeof(T) == 8;
  constexpr int max_sweeps = dbl ? 12 : 6;
  const T tol2 = dbl ? T(1e-24) : T(1e-14);
  T A[9];
  matmul_tn(F, F, A);
  mat_eye(V);
  T scale = A[0] * A[0] + A[4] * A[4] + A[8] * A[8] + (dbl ? T(1e-300) : T(1e-36));
  bool conv = false;
  for (int sweep = 0; sweep < max_sweeps; sweep++) {
    T off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
    if (off <= tol2 * scale) { conv = true; break; }
    jacobi_rotate(A, V, 0, 1);
    jacobi_rotate(A, V, 0, 2);
    jacobi_rotate(A, V, 1, 2);
  }
  if (!conv) conv = A[1] * A[1] + A[2] * A[2] + A[5] * A[5] <= tol2 * scale;
  T lam[3] = {A[0], A[4], A[8]};
  // sort descending, permuting the columns of V
#pragma unroll
  for (int pass = 0; pass < 2; pass++) {
#pragma unroll
    for (int i = 0; i < 2; i++) {
      if (lam[i] < lam[i + 1]) {
        T tl = lam[i]; lam[i] = lam[i + 1]; lam[i + 1] = tl;
#pragma unroll
        for (int k = 0; k < 3; k++) { T tv = V[k * 3 + i]; V[k * 3 + i] = V[k * 3 + i + 1]; V[k * 3 + i + 1] = tv; }
      }
    }
  }
  if (det3(V) < T(0)) {
#pragma unroll
    for (int k = 0; k < 3; k++) V[k * 3 + 2] = -V[k * 3 + 2];
  }
  T B[9];
  matmul(F, V, B);
  T b0[3] = {B[0], B[3], B[6]}, b1[3] = {B[1], B[4], B[7]}, b2[3] = {B[2], B[5], B[8]};
  // norms and normalisations from one reciprocal square root each
  const T q0 = b0[0] * b0[0] + b0[1] * b0[1] + b0[2] * b0[2];
  T n0 = T(0);
  T u0[3], u1[3], u2[3];
  if (q0 > T(0)) {
    const T r0 = t_rsqrt(q0);
    n0 = q0 * r0;
    u0[0] = b0[0] * r0; u0[1] = b0[1] * r0; u0[2] = b0[2] * r0;
  } else {
    u0[0] = T(1); u0[1] = T(0); u0[2] = T(0);
  }
  T d01 = u0[0] * b1[0] + u0[1] * b1[1] + u0[2] * b1[2];
  T w1[3] = {b1[0] - d01 * u0[0], b1[1] - d01 * u0[1], b1[2] - d01 * u0[2]};
  const T q1 = w1[0] * w1[0] + w1[1] * w1[1] + w1[2] * w1[2];
  T n1 = T(0);
  if (q1 > (dbl ? T(1e-28) : T(1e-12)) * q0 && q1 > T(0)) {
    const T r1 = t_rsqrt(q1);
    n1 = q1 * r1;
    u1[0] = w1[0] * r1; u1[1] = w1[1] * r1; u1[2] = w1[2] * r1;
  } else {
    // any unit vector orthogonal to u0
    T a[3] = {T(0), T(0), T(0)};
    int k = (t_abs(u0[0]) < T(0.57)) ? 0 : ((t_abs(u0[1]) < T(0.57)) ? 1 : 2);
    a[k] = T(1);
    T d = a[0] * u0[0] + a[1] * u0[1] + a[2] * u0[2];
    w1[0] = a[0] - d * u0[0]; w1[1] = a[1] - d * u0[1]; w1[2] = a[2] - d * u0[2];
    T rn = t_rsqrt(w1[0] * w1[0] + w1[1] * w1[1] + w1[2] * w1[2]);
    u1[0] = w1[0] * rn; u1[1] = w1[1] * rn; u1[2] = w1[2] * rn;
    n1 = u1[0] * b1[0] + u1[1] * b1[1] + u1[2] * b1[2];
  }
  u2[0] = u0[1] * u1[2] - u0[2] * u1[1];
  u2[1] = u0[2] * u1[0] - u0[0] * u1[2];
  u2[2] = u0[0] * u1[1] - u0[1] * u1[0];
  s[0] = n0;
  s[1] = n1;
  s[2] = u2[0] * b2[0] + u2[1] * b2[1] + u2[2] * b2[2];
#pragma unroll
  for (int k = 0; k < 3; k++) { U[k * 3 + 0] = u0[k]; U[k * 3 + 1] = u1[k]; U[k * 3 + 2] = u2[k]; }
  return conv;
}

// U diag(g) V^T
template <typename T> MPM_DI void usv(const T* U, const T* g, const T* V, T* out) {
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++)
      out[i * 3 + j] = U[i * 3] * g[0] * V[j * 3] + U[i * 3 + 1] * g[1] * V[j * 3 + 1] + U[i * 3 + 2] * g[2] * V[j * 3 + 2];
}

// Adjoint of an isotropic map Phi(F) = U diag(g(s)) V^T.  Given Phibar,
// returns Fbar = U Abar V^T with M = U^T Phibar V and
//   Abar_kk = sum_i M_ii dg[i][k]
//   Abar_ij = sdd[i][j] (M_ij + M_ji)/2 + (g_i + g_j)/(s_i + s_j) (M_ij - M_ji)/2
// where sdd[i][j] is the divided difference (g_i - g_j)/(s_i - s_j) supplied
// by the caller in a form that is exact at s_i = s_j.
template <typename T>
MPM_DI void iso_adjoint(const T* U, const T* s, const T* V, const T* g, const T* dg, const T* sdd, const T* Pbar,
                        T* Fbar) {
  T T1[9], M[9];
  matmul_tn(U, Pbar, T1);
  matmul(T1, V, M);
  T A[9];
#pragma unroll
  for (int k = 0; k < 3; k++) A[k * 4] = M[0] * dg[0 * 3 + k] + M[4] * dg[1 * 3 + k] + M[8] * dg[2 * 3 + k];
  // (g_i + g_j)/(s_i + s_j) is symmetric: one division per pair
  const T t01 = t_div(g[0] + g[1], s[0] + s[1]), t02 = t_div(g[0] + g[2], s[0] + s[2]),
          t12 = t_div(g[1] + g[2], s[1] + s[2]);
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) {
      if (i == j) continue;
      const T t = (i + j == 1) ? t01 : ((i + j == 2) ? t02 : t12);
      A[i * 3 + j] = sdd[i * 3 + j] * T(0.5) * (M[i * 3 + j] + M[j * 3 + i]) + t * T(0.5) * (M[i * 3 + j] - M[j * 3 + i]);
    }
  matmul(U, A, T1);
  matmul_nt(T1, V, Fbar);
}

MPM_DI double t_log1p(double x) { return log1p(x); }
MPM_DI float t_log1p(float x) { return log1pf(x); }
MPM_DI double t_expm1(double x) { return expm1(x); }
MPM_DI float t_expm1(float x) { return expm1f(x); }

// (log a - log b)/(a - b) for a, b > 0, exact as a -> b.
template <typename T> MPM_DI T log_divdiff(T a, T b) {
  const T x = t_div(a - b, b);
  if (t_abs(x) < T(1e-4)) return t_div(T(1) - x * (T(0.5) - x * (T(1) / T(3) - T(0.25) * x)), b);
  return t_div(t_log1p(x), a - b);
}

// expm1(beta d) / expm1(d), exact as d -> 0.
template <typename T> MPM_DI T expm1_ratio(T beta, T d) {
  if (t_abs(d) < T(1e-6)) return beta * (T(1) + T(0.5) * (beta - T(1)) * d);
  return t_div(t_expm1(beta * d), t_expm1(d));
}

// Both expm1(beta d)/expm1(d) (into r) and expm1(-beta d)/expm1(-d) (into
// rm) from one pair of expm1 evaluations: with E1 = expm1(beta d) and
// E0 = expm1(d), expm1(-x) = -expm1(x)/(1 + expm1(x)) gives
// rm = r (1 + E0)/(1 + E1).
template <typename T> MPM_DI void expm1_ratio_pair(T beta, T d, T& r, T& rm) {
  if (t_abs(d) < T(1e-6)) {
    r = beta * (T(1) + T(0.5) * (beta - T(1)) * d);
    rm = beta * (T(1) - T(0.5) * (beta - T(1)) * d);
    return;
  }
  const T E1 = t_expm1(beta * d), E0 = t_expm1(d);
  r = t_div(E1, E0);
  rm = t_div(r * (T(1) + E0), T(1) + E1);
}

}  // namespace mpm
