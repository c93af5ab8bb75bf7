// Sums over the 27 nodes of a particle's quadratic B-spline stencil, read
// from a tile of E^3 nodes staged in LDS (E = VT for a block's velocity
// tile, 3 for one particle's own stencil; lb = the stencil's first node in
// the tile), shared by the forward and adjoint transfer kernels.
//
// Both sums run over z inside y inside x, so that each partial sum is
// weighted once by the outer weights (w = wx wy wz factorises); the loads of
// one x plane are issued together, and a compiler barrier between planes
// keeps the next plane's loads from being hoisted (nine loads in flight
// rather than 27 bounds the register count).
#pragma once
#include <hip/hip_runtime.h>
#include "mpm_fast.h"
#include "mpm_phys.h"

namespace mpm {

// G2P gather: vn = sum_i w_i v_i and Bi = sum_i w_i v_i idx_i^T with idx_i
// in {0,1,2}^3 the node's offset in the stencil (v_i = the tile's xyz).
template <int E = VT>
__device__ __forceinline__ void g2p_gather(const float4* __restrict__ s_v, const int* lb, const Stencil& S,
                                           float* vn, float* Bi) {
#pragma unroll
  for (int q = 0; q < 3; q++) vn[q] = 0.f;
#pragma unroll
  for (int q = 0; q < 9; q++) Bi[q] = 0.f;
  const float wz1 = S.w[2][1], wz2 = S.w[2][2], wz2x2 = 2.f * S.w[2][2];
#pragma unroll
  for (int i = 0; i < 3; i++) {
    float p0[3] = {0, 0, 0}, pj[3] = {0, 0, 0}, pk[3] = {0, 0, 0};
#pragma unroll
    for (int jj = 0; jj < 3; jj++) {
      const float4* row = s_v + ((lb[0] + i) * E + lb[1] + jj) * E + lb[2];
      const float4 g0 = row[0], g1 = row[1], g2 = row[2];
      // r = sum_k w_k v_k, rk = sum_k k w_k v_k along z
      const float r[3] = {S.w[2][0] * g0.x + wz1 * g1.x + wz2 * g2.x, S.w[2][0] * g0.y + wz1 * g1.y + wz2 * g2.y,
                          S.w[2][0] * g0.z + wz1 * g1.z + wz2 * g2.z};
      const float rk[3] = {wz1 * g1.x + wz2x2 * g2.x, wz1 * g1.y + wz2x2 * g2.y, wz1 * g1.z + wz2x2 * g2.z};
      const float wy = S.w[1][jj];
#pragma unroll
      for (int a = 0; a < 3; a++) {
        p0[a] += wy * r[a];
        if (jj) pj[a] += ((float)jj * wy) * r[a];
        pk[a] += wy * rk[a];
      }
    }
    const float wx = S.w[0][i];
#pragma unroll
    for (int a = 0; a < 3; a++) {
      vn[a] += wx * p0[a];
      if (i) Bi[a * 3 + 0] += ((float)i * wx) * p0[a];
      Bi[a * 3 + 1] += wx * pj[a];
      Bi[a * 3 + 2] += wx * pk[a];
    }
    asm volatile("" ::: "memory");
  }
}

// The weight-gradient sum of the transfers' adjoints:
//   X = sum_i (dw_x wy wz, wx dw_y wz, wx wy dw_z)_i s_i  (dw = dw/df; the
//   caller divides by dx), with s_i = mw g_i.w + g_i.xyz . (c0 + Ad idx_i)
// for the tile's values g_i (the term affine in the node offset is the
// adjoint of the node's momentum, mom = mvp + A (x_i - x_p), or of the G2P
// terms v_i (vbt + Bb (x_i - x_p)), written as c0 + Ad idx).  With WANT_G it
// also returns G0 = sum_i w_i g_i.xyz and Gi = sum_i w_i g_i.xyz idx_i^T.
template <bool WANT_G, int E = VT>
__device__ __forceinline__ void weight_grad_sum(const float4* __restrict__ tile, const int* lb, const Stencil& S,
                                                const float* c0, const float* Ad, float mw, float* X, float* G0,
                                                float* Gi) {
#pragma unroll
  for (int a = 0; a < 3; a++) X[a] = 0.f;
  if (WANT_G) {
#pragma unroll
    for (int q = 0; q < 3; q++) G0[q] = 0.f;
#pragma unroll
    for (int q = 0; q < 9; q++) Gi[q] = 0.f;
  }
#pragma unroll
  for (int i = 0; i < 3; i++) {
    float m1[3];
#pragma unroll
    for (int a = 0; a < 3; a++) m1[a] = c0[a] + (float)i * Ad[a * 3];
    float Px = 0.f, Py = 0.f, Pz = 0.f;
    float p0[3] = {0, 0, 0}, pj[3] = {0, 0, 0}, pk[3] = {0, 0, 0};
#pragma unroll
    for (int jj = 0; jj < 3; jj++) {
      const float4* row = tile + ((lb[0] + i) * E + lb[1] + jj) * E + lb[2];
      const float4 g[3] = {row[0], row[1], row[2]};
      float m2[3];
#pragma unroll
      for (int a = 0; a < 3; a++) m2[a] = m1[a] + (float)jj * Ad[a * 3 + 1];
      float sk[3];
#pragma unroll
      for (int k = 0; k < 3; k++) {
        const float u0 = m2[0] + (float)k * Ad[2], u1 = m2[1] + (float)k * Ad[5], u2 = m2[2] + (float)k * Ad[8];
        sk[k] = g[k].x * u0 + g[k].y * u1 + g[k].z * u2;
        if (mw != 0.f) sk[k] += mw * g[k].w;
      }
      // z sums: with w_z and with dw_z
      const float R0 = S.w[2][0] * sk[0] + S.w[2][1] * sk[1] + S.w[2][2] * sk[2];
      const float R1 = S.dw[2][0] * sk[0] + S.dw[2][1] * sk[1] + S.dw[2][2] * sk[2];
      const float wy = S.w[1][jj], dwy = S.dw[1][jj];
      Px += wy * R0;
      Py += dwy * R0;
      Pz += wy * R1;
      if (WANT_G) {
        const float r[3] = {S.w[2][0] * g[0].x + S.w[2][1] * g[1].x + S.w[2][2] * g[2].x,
                            S.w[2][0] * g[0].y + S.w[2][1] * g[1].y + S.w[2][2] * g[2].y,
                            S.w[2][0] * g[0].z + S.w[2][1] * g[1].z + S.w[2][2] * g[2].z};
        const float wz22 = 2.f * S.w[2][2];
        const float rk[3] = {S.w[2][1] * g[1].x + wz22 * g[2].x, S.w[2][1] * g[1].y + wz22 * g[2].y,
                             S.w[2][1] * g[1].z + wz22 * g[2].z};
#pragma unroll
        for (int a = 0; a < 3; a++) {
          p0[a] += wy * r[a];
          if (jj) pj[a] += ((float)jj * wy) * r[a];
          pk[a] += wy * rk[a];
        }
      }
    }
    const float wx = S.w[0][i], dwx = S.dw[0][i];
    X[0] += dwx * Px;
    X[1] += wx * Py;
    X[2] += wx * Pz;
    if (WANT_G) {
#pragma unroll
      for (int a = 0; a < 3; a++) {
        G0[a] += wx * p0[a];
        if (i) Gi[a * 3 + 0] += ((float)i * wx) * p0[a];
        Gi[a * 3 + 1] += wx * pj[a];
        Gi[a * 3 + 2] += wx * pk[a];
      }
    }
    asm volatile("" ::: "memory");
  }
}

}  // namespace mpm
