// Tiled adjoint of the MLS-MPM step for gfx950 (FluidLab section 3.3 and
// App. A: the gradient of a loss through the rollout by reverse-mode
// differentiation, with checkpoints recomputed segment by segment).
//
// Every state of a recomputed segment is kept sorted by the 4^3 block key of
// its own positions, so that the particles of one block sit in contiguous
// rows, like the forward path's.  The adjoint of step t (state s_t -> s_{t+1})
// then runs on s_t's blocks:
//   fast_p2g, fast_grid   recompute the grid of step t: node momenta and
//                         masses (block layout) and the updated velocities
//   k_g2p_adj_tiled       one workgroup per occupied block: G2P recomputed
//                         from an LDS copy of the velocities, the adjoint of
//                         the particle update, and the scatter of the
//                         velocity adjoint into a fixed-point LDS tile whose
//                         non-zero box is published (no global float atomics)
//   k_g2p_adj_redo        the particles whose plastic-return adjoint is
//                         ill-conditioned in FP32, listed by the kernel
//                         above: the same steps with the FP64 adjoint, the
//                         scatter added to the published tiles
//   k_grid_adj_tiled      per node of the blocks claimed in the recompute:
//                         sum of the 27 neighbouring tiles, then the adjoint
//                         of the node update (walls, contact, gravity,
//                         normalisation) and the collider partials, reduced
//                         per wavefront before one FP64 atomic per scene
//   k_p2g_adj_tiled       one workgroup per occupied block: the P2G adjoint
//                         gathered from an LDS copy of the node adjoints,
//                         through the stress adjoint
//   k_p2g_adj_redo        the solids whose F is ill-conditioned in FP32,
//                         listed by the kernel above: the same with FP64 SVDs.
// The FP64 paths run in kernels of their own so that their register demand
// does not set the occupancy of the common FP32 path.
// The adjoint of s_{t+1} is read through the row map that the segment's sort
// recorded, so no separate permutation pass is needed.
#include <hip/hip_runtime.h>
#include <math.h>
#include "mpm_adjoint.h"
#include "mpm_blocks.h"
#include "mpm_math.h"
#include "mpm_phys.h"
#include "mpm_transfer.h"

namespace mpm {

namespace {

__device__ inline float4 stage_node(const float4* __restrict__ src, const FastGeom& g, int sc, int gx, int gy, int gz) {
  if (gx < 0 || gy < 0 || gz < 0 || gx >= g.n || gy >= g.n || gz >= g.n) return make_float4(0.f, 0.f, 0.f, 0.f);
  uint32_t kk = block_key(g, sc, gx >> 2, gy >> 2, gz >> 2);
  return src[(size_t)kk * 64 + (((gx & 3) << 4) | ((gy & 3) << 2) | (gz & 3))];
}

}  // namespace

// ---------------------------------------------------------------------------
// Adjoint of G2P and of the particle update; scatter of the grid velocity
// adjoint.  Writes the direct part of the state adjoint of s_t (x, F, J; the
// v and C adjoints of s_t come only through P2G and are added later).
// ---------------------------------------------------------------------------
// (three workgroups per CU; the FP64 plastic-return adjoint runs in
// k_g2p_adj_redo, so that its registers do not count here)
template <int NT>
__global__ __launch_bounds__(NT, 3) void k_g2p_adj_tiled(AdjArgs A, StepParams P, FastGeom g) {
  constexpr int NW = NT / 64;
  constexpr int NQ = 3;   // velocity adjoint components
  __shared__ float4 s_v[VT_NODES];
  __shared__ float s_tile[NQ * TILE_NODES];
  __shared__ int s_itile[NQ * TILE_NODES];
  __shared__ int s_lo[3], s_hi[3];
  __shared__ float s_red[NW * NQ], s_scale[2 * NQ];
  __shared__ int s_ired[NW * 6 + 6];
  const int tid = threadIdx.x;
  const int N = A.N;
  const PState st = packed_state(A.st.f, N);
  const uint32_t n_list = A.list_n[0];
  const uint32_t stamp = (A.gen[0] << 16) | A.sid;
  for (uint32_t e = blockIdx.x; e < n_list; e += gridDim.x) {
    const int4 ent = A.list[e];
    int sc, bx, by, bz;
    key_decode(g, (uint32_t)ent.x, sc, bx, by, bz);
    const int ox = 4 * bx, oy = 4 * by, oz = 4 * bz;
    for (int q = tid; q < VT_NODES; q += NT) {
      const int qi = q / (VT * VT), qj = (q / VT) % VT, qk = q % VT;
      s_v[q] = stage_node(A.vgrid, g, sc, ox - 1 + qi, oy - 1 + qj, oz - 1 + qk);
    }
    for (int q = tid; q < NQ * TILE_NODES; q += NT) { s_tile[q] = 0.f; s_itile[q] = 0; }
    if (tid < 3) { s_lo[tid] = 1 << 20; s_hi[tid] = -(1 << 20); }
    __syncthreads();
    const int start = ent.y, count = ent.z;
    for (int c0 = 0; c0 < count; c0 += NT) {
      const int j = start + c0 + tid;
      const bool has = (c0 + tid) < count && j < N;
      bool ok = has;
      float x[3] = {0, 0, 0};
      int m = 0;
      if (has) {
#pragma unroll
        for (int a = 0; a < 3; a++) x[a] = st.x[a * (size_t)N + j];
        m = A.st.mat[j];
      }
      const MatDev& M = P.mats[m];
      Stencil S;
      int lb[3] = {0, 0, 0}, lv[3] = {0, 0, 0};
      if (ok) {
        const bool in_grid = stencil_setup(x, P, S);
#pragma unroll
        for (int a = 0; a < 3; a++) {
          lv[a] = S.base[a] - ((a == 0 ? ox : a == 1 ? oy : oz) - 1);
          lb[a] = S.base[a] - ((a == 0 ? ox : a == 1 ? oy : oz) - 2);
        }
        const bool in_tile = lv[0] >= 0 && lv[1] >= 0 && lv[2] >= 0 && lv[0] <= VT - 3 && lv[1] <= VT - 3 &&
                             lv[2] <= VT - 3 && lb[0] <= TILE - 3 && lb[1] <= TILE - 3 && lb[2] <= TILE - 3;
        if (!in_grid) { atomicOr(P.err, ERR_OUTSIDE); ok = false; }
        else if (!in_tile) { atomicOr(P.err, ERR_TILE); ok = false; }
        else if (A.map[j] >= (uint32_t)N) { atomicOr(P.err, ERR_TILE); ok = false; }
      }
      float vbt[3] = {0, 0, 0}, Bb[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, bnd[NQ] = {0, 0, 0};
      float vn[3], xb[3], Fbo[9], Jbo = 0.f;
      bool defer = false;
      if (ok) {
        // G2P recomputed from the staged velocities
        float Bi[9];
        g2p_gather(s_v, lv, S, vn, Bi);
        float B[9];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
          for (int b = 0; b < 3; b++) B[a * 3 + b] = P.dx * (Bi[a * 3 + b] - vn[a] * S.f[b]);
        // adjoint of s_{t+1}, row jn of the next state's order
        const uint32_t jn = A.map[j];
        const float* an = A.abar_next;
        float vb[3], Cb[9], Fb[9];
#pragma unroll
        for (int a = 0; a < 3; a++) { xb[a] = an[a * (size_t)N + jn]; vb[a] = an[(3 + a) * (size_t)N + jn]; }
#pragma unroll
        for (int k = 0; k < 9; k++) { Cb[k] = an[(6 + k) * (size_t)N + jn]; Fb[k] = an[(15 + k) * (size_t)N + jn]; }
        const float Jb = an[24 * (size_t)N + jn];
        defer = !particle_update_adjoint<ADJ_FP32>(x, vn, B, M, P, st, j, xb, vb, Cb, Fb, Jb, vbt, Bb, Fbo, Jbo);
      }
      if (defer) {
        // listed for the FP64 pass; it stays in the tile box, scatters nothing here
        const uint32_t r = atomicAdd(A.redo_n, 1u);
        A.redo[r] = make_uint2((uint32_t)j, (uint32_t)ent.x);
      } else if (ok) {
        // position adjoint through the weights and the node offsets:
        // xo = xb + sum_i grad w_i (v_i . (vbt + Bb (x_i - x_p))) - Bb^T vn
        float xo[3];
        {
          float c0[3], Ad[9], X[3];
#pragma unroll
          for (int a = 0; a < 3; a++) {
#pragma unroll
            for (int b = 0; b < 3; b++) Ad[a * 3 + b] = P.dx * Bb[a * 3 + b];
            c0[a] = vbt[a] - (Ad[a * 3] * S.f[0] + Ad[a * 3 + 1] * S.f[1] + Ad[a * 3 + 2] * S.f[2]);
          }
          weight_grad_sum<false>(s_v, lv, S, c0, Ad, 0.f, X, nullptr, nullptr);
#pragma unroll
          for (int a = 0; a < 3; a++)
            xo[a] = xb[a] + P.inv_dx * X[a] - (Bb[a] * vn[0] + Bb[3 + a] * vn[1] + Bb[6 + a] * vn[2]);
        }
        float* ab = A.abar;
#pragma unroll
        for (int a = 0; a < 3; a++) { ab[a * (size_t)N + j] = xo[a]; ab[(3 + a) * (size_t)N + j] = 0.f; }
#pragma unroll
        for (int k = 0; k < 9; k++) { ab[(6 + k) * (size_t)N + j] = 0.f; ab[(15 + k) * (size_t)N + j] = Fbo[k]; }
        ab[24 * (size_t)N + j] = Jbo;
#pragma unroll
        for (int a = 0; a < 3; a++)
          bnd[a] = fabsf(vbt[a]) + 1.5f * P.dx * (fabsf(Bb[a * 3]) + fabsf(Bb[a * 3 + 1]) + fabsf(Bb[a * 3 + 2]));
        if (!isfinite(bnd[0] + bnd[1] + bnd[2])) {
          atomicOr(P.err, ERR_NONFINITE);
          ok = false;
#pragma unroll
          for (int a = 0; a < NQ; a++) bnd[a] = 0.f;
        }
      } else if (has) {
        // a particle outside the grid carries no adjoint (the call reports it)
        float* ab = A.abar;
#pragma unroll
        for (int k = 0; k < STATE_FLOATS; k++) ab[k * (size_t)N + j] = 0.f;
      }
      // chunk-wide bound sums and box, as in the forward P2G
      int clo[3], chi[3];
#pragma unroll
      for (int a = 0; a < 3; a++) { clo[a] = ok ? lb[a] : 1 << 20; chi[a] = ok ? lb[a] : -(1 << 20); }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int q = 0; q < NQ; q++) bnd[q] += __shfl_xor(bnd[q], off);
#pragma unroll
        for (int a = 0; a < 3; a++) { clo[a] = min(clo[a], __shfl_xor(clo[a], off)); chi[a] = max(chi[a], __shfl_xor(chi[a], off)); }
      }
      const int wv = tid >> 6;
      if ((tid & 63) == 0) {
#pragma unroll
        for (int q = 0; q < NQ; q++) s_red[wv * NQ + q] = bnd[q];
#pragma unroll
        for (int a = 0; a < 3; a++) { s_ired[wv * 6 + a] = clo[a]; s_ired[wv * 6 + 3 + a] = chi[a]; }
      }
      __syncthreads();
      if (tid == 0) {
#pragma unroll
        for (int q = 0; q < NQ; q++) {
          float T = 0.f;
#pragma unroll
          for (int w = 0; w < NW; w++) T += s_red[w * NQ + q];
          T *= 0.421875f;   // largest weight of one node, (3/4)^3
          if (!isfinite(T)) { atomicOr(P.err, ERR_NONFINITE); T = 1.f; }
          int ex = 0;
          frexpf(T > 0.f ? T : 1.f, &ex);
          ex = max(ex, -90);
          s_scale[q] = ldexpf(1.f, 30 - ex);
          s_scale[NQ + q] = ldexpf(1.f, ex - 30);
        }
#pragma unroll
        for (int a = 0; a < 3; a++) {
          int lo = s_ired[a], hi = s_ired[3 + a];
#pragma unroll
          for (int w = 1; w < NW; w++) { lo = min(lo, s_ired[w * 6 + a]); hi = max(hi, s_ired[w * 6 + 3 + a]); }
          s_ired[NW * 6 + a] = lo;
          s_ired[NW * 6 + 3 + a] = hi;
          if (lo <= hi) { s_lo[a] = min(s_lo[a], lo); s_hi[a] = max(s_hi[a], hi); }
        }
      }
      __syncthreads();
      if (ok && !defer) {
        // c_a(node) = w (vbt_a + sum_b Bb_ab (idx_b - f_b) dx), scaled
        float c0[3], Ad[9];
#pragma unroll
        for (int a = 0; a < 3; a++) {
          const float sa = s_scale[a];
#pragma unroll
          for (int b = 0; b < 3; b++) Ad[a * 3 + b] = sa * P.dx * Bb[a * 3 + b];
          c0[a] = sa * vbt[a] - (Ad[a * 3] * S.f[0] + Ad[a * 3 + 1] * S.f[1] + Ad[a * 3 + 2] * S.f[2]);
        }
        int* T = s_itile + (lb[0] * TILE + lb[1]) * TILE + lb[2];
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
          for (int jj = 0; jj < 3; jj++) {
            const float wxy = S.w[0][i] * S.w[1][jj];
#pragma unroll
            for (int k = 0; k < 3; k++) {
              const float w = wxy * S.w[2][k];
              const int q = (i * TILE + jj) * TILE + k;
#pragma unroll
              for (int a = 0; a < 3; a++)
                atomicAdd(&T[a * TILE_NODES + q],
                          __float2int_rn(w * (c0[a] + (float)i * Ad[a * 3] + (float)jj * Ad[a * 3 + 1] + (float)k * Ad[a * 3 + 2])));
            }
          }
      }
      __syncthreads();
      {
        const int lo0 = s_ired[NW * 6], lo1 = s_ired[NW * 6 + 1], lo2 = s_ired[NW * 6 + 2];
        const int hi0 = s_ired[NW * 6 + 3], hi1 = s_ired[NW * 6 + 4], hi2 = s_ired[NW * 6 + 5];
        if (lo0 <= hi0) {
          const int ex = hi0 - lo0 + 3, ey = hi1 - lo1 + 3, ez = hi2 - lo2 + 3;
          const int cnt = ex * ey * ez;
          for (int r = tid; r < cnt; r += NT) {
            const int qq = ((lo0 + r / (ey * ez)) * TILE + lo1 + (r / ez) % ey) * TILE + lo2 + r % ez;
#pragma unroll
            for (int c = 0; c < NQ; c++) {
              const int iv = s_itile[c * TILE_NODES + qq];
              if (iv != 0) {
                s_tile[c * TILE_NODES + qq] += (float)iv * s_scale[NQ + c];
                s_itile[c * TILE_NODES + qq] = 0;
              }
            }
          }
        }
      }
      __syncthreads();
    }
    // publish the tile's non-zero box (rows 0..2 of the block's tile slot)
    const int lo0 = s_lo[0], lo1 = s_lo[1], lo2 = s_lo[2];
    const int hi0 = s_hi[0] + 2, hi1 = s_hi[1] + 2, hi2 = s_hi[2] + 2;
    const uint32_t bkey = (uint32_t)ent.x;
    if (lo0 <= hi0 - 2) {
      const int ex = hi0 - lo0 + 1, ey = hi1 - lo1 + 1, ez = hi2 - lo2 + 1;
      const int cnt = ex * ey * ez;
      float* T = A.tiles + (size_t)bkey * 4 * TILE_NODES;
      for (int r = tid; r < cnt; r += NT) {
        const int q = ((lo0 + r / (ey * ez)) * TILE + lo1 + (r / ez) % ey) * TILE + lo2 + r % ez;
#pragma unroll
        for (int c = 0; c < NQ; c++) T[c * TILE_NODES + q] = s_tile[c * TILE_NODES + q];
      }
      if (tid == 0) {
        const int packed = lo0 | (lo1 << 4) | (lo2 << 8) | (hi0 << 12) | (hi1 << 16) | (hi2 << 20);
        A.tile_box[bkey] = make_int2(packed, (int)stamp);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// The FP64 pass of the G2P adjoint over the particles k_g2p_adj_tiled listed:
// each thread stages its particle's 27 stencil nodes in LDS and repeats the
// steps above with the FP64 plastic-return adjoint; its velocity-adjoint
// scatter goes into the block's published tile with float atomics (the
// listed particles were kept inside the tile's box).
// ---------------------------------------------------------------------------
constexpr int REDO_NT = 64, REDO_WGS = 256;

__global__ __launch_bounds__(REDO_NT) void k_g2p_adj_redo(AdjArgs A, StepParams P, FastGeom g) {
  __shared__ float4 s_loc[REDO_NT * 27];
  float4* loc = s_loc + threadIdx.x * 27;
  const int N = A.N;
  const PState st = packed_state(A.st.f, N);
  const uint32_t n = A.redo_n[0];
  for (uint32_t e = blockIdx.x * REDO_NT + threadIdx.x; e < n; e += gridDim.x * REDO_NT) {
    const uint2 r = A.redo[e];
    const int j = (int)r.x;
    int sc, bx, by, bz;
    key_decode(g, r.y, sc, bx, by, bz);
    float x[3];
#pragma unroll
    for (int a = 0; a < 3; a++) x[a] = st.x[a * (size_t)N + j];
    const MatDev& M = P.mats[A.st.mat[j]];
    Stencil S;
    stencil_setup(x, P, S);   // inside the grid and the tile: checked when listed
    const int lb[3] = {S.base[0] - (4 * bx - 2), S.base[1] - (4 * by - 2), S.base[2] - (4 * bz - 2)};
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int jj = 0; jj < 3; jj++)
#pragma unroll
        for (int k = 0; k < 3; k++)
          loc[(i * 3 + jj) * 3 + k] = stage_node(A.vgrid, g, sc, S.base[0] + i, S.base[1] + jj, S.base[2] + k);
    const int l0[3] = {0, 0, 0};
    float vn[3], Bi[9], B[9];
    g2p_gather<3>(loc, l0, S, vn, Bi);
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) B[a * 3 + b] = P.dx * (Bi[a * 3 + b] - vn[a] * S.f[b]);
    const uint32_t jn = A.map[j];
    const float* an = A.abar_next;
    float xb[3], vb[3], Cb[9], Fb[9];
#pragma unroll
    for (int a = 0; a < 3; a++) { xb[a] = an[a * (size_t)N + jn]; vb[a] = an[(3 + a) * (size_t)N + jn]; }
#pragma unroll
    for (int k = 0; k < 9; k++) { Cb[k] = an[(6 + k) * (size_t)N + jn]; Fb[k] = an[(15 + k) * (size_t)N + jn]; }
    const float Jb = an[24 * (size_t)N + jn];
    float vbt[3], Bb[9], Fbo[9], Jbo;
    particle_update_adjoint<ADJ_FP64>(x, vn, B, M, P, st, j, xb, vb, Cb, Fb, Jb, vbt, Bb, Fbo, Jbo);
    float c0[3], Ad[9], X[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
#pragma unroll
      for (int b = 0; b < 3; b++) Ad[a * 3 + b] = P.dx * Bb[a * 3 + b];
      c0[a] = vbt[a] - (Ad[a * 3] * S.f[0] + Ad[a * 3 + 1] * S.f[1] + Ad[a * 3 + 2] * S.f[2]);
    }
    weight_grad_sum<false, 3>(loc, l0, S, c0, Ad, 0.f, X, nullptr, nullptr);
    float* ab = A.abar;
#pragma unroll
    for (int a = 0; a < 3; a++) {
      ab[a * (size_t)N + j] = xb[a] + P.inv_dx * X[a] - (Bb[a] * vn[0] + Bb[3 + a] * vn[1] + Bb[6 + a] * vn[2]);
      ab[(3 + a) * (size_t)N + j] = 0.f;
    }
#pragma unroll
    for (int k = 0; k < 9; k++) { ab[(6 + k) * (size_t)N + j] = 0.f; ab[(15 + k) * (size_t)N + j] = Fbo[k]; }
    ab[24 * (size_t)N + j] = Jbo;
    bool fin = true;
#pragma unroll
    for (int k = 0; k < 9; k++) fin = fin && isfinite(Ad[k]);
    if (!(fin && isfinite(c0[0] + c0[1] + c0[2]))) { atomicOr(P.err, ERR_NONFINITE); continue; }
    float* T = A.tiles + (size_t)r.y * 4 * TILE_NODES + (lb[0] * TILE + lb[1]) * TILE + lb[2];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int jj = 0; jj < 3; jj++) {
        const float wxy = S.w[0][i] * S.w[1][jj];
#pragma unroll
        for (int k = 0; k < 3; k++) {
          const float w = wxy * S.w[2][k];
          const int q = (i * TILE + jj) * TILE + k;
#pragma unroll
          for (int a = 0; a < 3; a++)
            atomicAdd(&T[a * TILE_NODES + q],
                      w * (c0[a] + (float)i * Ad[a * 3] + (float)jj * Ad[a * 3 + 1] + (float)k * Ad[a * 3 + 2]));
        }
      }
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the grid update on the nodes of the blocks claimed in the
// recompute of step t (the same blocks the velocity-adjoint tiles touch).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_grid_adj_tiled(AdjArgs A, StepParams P, FastGeom g,
                                                        const double* __restrict__ pose_t,
                                                        const float* __restrict__ act_t, double* __restrict__ acc_t) {
  const uint32_t n_cl = A.cl_count[0];
  const uint32_t stamp = (A.gen[0] << 16) | A.sid;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane >> 4, lj = (lane >> 2) & 3, lk = lane & 3;
  // one claimed block per wavefront (see k_grid)
  const uint32_t n_waves = 4u * gridDim.x;
  for (uint32_t it = 4u * blockIdx.x + (uint32_t)wv; it < n_cl && it < (uint32_t)g.n_keys; it += n_waves) {
    const uint32_t key = A.cl_list[it];
    int sc, cx, cy, cz;
    key_decode(g, key, sc, cx, cy, cz);
    {
      int2 nbox = make_int2(0, 0);
      uint32_t nkey = 0;
      if (lane < 27) {
        const int sx = cx + lane / 9 - 1, sy = cy + (lane / 3) % 3 - 1, sz = cz + lane % 3 - 1;
        if (sx >= 0 && sy >= 0 && sz >= 0 && sx < g.nb && sy < g.nb && sz < g.nb) {
          nkey = block_key(g, sc, sx, sy, sz);
          nbox = A.tile_box[nkey];
          if ((uint32_t)nbox.y != stamp) nbox.y = 0;
        }
      }
      const int gx = 4 * cx + li, gy = 4 * cy + lj, gz = 4 * cz + lk;
      // branch-free over the 27 neighbours (see k_grid)
      float vb[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int dd = 0; dd < 27; dd++) {
        const int bxv = __shfl(nbox.x, dd);
        const int valid = __shfl(nbox.y, dd);
        const uint32_t kk = __shfl(nkey, dd);
        const int sx = cx + dd / 9 - 1, sy = cy + (dd / 3) % 3 - 1, sz = cz + dd % 3 - 1;
        const int qi = gx - (4 * sx - 2), qj = gy - (4 * sy - 2), qk = gz - (4 * sz - 2);
        const int lo0 = bxv & 15, lo1 = (bxv >> 4) & 15, lo2 = (bxv >> 8) & 15;
        const int hi0 = (bxv >> 12) & 15, hi1 = (bxv >> 16) & 15, hi2 = (bxv >> 20) & 15;
        const bool in = valid && qi >= lo0 && qi <= hi0 && qj >= lo1 && qj <= hi1 && qk >= lo2 && qk <= hi2;
        const int q = in ? (qi * TILE + qj) * TILE + qk : 0;
        const float* T = A.tiles + (size_t)(in ? kk : 0u) * 4 * TILE_NODES;
        const float t0 = T[q], t1 = T[TILE_NODES + q], t2 = T[2 * TILE_NODES + q];
        vb[0] += in ? t0 : 0.f;
        vb[1] += in ? t1 : 0.f;
        vb[2] += in ? t2 : 0.f;
      }
      const size_t node = (size_t)key * 64 + lane;
      const float4 gm = A.mmv[node];
      float loc[ACC_DOUBLES];
#pragma unroll
      for (int q = 0; q < ACC_DOUBLES; q++) loc[q] = 0.f;
      float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
      if (gm.w > 0.f && gx < g.n && gy < g.n && gz < g.n) {
        const int idx[3] = {gx, gy, gz};
        float mb, mvb[3];
        grid_node_adjoint(P, sc, idx, gm, pose_t, act_t, vb, mb, mvb, loc);
        out = make_float4(mvb[0], mvb[1], mvb[2], mb);
      }
      A.mmvb[node] = out;
      // collider partials: one scene per block, reduced over the wavefront
      bool any = false;
#pragma unroll
      for (int q = 0; q < ACC_DOUBLES; q++) any |= (loc[q] != 0.f);
      if (__ballot(any)) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
          for (int q = 0; q < ACC_DOUBLES; q++) loc[q] += __shfl_xor(loc[q], off);
        if (lane == 0) {
          double* dst = acc_t + (size_t)sc * ACC_DOUBLES;
#pragma unroll
          for (int q = 0; q < ACC_DOUBLES; q++)
            if (loc[q] != 0.f) atomicAdd(dst + q, (double)loc[q]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint of P2G: gather of the node adjoints, through the stress adjoint;
// added to the state adjoint of s_t.
// ---------------------------------------------------------------------------
// One particle.  FP64 = false: the stress and its adjoint from one FP32 SVD;
// returns false, before doing anything, for a solid whose F is
// ill-conditioned (s2 < s0/4) or whose FP32 sweeps do not converge.
// FP64 = true: the stress and its adjoint from FP64 SVDs, for the particles
// the FP32 pass returned (k_p2g_adj_redo).  The tile holds E^3 nodes, lv is
// the stencil's first node in it.
template <bool FP64, int E>
MPM_DI bool p2g_adj_particle(const AdjArgs& A, const StepParams& P, const PState& st, const float4* tile,
                             const int* lv, const Stencil& S, int j) {
  const int N = A.N;
  const MatDev& M = P.mats[A.st.mat[j]];
  const bool liquid = M.kind == KIND_LIQUID;
  float Ff[9], U[9], sv[3], V[9], tau[9];
  const float Jv = st.J[j];
  float C[9];
#pragma unroll
  for (int k = 0; k < 9; k++) C[k] = st.C[k * (size_t)N + j];
  if (liquid) {
    if (FP64) return true;
    stress_liquid(Jv, C, M, tau);
  } else {
#pragma unroll
    for (int k = 0; k < 9; k++) Ff[k] = st.F[k * (size_t)N + j];
    if (FP64) {
      stress_solid(Ff, M, tau);
    } else {
      if (!(svd3(Ff, U, sv, V) && sv[2] > 0.25f * sv[0])) return false;
      stress_solid_usv(Ff, U, sv, V, M, tau);
    }
  }
  float v[3] = {st.v[j], st.v[(size_t)N + j], st.v[2 * (size_t)N + j]};
  float Am[9];
  const float scl = -P.dt * M.vol * 4.f * P.inv_dx * P.inv_dx;
#pragma unroll
  for (int k = 0; k < 9; k++) Am[k] = scl * tau[k] + M.mass * C[k];
  const float mvp[3] = {M.mass * v[0], M.mass * v[1], M.mass * v[2]};
  // node adjoints gathered: mom_i = mvp + Am (x_i - x_p) = c0 + Ad idx_i
  float vb[3], Ab[9], xb[3];
  {
    float c0[3], Ad[9], X[3], G0[3], Gi[9];
#pragma unroll
    for (int a = 0; a < 3; a++) {
#pragma unroll
      for (int b = 0; b < 3; b++) Ad[a * 3 + b] = P.dx * Am[a * 3 + b];
      c0[a] = mvp[a] - (Ad[a * 3] * S.f[0] + Ad[a * 3 + 1] * S.f[1] + Ad[a * 3 + 2] * S.f[2]);
    }
    weight_grad_sum<true, E>(tile, lv, S, c0, Ad, M.mass, X, G0, Gi);
#pragma unroll
    for (int a = 0; a < 3; a++) {
      vb[a] = M.mass * G0[a];
#pragma unroll
      for (int b = 0; b < 3; b++) Ab[a * 3 + b] = P.dx * (Gi[a * 3 + b] - G0[a] * S.f[b]);
      xb[a] = P.inv_dx * X[a] - (Am[a] * G0[0] + Am[3 + a] * G0[1] + Am[6 + a] * G0[2]);
    }
  }
  float taub[9], Cb[9], Fb[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < 9; k++) { taub[k] = scl * Ab[k]; Cb[k] = M.mass * Ab[k]; }
  float Jb = 0.f;
  if (liquid) stress_liquid_adjoint(Jv, C, M, taub, Jb, Cb);
  else if (FP64) stress_solid_adjoint(Ff, M, taub, Fb);
  else stress_solid_adjoint_usv(Ff, U, sv, V, M, taub, Fb);
  float* ab = A.abar;
#pragma unroll
  for (int a = 0; a < 3; a++) { ab[a * (size_t)N + j] += xb[a]; ab[(3 + a) * (size_t)N + j] += vb[a]; }
#pragma unroll
  for (int k = 0; k < 9; k++) { ab[(6 + k) * (size_t)N + j] += Cb[k]; ab[(15 + k) * (size_t)N + j] += Fb[k]; }
  ab[24 * (size_t)N + j] += Jb;
  return true;
}

template <int NT>
__global__ __launch_bounds__(NT) void k_p2g_adj_tiled(AdjArgs A, StepParams P, FastGeom g) {
  __shared__ float4 s_g[VT_NODES];
  const int tid = threadIdx.x;
  const int N = A.N;
  const PState st = packed_state(A.st.f, N);
  const uint32_t n_list = A.list_n[0];
  for (uint32_t e = blockIdx.x; e < n_list; e += gridDim.x) {
    const int4 ent = A.list[e];
    int sc, bx, by, bz;
    key_decode(g, (uint32_t)ent.x, sc, bx, by, bz);
    const int ox = 4 * bx, oy = 4 * by, oz = 4 * bz;
    for (int q = tid; q < VT_NODES; q += NT) {
      const int qi = q / (VT * VT), qj = (q / VT) % VT, qk = q % VT;
      s_g[q] = stage_node(A.mmvb, g, sc, ox - 1 + qi, oy - 1 + qj, oz - 1 + qk);
    }
    __syncthreads();
    const int start = ent.y, count = ent.z;
    for (int c0 = 0; c0 < count; c0 += NT) {
      const int j = start + c0 + tid;
      if ((c0 + tid) >= count || j >= N) continue;
      float x[3] = {st.x[j], st.x[(size_t)N + j], st.x[2 * (size_t)N + j]};
      Stencil S;
      if (!stencil_setup(x, P, S)) continue;   // reported by the G2P adjoint
      int lv[3] = {S.base[0] - (ox - 1), S.base[1] - (oy - 1), S.base[2] - (oz - 1)};
      if (lv[0] < 0 || lv[1] < 0 || lv[2] < 0 || lv[0] > VT - 3 || lv[1] > VT - 3 || lv[2] > VT - 3) continue;
      if (!p2g_adj_particle<false, VT>(A, P, st, s_g, lv, S, j)) {
        const uint32_t r = atomicAdd(A.redo_n, 1u);
        A.redo[r] = make_uint2((uint32_t)j, (uint32_t)ent.x);
      }
    }
    __syncthreads();
  }
}

// The FP64 pass of the P2G adjoint over the solids k_p2g_adj_tiled listed:
// each thread stages its particle's 27 stencil nodes in LDS.
__global__ __launch_bounds__(REDO_NT) void k_p2g_adj_redo(AdjArgs A, StepParams P, FastGeom g) {
  __shared__ float4 s_loc[REDO_NT * 27];
  float4* loc = s_loc + threadIdx.x * 27;
  const int N = A.N;
  const PState st = packed_state(A.st.f, N);
  const uint32_t n = A.redo_n[0];
  for (uint32_t e = blockIdx.x * REDO_NT + threadIdx.x; e < n; e += gridDim.x * REDO_NT) {
    const uint2 r = A.redo[e];
    const int j = (int)r.x;
    int sc, bx, by, bz;
    key_decode(g, r.y, sc, bx, by, bz);
    float x[3] = {st.x[j], st.x[(size_t)N + j], st.x[2 * (size_t)N + j]};
    Stencil S;
    stencil_setup(x, P, S);   // inside the grid and the block's tile: checked when listed
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
      for (int jj = 0; jj < 3; jj++)
#pragma unroll
        for (int k = 0; k < 3; k++)
          loc[(i * 3 + jj) * 3 + k] = stage_node(A.mmvb, g, sc, S.base[0] + i, S.base[1] + jj, S.base[2] + k);
    const int l0[3] = {0, 0, 0};
    p2g_adj_particle<true, 3>(A, P, st, loc, l0, S, j);
  }
}

// state adjoint rows from sorted order to user order, as a gather:
// k_adj_pos records the sorted row of every user index (one scattered word
// per particle), then every row is read through it and written in order
__global__ __launch_bounds__(256) void k_adj_pos(const uint32_t* __restrict__ id, int N, uint32_t* __restrict__ pos) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const uint32_t p = id[j];
  if (p < (uint32_t)N) pos[p] = (uint32_t)j;
}
__global__ __launch_bounds__(256) void k_adj_gather(const float* __restrict__ in, float* __restrict__ out,
                                                    const uint32_t* __restrict__ pos, int N) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const uint32_t j = pos[p];
  if (j >= (uint32_t)N) return;
#pragma unroll
  for (int k = 0; k < STATE_FLOATS; k++) out[k * (size_t)N + p] = in[k * (size_t)N + j];
}

static inline unsigned nblk(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

void launch_g2p_adj_tiled(const AdjArgs& A, const StepParams& P, const FastGeom& g, int n_wgs, hipStream_t s) {
  k_g2p_adj_tiled<256><<<n_wgs, 256, 0, s>>>(A, P, g);
  k_g2p_adj_redo<<<REDO_WGS, REDO_NT, 0, s>>>(A, P, g);
}
void launch_grid_adj_tiled(const AdjArgs& A, const StepParams& P, const FastGeom& g, int n_wgs, const double* pose_t,
                           const float* act_t, double* acc_t, hipStream_t s) {
  k_grid_adj_tiled<<<n_wgs, 256, 0, s>>>(A, P, g, pose_t, act_t, acc_t);
}
void launch_p2g_adj_tiled(const AdjArgs& A, const StepParams& P, const FastGeom& g, int n_wgs, hipStream_t s) {
  k_p2g_adj_tiled<256><<<n_wgs, 256, 0, s>>>(A, P, g);
  k_p2g_adj_redo<<<REDO_WGS, REDO_NT, 0, s>>>(A, P, g);
}
__global__ __launch_bounds__(256) void k_row_map(const uint32_t* __restrict__ prev_id, const uint32_t* __restrict__ pos,
                                                 int N, uint32_t* __restrict__ map) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const uint32_t p = prev_id[j];
  map[j] = p < (uint32_t)N ? pos[p] : 0xffffffffu;
}

void launch_row_map(const uint32_t* prev_id, const uint32_t* cur_id, int N, uint32_t* pos, uint32_t* map,
                    hipStream_t s) {
  k_adj_pos<<<nblk(N, 256), 256, 0, s>>>(cur_id, N, pos);
  k_row_map<<<nblk(N, 256), 256, 0, s>>>(prev_id, pos, N, map);
}

__global__ __launch_bounds__(256) void k_copy_list(const int4* __restrict__ src, const uint32_t* __restrict__ src_n,
                                                   int4* __restrict__ dst, uint32_t* __restrict__ dst_n) {
  const uint32_t n = src_n[0];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) dst_n[0] = n;
}

void launch_copy_list(const int4* src, const uint32_t* src_n, int4* dst, uint32_t* dst_n, hipStream_t s) {
  k_copy_list<<<16, 256, 0, s>>>(src, src_n, dst, dst_n);
}

void launch_adj_reorder(const float* in, float* out, const uint32_t* id, int N, uint32_t* pos, hipStream_t s) {
  k_adj_pos<<<nblk(N, 256), 256, 0, s>>>(id, N, pos);
  k_adj_gather<<<nblk(N, 256), 256, 0, s>>>(in, out, pos, N);
}

}  // namespace mpm
