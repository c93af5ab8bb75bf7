// Tiled forward path of the MLS-MPM step for gfx950.
//
// Per step (after an import that sorts the particles by grid block):
//   k_particles<FUSED>  one workgroup per occupied 4^3 block of the sorted
//                       buffer: G2P of the previous step from an LDS copy of
//                       the grid velocities, particle update, stress, then
//                       P2G of this step into a 10^3-node LDS tile with LDS
//                       atomics; the tile's non-zero box goes to global
//                       memory (no global float atomics).  Each particle is
//                       written to its slot in the other buffer, which is
//                       sorted by the block key of the previous position, and
//                       the key of its new position is counted.
//   k_grid              one wavefront per active block: sum the overlapping
//                       tiles of the 27 neighbouring blocks, then normalise,
//                       gravity, soft cylinder contact, slip walls.
//   k_scan              exclusive scan of the key counts -> destination
//                       offsets and the list of occupied blocks.
// The particle order therefore lags the positions by one step: a particle's
// new stencil lies within 2 cells of its block, which the 10^3 tile covers
// (a displacement of more than one cell per step is reported as
// MPM_ERR_TILE, the CFL > 1 condition).
#include <hip/hip_runtime.h>
#include <math.h>
#include "mpm_fast.h"
#include "mpm_math.h"
#include "mpm_phys.h"

namespace mpm {

namespace {

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ __device__ inline uint32_t spread3(uint32_t v) {
  v &= 0x3ff;
  v = (v | (v << 16)) & 0x030000FF;
  v = (v | (v << 8)) & 0x0300F00F;
  v = (v | (v << 4)) & 0x030C30C3;
  v = (v | (v << 2)) & 0x09249249;
  return v;
}
__host__ __device__ inline uint32_t compact3(uint32_t v) {
  v &= 0x09249249;
  v = (v | (v >> 2)) & 0x030C30C3;
  v = (v | (v >> 4)) & 0x0300F00F;
  v = (v | (v >> 8)) & 0x030000FF;
  v = (v | (v >> 16)) & 0x000003FF;
  return v;
}
__device__ inline uint32_t block_key(const FastGeom& g, int s, int bx, int by, int bz) {
  return ((uint32_t)s << (3 * g.kb)) | (spread3(bx) << 2) | (spread3(by) << 1) | spread3(bz);
}
__device__ inline void key_decode(const FastGeom& g, uint32_t key, int& s, int& bx, int& by, int& bz) {
  s = (int)(key >> (3 * g.kb));
  uint32_t m = key & ((1u << (3 * g.kb)) - 1u);
  bx = (int)compact3(m >> 2);
  by = (int)compact3(m >> 1);
  bz = (int)compact3(m);
}

// Rank of each lane's key among equal keys, with one global atomic per
// distinct key of the wavefront.  Every lane of the wave must call it.
__device__ inline uint32_t wave_rank(uint32_t* counts, uint32_t key, bool valid) {
  const int lane = __lane_id();
  unsigned long long pending = __ballot(valid);
  uint32_t myrank = 0;
  while (pending) {
    int leader = __ffsll((long long)pending) - 1;
    uint32_t k = __shfl(key, leader);
    unsigned long long m = __ballot(valid && key == k) & pending;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&counts[k], (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    if ((m >> lane) & 1ull) myrank = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
    pending &= ~m;
  }
  return myrank;
}

__device__ inline void load_state(const PBuf& b, int N, int j, float* x, float* v, float* C, float* F, float& J) {
#pragma unroll
  for (int a = 0; a < 3; a++) { x[a] = b.f[a * (size_t)N + j]; v[a] = b.f[(3 + a) * (size_t)N + j]; }
#pragma unroll
  for (int k = 0; k < 9; k++) C[k] = b.f[(6 + k) * (size_t)N + j];
}

}  // namespace

// ---------------------------------------------------------------------------
// import: block key and rank of every particle (user order)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_import_keys(PState u, StepParams P, FastGeom g, uint32_t* __restrict__ counts,
                                                     uint32_t* __restrict__ key_tmp, uint32_t* __restrict__ rank_tmp) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  bool has = p < u.N;
  uint32_t key = 0;
  if (has) {
    const int N = u.N;
    float x[3] = {u.x[p], u.x[N + p], u.x[2 * N + p]};
    Stencil S;
    if (!stencil_setup(x, P, S)) {
      atomicOr(P.err, ERR_OUTSIDE);
    } else {
      key = block_key(g, P.pscene[p], S.base[0] >> 2, S.base[1] >> 2, S.base[2] >> 2);
    }
  }
  uint32_t r = wave_rank(counts, key, has);
  if (has) { key_tmp[p] = key; rank_tmp[p] = r; }
}

// exclusive scan of counts -> offsets, compact list of occupied keys, zero
// counts; resets the NSUB active-list counters the next step appends to and
// advances the step stamp.  One workgroup; each thread owns a contiguous
// range of keys read and written with 16-byte vector accesses.
__global__ __launch_bounds__(1024) void k_scan(uint32_t* __restrict__ counts, uint32_t* __restrict__ offsets,
                                               int4* __restrict__ list, uint32_t* __restrict__ list_n, int n_keys,
                                               uint32_t* __restrict__ active_n_reset, uint32_t* __restrict__ gen) {
  __shared__ uint32_t s_sum[1024], s_nz[1024];
  const int t = threadIdx.x;
  const int per = ((n_keys + 1023) / 1024 + 3) & ~3;       // multiple of 4
  const int k0 = t * per;
  uint32_t sum = 0, nz = 0;
  for (int b = 0; b < per; b += 32) {
    uint4 v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      int k = k0 + b + 4 * u;
      v[u] = (b + 4 * u < per && k + 3 < n_keys) ? *(const uint4*)(counts + k) : make_uint4(0, 0, 0, 0);
      if (b + 4 * u < per && k < n_keys && k + 3 >= n_keys) {
        v[u].x = counts[k];
        v[u].y = k + 1 < n_keys ? counts[k + 1] : 0;
        v[u].z = k + 2 < n_keys ? counts[k + 2] : 0;
      }
    }
#pragma unroll
    for (int u = 0; u < 8; u++) {
      sum += v[u].x + v[u].y + v[u].z + v[u].w;
      nz += (v[u].x > 0) + (v[u].y > 0) + (v[u].z > 0) + (v[u].w > 0);
    }
  }
  s_sum[t] = sum;
  s_nz[t] = nz;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t a = (t >= off) ? s_sum[t - off] : 0, b = (t >= off) ? s_nz[t - off] : 0;
    __syncthreads();
    s_sum[t] += a;
    s_nz[t] += b;
    __syncthreads();
  }
  uint32_t run = s_sum[t] - sum, li = s_nz[t] - nz;
  for (int b = 0; b < per; b += 4) {
    int k = k0 + b;
    if (k >= n_keys) break;
    uint32_t c[4], o[4];
    bool full = k + 3 < n_keys;
    if (full) { uint4 v = *(const uint4*)(counts + k); c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w; }
    else {
#pragma unroll
      for (int u = 0; u < 4; u++) c[u] = (k + u < n_keys) ? counts[k + u] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      o[u] = run;
      if (c[u] > 0) { list[li] = make_int4(k + u, (int)run, (int)c[u], 0); li++; }
      run += c[u];
    }
    if (full) {
      *(uint4*)(offsets + k) = make_uint4(o[0], o[1], o[2], o[3]);
      *(uint4*)(counts + k) = make_uint4(0, 0, 0, 0);
    } else {
#pragma unroll
      for (int u = 0; u < 4; u++)
        if (k + u < n_keys) { offsets[k + u] = o[u]; counts[k + u] = 0; }
    }
  }
  if (t < NSUB && active_n_reset) active_n_reset[t] = 0;
  if (t == 1023) {
    list_n[0] = s_nz[1023];
    if (gen) gen[0] = gen[0] + 1;
  }
}

__global__ void k_bookkeep(uint32_t* active_n_reset, uint32_t* gen) {
  if (threadIdx.x < NSUB) active_n_reset[threadIdx.x] = 0;
  if (threadIdx.x == 0) gen[0] = gen[0] + 1;
}

// scatter the user-order particles to their sorted slots
__global__ __launch_bounds__(256) void k_permute(PState u, const uint8_t* __restrict__ umat, PBuf X,
                                                 const uint32_t* __restrict__ key_tmp, const uint32_t* __restrict__ rank_tmp,
                                                 const uint32_t* __restrict__ offsets) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= u.N) return;
  const int N = u.N;
  uint32_t key = key_tmp[p], r = rank_tmp[p];
  uint32_t d = offsets[key] + r;
  if (d >= (uint32_t)N) return;
#pragma unroll
  for (int a = 0; a < 3; a++) { X.f[a * (size_t)N + d] = u.x[a * N + p]; X.f[(3 + a) * (size_t)N + d] = u.v[a * N + p]; }
#pragma unroll
  for (int k = 0; k < 9; k++) { X.f[(6 + k) * (size_t)N + d] = u.C[k * N + p]; X.f[(15 + k) * (size_t)N + d] = u.F[k * N + p]; }
  X.f[24 * (size_t)N + d] = u.J[p];
  X.id[d] = (uint32_t)p;
  X.key[d] = key;
  X.rank[d] = r;
  X.mat[d] = umat[p];
}

// scatter the sorted buffer back to the user arrays; liquids keep the user's
// F and solids the user's J (those rows are not carried by the kernels)
__global__ __launch_bounds__(256) void k_export(PBuf X, PState u, const MatDev* __restrict__ mats) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= u.N) return;
  const int N = u.N;
  uint32_t p = X.id[j];
  if (p >= (uint32_t)N) return;
#pragma unroll
  for (int a = 0; a < 3; a++) { u.x[a * N + p] = X.f[a * (size_t)N + j]; u.v[a * N + p] = X.f[(3 + a) * (size_t)N + j]; }
#pragma unroll
  for (int k = 0; k < 9; k++) u.C[k * N + p] = X.f[(6 + k) * (size_t)N + j];
  if (mats[X.mat[j]].kind == KIND_LIQUID) {
    u.J[p] = X.f[24 * (size_t)N + j];
  } else {
#pragma unroll
    for (int k = 0; k < 9; k++) u.F[k * N + p] = X.f[(15 + k) * (size_t)N + j];
  }
}

// ---------------------------------------------------------------------------
// particle kernel
// ---------------------------------------------------------------------------
enum { MODE_P2G = 0, MODE_FUSED = 1, MODE_G2P = 2 };

struct PartArgs {
  PBuf in, out;
  int N;
  const int4* list;
  const uint32_t* list_n;
  const uint32_t* offsets;     // destination offsets of the keys stored with `in`
  uint32_t* counts;            // histogram of the new keys
  float* tiles;
  int2* tile_box;
  uint32_t* active_stamp;
  uint32_t* active;            // active sub-lists appended this step: NSUB x n_keys
  uint32_t* active_n;          // NSUB counters
  int n_keys;
  const uint32_t* gen;
  const float4* vgrid;
};

template <int MODE>
__global__ __launch_bounds__(256) void k_particles(PartArgs A, StepParams P, FastGeom g) {
  __shared__ float s_tile[4 * TILE_NODES];
  __shared__ int s_itile[4 * TILE_NODES];
  __shared__ float4 s_v[VT_NODES];
  __shared__ int s_lo[3], s_hi[3];
  __shared__ float s_red[16], s_scale[8];
  __shared__ int s_ired[32];
  const int tid = threadIdx.x;
  const int N = A.N;
  const uint32_t n_list = A.list_n[0];
  const uint32_t stamp = A.gen[0];
  for (uint32_t e = blockIdx.x; e < n_list; e += gridDim.x) {
    const int4 ent = A.list[e];
    int sc, bx, by, bz;
    key_decode(g, (uint32_t)ent.x, sc, bx, by, bz);
    const int ox = 4 * bx, oy = 4 * by, oz = 4 * bz;
    // ---- stage grid velocities of nodes [4b-1, 4b+7) for G2P
    if (MODE != MODE_P2G) {
      for (int q = tid; q < VT_NODES; q += 256) {
        int qi = q / (VT * VT), qj = (q / VT) % VT, qk = q % VT;
        int gx = ox - 1 + qi, gy = oy - 1 + qj, gz = oz - 1 + qk;
        float4 val = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gx >= 0 && gy >= 0 && gz >= 0 && gx < g.n && gy < g.n && gz < g.n) {
          uint32_t kk = block_key(g, sc, gx >> 2, gy >> 2, gz >> 2);
          val = A.vgrid[(size_t)kk * 64 + (((gx & 3) << 4) | ((gy & 3) << 2) | (gz & 3))];
        }
        s_v[q] = val;
      }
    }
    if (MODE != MODE_G2P) {
      for (int q = tid; q < 4 * TILE_NODES; q += 256) { s_tile[q] = 0.f; s_itile[q] = 0; }
      if (tid < 3) { s_lo[tid] = 1 << 20; s_hi[tid] = -(1 << 20); }
    }
    __syncthreads();
    const int start = ent.y, count = ent.z;
    for (int c0 = 0; c0 < count; c0 += 256) {
      const int j = start + c0 + tid;
      const bool has = (c0 + tid) < count && j < N;
      float x[3] = {0, 0, 0}, v[3] = {0, 0, 0}, C[9], F[9], J = 1.f;
      int m = 0;
      bool ok = has;
      uint32_t dst = 0;
      if (has) {
        load_state(A.in, N, j, x, v, C, F, J);
        m = A.in.mat[j];
      }
      const MatDev& M = P.mats[m];
      const bool liquid = M.kind == KIND_LIQUID;
      if (has) {
        if (liquid) J = A.in.f[24 * (size_t)N + j];
        else {
#pragma unroll
          for (int k = 0; k < 9; k++) F[k] = A.in.f[(15 + k) * (size_t)N + j];
        }
      }
      float tau[9];
      bool have_tau = false;
      // ---------------- G2P of the previous step ----------------
      if (MODE != MODE_P2G && has) {
        Stencil S;
        bool in_grid = stencil_setup(x, P, S);
        int lb[3] = {S.base[0] - (ox - 1), S.base[1] - (oy - 1), S.base[2] - (oz - 1)};
        bool in_tile = lb[0] >= 0 && lb[1] >= 0 && lb[2] >= 0 && lb[0] <= VT - 3 && lb[1] <= VT - 3 && lb[2] <= VT - 3;
        if (!in_grid) { atomicOr(P.err, ERR_OUTSIDE); ok = false; }
        else if (!in_tile) { atomicOr(P.err, ERR_TILE); ok = false; }
        if (ok) {
          float vn[3] = {0, 0, 0}, B[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
          for (int i = 0; i < 3; i++)
#pragma unroll
            for (int jj = 0; jj < 3; jj++)
#pragma unroll
              for (int k = 0; k < 3; k++) {
                float w = S.w[0][i] * S.w[1][jj] * S.w[2][k];
                float d[3] = {(i - S.f[0]) * P.dx, (jj - S.f[1]) * P.dx, (k - S.f[2]) * P.dx};
                float4 gv4 = s_v[((lb[0] + i) * VT + lb[1] + jj) * VT + lb[2] + k];
                float gv[3] = {w * gv4.x, w * gv4.y, w * gv4.z};
#pragma unroll
                for (int a = 0; a < 3; a++) {
                  vn[a] += gv[a];
#pragma unroll
                  for (int b = 0; b < 3; b++) B[a * 3 + b] += gv[a] * d[b];
                }
              }
          // particle update (+ stress of the new state for the fused mode)
          const float d4 = 4.f * P.inv_dx * P.inv_dx;
          float Md[9];
#pragma unroll
          for (int k = 0; k < 9; k++) { C[k] = d4 * B[k]; Md[k] = P.dt * C[k] + ((k % 4 == 0) ? 1.f : 0.f); }
#pragma unroll
          for (int a = 0; a < 3; a++) { x[a] += P.dt * vn[a]; v[a] = vn[a]; }
          bool fin = isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]) && isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
          if (liquid) {
            J = J * det3(Md);
            fin = fin && isfinite(J);
          } else if (M.kind == KIND_ELASTIC) {
            float Fn[9];
            matmul(Md, F, Fn);
#pragma unroll
            for (int k = 0; k < 9; k++) F[k] = Fn[k];
          } else {
            double Mdd[9], Fd[9], Ft[9], Uu[9], s[3], V[9];
#pragma unroll
            for (int k = 0; k < 9; k++) { Mdd[k] = Md[k]; Fd[k] = F[k]; }
            matmul(Mdd, Fd, Ft);
            svd3(Ft, Uu, s, V);
            if (!(s[2] > 0.0)) {
              atomicOr(P.err, ERR_SAND_SIGMA);
              ok = false;
#pragma unroll
              for (int k = 0; k < 9; k++) F[k] = (float)Ft[k];
            } else {
              double e[3] = {log(s[0]), log(s[1]), log(s[2])}, ep[3];
              DPInfo I;
              dp_project(e, M, ep, I);
              double gg[3], Fo[9];
              if (I.cse == 0) {
#pragma unroll
                for (int k = 0; k < 9; k++) F[k] = (float)Ft[k];
              } else {
#pragma unroll
                for (int a = 0; a < 3; a++) gg[a] = exp(ep[a]);
                usv(Uu, gg, V, Fo);
#pragma unroll
                for (int k = 0; k < 9; k++) F[k] = (float)Fo[k];
              }
              if (MODE == MODE_FUSED) {
                // Hencky stress of the projected state from the same SVD
                double tr = ep[0] + ep[1] + ep[2];
                double h[3];
#pragma unroll
                for (int a = 0; a < 3; a++) h[a] = 2.0 * (double)M.mu * ep[a] + (double)M.lam * tr;
#pragma unroll
                for (int i = 0; i < 3; i++)
#pragma unroll
                  for (int jj = 0; jj < 3; jj++)
                    tau[i * 3 + jj] = (float)(Uu[i * 3] * h[0] * Uu[jj * 3] + Uu[i * 3 + 1] * h[1] * Uu[jj * 3 + 1] +
                                              Uu[i * 3 + 2] * h[2] * Uu[jj * 3 + 2]);
                have_tau = true;
              }
            }
          }
          if (!liquid) {
#pragma unroll
            for (int k = 0; k < 9; k++) fin = fin && isfinite(F[k]);
          }
#pragma unroll
          for (int k = 0; k < 9; k++) fin = fin && isfinite(C[k]);
          if (!fin) { atomicOr(P.err, ERR_NONFINITE); ok = false; }
        }
        // write the particle to its slot in the output buffer
        dst = A.offsets[A.in.key[j]] + A.in.rank[j];
        if (dst < (uint32_t)N) {
          PBuf& O = A.out;
#pragma unroll
          for (int a = 0; a < 3; a++) { O.f[a * (size_t)N + dst] = x[a]; O.f[(3 + a) * (size_t)N + dst] = v[a]; }
#pragma unroll
          for (int k = 0; k < 9; k++) O.f[(6 + k) * (size_t)N + dst] = C[k];
          if (liquid) O.f[24 * (size_t)N + dst] = J;
          else {
#pragma unroll
            for (int k = 0; k < 9; k++) O.f[(15 + k) * (size_t)N + dst] = F[k];
          }
          O.id[dst] = A.in.id[j];
          O.mat[dst] = (uint8_t)m;
        } else {
          ok = false;
        }
      }
      // ---------------- P2G of this step ----------------
      // LDS float atomics are slow on gfx950 (about 1/30 of the integer
      // rate), so each 256-particle chunk accumulates in exact 32-bit fixed
      // point: a power-of-two scale per quantity, chosen from a bound on the
      // chunk's contributions so that no node sum can overflow, then the
      // integer tile is flushed into the float tile by its owner threads.
      uint32_t nkey = 0;
      bool counted = false;
      if (MODE != MODE_G2P) {
        Stencil S;
        int lb[3] = {0, 0, 0};
        if (ok) {
          bool in_grid = stencil_setup(x, P, S);
          lb[0] = S.base[0] - (ox - 2); lb[1] = S.base[1] - (oy - 2); lb[2] = S.base[2] - (oz - 2);
          bool in_tile = lb[0] >= 0 && lb[1] >= 0 && lb[2] >= 0 && lb[0] <= TILE - 3 && lb[1] <= TILE - 3 && lb[2] <= TILE - 3;
          if (!in_grid) { atomicOr(P.err, ERR_OUTSIDE); ok = false; }
          else if (!in_tile) { atomicOr(P.err, ERR_TILE); ok = false; }
        }
        float Am[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, mvp[3] = {0, 0, 0}, bnd[4] = {0, 0, 0, 0};
        if (ok) {
          if (liquid) stress_liquid(J, C, M, tau);
          else if (!have_tau && !stress_solid(F, M, tau)) atomicOr(P.err, ERR_SAND_SIGMA);
          const float scl = -P.dt * M.vol * 4.f * P.inv_dx * P.inv_dx;
#pragma unroll
          for (int k = 0; k < 9; k++) Am[k] = scl * tau[k] + M.mass * C[k];
#pragma unroll
          for (int a = 0; a < 3; a++) {
            mvp[a] = M.mass * v[a];
            bnd[1 + a] = fabsf(mvp[a]) + 1.5f * P.dx * (fabsf(Am[a * 3]) + fabsf(Am[a * 3 + 1]) + fabsf(Am[a * 3 + 2]));
          }
          bnd[0] = M.mass;
          if (!isfinite(bnd[1] + bnd[2] + bnd[3])) {
            // a non-finite velocity or stress must not reach the integer tile
            atomicOr(P.err, ERR_NONFINITE);
            ok = false;
#pragma unroll
            for (int q = 0; q < 4; q++) bnd[q] = 0.f;
          } else {
            nkey = block_key(g, sc, S.base[0] >> 2, S.base[1] >> 2, S.base[2] >> 2);
            counted = true;
          }
        }
        // chunk-wide bound sums and box (wave shuffles, then 4 waves in LDS)
        int clo[3], chi[3];
#pragma unroll
        for (int a = 0; a < 3; a++) { clo[a] = ok ? lb[a] : 1 << 20; chi[a] = ok ? lb[a] : -(1 << 20); }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
          for (int q = 0; q < 4; q++) bnd[q] += __shfl_xor(bnd[q], off);
#pragma unroll
          for (int a = 0; a < 3; a++) { clo[a] = min(clo[a], __shfl_xor(clo[a], off)); chi[a] = max(chi[a], __shfl_xor(chi[a], off)); }
        }
        const int wv = tid >> 6;
        if ((tid & 63) == 0) {
#pragma unroll
          for (int q = 0; q < 4; q++) s_red[wv * 4 + q] = bnd[q];
#pragma unroll
          for (int a = 0; a < 3; a++) { s_ired[wv * 6 + a] = clo[a]; s_ired[wv * 6 + 3 + a] = chi[a]; }
        }
        __syncthreads();
        if (tid == 0) {
#pragma unroll
          for (int q = 0; q < 4; q++) {
            float T = 0.421875f * (s_red[q] + s_red[4 + q] + s_red[8 + q] + s_red[12 + q]);
            if (!isfinite(T)) { atomicOr(P.err, ERR_NONFINITE); T = 1.f; }
            int e = 0;
            frexpf(T > 0.f ? T : 1.f, &e);
            e = max(e, -90);
            s_scale[q] = ldexpf(1.f, 30 - e);
            s_scale[4 + q] = ldexpf(1.f, e - 30);
          }
#pragma unroll
          for (int a = 0; a < 3; a++) {
            int lo = min(min(s_ired[a], s_ired[6 + a]), min(s_ired[12 + a], s_ired[18 + a]));
            int hi = max(max(s_ired[3 + a], s_ired[9 + a]), max(s_ired[15 + a], s_ired[21 + a]));
            s_ired[24 + a] = lo;
            s_ired[27 + a] = hi;
            if (lo <= hi) { s_lo[a] = min(s_lo[a], lo); s_hi[a] = max(s_hi[a], hi); }
          }
        }
        __syncthreads();
        if (ok) {
          const float sm = s_scale[0], sx = s_scale[1], sy = s_scale[2], sz = s_scale[3];
#pragma unroll
          for (int i = 0; i < 3; i++)
#pragma unroll
            for (int jj = 0; jj < 3; jj++)
#pragma unroll
              for (int k = 0; k < 3; k++) {
                float w = S.w[0][i] * S.w[1][jj] * S.w[2][k];
                float d0 = (i - S.f[0]) * P.dx, d1 = (jj - S.f[1]) * P.dx, d2 = (k - S.f[2]) * P.dx;
                int q = ((lb[0] + i) * TILE + lb[1] + jj) * TILE + lb[2] + k;
                atomicAdd(&s_itile[q], __float2int_rn(w * M.mass * sm));
                atomicAdd(&s_itile[TILE_NODES + q], __float2int_rn(w * (mvp[0] + Am[0] * d0 + Am[1] * d1 + Am[2] * d2) * sx));
                atomicAdd(&s_itile[2 * TILE_NODES + q], __float2int_rn(w * (mvp[1] + Am[3] * d0 + Am[4] * d1 + Am[5] * d2) * sy));
                atomicAdd(&s_itile[3 * TILE_NODES + q], __float2int_rn(w * (mvp[2] + Am[6] * d0 + Am[7] * d1 + Am[8] * d2) * sz));
              }
        }
        __syncthreads();
        {
          // flush the chunk's box into the float tile and clear the integers
          const int lo0 = s_ired[24], lo1 = s_ired[25], lo2 = s_ired[26];
          const int hi0 = s_ired[27], hi1 = s_ired[28], hi2 = s_ired[29];
          if (lo0 <= hi0) {
            const int ex = hi0 - lo0 + 3, ey = hi1 - lo1 + 3, ez = hi2 - lo2 + 3;
            const int cnt = ex * ey * ez;
            for (int r = tid; r < cnt; r += 256) {
              int qq = ((lo0 + r / (ey * ez)) * TILE + lo1 + (r / ez) % ey) * TILE + lo2 + r % ez;
#pragma unroll
              for (int c = 0; c < 4; c++) {
                int iv = s_itile[c * TILE_NODES + qq];
                if (iv != 0) {
                  s_tile[c * TILE_NODES + qq] += (float)iv * s_scale[4 + c];
                  s_itile[c * TILE_NODES + qq] = 0;
                }
              }
            }
          }
        }
        __syncthreads();
        if (MODE == MODE_FUSED) {
          uint32_t r = wave_rank(A.counts, nkey, counted && has);
          if (has && dst < (uint32_t)N) { A.out.key[dst] = nkey; A.out.rank[dst] = counted ? r : 0u; }
          // a particle that could not be counted keeps a valid (key 0) slot
          if (has && !counted && dst < (uint32_t)N) {
            uint32_t r0 = atomicAdd(&A.counts[0], 1u);
            A.out.key[dst] = 0u;
            A.out.rank[dst] = r0;
          }
        }
      }
    }
    __syncthreads();
    if (MODE != MODE_G2P) {
      // ---- publish the tile's non-zero box and mark the blocks it touches
      const int lo0 = s_lo[0], lo1 = s_lo[1], lo2 = s_lo[2];
      const int hi0 = s_hi[0] + 2, hi1 = s_hi[1] + 2, hi2 = s_hi[2] + 2;
      const uint32_t bkey = (uint32_t)ent.x;
      if (lo0 <= hi0 - 2) {
        const int ex = hi0 - lo0 + 1, ey = hi1 - lo1 + 1, ez = hi2 - lo2 + 1;
        const int cnt = ex * ey * ez;
        float* T = A.tiles + (size_t)bkey * 4 * TILE_NODES;
        for (int r = tid; r < cnt; r += 256) {
          int qi = lo0 + r / (ey * ez), qj = lo1 + (r / ez) % ey, qk = lo2 + r % ez;
          int q = (qi * TILE + qj) * TILE + qk;
#pragma unroll
          for (int c = 0; c < 4; c++) T[c * TILE_NODES + q] = s_tile[c * TILE_NODES + q];
        }
        if (tid == 0) {
          int packed = lo0 | (lo1 << 4) | (lo2 << 8) | (hi0 << 12) | (hi1 << 16) | (hi2 << 20);
          A.tile_box[bkey] = make_int2(packed, (int)stamp);
        }
        if (tid < 27) {
          int dx = tid / 9 - 1, dy = (tid / 3) % 3 - 1, dz = tid % 3 - 1;
          int nbx = bx + dx, nby = by + dy, nbz = bz + dz;
          // node range of that block in tile coordinates: [4 nb - (4b - 2), +3]
          int l0 = 4 * dx + 2, l1 = 4 * dy + 2, l2 = 4 * dz + 2;
          bool hit = nbx >= 0 && nby >= 0 && nbz >= 0 && nbx < g.nb && nby < g.nb && nbz < g.nb &&
                     l0 <= hi0 && l0 + 3 >= lo0 && l1 <= hi1 && l1 + 3 >= lo1 && l2 <= hi2 && l2 + 3 >= lo2;
          if (hit) {
            uint32_t nk = block_key(g, sc, nbx, nby, nbz);
            uint32_t old = atomicExch(&A.active_stamp[nk], stamp);
            if (old != stamp) {
              // spread the appends over NSUB counters to avoid one hot address
              const uint32_t sub = blockIdx.x & (NSUB - 1);
              uint32_t i = atomicAdd(A.active_n + sub, 1u);
              A.active[(size_t)sub * A.n_keys + i] = nk;
            }
          }
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// grid update over active blocks: gather tiles, then the node update
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_grid(StepParams P, FastGeom g, const uint32_t* __restrict__ active,
                                             const uint32_t* __restrict__ active_n, const int2* __restrict__ tile_box,
                                             const float* __restrict__ tiles, const uint32_t* __restrict__ gen,
                                             float4* __restrict__ vgrid, const double* __restrict__ pose_t,
                                             const float* __restrict__ act_t) {
  __shared__ uint32_t s_pre[NSUB + 1];
  const int lane = threadIdx.x;
  // prefix over the sub-list counters (NSUB == 64 == one wavefront)
  uint32_t cnt = active_n[lane];
  uint32_t inc = cnt;
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t o = __shfl_up(inc, off);
    if (lane >= off) inc += o;
  }
  s_pre[lane + 1] = inc;
  if (lane == 0) s_pre[0] = 0;
  __syncthreads();
  const uint32_t n_act = s_pre[NSUB];
  const uint32_t stamp = gen[0];
  const int li = lane >> 4, lj = (lane >> 2) & 3, lk = lane & 3;
  for (uint32_t e = blockIdx.x; e < n_act; e += gridDim.x) {
    int sub = 0;
    while (sub < NSUB - 1 && s_pre[sub + 1] <= e) sub++;
    const uint32_t key = active[(size_t)sub * g.n_keys + (e - s_pre[sub])];
    int sc, bx, by, bz;
    key_decode(g, key, sc, bx, by, bz);
    const int gx = 4 * bx + li, gy = 4 * by + lj, gz = 4 * bz + lk;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 1
    for (int d = 0; d < 27; d++) {
      int sx = bx + d / 9 - 1, sy = by + (d / 3) % 3 - 1, sz = bz + d % 3 - 1;
      if (sx < 0 || sy < 0 || sz < 0 || sx >= g.nb || sy >= g.nb || sz >= g.nb) continue;
      uint32_t sk = block_key(g, sc, sx, sy, sz);
      int2 box = tile_box[sk];
      if ((uint32_t)box.y != stamp) continue;
      int qi = gx - (4 * sx - 2), qj = gy - (4 * sy - 2), qk = gz - (4 * sz - 2);
      int lo0 = box.x & 15, lo1 = (box.x >> 4) & 15, lo2 = (box.x >> 8) & 15;
      int hi0 = (box.x >> 12) & 15, hi1 = (box.x >> 16) & 15, hi2 = (box.x >> 20) & 15;
      if (qi < lo0 || qi > hi0 || qj < lo1 || qj > hi1 || qk < lo2 || qk > hi2) continue;
      int q = (qi * TILE + qj) * TILE + qk;
      const float* T = tiles + (size_t)sk * 4 * TILE_NODES;
      acc.w += T[q];
      acc.x += T[TILE_NODES + q];
      acc.y += T[2 * TILE_NODES + q];
      acc.z += T[3 * TILE_NODES + q];
    }
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
    if (acc.w > 0.f && gx < g.n && gy < g.n && gz < g.n) {
      int idx[3] = {gx, gy, gz};
      float vv[3];
      grid_node_forward(P, sc, idx, acc, pose_t, act_t, vv, nullptr);
      out = make_float4(vv[0], vv[1], vv[2], acc.w);
    }
    vgrid[(size_t)key * 64 + lane] = out;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static FastGeom make_geom(int n_grid, int S) {
  FastGeom g;
  g.n = n_grid;
  g.nb = (n_grid + 3) / 4;
  g.kb = 0;
  while ((1 << g.kb) < g.nb) g.kb++;
  g.S = S;
  g.n_keys = S << (3 * g.kb);
  return g;
}

struct FastLayout {
  size_t buf_f[2], buf_id[2], buf_key[2], buf_rank[2], buf_mat[2];
  size_t key_tmp, rank_tmp, counts, offsets, list[2], list_n, active[2], active_n, active_stamp, tile_box, tiles, vgrid, gen;
  size_t total;
};

static FastLayout fast_plan(int n_grid, int S, int N) {
  FastGeom g = make_geom(n_grid, S);
  FastLayout L;
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o += a256(b); return r; };
  for (int b = 0; b < 2; b++) {
    L.buf_f[b] = take((size_t)STATE_FLOATS * N * 4);
    L.buf_id[b] = take((size_t)N * 4);
    L.buf_key[b] = take((size_t)N * 4);
    L.buf_rank[b] = take((size_t)N * 4);
    L.buf_mat[b] = take((size_t)N);
  }
  L.key_tmp = take((size_t)N * 4);
  L.rank_tmp = take((size_t)N * 4);
  L.counts = take((size_t)g.n_keys * 4);
  L.offsets = take((size_t)g.n_keys * 4);
  L.list[0] = take((size_t)g.n_keys * 16);
  L.list[1] = take((size_t)g.n_keys * 16);
  L.list_n = take(16);
  L.active[0] = take((size_t)g.n_keys * 4 * NSUB);
  L.active[1] = take((size_t)g.n_keys * 4 * NSUB);
  L.active_n = take(2 * NSUB * 4);
  L.active_stamp = take((size_t)g.n_keys * 4);
  L.tile_box = take((size_t)g.n_keys * 8);
  L.tiles = take((size_t)g.n_keys * 4 * TILE_NODES * 4);
  L.vgrid = take((size_t)g.n_keys * 64 * 16);
  L.gen = take(16);
  L.total = o;
  return L;
}

size_t fast_workspace_bytes(int n_grid, int n_scenes, int N) { return fast_plan(n_grid, n_scenes, N).total; }

static inline unsigned nblk(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

int fast_init(FastPath& f, char* ws, int n_grid, int n_scenes, int N, hipStream_t s) {
  FastLayout L = fast_plan(n_grid, n_scenes, N);
  f.ws = ws;
  f.g = make_geom(n_grid, n_scenes);
  f.N = N;
  for (int b = 0; b < 2; b++) {
    f.buf[b].f = (float*)(ws + L.buf_f[b]);
    f.buf[b].id = (uint32_t*)(ws + L.buf_id[b]);
    f.buf[b].key = (uint32_t*)(ws + L.buf_key[b]);
    f.buf[b].rank = (uint32_t*)(ws + L.buf_rank[b]);
    f.buf[b].mat = (uint8_t*)(ws + L.buf_mat[b]);
    f.list[b] = (int4*)(ws + L.list[b]);
    f.active[b] = (uint32_t*)(ws + L.active[b]);
  }
  f.key_tmp = (uint32_t*)(ws + L.key_tmp);
  f.rank_tmp = (uint32_t*)(ws + L.rank_tmp);
  f.counts = (uint32_t*)(ws + L.counts);
  f.offsets = (uint32_t*)(ws + L.offsets);
  f.list_n = (uint32_t*)(ws + L.list_n);
  f.active_n = (uint32_t*)(ws + L.active_n);
  f.active_stamp = (uint32_t*)(ws + L.active_stamp);
  f.tile_box = (int2*)(ws + L.tile_box);
  f.tiles = (float*)(ws + L.tiles);
  f.vgrid = (float4*)(ws + L.vgrid);
  f.gen = (uint32_t*)(ws + L.gen);
  f.part_wgs = 2048;
  f.grid_wgs = 4096;
  f.valid = false;
  // zero the bookkeeping (counts, stamps, counters, velocity grid)
  launch_zero(ws + L.counts, a256((size_t)f.g.n_keys * 4), s);
  launch_zero(ws + L.list_n, 256, s);
  launch_zero(ws + L.active_n, a256(2 * NSUB * 4), s);
  launch_zero(ws + L.active_stamp, a256((size_t)f.g.n_keys * 4), s);
  launch_zero(ws + L.tile_box, a256((size_t)f.g.n_keys * 8), s);
  launch_zero(ws + L.vgrid, a256((size_t)f.g.n_keys * 64 * 16), s);
  launch_zero(ws + L.gen, 256, s);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

void fast_bind_grid(FastPath& f, float4* mmv, float4* vgrid) { f.mmv = mmv; f.vdense = vgrid; }
void fast_invalidate(FastPath& f) { f.valid = false; }
void fast_destroy(FastPath&) {}

int fast_run(FastPath& f, const StepParams& P, const PState& user, int t0, int n, const double* pose, const float* act,
             hipStream_t s, KernelTimer* timer) {
  const FastGeom g = f.g;
  const int N = f.N;
  const int S = g.S;
  // ---- import: sort the user-order state into buf[0] by block key
  k_import_keys<<<nblk(N, 256), 256, 0, s>>>(user, P, g, f.counts, f.key_tmp, f.rank_tmp);
  k_scan<<<1, 1024, 0, s>>>(f.counts, f.offsets, f.list[0], f.list_n + 0, g.n_keys, f.active_n, f.gen);
  k_permute<<<nblk(N, 256), 256, 0, s>>>(user, P.mat, f.buf[0], f.key_tmp, f.rank_tmp, f.offsets);
  // The particle kernels read the material of the sorted buffer.
  StepParams Q = P;
  PartArgs A;
  A.N = N;
  A.counts = f.counts;
  A.offsets = f.offsets;
  A.tiles = f.tiles;
  A.tile_box = f.tile_box;
  A.active_stamp = f.active_stamp;
  A.gen = f.gen;
  A.vgrid = f.vgrid;
  A.n_keys = g.n_keys;
  // Bookkeeping: `rd` is the list describing buf[cur] (the buffer the next
  // particle kernel reads); `wr` is the list describing the order in which
  // the current offsets place particles (the buffer the next kernel writes).
  int cur = 0, rd = 0, wr = 0;
  for (int step = 0; step <= n; step++) {
    const int t = t0 + step;
    const int ap = step & 1;   // active list of this step
    A.in = f.buf[cur];
    A.out = f.buf[cur ^ 1];
    A.list = f.list[rd];
    A.list_n = f.list_n + rd;
    A.active = f.active[ap];
    A.active_n = f.active_n + ap * NSUB;
    if (step == n) {
      k_particles<MODE_G2P><<<f.part_wgs, 256, 0, s>>>(A, Q, g);
      cur ^= 1;
      break;
    }
    if (step == 0) {
      k_particles<MODE_P2G><<<f.part_wgs, 256, 0, s>>>(A, Q, g);
    } else {
      if (timer) timer->begin(s);
      k_particles<MODE_FUSED><<<f.part_wgs, 256, 0, s>>>(A, Q, g);
      if (timer) timer->end(s);
    }
    k_grid<<<f.grid_wgs, 64, 0, s>>>(Q, g, f.active[ap], f.active_n + ap * NSUB, f.tile_box, f.tiles, f.gen, f.vgrid,
                                      pose + (size_t)t * S * POSE_DOUBLES, act + (size_t)t * S * 6);
    if (step == 0) {
      // nothing counted: keep the import's offsets, advance the stamp and
      // reset the next step's active list
      k_bookkeep<<<1, 64, 0, s>>>(f.active_n + (ap ^ 1) * NSUB, f.gen);
    } else {
      cur ^= 1;
      rd = wr;
      wr = 1 - rd;
      k_scan<<<1, 1024, 0, s>>>(f.counts, f.offsets, f.list[wr], f.list_n + wr, g.n_keys, f.active_n + (ap ^ 1) * NSUB,
                                f.gen);
    }
  }
  k_export<<<nblk(N, 256), 256, 0, s>>>(f.buf[cur], user, P.mats);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace mpm
