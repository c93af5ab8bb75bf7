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
//                       The blocks a tile touches are claimed (first entry
//                       wins) and recorded per entry.
//   k_grid              per occupied-block entry, its claimed blocks: sum
//                       the overlapping tiles of the 27 neighbouring blocks,
//                       then normalise, gravity, soft cylinder contact, walls.
//   k_scan              exclusive scan of the key counts -> destination
//                       offsets and the list of occupied blocks.
// The particle order therefore lags the positions by one step: a particle's
// new stencil lies within 2 cells of its block, which the 10^3 tile covers
// (a displacement of more than one cell per step is reported as
// MPM_ERR_TILE, the CFL > 1 condition).
#include <hip/hip_runtime.h>
#include <math.h>
#include <vector>
#include "mpm_fast.h"
#include "mpm_blocks.h"
#include "mpm_math.h"
#include "mpm_mlp.h"
#include "mpm_phys.h"
#include "mpm_transfer.h"

namespace mpm {

namespace {

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// ---------------------------------------------------------------------------
// import: block key and rank of every particle (user order)
// ---------------------------------------------------------------------------
constexpr int IMPORT_PAD = 16;   // uint32 words between two keys' import counters
__global__ __launch_bounds__(256) void k_import_keys(PState u, StepParams P, FastGeom g, uint32_t* __restrict__ counts,
                                                     uint32_t* __restrict__ key_tmp, uint32_t* __restrict__ rank_tmp,
                                                     uint32_t* __restrict__ touched, uint32_t* __restrict__ n_touched) {
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
  // user order is arbitrary, so the lanes of a wavefront rarely share a key:
  // one atomic per particle into counters padded to one per 64 bytes (packed
  // counters would put hundreds of keys' atomics on a few cache lines); the
  // first reservation of a key appends it to the touched list
  if (has) {
    const uint32_t r = atomicAdd(&counts[(size_t)key * IMPORT_PAD], 1u);
    if (r == 0u) touch_key(key, touched, n_touched, (uint32_t)g.n_keys);
    key_tmp[p] = key;
    rank_tmp[p] = r;
  }
}

// Exclusive scan of the counts of the touched keys -> their offsets, the
// list of occupied keys {key, offset, count, sub}, and the counts and the
// touched counter cleared.  Run by one workgroup of NT threads.  The
// particles of the blocks follow the order in which their keys were first
// touched; only contiguity matters.  With split_nt > 0 a block of more than
// max_chunks chunks of split_nt particles is listed twice, sub 0 with the
// first ceil(chunks / 2) chunks and sub 1 with the rest, so that two
// workgroups share it (each publishes its own tile slot); with fill_slots >
// 0 as well, blocks of two chunks are split too (the first ones in touch
// order, at most one added entry in 16) while the list has fewer entries
// than fill_slots, the particle kernel's resident workgroups.  Entries of
// two or more chunks (of split_nt
// particles, else of order_nt; none if both are 0) are listed before those
// of one: the particle kernels' workgroups are dispatched round-robin over
// the CUs, so each CU then receives about as many chunks as the others, the
// longest first.
template <int NT>
__device__ void scan_touched(uint32_t* __restrict__ counts, uint32_t* __restrict__ offsets,
                             const uint32_t* __restrict__ touched, uint32_t* __restrict__ n_touched,
                             int4* __restrict__ list, uint32_t* __restrict__ list_n, int n_keys, int stride = 1,
                             int split_nt = 0, int max_chunks = 2, int order_nt = 0, int fill_slots = 0) {
  constexpr int NW = NT / 64;
  __shared__ uint32_t s_sum[NW], s_big[NW], s_sm[NW], s_cand[NW];
  __shared__ uint32_t s_run, s_runbig, s_runsm, s_runcand, s_nbig, s_nent, s_ncand;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const uint32_t n = min(n_touched[0], (uint32_t)n_keys);
  // the chunks of a key with c particles, whether it is split by size, and
  // whether it may be split to fill the resident workgroups
  const uint32_t cs = (uint32_t)(split_nt > 0 ? split_nt : order_nt);
  auto chunks = [&](uint32_t c) { return cs > 0 ? (c + cs - 1) / cs : 0u; };
  auto size_split = [&](uint32_t nch) { return split_nt > 0 && nch > (uint32_t)max_chunks; };
  auto fill_candidate = [&](uint32_t nch) { return fill_slots > 0 && split_nt > 0 && nch == 2u && !size_split(nch); };
  // its entries' classes (two or more chunks: big)
  auto classes = [&](uint32_t nch, bool valid, bool sp, uint32_t& ch0, bool& big0, bool& big1) {
    ch0 = sp ? (nch + 1) / 2 : nch;
    big0 = valid && ch0 >= 2u;
    big1 = sp && (nch - ch0) >= 2u;
  };
  if (t == 0) { s_run = 0; s_runbig = 0; s_runsm = 0; s_runcand = 0; s_nbig = 0; s_nent = 0; s_ncand = 0; }
  __syncthreads();
  if (cs > 0) {
    // first pass: the entries (big ones, all) and the fill candidates
    uint32_t nb = 0, ne = 0, nc = 0;
    for (uint32_t i = t; i < n; i += NT) {
      const uint32_t nch = chunks(counts[(size_t)touched[i] * stride]);
      const bool sp = size_split(nch);
      uint32_t ch0;
      bool b0, b1;
      classes(nch, true, sp, ch0, b0, b1);
      nb += (b0 ? 1u : 0u) + (b1 ? 1u : 0u);
      ne += sp ? 2u : 1u;
      nc += fill_candidate(nch) ? 1u : 0u;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      nb += __shfl_xor(nb, off);
      ne += __shfl_xor(ne, off);
      nc += __shfl_xor(nc, off);
    }
    if (lane == 0) {
      atomicAdd(&s_nbig, nb);
      atomicAdd(&s_nent, ne);
      atomicAdd(&s_ncand, nc);
    }
    __syncthreads();
  }
  // the first `fill` candidates are split: each turns one big entry into two
  // of one chunk.  At most one entry in 16 is added (every split adds a
  // second tile slot that the grid kernel reads one at a time)
  const uint32_t fill = (fill_slots > 0 && (uint32_t)fill_slots > s_nent)
                            ? min(min((uint32_t)fill_slots - s_nent, s_ncand), s_nent / 16u)
                            : 0u;
  const uint32_t nbig = s_nbig - fill;
  for (uint32_t c0 = 0; c0 < n; c0 += NT) {
    const uint32_t i = c0 + t;
    const bool valid = i < n;
    uint32_t key = 0, c = 0;
    if (valid) { key = touched[i]; c = counts[(size_t)key * stride]; }
    const uint32_t nch = valid ? chunks(c) : 0u;
    const bool cand = valid && fill_candidate(nch);
    uint32_t icand = cand ? 1u : 0u;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t o = __shfl_up(icand, off);
      if (lane >= off) icand += o;
    }
    if (lane == 63) s_cand[wv] = icand;
    __syncthreads();
    uint32_t wcand = s_runcand, totcand = s_runcand;
#pragma unroll
    for (int q = 0; q < NW; q++) {
      if (q < wv) wcand += s_cand[q];
      totcand += s_cand[q];
    }
    const bool sp = valid && (size_split(nch) || (cand && wcand + icand - 1u < fill));
    uint32_t ch0;
    bool big0, big1;
    classes(nch, valid, sp, ch0, big0, big1);
    const uint32_t eb = (big0 ? 1u : 0u) + (big1 ? 1u : 0u);
    const uint32_t es = (valid ? 1u : 0u) + (sp ? 1u : 0u) - eb;
    uint32_t is = c, ib = eb, ism = es;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t o = __shfl_up(is, off), o2 = __shfl_up(ib, off), o3 = __shfl_up(ism, off);
      if (lane >= off) { is += o; ib += o2; ism += o3; }
    }
    if (lane == 63) { s_sum[wv] = is; s_big[wv] = ib; s_sm[wv] = ism; }
    __syncthreads();
    uint32_t woff = s_run, tot = s_run, wb = s_runbig, totb = s_runbig, wsm = s_runsm, totsm = s_runsm;
#pragma unroll
    for (int q = 0; q < NW; q++) {
      if (q < wv) { woff += s_sum[q]; wb += s_big[q]; wsm += s_sm[q]; }
      tot += s_sum[q];
      totb += s_big[q];
      totsm += s_sm[q];
    }
    if (valid) {
      const uint32_t o = woff + is - c;
      uint32_t pb = wb + ib - eb, ps = nbig + wsm + ism - es;
      offsets[key] = o;
      counts[(size_t)key * stride] = 0u;
      if (sp) {
        const uint32_t c1 = ch0 * (uint32_t)split_nt;
        list[big0 ? pb++ : ps++] = make_int4((int)key, (int)o, (int)c1, 0);
        list[big1 ? pb : ps] = make_int4((int)key, (int)(o + c1), (int)(c - c1), 1);
      } else {
        list[big0 ? pb : ps] = make_int4((int)key, (int)o, (int)c, 0);
      }
    }
    __syncthreads();
    if (t == 0) { s_run = tot; s_runbig = totb; s_runsm = totsm; s_runcand = totcand; }
    __syncthreads();
  }
  if (t == 0) { list_n[0] = s_runbig + s_runsm; n_touched[0] = 0u; }
}

// Dense variant: exclusive scan of all counts -> offsets, the list of
// occupied keys in key (Morton) order, and the counts zeroed (the counter of
// key k at counts[k * stride]).  Run by one workgroup of NT threads: each
// wavefront owns a contiguous range of 256-key groups, one group per pass of
// its lanes (4 keys a lane, one coalesced 16-byte load); a first pass sums
// the range, the wavefront totals give each range its base, and a second
// pass scans the groups in order.  Loads are issued eight groups at a time,
// and the first eight groups stay in registers from the first pass to the
// second (at 128^3, 32768 keys, that is every group: one round trip).
template <int NT>
__device__ void scan_keys(uint32_t* __restrict__ counts, uint32_t* __restrict__ offsets, int4* __restrict__ list,
                          uint32_t* __restrict__ list_n, int n_keys, int stride = 1) {
  constexpr int NW = NT / 64;
  __shared__ uint32_t s_tot[NW], s_nzw[NW];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int groups = (n_keys + 255) / 256;
  const int gpw = (groups + NW - 1) / NW;
  const int g0 = min(groups, wv * gpw), g1 = min(groups, g0 + gpw);
  auto load4 = [&](int g, uint32_t* c) {
    const int k = g * 256 + 4 * lane;
    if (g < g1 && stride == 1 && k + 3 < n_keys) {
      const uint4 v = *(const uint4*)(counts + k);
      c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w;
    } else {
#pragma unroll
      for (int q = 0; q < 4; q++) c[q] = (g < g1 && k + q < n_keys) ? counts[(size_t)(k + q) * stride] : 0u;
    }
  };
  constexpr int GB = 8;   // groups per batch of loads
  uint32_t first[GB][4];
#pragma unroll
  for (int u = 0; u < GB; u++) load4(g0 + u, first[u]);
  uint32_t sum = 0, nz = 0;
#pragma unroll
  for (int u = 0; u < GB; u++)
#pragma unroll
    for (int q = 0; q < 4; q++) { sum += first[u][q]; nz += first[u][q] > 0u ? 1u : 0u; }
  for (int g = g0 + GB; g < g1; g += GB) {
    uint32_t c[GB][4];
#pragma unroll
    for (int u = 0; u < GB; u++) load4(g + u, c[u]);
#pragma unroll
    for (int u = 0; u < GB; u++)
#pragma unroll
      for (int q = 0; q < 4; q++) { sum += c[u][q]; nz += c[u][q] > 0u ? 1u : 0u; }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) { sum += __shfl_xor(sum, off); nz += __shfl_xor(nz, off); }
  if (lane == 0) { s_tot[wv] = sum; s_nzw[wv] = nz; }
  __syncthreads();
  uint32_t run = 0, li = 0, totnz = 0;
#pragma unroll
  for (int q = 0; q < NW; q++) {
    if (q < wv) { run += s_tot[q]; li += s_nzw[q]; }
    totnz += s_nzw[q];
  }
  for (int gb = g0; gb < g1; gb += GB) {
    uint32_t cb[GB][4];
#pragma unroll
    for (int u = 0; u < GB; u++) {
      if (gb == g0) {
#pragma unroll
        for (int q = 0; q < 4; q++) cb[u][q] = first[u][q];
      } else {
        load4(gb + u, cb[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < GB; u++) {
      const int g = gb + u;
      if (g >= g1) break;
      const uint32_t* c = cb[u];
      const uint32_t ls = c[0] + c[1] + c[2] + c[3];
      const uint32_t ln = (c[0] > 0u) + (c[1] > 0u) + (c[2] > 0u) + (c[3] > 0u);
      uint32_t is = ls, in = ln;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o1 = __shfl_up(is, off), o2 = __shfl_up(in, off);
        if (lane >= off) { is += o1; in += o2; }
      }
      uint32_t o = run + is - ls, l = li + in - ln;
      const int k = g * 256 + 4 * lane;
      uint32_t offs[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        offs[q] = o;
        if (c[q] > 0u) { list[l] = make_int4(k + q, (int)o, (int)c[q], 0); l++; }
        o += c[q];
      }
      if (stride == 1 && k + 3 < n_keys) {
        *(uint4*)(offsets + k) = make_uint4(offs[0], offs[1], offs[2], offs[3]);
        *(uint4*)(counts + k) = make_uint4(0u, 0u, 0u, 0u);
      } else {
#pragma unroll
        for (int q = 0; q < 4; q++)
          if (k + q < n_keys) { offsets[k + q] = offs[q]; counts[(size_t)(k + q) * stride] = 0u; }
      }
      run += (uint32_t)__shfl((int)is, 63);
      li += (uint32_t)__shfl((int)in, 63);
    }
  }
  if (threadIdx.x == 0) list_n[0] = totnz;
}

// The scan of a sort; also advances the per-call epoch of the step stamps
// (and clears the two claimed-block counters of the steps that follow).
// mode SCAN_TOUCHED: the touched keys, blocks listed in first-touch order;
// SCAN_DENSE: all keys, blocks listed in key (Morton) order.
constexpr int SCAN_TOUCHED = 0, SCAN_DENSE = 1;

__global__ __launch_bounds__(1024) void k_scan(uint32_t* __restrict__ counts, uint32_t* __restrict__ offsets,
                                               const uint32_t* __restrict__ touched, uint32_t* __restrict__ n_touched,
                                               int4* __restrict__ list, uint32_t* __restrict__ list_n, int n_keys,
                                               uint32_t* __restrict__ epoch, uint32_t* __restrict__ cl_count,
                                               int mode, int stride, int split_nt, int max_chunks, int order_nt,
                                               int fill_slots) {
  constexpr int NT = 1024;
  if (mode == SCAN_DENSE) {
    scan_keys<NT>(counts, offsets, list, list_n, n_keys, stride);
    if (threadIdx.x == 0) n_touched[0] = 0u;
  } else {
    scan_touched<1024>(counts, offsets, touched, n_touched, list, list_n, n_keys, stride, split_nt, max_chunks,
                       order_nt, fill_slots);
  }
  if (threadIdx.x == 0) { epoch[0] = epoch[0] + 1; cl_count[0] = 0u; cl_count[1] = 0u; }
}



// The user-order particles to their sorted slots, as a gather: k_inv records
// the user index of every slot (one scattered word per particle), k_gather_in
// then reads each slot's particle (scattered reads) and writes the sorted rows
// in order.
__global__ __launch_bounds__(256) void k_inv(int N, const uint32_t* __restrict__ key_tmp,
                                             const uint32_t* __restrict__ rank_tmp,
                                             const uint32_t* __restrict__ offsets, uint32_t* __restrict__ inv) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const uint32_t d = offsets[key_tmp[p]] + rank_tmp[p];
  if (d < (uint32_t)N) inv[d] = (uint32_t)p;
}

__global__ __launch_bounds__(256) void k_gather_in(PState u, const uint8_t* __restrict__ umat, PBuf X,
                                                   const uint32_t* __restrict__ inv,
                                                   const uint32_t* __restrict__ key_tmp,
                                                   const uint32_t* __restrict__ rank_tmp) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = u.N;
  if (d >= N) return;
  const uint32_t p = inv[d];
  if (p >= (uint32_t)N) return;
#pragma unroll
  for (int a = 0; a < 3; a++) { X.f[a * (size_t)N + d] = u.x[a * N + p]; X.f[(3 + a) * (size_t)N + d] = u.v[a * N + p]; }
#pragma unroll
  for (int k = 0; k < 9; k++) { X.f[(6 + k) * (size_t)N + d] = u.C[k * N + p]; X.f[(15 + k) * (size_t)N + d] = u.F[k * N + p]; }
  X.f[24 * (size_t)N + d] = u.J[p];
  X.id[d] = p;
  X.key[d] = key_tmp[p];
  X.rank[d] = rank_tmp[p];
  X.mat[d] = umat[p];
}

// block key and rank of the state produced from a sorted state (same rows);
// the scene comes from the previous key
__global__ __launch_bounds__(256) void k_keys_next(const float* __restrict__ xf, const uint32_t* __restrict__ key_prev,
                                                   int N, StepParams P, FastGeom g, uint32_t* __restrict__ counts,
                                                   uint32_t* __restrict__ key_tmp, uint32_t* __restrict__ rank_tmp,
                                                   uint32_t* __restrict__ touched, uint32_t* __restrict__ n_touched) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  bool has = p < N;
  uint32_t key = 0;
  if (has) {
    float x[3] = {xf[p], xf[(size_t)N + p], xf[2 * (size_t)N + p]};
    const uint32_t sc = key_prev[p] >> (3 * g.kb);
    Stencil S;
    if (!stencil_setup(x, P, S) || sc >= (uint32_t)g.S) atomicOr(P.err, ERR_OUTSIDE);
    else key = block_key(g, (int)sc, S.base[0] >> 2, S.base[1] >> 2, S.base[2] >> 2);
  }
  uint32_t r = wave_rank(counts, key, has, touched, n_touched, (uint32_t)g.n_keys);
  if (has) { key_tmp[p] = key; rank_tmp[p] = r; }
}

// move the rows of `in` to their sorted slots in `out`; map[p] = new row of p
__global__ __launch_bounds__(256) void k_sort_permute(PBuf in, PBuf out, int N, const uint32_t* __restrict__ key_tmp,
                                                      const uint32_t* __restrict__ rank_tmp,
                                                      const uint32_t* __restrict__ offsets, uint32_t* __restrict__ map) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  uint32_t key = key_tmp[p], r = rank_tmp[p];
  uint32_t d = offsets[key] + r;
  if (d >= (uint32_t)N) return;
#pragma unroll
  for (int k = 0; k < STATE_FLOATS; k++) out.f[k * (size_t)N + d] = in.f[k * (size_t)N + p];
  out.id[d] = in.id[p];
  out.mat[d] = in.mat[p];
  out.key[d] = key;
  out.rank[d] = r;
  map[p] = d;
}

// The sorted buffer back to the user arrays, as a gather: k_pos records the
// sorted slot of every particle, k_gather_out reads each particle's slot and
// writes the user rows in order.  Liquids keep the user's F and solids the
// user's J (those rows are not carried by the kernels).
__global__ __launch_bounds__(256) void k_pos(PBuf X, int N, uint32_t* __restrict__ pos) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= N) return;
  const uint32_t p = X.id[d];
  if (p < (uint32_t)N) pos[p] = (uint32_t)d;
}

__global__ __launch_bounds__(256) void k_gather_out(PBuf X, PState u, const MatDev* __restrict__ mats,
                                                    const uint32_t* __restrict__ pos) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = u.N;
  if (p >= N) return;
  const uint32_t j = pos[p];
  if (j >= (uint32_t)N) return;
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
  uint32_t* touched;           // keys counted in this step (first touch appends)
  uint32_t* n_touched;
  float* tiles;
  int2* tile_box;
  int n_keys;
  uint32_t* claim;             // per-block stamp of the step that claimed it
  uint32_t* cl_list;           // keys of the blocks claimed in this step
  uint32_t* cl_count;          // their number
  const uint32_t* gen;         // per-call epoch
  uint32_t step_id;            // 1-based step within the call
  const float4* vgrid;
  // learned closure and sample logging (sand, cone case)
  const MlpBlob* mlp;
  float closure_tol;
  unsigned long long* closure_stats;   // [0] accepted, [1] fell back to the exact return
  float* log_buf;                      // samples of 9 floats: log sigma_tr (desc), alpha, c, kappa, eps'
  unsigned long long* log_count;
  unsigned long long log_cap;
  uint32_t* map_out;                   // (records) output row of each input row, or nullptr
};

enum { FEAT_NONE = 0, FEAT_LOG = 1, FEAT_CLOSURE = 2 };

// The fused kernel (MODE 1 without the closure features) in 256-thread
// workgroups runs fastest held to three wavefronts per SIMD (168 VGPRs and a
// few spills): 65.5 us per config-2 step against 69.5 us at two (231 VGPRs)
// and 81.7 us at four.  In 512-thread workgroups the same bound made the
// 1e5-particle 64^3 step slower (66 against 62 us), so they keep two.  The
// separate P2G (MODE 0, 190 VGPRs unbounded) gains from the same bound too:
// the rigid-body step at config-2 size 0.126 -> 0.121 ms.  The learned-
// closure variant (FP64 return, network on the matrix cores) held to two
// wavefronts per SIMD keeps its accumulators in VGPRs (256, a few spills)
// instead of running at one (0.76 -> 0.57 ms per config-5 step).
template <int MODE, int NT, int FEAT>
__global__ __launch_bounds__(NT, (NT == 256 && ((MODE == 1 && FEAT == FEAT_NONE) || MODE == 0))
                                     ? 3
                                     : ((MODE == 1 && FEAT == FEAT_CLOSURE) ? 2 : 1)) void
k_particles(PartArgs A, StepParams P, FastGeom g) {
  constexpr int NW = NT / 64;
  __shared__ MlpBlob s_mlp;
  __shared__ MlpScratch s_mscr[NW];
  if (FEAT == FEAT_CLOSURE) {
    const uint32_t* src = (const uint32_t*)A.mlp;
    uint32_t* dstw = (uint32_t*)&s_mlp;
    for (int q = threadIdx.x; q < (int)(sizeof(MlpBlob) / 4); q += NT) dstw[q] = src[q];
    __syncthreads();
  }
  __shared__ float s_tile[4 * TILE_NODES];
  __shared__ int s_itile[4 * TILE_NODES];
  __shared__ float4 s_v[VT_NODES];
  __shared__ float s_red[NW * 4];     // per-wave bound sums of the chunk
  __shared__ uint32_t s_ired[NW];      // per-wave box bits of the chunk
  const int tid = threadIdx.x;
  const int N = A.N;
  const uint32_t n_list = A.list_n[0];
  // step stamp: per-call epoch (advanced by the import) and step within the call
  const uint32_t stamp = (A.gen[0] << 16) | A.step_id;
  for (uint32_t e = blockIdx.x; e < n_list; e += gridDim.x) {
    const int4 ent = A.list[e];
    int sc, bx, by, bz;
    key_decode(g, (uint32_t)ent.x, sc, bx, by, bz);
    const int ox = 4 * bx, oy = 4 * by, oz = 4 * bz;
    const int start = ent.y, count = ent.z;
    // The inputs of a chunk are loaded one chunk ahead (the first chunk's
    // before the staging below), so that their latency overlaps other work.
    // F and J are both loaded, whatever the material, so that no load waits
    // for the material's kind; v and C are replaced by G2P and not read.
    float px[3] = {0, 0, 0}, pF[9], pJ = 1.f;
    int pm = 0;
    uint32_t pkey = 0, prank = 0;
    auto prefetch = [&](int c0n) {
      const int jn = start + c0n + tid;
      if (c0n + tid < count && jn < N) {
#pragma unroll
        for (int a = 0; a < 3; a++) px[a] = A.in.f[a * (size_t)N + jn];
#pragma unroll
        for (int k = 0; k < 9; k++) pF[k] = A.in.f[(15 + k) * (size_t)N + jn];
        pJ = A.in.f[24 * (size_t)N + jn];
        pm = A.in.mat[jn];
        if (MODE != MODE_P2G) { pkey = A.in.key[jn]; prank = A.in.rank[jn]; }
      }
    };
    prefetch(0);
    // ---- stage grid velocities of nodes [4b-1, 4b+7) for G2P
    if (MODE != MODE_P2G) {
      for (int q = tid; q < VT_NODES; q += NT) {
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
      for (int q = tid; q < 4 * TILE_NODES; q += NT) { s_tile[q] = 0.f; s_itile[q] = 0; }

    }
    __syncthreads();
    // the tile's non-zero box over all chunks (every thread keeps the same copy)
    int blo[3] = {1 << 20, 1 << 20, 1 << 20}, bhi[3] = {-(1 << 20), -(1 << 20), -(1 << 20)};
    for (int c0 = 0; c0 < count; c0 += NT) {
      const int j = start + c0 + tid;
      const bool has = (c0 + tid) < count && j < N;
      float x[3] = {px[0], px[1], px[2]}, v[3] = {0, 0, 0}, C[9], F[9], J = pJ;
#pragma unroll
      for (int k = 0; k < 9; k++) { F[k] = pF[k]; C[k] = 0.f; }
      const int m = has ? pm : 0;
      bool ok = has;
      // destination slot in the output buffer (the key -> offset lookup
      // overlaps the G2P arithmetic); the P2G-only mode reads v and C
      uint32_t dst = 0;
      if (has) {
        if (MODE == MODE_P2G) load_state(A.in, N, j, x, v, C, F, J);
        else dst = A.offsets[pkey] + prank;
      }
      const MatDev& M = P.mats[m];
      const bool liquid = M.kind == KIND_LIQUID;
      float tau[9];
      bool have_tau = false;
      // cone-case sample of this particle (closure input and exact answer)
      bool cone = false;
      float xin[MLP_IN] = {0, 0, 0, 0, 0, 0}, eex[MLP_OUT] = {0, 0, 0};
      float Uk[9], Vk[9];
      // ---------------- G2P of the previous step ----------------
      if (MODE != MODE_P2G && has) {
        Stencil S;
        bool in_grid = stencil_setup(x, P, S);
        int lb[3] = {S.base[0] - (ox - 1), S.base[1] - (oy - 1), S.base[2] - (oz - 1)};
        bool in_tile = lb[0] >= 0 && lb[1] >= 0 && lb[2] >= 0 && lb[0] <= VT - 3 && lb[1] <= VT - 3 && lb[2] <= VT - 3;
        if (!in_grid) { atomicOr(P.err, ERR_OUTSIDE); ok = false; }
        else if (!in_tile) { atomicOr(P.err, ERR_TILE); ok = false; }
        if (ok) {
          // sum_i w v_i and sum_i w v_i idx^T (idx = the node offset in
          // {0,1,2}^3); then B = sum w v (x_i - x_p)^T = dx (Bi - vn f^T)
          float vn[3], Bi[9];
          g2p_gather(s_v, lb, S, vn, Bi);
          float B[9];
#pragma unroll
          for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) B[a * 3 + b] = P.dx * (Bi[a * 3 + b] - vn[a] * S.f[b]);
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
          } else if (elastic_update_kind(M.kind)) {
            float Fn[9];
            matmul(Md, F, Fn);
#pragma unroll
            for (int k = 0; k < 9; k++) F[k] = Fn[k];
          } else {
            // plastic solids: FP32 SVD and return map, redone in FP64 for an
            // ill-conditioned trial state (or an unconverged sweep).  Sample
            // logging keeps the FP64 SVD throughout: its records are the
            // exact FP64 return
            float Fn[9];
            PlasticStep<float> R;
            int st = FEAT != FEAT_LOG ? plastic_step<float, MODE == MODE_FUSED>(Md, F, M, Fn, tau, R) : PLASTIC_RETRY;
            if (st == PLASTIC_RETRY) {
              PlasticStep<double> R2;
              st = plastic_step<double, MODE == MODE_FUSED>(Md, F, M, Fn, tau, R2);
              R.cse = R2.cse;
#pragma unroll
              for (int k = 0; k < 9; k++) { R.U[k] = (float)R2.U[k]; R.V[k] = (float)R2.V[k]; }
#pragma unroll
              for (int a = 0; a < 3; a++) { R.e[a] = (float)R2.e[a]; R.ep[a] = (float)R2.ep[a]; }
            }
#pragma unroll
            for (int k = 0; k < 9; k++) F[k] = Fn[k];
            if (st == PLASTIC_SIGMA) {
              atomicOr(P.err, ERR_SAND_SIGMA);
              ok = false;
            } else {
              have_tau = MODE == MODE_FUSED && M.kind != KIND_BOX;
              if (FEAT != FEAT_NONE && M.kind == KIND_SAND && R.cse == 2) {
                cone = true;
#pragma unroll
                for (int a = 0; a < 3; a++) { xin[a] = R.e[a]; eex[a] = R.ep[a]; }
                xin[3] = M.alpha;
                xin[4] = M.coh;
                xin[5] = M.kappa;
                if (FEAT == FEAT_CLOSURE) {
#pragma unroll
                  for (int k = 0; k < 9; k++) { Uk[k] = R.U[k]; Vk[k] = R.V[k]; }
                }
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
          if (A.map_out) A.map_out[j] = dst;
        } else {
          ok = false;
        }
      }
      if (MODE == MODE_G2P && c0 + NT < count) prefetch(c0 + NT);
      if (FEAT == FEAT_LOG) {
        // append the exact cone-case samples, one counter atomic per wavefront
        const unsigned long long m = __ballot(cone);
        if (m) {
          const int lane = __lane_id();
          const int leader = __ffsll((long long)m) - 1;
          unsigned long long base = 0;
          if (lane == leader) base = atomicAdd(A.log_count, (unsigned long long)__popcll(m));
          base = __shfl(base, leader);
          if (cone) {
            const unsigned long long idx = base + (unsigned long long)__popcll(m & ((1ull << lane) - 1ull));
            if (idx < A.log_cap) {
              float* o = A.log_buf + idx * 9;
#pragma unroll
              for (int q = 0; q < MLP_IN; q++) o[q] = xin[q];
#pragma unroll
              for (int q = 0; q < MLP_OUT; q++) o[MLP_IN + q] = eex[q];
            }
          }
        }
      }
      if (FEAT == FEAT_CLOSURE) {
        // learned cone return on the matrix cores for the wave's cone-case
        // lanes; a prediction whose yield residual exceeds the tolerance
        // falls back to the exact return already in F and tau
        const unsigned long long m = __ballot(cone);
        if (m) {
          float yp[MLP_OUT];
          mlp_wave_forward(s_mlp, xin, yp, s_mscr[tid >> 6]);
          bool accepted = false;
          if (cone) {
            const double c = (double)xin[4], ka = (double)xin[5] * (double)xin[3];
            double es[3] = {yp[0] - c, yp[1] - c, yp[2] - c};
            const double tr = es[0] + es[1] + es[2];
            const double d0 = es[0] - tr / 3.0, d1 = es[1] - tr / 3.0, d2 = es[2] - tr / 3.0;
            const double f = sqrt(d0 * d0 + d1 * d1 + d2 * d2) + ka * tr;
            const double r = fabs(f) + fabs(((double)yp[0] + yp[1] + yp[2]) - ((double)xin[0] + xin[1] + xin[2]));
            accepted = r <= (double)A.closure_tol && isfinite(r);
            if (accepted) {
              float gg[3] = {expf(yp[0]), expf(yp[1]), expf(yp[2])}, Fo[9];
              usv(Uk, gg, Vk, Fo);
#pragma unroll
              for (int k = 0; k < 9; k++) F[k] = Fo[k];
              if (MODE == MODE_FUSED) hencky_tau(Uk, yp, M, tau);
              // the corrected F goes to the output slot written above
              if (dst < (uint32_t)N) {
#pragma unroll
                for (int k = 0; k < 9; k++) A.out.f[(15 + k) * (size_t)N + dst] = F[k];
              }
            }
          }
          const unsigned long long acc = __ballot(accepted);
          if (__lane_id() == 0) {
            atomicAdd(A.closure_stats, (unsigned long long)__popcll(acc));
            atomicAdd(A.closure_stats + 1, (unsigned long long)(__popcll(m) - __popcll(acc)));
          }
        }
      }
      // ---------------- P2G of this step ----------------
      // LDS float atomics are slow on gfx950 (about 1/30 of the integer
      // rate), so each chunk of NT particles accumulates in exact 32-bit fixed
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
          else if (!have_tau && !stress_solid_fast(F, M, tau)) atomicOr(P.err, ERR_SAND_SIGMA);
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
        // reserve this particle's rank under its new key now; the result is
        // consumed after the scatter, so the atomic's latency is hidden
        WaveRank WR = {0, 0, 0};
        if (MODE == MODE_FUSED) WR = rank_issue(A.counts, nkey, counted && has);
        // chunk-wide bound sums and box: DPP reductions over the wavefront,
        // then the waves' results combined in LDS.  The box is kept as one
        // bit per occupied stencil origin and axis (bit lb_a of byte a; lb
        // is at most TILE - 3 = 7), so that one OR gives it.
        const uint32_t obits = ok ? ((1u << lb[0]) | (1u << (8 + lb[1])) | (1u << (16 + lb[2]))) : 0u;
        const uint32_t wbits = wave_or(obits);
        float wb[4];
#pragma unroll
        for (int q = 0; q < 4; q++) wb[q] = wave_sum(bnd[q]);
        const int wv = tid >> 6;
        if ((tid & 63) == 0) {
#pragma unroll
          for (int q = 0; q < 4; q++) s_red[wv * 4 + q] = wb[q];
          s_ired[wv] = wbits;
        }
        __syncthreads();
        // every thread derives the chunk's scales and box from the waves'
        // partial results (no second barrier); the previous chunk's flush,
        // which ran after its scatter barrier, is complete here as well
        float sc[4], isc[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
          float T = 0.f;
#pragma unroll
          for (int w = 0; w < NW; w++) T += s_red[w * 4 + q];
          T *= 0.421875f;
          if (!isfinite(T)) {
            if (tid == 0) atomicOr(P.err, ERR_NONFINITE);
            T = 1.f;
          }
          int e = 0;
          frexpf(T > 0.f ? T : 1.f, &e);
          e = max(e, -90);
          sc[q] = ldexpf(1.f, 30 - e);
          isc[q] = ldexpf(1.f, e - 30);
        }
        int clo[3], chi[3];
        {
          uint32_t cb = 0;
#pragma unroll
          for (int w = 0; w < NW; w++) cb |= s_ired[w];
#pragma unroll
          for (int a = 0; a < 3; a++) {
            const uint32_t ab = (cb >> (8 * a)) & 0xffu;
            clo[a] = ab ? __ffs(ab) - 1 : 1 << 20;
            chi[a] = ab ? 31 - __clz(ab) : -(1 << 20);
            if (clo[a] <= chi[a]) { blo[a] = min(blo[a], clo[a]); bhi[a] = max(bhi[a], chi[a]); }
          }
        }
        if (ok) {
          // mom_a(node) = mvp_a + sum_b A_ab (idx_b - f_b) dx = c0_a + sum_b Ad_ab idx_b,
          // with the quantity's power-of-two scale folded into c0 and Ad
          const float sm = M.mass * sc[0];
          float c0[3], Ad[9];
#pragma unroll
          for (int a = 0; a < 3; a++) {
            const float sa = sc[1 + a];
#pragma unroll
            for (int b = 0; b < 3; b++) Ad[a * 3 + b] = sa * P.dx * Am[a * 3 + b];
            c0[a] = sa * mvp[a] - (Ad[a * 3] * S.f[0] + Ad[a * 3 + 1] * S.f[1] + Ad[a * 3 + 2] * S.f[2]);
          }
          int* T = s_itile + (lb[0] * TILE + lb[1]) * TILE + lb[2];
#pragma unroll
          for (int i = 0; i < 3; i++) {
            float m1[3];
#pragma unroll
            for (int a = 0; a < 3; a++) m1[a] = c0[a] + (float)i * Ad[a * 3];
#pragma unroll
            for (int jj = 0; jj < 3; jj++) {
              const float wxy = S.w[0][i] * S.w[1][jj];
              float m2[3];
#pragma unroll
              for (int a = 0; a < 3; a++) m2[a] = m1[a] + (float)jj * Ad[a * 3 + 1];
#pragma unroll
              for (int k = 0; k < 3; k++) {
                const float w = wxy * S.w[2][k];
                const int q = (i * TILE + jj) * TILE + k;
                atomicAdd(&T[q], __float2int_rn(w * sm));
                atomicAdd(&T[TILE_NODES + q], __float2int_rn(w * (m2[0] + (float)k * Ad[2])));
                atomicAdd(&T[2 * TILE_NODES + q], __float2int_rn(w * (m2[1] + (float)k * Ad[5])));
                atomicAdd(&T[3 * TILE_NODES + q], __float2int_rn(w * (m2[2] + (float)k * Ad[8])));
              }
            }
          }
        }
        if (c0 + NT < count) prefetch(c0 + NT);
        __syncthreads();
        {
          // flush the chunk's box into the float tile and clear the integers
          // (the next chunk scatters only after its bound barrier)
          if (clo[0] <= chi[0]) {
            const int ex = chi[0] - clo[0] + 3, ey = chi[1] - clo[1] + 3, ez = chi[2] - clo[2] + 3;
            const int cnt = ex * ey * ez;
            for (int r = tid; r < cnt; r += NT) {
              int qq = ((clo[0] + r / (ey * ez)) * TILE + clo[1] + (r / ez) % ey) * TILE + clo[2] + r % ez;
#pragma unroll
              for (int c = 0; c < 4; c++) {
                int iv = s_itile[c * TILE_NODES + qq];
                if (iv != 0) {
                  s_tile[c * TILE_NODES + qq] += (float)iv * isc[c];
                  s_itile[c * TILE_NODES + qq] = 0;
                }
              }
            }
          }
        }
        if (MODE == MODE_FUSED) {
          uint32_t r = rank_finish(WR, A.touched, A.n_touched, (uint32_t)A.n_keys);
          if (has && dst < (uint32_t)N) { A.out.key[dst] = nkey; A.out.rank[dst] = counted ? r : 0u; }
          // a particle that could not be counted keeps a valid (key 0) slot
          if (has && !counted && dst < (uint32_t)N) {
            uint32_t r0 = atomicAdd(&A.counts[0], 1u);
            if (r0 == 0u) touch_key(0u, A.touched, A.n_touched, (uint32_t)A.n_keys);
            A.out.key[dst] = 0u;
            A.out.rank[dst] = r0;
          }
        }
      }
    }
    __syncthreads();
    if (MODE != MODE_G2P) {
      // ---- publish the tile's non-zero box and mark the blocks it touches
      const int lo0 = blo[0], lo1 = blo[1], lo2 = blo[2];
      const int hi0 = bhi[0] + 2, hi1 = bhi[1] + 2, hi2 = bhi[2] + 2;
      const uint32_t bkey = (uint32_t)ent.x;
      const size_t slot = (size_t)bkey + (size_t)ent.w * (size_t)A.n_keys;   // the entry's tile slot
      if (lo0 <= hi0 - 2) {
        const int ex = hi0 - lo0 + 1, ey = hi1 - lo1 + 1, ez = hi2 - lo2 + 1;
        const int cnt = ex * ey * ez;
        // in global memory a node's (m, mv) is one 16-byte word
        float4* T = reinterpret_cast<float4*>(A.tiles + slot * 4 * TILE_NODES);
        for (int r = tid; r < cnt; r += NT) {
          int qi = lo0 + r / (ey * ez), qj = lo1 + (r / ez) % ey, qk = lo2 + r % ez;
          int q = (qi * TILE + qj) * TILE + qk;
          T[q] = make_float4(s_tile[q], s_tile[TILE_NODES + q], s_tile[2 * TILE_NODES + q], s_tile[3 * TILE_NODES + q]);
        }
        if (tid == 0) {
          int packed = lo0 | (lo1 << 4) | (lo2 << 8) | (hi0 << 12) | (hi1 << 16) | (hi2 << 20);
          A.tile_box[slot] = make_int2(packed, (int)stamp);
        }
        // claim the blocks this tile touches: the first entry to claim a block
        // in this step appends it to the list the grid kernel works through
        if (tid < 64) {
          bool won = false;
          uint32_t nk = 0;
          if (tid < 27) {
            const int dx = tid / 9 - 1, dy = (tid / 3) % 3 - 1, dz = tid % 3 - 1;
            const int nbx = bx + dx, nby = by + dy, nbz = bz + dz;
            const int l0 = 4 * dx + 2, l1 = 4 * dy + 2, l2 = 4 * dz + 2;
            const bool hit = nbx >= 0 && nby >= 0 && nbz >= 0 && nbx < g.nb && nby < g.nb && nbz < g.nb &&
                             l0 <= hi0 && l0 + 3 >= lo0 && l1 <= hi1 && l1 + 3 >= lo1 && l2 <= hi2 && l2 + 3 >= lo2;
            if (hit) {
              nk = block_key(g, sc, nbx, nby, nbz);
              won = atomicExch(&A.claim[nk], stamp) != stamp;
            }
          }
          const unsigned long long wm = __ballot(won);
          if (wm) {
            uint32_t base = 0;
            if (tid == 0) base = atomicAdd(A.cl_count, (uint32_t)__popcll(wm));
            base = __shfl(base, 0);
            // a block is claimed once per step, so at most n_keys keys arrive
            const uint32_t slot = base + (uint32_t)__popcll(wm & ((1ull << tid) - 1ull));
            if (won && slot < (uint32_t)A.n_keys) A.cl_list[slot] = nk;
          }
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// grid update: one workgroup (4 wavefronts) per entry of the occupied-block
// list; the entry's claimed neighbour blocks (claimed by the particle kernel)
// are shared among the wavefronts; for each block the 64 node lanes sum the
// overlapping tiles of its 27 neighbours and apply the node update
// (normalise, gravity, soft cylinder contact, slip walls).
// ---------------------------------------------------------------------------
struct ScanArgs {
  uint32_t* counts;
  uint32_t* offsets;
  uint32_t* touched;
  uint32_t* n_touched;
  int4* list;
  uint32_t* list_n;
  int n_keys;
  int split_nt;     // particles per chunk of the particle kernel that reads the list (0: no sharing)
  int max_chunks;   // chunks above which a block is shared by two workgroups
  int order_nt;     // chunk size that orders the entries when split_nt is 0 (0: first-touch order)
  int fill_slots;   // resident workgroups of the particle kernel that split blocks may fill (0: none)
};

// With do_scan, workgroup 0 scans the key counts of this step's particle
// kernel (independent of the grid work) and the others do the grid update.
__global__ __launch_bounds__(256) void k_grid(StepParams P, FastGeom g, const uint32_t* __restrict__ cl_list,
                                              const uint32_t* __restrict__ cl_count, uint32_t* __restrict__ cl_zero,
                                              const int2* __restrict__ tile_box, const float* __restrict__ tiles,
                                              const uint32_t* __restrict__ gen, uint32_t step_id,
                                              float4* __restrict__ vgrid, const double* __restrict__ pose_base,
                                              const float* __restrict__ act_base, const int* __restrict__ t0_dev,
                                              int do_scan, ScanArgs SA, int t_fixed, float4* __restrict__ mmv_out) {
  if (do_scan && blockIdx.x == 0) {
    scan_touched<256>(SA.counts, SA.offsets, SA.touched, SA.n_touched, SA.list, SA.list_n, SA.n_keys, 1, SA.split_nt,
                      SA.max_chunks, SA.order_nt, SA.fill_slots);
    return;
  }
  const uint32_t wg = blockIdx.x - (do_scan ? 1 : 0), n_wg = gridDim.x - (do_scan ? 1 : 0);
  // the clock lives in device memory so that a captured call can be replayed
  // at any start time: this launch is step (step_id - 1) of the call
  // (the adjoint's recompute passes its step explicitly in t_fixed)
  const size_t t = t_fixed >= 0 ? (size_t)t_fixed : (size_t)t0_dev[0] + step_id - 1;
  const double* pose_t = pose_base + t * g.S * POSE_DOUBLES;
  const float* act_t = act_base + t * g.S * 6;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int li = lane >> 4, lj = (lane >> 2) & 3, lk = lane & 3;
  // one claimed block per wavefront; a wavefront's first key is loaded
  // together with the claim count (a list row past the count is stale and
  // not used)
  const uint32_t n_waves = 4u * n_wg;
  uint32_t it = 4u * wg + (uint32_t)wv;
  uint32_t key_it = it < (uint32_t)g.n_keys ? cl_list[it] : 0u;
  const uint32_t n_cl = cl_count[0];
  // the counter of the next step's claims starts at zero (nothing reads it now)
  if (cl_zero && wg == 0 && threadIdx.x == 0) cl_zero[0] = 0u;
  const uint32_t stamp = (gen[0] << 16) | step_id;
  for (; it < n_cl && it < (uint32_t)g.n_keys; it += n_waves) {
    const uint32_t key = key_it;
    if (it + n_waves < (uint32_t)g.n_keys) key_it = cl_list[it + n_waves];
    int sc, cx, cy, cz;
    key_decode(g, key, sc, cx, cy, cz);
    {
      // lanes 0..26 read the boxes of the 27 neighbours' tiles, lanes 32..58
      // those of their second slots (blocks shared by two workgroups)
      int2 nbox = make_int2(0, 0);
      uint32_t nkey = 0;
      const int dl = lane < 32 ? lane : lane - 32;
      if (dl < 27) {
        const int sx = cx + dl / 9 - 1, sy = cy + (dl / 3) % 3 - 1, sz = cz + dl % 3 - 1;
        if (sx >= 0 && sy >= 0 && sz >= 0 && sx < g.nb && sy < g.nb && sz < g.nb) {
          nkey = block_key(g, sc, sx, sy, sz) + (lane < 32 ? 0u : (uint32_t)g.n_keys);
          nbox = tile_box[nkey];
          if ((uint32_t)nbox.y != stamp) nbox.y = 0;
        }
      }
      const int gx = 4 * cx + li, gy = 4 * cy + lj, gz = 4 * cz + lk;
      // branch-free over the 27 neighbours so that all tile loads are in
      // flight together (a lane outside a tile's box reads slot 0 and adds 0)
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
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
        const float4 tv = reinterpret_cast<const float4*>(tiles + (size_t)(in ? kk : 0u) * 4 * TILE_NODES)[q];
        acc.w += in ? tv.x : 0.f;
        acc.x += in ? tv.y : 0.f;
        acc.y += in ? tv.z : 0.f;
        acc.z += in ? tv.w : 0.f;
      }
      // the few valid second slots, one at a time
      unsigned long long m1 = __ballot(lane >= 32 && nbox.y != 0);
      while (m1) {
        const int src = __ffsll((long long)m1) - 1;
        m1 &= m1 - 1ull;
        const int dd = src - 32;
        const int bxv = __shfl(nbox.x, src);
        const uint32_t kk = __shfl(nkey, src);
        const int sx = cx + dd / 9 - 1, sy = cy + (dd / 3) % 3 - 1, sz = cz + dd % 3 - 1;
        const int qi = gx - (4 * sx - 2), qj = gy - (4 * sy - 2), qk = gz - (4 * sz - 2);
        const int lo0 = bxv & 15, lo1 = (bxv >> 4) & 15, lo2 = (bxv >> 8) & 15;
        const int hi0 = (bxv >> 12) & 15, hi1 = (bxv >> 16) & 15, hi2 = (bxv >> 20) & 15;
        if (qi >= lo0 && qi <= hi0 && qj >= lo1 && qj <= hi1 && qk >= lo2 && qk <= hi2) {
          const float4 tv = reinterpret_cast<const float4*>(tiles + (size_t)kk * 4 * TILE_NODES)[(qi * TILE + qj) * TILE + qk];
          acc.w += tv.x;
          acc.x += tv.y;
          acc.y += tv.z;
          acc.z += tv.w;
        }
      }
      float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
      if (acc.w > 0.f && gx < g.n && gy < g.n && gz < g.n) {
        int idx[3] = {gx, gy, gz};
        float vv[3];
        grid_node_forward(P, sc, idx, acc, pose_t, act_t, vv, nullptr);
        out = make_float4(vv[0], vv[1], vv[2], acc.w);
      }
      vgrid[(size_t)key * 64 + lane] = out;
      if (mmv_out) mmv_out[(size_t)key * 64 + lane] = (out.w > 0.f) ? acc : make_float4(0.f, 0.f, 0.f, 0.f);
    }
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
  size_t buf_f[2], buf_id[2], buf_key[2], buf_rank[2], buf_mat[2], list[3];
  size_t key_tmp, rank_tmp, inv, cpad, counts, offsets, list_n, claim, cl_list, cl_count, touched, n_touched, tile_box, tiles,
      vgrid, gen, t0;
  size_t total;
};

static FastLayout fast_plan(int n_grid, int S, int N) {
  FastGeom g = make_geom(n_grid, S);
  FastLayout L;
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o += a256(b); return r; };
  for (int b = 0; b < 3; b++) L.list[b] = take((size_t)g.n_keys * NSUB * 16);
  for (int b = 0; b < 2; b++) {
    L.buf_f[b] = take((size_t)STATE_FLOATS * N * 4);
    L.buf_id[b] = take((size_t)N * 4);
    L.buf_key[b] = take((size_t)N * 4);
    L.buf_rank[b] = take((size_t)N * 4);
    L.buf_mat[b] = take((size_t)N);
  }
  L.key_tmp = take((size_t)N * 4);
  L.rank_tmp = take((size_t)N * 4);
  L.inv = take((size_t)N * 4);
  L.cpad = take((size_t)g.n_keys * IMPORT_PAD * 4);
  L.counts = take((size_t)g.n_keys * 4);
  L.offsets = take((size_t)g.n_keys * 4);
  L.list_n = take(16);
  L.claim = take((size_t)g.n_keys * 4);
  L.cl_list = take((size_t)g.n_keys * 4);
  L.cl_count = take(16);
  L.touched = take((size_t)g.n_keys * 4);
  L.n_touched = take(16);
  L.tile_box = take((size_t)g.n_keys * NSUB * 8);
  L.tiles = take((size_t)g.n_keys * NSUB * 4 * TILE_NODES * 4);
  L.vgrid = take((size_t)g.n_keys * 64 * 16);
  L.gen = take(16);
  L.t0 = take(16);
  L.total = o;
  return L;
}

size_t fast_workspace_bytes(int n_grid, int n_scenes, int N) { return fast_plan(n_grid, n_scenes, N).total; }
int fast_n_keys(int n_grid, int n_scenes) { return make_geom(n_grid, n_scenes).n_keys; }

static inline unsigned nblk(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

// the import's permutation (after its key count and scan) and the export,
// both as a scattered word per particle plus a gather
static void import_permute(FastPath& f, const PState& user, const uint8_t* umat, const PBuf& X, hipStream_t s) {
  const int N = f.N;
  k_inv<<<nblk(N, 256), 256, 0, s>>>(N, f.key_tmp, f.rank_tmp, f.offsets, f.inv);
  k_gather_in<<<nblk(N, 256), 256, 0, s>>>(user, umat, X, f.inv, f.key_tmp, f.rank_tmp);
}
static void export_state(FastPath& f, const PBuf& X, const PState& user, const MatDev* mats, hipStream_t s) {
  const int N = f.N;
  k_pos<<<nblk(N, 256), 256, 0, s>>>(X, N, f.inv);
  k_gather_out<<<nblk(N, 256), 256, 0, s>>>(X, user, mats, f.inv);
}

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
  }
  for (int b = 0; b < 3; b++) f.list[b] = (int4*)(ws + L.list[b]);
  f.key_tmp = (uint32_t*)(ws + L.key_tmp);
  f.rank_tmp = (uint32_t*)(ws + L.rank_tmp);
  f.inv = (uint32_t*)(ws + L.inv);
  f.cpad = (uint32_t*)(ws + L.cpad);
  f.counts = (uint32_t*)(ws + L.counts);
  f.offsets = (uint32_t*)(ws + L.offsets);
  f.list_n = (uint32_t*)(ws + L.list_n);
  f.claim = (uint32_t*)(ws + L.claim);
  f.cl_list = (uint32_t*)(ws + L.cl_list);
  f.cl_count = (uint32_t*)(ws + L.cl_count);
  f.touched = (uint32_t*)(ws + L.touched);
  f.n_touched = (uint32_t*)(ws + L.n_touched);
  f.tile_box = (int2*)(ws + L.tile_box);
  f.tiles = (float*)(ws + L.tiles);
  f.vgrid = (float4*)(ws + L.vgrid);
  f.gen = (uint32_t*)(ws + L.gen);
  f.t0_dev = (int*)(ws + L.t0);
  f.part_threads = 256;
  f.share_chunks = 2;
  f.use_graph = false;
  f.do_export = true;
  f.mlp_blob = nullptr;
  f.closure_tol = 1e-3f;
  f.closure_stats = nullptr;
  f.log_buf = nullptr;
  f.log_count = nullptr;
  f.log_cap = 0;
  f.part_wgs = 2048;
  f.calls = 0;
  f.ck_base = nullptr;
  f.ck_stride = 0;
  f.ck_k = 0;
  f.ck_t0 = 0;
  f.grid_wgs = 2048;
  f.valid = false;
  f.sid = 0;
  {
    // resident 256-thread workgroups of the fused kernel: CUs x occupancy
    int dev = 0, cus = 0, occ = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_particles<MODE_FUSED, 256, FEAT_NONE>, 256, 0) != hipSuccess)
      occ = 0;
    f.fused_slots = cus * occ;
  }
  // zero the bookkeeping (counts, stamps, counters, velocity grid)
  launch_zero(ws + L.counts, a256((size_t)f.g.n_keys * 4), s);
  launch_zero(ws + L.cpad, a256((size_t)f.g.n_keys * IMPORT_PAD * 4), s);
  launch_zero(ws + L.list_n, 256, s);
  launch_zero(ws + L.claim, a256((size_t)f.g.n_keys * 4), s);
  launch_zero(ws + L.cl_count, 256, s);
  launch_zero(ws + L.n_touched, 256, s);
  launch_zero(ws + L.tile_box, a256((size_t)f.g.n_keys * NSUB * 8), s);
  launch_zero(ws + L.vgrid, a256((size_t)f.g.n_keys * 64 * 16), s);
  launch_zero(ws + L.gen, 256, s);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

void fast_bind_grid(FastPath& f, float4* mmv, float4* vgrid) { f.mmv = mmv; f.vdense = vgrid; }

__global__ void k_set_word(int* w, int v) { w[0] = v; }

// Every import scan advances the device epoch of the step stamps by one; the
// host counts them so that the 16-bit epoch's wrap clears the stamps first.
static void new_epoch(FastPath& f, hipStream_t s) {
  if ((++f.calls & 0xffff) == 0) {
    launch_zero(f.claim, (size_t)f.g.n_keys * 4, s);
    launch_zero(f.tile_box, (size_t)f.g.n_keys * NSUB * 8, s);
  }
  f.sid = 0;
}

// Enqueue one call of n steps: import (sort by block), n steps, export.  With
// `ev` the fused kernel's launches are bracketed by the given event pairs.
template <int NT, int FEAT>
static void enqueue_call(FastPath& f, const StepParams& P, const PState& user, int n, const double* pose,
                         const float* act, hipStream_t s, std::vector<hipEvent_t>* ev) {
  const FastGeom g = f.g;
  const int N = f.N;
  // blocks of two chunks are also split while the list has fewer entries
  // than the particle kernel has resident workgroups, in 256-thread
  // workgroups (three resident per CU) without the closure features
  const int fill_slots = (NT == 256 && FEAT == FEAT_NONE && f.share_chunks > 0) ? std::min(f.part_wgs, f.fused_slots) : 0;
  k_import_keys<<<nblk(N, 256), 256, 0, s>>>(user, P, g, f.cpad, f.key_tmp, f.rank_tmp, f.touched, f.n_touched);
  k_scan<<<1, 1024, 0, s>>>(f.cpad, f.offsets, f.touched, f.n_touched, f.list[0], f.list_n + 0, g.n_keys, f.gen,
                            f.cl_count, SCAN_TOUCHED, IMPORT_PAD, f.share_chunks > 0 ? NT : 0, f.share_chunks, NT,
                            fill_slots);
  import_permute(f, user, P.mat, f.buf[0], s);
  PartArgs A;
  A.N = N;
  A.counts = f.counts;
  A.touched = f.touched;
  A.n_touched = f.n_touched;
  A.offsets = f.offsets;
  A.tiles = f.tiles;
  A.tile_box = f.tile_box;
  A.gen = f.gen;
  A.vgrid = f.vgrid;
  A.n_keys = g.n_keys;
  A.claim = f.claim;
  A.cl_list = f.cl_list;
  A.mlp = (const MlpBlob*)f.mlp_blob;
  A.closure_tol = f.closure_tol;
  A.closure_stats = f.closure_stats;
  A.log_buf = f.log_buf;
  A.log_count = f.log_count;
  A.log_cap = f.log_cap;
  A.map_out = nullptr;
  // Bookkeeping: `rd` is the list describing buf[cur] (the buffer the next
  // particle kernel reads); `wr` is the list describing the order in which
  // the current offsets place particles (the buffer the next kernel writes).
  int cur = 0, rd = 0, wr = 0, ei = 0;
  for (int step = 0; step <= n; step++) {
    A.in = f.buf[cur];
    A.out = f.buf[cur ^ 1];
    A.list = f.list[rd];
    A.list_n = f.list_n + rd;
    A.step_id = (uint32_t)(step + 1);
    // claims of step_id s go to counter s & 1 (the other is cleared by the
    // grid kernel of step s for step s + 1)
    A.cl_count = f.cl_count + ((step + 1) & 1);
    if (step == n) {
      k_particles<MODE_G2P, NT, FEAT><<<f.part_wgs, NT, 0, s>>>(A, P, g);
      cur ^= 1;
      break;
    }
    if (step == 0) {
      k_particles<MODE_P2G, NT, FEAT_NONE><<<f.part_wgs, NT, 0, s>>>(A, P, g);
    } else {
      if (ev) hipEventRecord((*ev)[2 * ei], s);
      k_particles<MODE_FUSED, NT, FEAT><<<f.part_wgs, NT, 0, s>>>(A, P, g);
      if (ev) { hipEventRecord((*ev)[2 * ei + 1], s); ei++; }
      // the state at time t0 + step now sits in the output buffer
      if (f.ck_k > 0 && (f.ck_t0 + step) % f.ck_k == 0) {
        PState ck = packed_state((float*)(f.ck_base + (size_t)((f.ck_t0 + step) / f.ck_k) * f.ck_stride), N);
        export_state(f, A.out, ck, P.mats, s);
      }
    }
    // grid update of this step; from step 1 on, workgroup 0 also scans the
    // keys the particle kernel counted (the step-0 kernel counts nothing and
    // the import's offsets stay in force)
    const int do_scan = step >= 1 ? 1 : 0;
    // three lists rotate: rd is read by this launch's grid workgroups, wr
    // describes the buffer just written (read next step), the scan fills the
    // third one
    const int nwr = (rd == wr) ? (rd + 1) % 3 : 3 - rd - wr;
    const int nrd = do_scan ? wr : rd;
    ScanArgs SA;
    SA.counts = f.counts;
    SA.offsets = f.offsets;
    SA.touched = f.touched;
    SA.n_touched = f.n_touched;
    SA.list = f.list[nwr];
    SA.list_n = f.list_n + nwr;
    SA.n_keys = g.n_keys;
    SA.split_nt = f.share_chunks > 0 ? NT : 0;
    SA.max_chunks = f.share_chunks;
    SA.order_nt = NT;
    SA.fill_slots = fill_slots;
    k_grid<<<f.grid_wgs + do_scan, 256, 0, s>>>(P, g, f.cl_list, f.cl_count + ((step + 1) & 1),
                                               f.cl_count + ((step + 2) & 1), f.tile_box, f.tiles, f.gen,
                                               (uint32_t)(step + 1), f.vgrid, pose, act, f.t0_dev, do_scan, SA, -1, nullptr);
    if (do_scan) {
      cur ^= 1;
      rd = nrd;
      wr = nwr;
    }
  }
  if (f.do_export) export_state(f, f.buf[cur], user, P.mats, s);
  f.last_buf = cur;
}

static void enqueue(FastPath& f, const StepParams& P, const PState& user, int n, const double* pose, const float* act,
                    hipStream_t s, std::vector<hipEvent_t>* ev) {
  if (f.mlp_blob) enqueue_call<256, FEAT_CLOSURE>(f, P, user, n, pose, act, s, ev);
  else if (f.log_buf) enqueue_call<256, FEAT_LOG>(f, P, user, n, pose, act, s, ev);
  else if (f.part_threads == 128) enqueue_call<128, FEAT_NONE>(f, P, user, n, pose, act, s, ev);
  else if (f.part_threads == 512) enqueue_call<512, FEAT_NONE>(f, P, user, n, pose, act, s, ev);
  else enqueue_call<256, FEAT_NONE>(f, P, user, n, pose, act, s, ev);
}

static void destroy_graph(FastGraph& G) {
  if (G.exec) hipGraphExecDestroy(G.exec);
  if (G.graph) hipGraphDestroy(G.graph);
  for (hipEvent_t e : G.ev) hipEventDestroy(e);
  G = FastGraph();
}

int fast_run(FastPath& f, const StepParams& P, const PState& user, int t0, int n, const double* pose, const float* act,
             hipStream_t s, KernelTimer* timer) {
  const FastGeom g = f.g;
  if (n < 1 || n >= 65535) return -1;
  new_epoch(f, s);
  k_set_word<<<1, 1, 0, s>>>(f.t0_dev, t0);
  // a timed call runs eagerly: its per-launch events bracket real launches
  // (events recorded inside a captured graph do not give elapsed times here)
  const bool timed = timer && timer->on;
  if (!f.use_graph || timed) {
    std::vector<hipEvent_t> ev;
    if (timed) {
      ev.resize(2 * (size_t)(n - 1));
      for (auto& e : ev) hipEventCreate(&e);
    }
    enqueue(f, P, user, n, pose, act, s, timed ? &ev : nullptr);
    if (timed) timer->adopt(ev, n - 1, true);
    return hipGetLastError() == hipSuccess ? 0 : -3;
  }
  // graph mode: one captured call per (n, state pointers, launch shape,
  // checkpoint slots), replayed with the clock taken from device memory
  FastGraph* G = nullptr;
  for (auto& c : f.graphs)
    if (c.exec && c.n == n && c.x == user.x && c.v == user.v && c.C == user.C && c.F == user.F && c.J == user.J &&
        c.mat == P.mat && c.part_threads == f.part_threads && c.part_wgs == f.part_wgs && c.grid_wgs == f.grid_wgs &&
        c.share_chunks == f.share_chunks && c.ck_k == f.ck_k && c.ck_t0 == f.ck_t0 && c.ck_base == f.ck_base &&
        c.ck_stride == f.ck_stride &&
        c.timed == timed && c.do_export == f.do_export && c.mlp == f.mlp_blob && c.log == f.log_buf &&
        c.log_count == f.log_count && c.log_cap == f.log_cap && c.tol == f.closure_tol)
      G = &c;
  if (!G) {
    FastGraph c;
    c.n = n; c.x = user.x; c.v = user.v; c.C = user.C; c.F = user.F; c.J = user.J; c.mat = P.mat;
    c.part_threads = f.part_threads; c.part_wgs = f.part_wgs; c.share_chunks = f.share_chunks;
    c.ck_k = f.ck_k; c.ck_t0 = f.ck_t0; c.ck_base = f.ck_base; c.ck_stride = f.ck_stride;
    c.grid_wgs = f.grid_wgs; c.timed = timed; c.do_export = f.do_export;
    c.mlp = f.mlp_blob; c.log = f.log_buf; c.log_count = f.log_count; c.log_cap = f.log_cap; c.tol = f.closure_tol;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return -3;
    enqueue(f, P, user, n, pose, act, s, nullptr);
    if (hipStreamEndCapture(s, &c.graph) != hipSuccess) { destroy_graph(c); return -3; }
    if (hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0) != hipSuccess) { destroy_graph(c); return -3; }
    if (f.graphs.size() >= 8) { destroy_graph(f.graphs.front()); f.graphs.erase(f.graphs.begin()); }
    f.graphs.push_back(c);
    G = &f.graphs.back();
  }
  if (hipGraphLaunch(G->exec, s) != hipSuccess) return -3;
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

uint32_t fast_next_sid(FastPath& f) { return ++f.sid; }

// workgroup size of the kernels that read the lists of sorted states (the
// records' forward kernels and the tiled adjoint's)
constexpr int SORTED_NT = 256;

void fast_sort_user(FastPath& f, const StepParams& P, const PState& user, SortedState& out, hipStream_t s,
                    bool touched) {
  const int N = f.N;
  new_epoch(f, s);
  k_import_keys<<<nblk(N, 256), 256, 0, s>>>(user, P, f.g, f.cpad, f.key_tmp, f.rank_tmp, f.touched, f.n_touched);
  k_scan<<<1, 1024, 0, s>>>(f.cpad, f.offsets, f.touched, f.n_touched, out.list, out.list_n, f.g.n_keys, f.gen,
                            out.cl_count ? out.cl_count : f.cl_count, touched ? SCAN_TOUCHED : SCAN_DENSE,
                            IMPORT_PAD, 0, 0, SORTED_NT, 0);
  import_permute(f, user, P.mat, out.b, s);
}

void fast_sort_next(FastPath& f, const StepParams& P, const SortedState& prev, const PBuf& next, SortedState& out,
                    uint32_t* map, hipStream_t s, bool touched) {
  const int N = f.N;
  new_epoch(f, s);
  k_keys_next<<<nblk(N, 256), 256, 0, s>>>(next.f, prev.b.key, N, P, f.g, f.counts, f.key_tmp, f.rank_tmp,
                                           touched ? f.touched : nullptr, f.n_touched);
  k_scan<<<1, 1024, 0, s>>>(f.counts, f.offsets, f.touched, f.n_touched, out.list, out.list_n, f.g.n_keys, f.gen,
                            out.cl_count ? out.cl_count : f.cl_count, touched ? SCAN_TOUCHED : SCAN_DENSE, 1, 0, 0,
                            SORTED_NT, 0);
  k_sort_permute<<<nblk(N, 256), 256, 0, s>>>(next, out.b, N, f.key_tmp, f.rank_tmp, f.offsets, map);
}

static PartArgs sorted_args(FastPath& f, const SortedState& st, uint32_t sid) {
  PartArgs A = {};
  A.in = st.b;
  A.out = st.b;
  A.N = f.N;
  A.list = st.list;
  A.list_n = st.list_n;
  A.offsets = f.offsets;
  A.counts = f.counts;
  A.touched = f.touched;
  A.n_touched = f.n_touched;
  A.tiles = f.tiles;
  A.tile_box = f.tile_box;
  A.n_keys = f.g.n_keys;
  A.claim = f.claim;
  A.cl_list = st.cl_list ? st.cl_list : f.cl_list;
  A.cl_count = st.cl_count ? st.cl_count : f.cl_count;
  A.gen = f.gen;
  A.step_id = sid;
  A.vgrid = st.vgrid ? st.vgrid : f.vgrid;
  return A;
}

void fast_p2g(FastPath& f, const StepParams& P, const SortedState& st, uint32_t sid, hipStream_t s) {
  PartArgs A = sorted_args(f, st, sid);
  k_particles<MODE_P2G, 256, FEAT_NONE><<<f.part_wgs, 256, 0, s>>>(A, P, f.g);
}

void fast_fused(FastPath& f, const StepParams& P, const SortedState& in, const SortedState& out, uint32_t* map,
                uint32_t sid, hipStream_t s) {
  PartArgs A = sorted_args(f, in, sid);
  A.out = out.b;
  A.cl_list = out.cl_list ? out.cl_list : f.cl_list;
  A.cl_count = out.cl_count ? out.cl_count : f.cl_count;
  A.map_out = map;
  k_particles<MODE_FUSED, 256, FEAT_NONE><<<f.part_wgs, 256, 0, s>>>(A, P, f.g);
}

void fast_grid_scan(FastPath& f, const StepParams& P, const SortedState& st, uint32_t sid, int t,
                    const double* pose_base, const float* act_base, uint32_t* cl_zero, int4* scan_list,
                    uint32_t* scan_list_n, hipStream_t s) {
  ScanArgs SA = {};
  SA.counts = f.counts;
  SA.offsets = f.offsets;
  SA.touched = f.touched;
  SA.n_touched = f.n_touched;
  SA.list = scan_list;
  SA.list_n = scan_list_n;
  SA.n_keys = f.g.n_keys;
  SA.split_nt = 0;       // the adjoint's records list each block once
  SA.max_chunks = 0;
  SA.order_nt = SORTED_NT;
  SA.fill_slots = 0;
  const int do_scan = scan_list ? 1 : 0;
  k_grid<<<f.grid_wgs + do_scan, 256, 0, s>>>(P, f.g, st.cl_list ? st.cl_list : f.cl_list,
                                              st.cl_count ? st.cl_count : f.cl_count, cl_zero, f.tile_box, f.tiles,
                                              f.gen, sid, st.vgrid ? st.vgrid : f.vgrid, pose_base, act_base, f.t0_dev,
                                              do_scan, SA, t, st.mmv);
}

void fast_grid(FastPath& f, const StepParams& P, const SortedState& st, uint32_t sid, int t, const double* pose_base,
               const float* act_base, hipStream_t s) {
  ScanArgs SA = {};
  k_grid<<<f.grid_wgs, 256, 0, s>>>(P, f.g, st.cl_list ? st.cl_list : f.cl_list, st.cl_count ? st.cl_count : f.cl_count,
                                    nullptr, f.tile_box, f.tiles, f.gen,
                                    sid, st.vgrid ? st.vgrid : f.vgrid, pose_base, act_base, f.t0_dev, 0, SA, t, st.mmv);
}

// the G2P kernel writes row j to offsets[key[j]] + rank[j], which is j itself
// while the offsets are those of st's own sort (the latest one)
void fast_g2p(FastPath& f, const StepParams& P, const SortedState& st, const PBuf& out, hipStream_t s) {
  PartArgs A = sorted_args(f, st, 0);
  A.out = out;
  k_particles<MODE_G2P, 256, FEAT_NONE><<<f.part_wgs, 256, 0, s>>>(A, P, f.g);
}

SortedState fast_own_state(FastPath& f, int b) {
  SortedState S = {};
  S.b = f.buf[b];
  S.list = f.list[b];
  S.list_n = f.list_n + b;
  return S;
}

int fast_sort_snapshot(FastPath& f, const StepParams& P, const PState& user, int which, uint32_t* id_out,
                       uint32_t* key_out, int4* list_out, int* n_list_host, hipStream_t s) {
  const size_t N = (size_t)f.N;
  if (which == 0 || which == 2) {
    SortedState st = fast_own_state(f, 0);
    fast_sort_user(f, P, user, st, s, which == 0);
    f.last_buf = -1;   // buffer 0 no longer holds the last call's state
    uint32_t nl = 0;
    if (hipMemcpyAsync(id_out, st.b.id, N * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(key_out, st.b.key, N * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(list_out, st.list, (size_t)f.g.n_keys * sizeof(int4), hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(&nl, st.list_n, 4, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      return -3;
    *n_list_host = (int)nl;
    return 0;
  }
  if (f.last_buf < 0) return -1;
  if (hipMemcpyAsync(id_out, f.buf[f.last_buf].id, N * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return -3;
  return 0;
}

void fast_export(FastPath& f, const StepParams& P, const PBuf& X, const PState& user, hipStream_t s) {
  export_state(f, X, user, P.mats, s);
}

void fast_destroy(FastPath& f) {
  for (auto& c : f.graphs) destroy_graph(c);
  f.graphs.clear();
}

void fast_invalidate(FastPath& f) {
  for (auto& c : f.graphs) destroy_graph(c);
  f.graphs.clear();
}

}  // namespace mpm
