// Block keys of the tiled path (4^3-node grid blocks keyed by scene and the
// Morton code of the block coordinates) and the wavefront-level rank
// reservation used by the counting sort of the particles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "mpm_fast.h"

namespace mpm {

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

// Reductions over the 64 lanes of a wavefront without LDS: DPP lane moves
// within each row of 16 lanes (swap of neighbours, swap of pairs, mirror of
// each half row, mirror of the row) leave every lane with its row's result,
// and the four rows are combined from readlanes.  Every lane of the wave must
// be active.
namespace dpp {
constexpr int kSwap1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kSwap2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kHalfMirror = 0x141;  // row_half_mirror
constexpr int kMirror = 0x140;      // row_mirror
template <int CTRL> __device__ __forceinline__ int mov(int x) { return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false); }
}  // namespace dpp

__device__ __forceinline__ float wave_sum(float x) {
  x += __int_as_float(dpp::mov<dpp::kSwap1>(__float_as_int(x)));
  x += __int_as_float(dpp::mov<dpp::kSwap2>(__float_as_int(x)));
  x += __int_as_float(dpp::mov<dpp::kHalfMirror>(__float_as_int(x)));
  x += __int_as_float(dpp::mov<dpp::kMirror>(__float_as_int(x)));
  const int xi = __float_as_int(x);
  return (__int_as_float(__builtin_amdgcn_readlane(xi, 0)) + __int_as_float(__builtin_amdgcn_readlane(xi, 16))) +
         (__int_as_float(__builtin_amdgcn_readlane(xi, 32)) + __int_as_float(__builtin_amdgcn_readlane(xi, 48)));
}

__device__ __forceinline__ uint32_t wave_or(uint32_t x) {
  int v = (int)x;
  v |= dpp::mov<dpp::kSwap1>(v);
  v |= dpp::mov<dpp::kSwap2>(v);
  v |= dpp::mov<dpp::kHalfMirror>(v);
  v |= dpp::mov<dpp::kMirror>(v);
  return (uint32_t)(__builtin_amdgcn_readlane(v, 0) | __builtin_amdgcn_readlane(v, 16) |
                    __builtin_amdgcn_readlane(v, 32) | __builtin_amdgcn_readlane(v, 48));
}

// Rank of each lane's key among equal keys of the wavefront, in two phases
// so that the global atomic's latency overlaps other work: rank_issue groups
// the lanes by key (ballots only) and lets one leader lane per distinct key
// reserve the group's range; rank_finish broadcasts the leader's base.
// Every lane of the wave must call both.
struct WaveRank {
  int leader;
  uint32_t prefix;
  uint32_t lbase;
  bool lead;      // this lane reserved its key's range
  uint32_t key;
};
__device__ inline WaveRank rank_issue(uint32_t* counts, uint32_t key, bool valid) {
  const int lane = __lane_id();
  unsigned long long pending = __ballot(valid);
  WaveRank R;
  R.leader = lane;
  R.prefix = 0;
  R.lbase = 0;
  R.key = key;
  uint32_t lcount = 0;
  while (pending) {
    int leader = __ffsll((long long)pending) - 1;
    const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
    unsigned long long m = __ballot(valid && key == k) & pending;
    if ((m >> lane) & 1ull) { R.leader = leader; R.prefix = (uint32_t)__popcll(m & ((1ull << lane) - 1ull)); }
    if (lane == leader) lcount = (uint32_t)__popcll(m);
    pending &= ~m;
  }
  R.lead = lcount > 0;
  if (R.lead) R.lbase = atomicAdd(&counts[key], lcount);
  return R;
}
// The key's first reservation in the step (base 0) also appends the key to
// the list of touched keys, which is what the scan works through.
__device__ inline void touch_key(uint32_t key, uint32_t* touched, uint32_t* n_touched, uint32_t n_keys) {
  const uint32_t slot = atomicAdd(n_touched, 1u);
  if (slot < n_keys) touched[slot] = key;
}
// (touched == NULL: no list is kept, for a scan over all keys)
__device__ inline uint32_t rank_finish(const WaveRank& R, uint32_t* touched, uint32_t* n_touched, uint32_t n_keys) {
  if (touched && R.lead && R.lbase == 0) touch_key(R.key, touched, n_touched, n_keys);
  return __shfl(R.lbase, R.leader) + R.prefix;
}

// Rank of each lane's key among equal keys of the wavefront, with one global
// atomic per distinct key, all issued together (one round trip however many
// distinct keys the wavefront holds).  Every lane of the wave must call it.
__device__ inline uint32_t wave_rank(uint32_t* counts, uint32_t key, bool valid, uint32_t* touched, uint32_t* n_touched,
                                     uint32_t n_keys) {
  return rank_finish(rank_issue(counts, key, valid), touched, n_touched, n_keys);
}

__device__ inline void load_state(const PBuf& b, int N, int j, float* x, float* v, float* C, float* F, float& J) {
#pragma unroll
  for (int a = 0; a < 3; a++) { x[a] = b.f[a * (size_t)N + j]; v[a] = b.f[(3 + a) * (size_t)N + j]; }
#pragma unroll
  for (int k = 0; k < 9; k++) C[k] = b.f[(6 + k) * (size_t)N + j];
}

}  // namespace mpm
