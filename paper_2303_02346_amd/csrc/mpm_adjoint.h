// Tiled adjoint of one MLS-MPM step on a block-sorted state (mpm_adjoint.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "mpm_fast.h"
#include "mpm_internal.h"

namespace mpm {

struct AdjArgs {
  PBuf st;                   // s_t sorted by its own block key
  const int4* list;          // its occupied blocks
  const uint32_t* list_n;
  int N;
  const float* abar_next;    // adjoint of s_{t+1}, packed 25 x N
  const uint32_t* map;       // row of particle j (s_t's order) in abar_next
  float* abar;               // adjoint of s_t in s_t's order, packed 25 x N
  const float4* vgrid;       // updated node velocities of step t (block layout)
  float* tiles;              // per-block tile slots (velocity-adjoint tiles)
  int2* tile_box;
  const uint32_t* gen;       // stamp epoch
  uint32_t sid;              // stamp step id of the velocity-adjoint tiles
  const uint32_t* cl_list;   // blocks claimed by the recompute of step t
  const uint32_t* cl_count;
  const float4* mmv;         // node momenta and masses of step t (block layout)
  float4* mmvb;              // their adjoints (block layout)
  // particles whose FP32 adjoint is ill-conditioned, {row, block key}, for
  // the FP64 pass; the count starts at zero (one counter per step and kernel)
  uint32_t* redo_n;
  uint2* redo;               // room for N entries
};

void launch_g2p_adj_tiled(const AdjArgs& A, const StepParams& P, const FastGeom& g, int n_wgs, hipStream_t s);
void launch_grid_adj_tiled(const AdjArgs& A, const StepParams& P, const FastGeom& g, int n_wgs, const double* pose_t,
                           const float* act_t, double* acc_t, hipStream_t s);
void launch_p2g_adj_tiled(const AdjArgs& A, const StepParams& P, const FastGeom& g, int n_wgs, hipStream_t s);
// adjoint rows in sorted order (row j of particle id[j]) -> user order; pos:
// N words of scratch
void launch_adj_reorder(const float* in, float* out, const uint32_t* id, int N, uint32_t* pos, hipStream_t s);
// map[j] = the row of particle prev_id[j] in the order cur_id lists (pos: N
// words of scratch); a map past N marks an id that is out of range
void launch_row_map(const uint32_t* prev_id, const uint32_t* cur_id, int N, uint32_t* pos, uint32_t* map,
                    hipStream_t s);
// dst[0 .. n) = src[0 .. n) and *dst_n = n, for n = *src_n (a block list and
// its length; dst holds as many rows as src)
void launch_copy_list(const int4* src, const uint32_t* src_n, int4* dst, uint32_t* dst_n, hipStream_t s);

}  // namespace mpm
