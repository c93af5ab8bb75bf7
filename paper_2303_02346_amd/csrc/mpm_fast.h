// Forward path used by mpm_step: particles kept sorted by grid block, a
// fused grid-to-particle / particle-to-grid kernel accumulating into LDS
// tiles, and a sparse grid update that gathers the tiles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "mpm_internal.h"

namespace mpm {

// Block geometry: 4^3-node blocks, keyed by scene and the Morton code of the
// block coordinates.
struct FastGeom {
  int n;        // nodes per axis
  int nb;       // blocks per axis
  int kb;       // Morton bits per axis
  int S;        // scenes
  int n_keys;   // S << (3 kb)
};

constexpr int TILE = 10;                     // P2G tile edge (nodes): block +-2 layers of drift
constexpr int TILE_NODES = TILE * TILE * TILE;
constexpr int VT = 8;                        // G2P velocity tile edge
constexpr int VT_NODES = VT * VT * VT;

// Particle buffer: packed state (25 rows of N floats) plus bookkeeping.
struct PBuf {
  float* f;       // 25 x N
  uint32_t* id;   // original particle index
  uint32_t* key;  // block key of the particle's current position
  uint32_t* rank; // rank within that key
  uint8_t* mat;
};

struct FastPath {
  char* ws;
  FastGeom g;
  int N;
  PBuf buf[2];
  uint32_t *key_tmp, *rank_tmp;
  uint32_t *counts, *offsets;
  int4* list[3];           // occupied-block lists (rotating)
  uint32_t* list_n;        // [3]
  uint32_t* claim;         // per-block stamp: which step last updated the block
  uint32_t* won;           // per list entry: mask of the neighbour blocks it claimed
  int2* tile_box;          // {packed lo/hi, stamp}
  float* tiles;            // n_keys x 4 x TILE_NODES
  float4* vgrid;           // n_keys x 64
  uint32_t* gen;           // device per-call epoch of the step stamps
  unsigned long long calls;
  int grid_wgs, part_wgs;
  // plain dense grid (shared with the adjoint path), unused here
  float4* mmv;
  float4* vdense;
  bool valid;
};

size_t fast_workspace_bytes(int n_grid, int n_scenes, int N);
int fast_init(FastPath& f, char* ws, int n_grid, int n_scenes, int N, hipStream_t s);
void fast_bind_grid(FastPath& f, float4* mmv, float4* vgrid);
void fast_invalidate(FastPath& f);
int fast_run(FastPath& f, const StepParams& P, const PState& user, int t0, int n, const double* pose, const float* act,
             hipStream_t s, KernelTimer* timer);
void fast_destroy(FastPath& f);

}  // namespace mpm
