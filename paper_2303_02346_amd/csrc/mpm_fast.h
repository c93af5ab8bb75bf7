// Forward path used by mpm_step: particles kept sorted by grid block, a
// fused grid-to-particle / particle-to-grid kernel accumulating into LDS
// tiles, and a sparse grid update that gathers the tiles.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <vector>
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
// Tile slots per block key: the forward lists a block of more than two
// chunks twice, and the second workgroup publishes its tile in slot
// key + n_keys (the adjoint uses slot key only).
constexpr int NSUB = 2;

// Particle buffer: packed state (25 rows of N floats) plus bookkeeping.
struct PBuf {
  float* f;       // 25 x N
  uint32_t* id;   // original particle index
  uint32_t* key;  // block key of the particle's current position
  uint32_t* rank; // rank within that key
  uint8_t* mat;
};

// A captured call (graph mode).
struct FastGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int n = 0, part_threads = 0, part_wgs = 0, grid_wgs = 0, share_chunks = 0;
  // the checkpoints the call writes (slots from its start time)
  int ck_k = 0, ck_t0 = 0;
  char* ck_base = nullptr;
  size_t ck_stride = 0;
  bool timed = false, do_export = true;
  // every user pointer and logging argument the captured launches bake in
  const float *x = nullptr, *v = nullptr, *C = nullptr, *F = nullptr, *J = nullptr;
  const uint8_t* mat = nullptr;
  const void* mlp = nullptr;
  const float* log = nullptr;
  const unsigned long long* log_count = nullptr;
  unsigned long long log_cap = 0;
  float tol = 0.f;
  std::vector<hipEvent_t> ev;   // fused-kernel event pairs recorded by the graph
};

struct FastPath {
  char* ws;
  FastGeom g;
  int N;
  PBuf buf[2];
  uint32_t *key_tmp, *rank_tmp;
  uint32_t* inv;           // slot -> user index (import) or user index -> slot (export)
  uint32_t* cpad;          // the import's key counters, 64 bytes apart
  uint32_t *counts, *offsets;
  uint32_t *touched, *n_touched;   // keys counted in the current step, in first-touch order
  int4* list[3];           // occupied-block lists (rotating; up to NSUB entries per key)
  uint32_t* list_n;        // [3]
  uint32_t* claim;         // per-block stamp: which step last updated the block
  uint32_t* cl_list;       // keys of the blocks claimed in the current step
  uint32_t* cl_count;      // [2]: claims of odd and even step ids
  int2* tile_box;          // {packed lo/hi, stamp} per tile slot
  float* tiles;            // NSUB n_keys slots of 4 TILE_NODES floats (forward: a float4 (m, mv) per node)
  float4* vgrid;           // n_keys x 64
  uint32_t* gen;           // device per-call epoch of the step stamps
  int* t0_dev;             // device clock at the start of the call
  unsigned long long calls;
  // launch shape and mode (set by mpm_set_option / the autotuner)
  int part_threads;        // 128, 256 or 512 threads (particles per chunk) per particle workgroup
  int share_chunks;        // a block of more chunks than this is shared by two workgroups (0: never)
  int fused_slots;         // resident 256-thread workgroups of the fused kernel (CUs x occupancy)
  bool use_graph;          // capture each call shape once and replay it
  bool do_export;          // write the result back to the user arrays
  std::vector<FastGraph> graphs;
  // learned closure (device MLP blob, residual tolerance, counters) and
  // cone-case sample logging
  const void* mlp_blob;
  float closure_tol;
  unsigned long long* closure_stats;
  float* log_buf;
  unsigned long long* log_count;
  unsigned long long log_cap;
  int grid_wgs, part_wgs;
  // checkpoints written inside a call (requires_grad contexts): the state at
  // every time t0 + s with (t0 + s) % ck_k == 0, 0 < s < n, goes to slot
  // (t0 + s) / ck_k of ck_base (user order, ck_stride bytes apart); ck_k = 0: none
  char* ck_base;
  size_t ck_stride;
  int ck_k, ck_t0;
  // plain dense grid (shared with the adjoint path), unused here
  float4* mmv;
  float4* vdense;
  bool valid;
  uint32_t sid;            // last step id handed out under the current epoch
  int last_buf = -1;       // sorted buffer holding the state after the last call
};

// A state sorted by the block key of its own positions (the tiled adjoint
// keeps one per step of a checkpoint segment).
struct SortedState {
  PBuf b;                  // f (25 x N), id (user index), key, rank, mat
  int4* list;              // occupied blocks {key, offset, count, 0}
  uint32_t* list_n;
  // the step's grid, kept for the adjoint (block layout; NULL = the path's
  // shared arrays): updated velocities and masses, node momenta and masses,
  // and the list and number of the blocks claimed by its P2G
  float4* vgrid;
  float4* mmv;
  uint32_t* cl_list;
  uint32_t* cl_count;      // [2]
};

size_t fast_workspace_bytes(int n_grid, int n_scenes, int N);
int fast_n_keys(int n_grid, int n_scenes);
int fast_init(FastPath& f, char* ws, int n_grid, int n_scenes, int N, hipStream_t s);
void fast_bind_grid(FastPath& f, float4* mmv, float4* vgrid);
void fast_invalidate(FastPath& f);
int fast_run(FastPath& f, const StepParams& P, const PState& user, int t0, int n, const double* pose, const float* act,
             hipStream_t s, KernelTimer* timer);
void fast_destroy(FastPath& f);

// Building blocks of the tiled adjoint.  fast_sort_user sorts a user-order
// state (and starts a new stamp epoch); fast_sort_next sorts the state that
// fast_g2p produced from `prev` (same row order as prev) and records in
// map[j] the new row of prev's row j.  fast_p2g / fast_grid / fast_g2p run
// one forward step's parts on a sorted state: P2G tiles and block claims
// under step id `sid` (from fast_next_sid), the grid update of step t (with
// st.mmv, also the node momenta and masses), and G2P into `out` in the same
// row order.  The sorts scan the keys they counted; the blocks are listed in
// key (Morton) order unless `touched` is set: then in first-touch order.
uint32_t fast_next_sid(FastPath& f);
void fast_sort_user(FastPath& f, const StepParams& P, const PState& user, SortedState& out, hipStream_t s,
                    bool touched = false);
void fast_sort_next(FastPath& f, const StepParams& P, const SortedState& prev, const PBuf& next, SortedState& out,
                    uint32_t* map, hipStream_t s, bool touched = false);
void fast_p2g(FastPath& f, const StepParams& P, const SortedState& st, uint32_t sid, hipStream_t s);
void fast_grid(FastPath& f, const StepParams& P, const SortedState& st, uint32_t sid, int t, const double* pose_base,
               const float* act_base, hipStream_t s);
void fast_g2p(FastPath& f, const StepParams& P, const SortedState& st, const PBuf& out, hipStream_t s);
// The fused kernel on records: G2P of step t - 1 from `in` (with in's grid),
// the update, and P2G of step t, the state written to `out` in the slots of
// the latest scan (so `out` is sorted by the block keys of in's positions,
// one step behind its own; map[j] = out's row of in's row j), its tiles under
// `sid` and its block claims into out's claim list; the keys of the new
// positions are counted for the next scan.  fast_grid_scan is fast_grid that
// also clears the claim counter cl_zero and, with scan_list, scans those
// counts into scan_list (each block listed once).
void fast_fused(FastPath& f, const StepParams& P, const SortedState& in, const SortedState& out, uint32_t* map,
                uint32_t sid, hipStream_t s);
void fast_grid_scan(FastPath& f, const StepParams& P, const SortedState& st, uint32_t sid, int t,
                    const double* pose_base, const float* act_base, uint32_t* cl_zero, int4* scan_list,
                    uint32_t* scan_list_n, hipStream_t s);
// The path's own sorted state over buffer b (0 or 1) and list b, using the
// path's shared grid arrays; and the scatter of a sorted buffer to user order.
SortedState fast_own_state(FastPath& f, int b);
// Integer outputs of the block sort (for checking it): which = 0 sorts the
// user state (the import of every call) and copies the sorted ids and keys
// (N each) and the occupied-block list (n_keys rows) to the given device
// arrays and the list length to *n_list_host; which = 2 the same with the
// blocks in key order (the adjoint's sorts); which = 1 copies the ids of
// the buffer the last call left.  Returns 0, or -1 (nothing recorded yet).
int fast_sort_snapshot(FastPath& f, const StepParams& P, const PState& user, int which, uint32_t* id_out,
                       uint32_t* key_out, int4* list_out, int* n_list_host, hipStream_t s);
void fast_export(FastPath& f, const StepParams& P, const PBuf& X, const PState& user, hipStream_t s);

}  // namespace mpm
