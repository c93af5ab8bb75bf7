// C ABI of the MLS-MPM step (declared in include/mpm.h): workspace planning,
// context state, step/backward orchestration and error handling.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>
#include <new>
#include <vector>

#include "../../include/mpm.h"
#include "mpm_internal.h"
#include "mpm_adjoint.h"
#include "mpm_fast.h"
#include "mpm_rigid.h"

using namespace mpm;

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

// Per-step record of a block-sorted segment state of the tiled adjoint
// (offsets relative to the record's start).
struct SortedRec {
  size_t f, id, key, rank, mat, map, list, list_n, vgrid, mmv, cl_list, cl_count, bytes;
  bool has_grid;
};

// with_grid: the record also keeps its step's grid for the adjoint
SortedRec sorted_rec(size_t N, size_t n_keys, bool with_grid) {
  SortedRec r;
  r.has_grid = with_grid;
  size_t o = 0;
  auto take = [&](size_t b) { size_t q = o; o += align_up(b); return q; };
  r.vgrid = with_grid ? take(n_keys * 64 * sizeof(float4)) : 0;
  r.mmv = with_grid ? take(n_keys * 64 * sizeof(float4)) : 0;
  r.cl_list = with_grid ? take(n_keys * 4) : 0;
  r.cl_count = with_grid ? take(16) : 0;
  r.f = take(STATE_FLOATS * N * sizeof(float));
  r.id = take(N * 4);
  r.key = take(N * 4);
  r.rank = take(N * 4);
  r.mat = take(N);
  r.map = take(N * 4);
  r.list = take(n_keys * 16);
  r.list_n = take(16);
  r.bytes = o;
  return r;
}

struct Layout {
  size_t mats, offs, pscene, cyl_radius, err, mmv, vgrid, vbar, mmvb, pose, act, acc, ckpt, seg, adj0, adj1, scratch;
  size_t fast, cstats;
  size_t tmp, mmvb_blk;   // tiled adjoint: G2P output, node adjoints of (mv, m)
  size_t redo_n, redo;    // tiled adjoint: FP64-pass counters (two per step) and list
  SortedRec rec, tmp_rec;
  // rigid bodies: rest offsets, material -> body table, body constants,
  // sums, per-step projection records, adjoint terms, set-up sums, status
  size_t r_rest, r_body_of, r_bodies, r_acc, r_rec, r_adj, r_rest_acc, r_status;
  int n_bodies, n_rec;
  size_t total;
  int n_ckpt;
};

int count_bodies(const mpm_desc* d) {
  int n = 0;
  for (int m = 0; m < d->n_materials; m++) n += d->materials[m].kind == MPM_RIGID ? 1 : 0;
  return n;
}

bool desc_ok(const mpm_desc* d) {
  if (!d) return false;
  if (d->n_grid < 8 || d->n_grid > 1024) return false;
  if (d->n_particles < 1 || d->n_materials < 1 || d->n_materials > 256 || !d->materials) return false;
  if (d->n_scenes < 1) return false;
  if (d->n_scenes > 1 && !d->scene_offsets) return false;
  if (!d->cyl_radius || !d->cyl_pos0 || !d->cyl_rot0) return false;
  if (!(d->dt > 0.f) || d->horizon < 1 || d->bound < 0) return false;
  // (the tiled adjoint hands out 2 k + 1 step stamps per 16-bit epoch)
  if (d->requires_grad && (d->ckpt_every < 0 || d->ckpt_every > 16384)) return false;
  // (ckpt_every = 0, a record of every step, is the tiled adjoint's; rigid
  // bodies need the checkpointed recompute)
  if (d->requires_grad && d->ckpt_every == 0 && count_bodies(d) > 0) return false;
  if (d->scene_offsets) {
    if (d->scene_offsets[0] != 0 || d->scene_offsets[d->n_scenes] != d->n_particles) return false;
    for (int s = 0; s < d->n_scenes; s++)
      if (d->scene_offsets[s + 1] < d->scene_offsets[s]) return false;
  }
  size_t nodes = (size_t)d->n_grid * d->n_grid * d->n_grid * d->n_scenes;
  if (nodes > ((size_t)1 << 34)) return false;
  return true;
}

Layout plan(const mpm_desc* d) {
  Layout L;
  size_t N = d->n_particles, S = d->n_scenes, T = d->horizon;
  size_t nodes = (size_t)d->n_grid * d->n_grid * d->n_grid * S;
  size_t st = align_up(STATE_FLOATS * N * sizeof(float));
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o += align_up(b); return r; };
  L.mats = take(256 * sizeof(MatDev));
  L.offs = take((S + 1) * sizeof(int64_t));
  L.pscene = take(N * sizeof(int));
  L.cyl_radius = take(S * sizeof(float));
  L.err = take(64);
  L.mmv = take(nodes * sizeof(float4));
  L.vgrid = take(nodes * sizeof(float4));
  L.pose = take((T + 1) * S * POSE_DOUBLES * sizeof(double));
  L.act = take(T * S * 6 * sizeof(float));
  L.scratch = take((2 + 2 * LOSS_SLOTS) * sizeof(double));
  L.cstats = take(64);
  L.fast = take(fast_workspace_bytes(d->n_grid, (int)S, (int)N));
  if (d->requires_grad) {
    const int k = d->ckpt_every;
    const bool keep_all = k == 0;   // a block-sorted record of every step, no recompute
    L.n_ckpt = keep_all ? 1 : (int)((T + k - 1) / k) + 1;
    L.vbar = take(nodes * sizeof(float4));
    L.mmvb = take(nodes * sizeof(float4));
    L.acc = take(T * S * ACC_DOUBLES * sizeof(double));
    L.ckpt = take(st * L.n_ckpt);
    // the plain adjoint's k + 1 segment states and the tiled adjoint's k
    // sorted records share one region
    size_t n_keys = (size_t)fast_n_keys(d->n_grid, (int)S);
    L.rec = sorted_rec(N, n_keys, true);
    L.tmp_rec = sorted_rec(N, n_keys, false);
    size_t plain_seg = keep_all ? 0 : st * (size_t)(k + 1), tiled_seg = L.rec.bytes * (size_t)(keep_all ? T : k);
    L.seg = take(plain_seg > tiled_seg ? plain_seg : tiled_seg);
    L.tmp = take(L.tmp_rec.bytes);
    L.mmvb_blk = take(n_keys * 64 * sizeof(float4));
    L.redo_n = take(2 * T * sizeof(uint32_t));
    L.redo = take(N * sizeof(uint2));
    L.adj0 = take(st);
    L.adj1 = take(st);
  } else {
    L.n_ckpt = 0;
    L.vbar = L.mmvb = L.acc = L.ckpt = L.seg = L.adj0 = L.adj1 = 0;
    L.tmp = L.mmvb_blk = L.redo_n = L.redo = 0;
    L.rec = L.tmp_rec = SortedRec{};
  }
  L.n_bodies = count_bodies(d);
  L.n_rec = (d->requires_grad && d->ckpt_every > 0) ? d->ckpt_every : 1;
  if (L.n_bodies > 0) {
    size_t B = L.n_bodies;
    L.r_rest = take(3 * N * sizeof(float));
    L.r_body_of = take(256 * sizeof(int));
    L.r_bodies = take(B * sizeof(RigidBody));
    L.r_acc = take((size_t)RIGID_SLOTS * B * RIGID_ACC * sizeof(double));
    L.r_rec = take((size_t)L.n_rec * B * RIGID_REC * sizeof(double));
    L.r_adj = take(B * sizeof(RigidAdjTerms));
    L.r_rest_acc = take(B * 16 * sizeof(double));
    L.r_status = take(64);
  } else {
    L.r_rest = L.r_body_of = L.r_bodies = L.r_acc = L.r_rec = L.r_adj = L.r_rest_acc = L.r_status = 0;
  }
  L.total = o;
  return L;
}

}  // namespace

struct mpm_ctx {
  mpm_desc d;
  Layout L;
  hipStream_t stream;
  char* ws;
  std::vector<MatDev> mats;
  std::vector<float> cyl_pos0, cyl_rot0, cyl_radius;
  std::vector<char> act_set;
  mpm_state user;
  bool has_state;
  int t;
  int last_err_bits;
  size_t state_bytes;
  FastPath fast;
  KernelTimer timer;
  bool plain_adjoint;
  RigidCtx rigid;           // n_bodies = 0: no rigid bodies
  // captured calls (graph mode), keyed by their start, steps, pointers and
  // launch shape: the tiled backward without rigid bodies (bgraphs: the
  // horizon and the gradient pointers) and the forward of a context that
  // keeps every step's record (rgraphs: start, steps and state pointers)
  struct CallGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int t0 = 0, n = 0, part_wgs = 0, grid_wgs = 0;
    const void* ptr[11] = {};
    unsigned long long n_ep = 0;   // stamp epochs one call advances
  };
  std::vector<CallGraph> bgraphs, rgraphs;
};

static void destroy_call_graph(mpm_ctx::CallGraph& G) {
  if (G.exec) hipGraphExecDestroy(G.exec);
  if (G.graph) hipGraphDestroy(G.graph);
  G.exec = nullptr;
  G.graph = nullptr;
}

// Run the work that enq() puts on the context's stream as a graph: captured
// the first time `key` is seen (the newest 4 kept in `cache`), replayed
// after.  The captured sorts advance the device epoch of the step stamps; the
// host keeps its count in step, clearing the stamps before a replay that
// crosses the epoch's 16-bit wrap.
template <class Enq>
static int graph_call(mpm_ctx* c, std::vector<mpm_ctx::CallGraph>& cache, const mpm_ctx::CallGraph& key, Enq enq) {
  FastPath& f = c->fast;
  hipStream_t s = c->stream;
  mpm_ctx::CallGraph* G = nullptr;
  for (auto& g : cache) {
    bool same = g.exec && g.t0 == key.t0 && g.n == key.n && g.part_wgs == key.part_wgs && g.grid_wgs == key.grid_wgs;
    for (int q = 0; q < 11 && same; q++) same = g.ptr[q] == key.ptr[q];
    if (same) G = &g;
  }
  if (!G) {
    mpm_ctx::CallGraph g = key;
    g.graph = nullptr;
    g.exec = nullptr;
    const unsigned long long calls0 = f.calls;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return MPM_EHIP;
    const int rc = enq();
    const hipError_t ec = hipStreamEndCapture(s, &g.graph);
    if (rc != MPM_OK || ec != hipSuccess || hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0) != hipSuccess) {
      f.calls = calls0;   // nothing of the capture ran
      destroy_call_graph(g);
      return rc != MPM_OK ? rc : MPM_EHIP;
    }
    g.n_ep = f.calls - calls0;
    if (cache.size() >= 4) { destroy_call_graph(cache.front()); cache.erase(cache.begin()); }
    cache.push_back(g);
    G = &cache.back();
  } else {
    if ((f.calls & 0xffffull) + G->n_ep >= 0x10000ull) {
      launch_zero(f.claim, (size_t)f.g.n_keys * 4, s);
      launch_zero(f.tile_box, (size_t)f.g.n_keys * NSUB * 8, s);
    }
    f.calls += G->n_ep;
  }
  if (hipGraphLaunch(G->exec, s) != hipSuccess) return MPM_EHIP;
  return hipGetLastError() == hipSuccess ? MPM_OK : MPM_EHIP;
}

// Projection record slot i of the rigid bodies.
static double* rigid_rec(mpm_ctx* c, int i) {
  return (double*)(c->ws + c->L.r_rec) + (size_t)i * c->L.n_bodies * RIGID_REC;
}

static int hip_ok(hipError_t e) { return e == hipSuccess ? MPM_OK : MPM_EHIP; }

static StepParams make_params(mpm_ctx* c) {
  StepParams P;
  P.n_grid = c->d.n_grid;
  P.n_scenes = c->d.n_scenes;
  P.n_particles = c->d.n_particles;
  P.bound = c->d.bound;
  P.dx = 1.0f / c->d.n_grid;
  P.inv_dx = (float)c->d.n_grid;
  P.dt = c->d.dt;
  for (int k = 0; k < 3; k++) P.grav[k] = c->d.gravity[k];
  P.band = c->d.contact_band;
  P.friction = c->d.contact_friction;
  P.mats = (const MatDev*)(c->ws + c->L.mats);
  P.mat = c->user.mat;
  P.pscene = (const int*)(c->ws + c->L.pscene);
  P.cyl_radius = (const float*)(c->ws + c->L.cyl_radius);
  P.err = (int*)(c->ws + c->L.err);
  return P;
}

static PState user_pstate(const mpm_state* s, int N) {
  PState p;
  p.x = s->x; p.v = s->v; p.C = s->C; p.F = s->F; p.J = s->J; p.N = N;
  return p;
}

static float4* G(mpm_ctx* c, size_t off) { return (float4*)(c->ws + off); }

// Read and clear the device error word; the call's only host synchronisation.
static int finish(mpm_ctx* c) {
  int* err = (int*)(c->ws + c->L.err);
  int host = 0;
  if (hipMemcpyAsync(&host, err, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess) return MPM_EHIP;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return MPM_EHIP;
  if (hipGetLastError() != hipSuccess) return MPM_EHIP;
  c->timer.collect();
  if (host) {
    c->last_err_bits = host;
    if (hipMemsetAsync(err, 0, sizeof(int), c->stream) != hipSuccess) return MPM_EHIP;
    return MPM_EDOMAIN;
  }
  return MPM_OK;
}

extern "C" {

size_t mpm_workspace_bytes(const mpm_desc* d) {
  if (!desc_ok(d)) return 0;
  return plan(d).total;
}

int mpm_create(const mpm_desc* d, void* workspace_dev, size_t ws_bytes, void* stream, mpm_ctx** out) {
  if (!out) return MPM_EINVAL;
  *out = nullptr;
  if (!desc_ok(d) || !workspace_dev) return MPM_EINVAL;
  if (((uintptr_t)workspace_dev) % ALIGN) return MPM_EINVAL;
  Layout L = plan(d);
  if (ws_bytes < L.total) return MPM_EWORKSPACE;
  mpm_ctx* c = new (std::nothrow) mpm_ctx();
  if (!c) return MPM_EINVAL;
  c->d = *d;
  c->L = L;
  c->stream = (hipStream_t)stream;
  c->ws = (char*)workspace_dev;
  c->has_state = false;
  c->t = 0;
  c->last_err_bits = 0;
  c->state_bytes = align_up(STATE_FLOATS * (size_t)d->n_particles * sizeof(float));
  c->timer.name = "k_p2g_plain";
  c->plain_adjoint = false;
  int S = d->n_scenes;
  c->mats.resize(256);
  memset(c->mats.data(), 0, 256 * sizeof(MatDev));
  for (int m = 0; m < d->n_materials; m++) {
    const mpm_material& src = d->materials[m];
    if (src.kind < 0 || src.kind > MPM_RIGID || !(src.p_mass > 0.f) || !(src.p_vol > 0.f)) { delete c; return MPM_EINVAL; }
    MatDev& M = c->mats[m];
    M.kind = src.kind;
    M.mu = src.mu;
    M.lam = src.lambda;
    M.eta = src.viscosity;
    double sphi = sin(src.friction_deg * M_PI / 180.0);
    M.alpha = (float)(sqrt(2.0 / 3.0) * 2.0 * sphi / (3.0 - sphi));
    M.kappa = src.mu > 0.f ? (float)((3.0 * src.lambda + 2.0 * src.mu) / (2.0 * src.mu)) : 0.f;
    M.coh = src.cohesion;
    M.vol = src.p_vol;
    M.mass = src.p_mass;
    M.yrad = src.mu > 0.f ? src.yield_stress / (2.f * src.mu) : 0.f;
    if ((src.kind == MPM_SAND_DP || src.kind == MPM_PLASTIC_VM) && !(src.mu > 0.f)) { delete c; return MPM_EINVAL; }
    if (src.kind == MPM_PLASTIC_VM && !(src.yield_stress >= 0.f)) { delete c; return MPM_EINVAL; }
    M.box_lo = 1.f - src.theta_c;
    M.box_hi = 1.f + src.theta_s;
    if (src.kind == MPM_PLASTIC_BOX && !(src.theta_c >= 0.f && src.theta_c < 1.f && src.theta_s >= 0.f)) {
      delete c;
      return MPM_EINVAL;
    }
  }
  // rigid bodies: one per rigid material
  std::vector<int> body_of(256, -1);
  {
    int nb = 0;
    for (int m = 0; m < d->n_materials; m++)
      if (d->materials[m].kind == MPM_RIGID) body_of[m] = nb++;
  }
  c->rigid = RigidCtx{};
  c->rigid.n_bodies = L.n_bodies;
  if (L.n_bodies > 0) {
    char* w = (char*)workspace_dev;
    c->rigid.body_of = (const int*)(w + L.r_body_of);
    c->rigid.rest = (float*)(w + L.r_rest);
    c->rigid.bodies = (RigidBody*)(w + L.r_bodies);
    c->rigid.acc = (double*)(w + L.r_acc);
    c->rigid.rec = (double*)(w + L.r_rec);
    c->rigid.adj = (RigidAdjTerms*)(w + L.r_adj);
    c->rigid.rest_acc = (double*)(w + L.r_rest_acc);
    c->rigid.status = (int*)(w + L.r_status);
  }
  c->cyl_radius.assign(d->cyl_radius, d->cyl_radius + S);
  c->cyl_pos0.assign(d->cyl_pos0, d->cyl_pos0 + 3 * S);
  c->cyl_rot0.assign(d->cyl_rot0, d->cyl_rot0 + 9 * S);
  c->act_set.assign(d->horizon, 0);
  // static tables
  std::vector<int64_t> offs(S + 1);
  if (d->scene_offsets) for (int s = 0; s <= S; s++) offs[s] = d->scene_offsets[s];
  else { offs[0] = 0; offs[1] = d->n_particles; }
  int rc = MPM_OK;
  if (hipMemcpyAsync(c->ws + L.mats, c->mats.data(), 256 * sizeof(MatDev), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->ws + L.offs, offs.data(), (S + 1) * sizeof(int64_t), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->ws + L.cyl_radius, c->cyl_radius.data(), S * sizeof(float), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemsetAsync(c->ws + L.err, 0, 64, c->stream) != hipSuccess)
    rc = MPM_EHIP;
  if (rc == MPM_OK && L.n_bodies > 0) {
    if (hipMemcpyAsync(c->ws + L.r_body_of, body_of.data(), 256 * sizeof(int), hipMemcpyHostToDevice, c->stream) != hipSuccess)
      rc = MPM_EHIP;
    else
      launch_zero(c->ws + L.r_acc, (size_t)RIGID_SLOTS * L.n_bodies * RIGID_ACC * sizeof(double), c->stream);
  }
  if (rc == MPM_OK) {
    launch_scene_index((const int64_t*)(c->ws + L.offs), S, d->n_particles, (int*)(c->ws + L.pscene), c->stream);
    launch_zero(c->ws + L.vgrid, (size_t)d->n_grid * d->n_grid * d->n_grid * S * sizeof(float4), c->stream);
    rc = fast_init(c->fast, c->ws + L.fast, d->n_grid, S, d->n_particles, c->stream);
    fast_bind_grid(c->fast, G(c, L.mmv), G(c, L.vgrid));
    c->fast.closure_stats = (unsigned long long*)(c->ws + L.cstats);
    if (hipMemsetAsync(c->ws + L.cstats, 0, 64, c->stream) != hipSuccess) rc = MPM_EHIP;
  }
  if (rc == MPM_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = MPM_EHIP;
  if (rc != MPM_OK) { delete c; return rc; }
  *out = c;
  return MPM_OK;
}

int mpm_set_state(mpm_ctx* c, const mpm_state* st) {
  if (!c || !st || !st->x || !st->v || !st->C || !st->F || !st->J || !st->mat) return MPM_EINVAL;
  // captured graphs bake in every state pointer: rebinding any of them drops them
  if (c->has_state && (c->user.x != st->x || c->user.v != st->v || c->user.C != st->C || c->user.F != st->F ||
                       c->user.J != st->J || c->user.mat != st->mat))
    fast_invalidate(c->fast);
  c->user = *st;
  c->has_state = true;
  c->t = 0;
  int S = c->d.n_scenes;
  std::vector<double> pose0((size_t)S * POSE_DOUBLES);
  for (int s = 0; s < S; s++) {
    for (int k = 0; k < 3; k++) pose0[s * POSE_DOUBLES + k] = c->cyl_pos0[3 * s + k];
    for (int k = 0; k < 9; k++) pose0[s * POSE_DOUBLES + 3 + k] = c->cyl_rot0[9 * s + k];
  }
  if (hipMemcpyAsync(c->ws + c->L.pose, pose0.data(), pose0.size() * sizeof(double), hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return MPM_EHIP;
  int rstat = 0;
  if (c->rigid.n_bodies > 0) {
    // rest shapes of the rigid bodies from this state
    StepParams P = make_params(c);
    rigid_setup(c->rigid, P, user_pstate(st, c->d.n_particles), c->stream);
    if (hipMemcpyAsync(&rstat, c->rigid.status, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
      return MPM_EHIP;
  }
  // pose0 and rstat are host temporaries: wait for the copies
  if (hipStreamSynchronize(c->stream) != hipSuccess) return MPM_EHIP;
  if (rstat) {
    c->has_state = false;
    return MPM_EINVAL;
  }
  return MPM_OK;
}

int mpm_set_actions(mpm_ctx* c, int32_t t0, int32_t n, const float* actions_dev) {
  if (!c || !actions_dev || t0 < 0 || n < 1 || t0 + n > c->d.horizon) return MPM_EINVAL;
  size_t row = (size_t)c->d.n_scenes * 6 * sizeof(float);
  if (hipMemcpyAsync(c->ws + c->L.act + (size_t)t0 * row, actions_dev, (size_t)n * row, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return MPM_EHIP;
  for (int t = t0; t < t0 + n; t++) c->act_set[t] = 1;
  return MPM_OK;
}

static const double* pose_at(mpm_ctx* c, int t) {
  return (const double*)(c->ws + c->L.pose) + (size_t)t * c->d.n_scenes * POSE_DOUBLES;
}
static const float* act_at(mpm_ctx* c, int t) {
  return (const float*)(c->ws + c->L.act) + (size_t)t * c->d.n_scenes * 6;
}

// One plain step: state `in` -> `out` (may alias); with rigid bodies, the
// projection follows G2P and its record goes to slot rec_slot.
static void plain_step(mpm_ctx* c, const StepParams& P, const PState& in, const PState& out, int t, int rec_slot) {
  size_t nodes = (size_t)c->d.n_grid * c->d.n_grid * c->d.n_grid * c->d.n_scenes;
  launch_zero(G(c, c->L.mmv), nodes * sizeof(float4), c->stream);
  c->timer.begin(c->stream);
  launch_p2g_plain(in, P, G(c, c->L.mmv), c->stream);
  c->timer.end(c->stream);
  launch_grid_plain(P, G(c, c->L.mmv), G(c, c->L.vgrid), pose_at(c, t), act_at(c, t), c->stream);
  launch_g2p_plain(in, out, P, G(c, c->L.vgrid), c->stream);
  if (c->rigid.n_bodies > 0)
    rigid_forward(c->rigid, P, RigidRows{out, P.mat, nullptr}, rigid_rec(c, rec_slot), true, c->stream);
}

// n steps on the block-sorted path for scenes with rigid bodies.  The
// projection needs every particle of a body after G2P, so the steps run
// unfused: P2G, grid update, G2P into the second buffer, projection, sort
// back into the first buffer.  Checkpoints as in fast_run.
static void rigid_tiled_run(mpm_ctx* c, const StepParams& P, const PState& us, int t0, int n) {
  FastPath& f = c->fast;
  hipStream_t s = c->stream;
  const int N = c->d.n_particles;
  SortedState R0 = fast_own_state(f, 0);
  const PBuf tmp = f.buf[1];
  const RigidRows rows{packed_state(tmp.f, N), tmp.mat, tmp.id};
  // (the forward's sorts scan only the keys they counted)
  fast_sort_user(f, P, us, R0, s, true);
  for (int t = t0; t < t0 + n; t++) {
    const uint32_t sid = fast_next_sid(f);
    fast_p2g(f, P, R0, sid, s);
    fast_grid(f, P, R0, sid, t, pose_at(c, 0), act_at(c, 0), s);
    fast_g2p(f, P, R0, tmp, s);
    rigid_forward(c->rigid, P, rows, rigid_rec(c, 0), true, s);
    if (t + 1 == t0 + n) break;
    if (f.ck_k > 0 && (t + 1) % f.ck_k == 0)
      fast_export(f, P, tmp, packed_state((float*)(f.ck_base + (size_t)((t + 1) / f.ck_k) * f.ck_stride), N), s);
    // (the G2P buffer's key row is free: it serves as the sort's row map)
    fast_sort_next(f, P, R0, tmp, R0, tmp.key, s, true);
  }
  if (f.do_export) fast_export(f, P, tmp, us, s);
}

static int record_run(mpm_ctx* c, const StepParams& P, const PState& us, int t0, int n);

int mpm_step(mpm_ctx* c, int32_t n_steps) {
  if (!c || n_steps < 0) return MPM_EINVAL;
  if (!c->has_state) return MPM_ESTATE;
  if (n_steps == 0) return MPM_OK;
  if (c->t + n_steps > c->d.horizon) return MPM_EINVAL;
  for (int t = c->t; t < c->t + n_steps; t++)
    if (!c->act_set[t]) return MPM_ESTATE;
  StepParams P = make_params(c);
  const int N = c->d.n_particles;
  PState us = user_pstate(&c->user, N);
  c->fast.last_buf = -1;
  launch_pose(c->d.n_scenes, c->t, n_steps, c->d.dt, (const float*)(c->ws + c->L.act), (double*)(c->ws + c->L.pose), c->stream);
  c->timer.name = (c->d.requires_grad && c->plain_adjoint) ? "k_p2g_plain" : "k_g2p2g";
  if (c->d.requires_grad && c->plain_adjoint) {
    // plain path, recording checkpoints every k steps
    int k = c->d.ckpt_every;
    for (int t = c->t; t < c->t + n_steps; t++) {
      if (t % k == 0) {
        PState ck = packed_state((float*)(c->ws + c->L.ckpt + (size_t)(t / k) * c->state_bytes), N);
        launch_copy_state(us, ck, c->stream);
      }
      plain_step(c, P, us, us, t, 0);
    }
  } else if (c->d.requires_grad && c->d.ckpt_every == 0) {
    // (graph mode: captured once per start, steps, state pointers and launch shape)
    int rc;
    if (c->fast.use_graph && !c->timer.on) {
      mpm_ctx::CallGraph key;
      key.t0 = c->t;
      key.n = n_steps;
      key.part_wgs = c->fast.part_wgs;
      key.grid_wgs = c->fast.grid_wgs;
      const void* ptr[6] = {us.x, us.v, us.C, us.F, us.J, P.mat};
      for (int q = 0; q < 6; q++) key.ptr[q] = ptr[q];
      const int t0 = c->t;
      rc = graph_call(c, c->rgraphs, key, [&] { return record_run(c, P, us, t0, n_steps); });
    } else {
      rc = record_run(c, P, us, c->t, n_steps);
    }
    if (rc != MPM_OK) return rc;
  } else if (c->d.requires_grad) {
    // tiled path in one call; the checkpoints inside it are written by the
    // call itself, the one at its start is copied here
    const int k = c->d.ckpt_every;
    if (c->t % k == 0) {
      PState ck = packed_state((float*)(c->ws + c->L.ckpt + (size_t)(c->t / k) * c->state_bytes), N);
      launch_copy_state(us, ck, c->stream);
    }
    c->fast.ck_base = c->ws + c->L.ckpt;
    c->fast.ck_stride = c->state_bytes;
    c->fast.ck_k = k;
    c->fast.ck_t0 = c->t;
    int rc = MPM_OK;
    if (c->rigid.n_bodies > 0) rigid_tiled_run(c, P, us, c->t, n_steps);
    else rc = fast_run(c->fast, P, us, c->t, n_steps, pose_at(c, 0), act_at(c, 0), c->stream, &c->timer);
    c->fast.ck_k = 0;
    if (rc != MPM_OK) return MPM_EHIP;
  } else if (c->rigid.n_bodies > 0) {
    rigid_tiled_run(c, P, us, c->t, n_steps);
  } else {
    int rc = fast_run(c->fast, P, us, c->t, n_steps, pose_at(c, 0), act_at(c, 0), c->stream, &c->timer);
    if (rc != MPM_OK) return rc;
  }
  c->t += n_steps;
  if (hipGetLastError() != hipSuccess) return MPM_EHIP;
  return finish(c);
}

// The k block-sorted records of a segment, and the G2P output record.
static SortedState sorted_state(mpm_ctx* c, size_t base, bool tmp = false) {
  const SortedRec& r = tmp ? c->L.tmp_rec : c->L.rec;
  char* b = c->ws + base;
  SortedState S;
  S.vgrid = r.has_grid ? (float4*)(b + r.vgrid) : nullptr;
  S.mmv = r.has_grid ? (float4*)(b + r.mmv) : nullptr;
  S.cl_list = r.has_grid ? (uint32_t*)(b + r.cl_list) : nullptr;
  S.cl_count = r.has_grid ? (uint32_t*)(b + r.cl_count) : nullptr;
  S.b.f = (float*)(b + r.f);
  S.b.id = (uint32_t*)(b + r.id);
  S.b.key = (uint32_t*)(b + r.key);
  S.b.rank = (uint32_t*)(b + r.rank);
  S.b.mat = (uint8_t*)(b + r.mat);
  S.list = (int4*)(b + r.list);
  S.list_n = (uint32_t*)(b + r.list_n);
  return S;
}
static uint32_t* sorted_map(mpm_ctx* c, size_t base) { return (uint32_t*)(c->ws + base + c->L.rec.map); }

// Forward with ckpt_every = 0: the steps t0 .. t0 + n - 1 of one call run as
// the tiled adjoint's recompute does, each step's state kept as its record
// (block-sorted, with its grid, claims and the row map to the next record),
// so that the backward recomputes nothing.  The call imports the user state
// into record t0 (and maps record t0 - 1, left by the previous call, onto
// it), runs the P2G of step t0, one fused kernel per further step, and the
// G2P of the last step, whose output it exports to the user arrays.
static int record_run(mpm_ctx* c, const StepParams& P, const PState& us, int t0, int n) {
  FastPath& f = c->fast;
  hipStream_t s = c->stream;
  const int N = c->d.n_particles;
  const size_t rb = c->L.rec.bytes;
  auto rec = [&](int t) { return sorted_state(c, c->L.seg + (size_t)t * rb); };
  SortedState R0 = rec(t0);
  fast_sort_user(f, P, us, R0, s, true);
  if (t0 > 0) launch_row_map(rec(t0 - 1).b.id, R0.b.id, N, f.inv, sorted_map(c, c->L.seg + (size_t)(t0 - 1) * rb), s);
  uint32_t sid = fast_next_sid(f);
  fast_p2g(f, P, R0, sid, s);
  if (n > 1) {
    // the first fused step places its output by the import's offsets:
    // record t0 + 1 keeps record t0's order and list
    const SortedState R1 = rec(t0 + 1);
    launch_copy_list(R0.list, R0.list_n, R1.list, R1.list_n, s);
  }
  fast_grid_scan(f, P, R0, sid, t0, pose_at(c, 0), act_at(c, 0), n > 1 ? rec(t0 + 1).cl_count : nullptr, nullptr,
                 nullptr, s);
  for (int t = t0 + 1; t < t0 + n; t++) {
    const SortedState Sp = rec(t - 1), Si = rec(t);
    sid = fast_next_sid(f);
    fast_fused(f, P, Sp, Si, sorted_map(c, c->L.seg + (size_t)(t - 1) * rb), sid, s);
    const bool more = t + 1 < t0 + n;
    SortedState Sn = more ? rec(t + 1) : SortedState{};
    fast_grid_scan(f, P, Si, sid, t, pose_at(c, 0), act_at(c, 0), more ? Sn.cl_count : nullptr,
                   more ? Sn.list : f.list[0], more ? Sn.list_n : f.list_n, s);
  }
  // G2P of the last step (in the order the latest scan gives), exported
  const SortedState tmp = sorted_state(c, c->L.tmp, true);
  fast_g2p(f, P, rec(t0 + n - 1), tmp.b, s);
  fast_export(f, P, tmp.b, us, s);
  return hipGetLastError() == hipSuccess ? MPM_OK : MPM_EHIP;
}

// The tiled adjoint of step t on its block-sorted record Si: the adjoint of
// s_{t+1} (a_cur, read through `map`: Si's row -> s_{t+1}'s row) becomes
// that of s_t (a_nxt, Si's rows); the pose partials of step t go to acc.
// With rigid bodies, rrec is the step's projection record.  Swaps a_cur and
// a_nxt.
static void adjoint_step(mpm_ctx* c, const StepParams& P, const SortedState& Si, const uint32_t* map, int t,
                         double* rrec, PState& a_cur, PState& a_nxt, double* acc) {
  FastPath& f = c->fast;
  const int N = c->d.n_particles;
  hipStream_t s = c->stream;
  AdjArgs A;
  A.st = Si.b;
  A.list = Si.list;
  A.list_n = Si.list_n;
  A.N = N;
  A.abar_next = a_cur.x;
  A.map = map;
  A.abar = a_nxt.x;
  A.vgrid = Si.vgrid;
  A.tiles = f.tiles;
  A.tile_box = f.tile_box;
  A.gen = f.gen;
  A.sid = fast_next_sid(f);
  A.cl_list = Si.cl_list;
  A.cl_count = Si.cl_count;
  A.mmv = Si.mmv;
  A.mmvb = G(c, c->L.mmvb_blk);
  A.redo = (uint2*)(c->ws + c->L.redo);
  A.redo_n = (uint32_t*)(c->ws + c->L.redo_n) + 2 * t;
  // the adjoint of the rigid projection turns the body rows of the adjoint
  // of s_{t+1} into the adjoint of the G2P output
  if (rrec)
    rigid_adjoint(c->rigid, P, RigidRows{packed_state(Si.b.f, N), Si.b.mat, Si.b.id}, A.map, a_cur.x, rrec, Si.vgrid,
                  &f.g, s);
  launch_g2p_adj_tiled(A, P, f.g, f.part_wgs, s);
  launch_grid_adj_tiled(A, P, f.g, f.grid_wgs, pose_at(c, t), act_at(c, t), acc + (size_t)t * c->d.n_scenes * ACC_DOUBLES,
                        s);
  A.redo_n += 1;
  launch_p2g_adj_tiled(A, P, f.g, f.part_wgs, s);
  PState tsw = a_cur; a_cur = a_nxt; a_nxt = tsw;
}

// With ckpt_every = 0 the forward keeps a record of every step (see
// record_run), so the adjoint walks them all without recomputing anything.
static int backward_records(mpm_ctx* c, const StepParams& P, PState& a_cur, PState& a_nxt, double* acc) {
  const int N = c->d.n_particles, T = c->t;
  const size_t rb = c->L.rec.bytes;
  for (int t = T - 1; t >= 0; t--) {
    const size_t bi = c->L.seg + (size_t)t * rb;
    const SortedState Si = sorted_state(c, bi);
    adjoint_step(c, P, Si, (t == T - 1) ? Si.b.id : sorted_map(c, bi), t, nullptr, a_cur, a_nxt, acc);
  }
  launch_adj_reorder(a_cur.x, a_nxt.x, sorted_state(c, c->L.seg).b.id, N, c->fast.inv, c->stream);
  PState tsw = a_cur; a_cur = a_nxt; a_nxt = tsw;
  return hipGetLastError() == hipSuccess ? MPM_OK : MPM_EHIP;
}

// Tiled adjoint over all segments, last first.  On entry a_cur holds the
// adjoint of the final state in user order; on return it holds the adjoint
// of the initial state in user order (a_cur / a_nxt swapped as needed).
static int backward_tiled(mpm_ctx* c, const StepParams& P, PState& a_cur, PState& a_nxt, double* acc) {
  FastPath& f = c->fast;
  const int N = c->d.n_particles, T = c->t, k = c->d.ckpt_every;
  hipStream_t s = c->stream;
  const size_t rb = c->L.rec.bytes;
  SortedState tmp = sorted_state(c, c->L.tmp, true);
  const bool rigid = c->rigid.n_bodies > 0;
  const RigidRows trows{packed_state(tmp.b.f, N), tmp.b.mat, tmp.b.id};
  const int n_seg = (T + k - 1) / k;
  for (int seg = n_seg - 1; seg >= 0; seg--) {
    const int ts = seg * k, te = ts + k < T ? ts + k : T;
    // recompute: block-sorted records of s_ts .. s_{te-1}, each with its step's grid
    PState ck = packed_state((float*)(c->ws + c->L.ckpt + (size_t)seg * c->state_bytes), N);
    SortedState S0 = sorted_state(c, c->L.seg);
    fast_sort_user(f, P, ck, S0, s, true);   // (the padded import counters: the touched scan)
    // record of step t (record 1 keeps record 0's order: the first fused
    // step places its output by the import's offsets)
    auto rec = [&](int t) {
      SortedState R = sorted_state(c, c->L.seg + (size_t)(t - ts) * rb);
      if (!rigid && t - ts == 1) { R.list = S0.list; R.list_n = S0.list_n; }
      return R;
    };
    if (!rigid) {
      // P2G of s_ts, then one fused kernel per further step: each record is
      // sorted by the block keys of the previous step's positions (the
      // adjoint kernels' velocity and tile windows allow that drift) and the
      // fused kernel records the row map, so the recompute needs no sort
      uint32_t sid = fast_next_sid(f);
      fast_p2g(f, P, S0, sid, s);
      fast_grid_scan(f, P, S0, sid, ts, pose_at(c, 0), act_at(c, 0), te - ts > 1 ? rec(ts + 1).cl_count : nullptr,
                     nullptr, nullptr, s);
      for (int t = ts + 1; t < te; t++) {
        const SortedState Sp = rec(t - 1), Si = rec(t);
        sid = fast_next_sid(f);
        fast_fused(f, P, Sp, Si, sorted_map(c, c->L.seg + (size_t)(t - 1 - ts) * rb), sid, s);
        // the keys it counted describe record t + 1's order (or, after the
        // segment's last step, only need clearing)
        const bool more = t + 1 < te;
        SortedState Sn = more ? rec(t + 1) : SortedState{};
        fast_grid_scan(f, P, Si, sid, t, pose_at(c, 0), act_at(c, 0), more ? Sn.cl_count : nullptr,
                       more ? Sn.list : f.list[0], more ? Sn.list_n : f.list_n, s);
      }
    }
    for (int t = ts; t < te && rigid; t++) {
      const size_t bi = c->L.seg + (size_t)(t - ts) * rb;
      SortedState Si = sorted_state(c, bi);
      const uint32_t sid = fast_next_sid(f);
      fast_p2g(f, P, Si, sid, s);
      fast_grid(f, P, Si, sid, t, pose_at(c, 0), act_at(c, 0), s);
      // (with rigid bodies the last step's G2P also runs, for its projection record)
      if (t + 1 < te || rigid) {
        fast_g2p(f, P, Si, tmp.b, s);
        if (rigid) rigid_forward(c->rigid, P, trows, rigid_rec(c, t - ts), t + 1 < te, s);
      }
      if (t + 1 < te) {
        SortedState Sn = sorted_state(c, bi + rb);
        fast_sort_next(f, P, Si, tmp.b, Sn, sorted_map(c, bi), s);
      }
    }
    // adjoint, step te-1 down to ts; the adjoint of s_te is in user order,
    // read through s_{te-1}'s ids, the later ones through the recorded maps
    for (int t = te - 1; t >= ts; t--) {
      const size_t bi = c->L.seg + (size_t)(t - ts) * rb;
      const SortedState Si = rec(t);
      adjoint_step(c, P, Si, (t == te - 1) ? Si.b.id : sorted_map(c, bi), t, rigid ? rigid_rec(c, t - ts) : nullptr,
                   a_cur, a_nxt, acc);
    }
    // back to user order for the previous segment
    launch_adj_reorder(a_cur.x, a_nxt.x, S0.b.id, N, f.inv, s);   // (the import's map is free here)
    PState tsw = a_cur; a_cur = a_nxt; a_nxt = tsw;
  }
  return hipGetLastError() == hipSuccess ? MPM_OK : MPM_EHIP;
}

// The work of one backward call, enqueued on the context's stream.
static int enqueue_backward(mpm_ctx* c, const mpm_state* grad_T, float* grad_actions_dev, mpm_state* grad_0) {
  const int N = c->d.n_particles;
  const int T = c->t;
  const int k = c->d.ckpt_every;
  const int S = c->d.n_scenes;
  StepParams P = make_params(c);
  size_t nodes = (size_t)c->d.n_grid * c->d.n_grid * c->d.n_grid * S;
  hipStream_t s = c->stream;
  PState a_cur = packed_state((float*)(c->ws + c->L.adj0), N);
  PState a_nxt = packed_state((float*)(c->ws + c->L.adj1), N);
  // seed with dL/d(state_T); missing components are zero
  launch_zero(c->ws + c->L.adj0, c->state_bytes, s);
  size_t fN = (size_t)N * sizeof(float);
  if (hipMemcpyAsync(a_cur.x, grad_T->x, 3 * fN, hipMemcpyDeviceToDevice, s) != hipSuccess) return MPM_EHIP;
  if (hipMemcpyAsync(a_cur.v, grad_T->v, 3 * fN, hipMemcpyDeviceToDevice, s) != hipSuccess) return MPM_EHIP;
  if (grad_T->C && hipMemcpyAsync(a_cur.C, grad_T->C, 9 * fN, hipMemcpyDeviceToDevice, s) != hipSuccess) return MPM_EHIP;
  if (grad_T->F && hipMemcpyAsync(a_cur.F, grad_T->F, 9 * fN, hipMemcpyDeviceToDevice, s) != hipSuccess) return MPM_EHIP;
  if (grad_T->J && hipMemcpyAsync(a_cur.J, grad_T->J, fN, hipMemcpyDeviceToDevice, s) != hipSuccess) return MPM_EHIP;
  double* acc = (double*)(c->ws + c->L.acc);
  launch_zero(acc, align_up((size_t)T * S * ACC_DOUBLES * sizeof(double)), s);
  int n_seg = k > 0 ? (T + k - 1) / k : 0;
  if (!c->plain_adjoint) {
    launch_zero(c->ws + c->L.redo_n, align_up(2 * (size_t)T * sizeof(uint32_t)), s);
    int rc = k > 0 ? backward_tiled(c, P, a_cur, a_nxt, acc) : backward_records(c, P, a_cur, a_nxt, acc);
    if (rc != MPM_OK) return rc;
    n_seg = 0;
  }
  for (int seg = n_seg - 1; seg >= 0; seg--) {
    int ts = seg * k, te = ts + k < T ? ts + k : T;
    PState ck = packed_state((float*)(c->ws + c->L.ckpt + (size_t)seg * c->state_bytes), N);
    PState s0 = packed_state((float*)(c->ws + c->L.seg), N);
    launch_copy_state(ck, s0, s);
    // (with rigid bodies the last step runs too, into the spare slot te - ts,
    // for its projection record)
    const int t_end = c->rigid.n_bodies > 0 ? te : te - 1;
    for (int t = ts; t < t_end; t++) {
      PState a = packed_state((float*)(c->ws + c->L.seg + (size_t)(t - ts) * c->state_bytes), N);
      PState b = packed_state((float*)(c->ws + c->L.seg + (size_t)(t - ts + 1) * c->state_bytes), N);
      plain_step(c, P, a, b, t, t - ts);
    }
    for (int t = te - 1; t >= ts; t--) {
      PState st = packed_state((float*)(c->ws + c->L.seg + (size_t)(t - ts) * c->state_bytes), N);
      launch_zero(G(c, c->L.mmv), nodes * sizeof(float4), s);
      launch_p2g_plain(st, P, G(c, c->L.mmv), s);
      launch_grid_plain(P, G(c, c->L.mmv), G(c, c->L.vgrid), pose_at(c, t), act_at(c, t), s);
      if (c->rigid.n_bodies > 0)
        rigid_adjoint(c->rigid, P, RigidRows{st, P.mat, nullptr}, nullptr, a_cur.x, rigid_rec(c, t - ts),
                      G(c, c->L.vgrid), nullptr, s);
      launch_zero(G(c, c->L.vbar), nodes * sizeof(float4), s);
      launch_g2p_adj_plain(st, a_cur, a_nxt, P, G(c, c->L.vgrid), G(c, c->L.vbar), s);
      launch_grid_adj_plain(P, G(c, c->L.mmv), G(c, c->L.vbar), G(c, c->L.mmvb), pose_at(c, t), act_at(c, t),
                            acc + (size_t)t * S * ACC_DOUBLES, s);
      launch_p2g_adj_plain(st, a_nxt, P, G(c, c->L.mmvb), s);
      PState tmp = a_cur; a_cur = a_nxt; a_nxt = tmp;
    }
  }
  launch_pose_adj(S, T, c->d.dt, (const float*)(c->ws + c->L.act), (const double*)(c->ws + c->L.pose), acc,
                  grad_actions_dev, s);
  if (grad_0) {
    PState g0 = user_pstate(grad_0, N);
    launch_copy_state(a_cur, g0, s);
  }
  return hipGetLastError() == hipSuccess ? MPM_OK : MPM_EHIP;
}

int mpm_step_backward(mpm_ctx* c, const mpm_state* grad_T, float* grad_actions_dev, mpm_state* grad_0) {
  if (!c || !grad_T || !grad_T->x || !grad_T->v || !grad_actions_dev) return MPM_EINVAL;
  if (!c->has_state || !c->d.requires_grad || c->t < 1) return MPM_ESTATE;
  if (grad_0 && (!grad_0->x || !grad_0->v || !grad_0->C || !grad_0->F || !grad_0->J)) return MPM_EINVAL;
  c->fast.last_buf = -1;   // the recompute reuses the forward's buffers
  FastPath& f = c->fast;
  // graph mode: the tiled backward (without rigid bodies, whose steps run
  // eagerly) is captured once per horizon, gradient pointers and launch shape
  if (f.use_graph && !c->plain_adjoint && c->rigid.n_bodies == 0) {
    mpm_ctx::CallGraph key;
    key.n = c->t;
    key.part_wgs = f.part_wgs;
    key.grid_wgs = f.grid_wgs;
    const void* ptr[11] = {grad_T->x, grad_T->v, grad_T->C, grad_T->F, grad_T->J, grad_actions_dev,
                           grad_0 ? grad_0->x : nullptr, grad_0 ? grad_0->v : nullptr, grad_0 ? grad_0->C : nullptr,
                           grad_0 ? grad_0->F : nullptr, grad_0 ? grad_0->J : nullptr};
    for (int q = 0; q < 11; q++) key.ptr[q] = ptr[q];
    const int rc = graph_call(c, c->bgraphs, key, [&] { return enqueue_backward(c, grad_T, grad_actions_dev, grad_0); });
    if (rc != MPM_OK) return rc;
    return finish(c);
  }
  const int rc = enqueue_backward(c, grad_T, grad_actions_dev, grad_0);
  if (rc != MPM_OK) return rc;
  return finish(c);
}

int mpm_loss_blob(mpm_ctx* c, const float mu_g[3], float sigma_g, float* loss_dev, mpm_state* grad_out) {
  if (!c || !mu_g || !loss_dev) return MPM_EINVAL;
  if (!c->has_state) return MPM_ESTATE;
  StepParams P = make_params(c);
  PState us = user_pstate(&c->user, c->d.n_particles);
  double* scratch = (double*)(c->ws + c->L.scratch);
  launch_zero(scratch, align_up((2 + 2 * LOSS_SLOTS) * sizeof(double)), c->stream);
  launch_loss_blob(P, us, mu_g[0], mu_g[1], mu_g[2], sigma_g, scratch, loss_dev,
                   (grad_out && grad_out->x) ? grad_out->x : nullptr, c->stream);
  if (hipGetLastError() != hipSuccess) return MPM_EHIP;
  return finish(c);
}

int mpm_clock(const mpm_ctx* c, int32_t* t_out) {
  if (!c || !t_out) return MPM_EINVAL;
  *t_out = c->t;
  return MPM_OK;
}

int mpm_last_error_bits(const mpm_ctx* c, int32_t* bits_out) {
  if (!c || !bits_out) return MPM_EINVAL;
  *bits_out = c->last_err_bits;
  return MPM_OK;
}

int mpm_set_option(mpm_ctx* c, int32_t key, int32_t value) {
  if (!c) return MPM_EINVAL;
  switch (key) {
    case MPM_OPT_GRAPH: c->fast.use_graph = value != 0; return MPM_OK;
    case MPM_OPT_PART_THREADS:
      if (value != 128 && value != 256 && value != 512) return MPM_EINVAL;
      c->fast.part_threads = value;
      return MPM_OK;
    case MPM_OPT_PART_WGS:
      if (value < 64 || value > 65536) return MPM_EINVAL;
      c->fast.part_wgs = value;
      return MPM_OK;
    case MPM_OPT_GRID_WGS:
      if (value < 64 || value > 65536) return MPM_EINVAL;
      c->fast.grid_wgs = value;
      return MPM_OK;
    case MPM_OPT_ADJOINT:
      if (value != 0 && value != 1) return MPM_EINVAL;
      if (value == 1 && c->d.requires_grad && c->d.ckpt_every == 0) return MPM_EINVAL;   // (records are tiled)
      c->plain_adjoint = value == 1;
      return MPM_OK;
    case MPM_OPT_SHARE_CHUNKS:
      if (value < 0 || value > 64) return MPM_EINVAL;
      c->fast.share_chunks = value;
      return MPM_OK;
    default: return MPM_EINVAL;
  }
}

int mpm_get_option(const mpm_ctx* c, int32_t key, int32_t* value) {
  if (!c || !value) return MPM_EINVAL;
  switch (key) {
    case MPM_OPT_GRAPH: *value = c->fast.use_graph ? 1 : 0; return MPM_OK;
    case MPM_OPT_PART_THREADS: *value = c->fast.part_threads; return MPM_OK;
    case MPM_OPT_PART_WGS: *value = c->fast.part_wgs; return MPM_OK;
    case MPM_OPT_GRID_WGS: *value = c->fast.grid_wgs; return MPM_OK;
    case MPM_OPT_SHARE_CHUNKS: *value = c->fast.share_chunks; return MPM_OK;
    case MPM_OPT_ADJOINT: *value = c->plain_adjoint ? 1 : 0; return MPM_OK;
    case MPM_OPT_N_KEYS: *value = c->fast.g.n_keys; return MPM_OK;
    default: return MPM_EINVAL;
  }
}

int mpm_sort_snapshot(mpm_ctx* c, int32_t which, uint32_t* id_dev, uint32_t* key_dev, int32_t* list_dev,
                      int32_t* n_list_out) {
  if (!c || !id_dev || which < 0 || which > 2) return MPM_EINVAL;
  if (which != 1 && (!key_dev || !list_dev || !n_list_out)) return MPM_EINVAL;
  if (!c->has_state) return MPM_ESTATE;
  StepParams P = make_params(c);
  int nl = 0;
  const int rc = fast_sort_snapshot(c->fast, P, user_pstate(&c->user, c->d.n_particles), which, id_dev, key_dev,
                                    (int4*)list_dev, &nl, c->stream);
  if (rc == -1) return MPM_ESTATE;
  if (rc != 0) return MPM_EHIP;
  if (which != 1) *n_list_out = nl;
  return finish(c);
}

int mpm_autotune(mpm_ctx* c, int32_t n_steps, int32_t* best) {
  if (!c || !best || n_steps < 1) return MPM_EINVAL;
  if (!c->has_state) return MPM_ESTATE;
  if (c->t + n_steps > c->d.horizon) return MPM_EINVAL;
  for (int t = c->t; t < c->t + n_steps; t++)
    if (!c->act_set[t]) return MPM_ESTATE;
  StepParams P = make_params(c);
  PState us = user_pstate(&c->user, c->d.n_particles);
  hipStream_t s = c->stream;
  launch_pose(c->d.n_scenes, c->t, n_steps, c->d.dt, (const float*)(c->ws + c->L.act), (double*)(c->ws + c->L.pose), s);
  const int pts[3] = {128, 256, 512};
  const int pws[4] = {512, 1024, 2048, 4096};
  const int gws[3] = {512, 1024, 2048};
  const int shs[3] = {2, 1, 0};   // chunks above which a block is shared by two workgroups
  const int save_pt = c->fast.part_threads, save_pw = c->fast.part_wgs, save_gw = c->fast.grid_wgs;
  const int save_sh = c->fast.share_chunks;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MPM_EHIP;
  float best_ms = 1e30f;
  int bpt = save_pt, bpw = save_pw, bgw = save_gw, bsh = save_sh;
  c->fast.do_export = false;     // the trial runs leave the user state untouched
  int rc = MPM_OK;
  for (int a = 0; a < 3 && rc == MPM_OK; a++)
    for (int b = 0; b < 4 && rc == MPM_OK; b++)
      for (int d = 0; d < 3 && rc == MPM_OK; d++)
        for (int h = 0; h < 3 && rc == MPM_OK; h++) {
          c->fast.part_threads = pts[a];
          c->fast.part_wgs = pws[b];
          c->fast.grid_wgs = gws[d];
          c->fast.share_chunks = shs[h];
          float ms_min = 1e30f;
          for (int rep = 0; rep < 3; rep++) {
            hipEventRecord(e0, s);
            if (fast_run(c->fast, P, us, c->t, n_steps, pose_at(c, 0), act_at(c, 0), s, nullptr) != 0) {
              rc = MPM_EHIP;
              break;
            }
            hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) { rc = MPM_EHIP; break; }
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0 && ms < ms_min) ms_min = ms;   // first run warms up (and captures)
          }
          if (rc == MPM_OK && ms_min < best_ms) {
            best_ms = ms_min; bpt = pts[a]; bpw = pws[b]; bgw = gws[d]; bsh = shs[h];
          }
        }
  c->fast.do_export = true;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != MPM_OK) {
    c->fast.part_threads = save_pt; c->fast.part_wgs = save_pw; c->fast.grid_wgs = save_gw;
    c->fast.share_chunks = save_sh;
    return rc;
  }
  c->fast.part_threads = bpt;
  c->fast.part_wgs = bpw;
  c->fast.grid_wgs = bgw;
  c->fast.share_chunks = bsh;
  best[0] = bpt;
  best[1] = bpw;
  best[2] = bgw;
  best[3] = (int32_t)(best_ms * 1000.f / n_steps);
  best[4] = bsh;
  int frc = finish(c);
  return frc == MPM_OK ? MPM_OK : frc;
}

size_t mpm_mlp_blob_offset(void);

int mpm_log_samples(mpm_ctx* c, float* buf_dev, uint64_t capacity, uint64_t* count_dev) {
  if (!c) return MPM_EINVAL;
  if (buf_dev && (!count_dev || capacity == 0)) return MPM_EINVAL;
  if (buf_dev && (c->fast.mlp_blob || c->rigid.n_bodies > 0)) return MPM_ESTATE;
  // (a context that keeps every step's record runs its forward without the logging kernel)
  if (buf_dev && c->d.requires_grad && c->d.ckpt_every == 0) return MPM_ESTATE;
  c->fast.log_buf = buf_dev;
  c->fast.log_count = (unsigned long long*)count_dev;
  c->fast.log_cap = buf_dev ? capacity : 0;
  return MPM_OK;
}

int mpm_set_closure(mpm_ctx* c, const void* mlp_state_dev, float residual_tol) {
  if (!c || (mlp_state_dev && !(residual_tol >= 0.f))) return MPM_EINVAL;
  if (mlp_state_dev && (c->fast.log_buf || c->d.requires_grad || c->rigid.n_bodies > 0)) return MPM_ESTATE;
  c->fast.mlp_blob = mlp_state_dev ? (const void*)((const char*)mlp_state_dev + mpm_mlp_blob_offset()) : nullptr;
  c->fast.closure_tol = residual_tol;
  return MPM_OK;
}

int mpm_closure_stats(mpm_ctx* c, uint64_t* accepted, uint64_t* fallback) {
  if (!c || !accepted || !fallback) return MPM_EINVAL;
  unsigned long long h[2] = {0, 0};
  if (hipMemcpyAsync(h, c->fast.closure_stats, sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess) return MPM_EHIP;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return MPM_EHIP;
  *accepted = h[0];
  *fallback = h[1];
  if (hipMemsetAsync(c->fast.closure_stats, 0, sizeof(h), c->stream) != hipSuccess) return MPM_EHIP;
  return hip_ok(hipStreamSynchronize(c->stream));
}

int mpm_timing_enable(mpm_ctx* c, int32_t enable) {
  if (!c) return MPM_EINVAL;
  c->timer.on = enable != 0;
  c->timer.total_ms = 0.0;
  c->timer.launches = 0;
  c->timer.used = 0;
  return MPM_OK;
}

int mpm_timing_read(mpm_ctx* c, double* total_ms, int64_t* launches, char* name, int32_t name_len) {
  if (!c || !total_ms || !launches) return MPM_EINVAL;
  *total_ms = c->timer.total_ms;
  *launches = c->timer.launches;
  if (name && name_len > 0) {
    strncpy(name, c->timer.name, name_len - 1);
    name[name_len - 1] = 0;
  }
  c->timer.total_ms = 0.0;
  c->timer.launches = 0;
  return MPM_OK;
}

int mpm_destroy(mpm_ctx* c) {
  if (!c) return MPM_EINVAL;
  for (auto& g : c->bgraphs) destroy_call_graph(g);
  for (auto& g : c->rgraphs) destroy_call_graph(g);
  c->timer.destroy();
  fast_destroy(c->fast);
  delete c;
  return MPM_OK;
}

const char* mpm_strerror(int status) {
  switch (status) {
    case MPM_OK: return "ok";
    case MPM_EINVAL: return "invalid argument";
    case MPM_EWORKSPACE: return "workspace too small";
    case MPM_EHIP: return "HIP runtime error";
    case MPM_EDOMAIN: return "simulation left its valid domain (particle outside grid, non-finite value or sand sigma <= 0)";
    case MPM_ESTATE: return "call out of order (no state, missing actions or no recorded forward)";
    default: return "unknown status";
  }
}

}  // extern "C"
