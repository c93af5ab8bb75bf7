// The gas step (include/gas.h): incompressible advection-projection on a
// staggered grid (FluidLab section 3.2, after Stam 1999) and its adjoint.
//
// Forward step, three launches plus the pressure solve:
//   k_gas_advect   every grid point of u, v, w and the cells: the velocity
//                  at the point from its stencils, back-trace, trilinear
//                  sample, emitter blend (one launch for the four grids)
//   k_gas_div      per cell: divergence of the advected velocity with the
//                  buoyancy of the y-faces added on the fly and the walls
//                  closed; right-hand side of the pressure equation
//   pressure       A psi = div (A: 7-point Neumann Laplacian in cell units;
//                  psi = pressure * dt / h), by default exactly: DCT-II
//                  transforms along z, y and x on the matrix cores (k_axis),
//                  division by the eigenvalue sums, inverse transforms; or
//                  multigrid V-cycles (mg_solve: red-black half-sweeps on
//                  the finest level, tiled full sweeps on the coarser grid
//                  levels, the levels of at most 4096 cells in one workgroup)
//   k_gas_final    u = u* - grad psi on the interior faces, walls zero,
//                  scalars copied
// Adjoint step: the projection of the adjoint (k_gas_adj_div, the same
// pressure solve, k_gas_adj_sub; the projector is self-adjoint on
// wall-closed fields), then k_gas_adj_advect, which recomputes the
// back-traces, applies the buoyancy and emitter adjoints and scatters the
// advection adjoint at the back-traced points with float atomics (lanes
// merge the corners they share first), and k_gas_adj_ugather, which gathers
// the adjoint of the grid-point velocities over their stencils; the
// emitter's pose partials are reduced per wavefront into 128 FP64
// accumulator copies.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>
#include <new>
#include <vector>

#include "../../include/gas.h"
#include "mpm_internal.h"

namespace mpm {
namespace {

constexpr int MAXK = 4;
constexpr int SLOTS = 128;
constexpr int POSE_PARTIALS = 6;          // c (3), a = R e_y (3)
constexpr int BOTTOM_CELLS = 4096;        // levels this small run inside one workgroup, in LDS
constexpr int BOTTOM_LDS = 4800;          // >= 4096 * 8 / 7
#ifndef GAS_BOTTOM_THREADS
#define GAS_BOTTOM_THREADS 1024
#endif
constexpr int BOTTOM_THREADS = GAS_BOTTOM_THREADS;
constexpr int MAX_LEVELS = 12;
#ifndef GAS_COARSE_SWEEPS
#define GAS_COARSE_SWEEPS 4
#endif
constexpr int COARSE_SWEEPS = GAS_COARSE_SWEEPS;
#ifndef GAS_HALF_LEVELS
#define GAS_HALF_LEVELS 1
#endif
constexpr int HALF_LEVELS = GAS_HALF_LEVELS;   // finest levels smoothed by separate half-sweeps
#ifndef GAS_NU0_PRE
#define GAS_NU0_PRE 2
#endif
#ifndef GAS_NU0_POST
#define GAS_NU0_POST 1
#endif
#ifndef GAS_NU_POST
#define GAS_NU_POST 2
#endif
#ifndef GAS_NU_BOTTOM
#define GAS_NU_BOTTOM 2
#endif
// sweeps before / after the coarse correction on the finest level, after it
// on the coarser grid levels, and before and after it inside the bottom solve
constexpr int NU0_PRE = GAS_NU0_PRE, NU0_POST = GAS_NU0_POST, NU_POST = GAS_NU_POST, NU_BOTTOM = GAS_NU_BOTTOM;
// smoother tiles: TX x TY x TZ cells per workgroup; psi staged with a 2-cell
// halo, f with a 1-cell halo
#ifndef GAS_TILE_X
#define GAS_TILE_X 8
#endif
#ifndef GAS_TILE_Y
#define GAS_TILE_Y 8
#endif
#ifndef GAS_TILE_Z
#define GAS_TILE_Z 8
#endif
constexpr int TX = GAS_TILE_X, TY = GAS_TILE_Y, TZ = GAS_TILE_Z;
constexpr int PX = TX + 4, PY = TY + 4, PZ = TZ + 4;
constexpr int FX = TX + 2, FY = TY + 2, FZ = TZ + 2;

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
inline unsigned nblk(size_t n, unsigned b) {
  size_t g = (n + b - 1) / b;
  return (unsigned)(g < 65536 * 16 ? g : 65536 * 16);
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  The advection reads its neighbours' rows (stencils and samples), so
// its workgroup order is permuted to give every XCD one contiguous eighth of
// the points: workgroup b takes block start(b % 8) + b / 8 of the range (a
// bijection of [0, gridDim.x)).  At 128^3 this cuts the advection's fetched
// bytes by 40% (the kernel's time is set by its VALU issue, not by them).
__device__ inline unsigned xcd_block() {
  const unsigned nb = gridDim.x, b = blockIdx.x, x = b & 7u, per = nb >> 3, rem = nb & 7u;
  return x * per + min(x, rem) + (b >> 3);
}

struct Dims {
  int x, y, z;
  __host__ __device__ size_t cells() const { return (size_t)x * y * z; }
};

struct GP {
  int nx, ny, nz, K;
  float h, inv_h, dt, beta, t_amb;
  float s2inv;          // 1 / (2 sigma^2)
  float kappa, speed;
  float src[MAXK];
  size_t nu, nv, nw, nc;
  int* err;             // device error word (MPM_ERR_NONFINITE)
};

// grid q: 0 = u (x-faces), 1 = v, 2 = w, 3 = cells
__device__ inline void gdims(const GP& P, int q, int& d0, int& d1, int& d2) {
  d0 = P.nx + (q == 0);
  d1 = P.ny + (q == 1);
  d2 = P.nz + (q == 2);
}
__device__ inline float gorigin(int q, int a) { return (q == a) ? 0.f : 0.5f; }

// trilinear sample of grid q at a point: base node, fractions, clamped axes
struct Lerp {
  int i0, j0, k0;
  float f[3];
  bool cl[3];
};

__device__ inline Lerp lerp_setup(const GP& P, int q, const float* x) {
  int d[3];
  gdims(P, q, d[0], d[1], d[2]);
  Lerp L;
  int b[3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    float g = x[a] * P.inv_h - gorigin(q, a);
    const float hi = (float)(d[a] - 1);
    L.cl[a] = !(g >= 0.f && g <= hi);        // (also NaN)
    g = fminf(fmaxf(g, 0.f), hi);
    b[a] = min((int)floorf(g), d[a] - 2);
    L.f[a] = g - (float)b[a];
  }
  L.i0 = b[0]; L.j0 = b[1]; L.k0 = b[2];
  return L;
}

// flat index in one grid array (every array has fewer than 2^32 values:
// 32-bit arithmetic, widened for the address)
__device__ inline size_t gidx(int i, int j, int k, int d1, int d2) {
  return (size_t)(((uint32_t)i * (uint32_t)d1 + (uint32_t)j) * (uint32_t)d2 + (uint32_t)k);
}

__device__ inline void cell_of(const Dims& D, size_t g, int& i, int& j, int& k) {
  const uint32_t g32 = (uint32_t)g, r = g32 / (uint32_t)D.z;
  k = (int)(g32 - r * (uint32_t)D.z);
  i = (int)(r / (uint32_t)D.y);
  j = (int)(r - (uint32_t)i * (uint32_t)D.y);
}

// the 8 corner values
__device__ inline void lerp_load(const float* __restrict__ F, const Lerp& L, int d1, int d2, float* c) {
  const float* b = F + gidx(L.i0, L.j0, L.k0, d1, d2);
  const uint32_t sy = (uint32_t)d2, sx = (uint32_t)d1 * (uint32_t)d2;
#pragma unroll
  for (int n = 0; n < 8; n++) c[n] = b[((n >> 2) ? sx : 0u) + (((n >> 1) & 1) ? sy : 0u) + (uint32_t)(n & 1)];
}
__device__ inline float lerp_weight(const Lerp& L, int n) {
  return ((n >> 2) ? L.f[0] : 1.f - L.f[0]) * (((n >> 1) & 1) ? L.f[1] : 1.f - L.f[1]) * ((n & 1) ? L.f[2] : 1.f - L.f[2]);
}
__device__ inline float lerp_eval(const float* c, const Lerp& L) {
  float s = 0.f;
#pragma unroll
  for (int n = 0; n < 8; n++) s += lerp_weight(L, n) * c[n];
  return s;
}
// d(sample)/d(fraction) per axis
__device__ inline void lerp_grad(const float* c, const Lerp& L, float* g) {
  const float fx = L.f[0], fy = L.f[1], fz = L.f[2];
  g[0] = (1 - fy) * (1 - fz) * (c[4] - c[0]) + (1 - fy) * fz * (c[5] - c[1]) + fy * (1 - fz) * (c[6] - c[2]) +
         fy * fz * (c[7] - c[3]);
  g[1] = (1 - fx) * (1 - fz) * (c[2] - c[0]) + (1 - fx) * fz * (c[3] - c[1]) + fx * (1 - fz) * (c[6] - c[4]) +
         fx * fz * (c[7] - c[5]);
  g[2] = (1 - fx) * (1 - fy) * (c[1] - c[0]) + (1 - fx) * fy * (c[3] - c[2]) + fx * (1 - fy) * (c[5] - c[4]) +
         fx * fy * (c[7] - c[6]);
}

struct VelPtrs {
  const float* u;
  const float* v;
  const float* w;
};

__device__ inline float sample(const GP& P, int q, const float* F, const float* x) {
  int d0, d1, d2;
  gdims(P, q, d0, d1, d2);
  const Lerp L = lerp_setup(P, q, x);
  float c[8];
  lerp_load(F, L, d1, d2, c);
  return lerp_eval(c, L);
}

// The velocity at a grid point of grid q: the trilinear sample of each
// component grid there reduces to the point's own value on its own grid and
// to averages of 2 or 4 neighbours on the others (sample fractions 0 or 1/2,
// clamped at the walls like every sample).
__device__ inline void node_velocity(const GP& P, const VelPtrs& vel, int q, int i, int j, int k, float* U) {
  const int ny = P.ny, nz = P.nz;
  if (q == 3) {
    U[0] = 0.5f * (vel.u[gidx(i, j, k, ny, nz)] + vel.u[gidx(i + 1, j, k, ny, nz)]);
    U[1] = 0.5f * (vel.v[gidx(i, j, k, ny + 1, nz)] + vel.v[gidx(i, j + 1, k, ny + 1, nz)]);
    U[2] = 0.5f * (vel.w[gidx(i, j, k, ny, nz + 1)] + vel.w[gidx(i, j, k + 1, ny, nz + 1)]);
  } else if (q == 0) {
    const int ia = max(i - 1, 0), ib = min(i, P.nx - 1);
    U[0] = vel.u[gidx(i, j, k, ny, nz)];
    U[1] = 0.25f * ((vel.v[gidx(ia, j, k, ny + 1, nz)] + vel.v[gidx(ib, j, k, ny + 1, nz)]) +
                    (vel.v[gidx(ia, j + 1, k, ny + 1, nz)] + vel.v[gidx(ib, j + 1, k, ny + 1, nz)]));
    U[2] = 0.25f * ((vel.w[gidx(ia, j, k, ny, nz + 1)] + vel.w[gidx(ib, j, k, ny, nz + 1)]) +
                    (vel.w[gidx(ia, j, k + 1, ny, nz + 1)] + vel.w[gidx(ib, j, k + 1, ny, nz + 1)]));
  } else if (q == 1) {
    const int ja = max(j - 1, 0), jb = min(j, ny - 1);
    U[0] = 0.25f * ((vel.u[gidx(i, ja, k, ny, nz)] + vel.u[gidx(i, jb, k, ny, nz)]) +
                    (vel.u[gidx(i + 1, ja, k, ny, nz)] + vel.u[gidx(i + 1, jb, k, ny, nz)]));
    U[1] = vel.v[gidx(i, j, k, ny + 1, nz)];
    U[2] = 0.25f * ((vel.w[gidx(i, ja, k, ny, nz + 1)] + vel.w[gidx(i, jb, k, ny, nz + 1)]) +
                    (vel.w[gidx(i, ja, k + 1, ny, nz + 1)] + vel.w[gidx(i, jb, k + 1, ny, nz + 1)]));
  } else {
    const int ka = max(k - 1, 0), kb = min(k, nz - 1);
    U[0] = 0.25f * ((vel.u[gidx(i, j, ka, ny, nz)] + vel.u[gidx(i, j, kb, ny, nz)]) +
                    (vel.u[gidx(i + 1, j, ka, ny, nz)] + vel.u[gidx(i + 1, j, kb, ny, nz)]));
    U[1] = 0.25f * ((vel.v[gidx(i, j, ka, ny + 1, nz)] + vel.v[gidx(i, j, kb, ny + 1, nz)]) +
                    (vel.v[gidx(i, j + 1, ka, ny + 1, nz)] + vel.v[gidx(i, j + 1, kb, ny + 1, nz)]));
    U[2] = vel.w[gidx(i, j, k, ny, nz + 1)];
  }
}

// grid point of flat index g of grid q, and its position
__device__ inline void point_of(const GP& P, int q, size_t g, int& i, int& j, int& k, float* x) {
  int d0, d1, d2;
  gdims(P, q, d0, d1, d2);
  // (every grid has fewer than 2^32 points: 32-bit divisions)
  const uint32_t g32 = (uint32_t)g, r = g32 / (uint32_t)d2;
  k = (int)(g32 - r * (uint32_t)d2);
  i = (int)(r / (uint32_t)d1);
  j = (int)(r - (uint32_t)i * (uint32_t)d1);
  x[0] = ((float)i + gorigin(q, 0)) * P.h;
  x[1] = ((float)j + gorigin(q, 1)) * P.h;
  x[2] = ((float)k + gorigin(q, 2)) * P.h;
}

// which grid a flat index of the concatenated point sets belongs to
__device__ inline int split_points(const GP& P, size_t& g) {
  if (g < P.nu) return 0;
  g -= P.nu;
  if (g < P.nv) return 1;
  g -= P.nv;
  if (g < P.nw) return 2;
  g -= P.nw;
  return 3;
}

struct Pose {
  float c[3], a[3];   // centre and outflow axis R e_y
};
__device__ inline Pose load_pose(const double* p) {
  Pose o;
#pragma unroll
  for (int k = 0; k < 3; k++) { o.c[k] = (float)p[k]; o.a[k] = (float)p[3 + k * 3 + 1]; }
  return o;
}
__device__ inline float emitter_chi(const GP& P, const Pose& E, const float* x) {
  const float d0 = x[0] - E.c[0], d1 = x[1] - E.c[1], d2 = x[2] - E.c[2];
  return P.kappa * expf(-(d0 * d0 + d1 * d1 + d2 * d2) * P.s2inv);
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_gas_advect(GP P, VelPtrs vel, const float* __restrict__ s,
                                                    float* __restrict__ u1, float* __restrict__ v1,
                                                    float* __restrict__ w1, float* __restrict__ s1,
                                                    const double* __restrict__ pose) {
  const size_t total = P.nu + P.nv + P.nw + P.nc;
  const Pose E = load_pose(pose);
  for (size_t g0 = xcd_block() * (size_t)blockDim.x + threadIdx.x; g0 < total; g0 += (size_t)gridDim.x * blockDim.x) {
    size_t g = g0;
    const int q = split_points(P, g);
    int i, j, k;
    float x[3];
    point_of(P, q, g, i, j, k, x);
    float U[3];
    node_velocity(P, vel, q, i, j, k, U);
    const float xb[3] = {x[0] - P.dt * U[0], x[1] - P.dt * U[1], x[2] - P.dt * U[2]};
    const float chi = emitter_chi(P, E, x);
    if (q < 3) {
      const float* F = q == 0 ? vel.u : (q == 1 ? vel.v : vel.w);
      float val = sample(P, q, F, xb);
      val += chi * (P.speed * E.a[q] - val);
      float* O = q == 0 ? u1 : (q == 1 ? v1 : w1);
      O[g] = val;
    } else {
      const Lerp L = lerp_setup(P, 3, xb);
#pragma unroll
      for (int kk = 0; kk < MAXK; kk++) {
        if (kk >= P.K) break;
        float c[8];
        lerp_load(s + kk * P.nc, L, P.ny, P.nz, c);
        float val = lerp_eval(c, L);
        val += chi * (P.src[kk] - val);
        s1[kk * P.nc + g] = val;
      }
    }
  }
}

// y-face value after buoyancy (interior faces j in [1, ny - 1])
__device__ inline float buoyant_v(const GP& P, const float* v1, const float* T1, int i, int j, int k) {
  const float Tf = 0.5f * (T1[gidx(i, j - 1, k, P.ny, P.nz)] + T1[gidx(i, j, k, P.ny, P.nz)]);
  return v1[gidx(i, j, k, P.ny + 1, P.nz)] + P.dt * P.beta * (Tf - P.t_amb);
}

// divergence (sum of face differences, walls closed) of (u1, buoyant v1, w1)
__global__ __launch_bounds__(256) void k_gas_div(GP P, const float* __restrict__ u1, const float* __restrict__ v1,
                                                 const float* __restrict__ w1, const float* __restrict__ T1,
                                                 float* __restrict__ f, float* __restrict__ psi) {
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < P.nc; g += (size_t)gridDim.x * blockDim.x) {
    int i, j, k;
    cell_of(Dims{P.nx, P.ny, P.nz}, g, i, j, k);
    const float ur = (i + 1 < P.nx) ? u1[gidx(i + 1, j, k, P.ny, P.nz)] : 0.f;
    const float ul = (i > 0) ? u1[gidx(i, j, k, P.ny, P.nz)] : 0.f;
    const float vt = (j + 1 < P.ny) ? buoyant_v(P, v1, T1, i, j + 1, k) : 0.f;
    const float vb = (j > 0) ? buoyant_v(P, v1, T1, i, j, k) : 0.f;
    const float wf = (k + 1 < P.nz) ? w1[gidx(i, j, k + 1, P.ny, P.nz + 1)] : 0.f;
    const float wb = (k > 0) ? w1[gidx(i, j, k, P.ny, P.nz + 1)] : 0.f;
    f[g] = (ur - ul) + (vt - vb) + (wf - wb);
    psi[g] = 0.f;
  }
}

// u = u* - grad psi on the interior faces (v with its buoyancy), walls zero,
// scalars copied
__global__ __launch_bounds__(256) void k_gas_final(GP P, const float* __restrict__ u1, const float* __restrict__ v1,
                                                   const float* __restrict__ w1, const float* __restrict__ s1,
                                                   const float* __restrict__ psi, float* __restrict__ u,
                                                   float* __restrict__ v, float* __restrict__ w, float* __restrict__ s) {
  const size_t total = P.nu + P.nv + P.nw + (size_t)P.K * P.nc;
  for (size_t g0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g0 < total; g0 += (size_t)gridDim.x * blockDim.x) {
    size_t g = g0;
    const int q = split_points(P, g);
    if (q == 3) {
      s[g] = s1[g];
      if (!isfinite(s1[g])) atomicOr(P.err, ERR_NONFINITE);
      continue;
    }
    int i, j, k;
    float x[3];
    point_of(P, q, g, i, j, k, x);
    const int c = q == 0 ? i : (q == 1 ? j : k);
    const int n = q == 0 ? P.nx : (q == 1 ? P.ny : P.nz);
    float val = 0.f;
    if (c > 0 && c < n) {
      const size_t hi = gidx(i, j, k, P.ny, P.nz);
      const size_t lo = gidx(i - (q == 0), j - (q == 1), k - (q == 2), P.ny, P.nz);
      const float gp = psi[hi] - psi[lo];
      if (q == 0) val = u1[g] - gp;
      else if (q == 1) val = buoyant_v(P, v1, s1, i, j, k) - gp;
      else val = w1[g] - gp;
    }
    if (!isfinite(val)) atomicOr(P.err, ERR_NONFINITE);
    float* O = q == 0 ? u : (q == 1 ? v : w);
    O[g] = val;
  }
}

// ---------------------------------------------------------------------------
// multigrid for A psi = f, A the 7-point Neumann Laplacian in cell units
// (A psi)_c = sum over in-domain neighbours (psi_n - psi_c).  Red-black
// Gauss-Seidel smoothing, residual restriction f_c = (1/2) sum of the 8
// children's residuals (the coarse operator is A again at twice the
// spacing), cell-centred trilinear prolongation.
// ---------------------------------------------------------------------------

// sum of the in-domain neighbours and their number
__device__ inline float nb_sum(const float* psi, const Dims& D, int i, int j, int k, int& cnt) {
  float s = 0.f;
  cnt = 0;
  const size_t c = gidx(i, j, k, D.y, D.z);
  if (i > 0) { s += psi[c - (size_t)D.y * D.z]; cnt++; }
  if (i + 1 < D.x) { s += psi[c + (size_t)D.y * D.z]; cnt++; }
  if (j > 0) { s += psi[c - D.z]; cnt++; }
  if (j + 1 < D.y) { s += psi[c + D.z]; cnt++; }
  if (k > 0) { s += psi[c - 1]; cnt++; }
  if (k + 1 < D.z) { s += psi[c + 1]; cnt++; }
  return s;
}

// 1 / cnt for a neighbour count of 1..6 (a division would cost a long sequence)
__device__ inline float inv_count(int cnt) {
  return cnt == 6 ? (1.f / 6.f) : (cnt == 5 ? 0.2f : (cnt == 4 ? 0.25f : (cnt == 3 ? (1.f / 3.f) : (cnt == 2 ? 0.5f : 1.f))));
}

__device__ inline bool inside(const Dims& D, int i, int j, int k) {
  return i >= 0 && j >= 0 && k >= 0 && i < D.x && j < D.y && k < D.z;
}
__device__ inline float prolong_at(const float* psi_c, const Dims& Dc, int i, int j, int k);

// One full red-black Gauss-Seidel sweep (colour c1, then the other colour)
// per tile.  The tile's colour-c1 cells are updated on the tile and its
// 1-cell halo (the halo values are the ones the neighbouring tiles compute
// from the same old values), then the other colour on the tile itself, so
// the result equals two separate half-sweeps over the whole grid.  With
// psi_c, the prolonged coarse correction is added to every staged value
// first (the correction step fused into the sweep that follows it).
__global__ __launch_bounds__(256) void k_rb_sweep(float* __restrict__ psi, const float* __restrict__ f, Dims D, int c1,
                                                  const float* __restrict__ psi_c, Dims Dc) {
  constexpr int NP = PX * PY * PZ, NF = FX * FY * FZ;
  constexpr int RP = (NP + 255) / 256, RF = (NF + 255) / 256;
  __shared__ float sP[NP], sF[NF];
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY, k0 = blockIdx.z * TZ;
  // staging: every load of the thread is issued before the first is used
  // (a loop that stored each value to LDS as it arrived would wait out one
  // memory latency per iteration)
  float vp[RP], vf[RF];
#pragma unroll
  for (int r = 0; r < RP; r++) {
    const int q = tid + r * 256;
    const int a = q / (PY * PZ), b = (q / PZ) % PY, c = q % PZ;
    const int i = i0 - 2 + a, j = j0 - 2 + b, k = k0 - 2 + c;
    vp[r] = (q < NP && inside(D, i, j, k)) ? psi[gidx(i, j, k, D.y, D.z)] : 0.f;
  }
#pragma unroll
  for (int r = 0; r < RF; r++) {
    const int q = tid + r * 256;
    const int a = q / (FY * FZ), b = (q / FZ) % FY, c = q % FZ;
    const int i = i0 - 1 + a, j = j0 - 1 + b, k = k0 - 1 + c;
    vf[r] = (q < NF && inside(D, i, j, k)) ? f[gidx(i, j, k, D.y, D.z)] : 0.f;
  }
  if (psi_c) {
#pragma unroll
    for (int r = 0; r < RP; r++) {
      const int q = tid + r * 256;
      const int a = q / (PY * PZ), b = (q / PZ) % PY, c = q % PZ;
      const int i = i0 - 2 + a, j = j0 - 2 + b, k = k0 - 2 + c;
      if (q < NP && inside(D, i, j, k)) vp[r] += prolong_at(psi_c, Dc, i, j, k);
    }
  }
#pragma unroll
  for (int r = 0; r < RP; r++) {
    const int q = tid + r * 256;
    if (q < NP) sP[q] = vp[r];
  }
#pragma unroll
  for (int r = 0; r < RF; r++) {
    const int q = tid + r * 256;
    if (q < NF) sF[q] = vf[r];
  }
  __syncthreads();
  auto update = [&](int i, int j, int k, int pq, int fq) {
    float s = 0.f;
    int cnt = 0;
    if (i > 0) { s += sP[pq - PY * PZ]; cnt++; }
    if (i + 1 < D.x) { s += sP[pq + PY * PZ]; cnt++; }
    if (j > 0) { s += sP[pq - PZ]; cnt++; }
    if (j + 1 < D.y) { s += sP[pq + PZ]; cnt++; }
    if (k > 0) { s += sP[pq - 1]; cnt++; }
    if (k + 1 < D.z) { s += sP[pq + 1]; cnt++; }
    sP[pq] = (s - sF[fq]) * inv_count(cnt);
  };
  for (int q = tid; q < FX * FY * FZ; q += 256) {
    const int a = q / (FY * FZ), b = (q / FZ) % FY, c = q % FZ;
    const int i = i0 - 1 + a, j = j0 - 1 + b, k = k0 - 1 + c;
    if (inside(D, i, j, k) && ((i + j + k) & 1) == c1) update(i, j, k, ((a + 1) * PY + b + 1) * PZ + c + 1, q);
  }
  __syncthreads();
  for (int q = tid; q < TX * TY * TZ; q += 256) {
    const int a = q / (TY * TZ), b = (q / TZ) % TY, c = q % TZ;
    const int i = i0 + a, j = j0 + b, k = k0 + c;
    if (inside(D, i, j, k) && ((i + j + k) & 1) != c1)
      update(i, j, k, ((a + 2) * PY + b + 2) * PZ + c + 2, ((a + 1) * FY + b + 1) * FZ + c + 1);
  }
  __syncthreads();
  for (int q = tid; q < TX * TY * TZ; q += 256) {
    const int a = q / (TY * TZ), b = (q / TZ) % TY, c = q % TZ;
    const int i = i0 + a, j = j0 + b, k = k0 + c;
    if (inside(D, i, j, k)) psi[gidx(i, j, k, D.y, D.z)] = sP[((a + 2) * PY + b + 2) * PZ + c + 2];
  }
}

__device__ inline float residual_at(const float* psi, const float* f, const Dims& D, int i, int j, int k) {
  int cnt;
  const float s = nb_sum(psi, D, i, j, k, cnt);
  const size_t c = gidx(i, j, k, D.y, D.z);
  return f[c] - (s - (float)cnt * psi[c]);
}

// One red-black half-sweep (the cells of one colour), one thread per pair of
// z-neighbours (one cell of each colour), for the finest levels.
__global__ __launch_bounds__(256) void k_rb_half(float* __restrict__ psi, const float* __restrict__ f, Dims D,
                                                 int color) {
  const uint32_t nzp = (uint32_t)D.z >> 1;
  const uint32_t n = (uint32_t)D.x * (uint32_t)D.y * nzp;
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < n; g += gridDim.x * blockDim.x) {
    const uint32_t r = g / nzp, kp = g - r * nzp;
    const int i = (int)(r / (uint32_t)D.y), j = (int)(r - (uint32_t)i * (uint32_t)D.y);
    const int k = 2 * (int)kp + ((color + i + j) & 1);
    int cnt;
    const float sn = nb_sum(psi, D, i, j, k, cnt);
    const size_t c = gidx(i, j, k, D.y, D.z);
    psi[c] = (sn - f[c]) * inv_count(cnt);
  }
}

__global__ __launch_bounds__(256) void k_prolong(const float* __restrict__ psi_c, Dims Dc, float* __restrict__ psi,
                                                 Dims Df) {
  const size_t n = Df.cells();
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n; g += (size_t)gridDim.x * blockDim.x) {
    int i, j, k;
    cell_of(Df, g, i, j, k);
    psi[g] += prolong_at(psi_c, Dc, i, j, k);
  }
}

__global__ __launch_bounds__(256) void k_restrict(const float* __restrict__ psi, const float* __restrict__ f, Dims Df,
                                                  float* __restrict__ psi_c, float* __restrict__ f_c, Dims Dc) {
  const size_t n = Dc.cells();
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n; g += (size_t)gridDim.x * blockDim.x) {
    int I, J, K;
    cell_of(Dc, g, I, J, K);
    float r = 0.f;
#pragma unroll
    for (int c = 0; c < 8; c++) r += residual_at(psi, f, Df, 2 * I + (c >> 2), 2 * J + ((c >> 1) & 1), 2 * K + (c & 1));
    f_c[g] = 0.5f * r;
    psi_c[g] = 0.f;
  }
}

// trilinear interpolation from the coarse cell centres at fine cell (i, j, k)
__device__ inline float prolong_at(const float* psi_c, const Dims& Dc, int i, int j, int k) {
  const int I = i >> 1, J = j >> 1, K = k >> 1;
  const int I2 = min(max(I + ((i & 1) ? 1 : -1), 0), Dc.x - 1);
  const int J2 = min(max(J + ((j & 1) ? 1 : -1), 0), Dc.y - 1);
  const int K2 = min(max(K + ((k & 1) ? 1 : -1), 0), Dc.z - 1);
  const int ii[2] = {I, I2}, jj[2] = {J, J2}, kk[2] = {K, K2};
  const float wt[2] = {0.75f, 0.25f};
  float s = 0.f;
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
      for (int c = 0; c < 2; c++) s += wt[a] * wt[b] * wt[c] * psi_c[gidx(ii[a], jj[b], kk[c], Dc.y, Dc.z)];
  return s;
}


struct BottomArgs {
  int n_levels;              // levels handled here (the first is the entry level)
  Dims D[MAX_LEVELS];
  float* psi;                // entry level's psi (global): initial guess in, solution out
  const float* f;            // entry level's right-hand side (global)
};

// The V-cycle below the entry level, in one workgroup with every level in LDS.
__global__ __launch_bounds__(BOTTOM_THREADS) void k_bottom(BottomArgs B) {
  __shared__ float s_psi[BOTTOM_LDS], s_f[BOTTOM_LDS];
  __shared__ int s_ijk[BOTTOM_LDS];   // packed i | j << 10 | k << 20 of every cell of every level
  const int tid = threadIdx.x, NT = blockDim.x;
  int off[MAX_LEVELS];
  {
    int o = 0;
    for (int l = 0; l < B.n_levels; l++) { off[l] = o; o += (int)B.D[l].cells(); }
  }
  const int n0 = (int)B.D[0].cells();
  for (int c = tid; c < n0; c += NT) { s_psi[c] = B.psi[c]; s_f[c] = B.f[c]; }
  // the cell coordinates, decoded once (the phases below only read them)
  for (int l = 0; l < B.n_levels; l++)
    for (int c = tid; c < (int)B.D[l].cells(); c += NT) {
      int i, j, k;
      cell_of(B.D[l], c, i, j, k);
      s_ijk[off[l] + c] = i | (j << 10) | (k << 20);
    }
  __syncthreads();
  auto sweep = [&](int l, int color) {
    const Dims D = B.D[l];
    float* p = s_psi + off[l];
    const float* fl = s_f + off[l];
    const int* ijk = s_ijk + off[l];
    for (int c = tid; c < (int)D.cells(); c += NT) {
      const int e = ijk[c];
      const int i = e & 1023, j = (e >> 10) & 1023, k = e >> 20;
      if (((i + j + k) & 1) != color) continue;
      int cnt;
      const float s = nb_sum(p, D, i, j, k, cnt);
      p[c] = (s - fl[c]) / (float)cnt;
    }
    __syncthreads();
  };
  const int L = B.n_levels;
  for (int l = 0; l + 1 < L; l++) {
    for (int sw = 0; sw < NU_BOTTOM; sw++) { sweep(l, 0); sweep(l, 1); }
    const Dims Df = B.D[l], Dc = B.D[l + 1];
    for (int c = tid; c < (int)Dc.cells(); c += NT) {
      const int e = s_ijk[off[l + 1] + c];
      const int I = e & 1023, J = (e >> 10) & 1023, K = e >> 20;
      float r = 0.f;
      for (int q = 0; q < 8; q++)
        r += residual_at(s_psi + off[l], s_f + off[l], Df, 2 * I + (q >> 2), 2 * J + ((q >> 1) & 1), 2 * K + (q & 1));
      s_f[off[l + 1] + c] = 0.5f * r;
      s_psi[off[l + 1] + c] = 0.f;
    }
    __syncthreads();
  }
  for (int it = 0; it < COARSE_SWEEPS; it++) { sweep(L - 1, 0); sweep(L - 1, 1); }
  for (int l = L - 2; l >= 0; l--) {
    const Dims Df = B.D[l], Dc = B.D[l + 1];
    for (int c = tid; c < (int)Df.cells(); c += NT) {
      const int e = s_ijk[off[l] + c];
      const int i = e & 1023, j = (e >> 10) & 1023, k = e >> 20;
      s_psi[off[l] + c] += prolong_at(s_psi + off[l + 1], Dc, i, j, k);
    }
    __syncthreads();
    for (int sw = 0; sw < NU_BOTTOM; sw++) { sweep(l, 1); sweep(l, 0); }
  }
  for (int c = tid; c < n0; c += NT) B.psi[c] = s_psi[c];
}

// ---------------------------------------------------------------------------
// Spectral pressure solve.  With closed walls on a box of uniform cells the
// 7-point Neumann Laplacian is the Kronecker sum of 1-D Neumann Laplacians,
// each diagonalised by the DCT-II basis cos(pi k (i + 1/2) / n) with
// eigenvalues -4 sin^2(pi k / 2n).  So A psi = f is solved exactly by three
// axis transforms, a division by lambda_x + lambda_y + lambda_z (the
// constant mode, lambda = 0, set to zero: the gauge), and three inverse
// transforms.  Each axis transform is a dense contraction with an n x n
// matrix: out[k] = sum_i M[i][k] in[i] along the axis.
// ---------------------------------------------------------------------------
// The contraction runs on the matrix cores in FP32 (v_mfma_f32_16x16x4f32):
// a workgroup of four wavefronts takes XB = 64 lines and XK outputs along the
// axis, each wavefront 16 lines x XK outputs as XK / 16 tiles of 16 x 16;
// input chunks of XI values and the matching XI x XK block of the matrix are
// staged in LDS with every global load of a chunk issued before the first
// LDS write (float4 loads: every axis length and line count is a multiple
// of 4).
constexpr int XB = 64;
typedef float floatx4 __attribute__((ext_vector_type(4)));

struct AxisArgs {
  const float* in;
  float* out;
  const float* M;        // n x n, row = input index
  int n;                 // length of the transformed axis
  int A, B;              // layout [A][n][B]; inner transform (B == 1): A lines of n contiguous values
  // optional division by the 3-D eigenvalue (the last forward pass, along x):
  // out index k = kx, line index b = ky * nz + kz
  const float* lx;
  const float* ly;
  const float* lz;
  int nz;
};

template <bool INNER, int XK, int XI>
__global__ __launch_bounds__(256) void k_axis(AxisArgs X) {
  constexpr int XM = XK / 16;
  // two accumulator sets over alternate i-steps, added at the end: the same
  // speed as one, and a shorter rounding chain (pressure residual at 128^3
  // 1.2e-4 against 1.6e-4)
  constexpr int NACC = 2;
  static_assert(XI % (4 * NACC) == 0, "chunk split");
  constexpr int NS = XB * XI / 1024;      // float4 loads of the input chunk per thread
  constexpr int NMAT = XI * XK / 1024;    // float4 loads of the matrix block per thread
  static_assert(XK % 16 == 0 && XI % 16 == 0 && NS >= 1 && NMAT >= 1, "tile shape");
  static_assert(XK * XB <= XI * (XK + 1), "the output tile reuses the matrix chunk's LDS");
  __shared__ float sS[XI][XB + 1];       // input chunk, [i][line]
  __shared__ float sM[XI][XK + 1];       // matrix chunk, [i][k]; reused for the output tile [k][line]
  float* sO = &sM[0][0];                 // output tile: k * XB + line
  const int tid = threadIdx.x;
  // wavefront wv: lines 16 wv .. 16 wv + 15; lane (lr, lc)
  const int wv = tid >> 6, ln = tid & 63, lr = ln >> 4, lc = ln & 15;
  const int n = X.n;
  const int a = INNER ? 0 : (int)blockIdx.y;
  const int line0 = blockIdx.x * XB;        // first line (INNER: row; OUTER: b)
  const int nlines = INNER ? X.A : X.B;
  const int k0 = blockIdx.z * XK;
  floatx4 acc[NACC][XM];
#pragma unroll
  for (int u = 0; u < NACC; u++)
#pragma unroll
    for (int m = 0; m < XM; m++) acc[u][m] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int i0 = 0; i0 < n; i0 += XI) {
    float4 rs[NS], rm[NMAT];
#pragma unroll
    for (int r = 0; r < NS; r++) {
      const int q = tid + 256 * r;
      int line, ii;
      if (INNER) { line = line0 + q / (XI / 4); ii = i0 + 4 * (q % (XI / 4)); }
      else { ii = i0 + q / (XB / 4); line = line0 + 4 * (q % (XB / 4)); }
      rs[r] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (line < nlines && ii < n)
        rs[r] = INNER ? *(const float4*)(X.in + (size_t)line * n + ii)
                      : *(const float4*)(X.in + ((size_t)a * n + ii) * X.B + line);
    }
#pragma unroll
    for (int r = 0; r < NMAT; r++) {
      const int q = tid + 256 * r;
      const int ii = i0 + q / (XK / 4), kk = k0 + 4 * (q % (XK / 4));
      rm[r] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (ii < n && kk < n) rm[r] = *(const float4*)(X.M + (size_t)ii * n + kk);
    }
    __syncthreads();    // the previous chunk's reads are done
#pragma unroll
    for (int r = 0; r < NS; r++) {
      const int q = tid + 256 * r;
      if (INNER) {
        const int b = q / (XI / 4), i = 4 * (q % (XI / 4));
        sS[i][b] = rs[r].x; sS[i + 1][b] = rs[r].y; sS[i + 2][b] = rs[r].z; sS[i + 3][b] = rs[r].w;
      } else {
        const int i = q / (XB / 4), b = 4 * (q % (XB / 4));
        sS[i][b] = rs[r].x; sS[i][b + 1] = rs[r].y; sS[i][b + 2] = rs[r].z; sS[i][b + 3] = rs[r].w;
      }
    }
#pragma unroll
    for (int r = 0; r < NMAT; r++) {
      const int q = tid + 256 * r;
      const int i = q / (XK / 4), k = 4 * (q % (XK / 4));
      sM[i][k] = rm[r].x; sM[i][k + 1] = rm[r].y; sM[i][k + 2] = rm[r].z; sM[i][k + 3] = rm[r].w;
    }
    __syncthreads();
    // D(16 lines x 16 outputs) += A(16 x 4) B(4 x 16): lane (lr, lc) holds
    // A[lc][lr] = in[line 16 wv + lc][i + lr] and B[lr][lc] = M[i + lr][16 m + lc]
#pragma unroll 2
    for (int i = 0; i < XI; i += 4 * NACC) {
#pragma unroll
      for (int u = 0; u < NACC; u++) {
        const float av = sS[i + 4 * u + lr][16 * wv + lc];
#pragma unroll
        for (int m = 0; m < XM; m++)
          acc[u][m] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, sM[i + 4 * u + lr][16 * m + lc], acc[u][m], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int u = 1; u < NACC; u++)
#pragma unroll
    for (int m = 0; m < XM; m++) acc[0][m] += acc[u][m];
  __syncthreads();
  // output tile through LDS ([k][line] in sM), then coalesced stores; lane
  // (lr, lc) holds D[4 lr + r][lc], r < 4
#pragma unroll
  for (int m = 0; m < XM; m++)
#pragma unroll
    for (int r = 0; r < 4; r++) sO[(16 * m + lc) * XB + 16 * wv + 4 * lr + r] = acc[0][m][r];
  __syncthreads();
  if (INNER) {
    for (int q = tid; q < XB * XK; q += 256) {
      const int b = q / XK, k = q % XK;
      const int line = line0 + b, kk = k0 + k;
      if (line < nlines && kk < n) X.out[(size_t)line * n + kk] = sO[k * XB + b];
    }
  } else {
    for (int q = tid; q < XB * XK; q += 256) {
      const int k = q / XB, b = q % XB;
      const int line = line0 + b, kk = k0 + k;
      if (line < nlines && kk < n) {
        float v = sO[k * XB + b];
        if (X.lx) {
          const int ky = line / X.nz, kz = line - ky * X.nz;
          const float lam = X.lx[kk] + X.ly[ky] + X.lz[kz];
          v = lam != 0.f ? v / lam : 0.f;
        }
        X.out[((size_t)a * n + kk) * X.B + line] = v;
      }
    }
  }
}

// |f - A psi|^2 and |f|^2 per block into part[2 * block]; the last step sums
__global__ __launch_bounds__(256) void k_resnorm(const float* __restrict__ psi, const float* __restrict__ f, Dims D,
                                                 double* __restrict__ part) {
  __shared__ double s_r[256], s_b[256];
  double r2 = 0.0, b2 = 0.0;
  const size_t n = D.cells();
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < n; g += (size_t)gridDim.x * blockDim.x) {
    int i, j, k;
    cell_of(D, g, i, j, k);
    const double r = residual_at(psi, f, D, i, j, k);
    r2 += r * r;
    b2 += (double)f[g] * f[g];
  }
  s_r[threadIdx.x] = r2;
  s_b[threadIdx.x] = b2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) { s_r[threadIdx.x] += s_r[threadIdx.x + o]; s_b[threadIdx.x] += s_b[threadIdx.x + o]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { part[2 * blockIdx.x] = s_r[0]; part[2 * blockIdx.x + 1] = s_b[0]; }
}
__global__ void k_resnorm_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double r = 0.0, b = 0.0;
  for (int q = 0; q < nb; q++) { r += part[2 * q]; b += part[2 * q + 1]; }
  out[0] = b > 0.0 ? sqrt(r / b) : 0.0;
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
// divergence of the wall-closed adjoint velocity (right-hand side of the
// adjoint projection)
__global__ __launch_bounds__(256) void k_gas_adj_div(GP P, const float* __restrict__ ub, const float* __restrict__ vb,
                                                     const float* __restrict__ wb, float* __restrict__ f,
                                                     float* __restrict__ psi) {
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < P.nc; g += (size_t)gridDim.x * blockDim.x) {
    int i, j, k;
    cell_of(Dims{P.nx, P.ny, P.nz}, g, i, j, k);
    const float ur = (i + 1 < P.nx) ? ub[gidx(i + 1, j, k, P.ny, P.nz)] : 0.f;
    const float ul = (i > 0) ? ub[gidx(i, j, k, P.ny, P.nz)] : 0.f;
    const float vt = (j + 1 < P.ny) ? vb[gidx(i, j + 1, k, P.ny + 1, P.nz)] : 0.f;
    const float vl = (j > 0) ? vb[gidx(i, j, k, P.ny + 1, P.nz)] : 0.f;
    const float wf = (k + 1 < P.nz) ? wb[gidx(i, j, k + 1, P.ny, P.nz + 1)] : 0.f;
    const float wl = (k > 0) ? wb[gidx(i, j, k, P.ny, P.nz + 1)] : 0.f;
    f[g] = (ur - ul) + (vt - vl) + (wf - wl);
    psi[g] = 0.f;
  }
}

// projected adjoint velocity: interior faces minus grad psi, walls zero
__global__ __launch_bounds__(256) void k_gas_adj_sub(GP P, const float* __restrict__ ub, const float* __restrict__ vb,
                                                     const float* __restrict__ wb, const float* __restrict__ psi,
                                                     float* __restrict__ ub1, float* __restrict__ vb1,
                                                     float* __restrict__ wb1) {
  const size_t total = P.nu + P.nv + P.nw;
  for (size_t g0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g0 < total; g0 += (size_t)gridDim.x * blockDim.x) {
    size_t g = g0;
    const int q = split_points(P, g);
    int i, j, k;
    float x[3];
    point_of(P, q, g, i, j, k, x);
    const int c = q == 0 ? i : (q == 1 ? j : k);
    const int n = q == 0 ? P.nx : (q == 1 ? P.ny : P.nz);
    const float* In = q == 0 ? ub : (q == 1 ? vb : wb);
    float* O = q == 0 ? ub1 : (q == 1 ? vb1 : wb1);
    float val = 0.f;
    if (c > 0 && c < n) {
      const size_t hi = gidx(i, j, k, P.ny, P.nz);
      const size_t lo = gidx(i - (q == 0), j - (q == 1), k - (q == 2), P.ny, P.nz);
      val = In[g] - (psi[hi] - psi[lo]);
    }
    if (!isfinite(val)) atomicOr(P.err, ERR_NONFINITE);
    O[g] = val;
  }
}

struct AdjOut {
  float* u;
  float* v;
  float* w;
  float* s;
};

// Scatter of val times the trilinear weights of L into F, called by every
// lane of a wavefront together (on = false: no contribution).  Consecutive
// lanes hold consecutive points along z, whose back-traced samples usually
// share four of their eight corners: when the previous lane samples the same
// array at the same (i0, j0) with k0 one less, its k0 + 1 corners are this
// lane's k0 corners, so this lane adds them in and issues one atomic for
// both (about 4 atomics per sample instead of 8).
__device__ inline void scatter_lerp_wave(float* F, const Lerp& L, int d1, int d2, float val, bool on) {
  float lo[4], hi[4];
#pragma unroll
  for (int c = 0; c < 4; c++) {
    lo[c] = on ? lerp_weight(L, 2 * c) * val : 0.f;
    hi[c] = on ? lerp_weight(L, 2 * c + 1) * val : 0.f;
  }
  const int lane = (int)__lane_id();
  const unsigned long long fp = (unsigned long long)F;
  const unsigned long long fprev = __shfl_up(fp, 1);
  const int i0p = __shfl_up(L.i0, 1), j0p = __shfl_up(L.j0, 1), k0p = __shfl_up(L.k0, 1);
  const int onp = __shfl_up(on ? 1 : 0, 1);
  const bool take = on && lane > 0 && onp && fprev == fp && i0p == L.i0 && j0p == L.j0 && k0p + 1 == L.k0;
#pragma unroll
  for (int c = 0; c < 4; c++) {
    const float h = __shfl_up(hi[c], 1);
    if (take) lo[c] += h;
  }
  const int took = __shfl_down(take ? 1 : 0, 1);
  const bool given = lane < 63 && took;     // the next lane issues this lane's k0 + 1 corners
  if (!on) return;
  float* base = F + gidx(L.i0, L.j0, L.k0, d1, d2);
  const uint32_t sy = (uint32_t)d2, sx = (uint32_t)d1 * (uint32_t)d2;
#pragma unroll
  for (int c = 0; c < 4; c++) {
    const uint32_t off = ((c >> 1) ? sx : 0u) + ((c & 1) ? sy : 0u);
    if (lo[c] != 0.f) atomicAdd(base + off, lo[c]);
    if (!given && hi[c] != 0.f) atomicAdd(base + off + 1, hi[c]);
  }
}

// Adjoint of advection + emitter + buoyancy for every grid point of state s_t.
// ub1/vb1/wb1: adjoint of the blended velocities (already projected, walls
// zero); sb: adjoint of the output scalars; out: adjoint of s_t (cleared
// before; accumulated with atomics); slots: pose partials.  The loop runs
// wavefront-uniformly (the scatter exchanges corners between lanes).
__global__ __launch_bounds__(256) void k_gas_adj_advect(GP P, VelPtrs vel, const float* __restrict__ s,
                                                        const float* __restrict__ ub1, const float* __restrict__ vb1,
                                                        const float* __restrict__ wb1, const float* __restrict__ sb,
                                                        AdjOut out, const double* __restrict__ pose,
                                                        double* __restrict__ slots, float* __restrict__ ub) {
  const size_t total = P.nu + P.nv + P.nw + P.nc;
  const Pose E = load_pose(pose);
  double part[POSE_PARTIALS] = {0, 0, 0, 0, 0, 0};
  for (size_t base = blockIdx.x * (size_t)blockDim.x; base < total; base += (size_t)gridDim.x * blockDim.x) {
    const size_t g0 = base + threadIdx.x;
    const bool live = g0 < total;
    int q = 3;
    Lerp L = {};
    int d1 = P.ny, d2 = P.nz;
    float* tgt = out.s;
    bool on = false;                   // this lane scatters (face lanes: once; cell lanes: per scalar)
    bool s_on[MAXK] = {false, false, false, false};
    float sval[MAXK] = {0.f, 0.f, 0.f, 0.f};
    float xbb[3] = {0.f, 0.f, 0.f};   // adjoint of the back-traced point
    if (live) {
      size_t g = g0;
      q = split_points(P, g);
      int i, j, k;
      float x[3];
      point_of(P, q, g, i, j, k, x);
      float U[3];
      node_velocity(P, vel, q, i, j, k, U);
      const float xb[3] = {x[0] - P.dt * U[0], x[1] - P.dt * U[1], x[2] - P.dt * U[2]};
      const float chi = emitter_chi(P, E, x);
      const float dchi[3] = {chi * (x[0] - E.c[0]) * 2.f * P.s2inv, chi * (x[1] - E.c[1]) * 2.f * P.s2inv,
                             chi * (x[2] - E.c[2]) * 2.f * P.s2inv};
      if (q < 3) {
        int d0;
        gdims(P, q, d0, d1, d2);
        const float* F = q == 0 ? vel.u : (q == 1 ? vel.v : vel.w);
        const float* Ab = q == 0 ? ub1 : (q == 1 ? vb1 : wb1);
        const float ab = Ab[g];
        if (ab != 0.f) {
          L = lerp_setup(P, q, xb);
          float c[8];
          lerp_load(F, L, d1, d2, c);
          const float val = lerp_eval(c, L);
          const float target = P.speed * E.a[q];
          // emitter: out = val + chi (target - val)
#pragma unroll
          for (int a = 0; a < 3; a++) part[a] += (double)(ab * (target - val) * dchi[a]);
          part[3 + q] += (double)(ab * chi * P.speed);
          const float vbar = (1.f - chi) * ab;
          tgt = q == 0 ? out.u : (q == 1 ? out.v : out.w);
          on = true;
          sval[0] = vbar;
          float gr[3];
          lerp_grad(c, L, gr);
#pragma unroll
          for (int a = 0; a < 3; a++) xbb[a] = L.cl[a] ? 0.f : vbar * gr[a] * P.inv_h;
        }
      } else {
        L = lerp_setup(P, 3, xb);
#pragma unroll
        for (int kk = 0; kk < MAXK; kk++) {
          if (kk >= P.K) break;
          float ab = sb[kk * P.nc + g];
          if (kk == 0) {
            // buoyancy: each interior y-face of this cell took dt beta T / 2
            float vs = 0.f;
            if (j > 0) vs += vb1[gidx(i, j, k, P.ny + 1, P.nz)];
            if (j + 1 < P.ny) vs += vb1[gidx(i, j + 1, k, P.ny + 1, P.nz)];
            ab += 0.5f * P.dt * P.beta * vs;
          }
          if (ab == 0.f) continue;
          float c[8];
          lerp_load(s + kk * P.nc, L, P.ny, P.nz, c);
          const float val = lerp_eval(c, L);
#pragma unroll
          for (int a = 0; a < 3; a++) part[a] += (double)(ab * (P.src[kk] - val) * dchi[a]);
          const float sbar = (1.f - chi) * ab;
          s_on[kk] = true;
          sval[kk] = sbar;
          float gr[3];
          lerp_grad(c, L, gr);
#pragma unroll
          for (int a = 0; a < 3; a++) xbb[a] += L.cl[a] ? 0.f : sbar * gr[a] * P.inv_h;
        }
      }
    }
    // the scatters, every lane of the wavefront together
#pragma unroll
    for (int kk = 0; kk < MAXK; kk++) {
      if (kk >= P.K) break;
      // (one call for all lanes: the lanes of a wavefront may straddle two grids)
      const bool face = q < 3;
      float* F = face ? tgt : out.s + kk * P.nc;
      const float val = face ? (kk == 0 ? sval[0] : 0.f) : sval[kk];
      const bool lane_on = face ? (on && kk == 0) : s_on[kk];
      scatter_lerp_wave(F, L, d1, d2, val, lane_on);
    }
    // back-trace xb = x - dt U(x): U's adjoint -dt xbb is kept per point;
    // k_gas_adj_ugather spreads it over the velocity grids
    if (live) {
#pragma unroll
      for (int a = 0; a < 3; a++) ub[(size_t)a * total + g0] = -P.dt * xbb[a];
    }
  }
  // pose partials: wave sums, one FP64 atomic per component into the
  // wavefront's accumulator copy
  const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  double* dst = slots + (size_t)(wave % SLOTS) * POSE_PARTIALS;
#pragma unroll
  for (int qn = 0; qn < POSE_PARTIALS; qn++) {
    double v = part[qn];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (__lane_id() == 0 && v != 0.0) atomicAdd(dst + qn, v);
  }
}

// Adjoint of the velocity at every grid point (U of the back-traces, from
// the stencils of node_velocity) as a gather: each velocity node of grid a
// sums the U_a adjoints (ub, from k_gas_adj_advect) of the points whose
// stencil holds it, with the stencil's weights: its own point (1), the two
// cells beside it along a (1/2 each), and on each other face grid b the
// points beside it along a (1/2) whose clamped pair along b holds it (1/2
// per hit).
__global__ __launch_bounds__(256) void k_gas_adj_ugather(GP P, const float* __restrict__ ub, AdjOut out) {
  const size_t total = P.nu + P.nv + P.nw + P.nc;
  const size_t nvel = P.nu + P.nv + P.nw;
  const size_t qoff[4] = {0, P.nu, P.nu + P.nv, nvel};
  const int N[3] = {P.nx, P.ny, P.nz};
  for (size_t g0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g0 < nvel; g0 += (size_t)gridDim.x * blockDim.x) {
    size_t g = g0;
    const int a = split_points(P, g);
    int n[3];
    float xn[3];
    point_of(P, a, g, n[0], n[1], n[2], xn);
    const float* U = ub + (size_t)a * total;
    float acc = U[qoff[a] + g];
    float cs = 0.f;
#pragma unroll
    for (int t = 0; t < 2; t++) {
      int c[3] = {n[0], n[1], n[2]};
      c[a] = n[a] - 1 + t;
      if (c[a] >= 0 && c[a] < N[a]) cs += U[qoff[3] + gidx(c[0], c[1], c[2], P.ny, P.nz)];
    }
    acc += 0.5f * cs;
#pragma unroll
    for (int b = 0; b < 3; b++) {
      if (b == a) continue;
      int db0, db1, db2;
      gdims(P, b, db0, db1, db2);
      float fs = 0.f;
#pragma unroll
      for (int ta = 0; ta < 2; ta++) {
#pragma unroll
        for (int tb = 0; tb < 2; tb++) {
          int p[3] = {n[0], n[1], n[2]};
          p[a] = n[a] - 1 + ta;
          p[b] = n[b] + tb;
          if (p[a] < 0 || p[a] >= N[a] || p[b] > N[b]) continue;
          const int hits = (max(p[b] - 1, 0) == n[b]) + (min(p[b], N[b] - 1) == n[b]);
          if (hits) fs += (float)hits * U[qoff[b] + gidx(p[0], p[1], p[2], db1, db2)];
        }
      }
      acc += 0.25f * fs;
    }
    float* O = a == 0 ? out.u : (a == 1 ? out.v : out.w);
    O[g] += acc;
  }
}

// sum of the accumulator copies into the step's pose partials (c at 6..8 and
// the axis a = R e_y at 9..11 of the ACC_DOUBLES layout); copies cleared
__global__ __launch_bounds__(64) void k_gas_pose_acc(double* __restrict__ slots, double* __restrict__ acc_t) {
  const int lane = threadIdx.x;
  double tot[POSE_PARTIALS];
#pragma unroll
  for (int qn = 0; qn < POSE_PARTIALS; qn++) tot[qn] = 0.0;
  for (int sl = lane; sl < SLOTS; sl += 64) {
#pragma unroll
    for (int qn = 0; qn < POSE_PARTIALS; qn++) { tot[qn] += slots[sl * POSE_PARTIALS + qn]; slots[sl * POSE_PARTIALS + qn] = 0.0; }
  }
#pragma unroll
  for (int qn = 0; qn < POSE_PARTIALS; qn++)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tot[qn] += __shfl_xor(tot[qn], o);
  if (lane == 0) {
#pragma unroll
    for (int qn = 0; qn < POSE_PARTIALS; qn++) acc_t[6 + qn] += tot[qn];
  }
}

// sensor loss: one workgroup
__global__ __launch_bounds__(256) void k_gas_sensors(const float* __restrict__ T, size_t nc, int n,
                                                     const int* __restrict__ cells, const float* __restrict__ targets,
                                                     float* __restrict__ loss, float* __restrict__ gT) {
  __shared__ double s_l[256];
  double l = 0.0;
  for (int m = threadIdx.x; m < n; m += blockDim.x) {
    const int c = cells[m];
    if (c < 0 || (size_t)c >= nc) continue;
    const float e = T[c] - targets[m];
    l += fabs((double)e);
    if (gT) atomicAdd(&gT[c], e > 0.f ? 1.f : (e < 0.f ? -1.f : 0.f));
  }
  s_l[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s_l[threadIdx.x] += s_l[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)s_l[0];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct Layout {
  size_t tmp, pose, act, acc, slots, resp, resout, err, ckpt, seg, adj0, adj1, ub;
  size_t spec_tmp, dct[3], idct[3], lam[3];   // spectral solve: a cell array, per-axis matrices and eigenvalues
  size_t psi[MAX_LEVELS], f[MAX_LEVELS];
  size_t total;
  size_t state_floats;
  int n_levels, n_grid_levels, n_ckpt;
  Dims D[MAX_LEVELS];
};

bool desc_ok(const gas_desc* d) {
  if (!d) return false;
  const int n[3] = {d->nx, d->ny, d->nz};
  for (int a = 0; a < 3; a++)
    if (n[a] < 8 || n[a] > 1024 || (n[a] % 4) != 0) return false;
  if (!(d->h > 0.f) || !(d->dt > 0.f)) return false;
  if (d->n_scalars < 1 || d->n_scalars > MAXK || !d->src) return false;
  if (!(d->emit_sigma > 0.f) || !(d->emit_kappa >= 0.f && d->emit_kappa <= 1.f)) return false;
  if (d->horizon < 1 || d->mg_cycles < 1 || d->mg_cycles > 64) return false;
  if (d->pressure_solver != 0 && d->pressure_solver != 1) return false;
  if (d->requires_grad && (d->ckpt_every < 1 || d->ckpt_every > 4096)) return false;
  return true;
}

Layout plan(const gas_desc* d);

// (the coarsest level must fit the one-workgroup bottom solve)
bool levels_ok(const gas_desc* d);

Layout plan(const gas_desc* d) {
  Layout L;
  const size_t nx = d->nx, ny = d->ny, nz = d->nz, K = d->n_scalars, T = d->horizon;
  const size_t nc = nx * ny * nz;
  L.state_floats = (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1) + K * nc;
  // levels: halve while every dimension stays even and at least 2
  L.D[0] = Dims{d->nx, d->ny, d->nz};
  L.n_levels = 1;
  while (L.n_levels < MAX_LEVELS) {
    const Dims p = L.D[L.n_levels - 1];
    if ((p.x & 1) || (p.y & 1) || (p.z & 1) || p.x < 4 || p.y < 4 || p.z < 4) break;
    L.D[L.n_levels++] = Dims{p.x / 2, p.y / 2, p.z / 2};
  }
  // the grid levels end where the levels fit one workgroup's LDS
  L.n_grid_levels = 0;
  while (L.n_grid_levels < L.n_levels && L.D[L.n_grid_levels].cells() > (size_t)BOTTOM_CELLS) L.n_grid_levels++;
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o += al256(b); return r; };
  L.tmp = take(L.state_floats * 4);
  {
    const int nn[3] = {d->nx, d->ny, d->nz};
    L.spec_tmp = take(nc * 4);
    for (int a = 0; a < 3; a++) {
      L.dct[a] = take((size_t)nn[a] * nn[a] * 4);
      L.idct[a] = take((size_t)nn[a] * nn[a] * 4);
      L.lam[a] = take((size_t)nn[a] * 4);
    }
  }
  for (int l = 0; l < L.n_levels; l++) { L.psi[l] = take(L.D[l].cells() * 4); L.f[l] = take(L.D[l].cells() * 4); }
  L.pose = take((T + 1) * POSE_DOUBLES * sizeof(double));
  L.act = take(T * 6 * sizeof(float));
  L.slots = take(SLOTS * POSE_PARTIALS * sizeof(double));
  L.resp = take(2 * 4096 * sizeof(double));
  L.resout = take(64);
  L.err = take(64);
  if (d->requires_grad) {
    const int k = d->ckpt_every;
    L.n_ckpt = (int)((T + k - 1) / k) + 1;
    L.acc = take(T * ACC_DOUBLES * sizeof(double));
    L.ckpt = take(al256(L.state_floats * 4) * L.n_ckpt);
    L.seg = take(al256(L.state_floats * 4) * (size_t)k);
    L.adj0 = take(L.state_floats * 4);
    L.adj1 = take(L.state_floats * 4);
    L.ub = take(3 * (nc + (nx + 1) * ny * nz + nx * (ny + 1) * nz + nx * ny * (nz + 1)) * 4);
  } else {
    L.n_ckpt = 0;
    L.acc = L.ckpt = L.seg = L.adj0 = L.adj1 = L.ub = 0;
  }
  L.total = o;
  return L;
}

bool levels_ok(const gas_desc* d) {
  if (d->pressure_solver == 0) return true;   // (the spectral solve has no hierarchy)
  const Layout L = plan(d);
  return L.n_grid_levels < L.n_levels;
}

}  // namespace
}  // namespace mpm

using namespace mpm;

struct gas_ctx {
  gas_desc d;
  Layout L;
  GP P;
  hipStream_t stream;
  char* ws;
  std::vector<float> src;
  std::vector<char> act_set;
  gas_state user;
  bool has_state;
  int t;
  bool stats;
  double last_res;
  int last_err_bits;
  KernelTimer t_adv, t_smooth;
};

namespace {

// a packed state: u, v, w, s consecutive
gas_state packed(gas_ctx* c, char* base) {
  const GP& P = c->P;
  gas_state s;
  s.u = (float*)base;
  s.v = s.u + P.nu;
  s.w = s.v + P.nv;
  s.s = s.w + P.nw;
  return s;
}
size_t state_stride(gas_ctx* c) { return al256(c->L.state_floats * 4); }
const double* pose_at(gas_ctx* c, int t) { return (const double*)(c->ws + c->L.pose) + (size_t)t * POSE_DOUBLES; }

void copy_state(gas_ctx* c, const gas_state& a, const gas_state& b) {
  const GP& P = c->P;
  hipMemcpyAsync(b.u, a.u, P.nu * 4, hipMemcpyDeviceToDevice, c->stream);
  hipMemcpyAsync(b.v, a.v, P.nv * 4, hipMemcpyDeviceToDevice, c->stream);
  hipMemcpyAsync(b.w, a.w, P.nw * 4, hipMemcpyDeviceToDevice, c->stream);
  hipMemcpyAsync(b.s, a.s, (size_t)P.K * P.nc * 4, hipMemcpyDeviceToDevice, c->stream);
}

// A psi = f on level 0 (psi0 holds the initial guess)
void mg_solve(gas_ctx* c, float* psi0, float* f0) {
  const Layout& L = c->L;
  hipStream_t s = c->stream;
  auto psi = [&](int l) { return l == 0 ? psi0 : (float*)(c->ws + L.psi[l]); };
  auto fl = [&](int l) { return l == 0 ? f0 : (float*)(c->ws + L.f[l]); };
  const int G = L.n_grid_levels;
  BottomArgs B;
  B.n_levels = L.n_levels - G;
  for (int l = 0; l < B.n_levels; l++) B.D[l] = L.D[G + l];
  B.psi = psi(G);
  B.f = fl(G);
  auto tiles = [&](int l) {
    const Dims& D = L.D[l];
    return dim3((D.x + TX - 1) / TX, (D.y + TY - 1) / TY, (D.z + TZ - 1) / TZ);
  };
  // V(2,2): red-black sweeps before each restriction, black-red sweeps after
  // each correction (the first of them adds the correction as it stages)
  for (int cyc = 0; cyc < c->d.mg_cycles; cyc++) {
    for (int l = 0; l < G; l++) {
      for (int sw = 0; sw < (l == 0 ? NU0_PRE : 2); sw++) {
        if (l < HALF_LEVELS) {
          for (int color = 0; color < 2; color++) {
            if (l == 0) c->t_smooth.begin(s);
            k_rb_half<<<nblk(L.D[l].cells() / 2, 256), 256, 0, s>>>(psi(l), fl(l), L.D[l], color);
            if (l == 0) c->t_smooth.end(s);
          }
          continue;
        }
        if (l == 0) c->t_smooth.begin(s);
        k_rb_sweep<<<tiles(l), 256, 0, s>>>(psi(l), fl(l), L.D[l], 0, nullptr, L.D[l]);
        if (l == 0) c->t_smooth.end(s);
      }
      k_restrict<<<nblk(L.D[l + 1].cells(), 256), 256, 0, s>>>(psi(l), fl(l), L.D[l], psi(l + 1), fl(l + 1), L.D[l + 1]);
    }
    k_bottom<<<1, BOTTOM_THREADS, 0, s>>>(B);
    for (int l = G - 1; l >= 0; l--) {
      if (l < HALF_LEVELS)
        k_prolong<<<nblk(L.D[l].cells(), 256), 256, 0, s>>>(psi(l + 1), L.D[l + 1], psi(l), L.D[l]);
      for (int sw = 0; sw < (l == 0 ? NU0_POST : NU_POST); sw++) {
        if (l < HALF_LEVELS) {
          for (int color = 1; color >= 0; color--) {
            if (l == 0) c->t_smooth.begin(s);
            k_rb_half<<<nblk(L.D[l].cells() / 2, 256), 256, 0, s>>>(psi(l), fl(l), L.D[l], color);
            if (l == 0) c->t_smooth.end(s);
          }
          continue;
        }
        if (l == 0) c->t_smooth.begin(s);
        k_rb_sweep<<<tiles(l), 256, 0, s>>>(psi(l), fl(l), L.D[l], 1, sw == 0 ? psi(l + 1) : nullptr, L.D[l + 1]);
        if (l == 0) c->t_smooth.end(s);
      }
    }
  }
  if (c->stats) {
    const unsigned nb = min(nblk(L.D[0].cells(), 256), 4096u);
    k_resnorm<<<nb, 256, 0, s>>>(psi0, f0, L.D[0], (double*)(c->ws + L.resp));
    k_resnorm_final<<<1, 64, 0, s>>>((const double*)(c->ws + L.resp), (int)nb, (double*)(c->ws + L.resout));
  }
}

// one transform pass; grid.z splits the n outputs into chunks of XK (16 up to
// n = 128, 64 above: measured fastest at 64^3, 128^3 and 256^3)
template <bool INNER>
void launch_axis(const AxisArgs& X, dim3 grid, hipStream_t s) {
  if (X.n <= 128) {
    grid.z = (X.n + 15) / 16;
    k_axis<INNER, 16, 64><<<grid, 256, 0, s>>>(X);
  } else {
    grid.z = (X.n + 63) / 64;
    k_axis<INNER, 64, 64><<<grid, 256, 0, s>>>(X);
  }
}

// A psi = f exactly by the axis transforms (psi0 receives the solution with
// zero mean; f0 is left unchanged)
void spectral_solve(gas_ctx* c, float* psi0, const float* f0) {
  const GP& P = c->P;
  hipStream_t s = c->stream;
  float* T = (float*)(c->ws + c->L.spec_tmp);
  const float* Mf[3] = {(const float*)(c->ws + c->L.dct[0]), (const float*)(c->ws + c->L.dct[1]),
                        (const float*)(c->ws + c->L.dct[2])};
  const float* Mi[3] = {(const float*)(c->ws + c->L.idct[0]), (const float*)(c->ws + c->L.idct[1]),
                        (const float*)(c->ws + c->L.idct[2])};
  const float* lam[3] = {(const float*)(c->ws + c->L.lam[0]), (const float*)(c->ws + c->L.lam[1]),
                         (const float*)(c->ws + c->L.lam[2])};
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  auto pass = [&](int axis, const float* in, float* out, const float* M, bool divide) {
    AxisArgs X = {};
    X.in = in; X.out = out; X.M = M;
    if (axis == 2) {
      X.n = nz; X.A = nx * ny; X.B = 1;
      launch_axis<true>(X, dim3((X.A + XB - 1) / XB, 1, 1), s);
      return;
    }
    X.n = axis == 0 ? nx : ny;
    X.A = axis == 0 ? 1 : nx;
    X.B = axis == 0 ? ny * nz : nz;
    if (divide) { X.lx = lam[0]; X.ly = lam[1]; X.lz = lam[2]; X.nz = nz; }
    launch_axis<false>(X, dim3((X.B + XB - 1) / XB, X.A, 1), s);
  };
  // one event pair around the six back-to-back transforms (read as six
  // launches): a pair per launch would add its own overhead to each
  c->t_smooth.begin(s);
  pass(2, f0, T, Mf[2], false);
  pass(1, T, psi0, Mf[1], false);
  pass(0, psi0, T, Mf[0], true);
  pass(0, T, psi0, Mi[0], false);
  pass(1, psi0, T, Mi[1], false);
  pass(2, T, psi0, Mi[2], false);
  c->t_smooth.end(s);
}

void pressure_solve(gas_ctx* c, float* psi0, float* f0) {
  if (c->d.pressure_solver != 0) {
    mg_solve(c, psi0, f0);
    return;
  }
  spectral_solve(c, psi0, f0);
  if (c->stats) {
    const Layout& L = c->L;
    const unsigned nb = min(nblk(L.D[0].cells(), 256), 4096u);
    k_resnorm<<<nb, 256, 0, c->stream>>>(psi0, f0, L.D[0], (double*)(c->ws + L.resp));
    k_resnorm_final<<<1, 64, 0, c->stream>>>((const double*)(c->ws + L.resp), (int)nb, (double*)(c->ws + L.resout));
  }
}

// one forward step from `in` to `out` (distinct), emitter at pose t
void gas_forward_step(gas_ctx* c, const gas_state& in, const gas_state& out, int t) {
  const GP& P = c->P;
  hipStream_t s = c->stream;
  gas_state tmp = packed(c, c->ws + c->L.tmp);
  float* psi0 = (float*)(c->ws + c->L.psi[0]);
  float* f0 = (float*)(c->ws + c->L.f[0]);
  const size_t pts = P.nu + P.nv + P.nw + P.nc;
  c->t_adv.begin(s);
  k_gas_advect<<<nblk(pts, 256), 256, 0, s>>>(P, VelPtrs{in.u, in.v, in.w}, in.s, tmp.u, tmp.v, tmp.w, tmp.s,
                                             pose_at(c, t));
  c->t_adv.end(s);
  k_gas_div<<<nblk(P.nc, 256), 256, 0, s>>>(P, tmp.u, tmp.v, tmp.w, tmp.s, f0, psi0);
  pressure_solve(c, psi0, f0);
  const size_t tot = P.nu + P.nv + P.nw + (size_t)P.K * P.nc;
  k_gas_final<<<nblk(tot, 256), 256, 0, s>>>(P, tmp.u, tmp.v, tmp.w, tmp.s, psi0, out.u, out.v, out.w, out.s);
}

// one adjoint step: abar_next (adjoint of s_{t+1}) -> abar (adjoint of s_t);
// st is s_t
void gas_adjoint_step(gas_ctx* c, const gas_state& st, const gas_state& an, const gas_state& ab, int t, double* acc_t) {
  const GP& P = c->P;
  hipStream_t s = c->stream;
  gas_state tmp = packed(c, c->ws + c->L.tmp);
  float* psi0 = (float*)(c->ws + c->L.psi[0]);
  float* f0 = (float*)(c->ws + c->L.f[0]);
  k_gas_adj_div<<<nblk(P.nc, 256), 256, 0, s>>>(P, an.u, an.v, an.w, f0, psi0);
  pressure_solve(c, psi0, f0);
  k_gas_adj_sub<<<nblk(P.nu + P.nv + P.nw, 256), 256, 0, s>>>(P, an.u, an.v, an.w, psi0, tmp.u, tmp.v, tmp.w);
  launch_zero(ab.u, c->L.state_floats * 4, s);
  const size_t pts = P.nu + P.nv + P.nw + P.nc;
  k_gas_adj_advect<<<nblk(pts, 256), 256, 0, s>>>(P, VelPtrs{st.u, st.v, st.w}, st.s, tmp.u, tmp.v, tmp.w, an.s,
                                                 AdjOut{ab.u, ab.v, ab.w, ab.s}, pose_at(c, t),
                                                 (double*)(c->ws + c->L.slots), (float*)(c->ws + c->L.ub));
  k_gas_adj_ugather<<<nblk(P.nu + P.nv + P.nw, 256), 256, 0, s>>>(P, (const float*)(c->ws + c->L.ub),
                                                                  AdjOut{ab.u, ab.v, ab.w, ab.s});
  k_gas_pose_acc<<<1, 64, 0, s>>>((double*)(c->ws + c->L.slots), acc_t);
}

// Waits for the call's work; reads (and clears) the device error word.
int sync_ok(gas_ctx* c) {
  int bits = 0;
  if (hipMemcpyAsync(&bits, c->ws + c->L.err, sizeof(int), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return MPM_EHIP;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return MPM_EHIP;
  if (hipGetLastError() != hipSuccess) return MPM_EHIP;
  c->t_adv.collect();
  c->t_smooth.collect();
  if (c->stats) {
    double r = 0.0;
    if (hipMemcpy(&r, c->ws + c->L.resout, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return MPM_EHIP;
    c->last_res = r;
  }
  if (bits) {
    c->last_err_bits = bits;
    if (hipMemsetAsync(c->ws + c->L.err, 0, sizeof(int), c->stream) != hipSuccess) return MPM_EHIP;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return MPM_EHIP;
    return MPM_EDOMAIN;
  }
  return MPM_OK;
}

}  // namespace

extern "C" {

size_t gas_workspace_bytes(const gas_desc* d) {
  if (!desc_ok(d) || !levels_ok(d)) return 0;
  return plan(d).total;
}

int gas_create(const gas_desc* d, void* workspace_dev, size_t ws_bytes, void* stream, gas_ctx** out) {
  if (!out) return MPM_EINVAL;
  *out = nullptr;
  if (!desc_ok(d) || !levels_ok(d) || !workspace_dev || ((uintptr_t)workspace_dev % 256)) return MPM_EINVAL;
  Layout L = plan(d);
  if (ws_bytes < L.total) return MPM_EWORKSPACE;
  gas_ctx* c = new (std::nothrow) gas_ctx();
  if (!c) return MPM_EINVAL;
  c->d = *d;
  c->src.assign(d->src, d->src + d->n_scalars);
  c->d.src = c->src.data();
  c->L = L;
  c->stream = (hipStream_t)stream;
  c->ws = (char*)workspace_dev;
  c->has_state = false;
  c->t = 0;
  c->stats = false;
  c->last_res = 0.0;
  c->last_err_bits = 0;
  c->t_adv.name = "k_gas_advect";
  c->t_smooth.name = d->pressure_solver == 0 ? "k_axis" : "k_rb_half";
  c->act_set.assign(d->horizon, 0);
  GP& P = c->P;
  P.nx = d->nx; P.ny = d->ny; P.nz = d->nz; P.K = d->n_scalars;
  P.h = d->h; P.inv_h = 1.f / d->h; P.dt = d->dt; P.beta = d->buoyancy; P.t_amb = d->t_amb;
  P.s2inv = 1.f / (2.f * d->emit_sigma * d->emit_sigma);
  P.kappa = d->emit_kappa;
  P.speed = d->emit_speed;
  for (int k = 0; k < MAXK; k++) P.src[k] = k < d->n_scalars ? d->src[k] : 0.f;
  P.nu = (size_t)(d->nx + 1) * d->ny * d->nz;
  P.nv = (size_t)d->nx * (d->ny + 1) * d->nz;
  P.nw = (size_t)d->nx * d->ny * (d->nz + 1);
  P.nc = (size_t)d->nx * d->ny * d->nz;
  P.err = (int*)(c->ws + L.err);
  launch_zero(c->ws + L.slots, SLOTS * POSE_PARTIALS * sizeof(double), c->stream);
  launch_zero(c->ws + L.err, 64, c->stream);
  // spectral tables: per axis the DCT-II matrix C[i][k] = cos(pi k (i + 1/2) / n),
  // its inverse Ci[k][i] = w_k C[i][k] (w_0 = 1/n, w_k = 2/n) and the 1-D
  // Neumann eigenvalues -4 sin^2(pi k / 2n), computed in FP64
  {
    const int nn[3] = {d->nx, d->ny, d->nz};
    for (int a = 0; a < 3; a++) {
      const int n = nn[a];
      std::vector<float> C((size_t)n * n), Ci((size_t)n * n), lam(n);
      for (int i = 0; i < n; i++)
        for (int k = 0; k < n; k++) {
          const double v = cos(M_PI * k * (i + 0.5) / n);
          C[(size_t)i * n + k] = (float)v;
          Ci[(size_t)k * n + i] = (float)(v * (k == 0 ? 1.0 / n : 2.0 / n));
        }
      for (int k = 0; k < n; k++) {
        const double sk = sin(M_PI * k / (2.0 * n));
        lam[k] = (float)(-4.0 * sk * sk);
      }
      if (hipMemcpy(c->ws + L.dct[a], C.data(), C.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(c->ws + L.idct[a], Ci.data(), Ci.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
          hipMemcpy(c->ws + L.lam[a], lam.data(), lam.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
        delete c;
        return MPM_EHIP;
      }
    }
  }
  if (hipStreamSynchronize(c->stream) != hipSuccess || hipGetLastError() != hipSuccess) { delete c; return MPM_EHIP; }
  *out = c;
  return MPM_OK;
}

int gas_set_state(gas_ctx* c, const gas_state* st) {
  if (!c || !st || !st->u || !st->v || !st->w || !st->s) return MPM_EINVAL;
  c->user = *st;
  c->has_state = true;
  c->t = 0;
  double pose0[POSE_DOUBLES];
  for (int k = 0; k < 3; k++) pose0[k] = c->d.emit_pos0[k];
  for (int k = 0; k < 9; k++) pose0[3 + k] = c->d.emit_rot0[k];
  if (hipMemcpyAsync(c->ws + c->L.pose, pose0, sizeof(pose0), hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return MPM_EHIP;
  return sync_ok(c);
}

int gas_set_actions(gas_ctx* c, int32_t t0, int32_t n, const float* actions_dev) {
  if (!c || !actions_dev || t0 < 0 || n < 1 || t0 + n > c->d.horizon) return MPM_EINVAL;
  if (hipMemcpyAsync(c->ws + c->L.act + (size_t)t0 * 6 * sizeof(float), actions_dev, (size_t)n * 6 * sizeof(float),
                     hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return MPM_EHIP;
  for (int t = t0; t < t0 + n; t++) c->act_set[t] = 1;
  return MPM_OK;
}

int gas_step(gas_ctx* c, int32_t n_steps) {
  if (!c || n_steps < 0) return MPM_EINVAL;
  if (!c->has_state) return MPM_ESTATE;
  if (n_steps == 0) return MPM_OK;
  if (c->t + n_steps > c->d.horizon) return MPM_EINVAL;
  for (int t = c->t; t < c->t + n_steps; t++)
    if (!c->act_set[t]) return MPM_ESTATE;
  launch_pose(1, c->t, n_steps, c->d.dt, (const float*)(c->ws + c->L.act), (double*)(c->ws + c->L.pose), c->stream);
  // the step reads the user arrays and writes them back through the
  // temporaries; a checkpoint is taken before every k-th step
  for (int t = c->t; t < c->t + n_steps; t++) {
    if (c->d.requires_grad && t % c->d.ckpt_every == 0)
      copy_state(c, c->user, packed(c, c->ws + c->L.ckpt + (size_t)(t / c->d.ckpt_every) * state_stride(c)));
    gas_forward_step(c, c->user, c->user, t);
  }
  c->t += n_steps;
  if (hipGetLastError() != hipSuccess) return MPM_EHIP;
  return sync_ok(c);
}

int gas_step_backward(gas_ctx* c, const gas_state* grad_T, float* grad_actions_dev, gas_state* grad_0) {
  if (!c || !grad_T || !grad_T->u || !grad_T->v || !grad_T->w || !grad_actions_dev) return MPM_EINVAL;
  if (!c->has_state || !c->d.requires_grad || c->t < 1) return MPM_ESTATE;
  if (grad_0 && (!grad_0->u || !grad_0->v || !grad_0->w || !grad_0->s)) return MPM_EINVAL;
  const GP& P = c->P;
  hipStream_t s = c->stream;
  const int T = c->t, k = c->d.ckpt_every;
  gas_state a_cur = packed(c, c->ws + c->L.adj0), a_nxt = packed(c, c->ws + c->L.adj1);
  launch_zero(a_cur.u, c->L.state_floats * 4, s);
  hipMemcpyAsync(a_cur.u, grad_T->u, P.nu * 4, hipMemcpyDeviceToDevice, s);
  hipMemcpyAsync(a_cur.v, grad_T->v, P.nv * 4, hipMemcpyDeviceToDevice, s);
  hipMemcpyAsync(a_cur.w, grad_T->w, P.nw * 4, hipMemcpyDeviceToDevice, s);
  if (grad_T->s) hipMemcpyAsync(a_cur.s, grad_T->s, (size_t)P.K * P.nc * 4, hipMemcpyDeviceToDevice, s);
  double* acc = (double*)(c->ws + c->L.acc);
  launch_zero(acc, al256((size_t)T * ACC_DOUBLES * sizeof(double)), s);
  const int n_seg = (T + k - 1) / k;
  for (int seg = n_seg - 1; seg >= 0; seg--) {
    const int ts = seg * k, te = ts + k < T ? ts + k : T;
    // recompute s_ts .. s_{te-1} into the segment slots
    copy_state(c, packed(c, c->ws + c->L.ckpt + (size_t)seg * state_stride(c)), packed(c, c->ws + c->L.seg));
    for (int t = ts; t + 1 < te; t++)
      gas_forward_step(c, packed(c, c->ws + c->L.seg + (size_t)(t - ts) * state_stride(c)),
                       packed(c, c->ws + c->L.seg + (size_t)(t - ts + 1) * state_stride(c)), t);
    for (int t = te - 1; t >= ts; t--) {
      gas_adjoint_step(c, packed(c, c->ws + c->L.seg + (size_t)(t - ts) * state_stride(c)), a_cur, a_nxt, t,
                       acc + (size_t)t * ACC_DOUBLES);
      gas_state sw = a_cur; a_cur = a_nxt; a_nxt = sw;
    }
  }
  launch_pose_adj(1, T, c->d.dt, (const float*)(c->ws + c->L.act), (const double*)(c->ws + c->L.pose), acc,
                  grad_actions_dev, s);
  if (grad_0) copy_state(c, a_cur, *grad_0);
  if (hipGetLastError() != hipSuccess) return MPM_EHIP;
  return sync_ok(c);
}

int gas_sensor_loss(gas_ctx* c, int32_t n, const int32_t* cells_dev, const float* targets_dev, float* loss_dev,
                    gas_state* grad_out) {
  if (!c || n < 1 || !cells_dev || !targets_dev || !loss_dev) return MPM_EINVAL;
  if (!c->has_state) return MPM_ESTATE;
  const GP& P = c->P;
  float* gT = nullptr;
  if (grad_out) {
    if (!grad_out->u || !grad_out->v || !grad_out->w || !grad_out->s) return MPM_EINVAL;
    hipMemsetAsync(grad_out->u, 0, P.nu * 4, c->stream);
    hipMemsetAsync(grad_out->v, 0, P.nv * 4, c->stream);
    hipMemsetAsync(grad_out->w, 0, P.nw * 4, c->stream);
    hipMemsetAsync(grad_out->s, 0, (size_t)P.K * P.nc * 4, c->stream);
    gT = grad_out->s;
  }
  k_gas_sensors<<<1, 256, 0, c->stream>>>(c->user.s, P.nc, n, cells_dev, targets_dev, loss_dev, gT);
  if (hipGetLastError() != hipSuccess) return MPM_EHIP;
  return sync_ok(c);
}

int gas_enable_stats(gas_ctx* c, int32_t enable) {
  if (!c) return MPM_EINVAL;
  c->stats = enable != 0;
  return MPM_OK;
}

int gas_solver_residual(gas_ctx* c, double* rel_residual) {
  if (!c || !rel_residual) return MPM_EINVAL;
  *rel_residual = c->last_res;
  return MPM_OK;
}

int gas_timing_enable(gas_ctx* c, int32_t enable) {
  if (!c) return MPM_EINVAL;
  c->t_adv.on = c->t_smooth.on = enable != 0;
  c->t_adv.total_ms = c->t_smooth.total_ms = 0.0;
  c->t_adv.launches = c->t_smooth.launches = 0;
  c->t_adv.used = c->t_smooth.used = 0;
  return MPM_OK;
}

int gas_timing_read(gas_ctx* c, double* advect_ms, int64_t* advect_launches, double* smooth_ms,
                    int64_t* smooth_launches) {
  if (!c || !advect_ms || !advect_launches || !smooth_ms || !smooth_launches) return MPM_EINVAL;
  *advect_ms = c->t_adv.total_ms;
  *advect_launches = c->t_adv.launches;
  *smooth_ms = c->t_smooth.total_ms;
  *smooth_launches = c->t_smooth.launches * (c->d.pressure_solver == 0 ? 6 : 1);
  c->t_adv.total_ms = c->t_smooth.total_ms = 0.0;
  c->t_adv.launches = c->t_smooth.launches = 0;
  return MPM_OK;
}

int gas_last_error_bits(const gas_ctx* c, int32_t* bits_out) {
  if (!c || !bits_out) return MPM_EINVAL;
  *bits_out = c->last_err_bits;
  return MPM_OK;
}

int gas_clock(const gas_ctx* c, int32_t* t_out) {
  if (!c || !t_out) return MPM_EINVAL;
  *t_out = c->t;
  return MPM_OK;
}

int gas_destroy(gas_ctx* c) {
  if (!c) return MPM_EINVAL;
  c->t_adv.destroy();
  c->t_smooth.destroy();
  delete c;
  return MPM_OK;
}

}  // extern "C"
