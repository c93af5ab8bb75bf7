// Small MLP (6 -> 64 -> 64 -> 3, ReLU) standing in for the Drucker-Prager
// cone return: BF16 weights, FP32 accumulation on the gfx950 matrix cores
// (v_mfma_f32_16x16x16_bf16), evaluated by one wavefront for its 64 lanes.
//
// Input (per sample): log singular values of the trial F sorted descending,
// then the cone slope alpha, the cohesion c and kappa = (3 lam + 2 mu)/(2 mu).
// Output: the projected log singular values (same order), shifted equally so
// that their sum equals that of the trial ones (the return is deviatoric).
// Inputs and outputs are normalised with fixed means and deviations stored
// with the weights.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpm {

// Order the LDS writes of a wavefront's lanes before the other lanes' reads
// of them: a wavefront-scope release/acquire pair around the wave barrier
// (the lanes of a 64-wide wavefront execute together; only the compiler's
// and the memory counters' ordering has to be enforced).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


constexpr int MLP_IN = 6, MLP_H = 64, MLP_OUT = 3;
constexpr int MLP_NPARAM = MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_OUT * MLP_H + MLP_OUT;  // 4803
constexpr int MLP_K1 = 16;   // layer-1 reduction dim padded to the MFMA k
constexpr int MLP_N3 = 16;   // layer-3 output dim padded to the MFMA n

// Offsets (in floats) of the FP32 parameter vector (the training master copy).
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + MLP_H * MLP_IN;
constexpr int OFF_W2 = OFF_B1 + MLP_H;
constexpr int OFF_B2 = OFF_W2 + MLP_H * MLP_H;
constexpr int OFF_W3 = OFF_B2 + MLP_H;
constexpr int OFF_B3 = OFF_W3 + MLP_OUT * MLP_H;

// Device blob used for inference: normalisation, FP32 biases and BF16
// weights, row-major [n][k] with padding (so a B fragment is 8 contiguous bytes).
struct MlpBlob {
  float in_mean[MLP_IN], in_std[MLP_IN], out_mean[MLP_OUT], out_std[MLP_OUT];
  float b1[MLP_H], b2[MLP_H], b3[MLP_N3];
  uint16_t W1[MLP_H * MLP_K1];
  uint16_t W2[MLP_H * MLP_H];
  uint16_t W3[MLP_N3 * MLP_H];
};

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even
  uint32_t u = __float_as_uint(f);
  uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(r >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// Per-wavefront LDS scratch of the forward: one 16 x 64 BF16 activation row
// block (with a pad column to spread banks) and the 64 x 3 outputs.
constexpr int MLP_HROW = MLP_H + 4;
struct MlpScratch {
  uint16_t h[16 * MLP_HROW];
  float y[64 * MLP_OUT];
};

// Forward of the 64 samples held by the lanes of one wavefront (lane l holds
// sample l).  Every lane must call it.  Optionally returns the BF16-rounded
// hidden activations of the lane's sample (as the next layer consumed them).
// Matrix-core layout of v_mfma_f32_16x16x16_bf16 (a 16-sample row block):
//   A[row = l % 16][k = 4 (l / 16) + q], B[k = 4 (l / 16) + q][col = l % 16],
//   D[row = 4 (l / 16) + q][col = l % 16],  q = 0..3.
__device__ inline void mlp_wave_forward(const MlpBlob& W, const float* x, float* y, MlpScratch& S,
                                        float* h1_out = nullptr, float* h2_out = nullptr) {
  const int l = __lane_id();
  const int lr = l & 15, lg = l >> 4;
  float xn[MLP_IN];
#pragma unroll
  for (int i = 0; i < MLP_IN; i++) xn[i] = (x[i] - W.in_mean[i]) / W.in_std[i];
  for (int rb = 0; rb < 4; rb++) {
    // ---- layer 1: A = inputs of samples 16 rb + lr, k = 4 lg + q
    const int src = 16 * rb + lr;
    float xs[MLP_IN];
#pragma unroll
    for (int i = 0; i < MLP_IN; i++) xs[i] = __shfl(xn[i], src);
    bf16x4_t a1;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int k = 4 * lg + q;
      float v = 0.f;
#pragma unroll
      for (int i = 0; i < MLP_IN; i++) v = (k == i) ? xs[i] : v;
      a1[q] = (short)f2bf(v);
    }
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      bf16x4_t b;
      const uint16_t* wp = W.W1 + (16 * nt + lr) * MLP_K1 + 4 * lg;
#pragma unroll
      for (int q = 0; q < 4; q++) b[q] = (short)wp[q];
      f32x4_t c = {0.f, 0.f, 0.f, 0.f};
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b, c, 0, 0, 0);
      const int col = 16 * nt + lr;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        float h = fmaxf(c[q] + W.b1[col], 0.f);
        S.h[(4 * lg + q) * MLP_HROW + col] = f2bf(h);
      }
    }
    wave_lds_sync();
    // ---- layer 2: A = H1 (row lr, k = 16 kt + 4 lg + q)
    bf16x4_t a2[4];
#pragma unroll
    for (int kt = 0; kt < 4; kt++)
#pragma unroll
      for (int q = 0; q < 4; q++) a2[kt][q] = (short)S.h[lr * MLP_HROW + 16 * kt + 4 * lg + q];
    if (h1_out) {
      // the lane's own sample, if it lies in this row block
      if ((l >> 4) == rb) {
#pragma unroll
        for (int k = 0; k < MLP_H; k++) h1_out[k] = bf2f(S.h[(l & 15) * MLP_HROW + k]);
      }
    }
    wave_lds_sync();
    f32x4_t c2[4];
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      c2[nt] = f32x4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kt = 0; kt < 4; kt++) {
        bf16x4_t b;
        const uint16_t* wp = W.W2 + (16 * nt + lr) * MLP_H + 16 * kt + 4 * lg;
#pragma unroll
        for (int q = 0; q < 4; q++) b[q] = (short)wp[q];
        c2[nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2[kt], b, c2[nt], 0, 0, 0);
      }
    }
#pragma unroll
    for (int nt = 0; nt < 4; nt++) {
      const int col = 16 * nt + lr;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        float h = fmaxf(c2[nt][q] + W.b2[col], 0.f);
        S.h[(4 * lg + q) * MLP_HROW + col] = f2bf(h);
      }
    }
    wave_lds_sync();
    // ---- layer 3: A = H2, B = W3 (n padded to 16)
    bf16x4_t a3[4];
#pragma unroll
    for (int kt = 0; kt < 4; kt++)
#pragma unroll
      for (int q = 0; q < 4; q++) a3[kt][q] = (short)S.h[lr * MLP_HROW + 16 * kt + 4 * lg + q];
    if (h2_out) {
      if ((l >> 4) == rb) {
#pragma unroll
        for (int k = 0; k < MLP_H; k++) h2_out[k] = bf2f(S.h[(l & 15) * MLP_HROW + k]);
      }
    }
    f32x4_t c3 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kt = 0; kt < 4; kt++) {
      bf16x4_t b;
      const uint16_t* wp = W.W3 + lr * MLP_H + 16 * kt + 4 * lg;
#pragma unroll
      for (int q = 0; q < 4; q++) b[q] = (short)wp[q];
      c3 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a3[kt], b, c3, 0, 0, 0);
    }
    if (lr < MLP_OUT) {
#pragma unroll
      for (int q = 0; q < 4; q++) S.y[(16 * rb + 4 * lg + q) * MLP_OUT + lr] = c3[q] + W.b3[lr];
    }
    wave_lds_sync();
  }
#pragma unroll
  for (int o = 0; o < MLP_OUT; o++) y[o] = S.y[l * MLP_OUT + o] * W.out_std[o] + W.out_mean[o];
  // the cone return changes only the deviatoric part of the log strain, so
  // the output is projected onto the inputs' trace: tr y = tr x
  const float dtr = ((x[0] + x[1] + x[2]) - (y[0] + y[1] + y[2])) * (1.f / 3.f);
#pragma unroll
  for (int o = 0; o < MLP_OUT; o++) y[o] += dtr;
  wave_lds_sync();
}

}  // namespace mpm
