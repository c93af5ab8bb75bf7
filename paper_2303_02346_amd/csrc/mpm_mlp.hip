// Training and batch inference of the learned cone-return closure
// (6 -> 64 -> 64 -> 3 MLP, ReLU).  The forward runs on the matrix cores in
// BF16 with FP32 accumulation (mlp_wave_forward); the backward and Adam run
// in FP32.  Loss: mean squared error of the normalised outputs.
//
// State layout (device, caller-owned, mpm_mlp_state_bytes()):
//   params  FP32 [MLP_NPARAM]   master weights W1 b1 W2 b2 W3 b3 (row-major [out][in])
//   adam_m  FP32 [MLP_NPARAM]
//   adam_v  FP32 [MLP_NPARAM]
//   grad    FP32 [MLP_NPARAM]
//   misc    FP64 [8]            loss accumulator, step count
//   blob    MlpBlob             inference copy (normalisation, FP32 biases, BF16 weights)
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <mutex>
#include <random>
#include <vector>

#include "../../include/mpm.h"
#include "mpm_mlp.h"

namespace mpm {

namespace {
constexpr size_t A256 = 256;
inline size_t al(size_t x) { return (x + A256 - 1) & ~(A256 - 1); }

struct MlpLayout {
  size_t params, m, v, grad, misc, blob, total;
};
MlpLayout mlp_layout() {
  MlpLayout L;
  size_t o = 0;
  L.params = o; o += al(MLP_NPARAM * 4);
  L.m = o; o += al(MLP_NPARAM * 4);
  L.v = o; o += al(MLP_NPARAM * 4);
  L.grad = o; o += al(MLP_NPARAM * 4);
  L.misc = o; o += al(64);
  L.blob = o; o += al(sizeof(MlpBlob));
  L.total = o;
  return L;
}
constexpr int SAMPLE = MLP_IN + MLP_OUT;   // floats per logged sample
// per-sample backward scratch: xn 6, dy 3 (slots 6..8), pad, h1 64, h2 64,
// dh1 64, dh2 64 (from slot 12)
constexpr int HDR = 12;
constexpr int SCR = HDR + 4 * MLP_H;
}  // namespace

// normalisation statistics (mean, std) of the 9 sample columns, FP64 sums
__global__ void k_mlp_stats(const float* __restrict__ samples, long long n, double* __restrict__ acc) {
  double s[SAMPLE], q[SAMPLE];
#pragma unroll
  for (int c = 0; c < SAMPLE; c++) { s[c] = 0.0; q[c] = 0.0; }
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < SAMPLE; c++) { double v = samples[i * SAMPLE + c]; s[c] += v; q[c] += v * v; }
  }
#pragma unroll
  for (int c = 0; c < SAMPLE; c++) {
    for (int off = 32; off > 0; off >>= 1) { s[c] += __shfl_xor(s[c], off); q[c] += __shfl_xor(q[c], off); }
    if ((threadIdx.x & 63) == 0) { atomicAdd(acc + c, s[c]); atomicAdd(acc + SAMPLE + c, q[c]); }
  }
}

__global__ void k_mlp_stats_final(const double* __restrict__ acc, long long n, MlpBlob* __restrict__ blob) {
  int c = threadIdx.x;
  if (c >= SAMPLE) return;
  double mean = acc[c] / (double)n;
  double var = acc[SAMPLE + c] / (double)n - mean * mean;
  double sd = sqrt(var > 0.0 ? var : 0.0);
  // a column that barely varies in the training set (one material) keeps a
  // deviation floor so that other values stay in a sane range
  double floor_sd = 1e-4 + 1e-3 * fabs(mean);
  if (sd < floor_sd) sd = floor_sd;
  if (c < MLP_IN) { blob->in_mean[c] = (float)mean; blob->in_std[c] = (float)sd; }
  else { blob->out_mean[c - MLP_IN] = (float)mean; blob->out_std[c - MLP_IN] = (float)sd; }
}

// FP32 master parameters -> inference blob (BF16 weights, padded; FP32 biases)
__global__ void k_mlp_publish(const float* __restrict__ p, MlpBlob* __restrict__ blob) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < MLP_H * MLP_K1 + MLP_H * MLP_H + MLP_N3 * MLP_H + 2 * MLP_H + MLP_N3;
       i += gridDim.x * blockDim.x) {
    if (i < MLP_H * MLP_K1) {
      int n = i / MLP_K1, k = i % MLP_K1;
      blob->W1[i] = f2bf(k < MLP_IN ? p[OFF_W1 + n * MLP_IN + k] : 0.f);
      continue;
    }
    int j = i - MLP_H * MLP_K1;
    if (j < MLP_H * MLP_H) { blob->W2[j] = f2bf(p[OFF_W2 + j]); continue; }
    j -= MLP_H * MLP_H;
    if (j < MLP_N3 * MLP_H) {
      int n = j / MLP_H, k = j % MLP_H;
      blob->W3[j] = f2bf(n < MLP_OUT ? p[OFF_W3 + n * MLP_H + k] : 0.f);
      continue;
    }
    j -= MLP_N3 * MLP_H;
    if (j < MLP_H) { blob->b1[j] = p[OFF_B1 + j]; continue; }
    j -= MLP_H;
    if (j < MLP_H) { blob->b2[j] = p[OFF_B2 + j]; continue; }
    j -= MLP_H;
    blob->b3[j] = j < MLP_OUT ? p[OFF_B3 + j] : 0.f;
  }
}

// Forward (matrix cores) and per-sample backward of a batch.  One sample
// per thread, 256 threads; samples i0 .. i0 + nb - 1 (indices wrap at n).
// Writes the per-sample activations and adjoints to scr for the weight
// gradient kernel and adds the batch loss to misc[0].
__global__ __launch_bounds__(256) void k_mlp_batch(const MlpBlob* __restrict__ blob, const float* __restrict__ samples,
                                                   long long n, long long i0, int nb, float* __restrict__ scr,
                                                   double* __restrict__ misc, float* __restrict__ y_out) {
  __shared__ MlpBlob W;
  __shared__ MlpScratch S[4];
  {
    const uint32_t* src = (const uint32_t*)blob;
    uint32_t* dst = (uint32_t*)&W;
    for (int q = threadIdx.x; q < (int)(sizeof(MlpBlob) / 4); q += 256) dst[q] = src[q];
  }
  __syncthreads();
  const int b = blockIdx.x * 256 + threadIdx.x;        // sample slot in the batch
  const bool has = b < nb;
  long long si = (i0 + (has ? b : 0)) % n;
  float x[MLP_IN], t[MLP_OUT];
#pragma unroll
  for (int c = 0; c < MLP_IN; c++) x[c] = samples[si * SAMPLE + c];
#pragma unroll
  for (int c = 0; c < MLP_OUT; c++) t[c] = samples[si * SAMPLE + MLP_IN + c];
  float* rec = scr ? scr + (size_t)(has ? b : 0) * SCR : nullptr;
  float* h1 = rec ? rec + HDR : nullptr;
  float* h2 = rec ? rec + HDR + MLP_H : nullptr;
  float* dh1 = rec ? rec + HDR + 2 * MLP_H : nullptr;
  float* dh2 = rec ? rec + HDR + 3 * MLP_H : nullptr;
  float y[MLP_OUT];
  // all lanes run the wavefront forward; lanes without a sample write to a
  // dummy row that is never read (slot 0 is overwritten by its owner below)
  __shared__ float s_dummy[2 * MLP_H * 4];
  float* h1o = !scr ? nullptr : (has ? h1 : s_dummy + (threadIdx.x >> 6) * 2 * MLP_H);
  float* h2o = !scr ? nullptr : (has ? h2 : s_dummy + (threadIdx.x >> 6) * 2 * MLP_H + MLP_H);
  mlp_wave_forward(W, x, y, S[threadIdx.x >> 6], h1o, h2o);
  if (y_out && has) {
#pragma unroll
    for (int c = 0; c < MLP_OUT; c++) y_out[(size_t)b * MLP_OUT + c] = y[c];
  }
  double loss = 0.0;
  if (has && rec) {
    // normalised error of the trace-projected output y; the adjoint of the
    // network's normalised output yn goes back through the projection
    // y = P(yn * std + mean), P(u) = u + (tr x - sum u) / 3
    float g[MLP_OUT], dy[MLP_OUT], gs = 0.f;
#pragma unroll
    for (int c = 0; c < MLP_OUT; c++) {
      const float yn = (y[c] - W.out_mean[c]) / W.out_std[c];
      const float tn = (t[c] - W.out_mean[c]) / W.out_std[c];
      const float e = yn - tn;
      loss += (double)e * e;
      g[c] = 2.f * e / (float)(MLP_OUT * nb) / W.out_std[c];   // dL/dy
      gs += g[c];
    }
#pragma unroll
    for (int c = 0; c < MLP_OUT; c++) dy[c] = (g[c] - gs * (1.f / 3.f)) * W.out_std[c];
#pragma unroll
    for (int c = 0; c < MLP_IN; c++) rec[c] = (x[c] - W.in_mean[c]) / W.in_std[c];
    // dh2 = W3^T dy masked by ReLU; dh1 = W2^T dh2 masked by ReLU (BF16 weights)
    float g2[MLP_H];
#pragma unroll
    for (int k = 0; k < MLP_H; k++) {
      float s = 0.f;
#pragma unroll
      for (int c = 0; c < MLP_OUT; c++) s += bf2f(W.W3[c * MLP_H + k]) * dy[c];
      g2[k] = h2[k] > 0.f ? s : 0.f;
      dh2[k] = g2[k];
    }
    for (int j = 0; j < MLP_H; j++) {
      float s = 0.f;
#pragma unroll
      for (int i = 0; i < MLP_H; i++) s += bf2f(W.W2[i * MLP_H + j]) * g2[i];
      dh1[j] = h1[j] > 0.f ? s : 0.f;
    }
#pragma unroll
    for (int c = 0; c < MLP_OUT; c++) rec[MLP_IN + c] = dy[c];
  }
  for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off);
  if ((threadIdx.x & 63) == 0 && misc) atomicAdd(misc, loss / (double)(MLP_OUT * nb));
}

// Weight gradients: each thread owns one parameter and sums its term over a
// slice of the batch; slices are combined with atomic adds into grad.
__global__ __launch_bounds__(256) void k_mlp_wgrad(const float* __restrict__ scr, int nb, int slices, float* __restrict__ grad) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= MLP_NPARAM) return;
  const int sl = blockIdx.y;
  const int b0 = (int)((long long)nb * sl / slices), b1 = (int)((long long)nb * (sl + 1) / slices);
  float acc = 0.f;
  // decode the parameter
  int kind, i = 0, j = 0;
  if (p < OFF_B1) { kind = 0; i = p / MLP_IN; j = p % MLP_IN; }
  else if (p < OFF_W2) { kind = 1; i = p - OFF_B1; }
  else if (p < OFF_B2) { kind = 2; i = (p - OFF_W2) / MLP_H; j = (p - OFF_W2) % MLP_H; }
  else if (p < OFF_W3) { kind = 3; i = p - OFF_B2; }
  else if (p < OFF_B3) { kind = 4; i = (p - OFF_W3) / MLP_H; j = (p - OFF_W3) % MLP_H; }
  else { kind = 5; i = p - OFF_B3; }
  for (int b = b0; b < b1; b++) {
    const float* r = scr + (size_t)b * SCR;
    switch (kind) {
      case 0: acc += r[HDR + 2 * MLP_H + i] * r[j]; break;              // dh1_i * xn_j
      case 1: acc += r[HDR + 2 * MLP_H + i]; break;
      case 2: acc += r[HDR + 3 * MLP_H + i] * r[HDR + j]; break;        // dh2_i * h1_j
      case 3: acc += r[HDR + 3 * MLP_H + i]; break;
      case 4: acc += r[MLP_IN + i] * r[HDR + MLP_H + j]; break;         // dy_i * h2_j
      default: acc += r[MLP_IN + i]; break;
    }
  }
  atomicAdd(grad + p, acc);
}

// Adam (Kingma and Ba 2015) on the FP32 master weights; clears the gradient.
__global__ void k_mlp_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v, float* __restrict__ g,
                           float lr, float b1, float b2, float eps, float c1, float c2) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MLP_NPARAM) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  g[i] = 0.f;
}

// Per-sample backward scratch of mpm_mlp_grad_noalloc: at most
// MPM_MLP_NOALLOC_MAX_BATCH samples of SCR floats (2.2 MB), one copy per
// device for the life of the process.  Host code never passes this name to
// a kernel: it uses the address hipGetSymbolAddress returns for the device.
static __device__ __align__(256) float scratch[MPM_MLP_NOALLOC_MAX_BATCH * SCR];

}  // namespace mpm

using namespace mpm;

static int hipok(hipError_t e) { return e == hipSuccess ? MPM_OK : MPM_EHIP; }

// Device address of `scratch` on device dev, looked up once per device (with
// that device current: the caller's) and kept.
static void* noalloc_scratch(int dev) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* ptr[kMaxDevices] = {};
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(mpm::scratch)) != hipSuccess || !p) return nullptr;
    ptr[dev] = p;
  }
  return ptr[dev];
}

extern "C" {

size_t mpm_mlp_state_bytes(void) { return mlp_layout().total; }

size_t mpm_mlp_scratch_bytes(int32_t batch) {
  if (batch < 1) return 0;
  return al((size_t)batch * SCR * sizeof(float));
}

int mpm_mlp_init(void* state_dev, const float* samples_dev, int64_t n, const float* init_params, uint64_t seed,
                 void* stream) {
  if (!state_dev || !samples_dev || n < 2) return MPM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  MlpLayout L = mlp_layout();
  char* st = (char*)state_dev;
  std::vector<float> p(MLP_NPARAM, 0.f);
  if (init_params) {
    memcpy(p.data(), init_params, sizeof(float) * MLP_NPARAM);
  } else {
    // He-uniform initialisation, zero biases
    std::mt19937_64 rng(seed);
    auto fill = [&](int off, int fan_in, int count) {
      float lim = sqrtf(6.f / fan_in);
      std::uniform_real_distribution<float> u(-lim, lim);
      for (int q = 0; q < count; q++) p[off + q] = u(rng);
    };
    fill(OFF_W1, MLP_IN, MLP_H * MLP_IN);
    fill(OFF_W2, MLP_H, MLP_H * MLP_H);
    fill(OFF_W3, MLP_H, MLP_OUT * MLP_H);
  }
  int rc = MPM_OK;
  if (hipMemcpyAsync(st + L.params, p.data(), sizeof(float) * MLP_NPARAM, hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemsetAsync(st + L.m, 0, L.misc - L.m, s) != hipSuccess || hipMemsetAsync(st + L.misc, 0, 64, s) != hipSuccess ||
      hipMemsetAsync(st + L.blob, 0, sizeof(MlpBlob), s) != hipSuccess)
    rc = MPM_EHIP;
  if (rc == MPM_OK) {
    // the statistics need 18 doubles: accumulate in the (still zero) gradient block
    double* acc = (double*)(st + L.grad);
    k_mlp_stats<<<256, 256, 0, s>>>((const float*)samples_dev, n, acc);
    k_mlp_stats_final<<<1, 64, 0, s>>>(acc, n, (MlpBlob*)(st + L.blob));
    if (hipMemsetAsync(st + L.grad, 0, al(MLP_NPARAM * 4), s) != hipSuccess) rc = MPM_EHIP;
    k_mlp_publish<<<32, 256, 0, s>>>((const float*)(st + L.params), (MlpBlob*)(st + L.blob));
  }
  if (rc == MPM_OK) rc = hipok(hipStreamSynchronize(s));
  return rc;
}

// Gradient of the batch loss (samples i0 .. i0 + nb - 1) into the state's
// gradient block (added), the loss into misc[0] (added).
static void batch_grad(char* st, const float* samples, long long n, long long i0, int nb, float* scr, hipStream_t s) {
  MlpLayout L = mlp_layout();
  k_mlp_batch<<<(nb + 255) / 256, 256, 0, s>>>((const MlpBlob*)(st + L.blob), samples, n, i0, nb, scr,
                                              (double*)(st + L.misc), nullptr);
  dim3 grid((MLP_NPARAM + 255) / 256, 16);
  k_mlp_wgrad<<<grid, 256, 0, s>>>(scr, nb, 16, (float*)(st + L.grad));
}

// Loss and gradient of the first nb records with the per-sample scratch scr
// (shared by mpm_mlp_grad and mpm_mlp_grad_noalloc).
static int grad_impl(void* state_dev, const float* samples_dev, int64_t n, int nb, float* scr, float* grad_out_dev,
                     double* loss_out_host, hipStream_t s) {
  MlpLayout L = mlp_layout();
  char* st = (char*)state_dev;
  if (hipMemsetAsync(st + L.grad, 0, al(MLP_NPARAM * 4), s) != hipSuccess) return MPM_EHIP;
  if (hipMemsetAsync(st + L.misc, 0, 64, s) != hipSuccess) return MPM_EHIP;
  batch_grad(st, samples_dev, n, 0, nb, scr, s);
  if (hipMemcpyAsync(grad_out_dev, st + L.grad, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return MPM_EHIP;
  double loss = 0.0;
  if (hipMemcpyAsync(&loss, st + L.misc, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return MPM_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return MPM_EHIP;
  if (loss_out_host) *loss_out_host = loss;
  return hipok(hipMemsetAsync(st + L.grad, 0, al(MLP_NPARAM * 4), s));
}

int mpm_mlp_grad(void* state_dev, const float* samples_dev, int64_t n, int32_t batch, void* scratch_dev,
                 float* grad_out_dev, double* loss_out_host, void* stream) {
  if (!state_dev || !samples_dev || n < 1 || batch < 1 || !scratch_dev || !grad_out_dev) return MPM_EINVAL;
  const int nb = (int)(n < batch ? n : batch);
  return grad_impl(state_dev, samples_dev, n, nb, (float*)scratch_dev, grad_out_dev, loss_out_host, (hipStream_t)stream);
}

int mpm_mlp_grad_noalloc(void* state_dev, const float* samples_dev, int64_t n, int32_t batch, float* grad_out_dev,
                         double* loss_out_host, void* stream) {
  if (!state_dev || !samples_dev || n < 1 || batch < 1 || !grad_out_dev) return MPM_EINVAL;
  const int64_t nb = n < batch ? n : batch;
  if (nb > MPM_MLP_NOALLOC_MAX_BATCH) return MPM_EWORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return MPM_EHIP;
  float* scr = (float*)noalloc_scratch(dev);
  if (!scr) return MPM_EHIP;
  return grad_impl(state_dev, samples_dev, n, (int)nb, scr, grad_out_dev, loss_out_host, (hipStream_t)stream);
}

int mpm_mlp_train(void* state_dev, const float* samples_dev, int64_t n, int32_t batch, int32_t epochs, float lr,
                  uint64_t seed, void* scratch_dev, double* loss_hist_host, void* stream) {
  if (!state_dev || !samples_dev || n < 1 || batch < 1 || epochs < 1 || !scratch_dev || !(lr > 0.f)) return MPM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  MlpLayout L = mlp_layout();
  char* st = (char*)state_dev;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  double t_adam = 0.0;
  {
    double misc[8];
    if (hipMemcpyAsync(misc, st + L.misc, sizeof(misc), hipMemcpyDeviceToHost, s) != hipSuccess) return MPM_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return MPM_EHIP;
    t_adam = misc[1];
  }
  std::mt19937_64 rng(seed);
  const int nb = (int)(n < batch ? n : batch);
  const long long steps_per_epoch = (n + nb - 1) / nb;
  for (int ep = 0; ep < epochs; ep++) {
    if (hipMemsetAsync(st + L.misc, 0, sizeof(double), s) != hipSuccess) return MPM_EHIP;
    const long long offset = (long long)(rng() % (unsigned long long)n);
    for (long long k = 0; k < steps_per_epoch; k++) {
      batch_grad(st, samples_dev, n, (offset + k * nb) % n, nb, (float*)scratch_dev, s);
      t_adam += 1.0;
      float c1 = (float)(1.0 - pow((double)b1, t_adam)), c2 = (float)(1.0 - pow((double)b2, t_adam));
      k_mlp_adam<<<(MLP_NPARAM + 255) / 256, 256, 0, s>>>((float*)(st + L.params), (float*)(st + L.m), (float*)(st + L.v),
                                                          (float*)(st + L.grad), lr, b1, b2, eps, c1, c2);
      k_mlp_publish<<<32, 256, 0, s>>>((const float*)(st + L.params), (MlpBlob*)(st + L.blob));
    }
    double loss = 0.0;
    if (hipMemcpyAsync(&loss, st + L.misc, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return MPM_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return MPM_EHIP;
    if (loss_hist_host) loss_hist_host[ep] = loss / (double)steps_per_epoch;
  }
  double t_store[2] = {0.0, t_adam};
  if (hipMemcpyAsync(st + L.misc, t_store, sizeof(t_store), hipMemcpyHostToDevice, s) != hipSuccess) return MPM_EHIP;
  return hipok(hipStreamSynchronize(s));
}

int mpm_mlp_predict(const void* state_dev, const float* x_dev, int64_t n, float* y_dev, void* stream) {
  if (!state_dev || !x_dev || !y_dev || n < 1) return MPM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  MlpLayout L = mlp_layout();
  const char* st = (const char*)state_dev;
  // x_dev holds n samples of 6 inputs; run the batch kernel over them as
  // 9-float records is not possible, so rows are read with stride 6 via a
  // strided view: the batch kernel reads SAMPLE floats per sample, hence the
  // inputs are expected in 9-float records (targets ignored)
  for (long long i0 = 0; i0 < n; i0 += 1 << 20) {
    int nb = (int)((n - i0) < (1 << 20) ? (n - i0) : (1 << 20));
    k_mlp_batch<<<(nb + 255) / 256, 256, 0, s>>>((const MlpBlob*)(st + L.blob), x_dev + i0 * SAMPLE, nb, 0, nb, nullptr,
                                                nullptr, y_dev + i0 * MLP_OUT);
  }
  return hipok(hipStreamSynchronize(s));
}

int mpm_mlp_params(const void* state_dev, float* params_host, void* blob_host, void* stream) {
  if (!state_dev) return MPM_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  MlpLayout L = mlp_layout();
  const char* st = (const char*)state_dev;
  if (params_host && hipMemcpyAsync(params_host, st + L.params, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToHost, s) != hipSuccess)
    return MPM_EHIP;
  if (blob_host && hipMemcpyAsync(blob_host, st + L.blob, sizeof(MlpBlob), hipMemcpyDeviceToHost, s) != hipSuccess)
    return MPM_EHIP;
  return hipok(hipStreamSynchronize(s));
}

size_t mpm_mlp_blob_offset(void) { return mlp_layout().blob; }

}  // extern "C"
