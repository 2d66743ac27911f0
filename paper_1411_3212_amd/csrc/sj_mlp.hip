// Cost model: an MLP 4 -> 64 -> 64 -> 1 (ReLU) with BF16 parameters and
// FP32 arithmetic, predicting the join time of a quadtree leaf (natural log
// of microseconds) from (log2(1 + objects), log2(1 + intersecting
// subqueries), level / 16, mean overlap of the subqueries with the leaf).
// Training keeps FP32 master parameters; the forward and backward passes use
// their BF16 rounding (round to nearest even) and the gradient with respect
// to the rounded values updates the masters (Adam).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "sj.h"
#include "sj_device.h"
#include "sj_mlp.h"
#include "sj_scene.h"

namespace sj {

__global__ void k_mlp_round(const float *master, uint16_t *w, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    w[i] = f2bf(master[i]);
}

// Forward pass, one sample per thread, parameters staged in LDS as FP32.
__global__ void __launch_bounds__(256) k_mlp_forward(const uint16_t *w, const float *x, uint32_t n,
                                                     float *y) {
  __shared__ float p[kMlpParams];
  for (int i = threadIdx.x; i < kMlpParams; i += 256) p[i] = bf2f(w[i]);
  __syncthreads();
  for (uint32_t s = blockIdx.x * 256 + threadIdx.x; s < n; s += gridDim.x * 256) {
    float xs[kF];
#pragma unroll
    for (int k = 0; k < kF; ++k) xs[k] = x[(uint64_t)s * kF + k];
    float h1[kH];
#pragma unroll
    for (int j = 0; j < kH; ++j) {
      float a = p[kOB1 + j];
#pragma unroll
      for (int k = 0; k < kF; ++k) a = fmaf(p[kOW1 + j * kF + k], xs[k], a);
      h1[j] = a > 0.0f ? a : 0.0f;
    }
    float out = p[kOB3];
    for (int i = 0; i < kH; ++i) {
      float a = p[kOB2 + i];
#pragma unroll
      for (int j = 0; j < kH; ++j) a = fmaf(p[kOW2 + i * kH + j], h1[j], a);
      out = fmaf(p[kOW3 + i], a > 0.0f ? a : 0.0f, out);
    }
    y[s] = out;
  }
}

// Loss L = (1/n) sum (y - t)^2 and its gradient.  One wave per block; the
// block takes tiles of 64 samples (one per lane) in a grid-stride loop:
// lanes run the forward and backward pass of their sample, the tile's
// hidden activations and deltas go to LDS, and lane j then accumulates row
// j of every weight gradient over the tile.  Each block writes its partial
// gradient (and loss sum) to partial[block]; k_mlp_reduce adds the blocks
// in order, so the result does not depend on scheduling.  LDS: BF16
// parameters (9 KB) and three 64 x 65 FP32 tiles reused across the two
// halves of the backward pass (51 KB), under the 64 KB of a workgroup.
__global__ void __launch_bounds__(64) k_mlp_grad(const uint16_t *w, const float *x, const float *t,
                                                 uint32_t n, float *partial) {
  __shared__ uint16_t pw[kMlpParams + 1];
  __shared__ float sA[kH][kH + 1], sB[kH][kH + 1], sC[kH][kH + 1];
  __shared__ float sX[kH][kF], sDy[kH];
  const int lane = threadIdx.x;
  for (int i = lane; i < kMlpParams; i += 64) pw[i] = w[i];
  __syncthreads();
  const float inv_n = 1.0f / (float)(n ? n : 1);
  float gW2[kH], gW1[kF], gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, loss = 0.f;
#pragma unroll
  for (int c = 0; c < kH; ++c) gW2[c] = 0.f;
#pragma unroll
  for (int k = 0; k < kF; ++k) gW1[k] = 0.f;
  const int j = lane;  // the hidden unit whose gradient rows this lane sums
  const uint32_t ntile = (n + 63) / 64;
  for (uint32_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const uint32_t s = tile * 64 + lane;
    const bool valid = s < n;
    __syncthreads();  // the previous tile's LDS reads are done
    // forward: row `lane` of the tiles holds this lane's sample
    float xs[kF];
#pragma unroll
    for (int k = 0; k < kF; ++k) xs[k] = valid ? x[(uint64_t)s * kF + k] : 0.0f;
    float h1[kH];
#pragma unroll
    for (int i = 0; i < kH; ++i) {
      float a = bf2f(pw[kOB1 + i]);
#pragma unroll
      for (int k = 0; k < kF; ++k) a = fmaf(bf2f(pw[kOW1 + i * kF + k]), xs[k], a);
      h1[i] = a > 0.0f ? a : 0.0f;
      sA[lane][i] = h1[i];
    }
    float y = bf2f(pw[kOB3]);
    for (int i = 0; i < kH; ++i) {
      float a = bf2f(pw[kOB2 + i]);
#pragma unroll
      for (int c = 0; c < kH; ++c) a = fmaf(bf2f(pw[kOW2 + i * kH + c]), h1[c], a);
      const float h2 = a > 0.0f ? a : 0.0f;
      y = fmaf(bf2f(pw[kOW3 + i]), h2, y);
      sB[lane][i] = h2;
    }
    const float r = valid ? y - t[s] : 0.0f;
    loss = fmaf(r, r, loss);
    const float dy = 2.0f * r * inv_n;
    for (int i = 0; i < kH; ++i)  // delta2 = dy w3 where h2 > 0
      sC[lane][i] = sB[lane][i] > 0.0f ? dy * bf2f(pw[kOW3 + i]) : 0.0f;
#pragma unroll
    for (int k = 0; k < kF; ++k) sX[lane][k] = xs[k];
    sDy[lane] = dy;
    __syncthreads();
    // first half: gradients of W2, b2, w3, b3 (tiles h1, h2, delta2)
    for (int q = 0; q < 64; ++q) {
      const float g2j = sC[q][j];
#pragma unroll
      for (int c = 0; c < kH; ++c) gW2[c] = fmaf(g2j, sA[q][c], gW2[c]);
      gb2 += g2j;
      gw3 = fmaf(sDy[q], sB[q][j], gw3);
      gb3 += (j == 0) ? sDy[q] : 0.0f;
    }
    __syncthreads();  // h2 tile consumed: it now takes delta1
    {
      float g2[kH];
#pragma unroll
      for (int i = 0; i < kH; ++i) g2[i] = sC[lane][i];
      for (int c = 0; c < kH; ++c) {
        float a = 0.0f;
#pragma unroll
        for (int i = 0; i < kH; ++i) a = fmaf(bf2f(pw[kOW2 + i * kH + c]), g2[i], a);
        sB[lane][c] = sA[lane][c] > 0.0f ? a : 0.0f;
      }
    }
    __syncthreads();
    // second half: gradients of W1, b1 (tiles x, delta1)
    for (int q = 0; q < 64; ++q) {
      const float g1j = sB[q][j];
#pragma unroll
      for (int k = 0; k < kF; ++k) gW1[k] = fmaf(g1j, sX[q][k], gW1[k]);
      gb1 += g1j;
    }
  }
  float *out = partial + (uint64_t)blockIdx.x * (kMlpParams + 1);
#pragma unroll
  for (int c = 0; c < kH; ++c) out[kOW2 + j * kH + c] = gW2[c];
#pragma unroll
  for (int k = 0; k < kF; ++k) out[kOW1 + j * kF + k] = gW1[k];
  out[kOB1 + j] = gb1;
  out[kOB2 + j] = gb2;
  out[kOW3 + j] = gw3;
  if (j == 0) out[kOB3] = gb3;
  loss = wave_sum(loss);
  if (j == 0) out[kMlpParams] = loss * inv_n;
}

__global__ void k_mlp_reduce(const float *partial, uint32_t nblocks, float *grad) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i <= (uint32_t)kMlpParams;
       i += gridDim.x * blockDim.x) {
    float a = 0.0f;
    for (uint32_t b = 0; b < nblocks; ++b) a += partial[(uint64_t)b * (kMlpParams + 1) + i];
    grad[i] = a;
  }
}

__global__ void k_mlp_adam(float *master, const float *grad, float *m, float *v, uint16_t *w,
                           uint32_t n, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float g = grad[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    const float wi = master[i] - lr * mh / (sqrtf(vh) + eps);
    master[i] = wi;
    w[i] = f2bf(wi);
  }
}

constexpr uint32_t kGradBlocks = 256;

// Per-block partial gradients of sj_mlp_grad_noalloc: a fixed array in the
// library's device memory (one copy per GPU, held until the process ends),
// for callers that cannot allocate.  Every block writes its whole partial
// on every call, so nothing has to start at zero.  Host code reaches it
// only through the address hipGetSymbolAddress returns for the device.
constexpr size_t kGradScratchFloats = (size_t)kGradBlocks * (kMlpParams + 1);
static __device__ __align__(256) float scratch[kGradScratchFloats];

}  // namespace sj

using namespace sj;

namespace {

// Device address of `scratch` on each GPU, looked up on the first call made
// with that GPU current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

int scratch_address(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    sj_set_global_error("sj_mlp_grad_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    return SJ_EDEVICE;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    sj_set_global_error("sj_mlp_grad_noalloc: device %d above the supported %d", dev,
                        kMaxDevices);
    return SJ_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(sj::scratch));
    if (e != hipSuccess || !p) {
      sj_set_global_error("sj_mlp_grad_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
      return SJ_EDEVICE;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return SJ_OK;
}

// Status of the launches since the matching launch_begin(): errors that
// earlier calls of other code left pending are cleared first, so a failure
// reported here is one of these launches.
void launch_begin() { (void)hipGetLastError(); }

int launch_end(const char *what) {
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) return SJ_OK;
  sj_set_global_error("%s: %s (%s)", what, hipGetErrorName(e), hipGetErrorString(e));
  return SJ_EDEVICE;
}

}  // namespace

extern "C" {

uint32_t sj_mlp_param_count(void) { return (uint32_t)kMlpParams; }

size_t sj_mlp_scratch_bytes(uint32_t n) {
  (void)n;
  return (size_t)kGradBlocks * (kMlpParams + 1) * sizeof(float);
}

int sj_mlp_round(const float *d_master, uint16_t *d_w, hipStream_t s) {
  if (!d_master || !d_w) return SJ_EINVAL;
  launch_begin();
  hipLaunchKernelGGL(k_mlp_round, dim3(18), dim3(256), 0, s, d_master, d_w, (uint32_t)kMlpParams);
  return launch_end("sj_mlp_round");
}

int sj_mlp_forward(const uint16_t *d_w, const float *d_x, uint32_t n, float *d_y, hipStream_t s) {
  if (!d_w || (n && (!d_x || !d_y))) return SJ_EINVAL;
  if (!n) return SJ_OK;
  const unsigned g = (unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
  launch_begin();
  hipLaunchKernelGGL(k_mlp_forward, dim3(g), dim3(256), 0, s, d_w, d_x, n, d_y);
  return launch_end("sj_mlp_forward");
}

int sj_mlp_grad(const uint16_t *d_w, const float *d_x, const float *d_t, uint32_t n,
                float *d_grad, void *d_scratch, size_t scratch_bytes, hipStream_t s) {
  if (!d_w || !d_grad || !d_scratch || (n && (!d_x || !d_t))) return SJ_EINVAL;
  if (scratch_bytes < sj_mlp_scratch_bytes(n)) return SJ_ENOSPACE;
  float *partial = (float *)d_scratch;
  launch_begin();
  hipLaunchKernelGGL(k_mlp_grad, dim3(kGradBlocks), dim3(64), 0, s, d_w, d_x, d_t, n, partial);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(18), dim3(256), 0, s, (const float *)partial, kGradBlocks,
                     d_grad);
  return launch_end("sj_mlp_grad");
}

size_t sj_mlp_noalloc_scratch_bytes(void) { return kGradScratchFloats * sizeof(float); }

int sj_mlp_grad_noalloc(const uint16_t *d_w, const float *d_x, const float *d_t, uint32_t n,
                        float *d_grad, hipStream_t s) {
  if (!d_w || !d_grad || (n && (!d_x || !d_t))) return SJ_EINVAL;
  // the partials are per block (kGradBlocks of them whatever n is), so
  // every n fits the fixed array
  void *p = nullptr;
  const int rc = scratch_address(&p);
  if (rc != SJ_OK) return rc;
  float *partial = (float *)p;
  launch_begin();
  hipLaunchKernelGGL(k_mlp_grad, dim3(kGradBlocks), dim3(64), 0, s, d_w, d_x, d_t, n, partial);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(18), dim3(256), 0, s, (const float *)partial, kGradBlocks,
                     d_grad);
  return launch_end("sj_mlp_grad_noalloc");
}

int sj_mlp_adam(float *d_master, const float *d_grad, float *d_m, float *d_v, uint16_t *d_w,
                uint32_t step, float lr, hipStream_t s) {
  if (!d_master || !d_grad || !d_m || !d_v || !d_w || step == 0) return SJ_EINVAL;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  launch_begin();
  hipLaunchKernelGGL(k_mlp_adam, dim3(18), dim3(256), 0, s, d_master, d_grad, d_m, d_v, d_w,
                     (uint32_t)kMlpParams, lr, b1, b2, eps, c1, c2);
  return launch_end("sj_mlp_adam");
}

}  // extern "C"
