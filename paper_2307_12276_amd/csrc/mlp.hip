// Learned spectral-interval predictor: field statistics and a 9-64-64-64-3
// tanh MLP in FP32 with hand-written forward, backward and Adam kernels.
//
// Packed parameters: for each layer l, W_l [in][out] row-major then b_l[out].
// Activation cache per row: X (9) | H1 (64) | H2 (64) | H3 (64).
//
// These networks are tiny (9155 parameters) and latency-bound: the forward
// kernel gives each sample one wave64 (one lane per hidden unit, activations
// in LDS); the backward kernel runs in a single block and walks the batch in
// chunks so that every parameter gradient is a fixed-order sum over samples
// (bitwise reproducible, no atomics).
#include "bounds.h"

namespace adl {

constexpr int kIn = 9, kH = 64, kOut = 3;
constexpr int oW1 = 0, oB1 = oW1 + kIn * kH;
constexpr int oW2 = oB1 + kH, oB2 = oW2 + kH * kH;
constexpr int oW3 = oB2 + kH, oB3 = oW3 + kH * kH;
constexpr int oW4 = oB3 + kH, oB4 = oW4 + kH * kOut;
constexpr int kParams = oB4 + kOut;
static_assert(kParams == 9155, "parameter count");
constexpr int kCache = kIn + 3 * kH;  // 201

// ---------------------------------------------------------------------------
// forward: one wave per sample
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ W, const float* __restrict__ X,
                                                          float* __restrict__ Y, float* __restrict__ cache, int B) {
  __shared__ float act[4][kH];
  __shared__ float xin[4][kIn];
  const int w = threadIdx.x >> 6, t = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + w;
  const bool valid = b < B;
  if (valid && t < kIn) {
    const float v = X[(long)b * kIn + t];
    xin[w][t] = v;
    if (cache) cache[(long)b * kCache + t] = v;
  }
  __syncthreads();
  // layer 1
  float z = W[oB1 + t];
  for (int i = 0; i < kIn; ++i) z += xin[w][i] * W[oW1 + i * kH + t];
  float h = tanhf(z);
  if (valid && cache) cache[(long)b * kCache + kIn + t] = h;
  act[w][t] = h;
  __syncthreads();
  // layers 2 and 3
  for (int layer = 0; layer < 2; ++layer) {
    const int oW = layer == 0 ? oW2 : oW3, oB = layer == 0 ? oB2 : oB3;
    z = W[oB + t];
    for (int k = 0; k < kH; ++k) z += act[w][k] * W[oW + k * kH + t];
    h = tanhf(z);
    __syncthreads();
    act[w][t] = h;
    if (valid && cache) cache[(long)b * kCache + kIn + (layer + 1) * kH + t] = h;
    __syncthreads();
  }
  // output layer (linear)
  if (valid && t < kOut) {
    float y = W[oB4 + t];
    for (int k = 0; k < kH; ++k) y += act[w][k] * W[oW4 + k * kOut + t];
    Y[(long)b * kOut + t] = y;
  }
}

// ---------------------------------------------------------------------------
// backward: single block, batch walked in chunks of kChunk samples.
//   G4 = dY;  G3 = (G4 W4^T) (1 - H3^2);  G2 = (G3 W3^T)(1 - H2^2);  G1 = ...
//   dW_l[i][o] = sum_b Hin_l[b][i] G_l[b][o],   db_l[o] = sum_b G_l[b][o]
// ---------------------------------------------------------------------------
constexpr int kChunk = 32;
constexpr int kBwdThreads = 1024;
constexpr int kPerThread = (kParams + kBwdThreads - 1) / kBwdThreads;  // 9

__global__ __launch_bounds__(kBwdThreads) void mlp_backward_kernel(const float* __restrict__ W,
                                                                   const float* __restrict__ cache,
                                                                   const float* __restrict__ dY,
                                                                   float* __restrict__ dW, int B) {
  __shared__ float G4[kChunk][kOut];
  __shared__ float G3[kChunk][kH];
  __shared__ float G2[kChunk][kH];
  __shared__ float G1[kChunk][kH];
  __shared__ float Hc[kChunk][kCache];
  const int tid = threadIdx.x;
  float acc[kPerThread];
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) acc[q] = 0.0f;

  for (int b0 = 0; b0 < B; b0 += kChunk) {
    const int nb = min(kChunk, B - b0);
    __syncthreads();
    for (int e = tid; e < nb * kCache; e += kBwdThreads) Hc[e / kCache][e % kCache] = cache[(long)b0 * kCache + e];
    for (int e = tid; e < nb * kOut; e += kBwdThreads) G4[e / kOut][e % kOut] = dY[(long)b0 * kOut + e];
    __syncthreads();
    // G3: thread -> (sample, unit)
    for (int e = tid; e < nb * kH; e += kBwdThreads) {
      const int s = e / kH, k = e % kH;
      float g = 0.0f;
      for (int o = 0; o < kOut; ++o) g += G4[s][o] * W[oW4 + k * kOut + o];
      const float hv = Hc[s][kIn + 2 * kH + k];
      G3[s][k] = g * (1.0f - hv * hv);
    }
    __syncthreads();
    for (int e = tid; e < nb * kH; e += kBwdThreads) {
      const int s = e / kH, k = e % kH;
      float g = 0.0f;
      for (int o = 0; o < kH; ++o) g += G3[s][o] * W[oW3 + k * kH + o];
      const float hv = Hc[s][kIn + kH + k];
      G2[s][k] = g * (1.0f - hv * hv);
    }
    __syncthreads();
    for (int e = tid; e < nb * kH; e += kBwdThreads) {
      const int s = e / kH, k = e % kH;
      float g = 0.0f;
      for (int o = 0; o < kH; ++o) g += G2[s][o] * W[oW2 + k * kH + o];
      const float hv = Hc[s][kIn + k];
      G1[s][k] = g * (1.0f - hv * hv);
    }
    __syncthreads();
    // accumulate parameter gradients, samples in order
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
      const int idx = tid + q * kBwdThreads;
      if (idx >= kParams) continue;
      float a = acc[q];
      if (idx < oB1) {
        const int i = (idx - oW1) / kH, o = (idx - oW1) % kH;
        for (int s = 0; s < nb; ++s) a += Hc[s][i] * G1[s][o];
      } else if (idx < oW2) {
        const int o = idx - oB1;
        for (int s = 0; s < nb; ++s) a += G1[s][o];
      } else if (idx < oB2) {
        const int i = (idx - oW2) / kH, o = (idx - oW2) % kH;
        for (int s = 0; s < nb; ++s) a += Hc[s][kIn + i] * G2[s][o];
      } else if (idx < oW3) {
        const int o = idx - oB2;
        for (int s = 0; s < nb; ++s) a += G2[s][o];
      } else if (idx < oB3) {
        const int i = (idx - oW3) / kH, o = (idx - oW3) % kH;
        for (int s = 0; s < nb; ++s) a += Hc[s][kIn + kH + i] * G3[s][o];
      } else if (idx < oW4) {
        const int o = idx - oB3;
        for (int s = 0; s < nb; ++s) a += G3[s][o];
      } else if (idx < oB4) {
        const int i = (idx - oW4) / kOut, o = (idx - oW4) % kOut;
        for (int s = 0; s < nb; ++s) a += Hc[s][kIn + 2 * kH + i] * G4[s][o];
      } else {
        const int o = idx - oB4;
        for (int s = 0; s < nb; ++s) a += G4[s][o];
      }
      acc[q] = a;
    }
  }
#pragma unroll
  for (int q = 0; q < kPerThread; ++q) {
    const int idx = tid + q * kBwdThreads;
    if (idx < kParams) dW[idx] = acc[q];
  }
}

// Mean squared error L = mean((Y - T)^2) over B x 3 and dL/dY = 2 (Y - T) / (3 B);
// one block, fixed-order sum.
__global__ __launch_bounds__(256) void mlp_mse_grad_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                                           float* __restrict__ dY, float* __restrict__ loss, int B) {
  __shared__ float sh[256];
  const int n = B * kOut;
  const float sc = 2.0f / (float)n;
  float acc = 0.0f;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const float d = Y[i] - T[i];
    dY[i] = sc * d;
    acc += d * d;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) loss[0] = sh[0] / (float)n;
}

// Adam (Kingma & Ba 2015): bias corrections bc1 = 1 - b1^t, bc2 = 1 - b2^t.
__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ W, const float* __restrict__ dW,
                                                       float* __restrict__ m1, float* __restrict__ m2, float lr,
                                                       float b1, float b2, float eps, float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kParams) return;
  const float g = dW[i];
  const float m = b1 * m1[i] + (1.0f - b1) * g;
  const float v = b2 * m2[i] + (1.0f - b2) * g * g;
  m1[i] = m;
  m2[i] = v;
  const float mh = m / bc1, vh = v / bc2;
  W[i] = W[i] - lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------------------------
// field statistics: per-node eigenvalues of [[Dxx, Dxy], [Dxy, Dyy]] and |a|
// ---------------------------------------------------------------------------
template <typename TF, bool ADVF>
__global__ __launch_bounds__(kBlock) void field_stats_kernel(FieldView F, double hx, double hy, double dt,
                                                             float* __restrict__ feats, double* partials,
                                                             Ctl* ctl) {
  field_stats_blocks<TF, ADVF>(F, hx, hy, dt, feats, partials, ctl, (int)gridDim.x, (int)blockIdx.x);
}

hipError_t launch_field_stats(const FieldView& f, double hx, double hy, double dt, float* feats, double* partials,
                              Ctl* ctl, hipStream_t st) {
  const int nb = stats_blocks((long)f.nx * f.ny);
  const bool advf = f.ax != nullptr;
  if (f.f32) {
    if (advf)
      hipLaunchKernelGGL((field_stats_kernel<float, true>), dim3(nb), dim3(kBlock), 0, st, f, hx, hy, dt, feats, partials, ctl);
    else
      hipLaunchKernelGGL((field_stats_kernel<float, false>), dim3(nb), dim3(kBlock), 0, st, f, hx, hy, dt, feats, partials, ctl);
  } else {
    if (advf)
      hipLaunchKernelGGL((field_stats_kernel<double, true>), dim3(nb), dim3(kBlock), 0, st, f, hx, hy, dt, feats, partials, ctl);
    else
      hipLaunchKernelGGL((field_stats_kernel<double, false>), dim3(nb), dim3(kBlock), 0, st, f, hx, hy, dt, feats, partials, ctl);
  }
  return hipGetLastError();
}

// Batched statistics: every job's ctl[0] and ctl[1] cleared, one thread per job.
__global__ __launch_bounds__(kBlock) void bound_jobs_reset_kernel(const BoundJob* __restrict__ jobs, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    Ctl* c = jobs[i].ctl;
    const Ctl z{};
    c[0] = z;
    c[1] = z;
  }
}

// Block b finds its job (the one i with blk0[i] <= b < blk0[i + 1]; blk0 is
// strictly increasing from 0 and the grid has blk0[n] blocks, so exactly one
// thread finds it) and runs that job's statistics or Gershgorin block.
__global__ __launch_bounds__(kBlock) void bound_stats_many_kernel(const BoundJob* __restrict__ jobs,
                                                                  const int* __restrict__ blk0, int n, double dt,
                                                                  float* __restrict__ feats, double* gmin) {
  __shared__ int s_job;
  const int b = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    if (blk0[i] <= b && b < blk0[i + 1]) s_job = i;
  __syncthreads();
  const int i = s_job;
  const BoundJob J = jobs[i];
  const int lb = b - J.blk0;
  const bool advf = J.f.ax != nullptr;
  if (lb < J.nb_s) {
    float* fo = feats + 9L * i;
    if (J.f.f32) {
      if (advf) field_stats_blocks<float, true>(J.f, J.hx, J.hy, dt, fo, J.partials, J.ctl, J.nb_s, lb);
      else field_stats_blocks<float, false>(J.f, J.hx, J.hy, dt, fo, J.partials, J.ctl, J.nb_s, lb);
    } else {
      if (advf) field_stats_blocks<double, true>(J.f, J.hx, J.hy, dt, fo, J.partials, J.ctl, J.nb_s, lb);
      else field_stats_blocks<double, false>(J.f, J.hx, J.hy, dt, fo, J.partials, J.ctl, J.nb_s, lb);
    }
  } else {
    double* pg = J.partials + kGershPartials;
    const int gb = lb - J.nb_s;
    if (J.f.f32) {
      if (advf) gershgorin_blocks<float, true>(J.f, pg, J.ctl + 1, J.nb_g, gb, gmin + i);
      else gershgorin_blocks<float, false>(J.f, pg, J.ctl + 1, J.nb_g, gb, gmin + i);
    } else {
      if (advf) gershgorin_blocks<double, true>(J.f, pg, J.ctl + 1, J.nb_g, gb, gmin + i);
      else gershgorin_blocks<double, false>(J.f, pg, J.ctl + 1, J.nb_g, gb, gmin + i);
    }
  }
}

hipError_t launch_bound_stats_many(const BoundJob* jobs, const int* blk0, int n, int nblocks, double dt,
                                   float* feats, double* gmin, hipStream_t st) {
  if (n < 1 || nblocks < n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(bound_jobs_reset_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, st, jobs, n);
  hipLaunchKernelGGL(bound_stats_many_kernel, dim3(nblocks), dim3(kBlock), 0, st, jobs, blk0, n, dt, feats, gmin);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* W, const float* X, float* Y, float* cache, int B, hipStream_t st) {
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((B + 3) / 4), dim3(256), 0, st, W, X, Y, cache, B);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const float* W, const float* cache, const float* dY, float* dW, int B, hipStream_t st) {
  hipLaunchKernelGGL(mlp_backward_kernel, dim3(1), dim3(kBwdThreads), 0, st, W, cache, dY, dW, B);
  return hipGetLastError();
}

hipError_t launch_mlp_mse_grad(const float* Y, const float* T, float* dY, float* loss, int B, hipStream_t st) {
  hipLaunchKernelGGL(mlp_mse_grad_kernel, dim3(1), dim3(256), 0, st, Y, T, dY, loss, B);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* W, const float* dW, float* m1, float* m2, int t, float lr, float b1, float b2,
                           float eps, hipStream_t st) {
  const double bc1 = 1.0 - pow((double)b1, (double)t), bc2 = 1.0 - pow((double)b2, (double)t);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, st, W, dW, m1, m2, lr, b1, b2, eps,
                     (float)bc1, (float)bc2);
  return hipGetLastError();
}

}  // namespace adl
