// The spectral-scaling network: float32 inference, backpropagation and Adam.
//   x = (f - mean) / std (16) -> h1 = tanh(W1 x + b1) (64) -> h2 = tanh(W2 h1 + b2) (64)
//   -> y = W3 h2 + b3 (2);   loss = 1/n sum (y - t)^2
// Parameters packed as W1 (64x16 row-major), b1, W2 (64x64), b2, W3 (2x64), b3.
// Gradients are reduced through per-block partials in a fixed order (no float
// atomics), so training is bitwise reproducible.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "mlp.h"

namespace sm {

constexpr int kIn = 16, kH = 64, kOut = 2;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kOut * kH, kParams = oB3 + kOut;
static_assert(kParams == kMlpParams, "parameter count");

// ---- inference: one wavefront per sample (lane j = hidden unit j),
// parameters staged in LDS, kInferPerWave samples per wavefront in turn ----
constexpr int kInferPerWave = 1;

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__global__ __launch_bounds__(256) void mlp_infer_kernel(const float* __restrict__ theta,
                                                        const float* __restrict__ norm,
                                                        const float* __restrict__ X, int64_t ldx,
                                                        int64_t n, float* __restrict__ Y) {
  __shared__ float w[kParams + 2 * kIn];
  __shared__ float hs[4][kH];
  for (int k = threadIdx.x; k < kParams; k += blockDim.x) w[k] = theta[k];
  for (int k = threadIdx.x; k < 2 * kIn; k += blockDim.x) w[kParams + k] = norm[k];
  __syncthreads();
  const int j = threadIdx.x & (kWave - 1);
  const int wv = threadIdx.x / kWave;
  const int64_t first = ((int64_t)blockIdx.x * 4 + wv) * kInferPerWave;
  for (int q = 0; q < kInferPerWave; ++q) {
    const int64_t sidx = first + q;
    if (sidx >= n) break;   // uniform across the wavefront
    float z = w[oB1 + j];
#pragma unroll
    for (int i = 0; i < kIn; ++i)
      z += w[oW1 + j * kIn + i] * ((X[sidx * ldx + i] - w[kParams + i]) / w[kParams + kIn + i]);
    hs[wv][j] = tanhf(z);
    wave_sync();
    z = w[oB2 + j];
#pragma unroll 8
    for (int k = 0; k < kH; ++k) z += w[oW2 + j * kH + k] * hs[wv][k];
    const float h2 = tanhf(z);
    const float y0 = wave_sum_f(w[oW3 + j] * h2) + w[oB3];
    const float y1 = wave_sum_f(w[oW3 + kH + j] * h2) + w[oB3 + 1];
    if (j == 0) {
      Y[sidx * 2] = y0;
      Y[sidx * 2 + 1] = y1;
    }
    wave_sync();   // hs is rewritten for the next sample
  }
}

// ---- loss and gradient partials: 32 samples per block, activations in LDS ----
constexpr int kTS = 32;

__global__ __launch_bounds__(256) void mlp_grad_kernel(const float* __restrict__ theta,
                                                       const float* __restrict__ norm,
                                                       const float* __restrict__ X, int64_t ldx,
                                                       const float* __restrict__ T,
                                                       const int32_t* __restrict__ perm, int64_t b0,
                                                       int64_t nb, float inv_n,
                                                       float* __restrict__ part,
                                                       double* __restrict__ loss_part) {
  __shared__ float sx[kTS][kIn];
  __shared__ float sh1[kTS][kH + 1];
  __shared__ float sh2[kTS][kH + 1];
  __shared__ float sdz2[kTS][kH + 1];
  __shared__ float sdz1[kTS][kH + 1];
  __shared__ float sdy[kTS][kOut];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kTS;
  // inputs (samples beyond the batch contribute zero)
  for (int e = tid; e < kTS * kIn; e += blockDim.x) {
    const int s = e / kIn, i = e % kIn;
    const int64_t q = base + s;
    float v = 0.f;
    if (q < nb) {
      const int64_t src = perm ? perm[b0 + q] : b0 + q;
      v = (X[src * ldx + i] - norm[i]) / norm[kIn + i];
    }
    sx[s][i] = v;
  }
  __syncthreads();
  for (int e = tid; e < kTS * kH; e += blockDim.x) {
    const int s = e / kH, j = e % kH;
    float z = theta[oB1 + j];
    for (int i = 0; i < kIn; ++i) z += theta[oW1 + j * kIn + i] * sx[s][i];
    sh1[s][j] = tanhf(z);
  }
  __syncthreads();
  for (int e = tid; e < kTS * kH; e += blockDim.x) {
    const int s = e / kH, j = e % kH;
    float z = theta[oB2 + j];
    for (int k = 0; k < kH; ++k) z += theta[oW2 + j * kH + k] * sh1[s][k];
    sh2[s][j] = tanhf(z);
  }
  __syncthreads();
  double l = 0.0;
  if (tid < kTS * kOut) {
    const int s = tid / kOut, o = tid % kOut;
    const int64_t q = base + s;
    float dy = 0.f;
    if (q < nb) {
      const int64_t src = perm ? perm[b0 + q] : b0 + q;
      float y = theta[oB3 + o];
      for (int j = 0; j < kH; ++j) y += theta[oW3 + o * kH + j] * sh2[s][j];
      const float d = y - T[src * 2 + o];
      l = (double)d * (double)d;
      dy = 2.f * d * inv_n;
    }
    sdy[s][o] = dy;
  }
  l = wave_sum(l);
  if ((tid & 63) == 0) red[tid >> 6] = l;
  __syncthreads();
  for (int e = tid; e < kTS * kH; e += blockDim.x) {
    const int s = e / kH, j = e % kH;
    const float dh = sdy[s][0] * theta[oW3 + j] + sdy[s][1] * theta[oW3 + kH + j];
    sdz2[s][j] = dh * (1.f - sh2[s][j] * sh2[s][j]);
  }
  __syncthreads();
  for (int e = tid; e < kTS * kH; e += blockDim.x) {
    const int s = e / kH, k = e % kH;
    float dh = 0.f;
    for (int j = 0; j < kH; ++j) dh += sdz2[s][j] * theta[oW2 + j * kH + k];
    sdz1[s][k] = dh * (1.f - sh1[s][k] * sh1[s][k]);
  }
  __syncthreads();
  float* out = part + (int64_t)blockIdx.x * kParams;
  for (int pidx = tid; pidx < kParams; pidx += blockDim.x) {
    float g = 0.f;
    if (pidx < oB1) {
      const int k = (pidx - oW1) / kIn, i = (pidx - oW1) % kIn;
      for (int s = 0; s < kTS; ++s) g += sdz1[s][k] * sx[s][i];
    } else if (pidx < oW2) {
      const int k = pidx - oB1;
      for (int s = 0; s < kTS; ++s) g += sdz1[s][k];
    } else if (pidx < oB2) {
      const int j = (pidx - oW2) / kH, k = (pidx - oW2) % kH;
      for (int s = 0; s < kTS; ++s) g += sdz2[s][j] * sh1[s][k];
    } else if (pidx < oW3) {
      const int j = pidx - oB2;
      for (int s = 0; s < kTS; ++s) g += sdz2[s][j];
    } else if (pidx < oB3) {
      const int o = (pidx - oW3) / kH, j = (pidx - oW3) % kH;
      for (int s = 0; s < kTS; ++s) g += sdy[s][o] * sh2[s][j];
    } else {
      const int o = pidx - oB3;
      for (int s = 0; s < kTS; ++s) g += sdy[s][o];
    }
    out[pidx] = g;
  }
  if (tid == 0) loss_part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// sum of the block partials in block order
__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float* __restrict__ part, int nblk,
                                                         float* __restrict__ grad,
                                                         const double* __restrict__ loss_part,
                                                         double* __restrict__ loss_out) {
  const int pidx = blockIdx.x * blockDim.x + threadIdx.x;
  if (pidx < kParams) {
    float g = 0.f;
    for (int b = 0; b < nblk; ++b) g += part[(int64_t)b * kParams + pidx];
    grad[pidx] = g;
  }
  if (pidx == 0 && loss_out) {
    double l = 0.0;
    for (int b = 0; b < nblk; ++b) l += loss_part[b];
    *loss_out = l;
  }
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ theta, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, float lr,
                                                   float c1, float c2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= kParams) return;
  const float gk = g[k];
  const float mk = 0.9f * m[k] + 0.1f * gk;
  const float vk = 0.999f * v[k] + 0.001f * gk * gk;
  m[k] = mk;
  v[k] = vk;
  theta[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + 1e-8f);
}

hipError_t launch_mlp_infer(const float* theta, const float* norm, const float* X, int64_t ldx, int64_t n,
                            float* Y, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t per_block = 4 * kInferPerWave;
  hipLaunchKernelGGL(mlp_infer_kernel, dim3((unsigned)((n + per_block - 1) / per_block)), dim3(256), 0, s, theta,
                     norm, X, ldx, n, Y);
  return hipGetLastError();
}

int mlp_grad_blocks(int64_t nb) { return (int)((nb + kTS - 1) / kTS); }

hipError_t launch_mlp_grad(const float* theta, const float* norm, const float* X, int64_t ldx, const float* T,
                           const int32_t* perm, int64_t b0, int64_t nb, float inv_n, float* part,
                           double* loss_part, float* grad, double* loss_out, hipStream_t s) {
  const int nblk = mlp_grad_blocks(nb);
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(nblk), dim3(256), 0, s, theta, norm, X, ldx, T, perm, b0, nb,
                     inv_n, part, loss_part);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, part, nblk, grad,
                     loss_part, loss_out);
  return hipGetLastError();
}

hipError_t launch_adam(float* theta, const float* g, float* m, float* v, float lr, int step, hipStream_t s) {
  const float c1 = 1.f - powf(0.9f, (float)step);
  const float c2 = 1.f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, theta, g, m, v, lr, c1, c2);
  return hipGetLastError();
}

// Training pairs from the per-submatrix records of an explicit pass (power
// scale, plain Newton-Schulz): every record with both bounds found (rho_est
// > 0, lb_est > 0) gives x = its 16 features and t = (log(rho_est / c_G),
// log(lb_est c / c_G)), written in record order (one workgroup: a scan over
// tiles of 1024 records).  n_out[0] = number of pairs.
__global__ __launch_bounds__(1024) void scaling_pairs_kernel(const sm_sub_stats* __restrict__ st, int64_t n,
                                                             float* __restrict__ X, float* __restrict__ T,
                                                             int64_t* __restrict__ n_out) {
  __shared__ int wsum[16];
  __shared__ int64_t base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  for (int64_t t0 = 0; t0 < n; t0 += blockDim.x) {
    const int64_t i = t0 + threadIdx.x;
    const bool ok = i < n && st[i].rho_est > 0.0 && st[i].lb_est > 0.0 && st[i].gersh > 0.0;
    const unsigned long long bal = __ballot(ok);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wv] = __popcll(bal);
    __syncthreads();
    int off = 0;
    for (int w = 0; w < wv; ++w) off += wsum[w];
    if (ok) {
      const int64_t k = base + off + before;
      for (int f = 0; f < kIn; ++f) X[k * kIn + f] = st[i].feat[f];
      T[2 * k] = (float)log(st[i].rho_est / st[i].gersh);
      T[2 * k + 1] = (float)log(st[i].lb_est * st[i].scale / st[i].gersh);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < (int)(blockDim.x / kWave); ++w) tot += wsum[w];
      base += tot;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *n_out = base;
}

hipError_t launch_scaling_pairs(const sm_sub_stats* st, int64_t n, float* X, float* T, int64_t* n_out,
                                hipStream_t s) {
  hipLaunchKernelGGL(scaling_pairs_kernel, dim3(1), dim3(1024), 0, s, st, n, X, T, n_out);
  return hipGetLastError();
}

}  // namespace sm
