// C ABI of the spectral-scaling network: creation, weights, inference,
// loss / gradient, Adam training loop.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "plan.h"

using namespace sm;

namespace {

uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform01(uint64_t& s) { return (double)(splitmix64(s) >> 11) * 0x1.0p-53; }

int mlp_ensure_parts(sm_mlp* m, int64_t blocks) {
  if (blocks <= m->part_blocks) return SM_OK;
  if (m->part) (void)hipFree(m->part);
  if (m->loss) (void)hipFree(m->loss);
  m->part = nullptr;
  m->loss = nullptr;
  SM_HIP(hipMalloc(&m->part, (size_t)blocks * kMlpParams * sizeof(float)));
  SM_HIP(hipMalloc(&m->loss, (size_t)(blocks + 4096 + 8) * sizeof(double)));
  m->part_blocks = blocks;
  return SM_OK;
}

}  // namespace

extern "C" {

int sm_mlp_create(uint64_t seed, sm_mlp** out) {
  if (!out) return set_error(SM_ERR_ARG, "sm_mlp_create: null output");
  *out = nullptr;
  sm_mlp* m = new (std::nothrow) sm_mlp();
  if (!m) return set_error(SM_ERR_OOM, "sm_mlp_create: out of host memory");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipMalloc(&m->theta, kMlpParams * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->norm, 32 * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->m, kMlpParams * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->v, kMlpParams * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->grad, kMlpParams * sizeof(float));
  if (e != hipSuccess) {
    sm_mlp_destroy(m);
    return hip_error(e, "sm_mlp_create");
  }
  m->device = dev;
  // U(-1/sqrt(fan_in), 1/sqrt(fan_in)) in packing order from a SplitMix64 stream
  std::vector<float> th(kMlpParams);
  const int sizes[6] = {64 * 16, 64, 64 * 64, 64, 2 * 64, 2};
  const int fan[6] = {16, 16, 64, 64, 64, 64};
  uint64_t st = seed;
  int o = 0;
  for (int k = 0; k < 6; ++k) {
    const double a = 1.0 / std::sqrt((double)fan[k]);
    for (int j = 0; j < sizes[k]; ++j) th[o++] = (float)((2.0 * uniform01(st) - 1.0) * a);
  }
  std::vector<float> nm(32, 0.f);
  for (int k = 16; k < 32; ++k) nm[k] = 1.f;
  std::vector<float> z(kMlpParams, 0.f);
  e = hipMemcpy(m->theta, th.data(), kMlpParams * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->norm, nm.data(), 32 * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->m, z.data(), kMlpParams * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m->v, z.data(), kMlpParams * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    sm_mlp_destroy(m);
    return hip_error(e, "sm_mlp_create upload");
  }
  *out = m;
  return SM_OK;
}

void sm_mlp_destroy(sm_mlp* m) {
  if (!m) return;
  for (void* p : {(void*)m->theta, (void*)m->norm, (void*)m->m, (void*)m->v, (void*)m->grad,
                  (void*)m->part, (void*)m->loss, (void*)m->perm})
    if (p) (void)hipFree(p);
  delete m;
}

int sm_mlp_set_weights(sm_mlp* m, const float* params, const float* norm) {
  if (!m) return set_error(SM_ERR_ARG, "sm_mlp_set_weights: null network");
  if (params) {
    SM_HIP(hipMemcpy(m->theta, params, kMlpParams * 4, hipMemcpyHostToDevice));
    std::vector<float> z(kMlpParams, 0.f);
    SM_HIP(hipMemcpy(m->m, z.data(), kMlpParams * 4, hipMemcpyHostToDevice));
    SM_HIP(hipMemcpy(m->v, z.data(), kMlpParams * 4, hipMemcpyHostToDevice));
    m->adam_step = 0;
  }
  if (norm) {
    for (int k = 16; k < 32; ++k)
      if (!(norm[k] > 0.f)) return set_error(SM_ERR_ARG, "sm_mlp_set_weights: feature std must be > 0");
    SM_HIP(hipMemcpy(m->norm, norm, 32 * 4, hipMemcpyHostToDevice));
  }
  return SM_OK;
}

int sm_mlp_get_weights(const sm_mlp* m, float* params, float* norm) {
  if (!m) return set_error(SM_ERR_ARG, "sm_mlp_get_weights: null network");
  if (params) SM_HIP(hipMemcpy(params, m->theta, kMlpParams * 4, hipMemcpyDeviceToHost));
  if (norm) SM_HIP(hipMemcpy(norm, m->norm, 32 * 4, hipMemcpyDeviceToHost));
  return SM_OK;
}

int sm_mlp_infer(sm_mlp* m, const float* X, int64_t ldx, int64_t n, float* Y, void* stream) {
  if (!m || (!X && n > 0) || (!Y && n > 0)) return set_error(SM_ERR_ARG, "sm_mlp_infer: null argument");
  if (ldx < 16 || n < 0) return set_error(SM_ERR_ARG, "sm_mlp_infer: ldx must be >= 16 and n >= 0");
  SM_HIP(launch_mlp_infer(m->theta, m->norm, X, ldx, n, Y, reinterpret_cast<hipStream_t>(stream)));
  return SM_OK;
}

int sm_mlp_loss_grad(sm_mlp* m, const float* X, int64_t ldx, const float* T, int64_t n, double* loss,
                     float* grad_host, void* stream) {
  if (!m || !X || !T || n <= 0) return set_error(SM_ERR_ARG, "sm_mlp_loss_grad: bad argument");
  if (ldx < 16) return set_error(SM_ERR_ARG, "sm_mlp_loss_grad: ldx must be >= 16");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int rc;
  if ((rc = mlp_ensure_parts(m, mlp_grad_blocks(n)))) return rc;
  SM_HIP(launch_mlp_grad(m->theta, m->norm, X, ldx, T, nullptr, 0, n, 1.f / (float)n, m->part, m->loss + 1,
                         m->grad, m->loss, s));
  double l = 0.0;
  SM_HIP(hipMemcpyAsync(&l, m->loss, 8, hipMemcpyDeviceToHost, s));
  if (grad_host) SM_HIP(hipMemcpyAsync(grad_host, m->grad, kMlpParams * 4, hipMemcpyDeviceToHost, s));
  SM_HIP(hipStreamSynchronize(s));
  if (loss) *loss = l / (double)n;
  return SM_OK;
}

int sm_mlp_train(sm_mlp* m, const float* X, int64_t ldx, const float* T, int64_t n, int32_t epochs,
                 int32_t batch, float lr, int32_t fit_norm, uint64_t shuffle_seed, double* loss_hist,
                 void* stream) {
  if (!m || !X || !T || n <= 0) return set_error(SM_ERR_ARG, "sm_mlp_train: bad argument");
  if (ldx < 16 || epochs < 0 || batch <= 0 || !(lr > 0.f))
    return set_error(SM_ERR_ARG, "sm_mlp_train: ldx >= 16, epochs >= 0, batch > 0, lr > 0 required");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int rc;
  const int64_t bsz = std::min<int64_t>(batch, n);
  if ((rc = mlp_ensure_parts(m, mlp_grad_blocks(bsz)))) return rc;
  const int64_t nbatch = (n + bsz - 1) / bsz;
  if (nbatch > 4096) return set_error(SM_ERR_ARG, "sm_mlp_train: more than 4096 batches per epoch");
  if (fit_norm) {
    std::vector<float> h((size_t)(n - 1) * ldx + 16);
    SM_HIP(hipMemcpyAsync(h.data(), X, h.size() * 4, hipMemcpyDeviceToHost, s));
    SM_HIP(hipStreamSynchronize(s));
    float nm[32];
    for (int i = 0; i < 16; ++i) {
      double a = 0.0, b = 0.0;
      for (int64_t k = 0; k < n; ++k) {
        const double x = h[k * ldx + i];
        a += x;
        b += x * x;
      }
      const double mean = a / n;
      const double var = std::max(b / n - mean * mean, 0.0);
      nm[i] = (float)mean;
      nm[16 + i] = (float)std::max(std::sqrt(var), 1e-6);
    }
    SM_HIP(hipMemcpy(m->norm, nm, sizeof(nm), hipMemcpyHostToDevice));
  }
  if (m->perm_n < n) {
    if (m->perm) (void)hipFree(m->perm);
    m->perm = nullptr;
    SM_HIP(hipMalloc(&m->perm, (size_t)n * 4));
    m->perm_n = n;
  }
  std::vector<int32_t> perm((size_t)n);
  std::vector<double> bl((size_t)nbatch);
  double* batch_loss = m->loss + 1 + m->part_blocks;   // after the block partials
  uint64_t st = shuffle_seed;
  for (int ep = 0; ep < epochs; ++ep) {
    for (int64_t k = 0; k < n; ++k) perm[k] = (int32_t)k;
    if (shuffle_seed)
      for (int64_t k = n - 1; k > 0; --k) std::swap(perm[k], perm[splitmix64(st) % (uint64_t)(k + 1)]);
    SM_HIP(hipMemcpyAsync(m->perm, perm.data(), (size_t)n * 4, hipMemcpyHostToDevice, s));
    for (int64_t bi = 0; bi < nbatch; ++bi) {
      const int64_t b0 = bi * bsz;
      const int64_t nb = std::min(bsz, n - b0);
      SM_HIP(launch_mlp_grad(m->theta, m->norm, X, ldx, T, m->perm, b0, nb, 1.f / (float)nb, m->part,
                             m->loss + 1, m->grad, batch_loss + bi, s));
      SM_HIP(launch_adam(m->theta, m->grad, m->m, m->v, lr, (int)++m->adam_step, s));
    }
    SM_HIP(hipMemcpyAsync(bl.data(), batch_loss, (size_t)nbatch * 8, hipMemcpyDeviceToHost, s));
    SM_HIP(hipStreamSynchronize(s));   // also keeps the host permutation alive for the copy
    if (loss_hist) {
      double t = 0.0;
      for (double x : bl) t += x;
      loss_hist[ep] = t / (double)n;
    }
  }
  return SM_OK;
}

int sm_plan_set_mlp(sm_plan* p, sm_mlp* m) {
  if (!p) return set_error(SM_ERR_ARG, "sm_plan_set_mlp: null plan");
  p->mlp = m;
  return SM_OK;
}

int sm_scaling_pairs(const sm_sub_stats* stats, int64_t n, float* X, float* T, int64_t* n_pairs, void* stream) {
  if (!stats || !X || !T || !n_pairs) return set_error(SM_ERR_ARG, "sm_scaling_pairs: null argument");
  if (n < 0) return set_error(SM_ERR_ARG, "sm_scaling_pairs: n < 0");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  int64_t* d = nullptr;
  SM_HIP(hipMalloc(&d, sizeof(int64_t)));
  hipError_t e = launch_scaling_pairs(stats, n, X, T, d, s);
  if (e == hipSuccess) e = hipMemcpyAsync(n_pairs, d, sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(d);
  if (e != hipSuccess) return hip_error(e, "sm_scaling_pairs");
  return SM_OK;
}

}  // extern "C"
