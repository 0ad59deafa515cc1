// Internal: the scaling network object and its kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/smsign.h"

namespace sm {

constexpr int kMlpParams = 16 * 64 + 64 + 64 * 64 + 64 + 2 * 64 + 2;   // 5378

hipError_t launch_mlp_infer(const float* theta, const float* norm, const float* X, int64_t ldx, int64_t n,
                            float* Y, hipStream_t s);
int mlp_grad_blocks(int64_t nb);
hipError_t launch_mlp_grad(const float* theta, const float* norm, const float* X, int64_t ldx, const float* T,
                           const int32_t* perm, int64_t b0, int64_t nb, float inv_n, float* part,
                           double* loss_part, float* grad, double* loss_out, hipStream_t s);
hipError_t launch_adam(float* theta, const float* g, float* m, float* v, float lr, int step, hipStream_t s);
hipError_t launch_scaling_pairs(const sm_sub_stats* st, int64_t n, float* X, float* T, int64_t* n_out,
                                hipStream_t s);

}  // namespace sm

struct sm_mlp {
  int device = -1;
  float* theta = nullptr;   // [kMlpParams]
  float* norm = nullptr;    // [32] feature mean, std
  float* m = nullptr;       // Adam moments
  float* v = nullptr;
  float* grad = nullptr;
  float* part = nullptr;    // per-block gradient partials
  double* loss = nullptr;   // [1 + partial blocks]
  int64_t part_blocks = 0;
  int32_t* perm = nullptr;  // sample permutation of the current epoch
  int64_t perm_n = 0;
  int64_t adam_step = 0;
};
