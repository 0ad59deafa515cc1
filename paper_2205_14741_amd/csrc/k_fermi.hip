// Finite-temperature occupation of every submatrix: the matrix function of
// Fig. 2 taken as the Fermi-Dirac function f(x) = 1 / (1 + exp(beta x)) of
// T_i = H[idx_i, idx_i] - mu I, in float64.
//
// f is never formed from eigenvalues.  With x = beta T_i and z = x / 2^(m+1)
// small (|z| <= 1/4 by a Gershgorin bound), f(x / 2^m) = 1/2 (1 - tanh z) comes
// from the Taylor polynomial of tanh to z^15; then m doublings of the argument
// use f(2y) = f(y)^2 / (f(y)^2 + (1 - f(y))^2), which holds because
// exp(2y) = exp(y)^2.  The denominator D = I - 2F(I - F) has its spectrum in
// [1/2, 1], so D^-1 = 4/3 (I - R)^-1 with R = I - 4/3 D, |R| <= 1/3, is the
// product (I + R)(I + R^2)(I + R^4)(I + R^8)(I + R^16) to 3^-32.  Every
// matrix is a polynomial or rational function of T_i: symmetric, and all of
// them commute, so every product is a lower-triangle product mirrored (the
// float64 tile kernel of k_ovl.hip, kind 0).  This file holds the
// elementwise and per-submatrix kernels around those products.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "ovl_internal.h"

namespace sm {

__device__ __forceinline__ double* fd_buf(const DevPlan& p, double* mats, int g, int b) {
  const int64_t np = p.npad_g[g];
  return mats + p.mat_off_g[g] + (int64_t)b * np * np;
}

// out[l] = beta * max(c_G, c) for submatrix l of the chunk: a bound on |x| over
// the spectrum of x = beta T_i (c_G bounds T_i) and over the identity pad of
// X_0 = T_i / c (which stands for the eigenvalue c of T_i).
__global__ void fd_bound_kernel(DevPlan p, int g0, int nsub, const sm_sub_stats* __restrict__ stats, double beta,
                                double* __restrict__ out) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nsub) return;
  const sm_sub_stats& st = stats[p.order_g[g0 + l]];
  out[l] = beta * fmax(st.gersh, st.scale);
}

// s[l] = beta c / 2^(m+1) (z = s X_0) and s2[l] = s^2.
__global__ void fd_coef_kernel(DevPlan p, int g0, int nsub, const sm_sub_stats* __restrict__ stats, double beta,
                               double inv2m1, double* __restrict__ s, double* __restrict__ s2) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nsub) return;
  const double v = beta * stats[p.order_g[g0 + l]].scale * inv2m1;
  s[l] = v;
  s2[l] = v * v;
}

// Buffer cb = a * buffer xb + b * buffer yb + d I over the whole padded
// submatrix (xb or yb < 0: that term is absent; cb may equal xb or yb).
__global__ __launch_bounds__(256) void fd_lincomb_kernel(DevPlan p, int g0, double* mats, int xb, double a, int yb,
                                                         double b, double d, int cb) {
  const int g = g0 + blockIdx.x;
  const int npad = p.npad_g[g];
  const double* X = xb >= 0 ? fd_buf(p, mats, g, xb) : nullptr;
  const double* Y = yb >= 0 ? fd_buf(p, mats, g, yb) : nullptr;
  double* C = fd_buf(p, mats, g, cb);
  const int64_t nn = (int64_t)npad * npad;
  for (int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.y * blockDim.x) {
    const int c = (int)(e / npad), r = (int)(e - (int64_t)c * npad);
    double v = r == c ? d : 0.0;
    if (X) v += a * X[e];
    if (Y) v += b * Y[e];
    C[e] = v;
  }
}

// Electron count of atom i = order_g[g] and its mu-derivative from F = f(T_i)
// (buffer fb): ne[i] = sum_q F_qq and dne[i] = beta sum_q (F_qq - sum_r F_rq^2)
// over the atom's own columns q (f' = -beta f (1 - f), F symmetric, rows r
// of the valid block only).  One workgroup per submatrix, one wave per column
// in turn, partial sums reduced in a fixed order.
__global__ __launch_bounds__(256) void fd_count_kernel(DevPlan p, int g0, const double* mats, int fb, double beta,
                                                       double* __restrict__ ne, double* __restrict__ dne) {
  __shared__ double rd[4], rn[4];
  const int g = g0 + blockIdx.x;
  const int i = p.order_g[g];
  const int npad = p.npad_g[g];
  const int n = p.height[i];
  const int loc = p.loc[i], b = p.bs[i];
  const double* F = fd_buf(p, const_cast<double*>(mats), g, fb);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double sd = 0.0, sn = 0.0;
  for (int q = wid; q < b; q += 4) {
    const double* col = F + (int64_t)(loc + q) * npad;
    double ss = 0.0;
    for (int r = lane; r < n; r += 64) ss += col[r] * col[r];
    ss = wave_sum(ss);
    const double fqq = col[loc + q];
    sn += fqq;
    sd += fqq - ss;
  }
  if (lane == 0) {
    rd[wid] = sd;
    rn[wid] = sn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    ne[i] = (rn[0] + rn[1]) + (rn[2] + rn[3]);
    dne[i] = beta * ((rd[0] + rd[1]) + (rd[2] + rd[3]));
  }
}

static int fd_spread(int64_t work) {
  return (int)std::min<int64_t>(64, std::max<int64_t>(1, work / (256 * 64)));
}

hipError_t launch_fd_bound(const DevPlan& p, int g0, int nsub, const sm_sub_stats* stats, double beta, double* out,
                           hipStream_t s) {
  hipLaunchKernelGGL(fd_bound_kernel, dim3((nsub + 255) / 256), dim3(256), 0, s, p, g0, nsub, stats, beta, out);
  return hipGetLastError();
}

hipError_t launch_fd_coef(const DevPlan& p, int g0, int nsub, const sm_sub_stats* stats, double beta, double inv2m1,
                          double* sv, double* s2, hipStream_t s) {
  hipLaunchKernelGGL(fd_coef_kernel, dim3((nsub + 255) / 256), dim3(256), 0, s, p, g0, nsub, stats, beta, inv2m1,
                     sv, s2);
  return hipGetLastError();
}

hipError_t launch_fd_lincomb(const DevPlan& p, int g0, int nsub, int max_npad, double* mats, int xb, double a, int yb,
                             double b, double d, int cb, hipStream_t s) {
  hipLaunchKernelGGL(fd_lincomb_kernel, dim3(nsub, fd_spread((int64_t)max_npad * max_npad)), dim3(256), 0, s, p, g0,
                     mats, xb, a, yb, b, d, cb);
  return hipGetLastError();
}

hipError_t launch_fd_count(const DevPlan& p, int g0, int nsub, const double* mats, int fb, double beta, double* ne,
                           double* dne, hipStream_t s) {
  hipLaunchKernelGGL(fd_count_kernel, dim3(nsub), dim3(256), 0, s, p, g0, mats, fb, beta, ne, dne);
  return hipGetLastError();
}

}  // namespace sm
