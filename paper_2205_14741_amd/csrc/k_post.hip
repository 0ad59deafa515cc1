// After the sign iteration: float64 probe check of sign(T)^2 = I, step 3 of
// the submatrix method (Fig. 2 of the paper: insert block i's columns into P),
// and the float64 reductions tr(PH), tr P of Eq. 14's density matrix.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device_common.h"
#include "row_map.h"
#include "smsign_internal.h"

namespace sm {

template <typename T>
__device__ __forceinline__ const T* final_x(const DevPlan& p, int g, const T* mats, const SubState* st,
                                             int l) {
  const int64_t np = p.npad_g[g];
  return mats + p.mat_off_g[g] + (int64_t)(st[l].iters & 1) * np * np;
}

// The last full iterate: the final X, or, where the last refinement update
// computed only the atom's own columns, the X it was computed from.
template <typename T>
__device__ __forceinline__ const T* full_x(const DevPlan& p, int g, const T* mats, const SubState* st, int l) {
  const int64_t np = p.npad_g[g];
  return mats + p.mat_off_g[g] + (int64_t)((st[l].iters - st[l].last_slab) & 1) * np * np;
}

// One workgroup per submatrix whose final X is not yet in float32 form in its
// buffer: the iteration ended in a low-precision main phase (no refinement
// step ran, status != 2), so X exists only as the 16-bit operand copies (hi +
// lo for split bf16), and / or no update ran at all, so the buffer holds T
// and X = x0s T.  Writes the float32 values the read-out kernels below use.
__global__ __launch_bounds__(256) void materialize_kernel(DevPlan p, int g0, float* __restrict__ mats,
                                                          const SubState* __restrict__ st, int kind,
                                                          int64_t shadow_off) {
  const int l = blockIdx.x;
  const SubState s = st[l];
  const bool from_copies = kind != 0 && s.status != 2;
  const bool x0 = s.iters == 0;
  if (!from_copies && !x0) return;
  const float sc = x0 ? (float)s.x0s : 1.0f;
  const int g = g0 + l;
  const int npad = p.npad_g[g];
  const int64_t nn = (int64_t)npad * npad;
  float* X = mats + p.mat_off_g[g] + (int64_t)(s.iters & 1) * nn;
  const uint16_t* h = reinterpret_cast<const uint16_t*>(X + shadow_off);
  const int lane = threadIdx.x & (kWave - 1);
  for (int c = threadIdx.x / kWave; c < npad; c += blockDim.x / kWave)
    for (int d = lane; d < npad; d += kWave) {
      float x;
      if (!from_copies) {
        x = X[(int64_t)c * npad + d];
      } else if (kind == SM_BF16X3) {
        const int64_t k = copy_idx<true>(c, d, npad);
        x = bf16_bits_to_f32(h[k]) + bf16_bits_to_f32(h[k + 32]);
      } else {
        x = copy_value(h[copy_idx<false>(c, d, npad)], kind);
      }
      X[(int64_t)c * npad + d] = x * sc;
    }
}

hipError_t launch_materialize(const DevPlan& p, int g0, int nsub, float* mats, const SubState* st,
                              int shadow_kind, int64_t shadow_off, hipStream_t s) {
  if (nsub <= 0) return hipSuccess;
  hipLaunchKernelGGL(materialize_kernel, dim3(nsub), dim3(256), 0, s, p, g0, mats, st, shadow_kind, shadow_off);
  return hipGetLastError();
}

// One workgroup per submatrix: copy the per-submatrix iteration record into
// `stats` and, with P > 0 probes, estimate max_v ||X (X v) - v|| / ||v|| in
// float64 for fixed +-1 vectors v (a residual of sign(T)^2 = I, Eq. 13):
// two block matrix-vector passes over X, every probe in the same pass.
template <typename T, int P>
__global__ __launch_bounds__(512) void finish_kernel(DevPlan p, int g0, const T* __restrict__ mats,
                                                     const SubState* __restrict__ st,
                                                     double* __restrict__ vecs,
                                                     sm_sub_stats* __restrict__ stats, int vec_lds) {
  constexpr int Q = P > 0 ? P : 1;
  __shared__ double red[matvec_red<Q, T>(8)];
  __shared__ double red2[8];
  extern __shared__ double fvec[];   // vec_lds: the probe vectors and X v in LDS
  const int l = blockIdx.x;
  const int g = g0 + l;
  const int i = p.order_g[g];
  const int npad = p.npad_g[g];
  const int n = p.height[i];
  const T* X = full_x(p, g, mats, st, l);
  double worst = -1.0;
  if constexpr (P > 0) {
    double* v = vec_lds ? fvec : vecs + p.vec_off_g[g];   // [P][npad]
    double* w = v + (int64_t)P * npad;                     // [P][npad] = X v
    for (int d = threadIdx.x; d < n; d += blockDim.x)
#pragma unroll
      for (int q = 0; q < P; ++q) v[q * npad + d] = probe_entry(q, d);
    __syncthreads();
    block_matvec<P>(X, npad, n, v, npad, red, [&](int q, int r, double y) { w[q * npad + r] = y; });
    double e[P];
#pragma unroll
    for (int q = 0; q < P; ++q) e[q] = 0.0;
    block_matvec<P>(X, npad, n, w, npad, red, [&](int q, int r, double y) {
      const double t = y - v[q * npad + r];
      e[q] += t * t;
    });
    worst = 0.0;
#pragma unroll
    for (int q = 0; q < P; ++q) worst = fmax(worst, sqrt(block_reduce<0>(e[q], red2) / (double)n));
  }
  if (threadIdx.x == 0) {
    const SubState s = st[l];
    sm_sub_stats& r = stats[i];
    r.iters = s.iters;
    r.iters_low = s.iters_low;
    r.status = s.status;
    r.retried = s.retried;
    r.top1 = (float)s.top1;
    r.res = s.res;
    r.lb_est = s.lb_est;
    r.res_probe = worst;   // -1 without probes
    r.res_comm = -1.0;     // set by the commutator probe when it runs
  }
}

template <typename T>
static hipError_t launch_finish_t(const DevPlan& p, int g0, int nsub, const T* mats, const SubState* st,
                                  int probes, double* vecs, sm_sub_stats* stats, int max_npad, hipStream_t s) {
  // probe vectors and X v in LDS while they take at most 16 KiB (lattice
  // submatrices), else in the workspace
  const size_t vb = (size_t)2 * probes * max_npad * sizeof(double);
  const size_t lds = vb <= 16 * 1024 ? vb : 0;
#define SM_FINISH(PR)                                                                                 \
  case PR:                                                                                            \
    hipLaunchKernelGGL((finish_kernel<T, PR>), dim3(nsub), dim3(512), lds, s, p, g0, mats, st, vecs, stats, \
                       lds ? 1 : 0);                                                                  \
    break;
  switch (probes) {
    SM_FINISH(0) SM_FINISH(1) SM_FINISH(2) SM_FINISH(3) SM_FINISH(4) SM_FINISH(5) SM_FINISH(6)
    SM_FINISH(7) SM_FINISH(8)
    default: return hipErrorInvalidValue;
  }
#undef SM_FINISH
  return hipGetLastError();
}

hipError_t launch_finish(const DevPlan& p, int g0, int nsub, const void* mats, int storage_f64,
                         const SubState* st, int probes, double* vecs, sm_sub_stats* stats, int max_npad,
                         hipStream_t s) {
  static_assert(kMaxProbes == 8, "finish kernels are instantiated for 0..8 probes");
  if (nsub <= 0) return hipSuccess;
  if (storage_f64)
    return launch_finish_t(p, g0, nsub, (const double*)mats, st, probes, vecs, stats, max_npad, s);
  return launch_finish_t(p, g0, nsub, (const float*)mats, st, probes, vecs, stats, max_npad, s);
}

// y_q = T w_q (q < Q) for T = H[idx_i, idx_i] - mu I read straight from H's
// panels: the block's waves take the atoms j of I_i in turn, build the row
// map of block column j (row_map.h) and, for each of its columns c, form the
// dot product of column c of T with w_q (lanes over rows, float64); T is
// symmetric, so that is entry c of T w_q.  out(q, c, y) is called by lane 0 of
// the wave that owns column c.  LDS: smem holds the atoms of I_i, their row
// offsets and one row map per wave (as the gather).
template <int Q, typename Out>
__device__ __forceinline__ void t_matvec(const DevPlan& p, const double* __restrict__ H, double mu,
                                         const int* s_atom, const int* s_off, int m, int n, RowSrc* s_src,
                                         const double* __restrict__ w, int ws, Out out) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  for (int jj = wid; jj < m; jj += nw) {
    const int j = s_atom[jj];
    const int locj = s_off[jj];
    build_row_map(p, j, s_atom, s_off, m, n, s_src);
    const double* panel = H + p.panel_off[j];
    const int hj = p.height[j];
    for (int qc = 0; qc < p.bs[j]; ++qc) {
      const int c = locj + qc;
      const double* pc = panel + (int64_t)qc * hj;
      double dot[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) dot[q] = 0.0;
      for (int d = lane; d < n; d += kWave) {
        const int sr = s_src[d];
        double t = sr >= 0 ? pc[sr] : 0.0;
        if (d == c) t -= mu;
#pragma unroll
        for (int q = 0; q < Q; ++q) dot[q] += t * w[q * ws + d];
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const double y = wave_sum(dot[q]);
        if (lane == 0) out(q, c, y);
      }
    }
    wave_sync();   // the row map is rebuilt for the wave's next atom
  }
}

// One workgroup per submatrix: the commutator probe ||X (T v) - T (X v)|| /
// (c ||v||) for P fixed +-1 vectors (float64), X the last full iterate.
template <typename T, int P>
__global__ __launch_bounds__(256) void comm_probe_kernel(DevPlan p, int g0, const double* __restrict__ H,
                                                         double mu, const T* __restrict__ mats,
                                                         const SubState* __restrict__ st,
                                                         double* __restrict__ vecs,
                                                         sm_sub_stats* __restrict__ stats) {
  extern __shared__ int smem[];
  __shared__ double red[matvec_red<P, T>(4)];
  __shared__ double red2[8];
  const int l = blockIdx.x;
  const int g = g0 + l;
  const int i = p.order_g[g];
  const int npad = p.npad_g[g];
  const int n = p.height[i];
  const int64_t k0 = p.col_ptr[i];
  const int m = (int)(p.col_ptr[i + 1] - k0);
  int* s_atom = smem;
  int* s_off = smem + m;
  RowSrc* s_src = reinterpret_cast<RowSrc*>(smem + 2 * m) + (threadIdx.x / kWave) * npad;
  for (int t = threadIdx.x; t < m; t += blockDim.x) {
    s_atom[t] = p.row_idx[k0 + t];
    s_off[t] = p.blk_rowoff[k0 + t];
  }
  const T* X = full_x(p, g, mats, st, l);
  double* v = vecs + p.vec_off_g[g];   // [P][npad] probes
  double* a = v + P * npad;            // X v
  double* b = a + P * npad;            // T v
  double* c = b + P * npad;            // X (T v)
  for (int d = threadIdx.x; d < n; d += blockDim.x)
#pragma unroll
    for (int q = 0; q < P; ++q) v[q * npad + d] = probe_entry(100 + q, d);
  __syncthreads();
  block_matvec<P>(X, npad, n, v, npad, red, [&](int q, int r, double y) { a[q * npad + r] = y; });
  t_matvec<P>(p, H, mu, s_atom, s_off, m, n, s_src, v, npad, [&](int q, int r, double y) { b[q * npad + r] = y; });
  __syncthreads();
  block_matvec<P>(X, npad, n, b, npad, red, [&](int q, int r, double y) { c[q * npad + r] = y; });
  double e[P];
#pragma unroll
  for (int q = 0; q < P; ++q) e[q] = 0.0;
  t_matvec<P>(p, H, mu, s_atom, s_off, m, n, s_src, a, npad, [&](int q, int r, double y) {
    const double t = c[q * npad + r] - y;
    e[q] += t * t;
  });
  __syncthreads();
  double worst = 0.0;
#pragma unroll
  for (int q = 0; q < P; ++q) worst = fmax(worst, sqrt(block_reduce<0>(e[q], red2) / (double)n));
  if (threadIdx.x == 0) stats[i].res_comm = worst / stats[i].scale;
}

template <typename T>
static hipError_t launch_comm_t(const DevPlan& p, int g0, int nsub, int max_m, int max_npad, const double* H,
                                double mu, const T* mats, const SubState* st, int probes, double* vecs,
                                sm_sub_stats* stats, hipStream_t s) {
  const size_t lds = row_maps_bytes(max_m, 4, max_npad);
  switch (probes) {
    case 1: hipLaunchKernelGGL((comm_probe_kernel<T, 1>), dim3(nsub), dim3(256), lds, s, p, g0, H, mu, mats, st, vecs, stats); break;
    case 2: hipLaunchKernelGGL((comm_probe_kernel<T, 2>), dim3(nsub), dim3(256), lds, s, p, g0, H, mu, mats, st, vecs, stats); break;
    case 3: hipLaunchKernelGGL((comm_probe_kernel<T, 3>), dim3(nsub), dim3(256), lds, s, p, g0, H, mu, mats, st, vecs, stats); break;
    case 4: hipLaunchKernelGGL((comm_probe_kernel<T, 4>), dim3(nsub), dim3(256), lds, s, p, g0, H, mu, mats, st, vecs, stats); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_comm_probe(const DevPlan& p, int g0, int nsub, int max_m, int max_npad, const double* H,
                             double mu, const void* mats, int storage_f64, const SubState* st, int probes,
                             double* vecs, sm_sub_stats* stats, hipStream_t s) {
  static_assert(4 * 4 <= 2 * kMaxProbes, "probe vectors fit the per-submatrix vector space");
  if (nsub <= 0) return hipSuccess;
  if (storage_f64)
    return launch_comm_t(p, g0, nsub, max_m, max_npad, H, mu, (const double*)mats, st, probes, vecs, stats, s);
  return launch_comm_t(p, g0, nsub, max_m, max_npad, H, mu, (const float*)mats, st, probes, vecs, stats, s);
}

// Block column i of P = 1/2 (E - X[:, loc_i : loc_i + b_i]) over the n_i rows of
// submatrix i; P's panel of column i has exactly those rows in that order, so
// this is a contiguous, coalesced copy with one writer per block column.
template <typename T>
__global__ __launch_bounds__(256) void scatter_kernel(DevPlan p, int g0, const T* __restrict__ mats,
                                                      const SubState* __restrict__ st,
                                                      double* __restrict__ P) {
  const int l = blockIdx.x;
  const int g = g0 + l;
  const int i = p.order_g[g];
  const int npad = p.npad_g[g];
  const int n = p.height[i];
  const int loc = p.loc[i];
  const int b = p.bs[i];
  const T* X = final_x(p, g, mats, st, l);
  double* out = P + p.panel_off[i];
  const int total = n * b;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    const int q = e / n;
    const int r = e - q * n;
    const double x = (double)X[(int64_t)(loc + q) * npad + r];
    out[e] = 0.5 * ((r == loc + q ? 1.0 : 0.0) - x);
  }
}

hipError_t launch_scatter(const DevPlan& p, int g0, int nsub, const void* mats, int storage_f64,
                          const SubState* st, double* P, hipStream_t s) {
  if (nsub <= 0) return hipSuccess;
  if (storage_f64)
    hipLaunchKernelGGL(scatter_kernel<double>, dim3(nsub), dim3(256), 0, s, p, g0,
                       (const double*)mats, st, P);
  else
    hipLaunchKernelGGL(scatter_kernel<float>, dim3(nsub), dim3(256), 0, s, p, g0,
                       (const float*)mats, st, P);
  return hipGetLastError();
}

// tr(PH) = sum of P .* H over the common stored pattern (H symmetric) and
// tr P = sum of P's diagonal; block b reduces a fixed contiguous range, the
// final kernel adds the block partials in block order: bitwise reproducible.
__global__ __launch_bounds__(256) void trace_partial_kernel(const double* __restrict__ H,
                                                            const double* __restrict__ P, int64_t nvals,
                                                            const int64_t* __restrict__ diag,
                                                            int64_t ndiag, double* __restrict__ parts) {
  __shared__ double red[8];
  const int64_t per = (nvals + gridDim.x - 1) / gridDim.x;
  const int64_t a = blockIdx.x * per;
  const int64_t e = a + per < nvals ? a + per : nvals;
  double s = 0.0;
  for (int64_t k = a + threadIdx.x; k < e; k += blockDim.x) s += P[k] * H[k];
  s = block_reduce<0>(s, red);
  const int64_t perd = (ndiag + gridDim.x - 1) / gridDim.x;
  const int64_t ad = blockIdx.x * perd;
  const int64_t ed = ad + perd < ndiag ? ad + perd : ndiag;
  double t = 0.0;
  for (int64_t k = ad + threadIdx.x; k < ed; k += blockDim.x) t += P[diag[k]];
  t = block_reduce<0>(t, red);
  if (threadIdx.x == 0) {
    parts[blockIdx.x] = s;
    parts[gridDim.x + blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(256) void trace_final_kernel(const double* __restrict__ parts, int nb,
                                                          double* __restrict__ out) {
  __shared__ double red[8];
  double s = 0.0, t = 0.0;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    s += parts[k];
    t += parts[nb + k];
  }
  s = block_reduce<0>(s, red);
  t = block_reduce<0>(t, red);
  if (threadIdx.x == 0) {
    out[0] = s;
    out[1] = t;
  }
}

hipError_t launch_trace(const double* H, const double* P, int64_t nvals, const int64_t* diag_idx,
                        int64_t ndiag, double* partials, int nblocks, double* out2, hipStream_t s) {
  hipLaunchKernelGGL(trace_partial_kernel, dim3(nblocks), dim3(256), 0, s, H, P, nvals, diag_idx,
                     ndiag, partials);
  hipLaunchKernelGGL(trace_final_kernel, dim3(1), dim3(256), 0, s, partials, nblocks, out2);
  return hipGetLastError();
}

// Electron count of submatrix i: trace of P_ii = 1/2 (I - X_ii) read from X.
template <typename T>
__global__ void ne_kernel(DevPlan p, int g0, int nsub, const T* __restrict__ mats,
                          const SubState* __restrict__ st, double* __restrict__ ne) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nsub) return;
  const int g = g0 + l;
  const int i = p.order_g[g];
  const int npad = p.npad_g[g];
  const int loc = p.loc[i];
  const int b = p.bs[i];
  const T* X = final_x(p, g, mats, st, l);
  double s = 0.0;
  for (int q = 0; q < b; ++q) s += 0.5 * (1.0 - (double)X[(int64_t)(loc + q) * npad + loc + q]);
  ne[i] = s;
}

hipError_t launch_ne_from_x(const DevPlan& p, int g0, int nsub, const void* mats, int storage_f64,
                            const SubState* st, double* ne_parts, hipStream_t s) {
  if (nsub <= 0) return hipSuccess;
  const int grid = (nsub + 255) / 256;
  if (storage_f64)
    hipLaunchKernelGGL(ne_kernel<double>, dim3(grid), dim3(256), 0, s, p, g0, nsub,
                       (const double*)mats, st, ne_parts);
  else
    hipLaunchKernelGGL(ne_kernel<float>, dim3(grid), dim3(256), 0, s, p, g0, nsub,
                       (const float*)mats, st, ne_parts);
  return hipGetLastError();
}

// Global Gershgorin discs of H, one workgroup per block column c: for every
// orbital column q, [h_qq - R_q, h_qq + R_q] with R_q the off-diagonal abs sum
// (column sums equal row sums since H is symmetric).  Writes min / max per c.
__global__ __launch_bounds__(256) void gersh_kernel(DevPlan p, const double* __restrict__ H,
                                                    double* __restrict__ out) {
  __shared__ double red[8];
  const int c = blockIdx.x;
  const int h = p.height[c];
  const int b = p.bs[c];
  const int loc = p.loc[c];
  const double* panel = H + p.panel_off[c];
  double lo = 1e300, hi = -1e300;
  for (int q = 0; q < b; ++q) {
    double s = 0.0;
    for (int d = threadIdx.x; d < h; d += blockDim.x) s += fabs(panel[(int64_t)q * h + d]);
    s = block_reduce<0>(s, red);
    const double dg = panel[(int64_t)q * h + loc + q];
    const double R = s - fabs(dg);
    lo = fmin(lo, dg - R);
    hi = fmax(hi, dg + R);
  }
  if (threadIdx.x == 0) {
    out[2 * c] = lo;
    out[2 * c + 1] = hi;
  }
}

// Smallest lower and largest upper Gershgorin end over the atoms (order-free).
__global__ __launch_bounds__(256) void gersh_final_kernel(const double* __restrict__ lohi, int n_atoms,
                                                          double* __restrict__ out2) {
  __shared__ double red[8];
  double lo = 1e300, hi = -1e300;
  for (int c = threadIdx.x; c < n_atoms; c += blockDim.x) {
    lo = fmin(lo, lohi[2 * c]);
    hi = fmax(hi, lohi[2 * c + 1]);
  }
  lo = block_reduce<2>(lo, red);
  hi = block_reduce<1>(hi, red);
  if (threadIdx.x == 0) {
    out2[0] = lo;
    out2[1] = hi;
  }
}

hipError_t launch_gersh_rows(const DevPlan& p, int n_atoms, const double* H, double* lohi_parts,
                             double* out2, hipStream_t s) {
  hipLaunchKernelGGL(gersh_kernel, dim3(n_atoms), dim3(256), 0, s, p, H, lohi_parts);
  hipLaunchKernelGGL(gersh_final_kernel, dim3(1), dim3(256), 0, s, lohi_parts, n_atoms, out2);
  return hipGetLastError();
}

// Fixed scratch of the allocation-free bracket (sm_gershgorin_bracket_noalloc):
// the per-atom intervals of at most kNoAllocMaxAtoms atoms (8 MiB).  Every GPU
// the library runs on holds its own copy of the array until the process ends.
// In host code `scratch` names a host-side stand-in, not the device array:
// the device address comes from hipGetSymbolAddress, once per device, and is
// the only form in which host code passes the array on.
static __device__ __align__(256) double scratch[2 * kNoAllocMaxAtoms];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};
}  // namespace

// Device address of `scratch` on the current device (looked up on the first
// call on that device, then kept).
static hipError_t noalloc_scratch(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    double* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_dev[dev] = ptr;
  }
  *out = g_scratch_dev[dev];
  return hipSuccess;
}

hipError_t launch_gersh_rows_noalloc(const DevPlan& p, int n_atoms, const double* H, double* out2,
                                     hipStream_t s) {
  if (n_atoms < 1 || n_atoms > kNoAllocMaxAtoms) return hipErrorInvalidValue;
  double* lohi = nullptr;
  const hipError_t e = noalloc_scratch(&lohi);
  if (e != hipSuccess) return e;
  // the kernels write every one of the 2 n_atoms entries before reading it:
  // nothing of an earlier call's contents is used
  return launch_gersh_rows(p, n_atoms, H, lohi, out2, s);
}

// Electron count sum_i ne_i in a fixed order with compensation (Neumaier):
// each thread sums a contiguous run of atoms, thread 0 combines the runs in
// order.  out[0] = the sum (written by one thread: out may be host-mapped).
__device__ __forceinline__ void neumaier_add(double& sum, double& comp, double x) {
  const double t = sum + x;
  comp += fabs(sum) >= fabs(x) ? (sum - t) + x : (x - t) + sum;
  sum = t;
}

__global__ __launch_bounds__(256) void ne_sum_kernel(const double* __restrict__ ne_sub, int n_atoms,
                                                     double* __restrict__ out) {
  __shared__ double ps[256], pc[256];
  const int per = (n_atoms + blockDim.x - 1) / blockDim.x;
  const int a0 = threadIdx.x * per, a1 = min(n_atoms, a0 + per);
  double sum = 0.0, comp = 0.0;
  for (int a = a0; a < a1; ++a) neumaier_add(sum, comp, ne_sub[a]);
  ps[threadIdx.x] = sum;
  pc[threadIdx.x] = comp;
  __syncthreads();
  if (threadIdx.x == 0) {
    double S = 0.0, Cc = 0.0;
    for (int k = 0; k < (int)blockDim.x; ++k) {
      neumaier_add(S, Cc, ps[k]);
      Cc += pc[k];
    }
    out[0] = S + Cc;
  }
}

hipError_t launch_ne_sum(const double* ne_sub, int n_atoms, double* out, hipStream_t s) {
  hipLaunchKernelGGL(ne_sum_kernel, dim3(1), dim3(256), 0, s, ne_sub, n_atoms, out);
  return hipGetLastError();
}

}  // namespace sm
