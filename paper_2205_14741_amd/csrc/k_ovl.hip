// A non-orthogonal basis (S != I): Eq. 14 of the paper on the submatrix pair
// (T_i(H), T_i(S)) of every atom block i (Fig. 2), in float64.
//   Z_i = T_i(S)^(-1/2): Newton-Schulz on the block matrix [[0, A], [I, 0]],
//         A = T_i(S) / c_i, whose sign holds A^(1/2) and A^(-1/2) (Eq. 12).  The
//         iterate keeps the form [[0, Y], [Z, 0]], its square is
//         diag(Y Z, Z Y), so one step is W = 1/2 (3I - Z Y), Y <- Y W,
//         Z <- W Z (Y, Z, W are polynomials in A: symmetric, commuting).
//   K_i = Z_i T_i(H) Z_i - mu I, the start of the sign iteration (Eq. 14: the
//         sign of S^-1 H - mu I is Z^-1 sign(Z H Z - mu I) Z on the pair).
//   block column i of P_i = 1/2 Z_i (I - sign(K_i)) Z_i.
// The products run on 64 x 64 tiles of float64 matrix-core instructions,
// listed per (submatrix, tile row, tile column) by the host.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_common.h"
#include "ovl_internal.h"

namespace sm {

typedef double d4o __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double* buf_of(const DevPlan& p, double* mats, int g, int b) {
  const int64_t np = p.npad_g[g];
  return mats + p.mat_off_g[g] + (int64_t)b * np * np;
}

// Buffer b of every submatrix: zero, `dv` on the diagonal of the valid n x n
// block and `dp` on the diagonal of the pad.
__global__ __launch_bounds__(256) void ovl_fill_kernel(DevPlan p, int g0, double* mats, int b, double dv,
                                                       double dp) {
  const int g = g0 + blockIdx.x;
  const int npad = p.npad_g[g];
  const int n = p.height[p.order_g[g]];
  double* X = buf_of(p, mats, g, b);
  const int64_t nn = (int64_t)npad * npad;
  for (int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; e < nn; e += (int64_t)gridDim.y * blockDim.x) {
    const int c = (int)(e / npad), r = (int)(e - (int64_t)c * npad);
    X[e] = r == c ? (r < n ? dv : dp) : 0.0;
  }
}

// Position of atom a in the sorted row list [lo, hi) of a block column, or -1.
__device__ __forceinline__ int find_row(const int32_t* rows, int lo, int hi, int a) {
  while (lo < hi) {
    const int m = (lo + hi) >> 1;
    const int v = rows[m];
    if (v == a) return m;
    if (v < a) lo = m + 1; else hi = m;
  }
  return -1;
}

// T_i(V) (no shift) into buffer b: workgroup (l, j) copies the blocks of
// column atom I_i[j] whose row atoms are in I_i (the index set of i = the
// stored rows of block column i, in panel order), column by column from the
// panel of that atom.
__global__ __launch_bounds__(256) void ovl_gather_kernel(DevPlan p, int g0, const double* __restrict__ V,
                                                         double* mats, int b) {
  const int g = g0 + blockIdx.x;
  const int i = p.order_g[g];
  const int k0 = (int)p.col_ptr[i], k1 = (int)p.col_ptr[i + 1];
  const int j = blockIdx.y;
  if (j >= k1 - k0) return;
  const int npad = p.npad_g[g];
  double* T = buf_of(p, mats, g, b);
  const int cb_atom = p.row_idx[k0 + j];
  const int cb = p.blk_rowoff[k0 + j];          // column offset of that atom in T_i
  const int wb = p.bs[cb_atom];
  const int hb = p.height[cb_atom];
  const double* panel = V + p.panel_off[cb_atom];
  const int q0 = (int)p.col_ptr[cb_atom], q1 = (int)p.col_ptr[cb_atom + 1];
  for (int q = q0; q < q1; ++q) {
    const int ra_atom = p.row_idx[q];
    const int pos = find_row(p.row_idx, k0, k1, ra_atom);
    if (pos < 0) continue;                      // uniform over the workgroup
    const int ra = p.blk_rowoff[pos];           // row offset in T_i
    const int ro = p.blk_rowoff[q];             // row offset in the panel
    const int ba = p.bs[ra_atom];
    for (int e = threadIdx.x; e < ba * wb; e += blockDim.x) {
      const int cc = e / ba, rr = e - cc * ba;
      T[(int64_t)(cb + cc) * npad + ra + rr] = panel[(int64_t)cc * hb + ro + rr];
    }
  }
}

// Gershgorin bound of the valid block of buffer b (largest absolute column
// sum = row sum, symmetric) -> out[l]; with pad_one, the pad diagonal is set
// to 1 and stats.gersh to the bound.
__global__ __launch_bounds__(256) void ovl_gersh_kernel(DevPlan p, int g0, double* mats, int b, double* out,
                                                        int pad_one, sm_sub_stats* stats) {
  __shared__ double red[8];
  const int l = blockIdx.x;
  const int g = g0 + l;
  const int i = p.order_g[g];
  const int npad = p.npad_g[g];
  const int n = p.height[i];
  double* X = buf_of(p, mats, g, b);
  double mx = 0.0;
  for (int c = 0; c < n; ++c) {
    double s = 0.0;
    for (int r = threadIdx.x; r < n; r += blockDim.x) s += fabs(X[(int64_t)c * npad + r]);
    mx = fmax(mx, block_reduce<0>(s, red));
  }
  if (pad_one)
    for (int r = n + threadIdx.x; r < npad; r += blockDim.x) X[(int64_t)r * npad + r] = 1.0;
  if (threadIdx.x == 0) {
    out[l] = mx;
    if (pad_one) stats[i].gersh = mx;
  }
}

// Valid block of buffer b times f(l): mode 0 f = v[l], 1: 1 / v[l], 2: 1 / sqrt(v[l]).
__global__ __launch_bounds__(256) void ovl_scale_kernel(DevPlan p, int g0, double* mats, int b,
                                                        const double* __restrict__ v, int mode) {
  const int l = blockIdx.x;
  const int g = g0 + l;
  const int npad = p.npad_g[g];
  const int n = p.height[p.order_g[g]];
  const double f = mode == 0 ? v[l] : mode == 1 ? 1.0 / v[l] : 1.0 / sqrt(v[l]);
  double* X = buf_of(p, mats, g, b);
  for (int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; e < (int64_t)n * n;
       e += (int64_t)gridDim.y * blockDim.x) {
    const int c = (int)(e / n), r = (int)(e - (int64_t)c * n);
    X[(int64_t)c * npad + r] *= f;
  }
}

// Whole buffer copy src -> dst of every submatrix (within one workspace).
__global__ __launch_bounds__(256) void ovl_copy_kernel(DevPlan p, int g0, double* mats, int src, int dst) {
  const int g = g0 + blockIdx.x;
  const int64_t np = p.npad_g[g];
  const double* S = buf_of(p, mats, g, src);
  double* D = buf_of(p, mats, g, dst);
  for (int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; e < np * np; e += (int64_t)gridDim.y * blockDim.x)
    D[e] = S[e];
}

// One 64 x 64 output tile of C = alpha M + beta I + gamma E, M = alpha_l A^T B,
// per workgroup (A, B column-major n_pad x n_pad, so A^T B = A B for symmetric
// A): 4 waves of 32 x 32, float64 16x16x4 instructions (register v of lane l
// holds row l / 16 + 4 v, column l % 16), k stages of 16 through LDS.  kind 0:
// tile on or below the diagonal, entries on or below the diagonal written to
// (r, c) and (c, r) (so M and E must be symmetric); kind 1: every entry as
// is.  abuf_l (may be null): per submatrix buffer of A.  Em (may be null):
// buffer ebuf of the same submatrix, read at (r, c); it may be A or B but not
// C.  res (may be null): the sum over the valid n x n block of (M - I)^2 per
// submatrix (atomic).
__global__ __launch_bounds__(256) void ovl_prod_kernel(DevPlan p, int g0, const OvlJob* __restrict__ jobs,
                                                       const double* Am, int abuf, const int32_t* __restrict__ abuf_l,
                                                       const double* Bm, int bbuf, double* Cm, int cbuf,
                                                       const double* __restrict__ alpha_l, double alpha, double beta,
                                                       const double* Em, int ebuf, double gamma, int kind,
                                                       double* __restrict__ res) {
  constexpr int KS = 16, LD = KS + 2;
  __shared__ double la[64 * LD], lb[64 * LD];
  __shared__ double red[8];
  const OvlJob job = jobs[blockIdx.x];
  const int l = job.l;
  const int g = g0 + l;
  const int npad = p.npad_g[g];
  const int n = p.height[p.order_g[g]];
  const int64_t nn = (int64_t)npad * npad;
  const double* A = Am + p.mat_off_g[g] + (int64_t)(abuf_l ? abuf_l[l] : abuf) * nn;
  const double* B = Bm + p.mat_off_g[g] + (int64_t)bbuf * nn;
  double* C = Cm + p.mat_off_g[g] + (int64_t)cbuf * nn;
  const double* E = Em ? Em + p.mat_off_g[g] + (int64_t)ebuf * nn : nullptr;
  const int r0 = job.bi * 64, c0 = job.bj * 64;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lrow = tid >> 2, lpart = (tid & 3) * 4;
  const bool va = r0 + lrow < npad, vb = c0 + lrow < npad;
  const double* pa = A + (int64_t)(va ? r0 + lrow : 0) * npad + lpart;
  const double* pb = B + (int64_t)(vb ? c0 + lrow : 0) * npad + lpart;
  const int rl = lane & 15, kq = lane >> 4;
  d4o acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = d4o{0, 0, 0, 0};
  for (int k0 = 0; k0 < npad; k0 += KS) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      la[lrow * LD + lpart + e] = va ? pa[k0 + e] : 0.0;
      lb[lrow * LD + lpart + e] = vb ? pb[k0 + e] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KS / 4; ++kk) {
      double av[2], bv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        av[x] = la[(wm * 32 + x * 16 + rl) * LD + kk * 4 + kq];
        bv[x] = lb[(wn * 32 + x * 16 + rl) * LD + kk * 4 + kq];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
  const double al = alpha_l ? alpha_l[l] : 1.0;
  double part = 0.0;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + wm * 32 + x * 16 + kq + 4 * v;
        const int c = c0 + wn * 32 + y * 16 + rl;
        if (r >= npad || c >= npad) continue;
        if (kind == 0 && r < c) continue;
        const double m = al * acc[x][y][v];
        const double dg = r == c ? 1.0 : 0.0;
        if (res && r < n && c < n) part += (kind == 0 && r != c ? 2.0 : 1.0) * (m - dg) * (m - dg);
        const double out = alpha * m + beta * dg + (E ? gamma * E[(int64_t)c * npad + r] : 0.0);
        C[(int64_t)c * npad + r] = out;
        if (kind == 0 && r != c) C[(int64_t)r * npad + c] = out;
      }
  if (res) {
    part = block_reduce<0>(part, red);
    if (tid == 0) atomicAdd(res + l, part);
  }
}

// The same product on 128 x 128 output tiles (the job's bi, bj count
// 128-tiles): 4 waves in 2 x 2, 64 x 64 outputs each (4 x 4 blocks of
// 16 x 16), k stages of 16 double-buffered through LDS, the next stage's
// operands loaded into registers while the current one is multiplied; one
// barrier per stage.  Four times the work per operand byte of the 64-wide
// tiles.
__global__ __launch_bounds__(256, 2) void ovl_prod128_kernel(DevPlan p, int g0, const OvlJob* __restrict__ jobs,
                                                           const double* Am, int abuf,
                                                           const int32_t* __restrict__ abuf_l, const double* Bm,
                                                           int bbuf, double* Cm, int cbuf,
                                                           const double* __restrict__ alpha_l, double alpha,
                                                           double beta, const double* Em, int ebuf, double gamma,
                                                           int kind, double* __restrict__ res) {
  constexpr int KS = 16, LD = KS + 1, TE = 128;
  __shared__ double la[2][TE * LD], lb[2][TE * LD];
  __shared__ double red[8];
  const OvlJob job = jobs[blockIdx.x];
  const int l = job.l;
  const int g = g0 + l;
  const int npad = p.npad_g[g];
  const int n = p.height[p.order_g[g]];
  const int64_t nn = (int64_t)npad * npad;
  const double* A = Am + p.mat_off_g[g] + (int64_t)(abuf_l ? abuf_l[l] : abuf) * nn;
  const double* B = Bm + p.mat_off_g[g] + (int64_t)bbuf * nn;
  double* C = Cm + p.mat_off_g[g] + (int64_t)cbuf * nn;
  const double* E = Em ? Em + p.mat_off_g[g] + (int64_t)ebuf * nn : nullptr;
  const int r0 = job.bi * TE, c0 = job.bj * TE;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  // loads: thread t fills row t / 2 of both operand stages, k half (t % 2) * 8
  const int lrow = tid >> 1, lk = (tid & 1) * 8;
  const bool va = r0 + lrow < npad, vb = c0 + lrow < npad;
  const double* pa = A + (int64_t)(va ? r0 + lrow : 0) * npad + lk;
  const double* pb = B + (int64_t)(vb ? c0 + lrow : 0) * npad + lk;
  typedef double d2 __attribute__((ext_vector_type(2)));
  d2 ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      ra[e] = va ? *reinterpret_cast<const d2*>(pa + k0 + 2 * e) : d2{0.0, 0.0};
      rb[e] = vb ? *reinterpret_cast<const d2*>(pb + k0 + 2 * e) : d2{0.0, 0.0};
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      la[buf][lrow * LD + lk + 2 * e] = ra[e].x;
      la[buf][lrow * LD + lk + 2 * e + 1] = ra[e].y;
      lb[buf][lrow * LD + lk + 2 * e] = rb[e].x;
      lb[buf][lrow * LD + lk + 2 * e + 1] = rb[e].y;
    }
  };
  const int rl = lane & 15, kq = lane >> 4;
  d4o acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = d4o{0, 0, 0, 0};
  const int nst = npad / KS;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int s = 0; s < nst; ++s) {
    const int buf = s & 1;
    if (s + 1 < nst) fetch((s + 1) * KS);
#pragma unroll
    for (int kk = 0; kk < KS / 4; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        av[x] = la[buf][(wm * 64 + x * 16 + rl) * LD + kk * 4 + kq];
        bv[x] = lb[buf][(wn * 64 + x * 16 + rl) * LD + kk * 4 + kq];
      }
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[y], acc[x][y], 0, 0, 0);
    }
    // the other buffer was last read in stage s - 1, before the barrier that
    // ended it
    if (s + 1 < nst) stash(buf ^ 1);
    __syncthreads();
  }
  const double al = alpha_l ? alpha_l[l] : 1.0;
  double part = 0.0;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + wm * 64 + x * 16 + kq + 4 * v;
        const int c = c0 + wn * 64 + y * 16 + rl;
        if (r >= npad || c >= npad) continue;
        if (kind == 0 && r < c) continue;
        const double m = al * acc[x][y][v];
        const double dg = r == c ? 1.0 : 0.0;
        if (res && r < n && c < n) part += (kind == 0 && r != c ? 2.0 : 1.0) * (m - dg) * (m - dg);
        const double out = alpha * m + beta * dg + (E ? gamma * E[(int64_t)c * npad + r] : 0.0);
        C[(int64_t)c * npad + r] = out;
        if (kind == 0 && r != c) C[(int64_t)r * npad + c] = out;
      }
  if (res) {
    part = block_reduce<0>(part, red);
    if (tid == 0) atomicAdd(res + l, part);
  }
}

// D[:, loc .. loc + b) = f(l) Z[:, ...] - U[:, ...] for the rows < n (f: 1 / sqrt(c)).
__global__ __launch_bounds__(256) void ovl_slab_diff_kernel(DevPlan p, int g0, const double* Zm, int zbuf,
                                                            const double* Um, int ubuf, double* Dm, int dbuf,
                                                            const double* __restrict__ f_l) {
  const int l = blockIdx.x;
  const int g = g0 + l;
  const int i = p.order_g[g];
  const int npad = p.npad_g[g];
  const int n = p.height[i];
  const int loc = p.loc[i], b = p.bs[i];
  const int64_t nn = (int64_t)npad * npad;
  const double* Z = Zm + p.mat_off_g[g] + (int64_t)zbuf * nn;
  const double* U = Um + p.mat_off_g[g] + (int64_t)ubuf * nn;
  double* D = Dm + p.mat_off_g[g] + (int64_t)dbuf * nn;
  const double f = f_l ? f_l[l] : 1.0;
  for (int e = threadIdx.x; e < npad * b; e += blockDim.x) {
    const int q = e / npad, r = e - q * npad;
    const int64_t k = (int64_t)(loc + q) * npad + r;
    D[k] = r < n ? f * Z[k] - U[k] : 0.0;
  }
}

// Block column i of P: rows < n of columns loc .. loc + b of R, into the
// panel of column i (rows idx_i in panel order: a contiguous copy).
__global__ __launch_bounds__(256) void ovl_scatter_kernel(DevPlan p, int g0, const double* Rm, int rbuf,
                                                          double* __restrict__ P) {
  const int g = g0 + blockIdx.x;
  const int i = p.order_g[g];
  const int npad = p.npad_g[g];
  const int n = p.height[i];
  const int loc = p.loc[i], b = p.bs[i];
  const double* R = Rm + p.mat_off_g[g] + (int64_t)rbuf * npad * npad;
  double* out = P + p.panel_off[i];
  for (int e = threadIdx.x; e < n * b; e += blockDim.x) {
    const int q = e / n, r = e - q * n;
    out[e] = R[(int64_t)(loc + q) * npad + r];
  }
}

// Buffer of the final X of every submatrix (the sign iteration's state).
__global__ void ovl_xbuf_kernel(const SubState* __restrict__ st, int nsub, int32_t* __restrict__ xbuf) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < nsub) xbuf[l] = st[l].iters & 1;
}

__global__ void ovl_zero_kernel(double* v, int n) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < n) v[l] = 0.0;
}

// Largest value of v[0 .. n) into mapped host memory.
__global__ __launch_bounds__(256) void ovl_max_kernel(const double* __restrict__ v, int n, double* out) {
  __shared__ double red[8];
  double m = 0.0;
  for (int l = threadIdx.x; l < n; l += blockDim.x) m = fmax(m, v[l]);
  m = block_reduce<1>(m, red);
  if (threadIdx.x == 0) *out = m;
}

static int spread(int64_t work) { return (int)std::min<int64_t>(64, std::max<int64_t>(1, work / (256 * 64))); }

hipError_t launch_ovl_fill(const DevPlan& p, int g0, int nsub, int max_npad, double* mats, int b, double dv, double dp,
                           hipStream_t s) {
  hipLaunchKernelGGL(ovl_fill_kernel, dim3(nsub, spread((int64_t)max_npad * max_npad)), dim3(256), 0, s, p, g0, mats,
                     b, dv, dp);
  return hipGetLastError();
}

hipError_t launch_ovl_gather(const DevPlan& p, int g0, int nsub, int max_m, const double* V, double* mats, int b,
                             hipStream_t s) {
  hipLaunchKernelGGL(ovl_gather_kernel, dim3(nsub, max_m), dim3(256), 0, s, p, g0, V, mats, b);
  return hipGetLastError();
}

hipError_t launch_ovl_gersh(const DevPlan& p, int g0, int nsub, double* mats, int b, double* out, int pad_one,
                            sm_sub_stats* stats, hipStream_t s) {
  hipLaunchKernelGGL(ovl_gersh_kernel, dim3(nsub), dim3(256), 0, s, p, g0, mats, b, out, pad_one, stats);
  return hipGetLastError();
}

hipError_t launch_ovl_scale(const DevPlan& p, int g0, int nsub, int max_npad, double* mats, int b, const double* v,
                            int mode, hipStream_t s) {
  hipLaunchKernelGGL(ovl_scale_kernel, dim3(nsub, spread((int64_t)max_npad * max_npad)), dim3(256), 0, s, p, g0,
                     mats, b, v, mode);
  return hipGetLastError();
}

hipError_t launch_ovl_copy(const DevPlan& p, int g0, int nsub, int max_npad, double* mats, int src, int dst,
                           hipStream_t s) {
  hipLaunchKernelGGL(ovl_copy_kernel, dim3(nsub, spread((int64_t)max_npad * max_npad)), dim3(256), 0, s, p, g0,
                     mats, src, dst);
  return hipGetLastError();
}

hipError_t launch_ovl_prod(const DevPlan& p, int g0, const OvlJob* jobs, int njobs, int edge, const double* A,
                           int abuf, const int32_t* abuf_l, const double* B, int bbuf, double* C, int cbuf,
                           const double* alpha_l, double alpha, double beta, const double* E, int ebuf,
                           double gamma, int kind, double* res, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  if (edge == 128)
    hipLaunchKernelGGL(ovl_prod128_kernel, dim3(njobs), dim3(256), 0, s, p, g0, jobs, A, abuf, abuf_l, B, bbuf, C,
                       cbuf, alpha_l, alpha, beta, E, ebuf, gamma, kind, res);
  else
    hipLaunchKernelGGL(ovl_prod_kernel, dim3(njobs), dim3(256), 0, s, p, g0, jobs, A, abuf, abuf_l, B, bbuf, C,
                       cbuf, alpha_l, alpha, beta, E, ebuf, gamma, kind, res);
  return hipGetLastError();
}

hipError_t launch_ovl_slab_diff(const DevPlan& p, int g0, int nsub, const double* Z, int zbuf, const double* U,
                                int ubuf, double* D, int dbuf, const double* f_l, hipStream_t s) {
  hipLaunchKernelGGL(ovl_slab_diff_kernel, dim3(nsub), dim3(256), 0, s, p, g0, Z, zbuf, U, ubuf, D, dbuf, f_l);
  return hipGetLastError();
}

hipError_t launch_ovl_scatter(const DevPlan& p, int g0, int nsub, const double* R, int rbuf, double* P, hipStream_t s) {
  hipLaunchKernelGGL(ovl_scatter_kernel, dim3(nsub), dim3(256), 0, s, p, g0, R, rbuf, P);
  return hipGetLastError();
}

hipError_t launch_ovl_xbuf(const SubState* st, int nsub, int32_t* xbuf, hipStream_t s) {
  hipLaunchKernelGGL(ovl_xbuf_kernel, dim3((nsub + 255) / 256), dim3(256), 0, s, st, nsub, xbuf);
  return hipGetLastError();
}

hipError_t launch_ovl_zero(double* v, int n, hipStream_t s) {
  hipLaunchKernelGGL(ovl_zero_kernel, dim3((n + 255) / 256), dim3(256), 0, s, v, n);
  return hipGetLastError();
}

hipError_t launch_ovl_max(const double* v, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(ovl_max_kernel, dim3(1), dim3(256), 0, s, v, n, out);
  return hipGetLastError();
}

}  // namespace sm
