// Step 1 of the submatrix method (Fig. 2 of the paper): build every dense
// principal submatrix T_i = H[idx_i, idx_i] - mu I (Eq. 14 with S = I) straight
// from the block-column panels of H, then pick the spectral scale c_i of
// X_0 = T_i / c_i, the starting point of the sign iteration.  The float64
// schedule stores X_0; the others keep T_i (float32, or straight in the
// 16-bit operand copies of the low-precision products) and the first square
// and update of the iteration multiply by 1 / c_i, which saves a pass over
// every submatrix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "device_common.h"
#include "row_map.h"
#include "smsign_internal.h"

namespace sm {

// Value of v held by lane `src` (wave-uniform src), for every lane.
__device__ __forceinline__ double lane_value(double v, int src) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
// Lanes 2k and 2k + 1 exchange v (a DPP quad permutation [1, 0, 3, 2], no LDS
// round trip); both lanes of the pair must be active.
__device__ __forceinline__ uint32_t lane_pair_swap(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
}

// Statistics of T_i gathered column by column: column abs sums (= row sums,
// T is symmetric) give the Gershgorin bound c_G >= rho(T); with the diagonal
// they give the 16 features of the scaling network.
struct ColStats {
  double cmax = 0.0, sdiag = 0.0, sdiag2 = 0.0, mind = 1e300, maxd = -1e300, sR = 0.0, maxR = 0.0;
  double minabs = 1e300, mingap = 1e300, nneg = 0.0, sown = 0.0, minown = 1e300, sabs = 0.0;
  __device__ void add(double s, double dg, bool own) {
    const double R = s - fabs(dg);
    cmax = fmax(cmax, s);
    sdiag += dg;
    sdiag2 += dg * dg;
    mind = fmin(mind, dg);
    maxd = fmax(maxd, dg);
    sR += R;
    maxR = fmax(maxR, R);
    minabs = fmin(minabs, fabs(dg));
    mingap = fmin(mingap, fabs(dg) - R);
    nneg += dg < 0.0 ? 1.0 : 0.0;
    sabs += fabs(dg);
    if (own) {
      sown += dg;
      minown = fmin(minown, fabs(dg));
    }
  }
};

// One workgroup per submatrix; its waves take the atoms j of the index set I_i
// in turn (wave w: atoms w, w + nw, ...), each wave independently:
//   (a) intersects the stored pattern of H's block column j with I_i by binary
//       search in LDS and records, in its own LDS row map, which panel row of
//       column j supplies every destination row of T_i (-1: block not stored);
//   (b) writes the b_j columns of T_i top to bottom (coalesced stores; reads
//       are runs of one contiguous panel column), subtracting mu on the
//       diagonal, and zeros in the padding rows, and accumulates each
//       column's abs sum, sum of squares and diagonal entry (float64).
// Only wave-level ordering is needed between (a) and (b), so the waves never
// wait for each other.  Then the identity padding columns, and the features
// of the submatrix from the statistics of all waves.
// LDS: atoms of I_i and their row offsets (2 m ints), one row map of n_pad
// ints per wave.
// POW: also the first power-iteration product w = T v0 (v0 the fixed +-1
// probe vector 11, Euclidean norm sqrt(n)) for the scale kernel, from the
// entries as they are gathered: each wave adds its columns' contributions to
// its own LDS row of partial sums, combined in wave order at the end.  This
// saves the scale kernel one read pass over T.
template <typename T, int KIND, bool POW>
__global__ __launch_bounds__(256, 4) void gather_kernel(DevPlan p, int g0, const double* __restrict__ H,
                                                     double mu, T* __restrict__ mats,
                                                     int64_t shadow_off, int* nonfinite,
                                                     float* __restrict__ features, double* __restrict__ cg_out,
                                                     sm_sub_stats* __restrict__ stats,
                                                     double* __restrict__ vecs,
                                                     const int32_t* __restrict__ subs) {
  extern __shared__ __attribute__((aligned(16))) int smem[];
  __shared__ double red[8];
  // workgroup -> local index of its submatrix in the chunk (all, or a list)
  const int l = subs ? subs[blockIdx.x] : (int)blockIdx.x;
  const int g = g0 + l;
  const int i = p.order_g[g];
  const int npad = p.npad_g[g];
  const int n = p.height[i];
  const int loc = p.loc[i];
  const int bsz = p.bs[i];
  const int64_t k0 = p.col_ptr[i];
  const int m = (int)(p.col_ptr[i + 1] - k0);
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  int* s_atom = smem;
  int* s_off = smem + m;
  RowSrc* s_src = reinterpret_cast<RowSrc*>(smem + 2 * m) + wid * npad;
  // POW: partial sums of T v0, one row of n_pad doubles per wave
  double* s_tv = reinterpret_cast<double*>(reinterpret_cast<char*>(smem) + row_maps_bytes(m, nw, npad)) + wid * npad;
  T* X = mats + p.mat_off_g[g];
  // low-precision schedules: T goes straight into the 16-bit operand copies
  // that the products read (the float32 buffer is not written).  Every lane
  // of the wave calls put for the same column and row lane + 64 j, so lanes
  // 2k and 2k + 1 hold rows d and d + 1 (both below n_pad, a multiple of 32)
  // and trade halves: the even lane stores both hi values, the odd lane both
  // lo values, each as one 4-byte store.
  uint16_t* cp = reinterpret_cast<uint16_t*>(X + shadow_off);
  auto put = [&](int c, int d, double x) {
    if constexpr (KIND != 0) {
      const float xf = (float)x;
      const uint32_t h = shadow_hi(xf, KIND);
      const bool odd = (lane & 1) != 0;
      if constexpr (KIND == SM_BF16X3) {
        const uint32_t lo = shadow_lo(xf, (uint16_t)h);
        const uint32_t other = lane_pair_swap(odd ? h : lo);
        // one store per lane, no divergent branch: the even lane's word goes
        // to the hi plane, the odd lane's to the lo plane 32 entries on
        const int64_t k = copy_idx<true>(c, d & ~1, npad) + (odd ? 32 : 0);
        const uint32_t word = odd ? (other | (lo << 16)) : (h | (other << 16));
        *reinterpret_cast<uint32_t*>(cp + k) = word;
      } else {
        const uint32_t other = lane_pair_swap(h);
        if (!odd) *reinterpret_cast<uint32_t*>(cp + copy_idx<false>(c, d, npad)) = h | (other << 16);
      }
    } else {
      X[(int64_t)c * npad + d] = (T)x;
    }
  };
  for (int t = threadIdx.x; t < m; t += blockDim.x) {
    s_atom[t] = p.row_idx[k0 + t];
    s_off[t] = p.blk_rowoff[k0 + t];
  }
  if constexpr (POW)
    for (int d = lane; d < npad; d += kWave) s_tv[d] = 0.0;
  __syncthreads();
  bool bad = false;
  ColStats cs;   // this wave's columns (identical in every lane)
  double ssq_lane = 0.0;   // sum of squares of this lane's entries, reduced once at the end
  for (int jj = wid; jj < m; jj += nw) {
    const int j = s_atom[jj];
    const int locj = s_off[jj];
    const int bj = p.bs[j];
    const int hj = p.height[j];
    build_row_map(p, j, s_atom, s_off, m, n, s_src);
    const double* panel = H + p.panel_off[j];
    // four columns of the atom at a time: one row-map read and four
    // independent panel loads per row
    for (int q0 = 0; q0 < bj; q0 += 4) {
      double sa[4] = {0.0, 0.0, 0.0, 0.0}, dl[4] = {0.0, 0.0, 0.0, 0.0};
      double pv[4] = {0.0, 0.0, 0.0, 0.0};   // probe entries of the four columns
      if constexpr (POW)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (q0 + u < bj) pv[u] = probe_entry(11, locj + q0 + u);
#pragma unroll 2
      for (int d = lane; d < npad; d += kWave) {
        const int s = d < n ? s_src[d] : -1;
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = (q0 + u < bj && s >= 0) ? panel[(int64_t)(q0 + u) * hj + s] : 0.0;
        double tv = 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = locj + q0 + u;
          if (q0 + u < bj) {
            // the diagonal (c < n, so only rows of T_i), without a branch
            const bool on_diag = d == c;
            const double x = on_diag ? v[u] - mu : v[u];
            dl[u] = on_diag ? x : dl[u];
            sa[u] += fabs(x);
            ssq_lane += x * x;
            tv += x * pv[u];
            put(c, d, x);
          }
        }
        if constexpr (POW) s_tv[d] += tv;
      }
      // per column: the abs sum over the wave (a NaN or Inf entry makes it
      // non-finite), and the diagonal entry from the one lane that holds it
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = locj + q0 + u;
        if (q0 + u < bj) {
          bad |= !isfinite(sa[u]);
          cs.add(wave_sum(sa[u]), lane_value(dl[u], c & (kWave - 1)), c >= loc && c < loc + bsz);
        }
      }
    }
    wave_sync();   // the row map is rebuilt for the wave's next atom
  }
  // identity padding: X stays exactly I on the pad under the iteration
  for (int c = n + wid; c < npad; c += nw)
    for (int d = lane; d < npad; d += kWave) put(c, d, d == c ? 1.0 : 0.0);
  if (bad) *nonfinite = 1 + i;
  if constexpr (POW) {   // w = T v0 = the waves' partial sums in wave order
    __syncthreads();
    const double* tv0 = s_tv - wid * npad;
    double* w = vecs + p.vec_off_g[g] + npad;
    for (int d = threadIdx.x; d < n; d += blockDim.x) {
      double y = 0.0;
      for (int k = 0; k < nw; ++k) y += tv0[k * npad + d];
      w[d] = y;
    }
  }
  // combine the waves (every lane of a wave holds its values)
  const double cmax = block_reduce<1>(cs.cmax, red);
  const double sdiag = block_reduce<0>(lane == 0 ? cs.sdiag : 0.0, red);
  const double sdiag2 = block_reduce<0>(lane == 0 ? cs.sdiag2 : 0.0, red);
  const double mind = block_reduce<2>(cs.mind, red);
  const double maxd = block_reduce<1>(cs.maxd, red);
  const double sR = block_reduce<0>(lane == 0 ? cs.sR : 0.0, red);
  const double maxR = block_reduce<1>(cs.maxR, red);
  const double minabs = block_reduce<2>(cs.minabs, red);
  const double mingap = block_reduce<2>(cs.mingap, red);
  const double nneg = block_reduce<0>(lane == 0 ? cs.nneg : 0.0, red);
  const double ssq = block_reduce<0>(ssq_lane, red);
  const double sown = block_reduce<0>(lane == 0 ? cs.sown : 0.0, red);
  const double minown = block_reduce<2>(cs.minown, red);
  const double sabs = block_reduce<0>(lane == 0 ? cs.sabs : 0.0, red);
  if (threadIdx.x == 0) {
    const double cG = cmax > 0.0 ? cmax : 1.0;
    const double nn = (double)n;
    const double mean = sdiag / nn;
    float f[kNumFeatures];
    f[0] = (float)log(nn);
    f[1] = (float)log(cG);
    f[2] = (float)(mean / cG);
    f[3] = (float)(sqrt(fmax(sdiag2 / nn - mean * mean, 0.0)) / cG);
    f[4] = (float)(mind / cG);
    f[5] = (float)(maxd / cG);
    f[6] = (float)(sR / nn / cG);
    f[7] = (float)(maxR / cG);
    f[8] = (float)(minabs / cG);
    f[9] = (float)(mingap / cG);
    f[10] = (float)(nneg / nn);
    f[11] = (float)(sqrt(ssq) / (cG * sqrt(nn)));
    f[12] = (float)(bsz / nn);
    f[13] = (float)(sown / bsz / cG);
    f[14] = (float)(minown / cG);
    f[15] = (float)(sabs / nn / cG);
    sm_sub_stats& r = stats[i];
    for (int k = 0; k < kNumFeatures; ++k) {
      features[(int64_t)l * kNumFeatures + k] = f[k];
      r.feat[k] = f[k];
    }
    r.gersh = cG;
    cg_out[l] = cG;
  }
}

size_t gather_lds_bytes(int max_m, int max_npad, bool power) {
  // 4 waves: atoms + offsets, a row map per wave, (power) a row of partial
  // sums of T v0 per wave
  size_t b = row_maps_bytes(max_m, 4, max_npad);
  if (power) b += (size_t)4 * max_npad * sizeof(double);
  return b;
}

hipError_t launch_gather(const DevPlan& p, int g0, int nsub, int max_m, int max_npad,
                         const double* H, double mu, void* mats, int storage_f64, int shadow_kind,
                         int64_t shadow_off, int* nonfinite, float* features, double* cg_out,
                         sm_sub_stats* stats, double* power_vecs, const int32_t* subs, hipStream_t s) {
  if (nsub <= 0) return hipSuccess;
  const bool pw = power_vecs != nullptr;
  const size_t lds = gather_lds_bytes(max_m, max_npad, pw);
#define SM_GATHER(TT, K, PW)                                                                             \
  hipLaunchKernelGGL((gather_kernel<TT, K, PW>), dim3(nsub), dim3(256), lds, s, p, g0, H, mu, (TT*)mats, \
                     shadow_off, nonfinite, features, cg_out, stats, power_vecs, subs)
#define SM_GATHER2(TT, K) \
  if (pw) SM_GATHER(TT, K, true); else SM_GATHER(TT, K, false)
  if (storage_f64) { SM_GATHER2(double, 0); }
  else if (shadow_kind == SM_BF16X3) { SM_GATHER2(float, SM_BF16X3); }
  else if (shadow_kind == SM_BF16) { SM_GATHER2(float, SM_BF16); }
  else if (shadow_kind == SM_F16) { SM_GATHER2(float, SM_F16); }
  else { SM_GATHER2(float, 0); }
#undef SM_GATHER2
#undef SM_GATHER
  return hipGetLastError();
}

// One workgroup per submatrix: optional power iteration on T (column dots with
// a vector kept in the workspace; est = ||T v_k|| <= rho(T)), the choice of c;
// float64: X_0 = T / c on the n x n block (the identity pad is left as is),
// otherwise x0s_out = 1 / c for the first products.
//   Gershgorin: c = c_G.   Power: c = min(c_G, (1 + margin) est).
//   Learned: c_hat = c_G exp(y0) (1 + margin) from the network, accepted only if
//   est <= c_hat <= c_G (the guard), else c = c_G.
template <typename T>
__global__ __launch_bounds__(512) void scale_kernel(DevPlan p, int g0, T* __restrict__ mats, int scaling,
                                                    int power_steps, double margin,
                                                    double* __restrict__ vecs,
                                                    const double* __restrict__ cg_in,
                                                    const float* __restrict__ pred,
                                                    sm_sub_stats* __restrict__ stats, int shadow_kind,
                                                    int64_t shadow_off, double lbound,
                                                    double* __restrict__ lb0_out,
                                                    double* __restrict__ top0_out,
                                                    double* __restrict__ x0s_out, int pre_w,
                                                    double force_scale,
                                                    const int32_t* __restrict__ subs) {
  __shared__ double red[16];
  __shared__ double mv[matvec_red<1, T>(8)];
  const int l = subs ? subs[blockIdx.x] : (int)blockIdx.x;
  const int g = g0 + l;
  const int i = p.order_g[g];
  const int npad = p.npad_g[g];
  const int n = p.height[i];
  T* X = mats + p.mat_off_g[g];
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const double cG = cg_in[l];
  // low-precision schedules hold T only in its 16-bit operand copies
  bool copies = false;
  if constexpr (std::is_same<T, float>::value) copies = shadow_kind != 0;
  const uint16_t* cp = reinterpret_cast<const uint16_t*>(X + shadow_off);

  double est = -1.0;
  if (scaling != SM_SCALE_GERSHGORIN && power_steps > 0) {
    double* v = vecs + p.vec_off_g[g];
    double* w = v + npad;
    int it0 = 0;
    double inv;
    if (pre_w) {
      // the gather formed w = T v0 for the unit-free probe v0 (+-1 entries,
      // norm sqrt(n)): the first step's estimate and the next direction
      double nw2 = 0.0;
      for (int d = threadIdx.x; d < n; d += blockDim.x) nw2 += w[d] * w[d];
      nw2 = block_reduce<0>(nw2, red);
      est = sqrt(nw2 / (double)n);
      inv = nw2 > 0.0 ? 1.0 / sqrt(nw2) : 0.0;
      for (int d = threadIdx.x; d < n; d += blockDim.x) v[d] = w[d] * inv;
      __syncthreads();
      it0 = 1;
    } else {
      double nv = 0.0;
      for (int d = threadIdx.x; d < n; d += blockDim.x) {
        const double x = probe_entry(11, d);
        v[d] = x;
        nv += x * x;
      }
      nv = block_reduce<0>(nv, red);
      inv = 1.0 / sqrt(nv);
      for (int d = threadIdx.x; d < n; d += blockDim.x) v[d] *= inv;
      __syncthreads();
    }
    for (int it = it0; it < power_steps; ++it) {
      if (copies) {   // w = T v
        if (shadow_kind == SM_BF16X3)
          block_matvec_copies<1, true>(cp, npad, n, shadow_kind, v, 0, mv, [&](int, int r, double y) { w[r] = y; });
        else
          block_matvec_copies<1, false>(cp, npad, n, shadow_kind, v, 0, mv, [&](int, int r, double y) { w[r] = y; });
      } else {
        block_matvec<1>(X, npad, n, v, 0, mv, [&](int, int r, double y) { w[r] = y; });
      }
      double nw2 = 0.0;
      for (int d = threadIdx.x; d < n; d += blockDim.x) nw2 += w[d] * w[d];
      nw2 = block_reduce<0>(nw2, red);
      est = sqrt(nw2);
      inv = est > 0.0 ? 1.0 / est : 0.0;
      for (int d = threadIdx.x; d < n; d += blockDim.x) v[d] = w[d] * inv;
      __syncthreads();
    }
  }
  double c = cG;
  int src = 0;
  // smallest |eigenvalue| of T as a fraction of c_G (scaled Newton-Schulz)
  double lrel = lbound;
  if (scaling == SM_SCALE_POWER && est > 0.0) {
    c = fmin(cG, (1.0 + margin) * est);
    src = 1;
  } else if (scaling == SM_SCALE_LEARNED) {
    const double y0 = pred ? (double)pred[2 * l] : 0.0;
    const double ch = cG * exp(fmin(y0, 0.0)) * (1.0 + margin);
    if (pred && isfinite(y0) && ch >= est && ch <= cG) {
      c = ch;
      src = 2;
      const double y1 = (double)pred[2 * l + 1];
      if (isfinite(y1)) lrel = exp(fmin(y1, 0.0));
    } else {
      src = 3;
    }
  }
  // testing: a scale forced below the spectral radius, with its bound withheld
  if (force_scale > 0.0) {
    c = force_scale * cG;
    src = 4;
  }
  const double sc = 1.0 / c;
  // float64: X_0 = T / c in place.  float32 and the 16-bit schedules keep T
  // in their buffers and the first square and update apply 1 / c (x0s); the
  // identity pad's diagonal becomes c there, so that the pad of X_0 stays I
  // (to the rounding of c and 1 / c) and does not iterate.
  if constexpr (std::is_same<T, double>::value) {
    for (int cc = wid; cc < n; cc += nw) {
      T* col = X + (int64_t)cc * npad;
      for (int d = lane; d < n; d += kWave) col[d] = col[d] * sc;
    }
  } else {
    const float cf = (float)c;
    for (int d = n + threadIdx.x; d < npad; d += blockDim.x) {
      if (!copies) {
        X[(int64_t)d * npad + d] = cf;
      } else {
        uint16_t* cw = reinterpret_cast<uint16_t*>(X + shadow_off);
        const uint16_t h = shadow_hi(cf, shadow_kind);
        if (shadow_kind == SM_BF16X3) {
          const int64_t k = copy_idx<true>(d, d, npad);
          cw[k] = h;
          cw[k + 32] = shadow_lo(cf, h);
        } else {
          cw[copy_idx<false>(d, d, npad)] = h;
        }
      }
    }
  }
  if (threadIdx.x == 0) {
    sm_sub_stats& r = stats[i];
    r.scale = c;
    r.scale_src = src;
    r.rho_est = est;
    // X_0 = T / c: |eigenvalues| in [lrel c_G / c, c_G / c] (the top is rigorous)
    const double lb = fmin(fmax(lrel, 0.0) * cG / c, 1.0);
    r.lb0 = lb;
    lb0_out[l] = lb;
    top0_out[l] = force_scale > 0.0 ? 1.0 : cG / c;
    x0s_out[l] = std::is_same<T, double>::value ? 1.0 : sc;
  }
}

hipError_t launch_scale(const DevPlan& p, int g0, int nsub, void* mats, int storage_f64, int scaling,
                        int power_steps, double margin, double* vecs, const double* cg_in,
                        const float* pred, sm_sub_stats* stats, int shadow_kind, int64_t shadow_off,
                        double lbound, double* lb0_out, double* top0_out, double* x0s_out, bool pre_w,
                        double force_scale, const int32_t* subs, hipStream_t s) {
  if (nsub <= 0) return hipSuccess;
  if (storage_f64)
    hipLaunchKernelGGL(scale_kernel<double>, dim3(nsub), dim3(512), 0, s, p, g0, (double*)mats, scaling,
                       power_steps, margin, vecs, cg_in, pred, stats, 0, (int64_t)0, lbound, lb0_out,
                       top0_out, x0s_out, pre_w ? 1 : 0, force_scale, subs);
  else
    hipLaunchKernelGGL(scale_kernel<float>, dim3(nsub), dim3(512), 0, s, p, g0, (float*)mats, scaling,
                       power_steps, margin, vecs, cg_in, pred, stats, shadow_kind, shadow_off, lbound,
                       lb0_out, top0_out, x0s_out, pre_w ? 1 : 0, force_scale, subs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// First-step bound of scaled Newton-Schulz (SubState.amode): the first square
// ran unscaled and left Y' = 3I - A, A = X_0^2, in buffer 2 of its submatrix.
// The largest column sum of |A| bounds rho(A) = rho(X_0)^2 (Gershgorin on the
// square, usually several times tighter than (c_G / c)^2, since the signs of
// the entries of X_0 cancel in its square); the scheduler takes the first
// update's scale from it, and Y = 3I - a^2 A is then formed in place.
// Storage kinds: 0 float64, 1 float32, 2 split-bf16 copies, 3 bf16, 4 f16.
// ---------------------------------------------------------------------------
typedef uint16_t y_h4 __attribute__((ext_vector_type(4)));
typedef float y_f4 __attribute__((ext_vector_type(4)));

template <int KIND>
__device__ __forceinline__ void y_load4(const void* base, int64_t col, int rb, int npad, double (&v)[4]) {
  if constexpr (KIND == 0) {
    const double* y = static_cast<const double*>(base) + col * npad + rb;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = y[e];
  } else if constexpr (KIND == 1) {
    const y_f4 t = *reinterpret_cast<const y_f4*>(static_cast<const float*>(base) + col * npad + rb);
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (double)t[e];
  } else if constexpr (KIND == 2) {
    const uint16_t* cp = static_cast<const uint16_t*>(base);
    const int64_t k = copy_idx<true>(col, rb, npad);
    const y_h4 hi = *reinterpret_cast<const y_h4*>(cp + k);
    const y_h4 lo = *reinterpret_cast<const y_h4*>(cp + k + 32);
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (double)bf16_bits_to_f32(hi[e]) + (double)bf16_bits_to_f32(lo[e]);
  } else {
    const uint16_t* cp = static_cast<const uint16_t*>(base);
    const y_h4 hi = *reinterpret_cast<const y_h4*>(cp + copy_idx<false>(col, rb, npad));
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (double)copy_value(hi[e], KIND == 4 ? SM_F16 : SM_BF16);
  }
}

// The same four entries written back in the storage's own form (the copies
// as the products write them: the float32 value rounded to hi, and lo).
template <int KIND>
__device__ __forceinline__ void y_store4(void* base, int64_t col, int rb, int npad, const double (&v)[4]) {
  if constexpr (KIND == 0) {
    double* y = static_cast<double*>(base) + col * npad + rb;
#pragma unroll
    for (int e = 0; e < 4; ++e) y[e] = v[e];
  } else if constexpr (KIND == 1) {
    *reinterpret_cast<y_f4*>(static_cast<float*>(base) + col * npad + rb) =
        y_f4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
  } else {
    uint16_t* cp = static_cast<uint16_t*>(base);
    y_h4 hi, lo;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float f = (float)v[e];
      hi[e] = shadow_hi(f, KIND == 4 ? SM_F16 : (KIND == 3 ? SM_BF16 : SM_BF16X3));
      if (KIND == 2) lo[e] = shadow_lo(f, hi[e]);
    }
    if constexpr (KIND == 2) {
      const int64_t k = copy_idx<true>(col, rb, npad);
      *reinterpret_cast<y_h4*>(cp + k) = hi;
      *reinterpret_cast<y_h4*>(cp + k + 32) = lo;
    } else {
      *reinterpret_cast<y_h4*>(cp + copy_idx<false>(col, rb, npad)) = hi;
    }
  }
}

// Buffer 2 of processing index g as stored (float64 / float32 values, or the
// operand copies).
template <int KIND>
__device__ __forceinline__ void* y_base(const DevPlan& p, void* mats, int g, int64_t shadow_off) {
  const int64_t np = p.npad_g[g];
  const int64_t off = p.mat_off_g[g] + 2 * np * np;
  if constexpr (KIND == 0) return static_cast<double*>(mats) + off;
  if constexpr (KIND == 1) return static_cast<float*>(mats) + off;
  return static_cast<float*>(mats) + off + shadow_off;
}

// One workgroup (16 waves) per submatrix, a wave per column in turn; column
// sums in float64 in a fixed order, so colmax does not depend on timing.
template <int KIND>
__global__ __launch_bounds__(1024) void first_colmax_kernel(DevPlan p, int g0, const void* mats,
                                                            int64_t shadow_off, const SubState* __restrict__ st,
                                                            double* __restrict__ colmax) {
  __shared__ double red[16];
  const int l = blockIdx.x;
  if (!(st[l].amode && st[l].iters == 0 && st[l].active)) {
    if (threadIdx.x == 0) colmax[l] = 0.0;
    return;
  }
  const int g = g0 + l;
  const int npad = p.npad_g[g];
  const void* y = y_base<KIND>(p, const_cast<void*>(mats), g, shadow_off);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double mx = 0.0;
  for (int c = wid; c < npad; c += 16) {
    double sum = 0.0;
    for (int rb = 4 * lane; rb < npad; rb += 256) {
      double v[4];
      y_load4<KIND>(y, c, rb, npad, v);
#pragma unroll
      for (int e = 0; e < 4; ++e) sum += (rb + e == c) ? fabs(3.0 - v[e]) : fabs(v[e]);
    }
    sum = wave_sum(sum);
    mx = (sum == sum) ? fmax(mx, sum) : INFINITY;   // a NaN leaves c_G / c in force
  }
  if (lane == 0) red[wid] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) m = fmax(m, red[w]);
    colmax[l] = m;
  }
}

// Y = a^2 Y' + 3 (1 - a^2) I over the padded submatrix, four rows of a
// column per thread and step.
template <int KIND>
__global__ __launch_bounds__(256) void first_fix_y_kernel(DevPlan p, int g0, void* mats, int64_t shadow_off,
                                                          const SubState* __restrict__ st) {
  const int l = blockIdx.x;
  if (!st[l].fix_y) return;
  const double a = st[l].alpha_upd;
  const double a2 = a * a, d = 3.0 * (1.0 - a2);
  const int g = g0 + l;
  const int npad = p.npad_g[g];
  const int q4 = npad / 4;
  void* y = y_base<KIND>(p, mats, g, shadow_off);
  const int64_t quads = (int64_t)npad * q4;
  for (int64_t q = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; q < quads;
       q += (int64_t)gridDim.y * blockDim.x) {
    const int64_t c = q / q4;
    const int rb = 4 * (int)(q - c * q4);
    double v[4];
    y_load4<KIND>(y, c, rb, npad, v);
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = a2 * v[e] + ((rb + e == c) ? d : 0.0);
    y_store4<KIND>(y, c, rb, npad, v);
  }
}

static int y_kind(int storage) {
  return storage == SM_F64 ? 0 : storage == SM_F32 ? 1 : storage == SM_BF16X3 ? 2 : storage == SM_BF16 ? 3 : 4;
}

hipError_t launch_first_colmax(const DevPlan& p, int g0, int nsub, const void* mats, int storage,
                               int64_t shadow_off, const SubState* st, double* colmax, hipStream_t s) {
  if (nsub <= 0) return hipSuccess;
#define SM_COLMAX(K)                                                                                        \
  hipLaunchKernelGGL(first_colmax_kernel<K>, dim3(nsub), dim3(1024), 0, s, p, g0, mats, shadow_off, st, colmax)
  switch (y_kind(storage)) {
    case 0: SM_COLMAX(0); break;
    case 1: SM_COLMAX(1); break;
    case 2: SM_COLMAX(2); break;
    case 3: SM_COLMAX(3); break;
    default: SM_COLMAX(4); break;
  }
#undef SM_COLMAX
  return hipGetLastError();
}

hipError_t launch_first_fix_y(const DevPlan& p, int g0, int nsub, int max_npad, void* mats, int storage,
                              int64_t shadow_off, SubState* st, hipStream_t s) {
  if (nsub <= 0) return hipSuccess;
  const int64_t quads = (int64_t)max_npad * (max_npad / 4);
  const int spread = (int)std::min<int64_t>(64, std::max<int64_t>(1, quads / (256 * 16)));
#define SM_FIXY(K)                                                                                          \
  hipLaunchKernelGGL(first_fix_y_kernel<K>, dim3(nsub, spread), dim3(256), 0, s, p, g0, mats, shadow_off, st)
  switch (y_kind(storage)) {
    case 0: SM_FIXY(0); break;
    case 1: SM_FIXY(1); break;
    case 2: SM_FIXY(2); break;
    case 3: SM_FIXY(3); break;
    default: SM_FIXY(4); break;
  }
#undef SM_FIXY
  return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t* dst, int32_t value, int64_t count) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x)
    dst[k] = value;
}

hipError_t launch_fill_i32(int32_t* dst, int32_t value, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int grid = (int)((count + 255) / 256 < 1024 ? (count + 255) / 256 : 1024);
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid), dim3(256), 0, s, dst, value, count);
  return hipGetLastError();
}

}  // namespace sm
