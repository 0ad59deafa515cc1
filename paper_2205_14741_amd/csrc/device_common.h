// Device helpers shared by the HIP kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/smsign.h"

namespace sm {

constexpr int kWave = 64;

// Butterfly reductions over one 64-lane wavefront.  The combination order is
// fixed, so results are bitwise reproducible.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, kWave));
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Orders the LDS accesses of one wavefront (lanes exchanging data through
// LDS without a workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Block-wide reduction through LDS; every thread gets the result.  The wave
// partials are combined in wave order.  `red` holds >= blockDim.x/64 doubles.
template <int OP>  // 0 sum, 1 max, 2 min
__device__ __forceinline__ double block_reduce(double v, double* red) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  const int nw = (blockDim.x + kWave - 1) / kWave;
  v = OP == 0 ? wave_sum(v) : OP == 1 ? wave_max(v) : wave_min(v);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double r = red[0];
  for (int w = 1; w < nw; ++w) r = OP == 0 ? r + red[w] : OP == 1 ? fmax(r, red[w]) : fmin(r, red[w]);
  __syncthreads();
  return r;
}

// Block matrix-vector products y_q = A v_q (q < Q) in float64 for a column-major
// n x n matrix A with leading dimension lda (a multiple of 32): each lane takes
// V consecutive rows of a column with one vector load (V = 4 float32 / 2
// float64 values for up to two vectors, fewer for more, so that the partial
// sums stay within 32 KiB of LDS for 8 waves), the block's waves split the
// columns (wave w: c = w, w + nw, ...) with eight columns in flight per lane;
// the wave partial sums are combined through LDS in wave order, so the result
// is deterministic.  v_q = v[q * vs + c].  For every row r < n, out(q, r,
// y_q[r]) is called by one thread of the block.  red: LDS scratch of
// matvec_red<Q, T>(waves) doubles.  Rows of a pass past n (up to the next
// multiple of V, always inside lda) are read and dropped.
template <int Q, typename T> struct MatvecShape {
  static constexpr int VT = 16 / (int)sizeof(T);
  static constexpr int VQ = Q <= 2 ? 4 : (Q <= 4 ? 2 : 1);
  static constexpr int V = VT < VQ ? VT : VQ;
  static constexpr int RW = kWave * V;   // rows per pass
};
template <int Q, typename T> constexpr int matvec_red(int waves) { return waves * Q * MatvecShape<Q, T>::RW; }

// Core of block_matvec over a loader: ld(c, rb, x) fills x[0 .. V) with the
// float64 values of rows rb .. rb + V - 1 of column c.
template <int Q, int V, typename Ld, typename Out>
__device__ __forceinline__ void block_matvec_ld(Ld ld, int n, const double* __restrict__ v, int vs,
                                                double* red, Out out) {
  constexpr int RW = kWave * V, U = 8;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  for (int r0 = 0; r0 < n; r0 += RW) {
    const int rb = r0 + lane * V;
    double acc[Q][V];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int e = 0; e < V; ++e) acc[q][e] = 0.0;
    if (rb < n) {
      int c = w;
      for (; c + (U - 1) * nw < n; c += U * nw) {
        double x[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) ld(c + u * nw, rb, x[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            const double vq = v[q * vs + c + u * nw];
#pragma unroll
            for (int e = 0; e < V; ++e) acc[q][e] += x[u][e] * vq;
          }
      }
      for (; c < n; c += nw) {
        double x[V];
        ld(c, rb, x);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const double vq = v[q * vs + c];
#pragma unroll
          for (int e = 0; e < V; ++e) acc[q][e] += x[e] * vq;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int e = 0; e < V; ++e) red[(w * Q + q) * RW + lane * V + e] = acc[q][e];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q)
      for (int rr = threadIdx.x; rr < RW; rr += blockDim.x)
        if (r0 + rr < n) {
          double s = 0.0;
          for (int k = 0; k < nw; ++k) s += red[(k * Q + q) * RW + rr];
          out(q, r0 + rr, s);
        }
    __syncthreads();
  }
}

template <int Q, typename T, typename Out>
__device__ __forceinline__ void block_matvec(const T* __restrict__ A, int64_t lda, int n,
                                             const double* __restrict__ v, int vs, double* red,
                                             Out out) {
  constexpr int V = MatvecShape<Q, T>::V;
  typedef T vec __attribute__((ext_vector_type(V)));
  block_matvec_ld<Q, V>(
      [&](int c, int rb, double (&x)[V]) {
        const vec t = *reinterpret_cast<const vec*>(A + (int64_t)c * lda + rb);
#pragma unroll
        for (int e = 0; e < V; ++e) x[e] = (double)t[e];
      },
      n, v, vs, red, out);
}

// float -> bfloat16 bits, round to nearest even: a plain conversion, which
// gfx950 executes as v_cvt_pk_bf16_f32.
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float x) {
  return __builtin_bit_cast(uint16_t, (__bf16)x);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}

__device__ __forceinline__ uint16_t f32_to_f16_bits(float x) {
  return __builtin_bit_cast(uint16_t, (_Float16)x);
}

// Operand copies of a float32 value for the matrix-core products (written by
// the producer of a buffer so the products read them without converting):
// SM_BF16 / SM_F16 keep one plane (the rounded value), SM_BF16X3 two planes,
// hi = bf16(x) and lo = bf16(x - hi), with x - hi exact in float32.
__device__ __forceinline__ uint16_t shadow_hi(float x, int kind) {
  return kind == SM_F16 ? f32_to_f16_bits(x) : f32_to_bf16_bits(x);
}
__device__ __forceinline__ uint16_t shadow_lo(float x, uint16_t hi) {
  return f32_to_bf16_bits(x - bf16_bits_to_f32(hi));
}

// Index (16-bit units) of element (row, col) of a column-major n_pad x n_pad
// matrix in its copy: one plane, col * n_pad + row; split bf16 keeps hi and
// lo of 32 consecutive rows side by side, col * 2 n_pad + (row / 32) * 64 +
// row % 32 (lo at + 32), so the hi and lo of a run of rows share one
// 128-byte line.  n_pad is a multiple of 32.
template <bool SPLIT>
__device__ __forceinline__ int64_t copy_idx(int64_t col, int row, int npad) {
  if (SPLIT) return col * 2 * npad + (int64_t)(row >> 5) * 64 + (row & 31);
  return col * npad + row;
}

// Value of a 16-bit copy entry of the precision `kind` (bf16 / f16).
__device__ __forceinline__ float copy_value(uint16_t b, int kind) {
  return kind == SM_F16 ? (float)__builtin_bit_cast(_Float16, b) : bf16_bits_to_f32(b);
}

// block_matvec over the 16-bit operand copies of a buffer (an entry is its
// bf16 / f16 copy, or hi + lo for split bf16; copy_idx layout).  Q <= 2.
// SPLIT: the copies are split-bf16 (hi and lo planes); a compile-time choice,
// so that the loads of all columns in flight are issued before any is used.
template <int Q, bool SPLIT, typename Out>
__device__ __forceinline__ void block_matvec_copies(const uint16_t* __restrict__ cp, int npad, int n, int kind,
                                                    const double* __restrict__ v, int vs, double* red,
                                                    Out out) {
  constexpr int V = MatvecShape<Q, float>::V;
  static_assert(V == 4, "four rows per lane: one 8-byte load per plane");
  typedef uint16_t h4 __attribute__((ext_vector_type(4)));
  block_matvec_ld<Q, V>(
      [&](int c, int rb, double (&x)[V]) {
        if constexpr (SPLIT) {
          const int64_t k = copy_idx<true>(c, rb, npad);
          const h4 hi = *reinterpret_cast<const h4*>(cp + k);
          const h4 lo = *reinterpret_cast<const h4*>(cp + k + 32);
#pragma unroll
          for (int e = 0; e < V; ++e) x[e] = (double)bf16_bits_to_f32(hi[e]) + (double)bf16_bits_to_f32(lo[e]);
        } else {
          const h4 hi = *reinterpret_cast<const h4*>(cp + copy_idx<false>(c, rb, npad));
#pragma unroll
          for (int e = 0; e < V; ++e) x[e] = (double)copy_value(hi[e], kind);
        }
      },
      n, v, vs, red, out);
}

// Deterministic probe-vector entry in {-1, +1} for (probe, row).
__device__ __forceinline__ double probe_entry(int probe, int row) {
  uint32_t h = (uint32_t)row * 0x9E3779B1u + (uint32_t)probe * 0x85EBCA77u + 0x165667B1u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return (h & 1u) ? 1.0 : -1.0;
}

}  // namespace sm
