// Row map of one block column of T_i = H[idx_i, idx_i] - mu I, shared by the
// kernels that read T_i straight from H's block-column panels.
#pragma once

#include "device_common.h"
#include "smsign_internal.h"

namespace sm {

// Row-map entries are panel rows of H (< 32768: sm_plan_create refuses taller
// panels), held as 16 bits so that four maps of the largest submatrices fit
// the LDS of a workgroup.
typedef int16_t RowSrc;

// LDS bytes of the atoms and row offsets of an index set of m atoms followed
// by `maps` row maps of n_pad entries, rounded up to 8 bytes.
__host__ __device__ inline size_t row_maps_bytes(int m, int maps, int npad) {
  return ((size_t)2 * m * sizeof(int) + (size_t)maps * npad * sizeof(RowSrc) + 7) & ~(size_t)7;
}

// For atom j of the index set (one block column of T_i): s_src[d] = the row
// of H's panel j that supplies row d of T_i, or -1 where the block (atom of
// row d, j) is not stored.  s_atom / s_off: the atoms of I_i (ascending) and
// their row offsets in T_i (m of them).  One wavefront builds the map; the
// caller orders it against the map's readers (wave_sync).
__device__ __forceinline__ void build_row_map(const DevPlan& p, int j, const int* s_atom, const int* s_off,
                                              int m, int n, RowSrc* s_src) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t kj0 = p.col_ptr[j];
  const int mj = (int)(p.col_ptr[j + 1] - kj0);
  for (int d = lane; d < n; d += kWave) s_src[d] = -1;
  wave_sync();
  for (int t = lane; t < mj; t += kWave) {
    const int k = p.row_idx[kj0 + t];
    int lo = 0, hi = m;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s_atom[mid] < k) lo = mid + 1; else hi = mid;
    }
    if (lo < m && s_atom[lo] == k) {
      const int dst = s_off[lo];
      const int src = p.blk_rowoff[kj0 + t];
      const int bk = p.bs[k];
      for (int q = 0; q < bk; ++q) s_src[dst + q] = (RowSrc)(src + q);
    }
  }
  wave_sync();
}

}  // namespace sm
