// Step 2 of the submatrix method (Fig. 2 of the paper) on the matrix cores:
// sign(T_i) (Eq. 13) of every submatrix by the Newton-Schulz iteration
//     A = X^2,  Y = 3I - A,  X' = 1/2 X Y,
// all submatrices of a chunk in the same launches.  X, A, Y and X' are
// polynomials in the symmetric T_i, so they are symmetric: only tiles on or
// below the diagonal are computed and each is stored twice (as itself and as
// its transpose), which halves the MFMA work and keeps every iterate exactly
// symmetric.  A device scheduler (one workgroup) retires converged
// submatrices and builds the tile lists of the next launches.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"
#include "smsign_internal.h"

namespace sm {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------------------
// per-precision traits
//   S    storage type of the iterate in the workspace
//   L    LDS element type
//   K    k-depth of one LDS stage
//   KP   LDS row padding (elements) against bank conflicts
// ---------------------------------------------------------------------------
template <int MODE> struct Traits;
template <> struct Traits<SM_F64> { using S = double; using L = double; static constexpr int K = 16, KP = 2; using Acc = d4; };
template <> struct Traits<SM_F32> { using S = float; using L = float; static constexpr int K = 32, KP = 4; using Acc = f4; };
template <> struct Traits<SM_BF16> { using S = float; using L = uint16_t; static constexpr int K = 64, KP = 8; using Acc = f4; };
template <> struct Traits<SM_F16> { using S = float; using L = _Float16; static constexpr int K = 64, KP = 8; using Acc = f4; };
template <> struct Traits<SM_BF16X3> { using S = float; using L = uint16_t; static constexpr int K = 64, KP = 8; using Acc = f4; };

constexpr int kBlock = 256;   // 4 waves in a 2 x 2 arrangement, 32 x 32 outputs each

// NL consecutive elements of one operand column as 16-byte vector loads
// (zeros for a row past n_pad).  The address is 16-byte aligned: n_pad and
// the per-thread k offset are multiples of 4 doubles / 8 floats.
template <typename S, int NL>
__device__ __forceinline__ void load_col(S (&r)[NL], const S* __restrict__ p, bool ok) {
  constexpr int V = 16 / (int)sizeof(S);
  static_assert(NL % V == 0, "vector width");
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  if (ok) {
#pragma unroll
    for (int q = 0; q < NL / V; ++q) {
      const u4 t = *reinterpret_cast<const u4*>(p + q * V);
      __builtin_memcpy(&r[q * V], &t, 16);
    }
  } else {
#pragma unroll
    for (int e = 0; e < NL; ++e) r[e] = S(0);
  }
}

// ---------------------------------------------------------------------------
// Operand sources.  float64 / float32 products read the iterate's own buffer.
// The bf16 / f16 / split-bf16 products read the 16-bit copies that the
// producer of the buffer wrote next to it (at float offset shadow_off): one
// plane of n_pad^2 values, or for split bf16 the hi plane followed by the lo
// plane.  Staging them is then a plain copy into LDS, with half the bytes of
// the float32 buffer for bf16 / f16, and no per-tile conversion work.
// ---------------------------------------------------------------------------
template <int MODE> struct Pre {
  static constexpr bool value = MODE == SM_BF16 || MODE == SM_F16 || MODE == SM_BF16X3;
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int MODE, bool PRE = Pre<MODE>::value> struct Operand;

// Operand panel row `row` of a buffer, the thread's k slice starting at
// `part` within each stage.
template <int MODE> struct Operand<MODE, false> {
  using S = typename Traits<MODE>::S;
  const S* p;
  __device__ Operand(const S* buf, int64_t, int row, int part, int npad)
      : p(buf + (int64_t)row * npad + part) {}
  template <int K, int NL>
  __device__ __forceinline__ void load(S (&r)[NL], int stage, bool ok) const {
    load_col<S, NL>(r, p + (int64_t)stage * K, ok);
  }
};

template <int MODE> struct Operand<MODE, true> {
  static constexpr bool SPLIT = MODE == SM_BF16X3;
  const uint16_t* p;
  int part;
  __device__ Operand(const float* buf, int64_t shadow_off, int row, int part_, int npad)
      : p(reinterpret_cast<const uint16_t*>(buf + shadow_off) + (int64_t)row * (SPLIT ? 2 * npad : npad)),
        part(part_) {}
  // NL 16-bit values per plane (NL / 2 words), hi then lo in r
  template <int K, int NL, int RN>
  __device__ __forceinline__ void load(uint32_t (&r)[RN], int stage, bool ok) const {
    constexpr int NW = NL / 2;
    static_assert(RN % NW == 0 && NW % 4 == 0 && NL <= 32, "operand register layout");
    const int k0 = stage * K + part;
    const uint16_t* src = p + (SPLIT ? (k0 >> 5) * 64 + (k0 & 31) : k0);
#pragma unroll
    for (int q = 0; q < RN / NW; ++q) {
#pragma unroll
      for (int v = 0; v < NW / 4; ++v) {
        u32x4 t = u32x4{0, 0, 0, 0};
        if (ok) t = *reinterpret_cast<const u32x4*>(src + 32 * q + 8 * v);
#pragma unroll
        for (int e = 0; e < 4; ++e) r[q * NW + 4 * v + e] = t[e];
      }
    }
  }
};

// registers -> LDS rows of one stage (hi / only plane to `dst`, lo to `dst_lo`)
template <int MODE, int NL, typename RT, int RN, typename LT>
__device__ __forceinline__ void stage_store(const RT (&r)[RN], LT* dst, LT* dst_lo) {
  if constexpr (!Pre<MODE>::value) {
#pragma unroll
    for (int e = 0; e < NL; ++e) dst[e] = r[e];
  } else {
    constexpr int NW = NL / 2;
#pragma unroll
    for (int q = 0; q < RN / NW; ++q) {
      u32x4* d = reinterpret_cast<u32x4*>(q == 0 ? dst : dst_lo);
#pragma unroll
      for (int v = 0; v < NW / 4; ++v)
        d[v] = u32x4{r[q * NW + 4 * v], r[q * NW + 4 * v + 1], r[q * NW + 4 * v + 2], r[q * NW + 4 * v + 3]};
    }
  }
}

// Epilogue of a float32-accumulating product for one lane's four results
// (rows rb .. rb + 3 of column cc): entries on or below the diagonal are
// written to (r, c) and mirrored to (c, r); for the square, Y = 3I - alpha^2 A
// is stored and (A - I)^2 is added to the residual partial sum; the update
// stores 1/2 alpha X Y (alpha = 1: plain Newton-Schulz).  Products of the
// low-precision main phases store only the 16-bit copies their consumers read
// (the float32 value is rebuilt where a refinement step or the final
// read-out needs it); float32 products store float32.
template <int MODE, int WHICH>
__device__ __forceinline__ void store_quad(const f4& a4, float* Out, int64_t shadow_off, int64_t nn,
                                           int npad, int rb, int cc, double alpha, double rscale,
                                           double& part, bool tri = true) {
  constexpr bool PRE = Pre<MODE>::value;
  float o[4];
  uint16_t h[4], l[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int rr = rb + v;
    const double a = (double)a4[v];
    if (WHICH == 0) {
      const double dg = (rr == cc) ? 1.0 : 0.0;
      const double e = a * rscale - dg;
      if (!tri) part += e * e;   // slab: every entry once
      else if (rr >= cc) part += (rr == cc) ? e * e : 2.0 * e * e;
      o[v] = (float)(3.0 * dg - (alpha * alpha) * a);
    } else {
      o[v] = (float)((0.5 * alpha) * a);
    }
    if constexpr (PRE) {
      h[v] = shadow_hi(o[v], MODE);
      l[v] = MODE == SM_BF16X3 ? shadow_lo(o[v], h[v]) : 0;
    }
  }
  constexpr bool SPLIT = MODE == SM_BF16X3;
  uint16_t* sh = PRE ? reinterpret_cast<uint16_t*>(Out + shadow_off) : nullptr;
  const int64_t dcol = (int64_t)cc * npad + rb;     // (rb .. rb + 3, cc): contiguous
  const int64_t dcp = copy_idx<SPLIT>(cc, rb, npad);
  // tri: keep the lower triangle and write its mirror image; otherwise (a
  // slab tile of a last refinement update) write all four as they are
  if (!tri || rb >= cc) {
    if constexpr (PRE) {
      typedef uint32_t u2 __attribute__((ext_vector_type(2)));
      *reinterpret_cast<u2*>(sh + dcp) = u2{h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16)};
      if (SPLIT)
        *reinterpret_cast<u2*>(sh + dcp + 32) = u2{l[0] | ((uint32_t)l[1] << 16), l[2] | ((uint32_t)l[3] << 16)};
    } else {
      *reinterpret_cast<f4*>(Out + dcol) = f4{o[0], o[1], o[2], o[3]};
    }
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (rb + v >= cc) {
        if constexpr (PRE) {
          sh[dcp + v] = h[v];
          if (SPLIT) sh[dcp + 32 + v] = l[v];
        } else {
          Out[dcol + v] = o[v];
        }
      }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
    if (tri && rb + v > cc) {
      if constexpr (PRE) {
        const int64_t m = copy_idx<SPLIT>(rb + v, cc, npad);
        sh[m] = h[v];
        if (SPLIT) sh[m + 32] = l[v];
      } else {
        Out[(int64_t)(rb + v) * npad + cc] = o[v];
      }
    }
}

// 16 consecutive rows (row0 .. row0 + 15, row0 % 16 == 0) of column col of
// a product's result: float32 values, or their 16-bit copies for the
// low-precision main phases.
template <int MODE>
__device__ __forceinline__ void store_run16(const float (&w)[16], float* Out, int64_t shadow_off, int col,
                                            int row0, int npad) {
  if constexpr (!Pre<MODE>::value) {
    f4* d = reinterpret_cast<f4*>(Out + (int64_t)col * npad + row0);
#pragma unroll
    for (int q = 0; q < 4; ++q) d[q] = f4{w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]};
  } else {
    constexpr bool SPLIT = MODE == SM_BF16X3;
    uint16_t* sh = reinterpret_cast<uint16_t*>(Out + shadow_off) + copy_idx<SPLIT>(col, row0, npad);
    uint32_t hw[8], lw[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const uint16_t h0 = shadow_hi(w[2 * q], MODE), h1 = shadow_hi(w[2 * q + 1], MODE);
      hw[q] = h0 | ((uint32_t)h1 << 16);
      if (SPLIT) lw[q] = shadow_lo(w[2 * q], h0) | ((uint32_t)shadow_lo(w[2 * q + 1], h1) << 16);
    }
    u32x4* dh = reinterpret_cast<u32x4*>(sh);
    dh[0] = u32x4{hw[0], hw[1], hw[2], hw[3]};
    dh[1] = u32x4{hw[4], hw[5], hw[6], hw[7]};
    if (SPLIT) {
      u32x4* dl = reinterpret_cast<u32x4*>(sh + 32);
      dl[0] = u32x4{lw[0], lw[1], lw[2], lw[3]};
      dl[1] = u32x4{lw[4], lw[5], lw[6], lw[7]};
    }
  }
}

// Operand sources of a tile (rows of X for the tile's rows, rows of R = X or
// Y for its columns; by symmetry these are the columns the product needs).
// TE: tile edge.  Rows past n_pad load as zeros.
template <int MODE> struct TileSrc {
  Operand<MODE> a, b;
  bool va, vb;
};

template <int MODE, int WHICH, int TE>
__device__ __forceinline__ TileSrc<MODE> tile_src(const TileRec& rec, typename Traits<MODE>::S* mats,
                                                  int64_t shadow_off, int lrow, int lpart) {
  using S = typename Traits<MODE>::S;
  const int npad = rec.npad;
  const int64_t nn = (int64_t)npad * npad;
  const S* base = mats + rec.mat_off;
  const S* Xp = base + (int64_t)((WHICH == 0 ? rec.it : rec.it + 1) & 1) * nn;
  const S* Rp = WHICH == 0 ? Xp : base + 2 * nn;
  const int r0 = (rec.bibj >> 16) * TE, c0 = (rec.bibj & 0xFFFF) * TE;
  const bool va = (r0 + lrow) < npad;
  const bool vb = (c0 + lrow) < npad;
  return TileSrc<MODE>{Operand<MODE>(Xp, shadow_off, va ? r0 + lrow : 0, lpart, npad),
                       Operand<MODE>(Rp, shadow_off, vb ? c0 + lrow : 0, lpart, npad), va, vb};
}

__device__ __forceinline__ void tile_coords(int lt, int& bi, int& bj) {
  int r = (int)((sqrtf(8.0f * (float)lt + 1.0f) - 1.0f) * 0.5f);
  while (r * (r + 1) / 2 > lt) --r;
  while ((r + 1) * (r + 2) / 2 <= lt) ++r;
  bi = r;
  bj = lt - r * (r + 1) / 2;
}

// WHICH = 0: A = X^2 -> Y = 3I - A, residual partial sum (A - I)^2 per tile.
// WHICH = 1: X' = 1/2 X Y.
// C[r][c] = sum_k L[k][r] R[k][c] with L = X and R = X or Y stored column-major;
// by symmetry L[k][r] = X[r][k], so C = X R.  Both operand panels are read as
// columns (contiguous k), i.e. LDS rows hold one output row's k-slab.
// KDIV: the LDS stage holds K / KDIV of the k range (KDIV = 2 halves the LDS
// footprint, so more workgroups fit on a compute unit, at twice the barriers).
// XCD: workgroups are dealt to the 8 XCDs round-robin (workgroup b on XCD
// b % 8), each with its own L2.  With XCD set, the workgroups of XCD x walk
// the x-th contiguous eighth of the tile list, so all tiles of a submatrix
// (adjacent in the list) share one L2 instead of pulling its operands into
// all eight.
constexpr int kXcds = 8;

// Updates walk their share of the tile list backwards (t -> mirror - t over
// [t_lo, t_end)): a square launch walks the submatrices forward, so the
// update after it starts on the ones the square wrote last, the likeliest to
// still sit in the memory-side cache, and the next square, forward again,
// starts on the ones the update wrote last.  mirror < 0: forward.
__device__ __forceinline__ int rec_index(int t, int mirror) { return mirror < 0 ? t : mirror - t; }

// Workgroups of the 64-tile kernel that its LDS stages leave room for on a
// compute unit (160 KiB), at most 4.  Each workgroup puts one wave on every
// SIMD, so this is also the number of waves per SIMD the register budget is
// held to (4: at most 128 registers per lane).
// Stage rows are padded by KP elements against LDS bank conflicts (an
// unpadded, XOR-swizzled layout measured the same).  The array also has to
// hold the 16-bit epilogue's result staging (4 waves x 32 x kStageStride
// floats) and the four residual slots.
constexpr int kStageStride = 36;   // floats per staged column: 16-byte aligned runs of 4 rows
template <int MODE, int KDIV> struct GemmOcc {
  using Tr = Traits<MODE>;
  static constexpr bool PRE = Pre<MODE>::value;
  static constexpr int NOP = MODE == SM_BF16X3 ? 4 : 2;
  static constexpr int LD = Tr::K / KDIV + Tr::KP;
  static constexpr int kStageBytes = NOP * 64 * LD * (int)sizeof(typename Tr::L);   // one buffer
  static constexpr int kStaged = PRE ? 4 * 32 * kStageStride * 4 : 0;
  static constexpr int kNeed = kStaged + 4 * 8;
  static constexpr int kLds = 2 * kStageBytes > kNeed ? 2 * kStageBytes : kNeed;
  static constexpr int by_lds = 160 * 1024 / kLds;
  static constexpr int value = by_lds < 4 ? by_lds : 4;
};

template <int MODE, int WHICH, int KDIV, bool XCD>
__global__ __launch_bounds__(kBlock, (GemmOcc<MODE, KDIV>::value)) void ns_gemm_kernel(typename Traits<MODE>::S* __restrict__ mats,
                                                         int64_t shadow_off,
                                                         const int32_t* __restrict__ count,
                                                         const TileRec* __restrict__ recs,
                                                         double* __restrict__ partials) {
  using Tr = Traits<MODE>;
  using S = typename Tr::S;
  using LT = typename Tr::L;
  using Occ = GemmOcc<MODE, KDIV>;
  constexpr int K = Tr::K / KDIV;
  constexpr int LD = Occ::LD;
  constexpr int NL = K / 4;              // elements per thread per operand per stage
  constexpr int KK = K / 4;              // k values per lane and stage (float64 / float32)
  constexpr bool SPLIT = (MODE == SM_BF16X3);
  constexpr bool PRE = Pre<MODE>::value;
  constexpr int NPL = SPLIT ? 2 : 1;     // operand planes (hi, lo)
  constexpr int NOP = 2 * NPL;           // A, B (+ A_lo, B_lo)
  using RT = typename std::conditional<PRE, uint32_t, S>::type;
  constexpr int RN = PRE ? NPL * NL / 2 : NL;   // registers per operand per stage
  __shared__ __attribute__((aligned(16))) char lds_bytes[Occ::kLds];
  LT (*lds)[NOP][64 * LD] = reinterpret_cast<LT (*)[NOP][64 * LD]>(lds_bytes);
  // element offset of 16-byte chunk c of stage row r (16-bit stages)
  auto chunk_at = [](int r, int c) { return r * LD + 8 * c; };

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lrow = tid >> 2;             // 0..63: row of the operand panel this thread loads
  const int lpart = (tid & 3) * NL;      // k offset inside the stage
  const int total = count[0];

  int t_begin = blockIdx.x, t_end = total, t_step = gridDim.x, t_lo = 0;
  if (XCD) {
    const int x = blockIdx.x % kXcds;
    t_step = ((int)gridDim.x - x + kXcds - 1) / kXcds;   // workgroups on XCD x
    t_lo = (int)((int64_t)total * x / kXcds);
    t_begin = t_lo + (int)blockIdx.x / kXcds;
    t_end = (int)((int64_t)total * (x + 1) / kXcds);
  }
  const int t_mirror = WHICH == 1 ? t_lo + t_end - 1 : -1;
  // Operand registers carry over from tile to tile: during the last stage of
  // a tile the first stage of the workgroup's next tile is loaded, so a tile
  // starts without waiting for memory.
  RT ra[RN], rb[RN];
  TileRec nxt;
  if (t_begin < t_end) {
    nxt = recs[rec_index(t_begin, t_mirror)];
    const TileSrc<MODE> s0 = tile_src<MODE, WHICH, 64>(nxt, mats, shadow_off, lrow, lpart);
    s0.a.template load<K, NL>(ra, 0, s0.va);
    s0.b.template load<K, NL>(rb, 0, s0.vb);
  }
  for (int t = t_begin; t < t_end; t += t_step) {
    const TileRec rec = nxt;
    const bool has_next = t + t_step < t_end;
    if (has_next) nxt = recs[rec_index(t + t_step, t_mirror)];   // the next tile's record, used at the last stage
    const int npad = rec.npad;
    const int64_t nn = (int64_t)npad * npad;
    const double alpha = (double)rec.alpha;
    const double rscale = (double)rec.rscale;
    S* base = mats + rec.mat_off;
    S* Out = base + (WHICH == 0 ? 2 * nn : (int64_t)(rec.it & 1) * nn);
    const int bi = rec.bibj >> 16, bj = rec.bibj & 0xFFFF;
    const int r0 = bi * 64, c0 = bj * 64;
    // the last tile row / column may reach past n_pad (a multiple of 32): its
    // operand rows load as zeros and the wave blocks there are skipped;
    // the block of a diagonal tile that lies wholly above the diagonal
    // computes nothing either
    const bool slab = (rec.flags & kTileSlab) != 0;   // all blocks, no mirror
    const bool wvalid = (r0 + wm * 32 < npad) && (c0 + wn * 32 < npad) &&
                        (slab ? (rec.flags & (kTileSlabWave << wn)) != 0 : !(bi == bj && wm < wn));
    const TileSrc<MODE> src = tile_src<MODE, WHICH, 64>(rec, mats, shadow_off, lrow, lpart);

    typename Tr::Acc acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = typename Tr::Acc{0, 0, 0, 0};

    // the next stage's operands are loaded into registers while the MFMAs
    // work on the current LDS stage
    const int nst = npad / K;
    auto k_loop = [&](auto compute_tag) {
    constexpr bool COMPUTE = decltype(compute_tag)::value;
    for (int s = 0; s < nst; ++s) {
      const int buf = s & 1;
      // ---- registers -> LDS ----
      if constexpr (PRE) {   // 16-byte chunks, hi (and lo) planes
        constexpr int NW = NL / 2;
#pragma unroll
        for (int q = 0; q < NPL; ++q)
#pragma unroll
          for (int c = 0; c < NL / 8; ++c) {
            const int at = chunk_at(lrow, lpart / 8 + c);
            *reinterpret_cast<u32x4*>(&lds[buf][q == 0 ? 0 : NOP - 2][at]) =
                u32x4{ra[q * NW + 4 * c], ra[q * NW + 4 * c + 1], ra[q * NW + 4 * c + 2], ra[q * NW + 4 * c + 3]};
            *reinterpret_cast<u32x4*>(&lds[buf][q == 0 ? 1 : NOP - 1][at]) =
                u32x4{rb[q * NW + 4 * c], rb[q * NW + 4 * c + 1], rb[q * NW + 4 * c + 2], rb[q * NW + 4 * c + 3]};
          }
      } else {
        stage_store<MODE, NL>(ra, &lds[buf][0][lrow * LD + lpart], &lds[buf][NOP - 2][lrow * LD + lpart]);
        stage_store<MODE, NL>(rb, &lds[buf][1][lrow * LD + lpart], &lds[buf][NOP - 1][lrow * LD + lpart]);
      }
      __syncthreads();
      // ---- prefetch the next stage (or the next tile's first) ----
      if (s + 1 < nst) {
        src.a.template load<K, NL>(ra, s + 1, src.va);
        src.b.template load<K, NL>(rb, s + 1, src.vb);
      } else if (has_next) {
        const TileSrc<MODE> sn = tile_src<MODE, WHICH, 64>(nxt, mats, shadow_off, lrow, lpart);
        sn.a.template load<K, NL>(ra, 0, sn.va);
        sn.b.template load<K, NL>(rb, 0, sn.vb);
      }
      // ---- MFMA on the LDS stage ----
      const int kq = lane >> 4;    // k group of this lane
      const int rl = lane & 15;    // row / column inside a 16 x 16 block
      if constexpr (!COMPUTE) {
        // wave block past n_pad (or above the diagonal): nothing to accumulate
      } else if constexpr (MODE == SM_F64) {
        // 16x16x4: lane supplies A[rl][kq], B[kq][rl]; the k index inside the
        // stage is permuted to KK kq + kk so each lane reads KK contiguous values.
        double a[2][KK], b[2][KK];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int kk = 0; kk < KK; ++kk) {
            a[x][kk] = lds[buf][0][(wm * 32 + x * 16 + rl) * LD + KK * kq + kk];
            b[x][kk] = lds[buf][1][(wn * 32 + x * 16 + rl) * LD + KK * kq + kk];
          }
#pragma unroll
        for (int kk = 0; kk < KK; ++kk)
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
              acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x][kk], b[y][kk], acc[x][y], 0, 0, 0);
      } else if constexpr (MODE == SM_F32) {
        float a[2][KK], b[2][KK];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int kk = 0; kk < KK; ++kk) {
            a[x][kk] = lds[buf][0][(wm * 32 + x * 16 + rl) * LD + KK * kq + kk];
            b[x][kk] = lds[buf][1][(wn * 32 + x * 16 + rl) * LD + KK * kq + kk];
          }
#pragma unroll
        for (int kk = 0; kk < KK; ++kk)
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
              acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x][kk], b[y][kk], acc[x][y], 0, 0, 0);
      } else {
        // 16x16x32: lane supplies A[rl][8 kq .. 8 kq + 7], B[8 kq .. 8 kq + 7][rl]
#pragma unroll
        for (int kh = 0; kh < K / 32; ++kh) {
          const int ko = kh * 32 + 8 * kq;
          if constexpr (MODE == SM_F16) {
            f16x8 a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
              a[x] = *reinterpret_cast<const f16x8*>(&lds[buf][0][chunk_at(wm * 32 + x * 16 + rl, ko / 8)]);
              b[x] = *reinterpret_cast<const f16x8*>(&lds[buf][1][chunk_at(wn * 32 + x * 16 + rl, ko / 8)]);
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
              for (int y = 0; y < 2; ++y)
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[x], b[y], acc[x][y], 0, 0, 0);
          } else {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
              a[x] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&lds[buf][0][chunk_at(wm * 32 + x * 16 + rl, ko / 8)]));
              b[x] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&lds[buf][1][chunk_at(wn * 32 + x * 16 + rl, ko / 8)]));
            }
            if constexpr (SPLIT) {
              bf16x8 al[2], bl[2];
#pragma unroll
              for (int x = 0; x < 2; ++x) {
                al[x] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&lds[buf][2][chunk_at(wm * 32 + x * 16 + rl, ko / 8)]));
                bl[x] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&lds[buf][3][chunk_at(wn * 32 + x * 16 + rl, ko / 8)]));
              }
#pragma unroll
              for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                  acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[x], b[y], acc[x][y], 0, 0, 0);
                  acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], bl[y], acc[x][y], 0, 0, 0);
                  acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], b[y], acc[x][y], 0, 0, 0);
                }
            } else {
#pragma unroll
              for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                  acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], b[y], acc[x][y], 0, 0, 0);
            }
          }
        }
      }
    }
    };
    if (wvalid) k_loop(std::true_type{}); else k_loop(std::false_type{});

    // ---- epilogue: 16 x 16 result block.  Register v of lane l holds column
    // l % 16 and row 4 (l / 16) + v for the float32-accumulating instructions,
    // row l / 16 + 4 v for the float64 one (checked by sm_selftest_mfma).
    // Only entries on or below the diagonal are kept and each is written to
    // both (r, c) and (c, r): the stored result is exactly symmetric.  This
    // matters because the kernels read X as X^T: a skew-symmetric part would
    // be multiplied by -2 in every iteration instead of being left alone. ----
    double part = 0.0;
    const int kq = lane >> 4;
    // the four wave sums of the residual meet in the stage buffer the last
    // stage did not use (past the result staging of the 16-bit epilogue)
    constexpr size_t kStageB = Occ::kStageBytes;
    constexpr int SS = kStageStride;
    constexpr size_t kStaged = Occ::kStaged;
    constexpr bool kIdleFits = kStageB >= kStaged + 4 * sizeof(double);
    static_assert((size_t)Occ::kLds >= kStaged + 4 * sizeof(double), "residual slots");
    double* red = reinterpret_cast<double*>(
        kIdleFits ? reinterpret_cast<char*>(&lds[nst & 1][0][0]) + kStaged
                  : reinterpret_cast<char*>(&lds[0][0][0]) + kStaged);
    if constexpr (MODE == SM_F64) {
#pragma unroll
      for (int x = 0; x < (wvalid ? 2 : 0); ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const int rb = r0 + wm * 32 + x * 16;
          const int cc = c0 + wn * 32 + y * 16 + (lane & 15);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int rr = rb + kq + 4 * v;
            if (!slab && rr < cc) continue;   // upper triangle: written by the mirror of (cc, rr)
            const double a = acc[x][y][v];
            double outv;
            if (WHICH == 0) {
              const double dg = (rr == cc) ? 1.0 : 0.0;
              const double e = a * rscale - dg;
              part += (slab || rr == cc) ? e * e : 2.0 * e * e;
              outv = 3.0 * dg - (alpha * alpha) * a;
            } else {
              outv = (0.5 * alpha) * a;
            }
            Out[(int64_t)cc * npad + rr] = outv;
            if (!slab && rr != cc) Out[(int64_t)rr * npad + cc] = outv;
          }
        }
    } else if constexpr (!Pre<MODE>::value) {
#pragma unroll
      for (int x = 0; x < (wvalid ? 2 : 0); ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          store_quad<MODE, WHICH>(acc[x][y], Out, shadow_off, nn, npad, r0 + wm * 32 + x * 16 + 4 * kq,
                                  c0 + wn * 32 + y * 16 + (lane & 15), alpha, rscale, part, !slab);
    } else {
      // 16-bit copies: each wave stages its 32 x 32 result block in LDS,
      // then writes it, and its mirror image, as runs of 16 rows per lane
      // (contiguous 16-byte stores instead of scattered 2-byte ones).  The stage buffer the last stage
      // did not use is free; with half-depth stages one buffer is too small
      // and the whole array is used after a barrier.
      float* stg;
      if constexpr (kIdleFits) {
        stg = reinterpret_cast<float*>(&lds[nst & 1][0][0]);
      } else {
        __syncthreads();
        stg = reinterpret_cast<float*>(&lds[0][0][0]);
      }
      float* my = stg + wid * (32 * SS);
      if (wvalid) {
        const int R0 = r0 + wm * 32, C0 = c0 + wn * 32;
        const float a2 = (float)(alpha * alpha), ha = (float)(0.5 * alpha), rsf = (float)rscale;
        // staging: my[lc * SS + lr]; a lane's four rows of a column are one
        // 16-byte store
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) {
            const int lc = y * 16 + (lane & 15);
            float o[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int lr = x * 16 + 4 * kq + v;
              const float a = acc[x][y][v];
              if (WHICH == 0) {
                const float dg = (R0 + lr == C0 + lc) ? 1.0f : 0.0f;
                const float e = a * rsf - dg;   // exact for rsf = 1: a ~ 1 on the diagonal
                if (R0 + lr >= C0 + lc) part += (double)(e * e) * (R0 + lr == C0 + lc ? 1.0 : 2.0);
                o[v] = __builtin_fmaf(-a2, a, 3.0f * dg);
              } else {
                o[v] = ha * a;
              }
            }
            *reinterpret_cast<f4*>(&my[lc * SS + x * 16 + 4 * kq]) = f4{o[0], o[1], o[2], o[3]};
          }
        wave_sync();
        const int li = lane >> 1, h = (lane & 1) * 16;
        const bool diag = R0 == C0;
        float w[16];
        // the block, column C0 + li, rows R0 + h .. (four 16-byte loads); on
        // a diagonal block the entries above the diagonal take the value of
        // their mirror
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const f4 t = *reinterpret_cast<const f4*>(&my[li * SS + h + 4 * q]);
#pragma unroll
          for (int e = 0; e < 4; ++e) w[4 * q + e] = t[e];
        }
        if (diag)
#pragma unroll
          for (int j = 0; j < 16; ++j)
            if (h + j < li) w[j] = my[(h + j) * SS + li];
        const bool f32out = WHICH == 1 && (rec.flags & kTileStoreF32);
        auto put16 = [&](int col, int row0) {
          if (f32out) store_run16<SM_F32>(w, Out, shadow_off, col, row0, npad);
          else store_run16<MODE>(w, Out, shadow_off, col, row0, npad);
        };
        put16(C0 + li, R0 + h);
        if (!diag) {   // the mirror: column R0 + li, rows C0 + h ..
#pragma unroll
          for (int j = 0; j < 16; ++j) w[j] = my[(h + j) * SS + li];
          put16(R0 + li, C0 + h);
        }
      }
    }
    if (WHICH == 0) {
      part = wave_sum(part);
      if (lane == 0) red[wid] = part;
      __syncthreads();
      if (tid == 0) {
        const double sum = ((red[0] + red[1]) + red[2]) + red[3];
        partials[rec.part_idx] = sum;
      }
    }
    __syncthreads();
  }
}

// The tile records of one listed submatrix in list L (0 / 1: updates, main /
// refinement precision; 2 / 3: squares of the next iteration): the tile
// walk of every GEMM reads its tile's buffers, scale and flags from these.
struct SubTiles {
  int64_t mo;
  float alpha, rscale;
  int npad, it, f, nt, po, t64;
  int T, c0;      // slab: tile rows, first tile column
  int loc, b;     // slab: the atom's columns loc .. loc + b - 1
  int16_t flags;
};

__device__ __forceinline__ SubTiles sub_tiles(const DevPlan& p, int g, int L, int tshift, int iters, int phase,
                                              double alpha_sq, double alpha_upd, double x0s_in, bool slab) {
  const int which = L < 2 ? 1 : 0;
  SubTiles t;
  t.npad = p.npad_g[g];
  const int T = (t.npad + (1 << tshift) - 1) >> tshift;
  t.f = 1 << (tshift - 6);
  t.nt = T * (T + 1) / 2;
  t.T = T;
  t.c0 = 0;
  t.loc = 0;
  t.b = 0;
  if (slab) {
    const int i = p.order_g[g];
    t.loc = p.loc[i];
    t.b = p.bs[i];
    t.nt = slab_tiles(t.npad, t.loc, t.b, tshift);
    t.c0 = t.loc >> tshift;
  }
  t.mo = p.mat_off_g[g];
  t.it = iters;
  // products that read X_0 (the square at it = 0, the update producing X_1)
  // apply its factor x0s to the buffer's contents
  const bool reads_x0 = which == 0 ? iters == 0 : iters == 1;
  const double x0s = reads_x0 ? x0s_in : 1.0;
  t.alpha = (float)((which == 0 ? alpha_sq : alpha_upd) * x0s);
  t.rscale = (float)(which == 0 ? x0s * x0s : 1.0);
  // list 0 also holds first refinement updates (phase 1): their result is
  // stored in float32 for the refinement steps that follow
  t.flags = (L == 0 && phase == 1) ? kTileStoreF32 : 0;
  if (slab) t.flags |= kTileSlab;
  t.po = p.tile_off_g[g];
  t.t64 = tiles_of(t.npad);
  return t;
}

__device__ __forceinline__ TileRec tile_rec(const SubTiles& t, int lt) {
  int bi, bj;
  if (t.flags & kTileSlab) {   // tile column by tile column, all tile rows
    bi = lt % t.T;
    bj = t.c0 + lt / t.T;
  } else {
    tile_coords(lt, bi, bj);
  }
  const int b64i = bi * t.f, b64j = bj * t.f;
  TileRec r;
  r.mat_off = t.mo;
  r.alpha = t.alpha;
  r.rscale = t.rscale;
  r.bibj = (bi << 16) | bj;
  r.npad = t.npad;
  r.it = t.it;
  // a slab square's tiles (fewer than the triangle's) take slots 0, 1, ...
  r.part_idx = (t.flags & kTileSlab) ? t.po + lt : t.po + b64i * (b64i + 1) / 2 + b64j;
  r.tiles64 = (int16_t)t.t64;
  r.flags = t.flags;
  if (t.flags & kTileSlab) {   // wave-block columns that hold atom columns
    const int wcol = 32 * t.f;     // wave-block width: half the tile
    const int cfirst = bj * 2 * wcol;
#pragma unroll
    for (int wn = 0; wn < 2; ++wn) {
      const int lo = cfirst + wn * wcol, hi = lo + wcol;
      if (lo < t.loc + t.b && hi > t.loc) r.flags |= (int16_t)(kTileSlabWave << wn);
    }
  }
  return r;
}

// Tile records of every list the scheduler just built, in one launch: one
// workgroup per (listed submatrix, list).  blockIdx.y picks the list: 0
// updates (main precision), 1 squares of the next iteration (main), 2 / 3 the
// same in the refinement precision.  List L's records go to recs + L *
// max_tiles.  Tiles have edge 1 << tshift (64 or 128); residual partial slots
// are always those of the 64-tiles.
__global__ __launch_bounds__(256) void expand_kernel(DevPlan p, int g0, const SubState* __restrict__ st,
                                                     const int32_t* __restrict__ lists, int max_subs,
                                                     TileRec* __restrict__ recs, int64_t max_tiles,
                                                     int tshift_main, int tshift_ref) {
  const int stride = 2 + 2 * max_subs + 1;
  const int y = blockIdx.y;
  const int L = (y & 1) ? 2 + (y >> 1) : (y >> 1);   // 0, 2, 1, 3
  const int32_t* Lb = lists + L * stride;
  TileRec* out = recs + L * max_tiles;
  const int a = blockIdx.x;
  if (a >= Lb[1]) return;
  const int l = Lb[2 + a];
  const int first = Lb[2 + max_subs + a];
  const SubState& s = st[l];
  const SubTiles t = sub_tiles(p, g0 + l, L, (L & 1) ? tshift_ref : tshift_main, s.iters, s.phase, s.alpha_sq,
                               s.alpha_upd, s.x0s, (L == 1 && s.last_slab) || (L == 3 && s.sq_slab));
  for (int lt = threadIdx.x; lt < t.nt; lt += blockDim.x) out[first + lt] = tile_rec(t, lt);
}

hipError_t launch_expand(const DevPlan& p, int g0, const SubState* st, const int32_t* lists, int max_subs,
                         TileRec* recs, int64_t max_tiles, int tshift_main, int tshift_ref, bool with_ref,
                         int grid_subs, hipStream_t s) {
  if (grid_subs <= 0) return hipSuccess;
  hipLaunchKernelGGL(expand_kernel, dim3(grid_subs, with_ref ? 4 : 2), dim3(256), 0, s, p, g0, st, lists,
                     max_subs, recs, max_tiles, tshift_main, tshift_ref);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 128 x 128 output tiles for large submatrices (float32 accumulation only):
// 4 waves in 2 x 2, 64 x 64 outputs each (4 x 4 MFMA blocks of 16 x 16), half
// the operand traffic per flop of the 64 x 64 tiles.  n_pad must be a multiple
// of 64; a 64-wide wave block past n_pad is skipped.  The tile's residual sum
// goes to the partial slot of its top-left 64-tile, zeros to the other 64-tile
// slots it covers, so the residual reduction is the same for both tile sizes.
// ---------------------------------------------------------------------------
template <int MODE> struct Traits128;
template <> struct Traits128<SM_F32> { using S = float; using L = float; static constexpr int K = 16, KP = 4; };
template <> struct Traits128<SM_BF16> { using S = float; using L = uint16_t; static constexpr int K = 32, KP = 8; };
template <> struct Traits128<SM_F16> { using S = float; using L = _Float16; static constexpr int K = 32, KP = 8; };
template <> struct Traits128<SM_BF16X3> { using S = float; using L = uint16_t; static constexpr int K = 32, KP = 8; };

// DEPTH > 1: operand stages are loaded DEPTH stages ahead into a ring of
// register sets (for large submatrices, whose operand panels come from the
// last-level cache or HBM with a latency of many stages); the ring restarts
// at every tile.
// Register budget of the 128-tile kernel: two waves per SIMD (at most 256
// registers per lane) where the LDS stages let two workgroups share a compute
// unit; the deep ring (DEPTH > 1) takes more registers and runs one.
// Stages in flight of variant 5 (a register ring at one wave per SIMD; on
// the water submatrices 3 / 4 / 6 / 8 stages took 1173 / 1015 / 1002 / 1005 ms
// per sign pass of a chunk).
constexpr int kDeepRing = 6;

template <int MODE, int DEPTH> struct Gemm128Occ {
  using Tr = Traits128<MODE>;
  static constexpr int NOP = MODE == SM_BF16X3 ? 4 : 2;
  static constexpr int kLds = 2 * NOP * 128 * (Tr::K + Tr::KP) * (int)sizeof(typename Tr::L);
  static constexpr int by_lds = 160 * 1024 / kLds;
  static constexpr int value = DEPTH > 1 ? 1 : (by_lds < 2 ? by_lds : 2);
};

template <int MODE, int WHICH, bool XCD, int DEPTH = 1>
__global__ __launch_bounds__(kBlock, (Gemm128Occ<MODE, DEPTH>::value)) void ns_gemm128_kernel(float* __restrict__ mats, int64_t shadow_off,
                                                            const int32_t* __restrict__ count,
                                                            const TileRec* __restrict__ recs,
                                                            double* __restrict__ partials) {
  using Tr = Traits128<MODE>;
  using S = typename Tr::S;
  using LT = typename Tr::L;
  constexpr int K = Tr::K;
  constexpr int LD = K + Tr::KP;
  constexpr int NL = K / 2;              // 128 rows x K per operand over 256 threads
  constexpr bool SPLIT = (MODE == SM_BF16X3);
  constexpr bool PRE = Pre<MODE>::value;
  constexpr int NPL = SPLIT ? 2 : 1;
  constexpr int NOP = 2 * NPL;
  using RT = typename std::conditional<PRE, uint32_t, S>::type;
  constexpr int RN = PRE ? NPL * NL / 2 : NL;
  // double-buffered LDS stages (a single buffer with two barriers per stage,
  // which lets two split-bf16 workgroups share a CU, measured slower)
  constexpr int NBUF = 2;
  __shared__ __attribute__((aligned(16))) LT lds[NBUF][NOP][128 * LD];
  static_assert(sizeof(lds) == (size_t)Gemm128Occ<MODE, DEPTH>::kLds, "LDS footprint");

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;
  const int lrow = tid >> 1;             // 0..127
  const int lpart = (tid & 1) * NL;
  const int total = count[0];
  int t_begin = blockIdx.x, t_end = total, t_step = gridDim.x, t_lo = 0;
  if (XCD) {
    const int x8 = blockIdx.x % kXcds;
    t_step = ((int)gridDim.x - x8 + kXcds - 1) / kXcds;
    t_lo = (int)((int64_t)total * x8 / kXcds);
    t_begin = t_lo + (int)blockIdx.x / kXcds;
    t_end = (int)((int64_t)total * (x8 + 1) / kXcds);
  }
  const int t_mirror = WHICH == 1 ? t_lo + t_end - 1 : -1;
  // DEPTH 1: operand registers carried from tile to tile (the next tile's
  // first stage is loaded during the last stage of the current one)
  RT rga[DEPTH][RN], rgb[DEPTH][RN];
  TileRec nxt;
  if (t_begin < t_end) {
    nxt = recs[rec_index(t_begin, t_mirror)];
    if constexpr (DEPTH == 1) {
      const TileSrc<MODE> s0 = tile_src<MODE, WHICH, 128>(nxt, mats, shadow_off, lrow, lpart);
      s0.a.template load<K, NL>(rga[0], 0, s0.va);
      s0.b.template load<K, NL>(rgb[0], 0, s0.vb);
    }
  }
  for (int t = t_begin; t < t_end; t += t_step) {
    const TileRec rec = nxt;
    const bool has_next = t + t_step < t_end;
    if (has_next) nxt = recs[rec_index(t + t_step, t_mirror)];
    const int npad = rec.npad;
    const int64_t nn = (int64_t)npad * npad;
    const double alpha = (double)rec.alpha;
    const double rscale = (double)rec.rscale;
    S* base = mats + rec.mat_off;
    S* Out = base + (WHICH == 0 ? 2 * nn : (int64_t)(rec.it & 1) * nn);
    const int bi = rec.bibj >> 16, bj = rec.bibj & 0xFFFF;
    const int r0 = bi * 128, c0 = bj * 128;
    const bool slab = (rec.flags & kTileSlab) != 0;   // all blocks, no mirror
    const bool wvalid = (r0 + wm * 64 < npad) && (c0 + wn * 64 < npad) &&
                        (slab ? (rec.flags & (kTileSlabWave << wn)) != 0 : !(bi == bj && wm < wn));
    const TileSrc<MODE> src = tile_src<MODE, WHICH, 128>(rec, mats, shadow_off, lrow, lpart);
    const int nst = npad / K;
    const int kq = lane >> 4;
    const int rl = lane & 15;

    f4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = f4{0, 0, 0, 0};

    if constexpr (DEPTH > 1) {   // ring prologue: stages 0 .. DEPTH - 1
#pragma unroll
      for (int u = 0; u < DEPTH; ++u)
        if (u < nst) {
          src.a.template load<K, NL>(rga[u], u, src.va);
          src.b.template load<K, NL>(rgb[u], u, src.vb);
        }
    }

    auto k_loop = [&](auto compute_tag) {
      constexpr bool COMPUTE = decltype(compute_tag)::value;
      for (int s0 = 0; s0 < nst; s0 += DEPTH)
#pragma unroll
      for (int u = 0; u < DEPTH; ++u) {
        const int s = s0 + u;
        if (DEPTH > 1 && s >= nst) break;   // uniform
        const int buf = s & 1;
        RT (&ra)[RN] = rga[u];
        RT (&rb)[RN] = rgb[u];
        stage_store<MODE, NL>(ra, &lds[buf][0][lrow * LD + lpart], &lds[buf][NOP - 2][lrow * LD + lpart]);
        stage_store<MODE, NL>(rb, &lds[buf][1][lrow * LD + lpart], &lds[buf][NOP - 1][lrow * LD + lpart]);
        __syncthreads();
        if (s + DEPTH < nst) {
          src.a.template load<K, NL>(ra, s + DEPTH, src.va);
          src.b.template load<K, NL>(rb, s + DEPTH, src.vb);
        } else if (DEPTH == 1 && has_next) {
          const TileSrc<MODE> sn = tile_src<MODE, WHICH, 128>(nxt, mats, shadow_off, lrow, lpart);
          sn.a.template load<K, NL>(ra, 0, sn.va);
          sn.b.template load<K, NL>(rb, 0, sn.vb);
        }
        if constexpr (!COMPUTE) {
        } else if constexpr (MODE == SM_F32) {
          // 16x16x4 with the stage's k permuted to 4 kq + kk (one 16-byte read per fragment)
          float a[4][4], b[4][4];
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
              a[x][kk] = lds[buf][0][(wm * 64 + x * 16 + rl) * LD + 4 * kq + kk];
              b[x][kk] = lds[buf][1][(wn * 64 + x * 16 + rl) * LD + 4 * kq + kk];
            }
#pragma unroll
          for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
              for (int y = 0; y < 4; ++y)
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x][kk], b[y][kk], acc[x][y], 0, 0, 0);
        } else if constexpr (MODE == SM_F16) {
          f16x8 a[4], b[4];
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            a[x] = *reinterpret_cast<const f16x8*>(&lds[buf][0][(wm * 64 + x * 16 + rl) * LD + 8 * kq]);
            b[x] = *reinterpret_cast<const f16x8*>(&lds[buf][1][(wn * 64 + x * 16 + rl) * LD + 8 * kq]);
          }
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
              acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[x], b[y], acc[x][y], 0, 0, 0);
        } else {
          bf16x8 a[4], b[4];
#pragma unroll
          for (int x = 0; x < 4; ++x) {
            a[x] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&lds[buf][0][(wm * 64 + x * 16 + rl) * LD + 8 * kq]));
            b[x] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&lds[buf][1][(wn * 64 + x * 16 + rl) * LD + 8 * kq]));
          }
          if constexpr (SPLIT) {
            bf16x8 al[4], bl[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
              al[x] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&lds[buf][2][(wm * 64 + x * 16 + rl) * LD + 8 * kq]));
              bl[x] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(&lds[buf][3][(wn * 64 + x * 16 + rl) * LD + 8 * kq]));
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
              for (int y = 0; y < 4; ++y) {
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[x], b[y], acc[x][y], 0, 0, 0);
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], bl[y], acc[x][y], 0, 0, 0);
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], b[y], acc[x][y], 0, 0, 0);
              }
          } else {
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
              for (int y = 0; y < 4; ++y)
                acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], b[y], acc[x][y], 0, 0, 0);
          }
        }
      }
    };
    if (wvalid) k_loop(std::true_type{}); else k_loop(std::false_type{});

    // epilogue: lower triangle mirrored (exactly symmetric result); the
    // wave sums of the residual meet in the stage buffer the last stage did
    // not use
    double part = 0.0;
    double* red = reinterpret_cast<double*>(&lds[nst & 1][0][0]);
    const bool f32out = Pre<MODE>::value && WHICH == 1 && (rec.flags & kTileStoreF32);
#pragma unroll
    for (int x = 0; x < (wvalid ? 4 : 0); ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) {
        const int rb = r0 + wm * 64 + x * 16 + 4 * kq, cc = c0 + wn * 64 + y * 16 + rl;
        if (f32out) store_quad<SM_F32, WHICH>(acc[x][y], Out, shadow_off, nn, npad, rb, cc, alpha, rscale, part);
        else store_quad<MODE, WHICH>(acc[x][y], Out, shadow_off, nn, npad, rb, cc, alpha, rscale, part, !slab);
      }
    if (WHICH == 0) {
      part = wave_sum(part);
      if (lane == 0) red[wid] = part;
      __syncthreads();
      if (tid == 0) {
        partials[rec.part_idx] = ((red[0] + red[1]) + red[2]) + red[3];
        // other 64-tile slots covered by this tile (lower triangle, inside
        // n_pad); a slab tile has a slot of its own
        const int b0i = 2 * bi, b0j = 2 * bj;
        const int s0 = b0i * (b0i + 1) / 2 + b0j;
#pragma unroll
        for (int q = 1; q < 4; ++q) {
          const int ti = b0i + (q >> 1), tj = b0j + (q & 1);
          if (!slab && ti < rec.tiles64 && tj < rec.tiles64 && ti >= tj)
            partials[rec.part_idx + (ti * (ti + 1) / 2 + tj - s0)] = 0.0;
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 256 x 256 output tiles for the large submatrices of the 16-bit main phases
// (bf16, f16, split bf16): 512 threads, 8 waves (two per SIMD) in 2 x 4, each
// computing 128 x 64 outputs (4 x 2 blocks of 32 x 32, 32x32x16 instructions:
// a measured 2.24 PF/s of bf16 issue against 1.67 for 16x16x32 at two waves
// per SIMD).  A tile reads half the operand bytes per flop of the 128-wide
// tiles and a wave reads half the LDS bytes per matrix-core instruction of a
// 64 x 64 wave block.  Operand stages (k depth KS = 32 or 16) go from the
// copies into LDS with direct 16-byte global -> LDS loads (no staging
// registers, no LDS store instructions), issued NBUF - 1 stages ahead into a
// ring of NBUF LDS buffers (2 x 32 or 4 x 16: 128 KiB for split bf16).
//
// LDS stage layout: [operand][plane (hi, lo)][256 rows][2 KS bytes].  Inside a
// row the 16-byte k-chunks sit at position c ^ swz(R), R the row within its
// operand (four chunks per row: (R >> 2) & 3; two: (R >> 3) & 1): any sixteen
// consecutive rows read at one k-chunk fall on sixteen distinct 16-byte bank
// groups (sixteen lanes of a 16-byte LDS read are served together).
// ---------------------------------------------------------------------------
constexpr int kBlock256 = 512;

template <int MODE, int KS> struct G256 {
  static constexpr int PL = MODE == SM_BF16X3 ? 2 : 1;     // planes (hi, lo)
  static constexpr int RB = 2 * KS;                          // bytes of one row of one plane per stage
  static constexpr int CPR = RB / 16;                        // 16-byte k-chunks per row
  static constexpr int RPC = 1024 / RB;                      // rows per 1 KiB chunk
  static constexpr int PLANE = 256 * RB;                     // bytes of one plane of one operand
  static constexpr int CHUNKS = 2 * PL * PLANE / 1024;       // 1 KiB chunks per stage
  static constexpr int LPW = CHUNKS / 8;                     // direct loads per wave per stage
  static constexpr int STAGE = CHUNKS * 1024;                // bytes per stage
};

template <int CPR>
__device__ __forceinline__ int swz256(int R) { return CPR == 4 ? (R >> 2) & 3 : (R >> 3) & 1; }

// One 16-byte direct global -> LDS load per lane: lane l's 16 bytes land at
// lds_wave + 16 l (lds_wave is wave-uniform).
__device__ __forceinline__ void lds_load16(const void* g, void* lds_wave) {
  __builtin_amdgcn_global_load_lds(g, lds_wave, 16, 0, 0);
}

// Wait until at most N of this wave's vector memory operations are in flight
// (N < 16; lgkmcnt and expcnt unconstrained).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 16, "vmcnt immediate");
  __builtin_amdgcn_s_waitcnt(0x0f70 | N);
}

// Byte offset in a stage of (operand op, row R, plane p, k-chunk c).
template <int MODE, int KS>
__device__ __forceinline__ int g256_off(int op, int R, int p, int c) {
  using G = G256<MODE, KS>;
  return (op * G::PL + p) * G::PLANE + R * G::RB + ((c ^ swz256<G::CPR>(R)) << 4);
}

// Round barriers of the synchronized walk (variant 8): `sync` (kXcds + 1
// counters in the workspace, zero before the first launch) holds per XCD the
// number of tile rounds its workgroups have finished, and the workgroups that
// have left the kernel (the last one resets all of it for the next launch).
// Only the timing depends on these counters: a wait gives up after
// kSyncSpins polls, and every access is a relaxed device-scope atomic (an
// acquire or release would invalidate or write back the L2 whose reuse the
// barrier is for).
constexpr int kSyncSpins = 4096;

template <int MODE, int WHICH, int KS, int NBUF, bool SYNC>
__device__ __forceinline__ void gemm256_body(float* __restrict__ mats, int64_t shadow_off,
                                             const int32_t* __restrict__ count, const TileRec* __restrict__ recs,
                                             double* __restrict__ partials, unsigned* __restrict__ sync) {
  using G = G256<MODE, KS>;
  constexpr bool SPLIT = MODE == SM_BF16X3;
  constexpr int AHEAD = NBUF - 1;
  static_assert(Pre<MODE>::value, "16-bit operand copies only");
  static_assert(AHEAD * G::LPW < 16, "loads in flight must fit the vmcnt counter");
  __shared__ __attribute__((aligned(1024))) char lds[NBUF * G::STAGE];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int wm = wid >> 2, wn = wid & 3;   // rows 128 wm .., columns 64 wn ..
  const int total = count[0];
  // the workgroups of XCD x walk the x-th contiguous eighth of the list
  // (updates backwards, see rec_index)
  const int x8 = blockIdx.x % kXcds;
  const int t_step = ((int)gridDim.x - x8 + kXcds - 1) / kXcds;
  const int t_lo = (int)((int64_t)total * x8 / kXcds);
  const int t_begin = t_lo + (int)blockIdx.x / kXcds;
  const int t_end = (int)((int64_t)total * (x8 + 1) / kXcds);
  const int t_mirror = WHICH == 1 ? t_lo + t_end - 1 : -1;

  // this lane's part of the wave's direct loads: load u of wave wid fills
  // chunk q = wid * LPW + u (plane region q / (PLANE / 1 KiB)); lane -> (row
  // in chunk, LDS k-chunk position)
  const int l_rr = lane / G::CPR;
  const int l_cp = lane % G::CPR;

  int round = 0;
  for (int t = t_begin; t < t_end; t += t_step, ++round) {
    if constexpr (SYNC) {
      // start round r once every workgroup of this XCD has finished round
      // r - 1: the XCD's tiles of a round (consecutive in the list, mostly of
      // one submatrix, sharing operand panels) then stream through k together
      // and reuse each other's panel slices from the L2
      if (round > 0) {
        if (tid == 0) {
          const unsigned target = (unsigned)round * (unsigned)t_step;
          for (int k = 0; k < kSyncSpins; ++k) {
            if (__hip_atomic_load(&sync[x8], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
            __builtin_amdgcn_s_sleep(4);
          }
        }
        __syncthreads();
      }
    }
    const TileRec rec = recs[rec_index(t, t_mirror)];
    const int npad = rec.npad;
    const int64_t nn = (int64_t)npad * npad;
    const double alpha = (double)rec.alpha;
    const double rscale = (double)rec.rscale;
    float* base = mats + rec.mat_off;
    float* Out = base + (WHICH == 0 ? 2 * nn : (int64_t)(rec.it & 1) * nn);
    const float* Xp = base + (int64_t)((WHICH == 0 ? rec.it : rec.it + 1) & 1) * nn;
    const float* Rp = WHICH == 0 ? Xp : base + 2 * nn;
    const int bi = rec.bibj >> 16, bj = rec.bibj & 0xFFFF;
    const int r0 = bi * 256, c0 = bj * 256;
    const bool wvalid = (r0 + wm * 128 < npad) && (c0 + wn * 64 < npad) &&
                        !(bi == bj && wm * 128 + 127 < wn * 64);
    // global source of this lane's loads: the LPW chunks of a wave lie in one
    // (operand, plane) region, rows R_0 + u RPC (u < LPW) at one k-chunk
    // (the swizzle of R_0 + u RPC is that of R_0); rows past n_pad read row
    // n_pad - 1 (their products land in outputs that are never stored)
    static_assert((G::PLANE / 1024) % G::LPW == 0, "a wave's loads stay in one plane region");
    const int q0 = wid * G::LPW;
    const int region = q0 / (G::PLANE / 1024);             // op * PL + plane
    const int op = region / G::PL, pl = region % G::PL;
    const int R0l = (q0 % (G::PLANE / 1024)) * G::RPC + l_rr;
    const int row0 = (op == 0 ? r0 : c0) + R0l;
    const int64_t rstride = SPLIT ? 2 * (int64_t)npad : npad;
    const uint16_t* cbase = reinterpret_cast<const uint16_t*>((op == 0 ? Xp : Rp) + shadow_off) + pl * 32 +
                            (l_cp ^ swz256<G::CPR>(R0l)) * 8;
    const int nst = npad / KS;
    // stage s starts at k = KS s: for split copies, 32-row run s KS / 32 (64
    // elements: hi then lo), offset (s KS) % 32 inside it
    auto issue = [&](int s) {
      char* dst = lds + (s % NBUF) * G::STAGE;
      const int64_t k0 = (int64_t)s * KS;
      const int64_t so = SPLIT ? (k0 >> 5) * 64 + (k0 & 31) : k0;
#pragma unroll
      for (int u = 0; u < G::LPW; ++u)
        lds_load16(cbase + (int64_t)min(row0 + u * G::RPC, npad - 1) * rstride + so,
                   dst + (q0 + u) * 1024);
    };

    // 32 x 32 result blocks: 4 (rows) x 2 (columns) per wave
    f32x16 acc[4][2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = f32x16{};

    // 32x32x16 operand fragments of one k-step: lane l supplies row l % 32
    // of each of its operand blocks and the 8 k values of k-chunk
    // 2 ks + l / 32 (16 bytes); A of the wave's 4 block rows, B of its 2
    // block columns, hi and (split) lo
    const int r32 = lane & 31, kh = lane >> 5;
    struct Frag {
      u32x4 ah[4], al[4], bh[2], bl[2];
    };
    auto load_frag = [&](Frag& f, const char* st, int ks) {
      const int kc = 2 * ks + kh;
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int R = wn * 64 + y * 32 + r32;
        f.bh[y] = *reinterpret_cast<const u32x4*>(st + g256_off<MODE, KS>(1, R, 0, kc));
        if (SPLIT) f.bl[y] = *reinterpret_cast<const u32x4*>(st + g256_off<MODE, KS>(1, R, 1, kc));
      }
#pragma unroll
      for (int x = 0; x < 4; ++x) {
        const int R = wm * 128 + x * 32 + r32;
        f.ah[x] = *reinterpret_cast<const u32x4*>(st + g256_off<MODE, KS>(0, R, 0, kc));
        if (SPLIT) f.al[x] = *reinterpret_cast<const u32x4*>(st + g256_off<MODE, KS>(0, R, 1, kc));
      }
    };
    auto mfma_frag = [&](const Frag& f) {
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          if constexpr (MODE == SM_F16) {
            acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, f.ah[x]),
                                                               __builtin_bit_cast(f16x8, f.bh[y]), acc[x][y], 0, 0, 0);
          } else {
            const bf16x8 a = __builtin_bit_cast(bf16x8, f.ah[x]), b = __builtin_bit_cast(bf16x8, f.bh[y]);
            if constexpr (SPLIT) {
              acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, f.al[x]), b, acc[x][y], 0, 0, 0);
              acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, __builtin_bit_cast(bf16x8, f.bl[y]), acc[x][y], 0, 0, 0);
            }
            acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[x][y], 0, 0, 0);
          }
        }
    };
    // a plain barrier, not __syncthreads(): its fence would wait for every
    // load in flight, the later stages' too
    auto barrier = [&]() {
      asm volatile("" ::: "memory");
      __builtin_amdgcn_s_barrier();
      asm volatile("" :: "v"(lds) : "memory");
    };

#pragma unroll
    for (int u = 0; u < AHEAD; ++u)
      if (u < nst) issue(u);
    for (int s = 0; s < nst; ++s) {
      // this wave's loads of stage s have landed (those of the later stages
      // already issued may still fly); after the barrier every wave's have,
      // and every wave is done with stage s - 1, whose buffer stage s + AHEAD
      // refills (every LDS read of stage s - 1 has returned: the matrix-core
      // instructions that use it were issued)
      if (s + AHEAD <= nst) wait_vm<(AHEAD - 1) * G::LPW>();
      else if (AHEAD >= 3 && s + 2 == nst) wait_vm<(AHEAD >= 3 ? G::LPW : 0)>();
      else wait_vm<0>();
      barrier();
      if (s + AHEAD < nst) issue(s + AHEAD);
      if (!wvalid) continue;
      const char* st = lds + (s % NBUF) * G::STAGE;
      if constexpr (SYNC && SPLIT && KS == 32) {
        // the stage's fragment reads in the order the matrix-core blocks
        // use them, each block row's reads issued while the previous row's
        // products run (left to itself the compiler reads a group, waits
        // for it and multiplies, so every wave waits on the LDS several
        // times per k-step)
        Frag f0, f1;
        load_frag(f0, st, 0);
        load_frag(f1, st, 1);
        mfma_frag(f0);
        mfma_frag(f1);
        __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);   // B of k-step 0, A of block row 0
#pragma unroll
        for (int q = 0; q < 6; ++q) {                         // rows 0-2; A of rows 1-3
          __builtin_amdgcn_sched_group_barrier(0x008, 3, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) {                         // row 3; B and A of row 0, k-step 1
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) {                         // k-step 1 rows 0-2; A of rows 1-3
          __builtin_amdgcn_sched_group_barrier(0x008, 3, 0);
          __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
        __builtin_amdgcn_sched_group_barrier(0x008, 6, 0);   // k-step 1 row 3
      } else {
#pragma unroll
        for (int ks = 0; ks < KS / 16; ++ks) {
          Frag f;
          load_frag(f, st, ks);
          mfma_frag(f);
        }
      }
    }

    // epilogue: register v of lane l in a 32 x 32 block holds row
    // 8 (v / 4) + 4 (l / 32) + v % 4 and column l % 32 (sm_selftest_mfma);
    // lower triangle mirrored, 16-bit copies (or float32 for a first
    // refinement update); residual partial sums of the square
    double part = 0.0;
    const bool f32out = WHICH == 1 && (rec.flags & kTileStoreF32);
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int R0 = r0 + wm * 128 + x * 32, C0 = c0 + wn * 64 + y * 32;
        if (!wvalid || R0 >= npad || C0 >= npad) continue;
        const int cc = C0 + (lane & 31);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int rb = R0 + 8 * g + 4 * (lane >> 5);
          const f4 q = f4{acc[x][y][4 * g], acc[x][y][4 * g + 1], acc[x][y][4 * g + 2], acc[x][y][4 * g + 3]};
          if (f32out) store_quad<SM_F32, WHICH>(q, Out, shadow_off, nn, npad, rb, cc, alpha, rscale, part);
          else store_quad<MODE, WHICH>(q, Out, shadow_off, nn, npad, rb, cc, alpha, rscale, part);
        }
      }
    if (WHICH == 0) {
      // the buffer of stage nst (no load fills it and no wave reads it)
      double* red = reinterpret_cast<double*>(lds + (nst % NBUF) * G::STAGE);
      part = wave_sum(part);
      if (lane == 0) red[wid] = part;
      __syncthreads();
      if (tid == 0) {
        double sum = 0.0;
#pragma unroll
        for (int w = 0; w < 8; ++w) sum += red[w];
        partials[rec.part_idx] = sum;
      }
      // the other 64-tile slots this tile covers (lower triangle, inside n_pad)
      if (tid > 0 && tid < 16) {
        const int ti = 4 * bi + (tid >> 2), tj = 4 * bj + (tid & 3);
        const int s0 = (4 * bi) * (4 * bi + 1) / 2 + 4 * bj;
        if (ti < rec.tiles64 && tj < rec.tiles64 && ti >= tj)
          partials[rec.part_idx + (ti * (ti + 1) / 2 + tj - s0)] = 0.0;
      }
    }
    __syncthreads();
    if constexpr (SYNC)
      if (tid == 0) __hip_atomic_fetch_add(&sync[x8], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if constexpr (SYNC) {
    if (tid == 0) {
      // the rounds this workgroup has no tile for count as finished
      const int rounds_x = (t_end - t_lo + t_step - 1) / t_step;
      if (rounds_x > round)
        __hip_atomic_fetch_add(&sync[x8], (unsigned)(rounds_x - round), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
      const unsigned out = __hip_atomic_fetch_add(&sync[kXcds], 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT) + 1;
      if (out == gridDim.x)
        for (int x = 0; x <= kXcds; ++x)
          __hip_atomic_exchange(&sync[x], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <int MODE, int WHICH, int KS, int NBUF>
__global__ __launch_bounds__(kBlock256, 1) void ns_gemm256_kernel(float* __restrict__ mats, int64_t shadow_off,
                                                                 const int32_t* __restrict__ count,
                                                                 const TileRec* __restrict__ recs,
                                                                 double* __restrict__ partials) {
  gemm256_body<MODE, WHICH, KS, NBUF, false>(mats, shadow_off, count, recs, partials, nullptr);
}

// Variant 8: variant 6 with the XCD's workgroups starting every tile round
// together (the round barriers above), and for split bf16 the fragment reads
// ordered into the products.
template <int MODE, int WHICH>
__global__ __launch_bounds__(kBlock256, 1) void ns_gemm256_sync_kernel(float* __restrict__ mats,
                                                                      int64_t shadow_off,
                                                                      const int32_t* __restrict__ count,
                                                                      const TileRec* __restrict__ recs,
                                                                      double* __restrict__ partials,
                                                                      unsigned* __restrict__ sync) {
  gemm256_body<MODE, WHICH, 32, 2, true>(mats, shadow_off, count, recs, partials, sync);
}

// 64-tile kernel variants: 0 = {full stage, linear walk}, 1 = {full stage,
// XCD-aware}, 2 = {half stage, XCD-aware}
template <int MODE, int WHICH, int V>
struct Var {
  static constexpr int KDIV = V == 2 ? 2 : 1;
  static constexpr bool XCD = V >= 1;
};

template <int MODE, int WHICH, int V>
static void* kernel_ptr() {
  return reinterpret_cast<void*>(&ns_gemm_kernel<MODE, WHICH, Var<MODE, WHICH, V>::KDIV, Var<MODE, WHICH, V>::XCD>);
}

// Grid, stream and optional timing events of one GEMM launch.  With events,
// the launch carries them (start / stop timestamps taken by the dispatch
// itself), so timing adds no separate packets to the stream.
struct Launch {
  int grid;
  hipStream_t s;
  hipEvent_t e0, e1;
  unsigned* sync;   // round counters of variant 8
  template <typename K, typename... A>
  hipError_t go(K kernel, A... args) const {
    return go_block(kBlock, kernel, args...);
  }
  template <typename K, typename... A>
  hipError_t go_block(int block, K kernel, A... args) const {
    if (e0)
      hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, e0, e1, 0, args...);
    else
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, args...);
    return hipGetLastError();
  }
};

template <int MODE, int WHICH, int V>
static hipError_t launch_one(void* mats, int64_t so, const int32_t* count, const TileRec* recs,
                             double* partials, const Launch& L) {
  using S = typename Traits<MODE>::S;
  return L.go(ns_gemm_kernel<MODE, WHICH, Var<MODE, WHICH, V>::KDIV, Var<MODE, WHICH, V>::XCD>, (S*)mats, so,
              count, recs, partials);
}

template <int MODE, int WHICH>
static hipError_t launch_which(int variant, void* mats, int64_t so, const int32_t* count,
                               const TileRec* recs, double* partials, const Launch& L) {
  switch (variant) {
    case 1: return launch_one<MODE, WHICH, 1>(mats, so, count, recs, partials, L);
    case 2: return launch_one<MODE, WHICH, 2>(mats, so, count, recs, partials, L);
    case 6:
      if constexpr (Pre<MODE>::value)
        return L.go_block(kBlock256, ns_gemm256_kernel<MODE, WHICH, 32, 2>, (float*)mats, so, count, recs,
                          partials);
      [[fallthrough]];
    case 7:
    case 8:
      if constexpr (Pre<MODE>::value) {
        if (variant == 7)
          return L.go_block(kBlock256, ns_gemm256_kernel<MODE, WHICH, 16, 4>, (float*)mats, so, count, recs,
                            partials);
        if (variant == 8 && L.sync)
          return L.go_block(kBlock256, ns_gemm256_sync_kernel<MODE, WHICH>, (float*)mats, so, count, recs,
                            partials, L.sync);
        if (variant == 8)   // no counters: the same tiles without the round barriers
          return L.go_block(kBlock256, ns_gemm256_kernel<MODE, WHICH, 32, 2>, (float*)mats, so, count, recs,
                            partials);
      }
      [[fallthrough]];
    case 3:
    case 4:
    case 5:
      if constexpr (MODE != SM_F64) {
        if (variant == 3)
          return L.go(ns_gemm128_kernel<MODE, WHICH, true>, (float*)mats, so, count, recs, partials);
        if (variant >= 5)
          return L.go(ns_gemm128_kernel<MODE, WHICH, true, kDeepRing>, (float*)mats, so, count, recs, partials);
        return L.go(ns_gemm128_kernel<MODE, WHICH, false>, (float*)mats, so, count, recs, partials);
      } else {
        return launch_one<MODE, WHICH, 1>(mats, so, count, recs, partials, L);
      }
    default: return launch_one<MODE, WHICH, 0>(mats, so, count, recs, partials, L);
  }
}

template <int MODE>
static hipError_t launch_mode(int which, int variant, void* mats, int64_t so, const int32_t* count,
                              const TileRec* recs, double* partials, const Launch& L) {
  return which == 0 ? launch_which<MODE, 0>(variant, mats, so, count, recs, partials, L)
                    : launch_which<MODE, 1>(variant, mats, so, count, recs, partials, L);
}

hipError_t launch_ns_gemm(int mode, int which, int variant, void* mats, int64_t so,
                          const int32_t* count, const TileRec* recs, double* partials, unsigned* sync, int grid,
                          hipStream_t s, hipEvent_t ev_start, hipEvent_t ev_stop) {
  // the bf16 / f16 / split-bf16 products need the copy region
  if (mode >= SM_BF16 && so <= 0) return hipErrorInvalidValue;
  const Launch L{grid, s, ev_start, ev_stop, sync};
  switch (mode) {
    case SM_F64: return launch_mode<SM_F64>(which, variant, mats, 0, count, recs, partials, L);
    case SM_F32: return launch_mode<SM_F32>(which, variant, mats, so, count, recs, partials, L);
    case SM_BF16: return launch_mode<SM_BF16>(which, variant, mats, so, count, recs, partials, L);
    case SM_F16: return launch_mode<SM_F16>(which, variant, mats, so, count, recs, partials, L);
    case SM_BF16X3: return launch_mode<SM_BF16X3>(which, variant, mats, so, count, recs, partials, L);
  }
  return hipErrorInvalidValue;
}

template <int MODE, int WHICH>
static void* ptr_which(int variant) {
  switch (variant) {
    case 1: return kernel_ptr<MODE, WHICH, 1>();
    case 2: return kernel_ptr<MODE, WHICH, 2>();
    case 3:
      if constexpr (MODE != SM_F64) return reinterpret_cast<void*>(&ns_gemm128_kernel<MODE, WHICH, true>);
      else return kernel_ptr<MODE, WHICH, 1>();
    case 4:
      if constexpr (MODE != SM_F64) return reinterpret_cast<void*>(&ns_gemm128_kernel<MODE, WHICH, false>);
      else return kernel_ptr<MODE, WHICH, 1>();
    case 6:
      if constexpr (Pre<MODE>::value) return reinterpret_cast<void*>(&ns_gemm256_kernel<MODE, WHICH, 32, 2>);
      [[fallthrough]];
    case 7:
    case 8:
      if constexpr (Pre<MODE>::value) {
        if (variant == 7) return reinterpret_cast<void*>(&ns_gemm256_kernel<MODE, WHICH, 16, 4>);
        if (variant == 8) return reinterpret_cast<void*>(&ns_gemm256_sync_kernel<MODE, WHICH>);
      }
      [[fallthrough]];
    case 5:
      if constexpr (MODE != SM_F64) return reinterpret_cast<void*>(&ns_gemm128_kernel<MODE, WHICH, true, kDeepRing>);
      else return kernel_ptr<MODE, WHICH, 1>();
    default: return kernel_ptr<MODE, WHICH, 0>();
  }
}

template <int MODE>
static void* ptr_mode(int which, int variant) {
  return which == 0 ? ptr_which<MODE, 0>(variant) : ptr_which<MODE, 1>(variant);
}

// Resident workgroups per compute unit of a GEMM kernel (persistent grid size).
int ns_gemm_blocks_per_cu(int mode, int which, int variant) {
  static int cache[5][2][kGemmVariants] = {};
  if (mode < 0 || mode > 4 || which < 0 || which > 1 || variant < 0 || variant >= kGemmVariants) return 1;
  int& c = cache[mode][which][variant];
  if (c) return c;
  void* f = nullptr;
  switch (mode) {
    case SM_F64: f = ptr_mode<SM_F64>(which, variant); break;
    case SM_F32: f = ptr_mode<SM_F32>(which, variant); break;
    case SM_BF16: f = ptr_mode<SM_BF16>(which, variant); break;
    case SM_F16: f = ptr_mode<SM_F16>(which, variant); break;
    default: f = ptr_mode<SM_BF16X3>(which, variant); break;
  }
  int nb = 0;
  const int block = (variant >= 6 && mode >= SM_BF16) ? kBlock256 : kBlock;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, block, 0) != hipSuccess || nb < 1) nb = 1;
  c = nb;
  return nb;
}

// ---------------------------------------------------------------------------
// device scheduler
// ---------------------------------------------------------------------------
struct SchedOpts {
  int refine_steps, max_iter, accel;
  double tol, switch_tol, stall_below, stall_ratio;
  int copies_main;   // the main phase keeps only 16-bit operand copies
  // entrywise error model of the first square as stored: |A~ - A| <= (eps_rep
  // + n_pad eps_acc) |X_0| |X_0| for the operands' representation and the
  // product's accumulation (precision of the main phase), with the storage
  // rounding of Y' inside eps_rep
  double eps_rep, eps_acc;
};

// The Newton-Schulz map with scale a on one eigenvalue x >= 0.
__device__ __forceinline__ double ns_map(double a, double x) { return 0.5 * a * x * (3.0 - a * a * x * x); }

// Scale for a spectrum inside [lb, top] (absolute values): the a for which
// lb and top have the same image, so that the image is [ns_map(a, lb), 1]
// (for top = 1: a^2 = 3 / (1 + lb + lb^2)), capped at sqrt(3) / (1.01 top) so
// every eigenvalue stays on the increasing branch with a margin for rounding.
// Rounded to float, the precision in which the kernels receive it.
__device__ __forceinline__ double ns_alpha(double lb, double top) {
  const double l = fmin(lb / top, 1.0);
  const double a = fmin(sqrt(3.0 / (1.0 + l + l * l)), 1.7320508075688772 / 1.01) / top;
  return (double)(float)a;
}

// x with g(x) = y, g(x) = x (3 - x^2) / 2, on [0, 1]: x = 2 sin(asin(y) / 3)
// (g(2 sin t) = sin 3t).
__device__ __forceinline__ double ns_map_inv(double y) { return 2.0 * sin(asin(fmin(y, 1.0)) / 3.0); }

enum { DEC_UPD = 1, DEC_SQ = 2, DEC_REF = 4 };

// exclusive scan over the block; returns the block total in `total`
// Exclusive prefix sums of K per-thread counts over the block, all K in one
// pass (wave scans by shuffles, one exchange of wave totals through LDS).
// sh: K * 16 ints of LDS.
template <int K>
__device__ void block_excl_scan(const int (&v)[K], int (&ex)[K], int (&total)[K], int* sh) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  int x[K];
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] = v[k];
#pragma unroll
  for (int o = 1; o < 64; o <<= 1)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int y = __shfl_up(x[k], o, 64);
      if (lane >= o) x[k] += y;
    }
  __syncthreads();   // the previous call's readers are done with sh
  if (lane == 63)
#pragma unroll
    for (int k = 0; k < K; ++k) sh[k * 16 + wid] = x[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    int off = 0, t = 0;
    for (int w = 0; w < nw; ++w) {
      const int c = sh[k * 16 + w];
      if (w < wid) off += c;
      t += c;
    }
    ex[k] = off + x[k] - v[k];
    total[k] = t;
  }
}

// A wavefront per submatrix: the residual ||X^2 - I||_F of the square just
// computed, from its per-tile partial sums added in tile order.
__global__ __launch_bounds__(256) void residual_kernel(DevPlan p, int g0, int nsub, SubState* st,
                                                       const double* __restrict__ partials, int tshift_ref) {
  const int lane = threadIdx.x & 63;
  const int l = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (l >= nsub || !st[l].active) return;
  const int g = g0 + l;
  const int T = tiles_of(p.npad_g[g]);
  const int i = p.order_g[g];
  // a slab square wrote one slot per slab tile
  const int nt = st[l].sq_slab ? slab_tiles(p.npad_g[g], p.loc[i], p.bs[i], tshift_ref) : T * (T + 1) / 2;
  const double* pp = partials + p.tile_off_g[g];
  double r = 0.0;
  for (int k = lane; k < nt; k += 64) r += pp[k];
  r = wave_sum(r);
  if (lane == 0) st[l].res_new = (isnan(r) ? r : sqrt(fmax(r, 0.0)));
}

// One workgroup, a thread per submatrix: apply the stopping / phase-switch
// rules to the new residual, advance the counters, and compact the
// submatrices into four tile lists by ordered block scans: update in the
// main / refinement precision, square (next iteration) in the main /
// refinement precision.  fuse_res: the residual of each square is summed
// here, by the submatrix's thread over its tile partials in tile order
// (chunks with few tiles per submatrix); otherwise residual_kernel ran first.
__global__ __launch_bounds__(1024) void schedule_kernel(DevPlan p, int g0, int nsub, SubState* st,
                                                        const double* __restrict__ partials, int fuse_res,
                                                        int32_t* lists, int max_subs, SchedOpts o,
                                                        int first, int tshift_main, int tshift_ref,
                                                        const double* __restrict__ lb0,
                                                        const double* __restrict__ top0,
                                                        const double* __restrict__ x0s,
                                                        int32_t* live_host,
                                                        const double* __restrict__ colmax) {
  __shared__ int sh[8 * 16];
  const int stride = 2 + 2 * max_subs + 1;
  int run_subs[4] = {0, 0, 0, 0}, run_tiles[4] = {0, 0, 0, 0};
  for (int base = 0; base < nsub; base += blockDim.x) {
    const int l = base + threadIdx.x;
    int dec = 0, ntm = 0, ntr = 0, ntr_sq = 0, refine_left = -1;
    if (l < nsub) {
      SubState s = st[l];
      const int np = p.npad_g[g0 + l];
      // tiles of a column slab of the refinement kernel (last square /
      // update), read from the plan only where it is needed
      auto slab_count = [&]() {
        const int i = p.order_g[g0 + l];
        return slab_tiles(np, p.loc[i], p.bs[i], tshift_ref);
      };
      if (!first && fuse_res && s.active) {
        const int T64 = tiles_of(np);
        const int nt = s.sq_slab ? slab_count() : T64 * (T64 + 1) / 2;
        const double* pp = partials + p.tile_off_g[g0 + l];
        double r = 0.0;
#pragma unroll 8
        for (int k = 0; k < nt; ++k) r += pp[k];
        s.res_new = (isnan(r) ? r : sqrt(fmax(r, 0.0)));
      }
      const int Tm = (np + (1 << tshift_main) - 1) >> tshift_main;
      const int Tr = (np + (1 << tshift_ref) - 1) >> tshift_ref;
      ntm = Tm * (Tm + 1) / 2;
      ntr = Tr * (Tr + 1) / 2;
      ntr_sq = ntr;
      // the last update and the square before it compute only the slab,
      // where it has fewer tiles than the triangle; not for the first
      // refinement update (it runs in full on the main-precision kernel) nor
      // for the square that decides the switch (a main-phase square)
      const bool slab_allowed = !(o.copies_main && o.refine_steps == 1);
      if (first == 2 && s.status > 0) {
        // fallback retry: this submatrix finished well in the first run
      } else if (first) {
        s.active = 1;
        s.phase = 0;
        s.iters = 0;
        s.iters_low = 0;
        s.refine_left = 0;
        s.status = 0;
        s.res = 1e300;
        s.res_prev = 1e300;
        s.lb = lb0 ? fmax(lb0[l], 0.0) : 0.0;
        s.top = top0 ? fmax(top0[l], 1.0) : 1.0;
        // the first step maps the top of the spectrum to at most sqrt 3 / 1.01
        // whatever the schedule: with a scale c below rho(T) / sqrt 3 (a learned
        // scale the guard could not refute) an unscaled step would send the
        // eigenvalues above sqrt 3 to the wrong sign
        const double cap = 1.7320508075688772 / (1.01 * s.top);
        // a scaled run with c_G / c > 1: the first square runs unscaled (Y' =
        // 3I - A) and the first update's scale waits for the bound on rho(X_0)
        // that A gives (accel 2: the scale from c_G / c, before the square)
        s.amode = (o.accel == 1 && s.top > 1.0) ? 1 : 0;
        s.fix_y = 0;
        s.top1 = 0.0;
        s.alpha_sq = s.amode ? 1.0
                   : (o.accel && s.lb > 0.0) ? ns_alpha(s.lb, s.top) : (cap < 1.0 ? (double)(float)cap : 1.0);
        s.alpha_upd = 1.0;
        s.a0 = 1.0;
        s.lb_est = -1.0;
        s.last_slab = 0;
        s.sq_slab = 0;
        s.x0s = x0s ? x0s[l] : 1.0;
        s.res_last = 1e300;
        s.cap_hit = 0;
        s.retried = first == 2 ? 1 : 0;
        dec = DEC_SQ;
      } else if (s.active) {
        const double r = s.res_new;
        double lb = s.lb, top = s.top;
        s.res_last = r;
        s.fix_y = 0;
        if (s.amode && s.iters == 0 && colmax) {
          // rho(X_0)^2 = rho(A) <= the largest column sum of |A|; the stored
          // A~ differs from A by at most (eps_rep + n_pad eps_acc) times the
          // column sums of |X_0| |X_0|, each at most top^2 (top = c_G / c
          // bounds the column sums of |X_0|), plus the rounding of the 3I
          const double slack = (2.0 * o.eps_rep + (double)np * o.eps_acc) * top * top + 6.0 * o.eps_rep;
          const double t1 = sqrt(colmax[l] + slack);
          if (isfinite(t1)) top = fmax(fmin(top, t1), 1.0);
        }
        if (s.sq_slab) {
          // a slab square (refinement, the last update next): its columns'
          // residual only flags a diverged iteration and decides the final
          // status; res keeps the last full one
          s.sq_slab = 0;
          if (!(r < 1e300)) {
            s.status = -1;
            s.active = 0;
          }
        } else {
          s.res_prev = s.res;
          s.res = r;
          const bool stalled = r < o.stall_below && r > o.stall_ratio * s.res_prev;
          // divergence: after the first update every eigenvalue of a valid
          // iterate lies in [-sqrt 3, sqrt 3], so |x^2 - 1| <= 2 and the
          // residual is at most 2 sqrt(n_pad); and an unscaled step never
          // increases it (|g(x)^2 - 1| <= |x^2 - 1| on that interval), so a
          // growth well beyond rounding above stall_below means an eigenvalue
          // has left the interval (a scale below rho / sqrt 3 was trusted)
          const bool diverged = s.iters >= 1 && (r > 2.02 * sqrt((double)np) ||
                                                 (s.alpha_upd == 1.0 && r >= o.stall_below && r > 1.05 * s.res_prev));
          // r < 1 bounds every eigenvalue x of the current X: |x^2 - 1| <= r
          if (r < 1.0) {
            lb = fmax(lb, sqrt(1.0 - r));
            top = fmin(top, sqrt(1.0 + r));
            // plain run: carry the bound back to X_0.  Only residuals >= 0.01:
            // near convergence the inverse map is steep at 1, and the rounding
            // of a tiny residual would be amplified into the bound.
            if (!o.accel && r >= 0.01) {
              double x = sqrt(1.0 - r);
              for (int j = 0; j < s.iters; ++j) x = ns_map_inv(x);
              // the first update was g(a0 X_0), the later ones plain
              s.lb_est = fmax(s.lb_est, s.iters >= 1 ? x / s.a0 : x);
            }
          }
          if (!(r < 1e300) || diverged) {
            s.status = -1;
            s.active = 0;
          } else if (s.phase == 0) {
            if (o.refine_steps == 0) {
              if (r < o.tol || stalled) {
                s.status = 1;
                s.active = 0;
              } else if (s.iters >= o.max_iter) {
                s.status = 0;
                s.active = 0;
              } else {
                dec = DEC_UPD | DEC_SQ;
                s.iters++;
                s.iters_low++;
              }
            } else if (r < o.switch_tol || stalled || s.iters >= o.max_iter) {
              s.phase = 1;
              s.refine_left = o.refine_steps;
              s.cap_hit = !(r < o.switch_tol) && !stalled;   // ran out of main-phase iterations
            } else {
              dec = DEC_UPD | DEC_SQ;
              s.iters++;
              s.iters_low++;
            }
          }
        }
        if (s.active && s.phase == 1 && dec == 0) {
          dec = DEC_UPD | DEC_REF;
          s.iters++;
          s.refine_left--;
          const int nslab = (slab_allowed && s.refine_left <= 1) ? slab_count() : ntr;
          const bool slab_ok = nslab < ntr;
          if (s.refine_left > 0) {
            dec |= DEC_SQ;
            // the square before the last update: the last update reads only
            // the slab columns of its Y
            if (s.refine_left == 1 && slab_ok) {
              s.sq_slab = 1;
              ntr_sq = nslab;
            }
          } else {
            // refinement done; not converged where the main phase ran out of
            // iterations, or where the square before this last update (r; for
            // a slab square its columns' part, a lower bound) is not below
            // the larger of switch_tol and stall_below, i.e. outside the
            // range in which the main phase hands over to refinement
            s.status = (s.cap_hit || !(r < fmax(o.switch_tol, o.stall_below))) ? 0 : 2;
            s.active = 0;
            // the last update needs only the atom's own columns of X (the
            // columns P takes); taken only where the slab has fewer tiles
            // than the triangle (which also keeps every submatrix within its
            // share of the tile lists)
            if (slab_ok) {
              s.last_slab = 1;
              ntr = nslab;
            }
          }
        }
        if (dec & DEC_UPD) {
          if (s.amode && s.iters == 1) {
            // the first update after an unscaled first square: its scale from
            // the bounds as they stand now (the square's column sums, the
            // residual), the same rule as for any other first step; Y = 3I -
            // a^2 A is formed from Y' before it runs (fix_y)
            const double cap = 1.7320508075688772 / (1.01 * top);
            s.alpha_sq = (o.accel && s.phase == 0 && lb > 0.0) ? ns_alpha(lb, top)
                                                                 : (cap < 1.0 ? (double)(float)cap : 1.0);
            s.fix_y = 1;
            s.top1 = top;
          }
          // the update of X uses its square's scale; bounds for the new X
          const double a = s.alpha_sq;
          s.alpha_upd = a;
          if (s.iters == 1) s.a0 = a;
          const double lo = fmin(ns_map(a, lb), ns_map(a, top));
          s.top = (a * top >= 1.0 && a * lb <= 1.0) ? 1.0 : fmax(ns_map(a, lb), ns_map(a, top));
          s.lb = fmax(lo, 0.0);
          // main-phase squares of an accelerated run are scaled, the rest plain
          s.alpha_sq = (o.accel && !(dec & DEC_REF) && s.phase == 0 && s.lb > 0.0) ? ns_alpha(s.lb, s.top) : 1.0;
        }
      }
      st[l] = s;
      refine_left = s.refine_left;
    }
    // a submatrix's first refinement update multiplies the main phase's
    // operand copies, so the main-precision kernel runs it (list 0) and
    // stores its result in float32 (tile flag)
    const bool first_ref_upd = o.copies_main && (dec & DEC_UPD) && (dec & DEC_REF) &&
                               refine_left == o.refine_steps - 1;
    bool in[4];
    int cnt[8], ex[8], tot[8];
#pragma unroll
    for (int L = 0; L < 4; ++L) {
      in[L] = (L == 0) ? ((dec & DEC_UPD) && (!(dec & DEC_REF) || first_ref_upd))
            : (L == 1) ? ((dec & DEC_UPD) && (dec & DEC_REF) && !first_ref_upd)
            : (L == 2) ? ((dec & DEC_SQ) && !(dec & DEC_REF))
                       : ((dec & DEC_SQ) && (dec & DEC_REF));
      cnt[2 * L] = in[L] ? 1 : 0;
      cnt[2 * L + 1] = in[L] ? (L == 1 ? ntr : L == 3 ? ntr_sq : ntm) : 0;
    }
    block_excl_scan<8>(cnt, ex, tot, sh);
#pragma unroll
    for (int L = 0; L < 4; ++L) {
      int32_t* Lb = lists + L * stride;
      if (in[L]) {
        Lb[2 + run_subs[L] + ex[2 * L]] = l;
        Lb[2 + max_subs + run_subs[L] + ex[2 * L]] = run_tiles[L] + ex[2 * L + 1];
      }
      run_subs[L] += tot[2 * L];
      run_tiles[L] += tot[2 * L + 1];
    }
  }
  if (threadIdx.x == 0) {
#pragma unroll
    for (int L = 0; L < 4; ++L) {
      int32_t* Lb = lists + L * stride;
      Lb[0] = run_tiles[L];
      Lb[1] = run_subs[L];
      Lb[2 + max_subs + run_subs[L]] = run_tiles[L];
    }
    // submatrices that square again (work after this iteration's updates),
    // for the host's stopping poll
    const int live = run_subs[2] + run_subs[3];
    lists[4 * stride] = live;
    if (live_host) {   // [live, square tiles main / refinement, refinement update tiles]
      live_host[0] = live;
      live_host[1] = run_tiles[2];
      live_host[2] = run_tiles[3];
      live_host[3] = run_tiles[1];
    }
  }
}

// One workgroup: the local indices of the submatrices of the chunk whose
// iteration failed (status 0 or -1), in ascending order, and their number
// (one thread writes the count: it may be host-mapped memory).
__global__ __launch_bounds__(1024) void collect_failed_kernel(int nsub, const SubState* __restrict__ st,
                                                              int32_t* __restrict__ list, int32_t* count) {
  __shared__ int sh[16];
  int run = 0;
  for (int base = 0; base < nsub; base += blockDim.x) {
    const int l = base + threadIdx.x;
    int v[1] = {(l < nsub && st[l].status <= 0) ? 1 : 0}, ex[1], tot[1];
    block_excl_scan<1>(v, ex, tot, sh);
    if (v[0]) list[run + ex[0]] = l;
    run += tot[0];
  }
  if (threadIdx.x == 0) *count = run;
}

hipError_t launch_collect_failed(int nsub, const SubState* st, int32_t* list, int32_t* count, hipStream_t s) {
  hipLaunchKernelGGL(collect_failed_kernel, dim3(1), dim3(1024), 0, s, nsub, st, list, count);
  return hipGetLastError();
}

hipError_t launch_schedule(const DevPlan& p, int g0, int nsub, SubState* st,
                           const double* partials, int32_t* lists, int max_subs,
                           const sm_sign_opts& so, int first, int tshift_main, int tshift_ref,
                           const double* lb0, const double* top0, const double* x0s, int32_t* live_host,
                           int max_tiles_sub, const double* colmax, hipStream_t s) {
  // representation error of the main phase's operands and stored results
  // (twice the unit roundoff of the value each holds: split bf16 about 17
  // bits, f16 11, bf16 8) and float32 / float64 accumulation
  const double eps_rep = so.phase1 == SM_F64 ? 0x1p-50 : so.phase1 == SM_F32 ? 0x1p-22
                       : so.phase1 == SM_BF16X3 ? 0x1p-15 : so.phase1 == SM_F16 ? 0x1p-10 : 0x1p-7;
  const double eps_acc = so.phase1 == SM_F64 ? 0x1p-52 : 0x1p-23;
  SchedOpts o{so.refine_steps, so.max_iter, so.accel, so.tol, so.switch_tol, so.stall_below, so.stall_ratio,
              so.phase1 >= SM_BF16 ? 1 : 0, eps_rep, eps_acc};
  // up to 64 partials per submatrix the scheduler's threads add them up
  // themselves; more are reduced by a wavefront each first
  const int fuse = max_tiles_sub <= 64;
  if (!first && !fuse && nsub > 0)
    hipLaunchKernelGGL(residual_kernel, dim3((nsub + 3) / 4), dim3(256), 0, s, p, g0, nsub, st, partials,
                       tshift_ref);
  hipLaunchKernelGGL(schedule_kernel, dim3(1), dim3(1024), 0, s, p, g0, nsub, st, partials, fuse, lists,
                     max_subs, o, first, tshift_main, tshift_ref, lb0, top0, x0s, live_host, colmax);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// self-test of the MFMA lane layout assumed above (one wavefront):
// A[r][k] = ((r + 3 k) mod 11) - 5, B[k][c] = ((2 k + 5 c) mod 13) - 6, exact in
// every precision; out[lane * 4 + v] = D element the lane holds in register v.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float st_a(int r, int k) { return (float)(((r + 3 * k) % 11) - 5); }
__device__ __forceinline__ float st_b(int k, int c) { return (float)(((2 * k + 5 * c) % 13) - 6); }

__global__ void selftest_kernel(int prec, double* out) {
  const int l = threadIdx.x;
  const int rl = l & 15, kq = l >> 4;
  if (prec == SM_F64) {
    d4 acc{0, 0, 0, 0};
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)st_a(rl, kq), (double)st_b(kq, rl), acc, 0, 0, 0);
    for (int v = 0; v < 4; ++v) out[l * 4 + v] = acc[v];
  } else if (prec == SM_F32) {
    f4 acc{0, 0, 0, 0};
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(st_a(rl, kq), st_b(kq, rl), acc, 0, 0, 0);
    for (int v = 0; v < 4; ++v) out[l * 4 + v] = acc[v];
  } else if (prec == SM_F16) {
    f16x8 a, b;
    for (int e = 0; e < 8; ++e) {
      a[e] = (_Float16)st_a(rl, 8 * kq + e);
      b[e] = (_Float16)st_b(8 * kq + e, rl);
    }
    f4 acc{0, 0, 0, 0};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc, 0, 0, 0);
    for (int v = 0; v < 4; ++v) out[l * 4 + v] = acc[v];
  } else if (prec == SM_BF16 || prec == SM_BF16X3) {
    u16x8 a, b;
    for (int e = 0; e < 8; ++e) {
      a[e] = f32_to_bf16_bits(st_a(rl, 8 * kq + e));
      b[e] = f32_to_bf16_bits(st_b(8 * kq + e, rl));
    }
    f4 acc{0, 0, 0, 0};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                  __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
    for (int v = 0; v < 4; ++v) out[l * 4 + v] = acc[v];
  } else {
    // 32x32x16 (prec 5: f16, 6: bf16): lane l supplies A[l % 32][8 (l / 32) ..]
    // and B[8 (l / 32) ..][l % 32]; out[lane * 16 + v] for the 16 registers
    const int r32 = l & 31, kh = l >> 5;
    f32x16 acc{};
    if (prec == 5) {
      f16x8 a, b;
      for (int e = 0; e < 8; ++e) {
        a[e] = (_Float16)st_a(r32, 8 * kh + e);
        b[e] = (_Float16)st_b(8 * kh + e, r32);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, acc, 0, 0, 0);
    } else {
      u16x8 a, b;
      for (int e = 0; e < 8; ++e) {
        a[e] = f32_to_bf16_bits(st_a(r32, 8 * kh + e));
        b[e] = f32_to_bf16_bits(st_b(8 * kh + e, r32));
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                    __builtin_bit_cast(bf16x8, b), acc, 0, 0, 0);
    }
    for (int v = 0; v < 16; ++v) out[l * 16 + v] = acc[v];
  }
}

hipError_t launch_selftest_mfma(int prec, double* out_dev, hipStream_t s) {
  hipLaunchKernelGGL(selftest_kernel, dim3(1), dim3(64), 0, s, prec, out_dev);
  return hipGetLastError();
}

}  // namespace sm
