// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/smsign.h"

namespace sm {

constexpr int kTile = 64;          // output tile edge of the Newton-Schulz GEMMs
// tiles per dimension of an n_pad x n_pad submatrix (the last one may be half full)
__host__ __device__ inline int tiles_of(int npad) { return (npad + kTile - 1) / kTile; }
constexpr int kNumFeatures = 16;   // per-submatrix features for the scaling network
constexpr int kMaxProbes = 8;

// Device view of the plan.  Arrays named *_g are indexed by the processing
// index g (submatrices in chunk order); the rest by atom id.
struct DevPlan {
  const int32_t* bs;         // [n_atoms] block sizes
  const int64_t* col_ptr;    // [n_atoms+1]
  const int32_t* row_idx;    // [nnzb]
  const int64_t* panel_off;  // [n_atoms+1]
  const int32_t* blk_rowoff; // [nnzb] row offset of stored block k inside its panel
  const int32_t* height;     // [n_atoms] panel height h_c (= n of submatrix c)
  const int32_t* loc;        // [n_atoms] row offset of the diagonal block in panel c
  const int32_t* order_g;    // [n_atoms] submatrix (atom) id at processing index g
  const int32_t* npad_g;     // [n_atoms] padded size
  const int64_t* mat_off_g;  // [n_atoms] element offset of the submatrix's 3 buffers in its chunk
  const int32_t* tile_off_g; // [n_atoms] offset of its residual partials in its chunk
  const int64_t* vec_off_g;  // [n_atoms] offset of its probe / power vectors in its chunk
};

// Per-submatrix iteration state (indexed by local index inside the chunk).
struct SubState {
  int32_t active;      // 1 while the submatrix still iterates
  int32_t phase;       // 0 main phase, 1 refinement
  int32_t iters;       // updates applied (parity selects the buffer holding X)
  int32_t iters_low;   // updates in the main phase
  int32_t refine_left; // refinement updates still to apply
  int32_t status;
  int32_t last_slab;   // 1: the last update (a refinement update) computed only the tile
                       // column(s) holding the atom's own columns; the last full X is the
                       // other buffer
  int32_t sq_slab;     // 1: the square just scheduled (the one before that last update)
                       // computes only the same tile columns of Y, all the last update
                       // reads; its residual partials are those columns' sums
  double res;          // last residual
  double res_prev;     // residual before that
  double res_new;      // residual of the square just computed (residual_kernel)
  // scaled Newton-Schulz: the spectrum of the current X is taken to lie in
  // [lb, top] in absolute value; alpha_sq scales the square about to run,
  // alpha_upd the update about to run (the update of X uses its square's alpha)
  double lb;
  double top;
  double alpha_sq;
  double alpha_upd;
  double lb_est;       // plain runs: lower bound on the smallest |eigenvalue| of X_0
  double x0s;          // X_0 = x0s * (buffer 0 as built): 1 / c except for float64 (1)
  double a0;           // scale of the first update (below 1 only where the top of the
                       // spectrum of X_0 could exceed sqrt 3 / 1.01; plain runs too)
  double res_last;     // residual of the last square (a slab square: its columns' part)
  int32_t cap_hit;     // 1: the main phase ended because max_iter was reached
  int32_t retried;     // 1: this run is the fallback retry (sm_sign_opts.retry)
  // first-step bound from the first square (scaled runs where c_G / c > 1):
  // that square stores Y' = 3I - A (A = X_0^2, scale 1), the largest column
  // sum of |A| bounds rho(X_0)^2, and the first update's scale comes from
  // that tighter top; fix_y: Y = 3I - a^2 A still has to be formed from Y'
  // before that update
  int32_t amode;
  int32_t fix_y;
  double top1;         // the top of the spectrum of X_0 the first update used (0: no bound)
};

// One output tile of a Newton-Schulz GEMM launch, written by expand_kernel so
// that a GEMM workgroup finds everything about its tile in one 40-byte record.
struct TileRec {
  int64_t mat_off;   // element offset of the submatrix's buffers in the chunk
  float alpha;       // Newton-Schulz scale: square Y = 3I - alpha^2 A, update 1/2 alpha X Y, with A
                     // and X the products / operands as stored (1 / c folded in for X_0)
  float rscale;      // squares: the residual is ||rscale A - I|| (1 / c^2 for X_0, else 1)
  int32_t bibj;      // tile row << 16 | tile column (row >= column)
  int32_t npad;
  int32_t it;        // iteration counter (parity selects the X buffer)
  int32_t part_idx;  // residual-partial slot of the 64-tile at the tile's top-left corner
  int16_t tiles64;   // 64-tiles per dimension of the submatrix (partial slots: lower triangle)
  int16_t flags;     // kTileStoreF32, kTileSlab, kTileSlabWave bits
};

// First refinement update of a submatrix, run by the main-precision update
// kernel on the main phase's operand copies (a split-bf16 product of them is
// the float32 product to float32 rounding): its result is stored in float32,
// for the refinement steps that follow, instead of as copies.
constexpr int16_t kTileStoreF32 = 2;
// Last refinement update of a submatrix (and, with two or more refinement
// steps, the square before it): only the tiles of the tile column(s) that
// hold the atom's own b_i columns (the columns P needs), all tile rows, the
// wave blocks of kTileSlabWave only, stored as they are (no mirror image).
constexpr int16_t kTileSlab = 4;
// Slab tiles: the two wave-block columns of the tile (32 wide in 64-wide
// tiles, 64 wide in 128-wide ones) that hold any of the atom's columns; the
// other wave blocks are skipped.  Bit kTileSlabWave << wn.
constexpr int16_t kTileSlabWave = 8;

// Tiles of that last update: all tile rows of the tile columns that
// columns loc .. loc + b - 1 fall into (tiles of edge 1 << tshift).
__host__ __device__ inline int slab_tiles(int npad, int loc, int b, int tshift) {
  const int T = (npad + (1 << tshift) - 1) >> tshift;
  return T * (((loc + b - 1) >> tshift) - (loc >> tshift) + 1);
}

// Workspace layout (bytes) for one chunk, given the storage element size.
struct WsLayout {
  int64_t mats;        // 3 * sum npad^2 elements
  int64_t state;       // SubState[max_subs]
  int64_t partials;    // double[max_tiles]
  int64_t lists;       // int32: counts[4], list[2][max_subs], prefix[2][max_subs+1]
  int64_t tiles;       // TileRec[4][max_tiles]: tile records of the four lists (updates main /
                       // refinement, squares main / refinement), indexed by list
  int64_t features;    // float[max_subs * kNumFeatures]
  int64_t scratch;     // double[max_subs * 8]: c_G, network outputs, lb0, top0, x0s, the
                       // failed list of the retry, column-sum bounds of the first square
  int64_t vecs;        // double[sum over chunk of npad * kMaxProbes*2] probe / power vectors
  int64_t flag;        // 256 bytes: the round counters of the synchronized GEMM walk
  int64_t total;
};

// Launchers (k_*.hip).  All return hipError_t from hipGetLastError.
// T_i of every submatrix of the chunk, plus its Gershgorin bound (cg_out,
// stats.gersh) and the features of the scaling network (features, stats.feat).
// shadow_kind: 0, or SM_BF16 / SM_F16 / SM_BF16X3 to write T_i only as the
// operand copies at float offset shadow_off from its float32 buffer.
// power_vecs (may be null): also w = T v0, the first power-iteration product
// of the scale kernel, into each submatrix's vectors (the scale kernel is then
// launched with pre_w).
// subs (may be null): build only these local indices (nsub of them).
hipError_t launch_gather(const DevPlan& p, int g0, int nsub, int max_m, int max_npad,
                         const double* H, double mu, void* mats, int storage_f64, int shadow_kind,
                         int64_t shadow_off, int* nonfinite, float* features, double* cg_out,
                         sm_sub_stats* stats, double* power_vecs, const int32_t* subs, hipStream_t s);
// Dynamic LDS bytes of the gather (with the power-product rows or without).
size_t gather_lds_bytes(int max_m, int max_npad, bool power);
// shadow_kind / shadow_off: where T_i is (as for the gather).  lbound:
// opts.lbound; lb0_out / top0_out [nsub]: bounds on the smallest / largest
// |eigenvalue| of X_0 for scaled Newton-Schulz (learned second output when the
// learned scale is accepted, else lbound; top c_G / c); x0s_out [nsub]: the
// factor the first products apply to buffer 0 (1 / c; 1 for float64, whose
// X_0 = T / c is stored).
hipError_t launch_scale(const DevPlan& p, int g0, int nsub, void* mats, int storage_f64, int scaling,
                        int power_steps, double margin, double* vecs, const double* cg_in,
                        const float* pred, sm_sub_stats* stats, int shadow_kind, int64_t shadow_off,
                        double lbound, double* lb0_out, double* top0_out, double* x0s_out, bool pre_w,
                        double force_scale, const int32_t* subs, hipStream_t s);
// The local indices of the chunk's submatrices with status 0 or -1 (list) and
// their number (count, one word, may be host-mapped).
hipError_t launch_collect_failed(int nsub, const SubState* st, int32_t* list, int32_t* count, hipStream_t s);
// first == 1 initialises the iteration state of every submatrix; first == 2
// (the fallback retry) only that of the submatrices whose status is 0 or -1,
// leaving the others finished; lb0 / top0 [nsub] (may be null):
// bounds on the smallest / largest |eigenvalue| of X_0 (scaled Newton-Schulz);
// x0s [nsub] (may be null: 1): SubState.x0s;
// live_host (may be null): device-mapped host words that receive the number
// of submatrices that square again after this iteration's updates (0: the
// iteration is over for the chunk), the tile counts of the next squares in
// the main and the refinement precision, and that of this iteration's
// refinement updates.  max_tiles_sub: most 64-tiles (lower triangle) of a
// submatrix in the chunk.
// colmax [nsub]: the first squares' bounds (launch_first_colmax), read at
// the decision after them.
hipError_t launch_schedule(const DevPlan& p, int g0, int nsub, SubState* st,
                           const double* partials, int32_t* lists, int max_subs,
                           const sm_sign_opts& o, int first, int tshift_main, int tshift_ref,
                           const double* lb0, const double* top0, const double* x0s, int32_t* live_host,
                           int max_tiles_sub, const double* colmax, hipStream_t s);
// First square of a submatrix with SubState.amode (its Y' = 3I - A in buffer
// 2: float64, float32 or the operand copies of `storage`): colmax[l] = the
// largest column sum of |A| over the padded matrix (A = 3I - Y'), 0 for the
// other submatrices.  One workgroup per submatrix, column sums in float64,
// so the value does not depend on the launch.
hipError_t launch_first_colmax(const DevPlan& p, int g0, int nsub, const void* mats, int storage,
                               int64_t shadow_off, const SubState* st, double* colmax, hipStream_t s);
// Submatrices with SubState.fix_y: Y = 3I - a^2 A = 3 (1 - a^2) I + a^2 Y'
// in place (a = SubState.alpha_upd, the first update's scale), then fix_y = 0.
hipError_t launch_first_fix_y(const DevPlan& p, int g0, int nsub, int max_npad, void* mats, int storage,
                              int64_t shadow_off, SubState* st, hipStream_t s);
// Tile records of all four lists (recs: TileRec[4][max_tiles], by list; the
// refinement lists only with with_ref).  Main-list tiles of a submatrix in
// refinement (its first refinement update) get kTileStoreF32.
hipError_t launch_expand(const DevPlan& p, int g0, const SubState* st, const int32_t* lists, int max_subs,
                         TileRec* recs, int64_t max_tiles, int tshift_main, int tshift_ref, bool with_ref,
                         int grid_subs, hipStream_t s);
// 0: linear, 1: XCD-aware, 2: XCD-aware with half-depth LDS stages, 3: XCD-aware 128 x 128 tiles,
// 4: 128 x 128 tiles walked linearly (all XCDs on the same submatrices),
// 5: as 3 with operands loaded six stages ahead,
// 6: XCD-aware 256 x 256 tiles of 512 threads (bf16, f16, split bf16 only),
// k-depth-32 stages one ahead, 7: the same with k-depth-16 stages three ahead
constexpr int kGemmVariants = SM_GEMM_VARIANTS;
// output tile edge (log2) of a GEMM variant for a precision; 128-wide tiles
// exist for the float32-accumulating precisions and need n_pad % 64 == 0,
// 256-wide ones for the 16-bit precisions (the launcher maps variants 6 and
// 7 to 5 for float32)
__host__ __device__ inline int tile_shift(int variant, int mode) {
  if (variant >= 6 && mode >= SM_BF16) return 8;
  return (variant >= 3 && mode != SM_F64) ? 7 : 6;
}
// shadow_off: float offset of the operand copies (bf16 / f16 / split-bf16
// products read them and write them for their outputs, except for
// kTileStoreF32 tiles); 0 otherwise.
// ev_start / ev_stop (may be null): events the launch itself records.
// sync: the workspace's round counters (variant 8; zero before the first launch)
hipError_t launch_ns_gemm(int mode, int which, int variant, void* mats, int64_t shadow_off,
                          const int32_t* count, const TileRec* recs, double* partials, unsigned* sync, int grid,
                          hipStream_t s, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// Commutator probes (1..4) of the final X against T read from H's panels.
hipError_t launch_comm_probe(const DevPlan& p, int g0, int nsub, int max_m, int max_npad, const double* H,
                             double mu, const void* mats, int storage_f64, const SubState* st, int probes,
                             double* vecs, sm_sub_stats* stats, hipStream_t s);
// Float32 values of the final X: from its 16-bit copies for submatrices whose
// iteration ended in a low-precision main phase (status != 2), times x0s when
// the final X is X_0 (no update ran); float32 schedules (shadow_kind 0): only
// the latter, in place.
hipError_t launch_materialize(const DevPlan& p, int g0, int nsub, float* mats, const SubState* st,
                              int shadow_kind, int64_t shadow_off, hipStream_t s);
int ns_gemm_blocks_per_cu(int mode, int which, int variant);

hipError_t launch_finish(const DevPlan& p, int g0, int nsub, const void* mats, int storage_f64,
                         const SubState* st, int probes, double* vecs, sm_sub_stats* stats, int max_npad,
                         hipStream_t s);
hipError_t launch_scatter(const DevPlan& p, int g0, int nsub, const void* mats, int storage_f64,
                          const SubState* st, double* P, hipStream_t s);
hipError_t launch_trace(const double* H, const double* P, int64_t nvals, const int64_t* diag_idx,
                        int64_t ndiag, double* partials, int nblocks, double* out2,
                        hipStream_t s);
hipError_t launch_ne_from_x(const DevPlan& p, int g0, int nsub, const void* mats,
                            int storage_f64, const SubState* st, double* ne_parts,
                            hipStream_t s);
// Gershgorin interval of every atom's rows (lohi_parts [2 n_atoms]) and
// their hull out2 = [lo, hi] (one thread writes: out2 may be host-mapped).
hipError_t launch_gersh_rows(const DevPlan& p, int n_atoms, const double* H, double* lohi_parts,
                             double* out2, hipStream_t s);
// The same into out2 (device memory), with the per-atom intervals in the
// library's fixed device scratch instead of lohi_parts: allocates nothing.
// hipErrorInvalidValue for n_atoms outside [1, kNoAllocMaxAtoms].
constexpr int kNoAllocMaxAtoms = 1 << 19;
hipError_t launch_gersh_rows_noalloc(const DevPlan& p, int n_atoms, const double* H, double* out2,
                                     hipStream_t s);
// out[0] = compensated sum of ne_sub[0 .. n_atoms) in a fixed order (one
// thread writes: out may be host-mapped).
hipError_t launch_ne_sum(const double* ne_sub, int n_atoms, double* out, hipStream_t s);
hipError_t launch_fill_i32(int32_t* dst, int32_t value, int64_t count, hipStream_t s);
hipError_t launch_selftest_mfma(int prec, double* out_dev, hipStream_t s);

}  // namespace sm
