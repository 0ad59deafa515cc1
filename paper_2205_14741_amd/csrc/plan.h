// Host-side plan object and error helpers (internal).
#pragma once

#include <string>
#include <vector>

#include "mlp.h"
#include "smsign_internal.h"

constexpr int kHostWords = 64;
constexpr int kHostCounts = 16;
constexpr int kHostBracket = 32;   // two doubles
constexpr int kHostNe = 36;        // one double
constexpr int kHostRetry = 40;     // submatrices of a chunk queued for the fallback retry
constexpr int kHostTrace = 10;     // E, Ne

struct sm_plan {
  // pattern (copied from the caller)
  int32_t n_atoms = 0;
  int64_t nnzb = 0;
  int64_t nvals = 0;
  std::vector<int32_t> bs;
  std::vector<int64_t> col_ptr;
  std::vector<int32_t> row_idx;
  std::vector<int64_t> panel_off;
  // derived, per atom
  std::vector<int32_t> blk_rowoff;  // [nnzb]
  std::vector<int32_t> height;      // panel height = submatrix size n_i
  std::vector<int32_t> loc;         // offset of the atom's own rows in its panel
  std::vector<int32_t> npad;
  std::vector<int64_t> diag_idx;    // [N] position of every diagonal entry in vals
  // processing order and chunks
  int32_t pad_to = sm::kTile;
  std::vector<int32_t> order_g;     // submatrix id at processing index g
  std::vector<int32_t> npad_g;
  std::vector<int64_t> mat_off_g;   // element offset inside the chunk
  std::vector<int32_t> tile_off_g;  // residual-partial offset inside the chunk
  std::vector<int64_t> vec_off_g;   // probe / power vector offset inside the chunk
  std::vector<int32_t> chunk_of;    // [n_atoms] chunk of every submatrix
  std::vector<int64_t> chunk_ptr;   // [n_chunks+1] ranges of g
  int64_t max_mats = 0;             // max over chunks of sum 3 npad^2
  int64_t max_subs = 0;
  int64_t max_tiles = 0;
  int64_t max_vecs = 0;             // max over chunks of sum npad * 2 * kMaxProbes
  int32_t max_m = 0;                // largest index-set size (atoms)
  int32_t max_npad = 0;

  // device copies (allocated on first device use)
  int device = -1;
  int num_cu = 256;
  sm::DevPlan dev{};
  std::vector<void*> dev_allocs;
  int64_t* d_diag_idx = nullptr;
  double* d_trace_parts = nullptr;  // [2 * kTraceBlocks + 2]
  double* d_ne_sub = nullptr;       // [n_atoms]
  double* d_gersh = nullptr;        // [2 * n_atoms]
  int32_t* h_pinned = nullptr;      // pinned, device-mapped host words [kHostWords]:
                                    // [0, 2) graph-path live counts, [8] nonfinite flag,
                                    // [kHostTrace, +4) E and Ne, [kHostCounts, +8)
                                    // scheduler counts (live, square tiles main /
                                    // refinement, refinement update tiles) by parity,
                                    // [kHostBracket, +4) Gershgorin hull, [kHostNe, +2)
                                    // electron count
  int32_t* d_pinned = nullptr;      // the device's address of h_pinned
  hipEvent_t ev[2] = {nullptr, nullptr};
  int last_storage = -1;            // workspace storage of the last build (ws_storage; -1: none)
  // the last build_submatrices call (the fallback retry builds again from it)
  int last_chunk = -1;
  const double* last_H = nullptr;
  double last_mu = 0.0;
  int32_t tuned[5] = {0, 0, 0, 0, 0};  // GEMM variant per precision (sm_autotune)
  // captured iteration graphs (sm_sign_opts.graph_iters)
  struct GraphEntry {
    int chunk;
    void* ws;
    sm_sign_opts opts;
    int32_t tuned[5];
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  hipStream_t capture_stream = nullptr;
  sm_mlp* mlp = nullptr;            // scaling network for SM_SCALE_LEARNED (not owned)
  // kernel timing (sm_profile_enable)
  bool profiling = false;
  std::vector<hipEvent_t> prof_ev;  // pool, pairs (start, stop)
  std::vector<int> prof_cls;        // class of every recorded pair

  // non-orthogonal basis: tile lists of the products by (chunk, kind: 0
  // lower triangle, 1 all tiles, 2 the tile columns of the atom's own
  // columns), per-submatrix scalars (c of T(S), its scratch), device copies
  struct OvlJobs {
    int chunk, kind, n;
    sm::OvlJob* d;
  };
  std::vector<OvlJobs> ovl_jobs;
  double* d_ovl = nullptr;          // [4 * max_subs]: c_i, residual sums, 1 / sqrt(c_i), spare
  int32_t* d_ovl_xbuf = nullptr;    // [max_subs]
  int ovl_chunk = -1;               // chunk whose Z_i the auxiliary workspace holds (-1: none)
  const void* ovl_aux = nullptr;    // that workspace

  sm::WsLayout layout(int storage) const;
  // float offset of a float32 buffer's pre-converted operand copy
  int64_t shadow_off() const { return max_mats; }
};

namespace sm {
constexpr int kTraceBlocks = 512;

int set_error(int code, const char* fmt, ...);
int hip_error(hipError_t e, const char* what);
int ensure_device(sm_plan* p);
int storage_is_f64(const sm_sign_opts* o);
int ws_storage(const sm_sign_opts* o);
bool valid_storage(int storage);
}  // namespace sm

#define SM_HIP(expr)                                         \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) return sm::hip_error(_e, #expr);   \
  } while (0)
