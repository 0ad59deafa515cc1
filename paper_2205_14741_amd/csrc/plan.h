// Host-side plan object and error helpers (internal).
#pragma once

#include <array>
#include <string>
#include <vector>

#include "mlp.h"
#include "ovl_internal.h"
#include "smsign_internal.h"

constexpr int kHostWords = 64;
constexpr int kHostCounts = 16;
constexpr int kHostBracket = 32;   // two doubles
constexpr int kHostNe = 36;        // one double
constexpr int kHostRetry = 40;     // submatrices of a chunk queued for the fallback retry
constexpr int kHostTrace = 10;     // E, Ne
constexpr int kHostOvl = 44;       // one double: largest residual of the S != I inverse square roots
constexpr int kHostFd = 46;        // one double: largest bound of |beta x| (finite temperature)
constexpr int kHostDne = 48;       // one double: dNe / dmu
constexpr int kClassRows = 256;    // size class of a chunk: 256-row tiles of its largest submatrix
constexpr int kMaxClasses = 32767 / kClassRows + 2;

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
  std::vector<int32_t> chunk_class; // [n_chunks] size class (kClassRows tiles of its largest n_pad)
  int64_t max_chunk_elems = 0;      // the chunk budget the plan was created with
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
  int32_t tuned[5] = {0, 0, 0, 0, 0};  // plan-wide GEMM variant per precision (sm_plan_tuning)
  // GEMM variants of every size class (sm_autotune of a chunk sets its
  // class's; [0] < 0: the class has no chunk), and the chunk whose class
  // the next launches use
  std::vector<std::array<int32_t, 5>> class_tuned;
  int active_chunk = -1;
  const int32_t* tuned_for(int chunk) const {
    if (chunk >= 0 && chunk < (int)chunk_class.size()) {
      const auto& t = class_tuned[chunk_class[chunk]];
      if (t[0] >= 0) return t.data();
    }
    return tuned;
  }
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
  int ovl_edge = 0;                 // tile edge of these products (64 or 128; 0: not chosen yet)
  double* d_ovl = nullptr;          // [4 * max_subs]: c_i, residual sums, 1 / sqrt(c_i), spare
  int32_t* d_ovl_xbuf = nullptr;    // [max_subs]
  int ovl_chunk = -1;               // chunk whose Z_i the auxiliary workspace holds (-1: none)
  const void* ovl_aux = nullptr;    // that workspace

  // finite temperature: [2 * max_subs] per-submatrix scalars (s, s^2) and
  // [n_atoms] dNe / dmu of every atom; the chunk, workspace and buffer that
  // hold the last f(T_i)
  double* d_fd = nullptr;
  double* d_fd_dne = nullptr;
  int fd_chunk = -1;
  const void* fd_ws = nullptr;
  int fd_buf = -1;

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
// float64 submatrix buffers of a workspace (the SM_F64 layout)
double* f64_mats(const sm_plan* p, const void* ws);
// device tables of the float64 tile products (api_ovl.cpp): per-submatrix
// scalars, and the tile list of a product kind over a chunk (0 lower
// triangle, 1 all tiles, 2 the tile columns of the atom's own columns),
// built once and kept on the device
int ensure_ovl(sm_plan* p);
int ovl_jobs(sm_plan* p, int chunk, int kind, const OvlJob** jobs, int* n);
}  // namespace sm

#define SM_HIP(expr)                                         \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) return sm::hip_error(_e, #expr);   \
  } while (0)
