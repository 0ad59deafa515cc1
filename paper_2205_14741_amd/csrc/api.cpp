// C-ABI entry points: argument checks, chunk loop, the host side of the
// Newton-Schulz iteration, chemical-potential bisection.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "plan.h"

using namespace sm;

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int check_opts(const sm_sign_opts* o) {
  if (!o) return set_error(SM_ERR_ARG, "null sm_sign_opts");
  if (o->phase1 < SM_F64 || o->phase1 > SM_BF16X3) return set_error(SM_ERR_ARG, "opts.phase1 = %d is not an sm_prec", o->phase1);
  if (o->refine_steps < 0 || o->refine_steps > 16) return set_error(SM_ERR_ARG, "opts.refine_steps = %d out of [0, 16]", o->refine_steps);
  if (o->refine_steps > 0 && o->refine != SM_F32 && o->refine != SM_F64)
    return set_error(SM_ERR_ARG, "opts.refine must be SM_F32 or SM_F64");
  if (o->refine_steps > 0 && (o->refine == SM_F64) != (o->phase1 == SM_F64))
    return set_error(SM_ERR_ARG, "refinement and main phase must both be float64 or both use float32 storage");
  if (o->max_iter < 0 || o->max_iter > 1000) return set_error(SM_ERR_ARG, "opts.max_iter = %d out of [0, 1000]", o->max_iter);
  if (o->scaling < SM_SCALE_GERSHGORIN || o->scaling > SM_SCALE_LEARNED) return set_error(SM_ERR_ARG, "opts.scaling = %d invalid", o->scaling);
  if (o->probes < 0 || o->probes > kMaxProbes) return set_error(SM_ERR_ARG, "opts.probes = %d out of [0, %d]", o->probes, kMaxProbes);
  if (o->variant < -1 || o->variant >= kGemmVariants) return set_error(SM_ERR_ARG, "opts.variant = %d out of [-1, %d)", o->variant, kGemmVariants);
  if (o->graph_iters < 0 || o->graph_iters > 64) return set_error(SM_ERR_ARG, "opts.graph_iters = %d out of [0, 64]", o->graph_iters);
  if (o->power_steps < 0 || o->power_steps > 200) return set_error(SM_ERR_ARG, "opts.power_steps out of [0, 200]");
  if (o->accel < 0 || o->accel > 2) return set_error(SM_ERR_ARG, "opts.accel = %d is not 0, 1 or 2", o->accel);
  if (o->comm_probes < 0 || o->comm_probes > 4) return set_error(SM_ERR_ARG, "opts.comm_probes = %d out of [0, 4]", o->comm_probes);
  if (o->retry != 0 && o->retry != 1) return set_error(SM_ERR_ARG, "opts.retry = %d is not 0 or 1", o->retry);
  if (!(o->force_scale >= 0.0) || !std::isfinite(o->force_scale))
    return set_error(SM_ERR_ARG, "opts.force_scale must be finite and >= 0");
  if (!(o->lbound >= 0.0 && o->lbound <= 1.0)) return set_error(SM_ERR_ARG, "opts.lbound out of [0, 1]");
  if (!(o->tol >= 0) || !(o->switch_tol >= 0) || !(o->stall_ratio >= 0) || !(o->stall_below >= 0) ||
      !(o->scale_margin >= 0))
    return set_error(SM_ERR_ARG, "negative or NaN tolerance in opts");
  return SM_OK;
}

int chunk_range(const sm_plan* p, int32_t chunk, int& g0, int& nsub) {
  const int nch = (int)p->chunk_ptr.size() - 1;
  if (chunk < 0 || chunk >= nch) return set_error(SM_ERR_ARG, "chunk %d out of [0, %d)", chunk, nch);
  g0 = (int)p->chunk_ptr[chunk];
  nsub = (int)(p->chunk_ptr[chunk + 1] - p->chunk_ptr[chunk]);
  return SM_OK;
}

struct WsPtrs {
  void* mats;
  TileRec* tiles;
  SubState* st;
  double* partials;
  int32_t* lists;
  float* features;
  double* scratch;
  double* vecs;
  int32_t* flag;
};

WsPtrs ws_ptrs(const sm_plan* p, void* ws, int storage) {
  const WsLayout L = p->layout(storage);
  char* w = static_cast<char*>(ws);
  return WsPtrs{w + L.mats, (TileRec*)(w + L.tiles), (SubState*)(w + L.state), (double*)(w + L.partials), (int32_t*)(w + L.lists),
                (float*)(w + L.features), (double*)(w + L.scratch), (double*)(w + L.vecs),
                (int32_t*)(w + L.flag)};
}

int64_t list_stride(const sm_plan* p) { return 2 + 2 * p->max_subs + 1; }

int chunk_tiles(const sm_plan* p, int g0, int nsub) {
  int64_t t = 0;
  for (int g = g0; g < g0 + nsub; ++g) {
    const int64_t T = tiles_of(p->npad_g[g]);
    t += T * (T + 1) / 2;
  }
  return (int)std::min<int64_t>(t, 1 << 30);
}

int chunk_max_tiles_sub(const sm_plan* p, int g0, int nsub) {
  int m = 0;
  for (int g = g0; g < g0 + nsub; ++g) {
    const int T = tiles_of(p->npad_g[g]);
    m = std::max(m, T * (T + 1) / 2);
  }
  return m;
}

// Launch one Newton-Schulz GEMM, bracketed by timing events when profiling.
// Variant that actually runs: the 128-wide tiles need n_pad % 64 == 0 and a
// float32-accumulating precision, otherwise the XCD-aware 64-wide kernel.
int effective_variant(const sm_plan* p, int mode, int variant) {
  int v = variant >= 0 ? variant : p->tuned_for(p->active_chunk)[mode];
  if (v >= 6 && mode < SM_BF16) v = 5;   // 256-wide tiles: 16-bit operand copies only
  if (v >= 3 && (mode == SM_F64 || p->pad_to < 64)) v = 1;
  // bf16 / f16 / split-bf16 on a plan padded to 32: only the half-depth
  // stages (k depth 32) divide n_pad
  if (mode >= SM_BF16 && p->pad_to < 64) v = 2;
  return v;
}

// Variant of the refinement products (opts->variant == -1): after a 16-bit
// main phase with at most two refinement steps, every refinement product is a
// slab product (the first refinement update runs on the main kernel; the
// square before the last update and that update take only the tile columns
// of the atom's own columns), and for those the 64-wide XCD-aware tiles
// waste the least (water, split bf16: 48 against 81 ms per pass on the
// 128-wide ring kernel); otherwise the tuned variant of the refinement
// precision.
int refine_variant(const sm_plan* p, const sm_sign_opts* o) {
  if (o->variant >= 0) return o->variant;
  if (o->phase1 >= SM_BF16 && o->refine_steps <= 2) return 1;
  return p->tuned_for(p->active_chunk)[o->refine];
}

int gemm_launch(sm_plan* p, int mode, int which, int variant, void* mats, int64_t shadow, const int32_t* cnt,
                const TileRec* recs, double* partials, unsigned* sync, int max_tiles, hipStream_t s) {
  const int v = effective_variant(p, mode, variant);
  // persistent grid: all resident workgroups, a multiple of the 8 XCDs
  int grid = std::min(max_tiles, p->num_cu * ns_gemm_blocks_per_cu(mode, which, v));
  grid = std::max(8, grid / 8 * 8);
  if (!p->profiling) {
    SM_HIP(launch_ns_gemm(mode, which, v, mats, shadow, cnt, recs, partials, sync, grid, s));
    return SM_OK;
  }
  const size_t k = p->prof_cls.size();
  while (p->prof_ev.size() < 2 * (k + 1)) {
    hipEvent_t e;
    SM_HIP(hipEventCreate(&e));
    p->prof_ev.push_back(e);
  }
  SM_HIP(launch_ns_gemm(mode, which, v, mats, shadow, cnt, recs, partials, sync, grid, s,
                        p->prof_ev[2 * k], p->prof_ev[2 * k + 1]));
  p->prof_cls.push_back(2 * mode + which);
  return SM_OK;
}

}  // namespace

extern "C" {

int sm_profile_enable(sm_plan* p, int32_t on) {
  if (!p) return set_error(SM_ERR_ARG, "sm_profile_enable: null plan");
  p->profiling = on != 0;
  return SM_OK;
}

int sm_profile_read(sm_plan* p, int64_t* launches, double* ms) {
  if (!p) return set_error(SM_ERR_ARG, "sm_profile_read: null plan");
  int64_t n[10] = {0};
  double t[10] = {0};
  for (size_t k = 0; k < p->prof_cls.size(); ++k) {
    SM_HIP(hipEventSynchronize(p->prof_ev[2 * k + 1]));
    float e = 0.f;
    SM_HIP(hipEventElapsedTime(&e, p->prof_ev[2 * k], p->prof_ev[2 * k + 1]));
    n[p->prof_cls[k]] += 1;
    t[p->prof_cls[k]] += e;
  }
  p->prof_cls.clear();
  if (launches) std::memcpy(launches, n, sizeof(n));
  if (ms) std::memcpy(ms, t, sizeof(t));
  return SM_OK;
}


int sm_plan_ws_layout(const sm_plan* p, int32_t storage_prec, int64_t* regions9, int64_t* mat_off_g) {
  if (!p) return set_error(SM_ERR_ARG, "sm_plan_ws_layout: null plan");
  if (!valid_storage(storage_prec)) return set_error(SM_ERR_ARG, "sm_plan_ws_layout: bad storage code %d", storage_prec);
  const WsLayout L = p->layout(storage_prec);
  if (regions9) {
    const int64_t r[9] = {L.mats, L.state, L.partials, L.lists, L.features, L.scratch, L.vecs, L.flag, L.total};
    std::memcpy(regions9, r, sizeof(r));
  }
  if (mat_off_g) std::memcpy(mat_off_g, p->mat_off_g.data(), p->mat_off_g.size() * 8);
  return SM_OK;
}

int build_submatrices(sm_plan* p, int32_t chunk, const double* H, double mu, const sm_sign_opts* o,
                      void* ws, sm_sub_stats* stats, void* stream) {
  if (!p || !H || !ws || !stats) return set_error(SM_ERR_ARG, "build_submatrices: null argument");
  if (!std::isfinite(mu)) return set_error(SM_ERR_ARG, "build_submatrices: mu is not finite");
  int rc = check_opts(o);
  if (rc) return rc;
  int g0, nsub;
  if ((rc = chunk_range(p, chunk, g0, nsub))) return rc;
  if ((rc = ensure_device(p))) return rc;
  const size_t lds = gather_lds_bytes(p->max_m, p->max_npad, false);   // gather: 4 row maps
  if (lds > 64 * 1024)
    return set_error(SM_ERR_ARG, "build_submatrices: index set too large for the gather (needs %zu B of LDS)", lds);
  // the gather also forms the first power-iteration product when the
  // schedule runs power steps and its partial sums fit the LDS
  const bool power_in_gather = o->scaling != SM_SCALE_GERSHGORIN && o->power_steps > 0 &&
                               gather_lds_bytes(p->max_m, p->max_npad, true) <= 64 * 1024;
  const int storage = ws_storage(o);
  const int f64 = storage == SM_F64;
  const int64_t shadow = storage >= SM_BF16 ? p->shadow_off() : 0;
  WsPtrs w = ws_ptrs(p, ws, storage);
  hipStream_t s = as_stream(stream);
  // the gather flags NaN / Inf in T straight into mapped host memory (reset
  // here in stream order); submatrix_sign reads it once its first poll has
  // waited past the gather
  int32_t* flag = p->d_pinned + 8;
  SM_HIP(launch_fill_i32(flag, 0, 1, s));
  double* cg = w.scratch;                                 // [max_subs]
  float* pred = reinterpret_cast<float*>(w.scratch + p->max_subs);  // [2 max_subs]
  const int shadow_kind = storage >= SM_BF16 ? storage : 0;
  SM_HIP(launch_gather(p->dev, g0, nsub, p->max_m, p->max_npad, H, mu, w.mats, f64, shadow_kind, shadow, flag,
                       w.features, cg, stats, power_in_gather ? w.vecs : nullptr, nullptr, s));
  const float* predp = nullptr;
  if (o->scaling == SM_SCALE_LEARNED) {
    if (!p->mlp) return set_error(SM_ERR_STATE, "build_submatrices: learned scaling needs a network (sm_plan_set_mlp)");
    if (p->mlp->device != p->device) return set_error(SM_ERR_STATE, "build_submatrices: network lives on another device");
    SM_HIP(launch_mlp_infer(p->mlp->theta, p->mlp->norm, w.features, kNumFeatures, nsub, pred, s));
    predp = pred;
  }
  SM_HIP(launch_scale(p->dev, g0, nsub, w.mats, f64, o->scaling, o->power_steps, o->scale_margin, w.vecs,
                      cg, predp, stats, shadow_kind, shadow, o->lbound, w.scratch + 2 * p->max_subs,
                      w.scratch + 3 * p->max_subs, w.scratch + 4 * p->max_subs, power_in_gather,
                      o->force_scale, nullptr, s));
  p->last_storage = storage;
  p->last_chunk = chunk;
  p->last_H = H;
  p->last_mu = mu;
  p->fd_chunk = -1;   // the workspace no longer holds a finite-temperature result
  return SM_OK;
}

int submatrix_sign(sm_plan* p, int32_t chunk, void* ws, const sm_sign_opts* o, sm_sub_stats* stats,
                   void* stream) {
  if (!p || !ws || !stats) return set_error(SM_ERR_ARG, "submatrix_sign: null argument");
  int rc = check_opts(o);
  if (rc) return rc;
  int g0, nsub;
  if ((rc = chunk_range(p, chunk, g0, nsub))) return rc;
  if ((rc = ensure_device(p))) return rc;
  const int storage = ws_storage(o);
  const int f64 = storage == SM_F64;
  const int64_t shadow = storage >= SM_BF16 ? p->shadow_off() : 0;
  if (p->last_storage != storage)
    return set_error(SM_ERR_STATE, "submatrix_sign: the workspace was not built for this precision schedule");
  p->fd_chunk = -1;
  p->active_chunk = chunk;   // its size class's GEMM variants
  WsPtrs w = ws_ptrs(p, ws, storage);
  hipStream_t s = as_stream(stream);   // the lambdas below launch on `s`
  // the round counters of the synchronized GEMM walk start at zero (a fill
  // kernel, outside any captured graph; each launch leaves them at zero)
  SM_HIP(launch_fill_i32(w.flag, 0, 16, s));
  const int64_t stride = list_stride(p);
  int32_t* L0 = w.lists;
  auto list_count = [&](int L) { return L0 + L * stride; };
  const int max_tiles = chunk_tiles(p, g0, nsub);
  const int max_tiles_sub = chunk_max_tiles_sub(p, g0, nsub);
  const int mode_main = o->phase1;
  const int mode_ref = o->refine;
  const bool has_ref = o->refine_steps > 0;
  const int ms = (int)p->max_subs;
  const int tsh_main = tile_shift(effective_variant(p, mode_main, o->variant), mode_main);
  const int var_ref = refine_variant(p, o);
  const int tsh_ref = tile_shift(effective_variant(p, mode_ref, var_ref), mode_ref);
  // tile records by list: 0 / 1 updates, 2 / 3 squares (main / refinement)
  auto recs_of = [&](int L) { return w.tiles + (int64_t)L * p->max_tiles; };
  // the main phase's products keep only 16-bit copies of their results; a
  // submatrix's first refinement update is run on those by the main kernel
  const int shadow_kind = storage >= SM_BF16 ? storage : 0;
  // the scheduler's lists -> tile records of this iteration's updates and
  // the next iteration's squares (one launch; written by the scheduler's
  // single workgroup itself they cost 49 instead of 4 us on the lattice)
  auto expand = [&]() -> int {
    SM_HIP(launch_expand(p->dev, g0, w.st, w.lists, ms, w.tiles, p->max_tiles, tsh_main, tsh_ref, has_ref,
                         nsub, s));
    return SM_OK;
  };
  // the GEMMs of kind `which` over lists Lm (main precision) and Lr
  // (refinement); a list the host knows to be empty is not launched
  auto gemms = [&](int Lm, int Lr, int which, bool run_main, bool run_ref) -> int {
    int r;
    unsigned* sync = reinterpret_cast<unsigned*>(w.flag);
    if (run_main && (r = gemm_launch(p, mode_main, which, o->variant, w.mats, shadow, list_count(Lm),
                                     recs_of(Lm), w.partials, sync, max_tiles, s)))
      return r;
    if (has_ref && run_ref && (r = gemm_launch(p, mode_ref, which, var_ref, w.mats, shadow, list_count(Lr),
                                               recs_of(Lr), w.partials, sync, max_tiles, s)))
      return r;
    return SM_OK;
  };
  // the schedule the scheduler applies: opts, or the fallback of the retry
  const sm_sign_opts* cur = o;
  // the first squares' column-sum bounds (scaled runs, accel 1)
  double* colmax = w.scratch + 6 * p->max_subs;
  auto schedule = [&](int first, int32_t* live_host) -> int {
    SM_HIP(launch_schedule(p->dev, g0, nsub, w.st, w.partials, w.lists, ms, *cur, first, tsh_main, tsh_ref,
                           first ? w.scratch + 2 * p->max_subs : nullptr,
                           first ? w.scratch + 3 * p->max_subs : nullptr,
                           first ? w.scratch + 4 * p->max_subs : nullptr, live_host, max_tiles_sub, colmax, s));
    return SM_OK;
  };
  // one iteration: squares (A = X^2, Y = 3I - A), residuals + scheduler,
  // tile records, updates (X' = 1/2 X Y).  live_host / ev: the scheduler's
  // counts and an event recorded after it; sq_main / sq_ref: whether the
  // square lists may be non-empty; upd_ref: launch the refinement updates now
  // (otherwise the host launches them after reading the scheduler's count,
  // still before the next squares).  A main-precision update needs a
  // main-precision square in the same iteration.
  // first_it: the first iteration of a scaled run (accel 1), whose squares
  // may have run unscaled: their column-sum bounds before the scheduler,
  // and Y formed for the first updates after it.
  auto iteration = [&](hipStream_t st, int32_t* live_host, hipEvent_t ev, bool sq_main, bool sq_ref,
                       bool upd_ref, bool first_it) -> int {
    hipStream_t keep = s;
    s = st;
    const bool amode = first_it && cur->accel == 1;
    int r = gemms(2, 3, 0, sq_main, sq_ref);
    if (!r && amode) {
      hipError_t e = launch_first_colmax(p->dev, g0, nsub, w.mats, storage, shadow, w.st, colmax, s);
      if (e != hipSuccess) r = hip_error(e, "first_colmax");
    }
    if (!r) r = schedule(0, live_host);
    if (!r && amode) {
      hipError_t e = launch_first_fix_y(p->dev, g0, nsub, p->max_npad, w.mats, storage, shadow, w.st, s);
      if (e != hipSuccess) r = hip_error(e, "first_fix_y");
    }
    if (!r && ev) {
      hipError_t e = hipEventRecord(ev, st);
      if (e != hipSuccess) r = hip_error(e, "hipEventRecord");
    }
    if (!r) r = expand();
    if (!r) r = gemms(0, 1, 1, sq_main, upd_ref);
    s = keep;
    return r;
  };
  // a NaN / Inf in T (flagged by the gather) ends the call at the first poll
  auto nonfinite = [&]() -> int {
    const int32_t f = p->h_pinned[8];
    if (f != 0) return set_error(SM_ERR_NONFINITE, "submatrix_sign: NaN/Inf in submatrix of atom %d", f - 1);
    return SM_OK;
  };

  // the host waits for each iteration's scheduler while that iteration's
  // updates run, stops as soon as no submatrix squares again, and launches
  // only the GEMMs whose lists can be non-empty: squares as counted by the
  // previous scheduler; refinement updates right away only while
  // submatrices refine (a submatrix entering refinement gets its first
  // refinement update launched once the count shows it); no submatrix
  // refines before its first square
  auto eager_loop = [&](int lim) -> int {
    bool sq_main = true, sq_ref = false;
    int r;
    for (int it = 0; it <= lim; ++it) {
      const int slot = kHostCounts + 4 * (it & 1);
      const bool upd_ref = sq_ref;
      if ((r = iteration(s, p->d_pinned + slot, p->ev[it & 1], sq_main, sq_ref, upd_ref, it == 0))) return r;
      SM_HIP(hipEventSynchronize(p->ev[it & 1]));
      if (it == 0 && (r = nonfinite())) return r;
      const int32_t* hc = p->h_pinned + slot;
      if (!upd_ref && hc[3] > 0 && (r = gemms(0, 1, 1, false, true))) return r;
      if (hc[0] == 0) break;
      sq_main = hc[1] > 0;
      sq_ref = hc[2] > 0;
    }
    return SM_OK;
  };

  // bounds on the spectrum of X_0 written by build_submatrices (scaled
  // Newton-Schulz), then the first squares' records
  if ((rc = schedule(1, nullptr)) || (rc = expand())) return rc;
  const int lim = o->max_iter + o->refine_steps + 2;
  const int G = p->profiling ? 0 : o->graph_iters;
  if (G == 0) {
    if ((rc = eager_loop(lim))) return rc;
  } else {
    // find or capture the graph of G iterations for this chunk / workspace / schedule
    hipGraphExec_t exec = nullptr;
    for (auto& e : p->graphs)
      if (e.chunk == chunk && e.ws == ws && std::memcmp(&e.opts, o, sizeof(*o)) == 0 &&
          std::memcmp(e.tuned, p->tuned_for(chunk), sizeof(e.tuned)) == 0)
        exec = e.exec;
    if (!exec) {
      if (!p->capture_stream) SM_HIP(hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking));
      for (int m = 0; m < 5; ++m)                    // occupancy queries outside the capture
        for (int wh = 0; wh < 2; ++wh) {
          (void)ns_gemm_blocks_per_cu(m, wh, effective_variant(p, m, o->variant));
          (void)ns_gemm_blocks_per_cu(m, wh, effective_variant(p, m, var_ref));
        }
      SM_HIP(hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal));
      int r = SM_OK;
      for (int k = 0; k < G && !r; ++k) r = iteration(p->capture_stream, nullptr, nullptr, true, true, true, false);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(p->capture_stream, &graph);
      if (r) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
      }
      if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return hip_error(e, "hipGraphInstantiate");
      sm_plan::GraphEntry ge{chunk, ws, *o, {0}, exec};
      std::memcpy(ge.tuned, p->tuned_for(chunk), sizeof(ge.tuned));
      p->graphs.push_back(ge);
    }
    // the first iteration outside the graph (its squares' bounds and the
    // forming of Y run only there)
    if ((rc = iteration(s, nullptr, nullptr, true, true, true, true))) return rc;
    const int replays = (lim + G) / G;
    for (int r = 0; r < replays; ++r) {
      SM_HIP(hipGraphLaunch(exec, s));
      SM_HIP(hipMemcpyAsync(&p->h_pinned[r & 1], L0 + 4 * stride, 4, hipMemcpyDeviceToHost, s));
      SM_HIP(hipEventRecord(p->ev[r & 1], s));
      if (r >= 1) {
        SM_HIP(hipEventSynchronize(p->ev[(r - 1) & 1]));
        if (r == 1 && (rc = nonfinite())) return rc;
        if (p->h_pinned[(r - 1) & 1] == 0) break;
      }
    }
    if (replays == 1) {
      SM_HIP(hipEventSynchronize(p->ev[0]));
      if ((rc = nonfinite())) return rc;
    }
  }
  // fallback retry: submatrices that did not converge or diverged are built
  // again from H and run once more with Gershgorin scaling and plain
  // Newton-Schulz (a scale or bound that misled the first run is not used
  // again) and twice the iteration cap; the others keep their result
  if (o->retry) {
    if (p->last_chunk != chunk || !p->last_H)
      return set_error(SM_ERR_STATE, "submatrix_sign: retry needs the build_submatrices call of this chunk");
    int32_t* fail = reinterpret_cast<int32_t*>(w.scratch + 5 * p->max_subs);
    SM_HIP(launch_collect_failed(nsub, w.st, fail, p->d_pinned + kHostRetry, s));
    SM_HIP(hipStreamSynchronize(s));
    const int nfail = p->h_pinned[kHostRetry];
    if (nfail > 0) {
      sm_sign_opts fb = *o;
      fb.scaling = SM_SCALE_GERSHGORIN;
      fb.accel = 0;
      fb.lbound = 0.0;
      fb.force_scale = 0.0;
      fb.retry = 0;
      fb.graph_iters = 0;
      fb.max_iter = std::min(std::max(2 * o->max_iter, 1), 1000);
      const int shadow_kind_b = storage >= SM_BF16 ? storage : 0;
      SM_HIP(launch_fill_i32(p->d_pinned + 8, 0, 1, s));
      SM_HIP(launch_gather(p->dev, g0, nfail, p->max_m, p->max_npad, p->last_H, p->last_mu, w.mats, f64,
                           shadow_kind_b, shadow, p->d_pinned + 8, w.features, w.scratch, stats, nullptr, fail, s));
      SM_HIP(launch_scale(p->dev, g0, nfail, w.mats, f64, SM_SCALE_GERSHGORIN, 0, 0.0, w.vecs, w.scratch, nullptr,
                          stats, shadow_kind_b, shadow, 0.0, w.scratch + 2 * p->max_subs,
                          w.scratch + 3 * p->max_subs, w.scratch + 4 * p->max_subs, false, 0.0, fail, s));
      cur = &fb;
      if ((rc = schedule(2, nullptr)) || (rc = expand())) return rc;
      rc = eager_loop(fb.max_iter + fb.refine_steps + 2);
      cur = o;
      if (rc) return rc;
    }
  }
  if (!f64)   // float32 final X where only its copies, or T (X = X_0), are in the buffer
    SM_HIP(launch_materialize(p->dev, g0, nsub, (float*)w.mats, w.st, shadow_kind, shadow, s));
  SM_HIP(launch_finish(p->dev, g0, nsub, w.mats, f64, w.st, o->probes, w.vecs, stats, p->max_npad, s));
  return SM_OK;
}

int sm_comm_probe(sm_plan* p, int32_t chunk, const double* H, double mu, const sm_sign_opts* o, void* ws,
                  sm_sub_stats* stats, void* stream) {
  if (!p || !H || !ws || !stats) return set_error(SM_ERR_ARG, "sm_comm_probe: null argument");
  int rc = check_opts(o);
  if (rc) return rc;
  if (o->comm_probes < 1) return set_error(SM_ERR_ARG, "sm_comm_probe: opts.comm_probes must be 1..4");
  int g0, nsub;
  if ((rc = chunk_range(p, chunk, g0, nsub))) return rc;
  if ((rc = ensure_device(p))) return rc;
  const int storage = ws_storage(o);
  if (p->last_storage != storage)
    return set_error(SM_ERR_STATE, "sm_comm_probe: the workspace was not built for this precision schedule");
  WsPtrs w = ws_ptrs(p, ws, storage);
  SM_HIP(launch_comm_probe(p->dev, g0, nsub, p->max_m, p->max_npad, H, mu, w.mats, storage == SM_F64, w.st,
                           o->comm_probes, w.vecs, stats, as_stream(stream)));
  return SM_OK;
}

int assemble_P(const sm_plan* p, int32_t chunk, const void* ws, double* P, void* stream) {
  if (!p || !ws || !P) return set_error(SM_ERR_ARG, "assemble_P: null argument");
  int g0, nsub, rc;
  if ((rc = chunk_range(p, chunk, g0, nsub))) return rc;
  if (p->device < 0) return set_error(SM_ERR_STATE, "assemble_P: plan has not been used on a device yet");
  const int storage = p->last_storage;
  if (storage < 0) return set_error(SM_ERR_STATE, "assemble_P: no submatrices built");
  const int f64 = storage == SM_F64;
  WsPtrs w = ws_ptrs(p, const_cast<void*>(ws), storage);
  SM_HIP(launch_scatter(p->dev, g0, nsub, w.mats, f64, w.st, P, as_stream(stream)));
  return SM_OK;
}

int energy_trace(const sm_plan* pc, const double* H, const double* P, double* E, double* Ne, void* stream) {
  if (!pc || !H || !P) return set_error(SM_ERR_ARG, "energy_trace: null argument");
  sm_plan* p = const_cast<sm_plan*>(pc);
  int rc;
  if ((rc = ensure_device(p))) return rc;
  hipStream_t s = as_stream(stream);
  // the final reduction writes E and Ne straight into mapped host memory
  SM_HIP(launch_trace(H, P, p->nvals, p->d_diag_idx, (int64_t)p->diag_idx.size(), p->d_trace_parts,
                      kTraceBlocks, reinterpret_cast<double*>(p->d_pinned + kHostTrace), s));
  SM_HIP(hipStreamSynchronize(s));
  const double* h = reinterpret_cast<const double*>(p->h_pinned + kHostTrace);
  if (E) *E = h[0];
  if (Ne) *Ne = h[1];
  return SM_OK;
}

int sm_density_matrix(sm_plan* p, const double* H, double mu, const sm_sign_opts* o, void* ws,
                      double* P, sm_sub_stats* stats, double* E, double* Ne, void* stream) {
  if (!p) return set_error(SM_ERR_ARG, "sm_density_matrix: null plan");
  const int nch = (int)p->chunk_ptr.size() - 1;
  int rc;
  for (int c = 0; c < nch; ++c) {
    if ((rc = build_submatrices(p, c, H, mu, o, ws, stats, stream))) return rc;
    if ((rc = submatrix_sign(p, c, ws, o, stats, stream))) return rc;
    if (o->comm_probes > 0 && (rc = sm_comm_probe(p, c, H, mu, o, ws, stats, stream))) return rc;
    if ((rc = assemble_P(p, c, ws, P, stream))) return rc;
  }
  return energy_trace(p, H, P, E, Ne, stream);
}

int sm_gershgorin_bracket(sm_plan* p, const double* H, double* lo, double* hi, void* stream) {
  if (!p || !H || !lo || !hi) return set_error(SM_ERR_ARG, "sm_gershgorin_bracket: null argument");
  int rc;
  if ((rc = ensure_device(p))) return rc;
  hipStream_t s = as_stream(stream);
  SM_HIP(launch_gersh_rows(p->dev, p->n_atoms, H, p->d_gersh,
                           reinterpret_cast<double*>(p->d_pinned + kHostBracket), s));
  SM_HIP(hipStreamSynchronize(s));
  const double* h = reinterpret_cast<const double*>(p->h_pinned + kHostBracket);
  *lo = h[0];
  *hi = h[1];
  return SM_OK;
}

int sm_gershgorin_bracket_noalloc(const sm_plan* p, const double* H, double* lohi, void* stream) {
  if (!p || !H || !lohi) return set_error(SM_ERR_ARG, "sm_gershgorin_bracket_noalloc: null argument");
  if (p->n_atoms > kNoAllocMaxAtoms)
    return set_error(SM_ERR_ARG, "sm_gershgorin_bracket_noalloc: %d atoms exceed the fixed scratch of %d atoms",
                     p->n_atoms, kNoAllocMaxAtoms);
  if (p->device < 0)
    return set_error(SM_ERR_STATE, "sm_gershgorin_bracket_noalloc: the plan has no device tables yet "
                                   "(make one device call with it first, e.g. sm_gershgorin_bracket)");
  int dev = -1;
  SM_HIP(hipGetDevice(&dev));
  if (dev != p->device)
    return set_error(SM_ERR_STATE, "sm_gershgorin_bracket_noalloc: plan lives on device %d, device %d is current",
                     p->device, dev);
  SM_HIP(launch_gersh_rows_noalloc(p->dev, p->n_atoms, H, lohi, as_stream(stream)));
  return SM_OK;
}

int sm_find_mu(sm_plan* p, const double* H, double n_target, double accept, int32_t max_steps,
               double mu_start, const sm_sign_opts* o, void* ws, double* P, sm_sub_stats* stats, double* mu_out,
               int32_t* steps_out, double* mu_hist, double* ne_hist, double* E_out, double* Ne_out,
               void* stream) {
  if (!p || !H || !ws || !stats || !mu_out) return set_error(SM_ERR_ARG, "sm_find_mu: null argument");
  if (max_steps < 1 || max_steps > 200) return set_error(SM_ERR_ARG, "sm_find_mu: max_steps out of [1, 200]");
  if (!(accept > 0)) return set_error(SM_ERR_ARG, "sm_find_mu: accept must be > 0");
  int rc = check_opts(o);
  if (rc) return rc;
  double lo, hi;
  if ((rc = sm_gershgorin_bracket(p, H, &lo, &hi, stream))) return rc;
  hipStream_t s = as_stream(stream);
  const int nch = (int)p->chunk_ptr.size() - 1;
  // a finite mu_start is evaluated first (warm start); if it is not
  // accepted it narrows the bracket like any midpoint, clamped into it
  const bool warm = std::isfinite(mu_start);
  double mid = 0.5 * (lo + hi);
  int step = 1;
  for (; step <= max_steps; ++step) {
    mid = (warm && step == 1) ? mu_start : 0.5 * (lo + hi);
    for (int c = 0; c < nch; ++c) {
      if ((rc = build_submatrices(p, c, H, mid, o, ws, stats, stream))) return rc;
      if ((rc = submatrix_sign(p, c, ws, o, stats, stream))) return rc;
      if (o->comm_probes > 0 && (rc = sm_comm_probe(p, c, H, mid, o, ws, stats, stream))) return rc;
      int g0, nsub;
      chunk_range(p, c, g0, nsub);
      WsPtrs w = ws_ptrs(p, ws, ws_storage(o));
      SM_HIP(launch_ne_from_x(p->dev, g0, nsub, w.mats, storage_is_f64(o), w.st, p->d_ne_sub, s));
      if (P && (rc = assemble_P(p, c, ws, P, stream))) return rc;
    }
    // tr(P H), tr P of this pass's P when asked for (so the accepted pass
    // needs no further round trip), and the compensated sum of the electron
    // counts over the atoms, all into mapped host memory
    const bool trace = P && (E_out || Ne_out);
    if (trace)
      SM_HIP(launch_trace(H, P, p->nvals, p->d_diag_idx, (int64_t)p->diag_idx.size(), p->d_trace_parts,
                          kTraceBlocks, reinterpret_cast<double*>(p->d_pinned + kHostTrace), s));
    SM_HIP(launch_ne_sum(p->d_ne_sub, p->n_atoms, reinterpret_cast<double*>(p->d_pinned + kHostNe), s));
    SM_HIP(hipStreamSynchronize(s));
    if (trace) {
      const double* h = reinterpret_cast<const double*>(p->h_pinned + kHostTrace);
      if (E_out) *E_out = h[0];
      if (Ne_out) *Ne_out = h[1];
    }
    const double ne = *reinterpret_cast<const double*>(p->h_pinned + kHostNe);
    if (mu_hist) mu_hist[step - 1] = mid;
    if (ne_hist) ne_hist[step - 1] = ne;
    if (std::fabs(ne - n_target) < accept) break;
    if (ne < n_target) lo = std::min(std::max(lo, mid), hi);
    else hi = std::max(std::min(hi, mid), lo);
  }
  *mu_out = mid;
  if (steps_out) *steps_out = std::min(step, (int)max_steps);
  return SM_OK;
}

int sm_autotune(sm_plan* p, int32_t chunk, const double* H, double mu, const sm_sign_opts* o, void* ws,
                sm_sub_stats* stats, int32_t repeats, int32_t variant_mask, int32_t* best_out,
                double* times_ms, void* stream) {
  int rc = check_opts(o);
  if (rc) return rc;
  if (!p || !H || !ws || !stats) return set_error(SM_ERR_ARG, "sm_autotune: null argument");
  if (repeats < 1 || repeats > 20) return set_error(SM_ERR_ARG, "sm_autotune: repeats out of [1, 20]");
  if (chunk < 0 || chunk >= (int)p->chunk_class.size())
    return set_error(SM_ERR_ARG, "sm_autotune: chunk %d out of [0, %d)", chunk, (int)p->chunk_class.size());
  if ((rc = ensure_device(p))) return rc;
  hipStream_t s = as_stream(stream);
  hipEvent_t e0, e1;
  SM_HIP(hipEventCreate(&e0));
  SM_HIP(hipEventCreate(&e1));
  double best_t = 1e300;
  int best = -1;
  for (int v = 0; v < kGemmVariants; ++v) {
    sm_sign_opts ov = *o;
    ov.variant = v;
    double tv = 1e300;
    if ((variant_mask && !(variant_mask & (1 << v))) ||
        (v >= 3 && effective_variant(p, o->phase1, v) != v)) {   // not requested / no 128-wide kernel
      if (times_ms) times_ms[v] = -1.0;
      continue;
    }
    for (int r = 0; r < repeats; ++r) {
      if ((rc = build_submatrices(p, chunk, H, mu, &ov, ws, stats, stream))) break;
      SM_HIP(hipEventRecord(e0, s));
      if ((rc = submatrix_sign(p, chunk, ws, &ov, stats, stream))) break;
      SM_HIP(hipEventRecord(e1, s));
      SM_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      SM_HIP(hipEventElapsedTime(&ms, e0, e1));
      tv = std::min(tv, (double)ms);
    }
    if (rc) break;
    if (times_ms) times_ms[v] = tv;
    if (tv < best_t) {
      best_t = tv;
      best = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (best < 0) return set_error(SM_ERR_ARG, "sm_autotune: no variant selected by the mask");
  // the plan-wide choice, and that of the chunk's size class (which its
  // chunks use from now on)
  // (the refinement precision's entry too when it is the same kind of
  // product: after a float64 main phase; see refine_variant)
  const bool ref_too = o->refine_steps > 0 && o->phase1 < SM_BF16;
  p->tuned[o->phase1] = best;
  if (ref_too) p->tuned[o->refine] = best;
  auto& ct = p->class_tuned[p->chunk_class[chunk]];
  ct[o->phase1] = best;
  if (ref_too) ct[o->refine] = best;
  if (best_out) *best_out = best;
  return SM_OK;
}

int32_t sm_gemm_variants(void) { return kGemmVariants; }

int sm_plan_chunk_variants(const sm_plan* p, int32_t chunk, int32_t* class_out, int32_t* variants_out) {
  if (!p) return set_error(SM_ERR_ARG, "sm_plan_chunk_variants: null plan");
  if (chunk < 0 || chunk >= (int)p->chunk_class.size())
    return set_error(SM_ERR_ARG, "sm_plan_chunk_variants: chunk %d out of [0, %d)", chunk, (int)p->chunk_class.size());
  if (class_out) *class_out = p->chunk_class[chunk];
  if (variants_out) std::memcpy(variants_out, p->tuned_for(chunk), 5 * sizeof(int32_t));
  return SM_OK;
}

int sm_plan_tuning(sm_plan* p, int32_t* get, const int32_t* set) {
  if (!p) return set_error(SM_ERR_ARG, "sm_plan_tuning: null plan");
  if (get) std::memcpy(get, p->tuned, sizeof(p->tuned));
  if (set) {
    for (int k = 0; k < 5; ++k)
      if (set[k] < 0 || set[k] >= kGemmVariants) return set_error(SM_ERR_ARG, "sm_plan_tuning: variant out of range");
    std::memcpy(p->tuned, set, sizeof(p->tuned));
    for (int32_t c : p->chunk_class) std::memcpy(p->class_tuned[c].data(), set, sizeof(p->tuned));
  }
  return SM_OK;
}

int sm_selftest_mfma(int32_t prec, double* out_host) {
  if (!out_host) return set_error(SM_ERR_ARG, "sm_selftest_mfma: null output");
  if (prec < SM_F64 || prec > 6) return set_error(SM_ERR_ARG, "sm_selftest_mfma: bad instruction code %d", prec);
  const size_t nout = prec >= 5 ? 1024 : 256;
  double* d = nullptr;
  SM_HIP(hipMalloc(&d, nout * sizeof(double)));
  hipError_t e = launch_selftest_mfma(prec, d, nullptr);
  if (e == hipSuccess) e = hipMemcpy(out_host, d, nout * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return hip_error(e, "sm_selftest_mfma");
  return SM_OK;
}

}  // extern "C"
