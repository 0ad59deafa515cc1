// C-ABI entry points of the non-orthogonal basis (S != I): Eq. 12 for the
// inverse square roots of the overlap submatrices, Eq. 14 on the submatrix
// pair, all in float64 (see k_ovl.hip for the arithmetic).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "plan.h"

using namespace sm;

namespace {

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int chunk_range(const sm_plan* p, int32_t chunk, int& g0, int& nsub) {
  const int nch = (int)p->chunk_ptr.size() - 1;
  if (chunk < 0 || chunk >= nch) return set_error(SM_ERR_ARG, "chunk %d out of [0, %d)", chunk, nch);
  g0 = (int)p->chunk_ptr[chunk];
  nsub = (int)(p->chunk_ptr[chunk + 1] - p->chunk_ptr[chunk]);
  return SM_OK;
}

}  // namespace

namespace sm {

double* f64_mats(const sm_plan* p, const void* ws) {
  return reinterpret_cast<double*>(static_cast<char*>(const_cast<void*>(ws)) + p->layout(SM_F64).mats);
}

int ensure_ovl(sm_plan* p) {
  int rc;
  if ((rc = ensure_device(p))) return rc;
  // 128-wide tiles once a submatrix spans two of them (the 64-wide kernel
  // for smaller ones: less padding work)
  if (p->ovl_edge == 0) p->ovl_edge = p->max_npad >= 256 ? 128 : 64;
  if (!p->d_ovl) {
    void* d = nullptr;
    SM_HIP(hipMalloc(&d, std::max<int64_t>(p->max_subs, 1) * 4 * sizeof(double)));
    p->dev_allocs.push_back(d);
    p->d_ovl = static_cast<double*>(d);
    SM_HIP(hipMalloc(&d, std::max<int64_t>(p->max_subs, 1) * sizeof(int32_t)));
    p->dev_allocs.push_back(d);
    p->d_ovl_xbuf = static_cast<int32_t*>(d);
  }
  return SM_OK;
}

// The tile list of a product kind over a chunk (built once, kept on the device).
int ovl_jobs(sm_plan* p, int chunk, int kind, const OvlJob** jobs, int* n) {
  for (auto& e : p->ovl_jobs)
    if (e.chunk == chunk && e.kind == kind) {
      *jobs = e.d;
      *n = e.n;
      return SM_OK;
    }
  int g0, nsub, rc;
  if ((rc = chunk_range(p, chunk, g0, nsub))) return rc;
  std::vector<OvlJob> v;
  for (int l = 0; l < nsub; ++l) {
    const int g = g0 + l;
    const int e = p->ovl_edge;
    const int T = (p->npad_g[g] + e - 1) / e;
    const int i = p->order_g[g];
    for (int bj = 0; bj < T; ++bj) {
      if (kind == 2 && (bj < p->loc[i] / e || bj > (p->loc[i] + p->bs[i] - 1) / e)) continue;
      for (int bi = (kind == 0 ? bj : 0); bi < T; ++bi) v.push_back(OvlJob{l, (int16_t)bi, (int16_t)bj});
    }
  }
  void* d = nullptr;
  SM_HIP(hipMalloc(&d, std::max<size_t>(v.size(), 1) * sizeof(OvlJob)));
  p->dev_allocs.push_back(d);
  if (!v.empty()) SM_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(OvlJob), hipMemcpyHostToDevice));
  p->ovl_jobs.push_back(sm_plan::OvlJobs{chunk, kind, (int)v.size(), static_cast<OvlJob*>(d)});
  *jobs = static_cast<OvlJob*>(d);
  *n = (int)v.size();
  return SM_OK;
}

}  // namespace sm

namespace {

int check_schedule(const sm_sign_opts* o, const char* who) {
  if (!o) return set_error(SM_ERR_ARG, "%s: null sm_sign_opts", who);
  if (o->phase1 != SM_F64 || o->refine_steps != 0)
    return set_error(SM_ERR_ARG, "%s: the non-orthogonal path runs the float64 schedule without refinement steps", who);
  if (o->scaling == SM_SCALE_LEARNED)
    return set_error(SM_ERR_ARG, "%s: learned scaling is not available for the non-orthogonal path", who);
  if (o->retry != 0)
    return set_error(SM_ERR_ARG, "%s: the fallback retry builds from H alone; set retry = 0 for S != I", who);
  return SM_OK;
}

}  // namespace

extern "C" {

int sm_overlap_inv_sqrt(sm_plan* p, int32_t chunk, const double* S, double tol, int32_t max_iter, void* ws_aux,
                        void* ws, int32_t* iters_out, double* res_out, void* stream) {
  if (!p || !S || !ws_aux || !ws) return set_error(SM_ERR_ARG, "sm_overlap_inv_sqrt: null argument");
  if (!(tol > 0) || max_iter < 1 || max_iter > 200)
    return set_error(SM_ERR_ARG, "sm_overlap_inv_sqrt: tol must be > 0 and max_iter in [1, 200]");
  int g0, nsub, rc;
  if ((rc = chunk_range(p, chunk, g0, nsub))) return rc;
  if ((rc = ensure_ovl(p))) return rc;
  const OvlJob* jobs;
  int nj;
  if ((rc = ovl_jobs(p, chunk, 0, &jobs, &nj))) return rc;
  hipStream_t s = as_stream(stream);
  double* aux = f64_mats(p, ws_aux);
  double* wm = f64_mats(p, ws);
  double* c = p->d_ovl;                    // Gershgorin bound of T(S)
  double* res = p->d_ovl + p->max_subs;    // ||Z Y - I||_F^2 per submatrix
  const int mp = p->max_npad;
  // Y_0 = T(S) / c (ws buffer 0, identity pad), Z_0 = I (aux buffer 0)
  SM_HIP(launch_ovl_fill(p->dev, g0, nsub, mp, wm, 0, 0.0, 1.0, s));
  SM_HIP(launch_ovl_gather(p->dev, g0, nsub, p->max_m, S, wm, 0, s));
  SM_HIP(launch_ovl_gersh(p->dev, g0, nsub, wm, 0, c, 0, nullptr, s));
  SM_HIP(launch_ovl_scale(p->dev, g0, nsub, mp, wm, 0, c, 1, s));
  SM_HIP(launch_ovl_fill(p->dev, g0, nsub, mp, aux, 0, 1.0, 1.0, s));
  int y = 0, z = 0, it = 0;
  double r = INFINITY;
  if (p->fd_ws == ws || p->fd_ws == ws_aux) p->fd_chunk = -1;   // both workspaces are overwritten
  const double* hres = reinterpret_cast<const double*>(p->h_pinned + kHostOvl);
  double* dres = reinterpret_cast<double*>(p->d_pinned + kHostOvl);
  for (;; ++it) {
    // W = 1/2 (3I - Z Y) into aux buffer 2, with ||Z Y - I||_F^2
    SM_HIP(launch_ovl_zero(res, nsub, s));
    SM_HIP(launch_ovl_prod(p->dev, g0, jobs, nj, p->ovl_edge, aux, z, nullptr, wm, y, aux, 2, nullptr, -0.5, 1.5,
                           nullptr, 0, 0.0, 0, res, s));
    SM_HIP(launch_ovl_max(res, nsub, dres, s));
    SM_HIP(hipStreamSynchronize(s));
    r = std::sqrt(*hres);
    if (!std::isfinite(r)) return set_error(SM_ERR_NONFINITE, "sm_overlap_inv_sqrt: non-finite residual at step %d", it);
    if (r < tol || it >= max_iter) break;
    // Y <- Y W (ws buffers 0 / 1), Z <- W Z (aux buffers 0 / 1)
    SM_HIP(launch_ovl_prod(p->dev, g0, jobs, nj, p->ovl_edge, wm, y, nullptr, aux, 2, wm, 1 - y, nullptr, 1.0, 0.0,
                           nullptr, 0, 0.0, 0, nullptr, s));
    SM_HIP(launch_ovl_prod(p->dev, g0, jobs, nj, p->ovl_edge, aux, 2, nullptr, aux, z, aux, 1 - z, nullptr, 1.0, 0.0,
                           nullptr, 0, 0.0, 0, nullptr, s));
    y = 1 - y;
    z = 1 - z;
  }
  if (z != 0) SM_HIP(launch_ovl_copy(p->dev, g0, nsub, mp, aux, z, 0, s));
  // Z = (T(S) / c)^(-1/2) -> T(S)^(-1/2) = Z / sqrt(c) (the pad stays the identity)
  SM_HIP(launch_ovl_scale(p->dev, g0, nsub, mp, aux, 0, c, 2, s));
  SM_HIP(hipStreamSynchronize(s));
  p->ovl_chunk = chunk;
  p->ovl_aux = ws_aux;
  if (iters_out) *iters_out = it;
  if (res_out) *res_out = r;
  if (r >= tol) return set_error(SM_ERR_STATE, "sm_overlap_inv_sqrt: residual %.3e after %d steps (tol %.1e)", r, it, tol);
  return SM_OK;
}

int build_submatrices_overlap(sm_plan* p, int32_t chunk, const double* H, double mu, const sm_sign_opts* o,
                              void* ws, const void* ws_aux, sm_sub_stats* stats, void* stream) {
  if (!p || !H || !ws || !ws_aux || !stats) return set_error(SM_ERR_ARG, "build_submatrices_overlap: null argument");
  if (!std::isfinite(mu)) return set_error(SM_ERR_ARG, "build_submatrices_overlap: mu is not finite");
  int rc;
  if ((rc = check_schedule(o, "build_submatrices_overlap"))) return rc;
  if (p->ovl_chunk != chunk || p->ovl_aux != ws_aux)
    return set_error(SM_ERR_STATE, "build_submatrices_overlap: run sm_overlap_inv_sqrt for chunk %d into this "
                                   "auxiliary workspace first", chunk);
  int g0, nsub;
  if ((rc = chunk_range(p, chunk, g0, nsub))) return rc;
  if ((rc = ensure_ovl(p))) return rc;
  const OvlJob *sym, *full;
  int ns, nf;
  if ((rc = ovl_jobs(p, chunk, 0, &sym, &ns)) || (rc = ovl_jobs(p, chunk, 1, &full, &nf))) return rc;
  hipStream_t s = as_stream(stream);
  const double* aux = f64_mats(p, ws_aux);
  double* wm = f64_mats(p, ws);
  const int mp = p->max_npad;
  const WsLayout L = p->layout(SM_F64);
  double* scratch = reinterpret_cast<double*>(static_cast<char*>(ws) + L.scratch);
  double* vecs = reinterpret_cast<double*>(static_cast<char*>(ws) + L.vecs);
  // T(H) (zero pad) -> ws buffer 1; Q = T(H) Z -> buffer 2; K - mu I = Q^T Z -> buffer 0
  SM_HIP(launch_ovl_fill(p->dev, g0, nsub, mp, wm, 1, 0.0, 0.0, s));
  SM_HIP(launch_ovl_gather(p->dev, g0, nsub, p->max_m, H, wm, 1, s));
  SM_HIP(launch_ovl_prod(p->dev, g0, full, nf, p->ovl_edge, wm, 1, nullptr, aux, 0, wm, 2, nullptr, 1.0, 0.0, nullptr,
                         0, 0.0, 1, nullptr, s));
  SM_HIP(launch_ovl_prod(p->dev, g0, sym, ns, p->ovl_edge, wm, 2, nullptr, aux, 0, wm, 0, nullptr, 1.0, -mu, nullptr,
                         0, 0.0, 0, nullptr, s));
  // the identity pad of the sign iteration, its Gershgorin bound (stats.gersh),
  // then the scale and X_0 = T / c exactly as build_submatrices leaves them
  double* cg = scratch;
  SM_HIP(launch_ovl_gersh(p->dev, g0, nsub, wm, 0, cg, 1, stats, s));
  SM_HIP(launch_scale(p->dev, g0, nsub, wm, 1, o->scaling, o->power_steps, o->scale_margin, vecs, cg, nullptr, stats,
                      0, 0, o->lbound, scratch + 2 * p->max_subs, scratch + 3 * p->max_subs,
                      scratch + 4 * p->max_subs, false, o->force_scale, nullptr, s));
  p->last_storage = SM_F64;
  p->last_chunk = chunk;
  p->last_H = nullptr;   // no fallback rebuild from H alone
  p->last_mu = mu;
  p->fd_chunk = -1;
  return SM_OK;
}

int assemble_P_overlap(sm_plan* p, int32_t chunk, void* ws, const void* ws_aux_in, double* P, void* stream) {
  if (!p || !ws || !ws_aux_in || !P) return set_error(SM_ERR_ARG, "assemble_P_overlap: null argument");
  if (p->ovl_chunk != chunk || p->ovl_aux != ws_aux_in)
    return set_error(SM_ERR_STATE, "assemble_P_overlap: the auxiliary workspace does not hold chunk %d", chunk);
  int g0, nsub, rc;
  if ((rc = chunk_range(p, chunk, g0, nsub))) return rc;
  if ((rc = ensure_ovl(p))) return rc;
  const OvlJob* slab;
  int nj;
  if ((rc = ovl_jobs(p, chunk, 2, &slab, &nj))) return rc;
  hipStream_t s = as_stream(stream);
  double* aux = f64_mats(p, ws_aux_in);
  double* wm = f64_mats(p, ws);
  const WsLayout L = p->layout(SM_F64);
  const SubState* st = reinterpret_cast<const SubState*>(static_cast<char*>(ws) + L.state);
  // U = X Z[:, cols] (aux buffer 2), D = Z[:, cols] - U (aux buffer 1),
  // R = 1/2 Z D (aux buffer 2): block column i of P_i
  SM_HIP(launch_ovl_xbuf(st, nsub, p->d_ovl_xbuf, s));
  SM_HIP(launch_ovl_prod(p->dev, g0, slab, nj, p->ovl_edge, wm, 0, p->d_ovl_xbuf, aux, 0, aux, 2, nullptr, 1.0, 0.0,
                         nullptr, 0, 0.0, 1, nullptr, s));
  SM_HIP(launch_ovl_slab_diff(p->dev, g0, nsub, aux, 0, aux, 2, aux, 1, nullptr, s));
  SM_HIP(launch_ovl_prod(p->dev, g0, slab, nj, p->ovl_edge, aux, 0, nullptr, aux, 1, aux, 2, nullptr, 0.5, 0.0,
                         nullptr, 0, 0.0, 1, nullptr, s));
  SM_HIP(launch_ovl_scatter(p->dev, g0, nsub, aux, 2, P, s));
  return SM_OK;
}

int sm_density_matrix_overlap(sm_plan* p, const double* H, const double* S, double mu, const sm_sign_opts* o,
                              void* ws, void* ws_aux, double* P, sm_sub_stats* stats, double* E_host,
                              double* Ne_host, void* stream) {
  if (!p || !H || !S || !ws || !ws_aux || !P || !stats)
    return set_error(SM_ERR_ARG, "sm_density_matrix_overlap: null argument");
  int rc;
  if ((rc = check_schedule(o, "sm_density_matrix_overlap"))) return rc;
  const int nch = (int)p->chunk_ptr.size() - 1;
  for (int c = 0; c < nch; ++c) {
    if ((rc = sm_overlap_inv_sqrt(p, c, S, 1e-12, 100, ws_aux, ws, nullptr, nullptr, stream))) return rc;
    if ((rc = build_submatrices_overlap(p, c, H, mu, o, ws, ws_aux, stats, stream))) return rc;
    if ((rc = submatrix_sign(p, c, ws, o, stats, stream))) return rc;
    if ((rc = assemble_P_overlap(p, c, ws, ws_aux, P, stream))) return rc;
  }
  // E = tr(P H), Ne = tr(P S) (the electron count in a non-orthogonal basis)
  if ((rc = energy_trace(p, H, P, E_host, nullptr, stream))) return rc;
  return energy_trace(p, S, P, Ne_host, nullptr, stream);
}

}  // extern "C"
