// C-ABI entry points of the finite-temperature occupation: the general matrix
// function of Fig. 2 taken as f(x) = 1 / (1 + exp(beta x)) on every
// submatrix T_i = H[idx_i, idx_i] - mu I, in float64, and mu from the electron
// count by a safeguarded Newton iteration with the exact derivative (see
// k_fermi.hip for the arithmetic).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "plan.h"

using namespace sm;

namespace {

// Taylor coefficients of tanh z = sum_k kTanh[k] z^(2k+1), k = 0 .. 7
// (the odd Bernoulli-number series, exact rationals rounded once).
constexpr double kTanh[8] = {1.0,
                             -1.0 / 3.0,
                             2.0 / 15.0,
                             -17.0 / 315.0,
                             62.0 / 2835.0,
                             -1382.0 / 155925.0,
                             21844.0 / 6081075.0,
                             -929569.0 / 638512875.0};
// |z| <= kZmax at the start: the first omitted term is below 6e-4 * 4^-17
constexpr double kZmax = 0.25;
constexpr int kMaxDoublings = 60;

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int chunk_range(const sm_plan* p, int32_t chunk, int& g0, int& nsub) {
  const int nch = (int)p->chunk_ptr.size() - 1;
  if (chunk < 0 || chunk >= nch) return set_error(SM_ERR_ARG, "chunk %d out of [0, %d)", chunk, nch);
  g0 = (int)p->chunk_ptr[chunk];
  nsub = (int)(p->chunk_ptr[chunk + 1] - p->chunk_ptr[chunk]);
  return SM_OK;
}

int ensure_fd(sm_plan* p) {
  int rc;
  if ((rc = ensure_ovl(p))) return rc;
  if (!p->d_fd) {
    void* d = nullptr;
    SM_HIP(hipMalloc(&d, (2 * std::max<int64_t>(p->max_subs, 1) + 2) * sizeof(double)));
    p->dev_allocs.push_back(d);
    p->d_fd = static_cast<double*>(d);
    SM_HIP(hipMalloc(&d, std::max<int64_t>(p->n_atoms, 1) * sizeof(double)));
    p->dev_allocs.push_back(d);
    p->d_fd_dne = static_cast<double*>(d);
  }
  return SM_OK;
}

int check_fd_opts(const sm_sign_opts* o, const char* who) {
  if (!o) return set_error(SM_ERR_ARG, "%s: null sm_sign_opts", who);
  if (o->phase1 != SM_F64 || o->refine_steps != 0)
    return set_error(SM_ERR_ARG, "%s: the finite-temperature path builds with the float64 schedule "
                                 "(phase1 = SM_F64, refine_steps = 0)", who);
  return SM_OK;
}

int check_beta(double beta, const char* who) {
  if (!(beta > 0) || !std::isfinite(beta)) return set_error(SM_ERR_ARG, "%s: beta must be finite and > 0", who);
  return SM_OK;
}

// One evaluation at mu over every chunk: P, and the electron count and its
// mu-derivative summed over the atoms in a fixed order into mapped host memory.
int evaluate(sm_plan* p, const double* H, double mu, double beta, const sm_sign_opts* o, void* ws, double* P,
             sm_sub_stats* stats, double* ne, double* dne, void* stream) {
  const int nch = (int)p->chunk_ptr.size() - 1;
  int rc;
  for (int c = 0; c < nch; ++c) {
    if ((rc = build_submatrices(p, c, H, mu, o, ws, stats, stream))) return rc;
    if ((rc = sm_fermi_dirac(p, c, ws, beta, stats, nullptr, stream))) return rc;
    if ((rc = assemble_P_fermi(p, c, ws, P, stream))) return rc;
  }
  hipStream_t s = as_stream(stream);
  SM_HIP(launch_ne_sum(p->d_ne_sub, p->n_atoms, reinterpret_cast<double*>(p->d_pinned + kHostNe), s));
  SM_HIP(launch_ne_sum(p->d_fd_dne, p->n_atoms, reinterpret_cast<double*>(p->d_pinned + kHostDne), s));
  SM_HIP(hipStreamSynchronize(s));
  *ne = *reinterpret_cast<const double*>(p->h_pinned + kHostNe);
  *dne = *reinterpret_cast<const double*>(p->h_pinned + kHostDne);
  return SM_OK;
}

}  // namespace

extern "C" {

int sm_fermi_dirac(sm_plan* p, int32_t chunk, void* ws, double beta, const sm_sub_stats* stats,
                   int32_t* doublings_out, void* stream) {
  if (!p || !ws || !stats) return set_error(SM_ERR_ARG, "sm_fermi_dirac: null argument");
  int rc;
  if ((rc = check_beta(beta, "sm_fermi_dirac"))) return rc;
  int g0, nsub;
  if ((rc = chunk_range(p, chunk, g0, nsub))) return rc;
  if (p->last_storage != SM_F64 || p->last_chunk != chunk || !p->last_H)
    return set_error(SM_ERR_STATE, "sm_fermi_dirac: build chunk %d with build_submatrices and the float64 schedule "
                                   "first", chunk);
  if ((rc = ensure_fd(p))) return rc;
  const OvlJob* jobs;
  int nj;
  if ((rc = ovl_jobs(p, chunk, 0, &jobs, &nj))) return rc;
  hipStream_t s = as_stream(stream);
  double* wm = f64_mats(p, ws);
  const int mp = p->max_npad;
  double* sv = p->d_fd;                    // s_l = beta c_l / 2^(m+1)
  double* s2 = p->d_fd + p->max_subs;      // s_l^2
  // m: the number of doublings that brings every |z| = |beta x| / 2^(m+1) to kZmax
  SM_HIP(launch_fd_bound(p->dev, g0, nsub, stats, beta, sv, s));
  SM_HIP(launch_ovl_max(sv, nsub, reinterpret_cast<double*>(p->d_pinned + kHostFd), s));
  SM_HIP(hipStreamSynchronize(s));
  const double bound = *reinterpret_cast<const double*>(p->h_pinned + kHostFd);
  if (!std::isfinite(bound)) return set_error(SM_ERR_NONFINITE, "sm_fermi_dirac: non-finite spectral bound");
  int m = 0;
  while (m <= kMaxDoublings && bound > kZmax * std::ldexp(2.0, m)) ++m;
  if (m > kMaxDoublings)
    return set_error(SM_ERR_ARG, "sm_fermi_dirac: beta times the spectral bound (%.3e) needs more than %d doublings",
                     bound, kMaxDoublings);
  SM_HIP(launch_fd_coef(p->dev, g0, nsub, stats, beta, std::ldexp(1.0, -(m + 1)), sv, s2, s));
  // Taylor start, X_0 = T / c in buffer 0: u = p(w), w = z^2 = s^2 X_0^2, by
  // Horner steps u <- c_k I + s^2 X_0 (X_0 u) (buffer 2, X_0 u in buffer 1),
  // then F_0 = 1/2 I - 1/2 s X_0 u = f(beta T / 2^m) into buffer 1
  SM_HIP(launch_fd_lincomb(p->dev, g0, nsub, mp, wm, 0, kTanh[7], -1, 0.0, 0.0, 1, s));
  SM_HIP(launch_ovl_prod(p->dev, g0, jobs, nj, p->ovl_edge, wm, 0, nullptr, wm, 1, wm, 2, s2, 1.0, kTanh[6], nullptr,
                         0, 0.0, 0, nullptr, s));
  for (int k = 5; k >= 0; --k) {
    SM_HIP(launch_ovl_prod(p->dev, g0, jobs, nj, p->ovl_edge, wm, 0, nullptr, wm, 2, wm, 1, nullptr, 1.0, 0.0,
                           nullptr, 0, 0.0, 0, nullptr, s));
    SM_HIP(launch_ovl_prod(p->dev, g0, jobs, nj, p->ovl_edge, wm, 0, nullptr, wm, 1, wm, 2, s2, 1.0, kTanh[k],
                           nullptr, 0, 0.0, 0, nullptr, s));
  }
  SM_HIP(launch_ovl_prod(p->dev, g0, jobs, nj, p->ovl_edge, wm, 0, nullptr, wm, 2, wm, 1, sv, -0.5, 0.5, nullptr, 0,
                         0.0, 0, nullptr, s));
  // m doublings, F in buffer f = 1 throughout, q and t the other two:
  //   Q = F F (q); R = 8/3 (F - Q) - 1/3 I (in place of F); acc = 4/3 (Q R + Q) (t);
  //   then four times: S <- S S (the free buffer), acc <- acc S + acc,
  //   so acc = 4/3 Q (I + R)(I + R^2)(I + R^4)(I + R^8)(I + R^16) = Q D^-1
  const int f = 1;
  for (int d = 0; d < m; ++d) {
    int b[3] = {f, 2, 0};   // b[0] F / R, b[1] Q, b[2] acc
    SM_HIP(launch_ovl_prod(p->dev, g0, jobs, nj, p->ovl_edge, wm, b[0], nullptr, wm, b[0], wm, b[1], nullptr, 1.0,
                           0.0, nullptr, 0, 0.0, 0, nullptr, s));
    SM_HIP(launch_fd_lincomb(p->dev, g0, nsub, mp, wm, b[0], 8.0 / 3.0, b[1], -8.0 / 3.0, -1.0 / 3.0, b[0], s));
    SM_HIP(launch_ovl_prod(p->dev, g0, jobs, nj, p->ovl_edge, wm, b[1], nullptr, wm, b[0], wm, b[2], nullptr,
                           4.0 / 3.0, 0.0, wm, b[1], 4.0 / 3.0, 0, nullptr, s));
    // buffers now: R at b[0], acc at b[2], b[1] free; S starts as R
    int S = b[0], acc = b[2], freeb = b[1];
    for (int j = 0; j < 4; ++j) {
      SM_HIP(launch_ovl_prod(p->dev, g0, jobs, nj, p->ovl_edge, wm, S, nullptr, wm, S, wm, freeb, nullptr, 1.0, 0.0,
                             nullptr, 0, 0.0, 0, nullptr, s));
      const int S2 = freeb;
      freeb = S;   // the old power is dead once squared
      SM_HIP(launch_ovl_prod(p->dev, g0, jobs, nj, p->ovl_edge, wm, acc, nullptr, wm, S2, wm, freeb, nullptr, 1.0,
                             0.0, wm, acc, 1.0, 0, nullptr, s));
      const int acc2 = freeb;
      freeb = acc;
      acc = acc2;
      S = S2;
    }
    if (acc != f) return set_error(SM_ERR_STATE, "sm_fermi_dirac: internal buffer rotation");
  }
  p->fd_chunk = chunk;
  p->fd_ws = ws;
  p->fd_buf = f;
  if (doublings_out) *doublings_out = m;
  return SM_OK;
}

int assemble_P_fermi(sm_plan* p, int32_t chunk, const void* ws, double* P, void* stream) {
  if (!p || !ws || !P) return set_error(SM_ERR_ARG, "assemble_P_fermi: null argument");
  if (p->fd_chunk != chunk || p->fd_ws != ws)
    return set_error(SM_ERR_STATE, "assemble_P_fermi: the workspace does not hold f(T_i) of chunk %d "
                                   "(run sm_fermi_dirac first)", chunk);
  int g0, nsub, rc;
  if ((rc = chunk_range(p, chunk, g0, nsub))) return rc;
  if ((rc = ensure_fd(p))) return rc;
  hipStream_t s = as_stream(stream);
  const double* wm = f64_mats(p, ws);
  SM_HIP(launch_ovl_scatter(p->dev, g0, nsub, wm, p->fd_buf, P, s));
  // the per-atom count and derivative need beta only as a factor of the
  // derivative: it is applied when the sums are formed
  SM_HIP(launch_fd_count(p->dev, g0, nsub, wm, p->fd_buf, 1.0, p->d_ne_sub, p->d_fd_dne, s));
  return SM_OK;
}

int sm_density_matrix_fermi(sm_plan* p, const double* H, double mu, double beta, const sm_sign_opts* o, void* ws,
                            double* P, sm_sub_stats* stats, double* E_host, double* Ne_host, double* dNe_host,
                            void* stream) {
  if (!p || !H || !ws || !P || !stats) return set_error(SM_ERR_ARG, "sm_density_matrix_fermi: null argument");
  int rc;
  if ((rc = check_fd_opts(o, "sm_density_matrix_fermi")) || (rc = check_beta(beta, "sm_density_matrix_fermi")))
    return rc;
  if (!std::isfinite(mu)) return set_error(SM_ERR_ARG, "sm_density_matrix_fermi: mu is not finite");
  if ((rc = ensure_fd(p))) return rc;
  double ne, dne;
  if ((rc = evaluate(p, H, mu, beta, o, ws, P, stats, &ne, &dne, stream))) return rc;
  if (dNe_host) *dNe_host = beta * dne;
  return energy_trace(p, H, P, E_host, Ne_host, stream);
}

int sm_find_mu_fermi(sm_plan* p, const double* H, double n_target, double beta, double tol, int32_t max_steps,
                     double mu_start, const sm_sign_opts* o, void* ws, double* P, sm_sub_stats* stats,
                     double* mu_out, int32_t* steps_out, double* mu_hist, double* ne_hist, double* E_out,
                     double* Ne_out, void* stream) {
  if (!p || !H || !ws || !P || !stats || !mu_out) return set_error(SM_ERR_ARG, "sm_find_mu_fermi: null argument");
  int rc;
  if ((rc = check_fd_opts(o, "sm_find_mu_fermi")) || (rc = check_beta(beta, "sm_find_mu_fermi"))) return rc;
  if (max_steps < 1 || max_steps > 200) return set_error(SM_ERR_ARG, "sm_find_mu_fermi: max_steps out of [1, 200]");
  if (!(tol > 0)) return set_error(SM_ERR_ARG, "sm_find_mu_fermi: tol must be > 0");
  if ((rc = ensure_fd(p))) return rc;
  double lo, hi;
  if ((rc = sm_gershgorin_bracket(p, H, &lo, &hi, stream))) return rc;
  // beyond the hull by 40 / beta every occupation is within e^-40 of 0 or 1
  lo -= 40.0 / beta;
  hi += 40.0 / beta;
  double mu = std::isfinite(mu_start) ? std::min(std::max(mu_start, lo), hi) : 0.5 * (lo + hi);
  int step = 1;
  for (; step <= max_steps; ++step) {
    double ne, dne;
    if ((rc = evaluate(p, H, mu, beta, o, ws, P, stats, &ne, &dne, stream))) return rc;
    if (!std::isfinite(ne) || !std::isfinite(dne))
      return set_error(SM_ERR_NONFINITE, "sm_find_mu_fermi: non-finite electron count at mu = %.17g", mu);
    dne *= beta;
    if (mu_hist) mu_hist[step - 1] = mu;
    if (ne_hist) ne_hist[step - 1] = ne;
    if (std::fabs(ne - n_target) <= tol) break;
    if (ne < n_target) lo = mu;
    else hi = mu;
    // Newton step with the exact derivative, kept inside the bracket
    // (bisection otherwise); Ne is increasing, so the bracket always holds mu
    const double nt = mu + (n_target - ne) / dne;
    const double next = (dne > 0 && nt > lo && nt < hi) ? nt : 0.5 * (lo + hi);
    if (!(next > lo && next < hi) || next == mu) break;   // the bracket cannot shrink further
    mu = next;
  }
  *mu_out = mu;
  if (steps_out) *steps_out = std::min(step, (int)max_steps);
  if (E_out || Ne_out) return energy_trace(p, H, P, E_out, Ne_out, stream);
  return SM_OK;
}

}  // extern "C"
