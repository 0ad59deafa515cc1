// Internal declarations of the float64 tile products and the per-submatrix
// kernels around them: the non-orthogonal basis (k_ovl.hip) and the
// finite-temperature occupation (k_fermi.hip).
#pragma once

#include "smsign_internal.h"

namespace sm {

// One output tile of a product (local submatrix index, tile row, tile
// column; 64- or 128-wide tiles, see launch_ovl_prod).
struct OvlJob {
  int32_t l;
  int16_t bi, bj;
};
hipError_t launch_ovl_fill(const DevPlan& p, int g0, int nsub, int max_npad, double* mats, int b, double dv, double dp,
                           hipStream_t s);
hipError_t launch_ovl_gather(const DevPlan& p, int g0, int nsub, int max_m, const double* V, double* mats, int b,
                             hipStream_t s);
hipError_t launch_ovl_gersh(const DevPlan& p, int g0, int nsub, double* mats, int b, double* out, int pad_one,
                            sm_sub_stats* stats, hipStream_t s);
hipError_t launch_ovl_scale(const DevPlan& p, int g0, int nsub, int max_npad, double* mats, int b, const double* v,
                            int mode, hipStream_t s);
hipError_t launch_ovl_copy(const DevPlan& p, int g0, int nsub, int max_npad, double* mats, int src, int dst,
                           hipStream_t s);
// edge: 64 or 128, the tile edge the job list was built for
hipError_t launch_ovl_prod(const DevPlan& p, int g0, const OvlJob* jobs, int njobs, int edge, const double* A,
                           int abuf, const int32_t* abuf_l, const double* B, int bbuf, double* C, int cbuf,
                           const double* alpha_l, double alpha, double beta, const double* E, int ebuf,
                           double gamma, int kind, double* res, hipStream_t s);
// Finite-temperature occupation (k_fermi.hip).
hipError_t launch_fd_bound(const DevPlan& p, int g0, int nsub, const sm_sub_stats* stats, double beta, double* out,
                           hipStream_t s);
hipError_t launch_fd_coef(const DevPlan& p, int g0, int nsub, const sm_sub_stats* stats, double beta, double inv2m1,
                          double* sv, double* s2, hipStream_t s);
hipError_t launch_fd_lincomb(const DevPlan& p, int g0, int nsub, int max_npad, double* mats, int xb, double a, int yb,
                             double b, double d, int cb, hipStream_t s);
hipError_t launch_fd_count(const DevPlan& p, int g0, int nsub, const double* mats, int fb, double beta, double* ne,
                           double* dne, hipStream_t s);
hipError_t launch_ovl_slab_diff(const DevPlan& p, int g0, int nsub, const double* Z, int zbuf, const double* U,
                                int ubuf, double* D, int dbuf, const double* f_l, hipStream_t s);
hipError_t launch_ovl_scatter(const DevPlan& p, int g0, int nsub, const double* R, int rbuf, double* P, hipStream_t s);
hipError_t launch_ovl_xbuf(const SubState* st, int nsub, int32_t* xbuf, hipStream_t s);
hipError_t launch_ovl_zero(double* v, int n, hipStream_t s);
hipError_t launch_ovl_max(const double* v, int n, double* out, hipStream_t s);

}  // namespace sm
