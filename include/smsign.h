/*
 * smsign.h -- C ABI of the MI355X submatrix-method density-matrix library.
 *
 * The library computes the density matrix of a sparse, atom-block-structured,
 * symmetric Kohn-Sham matrix H with an orthogonal basis,
 *
 *     P = 1/2 (I - sign(H - mu I))            (Eq. 14 of the paper with S = I)
 *
 * by the submatrix method (Fig. 2 of the paper): for every atom block i it
 * gathers the dense principal submatrix T_i of all orbitals coupled to block i
 * (build_submatrices), evaluates sign(T_i) (Eq. 13) by Newton-Schulz iteration
 * on the GPU (submatrix_sign), and writes block i's columns of the result into
 * the sparse P (assemble_P).  energy_trace reduces tr(PH) and tr P in float64.
 *
 * Conventions
 *   - Every function returns an int status: SM_OK (0) or a negative SM_ERR_*.
 *     The message of the last error of the calling thread is sm_last_error().
 *   - "host" pointers are CPU memory owned by the caller; the library copies
 *     what it keeps.  "device" pointers are GPU memory (hipMalloc'd or a torch
 *     tensor's data_ptr) owned by the caller, on the device that is current
 *     when the plan is first used.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls are asynchronous on that stream unless stated otherwise.
 *   - Matrices are symmetric with the full block pattern stored, in the
 *     block-column panel layout:
 *       col_ptr[c]..col_ptr[c+1]-1 index the stored blocks of block column c,
 *       row_idx[k] is the block row (atom) of stored block k, strictly
 *       ascending inside a column, and the diagonal block is present;
 *       the blocks of column c are stacked, in ascending row order, into one
 *       dense column-major panel of height h_c = sum block_size[row] and
 *       width block_size[c], starting at panel_off[c] (in elements).
 *     P is returned in the same layout and pattern as H.  The structural
 *     pattern (explicit zero blocks included) defines the index sets, so a
 *     wider pattern gives larger, more accurate submatrices.
 */
#ifndef SMSIGN_H
#define SMSIGN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define SM_OK             0
#define SM_ERR_ARG       -1   /* invalid argument (null pointer, bad pattern, bad option) */
#define SM_ERR_HIP       -2   /* a HIP runtime call failed; message names it */
#define SM_ERR_NONFINITE -3   /* NaN/Inf found in the input; message names the submatrix */
#define SM_ERR_OOM       -4   /* allocation of a library-owned table failed */
#define SM_ERR_STATE     -5   /* call out of order (e.g. sign before build) */

/* ---- precisions ----
 * Arithmetic of one Newton-Schulz phase.  SM_F64 / SM_F32 use the float64 /
 * float32 MFMA instructions.  SM_BF16 and SM_F16 round both GEMM operands to
 * bfloat16 / float16 and accumulate in float32.  SM_BF16X3 splits each float32
 * operand x = hi + lo into two bfloat16 values and forms
 * A.B ~ Ahi.Bhi + Ahi.Blo + Alo.Bhi with float32 accumulation (Henry, Tang and
 * Heinecke, ARITH 2019).  All phases except SM_F64 keep the iterate in float32. */
typedef enum { SM_F64 = 0, SM_F32 = 1, SM_BF16 = 2, SM_F16 = 3, SM_BF16X3 = 4 } sm_prec;

/* ---- scaling of X_0 = T / c ---- */
typedef enum {
  SM_SCALE_GERSHGORIN = 0, /* c = max_p sum_q |T_pq|  (an upper bound on rho(T)) */
  SM_SCALE_POWER      = 1, /* c = (1 + margin) * power-iteration estimate of rho(T) */
  SM_SCALE_LEARNED    = 2  /* c from the scaling network, accepted only if the
                              power-iteration guard confirms it, else Gershgorin */
} sm_scaling;

typedef struct {
  int32_t n_atoms;            /* number of atom blocks */
  const int32_t* block_size;  /* host [n_atoms]: orbitals per atom, >= 1 */
  const int64_t* col_ptr;     /* host [n_atoms+1] */
  const int32_t* row_idx;     /* host [col_ptr[n_atoms]] */
  const int64_t* panel_off;   /* host [n_atoms+1]: panel start of every block column */
} sm_bsr_pattern;

typedef struct {
  int32_t phase1;        /* sm_prec of the main Newton-Schulz phase */
  int32_t refine;        /* sm_prec of the refinement steps (SM_F32 or SM_F64) */
  int32_t refine_steps;  /* updates in `refine` after the switch; 0 = no refinement:
                            phase 1 then runs until ||X^2 - I||_F < tol */
  int32_t max_iter;      /* cap on the total number of updates per submatrix */
  double tol;            /* convergence threshold on ||X^2 - I||_F (no refinement) */
  double switch_tol;     /* switch to refinement once ||X^2 - I||_F < switch_tol */
  double stall_below;    /* stagnation test, only while ||X^2 - I||_F < stall_below: */
  double stall_ratio;    /*   res_k > stall_ratio * res_{k-1} ends the phase */
  int32_t scaling;       /* sm_scaling */
  int32_t power_steps;   /* power-iteration steps (SM_SCALE_POWER / the guard) */
  double scale_margin;   /* c = (1 + margin) * estimate for the power / learned scale */
  int32_t probes;        /* float64 probe vectors for the final residual check (0..8) */
  int32_t variant;       /* Newton-Schulz GEMM kernel variant: -1 = the plan's tuned choice
                            (see sm_autotune; before tuning: 1 for float64 and for submatrices
                            under 768 rows, 5 (float32) / 8 (16-bit) above, 2 for 16-bit
                            products on plans padded to 32); 0 = tiles dealt to workgroups
                            in list order, 1 = each XCD walks a contiguous range of the tile
                            list (a submatrix stays in one L2), 2 = as 1 with LDS stages
                            of half the k depth (more workgroups per CU), 3 = as 1 with 128 x 128 output
                            tiles (float32-accumulating precisions, plans padded to 64 or
                            128; otherwise runs as 1), 4 = 128 x 128 tiles walked in list
                            order (all XCDs on the same submatrices: their operands stay in
                            the shared last-level cache), 5 = as 3 with the operands loaded
                            six stages ahead (large submatrices), 6 = 256 x 256 tiles of
                            512 threads with direct global -> LDS operand loads one
                            k-depth-32 stage ahead (bf16 / f16 / split bf16; float32 runs
                            as 5), 7 = as 6 with k-depth-16 stages three ahead, 8 = as 6
                            with the workgroups of an XCD starting every round of tiles
                            together (the round's operand panels stream through its L2
                            together).  bf16 / f16 / split-bf16 products on a plan padded
                            to 32 always run as 2.  With -1, the float32 refinement after
                            a 16-bit main phase of at most two refinement steps runs as 1
                            (its products are the atom's own columns only) */
  int32_t graph_iters;   /* 0: launch every kernel of the iteration loop from the host;
                            G > 0: capture G iterations (tile expansion, squares, residuals,
                            scheduler, updates) into one HIP graph, cached per plan / chunk /
                            workspace, and replay it until no submatrix is left (the host
                            polls once per replay).  Ignored while kernel timing is on. */
  int32_t accel;         /* 0: plain Newton-Schulz.  1: scaled Newton-Schulz in the main
                            phase (Chen and Chow, 2014): X <- 1/2 a X (3I - a^2 X^2) with a
                            chosen from a running lower bound l on the smallest |eigenvalue|
                            of X (so that l and the top of the spectrum map to the same
                            value), l_0 from the scaling network when its scale is accepted,
                            else from lbound; l is carried through every step and raised to
                            sqrt(1 - ||X^2 - I||_F) once that residual is below 1.  The
                            scale a never exceeds sqrt(3) / 1.01 of the spectrum's top, so no
                            eigenvalue can change sign; a wrong l costs iterations only.
                            Refinement steps are plain.  With accel 0 every step is plain
                            except the first where the scale c is below c_G / (sqrt(3) / 1.01)
                            (a learned or power scale): that step is scaled by
                            a = sqrt(3) / (1.01 c_G / c), because c_G / c is the only a
                            priori bound on the top of the spectrum of X_0.  With accel 1
                            and c_G / c > 1 the first square runs unscaled and yields a
                            tighter rigorous bound: rho(X_0)^2 = rho(X_0^2) is at most the
                            largest column sum of |X_0^2| (plus a bound on the product's
                            rounding); the first update is scaled for that top
                            (sm_sub_stats.top1), after Y = 3I - a^2 X_0^2 is formed from
                            the stored 3I - X_0^2 by one elementwise pass.  2: as 1 with
                            the first step scaled for c_G / c (no such bound). */
  double lbound;         /* l_0 as a fraction of the Gershgorin bound: the smallest
                            |eigenvalue| of T is taken to be about lbound * c_G (0: none) */
  int32_t comm_probes;   /* 0..4: float64 commutator probes ||(X T - T X) v|| / (c ||v||) per
                            submatrix (sm_comm_probe), run by sm_density_matrix after every
                            chunk's sign and by sm_find_mu in every pass; 0 = off */
  int32_t retry;         /* 1: every submatrix that ends with status 0 (not converged) or -1
                            (diverged) is built and iterated once more, in the same call, with
                            the fallback schedule: Gershgorin scale, plain Newton-Schulz, the
                            same precisions, twice max_iter (at most 1000); its record gets
                            retried = 1 and the outcome of that second run.  0: no retry. */
  double force_scale;    /* testing only; 0 = off.  > 0: c = force_scale * c_G for every
                            submatrix, and the bound on the top of the spectrum of X_0 is
                            withheld (taken as 1), as if a wrong scale had been trusted: with
                            force_scale well below rho / c_G the iteration diverges, which
                            exercises the divergence test and the retry. */
} sm_sign_opts;

/* Per-submatrix result record, written on the device by build_submatrices
 * (scale, scale_src, gersh, rho_est, feat) and submatrix_sign (the rest).
 * 152 bytes, indexed by submatrix (atom) id. */
typedef struct {
  int32_t iters;       /* Newton-Schulz updates applied in total */
  int32_t iters_low;   /* ... of which in the phase-1 precision */
  int32_t status;      /* 1 converged (||X^2 - I||_F < tol, or stagnation below stall_below);
                          2 refinement steps done after the main phase reached switch_tol (or
                          stagnated);
                          0 not converged: max_iter reached -- with refinement, the main phase
                          ended at max_iter, or the square before the last update (its
                          columns' part where only the atom's columns were computed) was
                          not below max(switch_tol, stall_below);
                          -1 diverged: a non-finite residual, a residual above 2 sqrt(n_pad)
                          after the first update (no iterate of a valid run can have one:
                          every eigenvalue stays in [-sqrt 3, sqrt 3]), or, at or above
                          stall_below, a residual that grew by more than 5 % over an
                          unscaled step (plain Newton-Schulz never increases it) */
  int32_t scale_src;   /* 0 Gershgorin, 1 power, 2 learned accepted, 3 learned rejected,
                          4 forced (sm_sign_opts.force_scale, testing) */
  double scale;        /* c used for X_0 = T / c */
  double res;          /* ||X^2 - I||_F of the last full square, from the GEMM epilogue
                          (float64 sum); with two or more refinement steps the last
                          square computes only the atom's tile columns of Y (all the
                          last update reads) and its partial sum only flags divergence */
  double res_probe;    /* float64 probe: max_v ||X (X v) - v|| / ||v|| (-1 if off), X the
                          last full iterate: a submatrix's final refinement update
                          computes only the atom's own columns of X (the columns P
                          takes), so for status 2 it is the X that update started from */
  double gersh;        /* Gershgorin bound c_G = max_p sum_q |T_pq| */
  double rho_est;      /* power-iteration estimate of rho(T) (<= rho), -1 if not run */
  double lb0;          /* l_0 used by scaled Newton-Schulz, relative to X_0 (0: none) */
  double lb_est;       /* plain runs (accel 0): lower bound on the smallest |eigenvalue|
                          of X_0 that the iteration itself yields, the largest over steps
                          k with 0.01 <= r_k = ||X_k^2 - I||_F < 1 of g^-k(sqrt(1 - r_k)),
                          g(x) = x (3 - x^2) / 2 inverted on [0, 1] (rigorous up to the
                          rounding of r_k); -1 if none */
  double res_comm;     /* float64 commutator probe: max_v ||(X T - T X) v|| / (c ||v||) for
                          fixed +-1 vectors v (X the last full iterate, as for res_probe,
                          T = H[idx, idx] - mu I,
                          c the scale); it is the residual that sees an error in the
                          occupied subspace, which X^2 = I cannot.  -1 if not run */
  float feat[16];      /* features of the scaling network (see sm_mlp_create) */
  int32_t retried;     /* 1: the record is that of the fallback run (sm_sign_opts.retry) */
  float top1;          /* accel 1: the bound on the top of the spectrum of X_0 the first
                          update was scaled for, from the first square's column sums
                          (at most c_G / scale); 0 where that square ran scaled */
} sm_sub_stats;

typedef struct sm_plan sm_plan;
typedef struct sm_mlp sm_mlp;

/* Fills `o` with the defaults for a precision schedule: phase1 = prec; for
 * SM_F64 tol 1e-10 and no refinement; for SM_F32 no refinement with a
 * stagnation stop; for SM_BF16 / SM_F16 / SM_BF16X3 switch at 0.1 (or on
 * stagnation) and 2 (3 for SM_BF16) SM_F32 refinement steps; retry on. */
int sm_default_opts(int32_t prec, sm_sign_opts* o);

/* Symbolic plan (host only; no device work until the first device call).
 *   pattern         block pattern of H (copied).  Errors: SM_ERR_ARG if rows are
 *                   unsorted, the diagonal block is missing, panel_off does not
 *                   match the block sizes, or a block size is < 1.
 *   pad_to          every submatrix is stored padded to a multiple of this
 *                   (32, 64 or 128); the pad is the identity, a fixed point of
 *                   the iteration.
 *   max_chunk_elems workspace budget in matrix elements per chunk: submatrices
 *                   are processed in chunks whose three n_pad^2 buffers fit
 *                   (a single larger submatrix forms its own chunk); <= 0 means
 *                   one chunk.
 * Index set of atom i: the atoms of block column i's stored pattern (ascending);
 * n_i = panel height h_i; loc_i = offset of atom i's own rows in its panel. */
int sm_plan_create(const sm_bsr_pattern* pattern, int32_t pad_to,
                   int64_t max_chunk_elems, sm_plan** out);
void sm_plan_destroy(sm_plan* plan);

/* Processing order from atom positions (Fig. 2 leaves the order of the
 * submatrices open): size buckets of `bucket_rows` padded rows, larger first
 * (bucket_rows <= 0: one bucket), so that every chunk holds submatrices of
 * similar size, and inside a bucket the Morton (Z-order) curve of the atom
 * centres, so that consecutive gathers read neighbouring H panels.  Rebuilds
 * the chunks with the plan's budget (sm_plan_info reports the new order and
 * chunks; results do not depend on the order).
 *   xyz  host double[3 n_atoms]: x, y, z of every atom (any units and origin).
 * SM_ERR_STATE once the plan has been used on a device; SM_ERR_ARG for a
 * non-finite position. */
int sm_plan_set_positions(sm_plan* plan, const double* xyz, int32_t bucket_rows);

/* Workspace storage code of a schedule (the storage_prec argument below):
 * SM_F64 or SM_F32 for the iterate's type; for the SM_BF16 / SM_F16 /
 * SM_BF16X3 main phases that phase's code: float32 buffers followed by a
 * region of the same size with the 16-bit operand copies the products read
 * (one plane, or hi and lo planes for SM_BF16X3).  The main-phase products
 * store only those copies; the float32 refinement and the read-out use the
 * float32 buffers.  Returns -1 for a null pointer. */
int sm_ws_storage(const sm_sign_opts* opts);

/* Sizes for caller-owned buffers.
 *   storage_prec storage code (sm_ws_storage of the schedule); a workspace
 *               must be sized for the storage of every schedule run on it.
 *   n_sub       number of submatrices (= n_atoms), n_chunks number of chunks,
 *   ws_bytes    device workspace bytes needed by build/sign/assemble,
 *   p_nnz_vals  length of P's (and H's) value array.  Any pointer may be NULL. */
int sm_plan_sizes(const sm_plan* plan, int32_t storage_prec, int64_t* n_sub,
                  int64_t* n_chunks, int64_t* ws_bytes, int64_t* p_nnz_vals);

/* Host copies of the plan for inspection (each pointer may be NULL):
 *   n_out[n_atoms], npad_out[n_atoms], loc_out[n_atoms], chunk_out[n_atoms],
 *   order_out[n_atoms] (processing order: submatrix ids chunk by chunk). */
int sm_plan_info(const sm_plan* plan, int32_t* n_out, int32_t* npad_out, int32_t* loc_out,
                 int32_t* chunk_out, int32_t* order_out);

/* Step 1 of Fig. 2 for every submatrix of `chunk`: T_i = H[idx_i, idx_i] - mu I,
 * zero where H stores no block, identity-padded, then scaled to X_0 = T_i / c_i
 * with c_i from opts->scaling; also computes the 16 per-submatrix features.
 *   H_vals  device float64 [p_nnz_vals], panel layout.
 *   ws      device workspace of ws_bytes (caller-owned, reused across chunks).
 *   stats   device sm_sub_stats[n_atoms] indexed by submatrix id.
 * Asynchronous on `stream`: a NaN/Inf in some T_i is flagged by the device in
 * host-mapped memory and reported (SM_ERR_NONFINITE) by the submatrix_sign
 * call that follows. */
int build_submatrices(sm_plan* plan, int32_t chunk, const double* H_vals, double mu,
                      const sm_sign_opts* opts, void* ws, sm_sub_stats* stats, void* stream);

/* Step 2 of Fig. 2: sign(T_i) (Eq. 13) of every submatrix of `chunk` by the
 * Newton-Schulz iteration X <- 1/2 X (3I - X^2) under the precision schedule of
 * opts, all submatrices batched into the same launches; a device scheduler
 * retires converged submatrices.  Writes the per-submatrix records in `stats`.
 * Non-convergence is reported in stats[i].status, not as an error; with
 * opts->retry the failed submatrices are built again from the H_vals and mu
 * of the preceding build_submatrices call of this chunk (H_vals must still be
 * valid; SM_ERR_STATE if the last build was of another chunk) and iterated
 * once more with the fallback schedule before the call returns (one more
 * host synchronisation to count them);
 * SM_ERR_NONFINITE if the preceding build_submatrices found NaN/Inf in a T_i
 * (checked at the first poll, the queued work is left to finish).  Blocks the
 * host only to poll, once per iteration, the scheduler's count of submatrices
 * that continue (it returns as soon as that count is zero). */
int submatrix_sign(sm_plan* plan, int32_t chunk, void* ws, const sm_sign_opts* opts,
                   sm_sub_stats* stats, void* stream);

/* Step 3 of Fig. 2: for every submatrix i of `chunk`, block column i of P is
 * 1/2 (E - sign(T_i)[:, loc_i : loc_i + b_i]) over the rows idx_i (no
 * symmetrisation; each block column has exactly one writer).
 *   P_vals device float64 [p_nnz_vals], same layout as H. */
int assemble_P(const sm_plan* plan, int32_t chunk, const void* ws, double* P_vals,
               void* stream);

/* Float64 commutator check of every submatrix of `chunk` after submatrix_sign:
 * stats[i].res_comm = max over opts->comm_probes (1..4) fixed +-1 vectors v of
 * ||X (T v) - T (X v)|| / (c_i ||v||), X the last full iterate in the workspace,
 * T v formed straight from H's panels (H_vals and mu as given to
 * build_submatrices for this chunk).  sign(T) commutes with T (Eq. 13), so
 * this measures how far the converged X is from sign(T) in the direction the
 * iteration cannot repair (a rotation of the occupied subspace).
 * Asynchronous on `stream`. */
int sm_comm_probe(sm_plan* plan, int32_t chunk, const double* H_vals, double mu,
                  const sm_sign_opts* opts, void* ws, sm_sub_stats* stats, void* stream);

/* E = tr(P H) = sum over stored entries of P .* H (H symmetric) and
 * Ne = tr P, reduced in float64 in a fixed order (bitwise reproducible).
 * Synchronises `stream`; E_host / Ne_host may be NULL. */
int energy_trace(const sm_plan* plan, const double* H_vals, const double* P_vals,
                 double* E_host, double* Ne_host, void* stream);

/* Whole evaluation at fixed mu: for every chunk build, sign, assemble; then
 * energy_trace.  Synchronises `stream`. */
int sm_density_matrix(sm_plan* plan, const double* H_vals, double mu,
                      const sm_sign_opts* opts, void* ws, double* P_vals,
                      sm_sub_stats* stats, double* E_host, double* Ne_host, void* stream);

/* ---- Non-orthogonal basis (S != I), float64 ---------------------------------
 * Eq. 14 with an overlap matrix S, on the submatrix pair (T_i(H), T_i(S)) of
 * every atom block (Fig. 2): S is stored on H's block pattern (same col_ptr /
 * row_idx / panel layout; S_vals device, float64, symmetric positive definite
 * submatrices).  ws is a float64 workspace of the plan (sm_plan_sizes with
 * SM_F64) and ws_aux a second one of the same size, caller-owned; ws_aux holds
 * Z_i = T_i(S)^(-1/2) of the chunk last processed by sm_overlap_inv_sqrt.
 * Schedules: the float64 main phase without refinement steps, Gershgorin or
 * power scaling, retry = 0 (SM_ERR_ARG otherwise). */

/* Eq. 12: Z_i = T_i(S)^(-1/2) for every submatrix of `chunk`, by Newton-Schulz
 * on the block matrix [[0, A], [I, 0]], A = T_i(S) / c_i (c_i its Gershgorin
 * bound): the iterate stays [[0, Y], [Z, 0]] and one step is W = 1/2 (3I - Z Y),
 * Y <- Y W, Z <- W Z; Z / sqrt(c_i) goes to buffer 0 of each submatrix in
 * ws_aux (identity pad).  Stops when every ||Z Y - I||_F < tol, or after
 * max_iter steps (SM_ERR_STATE then).  ws is used as scratch.
 *   iters_out / res_out (may be NULL): steps taken, largest final residual.
 * Synchronises `stream` once per step. */
int sm_overlap_inv_sqrt(sm_plan* plan, int32_t chunk, const double* S_vals, double tol,
                        int32_t max_iter, void* ws_aux, void* ws, int32_t* iters_out,
                        double* res_out, void* stream);

/* Start of the sign iteration for S != I: K_i = Z_i T_i(H) Z_i - mu I (the sign
 * of S^-1 H - mu I in Eq. 14 is Z^-1 sign(K) Z on the pair), written as
 * build_submatrices writes T_i - mu I, then scaled the same way (stats.gersh,
 * stats.scale).  Needs sm_overlap_inv_sqrt of this chunk into ws_aux
 * (SM_ERR_STATE otherwise).  submatrix_sign then runs unchanged.
 * Asynchronous on `stream`. */
int build_submatrices_overlap(sm_plan* plan, int32_t chunk, const double* H_vals, double mu,
                              const sm_sign_opts* opts, void* ws, const void* ws_aux,
                              sm_sub_stats* stats, void* stream);

/* Step 3 of Fig. 2 for S != I: block column i of P_i = 1/2 Z_i (I - X_i) Z_i,
 * X_i the final sign iterate, into P's panel i (H's pattern).  ws_aux's
 * buffers 1 and 2 are used as scratch.  Asynchronous on `stream`. */
int assemble_P_overlap(sm_plan* plan, int32_t chunk, void* ws, const void* ws_aux,
                       double* P_vals, void* stream);

/* Whole evaluation for S != I at fixed mu: per chunk sm_overlap_inv_sqrt (tol
 * 1e-12), build_submatrices_overlap, submatrix_sign, assemble_P_overlap; then
 * E = tr(P H) and Ne = tr(P S) (the electron count of a non-orthogonal basis).
 * Synchronises `stream`. */
int sm_density_matrix_overlap(sm_plan* plan, const double* H_vals, const double* S_vals, double mu,
                              const sm_sign_opts* opts, void* ws, void* ws_aux, double* P_vals,
                              sm_sub_stats* stats, double* E_host, double* Ne_host, void* stream);

/* ---- finite temperature: the general f of Fig. 2 as Fermi-Dirac ----------
 * Step 2 of Fig. 2 with f(x) = 1 / (1 + exp(beta x)) instead of Eq. 14's step
 * 1/2 (1 - sign x), on T_i = H[idx_i, idx_i] - mu I, in float64 (beta > 0:
 * inverse temperature in the units of 1 / H).  As beta grows, f(T_i) tends
 * to the P_i of Eq. 14 where T_i has no eigenvalue at 0.  The workspace is a
 * float64 one (sm_plan_sizes with SM_F64) built by build_submatrices with
 * phase1 = SM_F64, refine_steps = 0 (any scaling: only T_i matters). */

/* f(T_i) for every submatrix of `chunk`, from X_0 = T_i / c in buffer 0 of ws
 * (build_submatrices of this chunk with the float64 schedule must be the last
 * build into ws: SM_ERR_STATE otherwise).  With m the smallest count such
 * that beta max(stats.gersh, stats.scale) <= 2^(m+1) / 4 over the chunk,
 * f(beta T / 2^m) = 1/2 (1 - tanh z), z = beta T / 2^(m+1), comes from the
 * Taylor polynomial of tanh to z^15, then m doublings of the argument,
 * f(2y) = f(y)^2 (f(y)^2 + (1 - f(y))^2)^-1, the inverse as a product of
 * five Neumann factors; 14 + 10 m float64 products per submatrix.  The result
 * stays in ws for assemble_P_fermi.  m > 60 is refused (SM_ERR_ARG).
 *   stats          the records build_submatrices wrote (device, read only).
 *   doublings_out  (may be NULL) m.
 * Synchronises `stream` once (to read the bound that sets m). */
int sm_fermi_dirac(sm_plan* plan, int32_t chunk, void* ws, double beta, const sm_sub_stats* stats,
                   int32_t* doublings_out, void* stream);

/* Step 3 of Fig. 2 for f(T_i): block column i of f(T_i) into P's panel i,
 * and the atom's electron count sum_q f(T_i)_qq and its mu-derivative
 * (without the factor beta) into the plan's per-atom arrays.  Needs
 * sm_fermi_dirac of this chunk into this ws (SM_ERR_STATE otherwise).
 * Asynchronous on `stream`. */
int assemble_P_fermi(sm_plan* plan, int32_t chunk, const void* ws, double* P_vals, void* stream);

/* Whole evaluation at fixed mu and beta: per chunk build_submatrices,
 * sm_fermi_dirac, assemble_P_fermi; then E = tr(P H), Ne = tr P and
 * dNe/dmu = beta sum_i sum_q [f(T_i)(I - f(T_i))]_qq (f' = -beta f (1 - f)),
 * each into host memory when not NULL.  Synchronises `stream`. */
int sm_density_matrix_fermi(sm_plan* plan, const double* H_vals, double mu, double beta,
                            const sm_sign_opts* opts, void* ws, double* P_vals, sm_sub_stats* stats,
                            double* E_host, double* Ne_host, double* dNe_host, void* stream);

/* mu with Ne(mu) = n_target at inverse temperature beta (Ne is continuous and
 * increasing in mu at finite temperature, so the root is unique): Newton
 * steps with the exact derivative, kept inside a bracket that starts as the
 * Gershgorin hull of H widened by 40 / beta on each side (bisection when a
 * step would leave it), from mu_start when finite (clamped into the bracket),
 * else from the bracket's midpoint.  Stops at |Ne - n_target| <= tol, when the
 * bracket cannot shrink further, or after max_steps evaluations (in [1, 200]).
 * On return P_vals holds P at *mu_out; mu_hist / ne_hist [max_steps] (may be
 * NULL) the evaluated points; E_out / Ne_out (may be NULL) tr(P H) and tr P
 * there.  SM_ERR_NONFINITE if a count or its derivative is not finite.
 * Synchronises `stream` once per evaluation. */
int sm_find_mu_fermi(sm_plan* plan, const double* H_vals, double n_target, double beta, double tol,
                     int32_t max_steps, double mu_start, const sm_sign_opts* opts, void* ws,
                     double* P_vals, sm_sub_stats* stats, double* mu_out, int32_t* steps_out,
                     double* mu_hist, double* ne_hist, double* E_out, double* Ne_out, void* stream);

/* Chemical potential by bisection on the electron count (Eq. 14's mu; the
 * paper leaves the rule open): start from the global Gershgorin bracket of H,
 * evaluate Ne(mid) = tr P with the full method at each midpoint, stop at the
 * first midpoint with |Ne - n_target| < accept, else after max_steps
 * evaluations.  On return P_vals (if not NULL) holds P at the returned mu.
 *   mu_start           warm start (NaN: none): evaluated first in place of the
 *                      first midpoint (e.g. the previous geometry's mu); if
 *                      it is not accepted it replaces lo (Ne short of the
 *                      target) or hi, clamped into the bracket.
 *   mu_hist / ne_hist  host arrays of max_steps entries (may be NULL).
 *   E_host / Ne_host   (may be NULL; need P_vals) energy_trace of the returned
 *                      P, reduced in the same pass as the electron count.
 * Synchronises `stream`. */
int sm_find_mu(sm_plan* plan, const double* H_vals, double n_target, double accept,
               int32_t max_steps, double mu_start, const sm_sign_opts* opts, void* ws, double* P_vals,
               sm_sub_stats* stats, double* mu_out, int32_t* steps_out,
               double* mu_hist, double* ne_hist, double* E_host, double* Ne_host, void* stream);

/* Global Gershgorin bracket [lo, hi] of H (synchronous). */
int sm_gershgorin_bracket(sm_plan* plan, const double* H_vals, double* lo, double* hi,
                          void* stream);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): sm_gershgorin_bracket without any
 * allocation or synchronisation.  lohi (device, 2 doubles) receives [lo, hi];
 * the per-atom intervals go to a fixed device scratch of the library (room for
 * 524288 atoms, 8 MiB, one copy per GPU, held until the process ends) instead
 * of the plan's own table.  The plan must already hold its device tables (any
 * earlier device call with it, e.g. sm_gershgorin_bracket; SM_ERR_STATE
 * otherwise) on the current device.  SM_ERR_ARG for a plan of more than
 * 524288 atoms.  Asynchronous on `stream`.  All calls on one GPU share its
 * scratch: calls that overlap in time on one GPU (other streams, other
 * threads) race and must be ordered by the caller. */
int sm_gershgorin_bracket_noalloc(const sm_plan* plan, const double* H_vals, double* lohi, void* stream);

/* Workspace layout, for inspection by tests: region offsets in bytes
 *   regions9 = [matrices, state, partials, lists, features, scratch, vecs, flag, total]
 * and, per processing index g, the element offset of submatrix order[g]'s three
 * n_pad x n_pad column-major buffers (X_even, X_odd, Y) inside the matrix region
 * of its chunk (float32 / float64 elements; for the 16-bit storage codes the
 * copies of buffer b start at float offset max_mats + off, max_mats being the
 * largest per-chunk sum of 3 n_pad^2).  After build_submatrices X_even holds
 * X_0 = T_i / c_i for the float64 code; the other codes keep T_i there (the
 * 16-bit codes only in the copies) with c_i on the identity pad's diagonal,
 * the first square and update applying 1 / c_i.  After submatrix_sign the
 * final X is the float32 (float64) buffer of parity stats[i].iters; where
 * the last refinement update computed only the tile columns holding the
 * atom's own columns (a refined submatrix whose slab has fewer tiles than
 * the triangle), only those columns of it are set, and the other X buffer
 * holds the last full iterate.
 * Either output may be NULL. */
int sm_plan_ws_layout(const sm_plan* plan, int32_t storage_prec, int64_t* regions9,
                      int64_t* mat_off_g);

/* Diagnostic: one matrix-core instruction on a single wavefront with the
 * operand lane layout the kernels assume.  prec = an sm_prec code: the 16x16
 * instruction of that precision; out_host receives 256 doubles,
 * out[lane*4 + v] = the result element held by `lane` in register v (to be
 * compared with D[4*(lane/16)+v][lane%16] of the exact product, float64:
 * D[lane/16 + 4v][lane%16]).  prec = 5 / 6: the 32x32x16 f16 / bf16
 * instruction; out_host receives 1024 doubles, out[lane*16 + v].
 * Synchronous; allocates and frees a device buffer of that size. */
int sm_selftest_mfma(int32_t prec, double* out_host);

/* ---- the spectral-scaling network (learned scaling, SM_SCALE_LEARNED) ----
 * The paper proposes no network; its closing remarks suggest models that are
 * trusted only where they are accurate and retrained on explicitly computed
 * cases.  Here a float32 multilayer perceptron 16 -> 64 -> 64 -> 2 with tanh
 * hidden layers maps the 16 features of a submatrix (sm_sub_stats.feat:
 * log n, log c_G, diagonal and Gershgorin-radius statistics relative to c_G)
 * to y0 ~ log(rho(T)/c_G) and y1 ~ log(l/c_G), l the smallest |eigenvalue|
 * of T (train on sm_sub_stats.lb_est * scale / gersh of plain runs); y1 sets
 * l_0 of scaled Newton-Schulz (opts.accel) where the learned scale is
 * accepted.  Inputs are normalised by a stored mean / std (32 floats).
 * Parameters are packed as W1 (64x16 row-major), b1, W2 (64x64), b2, W3 (2x64),
 * b3: 5378 floats.  Loss = mean over samples of sum over outputs of
 * (y - t)^2; Adam with beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected.
 * The network owns its device buffers (current device at creation). */

/* Weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from a SplitMix64 stream of
 * `seed`; normalisation mean 0, std 1. */
int sm_mlp_create(uint64_t seed, sm_mlp** out);
void sm_mlp_destroy(sm_mlp* mlp);
/* Host float[5378] parameters and float[32] (mean[16], std[16]); either may be
 * NULL.  Setting parameters resets the Adam state. */
int sm_mlp_set_weights(sm_mlp* mlp, const float* params, const float* norm);
int sm_mlp_get_weights(const sm_mlp* mlp, float* params, float* norm);
/* Y[n][2] (device) = network(X) for device X with row stride ldx >= 16 floats. */
int sm_mlp_infer(sm_mlp* mlp, const float* X, int64_t ldx, int64_t n, float* Y, void* stream);
/* Full-batch loss (host double) and gradient (host float[5378], may be NULL)
 * for device inputs X (stride ldx) and targets T[n][2].  Synchronous. */
int sm_mlp_loss_grad(sm_mlp* mlp, const float* X, int64_t ldx, const float* T, int64_t n,
                     double* loss, float* grad, void* stream);
/* Training pairs of the scaling network from the per-submatrix records of an
 * explicit pass (power-iteration scale, plain Newton-Schulz): every record
 * with rho_est > 0, lb_est > 0 and gersh > 0 gives X[k] = its 16 features and
 * T[k] = (log(rho_est / gersh), log(lb_est * scale / gersh)), the targets of
 * sm_mlp_train, in record order.  stats, X (float[n][16]) and T (float[n][2])
 * are device arrays of the caller; *n_pairs (host) = pairs written.
 * Synchronises `stream`. */
int sm_scaling_pairs(const sm_sub_stats* stats, int64_t n, float* X, float* T, int64_t* n_pairs,
                     void* stream);
/* Mini-batch Adam: `epochs` passes over the n samples in batches of `batch`
 * (order shuffled per epoch from shuffle_seed, or kept if 0), learning rate
 * lr; with fit_norm the normalisation is first set to the samples' mean/std.
 * loss_hist (host, `epochs` doubles, may be NULL) receives the mean loss of
 * every epoch.  Synchronous (one host sync per epoch). */
int sm_mlp_train(sm_mlp* mlp, const float* X, int64_t ldx, const float* T, int64_t n, int32_t epochs,
                 int32_t batch, float lr, int32_t fit_norm, uint64_t shuffle_seed, double* loss_hist,
                 void* stream);
/* Attach the network used by build_submatrices when opts->scaling is
 * SM_SCALE_LEARNED (not owned by the plan; NULL detaches). */
int sm_plan_set_mlp(sm_plan* plan, sm_mlp* mlp);

/* Autotuner: for every GEMM kernel variant, one build + submatrix_sign pass
 * over `chunk` at fixed mu (the sign phase timed with HIP events, best of
 * `repeats`), then records the fastest variant for the precisions of `opts`
 * (used when opts->variant == -1; the refinement precision's entry only
 * when the main phase is float64) as the choice of every chunk in the same
 * size class as `chunk` (the number of 256-row tiles of a chunk's largest
 * padded submatrix: one tuning per class serves a batch of mixed sizes) and
 * as the plan-wide choice that sm_plan_tuning reports.  Chunks of classes
 * never tuned keep the size-based defaults (see sm_sign_opts.variant).
 * variant_mask: bit v set = try variant v (0 = all).
 *   best_out   host int32 (may be NULL): the chosen variant
 *   times_ms   host double[SM_GEMM_VARIANTS] (may be NULL): sign time of each
 *              variant (-1: not tried, or not applicable to this plan / precision)
 * Synchronous.  Leaves the workspace holding the last variant's result. */
int sm_autotune(sm_plan* plan, int32_t chunk, const double* H_vals, double mu,
                const sm_sign_opts* opts, void* ws, sm_sub_stats* stats, int32_t repeats,
                int32_t variant_mask, int32_t* best_out, double* times_ms, void* stream);
/* Number of GEMM kernel variants (sm_sign_opts.variant in [0, SM_GEMM_VARIANTS)). */
#define SM_GEMM_VARIANTS 9
int32_t sm_gemm_variants(void);

/* Tuned variant per precision (int32[5], indexed by sm_prec): `get` receives
 * the plan-wide table, `set` (if not NULL) replaces it and the table of every
 * size class -- to persist the autotuner's choices across processes.  Either
 * pointer may be NULL. */
int sm_plan_tuning(sm_plan* plan, int32_t* get, const int32_t* set);
/* The size class of `chunk` (256-row tiles of its largest padded submatrix)
 * and the GEMM variant per precision (int32[5], indexed by sm_prec) its
 * launches use when opts->variant == -1.  Either output may be NULL. */
int sm_plan_chunk_variants(const sm_plan* plan, int32_t chunk, int32_t* class_out, int32_t* variants_out);

/* Kernel timing for measurement.  While enabled, every Newton-Schulz GEMM
 * launch made by submatrix_sign carries a pair of HIP events that the dispatch
 * itself records (start and end of that kernel on the caller's stream; no
 * extra stream packets).  Graph capture is off meanwhile (opts.graph_iters is
 * ignored).  sm_profile_read synchronises on the recorded
 * events, adds up their elapsed times per kernel class, and clears them:
 * class = 2 * precision + kind (precision = sm_prec, kind 0 = square
 * A = X^2 / Y = 3I - a^2 A, kind 1 = update X' = 1/2 a X Y), 10 classes.
 *   launches[10], ms[10]   host outputs (either may be NULL). */
int sm_profile_enable(sm_plan* plan, int32_t on);
int sm_profile_read(sm_plan* plan, int64_t* launches, double* ms);

/* Thread-local message of the last failing call ("" if none). */
const char* sm_last_error(void);

/* Library version string. */
const char* sm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SMSIGN_H */
