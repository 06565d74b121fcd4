/*
 * esd.h - C ABI of the MI355X (gfx950) error-vector-sampling accelerated ICCG
 * solver for a sequence of SPD systems A x_k = b_k sharing one matrix
 * (Iwashita, Ikehara, Fukaya, Mifune, arXiv 2203.08498).
 *
 * Problem statement (Sec. 2, eqs. (ak2), (ak3)): A is symmetric positive
 * definite and identical for every k; b_k depends on earlier solutions, so the
 * systems are solved in order.  During the first solve approximate solutions
 * are sampled (Sec. 4.2-4.3); afterwards an auxiliary matrix W is built from
 * the sampled error vectors by Gram-Schmidt and Rayleigh-Ritz (eqs. (ek)-(bk))
 * and later solves are accelerated by deflation (Sec. 3.3, Alg. "Deflated PCG
 * method") or by the additive subspace-correction preconditioner (Sec. 3.2,
 * eq. (mc)).  Each solve returns a condition-number estimate (Sec. 5.4).
 *
 * Conventions for every entry point
 *   - (h) marks a host pointer, (d) a device pointer on the context's device.
 *     Every device buffer is owned by the caller (e.g. torch tensors): the
 *     inputs and outputs of each call, and the one workspace given to
 *     esd_setup, which holds all of the context's device state (permuted
 *     matrix and factor, auxiliary space, work vectors, block partials, the
 *     alpha/beta history and sampling table).  The library never allocates
 *     or frees device memory; it keeps only the workspace (until
 *     esd_destroy) and never keeps a call's other buffers after it returns.
 *     The context itself holds host-side state (Ritz values, C, the history
 *     read back, pinned 1 KB scalar mirror), HIP events and, once a solve
 *     variant first runs, its captured iteration graphs.
 *   - Vectors (b, x0, x, lambda, v0, W) are float64 in the caller's row order;
 *     the library permutes internally.
 *   - Work is enqueued on the stream given to esd_setup.  Calls that return
 *     host-side results (solve, build_aux, factor_ic0) synchronise that stream
 *     before returning; their device outputs are then valid.
 *   - Return value: ESD_OK (0); a positive value is a warning and the outputs
 *     are valid; a negative value is an error, the outputs are undefined and
 *     esd_last_error() describes it.  No C++ exception crosses this ABI.  A NULL
 *     context or an out-of-range argument returns ESD_EINVAL.
 *   - One context must not be used from two threads at once.
 */
#ifndef ESD_H
#define ESD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct esd_ctx esd_ctx;

typedef enum {
    ESD_OK = 0,
    ESD_NOT_CONVERGED = 1, /* maxit reached (or inner stagnation); x = last iterate */
    ESD_AUX_EMPTY = 2,     /* no Ritz value below theta / no W: solved as plain ICCG */
    ESD_EINVAL = -1,       /* bad argument or call order */
    ESD_ENOTSPD = -2,      /* IC(0) pivot <= 0 (matrix not SPD or IC(0) breakdown) */
    ESD_EHIP = -3,         /* HIP runtime error */
    ESD_ENUMERIC = -4,     /* NaN/Inf in the iteration */
    ESD_ENOAUX = -5,       /* accelerated mode requested before build_aux/set_aux */
    ESD_ENOSAMPLES = -6,   /* build_aux without a sampling solve */
    ESD_EWORKSPACE = -7    /* workspace missing, too small or not 256-byte aligned */
} esd_status;

/* ordering of the rows (esd_options.order) */
#define ESD_ORDER_NATURAL 0       /* the caller's row order; IC(0) of A */
#define ESD_ORDER_COLORS 1        /* stable sort of the rows by colour (multicolour order); IC(0) of A */
#define ESD_ORDER_BLOCK_JACOBI 2  /* natural order; block-Jacobi IC(0) of the paper's parallel solver
                                     (Sec. 5.3): IC(0) of the block-diagonal part of A, blocks of
                                     block_rows consecutive rows */
/* arithmetic of the context (esd_options.prec) */
#define ESD_PREC_FP64 0   /* FP64 only: no FP32 copies are kept, ESD_FLAG_MIXED is rejected */
#define ESD_PREC_MIXED 1  /* FP64 plus FP32 copies of A, L, W, AW and FP32 work vectors */

typedef struct {
    int32_t order;      /* ESD_ORDER_* */
    int32_t block_rows; /* ESD_ORDER_BLOCK_JACOBI: rows per block (>= 1); ignored otherwise */
    int32_t prec;       /* ESD_PREC_* */
    int32_t m_max;      /* largest sample count (esd_sample_errors, esd_load_samples) and width of
                           W (esd_set_aux), 1..64 */
    int32_t max_iters;  /* largest maxit a solve may ask for (sizes the alpha/beta history and the
                           sampling table); 0 = 100000 */
    int32_t reserved[3];
} esd_options;

/* solver modes (Sec. 5.2: ICCG, ES-D-ICCG, ES-SC-ICCG) */
#define ESD_PLAIN 0    /* IC(0)-preconditioned CG */
#define ESD_DEFLATED 1 /* deflated PCG, Alg. "Deflated PCG method" */
#define ESD_SUBSPACE 2 /* PCG with M_sc^{-1} = M^{-1} + W (W^T A W)^{-1} W^T, eq. (mc) */

/* solve flags */
#define ESD_FLAG_NOPREC 1 /* M = I (unpreconditioned CG), used for closed-form checks */
#define ESD_FLAG_POWER 2  /* power iteration fused into the SpMV, (q v) = A (p v) (Alg. PCG-con) */
#define ESD_FLAG_MIXED 4  /* (ESD_PREC_MIXED contexts) FP32 inner solves inside an FP64 iterative-refinement loop; if a
                             refinement step fails to halve the FP64 residual, or its inner run
                             stagnated before reducing it 100-fold, the solve is
                             finished by FP64 CG (reported in esd_info.fp64_iters), restarted
                             from x (at most 4 times) while the recomputed residual misses tol */
#define ESD_FLAG_SYNC_EVERY 8 /* check convergence after every iteration (no speculative chunk) */
#define ESD_FLAG_TIMING 16    /* hipEvents around the SpMV, update and sweep launches of every executed iteration */
#define ESD_FLAG_TIMING_SPMV 32 /* hipEvents around the SpMV launch of every executed iteration only */
#define ESD_FLAG_TRUE_RES 64  /* FP64: after the recurrence test, restart from x while the recomputed
                                 residual misses tol (at most 4 restarts); a deflated restart that
                                 does not halve the recomputed residual is followed by plain PCG
                                 restarts (the same rule holds in the FP64 finish of ESD_FLAG_MIXED) */
#define ESD_FLAG_STREAM 128   /* launch every kernel on the stream; by default the iterations run as
                                 replays of captured 16- and 4-iteration HIP graphs (the short one
                                 near the stop the residual's rate predicts), cached in the context
                                 (solves with ESD_FLAG_TIMING, ESD_FLAG_TIMING_SPMV or
                                 ESD_FLAG_SYNC_EVERY always use stream launches) */
#define ESD_FLAG_MIXED_KEEP 256 /* with ESD_FLAG_MIXED: a refinement step whose inner run reached its
                                   target does not restart CG; the FP64 true residual replaces that
                                   run's FP32 recurrence residual and the run continues with its
                                   search direction (beta recomputed from the new residual's rho).
                                   An inner run that stagnated is followed by a fresh one. */
#define ESD_FLAG_MIXED_ADAPT 512 /* with ESD_FLAG_MIXED: the context remembers, per mode (plain,
                                    deflated, SC), that a mixed solve of its operator had to finish
                                    in FP64; a solve with this flag in a mode so marked runs in FP64
                                    from the start (FP32 cannot resolve the operator).  The record
                                    is cleared by esd_factor_ic0, esd_update_values,
                                    esd_set_mixed_params and, for deflated and SC, a new W. */

typedef struct {
    int32_t iters;        /* CG iterations (mixed: total inner iterations) */
    int32_t outer_iters;  /* refinement steps (1 for FP64 solves) */
    int32_t converged;    /* 1 if ||r||_2 <= tol ||b||_2 */
    int32_t m_tilde;      /* columns of W used by this solve (0 for PLAIN) */
    int32_t nsamples;     /* sampling stores made during this solve */
    int32_t mode_used;    /* ESD_PLAIN if an accelerated mode fell back */
    int32_t fp64_iters;   /* mixed: iterations finished in FP64 after the FP32 refinement stalled */
    int32_t reserved;
    double relres;        /* recurrence residual norm / ||b|| at exit */
    double true_relres;   /* ||b - A x||_2 / ||b||_2 recomputed in FP64 */
    double kappa;         /* K1: extreme Lanczos values from the CG alpha/beta */
    double kappa_es;      /* K2: power-method lambda_max / smallest Ritz value (Sec. 5.4) */
    double lambda_max;    /* (v, A v) of the power iteration of this solve, or of the last solve on
                             the current values that ran it (ESD_FLAG_POWER); 0 if none did.
                             With ESD_FLAG_MIXED the power iterate rides on the FP32 inner SpMV,
                             so A here is the FP32 copy of the values (the quotient itself is
                             accumulated in FP64); it differs from the FP64 lambda_max by about
                             the FP32 rounding of A, relative 1e-7 */
    double lambda_min_ritz; /* smallest Ritz value of the last build_aux (0 if none) */
    double lanczos_min, lanczos_max; /* extreme eigenvalues of the Lanczos matrix */
    double seconds;       /* wall time of the solve on the stream (hipEvent) */
} esd_info;

/*
 * esd_workspace_bytes - device workspace, in bytes, that esd_setup needs at
 * most for a matrix of n rows and nnz stored entries none of whose rows holds
 * more than max_row entries (diagonal included), with the options opt(h).
 * Pure host arithmetic (no GPU call).  The bound follows from the layouts'
 * construction: a 64-row slice of the sliced-ELL layout is as wide as its
 * longest row, the class-aligned copy is at most 5/4 of it, a level schedule
 * has at most n levels.  For stencil matrices it exceeds the exact need by a
 * few bytes per row.  Returns 0 for invalid arguments.
 */
size_t esd_workspace_bytes(int64_t n, int64_t nnz, int32_t max_row, const esd_options *opt);

/*
 * esd_setup - take one SPD matrix and an ordering; build the device formats
 * in the caller's workspace.
 *   n, nnz, rowptr(d) int64[n+1], col(d) int32[nnz], val(d) float64[nnz]: the
 *     full symmetric CSR of A (both triangles, diagonal stored, columns
 *     sorted).  The paper's test matrices are diagonally scaled beforehand
 *     (Sec. 5.1); the library solves the matrix it is given.  The CSR is read
 *     (copied to the host for the ordering and layout analysis, and into the
 *     workspace); the caller may free it after the call.
 *   colors(d) int32[n]: with ESD_ORDER_COLORS, rows are ordered by a stable
 *     sort on colour, which fixes the IC(0) factor; rows of one colour must
 *     not be coupled (checked: ESD_EINVAL).  Ignored (may be NULL) otherwise.
 *   opt(h): ordering, block size, precision, m_max, max_iters.
 *   hip_stream: a hipStream_t (NULL = default stream) all work is queued on.
 *   workspace(d), ws_bytes: device memory of at least the exact need, 256-byte
 *     aligned (torch's allocator returns such blocks); esd_workspace_bytes
 *     gives an upper bound without the analysis.  The context uses it until
 *     esd_destroy; the caller must not touch it meanwhile.
 *   ws_needed(h) out (may be NULL): the exact bytes this matrix needs, set
 *     whenever the analysis succeeded -- also on ESD_EWORKSPACE, so that a
 *     call with workspace = NULL is a size query.
 * ESD_EWORKSPACE: workspace NULL, smaller than the need or misaligned (no
 * context is created).  ESD_EINVAL: bad CSR, colours or options.
 */
esd_status esd_setup(esd_ctx **ctx, void *hip_stream, int64_t n, int64_t nnz, const int64_t *rowptr,
                     const int32_t *col, const double *val, const int32_t *colors, const esd_options *opt,
                     void *workspace, size_t ws_bytes, size_t *ws_needed);

/* esd_workspace_used - bytes(h) of the workspace the context occupies (its
 * exact need, as returned through ws_needed). */
esd_status esd_workspace_used(const esd_ctx *ctx, size_t *bytes);

/* Block-Jacobi IC(0) (ESD_ORDER_BLOCK_JACOBI): the preconditioner of the
 * paper's parallel solver (Sec. 5.3) instead of IC(0) of the whole matrix.
 * Rows stay in the natural order and are split into blocks of block_rows
 * consecutive rows (the last block may be shorter); esd_factor_ic0 then
 * computes IC(0) of the block-diagonal part of A, i.e. every coupling between
 * two blocks is left out of the preconditioner (A, the SpMV and everything
 * else keep them).  When every coupling inside a block joins two consecutive
 * rows (tridiagonal blocks; on a natural-order grid, blocks of at most one
 * grid line) and block_rows <= 512, each block's factor is its exact Cholesky
 * factor and M^{-1} r runs as one launch (two recurrences per block, one
 * wavefront each).  Other blocks (the paper's few large blocks, for
 * instance) run the level-scheduled sweeps of the in-block couplings: correct
 * for any block shape, one launch per level, so slow when the chains inside a
 * block are long.  Sampling, auxiliary space, all solver modes, mixed
 * precision and the gradient work as with IC(0) of A. */

/* esd_update_values - new values val(d) float64[nnz] for the same pattern, in
 * the caller's CSR order (a slowly varying matrix A_k, Sec. 2; finite-
 * difference checks).  The IC(0) factor must be recomputed with
 * esd_factor_ic0 before the next solve; an existing W is kept and AW, C =
 * W^T A W are recomputed for the new values. */
esd_status esd_update_values(esd_ctx *ctx, const double *val);

/* esd_factor_ic0 - IC(0) on the stored lower pattern in the chosen order (the
 * paper's IC preconditioner, Sec. 4.4); with ESD_ORDER_BLOCK_JACOBI, IC(0)
 * of the block-diagonal part (Sec. 5.3).  FP64 factor, plus an FP32 copy in
 * ESD_PREC_MIXED contexts.  ESD_ENOTSPD on a non-positive pivot. */
esd_status esd_factor_ic0(esd_ctx *ctx);

/* esd_sample_errors - arm sampling with m slots (1 <= m <= m_max) for the next
 * solve; only iterations that did not meet the stop test are sampled.
 *   method ESD_SAMPLING_A (Appendix A): x_i is stored in slot
 *     (sum_l (-1)^l floor((i-1)/m^l)) mod m when i mod h == 0, h doubling at
 *     i = h m.
 *   method ESD_SAMPLING_B (Sec. 4.3): slot s-1 (s = 1..m) takes x_i at the
 *     first i with ||r_i|| / ||b|| <= tol^{s/(m+1)} (tol = the solve's
 *     tolerance, squares compared); thresholds passed in one iteration share
 *     that sample, stored in the first of them, the others stay empty.
 *   | ESD_SAMPLE_RESIDUALS: store the residual r_i instead of x_i; build_aux
 *     then uses the residuals themselves instead of e = x_N - x_i (the
 *     residual-vector sampling of Sec. 5.2).
 * ESD_EINVAL for an unknown method. */
#define ESD_SAMPLING_A 0
#define ESD_SAMPLING_B 1
#define ESD_SAMPLE_RESIDUALS 16
esd_status esd_sample_errors(esd_ctx *ctx, int32_t m, int32_t method);

/* esd_load_samples - install k approximate solutions X(d) (n x k, column-major,
 * float64, user order; taken as sampled at iterations 1..k) and the final
 * solution xN(d) in place of a sampling solve, e.g. to resume from saved
 * samples; the next esd_build_aux uses them.  1 <= k <= m_max. */
esd_status esd_load_samples(esd_ctx *ctx, const double *X, int32_t k, const double *xN);

/* esd_build_aux - after a sampling solve: error vectors e = x_1 - x~ (eq.
 * (ek)), classical Gram-Schmidt applied twice with drop tolerance 1e-10
 * (eq. (ekd)), Ritz pairs of E^T A E (eq. (Rayleigh-Ritz)), W from the Ritz
 * vectors with Ritz value < theta (eq. (bk)), AW = A W, C = W^T A W and its
 * Cholesky factor.
 *   ritz(h) float64[m] out: all m_bar Ritz values ascending (may be NULL).
 *   m_bar(h), m_tilde(h) out: orthonormal basis size and selected columns.
 * ESD_AUX_EMPTY (warning) when m_tilde = 0; ESD_ENOSAMPLES without samples. */
esd_status esd_build_aux(esd_ctx *ctx, double theta, double *ritz, int32_t *m_bar,
                         int32_t *m_tilde);

/* esd_set_rayleigh_ritz - operator of the Rayleigh-Ritz step of the next
 * esd_build_aux calls: ESD_RR_A (default) solves E^T A E t = lambda t (eq.
 * (Rayleigh-Ritz)); ESD_RR_PRECONDITIONED uses the preconditioned matrix
 * M^{-1}A (the footnote of that equation) in the M inner product, where it
 * is self-adjoint: E^T A E t = lambda E^T M E t with M = L L^T the IC(0)
 * factor (esd_build_aux then needs esd_factor_ic0); theta then thresholds
 * Ritz values of M^{-1}A.  ESD_EINVAL for another op. */
#define ESD_RR_A 0
#define ESD_RR_PRECONDITIONED 1
esd_status esd_set_rayleigh_ritz(esd_ctx *ctx, int32_t op);

/* esd_set_aux - use a caller-given auxiliary matrix W(d): n x k, column-major,
 * float64, user row order, full column rank, 1 <= k <= m_max.  Replaces any W. */
esd_status esd_set_aux(esd_ctx *ctx, const double *W, int32_t k);

/* esd_get_aux - copy out W(d) (n x m_tilde, column-major, user order; NULL to
 * skip) and C = W^T A W (h, m_tilde x m_tilde row-major; NULL to skip). */
esd_status esd_get_aux(esd_ctx *ctx, double *W, double *C);

/* esd_set_power_start - unit start vector v0(d) of the power iteration
 * (Alg. PCG-con, "a unit random vector").  The iterate is carried across
 * solves that pass ESD_FLAG_POWER. */
esd_status esd_set_power_start(esd_ctx *ctx, const double *v0);

/* esd_set_mixed_params - inner relative tolerance of each FP32 inner solve
 * (default 1e-4) and the maximum number of FP64 refinement steps (default 30);
 * clears the record of earlier FP64 finishes (ESD_FLAG_MIXED_ADAPT).
 * With ESD_FLAG_MIXED_KEEP the inner tolerance is the reduction between two
 * residual replacements; about 1e-2 suits it: after much larger reductions the
 * FP32 recurrence has drifted far from the true residual, and replacing it
 * disturbs the conjugacy of the run. */
esd_status esd_set_mixed_params(esd_ctx *ctx, double inner_tol, int32_t max_outer);

/*
 * esd_solve - solve A x = b.
 *   b(d) float64[n]; x0(d) float64[n] or NULL (zero start); x(d) out.
 *   tol: stop when ||r_i||_2 <= tol ||b||_2 (Alg. "Deflated PCG method" loop
 *     test; for ESD_FLAG_MIXED the FP64 true residual is tested).
 *   maxit: iteration cap (mixed: total inner iterations), <= the context's
 *     max_iters (ESD_EINVAL above it).
 *   mode: ESD_PLAIN / ESD_DEFLATED / ESD_SUBSPACE; flags: ESD_FLAG_*.
 *   info(h) out (may be NULL).
 * A sampling solve is the first solve after esd_sample_errors.
 * Returns ESD_NOT_CONVERGED (warning) at maxit, ESD_AUX_EMPTY (warning) when an
 * accelerated mode had no W, ESD_ENOAUX if no aux space was ever built. */
esd_status esd_solve(esd_ctx *ctx, const double *b, const double *x0, double tol, int32_t maxit,
                     int32_t mode, int32_t flags, double *x, esd_info *info);

/* esd_solve_noalloc - esd_solve for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same arguments, results and kernels as esd_solve with ESD_FLAG_STREAM,
 * but the call allocates nothing -- no device memory, no HIP event, no graph
 * (the kernels are launched on the stream one by one).  The per-solve scratch
 * that esd_solve keeps in the context's workspace (the device scalar block
 * and the block-partial tables of every reduction) comes from one static
 * device array of 2.1 MB per GPU instead (4 KB scalar block, 4 x 384 KB
 * partial tables, 512 KB of sweep partials), held by every GPU the library
 * runs on until the process ends; the context's workspace still holds the
 * matrix, factor, auxiliary space and work vectors.  Every call on one GPU
 * shares that array, so calls that overlap on one GPU (on two streams or from
 * two threads) race: serialise them.  Nothing in it has to start at zero:
 * each solve writes the scalar block and every partial row before reading
 * them.  info->seconds is host wall time.  ESD_EINVAL for ESD_FLAG_TIMING /
 * ESD_FLAG_TIMING_SPMV, or when the context's sweep levels need more than
 * 65536 partial slots (more levels than the array holds: use esd_solve);
 * ESD_EHIP if the array's device address could not be resolved at setup. */
esd_status esd_solve_noalloc(esd_ctx *ctx, const double *b, const double *x0, double tol, int32_t maxit,
                             int32_t mode, int32_t flags, double *x, esd_info *info);

/* esd_sequence_rhs - right-hand side of the next system of the sequence
 * (Sec. 2: b_k depends on the earlier solutions): b = f + c * xprev, with
 * f(d), xprev(d), b(d) float64[n]; xprev may be NULL (b = f).  Enqueued on
 * the context's stream. */
esd_status esd_sequence_rhs(esd_ctx *ctx, const double *f, const double *xprev, double c, double *b);

/* esd_grad_values - gradient of a loss through x = A^{-1} b with respect to
 * every stored value: gval[k] = -lam[row k] * x[col k] in the caller's CSR
 * order, where lam = A^{-1} (dL/dx) is the adjoint solution.
 * lam(d), x(d) float64[n]; gval(d) float64[nnz] out.  Enqueued on the
 * context's stream without synchronising (device output only). */
esd_status esd_grad_values(esd_ctx *ctx, const double *lam, const double *x, double *gval);

/* esd_hbm_probe - streaming probe of the achievable HBM bandwidth on the
 * device of hip_stream (not part of the method; the benchmark's ceiling):
 * ESD_PROBE_COPY copies n float64 from src(d) to dst(d); ESD_PROBE_READ reads
 * src(d) and writes one partial sum per block to dst(d)[0 .. grid).  grid
 * blocks of 256 threads (0 = 4096), 16-byte accesses, grid-stride.  n even,
 * both pointers 16-byte aligned (ESD_EINVAL otherwise).  Enqueued on
 * hip_stream without synchronising; needs no context. */
#define ESD_PROBE_COPY 0
#define ESD_PROBE_READ 1
esd_status esd_hbm_probe(void *hip_stream, int32_t kind, const double *src, double *dst, int64_t n, int32_t grid);

/* Inspection entry points (used by tests and the benchmark). */
esd_status esd_spmv(esd_ctx *ctx, const double *x, double *y);       /* y = A x, FP64, (d) */
esd_status esd_prec_apply(esd_ctx *ctx, const double *r, double *z); /* z = (L L^T)^{-1} r, (d) */
esd_status esd_get_perm(esd_ctx *ctx, int32_t *perm);  /* (h) int32[n]: logical position -> user row */
esd_status esd_get_factor_diag(esd_ctx *ctx, double *ldiag); /* (h) float64[n] l_ii, user row order */
/* (h) alpha[cap], beta[cap] of the last solve (mixed: the first inner run, which with
 * ESD_FLAG_MIXED_KEEP spans every refinement step it continued through);
 * returns the count of alphas through *count; beta has count-1 entries. */
esd_status esd_get_history(esd_ctx *ctx, double *alpha, double *beta, int32_t cap, int32_t *count);
/* (h) int32[m]: iteration stored in each sampling slot (0 = empty) */
esd_status esd_get_samples(esd_ctx *ctx, int32_t *iters_by_slot);
/* (d) float64[n] out, user order: the vector stored in sampling slot `slot`
 * (0 <= slot < m of the last esd_sample_errors / esd_load_samples; the
 * content of an empty slot is undefined) */
esd_status esd_get_sample_vector(esd_ctx *ctx, int32_t slot, double *out);
/* (h) int32[8]: n, nnz, number of sweep levels (1 with block Jacobi), number of colours,
 * 1/0 whether the iteration kernels read A, L and U in the class-aligned
 * layout (per 64-row slice one column offset per slot instead of one column
 * index per entry; used when no slice needs more than 64 slots), and the
 * number of stored slots (entries + padding) of A in the layout the
 * iteration SpMV reads */
esd_status esd_get_layout(esd_ctx *ctx, int32_t *out8);
/* (h) double[4] from the last solve run with ESD_FLAG_TIMING: average ms per
 * executed iteration of out[0] the SpMV launch, out[1] the preconditioner
 * (all sweep launches; with block Jacobi and no subspace correction the one
 * launch that updates x, r and applies M^{-1}), out[2] what runs between the
 * two (alpha finalize and, unless fused into out[1], the vector update; with
 * subspace correction also W^T r and u); out[3] the number of timed
 * iterations. */
esd_status esd_get_timing(esd_ctx *ctx, double *out4);

const char *esd_status_string(esd_status s);
const char *esd_last_error(const esd_ctx *ctx);
void esd_destroy(esd_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* ESD_H */
