// Device-side data structures and kernel launchers of the esd library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace esd {

constexpr int kBlock = 256;     // threads per block of every row kernel
constexpr int kMaxGrid = 8192;  // largest grid of a reducing kernel
constexpr int kMaxNV = 72;      // largest number of values reduced together
constexpr int kFinThreads = 1024; // threads of a finalize kernel
constexpr int kPartBudget = 48 * 1024; // doubles a finalize kernel reads at most
constexpr int kTsBlock = 1024;        // threads per block of the tall-skinny W^T v kernel

// Solver scalars kept in device memory; every per-iteration quantity (rho,
// alpha, beta, the coarse vectors, the stop decision) is produced and
// consumed on the device.
struct Scal {
    double rho;      // (r, z) of the current preconditioned residual
    double alpha, beta;
    double rr;       // ||r||^2 of the recurrence residual
    double tol2;     // tol^2 ||b||^2
    double bnorm2;   // ||b||^2
    double vscale;   // 1 / ||v|| of the power iterate
    double out;      // generic reduction output (norms)
    double lam;      // Rayleigh quotient of the power iterate
    double rr_ref;   // stagnation reference
    int32_t it_ref;
    int32_t iter;    // completed iterations of the current solve
    int32_t done;    // 0 running, 1 converged, 2 maxit, 3 non-finite, 4 stagnated
    int32_t maxit;
    int32_t stag_window; // 0 = off
    int32_t hist_base;   // offset of this Krylov run in the alpha/beta history
    int32_t sample_base; // offset of this Krylov run in the sampling schedule
    int32_t pad;
    double xscale;       // sampled value = xbase + xscale * vector (mixed inner solves)
    int32_t smethod;     // sampling: 0 method A (iteration table from the host), 1 method B
    int32_t bnext;       // method B: thresholds already reached
    int32_t slot_iter[64]; // method B: iteration (counted from the solve's start) in each slot
    double bthr2[64];    // method B: squared relative thresholds tol^{2(s+1)/(m+1)}
    double mu[64];   // C^{-1} W^T q (deflation) or generic coarse coefficients
    double u[64];    // C^{-1} W^T r (subspace correction)
    double svec[64]; // last tall-skinny product W^T v
};

template <typename T> struct Ell {
    const int64_t *sptr;
    const int32_t *col;
    const T *val;
    // Class-aligned layout (soff != nullptr, col unused): every row of slice
    // s keeps the entry at column row + soff[j] in slot k of slice-column
    // j = sptr[s] / 64 + k, the offsets of a slice ascending; a row without
    // that entry holds the value 0 there (its column, clamped into [0, n],
    // is read and multiplied by zero).  The layout moves no column indices,
    // only one offset per 64 entries.
    const int32_t *soff;
    // nonzero: values (and columns) are loaded non-temporally, for matrices
    // that outgrow the last-level cache together with the iteration's vectors
    int nt;
};

// Reducing kernels write one row of `stride` doubles per block to `part`
// (plain stores; the kernel boundary publishes them to every XCD), and a
// one-block finalize kernel sums the rows in a fixed order.

// one iteration's SpMV: p_new = z + beta p_old (p_new = z on the first
// iteration), q = A p_new; partials (p_new, q) and ||v_new||^2; optional power
// iterate v_new = A v_old / ||v_old||; optional sampling store of the iterate.
// With z == nullptr the direction p_new is given (written by the deflation
// projection) and only gathered.
template <typename T> struct SpmvIt {
    int n;
    Scal *S;
    double *part;
    Ell<T> A;
    const T *z, *pold;
    T *pnew, *q;
    const T *vold;
    T *vnew;
    const int32_t *slot_table;
    double *slots;
    const T *xit;
    const double *xbase;
    const int32_t *tmap; // tile order (nullptr: natural)
};

// x += alpha p; r -= alpha q (q = A p of the plain, subspace-corrected or
// projected deflated direction); partials ||r||^2; rows [0, l0) also do their
// forward-sweep step y = r / l_ii (they have no logically-earlier neighbour).
template <typename T> struct UpdIt {
    int n;
    Scal *S;
    double *part;
    const T *p, *q;
    T *x, *r;
    int l0;      // rows of the first sweep level fused here (0 = none)
    const T *dinv;
    T *y;
    const int32_t *tmap; // tile order (nullptr: natural)
    // optional G^T r of the new residual (G column-major n x m, m <= 16):
    // G = M^{-1} A W gives the deflation's (AW)^T z = G^T r, G = W the
    // subspace correction's W^T r, without a separate pass over z or r
    const T *G;
    int m;
    int xnt; // nonzero: x (read and written only here) is loaded and stored non-temporally
    int gnt; // nonzero: the columns of G are loaded non-temporally (G read by no other launch)
    // partials: column 0 ||r||^2, column 1 ||y||^2 of the fused level-0 rows,
    // columns 2 .. 2 + m of G^T r (row stride update_stride(m))
};
// partial columns of an update launch with G^T r of m columns (m = 0: none)
inline int update_stride(int m) { return m <= 0 ? 2 : (m <= 8 ? 10 : 18); }

// Tall-skinny s = W^T v with W row-major (n x m, W[i m + k]): lane t of a
// wavefront owns column t % P and row offset t / P (P = next power of two
// >= m), so a row's m values are read by consecutive lanes; partial rows of P.
template <typename T> struct TsDot {
    int n, m;
    const T *Wrm;
    const T *v;
    double *part;
    const Scal *S; // skip when S->done (may be null)
};

// rho = (r, z) of z = M^{-1} r: without subspace correction it equals ||y||^2
// with y = L^{-1} r (M = L L^T), so the forward launches reduce y^2 and the
// backward ones reduce nothing; with subspace correction (z + W u) the last
// forward level and the backward levels reduce (r, z + W u) as before.
// one level of the forward (L y = r) or backward (L^T z = y) IC(0) sweep;
// launches that finish rows of z write one (r, z) partial per block
template <typename T> struct Sweep {
    int r0, r1; // physical row range of the level
    int n;
    Scal *S;
    double *part; // this launch's partial slots (one per block)
    Ell<T> M;     // L (forward) or U = L^T (backward)
    const T *dinv;
    const T *r;
    T *y, *z, *zsc;
    const T *W;
    int m;        // > 0: subspace correction adds W u to zsc
    const int32_t *tmap; // tile order within [r0, r1) (nullptr: natural)
};

// Block-Jacobi IC(0) (Sec. 5.3) with tridiagonal blocks: blocks of s
// consecutive rows whose only couplings inside the block join consecutive
// rows, so that the block's IC(0) factor is its exact Cholesky factor, lower
// bidiagonal: l_k = L(k, k-1) (0 at a block start) and d_k = L(k, k).  One
// wavefront per block, R consecutive rows per lane (s <= 64 R); z = M^{-1} r
// in one launch.  rho partials: ||y||^2 (y = L^{-1} r), or (r, z + W u) with
// subspace correction; one partial per block of kBlock threads.
template <typename T> struct BjSweep {
    int n, s, nb; // rows, rows per block, blocks
    Scal *S;
    double *part;
    const T *lsub; // l_k per row (0 at block starts)
    const T *dinv; // 1 / d_k
    const T *r;
    T *z, *zsc;
    const T *W;
    int m; // > 0: subspace correction adds W u to zsc
};

// x += alpha p, r -= alpha q and the block-Jacobi z = M^{-1} r of the new r in
// one launch (no subspace correction); partials ||r||^2 and ||y||^2 per block
// of kBlock threads (stride 2)
template <typename T> struct UpdBj {
    int n, s, nb;
    Scal *S;
    double *part;
    const T *p, *q;
    T *x, *r;
    const T *lsub, *dinv;
    T *z;
};

// finalize after the SpMV: alpha = rho / (p, q); with the power iterate also
// its scale 1 / ||v_new||
struct FinAlpha {
    Scal *S;
    const double *part;
    int nblk, stride, power;
    double *hist_alpha;
};
// finalize after the preconditioner: stop test on ||r||^2, rho, beta; with
// deflation also mu = C^{-1} (AW)^T z for the projected direction
struct FinRho {
    Scal *S;
    const double *part_upd; // column 0 = ||r||^2 partials, column 1 = ||y||^2 of the fused level-0 rows
    int nblk_upd, stride_upd;
    const double *part_sweep; // rho partials of the preconditioner launches
    int nsweep;
    int rho_upd; // rho also takes column 1 of the update partials (level 0 fused there)
    double *hist_beta;
    int init; // 1: first preconditioner application of a solve (only rho);
              // 2: after a residual replacement (rho and beta of the new residual)
    const double *part_s; // (AW)^T z partials (deflated), nblk_s x stride_s, columns c0_s ..
    int nblk_s, stride_s, c0_s, m;
    const double *Cinv;
    int32_t *slot_table;  // sampling method B: slot of the next store, set here (nullptr: none)
    int nslots;
};

// zhat = z - W mu (W column-major n x m, mu = S->mu), the projected
// preconditioned residual of the deflated iteration, and the next direction
// p_new = zhat + beta p_old (p_new = zhat before the first iteration)
template <typename T> struct Proj {
    int n, m;
    const Scal *S;
    const T *z, *W;
    const T *pold;
    T *pnew;
    const int32_t *tmap; // tile order (nullptr: natural)
};
// generic finalize of a per-solve reduction: tot[k] = column sums
struct FinGen {
    Scal *S;
    const double *part;
    int nblk, stride, ncol;
    double *out0;     // *out0 = scale0 * tot[0] (optional)
    double scale0;
    int check;        // S->rr = tot[0]; S->done = 1 when tot[0] <= S->tol2
    double settol;    // >= 0: S->bnorm2 = tot[0], S->tol2 = settol^2 tot[0]
    int vcol0, m;     // columns vcol0 .. vcol0+m-1 form a vector s (m > 0)
    const double *Cinv;
    double *coef;     // coef = cscale * C^{-1} s (optional)
    double cscale;
    int store_svec;   // S->svec = s
};

// y = diag(d) x + M x over the stored entries (sorted layout): L^T x with
// M = U, L x with M = L, d = diag(L)
void launch_tri_mul(int n, Ell<double> M, const double *d, const double *x, double *y, hipStream_t s);
// to64[e] = from[src[e]] (0 where src[e] < 0), to32 = (float)to64: values of
// a class-aligned copy from the sorted layout
void launch_repack(int64_t size, const int64_t *src, const double *from, double *to64, float *to32, hipStream_t s);
void launch_spmv_it(const SpmvIt<double> &a, bool power, int grid, hipStream_t s);
void launch_spmv_it(const SpmvIt<float> &a, bool power, int grid, hipStream_t s);
// kind 0 plain / subspace correction, 1 deflated
void launch_update_it(const UpdIt<double> &a, int grid, hipStream_t s);
void launch_update_it(const UpdIt<float> &a, int grid, hipStream_t s);
void launch_proj(const Proj<double> &a, int grid, hipStream_t s);
void launch_proj(const Proj<float> &a, int grid, hipStream_t s);
// the projection (m <= 16) with the backward sweep of the first level (b: rows
// [0, b.r1), b.M = U) in the same launch; grid as for launch_proj
void launch_bwd0_proj(const Sweep<double> &b, const Proj<double> &a, int grid, hipStream_t s);
void launch_bwd0_proj(const Sweep<float> &b, const Proj<float> &a, int grid, hipStream_t s);
void launch_tsdot_rm(const TsDot<double> &a, int grid, hipStream_t s);
void launch_tsdot_rm(const TsDot<float> &a, int grid, hipStream_t s);
int tsdot_stride(int m);
int tsdot_grid(int64_t n, int m);
// row-major copy Wrm[i m + k] = W[k n + i] (FP64 and FP32)
void launch_to_rowmajor(int n, int m, const double *W, double *Wrm, float *Wrm32, hipStream_t s);
void launch_fwd(const Sweep<double> &a, bool last, bool sc, int grid, hipStream_t s);
void launch_fwd(const Sweep<float> &a, bool last, bool sc, int grid, hipStream_t s);
void launch_bwd(const Sweep<double> &a, bool sc, int grid, hipStream_t s);
void launch_bwd(const Sweep<float> &a, bool sc, int grid, hipStream_t s);
// the same sweeps (forward: not the last level) with two rows per thread,
// for levels of more than kPairTiles tiles; the grid covers half of the
// level's tiles
void launch_fwd2(const Sweep<double> &a, bool sc, int grid, hipStream_t s);
void launch_fwd2(const Sweep<float> &a, bool sc, int grid, hipStream_t s);
void launch_bwd2(const Sweep<double> &a, bool sc, int grid, hipStream_t s);
void launch_bwd2(const Sweep<float> &a, bool sc, int grid, hipStream_t s);
// block-Jacobi z = M^{-1} r; returns the number of rho partials written (the
// grid: at most kMaxGrid blocks, wavefronts loop over the Jacobi blocks)
int bj_grid(int nb);
int launch_bj(const BjSweep<double> &a, bool sc, hipStream_t s);
int launch_bj(const BjSweep<float> &a, bool sc, hipStream_t s);
int launch_update_bj(const UpdBj<double> &a, hipStream_t s);
int launch_update_bj(const UpdBj<float> &a, hipStream_t s);
void launch_copyz(const Sweep<double> &a, bool sc, int grid, hipStream_t s);
void launch_copyz(const Sweep<float> &a, bool sc, int grid, hipStream_t s);
void launch_fin_alpha(const FinAlpha &f, hipStream_t s);
// u = C^{-1} s with s = columns c0 .. c0 + m of a partial table
void launch_fin_u(Scal *S, const double *part, int nblk, int stride, int c0, int m, const double *Cinv,
                  hipStream_t s);
void launch_fin_rho(const FinRho &f, hipStream_t s);
void launch_fin_gen(const FinGen &f, hipStream_t s);
// stride of the partial rows of the iteration kernels
int spmv_stride(bool power);
// grid of a reducing row kernel over `rows` rows with `stride` partials per block
int grid_red(int64_t rows, int stride);

// ---- per-solve and setup kernels (FP64 unless stated) ----
// Each reducing launcher writes partials to `part` with the grid it returns
// through *nblk; FinGen then reduces them.
void launch_gather(int n, const int32_t *idx, const double *src, double *dst, hipStream_t s);
void launch_scatter(int n, const int32_t *idx, const double *src, double *dst, hipStream_t s);
void launch_fill(int n, double *dst, double v, hipStream_t s);
void launch_fill(int n, float *dst, float v, hipStream_t s);
// partial x.y (stride 1)
void launch_dot(int n, const double *a, const double *b, double *part, int *nblk, hipStream_t s);
// t = b - A x (A in FP64); partials [||t||^2, W^T t] (stride 1 + bucket(m))
void launch_resid(int n, Ell<double> A, const double *b, const double *x, double *t, const double *W,
                  int m, double *part, int *nblk, int *stride, hipStream_t s);
// y += sign * M coef (M: n x m column-major); partials ||y||^2 when part != null
void launch_axpy_cols(int n, double *y, const double *M, int m, const double *coef, double sign,
                      double *part, int *nblk, hipStream_t s);
// partials W^T v (stride bucket(m))
void launch_tsdot(int n, const double *W, int m, const double *v, double *part, int *nblk, int *stride,
                  hipStream_t s);
// y = A x (FP64, either layout)
void launch_spmv(int n, Ell<double> A, const double *x, double *y, hipStream_t s);
// partials (v, A v)
void launch_rayleigh(int n, Ell<double> A, const double *v, double *part, int *nblk, hipStream_t s);
void launch_rayleigh(int n, Ell<float> A, const float *v, double *part, int *nblk, hipStream_t s);
// sample store of the iterate (used when a solve stops at maxit)
void launch_sample_store(int n, double *slot, const double *x, hipStream_t s);
// casts
void launch_cast_scale(int n, const double *src, float *dst, double scale, hipStream_t s);
void launch_cast(int64_t n, const double *src, float *dst, hipStream_t s);
void launch_add_scaled(int n, double *x, const float *d, double scale, hipStream_t s);
void launch_sub(int n, const double *a, const double *b, double *dst, hipStream_t s);
// b = f + c x (x may be null)
void launch_axpby(int n, const double *f, const double *x, double c, double *b, hipStream_t s);
void launch_scale_copy(int n, const double *src, double *dst, double scale, hipStream_t s);

// IC(0) factor of one level (FP64, in place on the L values; writes ldiag)
void launch_factor_level(int r0, int r1, int n, Ell<double> L, double *lval, const double *adiag,
                         double *ldiag, int *bad, hipStream_t s);
void launch_finish_factor(int n, const double *ldiag, double *dinv, float *dinv32, hipStream_t s);
// block-Jacobi factor of tridiagonal blocks (one lane per block, in place on
// lval = a_ij of L's sorted layout): ldiag, l_k as lsub / lsub32
void launch_factor_bj(int n, int s, Ell<double> L, double *lval, const double *adiag, double *ldiag, double *lsub,
                      float *lsub32, int *bad, hipStream_t st);
void launch_gather_u(int64_t cnt, const int64_t *map, const double *lval, double *uval,
                     hipStream_t s);
// dst[i] = val[src[i]] (0 where src < 0), optional FP32 copy
void launch_map_values(int64_t cnt, const int32_t *src, const double *val, double *dst, float *dst32,
                       hipStream_t s);

// A E for m columns (column-major, FP64)
void launch_spmm(int n, Ell<double> A, const double *E, int m, double *AE, hipStream_t s);
// block partials of E^T F (E: n x ma, F: n x mb, column-major) with FP64 MFMA;
// then the deterministic sum over blocks into G (ma x mb, row-major)
int gram_grid(int n);
void launch_gram(int n, const double *E, int ma, const double *F, int mb, double *part, double *G,
                 int grid, hipStream_t s);
// Y = X T (X: n x ma col-major, T: ma x mb col-major on device)
void launch_tsgemm(int n, const double *X, int ma, const double *T, int mb, double *Y, hipStream_t s);

// gradient with respect to stored values: g[k] = -lam[row k] x[col k] (user CSR)
void launch_grad(int n, const int64_t *rowptr, const int32_t *col, const double *lam,
                 const double *x, double *g, hipStream_t s);

// streaming probes (not part of the method): kind 0 copies n doubles src ->
// dst, kind 1 sums them (one partial per block into dst); n even, 16-byte
// aligned pointers
void launch_probe(int kind, const double *src, double *dst, int64_t n, int grid, hipStream_t s);

// a level of more tiles than one round of resident wavefronts (8 per SIMD
// on 256 CUs: 2048 blocks of kBlock threads) runs two rows per thread
constexpr int kPairTiles = 2048;
inline bool sweep_pairs(int64_t rows) { return (rows + kBlock - 1) / kBlock > kPairTiles; }

// FP32 update (plain / projected form) and projection launches (m <= 16)
// over more than kPairTiles tiles run two rows per thread; stream_grid is
// the grid (and partial count) of such a launch
template <typename T> inline bool stream_pairs(int64_t rows) {
    return sizeof(T) == 4 && (rows + kBlock - 1) / kBlock > kPairTiles;
}
template <typename T> inline int stream_grid(int64_t rows) {
    return grid_red(stream_pairs<T>(rows) ? (rows + 1) / 2 : rows, 1);
}

inline int grid_for(int64_t rows) {
    int64_t g = (rows + kBlock - 1) / kBlock;
    if (g > kMaxGrid) g = kMaxGrid;
    if (g > 8) g = (g + 7) / 8 * 8; // whole XCD rounds
    if (g < 1) g = 1;
    return (int)g;
}

} // namespace esd
