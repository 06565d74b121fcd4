/*
 * Oracle: a plain, slow, single-threaded FP64 CPU implementation of the
 * error-vector-sampling accelerated ICCG method of Iwashita, Ikehara, Fukaya
 * and Mifune, "Convergence Acceleration of Preconditioned CG Solver Based on
 * Error Vector Sampling for a Sequence of Linear Systems" (arXiv 2203.08498).
 *
 * THIS IS TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library; the two are compared on identical
 * seeded inputs.
 *
 * Every routine follows the paper's definition step by step, in the paper's
 * order, with no blocking, fusion or reordering:
 *   - ordering: rows sorted stably by colour (natural order = identity);
 *   - IC(0): incomplete Cholesky restricted to the stored lower pattern (the
 *     paper's "IC" preconditioner, Sec. 4.4 and Sec. 5.2);
 *   - PCG: Alg. "PCG method with condition number estimation" (Sec. 5.4),
 *     including the power iteration fused with the product (q v) = A (p v);
 *   - sampling method A: Appendix A, Alg. "Selection of approximate solution
 *     vectors";
 *   - error vectors, Gram-Schmidt, Rayleigh-Ritz, theta selection: Sec. 4.2,
 *     eqs. (ek), (ekd), (Rayleigh-Ritz), (Rayleigh-Ritz2), (bk);
 *   - deflated PCG: Alg. "Deflated PCG method" (Sec. 3.3) with projector
 *     eq. (deflation:projector) and the final assembly of eqs. (split)-(x2);
 *   - subspace-correction preconditioned CG: eq. (mc) (Sec. 3.2);
 *   - kappa: (K2) the paper's power-method lambda_max over the smallest Ritz
 *     value (Sec. 5.4); (K1) extreme eigenvalues of the Lanczos tridiagonal
 *     matrix built from the CG coefficients (textbook CG-Lanczos relation,
 *     Saad, Iterative Methods for Sparse Linear Systems, 2nd ed., Sec. 6.7.3);
 *   - adjoint gradient of a linear solve with respect to stored values;
 *   - block-Jacobi IC(0), the paper's parallel preconditioner (Sec. 5.3, with
 *     Saad's block Jacobi): rows split into blocks of consecutive rows, IC(0)
 *     of the block-diagonal part of A, i.e. every coupling between two blocks
 *     is left out of the factor (A itself keeps them).
 *
 * Readings where the paper is silent or garbled are taken as follows:
 *   - beta carries a plus sign (the minus printed in Alg. "Deflated PCG
 *     method" contradicts Alg. "PCG method with condition number estimation");
 *   - the stop test is ||r_i||_2 <= eps ||b||_2 on the recurrence residual and
 *     is also applied to r_0 (zero iterations when it already holds);
 *   - sampling happens only when the convergence check did not stop the loop;
 *     x_0 is never sampled;
 *   - Gram-Schmidt is classical with two passes, vectors in sampling order,
 *     normalised first, dropped when the re-orthogonalised norm is <= 1e-10;
 *   - Ritz values strictly below theta are selected; C = W^T A W is formed
 *     explicitly and factored by Cholesky;
 *   - subspace correction is a pure additive preconditioner (no coarse
 *     pre- or post-correction of x).
 *
 * Parity pins live in tests/: worked sampling examples (Sec. 4.3 and the
 * commented variant), dense solves, dense eigendecompositions, closed-form
 * Poisson eigenpairs, invariants W^T r = 0 and W^T W = I.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_AUX_EMPTY 2
#define OR_EINVAL (-1)
#define OR_ENOTSPD (-2)
#define OR_ENUMERIC (-4)
#define OR_ENOAUX (-5)
#define OR_ENOSAMPLES (-6)

#define MODE_PLAIN 0
#define MODE_DEFLATED 1
#define MODE_SUBSPACE 2

#define FLAG_NOPREC 1 /* M = I (plain CG) */
#define FLAG_POWER 2  /* run the power iteration of Alg. PCG-con */
#define FLAG_SAMPLE 4 /* sampling method A during this solve */

typedef struct {
    int64_t n, nnz;
    /* user matrix (full symmetric CSR) */
    int64_t *urp; int32_t *ucol; double *uval;
    /* permutation: perm[new] = old, iperm[old] = new */
    int32_t *perm, *iperm;
    /* permuted matrix */
    int64_t *rp; int32_t *col; double *val;
    /* IC(0) factor: lower triangle incl. diagonal, permuted order */
    int64_t *lrp; int32_t *lcol; double *lval;
    int factored;
    /* block-Jacobi IC(0): > 0 = rows per block (blocks of consecutive rows of
       the natural order); 0 = IC(0) of the whole matrix */
    int64_t block_rows;
    /* sampling */
    int m_req;
    int samp_method;   /* 0: method A (Appendix A), 1: method B (relative-residual thresholds) */
    int samp_resid;    /* 1: store residual vectors r_i instead of iterates x_i */
    int rr_op;         /* Rayleigh-Ritz operator: 0 A (eq. (Rayleigh-Ritz)), 1 M^{-1}A (its footnote) */
    double *slots; int32_t *slot_iter; double *xN;
    /* auxiliary space (permuted order, column-major n x k) */
    int m_bar, m_tilde;
    double *E, *AE, *W, *AW, *C, *R; /* R: lower Cholesky factor of C */
    double ritz[4096];
    /* power method */
    double *v; int have_v;
    /* history of the last solve */
    int iters; double *alpha, *beta; int hist_cap;
    int nsamples; int32_t sample_iters[4096];
} orc;

/* ------------------------------------------------------------------ */
/* small helpers                                                         */
/* ------------------------------------------------------------------ */

static double dot(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static void spmv(const orc *o, const double *x, double *y) {
    for (int64_t i = 0; i < o->n; ++i) {
        double s = 0.0;
        for (int64_t k = o->rp[i]; k < o->rp[i + 1]; ++k) s += o->val[k] * x[o->col[k]];
        y[i] = s;
    }
}

static void to_perm(const orc *o, const double *u, double *p) {
    for (int64_t i = 0; i < o->n; ++i) p[i] = u[o->perm[i]];
}
static void from_perm(const orc *o, const double *p, double *u) {
    for (int64_t i = 0; i < o->n; ++i) u[o->perm[i]] = p[i];
}

/* ------------------------------------------------------------------ */
/* setup: stable sort by colour, permuted CSR                           */
/* ------------------------------------------------------------------ */

orc *orc_create(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                const int32_t *colors) {
    if (n <= 0) return NULL;
    orc *o = (orc *)calloc(1, sizeof(orc));
    o->n = n;
    o->nnz = rowptr[n];
    o->urp = malloc((n + 1) * sizeof(int64_t));
    o->ucol = malloc(o->nnz * sizeof(int32_t));
    o->uval = malloc(o->nnz * sizeof(double));
    memcpy(o->urp, rowptr, (n + 1) * sizeof(int64_t));
    memcpy(o->ucol, col, o->nnz * sizeof(int32_t));
    memcpy(o->uval, val, o->nnz * sizeof(double));
    o->perm = malloc(n * sizeof(int32_t));
    o->iperm = malloc(n * sizeof(int32_t));
    /* stable sort of rows by colour: scan colours in increasing order */
    if (colors) {
        int32_t cmax = 0;
        for (int64_t i = 0; i < n; ++i) if (colors[i] > cmax) cmax = colors[i];
        int64_t p = 0;
        for (int32_t c = 0; c <= cmax; ++c)
            for (int64_t i = 0; i < n; ++i)
                if (colors[i] == c) o->perm[p++] = (int32_t)i;
    } else {
        for (int64_t i = 0; i < n; ++i) o->perm[i] = (int32_t)i;
    }
    for (int64_t i = 0; i < n; ++i) o->iperm[o->perm[i]] = (int32_t)i;
    /* permuted matrix, columns sorted ascending (insertion sort per row) */
    o->rp = malloc((n + 1) * sizeof(int64_t));
    o->col = malloc(o->nnz * sizeof(int32_t));
    o->val = malloc(o->nnz * sizeof(double));
    o->rp[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t old = o->perm[i];
        int64_t len = rowptr[old + 1] - rowptr[old];
        int64_t base = o->rp[i];
        for (int64_t t = 0; t < len; ++t) {
            int32_t c = o->iperm[col[rowptr[old] + t]];
            double v = val[rowptr[old] + t];
            int64_t pos = base + t;
            while (pos > base && o->col[pos - 1] > c) {
                o->col[pos] = o->col[pos - 1];
                o->val[pos] = o->val[pos - 1];
                --pos;
            }
            o->col[pos] = c;
            o->val[pos] = v;
        }
        o->rp[i + 1] = base + len;
    }
    return o;
}

/* Block-Jacobi IC(0) preconditioner (Sec. 5.3): natural order, blocks of
 * block_rows consecutive rows (the last one may be shorter). */
orc *orc_create_bj(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val, int64_t block_rows) {
    if (block_rows <= 0) return NULL;
    orc *o = orc_create(n, rowptr, col, val, NULL);
    if (o) o->block_rows = block_rows;
    return o;
}

/* entry (i, j) belongs to the matrix the preconditioner is built from */
static int in_factor(const orc *o, int64_t i, int64_t j) {
    return o->block_rows <= 0 || i / o->block_rows == j / o->block_rows;
}

static void free_aux(orc *o) {
    free(o->E); free(o->AE); free(o->W); free(o->AW); free(o->C); free(o->R);
    o->E = o->AE = o->W = o->AW = o->C = o->R = NULL;
    o->m_bar = o->m_tilde = 0;
}

void orc_free(orc *o) {
    if (!o) return;
    free(o->urp); free(o->ucol); free(o->uval);
    free(o->perm); free(o->iperm);
    free(o->rp); free(o->col); free(o->val);
    free(o->lrp); free(o->lcol); free(o->lval);
    free(o->slots); free(o->slot_iter); free(o->xN);
    free_aux(o);
    free(o->v); free(o->alpha); free(o->beta);
    free(o);
}

void orc_perm(const orc *o, int32_t *perm) { memcpy(perm, o->perm, o->n * sizeof(int32_t)); }

int64_t orc_permuted_csr(const orc *o, int64_t *rp, int32_t *col, double *val) {
    if (rp) memcpy(rp, o->rp, (o->n + 1) * sizeof(int64_t));
    if (col) memcpy(col, o->col, o->nnz * sizeof(int32_t));
    if (val) memcpy(val, o->val, o->nnz * sizeof(double));
    return o->nnz;
}

/* ------------------------------------------------------------------ */
/* IC(0): incomplete Cholesky on the stored lower pattern               */
/* (block Jacobi: of the block-diagonal part of the matrix)              */
/* ------------------------------------------------------------------ */

int orc_factor_ic0(orc *o) {
    int64_t n = o->n;
    free(o->lrp); free(o->lcol); free(o->lval);
    o->lrp = malloc((n + 1) * sizeof(int64_t));
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = o->rp[i]; k < o->rp[i + 1]; ++k)
            if (o->col[k] <= i && in_factor(o, i, o->col[k])) ++cnt;
    o->lcol = malloc(cnt * sizeof(int32_t));
    o->lval = malloc(cnt * sizeof(double));
    o->lrp[0] = 0;
    int64_t p = 0;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t k = o->rp[i]; k < o->rp[i + 1]; ++k)
            if (o->col[k] <= i && in_factor(o, i, o->col[k])) { o->lcol[p] = o->col[k]; o->lval[p] = o->val[k]; ++p; }
        o->lrp[i + 1] = p;
    }
    o->factored = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t rs = o->lrp[i], re = o->lrp[i + 1]; /* last entry is the diagonal */
        if (re == rs || o->lcol[re - 1] != i) return OR_ENOTSPD; /* no diagonal stored */
        for (int64_t a = rs; a < re - 1; ++a) {
            int32_t j = o->lcol[a];
            /* l_ij = (a_ij - sum_{k<j} l_ik l_jk) / l_jj over k stored in both rows */
            double s = o->lval[a];
            int64_t b = o->lrp[j], be = o->lrp[j + 1] - 1; /* row j without its diagonal */
            for (int64_t t = rs; t < a; ++t) {
                int32_t kk = o->lcol[t];
                while (b < be && o->lcol[b] < kk) ++b;
                if (b < be && o->lcol[b] == kk) s -= o->lval[t] * o->lval[b];
            }
            o->lval[a] = s / o->lval[o->lrp[j + 1] - 1];
        }
        double d = o->lval[re - 1];
        for (int64_t t = rs; t < re - 1; ++t) d -= o->lval[t] * o->lval[t];
        if (!(d > 0.0)) return OR_ENOTSPD;
        o->lval[re - 1] = sqrt(d);
    }
    o->factored = 1;
    return OR_OK;
}

int64_t orc_factor_csr(const orc *o, int64_t *rp, int32_t *col, double *val) {
    if (!o->lrp) return -1;
    int64_t cnt = o->lrp[o->n];
    if (rp) memcpy(rp, o->lrp, (o->n + 1) * sizeof(int64_t));
    if (col) memcpy(col, o->lcol, cnt * sizeof(int32_t));
    if (val) memcpy(val, o->lval, cnt * sizeof(double));
    return cnt;
}

/* z = (L L^T)^{-1} r: forward L y = r (ascending), backward L^T z = y (descending) */
static void prec_apply(const orc *o, const double *r, double *z) {
    int64_t n = o->n;
    for (int64_t i = 0; i < n; ++i) {
        double s = r[i];
        int64_t re = o->lrp[i + 1] - 1;
        for (int64_t k = o->lrp[i]; k < re; ++k) s -= o->lval[k] * z[o->lcol[k]];
        z[i] = s / o->lval[re];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        int64_t re = o->lrp[i + 1] - 1;
        z[i] = z[i] / o->lval[re];
        for (int64_t k = o->lrp[i]; k < re; ++k) z[o->lcol[k]] -= o->lval[k] * z[i];
    }
}

/* ------------------------------------------------------------------ */
/* user-order wrappers used by the tests                                */
/* ------------------------------------------------------------------ */

void orc_spmv(const orc *o, const double *x_user, double *y_user) {
    double *xp = malloc(o->n * sizeof(double)), *yp = malloc(o->n * sizeof(double));
    to_perm(o, x_user, xp);
    spmv(o, xp, yp);
    from_perm(o, yp, y_user);
    free(xp); free(yp);
}

int orc_prec_apply(const orc *o, const double *r_user, double *z_user) {
    if (!o->factored) return OR_EINVAL;
    double *rp = malloc(o->n * sizeof(double)), *zp = malloc(o->n * sizeof(double));
    to_perm(o, r_user, rp);
    prec_apply(o, rp, zp);
    from_perm(o, zp, z_user);
    free(rp); free(zp);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* sampling method A (Appendix A)                                        */
/* ------------------------------------------------------------------ */

/* slot index of iteration i: (sum_{l>=0} (-1)^l floor((i-1)/m^l)) mod m.
 * Terms with m^l > i-1 vanish, so the sum stops there (any l_max with
 * m^{l_max} > N_max gives the same value). */
static int sample_slot(int64_t i, int m) {
    int64_t s = 0, pw = 1, sign = 1;
    if (m == 1) return 0;
    while (pw <= i - 1) {
        s += sign * ((i - 1) / pw);
        sign = -sign;
        pw *= m;
    }
    return (int)(s % m);
}

/* Replays the schedule for a solve that stops at iteration N (convergence check
 * at N stops before sampling).  Writes the surviving (iteration, slot) pairs
 * ordered by slot and returns how many slots are filled. */
int orc_sample_schedule(int m, int64_t N, int64_t *iters_by_slot) {
    int64_t h = 1;
    for (int s = 0; s < m; ++s) iters_by_slot[s] = 0;
    for (int64_t i = 1; i < N; ++i) { /* iteration N converged: no sample there */
        if (i % h == 0) {
            iters_by_slot[sample_slot(i, m)] = i;
            if (i == h * m) h *= 2;
        }
    }
    int filled = 0;
    for (int s = 0; s < m; ++s) if (iters_by_slot[s] > 0) ++filled;
    return filled;
}

/* Install k approximate solutions X (n x k, column-major, user order) as if a
 * sampling solve had stored them at iterations 1..k, and x_N as its final
 * solution (checkpoint/resume of the sampling step). */
int orc_load_samples(orc *o, const double *X_user, int k, const double *xN_user) {
    if (k <= 0 || k > 4096) return OR_EINVAL;
    o->m_req = k;
    free(o->slots); free(o->slot_iter); free(o->xN);
    o->slots = malloc((size_t)k * o->n * sizeof(double));
    o->slot_iter = calloc(k, sizeof(int32_t));
    o->xN = malloc(o->n * sizeof(double));
    for (int s = 0; s < k; ++s) {
        to_perm(o, X_user + (int64_t)s * o->n, o->slots + (int64_t)s * o->n);
        o->slot_iter[s] = s + 1;
    }
    to_perm(o, xN_user, o->xN);
    o->nsamples = k;
    o->samp_resid = 0;
    return OR_OK;
}

/* method: 0 = sampling method A, 1 = sampling method B (Sec. 4.3), plus 16
 * to store the residual vectors r_i instead of the iterates x_i (the
 * comparison of Sec. 5.2, "Sampling of residual vectors"). */
int orc_arm_sampling(orc *o, int m, int method) {
    if (m <= 0 || m > 4096) return OR_EINVAL;
    if ((method & ~16) != 0 && (method & ~16) != 1) return OR_EINVAL;
    o->samp_method = method & 1;
    o->samp_resid = (method & 16) != 0;
    o->m_req = m;
    free(o->slots); free(o->slot_iter);
    o->slots = malloc((size_t)m * o->n * sizeof(double));
    o->slot_iter = calloc(m, sizeof(int32_t));
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* small dense linear algebra (own code)                                 */
/* ------------------------------------------------------------------ */

/* Cyclic Jacobi eigenvalue method for a symmetric k x k matrix (row-major in
 * a, overwritten).  Eigenvalues ascending in w, eigenvectors in the columns of
 * V (row-major k x k).  Golub & Van Loan, Matrix Computations, Sec. 8.5. */
void orc_sym_eig(int k, double *a, double *w, double *V) {
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) V[i * k + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                tot += a[i * k + j] * a[i * k + j];
                if (i != j) off += a[i * k + j] * a[i * k + j];
            }
        if (off <= 1e-32 * tot || off == 0.0) break;
        for (int p = 0; p < k - 1; ++p)
            for (int q = p + 1; q < k; ++q) {
                double apq = a[p * k + q];
                if (apq == 0.0) continue;
                double tau = (a[q * k + q] - a[p * k + p]) / (2.0 * apq);
                double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                for (int r = 0; r < k; ++r) { /* columns p, q */
                    double arp = a[r * k + p], arq = a[r * k + q];
                    a[r * k + p] = c * arp - s * arq;
                    a[r * k + q] = s * arp + c * arq;
                }
                for (int r = 0; r < k; ++r) { /* rows p, q */
                    double apr = a[p * k + r], aqr = a[q * k + r];
                    a[p * k + r] = c * apr - s * aqr;
                    a[q * k + r] = s * apr + c * aqr;
                }
                for (int r = 0; r < k; ++r) {
                    double vrp = V[r * k + p], vrq = V[r * k + q];
                    V[r * k + p] = c * vrp - s * vrq;
                    V[r * k + q] = s * vrp + c * vrq;
                }
            }
    }
    for (int i = 0; i < k; ++i) w[i] = a[i * k + i];
    /* selection sort ascending, permuting eigenvector columns */
    for (int i = 0; i < k; ++i) {
        int mi = i;
        for (int j = i + 1; j < k; ++j) if (w[j] < w[mi]) mi = j;
        if (mi != i) {
            double t = w[i]; w[i] = w[mi]; w[mi] = t;
            for (int r = 0; r < k; ++r) { t = V[r * k + i]; V[r * k + i] = V[r * k + mi]; V[r * k + mi] = t; }
        }
    }
}

/* Cholesky C = R R^T (R lower, row-major k x k). Returns 0 or OR_ENOTSPD. */
static int cholesky(int k, const double *C, double *R) {
    memset(R, 0, (size_t)k * k * sizeof(double));
    for (int i = 0; i < k; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = C[i * k + j];
            for (int t = 0; t < j; ++t) s -= R[i * k + t] * R[j * k + t];
            if (i == j) {
                if (!(s > 0.0)) return OR_ENOTSPD;
                R[i * k + i] = sqrt(s);
            } else {
                R[i * k + j] = s / R[j * k + j];
            }
        }
    return OR_OK;
}

/* u = C^{-1} f with C = R R^T */
static void coarse_solve(const orc *o, const double *f, double *u) {
    int k = o->m_tilde;
    const double *R = o->R;
    for (int i = 0; i < k; ++i) {
        double s = f[i];
        for (int t = 0; t < i; ++t) s -= R[i * k + t] * u[t];
        u[i] = s / R[i * k + i];
    }
    for (int i = k - 1; i >= 0; --i) {
        double s = u[i];
        for (int t = i + 1; t < k; ++t) s -= R[t * k + i] * u[t];
        u[i] = s / R[i * k + i];
    }
}

/* out = M^T v for a column-major n x k matrix M */
static void tmatvec(int64_t n, int k, const double *M, const double *v, double *out) {
    for (int j = 0; j < k; ++j) out[j] = dot(n, M + (int64_t)j * n, v);
}
/* y += M u */
static void matvec_add(int64_t n, int k, const double *M, const double *u, double *y, double sgn) {
    for (int j = 0; j < k; ++j) {
        const double *c = M + (int64_t)j * n;
        for (int64_t i = 0; i < n; ++i) y[i] += sgn * u[j] * c[i];
    }
}

/* ------------------------------------------------------------------ */
/* auxiliary matrix: AW, C = W^T A W, Cholesky                          */
/* ------------------------------------------------------------------ */

static int finish_aux(orc *o) {
    int64_t n = o->n;
    int k = o->m_tilde;
    if (k == 0) return OR_AUX_EMPTY;
    o->C = malloc((size_t)k * k * sizeof(double));
    o->R = malloc((size_t)k * k * sizeof(double));
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b)
            o->C[a * k + b] = dot(n, o->W + (int64_t)a * n, o->AW + (int64_t)b * n);
    for (int a = 0; a < k; ++a) /* symmetrise */
        for (int b = 0; b < a; ++b) {
            double s = 0.5 * (o->C[a * k + b] + o->C[b * k + a]);
            o->C[a * k + b] = o->C[b * k + a] = s;
        }
    return cholesky(k, o->C, o->R);
}

/* y = M x = L (L^T x) with the IC(0) factor L (lower, diagonal included). */
static void apply_M_product(const orc *o, const double *x, double *y) {
    int64_t n = o->n;
    double *t = calloc(n, sizeof(double));
    for (int64_t i = 0; i < n; ++i)              /* t = L^T x, row i of L scattered */
        for (int64_t a = o->lrp[i]; a < o->lrp[i + 1]; ++a) t[o->lcol[a]] += o->lval[a] * x[i];
    for (int64_t i = 0; i < n; ++i) {            /* y = L t */
        double s = 0.0;
        for (int64_t a = o->lrp[i]; a < o->lrp[i + 1]; ++a) s += o->lval[a] * t[o->lcol[a]];
        y[i] = s;
    }
    free(t);
}

/* Operator of the next build_aux's Rayleigh-Ritz step: 0 = A, 1 = the
 * preconditioned matrix M^{-1}A (footnote of eq. (Rayleigh-Ritz)), taken in
 * the M inner product where it is self-adjoint: E^T A E t = lambda E^T M E t. */
int orc_set_rr(orc *o, int op) {
    if (op != 0 && op != 1) return OR_EINVAL;
    if (op == 1 && !o->factored) return OR_EINVAL;
    o->rr_op = op;
    return OR_OK;
}

/* Rayleigh-Ritz on the span of the sampled error vectors (Sec. 4.2):
 * eq. (ek) error vectors, eq. (ekd) Gram-Schmidt, eq. (Rayleigh-Ritz) the
 * projected eigenproblem with A itself, eq. (bk) selection below theta. */
int orc_build_aux(orc *o, double theta, double *ritz_out, int *m_bar, int *m_tilde) {
    int64_t n = o->n;
    if (o->nsamples <= 0 || !o->slots || !o->xN) return OR_ENOSAMPLES;
    free_aux(o);
    int m = o->m_req;
    int order[4096], cnt = 0;
    for (int s = 0; s < m; ++s) if (o->slot_iter[s] > 0) order[cnt++] = s;
    for (int a = 1; a < cnt; ++a) { /* by sampled iteration, ascending */
        int t = order[a], b = a;
        while (b > 0 && o->slot_iter[order[b - 1]] > o->slot_iter[t]) { order[b] = order[b - 1]; --b; }
        order[b] = t;
    }
    double *E = malloc((size_t)(cnt > 0 ? cnt : 1) * n * sizeof(double));
    double *v = malloc(n * sizeof(double));
    double c[4096];
    int kept = 0;
    for (int a = 0; a < cnt; ++a) {
        const double *xs = o->slots + (int64_t)order[a] * n;
        if (o->samp_resid)
            for (int64_t i = 0; i < n; ++i) v[i] = xs[i];               /* sampled residual r_s */
        else
            for (int64_t i = 0; i < n; ++i) v[i] = o->xN[i] - xs[i];  /* eq. (ek) */
        double nv = sqrt(dot(n, v, v));
        if (!(nv > 0.0)) continue;
        for (int64_t i = 0; i < n; ++i) v[i] /= nv;
        for (int pass = 0; pass < 2; ++pass) {                          /* CGS, twice */
            tmatvec(n, kept, E, v, c);
            matvec_add(n, kept, E, c, v, -1.0);
        }
        nv = sqrt(dot(n, v, v));
        if (nv <= 1e-10) continue;                                        /* drop */
        for (int64_t i = 0; i < n; ++i) E[(int64_t)kept * n + i] = v[i] / nv;
        ++kept;
    }
    o->m_bar = kept;
    *m_bar = kept;
    *m_tilde = 0;
    if (kept == 0) { free(E); free(v); return OR_AUX_EMPTY; }
    /* G = E^T (A E), symmetrised */
    double *AE = malloc((size_t)kept * n * sizeof(double));
    for (int a = 0; a < kept; ++a) spmv(o, E + (int64_t)a * n, AE + (int64_t)a * n);
    double *G = malloc((size_t)kept * kept * sizeof(double));
    double *V = malloc((size_t)kept * kept * sizeof(double));
    for (int a = 0; a < kept; ++a)
        for (int b = 0; b < kept; ++b) G[a * kept + b] = dot(n, E + (int64_t)a * n, AE + (int64_t)b * n);
    for (int a = 0; a < kept; ++a)
        for (int b = 0; b < a; ++b) {
            double s = 0.5 * (G[a * kept + b] + G[b * kept + a]);
            G[a * kept + b] = G[b * kept + a] = s;
        }
    if (o->rr_op == 1) {
        /* generalised problem G t = lambda B t with B = E^T M E = R R^T:
         * eig of R^{-1} G R^{-T}, then t = R^{-T} v */
        double *ME = malloc(n * sizeof(double));
        double *B = malloc((size_t)kept * kept * sizeof(double));
        double *R = malloc((size_t)kept * kept * sizeof(double));
        double *H = malloc((size_t)kept * kept * sizeof(double));
        for (int b = 0; b < kept; ++b) {
            apply_M_product(o, E + (int64_t)b * n, ME);
            for (int a = 0; a < kept; ++a) B[a * kept + b] = dot(n, E + (int64_t)a * n, ME);
        }
        for (int a = 0; a < kept; ++a)
            for (int b = 0; b < a; ++b) {
                double sb = 0.5 * (B[a * kept + b] + B[b * kept + a]);
                B[a * kept + b] = B[b * kept + a] = sb;
            }
        if (cholesky(kept, B, R) != OR_OK) {
            free(ME); free(B); free(R); free(H); free(G); free(V); free(v); free(E); free(AE);
            return OR_ENUMERIC;
        }
        /* H = R^{-1} G R^{-T}: solve R X = G, then R H^T = X^T */
        for (int c2 = 0; c2 < kept; ++c2)
            for (int i = 0; i < kept; ++i) {
                double sx = G[i * kept + c2];
                for (int t = 0; t < i; ++t) sx -= R[i * kept + t] * H[t * kept + c2];
                H[i * kept + c2] = sx / R[i * kept + i];
            }
        for (int a = 0; a < kept; ++a)
            for (int b = 0; b < kept; ++b) G[a * kept + b] = H[b * kept + a]; /* G <- X^T */
        for (int c2 = 0; c2 < kept; ++c2)
            for (int i = 0; i < kept; ++i) {
                double sx = G[i * kept + c2];
                for (int t = 0; t < i; ++t) sx -= R[i * kept + t] * H[t * kept + c2];
                H[i * kept + c2] = sx / R[i * kept + i];
            }
        for (int a = 0; a < kept; ++a)
            for (int b = 0; b < a; ++b) {
                double sh = 0.5 * (H[a * kept + b] + H[b * kept + a]);
                H[a * kept + b] = H[b * kept + a] = sh;
            }
        double *Vh = malloc((size_t)kept * kept * sizeof(double));
        orc_sym_eig(kept, H, o->ritz, Vh);
        for (int j = 0; j < kept; ++j)           /* t_j = R^{-T} v_j */
            for (int i = kept - 1; i >= 0; --i) {
                double sv = Vh[i * kept + j];
                for (int t = i + 1; t < kept; ++t) sv -= R[t * kept + i] * V[t * kept + j];
                V[i * kept + j] = sv / R[i * kept + i];
            }
        free(ME); free(B); free(R); free(H); free(Vh);
    } else {
        orc_sym_eig(kept, G, o->ritz, V);
    }
    if (ritz_out) memcpy(ritz_out, o->ritz, kept * sizeof(double));
    int sel = 0;
    while (sel < kept && o->ritz[sel] < theta) ++sel;                   /* eq. (bk) */
    o->m_tilde = sel;
    *m_tilde = sel;
    o->E = E; o->AE = AE;
    if (sel == 0) { free(G); free(V); free(v); return OR_AUX_EMPTY; }
    /* W = E t_j, AW = (A E) t_j for the selected Ritz pairs */
    o->W = calloc((size_t)sel * n, sizeof(double));
    o->AW = calloc((size_t)sel * n, sizeof(double));
    for (int j = 0; j < sel; ++j)
        for (int a = 0; a < kept; ++a) {
            double t = V[a * kept + j];
            for (int64_t i = 0; i < n; ++i) {
                o->W[(int64_t)j * n + i] += t * E[(int64_t)a * n + i];
                o->AW[(int64_t)j * n + i] += t * AE[(int64_t)a * n + i];
            }
        }
    free(G); free(V); free(v);
    return finish_aux(o);
}

/* Use a caller-given W (n x k, column-major, user order). */
int orc_set_aux(orc *o, const double *W_user, int k) {
    int64_t n = o->n;
    if (k <= 0) return OR_EINVAL;
    free_aux(o);
    o->m_bar = o->m_tilde = k;
    o->W = malloc((size_t)k * n * sizeof(double));
    o->AW = malloc((size_t)k * n * sizeof(double));
    for (int j = 0; j < k; ++j) {
        to_perm(o, W_user + (int64_t)j * n, o->W + (int64_t)j * n);
        spmv(o, o->W + (int64_t)j * n, o->AW + (int64_t)j * n);
    }
    return finish_aux(o);
}

int orc_aux_dims(const orc *o, int *m_bar, int *m_tilde) {
    *m_bar = o->m_bar; *m_tilde = o->m_tilde;
    return OR_OK;
}

/* copies (user row order, column-major) of E, W, AW and C (row-major) */
void orc_get_aux(const orc *o, double *E, double *W, double *AW, double *C) {
    int64_t n = o->n;
    if (E) for (int j = 0; j < o->m_bar && o->E; ++j) from_perm(o, o->E + (int64_t)j * n, E + (int64_t)j * n);
    if (W) for (int j = 0; j < o->m_tilde; ++j) from_perm(o, o->W + (int64_t)j * n, W + (int64_t)j * n);
    if (AW) for (int j = 0; j < o->m_tilde; ++j) from_perm(o, o->AW + (int64_t)j * n, AW + (int64_t)j * n);
    if (C && o->C) memcpy(C, o->C, (size_t)o->m_tilde * o->m_tilde * sizeof(double));
}

void orc_get_ritz(const orc *o, double *ritz) { memcpy(ritz, o->ritz, o->m_bar * sizeof(double)); }

/* ------------------------------------------------------------------ */
/* kappa from the CG coefficients: Lanczos tridiagonal T_k               */
/* T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},  T_{j,j+1} = sqrt(beta_j)/alpha_j */
/* extreme eigenvalues by Sturm-sequence bisection                       */
/* ------------------------------------------------------------------ */

static int sturm_count(int k, const double *d, const double *e2, double x) {
    /* number of eigenvalues < x of the tridiagonal (d, off-diagonal^2 e2) */
    int cnt = 0;
    double q = d[0] - x;
    if (q < 0) ++cnt;
    for (int j = 1; j < k; ++j) {
        if (q == 0.0) q = 1e-300;
        q = d[j] - x - e2[j - 1] / q;
        if (q < 0) ++cnt;
    }
    return cnt;
}

int orc_lanczos_extremes(int k, const double *alpha, const double *beta, double *tmin, double *tmax) {
    /* beta[j] (0-based) is the beta that forms p_{j+2} from z_{j+1}: k-1 values */
    if (k <= 0) { *tmin = *tmax = 0.0; return OR_EINVAL; }
    double *d = malloc(k * sizeof(double)), *e2 = malloc(k * sizeof(double));
    double lo = 1e300, hi = -1e300;
    for (int j = 0; j < k; ++j) {
        d[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
        if (j < k - 1) e2[j] = beta[j] / (alpha[j] * alpha[j]);
    }
    for (int j = 0; j < k; ++j) { /* Gershgorin bounds */
        double r = 0.0;
        if (j > 0) r += sqrt(e2[j - 1]);
        if (j < k - 1) r += sqrt(e2[j]);
        if (d[j] - r < lo) lo = d[j] - r;
        if (d[j] + r > hi) hi = d[j] + r;
    }
    double a = lo, b = hi; /* smallest: count(x) >= 1 boundary */
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (a + b);
        if (mid == a || mid == b) break;
        if (sturm_count(k, d, e2, mid) >= 1) b = mid; else a = mid;
    }
    *tmin = 0.5 * (a + b);
    a = lo; b = hi; /* largest: count(x) >= k boundary */
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (a + b);
        if (mid == a || mid == b) break;
        if (sturm_count(k, d, e2, mid) >= k) b = mid; else a = mid;
    }
    *tmax = 0.5 * (a + b);
    free(d); free(e2);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* power-method start vector (user order)                               */
/* ------------------------------------------------------------------ */

void orc_set_power_start(orc *o, const double *v_user) {
    free(o->v);
    o->v = malloc(o->n * sizeof(double));
    to_perm(o, v_user, o->v);
    o->have_v = 1;
}

/* ------------------------------------------------------------------ */
/* the solvers                                                           */
/* iout: [0] iterations [1] converged [2] m_tilde used [3] samples taken */
/* dout: [0] relres (recurrence) [1] true relres [2] kappa_cg [3] kappa_es */
/*       [4] lambda_max (power) [5] lambda_min (smallest Ritz)            */
/*       [6] lanczos theta_min [7] lanczos theta_max                       */
/* ------------------------------------------------------------------ */

static void apply_M(const orc *o, int flags, const double *r, double *z) {
    if (flags & FLAG_NOPREC) memcpy(z, r, o->n * sizeof(double));
    else prec_apply(o, r, z);
}

int orc_solve(orc *o, const double *b_user, const double *x0_user, double tol, int maxit,
              int mode, int flags, double *x_user, int32_t *iout, double *dout) {
    int64_t n = o->n;
    if (!(flags & FLAG_NOPREC) && !o->factored) return OR_EINVAL;
    if (maxit < 0) return OR_EINVAL;
    if (mode != MODE_PLAIN && o->m_tilde == 0) {
        if (o->W == NULL && o->m_bar == 0) return OR_ENOAUX;
    }
    int st_aux = OR_OK;
    int eff_mode = mode;
    if (mode != MODE_PLAIN && o->m_tilde == 0) { eff_mode = MODE_PLAIN; st_aux = OR_AUX_EMPTY; }
    int k = o->m_tilde;
    double *b = malloc(n * sizeof(double)), *x = calloc(n, sizeof(double));
    double *r = malloc(n * sizeof(double)), *z = malloc(n * sizeof(double));
    double *p = malloc(n * sizeof(double)), *q = malloc(n * sizeof(double));
    double *w = malloc(n * sizeof(double)), *t = malloc(n * sizeof(double));
    double *vq = malloc(n * sizeof(double));
    double sk[4096], uk[4096];
    to_perm(o, b_user, b);
    if (x0_user) to_perm(o, x0_user, x);
    if (o->hist_cap < maxit + 1) {
        free(o->alpha); free(o->beta);
        o->hist_cap = maxit + 1;
        o->alpha = malloc(o->hist_cap * sizeof(double));
        o->beta = malloc(o->hist_cap * sizeof(double));
    }
    int sampling = (flags & FLAG_SAMPLE) && o->slots;
    if (sampling) { for (int s = 0; s < o->m_req; ++s) o->slot_iter[s] = 0; o->nsamples = 0; }
    int power = (flags & FLAG_POWER) != 0;
    if (power && !o->have_v) { free(b); free(x); free(r); free(z); free(p); free(q); free(w); free(t); free(vq); return OR_EINVAL; }

    const double bnorm2 = dot(n, b, b);
    double bnorm = sqrt(bnorm2);
    int b_next = 0; /* method B: thresholds 0 .. b_next-1 already reached */
    /* r_0 = b - A x_0 */
    spmv(o, x, t);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - t[i];
    if (eff_mode == MODE_DEFLATED) {
        /* r_0 = P^T (b - A x_0) with P^T = I - AW C^{-1} W^T */
        tmatvec(n, k, o->W, r, sk);
        coarse_solve(o, sk, uk);
        matvec_add(n, k, o->AW, uk, r, -1.0);
    }
    double rnorm = sqrt(dot(n, r, r));
    int it = 0, converged = 0, status = OR_OK;
    int64_t h = 1;
    double rho = 0.0, rho_prev = 0.0;
    if (rnorm <= tol * bnorm) converged = 1;
    while (!converged) {
        if (it >= maxit) { status = OR_NOT_CONVERGED; break; }
        ++it;
        /* z_{i-1} = M^{-1} r_{i-1}  (plus W C^{-1} W^T r for eq. (mc)) */
        apply_M(o, flags, r, z);
        if (eff_mode == MODE_SUBSPACE) {
            tmatvec(n, k, o->W, r, sk);
            coarse_solve(o, sk, uk);
            matvec_add(n, k, o->W, uk, z, 1.0);
        }
        rho = dot(n, r, z);
        if (it == 1) {
            memcpy(p, z, n * sizeof(double));
        } else {
            double beta = rho / rho_prev;
            o->beta[it - 2] = beta;
            for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        }
        /* (q v) = A (p v): the power iteration shares the product */
        spmv(o, p, q);
        if (power) {
            spmv(o, o->v, vq);
            double nv = sqrt(dot(n, vq, vq));
            for (int64_t i = 0; i < n; ++i) o->v[i] = vq[i] / nv;
        }
        double pAp;
        if (eff_mode == MODE_DEFLATED) {
            /* w = P^T A p = q - AW C^{-1} W^T q */
            memcpy(w, q, n * sizeof(double));
            tmatvec(n, k, o->W, q, sk);
            coarse_solve(o, sk, uk);
            matvec_add(n, k, o->AW, uk, w, -1.0);
            pAp = dot(n, p, w);
        } else {
            memcpy(w, q, n * sizeof(double));
            pAp = dot(n, p, q);
        }
        double alpha = rho / pAp;
        o->alpha[it - 1] = alpha;
        for (int64_t i = 0; i < n; ++i) x[i] += alpha * p[i];
        for (int64_t i = 0; i < n; ++i) r[i] -= alpha * w[i];
        rho_prev = rho;
        const double rr = dot(n, r, r);
        rnorm = sqrt(rr);
        if (!isfinite(rnorm) || !isfinite(alpha)) { status = OR_ENUMERIC; break; }
        if (rnorm <= tol * bnorm) { converged = 1; break; }
        /* sampling after the convergence check */
        int s_take = -1;
        if (sampling && o->samp_method == 0 && it % h == 0) {
            /* method A (Appendix A) */
            s_take = sample_slot(it, o->m_req);
            if (it == h * o->m_req) h *= 2;
        } else if (sampling && o->samp_method == 1) {
            /* method B (Sec. 4.3): slot s takes the iterate at which the
             * relative residual first reaches tol^{(s+1)/(m+1)}, compared in
             * squares; thresholds passed in one iteration share its sample,
             * which goes to the first of them */
            const int m = o->m_req;
            while (b_next < m && rr <= pow(tol, 2.0 * (b_next + 1) / (m + 1)) * bnorm2) {
                if (s_take < 0) s_take = b_next;
                ++b_next;
            }
        }
        if (s_take >= 0) {
            memcpy(o->slots + (int64_t)s_take * n, o->samp_resid ? r : x, n * sizeof(double));
            o->slot_iter[s_take] = it;
            if (o->nsamples < 4096) o->sample_iters[o->nsamples] = it;
            o->nsamples++;
        }
    }
    o->iters = it;
    double relres = bnorm > 0 ? rnorm / bnorm : rnorm;
    if (eff_mode == MODE_DEFLATED) {
        /* x = P x_i + W C^{-1} W^T b, with P x = x - W C^{-1} (AW)^T x */
        tmatvec(n, k, o->AW, x, sk);
        coarse_solve(o, sk, uk);
        matvec_add(n, k, o->W, uk, x, -1.0);
        tmatvec(n, k, o->W, b, sk);
        coarse_solve(o, sk, uk);
        matvec_add(n, k, o->W, uk, x, 1.0);
    }
    if (sampling) {
        free(o->xN);
        o->xN = malloc(n * sizeof(double));
        memcpy(o->xN, x, n * sizeof(double));
    }
    spmv(o, x, t);
    for (int64_t i = 0; i < n; ++i) t[i] = b[i] - t[i];
    double tres = sqrt(dot(n, t, t));
    from_perm(o, x, x_user);
    double lmin_l = 0, lmax_l = 0;
    if (it > 0) orc_lanczos_extremes(it, o->alpha, o->beta, &lmin_l, &lmax_l);
    double lam_max = 0.0;
    if (power) { spmv(o, o->v, vq); lam_max = dot(n, o->v, vq); }
    double lam_min = o->m_bar > 0 ? o->ritz[0] : 0.0;
    if (iout) {
        iout[0] = it; iout[1] = converged; iout[2] = (eff_mode == MODE_PLAIN) ? 0 : k;
        iout[3] = sampling ? o->nsamples : 0;
    }
    if (dout) {
        dout[0] = relres;
        dout[1] = bnorm > 0 ? tres / bnorm : tres;
        dout[2] = (lmin_l > 0) ? lmax_l / lmin_l : 0.0;
        dout[3] = (power && lam_min > 0) ? lam_max / lam_min : 0.0;
        dout[4] = lam_max; dout[5] = lam_min; dout[6] = lmin_l; dout[7] = lmax_l;
    }
    free(b); free(x); free(r); free(z); free(p); free(q); free(w); free(t); free(vq);
    if (status != OR_OK) return status;
    return st_aux;
}

/* alpha_1..alpha_k and beta_1..beta_{k-1} of the last solve */
int orc_history(const orc *o, double *alpha, double *beta) {
    if (alpha) memcpy(alpha, o->alpha, o->iters * sizeof(double));
    if (beta && o->iters > 1) memcpy(beta, o->beta, (o->iters - 1) * sizeof(double));
    return o->iters;
}

int orc_samples(const orc *o, int32_t *iters_by_slot) {
    if (!o->slot_iter) return 0;
    memcpy(iters_by_slot, o->slot_iter, o->m_req * sizeof(int32_t));
    return o->nsamples;
}

/* The stored sample vectors (n x m, column-major, user order; slots never
 * filled hold whatever the buffer held).  Returns m. */
int orc_slot_vectors(const orc *o, double *out_user) {
    if (!o->slots) return 0;
    for (int s = 0; s < o->m_req; ++s)
        for (int64_t l = 0; l < o->n; ++l) out_user[(int64_t)s * o->n + o->perm[l]] = o->slots[(int64_t)s * o->n + l];
    return o->m_req;
}

/* ------------------------------------------------------------------ */
/* adjoint gradient: for x = A^{-1} b and an adjoint lambda = A^{-1} g,  */
/* dL/dA_ij = -lambda_i x_j for every stored (i, j), user CSR order      */
/* ------------------------------------------------------------------ */

void orc_grad_values(const orc *o, const double *lam, const double *x, double *gval) {
    for (int64_t i = 0; i < o->n; ++i)
        for (int64_t k = o->urp[i]; k < o->urp[i + 1]; ++k) gval[k] = -lam[i] * x[o->ucol[k]];
}
