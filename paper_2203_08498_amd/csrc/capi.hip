// C ABI of the esd library: context, setup, factorisation, the solve loops
// (FP64 and FP32-inner / FP64-refinement), auxiliary-space construction and
// inspection entry points.  All per-iteration arithmetic happens in the
// kernels of kernels.hip; this file only sequences launches and reads back a
// small status block once per chunk of iterations.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/esd.h"
#include "esd_internal.h"
#include "kernels.h"

using esd::Ell;
using esd::Scal;

namespace {

struct DevEll {
    int64_t *sptr = nullptr;
    int32_t *col = nullptr;
    double *v64 = nullptr;
    float *v32 = nullptr;
    int64_t size = 0;
    // class-aligned copy for the iteration kernels (csize == 0: none)
    int64_t *csptr = nullptr;
    int32_t *soff = nullptr;
    int64_t *src = nullptr;
    double *cv64 = nullptr;
    float *cv32 = nullptr;
    int64_t csize = 0;
    Ell<double> e64() const { return {sptr, col, v64, nullptr}; }
    Ell<float> e32() const { return {sptr, col, v32, nullptr}; }
    // the layout the iteration kernels read
    Ell<double> it64() const { return csize ? Ell<double>{csptr, nullptr, cv64, soff} : e64(); }
    Ell<float> it32() const { return csize ? Ell<float>{csptr, nullptr, cv32, soff} : e32(); }
    // refresh the class-aligned values from the sorted layout
    void repack(hipStream_t s) const {
        if (csize) esd::launch_repack(csize, src, v64, cv64, cv32, s);
    }
};

template <typename T> struct VecSet {
    T *x, *r, *z, *zsc, *y, *q, *p[2], *v[2];
    const T *W, *AW, *Wrm, *AWrm, *dinv, *lsub;
    const T *Y; // M^{-1} A W (column-major), valid when the context's y_ok is set
    Ell<T> A, L, U;
};

constexpr int kFlagTiming = ESD_FLAG_TIMING | ESD_FLAG_TIMING_SPMV;

// Scratch of the allocation-free solve (esd_solve_noalloc): the device scalar
// block and the block-partial tables of one solve, in one array per GPU that
// lives as long as the process.  Host code never passes the array's name to a
// kernel: its device address on the current GPU comes from
// hipGetSymbolAddress, resolved once per device when a context is set up.
constexpr int64_t kScratchScal = 4096 / 8; // doubles reserved for the scalar block
constexpr int64_t kScratchSweep = 65536;   // sweep partial slots (one per block of every level launch)
constexpr int64_t kScratchDoubles = kScratchScal + 4 * (int64_t)esd::kPartBudget + kScratchSweep;
static_assert(sizeof(esd::Scal) <= 8 * kScratchScal, "scalar block larger than its scratch slot");

} // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
hipError_t scratch_for_current_device(double **out) {
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<double *>(g_scratch_ptr[dev]);
    return hipSuccess;
}
} // namespace

struct esd_ctx {
    hipStream_t stream = nullptr;
    std::string err;
    int64_t n = 0, nnz = 0;
    int ncolors = 1;
    int m_max = 0;
    bool mixed = true;      // FP32 copies kept (ESD_PREC_MIXED)
    int64_t max_iters = 0;  // capacity of the alpha/beta history and sampling table
    size_t ws_used = 0;     // bytes of the caller's workspace this context occupies
    std::vector<int64_t> lvl;
    std::vector<int32_t> p2u_h, lperm_h;
    DevEll A, L, U;
    int64_t *u_from_l = nullptr;
    double *l_orig = nullptr; // a_ij of the strictly lower entries (factor input)
    int32_t *a_src = nullptr, *l_src = nullptr, *d_src = nullptr; // caller-CSR positions
    double *adiag = nullptr, *ldiag = nullptr, *dinv = nullptr;
    float *dinv32 = nullptr;
    // block-Jacobi IC(0) (bj_rows > 0): blocks of bj_rows consecutive rows,
    // sub-diagonal of every block's bidiagonal factor
    int64_t bj_rows = 0;
    int bj_nb = 0;
    double *lsub = nullptr;
    float *lsub32 = nullptr;
    int32_t *p2u = nullptr;
    int32_t *tmap = nullptr, *tmap_lvl = nullptr; // XCD-local tile orders (whole range, per level)
    std::vector<int64_t> tmap_off;                 // start of every level's order in tmap_lvl
    int64_t *urp = nullptr;
    int32_t *ucol = nullptr;
    int *bad = nullptr;
    // FP64 vectors (n + 1 entries, zero at n)
    double *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *zsc = nullptr, *y = nullptr,
           *q = nullptr, *p[2] = {nullptr, nullptr}, *t = nullptr, *v[2] = {nullptr, nullptr};
    // FP32 vectors
    float *r32 = nullptr, *z32 = nullptr, *zsc32 = nullptr, *y32 = nullptr, *q32 = nullptr,
          *p32[2] = {nullptr, nullptr}, *d32 = nullptr, *v32[2] = {nullptr, nullptr};
    double *part_spmv = nullptr, *part_upd = nullptr, *part_gen = nullptr, *part_sweep = nullptr, *part_ts = nullptr;
    int64_t sweep_cap = 0;
    Scal *S = nullptr;
    Scal *Sh = nullptr; // pinned host mirror
    // sampling
    int m_req = 0;
    bool armed = false;
    int samp_method = 0;      // 0 method A, 1 method B
    bool samp_resid = false;  // store residual vectors instead of iterates
    // method B state carried across the Krylov runs of one solve
    int b_next = 0;
    std::vector<int32_t> b_slot_iter;
    std::vector<double> b_thr2;
    double *slots = nullptr;
    int32_t *slot_table = nullptr;
    std::vector<int32_t> table_h;
    std::vector<int32_t> slot_iter;
    int nsamples = 0;
    double *xN = nullptr;
    bool have_samples = false;
    // auxiliary space
    bool aux_built = false;
    int m_bar = 0, m_tilde = 0;
    double *E = nullptr, *AE = nullptr, *W = nullptr, *AW = nullptr;
    float *W32 = nullptr, *AW32 = nullptr;
    double *Y = nullptr;     // M^{-1} A W, column-major: (AW)^T z = Y^T r inside the update launch
    float *Y32 = nullptr;
    bool y_ok = false;       // Y matches the current W, values and factor
    double *W_rm = nullptr;  // row-major copies for the tall-skinny W^T v and (AW)^T v
    float *W32_rm = nullptr;
    double *AW_rm = nullptr;
    float *AW32_rm = nullptr;
    double *Cinv = nullptr, *gram_part = nullptr, *G = nullptr, *Tm = nullptr;
    std::vector<double> Ch, ritz;
    // power iteration state
    bool have_v = false;
    double lam_last = 0.0; // lambda_max of the last solve that ran the power iteration
    int vb64 = 0, vb32 = 0;
    double vs64 = 1.0, vs32 = 1.0;
    // history of the last solve
    double *ha = nullptr, *hb = nullptr;
    std::vector<double> ha_h, hb_h;
    std::vector<std::pair<int, int>> segments; // (base, count) of every Krylov run
    // mixed precision parameters
    double inner_tol = 1e-4;
    int max_outer = 30;
    int stag_window = 50;
    // per mode (plain, deflated, SC): a mixed solve of the current operator
    // had to finish in FP64 (FP32 cannot resolve it); later mixed solves in
    // that mode with ESD_FLAG_MIXED_ADAPT start in FP64.  Cleared by new
    // values, a new factor, new mixed parameters and (deflated, SC) a new W.
    bool fp32_short[3] = {false, false, false};
    bool factored = false;
    // captured iteration chunks (replayed with hipGraphLaunch), invalidated
    // whenever a buffer they reference is reallocated or the aux space changes
    struct GraphEntry {
        uint32_t key;
        uint32_t epoch;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    uint32_t epoch = 1;
    bool use_graphs = true;
    bool class_layout = true; // class-aligned matrix copies for the iteration kernels when they fit
    bool trace = false;       // ESD_TRACE set: one stderr line per refinement step of the mixed solver
    double *scratch = nullptr; // this device's copy of the allocation-free solve's scratch (null: unavailable)
    int rr_op = 0;            // Rayleigh-Ritz operator of build_aux: 0 A, 1 M^{-1}A
    hipStream_t cap = nullptr; // private stream the chunks are captured on
    // kernel timing
    std::vector<hipEvent_t> ev;
    double t_spmv = 0, t_sweep = 0, t_upd = 0;
    int t_count = 0;
};

namespace {

#define HIPCHK(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            c->err = std::string(#expr) + ": " + hipGetErrorString(e_);                            \
            return ESD_EHIP;                                                                       \
        }                                                                                          \
    } while (0)

esd_status fail(esd_ctx *c, esd_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

// Sizes of everything a context keeps in device memory.  Computed exactly by
// esd_setup from the host layout, and as an upper bound by
// esd_workspace_bytes from n, nnz and the longest row.
struct EllSizes {
    int64_t nsl = 0;   // 64-row slices
    int64_t size = 0;  // stored slots of the sorted layout
    int64_t csize = 0; // slots of the class-aligned copy (0: none)
};
struct Sizes {
    int64_t n = 0, nnz = 0;
    EllSizes A, L, U;
    int64_t tmap = 0, tmap_lvl = 0, sweep_cap = 0;
    int m_max = 1;
    bool mixed = true;
    int64_t max_iters = 0;
};

// Hands out consecutive 256-byte aligned pieces of the workspace; with a null
// base it only adds up the bytes.
struct Carver {
    char *base = nullptr;
    size_t off = 0;
    template <typename T> void take(T **p, int64_t count) {
        off = (off + 255) & ~size_t(255);
        if (count < 1) count = 1;
        if (base) *p = reinterpret_cast<T *>(base + off);
        off += sizeof(T) * (size_t)count;
    }
};

void carve_ell(Carver &cv, DevEll &D, const EllSizes &z, bool mixed) {
    D.size = z.size;
    cv.take(&D.sptr, z.nsl + 1);
    cv.take(&D.col, z.size);
    cv.take(&D.v64, z.size);
    if (mixed) cv.take(&D.v32, z.size);
    D.csize = z.csize;
    if (z.csize) {
        cv.take(&D.csptr, z.nsl + 1);
        cv.take(&D.soff, z.csize / esd::kSlice);
        cv.take(&D.src, z.csize);
        cv.take(&D.cv64, z.csize);
        if (mixed) cv.take(&D.cv32, z.csize);
    }
}

// Every device buffer of a context, in one fixed order.  FP32 copies exist
// only in mixed-precision contexts.  Returns the bytes used.
size_t carve(esd_ctx *c, const Sizes &z, char *base) {
    Carver cv;
    cv.base = base;
    const bool mx = z.mixed;
    const int64_t n = z.n, nv = n + 64, mm = std::max(1, z.m_max);
    carve_ell(cv, c->A, z.A, mx);
    carve_ell(cv, c->L, z.L, mx);
    carve_ell(cv, c->U, z.U, mx);
    cv.take(&c->a_src, z.A.size);
    cv.take(&c->l_src, z.L.size);
    cv.take(&c->d_src, n);
    cv.take(&c->l_orig, z.L.size);
    cv.take(&c->u_from_l, z.U.size);
    cv.take(&c->adiag, nv);
    cv.take(&c->ldiag, nv);
    cv.take(&c->dinv, nv);
    cv.take(&c->lsub, nv);
    if (mx) {
        cv.take(&c->dinv32, nv);
        cv.take(&c->lsub32, nv);
    }
    cv.take(&c->p2u, nv);
    cv.take(&c->tmap, z.tmap);
    cv.take(&c->tmap_lvl, z.tmap_lvl);
    cv.take(&c->urp, n + 1);
    cv.take(&c->ucol, z.nnz);
    cv.take(&c->bad, 1);
    double **v64[] = {&c->b, &c->x, &c->r, &c->z, &c->zsc, &c->y, &c->q, &c->p[0], &c->p[1], &c->t, &c->v[0],
                      &c->v[1], &c->xN};
    for (double **p : v64) cv.take(p, nv);
    if (mx) {
        float **v32[] = {&c->r32, &c->z32, &c->zsc32, &c->y32, &c->q32, &c->p32[0], &c->p32[1], &c->d32,
                         &c->v32[0], &c->v32[1]};
        for (float **p : v32) cv.take(p, nv);
    }
    // block partials: every reducing launch keeps grid x stride within kPartBudget
    cv.take(&c->part_spmv, esd::kPartBudget);
    cv.take(&c->part_upd, esd::kPartBudget);
    cv.take(&c->part_gen, esd::kPartBudget);
    cv.take(&c->part_ts, esd::kPartBudget);
    cv.take(&c->part_sweep, z.sweep_cap);
    cv.take(&c->S, 1);
    cv.take(&c->slots, mm * n);
    cv.take(&c->E, mm * n);
    cv.take(&c->AE, mm * n);
    cv.take(&c->W, mm * n);
    cv.take(&c->AW, mm * n);
    cv.take(&c->W_rm, mm * n);
    cv.take(&c->AW_rm, mm * n);
    cv.take(&c->Y, mm * n);
    if (mx) {
        cv.take(&c->Y32, mm * n);
        cv.take(&c->W32, mm * n);
        cv.take(&c->AW32, mm * n);
        cv.take(&c->W32_rm, mm * n);
        cv.take(&c->AW32_rm, mm * n);
    }
    cv.take(&c->Cinv, 64 * 64);
    cv.take(&c->G, 64 * 64);
    cv.take(&c->Tm, 64 * 64);
    cv.take(&c->gram_part, (int64_t)esd::gram_grid((int)n) * 4096);
    cv.take(&c->ha, z.max_iters + 4);
    cv.take(&c->hb, z.max_iters + 4);
    cv.take(&c->slot_table, z.max_iters + 2);
    return (cv.off + 255) & ~size_t(255);
}

// sweep partial slots: one per block of every level launch (or of the whole
// range, or of the block-Jacobi launch)
int64_t sweep_slots(int64_t n, const std::vector<int64_t> &lvl, int bj_nb) {
    int64_t tot = 0;
    for (size_t l = 0; l + 1 < lvl.size(); ++l) tot += esd::grid_red(lvl[l + 1] - lvl[l], 1);
    int64_t cap = std::max<int64_t>(esd::grid_red(n, 1), tot);
    if (bj_nb > 0) cap = std::max<int64_t>(cap, esd::bj_grid(bj_nb));
    return cap;
}

// Host copy of the class-aligned form of an ELL layout, computed before the
// workspace is carved (csptr empty: the sorted layout serves the iterations)
struct HostClass {
    std::vector<int64_t> csptr, src;
    std::vector<int32_t> soff;
};

esd_status upload_ell(esd_ctx *c, DevEll &D, const esd::HostEll &H, const HostClass &K, bool mixed) {
    HIPCHK(hipMemcpyAsync(D.sptr, H.sptr.data(), sizeof(int64_t) * H.sptr.size(), hipMemcpyHostToDevice, c->stream));
    if (D.size) {
        HIPCHK(hipMemcpyAsync(D.col, H.col.data(), sizeof(int32_t) * D.size, hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(D.v64, H.val.data(), sizeof(double) * D.size, hipMemcpyHostToDevice, c->stream));
    }
    if (mixed) esd::launch_cast(D.size, D.v64, D.v32, c->stream);
    if (D.csize) {
        HIPCHK(hipMemcpyAsync(D.csptr, K.csptr.data(), sizeof(int64_t) * K.csptr.size(), hipMemcpyHostToDevice,
                              c->stream));
        HIPCHK(hipMemcpyAsync(D.soff, K.soff.data(), sizeof(int32_t) * K.soff.size(), hipMemcpyHostToDevice,
                              c->stream));
        HIPCHK(hipMemcpyAsync(D.src, K.src.data(), sizeof(int64_t) * K.src.size(), hipMemcpyHostToDevice,
                              c->stream));
        D.repack(c->stream);
    }
    return ESD_OK;
}


esd_status sync_read(esd_ctx *c) {
    HIPCHK(hipMemcpyAsync(c->Sh, c->S, sizeof(Scal), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return ESD_OK;
}

esd_status put_scal(esd_ctx *c) {
    HIPCHK(hipMemcpyAsync(c->S, c->Sh, sizeof(Scal), hipMemcpyHostToDevice, c->stream));
    return ESD_OK;
}

// Last-level cache of the GPU (MI355X: 256 MB of Infinity Cache).
constexpr double kLlcBytes = 256.0 * 1024 * 1024;

// Non-temporal loads for the iteration's matrices in precision T, chosen
// against the last-level cache.  When A, the two triangles and eight vectors
// (plus `keep` bytes more that the iteration reads twice) outgrow it, the
// triangles stream (non-temporal loads), so that A and the vectors can stay
// cached from one iteration to the next; when A and the vectors alone
// outgrow it, A streams too.  Streamed data no longer evicts the gathered
// vectors and those the next launch reads.  The scan block-Jacobi iteration
// reads no triangle: its factor is two of the eight vectors.  Measured at
// 128^3 in FP64 (A and the vectors cached, triangles streamed, against all
// three streamed): plain iteration 127.9 -> 123.6 us, deflated 165.5 ->
// 160.7 us; the subspace correction, whose W is read twice, keeps A
// streamed (176.2 us with A cached against 168.8 us).
template <typename T> void stream_policy(const esd_ctx *c, double keep, int &a_nt, int &tri_nt) {
    auto slots = [](const DevEll &e) { return (double)(e.csize ? e.csize : e.size); };
    const double vec = 8.0 * (double)c->n * sizeof(T) + keep;
    const double a = slots(c->A) * sizeof(T);
    const double tri = c->bj_rows > 0 ? 0.0 : (slots(c->L) + slots(c->U)) * sizeof(T);
    tri_nt = a + tri + vec > kLlcBytes ? 1 : 0;
    a_nt = a + vec > kLlcBytes ? 1 : 0;
}

template <typename T> VecSet<T> vecs(esd_ctx *c);
template <> VecSet<double> vecs<double>(esd_ctx *c) {
    VecSet<double> V;
    V.x = c->x; V.r = c->r; V.z = c->z; V.zsc = c->zsc; V.y = c->y; V.q = c->q;
    V.p[0] = c->p[0]; V.p[1] = c->p[1]; V.v[0] = c->v[0]; V.v[1] = c->v[1];
    V.W = c->W; V.AW = c->AW; V.Wrm = c->W_rm; V.AWrm = c->AW_rm; V.dinv = c->dinv; V.lsub = c->lsub;
    V.Y = c->Y;
    V.A = c->A.it64(); V.L = c->L.it64(); V.U = c->U.it64();
    stream_policy<double>(c, 0.0, V.A.nt, V.L.nt);
    V.U.nt = V.L.nt;
    return V;
}
template <> VecSet<float> vecs<float>(esd_ctx *c) {
    VecSet<float> V;
    V.x = c->d32; V.r = c->r32; V.z = c->z32; V.zsc = c->zsc32; V.y = c->y32; V.q = c->q32;
    V.p[0] = c->p32[0]; V.p[1] = c->p32[1]; V.v[0] = c->v32[0]; V.v[1] = c->v32[1];
    V.W = c->W32; V.AW = c->AW32; V.Wrm = c->W32_rm; V.AWrm = c->AW32_rm; V.dinv = c->dinv32; V.lsub = c->lsub32;
    V.Y = c->Y32;
    V.A = c->A.it32(); V.L = c->L.it32(); V.U = c->U.it32();
    stream_policy<float>(c, 0.0, V.A.nt, V.L.nt);
    V.U.nt = V.L.nt;
    return V;
}

// One application of the preconditioner (all sweep launches, or the one
// block-Jacobi launch).  With sc the coarse term W u is added into zsc.
// rho partials, one per block: without subspace correction rho = (r, z) =
// ||L^{-1} r||^2, so the forward launches write ||y||^2; with it, the
// launches that finish rows of z write (r, z + W u).  Returns the number of
// partial slots.
template <typename T>
int launch_prec(esd_ctx *c, const VecSet<T> &V, bool noprec, bool sc, bool skip_l0 = false, bool skip_bwd0 = false) {
    esd::Sweep<T> s{};
    s.n = (int)c->n;
    s.S = c->S;
    s.dinv = V.dinv;
    s.r = V.r;
    s.y = V.y;
    s.z = V.z;
    s.zsc = sc ? V.zsc : V.z;
    s.W = V.W;
    s.m = sc ? c->m_tilde : 0;
    if (noprec) {
        s.r0 = 0; s.r1 = (int)c->n;
        s.tmap = c->tmap;
        s.part = c->part_sweep;
        const int g = esd::grid_red(c->n, 1);
        esd::launch_copyz(s, sc, g, c->stream);
        return g;
    }
    if (c->bj_rows > 0) {
        esd::BjSweep<T> bj{};
        bj.n = (int)c->n; bj.s = (int)c->bj_rows; bj.nb = c->bj_nb;
        bj.S = c->S; bj.part = c->part_sweep;
        bj.lsub = V.lsub; bj.dinv = V.dinv; bj.r = V.r; bj.z = V.z; bj.zsc = sc ? V.zsc : V.z;
        bj.W = V.W; bj.m = sc ? c->m_tilde : 0;
        return esd::launch_bj(bj, sc, c->stream);
    }
    // rho partial rows: every forward launch (||y||^2) without subspace
    // correction; the last forward and every backward launch with it
    int off = 0;
    const int nl = (int)c->lvl.size() - 1;
    s.M = V.L;
    for (int l = (skip_l0 && nl >= 2) ? 1 : 0; l < nl; ++l) {
        s.r0 = (int)c->lvl[l]; s.r1 = (int)c->lvl[l + 1];
        s.tmap = c->tmap_lvl + c->tmap_off[l];
        const bool last = (l == nl - 1);
        const bool pair = !last && esd::sweep_pairs(s.r1 - s.r0);
        const int g = esd::grid_red(pair ? (s.r1 - s.r0 + 1) / 2 : s.r1 - s.r0, 1);
        s.part = c->part_sweep + off;
        if (pair) esd::launch_fwd2(s, sc, g, c->stream);
        else esd::launch_fwd(s, last, sc, g, c->stream);
        if (last || !sc) off += g;
    }
    s.M = V.U;
    // skip_bwd0 (no subspace correction): the first level's backward step is
    // left to the projection launch (launch_bwd0_proj)
    for (int l = nl - 2; l >= ((skip_bwd0 && !sc && nl >= 2) ? 1 : 0); --l) {
        s.r0 = (int)c->lvl[l]; s.r1 = (int)c->lvl[l + 1];
        s.tmap = c->tmap_lvl + c->tmap_off[l];
        const bool pair = esd::sweep_pairs(s.r1 - s.r0);
        const int g = esd::grid_red(pair ? (s.r1 - s.r0 + 1) / 2 : s.r1 - s.r0, 1);
        s.part = c->part_sweep + off;
        if (pair) esd::launch_bwd2(s, sc, g, c->stream);
        else esd::launch_bwd(s, sc, g, c->stream);
        if (sc) off += g;
    }
    return off;
}

esd::FinGen fin_gen(esd_ctx *c, int nblk, int stride, int ncol) {
    esd::FinGen f{};
    f.S = c->S;
    f.part = c->part_gen;
    f.nblk = nblk;
    f.stride = stride;
    f.ncol = ncol;
    f.scale0 = 1.0;
    f.settol = -1.0;
    f.cscale = 1.0;
    return f;
}

// ||v||^2 -> *out (device)
void dev_norm2(esd_ctx *c, const double *v, double *out) {
    int nb = 0;
    esd::launch_dot((int)c->n, v, v, c->part_gen, &nb, c->stream);
    esd::FinGen f = fin_gen(c, nb, 1, 1);
    f.out0 = out;
    esd::launch_fin_gen(f, c->stream);
}

// t = b - A x; optionally coef = C^{-1} W^T t (m columns), *out = ||t||^2,
// stop check against S->tol2
void dev_resid(esd_ctx *c, const double *b, const double *x, double *t, const double *W, int m, double *coef,
               double *out, int check) {
    int nb = 0, st = 0;
    esd::launch_resid((int)c->n, c->A.e64(), b, x, t, W, W ? m : 0, c->part_gen, &nb, &st, c->stream);
    esd::FinGen f = fin_gen(c, nb, st, 1 + (W ? m : 0));
    f.out0 = out;
    f.check = check;
    if (W && m > 0) {
        f.vcol0 = 1;
        f.m = m;
        f.Cinv = c->Cinv;
        f.coef = coef;
    }
    esd::launch_fin_gen(f, c->stream);
}

// y += sign * M coef; optional *out = ||y||^2 and stop check
void dev_axpy(esd_ctx *c, double *y, const double *M, int m, const double *coef, double sign, double *out,
              int check) {
    const bool red = out || check;
    int nb = 0;
    esd::launch_axpy_cols((int)c->n, y, M, m, coef, sign, red ? c->part_gen : nullptr, &nb, c->stream);
    if (red) {
        esd::FinGen f = fin_gen(c, nb, 1, 1);
        f.out0 = out;
        f.check = check;
        esd::launch_fin_gen(f, c->stream);
    }
}

// S->svec = W^T v (m columns); optionally coef = cscale C^{-1} W^T v
void dev_tsdot(esd_ctx *c, const double *W, int m, const double *v, double *coef, double cscale) {
    int nb = 0, st = 0;
    esd::launch_tsdot((int)c->n, W, m, v, c->part_gen, &nb, &st, c->stream);
    esd::FinGen f = fin_gen(c, nb, st, m);
    f.vcol0 = 0;
    f.m = m;
    f.store_svec = 1;
    f.Cinv = c->Cinv;
    f.coef = coef;
    f.cscale = cscale;
    esd::launch_fin_gen(f, c->stream);
}

struct KrylovOpts {
    int kind = 0;        // 0 plain, 1 deflated, 2 subspace correction
    bool noprec = false;
    bool power = false;
    bool sampling = false;
    bool sync_every = false;
    bool stream_only = false;
    bool timing = false;
    bool timing_all = false;
    const double *xbase = nullptr; // mixed inner solves sample xbase + S.xscale * iterate
    bool resid = false;    // sampling stores residuals (no xbase)
    bool method_b = false; // sampling method B: slots chosen on the device
    // continue a run whose residual the caller replaced: S keeps iter, rho and
    // beta of that run, its last direction is in p[0]
    bool resume = false;
};

// Runs the CG loop from the state prepared by the caller (x, r, S with
// tol2/maxit/done set; u = C^{-1} W^T r for subspace correction).  Returns the
// number of iterations completed by this call through *iters and the exit
// code in Sh->done.
//
// Deflation iterates with projected directions: after the preconditioner,
// zhat = P z = z - W C^{-1} (AW)^T z and p = zhat + beta p in one pass, then
// q = A p; so
// (p, q) = (p, P^T A p) without cancellation and r -= alpha q is the deflated
// residual update of the deflated PCG (P^T A = A P for symmetric A).  The
// range(W) part of x is fixed by the final correction.
template <typename T>
esd_status krylov(esd_ctx *c, const VecSet<T> &V0, const KrylovOpts &o, int *iters, int *vbase) {
    const int n = (int)c->n;
    const int m = (o.kind != 0) ? c->m_tilde : 0;
    const bool sc = (o.kind == 2), defl = (o.kind == 1);
    VecSet<T> V = V0;
    if (sc && m > 0) {
        // the subspace correction reads W twice per iteration (W^T r in the
        // update, W u in the sweep): it counts against the cache with A
        stream_policy<T>(c, (double)m * n * sizeof(T), V.A.nt, V.L.nt);
        V.U.nt = V.L.nt;
    }
    const int gt = m > 0 ? esd::tsdot_grid(n, m) : 1;
    const int st_t = m > 0 ? esd::tsdot_stride(m) : 1;
    const int gn = esd::stream_grid<T>(n);
    // tall-skinny (AW)^T z (deflation) or W^T r (subspace correction)
    esd::TsDot<T> ta{};
    ta.n = n; ta.m = m; ta.Wrm = defl ? V.AWrm : V.Wrm; ta.v = defl ? V.z : V.r; ta.part = c->part_ts; ta.S = c->S;
    esd::Proj<T> pa{};
    pa.n = n; pa.m = m; pa.S = c->S; pa.z = V.z; pa.W = V.W; pa.tmap = c->tmap;
    // the first level's backward step inside the projection launch (see fuse_bp)
    esd::Sweep<T> b0{};
    b0.n = n; b0.S = c->S; b0.M = V.U; b0.dinv = V.dinv; b0.y = V.y; b0.z = V.z; b0.r = V.r; b0.zsc = V.z;
    b0.r0 = 0; b0.r1 = c->lvl.size() > 1 ? (int)c->lvl[1] : 0;
    // z_0 = M^{-1} r_0 (+ W u), rho_0 (and p_0 = zhat_0 for deflation)
    {
        const int ns = launch_prec<T>(c, V, o.noprec, sc);
        if (defl) esd::launch_tsdot_rm(ta, gt, c->stream);
        esd::FinRho fr{};
        fr.S = c->S; fr.part_sweep = c->part_sweep; fr.nsweep = ns; fr.init = o.resume ? 2 : 1;
        fr.hist_beta = o.resume ? c->hb : nullptr;
        fr.part_s = c->part_ts; fr.nblk_s = gt; fr.stride_s = st_t; fr.m = defl ? m : 0; fr.Cinv = c->Cinv;
        esd::launch_fin_rho(fr, c->stream);
        if (defl) {
            pa.pold = V.p[0];
            pa.pnew = V.p[1];
            esd::launch_proj(pa, gn, c->stream);
        }
    }
    const int sstride = esd::spmv_stride(o.power);
    const int gs = esd::grid_red(n, sstride);
    const int nl = (int)c->lvl.size() - 1;
    const bool fuse_l0 = !o.noprec && nl >= 2;
    // block Jacobi without subspace correction: the update kernel also applies
    // the preconditioner to the new residual
    const bool bj_fused = c->bj_rows > 0 && !o.noprec && !sc;
    // G^T r_{i+1} inside the update launch (m <= 16, not with the fused
    // block-Jacobi update): the subspace correction's W^T r with G = W, and
    // the deflation's (AW)^T z = (AW)^T M^{-1} r = (M^{-1} A W)^T r with
    // G = Y = M^{-1} A W (G = AW without a preconditioner); otherwise a
    // separate tall-skinny pass over r (W) or z (AW) after the update
    const T *G = nullptr;
    if (m > 0 && m <= 16 && !bj_fused) {
        if (sc) G = V.W;
        else if (defl) G = o.noprec ? V.AW : (c->y_ok ? V.Y : nullptr);
    }
    const int su = esd::update_stride(G ? m : 0); // partial columns of the update launch
    // deflation with Y^T r in the update: rho and mu are known once the
    // forward sweep is done, so the rho finalize runs before the first
    // level's backward step, which the projection launch then takes over
    // (one launch fewer: 128^3 FP64 deflated iteration 156.6 -> 153.4 us,
    // FP32 with two rows per thread 103.8 -> 101.1 us; Q1 FP64 730.7 ->
    // 726.9 us).  A first level of more than kPairTiles tiles keeps
    // its two-row backward launch (256^3: 1687 against 1703 us fused);
    // stream launches with per-launch timing keep the separate form, so that
    // the timed sweeps are the whole pair.
    const bool fuse_bp = defl && G != nullptr && !bj_fused && !o.noprec && nl >= 2 && !o.timing_all &&
                         !esd::sweep_pairs(c->lvl[1]);
    // update launches and their partial rows.  With G^T r the one-block
    // finalize reads 2 + m columns per block, so the grid gives each block
    // about eight tiles, 1024 to 2048 blocks (128^3: 1024 blocks, FP64
    // deflated iteration 161.1 -> 159.2 us, FP32 111.6 -> 107.3 us; on Q1
    // 2000 blocks, where 1024 cost 1 us)
    const int tiles8 = ((n + esd::kBlock - 1) / esd::kBlock / 8 + 7) / 8 * 8;
    const int gu = G ? std::min(esd::stream_grid<T>(n), std::min(2048, std::max(1024, tiles8)))
                     : esd::stream_grid<T>(n);
    esd::UpdBj<T> ub{};
    ub.n = n; ub.s = (int)c->bj_rows; ub.nb = c->bj_nb; ub.S = c->S; ub.part = c->part_upd;
    ub.q = V.q; ub.x = V.x; ub.r = V.r; ub.lsub = V.lsub; ub.dinv = V.dinv; ub.z = V.z;
    esd::SpmvIt<T> sa{};
    sa.n = n; sa.S = c->S; sa.part = c->part_spmv; sa.A = V.A; sa.tmap = c->tmap;
    sa.z = defl ? nullptr : (sc ? V.zsc : V.z); // deflation: p_new given by the projection
    sa.slot_table = o.sampling ? c->slot_table : nullptr;
    sa.slots = c->slots;
    sa.xit = o.resid ? V.r : V.x;
    sa.xbase = o.resid ? nullptr : o.xbase;
    sa.q = V.q;
    esd::FinAlpha fa{};
    fa.S = c->S; fa.part = c->part_spmv; fa.nblk = gs; fa.stride = sstride; fa.power = o.power;
    fa.hist_alpha = c->ha;
    esd::UpdIt<T> ua{};
    ua.n = n; ua.S = c->S; ua.part = c->part_upd; ua.q = V.q; ua.x = V.x; ua.r = V.r; ua.tmap = c->tmap;
    ua.l0 = fuse_l0 ? (int)c->lvl[1] : 0; ua.dinv = V.dinv; ua.y = V.y;
    ua.G = G; ua.m = G ? m : 0;
    ua.xnt = V.L.nt; // x (touched once per iteration) streams whenever the working set outgrows the cache
    ua.gnt = defl ? 1 : 0; // Y is read only here; the subspace correction's W again by the sweep
    esd::FinRho fr{};
    fr.S = c->S; fr.part_upd = c->part_upd; fr.nblk_upd = gu; fr.stride_upd = su;
    fr.rho_upd = (fuse_l0 && !sc) ? 1 : 0;
    if (bj_fused) {
        fr.nblk_upd = esd::bj_grid(c->bj_nb);
        fr.rho_upd = 1;
        fr.nsweep = 0;
    }
    fr.part_sweep = c->part_sweep; fr.hist_beta = c->hb; fr.init = 0;
    fr.part_s = c->part_ts; fr.nblk_s = gt; fr.stride_s = st_t; fr.c0_s = 0; fr.m = defl ? m : 0; fr.Cinv = c->Cinv;
    if (defl && G) {
        // (AW)^T z_{i+1} = Y^T r_{i+1}: columns 2 .. of the update partials
        fr.part_s = c->part_upd; fr.nblk_s = gu; fr.stride_s = su; fr.c0_s = 2;
    }
    if (o.sampling && o.method_b) {
        fr.slot_table = c->slot_table;
        fr.nslots = c->m_req;
    }
    const bool timing = o.timing;
    // one chunk of iterations; `it0` must be even so that a replay of the
    // chunk reuses the same ping-pong buffers
    auto body = [&](int it0, int count) -> hipError_t {
        for (int j = 0; j < count; ++j) {
            const int it = it0 + j;
            sa.pold = V.p[it & 1];
            sa.pnew = V.p[(it + 1) & 1];
            sa.vold = V.v[(*vbase + it) & 1];
            sa.vnew = V.v[(*vbase + it + 1) & 1];
            ua.p = V.p[(it + 1) & 1];
            hipError_t e;
            if (timing && (e = hipEventRecord(c->ev[4 * j + 0], c->stream)) != hipSuccess) return e;
            esd::launch_spmv_it(sa, o.power, gs, c->stream);
            if (timing && (e = hipEventRecord(c->ev[4 * j + 1], c->stream)) != hipSuccess) return e;
            esd::launch_fin_alpha(fa, c->stream);
            if (bj_fused) {
                // the "sweep" time of this variant is the fused update + preconditioner launch
                ub.p = ua.p;
                if (o.timing_all && (e = hipEventRecord(c->ev[4 * j + 2], c->stream)) != hipSuccess) return e;
                esd::launch_update_bj(ub, c->stream);
                if (o.timing_all && (e = hipEventRecord(c->ev[4 * j + 3], c->stream)) != hipSuccess) return e;
            } else {
                esd::launch_update_it(ua, gu, c->stream);
                if (sc) {
                    if (G) {
                        esd::launch_fin_u(c->S, c->part_upd, gu, su, 2, m, c->Cinv, c->stream);
                    } else {
                        esd::launch_tsdot_rm(ta, gt, c->stream);
                        esd::launch_fin_u(c->S, c->part_ts, gt, st_t, 0, m, c->Cinv, c->stream);
                    }
                }
                if (o.timing_all && (e = hipEventRecord(c->ev[4 * j + 2], c->stream)) != hipSuccess) return e;
                fr.nsweep = launch_prec<T>(c, V, o.noprec, sc, fuse_l0, fuse_bp);
                if (o.timing_all && (e = hipEventRecord(c->ev[4 * j + 3], c->stream)) != hipSuccess) return e;
            }
            if (defl && !G) esd::launch_tsdot_rm(ta, gt, c->stream);
            esd::launch_fin_rho(fr, c->stream);
            if (defl) {
                // direction of iteration it + 1
                pa.pold = V.p[(it + 1) & 1];
                pa.pnew = V.p[it & 1];
                if (fuse_bp) esd::launch_bwd0_proj(b0, pa, gn, c->stream);
                else esd::launch_proj(pa, gn, c->stream);
            }
        }
        return hipGetLastError();
    };
    const int iter0 = c->Sh->iter; // the caller's state, as put on the device
    auto harvest = [&](int launched, int chunk) {
        if (!timing) return;
        const int executed = std::min(chunk, std::max(0, c->Sh->iter - iter0 - launched));
        for (int j = 0; j < executed; ++j) {
            float a = 0, b = 0, d = 0;
            (void)hipEventElapsedTime(&a, c->ev[4 * j + 0], c->ev[4 * j + 1]);
            if (o.timing_all) {
                (void)hipEventElapsedTime(&b, c->ev[4 * j + 1], c->ev[4 * j + 2]);
                (void)hipEventElapsedTime(&d, c->ev[4 * j + 2], c->ev[4 * j + 3]);
            }
            c->t_spmv += a; c->t_upd += b; c->t_sweep += d; c->t_count++;
        }
    };
    // 16-iteration chunks; once the residual's recent rate predicts the end
    // within 12 iterations, 4-iteration chunks, so that fewer launches of a
    // chunk run (and return at once) after the stop
    constexpr int kChunk = 16, kTail = 4;
    const uint32_t key0 = (sizeof(T) == 4 ? 1u : 0u) | ((uint32_t)o.kind << 1) | ((uint32_t)o.noprec << 3) |
                          ((uint32_t)o.power << 4) | ((uint32_t)o.sampling << 5) | ((uint32_t)(*vbase & 1) << 6) |
                          ((uint32_t)fuse_l0 << 7) | ((uint32_t)o.resid << 8) | ((uint32_t)o.method_b << 9) |
                          // method B's finalize takes the slot count as an argument
                          ((uint32_t)((o.sampling && o.method_b) ? c->m_req : 0) << 11) |
                          ((uint32_t)(G != nullptr) << 18);
    // the cached graph of `count` iterations of this variant (nullptr: the
    // variant does not capture, stream launches for it)
    auto graph_for = [&](int count) -> hipGraphExec_t {
        const uint32_t key = key0 | ((uint32_t)(count == kTail) << 10);
        for (auto &g : c->graphs)
            if (g.key == key && g.epoch == c->epoch) return g.exec;
        if (!c->cap && hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
            c->cap = nullptr;
            c->use_graphs = false;
            return nullptr;
        }
        // capture on the private stream (the caller's may be the null
        // stream, which cannot be captured); replays go to the caller's
        hipGraphExec_t ex = nullptr;
        hipGraph_t graph = nullptr;
        hipStream_t user = c->stream;
        c->stream = c->cap;
        bool ok = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed) == hipSuccess;
        if (ok) {
            const hipError_t eb = body(0, count);
            const hipError_t ee = hipStreamEndCapture(c->stream, &graph);
            ok = eb == hipSuccess && ee == hipSuccess && graph;
        }
        c->stream = user;
        if (ok) ok = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        if (!ok) ex = nullptr;
        for (auto it = c->graphs.begin(); it != c->graphs.end();)
            if (it->key == key) {
                if (it->exec) (void)hipGraphExecDestroy(it->exec);
                it = c->graphs.erase(it);
            } else {
                ++it;
            }
        c->graphs.push_back({key, c->epoch, ex});
        return ex;
    };
    // kernel timing reads hipEvents recorded between stream launches (events
    // recorded as graph nodes give no elapsed time): timing solves stay off graphs
    hipGraphExec_t ex = nullptr;
    if (c->use_graphs && !o.sync_every && !o.stream_only && !timing) ex = graph_for(kChunk);
    int launched = 0;
    if (ex) {
        hipGraphExec_t tail = nullptr;
        bool tail_tried = false;
        int chunk = kChunk;
        double rr_prev = -1.0;
        for (;;) {
            HIPCHK(hipGraphLaunch(chunk == kChunk ? ex : tail, c->stream));
            esd_status st = sync_read(c);
            if (st != ESD_OK) return st;
            harvest(launched, chunk);
            launched += chunk;
            if (c->Sh->done) break;
            if (chunk == kChunk) {
                const double rr = c->Sh->rr, t2 = c->Sh->tol2;
                if (rr_prev > 0.0 && rr > t2 && rr < rr_prev) {
                    const double need = std::log(t2 / rr) / (std::log(rr / rr_prev) / kChunk);
                    if (need < 12.0) {
                        if (!tail_tried) {
                            tail = graph_for(kTail);
                            tail_tried = true;
                        }
                        if (tail) chunk = kTail;
                    }
                }
                rr_prev = rr;
            }
        }
    } else {
        int chunk = o.sync_every ? 1 : 8;
        for (;;) {
            HIPCHK(body(launched, chunk));
            esd_status st = sync_read(c);
            if (st != ESD_OK) return st;
            harvest(launched, chunk);
            launched += chunk;
            if (c->Sh->done) break;
            if (!o.sync_every && chunk < 32) chunk *= 2;
        }
    }
    *iters = c->Sh->iter - iter0;
    // the power iterate alternates between v[0] and v[1] only in runs that
    // carry it: a run without it must not move the next power run's start
    // to the other (possibly never written) buffer
    if (o.power) *vbase = (*vbase + *iters) & 1;
    return ESD_OK;
}

void init_scal(esd_ctx *c, int maxit, double vscale, int stag) {
    Scal &S = *c->Sh;
    std::memset(&S, 0, sizeof(Scal));
    S.maxit = maxit;
    S.done = (maxit <= 0) ? 2 : 0; // no iteration allowed: stop before the first one
    S.vscale = vscale;
    S.stag_window = stag;
    S.rr_ref = 1e300;
    S.rho = 1.0;
    S.xscale = 1.0;
}

void fill_lanczos(esd_ctx *c, esd_info *info) {
    double lo = 0, hi = 0;
    bool any = false;
    for (auto &sg : c->segments) {
        if (sg.second <= 0) continue;
        double a = 0, b = 0;
        esd::tridiag_extremes(sg.second, c->ha_h.data() + sg.first, c->hb_h.data() + sg.first, &a, &b);
        if (!any) { lo = a; hi = b; any = true; }
        else { lo = std::min(lo, a); hi = std::max(hi, b); }
    }
    info->lanczos_min = lo;
    info->lanczos_max = hi;
    info->kappa = (any && lo > 0) ? hi / lo : 0.0;
}

esd_status read_history(esd_ctx *c, int total) {
    c->ha_h.assign(std::max(total, 1), 0.0);
    c->hb_h.assign(std::max(total, 1), 0.0);
    if (total > 0) {
        HIPCHK(hipMemcpyAsync(c->ha_h.data(), c->ha, sizeof(double) * total, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipMemcpyAsync(c->hb_h.data(), c->hb, sizeof(double) * total, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
    }
    return ESD_OK;
}

esd_status ensure_tables(esd_ctx *c, int maxit, bool events) {
    // the alpha/beta history and the sampling table live in the workspace,
    // sized by the context's max_iters
    if ((int64_t)maxit > c->max_iters)
        return fail(c, ESD_EINVAL, "maxit exceeds the max_iters the workspace was sized for");
    if (c->armed) {
        if (c->samp_method == 0) esd::sampling_table(c->m_req, (int64_t)maxit + 2, c->table_h);
        else c->table_h.assign((size_t)maxit + 2, -1); // method B: slots set on the device
        HIPCHK(hipMemcpyAsync(c->slot_table, c->table_h.data(), sizeof(int32_t) * c->table_h.size(),
                              hipMemcpyHostToDevice, c->stream));
    }
    if (!events || (int)c->ev.size() >= 4 * 32) return ESD_OK;
    c->ev.resize(4 * 32);
    // timing-only markers: no system-scope fence (no L2 writeback) at each
    // record, so a pair brackets the kernel rather than the kernel plus a flush
    for (auto &e : c->ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    return ESD_OK;
}

// iterations kept in every slot for a sampling solve that ran `iters`
// iterations (`last_sampled`: the solve stopped at maxit, so its last iterate
// was sampled too)
void record_samples(esd_ctx *c, int iters, bool last_sampled) {
    c->slot_iter.assign(c->m_req, 0);
    c->nsamples = 0;
    if (c->samp_method == 1) {
        for (int s = 0; s < c->m_req; ++s)
            if (c->b_slot_iter[s] > 0 && (c->b_slot_iter[s] < iters || last_sampled)) {
                c->slot_iter[s] = c->b_slot_iter[s];
                c->nsamples++;
            }
        c->have_samples = c->nsamples > 0;
        return;
    }
    const int upto = last_sampled ? iters : iters - 1;
    for (int i = 1; i <= upto && i < (int)c->table_h.size(); ++i)
        if (c->table_h[i] >= 0) {
            c->slot_iter[c->table_h[i]] = i;
            c->nsamples++;
        }
    c->have_samples = c->nsamples > 0;
}

// The class-aligned layout gathers an arbitrary in-range element for the
// empty slots of a row (multiplied by zero): the sweep outputs must hold finite
// values before their rows are written, whatever an earlier solve left there.
void clear_sweep_vectors(esd_ctx *c) {
    const int nv = (int)c->n + 64;
    esd::launch_fill(nv, c->y, 0.0, c->stream);
    esd::launch_fill(nv, c->z, 0.0, c->stream);
    esd::launch_fill(nv, c->zsc, 0.0, c->stream);
    if (!c->mixed) return;
    esd::launch_fill(nv, c->y32, 0.0f, c->stream);
    esd::launch_fill(nv, c->z32, 0.0f, c->stream);
    esd::launch_fill(nv, c->zsc32, 0.0f, c->stream);
}

// Sampling method B state lives in the device scalar block during a Krylov
// run and on the host between runs (init_scal clears the block).
void arm_method_b(esd_ctx *c, double tol) {
    c->b_next = 0;
    c->b_slot_iter.assign(64, 0);
    c->b_thr2.assign(64, 0.0);
    for (int s = 0; s < c->m_req; ++s) c->b_thr2[s] = std::pow(tol, 2.0 * (s + 1) / (c->m_req + 1));
}
void put_method_b(esd_ctx *c) {
    Scal &S = *c->Sh;
    S.smethod = 1;
    S.bnext = c->b_next;
    for (int s = 0; s < 64; ++s) {
        S.slot_iter[s] = c->b_slot_iter[s];
        S.bthr2[s] = c->b_thr2[s];
    }
}
void get_method_b(esd_ctx *c) {
    const Scal &S = *c->Sh;
    c->b_next = S.bnext;
    for (int s = 0; s < 64; ++s) c->b_slot_iter[s] = S.slot_iter[s];
}

esd_status solve_fp64(esd_ctx *c, const double *b, const double *x0, double tol, int maxit, int kind,
                      int flags, double *xout, esd_info *info) {
    const int n = (int)c->n;
    int m = kind ? c->m_tilde : 0;
    const bool sampling = c->armed;
    const bool power = (flags & ESD_FLAG_POWER) != 0;
    const bool restart = (flags & ESD_FLAG_TRUE_RES) != 0;
    const int kind_in = kind;
    auto V = vecs<double>(c);
    clear_sweep_vectors(c);
    esd::launch_gather(n, c->p2u, b, c->b, c->stream);
    if (x0) esd::launch_gather(n, c->p2u, x0, c->x, c->stream);
    else esd::launch_fill(n, c->x, 0.0, c->stream);
    init_scal(c, maxit, c->vs64, 0);
    esd_status st = put_scal(c);
    if (st) return st;
    {
        int nb = 0;
        esd::launch_dot(n, c->b, c->b, c->part_gen, &nb, c->stream);
        esd::FinGen f = fin_gen(c, nb, 1, 1);
        f.settol = tol;
        esd::launch_fin_gen(f, c->stream);
    }
    st = sync_read(c);
    if (st) return st;
    const double bn2 = c->Sh->bnorm2, tol2 = c->Sh->tol2;
    c->segments.clear();
    const bool method_b = sampling && c->samp_method == 1;
    if (method_b) arm_method_b(c, tol);
    int total = 0, done = 0, cycles = 0;
    double rr = 0.0, tr2 = 0.0, tr2_prev = -1.0;
    for (;;) {
        // r_0 = b - A x_0; deflation: r_0 = P^T r_0 = r_0 - AW C^{-1} W^T r_0;
        // subspace correction: u = C^{-1} W^T r_0 for z_0
        init_scal(c, maxit - total, c->vs64, 0);
        c->Sh->bnorm2 = bn2;
        c->Sh->tol2 = tol2;
        c->Sh->hist_base = total;
        c->Sh->sample_base = total;
        if (method_b && cycles == 0) put_method_b(c);
        if ((st = put_scal(c))) return st;
        double *coef = (kind == 1) ? c->S->mu : (kind == 2 ? c->S->u : nullptr);
        dev_resid(c, c->b, c->x, c->r, m ? c->W : nullptr, m, coef, nullptr, kind != 1);
        if (kind == 1) dev_axpy(c, c->r, c->AW, m, c->S->mu, -1.0, nullptr, 1);
        KrylovOpts o;
        o.kind = kind;
        o.noprec = (flags & ESD_FLAG_NOPREC) != 0;
        o.power = power;
        o.sampling = sampling && cycles == 0;
        o.resid = c->samp_resid;
        o.method_b = method_b;
        o.sync_every = (flags & ESD_FLAG_SYNC_EVERY) != 0;
        o.stream_only = (flags & ESD_FLAG_STREAM) != 0;
        o.timing = (flags & kFlagTiming) != 0;
        o.timing_all = (flags & ESD_FLAG_TIMING) != 0;
        int iters = 0;
        st = krylov<double>(c, V, o, &iters, &c->vb64);
        if (st) return st;
        done = c->Sh->done;
        rr = c->Sh->rr;
        if (power) c->vs64 = c->Sh->vscale;
        c->segments.push_back({total, iters});
        if (o.sampling) {
            // a solve stopped by maxit: its last vector has no next SpMV to store it
            double *last = c->samp_resid ? c->r : c->x;
            if (method_b) {
                get_method_b(c);
                for (int sl = 0; sl < c->m_req; ++sl)
                    if (done == 2 && c->b_slot_iter[sl] == iters)
                        esd::launch_sample_store(n, c->slots + (size_t)sl * n, last, c->stream);
            } else if (done == 2 && iters < (int)c->table_h.size() && c->table_h[iters] >= 0) {
                esd::launch_sample_store(n, c->slots + (size_t)c->table_h[iters] * n, last, c->stream);
            }
            record_samples(c, iters, done == 2);
        }
        total += iters;
        if (kind == 1) {
            // x = P x_i + W C^{-1} W^T b  ==  x_i + W C^{-1} W^T (b - A x_i)
            dev_resid(c, c->b, c->x, c->t, c->W, m, c->S->mu, nullptr, 0);
            dev_axpy(c, c->x, c->W, m, c->S->mu, 1.0, nullptr, 0);
        }
        dev_resid(c, c->b, c->x, c->t, nullptr, 0, nullptr, &c->S->out, 0);
        if ((st = sync_read(c))) return st;
        tr2 = c->Sh->out;
        ++cycles;
        // optional: restart from x while the recomputed residual misses the tolerance
        if (!restart || done != 1 || tr2 <= tol2 || cycles > 4 || total >= maxit) break;
        // a deflated restart that did not halve the recomputed residual stops
        // deflating: what is left is the rounding of the projection and the
        // coarse correction, which plain PCG from this x removes in a few
        // iterations (Q1 160^3 with 20 columns of W: one iteration from
        // relres 3.3e-7 to 4.5e-8, where deflated restarts stayed at 2e-7)
        if (kind == 1 && tr2_prev >= 0.0 && tr2 > 0.25 * tr2_prev) {
            kind = 0;
            m = 0;
        }
        tr2_prev = tr2;
    }
    if (power) {
        int nb = 0;
        esd::launch_rayleigh(n, c->A.e64(), c->v[c->vb64], c->part_gen, &nb, c->stream);
        esd::FinGen f = fin_gen(c, nb, 1, 1);
        f.out0 = &c->S->lam;
        f.scale0 = c->vs64 * c->vs64;
        esd::launch_fin_gen(f, c->stream);
    }
    esd::launch_scatter(n, c->p2u, c->x, xout, c->stream);
    if (sampling) {
        HIPCHK(hipMemcpyAsync(c->xN, c->x, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
        c->armed = false;
    }
    st = sync_read(c);
    if (st) return st;
    st = read_history(c, total);
    if (st) return st;
    if (info) {
        info->iters = total;
        info->outer_iters = cycles;
        info->converged = (done == 1) && (!restart || tr2 <= tol2);
        info->m_tilde = kind_in ? c->m_tilde : 0;
        info->nsamples = sampling ? c->nsamples : 0;
        info->mode_used = kind_in;
        info->relres = bn2 > 0 ? std::sqrt(rr / bn2) : std::sqrt(rr);
        info->true_relres = bn2 > 0 ? std::sqrt(tr2 / bn2) : std::sqrt(tr2);
        info->lambda_max = power ? c->Sh->lam : 0.0;
        fill_lanczos(c, info);
    }
    if (done == 3) return fail(c, ESD_ENUMERIC, "non-finite value in the iteration");
    const bool ok = (done == 1) && (!restart || tr2 <= tol2);
    return ok ? ESD_OK : ESD_NOT_CONVERGED;
}

esd_status solve_mixed(esd_ctx *c, const double *b, const double *x0, double tol, int maxit, int kind,
                       int flags, double *xout, esd_info *info) {
    const int n = (int)c->n;
    const int m = kind ? c->m_tilde : 0;
    const bool sampling = c->armed;
    const bool power = (flags & ESD_FLAG_POWER) != 0;
    auto V = vecs<float>(c);
    clear_sweep_vectors(c);
    esd::launch_gather(n, c->p2u, b, c->b, c->stream);
    if (x0) esd::launch_gather(n, c->p2u, x0, c->x, c->stream);
    else esd::launch_fill(n, c->x, 0.0, c->stream);
    init_scal(c, maxit, c->vs32, 0);
    esd_status st = put_scal(c);
    if (st) return st;
    {
        int nb = 0;
        esd::launch_dot(n, c->b, c->b, c->part_gen, &nb, c->stream);
        esd::FinGen f = fin_gen(c, nb, 1, 1);
        f.settol = tol;
        esd::launch_fin_gen(f, c->stream);
    }
    st = sync_read(c);
    if (st) return st;
    const double bn2 = c->Sh->bnorm2, tol2 = c->Sh->tol2;
    // ESD_FLAG_MIXED_ADAPT: a context whose earlier mixed solve in this mode
    // had to finish in FP64 starts there (its first FP64 run counts as no
    // restart)
    bool fp64 = (flags & ESD_FLAG_MIXED_ADAPT) != 0 && c->fp32_short[kind];
    int total = 0, outer = 0, done_in = 0, fp64_iters = 0, fp64_restarts = fp64 ? -1 : 0;
    bool converged = false;
    const bool method_b = sampling && c->samp_method == 1;
    if (method_b) arm_method_b(c, tol);
    double rn2 = 0.0, rn2_prev = -1.0;
    // ESD_FLAG_MIXED_KEEP: a step that follows an inner run which reached its
    // target replaces that run's residual by the new FP64 one and continues
    // it (same search direction, same scale s_in of the inner quantities)
    const bool keep = (flags & ESD_FLAG_MIXED_KEEP) != 0;
    bool can_resume = false;
    double s_in = 1.0;
    int last_in = 0;
    c->segments.clear();
    // mode of the FP64 finish: deflated restarts that stop halving the
    // recomputed residual continue as plain PCG (as in solve_fp64)
    int kind_fin = kind;
    for (outer = 0; outer <= c->max_outer; ++outer) {
        // FP64 true residual; deflation: coarse correction x += W C^{-1} W^T r
        if (kind == 1 && kind_fin == 1) {
            dev_resid(c, c->b, c->x, c->r, c->W, m, c->S->mu, nullptr, 0);
            dev_axpy(c, c->x, c->W, m, c->S->mu, 1.0, nullptr, 0);
            dev_axpy(c, c->r, c->AW, m, c->S->mu, -1.0, &c->S->out, 0);
        } else {
            dev_resid(c, c->b, c->x, c->r, nullptr, 0, nullptr, &c->S->out, 0);
        }
        st = sync_read(c);
        if (st) return st;
        rn2 = c->Sh->out;
        if (c->trace)
            fprintf(stderr, "esd mixed: step %d relres %.3e after %d iterations (%d FP64), last inner exit %d\n",
                    outer, bn2 > 0 ? std::sqrt(rn2 / bn2) : std::sqrt(rn2), total, fp64_iters, done_in);
        if (!(rn2 <= 1e300)) return fail(c, ESD_ENUMERIC, "non-finite residual");
        if (rn2 <= tol2) { converged = true; break; }
        if (total >= maxit || outer == c->max_outer) break;
        // a refinement step that does not halve the residual: the FP32 inner
        // operator is too far from A (kappa * u_32 >~ 1); finish in FP64
        if (fp64) {
            // FP64 CG ran to the target on its recurrence residual and the
            // recomputed one missed it: restart from x, at most 4 times (as
            // ESD_FLAG_TRUE_RES does); a residual at the FP64 rounding floor of
            // b - A x ends the solve there, not converged
            if (++fp64_restarts > 4) break;
            if (kind_fin == 1 && fp64_restarts >= 2 && rn2 > 0.25 * rn2_prev) kind_fin = 0;
        } else if (rn2_prev >= 0.0 && (rn2 > 0.25 * rn2_prev || (done_in == 4 && rn2 > 1e-4 * rn2_prev))) {
            // ... or an inner run that stagnated before taking two orders of
            // magnitude off the residual: FP32 cannot resolve this operator
            fp64 = true;
            c->fp32_short[kind] = true;
        }
        rn2_prev = rn2;
        if (fp64) {
            auto V64 = vecs<double>(c);
            init_scal(c, maxit - total, c->vs64, 0);
            c->Sh->tol2 = tol2;
            c->Sh->bnorm2 = bn2;
            c->Sh->rr = rn2;
            c->Sh->hist_base = total;
            c->Sh->sample_base = total;
            // a sampling solve keeps sampling here: the FP64 iterate is the
            // solution itself (no base, scale 1), stored like the inner ones
            if (method_b) put_method_b(c);
            if ((st = put_scal(c))) return st;
            if (kind == 2) dev_tsdot(c, c->W, m, c->r, c->S->u, 1.0);
            KrylovOpts o;
            o.kind = kind_fin;
            o.noprec = (flags & ESD_FLAG_NOPREC) != 0;
            o.power = false;
            o.sampling = sampling;
            o.resid = c->samp_resid;
            o.method_b = method_b;
            o.sync_every = (flags & ESD_FLAG_SYNC_EVERY) != 0;
            o.stream_only = (flags & ESD_FLAG_STREAM) != 0;
            int it64 = 0;
            st = krylov<double>(c, V64, o, &it64, &c->vb64);
            if (st) return st;
            if (method_b) get_method_b(c);
            c->segments.push_back({total, it64});
            total += it64;
            fp64_iters += it64;
            if (c->Sh->done == 3) return fail(c, ESD_ENUMERIC, "non-finite value in the FP64 finish");
            if (kind_fin == 1) {
                dev_resid(c, c->b, c->x, c->t, c->W, m, c->S->mu, nullptr, 0);
                dev_axpy(c, c->x, c->W, m, c->S->mu, 1.0, nullptr, 0);
            }
            continue; // the next pass recomputes the FP64 residual and tests it
        }
        const double rn = std::sqrt(rn2);
        const bool cont = keep && can_resume;
        if (!cont) s_in = rn;
        esd::launch_cast_scale(n, c->r, c->r32, 1.0 / s_in, c->stream);
        esd::launch_fill(n, c->d32, 0.0f, c->stream);
        // inner relative target: the refinement tolerance, or just what is still missing
        const double want = std::max(c->inner_tol, 0.3 * std::sqrt(tol2) / rn);
        const double rel = rn / s_in; // ||r32||
        if (cont) {
            // the run's scalar block as the last synchronisation read it:
            // iteration count, rho, beta, history and sampling offsets stay
            Scal &S = *c->Sh;
            S.done = 0;
            S.tol2 = want * want * rel * rel;
            S.maxit = S.iter + (maxit - total);
            S.rr_ref = 1e300;
            S.it_ref = S.iter;
            // the run's last direction is in p[last_in & 1]; the next call reads it from p[0]
            if (last_in & 1)
                HIPCHK(hipMemcpyAsync(V.p[0], V.p[1], sizeof(float) * n, hipMemcpyDeviceToDevice, c->stream));
        } else {
            init_scal(c, maxit - total, c->vs32, c->stag_window);
            c->Sh->tol2 = want * want;
            c->Sh->bnorm2 = bn2;
            c->Sh->hist_base = total;
            c->Sh->sample_base = total;
            c->Sh->xscale = rn;
            if (method_b) put_method_b(c);
        }
        st = put_scal(c);
        if (st) return st;
        // u = C^{-1} W^T r / s_in for the first preconditioned inner residual
        if (kind == 2) dev_tsdot(c, c->W, m, c->r, c->S->u, 1.0 / s_in);
        KrylovOpts o;
        o.kind = kind;
        o.noprec = (flags & ESD_FLAG_NOPREC) != 0;
        o.power = power;
        o.sampling = sampling;
        o.resid = c->samp_resid;
        o.method_b = method_b;
        o.sync_every = (flags & ESD_FLAG_SYNC_EVERY) != 0;
        o.stream_only = (flags & ESD_FLAG_STREAM) != 0;
        o.timing = (flags & kFlagTiming) != 0;
        o.timing_all = (flags & ESD_FLAG_TIMING) != 0;
        o.xbase = c->x;
        o.resume = cont;
        int it_in = 0;
        st = krylov<float>(c, V, o, &it_in, &c->vb32);
        if (st) return st;
        if (method_b) get_method_b(c);
        done_in = c->Sh->done;
        if (cont) c->segments.back().second += it_in; // one Lanczos run
        else c->segments.push_back({total, it_in});
        total += it_in;
        if (power) c->vs32 = c->Sh->vscale;
        esd::launch_add_scaled(n, c->x, c->d32, s_in, c->stream);
        can_resume = done_in == 1 && it_in >= 1;
        last_in = it_in;
        if (done_in == 3) return fail(c, ESD_ENUMERIC, "non-finite value in the inner iteration");
    }
    dev_resid(c, c->b, c->x, c->t, nullptr, 0, nullptr, &c->S->out, 0);
    if (power) {
        int nb = 0;
        esd::launch_rayleigh(n, c->A.e32(), c->v32[c->vb32], c->part_gen, &nb, c->stream);
        esd::FinGen f = fin_gen(c, nb, 1, 1);
        f.out0 = &c->S->lam;
        f.scale0 = c->vs32 * c->vs32;
        esd::launch_fin_gen(f, c->stream);
    }
    esd::launch_scatter(n, c->p2u, c->x, xout, c->stream);
    if (sampling) {
        HIPCHK(hipMemcpyAsync(c->xN, c->x, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
        // iterates followed by another iteration of the same run (FP32 inner
        // run or FP64 finish) were sampled: a store rides on the next SpMV
        c->slot_iter.assign(c->m_req, 0);
        c->nsamples = 0;
        for (auto &sg : c->segments)
            for (int i = 1; i < sg.second; ++i) {
                const int tot = sg.first + i;
                if (method_b) {
                    for (int sl = 0; sl < c->m_req; ++sl)
                        if (c->b_slot_iter[sl] == tot) {
                            c->slot_iter[sl] = tot;
                            c->nsamples++;
                        }
                } else if (tot < (int)c->table_h.size() && c->table_h[tot] >= 0) {
                    c->slot_iter[c->table_h[tot]] = tot;
                    c->nsamples++;
                }
            }
        c->have_samples = c->nsamples > 0;
        c->armed = false;
    }
    st = sync_read(c);
    if (st) return st;
    st = read_history(c, total);
    if (st) return st;
    if (info) {
        info->iters = total;
        info->outer_iters = outer + 1;
        info->converged = converged;
        info->m_tilde = m;
        info->nsamples = sampling ? c->nsamples : 0;
        info->mode_used = kind;
        info->fp64_iters = fp64_iters;
        info->relres = bn2 > 0 ? std::sqrt(rn2 / bn2) : std::sqrt(rn2);
        info->true_relres = bn2 > 0 ? std::sqrt(c->Sh->out / bn2) : std::sqrt(c->Sh->out);
        info->lambda_max = power ? c->Sh->lam : 0.0;
        fill_lanczos(c, info);
    }
    return converged ? ESD_OK : ESD_NOT_CONVERGED;
}

// Y = M^{-1} A W, one column at a time through the preconditioner (FP64
// factor; FP32 copy for the mixed inner loop), so that the deflated
// iteration's (AW)^T z = Y^T r can be reduced inside the update launch.
// Needs the current factor: without it Y stays invalid until factor_ic0.
esd_status refresh_y(esd_ctx *c) {
    c->y_ok = false;
    if (!c->aux_built || c->m_tilde <= 0 || c->m_tilde > 16 || !c->factored) return ESD_OK;
    const int n = (int)c->n, k = c->m_tilde;
    auto V = vecs<double>(c);
    clear_sweep_vectors(c);
    init_scal(c, 1, 1.0, 0);
    esd_status st = put_scal(c);
    if (st) return st;
    for (int j = 0; j < k; ++j) {
        HIPCHK(hipMemcpyAsync(c->r, c->AW + (size_t)j * n, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
        launch_prec<double>(c, V, false, false);
        HIPCHK(hipMemcpyAsync(c->Y + (size_t)j * n, c->z, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    }
    if (c->mixed) esd::launch_cast((int64_t)k * n, c->Y, c->Y32, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    c->y_ok = true;
    return ESD_OK;
}

// C = W^T (A W) on the matrix cores, symmetrised; C^{-1} from its Cholesky
// factor (host, FP64); FP32 copies of W and AW for the mixed inner loop.
esd_status finish_aux(esd_ctx *c, int k) {
    const int n = (int)c->n;
    esd::launch_gram(n, c->W, k, c->AW, k, c->gram_part, c->G, esd::gram_grid(n), c->stream);
    std::vector<double> C((size_t)k * k), Cinv;
    HIPCHK(hipMemcpyAsync(C.data(), c->G, sizeof(double) * k * k, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < i; ++j) {
            const double s = 0.5 * (C[(size_t)i * k + j] + C[(size_t)j * k + i]);
            C[(size_t)i * k + j] = C[(size_t)j * k + i] = s;
        }
    if (!esd::cholesky_inverse(k, C, Cinv)) return fail(c, ESD_ENOTSPD, "W^T A W is not positive definite");
    c->Ch = C;
    c->fp32_short[1] = c->fp32_short[2] = false; // a new W: the deflated / SC operators changed
    HIPCHK(hipMemcpyAsync(c->Cinv, Cinv.data(), sizeof(double) * k * k, hipMemcpyHostToDevice, c->stream));
    if (c->mixed) {
        esd::launch_cast((int64_t)k * n, c->W, c->W32, c->stream);
        esd::launch_cast((int64_t)k * n, c->AW, c->AW32, c->stream);
    }
    esd::launch_to_rowmajor(n, k, c->W, c->W_rm, c->W32_rm, c->stream);
    esd::launch_to_rowmajor(n, k, c->AW, c->AW_rm, c->AW32_rm, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    c->m_tilde = k;
    c->aux_built = true;
    c->epoch++;
    return refresh_y(c);
}

} // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char *esd_status_string(esd_status s) {
    switch (s) {
    case ESD_OK: return "ok";
    case ESD_NOT_CONVERGED: return "not converged";
    case ESD_AUX_EMPTY: return "auxiliary space empty; solved as plain ICCG";
    case ESD_EINVAL: return "invalid argument";
    case ESD_ENOTSPD: return "IC(0) breakdown (matrix not SPD?)";
    case ESD_EHIP: return "HIP runtime error";
    case ESD_ENUMERIC: return "non-finite value";
    case ESD_ENOAUX: return "no auxiliary space built";
    case ESD_ENOSAMPLES: return "no samples";
    case ESD_EWORKSPACE: return "workspace missing, too small or misaligned";
    }
    return "unknown status";
}

const char *esd_last_error(const esd_ctx *c) { return c ? c->err.c_str() : "null context"; }

void esd_destroy(esd_ctx *c) {
    if (!c) return;
    // device memory belongs to the caller's workspace: only the host-side
    // state, events, graphs and the capture stream are released here
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    if (c->Sh) (void)hipHostFree(c->Sh);
    for (auto &e : c->ev) (void)hipEventDestroy(e);
    for (auto &g : c->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
}

} // extern "C"

namespace {

constexpr int64_t kDefaultMaxIters = 100000;

bool options_ok(const esd_options *o) {
    return o && o->m_max >= 1 && o->m_max <= esd::kMaxCols && o->max_iters >= 0 &&
           (o->prec == ESD_PREC_FP64 || o->prec == ESD_PREC_MIXED) &&
           (o->order == ESD_ORDER_NATURAL || o->order == ESD_ORDER_COLORS ||
            (o->order == ESD_ORDER_BLOCK_JACOBI && o->block_rows >= 1));
}

int64_t max_iters_of(const esd_options *o) { return o->max_iters > 0 ? o->max_iters : kDefaultMaxIters; }

// Upper bounds of every size for a matrix of n rows, nnz stored entries and
// at most max_row entries per row: a sorted-layout slice is at most max_row
// (L, U: max_row - 1) slots wide, a class-aligned copy at most 5/4 of it;
// a level launch has at most ceil(rows / 256) + 7 blocks and there are at
// most n levels, and a level of k rows at most ceil(k / 256) tiles.
Sizes size_bound(int64_t n, int64_t nnz, int64_t max_row, const esd_options *o) {
    Sizes z;
    z.n = n;
    z.nnz = nnz;
    const int64_t nsl = (n + esd::kSlice - 1) / esd::kSlice;
    const int64_t wa = std::min<int64_t>(max_row, n), wl = std::max<int64_t>(wa - 1, 0);
    z.A = {nsl, nsl * esd::kSlice * wa, 0};
    z.L = {nsl, nsl * esd::kSlice * wl, 0};
    z.U = z.L;
    for (EllSizes *e : {&z.A, &z.L, &z.U}) e->csize = e->size / 4 * 5 / esd::kSlice * esd::kSlice + esd::kSlice;
    const int64_t tiles = (n + esd::kBlock - 1) / esd::kBlock;
    z.tmap = tiles;
    z.tmap_lvl = tiles + n;
    z.sweep_cap = tiles + n + 7 * (n / 2048 + 1) + 8;
    z.m_max = o->m_max;
    z.mixed = o->prec == ESD_PREC_MIXED;
    z.max_iters = max_iters_of(o);
    return z;
}

esd_status setup_impl(esd_ctx **out, void *hip_stream, int64_t n, int64_t nnz, const int64_t *rowptr_d,
                      const int32_t *col_d, const double *val_d, const int32_t *colors_d, const esd_options *opt,
                      void *workspace, size_t ws_bytes, size_t *ws_needed) {
    if (ws_needed) *ws_needed = 0;
    if (!out) return ESD_EINVAL;
    *out = nullptr;
    if (!rowptr_d || !col_d || !val_d || n <= 0 || nnz < n || !options_ok(opt)) return ESD_EINVAL;
    if (opt->order == ESD_ORDER_COLORS && !colors_d) return ESD_EINVAL;
    if (n >= (int64_t(1) << 31) - 64 || nnz >= (int64_t(1) << 31)) return ESD_EINVAL;
    hipStream_t stream = (hipStream_t)hip_stream;
    // the caller's device CSR (and colours) to the host for the analysis
    std::vector<int64_t> rowptr(n + 1);
    std::vector<int32_t> col(nnz), colors;
    std::vector<double> val(nnz);
    bool hip_ok = hipMemcpyAsync(rowptr.data(), rowptr_d, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost,
                                 stream) == hipSuccess &&
                  hipMemcpyAsync(col.data(), col_d, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, stream) ==
                      hipSuccess &&
                  hipMemcpyAsync(val.data(), val_d, sizeof(double) * nnz, hipMemcpyDeviceToHost, stream) ==
                      hipSuccess;
    if (hip_ok && opt->order == ESD_ORDER_COLORS) {
        colors.resize(n);
        hip_ok = hipMemcpyAsync(colors.data(), colors_d, sizeof(int32_t) * n, hipMemcpyDeviceToHost, stream) ==
                 hipSuccess;
    }
    if (!hip_ok || hipStreamSynchronize(stream) != hipSuccess) return ESD_EHIP;
    if (rowptr[n] != nnz) {
        fprintf(stderr, "esd_setup: rowptr[n] != nnz\n");
        return ESD_EINVAL;
    }
    const int64_t block_rows = opt->order == ESD_ORDER_BLOCK_JACOBI ? opt->block_rows : 0;
    const int32_t *colp = opt->order == ESD_ORDER_COLORS ? colors.data() : nullptr;
    esd::HostLayout H;
    std::string why = esd::build_layout(n, rowptr.data(), col.data(), val.data(), colp, block_rows, H);
    if (!why.empty()) {
        fprintf(stderr, "esd_setup: %s\n", why.c_str());
        return ESD_EINVAL;
    }
    esd_ctx *c = new (std::nothrow) esd_ctx();
    if (!c) return ESD_EINVAL;
    c->stream = stream;
    c->m_max = opt->m_max;
    c->mixed = opt->prec == ESD_PREC_MIXED;
    c->max_iters = max_iters_of(opt);
    c->trace = std::getenv("ESD_TRACE") != nullptr;
    c->n = n;
    c->nnz = H.nnz;
    c->ncolors = H.ncolors;
    // the block kernels serve tridiagonal blocks; other block-Jacobi blocks
    // run through the level-scheduled sweeps of their in-block factor
    c->bj_rows = H.bj_scan ? H.block_rows : 0;
    c->bj_nb = c->bj_rows > 0 ? (int)((n + c->bj_rows - 1) / c->bj_rows) : 0;
    c->lvl = H.lvl_ptr;
    c->p2u_h = H.p2u;
    c->lperm_h = H.lperm;
    // class-aligned copies and tile orders on the host, then the exact sizes
    HostClass KA, KL, KU;
    const esd::HostEll *ells[3] = {&H.A, &H.L, &H.U};
    HostClass *ks[3] = {&KA, &KL, &KU};
    for (int e = 0; e < 3; ++e)
        if (c->class_layout && !ells[e]->col.empty() &&
            !esd::ell_classes(*ells[e], n, 64, ks[e]->csptr, ks[e]->soff, ks[e]->src))
            ks[e]->csptr.clear();
    std::vector<int32_t> tf, tl;
    esd::tile_orders(H, colp, esd::kBlock, tf, tl, c->tmap_off, esd::tile_parts(n), 1);
    Sizes z;
    z.n = n;
    z.nnz = H.nnz;
    EllSizes *zs[3] = {&z.A, &z.L, &z.U};
    for (int e = 0; e < 3; ++e) {
        zs[e]->nsl = (int64_t)ells[e]->sptr.size() - 1;
        zs[e]->size = (int64_t)ells[e]->col.size();
        zs[e]->csize = ks[e]->csptr.empty() ? 0 : ks[e]->csptr.back();
    }
    z.tmap = (int64_t)tf.size();
    z.tmap_lvl = (int64_t)tl.size();
    z.sweep_cap = sweep_slots(n, c->lvl, c->bj_nb);
    c->sweep_cap = z.sweep_cap;
    z.m_max = opt->m_max;
    z.mixed = c->mixed;
    z.max_iters = c->max_iters;
    const size_t need = carve(c, z, nullptr);
    if (ws_needed) *ws_needed = need;
    if (!workspace || ws_bytes < need || ((uintptr_t)workspace & 255)) {
        delete c;
        return ESD_EWORKSPACE;
    }
    (void)carve(c, z, static_cast<char *>(workspace));
    c->ws_used = need;
    esd_status st;
#define SETUP_CHK(x)                                                                               \
    do {                                                                                           \
        st = (x);                                                                                  \
        if (st != ESD_OK) { esd_destroy(c); return st; }                                           \
    } while (0)
#define SETUP_HIP(x)                                                                               \
    do {                                                                                           \
        if ((x) != hipSuccess) { esd_destroy(c); return ESD_EHIP; }                                \
    } while (0)
    SETUP_CHK(upload_ell(c, c->A, H.A, KA, c->mixed));
    SETUP_CHK(upload_ell(c, c->L, H.L, KL, c->mixed));
    SETUP_CHK(upload_ell(c, c->U, H.U, KU, c->mixed));
    if (c->A.size)
        SETUP_HIP(hipMemcpyAsync(c->a_src, H.a_src.data(), sizeof(int32_t) * c->A.size, hipMemcpyHostToDevice, c->stream));
    if (c->L.size)
        SETUP_HIP(hipMemcpyAsync(c->l_src, H.l_src.data(), sizeof(int32_t) * c->L.size, hipMemcpyHostToDevice, c->stream));
    SETUP_HIP(hipMemcpyAsync(c->d_src, H.d_src.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream));
    if (c->L.size)
        SETUP_HIP(hipMemcpyAsync(c->l_orig, c->L.v64, sizeof(double) * c->L.size, hipMemcpyDeviceToDevice, c->stream));
    if (!H.u_from_l.empty())
        SETUP_HIP(hipMemcpyAsync(c->u_from_l, H.u_from_l.data(), sizeof(int64_t) * H.u_from_l.size(),
                                 hipMemcpyHostToDevice, c->stream));
    const int64_t nv = n + 64;
    SETUP_HIP(hipMemcpyAsync(c->adiag, H.adiag.data(), sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    esd::launch_fill((int)nv, c->lsub, 0.0, c->stream);
    if (c->mixed) esd::launch_fill((int)nv, c->lsub32, 0.0f, c->stream);
    SETUP_HIP(hipMemcpyAsync(c->p2u, H.p2u.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, c->stream));
    SETUP_HIP(hipMemcpyAsync(c->tmap, tf.data(), sizeof(int32_t) * tf.size(), hipMemcpyHostToDevice, c->stream));
    if (!tl.empty())
        SETUP_HIP(hipMemcpyAsync(c->tmap_lvl, tl.data(), sizeof(int32_t) * tl.size(), hipMemcpyHostToDevice, c->stream));
    // the pattern in the caller's CSR order, for the gradient
    SETUP_HIP(hipMemcpyAsync(c->urp, rowptr_d, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToDevice, c->stream));
    SETUP_HIP(hipMemcpyAsync(c->ucol, col_d, sizeof(int32_t) * H.nnz, hipMemcpyDeviceToDevice, c->stream));
    double *v64[] = {c->b, c->x, c->r, c->z, c->zsc, c->y, c->q, c->p[0], c->p[1], c->t, c->v[0], c->v[1], c->xN};
    for (double *p : v64) esd::launch_fill((int)nv, p, 0.0, c->stream);
    if (c->mixed) {
        float *v32[] = {c->r32, c->z32, c->zsc32, c->y32, c->q32, c->p32[0], c->p32[1], c->d32, c->v32[0], c->v32[1]};
        for (float *p : v32) esd::launch_fill((int)nv, p, 0.0f, c->stream);
    }
    SETUP_HIP(hipMemsetAsync(c->S, 0, sizeof(Scal), c->stream));
    SETUP_HIP(hipHostMalloc((void **)&c->Sh, sizeof(Scal), hipHostMallocDefault));
    // the allocation-free solve's scratch on this device (a failure here only
    // disables esd_solve_noalloc)
    if (scratch_for_current_device(&c->scratch) != hipSuccess) {
        c->scratch = nullptr;
        (void)hipGetLastError();
    }
    std::memset(c->Sh, 0, sizeof(Scal));
    // the host copies die here: finish every transfer first
    if (hipStreamSynchronize(c->stream) != hipSuccess || hipGetLastError() != hipSuccess) {
        esd_destroy(c);
        return ESD_EHIP;
    }
#undef SETUP_CHK
#undef SETUP_HIP
    *out = c;
    return ESD_OK;
}
} // namespace

extern "C" {

size_t esd_workspace_bytes(int64_t n, int64_t nnz, int32_t max_row, const esd_options *opt) {
    if (n <= 0 || nnz < n || max_row < 1 || !options_ok(opt)) return 0;
    esd_ctx probe; // pointers are only counted, never assigned
    return carve(&probe, size_bound(n, nnz, max_row, opt), nullptr);
}

esd_status esd_setup(esd_ctx **out, void *hip_stream, int64_t n, int64_t nnz, const int64_t *rowptr,
                     const int32_t *col, const double *val, const int32_t *colors, const esd_options *opt,
                     void *workspace, size_t ws_bytes, size_t *ws_needed) {
    return setup_impl(out, hip_stream, n, nnz, rowptr, col, val, colors, opt, workspace, ws_bytes, ws_needed);
}

esd_status esd_workspace_used(const esd_ctx *c, size_t *bytes) {
    if (!c || !bytes) return ESD_EINVAL;
    *bytes = c->ws_used;
    return ESD_OK;
}


esd_status esd_factor_ic0(esd_ctx *c) {
    if (!c) return ESD_EINVAL;
    const int n = (int)c->n;
    HIPCHK(hipMemsetAsync(c->bad, 0, sizeof(int), c->stream));
    // L values start as a_ij; factor level by level, in place
    if (c->L.size)
        HIPCHK(hipMemcpyAsync(c->L.v64, c->l_orig, sizeof(double) * c->L.size, hipMemcpyDeviceToDevice, c->stream));
    const int nl = (int)c->lvl.size() - 1;
    Ell<double> L = c->L.e64();
    if (c->bj_rows > 0)
        esd::launch_factor_bj(n, (int)c->bj_rows, L, c->L.v64, c->adiag, c->ldiag, c->lsub, c->lsub32, c->bad,
                              c->stream);
    else
        for (int l = 0; l < nl; ++l)
            esd::launch_factor_level((int)c->lvl[l], (int)c->lvl[l + 1], n, L, c->L.v64, c->adiag, c->ldiag,
                                     c->bad, c->stream);
    esd::launch_finish_factor(n, c->ldiag, c->dinv, c->dinv32, c->stream);
    esd::launch_gather_u(c->U.size, c->u_from_l, c->L.v64, c->U.v64, c->stream);
    if (c->mixed) {
        esd::launch_cast(c->L.size, c->L.v64, c->L.v32, c->stream);
        esd::launch_cast(c->U.size, c->U.v64, c->U.v32, c->stream);
    }
    c->L.repack(c->stream);
    c->U.repack(c->stream);
    HIPCHK(hipGetLastError());
    int bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, c->bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (bad) {
        c->factored = false;
        c->y_ok = false;
        return fail(c, ESD_ENOTSPD, "IC(0) pivot <= 0");
    }
    c->factored = true;
    for (bool &f : c->fp32_short) f = false;
    return refresh_y(c); // M^{-1} A W for the new factor
}

esd_status esd_update_values(esd_ctx *c, const double *val) {
    if (!c || !val) return ESD_EINVAL;
    esd::launch_map_values(c->A.size, c->a_src, val, c->A.v64, c->A.v32, c->stream);
    c->A.repack(c->stream);
    esd::launch_map_values(c->L.size, c->l_src, val, c->l_orig, nullptr, c->stream);
    esd::launch_map_values(c->n, c->d_src, val, c->adiag, nullptr, c->stream);
    HIPCHK(hipGetLastError());
    c->factored = false;
    c->y_ok = false;
    c->lam_last = 0.0;
    for (bool &f : c->fp32_short) f = false;
    if (c->aux_built && c->m_tilde > 0) {
        // keep W, refresh AW = A W and C = W^T A W for the new values
        esd::launch_spmm((int)c->n, c->A.e64(), c->W, c->m_tilde, c->AW, c->stream);
        return finish_aux(c, c->m_tilde);
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return ESD_OK;
}

esd_status esd_sample_errors(esd_ctx *c, int32_t m, int32_t method) {
    if (!c) return ESD_EINVAL;
    if (m < 1 || m > c->m_max) return fail(c, ESD_EINVAL, "m must be in [1, m_max]");
    const int base = method & ~ESD_SAMPLE_RESIDUALS;
    if (base != ESD_SAMPLING_A && base != ESD_SAMPLING_B) return fail(c, ESD_EINVAL, "unknown sampling method");
    c->m_req = m;
    c->samp_method = base;
    c->samp_resid = (method & ESD_SAMPLE_RESIDUALS) != 0;
    c->armed = true;
    return ESD_OK;
}

esd_status esd_load_samples(esd_ctx *c, const double *X, int32_t k, const double *xN) {
    if (!c || !X || !xN) return ESD_EINVAL;
    if (k < 1 || k > c->m_max) return fail(c, ESD_EINVAL, "k must be in [1, m_max]");
    const int n = (int)c->n;
    for (int s = 0; s < k; ++s)
        esd::launch_gather(n, c->p2u, X + (size_t)s * n, c->slots + (size_t)s * n, c->stream);
    esd::launch_gather(n, c->p2u, xN, c->xN, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    c->m_req = k;
    c->slot_iter.resize(k);
    for (int s = 0; s < k; ++s) c->slot_iter[s] = s + 1;
    c->nsamples = k;
    c->have_samples = true;
    c->samp_resid = false;
    c->armed = false;
    return ESD_OK;
}

esd_status esd_set_mixed_params(esd_ctx *c, double inner_tol, int32_t max_outer) {
    if (!c || !(inner_tol > 0 && inner_tol < 1) || max_outer < 1) return ESD_EINVAL;
    c->inner_tol = inner_tol;
    c->max_outer = max_outer;
    for (bool &f : c->fp32_short) f = false;
    return ESD_OK;
}

esd_status esd_set_power_start(esd_ctx *c, const double *v0) {
    if (!c || !v0) return ESD_EINVAL;
    const int n = (int)c->n;
    esd::launch_gather(n, c->p2u, v0, c->v[0], c->stream);
    if (c->mixed) esd::launch_cast(n, c->v[0], c->v32[0], c->stream);
    c->vb64 = c->vb32 = 0;
    c->vs64 = c->vs32 = 1.0;
    c->have_v = true;
    HIPCHK(hipGetLastError());
    return ESD_OK;
}

} // extern "C"

namespace {
// Swaps the context's scalar block and block-partial tables for the scratch
// array for the duration of one allocation-free solve.
struct ScratchSwap {
    esd_ctx *c;
    Scal *S;
    double *spmv, *upd, *gen, *ts, *sweep;
    ScratchSwap(esd_ctx *ctx, double *base)
        : c(ctx), S(ctx->S), spmv(ctx->part_spmv), upd(ctx->part_upd), gen(ctx->part_gen), ts(ctx->part_ts),
          sweep(ctx->part_sweep) {
        c->S = reinterpret_cast<Scal *>(base);
        c->part_spmv = base + kScratchScal;
        c->part_upd = c->part_spmv + esd::kPartBudget;
        c->part_gen = c->part_upd + esd::kPartBudget;
        c->part_ts = c->part_gen + esd::kPartBudget;
        c->part_sweep = c->part_ts + esd::kPartBudget;
    }
    ~ScratchSwap() {
        c->S = S;
        c->part_spmv = spmv;
        c->part_upd = upd;
        c->part_gen = gen;
        c->part_ts = ts;
        c->part_sweep = sweep;
    }
};

esd_status solve_entry(esd_ctx *c, const double *b, const double *x0, double tol, int32_t maxit, int32_t mode,
                       int32_t flags, double *x, esd_info *info, bool noalloc) {
    if (!c || !b || !x || maxit < 0 || !(tol >= 0) || mode < 0 || mode > 2) return ESD_EINVAL;
    if (!c->factored && !(flags & ESD_FLAG_NOPREC)) return fail(c, ESD_EINVAL, "factor_ic0 not called");
    if ((flags & ESD_FLAG_POWER) && !c->have_v) return fail(c, ESD_EINVAL, "power start vector not set");
    if ((flags & ESD_FLAG_MIXED) && !c->mixed)
        return fail(c, ESD_EINVAL, "ESD_FLAG_MIXED needs a context set up with ESD_PREC_MIXED");
    if (noalloc) {
        if (flags & kFlagTiming) return fail(c, ESD_EINVAL, "esd_solve_noalloc takes no timing flags");
        if (!c->scratch) return fail(c, ESD_EHIP, "the scratch array of this device is unavailable");
        if (c->sweep_cap > kScratchSweep)
            return fail(c, ESD_EINVAL, "more sweep partial slots than the scratch array holds");
        flags |= ESD_FLAG_STREAM; // replaying a graph could need its instantiation first
    }
    esd_status warn = ESD_OK;
    int kind = mode;
    if (mode != ESD_PLAIN) {
        if (!c->aux_built) return fail(c, ESD_ENOAUX, "no auxiliary space: call build_aux or set_aux");
        if (c->m_tilde == 0) { kind = ESD_PLAIN; warn = ESD_AUX_EMPTY; }
    }
    esd_status st = ensure_tables(c, maxit, (flags & kFlagTiming) != 0);
    if (st) return st;
    if (flags & kFlagTiming) { c->t_spmv = c->t_sweep = c->t_upd = 0; c->t_count = 0; }
    esd_info tmp{};
    esd_info *inf = info ? info : &tmp;
    std::memset(inf, 0, sizeof(esd_info));
    if (noalloc) {
        // wall time on the host: the solve ends with a stream synchronisation
        const auto t0 = std::chrono::steady_clock::now();
        {
            ScratchSwap sw(c, c->scratch);
            if (flags & ESD_FLAG_MIXED) st = solve_mixed(c, b, x0, tol, maxit, kind, flags, x, inf);
            else st = solve_fp64(c, b, x0, tol, maxit, kind, flags, x, inf);
        }
        inf->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    } else {
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, c->stream));
        if (flags & ESD_FLAG_MIXED) st = solve_mixed(c, b, x0, tol, maxit, kind, flags, x, inf);
        else st = solve_fp64(c, b, x0, tol, maxit, kind, flags, x, inf);
        (void)hipEventRecord(e1, c->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        inf->seconds = ms * 1e-3;
    }
    if ((flags & ESD_FLAG_POWER) && st >= 0) c->lam_last = c->Sh->lam;
    inf->lambda_max = c->lam_last;
    inf->lambda_min_ritz = c->ritz.empty() ? 0.0 : c->ritz[0];
    inf->kappa_es = (inf->lambda_min_ritz > 0 && inf->lambda_max > 0) ? inf->lambda_max / inf->lambda_min_ritz : 0.0;
    if (st < 0) return st;
    if (st == ESD_OK && warn != ESD_OK) return warn;
    return st;
}
} // namespace

extern "C" {

esd_status esd_solve(esd_ctx *c, const double *b, const double *x0, double tol, int32_t maxit, int32_t mode,
                     int32_t flags, double *x, esd_info *info) {
    return solve_entry(c, b, x0, tol, maxit, mode, flags, x, info, false);
}

esd_status esd_solve_noalloc(esd_ctx *c, const double *b, const double *x0, double tol, int32_t maxit,
                             int32_t mode, int32_t flags, double *x, esd_info *info) {
    return solve_entry(c, b, x0, tol, maxit, mode, flags, x, info, true);
}

esd_status esd_sequence_rhs(esd_ctx *c, const double *f, const double *xprev, double cc, double *b) {
    if (!c || !f || !b) return ESD_EINVAL;
    esd::launch_axpby((int)c->n, f, xprev, cc, b, c->stream);
    HIPCHK(hipGetLastError());
    return ESD_OK;
}

esd_status esd_grad_values(esd_ctx *c, const double *lam, const double *x, double *gval) {
    if (!c || !lam || !x || !gval) return ESD_EINVAL;
    esd::launch_grad((int)c->n, c->urp, c->ucol, lam, x, gval, c->stream);
    HIPCHK(hipGetLastError()); // device output only: ordered on the stream, no synchronisation
    return ESD_OK;
}

esd_status esd_hbm_probe(void *hip_stream, int32_t kind, const double *src, double *dst, int64_t n, int32_t grid) {
    if ((kind != ESD_PROBE_COPY && kind != ESD_PROBE_READ) || !src || !dst || n < 2 || (n & 1) ||
        ((uintptr_t)src & 15) || ((uintptr_t)dst & 15) || grid < 0 || grid > 65536)
        return ESD_EINVAL;
    esd::launch_probe(kind == ESD_PROBE_COPY ? 0 : 1, src, dst, n, grid > 0 ? grid : 4096,
                      (hipStream_t)hip_stream);
    return hipGetLastError() == hipSuccess ? ESD_OK : ESD_EHIP;
}

esd_status esd_spmv(esd_ctx *c, const double *x, double *y) {
    if (!c || !x || !y) return ESD_EINVAL;
    const int n = (int)c->n;
    esd::launch_gather(n, c->p2u, x, c->t, c->stream);
    esd::launch_spmv(n, c->A.it64(), c->t, c->q, c->stream); // the layout of the iteration SpMV
    esd::launch_scatter(n, c->p2u, c->q, y, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return ESD_OK;
}

esd_status esd_prec_apply(esd_ctx *c, const double *r, double *z) {
    if (!c || !r || !z) return ESD_EINVAL;
    if (!c->factored) return fail(c, ESD_EINVAL, "factor_ic0 not called");
    const int n = (int)c->n;
    clear_sweep_vectors(c);
    esd::launch_gather(n, c->p2u, r, c->r, c->stream);
    init_scal(c, 1, 1.0, 0);
    esd_status st = put_scal(c);
    if (st) return st;
    auto V = vecs<double>(c);
    launch_prec<double>(c, V, false, false);
    esd::launch_scatter(n, c->p2u, c->z, z, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return ESD_OK;
}

esd_status esd_get_perm(esd_ctx *c, int32_t *perm) {
    if (!c || !perm) return ESD_EINVAL;
    std::memcpy(perm, c->lperm_h.data(), sizeof(int32_t) * c->n);
    return ESD_OK;
}

esd_status esd_get_factor_diag(esd_ctx *c, double *ldiag) {
    if (!c || !ldiag) return ESD_EINVAL;
    if (!c->factored) return fail(c, ESD_EINVAL, "factor_ic0 not called");
    std::vector<double> tmp(c->n);
    HIPCHK(hipMemcpy(tmp.data(), c->ldiag, sizeof(double) * c->n, hipMemcpyDeviceToHost));
    // physical -> user row order
    for (int64_t p = 0; p < c->n; ++p) ldiag[c->p2u_h[p]] = tmp[p];
    return ESD_OK;
}

esd_status esd_get_history(esd_ctx *c, double *alpha, double *beta, int32_t cap, int32_t *count) {
    if (!c) return ESD_EINVAL;
    int k = c->segments.empty() ? 0 : c->segments[0].second;
    if (count) *count = k;
    const int na = std::min<int>(k, cap), nb = std::min<int>(std::max(k - 1, 0), cap);
    if (alpha && na > 0) std::memcpy(alpha, c->ha_h.data(), sizeof(double) * na);
    if (beta && nb > 0) std::memcpy(beta, c->hb_h.data(), sizeof(double) * nb);
    return ESD_OK;
}

esd_status esd_get_samples(esd_ctx *c, int32_t *iters_by_slot) {
    if (!c || !iters_by_slot) return ESD_EINVAL;
    for (int s = 0; s < c->m_req; ++s) iters_by_slot[s] = s < (int)c->slot_iter.size() ? c->slot_iter[s] : 0;
    return ESD_OK;
}

esd_status esd_get_sample_vector(esd_ctx *c, int32_t slot, double *out) {
    if (!c || !out) return ESD_EINVAL;
    if (slot < 0 || slot >= c->m_req || !c->slots) return fail(c, ESD_EINVAL, "slot out of range");
    esd::launch_scatter((int)c->n, c->p2u, c->slots + (size_t)slot * c->n, out, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return ESD_OK;
}

esd_status esd_get_layout(esd_ctx *c, int32_t *out8) {
    if (!c || !out8) return ESD_EINVAL;
    out8[0] = (int32_t)c->n;
    out8[1] = (int32_t)c->nnz;
    out8[2] = (int32_t)c->lvl.size() - 1;
    out8[3] = c->ncolors;
    out8[4] = c->A.csize > 0;
    out8[5] = c->L.csize > 0;
    out8[6] = c->U.csize > 0;
    out8[7] = (int32_t)(c->A.csize ? c->A.csize : c->A.size);
    return ESD_OK;
}

esd_status esd_get_timing(esd_ctx *c, double *out4) {
    if (!c || !out4) return ESD_EINVAL;
    const double k = c->t_count > 0 ? (double)c->t_count : 1.0;
    out4[0] = c->t_spmv / k;
    out4[1] = c->t_sweep / k;
    out4[2] = c->t_upd / k;
    out4[3] = (double)c->t_count;
    return ESD_OK;
}

esd_status esd_build_aux(esd_ctx *c, double theta, double *ritz, int32_t *m_bar, int32_t *m_tilde) {
    if (!c) return ESD_EINVAL;
    if (!c->have_samples) return fail(c, ESD_ENOSAMPLES, "no sampling solve before build_aux");
    const int n = (int)c->n;
    std::vector<int> order;
    for (int s = 0; s < (int)c->slot_iter.size(); ++s)
        if (c->slot_iter[s] > 0) order.push_back(s);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return c->slot_iter[a] < c->slot_iter[b]; });
    c->aux_built = false;
    c->y_ok = false;
    c->m_tilde = 0;
    int kept = 0;
    esd_status st;
    for (int s : order) {
        double *v = c->E + (size_t)kept * n;
        // eq. (ek): e = x_1 - x~ (or the sampled residual itself), normalised,
        // then classical Gram-Schmidt twice
        if (c->samp_resid) esd::launch_scale_copy(n, c->slots + (size_t)s * n, v, 1.0, c->stream);
        else esd::launch_sub(n, c->xN, c->slots + (size_t)s * n, v, c->stream);
        dev_norm2(c, v, &c->S->out);
        if ((st = sync_read(c))) return st;
        double nv2 = c->Sh->out;
        if (!(nv2 > 0.0)) continue;
        esd::launch_scale_copy(n, v, v, 1.0 / std::sqrt(nv2), c->stream);
        if (kept > 0) {
            for (int pass = 0; pass < 2; ++pass) {
                dev_tsdot(c, c->E, kept, v, nullptr, 1.0);
                dev_axpy(c, v, c->E, kept, c->S->svec, -1.0, &c->S->out, 0);
            }
            if ((st = sync_read(c))) return st;
            nv2 = c->Sh->out;
        } else {
            nv2 = 1.0;
        }
        if (!(std::sqrt(nv2) > 1e-10)) continue; // dependent sample: dropped
        esd::launch_scale_copy(n, v, v, 1.0 / std::sqrt(nv2), c->stream);
        ++kept;
    }
    c->m_bar = kept;
    if (m_bar) *m_bar = kept;
    if (m_tilde) *m_tilde = 0;
    c->ritz.clear();
    if (kept == 0) {
        c->aux_built = true;
        return ESD_AUX_EMPTY;
    }
    // Rayleigh-Ritz: G = E^T (A E), eigenpairs on the host
    esd::launch_spmm(n, c->A.e64(), c->E, kept, c->AE, c->stream);
    esd::launch_gram(n, c->E, kept, c->AE, kept, c->gram_part, c->G, esd::gram_grid(n), c->stream);
    std::vector<double> G((size_t)kept * kept), w, V;
    HIPCHK(hipMemcpyAsync(G.data(), c->G, sizeof(double) * kept * kept, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int i = 0; i < kept; ++i)
        for (int j = 0; j < i; ++j) {
            const double s = 0.5 * (G[(size_t)i * kept + j] + G[(size_t)j * kept + i]);
            G[(size_t)i * kept + j] = G[(size_t)j * kept + i] = s;
        }
    if (c->rr_op == 1) {
        // preconditioned matrix (footnote of eq. (Rayleigh-Ritz)) in the M
        // inner product: G t = lambda B t with B = E^T M E, M e = L (L^T e)
        if (!c->factored) return fail(c, ESD_EINVAL, "Rayleigh-Ritz on M^{-1}A needs the IC(0) factor");
        // M E goes to W's buffer (m_max columns, rebuilt from E below)
        double *ME = c->W;
        for (int j = 0; j < kept; ++j) {
            esd::launch_tri_mul(n, c->U.e64(), c->ldiag, c->E + (size_t)j * n, c->t, c->stream);
            esd::launch_tri_mul(n, c->L.e64(), c->ldiag, c->t, ME + (size_t)j * n, c->stream);
        }
        esd::launch_gram(n, c->E, kept, ME, kept, c->gram_part, c->G, esd::gram_grid(n), c->stream);
        std::vector<double> B((size_t)kept * kept);
        HIPCHK(hipMemcpyAsync(B.data(), c->G, sizeof(double) * kept * kept, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (int i = 0; i < kept; ++i)
            for (int j = 0; j < i; ++j) {
                const double sb = 0.5 * (B[(size_t)i * kept + j] + B[(size_t)j * kept + i]);
                B[(size_t)i * kept + j] = B[(size_t)j * kept + i] = sb;
            }
        if (!esd::generalized_eigh(kept, G, B, w, V))
            return fail(c, ESD_ENUMERIC, "E^T M E is not positive definite");
    } else {
        esd::jacobi_eigh(kept, G, w, V);
    }
    c->ritz = w;
    if (ritz) std::memcpy(ritz, w.data(), sizeof(double) * kept);
    int sel = 0;
    while (sel < kept && w[sel] < theta) ++sel; // eq. (bk): Ritz values below theta
    if (m_tilde) *m_tilde = sel;
    if (sel == 0) {
        c->aux_built = true;
        return ESD_AUX_EMPTY;
    }
    // W = E T, AW = (A E) T with the selected Ritz vectors T (kept x sel, column-major)
    HIPCHK(hipMemcpyAsync(c->Tm, V.data(), sizeof(double) * kept * sel, hipMemcpyHostToDevice, c->stream));
    esd::launch_tsgemm(n, c->E, kept, c->Tm, sel, c->W, c->stream);
    esd::launch_tsgemm(n, c->AE, kept, c->Tm, sel, c->AW, c->stream);
    HIPCHK(hipGetLastError());
    return finish_aux(c, sel);
}

esd_status esd_set_rayleigh_ritz(esd_ctx *c, int32_t op) {
    if (!c) return ESD_EINVAL;
    if (op != ESD_RR_A && op != ESD_RR_PRECONDITIONED) return fail(c, ESD_EINVAL, "unknown Rayleigh-Ritz operator");
    c->rr_op = op;
    return ESD_OK;
}

esd_status esd_set_aux(esd_ctx *c, const double *W, int32_t k) {
    if (!c || !W) return ESD_EINVAL;
    if (k < 1 || k > c->m_max) return fail(c, ESD_EINVAL, "k must be in [1, m_max]");
    const int n = (int)c->n;
    for (int j = 0; j < k; ++j) esd::launch_gather(n, c->p2u, W + (size_t)j * n, c->W + (size_t)j * n, c->stream);
    esd::launch_spmm(n, c->A.e64(), c->W, k, c->AW, c->stream);
    HIPCHK(hipGetLastError());
    c->ritz.clear();
    c->m_bar = k;
    c->aux_built = false;
    c->y_ok = false;
    return finish_aux(c, k);
}

esd_status esd_get_aux(esd_ctx *c, double *W, double *C) {
    if (!c) return ESD_EINVAL;
    if (!c->aux_built) return fail(c, ESD_ENOAUX, "no auxiliary space");
    const int n = (int)c->n, k = c->m_tilde;
    if (W)
        for (int j = 0; j < k; ++j) esd::launch_scatter(n, c->p2u, c->W + (size_t)j * n, W + (size_t)j * n, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    if (C && k > 0) std::memcpy(C, c->Ch.data(), sizeof(double) * k * k);
    return ESD_OK;
}

} // extern "C"
