// Host-side setup of the esd library: ordering, level schedule, sliced-ELL
// formats, the sampling schedule and the small dense helpers.  Runs once per
// matrix (or once per solve for the schedule); nothing here is on the
// per-iteration path.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "esd_internal.h"

namespace esd {

namespace {

struct Ent {
    int32_t key; // sort key (physical or logical column)
    int32_t pc;  // physical column
    double v;
    int32_t src; // position in the caller's CSR
};

void ell_alloc(HostEll &E, const std::vector<int32_t> &len, int64_t n) {
    int64_t nsl = (n + kSlice - 1) / kSlice;
    E.sptr.assign(nsl + 1, 0);
    for (int64_t s = 0; s < nsl; ++s) {
        int32_t w = 0;
        for (int64_t r = s * kSlice; r < std::min<int64_t>(n, (s + 1) * kSlice); ++r) w = std::max(w, len[r]);
        E.sptr[s + 1] = E.sptr[s] + (int64_t)w * kSlice;
    }
    E.col.assign(E.sptr[nsl], 0);
    E.val.assign(E.sptr[nsl], 0.0);
    // padding: column n (every gathered vector holds a zero there), value 0
    std::fill(E.col.begin(), E.col.end(), (int32_t)n);
}

inline int64_t ell_pos(const HostEll &E, int64_t row, int64_t k) {
    return E.sptr[row / kSlice] + k * kSlice + (row % kSlice);
}

} // namespace

std::string build_layout(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                         const int32_t *colors, int64_t block_rows, HostLayout &H) {
    if (n <= 0 || n >= (int64_t(1) << 31) - 64) return "n out of range";
    if (rowptr[n] >= (int64_t(1) << 31)) return "nnz out of range";
    if (rowptr[0] != 0) return "rowptr[0] != 0";
    for (int64_t i = 0; i < n; ++i)
        if (rowptr[i + 1] < rowptr[i]) return "rowptr not monotone";
    const int64_t nnz = rowptr[n];
    H.n = n;
    H.nnz = nnz;
    H.block_rows = block_rows;
    if (block_rows < 0) return "block size out of range";
    if (block_rows > 0 && colors) return "block Jacobi keeps the natural order (no colours)";
    // block Jacobi: the factor keeps only couplings inside a block of
    // block_rows consecutive rows
    const auto in_blk = [block_rows](int64_t u, int64_t c) { return block_rows == 0 || u / block_rows == c / block_rows; };
    // validate rows: columns in range, strictly increasing, diagonal present
    for (int64_t i = 0; i < n; ++i) {
        bool diag = false;
        for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            if (col[k] < 0 || col[k] >= n) return "column index out of range";
            if (k > rowptr[i] && col[k] <= col[k - 1]) return "columns not strictly increasing in a row";
            if (col[k] == i) diag = true;
        }
        if (!diag) return "missing diagonal entry";
    }
    // tridiagonal blocks (every coupling inside a block joins consecutive rows)
    // take the one-launch block sweeps; other blocks the level schedule of
    // their in-block couplings
    H.bj_scan = block_rows > 0 && block_rows <= kMaxBlockRows;
    if (block_rows > 0)
        for (int64_t i = 0; i < n && H.bj_scan; ++i)
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (col[k] != i && in_blk(i, col[k]) && col[k] != i - 1 && col[k] != i + 1) {
                    H.bj_scan = false;
                    break;
                }
    // logical order: stable counting sort by colour
    H.lperm.resize(n);
    std::vector<int32_t> lpos(n);
    H.ncolors = 1;
    if (colors) {
        int32_t cmax = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (colors[i] < 0 || colors[i] > (1 << 20)) return "colour out of range";
            cmax = std::max(cmax, colors[i]);
        }
        for (int64_t i = 0; i < n; ++i)
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (col[k] != i && colors[col[k]] == colors[i]) return "coupled rows share a colour";
        std::vector<int64_t> cnt(cmax + 2, 0);
        for (int64_t i = 0; i < n; ++i) cnt[colors[i] + 1]++;
        for (int32_t c = 0; c <= cmax; ++c) cnt[c + 1] += cnt[c];
        for (int64_t i = 0; i < n; ++i) H.lperm[cnt[colors[i]]++] = (int32_t)i;
        H.ncolors = cmax + 1;
    } else {
        std::iota(H.lperm.begin(), H.lperm.end(), 0);
    }
    for (int64_t l = 0; l < n; ++l) lpos[H.lperm[l]] = (int32_t)l;
    // level of every logical row: longest chain of logically-lower couplings
    std::vector<int32_t> lev(n, 0);
    int32_t nlev = 1;
    // (tridiagonal block Jacobi: one level, the block sweeps do not use the
    // level schedule; other block Jacobi: chains of in-block couplings only)
    for (int64_t l = 0; l < (H.bj_scan ? 0 : n); ++l) {
        int32_t u = H.lperm[l], lv = 0;
        for (int64_t k = rowptr[u]; k < rowptr[u + 1]; ++k) {
            int32_t lc = lpos[col[k]];
            if (lc < l && in_blk(u, col[k])) lv = std::max(lv, lev[lc] + 1);
        }
        lev[l] = lv;
        nlev = std::max(nlev, lv + 1);
    }
    // physical order: by level, logical order inside a level
    std::vector<int64_t> lc(nlev + 1, 0);
    for (int64_t l = 0; l < n; ++l) lc[lev[l] + 1]++;
    for (int32_t v = 0; v < nlev; ++v) lc[v + 1] += lc[v];
    H.lvl_ptr.assign(lc.begin(), lc.end());
    H.p2l.resize(n);
    std::vector<int32_t> ppos(n);
    {
        std::vector<int64_t> fill(lc.begin(), lc.end() - 1);
        for (int64_t l = 0; l < n; ++l) {
            int64_t p = fill[lev[l]]++;
            H.p2l[p] = (int32_t)l;
            ppos[l] = (int32_t)p;
        }
    }
    H.p2u.resize(n);
    H.u2p.resize(n);
    for (int64_t p = 0; p < n; ++p) H.p2u[p] = H.lperm[H.p2l[p]];
    for (int64_t u = 0; u < n; ++u) H.u2p[u] = ppos[lpos[u]];
    // row lengths
    std::vector<int32_t> lenA(n), lenL(n), lenU(n);
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        int32_t u = H.p2u[p], l = H.p2l[p], a = 0, lo = 0, up = 0;
        for (int64_t k = rowptr[u]; k < rowptr[u + 1]; ++k) {
            ++a;
            int32_t q = lpos[col[k]];
            if (!in_blk(u, col[k])) continue;
            if (q < l) ++lo; else if (q > l) ++up;
        }
        lenA[p] = a; lenL[p] = lo; lenU[p] = up;
    }
    ell_alloc(H.A, lenA, n);
    ell_alloc(H.L, lenL, n);
    ell_alloc(H.U, lenU, n);
    H.adiag.assign(n, 0.0);
    H.a_src.assign(H.A.col.size(), -1);
    H.l_src.assign(H.L.col.size(), -1);
    H.d_src.assign(n, -1);
#pragma omp parallel
    {
        std::vector<Ent> ea, el, eu;
#pragma omp for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            int32_t u = H.p2u[p], l = H.p2l[p];
            ea.clear(); el.clear(); eu.clear();
            for (int64_t k = rowptr[u]; k < rowptr[u + 1]; ++k) {
                int32_t cu = col[k], q = lpos[cu], pc = ppos[q];
                ea.push_back({pc, pc, val[k], (int32_t)k});
                if (!in_blk(u, cu)) continue;
                if (q < l) el.push_back({q, pc, val[k], (int32_t)k});
                else if (q > l) eu.push_back({q, pc, val[k], (int32_t)k});
                else { H.adiag[p] = val[k]; H.d_src[p] = (int32_t)k; }
            }
            auto by = [](const Ent &a, const Ent &b) { return a.key < b.key; };
            std::sort(ea.begin(), ea.end(), by);
            std::sort(el.begin(), el.end(), by);
            std::sort(eu.begin(), eu.end(), by);
            for (size_t k = 0; k < ea.size(); ++k) {
                int64_t pos = ell_pos(H.A, p, k);
                H.A.col[pos] = ea[k].pc; H.A.val[pos] = ea[k].v; H.a_src[pos] = ea[k].src;
            }
            for (size_t k = 0; k < el.size(); ++k) {
                int64_t pos = ell_pos(H.L, p, k);
                H.L.col[pos] = el[k].pc; H.L.val[pos] = el[k].v; H.l_src[pos] = el[k].src;
            }
            for (size_t k = 0; k < eu.size(); ++k) {
                int64_t pos = ell_pos(H.U, p, k);
                H.U.col[pos] = eu[k].pc; H.U.val[pos] = eu[k].v;
            }
        }
    }
    // U slot -> L slot of the transposed entry (row pc of L holds column p)
    H.u_from_l.assign(H.U.col.size(), -1);
    std::string err;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; ++p) {
        for (int32_t k = 0; k < lenU[p]; ++k) {
            int64_t pos = ell_pos(H.U, p, k);
            int32_t pc = H.U.col[pos];
            int64_t found = -1;
            for (int32_t t = 0; t < lenL[pc]; ++t) {
                int64_t q = ell_pos(H.L, pc, t);
                if (H.L.col[q] == p) { found = q; break; }
            }
            H.u_from_l[pos] = found;
        }
    }
    for (int64_t p = 0; p < n; ++p)
        for (int32_t k = 0; k < lenU[p]; ++k)
            if (H.u_from_l[ell_pos(H.U, p, k)] < 0) return "matrix pattern is not symmetric";
    return std::string();
}

int sampling_slot(int64_t i, int m) {
    // (sum_{l >= 0} (-1)^l floor((i-1)/m^l)) mod m; the terms vanish once m^l > i-1
    if (m <= 1) return 0;
    int64_t acc = 0, div = 1;
    bool plus = true;
    for (;;) {
        int64_t t = (i - 1) / div;
        if (t == 0) break;
        acc += plus ? t : -t;
        plus = !plus;
        if (div > (int64_t(1) << 40) / m) break;
        div *= m;
    }
    return (int)(((acc % m) + m) % m);
}

void sampling_table(int m, int64_t maxit, std::vector<int32_t> &slot_of_iter) {
    slot_of_iter.assign(maxit + 2, -1);
    int64_t h = 1;
    for (int64_t i = 1; i <= maxit + 1; ++i) {
        if (i % h != 0) continue;
        slot_of_iter[i] = sampling_slot(i, m);
        if (i == h * (int64_t)m) h <<= 1;
    }
}

// Symmetric eigen-decomposition by Jacobi rotations with a threshold sweep
// (Rutishauser's formulation).  a: k x k column-major, destroyed.  w ascending,
// V column-major with the eigenvectors as columns.
void jacobi_eigh(int k, std::vector<double> &a, std::vector<double> &w, std::vector<double> &V) {
    auto A = [&](int i, int j) -> double & { return a[(size_t)j * k + i]; };
    V.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) V[(size_t)i * k + i] = 1.0;
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int j = 0; j < k; ++j) {
            diag += A(j, j) * A(j, j);
            for (int i = 0; i < j; ++i) off += 2.0 * A(i, j) * A(i, j);
        }
        if (off == 0.0 || off < 1e-30 * diag) break;
        double thresh = sweep < 3 ? 0.2 * std::sqrt(off) / ((double)k * k) : 0.0;
        for (int p = 0; p < k; ++p)
            for (int q = p + 1; q < k; ++q) {
                double apq = A(p, q);
                if (std::fabs(apq) <= thresh || apq == 0.0) continue;
                double theta = 0.5 * (A(q, q) - A(p, p)) / apq;
                double t = 1.0 / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                if (theta < 0) t = -t;
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c, tau = s / (1.0 + c);
                double app = A(p, p), aqq = A(q, q);
                A(p, p) = app - t * apq;
                A(q, q) = aqq + t * apq;
                A(p, q) = A(q, p) = 0.0;
                for (int r = 0; r < k; ++r) {
                    if (r == p || r == q) continue;
                    double arp = A(r, p), arq = A(r, q);
                    double nrp = arp - s * (arq + tau * arp);
                    double nrq = arq + s * (arp - tau * arq);
                    A(r, p) = A(p, r) = nrp;
                    A(r, q) = A(q, r) = nrq;
                }
                for (int r = 0; r < k; ++r) {
                    double vrp = V[(size_t)p * k + r], vrq = V[(size_t)q * k + r];
                    V[(size_t)p * k + r] = vrp - s * (vrq + tau * vrp);
                    V[(size_t)q * k + r] = vrq + s * (vrp - tau * vrq);
                }
            }
    }
    std::vector<int> idx(k);
    std::iota(idx.begin(), idx.end(), 0);
    std::vector<double> d(k);
    for (int i = 0; i < k; ++i) d[i] = A(i, i);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
    std::vector<double> V2((size_t)k * k);
    w.resize(k);
    for (int j = 0; j < k; ++j) {
        w[j] = d[idx[j]];
        std::memcpy(&V2[(size_t)j * k], &V[(size_t)idx[j] * k], sizeof(double) * k);
    }
    V.swap(V2);
}

// C (k x k, row-major, SPD) = R R^T; Cinv = R^{-T} R^{-1} (row-major).
bool cholesky_inverse(int k, const std::vector<double> &C, std::vector<double> &Cinv) {
    std::vector<double> R((size_t)k * k, 0.0), Ri((size_t)k * k, 0.0);
    for (int j = 0; j < k; ++j) {
        double d = C[(size_t)j * k + j];
        for (int t = 0; t < j; ++t) d -= R[(size_t)j * k + t] * R[(size_t)j * k + t];
        if (!(d > 0.0)) return false;
        R[(size_t)j * k + j] = std::sqrt(d);
        for (int i = j + 1; i < k; ++i) {
            double s = C[(size_t)i * k + j];
            for (int t = 0; t < j; ++t) s -= R[(size_t)i * k + t] * R[(size_t)j * k + t];
            R[(size_t)i * k + j] = s / R[(size_t)j * k + j];
        }
    }
    // Ri = R^{-1} (lower), column by column
    for (int c = 0; c < k; ++c) {
        for (int i = c; i < k; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int t = c; t < i; ++t) s -= R[(size_t)i * k + t] * Ri[(size_t)t * k + c];
            Ri[(size_t)i * k + c] = s / R[(size_t)i * k + i];
        }
    }
    Cinv.assign((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            double s = 0.0;
            for (int t = std::max(i, j); t < k; ++t) s += Ri[(size_t)t * k + i] * Ri[(size_t)t * k + j];
            Cinv[(size_t)i * k + j] = s;
        }
    return true;
}

// Extreme eigenvalues of the CG-Lanczos tridiagonal matrix (diagonal
// 1/alpha_j + beta_{j-1}/alpha_{j-1}, off-diagonal sqrt(beta_j)/alpha_j) by
// bisection on the LDL^T inertia count.
void tridiag_extremes(int k, const double *alpha, const double *beta, double *tmin, double *tmax) {
    if (k <= 0) { *tmin = *tmax = 0.0; return; }
    std::vector<double> d(k), o2(k > 1 ? k - 1 : 1);
    for (int j = 0; j < k; ++j) d[j] = 1.0 / alpha[j] + (j ? beta[j - 1] / alpha[j - 1] : 0.0);
    for (int j = 0; j + 1 < k; ++j) o2[j] = beta[j] / (alpha[j] * alpha[j]);
    double lo = d[0], hi = d[0];
    for (int j = 0; j < k; ++j) {
        double r = (j ? std::sqrt(o2[j - 1]) : 0.0) + (j + 1 < k ? std::sqrt(o2[j]) : 0.0);
        lo = std::min(lo, d[j] - r);
        hi = std::max(hi, d[j] + r);
    }
    auto below = [&](double x) { // eigenvalues strictly below x
        int c = 0;
        double piv = d[0] - x;
        if (piv < 0) ++c;
        for (int j = 1; j < k; ++j) {
            double prev = piv != 0.0 ? piv : 1e-300;
            piv = d[j] - x - o2[j - 1] / prev;
            if (piv < 0) ++c;
        }
        return c;
    };
    auto bisect = [&](int target) { // smallest x with below(x) >= target
        double a = lo, b = hi;
        for (int it = 0; it < 256; ++it) {
            double mid = a + 0.5 * (b - a);
            if (mid <= a || mid >= b) break;
            if (below(mid) >= target) b = mid; else a = mid;
        }
        return a + 0.5 * (b - a);
    };
    *tmin = bisect(1);
    *tmax = bisect(k);
}


void tile_orders(const HostLayout &H, const int32_t *colors, int tile_rows, std::vector<int32_t> &full,
                 std::vector<int32_t> &lvl, std::vector<int64_t> &lvl_off, int sub_full, int sub_lvl) {
    const int64_t n = H.n;
    const int nl = (int)H.lvl_ptr.size() - 1;
    // segment of every physical row: runs of equal (level, colour)
    std::vector<int64_t> seg_start(n), seg_len(n);
    for (int l = 0; l < nl; ++l) {
        int64_t a = H.lvl_ptr[l];
        const int64_t e = H.lvl_ptr[l + 1];
        while (a < e) {
            int64_t b = a + 1;
            if (colors)
                while (b < e && colors[H.p2u[b]] == colors[H.p2u[a]]) ++b;
            else
                b = e;
            for (int64_t p = a; p < b; ++p) {
                seg_start[p] = a;
                seg_len[p] = b - a;
            }
            a = b;
        }
    }
    // key of a tile: the eighth of its segment (the XCD), then the sub-th part
    // of that eighth; tiles of equal key keep their order (segment by
    // segment).  With sub > 1 an XCD walks its eighth of every colour
    // together, part by part, so the neighbours a part gathers from the
    // other colours were fetched into its L2 shortly before.
    auto order = [&](int64_t r0, int64_t r1, std::vector<int32_t> &out, int sub) {
        const int nk = 8 * std::max(sub, 1);
        const int64_t nt = (r1 - r0 + tile_rows - 1) / tile_rows;
        std::vector<std::vector<int32_t>> byk(nk);
        for (int64_t t = 0; t < nt; ++t) {
            const int64_t p = r0 + t * tile_rows;
            const int k = (int)std::min<int64_t>(nk - 1, nk * (p - seg_start[p]) / seg_len[p]);
            byk[k].push_back((int32_t)t);
        }
        for (auto &v : byk) out.insert(out.end(), v.begin(), v.end());
    };
    full.clear();
    lvl.clear();
    lvl_off.assign(nl + 1, 0);
    if (n == 0) return;
    order(0, n, full, sub_full);
    for (int l = 0; l < nl; ++l) {
        lvl_off[l] = (int64_t)lvl.size();
        order(H.lvl_ptr[l], H.lvl_ptr[l + 1], lvl, sub_lvl);
    }
    lvl_off[nl] = (int64_t)lvl.size();
}

bool ell_classes(const HostEll &E, int64_t n, int max_width, std::vector<int64_t> &sptr, std::vector<int32_t> &soff,
                 std::vector<int64_t> &src) {
    const int64_t nsl = (n + kSlice - 1) / kSlice;
    std::vector<std::vector<int32_t>> offs(nsl);
    bool ok = true;
#pragma omp parallel for schedule(static) reduction(&& : ok)
    for (int64_t s = 0; s < nsl; ++s) {
        std::vector<int32_t> &o = offs[s];
        const int64_t b = E.sptr[s], w = (E.sptr[s + 1] - b) / kSlice;
        for (int64_t k = 0; k < w; ++k)
            for (int64_t l = 0; l < kSlice; ++l) {
                const int32_t c = E.col[b + k * kSlice + l];
                if (c != (int32_t)n) o.push_back((int32_t)(c - (s * kSlice + l)));
            }
        std::sort(o.begin(), o.end());
        o.erase(std::unique(o.begin(), o.end()), o.end());
        if ((int)o.size() > max_width) ok = false;
    }
    sptr.assign(nsl + 1, 0);
    for (int64_t s = 0; s < nsl && ok; ++s) sptr[s + 1] = sptr[s] + (int64_t)offs[s].size() * kSlice;
    if (!ok || sptr[nsl] * 4 > (int64_t)E.col.size() * 5) {
        sptr.clear();
        return false;
    }
    soff.assign(sptr[nsl] / kSlice, 0);
    src.assign(sptr[nsl], -1);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < nsl; ++s) {
        const std::vector<int32_t> &o = offs[s];
        for (size_t k = 0; k < o.size(); ++k) soff[sptr[s] / kSlice + (int64_t)k] = o[k];
        const int64_t b = E.sptr[s], w = (E.sptr[s + 1] - b) / kSlice;
        for (int64_t k = 0; k < w; ++k)
            for (int64_t l = 0; l < kSlice; ++l) {
                const int64_t pos = b + k * kSlice + l;
                const int32_t c = E.col[pos];
                if (c == (int32_t)n) continue;
                const int64_t kk = std::lower_bound(o.begin(), o.end(), (int32_t)(c - (s * kSlice + l))) - o.begin();
                src[sptr[s] + kk * kSlice + l] = pos;
            }
    }
    return true;
}

bool generalized_eigh(int k, const std::vector<double> &G, const std::vector<double> &B, std::vector<double> &w,
                      std::vector<double> &T) {
    auto at = [k](const std::vector<double> &a, int i, int j) { return a[(size_t)j * k + i]; };
    std::vector<double> R((size_t)k * k, 0.0); // lower, column-major
    auto r = [&](int i, int j) -> double & { return R[(size_t)j * k + i]; };
    for (int j = 0; j < k; ++j) {
        double s = at(B, j, j);
        for (int t = 0; t < j; ++t) s -= r(j, t) * r(j, t);
        if (!(s > 0.0)) return false;
        r(j, j) = std::sqrt(s);
        for (int i = j + 1; i < k; ++i) {
            double u = at(B, i, j);
            for (int t = 0; t < j; ++t) u -= r(i, t) * r(j, t);
            r(i, j) = u / r(j, j);
        }
    }
    // X = R^{-1} G (forward substitution, column by column)
    std::vector<double> X((size_t)k * k);
    for (int c = 0; c < k; ++c)
        for (int i = 0; i < k; ++i) {
            double s = at(G, i, c);
            for (int t = 0; t < i; ++t) s -= r(i, t) * X[(size_t)c * k + t];
            X[(size_t)c * k + i] = s / r(i, i);
        }
    // H = X R^{-T}: row i of H solves R h = (row i of X)^T
    std::vector<double> H((size_t)k * k);
    for (int i = 0; i < k; ++i)
        for (int c = 0; c < k; ++c) {
            double s = X[(size_t)c * k + i];
            for (int t = 0; t < c; ++t) s -= r(c, t) * H[(size_t)t * k + i];
            H[(size_t)c * k + i] = s / r(c, c);
        }
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < i; ++j) {
            const double s = 0.5 * (H[(size_t)j * k + i] + H[(size_t)i * k + j]);
            H[(size_t)j * k + i] = H[(size_t)i * k + j] = s;
        }
    std::vector<double> V;
    jacobi_eigh(k, H, w, V);
    // T = R^{-T} V (back substitution, column by column)
    T.assign((size_t)k * k, 0.0);
    for (int c = 0; c < k; ++c)
        for (int i = k - 1; i >= 0; --i) {
            double s = V[(size_t)c * k + i];
            for (int t = i + 1; t < k; ++t) s -= r(t, i) * T[(size_t)c * k + t];
            T[(size_t)c * k + i] = s / r(i, i);
        }
    return true;
}

} // namespace esd
