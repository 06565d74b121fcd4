// Test driver for the host-side logic of the esd library (ordering, levels,
// sliced-ELL layouts, tile orders, sampling table, small dense eigen- and
// Cholesky routines).  Built and run by tests/test_host_logic.py with g++;
// it reads little-endian binary inputs and writes binary outputs that the
// test checks against numpy / scipy / the oracle.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../paper_2203_08498_amd/csrc/esd_internal.h"

namespace {

template <typename T> std::vector<T> read_vec(FILE *f, size_t n) {
    std::vector<T> v(n);
    if (n && fread(v.data(), sizeof(T), n, f) != n) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return v;
}
template <typename T> T read_one(FILE *f) { return read_vec<T>(f, 1)[0]; }
template <typename T> void write_vec(FILE *f, const std::vector<T> &v) {
    const int64_t n = (int64_t)v.size();
    fwrite(&n, sizeof(n), 1, f);
    if (n) fwrite(v.data(), sizeof(T), v.size(), f);
}

// COO triples (row, col, val) of a sorted sliced-ELL matrix, padding skipped
void ell_coo(const esd::HostEll &E, int64_t n, std::vector<int64_t> &r, std::vector<int64_t> &c,
             std::vector<double> &v) {
    const int64_t nsl = (n + 63) / 64;
    for (int64_t s = 0; s < nsl; ++s) {
        const int64_t b = E.sptr[s], w = (E.sptr[s + 1] - b) / 64;
        for (int64_t k = 0; k < w; ++k)
            for (int64_t l = 0; l < 64; ++l) {
                const int64_t pos = b + k * 64 + l;
                if (E.col[pos] == (int32_t)n) continue;
                r.push_back(s * 64 + l);
                c.push_back(E.col[pos]);
                v.push_back(E.val[pos]);
            }
    }
}

// COO triples of the class-aligned copy, decoded as the kernels decode it
// (column = row + slot offset; entries without a source are absent)
bool class_coo(const esd::HostEll &E, int64_t n, std::vector<int64_t> &r, std::vector<int64_t> &c,
               std::vector<double> &v) {
    std::vector<int64_t> cs, src;
    std::vector<int32_t> so;
    if (!esd::ell_classes(E, n, 64, cs, so, src)) return false;
    const int64_t nsl = (n + 63) / 64;
    for (int64_t s = 0; s < nsl; ++s) {
        const int64_t w = (cs[s + 1] - cs[s]) / 64;
        for (int64_t k = 0; k < w; ++k)
            for (int64_t l = 0; l < 64; ++l) {
                const int64_t e = cs[s] + k * 64 + l;
                if (src[e] < 0) continue;
                r.push_back(s * 64 + l);
                c.push_back(s * 64 + l + so[cs[s] / 64 + k]);
                v.push_back(E.val[src[e]]);
            }
    }
    return true;
}

int layout(const char *in, const char *out) {
    FILE *f = fopen(in, "rb");
    if (!f) return 2;
    const int64_t n = read_one<int64_t>(f), nnz = read_one<int64_t>(f);
    const int32_t has_colors = read_one<int32_t>(f);
    const int64_t block_rows = read_one<int64_t>(f);
    auto rp = read_vec<int64_t>(f, n + 1);
    auto col = read_vec<int32_t>(f, nnz);
    auto val = read_vec<double>(f, nnz);
    std::vector<int32_t> colors;
    if (has_colors) colors = read_vec<int32_t>(f, n);
    fclose(f);
    esd::HostLayout H;
    const std::string why = esd::build_layout(n, rp.data(), col.data(), val.data(), has_colors ? colors.data() : nullptr,
                                              block_rows, H);
    FILE *o = fopen(out, "wb");
    const int32_t ok = why.empty() ? 1 : 0;
    fwrite(&ok, sizeof(ok), 1, o);
    if (!ok) {
        fprintf(o, "%s", why.c_str());
        fclose(o);
        return 0;
    }
    write_vec(o, H.lperm);
    write_vec(o, H.p2u);
    write_vec(o, H.p2l);
    write_vec(o, H.lvl_ptr);
    const esd::HostEll *mats[3] = {&H.A, &H.L, &H.U};
    for (const esd::HostEll *E : mats) {
        std::vector<int64_t> r, c;
        std::vector<double> v;
        ell_coo(*E, n, r, c, v);
        write_vec(o, r);
        write_vec(o, c);
        write_vec(o, v);
        std::vector<int64_t> r2, c2;
        std::vector<double> v2;
        const int32_t cls = class_coo(*E, n, r2, c2, v2) ? 1 : 0;
        fwrite(&cls, sizeof(cls), 1, o);
        write_vec(o, r2);
        write_vec(o, c2);
        write_vec(o, v2);
    }
    std::vector<int32_t> tf, tl;
    std::vector<int64_t> toff;
    esd::tile_orders(H, has_colors ? colors.data() : nullptr, 256, tf, tl, toff);
    write_vec(o, tf);
    write_vec(o, tl);
    write_vec(o, toff);
    // the same with 4 parts per eighth in the whole range and 2 in the levels
    esd::tile_orders(H, has_colors ? colors.data() : nullptr, 256, tf, tl, toff, 4, 2);
    write_vec(o, tf);
    write_vec(o, tl);
    write_vec(o, toff);
    fclose(o);
    return 0;
}

int dense(const char *mode, const char *in, const char *out) {
    FILE *f = fopen(in, "rb");
    if (!f) return 2;
    const int32_t k = read_one<int32_t>(f);
    auto G = read_vec<double>(f, (size_t)k * k); // column-major
    std::vector<double> B;
    if (!strcmp(mode, "geig")) B = read_vec<double>(f, (size_t)k * k);
    fclose(f);
    FILE *o = fopen(out, "wb");
    std::vector<double> w, V;
    int32_t ok = 1;
    if (!strcmp(mode, "eig")) {
        esd::jacobi_eigh(k, G, w, V);
    } else if (!strcmp(mode, "geig")) {
        ok = esd::generalized_eigh(k, G, B, w, V) ? 1 : 0;
    } else if (!strcmp(mode, "cholinv")) {
        ok = esd::cholesky_inverse(k, G, V) ? 1 : 0;
    } else {
        fclose(o);
        return 2;
    }
    fwrite(&ok, sizeof(ok), 1, o);
    write_vec(o, w);
    write_vec(o, V);
    fclose(o);
    return 0;
}

int tridiag(const char *in, const char *out) {
    FILE *f = fopen(in, "rb");
    if (!f) return 2;
    const int32_t k = read_one<int32_t>(f);
    auto a = read_vec<double>(f, k);
    auto b = read_vec<double>(f, k);
    fclose(f);
    double lo = 0, hi = 0;
    esd::tridiag_extremes(k, a.data(), b.data(), &lo, &hi);
    FILE *o = fopen(out, "wb");
    fwrite(&lo, sizeof(lo), 1, o);
    fwrite(&hi, sizeof(hi), 1, o);
    fclose(o);
    return 0;
}

int sampling(int m, int64_t maxit, const char *out) {
    std::vector<int32_t> t;
    esd::sampling_table(m, maxit, t);
    FILE *o = fopen(out, "wb");
    write_vec(o, t);
    fclose(o);
    return 0;
}

} // namespace

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    const std::string mode = argv[1];
    if (mode == "layout" && argc == 4) return layout(argv[2], argv[3]);
    if ((mode == "eig" || mode == "geig" || mode == "cholinv") && argc == 4) return dense(argv[1], argv[2], argv[3]);
    if (mode == "tridiag" && argc == 4) return tridiag(argv[2], argv[3]);
    if (mode == "sampling" && argc == 5) return sampling(atoi(argv[2]), atoll(argv[3]), argv[4]);
    return 2;
}
