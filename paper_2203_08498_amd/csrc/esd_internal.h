// Internal structures of the esd library (not part of the public ABI).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace esd {

constexpr int kSlice = 64;   // sliced-ELL slice height = wavefront size
constexpr int kMaxCols = 64; // largest auxiliary-space dimension
constexpr int kMaxBlockRows = 512; // largest block of the block-scan sweeps (one wavefront, 8 rows per lane)

// Sliced-ELL matrix on the host while it is being built: slice s holds rows
// [64 s, 64 s + 64); entry k of lane t sits at sptr[s] + 64 k + t.  Padding
// entries carry value 0 and column n.
struct HostEll {
    std::vector<int64_t> sptr;
    std::vector<int32_t> col;
    std::vector<double> val;
};

// Everything the host computes once per matrix (ordering, levels, formats).
struct HostLayout {
    int64_t n = 0, nnz = 0;
    int ncolors = 0;
    int64_t block_rows = 0;        // > 0: block-Jacobi IC(0) with blocks of that many consecutive rows
    bool bj_scan = false;          // block Jacobi with tridiagonal blocks: one level, block-scan sweeps
    std::vector<int32_t> lperm;    // logical position -> user row
    std::vector<int32_t> p2u;      // physical row -> user row
    std::vector<int32_t> u2p;      // user row -> physical row
    std::vector<int32_t> p2l;      // physical row -> logical position
    std::vector<int64_t> lvl_ptr;  // physical row range of every level
    HostEll A;                     // all entries, physical columns sorted
    HostEll L;                     // strictly lower (logical) entries, sorted by logical column
    HostEll U;                     // strictly upper (logical) entries
    std::vector<int64_t> u_from_l; // position in L of the transposed entry of each U slot (-1 pad)
    std::vector<double> adiag;     // a_ii per physical row
    // position in the caller's CSR of every ELL slot (-1 padding) and of every
    // diagonal, so that new values of the same pattern can be scattered in
    std::vector<int32_t> a_src, l_src, d_src;
};

// Builds the layout; returns an empty string on success, else the reason.
// block_rows > 0 (block-Jacobi IC(0)): natural order, and L / U hold only
// couplings inside a block of block_rows consecutive rows (A keeps every
// entry).  When every such coupling joins consecutive rows (tridiagonal
// blocks) there is one level and bj_scan is set; otherwise the levels are
// the chains of in-block couplings and the ordinary level-scheduled sweeps
// apply the block-diagonal factor.
std::string build_layout(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
                         const int32_t *colors, int64_t block_rows, HostLayout &out);

// Order in which row tiles of `tile_rows` rows are handed to blocks, for the
// whole row range and for every level.  Rows are grouped in segments of equal
// (level, colour); a tile's key is the eighth of its segment that holds its
// first row, and tiles are ordered by key (stably).  Blocks are remapped so
// that each XCD takes one contiguous eighth of the order: it then works on
// the same spatial eighth of every colour, whose neighbours lie in the same
// eighth of the other colours, so gathered vectors are fetched into one XCD's
// L2 instead of several.  `lvl_off[l]` is the start of level l's order.
// With sub > 1 (sub_full for the whole range, sub_lvl inside the levels) each
// eighth is walked in sub parts, every colour's share of a part together, so
// that the neighbours a part gathers from the other colours are still in the
// XCD's L2 when the next colour of that part needs them.
void tile_orders(const HostLayout &H, const int32_t *colors, int tile_rows, std::vector<int32_t> &full,
                 std::vector<int32_t> &lvl, std::vector<int64_t> &lvl_off, int sub_full = 1, int sub_lvl = 1);
// parts per eighth of the whole-range order: 16 on grids whose gathered
// vectors outgrow the caches (measured at 256^3: FP64 SpMV 442 -> 357 us,
// FP32 174 -> 164 us; no gain at 128^3 or on the 4.1M-row Q1 matrix, and
// none inside the sweep levels)
inline int tile_parts(int64_t n) { return n > (int64_t(1) << 22) ? 16 : 1; }

// Class-aligned copy of a sliced-ELL matrix for the iteration kernels.  In
// every 64-row slice the distinct offsets col - row of its entries, ascending,
// become the slots: slot k of the slice holds, for each row, the entry at
// column row + soff[sptr[s] / 64 + k], or nothing (value 0).  Within a row
// the slots are in ascending physical column order (for A, whose sorted
// layout has that order too, a row's dot product adds the same terms in the
// same order, plus exact zeros).  src[e] is the sorted-layout position of
// class entry e (-1: none).
// Returns false when a slice would need more than max_width slots or the
// copy would exceed 5/4 of the sorted layout's entries.
bool ell_classes(const HostEll &E, int64_t n, int max_width, std::vector<int64_t> &sptr, std::vector<int32_t> &soff,
                 std::vector<int64_t> &src);

// Sampling method A: slot of iteration i (>= 1) for m slots, and the table of
// slots (or -1) for iterations 0..maxit.
int sampling_slot(int64_t i, int m);
void sampling_table(int m, int64_t maxit, std::vector<int32_t> &slot_of_iter);

// Small dense kernels of the host side (own implementations).
void jacobi_eigh(int k, std::vector<double> &a, std::vector<double> &w, std::vector<double> &V);
bool cholesky_inverse(int k, const std::vector<double> &C, std::vector<double> &Cinv);
// G t = lambda B t for symmetric G and SPD B (k x k, column-major): B = R R^T,
// eigenpairs of R^{-1} G R^{-T} (Jacobi), t = R^{-T} v, so T^T B T = I.
// Eigenvalues ascending in w, vectors in the columns of T.  False when B is
// not positive definite.
bool generalized_eigh(int k, const std::vector<double> &G, const std::vector<double> &B, std::vector<double> &w,
                      std::vector<double> &T);
void tridiag_extremes(int k, const double *alpha, const double *beta, double *tmin, double *tmax);

} // namespace esd
