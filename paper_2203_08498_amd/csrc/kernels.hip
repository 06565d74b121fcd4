// gfx950 kernels of the esd library.
//
// Row kernels use 256-thread blocks; a block walks a contiguous run of
// 256-row tiles, and block ids are remapped so that each of the eight XCDs
// (which receive hardware blocks round-robin) owns one contiguous eighth of
// the rows.  Matrices are sliced-ELL with slice height 64, so the 64 lanes of
// a wavefront read 64 consecutive values / column indices per entry slot.
// Padding slots point at column n, and every vector that is gathered has a
// zero at index n.
//
// Reductions are deterministic and need no cross-XCD fences: a reducing kernel
// reduces its values per block (wavefront butterflies, then LDS in wavefront
// order) and stores one row of partials per block; the kernel boundary makes
// them visible to every XCD, and a one-block finalize kernel sums the rows in
// a fixed order and runs the scalar step (alpha, beta, the coarse solve, the
// stop test) on the device.
#include <algorithm>
#include <cfloat>

#include "kernels.h"

namespace esd {
namespace {

__device__ __forceinline__ int xcd_block() {
    const int b = blockIdx.x, G = gridDim.x;
    if (G >= 16 && (G & 7) == 0) return (b & 7) * (G >> 3) + (b >> 3);
    return b;
}

struct Tiles {
    int t0, t1;
};

// Tiles [t0, t1) of the order for this block: the nt tiles split as evenly
// as possible over the grid's positions (xcd_block), so that every XCD gets
// an eighth of them whatever nt / gridDim is.
__device__ __forceinline__ Tiles my_tiles(int rows) {
    const int nt = (rows + kBlock - 1) / kBlock;
    const int64_t G = gridDim.x, pos = xcd_block();
    return {(int)(pos * nt / G), (int)((pos + 1) * nt / G)};
}

// Block reduction of NV doubles; thread k < NV stores the block total at
// part[blockIdx.x * stride + k].
template <int NV>
__device__ __forceinline__ void block_partials(double (&v)[NV], double *part, int stride) {
    __shared__ double lds[kBlock / 64][NV];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) lds[wid][k] = x;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < NV; k += kBlock) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) s += lds[w][k];
        part[(size_t)blockIdx.x * stride + k] = s;
    }
}

// One partial table for the finalize kernels: columns [c0, c0 + nc) of an
// nblk x stride row-major table, summed into tot[0 .. nc) (shared or global).
struct ColTab {
    const double *part;
    int nblk, stride, c0, nc;
    double *tot;
};

// Column sums of NTAB <= 4 tables at once; must be called by all kFinThreads
// threads.  The threads are split into equal slots, one per table.  In a slot
// of NT threads, thread t handles column t % p2 (p2 = nc rounded up to a power
// of two) and rows congruent to t / p2 modulo NT / p2, with 16 loads in flight;
// lanes of one column are then added by shuffles in a fixed pattern and the
// slot's waves through LDS, always in the same order (deterministic).
template <int NTAB>
__device__ void fin_colsums(const ColTab (&tab)[NTAB]) {
    constexpr int SLOTS = NTAB <= 1 ? 1 : (NTAB <= 2 ? 2 : 4);
    constexpr int NT = kFinThreads / SLOTS;
    constexpr int WPS = NT / 64;
    static_assert(NTAB >= 1 && NTAB <= 4, "at most four tables");
    __shared__ double red[kFinThreads / 64][64];
    const int slot = threadIdx.x / NT, t = threadIdx.x % NT;
    const int lane = threadIdx.x & 63;
    ColTab T = tab[0];
#pragma unroll
    for (int q = 1; q < NTAB; ++q)
        if (slot == q) T = tab[q];
    const bool active = slot < NTAB;
    int p2 = 1;
    while (p2 < T.nc) p2 <<= 1;
    const int groups = NT / p2, k = t % p2, g = t / p2;
    double acc = 0.0;
    if (active && k < T.nc) {
        for (int j0 = g; j0 < T.nblk; j0 += 16 * groups) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int j = j0 + u * groups;
                v[u] = (j < T.nblk) ? T.part[(size_t)j * T.stride + T.c0 + k] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 16; u += 2) v[u] += v[u + 1];
#pragma unroll
            for (int u = 0; u < 16; u += 4) v[u] += v[u + 2];
            acc += (v[0] + v[4]) + (v[8] + v[12]);
        }
    }
    // lanes l and l ^ off hold the same column for off >= p2
    for (int off = 32; off >= p2; off >>= 1) acc += __shfl_xor(acc, off, 64);
    red[threadIdx.x >> 6][lane] = acc;
    __syncthreads();
    if (active && t < T.nc) {
        double sum = 0.0;
        if (p2 <= 64) {
            for (int w = 0; w < WPS; ++w) sum += red[slot * WPS + w][t];
        } else {
            for (int q = 0; q < groups; ++q) {
                const int u = q * p2 + t;
                sum += red[slot * WPS + (u >> 6)][u & 63];
            }
        }
        T.tot[t] = sum;
    }
    __syncthreads();
}

__device__ __forceinline__ void fin_colsum(const double *part, int nblk, int stride, int c0, int nc, double *tot) {
    const ColTab tab[1] = {{part, nblk, stride, c0, nc, tot}};
    fin_colsums<1>(tab);
}

// ------------------------------------------------------------------------
// per-iteration kernels
// ------------------------------------------------------------------------

template <bool NT, typename T> __device__ __forceinline__ T ld_slot(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename T> __device__ __forceinline__ void st_slot(T v, T *p) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Columns of W, AW or Y are read once per iteration: non-temporal loads keep
// them from evicting the vectors that the next launches read again.
template <typename T> __device__ __forceinline__ T ld_col(const T *p) { return __builtin_nontemporal_load(p); }

template <bool NT, typename T, int K>
__device__ __forceinline__ void ell_chunk_ld(const Ell<T> &M, int64_t base, int w, int k0, int i, int n, int (&c)[K],
                                             T (&a)[K]) {
    const int lane = i & 63;
    if (M.soff) {
        int off[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k0 + k < w) {
                a[k] = ld_slot<NT>(&M.val[base + (int64_t)(k0 + k) * 64 + lane]);
                off[k] = M.soff[(base >> 6) + k0 + k];
            } else {
                a[k] = T(0);
                off[k] = n; // clamps to n
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) c[k] = min(max(i + off[k], 0), n);
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k0 + k < w) {
                const int64_t pos = base + (int64_t)(k0 + k) * 64 + lane;
                a[k] = ld_slot<NT>(&M.val[pos]);
                c[k] = ld_slot<NT>(&M.col[pos]);
            } else {
                a[k] = T(0);
                c[k] = n;
            }
        }
    }
}

// Loads the columns and values of slots k0 .. k0+K-1 of row i (slice starting
// at entry `base`, width w > k0); slots past w get column n and value 0.  No
// loaded value is used before all loads of the chunk are issued.  Class-
// aligned layout: column = row + offset of the slot, clamped into [0, n]; a
// row without an entry in a slot holds the value 0 there, so whatever finite
// value the clamped column gathers is multiplied by zero.  M.nt: the slot
// loads are non-temporal, so the matrix streams past the caches and they keep
// the gathered vectors instead.
template <typename T, int K = 8>
__device__ __forceinline__ void ell_chunk(const Ell<T> &M, int64_t base, int w, int k0, int i, int n, int (&c)[K],
                                          T (&a)[K]) {
    if (M.nt) ell_chunk_ld<true>(M, base, w, k0, i, n, c, a);
    else ell_chunk_ld<false>(M, base, w, k0, i, n, c, a);
}

// Start entry and width of row i's slice.  U: the caller guarantees that all
// active lanes of the wavefront lie in the same 64-row slice (the row range
// starts on a slice boundary), so the slice is read once per wavefront as a
// scalar and the per-slot column offsets become scalar loads too.
template <bool U, typename T>
__device__ __forceinline__ void ell_slice(const Ell<T> &M, int i, int64_t &base, int &w) {
    const int s = U ? __builtin_amdgcn_readfirstlane(i >> 6) : (i >> 6);
    base = M.sptr[s];
    w = (int)((M.sptr[s + 1] - base) >> 6);
}

// sum_k val_k * g(col_k) over one sliced-ELL row, eight slots at a time: the
// slot loads, then the eight gathers, then the products.
template <bool U = false, typename T, typename G>
__device__ __forceinline__ T ell_dot(const Ell<T> &M, int i, int n, G g) {
    int64_t base;
    int w;
    ell_slice<U>(M, i, base, w);
    T sum = T(0);
    for (int k0 = 0; k0 < w; k0 += 8) {
        int c[8];
        T a[8];
        ell_chunk(M, base, w, k0, i, n, c, a);
        T v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = g(c[k]);
#pragma unroll
        for (int k = 0; k < 8; ++k) sum += a[k] * v[k];
    }
    return sum;
}

// two right-hand sides sharing the matrix loads: (A x, A y)
template <bool U = false, typename T, typename G1, typename G2>
__device__ __forceinline__ void ell_dot2(const Ell<T> &M, int i, int n, G1 g1, G2 g2, T &s1, T &s2) {
    int64_t base;
    int w;
    ell_slice<U>(M, i, base, w);
    s1 = T(0);
    s2 = T(0);
    for (int k0 = 0; k0 < w; k0 += 8) {
        int c[8];
        T a[8];
        ell_chunk(M, base, w, k0, i, n, c, a);
        T v1[8], v2[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            v1[k] = g1(c[k]);
            v2[k] = g2(c[k]);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            s1 += a[k] * v1[k];
            s2 += a[k] * v2[k];
        }
    }
}

template <typename T, bool POW, bool PG>
__global__ __launch_bounds__(kBlock) void k_spmv_it(SpmvIt<T> a) {
    Scal *S = a.S;
    if (S->done) return;
    const int iter = S->iter;
    const bool first = (iter == 0);
    const T beta = (first || PG) ? T(0) : (T)S->beta;
    const T vs = POW ? (T)S->vscale : T(0);
    int slot = -1;
    if (a.slot_table && iter >= 1) slot = a.slot_table[S->sample_base + iter];
    constexpr int NV = 1 + (POW ? 1 : 0);
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    const int n = a.n;
    const T *z = a.z, *po = a.pold, *vo = a.vold, *pg = a.pnew;
    const Tiles tl = my_tiles(n);
    for (int t = tl.t0; t < tl.t1; ++t) {
        const int i = (a.tmap ? a.tmap[t] : t) * kBlock + threadIdx.x;
        if (i >= n) continue;
        T sum, vsum = T(0), pi;
        if constexpr (PG) {
            if constexpr (POW) ell_dot2<true>(a.A, i, n, [&](int c) { return pg[c]; }, [&](int c) { return vo[c]; }, sum, vsum);
            else sum = ell_dot<true>(a.A, i, n, [&](int c) { return pg[c]; });
            pi = pg[i];
        } else {
            if (first) {
                if constexpr (POW)
                    ell_dot2<true>(a.A, i, n, [&](int c) { return z[c]; }, [&](int c) { return vo[c]; }, sum, vsum);
                else sum = ell_dot<true>(a.A, i, n, [&](int c) { return z[c]; });
            } else {
                if constexpr (POW)
                    ell_dot2<true>(a.A, i, n, [&](int c) { return z[c] + beta * po[c]; }, [&](int c) { return vo[c]; },
                             sum, vsum);
                else sum = ell_dot<true>(a.A, i, n, [&](int c) { return z[c] + beta * po[c]; });
            }
            pi = first ? z[i] : z[i] + beta * po[i];
            a.pnew[i] = pi;
        }
        a.q[i] = sum;
        acc[0] += (double)pi * (double)sum;
        if constexpr (POW) {
            const T vn = vsum * vs;
            a.vnew[i] = vn;
            acc[1] += (double)vn * (double)vn;
        }
        if (slot >= 0)
            a.slots[(size_t)slot * n + i] = (a.xbase ? a.xbase[i] : 0.0) + S->xscale * (double)a.xit[i];
    }
    block_partials<NV>(acc, a.part, NV);
}

// x += alpha p, r -= alpha q, ||r||^2; rows of the first sweep level (i < l0)
// also take y = r / l_ii and ||y||^2 (the level-0 forward sweep fused here);
// MT > 0: also G^T r of the new residual (G column-major, a.m <= MT columns,
// one coalesced load per column).  XNT / GNT: x / the columns of G are
// loaded (and x stored) non-temporally.
template <typename T, int MT, bool XNT, bool GNT>
__global__ __launch_bounds__(kBlock) void k_update_it(UpdIt<T> a) {
    Scal *S = a.S;
    if (S->done) return;
    const T ta = (T)S->alpha;
    constexpr int NV = MT > 0 ? 2 + MT : 2;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    const int n = a.n;
    const Tiles tl = my_tiles(n);
    for (int t = tl.t0; t < tl.t1; ++t) {
        const int i = (a.tmap ? a.tmap[t] : t) * kBlock + threadIdx.x;
        if (i >= n) continue;
        T g[MT > 0 ? MT : 1];
        if constexpr (MT > 0) {
            // columns past m re-read column m - 1 (unused sums): no condition
            // on the loads, so they are all in flight together
#pragma unroll
            for (int k = 0; k < MT; ++k) g[k] = ld_slot<GNT>(&a.G[(size_t)(k < a.m ? k : a.m - 1) * n + i]);
        }
        st_slot<XNT>(ld_slot<XNT>(&a.x[i]) + ta * a.p[i], &a.x[i]);
        const T ri = a.r[i] - ta * a.q[i];
        a.r[i] = ri;
        acc[0] += (double)ri * (double)ri;
        if (i < a.l0) {
            const T yi = ri * a.dinv[i];
            a.y[i] = yi;
            acc[1] += (double)yi * (double)yi;
        }
        if constexpr (MT > 0) {
#pragma unroll
            for (int k = 0; k < MT; ++k) acc[2 + k] += (double)g[k] * (double)ri;
        }
    }
    block_partials<NV>(acc, a.part, NV);
}

// FP32 vector update (plain / projected form) with two rows per thread, tiles
// t and t + 1 of the block's range: all loads of both rows first.  A 4-byte
// row moves half the bytes of an FP64 one per load instruction, so one row
// per thread leaves the FP32 streams short of loads in flight.  Same
// arithmetic per row as k_update_it.
template <typename T, int MT, bool XNT, bool GNT>
__global__ __launch_bounds__(kBlock) void k_update_it2(UpdIt<T> a) {
    Scal *S = a.S;
    if (S->done) return;
    const T ta = (T)S->alpha;
    constexpr int NV = MT > 0 ? 2 + MT : 2;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    const int n = a.n;
    const Tiles tl = my_tiles(n);
    for (int t = tl.t0; t < tl.t1; t += 2) {
        int i[2];
        bool h[2];
        T qv[2], pv[2], xv[2], rv[2], dv[2];
        T g[2][MT > 0 ? MT : 1];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int tt = t + u;
            i[u] = tt < tl.t1 ? (a.tmap ? a.tmap[tt] : tt) * kBlock + threadIdx.x : n;
            h[u] = i[u] < n;
            qv[u] = h[u] ? a.q[i[u]] : T(0);
            pv[u] = h[u] ? a.p[i[u]] : T(0);
            xv[u] = h[u] ? ld_slot<XNT>(&a.x[i[u]]) : T(0);
            rv[u] = h[u] ? a.r[i[u]] : T(0);
            dv[u] = (h[u] && i[u] < a.l0) ? a.dinv[i[u]] : T(0);
            if constexpr (MT > 0) {
                const int iu = h[u] ? i[u] : 0;
#pragma unroll
                for (int k = 0; k < MT; ++k) g[u][k] = ld_slot<GNT>(&a.G[(size_t)(k < a.m ? k : a.m - 1) * n + iu]);
            }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (!h[u]) continue;
            st_slot<XNT>(xv[u] + ta * pv[u], &a.x[i[u]]);
            const T ri = rv[u] - ta * qv[u];
            a.r[i[u]] = ri;
            acc[0] += (double)ri * (double)ri;
            if (i[u] < a.l0) {
                const T yi = ri * dv[u];
                a.y[i[u]] = yi;
                acc[1] += (double)yi * (double)yi;
            }
            if constexpr (MT > 0) {
#pragma unroll
                for (int k = 0; k < MT; ++k) acc[2 + k] += (double)g[u][k] * (double)ri;
            }
        }
    }
    block_partials<NV>(acc, a.part, NV);
}

// s = W^T v, W row-major n x m; P = next power of two >= m.  Lane l of a
// wavefront takes column l % P of rows l / P, l / P + 64 / P, ...; blocks of
// kTsBlock threads keep the partial table (one row of P per block) short.
template <typename T, int P>
__global__ __launch_bounds__(kTsBlock) void k_tsdot_rm(TsDot<T> a) {
    if (a.S && a.S->done) return;
    constexpr int RPW = 64 / P;      // rows per wavefront step
    constexpr int WAVES = kTsBlock / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int k = lane % P, ro = lane / P;
    const int m = a.m, n = a.n;
    const int G = gridDim.x;
    constexpr int STEP = WAVES * RPW;
    // rows split evenly over the grid's positions (every XCD an eighth)
    const int r0 = (int)((int64_t)xcd_block() * n / G), r1 = (int)((int64_t)(xcd_block() + 1) * n / G);
    double acc = 0.0;
    if (k < m) {
#pragma unroll 4
        for (int r = r0 + wid * RPW + ro; r < r1; r += STEP)
            acc += (double)ld_col(&a.Wrm[(size_t)r * m + k]) * (double)a.v[r];
    }
#pragma unroll
    for (int off = 32; off >= P; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __shared__ double lds[WAVES][P];
    if (ro == 0) lds[wid][k] = acc;
    __syncthreads();
    if ((int)threadIdx.x < P) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) s += lds[w][threadIdx.x];
        a.part[(size_t)blockIdx.x * P + threadIdx.x] = s;
    }
}

__global__ void k_to_rowmajor(int n, int m, const double *W, double *Wrm, float *Wrm32) {  // also used for AW
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < m; ++k) {
        const double v = W[(size_t)k * n + i];
        Wrm[(size_t)i * m + k] = v;
        if (Wrm32) Wrm32[(size_t)i * m + k] = (float)v;
    }
}

template <typename T, bool SC>
__device__ __forceinline__ T add_coarse(const Sweep<T> &a, int i, T zi) {
    if constexpr (!SC) {
        return zi;
    } else {
        double s = (double)zi;
        for (int k = 0; k < a.m; ++k) s += (double)a.W[(size_t)k * a.n + i] * a.S->u[k];
        return (T)s;
    }
}

// The sweep launches are latency-bound (one dependent round trip per row, a
// level of 0.26-0.79 M rows takes more than one round of resident waves), so
// both ask for 8 waves per SIMD (at most 64 VGPRs; the FP64 forward kernel
// needed 66 without the bound).
template <typename T, bool LAST, bool SC>
__global__ __launch_bounds__(kBlock, 8) void k_fwd(Sweep<T> a) {
    if (a.S->done) return;
    double acc[1] = {0.0};
    const T *y = a.y;
    const bool aligned = (a.r0 & 63) == 0; // wavefronts then never straddle a slice
    const Tiles tl = my_tiles(a.r1 - a.r0);
    for (int t = tl.t0; t < tl.t1; ++t) {
        const int i = a.r0 + (a.tmap ? a.tmap[t] : t) * kBlock + threadIdx.x;
        if (i >= a.r1) continue;
        const T ri = a.r[i];
        const auto gy = [&](int c) { return y[c]; };
        const T s = ri - (aligned ? ell_dot<true>(a.M, i, a.n, gy) : ell_dot<false>(a.M, i, a.n, gy));
        const T yi = s * a.dinv[i];
        if constexpr (!SC) acc[0] += (double)yi * (double)yi;
        if constexpr (!LAST) {
            a.y[i] = yi;
        } else {
            // no logically-later neighbour: the backward solve of this row is immediate
            const T zi = yi * a.dinv[i];
            a.z[i] = zi;
            if constexpr (SC) {
                const T zs = add_coarse<T, SC>(a, i, zi);
                a.zsc[i] = zs;
                acc[0] += (double)ri * (double)zs;
            }
        }
    }
    if constexpr (!SC || LAST) block_partials<1>(acc, a.part, 1);
}

template <typename T, bool SC>
__global__ __launch_bounds__(kBlock, 8) void k_bwd(Sweep<T> a) {
    if (a.S->done) return;
    double acc[1] = {0.0};
    const T *z = a.z;
    const bool aligned = (a.r0 & 63) == 0; // wavefronts then never straddle a slice
    const Tiles tl = my_tiles(a.r1 - a.r0);
    for (int t = tl.t0; t < tl.t1; ++t) {
        const int i = a.r0 + (a.tmap ? a.tmap[t] : t) * kBlock + threadIdx.x;
        if (i >= a.r1) continue;
        const auto gz = [&](int c) { return z[c]; };
        const T s = a.y[i] - (aligned ? ell_dot<true>(a.M, i, a.n, gz) : ell_dot<false>(a.M, i, a.n, gz));
        const T zi = s * a.dinv[i];
        a.z[i] = zi;
        if constexpr (SC) {
            const T zs = add_coarse<T, SC>(a, i, zi);
            a.zsc[i] = zs;
            acc[0] += (double)a.r[i] * (double)zs;
        }
    }
    if constexpr (SC) block_partials<1>(acc, a.part, 1);
}

// Two rows per thread, from tiles t and t + 1 of the block's range: the slot
// loads of both rows, then both gathers, then the products.  A wavefront has
// twice the loads in flight, so a level with more tiles than one round of
// resident wavefronts finishes in about one round of dependent round trips.
// Each row's sum is formed as ell_dot forms it.  h0 / h1: the row exists.
template <bool U, typename T, typename G>
__device__ __forceinline__ void ell_dot_pair(const Ell<T> &M, int i0, bool h0, int i1, bool h1, int n, G g, T &s0,
                                             T &s1) {
    int64_t b0 = 0, b1 = 0;
    int w0 = 0, w1 = 0;
    if (h0) ell_slice<U>(M, i0, b0, w0);
    if (h1) ell_slice<U>(M, i1, b1, w1);
    s0 = T(0);
    s1 = T(0);
    // chunks of 4 slots (the sweeps' triangles are narrow) keep both rows
    // within the 64 registers of 8 wavefronts per SIMD
    constexpr int K = 4;
    const int w = max(w0, w1);
    for (int k0 = 0; k0 < w; k0 += K) {
        int c0[K], c1[K];
        T a0[K], a1[K];
        ell_chunk<T, K>(M, b0, w0, k0, i0, n, c0, a0); // w0 = 0: value 0, column n
        ell_chunk<T, K>(M, b1, w1, k0, i1, n, c1, a1);
        T v0[K], v1[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            v0[k] = g(c0[k]);
            v1[k] = g(c1[k]);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            s0 += a0[k] * v0[k];
            s1 += a1[k] * v1[k];
        }
    }
}

// rows i0 (tile t) and i1 (tile t + 1, if the range has it) of the thread
struct RowPair {
    int i0, i1;
    bool h0, h1;
};
template <typename T> __device__ __forceinline__ RowPair row_pair(const Sweep<T> &a, int t, int t1) {
    RowPair q;
    q.i0 = a.r0 + (a.tmap ? a.tmap[t] : t) * kBlock + threadIdx.x;
    q.i1 = (t + 1 < t1) ? a.r0 + (a.tmap ? a.tmap[t + 1] : t + 1) * kBlock + threadIdx.x : a.r1;
    q.h0 = q.i0 < a.r1;
    q.h1 = q.i1 < a.r1;
    return q;
}

// forward sweep of a level that is not the last one, two rows per thread
// (same arithmetic per row as k_fwd); RHO: reduce ||y||^2 (rho without
// subspace correction).  6 wavefronts per SIMD (at most 80 registers) hold
// 12 rows' loads in flight
template <typename T, bool RHO>
__global__ __launch_bounds__(kBlock, 6) void k_fwd2(Sweep<T> a) {
    if (a.S->done) return;
    double acc[1] = {0.0};
    const T *y = a.y;
    const bool aligned = (a.r0 & 63) == 0;
    const Tiles tl = my_tiles(a.r1 - a.r0);
    const auto gy = [&](int c) { return y[c]; };
    for (int t = tl.t0; t < tl.t1; t += 2) {
        const RowPair q = row_pair(a, t, tl.t1);
        const T ri0 = q.h0 ? a.r[q.i0] : T(0), ri1 = q.h1 ? a.r[q.i1] : T(0);
        const T d0 = q.h0 ? a.dinv[q.i0] : T(0), d1 = q.h1 ? a.dinv[q.i1] : T(0);
        T s0, s1;
        if (aligned) ell_dot_pair<true>(a.M, q.i0, q.h0, q.i1, q.h1, a.n, gy, s0, s1);
        else ell_dot_pair<false>(a.M, q.i0, q.h0, q.i1, q.h1, a.n, gy, s0, s1);
        if (q.h0) {
            const T yi = (ri0 - s0) * d0;
            a.y[q.i0] = yi;
            if constexpr (RHO) acc[0] += (double)yi * (double)yi;
        }
        if (q.h1) {
            const T yi = (ri1 - s1) * d1;
            a.y[q.i1] = yi;
            if constexpr (RHO) acc[0] += (double)yi * (double)yi;
        }
    }
    if constexpr (RHO) block_partials<1>(acc, a.part, 1);
}

// backward sweep of a level, two rows per thread (same arithmetic per row as
// k_bwd); SC: subspace correction, z + W u and rho = (r, z + W u) as in k_bwd
template <typename T, bool SC>
__global__ __launch_bounds__(kBlock, 6) void k_bwd2(Sweep<T> a) {
    if (a.S->done) return;
    double acc[1] = {0.0};
    const T *z = a.z;
    const bool aligned = (a.r0 & 63) == 0;
    const Tiles tl = my_tiles(a.r1 - a.r0);
    const auto gz = [&](int c) { return z[c]; };
    for (int t = tl.t0; t < tl.t1; t += 2) {
        const RowPair q = row_pair(a, t, tl.t1);
        const T y0 = q.h0 ? a.y[q.i0] : T(0), y1 = q.h1 ? a.y[q.i1] : T(0);
        const T d0 = q.h0 ? a.dinv[q.i0] : T(0), d1 = q.h1 ? a.dinv[q.i1] : T(0);
        T s0, s1;
        if (aligned) ell_dot_pair<true>(a.M, q.i0, q.h0, q.i1, q.h1, a.n, gz, s0, s1);
        else ell_dot_pair<false>(a.M, q.i0, q.h0, q.i1, q.h1, a.n, gz, s0, s1);
        if (q.h0) {
            const T zi = (y0 - s0) * d0;
            a.z[q.i0] = zi;
            if constexpr (SC) {
                const T zs = add_coarse<T, SC>(a, q.i0, zi);
                a.zsc[q.i0] = zs;
                acc[0] += (double)a.r[q.i0] * (double)zs;
            }
        }
        if (q.h1) {
            const T zi = (y1 - s1) * d1;
            a.z[q.i1] = zi;
            if constexpr (SC) {
                const T zs = add_coarse<T, SC>(a, q.i1, zi);
                a.zsc[q.i1] = zs;
                acc[0] += (double)a.r[q.i1] * (double)zs;
            }
        }
    }
    if constexpr (SC) block_partials<1>(acc, a.part, 1);
}

// Block-Jacobi z = M^{-1} r with tridiagonal blocks, one wavefront per block,
// lane t holding rows t R .. t R + R - 1 of it.  Forward y_k = (r_k - l_k
// y_{k-1}) / d_k and backward z_k = (y_k - l_{k+1} z_{k+1}) / d_k are
// first-order linear recurrences: every lane composes the affine maps of its
// rows, an inclusive 64-lane scan of the compositions (towards higher lanes
// for the forward sweep, towards lower lanes for the backward one) gives the
// value entering each lane's rows, and the lane then runs the substitution
// over its rows from that value, so every row is computed by the sequential
// sweep's own formula.  y stays in registers between the two sweeps.  Rows
// past the block's end carry d = l = r = 0 and hence y = z = 0.
template <typename T, int R> struct alignas(sizeof(T) * R) BjPack {
    T v[R];
};

// the lane's R rows of a vector (zero past the block end).  Blocks of a
// multiple of R rows start every lane's rows on an R-row boundary: one aligned
// R-wide load (the vectors hold 64 entries past n, so the last block's
// partial group stays in bounds and its rows past the end are zeroed).
template <typename T, int R>
__device__ __forceinline__ void bj_load(const T *src, int r0, int k0, int len, bool vec, T (&v)[R]) {
    if (vec && k0 < len) {
        const BjPack<T, R> q = *reinterpret_cast<const BjPack<T, R> *>(src + r0 + k0);
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = (k0 + j < len) ? q.v[j] : T(0);
    } else {
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = (k0 + j < len) ? src[r0 + k0 + j] : T(0);
    }
}
// entry n of a vector must stay zero (gathers of padding slots read it): only
// whole groups are written as one R-wide store
template <typename T, int R>
__device__ __forceinline__ void bj_store(T *dst, int r0, int k0, int len, bool vec, const T (&v)[R]) {
    if (vec && k0 + R <= len) {
        BjPack<T, R> q;
#pragma unroll
        for (int j = 0; j < R; ++j) q.v[j] = v[j];
        *reinterpret_cast<BjPack<T, R> *>(dst + r0 + k0) = q;
    } else {
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (k0 + j < len) dst[r0 + k0 + j] = v[j];
    }
}

// one block's z = M^{-1} r on registers; adds ||y||^2 of the lane's rows to ysq
template <typename T, int R>
__device__ __forceinline__ void bj_block(int lane, const T (&l)[R], const T (&di)[R], const T (&rr)[R], T (&zr)[R],
                                         double &ysq) {
    // forward: y leaving the lane's rows = A * (y entering) + C
    T A = T(1), C = T(0);
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const T aj = -l[j] * di[j];
        C = aj * C + rr[j] * di[j];
        A = aj * A;
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T Ap = __shfl_up(A, d, 64), Cp = __shfl_up(C, d, 64);
        if (lane >= d) {
            C = A * Cp + C;
            A = A * Ap;
        }
    }
    T yv = __shfl_up(C, 1, 64);
    if (lane == 0) yv = T(0); // l = 0 at the block start: nothing enters
    T y[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
        yv = (rr[j] - l[j] * yv) * di[j];
        y[j] = yv;
        ysq += (double)yv * (double)yv;
    }
    // backward: l_{k+1} of the lane's last row is the next lane's first l
    T lnext = __shfl_down(l[0], 1, 64);
    if (lane == 63) lnext = T(0);
    T E = T(1), G = T(0);
#pragma unroll
    for (int j = R - 1; j >= 0; --j) {
        const T ej = -((j + 1 < R) ? l[j + 1] : lnext) * di[j];
        G = ej * G + y[j] * di[j];
        E = ej * E;
    }
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T Ep = __shfl_down(E, d, 64), Gp = __shfl_down(G, d, 64);
        if (lane + d < 64) {
            G = E * Gp + G;
            E = E * Ep;
        }
    }
    T zv = __shfl_down(G, 1, 64);
    if (lane == 63) zv = T(0);
#pragma unroll
    for (int j = R - 1; j >= 0; --j) {
        zv = (y[j] - ((j + 1 < R) ? l[j + 1] : lnext) * zv) * di[j];
        zr[j] = zv;
    }
}

// wavefront w of the grid takes blocks w, w + (waves in the grid), ...
template <typename T, int R, bool SC>
__global__ __launch_bounds__(kBlock) void k_bj(BjSweep<T> a) {
    if (a.S->done) return;
    const int lane = threadIdx.x & 63;
    const int stride = gridDim.x * (kBlock / 64);
    const bool vec = R > 1 && a.s % R == 0;
    double acc[1] = {0.0};
    for (int blk = blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6); blk < a.nb; blk += stride) {
        const int r0 = blk * a.s;
        const int len = min(a.s, a.n - r0);
        const int k0 = lane * R;
        T l[R], di[R], rr[R], zr[R];
        bj_load<T, R>(a.lsub, r0, k0, len, vec, l);
        bj_load<T, R>(a.dinv, r0, k0, len, vec, di);
        bj_load<T, R>(a.r, r0, k0, len, vec, rr);
        double ysq = 0.0;
        bj_block<T, R>(lane, l, di, rr, zr, ysq);
        if constexpr (!SC) acc[0] += ysq;
        bj_store<T, R>(a.z, r0, k0, len, vec, zr);
        if constexpr (SC) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if (k0 + j < len) {
                    const int p = r0 + k0 + j;
                    double sc = (double)zr[j];
                    for (int q = 0; q < a.m; ++q) sc += (double)a.W[(size_t)q * a.n + p] * a.S->u[q];
                    const T zs = (T)sc;
                    a.zsc[p] = zs;
                    acc[0] += (double)rr[j] * (double)zs;
                }
            }
        }
    }
    block_partials<1>(acc, a.part, 1);
}

// x += alpha p, r -= alpha q, then z = M^{-1} r (block Jacobi) on the updated r
// held in registers: one pass over the block's rows instead of the update
// kernel followed by k_bj.  Partials: column 0 ||r||^2, column 1 ||y||^2.
template <typename T, int R>
__global__ __launch_bounds__(kBlock) void k_update_bj(UpdBj<T> a) {
    Scal *S = a.S;
    if (S->done) return;
    const T ta = (T)S->alpha;
    const int lane = threadIdx.x & 63;
    const int stride = gridDim.x * (kBlock / 64);
    const bool vec = R > 1 && a.s % R == 0;
    double acc[2] = {0.0, 0.0};
    for (int blk = blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6); blk < a.nb; blk += stride) {
        const int r0 = blk * a.s;
        const int len = min(a.s, a.n - r0);
        const int k0 = lane * R;
        T pv[R], qv[R], xv[R], rv[R], l[R], di[R], zr[R];
        bj_load<T, R>(a.p, r0, k0, len, vec, pv);
        bj_load<T, R>(a.q, r0, k0, len, vec, qv);
        bj_load<T, R>(a.x, r0, k0, len, vec, xv);
        bj_load<T, R>(a.r, r0, k0, len, vec, rv);
        bj_load<T, R>(a.lsub, r0, k0, len, vec, l);
        bj_load<T, R>(a.dinv, r0, k0, len, vec, di);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            xv[j] += ta * pv[j];
            rv[j] = rv[j] - ta * qv[j];
            acc[0] += (double)rv[j] * (double)rv[j];
        }
        bj_store<T, R>(a.x, r0, k0, len, vec, xv);
        bj_store<T, R>(a.r, r0, k0, len, vec, rv);
        bj_block<T, R>(lane, l, di, rv, zr, acc[1]);
        bj_store<T, R>(a.z, r0, k0, len, vec, zr);
    }
    block_partials<2>(acc, a.part, 2);
}

// M = I: z = r (+ W u for subspace correction)
template <typename T, bool SC>
__global__ __launch_bounds__(kBlock) void k_copyz(Sweep<T> a) {
    if (a.S->done) return;
    double acc[1] = {0.0};
    const Tiles tl = my_tiles(a.r1 - a.r0);
    for (int t = tl.t0; t < tl.t1; ++t) {
        const int i = a.r0 + (a.tmap ? a.tmap[t] : t) * kBlock + threadIdx.x;
        if (i >= a.r1) continue;
        const T ri = a.r[i];
        a.z[i] = ri;
        const T zs = add_coarse<T, SC>(a, i, ri);
        if constexpr (SC) a.zsc[i] = zs;
        acc[0] += (double)ri * (double)zs;
    }
    block_partials<1>(acc, a.part, 1);
}

// ------------------------------------------------------------------------
// finalize kernels (one block of kFinThreads)
// ------------------------------------------------------------------------

__global__ __launch_bounds__(kFinThreads) void k_fin_alpha(FinAlpha f) {
    Scal *S = f.S;
    __shared__ double tot[2];
    const int done0 = S->done;
    const int t = threadIdx.x;
    double rho = 0.0;
    int iter = 0, hbase = 0;
    if (t == 0) { rho = S->rho; iter = S->iter; hbase = S->hist_base; }
    fin_colsum(f.part, f.nblk, f.stride, 0, f.stride, tot);
    if (done0) return;
    if (t == 0) {
        // (p, q) of the direction the SpMV multiplied: for deflation the
        // projected p, so (p, q) = (p, P^T A p) needs no correction term
        const double alpha = rho / tot[0];
        S->alpha = alpha;
        if (f.hist_alpha) f.hist_alpha[hbase + iter] = alpha;
        if (!isfinite(alpha)) S->done = 3;
        if (f.power) S->vscale = 1.0 / sqrt(tot[1]);
    }
}

__global__ __launch_bounds__(kFinThreads) void k_fin_u(Scal *S, const double *part, int nblk, int stride, int c0,
                                                       int m, const double *Cinv) {
    if (S->done) return;
    __shared__ double tot[64];
    fin_colsum(part, nblk, stride, c0, m, tot);
    const int t = threadIdx.x;
    if (t < m) {
        double acc = 0.0;
        for (int j = 0; j < m; ++j) acc += Cinv[t * m + j] * tot[j];
        S->u[t] = acc;
    }
}

__global__ __launch_bounds__(kFinThreads) void k_fin_rho(FinRho f) {
    Scal *S = f.S;
    __shared__ double tot[3];
    __shared__ double sv[64];
    __shared__ double cinv[64 * 64];
    // every load of the scalar block and of C^{-1} is issued before the
    // partial sums, so their latencies overlap; nothing is written while
    // `done` is set
    const int done0 = S->done;
    const int t = threadIdx.x;
    double rho_old = 0.0, tol2 = 0.0, rr_ref = 0.0, bnorm2 = 0.0, xs = 1.0;
    int iter = 0, maxit = 0, stag = 0, it_ref = 0, hbase = 0, sbase = 0, bnext = 0;
    if (t == 0) {
        rho_old = S->rho; tol2 = S->tol2; rr_ref = S->rr_ref;
        iter = S->iter; maxit = S->maxit; stag = S->stag_window; it_ref = S->it_ref; hbase = S->hist_base;
        if (f.slot_table) { bnorm2 = S->bnorm2; xs = S->xscale; sbase = S->sample_base; bnext = S->bnext; }
    }
    const int mm = f.m * f.m;
    for (int k = t; k < mm; k += kFinThreads) cinv[k] = f.Cinv[k];
    {
        // rho partials, (r, r) and level-0 ||y||^2, and for deflation (AW)^T z
        // in one pass; tot = {(r, r), level-0 ||y||^2, preconditioner rho}
        const int nu = f.init ? 0 : f.nblk_upd;
        if (f.m > 0 && !f.init && f.part_s == f.part_upd && f.c0_s == 2 && f.nblk_s == f.nblk_upd &&
            f.stride_s == f.stride_upd) {
            // (AW)^T z rides on the update partials (columns 2 ..): one table of
            // 2 + m columns, read once with half the threads
            __shared__ double tu[2 + 64];
            const ColTab tab[2] = {{f.part_sweep, f.nsweep, 1, 0, 1, tot + 2},
                                   {f.part_upd, nu, f.stride_upd, 0, 2 + f.m, tu}};
            fin_colsums<2>(tab);
            if (t < 2) tot[t] = tu[t];
            if (t < f.m) sv[t] = tu[2 + t];
            __syncthreads();
        } else if (f.m > 0) {
            const ColTab tab[3] = {{f.part_sweep, f.nsweep, 1, 0, 1, tot + 2},
                                   {f.part_upd, nu, f.stride_upd, 0, 2, tot + 0},
                                   {f.part_s, f.nblk_s, f.stride_s, f.c0_s, f.m, sv}};
            fin_colsums<3>(tab);
        } else {
            const ColTab tab[2] = {{f.part_sweep, f.nsweep, 1, 0, 1, tot + 2},
                                   {f.part_upd, nu, f.stride_upd, 0, 2, tot + 0}};
            fin_colsums<2>(tab);
        }
    }
    if (done0) return;
    if (t < f.m) {
        double acc = 0.0;
        for (int j = 0; j < f.m; ++j) acc += cinv[t * f.m + j] * sv[j];
        S->mu[t] = acc;
    }
    if (t == 0) {
        const double rn = tot[2] + (f.rho_upd ? tot[1] : 0.0);
        if (f.init == 1) {
            S->rho = rn;
            if (!isfinite(rn)) S->done = 3;
            return;
        }
        if (f.init == 2) {
            // residual replacement in a running iteration: the recurrence
            // residual of iteration `iter` was replaced by the true one, so
            // its rho and the beta that joins it to rho_{iter-1} follow the
            // new residual (rho_{iter-1} = rho_old / beta_old)
            const double b = rn * S->beta / rho_old;
            S->beta = b;
            S->rho = rn;
            if (f.hist_beta && iter >= 1) f.hist_beta[hbase + iter - 1] = b;
            if (!isfinite(b)) S->done = 3;
            return;
        }
        const double rr = tot[0];
        const int it = iter + 1;
        S->iter = it;
        S->rr = rr;
        int d = 0;
        if (!(rr <= DBL_MAX) || !isfinite(rn)) d = 3;
        else if (rr <= tol2) d = 1;
        else if (it >= maxit) d = 2;
        else if (stag > 0) {
            // FP32 inner solves: no 10% drop of ||r|| for `stag` iterations once
            // the residual is within 100x of the target (the rounding floor),
            // or for 10 x stag iterations before (CG residual norms may stall
            // for a while early on without the iteration being stuck)
            if (rr < 0.81 * rr_ref) {
                S->rr_ref = rr;
                S->it_ref = it;
            } else if (it - it_ref >= (rr_ref <= 1e4 * tol2 ? stag : 10 * stag)) {
                d = 4;
            }
        }
        S->done = d;
        const double b = rn / rho_old;
        S->beta = b;
        if (f.hist_beta) f.hist_beta[hbase + it - 1] = b;
        S->rho = rn;
        // sampling method B (Sec. 4.3): after the stop test, a sample when the
        // relative residual first reaches tol^{(s+1)/(m+1)} (squares compared);
        // thresholds passed together share the sample, stored in the first
        if (f.slot_table && (d == 0 || d == 2)) {
            const double lhs = rr * xs * xs;
            int take = -1, bn = bnext;
            while (bn < f.nslots && lhs <= S->bthr2[bn] * bnorm2) {
                if (take < 0) take = bn;
                ++bn;
            }
            if (take >= 0) {
                S->bnext = bn;
                f.slot_table[sbase + it] = take;
                S->slot_iter[take] = sbase + it;
            }
        }
    }
}

template <typename T, int MT>
__global__ __launch_bounds__(kBlock) void k_proj(Proj<T> a) {
    const Scal *S = a.S;
    if (S->done) return;
    const bool first = (S->iter == 0);
    const T beta = first ? T(0) : (T)S->beta;
    double mu[MT];
#pragma unroll
    for (int k = 0; k < MT; ++k) mu[k] = (k < a.m) ? S->mu[k] : 0.0;
    const int n = a.n;
    const Tiles tl = my_tiles(n);
    for (int t = tl.t0; t < tl.t1; ++t) {
        const int i = (a.tmap ? a.tmap[t] : t) * kBlock + threadIdx.x;
        if (i >= n) continue;
        // every column load issued before the sums: columns past m re-read
        // column m - 1 (cached) and meet mu = 0, so the loads carry no
        // condition and stay in flight together
        T w[MT];
#pragma unroll
        for (int k = 0; k < MT; ++k) w[k] = ld_col(&a.W[(size_t)(k < a.m ? k : a.m - 1) * n + i]);
        const T zi = a.z[i];
        const T po = first ? T(0) : a.pold[i];
        double s = (double)zi;
#pragma unroll
        for (int k = 0; k < MT; ++k) s -= (double)w[k] * mu[k];
        const T zh = (T)s;
        a.pnew[i] = first ? zh : zh + beta * po;
    }
}

// The projection of k_proj over all rows, with the backward sweep of the
// first level (rows [0, b.r1), b.M = U) done in the same launch: a row of that
// level forms z_i as k_bwd forms it (from z of the later levels, complete) and
// projects it at once.  Needs beta and mu before the launch, so the rho
// finalize runs before it (rho = ||y||^2 is complete after the forward sweep;
// mu comes from the update's Y^T r).  Tiles of the whole range are 256-row
// aligned, so a wavefront's rows share one slice.
template <typename T, int MT>
__global__ __launch_bounds__(kBlock) void k_bwd0_proj(Sweep<T> b, Proj<T> a) {
    const Scal *S = a.S;
    if (S->done) return;
    const bool first = (S->iter == 0);
    const T beta = first ? T(0) : (T)S->beta;
    double mu[MT];
#pragma unroll
    for (int k = 0; k < MT; ++k) mu[k] = (k < a.m) ? S->mu[k] : 0.0;
    const int n = a.n;
    const T *z = b.z;
    const Tiles tl = my_tiles(n);
    for (int t = tl.t0; t < tl.t1; ++t) {
        const int i = (a.tmap ? a.tmap[t] : t) * kBlock + threadIdx.x;
        if (i >= n) continue;
        T w[MT];
#pragma unroll
        for (int k = 0; k < MT; ++k) w[k] = ld_col(&a.W[(size_t)(k < a.m ? k : a.m - 1) * n + i]);
        const T po = first ? T(0) : a.pold[i];
        T zi;
        if (i < b.r1) {
            const T sb = b.y[i] - ell_dot<true>(b.M, i, n, [&](int c) { return z[c]; });
            zi = sb * b.dinv[i];
            b.z[i] = zi;
        } else {
            zi = z[i];
        }
        double s = (double)zi;
#pragma unroll
        for (int k = 0; k < MT; ++k) s -= (double)w[k] * mu[k];
        const T zh = (T)s;
        a.pnew[i] = first ? zh : zh + beta * po;
    }
}

// k_bwd0_proj with two rows per thread (tiles t and t + 1, all loads of both
// rows first) for FP32 vectors of more than kPairTiles tiles, as k_proj2
// does; each row computed as k_bwd0_proj computes it
template <typename T, int MT>
__global__ __launch_bounds__(kBlock) void k_bwd0_proj2(Sweep<T> b, Proj<T> a) {
    const Scal *S = a.S;
    if (S->done) return;
    const bool first = (S->iter == 0);
    const T beta = first ? T(0) : (T)S->beta;
    double mu[MT];
#pragma unroll
    for (int k = 0; k < MT; ++k) mu[k] = (k < a.m) ? S->mu[k] : 0.0;
    const int n = a.n;
    const T *z = b.z;
    const auto gz = [&](int c) { return z[c]; };
    const Tiles tl = my_tiles(n);
    for (int t = tl.t0; t < tl.t1; t += 2) {
        int i[2];
        bool h[2], l0[2];
        T zv[2], pv[2], yv[2], dv[2], wv[2][MT];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int tt = t + u;
            i[u] = tt < tl.t1 ? (a.tmap ? a.tmap[tt] : tt) * kBlock + threadIdx.x : n;
            h[u] = i[u] < n;
            l0[u] = h[u] && i[u] < b.r1;
            const int iu = h[u] ? i[u] : 0;
            pv[u] = (h[u] && !first) ? a.pold[i[u]] : T(0);
            zv[u] = (h[u] && !l0[u]) ? z[i[u]] : T(0);
            yv[u] = l0[u] ? b.y[i[u]] : T(0);
            dv[u] = l0[u] ? b.dinv[i[u]] : T(0);
#pragma unroll
            for (int k = 0; k < MT; ++k) wv[u][k] = ld_col(&a.W[(size_t)(k < a.m ? k : a.m - 1) * n + iu]);
        }
        T s0, s1;
        ell_dot_pair<true>(b.M, i[0], l0[0], i[1], l0[1], n, gz, s0, s1);
        if (l0[0]) {
            zv[0] = (yv[0] - s0) * dv[0];
            b.z[i[0]] = zv[0];
        }
        if (l0[1]) {
            zv[1] = (yv[1] - s1) * dv[1];
            b.z[i[1]] = zv[1];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (!h[u]) continue;
            double s = (double)zv[u];
#pragma unroll
            for (int k = 0; k < MT; ++k) s -= (double)wv[u][k] * mu[k];
            const T zh = (T)s;
            a.pnew[i[u]] = first ? zh : zh + beta * pv[u];
        }
    }
}

// FP32 projection with two rows per thread (tiles t and t + 1), all loads of
// both rows first; same arithmetic per row as k_proj
template <typename T, int MT>
__global__ __launch_bounds__(kBlock) void k_proj2(Proj<T> a) {
    const Scal *S = a.S;
    if (S->done) return;
    const bool first = (S->iter == 0);
    const T beta = first ? T(0) : (T)S->beta;
    double mu[MT];
#pragma unroll
    for (int k = 0; k < MT; ++k) mu[k] = (k < a.m) ? S->mu[k] : 0.0;
    const int n = a.n;
    const Tiles tl = my_tiles(n);
    for (int t = tl.t0; t < tl.t1; t += 2) {
        int i[2];
        bool h[2];
        T zv[2], pv[2], wv[2][MT];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int tt = t + u;
            i[u] = tt < tl.t1 ? (a.tmap ? a.tmap[tt] : tt) * kBlock + threadIdx.x : n;
            h[u] = i[u] < n;
            zv[u] = h[u] ? a.z[i[u]] : T(0);
            pv[u] = (h[u] && !first) ? a.pold[i[u]] : T(0);
            const int iu = h[u] ? i[u] : 0;
#pragma unroll
            for (int k = 0; k < MT; ++k) wv[u][k] = ld_col(&a.W[(size_t)(k < a.m ? k : a.m - 1) * n + iu]);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (!h[u]) continue;
            double s = (double)zv[u];
#pragma unroll
            for (int k = 0; k < MT; ++k) s -= (double)wv[u][k] * mu[k];
            const T zh = (T)s;
            a.pnew[i[u]] = first ? zh : zh + beta * pv[u];
        }
    }
}

__global__ __launch_bounds__(kFinThreads) void k_fin_gen(FinGen f) {
    Scal *S = f.S;
    __shared__ double tot[kMaxNV];
    fin_colsum(f.part, f.nblk, f.stride, 0, f.ncol, tot);
    const int t = threadIdx.x;
    if (f.m > 0) {
        if (t < f.m) {
            if (f.store_svec) S->svec[t] = tot[f.vcol0 + t];
            if (f.coef) {
                double acc = 0.0;
                for (int j = 0; j < f.m; ++j) acc += f.Cinv[t * f.m + j] * tot[f.vcol0 + j];
                f.coef[t] = f.cscale * acc;
            }
        }
    }
    if (t == 0) {
        if (f.out0) *f.out0 = f.scale0 * tot[0];
        if (f.check) {
            S->rr = tot[0];
            if (tot[0] <= S->tol2) S->done = 1;
        }
        if (f.settol >= 0.0) {
            S->bnorm2 = tot[0];
            S->tol2 = f.settol * f.settol * tot[0];
        }
    }
}

// ------------------------------------------------------------------------
// per-solve kernels
// ------------------------------------------------------------------------

__global__ void k_repack(int64_t size, const int64_t *src, const double *from, double *to64, float *to32) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= size) return;
    const int64_t j = src[e];
    const double v = j >= 0 ? from[j] : 0.0;
    to64[e] = v;
    if (to32) to32[e] = (float)v;
}

__global__ void k_gather(int n, const int32_t *idx, const double *src, double *dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}
__global__ void k_scatter(int n, const int32_t *idx, const double *src, double *dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[idx[i]] = src[i];
}
template <typename T> __global__ void k_fill(int n, T *dst, T v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = v;
}
__global__ void k_cast_scale(int n, const double *src, float *dst, double scale) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)(src[i] * scale);
}
__global__ void k_cast(int64_t n, const double *src, float *dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (float)src[i];
}
__global__ void k_add_scaled(int n, double *x, const float *d, double scale) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += scale * (double)d[i];
}
__global__ void k_axpby(int n, const double *f, const double *x, double c, double *b) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = x ? f[i] + c * x[i] : f[i];
}
__global__ void k_sub(int n, const double *a, const double *b, double *dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = a[i] - b[i];
}
__global__ void k_scale_copy(int n, const double *src, double *dst, double scale) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i] * scale;
}

__global__ __launch_bounds__(kBlock) void k_dot(int n, const double *x, const double *y, double *part) {
    double acc[1] = {0.0};
    const Tiles tl = my_tiles(n);
    for (int t = tl.t0; t < tl.t1; ++t) {
        const int i = t * kBlock + threadIdx.x;
        if (i < n) acc[0] += x[i] * y[i];
    }
    block_partials<1>(acc, part, 1);
}

template <int MT>
__global__ __launch_bounds__(kBlock) void k_resid(int n, Ell<double> A, const double *b, const double *x,
                                                  double *t, const double *W, int m, double *part) {
    constexpr int NV = 1 + MT;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    const Tiles tl = my_tiles(n);
    for (int tt = tl.t0; tt < tl.t1; ++tt) {
        const int i = tt * kBlock + threadIdx.x;
        if (i >= n) continue;
        const int lane = i & 63;
        const int64_t base = A.sptr[i >> 6];
        const int w = (int)((A.sptr[(i >> 6) + 1] - base) >> 6);
        double s = 0.0;
        for (int k = 0; k < w; ++k) {
            const int64_t pos = base + (int64_t)k * 64 + lane;
            s += A.val[pos] * x[A.col[pos]];
        }
        const double ri = b[i] - s;
        t[i] = ri;
        acc[0] += ri * ri;
        if constexpr (MT > 0) {
#pragma unroll
            for (int k = 0; k < MT; ++k)
                if (k < m) acc[1 + k] += W[(size_t)k * n + i] * ri;
        }
    }
    block_partials<NV>(acc, part, NV);
}

template <int MT, bool RED>
__global__ __launch_bounds__(kBlock) void k_axpy_cols(int n, double *y, const double *M, int m,
                                                      const double *coef, double sign, double *part) {
    double acc[1] = {0.0};
    double c[MT];
#pragma unroll
    for (int k = 0; k < MT; ++k) c[k] = (k < m) ? sign * coef[k] : 0.0;
    const Tiles tl = my_tiles(n);
    for (int t = tl.t0; t < tl.t1; ++t) {
        const int i = t * kBlock + threadIdx.x;
        if (i >= n) continue;
        double s = y[i];
#pragma unroll
        for (int k = 0; k < MT; ++k)
            if (k < m) s += M[(size_t)k * n + i] * c[k];
        y[i] = s;
        acc[0] += s * s;
    }
    if constexpr (RED) block_partials<1>(acc, part, 1);
}

template <int MT>
__global__ __launch_bounds__(kBlock) void k_tsdot(int n, const double *W, int m, const double *v, double *part) {
    double acc[MT];
#pragma unroll
    for (int k = 0; k < MT; ++k) acc[k] = 0.0;
    const Tiles tl = my_tiles(n);
    for (int t = tl.t0; t < tl.t1; ++t) {
        const int i = t * kBlock + threadIdx.x;
        if (i >= n) continue;
        const double vi = v[i];
#pragma unroll
        for (int k = 0; k < MT; ++k)
            if (k < m) acc[k] += W[(size_t)k * n + i] * vi;
    }
    block_partials<MT>(acc, part, MT);
}

// y = A x in either layout (x holds a zero at index n)
__global__ __launch_bounds__(kBlock) void k_spmv(int n, Ell<double> A, const double *x, double *y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = ell_dot<true>(A, i, n, [&](int c) { return x[c]; });
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_rayleigh(int n, Ell<T> A, const T *v, double *part) {
    double acc[1] = {0.0};
    const Tiles tl = my_tiles(n);
    for (int t = tl.t0; t < tl.t1; ++t) {
        const int i = t * kBlock + threadIdx.x;
        if (i >= n) continue;
        const int lane = i & 63;
        const int64_t base = A.sptr[i >> 6];
        const int w = (int)((A.sptr[(i >> 6) + 1] - base) >> 6);
        double s = 0.0;
        for (int k = 0; k < w; ++k) {
            const int64_t pos = base + (int64_t)k * 64 + lane;
            s += (double)A.val[pos] * (double)v[A.col[pos]];
        }
        acc[0] += (double)v[i] * s;
    }
    block_partials<1>(acc, part, 1);
}

// ------------------------------------------------------------------------
// IC(0) factor, one level of rows at a time
// ------------------------------------------------------------------------

__global__ void k_factor_level(int r0, int r1, int n, Ell<double> L, double *lval, const double *adiag,
                               double *ldiag, int *bad) {
    const int i = r0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= r1) return;
    const int lane = i & 63;
    const int64_t base = L.sptr[i >> 6];
    const int w = (int)((L.sptr[(i >> 6) + 1] - base) >> 6);
    double dsum = 0.0;
    for (int e = 0; e < w; ++e) {
        const int64_t pe = base + (int64_t)e * 64 + lane;
        const int j = L.col[pe];
        if (j >= n) break; // padding sits after the row's entries
        double s = lval[pe];
        const int64_t bj = L.sptr[j >> 6];
        const int wj = (int)((L.sptr[(j >> 6) + 1] - bj) >> 6);
        const int lj = j & 63;
        // entries k of row i that precede j (logically) and also appear in row j
        for (int t = 0; t < e; ++t) {
            const int64_t pt = base + (int64_t)t * 64 + lane;
            const int k = L.col[pt];
            for (int b = 0; b < wj; ++b) {
                const int64_t pb = bj + (int64_t)b * 64 + lj;
                if (L.col[pb] == k) {
                    s -= lval[pt] * lval[pb];
                    break;
                }
            }
        }
        s /= ldiag[j];
        lval[pe] = s;
        dsum += s * s;
    }
    double d = adiag[i] - dsum;
    if (!(d > 0.0)) {
        *bad = 1;
        d = 1.0;
    }
    ldiag[i] = sqrt(d);
}

__global__ void k_finish_factor(int n, const double *ldiag, double *dinv, float *dinv32) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const double d = 1.0 / ldiag[i];
        dinv[i] = d;
        if (dinv32) dinv32[i] = (float)d;
    }
}

// Block-Jacobi factor of tridiagonal blocks, one lane per block walking its
// rows in order: l_k = a_{k,k-1} / d_{k-1}, d_k = sqrt(a_kk - l_k^2) (IC(0) of
// the block, which has no fill to drop).  lval holds a_ij of L's sorted layout
// on entry, whose only entry in row k is column k - 1 (or none).
__global__ void k_factor_bj(int n, int s, Ell<double> L, double *lval, const double *adiag, double *ldiag,
                            double *lsub, float *lsub32, int *bad) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int nb = (n + s - 1) / s;
    if (b >= nb) return;
    const int r0 = b * s, r1 = min(n, r0 + s);
    double dprev = 1.0;
    for (int p = r0; p < r1; ++p) {
        double l = 0.0;
        if (p > r0) {
            const int64_t base = L.sptr[p >> 6];
            const int w = (int)((L.sptr[(p >> 6) + 1] - base) >> 6);
            const int64_t pe = base + (p & 63);
            if (w > 0 && L.col[pe] == p - 1) {
                l = lval[pe] / dprev;
                lval[pe] = l;
            }
        }
        double d = adiag[p] - l * l;
        if (!(d > 0.0)) {
            *bad = 1;
            d = 1.0;
        }
        dprev = sqrt(d);
        ldiag[p] = dprev;
        lsub[p] = l;
        if (lsub32) lsub32[p] = (float)l;
    }
}

__global__ void k_map_values(int64_t cnt, const int32_t *src, const double *val, double *dst, float *dst32) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) {
        const int32_t k = src[i];
        const double v = k >= 0 ? val[k] : 0.0;
        dst[i] = v;
        if (dst32) dst32[i] = (float)v;
    }
}

__global__ void k_gather_u(int64_t cnt, const int64_t *map, const double *lval, double *uval) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) {
        const int64_t s = map[i];
        uval[i] = s >= 0 ? lval[s] : 0.0;
    }
}

// ------------------------------------------------------------------------
// auxiliary-space construction
// ------------------------------------------------------------------------

// AE = A E for m columns (column-major), 16 columns per pass over the row
__global__ __launch_bounds__(kBlock) void k_spmm(int n, Ell<double> A, const double *E, int m, double *AE) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int lane = i & 63;
    const int64_t base = A.sptr[i >> 6];
    const int w = (int)((A.sptr[(i >> 6) + 1] - base) >> 6);
    for (int k0 = 0; k0 < m; k0 += 16) {
        double acc[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) acc[k] = 0.0;
        for (int e = 0; e < w; ++e) {
            const int64_t pos = base + (int64_t)e * 64 + lane;
            const int c = A.col[pos];
            if (c >= n) continue;
            const double av = A.val[pos];
#pragma unroll
            for (int k = 0; k < 16; ++k)
                if (k0 + k < m) acc[k] += av * E[(size_t)(k0 + k) * n + c];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k)
            if (k0 + k < m) AE[(size_t)(k0 + k) * n + i] = acc[k];
    }
}

// y_i = d_i x_i + sum_j M_ij x_j over the stored entries of row i (sorted
// layout; padding skipped): with M = U and d = diag(L) this is L^T x, with
// M = L it is L x.
__global__ __launch_bounds__(kBlock) void k_tri_mul(int n, Ell<double> M, const double *d, const double *x,
                                                    double *y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int lane = i & 63;
    const int64_t base = M.sptr[i >> 6];
    const int w = (int)((M.sptr[(i >> 6) + 1] - base) >> 6);
    double s = d[i] * x[i];
    for (int e = 0; e < w; ++e) {
        const int64_t pos = base + (int64_t)e * 64 + lane;
        const int c = M.col[pos];
        if (c < n) s += M.val[pos] * x[c];
    }
    y[i] = s;
}

typedef double double4_t __attribute__((ext_vector_type(4)));

// Block partial of G = E^T F (E: n x ma, F: n x mb, column-major, ma, mb <= 64)
// with the FP64 matrix cores.  v_mfma_f64_16x16x4: lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; accumulator value r of lane l is D[l/16 + 4r][l%16]
// (checked on gfx950 with an in-bounds layout probe).
// Each of the 4 wavefronts owns up to 4 of the 16 output tiles.
__global__ __launch_bounds__(256) void k_gram_part(int n, const double *E, int ma, const double *F, int mb,
                                                   double *part) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int ta = (ma + 15) / 16, tb = (mb + 15) / 16, ntile = ta * tb;
    const int G = gridDim.x;
    const int chunk = ((n + G - 1) / G + 3) / 4 * 4;
    const int row0 = blockIdx.x * chunk, row1 = min(n, row0 + chunk);
    double4_t acc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = double4_t{0.0, 0.0, 0.0, 0.0};
    const int li = lane & 15, lk = lane >> 4;
    for (int r = row0; r < row1; r += 4) {
        const int row = r + lk;
        const bool ok = row < row1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int tile = wid + 4 * q;
            if (tile >= ntile) break;
            const int a0 = (tile / tb) * 16, b0 = (tile % tb) * 16;
            const int ca = a0 + li, cb = b0 + li;
            const double av = (ok && ca < ma) ? E[(size_t)ca * n + row] : 0.0;
            const double bv = (ok && cb < mb) ? F[(size_t)cb * n + row] : 0.0;
            acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[q], 0, 0, 0);
        }
    }
    double *out = part + (size_t)blockIdx.x * 64 * 64;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int tile = wid + 4 * q;
        if (tile >= ntile) break;
        const int a0 = (tile / tb) * 16, b0 = (tile % tb) * 16;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
            const int ii = a0 + lk + 4 * rr, jj = b0 + li;
            out[ii * 64 + jj] = acc[q][rr];
        }
    }
}

__global__ void k_gram_sum(int nblk, const double *part, int ma, int mb, double *G) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ma * mb) return;
    const int a = e / mb, b = e % mb;
    double s = 0.0;
    for (int k = 0; k < nblk; ++k) s += part[(size_t)k * 4096 + a * 64 + b];
    G[e] = s;
}

// Y = X T (X: n x ma column-major; T: ma x mb column-major)
__global__ __launch_bounds__(kBlock) void k_tsgemm(int n, const double *X, int ma, const double *T, int mb,
                                                   double *Y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x[64];
#pragma unroll
    for (int a = 0; a < 64; ++a) x[a] = (a < ma) ? X[(size_t)a * n + i] : 0.0;
    for (int j = 0; j < mb; ++j) {
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < 64; ++a)
            if (a < ma) s += x[a] * T[(size_t)j * ma + a];
        Y[(size_t)j * n + i] = s;
    }
}

// g_k = -lam_row(k) x_col(k) for every stored entry, CSR order.  One wavefront
// per 64 rows: their entries are one contiguous range, which the lanes stream
// in order (coalesced col and g); lane j holds the start of row j, and each
// entry finds its row by a binary search over those starts (shuffles), the
// last row whose start is <= k, so empty rows are passed over.
__global__ __launch_bounds__(kBlock) void k_grad(int n, const int64_t *rowptr, const int32_t *col, const double *lam,
                                                 const double *x, double *g) {
    const int lane = threadIdx.x & 63;
    const int r0 = ((blockIdx.x * blockDim.x + threadIdx.x) >> 6) * 64;
    if (r0 >= n) return; // uniform over the wavefront
    const int rl = min(64, n - r0);
    // entry offsets fit in int32 (setup rejects nnz >= 2^31); lanes >= rl hold the end
    const int st = (int)rowptr[r0 + min(lane, rl)];
    const int e0 = __shfl(st, 0, 64), e1 = (int)rowptr[r0 + rl];
    const double li = lane < rl ? lam[r0 + lane] : 0.0;
    for (int base = e0; base < e1; base += 64) {
        const int k = base + lane;
        int lo = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
            const int s = __shfl(st, lo + step, 64); // lo + step <= 63
            if (s <= k) lo += step;
        }
        const double lr = __shfl(li, lo, 64);
        if (k < e1) g[k] = -lr * x[col[k]];
    }
}

inline int blocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

inline int mt_bucket(int m) {
    if (m <= 0) return 0;
    if (m <= 8) return 8;
    if (m <= 16) return 16;
    if (m <= 32) return 32;
    return 64;
}

} // namespace

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------

#define ESD_MT_SWITCH(mt, CALL)                                                                    \
    switch (mt_bucket(mt)) {                                                                       \
    case 0: { constexpr int MTV = 0; CALL; } break;                                                \
    case 8: { constexpr int MTV = 8; CALL; } break;                                                \
    case 16: { constexpr int MTV = 16; CALL; } break;                                              \
    case 32: { constexpr int MTV = 32; CALL; } break;                                              \
    default: { constexpr int MTV = 64; CALL; } break;                                              \
    }

int spmv_stride(bool power) { return power ? 2 : 1; }
int grid_red(int64_t rows, int stride) {
    int g = grid_for(rows);
    const int cap = kPartBudget / stride;
    if (g > cap) g = cap / 8 * 8;
    return g < 1 ? 1 : g;
}
static int pow2_at_least(int m) {
    int p = 1;
    while (p < m) p <<= 1;
    return p;
}
int tsdot_stride(int m) { return pow2_at_least(m); }
int tsdot_grid(int64_t n, int m) {
    int64_t g = (n + 4095) / 4096;
    if (g > 512) g = 512;
    const int cap = kPartBudget / pow2_at_least(m);
    if (g > cap) g = cap;
    if (g > 8) g = g / 8 * 8;
    return g < 1 ? 1 : (int)g;
}

void launch_tri_mul(int n, Ell<double> M, const double *d, const double *x, double *y, hipStream_t s) {
    k_tri_mul<<<blocks(n), kBlock, 0, s>>>(n, M, d, x, y);
}

void launch_repack(int64_t size, const int64_t *src, const double *from, double *to64, float *to32, hipStream_t s) {
    if (size <= 0) return;
    k_repack<<<(unsigned)((size + 255) / 256), 256, 0, s>>>(size, src, from, to64, to32);
}

template <typename T> static void spmv_it_impl(const SpmvIt<T> &a, bool power, int grid, hipStream_t s) {
    if (a.z) {
        if (power) k_spmv_it<T, true, false><<<grid, kBlock, 0, s>>>(a);
        else k_spmv_it<T, false, false><<<grid, kBlock, 0, s>>>(a);
    } else {
        if (power) k_spmv_it<T, true, true><<<grid, kBlock, 0, s>>>(a);
        else k_spmv_it<T, false, true><<<grid, kBlock, 0, s>>>(a);
    }
}
void launch_spmv_it(const SpmvIt<double> &a, bool power, int grid, hipStream_t s) { spmv_it_impl(a, power, grid, s); }
void launch_spmv_it(const SpmvIt<float> &a, bool power, int grid, hipStream_t s) { spmv_it_impl(a, power, grid, s); }

template <typename T, int MT, bool XNT, bool GNT>
static void update_it_nt(const UpdIt<T> &a, int grid, hipStream_t s) {
    // with G^T r a row already has MT + 4 loads in flight: one row per thread
    if constexpr (MT == 0) {
        if (stream_pairs<T>(a.n)) {
            k_update_it2<T, 0, XNT, false><<<grid, kBlock, 0, s>>>(a);
            return;
        }
    }
    k_update_it<T, MT, XNT, GNT><<<grid, kBlock, 0, s>>>(a);
}
template <typename T, int MT> static void update_it_mt(const UpdIt<T> &a, int grid, hipStream_t s) {
    const bool gnt = MT > 0 && a.gnt; // without G the flag means nothing: one kernel fewer
    if (a.xnt) {
        if (gnt) update_it_nt<T, MT, true, MT != 0>(a, grid, s);
        else update_it_nt<T, MT, true, false>(a, grid, s);
    } else {
        if (gnt) update_it_nt<T, MT, false, MT != 0>(a, grid, s);
        else update_it_nt<T, MT, false, false>(a, grid, s);
    }
}
template <typename T> static void update_it_impl(const UpdIt<T> &a, int grid, hipStream_t s) {
    if (!a.G || a.m <= 0) update_it_mt<T, 0>(a, grid, s);
    else if (a.m <= 8) update_it_mt<T, 8>(a, grid, s);
    else update_it_mt<T, 16>(a, grid, s);
}
void launch_update_it(const UpdIt<double> &a, int grid, hipStream_t s) { update_it_impl(a, grid, s); }
void launch_update_it(const UpdIt<float> &a, int grid, hipStream_t s) { update_it_impl(a, grid, s); }

template <typename T> static void proj_impl(const Proj<T> &a, int grid, hipStream_t s) {
    if (stream_pairs<T>(a.n) && a.m <= 8) {
        k_proj2<T, 8><<<grid, kBlock, 0, s>>>(a);
        return;
    }
    ESD_MT_SWITCH(a.m, (k_proj<T, (MTV > 0 ? MTV : 8)><<<grid, kBlock, 0, s>>>(a)));
}
void launch_proj(const Proj<double> &a, int grid, hipStream_t s) { proj_impl(a, grid, s); }
void launch_proj(const Proj<float> &a, int grid, hipStream_t s) { proj_impl(a, grid, s); }
template <typename T> static void bwd0_proj_impl(const Sweep<T> &b, const Proj<T> &a, int grid, hipStream_t s) {
    if (stream_pairs<T>(a.n) && a.m <= 8) k_bwd0_proj2<T, 8><<<grid, kBlock, 0, s>>>(b, a);
    else if (a.m <= 8) k_bwd0_proj<T, 8><<<grid, kBlock, 0, s>>>(b, a);
    else k_bwd0_proj<T, 16><<<grid, kBlock, 0, s>>>(b, a);
}
void launch_bwd0_proj(const Sweep<double> &b, const Proj<double> &a, int grid, hipStream_t s) {
    bwd0_proj_impl(b, a, grid, s);
}
void launch_bwd0_proj(const Sweep<float> &b, const Proj<float> &a, int grid, hipStream_t s) {
    bwd0_proj_impl(b, a, grid, s);
}

template <typename T> static void tsdot_impl(const TsDot<T> &a, int grid, hipStream_t s) {
    switch (pow2_at_least(a.m)) {
    case 1: k_tsdot_rm<T, 1><<<grid, kTsBlock, 0, s>>>(a); break;
    case 2: k_tsdot_rm<T, 2><<<grid, kTsBlock, 0, s>>>(a); break;
    case 4: k_tsdot_rm<T, 4><<<grid, kTsBlock, 0, s>>>(a); break;
    case 8: k_tsdot_rm<T, 8><<<grid, kTsBlock, 0, s>>>(a); break;
    case 16: k_tsdot_rm<T, 16><<<grid, kTsBlock, 0, s>>>(a); break;
    case 32: k_tsdot_rm<T, 32><<<grid, kTsBlock, 0, s>>>(a); break;
    default: k_tsdot_rm<T, 64><<<grid, kTsBlock, 0, s>>>(a); break;
    }
}
void launch_tsdot_rm(const TsDot<double> &a, int grid, hipStream_t s) { tsdot_impl(a, grid, s); }
void launch_tsdot_rm(const TsDot<float> &a, int grid, hipStream_t s) { tsdot_impl(a, grid, s); }
void launch_to_rowmajor(int n, int m, const double *W, double *Wrm, float *Wrm32, hipStream_t s) {
    k_to_rowmajor<<<blocks(n), kBlock, 0, s>>>(n, m, W, Wrm, Wrm32);
}

template <typename T> static void fwd_impl(const Sweep<T> &a, bool last, bool sc, int grid, hipStream_t s) {
    if (!last) k_fwd<T, false, false><<<grid, kBlock, 0, s>>>(a);
    else if (sc) k_fwd<T, true, true><<<grid, kBlock, 0, s>>>(a);
    else k_fwd<T, true, false><<<grid, kBlock, 0, s>>>(a);
}
void launch_fwd(const Sweep<double> &a, bool last, bool sc, int grid, hipStream_t s) { fwd_impl(a, last, sc, grid, s); }
void launch_fwd(const Sweep<float> &a, bool last, bool sc, int grid, hipStream_t s) { fwd_impl(a, last, sc, grid, s); }

template <typename T> static void bwd_impl(const Sweep<T> &a, bool sc, int grid, hipStream_t s) {
    if (sc) k_bwd<T, true><<<grid, kBlock, 0, s>>>(a);
    else k_bwd<T, false><<<grid, kBlock, 0, s>>>(a);
}
void launch_bwd(const Sweep<double> &a, bool sc, int grid, hipStream_t s) { bwd_impl(a, sc, grid, s); }
void launch_bwd(const Sweep<float> &a, bool sc, int grid, hipStream_t s) { bwd_impl(a, sc, grid, s); }
template <typename T> static void fwd2_impl(const Sweep<T> &a, bool sc, int grid, hipStream_t s) {
    if (sc) k_fwd2<T, false><<<grid, kBlock, 0, s>>>(a);
    else k_fwd2<T, true><<<grid, kBlock, 0, s>>>(a);
}
template <typename T> static void bwd2_impl(const Sweep<T> &a, bool sc, int grid, hipStream_t s) {
    if (sc) k_bwd2<T, true><<<grid, kBlock, 0, s>>>(a);
    else k_bwd2<T, false><<<grid, kBlock, 0, s>>>(a);
}
void launch_fwd2(const Sweep<double> &a, bool sc, int grid, hipStream_t s) { fwd2_impl(a, sc, grid, s); }
void launch_fwd2(const Sweep<float> &a, bool sc, int grid, hipStream_t s) { fwd2_impl(a, sc, grid, s); }
void launch_bwd2(const Sweep<double> &a, bool sc, int grid, hipStream_t s) { bwd2_impl(a, sc, grid, s); }
void launch_bwd2(const Sweep<float> &a, bool sc, int grid, hipStream_t s) { bwd2_impl(a, sc, grid, s); }

int bj_grid(int nb) { return std::min(kMaxGrid, (nb + kBlock / 64 - 1) / (kBlock / 64)); }

template <typename T> static int bj_impl(const BjSweep<T> &a, bool sc, hipStream_t s) {
    const int grid = bj_grid(a.nb);
    if (a.s <= 64) {
        if (sc) k_bj<T, 1, true><<<grid, kBlock, 0, s>>>(a);
        else k_bj<T, 1, false><<<grid, kBlock, 0, s>>>(a);
    } else if (a.s <= 128) {
        if (sc) k_bj<T, 2, true><<<grid, kBlock, 0, s>>>(a);
        else k_bj<T, 2, false><<<grid, kBlock, 0, s>>>(a);
    } else if (a.s <= 256) {
        if (sc) k_bj<T, 4, true><<<grid, kBlock, 0, s>>>(a);
        else k_bj<T, 4, false><<<grid, kBlock, 0, s>>>(a);
    } else {
        if (sc) k_bj<T, 8, true><<<grid, kBlock, 0, s>>>(a);
        else k_bj<T, 8, false><<<grid, kBlock, 0, s>>>(a);
    }
    return grid;
}
int launch_bj(const BjSweep<double> &a, bool sc, hipStream_t s) { return bj_impl(a, sc, s); }
int launch_bj(const BjSweep<float> &a, bool sc, hipStream_t s) { return bj_impl(a, sc, s); }

template <typename T> static int update_bj_impl(const UpdBj<T> &a, hipStream_t s) {
    const int grid = bj_grid(a.nb);
    if (a.s <= 64) k_update_bj<T, 1><<<grid, kBlock, 0, s>>>(a);
    else if (a.s <= 128) k_update_bj<T, 2><<<grid, kBlock, 0, s>>>(a);
    else if (a.s <= 256) k_update_bj<T, 4><<<grid, kBlock, 0, s>>>(a);
    else k_update_bj<T, 8><<<grid, kBlock, 0, s>>>(a);
    return grid;
}
int launch_update_bj(const UpdBj<double> &a, hipStream_t s) { return update_bj_impl(a, s); }
int launch_update_bj(const UpdBj<float> &a, hipStream_t s) { return update_bj_impl(a, s); }

template <typename T> static void copyz_impl(const Sweep<T> &a, bool sc, int grid, hipStream_t s) {
    if (sc) k_copyz<T, true><<<grid, kBlock, 0, s>>>(a);
    else k_copyz<T, false><<<grid, kBlock, 0, s>>>(a);
}
void launch_copyz(const Sweep<double> &a, bool sc, int grid, hipStream_t s) { copyz_impl(a, sc, grid, s); }
void launch_copyz(const Sweep<float> &a, bool sc, int grid, hipStream_t s) { copyz_impl(a, sc, grid, s); }

void launch_fin_alpha(const FinAlpha &f, hipStream_t s) { k_fin_alpha<<<1, kFinThreads, 0, s>>>(f); }
void launch_fin_u(Scal *S, const double *part, int nblk, int stride, int c0, int m, const double *Cinv,
                  hipStream_t s) {
    k_fin_u<<<1, kFinThreads, 0, s>>>(S, part, nblk, stride, c0, m, Cinv);
}
void launch_fin_rho(const FinRho &f, hipStream_t s) { k_fin_rho<<<1, kFinThreads, 0, s>>>(f); }
void launch_fin_gen(const FinGen &f, hipStream_t s) { k_fin_gen<<<1, kFinThreads, 0, s>>>(f); }

void launch_gather(int n, const int32_t *idx, const double *src, double *dst, hipStream_t s) {
    k_gather<<<blocks(n), kBlock, 0, s>>>(n, idx, src, dst);
}
void launch_scatter(int n, const int32_t *idx, const double *src, double *dst, hipStream_t s) {
    k_scatter<<<blocks(n), kBlock, 0, s>>>(n, idx, src, dst);
}
void launch_fill(int n, double *dst, double v, hipStream_t s) { k_fill<double><<<blocks(n), kBlock, 0, s>>>(n, dst, v); }
void launch_fill(int n, float *dst, float v, hipStream_t s) { k_fill<float><<<blocks(n), kBlock, 0, s>>>(n, dst, v); }
void launch_dot(int n, const double *a, const double *b, double *part, int *nblk, hipStream_t s) {
    const int g = grid_red(n, 1);
    k_dot<<<g, kBlock, 0, s>>>(n, a, b, part);
    *nblk = g;
}
void launch_resid(int n, Ell<double> A, const double *b, const double *x, double *t, const double *W, int m,
                  double *part, int *nblk, int *stride, hipStream_t s) {
    if (!W) m = 0;
    const int st = 1 + (m > 0 ? mt_bucket(m) : 0);
    const int g = grid_red(n, st);
    ESD_MT_SWITCH(m, (k_resid<MTV><<<g, kBlock, 0, s>>>(n, A, b, x, t, W, m, part)));
    *nblk = g;
    *stride = st;
}
void launch_axpy_cols(int n, double *y, const double *M, int m, const double *coef, double sign, double *part,
                      int *nblk, hipStream_t s) {
    const int g = grid_red(n, 1);
    if (part) {
        ESD_MT_SWITCH(m, (k_axpy_cols<(MTV > 0 ? MTV : 8), true><<<g, kBlock, 0, s>>>(n, y, M, m, coef, sign, part)));
    } else {
        ESD_MT_SWITCH(m, (k_axpy_cols<(MTV > 0 ? MTV : 8), false><<<g, kBlock, 0, s>>>(n, y, M, m, coef, sign, part)));
    }
    if (nblk) *nblk = g;
}
void launch_tsdot(int n, const double *W, int m, const double *v, double *part, int *nblk, int *stride,
                  hipStream_t s) {
    const int st = mt_bucket(m) > 0 ? mt_bucket(m) : 8;
    const int g = grid_red(n, st);
    ESD_MT_SWITCH(m, (k_tsdot<(MTV > 0 ? MTV : 8)><<<g, kBlock, 0, s>>>(n, W, m, v, part)));
    *nblk = g;
    *stride = st;
}
void launch_spmv(int n, Ell<double> A, const double *x, double *y, hipStream_t s) {
    k_spmv<<<blocks(n), kBlock, 0, s>>>(n, A, x, y);
}
void launch_rayleigh(int n, Ell<double> A, const double *v, double *part, int *nblk, hipStream_t s) {
    const int g = grid_red(n, 1);
    k_rayleigh<double><<<g, kBlock, 0, s>>>(n, A, v, part);
    *nblk = g;
}
void launch_rayleigh(int n, Ell<float> A, const float *v, double *part, int *nblk, hipStream_t s) {
    const int g = grid_red(n, 1);
    k_rayleigh<float><<<g, kBlock, 0, s>>>(n, A, v, part);
    *nblk = g;
}
void launch_sample_store(int n, double *slot, const double *x, hipStream_t s) {
    k_scale_copy<<<blocks(n), kBlock, 0, s>>>(n, x, slot, 1.0);
}
void launch_cast_scale(int n, const double *src, float *dst, double scale, hipStream_t s) {
    k_cast_scale<<<blocks(n), kBlock, 0, s>>>(n, src, dst, scale);
}
void launch_cast(int64_t n, const double *src, float *dst, hipStream_t s) {
    if (n > 0) k_cast<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, s>>>(n, src, dst);
}
void launch_add_scaled(int n, double *x, const float *d, double scale, hipStream_t s) {
    k_add_scaled<<<blocks(n), kBlock, 0, s>>>(n, x, d, scale);
}
void launch_axpby(int n, const double *f, const double *x, double c, double *b, hipStream_t s) {
    k_axpby<<<blocks(n), kBlock, 0, s>>>(n, f, x, c, b);
}
void launch_sub(int n, const double *a, const double *b, double *dst, hipStream_t s) {
    k_sub<<<blocks(n), kBlock, 0, s>>>(n, a, b, dst);
}
void launch_scale_copy(int n, const double *src, double *dst, double scale, hipStream_t s) {
    k_scale_copy<<<blocks(n), kBlock, 0, s>>>(n, src, dst, scale);
}
void launch_factor_level(int r0, int r1, int n, Ell<double> L, double *lval, const double *adiag, double *ldiag,
                         int *bad, hipStream_t s) {
    // padding slots carry column n
    const int rows = r1 - r0;
    k_factor_level<<<blocks(rows), kBlock, 0, s>>>(r0, r1, n, L, lval, adiag, ldiag, bad);
}
void launch_factor_bj(int n, int s, Ell<double> L, double *lval, const double *adiag, double *ldiag, double *lsub,
                      float *lsub32, int *bad, hipStream_t st) {
    const int nb = (n + s - 1) / s;
    k_factor_bj<<<(nb + 63) / 64, 64, 0, st>>>(n, s, L, lval, adiag, ldiag, lsub, lsub32, bad);
}
void launch_finish_factor(int n, const double *ldiag, double *dinv, float *dinv32, hipStream_t s) {
    k_finish_factor<<<blocks(n), kBlock, 0, s>>>(n, ldiag, dinv, dinv32);
}
void launch_map_values(int64_t cnt, const int32_t *src, const double *val, double *dst, float *dst32, hipStream_t s) {
    if (cnt > 0) k_map_values<<<(unsigned)((cnt + kBlock - 1) / kBlock), kBlock, 0, s>>>(cnt, src, val, dst, dst32);
}
void launch_gather_u(int64_t cnt, const int64_t *map, const double *lval, double *uval, hipStream_t s) {
    if (cnt > 0) k_gather_u<<<(unsigned)((cnt + kBlock - 1) / kBlock), kBlock, 0, s>>>(cnt, map, lval, uval);
}
void launch_spmm(int n, Ell<double> A, const double *E, int m, double *AE, hipStream_t s) {
    k_spmm<<<blocks(n), kBlock, 0, s>>>(n, A, E, m, AE);
}
int gram_grid(int n) {
    int g = (n + 4095) / 4096;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    return g;
}
void launch_gram(int n, const double *E, int ma, const double *F, int mb, double *part, double *G, int grid,
                 hipStream_t s) {
    k_gram_part<<<grid, 256, 0, s>>>(n, E, ma, F, mb, part);
    k_gram_sum<<<(ma * mb + 255) / 256, 256, 0, s>>>(grid, part, ma, mb, G);
}
void launch_tsgemm(int n, const double *X, int ma, const double *T, int mb, double *Y, hipStream_t s) {
    k_tsgemm<<<blocks(n), kBlock, 0, s>>>(n, X, ma, T, mb, Y);
}
void launch_grad(int n, const int64_t *rowptr, const int32_t *col, const double *lam, const double *x, double *g,
                 hipStream_t s) {
    k_grad<<<blocks(n), kBlock, 0, s>>>(n, rowptr, col, lam, x, g);
}

// ---- streaming probes of the achievable HBM bandwidth (not part of the method)
// Grid-stride over 16-byte vectors, consecutive lanes on consecutive vectors
// (one 1 KB coalesced access per wavefront and load), four independent loads
// in flight per thread before any store or add; non-temporal loads and
// stores (streamed data is not kept in the caches).
typedef double probe_v2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(kBlock) void k_probe_copy(const probe_v2 *__restrict__ src, probe_v2 *__restrict__ dst,
                                                        int64_t n2) {
    const int64_t st = (int64_t)gridDim.x * kBlock;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (; i + 3 * st < n2; i += 4 * st) {
        const probe_v2 a = __builtin_nontemporal_load(src + i), b = __builtin_nontemporal_load(src + i + st),
                       c = __builtin_nontemporal_load(src + i + 2 * st),
                       d = __builtin_nontemporal_load(src + i + 3 * st);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + st);
        __builtin_nontemporal_store(c, dst + i + 2 * st);
        __builtin_nontemporal_store(d, dst + i + 3 * st);
    }
    for (; i < n2; i += st) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

__global__ __launch_bounds__(kBlock) void k_probe_read(const probe_v2 *__restrict__ src, int64_t n2, double *part) {
    const int64_t st = (int64_t)gridDim.x * kBlock;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double acc[1] = {0.0};
    for (; i + 3 * st < n2; i += 4 * st) {
        const probe_v2 a = __builtin_nontemporal_load(src + i), b = __builtin_nontemporal_load(src + i + st),
                       c = __builtin_nontemporal_load(src + i + 2 * st),
                       d = __builtin_nontemporal_load(src + i + 3 * st);
        acc[0] += ((a.x + a.y) + (b.x + b.y)) + ((c.x + c.y) + (d.x + d.y));
    }
    for (; i < n2; i += st) {
        const probe_v2 a = __builtin_nontemporal_load(src + i);
        acc[0] += a.x + a.y;
    }
    block_partials<1>(acc, part, 1);
}

void launch_probe(int kind, const double *src, double *dst, int64_t n, int grid, hipStream_t s) {
    const int64_t n2 = n / 2;
    if (kind == 0) k_probe_copy<<<grid, kBlock, 0, s>>>((const probe_v2 *)src, (probe_v2 *)dst, n2);
    else k_probe_read<<<grid, kBlock, 0, s>>>((const probe_v2 *)src, n2, dst);
}

} // namespace esd
