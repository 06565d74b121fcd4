"""Seeded synthetic SPD workloads shaped like the paper's test problems.

This module is shared by the oracle side and the GPU side of the test suite and
by the benchmark.  It only *defines inputs*: it discretises heterogeneous
diffusion problems, applies the diagonal scaling that the paper applies to every
test matrix (Sec. 5.1, test conditions; also Sec. 5.4), assigns parity colours,
and draws right-hand sides and other random inputs.  It contains none of the
solver's arithmetic (no factorisation, no Krylov step, no projection).

Every random quantity comes from ``numpy.random.default_rng([cfg, stream])``
with the streams

    0 coefficient field, 1 inclusion placement, 2 f ~ U[0,1),
    3 power-method start vector, 4 x_target ~ N(0,1), 5 FD directions.

Matrices are returned as full symmetric CSR: ``rowptr`` int64[n+1],
``col`` int32[nnz] (sorted ascending within a row, diagonal included) and
``val`` float64[nnz].
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

STREAM_FIELD, STREAM_PLACE, STREAM_RHS, STREAM_V0, STREAM_XT, STREAM_FD = range(6)


@dataclass
class Problem:
    """One SPD matrix plus the inputs of a sequence of systems that share it."""

    name: str
    n: int
    rowptr: np.ndarray  # int64[n+1]
    col: np.ndarray  # int32[nnz]
    val: np.ndarray  # float64[nnz], diagonally scaled (unit diagonal)
    colors: Optional[np.ndarray]  # int32[n] or None (natural order)
    f: np.ndarray  # float64[n], the fixed part of every right-hand side
    shape: tuple
    params: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def rng(self, stream: int) -> np.random.Generator:
        return np.random.default_rng([self.params.get("cfg", 0), stream])


def rng_for(cfg: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([cfg, stream])


# --------------------------------------------------------------------------
# CSR helpers (format only)
# --------------------------------------------------------------------------

def _stencil_to_csr(n: int, cols: np.ndarray, vals: np.ndarray, mask: np.ndarray):
    """Compress an (n, s) padded stencil table into CSR.

    ``cols[:, t]`` must be increasing in t for each row where ``mask`` holds, so
    the CSR columns come out sorted.
    """
    counts = mask.sum(axis=1, dtype=np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = cols[mask].astype(np.int32, copy=False)
    val = vals[mask].astype(np.float64, copy=False)
    return rowptr, col, val


def diag_scale(rowptr: np.ndarray, col: np.ndarray, val: np.ndarray) -> np.ndarray:
    """Return the values of D^{-1/2} A D^{-1/2} (unit diagonal).

    The paper solves diagonally scaled matrices (Sec. 5.1); the threshold on Ritz
    values only makes sense for such a scaling (Sec. 4.2, after eq. (bk)).
    """
    n = rowptr.shape[0] - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    isdiag = rows == col
    d = np.zeros(n)
    d[rows[isdiag]] = val[isdiag]
    if np.any(d <= 0):
        raise ValueError("diagonal scaling needs a positive diagonal")
    s = 1.0 / np.sqrt(d)
    out = val * (s[rows] * s[col])  # s_i*s_j commutes: exact symmetry
    out[isdiag] = 1.0
    return out


def csr_to_dense(rowptr, col, val, n=None) -> np.ndarray:
    n = rowptr.shape[0] - 1 if n is None else n
    A = np.zeros((n, n))
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    A[rows, col] = val
    return A


# --------------------------------------------------------------------------
# Finite-volume diffusion (2-D 5-point, 3-D 7-point)
# --------------------------------------------------------------------------

def fv_matrix(k: np.ndarray):
    """Cell-centred FV diffusion matrix on a uniform grid, Dirichlet outside.

    ``k`` has shape (N0,) x d in (x, y[, z]) index order; unknown index is
    ``i + N0*j + N0*N1*l`` (x fastest).  Interior faces use the harmonic
    transmissibility 2 k_a k_b / (k_a + k_b); a boundary face uses k_a (ghost
    cell with the same coefficient at zero value).  With k == 1 this is the
    standard 5-/7-point finite-difference Laplacian.
    """
    d = k.ndim
    shape = k.shape
    n = int(np.prod(shape))
    kf = np.asarray(k, dtype=np.float64).transpose(tuple(range(d))[::-1]).ravel()  # x fastest
    # neighbour offsets in increasing column order
    strides = [1]
    for ax in range(1, d):
        strides.append(strides[-1] * shape[ax - 1])
    offs = []
    for ax in reversed(range(d)):
        offs.append((ax, -1))
    offs_neg = offs
    offs_pos = [(ax, +1) for ax in range(d)]
    coords = np.indices(shape[::-1]).reshape(d, -1)[::-1]  # coords[ax][row]
    diag = np.zeros(n)
    table_cols, table_vals, table_mask = [], [], []

    def neighbour(ax, sgn):
        c = coords[ax] + sgn
        inside = (c >= 0) & (c < shape[ax])
        idx = np.arange(n, dtype=np.int64) + sgn * strides[ax]
        kn = np.ones(n)
        kn[inside] = kf[idx[inside]]
        ka = kf
        t = np.where(inside, 2.0 * ka * kn / (ka + kn), ka)
        return idx, t, inside

    for ax, sgn in offs_neg:
        idx, t, inside = neighbour(ax, sgn)
        diag += t
        table_cols.append(np.where(inside, idx, 0))
        table_vals.append(-t)
        table_mask.append(inside)
    pos_parts = []
    for ax, sgn in offs_pos:
        idx, t, inside = neighbour(ax, sgn)
        diag += t
        pos_parts.append((np.where(inside, idx, 0), -t, inside))
    table_cols.append(np.arange(n, dtype=np.int64))
    table_vals.append(diag)
    table_mask.append(np.ones(n, dtype=bool))
    for c, v, msk in pos_parts:
        table_cols.append(c)
        table_vals.append(v)
        table_mask.append(msk)
    cols = np.stack(table_cols, axis=1)
    vals = np.stack(table_vals, axis=1)
    mask = np.stack(table_mask, axis=1)
    return _stencil_to_csr(n, cols, vals, mask)


def parity_colors(shape) -> np.ndarray:
    """Colour (i&1) + 2(j&1) + 4(l&1) of every cell/node, x fastest.

    Every face, edge or corner neighbour flips at least one parity bit, so no two
    coupled unknowns of a 5-, 7- or 27-point stencil share a colour.
    """
    d = len(shape)
    coords = np.indices(shape[::-1]).reshape(d, -1)[::-1]
    c = np.zeros(coords.shape[1], dtype=np.int32)
    for ax in range(d):
        c += ((coords[ax] & 1) << ax).astype(np.int32)
    return c


# --------------------------------------------------------------------------
# Coefficient fields
# --------------------------------------------------------------------------

def place_boxes(rng, N: int, size: int, count: int, dim: int, max_tries: int = 200000):
    """Non-overlapping boxes of ``size`` cells, >= 1 cell from each other and the boundary."""
    lo, hi = 1, N - size - 1  # corner range, inclusive
    if hi < lo:
        raise ValueError("grid too small for the boxes")
    corners = []
    tries = 0
    while len(corners) < count:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("box placement by rejection failed")
        c = rng.integers(lo, hi + 1, size=dim)
        ok = True
        for o in corners:
            # separated along some axis by at least one cell of gap
            if not np.any(np.abs(c - o) >= size + 1):
                ok = False
                break
        if ok:
            corners.append(c)
    return np.array(corners, dtype=np.int64)


def lognormal_spheres_field(cfg: int, N: int, sigma: float = 2.0, nsph: int = 16,
                            radius: float = 6.0, contrast: float = 1e-5) -> np.ndarray:
    """k = exp(sigma*xi), xi iid N(0,1) per cell, times ``contrast`` inside spheres.

    Sphere centres are uniform in [radius, N - radius)^3; a cell is inside when
    its centre (index + 0.5) is within ``radius``.  Shape (N, N, N) indexed (x, y, z).
    """
    g0 = rng_for(cfg, STREAM_FIELD)
    xi = g0.standard_normal((N, N, N))
    k = np.exp(sigma * xi)
    g1 = rng_for(cfg, STREAM_PLACE)
    centres = g1.uniform(radius, N - radius, size=(nsph, 3))
    inside = np.zeros((N, N, N), dtype=bool)
    ax = np.arange(N) + 0.5
    r = int(np.ceil(radius)) + 1
    for c in centres:
        lo = np.maximum(np.floor(c - r).astype(int), 0)
        hi = np.minimum(np.ceil(c + r).astype(int), N)
        X, Y, Z = np.meshgrid(ax[lo[0]:hi[0]], ax[lo[1]:hi[1]], ax[lo[2]:hi[2]], indexing="ij")
        d2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2
        inside[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] |= d2 <= radius * radius
    k[inside] *= contrast
    return k


# --------------------------------------------------------------------------
# Q1 (trilinear) FEM Laplacian, 27-point stencil
# --------------------------------------------------------------------------

# Reference stiffness of the trilinear element on the unit cube, by how many
# coordinates the two vertices differ in: 0 -> 1/3, 1 (shared edge) -> 0,
# 2 (face diagonal) -> -1/12, 3 (body diagonal) -> -1/12.
Q1_REF = (1.0 / 3.0, 0.0, -1.0 / 12.0, -1.0 / 12.0)


def q1_matrix(ce: np.ndarray, h: float):
    """Assemble the Q1 Laplacian with element coefficients ``ce`` (Ne^3, (x,y,z)).

    Nodes are the (Ne-1)^3 interior vertices (Dirichlet boundary eliminated);
    unknown index ``a + M*b + M*M*c`` over interior vertex indices 1..Ne-1.
    Every one of the 27 couplings is stored, including the exact zeros between
    vertices that share an element edge.  Element matrix = c_e * h * K_ref.
    """
    Ne = ce.shape[0]
    M = Ne - 1
    n = M ** 3
    # node coordinates (1..M) as arrays over rows, x fastest
    c3 = np.indices((M, M, M)).reshape(3, -1)[::-1] + 1  # c3[0]=x index ...
    cols, vals, masks = [], [], []
    ce_flat = np.ascontiguousarray(ce.transpose(2, 1, 0)).ravel()  # element (ex,ey,ez) -> ex + Ne*ey + Ne^2*ez

    def eidx(ex, ey, ez):
        return ex + Ne * ey + Ne * Ne * ez

    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                d = (dx, dy, dz)
                q = [c3[ax] + d[ax] for ax in range(3)]
                inside = np.ones(n, dtype=bool)
                for ax in range(3):
                    inside &= (q[ax] >= 1) & (q[ax] <= M)
                # shared elements: per axis, e in {p-1, p} if d==0 else {min(p, p+d)}
                choices = []
                for ax in range(3):
                    p = c3[ax]
                    if d[ax] == 0:
                        choices.append([p - 1, p])
                    else:
                        choices.append([np.minimum(p, p + d[ax])])
                s = np.zeros(n)
                for ex in choices[0]:
                    for ey in choices[1]:
                        for ez in choices[2]:
                            s += ce_flat[eidx(ex, ey, ez)]
                nz = sum(1 for t in d if t != 0)
                v = h * Q1_REF[nz] * s
                col = (q[0] - 1) + M * (q[1] - 1) + M * M * (q[2] - 1)
                cols.append(np.where(inside, col, 0))
                vals.append(v)
                masks.append(inside)
    return _stencil_to_csr(n, np.stack(cols, 1), np.stack(vals, 1), np.stack(masks, 1))


# --------------------------------------------------------------------------
# The five configurations
# --------------------------------------------------------------------------

def _rhs(cfg: int, n: int) -> np.ndarray:
    return rng_for(cfg, STREAM_RHS).random(n)


def config1(N: int = 64, nbox: int = 4, box: int = 8, kin: float = 1e-4) -> Problem:
    """2-D 5-point FV, k = 1 with ``nbox`` floating squares of coefficient ``kin``; natural order."""
    cfg = 1
    k = np.ones((N, N))
    corners = place_boxes(rng_for(cfg, STREAM_PLACE), N, box, nbox, 2)
    for c in corners:
        k[c[0]:c[0] + box, c[1]:c[1] + box] = kin
    rowptr, col, val = fv_matrix(k)
    val = diag_scale(rowptr, col, val)
    n = N * N
    return Problem("cfg1_fv2d_%d" % N, n, rowptr, col, val, None, _rhs(cfg, n), (N, N),
                   dict(cfg=cfg, m=8, systems=4, theta=(1e-2, 1e-3), corners=corners.tolist()))


def config2(N: int = 128, nsph: int = 16, radius: float = 6.0, cfg: int = 2,
            m: int = 16, systems: int = 10) -> Problem:
    """3-D 7-point FV, lognormal sigma=2 field with spheres of contrast 1e-5; 8 parity colours."""
    k = lognormal_spheres_field(cfg, N, 2.0, nsph, radius, 1e-5)
    rowptr, col, val = fv_matrix(k)
    val = diag_scale(rowptr, col, val)
    n = N ** 3
    return Problem("cfg%d_fv3d_%d" % (cfg, N), n, rowptr, col, val, parity_colors((N, N, N)),
                   _rhs(cfg, n), (N, N, N), dict(cfg=cfg, m=m, systems=systems, theta=1e-3))


def config3(N: int = 256) -> Problem:
    """Config-2 recipe at 256^3 (mixed precision workload); m = 32."""
    return config2(N=N, cfg=3, m=32, systems=10)


def config4(Ne: int = 161, nblk: int = 64, blk: int = 10, cin: float = 1e6) -> Problem:
    """Q1 FEM on Ne^3 elements ((Ne-1)^3 unknowns), floating stiff blocks; 27-point; 8 colours."""
    cfg = 4
    ce = np.ones((Ne, Ne, Ne))
    corners = place_boxes(rng_for(cfg, STREAM_PLACE), Ne, blk, nblk, 3)
    for c in corners:
        ce[c[0]:c[0] + blk, c[1]:c[1] + blk, c[2]:c[2] + blk] = cin
    h = 1.0 / Ne
    rowptr, col, val = q1_matrix(ce, h)
    val = diag_scale(rowptr, col, val)
    M = Ne - 1
    n = M ** 3
    return Problem("cfg4_q1_%d" % M, n, rowptr, col, val, parity_colors((M, M, M)), _rhs(cfg, n),
                   (M, M, M), dict(cfg=cfg, m=64, systems=20, theta=1e-3, nblk=nblk))


def config5_dense(N: int = 8) -> Problem:
    """Tiny instance for dense gradient checks: sigma=2 field plus one sphere r=2, 8 colours."""
    k = lognormal_spheres_field(5, N, 2.0, 1, 2.0, 1e-5)
    rowptr, col, val = fv_matrix(k)
    val = diag_scale(rowptr, col, val)
    n = N ** 3
    return Problem("cfg5_fv3d_%d" % N, n, rowptr, col, val, parity_colors((N, N, N)),
                   _rhs(5, n), (N, N, N), dict(cfg=5, m=16, systems=1, theta=1e-3))


def poisson(shape) -> Problem:
    """Constant-coefficient FD Laplacian (k == 1), diagonally scaled; natural order."""
    k = np.ones(shape)
    rowptr, col, val = fv_matrix(k)
    val = diag_scale(rowptr, col, val)
    n = int(np.prod(shape))
    return Problem("poisson_%s" % "x".join(map(str, shape)), n, rowptr, col, val, None,
                   _rhs(0, n), tuple(shape), dict(cfg=0))


def poisson_eigvec(shape, modes) -> tuple:
    """Closed-form eigenpairs of the scaled constant-coefficient Laplacian.

    For Dirichlet FD on N_ax points per axis, the eigenvectors are products of
    sin(j*pi*(i+1)/(N+1)) and the eigenvalues of the scaled matrix are
    1 - (1/d) * sum_ax cos(j_ax*pi/(N_ax+1)).  ``modes`` is a list of
    multi-indices (1-based).  Returns (lambdas, V with orthonormal columns).
    """
    d = len(shape)
    lams, vecs = [], []
    for j in modes:
        lam = 1.0 - sum(np.cos(j[ax] * np.pi / (shape[ax] + 1)) for ax in range(d)) / d
        v = np.ones(1)
        # build with x fastest: outer product in reverse axis order
        for ax in reversed(range(d)):
            s = np.sin(j[ax] * np.pi * np.arange(1, shape[ax] + 1) / (shape[ax] + 1))
            v = np.kron(v, s)
        v /= np.linalg.norm(v)
        lams.append(lam)
        vecs.append(v)
    return np.array(lams), np.stack(vecs, axis=1)


def poisson_spectrum(shape) -> np.ndarray:
    """All eigenvalues of the scaled constant-coefficient Laplacian, ascending."""
    d = len(shape)
    parts = [np.cos(np.arange(1, N + 1) * np.pi / (N + 1)) for N in shape]
    tot = np.zeros(1)
    for p in parts:
        tot = (tot[:, None] + p[None, :]).ravel()
    return np.sort(1.0 - tot / d)


def make_config(cfg: int, **kw) -> Problem:
    return {1: config1, 2: config2, 3: config3, 4: config4, 5: config5_dense}[cfg](**kw)


def sequence_rhs(f: np.ndarray, x_prev: Optional[np.ndarray]) -> np.ndarray:
    """Right-hand side of system k: f + 0.1 * x_{k-1} (f for the first system)."""
    return f.copy() if x_prev is None else f + 0.1 * x_prev


def power_start(cfg: int, n: int) -> np.ndarray:
    """Unit random start vector of the power method (stream 3)."""
    v = rng_for(cfg, STREAM_V0).standard_normal(n)
    return v / np.linalg.norm(v)
