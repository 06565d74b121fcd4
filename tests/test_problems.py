"""Input generators: structure, closed forms and the Q1 element matrix."""
import numpy as np
import pytest

from paper_2203_08498_amd import problems as P


def _dense(p):
    return P.csr_to_dense(p.rowptr, p.col, p.val)


def test_config1_sizes_and_structure():
    p = P.config1()
    assert p.n == 4096 and p.nnz == 20224  # 5-point: n + 4(N-1)N
    A = _dense(p)
    assert np.abs(A - A.T).max() == 0.0
    assert np.all(np.diag(A) == 1.0)
    off = A - np.diag(np.diag(A))
    assert off.max() <= 0.0  # M-matrix sign pattern
    # columns sorted inside every row
    for i in range(0, p.n, 97):
        c = p.col[p.rowptr[i]:p.rowptr[i + 1]]
        assert np.all(np.diff(c) > 0)


@pytest.mark.parametrize("N", [6, 9])
def test_fv3d_nnz_formula_and_spd(N):
    p = P.config2(N=N, nsph=1, radius=2.0)
    assert p.nnz == N ** 3 + 6 * (N - 1) * N * N
    A = _dense(p)
    assert np.abs(A - A.T).max() < 1e-15
    assert np.linalg.eigvalsh(A)[0] > 0


def test_constant_coefficient_is_scaled_fd_laplacian():
    shape = (5, 4, 3)
    p = P.poisson(shape)
    A = _dense(p)
    # FD Laplacian with Dirichlet: diagonal 6, neighbours -1; scaled by 1/6
    n = p.n
    L = np.zeros((n, n))
    idx = lambda i, j, k: i + shape[0] * (j + shape[1] * k)
    for k in range(shape[2]):
        for j in range(shape[1]):
            for i in range(shape[0]):
                r = idx(i, j, k)
                L[r, r] = 6
                for d in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
                    for s in (-1, 1):
                        a, b, c = i + s * d[0], j + s * d[1], k + s * d[2]
                        if 0 <= a < shape[0] and 0 <= b < shape[1] and 0 <= c < shape[2]:
                            L[r, idx(a, b, c)] = -1
    assert np.abs(A - L / 6).max() < 1e-15
    lam, V = P.poisson_eigvec(shape, [(1, 1, 1), (3, 2, 1)])
    assert np.abs(A @ V - V * lam).max() < 1e-14
    assert np.abs(np.linalg.eigvalsh(A) - P.poisson_spectrum(shape)).max() < 1e-14


def test_q1_reference_element_by_quadrature():
    # stiffness of trilinear shape functions on the unit cube, Gauss-Legendre 3^3
    g, w = np.polynomial.legendre.leggauss(3)
    g = 0.5 * (g + 1)
    w = 0.5 * w
    verts = [(a, b, c) for c in (0, 1) for b in (0, 1) for a in (0, 1)]

    def grad(v, x):
        f = [(x[ax] if v[ax] else 1 - x[ax]) for ax in range(3)]
        df = [(1.0 if v[ax] else -1.0) for ax in range(3)]
        return np.array([df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]])

    K = np.zeros((8, 8))
    for i, xi in enumerate(g):
        for j, yj in enumerate(g):
            for k, zk in enumerate(g):
                x = (xi, yj, zk)
                wt = w[i] * w[j] * w[k]
                G = [grad(v, x) for v in verts]
                for a in range(8):
                    for b in range(8):
                        K[a, b] += wt * G[a] @ G[b]
    for a in range(8):
        for b in range(8):
            nd = sum(1 for ax in range(3) if verts[a][ax] != verts[b][ax])
            assert abs(K[a, b] - P.Q1_REF[nd]) < 1e-14


def test_q1_matrix_nnz_and_rowsum():
    Ne = 7
    ce = np.ones((Ne, Ne, Ne))
    rp, col, val = P.q1_matrix(ce, 1.0 / Ne)
    M = Ne - 1
    assert rp[-1] == (3 * M - 2) ** 3
    A = P.csr_to_dense(rp, col, val)
    assert np.abs(A - A.T).max() < 1e-16
    # interior node far from the boundary: row sums to zero (constants in the kernel)
    c = 3 + M * (3 + M * 3)
    assert abs(A[c].sum()) < 1e-15
    assert np.linalg.eigvalsh(A)[0] > 0


def test_config4_small_has_isolated_small_eigenvalues():
    p = P.config4(Ne=13, nblk=2, blk=3)
    ev = np.linalg.eigvalsh(_dense(p))
    assert ev[1] < 1e-5 and ev[2] > 1e-2  # one near-zero mode per floating stiff block


def test_parity_colors_are_proper_for_27_point():
    p = P.config4(Ne=7, nblk=1, blk=2)
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    off = rows != p.col
    assert np.all(p.colors[rows[off]] != p.colors[p.col[off]])


def test_seeds_are_deterministic():
    a = P.config2(N=8, nsph=1, radius=2.0)
    b = P.config2(N=8, nsph=1, radius=2.0)
    assert np.array_equal(a.val, b.val) and np.array_equal(a.f, b.f)
