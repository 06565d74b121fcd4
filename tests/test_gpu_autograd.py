"""Gradients through the GPU solver (torch.autograd.Function): dense reference
on a small instance, central finite differences with symmetric directions, and
the adjoint solve with the deflated mixed solver at the config-5 size."""
import numpy as np
import pytest

from paper_2203_08498_amd import problems as P

pytestmark = pytest.mark.gpu


def _setup(p, m_max=16):
    import torch

    from paper_2203_08498_amd import esd

    s = esd.Solver.from_problem(p, m_max=m_max)
    s.factor_ic0()
    vals = torch.tensor(p.val, device="cuda", dtype=torch.float64, requires_grad=True)
    return s, vals


def _transpose_map(p):
    """Position of the transposed entry (j, i) of every stored (i, j) (the
    pattern is symmetric)."""
    import scipy.sparse as sp

    M = sp.csr_matrix((np.arange(1, p.nnz + 1, dtype=np.float64), p.col, p.rowptr), shape=(p.n, p.n))
    T = M.T.tocsr()
    T.sort_indices()
    assert np.array_equal(T.indptr, p.rowptr) and np.array_equal(T.indices, p.col)
    return T.data.astype(np.int64) - 1


def _sym_direction(p, rng, tmap=None):
    """A symmetric perturbation of the stored values: (D + D^T) / 2 for D with
    N(0,1) entries on the pattern."""
    d = rng.standard_normal(p.nnz)
    tmap = _transpose_map(p) if tmap is None else tmap
    return 0.5 * (d + d[tmap])


def test_gradient_matches_dense_reference():
    import torch

    from paper_2203_08498_amd import autograd as AG, esd

    p = P.config5_dense(N=8)
    s, vals = _setup(p)
    xt = P.rng_for(5, P.STREAM_XT).standard_normal(p.n)
    b = torch.tensor(p.f, device="cuda", requires_grad=True)
    x = AG.solve(vals, b, s, tol=1e-14, maxit=5000)
    loss = 0.5 * ((x - torch.tensor(xt, device="cuda")) ** 2).sum()
    loss.backward()
    A = P.csr_to_dense(p.rowptr, p.col, p.val)
    xd = np.linalg.solve(A, p.f)
    lam = np.linalg.solve(A, xd - xt)
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    gref = -lam[rows] * xd[p.col]
    gb = b.grad.cpu().numpy()
    gv = vals.grad.cpu().numpy()
    assert np.abs(gb - lam).max() <= 1e-8 * np.abs(lam).max()
    assert np.abs(gv - gref).max() <= 1e-8 * np.abs(gref).max()
    s.close()


def test_gradient_central_differences_small():
    import torch

    from paper_2203_08498_amd import autograd as AG

    p = P.config5_dense(N=8)
    s, vals = _setup(p)
    xt = torch.tensor(P.rng_for(5, P.STREAM_XT).standard_normal(p.n), device="cuda")
    b = torch.tensor(p.f, device="cuda", requires_grad=True)
    x = AG.solve(vals, b, s, tol=1e-14, maxit=5000)
    loss = 0.5 * ((x - xt) ** 2).sum()
    loss.backward()
    gv = vals.grad.cpu().numpy()
    gb = b.grad.cpu().numpy()
    rng = P.rng_for(5, P.STREAM_FD)
    h = 1e-6

    def L(v, bb):
        s.update_values(v)
        s.factor_ic0()
        xx, info = s.solve(bb, tol=1e-14, maxit=5000)
        return 0.5 * float(((xx - xt) ** 2).sum())

    for _ in range(8):
        d = _sym_direction(p, rng)
        db = rng.standard_normal(p.n)
        fd = (L(p.val + h * d, p.f + h * db) - L(p.val - h * d, p.f - h * db)) / (2 * h)
        an = gv @ d + gb @ db
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
    s.close()


def test_gradient_config5_full_size_deflated_mixed():
    """Config 5 as specified: the 128^3 config-2 field, forward and adjoint
    solves with the deflated FP32/FP64 mixed solver (m = 16, theta = 1e-3)
    inside the autograd Function, loss 0.5 ||x - x_t||^2; the gradient with
    respect to b and all stored values against central differences with
    h = 1e-6 along 32 seeded directions (symmetric value perturbation and a
    right-hand-side perturbation, both N(0,1)).

    Error budget, relative to the directional derivative.  The forward and
    adjoint solves at relres 1e-12 (the mixed solver's FP64 floor here is
    about 7e-13) give the gradient to about kappa(A) 1e-12 ~ 1e-8 (lambda_max
    ~ 2 over a smallest eigenvalue ~ 4e-4).  The central difference itself
    carries its truncation, h^2 / 6 times the third derivative: the b part of
    the loss is quadratic (exact), the value part is not, and along these
    directions its relative size is 2.6e-7 to 1.2e-6 at h = 1e-6 -- so the
    central difference alone cannot certify 1e-6.  The test checks that this
    is truncation: at 2h the difference grows 4x (between 3.5x and 4.5x), and
    the Richardson combination (4 D(h) - D(2h)) / 3, whose error is O(h^4),
    agrees with the adjoint gradient to 1e-8 on every direction (measured
    <= 3e-9).  FD solves are FP64 deflated at recurrence relres 1e-13 (true
    residual at the FP64 floor, 3e-12)."""
    import torch

    from paper_2203_08498_amd import autograd as AG, esd

    p = P.config2(N=128, cfg=2)
    print("config 5 at 128^3: n", p.n, "nnz", p.nnz, flush=True)
    s, vals = _setup(p, m_max=16)
    s.sample_errors(16)
    s.solve(p.f, tol=1e-8, maxit=20000)
    st, ritz, mb, mt = s.build_aux(1e-3)
    assert mt > 0
    xt = torch.tensor(P.rng_for(5, P.STREAM_XT).standard_normal(p.n), device="cuda")
    b = torch.tensor(p.f, device="cuda", requires_grad=True)
    x = AG.solve(vals, b, s, mode=esd.DEFLATED, tol=1e-12, maxit=20000, flags=esd.FLAG_MIXED)
    loss = 0.5 * ((x - xt) ** 2).sum()
    loss.backward()
    gv = vals.grad.cpu().numpy()
    gb = b.grad.cpu().numpy()
    assert np.all(np.isfinite(gv)) and np.all(np.isfinite(gb))
    rng = P.rng_for(5, P.STREAM_FD)
    h = 1e-6

    def L(v, bb):
        s.update_values(v)
        s.factor_ic0()
        xx, info = s.solve(bb, tol=1e-13, maxit=50000, mode=esd.DEFLATED)
        assert info["converged"]
        return 0.5 * float(((xx - xt) ** 2).sum())

    def D(d, db, hh):
        return (L(p.val + hh * d, p.f + hh * db) - L(p.val - hh * d, p.f - hh * db)) / (2 * hh)

    tmap = _transpose_map(p)
    errs, rich = [], []
    for k in range(32):
        d = _sym_direction(p, rng, tmap)
        db = rng.standard_normal(p.n)
        an = gv @ d + gb @ db
        d1, d2 = D(d, db, h), D(d, db, 2 * h)
        e1, e2 = (d1 - an) / an, (d2 - an) / an
        r = ((4 * d1 - d2) / 3 - an) / an
        errs.append(abs(e1))
        rich.append(abs(r))
        print("config-5 direction", k, "adjoint", an, "CD rel err h %.2e 2h %.2e ratio %.3f Richardson %.2e"
              % (e1, e2, e2 / e1, r), flush=True)
        assert 3.5 <= e2 / e1 <= 4.5
    s.update_values(p.val)
    print("config-5 central differences: max", max(errs), "median", float(np.median(errs)),
          "; Richardson: max", max(rich), flush=True)
    assert max(errs) <= 2e-6 and max(rich) <= 1e-8
    s.close()
