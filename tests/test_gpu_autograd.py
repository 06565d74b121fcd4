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


def _sym_direction(p, rng):
    import scipy.sparse as sp

    d = rng.standard_normal(p.nnz)
    M = sp.csr_matrix((d, p.col, p.rowptr), shape=(p.n, p.n))
    Ms = (0.5 * (M + M.T)).tocsr()
    rows = np.repeat(np.arange(p.n), np.diff(p.rowptr))
    return np.asarray(Ms[rows, p.col]).ravel()


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
    """128^3 config-5 field: forward and adjoint with the deflated mixed solver."""
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
    x = AG.solve(vals, b, s, mode=esd.DEFLATED, tol=1e-10, maxit=20000, flags=esd.FLAG_MIXED)
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
        xx, info = s.solve(bb, tol=1e-13, maxit=50000)
        assert info["converged"]
        return 0.5 * float(((xx - xt) ** 2).sum())

    errs = []
    for _ in range(3):
        d = _sym_direction(p, rng)
        db = rng.standard_normal(p.n)
        fd = (L(p.val + h * d, p.f + h * db) - L(p.val - h * d, p.f - h * db)) / (2 * h)
        an = gv @ d + gb @ db
        errs.append(abs(fd - an) / abs(an))
    print("config-5 FD relative errors", errs, flush=True)
    # the gradient comes from solves at relres 1e-10 (mixed): its error is
    # bounded by about kappa * 1e-10 relative to the exact gradient
    assert max(errs) <= 1e-4
    s.close()
