"""esd_solve_noalloc, the allocation-free variant of esd_solve (its per-solve
scratch in a static device array instead of the context's workspace), called
through the C ABI and checked against esd_solve with stream launches: the
same kernels in the same order, so the results must be bit-identical.  Two
problems in a row, the second smaller, so that the second call runs on what
the first left in the shared array."""
import ctypes

import numpy as np
import pytest

from paper_2203_08498_amd import problems as P

pytestmark = pytest.mark.gpu


def _call(s, fn, b, tol, maxit, mode, flags):
    import torch

    from paper_2203_08498_amd import esd

    x = torch.empty(s.n, dtype=torch.float64, device=s.device)
    info = esd.EsdInfo()
    st = fn(s.h, esd._dptr(b), None, float(tol), int(maxit), int(mode), int(flags), esd._dptr(x), ctypes.byref(info))
    return st, x, info


def test_noalloc_solve_matches_solve_on_two_problems():
    import torch

    from paper_2203_08498_amd import esd

    problems = [("24^3", P.config2(N=24, nsph=4, radius=3.0)), ("13^3", P.config2(N=13, nsph=2, radius=2.5))]
    for name, p in problems:
        print("no-alloc solve on", name, "n", p.n, flush=True)
        s = esd.Solver.from_problem(p, m_max=8)
        try:
            s.factor_ic0()
            W, _ = np.linalg.qr(np.random.default_rng(4).standard_normal((p.n, 6)))
            s.set_aux(W)
            b = torch.as_tensor(p.f, device=s.device)
            L = s.L
            for mode, flags in ((esd.PLAIN, 0), (esd.DEFLATED, 0), (esd.SUBSPACE, 0),
                                (esd.DEFLATED, esd.FLAG_MIXED), (esd.PLAIN, esd.FLAG_MIXED | esd.FLAG_MIXED_KEEP)):
                st_r, x_r, i_r = _call(s, L.esd_solve, b, 1e-8, 5000, mode, flags | esd.FLAG_STREAM)
                st_n, x_n, i_n = _call(s, L.esd_solve_noalloc, b, 1e-8, 5000, mode, flags)
                print(name, "mode", mode, "flags", flags, "iters", i_n.iters, i_r.iters, flush=True)
                assert st_n == st_r == 0
                assert i_n.iters == i_r.iters and i_n.outer_iters == i_r.outer_iters
                assert torch.equal(x_n, x_r)
                assert i_n.kappa == i_r.kappa and i_n.true_relres == i_r.true_relres
                assert i_n.true_relres <= 1e-8
            # a sampling solve: the same sampled iterations and stored vectors
            s.sample_errors(8)
            _, x_r, i_r = _call(s, L.esd_solve, b, 1e-8, 5000, esd.PLAIN, esd.FLAG_STREAM)
            its_r = s.samples(8)
            vec_r = [s.sample_vector(k) for k in range(8)]
            s.sample_errors(8)
            _, x_n, i_n = _call(s, L.esd_solve_noalloc, b, 1e-8, 5000, esd.PLAIN, 0)
            assert np.array_equal(s.samples(8), its_r) and (its_r > 0).all()
            for k in range(8):
                assert torch.equal(s.sample_vector(k), vec_r[k])
            # timing needs events: refused
            st, _, _ = _call(s, L.esd_solve_noalloc, b, 1e-8, 5000, esd.PLAIN, esd.FLAG_TIMING)
            assert st == esd.EINVAL
        finally:
            s.close()
