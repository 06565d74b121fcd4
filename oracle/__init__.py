"""ctypes shim over the plain FP64 C oracle (``oracle.c``).

Test infrastructure only: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may use it; the GPU library never does.
Vectors are float64 numpy arrays in the caller's (user) row order.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

PLAIN, DEFLATED, SUBSPACE = 0, 1, 2
NOPREC, POWER, SAMPLE = 1, 2, 4
OK, NOT_CONVERGED, AUX_EMPTY = 0, 1, 2
EINVAL, ENOTSPD, ENUMERIC, ENOAUX, ENOSAMPLES = -1, -2, -4, -5, -6


# ORACLE_SANITIZE=1: a separate build with AddressSanitizer and
# UndefinedBehaviorSanitizer (aborting on the first report), loaded instead
# of the plain one; the process must preload libasan (the sanitizer test does)
_SANITIZE = os.environ.get("ORACLE_SANITIZE") == "1"
if _SANITIZE:
    _SO = os.path.join(_HERE, "liboracle_san.so")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        flags = ["-O2"]
        if _SANITIZE:
            flags = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                     "-fno-omit-frame-pointer"]
        cmd = ["gcc", *flags, "-ffp-contract=off", "-fPIC", "-shared", "-o", _SO, _SRC, "-lm"]
        subprocess.check_call(cmd)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_SO)
        P = C.c_void_p
        i64, i32, dbl = C.c_int64, C.c_int32, C.c_double
        L.orc_create.restype = P
        L.orc_create.argtypes = [i64, P, P, P, P]
        L.orc_create_bj.restype = P
        L.orc_create_bj.argtypes = [i64, P, P, P, i64]
        L.orc_free.argtypes = [P]
        L.orc_perm.argtypes = [P, P]
        L.orc_permuted_csr.argtypes = [P, P, P, P]
        L.orc_permuted_csr.restype = i64
        L.orc_factor_ic0.argtypes = [P]
        L.orc_factor_csr.argtypes = [P, P, P, P]
        L.orc_factor_csr.restype = i64
        L.orc_spmv.argtypes = [P, P, P]
        L.orc_prec_apply.argtypes = [P, P, P]
        L.orc_sample_schedule.argtypes = [C.c_int, i64, P]
        L.orc_arm_sampling.argtypes = [P, C.c_int, C.c_int]
        L.orc_load_samples.argtypes = [P, P, C.c_int, P]
        L.orc_sym_eig.argtypes = [C.c_int, P, P, P]
        L.orc_build_aux.argtypes = [P, dbl, P, P, P]
        L.orc_set_aux.argtypes = [P, P, C.c_int]
        L.orc_aux_dims.argtypes = [P, P, P]
        L.orc_get_aux.argtypes = [P, P, P, P, P]
        L.orc_get_ritz.argtypes = [P, P]
        L.orc_lanczos_extremes.argtypes = [C.c_int, P, P, P, P]
        L.orc_set_power_start.argtypes = [P, P]
        L.orc_solve.argtypes = [P, P, P, dbl, C.c_int, C.c_int, C.c_int, P, P, P]
        L.orc_history.argtypes = [P, P, P]
        L.orc_samples.argtypes = [P, P]
        L.orc_slot_vectors.argtypes = [P, P]
        L.orc_set_rr.argtypes = [P, C.c_int]
        L.orc_grad_values.argtypes = [P, P, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def sample_schedule(m: int, N: int) -> np.ndarray:
    """Iterations kept in each slot by sampling method A for a solve stopping at N."""
    out = np.zeros(m, dtype=np.int64)
    lib().orc_sample_schedule(m, N, _p(out))
    return out


def sym_eig(A: np.ndarray):
    """Cyclic Jacobi eigen-decomposition (ascending) of a symmetric matrix."""
    k = A.shape[0]
    a = np.ascontiguousarray(A, dtype=np.float64).copy()
    w = np.zeros(k)
    V = np.zeros((k, k))
    lib().orc_sym_eig(k, _p(a), _p(w), _p(V))
    return w, V


def lanczos_extremes(alpha, beta):
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    tmin, tmax = C.c_double(), C.c_double()
    lib().orc_lanczos_extremes(len(alpha), _p(alpha), _p(beta), C.byref(tmin), C.byref(tmax))
    return tmin.value, tmax.value


class SolveInfo(dict):
    __getattr__ = dict.get


class Oracle:
    """One matrix, in the given ordering, with its IC(0) factor and auxiliary space."""

    def __init__(self, rowptr, col, val, colors=None, block_rows=None):
        """colors: ordering by a stable sort on colour (None: natural order).
        block_rows: block-Jacobi IC(0) (Sec. 5.3) with blocks of that many
        consecutive rows in natural order (colors must then be None)."""
        self.rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.colors = None if colors is None else np.ascontiguousarray(colors, dtype=np.int32)
        self.block_rows = block_rows
        self.n = self.rowptr.shape[0] - 1
        if block_rows is not None:
            if colors is not None:
                raise ValueError("oracle: block Jacobi takes the natural order")
            self.h = lib().orc_create_bj(self.n, _p(self.rowptr), _p(self.col), _p(self.val), int(block_rows))
        else:
            self.h = lib().orc_create(self.n, _p(self.rowptr), _p(self.col), _p(self.val), _p(self.colors))
        if not self.h:
            raise ValueError("oracle: bad matrix")

    @classmethod
    def from_problem(cls, prob, block_rows=None):
        return cls(prob.rowptr, prob.col, prob.val, None if block_rows is not None else prob.colors,
                   block_rows=block_rows)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_free(h)
            self.h = None

    @property
    def perm(self):
        out = np.zeros(self.n, dtype=np.int32)
        lib().orc_perm(self.h, _p(out))
        return out

    def permuted_csr(self):
        nnz = int(self.rowptr[-1])
        rp = np.zeros(self.n + 1, np.int64)
        c = np.zeros(nnz, np.int32)
        v = np.zeros(nnz)
        lib().orc_permuted_csr(self.h, _p(rp), _p(c), _p(v))
        return rp, c, v

    def factor_ic0(self) -> int:
        return lib().orc_factor_ic0(self.h)

    def factor_csr(self):
        cnt = lib().orc_factor_csr(self.h, None, None, None)
        rp = np.zeros(self.n + 1, np.int64)
        c = np.zeros(cnt, np.int32)
        v = np.zeros(cnt)
        lib().orc_factor_csr(self.h, _p(rp), _p(c), _p(v))
        return rp, c, v

    def spmv(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.n)
        lib().orc_spmv(self.h, _p(x), _p(y))
        return y

    def prec(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.zeros(self.n)
        st = lib().orc_prec_apply(self.h, _p(r), _p(z))
        if st != 0:
            raise RuntimeError("oracle prec: status %d" % st)
        return z

    def arm_sampling(self, m: int, method: int = 0, residuals: bool = False):
        """method 0: sampling method A (Appendix A); 1: method B (relative-
        residual thresholds, Sec. 4.3).  residuals: store r_i instead of x_i."""
        st = lib().orc_arm_sampling(self.h, m, int(method) | (16 if residuals else 0))
        if st != 0:
            raise ValueError("bad m or method")

    def load_samples(self, X, xN):
        """X: n x k approximate solutions (taken as iterations 1..k), xN: final solution."""
        X = np.asfortranarray(X, dtype=np.float64)
        xN = np.ascontiguousarray(xN, dtype=np.float64)
        st = lib().orc_load_samples(self.h, X.ctypes.data_as(C.c_void_p), X.shape[1], _p(xN))
        if st != 0:
            raise ValueError("bad samples")

    def set_power_start(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64)
        lib().orc_set_power_start(self.h, _p(v))

    def solve(self, b, x0=None, tol=1e-8, maxit=10000, mode=PLAIN, flags=0):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x0 = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        x = np.zeros(self.n)
        iout = np.zeros(4, np.int32)
        dout = np.zeros(8)
        st = lib().orc_solve(self.h, _p(b), _p(x0), float(tol), int(maxit), int(mode), int(flags),
                             _p(x), _p(iout), _p(dout))
        info = SolveInfo(status=st, iters=int(iout[0]), converged=bool(iout[1]), m_tilde=int(iout[2]),
                         nsamples=int(iout[3]), relres=dout[0], true_relres=dout[1], kappa=dout[2],
                         kappa_es=dout[3], lambda_max=dout[4], lambda_min_ritz=dout[5],
                         lanczos_min=dout[6], lanczos_max=dout[7])
        if st < 0:
            raise RuntimeError("oracle solve failed: status %d" % st)
        return x, info

    def history(self):
        k = lib().orc_history(self.h, None, None)
        a = np.zeros(max(k, 1))
        b = np.zeros(max(k - 1, 1))
        lib().orc_history(self.h, _p(a), _p(b))
        return a[:k], b[:max(k - 1, 0)]

    def samples(self, m):
        out = np.zeros(m, np.int32)
        lib().orc_samples(self.h, _p(out))
        return out

    def slot_vectors(self, m):
        """Stored sample vectors, n x m (user order); unfilled slots are undefined."""
        out = np.zeros((self.n, m), order="F")
        lib().orc_slot_vectors(self.h, out.ctypes.data_as(C.c_void_p))
        return out

    def set_rayleigh_ritz(self, op: int):
        """Operator of the next build_aux: 0 = A (eq. (Rayleigh-Ritz)), 1 = the
        preconditioned matrix M^{-1}A in the M inner product (its footnote)."""
        if lib().orc_set_rr(self.h, int(op)) != 0:
            raise ValueError("bad Rayleigh-Ritz operator (or no IC(0) factor)")

    def build_aux(self, theta: float):
        ritz = np.zeros(4096)
        mb, mt = C.c_int(), C.c_int()
        st = lib().orc_build_aux(self.h, float(theta), _p(ritz), C.byref(mb), C.byref(mt))
        if st < 0:
            raise RuntimeError("oracle build_aux failed: status %d" % st)
        return st, ritz[: mb.value].copy(), mb.value, mt.value

    def set_aux(self, W):
        W = np.asfortranarray(W, dtype=np.float64)
        k = W.shape[1]
        st = lib().orc_set_aux(self.h, W.ctypes.data_as(C.c_void_p), k)
        if st < 0:
            raise RuntimeError("oracle set_aux failed: status %d" % st)
        return st

    def aux(self):
        mb, mt = C.c_int(), C.c_int()
        lib().orc_aux_dims(self.h, C.byref(mb), C.byref(mt))
        mb, mt = mb.value, mt.value
        E = np.zeros((self.n, mb), order="F")
        W = np.zeros((self.n, mt), order="F")
        AW = np.zeros((self.n, mt), order="F")
        Cm = np.zeros((mt, mt))
        lib().orc_get_aux(self.h, E.ctypes.data_as(C.c_void_p) if mb else None,
                          W.ctypes.data_as(C.c_void_p) if mt else None,
                          AW.ctypes.data_as(C.c_void_p) if mt else None, _p(Cm) if mt else None)
        return E, W, AW, Cm

    def grad_values(self, lam, x):
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        g = np.zeros(int(self.rowptr[-1]))
        lib().orc_grad_values(self.h, _p(lam), _p(x), _p(g))
        return g
