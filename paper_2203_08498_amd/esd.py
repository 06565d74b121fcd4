"""Thin ctypes binding of the esd C ABI (``include/esd.h``).

Argument marshalling only: every step of the solver runs in the HIP kernels of
``libesd.so``.  Device vectors are torch float64 CUDA tensors; the library is
given torch's current HIP stream.  There is no CPU fallback: without the
built library or a GPU every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libesd.so")

PLAIN, DEFLATED, SUBSPACE = 0, 1, 2
FLAG_NOPREC, FLAG_POWER, FLAG_MIXED, FLAG_SYNC_EVERY, FLAG_TIMING, FLAG_TIMING_SPMV, FLAG_TRUE_RES = 1, 2, 4, 8, 16, 32, 64
FLAG_STREAM = 128
FLAG_MIXED_KEEP = 256
FLAG_MIXED_ADAPT = 512
SAMPLING_A, SAMPLING_B, SAMPLE_RESIDUALS = 0, 1, 16
RR_A, RR_PRECONDITIONED = 0, 1
OK, NOT_CONVERGED, AUX_EMPTY = 0, 1, 2
EINVAL, ENOTSPD, EHIP, ENUMERIC, ENOAUX, ENOSAMPLES, EWORKSPACE = -1, -2, -3, -4, -5, -6, -7
ORDER_NATURAL, ORDER_COLORS, ORDER_BLOCK_JACOBI = 0, 1, 2
PROBE_COPY, PROBE_READ = 0, 1
PREC_FP64, PREC_MIXED = 0, 1


class EsdOptions(C.Structure):
    _fields_ = [("order", C.c_int32), ("block_rows", C.c_int32), ("prec", C.c_int32), ("m_max", C.c_int32),
                ("max_iters", C.c_int32), ("reserved", C.c_int32 * 3)]


class EsdInfo(C.Structure):
    _fields_ = [
        ("iters", C.c_int32), ("outer_iters", C.c_int32), ("converged", C.c_int32),
        ("m_tilde", C.c_int32), ("nsamples", C.c_int32), ("mode_used", C.c_int32),
        ("fp64_iters", C.c_int32), ("reserved", C.c_int32),
        ("relres", C.c_double), ("true_relres", C.c_double), ("kappa", C.c_double),
        ("kappa_es", C.c_double), ("lambda_max", C.c_double), ("lambda_min_ritz", C.c_double),
        ("lanczos_min", C.c_double), ("lanczos_max", C.c_double), ("seconds", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = [
    "esd_workspace_bytes", "esd_setup", "esd_workspace_used", "esd_update_values", "esd_factor_ic0", "esd_sample_errors", "esd_load_samples", "esd_build_aux", "esd_set_aux", "esd_get_aux",
    "esd_hbm_probe", "esd_set_power_start", "esd_set_mixed_params", "esd_solve", "esd_solve_noalloc", "esd_sequence_rhs", "esd_grad_values", "esd_spmv",
    "esd_prec_apply", "esd_get_perm", "esd_get_factor_diag", "esd_get_history", "esd_get_samples",
    "esd_get_sample_vector", "esd_set_rayleigh_ritz",
    "esd_get_layout", "esd_get_timing", "esd_status_string", "esd_last_error", "esd_destroy",
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libesd.so and declare the signatures (no GPU needed to load)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libesd.so is not built (run __graft_entry__.build() or "
                           "python paper_2203_08498_amd/build.py): %s" % path)
    L = C.CDLL(path)
    P, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.esd_workspace_bytes.argtypes = [i64, i64, i32, C.POINTER(EsdOptions)]
    L.esd_workspace_bytes.restype = C.c_size_t
    L.esd_setup.argtypes = [C.POINTER(P), P, i64, i64, P, P, P, P, C.POINTER(EsdOptions), P, C.c_size_t,
                            C.POINTER(C.c_size_t)]
    L.esd_workspace_used.argtypes = [P, C.POINTER(C.c_size_t)]
    L.esd_hbm_probe.argtypes = [P, i32, P, P, i64, i32]
    L.esd_hbm_probe.restype = C.c_int
    L.esd_factor_ic0.argtypes = [P]
    L.esd_update_values.argtypes = [P, P]
    L.esd_sample_errors.argtypes = [P, i32, i32]
    L.esd_load_samples.argtypes = [P, P, i32, P]
    L.esd_build_aux.argtypes = [P, dbl, P, P, P]
    L.esd_set_aux.argtypes = [P, P, i32]
    L.esd_get_aux.argtypes = [P, P, P]
    L.esd_set_power_start.argtypes = [P, P]
    L.esd_set_mixed_params.argtypes = [P, dbl, i32]
    L.esd_solve.argtypes = [P, P, P, dbl, i32, i32, i32, P, C.POINTER(EsdInfo)]
    L.esd_solve_noalloc.argtypes = [P, P, P, dbl, i32, i32, i32, P, C.POINTER(EsdInfo)]
    L.esd_sequence_rhs.argtypes = [P, P, P, dbl, P]
    L.esd_grad_values.argtypes = [P, P, P, P]
    L.esd_spmv.argtypes = [P, P, P]
    L.esd_prec_apply.argtypes = [P, P, P]
    L.esd_get_perm.argtypes = [P, P]
    L.esd_get_factor_diag.argtypes = [P, P]
    L.esd_get_history.argtypes = [P, P, P, i32, P]
    L.esd_get_samples.argtypes = [P, P]
    L.esd_get_sample_vector.argtypes = [P, i32, P]
    L.esd_set_rayleigh_ritz.argtypes = [P, i32]
    L.esd_get_layout.argtypes = [P, P]
    L.esd_get_timing.argtypes = [P, P]
    L.esd_status_string.argtypes = [C.c_int]
    L.esd_status_string.restype = C.c_char_p
    L.esd_last_error.argtypes = [P]
    L.esd_last_error.restype = C.c_char_p
    L.esd_destroy.argtypes = [P]
    for name in ("esd_setup", "esd_workspace_used", "esd_update_values", "esd_factor_ic0", "esd_sample_errors", "esd_load_samples", "esd_build_aux",
                 "esd_set_aux",
                 "esd_get_aux", "esd_set_power_start", "esd_set_mixed_params", "esd_solve", "esd_solve_noalloc", "esd_sequence_rhs",
                 "esd_grad_values", "esd_spmv", "esd_prec_apply", "esd_get_perm", "esd_get_factor_diag",
                 "esd_get_history", "esd_get_samples", "esd_get_sample_vector", "esd_get_layout", "esd_get_timing",
                 "esd_set_rayleigh_ritz"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


class EsdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("esd status %d: %s" % (status, msg))
        self.status = status


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def options(order=ORDER_COLORS, block_rows=0, prec=PREC_MIXED, m_max=16, max_iters=0):
    o = EsdOptions()
    o.order, o.block_rows, o.prec, o.m_max, o.max_iters = int(order), int(block_rows), int(prec), int(m_max), \
        int(max_iters)
    return o


def workspace_bytes(n, nnz, max_row, opt):
    """esd_workspace_bytes: upper bound of the device workspace esd_setup needs."""
    return int(load_library().esd_workspace_bytes(int(n), int(nnz), int(max_row), C.byref(opt)))


class Solver:
    """One SPD matrix on the GPU: ordering, IC(0) factor, auxiliary space W.

    The device workspace is a torch uint8 tensor sized by esd_workspace_bytes
    (held by this object for the context's life); the CSR is handed to
    esd_setup as device tensors and dropped afterwards."""

    def __init__(self, rowptr, col, val, colors=None, m_max: int = 16, device="cuda:0", block_rows=None,
                 precision: str = "mixed", max_iters: int = 100000):
        """colors: ordering by a stable sort on colour (None: natural order).
        block_rows: block-Jacobi IC(0) (Sec. 5.3) with blocks of that many
        consecutive rows (natural order; colors must be None).
        precision: "mixed" keeps FP32 copies for ESD_FLAG_MIXED, "fp64" does not.
        max_iters: the largest maxit a solve may use."""
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("esd.Solver needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.torch = torch
        self.device = torch.device(device)
        self.L = load_library()
        rowptr = _np(rowptr, np.int64)
        self.n = rowptr.shape[0] - 1
        self.nnz = int(rowptr[-1])
        self.m_max = m_max
        self.block_rows = block_rows
        if block_rows is not None and colors is not None:
            raise ValueError("block Jacobi keeps the natural order: pass colors=None")
        if precision not in ("mixed", "fp64"):
            raise ValueError("precision is 'mixed' or 'fp64'")
        if block_rows is not None:
            order = ORDER_BLOCK_JACOBI
        else:
            order = ORDER_NATURAL if colors is None else ORDER_COLORS
        self.opt = options(order, 0 if block_rows is None else block_rows,
                           PREC_MIXED if precision == "mixed" else PREC_FP64, m_max, max_iters)
        max_row = int(np.diff(rowptr).max()) if self.n > 0 else 1
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            dev = dict(device=self.device)
            rp = torch.as_tensor(rowptr, **dev)
            cl = torch.as_tensor(_np(col, np.int32), **dev)
            vl = torch.as_tensor(_np(val, np.float64), **dev)
            co = None if colors is None else torch.as_tensor(_np(colors, np.int32), **dev)
            nbytes = self.L.esd_workspace_bytes(self.n, self.nnz, max_row, C.byref(self.opt))
            if nbytes == 0:
                raise EsdError(EINVAL, "invalid setup arguments")
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, **dev)
            h = C.c_void_p()
            need = C.c_size_t()
            torch.cuda.synchronize(self.device)
            t0 = time.perf_counter()
            st = self.L.esd_setup(C.byref(h), C.c_void_p(self.stream.cuda_stream), self.n, self.nnz, _dptr(rp),
                                  _dptr(cl), _dptr(vl), None if co is None else _dptr(co), C.byref(self.opt),
                                  _dptr(self.workspace), nbytes, C.byref(need))
            self.setup_s = time.perf_counter() - t0  # esd_setup synchronises before returning
            del rp, cl, vl, co
        if st != 0:
            raise EsdError(st, self.L.esd_status_string(st).decode())
        self.h = h
        self.ws_needed = need.value

    @classmethod
    def from_problem(cls, prob, m_max=None, block_rows=None, **kw):
        return cls(prob.rowptr, prob.col, prob.val, None if block_rows is not None else prob.colors,
                   m_max=prob.params.get("m", 16) if m_max is None else m_max, block_rows=block_rows, **kw)

    # -------------------------------------------------------------- plumbing
    def _check(self, st):
        if st < 0:
            raise EsdError(st, self.L.esd_last_error(self.h).decode())
        return st

    def _vec(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            a = a.to(device=self.device, dtype=t.float64)
        else:
            a = t.as_tensor(np.asarray(a, dtype=np.float64), device=self.device)
        return a.contiguous()

    def close(self):
        if getattr(self, "h", None):
            self.torch.cuda.synchronize(self.device)
            self.L.esd_destroy(self.h)
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- API
    def factor_ic0(self):
        st = self.L.esd_factor_ic0(self.h)
        if st != 0:
            raise EsdError(st, self.L.esd_last_error(self.h).decode())

    def update_values(self, val):
        """New stored values (same pattern, caller CSR order); call factor_ic0 afterwards."""
        v = self._vec(val)
        if v.numel() != self.nnz:
            raise ValueError("expected %d values" % self.nnz)
        self._check(self.L.esd_update_values(self.h, _dptr(v)))

    def sample_errors(self, m: int, method: int = 0, residuals: bool = False):
        """Arm sampling for the next solve: method 0 = sampling method A
        (Appendix A), 1 = method B (relative-residual thresholds, Sec. 4.3);
        residuals=True stores r_i instead of x_i (Sec. 5.2)."""
        code = int(method) | (SAMPLE_RESIDUALS if residuals else 0)
        st = self.L.esd_sample_errors(self.h, int(m), code)
        if st != 0:
            raise EsdError(st, self.L.esd_last_error(self.h).decode())

    def load_samples(self, X, xN):
        """X: n x k approximate solutions (as sampled at iterations 1..k), xN: final solution."""
        X = self._vec(X)
        Xc = X.t().contiguous()
        xN = self._vec(xN)
        self._check(self.L.esd_load_samples(self.h, _dptr(Xc), int(X.shape[1]), _dptr(xN)))

    def build_aux(self, theta: float):
        ritz = np.zeros(max(self.m_max, 1))
        mb, mt = C.c_int32(), C.c_int32()
        st = self.L.esd_build_aux(self.h, float(theta), ritz.ctypes.data_as(C.c_void_p), C.byref(mb), C.byref(mt))
        self._check(st)
        self.m_tilde = mt.value
        return st, ritz[: mb.value].copy(), mb.value, mt.value

    def set_aux(self, W):
        W = self._vec(W)
        k = W.shape[1]
        Wc = W.t().contiguous()  # column-major n x k
        st = self.L.esd_set_aux(self.h, _dptr(Wc), int(k))
        self.torch.cuda.synchronize(self.device)
        self._check(st)
        self.m_tilde = int(k)
        return st

    def get_aux(self):
        """W (n x m_tilde, user order) as a torch tensor and C = W^T A W (numpy)."""
        mt = getattr(self, "m_tilde", 0)
        Wt = self.torch.zeros((max(mt, 1), self.n), dtype=self.torch.float64, device=self.device)
        Cm = np.zeros((max(mt, 1), max(mt, 1)))
        self._check(self.L.esd_get_aux(self.h, _dptr(Wt), Cm.ctypes.data_as(C.c_void_p)))
        return Wt[:mt].t(), Cm[:mt, :mt]

    def set_power_start(self, v0):
        v0 = self._vec(v0)
        st = self.L.esd_set_power_start(self.h, _dptr(v0))
        self.torch.cuda.synchronize(self.device)
        if st != 0:
            raise EsdError(st, self.L.esd_last_error(self.h).decode())

    def set_mixed_params(self, inner_tol: float = 1e-4, max_outer: int = 30):
        st = self.L.esd_set_mixed_params(self.h, float(inner_tol), int(max_outer))
        if st != 0:
            raise EsdError(st, "bad mixed parameters")

    def solve(self, b, x0=None, tol=1e-8, maxit=10000, mode=PLAIN, flags=0, out=None, noalloc=False):
        """esd_solve (noalloc=True: esd_solve_noalloc, which allocates nothing)."""
        b = self._vec(b)
        x0 = None if x0 is None else self._vec(x0)
        x = out if out is not None else self.torch.empty(self.n, dtype=self.torch.float64, device=self.device)
        info = EsdInfo()
        fn = self.L.esd_solve_noalloc if noalloc else self.L.esd_solve
        st = fn(self.h, _dptr(b), None if x0 is None else _dptr(x0), float(tol), int(maxit),
                int(mode), int(flags), _dptr(x), C.byref(info))
        if st < 0:
            raise EsdError(st, self.L.esd_last_error(self.h).decode())
        d = info.as_dict()
        d["status"] = st
        return x, d

    def sequence_rhs(self, f, xprev=None, c=0.1, out=None):
        """b = f + c * xprev on the device (b = f without xprev)."""
        f = self._vec(f)
        xprev = None if xprev is None else self._vec(xprev)
        b = out if out is not None else self.torch.empty(self.n, dtype=self.torch.float64, device=self.device)
        self._check(self.L.esd_sequence_rhs(self.h, _dptr(f), None if xprev is None else _dptr(xprev), float(c),
                                            _dptr(b)))
        return b

    def grad_values(self, lam, x):
        lam, x = self._vec(lam), self._vec(x)
        g = self.torch.empty(self.nnz, dtype=self.torch.float64, device=self.device)
        st = self.L.esd_grad_values(self.h, _dptr(lam), _dptr(x), _dptr(g))
        if st != 0:
            raise EsdError(st, self.L.esd_last_error(self.h).decode())
        return g

    def spmv(self, x):
        x = self._vec(x)
        y = self.torch.empty(self.n, dtype=self.torch.float64, device=self.device)
        st = self.L.esd_spmv(self.h, _dptr(x), _dptr(y))
        if st != 0:
            raise EsdError(st, self.L.esd_last_error(self.h).decode())
        return y

    def prec(self, r):
        r = self._vec(r)
        z = self.torch.empty(self.n, dtype=self.torch.float64, device=self.device)
        st = self.L.esd_prec_apply(self.h, _dptr(r), _dptr(z))
        if st != 0:
            raise EsdError(st, self.L.esd_last_error(self.h).decode())
        return z

    def perm(self):
        out = np.zeros(self.n, np.int32)
        self._check(self.L.esd_get_perm(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def factor_diag(self):
        out = np.zeros(self.n)
        self._check(self.L.esd_get_factor_diag(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def history(self, cap=1 << 20):
        cnt = C.c_int32()
        self.L.esd_get_history(self.h, None, None, 0, C.byref(cnt))
        k = cnt.value
        a = np.zeros(max(k, 1))
        b = np.zeros(max(k, 1))
        self.L.esd_get_history(self.h, a.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p), max(k, 1),
                               C.byref(cnt))
        return a[:k], b[:max(k - 1, 0)]

    def samples(self, m):
        out = np.zeros(m, np.int32)
        self._check(self.L.esd_get_samples(self.h, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_rayleigh_ritz(self, op: int):
        """0: Rayleigh-Ritz with A (eq. (Rayleigh-Ritz)); 1: with the
        preconditioned matrix M^{-1}A in the M inner product (its footnote)."""
        self._check(self.L.esd_set_rayleigh_ritz(self.h, int(op)))

    def sample_vector(self, slot: int):
        """The vector stored in sampling slot `slot` (user order, float64 tensor)."""
        import torch

        out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        self._check(self.L.esd_get_sample_vector(self.h, int(slot), _dptr(out)))
        return out

    def workspace_used(self):
        out = C.c_size_t()
        self._check(self.L.esd_workspace_used(self.h, C.byref(out)))
        return int(out.value)

    def layout(self):
        out = np.zeros(8, np.int32)
        self._check(self.L.esd_get_layout(self.h, out.ctypes.data_as(C.c_void_p)))
        return dict(n=int(out[0]), nnz=int(out[1]), levels=int(out[2]), colors=int(out[3]),
                    class_layout=(bool(out[4]), bool(out[5]), bool(out[6])), a_slots=int(out[7]))

    def timing(self):
        out = np.zeros(4)
        self._check(self.L.esd_get_timing(self.h, out.ctypes.data_as(C.c_void_p)))
        return dict(spmv_ms=out[0], sweep_ms=out[1], update_ms=out[2], iters=int(out[3]))


def hbm_probe(kind, src, dst, grid=0, stream=None):
    """esd_hbm_probe on torch float64 CUDA tensors (enqueued, no sync)."""
    import torch

    st = torch.cuda.current_stream() if stream is None else stream
    r = load_library().esd_hbm_probe(C.c_void_p(st.cuda_stream), int(kind), _dptr(src), _dptr(dst),
                                     int(src.numel()), int(grid))
    if r != 0:
        raise EsdError(r, "bad probe arguments")
