"""Host-side checks of the HIP library that need no GPU: it loads and exports
every entry point that include/esd.h declares, and the binding's structure
matches the C struct."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "esd.h")
LIB = os.path.join(ROOT, "paper_2203_08498_amd", "libesd.so")


def declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(esd_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2203_08498_amd import build

        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header(lib):
    from paper_2203_08498_amd import esd

    assert sorted(esd.EXPORTS) == declared()
    L = esd.load_library()
    assert L.esd_status_string(-2).decode().startswith("IC(0)")


def test_binding_constants_match_header():
    """Every mode, flag and status value of include/esd.h has the same value
    in the binding (ESD_X -> esd.X)."""
    from paper_2203_08498_amd import esd

    src = open(HDR).read()
    consts = dict(re.findall(r"#define ESD_([A-Z_0-9]+) (-?\d+)", src))
    consts.update(re.findall(r"\bESD_([A-Z_0-9]+) = (-?\d+)", src))
    assert len(consts) >= 25
    for name, val in consts.items():
        assert getattr(esd, name) == int(val), name


def test_binding_argument_counts_match_header():
    """Every ctypes signature in the binding has as many parameters as the C
    declaration in include/esd.h."""
    from paper_2203_08498_amd import esd

    src = re.sub(r"/\*.*?\*/", "", open(HDR).read(), flags=re.S)
    L = esd.load_library()
    checked = 0
    for name, params in re.findall(r"\b(esd_[a-z_0-9]+)\s*\(([^)]*)\)\s*;", src):
        params = params.strip()
        n = 0 if params in ("", "void") else params.count(",") + 1
        fn = getattr(L, name)
        if fn.argtypes is not None:
            assert len(fn.argtypes) == n, (name, len(fn.argtypes), n)
            checked += 1
    assert checked >= 20


def test_info_struct_layout():
    from paper_2203_08498_amd import esd

    # 8 int32 followed by 9 doubles, no padding
    assert ctypes.sizeof(esd.EsdInfo) == 8 * 4 + 9 * 8


def test_setup_rejects_bad_input_without_gpu(lib):
    # argument validation happens before any device work
    from paper_2203_08498_amd import esd

    L = esd.load_library()
    h = ctypes.c_void_p()
    opt = esd.options(esd.ORDER_NATURAL, 0, esd.PREC_MIXED, 4)
    need = ctypes.c_size_t(7)
    assert L.esd_setup(ctypes.byref(h), None, 0, 0, None, None, None, None, ctypes.byref(opt), None, 0,
                       ctypes.byref(need)) == esd.EINVAL
    assert need.value == 0 and not h.value
    bad = esd.options(esd.ORDER_BLOCK_JACOBI, 0, esd.PREC_MIXED, 4)  # block Jacobi without a block size
    assert L.esd_setup(ctypes.byref(h), None, 4, 4, None, None, None, None, ctypes.byref(bad), None, 0,
                       None) == esd.EINVAL
    assert L.esd_solve(None, None, None, 1e-8, 10, 0, 0, None, None) == esd.EINVAL
    assert L.esd_factor_ic0(None) == esd.EINVAL


def test_solver_refuses_without_gpu():
    import torch

    from paper_2203_08498_amd import esd, problems as P

    if torch.cuda.is_available():
        pytest.skip("GPU present")
    p = P.config1(N=16, nbox=1, box=4)
    with pytest.raises(RuntimeError):
        esd.Solver.from_problem(p)


def test_workspace_bound_arithmetic():
    """esd_workspace_bytes is host arithmetic (no GPU): 0 for invalid
    arguments; it grows with the longest row, m_max and max_iters; an FP64
    context needs less than a mixed one (no FP32 copies); and for a 7-point
    stencil (at most 7 entries per row) the mixed bound at 128^3, m_max = 16,
    lies between the bytes the data structures must hold and that plus a
    small per-row slack."""
    from paper_2203_08498_amd import esd

    n, nnz = 128 ** 3, 14581760
    mixed = esd.options(esd.ORDER_COLORS, 0, esd.PREC_MIXED, 16)
    fp64 = esd.options(esd.ORDER_COLORS, 0, esd.PREC_FP64, 16)
    b = esd.workspace_bytes(n, nnz, 7, mixed)
    assert esd.workspace_bytes(0, 0, 7, mixed) == 0
    assert esd.workspace_bytes(n, nnz, 0, mixed) == 0
    assert esd.workspace_bytes(n, nnz, 7, esd.options(esd.ORDER_COLORS, 0, esd.PREC_MIXED, 65)) == 0
    assert esd.workspace_bytes(n, nnz, 7, esd.options(esd.ORDER_BLOCK_JACOBI, 0, esd.PREC_MIXED, 16)) == 0
    assert esd.workspace_bytes(n, nnz, 8, mixed) > b
    assert esd.workspace_bytes(n, nnz, 7, esd.options(esd.ORDER_COLORS, 0, esd.PREC_MIXED, 32)) > b
    assert esd.workspace_bytes(n, nnz, 7, esd.options(esd.ORDER_COLORS, 0, esd.PREC_MIXED, 16, 200000)) > b
    assert esd.workspace_bytes(n, nnz, 7, fp64) < b
    # what must be stored at least: A's nnz values (FP64 + FP32) with their
    # column indices, 13 FP64 and 10 FP32 vectors, 7 n x m_max FP64 blocks
    # (samples, E, AE, W, AW and row-major W, AW) and 4 FP32 ones; the bound
    # takes every slice of L and U as wide as the longest row less one
    floor = 16 * nnz + 13 * 8 * n + 10 * 4 * n + 16 * n * (7 * 8 + 4 * 4)
    assert floor < b < 2 * floor
