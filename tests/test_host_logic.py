"""Host-side logic of the esd library, checked on the CPU through a small C++
driver (tests/host_driver.cpp) compiled with g++ against csrc/host_setup.cpp:
colour ordering and level schedule, the sorted and class-aligned sliced-ELL
layouts (decoded back to coordinates and compared with the CSR input), the
XCD tile orders, the sampling-A table, and the small dense routines (Jacobi
eigensolver, generalised eigensolver, Cholesky inverse, Lanczos extremes)
against numpy / scipy."""
import os
import subprocess

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import oracle as O
from paper_2203_08498_amd import problems as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_08498_amd", "csrc")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("host") / "host_driver")
    # ESD_HOST_SANITIZE=1: the driver and the host setup code built with
    # AddressSanitizer and UndefinedBehaviorSanitizer (abort on the first report)
    san = ["-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"] \
        if os.environ.get("ESD_HOST_SANITIZE") == "1" else []
    subprocess.check_call(["g++", "-O1", *san, "-std=c++17", "-fopenmp", "-I", CSRC, "-I",
                           os.path.join(ROOT, "include"), os.path.join(os.path.dirname(__file__), "host_driver.cpp"),
                           os.path.join(CSRC, "host_setup.cpp"), "-o", exe])
    return exe


class _Reader:
    def __init__(self, path):
        self.b = open(path, "rb").read()
        self.o = 0

    def one(self, dt):
        v = np.frombuffer(self.b, dtype=dt, count=1, offset=self.o)[0]
        self.o += np.dtype(dt).itemsize
        return v

    def vec(self, dt):
        n = int(self.one(np.int64))
        v = np.frombuffer(self.b, dtype=dt, count=n, offset=self.o).copy()
        self.o += n * np.dtype(dt).itemsize
        return v


def _run_layout(driver, tmp, p, block_rows=0):
    fin, fout = os.path.join(tmp, "csr.bin"), os.path.join(tmp, "layout.bin")
    with open(fin, "wb") as f:
        f.write(np.int64(p.n).tobytes())
        f.write(np.int64(p.nnz).tobytes())
        f.write(np.int32(0 if p.colors is None else 1).tobytes())
        f.write(np.int64(block_rows).tobytes())
        f.write(np.asarray(p.rowptr, np.int64).tobytes())
        f.write(np.asarray(p.col, np.int32).tobytes())
        f.write(np.asarray(p.val, np.float64).tobytes())
        if p.colors is not None:
            f.write(np.asarray(p.colors, np.int32).tobytes())
    subprocess.check_call([driver, "layout", fin, fout])
    R = _Reader(fout)
    out = {"ok": int(R.one(np.int32))}
    if not out["ok"]:
        out["why"] = R.b[R.o:].decode()
        return out
    for k, dt in (("lperm", np.int32), ("p2u", np.int32), ("p2l", np.int32), ("lvl", np.int64)):
        out[k] = R.vec(dt)
    for name in ("A", "L", "U"):
        out[name] = (R.vec(np.int64), R.vec(np.int64), R.vec(np.float64))
        out[name + "_cls"] = int(R.one(np.int32))
        out[name + "_c"] = (R.vec(np.int64), R.vec(np.int64), R.vec(np.float64))
    out["tf"], out["tl"], out["toff"] = R.vec(np.int32), R.vec(np.int32), R.vec(np.int64)
    out["tf4"], out["tl2"], out["toff2"] = R.vec(np.int32), R.vec(np.int32), R.vec(np.int64)
    return out


def _greedy_colouring(A):
    n = A.shape[0]
    col = -np.ones(n, np.int32)
    for i in range(n):
        used = set(col[A.indices[A.indptr[i]:A.indptr[i + 1]]])
        c = 0
        while c in used:
            c += 1
        col[i] = c
    return col


def _random_spd(n=700, seed=4):
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=6.0 / n, random_state=rng, format="csr")
    M = M + M.T
    M.data[:] = -np.abs(M.data)
    d = np.asarray(abs(M).sum(axis=1)).ravel() + 1.0
    A = (M + sp.diags(d)).tocsr()
    A.sort_indices()
    return P.Problem(name="random_spd", n=n, rowptr=A.indptr.astype(np.int64), col=A.indices.astype(np.int32),
                     val=A.data.astype(np.float64), colors=_greedy_colouring(A), f=np.ones(n), shape=(n,), params={})


def _cases():
    return {
        "fv2d_natural": P.config1(N=24, nbox=2, box=4),
        "fv3d_12": P.config2(N=12, nsph=1, radius=2.0),
        "fv3d_16": P.config2(N=16, nsph=1, radius=2.0),
        "q1_7": P.config4(Ne=7, nblk=1, blk=2),
        "random_spd": _random_spd(),
    }


CASES = _cases()


@pytest.mark.parametrize("name", list(CASES))
def test_layout_reproduces_the_matrix(driver, tmp_path, name):
    p = CASES[name]
    out = _run_layout(driver, str(tmp_path), p)
    assert out["ok"] == 1
    n = p.n
    # logical order: stable sort by colour (identity without colours)
    want = np.arange(n) if p.colors is None else np.argsort(p.colors, kind="stable")
    assert np.array_equal(out["lperm"], want)
    lpos = np.empty(n, np.int64)
    lpos[want] = np.arange(n)
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(n, n))
    # levels: longest chain of logically-earlier couplings, by brute force
    lev = np.zeros(n, np.int64)
    for l in range(n):
        u = want[l]
        nb = lpos[A.indices[A.indptr[u]:A.indptr[u + 1]]]
        earlier = nb[nb < l]
        lev[l] = 1 + lev[earlier].max() if earlier.size else 0
    counts = np.bincount(lev)
    assert np.array_equal(np.diff(out["lvl"]), counts)
    # physical order: level-major, logical order inside a level
    assert np.array_equal(out["p2l"], np.lexsort((np.arange(n), lev)))
    assert np.array_equal(out["p2u"], want[out["p2l"]])
    p2u = out["p2u"]
    coo = A.tocoo()
    ref = {(int(i), int(j)): v for i, j, v in zip(coo.row, coo.col, coo.data)}

    def user_set(t):
        r, c, v = t
        return {(int(p2u[a]), int(p2u[b])): x for a, b, x in zip(r, c, v)}

    assert user_set(out["A"]) == ref
    low = {k: v for k, v in ref.items() if lpos[k[1]] < lpos[k[0]]}
    assert user_set(out["L"]) == low
    assert set(user_set(out["U"])) == {(j, i) for (i, j) in low}
    for m in ("A", "L", "U"):
        if out[m + "_cls"]:
            got = sorted(zip(*[x.tolist() for x in out[m + "_c"]]))
            exp = sorted(zip(*[x.tolist() for x in out[m]]))
            assert got == exp
    # tile orders are permutations of the tiles of each range, with one or
    # several parts per eighth
    nt = (n + 255) // 256
    for tf, tl, toff in ((out["tf"], out["tl"], out["toff"]), (out["tf4"], out["tl2"], out["toff2"])):
        assert np.array_equal(np.sort(tf), np.arange(nt))
        for lv in range(len(out["lvl"]) - 1):
            rows = out["lvl"][lv + 1] - out["lvl"][lv]
            seg = tl[toff[lv]:toff[lv + 1]]
            assert np.array_equal(np.sort(seg), np.arange((rows + 255) // 256))
    assert np.array_equal(out["toff"], out["toff2"])


def test_class_layout_is_taken_where_it_fits(driver, tmp_path):
    out = _run_layout(driver, str(tmp_path), CASES["fv3d_16"])
    assert (out["A_cls"], out["L_cls"], out["U_cls"]) == (1, 1, 1)
    # no padding beyond the sorted layout for an even 3-D grid
    assert len(out["A_c"][0]) == len(out["A"][0])
    out = _run_layout(driver, str(tmp_path), CASES["random_spd"])
    assert out["A_cls"] == 0  # unstructured: offsets spread too widely, sorted layout kept


def test_layout_rejects_coupled_rows_of_one_colour(driver, tmp_path):
    p = CASES["fv3d_12"]
    bad = P.Problem(name="bad", n=p.n, rowptr=p.rowptr, col=p.col, val=p.val, colors=np.zeros(p.n, np.int32),
                    f=p.f, shape=p.shape, params={})
    assert _run_layout(driver, str(tmp_path), bad)["ok"] == 0


@pytest.mark.parametrize("name,s", [("fv3d_12", 12), ("fv3d_12", 5), ("fv2d_natural", 24), ("q1_7", 6)])
def test_block_jacobi_layout(driver, tmp_path, name, s):
    """Block Jacobi: natural order in one level; A keeps every entry, L / U
    hold exactly the couplings inside blocks of s consecutive rows."""
    base = CASES[name]
    p = P.Problem(name=name, n=base.n, rowptr=base.rowptr, col=base.col, val=base.val, colors=None, f=base.f,
                  shape=base.shape, params={})
    out = _run_layout(driver, str(tmp_path), p, block_rows=s)
    assert out["ok"] == 1, out.get("why")
    n = p.n
    assert np.array_equal(out["p2u"], np.arange(n)) and list(out["lvl"]) == [0, n]
    coo = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(n, n)).tocoo()
    ref = {(int(i), int(j)): v for i, j, v in zip(coo.row, coo.col, coo.data)}

    def as_set(t):
        r, c, v = t
        return {(int(a), int(b)): x for a, b, x in zip(r, c, v)}

    assert as_set(out["A"]) == ref
    low = {k: v for k, v in ref.items() if k[1] < k[0] and k[0] // s == k[1] // s}
    assert as_set(out["L"]) == low and all(i - j == 1 for (i, j) in low)
    assert set(as_set(out["U"])) == {(j, i) for (i, j) in low}


@pytest.mark.parametrize("name,s", [("fv3d_12", 2 * 144 + 5), ("fv2d_natural", 3 * 24), ("q1_7", 700)])
def test_block_jacobi_layout_general_blocks(driver, tmp_path, name, s):
    """Blocks that are not tridiagonal (several grid lines or planes, or one
    block for the whole Q1 matrix): natural logical order, levels = longest
    chains of in-block couplings (brute force), L / U = the in-block couplings."""
    base = CASES[name]
    p = P.Problem(name=name, n=base.n, rowptr=base.rowptr, col=base.col, val=base.val, colors=None, f=base.f,
                  shape=base.shape, params={})
    out = _run_layout(driver, str(tmp_path), p, block_rows=s)
    assert out["ok"] == 1, out.get("why")
    n = p.n
    A = sp.csr_matrix((p.val, p.col, p.rowptr), shape=(n, n))
    lev = np.zeros(n, np.int64)
    for u in range(n):
        nb = A.indices[A.indptr[u]:A.indptr[u + 1]]
        nb = nb[(nb < u) & (nb // s == u // s)]
        lev[u] = 1 + lev[nb].max() if nb.size else 0
    assert len(out["lvl"]) - 1 == lev.max() + 1 > 2
    assert np.array_equal(np.diff(out["lvl"]), np.bincount(lev))
    assert np.array_equal(out["p2u"], np.lexsort((np.arange(n), lev)))
    p2u = out["p2u"]
    coo = A.tocoo()
    ref = {(int(i), int(j)): v for i, j, v in zip(coo.row, coo.col, coo.data)}

    def user_set(t):
        r, c, v = t
        return {(int(p2u[a]), int(p2u[b])): x for a, b, x in zip(r, c, v)}

    assert user_set(out["A"]) == ref
    low = {k: v for k, v in ref.items() if k[1] < k[0] and k[0] // s == k[1] // s}
    assert user_set(out["L"]) == low
    assert set(user_set(out["U"])) == {(j, i) for (i, j) in low}


def test_block_jacobi_layout_rejects_colours_and_bad_sizes(driver, tmp_path):
    p = CASES["fv3d_12"]
    assert _run_layout(driver, str(tmp_path), p, block_rows=12)["ok"] == 0  # colours given
    q = P.Problem(name="x", n=p.n, rowptr=p.rowptr, col=p.col, val=p.val, colors=None, f=p.f, shape=p.shape, params={})
    assert _run_layout(driver, str(tmp_path), q, block_rows=-3)["ok"] == 0


def test_sampling_table_matches_worked_examples_and_oracle(driver, tmp_path):
    out = os.path.join(str(tmp_path), "t.bin")
    rows = [l.split() for l in open(os.path.join(GOLDEN, "sampling_method_a.txt")) if l[0] != "#"]
    for r in rows:
        m, N = int(r[0]), int(r[1])
        subprocess.check_call([driver, "sampling", str(m), str(N + 2), out])
        t = _Reader(out).vec(np.int32)
        kept = {}
        for i in range(1, N):  # iteration N converged: not sampled
            if t[i] >= 0:
                kept[int(t[i])] = i
        assert sorted(kept.values()) == sorted(int(x) for x in r[2:])
    for m in (3, 8, 16):
        for N in (50, 777):
            subprocess.check_call([driver, "sampling", str(m), str(N + 2), out])
            t = _Reader(out).vec(np.int32)
            kept = np.zeros(m, np.int64)
            for i in range(1, N):
                if t[i] >= 0:
                    kept[t[i]] = i
            assert np.array_equal(kept, O.sample_schedule(m, N))


def _dense_call(driver, tmp, mode, *mats):
    fin, fout = os.path.join(tmp, "d.bin"), os.path.join(tmp, "o.bin")
    k = mats[0].shape[0]
    with open(fin, "wb") as f:
        f.write(np.int32(k).tobytes())
        for M in mats:
            f.write(np.asfortranarray(M, dtype=np.float64).tobytes(order="F"))
    subprocess.check_call([driver, mode, fin, fout])
    R = _Reader(fout)
    ok = int(R.one(np.int32))
    w = R.vec(np.float64)
    V = R.vec(np.float64)
    return ok, w, (V.reshape(k, k, order="F") if V.size == k * k else V)


@pytest.mark.parametrize("k", [1, 5, 17, 64])
def test_dense_routines_against_numpy(driver, tmp_path, k):
    rng = np.random.default_rng(k)
    X = rng.standard_normal((k, k))
    G = 0.5 * (X + X.T)
    Y = rng.standard_normal((k, k))
    B = Y @ Y.T + k * np.eye(k)
    ok, w, V = _dense_call(driver, str(tmp_path), "eig", G)
    assert ok == 1
    assert np.abs(w - np.linalg.eigvalsh(G)).max() <= 1e-12 * max(1.0, np.abs(w).max())
    assert np.abs(V.T @ V - np.eye(k)).max() <= 1e-12
    assert np.abs(G @ V - V * w).max() <= 1e-11 * max(1.0, np.abs(w).max())
    ok, w, T = _dense_call(driver, str(tmp_path), "geig", G, B)
    assert ok == 1
    lam = sla.eigh(G, B, eigvals_only=True)
    assert np.abs(w - lam).max() <= 1e-11 * max(1.0, np.abs(lam).max())
    assert np.abs(T.T @ B @ T - np.eye(k)).max() <= 1e-10
    assert np.abs(G @ T - B @ T * w).max() <= 1e-9 * max(1.0, np.abs(G).max())
    ok, _, Ci = _dense_call(driver, str(tmp_path), "cholinv", B)
    assert ok == 1
    assert np.abs(Ci - np.linalg.inv(B)).max() <= 1e-12 * np.abs(np.linalg.inv(B)).max()
    ok, _, _ = _dense_call(driver, str(tmp_path), "cholinv", G - (np.abs(G).sum() + 1) * np.eye(k))
    assert ok == 0


def test_lanczos_extremes_against_dense_tridiagonal(driver, tmp_path):
    rng = np.random.default_rng(9)
    k = 40
    a = rng.uniform(0.5, 2.0, k)
    b = rng.uniform(0.1, 0.9, k)
    fin, fout = os.path.join(str(tmp_path), "t.bin"), os.path.join(str(tmp_path), "o.bin")
    with open(fin, "wb") as f:
        f.write(np.int32(k).tobytes())
        f.write(a.tobytes())
        f.write(b.tobytes())
    subprocess.check_call([driver, "tridiag", fin, fout])
    lo, hi = np.frombuffer(open(fout, "rb").read(), np.float64)
    olo, ohi = O.lanczos_extremes(a, b)
    assert abs(lo / olo - 1) <= 1e-12 and abs(hi / ohi - 1) <= 1e-12
