#!/usr/bin/env python3
"""Benchmark: time-to-solution per system of a sequence of SPD systems sharing
one matrix, deflated (error-vector sampling) versus plain ICCG, on one MI355X.

Workload (default, `value`): 3-D 7-point FV diffusion on 128^3 cells,
lognormal coefficients (sigma = 2) with 16 low-conductivity spheres (radius
6, contrast 1e-5), diagonal scaling, 8 parity colours, IC(0); a sequence of
10 systems b_k = f + 0.1 x_{k-1} (built on the device); m = 16 sampled
vectors, theta = 1e-3; FP64; relative residual 1e-8.  All inputs are seeded
and synthetic; the matrix, its layouts and f are in device memory before the
timed region.

One step = factor_ic0 + the whole sequence: system 1 is plain ICCG with
sampling method A and the power iteration, then build_aux (error vectors,
Gram-Schmidt, Rayleigh-Ritz, W, C = W^T A W), then systems 2..10 deflated.
`value` = mean seconds per system of that step (sampling and build included).
Timed beside it on the same sequence (extra fields, not `value`): plain ICCG
throughout, the subspace-correction preconditioner, the FP32/FP64 mixed
solver, deflated and plain, with restarted refinement steps and with
residual replacement (ESD_FLAG_MIXED_KEEP, one continued FP32 CG run), and the
block-Jacobi IC(0) preconditioner of the paper's parallel solver (natural
order, one grid line of N rows per block), plain, deflated and
mixed-precision plain (both refinement forms).  `setup_s`: the constructor
(ordering, level schedule, layouts, upload), once per matrix.

Roofline: the dominant kernel is the per-iteration SpMV launch; its duration
is measured with hipEvents on the solver's stream around every executed
launch of system 2 of the deflated and of the plain sequence of each timed
step (both run that system with stream launches, all other solves replay the
captured iteration graphs).  The same events bracket the IC(0) sweep
launches (sweeps GB/s; the timed system keeps the first level's backward
launch apart from the projection, which the other deflated FP64 solves fold
into it, so the pair is whole).  `traffic` comes from the committed rocprofv3 counter
summary.  `hbm_ceiling`: the library's hand-written streaming probes (copy
and read-only reduction) beside torch's copy.  cpu_baseline: the FP64 C
oracle, one thread.

After the timed steps, once each (not part of `value`): configs 3 (256^3,
mixed, m = 32, 10 systems, deflated vs plain, per-system error against the
FP64 GPU solution), 4 (Q1 27-point on 160^3 nodes with 64 floating blocks,
m = 64, 20 systems, FP64 and mixed, plain vs deflated, all at one
true-residual target, kappa per system) and 5 (gradient of a loss through
the deflated mixed solver at 128^3 against central differences along 32
directions), with the FP32 SpMV and sweep rates of configs 3 and 4.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=128, help="grid cells per axis")
    ap.add_argument("--systems", type=int, default=10)
    ap.add_argument("--m", type=int, default=16)
    ap.add_argument("--theta", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-bj", action="store_true", help="skip the block-Jacobi sequences")
    ap.add_argument("--no-large", action="store_true", help="skip configs 3 (256^3) and 4 (Q1 160^3)")
    ap.add_argument("--no-grad", action="store_true", help="skip the config-5 gradient check")
    ap.add_argument("--cpu-iters", type=int, default=300)
    ap.add_argument("--keep-eta", type=float, default=1e-2,
                    help="reduction between residual replacements of the mixed solver with ESD_FLAG_MIXED_KEEP")
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run a plain 256 MiB device copy (reference kernel for HBM counters)")
    ap.add_argument("--profile-case", choices=("cfg3", "cfg4"), default=None,
                    help="a short run for rocprofv3 counters instead of the benchmark: the probe copy "
                         "of 256 MiB (calibration), then 200 FP32 inner iterations and 50 FP64 "
                         "iterations of the named matrix with stream launches")
    return ap.parse_args()


def run_sequence(s, p, args, mode, esd, P, timing, prec_flags, f):
    """One step: factor + the whole sequence; returns per-system records, the
    wall time and the kernel timings of the timed system.  f: the source
    vector already in device memory (uploaded before the timed region)."""
    import torch

    # kernel timing (hipEvents between stream launches) on one system of the
    # step; every other solve replays the captured iteration graphs
    t_sys = min(1, args.systems - 1)
    recs = []
    tm = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.factor_ic0()
    x = None
    for k in range(args.systems):
        flags_t = esd.FLAG_TIMING if (timing and k == t_sys) else 0
        bt = s.sequence_rhs(f, x, 0.1)
        if k == 0 and mode != esd.PLAIN:
            s.sample_errors(args.m)
            # K2: the power iteration rides on the SpMV of the first solve only;
            # later systems report kappa_es with that lambda_max (same A)
            x, info = s.solve(bt, tol=args.tol, maxit=20000, flags=esd.FLAG_POWER | flags_t | prec_flags)
            tb = time.perf_counter()
            st, ritz, mb, mt = s.build_aux(args.theta)
            info["build_aux_s"] = time.perf_counter() - tb
            info["m_bar"], info["m_tilde_built"] = mb, mt
            info["ritz"] = [float(v) for v in ritz[:mb]]
        else:
            pw = esd.FLAG_POWER if k == 0 else 0
            x, info = s.solve(bt, tol=args.tol, maxit=20000, mode=mode, flags=pw | flags_t | prec_flags)
        if flags_t:
            tm = s.timing()
        recs.append(info)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return recs, wall, tm


def grad_rate(s, p):
    """esd_grad_values on the benchmark matrix: g_k = -lam_row(k) x_col(k) for
    every stored entry; algorithmic bytes: column index and g per entry, row
    pointer, lam and x per row.  Mean of 20 launches between hipEvents."""
    import torch

    from paper_2203_08498_amd import esd

    g0 = torch.Generator(device="cpu").manual_seed(5)
    lam = torch.randn(p.n, generator=g0, dtype=torch.float64).to(s.device)
    x = torch.randn(p.n, generator=g0, dtype=torch.float64).to(s.device)
    g = torch.empty(p.nnz, dtype=torch.float64, device=s.device)
    call = lambda: s.L.esd_grad_values(s.h, esd._dptr(lam), esd._dptr(x), esd._dptr(g))
    for _ in range(3):
        call()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s.stream)
    for _ in range(20):
        call()
    b.record(s.stream)
    b.synchronize()
    us = a.elapsed_time(b) * 1e3 / 20
    nbytes = 12.0 * p.nnz + 24.0 * p.n
    return {"bytes_per_launch": nbytes, "avg_us": us, "gbs": nbytes / us / 1e3, "frac": nbytes / us / 1e3 / HBM_PEAK_GBS}


def copy_ceiling():
    """The practical HBM ceiling on this GPU: the library's hand-written
    streaming probes (esd_hbm_probe) over 1 GiB of FP64, a copy (read + write)
    and a read-only reduction, each at grids of 1024-16384 blocks (best
    reported), beside torch's device copy; bytes moved over the mean of 10
    launches between hipEvents."""
    import torch

    from paper_2203_08498_amd import esd

    n = 128 * 1024 * 1024
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def rate(fn, nbytes):
        for _ in range(3):
            fn()
        a, b = ev(), ev()
        a.record()
        for _ in range(10):
            fn()
        b.record()
        b.synchronize()
        us = a.elapsed_time(b) * 1e3 / 10
        return {"avg_us": us, "gbs": nbytes / us / 1e3, "frac": nbytes / us / 1e3 / HBM_PEAK_GBS}

    out = {"bytes": 8.0 * n, "torch_copy": rate(lambda: dst.copy_(src), 16.0 * n)}
    for kind, name, nb in ((esd.PROBE_COPY, "probe_copy", 16.0 * n), (esd.PROBE_READ, "probe_read", 8.0 * n)):
        best = None
        for g in (1024, 2048, 4096, 8192, 16384):
            r = rate(lambda: esd.hbm_probe(kind, src, dst, g), nb)
            r["grid"] = g
            if best is None or r["gbs"] > best["gbs"]:
                best = r
        out[name] = best
    del src, dst
    out["gbs"] = max(out["probe_copy"]["gbs"], out["probe_read"]["gbs"], out["torch_copy"]["gbs"])
    out["frac"] = out["gbs"] / HBM_PEAK_GBS
    return out


def _rec(info, extra=None):
    r = {k: info[k] for k in ("iters", "outer_iters", "fp64_iters", "true_relres", "seconds", "kappa", "kappa_es")}
    r["kappa"], r["kappa_es"] = round(r["kappa"], 3), round(r["kappa_es"], 3)
    if extra:
        r.update(extra)
    return r


def _fp64_floor(p, x, b):
    """Attainable relative residual of an FP64 solve: b - A x is itself only
    known to about gamma_k || |A| |x| || / ||b|| (k = longest row)."""
    import numpy as np
    import scipy.sparse as sp

    absA = sp.csr_matrix((np.abs(p.val), p.col, p.rowptr), shape=(p.n, p.n))
    k = int(np.diff(p.rowptr).max())
    u = 2.0 ** -53
    return k * u / (1 - k * u) * float(np.linalg.norm(absA @ np.abs(x)) / np.linalg.norm(b))


def run_spec_sequence(s, f, esd, K, m, theta, mode, flags, tol, maxit, ref=None, ref_tol=None):
    """One sequence as the configs specify it: b_1 = f, b_k = f + 0.1 x_{k-1}
    built on the device; an accelerated mode samples m vectors in system 1
    (method A, power iteration on) and builds W at theta after it.  With
    ref (flags of an FP64 reference solve), every system's solution is also
    compared with the FP64 GPU solution of the same b at ref_tol (deflated
    where the sequence is, plain for system 1).  Returns per-system records,
    the sequence's wall time (sampling and build_aux included, reference
    solves excluded) and the build record."""
    import torch

    recs, x = [], None
    build = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_ref = 0.0
    for k in range(K):
        b = s.sequence_rhs(f, x, 0.1)
        if k == 0:
            if mode != esd.PLAIN:
                s.sample_errors(m)
            x, info = s.solve(b, tol=tol, maxit=maxit, flags=flags | esd.FLAG_POWER)
            if mode != esd.PLAIN:
                tb = time.perf_counter()
                st, ritz, mb, mt = s.build_aux(theta)
                build = {"build_aux_s": time.perf_counter() - tb, "m_bar": mb, "m_tilde": mt,
                         "ritz_smallest": [float(v) for v in ritz[:8]],
                         "theta_sweep_m_tilde": {"%g" % th: int(sum(1 for v in ritz if v < th))
                                                 for th in (1e-2, 1e-3, 1e-4, 1e-5)}}
        else:
            x, info = s.solve(b, tol=tol, maxit=maxit, mode=mode, flags=flags)
        extra = {}
        if ref is not None:
            torch.cuda.synchronize()
            tr = time.perf_counter()
            rmode = esd.DEFLATED if (k > 0 and mode != esd.PLAIN) else esd.PLAIN
            xr, ir = s.solve(b, tol=ref_tol, maxit=maxit, mode=rmode, flags=ref)
            extra = {"err_vs_fp64": float(torch.linalg.norm(x - xr) / torch.linalg.norm(xr)),
                     "fp64_ref_true_relres": ir["true_relres"], "fp64_ref_iters": ir["iters"]}
            torch.cuda.synchronize()
            t_ref += time.perf_counter() - tr
        recs.append(_rec(info, extra))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0 - t_ref
    return recs, wall, build, x


def _seq_summary(recs, wall, build, K):
    import numpy as np

    out = {"s_per_system": wall / K,
           "s_systems_2_to_K": float(np.mean([r["seconds"] for r in recs[1:]])),
           "iters_systems_2_to_K": float(np.mean([r["iters"] for r in recs[1:]])),
           "iters_system_1": recs[0]["iters"],
           "true_relres_max": max(r["true_relres"] for r in recs),
           "fp64_iters_total": int(sum(r["fp64_iters"] for r in recs)),
           "per_system": {k: [r[k] for r in recs] for k in recs[0]}}
    if build:
        out.update(build)
    if "err_vs_fp64" in recs[0]:
        out["err_vs_fp64_max"] = max(r["err_vs_fp64"] for r in recs)
    return out


def fp32_kernel_rates(s, f, esd, maxit):
    """FP32 SpMV and sweep-pair rates of the mixed solver's inner iterations
    (plain form; hipEvents around every launch of one solve)."""
    x, info = s.solve(f, tol=1e-8, maxit=maxit, flags=esd.FLAG_MIXED | esd.FLAG_TIMING)
    tm = s.timing()
    n, nnz = s.n, s.nnz
    # FP32 (w = 4): plain-form SpMV gathers z and p_old, writes p and q;
    # sweep pair reads both triangles with their diagonals, r, y, writes y, z
    b_spmv = 8.0 * nnz + 16.0 * n
    b_sw = 8.0 * (nnz + n) + 16.0 * n
    ok = info["fp64_iters"] == 0 and tm["iters"] > 0
    sp_s, sw_s = tm["spmv_ms"] * 1e-3, tm["sweep_ms"] * 1e-3
    return {
        "fp32_iterations_timed": tm["iters"],
        "spmv": {"bytes_per_launch": b_spmv, "avg_launch_us": sp_s * 1e6,
                 "achieved": b_spmv / sp_s / 1e9 if ok else None,
                 "frac": b_spmv / sp_s / 1e9 / HBM_PEAK_GBS if ok else None},
        "sweeps": {"bytes_per_pair": b_sw, "avg_pair_us": sw_s * 1e6,
                   "achieved": b_sw / sw_s / 1e9 if ok else None,
                   "frac": b_sw / sw_s / 1e9 / HBM_PEAK_GBS if ok else None},
        "unit": "GB/s", "peak": HBM_PEAK_GBS,
    }


def config3_spec(esd, P, theta):
    """Config 3 as specified: 256^3 config-2 recipe, FP32 inner / FP64 outer
    (mixed), m = 32, 10 systems, deflated against plain (and FP64 plain ICCG
    on the same sequence recipe, for reference); every system of the
    mixed deflated sequence against the FP64 deflated GPU solution of the same
    b at relres 1e-12 (whose parity with the oracle is pinned at 128^3 and
    131^3)."""
    import torch

    p = P.config3()
    m, K = p.params["m"], p.params["systems"]
    print("# config 3: n=%d nnz=%d" % (p.n, p.nnz), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    s = esd.Solver.from_problem(p, m_max=m, max_iters=60000)
    setup_s = time.perf_counter() - t0
    try:
        t0 = time.perf_counter()
        s.factor_ic0()
        torch.cuda.synchronize()
        fac_s = time.perf_counter() - t0
        s.set_power_start(P.power_start(3, p.n))
        f = torch.as_tensor(p.f, device=s.device)
        out = {"n": p.n, "nnz": p.nnz, "m": m, "theta": theta, "systems": K, "setup_s": setup_s,
               "esd_setup_s": s.setup_s, "factor_s": fac_s, "workspace_bytes": s.ws_needed}
        out.update(fp32_kernel_rates(s, f, esd, 60000))
        for label, mode, flags, ref in (("mixed_plain", esd.PLAIN, esd.FLAG_MIXED, None),
                                        ("mixed_deflated", esd.DEFLATED, esd.FLAG_MIXED, 0),
                                        ("fp64_plain", esd.PLAIN, 0, None)):
            recs, wall, build, _ = run_spec_sequence(s, f, esd, K, m, theta, mode, flags, 1e-8, 60000,
                                                     ref=ref, ref_tol=1e-12)
            out[label] = _seq_summary(recs, wall, build, K)
            print("# config 3 %s: %.4f s/system" % (label, out[label]["s_per_system"]), file=sys.stderr, flush=True)
        out["speedup_deflated_vs_plain"] = out["mixed_plain"]["s_per_system"] / out["mixed_deflated"]["s_per_system"]
        out["speedup_mixed_deflated_vs_fp64_plain"] = out["fp64_plain"]["s_per_system"] / \
            out["mixed_deflated"]["s_per_system"]
        return out
    finally:
        s.close()


def config4_spec(esd, P, theta):
    """Config 4 as specified: Q1 27-point on 160^3 nodes with 64 floating
    blocks, m = 64, 20 systems, kappa per system; FP64 and FP32/FP64 mixed
    (adaptive: ESD_FLAG_MIXED_ADAPT), plain against deflated.  Every solve is driven to one true-residual
    target: relres 1e-8, or 3x the FP64 rounding floor of b - A x when that
    is higher (FP64 solves test the recomputed residual, ESD_FLAG_TRUE_RES;
    mixed solves test it by construction).  The mixed deflated sequence's
    systems are compared with the FP64 deflated solution of the same b."""
    import torch

    p = P.config4()
    m, K = p.params["m"], p.params["systems"]
    print("# config 4: n=%d nnz=%d" % (p.n, p.nnz), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    s = esd.Solver.from_problem(p, m_max=m, max_iters=60000)
    setup_s = time.perf_counter() - t0
    try:
        s.factor_ic0()
        s.set_power_start(P.power_start(4, p.n))
        f = torch.as_tensor(p.f, device=s.device)
        out = {"n": p.n, "nnz": p.nnz, "m": m, "theta": theta, "systems": K, "setup_s": setup_s,
               "esd_setup_s": s.setup_s, "workspace_bytes": s.ws_needed}
        # the first 300 FP32 inner iterations (the solve may finish in FP64)
        out.update(fp32_kernel_rates(s, f, esd, 300))
        x1, i1 = s.solve(f, tol=1e-8, maxit=60000)
        floor = _fp64_floor(p, x1.cpu().numpy(), p.f)
        tol = max(1e-8, 3.0 * floor)
        out["fp64_floor"] = floor
        out["tol_true_relres"] = tol
        # the mixed sequences run adaptively (ESD_FLAG_MIXED_ADAPT): FP32 cannot
        # resolve this operator, and once a mixed solve in a mode has had to
        # finish in FP64, the later ones in that mode start there
        adapt = esd.FLAG_MIXED | esd.FLAG_MIXED_ADAPT
        for label, mode, flags, ref in (("fp64_plain", esd.PLAIN, esd.FLAG_TRUE_RES, None),
                                        ("fp64_deflated", esd.DEFLATED, esd.FLAG_TRUE_RES, None),
                                        ("mixed_plain", esd.PLAIN, adapt, None),
                                        ("mixed_deflated", esd.DEFLATED, adapt, esd.FLAG_TRUE_RES)):
            recs, wall, build, _ = run_spec_sequence(s, f, esd, K, m, theta, mode, flags, tol, 60000,
                                                     ref=ref, ref_tol=tol)
            out[label] = _seq_summary(recs, wall, build, K)
            print("# config 4 %s: %.4f s/system" % (label, out[label]["s_per_system"]), file=sys.stderr, flush=True)
        for pre in ("fp64", "mixed"):
            out["speedup_deflated_vs_plain_" + pre] = out[pre + "_plain"]["s_per_system"] / \
                out[pre + "_deflated"]["s_per_system"]
        out["speedup_mixed_deflated_vs_fp64_plain"] = out["fp64_plain"]["s_per_system"] / \
            out["mixed_deflated"]["s_per_system"]
        return out
    finally:
        s.close()


def config5_spec(esd, P):
    """Config 5 as specified: the 128^3 config-2 field, forward and adjoint
    solves with the deflated mixed solver (m = 16, theta = 1e-3, relres
    1e-12) in the autograd Function, loss 0.5 ||x - x_t||^2, gradients with
    respect to b and every stored value against central differences
    (h = 1e-6) along 32 seeded directions (symmetric value perturbation and a
    right-hand-side perturbation), and the Richardson combination of h and
    2h; FD solves FP64 deflated at relres 1e-13."""
    import numpy as np
    import scipy.sparse as sp
    import torch

    from paper_2203_08498_amd import autograd as AG

    p = P.config2(N=128, cfg=2)
    s = esd.Solver.from_problem(p, m_max=16)
    try:
        s.factor_ic0()
        s.sample_errors(16)
        s.solve(p.f, tol=1e-8, maxit=20000)
        s.build_aux(1e-3)
        vals = torch.tensor(p.val, device=s.device, dtype=torch.float64, requires_grad=True)
        b = torch.tensor(p.f, device=s.device, requires_grad=True)
        xt = torch.tensor(P.rng_for(5, P.STREAM_XT).standard_normal(p.n), device=s.device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = AG.solve(vals, b, s, mode=esd.DEFLATED, tol=1e-12, maxit=20000, flags=esd.FLAG_MIXED)
        loss = 0.5 * ((x - xt) ** 2).sum()
        loss.backward()
        torch.cuda.synchronize()
        t_grad = time.perf_counter() - t0
        gv, gb = vals.grad.cpu().numpy(), b.grad.cpu().numpy()
        M = sp.csr_matrix((np.arange(1, p.nnz + 1, dtype=np.float64), p.col, p.rowptr), shape=(p.n, p.n))
        T = M.T.tocsr()
        T.sort_indices()
        tmap = T.data.astype(np.int64) - 1
        rng = P.rng_for(5, P.STREAM_FD)
        h = 1e-6

        def L(v, bb):
            s.update_values(v)
            s.factor_ic0()
            xx, info = s.solve(bb, tol=1e-13, maxit=50000, mode=esd.DEFLATED)
            return 0.5 * float(((xx - xt) ** 2).sum())

        def D(d, db, hh):
            return (L(p.val + hh * d, p.f + hh * db) - L(p.val - hh * d, p.f - hh * db)) / (2 * hh)

        errs, errs2, rich = [], [], []
        for _ in range(32):
            d = rng.standard_normal(p.nnz)
            d = 0.5 * (d + d[tmap])
            db = rng.standard_normal(p.n)
            an = gv @ d + gb @ db
            d1, d2 = D(d, db, h), D(d, db, 2 * h)
            errs.append(abs(d1 - an) / abs(an))
            errs2.append(abs(d2 - an) / abs(an))
            rich.append(abs((4 * d1 - d2) / 3 - an) / abs(an))
        s.update_values(p.val)
        # the central difference's own O(h^2) truncation dominates its error
        # (4x at 2h); Richardson's (4 D(h) - D(2h)) / 3 removes it
        return {"directions": 32, "h": h, "forward_plus_adjoint_s": t_grad,
                "cd_rel_err_max": max(errs), "cd_rel_err_median": float(np.median(errs)),
                "cd_2h_over_h_err_ratio_median": float(np.median(np.array(errs2) / np.array(errs))),
                "richardson_rel_err_max": max(rich), "richardson_rel_err_median": float(np.median(rich))}
    finally:
        s.close()


def profile_case(esd, P, case):
    """A short, fixed launch sequence for HBM counters: 3 probe copies of
    256 MiB (known bytes, the calibration kernel), then on the 256^3 (cfg3)
    or Q1 160^3 (cfg4) matrix 200 FP32 inner iterations of the mixed solver
    and 50 FP64 iterations, every kernel launched on the stream."""
    import torch

    src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        esd.hbm_probe(esd.PROBE_COPY, src, dst, 4096)
    torch.cuda.synchronize()
    del src, dst
    print("# calibration: 3 probe copies of 268435456 bytes", file=sys.stderr, flush=True)
    p = P.config3() if case == "cfg3" else P.config4()
    s = esd.Solver.from_problem(p, m_max=1)
    s.factor_ic0()
    f = torch.as_tensor(p.f, device=s.device)
    x, i32 = s.solve(f, tol=1e-8, maxit=200, flags=esd.FLAG_MIXED | esd.FLAG_STREAM)
    x, i64 = s.solve(f, tol=1e-8, maxit=50, flags=esd.FLAG_STREAM)
    torch.cuda.synchronize()
    print("# %s: n=%d nnz=%d, %d FP32 inner and %d FP64 iterations" % (case, p.n, p.nnz, i32["iters"], i64["iters"]),
          file=sys.stderr, flush=True)
    s.close()


def counter_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, calibrated against a plain copy), or None
    when the summary is missing, covers another kernel, or was taken from other
    kernel sources than the ones built now."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "k_spmv_it_fv3d128_hbm_counters.txt")
    src = os.path.join(ROOT, "paper_2203_08498_amd", "csrc")
    try:
        text = open(path).read()
        h = hashlib.sha256(open(os.path.join(src, "kernels.hip"), "rb").read()
                           + open(os.path.join(src, "kernels.h"), "rb").read()).hexdigest()
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in text.splitlines()
                  if line.split(": ", 1)[0] in ("traffic_kernel", "traffic_bytes_per_launch", "kernels_sha256"))
    if fields.get("kernels_sha256") != h or fields.get("traffic_kernel") != kernel:
        return None
    return float(fields["traffic_bytes_per_launch"])


def cpu_baseline(p, args, mt, iters_per_system):
    """Oracle (plain C, 1 thread): a bounded number of deflated PCG iterations
    on the same matrix with a seeded random W of the same width."""
    import numpy as np

    import oracle as O

    o = O.Oracle.from_problem(p)
    t0 = time.perf_counter()
    o.factor_ic0()
    t_fac = time.perf_counter() - t0
    k = max(mt, 1)
    W = np.random.default_rng([2, 9]).standard_normal((p.n, k))
    W, _ = np.linalg.qr(W)
    o.set_aux(W)
    t0 = time.perf_counter()
    o.solve(p.f, tol=0.0, maxit=args.cpu_iters, mode=O.DEFLATED if mt > 0 else O.PLAIN)
    t_it = (time.perf_counter() - t0) / args.cpu_iters
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": t_it * iters_per_system,
        "unit": "s/system",
        "cores": 1,
        "kind": "oracle",
        "host": {"cpu_model": model, "nproc": os.cpu_count(),
                 "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None},
        "sample": "FP64 C oracle, 1 thread: %d deflated PCG iterations (m_tilde=%d, seeded random W) on the "
                  "same %d-row matrix, %.3f s/iteration x %.1f iterations per system (mean of this run); "
                  "IC(0) factor %.2f s not included" % (args.cpu_iters, k, p.n, t_it, iters_per_system, t_fac),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this solver is a single-GPU build "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2203_08498_amd import esd, problems as P

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.profile_case:
        profile_case(esd, P, args.profile_case)
        return
    if args.copy_calib:
        # a plain copy of known size (the library's probe kernel): what the HBM
        # byte counters read for it calibrates the counters of the solver
        # kernels (256 MiB read + written per copy)
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            esd.hbm_probe(esd.PROBE_COPY, src, dst, 4096)
        torch.cuda.synchronize()
        del src, dst
        print("# copy calibration: 3 probe copies of 268435456 bytes", file=sys.stderr, flush=True)
    p = P.config2(N=args.N, m=args.m, systems=args.systems)
    print("# workload %s n=%d nnz=%d" % (p.name, p.n, p.nnz), file=sys.stderr, flush=True)
    # setup (ordering, level schedule, layouts, upload; once per matrix, not
    # part of a step): the whole constructor and the esd_setup call inside it
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = esd.Solver.from_problem(p, m_max=args.m)
    setup_wall = time.perf_counter() - t0
    s.set_power_start(P.power_start(2, p.n))
    # block-Jacobi IC(0), one grid line (N consecutive rows) per block
    sbj = None
    if not args.no_bj:
        sbj = esd.Solver.from_problem(p, m_max=args.m, block_rows=args.N)
        sbj.set_power_start(P.power_start(2, p.n))
    keep = esd.FLAG_MIXED | esd.FLAG_MIXED_KEEP
    seqs = (("deflated", esd.DEFLATED, 0), ("plain", esd.PLAIN, 0), ("subspace", esd.SUBSPACE, 0),
            ("mixed_deflated", esd.DEFLATED, esd.FLAG_MIXED), ("mixed_plain", esd.PLAIN, esd.FLAG_MIXED),
            ("mixed_keep_deflated", esd.DEFLATED, keep), ("mixed_keep_plain", esd.PLAIN, keep))
    if sbj is not None:
        seqs = seqs + (("bj_deflated", esd.DEFLATED, 0), ("bj_plain", esd.PLAIN, 0),
                       ("bj_mixed_plain", esd.PLAIN, esd.FLAG_MIXED), ("bj_mixed_keep_plain", esd.PLAIN, keep))
    solver_of = lambda name: sbj if name.startswith("bj_") else s

    f_dev = torch.as_tensor(p.f, device=s.device)  # input resident before any timed step

    def run(name, mode, pf, timing):
        sv = solver_of(name)
        if pf & esd.FLAG_MIXED_KEEP:
            sv.set_mixed_params(args.keep_eta, 60)
        try:
            return run_sequence(sv, p, args, mode, esd, P, timing, pf, f=f_dev)
        finally:
            if pf & esd.FLAG_MIXED_KEEP:
                sv.set_mixed_params()

    for _ in range(args.warmup):
        for name, mode, pf in seqs:
            run(name, mode, pf, False)
        print("# warmup step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    walls = {name: [] for name, _, _ in seqs}
    recs = {}
    # kernel timing: system 2 of the deflated and the plain sequence (and of
    # both block-Jacobi ones) runs with hipEvents around its launches, so
    # deflated and plain carry the same (small) cost of stream launches
    timed_seqs = ("deflated", "plain", "bj_deflated", "bj_plain")
    spmv_ms = sweep_ms = 0.0
    spmv_n = 0
    spmv_plain_ms, spmv_plain_n = 0.0, 0
    bj_ms = 0.0
    bj_n = 0
    for k in range(args.steps):
        for name, mode, pf in seqs:
            r, wall, tm = run(name, mode, pf, name in timed_seqs)
            walls[name].append(wall)
            recs[name] = r
            if tm and name == "deflated":
                spmv_ms += tm["spmv_ms"] * tm["iters"]
                sweep_ms += tm["sweep_ms"] * tm["iters"]
                spmv_n += tm["iters"]
            elif tm and name == "plain":
                spmv_plain_ms += tm["spmv_ms"] * tm["iters"]
                spmv_plain_n += tm["iters"]
            elif tm:
                bj_ms += tm["sweep_ms"] * tm["iters"]
                bj_n += tm["iters"]
        print("# step %d: " % k + ", ".join("%s %.4f s" % (nm, walls[nm][-1]) for nm, _, _ in seqs),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    per = {nm: float(np.mean(w)) / args.systems for nm, w in walls.items()}
    per_sys, per_sys_plain = per["deflated"], per["plain"]
    T = per_sys * args.systems
    rd, rp = recs["deflated"], recs["plain"]
    mt = rd[0].get("m_tilde_built", 0)
    its_defl = [r["iters"] for r in rd[1:]]
    its_plain = [r["iters"] for r in rp]
    # theta sweep on the same samples (m_tilde only; the timed runs use args.theta)
    theta_sweep = {}
    for th in (1e-3, 1e-4, 1e-5, args.theta):
        theta_sweep["%g" % th] = int(sum(1 for v in rd[0]["ritz"] if v < th))
    # roofline of the per-iteration SpMV launch of the deflated form
    avg_spmv_s = (spmv_ms / max(spmv_n, 1)) * 1e-3
    avg_sweep_s = (sweep_ms / max(spmv_n, 1)) * 1e-3
    n, nnz = p.n, p.nnz
    # deflated iterations: the projection has written p = zhat + beta p_old, so
    # the SpMV reads the matrix (8 B value + 4 B index per stored entry) and p,
    # and writes q (the timed system runs without the power iterate)
    bytes_spmv = 12.0 * nnz + 16.0 * n
    achieved = bytes_spmv / avg_spmv_s / 1e9 if avg_spmv_s > 0 else 0.0
    # what the layout the kernel reads has to move: the class-aligned copy has
    # no column indices (8 B per slot plus 4 B per 64 slots), the sorted one 12 B
    lay = s.layout()
    slots = lay["a_slots"]
    fmt_spmv = (8.0 * slots + 4.0 * slots / 64 if lay["class_layout"][0] else 12.0 * slots) + 16.0 * n
    # one forward + backward IC(0) sweep pair: both triangles with their
    # diagonals (12 B per entry), r read, y written and read, z written
    bytes_sweeps = 12.0 * (nnz + n) + 32.0 * n
    sweeps_gbs = bytes_sweeps / avg_sweep_s / 1e9 if avg_sweep_s > 0 else 0.0
    bj = None
    if sbj is not None:
        # x += alpha p, r -= alpha q and z = M^{-1} r (block Jacobi) in one
        # launch: x, p, q, r, the sub-diagonal and the inverse diagonal of the
        # bidiagonal block factors read, x, r and z written
        avg_bj_s = (bj_ms / max(bj_n, 1)) * 1e-3
        bytes_bj = 72.0 * n
        bj_gbs = bytes_bj / avg_bj_s / 1e9 if avg_bj_s > 0 else 0.0
        rbd, rbp = recs["bj_deflated"], recs["bj_plain"]
        bj = {
            "block_rows": args.N,
            "deflated_s_per_system": per["bj_deflated"],
            "plain_s_per_system": per["bj_plain"],
            "mixed_plain_s_per_system": per["bj_mixed_plain"],
            "iters_mixed_plain_mean": float(np.mean([r["iters"] for r in recs["bj_mixed_plain"]])),
            "mixed_keep_plain_s_per_system": per["bj_mixed_keep_plain"],
            "iters_mixed_keep_plain_mean": float(np.mean([r["iters"] for r in recs["bj_mixed_keep_plain"]])),
            "iters_sampling_solve": rbd[0]["iters"],
            "iters_deflated_mean": float(np.mean([r["iters"] for r in rbd[1:]])) if args.systems > 1 else None,
            "iters_plain_mean": float(np.mean([r["iters"] for r in rbp])),
            "m_tilde": rbd[0].get("m_tilde_built", 0),
            "ritz_smallest": rbd[0]["ritz"][:8],
            "true_relres_max": max(r["true_relres"] for r in rbd + rbp),
            "kappa_cg_plain": round(rbp[-1]["kappa"], 3),
            "prec": {"kernel": "k_update_bj (vector update + forward and backward block sweeps, one launch)",
                     "unit": "GB/s",
                     "achieved": bj_gbs, "peak": HBM_PEAK_GBS, "frac": bj_gbs / HBM_PEAK_GBS,
                     "bytes_per_launch": bytes_bj, "avg_launch_us": avg_bj_s * 1e6, "launches": bj_n},
        }
    out = {
        "metric": "time-to-solution/system at relres 1e-8, deflated vs plain ICCG; SpMV GB/s",
        "value": per_sys,
        "unit": "s/system",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded lognormal-coefficient FV diffusion, config-2 recipe)",
        "config": {
            "workload": "fv3d-7pt %d^3, lognormal sigma=2 + 16 spheres r=6 contrast 1e-5, diag-scaled, "
                        "8 colours, IC(0); %d systems b_k=f+0.1x_(k-1); m=%d theta=%g; deflated ICCG"
                        % (args.N, args.systems, args.m, args.theta),
            "n": n, "nnz": nnz, "systems": args.systems, "m": args.m, "theta": args.theta,
        },
        "setup_s": setup_wall,
        "esd_setup_s": s.setup_s,
        "workspace_bytes": s.ws_needed,
        "workspace_bound_bytes": int(s.workspace.numel()),
        "plain_s_per_system": per_sys_plain,
        "speedup_vs_plain": per_sys_plain / per_sys if per_sys > 0 else None,
        "subspace_s_per_system": per["subspace"],
        "mixed_deflated_s_per_system": per["mixed_deflated"],
        "mixed_plain_s_per_system": per["mixed_plain"],
        # the same mixed solver with ESD_FLAG_MIXED_KEEP: each refinement step
        # replaces the residual of the running FP32 CG instead of restarting it
        "mixed_keep_eta": args.keep_eta,
        "mixed_keep_deflated_s_per_system": per["mixed_keep_deflated"],
        "mixed_keep_plain_s_per_system": per["mixed_keep_plain"],
        "iters_mixed_keep_deflated_mean": float(np.mean([r["iters"] for r in recs["mixed_keep_deflated"][1:]])) if args.systems > 1 else None,
        "iters_mixed_keep_plain_mean": float(np.mean([r["iters"] for r in recs["mixed_keep_plain"]])),
        "mixed_keep_m_tilde": recs["mixed_keep_deflated"][0].get("m_tilde_built", 0),
        "mixed_keep_fp64_iters_total": int(sum(r["fp64_iters"] for r in recs["mixed_keep_deflated"] + recs["mixed_keep_plain"])),
        "mixed_keep_true_relres_max": max(r["true_relres"] for r in recs["mixed_keep_deflated"] + recs["mixed_keep_plain"]),
        "deflated_s_systems_2_to_K": float(np.mean([r["seconds"] for r in rd[1:]])) if len(rd) > 1 else None,
        "plain_s_systems_2_to_K": float(np.mean([r["seconds"] for r in rp[1:]])) if len(rp) > 1 else None,
        "iters_sampling_solve": rd[0]["iters"],
        "build_aux_s": rd[0].get("build_aux_s"),
        "m_bar": rd[0].get("m_bar"),
        "m_tilde": mt,
        "ritz_smallest": rd[0]["ritz"][:8],
        "theta_sweep_m_tilde": theta_sweep,
        "iters_deflated_mean": float(np.mean(its_defl)) if its_defl else None,
        "iters_plain_mean": float(np.mean(its_plain)),
        "iters_subspace_mean": float(np.mean([r["iters"] for r in recs["subspace"][1:]])) if args.systems > 1 else None,
        "iters_mixed_deflated_mean": float(np.mean([r["iters"] for r in recs["mixed_deflated"][1:]])) if args.systems > 1 else None,
        "iters_mixed_plain_mean": float(np.mean([r["iters"] for r in recs["mixed_plain"]])),
        "mixed_fp64_iters_total": int(sum(r["fp64_iters"] for r in recs["mixed_deflated"])),
        "true_relres_max": max(r["true_relres"] for r in rd),
        "mixed_true_relres_max": max(r["true_relres"] for r in recs["mixed_deflated"]),
        "kappa_cg_per_system": [round(r["kappa"], 3) for r in rd],
        "kappa_es_per_system": [round(r["kappa_es"], 3) for r in rd],
        "block_jacobi": bj,
        "sweeps": {"unit": "GB/s", "achieved": sweeps_gbs, "peak": HBM_PEAK_GBS, "frac": sweeps_gbs / HBM_PEAK_GBS,
                   "bytes_per_pair": bytes_sweeps, "avg_pair_us": avg_sweep_s * 1e6},
        "roofline": {
            "kernel": "k_spmv_it, deflated form (q = A p for the projected direction p, and (p, q))",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": counter_traffic("k_spmv_it<double, false, true>") if args.N == 128 else None,
            "bytes_per_launch": bytes_spmv,
            "layout_bytes_per_launch": fmt_spmv,
            "layout_gbs": fmt_spmv / avg_spmv_s / 1e9 if avg_spmv_s > 0 else 0.0,
            "avg_launch_us": avg_spmv_s * 1e6,
            "launches": spmv_n,
        },
        # the plain form's SpMV (p = z + beta p_old formed on the fly: z and
        # p_old gathered, p and q written), timed the same way in the plain sequence
        "spmv_plain_form": {"bytes_per_launch": 12.0 * nnz + 32.0 * n,
                            "avg_launch_us": spmv_plain_ms / max(spmv_plain_n, 1) * 1e3,
                            "achieved": (12.0 * nnz + 32.0 * n) / (spmv_plain_ms / max(spmv_plain_n, 1) * 1e-3) / 1e9
                            if spmv_plain_n else None},
    }
    out["hbm_ceiling"] = copy_ceiling()
    out["gradient"] = grad_rate(s, p)
    # the other configurations as specified, once, after the timed steps
    if not args.no_large and args.N == 128:
        out["config3"] = config3_spec(esd, P, args.theta)
        out["config4"] = config4_spec(esd, P, args.theta)
    if not args.no_grad and args.N == 128:
        print("# config 5 gradient check ...", file=sys.stderr, flush=True)
        out["config5"] = config5_spec(esd, P)
    if not args.no_cpu:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(p, args, mt, float(np.mean(its_defl)) if its_defl else its_plain[0])
    print(json.dumps(out), flush=True)
    s.close()
    if sbj is not None:
        sbj.close()


if __name__ == "__main__":
    main()
