#!/usr/bin/env python3
"""Benchmark: time-to-solution per system of a sequence of SPD systems sharing
one matrix, deflated (error-vector sampling) versus plain ICCG, on one MI355X.

Workload (default): 3-D 7-point FV diffusion on 128^3 cells, lognormal
coefficients (sigma = 2) with 16 low-conductivity spheres (radius 6, contrast
1e-5), diagonal scaling, 8 parity colours, IC(0); a sequence of 10 systems
b_k = f + 0.1 x_{k-1}; m = 16 sampled vectors, theta = 1e-3; FP64; relative
residual 1e-8.  All inputs are seeded and synthetic.

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
mixed-precision plain (both refinement forms), with the duration of its one
launch per iteration that updates x and r and applies the preconditioner to
the new r.

Roofline: the dominant kernel is the per-iteration SpMV launch; its duration
is measured with hipEvents on the solver's stream around every executed
launch of system 2 (the first deflated solve) of each timed step, which runs
with stream launches; all other solves replay the captured iteration graphs.
The same events bracket the IC(0) sweep launches of each iteration (sweeps
GB/s).  `traffic` comes from the committed rocprofv3 counter summary.
cpu_baseline: the FP64 C oracle, one thread.

`large_kernels` (after the timed steps, not part of `value`): the FP32 SpMV
and IC(0) sweep launches of the mixed solver's inner iterations at 256^3
(config-3 recipe) and on the Q1 27-point matrix with 160^3 nodes (config-4
recipe), timed the same way; at 128^3 the FP64 working set is about the size
of the 256 MB last-level cache, these two are well beyond it.  On the Q1
matrix also FP64 deflated against plain ICCG for one system after a sampling
solve (its 64 floating blocks give isolated small eigenvalues).
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
    ap.add_argument("--no-large", action="store_true", help="skip the 256^3 and Q1 160^3 kernel timings")
    ap.add_argument("--cpu-iters", type=int, default=300)
    ap.add_argument("--keep-eta", type=float, default=1e-2,
                    help="reduction between residual replacements of the mixed solver with ESD_FLAG_MIXED_KEEP")
    ap.add_argument("--copy-calib", action="store_true",
                    help="first run a plain 256 MiB device copy (reference kernel for HBM counters)")
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
    """Device-to-device copy of 1 GiB (FP64), the practical HBM ceiling on this
    GPU: read + written bytes over the mean of 10 copies (hipEvents)."""
    import torch

    src = torch.ones(128 * 1024 * 1024, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(10):
        dst.copy_(src)
    b.record()
    b.synchronize()
    us = a.elapsed_time(b) * 1e3 / 10
    nbytes = 2.0 * src.numel() * 8
    del src, dst
    return {"bytes_per_copy": nbytes, "avg_us": us, "gbs": nbytes / us / 1e3, "frac": nbytes / us / 1e3 / HBM_PEAK_GBS}


def large_kernels(esd, P):
    """FP32 SpMV and sweep-pair rates inside the mixed solver's inner
    iterations on the config-3 and config-4 matrices (plain form, no W)."""
    import torch

    out = {}
    for name, make, maxit in (("cfg3_fv3d_256", P.config3, 50000), ("cfg4_q1_160", P.config4, 300)):
        p = make()
        print("# large kernels: %s n=%d nnz=%d" % (name, p.n, p.nnz), file=sys.stderr, flush=True)
        s = esd.Solver.from_problem(p, m_max=p.params["m"] if name == "cfg4_q1_160" else 1)
        s.factor_ic0()
        f = torch.as_tensor(p.f, device=s.device)
        # config 4: the first 300 FP32 inner iterations only (its mixed solve
        # later finishes in FP64, whose iterations would enter the averages)
        x, info = s.solve(f, tol=1e-8, maxit=maxit, flags=esd.FLAG_MIXED | esd.FLAG_TIMING)
        tm = s.timing()
        n, nnz = p.n, p.nnz
        # FP32 (w = 4): plain-form SpMV gathers z and p_old, writes p and q;
        # sweep pair reads both triangles with their diagonals, r, y, writes y, z
        b_spmv = 8.0 * nnz + 16.0 * n
        b_sw = 8.0 * (nnz + n) + 16.0 * n
        ok = info["fp64_iters"] == 0 and tm["iters"] > 0
        sp_s, sw_s = tm["spmv_ms"] * 1e-3, tm["sweep_ms"] * 1e-3
        out[name] = {
            "n": n, "nnz": nnz, "fp32_iterations_timed": tm["iters"],
            "spmv": {"bytes_per_launch": b_spmv, "avg_launch_us": sp_s * 1e6,
                     "achieved": b_spmv / sp_s / 1e9 if ok else None,
                     "frac": b_spmv / sp_s / 1e9 / HBM_PEAK_GBS if ok else None},
            "sweeps": {"bytes_per_pair": b_sw, "avg_pair_us": sw_s * 1e6,
                       "achieved": b_sw / sw_s / 1e9 if ok else None,
                       "frac": b_sw / sw_s / 1e9 / HBM_PEAK_GBS if ok else None},
            "unit": "GB/s", "peak": HBM_PEAK_GBS,
        }
        if name == "cfg4_q1_160":
            # FP64 deflated vs plain ICCG on this matrix's many isolated small
            # eigenvalues: sampling solve (m = 64), build_aux, system 2 both ways
            m, theta = p.params["m"], 1e-3
            s.sample_errors(m)
            x1, i1 = s.solve(f, tol=1e-8, maxit=50000)
            st, ritz, mb, mt = s.build_aux(theta)
            b2 = s.sequence_rhs(f, x1, 0.1)
            res = {}
            for label, mode in (("plain", esd.PLAIN), ("deflated", esd.DEFLATED)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x2, i2 = s.solve(b2, tol=1e-8, maxit=50000, mode=mode)
                torch.cuda.synchronize()
                res[label] = {"iters": i2["iters"], "s": time.perf_counter() - t0, "true_relres": i2["true_relres"]}
            out[name]["fp64_deflation"] = {
                "m": m, "theta": theta, "m_bar": mb, "m_tilde": mt, "sampling_iters": i1["iters"],
                "plain": res["plain"], "deflated": res["deflated"],
                "speedup_vs_plain": res["plain"]["s"] / res["deflated"]["s"],
            }
        s.close()
        del p
    return out


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
    if args.copy_calib:
        # a plain copy of known size: what the HBM byte counters read for it
        # calibrates the counters of the solver kernels (256 MiB read + written)
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print("# copy calibration: 3 copies of 268435456 bytes", file=sys.stderr, flush=True)
    p = P.config2(N=args.N, m=args.m, systems=args.systems)
    print("# workload %s n=%d nnz=%d" % (p.name, p.n, p.nnz), file=sys.stderr, flush=True)
    s = esd.Solver.from_problem(p, m_max=args.m)
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
    spmv_ms = sweep_ms = 0.0
    spmv_n = 0
    bj_ms = 0.0
    bj_n = 0
    for k in range(args.steps):
        for name, mode, pf in seqs:
            r, wall, tm = run(name, mode, pf, name in ("deflated", "bj_deflated"))
            walls[name].append(wall)
            recs[name] = r
            if tm and name == "deflated":
                spmv_ms += tm["spmv_ms"] * tm["iters"]
                sweep_ms += tm["sweep_ms"] * tm["iters"]
                spmv_n += tm["iters"]
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
    }
    out["hbm_copy"] = copy_ceiling()
    out["gradient"] = grad_rate(s, p)
    if not args.no_large and args.N == 128:
        out["large_kernels"] = large_kernels(esd, P)
    if not args.no_cpu:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(p, args, mt, float(np.mean(its_defl)) if its_defl else its_plain[0])
    print(json.dumps(out), flush=True)
    s.close()
    if sbj is not None:
        sbj.close()


if __name__ == "__main__":
    main()
