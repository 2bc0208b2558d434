#!/usr/bin/env python
"""Benchmark: time-to-1e-8 PMINRES solve and per-iteration HBM GB/s on one MI355X.

Workload (default): 2D time-fractional sub-diffusion, L1 scheme, gamma = 0.3,
M = 511^2 interior points (h = 1/512), N = 1024 time steps on T = 1,
alpha = 0.01, f ~ N(0,1) seeded (seed 3), tolerance 1e-8 on the relative
symmetrised residual.  A "step" is one complete solve A u = f by the mixed
path (FP32 MINRES sweeps inside FP64 iterative refinement) with f already in
HBM; the FP64 path is timed beside it on the same input.

Prints one JSON line (rank 0).  `value` is mixed-path solves per second.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# kernel classes run once per MINRES iteration, per Krylov basis
HOT_CLASSES = {"sine": ["matvec", "time_prec", "wx_update"],
               "physical": ["matvec", "dst_x_vupd", "dst_strided", "time_prec", "dst_x_dot", "wx_update"]}


def cpu_baseline(workload: str, tol: float, budget_s: float = 12.0) -> dict:
    """The CPU oracle, as it stands, on a bounded sample of the workload: the
    same problem with m = 127 (M = 127^2) instead of 511, solved repeatedly until
    `budget_s` seconds have passed; scaled to the full M linearly (a lower
    bound on the oracle's time, whose sine transforms grow faster than M)."""
    import numpy as np
    from oracle import bltt_oracle as O
    from paper_2307_07749_amd import workloads as W

    full, seed = W.workload(workload)
    m_s = 127
    prob = W.fractional_l1(full.dim, m_s, full.N, full.meta["gamma"], full.alpha)
    f = W.rhs_normal(prob, seed)
    sysm = O.from_problem(prob)
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    t0 = time.perf_counter()
    runs = 0
    while True:
        res = O.pminres(sysm, f, tol, 200)
        runs += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    per = (time.perf_counter() - t0) / runs
    scale = full.M / prob.M
    return {"value": 1.0 / (per * scale), "unit": "solve/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"oracle PMINRES (dense DFT/DST products, explicit residual each iteration) on the same "
                       f"problem with m={m_s} (M={prob.M}), N={full.N}: {per:.2f} s/solve over {runs} run(s), "
                       f"{res.iters} iterations; scaled linearly by M x{scale:.1f} to M={full.M}")}


def error_vs_oracle(workload: str, answers: dict, nmodes: int = 8) -> dict:
    """Relative error of each GPU answer against the oracle's exact solution
    u* = A^{-1} f on sampled sine modes (mode 0, the last mode and random
    ones), each mode's error divided by that mode's own exact norm; computed
    after the timed regions.  answers: {path: time-major FP64 solution}."""
    import numpy as np
    from oracle import bltt_oracle as O
    from paper_2307_07749_amd import workloads as W

    prob, seed = W.workload(workload)
    sysm = O.from_problem(prob)
    f = W.rhs_normal(prob, seed)
    rng = np.random.default_rng(12345)
    modes = sorted(set([0, 1, prob.M - 1] + [int(i) for i in rng.integers(0, prob.M, nmodes)]))
    ref = O.exact_modes(sysm, f, modes)
    out = {"modes": modes, "norm": "per-mode ||u_i - u*_i|| / ||u*_i||, max over the sampled modes"}
    for name, u in answers.items():
        got = O.project_modes(sysm, u, modes)
        out[name] = float((np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0)).max())
    return out


def counters_from_profiles(kernel: str, basis: str):
    """Per-launch SQ counter figures (VALU and LDS instructions, their issue
    time) of kernel class `kernel` from the committed counter summary, if it
    was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            entry = json.load(fh).get(basis, {}).get(kernel)
        if not entry or entry.get("source_sha256") != source_sha256():
            return None
        return entry
    except Exception:
        return None


def source_sha256() -> str:
    import hashlib
    src = os.path.join(ROOT, "paper_2307_07749_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(src)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(src, name), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def traffic_from_profiles(kernel: str, basis: str):
    """HBM bytes per launch of kernel class `kernel` (Krylov basis `basis`)
    from the committed rocprofv3 counter summary, if one exists for the
    current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            data = json.load(fh)
        entry = data.get(basis, {}).get(kernel)
        if not entry:
            return None
        if entry.get("source_sha256") != source_sha256():
            return None
        return entry.get("bytes_per_launch")
    except Exception:
        return None


def batched_bench(args) -> int:
    """The uneven batched workload (64 2D fractional instances, M from {63^2,
    127^2, 255^2}, N from {64, 256, 1024}, gamma ~ U(0.2, 0.8), alpha ~
    logU(1e-3, 1e-1), 4 right-hand sides each, seeds 4000 + 4i + r): one step
    is one batched solve of all 256 systems to tol.  Prints one JSON line."""
    import torch
    from paper_2307_07749_amd import bltt
    from paper_2307_07749_amd import workloads as W

    torch.cuda.set_device(0)
    params = W.batched_instances(64, 4)
    probs = [W.fractional_l1(2, m, N, g, a) for (m, N, g, a) in params]
    nrhs = 4
    fs = [torch.from_numpy(W.rhs_normal(pr, 4000 + 4 * i + r)).cuda() for i, pr in enumerate(probs)
          for r in range(nrhs)]
    us = [torch.empty_like(f) for f in fs]
    unknowns = sum(f.numel() for f in fs)
    print(f"[bench] batched: {len(fs)} systems, {unknowns / 1e9:.2f} G unknowns", file=sys.stderr, flush=True)
    b = bltt.Batch(probs, nrhs)
    for _ in range(args.warmup):
        b.pminres(fs, args.tol, args.maxit, us)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        _, iters, _, infos, rc = b.pminres(fs, args.tol, args.maxit, us)
        print(f"[bench] batched step {k}: {infos[0]['solve_ms']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    tpbs = b.classes()
    radix_plans = b.plans()  # per class: 0 = 16*8*8 / 16*8*4, 1 = 16*16*4 / 16*4*8 (N = 1024 / 512)
    b.close()
    out = {"metric": "batched time-to-1e-8 solves, 64 uneven 2D fractional instances x 4 RHS",
           "value": len(fs) * 1e3 / ms, "unit": "system-solves/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
           "config": {"workload": "batched64x4", "systems": len(fs), "unknowns": unknowns, "tol": args.tol,
                      "classes": len(tpbs), "workgroup_sizes": tpbs, "radix_plans": radix_plans},
           "iters": {"min": min(iters), "max": max(iters)},
           "max_true_relres": max(inf["true_relres"] for inf in infos), "status": int(rc),
           "unknowns_per_s": unknowns * 1e3 / ms}
    print(json.dumps(out), flush=True)
    return 0


# FP32 vector peak without packed FP32 (which the build disables): 256 CUs x
# 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 78.6
# algorithmic flops per element of one time-pass launch: four N-point complex
# FFTs per pair of real mode lines (5 N log2 N each, so 10 log2 N per
# element), plus the alpha scalings, the spectral multiplies with the
# eigenvalue square roots computed on the fly, and the Lanczos update (~24)
def time_pass_flops_per_elt(N: int) -> float:
    import math
    return 10.0 * math.log2(N) + 24.0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="frac2d_m511_n1024_g03",
                    help="a named single workload, or batched64x4 for the uneven batched workload")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=300)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64-path comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU leg (the oracle's timing and its check of the GPU answers)")
    ap.add_argument("--profile-steps", type=int, default=3,
                    help="solves of the separate per-kernel event-timing pass (0: none)")
    ap.add_argument("--basis", choices=["sine", "physical"], default="sine",
                    help="Krylov basis: sine coordinates (transform once) or physical space")
    ap.add_argument("--calibrate", action="store_true",
                    help="first run a plain streaming kernel of known size (2^28 floats negated into a second "
                         "buffer: 1 GiB read, 1 GiB written), whose FETCH_SIZE / WRITE_SIZE counters scale "
                         "the solver kernels' counters to bytes")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; the solver runs on one GPU only "
              f"(one MI355X holds the whole workload; a run over several GPUs would split the sine modes, "
              f"with two all-to-all transposes per solve)", file=sys.stderr)
        return 2

    if args.workload == "batched64x4":
        return batched_bench(args)

    import torch
    from paper_2307_07749_amd import bltt
    from paper_2307_07749_amd import workloads as W

    torch.cuda.set_device(0)
    if args.calibrate:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    prob, seed = W.workload(args.workload)
    f = torch.from_numpy(W.rhs_normal(prob, seed)).cuda()
    torch.cuda.synchronize()

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    basis = bltt.SINE if args.basis == "sine" else bltt.PHYSICAL
    hot = HOT_CLASSES[args.basis]

    def timed(solver, u, label):
        """warmup, then exactly args.steps solves with profiling off"""
        for _ in range(args.warmup):
            solver.pminres(f, args.tol, args.maxit, u)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last = None
        for k in range(args.steps):
            _, it, _, info, rc = solver.pminres(f, args.tol, args.maxit, u)
            last = (it, info, rc)
            log(f"[bench] {label} step {k}: {info['solve_ms']:.1f} ms iters={it} outer={info['iters_outer']} "
                f"relres={info['true_relres']:.2e}")
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps, last

    # ---- mixed path (the headline): timed with profiling off
    mixed = bltt.Solver.from_problem(prob, precision=bltt.MIXED, basis=basis)
    plans = mixed.plan_info()  # what the setup autotuner chose (or read from a plan cache)
    u_mixed = torch.empty_like(f)
    log(f"[bench] {args.workload}: n={prob.n} warmup={args.warmup} steps={args.steps}")
    ms_mixed, (iters_mixed, info_mixed, rc_mixed) = timed(mixed, u_mixed, "mixed")

    # ---- separate profiled pass: every kernel launch bracketed by HIP events
    # on the handle's stream, algorithmic bytes per launch accumulated per class
    prof = None
    ms_prof = None
    if args.profile_steps > 0:
        mixed.profile(True)
        t0 = time.perf_counter()
        for _ in range(args.profile_steps):
            mixed.pminres(f, args.tol, args.maxit, u_mixed)
        torch.cuda.synchronize()
        ms_prof = (time.perf_counter() - t0) * 1e3 / args.profile_steps
        prof = mixed.profile_read()
        mixed.profile(False)
    mixed.close()

    kernels, roofline, per_iter = {}, None, None
    if prof:
        total_ms = max(sum(v["ms"] for v in prof.values()), 1e-12)
        kernels = {c: {"launches": prof[c]["launches"],
                       "avg_us": 1e3 * prof[c]["ms"] / max(prof[c]["launches"], 1),
                       "GBps": prof[c]["bytes"] / (prof[c]["ms"] * 1e-3) / 1e9 if prof[c]["ms"] > 0 else 0.0,
                       "share": prof[c]["ms"] / total_ms}
                   for c in prof}
        # per MINRES iteration: the classes every iteration runs (algorithmic bytes / their time)
        hot_ms = sum(prof[c]["ms"] for c in hot)
        hot_bytes = sum(prof[c]["bytes"] for c in hot)
        hot_gbps = hot_bytes / (hot_ms * 1e-3) / 1e9 if hot_ms > 0 else 0.0
        per_iter = {"GBps": hot_gbps, "frac": hot_gbps / HBM_PEAK_GBPS, "classes": hot,
                    "bytes_per_elt_per_iter": hot_bytes / max(prof["time_prec"]["launches"], 1) / prob.n,
                    "ms_per_iter": hot_ms / max(prof["time_prec"]["launches"], 1)}
        # the dominant hot-path kernel class against its roofline
        dom = max(hot, key=lambda c: prof[c]["ms"])
        d = prof[dom]
        launch_s = d["ms"] * 1e-3 / max(d["launches"], 1)
        per_launch_bytes = d["bytes"] / max(d["launches"], 1)
        achieved = per_launch_bytes / launch_s / 1e9
        # the roofline that binds: arithmetic intensity against the ridge point
        flops_elt = time_pass_flops_per_elt(prob.N) if dom == "time_prec" else None
        alu = None
        bound = "hbm"
        if flops_elt is not None:
            ai = flops_elt * prob.n / per_launch_bytes
            ridge = FP32_VALU_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBPS * 1e9)
            bound = "hbm" if ai < ridge else "alu"
            tflops = flops_elt * prob.n / launch_s / 1e12
            alu = {"achieved": tflops, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": tflops / FP32_VALU_PEAK_TFLOPS, "flops_per_elt": flops_elt,
                   "arithmetic_intensity": ai, "ridge_flop_per_byte": ridge}
        cnt = counters_from_profiles(dom, args.basis)
        roofline = {"bound": bound, "kernel": dom, "achieved": achieved if bound == "hbm" else alu["achieved"],
                    "peak": HBM_PEAK_GBPS if bound == "hbm" else FP32_VALU_PEAK_TFLOPS,
                    "unit": "GB/s" if bound == "hbm" else "TFLOP/s",
                    "frac": (achieved / HBM_PEAK_GBPS) if bound == "hbm" else alu["frac"],
                    "traffic": traffic_from_profiles(dom, args.basis),
                    "algorithmic_bytes_per_launch": per_launch_bytes,
                    "avg_launch_us": launch_s * 1e6,
                    "hbm_frac": achieved / HBM_PEAK_GBPS,
                    "alu": alu,
                    # VALU issue time (SQ_INSTS_VALU x 4 cycles over 1024 SIMDs at 2.4 GHz) over the
                    # launch time, from the committed counter summary of the same kernel source
                    "valu_issue_frac": (cnt["valu_issue_us"] / (launch_s * 1e6)) if cnt else None}

    # ---- FP64 path beside it, timed the same way
    fp64 = None
    u64 = None
    if not args.no_fp64:
        s64 = bltt.Solver.from_problem(prob, precision=bltt.FP64, basis=basis)
        u64 = torch.empty_like(f)
        ms64, (it64, info64, rc64) = timed(s64, u64, "fp64")
        s64.close()
        fp64 = {"ms_per_solve": ms64, "iters": it64, "true_relres": info64["true_relres"], "status": int(rc64),
                "mixed_speedup": ms64 / ms_mixed}

    out = {
        "metric": "time-to-1e-8 solve + GB/s per PMINRES iter, 2D M=511²,N=1024, mixed vs FP64",
        "value": 1e3 / ms_mixed,
        "unit": "solve/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_mixed,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "dim": prob.dim, "m": prob.m[0], "M": prob.M, "N": prob.N,
                   "gamma": prob.meta.get("gamma"), "alpha": prob.alpha, "tol": args.tol, "seed": seed,
                   "precision": "mixed (FP32 MINRES sweeps, FP64 refinement)", "basis": args.basis},
        "mixed": {"ms_per_solve": ms_mixed, "ms_per_solve_profiled": ms_prof, "iters_inner": iters_mixed,
                  "iters_outer": info_mixed["iters_outer"], "true_relres": info_mixed["true_relres"],
                  "status": int(rc_mixed), "plans": plans, "kernels": kernels},
        "fp64": fp64,
        "per_iter": per_iter,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        # the CPU leg: the oracle's check of both GPU answers (after the timed
        # regions), then the oracle's own time on a bounded sample
        log("[bench] cpu leg: oracle error of the GPU answers ...")
        answers = {"mixed": u_mixed.cpu().numpy()}
        if u64 is not None:
            answers["fp64"] = u64.cpu().numpy()
        out["error_vs_oracle"] = error_vs_oracle(args.workload, answers)
        del answers
        log("[bench] cpu leg: oracle timing sample ...")
        out["cpu_baseline"] = cpu_baseline(args.workload, args.tol)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
