#!/usr/bin/env python3
"""Benchmark of the NBJM-preconditioned PCG solve of the grid LQ problem.

One step = one pass of the whole path over one synthetic problem whose arrays
are already resident in HBM: lqgrid_setup (ingest + Schur-block assembly),
lqgrid_factor (banded block Cholesky of every Phi_bar), lqgrid_pcg_solve
(Algorithm 1 + Algorithm 2 preconditioner to the tolerance, true FP64
residual check, output transpose and the recovery of x~ and u~).  Both forms
run in one invocation on the same inputs: plain FP64 PCG, then the chosen form
(default: FP32 stencil apply and sweeps inside FP64 iterative refinement).
value = steps / wall time of the chosen form's timed steps (solves/s); the
plain figures are reported beside it.  After timing, the FP64 oracle evaluates
the KKT residual of each form's last solution (delta~, x~, u~).  The default
headline run also times the batched form (256 uneven problems) and the learned
warm start (64 x 64 x 100) on their own workloads, and the other problem
classes at the headline's dimensions (time-varying data, the node-temporal
preconditioner, boundary states with per-node sizes) and the standalone NBJM,
and adds their summaries to the same line (`batched`, `learned`, `rows`).
`--workload` runs any of them alone as the line's value.

Prints ONE JSON line.  Only one GPU is used; --gpus N > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("solves/s to 1e-8 rel. KKT residual, K=N=128 T=200 (plain vs chosen); "
          "HBM %")
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, 8 TB/s
# Kernel durations come from HIP events around every PROFILE_STRIDE-th launch
# of each hot kernel inside the timed steps: an event pair serialises the
# dispatch of the launches around it (timing every launch costs ~11% of the
# solve rate), so only a sample is timed.
PROFILE_STRIDE = 16
PROFILE_DIR = os.path.join(ROOT, "profiles")
TRAFFIC = os.path.join(PROFILE_DIR, "traffic.json")

from paper_2304_04980_amd.roofline import (  # noqa: E402
    KERNEL_NAMES, iteration_bytes, kernel_bytes, traffic_from_record)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(p, tol, gpu_iters):
    """The FP64 oracle (numpy/scipy slab operators, Algorithm 1 with the
    Algorithm 2 preconditioner) timed on complete solves of a bounded sample:
    the 32 x 32 x 100 problem (n = 4, m = 2, seed 0) to the same tolerance,
    once with every core of this process's affinity mask available to the
    numerical libraries and once with one thread.  Generation is excluded;
    operator setup and factorisation are included.  The per-solve time of
    the benchmarked workload is estimated from the measured one by the
    per-iteration cost being linear in the number of unknowns (Table I):
    t_solve * (U / U_sample) * (iterations / sample iterations)."""
    from threadpoolctl import threadpool_limits
    from lqgrid_synth import config_problem
    from oracle import slab, nbjm, pcg
    sample, _ = config_problem("plain", 0)
    cores = len(os.sched_getaffinity(0))

    def timed(threads):
        with threadpool_limits(threads):
            t0 = time.perf_counter()
            ops = slab.SlabOperators(sample)
            pre = nbjm.slab_preconditioner(ops, 2, 2)
            _, it, _ = pcg.pcg(ops.delta, pre, ops.r_delta(), tol=tol)
            return time.perf_counter() - t0, it

    t_all, it_all = timed(cores)
    t_one, it_one = timed(1)
    scale = (p.unknowns / sample.unknowns) * (gpu_iters / it_all)
    est = t_all * scale
    return {
        "value": 1.0 / est, "unit": "solves/s", "cores": cores, "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": (f"complete oracle solves (setup + factor + PCG to tol {tol}) at "
                   f"K={sample.K} N={sample.N} T={sample.T} n={sample.n} m={sample.m}: "
                   f"{t_all:.2f} s with {cores} threads, {t_one:.2f} s with 1 thread, "
                   f"{it_all} iterations; value = estimated solves/s at K={p.K} N={p.N} "
                   f"T={p.T}: measured time x {p.unknowns}/{sample.unknowns} unknowns x "
                   f"{gpu_iters}/{it_all} iterations (cost per iteration linear in the "
                   f"unknowns); the sparse products run on one thread whatever the limit"),
        "measured": {"K": sample.K, "N": sample.N, "T": sample.T, "tol": tol,
                     "iterations": it_all,
                     "seconds_all_cores": t_all, "solves_per_s_all_cores": 1.0 / t_all,
                     "seconds_1_thread": t_one, "solves_per_s_1_thread": 1.0 / t_one,
                     "iterations_1_thread": it_one},
        "estimated_seconds_per_solve": est,
    }


def make_inputs(p, torch, dev):
    f64 = dict(dtype=torch.float64, device=dev)
    arrays = {k: torch.as_tensor(getattr(p, k)).to(**f64).contiguous()
              for k in ("A", "A_nbr", "B", "Q", "R", "QT")}
    for k in ("n_node", "m_node"):
        v = getattr(p, k, None)
        if v is not None:
            arrays[k] = torch.as_tensor(v).to(dtype=torch.int32, device=dev).contiguous()
    x0 = torch.as_tensor(p.x0).to(**f64).contiguous()
    return arrays, x0


def measure(p, tol, arrays, x0, ws, precision, inner_tol, steps, warmup, torch,
            lqgrid, path="ti", opts_kw=None, ctx_kw=None, boundary=None):
    """Time `steps` full passes (setup + factor + solve) of one form after
    `warmup` untimed ones; per-kernel averages from the library's HIP events
    on its stream over the timed steps.  path: "ti" (time-invariant data),
    "tv" (time-varying data) or "nt" (node-temporal preconditioner), for the
    kernel names and byte models; opts_kw / ctx_kw: extra solve options and
    Context arguments; boundary: known boundary states for the solve."""
    extra = dict(opts_kw or {})
    if precision == "fp32r":
        opts = lqgrid.default_opts(tol=tol, precision=lqgrid.FP32_REFINE,
                                   inner_tol=inner_tol, **extra)
    else:
        opts = lqgrid.default_opts(tol=tol, **extra)
    w = 4 if precision == "fp32r" else 8
    f64 = dict(dtype=torch.float64, device=x0.device)
    delta = torch.empty((p.T + 1, p.N, p.K, p.n), **f64)
    xs = torch.empty((p.T + 1, p.N, p.K, p.n), **f64)
    us = torch.empty((p.T, p.N, p.K, p.m), **f64)

    def step(profile):
        ctx = lqgrid.Context(p, workspace=ws, arrays=arrays, factor=False,
                             **(ctx_kw or {}))
        if profile:
            ctx.profile_enable(True, stride=PROFILE_STRIDE)
        ctx.factor()
        _, _, _, info = ctx.solve(x0, opts, out=delta, out_x=xs, out_u=us,
                                  boundary=boundary)
        prof = {k: ctx.profile_read(k) for k in range(4)} if profile else None
        ctx.close()
        return info, prof

    for s in range(warmup):
        info, _ = step(False)
        log(f"[{precision}] warmup {s}: {info['iterations']} it, "
            f"res {info['rel_kkt_residual']:.2e}, {info['seconds']*1e3:.1f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step(True) for _ in range(steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    infos = [r[0] for r in runs]
    for s, info in enumerate(infos):
        log(f"[{precision}] step {s}: status {info['status']} {info['iterations']} it, "
            f"{info['refinements']} passes, res {info['rel_kkt_residual']:.2e}, "
            f"solve {info['seconds']*1e3:.1f} ms")
    names = {0: "delta", 1: "phi_solve", 2: "rhs", 3: "update"}
    kern = {}
    for k, nm in names.items():
        launches = sum(r[1][k][0] for r in runs)
        ms = sum(r[1][k][1] for r in runs)
        kern[nm] = {"timed_launches": launches, "timed_ms": round(ms, 3),
                    "avg_ms": ms / launches if launches else None}
    kb = kernel_bytes(p, w, path=path)
    if path == "nt":  # the Delta apply of the time-invariant path
        kb["delta"] = kernel_bytes(p, w)["delta"]
    per_kernel = {}
    for nm in ("delta", "phi_solve"):
        if kern[nm]["avg_ms"]:
            names = KERNEL_NAMES.get(("ti" if nm == "delta" and path == "nt" else path,
                                      nm, w), [])
            per_kernel[nm] = {
                "kernels": names,
                "achieved": round(kb[nm] / (kern[nm]["avg_ms"] * 1e-3) / 1e9, 1),
                "avg_launch_ms": kern[nm]["avg_ms"], "algorithmic_bytes": kb[nm],
                "traffic": traffic_from_record(TRAFFIC, names)}
    dom = max(per_kernel, key=lambda k: kern[k]["timed_ms"])
    iters = sum(i["iterations"] for i in infos) / len(infos)
    return {
        "value": steps / elapsed, "ms_per_step": elapsed / steps * 1e3,
        "converged": all(i["status"] == lqgrid.OK and i["rel_kkt_residual"] <= tol
                         for i in infos),
        "pcg_iterations": iters,
        "refinements": sum(i["refinements"] for i in infos) / len(infos),
        "pcg_iters_per_s": iters * steps / elapsed,
        "rel_kkt_residual": max(i["rel_kkt_residual"] for i in infos),
        "kernels": kern, "hot": per_kernel, "dominant": dom,
        "solution": (delta, xs, us),
    }


def bench_batched(args, torch, lqgrid):
    """256 problems with K, N ~ U{8..64}, T ~ U{50..200} (FP64, tol 1e-8):
    one lqgrid_batch_solve per step, against the same problems solved one
    after another by the single-problem path (setup + factor + solve each)."""
    from lqgrid_synth import batched_problems, BATCHED_TOL
    probs, tol = batched_problems(), BATCHED_TOL
    U = sum(p.unknowns for p in probs)
    log(f"batched workload: {len(probs)} problems, {U / 1e6:.1f} M unknowns, tol {tol}")
    opts = lqgrid.default_opts(tol=tol)
    b = lqgrid.Batch(probs, opts=opts)
    for w in range(args.warmup):
        _, infos, st = b.solve()
        log(f"warmup {w}: status {st}, {infos[0]['seconds']:.3f} s")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [b.solve() for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    infos = runs[-1][1]
    ok = all(r[2] == lqgrid.OK for r in runs) and all(
        i["rel_kkt_residual"] <= tol for r in runs for i in r[1])
    its = [i["iterations"] for i in infos]
    del b, runs
    torch.cuda.empty_cache()

    # the same problems, one after another through the single-problem path
    seq = None
    if not args.no_plain:
        f64 = dict(dtype=torch.float64, device="cuda")
        dev = []
        for p in probs:
            arrays, x0 = make_inputs(p, torch, "cuda")
            dev.append((p, arrays, x0))
        maxb = max(lqgrid.workspace_bytes(p.K, p.N, p.T, p.n, p.m) for p in probs)
        ws = torch.empty(maxb + 256, dtype=torch.uint8, device="cuda")

        def one_pass():
            res = []
            for p, arrays, x0 in dev:
                ctx = lqgrid.Context(p, workspace=ws, arrays=arrays, factor=True)
                out = torch.empty((p.T + 1, p.N, p.K, p.n), **f64)
                _, _, _, info = ctx.solve(x0, opts, out=out)
                ctx.close()
                res.append(info)
            return res

        one_pass()  # warm
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sinfos = one_pass()
        torch.cuda.synchronize()
        st = time.perf_counter() - t1
        seq = {"value": len(probs) / st, "seconds": st,
               "pcg_iterations_total": sum(i["iterations"] for i in sinfos),
               "converged": all(i["status"] == lqgrid.OK for i in sinfos)}
        log(f"sequential single-problem path: {st:.3f} s for {len(probs)} solves")
    value = len(probs) * args.steps / elapsed
    path_bytes = sum(i["iterations"] * iteration_bytes(p, 8) for p, i in zip(probs, infos))
    achieved = path_bytes / (elapsed / args.steps) / 1e9
    result = {
        "metric": "batched solves/s to 1e-8 rel. KKT residual, 256 problems "
                  "K,N~U{8..64} T~U{50..200}",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batched: {len(probs)} problems, K,N~U{{8..64}}, "
                               f"T~U{{50..200}}, n=4, m=2, FP64 PCG, S=L=2, tol={tol}",
                   "problems": len(probs), "unknowns": U, "tol": tol,
                   "step": "lqgrid_batch_solve (setup+factor+solve of all problems)"},
        "converged": ok, "pcg_iterations_min": min(its), "pcg_iterations_max": max(its),
        "pcg_iterations_total": sum(its),
        "rel_kkt_residual": max(i["rel_kkt_residual"] for i in infos),
        "sequential_fp64": seq,
        "speedup_vs_sequential": None if seq is None else value / seq["value"],
        "roofline": {"bound": "hbm", "kernel": "whole path (every kernel of the batched "
                     "solve)", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None,
                     "note": "algorithmic bytes of every problem's PCG iterations "
                             "(21 vector passes + factor rows + operator blocks per "
                             "iteration) over the wall time of one batched solve"},
        "cpu_baseline": None,
    }
    return result


def bench_learned(args, torch, lqgrid):
    """K = N = 64, T = 100 (FP64, tol 1e-8): solves from the learned warm start
    (features + network inference + solve, with the fallback to a zero start)
    against the zero start, on held-out test seeds, with the committed
    network.  A step is one solve of each test problem."""
    from paper_2304_04980_amd import warmstart
    net = lqgrid.WarmNet.load_file(warmstart.WEIGHTS)
    seeds = list(range(warmstart.TEST_SEEDS[0], warmstart.TEST_SEEDS[0] + 8))
    rows = warmstart.evaluate(net, seeds, repeats=max(1, args.steps))
    zi = sum(r["zero_it"] for r in rows) / len(rows)
    wi = sum(r["warm_it"] for r in rows) / len(rows)
    zs = sum(r["zero_s"] for r in rows)
    wsec = sum(r["warm_s"] for r in rows)
    result = {
        "metric": "solves/s to 1e-8 rel. KKT residual with the learned warm start "
                  "(inference included) vs zero start, K=N=64 T=100",
        "value": len(rows) / wsec, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": wsec * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16+f64", "data": "synthetic",
        "config": {"workload": "learned: K=64 N=64 T=100 n=4 m=2, FP64 PCG S=L=2, tol=1e-8, "
                               "6-layer 3x3 conv net (64 ch, BF16 MFMA), 16 Chebyshev "
                               "coefficients per state component",
                   "test_seeds": [seeds[0], seeds[-1]]},
        "converged": all(r["ok"] for r in rows),
        "warm_pcg_iterations": wi, "zero_pcg_iterations": zi,
        "zero_start_solves_per_s": len(rows) / zs,
        "speedup_vs_zero_start": zs / wsec,
        "predictions_kept": sum(r["warm_used"] for r in rows),
        "predictions": len(rows),
        "roofline": None, "cpu_baseline": None,
    }
    from lqgrid_synth import learned_problem
    p = learned_problem(seeds[0])
    achieved = wi * iteration_bytes(p, 8) / (wsec / len(rows)) / 1e9
    result["roofline"] = {
        "bound": "hbm", "kernel": "whole path (inference + solve)",
        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
        "note": "algorithmic bytes of the PCG iterations over the wall time of a "
                "warm-started solve (features and network inference included)"}
    return result


# Problem classes beyond the headline's, on the headline's dimensions
# (K = N = 128, T = 200, n = 4, m = 2, tol 1e-8): each runs both forms like
# the headline (the device FP64 KKT residual decides convergence; the oracle's
# parity on these classes is covered by the GPU tests at smaller sizes).
ROWS = {
    "tv": {"desc": "time-varying data (A_t, A_nbr_t, B_t, Q_t, R_t per step)",
           "path": "tv", "make": {"time_varying": True}},
    "nodetemporal": {"desc": "node-temporal block Jacobi preconditioner",
                     "path": "nt", "make": {}},
    "boundary": {"desc": "known boundary states, per-node sizes n_ij in 1..4, "
                         "m_ij in 1..2", "path": "ti",
                 "make": {"boundary": True, "sizes": True}},
}


def row_problem(name, seed):
    from lqgrid_synth import CONFIGS, make_problem
    c = dict(CONFIGS["headline"])
    tol = c.pop("tol")
    return make_problem(seed=seed, **c, **ROWS[name]["make"]), tol


def bench_nbjm(args, torch, lqgrid):
    """Algorithm 2 run as a solver (S = 1 outer sweep per step, L = 2 inner,
    outer sweeps to the tolerance; FP64) on the headline problem, beside
    Algorithm 1 with the same sweeps as preconditioner, and the Lanczos
    estimates of kappa(Delta) and kappa(P^-1 Delta) from one CG and one PCG
    run.  A step is one standalone NBJM solve (setup + factor + sweeps)."""
    from lqgrid_synth import config_problem
    p, tol = config_problem("headline", args.seed)
    arrays, x0 = make_inputs(p, torch, "cuda")
    ws = torch.empty(lqgrid.workspace_bytes(p.K, p.N, p.T, p.n, p.m) + 256,
                     dtype=torch.uint8, device="cuda")
    opts = lqgrid.default_opts(tol=tol, check_every=32)
    torch.cuda.synchronize()

    def step(profile):
        ctx = lqgrid.Context(p, workspace=ws, arrays=arrays, factor=False)
        if profile:
            ctx.profile_enable(True, stride=PROFILE_STRIDE)
        ctx.factor()
        _, _, _, info = ctx.nbjm_solve(x0, opts)
        prof = {k: ctx.profile_read(k) for k in range(4)} if profile else None
        ctx.close()
        return info, prof

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [step(True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    infos = [r[0] for r in runs]
    sweeps = sum(i["iterations"] for i in infos) / len(infos)
    log(f"[nbjm] {sweeps:.0f} sweeps, res {infos[-1]['rel_kkt_residual']:.2e}, "
        f"{elapsed / args.steps:.3f} s per solve")
    kern = {}
    for k, nm in {1: "phi_solve", 2: "rhs"}.items():
        launches = sum(r[1][k][0] for r in runs)
        ms = sum(r[1][k][1] for r in runs)
        kern[nm] = {"timed_launches": launches, "timed_ms": round(ms, 3),
                    "avg_ms": ms / launches if launches else None}
    kb = kernel_bytes(p, 8)["phi_solve"]
    names = KERNEL_NAMES[("ti", "phi_solve", 8)]
    avg = kern["phi_solve"]["avg_ms"]
    achieved = kb / (avg * 1e-3) / 1e9
    # Algorithm 1 with the same sweeps, and the conditioning estimates
    ctx = lqgrid.Context(p, workspace=ws, arrays=arrays, factor=True)
    t1 = time.perf_counter()
    _, _, _, pinfo = ctx.solve(x0, lqgrid.default_opts(tol=tol))
    t_pcg = time.perf_counter() - t1
    kap = {}
    for key, mode in (("cg", 0), ("pcg", 1)):
        kap[key] = ctx.condition_estimate(x0, preconditioned=mode, tol=tol)
    ctx.close()
    return {
        "metric": "standalone NBJM solves/s to 1e-8 rel. KKT residual, K=N=128 T=200 "
                  "(vs Algorithm 1 with the same preconditioner); HBM %",
        "value": args.steps / elapsed, "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"nbjm: K={p.K} N={p.N} T={p.T} n={p.n} m={p.m}, FP64 "
                               f"Algorithm 2 to convergence (L=2, inner start from the "
                               f"outer iterate), tol={tol}",
                   "check_every": 32},
        "converged": all(i["status"] == lqgrid.OK and i["rel_kkt_residual"] <= tol
                         for i in infos),
        "sweeps": sweeps, "rel_kkt_residual": max(i["rel_kkt_residual"] for i in infos),
        "kernels": kern,
        "pcg": {"iterations": pinfo["iterations"], "seconds": t_pcg,
                "solves_per_s": 1.0 / t_pcg, "rel_kkt_residual": pinfo["rel_kkt_residual"]},
        "speedup_pcg_vs_nbjm": (elapsed / args.steps) / t_pcg,
        "condition": {k: {kk: v[kk] for kk in ("kappa", "lambda_min", "lambda_max",
                                               "iterations")} for k, v in kap.items()},
        "roofline": {"bound": "hbm", "kernel": "phi_solve", "kernels": names,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_record(TRAFFIC, names),
                     "algorithmic_bytes": kb, "avg_launch_ms": avg},
        "cpu_baseline": None,
    }


def bench_single(args, torch, lqgrid):
    """One problem of args.workload (headline, plain, tiny or a ROWS class):
    plain FP64 and the chosen form measured on the same inputs; returns the
    result dict of the JSON line (with the oracle check and the CPU baseline
    for the non-row workloads unless switched off)."""
    from lqgrid_synth import config_problem
    row = ROWS.get(args.workload)
    if row is None:
        p, tol = config_problem(args.workload, args.seed)
    else:
        p, tol = row_problem(args.workload, args.seed)
    path = row["path"] if row else "ti"
    dev = "cuda"
    arrays, x0 = make_inputs(p, torch, dev)
    nbytes = lqgrid.workspace_bytes(p.K, p.N, p.T, p.n, p.m,
                                    time_varying=path == "tv", node_temporal=path == "nt")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    mkw = {}
    if path == "nt":
        mkw = dict(opts_kw={"preconditioner": lqgrid.PRECOND_NODE_TEMPORAL},
                   ctx_kw={"node_temporal": True})
    if row is not None and p.has_boundary:
        mkw["boundary"] = {k: torch.as_tensor(getattr(p, k)).to(
            dtype=torch.float64, device=dev).contiguous()
            for k in ("alpha_lo", "alpha_hi", "beta_lo", "beta_hi")}
    torch.cuda.synchronize()
    log(f"workload {args.workload}: K={p.K} N={p.N} T={p.T} n={p.n} m={p.m} "
        f"U={p.unknowns} tol={tol} workspace {nbytes / 2**30:.1f} GiB")

    plain = None
    if not args.no_plain and args.precision != "fp64":
        plain = measure(p, tol, arrays, x0, ws, "fp64", args.inner_tol,
                        args.steps, args.warmup, torch, lqgrid, path=path, **mkw)
    chosen = measure(p, tol, arrays, x0, ws, args.precision, args.inner_tol,
                     args.steps, args.warmup, torch, lqgrid, path=path, **mkw)

    dom = chosen["dominant"]
    hot = chosen["hot"][dom]
    roofline = {"bound": "hbm", "kernel": dom, "kernels": hot["kernels"],
                "achieved": hot["achieved"],
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hot["achieved"] / HBM_PEAK_GBS, 4),
                "traffic": hot["traffic"], "algorithmic_bytes": hot["algorithmic_bytes"],
                "avg_launch_ms": hot["avg_launch_ms"],
                "other_kernels": {k: v for k, v in chosen["hot"].items() if k != dom}}

    # plain copy of known size: reference for scaling the PMC byte counters
    nel = args.copy_ref_mib * (1 << 20) // 8
    a = torch.ones(nel, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b

    form = ("FP32 stencil apply and sweeps, FP64 scalars, factors and outer "
            "refinement" if args.precision == "fp32r" else "plain FP64 PCG")
    metric = METRIC if row is None else (
        f"solves/s to {tol:g} rel. KKT residual, K={p.K} N={p.N} T={p.T}, "
        f"{row['desc']} (plain vs chosen); HBM %")
    wname = args.workload if row is None else f"{args.workload} ({row['desc']})"
    result = {
        "metric": metric,
        "value": chosen["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": chosen["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{wname}: K={p.K} N={p.N} T={p.T} n={p.n} "
                               f"m={p.m}, {form}, S=L=2, tol={tol}",
                   "K": p.K, "N": p.N, "T": p.T, "n": p.n, "m": p.m,
                   "S": 2, "L": 2, "tol": tol, "precision": args.precision,
                   "inner_tol": args.inner_tol if args.precision == "fp32r" else None,
                   "step": "setup+factor+pcg_solve"},
        "converged": chosen["converged"],
        "pcg_iterations": chosen["pcg_iterations"],
        "refinements": chosen["refinements"],
        "pcg_iters_per_s": chosen["pcg_iters_per_s"],
        "rel_kkt_residual": chosen["rel_kkt_residual"],
        "kernels": chosen["kernels"],
        "kernel_timing": f"HIP events on the library's stream around every "
                         f"{PROFILE_STRIDE}th launch of each kernel in the timed steps, "
                         "without the check batch in which each PCG run stops (its "
                         "launches may exit at once); a timed launch includes its "
                         "dispatch and completion",
        "roofline": roofline,
        "plain_fp64": None if plain is None else {
            k: plain[k] for k in ("value", "ms_per_step", "converged", "pcg_iterations",
                                  "pcg_iters_per_s", "rel_kkt_residual", "hot")},
        "speedup_vs_plain": None if plain is None else chosen["value"] / plain["value"],
        "cpu_baseline": None,
    }
    if not args.no_oracle_check and row is None:
        # the oracle's FP64 KKT residual of the last timed step's delta~, x~, u~
        # (all three blocks of the KKT system), for each form
        from oracle import slab, residual
        log("checking the solutions with the FP64 oracle ...")
        ops = slab.SlabOperators(p)
        for name, rec in (("chosen", chosen), ("plain", plain)):
            if rec is None:
                continue
            d, xs, us = (t.cpu().numpy() for t in rec["solution"])
            g = residual.kkt_residual(ops, d.reshape(p.T + 1, -1),
                                      xs.reshape(p.T + 1, -1), us.reshape(p.T, -1))
            target = result if name == "chosen" else result["plain_fp64"]
            target["oracle_rel_kkt_residual"] = g["rel2"]
            target["converged"] = bool(target["converged"] and g["rel2"] <= tol)
            log(f"  {name}: oracle relative KKT residual {g['rel2']:.3e}")
        del ops
    if not args.no_cpu_baseline and row is None:
        log("timing the CPU oracle on a bounded sample ...")
        result["cpu_baseline"] = cpu_baseline(p, tol, int(round(
            plain["pcg_iterations"] if plain else chosen["pcg_iterations"])))
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "plain", "tiny", "learned", "batched", "nbjm"]
                    + list(ROWS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp32r", choices=["fp64", "fp32r"],
                    help="form reported as value (fp32r: FP32 sweeps inside FP64 "
                         "iterative refinement); plain FP64 is always measured "
                         "beside it unless --no-plain")
    ap.add_argument("--inner-tol", type=float, default=1e-4)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="headline only: skip the batched and learned summaries")
    ap.add_argument("--no-rows", action="store_true",
                    help="headline only: skip the summaries of the other problem "
                         "classes (time-varying, node-temporal, boundary + sizes) "
                         "and of the standalone NBJM")
    ap.add_argument("--form-steps", type=int, default=2,
                    help="timed steps of the batched, learned and row summaries")
    ap.add_argument("--copy-ref-mib", type=int, default=512,
                    help="size of the plain copy used to scale PMC counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path; "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2304_04980_amd import lqgrid

    if args.workload == "batched":
        print(json.dumps(bench_batched(args, torch, lqgrid)), flush=True)
        return
    if args.workload == "learned":
        print(json.dumps(bench_learned(args, torch, lqgrid)), flush=True)
        return
    if args.workload == "nbjm":
        print(json.dumps(bench_nbjm(args, torch, lqgrid)), flush=True)
        return
    result = bench_single(args, torch, lqgrid)
    torch.cuda.empty_cache()
    if args.workload == "headline" and not args.no_forms:
        # the other two forms of the method on their own workloads, as
        # summaries in the same line
        sub = argparse.Namespace(**vars(args))
        sub.steps, sub.warmup = args.form_steps, 1
        for key, fn in (("batched", bench_batched), ("learned", bench_learned)):
            try:
                r = fn(sub, torch, lqgrid)
                result[key] = {k: r.get(k) for k in (
                    "metric", "value", "unit", "ms_per_step", "converged", "config",
                    "roofline", "speedup_vs_sequential", "sequential_fp64",
                    "speedup_vs_zero_start", "zero_start_solves_per_s",
                    "warm_pcg_iterations", "zero_pcg_iterations", "predictions_kept",
                    "predictions", "pcg_iterations_total", "rel_kkt_residual")
                    if k in r}
            except Exception as e:  # reported, never hides the headline line
                result[key] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.empty_cache()
    if args.workload == "headline" and not args.no_rows:
        # the other problem classes and the standalone NBJM at the headline's
        # dimensions, as summaries in the same line
        rows = {}
        for name in list(ROWS) + ["nbjm"]:
            sub = argparse.Namespace(**vars(args))
            sub.workload, sub.steps, sub.warmup = name, args.form_steps, 1
            sub.no_oracle_check = sub.no_cpu_baseline = True
            try:
                r = (bench_nbjm if name == "nbjm" else bench_single)(sub, torch, lqgrid)
                rows[name] = {k: r.get(k) for k in (
                    "metric", "value", "unit", "ms_per_step", "converged", "config",
                    "pcg_iterations", "refinements", "sweeps", "rel_kkt_residual",
                    "speedup_vs_plain", "pcg", "speedup_pcg_vs_nbjm", "condition",
                    "roofline") if k in r}
                if r.get("plain_fp64"):
                    rows[name]["plain_fp64"] = {k: r["plain_fp64"].get(k) for k in (
                        "value", "ms_per_step", "converged", "pcg_iterations")}
            except Exception as e:  # reported, never hides the headline line
                rows[name] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.empty_cache()
        result["rows"] = rows
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
