#!/usr/bin/env python3
"""Benchmark of the NBJM-preconditioned PCG solve of the grid LQ problem.

One step = one pass of the whole path over one synthetic problem whose arrays
are already resident in HBM: lqgrid_setup (ingest + Schur-block assembly),
lqgrid_factor (banded block Cholesky of every Phi_bar), lqgrid_pcg_solve
(Algorithm 1 + Algorithm 2 preconditioner to the tolerance, true-residual
check) and the output transpose.  value = steps / wall time of the timed
steps (solves/s).

Prints ONE JSON line.  Only one GPU is used; --gpus N > 1 exits with a message.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("solves/s to 1e-8 rel. KKT residual, K=N=128 T=200 (plain vs chosen); "
          "HBM %")
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, 8 TB/s
PROFILE_DIR = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(p, precision_bytes=8):
    """Algorithmic HBM bytes of one launch of each hot kernel.

    U = K N n (T+1) unknowns, w = bytes per vector element.
      Delta apply: read d, write y (2 U w) + the operator blocks read once:
                   per node 13 (G) + 5 (Cdn) + 5 (Cup) + 2 (Q^-1, Q_T^-1 - Q^-1)
                   n x n FP64 blocks.
      Phi solve:   read tau, write theta (2 U w) + the factors of the one
                   interior class: V K block rows x 6 (2n)^2 FP64 + Q (t = 0).
    """
    K, N, T, n = p.K, p.N, p.T, p.n
    U = K * N * n * (T + 1)
    V = (N + 1) // 2
    w = precision_bytes
    nodes = K * N
    return {
        "delta": 2 * U * w + nodes * 25 * n * n * 8,
        "phi_solve": 2 * U * w + V * K * 6 * (2 * n) ** 2 * 8 + nodes * n * n * 8,
    }


def src_hash():
    h = hashlib.sha256()
    for f in ("ops.hip", "lqg_internal.h"):
        with open(os.path.join(ROOT, "paper_2304_04980_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_name):
    """HBM bytes per launch measured with rocprofv3 --pmc FETCH_SIZE and
    WRITE_SIZE (see profiles/traffic.json), only if taken on the current
    kernel source; else None."""
    path = os.path.join(PROFILE_DIR, "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("src_sha") != src_hash():
        return None
    k = rec.get("kernels", {}).get(kernel_name)
    return None if k is None else k.get("bytes_per_launch")


def cpu_baseline(p, tol, gpu_iters):
    """The FP64 oracle (numpy/scipy, one thread) timed on a bounded sample of
    the same workload: slab-operator setup with the Phi_bar factorisation,
    the initial residual and preconditioner, and one PCG iteration; the
    per-solve time is extrapolated with the GPU's iteration count."""
    from threadpoolctl import threadpool_limits
    from oracle import slab, nbjm, pcg
    with threadpool_limits(1):
        t0 = time.perf_counter()
        ops = slab.SlabOperators(p)
        for t in sorted({0, 1, p.T}):
            ops._factor(t)
        t1 = time.perf_counter()
        pre = nbjm.slab_preconditioner(ops, 2, 2)
        r = ops.r_delta()
        d = pre(r)
        float((d * r).sum())
        t2 = time.perf_counter()
        y = ops.delta(d)
        th = float((r * d).sum()) / float((y * d).sum())
        r = r - th * y
        q = pre(r)
        float((q * r).sum())
        t3 = time.perf_counter()
    setup, init, it = t1 - t0, t2 - t1, t3 - t2
    per_solve = setup + init + gpu_iters * it
    return {
        "value": 1.0 / per_solve, "unit": "solves/s", "cores": 1, "kind": "oracle",
        "sample": (f"oracle slab setup+factor ({setup:.1f}s), initial preconditioner "
                   f"({init:.1f}s) and 1 PCG iteration ({it:.2f}s) at K={p.K} N={p.N} "
                   f"T={p.T}; per-solve time = setup + init + {gpu_iters} iterations"),
        "seconds_per_solve": per_solve,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "plain", "tiny", "learned"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32r"],
                    help="fp32r: FP32 sweeps inside FP64 iterative refinement")
    ap.add_argument("--inner-tol", type=float, default=1e-4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-ref-mib", type=int, default=512,
                    help="size of the plain copy used to scale PMC counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path; "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from lqgrid_synth import config_problem
    from paper_2304_04980_amd import lqgrid

    p, tol = config_problem(args.workload, args.seed)
    dev = "cuda"
    f64 = dict(dtype=torch.float64, device=dev)
    arrays = {k: torch.as_tensor(getattr(p, k)).to(**f64).contiguous()
              for k in ("A", "A_nbr", "B", "Q", "R", "QT")}
    x0 = torch.as_tensor(p.x0).to(**f64).contiguous()
    nbytes = lqgrid.workspace_bytes(p.K, p.N, p.T, p.n, p.m)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    delta = torch.empty((p.T + 1, p.N, p.K, p.n), **f64)
    if args.precision == "fp32r":
        opts = lqgrid.default_opts(tol=tol, precision=lqgrid.FP32_REFINE,
                                   inner_tol=args.inner_tol)
    else:
        opts = lqgrid.default_opts(tol=tol)
    wbytes = 4 if args.precision == "fp32r" else 8
    torch.cuda.synchronize()

    def step(profile=False):
        ctx = lqgrid.Context(p, workspace=ws, arrays=arrays, factor=False)
        if profile:
            ctx.profile_enable(True)
        ctx.factor()
        _, _, _, info = ctx.solve(x0, opts, out=delta)
        prof = None
        if profile:
            prof = {k: ctx.profile_read(k) for k in range(4)}
        ctx.close()
        return info, prof

    log(f"workload {args.workload}: K={p.K} N={p.N} T={p.T} n={p.n} m={p.m} "
        f"U={p.unknowns} tol={tol}")
    for w in range(args.warmup):
        info, _ = step()
        log(f"warmup {w}: {info['iterations']} it, res {info['rel_kkt_residual']:.2e}, "
            f"{info['seconds']*1e3:.1f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, profs = [], []
    for s in range(args.steps):
        info, prof = step(profile=True)
        infos.append(info)
        profs.append(prof)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for s, info in enumerate(infos):
        log(f"step {s}: status {info['status']} {info['iterations']} it, "
            f"res {info['rel_kkt_residual']:.2e}, solve {info['seconds']*1e3:.1f} ms")
    ok = all(i["status"] == lqgrid.OK and i["rel_kkt_residual"] <= tol for i in infos)
    iters = sum(i["iterations"] for i in infos) / len(infos)

    # per-kernel averages from the live HIP events over the timed steps
    names = {0: "delta", 1: "phi_solve", 2: "rhs", 3: "update"}
    kern = {}
    for k, nm in names.items():
        launches = sum(pr[k][0] for pr in profs)
        ms = sum(pr[k][1] for pr in profs)
        kern[nm] = {"launches": launches, "total_ms": ms,
                    "avg_ms": ms / launches if launches else None}
    dom = max(("delta", "phi_solve"), key=lambda k: kern[k]["total_ms"])
    alg = kernel_bytes(p, wbytes)[dom]
    achieved = alg / (kern[dom]["avg_ms"] * 1e-3) / 1e9
    traffic = traffic_from_profiles(dom)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic, "algorithmic_bytes": alg,
                "avg_launch_ms": kern[dom]["avg_ms"]}
    other = "phi_solve" if dom == "delta" else "delta"
    if kern[other]["avg_ms"]:
        roofline["other_kernel"] = {
            "kernel": other,
            "achieved": round(kernel_bytes(p, wbytes)[other] / (kern[other]["avg_ms"] * 1e-3) / 1e9, 1),
            "avg_launch_ms": kern[other]["avg_ms"]}

    # plain copy of known size: reference for scaling the PMC byte counters
    nel = args.copy_ref_mib * (1 << 20) // 8
    a = torch.ones(nel, **f64)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b

    result = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: K={p.K} N={p.N} T={p.T} n={p.n} "
                               f"m={p.m}, {'plain FP64 PCG' if args.precision == 'fp64' else 'FP32 sweeps + FP64 refinement'}, S=L=2, tol={tol}",
                   "K": p.K, "N": p.N, "T": p.T, "n": p.n, "m": p.m,
                   "S": 2, "L": 2, "tol": tol, "precision": args.precision,
                   "step": "setup+factor+pcg_solve"},
        "converged": ok,
        "pcg_iterations": iters,
        "refinements": sum(i["refinements"] for i in infos) / len(infos),
        "pcg_iters_per_s": iters * args.steps / elapsed,
        "rel_kkt_residual": max(i["rel_kkt_residual"] for i in infos),
        "kernels": kern,
        "roofline": roofline,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        result["cpu_baseline"] = cpu_baseline(p, tol, int(round(iters)))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
