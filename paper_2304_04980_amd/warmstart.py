"""Training and use of the learned warm start (the lqgrid_wsnet_* kernels).

The network predicts the Chebyshev-in-time coefficients of delta~ for a
problem from its x0 and per-node parameters; the expansion is passed to
lqgrid_pcg_solve as delta_init, with the fallback to a zero start when it
does not lower the residual.  Training data are solves of the method itself:
each training problem is solved to a relative KKT residual of 1e-8 by the
batched FP64 path (the library's FP64 true residual confirms every one), and
the network is trained by the library's forward and backward kernels with
Adam.  This module only orchestrates those calls (data generation, epochs,
learning-rate schedule, evaluation).

    python -m paper_2304_04980_amd.warmstart --train 2048 --val 128 --test 32

writes the trained parameters to weights/wsnet_K64_N64_T100.npz and prints
one JSON line with the training history and the measured gain.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from lqgrid_synth import CONFIGS, learned_problem  # noqa: E402

from . import lqgrid  # noqa: E402

WEIGHTS = os.path.join(HERE, "weights", "wsnet_K64_N64_T100.npz")
TRAIN_SEEDS = (0, 20000)
VAL_SEEDS = (20000, 20500)
TEST_SEEDS = (10 ** 6, 10 ** 6 + 200)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def learned_net(**kw):
    c = CONFIGS["learned"]
    return lqgrid.WarmNet(c["K"], c["N"], c["n"], c["m"], c["T"], **kw)


def _gen(seed):
    return learned_problem(seed)


def cpu_pool(workers):
    """Worker processes for problem generation.  Create it before anything
    touches the GPU: the workers are forked and only run numpy."""
    if workers <= 1:
        return None
    import multiprocessing as mp
    return mp.get_context("fork").Pool(workers)


def problems(seeds, pool=None):
    """Problems of the learned configuration (deterministic per seed)."""
    if pool is None:
        return [learned_problem(s) for s in seeds]
    return pool.map(_gen, seeds, chunksize=4)


def build_dataset(net, seeds, tol=1e-8, chunk=128, pool=None):
    """Features and targets of the problems `seeds`, each solved by the
    batched FP64 path to `tol`.  Returns (feats, tgts, stats)."""
    import torch
    feats = net.alloc_features(len(seeds))
    tgts = net.alloc_targets(len(seeds))
    iters, worst = [], 0.0
    opts = lqgrid.default_opts(tol=tol)
    t0 = time.perf_counter()
    for c0 in range(0, len(seeds), chunk):
        ps = problems(seeds[c0:c0 + chunk], pool)
        b = lqgrid.Batch(ps, opts=opts)
        outs, infos, st = b.solve()
        if st != lqgrid.OK or any(i["rel_kkt_residual"] > tol for i in infos):
            raise RuntimeError(f"training solve failed: status {st}")
        for k in range(len(ps)):
            net.features(b.descs[k], b.x0s[k], feats[c0 + k])
            net.targets(outs[k], tgts[c0 + k])
        iters += [i["iterations"] for i in infos]
        worst = max(worst, max(i["rel_kkt_residual"] for i in infos))
        torch.cuda.synchronize()
        del b, outs
        log(f"  dataset {c0 + len(ps)}/{len(seeds)} ({time.perf_counter() - t0:.1f} s)")
    return feats, tgts, dict(mean_iterations=float(np.mean(iters)),
                             max_residual=worst, seconds=time.perf_counter() - t0)


def mean_loss(net, feats, tgts, batch=16):
    import torch
    S = feats.shape[0]
    tot = 0.0
    for c0 in range(0, S, batch):
        idx = torch.arange(c0, min(S, c0 + batch), dtype=torch.int32, device=net.device)
        loss, _ = net.gradient(feats, tgts, idx)
        tot += loss * idx.numel()
    return tot / S


def train(net, feats, tgts, epochs=30, batch=16, lr=2e-3, val=None, seed=0):
    """Adam with a cosine learning-rate decay over `epochs` passes of
    shuffled minibatches.  Returns the history of (epoch, train, val) loss."""
    import torch
    rng = np.random.default_rng(seed)
    S = feats.shape[0]
    per = max(1, S // batch)
    total = epochs * per
    grad = torch.empty(net.count, dtype=torch.float32, device=net.device)
    hist = []
    step = 0
    t0 = time.perf_counter()
    for e in range(epochs):
        perm = rng.permutation(S)
        run = 0.0
        for k in range(per):
            idx = torch.as_tensor(perm[k * batch:(k + 1) * batch].astype(np.int32),
                                  device=net.device)
            loss, _ = net.gradient(feats, tgts, idx, grad=grad)
            net.adam(grad, lr * 0.5 * (1.0 + math.cos(math.pi * step / total)))
            run += loss
            step += 1
        vl = mean_loss(net, *val) if val is not None else None
        hist.append((e, run / per, vl))
        log(f"  epoch {e}: train {run / per:.4f} val {vl if vl is None else round(vl, 4)} "
            f"({time.perf_counter() - t0:.1f} s)")
    return hist


def warm_solve(ctx, net, feat, x0, opts, out=None):
    """Predict delta_init and solve; returns (delta, info)."""
    d0 = net.predict(feat)
    delta, _, _, info = ctx.solve(x0, opts, delta_init=d0, out=out)
    return delta, info


def evaluate(net, seeds, tol=1e-8, repeats=3):
    """Per test problem: PCG iterations and wall time (setup excluded, CNN
    inference included) of the zero start and of the warm start."""
    import torch
    opts = lqgrid.default_opts(tol=tol)
    rows = []
    feat = net.alloc_features(1)[0]
    for s in seeds:
        p = learned_problem(s)
        ctx = lqgrid.Context(p)
        x0 = torch.as_tensor(p.x0).to(dtype=torch.float64, device=net.device).contiguous()
        out = torch.empty((p.T + 1, p.N, p.K, p.n), dtype=torch.float64, device=net.device)
        net.features(ctx.desc, x0, feat)
        ctx.solve(x0, opts, out=out)                 # warm the caches
        tz, tw = [], []
        for _ in range(repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, _, _, iz = ctx.solve(x0, opts, out=out)
            torch.cuda.synchronize()
            tz.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            net.features(ctx.desc, x0, feat)
            _, iw = warm_solve(ctx, net, feat, x0, opts, out=out)
            torch.cuda.synchronize()
            tw.append(time.perf_counter() - t0)
        ctx.close()
        rows.append(dict(seed=s, zero_it=iz["iterations"], warm_it=iw["iterations"],
                         zero_s=min(tz), warm_s=min(tw), warm_used=iw["warm_start_used"],
                         zero_res=iz["rel_kkt_residual"], warm_res=iw["rel_kkt_residual"],
                         ok=iz["status"] == lqgrid.OK and iw["status"] == lqgrid.OK))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2048)
    ap.add_argument("--val", type=int, default=128)
    ap.add_argument("--test", type=int, default=32)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--layers", type=int, default=6)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--out", default=WEIGHTS)
    args = ap.parse_args()
    pool = cpu_pool(args.workers)
    net = learned_net(layers=args.layers, seed=0)
    tr = list(range(TRAIN_SEEDS[0], TRAIN_SEEDS[0] + args.train))
    va = list(range(VAL_SEEDS[0], VAL_SEEDS[0] + args.val))
    te = list(range(TEST_SEEDS[0], TEST_SEEDS[0] + args.test))
    log(f"building the training set ({len(tr)} solves) ...")
    ftr, ttr, s_tr = build_dataset(net, tr, pool=pool)
    log(f"building the validation set ({len(va)} solves) ...")
    fva, tva, s_va = build_dataset(net, va, pool=pool)
    if pool is not None:
        pool.close()
    init_val = mean_loss(net, fva, tva)
    log(f"training: initial validation loss {init_val:.4f}")
    t0 = time.perf_counter()
    hist = train(net, ftr, ttr, epochs=args.epochs, batch=args.batch, lr=args.lr,
                 val=(fva, tva))
    t_train = time.perf_counter() - t0
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    net.save(args.out)
    rows = evaluate(net, te)
    zi = float(np.mean([r["zero_it"] for r in rows]))
    wi = float(np.mean([r["warm_it"] for r in rows]))
    zs = float(np.mean([r["zero_s"] for r in rows]))
    wsv = float(np.mean([r["warm_s"] for r in rows]))
    res = dict(train_solves=len(tr), val_solves=len(va), test_solves=len(te),
               dataset=s_tr, init_val_loss=init_val, history=hist,
               train_seconds=t_train, zero_iterations=zi, warm_iterations=wi,
               zero_solves_per_s=1.0 / zs, warm_solves_per_s=1.0 / wsv,
               warm_used=sum(r["warm_used"] for r in rows),
               all_ok=all(r["ok"] for r in rows), rows=rows, weights=args.out)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
