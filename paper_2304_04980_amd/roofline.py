"""Algorithmic byte counts of the hot kernels and rocprofv3 summaries.

The byte models (what a kernel must read and write at the least, per launch)
feed the roofline figures that `bench.py` reports; the command-line part
turns rocprofv3 output (kernel trace + stats, or one `--pmc` counter run) into
the short text summaries kept under `profiles/`, and the FETCH_SIZE /
WRITE_SIZE runs into `profiles/traffic.json`, which `bench.py` reads back as
measured HBM traffic while the kernel sources are unchanged.

    python -m paper_2304_04980_amd.roofline stats DIR/PREFIX --title T --command C
    python -m paper_2304_04980_amd.roofline traffic FETCH_PREFIX WRITE_PREFIX [...] \
        --copy-bytes B --title T --command C --json profiles/traffic.json

(PREFIX is rocprofv3's `-o`; the files read are PREFIX_kernel_stats.csv,
PREFIX_kernel_trace.csv and PREFIX_counter_collection.csv.)
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
TWIST_MIN = 8          # block rows from which Phi_bar is solved in the twisted order
FW_ROW, BW_ROW = 32, 16  # doubles per row of a forward / backward factor block row
EARLY_EXIT_NS = 8000   # dispatches this short are launches that found the solve stopped

# rocprofv3 names of the hot kernels per (path, kernel, element bytes); the
# Delta apply of the time-invariant path is two launches (w pass, y pass)
KERNEL_NAMES = {
    ("ti", "delta", 8): ["k_delta_w<double, 4>", "k_delta_y<double, 4>"],
    ("ti", "delta", 4): ["k_delta_w<float, 4>", "k_delta_y<float, 4>"],
    ("ti", "phi_solve", 8): ["k_phi_solve_twisted<double, 4>"],
    ("ti", "phi_solve", 4): ["k_phi_solve_twisted<float, 4>"],
    ("tv", "delta", 8): ["k_tv_delta_w<double, 4>", "k_tv_delta_y<double, 4>"],
    ("tv", "delta", 4): ["k_tv_delta_w<float, 4>", "k_tv_delta_y<float, 4>"],
    ("tv", "phi_solve", 8): ["k_tv_phi_solve<double, 4>"],
    ("tv", "phi_solve", 4): ["k_tv_phi_solve<float, 4>"],
    ("nt", "phi_solve", 8): ["k_nt_solve<double, 4, 8>"],
    ("nt", "phi_solve", 4): ["k_nt_solve<float, 4, 16>"],
}


def kernel_bytes(p, w=8, qt_distinct=False, path="ti"):
    """Algorithmic bytes per launch of the Delta apply ("delta") and of one
    block solve ("phi_solve"; for path "nt" the node-temporal solve) for
    problem p with w-byte vector elements (U = K N n (T+1) unknowns):

    ti, delta:      2 U w (read d, write y) + 13 n^2 w per node (the factored
                    form's blocks: 5 Cup, Q^-1, Q_T^-1 in the w pass, 5 A-hat,
                    B R^-1 B' in the y pass).
    ti, phi_solve:  2 U w (read tau, write theta) + the factor tables of the
                    time classes used (32 + 16 doubles per row of a 2n-row
                    block row; K+1 forward rows in the one-chain order, K+2
                    plus one row of middle couplings in the twisted order,
                    K >= 8) + the t = 0 block Q^-1 per node.
    tv, delta:      2 U w + 12 n^2 w per node and step (the factored form's
                    blocks, all per t: 5 Cup_t and Q_t^-1 in the w pass,
                    5 A-hat_{t-1} and B R^-1 B'_{t-1} in the y pass).
    tv, phi_solve:  2 U w + a one-chain factor per (super-column, t).
    nt, phi_solve:  2 U w + 3 n^2 w per node and step (L_t^-1, M_t, N_t).

    Intermediate round trips (the parked forward-sweep result, the Delta
    apply's w) are not algorithmic and show up as measured traffic above
    these figures."""
    K, N, T, n = p.K, p.N, p.T, p.n
    U = K * N * n * (T + 1)
    V = (N + 1) // 2
    nodes = K * N
    if path == "ti":
        ncls = 2 if qt_distinct else 1
        fw_rows = K + 3 if K >= TWIST_MIN else K + 1
        factors = ncls * V * 2 * n * (FW_ROW * fw_rows + BW_ROW * K) * w
        return {"delta": 2 * U * w + nodes * 13 * n * n * w,
                "phi_solve": 2 * U * w + factors + nodes * n * n * w}
    if path == "tv":
        factors = V * (T + 1) * 2 * n * (FW_ROW * (K + 1) + BW_ROW * K) * w
        return {"delta": 2 * U * w + nodes * (T + 1) * 12 * n * n * w,
                "phi_solve": 2 * U * w + factors}
    if path == "nt":
        return {"phi_solve": 2 * U * w + nodes * (T + 1) * 3 * n * n * w}
    raise ValueError(path)


def iteration_bytes(p, w, qt_distinct=False):
    """Algorithmic HBM bytes of one PCG iteration (S = L = 2) over the whole
    path: 21 full vector passes (Delta apply 2, update + first solve 7,
    second and third solves 3 each, fourth solve with the dot product 4 --
    the count of a fully fused iteration) plus the factor rows of four block
    solves and the operator blocks of the Delta apply (13 n^2 per node), the
    two Omega~ and the Xi~ right-hand sides (10 n^2 each)."""
    kb = kernel_bytes(p, w, qt_distinct)
    U = p.K * p.N * p.n * (p.T + 1)
    nodes = p.K * p.N
    factors = kb["phi_solve"] - 2 * U * w - nodes * p.n * p.n * w
    return 21 * U * w + 4 * factors + nodes * (13 + 3 * 10) * p.n * p.n * w


def src_hash():
    """Hash of every kernel source: counters taken on other sources are stale."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(PKG, "csrc", "*.h")) +
                    glob.glob(os.path.join(PKG, "csrc", "*.hip"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_record(path, names):
    """Measured HBM bytes per launch summed over the kernels `names` from a
    traffic record written by `traffic` below; None unless the record was
    taken on the current kernel sources and holds every name."""
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("src_sha") != src_hash():
        return None
    ks = rec.get("kernels", {})
    if not names or any(nm not in ks for nm in names):
        return None
    return sum(ks[nm]["bytes_per_launch"] for nm in names)


# ---------------------------------------------------------------------------
# rocprofv3 csv summaries

def short_name(full):
    """`void ns::(anonymous namespace)::k<double, 4>(args)` -> `k<double, 4>`."""
    s = full.strip()
    if s.startswith("void "):
        s = s[5:]
    depth, cut = 0, len(s)
    for i, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0 and not s.startswith("(anonymous", i):
            cut = i
            break
    s = s[:cut]
    for pre in ("lqg::(anonymous namespace)::", "(anonymous namespace)::", "lqg::"):
        s = s.replace(pre, "")
    return s


def _rows(path):
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def stats_table(prefix):
    """Per kernel: calls, total and average time from the stats file, and
    the average over the dispatches longer than EARLY_EXIT_NS from the
    trace."""
    stats = _rows(prefix + "_kernel_stats.csv")
    trace = _rows(prefix + "_kernel_trace.csv")
    full = {}
    for r in trace:
        dt = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        nm = short_name(r["Kernel_Name"])
        if dt > EARLY_EXIT_NS:
            c, s = full.get(nm, (0, 0))
            full[nm] = (c + 1, s + dt)
    total = sum(float(r["TotalDurationNs"]) for r in stats)
    out = []
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        nm = short_name(r["Name"])
        fc, fs = full.get(nm, (0, 0))
        out.append(dict(name=nm, calls=int(r["Calls"]),
                        total_ms=float(r["TotalDurationNs"]) / 1e6,
                        avg_us=float(r["AverageNs"]) / 1e3, full=fc,
                        full_avg_us=fs / fc / 1e3 if fc else 0.0,
                        pct=100.0 * float(r["TotalDurationNs"]) / total))
    return out


def counter_per_dispatch(prefix, counter):
    """{kernel: [value per dispatch]} of one counter (summed over the rows of
    a dispatch), with each dispatch's duration where the file has one."""
    rows = _rows(prefix + "_counter_collection.csv")
    disp = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        d = disp.setdefault(key, {"name": short_name(r["Kernel_Name"]), "v": 0.0,
                                  "dt": None})
        d["v"] += float(r["Counter_Value"])
        if r.get("Start_Timestamp") and r.get("End_Timestamp"):
            d["dt"] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    out = {}
    for d in disp.values():
        out.setdefault(d["name"], []).append((d["v"], d["dt"]))
    return out


def _working(vals):
    """The dispatches that did work: longer than EARLY_EXIT_NS where the
    duration is known, else above 1 % of the kernel's largest value."""
    if vals and all(dt is not None for _, dt in vals):
        keep = [v for v, dt in vals if dt > EARLY_EXIT_NS]
    else:
        top = max((v for v, _ in vals), default=0.0)
        keep = [v for v, _ in vals if v > 0.01 * top]
    return keep or [v for v, _ in vals]


def traffic_table(pairs, copy_bytes):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled to bytes by what
    they read for the largest plain copy in the same runs (a copy of
    copy_bytes reads and writes copy_bytes).  pairs: (fetch prefix, write
    prefix) of one workload each; each pair is scaled by its own copy."""
    kern, refs = {}, []
    for fetch_prefix, write_prefix in pairs:
        fetch = counter_per_dispatch(fetch_prefix, "FETCH_SIZE")
        write = counter_per_dispatch(write_prefix, "WRITE_SIZE")
        copy = [k for k in fetch if "copyBuffer" in k]
        if not copy:
            raise SystemExit(f"no plain copy dispatch in {fetch_prefix}")
        cname = copy[0]
        f_ref = max(v for v, _ in fetch[cname])
        w_ref = max(v for v, _ in write.get(cname, [(0.0, None)]))
        fscale = copy_bytes / (f_ref * 1024.0)
        wscale = copy_bytes / (w_ref * 1024.0) if w_ref > 0 else 1.0
        refs.append({"run": os.path.basename(fetch_prefix), "copy": cname,
                     "copy_fetch_kib": f_ref, "copy_write_kib": w_ref,
                     "fetch_scale": fscale, "write_scale": wscale})
        for nm, vals in fetch.items():
            if nm == cname or nm in kern:
                continue
            fv = _working(vals)
            wv = _working(write.get(nm, []))
            rb = sum(fv) / len(fv) * 1024.0 * fscale
            wb = (sum(wv) / len(wv) * 1024.0 * wscale) if wv else 0.0
            kern[nm] = {"dispatches": len(vals), "working_dispatches": len(fv),
                        "read_bytes": rb, "write_bytes": wb, "bytes_per_launch": rb + wb,
                        "run": os.path.basename(fetch_prefix)}
    return {"src_sha": src_hash(), "copy_bytes": copy_bytes, "references": refs,
            "kernels": dict(sorted(kern.items(), key=lambda kv: -kv[1]["bytes_per_launch"]))}


def _header(title, command, extra=""):
    return (f"# {title}\n\n{extra}Command (from the repository root on the MI355X "
            f"machine, after `cd /tmp && export TMPDIR=/tmp` and back):\n\n```\n"
            f"{command}\n```\n\n")


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2304_04980_amd.roofline")
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("prefix")
    a.add_argument("--title", required=True)
    a.add_argument("--command", required=True)
    a.add_argument("--note", default="")
    a.add_argument("--top", type=int, default=30)
    b = sub.add_parser("traffic")
    b.add_argument("prefixes", nargs="+",
                   help="FETCH_SIZE run prefix, WRITE_SIZE run prefix, per workload")
    b.add_argument("--copy-bytes", type=int, required=True)
    b.add_argument("--title", required=True)
    b.add_argument("--command", required=True)
    b.add_argument("--note", default="")
    b.add_argument("--json", default=None)
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        rows = stats_table(args.prefix)
        out = [_header(args.title, args.command, args.note + "\n\n" if args.note else ""),
               f"`avg us` is rocprofv3's average over all dispatches; `full avg us` "
               f"leaves out dispatches of {EARLY_EXIT_NS // 1000} us or less (launches "
               f"enqueued after a PCG run stopped, which exit at once), from the kernel "
               f"trace of the same run.\n\n",
               "| kernel | calls | total ms | avg us | full launches | full avg us | % |\n",
               "|---|---|---|---|---|---|---|\n"]
        for r in rows[:args.top]:
            out.append(f"| {r['name']} | {r['calls']} | {r['total_ms']:.2f} | "
                       f"{r['avg_us']:.1f} | {r['full']} | {r['full_avg_us']:.1f} | "
                       f"{r['pct']:.1f} |\n")
        sys.stdout.write("".join(out))
        return 0
    if len(args.prefixes) % 2:
        raise SystemExit("traffic takes FETCH_SIZE / WRITE_SIZE prefixes in pairs")
    pairs = list(zip(args.prefixes[0::2], args.prefixes[1::2]))
    rec = traffic_table(pairs, args.copy_bytes)
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")
    scal = "; ".join(
        f"run {r['run']}: the copy reads {r['copy_fetch_kib']:.0f} KiB of FETCH_SIZE and "
        f"{r['copy_write_kib']:.0f} KiB of WRITE_SIZE (x{r['fetch_scale'] * 1024:.1f} and "
        f"x{r['write_scale'] * 1024:.1f} bytes per KiB)" for r in rec["references"])
    out = [_header(args.title, args.command, args.note + "\n\n" if args.note else ""),
           f"Scaling: each run also copies {rec['copy_bytes']} bytes with a plain device "
           f"copy (__amd_rocclr_copyBuffer), which reads and writes that many bytes; "
           f"{scal}.  FETCH_SIZE counts L2 misses served by the fabric (MALL or HBM).  "
           f"Averages are over the dispatches that did work (longer than "
           f"{EARLY_EXIT_NS // 1000} us).  Kernel sources: {rec['src_sha']}.\n\n",
           "| kernel | run | dispatches | working | read MiB | write MiB |\n",
           "|---|---|---|---|---|---|\n"]
    for nm, k in rec["kernels"].items():
        out.append(f"| {nm} | {k['run']} | {k['dispatches']} | {k['working_dispatches']} | "
                   f"{k['read_bytes'] / 2**20:.1f} | {k['write_bytes'] / 2**20:.1f} |\n")
    sys.stdout.write("".join(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
