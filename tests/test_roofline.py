"""Host logic of the measurement tooling (paper_2304_04980_amd/roofline.py):
the algorithmic byte models, the rocprofv3 name parsing, the scaling of the
FETCH_SIZE / WRITE_SIZE counters by the plain-copy reference, and the rule
that a traffic record only counts while the kernel sources are unchanged."""
import csv
import json
import os
from types import SimpleNamespace

import pytest

from paper_2304_04980_amd import roofline as rf


def prob(K, N, T, n=4, m=2):
    return SimpleNamespace(K=K, N=N, T=T, n=n, m=m)


def test_short_names():
    assert rf.short_name("void lqg::(anonymous namespace)::k_phi_solve_twisted<double, 4>"
                         "(lqg::Dims, lqg::OpCoef<double>, double const*)") == \
        "k_phi_solve_twisted<double, 4>"
    assert rf.short_name("void lqg::(anonymous namespace)::k_nt_solve<float, 4, 16>"
                         "(lqg::Dims, float const*)") == "k_nt_solve<float, 4, 16>"
    assert rf.short_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_byte_models_scale_as_stated():
    p = prob(16, 16, 40)
    U = p.K * p.N * p.n * (p.T + 1)
    for path in ("ti", "tv", "nt"):
        b8, b4 = rf.kernel_bytes(p, 8, path=path), rf.kernel_bytes(p, 4, path=path)
        for k in b8:  # every term is linear in the element size
            assert b8[k] == 2 * b4[k]
            assert b8[k] > 2 * U * 8  # the two vector passes plus coefficients
    # time-varying coefficients grow with T + 1, time-invariant ones do not
    q = prob(16, 16, 81)
    Uq = q.K * q.N * q.n * (q.T + 1)
    ti_p, ti_q = rf.kernel_bytes(p, 8), rf.kernel_bytes(q, 8)
    assert ti_q["delta"] - 2 * Uq * 8 == ti_p["delta"] - 2 * U * 8
    tv_p, tv_q = rf.kernel_bytes(p, 8, path="tv"), rf.kernel_bytes(q, 8, path="tv")
    per_t_p = (tv_p["delta"] - 2 * U * 8) / (p.T + 1)
    per_t_q = (tv_q["delta"] - 2 * Uq * 8) / (q.T + 1)
    assert per_t_p == per_t_q == p.K * p.N * 12 * p.n ** 2 * 8
    nt = rf.kernel_bytes(p, 8, path="nt")["phi_solve"]
    assert nt == 2 * U * 8 + p.K * p.N * (p.T + 1) * 3 * p.n ** 2 * 8
    # the twisted order (K >= 8) holds two more factor rows per super-column
    a, b = rf.kernel_bytes(prob(7, 4, 10), 8), rf.kernel_bytes(prob(8, 4, 10), 8)
    Ua, Ub = 7 * 4 * 4 * 11, 8 * 4 * 4 * 11
    fa = a["phi_solve"] - 2 * Ua * 8 - 7 * 4 * 16 * 8
    fb = b["phi_solve"] - 2 * Ub * 8 - 8 * 4 * 16 * 8
    V = 2
    assert fa == V * 8 * (32 * 8 + 16 * 7) * 8
    assert fb == V * 8 * (32 * 11 + 16 * 8) * 8
    with pytest.raises(ValueError):
        rf.kernel_bytes(p, 8, path="xx")


def _write_counters(path, counter, rows):
    """rows: (dispatch, kernel name, value KiB, start ns, end ns)."""
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name",
                    "Counter_Value", "Start_Timestamp", "End_Timestamp"])
        for d, name, v, t0, t1 in rows:
            w.writerow([d, d, name, counter, v, t0, t1])


def test_traffic_scaling_and_early_exit_filter(tmp_path, monkeypatch):
    monkeypatch.setattr(rf, "src_hash", lambda: "h0")
    copy = "__amd_rocclr_copyBuffer"
    kern = "void lqg::(anonymous namespace)::k_x<float, 4>(lqg::Dims)"
    # the copy of 1 MiB reads 512 KiB of FETCH_SIZE (x2) and 1024 KiB of WRITE_SIZE
    fetch = [(1, copy, 512.0, 0, 50_000),
             (2, kern, 100.0, 0, 20_000), (3, kern, 300.0, 0, 20_000),
             (4, kern, 1.0, 0, 2_000)]  # a launch that exited at once: left out
    write = [(1, copy, 1024.0, 0, 50_000),
             (2, kern, 10.0, 0, 20_000), (3, kern, 30.0, 0, 20_000),
             (4, kern, 0.0, 0, 2_000)]
    _write_counters(tmp_path / "f_counter_collection.csv", "FETCH_SIZE", fetch)
    _write_counters(tmp_path / "w_counter_collection.csv", "WRITE_SIZE", write)
    rec = rf.traffic_table([(str(tmp_path / "f"), str(tmp_path / "w"))], 1 << 20)
    k = rec["kernels"]["k_x<float, 4>"]
    assert k["dispatches"] == 3 and k["working_dispatches"] == 2
    assert k["read_bytes"] == pytest.approx(200.0 * 1024 * 2)
    assert k["write_bytes"] == pytest.approx(20.0 * 1024)
    assert k["bytes_per_launch"] == pytest.approx(k["read_bytes"] + k["write_bytes"])
    assert rec["src_sha"] == "h0"

    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    assert rf.traffic_from_record(str(path), ["k_x<float, 4>"]) == \
        pytest.approx(k["bytes_per_launch"])
    assert rf.traffic_from_record(str(path), ["k_x<float, 4>", "k_missing"]) is None
    monkeypatch.setattr(rf, "src_hash", lambda: "h1")  # sources changed: stale
    assert rf.traffic_from_record(str(path), ["k_x<float, 4>"]) is None
    assert rf.traffic_from_record(str(tmp_path / "none.json"), ["k_x<float, 4>"]) is None


def test_committed_record_names_the_hot_kernels():
    """The committed record covers every kernel the bench reports a roofline
    for (it may be stale; bench.py then reports traffic as null)."""
    path = os.path.join(os.path.dirname(__file__), "..", "profiles", "traffic.json")
    rec = json.load(open(path))
    for names in rf.KERNEL_NAMES.values():
        for nm in names:
            assert nm in rec["kernels"], nm
