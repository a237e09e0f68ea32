"""bench.py --summarize on small synthetic rocprofv3 outputs (CPU): the FP64
flops per evaluation from the VALU counters, the copy-calibrated HBM bytes,
and the source hash that bench.py checks before it uses either."""
from __future__ import annotations

import csv
import os

import pytest

import bench

KR = "void gpw::k_rho<1, 1, 1, 2, true, false, double>(gpw::SegTable<gpw::RhoSeg>)"
KM = "void gpw::k_mat<1, 1, double, false>(gpw::SegTable<gpw::PairSeg>)"
KP = "void gpw::k_pack_direct<double, 3, 3>(gpw::SegTable<gpw::PackSeg>)"
COPY = "__amd_rocclr_copyBuffer"


def _write(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=list(rows[0]))
        w.writeheader()
        w.writerows(rows)


def _counter_rows(disp):
    """disp: list of (kernel, duration ns, {counter: value})."""
    rows = []
    for i, (k, dur, cs) in enumerate(disp):
        for n, v in cs.items():
            rows.append({"Dispatch_Id": i, "Kernel_Name": k, "Counter_Name": n, "Counter_Value": v,
                         "Start_Timestamp": 1000, "End_Timestamp": 1000 + dur})
    return rows


def _trace_rows(disp):
    return [{"Kernel_Name": k, "Start_Timestamp": 0, "End_Timestamp": dur} for k, dur in disp]


@pytest.fixture
def prof_dir(tmp_path):
    d = tmp_path / "prof"
    inc = [0] * 15
    inc[2] = 1000                  # (p|p) incidences
    with open(d.mkdir() or d / "bench.err", "w") as f:
        f.write("[bench] per class: " + ", ".join(f"x: 1 pairs / {i} blocks" for i in inc) + "\n")
    ev = [(KR, 2_000_000), (KM, 3_000_000), (KP, 100_000)] * 6
    _write(str(d / "stats" / "run_kernel_stats.csv"),
           [{"Name": k, "Calls": 6, "TotalDurationNs": 6 * t, "AverageNs": t} for k, t in ev[:3]])
    _write(str(d / "stats" / "run_kernel_trace.csv"), _trace_rows(ev))
    _write(str(d / "stats_x" / "run_kernel_trace.csv"),
           _trace_rows([("void gpw::k_grad<1, 1, double, false>(gpw::SegTable<gpw::PairSeg>)", 5_000_000)] * 3))
    f64 = {"SQ_INSTS_VALU_FMA_F64": 100.0, "SQ_INSTS_VALU_ADD_F64": 10.0, "SQ_INSTS_VALU_MUL_F64": 20.0,
           "SQ_INSTS_VALU_TRANS_F64": 0.0, "SQ_INSTS_VALU": 200.0, "SQ_BUSY_CU_CYCLES": 400.0,
           "GRBM_GUI_ACTIVE": 8 * 2.0e6 * 2.0}
    _write(str(d / "f64" / "run_counter_collection.csv"),
           _counter_rows([(KR, 2_000_000, f64), (KM, 2_000_000, f64)] * 3))
    _write(str(d / "fetch" / "run_counter_collection.csv"),
           _counter_rows([(KR, 1, {"FETCH_SIZE": 1000.0}), (KP, 1, {"FETCH_SIZE": 200.0}),
                          (KM, 1, {"FETCH_SIZE": 50.0})] * 6))
    _write(str(d / "write" / "run_counter_collection.csv"),
           _counter_rows([(KR, 1, {"WRITE_SIZE": 10.0}), (KM, 1, {"WRITE_SIZE": 30.0})] * 6))
    _write(str(d / "cal_fetch" / "run_counter_collection.csv"),
           _counter_rows([("fill", 1, {"FETCH_SIZE": 0.0}), (COPY, 1, {"FETCH_SIZE": float(1 << 19)})]))
    _write(str(d / "cal_write" / "run_counter_collection.csv"),
           _counter_rows([("fill", 1, {"WRITE_SIZE": float(1 << 20)}), (COPY, 1, {"WRITE_SIZE": float(1 << 20)})]))
    sq = {"SQ_INSTS_VALU": 100.0, "SQ_INSTS_SALU": 50.0, "SQ_ACTIVE_INST_VALU": 1.0, "SQ_BUSY_CYCLES": 1.0}
    _write(str(d / "sq1" / "run_counter_collection.csv"), _counter_rows([(KR, 1, sq), (KM, 1, sq)]))
    sq2 = {"SQ_INSTS_LDS": 20.0, "SQ_INSTS_VMEM_RD": 5.0, "SQ_BUSY_CU_CYCLES": 200.0}
    _write(str(d / "sq2" / "run_counter_collection.csv"), _counter_rows([(KR, 1, sq2), (KM, 1, sq2)]))
    return d


def _values(path):
    out = {}
    for line in open(path):
        parts = line.split()
        if len(parts) == 2 and not line.startswith(("#", "|")):
            out[parts[0]] = parts[1]
    return out


def test_counters_and_traffic_from_synthetic_outputs(prof_dir, tmp_path):
    out = tmp_path / "profiles"
    out.mkdir()
    bench.summarize_profiles(str(prof_dir), str(out))
    v = _values(out / "k_rho_k_mat_water256_fp64_counters.md")
    # (2 FMA + ADD + MUL) x 64 lanes per dispatch, 3 dispatches per kernel
    assert float(v["eval_rho_flops"]) == pytest.approx((2 * 100 + 10 + 20) * 64)
    assert float(v["eval_mat_flops"]) == pytest.approx((2 * 100 + 10 + 20) * 64)
    assert v["source_sha256"] == bench._sources_sha()
    t = _values(out / "eval_rho_eval_mat_water256_hbm_traffic.txt")
    # the copy kernel alone calibrates: FETCH x 2, WRITE x 1; KiB -> bytes; 6 evaluations
    assert float(t["eval_rho_fetch_bytes"]) == pytest.approx((1000 + 200) * 2 * 1024)
    assert float(t["eval_rho_write_bytes"]) == pytest.approx(10 * 1024)
    assert float(t["eval_mat_bytes"]) == pytest.approx((50 * 2 + 30) * 1024)
    stats = open(out / "k_rho_k_mat_water256_kernel_stats.md").read()
    assert "| pp | 1000 | 2.000 |" in stats
    grad = open(out / "k_grad_k_tau_water256_kernel_stats.md").read()
    assert "grad 5.000 ms" in grad


def test_bench_ignores_summaries_of_other_sources(tmp_path, monkeypatch):
    sha = bench._sources_sha()
    f = tmp_path / "profiles" / "k_rho_k_mat_water256_fp64_counters.md"
    f.parent.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "_sources_sha", lambda: sha)
    f.write_text(f"eval_rho_flops 1e11\neval_mat_flops 2e11\nsource_sha256 {sha}\n")
    assert bench.counter_flops() == {"eval_rho": 1e11, "eval_mat": 2e11}
    f.write_text("eval_rho_flops 1e11\neval_mat_flops 2e11\nsource_sha256 0123\n")
    assert bench.counter_flops() is None
