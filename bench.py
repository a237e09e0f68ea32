#!/usr/bin/env python3
"""Benchmark of the multigrid GPW hot path on one MI355X.

One step = eval_rho (density matrix -> rho on every level) + eval_mat (level
potentials -> matrix) of the 256-water-like system (config-5 member with 256
water units: 768 atoms, 10496 Cartesian AOs, levels 400/130/45/15 Ry, mesh
192^3/108^3/64^3/40^3, tau = 1e-6), FP64, inputs resident in HBM.

Prints ONE JSON line.  ``value`` is GFLOP/s of the FP64 arithmetic the rho
and mat kernels execute: (2 FMA + ADD + MUL) x 64 lanes per evaluation from
the rocprofv3 FP64 VALU counters in profiles/ while the kernel sources still
hash to the value recorded there, else the plan's kernel flop model (the
direct evaluation for the classes evaluated directly, the coefficient-tensor
Horner evaluation of Eq. (rho1) and the potential moments for the others).
``roofline`` prices the slower of eval_rho and eval_mat (all its launches, timed
with events on the stream they run on) against the FP64 vector peak, with its
HBM bytes from the counter summary.  ``convention_gflops`` counts instead the
fixed per-(pair image, grid point) convention F = 2 n_a n_b + 2 (n_a + n_b) + 4
of the direct evaluation over the 64 points of every 4x4x4 block a truncation
sphere meets; the factorised kernels need fewer operations than that, so the
convention rate of a class can exceed the hardware peak.  ``useful_gflops``
counts the convention over the points inside the spheres only.  The serving
block replays a Poisson trace of mixed requests at several rates, continuous
batching against one request at a time; ``cpu_baseline`` times the oracle on
a bounded sample of the same workload on the host.

``--summarize DIR`` writes the profiles/ summaries from rocprofv3 outputs.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12      # MI355X FP64 vector FMA peak: 256 CU x 128 flop/clk x 2.4 GHz


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="water256", choices=["water256", "c2", "c3", "c4"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-atoms", type=int, default=0, help="atoms in the oracle sample (0 = auto)")
    ap.add_argument("--extras", type=int, default=1, help="also time grad, fp32 and the plan")
    ap.add_argument("--serve-requests", type=int, default=600, help="requests in the serving run (0 = skip)")
    ap.add_argument("--serve-rates", default="20,50,100,200", help="Poisson arrival rates (requests/s), comma-separated")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0, help="HBM budget of the serving run")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device to device (reference for the HBM byte counters) and exit")
    ap.add_argument("--summarize", metavar="DIR",
                    help="write the profiles/ summaries from the rocprofv3 outputs under DIR (no GPU; see "
                         "summarize_profiles) and exit")
    return ap.parse_args()


def make_system(name):
    from paper_2603_24881_amd import synth
    if name == "water256":
        return synth.water256(), "water256: 256 water-like units, L=29.53 bohr, 768 atoms, 10496 AOs, O 3s2p2d1f / H 2s1p"
    s = synth.CONFIGS[name]()
    return s, f"{name}: {s.natm} atoms, {s.n_ao} AOs"


def timed(fn, steps, stream):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end) / 1e3 / steps


def _sources_sha():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2603_24881_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith((".hip", ".h")):
            with open(os.path.join(csrc, fn), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def counter_flops():
    """FP64 flops per evaluation of eval_rho and eval_mat on the 256-water system,
    from the committed rocprofv3 FP64 VALU counter summary ((2 FMA + ADD + MUL) x 64
    lanes), or None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "k_rho_k_mat_water256_fp64_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        parts = line.split()
        if len(parts) == 2 and parts[0] in ("eval_rho_flops", "eval_mat_flops", "source_sha256"):
            vals[parts[0]] = parts[1]
    if vals.get("source_sha256") != _sources_sha() or len(vals) != 3:
        return None
    return {"eval_rho": float(vals["eval_rho_flops"]), "eval_mat": float(vals["eval_mat_flops"])}


def measured_traffic(op):
    """HBM bytes per evaluation of ``op`` from the committed rocprofv3 counter
    summary, or None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "eval_rho_eval_mat_water256_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()[:2]
        vals[k] = v
    if vals.get("source_sha256") != _sources_sha() or f"{op}_bytes" not in vals:
        return None
    return int(vals[f"{op}_bytes"])


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_small_configs():
    """The oracle (rho + mat) on configs 1 and 2: median of 3 runs with all
    host threads, and with one thread (config 1: median of 3; config 2: one
    run), seconds."""
    import oracle
    from paper_2603_24881_amd import synth
    nall = oracle.num_threads()
    out = {}
    for name, reps1 in (("config1", 3), ("config2", 1)):
        s = getattr(synth, name)()
        o = oracle.Oracle(s)
        D = synth.make_density(s)
        V = synth.make_potentials(o.meshes, s.seed)
        res = {}
        for nt, reps in ((nall, 3), (1, reps1)):
            oracle.set_num_threads(nt)
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                o.rho(D)
                o.mat(V)
                ts.append(time.perf_counter() - t0)
            res[f"s_{nt}_threads"] = round(float(np.median(ts)), 4)
            res[f"runs_{nt}_threads"] = reps
        oracle.set_num_threads(nall)
        out[name] = res
        log(f"[bench] oracle {name}: {res}")
    return out


def cpu_baseline(system, D_np, V_np, natoms_hint, info, job_work):
    """The oracle on a bounded sample: the ordered pair images whose first
    primitive sits on the first ``n`` atoms; rho and mat.  Its rate is stated
    in the GPU's unit: the oracle evaluates ordered pairs (each canonical pair
    image twice), so the sample is the fraction ordered_sample / (2 x canonical
    in-sphere work of the job) of the job, and value = that fraction of the
    job's work (``job_work``, the same count as the GPU value) per second of
    oracle time: both values measure job throughput."""
    import oracle
    n = natoms_hint or max(3, int(round(system.natm * 0.30)))
    mask = np.zeros(system.natm, dtype=np.uint8)
    mask[:n] = 1
    o = oracle.Oracle(system, atom_mask=mask)
    t0 = time.perf_counter()
    o.rho(D_np)
    t1 = time.perf_counter()
    c_rho = o.counts.copy()
    o.mat(V_np)
    t2 = time.perf_counter()
    c_mat = o.counts.copy()
    flops = 0.0
    for la in range(5):
        for lb in range(5):
            na, nb = (la + 1) * (la + 2) // 2, (lb + 1) * (lb + 2) // 2
            f = 2 * na * nb + 2 * (na + nb) + 4
            flops += f * (c_rho[5 * la + lb] + c_mat[5 * la + lb])
    secs = t2 - t0
    job_sphere = info["flops_rho_sphere"] + info["flops_mat_sphere"]
    frac = flops / (2.0 * job_sphere)
    return {"value": round(frac * job_work / secs / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"oracle eval_rho+eval_mat over the ordered pair images whose first primitive sits on the "
                      f"first {n} of {system.natm} atoms: {flops:.3e} in-sphere flops in {secs:.1f} s, "
                      f"{100 * frac:.2f}% of the job",
            "oracle_gflops": round(flops / secs / 1e9, 3), "seconds": round(secs, 2),
            "cpu": cpu_model(), "small_configs": cpu_small_configs()}


def fp32_errors():
    """FP32 pipeline (rho, Poisson, J, gradient) against the FP64 kernels on the
    diamond configuration (216 C, 5 levels, 600 Ry)."""
    import torch
    from paper_2603_24881_amd import synth
    from paper_2603_24881_amd.gpw import GPW
    s = synth.config4()
    dev = torch.device("cuda", 0)
    D = torch.as_tensor(synth.make_density(s), device=dev)
    res = {}
    for prec in ("fp64", "fp32"):
        g = GPW(s, precision=prec)
        v, e = g.poisson().solve(g.rho(D))
        res[prec] = (e, g.mat(v), g.grad(D, v))
        torch.cuda.synchronize()
        g.close()
    (e64, J64, F64), (e32, J32, F32) = res["fp64"], res["fp32"]
    return {"system": "diamond 216 C, 3024 AOs, 5 levels", "vs": "FP64 kernels",
            "E_J": e64, "E_J_abs_err": abs(e32 - e64), "E_J_rel_err": abs(e32 - e64) / abs(e64),
            "J_max_abs_err": float((J32 - J64).abs().max()), "J_rel_err": float((J32 - J64).abs().max() / J64.abs().max()),
            "grad_max_abs_err": float((F32 - F64).abs().max()),
            "grad_rel_err": float((F32 - F64).abs().max() / F64.abs().max())}


def serving(n, rates, budget_gb):
    """Poisson arrivals of mixed Fock / gradient requests on water-like
    clusters of 8..256 units (two geometries each): continuous batching vs
    one-at-a-time plain calls on the same trace and resident plans, per
    arrival rate."""
    from paper_2603_24881_amd import synth
    from paper_2603_24881_amd.serve import GPUExecutor, Scheduler, poisson_trace, summarize, system_key
    sizes = (8, 16, 32, 64, 128, 256)
    ex = GPUExecutor()
    t0 = time.perf_counter()
    for nw in sizes:
        for geo in range(2):
            ex.register(system_key(nw, geo), synth.config5(nw, geo))
    reg = time.perf_counter() - t0
    log(f"[bench] serving: 12 plans registered in {reg:.1f} s")
    out = {"requests": n, "sizes_waters": list(sizes), "geometries": 2, "grad_fraction": 0.5,
           "budget_gb": budget_gb, "max_active": 32, "max_batch": 16, "lanes": ex.n_lanes, "heavy_alone": True,
           "plan_register_s": round(reg, 2), "runs": []}
    warm = poisson_trace(24, 1000.0, seed=1999)
    Scheduler(ex, budget_gb * 2 ** 30).run(warm)
    for rate in rates:
        run = {"rate_per_s": rate}
        for mode in ("continuous", "sequential"):
            trace = poisson_trace(n, rate, seed=2000)
            sch = Scheduler(ex, budget_gb * 2 ** 30)
            (sch.run if mode == "continuous" else sch.run_sequential)(trace)
            sm = summarize(trace)
            if mode == "continuous":
                sm["rounds"] = len(sch.rounds)
                sm["mean_requests_per_round"] = float(np.mean(sch.rounds))
            run[mode] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in sm.items()}
            log(f"[bench] serving {rate:g}/s {mode}: {run[mode]}")
        out["runs"].append(run)
    return out


# ---------------------------------------------------------------- profile summaries
#
# The rocprofv3 runs behind profiles/ (each its own process, from /tmp with
# TMPDIR=/tmp, <repo> the repository root, <out> = DIR/<name>):
#   stats:     rocprofv3 --kernel-trace --stats --output-format csv -d <out> -o run -- python3 <repo>/bench.py
#                --steps 3 --warmup 1 --extras 0 --serve-requests 0 --no-cpu-baseline   (stderr to DIR/bench.err)
#   stats_x:   the same without --extras 0 (gradient and meta-GGA terms)
#   f64:       rocprofv3 --pmc SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64
#                SQ_INSTS_VALU_TRANS_F64 SQ_INSTS_VALU SQ_BUSY_CU_CYCLES GRBM_GUI_ACTIVE --output-format csv
#                -d <out> -o run -- python3 <repo>/bench.py --steps 1 --warmup 0 --extras 0 --serve-requests 0
#                --no-cpu-baseline
#   fetch, write: rocprofv3 --pmc FETCH_SIZE (WRITE_SIZE) ... the stats command's bench.py arguments
#   cal_fetch, cal_write: the same two counters on python3 <repo>/bench.py --calibrate-copy
#   sq1:       rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_ACTIVE_INST_VALU SQ_BUSY_CYCLES ... (stats arguments)
#   sq2:       rocprofv3 --pmc SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_BUSY_CU_CYCLES ... (stats arguments)

CLASS_NAMES = ["ss", "ps", "pp", "ds", "dp", "dd", "fs", "fp", "fd", "ff", "gs", "gp", "gd", "gf", "gg"]


def _rows(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _short(name):
    import re
    n = re.sub(r"\(.*", "", name).replace("void ", "")
    return n if len(n) <= 60 else n[:40] + "... (library GEMM)" if n.startswith("Cijk") else n[:57] + "..."


def _class_kernel(name):
    """(operation, class index) of an FP64 class kernel, else None."""
    import re
    m = re.match(r"gpw::k_(rho2?|mat|grad|tau|mat_tau|grad_tau)<(\d), (\d)[,>]", name)
    if not m or "double" not in name or "true>" in name:
        return None
    la, lb = int(m.group(2)), int(m.group(3))
    op = {"rho2": "rho"}.get(m.group(1), m.group(1))
    return op, la * (la + 1) // 2 + lb


def _counters(path):
    """Per kernel: counter sums over its dispatches, the dispatch count and the
    summed dispatch durations (ns)."""
    import collections
    disp, meta = collections.defaultdict(dict), {}
    for r in _rows(path):
        d = int(r["Dispatch_Id"])
        disp[d][r["Counter_Name"]] = disp[d].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        meta[d] = (_short(r["Kernel_Name"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for d, c in disp.items():
        k, dur = meta[d]
        per[k]["_n"] += 1
        per[k]["_ns"] += dur
        for n, v in c.items():
            per[k][n] += v
    return per


def _trace(path):
    import collections
    tr = collections.defaultdict(list)
    for r in _rows(path):
        tr[_short(r["Kernel_Name"])].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return tr


def _flop_model(op, c, inc):
    """The plan's kernel flop model of one class (per evaluation), as in the partitioner."""
    la = next(l for l in range(5) if (l + 1) * (l + 2) // 2 > c)
    lb = c - la * (la + 1) // 2
    L = la + lb
    na, nb = (la + 1) * (la + 2) // 2, (lb + 1) * (lb + 2) // 2
    f1 = 2 * na * nb + 2 * (na + nb) + 4
    tensor_rho = la == 2 or la == 3 or (la == 4 and lb >= 1)
    ft = 8 * (L + 2) * (L + 1) * L / 6 + 32 * (L + 1) * L / 2 + 16 + 64 * (2 * L + 3)
    if op == "rho":
        return (ft if tensor_rho else 64 * f1) * inc, 64 * f1 * inc
    return 64 * ((2 * L + 3) if L >= 2 else f1) * inc, 64 * f1 * inc


def summarize_profiles(d, prof=None):
    """Write the *water256* summaries into prof (default profiles/) from the
    rocprofv3 outputs under d (layout above)."""
    import re
    import statistics
    prof = prof or os.path.join(ROOT, "profiles")
    inc = None
    for line in open(os.path.join(d, "bench.err")):
        if "[bench] per class:" in line:
            inc = [int(x) for x in re.findall(r"/ (\d+) blocks", line)]
    assert inc and len(inc) == 15, "bench.err lacks the per-class line"
    sha = _sources_sha()
    stats = _rows(os.path.join(d, "stats", "run_kernel_stats.csv"))
    tr = _trace(os.path.join(d, "stats", "run_kernel_trace.csv"))
    NEV = 6     # evaluations of eval_rho and of eval_mat in the stats command
    hdr = ("Command (from the repository root on one MI355X, `<repo>` its absolute path; `cd /tmp && export "
           "TMPDIR=/tmp` first):\n\n```\n")
    cmd_stats = ("rocprofv3 --kernel-trace --stats --output-format csv -d <out> -o run -- python3 <repo>/bench.py "
                 "--steps 3 --warmup 1 --extras 0 --serve-requests 0 --no-cpu-baseline")
    # ---- kernel stats of eval_rho / eval_mat
    lines, tot = [], {"rho": 0.0, "mat": 0.0}
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        k = _short(r["Name"])
        ck = _class_kernel(k)
        calls, total = int(r["Calls"]), float(r["TotalDurationNs"]) * 1e-6
        extra = ""
        if ck and ck[0] in ("rho", "mat"):
            model, conv = _flop_model(ck[0], ck[1], inc[ck[1]])
            t = total / NEV * 1e-3
            tot[ck[0]] += t
            extra = (f" {CLASS_NAMES[ck[1]]} | {inc[ck[1]]} | {t * 1e3:.3f} | {conv / t / 1e12:.2f} | "
                     f"{model / t / 1e12:.2f} | {model / t / PEAK_FP64:.3f} |")
        else:
            extra = " | | | | | |"
        if total < 0.05 and not ck:
            continue
        lines.append(f"| `{k}` | {calls} | {total:.3f} | {float(r['AverageNs']) * 1e-3:.1f} |{extra}")
    txt = ("# Kernel times of eval_rho / eval_mat, 256-water-like system (768 atoms, 10496 AOs, 4 levels, "
           "tau 1e-6), FP64\n\n" + hdr + cmd_stats + "\n```\n\n"
           f"`rocprofv3 --kernel-trace --stats` totals (`run_kernel_stats.csv`); the run evaluates eval_rho and "
           f"eval_mat {NEV} times each (1 warm-up + 3 steps + 2 + 2 timed single-op repeats), one launch per "
           "(operation, class) per evaluation.  conv = the counting convention F = 2 n_a n_b + 2 (n_a + n_b) + 4 "
           "per point of every visited 4^3 block; model = the plan's kernel flop model (the arithmetic of the "
           "form each class uses); frac = model rate / 78.6 TFLOP/s.\n\n"
           "| kernel | calls | total ms | avg us | class | incidences | ms / eval | conv TF/s | model TF/s | "
           "model frac |\n|---|---:|---:|---:|---|---:|---:|---:|---:|---:|\n" + "\n".join(lines) +
           f"\n\nPer evaluation, class kernels only: eval_rho {tot['rho'] * 1e3:.3f} ms, eval_mat "
           f"{tot['mat'] * 1e3:.3f} ms (bench.py's `ms_rho` / `ms_mat` add the packing, fills and block copies).\n"
           f"\nsource_sha256 {sha}\n")
    open(os.path.join(prof, "k_rho_k_mat_water256_kernel_stats.md"), "w").write(txt)
    # ---- gradient and meta-GGA kernels (the 256-water launches: the longest of each)
    trx = _trace(os.path.join(d, "stats_x", "run_kernel_trace.csv"))
    lines, tot2 = [], {}
    for k in sorted(trx):
        ck = _class_kernel(k)
        if not ck or ck[0] not in ("grad", "tau", "mat_tau", "grad_tau"):
            continue
        durs = sorted(trx[k])[-3:]
        t = statistics.median(durs) * 1e-6
        tot2[ck[0]] = tot2.get(ck[0], 0.0) + t
        lines.append(f"| `{k}` | {ck[0]} | {CLASS_NAMES[ck[1]]} | {len(trx[k])} | {t:.3f} |")
    txt = ("# Kernel times of eval_grad and the meta-GGA terms, 256-water-like system, FP64\n\n" + hdr +
           cmd_stats.replace(" --extras 0", "") + "\n```\n\n"
           "From `run_kernel_trace.csv`: the 256-water gradient and meta-GGA terms are evaluated 3 times each; "
           "the FP32 error report also evaluates the smaller diamond system with the FP64 kernels (shorter "
           "launches), so each row is the median of the 3 longest launches.\n\n"
           "| kernel | operation | class | launches | ms / eval |\n|---|---|---|---:|---:|\n" + "\n".join(lines) +
           "\n\nPer evaluation: " + ", ".join(f"{op} {t:.3f} ms" for op, t in sorted(tot2.items())) +
           f"\n\nsource_sha256 {sha}\n")
    open(os.path.join(prof, "k_grad_k_tau_water256_kernel_stats.md"), "w").write(txt)
    # ---- FP64 counters
    per = _counters(os.path.join(d, "f64", "run_counter_collection.csv"))
    lines, tot = [], {"rho": [0.0, 0.0, 0.0], "mat": [0.0, 0.0, 0.0]}
    for k in sorted(per, key=lambda k: (_class_kernel(k) or ("z", 0))):
        ck = _class_kernel(k)
        if not ck or ck[0] not in ("rho", "mat"):
            continue
        op, c = ck
        p = per[k]
        n = p["_n"]
        model, conv = _flop_model(op, c, inc[c])
        cnt = (2 * p["SQ_INSTS_VALU_FMA_F64"] + p["SQ_INSTS_VALU_ADD_F64"] + p["SQ_INSTS_VALU_MUL_F64"]) * 64 / n
        t = statistics.median(sorted(tr[k])) * 1e-9
        clk = p["GRBM_GUI_ACTIVE"] / 8 / (p["_ns"] * 1e-9) / 1e9
        valu = p["SQ_INSTS_VALU"] / n
        tot[op][0] += t
        tot[op][1] += model
        tot[op][2] += cnt
        lines.append(f"| `{k}` | {CLASS_NAMES[c]} | {inc[c]} | {t * 1e3:.3f} | {conv / t / 1e12:.2f} | "
                     f"{model / t / 1e12:.2f} | {model / t / PEAK_FP64:.3f} | {cnt / t / 1e12:.2f} | "
                     f"**{cnt / t / PEAK_FP64:.3f}** | {cnt / model:.2f} | {valu / (256 * t * 2.4e9):.2f} | {clk:.2f} |")
    txt = ("# FP64 work of k_rho / k_mat per (l_a, l_b) class, 256-water-like system (768 atoms, 10496 AOs, 4 "
           "levels, tau 1e-6), FP64\n\nCommands (from the repository root on one MI355X, `<repo>` its absolute "
           "path; `cd /tmp && export TMPDIR=/tmp` first), each in its own run:\n\n```\n"
           "rocprofv3 --pmc SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_TRANS_F64 "
           "SQ_INSTS_VALU SQ_BUSY_CU_CYCLES GRBM_GUI_ACTIVE --output-format csv -d <out> -o run -- python3 "
           "<repo>/bench.py --steps 1 --warmup 0 --extras 0 --serve-requests 0 --no-cpu-baseline\n" + cmd_stats +
           "\n```\n\nThe counter run evaluates eval_rho and eval_mat 3 times each; counts below are per "
           "evaluation.  Durations: median launch of each kernel in the kernel-trace run (no counters attached).\n"
           "* conv: the counting convention F = 2 n_a n_b + 2 (n_a + n_b) + 4 per point of every visited 4^3 block "
           "(the direct evaluation; the factorised classes do less, so it can exceed the peak).\n"
           "* model: the plan's kernel flop model (`flops_rho_exec`, `flops_mat_exec`).\n"
           "* counters: (2 FMA_F64 + ADD_F64 + MUL_F64) x 64 lanes, the FP64 arithmetic the kernel executes (exp "
           "and address arithmetic in FP64 included; TRANS_F64 is 0: FP64 exp is FMA code).\n"
           "* frac = rate / 78.6 TFLOP/s (MI355X FP64 vector peak at 2.4 GHz); VALU/CU-cyc = SQ_INSTS_VALU wave "
           "instructions per CU and 2.4 GHz cycle of the kernel's duration (one FP64 VALU instruction per CU-cycle "
           "at most); clock = GRBM_GUI_ACTIVE / 8 XCDs / duration in the counter run (GHz).\n\n"
           "| kernel | class | incidences | ms / eval | conv TF/s | model TF/s | model frac | counter TF/s | "
           "counter frac | counter/model | VALU/CU-cyc | clock |\n"
           "|---|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|\n" + "\n".join(lines) +
           f"\n\nPer evaluation: eval_rho kernels {tot['rho'][0] * 1e3:.3f} ms, model {tot['rho'][1]:.4e} flops "
           f"({tot['rho'][1] / tot['rho'][0] / PEAK_FP64:.3f} of peak), counters {tot['rho'][2]:.4e} flops "
           f"({tot['rho'][2] / tot['rho'][0] / PEAK_FP64:.3f} of peak); eval_mat kernels {tot['mat'][0] * 1e3:.3f} "
           f"ms, model {tot['mat'][1]:.4e} ({tot['mat'][1] / tot['mat'][0] / PEAK_FP64:.3f}), counters "
           f"{tot['mat'][2]:.4e} ({tot['mat'][2] / tot['mat'][0] / PEAK_FP64:.3f}).\n\n"
           "bench.py reads the two lines below (FP64 flops per evaluation from the counters) while the kernel "
           "sources hash to `source_sha256`, and reports `value` and `roofline` from them; otherwise it falls back "
           "to the plan's model.\n\n```\n"
           f"eval_rho_flops {tot['rho'][2]:.6e}\neval_mat_flops {tot['mat'][2]:.6e}\nsource_sha256 {sha}\n```\n")
    open(os.path.join(prof, "k_rho_k_mat_water256_fp64_counters.md"), "w").write(txt)
    # ---- HBM traffic
    def counter_sum(sub, name):
        per = _counters(os.path.join(d, sub, "run_counter_collection.csv"))
        return {k: p[name] for k, p in per.items()}
    cf, cw = counter_sum("cal_fetch", "FETCH_SIZE"), counter_sum("cal_write", "WRITE_SIZE")
    copy = max(cf, key=cf.get)      # the copy kernel (the fill before it reads nothing)
    moved = 1 << 20     # KiB: one 1 GiB copy
    sf, sw = moved / cf[copy], moved / cw[copy]
    fe, wr = counter_sum("fetch", "FETCH_SIZE"), counter_sum("write", "WRITE_SIZE")
    ops = {"eval_rho": lambda k: re.match(r"gpw::k_(rho2?<|pack_)", k) is not None,
           "eval_mat": lambda k: re.match(r"gpw::k_(mat<|block_grid)", k) is not None}
    out = [f"# HBM traffic of eval_rho and eval_mat, 256-water-like system, FP64",
           "#", "# Commands (from the repository root on one MI355X, <repo> its absolute path; cd /tmp && export "
           "TMPDIR=/tmp first), each its own run:",
           "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out> -o run -- python3 <repo>/bench.py --steps 3 "
           "--warmup 1 --extras 0 --serve-requests 0 --no-cpu-baseline",
           "#   rocprofv3 --pmc WRITE_SIZE (the same)",
           "#   calibration: the same two counters on `python3 <repo>/bench.py --calibrate-copy` (one 1 GiB "
           "device-to-device copy)",
           f"#   copy ({copy}): FETCH_SIZE {cf[copy]:.0f} KiB, WRITE_SIZE {cw[copy]:.0f} KiB for {moved} KiB "
           f"moved -> scale FETCH by {sf:.4f}, WRITE by {sw:.4f}",
           f"# Per evaluation = counter sums over the operation's kernels / {NEV} evaluations, scaled, in bytes:",
           "# eval_rho = the packing and density kernels, eval_mat = the block copies of the potentials and the",
           "# integration kernels; the zero fills of the outputs (k_fill: the rho grids, 70 MB, and M, 0.88 GB,",
           "# written per evaluation) are shared by both operations and left out.",
           "# bench.py reports `traffic` only while the kernel sources hash to source_sha256.",
           f"source_sha256 {sha}"]
    for op, sel in ops.items():
        f = sum(v for k, v in fe.items() if sel(k)) * sf * 1024 / NEV
        w = sum(v for k, v in wr.items() if sel(k)) * sw * 1024 / NEV
        out += [f"{op}_fetch_bytes {f:.0f}", f"{op}_write_bytes {w:.0f}", f"{op}_bytes {f + w:.0f}"]
    out.append("# per kernel (GB per evaluation, fetch / write):")
    for k in sorted(fe, key=lambda k: -fe[k]):
        if fe[k] * sf * 1024 / NEV < 1e6:
            continue
        out.append(f"#   {k:45s} {fe[k] * sf * 1024 / NEV / 1e9:7.3f} / {wr.get(k, 0.0) * sw * 1024 / NEV / 1e9:7.3f}")
    open(os.path.join(prof, "eval_rho_eval_mat_water256_hbm_traffic.txt"), "w").write("\n".join(out) + "\n")
    # ---- SQ issue counters
    p1 = _counters(os.path.join(d, "sq1", "run_counter_collection.csv"))
    p2 = _counters(os.path.join(d, "sq2", "run_counter_collection.csv"))
    lines = []
    for k in sorted(p1, key=lambda k: -p1[k].get("SQ_INSTS_VALU", 0.0)):
        ck = _class_kernel(k)
        if not ck or ck[0] not in ("rho", "mat") or k not in p2:
            continue
        a, b = p1[k], p2[k]
        v = a["SQ_INSTS_VALU"]
        lines.append(f"| `{k}` | {v / a['_n']:.3g} | {v / b['SQ_BUSY_CU_CYCLES']:.2f} | "
                     f"{a['SQ_INSTS_SALU'] / v:.2f} | {b['SQ_INSTS_LDS'] / v:.2f} | {b['SQ_INSTS_VMEM_RD'] / v:.3f} |")
    txt = ("# SQ issue counters of the k_rho / k_mat kernels, 256-water-like system, FP64\n\nCommands (as for the "
           "kernel stats, `cd /tmp && export TMPDIR=/tmp` first), each its own run:\n\n```\n"
           "rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_ACTIVE_INST_VALU SQ_BUSY_CYCLES --output-format csv -d <out> "
           "-o run -- python3 <repo>/bench.py --steps 3 --warmup 1 --extras 0 --serve-requests 0 --no-cpu-baseline\n"
           "rocprofv3 --pmc SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_BUSY_CU_CYCLES --output-format csv -d <out> -o run -- "
           "python3 <repo>/bench.py --steps 3 --warmup 1 --extras 0 --serve-requests 0 --no-cpu-baseline\n```\n\n"
           "VALU per evaluation (wave64 instructions); VALU / CU-cycle = SQ_INSTS_VALU / SQ_BUSY_CU_CYCLES (at most 1 "
           "for FP64: a wave64 FP64 instruction occupies one of the CU's 4 SIMDs for 4 cycles); SALU, LDS, VMEM per "
           "VALU instruction.\n\n"
           "| kernel | VALU / eval | VALU / CU-cycle | SALU / VALU | LDS / VALU | VMEM / VALU |\n"
           "|---|---:|---:|---:|---:|---:|\n" + "\n".join(lines) + f"\n\nsource_sha256 {sha}\n")
    open(os.path.join(prof, "k_rho_k_mat_water256_sq_counters.md"), "w").write(txt)
    print("profiles written", file=sys.stderr)


def main():
    args = parse()
    if args.summarize:
        summarize_profiles(args.summarize)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus above 1 is not supported (the path would shard by "
                                   "grid blocks, with one all-reduce of M per evaluation)"}))
        sys.exit(2)
    import torch
    from paper_2603_24881_amd import synth
    from paper_2603_24881_amd.gpw import GPW

    dev = torch.device("cuda", 0)
    if args.calibrate_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30}), flush=True)
        return
    system, desc = make_system(args.workload)
    log(f"[bench] {desc}")
    t0 = time.perf_counter()
    g = GPW(system)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = g.info
    log(f"[bench] plan {plan_s:.2f} s, pairs {sum(info['n_pairs'])}, incidences {sum(info['n_incidences'])}, "
        f"mesh {info['mesh']}, device bytes {info['device_bytes'] / 1e9:.2f} GB")
    names = ["ss", "ps", "pp", "ds", "dp", "dd", "fs", "fp", "fd", "ff", "gs", "gp", "gd", "gf", "gg"]
    log("[bench] per class: " + ", ".join(f"{n}: {p} pairs / {i} blocks" for n, p, i in
                                          zip(names, info["n_pairs_class"], info["n_incidences_class"])))
    C = synth.draw_orbitals(system)
    Cd = torch.as_tensor(C, device=dev)
    D = (Cd @ Cd.T).contiguous()
    del Cd
    V_np = synth.make_potentials(info["mesh"], system.seed)
    V = [torch.as_tensor(v, device=dev).contiguous() for v in V_np]
    rho = g.new_grids()
    M = torch.empty((g.n_ao, g.n_ao), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        g.rho(D, out=rho)
        g.mat(V, out=M)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_step = timed(step, args.steps, stream)
    t_rho = timed(lambda: g.rho(D, out=rho), max(2, args.steps // 2), stream)
    t_mat = timed(lambda: g.mat(V, out=M), max(2, args.steps // 2), stream)
    f_rho_s, f_mat_s = info["flops_rho_sphere"], info["flops_mat_sphere"]
    f_rho_b, f_mat_b = info["flops_rho_block"], info["flops_mat_block"]
    # the work of one evaluation: the FP64 arithmetic the kernels execute, from the
    # committed counter summary of this system while it matches the sources, else
    # the plan's kernel flop model
    cf = counter_flops() if args.workload == "water256" else None
    if cf is not None:
        f_rho_x, f_mat_x = cf["eval_rho"], cf["eval_mat"]
        work = "FP64 VALU instructions executed, (2 FMA + ADD + MUL) x 64 lanes (rocprofv3 counters, " \
               "profiles/k_rho_k_mat_water256_fp64_counters.md)"
    else:
        f_rho_x, f_mat_x = info["flops_rho_exec"], info["flops_mat_exec"]
        work = "the plan's kernel flop model (flops_rho_exec, flops_mat_exec)"
    value = (f_rho_x + f_mat_x) / t_step / 1e9
    conv = (f_rho_b + f_mat_b) / t_step / 1e9
    log(f"[bench] step {t_step * 1e3:.2f} ms (rho {t_rho * 1e3:.2f} ms, mat {t_mat * 1e3:.2f} ms), "
        f"{value:.0f} GFLOP/s executed, {conv:.0f} GFLOP/s by the block convention, "
        f"{(f_rho_s + f_mat_s) / t_step / 1e9:.0f} GFLOP/s in-sphere convention")
    if t_rho >= t_mat:
        dom, dt, fl, op = "k_rho (density collocation, all classes and levels of one eval_rho)", t_rho, f_rho_x, "eval_rho"
    else:
        dom, dt, fl, op = "k_mat (potential integration, all classes and levels of one eval_mat)", t_mat, f_mat_x, "eval_mat"
    traffic = measured_traffic(op) if args.workload == "water256" else None
    out = {
        "metric": "eval_rho+eval_mat FP64 GFLOP/s & %peak; served requests/s + p50/p99 latency",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "tau": system.tau, "levels_ry": system.ke_cutoff_ry,
                   "mesh": info["mesh"], "rel_cutoff_ry": system.rel_cutoff_ry},
        "roofline": {"bound": "alu", "kernel": dom, "work": work,
                     "achieved": round(fl / dt / 1e12, 3), "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                     "frac": round(fl / dt / PEAK_FP64, 4), "traffic": traffic},
        "pct_fp64_peak": round(100 * value * 1e9 / PEAK_FP64, 2),
        "ms_rho": round(t_rho * 1e3, 4),
        "ms_mat": round(t_mat * 1e3, 4),
        "rho_gflops": round(f_rho_x / t_rho / 1e9, 2),
        "mat_gflops": round(f_mat_x / t_mat / 1e9, 2),
        "model_gflops": round((info["flops_rho_exec"] + info["flops_mat_exec"]) / t_step / 1e9, 2),
        "convention_gflops": round(conv, 2),
        "pct_fp64_peak_convention": round(100 * conv * 1e9 / PEAK_FP64, 2),
        "useful_gflops": round((f_rho_s + f_mat_s) / t_step / 1e9, 2),
        "pct_fp64_peak_useful": round(100 * (f_rho_s + f_mat_s) / t_step / PEAK_FP64, 2),
        "max_box_width": info["max_box_width"],
        "plan_s": round(plan_s, 3),
        "n_pair_images": int(sum(info["n_pairs"])),
        "n_block_incidences": int(sum(info["n_incidences"])),
    }
    if args.extras:
        G = torch.empty((g.natm, 3), dtype=torch.float64, device=dev)
        g.grad(D, V, out=G)
        t_grad = timed(lambda: g.grad(D, V, out=G), max(2, args.steps // 2), stream)
        out["ms_grad"] = round(t_grad * 1e3, 4)
        out["grad_gflops"] = round(info["flops_grad_exec"] / t_grad / 1e9, 2)
        out["grad_convention_gflops"] = round(info["flops_grad_block"] / t_grad / 1e9, 2)
        log(f"[bench] grad {t_grad * 1e3:.2f} ms")
        # meta-GGA kinetic-energy-density terms on the same plan
        T = g.new_grids()
        g.tau(D, out=T)
        g.mat_tau(V, out=M)
        g.grad_tau(D, V, out=G)
        reps = max(2, args.steps // 4)
        t_tau = timed(lambda: g.tau(D, out=T), reps, stream)
        t_mtau = timed(lambda: g.mat_tau(V, out=M), reps, stream)
        t_gtau = timed(lambda: g.grad_tau(D, V, out=G), reps, stream)
        out["meta_gga"] = {
            "ms_tau": round(t_tau * 1e3, 4), "ms_mat_tau": round(t_mtau * 1e3, 4),
            "ms_grad_tau": round(t_gtau * 1e3, 4),
            "tau_gflops": round(info["flops_tau_exec"] / t_tau / 1e9, 2),
            "mat_tau_gflops": round(info["flops_mat_tau_exec"] / t_mtau / 1e9, 2),
            "grad_tau_gflops": round(info["flops_grad_tau_exec"] / t_gtau / 1e9, 2),
            "frac_tau": round(info["flops_tau_exec"] / t_tau / PEAK_FP64, 4),
        }
        log(f"[bench] meta-GGA: {out['meta_gga']}")
        del T
        g32 = GPW(system, precision="fp32")
        rho32 = g32.new_grids()
        M32 = torch.empty_like(M)
        g32.rho(D, out=rho32)
        g32.mat(V, out=M32)
        t32 = timed(lambda: (g32.rho(D, out=rho32), g32.mat(V, out=M32)), max(2, args.steps // 2), stream)
        out["ms_step_fp32"] = round(t32 * 1e3, 4)
        # the FP32 kernels against the FP64 ones on this system (rho per level, M)
        g.rho(D, out=rho)
        g.mat(V, out=M)
        torch.cuda.synchronize()
        out["fp32_vs_fp64_here"] = {
            "rho_rel_err": max(float((a - b).abs().max() / b.abs().max()) for a, b in zip(rho32, rho)),
            "M_rel_err": float((M32 - M).abs().max() / M.abs().max())}
        log(f"[bench] fp32 step {t32 * 1e3:.2f} ms, errors {out['fp32_vs_fp64_here']}")
        del rho32, M32
        g32.close()
    if args.extras:
        out["fp32_error"] = fp32_errors()
        log(f"[bench] fp32 errors: {out['fp32_error']}")
    Dn = None if args.no_cpu_baseline else D.cpu().numpy()
    if args.serve_requests > 0:
        del rho, M, V, D
        torch.cuda.empty_cache()
        out["serving"] = serving(args.serve_requests, [float(x) for x in args.serve_rates.split(",")],
                                 args.serve_budget_gb)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle sample)...")
        out["cpu_baseline"] = cpu_baseline(system, Dn, V_np, args.cpu_atoms, info, f_rho_x + f_mat_x)
        log(f"[bench] cpu {out['cpu_baseline']['value']:.2f} GFLOP/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
