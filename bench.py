"""Benchmark of per-element local assembly on one MI355X.

Headline workload (one step = one pass over it): the Helmholtz form
(grad u . grad v + u v) on 750,000 jittered tetrahedra (50^3 cubes x 6 Kuhn
tetrahedra), scalar Lagrange P1, P2, P3 and P4, float64 -- four launches per
step.  value = element matrices per second over the timed steps.

Also measured (fields "workloads"): P1 triangle mass on 4,096 elements,
vector P2 elasticity on 1,971,054 tetrahedra (float64 and the split-precision
MFMA variants), the neo-Hookean tangent on 998,250 tetrahedra (P1, P2; float64
and split), a 16-sub-batch mixed persistent launch replayed from a HIP
graph (one persistent work-queue kernel per kernel variant), and the
experiment matrix of Sec. 7.1 (mass and Helmholtz, q = 1..4, nf = 0..3
coefficient functions) with Algorithm 3's choice against both forced modes,
local plus global assembly (insertion into the compressed-row matrix of
the continuous space) of the headline form and mesh, Helmholtz on
non-affine (z-jittered) prisms with per-point geometry, and a full-tensor
diffusion form through automatically sharing-eliminated generated kernels.
Inputs are seeded
synthetic meshes resident in HBM before timing.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
       python bench.py summarize-trace DB_DIR OUT.md TITLE COMMAND [NAME_FILTER [LABELS]]
       python bench.py summarize-traffic FETCH_DIR WRITE_DIR OUT.md TITLE CMD_FETCH CMD_WRITE
(the last two turn rocprofv3 output into the text summaries under profiles/).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_preeval_stream_helmholtz_tet_p4_750k.traffic.md")
# the device code of the pre-evaluated kernels (every function they run is
# defined in these files): a profile of their HBM traffic is only reported
# while these are unchanged
PREEVAL_SOURCES = ["paper_1604_05872_amd/csrc/fe_common.hpp", "paper_1604_05872_amd/csrc/device_common.hpp",
                   "paper_1604_05872_amd/csrc/preeval.hpp", "paper_1604_05872_amd/csrc/assemble_preeval.hip"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# Algorithmic work per element (flop-reduced formulation; compulsory bytes)
# ---------------------------------------------------------------------------

def n_scalar(cell, p):
    return {"triangle": (p + 1) * (p + 2) // 2, "tetrahedron": (p + 1) * (p + 2) * (p + 3) // 6,
            "prism": (p + 1) * (p + 2) // 2 * (p + 1)}[cell]


GD = {"triangle": 2, "tetrahedron": 3, "prism": 3}
NV = {"triangle": 3, "tetrahedron": 4, "prism": 6}


def rule_size(cell, qdeg):
    m = max(1, (qdeg + 2) // 2)
    tri = 3 if qdeg <= 2 else m * m
    return {"triangle": tri, "tetrahedron": m ** 3, "prism": tri * m}[cell]


def default_qdeg(form, cell, p):
    if form in ("mass", "helmholtz"):
        return 2 * p
    if form == "elasticity":
        return 2 * p + 1 if cell == "prism" else 2 * p - 1
    return 4


def alg_bytes(form, cell, p):
    d, ns = GD[cell], n_scalar(cell, p)
    n = d * ns if form in ("elasticity", "hyperelastic") else ns
    coeff = {"mass": 0, "helmholtz": 0, "elasticity": 2 * NV[cell], "hyperelastic": d * ns}[form]
    return 8 * (NV[cell] * d + coeff + n * n)


def alg_flops(form, cell, p, collapsed=True, preeval=False):
    """Operation count of the flop-reduced evaluation (counting + and * once);
    preeval: elasticity in the pre-evaluated mode (one multiply-add per table
    term and entry, rho iota = n_c d^2 terms per entry of the d^2 blocks)."""
    d, ns = GD[cell], n_scalar(cell, p)
    geo = 24 if d == 2 else 87
    if form == "elasticity" and preeval:
        return 2 * NV[cell] * d * d * ns * ns * d * d + geo
    if form == "mass":
        return ns * ns + geo
    if form == "helmholtz":
        return (2 * (1 + d * (d + 1) // 2) - 1) * ns * ns + geo
    nq = rule_size(cell, default_qdeg(form, cell, p))
    nqi = 1 if (collapsed and p == 1 and cell != "prism") else nq   # q-invariant P1 gradients
    inner = nqi * ns * ns * (4 * d * d + 3 * d)
    if form == "hyperelastic" and nqi > 1:
        # the plan pre-evaluates the trace monomial mu |det J| g_j . g_k:
        # rho = d(d+1)/2 tables per pair, then d diagonal-block additions
        inner = nqi * ns * ns * 4 * d * d + ns * ns * (d * (d + 1) + d)
    if form == "elasticity":
        return inner + nq * (ns * d * (2 * d - 1) + 4 * NV[cell] + 4) + geo
    return inner + nq * (2 * ns * d * (2 * d - 1) + 2 * d * d * ns + 60) + geo


# ---------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="time the built-in default launch shapes instead of the autotuned ones")
    ap.add_argument("--only-headline", action="store_true")
    ap.add_argument("--no-headline", action="store_true",
                    help="time only the --workloads (for profiler runs); prints their rows as one JSON line")
    ap.add_argument("--workloads", default="mass,elasticity,hyperelastic,batch,sweep,global,nonaffine,forms",
                    help="comma list of the extra workloads to time")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB device-to-device (a known-size kernel for the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); local assembly shards by element "
              f"ranges with no exchange, so run one process per GPU on its own range.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1604_05872_amd import felocal, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    felocal.lib()
    stream = torch.cuda.current_stream()

    def ev():
        return torch.cuda.Event(enable_timing=True)

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        del src, dst

    if args.no_headline:
        rows = other_workloads(torch, felocal, inputs, stream, ev, max(3, args.steps // 2),
                               set(args.workloads.split(",")), autotune=not args.no_autotune)
        print(json.dumps({"workloads": rows}), flush=True)
        return

    # ------------------------------------------------------------------ headline
    log("headline: helmholtz P1-P4 on 750k tets")
    coords_np, V, cells = inputs.tet_workload(50, seed=2)
    E = coords_np.shape[0]
    coords = torch.from_numpy(coords_np).cuda()
    outs = {p: torch.empty((E, n_scalar("tetrahedron", p), n_scalar("tetrahedron", p)), dtype=torch.float64,
                           device="cuda") for p in (1, 2, 3, 4)}
    status = torch.zeros(1, dtype=torch.int32, device="cuda")

    def step(times=None):
        for p in (1, 2, 3, 4):
            if times is not None:
                a, b = ev(), ev()
                a.record(stream)
            felocal.fe_assemble_local("helmholtz", "tetrahedron", p, coords, None, outs[p], status=status)
            if times is not None:
                b.record(stream)
                times[p].append((a, b))

    # untimed: pick each degree's launch shape on this workload (kept by the
    # library for the timed launches)
    tuned = {}
    if not args.no_autotune:
        for p in (1, 2, 3, 4):
            ms_best, shape = felocal.fe_autotune("helmholtz", "tetrahedron", p, coords, None, outs[p],
                                                 return_shape=True)
            tuned[f"P{p}"] = dict(shape, ms=round(ms_best, 4))
            log(f"  autotuned P{p}: {shape} {ms_best:.4f} ms")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    per = {p: [] for p in (1, 2, 3, 4)}
    t0, t1 = ev(), ev()
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    for _ in range(args.steps):
        step(per)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = t0.elapsed_time(t1)
    ms_step = ms_total / args.steps
    value = 4 * E / (ms_step * 1e-3)
    kern_ms = {p: float(np.mean([a.elapsed_time(b) for a, b in per[p]])) for p in per}
    assert int(status.item()) == 0
    per_degree = {}
    for p in (1, 2, 3, 4):
        B = alg_bytes("helmholtz", "tetrahedron", p) * E
        F = alg_flops("helmholtz", "tetrahedron", p) * E
        per_degree[f"P{p}"] = {
            "ms": round(kern_ms[p], 4), "elem_per_s": E / (kern_ms[p] * 1e-3),
            "alg_GBs": B / (kern_ms[p] * 1e-3) / 1e9, "alg_GFLOPs": F / (kern_ms[p] * 1e-3) / 1e9,
            "frac_hbm": B / (kern_ms[p] * 1e-3) / 1e9 / HBM_PEAK_GBS,
        }
    dom = max(kern_ms, key=kern_ms.get)
    dom_bytes = alg_bytes("helmholtz", "tetrahedron", dom) * E
    achieved = dom_bytes / (kern_ms[dom] * 1e-3) / 1e9
    dom_shape = tuned.get(f"P{dom}", {})
    kname = "k_preeval" if dom_shape.get("kernel") == 1 else "k_preeval_stream"
    roofline = {"kernel": f"{kname}<HELMHOLTZ,TET> P{dom}", "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "bytes_per_launch": dom_bytes, "ms_per_launch": round(kern_ms[dom], 4)}
    roofline.update(profiled_traffic(kname, dom_shape))
    # context, after the timed region: a plain fill (torch's fill_) of as many
    # bytes as the dominant launch writes, the practical write ceiling
    nfill = int(E * n_scalar("tetrahedron", dom) ** 2)
    fbuf = torch.empty(nfill, dtype=torch.float64, device="cuda")
    fbuf.fill_(0.0)
    torch.cuda.synchronize()
    fts = []
    for i in range(5):
        fa, fb = ev(), ev()
        fa.record(stream)
        fbuf.fill_(float(i))
        fb.record(stream)
        fts.append((fa, fb))
    torch.cuda.synchronize()
    fill_ms = sorted(fa.elapsed_time(fb) for fa, fb in fts)[2]
    del fbuf
    torch.cuda.empty_cache()
    fill_gbs = nfill * 8 / (fill_ms * 1e-3) / 1e9
    roofline["fill_ceiling"] = {"what": "torch fill_ of the dominant launch's output bytes", "ms": round(fill_ms, 4),
                                "GB/s": round(fill_gbs, 1), "frac_of_fill": round(achieved / fill_gbs, 4)}
    step_bytes = sum(alg_bytes("helmholtz", "tetrahedron", p) for p in (1, 2, 3, 4)) * E
    step_flops = sum(alg_flops("helmholtz", "tetrahedron", p) for p in (1, 2, 3, 4)) * E
    # the last timed step's matrices, kept for the element-by-element check of
    # the CPU-baseline leg: only the first elements (the oracle's sample) go
    # to the host
    headline_out = None
    if not args.no_cpu_baseline:
        headline_out = outs
    else:
        del outs
        torch.cuda.empty_cache()

    result = {
        "metric": "element matrices/s", "value": round(value, 1), "unit": "element matrices/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded jittered Kuhn-tetrahedron mesh)",
        "config": {"workload": "helmholtz_tet_p1-p4", "elements": E, "mesh": "50^3 cubes x 6 tets, +-0.15h jitter",
                   "degrees": [1, 2, 3, 4], "launches_per_step": 4, "quadrature": "exact to degree 2p"},
        "alg_GBs": round(step_bytes / (ms_step * 1e-3) / 1e9, 1),
        "alg_GFLOPs": round(step_flops / (ms_step * 1e-3) / 1e9, 1),
        "wall_s_timed": round(wall, 3),
        "per_degree": per_degree,
        "launch_shapes": tuned or "defaults",
        "roofline": roofline,
    }

    # ------------------------------------------------------------------ other workloads
    if not args.only_headline:
        result["workloads"] = other_workloads(torch, felocal, inputs, stream, ev, max(3, args.steps // 2),
                                             set(args.workloads.split(",")), autotune=not args.no_autotune)

    # ------------------------------------------------------------------ CPU baseline (oracle)
    if not args.no_cpu_baseline:
        result["cpu_baseline"], result["parity"] = cpu_baseline(coords_np, headline_out)
        result["max_err"] = result["parity"]["max_err"]
        del headline_out
    print(json.dumps(result), flush=True)


# ---------------------------------------------------------------------------
# rocprofv3 summaries (profiles/) and the measured HBM traffic
# ---------------------------------------------------------------------------

def sources_sha256(paths=PREEVAL_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read())
    return h.hexdigest()


def profiled_traffic(kname, shape):
    """HBM bytes per launch of the dominant kernel from the committed counter
    profile, when it was taken with the current kernel sources and the same
    launch shape; else traffic stays null."""
    if not os.path.exists(TRAFFIC_PROFILE) or not shape:
        return {}
    rec = None
    with open(TRAFFIC_PROFILE) as f:
        for line in f:
            if line.startswith("<!-- dominant "):
                rec = json.loads(line[len("<!-- dominant "):].rsplit("-->", 1)[0])
    if rec is None or rec.get("sources_sha256") != sources_sha256():
        return {"traffic_note": "counters predate the current kernel sources"}
    if not rec.get("kernel", "").startswith(kname + "<") or rec.get("block") != shape.get("block"):
        return {"traffic_note": "counters were taken with another launch shape"}
    return {"traffic": rec["fetch_bytes"] + rec["write_bytes"], "traffic_fetch": rec["fetch_bytes"],
            "traffic_write": rec["write_bytes"], "traffic_profile": os.path.relpath(TRAFFIC_PROFILE, ROOT)}


def _rocpd(path_dir):
    import glob
    import sqlite3
    dbs = sorted(glob.glob(os.path.join(path_dir, "**", "*_results.db"), recursive=True))
    if not dbs:
        raise SystemExit(f"no rocprofv3 *_results.db under {path_dir}")
    return sqlite3.connect(dbs[0])


def _short(name):
    name = name.replace("void ", "").replace("fe::", "").replace("(anonymous namespace)::", "")
    return name.split("(")[0] if name.startswith("k_") else name[:60]


def summarize_trace(db_dir, out, title, command, only="", labels=""):
    """Per-kernel duration statistics of a --kernel-trace run, one row per
    (kernel, block, grid, LDS); `only` (comma-separated) keeps kernels whose
    name contains one of its parts.  With `labels` (';'-separated) the kept
    dispatches, in launch order, are cut into runs of consecutive dispatches
    of one (kernel, block, grid, LDS), and run i is reported as labels[i]
    (for kernels that share a name, such as run-time generated ones)."""
    cur = _rocpd(db_dir).cursor()
    parts = only.split(",")
    rows = [r for r in cur.execute("select name, workgroup_x, grid_x, lds_size, duration, vgpr_count from kernels "
                                   "order by start").fetchall() if any(f in r[0] for f in parts)]
    agg, regs = {}, {}
    if labels:
        names = labels.split(";")
        runs = []
        for name, wg, grid, lds, dur, vg in rows:
            sig = (_short(name), wg, grid // max(1, wg), lds)
            if not runs or runs[-1][0] != sig:
                runs.append((sig, []))
            runs[-1][1].append(dur)
            regs[sig] = vg
        if len(runs) != len(names):
            raise SystemExit(f"{len(runs)} runs of dispatches but {len(names)} labels")
        for lab, (sig, d) in zip(names, runs):
            agg[(lab,) + sig] = d
    else:
        for name, wg, grid, lds, dur, vg in rows:
            agg.setdefault((_short(name), wg, grid // max(1, wg), lds), []).append(dur)
    total = sum(sum(v) for v in agg.values())
    lines = [f"# {title}", "", "Command (from the repository root on the GPU host):", "", "```", command, "```", "",
             f"{len(rows)} dispatches.  Durations from the kernel trace (ns -> us).", ""]
    if labels:
        lines += ["| case | kernel | block | grid | LDS B | VGPRs | calls | avg us | min us | max us | share |",
                  "|---|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
        for (lab, name, wg, grid, lds), d in agg.items():
            lines.append(f"| {lab} | `{name}` | {wg} | {grid} | {lds} | {regs[(name, wg, grid, lds)]} | {len(d)} | "
                         f"{np.mean(d) / 1e3:.2f} | {min(d) / 1e3:.2f} | {max(d) / 1e3:.2f} | "
                         f"{100 * sum(d) / total:.1f}% |")
    else:
        lines += ["| kernel | block | grid | LDS B | calls | avg us | min us | max us | share |",
                  "|---|---:|---:|---:|---:|---:|---:|---:|---:|"]
        for (name, wg, grid, lds), d in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
            lines.append(f"| `{name}` | {wg} | {grid} | {lds} | {len(d)} | {np.mean(d) / 1e3:.2f} | "
                         f"{min(d) / 1e3:.2f} | {max(d) / 1e3:.2f} | {100 * sum(d) / total:.1f}% |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_traffic(fetch_dir, write_dir, out, title, command_fetch, command_write):
    """FETCH_SIZE / WRITE_SIZE per dispatch (two counter runs), scaled by what
    the same counters read for a 1 GiB device copy (1 GiB read + 1 GiB
    written) in the same runs."""
    def load(d, counter):
        cur = _rocpd(d).cursor()
        q = ("select k.name, k.workgroup_x, k.grid_x, k.lds_size, p.counter_value from pmc_events p join kernels k "
             "on k.dispatch_id = p.dispatch_id where p.counter_name = ?")
        agg = {}
        for name, wg, grid, lds, v in cur.execute(q, (counter,)).fetchall():
            agg.setdefault((name, wg, grid // max(1, wg), lds), []).append(v)
        return agg
    fa, wa = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    copy_f = [v for k, v in fa.items() if "copyBuffer" in k[0]]
    copy_w = [v for k, v in wa.items() if "copyBuffer" in k[0]]
    if not copy_f or not copy_w:
        raise SystemExit("no 1 GiB calibration copy in the counter runs (bench.py --calibrate-copy)")
    gib_kib = float(1 << 20)
    sf, sw = gib_kib / max(copy_f[0]), gib_kib / max(copy_w[0])
    lines = [f"# {title}", "", "Counter runs (from the repository root on the GPU host):", "", "```", command_fetch,
             command_write, "```", "",
             f"Calibration: the 1 GiB device copy reads FETCH_SIZE {max(copy_f[0]):.1f} KiB and WRITE_SIZE "
             f"{max(copy_w[0]):.1f} KiB per dispatch, so HBM bytes = FETCH_SIZE x {sf:.4f} KiB and "
             f"WRITE_SIZE x {sw:.4f} KiB.", "",
             "| kernel | block | grid | LDS B | dispatches | fetch MB/dispatch | write MB/dispatch |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    best = None
    for key in sorted(fa, key=lambda k: -np.mean(wa.get(k, [0]))):
        name, wg, grid, lds = key
        if "fe::" not in name:
            continue
        fb = float(np.mean(fa[key])) * sf * 1024
        wb = float(np.mean(wa.get(key, [0]))) * sw * 1024
        lines.append(f"| `{_short(name)}` | {wg} | {grid} | {lds} | {len(fa[key])} | {fb / 1e6:.1f} | "
                     f"{wb / 1e6:.1f} |")
        if best is None:
            best = {"kernel": _short(name), "block": wg, "grid": grid, "fetch_bytes": round(fb),
                    "write_bytes": round(wb), "sources_sha256": sources_sha256()}
    lines += ["", "The kernel with the most bytes written is the one whose traffic bench.py reports:", "",
              "<!-- dominant " + json.dumps(best) + " -->"]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def roofline_row(B, F, ms, prec):
    """t_roof = max(algorithmic bytes / 8 TB/s, algorithmic float64 flops /
    78.6 TFLOP/s) for float64; the split precisions run the contraction on the
    bf16/fp32 matrix cores (2.5 / 0.157 PFLOP/s), so their bound is the HBM
    term (their float64 point work is a small part of F)."""
    t_hbm = B / (HBM_PEAK_GBS * 1e9)
    t_f64 = F / (FP64_PEAK_TFLOPS * 1e12)
    if prec == "fp64" and t_f64 > t_hbm:
        bound, t_roof = "fp64", t_f64
    else:
        bound, t_roof = "hbm", t_hbm
    return {"bound": bound, "t_roof_ms": round(t_roof * 1e3, 4), "frac": round(t_roof / (ms * 1e-3), 4)}


def summarize_counters(db_dir, out, title, command, only=""):
    """Mean value per dispatch of every counter of a --pmc run, one row per
    (kernel, block, grid, LDS); `only` (comma-separated) keeps kernels whose
    name contains one of its parts."""
    cur = _rocpd(db_dir).cursor()
    q = ("select k.name, k.workgroup_x, k.grid_x, k.lds_size, p.counter_name, p.counter_value from pmc_events p "
         "join kernels k on k.dispatch_id = p.dispatch_id")
    parts = [x for x in only.split(",") if x]
    agg, names = {}, []
    for name, wg, grid, lds, cname, v in cur.execute(q).fetchall():
        if parts and not any(f in name for f in parts):
            continue
        if cname not in names:
            names.append(cname)
        agg.setdefault((_short(name), wg, grid // max(1, wg), lds), {}).setdefault(cname, []).append(v)
    lines = [f"# {title}", "", "Counter run (from the repository root on the GPU host):", "", "```", command, "```", "",
             "Mean counter value per dispatch.", "",
             "| kernel | block | grid | LDS B | dispatches | " + " | ".join(names) + " |",
             "|---|---:|---:|---:|---:|" + "---:|" * len(names)]
    for (name, wg, grid, lds), d in sorted(agg.items()):
        nd = max(len(v) for v in d.values())
        vals = " | ".join(f"{np.mean(d[c]):.4g}" if c in d else "" for c in names)
        lines.append(f"| `{name}` | {wg} | {grid} | {lds} | {nd} | {vals} |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def time_launch(torch, fn, stream, ev, reps):
    fn()
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def other_workloads(torch, felocal, inputs, stream, ev, reps, which, autotune=True):
    res = []

    def record(name, form, cell, p, E, ms, prec="fp64", **extra):
        B = alg_bytes(form, cell, p) * E
        F = alg_flops(form, cell, p) * E
        row = {"workload": name, "form": form, "cell": cell, "degree": p, "elements": E, "precision": prec,
               "ms": round(ms, 4), "elem_per_s": round(E / (ms * 1e-3), 1),
               "alg_GBs": round(B / (ms * 1e-3) / 1e9, 1), "alg_GFLOPs": round(F / (ms * 1e-3) / 1e9, 1),
               "frac_hbm": round(B / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "frac_fp64": round(F / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4)}
        row["roofline"] = roofline_row(B, F, ms, prec)
        row.update(extra)
        res.append(row)
        log(f"  {name} {prec} {extra.get('kernel', '')}: {ms:.4f} ms, {row['elem_per_s']:.3e} elem/s, "
            f"{row['alg_GBs']} GB/s")

    # mass P1 triangles, 4096 elements (launch-latency bound)
    if "mass" in which:
        mass_workload(torch, felocal, inputs, stream, ev, record)
    if "elasticity" in which:
        elasticity_workload(torch, felocal, inputs, stream, ev, record, reps)
    if "hyperelastic" in which:
        hyperelastic_workload(torch, felocal, inputs, stream, ev, record, reps)
    if "batch" in which:
        res.append(batch_workload(torch, felocal, inputs, stream, ev, reps, autotune))
    if "sweep" in which:
        res.append(sweep_workload(torch, felocal, inputs, stream, ev, max(2, reps // 3)))
    if "global" in which:
        res.append(global_workload(torch, felocal, inputs, stream, ev, reps))
    if "nonaffine" in which:
        res.append(nonaffine_workload(torch, felocal, inputs, stream, ev, reps))
    if "forms" in which:
        res.append(forms_workload(torch, felocal, inputs, stream, ev, reps))
    return res


def forms_workload(torch, felocal, inputs, stream, ev, reps):
    """Automatic sharing elimination (Sec. 3.2, Algorithm 1) on a form no
    hand-written kernel covers: full-tensor diffusion sum_ab K_ab d_a u d_b v
    (9 products between 3 test and 3 trial symbols; the ILP factorises the 3
    test gradients) on 82,944 tetrahedra, P2-P4, with the generated
    sharing-eliminated nest against the generated expanded nest; then a
    vector-valued form (advection-diffusion with a P1 velocity, component
    blocks) the same way, and elasticity written as component terms against
    the library's own elasticity kernel.  Each row carries the algorithmic
    float64 rate (theta_se x elements / time) against the FP64 peak."""
    import itertools
    terms = [(a, b, -1, 1.0 + 0.25 * i) for i, (a, b) in enumerate(itertools.product(("dx", "dy", "dz"), repeat=2))]
    coords, V, cells, h = inputs.first_elements("tetrahedron", 82944, 46)
    c = torch.from_numpy(coords).cuda()
    out = {"workload": "sharing_elimination_full_tensor_tet_83k", "elements": int(c.shape[0]), "per_degree": {}}
    for p in (2, 3, 4):
        n = felocal.NBASIS("tetrahedron", p)
        o = torch.empty((int(c.shape[0]), n, n), dtype=torch.float64, device="cuda")
        pl = felocal.fe_sharing_plan(terms, "tetrahedron", p)
        ms = {}
        for ex in (False, True):
            ms[ex] = time_launch(torch, lambda: felocal.fe_assemble_form(terms, "tetrahedron", p, c, None, o,
                                                                         expanded=ex), stream, ev, reps)
        tf = pl["theta_se"] * int(c.shape[0]) / (ms[False] * 1e-3) / 1e12
        out["per_degree"][f"P{p}"] = {"factorised_ms": round(ms[False], 4), "expanded_ms": round(ms[True], 4),
                                      "theta_se": pl["theta_se"], "theta_expanded": pl["theta_expanded"],
                                      "factorised_symbols": int(sum(pl["factorized"])),
                                      "roofline": {"bound": "fp64", "achieved": round(tf, 2), "peak": FP64_PEAK_TFLOPS,
                                                   "unit": "TFLOP/s", "frac": round(tf / FP64_PEAK_TFLOPS, 4)}}
        log(f"  sharing elimination P{p}: factorised {ms[False]:.4f} ms, expanded {ms[True]:.4f} ms")
        del o
    # a vector-valued form (component-blocked, one loop nest per block):
    # nu grad u : grad v + (w . grad) u . v with a P1 velocity w, whose
    # diagonal blocks factorise to the 3 trial derivatives (6 products each);
    # and the elasticity form as component terms (every block a matching, so
    # expanded) against the library's own elasticity kernel
    D3 = ("dx", "dy", "dz")
    vterms = [t for a in range(3) for b in range(3)
              for t in ((D3[b], D3[b], -1, 0.1, a, a), ("value", D3[b], b, 1.0, a, a))]
    eterms = [t for a in range(3) for b in range(3)
              for t in ((D3[b], D3[b], 1, 1.0, a, a), (D3[b], D3[a], 1, 1.0, a, b), (D3[a], D3[b], 0, 1.0, a, b))]
    g = torch.from_numpy(np.random.default_rng(47).uniform(0.5, 2.0, size=(int(c.shape[0]), 3, 4))).cuda()
    vec = {"form": "vector advection-diffusion, P1 velocity", "per_degree": {}}
    for p in (2, 3, 4):
        n = 3 * felocal.NBASIS("tetrahedron", p)
        o = torch.empty((int(c.shape[0]), n, n), dtype=torch.float64, device="cuda")
        pl = felocal.fe_sharing_plan(vterms, "tetrahedron", p, n_fields=3, n_comp=3)
        ms = {}
        for ex in (False, True):
            ms[ex] = time_launch(torch, lambda: felocal.fe_assemble_form(vterms, "tetrahedron", p, c, g, o, n_fields=3,
                                                                         expanded=ex, n_comp=3), stream, ev, reps)
        row = {"factorised_ms": round(ms[False], 4), "expanded_ms": round(ms[True], 4), "theta_se": pl["theta_se"],
               "theta_expanded": pl["theta_expanded"], "factorised_symbols": int(sum(pl["factorized"]))}
        if p == 2:
            lm = g[:, :2].contiguous()
            row["elasticity_generated_ms"] = round(time_launch(
                torch, lambda: felocal.fe_assemble_form(eterms, "tetrahedron", p, c, lm, o, n_fields=2, n_comp=3),
                stream, ev, reps), 4)
            row["elasticity_library_ms"] = round(time_launch(
                torch, lambda: felocal.fe_assemble_local("elasticity", "tetrahedron", p, c, lm.reshape(len(lm), -1), o,
                                                         stream=stream), stream, ev, reps), 4)
        tf = pl["theta_se"] * int(c.shape[0]) / (ms[False] * 1e-3) / 1e12
        row["roofline"] = {"bound": "fp64", "achieved": round(tf, 2), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": round(tf / FP64_PEAK_TFLOPS, 4)}
        vec["per_degree"][f"P{p}"] = row
        log(f"  vector form P{p}: factorised {ms[False]:.4f} ms, expanded {ms[True]:.4f} ms"
            + (f"; elasticity generated {row['elasticity_generated_ms']} ms, library "
               f"{row['elasticity_library_ms']} ms" if p == 2 else ""))
        del o
    out["vector"] = vec
    del c, g
    torch.cuda.empty_cache()
    return out


def nonaffine_workload(torch, felocal, inputs, stream, ev, reps):
    """Prisms without the affine assumption: Helmholtz P1-P3 on 2 x 63^3 =
    500,094 prisms.  On the affine mesh: the planner's choice (pre-evaluated)
    and forced quadrature; on the same mesh with every interior layer
    z-jittered (no prism affine): quadrature with the vertex map's geometry
    at every point (fe_options_t.pointgeo), the only legal mode there."""
    out = {"workload": "nonaffine_helmholtz_prism_500k", "per_degree": {}}
    Va, cells = inputs.prism_mesh(63, 63, 25)
    Vj, _ = inputs.prism_mesh(63, 63, 25, zjitter=0.3)
    ca = torch.from_numpy(inputs.gather(Va, cells)).cuda()
    cj = torch.from_numpy(inputs.gather(Vj, cells)).cuda()
    E = int(ca.shape[0])
    out["elements"] = E
    for p in (1, 2, 3):
        log(f"non-affine prisms: helmholtz P{p}")
        n, _ = felocal.fe_local_dims("helmholtz", "prism", p)
        o = torch.empty((E, n, n), dtype=torch.float64, device="cuda")
        ms_pre = time_launch(torch, lambda: felocal.fe_assemble_local("helmholtz", "prism", p, ca, None, o),
                             stream, ev, reps)
        ms_quad = time_launch(torch, lambda: felocal.fe_assemble_local("helmholtz", "prism", p, ca, None, o,
                                                                       mode="quadrature"), stream, ev, reps)
        ms_pg = time_launch(torch, lambda: felocal.fe_assemble_local("helmholtz", "prism", p, cj, None, o,
                                                                     pointgeo=True), stream, ev, reps)
        B = E * n * n * 8
        row = {"affine_planner_ms": round(ms_pre, 4), "affine_quadrature_ms": round(ms_quad, 4),
               "pointgeo_ms": round(ms_pg, 4), "pointgeo_elem_per_s": round(E / (ms_pg * 1e-3), 1),
               "pointgeo_store_GBs": round(B / (ms_pg * 1e-3) / 1e9, 1)}
        out["per_degree"][f"P{p}"] = row
        log(f"  P{p}: affine planner {ms_pre:.4f} ms, affine quadrature {ms_quad:.4f} ms, "
            f"non-affine per-point geometry {ms_pg:.4f} ms")
        del o
        torch.cuda.empty_cache()
    del ca, cj
    out["curved_tet"] = curved_workload(torch, felocal, inputs, stream, ev, reps)
    return out


def curved_workload(torch, felocal, inputs, stream, ev, reps):
    """Curved tetrahedra (an isoparametric P2 coordinate field, interior edges
    bent by U(+-0.04 h)): Helmholtz P1-P3 on 50^3 x 6 = 750,000 tetrahedra
    with J at every point (fe_options_t.coord_degree = 2, quadrature only),
    against the straight mesh's planner choice (pre-evaluated) and forced
    quadrature."""
    x2, V, cells, h = inputs.curved_mesh("tetrahedron", 50, 26)
    cc = torch.from_numpy(x2).cuda()
    ca = torch.from_numpy(inputs.gather(V, cells)).cuda()
    E = int(cc.shape[0])
    res = {"elements": E, "per_degree": {}}
    for p in (1, 2, 3):
        log(f"curved tetrahedra: helmholtz P{p}")
        n, _ = felocal.fe_local_dims("helmholtz", "tetrahedron", p)
        o = torch.empty((E, n, n), dtype=torch.float64, device="cuda")
        ms_pre = time_launch(torch, lambda: felocal.fe_assemble_local("helmholtz", "tetrahedron", p, ca, None, o),
                             stream, ev, reps)
        ms_quad = time_launch(torch, lambda: felocal.fe_assemble_local("helmholtz", "tetrahedron", p, ca, None, o,
                                                                       mode="quadrature"), stream, ev, reps)
        ms_cv = time_launch(torch, lambda: felocal.fe_assemble_local("helmholtz", "tetrahedron", p, cc, None, o,
                                                                     coord_degree=2), stream, ev, reps)
        B = E * n * n * 8
        res["per_degree"][f"P{p}"] = {"affine_planner_ms": round(ms_pre, 4), "affine_quadrature_ms": round(ms_quad, 4),
                                      "curved_ms": round(ms_cv, 4), "curved_elem_per_s": round(E / (ms_cv * 1e-3), 1),
                                      "curved_store_GBs": round(B / (ms_cv * 1e-3) / 1e9, 1)}
        log(f"  P{p}: affine planner {ms_pre:.4f} ms, affine quadrature {ms_quad:.4f} ms, curved {ms_cv:.4f} ms")
        del o
        torch.cuda.empty_cache()
    del cc, ca
    return res


def mass_workload(torch, felocal, inputs, stream, ev, record):
    log("mass P1 triangles 4096")
    c1 = torch.from_numpy(inputs.mass_tri_workload(seed=1)).cuda()
    o1 = torch.empty((4096, 3, 3), dtype=torch.float64, device="cuda")
    ms = time_launch(torch, lambda: felocal.fe_assemble_local("mass", "triangle", 1, c1, None, o1, qdeg=2),
                     stream, ev, 50)
    record("mass_tri_p1_4096", "mass", "triangle", 1, 4096, ms, note="launch-latency bound (0.49 MB)")


# float64 through the VALU quadrature kernel (launch-shape kernel 3) and the
# matrix-core Gram kernel (kernel 4; the default except at degree 1), then
# the two split precisions; at degree 1 also the hoisted kernel (kernel 5,
# the default there)
FP64_AND_SPLIT = [("fp64", {"kernel": 3}), ("fp64", {"kernel": 4}), ("fp32", None), ("bf16x3", None)]
FP64_P1 = [("fp64", {"kernel": 5})]


def kernel_name(prec, shape, degree=2):
    if prec != "fp64":
        # degree 1 on simplices: the split precisions run the float64 hoisted kernel
        return "k_vec_p1 (hoisted degree 1, float64)" if degree == 1 else f"k_split {prec} MFMA"
    return {3: "k_quad (VALU)", 4: "k_gram64 (f64 MFMA)", 5: "k_vec_p1 (hoisted degree 1)"}[shape["kernel"]]


def elasticity_workload(torch, felocal, inputs, stream, ev, record, reps):
    log("elasticity P2 on 1.97M tets")
    cn, V, cells = inputs.tet_workload(69, seed=3)
    E3 = cn.shape[0]
    c3 = torch.from_numpy(cn).cuda()
    cf3 = torch.from_numpy(inputs.lame_p1(V.shape[0], cells, seed=3)).cuda()
    o3 = torch.empty((E3, 30, 30), dtype=torch.float64, device="cuda")
    for prec, kern in FP64_AND_SPLIT:
        ms = time_launch(torch, lambda: felocal.fe_assemble_local("elasticity", "tetrahedron", 2, c3, cf3, o3,
                                                                  precision=prec, shape=kern), stream, ev, reps)
        record("elasticity_tet_p2_2m", "elasticity", "tetrahedron", 2, E3, ms, prec, kernel=kernel_name(prec, kern))
    del o3, c3, cf3
    torch.cuda.empty_cache()


def hyperelastic_workload(torch, felocal, inputs, stream, ev, record, reps):
    cn, V, cells = inputs.tet_workload(55, seed=4)
    E4 = cn.shape[0]
    c4 = torch.from_numpy(cn).cuda()
    for p in (1, 2):
        log(f"hyperelastic P{p} on 998k tets")
        ns = n_scalar("tetrahedron", p)
        u = torch.from_numpy(inputs.displacement_dofs(E4, 3, ns, 1.0 / 55, seed=40 + p)).cuda()
        o4 = torch.empty((E4, 3 * ns, 3 * ns), dtype=torch.float64, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        for prec, kern in (FP64_P1 if p == 1 else []) + FP64_AND_SPLIT:
            st.zero_()
            ms = time_launch(torch, lambda: felocal.fe_assemble_local("hyperelastic", "tetrahedron", p, c4, u, o4,
                                                                      precision=prec, status=st, shape=kern),
                             stream, ev, reps)
            record(f"hyperelastic_tet_p{p}_1m", "hyperelastic", "tetrahedron", p, E4, ms, prec,
                   kernel=kernel_name(prec, kern, p), flagged_per_launch=int(st.item()) // (reps + 1))
        del o4, u
        torch.cuda.empty_cache()
    del c4


def global_workload(torch, felocal, inputs, stream, ev, reps):
    """Local plus global assembly (Sec. 2; Sec. 7.1 times the two together) of
    the Helmholtz form on the 750,000-tetrahedron mesh, P1-P4: the element
    matrices (pre-evaluated kernel), then their insertion into the
    compressed-row matrix of the continuous space (fe_csr_insert); and both in
    one pass (fe_assemble_csr), which forms each entry where it is added.
    Algorithmic bytes of the insertion: the element matrices read and the
    stored entries written; the index data it also reads (2 B per
    element-matrix entry, 4 B per element row, 16 B per global row) is
    reported beside them.  The one pass moves the stored entries and the
    index data."""
    cn, V, cells = inputs.tet_workload(50, seed=2)
    c = torch.from_numpy(cn).cuda()
    out = {"workload": "global_helmholtz_tet_750k", "elements": int(cn.shape[0]), "per_degree": {}}
    for p in (1, 2, 3, 4):
        log(f"global assembly helmholtz P{p} 750k tets")
        dofs, N = inputs.global_dofs("tetrahedron", p, cells, 50)
        E, n = dofs.shape
        d = torch.from_numpy(dofs).cuda()
        torch.cuda.synchronize()
        t0 = time.time()
        pat = felocal.CsrPattern(d, N)
        create_s = time.time() - t0
        info = pat.info()
        local = torch.empty((E, n, n), dtype=torch.float64, device="cuda")
        vals = torch.empty(info["nnz"], dtype=torch.float64, device="cuda")
        ms_local = time_launch(torch, lambda: felocal.fe_assemble_local("helmholtz", "tetrahedron", p, c, None, local),
                               stream, ev, reps)
        ms_ins = time_launch(torch, lambda: pat.insert(local, vals), stream, ev, reps)

        def both():
            felocal.fe_assemble_local("helmholtz", "tetrahedron", p, c, None, local)
            pat.insert(local, vals)
        ms_both = time_launch(torch, both, stream, ev, reps)
        ms_fused = time_launch(torch, lambda: pat.assemble("helmholtz", "tetrahedron", p, c, vals), stream, ev, reps)
        alg = E * n * n * 8 + info["nnz"] * 8
        index = E * n * n * 2 + E * n * 4 + 2 * (N + 1) * 8
        row = {"rows": N, "nnz": info["nnz"], "max_row_len": info["max_row_len"],
               "pattern_build_s": round(create_s, 3), "local_ms": round(ms_local, 4),
               "insert_ms": round(ms_ins, 4), "local_plus_insert_ms": round(ms_both, 4),
               "insert_alg_GBs": round(alg / (ms_ins * 1e-3) / 1e9, 1),
               "insert_alg_plus_index_GBs": round((alg + index) / (ms_ins * 1e-3) / 1e9, 1),
               "insert_frac_hbm": round(alg / (ms_ins * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "global_elem_per_s": round(E / (ms_both * 1e-3), 1),
               "one_pass_ms": round(ms_fused, 4),
               "one_pass_elem_per_s": round(E / (ms_fused * 1e-3), 1),
               "one_pass_GBs": round((info["nnz"] * 8 + E * n * n * 2 + E * n * 4 + 2 * (N + 1) * 8)
                                     / (ms_fused * 1e-3) / 1e9, 1)}
        out["per_degree"][f"P{p}"] = row
        log(f"  P{p}: N {N} nnz {info['nnz']} local {ms_local:.4f} ms insert {ms_ins:.4f} ms "
            f"({row['insert_alg_GBs']} GB/s alg, {row['insert_alg_plus_index_GBs']} with index) "
            f"both {ms_both:.4f} ms; one pass {ms_fused:.4f} ms; pattern {create_s:.2f} s")
        pat.close()
        del local, vals, d
        torch.cuda.empty_cache()
    del c
    return out


def sweep_workload(torch, felocal, inputs, stream, ev, reps):
    """The experiment matrix of Sec. 7.1 on one GPU: mass and Helmholtz,
    degree q = 1..4, nf = 0..3 pre-multiplying coefficient functions of
    degree q, on 82,944 jittered tetrahedra (24^3 cubes x 6; the paper's mesh
    has 4,374).  Per case: Algorithm 3's choice (T_H = LDS per CU) and the
    time of the chosen mode, of forced quadrature and of forced
    pre-evaluation (where a tile of the expanded tensor fits in LDS)."""
    log("sweep: mass / helmholtz, q = 1..4, nf = 0..3 on 82,944 tets")
    # Algorithm 3's own choices: forget the modes the autotuner measured
    felocal.lib().fe_autotune_clear()
    cn, V, cells = inputs.tet_workload(24, seed=6)
    E = cn.shape[0]
    c = torch.from_numpy(cn).cuda()
    rng = np.random.default_rng(7)
    cases = []
    for form in ("mass", "helmholtz"):
        for q in (1, 2, 3, 4):
            ns = n_scalar("tetrahedron", q)
            out = torch.empty((E, ns, ns), dtype=torch.float64, device="cuda")
            for nf in (0, 1, 2, 3):
                cf = torch.from_numpy(rng.uniform(0.5, 1.5, size=(E, nf, ns))).cuda() if nf else None
                plan = felocal.fe_plan(form, "tetrahedron", q, nf=nf)
                row = {"form": form, "q": q, "nf": nf, "plan": plan["mode"],
                       "preevaluated": plan["preevaluated"], "iota": plan["iota"][0]}
                for mode in ("auto", "quadrature", "preeval"):
                    try:
                        ms = time_launch(torch, lambda: felocal.fe_assemble_local(
                            form, "tetrahedron", q, c, cf, out, nf=nf, mode=mode), stream, ev, reps)
                        row[f"ms_{mode}"] = round(ms, 4)
                    except felocal.FeError:
                        row[f"ms_{mode}"] = None
                t = [v for k, v in row.items() if k.startswith("ms_") and k != "ms_auto" and v is not None]
                # within 5% (and 5 us, the launch-to-launch noise) of the faster forced mode
                row["planner_fastest"] = row["ms_auto"] is not None and row["ms_auto"] <= 1.05 * min(t) + 0.005
                row["elem_per_s"] = round(E / (row["ms_auto"] * 1e-3), 1)
                cases.append(row)
                log(f"  {form} q={q} nf={nf}: plan {plan['mode']} {plan['preevaluated']} auto {row['ms_auto']} "
                    f"quad {row['ms_quadrature']} pre {row['ms_preeval']} ms")
                del cf
            del out
            torch.cuda.empty_cache()
    hits = sum(r["planner_fastest"] for r in cases)
    vec = vector_sweep(torch, felocal, inputs, stream, ev, reps)
    vhits = sum(r["planner_fastest"] for r in vec["cases"])
    return {"workload": "nf_sweep_tet_83k", "elements": E, "cases": cases,
            "planner_fastest_cases": f"{hits}/{len(cases)}", "vector": vec,
            "vector_planner_fastest_cases": f"{vhits}/{len(vec['cases'])}"}


def vector_sweep(torch, felocal, inputs, stream, ev, reps):
    """The Sec. 7.1 matrix for Elasticity (P1 Lame fields) and the neo-Hookean
    tangent: q = 1..4, nf = 0..3 functions of degree q, on the paper's mesh
    size, 4,374 jittered tetrahedra (9^3 cubes x 6).  Per case: Algorithm 3's
    choice and the time of the chosen mode, of forced quadrature and of forced
    pre-evaluation (elasticity where a tile fits the LDS; illegal for the
    hyperelastic terms in F)."""
    log("sweep: elasticity / hyperelastic, q = 1..4, nf = 0..3 on 4,374 tets")
    cn, V, cells = inputs.tet_workload(9, seed=8)
    E = cn.shape[0]
    c = torch.from_numpy(cn).cuda()
    rng = np.random.default_rng(9)
    cases = []
    for form in ("elasticity", "hyperelastic"):
        for q in (1, 2, 3, 4):
            ns = n_scalar("tetrahedron", q)
            out = torch.empty((E, 3 * ns, 3 * ns), dtype=torch.float64, device="cuda")
            own = inputs.lame_p1(V.shape[0], cells, seed=10).reshape(E, -1) if form == "elasticity" else \
                inputs.displacement_dofs(E, 3, ns, 1.0 / 9, seed=11, rel=0.05 / max(1, q - 1))
            for nf in (0, 1, 2, 3):
                cf = np.concatenate([own, rng.uniform(0.5, 1.5, size=(E, nf * ns))], axis=1)
                cft = torch.from_numpy(np.ascontiguousarray(cf)).cuda()
                plan = felocal.fe_plan(form, "tetrahedron", q, nf=nf)
                row = {"form": form, "q": q, "nf": nf, "plan": plan["mode"],
                       "preevaluated": plan["preevaluated"], "iota": plan["iota"]}
                for mode in ("auto", "quadrature", "preeval"):
                    try:
                        ms = time_launch(torch, lambda: felocal.fe_assemble_local(
                            form, "tetrahedron", q, c, cft, out, nf=nf, mode=mode), stream, ev, reps)
                        row[f"ms_{mode}"] = round(ms, 4)
                    except felocal.FeError:
                        row[f"ms_{mode}"] = None
                t = [v for k, v in row.items() if k.startswith("ms_") and k != "ms_auto" and v is not None]
                row["planner_fastest"] = row["ms_auto"] is not None and row["ms_auto"] <= 1.05 * min(t) + 0.005
                cases.append(row)
                log(f"  {form} q={q} nf={nf}: plan {plan['preevaluated']} auto {row['ms_auto']} "
                    f"quad {row['ms_quadrature']} pre {row['ms_preeval']} ms")
                del cft
            del out
            torch.cuda.empty_cache()
    return {"elements": E, "cases": cases}


def batch_workload(torch, felocal, inputs, stream, ev, reps, autotune=True):
    log("mixed batch: 16 sub-batches, one graph launch of per-variant persistent kernels")
    rng = np.random.default_rng(5)
    subs, tot_e, tot_b, tot_f = [], 0, 0, 0
    desc, bounds = [], []
    for i in range(16):
        form = ["mass", "helmholtz", "elasticity"][rng.integers(3)]
        cell = ["triangle", "tetrahedron", "prism"][rng.integers(3)]
        p = int(rng.integers(1, 5))
        E = int(round(math.exp(rng.uniform(math.log(1e4), math.log(5e5)))))
        n = n_scalar(cell, p) * (GD[cell] if form == "elasticity" else 1)
        E = min(E, (4 << 30) // (8 * n * n))
        coords, Vb, cb, h = inputs.first_elements(cell, E, seed=500 + i)
        cf = inputs.lame_p1(Vb.shape[0], cb, seed=600 + i) if form == "elasticity" else None
        subs.append(dict(form=form, cell=cell, degree=p, coords=torch.from_numpy(coords).cuda(),
                         coeff=torch.from_numpy(cf).cuda() if cf is not None else None,
                         out=torch.empty((E, n, n), dtype=torch.float64, device="cuda")))
        desc.append(f"{form}/{cell}/P{p}/{E}")
        tot_e += E
        tot_b += alg_bytes(form, cell, p) * E
        pre = form == "elasticity" and felocal.fe_plan(form, cell, p)["mode"] == "preeval"
        tot_f += alg_flops(form, cell, p, preeval=pre) * E
        tb = alg_bytes(form, cell, p) * E / (HBM_PEAK_GBS * 1e9)
        tf = alg_flops(form, cell, p, preeval=pre) * E / (FP64_PEAK_TFLOPS * 1e12)
        bounds.append({"sub": desc[-1], "bound": "hbm" if tb >= tf else "fp64", "t_roof": max(tb, tf)})
    # untimed: the autotuner picks each sub-batch's kernel shape (the batch and
    # the separate launches both use it)
    # (--no-autotune: the shapes already in the cache, e.g. from FE_AUTOTUNE_CACHE)
    tuned = []
    for sb in subs if autotune else []:
        ms_t, shape = felocal.fe_autotune(sb["form"], sb["cell"], sb["degree"], sb["coords"], sb["coeff"], sb["out"],
                                          return_shape=True)
        tuned.append(dict({k: v for k, v in shape.items() if v}, ms=round(ms_t, 4)))
    b = felocal.Batch(subs)
    ntiles, grid = b.info()
    ms = time_launch(torch, b.run, stream, ev, reps)
    seq = time_launch(torch, lambda: [felocal.fe_assemble_local(s["form"], s["cell"], s["degree"], s["coords"],
                                                                 s["coeff"], s["out"]) for s in subs],
                      stream, ev, reps)
    b.close()
    t_roof = sum(r["t_roof"] for r in bounds)
    row = {"workload": "mixed_batch_16", "elements": tot_e, "ms": round(ms, 4),
           "elem_per_s": round(tot_e / (ms * 1e-3), 1), "alg_GBs": round(tot_b / (ms * 1e-3) / 1e9, 1),
           "alg_GFLOPs": round(tot_f / (ms * 1e-3) / 1e9, 1), "tiles": ntiles, "grid": grid,
           "separate_launches_ms": round(seq, 4), "sub_batches": desc, "tuned_shapes": tuned,
           "roofline": {"bound": "sum of the sub-batches' bounds", "t_roof_ms": round(t_roof * 1e3, 4),
                        "frac": round(t_roof / (ms * 1e-3), 4),
                        "per_sub_batch": [dict(r, t_roof=round(r["t_roof"] * 1e3, 4)) for r in bounds]}}
    log(f"  mixed batch: {ms:.3f} ms graph vs {seq:.3f} ms separate launches, {tot_e} elements")
    del subs
    torch.cuda.empty_cache()
    return row


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_leg(oracle, coords_np, nthreads, t_target, n_cap):
    """For each degree, the first n elements (n grown until the degree takes
    t_target seconds, at most n_cap): seconds per element and the matrices."""
    t_per, sample, mats = {}, {}, {}
    for p in (1, 2, 3, 4):
        n = 64
        while True:
            t = time.perf_counter()
            A, _ = oracle.assemble("helmholtz", "tetrahedron", p, coords_np[:n], nthreads=nthreads)
            dt = time.perf_counter() - t
            if dt >= t_target or n >= n_cap:
                break
            n = min(n_cap, n * 4 if dt < t_target / 5 else n * 2)
        t_per[p], sample[p], mats[p] = dt / n, n, A
        log(f"cpu oracle P{p}: {n} elements in {dt:.2f} s on {nthreads} thread(s)")
    return t_per, sample, mats


def cpu_baseline(coords_np, gpu_out=None):
    """The float64 oracle (naive Eq. (7) nest, OpenMP over elements) on a
    bounded sample of the headline workload, on all host threads (for each
    degree the first n elements, n grown until that degree takes >= 2.5 s)
    and on one thread (the paper's single-core setting of Sec. 7.1; the
    first elements, at most 16,384, per degree, extrapolated per element).
    With gpu_out (the headline's device outputs per degree), every matrix the
    all-threads leg computed is compared with the GPU's, element by element:
    max over elements of max|A_gpu - A_oracle| / max|A_oracle|."""
    import oracle

    cores = oracle.max_threads()
    t_per, sample, mats = _oracle_leg(oracle, coords_np, cores, 2.5, coords_np.shape[0])
    t1, sample1, _ = _oracle_leg(oracle, coords_np, 1, 2.5, 16384)
    per_step = sum(t_per.values())
    base = {"value": round(4.0 / per_step, 1), "unit": "element matrices/s", "cores": cores, "kind": "oracle",
            "sample": "helmholtz tet P1-P4, first " + ", ".join(f"P{p}:{sample[p]}" for p in sample)
                      + " elements of the 750k mesh; rate = 4 / sum_p(seconds per element)",
            "cpu_model": cpu_model(),
            "one_core": {"value": round(4.0 / sum(t1.values()), 1), "unit": "element matrices/s", "cores": 1,
                         "sample": "first " + ", ".join(f"P{p}:{sample1[p]}" for p in sample1)
                                   + " elements, extrapolated per element"}}
    parity = None
    if gpu_out is not None:
        per = {}
        for p in (1, 2, 3, 4):
            B = mats[p]
            A = gpu_out[p][:B.shape[0]].cpu().numpy()
            err = np.max(np.abs(A - B), axis=(1, 2)) / np.max(np.abs(B), axis=(1, 2))
            per[f"P{p}"] = {"elements": int(B.shape[0]), "max_err": float(err.max())}
            log(f"parity P{p}: {B.shape[0]} elements, max normwise error {err.max():.3e}")
        parity = {"metric": "max_e max|A_gpu - A_oracle| / max|A_oracle|", "bar": 1e-12,
                  "max_err": max(v["max_err"] for v in per.values()), "per_degree": per}
    return base, parity


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "summarize-trace":
        # summarize-trace DB_DIR OUT.md TITLE COMMAND [NAME_FILTER [LABELS]]
        summarize_trace(*sys.argv[2:8])
    elif len(sys.argv) > 1 and sys.argv[1] == "summarize-counters":
        # summarize-counters DB_DIR OUT.md TITLE COMMAND [NAME_FILTER]
        summarize_counters(*sys.argv[2:7])
    elif len(sys.argv) > 1 and sys.argv[1] == "summarize-traffic":
        # summarize-traffic FETCH_DIR WRITE_DIR OUT.md TITLE COMMAND_FETCH COMMAND_WRITE
        summarize_traffic(*sys.argv[2:8])
    else:
        main()
