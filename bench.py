"""Benchmark of the AIR reconstruction path on one MI355X.

A step is one full AIR reconstruction of a batch of independent 512 x 512
fan-beam cases (720 views x 736 bins, split Bregman 50 x 5 CG, the whole hot
path: Joseph projector, ramp GEMM, matched backprojector, CG updates,
framelet shrinkage), from the noisy sinograms already resident in HBM.

    python bench.py [--steps K] [--warmup W] [--batch B]

Prints one JSON line with
  value / p50_ms / p99_ms   recon/s and step latency of the float32 path (the
                            batch runs as two sub-batches on two streams),
  mixed                     the same for the mixed-precision path,
  rel_l2_vs_oracle          image 0 (seed 0) of the last timed step of each path
                            against the stored FP64 oracle reconstruction,
  c2_25                     the same scan with 25% of the views (180),
  served                    continuous-batching serving of the mixed-geometry
                            request stream (Poisson arrivals at 40/s, both
                            paths; p50/p99 arrival-to-result latency; a short
                            rate sweep of the mixed path),
  kernel_ms / roofline      HIP-event times of every kernel in a solve of the
                            timed configuration, and the dominant kernel on its
                            roofline (kernel_ms_alone / roofline_alone: the
                            same with every kernel running alone),
  cpu_baseline              the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import copy
import hashlib
import json
import os
import sys
import time

import numpy as np


ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "mixed_f16": 2500.0, "mixed_bf16": 2500.0}
# Published float32 vector peak, 157.3 TFLOP/s, counts packed float32 FMAs (two
# per lane and instruction).  This build issues no packed float32 operations; a
# wave64 VALU instruction holds its 16-lane SIMD four cycles, so the issue peak
# is 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 39.3 T lane operations per second
# (78.6 TFLOP/s of non-packed FMAs; a register-only v_fmac_f32 loop measures
# 37.2 T FMA/s).  `frac` is taken against the published peak, as required;
# `frac_nonpacked` against the non-packed one.
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP32_NONPACKED_PEAK_TFLOPS = 78.6
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Work of the projectors per Joseph sample (ray-step): two fused multiply-adds
# per image (the two interpolation taps), plus the index work a thread shares
# over its group of images (advance the intercept, convert its fraction, the
# two weights, the sample address: 5 lane operations per group).
FMA_PER_SAMPLE_IMAGE = 2
SHARED_OPS_PER_SAMPLE_GROUP = 5
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c2.json")
GOLDEN = os.path.join(ROOT, "tests", "golden")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c2_25", "c5", "c3_gemm"],
                    help="c3_gemm: the ramp GEMM alone at the 736 x 736 filter x 11,520-row measurement shape")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-quarter", action="store_true", help="skip the 25%%-data (180-view) leg")
    ap.add_argument("--kernel-timing-only", action="store_true",
                    help="skip the timed steps; run only the instrumented pass (for profiler runs)")
    ap.add_argument("--one-stream", action="store_true",
                    help="profiler runs only: the instrumented pass runs every kernel alone")
    ap.add_argument("--outer", type=int, default=0,
                    help="profiler runs only: Bregman iterations of the instrumented pass (0 = the workload's)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="profiler runs only: also run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--serve", action="store_true",
                    help="run only the continuous-batching serving benchmark (Poisson arrivals, mixed geometries)")
    ap.add_argument("--serve-requests", type=int, default=330)
    ap.add_argument("--serve-warmup", type=int, default=30, help="first requests left out of the latency figures")
    ap.add_argument("--serve-rate", type=float, default=40.0, help="offered load, requests per second")
    ap.add_argument("--serve-capacity", type=int, default=8, help="slots per geometry group")
    ap.add_argument("--hw-queues", type=int, default=16,
                    help="GPU_MAX_HW_QUEUES for this process (1-32; 0 keeps the environment's value)")
    ap.add_argument("--serve-max-active", type=int, default=5,
                    help="groups stepping at a time, those holding the oldest requests (0: all)")
    ap.add_argument("--serve-precision", default="mixed_f16", choices=["fp32", "mixed_f16", "mixed_bf16"])
    ap.add_argument("--quality", action="store_true",
                    help="run the FBP / IR / AIR image-quality comparison (CNR, FWHM) on the paper-shaped scan")
    ap.add_argument("--quality-i0", type=float, default=2e4, help="incident photons per ray of the quality scans")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) into profiles/traffic_c2.json")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="print a markdown table of a rocprofv3 --kernel-trace --stats output directory")
    ap.add_argument("--summarize-timeline", metavar="DIR",
                    help="print a markdown summary of a rocprofv3 --kernel-trace output directory (busy fraction, "
                         "concurrency, time per kernel)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="print a markdown table of rocprofv3 --pmc output directories (per-dispatch averages of the "
                         "projector, backprojector and ramp kernels, with derived rates)")
    return ap.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1310_1434_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def rel_l2(x, ref) -> float:
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))


def timed_steps(torch, plan, y, w, steps, warmup, ws):
    """W untimed steps, then K timed steps between two synchronisations; returns
    (wall seconds, per-step event latencies in ms, the last step's images)."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.solve(y, w.lam, w.mu, w.n_outer, w.n_cg, workspace=ws, with_resid=False)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    x = None
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(steps):
        x, _ = plan.solve(y, w.lam, w.mu, w.n_outer, w.n_cg, workspace=ws, with_resid=False)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    return wall, lat, x


def ray_steps(plan) -> int:
    _, lo, hi = plan.tables()
    return int(np.maximum(hi - lo + 1, 0).sum())


def image_group(batch: int) -> int:
    """Images per backprojector thread (the library's own choice for a launch of `batch`)."""
    best, cost = 1, 3 * batch
    for g in (2, 4, 8, 16):
        c = -(-batch // g) * (2 + g)
        if c < cost:
            best, cost = g, c
    return best


def golden_image(name: str):
    path = os.path.join(GOLDEN, name + ".npz")
    return np.load(path)["x"] if os.path.exists(path) else None


def instrumented(torch, air, plan, y, w, ws, mode, n_outer):
    """One solve with every kernel bracketed by HIP events on its launch stream."""
    plan.kernel_timing(mode)
    plan.solve(y, w.lam, w.mu, n_outer, w.n_cg, workspace=ws, with_resid=False)
    torch.cuda.synchronize()
    kt = plan.collect_kernel_timing()
    plan.kernel_timing("off")
    return {k: {"avg_ms": (v[0] / v[1]) if v[1] else 0.0, "launches": v[1], "total_ms": v[0]} for k, v in kt.items()}


def operator_applies(kind, n_outer, n_cg):
    """Launches of one operator per image in a split-Bregman solve: the CG
    products, the start image's residual (one apply at the start: later CG runs
    start from the carried residual) and, for the ramp and the backprojector,
    A'^T Y."""
    return n_outer * n_cg + (1 if kind == "project" else 2)


def roofline(kernel_ms, g, B, n_outer, n_cg, rsteps, precision, label):
    """The dominant kernel of an instrumented solve on its roofline.  Images per
    launch follow from the launch count (a split batch launches each operator
    once per sub-batch)."""
    dom = max(("project", "backproject", "ramp"), key=lambda k: kernel_ms[k]["total_ms"])
    km = kernel_ms[dom]
    t = km["avg_ms"] * 1e-3
    ipl = B * operator_applies(dom, n_outer, n_cg) / km["launches"]
    if dom == "ramp":
        flops = 2.0 * ipl * g.n_views * g.n_bins * g.n_bins
        peak = MFMA_PEAK_TFLOPS["fp32" if precision == "fp32" else precision]
        achieved = flops / t / 1e12
        return {"kernel": "k_ramp_" + ("f32" if precision == "fp32" else "split"), "config": label, "bound": "mfma",
                "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "images_per_launch": ipl, "avg_launch_ms": t * 1e3}
    flops = 2.0 * FMA_PER_SAMPLE_IMAGE * ipl * rsteps
    achieved = flops / t / 1e12
    G = image_group(int(round(ipl))) if dom == "backproject" else (4 if precision != "fp32" else 2)
    groups = -(-int(round(ipl)) // G)
    lane_ops = (FMA_PER_SAMPLE_IMAGE * ipl + SHARED_OPS_PER_SAMPLE_GROUP * groups) * rsteps
    return {"kernel": "k_" + dom, "config": label, "bound": "alu", "achieved": achieved,
            "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
            "frac_nonpacked": achieved / FP32_NONPACKED_PEAK_TFLOPS,
            "work": f"{FMA_PER_SAMPLE_IMAGE} FMA (4 flop) per Joseph sample per image, {rsteps} samples per image, "
                    f"{ipl:g} images per launch",
            "valu_issue_frac": lane_ops / t / (VALU_PEAK_TOPS * 1e12),
            "valu_issue_work": f"the FMAs plus {SHARED_OPS_PER_SAMPLE_GROUP} shared index operations per sample "
                               f"per group of {G} images, against {VALU_PEAK_TOPS:.1f} T lane operations/s",
            "images_per_launch": ipl, "avg_launch_ms": t * 1e3, "ray_steps_per_image": rsteps}


def traffic_for(kernel_instance: str, batch: int):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources at this batch."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    tr = json.load(open(TRAFFIC_FILE))
    if tr.get("source_hash") != kernel_source_hash() or tr.get("batch") != batch:
        return None
    ent = tr.get("kernels", {}).get(kernel_instance)
    return ent["bytes_per_launch"] if ent else None


def cpu_baseline(w, y0):
    """FP64 oracle on the host's cores, bounded: solves of 1 and 3 Bregman
    iterations of one C2 case give the cost per iteration and the one-off set-up
    (g = A'^T Y), from which the 50-iteration solve is extrapolated; plus the
    time per apply of A and A'^T on all cores and on one, and a full C1 solve."""
    import oracle
    import synth
    oracle.build(force=False)
    cores = oracle.num_threads()
    g = oracle.Geom(w.geom)
    y = y0.astype(np.float64)

    def clock(f):
        t = time.perf_counter()
        f()
        return time.perf_counter() - t

    t1 = clock(lambda: oracle.solve(g, y, w.lam, w.mu, 1, w.n_cg))
    t3 = clock(lambda: oracle.solve(g, y, w.lam, w.mu, 3, w.n_cg))
    per_outer = (t3 - t1) / 2.0
    setup = t1 - per_outer
    full = setup + w.n_outer * per_outer
    x = np.zeros((w.geom.n, w.geom.n)) + 0.01
    per_apply = {"cores": cores}
    per_apply["A_s"] = min(clock(lambda: oracle.project(g, x)) for _ in range(2))
    per_apply["AtC_s"] = min(clock(lambda: oracle.filtered_backproject(g, y, 1)) for _ in range(2))
    oracle.set_threads(1)
    try:
        per_apply["A_s_1core"] = clock(lambda: oracle.project(g, x))
        per_apply["AtC_s_1core"] = clock(lambda: oracle.filtered_backproject(g, y, 1))
    finally:
        oracle.set_threads(cores)
    w1 = synth.workload("c1")
    y1 = synth.make_case(w1, 0)["y"].astype(np.float32).astype(np.float64)
    t_c1 = clock(lambda: oracle.solve(oracle.Geom(w1.geom), y1, w1.lam, w1.mu, w1.n_outer, w1.n_cg))
    return {"value": 1.0 / full, "unit": "recon/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle on {cores} threads, one {w.geom.n}^2 x {w.geom.n_views}-view case: solves of 1 and "
                      f"3 Bregman iterations (x{w.n_cg} CG) took {t1:.2f} s and {t3:.2f} s, i.e. {per_outer:.2f} s per "
                      f"iteration and {setup:.2f} s of set-up; value is the {w.n_outer}-iteration solve extrapolated "
                      f"from them ({full:.1f} s)",
            "extrapolated": True, "per_apply": per_apply,
            "c1_solve_s": t_c1, "c1_solve": f"{w1.geom.n}^2 x {w1.geom.n_views} views, {w1.n_outer} x {w1.n_cg}, "
                                             f"measured whole on {cores} threads"}


def summarize_pmc(fetch_dir: str, write_dir: str, batch: int):
    """Per-dispatch HBM bytes of each kernel from FETCH_SIZE / WRITE_SIZE (KiB),
    each scaled so that the calibration copy of 256 MiB reads/writes 256 MiB."""
    import csv
    import glob

    def per_kernel(d):
        files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        vals = {}
        for f in files:
            for r in csv.DictReader(open(f)):
                # "void air::k_x<...>(args)" -> "air::k_x<...>"
                name = r["Kernel_Name"].split("(")[0].strip()
                name = name[5:] if name.startswith("void ") else name
                vals.setdefault(name, []).append(float(r["Counter_Value"]))
        return vals

    fetch, write = per_kernel(fetch_dir), per_kernel(write_dir)
    copy_bytes = 256 * 1024 * 1024
    cf = max(fetch.get("__amd_rocclr_copyBuffer", [0.0]))
    cw = max(write.get("__amd_rocclr_copyBuffer", [0.0]))
    sf = copy_bytes / (cf * 1024.0) if cf else None
    sw = copy_bytes / (cw * 1024.0) if cw else None
    out = {"batch": batch, "source_hash": kernel_source_hash(), "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_scale": sf, "write_scale": sw, "kernels": {}}
    for name in sorted(set(fetch) & set(write)):
        if not name.startswith("air::") or not sf or not sw:
            continue
        fk, wk = fetch[name], write[name]
        fb = sum(fk) / len(fk) * 1024.0 * sf
        wb = sum(wk) / len(wk) * 1024.0 * sw
        out["kernels"][name] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                                "dispatches": len(fk)}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    json.dump(out, open(TRAFFIC_FILE, "w"), indent=1)
    print(json.dumps(out, indent=1))


def _csv_rows(d, suffix):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)):
        rows += list(csv.DictReader(open(f)))
    return rows


def _short(name: str) -> str:
    name = name.split("(")[0].strip()
    return name[5:] if name.startswith("void ") else name


def summarize_trace(d: str) -> str:
    """Markdown table of a kernel-trace statistics file (rocprofv3 --stats)."""
    rows = _csv_rows(d, "kernel_stats.csv")
    out = ["| kernel | calls | avg us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in rows[:16]:
        out.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def summarize_timeline(d: str) -> str:
    """Markdown summary of a rocprofv3 --kernel-trace output directory (the
    dispatch timeline): the GPU's busy fraction (union of the kernels' intervals
    over the traced span), the mean number of kernels running while busy, time
    per kernel, and the backprojector launches by group size and grid."""
    import collections
    rows = []
    for r in _csv_rows(d, "kernel_trace.csv"):
        if r.get("Kind", "KERNEL_DISPATCH") != "KERNEL_DISPATCH":
            continue
        grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), _short(r["Kernel_Name"]), grid))
    rows.sort()
    t0, t1 = rows[0][0], max(r[1] for r in rows)
    busy, cs, ce = 0, None, None
    for s, e, _, _ in rows:
        if ce is None or s > ce:
            if ce is not None:
                busy += ce - cs
            cs, ce = s, e
        else:
            ce = max(ce, e)
    busy += ce - cs
    total = sum(e - s for s, e, _, _ in rows)
    out = [f"{len(rows)} dispatches over {(t1 - t0) / 1e9:.2f} s; GPU busy (some kernel running) "
           f"{busy / (t1 - t0):.3f} of the span; {total / busy:.2f} kernels running on average while busy.", "",
           "| kernel | calls | total s | avg us | share of kernel time |", "|---|---|---|---|---|"]
    by = collections.defaultdict(lambda: [0, 0])
    for s, e, n, _ in rows:
        by[n][0] += 1
        by[n][1] += e - s
    for n, (c, t) in sorted(by.items(), key=lambda x: -x[1][1])[:20]:
        out.append(f"| `{n}` | {c} | {t / 1e9:.3f} | {t / c / 1e3:.1f} | {t / total:.3f} |")
    bp = collections.defaultdict(lambda: [0, 0])
    for s, e, n, g in rows:
        if n.startswith("air::k_backproject<"):
            bp[(n, g)][0] += 1
            bp[(n, g)][1] += e - s
    out += ["", "| backprojector launch | work-items | calls | avg us |", "|---|---|---|---|"]
    for (n, g), (c, t) in sorted(bp.items(), key=lambda x: -x[1][1])[:16]:
        out.append(f"| `{n}` | {g} | {c} | {t / c / 1e3:.1f} |")
    return "\n".join(out)


def summarize_counters(dirs, batch: int) -> str:
    """Per-dispatch counter averages of the projector, backprojector and ramp
    kernels over several rocprofv3 --pmc directories (one counter set each),
    with the rates derived from them: VALU busy = SQ_ACTIVE_INST_VALU (quad
    cycles, summed over the 1024 SIMDs) x 4 / (1024 x kernel cycles), kernel
    cycles = GRBM_GUI_ACTIVE / 8 (summed over the eight XCDs); VALU lane
    operations per useful FMA = 64 SQ_INSTS_VALU / (2 samples x images)."""
    import collections
    import synth
    from paper_1310_1434_amd import air
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    meta = {}
    for d in dirs:
        for r in _csv_rows(d, "counter_collection.csv"):
            name = _short(r["Kernel_Name"])
            if not name.startswith(("air::k_backproject", "air::k_project", "air::k_ramp")):
                continue
            vals[name][r["Counter_Name"]].append(float(r["Counter_Value"]))
            meta[name] = (r.get("LDS_Block_Size"), r.get("Grid_Size"), r.get("Workgroup_Size"))
    w = synth.workload("c2")
    _, lo, hi = air.host_tables(w.geom)
    samples = int(np.maximum(hi - lo + 1, 0).sum())
    # the projectors of a run work on the same sub-batches as its backprojector groups
    groups = [int(n.split("<")[1].split(",")[2]) for n in vals if n.startswith("air::k_backproject<")]
    proj_imgs = max(groups) if groups else (batch // 2 if batch >= 8 else batch)
    out = []
    for name in sorted(vals):
        c = {k: sum(v) / len(v) for k, v in vals[name].items()}
        lds, grid, wg = meta[name]
        out.append(f"**`{name}`** (LDS bytes {lds}, grid {grid} work-items in groups of {wg})\n")
        out.append("| counter | per dispatch |")
        out.append("|---|---|")
        for k in sorted(c):
            out.append(f"| {k} | {c[k]:.4g} |")
        cyc = c.get("GRBM_GUI_ACTIVE", 0) / 8.0
        if cyc and "SQ_ACTIVE_INST_VALU" in c:
            out.append(f"| *VALU busy (derived)* | {c['SQ_ACTIVE_INST_VALU'] * 4 / (1024 * cyc):.2f} |")
        if "k_backproject" in name or "k_project" in name:
            imgs = int(name.split("<")[1].split(",")[2]) if "k_backproject" in name else proj_imgs
            fma = 2.0 * samples * imgs
            if "SQ_INSTS_VALU" in c:
                out.append(f"| *VALU lane operations per useful FMA (derived, {imgs} images, {samples} samples "
                           f"per image)* | {64 * c['SQ_INSTS_VALU'] / fma:.2f} |")
        out.append("")
    return "\n".join(out)


def serving_workload(n_requests: int, rate: float, seed: int = 0):
    """The serving mix: image size uniform over {256, 512, 768} (0.78 mm pixels,
    1.4375 n bins of 1.2 mm), views uniform over {180, 360, 720, 1440} over 2 pi,
    100% or 25% of them, I0 ~ U[1e4, 1e5], Bregman iterations uniform in [20, 50],
    Poisson arrivals.  One 20-ellipse phantom per (size, views) scan (its exact
    line integrals computed once); each request draws its own Poisson noise."""
    import synth
    from synth.configs import Workload, serving_geometry
    from synth.phantom import draw_phantom, line_integrals
    from paper_1310_1434_amd.serve import Request, poisson_arrivals

    rng = np.random.default_rng(seed)
    arrivals = poisson_arrivals(rate, n_requests, seed)
    scans = {}
    reqs = []
    for i in range(n_requests):
        n = int(rng.choice([256, 512, 768]))
        views = int(rng.choice([180, 360, 720, 1440]))
        step = int(rng.choice([1, 4]))
        i0 = float(rng.uniform(1e4, 1e5))
        n_outer = int(rng.integers(20, 51))
        if (n, views) not in scans:
            full = serving_geometry(n, views)
            w = Workload(f"serve_{n}_{views}", full, disk_radius=190.0 * n / 512.0, n_ellipses=20, i0=i0)
            ell = draw_phantom(np.random.default_rng(1000 + len(scans)), w)
            scans[(n, views)] = line_integrals(ell, full)
        p = scans[(n, views)][::step]
        y = synth.noisy_sinogram(rng, p, i0).astype(np.float32)
        reqs.append(Request(i, serving_geometry(n, views, step), np.ascontiguousarray(y), n_outer,
                            arrival=float(arrivals[i])))
    return reqs



def serve_run(torch, reqs, precision, rate, base_rate, capacity, warmup, max_active=None):
    """Serve `reqs`, generated at base_rate requests/s, at `rate` (arrival times
    scaled by base_rate / rate) on a fresh executor; latency figures leave out
    the first `warmup` requests."""
    from paper_1310_1434_amd.serve import GpuExecutor, Server, geometry_key, latency_stats

    reqs = [copy.copy(r) for r in reqs]
    for r in reqs:
        r.arrival = r.arrival * base_rate / rate if rate else 0.0      # rate 0: all at once
    ex = GpuExecutor(lam=0.005, mu=1.0, n_cg=5, max_outer=50, capacity=capacity, precision=precision)
    for r in reqs:                    # ray tables are built before the clock starts
        ex.plan(geometry_key(r.geom), r.geom)
    torch.cuda.synchronize()
    free, _ = torch.cuda.mem_get_info()
    srv = Server(ex, int(0.8 * free) + ex.resident_bytes(), capacity, max_active=max_active)
    t = time.perf_counter()
    done = srv.run(reqs)
    wall = time.perf_counter() - t
    ok = [r for r in done if r.error is None]
    measured = [r for r in done if r.rid >= warmup]
    st = latency_stats(measured)
    # queue build-up: mean latency of the last third of the measured requests
    # (by arrival) over that of the first third; about 1 when the rate is served
    lat = [r.latency for r in sorted(measured, key=lambda r: r.arrival) if r.latency is not None]
    k = max(len(lat) // 3, 1)
    growth = float(np.mean(lat[-k:]) / np.mean(lat[:k])) if len(lat) >= 3 else None
    out = {"precision": precision, "requests": len(reqs), "warmup_requests": warmup,
           "offered_rate_per_s": rate, "completed": len(ok),
           "failed": len(done) - len(ok), "recon_per_s": len(ok) / wall, "wall_s": wall,
           "p50_s": st.get("p50_s"), "p99_s": st.get("p99_s"), "max_s": st.get("max_s"),
           "latency_growth": growth, "geometry_groups": len({geometry_key(r.geom) for r in reqs}), "slots_per_group": capacity,
           "max_active_groups": max_active, "steps": srv.steps}
    del srv, ex
    torch.cuda.synchronize()
    return out


def serve_leg(torch, a):
    """The serving mix at 40 requests/s on both paths, then the mixed path at 20
    and 30 requests/s on the first 150 requests, and the same 150 requests all
    at once: the rate at which that backlog drains is the server's capacity
    for this mix, and Poisson arrivals are stable at any rate below it.  Each
    run also reports its latency trend (mean latency of the last third of the
    requests over the first third: about 1 while arrivals are served, growing
    beyond capacity; noisy on short streams whose request mix drifts)."""
    reqs = serving_workload(a.serve_requests, a.serve_rate)
    print(f"bench: serving leg, {len(reqs)} requests", file=sys.stderr, flush=True)
    k = a.serve_max_active or None
    out = {"workload": f"{len(reqs)} requests: n in {{256, 512, 768}}, views in {{180, 360, 720, 1440}}, "
                       "100% or 25%, I0 U[1e4, 1e5], 20-50 Bregman x 5 CG, Poisson arrivals",
           "stable_if": "offered rate below the capacity (capacity_mixed: a 150-request backlog's drain rate)",
           "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"), "max_active_groups": k}
    for prec in ("fp32", "mixed_f16"):
        out[prec] = serve_run(torch, reqs, prec, a.serve_rate, a.serve_rate, a.serve_capacity, a.serve_warmup, k)
    sweep = []
    for rate in (20.0, 30.0):
        sub = reqs[:150]
        sweep.append(serve_run(torch, sub, "mixed_f16", rate, a.serve_rate, a.serve_capacity, 15, k))
    sweep.append(out["mixed_f16"])
    out["rate_sweep_mixed"] = [{k: s[k] for k in ("offered_rate_per_s", "recon_per_s", "p50_s", "p99_s",
                                                  "latency_growth")} for s in sweep]
    burst = serve_run(torch, reqs[:150], "mixed_f16", 0.0, a.serve_rate, a.serve_capacity, 0, k)
    out["capacity_mixed"] = {"requests": burst["requests"], "recon_per_s": burst["recon_per_s"],
                             "wall_s": burst["wall_s"], "note": "all requests arrive at once"}
    out["max_stable_rate_per_s"] = burst["recon_per_s"]
    out["stable_at_40_per_s"] = burst["recon_per_s"] > a.serve_rate
    return out


def c5_leg(torch, air, batch: int = 16):
    """1024^2 fan beam, 2304 views x 1536 bins, a batch of 16 (one seeded case
    replicated; the kernels' work does not depend on the values): solves of 1
    and 2 Bregman iterations on each path (two sub-batch streams, as timed for
    C2) give the time per iteration, from which a 50-iteration solve is
    extrapolated; plus the kernels of one iteration, alone and in the two-stream
    configuration, and the dominant kernel's roofline."""
    import synth
    w = synth.workload("c5")
    y1 = synth.make_case(w, 0)["y"].astype(np.float32)
    y = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(y1, (batch,) + y1.shape))).cuda()
    out = {"workload": w.name, "batch": batch, "n": w.geom.n, "views": w.geom.n_views, "bins": w.geom.n_bins,
           "n_outer": w.n_outer, "n_cg": w.n_cg}
    for prec in ("fp32", "mixed_f16"):
        plan = air.Plan(w.geom, max_batch=batch, precision=prec)
        ws = torch.empty(plan.solve_workspace_bytes(batch), dtype=torch.uint8, device="cuda")
        t = {}
        for k in (1, 2, 1, 2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.solve(y, w.lam, w.mu, k, w.n_cg, workspace=ws, with_resid=False)
            torch.cuda.synchronize()
            t[k] = time.perf_counter() - t0          # (the second of each pair: warm)
        per_outer = t[2] - t[1]
        setup = t[1] - per_outer
        full = setup + w.n_outer * per_outer
        r = {"s_per_outer_iteration": per_outer, "setup_s": setup, "recon_per_s_extrapolated": batch / full,
             "extrapolated": f"a {w.n_outer}-iteration solve from timed solves of 1 and 2 iterations"}
        if prec == "fp32":
            rsteps = ray_steps(plan)
            km = instrumented(torch, air, plan, y, w, ws, "on", 1)
            kma = instrumented(torch, air, plan, y, w, ws, "one_stream", 1)
            r["kernel_ms"] = {k: {"avg_ms": v["avg_ms"], "launches": v["launches"]} for k, v in km.items()}
            r["roofline"] = roofline(km, w.geom, batch, 1, w.n_cg, rsteps, prec, "two sub-batch streams")
            r["roofline_alone"] = roofline(kma, w.geom, batch, 1, w.n_cg, rsteps, prec, "every kernel alone")
        out[prec] = r
        del plan, ws
        torch.cuda.synchronize()
    return out


def c3_gemm_bench(a):
    """The ramp GEMM alone at the C3 measurement shape: a 736 x 736 Toeplitz filter
    times 11,520 sinogram rows (180 views x 64 images of the 512^2 fan geometry's
    detector), in each precision, timed with HIP events over many launches."""
    import torch
    import synth
    from paper_1310_1434_amd import air

    g = synth.workload("c2_25").geom
    rows_imgs = 64
    y = torch.rand((rows_imgs, g.n_views, g.n_bins), device="cuda")
    out = {"workload": "c3_ramp_gemm_736x736_x_11520", "shape": [rows_imgs * g.n_views, g.n_bins, g.n_bins]}
    for prec in ("fp32", "mixed_f16", "mixed_bf16"):
        plan = air.Plan(g, max_batch=rows_imgs, precision=prec)
        yf = plan.ramp(y)
        torch.cuda.synchronize()
        plan.kernel_timing("on")
        for _ in range(20):
            plan.ramp(y, out=yf)
        torch.cuda.synchronize()
        kt = plan.collect_kernel_timing()
        plan.kernel_timing("off")
        ms = kt["ramp"][0] / kt["ramp"][1]
        terms = {"fp32": 1, "mixed_f16": 3, "mixed_bf16": 6}[prec]
        flops = 2.0 * rows_imgs * g.n_views * g.n_bins * g.n_bins
        peak = MFMA_PEAK_TFLOPS[prec]
        out[prec] = {"avg_launch_ms": ms, "achieved_tflops": flops / (ms * 1e-3) / 1e12,
                     "achieved_tflops_all_terms": terms * flops / (ms * 1e-3) / 1e12, "peak_tflops": peak,
                     "frac": flops / (ms * 1e-3) / 1e12 / peak,
                     "frac_all_terms": terms * flops / (ms * 1e-3) / 1e12 / peak, "products": terms}
    return out


def quality_bench(a):
    """FBP, IR and AIR on the resolution and contrast phantoms, 100% and 25% data
    of the paper-shaped scan (350^2, 528 bins, 800 / 200 views), 50 x 5 iterations."""
    import torch
    from paper_1310_1434_amd import air
    from paper_1310_1434_amd import quality as Q
    from synth import quality as SQ

    lam, mu, n_outer, n_cg = 0.005, 1.0, 50, 5
    phantoms = [SQ.resolution_phantom(), SQ.contrast_phantom()]
    out = {"geometry": "fan 350^2 x 1 mm, 528 bins x 1.1 mm, SOD 850, SDD 1450", "i0": a.quality_i0,
           "lambda": lam, "mu": mu, "n_outer": n_outer, "n_cg": n_cg, "data": {}}
    for label, step in (("100%", 1), ("25%", 4)):
        g = SQ.paper_geometry(step)
        cases = [SQ.make_quality_case(ph, g, a.quality_i0, 11 + k) for k, ph in enumerate(phantoms)]
        plan = air.Plan(g, max_batch=len(cases))
        s = Q.top_eigenvalue(plan, 0) / Q.top_eigenvalue(plan, 1)
        y = torch.from_numpy(np.stack([c["y"] for c in cases]).astype(np.float32)).cuda()
        torch.cuda.synchronize()
        t = time.perf_counter()
        arms = Q.run_arms(plan, y, lam, mu, n_outer, n_cg, s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        res = {"views": g.n_views, "ir_scale": s, "wall_s_all_arms": wall, "arms": {}}
        for arm, x in arms.items():
            imgs = x.cpu().numpy().astype(np.float64)
            r = {}
            for ph, img, c in zip(phantoms, imgs, cases):
                r["rmse_vs_truth"] = r.get("rmse_vs_truth", []) + [float(np.sqrt(np.mean((img - c["x_true"]) ** 2)))]
                if ph.bar_groups:
                    r["fwhm"] = [Q.bar_fwhm(img, gr, g.pixel) for gr in ph.bar_groups]
                else:
                    r["cnr"] = Q.target_cnrs(img, ph, g.pixel)
            res["arms"][arm] = r
        out["data"][label] = res
    return out



def c2_leg(torch, air, w, B, steps, warmup, precisions, golden):
    """Timed solves of B cases of workload w in each precision; image 0 (seed 0)
    of the last step against the stored oracle image."""
    import synth
    ys = np.stack([synth.make_case(w, s)["y"] for s in range(B)]).astype(np.float32)
    y = torch.from_numpy(ys).cuda()
    ref = golden_image(golden)
    res = {}
    plans = {}
    for prec in precisions:
        plan = air.Plan(w.geom, max_batch=B, precision=prec)
        ws = torch.empty(plan.solve_workspace_bytes(B), dtype=torch.uint8, device="cuda")
        wall, lat, x = timed_steps(torch, plan, y, w, steps, warmup, ws)
        r = {"value": B * steps / wall, "ms_per_step": 1e3 * wall / steps,
             "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99))}
        if ref is not None:
            r["rel_l2_vs_oracle"] = rel_l2(x[0].cpu().numpy(), ref)
        res[prec] = r
        plans[prec] = (plan, ws)
    return res, plans, y, ys


def main():
    a = parse()
    # HIP maps streams onto GPU_MAX_HW_QUEUES hardware queues (4 by default):
    # the serving leg runs one stream per geometry group, and groups whose
    # streams share a queue cannot overlap.  HIP reads it when it initialises,
    # so it is set here, before anything imports torch.
    if not 0 <= a.hw_queues <= 32:
        print("bench.py: --hw-queues takes 1 to 32 (0 keeps the environment's value)", file=sys.stderr)
        sys.exit(2)
    if a.hw_queues:
        os.environ["GPU_MAX_HW_QUEUES"] = str(a.hw_queues)
    if a.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {a.gpus} is not supported (independent reconstructions "
              "shard across GPUs with no communication; this build runs on one GPU)", file=sys.stderr)
        sys.exit(2)
    if a.summarize_pmc:
        summarize_pmc(a.summarize_pmc[0], a.summarize_pmc[1], a.batch)
        return
    if a.summarize_trace:
        print(summarize_trace(a.summarize_trace))
        return
    if a.summarize_timeline:
        print(summarize_timeline(a.summarize_timeline))
        return
    if a.summarize_counters:
        print(summarize_counters(a.summarize_counters, a.batch))
        return
    if a.quality:
        print(json.dumps({"quality": quality_bench(a)}), flush=True)
        return
    if a.workload == "c3_gemm":
        print(json.dumps({"c3_gemm": c3_gemm_bench(a)}), flush=True)
        return
    import torch
    import synth
    from paper_1310_1434_amd import air
    if a.serve:
        print(json.dumps({"served": serve_leg(torch, a)}), flush=True)
        return

    w = synth.workload(a.workload)
    B = a.batch
    g = w.geom
    golden = {"c2": "c2_fan_512_720_seed0", "c2_25": "c2_fan_512_180_seed0"}.get(a.workload, "")
    precisions = ["fp32"] + ([] if a.no_mixed else ["mixed_f16"])
    out = {"metric": "recon/s + p99 latency, 512^2x720-view AIR, mixed vs FP32; proj GRays/s",
           "unit": "recon/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded ellipse phantoms, exact line integrals, Poisson noise)",
           "config": {"workload": w.name, "beam": g.beam, "n": g.n, "views": g.n_views, "bins": g.n_bins,
                      "batch": B, "n_outer": w.n_outer, "n_cg": w.n_cg, "lambda": w.lam, "mu": w.mu,
                      "precision": "fp32"}}
    if a.kernel_timing_only:
        ys = np.stack([synth.make_case(w, s)["y"] for s in range(B)]).astype(np.float32)
        y = torch.from_numpy(ys).cuda()
        plans = {}
        for prec in precisions:
            plan = air.Plan(g, max_batch=B, precision=prec)
            plans[prec] = (plan, torch.empty(plan.solve_workspace_bytes(B), dtype=torch.uint8, device="cuda"))
    else:
        res, plans, y, ys = c2_leg(torch, air, w, B, a.steps, a.warmup, precisions, golden)
        f = res["fp32"]
        out.update({"value": f["value"], "ms_per_step": f["ms_per_step"], "p50_ms": f["p50_ms"],
                    "p99_ms": f["p99_ms"]})
        out["rel_l2_vs_oracle"] = {p: res[p].get("rel_l2_vs_oracle") for p in precisions}
        out["rel_l2_vs_oracle"]["reference"] = (f"image 0 (seed 0) of the last timed step against the FP64 oracle's "
                                                f"reconstruction tests/golden/{golden}.npz" if golden else None)
        if "mixed_f16" in res:
            out["mixed"] = dict(precision="mixed_f16 (ramp as f16 hi/lo MFMA, float16 image copies in the forward "
                                          "projector)", **res["mixed_f16"])
        if a.workload == "c2" and not a.no_quarter:
            w25 = synth.workload("c2_25")
            r25, _, _, _ = c2_leg(torch, air, w25, B, a.steps, min(a.warmup, 2), precisions, "c2_fan_512_180_seed0")
            out["c2_25"] = {"workload": w25.name, "views": w25.geom.n_views, "batch": B, **r25}
            torch.cuda.synchronize()

    # instrumented passes: every kernel bracketed by HIP events on its launch stream
    n_outer = a.outer if (a.kernel_timing_only and a.outer > 0) else w.n_outer
    plan, ws = plans["fp32"]
    rsteps = ray_steps(plan)
    mode = "one_stream" if a.one_stream else "on"
    km = instrumented(torch, air, plan, y, w, ws, mode, n_outer)
    out["kernel_ms"] = km
    out["kernel_ms_config"] = ("every kernel alone (one stream)" if a.one_stream else
                               "as timed: a batch of 8 or more runs as two sub-batches on two streams")
    out["roofline"] = roofline(km, g, B, n_outer, w.n_cg, rsteps, "fp32", out["kernel_ms_config"])
    if not a.one_stream and not a.kernel_timing_only:
        kma = instrumented(torch, air, plan, y, w, ws, "one_stream", n_outer)
        out["kernel_ms_alone"] = kma
        out["roofline_alone"] = roofline(kma, g, B, n_outer, w.n_cg, rsteps, "fp32", "every kernel alone")
    if "mixed_f16" in plans:
        mp, mws = plans["mixed_f16"]
        out["mixed_kernel_ms"] = instrumented(torch, air, mp, y, w, mws, mode, n_outer)
    if a.kernel_timing_only:
        for key in ("kernel_ms", "mixed_kernel_ms"):
            if key in out:
                tot = sum(v["total_ms"] for v in out[key].values())
                out[key.replace("kernel_ms", "gpu_ms_per_outer_iteration")] = tot / max(n_outer, 1)
    # the roofline kernel's HBM traffic from the committed counter summary
    inst = None
    roof = out["roofline"]
    if roof["kernel"] == "k_backproject":
        bt = image_group(int(round(roof["images_per_launch"])))
        inst = f"air::k_backproject<1, true, {bt}, 2, {1 if g.beam == 'fan' else 0}>"
    elif roof["kernel"] == "k_project":
        inst = f"air::k_project<{2 if roof['images_per_launch'] >= 2 else 1}>"
    roof["traffic"] = traffic_for(inst, B) if inst else None
    roof["traffic_kernel"] = inst
    rays_launch = g.n_views * g.n_bins
    for kind, key in (("project", "proj_grays_s"), ("backproject", "backproj_grays_s")):
        k = km[kind]
        ipl = B * operator_applies(kind, n_outer, w.n_cg) / k["launches"] if k["launches"] else 0
        out[key] = ipl * rays_launch / (k["avg_ms"] * 1e-3) / 1e9 if k["avg_ms"] else None
    out["grays_note"] = "rays per launch / launch duration in the instrumented solve (kernel_ms_config)"
    out["kernel_source_hash"] = kernel_source_hash()

    if a.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * 4
    del plans
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if a.workload == "c2" and not a.kernel_timing_only:
        print("bench: C5 and C3 ramp-GEMM legs", file=sys.stderr, flush=True)
        out["c5"] = c5_leg(torch, air)
        out["c3_ramp_gemm"] = c3_gemm_bench(a)
        torch.cuda.empty_cache()
    if a.workload == "c2" and not (a.no_serve or a.kernel_timing_only):
        out["served"] = serve_leg(torch, a)
    if not (a.no_cpu_baseline or a.kernel_timing_only):
        out["cpu_baseline"] = cpu_baseline(w, ys[0])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
