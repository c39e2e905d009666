"""Benchmark of the AIR reconstruction path on one MI355X.

A step is one full AIR reconstruction of a batch of independent 512 x 512
fan-beam cases (720 views x 736 bins, split Bregman 50 x 5 CG, the whole hot
path: Joseph projector, ramp GEMM, matched backprojector, CG updates,
framelet shrinkage), from the noisy sinograms already resident in HBM.

    python bench.py [--steps K] [--warmup W] [--batch B]

Prints one JSON line: recon/s (float32 path) with p50/p99 step latency, the
same for the mixed-precision ramp, projector GRays/s, the roofline position of
the dominant kernel (HIP-event timing inside this run) and the FP64 CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
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
# VALU issue peak: 256 CUs x 4 SIMD x 32 lanes per clock x 2.4 GHz (non-packed lane
# operations; a wave64 float32 operation issues in two cycles, so the published
# float32 vector rate, 157.3 TFLOP/s, is 78.6 T fused multiply-adds per second)
VALU_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
# essential VALU lane operations of one Joseph sample (ray-step): advance the
# fixed-point intercept, convert its fraction, form the two weights, form the
# sample address, two fused multiply-adds
VALU_OPS_PER_SAMPLE = 7
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_c2.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c2_25", "c5"])
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-timing-only", action="store_true",
                    help="skip the timed steps; run only the instrumented pass (for profiler runs)")
    ap.add_argument("--outer", type=int, default=0,
                    help="profiler runs only: Bregman iterations of the instrumented pass (0 = the workload's)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="profiler runs only: also run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--serve", action="store_true",
                    help="run the continuous-batching serving benchmark instead (Poisson arrivals, mixed geometries)")
    ap.add_argument("--serve-requests", type=int, default=120)
    ap.add_argument("--serve-rate", type=float, default=40.0, help="offered load, requests per second")
    ap.add_argument("--serve-capacity", type=int, default=8, help="slots per geometry group")
    ap.add_argument("--serve-precision", default="mixed_f16", choices=["fp32", "mixed_f16", "mixed_bf16"])
    ap.add_argument("--quality", action="store_true",
                    help="run the FBP / IR / AIR image-quality comparison (CNR, FWHM) on the paper-shaped scan")
    ap.add_argument("--quality-i0", type=float, default=2e4, help="incident photons per ray of the quality scans")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) into profiles/traffic_c2.json")
    return ap.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1310_1434_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".cuh", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def timed_steps(torch, plan, y, w, steps, warmup, ws):
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        plan.solve(y, w.lam, w.mu, w.n_outer, w.n_cg, workspace=ws, with_resid=False)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for k in range(steps):
        plan.solve(y, w.lam, w.mu, w.n_outer, w.n_cg, workspace=ws, with_resid=False)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    return wall, lat


def ray_steps(plan) -> int:
    _, lo, hi = plan.tables()
    return int(np.maximum(hi - lo + 1, 0).sum())


def cpu_baseline(w, y0):
    """FP64 oracle on 2 of the 50 Bregman iterations of one case, scaled to a full solve."""
    import oracle
    oracle.build(force=False)
    g = oracle.Geom(w.geom)
    k = 2
    t = time.perf_counter()
    oracle.solve(g, y0.astype(np.float64), w.lam, w.mu, k, w.n_cg)
    dt = time.perf_counter() - t
    per_recon = dt * w.n_outer / k
    return {"value": 1.0 / per_recon, "unit": "recon/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"FP64 oracle, {k} of {w.n_outer} Bregman iterations (x{w.n_cg} CG) of one "
                      f"{w.geom.n}^2 x {w.geom.n_views}-view case in {dt:.2f} s, scaled x{w.n_outer // k}"}


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
                name = r["Kernel_Name"]
                vals.setdefault(name, []).append(float(r["Counter_Value"]))
        return vals

    fetch, write = per_kernel(fetch_dir), per_kernel(write_dir)
    copy_bytes = 256 * 1024 * 1024
    cf = max(fetch.get("__amd_rocclr_copyBuffer", [0.0]))
    cw = max(write.get("__amd_rocclr_copyBuffer", [0.0]))
    sf = copy_bytes / (cf * 1024.0) if cf else None
    sw = copy_bytes / (cw * 1024.0) if cw else None
    names = {"k_project": "air::k_project<2>", "k_backproject": "air::k_backproject<1, true",
             "k_ramp_f32": "air::k_ramp_f32<2>"}
    out = {"batch": batch, "source_hash": kernel_source_hash(), "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_scale": sf, "write_scale": sw, "kernels": {}}
    for short, prefix in names.items():
        fk = [v for k, vs in fetch.items() if k.startswith(prefix) or prefix in k for v in vs]
        wk = [v for k, vs in write.items() if k.startswith(prefix) or prefix in k for v in vs]
        if fk and wk and sf and sw:
            fb = sum(fk) / len(fk) * 1024.0 * sf
            wb = sum(wk) / len(wk) * 1024.0 * sw
            out["kernels"][short] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                                     "dispatches": len(fk)}
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    json.dump(out, open(TRAFFIC_FILE, "w"), indent=1)
    print(json.dumps(out, indent=1))


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


def serve_bench(a):
    import torch
    from paper_1310_1434_amd.serve import GpuExecutor, Server, geometry_key, latency_stats

    reqs = serving_workload(a.serve_requests, a.serve_rate)
    ex = GpuExecutor(lam=0.005, mu=1.0, n_cg=5, max_outer=50, capacity=a.serve_capacity,
                     precision=a.serve_precision)
    for r in reqs:                    # ray tables are built before the clock starts
        ex.plan(geometry_key(r.geom), r.geom)
    free, _ = torch.cuda.mem_get_info()
    srv = Server(ex, int(0.8 * free), a.serve_capacity)
    t = time.perf_counter()
    done = srv.run(reqs)
    wall = time.perf_counter() - t
    ok = [r for r in done if r.error is None]
    st = latency_stats(done)
    return {"requests": len(reqs), "offered_rate_per_s": a.serve_rate, "completed": len(ok),
            "failed": len(done) - len(ok), "recon_per_s": len(ok) / wall, "wall_s": wall,
            "p50_latency_s": st.get("p50_s"), "p99_latency_s": st.get("p99_s"), "max_latency_s": st.get("max_s"),
            "geometry_groups": len({geometry_key(r.geom) for r in reqs}), "slots_per_group": a.serve_capacity,
            "precision": a.serve_precision, "steps": srv.steps,
            "mean_bregman_iterations": float(np.mean([r.n_outer for r in reqs]))}


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


def main():
    a = parse()
    if a.quality:
        if a.gpus != 1:
            print("bench.py: one GPU only", file=sys.stderr)
            sys.exit(2)
        print(json.dumps({"quality": quality_bench(a)}), flush=True)
        return
    if a.serve:
        if a.gpus != 1:
            print("bench.py: one GPU only", file=sys.stderr)
            sys.exit(2)
        print(json.dumps({"serving": serve_bench(a)}), flush=True)
        return
    if a.summarize_pmc:
        summarize_pmc(a.summarize_pmc[0], a.summarize_pmc[1], a.batch)
        return
    if a.gpus != 1:
        print(f"bench.py: measures one GPU; --gpus {a.gpus} is not supported "
              "(independent reconstructions shard across GPUs with no communication)", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_1310_1434_amd import air

    w = synth.workload(a.workload)
    B = a.batch
    ys = np.stack([synth.make_case(w, s)["y"] for s in range(B)]).astype(np.float32)
    y = torch.from_numpy(ys).cuda()
    g = w.geom
    plan = air.Plan(g, max_batch=B, precision="fp32")
    ws = torch.empty(plan.solve_workspace_bytes(B), dtype=torch.uint8, device="cuda")
    rsteps = ray_steps(plan)

    out = {"metric": "recon/s + p99 latency, 512^2x720-view AIR, mixed vs FP32; proj GRays/s",
           "unit": "recon/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded ellipse phantoms, exact line integrals, Poisson noise)",
           "config": {"workload": w.name, "beam": g.beam, "n": g.n, "views": g.n_views, "bins": g.n_bins,
                      "batch": B, "n_outer": w.n_outer, "n_cg": w.n_cg, "lambda": w.lam, "mu": w.mu,
                      "precision": "fp32"}}

    if not a.kernel_timing_only:
        wall, lat = timed_steps(torch, plan, y, w, a.steps, a.warmup, ws)
        out["value"] = B * a.steps / wall
        out["ms_per_step"] = 1e3 * wall / a.steps
        out["p50_ms"] = float(np.percentile(lat, 50))
        out["p99_ms"] = float(np.percentile(lat, 99))
        if not a.no_mixed:
            mp = air.Plan(g, max_batch=B, precision="mixed_f16")
            wall_m, lat_m = timed_steps(torch, mp, y, w, a.steps, a.warmup, ws)
            out["mixed"] = {"precision": "mixed_f16 (ramp as f16 hi/lo MFMA, float16 image copies in the forward projector)",
                            "value": B * a.steps / wall_m,
                            "ms_per_step": 1e3 * wall_m / a.steps, "p50_ms": float(np.percentile(lat_m, 50)),
                            "p99_ms": float(np.percentile(lat_m, 99))}
            del mp

    # instrumented pass: one more step with every kernel bracketed by HIP events
    n_outer = a.outer if (a.kernel_timing_only and a.outer > 0) else w.n_outer
    plan.kernel_timing(True)
    plan.solve(y, w.lam, w.mu, n_outer, w.n_cg, workspace=ws, with_resid=False)
    kt = plan.collect_kernel_timing()
    plan.kernel_timing(False)
    kernel_ms = {k: {"avg_ms": (v[0] / v[1]) if v[1] else 0.0, "launches": v[1], "total_ms": v[0]}
                 for k, v in kt.items()}
    out["kernel_ms"] = kernel_ms
    if a.kernel_timing_only and not a.no_mixed:
        # the same instrumented pass on the mixed path (large configurations, where a
        # full timed solve would take minutes, are reported per outer iteration)
        mp = air.Plan(g, max_batch=B, precision="mixed_f16")
        mp.kernel_timing(True)
        mp.solve(y, w.lam, w.mu, n_outer, w.n_cg, workspace=ws, with_resid=False)
        ktm = mp.collect_kernel_timing()
        mp.kernel_timing(False)
        out["mixed_kernel_ms"] = {k: {"avg_ms": (v[0] / v[1]) if v[1] else 0.0, "launches": v[1], "total_ms": v[0]}
                                  for k, v in ktm.items()}
        del mp
    if a.kernel_timing_only:
        for key in ("kernel_ms", "mixed_kernel_ms"):
            if key in out:
                tot = sum(v["total_ms"] for v in out[key].values())
                out[key.replace("kernel_ms", "gpu_ms_per_outer_iteration")] = tot / max(n_outer, 1)
    rays = B * g.n_views * g.n_bins
    t_proj = kernel_ms["project"]["avg_ms"] * 1e-3
    t_bp = kernel_ms["backproject"]["avg_ms"] * 1e-3
    out["proj_grays_s"] = rays / t_proj / 1e9 if t_proj else None
    out["backproj_grays_s"] = rays / t_bp / 1e9 if t_bp else None

    # Roofline of the dominant kernel.  The projectors' HBM traffic is small
    # (the images live in L2/MALL), so they are placed on the VALU issue
    # roofline: algorithmic work = VALU_OPS_PER_SAMPLE lane operations per
    # Joseph sample, ray-steps per image from the index tables.
    dom = max(("project", "backproject", "ramp"), key=lambda k: kernel_ms[k]["total_ms"])
    t_dom = kernel_ms[dom]["avg_ms"] * 1e-3
    if dom == "ramp":
        flops = 2.0 * B * g.n_views * g.n_bins * g.n_bins
        achieved = flops / t_dom / 1e12
        roof = {"kernel": "k_ramp_f32", "bound": "mfma", "achieved": achieved, "peak": MFMA_PEAK_TFLOPS["fp32"],
                "unit": "TFLOP/s", "frac": achieved / MFMA_PEAK_TFLOPS["fp32"]}
    else:
        ops = VALU_OPS_PER_SAMPLE * B * float(rsteps)
        achieved = ops / t_dom / 1e12
        roof = {"kernel": "k_project" if dom == "project" else "k_backproject", "bound": "alu",
                "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s (VALU lane ops)",
                "frac": achieved / VALU_PEAK_TOPS, "ops_per_launch": ops, "avg_launch_ms": t_dom * 1e3,
                "ray_steps_per_image": rsteps}
    roof["traffic"] = None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        ent = tr.get("kernels", {}).get(roof["kernel"])
        if ent and tr.get("source_hash") == kernel_source_hash() and tr.get("batch") == B:
            roof["traffic"] = ent["bytes_per_launch"]
    out["roofline"] = roof
    # the same kernels measured as an explicit sparse matrix would be (4 bytes per nonzero)
    out["sparse_equivalent_gbs"] = {
        "project": B * (8.0 * rsteps + 4.0 * g.n_views * g.n_bins) / t_proj / 1e9 if t_proj else None,
        "backproject": B * (8.0 * rsteps + 4.0 * g.n * g.n) / t_bp / 1e9 if t_bp else None}
    out["kernel_source_hash"] = kernel_source_hash()

    if a.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = src.numel() * 4
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, ys[0])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
