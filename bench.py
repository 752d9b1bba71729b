"""Benchmark: null-collision path tracing of the broken-cumulus field on one MI355X.

One step = build the hierarchical majorant grid over the 512x512x160 field
(25 m cells) and render the 1024x1024 oblique view at 64 samples per pixel
(backward paths with the sun's local estimate).  Inputs are resident in HBM
before timing starts.  Prints one JSON line.
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

METRIC = "paths/s + time to 1% rel. std err radiance, plain vs guided, 1 MI355X"
HBM_PEAK_GBS = 8000.0
GRANULE = 64  # bytes moved by one random 4- or 8-byte read from HBM
PHASES = ("cross", "collide", "event", "ray", "sample")


def kernel_sources_digest():
    """SHA-256 over the HIP sources: measured HBM traffic is only reported for the build it was measured on."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1902_01137_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per render launch from the committed rocprofv3 counter runs, or None if stale."""
    path = os.path.join(ROOT, "profiles", "render_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    return rec["bytes_per_launch"] if rec.get("sources_sha256") == kernel_sources_digest() else None


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", choices=["cumulus", "small"], default="cumulus")
    p.add_argument("--spp", type=int, default=None)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--block", type=int, default=0, help="launch knob (0: library default)")
    p.add_argument("--waves-per-cu", type=int, default=0, help="launch knob (0: library default)")
    p.add_argument("--spi", type=int, default=0, help="samples per queue item (0: library default)")
    p.add_argument("--lds-levels", type=int, default=-1, help="grid levels staged in LDS (-1: auto)")
    p.add_argument("--no-batch", action="store_true", help="skip the 48-view x 4-sun batched launch")
    p.add_argument("--batch-spp", type=int, default=4)
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1902_01137_amd import api, inputs

    if args.workload == "cumulus":
        sc = inputs.scene_cumulus()
        name = "cumulus_512x512x160_25m_view1024x1024"
    else:
        sc = inputs.scene_small()
        name = "blob_32x32x32_100m_nadir64x64"
    spp = args.spp or sc.sampling.spp
    cam = sc.camera
    npix = cam.width * cam.height
    paths_per_step = npix * spp

    ctx = api.Context(0)
    ctx.set_launch(args.block, args.waves_per_cu, args.spi, args.lds_levels)
    kc = torch.from_numpy(sc.kc).cuda()
    torch.cuda.synchronize()
    cnt = api.new_counters("cuda")
    ev = []

    def step(i, counters=None):
        g = api.build_grid(ctx, kc, sc.desc, sc.grid)
        s = torch.zeros((cam.height, cam.width), dtype=torch.float64, device="cuda")
        s2 = torch.zeros_like(s)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        api.render(ctx, g, kc, sc.optics, cam, inputs.Sampling(seed=sc.sampling.seed + 7919 * i, spp=spp), s, s2,
                   counters)
        e1.record()
        ev.append((e0, e1))
        return g, s, s2

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    ev.clear()
    t0 = time.perf_counter()
    last = None
    for i in range(args.steps):
        last = step(args.warmup + i, cnt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    render_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    c = api.counters_dict(cnt)
    _, s, s2 = last
    sm = s.cpu().numpy().ravel() / spp
    var = np.maximum(s2.cpu().numpy().ravel() / spp - sm ** 2, 0) * spp / (spp - 1)
    se = np.sqrt(var / spp)
    eps = float(np.sqrt(np.mean(se ** 2)) / np.mean(sm))
    t_1pct = ms_step / 1e3 * (eps / 0.01) ** 2

    paths_s = paths_per_step / (ms_step / 1e3)
    gathers_per_launch = (c["gathers"] + c["node_reads"]) / args.steps
    achieved = gathers_per_launch * GRANULE / (render_ms / 1e3) / 1e9
    out = {
        "metric": METRIC,
        "value": paths_s,
        "unit": "paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": name, "spp": spp, "image": [cam.width, cam.height],
                   "field": [sc.desc.nx, sc.desc.ny, sc.desc.nz], "tau_tilde": sc.grid.tau_tilde,
                   "paths_per_step": paths_per_step},
        "render_ms": render_ms,
        "segments_per_s": c["segments"] / args.steps / (render_ms / 1e3),
        "tentative_per_s": c["tentative"] / args.steps / (render_ms / 1e3),
        "per_path": {k: c[k] / max(c["paths"], 1) for k in ("segments", "tentative", "nulls", "reals",
                                                            "leaf_visits", "gathers", "node_reads", "nee_rays")},
        "truncated": c["truncated"],
        "sched": {"trips": {k: c["trips_" + k] for k in PHASES},
                  "lanes_per_trip": {k: round(c["lanes_" + k] / max(c["trips_" + k], 1), 2) for k in PHASES},
                  "ticks_per_trip": {k: round(c["ticks_" + k] / max(c["trips_" + k], 1), 1) for k in PHASES}},
        "rel_std_err": eps,
        "time_to_1pct_s": {"plain": t_1pct, "guided": None},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if args.workload == "cumulus" and spp == 64 else None},
    }
    if args.workload == "cumulus" and not args.no_batch:
        out["batch"] = batch_run(ctx, sc, kc, args.batch_spp)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, spp, args.cpu_seconds)
    print(json.dumps(out))


def batch_run(ctx, sc, kc, spp):
    """48 views (256^2 .. 1024^2) x 4 sun zeniths of the same field in one persistent launch."""
    import torch

    from paper_1902_01137_amd import api, inputs
    g = api.build_grid(ctx, kc, sc.desc, sc.grid)
    views = inputs.batch_views()
    jobs = [(cam, inputs.Optics(**{**vars(sc.optics), "sun_zenith_deg": sz})) for cam, sz in views]
    px = sum(c.width * c.height for c, _ in jobs)
    smp = inputs.Sampling(seed=sc.sampling.seed + 17, spp=spp)
    api.render_batch(ctx, g, kc, jobs, smp)                       # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    api.render_batch(ctx, g, kc, jobs, inputs.Sampling(seed=sc.sampling.seed + 18, spp=spp))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"jobs": len(jobs), "pixels": px, "spp": spp, "paths": px * spp, "ms": dt * 1e3,
            "paths_per_s": px * spp / dt}


def cpu_baseline(sc, spp, budget_s):
    """The oracle on a bounded sample of the same workload: pixels spread over
    the image (a strided subset), all spp samples each, one host core."""
    import oracle
    from paper_1902_01137_amd import inputs
    cam = sc.camera
    npix = cam.width * cam.height
    rng = np.random.default_rng(0)
    order = rng.permutation(npix).astype(np.int32)
    done, paths, t_used = 0, 0, 0.0
    chunk = 16
    while t_used < budget_s and done < npix:
        px = order[done:done + chunk]
        t0 = time.perf_counter()
        oracle.render(sc.desc, sc.kc, sc.grid.k_gas, sc.optics, cam, spp, inputs.SEED_ORACLE_BASE + 2, pixels=px)
        t_used += time.perf_counter() - t0
        done += len(px)
        paths += len(px) * spp
        chunk = min(chunk * 2, 1024)
    return {"value": paths / t_used, "unit": "paths/s", "cores": 1, "kind": "oracle",
            "sample": "%d random pixels x %d spp of the same image (%d paths, %.1f s)" % (done, spp, paths, t_used)}


if __name__ == "__main__":
    main()
