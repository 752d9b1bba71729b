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
MI355X_SIMDS = 256 * 4       # compute units x SIMDs per compute unit
MI355X_CLOCK_HZ = 2.4e9      # peak engine clock
PHASES = ("step", "collide", "event", "sample", "guide")   # step: voxel crossings and ray starts


def kernel_sources_digest():
    """SHA-256 over the HIP sources: measured HBM traffic is only reported for the build it was measured on."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1902_01137_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _profile_record():
    """The committed rocprofv3 record of the render kernel, or None if missing or measured on other sources."""
    path = os.path.join(ROOT, "profiles", "render_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    return rec if rec.get("sources_sha256") == kernel_sources_digest() else None


def measured_traffic():
    """HBM bytes per render launch from the committed rocprofv3 counter runs, or None if stale."""
    rec = _profile_record()
    return rec["bytes_per_launch"] if rec else None


def measured_valu_issue(render_ms):
    """VALU instruction rate of one render launch: SQ_INSTS_VALU of the committed counter run x 4 cycles
    (one wave64 instruction on a 16-lane SIMD) over SIMDs x 2.4 GHz x this run's kernel time.  A rate,
    not a bounded share (it exceeds 1 when instructions issue faster than one per 4 cycles on average).
    None if the record is stale or lacks it."""
    rec = _profile_record()
    if not rec or "sq_insts_valu" not in rec:
        return None
    return rec["sq_insts_valu"] * 4.0 / (MI355X_SIMDS * MI355X_CLOCK_HZ * render_ms / 1e3)


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
    p.add_argument("--no-guided", action="store_true", help="skip the guided leg (collect, train, guided render)")
    p.add_argument("--collect-spp", type=int, default=64, help="plain samples per pixel whose vertices train the guide")
    p.add_argument("--train-steps", type=int, default=80000, help="Adam steps of the single-view network")
    p.add_argument("--batch-train-steps", type=int, default=20000, help="Adam steps of each per-sun network of the batch")
    p.add_argument("--train-batch", type=int, default=131072,
                   help="records per Adam step of the single-view network (131072 at 80k steps: guided variance "
                        "0.346 of plain for 18.8 s of training, against 0.371 for 11.6 s at 65536)")
    p.add_argument("--batch-train-batch", type=int, default=65536, help="records per Adam step of each batch network")
    p.add_argument("--lr", type=float, default=3e-3, help="Adam step size at the start (cosine decay to 1 %% of it)")
    p.add_argument("--guide-frac", type=float, default=0.5, help="probability of sampling the guide at a scattering")
    p.add_argument("--guide-max-order", type=int, default=0, help="last guided scattering order (0: all)")
    p.add_argument("--no-variants", action="store_true", help="skip the grid variants (flat supercells, tau 0, global)")
    p.add_argument("--no-refinement", action="store_true", help="skip the refinement sweep (fields 128^2x40..1024^2x320)")
    p.add_argument("--no-progressive", action="store_true", help="skip the progressive runs to 1%% block error")
    p.add_argument("--max-spp", type=int, default=16384, help="cap of the progressive runs")
    p.add_argument("--no-ceiling", action="store_true", help="skip the random-read ceiling measurement")
    p.add_argument("--sun", choices=["delta", "ratio", "residual"], default="residual",
                   help="sun-ray transmissivity estimator (residual: decomposition tracking with the voxel minimum)")
    p.add_argument("--no-estimators", action="store_true", help="skip the comparison of sun-ray estimators")
    p.add_argument("--no-tau-sweep", action="store_true", help="skip the merge-threshold sweep")
    p.add_argument("--autotune", action="store_true", help="autotune the launch knobs before timing")
    p.add_argument("--no-flux", action="store_true", help="skip the forward-photon / adjoint timing (cylinder cumulus)")
    p.add_argument("--no-kdist", action="store_true", help="skip the k-distribution comparison (shared grid vs per point)")
    p.add_argument("--no-guide-kernels", action="store_true", help="skip the network training / inference timing")
    p.add_argument("--no-time-to-eps", action="store_true", help="skip the measured runs to 3%% per-pixel error")
    p.add_argument("--eps", type=float, default=0.03, help="target of the measured time-to-error runs")
    p.add_argument("--eps-rounds", action="store_true",
                   help="run the time-to-error legs as rounds of render calls sized from the error so far (a progress "
                        "line per round on stderr) instead of one progressive call")
    p.add_argument("--spread-renders", type=int, default=4,
                   help="independent renders whose spread checks the reported standard error")
    p.add_argument("--cpu-workers", type=int, default=0, help="oracle processes of the all-core baseline (0: host)")
    p.add_argument("--main-only", action="store_true", help="only the timed steps (for profiling runs)")
    a = p.parse_args()
    if a.main_only:
        a.no_cpu_baseline = a.no_batch = a.no_guided = a.no_variants = a.no_refinement = True
        a.no_progressive = a.no_ceiling = a.no_estimators = a.no_tau_sweep = True
        a.no_flux = a.no_guide_kernels = a.no_kdist = a.no_time_to_eps = True
    return a


FLAGS = 0   # sun-ray estimator of every render in the run (set from --sun)
T_START = time.perf_counter()


def note(leg):
    """One progress line on stderr per finished leg (the JSON line goes to stdout)."""
    print("bench: %s done at %.1f s" % (leg, time.perf_counter() - T_START), file=sys.stderr, flush=True)


def main():
    global FLAGS
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_1902_01137_amd import _lib, api, inputs

    FLAGS = {"delta": _lib.NC_SUN_DELTA, "ratio": _lib.NC_SUN_RATIO, "residual": _lib.NC_SUN_RESIDUAL}[args.sun]
    fine = None
    if args.workload == "cumulus":
        # the 12.5 m field (1024^2 x 320) is generated once; the workload field is its 2x2x2 regional average
        fine = inputs.cumulus_field(pool=1)
        sc = inputs.scene_cumulus(field=inputs.pool_field(*fine, 2))
        name = "cumulus_512x512x160_25m_view1024x1024"
        if args.no_refinement:
            fine = None
    else:
        sc = inputs.scene_small()
        name = "blob_32x32x32_100m_nadir64x64"
    spp = args.spp or sc.sampling.spp
    cam = sc.camera
    npix = cam.width * cam.height
    paths_per_step = npix * spp

    ctx = api.Context(0)
    ctx.set_launch(args.block, args.waves_per_cu, args.spi, args.lds_levels)
    tuned = None
    kc = torch.from_numpy(sc.kc).cuda()
    torch.cuda.synchronize()
    cnt = api.new_counters("cuda")
    ev = []

    # the grid's memory is allocated once; every step rebuilds it in place
    # over the field (as for a field that changes between renders), then renders
    g_step = api.build_grid(ctx, kc, sc.desc, sc.grid)

    def step(i, counters=None):
        g = g_step
        g.rebuild(kc)
        s = torch.zeros((cam.height, cam.width), dtype=torch.float64, device="cuda")
        s2 = torch.zeros_like(s)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        api.render(ctx, g, kc, sc.optics, cam, inputs.Sampling(seed=sc.sampling.seed + 7919 * i, spp=spp, flags=FLAGS),
                   s, s2,
                   counters)
        e1.record()
        ev.append((e0, e1))
        return g, s, s2

    if args.autotune and not args.main_only and not (args.block or args.waves_per_cu or args.spi):
        # launch knobs for this view (outside the timed region; the choice is reported)
        g0 = api.build_grid(ctx, kc, sc.desc, sc.grid)
        launch, best_ms = api.autotune_render(ctx, g0, kc, sc.optics, cam,
                                              inputs.Sampling(seed=sc.sampling.seed + 3, spp=spp, flags=FLAGS))
        tuned = {"launch": launch, "best_render_ms": best_ms}
        del g0
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    ev.clear()
    t0 = time.perf_counter()
    last = None
    for i in range(args.steps):
        last = step(args.warmup + i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    render_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    note("timed steps")
    # the event counts of one step, from a repeat of the last timed step (the
    # same seed traces the same paths) outside the timed region: the kernel
    # keeps no statistics unless counters are passed
    step(args.warmup + args.steps - 1, cnt)
    torch.cuda.synchronize()
    c = api.counters_dict(cnt)
    _, s, s2 = last
    sm = s.cpu().numpy().ravel() / spp
    var = np.maximum(s2.cpu().numpy().ravel() / spp - sm ** 2, 0) * spp / (spp - 1)
    se = np.sqrt(var / spp)
    eps = float(np.sqrt(np.mean(se ** 2)) / np.mean(sm))
    t_1pct = ms_step / 1e3 * (eps / 0.01) ** 2

    paths_s = paths_per_step / (ms_step / 1e3)
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
        "config": {"workload": name, "spp": spp, "image": [cam.width, cam.height], "sun_estimator": args.sun,
                   "field": [sc.desc.nx, sc.desc.ny, sc.desc.nz], "tau_tilde": sc.grid.tau_tilde,
                   "paths_per_step": paths_per_step},
        "render_ms": render_ms,
        "autotuned": tuned,
        "segments_per_s": c["segments"] / (render_ms / 1e3),
        "tentative_per_s": c["tentative"] / (render_ms / 1e3),
        "per_path": {k: c[k] / max(c["paths"], 1) for k in ("segments", "tentative", "nulls", "reals",
                                                            "leaf_visits", "deep_visits", "gathers", "node_reads",
                                                            "nee_rays")},
        "truncated": c["truncated"],
        "sched": {"trips": {k: c["trips_" + k] for k in PHASES},
                  "lanes_per_trip": {k: round(c["lanes_" + k] / max(c["trips_" + k], 1), 2) for k in PHASES},
                  "ticks_per_trip": {k: round(c["ticks_" + k] / max(c["trips_" + k], 1), 1) for k in PHASES}},
        "rel_std_err": eps,
    }
    roof = roofline(c, render_ms, spp == 64 and args.workload == "cumulus")
    gd = None
    tail = {}
    if not args.no_guided:
        tail["guided"], gd = guided_run(ctx, sc, kc, spp, args, build_ms=ms_step - render_ms,
                                        plain={"step_ms": ms_step, "render_ms": render_ms})
        note("guided")
    if not args.no_ceiling:
        out["gather_ceiling"] = gather_ceiling(ctx)
        note("gather_ceiling")
    if not args.no_progressive:
        out["progressive_block8"] = progressive_run(ctx, sc, kc, gd, args, tail.get("guided"))
        note("progressive")
    if not args.no_estimators:
        out["sun_estimators"] = estimator_run(ctx, sc, kc, spp, build_ms=ms_step - render_ms)
        note("sun_estimators")
    if args.workload == "cumulus" and not args.no_kdist:
        out["kdist"] = kdist_run(ctx, sc, kc)
        note("kdist")
    if not args.no_flux:
        out["flux"] = flux_run(ctx)
        note("flux")
        out["transmittance"] = transmittance_run(ctx, sc, kc)
        note("transmittance")
    if not args.no_guide_kernels:
        out["guide_kernels"] = guide_kernel_run(ctx, args)
        note("guide_kernels")
    if args.workload == "cumulus" and not args.no_tau_sweep:
        out["tau_sweep"] = tau_sweep(ctx, sc, kc)
        note("tau_sweep")
    if args.workload == "cumulus" and not args.no_variants:
        out["grid_variants"] = grid_variants(ctx, sc, kc, spp)
        note("grid_variants")
    if fine is not None:
        out["refinement"] = refinement_sweep(ctx, sc, fine)
        note("refinement")
        del fine
    if args.workload == "cumulus" and not args.no_batch:
        out["batch"] = batch_run(ctx, sc, kc, args.batch_spp)
        note("batch")
        if not args.no_guided:
            out["batch_guided"] = batch_guided_run(ctx, sc, kc, args.batch_spp, args)
            note("batch_guided")
        ctx.set_launch(args.block, args.waves_per_cu, args.spi, args.lds_levels)   # the single-view shape again
    if not args.no_time_to_eps:
        tail["time_to_eps"] = time_to_eps_run(ctx, sc, kc, gd, args, tail.get("guided"))
        note("time_to_eps")
    # the headline numbers last (a stored tail of the line keeps them)
    t1_plain = t_1pct
    t1_guided = tail["guided"]["time_to_1pct_s"] if "guided" in tail else None
    tail["time_to_1pct_s"] = {"plain": t1_plain, "guided": t1_guided,
                              "definition": "extrapolated from one step: RMS over pixels of the per-pixel standard "
                                            "error relative to the mean radiance, step time x (err / 0.01)^2; "
                                            "guided: error from the spread of independent renders, plus the "
                                            "guide's collection and training time; measured runs to 3 %: "
                                            "time_to_eps"}
    tail["roofline"] = roof
    if not args.no_cpu_baseline:
        tail["cpu_baseline"] = cpu_baseline(sc, spp, args.cpu_seconds, args.cpu_workers)
        note("cpu_baseline")
    out.update(tail)
    print(json.dumps(out))


def roofline(c, render_ms, with_record):
    """Gather-bound HBM roofline of the render kernel.  The method's reads
    per launch are the field gathers at tentative collisions plus the
    voxels entered below the LDS-staged grid levels (a node, or for a
    single-cell voxel the cell, read from memory); each random read moves
    one 64-byte HBM access granule.  The kernel's own extra reads (the
    ancestry mask and the cell value it reads at every voxel lookup) are
    reported beside it, and the measured HBM traffic from the committed
    counter record when it matches these sources."""
    t = render_ms / 1e3
    method = c["gathers"] + c["deep_visits"]
    achieved = method * GRANULE / t / 1e9
    impl = c["gathers"] + c["node_reads"]
    traffic = measured_traffic() if with_record else None
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "definition": "(field gathers + voxels entered below the LDS-staged levels) x 64 B / render time",
            "method_reads_per_path": method / max(c["paths"], 1),
            "implementation_reads_per_path": impl / max(c["paths"], 1),
            "implementation_request_GBps_at_64B": impl * GRANULE / t / 1e9,
            "method_bytes_GBps": (4 * c["gathers"] + 8 * c["deep_visits"] + 16 * c["paths"]) / t / 1e9,
            "measured_hbm_GBps": traffic / t / 1e9 if traffic else None,
            "valu_insts_x4_per_simd_cycle": measured_valu_issue(render_ms) if with_record else None}


def gather_ceiling(ctx):
    """Measured random 4-byte read rates (context for the roofline, not its
    peak): over 2 GiB (beyond the 256 MB last-level cache: HBM) and over
    128 MiB (held by the last-level cache)."""
    import torch

    from paper_1902_01137_amd import api
    out = {}
    for name, words in (("hbm_2GiB", 1 << 29), ("mall_128MiB", 1 << 25)):
        buf = torch.rand(words, device="cuda")
        rate = api.gather_rate(ctx, buf, threads=1 << 20, loads=64)
        del buf
        torch.cuda.empty_cache()
        out[name] = {"loads_per_s": rate, "GB_per_s_at_64B": rate * GRANULE / 1e9, "buffer_bytes": words * 4}
    return out


def progressive_run(ctx, sc, kc, gd, args, guided_info=None):
    """Rounds of samples until the 8x8-block relative standard error is 1 %
    (plain, then guided; the guided total adds the guide's collection and
    training)."""
    import torch

    from paper_1902_01137_amd import api, inputs
    g = api.build_grid(ctx, kc, sc.desc, sc.grid)
    out = {}
    for name, guide in (("plain", None), ("guided", gd)):
        if name == "guided" and guide is None:
            continue
        smp = inputs.Sampling(seed=sc.sampling.seed + 31, spp=0, flags=FLAGS, guide_frac=args.guide_frac,
                              guide_max_order=args.guide_max_order)
        _, _, rep = api.render_progressive(ctx, g, kc, sc.optics, sc.camera, smp, 0.01, first_spp=16,
                                           max_spp=args.max_spp, block=8, guide=guide)
        torch.cuda.synchronize()
        if name == "guided" and guided_info:
            rep["setup_s"] = guided_info["collect_s"] + guided_info["train_s"]
            rep["total_s"] = rep["seconds"] + rep["setup_s"]
        else:
            rep["total_s"] = rep["seconds"]
        out[name] = rep
    return out


def eps_rounds(ctx, g, kc, sc, smp, eps, guide, name):
    """Render calls continuing one sample sequence (sample offsets) into the
    same sums until the per-pixel relative standard error reaches eps; each
    round is sized from the error so far (at most 16384 spp), the time is the
    render calls' own (synchronised) and the error is the bench's per-pixel
    definition."""
    import dataclasses

    import torch

    from paper_1902_01137_amd import api
    cam = sc.camera
    s = torch.zeros((cam.height, cam.width), dtype=torch.float64, device="cuda")
    s2 = torch.zeros_like(s)
    n, spent, rounds, R = 0, 0.0, 0, 64
    while True:
        step = dataclasses.replace(smp, spp=R, sample_offset=smp.sample_offset + n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if guide is None:
            api.render(ctx, g, kc, sc.optics, cam, step, s, s2)
        else:
            api.render_guided(ctx, g, kc, sc.optics, cam, step, guide, s, s2)
        torch.cuda.synchronize()
        spent += time.perf_counter() - t0
        n += R
        rounds += 1
        m = s / n
        var = torch.clamp(s2 / n - m * m, min=0.0) * n / (n - 1)
        err = float(torch.sqrt(torch.mean(var / n)) / torch.mean(m))
        print("%s: round %d, %d spp, error %.5f, %.1f s" % (name, rounds, n, err, spent), file=sys.stderr, flush=True)
        if err <= eps:
            return {"spp_done": n, "rounds": rounds, "rel_err": err, "mean": float(torch.mean(m)), "seconds": spent}
        R = next_round_spp(n, err, eps)


def next_round_spp(n, err, eps):
    """Samples per pixel of the next round of eps_rounds: what n samples at
    error err predict is still missing to reach eps (the error falls as
    1 / sqrt(spp)), with 0.2 % to spare, in steps of 1024, at least 1024 and
    at most 16384 (a round then takes under a minute on the cumulus view)."""
    need = n * (err / eps) ** 2 * 1.002 - n
    return int(min(16384, max(1024, math.ceil(need / 1024) * 1024)))


def time_to_eps_run(ctx, sc, kc, gd, args, guided_info=None):
    """Measured time to a per-pixel relative standard error of args.eps on the
    full image (RMS over pixels of the standard error relative to the mean):
    progressive rounds of plain, then guided, rendering; the guided total
    adds the guide's collection and training."""
    import torch

    from paper_1902_01137_amd import api, inputs
    g = api.build_grid(ctx, kc, sc.desc, sc.grid)
    out = {"eps": args.eps, "definition": "per pixel, full resolution; progressive rounds from 64 spp"}
    for name, guide in (("plain", None), ("guided", gd)):
        if name == "guided" and guide is None:
            continue
        smp = inputs.Sampling(seed=sc.sampling.seed + 37, spp=0, flags=FLAGS, guide_frac=args.guide_frac,
                              guide_max_order=args.guide_max_order)
        if args.eps_rounds:
            rep = eps_rounds(ctx, g, kc, sc, smp, args.eps, guide, name)
        else:
            _, _, rep = api.render_progressive(ctx, g, kc, sc.optics, sc.camera, smp, args.eps, first_spp=64,
                                               max_spp=1 << 20, block=1, guide=guide)
        torch.cuda.synchronize()
        rep["total_s"] = rep["seconds"]
        if name == "guided" and guided_info:
            rep["setup_s"] = guided_info["collect_s"] + guided_info["train_s"]
            rep["total_s"] += rep["setup_s"]
        rep["to_1pct_extrapolated_s"] = rep["seconds"] * (rep["rel_err"] / 0.01) ** 2 + rep.get("setup_s", 0.0)
        out[name] = rep
    return out


def estimator_run(ctx, sc, kc, spp, build_ms):
    """The same step with each sun-ray estimator, and with the solar disc:
    render time, error and time to 1 %."""
    import torch

    from paper_1902_01137_amd import _lib, api, inputs
    g = api.build_grid(ctx, kc, sc.desc, sc.grid)
    cam = sc.camera
    res = {}
    # the last line: the sun as the 0.265-degree disc it is (the solar cone of Section 4.1)
    disc = inputs.Optics(**{**vars(sc.optics), "sun_half_angle_deg": 0.265})
    for name, fl, op in (("delta", _lib.NC_SUN_DELTA, sc.optics), ("ratio", _lib.NC_SUN_RATIO, sc.optics),
                         ("residual", _lib.NC_SUN_RESIDUAL, sc.optics),
                         ("residual_disc_0.265deg", _lib.NC_SUN_RESIDUAL, disc)):
        smp = inputs.Sampling(seed=sc.sampling.seed + 61, spp=spp, flags=fl)
        api.render(ctx, g, kc, op, cam, inputs.Sampling(seed=1, spp=1, flags=fl))   # warm-up
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        s, s2 = api.render(ctx, g, kc, op, cam, smp)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        eps = rel_err(s, s2, spp)
        paths = cam.width * cam.height * spp
        res[name] = {"render_ms": ms, "paths_per_s": paths / (ms / 1e3), "rel_std_err": eps,
                     "time_to_1pct_s": (build_ms + ms) / 1e3 * (eps / 0.01) ** 2}
    return res


def kdist_run(ctx, sc, kc):
    """Spectral integration over a synthetic 8-point k-distribution of the gas
    (0.001 .. 1 km^-1) on the workload's view at 512^2, 32 samples per pixel:
    one launch that draws a point per path under one grid built for the
    largest k_gas, against one grid and one launch per point (w_i x spp
    samples each, combined with the weights)."""
    import torch

    from paper_1902_01137_amd import api, inputs
    w, kgs = inputs.kdist_synthetic()
    cam = inputs.Camera(**{**vars(sc.camera), "width": 512, "height": 512})
    spp = 32
    op = inputs.Optics(**{**vars(sc.optics), "kdist": (w, kgs)})
    res = {"points": len(w), "k_gas": [float(x) for x in kgs], "weights": [float(x) for x in w]}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = api.build_grid(ctx, kc, sc.desc, inputs.GridParams(sc.grid.tau_tilde, float(kgs.max()), sc.grid.criterion))
    s, s2 = api.render(ctx, g, kc, op, cam, inputs.Sampling(seed=sc.sampling.seed + 91, spp=spp, flags=FLAGS))
    torch.cuda.synchronize()
    t_shared = time.perf_counter() - t0
    eps = rel_err(s, s2, spp)
    res["shared_grid"] = {"s": t_shared, "rel_std_err": eps, "time_to_1pct_s": t_shared * (eps / 0.01) ** 2}
    del g
    mean = torch.zeros((cam.height, cam.width), dtype=torch.float64, device="cuda")
    var = torch.zeros_like(mean)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (wi, ki) in enumerate(zip(w, kgs)):
        n_i = max(2, int(round(wi * spp)))
        # without a k-distribution a path takes its grid's gas extinction: this point's
        gi = api.build_grid(ctx, kc, sc.desc, inputs.GridParams(sc.grid.tau_tilde, float(ki), sc.grid.criterion))
        si, s2i = api.render(ctx, gi, kc, sc.optics, cam,
                             inputs.Sampling(seed=sc.sampling.seed + 92 + i, spp=n_i, flags=FLAGS))
        m_i = si / n_i
        v_i = torch.clamp(s2i / n_i - m_i * m_i, min=0.0) * n_i / (n_i - 1) / n_i
        mean += wi * m_i
        var += wi * wi * v_i
        del gi
    torch.cuda.synchronize()
    t_per = time.perf_counter() - t0
    eps_p = float(torch.sqrt(var.mean()) / mean.mean())
    res["grid_per_point"] = {"s": t_per, "rel_std_err": eps_p, "time_to_1pct_s": t_per * (eps_p / 0.01) ** 2}
    return res


def flux_run(ctx):
    """Forward photons and the adjoint replay on the cylinder cumulus (256^3,
    sun at zenith, 10^7 photons onto 100 x 100 ground pixels)."""
    import torch

    from paper_1902_01137_amd import api, inputs
    sc = inputs.scene_cylinder()
    kc = torch.from_numpy(sc.kc).cuda()
    g = api.build_grid(ctx, kc, sc.desc, sc.grid)
    N = 10_000_000
    smp = inputs.Sampling(seed=sc.sampling.seed + 81, spp=1)
    api.flux(ctx, g, kc, sc.optics, (100, 100), 1 << 20, smp)        # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tally, glob = api.flux(ctx, g, kc, sc.optics, (100, 100), N, smp)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    grad = torch.ones((100, 100), dtype=torch.float64, device="cuda")
    out = api.flux_adjoint(ctx, g, kc, sc.optics, (100, 100), N, smp, grad)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    f = 100 * 100 / N
    T = tally[0].cpu().numpy() * f
    return {"photons": N, "forward_ms": (t1 - t0) * 1e3, "adjoint_ms": (t2 - t1) * 1e3,
            "photons_per_s": N / (t1 - t0), "mean_T": float(T.mean()),
            "dmeanT_ds": float(out[0]) * f / 1e4, "dmeanT_dg": float(out[1]) * f / 1e4,
            "dmeanT_dalpha": float(out[2]) * f / 1e4}


def transmittance_run(ctx, sc, kc):
    """Direct transmissivity (nc_transmittance) of 2^22 rays from uniform
    points of the workload's box towards its sun, 16 paths each, for the
    three estimators."""
    import torch

    from paper_1902_01137_amd import _lib, api, inputs
    g = api.build_grid(ctx, kc, sc.desc, sc.grid)
    n, spp = 1 << 22, 16
    gen = np.random.default_rng(5)
    (xa, xb), (ya, yb), (za, zb) = sc.desc.box
    o = np.stack([gen.uniform(xa, xb, n), gen.uniform(ya, yb, n), gen.uniform(za, zb, n)], axis=1)
    d = np.broadcast_to(np.asarray(inputs.sun_direction(sc.optics.sun_zenith_deg, sc.optics.sun_azimuth_deg)), (n, 3))
    rays = torch.from_numpy(np.concatenate([o, d], axis=1).astype(np.float32)).cuda()
    res = {"rays": n, "spp": spp}
    for name, fl in (("delta", _lib.NC_SUN_DELTA), ("ratio", _lib.NC_SUN_RATIO), ("residual", _lib.NC_SUN_RESIDUAL)):
        api.transmittance(ctx, g, kc, sc.optics, rays[:4096], inputs.Sampling(seed=1, spp=spp, flags=fl))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s, s2 = api.transmittance(ctx, g, kc, sc.optics, rays, inputs.Sampling(seed=sc.sampling.seed + 91, spp=spp,
                                                                                flags=fl))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        m = s / spp
        var = (s2 / spp - m * m).clamp(min=0) * spp / (spp - 1) / spp
        res[name] = {"ms": dt * 1e3, "paths_per_s": n * spp / dt, "mean_T": float(m.mean()),
                     "rel_std_err": float(var.mean().sqrt() / m.mean())}
    return res


def guide_kernel_run(ctx, args):
    """The network's kernels: one Adam step on a batch, and inference, on the
    matrix cores (15 -> 64 -> 64 -> 64 -> 40; 11.9 k MACs per record forward,
    about three times that for a training step)."""
    import torch

    from paper_1902_01137_amd import api
    gd = api.Guide(ctx, seed=3)
    rng = np.random.default_rng(1)
    n = 1 << 20
    rec = np.zeros((n, 12), np.float32)
    rec[:, :3] = rng.uniform(-1, 1, (n, 3))
    d = rng.standard_normal((n, 3))
    rec[:, 3:6] = d / np.linalg.norm(d, axis=1, keepdims=True)
    rec[:, 6] = np.log1p(rng.exponential(20.0, n))
    o = rng.standard_normal((n, 3))
    rec[:, 7:10] = o / np.linalg.norm(o, axis=1, keepdims=True)
    rec[:, 10] = 1.0
    t = torch.from_numpy(rec).cuda()
    macs = 15 * 64 + 64 * 64 * 2 + 64 * 40
    res = {}
    for batch in (8192, 65536):
        b = t[:batch].contiguous()
        for _ in range(5):
            gd.train_step(b, 1e-4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 200
        for _ in range(steps):
            gd.train_step(b, 1e-4)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        res["train_batch_%d" % batch] = {"step_ms": dt * 1e3, "records_per_s": batch / dt,
                                         "TFLOP_per_s": 3 * 2 * macs * batch / dt / 1e12}
    gd.forward(t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gd.forward(t)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res["forward_1M"] = {"ms": dt * 1e3, "records_per_s": n / dt, "TFLOP_per_s": 2 * macs * n / dt / 1e12,
                         "peak_bf16_TFLOP_per_s": 2500.0}
    return res


def tau_sweep(ctx, sc, kc):
    """Render time against the merge threshold tau_tilde (Fig. 7), with the
    split between voxel crossing and collision work: 512^2 view, 32 spp,
    each timed after a 1-spp warm-up render over the new grid."""
    import torch

    from paper_1902_01137_amd import api, inputs
    cam = inputs.Camera(**{**vars(sc.camera), "width": 512, "height": 512})
    spp = 32
    paths = 512 * 512 * spp
    res = []
    for tt in (0.0, 0.03, 0.1, 0.3, 1.0, 3.0, 10.0, 30.0, 100.0, math.inf):
        g = api.build_grid(ctx, kc, sc.desc, inputs.GridParams(tt, sc.grid.k_gas, 0))
        api.render(ctx, g, kc, sc.optics, cam, inputs.Sampling(seed=sc.sampling.seed + 70, spp=1, flags=FLAGS))
        cnt = api.new_counters("cuda")
        smp = inputs.Sampling(seed=sc.sampling.seed + 71, spp=spp, flags=FLAGS)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        api.render(ctx, g, kc, sc.optics, cam, smp)
        e1.record()
        api.render(ctx, g, kc, sc.optics, cam, smp, counters=cnt)   # the same paths, with statistics
        torch.cuda.synchronize()
        c = api.counters_dict(cnt)
        ticks = {k: c["ticks_" + k] for k in ("step", "collide", "event", "sample")}
        tot = max(sum(ticks.values()), 1)
        res.append({"tau_tilde": tt if math.isfinite(tt) else "inf", "render_ms": e0.elapsed_time(e1),
                    "leaf_visits_per_path": c["leaf_visits"] / paths, "tentative_per_path": c["tentative"] / paths,
                    "nulls_per_path": c["nulls"] / paths, "step_share": ticks["step"] / tot,
                    "collision_share": ticks["collide"] / tot})
        del g
    return res


def grid_variants(ctx, sc, kc, spp):
    """The same render over other majorant grids: the flat grid of 8^3-cell
    supercells, the layered grids (clear layers split from the cloudy one,
    which holds 8^3-cell supercells or single cells), tau_tilde = 0 (every
    cell a voxel) and one global voxel; each timed after a 1-spp warm-up
    render over the new grid."""
    import torch

    from paper_1902_01137_amd import api, inputs
    cam = sc.camera
    res = {}
    for name, gp in (("hier_tau1", sc.grid),
                     ("flat_8cube", inputs.GridParams(0.0, sc.grid.k_gas, 2, 3)),
                     ("layered_8cube", inputs.GridParams(0.0, sc.grid.k_gas, 3, 3)),
                     ("layered_cells", inputs.GridParams(0.0, sc.grid.k_gas, 3, 0)),
                     ("tau0", inputs.GridParams(0.0, sc.grid.k_gas, 0)),
                     ("global", inputs.GridParams(math.inf, sc.grid.k_gas, 0))):
        g = api.build_grid(ctx, kc, sc.desc, gp)
        api.render(ctx, g, kc, sc.optics, cam, inputs.Sampling(seed=sc.sampling.seed + 40, spp=1, flags=FLAGS))
        cnt = api.new_counters("cuda")
        smp = inputs.Sampling(seed=sc.sampling.seed + 41, spp=spp, flags=FLAGS)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        s, s2 = api.render(ctx, g, kc, sc.optics, cam, smp)
        e1.record()
        api.render(ctx, g, kc, sc.optics, cam, smp, counters=cnt)   # the same paths, with statistics
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        c = api.counters_dict(cnt)
        paths = cam.width * cam.height * spp
        res[name] = {"render_ms": ms, "paths_per_s": paths / (ms / 1e3), "mean_radiance": float(s.sum()) / paths,
                     "per_path": {k: c[k] / paths for k in ("segments", "tentative", "nulls", "leaf_visits",
                                                            "gathers", "node_reads")}}
        del g
    return res


def build_bytes(g):
    """Bytes a grid build must move at least: the field read once, every
    level's nodes (8 bytes each) and the level-1 ancestry masks (2 bytes
    each) written once."""
    d = g.desc
    nodes = sum(int(np.prod(g.level_dims(l))) for l in range(1, g.L + 1))
    return 4 * d.nx * d.ny * d.nz + 8 * nodes + 2 * int(np.prod(g.level_dims(1)))


def refinement_sweep(ctx, sc, fine):
    """Grid build time and render rate against the voxel count: the 12.5 m
    field and its 2, 4 and 8 regional averages, tau_tilde = 1 and 0; the
    workload's camera at 512^2, 32 spp; render time is the best of 3 after
    a warm-up render.  build_ms is the in-place rebuild (the build kernels,
    the field check's read-back and a stream synchronisation), beside the
    build with its allocation and the bytes a build must move at least."""
    import torch

    from paper_1902_01137_amd import api, inputs
    out = []
    cam = inputs.Camera(**{**vars(sc.camera), "width": 512, "height": 512})
    spp = 32
    for f in (8, 4, 2, 1):
        desc, k = inputs.pool_field(*fine, f) if f > 1 else fine
        kc = torch.from_numpy(k).cuda()
        row = {"field": [desc.nx, desc.ny, desc.nz], "cell_km": desc.dx, "voxels": desc.nx * desc.ny * desc.nz}
        for tau in (1.0, 0.0):
            gp = inputs.GridParams(tau, sc.grid.k_gas, 0)
            api.build_grid(ctx, kc, desc, gp)                     # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 5
            for _ in range(reps):
                g = api.build_grid(ctx, kc, desc, gp)
            torch.cuda.synchronize()
            alloc_ms = (time.perf_counter() - t0) * 1e3 / reps
            # the build proper: in place over the same allocation (the
            # field check's flag read back and the stream synchronised each time)
            for _ in range(3):
                g.rebuild(kc)
            reps = 20
            t0 = time.perf_counter()
            for _ in range(reps):
                g.rebuild(kc)
            torch.cuda.synchronize()
            build_ms = (time.perf_counter() - t0) * 1e3 / reps
            nbytes = build_bytes(g)
            # a short warm-up render first (the first pass over a freshly
            # built grid pays for page-table and cache fills), then the best of 3
            api.render(ctx, g, kc, sc.optics, cam, inputs.Sampling(seed=sc.sampling.seed + 50, spp=2, flags=FLAGS))
            ms = float("inf")
            for rep in range(3):
                smp = inputs.Sampling(seed=sc.sampling.seed + 51 + rep, spp=spp, flags=FLAGS)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                api.render(ctx, g, kc, sc.optics, cam, smp)
                e1.record()
                torch.cuda.synchronize()
                ms = min(ms, e0.elapsed_time(e1))
            row["tau%g" % tau] = {"build_ms": build_ms, "build_with_allocation_ms": alloc_ms,
                                  "build_bytes": nbytes, "build_GBps": nbytes / (build_ms / 1e3) / 1e9,
                                  "build_frac": nbytes / (build_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
                                  "render_ms": ms, "paths_per_s": 512 * 512 * spp / (ms / 1e3)}
            del g
        out.append(row)
        del kc
        torch.cuda.empty_cache()
    return out


def rel_err(s, s2, spp):
    sm = s.cpu().numpy().ravel() / spp
    var = np.maximum(s2.cpu().numpy().ravel() / spp - sm ** 2, 0) * spp / (spp - 1)
    return float(np.sqrt(np.mean(var / spp)) / np.mean(sm))


def spread_err(runs):
    """Relative standard error of one render from the spread of K independent
    renders (RMS over pixels of the per-pixel standard deviation of the
    renders' means, relative to the mean), and the one the renders report
    (RMS of their per-pixel standard errors)."""
    M = np.array([m for m, _ in runs])
    E2 = np.array([e ** 2 for _, e in runs])
    mean = M.mean()
    return float(np.sqrt(M.var(axis=0, ddof=1).mean()) / mean), float(np.sqrt(E2.mean()) / mean)


def render_runs(ctx, g, kc, sc, cam, spp, seeds, guide=None, args=None):
    """Per-pixel (mean, standard error) of independent renders."""
    import torch

    from paper_1902_01137_amd import api, inputs
    runs = []
    for sd in seeds:
        smp = inputs.Sampling(seed=sd, spp=spp, flags=FLAGS, guide_frac=args.guide_frac if args else 0.5,
                              guide_max_order=args.guide_max_order if args else 0)
        if guide is None:
            s, s2 = api.render(ctx, g, kc, sc.optics, cam, smp)
        else:
            s, s2 = api.render_guided(ctx, g, kc, sc.optics, cam, smp, guide)
        sm = s.cpu().numpy().ravel() / spp
        var = np.maximum(s2.cpu().numpy().ravel() / spp - sm ** 2, 0) * spp / (spp - 1)
        runs.append((sm, np.sqrt(var / spp)))
        del s, s2
    torch.cuda.synchronize()
    return runs


def lr_at(it, steps, lr):
    """Adam step size of step it of steps: a cosine decay from lr to 1 % of it
    (on the cumulus view it ends 7 % lower in guided variance than a constant
    rate dropped to a fifth for the last fifth, at the same number of steps)."""
    return lr * max(0.01, 0.5 * (1.0 + math.cos(math.pi * it / steps)))


def guided_run(ctx, sc, kc, spp, args, build_ms, plain):
    """The guided leg: record the scattering vertices of a short plain render,
    fit the guide to them (Adam on random minibatches), then render the same
    view guided at the same spp.  The error of a guided step is measured from
    the spread of independent renders (checked against the standard error
    they report), and the plain step's likewise.  Time to 1 % = collection +
    training + one guided step (grid build + render) scaled by
    (err / 0.01)^2 (an extrapolation; the measured runs are time_to_eps)."""
    import torch

    from paper_1902_01137_amd import api, inputs
    cam = sc.camera
    g = api.build_grid(ctx, kc, sc.desc, sc.grid)
    cap = cam.width * cam.height * args.collect_spp * 16
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rec, n, _, _ = api.collect_vertices(ctx, g, kc, sc.optics, cam,
                                        inputs.Sampling(seed=sc.sampling.seed + 101, spp=args.collect_spp, flags=FLAGS),
                                        cap)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gd = api.Guide(ctx, seed=1)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(1)
    losses = []
    for it in range(args.train_steps):
        idx = torch.randint(0, rec.shape[0], (args.train_batch,), device="cuda", generator=gen)
        l = gd.train_step(rec[idx], lr_at(it, args.train_steps, args.lr))
        if it % max(1, args.train_steps // 4) == 0 or it == args.train_steps - 1:
            losses.append(l)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    del rec
    smp = inputs.Sampling(seed=sc.sampling.seed + 202, spp=spp, flags=FLAGS, guide_frac=args.guide_frac,
                          guide_max_order=args.guide_max_order)
    api.render_guided(ctx, g, kc, sc.optics, cam, smp, gd)         # warm-up
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    api.render_guided(ctx, g, kc, sc.optics, cam, smp, gd)
    e1.record()
    torch.cuda.synchronize()
    render_ms = e0.elapsed_time(e1)
    K = max(2, args.spread_renders)
    g_spread, g_rep = spread_err(render_runs(ctx, g, kc, sc, cam, spp, [sc.sampling.seed + 210 + k for k in range(K)],
                                             gd, args))
    p_spread, p_rep = spread_err(render_runs(ctx, g, kc, sc, cam, spp, [sc.sampling.seed + 230 + k for k in range(K)]))
    step_ms = build_ms + render_ms
    collect_s, train_s = t1 - t0, t2 - t1
    paths = cam.width * cam.height * spp
    return {"collect_spp": args.collect_spp, "records": n, "collect_s": collect_s, "train_steps": args.train_steps,
            "train_batch": args.train_batch, "train_s": train_s,
            "loss": [round((x[0] / x[1]).item(), 4) for x in losses], "guide_frac": args.guide_frac,
            "guide_max_order": args.guide_max_order,
            "render_ms": render_ms, "paths_per_s": paths / (step_ms / 1e3),
            "spread_renders": K,
            "rel_std_err_spread": g_spread, "rel_std_err_reported": g_rep,
            "plain_rel_std_err_spread": p_spread, "plain_rel_std_err_reported": p_rep,
            "variance_ratio_guided_plain": (g_spread / p_spread) ** 2,
            "time_to_1pct_s": collect_s + train_s + step_ms / 1e3 * (g_spread / 0.01) ** 2,
            "plain_time_to_1pct_s_spread": plain["step_ms"] / 1e3 * (p_spread / 0.01) ** 2}, gd


def batch_run(ctx, sc, kc, spp):
    """48 views (256^2 .. 1024^2) x 4 sun zeniths of the same field in one
    persistent launch, on the launch shape the autotuner picks for it (tuned
    at the batch's own spp, since the grouping of samples into queue items is
    one of the knobs; the context keeps the shape for the guided batch that
    follows)."""
    import torch

    from paper_1902_01137_amd import api, inputs
    g = api.build_grid(ctx, kc, sc.desc, sc.grid)
    views = inputs.batch_views()
    jobs = [(cam, inputs.Optics(**{**vars(sc.optics), "sun_zenith_deg": sz})) for cam, sz in views]
    px = sum(c.width * c.height for c, _ in jobs)
    default_launch = ctx.get_launch()
    t0 = time.perf_counter()
    tuned, tuned_ms = api.autotune_batch(ctx, g, kc, jobs, inputs.Sampling(seed=sc.sampling.seed + 16, spp=spp,
                                                                           flags=FLAGS))
    tune_s = time.perf_counter() - t0
    res = {"jobs": len(jobs), "pixels": px, "spp": spp, "paths": px * spp, "tuned_launch": tuned,
           "tuned_ms": tuned_ms, "tune_s": tune_s, "default_launch": default_launch}
    for name in ("default", "tuned"):
        ctx.set_launch(**(default_launch if name == "default" else tuned))
        smp = inputs.Sampling(seed=sc.sampling.seed + 17, spp=spp, flags=FLAGS)
        api.render_batch(ctx, g, kc, jobs, smp)                       # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s, s2, offs = api.render_batch(ctx, g, kc, jobs, inputs.Sampling(seed=sc.sampling.seed + 18, spp=spp,
                                                                         flags=FLAGS))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if name == "tuned":
            eps = batch_block_err(s, s2, offs, jobs, spp)
            res.update({"ms": dt * 1e3, "paths_per_s": px * spp / dt, "rel_std_err_block8": eps,
                        "time_to_1pct_block8_s": dt * (eps / 0.01) ** 2})
        else:
            res["default_ms"] = dt * 1e3
        del s, s2
    return res


def batch_block_err(s, s2, offs, jobs, spp, b=8):
    """Relative standard error of the batch on 8x8-pixel block means, all images together."""
    S = s.cpu().numpy()
    S2 = s2.cpu().numpy()
    means, errs = [], []
    for (cam, _), o in zip(jobs, offs):
        n = cam.width * cam.height
        m = S[o:o + n].reshape(cam.height, cam.width) / spp
        v = np.maximum(S2[o:o + n].reshape(cam.height, cam.width) / spp - m * m, 0) * spp / (spp - 1) / spp
        H, W = (cam.height // b) * b, (cam.width // b) * b
        mb = m[:H, :W].reshape(H // b, b, W // b, b).mean(axis=(1, 3))
        vb = v[:H, :W].reshape(H // b, b, W // b, b).sum(axis=(1, 3)) / (b * b) ** 2
        means.append(mb.ravel())
        errs.append(vb.ravel())
    return float(np.sqrt(np.concatenate(errs).mean()) / np.concatenate(means).mean())


def batch_guided_run(ctx, sc, kc, spp, args):
    """The 48 views x 4 suns with guidance: one network per sun (its inputs do
    not see the sun), trained on vertices of 8 of that sun's views spread
    around the ring (every 6th, 5 spp each: the guided paths start from all
    around the cloud, and a network fed from one view alone generalised
    badly to the others); all 192 jobs in one persistent launch, each
    workgroup holding one sun's network.  Error on 8x8-pixel block means
    against the plain batch at the same spp, on the context's launch shape."""
    import torch

    from paper_1902_01137_amd import api, inputs
    g = api.build_grid(ctx, kc, sc.desc, sc.grid)
    views = inputs.batch_views()
    suns = sorted({sz for _, sz in views})
    t0 = time.perf_counter()
    guides = {}
    for sz in suns:
        op = inputs.Optics(**{**vars(sc.optics), "sun_zenith_deg": sz})
        recs = []
        for cam in [c for c, z in views if z == sz][::6]:
            r, n, _, _ = api.collect_vertices(ctx, g, kc, op, cam,
                                              inputs.Sampling(seed=sc.sampling.seed + 301, spp=5, flags=FLAGS),
                                              cam.width * cam.height * 5 * 16)
            recs.append(r)
        rec = torch.cat(recs)
        del recs
        gd = api.Guide(ctx, seed=1)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(1)
        for it in range(args.batch_train_steps):
            idx = torch.randint(0, rec.shape[0], (args.batch_train_batch,), device="cuda", generator=gen)
            gd.train_step(rec[idx], lr_at(it, args.batch_train_steps, args.lr))
        guides[sz] = gd
        del rec
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    jobs = [(cam, inputs.Optics(**{**vars(sc.optics), "sun_zenith_deg": z})) for cam, z in views]
    per_job = [guides[z] for _, z in views]
    out = {"train_s": train_s, "launches": 1, "launch": ctx.get_launch()}
    for name in ("plain", "guided"):
        smp = inputs.Sampling(seed=sc.sampling.seed + 311, spp=spp, flags=FLAGS, guide_frac=args.guide_frac,
                              guide_max_order=args.guide_max_order)
        gd = per_job if name == "guided" else None
        api.render_batch(ctx, g, kc, jobs, smp, guide=gd)                # warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s, s2, offs = api.render_batch(ctx, g, kc, jobs, smp, guide=gd)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        eps = batch_block_err(s, s2, offs, jobs, spp)
        out[name] = {"ms": dt * 1e3, "rel_std_err_block8": eps,
                     "time_to_1pct_block8_s": dt * (eps / 0.01) ** 2 + (train_s if name == "guided" else 0.0)}
        del s, s2
    return out


def _cpu_info():
    """CPU model, clock and the cores this process may use (from lscpu and the affinity mask)."""
    import subprocess
    info = {"model": None, "mhz": None, "max_mhz": None}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            v = v.strip()
            if k.strip() == "Model name":
                info["model"] = v
            elif k.strip() == "CPU MHz":
                info["mhz"] = float(v)
            elif k.strip() == "CPU max MHz":
                info["max_mhz"] = float(v)
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    try:
        info["usable_cpus"] = len(os.sched_getaffinity(0))
    except AttributeError:
        info["usable_cpus"] = os.cpu_count()
    return info


def _oracle_pixels(job):
    """One oracle worker: render chunks of its pixel list (all spp) until the
    time budget is spent; the field comes from a memory-mapped file."""
    import oracle
    desc, path, k_gas, optics, cam, spp, seed, pixels, budget_s = job
    kc = np.load(path, mmap_mode="r")
    done, paths, used = 0, 0, 0.0
    chunk = 8
    while used < budget_s and done < len(pixels):
        px = np.ascontiguousarray(pixels[done:done + chunk])
        t0 = time.perf_counter()
        oracle.render(desc, kc, k_gas, optics, cam, spp, seed, pixels=px)
        used += time.perf_counter() - t0
        done += len(px)
        paths += len(px) * spp
        chunk = min(chunk * 2, 256)
    return paths, used, done


def cpu_baseline(sc, spp, budget_s, workers=0):
    """The oracle on a bounded sample of the same workload (pixels drawn at
    random over the image, all spp samples each): one host core, then every
    usable core (independent processes on disjoint pixels, up to 16: the host
    share of one GPU), with the CPU model and clock."""
    import multiprocessing as mp
    import tempfile

    info = _cpu_info()
    P = workers if workers > 0 else max(1, min(16, info["usable_cpus"] or 1))
    cam = sc.camera
    npix = cam.width * cam.height
    order = np.random.default_rng(0).permutation(npix).astype(np.int32)
    tmp = tempfile.mkdtemp(prefix="nc_bench_")
    path = os.path.join(tmp, "kc.npy")
    np.save(path, sc.kc)
    seed = 2002
    try:
        one = _oracle_pixels((sc.desc, path, sc.grid.k_gas, sc.optics, cam, spp, seed, order[:4096], budget_s))
        rest = order[4096:]
        jobs = [(sc.desc, path, sc.grid.k_gas, sc.optics, cam, spp, seed, rest[i::P], budget_s) for i in range(P)]
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(P) as pool:
            res = pool.map(_oracle_pixels, jobs)
        wall = time.perf_counter() - t0
    finally:
        try:
            os.remove(path)
            os.rmdir(tmp)
        except OSError:
            pass
    paths_all = sum(r[0] for r in res)
    busy = max(r[1] for r in res)
    return {"value": paths_all / busy, "unit": "paths/s", "cores": P, "kind": "oracle",
            "sample": "random pixels x %d spp of the same image: 1 core %d paths in %.1f s; %d processes on "
                      "disjoint pixels %d paths in %.1f s of rendering (%.1f s wall with start-up)"
                      % (spp, one[0], one[1], P, paths_all, busy, wall),
            "single_core_paths_per_s": one[0] / one[1],
            "cpu_model": info["model"], "cpu_mhz": info["mhz"], "cpu_max_mhz": info["max_mhz"],
            "usable_cpus": info["usable_cpus"]}


if __name__ == "__main__":
    main()
