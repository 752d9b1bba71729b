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
PHASES = ("cross", "collide", "event", "ray", "sample", "guide")


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
    """Share of the SIMDs' cycles spent issuing VALU instructions during one render launch:
    SQ_ACTIVE_INST_VALU of the committed counter run (units of 4 cycles, summed over waves)
    x 4 over SIMDs x clock x this run's kernel time; None if the record is stale or lacks it."""
    rec = _profile_record()
    if not rec or "sq_active_inst_valu" not in rec:
        return None
    return rec["sq_active_inst_valu"] * 4.0 / (MI355X_SIMDS * MI355X_CLOCK_HZ * render_ms / 1e3)


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
    p.add_argument("--train-batch", type=int, default=65536)
    p.add_argument("--lr", type=float, default=3e-3)
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
    p.add_argument("--main-only", action="store_true", help="only the timed steps (for profiling runs)")
    a = p.parse_args()
    if a.main_only:
        a.no_cpu_baseline = a.no_batch = a.no_guided = a.no_variants = a.no_refinement = True
        a.no_progressive = a.no_ceiling = a.no_estimators = a.no_tau_sweep = True
        a.no_flux = a.no_guide_kernels = a.no_kdist = True
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

    def step(i, counters=None):
        g = api.build_grid(ctx, kc, sc.desc, sc.grid)
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
    gathers_per_launch = c["gathers"] + c["node_reads"]
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
        "config": {"workload": name, "spp": spp, "image": [cam.width, cam.height], "sun_estimator": args.sun,
                   "field": [sc.desc.nx, sc.desc.ny, sc.desc.nz], "tau_tilde": sc.grid.tau_tilde,
                   "paths_per_step": paths_per_step},
        "render_ms": render_ms,
        "autotuned": tuned,
        "segments_per_s": c["segments"] / (render_ms / 1e3),
        "tentative_per_s": c["tentative"] / (render_ms / 1e3),
        "per_path": {k: c[k] / max(c["paths"], 1) for k in ("segments", "tentative", "nulls", "reals",
                                                            "leaf_visits", "gathers", "node_reads", "nee_rays")},
        "truncated": c["truncated"],
        "sched": {"trips": {k: c["trips_" + k] for k in PHASES},
                  "lanes_per_trip": {k: round(c["lanes_" + k] / max(c["trips_" + k], 1), 2) for k in PHASES},
                  "ticks_per_trip": {k: round(c["ticks_" + k] / max(c["trips_" + k], 1), 1) for k in PHASES}},
        "rel_std_err": eps,
        "time_to_1pct_s": {"plain": t_1pct, "guided": None},
        "time_to_1pct_definition": "RMS over pixels of the per-pixel standard error, relative to the mean radiance; "
                                   "step time x (err / 0.01)^2, plus the guide's collection and training time",
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if args.workload == "cumulus" and spp == 64 else None,
                     "valu_issue_frac": measured_valu_issue(render_ms)
                     if args.workload == "cumulus" and spp == 64 else None},
    }
    gd = None
    if not args.no_guided:
        out["guided"], gd = guided_run(ctx, sc, kc, spp, args, build_ms=ms_step - render_ms)
        out["time_to_1pct_s"]["guided"] = out["guided"]["time_to_1pct_s"]
        note("guided")
    if not args.no_ceiling:
        out["gather_ceiling"] = gather_ceiling(ctx)
        out["roofline"]["frac_of_measured_gather_rate"] = achieved / out["gather_ceiling"]["GB_per_s_at_64B"]
        note("gather_ceiling")
    if not args.no_progressive:
        out["progressive_block8"] = progressive_run(ctx, sc, kc, gd, args)
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
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sc, spp, args.cpu_seconds)
        note("cpu_baseline")
    print(json.dumps(out))


def gather_ceiling(ctx):
    """Measured random 4-byte read rate over a 2 GiB buffer (larger than the 256 MB last-level cache)."""
    import torch

    from paper_1902_01137_amd import api
    buf = torch.rand(1 << 29, device="cuda")
    rate = api.gather_rate(ctx, buf, threads=1 << 20, loads=64)
    del buf
    torch.cuda.empty_cache()
    return {"loads_per_s": rate, "GB_per_s_at_64B": rate * GRANULE / 1e9, "buffer_bytes": 1 << 31}


def progressive_run(ctx, sc, kc, gd, args):
    """Rounds of samples until the 8x8-block relative standard error is 1 % (plain, then guided)."""
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
        ticks = {k: c["ticks_" + k] for k in ("cross", "collide", "event", "ray", "sample")}
        tot = max(sum(ticks.values()), 1)
        res.append({"tau_tilde": tt if math.isfinite(tt) else "inf", "render_ms": e0.elapsed_time(e1),
                    "leaf_visits_per_path": c["leaf_visits"] / paths, "tentative_per_path": c["tentative"] / paths,
                    "nulls_per_path": c["nulls"] / paths, "crossing_share": ticks["cross"] / tot,
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


def refinement_sweep(ctx, sc, fine):
    """Grid build time and render rate against the voxel count: the 12.5 m
    field and its 2, 4 and 8 regional averages, tau_tilde = 1 and 0; the
    workload's camera at 512^2, 32 spp; render time is the best of 3 after
    a warm-up render."""
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
            build_ms = (time.perf_counter() - t0) * 1e3 / reps
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
            row["tau%g" % tau] = {"build_ms": build_ms, "render_ms": ms, "paths_per_s": 512 * 512 * spp / (ms / 1e3)}
            del g
        out.append(row)
        del kc
        torch.cuda.empty_cache()
    return out


def rel_err(s, s2, spp):
    sm = s.cpu().numpy().ravel() / spp
    var = np.maximum(s2.cpu().numpy().ravel() / spp - sm ** 2, 0) * spp / (spp - 1)
    return float(np.sqrt(np.mean(var / spp)) / np.mean(sm))


def guided_run(ctx, sc, kc, spp, args, build_ms):
    """The guided leg: record the scattering vertices of a short plain render,
    fit the guide to them (Adam on random minibatches), then render the same
    view guided at the same spp.  Time to 1% = collection + training + one
    guided step (grid build + render) scaled by (err / 0.01)^2."""
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
        lr = args.lr * (0.2 if it >= 0.8 * args.train_steps else 1.0)
        l = gd.train_step(rec[idx], lr)
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
    s, s2 = api.render_guided(ctx, g, kc, sc.optics, cam, smp, gd)
    e1.record()
    torch.cuda.synchronize()
    render_ms = e0.elapsed_time(e1)
    eps = rel_err(s, s2, spp)
    step_ms = build_ms + render_ms
    collect_s, train_s = t1 - t0, t2 - t1
    paths = cam.width * cam.height * spp
    return {"collect_spp": args.collect_spp, "records": n, "collect_s": collect_s, "train_steps": args.train_steps,
            "train_batch": args.train_batch, "train_s": train_s,
            "loss": [round((x[0] / x[1]).item(), 4) for x in losses], "guide_frac": args.guide_frac,
            "guide_max_order": args.guide_max_order,
            "render_ms": render_ms, "paths_per_s": paths / (step_ms / 1e3), "rel_std_err": eps,
            "time_to_1pct_s": collect_s + train_s + step_ms / 1e3 * (eps / 0.01) ** 2}, gd


def batch_run(ctx, sc, kc, spp):
    """48 views (256^2 .. 1024^2) x 4 sun zeniths of the same field in one persistent launch."""
    import torch

    from paper_1902_01137_amd import api, inputs
    g = api.build_grid(ctx, kc, sc.desc, sc.grid)
    views = inputs.batch_views()
    jobs = [(cam, inputs.Optics(**{**vars(sc.optics), "sun_zenith_deg": sz})) for cam, sz in views]
    px = sum(c.width * c.height for c, _ in jobs)
    smp = inputs.Sampling(seed=sc.sampling.seed + 17, spp=spp, flags=FLAGS)
    api.render_batch(ctx, g, kc, jobs, smp)                       # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s, s2, offs = api.render_batch(ctx, g, kc, jobs, inputs.Sampling(seed=sc.sampling.seed + 18, spp=spp,
                                                                     flags=FLAGS))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    eps = batch_block_err(s, s2, offs, jobs, spp)
    return {"jobs": len(jobs), "pixels": px, "spp": spp, "paths": px * spp, "ms": dt * 1e3,
            "paths_per_s": px * spp / dt, "rel_std_err_block8": eps,
            "time_to_1pct_block8_s": dt * (eps / 0.01) ** 2}


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
    badly to the others); one guided launch per sun.  Error on 8x8-pixel
    block means against the plain batch at the same spp."""
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
            idx = torch.randint(0, rec.shape[0], (args.train_batch,), device="cuda", generator=gen)
            gd.train_step(rec[idx], args.lr * (0.2 if it >= 0.8 * args.batch_train_steps else 1.0))
        guides[sz] = gd
        del rec
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    out = {"train_s": train_s}
    for name in ("plain", "guided"):
        t_total, errs, means = 0.0, [], []
        S_all = []
        for sz in suns:
            jobs = [(cam, inputs.Optics(**{**vars(sc.optics), "sun_zenith_deg": z})) for cam, z in views if z == sz]
            smp = inputs.Sampling(seed=sc.sampling.seed + 311, spp=spp, flags=FLAGS, guide_frac=args.guide_frac,
                                  guide_max_order=args.guide_max_order)
            gd = guides[sz] if name == "guided" else None
            api.render_batch(ctx, g, kc, jobs, smp, guide=gd)                # warm-up
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            s, s2, offs = api.render_batch(ctx, g, kc, jobs, smp, guide=gd)
            torch.cuda.synchronize()
            t_total += time.perf_counter() - t1
            S_all.append((s, s2, offs, jobs))
        eps = batch_block_err(torch.cat([x[0] for x in S_all]), torch.cat([x[1] for x in S_all]),
                              [o + sum(x[0].numel() for x in S_all[:k]) for k, x in enumerate(S_all) for o in x[2]],
                              [j for x in S_all for j in x[3]], spp)
        out[name] = {"ms": t_total * 1e3, "rel_std_err_block8": eps,
                     "time_to_1pct_block8_s": t_total * (eps / 0.01) ** 2 + (train_s if name == "guided" else 0.0)}
    return out


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
