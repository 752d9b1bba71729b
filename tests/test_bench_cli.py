"""The benchmark's command line on the host: its help text renders, and a
request for more than one GPU is refused with a message (the library has no
multi-GPU path)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_help_renders():
    r = _run("--help")
    assert r.returncode == 0, r.stderr
    assert "--gpus" in r.stdout and "--main-only" in r.stdout


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_profile_record_is_used_only_for_the_sources_it_was_measured_on(monkeypatch):
    """Measured traffic and VALU issue come from the committed rocprofv3
    record only while the HIP sources hash to the digest stored with it."""
    import json
    b = _bench_module()
    with open(os.path.join(ROOT, "profiles", "render_traffic.json")) as fh:
        rec = json.load(fh)
    monkeypatch.setattr(b, "kernel_sources_digest", lambda: rec["sources_sha256"])
    assert b.measured_traffic() == rec["bytes_per_launch"]
    ms = 150.0
    frac = b.measured_valu_issue(ms)
    assert frac == rec["sq_insts_valu"] * 4.0 / (1024 * 2.4e9 * ms / 1e3)
    assert 0.0 < frac < 1.5
    monkeypatch.setattr(b, "kernel_sources_digest", lambda: "0" * 64)
    assert b.measured_traffic() is None
    assert b.measured_valu_issue(ms) is None


def test_roofline_counts_the_methods_reads(monkeypatch):
    """frac comes from field gathers plus voxels entered below the LDS-staged
    levels (one 64-byte granule each); the kernel's extra mask and cell reads
    are reported apart."""
    b = _bench_module()
    monkeypatch.setattr(b, "kernel_sources_digest", lambda: "0" * 64)
    c = {"paths": 1000, "gathers": 800, "deep_visits": 20000, "node_reads": 90000}
    r = b.roofline(c, 2.0, True)
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and r["traffic"] is None
    assert r["achieved"] == (800 + 20000) * 64 / 2e-3 / 1e9
    assert r["frac"] == r["achieved"] / 8000.0
    assert r["method_reads_per_path"] == 20.8 and r["implementation_reads_per_path"] == 90.8


def test_spread_error_of_independent_renders():
    """Renders whose pixel means scatter by exactly their reported standard
    error give equal spread and reported errors."""
    import numpy as np
    b = _bench_module()
    rng = np.random.default_rng(3)
    truth = rng.uniform(1.0, 2.0, 4000)
    se = 0.05 * truth
    runs = [(truth + se * rng.standard_normal(4000), se) for _ in range(8)]
    spread, rep = b.spread_err(runs)
    assert abs(spread / rep - 1.0) < 0.03
    assert abs(rep - np.sqrt((se ** 2).mean()) / truth.mean()) < 1e-3


def test_training_step_size_decays_by_a_cosine():
    """The guide's Adam step size starts at lr, halves at mid-training and
    ends at the 1 % floor."""
    import math
    b = _bench_module()
    lr, n = 3e-3, 80000
    assert b.lr_at(0, n, lr) == lr
    assert abs(b.lr_at(n // 2, n, lr) - lr / 2) < 1e-12
    assert b.lr_at(n - 1, n, lr) == lr * 0.01
    vals = [b.lr_at(i, n, lr) for i in range(0, n, 997)]
    assert all(x >= y for x, y in zip(vals, vals[1:]))
    assert abs(b.lr_at(n // 4, n, lr) - lr * 0.5 * (1 + math.cos(math.pi / 4))) < 1e-12


def test_rounds_to_a_target_error_are_sized_from_the_error_so_far():
    """A round asks for what 1/sqrt(spp) scaling predicts is missing, in
    multiples of 1024 between 1024 and 16384."""
    b = _bench_module()
    # 64 spp at twice the target: 3 x 64 missing -> the minimum round
    assert b.next_round_spp(64, 0.02, 0.01) == 1024
    # 40000 spp at 1.1 x the target: 21 % more, 8400 spp -> rounded up to 9216
    n = b.next_round_spp(40000, 0.011, 0.01)
    assert n % 1024 == 0 and 40000 * (1.1 ** 2 * 1.002 - 1) <= n < 40000 * (1.1 ** 2 * 1.002 - 1) + 1024
    # far from the target: capped
    assert b.next_round_spp(1024, 0.1, 0.01) == 16384
    # at or below the target already: the smallest round
    assert b.next_round_spp(5000, 0.01, 0.01) == 1024
