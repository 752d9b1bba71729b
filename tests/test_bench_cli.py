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
