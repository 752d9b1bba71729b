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
    assert frac == rec["sq_active_inst_valu"] * 4.0 / (1024 * 2.4e9 * ms / 1e3)
    assert 0.0 < frac < 1.5
    monkeypatch.setattr(b, "kernel_sources_digest", lambda: "0" * 64)
    assert b.measured_traffic() is None
    assert b.measured_valu_issue(ms) is None
