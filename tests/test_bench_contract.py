"""Host-side parts of the benchmark's contract: it runs on one GPU only and
says so for any other count; its stage-kernel counter figures are tied to the
digest of the kernel's sources (reported as null once the sources differ)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_counter_figures_follow_the_source_digest(monkeypatch):
    b = _bench_module()
    n = b.STAGE_TRAFFIC["n"]
    want_bytes = b.STAGE_TRAFFIC["bytes_per_launch"]
    got = b.stage_measured(n, "bytes_per_launch")
    # either the sources are the measured ones, or the figure is withheld
    assert got in (want_bytes, None)
    assert b.stage_measured(n + 1, "bytes_per_launch") is None      # other grid
    monkeypatch.setitem(b.STAGE_TRAFFIC, "sha256", "0" * 64)      # other sources
    assert b.stage_measured(n, "bytes_per_launch") is None
    assert b.stage_measured(n, "valu_insts_per_launch") is None


def test_host_cpu_description():
    b = _bench_module()
    h = b.host_cpu()
    assert set(h) == {"model", "logical_cpus"}
    assert h["logical_cpus"] is None or h["logical_cpus"] >= 1
