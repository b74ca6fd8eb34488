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
    for w, fig in b.STAGE_COUNTERS["workloads"].items():
        got = b.stage_measured(w, "bytes_per_launch")
        # either the sources are the measured ones, or the figure is withheld
        assert got in (fig["bytes_per_launch"], None)
    assert b.stage_measured("some_other_workload", "bytes_per_launch") is None
    monkeypatch.setitem(b.STAGE_COUNTERS, "sha256", "0" * 64)      # other sources
    for w in b.STAGE_COUNTERS["workloads"]:
        assert b.stage_measured(w, "bytes_per_launch") is None
        assert b.stage_measured(w, "valu_insts_per_launch") is None


def test_roofline_units():
    b = _bench_module()
    # 1210 flops per cell-stage (Cartesian, uniform gravity); the polytrope adds
    # its cylindrical sources and the pressure floor's primitives
    assert b.FLOPS_PER_CELL_STAGE == 1210
    assert b.FLOPS_PER_CELL_STAGE_CYL_FLOORS == 1249
    assert b.BYTES_PER_CELL_STEP == 256 and b.BYTES_PER_CELL_STEP_FIELD == 304


def test_golden_digest_lookup():
    b = _bench_module()
    assert b.golden_state_digest("no_such_workload", 10) is None
    d = b.golden_state_digest("polytrope_1024", 1000)
    assert d is None or len(d) == 64


def test_host_cpu_description():
    b = _bench_module()
    h = b.host_cpu()
    assert set(h) == {"model", "logical_cpus"}
    assert h["logical_cpus"] is None or h["logical_cpus"] >= 1
