"""The benchmark's achievable-peak probe (a measurement library of its own,
outside the solver's ABI): a positive FP64 fma rate below the vector peak
(78.6 TFLOP/s) by construction of its instruction stream, and well above a
host rate; invalid arguments are refused before any launch."""
import ctypes
import importlib.util
import os

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_fma_probe_reports_a_plausible_rate():
    import torch
    b = _bench()
    r = b.fma_probe_rate(torch, 2000)
    assert 1e12 < r < 80e12, r
    lib = ctypes.CDLL(b.PROBE_LIB)
    out = ctypes.c_double()
    assert lib.hydro_probe_fma_rate(0, None, ctypes.byref(out)) == -1
    assert lib.hydro_probe_fma_rate(10, None, None) == -1
