"""The stored oracle digests of the full-length workloads (tests/golden/
full_length.json, written by tests/golden/make_full_length.py) reproduce on
this host: every initial state and gravity field digests to the stored value,
and the oracle re-derives the shear layer's first checkpoint (100 steps at
512^2) with the stored time, step records and state."""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_1507_08549_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "full_length.json")


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<f8").tobytes()).hexdigest()


@pytest.fixture(scope="module")
def golden():
    return json.load(open(GOLDEN))["workloads"]


def test_all_workloads_present(golden):
    assert set(golden) == {"shear_layer_512", "heavy_over_light_256x1024", "polytrope_1024",
                           "sine_mode_shear_layer_1024"}
    for name, w in golden.items():
        assert len(w["checkpoints"]) == w["steps"] // w["every"], name
        assert [c["step"] for c in w["checkpoints"]] == list(range(w["every"], w["steps"] + 1, w["every"]))


def test_initial_states_reproduce(golden):
    prm, U = inputs.kelvin_helmholtz(512, seed=2)
    assert digest(U) == golden["shear_layer_512"]["initial_state"]
    prm, U = inputs.rayleigh_taylor()
    assert digest(U) == golden["heavy_over_light_256x1024"]["initial_state"]
    prm, U, g = inputs.polytrope(1024)
    assert digest(U) == golden["polytrope_1024"]["initial_state"]
    assert digest(g) == golden["polytrope_1024"]["gravity"]
    prm = inputs.kh_sine_params(1024)
    U = inputs.kh_sine_state(inputs.kh_sine_amplitudes(), prm)
    assert digest(U) == golden["sine_mode_shear_layer_1024"]["initial_state"]


def test_first_checkpoint_reproduces(oracle_mod, golden):
    w = golden["shear_layer_512"]
    cp = w["checkpoints"][0]
    prm, U0 = inputs.kelvin_helmholtz(512, seed=2)
    U, t, dts, als = oracle_mod.Oracle(prm).run(U0, w["every"])
    assert t == float.fromhex(cp["t"])
    assert digest(dts) == cp["dt"] and digest(als) == cp["alpha"]
    assert digest(U) == cp["state"]
