"""Write tests/golden/full_length.json: digests of the oracle's states along the
four benchmark workloads at their full lengths, and the growth of small
initial differences under the oracle's own FP64 arithmetic.

Calls only the oracle (oracle/) and the seeded input generators.  Every
digest is SHA-256 of float64 little-endian C-order bytes.  For each workload:
the initial state (and gravity field), then at every checkpoint the time
reached (as a hex float), the state, and the time-step and LF-speed records of
the steps since the previous checkpoint.

Growth of initial differences (no device involved), reported beside the
FP32-bulk errors: the shear layer from its initial state with m_y moved by one
ulp in every cell, and each workload from its initial state rounded to FP32
(the size of difference the FP32-bulk form makes in its first step), each
compared with the unperturbed oracle run as the relative L1 density difference
at every checkpoint.

Run:  python tests/golden/make_full_length.py [workload ...]   (minutes: the
oracle runs about 1e9 cell-updates per workload; it uses every core).
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1507_08549_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "full_length.json")


def digest(a) -> str:
    a = np.ascontiguousarray(a, dtype="<f8")
    return hashlib.sha256(a.tobytes()).hexdigest()


def workload(name):
    """(params, initial state, gravity or None, steps, checkpoint interval)."""
    if name == "shear_layer_512":
        prm, U0 = inputs.kelvin_helmholtz(512, seed=2)
        return prm, U0, None, 2000, 100
    if name == "heavy_over_light_256x1024":
        prm, U0 = inputs.rayleigh_taylor()
        return prm, U0, None, 5000, 250
    if name == "polytrope_1024":
        prm, U0, grav = inputs.polytrope(1024)
        return prm, U0, grav, 1000, 50
    if name == "sine_mode_shear_layer_1024":
        prm = inputs.kh_sine_params(1024)
        return prm, inputs.kh_sine_state(inputs.kh_sine_amplitudes(), prm), None, 500, 50
    raise KeyError(name)


WORKLOADS = ("shear_layer_512", "heavy_over_light_256x1024", "polytrope_1024",
             "sine_mode_shear_layer_1024")
# initial differences whose growth is recorded, per workload
PERTURBED = {
    "shear_layer_512": ("my_one_ulp", "fp32_rounded"),
    "heavy_over_light_256x1024": ("fp32_rounded",),
    "polytrope_1024": ("fp32_rounded",),
}


def perturb(U0, kind):
    U = U0.copy()
    if kind == "my_one_ulp":
        U[2] = np.nextafter(U[2], np.inf)
    elif kind == "fp32_rounded":
        U = U.astype(np.float32).astype(np.float64)
    else:
        raise KeyError(kind)
    return U


def l1_rho(a, b):
    return float(np.abs(a[0] - b[0]).sum() / np.abs(b[0]).sum())


def run_one(name, log=print):
    prm, U0, grav, n, every = workload(name)
    o = oracle.Oracle(prm, gravity=grav)
    kinds = PERTURBED.get(name, ())
    rec = {"steps": n, "every": every, "nx": prm["nx"], "ny": prm["ny"],
           "initial_state": digest(U0), "gravity": None if grav is None else digest(grav),
           "checkpoints": []}
    W, t = U0.copy(), 0.0
    P = {k: perturb(U0, k) for k in kinds}
    tp = {k: 0.0 for k in kinds}
    growth = {k: [] for k in kinds}
    t_start = time.time()
    for done in range(every, n + 1, every):
        W, t, dts, als = o.run(W, every, t0=t)
        assert len(dts) == every
        rec["checkpoints"].append({"step": done, "t": float(t).hex(), "state": digest(W),
                                   "dt": digest(dts), "alpha": digest(als)})
        for k in kinds:
            P[k], tp[k], _, _ = o.run(P[k], every, t0=tp[k])
            growth[k].append(l1_rho(P[k], W))
        log(f"{name}: {done}/{n} steps ({time.time() - t_start:.0f} s)"
            + "".join(f", {k} {growth[k][-1]:.3e}" for k in kinds))
    if kinds:
        rec["initial_difference_growth"] = {
            k: {"l1_rho": growth[k],
                "initial_l1_rho": l1_rho(perturb(U0, k), U0)} for k in kinds}
    return rec


def main(names):
    oracle.build(force=False)
    oracle.set_threads(os.cpu_count() or 1)
    data = {}
    if os.path.exists(OUT):
        data = json.load(open(OUT))
    data["format"] = ("sha256 of float64 little-endian C-order bytes; t as a hex float; "
                      "dt [every], alpha [every][3][2] (ax, ay per stage) of the steps since the "
                      "previous checkpoint")
    data.setdefault("workloads", {})
    for name in names:
        data["workloads"][name] = run_one(name, log=lambda s: print(s, flush=True))
        data["workloads"] = {k: data["workloads"][k] for k in WORKLOADS if k in data["workloads"]}
        tmp = OUT + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1)
            f.write("\n")
        os.replace(tmp, OUT)


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
