"""Loads complete workloads: generator draws plus the stored inputs written by
`synth/make_inputs.py` (MP1-like amplitudes and E0)."""
from __future__ import annotations

import hashlib
import os

import numpy as np

from synth import generator as G

_DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data")


def data_path(name: str) -> str:
    return os.path.join(_DATA, f"{name}.npz")


def fingerprint(a: np.ndarray) -> np.ndarray:
    h = hashlib.sha256(np.ascontiguousarray(a).tobytes()).digest()
    return np.frombuffer(h, dtype=np.uint8).copy()


def load(name: str, check: bool = True, progress=None) -> G.Inputs:
    """Regenerate workload `name` and attach its stored c and E0."""
    x = G.make_raw(name, progress=progress)
    with np.load(data_path(name), allow_pickle=False) as z:
        amp = z["mp1"]
        x.e0 = float(z["e0"])
        fps = {k: z[k] for k in ("fp_dets", "fp_eri", "fp_c")}
    x.c = G.assemble_coefficients(x.noise, x.levels, amp)
    if check:
        got = {"fp_dets": fingerprint(x.dets), "fp_eri": fingerprint(x.eri),
               "fp_c": fingerprint(x.c)}
        for k, v in fps.items():
            if not np.array_equal(v, got[k]):
                raise RuntimeError(f"workload {name}: regenerated {k[3:]} differs from the stored one")
    return x
