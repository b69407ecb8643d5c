"""Writes the stored oracle results of the 76-orbital, 10^6-determinant
semistochastic workload (w3) used by the full-size GPU parity tests.

Every stored value comes from the CPU oracle (`oracle/`) on the seeded w3
inputs; nothing here touches the GPU library.

  python tests/golden/make_w3_oracle.py det       -> tests/golden/w3_det_oracle.json
  python tests/golden/make_w3_oracle.py samples   -> tests/golden/w3_samples_oracle.json

det: the deterministic screened PT2 at eps2^d (paper, section II.B, screened
PT2 equation) over all of V: E2, dE2/dE0, the term and determinant counts, a
SHA-256 digest of the perturbative determinants in ascending key order with
their kept-term counts, and 1024 of them (evenly spaced in that order) with
A_a, E0 - H_aa and the count.

samples: the per-sample stochastic estimates S_s(eps2) - S_s(eps2^d)
(stochastic PT2 equation) of 256 samples of 2000 draws made by the oracle's
alias sampler from the seed (draws of sample s, draw k: outputs 2(s N_d + k) + 1
and + 2 of SplitMix64 seeded with the workload's draw seed), with a digest of
the draws, and per sample sum_a |contribution_a| / |E0 - H_aa|, the
estimate's first-order sensitivity to the rounding of the denominators.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import ref  # noqa: E402
from synth import store  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_SAMPLED = 1024


def unique_digest(keys: np.ndarray, counts: np.ndarray) -> str:
    """SHA-256 of the keys ([n, 4] little-endian uint64, ascending in the
    order (word 3, word 2, word 1, word 0)) followed by the counts (int64)."""
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(keys, dtype="<u8").tobytes())
    h.update(np.ascontiguousarray(counts, dtype="<i8").tobytes())
    return h.hexdigest()


def run_det(x) -> dict:
    wl = x.wl
    t = time.time()
    o = ref.pt2_det(wl.n_orb, wl.n_alpha, wl.n_beta, x.h1, x.eri, x.dets, x.c, x.e0, wl.eps2,
                    unique=True)
    dt = time.time() - t
    nu = o.n_unique
    pick = (np.arange(N_SAMPLED, dtype=np.int64) * nu) // N_SAMPLED
    return {
        "workload": "w3",
        "eps2": wl.eps2,
        "e0": x.e0,
        "e2": o.e2,
        "de2_de0": o.de2_de0,
        "min_abs_denom": o.min_abs_denom,
        "n_terms": o.n_terms,
        "n_terms_gen": o.n_terms_gen,
        "n_unique": nu,
        "n_intruder": o.n_intruder,
        "n_zero_denom": o.n_zero_denom,
        "unique_digest": unique_digest(o.keys, o.counts),
        "sampled": {
            "index": pick.tolist(),
            "keys": [[f"{int(w):016x}" for w in o.keys[k]] for k in pick],
            "A": [float(o.A[k]) for k in pick],
            "D": [float(o.D[k]) for k in pick],
            "count": [int(o.counts[k]) for k in pick],
        },
        "oracle_seconds": dt,
        "oracle_threads": ref.max_threads(),
    }


def run_samples(x) -> dict:
    wl = x.wl
    t = time.time()
    draws = ref.alias_draws(x.c, wl.n_samples, wl.n_draws, wl.draw_seed)
    out, cnt, sens = ref.pt2_sample_counts(wl.n_orb, wl.n_alpha, wl.n_beta, x.h1, x.eri, x.dets, x.c, x.e0,
                                           wl.eps2_sto, wl.eps2, draws, sens=True)
    dt = time.time() - t
    return {
        "workload": "w3",
        "eps2": wl.eps2_sto,
        "eps2_d": wl.eps2,
        "e0": x.e0,
        "n_samples": wl.n_samples,
        "n_draws": wl.n_draws,
        "seed": wl.draw_seed,
        "draws_digest": hashlib.sha256(np.ascontiguousarray(draws, dtype="<u4").tobytes()).hexdigest(),
        "per_sample": [float(v) for v in out],
        "per_sample_terms": [int(v) for v in cnt],
        "per_sample_sensitivity": [float(v) for v in sens],
        "n_terms": int(cnt.sum()),
        "mean": float(np.mean(out)),
        "oracle_seconds": dt,
        "oracle_threads": ref.max_threads(),
    }


def main(argv):
    part = argv[1] if len(argv) > 1 else "det"
    x = store.load("w3")
    if part == "det":
        res, name = run_det(x), "w3_det_oracle.json"
    elif part == "samples":
        res, name = run_samples(x), "w3_samples_oracle.json"
    else:
        raise SystemExit(f"unknown part {part!r} (det | samples)")
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(res, f, indent=1)
    print(f"wrote {name} ({res['oracle_seconds']:.0f} s)")


if __name__ == "__main__":
    main(sys.argv)
