"""Writes the Hamiltonian-dependent workload inputs to synth/data/<name>.npz.

For each workload the seeded generator draws integrals, determinants and
noise; the CPU reference then supplies the MP1-like amplitudes of the doubles
of the Hartree-Fock determinant and E0 = <c|H|c>.  The stored file holds those
two items plus fingerprints of the generated arrays, so that a later run can
check that it regenerated the same workload.

Usage: python -m synth.make_inputs w0 w1 w2 w3
"""
from __future__ import annotations

import sys

import numpy as np

from oracle import ref
from synth import generator as G
from synth.store import data_path, fingerprint


def make(name: str) -> None:
    x = G.make_raw(name)
    wl = x.wl
    n, na, nb = wl.n_orb, wl.n_alpha, wl.n_beta
    mask = G.double_of_hf_mask(x.levels)
    amp = ref.mp1(n, na, nb, x.h1, x.eri, x.dets, mask, x.dets[0])
    c = G.assemble_coefficients(x.noise, x.levels, amp)
    if len(c) <= 100_000:
        e0 = ref.energy(n, na, nb, x.h1, x.eri, x.dets, c)
    else:
        e0, _ = ref.energy_cores(n, na, nb, x.h1, x.eri, x.dets, c)
    np.savez(data_path(name), mp1=amp, e0=np.float64(e0),
             fp_dets=fingerprint(x.dets), fp_eri=fingerprint(x.eri), fp_c=fingerprint(c))
    print(f"{name}: n_var={len(c)} doubles={len(amp)} E0={e0!r}")


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["w0", "w1", "w2"]:
        make(nm)
