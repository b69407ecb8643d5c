"""Test-side assembly of complete workloads (generator draws + reference helpers).

The seeded generator draws integrals, determinants and noise; the two
Hamiltonian-dependent inputs (MP1-like amplitudes of the doubles of HF and
E0 = <c|H|c>) come from the CPU reference.  Tests may call the reference; the
product code never does.
"""
from __future__ import annotations

import numpy as np

from oracle import ref
from synth import generator as G


def complete(x: G.Inputs) -> G.Inputs:
    wl = x.wl
    n, na, nb = wl.n_orb, wl.n_alpha, wl.n_beta
    mask = G.double_of_hf_mask(x.levels)
    amp = ref.mp1(n, na, nb, x.h1, x.eri, x.dets, mask, x.dets[0])
    x.c = G.assemble_coefficients(x.noise, x.levels, amp)
    x.e0 = ref.energy(n, na, nb, x.h1, x.eri, x.dets, x.c)
    return x


def small(n, na, nb, n_var, max_level=3, seed=0):
    return complete(G.make_small(n, na, nb, n_var, max_level, seed))


def workload(name, n_var=None):
    return complete(G.make_raw(name, n_var=n_var))
