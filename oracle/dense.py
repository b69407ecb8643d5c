"""Tiny full-CI checker (TEST INFRASTRUCTURE).

Builds the Hamiltonian of a small full CI space by applying the second
quantised operator

    H = sum_{pq,s} h_pq a+_{ps} a_{qs}
        + 1/2 sum_{pqrs,s,t} (pq|rs) a+_{ps} a+_{rt} a_{st} a_{qs}

to occupation-number bit strings, with the fermion sign of every creation and
annihilation counted explicitly.  It knows nothing of Slater-Condon rules,
excitation classes or phases, so it pins those parts of the C++ reference.

Spin orbitals are ordered alpha_0..alpha_{n-1}, beta_0..beta_{n-1}; a
determinant is a Python int with bit k set when spin orbital k is occupied.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def fci_space(n: int, na: int, nb: int) -> list[int]:
    dets = []
    for a in itertools.combinations(range(n), na):
        for b in itertools.combinations(range(n), nb):
            d = 0
            for p in a:
                d |= 1 << p
            for p in b:
                d |= 1 << (n + p)
            dets.append(d)
    return dets


def to_words(d: int, n: int) -> np.ndarray:
    """Spin-orbital bit string -> (alpha_lo, alpha_hi, beta_lo, beta_hi)."""
    a = d & ((1 << n) - 1)
    b = d >> n
    m = (1 << 64) - 1
    return np.array([a & m, a >> 64, b & m, b >> 64], dtype=np.uint64)


def from_words(w, n: int) -> int:
    a = int(w[0]) | (int(w[1]) << 64)
    b = int(w[2]) | (int(w[3]) << 64)
    return a | (b << n)


def _annihilate(d: int, k: int):
    if not (d >> k) & 1:
        return None, 0
    sign = -1 if bin(d & ((1 << k) - 1)).count("1") & 1 else 1
    return d ^ (1 << k), sign


def _create(d: int, k: int):
    if (d >> k) & 1:
        return None, 0
    sign = -1 if bin(d & ((1 << k) - 1)).count("1") & 1 else 1
    return d | (1 << k), sign


def apply_h(d: int, n: int, h1: np.ndarray, eri: np.ndarray) -> dict[int, float]:
    """H|d> as {det: amplitude}."""
    out: dict[int, float] = {}
    nso = 2 * n
    occ = [k for k in range(nso) if (d >> k) & 1]
    # one-body: a+_p a_q, same spin
    for q in occ:
        d1, s1 = _annihilate(d, q)
        sp = q // n
        for pp in range(n):
            p = sp * n + pp
            d2, s2 = _create(d1, p)
            if d2 is None:
                continue
            v = h1[pp, q % n]
            if v != 0.0:
                out[d2] = out.get(d2, 0.0) + s1 * s2 * v
    # two-body: 1/2 (pq|rs) a+_p a+_r a_s a_q ; operators act right to left
    for q in occ:
        d1, s1 = _annihilate(d, q)
        for s in occ:
            if s == q:
                continue
            d2, s2 = _annihilate(d1, s)
            sq, ss = q // n, s // n
            for rr in range(n):
                r = ss * n + rr
                d3, s3 = _create(d2, r)
                if d3 is None:
                    continue
                for pp in range(n):
                    p = sq * n + pp
                    d4, s4 = _create(d3, p)
                    if d4 is None:
                        continue
                    v = eri[pp, q % n, rr, s % n]
                    if v != 0.0:
                        out[d4] = out.get(d4, 0.0) + 0.5 * s1 * s2 * s3 * s4 * v
    return out


def hamiltonian(n: int, na: int, nb: int, h1: np.ndarray, eri: np.ndarray):
    """(dets list, index dict, dense H) of the full CI space."""
    dets = fci_space(n, na, nb)
    index = {d: k for k, d in enumerate(dets)}
    H = np.zeros((len(dets), len(dets)))
    for j, d in enumerate(dets):
        for t, v in apply_h(d, n, h1, eri).items():
            H[index[t], j] += v
    return dets, index, H


def e2_dense(H: np.ndarray, v_idx, c: np.ndarray, e0: float, eps2: float) -> float:
    """Screened EN-PT2 by dense linear algebra on a full CI Hamiltonian.

    v_idx: indices of V in the FCI basis; c: coefficients on V.
    mask_ai = |H_ai c_i| > eps2; A = (H_PV * mask) c; E2 = sum A^2 / (e0 - H_aa)
    over a outside V with at least one kept term.
    """
    v_idx = np.asarray(v_idx)
    outside = np.setdiff1d(np.arange(H.shape[0]), v_idx)
    hpv = H[np.ix_(outside, v_idx)]
    mask = np.abs(hpv * c[None, :]) > eps2
    A = (hpv * mask) @ c
    has = mask.any(axis=1)
    d = e0 - np.diag(H)[outside]
    return float(np.sum(A[has] ** 2 / d[has]))


def n_excitations_closed_form(n: int, na: int, nb: int) -> int:
    """Singles + doubles of one determinant: n_s v_s per spin, C(n_s,2) C(v_s,2)
    per spin, and n_a v_a n_b v_b opposite-spin doubles."""
    va, vb = n - na, n - nb
    return (na * va + nb * vb + math.comb(na, 2) * math.comb(va, 2)
            + math.comb(nb, 2) * math.comb(vb, 2) + na * va * nb * vb)
