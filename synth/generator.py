"""Seeded synthetic PT2 workloads (integrals, variational space, coefficient draws).

This module draws random numbers and does bookkeeping on bit strings; it holds
none of the perturbative method's arithmetic (no Hamiltonian matrix element,
no screening, no energy).  The two quantities of a workload that need the
Hamiltonian -- the MP1-like amplitudes of the doubles of the Hartree-Fock
determinant and E0 = <c|H|c> -- are supplied from outside through
`assemble_coefficients` (they are computed by the CPU reference and stored by
`synth/make_inputs.py`).

Workload recipe (the paper's Cu and Cr2 integrals and wavefunctions are not
available, so seeded synthetic inputs of the same shapes stand in for them):

* one-electron integrals: h_pp = -2 + 0.1 p (p is 0-based); for p < q,
  h_pq ~ N(0, 0.05^2) exp(-|p-q|/8), mirrored;
* two-electron integrals in chemists' notation,
  (pq|rs) = sum_{L < 2n} B^L_pq B^L_rs with B^L_pq = B^L_qp drawn on p <= q as
  N(0,1) * 0.3 exp(-|p-q|/6) / sqrt(2n); the sum is formed on canonical pair
  indices and mirrored, so all eight index permutations agree bit for bit and
  the supermatrix is positive semidefinite;
* determinants: the Hartree-Fock determinant (lowest n_sigma orbitals of each
  spin) first, then random excitations of it: level l uniform in
  {1..max_level}, split l = l_alpha + l_beta uniformly over feasible splits,
  holes and particles uniform without replacement; duplicates dropped in
  order of first appearance until n_var determinants are unique;
* coefficients: HF 0.9, doubles of HF get an MP1-like amplitude supplied by
  the caller, everything else N(0, 1e-3^2); the vector is normalised with an
  exactly rounded sum of squares.

Determinant layout: uint64 [N, 4] = (alpha_lo, alpha_hi, beta_lo, beta_hi);
orbital p of a spin sits at bit (p & 63) of word (p >> 6) of that spin
(paper, section V.A, determinant representation).

Everything here is elementwise IEEE arithmetic or libm calls on scalars, so
the same seed gives the same bits on any x86-64 host with this image.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# Workload table (sizes of the five standard workloads)
# ---------------------------------------------------------------------------


@dataclass(frozen=True)
class Workload:
    name: str
    n_orb: int
    n_alpha: int
    n_beta: int
    n_var: int
    max_level: int
    eps2: float            # deterministic threshold (epsilon_2 or epsilon_2^d)
    seed: int
    eps2_sto: float = 0.0  # stochastic threshold (epsilon_2), sample workloads
    n_samples: int = 0
    n_draws: int = 0
    draw_seed: int = 0
    fd_seed: int = 0
    description: str = ""


WORKLOADS = {
    "w0": Workload("w0", 12, 4, 4, 1000, 3, 0.0, 0,
                   description="deterministic FP64 PT2, (4a,4b) in 12 orbitals, N_var=1000, eps2=0"),
    "w1": Workload("w1", 40, 8, 8, 50_000, 3, 1e-5, 1,
                   description="deterministic PT2, (8a,8b) in 40 orbitals, N_var=5e4, eps2=1e-5, FP64 vs FP32c"),
    "w2": Workload("w2", 30, 6, 6, 20_000, 3, 1e-6, 2, fd_seed=102,
                   description="gradient dE2/dc, dE2/dE0, (6a,6b) in 30 orbitals, N_var=2e4, eps2=1e-6"),
    "w3": Workload("w3", 76, 14, 14, 1_000_000, 4, 2e-5, 3, eps2_sto=1e-7,
                   n_samples=256, n_draws=2000, draw_seed=1003,
                   description="semistochastic PT2, (14a,14b) in 76 orbitals, N_var=1e6"),
    "w4": Workload("w4", 76, 14, 14, 10_000_000, 4, 1e-5, 4, eps2_sto=5e-8,
                   n_samples=512, n_draws=4000, draw_seed=1004,
                   description="semistochastic PT2 + gradient, (14a,14b) in 76 orbitals, N_var=1e7"),
}


# ---------------------------------------------------------------------------
# Integrals
# ---------------------------------------------------------------------------


def _pair_index(n: int) -> np.ndarray:
    """Canonical pair index P(p,q) = max*(max+1)/2 + min for an n x n grid."""
    p = np.arange(n)[:, None]
    q = np.arange(n)[None, :]
    hi = np.maximum(p, q)
    lo = np.minimum(p, q)
    return (hi * (hi + 1) // 2 + lo).astype(np.int64)


def make_integrals(n: int, rng: np.random.Generator):
    """Return (h1 [n,n] f64, eri [n,n,n,n] f64) per the recipe above."""
    # decay factors through libm on scalars (no vectorised transcendental code)
    dec8 = np.array([math.exp(-d / 8.0) for d in range(n)])
    dec6 = np.array([math.exp(-d / 6.0) for d in range(n)])

    h1 = np.zeros((n, n))
    iu = np.triu_indices(n, k=1)                     # p < q, row major
    z = rng.standard_normal(len(iu[0]))
    vals = z * 0.05 * dec8[iu[1] - iu[0]]
    h1[iu] = vals
    h1[(iu[1], iu[0])] = vals
    h1[np.arange(n), np.arange(n)] = -2.0 + 0.1 * np.arange(n)

    nl = 2 * n
    npair = n * (n + 1) // 2
    # pairs in canonical order P = p*(p+1)/2 + q with q <= p
    pp = np.concatenate([np.full(p + 1, p) for p in range(n)])
    qq = np.concatenate([np.arange(p + 1) for p in range(n)])
    scale = 0.3 * dec6[pp - qq] / math.sqrt(nl)
    bmat = rng.standard_normal((nl, npair)) * scale[None, :]
    # M[P,R] = sum_L B[L,P] B[L,R], accumulated elementwise in L order
    m = np.zeros((npair, npair))
    for lvec in bmat:
        m += np.multiply.outer(lvec, lvec)
    # outer(v,v) is symmetric bit for bit, and so is every partial sum
    pidx = _pair_index(n)
    eri = m[pidx[:, :, None, None], pidx[None, None, :, :]]
    return np.ascontiguousarray(h1), np.ascontiguousarray(eri)


# ---------------------------------------------------------------------------
# Determinants
# ---------------------------------------------------------------------------


def occ_to_words(occ_rows: np.ndarray, valid: np.ndarray | None = None) -> np.ndarray:
    """Pack rows of orbital indices (< 128) into [rows, 2] uint64 words."""
    rows = occ_rows.shape[0]
    out = np.zeros((rows, 2), dtype=np.uint64)
    for k in range(occ_rows.shape[1]):
        o = occ_rows[:, k].astype(np.uint64)
        bit = np.left_shift(np.uint64(1), o & np.uint64(63))
        if valid is not None:
            bit = np.where(valid[:, k], bit, np.uint64(0))
        word = (o >> np.uint64(6)).astype(np.int64)
        out[word == 0, 0] |= bit[word == 0]
        out[word == 1, 1] |= bit[word == 1]
    return out


def hf_det(n_alpha: int, n_beta: int) -> np.ndarray:
    a = occ_to_words(np.arange(n_alpha)[None, :])[0]
    b = occ_to_words(np.arange(n_beta)[None, :])[0]
    return np.array([a[0], a[1], b[0], b[1]], dtype=np.uint64)


def _random_subset(rng, rows: int, pool: int, take: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Per row, `take[row]` distinct indices of range(pool), uniform."""
    if pool == 0:
        return np.zeros((rows, 0), dtype=np.int64), np.zeros((rows, 0), dtype=bool)
    keys = rng.random((rows, pool))
    perm = np.argsort(keys, axis=1, kind="stable")
    # only the first max(take) columns can be selected
    kmax = int(min(pool, max(int(take.max()), 1)))
    perm = perm[:, :kmax]
    valid = np.arange(kmax)[None, :] < take[:, None]
    return perm, valid


def _excite_spin(rng, rows: int, n: int, nsig: int, lev: np.ndarray) -> np.ndarray:
    """Return [rows, 2] words for spin strings excited from the lowest nsig."""
    holes, hv = _random_subset(rng, rows, nsig, lev)
    parts, pv = _random_subset(rng, rows, n - nsig, lev)
    occ = np.tile(np.arange(nsig), (rows, 1))
    base = occ_to_words(occ)
    hole_bits = occ_to_words(holes, hv) if nsig else np.zeros((rows, 2), np.uint64)
    part_bits = occ_to_words(parts + nsig, pv) if n - nsig else np.zeros((rows, 2), np.uint64)
    return (base & ~hole_bits) | part_bits


def make_dets(n: int, na: int, nb: int, n_var: int, max_level: int, rng: np.random.Generator,
              progress=None):
    """Return (dets uint64 [n_var,4], level int8 [n_var]); HF first.
    progress(have, n_var), if given, is called after each batch of draws."""
    va, vb = n - na, n - nb
    ma, mb = min(na, va), min(nb, vb)
    hf = hf_det(na, nb)
    dets = [hf[None, :]]
    levels = [np.zeros(1, dtype=np.int8)]
    have = 1
    seen = {hf.tobytes()}
    while have < n_var:
        rows = min(max(1024, 2 * (n_var - have)), 1 << 21)
        lev = rng.integers(1, max_level + 1, size=rows)
        lo = np.maximum(0, lev - mb)
        hi = np.minimum(lev, ma)
        ok = lo <= hi
        u = rng.random(rows)
        la = lo + np.floor(u * (hi - lo + 1)).astype(np.int64)
        la = np.minimum(la, hi)
        lb = lev - la
        aw = _excite_spin(rng, rows, n, na, np.where(ok, la, 0))
        bw = _excite_spin(rng, rows, n, nb, np.where(ok, lb, 0))
        cand = np.concatenate([aw, bw], axis=1)
        for r in np.nonzero(ok)[0]:
            key = cand[r].tobytes()
            if key in seen:
                continue
            seen.add(key)
            dets.append(cand[r][None, :])
            levels.append(np.array([lev[r]], dtype=np.int8))
            have += 1
            if have == n_var:
                break
        if progress is not None:
            progress(have, n_var)
    return np.ascontiguousarray(np.concatenate(dets)), np.concatenate(levels)


def double_of_hf_mask(levels: np.ndarray) -> np.ndarray:
    return levels == 2


# ---------------------------------------------------------------------------
# Coefficients
# ---------------------------------------------------------------------------


def noise_values(n_var: int, rng: np.random.Generator) -> np.ndarray:
    return rng.standard_normal(n_var) * 1e-3


def assemble_coefficients(noise: np.ndarray, levels: np.ndarray, mp1: np.ndarray) -> np.ndarray:
    """HF 0.9, doubles of HF take `mp1` (in determinant order), others noise; normalised."""
    raw = noise.copy()
    dmask = double_of_hf_mask(levels)
    if mp1.shape[0] != int(dmask.sum()):
        raise ValueError("mp1 length does not match the number of doubles of HF")
    raw[dmask] = mp1
    raw[0] = 0.9
    norm = math.sqrt(math.fsum((raw * raw).tolist()))
    return raw / norm


# ---------------------------------------------------------------------------
# Workload bundle
# ---------------------------------------------------------------------------


@dataclass
class Inputs:
    wl: Workload
    h1: np.ndarray
    eri: np.ndarray
    dets: np.ndarray
    levels: np.ndarray
    noise: np.ndarray
    c: np.ndarray | None = None
    e0: float | None = None
    extra: dict = field(default_factory=dict)


def make_raw(wl: Workload | str, n_var: int | None = None, progress=None) -> Inputs:
    """Draw integrals, determinants and noise for a workload (no c, no E0)."""
    if isinstance(wl, str):
        wl = WORKLOADS[wl]
    rng = np.random.default_rng(wl.seed)
    h1, eri = make_integrals(wl.n_orb, rng)
    nv = wl.n_var if n_var is None else n_var
    dets, levels = make_dets(wl.n_orb, wl.n_alpha, wl.n_beta, nv, wl.max_level, rng, progress)
    noise = noise_values(nv, rng)
    return Inputs(wl, h1, eri, dets, levels, noise)


def make_small(n: int, na: int, nb: int, n_var: int, max_level: int, seed: int) -> Inputs:
    """Same recipe at an arbitrary (small) shape, for tests."""
    wl = Workload(f"small_{n}_{na}_{nb}_{n_var}_{seed}", n, na, nb, n_var, max_level, 0.0, seed)
    return make_raw(wl)


def draws_uniform_u64(seed: int, count: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2**63, size=count, dtype=np.int64).astype(np.uint64)


def fd_coordinates(seed: int, n_var: int, count: int = 64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_var, size=min(count, n_var), replace=False))
