"""ctypes front end of the brute-force CPU reference (TEST INFRASTRUCTURE).

Every function follows the paper's section II.B definitions; see the header
of `pt2_oracle.cpp` for the conventions.  Inputs are numpy arrays:
h1 [n,n] f64, eri [n,n,n,n] f64 (chemists' (pq|rs)), dets uint64 [N,4]
(alpha_lo, alpha_hi, beta_lo, beta_hi), c [N] f64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB: another build of the same sources (the sanitizer test)
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle_pt2.so")
_lib = None

_d = C.c_double
_i = C.c_int
_i64 = C.c_int64
_p = C.c_void_p


def build():
    subprocess.run(["sh", os.path.join(_HERE, "build.sh")], check=True)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        L.oracle_last_error.restype = C.c_char_p
        L.oracle_hij.restype = _d
        L.oracle_hij.argtypes = [_i, _i, _i, _p, _p, _p, _p]
        L.oracle_diag.restype = _d
        L.oracle_diag.argtypes = [_i, _i, _i, _p, _p, _p]
        L.oracle_count_excitations.restype = _i64
        L.oracle_count_excitations.argtypes = [_i, _i, _i, _p, _p, _p]
        L.oracle_pt2_det.restype = _p
        L.oracle_pt2_det.argtypes = [_i, _i, _i, _p, _p, _p, _p, _i64, _d, _d, _i, C.POINTER(_i)]
        L.oracle_result_free.argtypes = [_p]
        L.oracle_result_scalars.argtypes = [_p, _p, _p]
        L.oracle_result_unique.argtypes = [_p, _p, _p, _p, _p]
        L.oracle_result_terms.argtypes = [_p, _p, _p, _p, _p]
        L.oracle_result_grad.argtypes = [_p, _p]
        L.oracle_result_fd_grad.argtypes = [_p, _p, _p, _i64, _d, _p]
        L.oracle_result_fd_de0.restype = _d
        L.oracle_result_fd_de0.argtypes = [_p, _d]
        L.oracle_pt2_at.restype = _i
        L.oracle_pt2_at.argtypes = [_i, _i, _i, _p, _p, _p, _p, _i64, _d, _d, _p, _i64,
                                    _p, _p, _p, _p]
        L.oracle_pt2_sample.restype = _i
        L.oracle_pt2_sample.argtypes = [_i, _i, _i, _p, _p, _p, _p, _i64, _d, _d, _d,
                                        C.c_int32, C.c_int32, _p, _p]
        L.oracle_pt2_sample_counts.restype = _i
        L.oracle_pt2_sample_counts.argtypes = [_i, _i, _i, _p, _p, _p, _p, _i64, _d, _d, _d,
                                               C.c_int32, C.c_int32, _p, _p, _p, _p]
        L.oracle_det_batch.restype = _i
        L.oracle_det_batch.argtypes = [_i, _i, _i, _p, _p, _p, _p, _i64, _d, _d, _d, _i, _i, _p, _p]
        L.oracle_pt2_sample_batched.restype = _i
        L.oracle_pt2_sample_batched.argtypes = [_i, _i, _i, _p, _p, _p, _p, _i64, _d, _d, _d, _i, _i,
                                                _p, _i, _p, _p]
        L.oracle_pt2_sample_frozen.restype = _i
        L.oracle_pt2_sample_frozen.argtypes = [_i, _i, _i, _p, _p, _p, _p, _p, _i64, _d, _d, _d,
                                               _i, _i, _p, _p]
        L.oracle_pt2_sample_grad.restype = _i
        L.oracle_pt2_sample_grad.argtypes = [_i, _i, _i, _p, _p, _p, _p, _i64, _d, _d, _d,
                                             _i, _i, _p, _p, _p, _p]
        L.oracle_energy.restype = _d
        L.oracle_energy.argtypes = [_i, _i, _i, _p, _p, _p, _p, _i64]
        L.oracle_terms_of.restype = _i64
        L.oracle_terms_of.argtypes = [_i, _i, _i, _p, _p, _p, _p, _i64, _d, _p, _i64, _p, _p, _p, _i64]
        L.oracle_energy_cores.restype = _d
        L.oracle_energy_cores.argtypes = [_i, _i, _i, _p, _p, _p, _p, _i64, _i, _i, _p]
        L.oracle_mp1.argtypes = [_i, _i, _i, _p, _p, _p, _p, _i64, _p, _p]
        L.oracle_hc_rows.restype = _i
        L.oracle_hc_rows.argtypes = [_i, _i, _i, _p, _p, _p, _p, _i64, _p, _i64, _p, _p]
        L.oracle_max_threads.restype = _i
        L.oracle_alias_last_error.restype = C.c_char_p
        L.oracle_splitmix64.restype = C.c_uint64
        L.oracle_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.oracle_alias_table.restype = _i
        L.oracle_alias_table.argtypes = [_p, _i64, _p, _p, _p, _p, _p, _p, _p]
        L.oracle_alias_draws.restype = _i
        L.oracle_alias_draws.argtypes = [_p, _i64, C.c_uint64, C.c_int32, C.c_int32, _p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _sys(h1, eri):
    h1 = np.ascontiguousarray(h1, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    return h1, eri


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle error {code}: {msg}")
        self.code = code


def hij(n, na, nb, h1, eri, a, i) -> float:
    h1, eri = _sys(h1, eri)
    a = np.ascontiguousarray(a, dtype=np.uint64)
    i = np.ascontiguousarray(i, dtype=np.uint64)
    return lib().oracle_hij(n, na, nb, _ptr(h1), _ptr(eri), _ptr(a), _ptr(i))


def diag(n, na, nb, h1, eri, d) -> float:
    h1, eri = _sys(h1, eri)
    d = np.ascontiguousarray(d, dtype=np.uint64)
    return lib().oracle_diag(n, na, nb, _ptr(h1), _ptr(eri), _ptr(d))


def count_excitations(n, na, nb, h1, eri, d) -> int:
    h1, eri = _sys(h1, eri)
    d = np.ascontiguousarray(d, dtype=np.uint64)
    return lib().oracle_count_excitations(n, na, nb, _ptr(h1), _ptr(eri), _ptr(d))


@dataclass
class DetResult:
    e2: float
    de2_de0: float
    min_abs_denom: float
    n_terms: int
    n_terms_gen: int
    n_unique: int
    n_intruder: int
    n_zero_denom: int
    keys: np.ndarray | None = None     # [n_unique, 4] ascending
    A: np.ndarray | None = None
    D: np.ndarray | None = None
    counts: np.ndarray | None = None
    term_keys: np.ndarray | None = None
    term_i: np.ndarray | None = None
    term_h: np.ndarray | None = None
    term_in_v: np.ndarray | None = None
    grad: np.ndarray | None = None
    fd: np.ndarray | None = None
    fd_de0: float | None = None


def pt2_det(n, na, nb, h1, eri, dets, c, e0, eps2, *, unique=True, terms=False, grad=False,
            fd_coords=None, fd_rel_step=1e-6, fd_de0_step=None) -> DetResult:
    """Screened deterministic PT2 by brute-force enumeration."""
    h1, eri = _sys(h1, eri)
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    L = lib()
    st = C.c_int(0)
    h = L.oracle_pt2_det(n, na, nb, _ptr(h1), _ptr(eri), _ptr(dets), _ptr(c), len(c),
                         float(e0), float(eps2), 1 if grad else 0, C.byref(st))
    if not h:
        raise OracleError(st.value, L.oracle_last_error().decode())
    try:
        dbl = np.zeros(3)
        cnt = np.zeros(5, dtype=np.int64)
        L.oracle_result_scalars(h, _ptr(dbl), _ptr(cnt))
        r = DetResult(float(dbl[0]), float(dbl[1]), float(dbl[2]), *[int(x) for x in cnt])
        if unique:
            nu = r.n_unique
            r.keys = np.zeros((nu, 4), dtype=np.uint64)
            r.A = np.zeros(nu)
            r.D = np.zeros(nu)
            r.counts = np.zeros(nu, dtype=np.int64)
            L.oracle_result_unique(h, _ptr(r.keys), _ptr(r.A), _ptr(r.D), _ptr(r.counts))
        if terms:
            nt = r.n_terms_gen
            r.term_keys = np.zeros((nt, 4), dtype=np.uint64)
            r.term_i = np.zeros(nt, dtype=np.uint32)
            r.term_h = np.zeros(nt)
            r.term_in_v = np.zeros(nt, dtype=np.uint8)
            L.oracle_result_terms(h, _ptr(r.term_keys), _ptr(r.term_i), _ptr(r.term_h),
                                  _ptr(r.term_in_v))
        if grad:
            r.grad = np.zeros(len(c))
            L.oracle_result_grad(h, _ptr(r.grad))
        if fd_coords is not None:
            co = np.ascontiguousarray(fd_coords, dtype=np.int64)
            r.fd = np.zeros(len(co))
            L.oracle_result_fd_grad(h, _ptr(c), _ptr(co), len(co), float(fd_rel_step), _ptr(r.fd))
        if fd_de0_step is not None:
            r.fd_de0 = L.oracle_result_fd_de0(h, float(fd_de0_step))
        return r
    finally:
        L.oracle_result_free(h)


def pt2_at(n, na, nb, h1, eri, dets, c, e0, eps2, alist):
    """A_a, D_a, kept-term count and V membership for the given determinants a."""
    h1, eri = _sys(h1, eri)
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    alist = np.ascontiguousarray(alist, dtype=np.uint64)
    m = alist.shape[0]
    A = np.zeros(m)
    D = np.zeros(m)
    cnt = np.zeros(m, dtype=np.int64)
    inv = np.zeros(m, dtype=np.uint8)
    lib().oracle_pt2_at(n, na, nb, _ptr(h1), _ptr(eri), _ptr(dets), _ptr(c), len(c), float(e0),
                        float(eps2), _ptr(alist), m, _ptr(A), _ptr(D), _ptr(cnt), _ptr(inv))
    return A, D, cnt, inv


def pt2_sample(n, na, nb, h1, eri, dets, c, e0, eps2, eps2_d, draws):
    """Per-sample S_s(eps2) - S_s(eps2_d) on explicit draws [ns, nd] (uint32)."""
    h1, eri = _sys(h1, eri)
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    draws = np.ascontiguousarray(draws, dtype=np.uint32)
    ns, nd = draws.shape
    out = np.zeros(ns)
    L = lib()
    st = L.oracle_pt2_sample(n, na, nb, _ptr(h1), _ptr(eri), _ptr(dets), _ptr(c), len(c),
                             float(e0), float(eps2), float(eps2_d), ns, nd, _ptr(draws), _ptr(out))
    if st:
        raise OracleError(st, L.oracle_last_error().decode())
    return out


def pt2_sample_counts(n, na, nb, h1, eri, dets, c, e0, eps2, eps2_d, draws, *, sens=False):
    """(per-sample estimates, per-sample kept terms with a outside V) on
    explicit draws; with sens=True also, per sample, sum_a |contribution_a| /
    |E0 - H_aa| (a change delta of every denominator moves the estimate by at
    most delta times this, to first order)."""
    h1, eri = _sys(h1, eri)
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    draws = np.ascontiguousarray(draws, dtype=np.uint32)
    ns, nd = draws.shape
    out = np.zeros(ns)
    cnt = np.zeros(ns, dtype=np.int64)
    sv = np.zeros(ns)
    L = lib()
    st = L.oracle_pt2_sample_counts(n, na, nb, _ptr(h1), _ptr(eri), _ptr(dets), _ptr(c), len(c),
                                    float(e0), float(eps2), float(eps2_d), ns, nd, _ptr(draws), _ptr(out),
                                    _ptr(cnt), _ptr(sv) if sens else None)
    if st:
        raise OracleError(st, L.oracle_last_error().decode())
    return (out, cnt, sv) if sens else (out, cnt)


def det_batch(n, na, nb, h1, eri, dets, c, e0, eps2, eps2_hi, n_batches, batch):
    """(sum e_a, sum e_a^2, number of a, kept terms) over the a of one hash
    batch, e_a = (A_a(eps2)^2 - A_a(eps2_hi)^2) / D_a."""
    h1, eri = _sys(h1, eri)
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    out = np.zeros(2)
    cnt = np.zeros(2, dtype=np.int64)
    L = lib()
    st = L.oracle_det_batch(n, na, nb, _ptr(h1), _ptr(eri), _ptr(dets), _ptr(c), len(c), float(e0),
                            float(eps2), float(eps2_hi), int(n_batches), int(batch), _ptr(out), _ptr(cnt))
    if st:
        raise OracleError(st, L.oracle_last_error().decode())
    return out[0], out[1], int(cnt[0]), int(cnt[1])


def pt2_sample_batched(n, na, nb, h1, eri, dets, c, e0, eps2, eps2_d, draws, n_batches, sample_batch):
    """Per-sample estimates keeping one hash batch of P per sample, times n_batches."""
    h1, eri = _sys(h1, eri)
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    draws = np.ascontiguousarray(draws, dtype=np.uint32)
    sb = np.ascontiguousarray(sample_batch, dtype=np.int32)
    ns, nd = draws.shape
    out = np.zeros(ns)
    L = lib()
    st = L.oracle_pt2_sample_batched(n, na, nb, _ptr(h1), _ptr(eri), _ptr(dets), _ptr(c), len(c),
                                     float(e0), float(eps2), float(eps2_d), ns, nd, _ptr(draws),
                                     int(n_batches), _ptr(sb), _ptr(out))
    if st:
        raise OracleError(st, L.oracle_last_error().decode())
    return out


def pt2_sample_frozen(n, na, nb, h1, eri, dets, c, c_ref, e0, eps2, eps2_d, draws):
    """Per-sample estimates with p_i and the screening taken from c_ref and
    the values from c (the function whose derivative the adjoint gives)."""
    h1, eri = _sys(h1, eri)
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    c_ref = np.ascontiguousarray(c_ref, dtype=np.float64)
    draws = np.ascontiguousarray(draws, dtype=np.uint32)
    ns, nd = draws.shape
    out = np.zeros(ns)
    L = lib()
    st = L.oracle_pt2_sample_frozen(n, na, nb, _ptr(h1), _ptr(eri), _ptr(dets), _ptr(c), _ptr(c_ref),
                                    len(c), float(e0), float(eps2), float(eps2_d), ns, nd,
                                    _ptr(draws), _ptr(out))
    if st:
        raise OracleError(st, L.oracle_last_error().decode())
    return out


def pt2_sample_grad(n, na, nb, h1, eri, dets, c, e0, eps2, eps2_d, draws):
    """(per-sample estimates, d(mean)/dc at frozen draws/p/masks, per-sample d/dE0)."""
    h1, eri = _sys(h1, eri)
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    draws = np.ascontiguousarray(draws, dtype=np.uint32)
    ns, nd = draws.shape
    out = np.zeros(ns)
    grad = np.zeros(len(c))
    de0 = np.zeros(ns)
    L = lib()
    st = L.oracle_pt2_sample_grad(n, na, nb, _ptr(h1), _ptr(eri), _ptr(dets), _ptr(c), len(c),
                                  float(e0), float(eps2), float(eps2_d), ns, nd, _ptr(draws),
                                  _ptr(out), _ptr(grad), _ptr(de0))
    if st:
        raise OracleError(st, L.oracle_last_error().decode())
    return out, grad, de0


def energy(n, na, nb, h1, eri, dets, c) -> float:
    """<c|H|c> by pairwise Slater-Condon elements."""
    h1, eri = _sys(h1, eri)
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    return lib().oracle_energy(n, na, nb, _ptr(h1), _ptr(eri), _ptr(dets), _ptr(c), len(c))


def hc_rows(n, na, nb, h1, eri, dets, c, rows=None):
    """Rows of H c on V by every pair: (y [m], connections [m]) for the given
    row indices (all rows when None); connections counts the j != i within
    two excitations."""
    h1, eri = _sys(h1, eri)
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    rows = np.arange(len(c), dtype=np.int64) if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    y = np.zeros(len(rows))
    cnt = np.zeros(len(rows), dtype=np.int64)
    L = lib()
    st = L.oracle_hc_rows(n, na, nb, _ptr(h1), _ptr(eri), _ptr(dets), _ptr(c), len(c), _ptr(rows), len(rows),
                          _ptr(y), _ptr(cnt))
    if st:
        raise OracleError(st, L.oracle_last_error().decode())
    return y, cnt


def terms_of(n, na, nb, h1, eri, dets, c, eps2, sources):
    """Kept terms (a outside V) of the given sources: (keys [m,4] uint64,
    H_ai [m], index into `sources` [m]), in enumeration order per source."""
    h1, eri = _sys(h1, eri)
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    src = np.ascontiguousarray(sources, dtype=np.int64)
    cap = 1 << 16
    while True:
        keys = np.zeros((cap, 4), dtype=np.uint64)
        hv = np.zeros(cap)
        which = np.zeros(cap, dtype=np.int64)
        m = lib().oracle_terms_of(n, na, nb, _ptr(h1), _ptr(eri), _ptr(dets), _ptr(c), len(c),
                                  float(eps2), _ptr(src), len(src), _ptr(keys), _ptr(hv),
                                  _ptr(which), cap)
        if m <= cap:
            return keys[:m], hv[:m], which[:m]
        cap = m


def energy_cores(n, na, nb, h1, eri, dets, c, hash_bits=64, part_bits=None):
    """<c|H|c> through shared (N-2)-electron cores (large V); returns
    (energy, number of connected off-diagonal pairs)."""
    h1, eri = _sys(h1, eri)
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    ne = na + nb
    if part_bits is None:
        entries = len(c) * ne * (ne - 1) // 2
        part_bits = max(0, int(np.ceil(np.log2(max(1.0, entries / 4e7)))))
    npairs = np.zeros(1, dtype=np.int64)
    e = lib().oracle_energy_cores(n, na, nb, _ptr(h1), _ptr(eri), _ptr(dets), _ptr(c), len(c),
                                  int(part_bits), int(hash_bits), _ptr(npairs))
    return e, int(npairs[0])


def mp1(n, na, nb, h1, eri, dets, mask, ref) -> np.ndarray:
    """H_i0 / (E_ref - H_ii) for the determinants flagged in mask, in order."""
    h1, eri = _sys(h1, eri)
    dets = np.ascontiguousarray(dets, dtype=np.uint64)
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    ref = np.ascontiguousarray(ref, dtype=np.uint64)
    out = np.zeros(int(m.sum()))
    lib().oracle_mp1(n, na, nb, _ptr(h1), _ptr(eri), _ptr(dets), _ptr(m), len(m), _ptr(ref),
                     _ptr(out))
    return out


def max_threads() -> int:
    return lib().oracle_max_threads()


def splitmix64(seed: int, m: int) -> int:
    """Output number m (m >= 1) of SplitMix64 seeded with `seed`."""
    return int(lib().oracle_splitmix64(seed & (2**64 - 1), m & (2**64 - 1)))


@dataclass
class AliasTable:
    threshold: np.ndarray   # [n] uint64: bucket k keeps k when v < threshold[k]
    alias: np.ndarray       # [n] uint32
    mass: list              # [n] exact integer masses N W_i (Python ints)
    own: list               # [n] exact own mass of each bucket
    capacity: int           # T = sum W_i


def alias_table(c) -> AliasTable:
    """Alias table of p_i = |c_i| / sum_j |c_j| (integer masses, Vose's sweep)."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    n = len(c)
    P = np.zeros(n, dtype=np.uint64)
    al = np.zeros(n, dtype=np.uint32)
    mlo = np.zeros(n, dtype=np.uint64)
    mhi = np.zeros(n, dtype=np.uint64)
    olo = np.zeros(n, dtype=np.uint64)
    ohi = np.zeros(n, dtype=np.uint64)
    t = np.zeros(2, dtype=np.uint64)
    L = lib()
    st = L.oracle_alias_table(_ptr(c), n, _ptr(P), _ptr(al), _ptr(mlo), _ptr(mhi), _ptr(olo), _ptr(ohi),
                              _ptr(t))
    if st:
        raise OracleError(st, L.oracle_alias_last_error().decode())
    mass = [int(h) << 64 | int(l) for l, h in zip(mlo, mhi)]
    own = [int(h) << 64 | int(l) for l, h in zip(olo, ohi)]
    return AliasTable(P, al, mass, own, int(t[1]) << 64 | int(t[0]))


def alias_draws(c, n_samples: int, n_draws: int, seed: int) -> np.ndarray:
    """Draws [n_samples, n_draws] (uint32) of the stochastic samples from the seed."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    out = np.zeros((n_samples, n_draws), dtype=np.uint32)
    L = lib()
    st = L.oracle_alias_draws(_ptr(c), len(c), seed & (2**64 - 1), n_samples, n_draws, _ptr(out))
    if st:
        raise OracleError(st, L.oracle_alias_last_error().decode())
    return out
