"""Pins of the CPU reference against facts that do not depend on it.

* Slater-Condon elements and phases against explicit second-quantised operator
  application on full CI spaces (oracle.dense);
* the screened PT2 energy against dense linear algebra on the same spaces;
* limits stated in the paper: eps2 = 0 keeps exactly the non-zero elements
  (definition of P, section II), V = full CI gives E2 = 0, eps2^d = eps2 makes
  the stochastic part vanish (section II.B);
* the stochastic estimator's exact multinomial expectation equals the
  deterministic sum (stochastic PT2 equation);
* gradients: Euler's identity for a degree-2 homogeneous function, dense
  linear algebra, and binary128 finite differences;
* closed-form excitation counts and the paper's Cr2 Hilbert-space size.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import dense, ref
from synth import generator as G
from tests import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _space(n, na, nb, seed):
    x = G.make_small(n, na, nb, 2, 1, seed)
    dets, index, H = dense.hamiltonian(n, na, nb, x.h1, x.eri)
    W = np.array([dense.to_words(d, n) for d in dets], dtype=np.uint64)
    return x, dets, index, H, W


@pytest.fixture(scope="module")
def space_227():
    return _space(7, 3, 2, 11)


@pytest.fixture(scope="module")
def space_226():
    return _space(6, 2, 2, 12)


@pytest.mark.parametrize("fix", ["space_226", "space_227"])
def test_slater_condon_matches_second_quantisation(fix, request):
    x, dets, index, H, W = request.getfixturevalue(fix)
    n, na, nb = x.wl.n_orb, x.wl.n_alpha, x.wl.n_beta
    Ho = np.array([[ref.hij(n, na, nb, x.h1, x.eri, W[a], W[i]) for i in range(len(W))]
                   for a in range(len(W))])
    assert np.abs(Ho - H).max() < 1e-12
    # Hermitian bit for bit (8-fold symmetric integrals, mirrored evaluation order)
    assert np.array_equal(Ho, Ho.T)
    # more than double excitations vanish exactly
    for a, i in itertools.product(range(0, len(W), 7), range(0, len(W), 5)):
        diff = sum(bin(int(W[a][k]) ^ int(W[i][k])).count("1") for k in range(4))
        if diff > 4:
            assert Ho[a, i] == 0.0 and abs(H[a, i]) < 1e-15


def test_diagonal_matches_second_quantisation(space_227):
    x, dets, index, H, W = space_227
    d = np.array([ref.diag(7, 3, 2, x.h1, x.eri, w) for w in W])
    assert np.abs(d - np.diag(H)).max() < 1e-12


def _random_v(rng, nfci, nv):
    return np.sort(rng.choice(nfci, size=nv, replace=False))


@pytest.mark.parametrize("eps2", [0.0, 1e-4, 3e-3])
def test_e2_matches_dense_linear_algebra(space_227, eps2):
    x, dets, index, H, W = space_227
    rng = np.random.default_rng(5)
    v = _random_v(rng, len(dets), 40)
    c = rng.standard_normal(40)
    c /= np.linalg.norm(c)
    e0 = float(np.min(np.diag(H))) - 0.5
    r = ref.pt2_det(7, 3, 2, x.h1, x.eri, W[v], c, e0, eps2)
    want = dense.e2_dense(H, v, c, e0, eps2)
    assert abs(r.e2 - want) <= 1e-12 * max(1.0, abs(want))
    # connection set: outside V with at least one kept term, |H_ai c_i| > eps2
    outside = np.setdiff1d(np.arange(len(dets)), v)
    mask = np.abs(H[np.ix_(outside, v)] * c[None, :]) > eps2
    dense_set = {dets[k] for k in outside[mask.any(axis=1)]}
    oracle_set = {dense.from_words(k, 7) for k in r.keys}
    if eps2 == 0.0:
        # exactly the determinants with a non-zero element (section II, P)
        assert oracle_set == dense_set
    else:
        # away from ties the sets agree; ties |H c| == eps2 have measure zero
        assert len(oracle_set ^ dense_set) == 0
    assert r.n_terms == int(mask.sum()) or eps2 > 0


def test_full_space_gives_zero(space_226):
    x, dets, index, H, W = space_226
    c = np.linalg.eigh(H)[1][:, 0]
    r = ref.pt2_det(6, 2, 2, x.h1, x.eri, W, c, -10.0, 0.0)
    assert r.e2 == 0.0 and r.n_unique == 0 and r.n_terms == 0
    assert r.n_terms_gen > 0  # every connection lands inside V


def test_single_reference(space_227):
    x, dets, index, H, W = space_227
    hf = G.hf_det(3, 2)
    k = index[dense.from_words(hf, 7)]
    ehf = H[k, k]
    r = ref.pt2_det(7, 3, 2, x.h1, x.eri, hf[None, :], np.array([1.0]), ehf, 0.0)
    others = [a for a in range(len(dets)) if a != k and H[a, k] != 0.0]
    want = sum(H[a, k] ** 2 / (ehf - H[a, a]) for a in others)
    assert abs(r.e2 - want) <= 1e-12 * abs(want)
    assert r.n_unique == len(others) == dense.n_excitations_closed_form(7, 3, 2)


def test_screening_limits_and_invariances():
    x = I.small(10, 3, 3, 150, 3, 3)
    n = 10
    base = ref.pt2_det(n, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0, 1e-4)
    huge = ref.pt2_det(n, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0, 1e3)
    assert huge.e2 == 0.0 and huge.n_unique == 0
    # sets shrink monotonically with eps2
    prev = None
    for eps in [0.0, 1e-6, 1e-4, 1e-3, 1e-2]:
        r = ref.pt2_det(n, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0, eps)
        s = {tuple(k) for k in r.keys}
        if prev is not None:
            assert s <= prev
        prev = s
    # c -> -c leaves every A_a^2 bit for bit
    neg = ref.pt2_det(n, 3, 3, x.h1, x.eri, x.dets, -x.c, x.e0, 1e-4)
    assert neg.e2 == base.e2 and np.array_equal(neg.A, -base.A)
    # permuting V changes only the summation order
    perm = np.random.default_rng(1).permutation(len(x.c))
    pr = ref.pt2_det(n, 3, 3, x.h1, x.eri, x.dets[perm], x.c[perm], x.e0, 1e-4)
    assert abs(pr.e2 - base.e2) <= 1e-14 * abs(base.e2)
    assert pr.n_terms == base.n_terms and np.array_equal(pr.keys, base.keys)


def test_from_a_side_matches_forward():
    x = I.small(10, 3, 3, 150, 3, 4)
    r = ref.pt2_det(10, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0, 1e-5)
    sel = np.random.default_rng(0).choice(r.n_unique, size=60, replace=False)
    A, D, cnt, inv = ref.pt2_at(10, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0, 1e-5, r.keys[sel])
    assert np.array_equal(A, r.A[sel]) and np.array_equal(D, r.D[sel])
    assert np.array_equal(cnt, r.counts[sel]) and not inv.any()
    _, _, _, inv2 = ref.pt2_at(10, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0, 1e-5, x.dets[:5])
    assert inv2.all()


@pytest.mark.parametrize("shape", [(6, 2, 2), (7, 3, 2), (12, 4, 4), (40, 8, 8), (66, 3, 2)])
def test_excitation_counts_closed_form(shape):
    n, na, nb = shape
    rng = np.random.default_rng(n)
    h1 = np.zeros((n, n))
    eri = np.zeros((n, n, n, n))
    # scattered occupations exercise both words of a spin string when n > 64
    occa = np.sort(rng.choice(n, size=na, replace=False))
    occb = np.sort(rng.choice(n, size=nb, replace=False))
    if n > 64:
        occa[-1] = n - 1
    a = G.occ_to_words(occa[None, :])[0]
    b = G.occ_to_words(occb[None, :])[0]
    d = np.array([a[0], a[1], b[0], b[1]], dtype=np.uint64)
    cnt = ref.count_excitations(n, na, nb, h1, eri, d)
    assert cnt == dense.n_excitations_closed_form(n, na, nb)  # positive: all distinct


def test_paper_hilbert_space_dimension():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        g = json.load(f)["cr2_hilbert_space"]
    s = g["shape"]
    dim = math.comb(s["n_orb"], s["n_alpha"]) * math.comb(s["n_orb"], s["n_beta"])
    assert float(f"{dim:.{g['significant_figures'] - 1}e}") == g["value"]
    assert abs(dim - 4.7233e29) / dim < 1e-4


def _multisets(nv, nd):
    for combo in itertools.combinations_with_replacement(range(nv), nd):
        yield combo


def test_stochastic_estimator_is_unbiased():
    x = I.small(8, 2, 2, 6, 2, 21)
    n = 8
    c = x.c
    p = np.abs(c) / np.abs(c).sum()
    eps2 = 2e-3
    det = ref.pt2_det(n, 2, 2, x.h1, x.eri, x.dets, c, x.e0, eps2)
    for nd in (2, 3, 4):
        expect = 0.0
        for combo in _multisets(len(c), nd):
            w = np.bincount(combo, minlength=len(c))
            prob = math.factorial(nd) * np.prod([p[i] ** w[i] / math.factorial(w[i])
                                                  for i in range(len(c))])
            draws = np.array(combo, dtype=np.uint32)[None, :]
            s = ref.pt2_sample(n, 2, 2, x.h1, x.eri, x.dets, c, x.e0, eps2, 1e30, draws)[0]
            expect += prob * s
        assert abs(expect - det.e2) <= 1e-12 * abs(det.e2), (nd, expect, det.e2)


def test_stochastic_deterministic_limit():
    x = I.small(10, 3, 3, 80, 3, 22)
    rng = np.random.default_rng(3)
    draws = rng.integers(0, 80, size=(4, 30)).astype(np.uint32)
    out = ref.pt2_sample(10, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0, 1e-4, 1e-4, draws)
    assert np.all(out == 0.0)


def test_gradient_pins(space_227):
    x, dets, index, H, W = space_227
    rng = np.random.default_rng(9)
    v = _random_v(rng, len(dets), 50)
    c = rng.standard_normal(50)
    c /= np.linalg.norm(c)
    e0 = float(np.min(np.diag(H))) - 0.3
    eps2 = 1e-3
    coords = np.arange(50)
    r = ref.pt2_det(7, 3, 2, x.h1, x.eri, W[v], c, e0, eps2, grad=True, fd_coords=coords,
                    fd_de0_step=1e-5)
    # Euler: E2 is homogeneous of degree 2 in c at a fixed mask
    assert abs(np.dot(c, r.grad) - 2 * r.e2) <= 1e-12 * abs(r.e2)
    # dense: g = 2 (H_PV * mask)^T (A / D)
    outside = np.setdiff1d(np.arange(len(dets)), v)
    hpv = H[np.ix_(outside, v)]
    mask = np.abs(hpv * c[None, :]) > eps2
    A = (hpv * mask) @ c
    D = e0 - np.diag(H)[outside]
    keep = mask.any(axis=1)
    g = 2 * ((hpv * mask)[keep]).T @ (A[keep] / D[keep])
    assert np.abs(g - r.grad).max() <= 1e-11 * np.abs(g).max()
    # binary128 central differences with the mask frozen
    assert np.abs(r.fd - r.grad).max() <= 1e-12 * np.abs(r.grad).max()
    de0 = -np.sum(A[keep] ** 2 / D[keep] ** 2)
    assert abs(r.de2_de0 - de0) <= 1e-12 * abs(de0)
    assert abs(r.fd_de0 - r.de2_de0) <= 1e-9 * abs(de0)


def test_energy_helper_matches_dense(space_227):
    x, dets, index, H, W = space_227
    rng = np.random.default_rng(4)
    v = _random_v(rng, len(dets), 60)
    c = rng.standard_normal(60)
    c /= np.linalg.norm(c)
    e = ref.energy(7, 3, 2, x.h1, x.eri, W[v], c)
    assert abs(e - c @ H[np.ix_(v, v)] @ c) < 1e-12
    # MP1-like amplitudes: <a|H|ref> / (E_ref - H_aa)
    hf = G.hf_det(3, 2)
    k = index[dense.from_words(hf, 7)]
    mask = np.array([1 if (i != k and H[i, k] != 0.0) else 0 for i in range(len(dets))], np.uint8)
    amp = ref.mp1(7, 3, 2, x.h1, x.eri, W, mask, hf)
    sel = np.nonzero(mask)[0]
    want = H[sel, k] / (H[k, k] - np.diag(H)[sel])
    assert np.abs(amp - want).max() < 1e-12 * np.abs(want).max()


def test_validation_errors():
    x = I.small(8, 2, 2, 20, 2, 1)
    bad = x.dets.copy()
    bad[3] = bad[2]
    with pytest.raises(ref.OracleError) as e:
        ref.pt2_det(8, 2, 2, x.h1, x.eri, bad, x.c, x.e0, 0.0)
    assert e.value.code == -4
    bad = x.dets.copy()
    bad[1, 0] |= np.uint64(1 << 7)
    with pytest.raises(ref.OracleError) as e:
        ref.pt2_det(8, 2, 2, x.h1, x.eri, bad, x.c, x.e0, 0.0)
    assert e.value.code == -3
    c = x.c.copy()
    c[4] = np.nan
    with pytest.raises(ref.OracleError) as e:
        ref.pt2_det(8, 2, 2, x.h1, x.eri, x.dets, c, x.e0, 0.0)
    assert e.value.code == -5


@pytest.mark.parametrize("shape", [(10, 3, 3, 400, 3, 1), (14, 4, 3, 600, 4, 2), (70, 2, 2, 150, 2, 3)])
def test_energy_through_cores_matches_pairwise(shape):
    # <c|H|c> through shared (N-2)-electron cores: the same value as the
    # pairwise sum, also when a short hash makes unrelated cores collide, and
    # exactly the connected pairs of V (brute force)
    n, na, nb, nv, lev, seed = shape
    x = I.small(n, na, nb, nv, lev, seed)
    e_pair = ref.energy(n, na, nb, x.h1, x.eri, x.dets, x.c)
    e64, npairs = ref.energy_cores(n, na, nb, x.h1, x.eri, x.dets, x.c)
    e6, npairs6 = ref.energy_cores(n, na, nb, x.h1, x.eri, x.dets, x.c, hash_bits=6, part_bits=2)
    assert abs(e64 - e_pair) <= 1e-13 * abs(e_pair)
    assert abs(e6 - e_pair) <= 1e-13 * abs(e_pair)
    d = x.dets
    diff = np.zeros((len(d), len(d)), dtype=np.int64)
    for w in range(4):
        xo = np.bitwise_xor(d[:, None, w], d[None, :, w])
        diff += np.array([bin(int(v)).count("1") for v in xo.ravel()]).reshape(xo.shape)
    brute = int(((diff > 0) & (diff <= 4)).sum() // 2)
    assert npairs == npairs6 == brute


def test_terms_of_sources_match_full_enumeration():
    # the per-source term listing used by the large-workload parity tests
    # finds exactly the kept terms with a outside V
    x = I.small(10, 3, 3, 150, 3, 5)
    o = ref.pt2_det(10, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0, 1e-5, terms=True)
    keys, hv, which = ref.terms_of(10, 3, 3, x.h1, x.eri, x.dets, x.c, 1e-5, np.arange(len(x.c)))
    assert len(keys) == o.n_terms
    out_v = [tuple(r) for r in o.keys]
    assert set(map(tuple, keys)) == set(out_v)
    cnt = {}
    for r in map(tuple, keys):
        cnt[r] = cnt.get(r, 0) + 1
    assert all(cnt[tuple(k)] == n for k, n in zip(o.keys, o.counts))


def test_stochastic_gradient_pins():
    # derivative of the mean stochastic estimate at frozen draws, p and masks:
    # Euler identity (degree-2 homogeneous in c), central differences of the
    # frozen-mask estimator (exact for a quadratic up to rounding), and the
    # E0 derivative against Richardson-extrapolated differences
    x = I.small(8, 3, 2, 120, 3, 21)
    rng = np.random.default_rng(8)
    p = np.abs(x.c) / np.abs(x.c).sum()
    draws = rng.choice(len(x.c), size=(5, 30), p=p).astype(np.uint32)
    eps2, eps2_d = 1e-5, 1e-3
    args = (8, 3, 2, x.h1, x.eri, x.dets)
    out, grad, de0 = ref.pt2_sample_grad(*args, x.c, x.e0, eps2, eps2_d, draws)
    assert np.allclose(out, ref.pt2_sample(*args, x.c, x.e0, eps2, eps2_d, draws), rtol=0, atol=1e-15)
    mean = out.mean()
    assert abs(np.dot(x.c, grad) - 2.0 * mean) <= 1e-12 * abs(mean)
    for i in rng.choice(len(x.c), size=8, replace=False):
        h = 1e-4 * abs(x.c[i])
        cp, cm = x.c.copy(), x.c.copy()
        cp[i] += h
        cm[i] -= h
        hp, hm = cp[i] - x.c[i], x.c[i] - cm[i]
        fp = ref.pt2_sample_frozen(*args, cp, x.c, x.e0, eps2, eps2_d, draws).mean()
        fm = ref.pt2_sample_frozen(*args, cm, x.c, x.e0, eps2, eps2_d, draws).mean()
        fd = (fp - fm) / (hp + hm)
        assert abs(fd - grad[i]) <= 1e-7 * max(np.abs(grad).max(), 1e-300)
    # dS/dE0: Richardson on central differences
    def s_at(e0):
        return ref.pt2_sample(*args, x.c, e0, eps2, eps2_d, draws)
    d1 = 1e-4
    c1 = (s_at(x.e0 + d1) - s_at(x.e0 - d1)) / (2 * d1)
    c2 = (s_at(x.e0 + d1 / 2) - s_at(x.e0 - d1 / 2)) / d1
    rich = (4 * c2 - c1) / 3
    assert np.abs(rich - de0).max() <= 1e-6 * np.abs(de0).max()


def test_hash_batches_partition_p():
    # the hash batches partition P: batch sums add up to E2 (and, with an
    # upper threshold, to E2(eps2) - E2(eps2_hi)); counts add up; batches are
    # evenly filled
    x = I.small(10, 3, 3, 200, 3, 23)
    args = (10, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0)
    nbat = 8
    o = ref.pt2_det(*args, 1e-6, unique=False)
    oh = ref.pt2_det(*args, 1e-4, unique=False)
    rows = [ref.det_batch(*args, 1e-6, np.inf, nbat, b) for b in range(nbat)]
    assert abs(sum(r[0] for r in rows) - o.e2) <= 1e-12 * abs(o.e2)
    assert sum(r[2] for r in rows) == o.n_unique and sum(r[3] for r in rows) == o.n_terms
    cnt = np.array([r[2] for r in rows], dtype=float)
    assert np.all(np.abs(cnt - cnt.mean()) <= 5 * np.sqrt(cnt.mean()) + 1)
    rows2 = [ref.det_batch(*args, 1e-6, 1e-4, nbat, b) for b in range(nbat)]
    assert abs(sum(r[0] for r in rows2) - (o.e2 - oh.e2)) <= 1e-12 * abs(o.e2)
    # one batch of P per sample: averaged over the batch choice, the estimate
    # is the unbatched one
    rng = np.random.default_rng(29)
    p = np.abs(x.c) / np.abs(x.c).sum()
    draws = rng.choice(len(x.c), size=(3, 25), p=p).astype(np.uint32)
    full = ref.pt2_sample(*args, 1e-6, 1e-4, draws)
    per_b = np.array([ref.pt2_sample_batched(*args, 1e-6, 1e-4, draws, nbat, np.full(3, b, np.int32))
                      for b in range(nbat)])
    assert np.abs(per_b.mean(axis=0) - full).max() <= 1e-12 * max(1.0, np.abs(full).max())


def test_hc_rows_match_dense_linear_algebra(space_227, space_226):
    """H c on V against the second-quantised Hamiltonian restricted to V, and
    the connection counts against the excitation degree counted on the bit
    strings."""
    for (x, dets, index, H, W), (n, na, nb) in ((space_227, (7, 3, 2)), (space_226, (6, 2, 2))):
        rng = np.random.default_rng(17)
        v = _random_v(rng, len(dets), min(len(dets), 90))
        c = rng.standard_normal(len(v))
        y, cnt = ref.hc_rows(n, na, nb, x.h1, x.eri, W[v], c)
        want = H[np.ix_(v, v)] @ c
        assert np.abs(y - want).max() <= 1e-12 * max(1.0, np.abs(want).max())
        # degree: half the number of differing spin orbitals
        deg = np.array([[bin(dets[i] ^ dets[j]).count("1") // 2 for j in v] for i in v])
        assert np.array_equal(cnt, ((deg >= 1) & (deg <= 2)).sum(axis=1))
        # a subset of rows gives the same values
        rows = np.array([3, 0, len(v) - 1])
        y2, cnt2 = ref.hc_rows(n, na, nb, x.h1, x.eri, W[v], c, rows)
        assert np.array_equal(y2, y[rows]) and np.array_equal(cnt2, cnt[rows])
        # c^T H c of the rows is the variational energy
        assert abs(c @ y - c @ want) <= 1e-12 * max(1.0, abs(c @ want))


def test_hc_rows_rejects_bad_rows(space_227):
    x, dets, index, H, W = space_227
    with pytest.raises(ref.OracleError):
        ref.hc_rows(7, 3, 2, x.h1, x.eri, W[:5], np.ones(5), np.array([5]))


def test_sample_sensitivity_bounds_the_e0_derivative():
    # sum_a |contribution_a| / |D_a| bounds |dS_s/dE0| = |sum_a contribution_a / D_a|
    # and equals it when every group has the same sign of contribution / D
    x = I.small(8, 2, 2, 40, 2, 3)
    a = (8, 2, 2, x.h1, x.eri)
    rng = np.random.default_rng(3)
    p = np.abs(x.c) / np.abs(x.c).sum()
    dr = rng.choice(len(x.c), size=(4, 9), p=p).astype(np.uint32)
    out, cnt, sens = ref.pt2_sample_counts(*a, x.dets, x.c, x.e0, 1e-7, 1e-5, dr, sens=True)
    o2, _, de0 = ref.pt2_sample_grad(*a, x.dets, x.c, x.e0, 1e-7, 1e-5, dr)
    assert np.array_equal(out, o2)
    assert np.all(sens >= np.abs(de0) * (1 - 1e-12))
    # a single-reference system far below its perturbers: every D_a < 0 and
    # every bracket > 0, so sens = |dS/dE0|
    one = np.zeros((1, 8), dtype=np.uint32)
    o1, _, s1 = ref.pt2_sample_counts(*a, x.dets[:1], np.array([1.0]), x.e0 - 50.0, 0.0, 1e9, one, sens=True)
    _, _, d1 = ref.pt2_sample_grad(*a, x.dets[:1], np.array([1.0]), x.e0 - 50.0, 0.0, 1e9, one)
    assert abs(s1[0] - abs(d1[0])) <= 1e-12 * abs(d1[0])
