"""The 76-orbital, 10^7-determinant workload (w4) at full size, sampled.

The whole deterministic part is out of the oracle's reach at this size (some
1e13 candidate evaluations), so the checks are sampled or structural:

- deterministic part at eps2^d (screened PT2 equation): 256 perturbative
  determinants spread over the exported set, each against the oracle's own
  sum over V (A_a, E0 - H_aa and the kept-term count, so the full connection
  set of each sampled a); the exported count equals n_unique; the singleton
  split and the all-records grouping agree on every count and on E2 up to
  the summation order;
- stochastic part (stochastic PT2 equation): sample 0 of the seed path, its
  4000 draws bit-exact against the oracle's alias method; on its first 1000
  draws (the oracle's share of the test time), the kept-term count exact and
  the estimate within 1e-9 relative plus the first-order
  effect of the denominators' rounding (2e-11 Ha times the oracle's
  sum_a |contribution_a| / |E0 - H_aa|): w4's samples reach |E0 - H_aa|
  below 1e-9 Ha, where two FP64 evaluations of H_aa in different orders move
  a single contribution by far more than 1e-9 relative.
"""
import numpy as np
import pytest
import torch

from oracle import ref
from synth import store
from tests.gpu_util import context

pytestmark = pytest.mark.gpu

COUNTS = ("n_terms", "n_terms_gen", "n_unique", "n_intruder")
N_PICK = 256
U_CAP = 1 << 16
N_DRAWS_CHECKED = 1000


@pytest.fixture(scope="module")
def w4():
    x = store.load("w4")
    ctx, dets, c = context(x)
    yield x, ctx, dets, c
    ctx.close()


def test_w4_deterministic_part_sampled(w4):
    x, ctx, dets, c = w4
    wl = x.wl
    ctx.set_grouping("records")
    try:
        r = ctx.det(dets, c, x.e0, wl.eps2, "fp64", unique_cap=U_CAP)
    finally:
        ctx.set_grouping("auto")
    st = r.stats
    u = r.unique
    print(f"w4 det (records): E2 {r.e2!r} stats {st}", flush=True)
    assert u["n"] == st["n_unique"] and st["n_unique"] >= U_CAP
    m = u["keys"].shape[0]
    pick = np.linspace(0, m - 1, N_PICK).astype(np.int64)
    keys = u["keys"].cpu().numpy().view(np.uint64)[pick]
    A = u["A"].cpu().numpy()[pick]
    D = u["D"].cpu().numpy()[pick]
    cnt = u["cnt"].cpu().numpy().astype(np.int64)[pick]
    oA, oD, ocnt, oin = ref.pt2_at(wl.n_orb, wl.n_alpha, wl.n_beta, x.h1, x.eri, x.dets, x.c, x.e0, wl.eps2,
                                   keys)
    print(f"w4 sampled a: max |dA| {np.abs(A - oA).max():.3e}, max |dD| {np.abs(D - oD).max():.3e}, "
          f"kept terms {int(cnt.sum())} oracle {int(ocnt.sum())}", flush=True)
    assert not oin.any()
    assert np.array_equal(cnt, ocnt)
    assert np.abs(A - oA).max() <= 1e-13 * max(1.0, np.abs(oA).max())
    assert np.abs(D - oD).max() <= 1e-12 * np.abs(oD).max()
    # the singleton split: same terms, determinants and intruders; E2 in
    # another summation order
    ctx.set_grouping("split")
    try:
        s = ctx.det(dets, c, x.e0, wl.eps2, "fp64")
    finally:
        ctx.set_grouping("auto")
    print(f"w4 det (split): E2 {s.e2!r}, |dE2| {abs(s.e2 - r.e2):.3e}, singletons "
          f"{s.stats['n_singletons']} of {s.stats['n_terms_all']}", flush=True)
    for k in COUNTS:
        assert s.stats[k] == st[k], k
    assert abs(s.e2 - r.e2) <= 1e-9
    # "auto" splits a deterministic pass of 1e8 kept terms or more: the same
    # bits as the forced split
    a = ctx.det(dets, c, x.e0, wl.eps2, "fp64")
    assert s.stats["n_terms_all"] >= 100_000_000
    assert a.stats["n_singletons"] == s.stats["n_singletons"] > 0 and a.e2 == s.e2


def test_w4_sample_vs_oracle(w4):
    x, ctx, dets, c = w4
    wl = x.wl
    d = ctx.draws(c, 1, wl.n_draws, wl.draw_seed).cpu().numpy().astype(np.uint32)
    od = ref.alias_draws(x.c, 1, wl.n_draws, wl.draw_seed)
    assert np.array_equal(d, od)
    sub = od[:, :N_DRAWS_CHECKED]
    out, mean, sem, st = ctx.sample(dets, c, x.e0, wl.eps2_sto, wl.eps2,
                                    torch.from_numpy(sub.astype(np.int32)).cuda(), "fp64")
    got = float(out.cpu().numpy()[0])
    want, ocnt, sens = ref.pt2_sample_counts(wl.n_orb, wl.n_alpha, wl.n_beta, x.h1, x.eri, x.dets, x.c, x.e0,
                                             wl.eps2_sto, wl.eps2, sub, sens=True)
    tol = 1e-9 * max(1.0, abs(want[0])) + 2e-11 * sens[0]
    print(f"w4 sample 0: gpu {got!r} oracle {want[0]!r} |d| {abs(got - want[0]):.3e} tol {tol:.3e}; "
          f"terms {st['n_terms']} oracle {int(ocnt[0])}; min |D| {st['min_abs_denom']:.3e}", flush=True)
    assert st["n_terms"] == int(ocnt[0])
    assert abs(got - want[0]) <= tol
