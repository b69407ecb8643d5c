"""The 76-orbital, 10^6-determinant semistochastic workload (w3) at full
size, in the launch configuration of the benchmark.  The CPU reference cannot
evaluate the whole sums in seconds here, so parity is checked on sampled
outputs it can compute one by one (A_a, D_a and term counts of sampled a;
every kept term of sampled sources; whole per-sample estimates of sampled
samples) and through properties that hold at any size."""
import math

import numpy as np
import pytest
import torch

from oracle import ref
from synth import store
from tests.gpu_util import context, keys_np, sort_keys

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def w3():
    x = store.load("w3")
    ctx, dets, c = context(x)
    return x, ctx, dets, c


def _draws(x):
    wl = x.wl
    p = np.abs(x.c) / np.abs(x.c).sum()
    return np.random.default_rng(wl.draw_seed).choice(len(x.c), size=(wl.n_samples, wl.n_draws),
                                                      p=p).astype(np.uint32)


def test_w3_deterministic_part(w3):
    x, ctx, dets, c = w3
    wl = x.wl
    n, na, nb = wl.n_orb, wl.n_alpha, wl.n_beta
    r = ctx.det(dets, c, x.e0, wl.eps2, "fp64", unique_cap=60_000_000)
    st = r.stats
    print(f"w3 det: E2={r.e2!r} stats={st}", flush=True)
    u = r.unique
    nu = u["n"]
    assert nu == st["n_unique"]
    keys = keys_np(u["keys"])
    A = u["A"].cpu().numpy()
    D = u["D"].cpu().numpy()
    cnt = u["cnt"].cpu().numpy()
    # properties: counts add up, E2 is the sum of the exported contributions
    assert int(cnt.astype(np.int64).sum()) == st["n_terms"]
    assert (cnt > 0).all()
    e2_host = math.fsum((A * A / D).tolist())
    assert abs(e2_host - r.e2) <= 1e-9
    assert int((D > 0).sum()) == st["n_intruder"]
    assert np.abs(D).min() == st["min_abs_denom"]
    # sampled a: A_a, D_a and counts one by one
    rng = np.random.default_rng(31)
    pick = rng.choice(nu, size=400, replace=False)
    oA, oD, oc, inv = ref.pt2_at(n, na, nb, x.h1, x.eri, x.dets, x.c, x.e0, wl.eps2, keys[pick])
    assert not inv.any()
    assert np.array_equal(cnt[pick], oc)
    assert np.abs(A[pick] - oA).max() <= 1e-13 * max(1.0, np.abs(oA).max())
    assert np.abs(D[pick] - oD).max() <= 1e-12 * np.abs(oD).max()
    # sampled sources (HF, a large MP1 double, random others): every kept term
    # with a outside V reaches a unique a of the export
    big = int(np.argsort(-np.abs(x.c[1:]))[0]) + 1
    srcs = np.concatenate([[0, big], rng.choice(len(x.c), size=60, replace=False)])
    tk, th, tw = ref.terms_of(n, na, nb, x.h1, x.eri, x.dets, x.c, wl.eps2, srcs)
    print(f"sampled sources: {len(srcs)}, kept terms {len(tk)}", flush=True)
    order = sort_keys(keys)
    sk = keys[order]
    ok = sort_keys(tk)
    tks = tk[ok]
    # merge: every term key must be present among the unique keys
    j = 0
    missing = 0
    for row in tks:
        while j < len(sk) and tuple(sk[j][::-1]) < tuple(row[::-1]):
            j += 1
        if j >= len(sk) or not np.array_equal(sk[j], row):
            missing += 1
    assert missing == 0
    # FP32-compensated form against FP64 at full size
    r32 = ctx.det(dets, c, x.e0, wl.eps2, "fp32c")
    print(f"w3 det fp32c: |dE2| vs fp64 = {abs(r32.e2 - r.e2):.3e}", flush=True)
    assert abs(r32.e2 - r.e2) <= 1e-6
    assert r32.stats["n_terms"] == st["n_terms"] and r32.stats["n_unique"] == st["n_unique"]


def test_w3_samples(w3):
    x, ctx, dets, c = w3
    wl = x.wl
    n, na, nb = wl.n_orb, wl.n_alpha, wl.n_beta
    draws = _draws(x)
    dr = torch.from_numpy(draws.view(np.int32)).cuda()
    out, mean, sem, st = ctx.sample(dets, c, x.e0, wl.eps2_sto, wl.eps2, dr, "fp64")
    out = out.cpu().numpy()
    print(f"w3 samples: mean {mean!r} +- {sem!r}, stats {st}", flush=True)
    assert np.isfinite(out).all()
    assert 0.0 < st["min_abs_denom"] < 1e-3  # intruder-rich: stated with the results
    assert abs(mean - out.mean()) <= 1e-15 * max(1.0, abs(mean))
    # two whole samples against the CPU reference
    for s in (0, 137):
        o = ref.pt2_sample(n, na, nb, x.h1, x.eri, x.dets, x.c, x.e0, wl.eps2_sto, wl.eps2,
                           draws[s:s + 1])
        print(f"sample {s}: gpu {out[s]!r} reference {o[0]!r}", flush=True)
        assert abs(out[s] - o[0]) <= 1e-9 * max(1.0, abs(o[0]))
    out32, mean32, _, _ = ctx.sample(dets, c, x.e0, wl.eps2_sto, wl.eps2, dr, "fp32c")
    out32 = out32.cpu().numpy()
    print(f"w3 samples fp32c: max |d| per sample {np.abs(out32 - out).max():.3e}, "
          f"|d mean| {abs(mean32 - mean):.3e}", flush=True)
    assert np.abs(out32 - out).max() <= 1e-6


def test_w3_sample_adjoint_properties(w3):
    # the stochastic adjoint at full size on 8 samples: Euler identity
    # (degree-2 homogeneous at frozen draws, p and masks) and FP32c vs FP64
    x, ctx, dets, c = w3
    wl = x.wl
    draws = _draws(x)[:8]
    dr = torch.from_numpy(np.ascontiguousarray(draws).view(np.int32)).cuda()
    out, mean, sem, g, de0, st = ctx.sample_grad(dets, c, x.e0, wl.eps2_sto, wl.eps2, dr, "fp64")
    g = g.cpu().numpy()
    euler = float(np.dot(x.c, g))
    print(f"w3 sample adjoint: mean {mean!r}, c.g/2 {euler / 2!r}, dE0 {de0!r}, stats {st}", flush=True)
    assert abs(euler - 2.0 * mean) <= 1e-8 * max(abs(mean), 1e-12)
    o8 = ctx.sample(dets, c, x.e0, wl.eps2_sto, wl.eps2, dr, "fp64")[0].cpu().numpy()
    assert np.abs(out.cpu().numpy() - o8).max() <= 1e-12 * max(1.0, np.abs(o8).max())
    _, _, _, g32, _, _ = ctx.sample_grad(dets, c, x.e0, wl.eps2_sto, wl.eps2, dr, "fp32c")
    rel = np.linalg.norm(g32.cpu().numpy() - g) / np.linalg.norm(g)
    print(f"w3 sample adjoint fp32c rel diff {rel:.3e}", flush=True)
    assert rel <= 1e-6
