"""The C-ABI boundary beyond the plain calls: the seed path of the stochastic
samples (alias table and draws made on the device), caller-owned
workspaces and the adjoint modes.  Every case runs the HIP path through the
C ABI and compares with the CPU oracle or with the same call in another
configuration.

Bars: alias tables and draws bit-exact (integer work); E2 within 1e-9 Ha and
counts bit-exact against the oracle; gradients within 1e-10 relative of the
oracle's.
"""
import numpy as np
import pytest
import torch

import paper_1809_04600_amd as P
from oracle import ref
from synth import store
from tests import inputs as I
from tests.gpu_util import context

pytestmark = pytest.mark.gpu

E2_TOL_FP64 = 1e-9


def _u64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def _coefficient_cases():
    rng = np.random.default_rng(5)
    cases = {
        "one": np.array([-0.7]),
        "two": np.array([0.25, -0.75]),
        "equal": np.full(300, -0.125),
        "zeros": np.where(rng.random(500) < 0.3, 0.0, rng.normal(size=500)),
        "spread": rng.normal(size=2000) * np.exp(rng.uniform(-40, 0, size=2000)),
        "subnormal": np.array([5e-324, 1e-310, 3e-320, 0.0, 2.2e-308]),
    }
    big = rng.normal(size=70001) * 1e-3
    big[0] = 0.9
    cases["big"] = big
    return cases


@pytest.fixture(scope="module")
def tiny_ctx():
    x = I.small(8, 2, 2, 30, 2, 3)
    ctx, dets, c = context(x)
    return ctx


@pytest.mark.parametrize("name", list(_coefficient_cases()))
def test_alias_table_and_draws_bit_exact(tiny_ctx, name):
    c = _coefficient_cases()[name]
    ct = torch.from_numpy(c).cuda()
    thr, al = tiny_ctx.alias_table(ct)
    t = ref.alias_table(c)
    assert np.array_equal(_u64(thr), t.threshold)
    assert np.array_equal(al.cpu().numpy().astype(np.uint32), t.alias)
    for ns, nd, seed in ((3, 5, 0), (17, 257, 2**64 - 1), (64, 1000, 12345)):
        d = tiny_ctx.draws(ct, ns, nd, seed).cpu().numpy().astype(np.uint32)
        assert np.array_equal(d, ref.alias_draws(c, ns, nd, seed))


def test_alias_errors(tiny_ctx):
    with pytest.raises(P.ShciError) as e:
        tiny_ctx.draws(torch.zeros(10, dtype=torch.float64, device="cuda"), 2, 3, 1)
    assert e.value.code == -5
    bad = torch.ones(10, dtype=torch.float64, device="cuda")
    bad[4] = float("inf")
    with pytest.raises(P.ShciError) as e:
        tiny_ctx.alias_table(bad)
    assert e.value.code == -5


def test_w3_draws_bit_exact():
    # the seed path on the 10^6-determinant coefficients, at the sample
    # shape of the benchmark (256 samples of 2000 draws)
    x = store.load("w3")
    wl = x.wl
    ctx, dets, c = context(x)
    thr, al = ctx.alias_table(c)
    t = ref.alias_table(x.c)
    assert np.array_equal(_u64(thr), t.threshold)
    assert np.array_equal(al.cpu().numpy().astype(np.uint32), t.alias)
    d = ctx.draws(c, wl.n_samples, wl.n_draws, wl.draw_seed).cpu().numpy().astype(np.uint32)
    assert np.array_equal(d, ref.alias_draws(x.c, wl.n_samples, wl.n_draws, wl.draw_seed))


def test_sample_seed_path():
    # draws made on the device give the same per-sample estimates as the same
    # draws passed in, and match the oracle on them
    x = I.small(10, 3, 3, 200, 3, 9)
    ctx, dets, c = context(x)
    eps2, eps2_d, seed = 1e-6, 1e-4, 77
    draws = ref.alias_draws(x.c, 9, 60, seed)
    o = ref.pt2_sample(10, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0, eps2, eps2_d, draws)
    dr = torch.from_numpy(draws.view(np.int32)).cuda()
    out_e, m_e, s_e, _ = ctx.sample(dets, c, x.e0, eps2, eps2_d, dr, "fp64")
    out_s, m_s, s_s, st = ctx.sample(dets, c, x.e0, eps2, eps2_d, None, "fp64", seed=seed, n_samples=9,
                                     n_draws=60)
    assert torch.equal(out_s, out_e) and m_s == m_e and s_s == s_e
    assert np.abs(out_s.cpu().numpy() - o).max() <= 1e-9 * max(1.0, np.abs(o).max())
    # the adjoint on the seed path equals the adjoint on the same draws
    _, _, _, g_e, de_e, _ = ctx.sample_grad(dets, c, x.e0, eps2, eps2_d, dr, "fp64")
    _, _, _, g_s, de_s, _ = ctx.sample_grad(dets, c, x.e0, eps2, eps2_d, None, "fp64", seed=seed, n_samples=9,
                                            n_draws=60)
    assert torch.equal(g_s, g_e) and de_s == de_e


def test_workspace_caller_owned():
    # every term a record (the sizes below are those of the records)
    x = I.small(12, 3, 3, 300, 3, 11)
    ctx, dets, c = context(x)
    ctx.set_grouping("records")
    eps2 = 1e-6
    o = ref.pt2_det(12, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0, eps2, unique=False)
    r0 = ctx.det(dets, c, x.e0, eps2, "fp64")
    nrec = r0.stats["n_records"]
    full = ctx.workspace_size("det", len(x.c), nrec)
    ws = torch.empty(full, dtype=torch.uint8, device="cuda")
    r1 = ctx.det(dets, c, x.e0, eps2, "fp64", ws=ws)
    print("workspace bytes for one pass:", full, "records", nrec, "stats", r1.stats)
    assert r1.stats["n_chunks"] == 1
    assert r1.e2 == r0.e2
    for k in ("n_terms", "n_terms_gen", "n_unique", "n_intruder"):
        assert r1.stats[k] == r0.stats[k] == getattr(o, k)
    # a third of the bytes: hash batches, same sums
    small = ws[: full // 3]
    r2 = ctx.det(dets, c, x.e0, eps2, "fp64", ws=small)
    print("third of the workspace:", r2.stats["n_chunks"], "batches")
    assert r2.stats["n_chunks"] > 1
    for k in ("n_terms", "n_terms_gen", "n_unique", "n_intruder"):
        assert r2.stats[k] == r0.stats[k]
    assert abs(r2.e2 - r0.e2) <= 1e-13 * abs(r0.e2)
    assert abs(r2.e2 - o.e2) <= E2_TOL_FP64
    # far too small, or misaligned: errors, not faults
    with pytest.raises(P.ShciError) as e:
        ctx.det(dets, c, x.e0, eps2, "fp64", ws=ws[:4096])
    assert e.value.code == -6
    with pytest.raises(P.ShciError) as e:
        ctx.det(dets, c, x.e0, eps2, "fp64", ws=ws[8:])
    assert e.value.code == -1
    # the same workspace serves a second, smaller call; samples too
    r3 = ctx.det(dets[:100].contiguous(), c[:100].contiguous(), x.e0, eps2, "fp64", ws=ws)
    o3 = ref.pt2_det(12, 3, 3, x.h1, x.eri, x.dets[:100], x.c[:100], x.e0, eps2, unique=False)
    assert abs(r3.e2 - o3.e2) <= E2_TOL_FP64 and r3.stats["n_unique"] == o3.n_unique
    sw = torch.empty(ctx.workspace_size("sample", len(x.c), 0, 5, 40), dtype=torch.uint8, device="cuda")
    out_w, _, _, _ = ctx.sample(dets, c, x.e0, 1e-7, 1e-5, None, seed=3, n_samples=5, n_draws=40, ws=sw)
    out_n, _, _, _ = ctx.sample(dets, c, x.e0, 1e-7, 1e-5, None, seed=3, n_samples=5, n_draws=40)
    assert torch.equal(out_w, out_n)


def test_grad_modes():
    x = I.small(12, 3, 3, 300, 3, 21)
    ctx, dets, c = context(x)
    eps2 = 1e-6
    o = ref.pt2_det(12, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0, eps2, unique=False, grad=True)
    res = {}
    for mode in ("keep", "recompute", "auto"):
        e2, g, de0, st = ctx.grad(dets, c, x.e0, eps2, "fp64", mode=mode)
        g = g.cpu().numpy()
        rel = np.linalg.norm(g - o.grad) / np.linalg.norm(o.grad)
        print(f"grad mode {mode}: rel err {rel:.3e}, chunks {st['n_chunks']}")
        assert abs(e2 - o.e2) <= E2_TOL_FP64
        assert rel <= 1e-10
        assert abs(de0 - o.de2_de0) <= 1e-10 * abs(o.de2_de0)
        res[mode] = g
    assert np.linalg.norm(res["keep"] - res["recompute"]) <= 1e-13 * np.linalg.norm(res["recompute"])
    # keep mode is deterministic
    _, g2, _, _ = ctx.grad(dets, c, x.e0, eps2, "fp64", mode="keep")
    assert np.array_equal(g2.cpu().numpy(), res["keep"])
    # auto with a workspace too small for one keep pass: recompute over batches
    _, _, _, st = ctx.grad(dets, c, x.e0, eps2, "fp64", mode="recompute")
    ws = torch.empty(ctx.workspace_size("grad_keep", len(x.c), st["n_records"]) // 3, dtype=torch.uint8,
                     device="cuda")
    e2a, ga, _, sta = ctx.grad(dets, c, x.e0, eps2, "fp64", mode="auto", ws=ws)
    print("auto with a third of the keep workspace:", sta["n_chunks"], "batches")
    assert sta["n_chunks"] > 1
    assert np.linalg.norm(ga.cpu().numpy() - o.grad) <= 1e-10 * np.linalg.norm(o.grad)
    # FP32c keep mode against the oracle
    _, g32, _, _ = ctx.grad(dets, c, x.e0, eps2, "fp32c", mode="keep")
    assert np.linalg.norm(g32.cpu().numpy() - o.grad) <= 1e-6 * np.linalg.norm(o.grad)


def test_three_step_seed_batches():
    # sample batches from the seed: the top log2(n_batches) bits of the
    # SplitMix64 output after those of the draws
    x = I.small(12, 3, 3, 300, 3, 31)
    ctx, dets, c = context(x)
    args = (12, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0)
    ns, nd, nb, seed = 6, 40, 8, 2024
    draws = ref.alias_draws(x.c, ns, nd, seed)
    sb = np.array([ref.splitmix64(seed, 2 * ns * nd + s + 1) >> 61 for s in range(ns)], dtype=np.int32)
    o = ref.pt2_sample_batched(*args, 1e-7, 1e-6, draws, nb, sb)
    out, mean, _, _ = ctx.sample_batched(dets, c, x.e0, 1e-7, 1e-6, None, nb, None, "fp64", seed=seed,
                                         n_samples=ns, n_draws=nd)
    assert np.abs(out.cpu().numpy() - o).max() <= 1e-9 * max(1.0, np.abs(o).max())
    res, per = ctx.three_step(dets, c, x.e0, 1e-4, 1e-6, 1e-7, 1e-30, 4, nb, None, None, "fp64", seed=seed,
                              n_samples=ns, n_draws=nd)
    assert abs(res["e2_sto"] - o.mean()) <= 1e-9
