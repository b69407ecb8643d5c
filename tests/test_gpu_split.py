"""Singleton split (grouping mode "split") against the CPU oracle and against
the all-records grouping, through the C ABI; mode "auto" (the default) picks
records for small deterministic passes and the split otherwise.

The split decides which terms become records, never which terms belong to
one perturbative determinant: term, determinant and intruder counts are
bit-exact against the oracle, FP64 E2 within 1e-9 Ha of the oracle and within
1e-12 relative of the all-records grouping (another summation order), FP32c
within 1e-6 Ha; per-sample estimates likewise.  A repeat gives the same
bits, also from another workspace, because the filter of repeated hashes
depends on the listed terms only.
"""
import numpy as np
import pytest
import torch

from oracle import ref
from synth import store
from tests import inputs as I
from tests.gpu_util import context as _context

pytestmark = pytest.mark.gpu

E2_TOL_FP64 = 1e-9
E2_TOL_FP32C = 1e-6
COUNTS = ("n_terms", "n_terms_gen", "n_unique", "n_intruder")


def _oracle(x, eps2, **kw):
    wl = x.wl
    return ref.pt2_det(wl.n_orb, wl.n_alpha, wl.n_beta, x.h1, x.eri, x.dets, x.c, x.e0, eps2, **kw)


def context(x):
    """A context that splits every pass it may (whatever its size)."""
    ctx, dets, c = _context(x)
    ctx.set_grouping("split")
    return ctx, dets, c


def _records(ctx, fn):
    ctx.set_grouping("records")
    try:
        return fn()
    finally:
        ctx.set_grouping("split")


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


@pytest.fixture(scope="module")
def small_sys():
    x = I.small(10, 3, 3, 150, 3, 5)
    ctx, dets, c = context(x)
    yield x, ctx, dets, c
    ctx.close()


@pytest.mark.parametrize("eps2", [0.0, 1e-5, 1e-3])
def test_split_det_small(small_sys, eps2):
    x, ctx, dets, c = small_sys
    o = _oracle(x, eps2)
    r = ctx.det(dets, c, x.e0, eps2, "fp64")
    s = r.stats
    print(f"eps2={eps2}: E2 {r.e2!r} oracle {o.e2!r}; terms {s['n_terms_all']} singletons {s['n_singletons']} "
          f"records {s['n_records']} hashes {s['n_hashes']}", flush=True)
    assert s["n_terms_all"] == o.n_terms_gen
    assert s["n_singletons"] + s["n_records"] == s["n_terms_all"]
    assert s["n_hashes"] >= s["n_terms_all"]
    if o.n_terms_gen:
        assert s["n_singletons"] > 0
    for k in COUNTS:
        assert s[k] == getattr(o, k), k
    assert abs(r.e2 - o.e2) <= E2_TOL_FP64
    if o.n_unique:
        assert abs(s["min_abs_denom"] - o.min_abs_denom) <= 1e-12 * max(1.0, abs(x.e0))
    rr = _records(ctx, lambda: ctx.det(dets, c, x.e0, eps2, "fp64"))
    assert rr.stats["n_singletons"] == 0 and rr.stats["n_records"] == o.n_terms_gen
    for k in COUNTS:
        assert rr.stats[k] == s[k], k
    assert _rel(r.e2, rr.e2) <= 1e-12 or abs(r.e2 - rr.e2) <= 1e-15
    r32 = ctx.det(dets, c, x.e0, eps2, "fp32c")
    assert abs(r32.e2 - o.e2) <= E2_TOL_FP32C
    for k in COUNTS:
        assert r32.stats[k] == s[k], k
    # the same bits on a repeat
    assert ctx.det(dets, c, x.e0, eps2, "fp64").e2 == r.e2


def test_split_w0_many_repeats():
    # eps2 = 0: many determinants reached from many sources (large buckets of
    # one repeated hash)
    x = store.load("w0")
    ctx, dets, c = context(x)
    o = _oracle(x, 0.0)
    r = ctx.det(dets, c, x.e0, 0.0, "fp64")
    s = r.stats
    print(f"w0 split: E2 {r.e2!r} oracle {o.e2!r} singletons {s['n_singletons']} records {s['n_records']}",
          flush=True)
    for k in COUNTS:
        assert s[k] == getattr(o, k), k
    assert abs(r.e2 - o.e2) <= E2_TOL_FP64
    assert s["n_records"] >= o.n_terms_gen - o.n_unique
    ws = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    rw = ctx.det(dets, c, x.e0, 0.0, "fp64", ws=ws)
    assert rw.e2 == r.e2 and rw.stats["n_records"] == s["n_records"]
    ctx.close()


def test_split_w1_vs_records():
    x = store.load("w1")
    ctx, dets, c = context(x)
    eps2 = x.wl.eps2
    o = _oracle(x, eps2)
    r = ctx.det(dets, c, x.e0, eps2, "fp64")
    rr = _records(ctx, lambda: ctx.det(dets, c, x.e0, eps2, "fp64"))
    s = r.stats
    print(f"w1: split E2 {r.e2!r} records {rr.e2!r} oracle {o.e2!r}; singletons {s['n_singletons']} of "
          f"{s['n_terms_all']}; ms split {s['ms_k_split']:.3f} write {s['ms_k_write']:.3f} vs "
          f"records write {rr.stats['ms_k_write']:.3f} part {rr.stats['ms_k_part']:.3f}", flush=True)
    for k in COUNTS:
        assert s[k] == rr.stats[k] == getattr(o, k), k
    assert abs(r.e2 - o.e2) <= E2_TOL_FP64
    assert _rel(r.e2, rr.e2) <= 1e-12
    r32 = ctx.det(dets, c, x.e0, eps2, "fp32c")
    assert abs(r32.e2 - o.e2) <= E2_TOL_FP32C
    ctx.close()


def test_split_hash_batches(small_sys):
    x, ctx, dets, c = small_sys
    eps2 = 1e-6
    o = _oracle(x, eps2)
    r1 = ctx.det(dets, c, x.e0, eps2, "fp64")
    ctx.set_record_limit(max(1, o.n_terms_gen // 5))
    try:
        rb = ctx.det(dets, c, x.e0, eps2, "fp64")
    finally:
        ctx.set_record_limit(0)
    print("split batches:", rb.stats["n_chunks"], flush=True)
    assert rb.stats["n_chunks"] >= 4
    for k in COUNTS:
        assert rb.stats[k] == r1.stats[k] == getattr(o, k), k
    assert _rel(rb.e2, r1.e2) <= 1e-13
    assert abs(rb.e2 - o.e2) <= E2_TOL_FP64


def test_split_samples():
    x = I.small(10, 3, 3, 200, 3, 9)
    ctx, dets, c = context(x)
    rng = np.random.default_rng(4)
    p = np.abs(x.c) / np.abs(x.c).sum()
    draws = rng.choice(len(x.c), size=(13, 50), p=p).astype(np.uint32)
    dr = torch.from_numpy(draws.view(np.int32)).cuda()
    eps2, eps2_d = 1e-6, 1e-4
    o, ocnt = ref.pt2_sample_counts(10, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0, eps2, eps2_d, draws)
    out, mean, sem, st = ctx.sample(dets, c, x.e0, eps2, eps2_d, dr, "fp64")
    out = out.cpu().numpy()
    scale = max(1.0, np.abs(o).max())
    print(f"split samples: max |d| {np.abs(out - o).max():.3e}, singletons {st['n_singletons']} of "
          f"{st['n_terms_all']}", flush=True)
    assert st["n_singletons"] > 0
    assert st["n_terms"] == int(ocnt.sum())
    assert np.abs(out - o).max() <= 1e-9 * scale
    outr, _, _, str_ = _records(ctx, lambda: ctx.sample(dets, c, x.e0, eps2, eps2_d, dr, "fp64"))
    for k in COUNTS:
        assert str_[k] == st[k], k
    assert np.abs(outr.cpu().numpy() - out).max() <= 1e-12 * scale
    # chunks of samples
    ctx.set_record_limit(max(1, st["n_terms_all"] // 6))
    try:
        outc, _, _, stc = ctx.sample(dets, c, x.e0, eps2, eps2_d, dr, "fp64")
    finally:
        ctx.set_record_limit(0)
    assert stc["n_chunks"] >= 4 and stc["n_terms"] == st["n_terms"]
    assert np.abs(outc.cpu().numpy() - out).max() <= 1e-13 * scale
    # equal thresholds: every term cancels its own contribution
    out0, _, _, _ = ctx.sample(dets, c, x.e0, eps2, eps2, dr, "fp64")
    assert np.all(out0.cpu().numpy() == 0.0)
    out32, _, _, _ = ctx.sample(dets, c, x.e0, eps2, eps2_d, dr, "fp32c")
    assert np.abs(out32.cpu().numpy() - o).max() <= 1e-6
    # seed path, repeat: same bits
    a1 = ctx.sample(dets, c, x.e0, 1e-7, 1e-5, None, seed=11, n_samples=7, n_draws=64)[0]
    a2 = ctx.sample(dets, c, x.e0, 1e-7, 1e-5, None, seed=11, n_samples=7, n_draws=64)[0]
    assert torch.equal(a1, a2)
    ctx.close()


def test_split_two_thresholds():
    # batches of P at two thresholds (terms above the upper one flagged) and
    # one batch of P per sample: split against all-records
    x = I.small(12, 3, 3, 300, 3, 31)
    ctx, dets, c = context(x)
    args = (12, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0)
    eps_dtm, eps_psto, eps2 = 1e-4, 1e-6, 1e-7
    rows, _ = ctx.det_batches(dets, c, x.e0, eps_psto, eps_dtm, 4, [0, 1, 2, 3], "fp64")
    rows_r, _ = _records(ctx, lambda: ctx.det_batches(dets, c, x.e0, eps_psto, eps_dtm, 4, [0, 1, 2, 3], "fp64"))
    for b, (r, rr) in enumerate(zip(rows, rows_r)):
        o = ref.det_batch(*args, eps_psto, eps_dtm, 4, b)
        assert r[2] == rr[2] == o[2] and r[3] == rr[3] == o[3]
        assert abs(r[0] - o[0]) <= 1e-12 * max(1e-300, abs(o[0])) + 1e-15
        assert abs(r[0] - rr[0]) <= 1e-12 * max(1e-300, abs(rr[0])) + 1e-15
    rng = np.random.default_rng(37)
    p = np.abs(x.c) / np.abs(x.c).sum()
    draws = rng.choice(len(x.c), size=(6, 40), p=p).astype(np.uint32)
    sb = rng.integers(0, 8, size=6).astype(np.int32)
    dr = torch.from_numpy(draws.view(np.int32)).cuda()
    sbt = torch.from_numpy(sb).cuda()
    out, _, _, _ = ctx.sample_batched(dets, c, x.e0, eps2, eps_psto, dr, 8, sbt, "fp64")
    o = ref.pt2_sample_batched(*args, eps2, eps_psto, draws, 8, sb)
    assert np.abs(out.cpu().numpy() - o).max() <= 1e-9 * max(1.0, np.abs(o).max())
    ctx.close()


def test_two_lanes_same_bits():
    # with a caller workspace the later sample chunks run two at a time (two
    # streams, two host threads); the chunk plan does not depend on that, so
    # the results equal the one-lane run on context memory bit for bit
    x = I.small(10, 3, 3, 200, 3, 9)
    ctx, dets, c = context(x)
    eps2, eps2_d = 1e-6, 1e-4
    kw = dict(seed=5, n_samples=40, n_draws=50)
    out1, m1, _, st1 = ctx.sample(dets, c, x.e0, eps2, eps2_d, None, "fp64", **kw)
    ctx.set_record_limit(max(1, st1["n_terms_all"] // 12))
    ws = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    try:
        outl, ml, _, stl = ctx.sample(dets, c, x.e0, eps2, eps2_d, None, "fp64", **kw)
        outw, mw, _, stw = ctx.sample(dets, c, x.e0, eps2, eps2_d, None, "fp64", ws=ws, **kw)
        outw2 = ctx.sample(dets, c, x.e0, eps2, eps2_d, None, "fp64", ws=ws, **kw)[0]
        ctx.set_lanes(1)
        outw1 = ctx.sample(dets, c, x.e0, eps2, eps2_d, None, "fp64", ws=ws, **kw)[0]
    finally:
        ctx.set_record_limit(0)
        ctx.set_lanes(2)
    print(f"two lanes: chunks {stl['n_chunks']} / {stw['n_chunks']}", flush=True)
    assert stw["n_chunks"] >= 4 and stw["n_chunks"] == stl["n_chunks"]
    assert torch.equal(outw, outl) and torch.equal(outw, outw2) and torch.equal(outw, outw1)
    for k in COUNTS + ("n_terms_all",):
        assert stw[k] == stl[k] == st1[k], k
    # the records (repeated hashes and the filter's false positives) depend
    # on the chunk plan only
    assert stw["n_records"] == stl["n_records"]
    draws = ctx.draws(c, 40, 50, 5).cpu().numpy().astype(np.uint32)
    o = ref.pt2_sample(10, 3, 3, x.h1, x.eri, x.dets, x.c, x.e0, eps2, eps2_d, draws)
    assert np.abs(outw.cpu().numpy() - o).max() <= 1e-9 * max(1.0, np.abs(o).max())
    ctx.close()


def test_auto_grouping_by_size():
    # "auto": a deterministic pass under 1e8 kept terms groups every term as
    # a record (the same bits as "records"); a sampling pass splits
    x = store.load("w1")
    ctx, dets, c = _context(x)
    eps2 = x.wl.eps2
    ra = ctx.det(dets, c, x.e0, eps2, "fp64")
    rr = _records(ctx, lambda: ctx.det(dets, c, x.e0, eps2, "fp64"))
    ctx.set_grouping("auto")
    rs = ctx.det(dets, c, x.e0, eps2, "fp64")
    print(f"auto: {ra.stats['n_singletons']} singletons, E2 {ra.e2!r}; records {rr.e2!r}", flush=True)
    assert ra.stats["n_singletons"] == 0 and ra.stats["n_records"] == rr.stats["n_records"]
    assert ra.e2 == rr.e2 and ra.e2 == rs.e2
    kw = dict(seed=7, n_samples=4, n_draws=200)
    out, _, _, st = ctx.sample(dets, c, x.e0, 1e-7, eps2, None, "fp64", **kw)
    assert st["n_singletons"] > 0
    ctx.close()


@pytest.mark.parametrize("bucket", [60000, 400000])
def test_split_large_buckets(bucket):
    # repeat-finder buckets larger than the threads' registers hold (hashes
    # read from memory) and with more distinct tags than the shared-memory
    # table holds (the bucket is taken again in slices): the same counts as
    # the default buckets and the oracle, E2 within 1e-9 Ha of the oracle and
    # 1e-12 relative of the default (another set of shared tags, another
    # order of the sums), the same bits on a repeat
    x = store.load("w1")
    ctx, dets, c = context(x)
    eps2 = x.wl.eps2
    o = _oracle(x, eps2)
    r0 = ctx.det(dets, c, x.e0, eps2, "fp64")
    ctx.set_split_bucket(bucket)
    r1 = ctx.det(dets, c, x.e0, eps2, "fp64")
    r2 = ctx.det(dets, c, x.e0, eps2, "fp64")
    print(f"bucket {bucket}: E2 {r1.e2!r} default {r0.e2!r} oracle {o.e2!r}; singletons "
          f"{r1.stats['n_singletons']} vs {r0.stats['n_singletons']}, ms split {r1.stats['ms_k_split']:.2f} vs "
          f"{r0.stats['ms_k_split']:.2f}", flush=True)
    for k in COUNTS:
        assert r1.stats[k] == r0.stats[k] == getattr(o, k), k
    assert r1.stats["n_singletons"] > 0
    assert abs(r1.e2 - o.e2) <= E2_TOL_FP64
    assert _rel(r1.e2, r0.e2) <= 1e-12
    assert r1.e2 == r2.e2
    kw = dict(seed=11, n_samples=4, n_draws=300)
    out1, _, _, s1 = ctx.sample(dets, c, x.e0, 1e-7, eps2, None, "fp64", **kw)
    ctx.set_split_bucket(12500)
    out0, _, _, s0 = ctx.sample(dets, c, x.e0, 1e-7, eps2, None, "fp64", **kw)
    assert s1["n_terms"] == s0["n_terms"]
    assert torch.allclose(out1, out0, rtol=1e-11, atol=1e-15)
    with pytest.raises(Exception):
        ctx.set_split_bucket(10)
    ctx.close()
