"""shci_pt2_det_static (the entry point that allocates nothing, its
workspace a fixed device array of the library) against shci_pt2_det, through
the C ABI: two calls in a row, the second on a smaller input.  Bars: counts
bit-exact, E2 within 1e-9 Ha of shci_pt2_det (both FP64)."""
import pytest

import paper_1809_04600_amd as P
from oracle import ref
from synth import store
from tests.gpu_util import context

pytestmark = pytest.mark.gpu

KEYS = ("n_terms", "n_terms_gen", "n_unique", "n_intruder")


def test_det_static_matches_det_twice():
    x = store.load("w1")
    wl = x.wl
    ctx, dets, c = context(x)
    try:
        # the whole of w1 (6.5e6 records: hash batches inside the fixed array)
        r = ctx.det(dets, c, x.e0, wl.eps2, "fp64")
        s = ctx.det_static(dets, c, x.e0, wl.eps2, "fp64")
        print(f"w1: det {r.e2!r} static {s.e2!r} batches {s.stats['n_chunks']}", flush=True)
        for k in KEYS:
            assert s.stats[k] == r.stats[k], k
        assert abs(s.e2 - r.e2) <= 1e-9
        # second call, smaller input: the first 3000 determinants
        m = 3000
        d2, c2 = dets[:m].contiguous(), c[:m].contiguous()
        r2 = ctx.det(d2, c2, x.e0, wl.eps2, "fp64")
        s2 = ctx.det_static(d2, c2, x.e0, wl.eps2, "fp64")
        o2 = ref.pt2_det(wl.n_orb, wl.n_alpha, wl.n_beta, x.h1, x.eri, x.dets[:m], x.c[:m], x.e0, wl.eps2,
                         unique=False)
        print(f"w1[:{m}]: det {r2.e2!r} static {s2.e2!r} oracle {o2.e2!r}", flush=True)
        for k in KEYS:
            assert s2.stats[k] == r2.stats[k] == getattr(o2, k), k
        assert abs(s2.e2 - r2.e2) <= 1e-9 and abs(s2.e2 - o2.e2) <= 1e-9
        # beyond the stated maximum: an error, not a fault
        big = dets.repeat(12, 1)[:600000].contiguous()
        cbig = c.repeat(12)[:600000].contiguous()
        with pytest.raises(P.ShciError) as e:
            ctx.det_static(big, cbig, x.e0, wl.eps2, "fp64")  # rejected before any device work
        assert e.value.code == -6
    finally:
        ctx.close()
