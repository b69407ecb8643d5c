"""The stored workload inputs are what the CPU reference computes now, and the
generator follows its recipe."""
import numpy as np
import pytest

from synth import generator as G
from synth import store
from tests import inputs as I


@pytest.mark.parametrize("name", ["w0", "w1", "w2"])
def test_stored_inputs_match_reference(name):
    x = store.load(name)           # checks the fingerprints of dets, eri and c
    y = I.workload(name)
    assert np.array_equal(x.c, y.c) and x.e0 == y.e0


def test_generator_recipe():
    x = G.make_raw("w0")
    n = 12
    e = x.eri
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        assert np.array_equal(e, e.transpose(perm))
    # positive semidefinite supermatrix (pq|rs) over pair indices
    m = e.reshape(n * n, n * n)
    assert np.linalg.eigvalsh(m).min() > -1e-12
    assert np.array_equal(np.diag(x.h1), -2.0 + 0.1 * np.arange(n))
    assert np.array_equal(x.h1, x.h1.T)
    # determinants: HF first, unique, right electron counts, levels <= 3
    assert np.array_equal(x.dets[0], G.hf_det(4, 4))
    assert len({d.tobytes() for d in x.dets}) == len(x.dets)
    pc = np.vectorize(lambda v: bin(int(v)).count("1"))
    assert np.all(pc(x.dets[:, 0]) + pc(x.dets[:, 1]) == 4)
    assert np.all(pc(x.dets[:, 2]) + pc(x.dets[:, 3]) == 4)
    hf = x.dets[0]
    lev = (pc(x.dets[:, 0] ^ hf[0]) + pc(x.dets[:, 2] ^ hf[2])) // 2
    assert np.array_equal(lev, x.levels) and lev.max() == 3
    y = store.load("w0")
    assert abs(np.linalg.norm(y.c) - 1.0) < 1e-15 and y.c[0] > 0.9
