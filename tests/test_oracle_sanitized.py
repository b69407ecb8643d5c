"""The CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, host code only), every entry point run once on a small system in a
child process: no sanitizer report and the same results as the plain build.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

CHILD = r"""
import numpy as np, sys, json
sys.path.insert(0, sys.argv[1])
from oracle import ref
from tests import inputs as I
x = I.small(8, 2, 2, 40, 2, 3)
n, na, nb = 8, 2, 2
a = (n, na, nb, x.h1, x.eri)
o = ref.pt2_det(*a, x.dets, x.c, x.e0, 1e-6, unique=True, terms=True, grad=True)
rng = np.random.default_rng(1)
p = np.abs(x.c) / np.abs(x.c).sum()
dr = rng.choice(len(x.c), size=(3, 12), p=p).astype(np.uint32)
s, cnt = ref.pt2_sample_counts(*a, x.dets, x.c, x.e0, 1e-7, 1e-5, dr)
sg = ref.pt2_sample_grad(*a, x.dets, x.c, x.e0, 1e-7, 1e-5, dr)
b = ref.det_batch(*a, x.dets, x.c, x.e0, 1e-6, 1e-4, 4, 1)
sb = ref.pt2_sample_batched(*a, x.dets, x.c, x.e0, 1e-7, 1e-5, dr, 4, np.array([0, 1, 3], dtype=np.int32))
y, conn = ref.hc_rows(*a, x.dets, x.c)
ec = ref.energy_cores(*a, x.dets, x.c, hash_bits=8)
t = ref.alias_table(x.c)
d = ref.alias_draws(x.c, 3, 17, 7)
h = ref.hij(n, na, nb, x.h1, x.eri, x.dets[1], x.dets[0])
def conv(v):
    if isinstance(v, np.ndarray):
        return conv(v.tolist())
    if isinstance(v, (list, tuple)):
        return [conv(u) for u in v]
    if isinstance(v, (np.floating, float)):
        return float(v).hex()
    if isinstance(v, (np.integer, int)):
        return int(v)
    return repr(v)
print(json.dumps(conv([o.e2, o.de2_de0, o.grad, o.A, o.counts, s, cnt, sg, b, sb, y, conn, ec, t.threshold,
                       t.alias, d, h])))
"""


def _run(env):
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT], env=env, capture_output=True, text=True, timeout=600)
    return r


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_oracle_under_asan_ubsan(tmp_path):
    so = str(tmp_path / "liboracle_asan.so")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                    "-fno-omit-frame-pointer", os.path.join(ORACLE, "pt2_oracle.cpp"),
                    os.path.join(ORACLE, "alias_oracle.cpp"), "-o", so, "-lquadmath"], check=True)
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    env = dict(os.environ)
    env.update({"ORACLE_LIB": so, "LD_PRELOAD": asan, "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1", "OMP_NUM_THREADS": "2"})
    r = _run(env)
    print(r.stderr[-2000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    plain = dict(os.environ)
    plain.pop("ORACLE_LIB", None)
    plain["OMP_NUM_THREADS"] = "2"
    r0 = _run(plain)
    assert r0.returncode == 0, r0.stderr[-4000:]
    # -O1 vs -O2, no contraction in either: the same numbers
    assert r.stdout.strip().splitlines()[-1] == r0.stdout.strip().splitlines()[-1]
