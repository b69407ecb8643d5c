"""Benchmark: screened PT2 terms/s and E2 wall time on one MI355X.

Default workload w1: deterministic screened PT2, (8 alpha, 8 beta) electrons in
40 orbitals, N_var = 5e4, eps2 = 1e-5, seeded synthetic inputs (the paper's
molecular data are not available).  One step = one shci_pt2_det call on inputs
already resident in HBM (validation, hash set of V, excitation generation,
hash partition, bucket sort + segmented reduce + H_aa, E2 reduction).
--workload w3 times the semistochastic 76-orbital, 1e6-determinant workload:
one step = the deterministic part at eps2^d plus 256 samples of 2000 draws at
eps2 (shci_pt2_det + shci_pt2_sample).  The heat-bath tables are built once per
integral set (context) and timed apart.  H c on the same variational space
(shci_pt2_hc, string lists + rows) is timed after the steps and reported
under "hc"; it is not part of the step.

Prints one JSON line.  --gpus above 1 is rejected: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("PT2 screened terms/s + E2 wall time, FP32-comp vs FP64 at ≤1e-6 Ha; HBM GB/s")
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="w1")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU reference baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration)")
    return ap.parse_args()


def kernel_sources_sha256():
    """Digest of the HIP sources: HBM counter figures taken with other sources
    are stale and not reported."""
    import hashlib
    d = os.path.join(ROOT, "paper_1809_04600_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def kernel_names(kind, kw, sampled):
    """Full FP64 kernel names behind a bench kernel label."""
    smp = "true" if sampled else "false"
    return {"k_gen(count)": [f"void shci::k_gen_count<{kw}, {smp}, double>(shci::GenArgs)"],
            "k_gen(write)": [f"void shci::k_gen_write_sample<{kw}, double>(shci::GenArgs)" if sampled
                             else f"void shci::k_gen_write<{kw}, double>(shci::GenArgs)"],
            "partition": [f"void shci::k_part_hist<{kw}>(shci::PassArgs)",
                          f"void shci::k_part_scatter<{kw}, double, {smp}, false>(shci::PassArgs)"],
            "k_reduce": [f"void shci::k_reduce_wave<{kw}, {smp}, double>(shci::WaveRedArgs)"]}[kind]


def measured_traffic(workload, names):
    """HBM bytes per launch (per pass for the partition) of the named kernels,
    from the committed counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a
    plain copy's readings); None when missing or taken with other kernel
    sources."""
    f = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        t = json.load(fh)
    if t.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    ks = t.get("kernels", {})
    if not all(n in ks for n in names):
        return None
    return sum(ks[n]["hbm_bytes_per_launch"] for n in names)


def copy_probe(mib):
    import torch
    n = mib * (1 << 20) // 8
    a = torch.arange(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    print(json.dumps({"copy_probe_bytes_read": 8 * n, "copy_probe_bytes_written": 8 * n,
                      "launches": 3}))


SUM_KEYS = ("n_terms", "n_terms_gen", "n_unique", "n_intruder", "n_records", "ms_gen", "ms_sort",
            "ms_reduce", "ms_total", "ms_k_count", "ms_k_write", "ms_k_reduce")


def one_step(ctx, x, dets, c, draws, prec):
    """One pass of the hot path: the deterministic part (at eps2^d for a
    semistochastic workload) and, if the workload samples, every sample."""
    wl = x.wl
    r = ctx.det(dets, c, x.e0, wl.eps2, prec)
    st = dict(r.stats)
    e2 = r.e2
    if draws is not None:
        _, mean, sem, ss = ctx.sample(dets, c, x.e0, wl.eps2_sto, wl.eps2, draws, prec)
        e2 = e2 + mean
        st["sem"] = sem
        st["sample"] = ss
        for k in SUM_KEYS:
            st[k] = st[k] + ss[k]
        st["n_buckets"] = max(st["n_buckets"], ss["n_buckets"])
        st["min_abs_denom"] = min(st["min_abs_denom"], ss["min_abs_denom"])
    return e2, st


def timed(ctx, x, dets, c, draws, prec, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    e2 = None
    for _ in range(steps):
        e2, st = one_step(ctx, x, dets, c, draws, prec)
        stats.append(st)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    avg = {k: sum(s[k] for s in stats) / len(stats) for k in stats[0]
           if isinstance(stats[0][k], float)}
    return wall, e2, stats[-1], avg


def cpu_baseline(x, budget_s):
    """The CPU reference on a bounded sample: the first M determinants of V
    (HF first), M chosen so the run takes about budget_s seconds."""
    from oracle import ref
    wl = x.wl
    n, na, nb = wl.n_orb, wl.n_alpha, wl.n_beta

    def run(m):
        t0 = time.perf_counter()
        r = ref.pt2_det(n, na, nb, x.h1, x.eri, x.dets[:m], x.c[:m], x.e0, wl.eps2, unique=False)
        return time.perf_counter() - t0, r

    m = min(2000 if wl.n_orb <= 50 else 100, len(x.c))
    t, r = run(m)
    if t < budget_s / 3 and m < len(x.c):
        m = min(len(x.c), int(m * budget_s / max(t, 1e-3)))
        t, r = run(m)
    return {"value": r.n_terms / t, "unit": "screened terms/s", "cores": ref.max_threads(),
            "kind": "oracle",
            "sample": f"first {m} of {len(x.c)} variational determinants of {wl.name} "
                      f"(HF first), eps2={wl.eps2:g}; {r.n_terms} screened terms in {t:.2f} s",
            "e2_sample": r.e2, "seconds": t}


def hc_timing(ctx, x, dets, c, reps=3):
    """H c on the same V (string lists and rows), outside the PT2 step:
    device time of the last of `reps` calls, connections per second, and the
    variational energy against the stored E0."""
    ctx.hc(dets, c)
    for _ in range(reps):
        _, _, ev, st = ctx.hc(dets, c)
    return {"ms_total": st["ms_total"], "ms_lists": st["ms_gen"], "ms_rows": st["ms_reduce"],
            "connections": st["n_terms"], "connections_per_s": st["n_terms"] / (st["ms_total"] * 1e-3),
            "e_var_minus_e0": ev - x.e0}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU; --gpus {a.gpus} is not supported "
              "(sharding across GPUs is designed but not implemented)",
              file=sys.stderr)
        sys.exit(2)
    if a.copy_probe:
        copy_probe(a.copy_probe)
        return
    import torch

    import paper_1809_04600_amd as P
    from synth import store

    x = store.load(a.workload)
    wl = x.wl
    dev = "cuda:0"
    h1 = torch.from_numpy(x.h1).to(dev)
    eri = torch.from_numpy(x.eri).to(dev)
    dets = P.dets_tensor(x.dets, dev)
    c = torch.from_numpy(x.c).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = P.Context(h1, eri, wl.n_alpha, wl.n_beta)
    torch.cuda.synchronize()
    table_ms = (time.perf_counter() - t0) * 1e3

    draws = None
    if wl.n_samples:
        # draws proportional to |c_i| (sampling-probability equation), drawn
        # on the host before timing
        import numpy as np
        p = np.abs(x.c) / np.abs(x.c).sum()
        dr = np.random.default_rng(wl.draw_seed).choice(len(x.c), size=(wl.n_samples, wl.n_draws), p=p)
        draws = torch.from_numpy(dr.astype(np.uint32).view(np.int32)).to(dev)
    for _ in range(a.warmup):
        one_step(ctx, x, dets, c, draws, "fp64")
        one_step(ctx, x, dets, c, draws, "fp32c")
    w64, e2_64, s64, avg64 = timed(ctx, x, dets, c, draws, "fp64", a.steps)
    w32, e2_32, s32, avg32 = timed(ctx, x, dets, c, draws, "fp32c", a.steps)

    n_terms = s64["n_terms"]
    n_rec = s64["n_records"]
    # roofline of the part that dominates the step: the samples of a
    # semistochastic workload, else the deterministic call (HIP-event times)
    sampled = "sample" in s64
    src = s64["sample"] if sampled else s64
    tsrc = src if sampled else avg64
    kw = src["key_words"]
    launches = src["n_chunks"] if sampled else 1
    # record bytes: packed key + value(s) + H_aa (FP64) + bucket id
    rec64 = 8 * kw + src["value_bytes"] + 8 + 4
    rec32 = 8 * kw + (s32["sample"] if sampled else s32)["value_bytes"] + 8 + 4
    nrec_src = src["n_records"]
    npass = math.ceil(math.log2(max(src["n_buckets"], 1)) / 8) if src["n_buckets"] > 1 else 0
    kernels = {"k_gen(count)": tsrc["ms_k_count"], "k_gen(write)": tsrc["ms_k_write"],
               "partition": tsrc["ms_sort"], "k_reduce": tsrc["ms_k_reduce"]}
    dom = max(kernels, key=kernels.get)
    # algorithmic bytes over all launches of each kernel
    alg = {"k_gen(count)": 40.0 * len(x.c),             # each source det read once
           "k_gen(write)": rec64 * nrec_src + 40.0 * len(x.c),
           "partition": (2.0 * rec64 + 4.0) * nrec_src * npass,  # hist reads ids; scatter reads + writes
           "k_reduce": rec64 * nrec_src}                 # each record read once
    per_launch = launches * (npass if dom == "partition" else 1)
    achieved = alg[dom] / (kernels[dom] * 1e-3) / 1e9
    reduce_gbs = alg["k_reduce"] / (avg64["ms_k_reduce"] * 1e-3) / 1e9
    sort_gbs = alg["partition"] / (avg64["ms_sort"] * 1e-3) / 1e9 if npass else None
    out = {
        "metric": METRIC,
        "value": n_terms / w64,
        "unit": "screened terms/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": w64 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.description}", "n_orb": wl.n_orb,
                   "n_alpha": wl.n_alpha, "n_beta": wl.n_beta, "n_var": len(x.c),
                   "eps2": wl.eps2, "n_terms": n_terms, "n_records": n_rec,
                   "n_unique": s64["n_unique"], "parallelism": "single GPU",
                   **({"eps2_sto": wl.eps2_sto, "n_samples": wl.n_samples, "n_draws": wl.n_draws,
                       "e2_sem": s64["sem"], "sample_chunks": s64["sample"]["n_chunks"]}
                      if wl.n_samples else {}),
                   "min_abs_denom": s64["min_abs_denom"], "n_intruder": s64["n_intruder"]},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(wl.name, kernel_names(dom, kw, sampled)),
                     "alg_bytes": alg[dom] / max(1, per_launch), "launches": per_launch},
        "e2_fp64": e2_64,
        "e2_wall_ms_fp64": w64 * 1e3,
        "fp32c": {"e2": e2_32, "e2_wall_ms": w32 * 1e3, "terms_per_s": n_terms / w32,
                  "speedup_vs_fp64": w64 / w32, "abs_diff_vs_fp64_gpu": abs(e2_32 - e2_64),
                  "ms_k_reduce": avg32["ms_k_reduce"], "ms_k_write": avg32["ms_k_write"]},
        "kernel_ms_fp64": kernels,
        "phase_ms_fp64": {"gen": avg64["ms_gen"], "sort": avg64["ms_sort"],
                          "reduce": avg64["ms_reduce"], "total_device": avg64["ms_total"]},
        "sort_gbs_fp64": sort_gbs,
        "reduce_gbs_fp64": reduce_gbs,
        "record_bytes": {"fp64": rec64, "fp32c": rec32},
        "table_build_ms": table_ms,
        "hc": hc_timing(ctx, x, dets, c),
    }
    if not a.no_cpu:
        cb = cpu_baseline(x, a.cpu_seconds)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
