"""Benchmark: screened PT2 terms/s and E2 wall time on one MI355X.

Default workload w3: semistochastic PT2, (14 alpha, 14 beta) electrons in 76
orbitals (the Cr2 active-space shape of the paper's section VII), N_var = 1e6,
seeded synthetic inputs (the paper's molecular data are not available).  One
step is one pass of the whole hot path on inputs already resident in HBM:
  - shci_pt2_det at eps2^d = 2e-5 (validation, hash set of V, excitation
    generation, hash partition, bucket sort + segmented reduce + H_aa, E2
    reduction), and
  - shci_pt2_sample on the seed path: the alias table of p_i = |c_i|/sum|c|
    and 256 x 2000 draws made on the device, then the per-sample estimators at
    eps2 = 1e-7 minus eps2^d, in chunks of samples.
Both calls use a caller-owned workspace (torch memory), so the step allocates
nothing.  The FP32-compensated step is timed beside the FP64 one.  The
heat-bath tables are built once per integral set and timed apart.  H c on the
same variational space (shci_pt2_hc) is timed after the steps ("hc"); it is
not part of the step.

--workload w1 times the deterministic 40-orbital workload (one shci_pt2_det
per step).  --workload w4 times the 10^7-determinant workload: FP32c forward
(deterministic part and 512 x 4000 samples) and both recomputing adjoints per
step, with the device memory footprint and the statistical error, plus a
labelled sensitivity run with E0' (the Rayleigh quotient over HF and its MP1
doubles) beside the literal E0.

Prints one JSON line.  --gpus above 1 is rejected: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("PT2 screened terms/s + E2 wall time, FP32-comp vs FP64 at ≤1e-6 Ha; HBM GB/s")
HBM_PEAK_GBS = 8000.0
# plain 32-bit VALU lane operations: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_GOPS = 256 * 4 * 16 * 2.4


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 20; w4: 1)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 3; w4: 0)")
    ap.add_argument("--fp32c-steps", type=int, default=None,
                    help="timed FP32c steps (default: min(steps, 5))")
    ap.add_argument("--workload", default="w3")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU reference baseline")
    ap.add_argument("--no-hc", action="store_true", help="skip the H c timing")
    ap.add_argument("--no-three-step", action="store_true", help="skip the 3-step run")
    ap.add_argument("--lanes", type=int, default=2, help="sample chunks in flight at once (1 or 2)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (HBM counter calibration)")
    ap.add_argument("--profile-summary", default=None, metavar="DIR",
                    help="only summarise the rocprofv3 runs under DIR into profiles/")
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


def measured(workload, kernel):
    """Counter figures of one kernel from the committed summary
    (profiles/counters_<workload>.json): HBM bytes per launch (FETCH_SIZE +
    WRITE_SIZE, scaled by a plain copy's readings) and VALU lane operations
    per launch; None when missing or taken with other kernel sources."""
    f = os.path.join(ROOT, "profiles", f"counters_{workload}.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        t = json.load(fh)
    if t.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return t.get("kernels", {}).get(kernel)


COPY_KERNEL = "__amd_rocclr_copyBuffer"


def _db(path):
    """The rocpd SQLite database under a rocprofv3 output directory."""
    import glob
    import sqlite3
    f = sorted(glob.glob(os.path.join(path, "**", "*_results.db"), recursive=True))
    if not f:
        raise SystemExit(f"no rocprofv3 results database under {path}")
    return sqlite3.connect(f[0])


def _counters(path):
    """Per kernel name: dispatches and the mean of each counter per dispatch."""
    import collections
    cur = _db(path).cursor()
    tot = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for name, cn, val, did in cur.execute(
            "select kernel_name, counter_name, value, dispatch_id from counters_collection"):
        tot[name][cn] += val
        disp[name].add(did)
    return {k: {"dispatches": len(disp[k]), **{c: v / len(disp[k]) for c, v in tot[k].items()}} for k in tot}


def profile_summary(root, workload):
    """Reads the rocprofv3 runs of the profiling recipe (the commands listed at
    the head of profiles/kernels_<workload>.md) under `root` (kernel traces:
    prof/, prof1/; counter passes: pmc_fetch/, pmc_write/, pmc_sq1/, pmc_sq2/;
    copy calibration: pmc_cfetch/, pmc_cwrite/) and writes
    profiles/counters_<workload>.json (per kernel: HBM bytes per launch from
    FETCH_SIZE and WRITE_SIZE scaled by the plain copy's readings, VALU-busy
    lane slots per launch, the counters; with the SHA-256 of the HIP sources)
    and profiles/kernels_<workload>.md."""
    def trace_of(sub):
        cur = _db(os.path.join(root, sub)).cursor()
        # kernel durations in ns
        return [(n, int(c), float(t), float(t) / int(c)) for n, c, t in
                cur.execute("select name, count(*), sum(duration) from kernels group by name "
                            "order by sum(duration) desc")]
    trace = trace_of("prof")
    cal = {}
    for kind, sub in (("FETCH_SIZE", "pmc_cfetch"), ("WRITE_SIZE", "pmc_cwrite")):
        # the probe's copies of 1 GiB read and write 2^30 bytes each; other
        # dispatches of the copy kernel (small transfers) are left out
        cur = _db(os.path.join(root, sub)).cursor()
        kib = [v for (v,) in cur.execute("select value from counters_collection where kernel_name = ? and "
                                         "counter_name = ?", (COPY_KERNEL, kind))]
        big = max(kib) if kib else 0.0
        cal[kind] = (2.0 ** 30) / (big * 1024.0) if big > 0 else None
    per = {}
    for sub in ("pmc_fetch", "pmc_write", "pmc_sq1", "pmc_sq2"):
        if os.path.isdir(os.path.join(root, sub)):
            for k, v in _counters(os.path.join(root, sub)).items():
                per.setdefault(k, {}).update(v)
    kernels = {}
    for name, v in per.items():
        e = {"dispatches": v.get("dispatches"), "counters": {c: x for c, x in v.items() if c != "dispatches"}}
        if cal.get("FETCH_SIZE") and cal.get("WRITE_SIZE") and "FETCH_SIZE" in v and "WRITE_SIZE" in v:
            e["hbm_bytes_per_launch"] = 1024.0 * (v["FETCH_SIZE"] * cal["FETCH_SIZE"] + v["WRITE_SIZE"] * cal["WRITE_SIZE"])
        if "SQ_ACTIVE_INST_VALU" in v:
            # SQ_ACTIVE_INST_VALU counts quad-cycles: 4 cycles x 16 lanes of a SIMD
            e["valu_busy_lane_slots_per_launch"] = 64.0 * v["SQ_ACTIVE_INST_VALU"]
        kernels[name] = e
    out = {"workload": workload, "kernel_sources_sha256": kernel_sources_sha256(),
           "calibration": {"copy_bytes": 2 ** 30, "fetch_factor": cal.get("FETCH_SIZE"),
                           "write_factor": cal.get("WRITE_SIZE")},
           "kernels": kernels}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"counters_{workload}.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    def table(tr, title):
        rows = [title, "",
                "| kernel | calls | total ms | average ms | HBM bytes / launch (counters) | HBM GB/s | VALU busy |",
                "|---|---|---|---|---|---|---|"]
        for n, c, t, a in tr[:24]:
            k = kernels.get(n, {})
            hb = k.get("hbm_bytes_per_launch")
            busy = None
            if k.get("valu_busy_lane_slots_per_launch") and a > 0:
                busy = k["valu_busy_lane_slots_per_launch"] / (a * 1e-9) / (VALU_PEAK_GOPS * 1e9)
            gbs = hb / a if (hb is not None and a > 0) else None
            rows.append(f"| `{n[:90]}` | {c} | {t / 1e6:.2f} | {a / 1e6:.3f} | "
                        f"{'' if hb is None else f'{hb / 1e9:.3f} GB'} | {'' if gbs is None else f'{gbs:.0f}'} | "
                        f"{'' if busy is None else f'{busy:.1%}'} |")
        return rows
    b = "bench.py --steps 1 --warmup 0 --fp32c-steps 0 --no-cpu --no-hc --no-three-step"
    lines = [f"# Kernels of the {workload} benchmark step (MI355X)", "",
             "Commands (repository root, TMPDIR=/tmp), then `python3 bench.py --profile-summary <dir>`:", "", "```",
             f"rocprofv3 --kernel-trace --stats -d <dir>/prof -o w3 -- python3 {b}",
             f"rocprofv3 --pmc FETCH_SIZE -d <dir>/pmc_fetch -o w3 -- python3 {b}",
             f"rocprofv3 --pmc WRITE_SIZE -d <dir>/pmc_write -o w3 -- python3 {b}",
             f"rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_THREAD_CYCLES_VALU SQ_BUSY_CYCLES "
             f"SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY SQ_INSTS_SALU GRBM_GUI_ACTIVE -d <dir>/pmc_sq1 -o w3 -- python3 {b}",
             f"rocprofv3 --pmc SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_VALU_INT64 SQ_INSTS_VALU_INT32 "
             f"SQ_INSTS_VALU_FLOPS_FP64 SQ_WAIT_INST_LDS SQ_LDS_BANK_CONFLICT -d <dir>/pmc_sq2 -o w3 -- python3 {b}",
             "rocprofv3 --pmc FETCH_SIZE -d <dir>/pmc_cfetch -o copy -- python3 bench.py --copy-probe 1024",
             "rocprofv3 --pmc WRITE_SIZE -d <dir>/pmc_cwrite -o copy -- python3 bench.py --copy-probe 1024",
             f"rocprofv3 --kernel-trace --stats -d <dir>/prof1 -o w3 -- python3 {b} --lanes 1",
             "```", ""]
    lines += table(trace, "Kernel trace of the benchmark command (two lanes: kernels of two sample chunks overlap):")
    if os.path.isdir(os.path.join(root, "prof1")):
        lines += [""] + table(trace_of("prof1"), "Kernel trace with one lane (every kernel alone on the GPU):")
    lines += ["", "HBM bytes: FETCH_SIZE and WRITE_SIZE per dispatch (KiB) scaled by a plain copy's readings; "
              "FETCH_SIZE counts L2 fills from the fabric, MALL hits included.",
              f"Calibration: FETCH_SIZE x {cal.get('FETCH_SIZE')}, WRITE_SIZE x {cal.get('WRITE_SIZE')} "
              "(a plain 1 GiB device copy reads and writes 2^30 bytes).",
              "VALU busy: SQ_ACTIVE_INST_VALU x 64 lane slots per launch over the average launch time, against "
              "256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.",
              f"HIP sources SHA-256: {out['kernel_sources_sha256']}"]
    with open(os.path.join(ROOT, "profiles", f"kernels_{workload}.md"), "w") as f:
        f.write("\n".join(lines) + "\n")
    print(json.dumps({"written": [f"profiles/counters_{workload}.json", f"profiles/kernels_{workload}.md"]}))


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
            "ms_reduce", "ms_total", "ms_k_count", "ms_k_write", "ms_k_reduce", "ms_k_part",
            "n_part_launches", "n_part_records", "n_chunks", "n_terms_all", "n_hashes", "n_singletons",
            "ms_k_split")


class Step:
    """One pass of the hot path on resident inputs."""

    def __init__(self, ctx, x, dets, c, ws, grad=False, e0=None):
        self.ctx, self.x, self.dets, self.c, self.ws, self.grad = ctx, x, dets, c, ws, grad
        self.e0 = x.e0 if e0 is None else e0

    def __call__(self, prec):
        ctx, x, wl = self.ctx, self.x, self.x.wl
        st = {}
        if self.grad:
            e2, _, _, sd = ctx.grad(self.dets, self.c, self.e0, wl.eps2, prec, mode="recompute", ws=self.ws)
        else:
            r = ctx.det(self.dets, self.c, self.e0, wl.eps2, prec, ws=self.ws)
            e2, sd = r.e2, r.stats
        st["det"] = sd
        if wl.n_samples:
            kw = dict(seed=wl.draw_seed, n_samples=wl.n_samples, n_draws=wl.n_draws, ws=self.ws)
            if self.grad:
                _, mean, sem, _, _, ss = ctx.sample_grad(self.dets, self.c, self.e0, wl.eps2_sto, wl.eps2, None,
                                                         prec, **kw)
            else:
                _, mean, sem, ss = ctx.sample(self.dets, self.c, self.e0, wl.eps2_sto, wl.eps2, None, prec, **kw)
            st["sample"] = ss
            st["sem"] = sem
            st["e2_det"] = e2
            e2 = e2 + mean
        tot = {k: st["det"][k] + (st["sample"][k] if "sample" in st else 0) for k in SUM_KEYS}
        tot["min_abs_denom"] = min(st["det"]["min_abs_denom"], st.get("sample", st["det"])["min_abs_denom"])
        tot["key_words"] = st.get("sample", st["det"])["key_words"]
        tot["value_bytes"] = st.get("sample", st["det"])["value_bytes"]
        st["total"] = tot
        return e2, st


def timed(step, prec, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    e2 = None
    for _ in range(steps):
        e2, st = step(prec)
        runs.append(st)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    avg = {k: sum(r["total"][k] for r in runs) / len(runs) for k in SUM_KEYS}
    return wall, e2, runs[-1], avg


def roofline(kernel, bound, alg_bytes, launches, ms, measured_kernel):
    """Roofline object of one kernel: algorithmic bytes per launch over its
    average launch duration (HIP events on the library's stream)."""
    if launches <= 0 or ms <= 0:
        return None
    per_launch = alg_bytes / launches
    avg_s = ms * 1e-3 / launches
    achieved = per_launch / avg_s / 1e9
    out = {"bound": bound, "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS, "traffic": None, "alg_bytes": per_launch, "launches": launches,
           "avg_ms": ms / launches}
    if measured_kernel:
        out["traffic"] = measured_kernel.get("hbm_bytes_per_launch")
        if bound == "alu" and measured_kernel.get("valu_busy_lane_slots_per_launch"):
            # VALU-busy lane slots (SQ_ACTIVE_INST_VALU x 64) per second against
            # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
            ops = measured_kernel["valu_busy_lane_slots_per_launch"] / avg_s / 1e9
            out.update({"achieved": ops, "peak": VALU_PEAK_GOPS, "unit": "G VALU lane-slots/s",
                        "frac": ops / VALU_PEAK_GOPS, "hbm_gbs": achieved})
    if bound == "alu" and out["unit"] == "GB/s":
        out["note"] = "VALU counters not taken for these kernel sources; HBM rate shown"
    return out


def split_bytes_per_hash(per_launch):
    """HBM bytes per listed hash of the singleton split's kernels: per
    partition pass the histogram reads the hash (8) and the scatter reads and
    writes hash and work item (24); the repeat finder reads the hash (8), the
    marks read hash and work item (12).  (The bucket bounds read a few hashes
    per bucket.)"""
    import math
    nbits = max(1, math.ceil(math.log2(max(1.0, math.ceil(per_launch / 12500.0)))))
    npass = (nbits + 7) // 8
    return 32.0 * npass + 20.0, npass


def kernel_rooflines(wl, run, avg, prec):
    """Per-kernel rooflines of one step.  Algorithmic bytes: the generator
    writes each record once; the partition reads and writes it once per pass;
    the reduce reads it once (key words, value(s), H_aa).  With the singleton
    split only the terms whose grouping hash repeats are records; every term
    leaves a listed hash (8) and work item (4) from the count walk."""
    tot = run["total"]
    kw, vb = tot["key_words"], tot["value_bytes"]
    rec = 8 * kw + vb + 8 + 4            # key words, value(s), H_aa, bucket id
    red = 8 * kw + vb + 8                # the reduce does not read the bucket id
    nrec = avg["n_records"]
    launches = avg["n_chunks"]           # one generator and one reduce launch per chunk / batch
    sampled = wl.n_samples > 0
    smp = "true" if sampled else "false"
    vt = "double" if prec == "fp64" else "float"
    names = {
        "k_gen_write": (f"void shci::k_gen_write_sample<{kw}, {vt}>(shci::GenArgs)" if sampled
                        else f"void shci::k_gen_write<{kw}, {vt}>(shci::GenArgs)"),
        "k_gen_count": f"void shci::k_gen_count<{kw}, {smp}, {vt}>(shci::GenArgs)",
        "k_part_scatter": f"void shci::k_part_scatter<{kw}, {vt}, {smp}, false>(shci::PassArgs)",
        "k_reduce_wave": f"void shci::k_reduce_wave<{kw}, {smp}, {vt}>(shci::WaveRedArgs)",
    }
    # the deterministic part uses one key word fewer on w3's orbitals when no
    # sample id is packed; its records are a small share and are counted with
    # the sample records' sizes
    out = {
        "k_part_scatter": roofline("k_part_scatter", "hbm", 2.0 * rec * avg["n_part_records"],
                                   avg["n_part_launches"], avg["ms_k_part"],
                                   measured(wl.name, names["k_part_scatter"])),
        "k_reduce_wave": roofline("k_reduce_wave", "hbm", red * nrec, launches, avg["ms_k_reduce"],
                                  measured(wl.name, names["k_reduce_wave"])),
        "k_gen_write": roofline("k_gen_write", "alu", rec * nrec, launches, avg["ms_k_write"],
                                measured(wl.name, names["k_gen_write"])),
        "k_gen_count": roofline("k_gen_count", "alu", 12.0 * avg["n_hashes"], launches, avg["ms_k_count"],
                                measured(wl.name, names["k_gen_count"])),
    }
    if avg["n_hashes"] > 0:
        bph, npass = split_bytes_per_hash(avg["n_hashes"] / max(1.0, launches))
        r = roofline("split", "hbm", bph * avg["n_hashes"], launches, avg["ms_k_split"], None)
        if r:
            r["kernels"] = f"k_hpart_hist + k_hpart_scatter ({npass} passes), k_hbounds, k_hdup, k_hmark"
        out["split"] = r
    ms = {"k_part_scatter": avg["ms_k_part"], "k_reduce_wave": avg["ms_k_reduce"],
          "k_gen_write": avg["ms_k_write"], "k_gen_count": avg["ms_k_count"], "split": avg["ms_k_split"]}
    return out, ms, rec


def cpu_baseline(x, budget_s):
    """The CPU oracle on a bounded sample of the step: the deterministic part
    on the first M determinants of V (HF first), and for a sampled workload
    the first sample (same seed-path draws) at eps2 - eps2^d."""
    from oracle import ref
    wl = x.wl
    n, na, nb = wl.n_orb, wl.n_alpha, wl.n_beta
    t_s, terms_s, desc_s = 0.0, 0, ""
    if wl.n_samples:
        draws = ref.alias_draws(x.c, 1, wl.n_draws, wl.draw_seed)
        t0 = time.perf_counter()
        _, cnt = ref.pt2_sample_counts(n, na, nb, x.h1, x.eri, x.dets, x.c, x.e0, wl.eps2_sto, wl.eps2, draws)
        t_s = time.perf_counter() - t0
        terms_s = int(cnt[0])
        desc_s = f"; sample 0 ({wl.n_draws} draws) at eps2={wl.eps2_sto:g}: {terms_s} terms in {t_s:.2f} s"

    def run(m):
        t0 = time.perf_counter()
        r = ref.pt2_det(n, na, nb, x.h1, x.eri, x.dets[:m], x.c[:m], x.e0, wl.eps2, unique=False)
        return time.perf_counter() - t0, r

    left = max(budget_s - t_s, budget_s / 4)
    m = min(2000 if wl.n_orb <= 50 else 200, len(x.c))
    t, r = run(m)
    if t < left / 3 and m < len(x.c):
        m = min(len(x.c), int(m * left / max(t, 1e-3)))
        t, r = run(m)
    total_t = t + t_s
    return {"value": (r.n_terms + terms_s) / total_t, "unit": "screened terms/s", "cores": ref.max_threads(),
            "kind": "oracle",
            "sample": f"first {m} of {len(x.c)} variational determinants of {wl.name} (HF first) at "
                      f"eps2={wl.eps2:g}: {r.n_terms} terms in {t:.2f} s{desc_s}",
            "seconds": total_t}


def achievable_copy_gbs(mib=2048, reps=5):
    """Bytes read plus written per second of a plain device copy of `mib` MiB
    (torch's copy kernel), the practical HBM rate next to the 8 TB/s peak."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * 8 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


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


def three_step_run(ctx, x, dets, c, ws):
    """The 3-step correction (section IV) once, at the paper's minimum sizes:
    16 pseudo-stochastic batches of P at eps2_psto = 2e-6 (evaluated until the
    error of the rest is below 0.4 x 1e-4 Ha), 16 samples of the workload's
    draws with one of 16 batches of P each; outside the timed steps."""
    import torch
    wl = x.wl
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, _ = ctx.three_step(dets, c, x.e0, wl.eps2, 2e-6, wl.eps2_sto, 1e-4, 16, 16, None, None, "fp64",
                            seed=wl.draw_seed, n_samples=16, n_draws=wl.n_draws, ws=ws)
    torch.cuda.synchronize()
    res["wall_ms"] = (time.perf_counter() - t0) * 1e3
    res.update({"eps2_dtm": wl.eps2, "eps2_psto": 2e-6, "eps2": wl.eps2_sto, "nb_psto": 16, "nb_sto": 16,
                "n_samples": 16, "target_error": 1e-4})
    return res


def e0_prime(ctx, x, dets, c):
    """E0' = <c'|H|c'>/<c'|c'> over HF and its MP1 doubles (their c as
    stored), by H c on that subspace on the device."""
    import numpy as np
    import torch

    from synth import generator as G
    mask = G.double_of_hf_mask(x.levels)
    mask[0] = True
    idx = torch.from_numpy(np.nonzero(mask)[0]).to(dets.device)
    _, _, ev, _ = ctx.hc(dets[idx].contiguous(), c[idx].contiguous())
    return float(ev), int(mask.sum())


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
    if a.profile_summary:
        profile_summary(a.profile_summary, a.workload)
        return
    import torch

    import paper_1809_04600_amd as P
    from synth import store

    big = a.workload == "w4"
    steps = a.steps if a.steps is not None else (1 if big else 20)
    warmup = a.warmup if a.warmup is not None else (0 if big else 3)
    steps32 = a.fp32c_steps if a.fp32c_steps is not None else min(steps, 5)
    print(f"bench: loading {a.workload}", file=sys.stderr, flush=True)
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
    ctx.set_lanes(a.lanes)
    del eri
    torch.cuda.empty_cache()
    # caller-owned workspace: the calls allocate nothing (w4 uses the
    # library's own grow-only buffers, so that the footprint can be read)
    ws = None
    if not big:
        free, _ = torch.cuda.mem_get_info()
        ws = torch.empty(int(0.8 * free) // 256 * 256, dtype=torch.uint8, device=dev)
    step = Step(ctx, x, dets, c, ws, grad=big)
    prec_main = "fp32c" if big else "fp64"
    copy_gbs = achievable_copy_gbs() if ws is not None else None
    for k in range(warmup):
        print(f"bench: warmup {k}", file=sys.stderr, flush=True)
        step(prec_main)
        if not big:
            step("fp32c")
    print(f"bench: timing {steps} {prec_main} steps", file=sys.stderr, flush=True)
    w_main, e2_main, run_main, avg_main = timed(step, prec_main, steps)
    out32 = None
    if not big and steps32 > 0:
        print(f"bench: timing {steps32} fp32c steps", file=sys.stderr, flush=True)
        w32, e2_32, run32, avg32 = timed(step, "fp32c", steps32)
        rl32, ms32, _ = kernel_rooflines(wl, run32, avg32, "fp32c")
        out32 = {"e2": e2_32, "e2_wall_ms": w32 * 1e3, "steps": steps32,
                 "terms_per_s": run32["total"]["n_terms"] / w32, "speedup_vs_fp64": w_main / w32,
                 "abs_diff_vs_fp64_gpu": abs(e2_32 - e2_main), "kernel_ms": ms32,
                 "record_bytes": 8 * run32["total"]["key_words"] + run32["total"]["value_bytes"] + 12}
    tot = run_main["total"]
    n_terms = tot["n_terms"]
    rl, ms, rec = kernel_rooflines(wl, run_main, avg_main, prec_main)
    # the dominant kernel by its own launch time (the split's figure spans
    # several kernels and, with two lanes, the other lane's kernels)
    dom = max((k for k in ms if rl.get(k) and k != "split"), key=ms.get)
    rl_alone = None
    two_lanes = a.lanes > 1 and wl.n_samples and ws is not None  # lanes need a caller workspace
    if two_lanes:
        for r in rl.values():
            if r:
                r["timing"] = ("HIP events around each launch while two sample chunks are in flight: the "
                               "other chunk's kernels share the GPU, so a launch takes longer than alone "
                               "(roofline_one_lane: the same figures from one untimed step on one lane)")
    if two_lanes and steps > 1:
        # one more step, untimed, with every kernel alone on the GPU: the
        # kernels' own launch times (not with a single timed step, the
        # profiling recipe's, whose traces hold the timed step alone)
        print("bench: one single-lane step (kernel times alone)", file=sys.stderr, flush=True)
        ctx.set_lanes(1)
        _, _, run1, avg1 = timed(step, prec_main, 1)
        ctx.set_lanes(a.lanes)
        rl_alone, _, _ = kernel_rooflines(wl, run1, avg1, prec_main)
        for r in rl_alone.values():
            if r:
                r["timing"] = "HIP events around each launch, one lane: each kernel alone on the GPU"
    out = {
        "metric": METRIC,
        "value": n_terms / w_main,
        "unit": "screened terms/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": w_main * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec_main == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.description}", "n_orb": wl.n_orb,
                   "n_alpha": wl.n_alpha, "n_beta": wl.n_beta, "n_var": len(x.c),
                   "eps2": wl.eps2, "n_terms": n_terms, "n_records": tot["n_records"],
                   "n_singletons": tot["n_singletons"], "n_hashes": tot["n_hashes"],
                   "n_unique": tot["n_unique"], "parallelism": "single GPU",
                   "precision": prec_main, "lanes": a.lanes,
                   "workspace_bytes": int(ws.numel()) if ws is not None else None,
                   **({"eps2_sto": wl.eps2_sto, "n_samples": wl.n_samples, "n_draws": wl.n_draws,
                       "draws": f"seed path, seed {wl.draw_seed}", "e2_sem": run_main["sem"],
                       "sample_chunks": run_main["sample"]["n_chunks"]}
                      if wl.n_samples else {}),
                   "min_abs_denom": tot["min_abs_denom"], "n_intruder": tot["n_intruder"]},
        "roofline": rl[dom],
        "roofline_kernels": rl,
        **({"roofline_one_lane": rl_alone[dom], "roofline_kernels_one_lane": rl_alone} if rl_alone else {}),
        "achievable_copy_gbs": copy_gbs,
        "alg_efficiency": {"bytes_per_term": 80.0, "gbs": 80.0 * n_terms / w_main / 1e9,
                           "frac": 80.0 * n_terms / w_main / 1e9 / HBM_PEAK_GBS},
        "e2": e2_main,
        "e2_wall_ms": w_main * 1e3,
        "kernel_ms": ms,
        "phase_ms": {"gen": avg_main["ms_gen"], "sort": avg_main["ms_sort"], "reduce": avg_main["ms_reduce"],
                     "total_device": avg_main["ms_total"]},
        "record_bytes": rec,
        "table_build_ms": table_ms,
    }
    if wl.n_samples:
        out["e2_det"] = run_main["e2_det"]
    if out32:
        out["fp32c"] = out32
    if big:
        free, total = torch.cuda.mem_get_info()
        out["hbm_footprint_gib"] = (total - free) / 2**30
        out["e2_stat_error"] = run_main["sem"]
        ep, nsub = e0_prime(ctx, x, dets, c)
        sens = Step(ctx, x, dets, c, None, grad=False, e0=ep)
        ts = time.perf_counter()
        e2p, runp = sens("fp32c")
        torch.cuda.synchronize()
        out["sensitivity_e0_prime"] = {
            "label": "E0' = Rayleigh quotient over HF and its MP1 doubles (not the workload's E0)",
            "e0_prime": ep, "e0": x.e0, "subspace": nsub, "e2": e2p, "e2_sem": runp["sem"],
            "min_abs_denom": runp["total"]["min_abs_denom"], "n_intruder": runp["total"]["n_intruder"],
            "wall_s": time.perf_counter() - ts}
    if wl.n_samples and not big and not a.no_three_step:
        out["three_step"] = three_step_run(ctx, x, dets, c, ws)
    if not a.no_hc:
        out["hc"] = hc_timing(ctx, x, dets, c)
    if not a.no_cpu:
        print("bench: cpu baseline", file=sys.stderr, flush=True)
        cb = cpu_baseline(x, a.cpu_seconds)
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
