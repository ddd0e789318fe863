#!/usr/bin/env python3
"""Benchmark of the positional cross-match hot path on one MI355X.

Default workload (the headline line): the largest single-GPU
configuration, 200M A x 200M B on the full sky with galactic-plane
clustering (density proportional to 1 + 20 exp(-|b| / 5 deg); B = 100M
jittered copies of A rows + 100M random from the same density), radius
1.5", all + best matches. One step = c3x_build_index over B + c3x_match of
A (both catalogues already resident in HBM): keying, sorting, directory, A
preparation, count and emission, band recheck, scan, placement, best,
ordering. The 10M x 10M full-sky workload with its dense caps (RA 0/360 and
the north pole, r = 2") is measured in the same run and reported under
"extra" (--no-extra skips it).

The headline value is A-sources matched per second of the mixed path (FP32
filter + FP64 recheck); the FP64 path, pair tests per second, the roofline of
the dominant kernel and the CPU oracle timed on this host are reported beside
it. --config picks the other workloads (one JSON line each):
  cfg1  10k x 10k patch, r = 1" (launch-latency bound; microseconds)
  cfg2  10M x 10M full sky + dense caps, r = 2"
  cfg3  100k galactic ellipses against 50M in-band sources, all matches
  cfg4  4,096 independent circular jobs in one graph launch (batched form)
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM counters of the count pass per workload (rocprofv3 --pmc FETCH_SIZE,
# WRITE_SIZE), committed with the digest of the sources they were taken on;
# reported as roofline.traffic only while those sources are unchanged.
COUNTERS = {
    "cfg2": os.path.join(ROOT, "profiles", "k_match_fullsky_10Mx10M_hbm_counters.md"),
    "cfg5": os.path.join(ROOT, "profiles", "k_match_plane_200Mx200M_hbm_counters.md"),
}
MATCH_SOURCES = ("paper_1611_08494_amd/csrc/c3x_match.hip",
                 "paper_1611_08494_amd/csrc/c3x_internal.h")


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for p in MATCH_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def committed_traffic(config: str, path_name: str):
    """HBM bytes per launch of the count pass on a workload from the committed
    counter summary, if it was taken on the kernel as built; else None."""
    if config not in COUNTERS:
        return None
    try:
        with open(COUNTERS[config]) as f:
            text = f.read()
    except OSError:
        return None
    d = re.search(r"source digest: ([0-9a-f]+)", text)
    t = re.search(rf"traffic {path_name}: (\d+) bytes", text)
    if d and t and d.group(1) == kernel_source_digest():
        return int(t.group(1))
    return None
METRIC = "A-sources matched/s + pair tests/s, mixed vs FP64 path (exact pair set)"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--config", choices=["cfg1", "cfg2", "cfg3", "cfg4", "cfg5"], default="cfg5")
    p.add_argument("--no-extra", action="store_true",
                   help="skip the 10M x 10M full-sky line reported beside the default one")
    p.add_argument("--no-per-job", action="store_true",
                   help="batched workload: skip timing the jobs as separate calls")
    p.add_argument("--core-only", action="store_true",
                   help="time the step only (no join-type or concentric-ellipse timings)")
    p.add_argument("--scale", type=float, default=1.0,
                   help="shrink the workload (testing only; the reported line uses 1.0)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-threads", type=int, default=0)
    p.add_argument("--precision", choices=["both", "mixed", "fp64"], default="both")
    p.add_argument("--separate-calls", action="store_true",
                   help="a step as c3x_build_index then c3x_match (default: c3x_cross_match, "
                        "which keys and sorts A while B's index is built)")
    p.add_argument("--calib-copy-mb", type=int, default=0,
                   help="also run one plain device copy of this size (to scale HBM counters)")
    return p.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def mean(xs):
    return sum(xs) / max(1, len(xs))


def run_path(c3x, torch, tens, cat, precision, steps, warmup, area_kw, frame, mode,
             separate=False):
    """One step: the index over B and the match of A, as one c3x_cross_match
    call (A keyed and sorted while B's index is built) or, with ``separate``,
    as c3x_build_index then c3x_match."""
    raA, decA, raB, decB = tens
    last = {}

    def step():
        if separate:
            ix = c3x.build_index(raB, decB, frame=frame, reach_hint_arcsec=cat.reach_arcsec(),
                                 precision=precision)
            r = c3x.match(ix, raA, decA, frame=frame, mode=mode, **area_kw)
        else:
            r, ix = c3x.cross_match(raB, decB, raA, decA, frame=frame,
                                    reach_hint_arcsec=cat.reach_arcsec(), precision=precision,
                                    mode=mode, keep_index=True, **area_kw)
        last["index"] = ix.stats()
        ix.free()
        last["r"] = r

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    kstats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
        kstats.append((last["index"], last["r"].stats))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / steps
    return ms, last["r"], kstats


def algorithmic_bytes(cat, n_pairs, pay, best):
    """Bytes the method must move for one cross-match (per B: 16 B of
    coordinates in and its 16 B (mixed) or 32 B (FP64) payload out; per A:
    16 B in, 24 B of ellipse parameters in, 12 B of best match out (BEST);
    per pair: 16 B out)."""
    per_a = 16 + (24 if cat.shape == 1 else 0) + (12 if best else 0)
    return cat.nB * (16 + pay) + cat.nA * per_a + int(n_pairs) * 16


def host_cores():
    """CPUs this process may run on, the host's count and its CPU model."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return avail, os.cpu_count() or 1, model


def time_unmatched(c3x, torch, cat, r, steps):
    """The join types' own step (c3x_result_unmatched, selection ALL) on a
    result: mean time over `steps` calls, each of which returns with its
    counts. Algorithmic bytes: the flags cleared (1 B per row of either
    catalogue), every stored pair read (8 B), the flags read twice (count,
    then compaction), 4 B written per unmatched row."""
    c3x.unmatched(r, c3x.ALL)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        ua, ub = c3x.unmatched(r, c3x.ALL)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / steps
    nu = int(ua.shape[0]) + int(ub.shape[0])
    alg = 3 * (cat.nA + cat.nB) + 8 * int(r.n_pairs) + 4 * nu
    return {"ms": round(ms, 4), "unmatched_a": int(ua.shape[0]), "unmatched_b": int(ub.shape[0]),
            "algorithmic_bytes": alg, "GB_per_s": round(alg / (ms / 1e3) / 1e9, 1)}


CONCENTRIC_SCALES = [0.5, 1.0, 1.5, 2.0]


def time_concentric(c3x, torch, tens, cat, precision, steps, area_kw, frame):
    """ClumpPopulator's concentric ellipses (c3x_match_concentric) at
    CONCENTRIC_SCALES over one index: mean time of a call (one certified
    elliptical match per scale plus the level marking), and the pairs per
    level."""
    raA, decA, raB, decB = tens
    ix = c3x.build_index(raB, decB, frame=frame, reach_hint_arcsec=cat.reach_arcsec(),
                         precision=precision)
    kw = dict(a=area_kw["a"], b=area_kw["b"], pa=area_kw["pa"], scales=CONCENTRIC_SCALES,
              frame=frame, pa_zero_deg=area_kw["pa_zero_deg"], pa_sense=area_kw["pa_sense"],
              mode=c3x.ALL)
    r = c3x.match_concentric(ix, raA, decA, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        r = c3x.match_concentric(ix, raA, decA, **kw)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / steps
    per = torch.bincount(r.level.long(), minlength=len(CONCENTRIC_SCALES)).tolist()
    ix.free()
    return {"scales": CONCENTRIC_SCALES, "ms": round(ms, 3), "pairs": int(r.n_pairs),
            "pairs_per_level": per}


def path_summary(cat, ms, r, ks, pay, best):
    ist = [k[0] for k in ks]
    mst = [k[1] for k in ks]
    alg = algorithmic_bytes(cat, r.n_pairs, pay, best)
    return dict(
        algorithmic_bytes=int(alg),
        step_hbm_frac=round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        ms_per_step=ms,
        a_per_s=cat.nA / (ms / 1e3),
        pair_tests=int(mst[-1]["n_tests"]),
        pair_tests_per_s=mst[-1]["n_tests"] / (ms / 1e3),
        n_pairs=int(r.n_pairs),
        n_band=int(mst[-1]["n_band"]),
        n_ambiguous=int(mst[-1]["n_ambiguous"]),
        n_best_ties=int(mst[-1]["n_best_ties"]),
        n_sort_retries=int(max(s["n_sort_retries"] for s in ist + mst)),
        phases_ms=dict(
            index=mean([s["ms_index"] for s in ist]),
            a_prep=mean([s["ms_a_prep"] for s in mst]),
            count=mean([s["ms_count"] for s in mst]),
            count_kernel=mean([s["ms_count_kernel"] for s in mst]),
            scan=mean([s["ms_scan"] for s in mst]),
            write=mean([s["ms_write"] for s in mst]),
            order=mean([s["ms_sort_pairs"] for s in mst]),
            match_total=mean([s["ms_total"] for s in mst]),
        ),
        cell_arcsec=ist[-1]["cell_arcsec"],
        n_cells=int(ist[-1]["n_cells"]),
    )


def oracle_baseline(cat, area_kw_np, threads, sample_rows, what):
    """The CPU oracle (plain C, FP64 certified + mpmath) on the first
    ``sample_rows`` A rows against all of B, timed on this host."""
    import numpy as np
    import oracle
    n = min(cat.nA, sample_rows)
    kw = dict(area_kw_np)
    for k in ("a", "b", "pa"):
        if k in kw:
            kw[k] = np.ascontiguousarray(kw[k][:n])
    t = time.perf_counter()
    o = oracle.match(cat.raA[:n], cat.decA[:n], cat.raB, cat.decB, nthreads=threads, **kw)
    dt = time.perf_counter() - t
    _, ncpu, model = host_cores()
    return {"value": round(n / dt, 1), "unit": "A-sources/s", "cores": int(o.threads),
            "kind": "oracle", "host_cpus": ncpu, "cpu_model": model,
            "sample": f"{what}: first {n} A rows against all {cat.nB} B rows "
            f"(index build included), {dt:.1f}s wall"}, o


def single_config(a, c3x, torch, np, name):
    import synth
    gen = {"cfg1": lambda: synth.cfg1_patch(),
           "cfg2": lambda: synth.cfg2_fullsky(scale=a.scale),
           "cfg3": lambda: synth.cfg3_galactic_ellipses(scale=a.scale),
           "cfg5": lambda: synth.cfg5_scale(scale=a.scale)}[name]
    t = time.perf_counter()
    cat = gen()
    log(f"generated {cat.name} ({cat.nA} A, {cat.nB} B) in {time.perf_counter() - t:.1f}s")
    dev = torch.device("cuda:0")
    tens = [torch.as_tensor(x, device=dev) for x in (cat.raA, cat.decA, cat.raB, cat.decB)]
    frame = c3x.GALACTIC if cat.frame == 1 else c3x.EQUATORIAL
    if cat.shape == 1:
        area_kw = dict(shape=c3x.ELLIPSE, a=torch.as_tensor(cat.a_arcsec, device=dev),
                       b=torch.as_tensor(cat.b_arcsec, device=dev),
                       pa=torch.as_tensor(cat.pa_deg, device=dev), pa_zero_deg=cat.pa_zero_deg,
                       pa_sense=cat.pa_sense)
        area_np = dict(shape=1, a=cat.a_arcsec, b=cat.b_arcsec, pa=cat.pa_deg,
                       pa_zero_deg=cat.pa_zero_deg, pa_sense=cat.pa_sense)
        mode = c3x.ALL
    else:
        area_kw = dict(shape=c3x.CIRCLE, radius_arcsec=cat.radius_arcsec)
        area_np = dict(shape=0, radius_arcsec=cat.radius_arcsec)
        mode = c3x.ALL | c3x.BEST
    torch.cuda.synchronize()
    if a.calib_copy_mb:
        n = a.calib_copy_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {a.calib_copy_mb} MiB done")
        del src, dst

    paths = {}
    order = {"both": ["mixed", "fp64"], "mixed": ["mixed"], "fp64": ["fp64"]}[a.precision]
    for pname in order:
        prec = c3x.MIXED if pname == "mixed" else c3x.FP64
        ms, r, ks = run_path(c3x, torch, tens, cat, prec, a.steps, a.warmup, area_kw, frame, mode,
                             separate=a.separate_calls)
        paths[pname] = path_summary(cat, ms, r, ks, 16 if pname == "mixed" else 32,
                                    bool(mode & c3x.BEST))
        if mode & c3x.ALL and not a.core_only:
            paths[pname]["join_unmatched"] = time_unmatched(c3x, torch, cat, r, a.steps)
        del r
        if cat.shape == 1 and not a.core_only:
            paths[pname]["concentric"] = time_concentric(c3x, torch, tens, cat, prec, a.steps,
                                                         area_kw, frame)
        log(f"{pname}: {ms:.3f} ms/step, {paths[pname]['phases_ms']}")

    head = paths[order[0]]
    # Dominant kernel of the path: the single pass that counts and emits the
    # matches (k_match<..., 2>, one launch per step); its duration is the
    # library's pair of HIP events around that launch alone, on the stream it
    # runs on (the count phase adds the wavefront-per-row kernel, the band
    # recheck and the read-back). Algorithmic bytes per launch: those of the
    # whole cross-match (algorithmic_bytes), since the one launch reads every
    # A and every B payload and decides every pair.
    # When most rows have many candidates (ellipses in a dense band), the
    # wavefront-per-row kernel does the counting instead: the count phase
    # (both kernels, the band recheck and one read-back) is then the figure.
    hp = head["phases_ms"]
    alg_bytes = head["algorithmic_bytes"]
    lane_kernel = hp["count_kernel"] >= 0.5 * hp["count"]
    kms = hp["count_kernel"] if lane_kernel else hp["count"]
    achieved = alg_bytes / (kms / 1e3) / 1e9
    roofline = {"bound": "hbm",
                "kernel": "k_match (count + emit pass)" if lane_kernel else
                          "count phase (k_match_wide + k_match)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": (committed_traffic(name, order[0])
                            if a.scale == 1.0 and lane_kernel else None),
                "algorithmic_bytes_per_launch": int(alg_bytes),
                "kernel_ms": round(kms, 4),
                "step_frac": head["step_hbm_frac"]}

    cpu = None
    if not a.no_cpu_baseline:
        avail, _, _ = host_cores()
        threads = a.cpu_threads or avail
        sample = {"cfg1": cat.nA, "cfg2": cat.nA, "cfg3": 20_000, "cfg5": 2_000_000}[name]
        cpu, o = oracle_baseline(cat, area_np, threads, sample, name)
        if sample >= cat.nA and int(len(o.ia)) != head["n_pairs"]:
            log(f"WARNING: oracle pairs {len(o.ia)} != GPU {head['n_pairs']}")

    workloads = {
        "cfg1": "1 deg patch 10k A x 10k B, r=1\", all+best, index build + match per step",
        "cfg2": "full-sky 10M A x 10M B + dense caps (RA 0/360, north pole), r=2\", all+best, "
                "index build + match per step",
        "cfg3": "galactic band 100k ellipse A (a 5-60\") x 50M B, all matches, index build + "
                "match per step",
        "cfg5": "full-sky 200M A x 200M B, galactic-plane clustering, r=1.5\", all+best, index "
                "build + match per step",
    }
    line = {
        "metric": METRIC,
        "value": round(head["a_per_s"], 1),
        "unit": "A-sources/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if order[0] == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": workloads[name], "nA": cat.nA, "nB": cat.nB,
                   "scale": a.scale, "parallelism": "single GPU"},
        "pair_tests_per_s": round(head["pair_tests_per_s"], 1),
        "step_calls": ("c3x_build_index + c3x_match" if a.separate_calls else "c3x_cross_match"),
        "paths": paths,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if "fp64" in paths and "mixed" in paths:
        line["speedup_mixed_vs_fp64"] = round(paths["fp64"]["ms_per_step"] /
                                              paths["mixed"]["ms_per_step"], 3)
    return line


def per_job_ms(c3x, torch, tens, jobs, prec, reps=2):
    """The batch's jobs as separate calls: for each job c3x_build_index over
    its B rows and c3x_match of its A rows (all + best) on slices of the
    same device arrays; the last of `reps` passes over all jobs is timed."""
    raA, decA, raB, decB = tens
    ms = 0.0
    for rep in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        for (ao, na, bo, nb, r) in jobs:
            ix = c3x.build_index(raB[bo:bo + nb], decB[bo:bo + nb], reach_hint_arcsec=r,
                                 precision=prec)
            res = c3x.match(ix, raA[ao:ao + na], decA[ao:ao + na], radius_arcsec=r,
                            mode=c3x.ALL | c3x.BEST)
            ix.free()
            del res
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3
    return ms


def batch_config(a, c3x, torch, np):
    import synth
    t = time.perf_counter()
    cat = synth.cfg4_jobs(scale=a.scale)
    jobs = [tuple(int(v) for v in r[:4]) + (float(r[4]),) for r in cat.jobs]
    log(f"generated {cat.name}: {len(jobs)} jobs, {cat.nA} A, {cat.nB} B in "
        f"{time.perf_counter() - t:.1f}s")
    dev = torch.device("cuda:0")
    tens = [torch.as_tensor(x, device=dev) for x in (cat.raA, cat.decA, cat.raB, cat.decB)]
    torch.cuda.synchronize()
    paths = {}
    order = {"both": ["mixed", "fp64"], "mixed": ["mixed"], "fp64": ["fp64"]}[a.precision]
    for pname in order:
        prec = c3x.MIXED if pname == "mixed" else c3x.FP64
        t = time.perf_counter()
        b = c3x.Batch(jobs, *tens, precision=prec)
        plan_s = time.perf_counter() - t
        for _ in range(a.warmup):
            b.run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gms = []
        for _ in range(a.steps):
            b.run()
            gms.append(b.stats()["ms_total"])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / a.steps
        st = b.stats()
        alg = algorithmic_bytes(cat, st["n_pairs"], 16 if prec == c3x.MIXED else 32, True)
        paths[pname] = dict(ms_per_step=ms, graph_ms=mean(gms), a_per_s=cat.nA / (ms / 1e3),
                            algorithmic_bytes=int(alg),
                            step_hbm_frac=round(alg / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
                            pair_tests=int(st["n_tests"]),
                            pair_tests_per_s=st["n_tests"] / (ms / 1e3),
                            n_pairs=int(st["n_pairs"]), n_band=int(st["n_band"]),
                            n_ambiguous=int(st["n_ambiguous"]),
                            n_best_ties=int(st["n_best_ties"]), plan_s=round(plan_s, 2),
                            cell_scale=st["cell_arcsec"], tile=int(st["tile"]),
                            queue=int(st["queue"]))
        log(f"{pname}: {ms:.3f} ms/step (graph {mean(gms):.3f} ms), plan {plan_s:.1f}s")
        b.free()
        if not a.no_per_job:
            pj = per_job_ms(c3x, torch, tens, jobs, prec)
            paths[pname]["per_job_ms"] = round(pj, 3)
            paths[pname]["batched_speedup_vs_per_job"] = round(pj / ms, 3)
            log(f"{pname}: the same jobs as separate calls {pj:.3f} ms")
    head = paths[order[0]]
    cpu = None
    if not a.no_cpu_baseline:
        import oracle
        avail, ncpu, model = host_cores()
        threads = a.cpu_threads or avail
        t = time.perf_counter()
        n = 0
        for (ao, na, bo, nb, r) in jobs:
            oracle.match(cat.raA[ao:ao + na], cat.decA[ao:ao + na], cat.raB[bo:bo + nb],
                         cat.decB[bo:bo + nb], radius_arcsec=r, nthreads=threads)
            n += na
            if time.perf_counter() - t > 20.0:
                break
        dt = time.perf_counter() - t
        cpu = {"value": round(n / dt, 1), "unit": "A-sources/s", "cores": threads,
               "kind": "oracle", "host_cpus": ncpu, "cpu_model": model,
               "sample": f"cfg4: jobs in order until 20 s ({n} A rows), {dt:.1f}s wall"}
    line = {
        "metric": METRIC,
        "value": round(head["a_per_s"], 1),
        "unit": "A-sources/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if order[0] == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"batched: {len(jobs)} circular jobs (nA lognormal median 2k, "
                               "nB = 10 nA, 0.5 deg caps, r U[0.5, 10)\"), one graph launch "
                               "per step", "nA": cat.nA, "nB": cat.nB, "scale": a.scale,
                   "parallelism": "single GPU"},
        "pair_tests_per_s": round(head["pair_tests_per_s"], 1),
        "paths": paths,
        # the whole batch is one graph launch: its algorithmic bytes over the
        # graph's own duration (HIP events around the launch)
        "roofline": {"bound": "hbm", "kernel": "batch graph (one launch per step)",
                     "achieved": round(head["algorithmic_bytes"] / (head["graph_ms"] / 1e3) / 1e9,
                                       1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(head["algorithmic_bytes"] / (head["graph_ms"] / 1e3) / 1e9 /
                                   HBM_PEAK_GBS, 4),
                     "traffic": None,
                     "algorithmic_bytes_per_launch": head["algorithmic_bytes"],
                     "kernel_ms": round(head["graph_ms"], 4),
                     "step_frac": head["step_hbm_frac"]},
        "cpu_baseline": cpu,
    }
    if "fp64" in paths and "mixed" in paths:
        line["speedup_mixed_vs_fp64"] = round(paths["fp64"]["ms_per_step"] /
                                              paths["mixed"]["ms_per_step"], 3)
    return line


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}): the cross-match is "
              "measured at N=1; splitting the sky across GPUs is a design, not run here.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1611_08494_amd as c3x

    if a.config == "cfg4":
        line = batch_config(a, c3x, torch, np)
    else:
        line = single_config(a, c3x, torch, np, a.config)
    if a.config == "cfg5" and not a.no_extra:
        # the 10M x 10M full-sky workload beside the headline (its CPU
        # baseline included: the oracle runs it whole in seconds)
        torch.cuda.empty_cache()
        x = single_config(a, c3x, torch, np, "cfg2")
        line["extra"] = {"cfg2": {k: x[k] for k in ("value", "unit", "ms_per_step", "dtype",
                                                     "config", "pair_tests_per_s", "paths",
                                                     "roofline", "cpu_baseline",
                                                     "speedup_mixed_vs_fp64") if k in x}}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
