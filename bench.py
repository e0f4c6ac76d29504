"""Benchmark of the MAG scan on one MI355X.

A step is one full scan of the workload's text, resident in HBM, through the
library's asynchronous entry point: filter, candidate compaction, exact
verification and the sorted output, all on the GPU. The plan (pattern-set
preprocessing, including the learned selector's pick) is built once before
the timed region and timed separately.

Prints ONE JSON line: throughput in GB/s (1e9 bytes of text per second) of
the 256 MiB Zipf workload with the learned selector's parameters (and with
the fixed heuristic's, beside it), the roofline of the dominant kernel (the
scan kernel, timed with HIP events recorded by the library on the scan's own
stream, in a second pass over the same steps so that the events stay out of
the per-step time), the CPU oracle timed on the host's cores, and further
measurements:

* mag_vs_smag: the same scan with the text encoded first (SMAG);
* learned_vs_fixed: held-out pattern sets over 64 MiB texts, scan-kernel time
  with the heuristic's parameters and with the selector's pick;
* batch: the 512-job workload (about 1.1 GB of text) as per-job scans with
  fixed parameters, and batched (one persistent launch, graph replay) with
  fixed and with learned parameters, every job checked against the oracle;
* workloads: the 1 MiB DNA and the 1 GiB protein-like scans, each with the
  heuristic's, the selector's and the q-gram map heuristic's plan.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# sources that determine the scan kernel's code; HBM traffic counted on an
# earlier build is reported only while these are unchanged
SCAN_SOURCES = ("scan.hip", "scan_common.hpp", "scan_args.hpp", "verify.hpp", "scan_dispatch.cpp")
PMC_SUMMARY = "profiles/k_scan_{workload}_pmc.md"
CPU_SHARE = 16          # host threads one GPU's share of the box may use
SAMPLE_BYTES = 16 << 20 # text prefix the autotuner times candidates on


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def plan_for(mag, patterns, select: str, text=None, selector=None):
    if select == "heuristic":
        return mag.Plan(patterns)
    if select == "learned":
        return mag.Plan(patterns, **selector.pick(patterns))
    if select == "autotune":
        sample = text[: min(text.numel(), SAMPLE_BYTES)]
        best = mag.autotune(patterns, sample)
        log(f"autotune picked {best}")
        return mag.Plan(patterns, q=best["q"], k=best["k"], sigma_prime=best["sigma_prime"],
                        map_kind=best["map_kind"])
    if select == "qgram":
        return mag.Plan(patterns, map_kind="qgram")
    if select.startswith("explicit:"):
        q, k, sp = (int(v) for v in select.split(":")[1].split(","))
        return mag.Plan(patterns, q=q, k=k, sigma_prime=sp)
    raise ValueError(f"unknown selection {select!r}")


def time_scans(torch, mag, text, plan, out, cnt, steps: int, warmup: int):
    """(ms per step, summed library profile) over `steps` scans.

    The steps run twice: first with nothing but the scans on the stream
    (the per-step time), then with the library's profiling events around
    each scan's kernels (the per-kernel durations). The events sit between
    kernels on the stream and add about 10 us per step of their own, so the
    step time is not taken from the instrumented pass."""
    for _ in range(warmup):
        mag.scan_async(text, plan, out, cnt)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        mag.scan_async(text, plan, out, cnt)
    t1.record()
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    mag.profile_read()                       # drop anything recorded before
    mag.profile_enable(True)
    for _ in range(steps):
        mag.scan_async(text, plan, out, cnt)
    torch.cuda.synchronize()
    mag.profile_enable(False)
    prof = mag.profile_read()
    return ms, prof


def scan_kernel_ms(mag, text, plan, out, cnt, repeats=2):
    best = math.inf
    mag.profile_enable(True)
    for _ in range(repeats):
        mag.profile_read()
        mag.scan_async(text, plan, out, cnt)
        best = min(best, mag.profile_read()["scan_ms"])
    mag.profile_enable(False)
    return best


def scan_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in SCAN_SOURCES:
        with open(os.path.join(ROOT, "paper_1405_5483_amd", "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def profiled_traffic(workload: str, info: dict):
    """HBM bytes per scan launch from the committed rocprofv3 FETCH_SIZE and
    WRITE_SIZE summary of this workload, each scaled by what the counter reads
    for a copy of known size; None when the summary is missing, was taken with
    other parameters, or the scan kernel's sources have changed since."""
    path = os.path.join(ROOT, PMC_SUMMARY.format(workload=workload))
    if not os.path.exists(path):
        return None, "no counter summary"
    rec = None
    with open(path) as f:
        for line in f:
            if line.startswith("traffic-record: "):
                rec = json.loads(line[len("traffic-record: "):])
    if rec is None:
        return None, "summary has no traffic record"
    if [rec["q"], rec["k"], rec["sigma_prime"], rec.get("map")] != \
            [info["q"], info["k"], info["sigma_prime"], _MAP_NAMES[info["map_kind"]]]:
        return None, "counters were taken with other parameters"
    if rec["src_sha256"] != scan_source_hash():
        return None, "scan kernel changed since the counters were taken"
    return rec["traffic_bytes"], path


def copy_calibration(torch) -> None:
    """Three device-to-device copies of 256 MiB: the reference kernel whose
    FETCH_SIZE and WRITE_SIZE readings calibrate the counters."""
    a = torch.empty(1 << 28, dtype=torch.uint8, device="cuda")
    b = torch.empty(1 << 28, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    assert bool((b[:: 1 << 20] == 1).all())
    del a, b


def stream_read_gbps(torch, mag, text, reps: int = 20) -> float:
    """Read bandwidth of the library's plain streaming-read kernel over the
    same resident text: the achievable ceiling for a kernel that reads it
    once."""
    sink = mag.stream_read(text)
    for _ in range(3):
        mag.stream_read(text, sink)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        mag.stream_read(text, sink)
    t1.record()
    torch.cuda.synchronize()
    return text.numel() / (t0.elapsed_time(t1) / reps * 1e-3) / 1e9


def cpu_baseline(job, threads: int, max_bytes: int):
    from oracle import match as om
    sample = job.text[:max_bytes]
    runs = []
    for _ in range(3):
        t = time.perf_counter()
        om.occ_hashed(sample, job.patterns, threads=threads)
        runs.append(time.perf_counter() - t)
    sec = statistics.median(runs)
    # one thread on a quarter of the sample
    one = job.text[: max_bytes // 4]
    t = time.perf_counter()
    om.occ_hashed(one, job.patterns, threads=1)
    sec1 = time.perf_counter() - t
    return {"value": round(sample.size / sec / 1e9, 4), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {sample.size} bytes of the same text, all {job.r} patterns, "
                      f"median of 3 runs of the C hashed matcher ({sec:.2f} s each)",
            "value_1_thread": round(one.size / sec1 / 1e9, 4),
            "sample_1_thread": f"first {one.size} bytes, one run on one thread ({sec1:.2f} s)"}


def oracle_equal(occ_np, ref):
    import numpy as np
    pos, ids = ref
    return bool(pos.size == occ_np.shape[0] and np.array_equal(occ_np[:, 0].astype(np.uint64), pos)
                and np.array_equal(occ_np[:, 1].astype(np.uint32), ids))


def learned_vs_fixed(torch, mag, selector, sets: int, text_bytes: int):
    import synth
    from paper_1405_5483_amd import train_selector as ts
    texts = ts.make_texts(synth, text_bytes, 6)
    dtexts = [torch.from_numpy(t).cuda() for t in texts]
    recipes = ts.set_recipes(sets, 6)
    psets = [ts.make_set(synth, texts, rec) for rec in recipes]
    picks = selector.picks(psets, threads=CPU_SHARE)
    out = torch.empty((8192, 2), dtype=torch.int64, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    ratios, th, tl, same = [], 0.0, 0.0, 0
    for rec, P, pk in zip(recipes, psets, picks):
        hp, lp = mag.Plan(P), mag.Plan(P, **pk)
        h = scan_kernel_ms(mag, dtexts[rec[0]], hp, out, cnt)
        zh = int(cnt.item())
        lt = scan_kernel_ms(mag, dtexts[rec[0]], lp, out, cnt)
        same += int(zh == int(cnt.item()))
        ratios.append(h / lt)
        th += h
        tl += lt
        hp.close()
        lp.close()
    geo = math.exp(sum(math.log(r) for r in ratios) / len(ratios))
    return {"sets": sets, "text_bytes": text_bytes, "held_out_seed": 6,
            "geomean_speedup": round(geo, 3), "win_rate": round(sum(r > 1 for r in ratios) / len(ratios), 3),
            "heuristic_total_ms": round(th, 3), "learned_total_ms": round(tl, 3),
            "total_speedup": round(th / tl, 3), "same_count": same,
            "timing": "scan-kernel device time, smaller of 2 runs"}


def batch_section(torch, mag, selector, steps: int):
    import numpy as np
    from oracle import match as om
    from synth import batch_jobs
    jobs = batch_jobs(512, workers=CPU_SHARE)
    total = sum(j.n for j in jobs)
    texts = [torch.from_numpy(j.text).cuda() for j in jobs]
    refs = [om.occ_hashed(j.text, j.patterns, threads=CPU_SHARE) for j in jobs]
    z = sum(r[0].size for r in refs)
    fixed = [mag.Plan(j.patterns) for j in jobs]
    t = time.perf_counter()
    picks = selector.picks([j.patterns for j in jobs], threads=CPU_SHARE)
    learned = [mag.Plan(j.patterns, **pk) for j, pk in zip(jobs, picks)]
    select_ms = (time.perf_counter() - t) * 1e3

    # per-job scans with fixed parameters, one after another
    torch.cuda.synchronize()
    per_job = []
    for rep in range(2):
        t = time.perf_counter()
        for tx, p in zip(texts, fixed):
            mag.scan(tx, p)
        torch.cuda.synchronize()
        per_job.append((time.perf_counter() - t) * 1e3)
    per_job_ms = min(per_job)

    def batched(plans):
        b = mag.Batch(plans)
        stream = torch.cuda.Stream()
        b.bind(texts, z + 4096, stream)
        out = torch.empty((z + 4096, 2), dtype=torch.int64, device="cuda")
        offs = torch.empty(513, dtype=torch.int64, device="cuda")
        cnt = torch.empty(1, dtype=torch.int64, device="cuda")
        with torch.cuda.stream(stream):
            b.run_async(out, offs, cnt, stream)
        stream.synchronize()
        off = offs.cpu().tolist()
        o = out.cpu().numpy()
        exact = all(oracle_equal(o[off[j]:off[j + 1]], refs[j]) for j in range(512))
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            b.run_async(out, offs, cnt, torch.cuda.current_stream())
        for _ in range(2):
            g.replay()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            g.replay()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        exact = exact and int(cnt.item()) == z
        del g
        b.close()
        return ms, exact

    bf_ms, bf_exact = batched(fixed)
    bl_ms, bl_exact = batched(learned)
    return {"jobs": 512, "text_bytes": total, "occurrences": z,
            "per_job_fixed_ms": round(per_job_ms, 3),
            "batched_fixed_ms": round(bf_ms, 3), "batched_learned_ms": round(bl_ms, 3),
            "batched_learned_GBps": round(total / (bl_ms * 1e-3) / 1e9, 2),
            "per_job_fixed_GBps": round(total / (per_job_ms * 1e-3) / 1e9, 2),
            "speedup_vs_per_job_fixed": round(per_job_ms / bl_ms, 2),
            "speedup_learned_vs_fixed_batched": round(bf_ms / bl_ms, 3),
            "selector_ms": round(select_ms, 1),
            "bit_exact": bool(bf_exact and bl_exact),
            "timing": "graph replays of bind-time launches; per-job scans wall clock"}


def mag_vs_smag(torch, mag, job, text, plan_for, select, selector, out, cnt, steps, warmup, mag_gbps):
    """The timed workload with the same parameters, but each scan first
    encodes the whole text (SMAG, Section 3.2): the paper reports the
    on-the-fly variant (MAG) as generally faster."""
    plan = plan_for(mag, job.patterns, select, text, selector)
    info = plan.info()
    smag = mag.Plan(job.patterns, q=info["q"], k=info["k"], sigma_prime=info["sigma_prime"],
                    map_kind={0: "greedy", 1: "rank", 2: "bits", 3: "qgram"}[info["map_kind"]],
                    encode=True, mode="filter")
    plan.close()
    ms, prof = time_scans(torch, mag, text, smag, out, cnt, steps, warmup)
    z = int(cnt.item())
    smag.close()
    gbps = job.n / (ms * 1e-3) / 1e9
    return {"smag_GBps": round(gbps, 2), "smag_ms_per_step": round(ms, 5),
            "smag_kernels_ms": round(prof["scan_ms"] / max(prof["launches"], 1), 5),
            "mag_GBps": round(mag_gbps, 2), "mag_over_smag": round(mag_gbps / gbps, 3),
            "occurrences": z}


def single_workload(torch, mag, selector, name: str, steps: int):
    import numpy as np
    from oracle import match as om
    from synth import workload
    job = workload(name)
    text = torch.from_numpy(job.text).cuda()
    ref = om.occ_hashed(job.text, job.patterns, threads=CPU_SHARE)
    res = {"text_bytes": job.n, "r": job.r, "m": job.m}
    for sel in ("heuristic", "learned", "qgram"):
        plan = plan_for(mag, job.patterns, sel, text, selector)
        info = plan.info()
        occ = mag.scan(text, plan, out_cap=ref[0].size + 1024)
        exact = oracle_equal(occ.cpu().numpy(), ref)
        out = torch.empty((ref[0].size + 1024, 2), dtype=torch.int64, device="cuda")
        cnt = torch.empty(1, dtype=torch.int64, device="cuda")
        ms, prof = time_scans(torch, mag, text, plan, out, cnt, steps, 2)
        res[sel] = {"GBps": round(job.n / (ms * 1e-3) / 1e9, 2), "ms_per_step": round(ms, 4),
                    "scan_kernel_ms": round(prof["scan_ms"] / max(prof["launches"], 1), 4),
                    "q": info["q"], "k": info["k"], "sigma_prime": info["sigma_prime"],
                    "map": _MAP_NAMES[info["map_kind"]], "dense": bool(info["dense"]),
                    "bit_exact": exact}
        plan.close()
    return res


_MAP_NAMES = {0: "greedy", 1: "rank", 2: "bits", 3: "qgram"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="zipf256m")
    ap.add_argument("--select", default="learned",
                    help="learned | heuristic | qgram | autotune | explicit:q,k,sigma'")
    ap.add_argument("--eval-sets", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the learned-vs-fixed, batch and other-workload sections")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run three 256 MiB device copies (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the scan shards by text range with no exchange; see the design notes)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1405_5483_amd as mag
    from synth import WORKLOADS, workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    selector = mag.Selector.load()
    log(f"generating workload {args.workload}")
    job = workload(args.workload)
    n = job.n
    text = torch.from_numpy(job.text).cuda()
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan = plan_for(mag, job.patterns, args.select, text, selector)
    plan_ms = (time.perf_counter() - t) * 1e3
    info = plan.info()
    log(f"plan q={info['q']} k={info['k']} sigma'={info['sigma_prime']} "
        f"map={_MAP_NAMES[info['map_kind']]} W={info['W']} "
        f"table={info['table_bytes']} B ({plan_ms:.1f} ms)")

    # exact occurrence list once, with counters, and verified against the oracle
    occ, st = mag.scan(text, plan, stats=True)
    z = occ.shape[0]
    verified = None
    ref = None
    if not args.no_verify:
        from oracle import match as om
        ref = om.occ_hashed(job.text, job.patterns, threads=min(os.cpu_count() or 1, CPU_SHARE))
        verified = oracle_equal(occ.cpu().numpy(), ref)
        log(f"bit-exact vs oracle: {verified} ({z} occurrences)")
        if not verified:
            return 1
    cap = max(1024, 2 * z)
    out = torch.empty((cap, 2), dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")

    log(f"timing {args.steps} steps after {args.warmup} warm-up steps")
    ms, prof = time_scans(torch, mag, text, plan, out, cnt, args.steps, args.warmup)
    assert int(cnt.item()) == z
    value = n / (ms * 1e-3) / 1e9
    scan_ms = prof["scan_ms"] / max(prof["launches"], 1)
    finish_ms = prof["finish_ms"] / max(prof["launches"], 1)
    alg_bytes = n                         # the filter kernel reads the text once
    achieved = alg_bytes / (scan_ms * 1e-3) / 1e9

    stream_gbps = stream_read_gbps(torch, mag, text)
    log(f"streaming-read reference: {stream_gbps:.0f} GB/s")
    traffic, traffic_src = profiled_traffic(args.workload, info)
    log(f"HBM traffic per launch: {traffic} ({traffic_src})")
    if args.copy_calibration:
        log("copy calibration: 3 x 256 MiB")
        copy_calibration(torch)

    # the same workload with the fixed heuristic's parameters
    fixed_plan = mag.Plan(job.patterns)
    finfo = fixed_plan.info()
    fixed_ms, fprof = time_scans(torch, mag, text, fixed_plan, out, cnt, args.steps, args.warmup)
    fixed_exact = int(cnt.item()) == z
    fixed = {"GBps": round(n / (fixed_ms * 1e-3) / 1e9, 3), "ms_per_step": round(fixed_ms, 5),
             "q": finfo["q"], "k": finfo["k"], "sigma_prime": finfo["sigma_prime"],
             "same_count": fixed_exact}
    fixed_plan.close()

    extras = {}
    if not args.no_extras:
        log("MAG vs SMAG (text encoded before the search) with the same plan")
        extras["mag_vs_smag"] = mag_vs_smag(torch, mag, job, text, plan_for, args.select, selector,
                                            out, cnt, args.steps, args.warmup, value)
        log(f"mag_vs_smag: {extras['mag_vs_smag']}")
        log(f"learned vs fixed on {args.eval_sets} held-out sets")
        extras["learned_vs_fixed"] = learned_vs_fixed(torch, mag, selector, args.eval_sets, 64 << 20)
        log(f"learned vs fixed: {extras['learned_vs_fixed']}")
        log("batched workload (512 jobs)")
        extras["batch"] = batch_section(torch, mag, selector, 10)
        log(f"batch: {extras['batch']}")
        extras["workloads"] = {}
        for name in ("dna1m", "prot1g"):
            log(f"workload {name}")
            extras["workloads"][name] = single_workload(torch, mag, selector, name,
                                                        args.steps if name == "dna1m" else 5)
            log(f"{name}: {extras['workloads'][name]}")

    cpu = None
    if not args.no_cpu_baseline:
        threads = min(os.cpu_count() or 1, CPU_SHARE)
        log(f"timing the CPU oracle on {threads} threads")
        cpu = cpu_baseline(job, threads, max_bytes=n)

    w = WORKLOADS[args.workload]
    line = {
        "metric": "text GB/s scanned (bit-exact) and % HBM peak; learned vs fixed params",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": args.workload, "text_bytes": n, "sigma": w["sigma"],
                   "dist": w["dist"], "r": job.r, "m": job.m, "select": args.select,
                   "q": info["q"], "k": info["k"], "sigma_prime": info["sigma_prime"],
                   "map": _MAP_NAMES[info["map_kind"]], "parallelism": "single GPU"},
        "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBS, 2),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_source": traffic_src,
                     "kernel": "k_scan", "kernel_ms": round(scan_ms, 5),
                     "alg_bytes_per_launch": alg_bytes,
                     "stream_read_GBps": round(stream_gbps, 1),
                     "frac_of_stream_read": round(achieved / stream_gbps, 4)},
        "fixed_params": fixed,
        "finish_kernel_ms": round(finish_ms, 5),
        "plan_ms": round(plan_ms, 3),
        "occurrences": z,
        "bit_exact": verified,
        "counters": st,
        **extras,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
