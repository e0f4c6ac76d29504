"""Benchmark of the MAG scan on one MI355X.

A step is one full scan of the workload's text, resident in HBM, through the
library's asynchronous entry point: filter (or, when the filter cannot prune,
the dense mode that tests every start position), candidate compaction, exact
verification and the sorted output, all on the GPU. The plan (pattern-set
preprocessing, including the learned selector's pick) is built once before
the timed region and timed separately.

Prints ONE JSON line: throughput in GB/s (1e9 bytes of text per second) of
the 1 GiB protein-like workload (100,000 patterns of 16 bytes) with the
learned selector's parameters (and with the fixed heuristic's, beside it),
the roofline of the dominant kernel (timed with HIP events recorded by the
library on the scan's own stream, in a second pass over the same steps so
that the events stay out of the per-step time), the CPU oracle timed on the
host's cores, and further measurements, each checked against the oracle:

* filter_mode: the same 1 GiB scan through the paper's filter kernel (the
  dense mode switched off), with the heuristic's parameters and with
  q = 5, k = 1, sigma' = 20, and each one's verifications per text byte;
* workloads.zipf256m: the 256 MiB Zipf scan (filter kernel) with its own
  roofline block, the fixed heuristic beside it, and MAG against SMAG (the
  text encoded first) with the same plan;
* workloads.dna1m: the 1 MiB DNA scan (launch-bound);
* learned_vs_fixed: 2,000 held-out pattern sets over 64 MiB texts,
  scan-kernel time with the heuristic's parameters and with the selector's
  pick, the two occurrence lists compared in full;
* batch: the 512-job workload (about 1.1 GB of text) as per-job scans with
  fixed parameters, and batched (one persistent launch, graph replay) with
  fixed and with learned parameters, every job's list checked against the
  oracle, with the roofline of the batched kernel.
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
# sources that determine each kernel's code; HBM traffic counted on an
# earlier build is reported only while these are unchanged
KERNEL_SOURCES = {
    "k_scan": ("scan.hip", "scan_common.hpp", "scan_args.hpp", "verify.hpp", "scan_dispatch.cpp"),
    "k_dense_slices": ("dense.hip", "dense.hpp", "verify.hpp", "scan_common.hpp", "mag_internal.hpp"),
    "k_dense": ("dense.hip", "dense.hpp", "verify.hpp", "scan_common.hpp", "mag_internal.hpp"),
    # the batch's two launches (filter jobs, dense jobs), measured together
    "k_batch": ("batch.hip", "batch.hpp", "batch.cpp", "dense.hpp", "verify.hpp", "scan_common.hpp"),
}
PMC_SUMMARY = "profiles/{kernel}_{workload}_pmc.md"
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
        return mag.Plan(patterns, **{k: v for k, v in best.items() if k != "sample_ms"})
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


def kernel_source_hash(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1405_5483_amd", "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def scan_kernel_name(info: dict) -> str:
    if info["dense"]:
        return "k_dense_slices" if info["dense_slices"] else "k_dense"
    return "k_scan"


def profiled_traffic(workload: str, info: dict, kernel: str):
    """HBM bytes per kernel launch from the committed rocprofv3 FETCH_SIZE and
    WRITE_SIZE summary of this kernel and workload, each scaled by what the
    counter reads for a copy of known size; None when the summary is missing,
    was taken with other parameters, or the kernel's sources have changed
    since."""
    path = os.path.join(ROOT, PMC_SUMMARY.format(kernel=kernel, workload=workload))
    if not os.path.exists(path):
        return None, "no counter summary"
    rec = None
    with open(path) as f:
        for line in f:
            if line.startswith("traffic-record: "):
                rec = json.loads(line[len("traffic-record: "):])
    if rec is None:
        return None, "summary has no traffic record"
    if info is not None and [rec["q"], rec["k"], rec["sigma_prime"], rec.get("map")] != \
            [info["q"], info["k"], info["sigma_prime"], _MAP_NAMES[info["map_kind"]]]:
        return None, "counters were taken with other parameters"
    if rec["src_sha256"] != kernel_source_hash(kernel):
        return None, "kernel changed since the counters were taken"
    return rec["traffic_bytes"], os.path.relpath(path, ROOT)


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
            "host_cores": os.cpu_count(), "kind": "oracle",
            "sample": f"first {sample.size} bytes of the same text, all {job.r} patterns, "
                      f"median of 3 runs of the C hashed matcher on {threads} threads "
                      f"({sec:.2f} s each; the host reports {os.cpu_count()} cores)",
            "value_1_thread": round(one.size / sec1 / 1e9, 4),
            "sample_1_thread": f"first {one.size} bytes, one run on one thread ({sec1:.2f} s)"}


def oracle_equal(occ_np, ref):
    import numpy as np
    pos, ids = ref
    return bool(pos.size == occ_np.shape[0] and np.array_equal(occ_np[:, 0].astype(np.uint64), pos)
                and np.array_equal(occ_np[:, 1].astype(np.uint32), ids))


def roofline_block(kernel: str, alg_bytes: int, kernel_ms: float, stream_gbps: float, traffic, src):
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "traffic_source": src,
            "kernel": kernel, "kernel_ms": round(kernel_ms, 5), "alg_bytes_per_launch": alg_bytes,
            "stream_read_GBps": round(stream_gbps, 1),
            "frac_of_stream_read": round(achieved / stream_gbps, 4) if stream_gbps else None}


def learned_vs_fixed(torch, mag, selector, sets: int, text_bytes: int, oracle_every: int = 50):
    """Held-out sets over 64 MiB texts: the scan kernel's time under the fixed
    heuristic and under the selector's pick; the two sorted occurrence lists
    are compared in full, and every `oracle_every`-th against the oracle."""
    import numpy as np
    import synth
    from oracle import match as om
    from paper_1405_5483_amd import train_selector as ts
    texts = ts.make_texts(synth, text_bytes, 6)
    dtexts = [torch.from_numpy(t).cuda() for t in texts]
    recipes = ts.set_recipes(sets, 6)
    psets = [ts.make_set(synth, texts, rec) for rec in recipes]
    picks = selector.picks(psets, threads=CPU_SHARE)
    cap = 1 << 20
    out_h = torch.empty((cap, 2), dtype=torch.int64, device="cuda")
    out_l = torch.empty((cap, 2), dtype=torch.int64, device="cuda")
    cnt_h = torch.empty(1, dtype=torch.int64, device="cuda")
    cnt_l = torch.empty(1, dtype=torch.int64, device="cuda")
    ratios, th, tl, same, compared, counts, checked, oracle_ok = [], 0.0, 0.0, 0, 0, 0, 0, 0
    for i, (rec, P, pk) in enumerate(zip(recipes, psets, picks)):
        hp, lp = mag.Plan(P), mag.Plan(P, **pk)
        h = scan_kernel_ms(mag, dtexts[rec[0]], hp, out_h, cnt_h)
        lt = scan_kernel_ms(mag, dtexts[rec[0]], lp, out_l, cnt_l)
        zh, zl = int(cnt_h.item()), int(cnt_l.item())
        counts += int(zh == zl)
        ok = zh == zl and zh <= cap and torch.equal(out_h[:zh], out_l[:zl])
        if zh <= cap:
            compared += 1
            same += int(ok)
        if i % oracle_every == 0 and zl <= cap:
            checked += 1
            ref = om.occ_hashed(texts[rec[0]], P, threads=CPU_SHARE)
            oracle_ok += int(ok and oracle_equal(out_l[:zl].cpu().numpy(), ref))
        ratios.append(h / lt)
        th += h
        tl += lt
        hp.close()
        lp.close()
        if (i + 1) % 250 == 0:
            log(f"learned vs fixed: {i + 1}/{sets} sets")
    geo = math.exp(sum(math.log(r) for r in ratios) / len(ratios))
    return {"sets": sets, "text_bytes": text_bytes, "held_out_seed": 6,
            "geomean_speedup": round(geo, 3), "win_rate": round(sum(r > 1 for r in ratios) / len(ratios), 3),
            "heuristic_total_ms": round(th, 3), "learned_total_ms": round(tl, 3),
            "total_speedup": round(th / tl, 3), "counts_equal": counts,
            "lists_compared": compared, "lists_equal": same,
            "oracle_checked": checked, "oracle_equal": oracle_ok,
            "timing": "scan-kernel device time, smaller of 2 runs; lists_equal counts the sets (of those "
                      f"with at most {cap} occurrences) whose two sorted occurrence lists are identical"}


def batch_section(torch, mag, selector, steps: int, stream_gbps: float, plans: str = "all"):
    """The 512-job workload: per-job scans with fixed parameters, and the
    batched kernel with fixed, learned and autotuned plans, every job's list
    checked against the oracle. plans="learned" runs only the batch of learned
    plans."""
    from oracle import match as om
    from synth import batch_jobs
    jobs = batch_jobs(512, workers=CPU_SHARE)
    total = sum(j.n for j in jobs)
    texts = [torch.from_numpy(j.text).cuda() for j in jobs]
    refs = [om.occ_hashed(j.text, j.patterns, threads=CPU_SHARE) for j in jobs]
    z = sum(r[0].size for r in refs)
    t = time.perf_counter()
    picks = selector.picks([j.patterns for j in jobs], threads=CPU_SHARE, batch=True)
    learned = [mag.Plan(j.patterns, **pk) for j, pk in zip(jobs, picks)]
    select_ms = (time.perf_counter() - t) * 1e3

    def batched(plans, words_per_lane=0):
        b = mag.Batch(plans, words_per_lane=words_per_lane)
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
        # the batched kernel alone: library events around it, eager runs
        mag.profile_read()
        mag.profile_enable(True)
        with torch.cuda.stream(stream):
            for _ in range(steps):
                b.run_async(out, offs, cnt, stream)
        stream.synchronize()
        mag.profile_enable(False)
        prof = mag.profile_read()
        del g
        b.close()
        return ms, exact, prof["scan_ms"] / max(prof["launches"], 1)

    bl_ms, bl_exact, bl_k = batched(learned)
    traffic, src = profiled_traffic("batch512", None, "k_batch")
    roof = roofline_block("k_batch", total, bl_k, stream_gbps, traffic, src)
    roof["launches"] = "k_batch (filter jobs) then k_batch_dense (dense jobs)"
    if plans == "learned":
        return {"jobs": 512, "text_bytes": total, "occurrences": z,
                "batched_learned_ms": round(bl_ms, 3), "k_batch_learned_ms": round(bl_k, 4),
                "batched_learned_GBps": round(total / (bl_ms * 1e-3) / 1e9, 2),
                "roofline": roof, "bit_exact": bool(bl_exact)}

    # per-job scans with fixed parameters, one after another
    fixed = [mag.Plan(j.patterns) for j in jobs]
    torch.cuda.synchronize()
    per_job = []
    for rep in range(2):
        t = time.perf_counter()
        for tx, p in zip(texts, fixed):
            mag.scan(tx, p)
        torch.cuda.synchronize()
        per_job.append((time.perf_counter() - t) * 1e3)
    per_job_ms = min(per_job)
    bf_ms, bf_exact, bf_k = batched(fixed)
    # autotuned: one tuned pick per job class, then the batched kernel's words
    # per lane, timed on the batch itself (host work before the timed region)
    t = time.perf_counter()
    tuned_kw, tuned_wpl = mag.autotune_batch([j.patterns for j in jobs], texts, sample_bytes=1 << 20,
                                             max_candidates=8)
    tuned = [mag.Plan(j.patterns, **kw) for j, kw in zip(jobs, tuned_kw)]
    tune_s = time.perf_counter() - t
    ba_ms, ba_exact, ba_k = batched(tuned, tuned_wpl)
    return {"jobs": 512, "text_bytes": total, "occurrences": z,
            "per_job_fixed_ms": round(per_job_ms, 3),
            "batched_fixed_ms": round(bf_ms, 3), "batched_learned_ms": round(bl_ms, 3),
            "batched_autotuned_ms": round(ba_ms, 3), "autotuned_words_per_lane": tuned_wpl,
            "autotune_s": round(tune_s, 1), "autotuned_bit_exact": bool(ba_exact),
            "autotuned_dense_jobs": sum(kw["mode"] == "dense" for kw in tuned_kw),
            "speedup_autotuned_vs_fixed_batched": round(bf_ms / ba_ms, 3),
            "batched_learned_GBps": round(total / (bl_ms * 1e-3) / 1e9, 2),
            "per_job_fixed_GBps": round(total / (per_job_ms * 1e-3) / 1e9, 2),
            "speedup_vs_per_job_fixed": round(per_job_ms / bl_ms, 2),
            "speedup_learned_vs_fixed_batched": round(bf_ms / bl_ms, 3),
            "k_batch_fixed_ms": round(bf_k, 4), "k_batch_learned_ms": round(bl_k, 4),
            "k_batch_autotuned_ms": round(ba_k, 4),
            "roofline": roof,
            "selector_ms": round(select_ms, 1),
            "bit_exact": bool(bf_exact and bl_exact and ba_exact),
            "timing": "graph replays of bind-time launches; k_batch (the filter and dense launches together) "
                      "from library events on eager runs; "
                      "per-job scans wall clock"}


def compare_section(torch, mag, job, text, ref, z, out, cnt, steps: int, warmup: int):
    """The headline workload with the fixed heuristic's parameters, and
    through the paper's filter kernel (the dense mode switched off) with the
    heuristic's parameters and with q = 5, k = 1, sigma' = 20; each checked
    against the oracle."""
    n = job.n
    # the same workload with the fixed heuristic's parameters
    fixed_plan = mag.Plan(job.patterns)
    finfo = fixed_plan.info()
    fixed_ms, fprof = time_scans(torch, mag, text, fixed_plan, out, cnt, steps, warmup)
    fz = int(cnt.item())
    fixed_exact = fz == z and (ref is None or oracle_equal(out[:fz].cpu().numpy(), ref))
    fixed = {"GBps": round(n / (fixed_ms * 1e-3) / 1e9, 3), "ms_per_step": round(fixed_ms, 5),
             "scan_kernel_ms": round(fprof["scan_ms"] / max(fprof["launches"], 1), 5),
             "q": finfo["q"], "k": finfo["k"], "sigma_prime": finfo["sigma_prime"],
             "kernel": scan_kernel_name(finfo), "bit_exact": fixed_exact}
    fixed_plan.close()

    # the paper's own filter on the same scan (no dense mode): the
    # heuristic's parameters, and sigma' = sigma = 20 with q = 5
    filter_mode = {}
    for label, kw in (("heuristic", {}), ("q5_k1_sigma20", dict(q=5, k=1, sigma_prime=20))):
        fp = mag.Plan(job.patterns, mode="filter", **kw)
        fi = fp.info()
        _, fst = mag.scan(text, fp, stats=True)
        f_ms, f_prof = time_scans(torch, mag, text, fp, out, cnt, max(3, steps // 4), 1)
        f_z = int(cnt.item())
        filter_mode[label] = {
            "GBps": round(n / (f_ms * 1e-3) / 1e9, 3), "ms_per_step": round(f_ms, 5),
            "scan_kernel_ms": round(f_prof["scan_ms"] / max(f_prof["launches"], 1), 5),
            "q": fi["q"], "k": fi["k"], "sigma_prime": fi["sigma_prime"],
            "table_bytes": fi["table_bytes"], "kernel": scan_kernel_name(fi),
            "verifications_per_byte": round(fst["verifications"] / n, 5),
            "bit_exact": f_z == z and (ref is None or oracle_equal(out[:f_z].cpu().numpy(), ref))}
        log(f"filter mode {label}: {filter_mode[label]}")
        fp.close()
    return fixed, filter_mode


def workload_section(torch, mag, selector, name: str, steps: int, warmup: int, stream_gbps,
                     smag: bool = False):
    """A single-job workload with the selector's pick (kernel roofline) and
    the fixed heuristic, both checked against the oracle in full."""
    from oracle import match as om
    from synth import workload
    job = workload(name)
    text = torch.from_numpy(job.text).cuda()
    ref = om.occ_hashed(job.text, job.patterns, threads=CPU_SHARE)
    cap = max(1024, 2 * ref[0].size)
    out = torch.empty((cap, 2), dtype=torch.int64, device="cuda")
    cnt = torch.empty(1, dtype=torch.int64, device="cuda")
    res = {"text_bytes": job.n, "r": job.r, "m": job.m}
    for sel in ("learned", "heuristic"):
        plan = plan_for(mag, job.patterns, sel, text, selector)
        info = plan.info()
        exact = oracle_equal(mag.scan(text, plan, out_cap=cap).cpu().numpy(), ref)
        ms, prof = time_scans(torch, mag, text, plan, out, cnt, steps, warmup)
        kms = prof["scan_ms"] / max(prof["launches"], 1)
        kernel = scan_kernel_name(info)
        r = {"GBps": round(job.n / (ms * 1e-3) / 1e9, 2), "ms_per_step": round(ms, 5),
             "scan_kernel_ms": round(kms, 5), "q": info["q"], "k": info["k"],
             "sigma_prime": info["sigma_prime"], "map": _MAP_NAMES[info["map_kind"]],
             "dense": bool(info["dense"]), "kernel": kernel, "bit_exact": exact}
        if sel == "learned":
            traffic, src = profiled_traffic(name, info, kernel)
            r["roofline"] = roofline_block(kernel, job.n, kms, stream_gbps, traffic, src)
            if smag and not info["dense"]:
                sm = mag.Plan(job.patterns, q=info["q"], k=info["k"], sigma_prime=info["sigma_prime"],
                              map_kind=_MAP_NAMES[info["map_kind"]], encode=True, mode="filter")
                sms, _ = time_scans(torch, mag, text, sm, out, cnt, steps, warmup)
                sexact = int(cnt.item()) == ref[0].size and oracle_equal(
                    out[:ref[0].size].cpu().numpy(), ref)
                res["mag_vs_smag"] = {"smag_GBps": round(job.n / (sms * 1e-3) / 1e9, 2),
                                      "smag_ms_per_step": round(sms, 5),
                                      "mag_GBps": r["GBps"], "mag_over_smag": round(sms / ms, 3),
                                      "bit_exact": sexact}
                sm.close()
        res[sel] = r
        plan.close()
    return res


_MAP_NAMES = {0: "greedy", 1: "rank", 2: "bits", 3: "qgram"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="prot1g")
    ap.add_argument("--select", default="learned",
                    help="learned | heuristic | qgram | autotune | explicit:q,k,sigma'")
    ap.add_argument("--eval-sets", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the learned-vs-fixed, batch and other-workload sections")
    ap.add_argument("--only-batch", action="store_true",
                    help="skip the headline timing; run the batch section only (profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run three 256 MiB device copies (counter calibration)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the fixed-parameter and filter-mode runs of the headline workload "
                         "(profiling: only the selected plan's kernels run)")
    ap.add_argument("--batch-plans", choices=("all", "learned"), default="all",
                    help="with --only-batch: 'learned' runs only the batch of learned plans "
                         "(profiling: every batched launch is the one the roofline reports)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(a multi-GPU scan would shard the text by range, each shard overlapping the next by m - 1 bytes)",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1405_5483_amd as mag
    from synth import WORKLOADS, workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    selector = mag.Selector.load()
    if args.only_batch:
        log("batched workload (512 jobs) only")
        probe = torch.zeros(1 << 28, dtype=torch.uint8, device="cuda")
        sgb = stream_read_gbps(torch, mag, probe)
        del probe
        if args.copy_calibration:
            log("copy calibration: 3 x 256 MiB")
            copy_calibration(torch)
        b = batch_section(torch, mag, selector, args.steps, sgb, plans=args.batch_plans)
        print(json.dumps({"batch": b}), flush=True)
        return 0
    log(f"generating workload {args.workload}")
    job = workload(args.workload)
    n = job.n
    text = torch.from_numpy(job.text).cuda()
    torch.cuda.synchronize()
    t = time.perf_counter()
    plan = plan_for(mag, job.patterns, args.select, text, selector)
    plan_ms = (time.perf_counter() - t) * 1e3
    info = plan.info()
    kernel = scan_kernel_name(info)
    log(f"plan q={info['q']} k={info['k']} sigma'={info['sigma_prime']} "
        f"map={_MAP_NAMES[info['map_kind']]} W={info['W']} dense={info['dense']} "
        f"slices={info['dense_slices']} kernel={kernel} ({plan_ms:.1f} ms)")

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

    stream_gbps = stream_read_gbps(torch, mag, text)
    log(f"streaming-read reference: {stream_gbps:.0f} GB/s")
    traffic, traffic_src = profiled_traffic(args.workload, info, kernel)
    log(f"HBM traffic per launch: {traffic} ({traffic_src})")
    if args.copy_calibration:
        log("copy calibration: 3 x 256 MiB")
        copy_calibration(torch)

    fixed, filter_mode = None, None
    if not args.no_compare:
        fixed, filter_mode = compare_section(torch, mag, job, text, ref, z, out, cnt, args.steps,
                                             args.warmup)

    extras = {}
    if not args.no_extras:
        extras["workloads"] = {}
        for name, steps in (("zipf256m", args.steps), ("dna1m", args.steps)):
            log(f"workload {name}")
            extras["workloads"][name] = workload_section(torch, mag, selector, name, steps, args.warmup,
                                                         stream_gbps, smag=(name == "zipf256m"))
            log(f"{name}: {extras['workloads'][name]}")
        log(f"learned vs fixed on {args.eval_sets} held-out sets")
        extras["learned_vs_fixed"] = learned_vs_fixed(torch, mag, selector, args.eval_sets, 64 << 20)
        log(f"learned vs fixed: {extras['learned_vs_fixed']}")
        log("batched workload (512 jobs)")
        extras["batch"] = batch_section(torch, mag, selector, 10, stream_gbps)
        log(f"batch: {extras['batch']}")

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
                   "map": _MAP_NAMES[info["map_kind"]], "dense": bool(info["dense"]),
                   "dense_slices": info["dense_slices"], "parallelism": "single GPU"},
        "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBS, 2),
        "roofline": roofline_block(kernel, n, scan_ms, stream_gbps, traffic, traffic_src),
        "fixed_params": fixed,
        "filter_mode": filter_mode,
        "finish_ms": round(finish_ms, 5),
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
