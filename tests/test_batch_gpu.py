"""Parity of batched scans (many jobs in one persistent launch) against the
oracle (GPU).

Each job's records, cut out of the shared output by the per-job offsets, must
equal the oracle's occurrence list of that job's text and pattern set,
element by element. The cases cover jobs of every kind in one batch (empty
texts, texts shorter than m, empty pattern sets, a plan shared by two jobs,
texts at unaligned addresses, mask tables too large for LDS), output
overflow, the device-wide sort, replays of a captured graph, rebinding, and
the full 512-job workload.
"""

import numpy as np
import pytest

from oracle import match as om
from synth import Job, batch_jobs, batch_recipes, gen_patterns, gen_text, make_job

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch


@pytest.fixture(scope="module")
def mag():
    import paper_1405_5483_amd as m
    return m


def _upload(torch, texts, offsets=None):
    """Device copies of the texts, job j at byte offset offsets[j] of its own
    buffer (so its address has that alignment)."""
    out = []
    for j, t in enumerate(texts):
        off = offsets[j] if offsets else 0
        buf = torch.empty(t.size + off + 16, dtype=torch.uint8, device="cuda")
        view = buf[off:off + t.size]
        if t.size:
            view.copy_(torch.from_numpy(t))
        out.append(view)
    return out


def _check_jobs(results, jobs):
    for j, (res, job) in enumerate(zip(results, jobs)):
        occ = res.cpu().numpy()
        rpos, rids = om.occ_hashed(job.text, job.patterns)
        assert occ.shape[0] == rpos.size, (j, occ.shape[0], rpos.size, job.recipe)
        assert np.array_equal(occ[:, 0].astype(np.uint64), rpos), (j, job.recipe)
        assert np.array_equal(occ[:, 1].astype(np.uint32), rids), (j, job.recipe)


def _small_jobs(count, seed, n_log2=(10.0, 17.0), r_log10=(1.0, 3.0)):
    return [make_job(rec["n"], rec["sigma"], rec["dist"], rec["r"], rec["m"], rec["frac"], ss)
            for rec, ss in batch_recipes(count, seed, n_log2, r_log10)]


def test_batch_mixed_jobs(torch_cuda, mag):
    torch = torch_cuda
    jobs = _small_jobs(24, seed=101)
    # special jobs
    jobs.append(make_job(0, 4, "uniform", 10, 8, 0.5, 7))                  # empty text
    jobs.append(make_job(5, 4, "uniform", 10, 8, 0.5, 8))                  # n < m
    t = gen_text(20_000, 20, rng=9)
    jobs.append(type(jobs[0])(t, np.zeros((0, 16), np.uint8), {"r": 0}))   # no patterns
    t = gen_text(300_000, 20, rng=10)
    p = gen_patterns(t, 400, 16, 300, 20, rng=11)
    jobs.append(type(jobs[0])(t, p, {"big_table": True}))                  # table read from L2
    # every third job scans densely
    plans = [mag.Plan(j.patterns, mode="dense" if i % 3 == 2 else "filter")
             for i, j in enumerate(jobs[:-1])]
    plans.append(mag.Plan(jobs[-1].patterns, q=4, k=1, sigma_prime=20, mode="filter"))
    assert plans[-1].info()["table_bytes"] > 64 * 1024
    # a plan shared by two jobs (same patterns, another text)
    t2 = gen_text(70_001, jobs[3].recipe["sigma"], rng=12)
    jobs.append(type(jobs[0])(t2, jobs[3].patterns, {"shared": True}))
    plans.append(plans[3])
    offsets = [(7 * j) % 16 for j in range(len(jobs))]
    texts = _upload(torch, [j.text for j in jobs], offsets)
    b = mag.Batch(plans)
    b.bind(texts, 1 << 16)
    _check_jobs(b.run(), jobs)
    # a second run of the same binding gives the same lists
    _check_jobs(b.run(), jobs)
    b.close()


def test_batch_overflow_reports_exact_count(torch_cuda, mag):
    torch = torch_cuda
    jobs = _small_jobs(6, seed=202)
    plans = [mag.Plan(j.patterns) for j in jobs]
    texts = _upload(torch, [j.text for j in jobs])
    total = sum(om.occ_hashed(j.text, j.patterns)[0].size for j in jobs)
    assert total > 16
    b = mag.Batch(plans)
    b.bind(texts, 16)
    out = torch.full((16, 2), -7, dtype=torch.int64, device="cuda")
    offsets = torch.empty(len(jobs) + 1, dtype=torch.int64, device="cuda")
    count = torch.empty(1, dtype=torch.int64, device="cuda")
    b.run_async(out, offsets, count)
    torch.cuda.synchronize()
    assert int(count.item()) == total
    assert int(offsets[-1].item()) == total
    # run() rebinds with the exact capacity
    _check_jobs(b.run(), jobs)
    b.close()


def test_batch_device_wide_sort(torch_cuda, mag):
    """Outputs above the finishing kernel's in-LDS limit go through the
    device-wide radix sort."""
    torch = torch_cuda
    jobs = []
    for s in range(4):
        jobs.append(make_job(1 << 18, 4, "uniform", 2000, 8, 0.5, 300 + s))
    total = sum(om.occ_hashed(j.text, j.patterns)[0].size for j in jobs)
    assert total > 8192
    plans = [mag.Plan(j.patterns, mode="dense" if i % 2 else "filter") for i, j in enumerate(jobs)]
    texts = _upload(torch, [j.text for j in jobs], [1, 2, 3, 0])
    b = mag.Batch(plans)
    b.bind(texts, total + 100)
    _check_jobs(b.run(), jobs)
    b.close()


def test_batch_dense_jobs_between_filter_jobs(torch_cuda, mag):
    """Dense jobs (protein-like and Zipf alphabets, m = 8, 16, 32), many of
    whose patterns occur, with DNA dense jobs and filter jobs between them in
    the job order (the dense launch's job switches restage bitmaps and move
    the found-key buffers, which must be flushed first). Text lengths fall on
    and around multiples of the slice tiles (8064 positions per 8 waves), at
    unaligned addresses."""
    torch = torch_cuda
    tile = 16 * 63 * 8
    jobs, plans = [], []
    cases = [(20, 8, 3 * tile + 7), (20, 16, tile), (20, 32, tile - 1), (64, 8, 2 * tile + 33),
             (64, 16, 5000), (64, 32, 4 * tile + 1), (20, 16, 17), (20, 8, 200_003)]
    for i, (sigma, m, n) in enumerate(cases):
        job = make_job(n, sigma, "uniform" if i % 2 else "zipf", 300 if m == 8 else 3000, m, 1.0, 500 + i)
        jobs.append(job)
        plans.append(mag.Plan(job.patterns, mode="dense"))
        if i % 3 == 1:                      # a DNA dense job, then a filter job
            dna = make_job(60_000, 4, "uniform", 500, 8, 0.5, 600 + i)
            jobs.append(dna)
            plans.append(mag.Plan(dna.patterns, mode="dense"))
            flt = make_job(90_000, 20, "uniform", 100, 16, 0.5, 700 + i)
            jobs.append(flt)
            plans.append(mag.Plan(flt.patterns, mode="filter"))
    total = sum(om.occ_hashed(j.text, j.patterns)[0].size for j in jobs)
    assert total > 8192
    texts = _upload(torch, [j.text for j in jobs], [(5 * j) % 16 for j in range(len(jobs))])
    b = mag.Batch(plans)
    b.bind(texts, total + 64)
    _check_jobs(b.run(), jobs)
    _check_jobs(b.run(), jobs)
    b.close()


def test_batch_dense_exact_codes(torch_cuda, mag):
    """Dense jobs whose patterns use at most four byte values that one 2-bit
    field of the byte tells apart (DNA letters, or bytes 0..3) take exact
    window codes; texts hold other bytes too (N, lowercase, 4..255), which
    no window may match through a shared code. Lengths 1..8, a two-letter
    pattern alphabet, texts at unaligned addresses and around tile ends."""
    torch = torch_cuda
    rng = np.random.default_rng(808)
    jobs, plans = [], []

    def job(text, pats):
        pats = np.asarray(pats, dtype=np.uint8)
        jobs.append(Job(text, pats, {}))
        plans.append(mag.Plan(pats, mode="dense"))

    acgt = np.frombuffer(b"ACGT", dtype=np.uint8)
    for m, n in ((8, 100_003), (5, 16_384 * 3 + 5), (2, 40_000), (1, 9_000), (7, 16_383)):
        t = acgt[rng.integers(0, 4, n)]
        other = rng.random(n) < 0.01                      # N, n, a and random bytes
        t[other] = rng.choice(np.frombuffer(b"NnaX\x00\xc1", dtype=np.uint8), int(other.sum()))
        starts = rng.integers(0, n - m, 300)
        pats = np.stack([t[i:i + m] for i in starts])
        pats = pats[np.all(np.isin(pats, acgt), axis=1)]
        job(t, pats)
    # two letters of ACGT in the patterns
    t = acgt[rng.integers(0, 4, 50_000)]
    job(t, np.frombuffer(b"ACACCAAC" b"CCCCAAAA", dtype=np.uint8).reshape(2, 8))
    # bytes 0..3 (field at shift 0) against text bytes 0..7
    t = rng.integers(0, 8, 70_000).astype(np.uint8)
    pats = rng.integers(0, 4, (400, 6)).astype(np.uint8)
    job(t, pats)
    total = sum(om.occ_hashed(j.text, j.patterns)[0].size for j in jobs)
    assert total > 8192
    texts = _upload(torch, [j.text for j in jobs], [(3 * j + 1) % 16 for j in range(len(jobs))])
    b = mag.Batch(plans)
    b.bind(texts, total + 64)
    _check_jobs(b.run(), jobs)
    _check_jobs(b.run(), jobs)
    b.close()


def test_batch_graph_replay(torch_cuda, mag):
    torch = torch_cuda
    jobs = _small_jobs(12, seed=404)
    jobs.append(make_job(1 << 17, 4, "uniform", 1500, 8, 0.5, 405))    # > 8192 occurrences in all
    plans = [mag.Plan(j.patterns) for j in jobs]
    texts = _upload(torch, [j.text for j in jobs])
    refs = [om.occ_hashed(j.text, j.patterns) for j in jobs]
    total = sum(r[0].size for r in refs)
    cap = total + 64
    b = mag.Batch(plans)
    stream = torch.cuda.Stream()
    b.bind(texts, cap, stream)
    out = torch.empty((cap, 2), dtype=torch.int64, device="cuda")
    offsets = torch.empty(len(jobs) + 1, dtype=torch.int64, device="cuda")
    count = torch.empty(1, dtype=torch.int64, device="cuda")
    with torch.cuda.stream(stream):
        b.run_async(out, offsets, count, stream)       # eager warm-up
    stream.synchronize()
    eager = (out[:total].clone(), offsets.clone(), count.clone())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        b.run_async(out, offsets, count, torch.cuda.current_stream())
    for rep in range(3):
        out.fill_(-1)
        offsets.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        assert int(count.item()) == total, rep
        assert torch.equal(offsets, eager[1]), rep
        assert torch.equal(out[:total], eager[0]), rep
        # eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        del junk
    off = offsets.cpu().tolist()
    _check_jobs([out[off[j]:off[j + 1]] for j in range(len(jobs))], jobs)
    b.close()


def test_batch_rebind_smaller(torch_cuda, mag):
    torch = torch_cuda
    jobs_a = _small_jobs(8, seed=505, n_log2=(15.0, 18.0))
    plans = [mag.Plan(j.patterns) for j in jobs_a]
    b = mag.Batch(plans)
    b.bind(_upload(torch, [j.text for j in jobs_a]), 1 << 15)
    _check_jobs(b.run(), jobs_a)
    # same pattern sets, shorter texts
    jobs_b = []
    for j, job in enumerate(jobs_a):
        t = gen_text(max(job.n // 5, 1), job.recipe["sigma"], job.recipe["dist"], rng=600 + j)
        jobs_b.append(type(job)(t, job.patterns, {}))
    b.bind(_upload(torch, [j.text for j in jobs_b]), 1 << 10)
    _check_jobs(b.run(), jobs_b)
    b.close()


def test_batch_rejects_wide_plans(torch_cuda, mag):
    t = gen_text(10_000, 64, rng=1)
    p = gen_patterns(t, 10, 64, 5, 64, rng=2)
    plan = mag.Plan(p, q=1, k=1, sigma_prime=64, mode="filter")       # W = 64
    with pytest.raises(mag.MagError):
        mag.Batch([plan])


def test_batch_full_workload(torch_cuda, mag):
    """The 512-job workload at full size (about 1.1 GB of text), heuristic
    parameters: every job's list equals the oracle's."""
    torch = torch_cuda
    jobs = batch_jobs(512, workers=16)
    plans = [mag.Plan(j.patterns) for j in jobs]
    texts = _upload(torch, [j.text for j in jobs])
    refs = [om.occ_hashed(j.text, j.patterns) for j in jobs]
    total = sum(r[0].size for r in refs)
    b = mag.Batch(plans)
    b.bind(texts, total + 1024)
    res = b.run()
    for j, (occ, (rpos, rids)) in enumerate(zip(res, refs)):
        occ = occ.cpu().numpy()
        assert occ.shape[0] == rpos.size, (j, occ.shape[0], rpos.size, jobs[j].recipe)
        assert np.array_equal(occ[:, 0].astype(np.uint64), rpos), j
        assert np.array_equal(occ[:, 1].astype(np.uint32), rids), j
    b.close()


def test_scan_batch_one_shot(torch_cuda, mag):
    # mag_scan_batch: one call builds, binds, runs and reads the offsets. A
    # plan serves two jobs, one text is empty, and the first capacity is too
    # small, so the binding rescans with the exact total it reports.
    torch = torch_cuda
    jobs = _small_jobs(6, seed=211)
    jobs.append(make_job(0, 4, "uniform", 10, 8, 0.5, 212))
    plans = [mag.Plan(j.patterns) for j in jobs]
    t2 = gen_text(40_003, jobs[1].recipe["sigma"], rng=213)
    jobs.append(type(jobs[0])(t2, jobs[1].patterns, {"shared": True}))
    plans.append(plans[1])
    texts = _upload(torch, [j.text for j in jobs], [j % 5 for j in range(len(jobs))])
    total = sum(om.occ_hashed(j.text, j.patterns)[0].size for j in jobs)
    assert total > 2
    res = mag.scan_batch(texts, plans, out_cap=total // 2)
    _check_jobs(res, jobs)
    res = mag.scan_batch(texts, plans, out_cap=total)
    _check_jobs(res, jobs)
    assert mag.scan_batch([], []) == []


def test_batch_rounds_with_more_keys_than_the_buffer(torch_cuda, mag):
    """Jobs whose verification rounds emit more keys than a wave's buffer:
    a^n against six copies of a^8 (384 keys per round of 64 starts), short
    enough to defer its starts to the batch verification kernel, as a filter
    and as a dense job, between two ordinary jobs."""
    torch = torch_cuda
    a = np.full(30_000, ord("a"), dtype=np.uint8)
    dup = np.full((6, 8), ord("a"), dtype=np.uint8)
    jobs = _small_jobs(2, seed=909)
    jobs[1:1] = [Job(a, dup, {"dup": "filter"}), Job(a.copy(), dup, {"dup": "dense"})]
    plans = [mag.Plan(jobs[0].patterns), mag.Plan(dup, q=2, k=2, sigma_prime=2, mode="filter"),
             mag.Plan(dup, mode="dense"), mag.Plan(jobs[3].patterns)]
    texts = _upload(torch, [j.text for j in jobs], [3, 0, 5, 1])
    total = sum(om.occ_hashed(j.text, j.patterns)[0].size for j in jobs)
    b = mag.Batch(plans)
    b.bind(texts, total + 64)
    _check_jobs(b.run(), jobs)
    _check_jobs(b.run(), jobs)
    b.close()


@pytest.mark.parametrize("plants", [3, 5], ids=["lds-sort", "radix-sort"])
def test_batch_many_jobs(torch_cuda, mag, plants):
    """2,100 jobs (more than the record writer stages in LDS), each a
    256-byte slice of one buffer scanned with one shared plan: 3 planted
    occurrences per job (6,300, sorted in the finishing kernel) or 5 (10,500,
    the device-wide sort)."""
    torch = torch_cuda
    rng = np.random.default_rng(77 + plants)
    njobs, seg, m = 2100, 256, 8
    pats = np.unique(np.concatenate([np.full((6, 1), ord("Z"), np.uint8),
                                     rng.integers(65, 85, (6, m - 1)).astype(np.uint8)], axis=1), axis=0)
    text = rng.integers(65, 85, njobs * seg).astype(np.uint8)
    at = np.array([10, 60, 110, 160, 210][:plants])
    which = rng.integers(0, pats.shape[0], (njobs, plants))
    for j in range(njobs):
        for t in range(plants):
            text[j * seg + at[t]:j * seg + at[t] + m] = pats[which[j, t]]
    big = torch.from_numpy(text).cuda()
    plan = mag.Plan(pats)
    b = mag.Batch([plan] * njobs)
    b.bind([big[j * seg:(j + 1) * seg] for j in range(njobs)], njobs * plants + 64)
    res = b.run()
    assert len(res) == njobs
    for j, occ in enumerate(res):
        occ = occ.cpu().numpy()
        assert np.array_equal(occ[:, 0], at.astype(np.int64)), j
        assert np.array_equal(occ[:, 1], which[j].astype(np.int64)), j
    b.close()


def test_batch_positions_past_32_bits(torch_cuda, mag):
    """Keys hold positions in the jobs' texts laid end to end: five views of
    one 900 MB text (4.5 GB in all, past 2^32) with planted patterns. Text
    bytes are A..T and every pattern starts with Z, so the planted copies
    are the only occurrences; each view starts 7 bytes later than the one
    before, and filter and dense plans alternate."""
    torch = torch_cuda
    rng = np.random.default_rng(4242)
    n = 900_000_000
    big = torch.randint(65, 85, (n,), dtype=torch.uint8, device="cuda")
    r, m = 150, 16
    pats = np.empty((r, m), dtype=np.uint8)
    pats[:, 0] = ord("Z")
    pats[:, 1:] = rng.integers(65, 85, (r, m - 1))
    pats = np.unique(pats, axis=0)
    r = pats.shape[0]
    starts = np.sort(rng.choice(n // 64, 400, replace=False)) * 64 + 40
    which = rng.integers(0, r, starts.size)
    idx = torch.from_numpy((starts[:, None] + np.arange(m)).reshape(-1)).cuda()
    big[idx] = torch.from_numpy(pats[which].reshape(-1)).cuda()
    plans = [mag.Plan(pats, mode="filter"), mag.Plan(pats, mode="dense")]
    views, bplans, expect = [], [], []
    for j in range(5):
        sh = 7 * j
        views.append(big[sh:])
        bplans.append(plans[j % 2])
        keep = starts >= sh
        expect.append((starts[keep] - sh, which[keep]))
    b = mag.Batch(bplans)
    b.bind(views, 5 * starts.size + 64)
    for res in (b.run(), b.run()):
        for j, (occ, (pos, ids)) in enumerate(zip(res, expect)):
            occ = occ.cpu().numpy()
            assert occ.shape[0] == pos.size, (j, occ.shape[0], pos.size)
            assert np.array_equal(occ[:, 0], pos.astype(np.int64)), j
            assert np.array_equal(occ[:, 1], ids.astype(np.int64)), j
    b.close()


@pytest.mark.parametrize("words", [8, 16])
def test_batch_words_per_lane(torch_cuda, mag, words):
    """Filter tiles of 1024 * words samples (dense jobs take their own launch):
    the same lists for every tile shape, jobs of a few tiles each."""
    jobs = _small_jobs(20, seed=303, n_log2=(12.0, 19.0))
    plans = [mag.Plan(j.patterns, mode="dense" if i % 4 == 3 else "filter") for i, j in enumerate(jobs)]
    texts = _upload(torch_cuda, [j.text for j in jobs], [(5 * j) % 16 for j in range(len(jobs))])
    b = mag.Batch(plans, words_per_lane=words)
    b.bind(texts, 1 << 17)
    _check_jobs(b.run(), jobs)
    b.close()


def test_autotuned_batch(torch_cuda, mag):
    """The batch autotuner's picks (one per job class, filter or dense, with
    their tile shapes) and its words per lane: every job's list equals the
    oracle's."""
    jobs = _small_jobs(32, seed=404, n_log2=(12.0, 18.0), r_log10=(1.0, 3.5))
    texts = _upload(torch_cuda, [j.text for j in jobs])
    kws, words = mag.autotune_batch([j.patterns for j in jobs], texts, sample_bytes=1 << 16,
                                    max_candidates=4, repeats=1)
    assert words in (8, 16) and len(kws) == len(jobs)
    assert all(kw["mode"] in ("filter", "dense") for kw in kws)
    plans = [mag.Plan(j.patterns, **kw) for j, kw in zip(jobs, kws)]
    b = mag.Batch(plans, words_per_lane=words)
    b.bind(texts, 1 << 18)
    _check_jobs(b.run(), jobs)
    b.close()
