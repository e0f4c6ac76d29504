"""Parity of the HIP scan against the oracle (GPU).

Every case compares the library's occurrence list element by element with the
oracle's (bit-exact: positions and ids are integers), and where the sizes let
the numpy oracle finish in seconds also the filter's work counters (candidate
windows and verified start positions) with the counts the oracle derives from
the definitions of Sections 2-3.
"""

import numpy as np
import pytest

from oracle import match as om
from oracle import method as mm
from synth import gen_patterns, gen_text, make_job, workload

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


def _gpu_occ(torch, mag, text_np, plan, offset=0, out_cap=None, stats=False):
    buf = torch.empty(text_np.size + offset + 16, dtype=torch.uint8, device="cuda")
    view = buf[offset:offset + text_np.size]
    view.copy_(torch.from_numpy(text_np))
    res = mag.scan(view, plan, out_cap=out_cap, stats=stats)
    if stats:
        occ, st = res
    else:
        occ, st = res, None
    occ = occ.cpu().numpy()
    return occ[:, 0].astype(np.uint64), occ[:, 1].astype(np.uint32), st


def _assert_same(pos, ids, ref):
    rpos, rids = ref
    assert pos.size == rpos.size, (pos.size, rpos.size)
    assert np.array_equal(pos, rpos)
    assert np.array_equal(ids, rids)


CASES = [
    # sigma, n, r, m, q, k, sigma', kind
    (4, 200_001, 30, 8, 2, 1, 4, "greedy"),
    (4, 150_003, 30, 8, 2, 2, 3, "rank"),
    (4, 300_007, 100, 16, 5, 1, 4, "greedy"),
    (4, 120_000, 50, 16, 3, 4, 4, "greedy"),
    (20, 250_013, 60, 16, 3, 4, 7, "greedy"),
    (20, 250_000, 60, 16, 1, 5, 20, "rank"),
    (20, 180_001, 500, 16, 4, 1, 12, "greedy"),
    (64, 200_000, 40, 32, 2, 3, 16, "greedy"),
    (64, 200_003, 40, 32, 2, 3, 64, "rank"),
    (64, 220_000, 40, 32, 4, 2, 16, "greedy"),
    (64, 100_000, 10, 64, 1, 1, 64, "greedy"),    # W = 64, u64 state
    (64, 100_000, 10, 64, 2, 7, 9, "rank"),       # W = 28
    (64, 100_000, 12, 64, 1, 32, 64, "greedy"),   # k = 32, m' = 2
    (2, 90_000, 5, 9, 5, 1, 2, "greedy"),         # m = 2q - 1
    (4, 80_000, 8, 12, 4, 1, 1, "greedy"),        # sigma' = 1: every window verified
    (20, 150_000, 30, 15, 7, 1, 6, "greedy"),     # q = 7: grams straddle two words
    (20, 150_000, 30, 17, 8, 1, 5, "rank"),       # q = 8
    (4, 100_000, 20, 16, 1, 16, 4, "greedy"),     # k = L
    (4, 200_003, 100, 16, 4, 1, 4, "bits"),       # bit-field map, DNA (shift 1)
    (64, 250_000, 60, 32, 4, 1, 16, "bits"),      # low nibbles
    (64, 180_001, 40, 32, 4, 2, 16, "bits"),
    (20, 150_000, 30, 17, 8, 1, 4, "bits"),       # q = 8 from two words
    (64, 120_000, 20, 32, 2, 3, 256, "bits"),     # l = 8: the byte itself
    (20, 200_003, 300, 16, 8, 1, 1 << 12, "qgram"),  # q-gram map: 1-bit entries in LDS
    (4, 150_001, 100, 16, 5, 1, 1 << 10, "qgram"),   # W = 2: 2-bit entries
    (64, 200_000, 40, 32, 6, 2, 1 << 9, "qgram"),    # W = 4: 4-bit entries
    (64, 180_000, 40, 32, 3, 3, 1 << 6, "qgram"),    # W = 9: 2-byte entries
    (64, 100_000, 10, 64, 1, 1, 1 << 5, "qgram"),    # W = 64, q = 1
    (20, 150_000, 30, 16, 2, 3, 1 << 8, "qgram"),    # q = 2
    (20, 150_000, 30, 15, 7, 1, 1 << 14, "qgram"),   # q = 7
    (4, 120_000, 20, 8, 3, 1, 1 << 20, "qgram"),     # 2-bit entries, table in global memory
    (20, 150_000, 60, 16, 4, 1, 1 << 22, "qgram"),   # 4-bit entries, 2 MiB table
    (64, 100_000, 20, 32, 4, 1, 1 << 17, "qgram"),   # W = 7: whole bytes, 128 KiB table
    (20, 100_000, 20, 16, 4, 1, 1, "qgram"),         # sigma' = 1: every window verified
]


@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}-n{c[1]}-r{c[2]}-m{c[3]}-q{c[4]}-k{c[5]}-sp{c[6]}-{c[7]}" for c in CASES])
def test_parity_and_counts(torch_cuda, mag, case):
    sigma, n, r, m, q, k, sp, kind = case
    T = gen_text(n, sigma, dist="zipf" if sigma == 64 else "uniform", rng=n + r)
    P = gen_patterns(T, r, m, (3 * r) // 4, sigma, rng=r * 31 + m)
    plan = mag.Plan(P, q=q, k=k, sigma_prime=sp, map_kind=kind, mode="filter")
    pos, ids, st = _gpu_occ(torch_cuda, mag, T, plan, stats=True)
    ref = om.occ_hashed(T, P)
    assert ref[0].size > 0
    _assert_same(pos, ids, ref)
    want = mm.Filter(P, q, k, sp, kind).counts(T)
    assert st["samples"] == want["samples"]
    assert st["cand_windows"] == want["cand_windows"]
    assert st["verifications"] == want["verifications"]
    assert st["matches"] == ref[0].size


@pytest.mark.parametrize("probe", ["bloom", "slices"])
@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}-n{c[1]}-r{c[2]}-m{c[3]}" for c in CASES])
def test_dense_mode_parity(torch_cuda, mag, case, probe):
    """Every start position through the dense bitmap (three-probe Bloom, or
    one probe per position into the slice bitmap): the same occurrence list;
    every occurring position passes the bitmap."""
    sigma, n, r, m, q, k, sp, kind = case
    T = gen_text(n, sigma, dist="zipf" if sigma == 64 else "uniform", rng=n + r)
    P = gen_patterns(T, r, m, (3 * r) // 4, sigma, rng=r * 31 + m)
    plan = mag.Plan(P, q=q, k=k, sigma_prime=sp, map_kind=kind, mode="dense", dense_probe=probe)
    info = plan.info()
    assert info["dense"] == 1
    assert (info["dense_slices"] > 0) == (probe == "slices")
    pos, ids, st = _gpu_occ(torch_cuda, mag, T, plan, stats=True)
    ref = om.occ_hashed(T, P)
    _assert_same(pos, ids, ref)
    assert st["samples"] == n - m + 1
    assert st["verifications"] == st["cand_windows"] >= np.unique(ref[0]).size
    assert st["matches"] == ref[0].size


@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}-n{c[1]}-r{c[2]}-m{c[3]}-q{c[4]}-{c[7]}" for c in CASES])
def test_deferred_verification_parity(torch_cuda, mag, case):
    """Starts deferred to the verification kernel: the same list and the same
    counters; with a 4096-entry buffer every case that verifies more starts
    than that also takes the inline fallback for the overflow."""
    sigma, n, r, m, q, k, sp, kind = case
    T = gen_text(n, sigma, dist="zipf" if sigma == 64 else "uniform", rng=n + r)
    P = gen_patterns(T, r, m, (3 * r) // 4, sigma, rng=r * 31 + m)
    ref = om.occ_hashed(T, P)
    want = mm.Filter(P, q, k, sp, kind).counts(T)
    for buf in (0, 4096):
        plan = mag.Plan(P, q=q, k=k, sigma_prime=sp, map_kind=kind, mode="filter",
                        verify="deferred", verify_buffer=buf)
        pos, ids, st = _gpu_occ(torch_cuda, mag, T, plan, stats=True)
        _assert_same(pos, ids, ref)
        assert (st["cand_windows"], st["verifications"]) == (want["cand_windows"], want["verifications"])
    # the dense mode defers its Bloom-bitmap survivors the same way
    plan = mag.Plan(P, mode="dense", verify="deferred", verify_buffer=4096)
    pos, ids, st = _gpu_occ(torch_cuda, mag, T, plan, stats=True)
    _assert_same(pos, ids, ref)


def test_dense_tile_edges(torch_cuda, mag):
    # the single-job dense kernel takes 16,384 start positions per tile, 16
    # per lane: texts whose last start falls on either side of a tile or lane
    # boundary, at every text alignment, with patterns copied from the
    # positions around those boundaries
    m, tile = 16, 16384
    T0 = gen_text(3 * tile + 64, 20, rng=91)
    at = [0, 15, 16, tile - 17, tile - 1, tile, tile + 1, 2 * tile - 1, 2 * tile, 2 * tile + 6]
    P = np.stack([T0[u:u + m] for u in at] + list(gen_patterns(T0, 20, m, 10, 20, rng=92)))
    plan = mag.Plan(P, mode="dense")
    assert plan.info()["dense"] == 1
    for npos in (1, 2, 16, 17, tile - 16, tile - 1, tile, tile + 1, tile + 2, 2 * tile + 7):
        T = T0[:npos + m - 1]
        ref = om.occ_hashed(T, P)
        for off in (0, 1, 2, 3):
            pos, ids, _ = _gpu_occ(torch_cuda, mag, T, plan, offset=off)
            _assert_same(pos, ids, ref)


def test_dense_slice_tile_edges(torch_cuda, mag):
    # the one-probe dense kernel takes 16,128 start positions per tile: 16
    # waves of 63 owning lanes with 16 positions each (1,008 per wave), the
    # 64th lane of a wave probing the next wave's first 16. Texts whose last
    # start falls around lane, wave and tile boundaries, at every alignment,
    # with patterns copied from around those boundaries, for every number of
    # slices per pattern (k = 1 .. 6 for m = 16, forced by the pattern count)
    m, tile, span = 16, 16128, 1008
    T0 = gen_text(3 * tile + 64, 20, rng=93)
    at = [0, 1, 15, 16, span - 17, span - 16, span - 1, span, span + 1, 2 * span - 1,
          tile - 17, tile - 16, tile - 1, tile, tile + 1, 2 * tile - 1, 2 * tile, 2 * tile + 6]
    base = np.stack([T0[u:u + m] for u in at])
    seen = set()
    # uniform extra patterns (all distinct): k = round(ln 2 * 2^20 / count)
    for extra in (0, 140_000, 180_000, 250_000, 400_000, 800_000):
        P = np.concatenate([base, gen_patterns(T0, extra, m, 0, 20, rng=94)]) if extra else base
        plan = mag.Plan(P, mode="dense", dense_probe="slices")
        k = plan.info()["dense_slices"]
        seen.add(k)
        for npos in (1, 17, span - 1, span, span + 1, tile - 1, tile, 2 * tile + 7):
            T = T0[:npos + m - 1]
            ref = om.occ_hashed(T, P)
            for off in (0, 1, 2, 3):
                pos, ids, _ = _gpu_occ(torch_cuda, mag, T, plan, offset=off)
                _assert_same(pos, ids, ref)
    assert seen == {1, 2, 3, 4, 5, 6}


@pytest.mark.parametrize("m", [6, 7, 8, 9, 10, 13, 20, 32, 64])
def test_dense_slice_lengths(torch_cuda, mag, m):
    """Slices at offsets 0, 2, .. within m bytes: every length from the
    shortest the slices allow, with occurrences planted near both ends."""
    T = gen_text(70_001, 20, rng=95 + m)
    P = gen_patterns(T, 400, m, 300, 20, rng=96 + m)
    plan = mag.Plan(P, mode="dense", dense_probe="slices")
    info = plan.info()
    assert 1 <= info["dense_slices"] <= min(8, (m - 6) // 2 + 1)
    Tm = np.concatenate([P[0], T, P[1]])
    pos, ids, st = _gpu_occ(torch_cuda, mag, Tm, plan, stats=True)
    ref = om.occ_hashed(Tm, P)
    _assert_same(pos, ids, ref)
    assert st["cand_windows"] >= np.unique(ref[0]).size


def test_deferred_overflow_and_repeat(torch_cuda, mag):
    """sigma' = 1 verifies every start: 300 000 deferred starts through a
    4096-entry buffer, twice in a row on the same plan (the deferred count
    must return to zero between scans), then a smaller text."""
    T = gen_text(300_000, 4, rng=77)
    P = gen_patterns(T, 40, 12, 30, 4, rng=78)
    plan = mag.Plan(P, q=4, k=1, sigma_prime=1, mode="filter", verify="deferred", verify_buffer=4096)
    for t in (T, T, T[:5000]):
        pos, ids, st = _gpu_occ(torch_cuda, mag, t, plan, stats=True)
        _assert_same(pos, ids, om.occ_hashed(t, P))
        assert st["verifications"] == t.size - 12 + 1


def _upload(torch, t, offset=0):
    buf = torch.empty(t.size + offset + 16, dtype=torch.uint8, device="cuda")
    view = buf[offset:offset + t.size]
    if t.size:
        view.copy_(torch.from_numpy(t))
    return view


@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}-q{c[4]}-k{c[5]}-sp{c[6]}-{c[7]}" for c in CASES])
def test_encoded_text_equals_oracle(torch_cuda, mag, case):
    """SMAG's encoding pass: every q-gram code, bit-exact, at two text
    alignments."""
    sigma, n, r, m, q, k, sp, kind = case
    T = gen_text(n, sigma, dist="zipf" if sigma == 64 else "uniform", rng=n + r)
    P = gen_patterns(T, r, m, (3 * r) // 4, sigma, rng=r * 31 + m)
    plan = mag.Plan(P, q=q, k=k, sigma_prime=sp, map_kind=kind)
    want = mm.Filter(P, q, k, sp, kind).encode(T)
    for offset in (0, 3):
        got = mag.encode(_upload(torch_cuda, T, offset), plan).cpu().numpy().astype(np.uint32)
        assert got.size == want.size
        assert np.array_equal(got, want.astype(np.uint32))


@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}-n{c[1]}-q{c[4]}-k{c[5]}-sp{c[6]}-{c[7]}" for c in CASES])
def test_smag_parity_and_counts(torch_cuda, mag, case):
    """The text encoded first (SMAG), then filtered from the codes: the same
    occurrence list and the same work counters as the definitions give."""
    sigma, n, r, m, q, k, sp, kind = case
    T = gen_text(n, sigma, dist="zipf" if sigma == 64 else "uniform", rng=n + r)
    P = gen_patterns(T, r, m, (3 * r) // 4, sigma, rng=r * 31 + m)
    plan = mag.Plan(P, q=q, k=k, sigma_prime=sp, map_kind=kind, mode="filter", encode=True)
    pos, ids, st = _gpu_occ(torch_cuda, mag, T, plan, offset=5, stats=True)
    ref = om.occ_hashed(T, P)
    _assert_same(pos, ids, ref)
    want = mm.Filter(P, q, k, sp, kind).counts(T)
    assert (st["samples"], st["cand_windows"], st["verifications"]) == \
        (want["samples"], want["cand_windows"], want["verifications"])


def test_smag_edges(torch_cuda, mag):
    """Texts shorter than q, exactly q, and a deferred-verification SMAG scan
    whose codes need 32 bits."""
    T = gen_text(100_000, 20, rng=91)
    P = gen_patterns(T, 200, 16, 150, 20, rng=92)
    plan = mag.Plan(P, q=5, k=1, sigma_prime=20, mode="filter", encode=True, verify="deferred")
    assert plan.info()["n_codes"] > 65536
    for t in (T[:3], T[:5], T[:16], T[:16 + 5 * 7 + 2], T):
        pos, ids, _ = _gpu_occ(torch_cuda, mag, t, plan)
        _assert_same(pos, ids, om.occ_hashed(t, P))
    assert mag.encode(_upload(torch_cuda, T[:4]), plan).numel() == 0


UNEQUAL = [
    # sigma, n, r, lengths, q, k, sigma', kind
    (4, 200_003, 60, (8, 9, 12, 16), 2, 2, 4, "greedy"),
    (20, 250_001, 300, (12, 16, 20, 32), 3, 1, 12, "greedy"),
    (64, 220_000, 80, (16, 24, 33, 64), 4, 2, 16, "rank"),
    (20, 150_000, 100, (5, 6, 7, 64), 1, 2, 20, "greedy"),
    (20, 180_000, 200, (16, 17, 31), 8, 1, 1 << 14, "qgram"),
]


def _unequal_case(case, seed=0):
    sigma, n, r, lens, q, k, sp, kind = case
    rng = np.random.default_rng(n + r + seed)
    T = gen_text(n, sigma, dist="zipf" if sigma == 64 else "uniform", rng=n + r)
    pats = []
    for i in range(r):
        L = int(rng.choice(lens))
        if i % 4 == 3:                               # random: mostly absent
            pats.append(bytes(gen_text(L, sigma, rng=int(rng.integers(1 << 30)))))
        else:
            u = int(rng.integers(0, n - L))
            pats.append(bytes(T[u:u + L]))
    pats.append(pats[0])                             # a duplicate
    pats.append(pats[1][: min(lens)])                # a prefix of another pattern
    tail = bytes(T[n - min(lens):])                  # occurs at the last start; its
    pats.append(tail + b"\x00" * (max(lens) - len(tail)))   # extension runs past the end
    pats.append(tail)
    return T, pats


@pytest.mark.parametrize("case", UNEQUAL, ids=[f"s{c[0]}-r{c[2]}-q{c[4]}-{c[7]}" for c in UNEQUAL])
def test_unequal_lengths_parity(torch_cuda, mag, case):
    """Patterns of several lengths: the filter over their shortest prefixes,
    verification over full lengths; filter, dense, deferred and SMAG scans
    all give the oracle's list, and the filter's counters are the prefix
    set's."""
    sigma, n, r, lens, q, k, sp, kind = case
    T, pats = _unequal_case(case)
    ref = om.occ_var(T, pats)
    assert ref[0].size > r // 2
    want = mm.Filter(mm.prefix_set(pats), q, k, sp, kind).counts(T)
    for kw in (dict(mode="filter"), dict(mode="dense"), dict(mode="filter", verify="deferred"),
               dict(mode="filter", encode=True)):
        plan = mag.Plan(pats, q=q, k=k, sigma_prime=sp, map_kind=kind, **kw)
        assert plan.info()["var"] == 1
        pos, ids, st = _gpu_occ(torch_cuda, mag, T, plan, offset=3, stats=True)
        _assert_same(pos, ids, ref)
        if kw["mode"] == "filter":
            assert (st["cand_windows"], st["verifications"]) == (want["cand_windows"], want["verifications"])


def test_unequal_lengths_nested_closed_form(torch_cuda, mag):
    # a^n with patterns a^1 .. a^9: a^L occurs at every i <= n - L
    n = 100_000
    T = np.full(n, ord("a"), dtype=np.uint8)
    pats = [b"a" * L for L in (3, 1, 9, 2, 5)]
    plan = mag.Plan(pats)
    pos, ids, _ = _gpu_occ(torch_cuda, mag, T, plan)
    assert pos.size == sum(n - len(p) + 1 for p in pats)
    _assert_same(pos, ids, om.occ_var(T, pats))


def test_batch_rejects_unequal_lengths(torch_cuda, mag):
    plan = mag.Plan([b"ACGTACGT", b"ACGTACGTAC"])
    with pytest.raises(mag.MagError):
        mag.Batch([plan])


@pytest.mark.parametrize("offset", [0, 1, 3, 7, 13])
def test_unaligned_text(torch_cuda, mag, offset):
    T = gen_text(100_003, 4, rng=offset)
    P = gen_patterns(T, 40, 16, 30, 4, rng=5)
    plan = mag.Plan(P)
    pos, ids, _ = _gpu_occ(torch_cuda, mag, T, plan, offset=offset)
    _assert_same(pos, ids, om.occ_hashed(T, P))


def test_edge_lengths(torch_cuda, mag):
    P = np.frombuffer(b"ACGTACGTAC", dtype=np.uint8).reshape(1, 10)
    plan = mag.Plan(P, q=2, k=2, sigma_prime=4)
    for n in (0, 1, 5, 9, 10, 11, 19, 20, 21, 64, 65):
        T = np.frombuffer((b"ACGT" * 20)[:n], dtype=np.uint8).copy()
        pos, ids, st = _gpu_occ(torch_cuda, mag, T, plan, stats=True)
        _assert_same(pos, ids, om.occ_hashed(T, P))
        want = mm.Filter(P, 2, 2, 4).counts(T)
        assert (st["cand_windows"], st["verifications"]) == (want["cand_windows"], want["verifications"])


def test_matches_at_both_ends_and_duplicates(torch_cuda, mag):
    rng = np.random.default_rng(2)
    n, m = 70_001, 16
    T = gen_text(n, 20, rng=3)
    P = gen_patterns(T, 20, m, 0, 20, rng=4)
    T[:m] = P[3]
    T[n - m:] = P[7]
    P = np.concatenate([P, P[[3, 7, 3]]])        # ids 20, 22 repeat pattern 3; 21 repeats 7
    for kw in (dict(), dict(q=3, k=2, sigma_prime=20), dict(q=1, k=1, sigma_prime=20)):
        plan = mag.Plan(P, **kw)
        pos, ids, _ = _gpu_occ(torch_cuda, mag, T, plan)
        ref = om.occ_hashed(T, P)
        _assert_same(pos, ids, ref)
        assert pos[0] == 0 and list(ids[pos == 0]) == [3, 20, 22]
        assert pos[-1] == n - m and list(ids[pos == n - m]) == [7, 21]


def test_extreme_bytes(torch_cuda, mag):
    rng = np.random.default_rng(9)
    T = rng.choice(np.array([0, 255, 1, 254], dtype=np.uint8), size=50_000)
    P = np.stack([T[u:u + 12] for u in rng.integers(0, 50_000 - 12, size=25)])
    P[0] = 0
    P[1] = 255
    T[100:112] = 0
    T[40_000:40_012] = 255
    for kw in (dict(), dict(q=3, k=1, sigma_prime=4, map_kind="rank")):
        plan = mag.Plan(P, **kw)
        pos, ids, _ = _gpu_occ(torch_cuda, mag, T, plan)
        _assert_same(pos, ids, om.occ_hashed(T, P))


@pytest.mark.parametrize("kw", [dict(q=2, k=2, sigma_prime=2), dict(mode="dense")],
                         ids=["filter", "dense"])
def test_many_matches_radix_path(torch_cuda, mag, kw):
    # a^n against {a^m} x 3 ids: 3(n-m+1) occurrences, far beyond the LDS sort.
    # The device sort passes over the position bits only; the three ids of a
    # start leave the verification as one ascending run, which the stable
    # passes keep in order.
    n, m = 200_000, 8
    T = np.full(n, ord("a"), dtype=np.uint8)
    P = np.full((3, m), ord("a"), dtype=np.uint8)
    plan = mag.Plan(P, **kw)
    pos, ids, st = _gpu_occ(torch_cuda, mag, T, plan, stats=True)
    assert pos.size == 3 * (n - m + 1)
    assert np.array_equal(pos, np.repeat(np.arange(n - m + 1, dtype=np.uint64), 3))
    assert np.array_equal(ids, np.tile(np.arange(3, dtype=np.uint32), n - m + 1))
    assert st["verifications"] == n - m + 1


@pytest.mark.parametrize("kw", [dict(q=2, k=2, sigma_prime=2, mode="filter"),
                                dict(q=2, k=2, sigma_prime=2, mode="filter", verify="deferred",
                                     verify_buffer=1 << 20),
                                dict(mode="dense"),
                                dict(mode="dense", verify="deferred", verify_buffer=1 << 20)],
                         ids=["filter", "filter-deferred", "dense", "dense-deferred"])
def test_rounds_with_more_keys_than_the_buffer(torch_cuda, mag, kw):
    # a^n against {a^m} x 6 ids: every verification round of 64 starts emits
    # 384 keys, more than a wave's found-key buffer holds (64 keys in the
    # scan kernels, 256 in the verification kernel), so those rounds go to
    # the output directly; the buffers' leftovers are flushed per workgroup.
    n, m, dup = 50_000, 8, 6
    T = np.full(n, ord("a"), dtype=np.uint8)
    P = np.full((dup, m), ord("a"), dtype=np.uint8)
    plan = mag.Plan(P, **kw)
    pos, ids, _ = _gpu_occ(torch_cuda, mag, T, plan)
    assert pos.size == dup * (n - m + 1)
    assert np.array_equal(pos, np.repeat(np.arange(n - m + 1, dtype=np.uint64), dup))
    assert np.array_equal(ids, np.tile(np.arange(dup, dtype=np.uint32), n - m + 1))


def test_many_matches_unequal_lengths_radix_path(torch_cuda, mag):
    # a^n against {a^10, a^8, a^9, a^8}: every pattern that fits matches at
    # every start, found through one prefix group in member order (not id
    # order), so the device sort also passes over the id bits here
    n = 30_000
    T = np.full(n, ord("a"), dtype=np.uint8)
    pats = [b"a" * 10, b"a" * 8, b"a" * 9, b"a" * 8]
    plan = mag.Plan(pats)
    assert plan.info()["var"] == 1
    pos, ids, _ = _gpu_occ(torch_cuda, mag, T, plan)
    ref = om.occ_var(T, pats)
    assert ref[0].size > 8192
    _assert_same(pos, ids, ref)


def test_small_outputs_around_rank_blocks(torch_cuda, mag):
    # Outputs up to 8192 occurrences are ranked by the finishing kernel in
    # blocks of 64 keys, with the first 1024 keys loaded before the count is
    # known; larger ones take the radix sort. Text a^L c^m against
    # {a^m, a^m} (+ c^m for odd counts) gives exactly z occurrences, with
    # two ids per position. The same two plans serve every scan in turn, so
    # counters that were not returned to zero would show in the next count.
    m = 8
    plans = {}
    for odd in (False, True):
        P = [np.full(m, ord("a"), dtype=np.uint8)] * 2
        if odd:
            P.append(np.full(m, ord("c"), dtype=np.uint8))
        P = np.stack(P)
        plans[odd] = (P, mag.Plan(P, q=2, k=1, sigma_prime=3))
    for z in (1, 2, 63, 64, 65, 127, 511, 1023, 1024, 1025, 1537, 4097, 8191, 8192, 8193, 9001):
        odd = bool(z % 2)
        P, plan = plans[odd]
        L = (z - 1) // 2 + m - 1 if odd else z // 2 + m - 1
        T = np.concatenate([np.full(L, ord("a"), dtype=np.uint8), np.full(m, ord("c"), dtype=np.uint8)])
        if z == 1:
            T = np.full(m, ord("c"), dtype=np.uint8)
        ref = om.occ_hashed(T, P)
        assert ref[0].size == z, (z, ref[0].size)
        pos, ids, st = _gpu_occ(torch_cuda, mag, T, plan, stats=True)
        _assert_same(pos, ids, ref)
        assert st["matches"] == z, (z, st)


def test_capacities_alternating_on_shared_plans(torch_cuda, mag):
    # Scans on shared plans alternate between a capacity the finishing kernel
    # sorts in LDS (8192 records) and one that takes the radix sort sized for
    # the count, so counters one scan left behind would show in the next
    # one's records or in its work counters, which must equal the oracle
    # filter's.
    cases = [(4, 120_000, 40, 16, 3, 1, 4), (20, 90_001, 300, 16, 4, 1, 16), (64, 50_000, 80, 32, 4, 2, 16)]
    plans = []
    for sigma, n, r, m, q, k, sp in cases:
        T = gen_text(n, sigma, rng=n)
        P = gen_patterns(T, r, m, r // 2, sigma, rng=n + 1)
        plans.append((T, P, mag.Plan(P, q=q, k=k, sigma_prime=sp, mode="filter")))
    want = []
    for (sigma, n, r, m, q, k, sp), (T, P, plan) in zip(cases, plans):
        ref = om.occ_hashed(T, P)
        assert 0 < ref[0].size <= 8192
        want.append((ref, mm.Filter(P, q, k, sp).counts(T)))
    for rep in range(3):
        for (T, P, plan), (ref, cnt) in zip(plans, want):
            for cap in (8192, 1_000_000) if rep % 2 == 0 else (1_000_000, 8192):
                pos, ids, st = _gpu_occ(torch_cuda, mag, T, plan, offset=rep, out_cap=cap, stats=True)
                _assert_same(pos, ids, ref)
                assert st["matches"] == ref[0].size
                for key in ("samples", "cand_windows", "verifications"):
                    assert st[key] == cnt[key], (cap, key, st[key], cnt[key])


def test_overflow_reports_exact_count(torch_cuda, mag):
    T = gen_text(100_000, 4, rng=1)
    P = gen_patterns(T, 50, 8, 50, 4, rng=2)
    plan = mag.Plan(P)
    ref = om.occ_hashed(T, P)
    z = ref[0].size
    assert z > 10
    buf = torch_cuda.from_numpy(T).cuda()
    with pytest.raises(mag.MagError) as ei:
        mag.scan(buf, plan, out_cap=z - 1)
    assert ei.value.status == -5
    occ = mag.scan(buf, plan, out_cap=z).cpu().numpy()
    _assert_same(occ[:, 0].astype(np.uint64), occ[:, 1].astype(np.uint32), ref)


def test_empty_pattern_set_and_absent_byte(torch_cuda, mag):
    T = gen_text(10_000, 4, rng=1)
    buf = torch_cuda.from_numpy(T).cuda()
    assert mag.scan(buf, mag.Plan(np.zeros((0, 8), dtype=np.uint8))).shape[0] == 0
    P = np.frombuffer(b"ACGTACGN", dtype=np.uint8).reshape(1, 8)
    assert mag.scan(buf, mag.Plan(P)).shape[0] == 0


def test_async_entry_point(torch_cuda, mag):
    torch = torch_cuda
    T = gen_text(300_000, 20, rng=4)
    P = gen_patterns(T, 200, 16, 150, 20, rng=5)
    plan = mag.Plan(P)
    ref = om.occ_hashed(T, P)
    buf = torch.from_numpy(T).cuda()
    out = torch.empty((4096, 2), dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.zeros(7, dtype=torch.int64, device="cuda")
    for _ in range(3):                 # repeated calls reuse the plan's scratch
        mag.scan_async(buf, plan, out, cnt, st)
    torch.cuda.synchronize()
    z = int(cnt.item())
    assert z == ref[0].size
    occ = out[:z].cpu().numpy()
    _assert_same(occ[:, 0].astype(np.uint64), occ[:, 1].astype(np.uint32), ref)
    assert int(st[3].item()) == z
    # mag_stats after the four counters: q, k, sigma', m' (int32), plan_ms,
    # scan_ms (float32; 0 from the asynchronous entry point)
    info = plan.info()
    words = st.cpu().numpy().view(np.int32)
    assert list(words[8:12]) == [info["q"], info["k"], info["sigma_prime"], info["m_prime"]]
    floats = st.cpu().numpy().view(np.float32)
    assert floats[12] > 0 and floats[13] == 0
    # the synchronous entry point also times the scan
    _, sync = mag.scan(buf, plan, stats=True)
    assert (sync["q"], sync["k"], sync["sigma_prime"], sync["m_prime"]) == \
        (info["q"], info["k"], info["sigma_prime"], info["m_prime"])
    assert sync["matches"] == z and sync["scan_ms"] > 0 and sync["plan_ms"] == floats[12]


@pytest.mark.parametrize("sel", ["heuristic", "explicit-best"])
def test_dna1m_workload(torch_cuda, mag, sel):
    job = workload("dna1m")
    kw = {} if sel == "heuristic" else dict(q=8, k=1, sigma_prime=4)
    plan = mag.Plan(job.patterns, mode="filter", **kw)
    pos, ids, st = _gpu_occ(torch_cuda, mag, job.text, plan, stats=True)
    ref = om.occ_hashed(job.text, job.patterns)
    _assert_same(pos, ids, ref)
    info = plan.info()
    want = mm.Filter(job.patterns, info["q"], info["k"], info["sigma_prime"]).counts(job.text)
    assert (st["cand_windows"], st["verifications"]) == (want["cand_windows"], want["verifications"])


def test_zipf256m_full_size(torch_cuda, mag):
    job = workload("zipf256m")
    ref = om.occ_hashed(job.text, job.patterns)
    buf = torch_cuda.from_numpy(job.text).cuda()
    for kw in (dict(mode="filter"), dict(q=4, k=1, sigma_prime=16), dict(q=4, k=2, sigma_prime=16),
               dict(mode="dense")):
        plan = mag.Plan(job.patterns, **kw)
        occ = mag.scan(buf, plan).cpu().numpy()
        _assert_same(occ[:, 0].astype(np.uint64), occ[:, 1].astype(np.uint32), ref)
    # counters on a prefix the numpy oracle finishes quickly
    pre = job.text[: 1 << 21]
    plan = mag.Plan(job.patterns, mode="filter")
    pos, ids, st = _gpu_occ(torch_cuda, mag, pre, plan, stats=True)
    _assert_same(pos, ids, om.occ_hashed(pre, job.patterns))
    info = plan.info()
    want = mm.Filter(job.patterns, info["q"], info["k"], info["sigma_prime"]).counts(pre)
    assert (st["cand_windows"], st["verifications"]) == (want["cand_windows"], want["verifications"])


def test_zipf256m_benchmark_configuration(torch_cuda, mag):
    # The configuration the benchmark times, at full size: the learned
    # selector's pick (q=4, k=1, sigma'=16, bit-field map, whose 4-bit fields
    # take the nibble code path), enqueued with scan_async into an output of
    # 8192 records, the text resident on the device.
    torch = torch_cuda
    job = workload("zipf256m")
    ref = om.occ_hashed(job.text, job.patterns)
    buf = torch.from_numpy(job.text).cuda()
    pick = mag.Selector.load().picks([job.patterns])[0]
    for kw in (pick, dict(q=4, k=1, sigma_prime=16, map_kind="bits", mode="filter")):
        plan = mag.Plan(job.patterns, **kw)
        out = torch.empty((8192, 2), dtype=torch.int64, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        for _ in range(2):                      # a second scan on the same plan
            mag.scan_async(buf, plan, out, cnt)
            torch.cuda.synchronize()
            z = int(cnt.item())
            occ = out[:z].cpu().numpy()
            _assert_same(occ[:, 0].astype(np.uint64), occ[:, 1].astype(np.uint32), ref)


def test_prot1g_full_size(torch_cuda, mag):
    job = workload("prot1g")
    ref = om.occ_hashed(job.text, job.patterns)
    buf = torch_cuda.from_numpy(job.text).cuda()
    for kw in (dict(mode="filter"), dict(q=5, k=1, sigma_prime=20), dict(mode="dense"),
               dict(map_kind="qgram", mode="filter")):
        plan = mag.Plan(job.patterns, **kw)
        occ = mag.scan(buf, plan).cpu().numpy()
        _assert_same(occ[:, 0].astype(np.uint64), occ[:, 1].astype(np.uint32), ref)


def test_async_many_matches_device_sort(torch_cuda, mag):
    # the asynchronous entry point sorts large outputs without the host: its
    # radix kernels are sized for the capacity and read the count on the device.
    # Two scans in a row, the second with fewer occurrences than the first.
    torch = torch_cuda
    n, m = 60_000, 8
    T = np.full(n, ord("a"), dtype=np.uint8)
    T[::97] = ord("b")
    P = np.stack([np.full(m, ord("a"), dtype=np.uint8)] * 2 +
                 [np.frombuffer(b"aaabaaaa", dtype=np.uint8)])
    plan = mag.Plan(P, q=2, k=1, sigma_prime=2)
    ref = om.occ_hashed(T, P)
    assert ref[0].size > 20_000
    buf = torch.from_numpy(T).cuda()
    out = torch.empty((ref[0].size + 10, 2), dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    mag.scan_async(buf, plan, out, cnt)
    torch.cuda.synchronize()
    z = int(cnt.item())
    occ = out[:z].cpu().numpy()
    _assert_same(occ[:, 0].astype(np.uint64), occ[:, 1].astype(np.uint32), ref)
    T2 = T[: 40_003]
    ref2 = om.occ_hashed(T2, P)
    mag.scan_async(buf[: T2.size], plan, out, cnt)
    torch.cuda.synchronize()
    z = int(cnt.item())
    occ = out[:z].cpu().numpy()
    _assert_same(occ[:, 0].astype(np.uint64), occ[:, 1].astype(np.uint32), ref2)


def test_device_sort_chunk_sizes(torch_cuda, mag):
    # the device-wide sort cuts up to 2^20 keys into 1024-key chunks and more
    # into 4096-key ones: counts on both sides of that switch, through the
    # asynchronous entry point (sized for the capacity, so the second and
    # third scans reuse the first one's buffers) and the synchronous one
    torch = torch_cuda
    m = 8
    P = np.stack([np.full(m, ord("a"), dtype=np.uint8), np.frombuffer(b"aaaaaaab", dtype=np.uint8)])
    plan = mag.Plan(P, q=2, k=1, sigma_prime=2)
    T = np.full(1_050_383, ord("a"), dtype=np.uint8)   # 2^20 + 1 occurrences
    T[1000::4099] = ord("b")
    buf = torch.from_numpy(T).cuda()
    out = torch.empty(((1 << 20) + 16, 2), dtype=torch.int64, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    for n, zref in ((T.size, (1 << 20) + 1), (T.size - 1, 1 << 20), (700_003, None)):
        ref = om.occ_hashed(T[:n], P)
        assert zref is None or ref[0].size == zref
        mag.scan_async(buf[:n], plan, out, cnt)
        torch.cuda.synchronize()
        z = int(cnt.item())
        assert z == ref[0].size
        occ = out[:z].cpu().numpy()
        _assert_same(occ[:, 0].astype(np.uint64), occ[:, 1].astype(np.uint32), ref)
    occ = mag.scan(buf, plan).cpu().numpy()
    _assert_same(occ[:, 0].astype(np.uint64), occ[:, 1].astype(np.uint32), om.occ_hashed(T, P))


def test_autotune_pick_is_exact(torch_cuda, mag):
    job = make_job(3 << 20, 64, "zipf", 300, 32, 0.5, seed=21)
    buf = torch_cuda.from_numpy(job.text).cuda()
    best = mag.autotune(job.patterns, buf[: 1 << 20], max_candidates=12)
    assert 2 * best["q"] - 1 <= 32 and best["sample_ms"] > 0
    assert best["mode"] in ("filter", "dense")
    plan = mag.Plan(job.patterns, **{k: v for k, v in best.items() if k != "sample_ms"})
    occ = mag.scan(buf, plan).cpu().numpy()
    _assert_same(occ[:, 0].astype(np.uint64), occ[:, 1].astype(np.uint32),
                 om.occ_hashed(job.text, job.patterns))


@pytest.mark.parametrize("case", [
    # sigma, r, m, plan keywords (a filter plan's entries per lane or chunk, a
    # dense plan's positions per lane)
    (64, 300, 32, dict(q=4, k=1, sigma_prime=16, map_kind="bits", mode="filter", words_per_lane=16)),
    (64, 300, 32, dict(q=4, k=1, sigma_prime=16, map_kind="bits", mode="filter", words_per_lane=200)),
    (20, 200, 16, dict(q=3, k=2, sigma_prime=8, mode="filter", chunk_bytes=4096)),
    (4, 100, 16, dict(q=5, k=1, sigma_prime=4, mode="filter", words_per_lane=64)),
    (20, 5000, 16, dict(mode="dense", dense_probe="slices", words_per_lane=32)),
    (20, 5000, 12, dict(mode="dense", dense_probe="slices", chunk_bytes=40000)),
], ids=["filter-wpl16", "filter-wpl200", "filter-chunk4k", "dna-wpl64", "dense-wpl32", "dense-chunk"])
def test_tile_shapes(torch_cuda, mag, case):
    """Tile shapes other than the default (entries per lane of the filter
    kernel, positions per lane of the one-probe dense kernel): the same lists,
    at several text lengths and alignments."""
    sigma, r, m, kw = case
    T0 = gen_text(300_013, sigma, dist="zipf" if sigma == 64 else "uniform", rng=r + m)
    P = gen_patterns(T0, r, m, (3 * r) // 4, sigma, rng=r + 7)
    plan = mag.Plan(P, **kw)
    assert plan.params()["words_per_lane"] == kw.get("words_per_lane", 0)
    for npos in (1, 40_000, 64_513, 300_013 - m + 1):
        T = T0[:npos + m - 1]
        ref = om.occ_hashed(T, P)
        for off in (0, 3):
            pos, ids, _ = _gpu_occ(torch_cuda, mag, T, plan, offset=off)
            _assert_same(pos, ids, ref)


def test_dense_slice_tile_edges_32(torch_cuda, mag):
    # 32 positions per lane: tiles of 32,256 positions (16 waves of 63 owning
    # lanes); last starts around lane, wave and tile boundaries
    m, span, tile = 16, 32 * 63, 32 * 63 * 16
    T0 = gen_text(2 * tile + 128, 20, rng=97)
    at = [0, 31, 32, span - 33, span - 1, span, tile - 1, tile, tile + 1]
    P = np.concatenate([np.stack([T0[u:u + m] for u in at]), gen_patterns(T0, 3000, m, 0, 20, rng=98)])
    plan = mag.Plan(P, mode="dense", dense_probe="slices", words_per_lane=32)
    for npos in (1, 33, span - 1, span, span + 1, tile - 1, tile, tile + 1, 2 * tile + 64):
        T = T0[:npos + m - 1]
        ref = om.occ_hashed(T, P)
        for off in (0, 1, 2, 3):
            pos, ids, _ = _gpu_occ(torch_cuda, mag, T, plan, offset=off)
            _assert_same(pos, ids, ref)
