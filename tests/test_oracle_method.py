"""Pins for the filter oracle (``oracle.method``).

Each object is tied to something other than its own definition: the worked
examples and printed numbers of Section 2, a bit-by-bit Shift-Or simulation
(the automaton of Section 3) against the closed-form window predicate, brute
force occurrence sets (the filter must never drop a true match), the q = 1
special case that reduces to the plain superimposed filter of Section 2, the
degenerate sigma' = 1 case that must verify every start exactly once, and
Graham's bound for the greedy bin packing.
"""

import itertools
import math
import json
import os

import numpy as np
import pytest

from oracle import match as om
from oracle import method as mm
from synth import gen_patterns, gen_text

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def _b(s):
    return np.frombuffer(s.encode(), dtype=np.uint8)


# --------------------------------------------------------- worked examples

def test_superimposition_example():
    g = GOLD["superimposition"]
    rows = [list(p) for p in g["patterns"]]
    cls = mm.superimpose(rows)
    assert [sorted(c) for c in cls] == [sorted(c) for c in g["classes"]]
    assert int(np.prod([len(c) for c in cls])) == g["matching_strings"]


def test_superimposition_example_through_classes():
    # the same example through the q-gram class builder with q = 1 and an
    # identity alphabet map
    g = GOLD["superimposition"]
    P = np.stack([_b(p) for p in g["patterns"]])
    mu = np.arange(256, dtype=np.int64)
    cls = mm.classes(P, mu, 256, 1, 4)
    assert [sorted(chr(c) for c in cl) for cl in cls] == [sorted(c) for c in g["classes"]]


def test_overlapping_q2_example():
    g = GOLD["overlapping_q2"]
    fac = [[x.decode() for x in mm.overlapping_grams(p.encode(), g["q"])] for p in g["patterns"]]
    assert fac == g["factored"]
    assert [sorted(c) for c in mm.superimpose(fac)] == [sorted(c) for c in g["classes"]]


def test_nonoverlapping_q2_example():
    g = GOLD["nonoverlapping_q2"]
    fac = [[x.decode() for x in mm.nonoverlapping_grams(p.encode(), g["q"], 0)] for p in g["patterns"]]
    assert [sorted(c) for c in mm.superimpose(fac)] == [sorted(c) for c in g["classes"]]


def test_nonoverlapping_all_shifts_through_codes():
    # Our reading (all q shifts, common length L = (m-q+1)//q): for {abba, bbac}
    # and q = 2, L = 1 and C[0] holds shift-0 grams {ab, bb} and shift-1 grams
    # {bb, ba}.
    P = np.stack([_b("abba"), _b("bbac")])
    mu = np.arange(256, dtype=np.int64)
    cls = mm.classes(P, mu, 256, 2, mm.gram_positions(4, 2))
    decoded = sorted(chr(c % 256) + chr(c // 256) for c in cls[0])
    assert decoded == ["ab", "ba", "bb"]


def test_class_density_numbers():
    g = GOLD["class_density"]
    for case in g["cases"]:
        alphabet = g["sigma"] ** case["q"]
        p = mm.class_hit_probability(alphabet, case["r"])
        assert abs(p - case["probability"]) <= case["probability_tol"] + (
            0.01 if case["relation"] == "over" else 0.0)
        if case["relation"] == "over":
            assert p > case["probability"]
        if "class_size" in case:
            size = mm.expected_class_size(alphabet, case["r"])
            assert abs(size - case["class_size"]) <= case["class_size_tol"] + (
                0.1 if case["relation"] == "over" else 0.0)
            if case["relation"] == "over":
                assert size > case["class_size"]


def test_class_density_by_simulation():
    # the closed form against a direct Monte Carlo of superimposing r random
    # symbols and hitting the union with another random symbol
    rng = np.random.default_rng(0)
    for alphabet, r in ((16, 16), (16, 64), (256, 16)):
        trials = 20000
        draws = rng.integers(0, alphabet, size=(trials, r))
        probe = rng.integers(0, alphabet, size=trials)
        hit = (draws == probe[:, None]).any(axis=1).mean()
        assert abs(hit - mm.class_hit_probability(alphabet, r)) < 0.015


# ------------------------------------------------------------- alphabet maps

def test_rank_map_orders_by_frequency():
    # counts e=5, x=5, d=4, c=3, b=2, a=1 (ties by byte value: e before x)
    P = np.stack([_b("eeeeeddddc"), _b("ccbbaxxxxx")])
    mu = mm.map_rank(P, 3)
    want3 = {"e": 0, "x": 1, "d": 2, "c": 2, "b": 2, "a": 2, "Q": 2}
    assert {ch: int(mu[ord(ch)]) for ch in want3} == want3
    mu7 = mm.map_rank(P, 7)
    want7 = {"e": 0, "x": 1, "d": 2, "c": 3, "b": 4, "a": 5, "Q": 6}
    assert {ch: int(mu7[ord(ch)]) for ch in want7} == want7


def _best_makespan(weights, bins):
    best = None
    for assign in itertools.product(range(bins), repeat=len(weights)):
        loads = [0] * bins
        for w, b in zip(weights, assign):
            loads[b] += w
        mk = max(loads)
        best = mk if best is None else min(best, mk)
    return best


@pytest.mark.parametrize("seed", range(25))
def test_greedy_map_lpt_bound(seed):
    # Graham: LPT makespan <= (4/3 - 1/(3 bins)) * optimum
    rng = np.random.default_rng(seed)
    nsym = int(rng.integers(2, 8))
    bins = int(rng.integers(2, 4))
    counts = rng.integers(1, 30, size=nsym)
    pat = np.concatenate([np.full(c, 65 + i, dtype=np.uint8) for i, c in enumerate(counts)])
    P = pat.reshape(1, -1)
    mu = mm.map_greedy(P, bins)
    loads = np.zeros(bins, dtype=np.int64)
    for i, c in enumerate(counts):
        loads[mu[65 + i]] += c
    assert loads.sum() == counts.sum()
    opt = _best_makespan(list(counts), bins)
    assert loads.max() <= (4 / 3 - 1 / (3 * bins)) * opt + 1e-9
    assert mu[0] == bins - 1                        # absent byte -> last bin


def test_greedy_map_even_split():
    # weights 4,4,2,2,2,2 into 2 bins: LPT reaches the perfect 8/8 split
    P = np.stack([_b("aaaabbbbccddeeff")])
    mu = mm.map_greedy(P, 2)
    loads = [0, 0]
    for ch, w in zip("abcdef", (4, 4, 2, 2, 2, 2)):
        loads[mu[ord(ch)]] += w
    assert loads == [8, 8]


# ------------------------------------------------------ Shift-Or simulation

def _shift_or_candidates(f: mm.Filter, text: np.ndarray) -> np.ndarray:
    """The bit-parallel automaton run sample by sample in plain Python ints:
    D <- (D << k) | B[g], D starting at all ones; window (x, j) fires when bit
    (m'-1)k + j of D is 0."""
    B = f.table()
    g = f.sample_codes(text)
    k, mp = f.k, f.mprime
    full = (1 << 64) - 1
    D = full
    out = np.zeros((g.size, k), dtype=bool)
    for x in range(g.size):
        D = ((D << k) | int(B[g[x]])) & full
        for j in range(k):
            out[x, j] = ((D >> ((mp - 1) * k + j)) & 1) == 0
    return out


CASES = [
    # sigma, n, r, m, q, k, sigma', kind
    (4, 3000, 6, 8, 2, 1, 4, "greedy"),
    (4, 3000, 6, 8, 2, 2, 3, "rank"),
    (4, 4000, 30, 16, 3, 2, 4, "greedy"),
    (20, 3000, 12, 16, 3, 4, 7, "greedy"),
    (20, 3000, 40, 16, 1, 5, 20, "rank"),
    (64, 3000, 20, 32, 2, 3, 16, "greedy"),
    (2, 2000, 5, 9, 5, 1, 2, "greedy"),
    (4, 2000, 8, 12, 4, 1, 1, "greedy"),
    (20, 3000, 30, 16, 8, 1, 1 << 12, "qgram"),     # q-gram map, W = 1
    (4, 3000, 10, 16, 5, 1, 1 << 10, "qgram"),      # W = 2
    (64, 3000, 20, 32, 6, 2, 1 << 9, "qgram"),      # W = 4
    (64, 3000, 20, 32, 3, 3, 1 << 6, "qgram"),      # W = 9: whole-byte entries
    (20, 2000, 12, 16, 4, 1, 2, "qgram"),
]


@pytest.mark.parametrize("case", CASES)
def test_candidates_equal_shift_or(case):
    sigma, n, r, m, q, k, sp, kind = case
    T = gen_text(n, sigma, rng=sigma * 7 + n)
    P = gen_patterns(T, r, m, r // 2, sigma, rng=r)
    f = mm.Filter(P, q, k, sp, kind)
    assert np.array_equal(f.candidates(T), _shift_or_candidates(f, T))


@pytest.mark.parametrize("case", CASES)
def test_filter_never_drops_a_match(case):
    sigma, n, r, m, q, k, sp, kind = case
    T = gen_text(n, sigma, rng=sigma + n)
    P = gen_patterns(T, r, m, (3 * r) // 4, sigma, rng=r + 1)
    f = mm.Filter(P, q, k, sp, kind)
    starts = f.verification_starts(T)
    assert np.unique(starts).size == starts.size        # each start verified once
    pos, _ = om.occ_brute(T, P)
    assert pos.size > 0
    assert np.isin(pos.astype(np.int64), starts).all()


@pytest.mark.parametrize("n", [0, 1, 7, 8, 9, 15, 16, 17, 31, 100, 257])
@pytest.mark.parametrize("qk", [(1, 1), (1, 3), (2, 1), (2, 3), (3, 2), (4, 1)])
def test_sigma1_verifies_every_start_once(n, qk):
    # with sigma' = 1 every window passes, so the verification starts must be
    # exactly 0..n-m, each once: this pins the (x, j, s) -> i0 arithmetic
    q, k = qk
    m = 16
    P = np.frombuffer(b"ABCDEFGHIJKLMNOP", dtype=np.uint8).reshape(1, m)
    f = mm.Filter(P, q, k, 1)
    T = gen_text(n, 4, rng=n)
    starts = f.verification_starts(T)
    expect = np.arange(max(n - m + 1, 0))
    assert np.array_equal(starts, expect)


def test_q1_k1_is_plain_superimposed_filter():
    # q = 1, k = 1 with an injective map: window x fires iff the text window
    # starting at x-m+1 matches the superimposed pattern of Section 2
    sigma, n, r, m = 4, 5000, 3, 6
    T = gen_text(n, sigma, rng=5)
    P = gen_patterns(T, r, m, 2, sigma, rng=6)
    sp = mm.sigma_p(P) + 1                       # absent bytes get their own code
    f = mm.Filter(P, 1, 1, sp, "greedy")
    cls = mm.superimpose([list(row) for row in P])
    direct = np.array([all(T[i + b] in cls[b] for b in range(m)) for i in range(n - m + 1)])
    cand = f.candidates(T)[:, 0]
    assert np.array_equal(cand[m - 1:], direct)
    assert not cand[:m - 1].any()


def test_candidate_rate_statistics():
    # sanity: on uniform data the window rate is near the analysis of Section 3.2
    sigma, n, r, m, q, k = 4, 400_000, 20, 16, 3, 1
    T = gen_text(n, sigma, rng=9)
    P = gen_patterns(T, r, m, 0, sigma, rng=10)
    f = mm.Filter(P, q, k, 4)
    cnt = f.counts(T)
    occ = np.mean([len(c) / f.n_codes for c in f.C])
    expect = occ ** f.mprime
    assert abs(cnt["cand_windows"] / cnt["samples"] - expect) < 0.25 * expect + 1e-3


# ----------------------------------------------------------- heuristic

def test_heuristic_invariants():
    for sigma, r, m in ((4, 100, 16), (64, 1000, 32), (20, 100_000, 16), (4, 10, 8),
                        (20, 10_000, 8), (64, 10, 32), (2, 50, 5)):
        T = gen_text(20_000, sigma, rng=r)
        P = gen_patterns(T, r, m, r // 2, sigma, rng=m)
        q, k, sp = mm.heuristic_params(P)
        L = mm.gram_positions(m, q)
        assert 1 <= q and 2 * q - 1 <= m and 1 <= k <= L
        W = k * mm.sub_pattern_length(L, k)
        assert sp == 1 or sp ** q * mm.entry_bytes(W) <= mm.DEFAULT_TABLE_BUDGET
        assert sp <= mm.sigma_p(P)


def test_heuristic_values_for_workloads():
    # Parity unpinned by the paper (it prints no parameter values). These are
    # the values our stated readings give for the three single-job workloads.
    from synth import workload
    expect = {"dna1m": (5, 1, 4), "zipf256m": (2, 3, 64), "prot1g": (5, 1, 9)}
    for name, want in expect.items():
        job = workload(name, n=1 << 20)
        assert mm.heuristic_params(job.patterns) == want, name


# ------------------------------------------------- bit-field alphabet map

def test_bits_map_matches_the_papers_dna_multiply_formula():
    """Section 3.3 computes DNA 4-gram codes as
    (((x >> 1) & 0x03030303) * 0x40100401) >> 24 with the first character in
    the high bits. For ACGT patterns the bit-field map picks the same shift
    (1), and our code is that value with its four 2-bit digits reversed."""
    P = np.frombuffer(b"ACGTTGCAACGGTTCA", dtype=np.uint8).reshape(2, 8)
    assert mm.bits_shift(P, 4) == 1
    mu = mm.map_bits(P, 4)
    for g in itertools.product(b"ACGTacgt", repeat=4):
        x = g[0] | g[1] << 8 | g[2] << 16 | g[3] << 24
        paper = ((((x >> 1) & 0x03030303) * 0x40100401) & 0xFFFFFFFF) >> 24
        rev = sum(((paper >> (2 * (3 - t))) & 3) << (2 * t) for t in range(4))
        assert mm.gram_code(bytes(g), mu, 4) == rev


def test_bits_map_low_nibbles():
    P = np.frombuffer(bytes(range(0x30, 0x70)), dtype=np.uint8).reshape(4, 16)
    # every byte 0x30..0x6F once: the low nibble spreads them evenly (4 per code)
    assert mm.bits_shift(P, 16) == 0
    mu = mm.map_bits(P, 16)
    assert [int(mu[c]) for c in (0x30, 0x4F, 0x6A)] == [0, 15, 10]
    assert mm.gram_code(bytes([0x31, 0x32]), mu, 16) == 1 + 2 * 16


# ------------------------------------------------ alphabet mapping on q-grams

def _unxorshift33(y):
    # x ^ (x >> 33) keeps the top 33 bits, so applying it again restores x
    return y ^ (y >> 33)


def test_fmix64_is_a_bijection():
    # invert each step from the mathematics: odd multipliers have inverses
    # modulo 2^64 and the 33-bit xor-shift is its own inverse
    inv1 = pow(mm.FMIX_C1, -1, 1 << 64)
    inv2 = pow(mm.FMIX_C2, -1, 1 << 64)
    rng = np.random.default_rng(11)
    for x in [0, 1, 2, (1 << 64) - 1, 1 << 63] + [int(v) for v in rng.integers(0, 1 << 63, 500)]:
        y = mm.fmix64(x)
        y = _unxorshift33(y)
        y = (y * inv2) % (1 << 64)
        y = _unxorshift33(y)
        y = (y * inv1) % (1 << 64)
        assert _unxorshift33(y) == x
    assert mm.FMIX_C1 % 2 == 1 and mm.FMIX_C2 % 2 == 1


def test_fmix64_avalanche():
    # the finalizer's purpose: flipping any input bit flips every output bit
    # with probability near 1/2 (a dropped or mistyped step breaks this)
    rng = np.random.default_rng(12)
    keys = [int(v) for v in rng.integers(0, 1 << 63, 4000, dtype=np.int64)]
    keys = [k | (int(rng.integers(0, 2)) << 63) for k in keys]
    flips = np.zeros((64, 64))
    for k in keys:
        h = mm.fmix64(k)
        for i in range(64):
            d = h ^ mm.fmix64(k ^ (1 << i))
            flips[i] += [(d >> j) & 1 for j in range(64)]
    bias = np.abs(flips / len(keys) - 0.5)
    assert bias.max() < 0.04, bias.max()


def test_qgram_codes_vectorized_equal_scalar():
    rng = np.random.default_rng(13)
    for q in range(1, 9):
        g = rng.integers(0, 256, (300, q), dtype=np.uint8)
        for b in (0, 1, 7, 16, 28):
            want = [mm.qgram_code(row, b) for row in g]
            assert mm.qgram_codes(g, b).tolist() == want
    assert mm.gram_key(b"\x01\x02") == 0x0201


def test_qgram_class_occupancy_is_balls_in_bins():
    # D distinct grams hashed into sigma' codes occupy sigma'(1-(1-1/sigma')^D)
    # codes on average (variance below the mean)
    T = gen_text(200_000, 20, rng=14)
    P = gen_patterns(T, 2000, 16, 1000, 20, rng=15)
    for b in (10, 12, 14):
        f = mm.Filter(P, 8, 1, 1 << b, "qgram")
        D = len(mm.class_grams(P, 8, 1)[0])
        sp = 1 << b
        expect = sp * (1 - (1 - 1 / sp) ** D)
        got = len(f.C[0])
        assert abs(got - expect) < 4 * math.sqrt(expect) + 2, (b, got, expect)
        assert max(f.C[0]) < sp


def test_qgram_candidate_rate():
    # uniform text over 20 symbols with q = 8: text grams almost never equal a
    # pattern gram, so a sample passes with probability |C[0]| / sigma'
    T = gen_text(300_000, 20, rng=16)
    P = gen_patterns(gen_text(50_000, 20, rng=17), 500, 16, 500, 20, rng=18)
    f = mm.Filter(P, 8, 1, 1 << 14, "qgram")
    cnt = f.counts(T)
    rate = cnt["cand_windows"] / cnt["samples"]
    expect = len(f.C[0]) / f.n_codes
    assert abs(rate - expect) < 5 * math.sqrt(expect / cnt["samples"]) + 1e-3, (rate, expect)


def test_qgram_heuristic_hand_counted():
    """heuristic_params_qgram on sets whose classes are counted by hand.

    * {abcabcab, abcdabcd}, m = 8: q = min(8, (8+1)//2) = 4, L = (8-4+1)//4 = 1,
      k = 1, m' = 1, W = 1 (1-bit entries). Class 0 holds the grams at
      offsets s = 0..3: abca, bcab, cabc, abca from the first pattern (3
      distinct) and abcd, bcda, cdab, dabc from the second (4), so D = 7.
      sigma' = the smallest power of two >= 32 * 7 = 224, i.e. 256: a
      256-bit table. A 16-byte budget (128 bits) halves it once to 128; an
      8-byte budget twice, to 64.
    * {a^24}, m = 24: q = 8, L = (24-8+1)//8 = 2, W = 2 (2-bit entries). Every
      gram is aaaaaaaa, so D = 1 and sigma' = 32 (64 bits); a 4-byte budget
      (32 bits) halves it to 16.
    * {(ab)^12}, m = 24: q = 8, W = 2. Class b holds, over s = 0..7, the
      grams at offsets s + 8b: abababab for even s and babababa for odd s,
      so D = 2 and sigma' = 64.
    """
    two = np.frombuffer(b"abcabcababcdabcd", dtype=np.uint8).reshape(2, 8)
    assert mm.heuristic_params_qgram(two) == (4, 1, 256)
    assert mm.heuristic_params_qgram(two, table_budget=16) == (4, 1, 128)
    assert mm.heuristic_params_qgram(two, table_budget=8) == (4, 1, 64)
    a24 = np.frombuffer(b"a" * 24, dtype=np.uint8).reshape(1, 24)
    assert mm.heuristic_params_qgram(a24) == (8, 1, 32)
    assert mm.heuristic_params_qgram(a24, table_budget=4) == (8, 1, 16)
    ab = np.frombuffer(b"ab" * 12, dtype=np.uint8).reshape(1, 24)
    assert mm.heuristic_params_qgram(ab) == (8, 1, 64)


def test_heuristic_q_formula_hand_computed():
    """Section 3.2's q = round(log_sigma(r m)), clamped to [1, (m+1)//2] only:
    sigma = 4, r = 4096, m = 32 gives log_4(131072) = 8.5 -> 9 (above the
    "2..6 in practice" of Section 2, and allowed); sigma = 4, r = 100,
    m = 16: log_4(1600) = 5.32 -> 5; sigma = 2, r = 1000, m = 8:
    log_2(8000) = 12.97 -> 13, clamped to (8+1)//2 = 4; sigma = 20,
    r = 10^5, m = 16: log_20(1.6e6) = 4.76 -> 5."""
    assert mm.heuristic_q(4, 4096, 32) == 9
    assert mm.heuristic_q(4, 100, 16) == 5
    assert mm.heuristic_q(2, 1000, 8) == 4
    assert mm.heuristic_q(20, 100_000, 16) == 5
    # the cap is only applied on request
    P = np.frombuffer(b"ACGT" * 8, dtype=np.uint8).reshape(1, 32).repeat(4096, axis=0)
    P = P.copy()
    P[:, 0] = np.frombuffer(b"ACGT", dtype=np.uint8)[np.arange(4096) % 4]
    q, k, sp = mm.heuristic_params(P)
    assert q == 9
    assert mm.heuristic_params(P, q_cap=8)[0] == 8


def test_qgram_heuristic_invariants():
    for sigma, r, m in ((4, 100, 16), (64, 1000, 32), (20, 3000, 16), (20, 50, 8), (2, 20, 5)):
        T = gen_text(30_000, sigma, rng=r)
        P = gen_patterns(T, r, m, r // 2, sigma, rng=m)
        q, k, sp = mm.heuristic_params_qgram(P)
        assert q == min(8, (m + 1) // 2) and k == 1
        f = mm.Filter(P, q, k, sp, "qgram")
        D = max(len(c) for c in mm.class_grams(P, q, f.W))
        assert sp & (sp - 1) == 0
        eb = mm.entry_bits(f.W, "qgram")
        assert sp * eb <= 8 * mm.QGRAM_TABLE_BUDGET
        assert sp >= mm.QGRAM_LOAD * D or 2 * sp * eb > 8 * mm.QGRAM_TABLE_BUDGET
        assert sp == 2 or sp < 2 * mm.QGRAM_LOAD * D


# ------------------------------------------------------ SMAG: encoded text

@pytest.mark.parametrize("kind", ["greedy", "rank", "bits", "qgram"])
def test_encoded_text_digits_are_the_mapped_bytes(kind):
    # decode every code: for the per-byte maps its base-sigma' digits, least
    # significant first, must be mu of the gram's bytes; for the q-gram map
    # each code must equal the scalar hash of its gram
    T = gen_text(3001, 20, rng=31)
    P = gen_patterns(T, 30, 16, 20, 20, rng=32)
    q, sp = 3, (8 if kind == "bits" else 1 << 12 if kind == "qgram" else 7)
    f = mm.Filter(P, q, 1, sp, kind)
    codes = f.encode(T)
    assert codes.size == (T.size - q) // q + 1
    for y in range(0, codes.size, 37):
        gram = T[y * q:y * q + q]
        if kind == "qgram":
            assert codes[y] == mm.qgram_code(gram, 12)
        else:
            c = int(codes[y])
            digits = [(c // sp ** t) % sp for t in range(q)]
            assert digits == [int(f.mu[b]) for b in gram]


def test_encoded_text_holds_the_filter_samples():
    # sample x of the sampled filter (byte x*k*q) is entry x*k of the encoded text
    T = gen_text(5000, 4, rng=33)
    P = gen_patterns(T, 10, 16, 5, 4, rng=34)
    for q, k in ((2, 3), (4, 2), (5, 1)):
        f = mm.Filter(P, q, k, 4)
        enc = f.encode(T)
        assert np.array_equal(f.sample_codes(T), enc[::k][: f.n_samples(T.size)])
    assert mm.Filter(P, 4, 1, 4).encode(T[:3]).size == 0
