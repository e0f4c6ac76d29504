"""Pins for the matching oracle (the plain definition of Section 1).

The C matchers are checked against an independent pure-Python double loop
(exhaustively on tiny inputs), against closed forms and against planted
occurrences whose positions are known by construction.
"""

import itertools

import numpy as np
import pytest

from oracle import match as om
from synth import gen_text


def _pairs(res):
    pos, ids = res
    return list(zip(pos.tolist(), ids.tolist()))


def test_exhaustive_binary_tiny():
    # every text of length 7 over {a,b} against every pair of length-3 patterns
    alphabet = b"ab"
    texts = [bytes(t) for t in itertools.product(alphabet, repeat=7)]
    pats3 = [bytes(p) for p in itertools.product(alphabet, repeat=3)]
    for pa, pb in itertools.product(pats3, repeat=2):
        P = np.array([list(pa), list(pb)], dtype=np.uint8)
        for t in texts[::3]:
            T = np.frombuffer(t, dtype=np.uint8)
            ref = _pairs(om.occ_python(T, P))
            assert _pairs(om.occ_brute(T, P)) == ref
            assert _pairs(om.occ_hashed(T, P, threads=3)) == ref


@pytest.mark.parametrize("seed", range(12))
def test_random_small_against_python(seed):
    rng = np.random.default_rng(seed)
    sigma = int(rng.choice([2, 3, 4, 20]))
    n = int(rng.integers(0, 400))
    m = int(rng.integers(1, 7))
    r = int(rng.integers(1, 12))
    T = (rng.integers(0, sigma, size=n) + 65).astype(np.uint8)
    P = (rng.integers(0, sigma, size=(r, m)) + 65).astype(np.uint8)
    if n >= m and r > 2:
        for row in range(r // 2):          # half the patterns come from the text
            u = int(rng.integers(0, n - m + 1))
            P[row] = T[u:u + m]
    ref = _pairs(om.occ_python(T, P))
    assert _pairs(om.occ_brute(T, P)) == ref
    for th in (1, 2, 5):
        assert _pairs(om.occ_hashed(T, P, threads=th)) == ref


def test_run_closed_form_with_duplicates():
    # a^n against {a^m} repeated d times: every start 0..n-m, every id
    n, m, d = 1000, 7, 3
    T = np.full(n, ord("a"), dtype=np.uint8)
    P = np.full((d, m), ord("a"), dtype=np.uint8)
    pos, ids = om.occ_hashed(T, P, threads=4)
    assert pos.size == (n - m + 1) * d
    assert np.array_equal(pos, np.repeat(np.arange(n - m + 1), d))
    assert np.array_equal(ids, np.tile(np.arange(d), n - m + 1))


def test_absent_byte_gives_no_match():
    T = gen_text(50_000, 4, rng=7)                  # ACGT only
    P = np.frombuffer(b"ACGTACGN", dtype=np.uint8).reshape(1, 8)
    pos, _ = om.occ_hashed(T, P)
    assert pos.size == 0


def test_planted_occurrences():
    # text over lowercase a..t, patterns over uppercase: occurrences are the
    # planted copies and nothing else
    rng = np.random.default_rng(11)
    n, m, r = 200_000, 16, 50
    T = (rng.integers(0, 20, size=n) + ord("a")).astype(np.uint8)
    P = (rng.integers(0, 20, size=(r, m)) + ord("A")).astype(np.uint8)
    starts = np.sort(rng.choice(np.arange(0, n - m, m), size=300, replace=False))
    which = rng.integers(0, r, size=starts.size)
    for s, w in zip(starts, which):
        T[s:s + m] = P[w]
    pos, ids = om.occ_hashed(T, P, threads=4)
    assert np.array_equal(pos, starts.astype(np.uint64))
    assert np.array_equal(ids, which.astype(np.uint32))


def test_edge_sizes():
    P = np.frombuffer(b"abc", dtype=np.uint8).reshape(1, 3)
    for t in (b"", b"ab", b"abc", b"abcabc"):
        T = np.frombuffer(t, dtype=np.uint8)
        assert _pairs(om.occ_hashed(T, P)) == _pairs(om.occ_python(T, P))
    assert _pairs(om.occ_hashed(np.frombuffer(b"abc", dtype=np.uint8), P)) == [(0, 0)]


def test_all_byte_values():
    T = np.arange(256, dtype=np.uint8).repeat(3)
    P = np.array([[0, 0, 0, 1], [255, 255, 255, 0], [127, 128, 128, 128]], dtype=np.uint8)
    assert _pairs(om.occ_hashed(T, P)) == _pairs(om.occ_python(T, P))
    assert _pairs(om.occ_hashed(T, P)) == [(0, 0), (383, 2)]


def test_occ_at_matches_list():
    T = gen_text(5000, 4, rng=3)
    rng = np.random.default_rng(3)
    P = np.stack([T[u:u + 6] for u in rng.integers(0, 4994, size=30)])
    pos, ids = om.occ_hashed(T, P)
    for i in range(0, 4995, 7):
        assert om.occ_at(T, P, i).tolist() == ids[pos == i].tolist()


# ------------------------------------------------- unequal pattern lengths

def _var_set(rng, text, r, lens, planted):
    pats = []
    for i in range(r):
        L = int(rng.choice(lens))
        if i < planted and text.size >= L:
            u = int(rng.integers(0, text.size - L + 1))
            pats.append(bytes(text[u:u + L]))
        else:
            pats.append(bytes(rng.integers(0, 4, L, dtype=np.uint8) + ord("A")))
    return pats


@pytest.mark.parametrize("seed", range(12))
def test_occ_var_equals_python_double_loop(seed):
    rng = np.random.default_rng(700 + seed)
    T = (rng.integers(0, 4, int(rng.integers(0, 400)), dtype=np.uint8) + ord("A"))
    pats = _var_set(rng, T, int(rng.integers(1, 12)), [1, 2, 3, 5, 8], 6)
    if rng.random() < 0.5 and pats:
        pats.append(pats[0])                      # a duplicate
        pats.append(pats[0] + b"A")               # an extension of another pattern
    want = om.occ_var_python(T, pats)
    got = om.occ_var(T, pats)
    assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])


def test_occ_var_nested_patterns_closed_form():
    # text a^n; patterns a^1 .. a^5: a^L occurs at every i <= n-L
    n = 50
    T = np.full(n, ord("a"), dtype=np.uint8)
    pats = [b"a" * L for L in (3, 1, 5, 2, 4)]
    pos, ids = om.occ_var(T, pats)
    expect = sorted((i, pid) for pid, p in enumerate(pats) for i in range(n - len(p) + 1))
    assert list(zip(pos.tolist(), ids.tolist())) == expect


def test_occ_var_equal_lengths_reduce_to_occ_hashed():
    rng = np.random.default_rng(9)
    T = rng.integers(0, 4, 5000, dtype=np.uint8)
    P = np.stack([T[u:u + 8] for u in rng.integers(0, 4990, 20)])
    a = om.occ_var(T, [bytes(row) for row in P])
    b = om.occ_hashed(T, P)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_prefix_filter_never_drops_a_match():
    from oracle import method as mm
    rng = np.random.default_rng(10)
    T = rng.integers(0, 4, 20_000, dtype=np.uint8) + ord("A")
    pats = _var_set(rng, T, 40, [9, 12, 16, 23], 30)
    pre = mm.prefix_set(pats)
    assert pre.shape == (40, 9)
    f = mm.Filter(pre, 3, 2, 4)
    starts = set(f.verification_starts(T).tolist())
    pos, _ = om.occ_var(T, pats)
    assert pos.size > 0 and set(pos.tolist()) <= starts
