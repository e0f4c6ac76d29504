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
