"""Features and candidate grid of the learned parameter selector, written
plainly from their definitions.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``). The paper proposes
fixed formulas for q and k (Section 3.2) and an alphabet reduction to keep
sigma'^q tables small (Section 3.3); the selector replaces those formulas by
a learned cost model over a fixed grid of (q, k, sigma') triples. Nothing
here is printed in the paper ("parity unpinned" by the paper); the tests pin
it by brute force on small sets.

Features of a pattern set P (r patterns of length m, N = r m bytes, p_c the
frequency of byte c over all pattern bytes, sigma_P the number of distinct
bytes):

  f0  log2(sigma_P) / 8
  f1  m / 32
  f2  log10(r) / 4
  f3  byte entropy -sum p_c log2 p_c, / 8
  f4  max_c p_c
  f5  distinct patterns / r
  f6+q-1 for q = 1..8: D_q = number of distinct q-byte substrings over all
      patterns and offsets; coverage D_q / sigma_P^q of the q-gram space;
      f = min(1, -log2(coverage) / 32) (0 when sigma_P = 1), and 1 when q > m
  f14 min(q of Section 3.2's formula, 8) / 8 (the feature saturates at 8)
  f15 log2(N) / 20

Choices c (0..31), each returned as (kind, q, k, sigma'):
  0   ("dense", 0, 0, 0): every start position tested (always feasible);
  1   ("qgram", 0, 0, 0): the alphabet mapping on q-grams with its own
      heuristic (feasible when r > 0);
  2.. filter triples ("filter", q, k, sigma') with the greedy map:
      c = 2..25: i = c - 2, q = (2, 3, 4, 5, 6, 8)[i // 4], k = (i // 2) % 2 + 1,
      level = i % 2; 26..29: (q, k) = (2, 3), (3, 3), (4, 3), (2, 4), level 0;
      30, 31: q = 7, k = 1, levels 0 and 1.
Feasible iff 2q - 1 <= m, k <= L = (m - q + 1) // q and W = k m' <= 32 with
m' = min(L // k, 64 // k) >= 1. Entry bytes e(W) in {1, 2, 4}; "fit" is the
largest s <= sigma_P with s^q e(W) <= 64 KiB; level 0 takes sigma' = fit,
level 1 sigma' = max(2, fit // 2), infeasible when that equals fit.
The network has 64 outputs: 0..31 predict each choice's cost, 32..63 its
verifications per byte; slots 32..63 are never choices (None).
"""

from __future__ import annotations

import math

import numpy as np

from . import method

N_FEATURES = 16
N_CANDIDATES = 64       # network outputs
N_CHOICES = 32          # outputs that are choices (the rest predict verifications)
_QS = (2, 3, 4, 5, 6, 8)
_EXTRA = {26: (2, 3, 0), 27: (3, 3, 0), 28: (4, 3, 0), 29: (2, 4, 0), 30: (7, 1, 0), 31: (7, 1, 1)}
TABLE_BUDGET = 64 * 1024
MAX_W_BATCH = 32


def distinct_substrings(patterns: np.ndarray, q: int) -> int:
    p = np.asarray(patterns, dtype=np.uint8)
    r, m = p.shape
    if q > m or r == 0:
        return 0
    seen = set()
    for i in range(r):
        row = p[i].tobytes()
        for s in range(m - q + 1):
            seen.add(row[s:s + q])
    return len(seen)


def features(patterns: np.ndarray) -> np.ndarray:
    p = np.asarray(patterns, dtype=np.uint8)
    r, m = p.shape
    N = r * m
    hist = method.byte_histogram(p)
    sp = int((hist > 0).sum())
    f = np.zeros(N_FEATURES, dtype=np.float64)
    freq = hist[hist > 0] / N
    f[0] = math.log2(sp) / 8.0
    f[1] = m / 32.0
    f[2] = math.log10(r) / 4.0
    f[3] = float(-(freq * np.log2(freq)).sum()) / 8.0
    f[4] = float(freq.max())
    f[5] = len({p[i].tobytes() for i in range(r)}) / r
    for q in range(1, 9):
        if q > m:
            f[5 + q] = 1.0
        elif sp <= 1:
            f[5 + q] = 0.0
        else:
            lg_cov = math.log2(distinct_substrings(p, q)) - q * math.log2(sp)
            f[5 + q] = min(1.0, -lg_cov / 32.0)
    f[14] = min(method.heuristic_q(sp, r, m), 8) / 8.0
    f[15] = math.log2(N) / 20.0
    return f


def grid_entry(c: int):
    """(q, k, level) of filter choice c (2 <= c < 32)."""
    if c < 26:
        i = c - 2
        return _QS[i // 4], (i // 2) % 2 + 1, i % 2
    return _EXTRA[c]


def candidate(patterns: np.ndarray, c: int):
    """(kind, q, k, sigma') of choice c for this set, or None if infeasible."""
    p = np.asarray(patterns, dtype=np.uint8)
    r, m = p.shape
    if c >= N_CHOICES:
        return None
    if c == 0:
        return ("dense", 0, 0, 0)
    if c == 1:
        return ("qgram", 0, 0, 0) if r > 0 else None
    sp = max(method.sigma_p(p), 1)
    q, k, level = grid_entry(c)
    if 2 * q - 1 > m:
        return None
    L = (m - q + 1) // q
    if k > L:
        return None
    mprime = min(L // k, 64 // k)
    W = k * mprime
    if mprime < 1 or W > MAX_W_BATCH:
        return None
    e = 1 if W <= 8 else 2 if W <= 16 else 4
    fit = 1
    for s in range(1, min(sp, 256) + 1):
        if s ** q * e <= TABLE_BUDGET:
            fit = s
    if level == 0:
        return ("filter", q, k, fit)
    half = max(2, fit // 2)
    if half >= fit:
        return None
    return ("filter", q, k, half)


def candidates(patterns: np.ndarray):
    return [candidate(patterns, c) for c in range(N_CANDIDATES)]
