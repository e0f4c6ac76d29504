"""Pins of the selector oracle (features, candidate grid, float64 MLP).

None of this is printed in the paper (it has no learned component), so the
pins are hand-computed small cases, closed forms, and central finite
differences of the loss.
"""

import math

import numpy as np
import pytest

from oracle import mlp, selector


def _pats(rows):
    return np.stack([np.frombuffer(r, dtype=np.uint8) for r in rows])


# ---------------------------------------------------------------- features

def test_features_hand_example():
    P = _pats([b"ACGT", b"ACGA"])
    f = selector.features(P)
    # byte counts A=3 C=2 G=2 T=1 over N=8
    H = -(3 / 8 * math.log2(3 / 8) + 2 * (1 / 4) * math.log2(1 / 4) + 1 / 8 * math.log2(1 / 8))
    want = np.zeros(16)
    want[0] = 2 / 8                      # log2(4) / 8
    want[1] = 4 / 32
    want[2] = math.log10(2) / 4
    want[3] = H / 8
    want[4] = 3 / 8
    want[5] = 1.0                        # both patterns distinct
    want[6] = 0.0                        # all 4 bytes seen: coverage 1
    want[7] = 2 / 32                     # {AC, CG, GT, GA}: 4 of 16
    want[8] = math.log2(64 / 3) / 32     # {ACG, CGT, CGA}: 3 of 64
    want[9] = math.log2(256 / 2) / 32    # 2 of 256
    want[10:14] = 1.0                    # q > m
    want[14] = 2 / 8                     # round(log_4(8)) = 2
    want[15] = math.log2(8) / 20
    assert np.allclose(f, want, rtol=0, atol=1e-12)


def test_features_duplicates_and_single_byte():
    P = _pats([b"aaaaaa"] * 3)
    f = selector.features(P)
    assert f[0] == 0.0 and f[3] == 0.0 and f[4] == 1.0
    assert abs(f[5] - 1 / 3) < 1e-15
    assert np.all(f[6:12] == 0.0)        # sigma_P = 1: every gram space is covered
    assert np.all(f[12:14] == 1.0)       # q = 7, 8 > m = 6


def test_distinct_substrings_brute_force():
    rng = np.random.default_rng(5)
    P = rng.integers(0, 3, size=(7, 9)).astype(np.uint8)
    for q in range(1, 10):
        grams = {tuple(P[i, s:s + q]) for i in range(7) for s in range(9 - q + 1)}
        assert selector.distinct_substrings(P, q) == len(grams)


# ------------------------------------------------------------ candidates

def test_candidates_dna_m8():
    P = _pats([b"ACGTACGT", b"TTGACCAG"])     # sigma_P = 4, m = 8
    c = selector.candidates(P)
    assert c[0] == ("dense", 0, 0, 0) and c[1] == ("qgram", 0, 0, 0)
    # choices 2..5: q = 2 with (k, level) = (1, 0), (1, 1), (2, 0), (2, 1)
    assert c[2] == ("filter", 2, 1, 4) and c[3] == ("filter", 2, 1, 2)   # 4^2 tiny
    assert c[4] == ("filter", 2, 2, 4)                       # L = 3, m' = 1, W = 2
    # choices 14..17: q = 5 (2q-1 = 9 > 8): infeasible; so is q = 8
    assert all(x is None for x in c[14:26])
    assert c[10] == ("filter", 4, 1, 4)                      # q = 4: L = 1
    assert c[12] is None                                     # q = 4, k = 2 > L
    assert c[26] == ("filter", 2, 3, 4)                      # k = 3 <= L = 3
    assert c[29] is None                                     # q = 2, k = 4 > L
    assert c[30] is None and c[31] is None                   # q = 7: 2q-1 = 13 > 8
    assert all(x is None for x in c[32:])                    # verification outputs


def test_candidates_protein_m16():
    rng = np.random.default_rng(1)
    P = rng.choice(np.frombuffer(b"ACDEFGHIKLMNPQRSTVWY", dtype=np.uint8), size=(200, 16))
    c = selector.candidates(P)
    assert c[10] == ("filter", 4, 1, 16)    # 16^4 = 65536 fits 64 KiB, 17^4 does not
    assert c[11] == ("filter", 4, 1, 8)
    assert c[28] == ("filter", 4, 3, 16)    # k = 3: m' = 1, W = 3
    assert c[22] == ("filter", 8, 1, 4)     # 4^8 = 65536
    assert c[23] == ("filter", 8, 1, 2)
    assert c[24] is None                    # q = 8, k = 2 > L = 1
    assert c[2] == ("filter", 2, 1, 20)     # 20^2 fits: the whole alphabet
    assert c[29] == ("filter", 2, 4, 20) and c[30] == ("filter", 7, 1, 4)
    assert c[0] == ("dense", 0, 0, 0) and c[1] == ("qgram", 0, 0, 0)
    # no patterns: the q-gram map has nothing to map
    assert selector.candidates(np.zeros((0, 16), np.uint8))[1] is None


def test_candidates_respect_budget_and_width():
    rng = np.random.default_rng(2)
    for m in (8, 16, 32):
        for sig in (2, 4, 20, 64):
            P = rng.integers(0, sig, size=(50, m)).astype(np.uint8)
            for c, t in enumerate(selector.candidates(P)):
                if t is None or t[0] != "filter":
                    continue
                _, q, k, sp = t
                L = (m - q + 1) // q
                W = k * min(L // k, 64 // k)
                e = 1 if W <= 8 else 2 if W <= 16 else 4
                assert 2 <= c < 32
                assert 2 * q - 1 <= m and 1 <= k <= L and 1 <= W <= 32
                assert sp ** q * e <= 64 * 1024 and sp <= max(len(np.unique(P)), 1)
                assert (q, k) == selector.grid_entry(c)[:2]


# -------------------------------------------------------------------- MLP

def _rand_params(seed):
    return mlp.init_params(np.random.default_rng(seed)) + \
        np.random.default_rng(seed + 1).normal(0, 0.05, mlp.param_count())


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(7)
    p = _rand_params(3)
    X = rng.random((5, 16))
    T = rng.normal(size=(5, 64))
    M = rng.random((5, 64)) < 0.3
    _, g = mlp.loss_and_grad(p, X, T, M)
    idx = np.concatenate([rng.choice(p.size, 300, replace=False), np.arange(p.size - 64, p.size)])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, T, M) - mlp.loss(p - e, X, T, M)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_zero_output_weights_closed_form():
    rng = np.random.default_rng(8)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(_rand_params(4))
    W3 = np.zeros_like(W3)
    b3 = rng.normal(size=64)
    p = mlp.pack(W1, b1, W2, b2, W3, b3)
    X = rng.random((6, 16))
    T = rng.normal(size=(6, 64))
    M = rng.random((6, 64)) < 0.5
    Y, _ = mlp.forward(p, X)
    assert np.array_equal(Y, np.broadcast_to(b3, (6, 64)))
    L, g = mlp.loss_and_grad(p, X, T, M)
    n = M.sum()
    assert abs(L - (M * (b3 - T) ** 2).sum() / n) < 1e-12
    gW1, gb1, gW2, gb2, gW3, gb3 = mlp.unpack(g)
    assert np.allclose(gb3, 2 * (M * (b3 - T)).sum(axis=0) / n, atol=1e-12)
    assert not gW1.any() and not gb1.any() and not gW2.any() and not gb2.any()


def test_forward_is_the_composed_linear_map_when_all_units_are_on():
    rng = np.random.default_rng(9)
    W1 = rng.random((64, 16))
    W2 = rng.random((64, 64))
    W3 = rng.normal(size=(64, 64))
    b1, b2, b3 = rng.random(64) + 1, rng.random(64) + 1, rng.normal(size=64)
    p = mlp.pack(W1, b1, W2, b2, W3, b3)
    X = rng.random((4, 16))               # nonnegative: every pre-activation is positive
    Y, _ = mlp.forward(p, X)
    for b in range(4):
        h1 = [b1[j] + sum(W1[j, i] * X[b, i] for i in range(16)) for j in range(64)]
        h2 = [b2[j] + sum(W2[j, i] * h1[i] for i in range(64)) for j in range(64)]
        y = [b3[c] + sum(W3[c, i] * h2[i] for i in range(64)) for c in range(64)]
        assert np.allclose(Y[b], y, rtol=1e-12)


def test_adam_first_step_is_a_signed_step():
    rng = np.random.default_rng(10)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    lr = 1e-3
    p1, m1, v1 = mlp.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr)
    # with zero moments the bias-corrected moments are g and g^2
    assert np.allclose(p1, p - lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_select_argmin_ties_and_infeasible():
    W1, b1, W2, b2, W3, b3 = mlp.unpack(np.zeros(mlp.param_count()))
    b3 = np.full(64, 5.0)
    b3[[3, 9, 40]] = [1.0, 1.0, 0.5]
    p = mlp.pack(W1, b1, W2, b2, W3, b3)
    F = np.zeros((3, 64), dtype=bool)
    F[0, [3, 9]] = True                   # tie: lowest index wins
    F[1, [3, 9, 40, 41]] = True
    pick = mlp.select(p, np.zeros((3, 16)), F)
    assert pick.tolist() == [3, 40, -1]
