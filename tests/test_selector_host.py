"""The library's selector features and candidate grid equal the oracle's
(host code; no GPU needed)."""

import numpy as np
import pytest

from oracle import selector as osel
from synth import gen_patterns, gen_text


@pytest.fixture(scope="module")
def mag():
    import paper_1405_5483_amd as m
    return m


def _sets():
    rng = np.random.default_rng(11)
    out = []
    for i in range(40):
        sigma = [2, 4, 20, 64, 200][i % 5]
        m = [1, 3, 8, 16, 32, 64][i % 6]
        r = int(rng.integers(1, 300))
        dist = "zipf" if i % 2 else "uniform"
        T = gen_text(5000, min(sigma, 64) if sigma != 200 else 64, dist, rng=i)
        if sigma == 200:
            T = rng.integers(0, 200, size=5000).astype(np.uint8)
        out.append(gen_patterns(T, r, m, r // 2, min(sigma, 64), rng=100 + i))
    out.append(np.frombuffer(b"ACGTACGA", dtype=np.uint8).reshape(2, 4))
    out.append(np.full((5, 7), 0x41, dtype=np.uint8))
    return out


def test_features_equal_oracle(mag):
    for P in _sets():
        f = mag.select_features(P)
        ref = osel.features(P)
        assert np.allclose(f, ref.astype(np.float32), rtol=1e-6, atol=1e-6), (P.shape, f, ref)


def test_candidates_equal_oracle(mag):
    for P in _sets():
        assert mag.select_candidates(P) == osel.candidates(P), P.shape


def test_features_reject_empty_set(mag):
    with pytest.raises(mag.MagError):
        mag.select_features(np.zeros((0, 8), dtype=np.uint8))
