"""Seeded synthetic texts and pattern sets for the multiple-pattern-matching scan.

This module only draws random bytes. It holds none of the matching method's
arithmetic, so both the CPU oracle and the HIP path can consume its arrays
without sharing any code with each other.

The paper measures on the Pizza&Chili ``dna``, ``english`` and ``proteins``
corpora (Section 4). They are not available here, so texts are drawn i.i.d.:
uniform over 4 symbols stands in for ``dna``, uniform over the 20 amino-acid
letters for ``proteins``, and Zipf(s) over 64 symbols for the skewed
``english`` distribution.

Recipes
-------
* symbol tables: sigma=4 ``b"ACGT"``, sigma=20 ``b"ACDEFGHIKLMNPQRSTVWY"``,
  sigma=64 the bytes 0x30..0x6F;
* Zipf(s): P(rank i) proportional to i**-s, rank i being the i-th symbol of
  the table (1-based);
* "sampled" patterns copy ``T[u:u+m]`` with ``u`` uniform in ``[0, n-m]``,
  drawn with replacement; "uniform" patterns draw i.i.d. uniform symbols;
  pattern ids run sampled first, then uniform;
* every draw uses ``numpy.random.Generator(PCG64(seed))``.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SYMBOLS = {
    4: b"ACGT",
    20: b"ACDEFGHIKLMNPQRSTVWY",
    64: bytes(range(0x30, 0x70)),
}

_CHUNK = 1 << 24


def symbol_table(sigma: int) -> np.ndarray:
    """Byte values used for an alphabet of size ``sigma``."""
    if sigma in SYMBOLS:
        return np.frombuffer(SYMBOLS[sigma], dtype=np.uint8).copy()
    if not 1 <= sigma <= 256:
        raise ValueError(f"sigma must be in [1, 256], got {sigma}")
    return np.arange(sigma, dtype=np.uint8)


def zipf_probs(sigma: int, s: float) -> np.ndarray:
    ranks = np.arange(1, sigma + 1, dtype=np.float64)
    w = ranks ** (-float(s))
    return w / w.sum()


def gen_text(n: int, sigma: int, dist: str = "uniform", zipf_s: float = 1.0,
             rng: np.random.Generator | int = 0) -> np.ndarray:
    """``n`` i.i.d. bytes over ``symbol_table(sigma)``; ``dist`` is
    ``"uniform"`` or ``"zipf"``."""
    if not isinstance(rng, np.random.Generator):
        rng = np.random.Generator(np.random.PCG64(rng))
    table = symbol_table(sigma)
    out = np.empty(n, dtype=np.uint8)
    if dist == "uniform":
        for a in range(0, n, _CHUNK):
            b = min(n, a + _CHUNK)
            out[a:b] = table[rng.integers(0, sigma, size=b - a, dtype=np.uint8)]
    elif dist == "zipf":
        cdf = np.cumsum(zipf_probs(sigma, zipf_s))
        cdf[-1] = 1.0
        for a in range(0, n, _CHUNK):
            b = min(n, a + _CHUNK)
            u = rng.random(b - a)
            idx = np.searchsorted(cdf, u, side="right")
            np.minimum(idx, sigma - 1, out=idx)
            out[a:b] = table[idx]
    else:
        raise ValueError(f"unknown distribution {dist!r}")
    return out


def gen_patterns(text: np.ndarray, r: int, m: int, n_sampled: int, sigma: int,
                 rng: np.random.Generator | int = 0) -> np.ndarray:
    """``r`` patterns of length ``m`` as a ``[r, m]`` uint8 array: the first
    ``n_sampled`` copied from random text positions, the rest uniform."""
    if not isinstance(rng, np.random.Generator):
        rng = np.random.Generator(np.random.PCG64(rng))
    n = len(text)
    n_sampled = min(n_sampled, r) if n >= m else 0
    pats = np.empty((r, m), dtype=np.uint8)
    if n_sampled:
        starts = rng.integers(0, n - m + 1, size=n_sampled)
        pats[:n_sampled] = text[starts[:, None] + np.arange(m)[None, :]]
    if r - n_sampled:
        table = symbol_table(sigma)
        pats[n_sampled:] = table[rng.integers(0, sigma, size=(r - n_sampled, m))]
    return pats


@dataclass
class Job:
    """One (text, pattern set) job with the recipe that produced it."""
    text: np.ndarray
    patterns: np.ndarray
    recipe: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.text.shape[0])

    @property
    def r(self) -> int:
        return int(self.patterns.shape[0])

    @property
    def m(self) -> int:
        return int(self.patterns.shape[1])


def make_job(n: int, sigma: int, dist: str, r: int, m: int, frac_sampled: float,
             seed, zipf_s: float = 1.0) -> Job:
    """Text then patterns from one PCG64 stream seeded with ``seed`` (an int or
    a ``numpy.random.SeedSequence``)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    text = gen_text(n, sigma, dist, zipf_s, rng)
    n_sampled = int(round(frac_sampled * r))
    pats = gen_patterns(text, r, m, n_sampled, sigma, rng)
    recipe = dict(n=n, sigma=sigma, dist=dist, zipf_s=zipf_s, r=r, m=m,
                  n_sampled=n_sampled)
    return Job(text, pats, recipe)


# The five workloads. ``scale`` shrinks the text (and nothing else) so the same
# recipe can run at sizes the oracle finishes in seconds.
WORKLOADS = {
    "dna1m": dict(n=1 << 20, sigma=4, dist="uniform", r=100, m=16, frac=1.0, seed=1),
    "zipf256m": dict(n=1 << 28, sigma=64, dist="zipf", r=1000, m=32, frac=0.5, seed=2),
    "prot1g": dict(n=1 << 30, sigma=20, dist="uniform", r=100_000, m=16, frac=0.9, seed=3),
}


def workload(name: str, n: int | None = None) -> Job:
    w = WORKLOADS[name]
    return make_job(n if n is not None else w["n"], w["sigma"], w["dist"], w["r"], w["m"],
                    w["frac"], w["seed"])


def batch_recipes(njobs: int = 512, seed: int = 4, n_log2_range=(12.0, 24.0),
                  r_log10_range=(1.0, 4.0)):
    """Per-job recipes of the batched workload: text lengths log-uniform over
    ``2**n_log2_range`` bytes, sigma in {4, 20, 64}, uniform or Zipf(1.0) at
    50/50, r log-uniform over ``10**r_log10_range``, m in {8, 16, 32}, half of
    each pattern set sampled from its text. Returns ``(recipe, SeedSequence)``
    pairs; the sequence drives that job's own draws."""
    children = np.random.SeedSequence(seed).spawn(njobs)
    out = []
    for child in children:
        rng = np.random.Generator(np.random.PCG64(child))
        n = int(math.floor(2.0 ** rng.uniform(*n_log2_range)))
        sigma = int(rng.choice([4, 20, 64]))
        dist = "uniform" if rng.random() < 0.5 else "zipf"
        r = int(round(10.0 ** rng.uniform(*r_log10_range)))
        m = int(rng.choice([8, 16, 32]))
        # the job's bytes come from a grandchild so the recipe draws above
        # never shift them
        data_seed = child.spawn(1)[0]
        out.append((dict(n=n, sigma=sigma, dist=dist, r=r, m=m, frac=0.5), data_seed))
    return out


def _job_from_recipe(item) -> Job:
    rec, ss = item
    return make_job(rec["n"], rec["sigma"], rec["dist"], rec["r"], rec["m"], rec["frac"], ss)


def batch_jobs(njobs: int = 512, seed: int = 4, n_log2_range=(12.0, 24.0),
               r_log10_range=(1.0, 4.0), workers: int = 1) -> list[Job]:
    """The jobs of :func:`batch_recipes`; ``workers > 1`` draws them in that
    many processes (each job's bytes depend only on its own seed)."""
    items = batch_recipes(njobs, seed, n_log2_range, r_log10_range)
    if workers <= 1:
        return [_job_from_recipe(it) for it in items]
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_job_from_recipe, items, chunksize=4))
