"""The MAG filter's intermediate objects, written from their definitions.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``). Plain numpy / Python,
no blocking or bit tricks beyond what the definitions state. Indices are
0-based where the paper's are 1-based.

Notation (Sections 2 and 3):

* ``mu``: alphabet reduction byte -> [0, sigma') (Section 3.3, "Alphabet
  mapping"); ``sigma_P`` is the number of distinct pattern bytes.
* ``q``: q-gram length. Patterns are cut into non-overlapping q-grams for every
  shift s = 0..q-1 (Section 2, non-overlapping q-grams). All shifts share
  ``L = (m - q + 1) // q`` gram positions.
* gram code of ``S[0..q)``: ``sum_t mu(S[t]) * sigma'**t`` (Section 3.2,
  "Implementation"; S[0] is the least significant digit). Under the alphabet
  mapping on q-grams (Section 3.3) the gram itself is mapped instead: its
  code is the top log2(sigma') bits of a 64-bit hash of its raw bytes.
* superimposed class at gram position b: ``C[b] = {code(P_i[s+bq .. s+bq+q)) :
  i < r, s < q}`` (Section 2, superimposition).
* ``k``: the sampling parameter of Section 3.1; sub-pattern j takes gram
  positions j, j+k, j+2k, ... and has length ``m' = L // k`` (capped so that
  ``W = k m' <= 64``).
* Shift-Or mask table: ``B[c]`` has bit b (b < W) equal to 0 iff c in C[b]
  (Shift-Or convention, 0 = match); bits >= W are 1.
* sampled filter: the text q-gram at offset x*k*q (x = 0, 1, ...) is sample x;
  window (x, j) is a candidate iff for every h < m' sample x-m'+1+h lies in
  C[j+hk]. Its verification starts are ``i0 = (x-m'+1)kq - jq - s`` for
  s < q with 0 <= i0 <= n-m (the occurrence relation of Section 3.1 with the
  q shifts of Section 2).

Readings of passages that are silent or garbled are listed in the design notes
of the repository; the ones that change numbers are repeated at each function.
"""

from __future__ import annotations

import math

import numpy as np

MAX_W = 64          # state bits of the bit-parallel automaton (w = 64 in Section 3.2)
MAX_Q = 8           # the q-gram map keys a gram by its raw bytes in one 64-bit word
DEFAULT_TABLE_BUDGET = 96 * 1024   # bytes of mask table the fixed heuristic allows


# ------------------------------------------------------------------ alphabet

def byte_histogram(patterns: np.ndarray) -> np.ndarray:
    """Occurrences of each byte value over all r*m pattern bytes."""
    p = np.asarray(patterns, dtype=np.uint8)
    return np.bincount(p.reshape(-1), minlength=256).astype(np.int64)


def sigma_p(patterns: np.ndarray) -> int:
    return int((byte_histogram(patterns) > 0).sum())


def _by_frequency(hist: np.ndarray) -> list[int]:
    """Present bytes, most frequent first; equal counts by ascending byte."""
    present = [c for c in range(256) if hist[c] > 0]
    return sorted(present, key=lambda c: (-int(hist[c]), c))


def map_rank(patterns: np.ndarray, sigma_prime: int) -> np.ndarray:
    """Frequency-rank map (Section 3.3): the most frequent pattern byte gets
    code 0, the next code 1, ...; ranks >= sigma'-1 and bytes absent from the
    patterns get sigma'-1. Reading: equal counts are ranked by byte value."""
    if sigma_prime < 1:
        raise ValueError("sigma' must be >= 1")
    hist = byte_histogram(patterns)
    mu = np.full(256, sigma_prime - 1, dtype=np.uint8)
    for rank, c in enumerate(_by_frequency(hist)):
        mu[c] = min(rank, sigma_prime - 1)
    return mu


def map_greedy(patterns: np.ndarray, sigma_prime: int) -> np.ndarray:
    """Equal-weight map (Section 3.3), by the greedy longest-processing-time
    rule. Reading: bytes are taken in descending pattern-set count (ties by
    ascending byte) and each goes to the bin of least total weight so far (ties
    to the lowest bin index); bytes absent from the patterns get sigma'-1."""
    if sigma_prime < 1:
        raise ValueError("sigma' must be >= 1")
    hist = byte_histogram(patterns)
    mu = np.full(256, sigma_prime - 1, dtype=np.uint8)
    load = [0] * sigma_prime
    for c in _by_frequency(hist):
        b = min(range(sigma_prime), key=lambda i: (load[i], i))
        mu[c] = b
        load[b] += int(hist[c])
    return mu


def bits_shift(patterns: np.ndarray, sigma_prime: int) -> int:
    """The shift s of the bit-field map (Section 3.3, combined alphabet mapping
    and q-gram generation): sigma' = 2^l and mu(c) = (c >> s) & (2^l - 1).
    Reading: s in 0..8-l is chosen so that the heaviest code carries the
    least pattern-byte weight (ties to the smaller s); the paper's DNA example
    shifts by one for the same reason (the low two bits of C and G agree)."""
    l = sigma_prime.bit_length() - 1
    if sigma_prime < 1 or (1 << l) != sigma_prime or l > 8:
        raise ValueError("the bit-field map needs sigma' = 2^l with l <= 8")
    hist = byte_histogram(patterns)
    best, best_s = None, 0
    for sh in range(0, 8 - l + 1):
        load = [0] * sigma_prime
        for c in range(256):
            load[(c >> sh) & (sigma_prime - 1)] += int(hist[c])
        if best is None or max(load) < best:
            best, best_s = max(load), sh
    return best_s


def map_bits(patterns: np.ndarray, sigma_prime: int) -> np.ndarray:
    """mu(c) = (c >> s) & (sigma' - 1), s from bits_shift: the gram code
    sum_t mu(S[t]) sigma'^t is then the concatenation of l-bit fields of the
    Section 3.3 formula, S[0] in the low bits."""
    sh = bits_shift(patterns, sigma_prime)
    return np.array([(c >> sh) & (sigma_prime - 1) for c in range(256)], dtype=np.uint8)


# --------------------------------------------- alphabet mapping on q-grams

MASK64 = (1 << 64) - 1
FMIX_C1 = 0xFF51AFD7ED558CCD
FMIX_C2 = 0xC4CEB9FE1A85EC53


def fmix64(x: int) -> int:
    """MurmurHash3's 64-bit finalizer (A. Appleby, public domain): three
    xor-shifts by 33 with two odd multiplies between them, modulo 2^64."""
    x &= MASK64
    x ^= x >> 33
    x = (x * FMIX_C1) & MASK64
    x ^= x >> 33
    x = (x * FMIX_C2) & MASK64
    x ^= x >> 33
    return x


def gram_key(seq) -> int:
    """The raw bytes of a q-gram (q <= 8) as one integer, S[0] in the low byte."""
    key = 0
    for t, c in enumerate(seq):
        key |= int(c) << (8 * t)
    return key


def qgram_code(seq, log2_sigma_prime: int) -> int:
    """Code of a q-gram under the alphabet mapping on q-grams (Section 3.3,
    "Alphabet mapping on the q-grams"): the mapped q-gram alphabet has
    sigma' = 2^b symbols and a gram's symbol is the top b bits of
    fmix64(key). Reading: the paper leaves the mapping method open (bin
    packing is one example) and stores the mapping by hashing; here the
    hash itself is the mapping, which fixes the table at exactly sigma'
    entries for any q, needs no stored keys, and keeps every gram of the
    text mappable. q is limited to 8 so that a gram is one 64-bit key."""
    b = log2_sigma_prime
    if b == 0:
        return 0
    return fmix64(gram_key(seq)) >> (64 - b)


def qgram_codes(grams: np.ndarray, log2_sigma_prime: int) -> np.ndarray:
    """qgram_code of every row of an [N, q] byte array, as int64."""
    g = np.asarray(grams, dtype=np.uint8)
    n, q = g.shape
    if q > 8:
        raise ValueError("q-grams of the q-gram map hold at most 8 bytes")
    b = log2_sigma_prime
    if b == 0 or n == 0:
        return np.zeros(n, dtype=np.int64)
    x = np.zeros(n, dtype=np.uint64)
    for t in range(q):
        x |= g[:, t].astype(np.uint64) << np.uint64(8 * t)
    s33 = np.uint64(33)
    x ^= x >> s33
    x *= np.uint64(FMIX_C1)          # wraps modulo 2^64
    x ^= x >> s33
    x *= np.uint64(FMIX_C2)
    x ^= x >> s33
    return (x >> np.uint64(64 - b)).astype(np.int64)


def log2_exact(v: int) -> int:
    b = int(v).bit_length() - 1
    if v < 1 or (1 << b) != v:
        raise ValueError("sigma' of this map must be a power of two")
    return b


def alphabet_map(patterns: np.ndarray, sigma_prime: int, kind: str = "greedy") -> np.ndarray:
    if kind == "greedy":
        return map_greedy(patterns, sigma_prime)
    if kind == "rank":
        return map_rank(patterns, sigma_prime)
    if kind == "bits":
        return map_bits(patterns, sigma_prime)
    raise ValueError(kind)


# ---------------------------------------------------------------- parameters

def round_half_up(v: float) -> int:
    return int(math.floor(v + 0.5))


def gram_positions(m: int, q: int) -> int:
    """L: gram positions shared by all q shifts of a length-m pattern."""
    return (m - q + 1) // q


def sub_pattern_length(L: int, k: int) -> int:
    """m' = floor(L/k), capped so that k*m' <= 64 state bits."""
    return min(L // k, MAX_W // k)


def entry_bytes(W: int) -> int:
    """Storage of one mask-table entry of W bits (1, 2, 4 or 8 bytes)."""
    for b in (1, 2, 4, 8):
        if W <= 8 * b:
            return b
    raise ValueError("W > 64")


def entry_bits(W: int, kind: str) -> int:
    """Bits one stored mask-table entry takes: tables of the q-gram map with
    W <= 4 are packed (1, 2 or 4 bits per entry), all others use whole bytes."""
    if kind == "qgram" and W <= 4:
        return 1 if W <= 1 else 2 if W <= 2 else 4
    return 8 * entry_bytes(W)


def heuristic_q(sigma: int, r: int, m: int) -> int:
    """q = log_sigma(r m) (Section 3.2). Reading: sigma is the number of
    distinct pattern bytes (at least 2), rounded half up, clamped to
    [1, (m+1)//2] so that at least one gram position exists (2q-1 <= m).
    Nothing else bounds it: Section 3.2's formula may give q above the
    "small constant" of Section 2 for large r*m over small alphabets."""
    s = max(sigma, 2)
    q = round_half_up(math.log(r * m) / math.log(s))
    return max(1, min(q, (m + 1) // 2))


def heuristic_k(sigma: int, r: int, m: int, L: int) -> int:
    """k from the O(.) expression of Section 3.2 with constant 1:
    k = m/log(rm) * log(1/rho) / (log(rm) + log(1/rho)), logs base sigma,
    rho = log(rm)/m. Reading: rounded half up, clamped to [1, L]; rho >= 1
    gives k = 1."""
    s = max(sigma, 2)
    lg = math.log(r * m) / math.log(s)
    rho = lg / m
    if rho >= 1.0 or lg <= 0:
        return 1
    inv = math.log(1.0 / rho) / math.log(s)
    k = round_half_up(m / lg * inv / (lg + inv))
    return max(1, min(k, max(L, 1)))


def heuristic_params(patterns: np.ndarray, table_budget: int = DEFAULT_TABLE_BUDGET,
                     q_cap: int | None = None):
    """The fixed heuristic: (q, k, sigma'). sigma' starts at sigma_P and is
    lowered until sigma'**q * entry_bytes(W) fits the table budget (the
    motivation of Section 3.3: table size grows as sigma**q).

    ``q_cap``: an upper limit a caller imposes on q before k and sigma' are
    derived from it (an implementation that supports grams of at most
    ``q_cap`` bytes); None keeps Section 3.2's q."""
    p = np.asarray(patterns, dtype=np.uint8)
    r, m = p.shape
    sp = sigma_p(p)
    q = heuristic_q(sp, r, m)
    if q_cap is not None:
        q = min(q, q_cap)
    L = gram_positions(m, q)
    k = heuristic_k(sp, r, m, L)
    mprime = sub_pattern_length(L, k)
    W = k * mprime
    eb = entry_bytes(W)
    sig = max(sp, 1)
    while sig > 1 and sig ** q * eb > table_budget:
        sig -= 1
    return q, k, sig


QGRAM_TABLE_BUDGET = 8 << 20     # bytes the q-gram map's heuristic allows for the mask table
QGRAM_LOAD = 32                  # target codes per distinct gram of the fullest class


def class_grams(patterns: np.ndarray, q: int, W: int) -> list[set]:
    """For b < W, the distinct raw q-grams (as bytes) of every pattern's
    shift-s gram at position b, over all q shifts: the classes before any
    alphabet mapping."""
    p = np.asarray(patterns, dtype=np.uint8)
    out = []
    for b in range(W):
        grams = set()
        for s in range(q):
            off = s + b * q
            grams.update(bytes(row) for row in p[:, off:off + q])
        out.append(grams)
    return out


def heuristic_params_qgram(patterns: np.ndarray, table_budget: int = QGRAM_TABLE_BUDGET):
    """(q, k, sigma') for the q-gram map. Reading (the paper gives none for
    this variant; Section 3.3 only says q may be large and sigma' is chosen to
    control the table): q is the largest allowed (min(8, (m+1)//2)), k = 1
    (the longest sub-pattern), and sigma' is the smallest power of two with
    at least QGRAM_LOAD codes per distinct gram of the fullest class, halved
    while the table exceeds the budget (sigma' >= 2)."""
    p = np.asarray(patterns, dtype=np.uint8)
    r, m = p.shape
    q = max(1, min(MAX_Q, (m + 1) // 2))
    L = gram_positions(m, q)
    k = 1
    W = k * sub_pattern_length(L, k)
    D = max((len(c) for c in class_grams(p, q, W)), default=0) if r else 0
    eb = entry_bits(W, "qgram")
    sp = 2
    while sp < QGRAM_LOAD * D:
        sp *= 2
    while sp > 2 and sp * eb > 8 * table_budget:
        sp //= 2
    return q, k, sp


# ----------------------------------------------------------- q-gram classes

def gram_code(seq, mu: np.ndarray, sigma_prime: int) -> int:
    """Numeric code of one q-gram: sum_t mu(S[t]) * sigma'**t."""
    code = 0
    for t, c in enumerate(seq):
        code += int(mu[int(c)]) * sigma_prime ** t
    return code


def overlapping_grams(pattern: bytes, q: int) -> list[bytes]:
    """P'[j] = P[j..j+q) for j = 0..m-q (Section 2, overlapping q-grams)."""
    return [pattern[j:j + q] for j in range(len(pattern) - q + 1)]


def nonoverlapping_grams(pattern: bytes, q: int, shift: int = 0) -> list[bytes]:
    """P'[j] = P[s+jq .. s+jq+q) for the pattern read from offset s
    (Section 2, non-overlapping q-grams)."""
    tail = pattern[shift:]
    return [tail[j * q:(j + 1) * q] for j in range(len(tail) // q)]


def superimpose(rows: list[list]) -> list[set]:
    """Character classes P[i] = union over patterns of P_j[i] (Section 2)."""
    length = min(len(r) for r in rows)
    return [set(r[i] for r in rows) for i in range(length)]


def classes(patterns: np.ndarray, mu: np.ndarray, sigma_prime: int, q: int, W: int) -> list[set]:
    """C[b] for b < W: codes of every pattern's shift-s gram at position b,
    over all q shifts."""
    p = np.asarray(patterns, dtype=np.uint8)
    r, m = p.shape
    if W and (q - 1) + W * q > m:
        raise ValueError("W gram positions do not fit every shift")
    mapped = mu[p].astype(np.int64)
    weights = np.array([sigma_prime ** t for t in range(q)], dtype=np.int64)
    out = []
    for b in range(W):
        cls = set()
        for s in range(q):
            off = s + b * q
            codes = mapped[:, off:off + q] @ weights
            cls.update(int(c) for c in np.unique(codes))
        out.append(cls)
    return out


def mask_table(cls: list[set], W: int, n_codes: int) -> np.ndarray:
    """B[c] for c < n_codes as uint64: bit b = 0 iff c in C[b] (b < W),
    bits >= W are 1."""
    B = np.full(n_codes, np.uint64(0xFFFFFFFFFFFFFFFF), dtype=np.uint64)
    for b in range(W):
        idx = np.fromiter(cls[b], dtype=np.int64, count=len(cls[b]))
        B[idx] &= np.uint64(~(1 << b) & 0xFFFFFFFFFFFFFFFF)
    return B


class Filter:
    """Everything the filter needs for one pattern set and (q, k, sigma', map)."""

    def __init__(self, patterns: np.ndarray, q: int, k: int, sigma_prime: int,
                 kind: str = "greedy"):
        p = np.asarray(patterns, dtype=np.uint8)
        self.patterns = p
        self.r, self.m = p.shape
        self.q, self.k, self.sigma_prime = q, k, sigma_prime
        if q < 1 or 2 * q - 1 > self.m:
            raise ValueError("need 1 <= q and 2q-1 <= m")
        self.L = gram_positions(self.m, q)
        if not 1 <= k <= self.L:
            raise ValueError("need 1 <= k <= L")
        self.mprime = sub_pattern_length(self.L, k)
        self.W = k * self.mprime
        self.kind = kind
        if kind == "qgram":
            if q > MAX_Q:
                raise ValueError("q above 8")
            self.log2_sp = log2_exact(sigma_prime)
            self.mu = None
            self.n_codes = sigma_prime
            self.C = [set(int(c) for c in qgram_codes(
                np.frombuffer(b"".join(sorted(g)), dtype=np.uint8).reshape(-1, q), self.log2_sp))
                for g in class_grams(p, q, self.W)]
        else:
            self.mu = alphabet_map(p, sigma_prime, kind)
            self.n_codes = sigma_prime ** q
            self.C = classes(p, self.mu, sigma_prime, q, self.W)
        self.entry_bits = entry_bits(self.W, kind)

    def table(self) -> np.ndarray:
        return mask_table(self.C, self.W, self.n_codes)

    def n_samples(self, n: int) -> int:
        """Samples x with x*k*q + q <= n."""
        if n < self.q:
            return 0
        return (n - self.q) // (self.k * self.q) + 1

    def sample_codes(self, text: np.ndarray) -> np.ndarray:
        t = np.asarray(text, dtype=np.uint8)
        X = self.n_samples(t.size)
        kq = self.k * self.q
        if self.kind == "qgram":
            idx = np.arange(X, dtype=np.int64)[:, None] * kq + np.arange(self.q)[None, :]
            return qgram_codes(t[idx].reshape(X, self.q), self.log2_sp)
        codes = np.zeros(X, dtype=np.int64)
        for d in range(self.q):
            codes += self.mu[t[np.arange(X, dtype=np.int64) * kq + d]].astype(np.int64) * self.sigma_prime ** d
        return codes

    def n_grams(self, n: int) -> int:
        """Complete non-overlapping text q-grams T[yq .. yq+q)."""
        return 0 if n < self.q else (n - self.q) // self.q + 1

    def encode(self, text: np.ndarray) -> np.ndarray:
        """The encoded text of the SMAG variant (Section 3.2,
        "Implementation"): the code of every complete non-overlapping q-gram
        T[yq .. yq+q), y = 0 .. (n-q)//q, computed before the search. The
        filter's sample x is entry x*k of it."""
        t = np.asarray(text, dtype=np.uint8)
        G = self.n_grams(t.size)
        idx = np.arange(G, dtype=np.int64)[:, None] * self.q + np.arange(self.q)[None, :]
        grams = t[idx].reshape(G, self.q)
        if self.kind == "qgram":
            return qgram_codes(grams, self.log2_sp)
        codes = np.zeros(G, dtype=np.int64)
        for d in range(self.q):
            codes += self.mu[grams[:, d]].astype(np.int64) * self.sigma_prime ** d
        return codes

    def candidates(self, text: np.ndarray) -> np.ndarray:
        """Boolean [X, k]: window (x, j) passes the filter."""
        g = self.sample_codes(text)
        X, k, mp = g.size, self.k, self.mprime
        member = []
        for b in range(self.W):
            cls = np.fromiter(self.C[b], dtype=np.int64, count=len(self.C[b]))
            member.append(np.isin(g, cls))
        cand = np.zeros((X, k), dtype=bool)
        if X < mp:
            return cand
        for j in range(k):
            ok = np.ones(X - mp + 1, dtype=bool)
            for h in range(mp):
                # sample x-m'+1+h for x = m'-1 .. X-1
                ok &= member[j + h * k][h:h + X - mp + 1]
            cand[mp - 1:, j] = ok
        return cand

    def verification_starts(self, text: np.ndarray, cand: np.ndarray | None = None) -> np.ndarray:
        """All i0 = (x-m'+1)kq - jq - s (s < q) of candidate windows with
        0 <= i0 <= n-m, in ascending order."""
        t = np.asarray(text, dtype=np.uint8)
        if cand is None:
            cand = self.candidates(t)
        xs, js = np.nonzero(cand)
        kq, q, mp = self.k * self.q, self.q, self.mprime
        starts = []
        for s in range(q):
            i0 = (xs.astype(np.int64) - mp + 1) * kq - js.astype(np.int64) * q - s
            starts.append(i0[(i0 >= 0) & (i0 <= t.size - self.m)])
        out = np.concatenate(starts) if starts else np.empty(0, dtype=np.int64)
        return np.sort(out)

    def counts(self, text: np.ndarray) -> dict:
        cand = self.candidates(text)
        return dict(samples=self.n_samples(np.asarray(text).size),
                    cand_windows=int(cand.sum()),
                    verifications=int(self.verification_starts(text, cand).size))


def filter_from_params(patterns, q=None, k=None, sigma_prime=None, kind="greedy",
                       table_budget=DEFAULT_TABLE_BUDGET) -> Filter:
    hq, hk, hs = heuristic_params(patterns, table_budget)
    return Filter(patterns, q or hq, k or hk, sigma_prime or hs, kind)


# ------------------------------------------------------- density estimates

def class_hit_probability(alphabet: int, items: int) -> float:
    """Probability that a random symbol of an alphabet of the given size
    falls in the union of ``items`` random symbols: 1 - (1 - 1/a)**items
    (the class-density example of Section 2)."""
    return 1.0 - (1.0 - 1.0 / alphabet) ** items


def expected_class_size(alphabet: int, items: int) -> float:
    return alphabet * class_hit_probability(alphabet, items)


# ------------------------------------------------- unequal pattern lengths

def prefix_set(patterns) -> np.ndarray:
    """Patterns of unequal lengths filter as the set of their first m_min
    bytes (m_min the shortest length): an occurrence of P_id at i contains
    an occurrence of its prefix at i, so the equal-length filter over the
    prefixes never drops it. Reading of the introduction's remark that the
    equal-length requirement may be removed; verification then checks each
    pattern over its full length."""
    pats = [np.asarray(np.frombuffer(bytes(p), dtype=np.uint8)) for p in patterns]
    m_min = min(p.size for p in pats)
    return np.stack([p[:m_min] for p in pats])
