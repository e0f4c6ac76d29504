"""MAG multiple pattern matching on MI355X.

Thin Python front end of ``libmag.so`` (C ABI in ``include/mag.h``): it only
marshals arguments. Every step of the scan runs in the library's HIP kernels;
PyTorch supplies device memory and streams.

    import torch, paper_1405_5483_amd as mag
    plan = mag.Plan(patterns)                 # [r, m] uint8 (numpy / bytes list;
                                              #  a list of unequal lengths also works)
    occ = mag.scan(text_cuda_u8, plan)        # int64 [z, 2]: (pos, pattern id)

The occurrence set is the one of Section 1 of the paper: every (i, id) with
``T[i..i+m) == P_id``, sorted by (i, id).
"""

from __future__ import annotations

import ctypes

import numpy as np

from ._lib import (DENSE_PROBE, MAG_E_OVERFLOW, MAP_KIND, MODE, SELECT, VERIFY, MagError, MagJob, MagParams, MagPlanDesc,
                   MagStats, MagTuneOpts, check, lib)

__all__ = ["Plan", "Batch", "Selector", "scan", "scan_async", "scan_batch", "autotune",
           "select_features", "select_candidates", "profile_enable", "profile_read", "MagError",
           "lib"]

_ENTRY_DTYPE = {1: np.uint8, 2: np.uint16, 4: np.uint32, 8: np.uint64}


def _as_patterns(patterns) -> np.ndarray:
    if isinstance(patterns, (list, tuple)):
        rows = [np.frombuffer(bytes(p), dtype=np.uint8) for p in patterns]
        if not rows:
            raise ValueError("empty pattern list needs an explicit length; pass a [0, m] array")
        return np.ascontiguousarray(np.stack(rows))
    if hasattr(patterns, "detach"):          # torch tensor
        patterns = patterns.detach().cpu().numpy()
    p = np.ascontiguousarray(patterns, dtype=np.uint8)
    if p.ndim != 2:
        raise ValueError("patterns must be [r, m]")
    return p


def _unequal(patterns):
    """(concatenated bytes, offsets) when ``patterns`` is a list whose
    entries differ in length, else None."""
    if not isinstance(patterns, (list, tuple)) or not patterns:
        return None
    rows = [np.frombuffer(bytes(p), dtype=np.uint8) for p in patterns]
    if len({r.size for r in rows}) == 1:
        return None
    offsets = np.zeros(len(rows) + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum([r.size for r in rows])
    return np.ascontiguousarray(np.concatenate(rows)), offsets


class Plan:
    """A pattern set prepared for scanning (``mag_plan_create``)."""

    def __init__(self, patterns, *, select: str = "heuristic", q: int | None = None,
                 k: int | None = None, sigma_prime: int | None = None,
                 map_kind: str = "greedy", table_budget: int = 0, mode: str = "auto",
                 verify: str = "auto", verify_buffer: int = 0, encode: bool = False,
                 dense_probe: str = "auto", chunk_bytes: int = 0, words_per_lane: int = 0,
                 candidate: int | None = None):
        var = _unequal(patterns)
        if var is None:
            p = _as_patterns(patterns)
            self.r, self.m = int(p.shape[0]), int(p.shape[1])
        else:
            data, offsets = var
            self.r, self.m = int(offsets.size - 1), int(np.diff(offsets).min())
        self.candidate = candidate        # selector grid index of a learned pick (informational)
        prm = MagParams()
        if q is not None or k is not None or sigma_prime is not None:
            if select == "heuristic":
                select = "explicit"
        prm.select = SELECT[select]
        prm.map_kind = MAP_KIND[map_kind]
        prm.q = int(q or 0)
        prm.k = int(k or 0)
        prm.sigma_prime = int(sigma_prime or 0)
        prm.table_budget = int(table_budget)
        prm.mode = MODE[mode]
        prm.verify = VERIFY[verify]
        prm.verify_buffer = int(verify_buffer)
        prm.encode = 1 if encode else 0
        prm.dense_probe = DENSE_PROBE[dense_probe]
        prm.chunk_bytes = int(chunk_bytes)
        prm.words_per_lane = int(words_per_lane)
        handle = ctypes.c_void_p()
        self._h = None
        if var is None:
            check(lib().mag_plan_create(p.ctypes.data if p.size else None, self.r, self.m,
                                        ctypes.byref(prm), ctypes.byref(handle)), "mag_plan_create")
        else:
            check(lib().mag_plan_create_var(data.ctypes.data, offsets.ctypes.data, self.r,
                                            ctypes.byref(prm), ctypes.byref(handle)),
                  "mag_plan_create_var")
        self._h = handle

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("plan is closed")
        return self._h

    def info(self) -> dict:
        d = MagPlanDesc()
        check(lib().mag_plan_info(self.handle, ctypes.byref(d)), "mag_plan_info")
        return {name: getattr(d, name) for name, _ in MagPlanDesc._fields_}

    def params(self) -> dict:
        """The resolved choices as Plan keyword arguments
        (``mag_plan_get_params``): ``Plan(patterns, **plan.params())`` builds
        the same filter and tables."""
        prm = MagParams()
        check(lib().mag_plan_get_params(self.handle, ctypes.byref(prm)), "mag_plan_get_params")
        inv = lambda d, v: next(name for name, code in d.items() if code == v)
        return {"select": inv(SELECT, prm.select), "map_kind": inv(MAP_KIND, prm.map_kind),
                "q": prm.q, "k": prm.k, "sigma_prime": prm.sigma_prime,
                "mode": inv(MODE, prm.mode), "verify": inv(VERIFY, prm.verify),
                "verify_buffer": prm.verify_buffer, "encode": bool(prm.encode),
                "dense_probe": inv(DENSE_PROBE, prm.dense_probe), "chunk_bytes": prm.chunk_bytes,
                "words_per_lane": prm.words_per_lane}

    def export(self, raw: bool = False):
        """(mu [256] uint8, mask table with one entry per code in the entry
        dtype). Packed tables (entry_bits < 8) are unpacked to uint8 entries
        whose bits above entry_bits are 1, or returned as the stored bytes
        with raw=True."""
        info = self.info()
        mu = np.empty(256, dtype=np.uint8)
        eb = info["entry_bits"]
        if eb < 8:
            buf = np.empty(info["table_bytes"], dtype=np.uint8)
            check(lib().mag_plan_export(self.handle, mu.ctypes.data, buf.ctypes.data,
                                        buf.nbytes), "mag_plan_export")
            if raw:
                return mu, buf
            n = info["n_codes"]
            bits = np.unpackbits(buf, bitorder="little")[: n * eb].reshape(n, eb).astype(np.uint16)
            vals = (bits << np.arange(eb, dtype=np.uint16)).sum(axis=1)
            return mu, (vals | ((0xFF << eb) & 0xFF)).astype(np.uint8)
        table = np.empty(info["n_codes"], dtype=_ENTRY_DTYPE[info["entry_bytes"]])
        check(lib().mag_plan_export(self.handle, mu.ctypes.data, table.ctypes.data,
                                    table.nbytes), "mag_plan_export")
        return mu, table

    def close(self):
        if self._h is not None:
            lib().mag_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_text(text):
    import torch
    if not isinstance(text, torch.Tensor) or text.dtype != torch.uint8 or not text.is_cuda:
        raise TypeError("text must be a torch.uint8 CUDA (HIP) tensor")
    if not text.is_contiguous():
        raise ValueError("text must be contiguous")


def scan(text, plan: Plan, out_cap: int | None = None, stats: bool = False, stream=None):
    """All occurrences as an int64 tensor [z, 2] of (pos, pattern id), sorted.
    With ``stats=True`` also returns the work counters as a dict."""
    import torch
    _check_text(text)
    n = text.numel()
    cap = int(out_cap) if out_cap is not None else max(1024, min(n // 8, 1 << 22))
    st = MagStats()
    count = ctypes.c_uint64(0)
    for _ in range(2):
        out = torch.empty((max(cap, 1), 2), dtype=torch.int64, device=text.device)
        status = lib().mag_scan(plan.handle, ctypes.c_void_p(text.data_ptr()), n,
                                ctypes.c_void_p(out.data_ptr()), cap, ctypes.byref(count),
                                ctypes.byref(st), _stream_ptr(stream))
        if status == MAG_E_OVERFLOW and out_cap is None:
            cap = int(count.value)
            continue
        check(status, "mag_scan")
        break
    z = int(count.value)
    res = out[:z]
    if stats:
        return res, {name: getattr(st, name) for name, _ in MagStats._fields_}
    return res


def encode(text, plan: Plan, stream=None):
    """SMAG's encoded text (``mag_encode``): the plan's code of every complete
    non-overlapping q-gram of ``text``, as an int32 CUDA tensor (codes are
    below 2^28, so the unsigned values read the same)."""
    import torch
    _check_text(text)
    n = text.numel()
    q = plan.info()["q"]
    G = (n - q) // q + 1 if n >= q else 0
    out = torch.empty(max(G, 1), dtype=torch.int32, device=text.device)
    got = ctypes.c_uint64(0)
    check(lib().mag_encode(plan.handle, ctypes.c_void_p(text.data_ptr()) if n else None, n,
                           ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.byref(got),
                           _stream_ptr(stream)), "mag_encode")
    assert got.value == G
    return out[:G]


def stream_read(buf, sink=None, stream=None):
    """Measurement aid: one plain streaming read of a uint8 CUDA tensor
    (``mag_stream_read``); returns the sink tensor of per-block xors."""
    import torch
    _check_text(buf)
    if sink is None:
        sink = torch.empty(max(int(lib().mag_stream_read_sink_words()), 1), dtype=torch.int32,
                           device=buf.device)
    check(lib().mag_stream_read(ctypes.c_void_p(buf.data_ptr()), buf.numel(),
                                ctypes.c_void_p(sink.data_ptr()), _stream_ptr(stream)),
          "mag_stream_read")
    return sink


def scan_async(text, plan: Plan, out, d_count, d_stats=None, stream=None) -> None:
    """Enqueues a scan without waiting (``mag_scan_async``). ``out`` is an
    int64 [cap, 2] CUDA tensor, ``d_count`` an int64 [1] CUDA tensor that
    receives the exact occurrence count, ``d_stats`` an optional CUDA tensor
    of at least 56 bytes (e.g. int64 [7]) for ``mag_stats``: the four counters
    as int64 [0:4], then q, k, sigma', m' as int32 and plan_ms as float32."""
    _check_text(text)
    check(lib().mag_scan_async(plan.handle, ctypes.c_void_p(text.data_ptr()), text.numel(),
                               ctypes.c_void_p(out.data_ptr()), out.shape[0],
                               ctypes.c_void_p(d_count.data_ptr()),
                               ctypes.c_void_p(d_stats.data_ptr()) if d_stats is not None else None,
                               _stream_ptr(stream)), "mag_scan_async")


def scan_noalloc(text, plan: Plan, out, d_count, d_stats=None, stream=None) -> None:
    """``scan_async`` through ``mag_scan_noalloc``: no device allocation, the
    scratch in the library's static per-GPU array (out_cap at most 2^20; the
    plan must have been scanned once on this device)."""
    _check_text(text)
    check(lib().mag_scan_noalloc(plan.handle, ctypes.c_void_p(text.data_ptr()), text.numel(),
                                 ctypes.c_void_p(out.data_ptr()), out.shape[0],
                                 ctypes.c_void_p(d_count.data_ptr()),
                                 ctypes.c_void_p(d_stats.data_ptr()) if d_stats is not None else None,
                                 _stream_ptr(stream)), "mag_scan_noalloc")


class Batch:
    """Many (text, plan) jobs scanned in one persistent launch (``mag_batch_*``).

    ``Batch(plans)`` fixes the jobs' pattern sets (a plan may serve several
    jobs); :meth:`bind` attaches their texts and the output capacity;
    :meth:`run_async` enqueues scan, sort and per-job offsets on a stream with
    no host synchronization or allocation, so it can be captured in a graph.
    """

    def __init__(self, plans, words_per_lane: int = 0):
        self.plans = list(plans)          # the library keeps raw pointers to them
        arr = (ctypes.c_void_p * max(len(self.plans), 1))(
            *[p.handle.value for p in self.plans])
        handle = ctypes.c_void_p()
        self._h = None
        check(lib().mag_batch_create(arr, len(self.plans), ctypes.byref(handle)),
              "mag_batch_create")
        self._h = handle
        self.texts = []
        self.out_cap = 0
        if words_per_lane:
            self.set_words_per_lane(words_per_lane)

    def set_words_per_lane(self, words_per_lane: int) -> None:
        """Filter tiles of 1024 * words_per_lane samples (8 or 16); takes
        effect at the next bind."""
        check(lib().mag_batch_set_words_per_lane(self.handle, int(words_per_lane)),
              "mag_batch_set_words_per_lane")

    @property
    def njobs(self) -> int:
        return len(self.plans)

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("batch is closed")
        return self._h

    def bind(self, texts, out_cap: int, stream=None) -> None:
        """Attach one uint8 CUDA tensor per job (kept referenced until the next
        bind) and size the scratch for ``out_cap`` occurrences in total."""
        texts = list(texts)
        if len(texts) != self.njobs:
            raise ValueError(f"{len(texts)} texts for {self.njobs} jobs")
        for t in texts:
            _check_text(t)
        nj = max(self.njobs, 1)
        ptrs = (ctypes.c_void_p * nj)(*[t.data_ptr() or None for t in texts])
        ns = (ctypes.c_uint64 * nj)(*[t.numel() for t in texts])
        check(lib().mag_batch_bind(self.handle, ptrs, ns, int(out_cap), _stream_ptr(stream)),
              "mag_batch_bind")
        self.texts = texts
        self.out_cap = int(out_cap)

    def run_async(self, out, offsets, count, stream=None) -> None:
        """``out``: int64 [out_cap, 2] CUDA tensor of (pos, pattern id) records,
        job after job; ``offsets``: int64 [njobs + 1] CUDA tensor, job j's
        records are ``out[offsets[j]:offsets[j+1]]``; ``count``: int64 [1]."""
        if out.shape[0] < self.out_cap:
            raise ValueError("out is smaller than the bound capacity")
        if offsets.numel() < self.njobs + 1:
            raise ValueError("offsets needs njobs + 1 entries")
        check(lib().mag_batch_run_async(self.handle, ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(offsets.data_ptr()),
                                        ctypes.c_void_p(count.data_ptr()), _stream_ptr(stream)),
              "mag_batch_run_async")

    def run(self, stream=None):
        """Runs the bound jobs and returns one int64 [z_j, 2] tensor per job.
        Rebinds with the exact capacity and runs again if the output overflowed."""
        import torch
        dev = self.texts[0].device if self.texts else torch.device("cuda")
        for _ in range(2):
            out = torch.empty((max(self.out_cap, 1), 2), dtype=torch.int64, device=dev)
            offsets = torch.empty(self.njobs + 1, dtype=torch.int64, device=dev)
            count = torch.empty(1, dtype=torch.int64, device=dev)
            self.run_async(out, offsets, count, stream)
            (stream if stream is not None else torch.cuda.current_stream()).synchronize()
            z = int(count.item())
            if z <= self.out_cap:
                off = offsets.cpu().tolist()
                return [out[off[j]:off[j + 1]] for j in range(self.njobs)]
            self.bind(self.texts, z, stream)
        raise MagError(MAG_E_OVERFLOW, "batch output still overflows after rebinding")

    def close(self):
        if self._h is not None:
            lib().mag_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def scan_batch(texts, plans, out_cap: int | None = None, stream=None):
    """One-shot batched scan (``mag_scan_batch``): job j scans ``texts[j]``
    with ``plans[j]``. Returns one int64 [z_j, 2] tensor of sorted
    (pos, pattern id) per job; an output above the capacity is rescanned with
    room for the exact total."""
    import torch
    if len(texts) != len(plans):
        raise ValueError("one plan per text")
    for t in texts:
        _check_text(t)
    njobs = len(texts)
    jobs = (MagJob * max(njobs, 1))()
    for j, (t, p) in enumerate(zip(texts, plans)):
        jobs[j].plan = p.handle.value
        jobs[j].d_text = t.data_ptr() if t.numel() else None
        jobs[j].n = t.numel()
    cap = out_cap if out_cap is not None else max(1 << 16, sum(t.numel() for t in texts) // 64)
    offsets = (ctypes.c_uint64 * (njobs + 1))()
    for _ in range(2):
        out = torch.empty((max(cap, 1), 2), dtype=torch.int64, device="cuda")
        status = lib().mag_scan_batch(jobs, njobs, ctypes.c_void_p(out.data_ptr()), cap, offsets,
                                      _stream_ptr(stream))
        if status == MAG_E_OVERFLOW:
            cap = int(offsets[njobs])
            continue
        check(status, "mag_scan_batch")
        off = list(offsets)
        return [out[off[j]:off[j + 1]] for j in range(njobs)]
    raise MagError(MAG_E_OVERFLOW, "batch output still overflows after resizing")


def profile_enable(on: bool = True) -> None:
    """Record HIP events around each scan's kernels (``mag_profile_enable``)."""
    check(lib().mag_profile_enable(1 if on else 0), "mag_profile_enable")


def profile_read() -> dict:
    """Summed kernel times since the last read (``mag_profile_read``)."""
    a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_uint64()
    check(lib().mag_profile_read(ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)),
          "mag_profile_read")
    return {"scan_ms": a.value, "finish_ms": b.value, "launches": int(n.value)}


_MAP_NAME = {v: k for k, v in MAP_KIND.items()}


def _tune_opts(map_kinds=0, max_q=0, max_k=0, table_budget=0, repeats=0, max_candidates=0,
               modes=0, fixed_tiles=False):
    o = MagTuneOpts()
    o.map_kinds, o.max_q, o.max_k = map_kinds, max_q, max_k
    o.table_budget, o.repeats, o.max_candidates = table_budget, repeats, max_candidates
    o.modes, o.fixed_tiles = modes, int(bool(fixed_tiles))
    return o


def _plan_kwargs(prm: MagParams) -> dict:
    """Plan keyword arguments of explicit parameters returned by the library."""
    inv = lambda d, v: next(name for name, code in d.items() if code == v)
    return {"q": prm.q, "k": prm.k, "sigma_prime": prm.sigma_prime, "map_kind": _MAP_NAME[prm.map_kind],
            "mode": inv(MODE, prm.mode), "words_per_lane": prm.words_per_lane}


def autotune(patterns, sample, *, stream=None, **opts) -> dict:
    """Parameters picked by ``mag_autotune`` from scans of ``sample`` (a uint8
    CUDA tensor): dict of :class:`Plan` keyword arguments (q, k, sigma_prime,
    map_kind, mode, words_per_lane) plus the sample's median scan time in ms
    (``sample_ms``, not a Plan argument). Options: map_kinds, max_q, max_k,
    table_budget, repeats, max_candidates, modes, fixed_tiles."""
    p = _as_patterns(patterns)
    _check_text(sample)
    o = _tune_opts(**opts)
    best = MagParams()
    ms = ctypes.c_float(0.0)
    check(lib().mag_autotune(p.ctypes.data if p.size else None, p.shape[0], p.shape[1],
                             ctypes.byref(o), ctypes.c_void_p(sample.data_ptr()), sample.numel(),
                             ctypes.byref(best), ctypes.byref(ms), _stream_ptr(stream)),
          "mag_autotune")
    return {**_plan_kwargs(best), "sample_ms": ms.value}


def autotune_batch(patterns, texts, *, sample_bytes: int = 0, stream=None, **opts):
    """``mag_autotune_batch``: per-job Plan keyword arguments (one tuned pick
    per job class) and the batched kernel's words per lane, for jobs given as
    pattern arrays and uint8 CUDA text tensors. Returns (list of dicts,
    words_per_lane)."""
    pats = [_as_patterns(p) for p in patterns]
    texts = list(texts)
    if len(pats) != len(texts):
        raise ValueError("one text per pattern set")
    for t in texts:
        _check_text(t)
    nj = len(pats)
    jobs = (MagJob * max(nj, 1))()
    for j, t in enumerate(texts):
        jobs[j].plan = None
        jobs[j].d_text = t.data_ptr() or None
        jobs[j].n = t.numel()
    pp = (ctypes.c_void_p * max(nj, 1))(*[p.ctypes.data if p.size else None for p in pats])
    rr = (ctypes.c_uint32 * max(nj, 1))(*[p.shape[0] for p in pats])
    mm = (ctypes.c_uint32 * max(nj, 1))(*[p.shape[1] for p in pats])
    out = (MagParams * max(nj, 1))()
    wpl = ctypes.c_int32(0)
    o = _tune_opts(**opts)
    check(lib().mag_autotune_batch(jobs, pp, rr, mm, nj, ctypes.byref(o), int(sample_bytes), out,
                                   ctypes.byref(wpl), _stream_ptr(stream)), "mag_autotune_batch")
    return [_plan_kwargs(out[j]) for j in range(nj)], wpl.value


# ------------------------------------------------------------------ learned selection

SEL_FEATURES = 16
SEL_CANDIDATES = 64      # network outputs
SEL_CHOICES = 32         # outputs 0..31: the choices' costs; 32..63: their verifications


def select_features(patterns) -> np.ndarray:
    """The selector's 16 features of a pattern set (``mag_select_features``)."""
    p = _as_patterns(patterns)
    out = np.empty(SEL_FEATURES, dtype=np.float32)
    check(lib().mag_select_features(p.ctypes.data if p.size else None, p.shape[0], p.shape[1],
                                    out.ctypes.data), "mag_select_features")
    return out


def _choice(prm: MagParams):
    if prm.mode == MODE["dense"]:
        return ("dense", 0, 0, 0)
    if prm.map_kind == MAP_KIND["qgram"]:
        return ("qgram", 0, 0, 0)
    return ("filter", prm.q, prm.k, prm.sigma_prime)


def choice_kwargs(choice) -> dict:
    """Plan keyword arguments of a selector choice (kind, q, k, sigma')."""
    kind, q, k, sp = choice
    if kind == "dense":
        return {"select": "learned", "mode": "dense"}
    if kind == "qgram":
        return {"select": "learned", "map_kind": "qgram", "mode": "filter"}
    return {"select": "learned", "q": q, "k": k, "sigma_prime": sp, "map_kind": "greedy",
            "mode": "filter"}


def select_candidates(patterns):
    """The selector's 64 output slots for a set: (kind, q, k, sigma') for
    the feasible choices among slots 0..31 (kind "dense", "qgram" or
    "filter"), None elsewhere."""
    p = _as_patterns(patterns)
    prm = (MagParams * SEL_CANDIDATES)()
    feas = np.zeros(SEL_CANDIDATES, dtype=np.uint8)
    check(lib().mag_select_candidates(p.ctypes.data if p.size else None, p.shape[0], p.shape[1],
                                      ctypes.cast(prm, ctypes.c_void_p), feas.ctypes.data),
          "mag_select_candidates")
    return [_choice(prm[c]) if feas[c] else None for c in range(SEL_CANDIDATES)]


class Selector:
    """The learned parameter selector (``mag_mlp_*``): 16 features -> 64 ReLU ->
    64 ReLU -> predicted cost of each of the 64 candidate triples."""

    def __init__(self, params=None):
        h = ctypes.c_void_p()
        self._h = None
        check(lib().mag_mlp_create(ctypes.byref(h)), "mag_mlp_create")
        self._h = h
        self.n_params = int(lib().mag_mlp_param_count())
        if params is not None:
            self.set_params(params)

    @classmethod
    def load(cls, path: str | None = None) -> "Selector":
        """The trained network shipped with the package (or the .npz at path)."""
        import os
        path = path or os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_model.npz")
        with np.load(path, allow_pickle=False) as z:
            return cls(z["params"])

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("selector is closed")
        return self._h

    def set_params(self, params) -> None:
        p = np.ascontiguousarray(params, dtype=np.float32).reshape(-1)
        if p.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {p.size}")
        check(lib().mag_mlp_set_params(self.handle, p.ctypes.data), "mag_mlp_set_params")

    def get_params(self) -> np.ndarray:
        p = np.empty(self.n_params, dtype=np.float32)
        check(lib().mag_mlp_get_params(self.handle, p.ctypes.data), "mag_mlp_get_params")
        return p

    def forward(self, x, stream=None):
        """x: float32 CUDA tensor [B, 16] -> [B, 64] predicted costs."""
        import torch
        y = torch.empty((x.shape[0], SEL_CANDIDATES), dtype=torch.float32, device=x.device)
        check(lib().mag_mlp_forward(self.handle, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                    ctypes.c_void_p(y.data_ptr()), _stream_ptr(stream)),
              "mag_mlp_forward")
        return y

    def grad(self, x, t, mask, stream=None):
        """Gradient and loss of the masked mean squared error (CUDA tensors)."""
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        check(lib().mag_mlp_grad(self.handle, ctypes.c_void_p(x.data_ptr()),
                                 ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(mask.data_ptr()),
                                 x.shape[0], ctypes.c_void_p(g.data_ptr()),
                                 ctypes.c_void_p(loss.data_ptr()), _stream_ptr(stream)),
              "mag_mlp_grad")
        return g, loss

    def adam(self, grad, lr: float, stream=None) -> None:
        check(lib().mag_mlp_adam(self.handle, ctypes.c_void_p(grad.data_ptr()), float(lr),
                                 _stream_ptr(stream)), "mag_mlp_adam")

    def train_step(self, x, t, mask, lr: float, loss=None, stream=None) -> None:
        check(lib().mag_mlp_train_step(self.handle, ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(t.data_ptr()),
                                       ctypes.c_void_p(mask.data_ptr()), x.shape[0], float(lr),
                                       ctypes.c_void_p(loss.data_ptr()) if loss is not None else None,
                                       _stream_ptr(stream)), "mag_mlp_train_step")

    def select(self, x, feasible, stream=None):
        """Per row the cheapest feasible candidate (int32 CUDA tensor, -1 if none)."""
        import torch
        pick = torch.empty(x.shape[0], dtype=torch.int32, device=x.device)
        check(lib().mag_mlp_select(self.handle, ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(feasible.data_ptr()), x.shape[0],
                                   ctypes.c_void_p(pick.data_ptr()), _stream_ptr(stream)),
              "mag_mlp_select")
        return pick

    def pick(self, patterns, stream=None) -> dict:
        """Parameters for one set (``mag_select_learned``), ready for :class:`Plan`."""
        p = _as_patterns(patterns)
        out = MagParams()
        check(lib().mag_select_learned(self.handle, p.ctypes.data if p.size else None, p.shape[0],
                                       p.shape[1], ctypes.byref(out), _stream_ptr(stream)),
              "mag_select_learned")
        if out.select == SELECT["learned"]:
            return choice_kwargs(_choice(out))
        return {"select": "heuristic"}

    def picks(self, pattern_sets, threads: int = 16, stream=None, batch: bool = False) -> list[dict]:
        """Parameters for many sets: features on host threads, one selection
        launch for all of them. batch=True leaves out the q-gram map, which
        batches do not take."""
        import concurrent.futures as cf
        import torch
        sets = [_as_patterns(p) for p in pattern_sets]

        def prep(p):
            if p.shape[0] == 0:
                return np.zeros(SEL_FEATURES, np.float32), [None] * SEL_CANDIDATES
            return select_features(p), select_candidates(p)
        with cf.ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
            prepped = list(ex.map(prep, sets))
        X = np.stack([f for f, _ in prepped]).astype(np.float32)
        F = np.array([[c is not None and not (batch and c[0] == "qgram") for c in cand]
                      for _, cand in prepped], dtype=np.uint8)
        xd = torch.from_numpy(X).cuda()
        fd = torch.from_numpy(F).cuda()
        pk = self.select(xd, fd, stream).cpu().numpy()
        out = []
        for (_, cand), c in zip(prepped, pk):
            if c < 0:
                out.append({"select": "heuristic"})
            else:
                out.append({**choice_kwargs(cand[c]), "candidate": int(c)})
        return out

    def close(self):
        if self._h is not None:
            lib().mag_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
