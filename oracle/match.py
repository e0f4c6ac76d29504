"""ctypes front end of ``occ.c`` (test infrastructure only).

``occ_hashed`` and ``occ_brute`` return the occurrence set of Section 1,
``{(i, id) : T[i..i+m) == P_id}``, as two arrays sorted by ``(i, id)``.
``occ_var`` and ``occ_var_python`` drop the equal-length requirement (the
introduction notes it may be removed): ``{(i, id) : T[i..i+m_id) == P_id}``.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "occ.c")
_LIB = os.path.join(_HERE, "_occ.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile ``occ.c`` into ``_occ.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-pthread",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            lib = ctypes.CDLL(build())
            vp, u64, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32
            lib.occ_hashed.restype = vp
            lib.occ_hashed.argtypes = [vp, u64, vp, u32, u32, ctypes.c_int]
            lib.occ_brute.restype = vp
            lib.occ_brute.argtypes = [vp, u64, vp, u32, u32]
            lib.occ_size.restype = u64
            lib.occ_size.argtypes = [vp]
            lib.occ_failed.restype = ctypes.c_int
            lib.occ_failed.argtypes = [vp]
            lib.occ_copy.restype = None
            lib.occ_copy.argtypes = [vp, vp, vp]
            lib.occ_free.restype = None
            lib.occ_free.argtypes = [vp]
            _lib = lib
    return _lib


def _prep(text, patterns):
    t = np.ascontiguousarray(np.frombuffer(text, dtype=np.uint8) if isinstance(text, (bytes, bytearray)) else text, dtype=np.uint8)
    if isinstance(patterns, (list, tuple)):
        patterns = np.array([np.frombuffer(p, dtype=np.uint8) for p in patterns], dtype=np.uint8)
    p = np.ascontiguousarray(patterns, dtype=np.uint8)
    if p.ndim != 2:
        raise ValueError("patterns must be a [r, m] array")
    return t, p


def _collect(lib, h):
    if not h:
        raise MemoryError("oracle allocation failed")
    try:
        if lib.occ_failed(h):
            raise MemoryError("oracle allocation failed")
        z = lib.occ_size(h)
        pos = np.empty(z, dtype=np.uint64)
        ids = np.empty(z, dtype=np.uint32)
        if z:
            lib.occ_copy(h, pos.ctypes.data, ids.ctypes.data)
        return pos, ids
    finally:
        lib.occ_free(h)


def occ_hashed(text, patterns, threads: int | None = None):
    """Hashed matcher; ``threads`` defaults to ``os.cpu_count()``."""
    lib = _load()
    t, p = _prep(text, patterns)
    r, m = p.shape
    nt = threads if threads else (os.cpu_count() or 1)
    h = lib.occ_hashed(t.ctypes.data, t.size, p.ctypes.data, r, m, nt)
    return _collect(lib, h)


def occ_brute(text, patterns):
    """O(n r m) double loop; for tiny inputs."""
    lib = _load()
    t, p = _prep(text, patterns)
    r, m = p.shape
    h = lib.occ_brute(t.ctypes.data, t.size, p.ctypes.data, r, m)
    return _collect(lib, h)


def occ_python(text, patterns):
    """Pure-Python double loop over bytes objects, for the smallest cases; an
    implementation independent of the C code."""
    t = bytes(np.asarray(text, dtype=np.uint8))
    pats = [bytes(row) for row in np.asarray(patterns, dtype=np.uint8)]
    m = len(pats[0]) if pats else 0
    pos, ids = [], []
    if m:
        for i in range(len(t) - m + 1):
            w = t[i:i + m]
            for pid, pat in enumerate(pats):
                if w == pat:
                    pos.append(i)
                    ids.append(pid)
    return np.array(pos, dtype=np.uint64), np.array(ids, dtype=np.uint32)


def occ_at(text, patterns, i: int) -> np.ndarray:
    """Ids of every pattern occurring at start position ``i`` (ascending)."""
    t, p = _prep(text, patterns)
    r, m = p.shape
    if i < 0 or i + m > t.size:
        return np.empty(0, dtype=np.uint32)
    return np.nonzero((p == t[i:i + m][None, :]).all(axis=1))[0].astype(np.uint32)


def occ_var(text, patterns, threads: int | None = None):
    """Occurrences of patterns of unequal lengths (a list of byte strings or
    uint8 arrays): the equal-length matcher run on each group of patterns of
    one length, its ids mapped back to the list's, merged and sorted by
    (pos, id)."""
    pats = [np.frombuffer(bytes(p), dtype=np.uint8) if not isinstance(p, np.ndarray)
            else np.asarray(p, dtype=np.uint8) for p in patterns]
    by_len: dict[int, list[int]] = {}
    for pid, pat in enumerate(pats):
        if pat.size == 0:
            raise ValueError("empty pattern")
        by_len.setdefault(int(pat.size), []).append(pid)
    allpos, allids = [], []
    for length, members in sorted(by_len.items()):
        group = np.stack([pats[pid] for pid in members])
        pos, ids = occ_hashed(text, group, threads)
        allpos.append(pos)
        allids.append(np.asarray(members, dtype=np.uint32)[ids.astype(np.int64)])
    if not allpos:
        return np.empty(0, dtype=np.uint64), np.empty(0, dtype=np.uint32)
    pos = np.concatenate(allpos)
    ids = np.concatenate(allids)
    order = np.lexsort((ids, pos))
    return pos[order], ids[order]


def occ_var_python(text, patterns):
    """Pure-Python double loop over start positions and patterns of any
    lengths, for the smallest cases."""
    t = bytes(np.asarray(text, dtype=np.uint8))
    pats = [bytes(p) for p in patterns]
    pos, ids = [], []
    for i in range(len(t)):
        for pid, pat in enumerate(pats):
            if i + len(pat) <= len(t) and t[i:i + len(pat)] == pat:
                pos.append(i)
                ids.append(pid)
    return np.array(pos, dtype=np.uint64), np.array(ids, dtype=np.uint32)
