"""ctypes front end of ``occ.c`` (test infrastructure only).

``occ_hashed`` and ``occ_brute`` return the occurrence set of Section 1,
``{(i, id) : T[i..i+m) == P_id}``, as two arrays sorted by ``(i, id)``.
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
