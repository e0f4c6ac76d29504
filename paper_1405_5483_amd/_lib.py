"""ctypes declarations mirroring ``include/mag.h``.

Loading fails loudly when ``libmag.so`` has not been built: there is no
fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmag.so")

MAG_OK = 0
MAG_E_INVALID = -1
MAG_E_UNSUPPORTED = -2
MAG_E_NOMEM = -3
MAG_E_DEVICE = -4
MAG_E_OVERFLOW = -5

SELECT = {"heuristic": 0, "explicit": 1, "learned": 2, "autotune": 3}
MAP_KIND = {"greedy": 0, "rank": 1, "bits": 2, "qgram": 3}
VERIFY = {"auto": 0, "inline": 1, "deferred": 2}
MODE = {"auto": 0, "filter": 1, "dense": 2}
DENSE_PROBE = {"auto": 0, "slices": 1, "bloom": 2}


class MagParams(ctypes.Structure):
    _fields_ = [
        ("select", ctypes.c_int32),
        ("map_kind", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("sigma_prime", ctypes.c_int32),
        ("table_budget", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("verify", ctypes.c_int32),
        ("verify_buffer", ctypes.c_int32),
        ("encode", ctypes.c_int32),
        ("chunk_bytes", ctypes.c_int32),
        ("words_per_lane", ctypes.c_int32),
        ("dense_probe", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 3),
    ]


class MagMatch(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_uint64), ("pattern_id", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class MagPlanDesc(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_int32), ("k", ctypes.c_int32), ("sigma_prime", ctypes.c_int32),
        ("L", ctypes.c_int32), ("m_prime", ctypes.c_int32), ("W", ctypes.c_int32),
        ("entry_bytes", ctypes.c_int32), ("map_kind", ctypes.c_int32), ("select", ctypes.c_int32),
        ("r", ctypes.c_uint32), ("m", ctypes.c_uint32), ("n_unique", ctypes.c_uint32),
        ("dense", ctypes.c_int32), ("bloom_log2", ctypes.c_int32),
        ("bits_shift", ctypes.c_int32), ("entry_bits", ctypes.c_int32),
        ("n_codes", ctypes.c_uint64), ("table_bytes", ctypes.c_uint64),
        ("est_verif", ctypes.c_double), ("m_max", ctypes.c_uint32), ("var", ctypes.c_uint32),
        ("q_formula", ctypes.c_int32), ("dense_slices", ctypes.c_int32),
        ("dense_pass", ctypes.c_double),
    ]


class MagJob(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("d_text", ctypes.c_void_p), ("n", ctypes.c_uint64)]


class MagTuneOpts(ctypes.Structure):
    _fields_ = [
        ("map_kinds", ctypes.c_int32), ("max_q", ctypes.c_int32), ("max_k", ctypes.c_int32),
        ("table_budget", ctypes.c_int64), ("repeats", ctypes.c_int32),
        ("max_candidates", ctypes.c_int32), ("modes", ctypes.c_int32),
        ("fixed_tiles", ctypes.c_int32), ("batch_only", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class MagStats(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_uint64), ("cand_windows", ctypes.c_uint64),
                ("verifications", ctypes.c_uint64), ("matches", ctypes.c_uint64),
                ("q", ctypes.c_int32), ("k", ctypes.c_int32), ("sigma_prime", ctypes.c_int32),
                ("m_prime", ctypes.c_int32), ("plan_ms", ctypes.c_float), ("scan_ms", ctypes.c_float)]


# name -> (restype, argtypes); every function declared in include/mag.h
SIGNATURES = {
    "mag_plan_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                       ctypes.POINTER(MagParams), ctypes.POINTER(ctypes.c_void_p)]),
    "mag_plan_destroy": (None, [ctypes.c_void_p]),
    "mag_plan_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MagPlanDesc)]),
    "mag_plan_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(MagParams)]),
    "mag_scan_batch": (ctypes.c_int, [ctypes.POINTER(MagJob), ctypes.c_uint32, ctypes.c_void_p,
                                      ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p]),
    "mag_plan_export": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_uint64]),
    "mag_plan_create_var": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                           ctypes.c_void_p, ctypes.c_void_p]),
    "mag_stream_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "mag_stream_read_sink_words": (ctypes.c_uint32, []),
    "mag_encode": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                  ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                  ctypes.c_void_p]),
    "mag_scan_async": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                      ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p]),
    "mag_scan_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                        ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "mag_scan": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                ctypes.c_void_p, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64),
                                ctypes.POINTER(MagStats), ctypes.c_void_p]),
    "mag_batch_set_words_per_lane": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "mag_batch_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "mag_batch_destroy": (None, [ctypes.c_void_p]),
    "mag_batch_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_uint64, ctypes.c_void_p]),
    "mag_batch_run_async": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]),
    "mag_select_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.c_void_p]),
    "mag_select_candidates": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_void_p, ctypes.c_void_p]),
    "mag_mlp_param_count": (ctypes.c_uint32, []),
    "mag_mlp_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p)]),
    "mag_mlp_destroy": (None, [ctypes.c_void_p]),
    "mag_mlp_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mag_mlp_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "mag_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    "mag_mlp_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p]),
    "mag_mlp_adam": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_float,
                                    ctypes.c_void_p]),
    "mag_mlp_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_uint32, ctypes.c_float,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "mag_mlp_select": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]),
    "mag_select_learned": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32,
                                          ctypes.c_uint32, ctypes.POINTER(MagParams),
                                          ctypes.c_void_p]),
    "mag_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.POINTER(MagTuneOpts), ctypes.c_void_p, ctypes.c_uint64,
                                    ctypes.POINTER(MagParams), ctypes.POINTER(ctypes.c_float),
                                    ctypes.c_void_p]),
    "mag_autotune_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_uint32, ctypes.POINTER(MagTuneOpts),
                                          ctypes.c_uint64, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]),
    "mag_profile_enable": (ctypes.c_int, [ctypes.c_int]),
    "mag_profile_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "mag_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "mag_last_error": (ctypes.c_char_p, []),
    "mag_version": (ctypes.c_int32, []),
}


class MagError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{status}: {detail}")
        self.status = status
        self.detail = detail


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1405_5483_amd.build` "
                "(there is no fallback path)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status: int, what: str = "") -> int:
    if status != MAG_OK:
        detail = lib().mag_last_error().decode(errors="replace")
        raise MagError(status, f"{what}: {detail}" if what else detail)
    return status
