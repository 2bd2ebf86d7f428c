"""ctypes declarations of librtsort.so (include/rtsort.h).

Loading fails loudly when the library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtsort.so")

RT_OK = 0
RT_ERR_INVALID_ARG = 1
RT_ERR_TOO_LARGE = 2
RT_ERR_OUT_OF_MEMORY = 3
RT_ERR_HIP = 4
RT_ERR_BUDGET = 5
RT_ERR_UNSUPPORTED = 6
RT_ERR_CANCELLED = 7
RT_ERR_TIMEOUT = 8
RT_ERR_NOT_FOUND = 9

RT_MAX_PASSES = 8
RT_MAX_DIGIT_BITS = 11
RT_FLAG_NO_SKIP = 0x1
RT_FLAG_NT_STORES = 0x2
RT_FLAG_DIRECT_SCATTER = 0x8
RT_FLAG_ONE_CHAIN = 0x10
RT_FLAG_CHUNKS = 0x20
RT_FLAG_FUSED_HISTOGRAM = 0x40
RT_FLAG_MSD_ONE_LEVEL = 0x80
RT_FLAG_MSD_TWO_LEVELS = 0x100
RT_FLAG_VALIDATE = 0x4
RT_PROBE_COPY = 0
RT_PROBE_COPY_NT = 1
RT_PROBE_READ = 2
RT_PROBE_WRITE = 3

RT_KIND_FILL = 1
RT_KIND_HISTOGRAM = 2
RT_KIND_PLAN = 3
RT_KIND_COPY_BACK = 4
RT_KIND_COPY = 5
RT_KIND_GENERATE = 6
RT_KIND_SEGMENTED = 7
RT_KIND_SEG_SMALL = 8
RT_KIND_MSD_PASS = 9
RT_KIND_PROBE = 10
RT_KIND_PASS = 16


class RtConfig(ctypes.Structure):
    _fields_ = [
        ("num_passes", ctypes.c_uint32),
        ("digit_bits", ctypes.c_uint32 * RT_MAX_PASSES),
        ("block_threads", ctypes.c_uint32),
        ("items_per_thread", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
    ]


class RtGenParams(ctypes.Structure):
    _fields_ = [
        ("dist", ctypes.c_uint32),
        ("state", ctypes.c_uint64),
        ("dictionary", ctypes.c_uint32 * 16),
        ("thresholds", ctypes.c_uint64 * 16),
    ]


class RtReplayRequest(ctypes.Structure):
    _fields_ = [
        ("arrival_us", ctypes.c_double),
        ("n", ctypes.c_uint64),
        ("params", RtGenParams),
    ]


class RtError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


_lib = None
_lock = threading.Lock()

vp = ctypes.c_void_p
sz = ctypes.c_size_t
u32 = ctypes.c_uint32
u64 = ctypes.c_uint64
i64 = ctypes.c_int64
dblp = ctypes.POINTER(ctypes.c_double)

# name -> (restype, argtypes)
SIGNATURES = {
    "rt_sort_keys": (ctypes.c_int, [vp, sz, vp]),
    "rt_sort_pairs": (ctypes.c_int, [vp, vp, sz, vp]),
    "rt_workspace_bytes": (sz, [sz, ctypes.c_int, ctypes.POINTER(RtConfig)]),
    "rt_sort_pairs_ex": (ctypes.c_int, [vp, vp, sz, ctypes.POINTER(RtConfig), vp, sz, vp]),
    "rt_sort_pairs_noalloc": (ctypes.c_int, [vp, vp, sz, ctypes.POINTER(RtConfig), vp]),
    "rt_bandwidth_probe": (ctypes.c_int, [vp, vp, sz, u32, vp, vp]),
    "rt_sort_pairs_batched": (ctypes.c_int, [vp, vp, vp, u32, sz, vp]),
    "rt_batched_workspace_bytes": (sz, [u32, sz, ctypes.c_int]),
    "rt_sort_batched_ex": (ctypes.c_int, [vp, vp, vp, u32, sz, u32, vp, sz, vp]),
    "rt_sort_keys64": (ctypes.c_int, [vp, sz, vp]),
    "rt_sort_pairs64": (ctypes.c_int, [vp, vp, sz, vp]),
    "rt_sort64_ex": (ctypes.c_int, [vp, vp, u32, sz, ctypes.POINTER(RtConfig), vp, sz, vp]),
    "rt_workspace_bytes64": (sz, [sz, u32, ctypes.POINTER(RtConfig)]),
    "rt_msd_first_workspace_bytes": (sz, [sz, ctypes.c_int]),
    "rt_segment_classes": (ctypes.c_int, [ctypes.POINTER(u32)] * 4),
    "rt_segment_config": (ctypes.c_int, [ctypes.POINTER(u32)] * 3),
    "rt_sort_msd_first": (ctypes.c_int, [vp, vp, sz, u32, vp, sz, vp]),
    "rt_digit_histograms": (ctypes.c_int, [vp, sz, ctypes.POINTER(RtConfig), vp, vp]),
    "rt_chunk_decision": (ctypes.c_int, [vp, sz, ctypes.c_int, ctypes.POINTER(RtConfig), vp, vp]),
    "rt_chunk_decision64": (ctypes.c_int, [vp, sz, u32, ctypes.POINTER(RtConfig), vp, vp]),
    "rt_counting_pass": (ctypes.c_int, [vp, vp, vp, vp, sz, u32, u32, vp]),
    "rt_copy": (ctypes.c_int, [vp, vp, sz, vp]),
    "rt_generate": (ctypes.c_int, [vp, vp, sz, ctypes.POINTER(RtGenParams), u32, vp]),
    "rt_server_create": (ctypes.c_int, [sz, u32, ctypes.POINTER(vp)]),
    "rt_server_submit": (ctypes.c_int, [vp, vp, vp, vp, vp, sz, ctypes.POINTER(u64)]),
    "rt_server_submit_generated": (ctypes.c_int, [vp, ctypes.POINTER(RtGenParams), sz, ctypes.POINTER(u64)]),
    "rt_server_wait": (ctypes.c_int, [vp, u64, i64, dblp]),
    "rt_server_wait_any": (ctypes.c_int, [vp, i64, ctypes.POINTER(u64), dblp]),
    "rt_server_fetch": (ctypes.c_int, [vp, u64, vp, vp]),
    "rt_server_release": (ctypes.c_int, [vp, u64]),
    "rt_server_cancel": (ctypes.c_int, [vp, u64]),
    "rt_server_stats": (ctypes.c_int, [vp, dblp, dblp, dblp]),
    "rt_server_stats_ex": (ctypes.c_int, [vp, dblp, dblp, dblp, ctypes.POINTER(u64), ctypes.POINTER(sz)]),
    "rt_server_replay": (ctypes.c_int, [vp, vp, sz, dblp, dblp]),
    "rt_server_destroy": (ctypes.c_int, [vp]),
    "rt_profile_start": (ctypes.c_int, [u32]),
    "rt_profile_stop": (ctypes.c_int, [ctypes.POINTER(u32), ctypes.POINTER(ctypes.c_float), u32,
                                       ctypes.POINTER(u32)]),
    "rt_load_tuning": (ctypes.c_int, [ctypes.c_char_p]),
    "rt_tuned_config": (ctypes.c_int, [sz, ctypes.c_int, ctypes.POINTER(RtConfig)]),
    "rt_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rt_last_error": (ctypes.c_char_p, []),
    "rt_version": (ctypes.c_char_p, []),
}


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is not built; run `python -m paper_1008_2849_amd.build` "
                    "(the sort has no non-HIP implementation)")
            so = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                f = getattr(so, name)
                f.restype = res
                f.argtypes = args
            _load_default_tuning(so)
            _lib = so
    return _lib


TUNING_PATH = os.path.join(HERE, "tuning", "gfx950.json")


def _load_default_tuning(so) -> None:
    """The autotuner's table for this GPU (RT_TUNING_FILE overrides the
    path; an empty value keeps the built-in defaults)."""
    path = os.environ.get("RT_TUNING_FILE", TUNING_PATH)
    if path and os.path.exists(path):
        status = so.rt_load_tuning(path.encode())
        if status != RT_OK:
            raise RuntimeError(f"tuning table {path}: {so.rt_last_error().decode(errors='replace')}")


def check(status: int, where: str) -> None:
    if status != RT_OK:
        so = lib()
        detail = so.rt_last_error().decode(errors="replace") or so.rt_status_string(status).decode()
        raise RtError(status, where, detail)
