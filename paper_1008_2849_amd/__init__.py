"""paper_1008_2849_amd: stable LSD radix sort of 32-bit keys (optionally with
32-bit values) on AMD MI355X (gfx950), after Wassenberg & Sanders, "Faster
Radix Sort via Virtual Memory and Write-Combining" (arXiv:1008.2849).

The sort runs in hand-written HIP kernels inside librtsort.so (C ABI in
include/rtsort.h); this package binds it for torch GPU tensors.  Importing
the package does not load the library; the first call does, and fails if it
is not built.
"""
from __future__ import annotations

__all__ = [
    "Config", "sort_keys", "sort_pairs", "sort_ex", "sort_noalloc", "bandwidth_probe", "sort_pairs_batched",
    "sort_batched_ex", "batched_workspace_bytes", "workspace_bytes", "sort_msd_first",
    "msd_first_workspace_bytes", "sort_keys64", "sort_pairs64", "sort64_ex", "workspace_bytes64",
    "segment_classes", "segment_config", "digit_histograms", "chunk_decision", "counting_pass", "copy",
    "generate", "load_tuning", "load_default_tuning", "tuned_config", "version", "Server", "RtError",
    "profile_start", "profile_stop",
]


def __getattr__(name):
    if name == "Server":
        from .server import Server
        return Server
    if name == "RtError":
        from ._lib import RtError
        return RtError
    if name in __all__:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
