"""Python binding of librtsort: argument marshalling only.

Every function takes torch tensors that live on the GPU (dtype uint32 or
int32, bit patterns read as unsigned 32-bit keys), hands their device
pointers and the current HIP stream to the C ABI, and returns.  All sorting
work happens in the library's HIP kernels; there is no other implementation.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Sequence

from . import _lib
from ._lib import RtConfig, RtGenParams, check, lib

FLAG_NO_SKIP = _lib.RT_FLAG_NO_SKIP
FLAG_NT_STORES = _lib.RT_FLAG_NT_STORES
FLAG_DIRECT_SCATTER = _lib.RT_FLAG_DIRECT_SCATTER
FLAG_ONE_CHAIN = _lib.RT_FLAG_ONE_CHAIN
FLAG_CHUNKS = _lib.RT_FLAG_CHUNKS
FLAG_VALIDATE = _lib.RT_FLAG_VALIDATE
FLAG_FUSED_HISTOGRAM = _lib.RT_FLAG_FUSED_HISTOGRAM
MAX_DIGIT_BITS = _lib.RT_MAX_DIGIT_BITS
MAX_PASSES = _lib.RT_MAX_PASSES


@dataclasses.dataclass
class Config:
    """Sort configuration; zeros / empty mean "tuned default"."""
    digit_bits: Sequence[int] = ()
    block_threads: int = 0
    items_per_thread: int = 0
    flags: int = 0

    def to_c(self) -> RtConfig:
        c = RtConfig()
        c.num_passes = len(self.digit_bits)
        for i, w in enumerate(self.digit_bits):
            c.digit_bits[i] = int(w)
        c.block_threads = int(self.block_threads)
        c.items_per_thread = int(self.items_per_thread)
        c.flags = int(self.flags)
        return c

    @staticmethod
    def from_c(c: RtConfig) -> "Config":
        return Config(tuple(int(c.digit_bits[i]) for i in range(c.num_passes)),
                      int(c.block_threads), int(c.items_per_thread), int(c.flags))


def _torch():
    import torch
    return torch


def _check_tensor(t, name: str):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype not in (torch.int32, torch.uint32):
        raise TypeError(f"{name} must be int32 or uint32, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def current_stream(device=None) -> int:
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


def _stream(stream) -> Optional[int]:
    if stream is None:
        return current_stream()
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _cfg_ptr(cfg: Optional[Config]):
    if cfg is None:
        return None, None
    c = cfg.to_c()
    return c, ctypes.byref(c)


def sort_keys(keys, stream=None) -> None:
    """Sort a 1-D uint32/int32 GPU tensor in place (unsigned order)."""
    _check_tensor(keys, "keys")
    check(lib().rt_sort_keys(_ptr(keys), keys.numel(), _stream(stream)), "rt_sort_keys")


def sort_pairs(keys, vals, stream=None) -> None:
    """Sort keys in place and move vals with them (stable)."""
    _check_tensor(keys, "keys")
    _check_tensor(vals, "vals")
    if vals.numel() != keys.numel():
        raise ValueError("keys and vals differ in length")
    check(lib().rt_sort_pairs(_ptr(keys), _ptr(vals), keys.numel(), _stream(stream)), "rt_sort_pairs")


def workspace_bytes(n: int, with_values: bool, cfg: Optional[Config] = None) -> int:
    c, p = _cfg_ptr(cfg)
    return int(lib().rt_workspace_bytes(n, 1 if with_values else 0, p))


def sort_ex(keys, vals=None, cfg: Optional[Config] = None, workspace=None, stream=None) -> None:
    """Sort with an explicit configuration and (optionally) a caller-owned
    workspace tensor of at least workspace_bytes() bytes."""
    _check_tensor(keys, "keys")
    _check_tensor(vals, "vals")
    if vals is not None and vals.numel() != keys.numel():
        raise ValueError("keys and vals differ in length")
    c, p = _cfg_ptr(cfg)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr = workspace.data_ptr()
        ws_bytes = workspace.numel() * workspace.element_size()
    check(lib().rt_sort_pairs_ex(_ptr(keys), _ptr(vals), keys.numel(), p, ws_ptr, ws_bytes, _stream(stream)),
          "rt_sort_pairs_ex")


def sort_noalloc(keys, vals=None, cfg: Optional[Config] = None, stream=None) -> None:
    """The sort of sort_ex with the library's static scratch as workspace:
    no device allocation (at most rt_workspace_bytes() <= 64 MiB of work)."""
    _check_tensor(keys, "keys")
    _check_tensor(vals, "vals")
    if vals is not None and vals.numel() != keys.numel():
        raise ValueError("keys and vals differ in length")
    c, p = _cfg_ptr(cfg)
    check(lib().rt_sort_pairs_noalloc(_ptr(keys), _ptr(vals), keys.numel(), p, _stream(stream)),
          "rt_sort_pairs_noalloc")


def _check_tensor64(t, name: str, dtypes):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} must be one of {dtypes}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def sort64_ex(keys, vals=None, cfg: Optional[Config] = None, workspace=None, stream=None) -> None:
    """Sort 64-bit keys (an int64/uint64 GPU tensor holding u64 bit
    patterns) in place, stably, moving vals (None, or int32/uint32 for
    4-byte values, int64/uint64 for 8-byte values) with them."""
    torch = _torch()
    _check_tensor64(keys, "keys", (torch.int64, torch.uint64))
    _check_tensor64(vals, "vals", (torch.int32, torch.uint32, torch.int64, torch.uint64))
    vb = 0 if vals is None else vals.element_size()
    if vals is not None and vals.numel() != keys.numel():
        raise ValueError("keys and vals differ in length")
    c, p = _cfg_ptr(cfg)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr = workspace.data_ptr()
        ws_bytes = workspace.numel() * workspace.element_size()
    check(lib().rt_sort64_ex(_ptr(keys), _ptr(vals), vb, keys.numel(), p, ws_ptr, ws_bytes, _stream(stream)),
          "rt_sort64_ex")


def sort_keys64(keys, stream=None) -> None:
    """Sort a 1-D int64/uint64 GPU tensor in place (unsigned 64-bit order)."""
    torch = _torch()
    _check_tensor64(keys, "keys", (torch.int64, torch.uint64))
    check(lib().rt_sort_keys64(_ptr(keys), keys.numel(), _stream(stream)), "rt_sort_keys64")


def sort_pairs64(keys, vals, stream=None) -> None:
    """Sort 64-bit keys in place and move 32-bit vals with them (stable)."""
    torch = _torch()
    _check_tensor64(keys, "keys", (torch.int64, torch.uint64))
    _check_tensor(vals, "vals")
    if vals.numel() != keys.numel():
        raise ValueError("keys and vals differ in length")
    check(lib().rt_sort_pairs64(_ptr(keys), _ptr(vals), keys.numel(), _stream(stream)), "rt_sort_pairs64")


def workspace_bytes64(n: int, value_bytes: int, cfg: Optional[Config] = None) -> int:
    c, p = _cfg_ptr(cfg)
    return int(lib().rt_workspace_bytes64(n, value_bytes, p))


def sort_pairs_batched(keys, vals, offsets, max_total: Optional[int] = None, stream=None) -> None:
    """Sort every segment [offsets[s], offsets[s+1]) independently (stable).
    vals may be None; offsets is a device tensor of num_segments + 1 entries."""
    _check_tensor(keys, "keys")
    _check_tensor(vals, "vals")
    _check_tensor(offsets, "offsets")
    if offsets.numel() < 1:
        raise ValueError("offsets needs num_segments + 1 entries")
    total = keys.numel() if max_total is None else int(max_total)
    check(lib().rt_sort_pairs_batched(_ptr(keys), _ptr(vals), _ptr(offsets), offsets.numel() - 1, total,
                                      _stream(stream)), "rt_sort_pairs_batched")


def batched_workspace_bytes(num_segments: int, max_total: int, with_values: bool = True) -> int:
    return int(lib().rt_batched_workspace_bytes(num_segments, max_total, 1 if with_values else 0))


def sort_batched_ex(keys, vals, offsets, max_total: Optional[int] = None, validate: bool = False,
                    workspace=None, stream=None) -> None:
    """Batched sort with an optional caller workspace (graph-capturable) and
    optional validation of the offsets (waits for the device)."""
    _check_tensor(keys, "keys")
    _check_tensor(vals, "vals")
    _check_tensor(offsets, "offsets")
    if offsets.numel() < 1:
        raise ValueError("offsets needs num_segments + 1 entries")
    total = keys.numel() if max_total is None else int(max_total)
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr = workspace.data_ptr()
        ws_bytes = workspace.numel() * workspace.element_size()
    check(lib().rt_sort_batched_ex(_ptr(keys), _ptr(vals), _ptr(offsets), offsets.numel() - 1, total,
                                   _lib.RT_FLAG_VALIDATE if validate else 0, ws_ptr, ws_bytes, _stream(stream)),
          "rt_sort_batched_ex")


def msd_first_workspace_bytes(n: int, with_values: bool = True) -> int:
    return int(lib().rt_msd_first_workspace_bytes(n, 1 if with_values else 0))


def sort_msd_first(keys, vals=None, validate: bool = False, workspace=None, stream=None,
                   levels: Optional[int] = None) -> None:
    """In-place stable sort by MSD partition passes, then LSD passes over the
    lower digits of each bucket (the paper's reverse sorting).  levels: 1 (one
    partition, then digits 0..2 of each of 256 buckets), 2 (a second
    partition on digit 2, then digits 0..1 of each of 65536 sub-buckets) or
    None (the library picks by size)."""
    if levels not in (None, 1, 2):
        raise ValueError("levels must be None, 1 or 2")
    _check_tensor(keys, "keys")
    _check_tensor(vals, "vals")
    if vals is not None and vals.numel() != keys.numel():
        raise ValueError("keys and vals differ in length")
    ws_ptr, ws_bytes = None, 0
    if workspace is not None:
        ws_ptr = workspace.data_ptr()
        ws_bytes = workspace.numel() * workspace.element_size()
    flags = (_lib.RT_FLAG_VALIDATE if validate else 0) | {None: 0, 1: _lib.RT_FLAG_MSD_ONE_LEVEL,
                                                           2: _lib.RT_FLAG_MSD_TWO_LEVELS}[levels]
    check(lib().rt_sort_msd_first(_ptr(keys), _ptr(vals), keys.numel(), flags, ws_ptr, ws_bytes, _stream(stream)),
          "rt_sort_msd_first")


def digit_histograms(keys, cfg: Optional[Config] = None, stream=None):
    """Per-pass digit counts, shape [passes, 2^MAX_DIGIT_BITS] (uint32 as int32)."""
    torch = _torch()
    _check_tensor(keys, "keys")
    passes = len(cfg.digit_bits) if cfg is not None and cfg.digit_bits else tuned_config(
        keys.numel(), False).digit_bits.__len__()
    hist = torch.empty((MAX_PASSES, 1 << MAX_DIGIT_BITS), dtype=torch.int32, device=keys.device)
    c, p = _cfg_ptr(cfg)
    check(lib().rt_digit_histograms(_ptr(keys), keys.numel(), p, hist.data_ptr(), _stream(stream)),
          "rt_digit_histograms")
    return hist[:passes]


def chunk_decision(keys, with_values: bool = True, cfg: Optional[Config] = None, value_bytes: int = 4,
                   stream=None) -> int:
    """The XCD-chunk decision a sort of these keys makes: 1 = chunks, 0 = one
    chain.  u32 keys ask for the 32-bit sort's decision (with or without
    values), u64 keys for the 64-bit sort's with value_bytes of 0, 4 or 8."""
    torch = _torch()
    _check_tensor64(keys, "keys", (torch.int32, torch.uint32, torch.int64, torch.uint64))
    mode = torch.full((1,), -1, dtype=torch.int32, device=keys.device)
    c, p = _cfg_ptr(cfg)
    if keys.element_size() == 8:
        check(lib().rt_chunk_decision64(_ptr(keys), keys.numel(), value_bytes, p, mode.data_ptr(), _stream(stream)),
              "rt_chunk_decision64")
    else:
        check(lib().rt_chunk_decision(_ptr(keys), keys.numel(), 1 if with_values else 0, p, mode.data_ptr(),
                                      _stream(stream)), "rt_chunk_decision")
    return int(mode.item())


def counting_pass(kin, vin, kout, vout, shift: int, width: int, stream=None) -> None:
    """One stable counting-sort pass on bits [shift, shift+width), out of place."""
    for t, nm in ((kin, "kin"), (vin, "vin"), (kout, "kout"), (vout, "vout")):
        _check_tensor(t, nm)
    check(lib().rt_counting_pass(_ptr(kin), _ptr(vin), _ptr(kout), _ptr(vout), kin.numel(), shift, width,
                                 _stream(stream)), "rt_counting_pass")


def copy(src, dst, stream=None) -> None:
    """Streaming device copy (the bandwidth probe)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst is smaller than src")
    check(lib().rt_copy(src.data_ptr(), dst.data_ptr(), nbytes, _stream(stream)), "rt_copy")


def bandwidth_probe(kind: int, src=None, dst=None, sink=None, stream=None) -> None:
    """One bandwidth probe (_lib.RT_PROBE_*) over the bytes of src (copy,
    read) or dst (write); sink: a device word the read probe may write."""
    t = src if src is not None else dst
    nbytes = t.numel() * t.element_size()
    check(lib().rt_bandwidth_probe(None if src is None else src.data_ptr(), None if dst is None else dst.data_ptr(),
                                   nbytes, int(kind), None if sink is None else sink.data_ptr(), _stream(stream)),
          "rt_bandwidth_probe")


def gen_params_to_c(p) -> RtGenParams:
    """Convert inputs.CounterGenParams to the C struct."""
    g = RtGenParams()
    g.dist = int(p.dist)
    g.state = int(p.state) & ((1 << 64) - 1)
    for i, x in enumerate(p.dictionary):
        g.dictionary[i] = int(x)
    for i, x in enumerate(p.thresholds):
        g.thresholds[i] = int(x)
    return g


def generate(keys, vals, params, value_base: int = 0, stream=None) -> None:
    """Fill keys (and vals = value_base + i) from the counter-based generator."""
    _check_tensor(keys, "keys")
    _check_tensor(vals, "vals")
    g = gen_params_to_c(params)
    check(lib().rt_generate(_ptr(keys), _ptr(vals), keys.numel(), ctypes.byref(g), int(value_base),
                            _stream(stream)), "rt_generate")


def load_tuning(path: Optional[str]) -> None:
    check(lib().rt_load_tuning(None if path is None else path.encode()), "rt_load_tuning")


def load_default_tuning() -> None:
    """Back to the table the library loads on first use: RT_TUNING_FILE, else
    the committed table for gfx950, else the built-in defaults."""
    so = lib()
    check(so.rt_load_tuning(None), "rt_load_tuning")
    _lib._load_default_tuning(so)


def tuned_config(n: int, with_values: bool) -> Config:
    c = RtConfig()
    check(lib().rt_tuned_config(n, 1 if with_values else 0, ctypes.byref(c)), "rt_tuned_config")
    return Config.from_c(c)


def segment_classes():
    """The segmented sort's whole-in-LDS size classes in force:
    [(max_n, block, ipt), ...] in increasing max_n."""
    count = ctypes.c_uint32(0)
    arrs = [(ctypes.c_uint32 * 4)() for _ in range(3)]
    check(lib().rt_segment_classes(ctypes.byref(count), *arrs), "rt_segment_classes")
    return [(int(arrs[0][c]), int(arrs[1][c]), int(arrs[2][c])) for c in range(count.value)]


def segment_config():
    """(digit bits of each whole-in-LDS class, (tile threads, tile items per
    thread) of the tiled segments' passes) in force."""
    count = ctypes.c_uint32(0)
    check(lib().rt_segment_classes(ctypes.byref(count), None, None, None), "rt_segment_classes")
    bits = (ctypes.c_uint32 * 4)()
    tb, ti = ctypes.c_uint32(0), ctypes.c_uint32(0)
    check(lib().rt_segment_config(bits, ctypes.byref(tb), ctypes.byref(ti)), "rt_segment_config")
    return [int(bits[c]) for c in range(count.value)], (int(tb.value), int(ti.value))


def version() -> str:
    return lib().rt_version().decode()


def profile_start(max_marks: int = 4096) -> None:
    """Start recording a HIP event after every kernel the library launches."""
    check(lib().rt_profile_start(int(max_marks)), "rt_profile_start")


def profile_stop(capacity: int = 4096):
    """Stop recording; returns [(kind, milliseconds)] per launch in order."""
    kinds = (ctypes.c_uint32 * capacity)()
    ms = (ctypes.c_float * capacity)()
    count = ctypes.c_uint32(0)
    check(lib().rt_profile_stop(kinds, ms, capacity, ctypes.byref(count)), "rt_profile_stop")
    return [(int(kinds[i]), float(ms[i])) for i in range(count.value)]
