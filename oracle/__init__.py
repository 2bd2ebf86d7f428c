"""CPU oracle for the stable LSD radix sort -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links
or calls it, and the two share no code.

Two independent definitions live here:

* ``lsd_sort`` / ``counting_pass`` / ``digit_histogram`` /
  ``lsd_sort_segmented``: ctypes wrappers over ``lsd_oracle.c``, a plain
  single-threaded LSD radix sort written from Sections 3 and 4 of Wassenberg
  & Sanders (naive counting sort per digit, digits least significant first,
  stable scatter in input order).
* ``reverse_sort``: Section 4's "reverse sorting" (Algorithm 2 on one
  processing element): an MSD partition into growable buckets, then each
  bucket sorted locally by LSD on the three lower digits, the last pass
  writing straight to the output.  Its buckets are filled by appending, not
  by counting, so it shares no step with ``lsd_sort`` beyond digit
  extraction.
* ``lsd_sort64``: the same LSD sort on 64-bit keys (digit widths summing
  to 64) with values of zero, one or two 32-bit words per item.
* ``brute_stable_sort``: the rank definition of the stable ascending sort
  in pure Python, O(n^2), for tiny inputs.

The shared library is compiled with gcc by :func:`build`; :func:`lib`
compiles it only when no built copy exists.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lsd_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

DEFAULT_WIDTHS: Tuple[int, ...] = (8, 8, 8, 8)

_lib: Optional[ctypes.CDLL] = None


def build(out_path: str = _SO, mutant: int = 0) -> str:
    """Compile lsd_oracle.c with gcc -O2 into ``out_path``.

    ``mutant`` > 0 plants one of the deliberate mistakes guarded by
    ``ORACLE_MUTANT`` in the C source; the test suite uses those builds to
    show that its pins catch each of them.
    """
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC"]
    if mutant:
        cmd.append(f"-DORACLE_MUTANT={int(mutant)}")
    tmp = out_path + f".tmp{os.getpid()}"
    cmd += [_SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out_path)
    return out_path


def _bind(so: ctypes.CDLL) -> ctypes.CDLL:
    u32p = ctypes.POINTER(ctypes.c_uint32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    uintp = ctypes.POINTER(ctypes.c_uint)
    so.oracle_digit_histogram.argtypes = [u32p, ctypes.c_uint64, ctypes.c_uint,
                                          ctypes.c_uint, u64p]
    so.oracle_counting_pass.argtypes = [u32p, u32p, u32p, u32p, ctypes.c_uint64,
                                        ctypes.c_uint, ctypes.c_uint]
    so.oracle_lsd_sort.argtypes = [u32p, u32p, ctypes.c_uint64, uintp, ctypes.c_uint]
    so.oracle_lsd_sort_segmented.argtypes = [u32p, u32p, u32p, ctypes.c_uint32,
                                             uintp, ctypes.c_uint]
    so.oracle_reverse_sort.argtypes = [u32p, u32p, ctypes.c_uint64]
    so.oracle_lsd_sort64.argtypes = [u64p, u32p, ctypes.c_uint, ctypes.c_uint64, uintp, ctypes.c_uint]
    for f in (so.oracle_digit_histogram, so.oracle_counting_pass,
              so.oracle_lsd_sort, so.oracle_lsd_sort_segmented, so.oracle_reverse_sort,
              so.oracle_lsd_sort64):
        f.restype = ctypes.c_int
    return so


def load(path: str) -> ctypes.CDLL:
    """Load an oracle build (the default one or a planted-mistake build)."""
    return _bind(ctypes.CDLL(path))


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = load(_SO)
    return _lib


def _u32(a) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype != np.uint32:
        a = a.astype(np.uint32)
    return a


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def _widths_arg(widths: Sequence[int]):
    arr = (ctypes.c_uint * len(widths))(*[int(w) for w in widths])
    return arr, len(widths)


def digit_histogram(keys, shift: int, width: int, so: Optional[ctypes.CDLL] = None) -> np.ndarray:
    """Counts of each value of bits [shift, shift+width) over the keys."""
    so = so or lib()
    k = _u32(keys)
    hist = np.zeros(1 << width, dtype=np.uint64)
    rc = so.oracle_digit_histogram(_ptr(k), k.size, shift, width,
                                   hist.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    _check(rc, "digit_histogram")
    return hist


def counting_pass(keys, vals, shift: int, width: int,
                  so: Optional[ctypes.CDLL] = None):
    """One stable counting-sort pass on one digit; returns new arrays."""
    so = so or lib()
    k = _u32(keys)
    ko = np.empty_like(k)
    v = None if vals is None else _u32(vals)
    vo = None if v is None else np.empty_like(v)
    rc = so.oracle_counting_pass(_ptr(k), _ptr(v), _ptr(ko), _ptr(vo), k.size, shift, width)
    _check(rc, "counting_pass")
    return ko, vo


def lsd_sort(keys, vals=None, widths: Sequence[int] = DEFAULT_WIDTHS,
             so: Optional[ctypes.CDLL] = None):
    """Stable LSD radix sort; returns (sorted_keys, moved_values or None)."""
    so = so or lib()
    k = _u32(keys).copy()
    v = None if vals is None else _u32(vals).copy()
    if v is not None and v.size != k.size:
        raise ValueError("keys and values differ in length")
    w, np_ = _widths_arg(widths)
    rc = so.oracle_lsd_sort(_ptr(k), _ptr(v), k.size, w, np_)
    _check(rc, "lsd_sort")
    return k, v


def lsd_sort_segmented(keys, vals, offsets, widths: Sequence[int] = DEFAULT_WIDTHS,
                       so: Optional[ctypes.CDLL] = None):
    """Sort every segment [off[s], off[s+1]) independently."""
    so = so or lib()
    k = _u32(keys).copy()
    v = None if vals is None else _u32(vals).copy()
    off = _u32(offsets)
    if off.size < 1:
        raise ValueError("offsets need at least one entry")
    if int(off[-1]) > k.size:
        raise ValueError("offsets run past the arrays")
    w, np_ = _widths_arg(widths)
    rc = so.oracle_lsd_sort_segmented(_ptr(k), _ptr(v), _ptr(off), off.size - 1, w, np_)
    _check(rc, "lsd_sort_segmented")
    return k, v


def reverse_sort(keys, vals=None, so: Optional[ctypes.CDLL] = None):
    """MSD partition then per-bucket LSD (32-bit keys, 8-bit digits);
    returns (sorted_keys, moved_values or None)."""
    so = so or lib()
    k = _u32(keys).copy()
    v = None if vals is None else _u32(vals).copy()
    if v is not None and v.size != k.size:
        raise ValueError("keys and values differ in length")
    rc = so.oracle_reverse_sort(_ptr(k), _ptr(v), k.size)
    _check(rc, "reverse_sort")
    return k, v


DEFAULT_WIDTHS64: Tuple[int, ...] = (8,) * 8


def lsd_sort64(keys, vals=None, widths: Sequence[int] = DEFAULT_WIDTHS64,
               so: Optional[ctypes.CDLL] = None):
    """Stable LSD radix sort of 64-bit keys; vals (optional) is uint32 of
    shape [n] or [n, 2] (one or two words per item) and moves with its key.
    Returns (sorted_keys, moved_values or None)."""
    so = so or lib()
    k = np.ascontiguousarray(keys, dtype=np.uint64).copy()
    v = None
    vw = 0
    if vals is not None:
        v = np.ascontiguousarray(vals, dtype=np.uint32).copy()
        if v.shape[0] != k.size or v.ndim not in (1, 2) or (v.ndim == 2 and v.shape[1] != 2):
            raise ValueError("values must be [n] or [n, 2] uint32")
        vw = 1 if v.ndim == 1 else 2
    w, np_ = _widths_arg(widths)
    rc = so.oracle_lsd_sort64(k.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), _ptr(v), vw, k.size, w, np_)
    _check(rc, "lsd_sort64")
    return k, v


def brute_stable_sort(keys: Sequence[int], vals: Optional[Sequence[int]] = None, bits: int = 32):
    """Stable ascending sort by its rank definition, in pure Python.

    rank(i) = #{j : k_j < k_i} + #{j < i : k_j == k_i}; item i goes to slot
    rank(i).  Keys are taken as unsigned `bits`-bit integers.  Quadratic:
    for tiny inputs only.
    """
    ks = [int(x) & ((1 << bits) - 1) for x in keys]
    n = len(ks)
    out_k = [0] * n
    out_v = None if vals is None else [0] * n
    for i in range(n):
        r = 0
        for j in range(n):
            if ks[j] < ks[i] or (ks[j] == ks[i] and j < i):
                r += 1
        out_k[r] = ks[i]
        if out_v is not None:
            out_v[r] = int(vals[i])
    return out_k, out_v
