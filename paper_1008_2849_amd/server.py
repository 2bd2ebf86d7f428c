"""Python handle of the library's serving loop (rt_server_* in rtsort.h).

Every step of the loop runs in the library's scheduler thread and HIP
kernels; this class only marshals arguments.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Tuple

from . import _lib
from ._lib import RtGenParams, check, lib


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Server:
    """Sorts requests submitted one by one; see rt_server_create."""

    def __init__(self, hbm_budget_bytes: int, max_active: int = 4096):
        h = ctypes.c_void_p()
        check(lib().rt_server_create(int(hbm_budget_bytes), int(max_active), ctypes.byref(h)), "rt_server_create")
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("server is closed")
        return self._h

    def submit(self, keys, vals=None, out_keys=None, out_vals=None) -> int:
        """Sort device tensors keys (and vals); returns a ticket.  The result
        replaces the inputs, or goes to out_keys / out_vals when given (the
        inputs are then only read).  Every tensor must stay alive and
        untouched until a wait reports the request."""
        for t, name in ((keys, "keys"), (vals, "vals"), (out_keys, "out_keys"), (out_vals, "out_vals")):
            if t is not None and (not t.is_cuda or t.element_size() != 4 or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous 4-byte device tensor")
            if t is not None and t.numel() != keys.numel():
                raise ValueError(f"{name} differs in length from keys")
        ticket = ctypes.c_uint64()
        check(lib().rt_server_submit(self.handle, _ptr(keys), _ptr(vals), _ptr(out_keys), _ptr(out_vals),
                                     keys.numel(), ctypes.byref(ticket)), "rt_server_submit")
        return ticket.value

    def submit_generated(self, params: RtGenParams, n: int) -> int:
        """A request whose input the server generates on the device."""
        ticket = ctypes.c_uint64()
        check(lib().rt_server_submit_generated(self.handle, ctypes.byref(params), int(n), ctypes.byref(ticket)),
              "rt_server_submit_generated")
        return ticket.value

    def wait(self, ticket: int, timeout_us: int = -1) -> float:
        """Block until the request is done; returns its latency in us."""
        lat = ctypes.c_double()
        check(lib().rt_server_wait(self.handle, int(ticket), int(timeout_us), ctypes.byref(lat)), "rt_server_wait")
        return lat.value

    def wait_any(self, timeout_us: int = -1):
        """(ticket, latency us) of the next request to finish, in completion order."""
        t, lat = ctypes.c_uint64(), ctypes.c_double()
        check(lib().rt_server_wait_any(self.handle, int(timeout_us), ctypes.byref(t), ctypes.byref(lat)),
              "rt_server_wait_any")
        return t.value, lat.value

    def replay(self, arrivals_s, sizes, params):
        """Open-loop replay of an arrival trace (rt_server_replay): request i,
        of sizes[i] generated pairs with generator parameters params[i]
        (RtGenParams), is submitted by a native thread arrivals_s[i] seconds
        after the start.  Returns (latencies in us from each scheduled
        arrival to completion, span in us from the start to the last
        completion)."""
        import numpy as np
        from ._lib import RtReplayRequest
        count = len(sizes)
        reqs = (RtReplayRequest * count)()
        base = ctypes.addressof(reqs)
        size = ctypes.sizeof(RtReplayRequest)
        arr = np.frombuffer((ctypes.c_uint8 * (count * size)).from_address(base), dtype=np.uint8)
        arr = arr.reshape(count, size)
        arr[:, 0:8] = np.ascontiguousarray(np.asarray(arrivals_s, dtype=np.float64) * 1e6).view(np.uint8).reshape(count, 8)
        arr[:, 8:16] = np.ascontiguousarray(np.asarray(sizes, dtype=np.uint64)).view(np.uint8).reshape(count, 8)
        off = RtReplayRequest.params.offset
        psize = ctypes.sizeof(RtGenParams)
        for i, p in enumerate(params):  # the generator parameters are copied as raw bytes
            ctypes.memmove(base + i * size + off, ctypes.addressof(p), psize)
        lat = np.full(count, -1.0, dtype=np.float64)
        span = ctypes.c_double()
        check(lib().rt_server_replay(self.handle, ctypes.cast(reqs, ctypes.c_void_p), count,
                                     lat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(span)),
              "rt_server_replay")
        return lat, span.value

    def fetch(self, ticket: int, out_keys, out_vals=None) -> None:
        check(lib().rt_server_fetch(self.handle, int(ticket), _ptr(out_keys), _ptr(out_vals)), "rt_server_fetch")

    def release(self, ticket: int) -> None:
        check(lib().rt_server_release(self.handle, int(ticket)), "rt_server_release")

    def cancel(self, ticket: int) -> None:
        """Cancel a request: it takes no further pass and its wait reports
        RT_ERR_CANCELLED.  Raises RtError (RT_ERR_INVALID_ARG) if it has
        finished or its last pass is under way."""
        check(lib().rt_server_cancel(self.handle, int(ticket)), "rt_server_cancel")

    def stats(self) -> Tuple[float, float, float, int, int]:
        """(p50 us, p99 us, Gkeys/s, completed requests, peak budgeted bytes)."""
        p50, p99, gk = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        done, peak = ctypes.c_uint64(), ctypes.c_size_t()
        check(lib().rt_server_stats_ex(self.handle, ctypes.byref(p50), ctypes.byref(p99), ctypes.byref(gk),
                                       ctypes.byref(done), ctypes.byref(peak)), "rt_server_stats_ex")
        return p50.value, p99.value, gk.value, done.value, peak.value

    def close(self) -> None:
        if self._h is not None:
            check(lib().rt_server_destroy(self._h), "rt_server_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
