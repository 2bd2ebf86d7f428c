"""Helpers for the GPU tests: host numpy <-> device torch tensors of u32."""
import sys

import numpy as np


def to_dev(a: np.ndarray):
    import torch
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32).copy()).cuda()


def to_host(t) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def sync():
    import torch
    torch.cuda.synchronize()


def announce(msg: str) -> None:
    """Name the case on stdout before its GPU work starts."""
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()
