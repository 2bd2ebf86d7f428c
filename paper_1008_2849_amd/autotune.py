"""Autotuner: measures the library's compiled sort configurations on this
GPU and writes the tuning table that rt_load_tuning() reads.

    python -m paper_1008_2849_amd.autotune --out paper_1008_2849_amd/tuning/gfx950.json

For keys-only and key/value sorts at each size class it times every
(digit widths, tile shape, store flavour) the library has kernels for and
keeps the fastest.  Each candidate's output is checked against a stable
argsort of the same keys on the device before its time counts, so a
configuration can only win by sorting correctly.  Entries cover size
ranges split at the geometric midpoints between measured sizes.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

from . import api
from .api import Config, FLAG_NT_STORES

# (bits class, threads, items per thread) the library compiles; keep in step
# with RT_FOR_EACH_SHAPE in csrc/rt_common.h
SHAPES = {8: [(256, 16), (512, 16), (1024, 8), (1024, 12), (1024, 16)],
          11: [(256, 16), (512, 8), (512, 16)]}
WIDTHS = [(8, 8, 8, 8), (11, 11, 10)]
SIZES = [1 << 16, 1 << 20, 1 << 24, 1 << 28]


def candidates():
    for w in WIDTHS:
        cls = 8 if max(w) <= 8 else 11
        for block, ipt in SHAPES[cls]:
            for flags in (0, FLAG_NT_STORES):
                yield Config(w, block, ipt, flags)


def time_config(cfg, keys0, vals0, reps, check):
    import torch
    n = keys0.numel()
    ws = torch.empty(api.workspace_bytes(n, vals0 is not None, cfg), dtype=torch.uint8, device=keys0.device)
    k = keys0.clone()
    v = None if vals0 is None else vals0.clone()
    api.sort_ex(k, v, cfg, ws)
    torch.cuda.synchronize()
    if check is not None and not (torch.equal(k, check[0]) and (v is None or torch.equal(v, check[1]))):
        raise RuntimeError(f"{cfg} sorted incorrectly")
    times = []
    for _ in range(reps):
        k.copy_(keys0)
        if v is not None:
            v.copy_(vals0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.sort_ex(k, v, cfg, ws)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    times.sort()
    return times[len(times) // 2]


def reference(keys0, vals0):
    """Stable ascending order of the keys by torch on the device (u32 via int64)."""
    import torch
    k64 = keys0.to(torch.int64) & 0xFFFFFFFF
    order = torch.sort(k64, stable=True).indices
    return keys0[order], (None if vals0 is None else vals0[order])


def tune(sizes, reps, log=print):
    import numpy as np
    import torch
    from . import inputs
    entries = []
    report = []
    for with_values in (False, True):
        best_by_size = []
        for n in sizes:
            keys = torch.from_numpy(inputs.uniform_keys(n, 900 + int(math.log2(n))).view(np.int32)).cuda()
            vals = torch.arange(n, dtype=torch.int32, device="cuda") if with_values else None
            check = reference(keys, vals)
            r = max(3, reps if n >= (1 << 24) else reps * 4)
            results = []
            for cfg in candidates():
                try:
                    t = time_config(cfg, keys, vals, r, check)
                except Exception as e:  # a shape this build lacks, or a wrong result
                    log(f"  skip {cfg}: {e}")
                    continue
                results.append((t, cfg))
                log(f"  {'pairs' if with_values else 'keys '} n=2^{int(math.log2(n))} {cfg}: {t * 1e3:.3f} ms")
            results.sort(key=lambda x: x[0])
            t, cfg = results[0]
            best_by_size.append((n, cfg, t))
            report.append({"op": "pairs" if with_values else "keys", "n": n, "best": cfg.__dict__,
                           "ms": round(t * 1e3, 4), "Gkeys/s": round(n / t / 1e9, 3),
                           "runner_up_ms": round(results[1][0] * 1e3, 4) if len(results) > 1 else None})
            del keys, vals, check
            torch.cuda.empty_cache()
        for i, (n, cfg, _) in enumerate(best_by_size):
            lo = 0 if i == 0 else int(math.sqrt(best_by_size[i - 1][0] * n)) + 1
            hi = (1 << 32) - 1 if i == len(best_by_size) - 1 else int(math.sqrt(n * best_by_size[i + 1][0]))
            entries.append({"op": "pairs" if with_values else "keys", "min_n": lo, "max_n": hi,
                            "digit_bits": list(cfg.digit_bits), "block": cfg.block_threads,
                            "ipt": cfg.items_per_thread, "flags": cfg.flags})
    return entries, report


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--sizes", default=",".join(str(int(math.log2(s))) for s in SIZES),
                    help="comma list of log2 sizes")
    args = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        print("autotune: no GPU visible", file=sys.stderr)
        return 1
    sizes = [1 << int(x) for x in args.sizes.split(",")]
    api.load_tuning(None)  # measure every candidate from the built-in defaults
    entries, report = tune(sizes, args.reps, log=lambda m: print(m, flush=True))
    table = {"arch": "gfx950", "device": torch.cuda.get_device_name(0),
             "cus": torch.cuda.get_device_properties(0).multi_processor_count,
             "library": api.version(), "entries": entries, "measurements": report}
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    api.load_tuning(args.out)  # the library accepts what was written
    print(f"wrote {args.out}: {len(entries)} entries", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
