"""Autotuner: measures the library's compiled sort configurations on this
GPU and writes the tuning table that rt_load_tuning() reads.

    python -m paper_1008_2849_amd.autotune --out paper_1008_2849_amd/tuning/gfx950.json
    python -m paper_1008_2849_amd.autotune --out ... --ops segments   # keep the other entries

Single-array sorts ("keys", "pairs"): at each measured size it times every
(digit widths, tile shape, store flavour) the library has kernels for and
keeps the fastest; entries cover size ranges split at the geometric
midpoints between measured sizes.  Each candidate's output is checked
against a stable argsort of the same keys on the device before its time
counts, so a configuration can only win by sorting correctly.

Segmented sort ("segments"): for each size range (2^(k-1), 2^k], k = 6..14,
it sorts a batch of about 2^23 items in segments of sizes uniform in the
range, once with each whole-in-LDS kernel shape that holds 2^k items under
each digit width it is built for (four 8-bit passes, or 11/11/10), and once
with the range left to the tiled path under each tile (1024x16, 512x16),
and keeps the fastest (each output must equal the built-in classes' output
bit for bit).  The classes are at most four contiguous runs of ranges, one
shape and digit width each, ending where tiling wins (the split with the
least per-segment time, found by dynamic programming).  The split and the
built-in classes are then timed on the batched workload's log-uniform mix
with either tile, and the fastest pair is written: the "segments" entries
(with their digit widths) and a "segments_tiled" entry (the tile).
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
SHAPES = {8: [(256, 16), (512, 16), (1024, 8), (1024, 12), (1024, 16), (512, 32)],
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
                except Exception as e:  # a shape the library lacks, or a wrong result
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


# whole-in-LDS shapes the library compiles; keep in step with
# RT_FOR_EACH_SEG_SMALL_SHAPE in csrc/rt_common.h
SEG_SHAPES = [(64, 4), (64, 8), (128, 4), (128, 8), (256, 4), (256, 8), (512, 4), (512, 8), (256, 16),
              (128, 9), (256, 9), (256, 17), (512, 16), (1024, 8), (1024, 16)]
# the 11-bit ones (11-bit counters need 8 KiB a wave: at most 512 threads)
SEG_SHAPES_11 = [(64, 4), (64, 8), (128, 4), (128, 8), (256, 4), (256, 8), (256, 16), (512, 4), (512, 8),
                 (512, 16)]
SEG_RANGES = list(range(6, 15))  # (2^(k-1), 2^k]
SEG_BATCH_ITEMS = 1 << 23


SEG_BITS = {8: (8, 8, 8, 8), 11: (11, 11, 10)}
SEG_TILES = [(1024, 16), (512, 16)]  # tiles of the tiled segments' passes; keep in step with rt_common.h


def seg_small_supported(b, i, bits):
    """Whether the library compiles the whole-in-LDS kernel b x i with
    bits-bit digits."""
    return (b, i) in (SEG_SHAPES if bits == 8 else SEG_SHAPES_11)


def _segment_table(classes, tile=(1024, 16)):
    """classes: [(max_n, block, ipt, bits)]; tile: (block, ipt) of the tiled passes."""
    entries = [{"op": "segments", "min_n": 0, "max_n": m, "digit_bits": list(SEG_BITS[bits]),
                "block": b, "ipt": i} for m, b, i, bits in classes]
    entries.append({"op": "segments_tiled", "min_n": 0, "max_n": 0, "digit_bits": [8, 8, 8, 8],
                    "block": tile[0], "ipt": tile[1]})
    return {"entries": entries}


def _time_batched(keys0, vals0, off, n, classes, reps, check, tmpdir, tile=(1024, 16), latencies=False):
    """Median call time (ms, from the library's kernel marks) of a batched
    sort under the given classes and tile, after checking its output (with
    latencies: also the sorted per-call times)."""
    import os
    import torch
    path = os.path.join(tmpdir, "seg_candidate.json")
    with open(path, "w") as f:
        json.dump(_segment_table(classes, tile), f)
    api.load_tuning(path)
    ws = torch.empty(api.batched_workspace_bytes(off.numel() - 1, n, True), dtype=torch.uint8, device=keys0.device)
    slots = [(keys0.clone(), vals0.clone()) for _ in range(reps + 1)]
    api.sort_batched_ex(slots[0][0], slots[0][1], off, n, workspace=ws)
    torch.cuda.synchronize()
    if check is not None and not (torch.equal(slots[0][0], check[0]) and torch.equal(slots[0][1], check[1])):
        raise RuntimeError(f"classes {classes}, tile {tile} sorted incorrectly")
    api.profile_start(64 * reps + 64)
    for k, v in slots[1:]:
        api.sort_batched_ex(k, v, off, n, workspace=ws)
    torch.cuda.synchronize()
    calls, cur = [], None
    for kind, ms in api.profile_stop(64 * reps + 64):
        if kind == 0:
            cur = [0.0]
            calls.append(cur)
        elif cur is not None:
            cur[0] += ms
    times = sorted(c[0] for c in calls)
    if latencies:
        return times[len(times) // 2], times
    return times[len(times) // 2], (slots[0][0], slots[0][1])


def _key(b, i, bits):
    return f"{b}x{i}@{bits}"


def tune_segments(reps, log=print):
    """Whole-in-LDS size classes of the segmented sort (shape and digit width
    per class) and the tile of its tiled passes; returns (entries, report)."""
    import tempfile
    import numpy as np
    import torch
    from . import inputs
    rng = np.random.default_rng(1234)
    report = []
    with tempfile.TemporaryDirectory() as tmpdir:
        for k in SEG_RANGES:
            lo, hi = (1 << (k - 1)) + 1, 1 << k
            count = max(1, SEG_BATCH_ITEMS // ((lo + hi) // 2))
            sizes = rng.integers(lo, hi + 1, size=count)
            off_h = np.zeros(count + 1, dtype=np.uint32)
            off_h[1:] = np.cumsum(sizes)
            n = int(off_h[-1])
            keys0 = torch.from_numpy(inputs.uniform_keys(n, 800 + k).view(np.int32)).cuda()
            vals0 = torch.arange(n, dtype=torch.int32, device="cuda")
            off = torch.from_numpy(off_h.view(np.int32)).cuda()
            api.load_tuning(None)  # the reference output: built-in classes (parity-tested)
            ref = keys0.clone(), vals0.clone()
            api.sort_pairs_batched(ref[0], ref[1], off, n)
            torch.cuda.synchronize()
            times = {}
            for b, i in SEG_SHAPES:
                if b * i < hi:
                    continue
                for bits in SEG_BITS:
                    if not seg_small_supported(b, i, bits):
                        continue
                    t, _ = _time_batched(keys0, vals0, off, n, [(hi, b, i, bits)], reps, ref, tmpdir)
                    times[_key(b, i, bits)] = t
                    log(f"  segments ({lo}..{hi}] x{count}: {b}x{i} {bits}-bit digits {t:.4f} ms")
            # one class that ends below the range: every segment of it is tiled
            for tb, ti in SEG_TILES:
                t, _ = _time_batched(keys0, vals0, off, n, [(lo - 1, 1024, 16, 8)], reps, ref, tmpdir, (tb, ti))
                times[f"tiled@{tb}x{ti}"] = t
                log(f"  segments ({lo}..{hi}] x{count}: tiled {tb}x{ti} {t:.4f} ms")
            times["tiled"] = min(v for c, v in times.items() if c.startswith("tiled@"))
            best = min((c for c in times if c != "tiled"), key=times.get)
            report.append({"op": "segments", "range": [lo, hi], "segments": count, "items": n,
                           "best": best, "ms": {c: round(v, 4) for c, v in times.items()}})
            del keys0, vals0, off, ref
            torch.cuda.empty_cache()
    api.load_tuning(None)
    entries = segment_entries(report)
    # the split and the tile must also pay off on a mix of sizes: the batched
    # workload (log-uniform sizes) under the split and under the built-in
    # classes, each with either tile
    sizes = inputs.batched_sizes()
    off_h = np.zeros(len(sizes) + 1, dtype=np.uint32)
    off_h[1:] = np.cumsum(sizes)
    n = int(off_h[-1])
    keys0 = torch.from_numpy(inputs.uniform_keys(n, inputs.SEED_BATCHED).view(np.int32)).cuda()
    vals0 = torch.arange(n, dtype=torch.int32, device="cuda")
    off = torch.from_numpy(off_h.view(np.int32)).cuda()
    ref = keys0.clone(), vals0.clone()
    api.sort_pairs_batched(ref[0], ref[1], off, n)
    torch.cuda.synchronize()
    split = [(e["max_n"], e["block"], e["ipt"], 8 if e["digit_bits"][0] == 8 else 11) for e in entries]
    builtin = [(2048, 256, 8, 8), (8192, 512, 16, 8), (16384, 1024, 16, 8)]
    results = {}
    with tempfile.TemporaryDirectory() as tmpdir:
        for name, cls in (("split", split), ("builtin", builtin)):
            for tile in SEG_TILES:
                t, _ = _time_batched(keys0, vals0, off, n, cls, max(reps, 9), ref, tmpdir, tile)
                results[(name, tile)] = t
                log(f"  batched workload: {name} classes, tile {tile[0]}x{tile[1]}: {t:.4f} ms")
    api.load_tuning(None)
    (chosen, tile), t_best = min(results.items(), key=lambda kv: kv[1])
    log(f"  batched workload: {chosen} classes with tile {tile[0]}x{tile[1]} ({t_best:.4f} ms)")
    report.append({"op": "segments_workload", "segments": len(sizes), "items": n,
                   "split": [list(c) for c in split],
                   "ms": {f"{nm} tile {tl[0]}x{tl[1]}": round(v, 4) for (nm, tl), v in results.items()},
                   "chosen": chosen, "tile": list(tile)})
    if chosen == "builtin":
        entries = [{"op": "segments", "min_n": lo + 1, "max_n": m, "digit_bits": list(SEG_BITS[bits]), "block": b,
                    "ipt": i, "flags": 0} for lo, (m, b, i, bits) in zip([0, 2048, 8192], builtin)]
    entries.append({"op": "segments_tiled", "min_n": 0, "max_n": 0, "digit_bits": [8, 8, 8, 8],
                    "block": tile[0], "ipt": tile[1], "flags": 0})
    return entries, report


def segment_entries(report):
    """Size classes from the per-range measurements of tune_segments.

    The ranges are split, from the smallest up, into at most four
    contiguous classes, each sorted by one whole-in-LDS shape and digit
    width (a "BxI@bits" candidate) that holds its largest range, with every
    range above the last class left to the tiled path.  Among all such
    splits (by dynamic programming over the ranges) the one with the least
    total time per segment wins; per-segment times (a range's time over its
    segment count) weigh the ranges as a log-uniform size mix does.
    """
    rows = sorted((r for r in report if r["op"] == "segments"), key=lambda r: r["range"][1])
    if not rows:
        return []
    per_seg = [{c: t / r["segments"] for c, t in r["ms"].items()} for r in rows]
    shapes = sorted({c for r in rows for c in r["ms"] if not c.startswith("tiled")},
                    key=lambda c: [int(x) for x in c.replace("@", "x").split("x")])
    cap = {c: int(c.split("x")[0]) * int(c.split("x")[1].split("@")[0]) for c in shapes}
    R = len(rows)
    tiled_tail = [0.0] * (R + 1)  # ranges i.. left to the tiled path
    for i in range(R - 1, -1, -1):
        tiled_tail[i] = tiled_tail[i + 1] + per_seg[i]["tiled"]

    def span(i, j):  # ranges i..j as one class: its best candidate and cost
        best = None
        for c in shapes:
            if cap[c] < rows[j]["range"][1] or any(c not in per_seg[q] for q in range(i, j + 1)):
                continue
            cost = sum(per_seg[q][c] for q in range(i, j + 1))
            if best is None or cost < best[0]:
                best = (cost, c)
        return best

    # best[k][j]: least cost of ranges 0..j-1 split into k classes
    INF = float("inf")
    best = [[(INF, None)] * (R + 1) for _ in range(5)]
    best[0][0] = (0.0, None)
    for k in range(1, 5):
        for j in range(1, R + 1):
            for i in range(j):
                prev = best[k - 1][i][0]
                sp = span(i, j - 1)
                if prev == INF or sp is None:
                    continue
                if prev + sp[0] < best[k][j][0]:
                    best[k][j] = (prev + sp[0], (i, sp[1]))
    choice = None
    for k in range(1, 5):
        for j in range(1, R + 1):
            total = best[k][j][0] + tiled_tail[j]
            if choice is None or total < choice[0]:
                choice = (total, k, j)
    classes = []
    _, k, j = choice
    while k > 0:
        i, c = best[k][j][1]
        classes.append((rows[j - 1]["range"][1], c))
        k, j = k - 1, i
    classes.reverse()
    entries, prev = [], 0
    for max_n, c in classes:
        shape, bits = c.split("@")
        b, i = (int(x) for x in shape.split("x"))
        entries.append({"op": "segments", "min_n": prev + 1, "max_n": max_n, "digit_bits": list(SEG_BITS[int(bits)]),
                        "block": b, "ipt": i, "flags": 0})
        prev = max_n
    return entries


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--sizes", default=",".join(str(int(math.log2(s))) for s in SIZES),
                    help="comma list of log2 sizes")
    ap.add_argument("--ops", default="keys,pairs,segments",
                    help="what to tune; the --out table's other entries are kept")
    args = ap.parse_args(argv)
    import os
    import torch
    if not torch.cuda.is_available():
        print("autotune: no GPU visible", file=sys.stderr)
        return 1
    ops = set(args.ops.split(","))
    old = {"entries": [], "measurements": []}
    if os.path.exists(args.out):
        with open(args.out) as f:
            old = json.load(f)
    sizes = [1 << int(x) for x in args.sizes.split(",")]
    api.load_tuning(None)  # measure every candidate from the built-in defaults
    log = lambda m: print(m, flush=True)
    single_ops = ops & {"keys", "pairs"}
    if single_ops:
        entries, report = tune(sizes, args.reps, log=log)
        entries = [e for e in entries if e["op"] in single_ops]
        report = [r for r in report if r["op"] in single_ops]
    else:
        entries, report = [], []
    if "segments" in ops:
        seg_entries, seg_report = tune_segments(args.reps, log=log)
        entries += seg_entries
        report += seg_report
    tuned = {e["op"] for e in entries} | ops
    if "segments" in tuned:
        tuned |= {"segments_workload", "segments_tiled"}
    entries = [e for e in old.get("entries", []) if e["op"] not in tuned] + entries
    report = [r for r in old.get("measurements", []) if r.get("op") not in tuned] + report
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
