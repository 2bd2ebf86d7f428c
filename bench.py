#!/usr/bin/env python3
"""Benchmark of the stable LSD radix sort on one MI355X.

A step is one whole sort (upfront histograms, plan, every counting-sort
pass) of 2^28 uniform u32 keys carrying u32 values equal to their original
index, the inputs already resident in HBM.  Each timed step sorts its own
pre-staged copy of the input, so no restore copy sits inside the timed
region.  The run prints one JSON line on stdout: whole-sort throughput
(Gkeys/s), per-pass HBM bandwidth against the chip's peak for the dominant
kernel (the counting-sort pass), and the CPU oracle timed on this host.
Further legs, each reported in the same line and each skippable: the
transfer-inclusive rate, the MSD-first sort of the same input, the batched
workload, 64-bit keys, the paper's Table 1 configurations with and
without the LDS staging (write-combining), and the serving loop.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0  # MI355X HBM3E, AMD published peak
METRIC = "Gkeys/s and HBM GB/s per pass vs peak (2^28 pairs); batched p50/p99 latency"
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1008_2849_amd", "csrc", f)
                  for f in ("rt_kernels.h", "rt_internal.h", "rt_common.h", "rt_sort.hip")]


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counters_from_profiles(digest: str):
    """From the committed rocprofv3 counter summary of the pass: HBM bytes
    per launch (traffic), VALU instructions per item, the share of 32-byte
    write requests and of LDS bank-conflict cycles; all None when that
    summary predates the current kernel source."""
    out = {"traffic": None, "valu_per_item": None, "write_32B_share": None, "lds_bank_conflict_share": None}
    path = os.path.join(PROFILES, "onesweep_pass_pairs_256m_counters.md")
    if not os.path.exists(path):
        return out
    text = open(path).read()
    m = re.search(r"kernel_source_digest:\s*([0-9a-f]+)", text)
    if not m or m.group(1) != digest:
        return out
    for key, name in (("traffic", "traffic_bytes_per_launch"), ("valu_per_item", "valu_per_item"),
                      ("write_32B_share", "write_32B_share"), ("lds_bank_conflict_share", "lds_bank_conflict_share")):
        t = re.search(name + r":\s*([0-9.eE+-]+)", text)
        if t:
            out[key] = float(t.group(1))
    return out


def cpu_model() -> str:
    """The host CPU's model name (/proc/cpuinfo), or "unknown"."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class pinned_to_one_core:
    """Runs the block on one core of this process's allowed set (restored
    afterwards): the oracle is single-threaded, and pinning keeps the
    scheduler from moving it between cores while it is timed."""

    def __enter__(self):
        self.saved = os.sched_getaffinity(0)
        self.core = min(self.saved)
        os.sched_setaffinity(0, {self.core})
        return self

    def __exit__(self, *exc):
        os.sched_setaffinity(0, self.saved)
        return False


def cpu_baseline(keys_h, vals_h, out_k, out_v):
    """Time the CPU oracle (single thread, pinned to one core) on the same
    input; its output also checks the GPU result bit for bit.  Returns
    (seconds, equal, core)."""
    import numpy as np
    import oracle
    with pinned_to_one_core() as pin:
        t0 = time.perf_counter()
        rk, rv = oracle.lsd_sort(keys_h, vals_h)
        dt = time.perf_counter() - t0
    same = bool(np.array_equal(rk, out_k) and (out_v is None or np.array_equal(rv, out_v)))
    return dt, same, pin.core


def split_calls(marks):
    """Group profile marks into calls: [(total ms, [(kind, ms), ...]), ...]."""
    calls = []
    for kind, ms in marks:
        if kind == 0:
            calls.append([0.0, []])
        elif calls:
            calls[-1][0] += ms
            calls[-1][1].append((kind, ms))
    return calls


def bench_workloads(rts, inputs, dev, names, K, W):
    """The other single-array workloads at full size (keys only at 2^28 and
    2^20; the skewed 2^26-pair inputs): whole-sort Gkeys/s, the mean pass
    time and its HBM fraction, the histogram time, and the last timed
    output against the CPU oracle (bit for bit, timed single-threaded on
    one core: the CPU baseline of that workload)."""
    import numpy as np
    import torch
    from paper_1008_2849_amd._lib import RT_KIND_HISTOGRAM, RT_KIND_PASS
    out = []
    for name in names:
        w = inputs.WORKLOADS[name]
        n = w.n
        k_h, v_h = inputs.make_workload(w)
        k0 = torch.from_numpy(k_h.view(np.int32)).to(dev)
        v0 = torch.from_numpy(v_h.view(np.int32)).to(dev) if v_h is not None else None
        tuned = rts.tuned_config(n, w.with_values)
        slots = [(k0.clone(), None if v0 is None else v0.clone()) for _ in range(K + W)]
        ws = torch.empty(rts.workspace_bytes(n, w.with_values, tuned), dtype=torch.uint8, device=dev)
        for i in range(W):
            rts.sort_ex(slots[i][0], slots[i][1], tuned, ws)
        torch.cuda.synchronize()
        # per-kernel times first (HIP events around every kernel), then the
        # same sorts of fresh copies timed without them
        rts.profile_start(max_marks=16 * K + 16)
        for i in range(W, W + K):
            rts.sort_ex(slots[i][0], slots[i][1], tuned, ws)
        torch.cuda.synchronize()
        marks = rts.profile_stop(capacity=16 * K + 16)
        for i in range(W, W + K):
            slots[i][0].copy_(k0)
            if v0 is not None:
                slots[i][1].copy_(v0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(W, W + K):
            rts.sort_ex(slots[i][0], slots[i][1], tuned, ws)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        passes = [ms for kind, ms in marks if RT_KIND_PASS <= kind < RT_KIND_PASS + 8]
        hist = [ms for kind, ms in marks if kind == RT_KIND_HISTOGRAM]
        ko, vo = slots[W + K - 1]
        out_k = ko.cpu().numpy().view(np.uint32)
        out_v = None if vo is None else vo.cpu().numpy().view(np.uint32)
        del slots, ws
        dt, same, core = cpu_baseline(k_h, v_h, out_k, out_v)
        item = 8 if w.with_values else 4
        pm = float(np.mean(passes)) if passes else float("nan")
        gk = n / (wall / K) / 1e9
        out.append({"workload": name, "n": n, "values": w.with_values, "Gkeys/s": round(gk, 3),
                    "ms_per_sort": round(1e3 * wall / K, 4),
                    "passes_per_sort": round(len(passes) / K, 2),
                    "pass_ms": round(pm, 4), "pass_GBps": round(2 * item * n / pm / 1e6, 1),
                    "pass_frac_of_peak": round(2 * item * n / pm / 1e6 / PEAK_HBM_GBPS, 4),
                    "histogram_ms": round(float(np.mean(hist)), 4) if hist else None,
                    "config": {"digit_bits": list(tuned.digit_bits), "block_threads": tuned.block_threads,
                               "items_per_thread": tuned.items_per_thread},
                    "matches_oracle_bit_exact": same,
                    "cpu_oracle": {"seconds": round(dt, 4), "Gkeys/s": round(n / dt / 1e9, 5), "cores": 1,
                                   "pinned_core": core}})
        log(f"{name}: {out[-1]}")
        del k0, v0, ko, vo
        torch.cuda.empty_cache()
    return out


def bench_batched(rts, inputs, dev, K, W, single_gkeys):
    """The batched workload: 4096 segments of log-uniform sizes totalling
    2^27 pairs, one sort call per step, each on its own staged copy.  Timed
    twice: as eager launches (with per-kernel marks) and as one captured
    hipGraph per call, replayed (the reported figure)."""
    import numpy as np
    import torch
    from paper_1008_2849_amd._lib import RT_KIND_PASS
    sizes = inputs.batched_sizes()
    off = np.zeros(len(sizes) + 1, dtype=np.uint64)
    off[1:] = np.cumsum(sizes)
    n = int(off[-1])
    k_h = inputs.uniform_keys(n, inputs.SEED_BATCHED)
    k0 = torch.from_numpy(k_h.view(np.int32)).to(dev)
    v0 = torch.arange(n, dtype=torch.int32, device=dev)
    o = torch.from_numpy(off.astype(np.uint32).view(np.int32)).to(dev)
    slots = [(k0.clone(), v0.clone()) for _ in range(K + W)]
    ws = torch.empty(rts.batched_workspace_bytes(len(sizes), n, True), dtype=torch.uint8, device=dev)
    for i in range(W):
        rts.sort_batched_ex(slots[i][0], slots[i][1], o, n, workspace=ws)
    torch.cuda.synchronize()
    rts.profile_start(max_marks=32 * K + 32)
    t0 = time.perf_counter()
    for i in range(W, W + K):
        rts.sort_batched_ex(slots[i][0], slots[i][1], o, n, workspace=ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    calls = split_calls(rts.profile_stop(capacity=32 * K + 32))
    per_call = [c[0] for c in calls]
    pass_ms = [ms for c in calls for kind, ms in c[1] if RT_KIND_PASS <= kind < RT_KIND_PASS + 8]
    eager_wall = wall
    # the same calls captured as graphs (one per staged copy), then replayed
    for k, v in slots:
        k.copy_(k0)
        v.copy_(v0)
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    graphs = []
    with torch.cuda.stream(cs):
        for k, v in slots:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=cs):
                rts.sort_batched_ex(k, v, o, n, workspace=ws, stream=cs)
            graphs.append(g)
    torch.cuda.current_stream().wait_stream(cs)
    for i in range(W):
        graphs[i].replay()
    torch.cuda.synchronize()
    # each replay bracketed by events on the stream it runs on (back to
    # back, as the wall-clock figure): its latency on the device
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    t0 = time.perf_counter()
    for j, i in enumerate(range(W, W + K)):
        ev[j][0].record()
        graphs[i].replay()
        ev[j][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    replay_ms = [a.elapsed_time(b) for a, b in ev]
    del graphs
    # properties of the last output: within every segment keys ascend, each
    # key arrives with its own index, indices stay in their segment and in
    # order among equal keys
    ko, vo = slots[W + K - 1]
    seg = torch.repeat_interleave(torch.arange(len(sizes), device=dev),
                                  torch.from_numpy(sizes.astype(np.int64)).to(dev))
    vl = vo.to(torch.int64)
    ok = bool(torch.equal(seg[vl], seg)) and bool(torch.equal(k0[vl], ko))
    k64 = ko.to(torch.int64) & 0xFFFFFFFF
    same = seg[1:] == seg[:-1]
    ok &= bool((k64[1:][same] >= k64[:-1][same]).all().item())
    eq = same & (k64[1:] == k64[:-1])
    ok &= bool((vl[1:][eq] > vl[:-1][eq]).all().item())
    cnt = torch.bincount(vl, minlength=n)
    ok &= bool((cnt == 1).all().item())
    del slots, seg, vl, k64, same, eq, cnt
    gk = n / (wall / K) / 1e9
    return {"workload": f"batched_{len(sizes)}_segments_loguniform_2^6..2^20_total_{n}", "n": n,
            "segments": len(sizes), "launch": "one hipGraph replay per call",
            "Gkeys/s": round(gk, 3), "ms_per_call": round(1e3 * wall / K, 4),
            "eager_Gkeys/s": round(n / (eager_wall / K) / 1e9, 3),
            "replay_p50_ms": round(float(np.percentile(replay_ms, 50)), 4),
            "replay_p99_ms": round(float(np.percentile(replay_ms, 99)), 4),
            "eager_call_p50_ms": round(float(np.percentile(per_call, 50)), 4),
            "eager_call_p99_ms": round(float(np.percentile(per_call, 99)), 4),
            "tiled_pass_ms": round(float(np.mean(pass_ms)), 4) if pass_ms else None,
            "size_classes": [list(c) + [b] for c, b in zip(rts.segment_classes(), rts.segment_config()[0])],
            "tiled_tile": list(rts.segment_config()[1]),
            "frac_of_single_array": round(gk / single_gkeys, 4), "parity_properties_ok": ok}


def bench_msd_first(rts, dev, k0, v0, slots, K, W, single_gkeys, ref_k, ref_v):
    """The MSD-first sort on the same workload, with two MSD levels (the
    default at this size: partition passes on digits 3 and 2, then digits 0
    and 1 of each of the 65536 sub-buckets whole in LDS) and with one (one
    partition pass, then LSD passes over the three lower digits of each of
    the 256 buckets); each call on its own re-staged copy, and each form's
    last output must equal the LSD sort's bit for bit."""
    import numpy as np
    import torch
    from paper_1008_2849_amd._lib import RT_KIND_HISTOGRAM, RT_KIND_MSD_PASS, RT_KIND_PASS, RT_KIND_SEG_SMALL
    n = k0.numel()
    ws = torch.empty(rts.msd_first_workspace_bytes(n, v0 is not None), dtype=torch.uint8, device=dev)
    out = {}
    for label, levels in (("two_levels", 2), ("one_level", 1)):
        for k, v in slots:
            k.copy_(k0)
            if v is not None:
                v.copy_(v0)
        for i in range(W):
            rts.sort_msd_first(slots[i][0], slots[i][1], workspace=ws, levels=levels)
        torch.cuda.synchronize()
        rts.profile_start(max_marks=32 * K + 32)
        t0 = time.perf_counter()
        for i in range(W, W + K):
            rts.sort_msd_first(slots[i][0], slots[i][1], workspace=ws, levels=levels)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        calls = split_calls(rts.profile_stop(capacity=32 * K + 32))
        part = [ms for c in calls for kind, ms in c[1] if kind == RT_KIND_MSD_PASS]
        hists = [[ms for kind, ms in c[1] if kind == RT_KIND_HISTOGRAM] for c in calls]
        ko, vo = slots[W + K - 1]
        same = bool(torch.equal(ko, ref_k)) and (vo is None or bool(torch.equal(vo, ref_v)))
        gk = n / (wall / K) / 1e9
        row = {"Gkeys/s": round(gk, 3), "ms_per_call": round(1e3 * wall / K, 4),
               "frac_of_single_array": round(gk / single_gkeys, 4),
               "partition_pass_ms": round(float(np.mean(part)), 4) if part else None,
               "msd_histogram_ms": round(float(np.mean([h[0] for h in hists if h])), 4) if hists else None,
               "bucket_histogram_ms": round(float(np.mean([h[1] for h in hists if len(h) > 1])), 4)
               if hists else None,
               "matches_lsd_sort": same}
        if levels == 2:
            # per call: the digit-2 pass inside the buckets is the largest
            # pass mark; the sub-buckets' tiled passes (none for uniform
            # keys) are the others
            second = [max(ms for kind, ms in c[1] if RT_KIND_PASS <= kind < RT_KIND_PASS + 8) for c in calls]
            local = [sum(ms for kind, ms in c[1] if kind == RT_KIND_SEG_SMALL) for c in calls]
            row["second_partition_pass_ms"] = round(float(np.mean(second)), 4)
            row["sub_bucket_lds_sort_ms"] = round(float(np.mean(local)), 4)
        else:
            local = [ms for c in calls for kind, ms in c[1] if RT_KIND_PASS <= kind < RT_KIND_PASS + 8]
            row["local_pass_ms"] = round(float(np.mean(local)), 4) if local else None
        out[label] = row
    del ws
    res = dict(out["two_levels"])
    res["levels"] = 2
    res["one_level"] = out["one_level"]
    res["note"] = ("default at this size: two MSD levels (digit 3, then digit 2 inside each bucket), then digits "
                   "0 and 1 of each sub-bucket whole in LDS; one_level: one partition, then three local LSD passes")
    return res


def bench_sort64(rts, inputs, dev, K, W):
    """64-bit keys: 2^28 uniform u64 keys carrying u32 index values, eight
    8-bit passes, each timed call on its own pre-staged copy."""
    import numpy as np
    import torch
    from paper_1008_2849_amd._lib import RT_KIND_HISTOGRAM, RT_KIND_PASS
    w = inputs.WORKLOADS["pairs64_256m_uniform"]
    n = w.n
    k_h, _ = inputs.make_workload(w)
    k0 = torch.from_numpy(k_h.view(np.int64)).to(dev)
    del k_h
    v0 = torch.arange(n, dtype=torch.int32, device=dev)
    slots = [(k0.clone(), v0.clone()) for _ in range(K + W)]
    ws = torch.empty(rts.workspace_bytes64(n, 4), dtype=torch.uint8, device=dev)
    for i in range(W):
        rts.sort64_ex(slots[i][0], slots[i][1], None, ws)
    torch.cuda.synchronize()
    rts.profile_start(max_marks=32 * K + 32)
    t0 = time.perf_counter()
    for i in range(W, W + K):
        rts.sort64_ex(slots[i][0], slots[i][1], None, ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    calls = split_calls(rts.profile_stop(capacity=32 * K + 32))
    pass_ms = [ms for c in calls for kind, ms in c[1] if RT_KIND_PASS <= kind < RT_KIND_PASS + 8]
    hist_ms = [ms for c in calls for kind, ms in c[1] if kind == RT_KIND_HISTOGRAM]
    ko, vo = slots[W + K - 1]
    # properties that fix a stable sort of original indices (unsigned order
    # through the sign flip)
    ku = ko ^ torch.tensor(-(1 << 63), dtype=torch.int64, device=dev)
    ok = bool((ku[1:] >= ku[:-1]).all().item())
    vl = vo.to(torch.int64)
    ok &= bool((torch.bincount(vl, minlength=n) == 1).all().item())
    ok &= bool(torch.equal(k0[vl], ko))
    eq = ko[1:] == ko[:-1]
    ok &= bool((vl[1:][eq] > vl[:-1][eq]).all().item())
    del slots, ws, ku, vl, eq
    pm = float(np.mean(pass_ms))
    pass_bytes = 2.0 * 12 * n
    gk = n / (wall / K) / 1e9
    return {"workload": w.name, "n": n, "key_bits": 64, "value_bytes": 4, "digit_bits": [8] * 8,
            "Gkeys/s": round(gk, 3), "ms_per_call": round(1e3 * wall / K, 4),
            "pass_ms": round(pm, 4), "pass_GBps": round(pass_bytes / pm / 1e6, 1),
            "pass_frac_of_peak": round(pass_bytes / pm / 1e6 / PEAK_HBM_GBPS, 4),
            "histogram_ms": round(float(np.mean(hist_ms)), 4) if hist_ms else None,
            "parity_properties_ok": ok}


def bench_write_combining(rts, inputs, dev, K, W):
    """The paper's Table 1 configurations on this GPU: N = 64 Mi uniform
    keys, without and with 32-bit values, sorted with the LDS staging by
    digit (the GPU form of write-combining) and with every item scattered
    straight from registers (RT_FLAG_DIRECT_SCATTER, the "VM only" row's
    counterpart).  Same tile shape for both; outputs must agree."""
    import numpy as np
    import torch
    from paper_1008_2849_amd._lib import RT_FLAG_DIRECT_SCATTER, RT_FLAG_NT_STORES, RT_KIND_PASS
    out = {}
    for name in ("keys_64m_uniform", "pairs_64m_uniform"):
        w = inputs.WORKLOADS[name]
        k_h, v_h = inputs.make_workload(w)
        k0 = torch.from_numpy(k_h.view(np.int32)).to(dev)
        v0 = torch.from_numpy(v_h.view(np.int32)).to(dev) if v_h is not None else None
        tuned = rts.tuned_config(w.n, w.with_values)
        # both sides in one tile shape; 512 x 32 has no direct form, so the
        # comparison then takes the 16K-item 1024 x 16 tiles, and the tuned
        # shape is timed as a third leg
        shape = (tuned.block_threads, tuned.items_per_thread)
        if shape == (512, 32):
            shape = (1024, 16)
        row = {}
        results = {}
        legs = [("staged", tuned.flags & ~RT_FLAG_NT_STORES if shape != (tuned.block_threads, tuned.items_per_thread)
                 else tuned.flags, shape),
                ("direct", (tuned.flags & ~RT_FLAG_NT_STORES) | RT_FLAG_DIRECT_SCATTER, shape)]
        if shape != (tuned.block_threads, tuned.items_per_thread):
            legs.append(("tuned", tuned.flags, (tuned.block_threads, tuned.items_per_thread)))
        for label, flags, (blk, ipt) in legs:
            cfg = rts.Config(tuned.digit_bits, blk, ipt, flags)
            slots = [(k0.clone(), None if v0 is None else v0.clone()) for _ in range(K + W)]
            ws = torch.empty(rts.workspace_bytes(w.n, w.with_values, cfg), dtype=torch.uint8, device=dev)
            for i in range(W):
                rts.sort_ex(slots[i][0], slots[i][1], cfg, ws)
            torch.cuda.synchronize()
            rts.profile_start(max_marks=16 * K + 16)
            t0 = time.perf_counter()
            for i in range(W, W + K):
                rts.sort_ex(slots[i][0], slots[i][1], cfg, ws)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            passes = [ms for kind, ms in rts.profile_stop(capacity=16 * K + 16)
                      if RT_KIND_PASS <= kind < RT_KIND_PASS + 8]
            pm = float(np.mean(passes))
            item = 8 if w.with_values else 4
            row[label + "_Gkeys/s"] = round(w.n / (wall / K) / 1e9, 3)
            row[label + "_pass_ms"] = round(pm, 4)
            row[label + "_pass_GBps"] = round(2 * item * w.n / pm / 1e6, 1)
            results[label] = slots[W + K - 1]
            del slots, ws
        row["staging_speedup"] = round(row["staged_Gkeys/s"] / row["direct_Gkeys/s"], 3)
        a, b = results["staged"], results["direct"]
        row["outputs_equal"] = bool(torch.equal(a[0], b[0])) and (a[1] is None or bool(torch.equal(a[1], b[1])))
        if "tuned" in results:
            c = results["tuned"]
            row["outputs_equal"] = row["outputs_equal"] and bool(torch.equal(a[0], c[0])) and (
                a[1] is None or bool(torch.equal(a[1], c[1])))
        row["config"] = {"digit_bits": list(tuned.digit_bits), "block_threads": shape[0], "items_per_thread": shape[1]}
        row["tuned_config"] = {"block_threads": tuned.block_threads, "items_per_thread": tuned.items_per_thread}
        out[name] = row
        del results, a, b, k0, v0
        torch.cuda.empty_cache()
    # context only: the paper's Table 1 rows on its dual-CPU machine
    out["paper_table1_context"] = {"unit": "M items/s", "machine": "2x Xeon W5580 (2010), N = 64 Mi",
                                   "keys": {"VM+WC": 621, "VM only": 334}, "pairs": {"VM+WC": 430, "VM only": 203}}
    return out


def bench_pcie(rts, dev, keys_h, vals_h, cfg, ref_k, ref_v, reps=3):
    """Transfer-inclusive rate for host-resident data (the paper's GPU+PCIe
    comparison in Section 5): pinned host keys/values -> device, sort,
    device -> pinned host, timed end to end on one stream."""
    import numpy as np
    import torch
    n = keys_h.size
    hk = torch.from_numpy(keys_h.view(np.int32)).pin_memory()
    hv = torch.from_numpy(vals_h.view(np.int32)).pin_memory()
    ok = torch.empty_like(hk).pin_memory()
    ov = torch.empty_like(hv).pin_memory()
    dk = torch.empty(n, dtype=torch.int32, device=dev)
    dv = torch.empty(n, dtype=torch.int32, device=dev)
    ws = torch.empty(rts.workspace_bytes(n, True, cfg), dtype=torch.uint8, device=dev)
    times, h2d, d2h = [], [], []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        e[0].record()
        dk.copy_(hk, non_blocking=True)
        dv.copy_(hv, non_blocking=True)
        e[1].record()
        rts.sort_ex(dk, dv, cfg, ws)
        e[2].record()
        ok.copy_(dk, non_blocking=True)
        ov.copy_(dv, non_blocking=True)
        e[3].record()
        torch.cuda.synchronize()
        if r == 0:
            continue  # warm-up
        times.append(e[0].elapsed_time(e[3]))
        h2d.append(e[0].elapsed_time(e[1]))
        d2h.append(e[2].elapsed_time(e[3]))
    ms = float(np.median(times))
    # the device result equals the checked sort of the same input
    same = bool(torch.equal(dk, ref_k)) and bool(torch.equal(dv, ref_v))
    return {"Gkeys/s": round(n / ms / 1e6, 3), "ms": round(ms, 3),
            "h2d_GBps": round(8.0 * n / float(np.median(h2d)) / 1e6, 1),
            "d2h_GBps": round(8.0 * n / float(np.median(d2h)) / 1e6, 1),
            "note": "pinned host -> HBM, sort, HBM -> pinned host; context for the paper's GPU+PCIe figure",
            "matches_device_sort": same}


def bench_serving_closed(rts, inputs, inflight, seconds, warm_s, single_gkeys, budget_gib=32):
    """Closed loop: `inflight` requests (the serving mix of sizes and key
    distributions, generated on the device) are kept outstanding; each
    completion is replaced by the next request.  Measures the server's
    capacity and the latency at that throughput."""
    import dataclasses
    import numpy as np
    from paper_1008_2849_amd.api import gen_params_to_c
    from paper_1008_2849_amd.server import Server
    seed = inputs.SEED_SERVING + 100
    count = 1 << 20
    sizes = inputs.serving_request_sizes(count, seed)
    dists = inputs.serving_request_dists(count, seed)
    states = inputs.splitmix64_words(seed, 0, count)
    templates = [gen_params_to_c(inputs.counter_params(d, seed, 0)) for d in range(3)]

    def params(i):
        g = templates[int(dists[i])]
        g.state = int(states[i])
        return g

    srv = Server(hbm_budget_bytes=budget_gib << 30, max_active=4096)
    nxt = 0
    submit_time = {}
    for _ in range(inflight):
        t = srv.submit_generated(params(nxt), int(sizes[nxt]))
        submit_time[t] = (nxt, time.perf_counter())
        nxt += 1
    t0 = time.perf_counter()
    lats, items = [], 0
    t_meas = None
    checked, wrong = 0, 0
    while True:
        t, ms = srv.wait_any()
        i, _ = submit_time.pop(t)
        if i % 997 == 0 and sizes[i] <= (1 << 16):  # sampled parity of served results
            import torch
            n_i = int(sizes[i])
            kk = torch.empty(n_i, dtype=torch.int32, device="cuda")
            vv = torch.empty(n_i, dtype=torch.int32, device="cuda")
            srv.fetch(t, kk, vv)
            p_i = inputs.counter_params(int(dists[i]), seed, 0)
            p_i = dataclasses.replace(p_i, state=int(states[i]))
            keys_i = inputs.counter_keys(p_i, n_i)
            order = np.argsort(keys_i, kind="stable")
            ok_i = (np.array_equal(kk.cpu().numpy().view(np.uint32), keys_i[order]) and
                    np.array_equal(vv.cpu().numpy().view(np.uint32), order.astype(np.uint32)))
            checked += 1
            wrong += 0 if ok_i else 1
        else:
            srv.release(t)
        now = time.perf_counter() - t0
        if now >= warm_s:
            if t_meas is None:
                t_meas = time.perf_counter()
            lats.append(ms / 1e3)
            items += int(sizes[i])
        if now >= warm_s + seconds:
            break
        t2 = srv.submit_generated(params(nxt), int(sizes[nxt]))
        submit_time[t2] = (nxt, time.perf_counter())
        nxt += 1
    span = time.perf_counter() - t_meas
    while submit_time:  # drain
        t, _ = srv.wait_any()
        submit_time.pop(t, None)
        srv.release(t)
    peak = srv.stats()[4]
    srv.close()
    gk = items / span / 1e9
    return {"mode": "closed_loop", "inflight": inflight, "achieved_Gkeys/s": round(gk, 3),
            "frac_of_single_array": round(gk / single_gkeys, 4),
            "budget_GiB": budget_gib, "peak_budgeted_GiB": round(peak / 2**30, 3),
            "p50_ms": round(float(np.percentile(lats, 50)), 3), "p99_ms": round(float(np.percentile(lats, 99)), 3),
            "requests_measured": len(lats), "seconds": seconds,
            "sampled_parity": {"checked": checked, "wrong": wrong}, "failures": ["parity"] if wrong else []}


def bench_serving(rts, inputs, load, seconds, warm_s, single_gkeys, budget_gib=32):
    """Poisson arrivals of device-generated requests (sizes 2^U[10,24],
    distribution uniform / AND-4 / Zipf-16) offered at `load` times the
    single-array throughput, replayed open loop by the library's native
    submitter (rt_server_replay); latency = completion - scheduled arrival.
    Requests arriving in the first warm_s seconds are not measured."""
    import ctypes
    import numpy as np
    from paper_1008_2849_amd.api import gen_params_to_c
    from paper_1008_2849_amd.server import Server
    from paper_1008_2849_amd._lib import RtError
    mean_n = (2.0 ** 24 - 2.0 ** 10) / (14 * np.log(2.0))
    rate = load * single_gkeys * 1e9 / mean_n  # requests per second
    count = int(rate * (seconds + warm_s) * 1.05) + 16
    seed = inputs.SEED_SERVING
    arrivals = inputs.poisson_arrivals(rate, count, seed)
    count = int(np.searchsorted(arrivals, seconds + warm_s))
    arrivals = arrivals[:count]
    sizes = inputs.serving_request_sizes(count, seed)
    dists = inputs.serving_request_dists(count, seed)
    # request i draws its keys from stream i of the serving seed
    states = inputs.splitmix64_words(seed, 0, count)
    templates = [gen_params_to_c(inputs.counter_params(d, seed, 0)) for d in range(3)]
    params = []
    for i in range(count):
        g = type(templates[0])()
        ctypes.memmove(ctypes.addressof(g), ctypes.addressof(templates[int(dists[i])]), ctypes.sizeof(g))
        g.state = int(states[i])
        params.append(g)
    failures = []
    t0 = time.perf_counter()
    with Server(hbm_budget_bytes=budget_gib << 30, max_active=4096) as srv:
        try:
            lat_us, span_us = srv.replay(arrivals, sizes, params)
        except RtError as e:
            failures.append(repr(e))
            lat_us, span_us = np.full(count, -1.0), 0.0
        p50_all, p99_all, gk_srv, done, peak = srv.stats()
    wall = time.perf_counter() - t0
    meas = (arrivals >= warm_s) & (lat_us >= 0)
    lm = lat_us[meas] / 1e3
    items = float(np.sum(sizes[meas].astype(np.float64)))
    window = span_us / 1e6 - warm_s
    return {"mode": "open_loop", "load": load, "offered_Gkeys/s": round(load * single_gkeys, 3),
            "achieved_Gkeys/s": round(items / window / 1e9, 3) if window > 0 and lm.size else None,
            "p50_ms": round(float(np.percentile(lm, 50)), 3) if lm.size else None,
            "p99_ms": round(float(np.percentile(lm, 99)), 3) if lm.size else None,
            "requests_measured": int(lm.size), "requests_submitted": count,
            "latency_from": "scheduled arrival", "submitter": "native (rt_server_replay)",
            "seconds": seconds, "warmup_s": warm_s, "budget_GiB": budget_gib,
            "peak_budgeted_GiB": round(peak / 2**30, 3), "failures": failures[:3],
            "wall_s": round(wall, 2)}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="pairs_256m_uniform",
                    help="named synthetic workload (paper_1008_2849_amd.inputs.WORKLOADS)")
    ap.add_argument("--log2n", type=int, default=0, help="override the workload's size (2^log2n)")
    ap.add_argument("--bits", default="", help="digit widths, e.g. 11,11,10 (default: tuned)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--ipt", type=int, default=0)
    ap.add_argument("--flags", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-msd-first", action="store_true", help="skip the MSD-first leg")
    ap.add_argument("--no-sort64", action="store_true", help="skip the 64-bit-key leg")
    ap.add_argument("--no-table1", action="store_true",
                    help="skip the write-combining leg (the paper's Table 1 configurations)")
    ap.add_argument("--no-pcie", action="store_true", help="skip the transfer-inclusive leg")
    ap.add_argument("--workloads", default="keys_256m_uniform,keys_1m_uniform,pairs_64m_and2,pairs_64m_and4,"
                    "pairs_64m_and8,pairs_64m_top_a5,pairs_64m_zipf16",
                    help="further single-array workloads timed and checked against the oracle (empty to skip)")
    ap.add_argument("--no-xcd-compare", action="store_true",
                    help="skip re-timing the headline sort on one lookback chain per pass")
    ap.add_argument("--no-widths-compare", action="store_true",
                    help="skip re-timing the headline sort with 11/11/10-bit digits")
    ap.add_argument("--no-fused-compare", action="store_true",
                    help="skip timing the fused next-digit histogram against the upfront read")
    ap.add_argument("--serve-loads", default="0.5,0.6,0.7,0.75", help="comma list of offered loads (fraction "
                    "of single-array throughput), replayed open loop; empty to skip")
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--serve-tight-gib", type=int, default=2,
                    help="budget (GiB) of a closed-loop leg with 256 requests in flight that presses admission "
                         "against memory (0 to skip)")
    ap.add_argument("--serve-inflight", default="64,256",
                    help="comma list of closed-loop request counts kept in flight (empty to skip)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library sorts on one GPU; multi-GPU runs are not provided "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    import paper_1008_2849_amd as rts
    from paper_1008_2849_amd import inputs
    from paper_1008_2849_amd._lib import RT_KIND_COPY, RT_KIND_HISTOGRAM, RT_KIND_PASS

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    wl = inputs.WORKLOADS[args.workload]
    n = (1 << args.log2n) if args.log2n else wl.n
    vals_on = wl.with_values
    K, W = args.steps, args.warmup

    tuned = rts.tuned_config(n, vals_on)
    cfg = rts.Config(tuple(int(x) for x in args.bits.split(",")) if args.bits else tuned.digit_bits,
                     args.block or tuned.block_threads, args.ipt or tuned.items_per_thread,
                     args.flags or tuned.flags)
    log(f"{wl.name}: n={n} {'pairs' if vals_on else 'keys'}, config {cfg}, steps {K}, warmup {W}")

    t = time.perf_counter()
    keys_h, vals_h = inputs.make_workload(wl, n)
    k0 = torch.from_numpy(keys_h.view(np.int32)).to(dev)
    v0 = torch.from_numpy(vals_h.view(np.int32)).to(dev) if vals_on else None
    # one private copy of the input per step, all resident before timing
    slots = [(k0.clone(), None if v0 is None else v0.clone()) for _ in range(K + W)]
    ws = torch.empty(rts.workspace_bytes(n, vals_on, cfg), dtype=torch.uint8, device=dev)
    item_bytes = 8 if vals_on else 4
    torch.cuda.synchronize()
    log(f"inputs staged in HBM ({(K + W) * item_bytes * n / 2**30:.1f} GiB) in {time.perf_counter() - t:.1f}s")

    for i in range(W):
        rts.sort_ex(slots[i][0], slots[i][1], cfg, ws)
    torch.cuda.synchronize()

    # the timed region: K sorts, nothing else on the stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(W, W + K):
        rts.sort_ex(slots[i][0], slots[i][1], cfg, ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / K
    gkeys = n / (wall / K) / 1e9
    log(f"{K} sorts in {wall * 1e3:.2f} ms: {ms_per_step:.3f} ms/sort, {gkeys:.2f} Gkeys/s")
    ko, vo = slots[W + K - 1]
    timed_out = (ko.clone(), None if vo is None else vo.clone())

    # per-kernel times: the same K sorts of fresh copies of the input again,
    # with a HIP event recorded on the launch stream around every kernel
    for i in range(W, W + K):
        slots[i][0].copy_(k0)
        if v0 is not None:
            slots[i][1].copy_(v0)
    rts.profile_start(max_marks=16 * K + 16)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(W, W + K):
        rts.sort_ex(slots[i][0], slots[i][1], cfg, ws)
    torch.cuda.synchronize()
    marked_wall = time.perf_counter() - t1
    marks = rts.profile_stop(capacity=16 * K + 16)
    same_marked = torch.equal(slots[W + K - 1][0], timed_out[0]) and (
        vo is None or torch.equal(slots[W + K - 1][1], timed_out[1]))
    log(f"with per-kernel marks: {1e3 * marked_wall / K:.3f} ms/sort, outputs equal: {same_marked}")

    def by_kind(base_kind):
        out = {}
        for kind, ms in marks:
            if base_kind <= kind < base_kind + 8:
                out.setdefault(kind - base_kind, []).append(ms)
        return {p: float(np.mean(v)) for p, v in sorted(out.items())}

    passes = by_kind(RT_KIND_PASS)
    hist_ms = [ms for kind, ms in marks if kind == RT_KIND_HISTOGRAM]
    pass_bytes = 2.0 * item_bytes * n  # the pass reads and writes every key (and value) once
    per_pass = []
    for p in sorted(passes):
        per_pass.append({"pass": p, "ms": round(passes[p], 4),
                         "GB/s": round(pass_bytes / passes[p] / 1e6, 1),
                         "frac_of_peak": round(pass_bytes / passes[p] / 1e6 / PEAK_HBM_GBPS, 4)})
    all_down = [ms for kind, ms in marks if RT_KIND_PASS <= kind < RT_KIND_PASS + 8]
    dom_ms = float(np.mean(all_down)) if all_down else float("nan")
    achieved = pass_bytes / dom_ms / 1e6
    hist = None
    if hist_ms:
        h = float(np.mean(hist_ms))
        hist = {"ms": round(h, 4), "GB/s": round(4.0 * n / h / 1e6, 1)}

    # parity of the last timed output, by the properties that fix a stable sort
    ko, vo = timed_out
    k64 = ko.to(torch.int64) & 0xFFFFFFFF
    props = bool((k64[1:] >= k64[:-1]).all().item())
    if vo is not None:
        vl = vo.to(torch.int64)
        props &= bool(((vl >= 0) & (vl < n)).all().item())
        seen = torch.zeros(n, dtype=torch.bool, device=dev)
        seen[vl] = True
        props &= bool(seen.all().item())
        props &= bool(torch.equal(k0[vl], ko))
        eq = k64[1:] == k64[:-1]
        props &= bool((vl[1:][eq] > vl[:-1][eq]).all().item())
        del seen, vl, eq
    else:  # keys only: the same multiset, by a histogram of all 32 bits' low and high halves
        src64 = k0.to(torch.int64) & 0xFFFFFFFF
        for sh in (0, 16):
            props &= bool(torch.equal(torch.bincount((src64 >> sh) & 0xFFFF, minlength=65536),
                                      torch.bincount((k64 >> sh) & 0xFFFF, minlength=65536)))
        props &= bool(torch.equal(src64.sum(), k64.sum()))
        del src64
    del k64

    # the achievable bandwidth on this device: copies of 2 GiB (2 GiB read +
    # 2 GiB written, the pass's mix), and 2 GiB read only and written only
    from paper_1008_2849_amd._lib import RT_PROBE_COPY, RT_PROBE_COPY_NT, RT_PROBE_READ, RT_PROBE_WRITE
    big_src = torch.empty(1 << 29, dtype=torch.int32, device=dev).fill_(7)
    big_dst = torch.empty_like(big_src)
    sink = torch.zeros(4, dtype=torch.int32, device=dev)
    probes = {}
    for name, kind, moved in (("copy", RT_PROBE_COPY, 2), ("copy_nt_x4", RT_PROBE_COPY_NT, 2),
                              ("read_only", RT_PROBE_READ, 1), ("write_only", RT_PROBE_WRITE, 1)):
        src_t = None if kind == RT_PROBE_WRITE else big_src
        dst_t = None if kind == RT_PROBE_READ else big_dst
        rts.bandwidth_probe(kind, src=src_t, dst=dst_t, sink=sink)
        torch.cuda.synchronize()
        rts.profile_start(64)
        for _ in range(7):
            rts.bandwidth_probe(kind, src=src_t, dst=dst_t, sink=sink)
        torch.cuda.synchronize()
        cm = [ms for kind_, ms in rts.profile_stop(64) if kind_ == RT_KIND_COPY]
        probes[name] = round(moved * big_src.numel() * 4 / float(np.median(cm)) / 1e6, 1) if cm else None
    copy_gbps = max(v for k_, v in probes.items() if k_.startswith("copy") and v)
    log(f"bandwidth probes (GB/s): {probes}")
    del big_src, big_dst, sink

    # the same sort on one lookback chain per pass (RT_FLAG_ONE_CHAIN), for
    # what the XCD chunks buy: the same W warm-up and K timed sorts of fresh
    # copies of the same input, under the same per-kernel timing marks, with
    # the pass and histogram times of both sides
    from paper_1008_2849_amd._lib import RT_FLAG_ONE_CHAIN
    xcd = None
    if not args.no_xcd_compare:
        oc_cfg = rts.Config(cfg.digit_bits, cfg.block_threads, cfg.items_per_thread, cfg.flags | RT_FLAG_ONE_CHAIN)
        ref = (ko.clone(), None if vo is None else vo.clone())
        for k, v in slots:
            k.copy_(k0)
            if v is not None:
                v.copy_(v0)
        oc_ws = ws if ws.numel() >= rts.workspace_bytes(n, vals_on, oc_cfg) else torch.empty(
            rts.workspace_bytes(n, vals_on, oc_cfg), dtype=torch.uint8, device=dev)
        for i in range(W):
            rts.sort_ex(slots[i][0], slots[i][1], oc_cfg, oc_ws)
        torch.cuda.synchronize()
        rts.profile_start(max_marks=16 * K + 16)
        t0 = time.perf_counter()
        for i in range(W, W + K):
            rts.sort_ex(slots[i][0], slots[i][1], oc_cfg, oc_ws)
        torch.cuda.synchronize()
        oc_ms = 1e3 * (time.perf_counter() - t0) / K
        oc_marks = rts.profile_stop(capacity=16 * K + 16)
        last = slots[W + K - 1]
        oc_same = bool(torch.equal(last[0], ref[0])) and (ref[1] is None or bool(torch.equal(last[1], ref[1])))
        # the headline output stays where the later legs expect it
        slots[W + K - 1][0].copy_(ref[0])
        if ref[1] is not None:
            slots[W + K - 1][1].copy_(ref[1])
        del ref

        def kind_ms(mk, lo, hi):
            v = [ms for kind, ms in mk if lo <= kind < hi]
            return round(float(np.mean(v)), 4) if v else None

        xcd = {"chunked_ms_per_sort": round(ms_per_step, 4), "one_chain_ms_per_sort": round(oc_ms, 4),
               "speedup": round(oc_ms / ms_per_step, 4), "one_chain_output_equal": oc_same,
               "chunked_pass_ms": kind_ms(marks, RT_KIND_PASS, RT_KIND_PASS + 8),
               "one_chain_pass_ms": kind_ms(oc_marks, RT_KIND_PASS, RT_KIND_PASS + 8),
               "chunked_histogram_ms": kind_ms(marks, RT_KIND_HISTOGRAM, RT_KIND_HISTOGRAM + 1),
               "one_chain_histogram_ms": kind_ms(oc_marks, RT_KIND_HISTOGRAM, RT_KIND_HISTOGRAM + 1),
               "timing": f"both sides: {W} warm-up then {K} timed sorts with per-kernel timing marks",
               "note": "same input and configuration with RT_FLAG_ONE_CHAIN (one lookback chain per pass)"}
        log(f"one chain per pass: {oc_ms:.3f} ms/sort; XCD chunks {oc_ms / ms_per_step:.3f}x faster")
        del oc_ws

    # the fused next-digit histogram (RT_FLAG_FUSED_HISTOGRAM) against the
    # upfront read of every digit, both on one chain (the fused form's
    # condition), same input, same W and K, same per-kernel marks
    from paper_1008_2849_amd._lib import RT_FLAG_FUSED_HISTOGRAM, RT_KIND_PLAN
    fused = None
    if not args.no_fused_compare and (cfg.block_threads, cfg.items_per_thread) != (512, 32):
        ref = (ko.clone(), None if vo is None else vo.clone())
        legs = {}
        for label, extra in (("upfront", RT_FLAG_ONE_CHAIN), ("fused", RT_FLAG_ONE_CHAIN | RT_FLAG_FUSED_HISTOGRAM)):
            fcfg = rts.Config(cfg.digit_bits, cfg.block_threads, cfg.items_per_thread, cfg.flags | extra)
            for k, v in slots:
                k.copy_(k0)
                if v is not None:
                    v.copy_(v0)
            fws = torch.empty(rts.workspace_bytes(n, vals_on, fcfg), dtype=torch.uint8, device=dev)
            for i in range(W):
                rts.sort_ex(slots[i][0], slots[i][1], fcfg, fws)
            torch.cuda.synchronize()
            rts.profile_start(max_marks=32 * K + 32)
            t0 = time.perf_counter()
            for i in range(W, W + K):
                rts.sort_ex(slots[i][0], slots[i][1], fcfg, fws)
            torch.cuda.synchronize()
            f_ms = 1e3 * (time.perf_counter() - t0) / K
            fm = rts.profile_stop(capacity=32 * K + 32)
            last = slots[W + K - 1]
            same = bool(torch.equal(last[0], ref[0])) and (ref[1] is None or bool(torch.equal(last[1], ref[1])))
            per = lambda lo, hi: [ms for kind, ms in fm if lo <= kind < hi]
            legs[label] = {"ms_per_sort": round(f_ms, 4),
                           "pass_ms": round(float(np.mean(per(RT_KIND_PASS, RT_KIND_PASS + 8))), 4),
                           "histogram_ms": round(float(np.mean(per(RT_KIND_HISTOGRAM, RT_KIND_HISTOGRAM + 1))), 4),
                           "plan_ms_per_sort": round(float(np.sum(per(RT_KIND_PLAN, RT_KIND_PLAN + 1))) / K, 4),
                           "output_equal": same}
            del fws
        slots[W + K - 1][0].copy_(ref[0])
        if ref[1] is not None:
            slots[W + K - 1][1].copy_(ref[1])
        del ref
        fused = dict(legs, speedup=round(legs["upfront"]["ms_per_sort"] / legs["fused"]["ms_per_sort"], 4),
                     note="both on one lookback chain; fused: the upfront read counts digit 0 only and passes "
                          "0-2 count the next digit while they write")
        log(f"fused histogram: {fused}")

    # the same sort with 11/11/10-bit digits (three passes instead of four),
    # the alternative the autotuner also weighs: a few sorts, same input,
    # output compared with the 8-bit sort's
    widths = None
    if not args.no_widths_compare and args.workload == "pairs_256m_uniform":
        ref = (ko.clone(), None if vo is None else vo.clone())
        wcfg = rts.Config((11, 11, 10), 512, 16, 0)
        wk = min(K, 5)
        for k, v in slots[:wk + 1]:
            k.copy_(k0)
            if v is not None:
                v.copy_(v0)
        wws = torch.empty(rts.workspace_bytes(n, vals_on, wcfg), dtype=torch.uint8, device=dev)
        rts.sort_ex(slots[0][0], slots[0][1], wcfg, wws)
        torch.cuda.synchronize()
        rts.profile_start(max_marks=32 * wk + 32)
        t0 = time.perf_counter()
        for i in range(1, wk + 1):
            rts.sort_ex(slots[i][0], slots[i][1], wcfg, wws)
        torch.cuda.synchronize()
        w_ms = 1e3 * (time.perf_counter() - t0) / wk
        wm = rts.profile_stop(capacity=32 * wk + 32)
        last = slots[wk]
        same = bool(torch.equal(last[0], ref[0])) and (ref[1] is None or bool(torch.equal(last[1], ref[1])))
        wpass = [ms for kind, ms in wm if RT_KIND_PASS <= kind < RT_KIND_PASS + 8]
        widths = {"digit_bits": [11, 11, 10], "shape": "512x16", "ms_per_sort": round(w_ms, 4),
                  "Gkeys/s": round(n / (w_ms / 1e3) / 1e9, 3),
                  "pass_ms": round(float(np.mean(wpass)), 4) if wpass else None,
                  "against_8x4_ms_per_sort": round(ms_per_step, 4), "output_equal": same,
                  "note": "three passes of 11, 11 and 10 bits; 2048-bin counters and lookback rows per tile"}
        del wws, ref
        log(f"11/11/10 digits: {widths}")

    digest = kernel_source_digest()
    counters = counters_from_profiles(digest)
    traffic = counters["traffic"]

    out_k = to_np = None
    cpu = None
    if not args.no_cpu_baseline:
        out_k = ko.cpu().numpy().view(np.uint32)
        out_v = None if vo is None else vo.cpu().numpy().view(np.uint32)
        log("timing the CPU oracle on the same input (single thread, one core)")
        dt, same, core = cpu_baseline(keys_h, vals_h, out_k, out_v)
        cpu = {"value": round(n / dt / 1e9, 5), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole workload: {wl.name} at n={n} (seed {wl.seed}), one sort, {dt:.1f} s, "
                         f"single thread pinned to core {core}",
               "cpu_model": cpu_model(), "host_logical_cpus": os.cpu_count(),
               "allowed_cpus": len(os.sched_getaffinity(0)),
               "matches_gpu_bit_exact": same}
        log(f"oracle {dt:.1f}s, GPU output {'==' if same else '!='} oracle")

    pcie = None
    if not args.no_pcie and vals_on:
        log("transfer-inclusive leg")
        pcie = bench_pcie(rts, dev, keys_h, vals_h, cfg, slots[W + K - 1][0], slots[W + K - 1][1])
        log(f"pcie: {pcie}")

    msd_first = None
    if not args.no_msd_first:
        log("MSD-first leg")
        ko, vo = slots[W + K - 1]
        ref = (ko.clone(), None if vo is None else vo.clone())
        msd_first = bench_msd_first(rts, dev, k0, v0, slots, K, W, gkeys, ref[0], ref[1])
        del ref
        log(f"msd_first: {msd_first}")

    workloads = []
    if args.workloads and args.workload == "pairs_256m_uniform":
        slots = ws = None  # the headline's copies and workspace (its output stays in ko / vo)
        torch.cuda.empty_cache()
        log("further workloads: " + args.workloads)
        workloads = bench_workloads(rts, inputs, dev, [x for x in args.workloads.split(",") if x], K, W)

    batched = None
    if not args.no_batched and args.workload == "pairs_256m_uniform":
        log("batched workload")
        batched = bench_batched(rts, inputs, dev, K, W, gkeys)
        log(f"batched: {batched}")
    del slots
    torch.cuda.empty_cache()
    sort64 = None
    if not args.no_sort64 and args.workload == "pairs_256m_uniform":
        log("64-bit keys leg")
        sort64 = bench_sort64(rts, inputs, dev, K, W)
        torch.cuda.empty_cache()
        log(f"sort64: {sort64}")
    table1 = None
    if not args.no_table1 and args.workload == "pairs_256m_uniform":
        log("write-combining leg (N = 64 Mi, staged vs direct scatter)")
        table1 = bench_write_combining(rts, inputs, dev, K, W)
        log(f"table1: {table1}")
    serving = []
    if (args.serve_loads or args.serve_inflight or args.serve_tight_gib) and args.workload == "pairs_256m_uniform":
        for load in (float(x) for x in args.serve_loads.split(",") if x):
            log(f"serving at load {load}")
            serving.append(bench_serving(rts, inputs, load, args.serve_seconds, 1.0, gkeys))
            log(f"serving: {serving[-1]}")
        for inflight in (int(x) for x in args.serve_inflight.split(",") if x):
            log(f"serving closed loop, {inflight} in flight")
            serving.append(bench_serving_closed(rts, inputs, inflight, args.serve_seconds, 1.0, gkeys))
            log(f"serving: {serving[-1]}")
        if args.serve_tight_gib > 0:
            log(f"serving closed loop, 256 in flight, {args.serve_tight_gib} GiB budget")
            serving.append(bench_serving_closed(rts, inputs, 256, args.serve_seconds, 1.0, gkeys,
                                                budget_gib=args.serve_tight_gib))
            log(f"serving: {serving[-1]}")

    line = {
        "metric": METRIC,
        "value": round(gkeys, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": n, "values": "original index" if vals_on else None,
                   "digit_bits": list(cfg.digit_bits), "block_threads": cfg.block_threads,
                   "items_per_thread": cfg.items_per_thread, "flags": cfg.flags},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(achieved / PEAK_HBM_GBPS, 4),
                     "traffic": traffic,
                     "valu_per_item": counters["valu_per_item"],
                     "write_32B_share": counters["write_32B_share"],
                     "lds_bank_conflict_share": counters["lds_bank_conflict_share"],
                     "kernel": "k_onesweep (one counting-sort pass: rank, lookback, scatter)",
                     "algorithmic_bytes_per_launch": pass_bytes,
                     "avg_launch_ms": round(dom_ms, 4)},
        "cpu_baseline": cpu,
        "per_pass": per_pass,
        "histogram": hist,
        "per_kernel_run": {"ms_per_sort_with_marks": round(1e3 * marked_wall / K, 4), "outputs_equal": same_marked,
                           "note": "per-kernel times come from a second run of the same K sorts with HIP events "
                                   "around every kernel; ms_per_step is the run without them"},
        "copy_peak_GBps": None if copy_gbps is None else round(copy_gbps, 1),
        "pass_frac_of_copy_peak": None if copy_gbps is None else round(achieved / copy_gbps, 4),
        "bandwidth_probes_GBps": probes,
        "parity_properties_ok": props,
        "xcd_chunks": xcd,
        "fused_histogram": fused,
        "digit_widths_11_11_10": widths,
        "transfer_inclusive": pcie,
        "msd_first": msd_first,
        "sort64": sort64,
        "write_combining": table1,
        "workloads": workloads,
        "batched": batched,
        "serving": serving,
        "kernel_source_digest": digest,
    }
    print(json.dumps(line), flush=True)
    ok = props and same_marked and (cpu is None or cpu["matches_gpu_bit_exact"])
    ok = ok and (batched is None or batched["parity_properties_ok"])
    ok = ok and all(w_["matches_oracle_bit_exact"] for w_ in workloads)
    ok = ok and all(not s.get("failures") for s in serving)
    ok = ok and (pcie is None or pcie["matches_device_sort"])
    ok = ok and (fused is None or all(fused[x]["output_equal"] for x in ("upfront", "fused")))
    ok = ok and (widths is None or widths["output_equal"])
    ok = ok and (msd_first is None or (msd_first["matches_lsd_sort"] and msd_first["one_level"]["matches_lsd_sort"]))
    ok = ok and (sort64 is None or sort64["parity_properties_ok"])
    ok = ok and (table1 is None or all(r["outputs_equal"] for k, r in table1.items() if "outputs_equal" in r))
    return 0 if ok else 3


if __name__ == "__main__":
    sys.exit(main())
