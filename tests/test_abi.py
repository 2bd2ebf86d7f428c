"""The C ABI library loads without a GPU, exports what include/rtsort.h
declares, and rejects bad arguments before any device work."""
import ctypes
import json
import os
import re

import pytest

from paper_1008_2849_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtsort.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = header_functions()
    for must in ("rt_sort_keys", "rt_sort_pairs", "rt_sort_pairs_batched", "rt_sort_pairs_ex",
                 "rt_server_create", "rt_server_submit", "rt_server_wait", "rt_server_stats"):
        assert must in names


def header_prototypes():
    """name -> list of parameter types (names dropped, spaces normalised)."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"\b[a-z_0-9 ]*?[\s*]+(rt_[a-z_0-9]+)\s*\(([^)]*)\)\s*;", text):
        params = []
        for p in m.group(2).split(","):
            p = " ".join(p.replace("*", " * ").split())
            toks = p.split(" ")
            if toks == ["void"]:
                continue
            if len(toks) > 1 and toks[-1] != "*":
                toks = toks[:-1]  # drop the parameter name
            params.append(" ".join(toks))
        out[m.group(1)] = params
    return out


# The boundary the task's design table asks for, call by call: the
# parameter types each call takes there, and how the header maps it.
# "exact": same name and parameter types.  Any other tag names a departure
# that the design doc's boundary table must list with its reason.
SPEC_8B = {
    "rt_sort_keys": (["uint32_t *", "size_t", "hipStream_t"], "exact"),
    "rt_sort_pairs": (["uint32_t *", "uint32_t *", "size_t", "hipStream_t"], "exact"),
    "rt_sort_pairs_batched": (["uint32_t *", "uint32_t *", "const uint32_t *", "uint32_t", "hipStream_t"],
                              "max_total"),
    "rt_workspace_bytes": (["size_t", "int", "const rt_config *"], "exact"),
    "rt_sort_pairs_ex": (["uint32_t *", "uint32_t *", "size_t", "const rt_config *", "void *", "size_t",
                          "hipStream_t"], "exact"),
    "rt_load_tuning": (["const char *"], "exact"),
    "rt_status_string": (["rt_status"], "exact"),
    "rt_last_error": ([], "exact"),
    "rt_server_create": (["size_t", "uint32_t", "rt_server * *"], "exact"),
    "rt_server_submit": (["rt_server *", "const uint32_t *", "const uint32_t *", "uint32_t *", "uint32_t *",
                          "size_t", "uint64_t *"], "exact"),
    "rt_server_submit_generated": (["rt_server *", "uint32_t", "uint64_t", "size_t", "uint64_t *"],
                                   "generator_params"),
    "rt_server_wait": (["rt_server *", "uint64_t", "int64_t", "double *"], "exact"),
    "rt_server_stats": (["rt_server *", "double *", "double *", "double *"], "exact"),
    "rt_server_destroy": (["rt_server *"], "exact"),
}


def test_every_boundary_call_maps_to_the_header():
    protos = header_prototypes()
    design = open(os.path.join(ROOT, "DESIGN.md")).read()
    for name, (params, how) in SPEC_8B.items():
        assert name in protos, name
        if how == "exact":
            assert protos[name] == params, (name, protos[name])
        else:  # a departure: documented with its reason in the boundary table
            assert protos[name] != params, name
            assert f"`{how}`" in design, (name, how)
    # the departures, as they stand
    assert protos["rt_sort_pairs_batched"] == SPEC_8B["rt_sort_pairs_batched"][0][:4] + ["size_t", "hipStream_t"]
    assert protos["rt_server_submit_generated"] == ["rt_server *", "const rt_gen_params *", "size_t", "uint64_t *"]


def test_library_exports_every_declared_symbol():
    so = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in header_functions() if not hasattr(so, n)]
    assert not missing, missing
    # and the Python binding binds each of them
    assert set(header_functions()) == set(_lib.SIGNATURES)


@pytest.fixture(scope="module")
def so():
    return _lib.lib()


def err(so):
    return so.rt_last_error().decode()


def test_argument_errors_are_synchronous(so):
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: checks fail first
    assert so.rt_sort_keys(None, 5, None) == _lib.RT_ERR_INVALID_ARG
    assert "NULL" in err(so)
    assert so.rt_sort_keys(fake, 1 << 32, None) == _lib.RT_ERR_TOO_LARGE
    assert so.rt_sort_pairs(fake, None, 10, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort_pairs(fake, fake, 10, None) == _lib.RT_ERR_INVALID_ARG  # aliasing
    assert "overlap" in err(so)
    assert so.rt_sort_pairs(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x1010), 10, None) \
        == _lib.RT_ERR_INVALID_ARG  # partial overlap
    assert so.rt_sort_keys(ctypes.c_void_p(0x1002), 10, None) == _lib.RT_ERR_INVALID_ARG  # misaligned
    # n = 0 and n = 1 are no-ops, even with NULL pointers
    assert so.rt_sort_keys(None, 0, None) == _lib.RT_OK
    assert so.rt_sort_keys(None, 1, None) == _lib.RT_OK
    assert so.rt_sort_pairs(None, None, 1, None) == _lib.RT_OK


def test_validate_flag_is_accepted_everywhere(so):
    """RT_FLAG_VALIDATE (wait and report device errors) is a valid flag of
    the single-array, 64-bit and batched sorts: their configurations with it
    resolve (a refused configuration sizes no workspace)."""
    c = _lib.RtConfig()
    c.flags = _lib.RT_FLAG_VALIDATE
    assert so.rt_workspace_bytes(1 << 20, 1, ctypes.byref(c)) > 0
    assert so.rt_workspace_bytes64(1 << 20, 4, ctypes.byref(c)) > 0
    c.flags = 0x400  # not a flag
    assert so.rt_workspace_bytes(1 << 20, 1, ctypes.byref(c)) == 0


def test_bandwidth_probe_argument_errors(so):
    fake = ctypes.c_void_p(0x10000)
    sink = ctypes.c_void_p(0x20000)
    assert so.rt_bandwidth_probe(fake, fake, 0, _lib.RT_PROBE_COPY, None, None) == _lib.RT_OK  # nothing to do
    assert so.rt_bandwidth_probe(fake, fake, 4096, 4, None, None) == _lib.RT_ERR_INVALID_ARG  # no such kind
    assert so.rt_bandwidth_probe(None, fake, 4096, _lib.RT_PROBE_COPY, None, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_bandwidth_probe(fake, None, 4096, _lib.RT_PROBE_READ, None, None) == _lib.RT_ERR_INVALID_ARG  # no sink
    assert so.rt_bandwidth_probe(None, fake, 4100, _lib.RT_PROBE_WRITE, None, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_bandwidth_probe(ctypes.c_void_p(0x10004), sink, 4096, _lib.RT_PROBE_READ, sink, None) \
        == _lib.RT_ERR_INVALID_ARG  # misaligned


def test_chunk_decision_argument_errors(so):
    """The chunk-decision hooks refuse what the sorts refuse, before any
    launch."""
    fake = ctypes.c_void_p(0x10000)
    mode = ctypes.c_void_p(0x20000)
    assert so.rt_chunk_decision(fake, 1 << 25, 1, None, None, None) == _lib.RT_ERR_INVALID_ARG  # mode NULL
    assert so.rt_chunk_decision(None, 1 << 25, 1, None, mode, None) == _lib.RT_ERR_INVALID_ARG  # keys NULL
    assert so.rt_chunk_decision(fake, 1 << 32, 1, None, mode, None) == _lib.RT_ERR_TOO_LARGE
    both = _lib.RtConfig()
    both.flags = _lib.RT_FLAG_ONE_CHAIN | _lib.RT_FLAG_CHUNKS
    assert so.rt_chunk_decision(fake, 1 << 25, 1, ctypes.byref(both), mode, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_chunk_decision64(fake, 1 << 25, 2, None, mode, None) == _lib.RT_ERR_INVALID_ARG  # value bytes
    assert so.rt_chunk_decision64(fake, 1 << 25, 4, None, None, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_chunk_decision64(fake, 1 << 32, 4, None, mode, None) == _lib.RT_ERR_TOO_LARGE
    assert so.rt_chunk_decision64(fake, 1 << 25, 4, ctypes.byref(both), mode, None) == _lib.RT_ERR_INVALID_ARG


def test_two_blocks_per_cu_shape_flags(so):
    """512 x 32 tiles (keys and values staged one after the other) are built
    for the plain staged pass: with it, non-temporal stores, the direct
    scatter and the fused histogram are refused before any launch."""
    fake_k, fake_v = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x90000)
    c = _lib.RtConfig()
    c.num_passes = 4
    for i in range(4):
        c.digit_bits[i] = 8
    c.block_threads, c.items_per_thread = 512, 32
    assert so.rt_workspace_bytes(1 << 20, 1, ctypes.byref(c)) > 0
    for flag in (_lib.RT_FLAG_NT_STORES, _lib.RT_FLAG_DIRECT_SCATTER, _lib.RT_FLAG_FUSED_HISTOGRAM):
        c.flags = flag
        assert so.rt_sort_pairs_ex(fake_k, fake_v, 1000, ctypes.byref(c), None, 0, None) == _lib.RT_ERR_UNSUPPORTED
        assert so.rt_workspace_bytes(1000, 1, ctypes.byref(c)) == 0


def test_fused_histogram_flag(so):
    """RT_FLAG_FUSED_HISTOGRAM resolves for 8-bit digits (and then never
    needs the second temporary: every pass runs), and is refused with wider
    digits, XCD chunks forced, the direct scatter, non-temporal stores, or
    64-bit keys."""
    fake_k, fake_v = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x90000)

    def cfg(bits, flags):
        c = _lib.RtConfig()
        c.num_passes = len(bits)
        for i, b in enumerate(bits):
            c.digit_bits[i] = b
        c.flags = flags
        return c

    F = _lib.RT_FLAG_FUSED_HISTOGRAM
    n = 1 << 20
    plain = so.rt_workspace_bytes(n, 1, ctypes.byref(cfg((8, 8, 8, 8), 0)))
    fused = so.rt_workspace_bytes(n, 1, ctypes.byref(cfg((8, 8, 8, 8), F)))
    assert fused > 0 and plain - fused >= 2 * 4 * n  # no second temporary (two arrays of n words)
    assert so.rt_workspace_bytes(n, 1, ctypes.byref(cfg((8, 8, 8, 8), F | _lib.RT_FLAG_ONE_CHAIN))) == fused
    for bits, flags in (((11, 11, 10), F), ((8, 8, 8, 8), F | _lib.RT_FLAG_CHUNKS),
                        ((8, 8, 8, 8), F | _lib.RT_FLAG_DIRECT_SCATTER), ((8, 8, 8, 8), F | _lib.RT_FLAG_NT_STORES)):
        c = cfg(bits, flags)
        assert so.rt_sort_pairs_ex(fake_k, fake_v, 1000, ctypes.byref(c), None, 0, None) == _lib.RT_ERR_UNSUPPORTED, \
            (bits, flags)
    assert so.rt_workspace_bytes64(n, 4, ctypes.byref(cfg((8,) * 8, F))) == 0


def test_config_validation(so):
    fake_k, fake_v = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x90000)
    for bits, want in [((8, 8, 8), _lib.RT_ERR_INVALID_ARG),        # sums to 24
                       ((16, 16), _lib.RT_ERR_INVALID_ARG),          # too wide
                       ((0, 16, 16), _lib.RT_ERR_INVALID_ARG),       # zero width
                       ((4,) * 9, _lib.RT_ERR_INVALID_ARG)]:         # too many passes
        c = _lib.RtConfig()
        c.num_passes = len(bits)
        for i, b in enumerate(bits[:8]):
            c.digit_bits[i] = b
        assert so.rt_sort_pairs_ex(fake_k, fake_v, 1000, ctypes.byref(c), None, 0, None) == want, bits
    c = _lib.RtConfig()
    c.num_passes = 4
    for i in range(4):
        c.digit_bits[i] = 8
    c.block_threads, c.items_per_thread = 128, 7
    assert so.rt_sort_pairs_ex(fake_k, fake_v, 1000, ctypes.byref(c), None, 0, None) == _lib.RT_ERR_UNSUPPORTED
    c.block_threads, c.items_per_thread = 1024, 16
    c.flags = _lib.RT_FLAG_DIRECT_SCATTER | _lib.RT_FLAG_NT_STORES  # not built
    assert so.rt_sort_pairs_ex(fake_k, fake_v, 1000, ctypes.byref(c), None, 0, None) == _lib.RT_ERR_UNSUPPORTED
    c.flags = 0x100  # unknown
    assert so.rt_sort_pairs_ex(fake_k, fake_v, 1000, ctypes.byref(c), None, 0, None) == _lib.RT_ERR_INVALID_ARG
    c.flags = _lib.RT_FLAG_ONE_CHAIN | _lib.RT_FLAG_CHUNKS  # exclude each other
    assert so.rt_sort_pairs_ex(fake_k, fake_v, 1000, ctypes.byref(c), None, 0, None) == _lib.RT_ERR_INVALID_ARG


def test_workspace_bytes(so):
    assert so.rt_workspace_bytes(0, 1, None) == 0
    assert so.rt_workspace_bytes(1, 1, None) == 0
    n = 1 << 20
    ws_pairs = so.rt_workspace_bytes(n, 1, None)
    ws_keys = so.rt_workspace_bytes(n, 0, None)
    # two temporaries per array (skipping may leave an odd pass count)
    assert ws_pairs >= 4 * 4 * n and ws_keys >= 2 * 4 * n
    assert ws_pairs - ws_keys == 2 * 4 * n
    c = _lib.RtConfig()
    c.num_passes = 4
    for i in range(4):
        c.digit_bits[i] = 8
    c.flags = _lib.RT_FLAG_NO_SKIP  # even pass count, no skipping: one temporary
    assert so.rt_workspace_bytes(n, 1, ctypes.byref(c)) < ws_pairs - 2 * 4 * n + 4096


def test_status_strings(so):
    for s in range(10):
        assert so.rt_status_string(s)
    assert b"gfx950" in so.rt_version()


def test_tuning_table_roundtrip(so, tmp_path):
    good = {"arch": "gfx950", "entries": [
        {"op": "pairs", "min_n": 0, "max_n": 1 << 30, "digit_bits": [11, 11, 10],
         "block": 512, "ipt": 16, "flags": 2},
        {"op": "keys", "min_n": 0, "max_n": 1 << 40, "digit_bits": [8, 8, 8, 8],
         "block": 1024, "ipt": 8, "flags": 0}]}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(good))
    assert so.rt_load_tuning(str(p).encode()) == _lib.RT_OK
    c = _lib.RtConfig()
    assert so.rt_tuned_config(1 << 20, 1, ctypes.byref(c)) == _lib.RT_OK
    assert [c.digit_bits[i] for i in range(c.num_passes)] == [11, 11, 10]
    assert (c.block_threads, c.items_per_thread, c.flags) == (512, 16, 2)
    assert so.rt_tuned_config(1 << 20, 0, ctypes.byref(c)) == _lib.RT_OK
    assert c.block_threads == 1024
    bad = {"entries": [{"op": "pairs", "min_n": 0, "max_n": 10, "digit_bits": [8, 8],
                        "block": 256, "ipt": 16}]}
    p.write_text(json.dumps(bad))
    assert so.rt_load_tuning(str(p).encode()) == _lib.RT_ERR_INVALID_ARG
    p.write_text("{not json")
    assert so.rt_load_tuning(str(p).encode()) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_load_tuning(None) == _lib.RT_OK
    assert so.rt_tuned_config(1 << 20, 1, ctypes.byref(c)) == _lib.RT_OK
    assert c.num_passes == 4 and c.block_threads == 1024


def test_segment_classes_from_tuning_table(so, tmp_path):
    from paper_1008_2849_amd import api
    builtin = [(2048, 256, 8), (8192, 512, 16), (16384, 1024, 16)]
    assert so.rt_load_tuning(None) == _lib.RT_OK
    assert api.segment_classes() == builtin
    seg = lambda mx, b, i, bits=(8, 8, 8, 8): {"op": "segments", "min_n": 0, "max_n": mx,
                                               "digit_bits": list(bits), "block": b, "ipt": i}
    p = tmp_path / "t.json"
    good = [seg(1024, 256, 4), seg(4096, 512, 8), seg(8192, 1024, 8), seg(16384, 1024, 16)]
    p.write_text(json.dumps({"entries": good}))
    assert so.rt_load_tuning(str(p).encode()) == _lib.RT_OK
    assert api.segment_classes() == [(1024, 256, 4), (4096, 512, 8), (8192, 1024, 8), (16384, 1024, 16)]
    n = 1 << 20
    tuned_ws = so.rt_batched_workspace_bytes(4096, n, 1)
    for bad in ([seg(4096, 256, 8)],                              # limit above the shape's capacity
                [seg(2048, 256, 8), seg(2048, 512, 8)],           # not increasing
                [seg(16385, 1024, 16)],                           # beyond the LDS limit
                [seg(2048, 128, 16)],                             # no such kernel
                [seg(2048, 256, 8, (16, 16))],                    # digits other than 8 x 4 or 11/11/10
                [seg(16384, 1024, 16, (11, 11, 10))],             # 11-bit counters do not fit 1024 threads
                [{"op": "segments_tiled", "min_n": 0, "max_n": 0, "digit_bits": [8, 8, 8, 8],
                  "block": 256, "ipt": 16}],                      # no such tile shape
                [seg(512 * (i + 1), 512, 8) for i in range(5)]):  # more than four classes
        p.write_text(json.dumps({"entries": bad}))
        assert so.rt_load_tuning(str(p).encode()) == _lib.RT_ERR_INVALID_ARG, bad
        assert api.segment_classes() == [(1024, 256, 4), (4096, 512, 8), (8192, 1024, 8), (16384, 1024, 16)]
    # 11-bit classes and the tile of the tiled segments
    mixed = [seg(1024, 256, 4, (11, 11, 10)), seg(4096, 256, 16), seg(8192, 512, 16, (11, 11, 10)),
             {"op": "segments_tiled", "min_n": 0, "max_n": 0, "digit_bits": [8, 8, 8, 8], "block": 512, "ipt": 16}]
    p.write_text(json.dumps({"entries": mixed}))
    assert so.rt_load_tuning(str(p).encode()) == _lib.RT_OK
    assert api.segment_classes() == [(1024, 256, 4), (4096, 256, 16), (8192, 512, 16)]
    assert api.segment_config() == ([11, 8, 11], (512, 16))
    # 8K-item tiles: twice the tiles, so more lookback words
    assert so.rt_batched_workspace_bytes(4096, n, 1) > so.rt_batched_workspace_bytes(4096, 0, 1)
    # a tile entry alone keeps the built-in classes
    p.write_text(json.dumps({"entries": [mixed[-1]]}))
    assert so.rt_load_tuning(str(p).encode()) == _lib.RT_OK
    assert api.segment_classes() == builtin and api.segment_config() == ([8, 8, 8], (512, 16))
    # a lower LDS limit leaves more segments tiled: the workspace grows
    p.write_text(json.dumps({"entries": [seg(2048, 256, 8)]}))
    assert so.rt_load_tuning(str(p).encode()) == _lib.RT_OK
    assert so.rt_batched_workspace_bytes(4096, n, 1) > tuned_ws
    assert so.rt_load_tuning(None) == _lib.RT_OK
    assert api.segment_classes() == builtin and api.segment_config() == ([8, 8, 8], (1024, 16))
    api.load_default_tuning()


def test_batched_argument_errors(so):
    fake = ctypes.c_void_p(0x10000)
    off = ctypes.c_void_p(0x90000)
    assert so.rt_sort_pairs_batched(fake, None, off, 4, 1 << 32, None) == _lib.RT_ERR_TOO_LARGE
    assert so.rt_sort_pairs_batched(fake, None, None, 4, 1000, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort_pairs_batched(None, None, off, 4, 1000, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort_pairs_batched(fake, fake, off, 4, 1000, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort_pairs_batched(ctypes.c_void_p(0x10002), None, off, 4, 1000, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort_batched_ex(fake, None, off, 4, 1000, 0x80, None, 0, None) == _lib.RT_ERR_INVALID_ARG
    # a caller workspace that is too small or misaligned
    need = so.rt_batched_workspace_bytes(4, 1000, 0)
    assert so.rt_sort_batched_ex(fake, None, off, 4, 1000, 0, ctypes.c_void_p(0x100000), need - 1,
                                 None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort_batched_ex(fake, None, off, 4, 1000, 0, ctypes.c_void_p(0x100010), need,
                                 None) == _lib.RT_ERR_INVALID_ARG
    # nothing to sort: no device work, even with NULL pointers
    assert so.rt_sort_pairs_batched(None, None, None, 0, 1000, None) == _lib.RT_OK
    assert so.rt_sort_pairs_batched(None, None, None, 5, 1, None) == _lib.RT_OK


def test_batched_workspace_bytes(so):
    assert so.rt_batched_workspace_bytes(0, 1000, 1) == 0
    assert so.rt_batched_workspace_bytes(10, 1, 1) == 0
    assert so.rt_batched_workspace_bytes(10, 1 << 32, 1) == 0
    cap = 1 << 27
    with_v = so.rt_batched_workspace_bytes(4096, cap, 1)
    keys = so.rt_batched_workspace_bytes(4096, cap, 0)
    # one temporary per array of the full capacity, plus modest metadata
    assert with_v - keys >= 4 * cap
    assert keys >= 4 * cap and keys < 4 * cap + (128 << 20)


def test_msd_first_argument_errors(so):
    fake = ctypes.c_void_p(0x10000)
    assert so.rt_sort_msd_first(fake, None, 1 << 32, 0, None, 0, None) == _lib.RT_ERR_TOO_LARGE
    assert so.rt_sort_msd_first(None, None, 100, 0, None, 0, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort_msd_first(ctypes.c_void_p(0x10002), None, 100, 0, None, 0, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort_msd_first(fake, ctypes.c_void_p(0x10100), 100, 0, None, 0, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort_msd_first(fake, None, 100, 0x1, None, 0, None) == _lib.RT_ERR_INVALID_ARG  # unknown flag
    need = so.rt_msd_first_workspace_bytes(100, 0)
    assert so.rt_sort_msd_first(fake, None, 100, 0, ctypes.c_void_p(0x100000), need - 1,
                                None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort_msd_first(fake, None, 100, 0, ctypes.c_void_p(0x100010), need,
                                None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort_msd_first(None, None, 1, 0, None, 0, None) == _lib.RT_OK  # nothing to sort


def test_msd_first_workspace_bytes(so):
    assert so.rt_msd_first_workspace_bytes(1, 1) == 0
    assert so.rt_msd_first_workspace_bytes(1 << 32, 1) == 0
    n = 1 << 28
    with_v = so.rt_msd_first_workspace_bytes(n, 1)
    keys = so.rt_msd_first_workspace_bytes(n, 0)
    # one temporary per array (the local passes use the caller's arrays as
    # the other buffer), plus lookback words and tables (whose size follows
    # the tuned tile of each); the second MSD level's tables are sized for
    # the most sub-buckets that can be too large for the LDS (n / 16385),
    # about one byte per item
    assert abs((with_v - keys) - 4 * n) < (16 << 20)
    assert keys >= 4 * n and keys < 5 * n + (128 << 20)


def test_sort64_argument_errors(so):
    fake_k, fake_v = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x900000)
    assert so.rt_sort_keys64(fake_k, 1 << 32, None) == _lib.RT_ERR_TOO_LARGE
    assert so.rt_sort_keys64(None, 10, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort_keys64(ctypes.c_void_p(0x10004), 10, None) == _lib.RT_ERR_INVALID_ARG  # not 8-aligned
    assert so.rt_sort_pairs64(fake_k, None, 10, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort64_ex(fake_k, fake_v, 3, 10, None, None, 0, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort64_ex(fake_k, None, 4, 10, None, None, 0, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort64_ex(fake_k, ctypes.c_void_p(0x900004), 8, 10, None, None, 0, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort64_ex(fake_k, ctypes.c_void_p(0x10040), 4, 10, None, None, 0, None) \
        == _lib.RT_ERR_INVALID_ARG  # overlap
    c = _lib.RtConfig()
    c.num_passes = 4
    for i in range(4):
        c.digit_bits[i] = 8  # sums to 32, not 64
    assert so.rt_sort64_ex(fake_k, fake_v, 4, 10, ctypes.byref(c), None, 0, None) == _lib.RT_ERR_INVALID_ARG
    c = _lib.RtConfig()
    c.flags = _lib.RT_FLAG_NT_STORES
    assert so.rt_sort64_ex(fake_k, fake_v, 4, 10, ctypes.byref(c), None, 0, None) == _lib.RT_ERR_UNSUPPORTED
    c = _lib.RtConfig()
    c.block_threads, c.items_per_thread = 256, 16  # not built for 64-bit keys
    assert so.rt_sort64_ex(fake_k, fake_v, 4, 10, ctypes.byref(c), None, 0, None) == _lib.RT_ERR_UNSUPPORTED
    need = so.rt_workspace_bytes64(100, 4, None)
    assert so.rt_sort64_ex(fake_k, fake_v, 4, 100, None, ctypes.c_void_p(0x100000), need - 1,
                           None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_sort_keys64(None, 1, None) == _lib.RT_OK


def test_sort64_workspace_bytes(so):
    assert so.rt_workspace_bytes64(1, 4, None) == 0
    assert so.rt_workspace_bytes64(100, 3, None) == 0
    n = 1 << 20
    k0 = so.rt_workspace_bytes64(n, 0, None)
    k4 = so.rt_workspace_bytes64(n, 4, None)
    k8 = so.rt_workspace_bytes64(n, 8, None)
    # two temporaries per array (skipping may leave an odd pass count)
    assert k0 >= 2 * 8 * n and k4 - k0 == 2 * 4 * n and k8 - k0 == 2 * 8 * n


def test_server_argument_errors(so):
    out = ctypes.c_void_p()
    assert so.rt_server_create(1 << 30, 0, ctypes.byref(out)) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_server_create(1000, 8, ctypes.byref(out)) == _lib.RT_ERR_INVALID_ARG  # budget below 1 MiB
    assert so.rt_server_create(1 << 30, 8, None) == _lib.RT_ERR_INVALID_ARG
    t = ctypes.c_uint64()
    assert so.rt_server_submit(None, None, None, None, None, 0, ctypes.byref(t)) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_server_submit_generated(None, None, 10, ctypes.byref(t)) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_server_wait(None, 1, 0, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_server_replay(None, None, 0, None, None) == _lib.RT_ERR_INVALID_ARG
    assert ctypes.sizeof(_lib.RtReplayRequest) == 224 and _lib.RtReplayRequest.params.offset == 16
    assert so.rt_server_wait_any(None, 0, ctypes.byref(t), None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_server_fetch(None, 1, None, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_server_release(None, 1) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_server_cancel(None, 1) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_server_stats(None, None, None, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_server_stats_ex(None, None, None, None, None, None) == _lib.RT_ERR_INVALID_ARG
    assert so.rt_server_destroy(None) == _lib.RT_OK


def test_committed_tuning_table_loads(so):
    """The autotuner's table for gfx950 parses, and every entry names a
    compiled configuration (the library validates each on load)."""
    path = os.path.join(ROOT, "paper_1008_2849_amd", "tuning", "gfx950.json")
    table = json.load(open(path))
    assert table["arch"] == "gfx950" and table["entries"]
    assert so.rt_load_tuning(path.encode()) == _lib.RT_OK
    c = _lib.RtConfig()
    for e in table["entries"]:
        if e["op"] in ("segments", "segments_tiled"):
            continue
        n = max(2, e["min_n"])
        assert so.rt_tuned_config(n, 1 if e["op"] == "pairs" else 0, ctypes.byref(c)) == _lib.RT_OK
        assert [c.digit_bits[i] for i in range(c.num_passes)] == e["digit_bits"]
        assert (c.block_threads, c.items_per_thread, c.flags) == (e["block"], e["ipt"], e["flags"])
    from paper_1008_2849_amd import api
    seg = [(e["max_n"], e["block"], e["ipt"]) for e in table["entries"] if e["op"] == "segments"]
    assert seg and api.segment_classes() == seg
    bits = [8 if e["digit_bits"][0] == 8 else 11 for e in table["entries"] if e["op"] == "segments"]
    tile = [(e["block"], e["ipt"]) for e in table["entries"] if e["op"] == "segments_tiled"]
    assert api.segment_config() == (bits, tile[0] if tile else (1024, 16))
    assert so.rt_load_tuning(None) == _lib.RT_OK


def test_autotuner_segment_shapes_match_the_library(so, tmp_path):
    """Every whole-in-LDS shape the autotuner may try loads as a class, and
    an 8-bit-only shape is refused with 11-bit digits (host-side checks)."""
    import json
    from paper_1008_2849_amd import autotune

    def load(block, ipt, bits):
        path = tmp_path / "t.json"
        path.write_text(json.dumps({"entries": [
            {"op": "segments", "min_n": 0, "max_n": min(block * ipt, 16384), "block": block, "ipt": ipt,
             "digit_bits": list(autotune.SEG_BITS[bits])}]}))
        return so.rt_load_tuning(str(path).encode())

    try:
        for b, i in autotune.SEG_SHAPES:
            assert load(b, i, 8) == 0, (b, i, 8)
        for b, i in autotune.SEG_SHAPES_11:
            assert load(b, i, 11) == 0, (b, i, 11)
        for b, i in set(autotune.SEG_SHAPES) - set(autotune.SEG_SHAPES_11):
            assert load(b, i, 11) == _lib.RT_ERR_INVALID_ARG, (b, i, 11)
    finally:
        from paper_1008_2849_amd import api
        api.load_default_tuning()  # the committed table, as the package loads it
