// rt_tuning.cpp -- tuned configurations: built-in defaults and the JSON table
// written by the autotuner (paper_1008_2849_amd/autotune.py).
//
// Table format:
//   {"arch": "gfx950", "entries": [
//      {"op": "keys"|"pairs"|"segments"|"segments_tiled", "min_n": N0, "max_n": N1,
//       "digit_bits": [w0, w1, ...], "block": B, "ipt": I, "flags": F}, ...]}
// A "keys" or "pairs" entry applies to single-array sorts of n in
// [min_n, max_n]; the first matching entry wins.  The "segments" entries, in
// increasing max_n, are the whole-in-LDS size classes of the segmented sort
// (batched calls, the MSD-first sort's buckets, small server requests): each
// sorts the segments of up to max_n items (and more than the previous
// entry's) in one block of B threads x I items, with the entry's digits
// (8,8,8,8 or 11,11,10); larger segments are tiled.  A "segments_tiled"
// entry sets the tile (B x I items, 1024x16 or 512x16) of the tiled
// segments' passes in batched calls and MSD-first sorts.  Without
// "segments" entries the built-in classes hold.
#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "rt_common.h"

namespace rt {

namespace {

// ---- minimal JSON reader (objects, arrays, numbers, strings, literals) ----
struct JValue {
    enum Kind { Null, Bool, Number, String, Array, Object } kind = Null;
    double num = 0;
    bool b = false;
    std::string str;
    std::vector<JValue> arr;
    std::vector<std::pair<std::string, JValue>> obj;
    const JValue *get(const char *key) const {
        for (const auto &kv : obj)
            if (kv.first == key) return &kv.second;
        return nullptr;
    }
};

struct JParser {
    const char *p;
    const char *end;
    std::string err;

    void ws() {
        while (p < end && isspace(static_cast<unsigned char>(*p))) ++p;
    }
    bool fail(const char *m) {
        if (err.empty()) err = m;
        return false;
    }
    bool parse_string(std::string &out) {
        if (p >= end || *p != '"') return fail("expected string");
        ++p;
        while (p < end && *p != '"') {
            if (*p == '\\') {
                ++p;
                if (p >= end) return fail("bad escape");
            }
            out.push_back(*p++);
        }
        if (p >= end) return fail("unterminated string");
        ++p;
        return true;
    }
    bool parse(JValue &v, int depth) {
        if (depth > 32) return fail("nesting too deep");
        ws();
        if (p >= end) return fail("unexpected end");
        if (*p == '{') {
            v.kind = JValue::Object;
            ++p;
            ws();
            if (p < end && *p == '}') { ++p; return true; }
            for (;;) {
                std::string k;
                ws();
                if (!parse_string(k)) return false;
                ws();
                if (p >= end || *p != ':') return fail("expected ':'");
                ++p;
                JValue child;
                if (!parse(child, depth + 1)) return false;
                v.obj.emplace_back(std::move(k), std::move(child));
                ws();
                if (p < end && *p == ',') { ++p; continue; }
                if (p < end && *p == '}') { ++p; return true; }
                return fail("expected ',' or '}'");
            }
        }
        if (*p == '[') {
            v.kind = JValue::Array;
            ++p;
            ws();
            if (p < end && *p == ']') { ++p; return true; }
            for (;;) {
                JValue child;
                if (!parse(child, depth + 1)) return false;
                v.arr.push_back(std::move(child));
                ws();
                if (p < end && *p == ',') { ++p; continue; }
                if (p < end && *p == ']') { ++p; return true; }
                return fail("expected ',' or ']'");
            }
        }
        if (*p == '"') {
            v.kind = JValue::String;
            return parse_string(v.str);
        }
        if (!strncmp(p, "true", 4)) { v.kind = JValue::Bool; v.b = true; p += 4; return true; }
        if (!strncmp(p, "false", 5)) { v.kind = JValue::Bool; v.b = false; p += 5; return true; }
        if (!strncmp(p, "null", 4)) { v.kind = JValue::Null; p += 4; return true; }
        char *q = nullptr;
        v.num = strtod(p, &q);
        if (q == p) return fail("bad value");
        v.kind = JValue::Number;
        p = q;
        return true;
    }
};

struct Entry {
    int op;  // 0 keys, 1 pairs, 2 segments, 3 segments_tiled
    double min_n, max_n;
    rt_config cfg;
};

std::mutex g_mu;
std::vector<Entry> g_table;
bool g_seg_tuned = false;
SegClassTable g_seg;

SegClassTable builtin_seg_classes() {
    SegClassTable t{};
    t.count = 3;
    t.cls[0] = SegClass{256 * 8, 256, 8, 8};
    t.cls[1] = SegClass{512 * 16, 512, 16, 8};
    t.cls[2] = SegClass{1024 * 16, 1024, 16, 8};
    t.tile_block = 1024;
    t.tile_ipt = 16;
    return t;
}

void builtin(size_t n, int op, rt_config *out) {
    (void)n;
    (void)op;
    memset(out, 0, sizeof *out);
    out->num_passes = 4;
    for (int p = 0; p < 4; ++p) out->digit_bits[p] = 8;
    // 16K-item tiles: the largest that fits LDS for key/value pairs, and the
    // fastest measured on gfx950 (longer digit runs, shorter lookback chains)
    out->block_threads = 1024;
    out->items_per_thread = 16;
    out->flags = 0;
}

}  // namespace

void tuned_config_op(size_t n, int op, rt_config *out) {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (const Entry &e : g_table) {
            if (e.op == op && static_cast<double>(n) >= e.min_n && static_cast<double>(n) <= e.max_n) {
                *out = e.cfg;
                return;
            }
        }
    }
    builtin(n, op, out);
}

void tuned_config(size_t n, int with_values, rt_config *out) { tuned_config_op(n, with_values ? 1 : 0, out); }

SegClassTable seg_class_table() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_seg_tuned ? g_seg : builtin_seg_classes();
}

}  // namespace rt

using namespace rt;

extern "C" rt_status rt_load_tuning(const char *json_path) {
    if (json_path == nullptr) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table.clear();
        g_seg_tuned = false;
        return RT_OK;
    }
    FILE *f = fopen(json_path, "rb");
    if (!f) return set_error(RT_ERR_INVALID_ARG, "rt_load_tuning: cannot open %s", json_path);
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    JParser jp{text.data(), text.data() + text.size(), {}};
    JValue root;
    if (!jp.parse(root, 0) || root.kind != JValue::Object)
        return set_error(RT_ERR_INVALID_ARG, "rt_load_tuning: %s: %s", json_path,
                         jp.err.empty() ? "top level is not an object" : jp.err.c_str());
    const JValue *entries = root.get("entries");
    if (!entries || entries->kind != JValue::Array)
        return set_error(RT_ERR_INVALID_ARG, "rt_load_tuning: no \"entries\" array");
    std::vector<Entry> table;
    SegClassTable seg{};
    for (size_t i = 0; i < entries->arr.size(); ++i) {
        const JValue &e = entries->arr[i];
        const JValue *op = e.get("op"), *lo = e.get("min_n"), *hi = e.get("max_n"), *bits = e.get("digit_bits"),
                     *block = e.get("block"), *ipt = e.get("ipt"), *flags = e.get("flags");
        if (!op || op->kind != JValue::String || !lo || !hi || !bits || bits->kind != JValue::Array || !block ||
            !ipt)
            return set_error(RT_ERR_INVALID_ARG, "rt_load_tuning: entry %zu is incomplete", i);
        Entry en{};
        if (op->str == "keys") en.op = 0;
        else if (op->str == "pairs") en.op = 1;
        else if (op->str == "segments") en.op = 2;
        else if (op->str == "segments_tiled") en.op = 3;
        else return set_error(RT_ERR_INVALID_ARG, "rt_load_tuning: entry %zu: unknown op %s", i, op->str.c_str());
        en.min_n = lo->num;
        en.max_n = hi->num;
        if (bits->arr.empty() || bits->arr.size() > static_cast<size_t>(kMaxPasses))
            return set_error(RT_ERR_INVALID_ARG, "rt_load_tuning: entry %zu: bad digit_bits", i);
        en.cfg.num_passes = static_cast<uint32_t>(bits->arr.size());
        for (size_t p = 0; p < bits->arr.size(); ++p) en.cfg.digit_bits[p] = static_cast<uint32_t>(bits->arr[p].num);
        en.cfg.block_threads = static_cast<uint32_t>(block->num);
        en.cfg.items_per_thread = static_cast<uint32_t>(ipt->num);
        en.cfg.flags = flags ? static_cast<uint32_t>(flags->num) : 0u;
        Resolved r;
        if (en.op < 2) {  // a single-array sort
            if (resolve_config(&en.cfg, 1024, en.op, &r) != RT_OK)
                return set_error(RT_ERR_INVALID_ARG, "rt_load_tuning: entry %zu: %s", i, last_error());
            table.push_back(en);
            continue;
        }
        const int blk = static_cast<int>(en.cfg.block_threads), ip = static_cast<int>(en.cfg.items_per_thread);
        // digits of the segmented sort: four of 8 bits, or (whole-in-LDS
        // classes) 11, 11 and 10 bits
        bool eight = en.cfg.num_passes == static_cast<uint32_t>(kSegPasses);
        for (uint32_t p = 0; p < en.cfg.num_passes; ++p) eight = eight && en.cfg.digit_bits[p] == kSegBits;
        const bool eleven = en.cfg.num_passes == 3 && en.cfg.digit_bits[0] == 11 && en.cfg.digit_bits[1] == 11 &&
                            en.cfg.digit_bits[2] == 10;
        if (en.op == 3) {  // the tile of the tiled segments' passes
            if (!eight || !seg_tile_shape_supported(blk, ip))
                return set_error(RT_ERR_INVALID_ARG,
                                 "rt_load_tuning: entry %zu: tiled segments take four 8-bit digits and a built "
                                 "tile shape (1024x16 or 512x16), not %dx%d",
                                 i, blk, ip);
            seg.tile_block = blk;
            seg.tile_ipt = ip;
            continue;
        }
        // a whole-in-LDS class of the segmented sort
        if (!eight && !eleven)
            return set_error(RT_ERR_INVALID_ARG,
                             "rt_load_tuning: entry %zu: segments use digits 8,8,8,8 or 11,11,10", i);
        const int cbits = eight ? 8 : 11;
        if (!seg_small_shape_supported(blk, ip, cbits))
            return set_error(RT_ERR_INVALID_ARG, "rt_load_tuning: entry %zu: no whole-in-LDS kernel %dx%d with "
                             "%d-bit digits", i, blk, ip, cbits);
        if (seg.count == static_cast<uint32_t>(kSegMaxClasses))
            return set_error(RT_ERR_INVALID_ARG, "rt_load_tuning: more than %d segment classes", kSegMaxClasses);
        const double prev = seg.count ? seg.cls[seg.count - 1].max_n : 0.0;
        if (en.max_n <= prev || en.max_n > static_cast<double>(blk) * ip || en.max_n > kSegLdsMax)
            return set_error(RT_ERR_INVALID_ARG,
                             "rt_load_tuning: entry %zu: segment class limit %.0f must rise, fit %dx%d and be at "
                             "most %u",
                             i, en.max_n, blk, ip, kSegLdsMax);
        seg.cls[seg.count++] = SegClass{static_cast<uint32_t>(en.max_n), blk, ip, cbits};
    }
    if (seg.count > 0 && seg.tile_block == 0) {  // classes without a tile entry: the built-in tile
        seg.tile_block = 1024;
        seg.tile_ipt = 16;
    }
    if (seg.count == 0 && seg.tile_block != 0) {  // a tile entry alone keeps the built-in classes
        SegClassTable b = builtin_seg_classes();
        b.tile_block = seg.tile_block;
        b.tile_ipt = seg.tile_ipt;
        seg = b;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.swap(table);
    g_seg_tuned = seg.count > 0;
    g_seg = seg;
    return RT_OK;
}

extern "C" rt_status rt_segment_config(uint32_t *bits, uint32_t *tile_block, uint32_t *tile_ipt) {
    const SegClassTable t = seg_class_table();
    for (uint32_t c = 0; c < t.count; ++c)
        if (bits) bits[c] = static_cast<uint32_t>(t.cls[c].bits);
    if (tile_block) *tile_block = static_cast<uint32_t>(t.tile_block);
    if (tile_ipt) *tile_ipt = static_cast<uint32_t>(t.tile_ipt);
    return RT_OK;
}

extern "C" rt_status rt_segment_classes(uint32_t *count, uint32_t *max_n, uint32_t *block, uint32_t *ipt) {
    if (count == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_segment_classes: count is NULL");
    const SegClassTable t = seg_class_table();
    *count = t.count;
    for (uint32_t c = 0; c < t.count; ++c) {
        if (max_n) max_n[c] = t.cls[c].max_n;
        if (block) block[c] = static_cast<uint32_t>(t.cls[c].block);
        if (ipt) ipt[c] = static_cast<uint32_t>(t.cls[c].ipt);
    }
    return RT_OK;
}

extern "C" rt_status rt_tuned_config(size_t n, int with_values, rt_config *out) {
    if (out == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_tuned_config: out is NULL");
    tuned_config(n, with_values, out);
    return RT_OK;
}
