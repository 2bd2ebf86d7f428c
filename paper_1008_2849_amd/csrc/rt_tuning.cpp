// rt_tuning.cpp -- tuned configurations: built-in defaults and the JSON table
// written by the autotuner (paper_1008_2849_amd/autotune.py).
//
// Table format:
//   {"arch": "gfx950", "entries": [
//      {"op": "keys"|"pairs"|"segments", "min_n": N0, "max_n": N1,
//       "digit_bits": [w0, w1, ...], "block": B, "ipt": I, "flags": F}, ...]}
// An entry applies to n in [min_n, max_n]; the first matching entry wins.
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
    int op;  // 0 keys, 1 pairs, 2 segments
    double min_n, max_n;
    rt_config cfg;
};

std::mutex g_mu;
std::vector<Entry> g_table;

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

}  // namespace rt

using namespace rt;

extern "C" rt_status rt_load_tuning(const char *json_path) {
    if (json_path == nullptr) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_table.clear();
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
        if (en.op != 2) {
            if (resolve_config(&en.cfg, 1024, en.op, &r) != RT_OK)
                return set_error(RT_ERR_INVALID_ARG, "rt_load_tuning: entry %zu: %s", i, last_error());
        }
        table.push_back(en);
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.swap(table);
    return RT_OK;
}

extern "C" rt_status rt_tuned_config(size_t n, int with_values, rt_config *out) {
    if (out == nullptr) return set_error(RT_ERR_INVALID_ARG, "rt_tuned_config: out is NULL");
    tuned_config(n, with_values, out);
    return RT_OK;
}
