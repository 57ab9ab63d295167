// tune.cpp - the autotuner's records: launch shapes chosen by timing, kept per
// (GPU architecture, compute-unit count, problem kind, size class) and
// persisted as a JSON cache.
//
// A size class is floor(log2(size)): the instance count of a batch, the arc
// count of a graph.  A solve that leaves its shape to the library takes the
// record of its own class on the current device, else the record of the
// nearest class of the same kind, else the built-in default.  Records made on
// another architecture or CU count are kept (a cache can serve several
// machines) but never used on this one.
//
// File format (written by tune_save, read back by tune_load):
//   {"llp_autotune": 1, "entries": [
//    {"arch": "gfx950", "cus": 256, "kind": "batch", "size_class": 13, "block": 512, "chunk": 1},
//    ...]}
// Host code only.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "llp_host.h"

namespace llp {

namespace {

struct Rec {
    int block, chunk;
    unsigned long long seq;   // recording order (the most recent answers llp_autotune_get)
};
using Key = std::tuple<std::string, int, int, int>;   // arch, cus, kind, class

std::mutex g_tmu;
std::map<Key, Rec> g_recs;
unsigned long long g_seq = 0;

std::string arch_name(const std::string& full) {
    // "gfx950:sramecc+:xnack-" -> "gfx950"
    const size_t c = full.find(':');
    return c == std::string::npos ? full : full.substr(0, c);
}

const char* kind_name(int kind) {
    switch (kind) {
        case LLP_KIND_BATCH: return "batch";
        case LLP_KIND_SSSP: return "sssp";
        case LLP_KIND_BFS: return "bfs";
        default: return nullptr;
    }
}

int kind_of(const std::string& s) {
    if (s == "batch") return LLP_KIND_BATCH;
    if (s == "sssp") return LLP_KIND_SSSP;
    if (s == "bfs") return LLP_KIND_BFS;
    return -1;
}

bool valid(int kind, int cls, int cus, int block, int chunk) {
    if (!kind_name(kind) || cls < 0 || cls > 62 || cus < 1 || chunk < 1 || chunk > 64) return false;
    if (kind == LLP_KIND_BATCH) return block >= 64 && block <= 1024 && block % 64 == 0;
    return block == 0 && chunk <= 4;   // the graph tuner's candidates: 1 to 4 workgroups per CU
}

// the text of field key in the object [b, e): a quoted string's contents or a number
bool field(const std::string& s, size_t b, size_t e, const char* key, std::string* out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = s.find(k, b);
    if (p == std::string::npos || p >= e) return false;
    p = s.find(':', p + k.size());
    if (p == std::string::npos || p >= e) return false;
    ++p;
    while (p < e && (s[p] == ' ' || s[p] == '\t' || s[p] == '\n' || s[p] == '\r')) ++p;
    if (p >= e) return false;
    if (s[p] == '"') {
        const size_t q = s.find('"', p + 1);
        if (q == std::string::npos || q >= e) return false;
        *out = s.substr(p + 1, q - p - 1);
        return true;
    }
    size_t q = p;
    while (q < e && (s[q] == '-' || (s[q] >= '0' && s[q] <= '9'))) ++q;
    if (q == p) return false;
    *out = s.substr(p, q - p);
    return true;
}

bool int_field(const std::string& s, size_t b, size_t e, const char* key, int* v) {
    std::string t;
    if (!field(s, b, e, key, &t)) return false;
    char* end = nullptr;
    const long x = strtol(t.c_str(), &end, 10);
    if (!end || *end || x < -2147483647l || x > 2147483647l) return false;
    *v = (int)x;
    return true;
}

}  // namespace

int size_class(long long size) {
    int c = 0;
    while (size > 1 && c < 62) {
        size >>= 1;
        ++c;
    }
    return c;
}

void tune_record(int kind, long long size, int block, int chunk) {
    const DeviceInfo& d = device_info();
    std::lock_guard<std::mutex> lk(g_tmu);
    g_recs[Key(arch_name(d.arch), d.cus, kind, size_class(size))] = Rec{block, chunk, ++g_seq};
}

bool tune_lookup(int kind, long long size, int* block, int* chunk) {
    const DeviceInfo& d = device_info();
    const std::string arch = arch_name(d.arch);
    const int cls = size_class(size);
    std::lock_guard<std::mutex> lk(g_tmu);
    const Rec* best = nullptr;
    int best_dist = 1 << 30;
    for (const auto& kv : g_recs) {
        if (std::get<0>(kv.first) != arch || std::get<1>(kv.first) != d.cus || std::get<2>(kv.first) != kind) continue;
        const int dist = abs(std::get<3>(kv.first) - cls);
        // nearest class; between two at the same distance, the larger
        if (dist < best_dist || (dist == best_dist && std::get<3>(kv.first) > cls)) {
            best = &kv.second;
            best_dist = dist;
        }
    }
    if (!best) return false;
    if (block) *block = best->block;
    if (chunk) *chunk = best->chunk;
    return true;
}

bool tune_last(int kind, int* block, int* chunk) {
    const DeviceInfo& d = device_info();
    const std::string arch = arch_name(d.arch);
    std::lock_guard<std::mutex> lk(g_tmu);
    const Rec* last = nullptr;
    for (const auto& kv : g_recs)
        if (std::get<0>(kv.first) == arch && std::get<1>(kv.first) == d.cus && std::get<2>(kv.first) == kind &&
            (!last || kv.second.seq > last->seq))
            last = &kv.second;
    if (!last) return false;
    if (block) *block = last->block;
    if (chunk) *chunk = last->chunk;
    return true;
}

void tune_clear() {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_recs.clear();
}

int tune_save(const char* path) {
    if (!path || !*path) return fail(LLP_E_ARG, "a cache path is required");
    std::string text = "{\"llp_autotune\": 1, \"entries\": [";
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        bool first = true;
        for (const auto& kv : g_recs) {
            text += first ? "\n {\"arch\": \"" : ",\n {\"arch\": \"";
            text += std::get<0>(kv.first);
            text += "\", \"cus\": " + std::to_string(std::get<1>(kv.first));
            text += ", \"kind\": \"" + std::string(kind_name(std::get<2>(kv.first)));
            text += "\", \"size_class\": " + std::to_string(std::get<3>(kv.first));
            text += ", \"block\": " + std::to_string(kv.second.block);
            text += ", \"chunk\": " + std::to_string(kv.second.chunk) + "}";
            first = false;
        }
    }
    text += "\n]}\n";
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "wb");
    if (!f) return fail(LLP_E_ARG, "cannot write %s", tmp.c_str());
    const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
    if (fclose(f) != 0 || !ok) {
        remove(tmp.c_str());
        return fail(LLP_E_ARG, "cannot write %s", tmp.c_str());
    }
    if (rename(tmp.c_str(), path) != 0) {
        remove(tmp.c_str());
        return fail(LLP_E_ARG, "cannot replace %s", path);
    }
    return LLP_OK;
}

int tune_load(const char* path, int* loaded) {
    if (loaded) *loaded = 0;
    if (!path || !*path) return fail(LLP_E_ARG, "a cache path is required");
    FILE* f = fopen(path, "rb");
    if (!f) return fail(LLP_E_ARG, "cannot open %s", path);
    std::string s;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof(buf), f)) > 0) {
        s.append(buf, k);
        if (s.size() > (64u << 20)) {
            fclose(f);
            return fail(LLP_E_INPUT, "%s is larger than 64 MB", path);
        }
    }
    fclose(f);
    if (s.find("\"llp_autotune\"") == std::string::npos) return fail(LLP_E_INPUT, "%s is not an autotuner cache", path);
    // every object holding an "arch" field is an entry; all are checked before any is taken
    std::map<Key, Rec> add;
    for (size_t p = s.find("\"arch\""); p != std::string::npos; p = s.find("\"arch\"", p + 1)) {
        const size_t b = s.rfind('{', p), e = s.find('}', p);
        if (b == std::string::npos || e == std::string::npos) return fail(LLP_E_INPUT, "%s: unbalanced entry", path);
        std::string arch, kind;
        int cus = 0, cls = 0, block = 0, chunk = 0;
        if (!field(s, b, e, "arch", &arch) || !field(s, b, e, "kind", &kind) || !int_field(s, b, e, "cus", &cus) ||
            !int_field(s, b, e, "size_class", &cls) || !int_field(s, b, e, "block", &block) ||
            !int_field(s, b, e, "chunk", &chunk))
            return fail(LLP_E_INPUT, "%s: entry at byte %zu lacks a field", path, b);
        const int kd = kind_of(kind);
        bool name_ok = !arch.empty() && arch.size() <= 64;
        for (char ch : arch)
            name_ok = name_ok && ((ch >= 'a' && ch <= 'z') || (ch >= 'A' && ch <= 'Z') || (ch >= '0' && ch <= '9') ||
                                  ch == '_' || ch == '-' || ch == '.' || ch == '+');
        if (!name_ok || !valid(kd, cls, cus, block, chunk))
            return fail(LLP_E_INPUT, "%s: entry at byte %zu is out of range", path, b);
        add[Key(arch, cus, kd, cls)] = Rec{block, chunk, 0};
    }
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto& kv : add) {
        kv.second.seq = ++g_seq;
        g_recs[kv.first] = kv.second;
    }
    if (loaded) *loaded = (int)add.size();
    return LLP_OK;
}

}  // namespace llp

extern "C" {

int llp_autotune_save(const char* path) { return llp::tune_save(path); }

int llp_autotune_load(const char* path, int32_t* loaded) {
    int n = 0;
    const int s = llp::tune_load(path, &n);
    if (loaded) *loaded = n;
    return s;
}

int llp_autotune_lookup(int32_t kind, int64_t size, int32_t* block, int32_t* chunk) {
    if (kind != LLP_KIND_BATCH && kind != LLP_KIND_SSSP && kind != LLP_KIND_BFS)
        return llp::fail(LLP_E_ARG, "kind must be LLP_KIND_BATCH, LLP_KIND_SSSP or LLP_KIND_BFS");
    if (size < 0) return llp::fail(LLP_E_ARG, "size must be >= 0");
    int b = 0, c = 0;
    if (!llp::tune_lookup(kind, size, &b, &c)) return llp::fail(LLP_E_ARG, "no record for this kind on this device");
    if (block) *block = b;
    if (chunk) *chunk = c;
    return LLP_OK;
}

}  // extern "C"
