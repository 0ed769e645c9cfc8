// Measured tuning of launch configurations (host code).
//
// Three kernel families have more than one correct launch configuration:
//   square    16-bit levels: 256 x 256 tiles on 8 waves (32 x 32 x 16 or
//             16 x 16 x 32 MFMAs) or on 4 waves (32 x 32 x 16), the last
//             partial round of workgroups split over k or not (6 candidates)
//   apply     16-bit and FP32 levels: the split-K count of the chain
//             application (default, half, double: 3 candidates)
//   residual  the split-K count of the FP64 residual product (3 candidates)
// A context in tuning mode times every candidate of a (family, type, shape)
// the first time it meets it, on the call's own data, and keeps the fastest;
// the choices and their times live in one table per process (keyed by the
// GPU's architecture name) that can be saved to and loaded from a JSON file
// (CDL_AUTOTUNE_CACHE names one that is loaded on first use and rewritten
// after every new entry).  The measured times also feed the chain-depth cost
// model.
#include <hip/hip_runtime.h>

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "tune.h"

namespace cdl {

namespace {

struct TuneEntry {
    int choice = 0;
    std::vector<double> ms;
};

std::mutex g_mu;
std::map<std::string, TuneEntry> g_table;   // "arch|key"
bool g_env_loaded = false;
std::map<int, std::string> g_arch;          // device -> architecture name

const char *prec_name(int prec) {
    switch (prec) {
    case 0: return "fp64";
    case 1: return "fp32";
    case 2: return "bf16";
    default: return "fp16";
    }
}

// ---- a small JSON reader for the cache file's own format --------------------

struct Json {
    enum Kind { NUL, NUM, STR, ARR, OBJ } kind = NUL;
    double num = 0.0;
    std::string str;
    std::vector<Json> arr;
    std::vector<std::pair<std::string, Json>> obj;
    const Json *get(const char *k) const {
        for (const auto &kv : obj)
            if (kv.first == k) return &kv.second;
        return nullptr;
    }
};

struct Parser {
    const char *p, *end;
    bool ok = true;
    void ws() {
        while (p < end && std::isspace((unsigned char)*p)) ++p;
    }
    bool lit(const char *w) {
        const size_t n = std::strlen(w);
        if ((size_t)(end - p) >= n && std::strncmp(p, w, n) == 0) {
            p += n;
            return true;
        }
        return false;
    }
    std::string string() {
        std::string out;
        if (p >= end || *p != '"') { ok = false; return out; }
        ++p;
        while (p < end && *p != '"') {
            if (*p == '\\' && p + 1 < end) ++p;
            out.push_back(*p++);
        }
        if (p >= end) { ok = false; return out; }
        ++p;
        return out;
    }
    Json value(int depth) {
        Json v;
        ws();
        if (!ok || p >= end || depth > 16) { ok = false; return v; }
        if (*p == '{') {
            v.kind = Json::OBJ;
            ++p;
            ws();
            if (p < end && *p == '}') { ++p; return v; }
            while (ok) {
                ws();
                std::string k = string();
                ws();
                if (p >= end || *p != ':') { ok = false; break; }
                ++p;
                v.obj.emplace_back(k, value(depth + 1));
                ws();
                if (p < end && *p == ',') { ++p; continue; }
                if (p < end && *p == '}') { ++p; break; }
                ok = false;
            }
        } else if (*p == '[') {
            v.kind = Json::ARR;
            ++p;
            ws();
            if (p < end && *p == ']') { ++p; return v; }
            while (ok) {
                v.arr.push_back(value(depth + 1));
                ws();
                if (p < end && *p == ',') { ++p; continue; }
                if (p < end && *p == ']') { ++p; break; }
                ok = false;
            }
        } else if (*p == '"') {
            v.kind = Json::STR;
            v.str = string();
        } else if (lit("null")) {
            v.kind = Json::NUL;
        } else {
            char *q = nullptr;
            v.num = std::strtod(p, &q);
            if (q == p) { ok = false; return v; }
            v.kind = Json::NUM;
            p = q;
        }
        return v;
    }
};

bool read_file(const char *path, std::string &out) {
    FILE *f = std::fopen(path, "rb");
    if (!f) return false;
    char buf[65536];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) out.append(buf, got);
    std::fclose(f);
    return true;
}

// Merges the entries of `path` into the table (caller holds the lock).
bool load_locked(const char *path, std::string *err) {
    std::string text;
    if (!read_file(path, text)) {
        if (err) *err = std::string("cannot read ") + path;
        return false;
    }
    Parser ps{text.data(), text.data() + text.size()};
    Json root = ps.value(0);
    const Json *fmt = root.get("format");
    const Json *ents = root.get("entries");
    if (!ps.ok || root.kind != Json::OBJ || !fmt || fmt->kind != Json::STR ||
        fmt->str != "caddelag-autotune-1" || !ents || ents->kind != Json::ARR) {
        if (err) *err = std::string("not an autotune cache: ") + path;
        return false;
    }
    for (const Json &e : ents->arr) {
        const Json *arch = e.get("arch"), *key = e.get("key"), *ch = e.get("choice"),
                   *ms = e.get("ms");
        if (!arch || !key || !ch || !ms || arch->kind != Json::STR || key->kind != Json::STR ||
            ch->kind != Json::NUM || ms->kind != Json::ARR)
            continue;
        TuneEntry t;
        t.choice = (int)ch->num;
        for (const Json &m : ms->arr) t.ms.push_back(m.kind == Json::NUM ? m.num : -1.0);
        if (t.choice < 0 || t.choice >= (int)t.ms.size()) continue;
        g_table[arch->str + "|" + key->str] = t;
    }
    return true;
}

bool save_locked(const char *path, std::string *err) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) {
        if (err) *err = std::string("cannot write ") + tmp;
        return false;
    }
    std::fprintf(f, "{\n  \"format\": \"caddelag-autotune-1\",\n  \"entries\": [");
    bool first = true;
    for (const auto &kv : g_table) {
        const size_t bar = kv.first.find('|');
        std::fprintf(f, "%s\n    {\"arch\": \"%s\", \"key\": \"%s\", \"choice\": %d, \"ms\": [",
                     first ? "" : ",", kv.first.substr(0, bar).c_str(),
                     kv.first.substr(bar + 1).c_str(), kv.second.choice);
        for (size_t i = 0; i < kv.second.ms.size(); ++i)
            std::fprintf(f, "%s%.17g", i ? ", " : "", kv.second.ms[i]);
        std::fprintf(f, "]}");
        first = false;
    }
    std::fprintf(f, "\n  ]\n}\n");
    const bool good = std::fclose(f) == 0;
    if (!good || std::rename(tmp.c_str(), path) != 0) {
        if (err) *err = std::string("cannot replace ") + path;
        return false;
    }
    return true;
}

void env_load_locked() {
    if (g_env_loaded) return;
    g_env_loaded = true;
    const char *path = std::getenv("CDL_AUTOTUNE_CACHE");
    if (path && *path) (void)load_locked(path, nullptr);
}

}  // namespace

std::string tune_arch(int device) {
    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_arch.find(device);
    if (it != g_arch.end()) return it->second;
    std::string a = "none";
    hipDeviceProp_t prop;
    if (device >= 0 && hipGetDeviceProperties(&prop, device) == hipSuccess) a = prop.gcnArchName;
    g_arch[device] = a;
    return a;
}

std::string tune_key(const char *family, int prec, int64_t ld, int64_t kpad) {
    char buf[96];
    if (kpad > 0)
        std::snprintf(buf, sizeof(buf), "%s/%s/ld%lld/k%lld", family, prec_name(prec),
                      (long long)ld, (long long)kpad);
    else
        std::snprintf(buf, sizeof(buf), "%s/%s/ld%lld", family, prec_name(prec), (long long)ld);
    return buf;
}

bool tune_get(const std::string &arch, const std::string &key, int *choice, double *ms,
              int *ncand) {
    std::lock_guard<std::mutex> lock(g_mu);
    env_load_locked();
    auto it = g_table.find(arch + "|" + key);
    if (it == g_table.end()) return false;
    if (choice) *choice = it->second.choice;
    if (ms) *ms = it->second.ms[it->second.choice];
    if (ncand) *ncand = (int)it->second.ms.size();
    return true;
}

int tune_put(const std::string &arch, const std::string &key, const std::vector<double> &ms) {
    int best = 0;
    for (size_t i = 1; i < ms.size(); ++i)
        if (ms[i] > 0.0 && (ms[best] <= 0.0 || ms[i] < ms[best])) best = (int)i;
    std::lock_guard<std::mutex> lock(g_mu);
    env_load_locked();
    TuneEntry t;
    t.choice = best;
    t.ms = ms;
    g_table[arch + "|" + key] = t;
    const char *path = std::getenv("CDL_AUTOTUNE_CACHE");
    if (path && *path) (void)save_locked(path, nullptr);
    return best;
}

bool tune_load(const char *path, std::string *err) {
    std::lock_guard<std::mutex> lock(g_mu);
    return load_locked(path, err);
}

bool tune_save(const char *path, std::string *err) {
    std::lock_guard<std::mutex> lock(g_mu);
    return save_locked(path, err);
}

void tune_clear() {
    std::lock_guard<std::mutex> lock(g_mu);
    g_table.clear();
    g_env_loaded = true;   // an explicit clear also forgets the environment's file
}

int tune_entries() {
    std::lock_guard<std::mutex> lock(g_mu);
    return (int)g_table.size();
}

}  // namespace cdl
