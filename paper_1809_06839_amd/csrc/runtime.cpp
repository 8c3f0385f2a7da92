// runtime.cpp -- host runtime of libmiaug: configuration from the environment,
// logging, device and pinned allocations (with an injectable failure for
// tests of the error paths), and the persisted autotuner cache.
//
// Environment (read once per process):
//   MIAUG_LOG=n               0 quiet (default), 1 errors, 2 tuner decisions and
//                             allocations, 3 every launch; messages go to stderr
//   MIAUG_FORCE_VARIANT=v     ragged launch variant used by every context,
//                             whatever the autotuner or miaug_ragged_set_variant chose
//   MIAUG_TUNE_CACHE=path     autotuner cache file of contexts created without one
//   MIAUG_FAIL_ALLOC_AFTER=k  the library's allocation number k + 1 (counted from
//                             0 across the process) fails with MIAUG_ENOMEM, once
//
// Tune cache: a JSON file {"version": 1, "entries": [{"key": ..., "variant": v,
// "name": ..., "ms": t}, ...]}.  A key names the GPU architecture, the chain and
// a bucket of the batch shape; an entry is used only while the variant table
// still has a variant of the stored name at the stored index.  Writes go to a
// temporary file renamed over the cache, so readers never see a partial file.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace miaug {
namespace {

EnvConfig g_env;
std::once_flag g_env_once;
std::atomic<long> g_alloc_count{0};
std::atomic<long> g_fail_at{-1};

long env_long(const char *name, long dflt) {
    const char *v = getenv(name);
    if (!v || !*v) return dflt;
    char *end = nullptr;
    const long x = strtol(v, &end, 10);
    return (end && *end == 0) ? x : dflt;
}

void load_env() {
    g_env.log_level = (int)env_long("MIAUG_LOG", 0);
    g_env.force_variant = (int)env_long("MIAUG_FORCE_VARIANT", -1);
    const char *tc = getenv("MIAUG_TUNE_CACHE");
    g_env.tune_cache = tc ? tc : "";
    g_env.fail_alloc_after = env_long("MIAUG_FAIL_ALLOC_AFTER", -1);
    g_fail_at.store(g_env.fail_alloc_after);
}

// Allocation number n (0-based) fails when it is the armed one; the injector
// then disarms itself.
bool injected_failure() {
    const long n = g_alloc_count.fetch_add(1);
    long armed = g_fail_at.load();
    return armed >= 0 && n == armed && g_fail_at.compare_exchange_strong(armed, -1);
}

// ---- a small JSON reader for the cache file's schema
struct Json {
    const char *p, *e;
    bool ok = true;
    int depth = 0;  // nesting of skipped values (bounded, so a hostile file cannot exhaust the stack)
    void ws() {
        while (p < e && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
    }
    bool lit(char c) {
        ws();
        if (p < e && *p == c) {
            ++p;
            return true;
        }
        return false;
    }
    bool str(std::string &out) {
        out.clear();
        if (!lit('"')) return ok = false;
        while (p < e && *p != '"') {
            char c = *p++;
            if (c == '\\') {
                if (p >= e) return ok = false;
                c = *p++;
                if (c == 'n') c = '\n';
                else if (c == 't') c = '\t';
                else if (c != '"' && c != '\\' && c != '/') return ok = false;
            }
            out.push_back(c);
        }
        if (p >= e) return ok = false;
        ++p;
        return true;
    }
    bool num(double &out) {
        ws();
        char buf[64];
        size_t n = 0;
        while (p < e && n + 1 < sizeof(buf) && (strchr("+-.eE", *p) || (*p >= '0' && *p <= '9'))) buf[n++] = *p++;
        buf[n] = 0;
        if (n == 0) return ok = false;
        char *end = nullptr;
        out = strtod(buf, &end);
        return ok = (end == buf + n);
    }
    // Skips any value (used for unknown fields).
    bool skip() {
        ws();
        if (p >= e) return ok = false;
        if (*p == '"') {
            std::string s;
            return str(s);
        }
        if (*p == '{' || *p == '[') {
            if (++depth > 32) return ok = false;
            const char open = *p, close = open == '{' ? '}' : ']';
            ++p;
            bool done = lit(close);
            while (!done) {
                if (open == '{') {
                    std::string k;
                    if (!str(k) || !lit(':')) return ok = false;
                }
                if (!skip()) return false;
                if (lit(',')) continue;
                if (!lit(close)) return ok = false;
                done = true;
            }
            --depth;
            return true;
        }
        double d;
        if (*p == 't' || *p == 'f' || *p == 'n') {
            while (p < e && *p >= 'a' && *p <= 'z') ++p;
            return true;
        }
        return num(d);
    }
};

bool parse_cache(const std::string &text, std::vector<TuneEntry> &out) {
    Json j{text.data(), text.data() + text.size()};
    if (!j.lit('{')) return false;
    if (j.lit('}')) return true;
    for (;;) {
        std::string k;
        if (!j.str(k) || !j.lit(':')) return false;
        if (k == "entries") {
            if (!j.lit('[')) return false;
            if (!j.lit(']')) {
                for (;;) {
                    TuneEntry t;
                    bool have_key = false, have_var = false;
                    if (!j.lit('{')) return false;
                    if (!j.lit('}')) {
                        for (;;) {
                            std::string f;
                            if (!j.str(f) || !j.lit(':')) return false;
                            double d = 0;
                            if (f == "key") {
                                if (!j.str(t.key)) return false;
                                have_key = true;
                            } else if (f == "name") {
                                if (!j.str(t.name)) return false;
                            } else if (f == "variant") {
                                if (!j.num(d) || d < 0 || d > 1e6) return false;
                                t.variant = (int)d;
                                have_var = true;
                            } else if (f == "ms") {
                                if (!j.num(d)) return false;
                                t.ms = (float)d;
                            } else if (!j.skip()) {
                                return false;
                            }
                            if (j.lit(',')) continue;
                            if (!j.lit('}')) return false;
                            break;
                        }
                    }
                    if (have_key && have_var) out.push_back(t);
                    if (j.lit(',')) continue;
                    if (!j.lit(']')) return false;
                    break;
                }
            }
        } else if (!j.skip()) {
            return false;
        }
        if (j.lit(',')) continue;
        return j.lit('}');
    }
}

void put_escaped(std::string &o, const std::string &s) {
    o.push_back('"');
    for (char c : s) {
        if (c == '"' || c == '\\') o.push_back('\\');
        if (c == '\n') {
            o += "\\n";
            continue;
        }
        if (c == '\t') {
            o += "\\t";
            continue;
        }
        o.push_back(c);
    }
    o.push_back('"');
}

std::mutex g_cache_mu;  // one writer at a time within the process

}  // namespace

const EnvConfig &env() {
    std::call_once(g_env_once, load_env);
    return g_env;
}

void log_msg(int level, const char *fmt, ...) {
    if (env().log_level < level) return;
    va_list ap;
    va_start(ap, fmt);
    fputs("[miaug] ", stderr);
    vfprintf(stderr, fmt, ap);
    fputc('\n', stderr);
    va_end(ap);
}

void arm_alloc_failure(long after) {
    env();
    g_alloc_count.store(0);
    g_fail_at.store(after);
}

int dev_alloc(void **p, size_t bytes, const char *what) {
    env();
    *p = nullptr;
    if (injected_failure()) {
        log_msg(2, "%s: %zu bytes: injected allocation failure", what, bytes);
        return set_error(MIAUG_ENOMEM, "%s: out of device memory (injected failure)", what);
    }
    const int st = hip_status(hipMalloc(p, bytes), what);
    log_msg(2, "%s: hipMalloc %zu bytes -> %s", what, bytes, st ? "failed" : "ok");
    return st;
}

int pinned_alloc(void **p, size_t bytes, const char *what) {
    env();
    *p = nullptr;
    if (injected_failure()) {
        log_msg(2, "%s: %zu bytes: injected allocation failure", what, bytes);
        return set_error(MIAUG_ENOMEM, "%s: out of pinned host memory (injected failure)", what);
    }
    const int st = hip_status(hipHostMalloc(p, bytes, hipHostMallocDefault), what);
    log_msg(2, "%s: hipHostMalloc %zu bytes -> %s", what, bytes, st ? "failed" : "ok");
    return st;
}

int tune_cache_read(const std::string &path, std::vector<TuneEntry> &out) {
    out.clear();
    FILE *f = fopen(path.c_str(), "rb");
    if (!f) return MIAUG_OK;  // no cache yet
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof(buf), f)) > 0) {
        text.append(buf, n);
        if (text.size() > (64u << 20)) break;
    }
    fclose(f);
    if (!parse_cache(text, out)) {
        out.clear();
        log_msg(1, "tune cache %s: not a cache file, ignored", path.c_str());
        return set_error(MIAUG_EINVAL, "tune cache %s: malformed", path.c_str());
    }
    return MIAUG_OK;
}

int tune_cache_get(const std::string &path, const std::string &key, TuneEntry *hit) {
    std::lock_guard<std::mutex> g(g_cache_mu);
    std::vector<TuneEntry> es;
    if (int st = tune_cache_read(path, es)) return st;
    for (const TuneEntry &t : es)
        if (t.key == key) {
            *hit = t;
            return MIAUG_OK;
        }
    return MIAUG_EUNSUPPORTED;  // not found
}

int tune_cache_put(const std::string &path, const TuneEntry &e) {
    std::lock_guard<std::mutex> g(g_cache_mu);
    std::vector<TuneEntry> es;
    tune_cache_read(path, es);  // a malformed file is replaced
    bool found = false;
    for (TuneEntry &t : es)
        if (t.key == e.key) {
            t = e;
            found = true;
        }
    if (!found) es.push_back(e);
    std::string o = "{\n  \"version\": 1,\n  \"entries\": [";
    for (size_t i = 0; i < es.size(); ++i) {
        o += i ? ",\n    {\"key\": " : "\n    {\"key\": ";
        put_escaped(o, es[i].key);
        char num[96];
        snprintf(num, sizeof(num), ", \"variant\": %d, \"ms\": %.6g, \"name\": ", es[i].variant, (double)es[i].ms);
        o += num;
        put_escaped(o, es[i].name);
        o += "}";
    }
    o += "\n  ]\n}\n";
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return set_error(MIAUG_EINVAL, "tune cache %s: cannot write %s", path.c_str(), tmp.c_str());
    const bool wrote = fwrite(o.data(), 1, o.size(), f) == o.size();
    const bool closed = fclose(f) == 0;
    if (!wrote || !closed || rename(tmp.c_str(), path.c_str()) != 0) {
        remove(tmp.c_str());
        return set_error(MIAUG_EINVAL, "tune cache %s: write failed", path.c_str());
    }
    log_msg(2, "tune cache %s: stored %s -> variant %d (%s), %.4f ms", path.c_str(), e.key.c_str(), e.variant,
         e.name.c_str(), (double)e.ms);
    return MIAUG_OK;
}

}  // namespace miaug
