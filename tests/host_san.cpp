// Host-code driver for the AddressSanitizer / UndefinedBehaviorSanitizer run
// of the library's host sources (sampler, parameter compile, tune cache,
// error reporting), built with g++ by tests/test_sanitizers.py.  It calls
// every host entry point over ordinary and edge-case arguments and feeds the
// tune-cache reader truncated, corrupted and hostile files; any memory or
// undefined-behaviour error aborts the run with the sanitizer's report.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <random>
#include <string>
#include <vector>

#include "../paper_1809_06839_amd/csrc/internal.h"

#define CHECK(c)                                                      \
    do {                                                              \
        if (!(c)) {                                                   \
            fprintf(stderr, "check failed at %d: %s\n", __LINE__, #c); \
            return 1;                                                 \
        }                                                             \
    } while (0)

static int samplers() {
    for (int n : {0, 1, 7, 1000}) {
        std::vector<int32_t> flags(4 * (size_t)n + 1), k(5 * (size_t)n + 1);
        std::vector<float> ab(2 * (size_t)n + 1), f(8 * (size_t)n + 1);
        std::vector<double> g(10 * (size_t)n + 1);
        CHECK(miaug_sample_d4bc(7, 3, n, flags.data(), ab.data()) == MIAUG_OK);
        CHECK(miaug_sample_c2(7, 3, n, 64, f.data(), k.data()) == MIAUG_OK);
        CHECK(miaug_sample_wc(7, 3, n, f.data()) == MIAUG_OK);
        CHECK(miaug_sample_grid(7, 3, n, 0.3, g.data()) == MIAUG_OK);
    }
    CHECK(miaug_sample_d4bc(7, 3, -1, nullptr, nullptr) == MIAUG_EINVAL);
    CHECK(miaug_sample_c2(7, 3, 2, -1, nullptr, nullptr) == MIAUG_EINVAL);
    CHECK(miaug_sample_grid(7, 3, 1, 2.0, nullptr) == MIAUG_EINVAL);
    CHECK(strlen(miaug_last_error()) > 0);
    return 0;
}

static int compiles() {
    const int n = 64;
    std::vector<float> f(5 * n);
    std::vector<int32_t> k(5 * n);
    CHECK(miaug_sample_c2(11, 0, n, 64, f.data(), k.data()) == MIAUG_OK);
    std::vector<miaug_c2_record> rec(n);
    for (int hw : {1, 2, 448, 512, 4097}) {
        const int st = miaug_compile_c2(f.data(), k.data(), n, hw, hw, hw < 448 ? hw : 448, rec.data());
        CHECK(st == MIAUG_OK || st == MIAUG_ESHAPE);
    }
    std::vector<float> ssr(4 * n);
    for (int i = 0; i < n; ++i) {
        ssr[4 * i] = f[5 * i];
        ssr[4 * i + 1] = f[5 * i + 1];
        ssr[4 * i + 2] = f[5 * i + 2];
        ssr[4 * i + 3] = f[5 * i + 3];
    }
    std::vector<int64_t> aq(6 * n);
    CHECK(miaug_compile_ssr_q32(ssr.data(), n, 512, 512, aq.data()) == MIAUG_OK);
    ssr[1] = 0.f;
    CHECK(miaug_compile_ssr_q32(ssr.data(), n, 512, 512, aq.data()) == MIAUG_ESHAPE);
    std::vector<float> ab(2 * n), shift(4 * n);
    for (int i = 0; i < 2 * n; ++i) ab[i] = i % 2 ? -60.f + i : 0.5f + 0.01f * i;
    for (int i = 0; i < 4 * n; ++i) shift[i] = -300.f + 7.f * i;
    for (int C = 1; C <= 4; ++C) {
        std::vector<uint8_t> luts((size_t)n * C * 256);
        CHECK(miaug_compile_color_luts(ab.data(), shift.data(), n, C, luts.data()) == MIAUG_OK);
        CHECK(miaug_compile_color_luts(nullptr, nullptr, n, C, luts.data()) == MIAUG_OK);
    }
    std::vector<float> gam(n);
    for (int i = 0; i < n; ++i) gam[i] = 0.05f + 0.1f * i;
    std::vector<uint8_t> gl((size_t)n * 3 * 256);
    CHECK(miaug_compile_gamma_luts(gam.data(), n, 3, gl.data()) == MIAUG_OK);
    return 0;
}

static int tune_cache(const std::string &dir) {
    using miaug::TuneEntry;
    const std::string path = dir + "/tune.json";
    remove(path.c_str());
    TuneEntry e, hit;
    CHECK(miaug::tune_cache_get(path, "absent", &hit) == MIAUG_EUNSUPPORTED);
    for (int i = 0; i < 50; ++i) {
        e.key = "key \"" + std::to_string(i) + "\" \\ end";
        e.name = std::string(i, 'x') + "\t\n";
        e.variant = i;
        e.ms = 0.5f * i;
        CHECK(miaug::tune_cache_put(path, e) == MIAUG_OK);
    }
    CHECK(miaug::tune_cache_get(path, "key \"17\" \\ end", &hit) == MIAUG_OK && hit.variant == 17);
    CHECK(hit.name == std::string(17, 'x') + "\t\n");
    // every truncation of a valid file, and bytes flipped at random, must be
    // rejected or read without touching memory outside the text
    FILE *f = fopen(path.c_str(), "rb");
    CHECK(f);
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    fclose(f);
    const std::string bad = dir + "/bad.json";
    std::mt19937 rng(5);
    for (size_t cut = 0; cut < text.size(); cut += 7) {
        std::string t = text.substr(0, cut);
        if (cut % 3 == 0 && !t.empty()) t[rng() % t.size()] = (char)(rng() & 255);
        FILE *w = fopen(bad.c_str(), "wb");
        fwrite(t.data(), 1, t.size(), w);
        fclose(w);
        std::vector<TuneEntry> es;
        const int st = miaug::tune_cache_read(bad, es);
        CHECK(st == MIAUG_OK || st == MIAUG_EINVAL);
    }
    const std::string hostile[] = {std::string(100000, '['), "{\"entries\": [" + std::string(5000, '{'),
                                   "{\"x\": \"\\", "{\"entries\": [{\"key\": \"k\", \"variant\": 1e308}]}",
                                   std::string("{\"a\"") + std::string(3, '\0') + "}"};
    for (const std::string &t : hostile) {
        FILE *w = fopen(bad.c_str(), "wb");
        fwrite(t.data(), 1, t.size(), w);
        fclose(w);
        std::vector<TuneEntry> es;
        CHECK(miaug::tune_cache_read(bad, es) == MIAUG_EINVAL);
    }
    return 0;
}

int main(int argc, char **argv) {
    if (argc < 2) return 2;
    if (samplers() || compiles() || tune_cache(argv[1])) return 1;
    printf("host sanitizer run: ok\n");
    return 0;
}
