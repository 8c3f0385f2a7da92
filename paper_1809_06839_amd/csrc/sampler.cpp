// sampler.cpp -- per-sample transform parameters from a counter-based
// generator (Philox4x64-10 of Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11).  The paper only implies randomness
// ("random transformation from the dihedral group", "random sized crop",
// Sec. II-A/II-B); the draw layout below is this library's definition.
//
// Draw d of global sample g: word 0 of Philox(counter {d, g, 0, stream},
// key {seed, 0}).  Host-side: per-sample records are tiny and are consumed
// by the kernels as device arrays supplied by the caller.
#include <math.h>
#include <stdint.h>

#include "internal.h"

namespace miaug {
namespace {

struct U128 {
    uint64_t hi, lo;
};

inline U128 mul64(uint64_t a, uint64_t b) {
    unsigned __int128 p = (unsigned __int128)a * b;
    return {(uint64_t)(p >> 64), (uint64_t)p};
}

// Philox4x64 with 10 rounds: each round multiplies words 0 and 2 by the two
// round constants, swaps the halves across lanes and mixes in the key; the key
// advances by the two Weyl constants between rounds.
void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    for (int r = 0; r < 10; ++r) {
        U128 p0 = mul64(M0, c[0]), p1 = mul64(M1, c[2]);
        uint64_t o0 = p1.hi ^ c[1] ^ k0, o2 = p0.hi ^ c[3] ^ k1;
        c[0] = o0; c[1] = p1.lo; c[2] = o2; c[3] = p0.lo;
        k0 += W0; k1 += W1;
    }
}

class Draws {
  public:
    Draws(uint64_t seed, uint64_t g) : seed_(seed), g_(g) {}
    uint64_t word(uint64_t d) const {
        uint64_t c[4] = {d, g_, 0, 0};
        philox4x64_10(c, seed_, 0);
        return c[0];
    }
    double uniform(uint64_t d) const { return (double)(word(d) >> 11) * 0x1.0p-53; }
    int32_t bern(uint64_t d, double p) const { return uniform(d) < p ? 1 : 0; }
    int32_t below(uint64_t d, uint32_t m) const { return (int32_t)(((word(d) >> 32) * (uint64_t)m) >> 32); }
    float range(uint64_t d, double lo, double hi) const { return (float)(lo + (hi - lo) * uniform(d)); }

  private:
    uint64_t seed_, g_;
};

}  // namespace
}  // namespace miaug

using miaug::Draws;
using miaug::set_error;

extern "C" int miaug_sample_d4bc(uint64_t seed, uint64_t first_index, int n, int32_t *flags, float *ab) {
    if (n < 0 || (n > 0 && (!flags || !ab))) return set_error(MIAUG_EINVAL, "sample_d4bc: bad arguments");
    for (int i = 0; i < n; ++i) {
        Draws D(seed, first_index + (uint64_t)i);
        flags[4 * i + 0] = D.bern(0, 0.5);
        flags[4 * i + 1] = D.bern(1, 0.5);
        flags[4 * i + 2] = D.below(2, 4);
        flags[4 * i + 3] = D.bern(3, 0.5);
        ab[2 * i + 0] = D.range(4, 0.8, 1.2);
        ab[2 * i + 1] = D.range(5, -51.0, 51.0);
    }
    return MIAUG_OK;
}

extern "C" int miaug_sample_c2(uint64_t seed, uint64_t first_index, int n, int crop_range, float *f, int32_t *k) {
    if (n < 0 || crop_range < 0 || (n > 0 && (!f || !k))) return set_error(MIAUG_EINVAL, "sample_c2: bad arguments");
    for (int i = 0; i < n; ++i) {
        Draws D(seed, first_index + (uint64_t)i);
        float *fi = f + 5 * i;
        int32_t *ki = k + 5 * i;
        fi[0] = D.range(0, -45.0, 45.0);
        fi[1] = D.range(1, 0.9, 1.1);
        fi[2] = D.range(2, -0.0625, 0.0625);
        fi[3] = D.range(3, -0.0625, 0.0625);
        ki[0] = D.below(4, (uint32_t)crop_range + 1);
        ki[1] = D.below(5, (uint32_t)crop_range + 1);
        ki[2] = (int32_t)rint((double)D.range(6, -20.0, 20.0));
        ki[3] = (int32_t)rint((double)D.range(7, -30.0, 30.0));
        fi[4] = D.range(8, 0.8, 1.2);
        ki[4] = D.bern(9, 0.3);
    }
    return MIAUG_OK;
}

extern "C" int miaug_sample_wc(uint64_t seed, uint64_t first_index, int n, float *f) {
    if (n < 0 || (n > 0 && !f)) return set_error(MIAUG_EINVAL, "sample_wc: bad arguments");
    static const double lo[7] = {-45.0, 0.9, -0.0625, -0.0625, 0.8, -0.2, 0.8};
    static const double hi[7] = {45.0, 1.1, 0.0625, 0.0625, 1.2, 0.2, 1.2};
    for (int i = 0; i < n; ++i) {
        Draws D(seed, first_index + (uint64_t)i);
        for (int j = 0; j < 7; ++j) f[7 * i + j] = D.range((uint64_t)j, lo[j], hi[j]);
    }
    return MIAUG_OK;
}

extern "C" int miaug_sample_grid(uint64_t seed, uint64_t first_index, int n, double limit, double *f) {
    if (n < 0 || !(limit >= 0.0 && limit < 1.0) || (n > 0 && !f))
        return set_error(MIAUG_EINVAL, "sample_grid: bad arguments");
    for (int i = 0; i < n; ++i) {
        Draws D(seed, first_index + (uint64_t)i);
        for (int j = 0; j < 10; ++j) f[10 * i + j] = 1.0 + (double)D.range((uint64_t)j, -limit, limit);
    }
    return MIAUG_OK;
}
