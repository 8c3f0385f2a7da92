// params.cpp -- host-side parameter compile (per-sample records -> integer
// records the kernels consume).  Transcendental functions run here, once per
// image in IEEE double, so every kernel is integer-only and reproducible.
#include <cmath>
#include <math.h>

#include "internal.h"

using miaug::set_error;

namespace {

// Q32 inverse of the shift-scale-rotate map p' = s R (p - c) + c + t,
// t = (dx W, dy H), c the image centre; f = {angle_deg, scale, dx, dy}.
void ssr_q32(const float *f, int H, int W, int64_t *aq) {
    const double deg = 3.14159265358979323846 / 180.0;
    const double th = (double)f[0] * deg, s = (double)f[1];
    const double c = cos(th), sn = sin(th);
    const double cx = (W - 1) / 2.0, cy = (H - 1) / 2.0;
    const double ux = cx + (double)f[2] * W, uy = cy + (double)f[3] * H;
    double m[6];
    m[0] = c / s;
    m[1] = -sn / s;
    m[3] = sn / s;
    m[4] = c / s;
    m[2] = cx - m[0] * ux - m[1] * uy;
    m[5] = cy - m[3] * ux - m[4] * uy;
    for (int j = 0; j < 6; ++j) aq[j] = (int64_t)llrint(m[j] * 4294967296.0);
}

}  // namespace

extern "C" int miaug_compile_ssr_q32(const float *f, int n, int H, int W, int64_t *aq) {
    if (n < 0 || (n > 0 && (!f || !aq))) return set_error(MIAUG_EINVAL, "compile_ssr_q32: bad arguments");
    if (H < 1 || W < 1) return set_error(MIAUG_ESHAPE, "compile_ssr_q32: H=%d W=%d", H, W);
    for (int i = 0; i < n; ++i) {
        if (!(f[4 * i + 1] != 0.0f)) return set_error(MIAUG_ESHAPE, "compile_ssr_q32: scale of image %d is 0", i);
        ssr_q32(f + 4 * i, H, W, aq + 6 * i);
    }
    return MIAUG_OK;
}

extern "C" int miaug_compile_color_luts(const float *ab, const float *shift, int n, int C, uint8_t *luts) {
    if (n < 0 || (n > 0 && !luts) || C < 1 || C > 4) return set_error(MIAUG_EINVAL, "compile_color_luts: bad arguments");
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < C; ++c)
            for (int v = 0; v < 256; ++v) {
                // brightness/contrast, then the channel shift, each rounded and saturated to u8
                int u = v;
                if (ab) {
                    const double t = rint((double)ab[2 * i] * (double)v + (double)ab[2 * i + 1]);
                    u = t < 0 ? 0 : (t > 255 ? 255 : (int)t);
                }
                if (shift) {
                    const double t = rint((double)u + (double)shift[C * i + c]);
                    u = t < 0 ? 0 : (t > 255 ? 255 : (int)t);
                }
                luts[((size_t)i * C + c) * 256 + v] = (uint8_t)u;
            }
    return MIAUG_OK;
}

extern "C" int miaug_compile_gamma_luts(const float *gamma, int n, int C, uint8_t *luts) {
    if (n < 0 || (n > 0 && (!gamma || !luts)) || C < 1 || C > 4)
        return set_error(MIAUG_EINVAL, "compile_gamma_luts: bad arguments");
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(gamma[i])) return set_error(MIAUG_EINVAL, "compile_gamma_luts: gamma %d not finite", i);
        const double g = (double)gamma[i];
        for (int v = 0; v < 256; ++v) {
            // the same LUT as the u8 chain's gamma step
            const double e = rint(255.0 * pow(v / 255.0, g));
            const uint8_t u = (uint8_t)(e < 0 ? 0 : (e > 255 ? 255 : e));
            for (int c = 0; c < C; ++c) luts[((size_t)i * C + c) * 256 + v] = u;
        }
    }
    return MIAUG_OK;
}

extern "C" int miaug_compile_c2(const float *f, const int32_t *k, int n, int H, int W, int crop,
                                miaug_c2_record *out) {
    if (n < 0 || (n > 0 && (!f || !k || !out))) return set_error(MIAUG_EINVAL, "compile_c2: bad arguments");
    if (H < 1 || W < 1 || crop < 1 || crop > H || crop > W)
        return set_error(MIAUG_ESHAPE, "compile_c2: H=%d W=%d crop=%d", H, W, crop);
    for (int i = 0; i < n; ++i) {
        const float *fi = f + 5 * i;
        const int32_t *ki = k + 5 * i;
        if (!(fi[1] != 0.0f)) return set_error(MIAUG_ESHAPE, "compile_c2: scale of image %d is 0", i);
        miaug_c2_record &r = out[i];
        ssr_q32(fi, H, W, r.aq);
        r.crop_x = ki[0] < 0 ? 0 : (ki[0] > W - crop ? W - crop : ki[0]);
        r.crop_y = ki[1] < 0 ? 0 : (ki[1] > H - crop ? H - crop : ki[1]);
        r.dh = ki[2];
        r.ds = ki[3];
        r.dv = 0;
        r.blur = ki[4] ? 1 : 0;
        const double g = (double)fi[4];
        for (int v = 0; v < 256; ++v) {
            const double e = rint(255.0 * pow(v / 255.0, g));
            r.gamma_lut[v] = (uint8_t)(e < 0 ? 0 : (e > 255 ? 255 : e));
        }
    }
    return MIAUG_OK;
}
