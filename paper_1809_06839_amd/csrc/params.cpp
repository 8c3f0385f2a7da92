// params.cpp -- host-side parameter compile (per-sample records -> integer
// records the kernels consume).  Transcendental functions run here, once per
// image in IEEE double, so every kernel is integer-only and reproducible.
#include <math.h>

#include "internal.h"

using miaug::set_error;

extern "C" int miaug_compile_c2(const float *f, const int32_t *k, int n, int H, int W, int crop,
                                miaug_c2_record *out) {
    if (n < 0 || (n > 0 && (!f || !k || !out))) return set_error(MIAUG_EINVAL, "compile_c2: bad arguments");
    if (H < 1 || W < 1 || crop < 1 || crop > H || crop > W)
        return set_error(MIAUG_ESHAPE, "compile_c2: H=%d W=%d crop=%d", H, W, crop);
    const double deg = 3.14159265358979323846 / 180.0;
    for (int i = 0; i < n; ++i) {
        const float *fi = f + 5 * i;
        const int32_t *ki = k + 5 * i;
        if (!(fi[1] != 0.0f)) return set_error(MIAUG_ESHAPE, "compile_c2: scale of image %d is 0", i);
        miaug_c2_record &r = out[i];
        // inverse of p' = s R (p - c) + c + t, t = (dx W, dy H)
        const double th = (double)fi[0] * deg, s = (double)fi[1];
        const double c = cos(th), sn = sin(th);
        const double cx = (W - 1) / 2.0, cy = (H - 1) / 2.0;
        const double ux = cx + (double)fi[2] * W, uy = cy + (double)fi[3] * H;
        double m[6];
        m[0] = c / s;
        m[1] = -sn / s;
        m[3] = sn / s;
        m[4] = c / s;
        m[2] = cx - m[0] * ux - m[1] * uy;
        m[5] = cy - m[3] * ux - m[4] * uy;
        for (int j = 0; j < 6; ++j) r.aq[j] = (int64_t)llrint(m[j] * 4294967296.0);
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
