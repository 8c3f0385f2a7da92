// pipeline.cpp -- op-list pipelines: a list of transforms with probabilities
// and parameter ranges (the way the paper composes augmentations, Sec. I and
// Sec. II) is matched, in order, against the fused chains of this library and
// executed by their kernels.  Host code only: sampling, parameter packing,
// device buffers, graphs.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <new>
#include <vector>

#include "internal.h"

namespace miaug {
namespace {

// Philox4x64-10 draws of the sampler section (same generator as sampler.cpp,
// restated here so this file has no dependence on that one's internals).
struct U128 {
    uint64_t hi, lo;
};
inline U128 mul64(uint64_t a, uint64_t b) {
    unsigned __int128 p = (unsigned __int128)a * b;
    return {(uint64_t)(p >> 64), (uint64_t)p};
}
// All four words of the block with counter {d, g, 0, 0} and key {seed, 0}.
void philox_block(uint64_t d, uint64_t g, uint64_t seed, uint64_t (&c)[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    c[0] = d; c[1] = g; c[2] = 0; c[3] = 0;
    uint64_t k0 = seed, k1 = 0;
    for (int r = 0; r < 10; ++r) {
        U128 p0 = mul64(M0, c[0]), p1 = mul64(M1, c[2]);
        uint64_t o0 = p1.hi ^ c[1] ^ k0, o2 = p0.hi ^ c[3] ^ k1;
        c[0] = o0; c[1] = p1.lo; c[2] = o2; c[3] = p0.lo;
        k0 += W0; k1 += W1;
    }
}
uint64_t philox_word0(uint64_t d, uint64_t g, uint64_t seed) {
    uint64_t c[4];
    philox_block(d, g, seed, c);
    return c[0];
}
double unit_of(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }
int below_of(uint64_t w, uint32_t m) { return (int)(((w >> 32) * (uint64_t)m) >> 32); }

// Random-sized crop window {y0, x0, h, w} of an H x W image: up to 10 tries,
// try t reading the four words of block d + t (area fraction, log aspect
// ratio, row offset, column offset); the first window that fits wins, else a
// centred window with the aspect ratio clamped into [rlo, rhi].
void sized_crop(uint64_t seed, uint64_t g, uint64_t d, int H, int W, double slo, double shi, double rlo,
                double rhi, int32_t (&win)[4]) {
    const double llo = log(rlo), lhi = log(rhi);
    for (int t = 0; t < 10; ++t) {
        uint64_t c[4];
        philox_block(d + (uint64_t)t, g, seed, c);
        const double s = slo + (shi - slo) * unit_of(c[0]);
        const double r = exp(llo + (lhi - llo) * unit_of(c[1]));
        const double area = (double)H * (double)W * s;
        const double wf = floor(sqrt(area * r) + 0.5), hf = floor(sqrt(area / r) + 0.5);
        if (wf >= 1.0 && wf <= (double)W && hf >= 1.0 && hf <= (double)H) {
            const int w = (int)wf, h = (int)hf;
            win[0] = below_of(c[2], (uint32_t)(H - h + 1));
            win[1] = below_of(c[3], (uint32_t)(W - w + 1));
            win[2] = h;
            win[3] = w;
            return;
        }
    }
    int h = H, w = W;
    const double in_r = (double)W / (double)H;
    if (in_r < rlo) {
        h = (int)floor((double)W / rlo + 0.5);
        h = h < 1 ? 1 : h;
    } else if (in_r > rhi) {
        w = (int)floor((double)H * rhi + 0.5);
        w = w < 1 ? 1 : w;
    }
    win[0] = (H - h) / 2;
    win[1] = (W - w) / 2;
    win[2] = h;
    win[3] = w;
}
struct Gen {
    uint64_t seed, g;
    double uniform(uint64_t d) const { return (double)(philox_word0(d, g, seed) >> 11) * 0x1.0p-53; }
    bool bern(uint64_t d, double p) const { return uniform(d) < p; }
    int below(uint64_t d, uint32_t m) const { return (int)(((philox_word0(d, g, seed) >> 32) * (uint64_t)m) >> 32); }
    float range(uint64_t d, double lo, double hi) const { return (float)(lo + (hi - lo) * uniform(d)); }
};

const char *op_name(uint32_t k) {
    static const char *names[] = {"?", "HFLIP", "VFLIP", "ROT90", "TRANSPOSE", "SSR", "CROP", "RESIZE",
                                  "BRIGHT_CONTRAST", "HSV", "GAMMA", "BLUR3", "BLUR5", "ELASTIC", "GRID",
                                  "NORMALIZE", "SIZED_CROP", "SHIFT_RGB", "TO_GRAY", "PAD", "ROTATE"};
    return k < sizeof(names) / sizeof(names[0]) ? names[k] : "?";
}

// Allowed op sequences per chain (each op at most once, in this order).
const uint32_t kSeqDih4[] = {MIAUG_OP_HFLIP,           MIAUG_OP_VFLIP,     MIAUG_OP_ROT90, MIAUG_OP_TRANSPOSE,
                             MIAUG_OP_BRIGHT_CONTRAST, MIAUG_OP_SHIFT_RGB, MIAUG_OP_GAMMA, MIAUG_OP_TO_GRAY};
const uint32_t kSeqRagged[] = {MIAUG_OP_HFLIP,      MIAUG_OP_VFLIP,           MIAUG_OP_ROT90,
                               MIAUG_OP_TRANSPOSE,  MIAUG_OP_SIZED_CROP,      MIAUG_OP_BRIGHT_CONTRAST,
                               MIAUG_OP_RESIZE,     MIAUG_OP_NORMALIZE};
const uint32_t kSeqU8[] = {MIAUG_OP_SSR, MIAUG_OP_CROP, MIAUG_OP_RESIZE, MIAUG_OP_HSV, MIAUG_OP_GAMMA, MIAUG_OP_BLUR3};
const uint32_t kSeqDistort[] = {MIAUG_OP_ELASTIC, MIAUG_OP_GRID};
const uint32_t kSeqRotate[] = {MIAUG_OP_ROTATE};
const uint32_t kSeqSsr[] = {MIAUG_OP_SSR};
const uint32_t kSeqPad[] = {MIAUG_OP_PAD};
const uint32_t kSeqHsv[] = {MIAUG_OP_HSV};
const uint32_t kSeqBlur3[] = {MIAUG_OP_BLUR3};
const uint32_t kSeqBlur5[] = {MIAUG_OP_BLUR5};

// Index of the first op of `ops` that breaks the order of `seq` (n if none).
int match_order(const miaug_op *ops, int n, const uint32_t *seq, int nseq) {
    int j = 0;
    for (int i = 0; i < n; ++i) {
        while (j < nseq && seq[j] != ops[i].kind) ++j;
        if (j == nseq) return i;
        ++j;
    }
    return n;
}

bool has(const miaug_op *ops, int n, uint32_t k) {
    for (int i = 0; i < n; ++i)
        if (ops[i].kind == k) return true;
    return false;
}

}  // namespace
}  // namespace miaug

using namespace miaug;

struct miaug_pipeline {
    miaug_ctx *ctx;
    int kind;
    std::vector<miaug_op> ops;
    int out_h, out_w;        // RESIZE size (RAGGED, U8CHAIN)
    int crop_h, crop_w;      // CROP size (U8CHAIN)
    float mean[3], stdv[3];  // NORMALIZE (RAGGED)
    int el_alpha, el_radius; // ELASTIC (DISTORT); el_alpha < 0: no elastic op
    bool wcrop;              // SIZED_CROP (RAGGED): records carry a crop window
    bool color;              // SHIFT_RGB or TO_GRAY (DIH4): per-channel LUTs and grayscale flags
    int interp, border;      // WARP: of the ROTATE / SSR op; PAD: border
    int pad_value;           // PAD, constant border
    int blur_k;              // BLUR chain: 3 or 5
    int chan;                // channels of the batch being staged (DIH4 colour LUT layout)
    double el_sigma;
    bool el_box;             // box-cascade approximation of the field
    // pinned staging of packed records, device copies, chain buffers
    void *pinned = nullptr;
    size_t pinned_cap = 0;
    hipEvent_t staged = nullptr;  // recorded after the last copy out of `pinned`
    void *dparams = nullptr;
    size_t dparams_cap = 0;
    void *dwork = nullptr;  // DISTORT: fields, elastic workspace, tables
    size_t dwork_cap = 0;
};

struct miaug_pipeline_graph {
    miaug_pipeline *p;
    int n, H, W, chan;
    void *pinned;  // this graph's own staging buffer (read by its copy node)
    size_t packed;
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipEvent_t done;
};

namespace {

int op_check(const miaug_op &o, int i) {
    const char *nm = op_name(o.kind);
    if (!(o.p >= 0.f && o.p <= 1.f)) return set_error(MIAUG_EINVAL, "pipeline: op %d (%s): p outside [0, 1]", i, nm);
    for (int k = 0; k < 4; ++k)
        if (!(o.lo[k] <= o.hi[k]) && o.kind != MIAUG_OP_NORMALIZE && o.kind != MIAUG_OP_ELASTIC &&
            o.kind != MIAUG_OP_GRID && o.kind != MIAUG_OP_PAD)
            return set_error(MIAUG_EINVAL, "pipeline: op %d (%s): lo[%d] > hi[%d]", i, nm, k, k);
    switch (o.kind) {
    case MIAUG_OP_ROT90:
        if (o.lo[0] < 0.f || o.hi[0] > 3.f || o.lo[0] != floorf(o.lo[0]) || o.hi[0] != floorf(o.hi[0]))
            return set_error(MIAUG_EINVAL, "pipeline: op %d (ROT90): k range must be integers in 0..3", i);
        break;
    case MIAUG_OP_SSR:
        if (o.interp != MIAUG_INTERP_BILINEAR && o.interp != MIAUG_INTERP_NEAREST)
            return set_error(MIAUG_EINVAL, "pipeline: op %d (SSR): interp %u", i, o.interp);
        if (o.border != MIAUG_BORDER_REFLECT101 && o.border != MIAUG_BORDER_CONSTANT)
            return set_error(MIAUG_EINVAL, "pipeline: op %d (SSR): border %u", i, o.border);
        if (!(o.lo[1] > 0.f)) return set_error(MIAUG_EINVAL, "pipeline: op %d (SSR): scale must be > 0", i);
        break;
    case MIAUG_OP_CROP:
    case MIAUG_OP_RESIZE:
        if (o.out_h < 1 || o.out_w < 1 || o.out_h > 4096 || o.out_w > 4096)
            return set_error(MIAUG_EINVAL, "pipeline: op %d (%s): size %dx%d outside 1..4096", i, nm, o.out_h, o.out_w);
        if (o.kind == MIAUG_OP_RESIZE && o.interp != MIAUG_INTERP_BILINEAR)
            return set_error(MIAUG_EUNSUPPORTED, "pipeline: op %d (RESIZE): images are resized bilinearly", i);
        if (o.kind == MIAUG_OP_CROP && o.p != 1.f)
            return set_error(MIAUG_EUNSUPPORTED, "pipeline: op %d (CROP): p must be 1", i);
        break;
    case MIAUG_OP_ELASTIC:
        if (o.p != 1.f) return set_error(MIAUG_EUNSUPPORTED, "pipeline: op %d (ELASTIC): p must be 1", i);
        if (!(o.lo[0] >= 0.f && o.lo[0] <= 65535.f && o.lo[0] == floorf(o.lo[0])) || !(o.lo[1] > 0.f) ||
            !(o.lo[2] >= 0.f && o.lo[2] <= 200.f))
            return set_error(MIAUG_EINVAL, "pipeline: op %d (ELASTIC): alpha, sigma or radius out of range", i);
        break;
    case MIAUG_OP_GRID:
        if (!(o.lo[0] >= 0.f && o.lo[0] < 1.f))
            return set_error(MIAUG_EINVAL, "pipeline: op %d (GRID): limit outside [0, 1)", i);
        break;
    case MIAUG_OP_NORMALIZE:
        if (o.p != 1.f) return set_error(MIAUG_EUNSUPPORTED, "pipeline: op %d (NORMALIZE): p must be 1", i);
        for (int c = 0; c < 3; ++c)
            if (!(o.hi[c] != 0.f)) return set_error(MIAUG_EINVAL, "pipeline: op %d (NORMALIZE): std[%d] is 0", i, c);
        break;
    case MIAUG_OP_ROTATE:
    case MIAUG_OP_PAD:
        if (o.interp != MIAUG_INTERP_BILINEAR && o.interp != MIAUG_INTERP_NEAREST)
            return set_error(MIAUG_EINVAL, "pipeline: op %d (%s): interp %u", i, nm, o.interp);
        if (o.border != MIAUG_BORDER_REFLECT101 && o.border != MIAUG_BORDER_CONSTANT)
            return set_error(MIAUG_EINVAL, "pipeline: op %d (%s): border %u", i, nm, o.border);
        if (o.kind == MIAUG_OP_PAD) {
            if (o.p != 1.f) return set_error(MIAUG_EUNSUPPORTED, "pipeline: op %d (PAD): p must be 1", i);
            if (o.out_h < 0 || o.out_w < 0 || o.out_h > 16384 || o.out_w > 16384)
                return set_error(MIAUG_EINVAL, "pipeline: op %d (PAD): size %dx%d outside 0..16384", i, o.out_h, o.out_w);
            if (!(o.lo[0] >= 0.f && o.lo[0] <= 255.f))
                return set_error(MIAUG_EINVAL, "pipeline: op %d (PAD): value outside 0..255", i);
        }
        break;
    case MIAUG_OP_SIZED_CROP:
        if (!(o.lo[0] > 0.f && o.hi[0] <= 1.f && o.lo[1] > 0.f))
            return set_error(MIAUG_EINVAL, "pipeline: op %d (SIZED_CROP): need 0 < scale <= 1, ratio > 0", i);
        break;
    default:
        if (o.kind < MIAUG_OP_HFLIP || o.kind > MIAUG_OP_ROTATE)
            return set_error(MIAUG_EINVAL, "pipeline: op %d: unknown kind %u", i, o.kind);
    }
    return MIAUG_OK;
}

int grow_pinned(miaug_pipeline *p, size_t bytes) {
    if (bytes <= p->pinned_cap) return MIAUG_OK;
    if (p->pinned) {
        if (p->staged) hipEventSynchronize(p->staged);
        hipHostFree(p->pinned);
        p->pinned = nullptr;
        p->pinned_cap = 0;
    }
    int st = pinned_alloc(&p->pinned, bytes, "pipeline: pinned staging");
    if (!st) p->pinned_cap = bytes;
    return st;
}

int grow_device(void **ptr, size_t *cap, size_t bytes, const char *what) {
    if (bytes <= *cap) return MIAUG_OK;
    if (*ptr) {
        hipDeviceSynchronize();  // the old buffer may still be read by enqueued work
        hipFree(*ptr);
        *ptr = nullptr;
        *cap = 0;
    }
    int st = dev_alloc(ptr, bytes, what);
    if (!st) *cap = bytes;
    return st;
}

// Packed device form of the records of one batch (host side), by chain:
//   DIH4, RAGGED: int32 flags [n][4], then float ab [n][2] (RAGGED with
//                 SIZED_CROP: then int32 windows [n][4]; DIH4: then the
//                 identity ab block of the masks, float [n][2], and with
//                 colour ops u8 LUTs [n][C][256] and int32 gray flags [n])
//   U8CHAIN:      miaug_c2_record [n]
//   DISTORT:      double grid [n][10]
//   WARP:         int64 Q32 matrices [n][6]
//   PAD:          nothing (8 bytes of padding)
//   HSV:          int32 shifts [n][3] (dh, ds, dv)
//   BLUR:         int32 on/off flags [n]
size_t packed_bytes(const miaug_pipeline *p, int n, int C) {
    switch (p->kind) {
    case MIAUG_PIPE_DIH4: return (size_t)n * 32 + (p->color ? (size_t)n * (256 * C + 4) : 0);
    case MIAUG_PIPE_RAGGED: return (size_t)n * (p->wcrop ? 40 : 24);
    case MIAUG_PIPE_U8CHAIN: return (size_t)n * sizeof(miaug_c2_record);
    case MIAUG_PIPE_WARP: return (size_t)n * 48;
    case MIAUG_PIPE_PAD: return 8;
    case MIAUG_PIPE_HSV: return (size_t)n * 12;
    case MIAUG_PIPE_BLUR: return (size_t)n * 4;
    default: return (size_t)n * 10 * sizeof(double);
    }
}

int pack(const miaug_pipeline *p, const miaug_params *r, int n, int H, int W, int C, void *dst) {
    if (p->kind == MIAUG_PIPE_PAD) return MIAUG_OK;
    if (p->kind == MIAUG_PIPE_BLUR) {
        int32_t *d = (int32_t *)dst;
        for (int i = 0; i < n; ++i) d[i] = r[i].blur;
        return MIAUG_OK;
    }
    if (p->kind == MIAUG_PIPE_HSV) {
        int32_t *d = (int32_t *)dst;
        for (int i = 0; i < n; ++i) {
            d[3 * i] = r[i].dh;
            d[3 * i + 1] = r[i].ds;
            d[3 * i + 2] = r[i].dv;
        }
        return MIAUG_OK;
    }
    if (p->kind == MIAUG_PIPE_WARP) {
        std::vector<float> f(4 * (size_t)n);
        for (int i = 0; i < n; ++i) {
            f[4 * i] = r[i].angle;
            f[4 * i + 1] = r[i].scale;
            f[4 * i + 2] = r[i].dx;
            f[4 * i + 3] = r[i].dy;
        }
        return miaug_compile_ssr_q32(f.data(), n, H, W, (int64_t *)dst);
    }
    if (p->kind == MIAUG_PIPE_DIH4 || p->kind == MIAUG_PIPE_RAGGED) {
        int32_t *fl = (int32_t *)dst;
        float *ab = (float *)((char *)dst + (size_t)n * 16);
        for (int i = 0; i < n; ++i) {
            for (int k = 0; k < 4; ++k) fl[4 * i + k] = r[i].flags[k];
            ab[2 * i] = r[i].alpha;
            ab[2 * i + 1] = r[i].beta;
        }
        if (p->kind == MIAUG_PIPE_DIH4) {
            float *ab1 = (float *)((char *)dst + (size_t)n * 24);
            for (int i = 0; i < n; ++i) {
                ab1[2 * i] = 1.f;
                ab1[2 * i + 1] = 0.f;
            }
        }
        if (p->kind == MIAUG_PIPE_DIH4 && p->color) {
            uint8_t *luts = (uint8_t *)dst + (size_t)n * 32;
            int32_t *gray = (int32_t *)(luts + (size_t)n * 256 * C);
            std::vector<float> sh((size_t)n * C, 0.f);
            for (int i = 0; i < n; ++i) {
                for (int c = 0; c < C && c < 3; ++c) sh[(size_t)C * i + c] = r[i].shift[c];
                gray[i] = r[i].gray;
            }
            int st = miaug_compile_color_luts(ab, sh.data(), n, C, luts);
            if (st) return st;
            if (has(p->ops.data(), (int)p->ops.size(), MIAUG_OP_GAMMA)) {
                // gamma after brightness/contrast and ShiftRGB, each step rounded to u8
                uint8_t g[256];
                for (int i = 0; i < n; ++i) {
                    const float gi = r[i].gamma;
                    if ((st = miaug_compile_gamma_luts(&gi, 1, 1, g))) return st;
                    uint8_t *l = luts + (size_t)i * C * 256;
                    for (int e = 0; e < C * 256; ++e) l[e] = g[l[e]];
                }
            }
        }
        if (p->wcrop) {
            int32_t *win = (int32_t *)((char *)dst + (size_t)n * 24);
            for (int i = 0; i < n; ++i) {
                win[4 * i] = r[i].crop_y;
                win[4 * i + 1] = r[i].crop_x;
                win[4 * i + 2] = r[i].crop_h;
                win[4 * i + 3] = r[i].crop_w;
            }
        }
        return MIAUG_OK;
    }
    if (p->kind == MIAUG_PIPE_U8CHAIN) {
        std::vector<float> f(5 * (size_t)n);
        std::vector<int32_t> k(5 * (size_t)n);
        for (int i = 0; i < n; ++i) {
            f[5 * i] = r[i].angle;
            f[5 * i + 1] = r[i].scale;
            f[5 * i + 2] = r[i].dx;
            f[5 * i + 3] = r[i].dy;
            f[5 * i + 4] = r[i].gamma;
            k[5 * i] = r[i].crop_x;
            k[5 * i + 1] = r[i].crop_y;
            k[5 * i + 2] = r[i].dh;
            k[5 * i + 3] = r[i].ds;
            k[5 * i + 4] = r[i].blur;
            if (r[i].crop_x < 0 || r[i].crop_y < 0 || r[i].crop_x + p->crop_w > W || r[i].crop_y + p->crop_h > H)
                return set_error(MIAUG_EINVAL, "apply: sample %d: crop offset outside the image", i);
        }
        miaug_c2_record *rec = (miaug_c2_record *)dst;
        int st = miaug_compile_c2(f.data(), k.data(), n, H, W, p->crop_h, rec);
        if (st) return st;
        for (int i = 0; i < n; ++i) rec[i].dv = r[i].dv;
        return MIAUG_OK;
    }
    double *g = (double *)dst;
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 10; ++k) g[10 * i + k] = r[i].grid[k];
    return MIAUG_OK;
}

int batch_check(const miaug_pipeline *p, const miaug_batch_in *in, const miaug_batch_out *out) {
    if (!in || !out) return set_error(MIAUG_EINVAL, "apply: NULL batch");
    if (in->n < 0) return set_error(MIAUG_EINVAL, "apply: n < 0");
    if (in->n == 0) return MIAUG_OK;
    if (!in->img || !out->img) return set_error(MIAUG_EINVAL, "apply: NULL image pointer");
    if (in->mask && !out->mask) return set_error(MIAUG_EINVAL, "apply: masks without an output");
    if (p->kind == MIAUG_PIPE_RAGGED) {
        if (in->channels != 3) return set_error(MIAUG_ESHAPE, "apply: the ragged chain takes RGB images");
        if (!in->img_off || !in->hw) return set_error(MIAUG_EINVAL, "apply: ragged batch without img_off / hw");
        if (in->mask && !in->mask_off) return set_error(MIAUG_EINVAL, "apply: masks without mask_off");
        if (in->boxes && (!in->box_off || !out->boxes)) return set_error(MIAUG_EINVAL, "apply: boxes without offsets/output");
        return MIAUG_OK;
    }
    if ((p->kind == MIAUG_PIPE_WARP || p->kind == MIAUG_PIPE_PAD || p->kind == MIAUG_PIPE_DIH4 ||
         p->kind == MIAUG_PIPE_BLUR) &&
        in->channels != 1 && in->channels != 3 && in->channels != 4)
        return set_error(MIAUG_ESHAPE, "apply: channels must be 1, 3 or 4");
    if (p->kind == MIAUG_PIPE_DIH4 && p->color && has(p->ops.data(), (int)p->ops.size(), MIAUG_OP_TO_GRAY) &&
        in->channels != 3)
        return set_error(MIAUG_ESHAPE, "apply: TO_GRAY takes RGB images");
    if (p->kind == MIAUG_PIPE_HSV && in->channels != 3) return set_error(MIAUG_ESHAPE, "apply: HSV takes RGB images");
    if (in->boxes && p->kind != MIAUG_PIPE_U8CHAIN && p->kind != MIAUG_PIPE_DISTORT)
        return set_error(MIAUG_EUNSUPPORTED, "apply: boxes are supported by the ragged, u8 and distortion chains only");
    if (in->boxes && (!in->box_off || !out->boxes)) return set_error(MIAUG_EINVAL, "apply: boxes without offsets/output");
    if (in->H < 1 || in->W < 1) return set_error(MIAUG_ESHAPE, "apply: dense batch needs H, W >= 1");
    if (p->kind == MIAUG_PIPE_U8CHAIN) {
        if (in->channels != 3) return set_error(MIAUG_ESHAPE, "apply: the u8 chain takes RGB images");
        if (p->crop_h != p->crop_w || p->out_h != p->out_w)
            return set_error(MIAUG_EUNSUPPORTED, "apply: the u8 chain needs a square crop and output");
        if (p->crop_h > in->H || p->crop_w > in->W) return set_error(MIAUG_ESHAPE, "apply: crop larger than the image");
    } else if (in->channels != 1 && in->channels != 3 && in->channels != 4) {
        return set_error(MIAUG_ESHAPE, "apply: channels must be 1, 3 or 4");
    }
    return MIAUG_OK;
}

// Enqueues the chain for a batch whose packed records are at device address
// `dp` (already copied or about to be copied on the same stream).
int run_chain(miaug_pipeline *p, const miaug_batch_in *in, const miaug_params *first, miaug_batch_out *out, void *dp,
              int per_image, hipStream_t s) {
    const int n = in->n;
    if (p->kind == MIAUG_PIPE_DIH4 || p->kind == MIAUG_PIPE_RAGGED) {
        const int32_t *fl = (const int32_t *)dp;
        const float *ab = (const float *)((char *)dp + (size_t)n * 16);
        if (p->kind == MIAUG_PIPE_RAGGED) {
            miaug_ragged_args a;
            memset(&a, 0, sizeof(a));
            a.n = n;
            a.out_h = p->out_h;
            a.out_w = p->out_w;
            a.img = in->img;
            a.img_off = in->img_off;
            a.hw = in->hw;
            a.flags = fl;
            a.ab = ab;
            a.crop = p->wcrop ? (const int32_t *)((char *)dp + (size_t)n * 24) : nullptr;
            a.mask = in->mask;
            a.mask_off = in->mask_off;
            a.boxes = in->boxes;
            a.box_off = in->box_off;
            for (int c = 0; c < 3; ++c) {
                a.mean[c] = p->mean[c];
                a.stdv[c] = p->stdv[c];
            }
            a.out = (float *)out->img;
            a.out_mask = out->mask;
            a.out_boxes = out->boxes;
            return per_image ? miaug_ragged_apply_per_image(p->ctx, &a, s) : miaug_ragged_apply(p->ctx, &a, s);
        }
        const size_t isz = (size_t)in->H * in->W * in->channels, msz = (size_t)in->H * in->W;
        const uint8_t *luts = (const uint8_t *)dp + (size_t)n * 32;
        const int32_t *gray = (const int32_t *)(luts + (size_t)n * 256 * in->channels);
        const bool to_gray = p->color && has(p->ops.data(), (int)p->ops.size(), MIAUG_OP_TO_GRAY);
        auto images = [&](int i0, int cnt) {
            const uint8_t *src = in->img + i0 * isz;
            uint8_t *dst = (uint8_t *)out->img + i0 * isz;
            if (p->color)
                return miaug_d4_lut_u8(src, cnt, in->H, in->W, in->channels, fl + 4 * i0,
                                       luts + (size_t)i0 * 256 * in->channels, to_gray ? gray + i0 : nullptr, dst, s);
            return miaug_d4_bc_u8(src, cnt, in->H, in->W, in->channels, fl + 4 * i0, ab + 2 * i0, dst, s);
        };
        if (!per_image) {
            int st = images(0, n);
            // masks: same Dih4 element, no colour change (alpha 1, beta 0 is the identity LUT)
            if (!st && in->mask) {
                float *ab1 = (float *)((char *)dp + (size_t)n * 24);
                st = miaug_d4_bc_u8(in->mask, n, in->H, in->W, 1, fl, ab1, out->mask, s);
            }
            return st;
        }
        for (int i = 0; i < n; ++i) {
            int st = images(i, 1);
            if (!st && in->mask) {
                float *ab1 = (float *)((char *)dp + (size_t)n * 24);
                st = miaug_d4_bc_u8(in->mask + i * msz, 1, in->H, in->W, 1, fl + 4 * i, ab1 + 2 * i,
                                    out->mask + i * msz, s);
            }
            if (st) return st;
        }
        return MIAUG_OK;
    }
    if (p->kind == MIAUG_PIPE_U8CHAIN) {
        const miaug_c2_record *rec = (const miaug_c2_record *)dp;
        int st = MIAUG_OK;
        if (!per_image) {
            st = miaug_ssr_crop_resize_hsv_gamma_blur_u8(in->img, n, in->H, in->W, rec, p->crop_h, p->out_h,
                                                         (uint8_t *)out->img, s);
            if (!st && in->mask)
                st = miaug_ssr_crop_resize_mask_u8(in->mask, n, in->H, in->W, rec, p->crop_h, p->out_h, out->mask, s);
        } else {
            const size_t isz = (size_t)in->H * in->W * 3, osz = (size_t)p->out_h * p->out_w * 3;
            const size_t msz = (size_t)in->H * in->W, mosz = (size_t)p->out_h * p->out_w;
            for (int i = 0; i < n && !st; ++i) {
                st = miaug_ssr_crop_resize_hsv_gamma_blur_u8(in->img + i * isz, 1, in->H, in->W, rec + i, p->crop_h,
                                                             p->out_h, (uint8_t *)out->img + i * osz, s);
                if (!st && in->mask)
                    st = miaug_ssr_crop_resize_mask_u8(in->mask + i * msz, 1, in->H, in->W, rec + i, p->crop_h,
                                                       p->out_h, out->mask + i * mosz, s);
            }
        }
        // boxes: one small launch over the whole batch in both forms (their offsets live on the device)
        if (!st && in->boxes)
            st = miaug_boxes_ssr_crop_resize(in->boxes, in->box_off, n, in->H, in->W, rec, p->crop_h, p->out_h,
                                             out->boxes, s);
        return st;
    }
    if (p->kind == MIAUG_PIPE_BLUR) {
        const size_t isz = (size_t)in->H * in->W * in->channels, msz = (size_t)in->H * in->W;
        const int32_t *d = (const int32_t *)dp;
        int st = MIAUG_OK;
        for (int i0 = 0; i0 < n && !st; i0 += per_image ? 1 : n)
            st = miaug_blur_u8(in->img + i0 * isz, per_image ? 1 : n, in->H, in->W, in->channels, p->blur_k, d + i0,
                               (uint8_t *)out->img + i0 * isz, s);
        // masks: a colour op leaves them as they are
        if (!st && in->mask && out->mask != in->mask)
            st = hip_status(hipMemcpyAsync(out->mask, in->mask, (size_t)n * msz, hipMemcpyDeviceToDevice,
                                           (hipStream_t)s), "apply: mask copy");
        return st;
    }
    if (p->kind == MIAUG_PIPE_HSV) {
        const size_t isz = (size_t)in->H * in->W * 3, msz = (size_t)in->H * in->W;
        const int32_t *d = (const int32_t *)dp;
        int st = MIAUG_OK;
        for (int i0 = 0; i0 < n && !st; i0 += per_image ? 1 : n)
            st = miaug_hsv_shift_u8(in->img + i0 * isz, per_image ? 1 : n, in->H, in->W, d + 3 * i0,
                                    (uint8_t *)out->img + i0 * isz, s);
        // masks: a point op leaves them as they are
        if (!st && in->mask && out->mask != in->mask)
            st = hip_status(hipMemcpyAsync(out->mask, in->mask, (size_t)n * msz, hipMemcpyDeviceToDevice,
                                           (hipStream_t)s), "apply: mask copy");
        return st;
    }
    if (p->kind == MIAUG_PIPE_WARP || p->kind == MIAUG_PIPE_PAD) {
        const int C = in->channels, H = in->H, W = in->W;
        const int Ho = p->kind == MIAUG_PIPE_PAD ? (H > p->out_h ? H : p->out_h) : H;
        const int Wo = p->kind == MIAUG_PIPE_PAD ? (W > p->out_w ? W : p->out_w) : W;
        const size_t isz = (size_t)H * W * C, osz = (size_t)Ho * Wo * C, msz = (size_t)H * W, mosz = (size_t)Ho * Wo;
        const int64_t *aq = (const int64_t *)dp;
        int st = MIAUG_OK;
        for (int i0 = 0; i0 < n && !st; i0 += per_image ? 1 : n) {
            const int cnt = per_image ? 1 : n;
            if (p->kind == MIAUG_PIPE_WARP) {
                st = miaug_warp_affine_u8(in->img + i0 * isz, cnt, H, W, C, aq + 6 * i0, p->interp, p->border,
                                          (uint8_t *)out->img + i0 * osz, s);
                // masks: the same map with nearest taps
                if (!st && in->mask)
                    st = miaug_warp_affine_u8(in->mask + i0 * msz, cnt, H, W, 1, aq + 6 * i0, MIAUG_INTERP_NEAREST,
                                              p->border, out->mask + i0 * mosz, s);
            } else {
                st = miaug_pad_u8(in->img + i0 * isz, cnt, H, W, C, p->out_h, p->out_w, p->border, p->pad_value,
                                  (uint8_t *)out->img + i0 * osz, s);
                // masks: the same border, constant padding with label 0
                if (!st && in->mask)
                    st = miaug_pad_u8(in->mask + i0 * msz, cnt, H, W, 1, p->out_h, p->out_w, p->border, 0,
                                      out->mask + i0 * mosz, s);
            }
        }
        return st;
    }
    // DISTORT: fields (or zero offsets), grid tables (from the records, or identity factors), remap chain
    const int H = in->H, W = in->W;
    const size_t field_bytes = (size_t)n * 2 * H * W * sizeof(int32_t);
    const size_t ews = p->el_alpha < 0 ? 0
                       : (p->el_box ? miaug_elastic_box_workspace_bytes(n, H, W) : miaug_elastic_workspace_bytes(n, H, W));
    const size_t tab_bytes = (size_t)n * (H + W) * sizeof(int32_t);
    char *w = (char *)p->dwork;
    int32_t *off = (int32_t *)w;
    void *ew = w + field_bytes;
    int32_t *mapx = (int32_t *)(w + field_bytes + ews);
    int32_t *mapy = mapx + (size_t)n * W;
    (void)tab_bytes;
    int st;
    if (p->el_alpha >= 0 && p->el_box)
        st = miaug_elastic_fields_box(first->seed, first->index, n, H, W, p->el_sigma, p->el_alpha, off, ew, ews, s);
    else if (p->el_alpha >= 0)
        st = miaug_elastic_fields(first->seed, first->index, n, H, W, p->el_sigma, p->el_alpha, p->el_radius, off, ew,
                                  ews, s);
    else
        st = hip_status(launch_fill_u32((uint32_t *)off, (size_t)n * 2 * H * W, 0u, s), "pipeline: zero offsets");
    if (!st) st = miaug_grid_tables((const double *)dp, n, H, W, mapx, mapy, s);
    if (!st)
        st = miaug_elastic_grid_u8(in->img, in->mask, n, H, W, in->channels, off, mapx, mapy, (uint8_t *)out->img,
                                   out->mask, per_image, s);
    if (!st && in->boxes)
        st = miaug_boxes_elastic_grid(in->boxes, in->box_off, n, H, W, off, mapx, mapy, out->boxes, s);
    return st;
}

size_t distort_work_bytes(const miaug_pipeline *p, int n, int H, int W) {
    size_t b = (size_t)n * 2 * H * W * sizeof(int32_t) + (size_t)n * (H + W) * sizeof(int32_t);
    if (p->el_alpha >= 0)
        b += p->el_box ? miaug_elastic_box_workspace_bytes(n, H, W) : miaug_elastic_workspace_bytes(n, H, W);
    return b + 256;
}

// Device buffers for a batch of this shape.
int prepare(miaug_pipeline *p, const miaug_batch_in *in) {
    const int n = in->n;
    p->chan = in->channels;
    size_t need = packed_bytes(p, n, in->channels);
    int st = grow_device(&p->dparams, &p->dparams_cap, need + 256, "pipeline: device records");
    if (st) return st;
    if (p->kind == MIAUG_PIPE_DISTORT) {
        if ((long long)in->H * in->W > (1ll << 30)) return set_error(MIAUG_ESHAPE, "apply: image too large");
        st = grow_device(&p->dwork, &p->dwork_cap, distort_work_bytes(p, n, in->H, in->W), "pipeline: distortion buffers");
    }
    return st;
}

// Host bytes staged per batch.
size_t staged_bytes(const miaug_pipeline *p, int n, int C) { return packed_bytes(p, n, C); }

int fill_staging(const miaug_pipeline *p, const miaug_batch_in *in, const miaug_params *params, void *buf) {
    const int n = in->n;
    if (p->kind == MIAUG_PIPE_DISTORT) {
        for (int i = 1; i < n; ++i)
            if (params[i].seed != params[0].seed || params[i].index != params[0].index + (uint64_t)i)
                return set_error(MIAUG_EUNSUPPORTED,
                                 "apply: distortion records must be consecutive samples of one seed (sample %d)", i);
    }
    return pack(p, params, n, in->H, in->W, in->channels, buf);
}

int apply_impl(miaug_pipeline *p, const miaug_batch_in *in, const miaug_params *params, miaug_batch_out *out,
               int per_image, void *stream) {
    clear_error();
    if (!p) return set_error(MIAUG_EINVAL, "apply: NULL pipeline");
    if (!p->ctx) return set_error(MIAUG_EINVAL, "apply: the pipeline was created without a context");
    if (int st = batch_check(p, in, out)) return st;
    if (in->n == 0) return MIAUG_OK;
    if (!params) return set_error(MIAUG_EINVAL, "apply: NULL params");
    hipStream_t s = as_stream(stream);
    int st = prepare(p, in);
    const size_t bytes = staged_bytes(p, in->n, in->channels);
    if (!st) st = grow_pinned(p, bytes);
    if (st) return st;
    if (p->staged) hipEventSynchronize(p->staged);  // the previous call's copy has left the staging buffer
    if ((st = fill_staging(p, in, params, p->pinned))) return st;
    st = hip_status(hipMemcpyAsync(p->dparams, p->pinned, bytes, hipMemcpyHostToDevice, s), "pipeline: record copy");
    if (!st && !p->staged) st = hip_status(hipEventCreateWithFlags(&p->staged, hipEventDisableTiming), "event");
    if (!st) st = hip_status(hipEventRecord(p->staged, s), "event record");
    if (!st) st = run_chain(p, in, params, out, p->dparams, per_image, s);
    return st;
}

}  // namespace

extern "C" {

int miaug_pipeline_create(miaug_ctx *ctx, const miaug_op *ops, int n_ops, miaug_pipeline **out) {
    clear_error();
    if (!out) return set_error(MIAUG_EINVAL, "pipeline_create: out is NULL");
    *out = nullptr;
    if (!ops || n_ops < 1) return set_error(MIAUG_EINVAL, "pipeline_create: empty op list");
    for (int i = 0; i < n_ops; ++i)
        if (int st = op_check(ops[i], i)) return st;
    for (int i = 0; i < n_ops; ++i)
        for (int j = 0; j < i; ++j)
            if (ops[i].kind == ops[j].kind)
                return set_error(MIAUG_EUNSUPPORTED, "pipeline_create: op %d (%s) appears twice", i, op_name(ops[i].kind));
    struct Cand {
        int kind;
        const uint32_t *seq;
        int nseq;
    } cands[] = {{MIAUG_PIPE_DIH4, kSeqDih4, 8},     {MIAUG_PIPE_RAGGED, kSeqRagged, 8},
                 {MIAUG_PIPE_U8CHAIN, kSeqU8, 6},    {MIAUG_PIPE_DISTORT, kSeqDistort, 2},
                 {MIAUG_PIPE_WARP, kSeqRotate, 1},   {MIAUG_PIPE_WARP, kSeqSsr, 1},
                 {MIAUG_PIPE_PAD, kSeqPad, 1},       {MIAUG_PIPE_HSV, kSeqHsv, 1},
                 {MIAUG_PIPE_BLUR, kSeqBlur3, 1},    {MIAUG_PIPE_BLUR, kSeqBlur5, 1}};
    int kind = 0, worst = -1;
    for (const Cand &c : cands) {
        const int at = match_order(ops, n_ops, c.seq, c.nseq);
        if (at < n_ops) {
            worst = worst < at ? at : worst;
            continue;
        }
        if (c.kind == MIAUG_PIPE_DIH4 && has(ops, n_ops, MIAUG_OP_RESIZE)) continue;
        if (c.kind == MIAUG_PIPE_RAGGED && !has(ops, n_ops, MIAUG_OP_RESIZE)) continue;
        if (c.kind == MIAUG_PIPE_U8CHAIN && (!has(ops, n_ops, MIAUG_OP_CROP) || !has(ops, n_ops, MIAUG_OP_RESIZE))) {
            worst = n_ops - 1;
            continue;
        }
        if (c.kind == MIAUG_PIPE_U8CHAIN)
            for (int i = 0; i < n_ops; ++i)
                if (ops[i].kind == MIAUG_OP_SSR &&
                    (ops[i].interp != MIAUG_INTERP_BILINEAR || ops[i].border != MIAUG_BORDER_REFLECT101))
                    return set_error(MIAUG_EUNSUPPORTED,
                                     "pipeline_create: op %d (SSR): the u8 chain warps bilinearly with reflect-101", i);
        kind = c.kind;
        break;
    }
    if (!kind)
        return set_error(MIAUG_EUNSUPPORTED, "pipeline_create: no fused chain takes this op list (op %d, %s, breaks it)",
                         worst < 0 ? 0 : worst, op_name(ops[worst < 0 ? 0 : worst].kind));
    miaug_pipeline *p = new (std::nothrow) miaug_pipeline;
    if (!p) return set_error(MIAUG_ENOMEM, "pipeline_create: host allocation");
    p->ctx = ctx;
    p->kind = kind;
    p->ops.assign(ops, ops + n_ops);
    p->out_h = p->out_w = p->crop_h = p->crop_w = 0;
    for (int c = 0; c < 3; ++c) {
        p->mean[c] = 0.f;
        p->stdv[c] = 1.f / 255.f;  // no NORMALIZE: the float output is the u8 value
    }
    p->el_alpha = -1;
    p->el_radius = 0;
    p->el_sigma = 0.0;
    p->el_box = false;
    p->wcrop = false;
    p->color = false;
    p->interp = MIAUG_INTERP_BILINEAR;
    p->border = MIAUG_BORDER_REFLECT101;
    p->pad_value = 0;
    p->blur_k = 3;
    p->chan = 3;
    for (const miaug_op &o : p->ops) {
        if (o.kind == MIAUG_OP_SIZED_CROP) p->wcrop = true;
        if (o.kind == MIAUG_OP_BLUR5) p->blur_k = 5;
        if (o.kind == MIAUG_OP_SHIFT_RGB || o.kind == MIAUG_OP_TO_GRAY || (o.kind == MIAUG_OP_GAMMA && kind == MIAUG_PIPE_DIH4))
            p->color = true;
        if (o.kind == MIAUG_OP_ROTATE || o.kind == MIAUG_OP_PAD || (o.kind == MIAUG_OP_SSR && kind == MIAUG_PIPE_WARP)) {
            p->interp = (int)o.interp;
            p->border = (int)o.border;
        }
        if (o.kind == MIAUG_OP_PAD) {
            p->out_h = o.out_h;
            p->out_w = o.out_w;
            p->pad_value = (int)o.lo[0];
        }
        if (o.kind == MIAUG_OP_RESIZE) {
            p->out_h = o.out_h;
            p->out_w = o.out_w;
        } else if (o.kind == MIAUG_OP_CROP) {
            p->crop_h = o.out_h;
            p->crop_w = o.out_w;
        } else if (o.kind == MIAUG_OP_NORMALIZE) {
            for (int c = 0; c < 3; ++c) {
                p->mean[c] = o.lo[c];
                p->stdv[c] = o.hi[c];
            }
        } else if (o.kind == MIAUG_OP_ELASTIC) {
            p->el_alpha = (int)o.lo[0];
            p->el_sigma = o.lo[1];
            p->el_box = o.hi[0] != 0.f;
            p->el_radius = o.lo[2] > 0.f ? (int)o.lo[2] : (int)ceil(3.0 * o.lo[1]);
            if (p->el_radius < 1 || p->el_radius > 200) {
                delete p;
                return set_error(MIAUG_EINVAL, "pipeline_create: ELASTIC radius %d outside 1..200", p->el_radius);
            }
        }
    }
    *out = p;
    return MIAUG_OK;
}

int miaug_pipeline_destroy(miaug_pipeline *p) {
    clear_error();
    if (!p) return MIAUG_OK;
    if (p->dparams || p->dwork) hipDeviceSynchronize();
    if (p->staged) {
        hipEventSynchronize(p->staged);
        hipEventDestroy(p->staged);
    }
    if (p->pinned) hipHostFree(p->pinned);
    if (p->dparams) hipFree(p->dparams);
    if (p->dwork) hipFree(p->dwork);
    delete p;
    return MIAUG_OK;
}

int miaug_pipeline_kind(const miaug_pipeline *p) {
    clear_error();
    return p ? p->kind : set_error(MIAUG_EINVAL, "pipeline_kind: NULL pipeline");
}

size_t miaug_param_bytes(const miaug_pipeline *p, int n) {
    return (p && n > 0) ? (size_t)n * sizeof(miaug_params) : 0;
}

int miaug_sample(const miaug_pipeline *p, uint64_t seed, uint64_t first_index, int n, const int32_t *hw,
                 miaug_params *params) {
    clear_error();
    if (!p || n < 0 || (n > 0 && !params)) return set_error(MIAUG_EINVAL, "sample: bad arguments");
    const bool crop = has(p->ops.data(), (int)p->ops.size(), MIAUG_OP_CROP) ||
                      has(p->ops.data(), (int)p->ops.size(), MIAUG_OP_SIZED_CROP);
    if (crop && n > 0 && !hw) return set_error(MIAUG_EINVAL, "sample: the op list crops: source sizes needed");
    for (int i = 0; i < n; ++i) {
        miaug_params &r = params[i];
        memset(&r, 0, sizeof(r));
        r.seed = seed;
        r.index = first_index + (uint64_t)i;
        r.alpha = 1.f;
        r.scale = 1.f;
        r.gamma = 1.f;
        for (int k = 0; k < 10; ++k) r.grid[k] = 1.0;
        const Gen G{seed, r.index};
        for (int j = 0; j < (int)p->ops.size(); ++j) {
            const miaug_op &o = p->ops[j];
            const uint64_t d = 16 * (uint64_t)j;
            const bool on = o.p >= 1.f ? true : G.bern(d, o.p);
            switch (o.kind) {
            case MIAUG_OP_HFLIP: r.flags[0] = on; break;
            case MIAUG_OP_VFLIP: r.flags[1] = on; break;
            case MIAUG_OP_TRANSPOSE: r.flags[3] = on; break;
            case MIAUG_OP_ROT90:
                if (on) r.flags[2] = (int)o.lo[0] + G.below(d + 1, (uint32_t)((int)o.hi[0] - (int)o.lo[0] + 1));
                break;
            case MIAUG_OP_BRIGHT_CONTRAST:
                if (on) {
                    r.alpha = G.range(d + 1, o.lo[0], o.hi[0]);
                    r.beta = G.range(d + 2, o.lo[1], o.hi[1]);
                }
                break;
            case MIAUG_OP_SSR:
                if (on) {
                    r.angle = G.range(d + 1, o.lo[0], o.hi[0]);
                    r.scale = G.range(d + 2, o.lo[1], o.hi[1]);
                    r.dx = G.range(d + 3, o.lo[2], o.hi[2]);
                    r.dy = G.range(d + 4, o.lo[3], o.hi[3]);
                }
                break;
            case MIAUG_OP_CROP: {
                const int H = hw[2 * i], W = hw[2 * i + 1];
                if (H < o.out_h || W < o.out_w)
                    return set_error(MIAUG_ESHAPE, "sample: sample %d: %dx%d image smaller than the crop", i, H, W);
                r.crop_y = G.below(d + 1, (uint32_t)(H - o.out_h + 1));
                r.crop_x = G.below(d + 2, (uint32_t)(W - o.out_w + 1));
                break;
            }
            case MIAUG_OP_ROTATE:
                if (on) r.angle = G.range(d + 1, o.lo[0], o.hi[0]);
                break;
            case MIAUG_OP_SHIFT_RGB:
                if (on)
                    for (int c = 0; c < 3; ++c) r.shift[c] = G.range(d + 1 + (uint64_t)c, o.lo[c], o.hi[c]);
                break;
            case MIAUG_OP_TO_GRAY: r.gray = on; break;
            case MIAUG_OP_SIZED_CROP:
                if (on) {
                    // the window lives in the Dih4 image (drawn by the ops before this one)
                    const bool swap = ((r.flags[2] & 1) != 0) != (r.flags[3] != 0);
                    const int H = swap ? hw[2 * i + 1] : hw[2 * i], W = swap ? hw[2 * i] : hw[2 * i + 1];
                    if (H < 1 || W < 1) return set_error(MIAUG_ESHAPE, "sample: sample %d: empty image", i);
                    int32_t win[4];
                    sized_crop(seed, r.index, d + 1, H, W, o.lo[0], o.hi[0], o.lo[1], o.hi[1], win);
                    r.crop_y = win[0];
                    r.crop_x = win[1];
                    r.crop_h = win[2];
                    r.crop_w = win[3];
                }
                break;
            case MIAUG_OP_HSV:
                if (on) {
                    r.dh = (int32_t)rint((double)G.range(d + 1, o.lo[0], o.hi[0]));
                    r.ds = (int32_t)rint((double)G.range(d + 2, o.lo[1], o.hi[1]));
                    r.dv = (int32_t)rint((double)G.range(d + 3, o.lo[2], o.hi[2]));
                }
                break;
            case MIAUG_OP_GAMMA:
                if (on) r.gamma = G.range(d + 1, o.lo[0], o.hi[0]);
                break;
            case MIAUG_OP_BLUR3:
            case MIAUG_OP_BLUR5: r.blur = on; break;
            case MIAUG_OP_GRID:
                if (on)
                    for (int k = 0; k < 10; ++k)
                        r.grid[k] = 1.0 + (double)G.range(d + 1 + (uint64_t)k, -(double)o.lo[0], (double)o.lo[0]);
                break;
            default: break;  // RESIZE, NORMALIZE, ELASTIC: no per-sample draws here
            }
        }
    }
    return MIAUG_OK;
}

int miaug_apply(miaug_pipeline *p, const miaug_batch_in *in, const miaug_params *params, miaug_batch_out *out,
                void *stream) {
    return apply_impl(p, in, params, out, 0, stream);
}

int miaug_apply_per_image(miaug_pipeline *p, const miaug_batch_in *in, const miaug_params *params,
                          miaug_batch_out *out, void *stream) {
    return apply_impl(p, in, params, out, 1, stream);
}

int miaug_pipeline_graph_capture(miaug_pipeline *p, const miaug_batch_in *in, const miaug_batch_out *out,
                                 void *stream, miaug_pipeline_graph **g) {
    clear_error();
    if (!p || !g) return set_error(MIAUG_EINVAL, "graph_capture: NULL pipeline or out");
    *g = nullptr;
    if (!p->ctx) return set_error(MIAUG_EINVAL, "graph_capture: the pipeline was created without a context");
    if (!stream) return set_error(MIAUG_EINVAL, "graph_capture: capture needs a non-null stream");
    miaug_batch_out o = out ? *out : miaug_batch_out{};
    if (int st = batch_check(p, in, &o)) return st;
    if (in->n == 0) return set_error(MIAUG_EINVAL, "graph_capture: empty batch");
    if (p->kind == MIAUG_PIPE_DISTORT && p->el_alpha >= 0)
        return set_error(MIAUG_EUNSUPPORTED,
                         "graph_capture: the elastic field's noise stream is a launch argument, not a record");
    int st = prepare(p, in);
    if (st) return st;
    miaug_pipeline_graph *G = new (std::nothrow) miaug_pipeline_graph{p, in->n, in->H, in->W, in->channels, nullptr,
                                                                       0, nullptr, nullptr, nullptr};
    if (!G) return set_error(MIAUG_ENOMEM, "graph_capture: host allocation");
    G->packed = staged_bytes(p, in->n, in->channels);
    st = pinned_alloc(&G->pinned, G->packed, "graph_capture: pinned staging");
    if (!st) st = hip_status(hipEventCreateWithFlags(&G->done, hipEventDisableTiming), "event");
    // every record the chains read comes from the staging buffer at replay time; run_chain only
    // reads seed and index of the first record, for the elastic field, which is rejected above
    std::vector<miaug_params> dummy(in->n);
    memset(dummy.data(), 0, dummy.size() * sizeof(miaug_params));
    hipStream_t s = as_stream(stream);
    if (!st) st = hip_status(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (!st) {
        int le = hip_status(hipMemcpyAsync(p->dparams, G->pinned, G->packed, hipMemcpyHostToDevice, s), "record copy");
        if (!le) le = run_chain(p, in, dummy.data(), &o, p->dparams, 0, s);
        hipGraph_t graph = nullptr;
        const int ee = hip_status(hipStreamEndCapture(s, &graph), "hipStreamEndCapture");
        st = le ? le : ee;
        if (!st) st = hip_status(hipGraphInstantiate(&G->exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
        G->graph = graph;
    }
    if (st) {
        miaug_pipeline_graph_destroy(G);
        return st;
    }
    *g = G;
    return MIAUG_OK;
}

int miaug_pipeline_graph_launch(miaug_pipeline_graph *G, const miaug_params *params, void *stream) {
    clear_error();
    if (!G || !params) return set_error(MIAUG_EINVAL, "graph_launch: NULL graph or params");
    hipEventSynchronize(G->done);  // the previous replay has copied its records
    miaug_batch_in in;
    memset(&in, 0, sizeof(in));
    in.n = G->n;
    in.H = G->H;
    in.W = G->W;
    in.channels = G->chan;
    int st = fill_staging(G->p, &in, params, G->pinned);
    if (st) return st;
    hipStream_t s = as_stream(stream);
    st = hip_status(hipGraphLaunch(G->exec, s), "hipGraphLaunch");
    if (!st) st = hip_status(hipEventRecord(G->done, s), "event record");
    return st;
}

int miaug_pipeline_graph_destroy(miaug_pipeline_graph *G) {
    clear_error();
    if (!G) return MIAUG_OK;
    if (G->done) {
        hipEventSynchronize(G->done);
        hipEventDestroy(G->done);
    }
    if (G->exec) hipGraphExecDestroy(G->exec);
    if (G->graph) hipGraphDestroy(G->graph);
    if (G->pinned) hipHostFree(G->pinned);
    delete G;
    return MIAUG_OK;
}

int miaug_pipeline_autotune(miaug_pipeline *p, const miaug_batch_in *in, const miaug_params *params,
                            miaug_batch_out *out, int reps, void *stream) {
    clear_error();
    if (!p) return set_error(MIAUG_EINVAL, "autotune: NULL pipeline");
    if (p->kind != MIAUG_PIPE_RAGGED) return apply_impl(p, in, params, out, 0, stream);
    int st = apply_impl(p, in, params, out, 0, stream);  // stages the records on the device
    if (st || in->n == 0) return st;
    miaug_ragged_args a;
    memset(&a, 0, sizeof(a));
    a.n = in->n;
    a.out_h = p->out_h;
    a.out_w = p->out_w;
    a.img = in->img;
    a.img_off = in->img_off;
    a.hw = in->hw;
    a.flags = (const int32_t *)p->dparams;
    a.ab = (const float *)((char *)p->dparams + (size_t)in->n * 16);
    a.crop = p->wcrop ? (const int32_t *)((char *)p->dparams + (size_t)in->n * 24) : nullptr;
    a.mask = in->mask;
    a.mask_off = in->mask_off;
    a.boxes = in->boxes;
    a.box_off = in->box_off;
    for (int c = 0; c < 3; ++c) {
        a.mean[c] = p->mean[c];
        a.stdv[c] = p->stdv[c];
    }
    a.out = (float *)out->img;
    a.out_mask = out->mask;
    a.out_boxes = out->boxes;
    int chosen = 0;
    float ms = 0.f;
    return miaug_ragged_autotune(p->ctx, &a, reps, stream, &chosen, &ms, nullptr);
}

}  // extern "C"
