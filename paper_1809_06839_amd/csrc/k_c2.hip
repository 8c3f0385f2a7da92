// k_c2.hip -- full u8 pipeline in one pass per output tile: shift-scale-rotate
// warp (bilinear, reflect-101) -> crop -> bilinear resize -> integer HSV shift
// -> gamma LUT -> 3x3 binomial blur (Table I ShiftScaleRotate, RandomCrop64,
// ShiftHSV, Gamma; Sec. II colour transforms).
//
// Every intermediate is rounded exactly as the sequential definition rounds
// it; only the order of evaluation differs.
#include "dev_common.h"
#include "q10_blend.h"
#include "internal.h"

namespace miaug {
namespace {

constexpr int kT = 32;
constexpr int kThreads = 256;
constexpr int kP = kT + 2;  // pre-blur pixels per tile side (halo included)
constexpr int kG = 2 * kP;  // warp samples per tile side

__device__ __forceinline__ int32_t resize_q(int j, int Ls, int Lo) {
    const int D = 2 * Lo;
    const int A = (2 * j + 1) * Ls - Lo;
    int qa = A / D, ra = A - qa * D;
    if (ra < 0) { qa -= 1; ra += D; }
    const int B = ra << kFBits;
    const int qb = B / D, rb = B - qb * D;
    const int q = (qa << kFBits) + qb;
    return q + ((2 * rb > D) | ((2 * rb == D) & (q & 1)));
}

// Three bytes of pixel p (RGB) through one or two aligned dword loads; the
// second dword is read only when the pixel crosses into it, so no load leaves
// the dwords that hold the pixel.
__device__ __forceinline__ uint32_t load_rgb(const uint8_t *p) {
    const uintptr_t a = (uintptr_t)p;
    const uint32_t *w = (const uint32_t *)(a & ~(uintptr_t)3);
    const int sh = (int)(a & 3);
    const uint32_t lo = w[0];
    if (sh <= 1) return lo >> (8 * sh);
    return __builtin_amdgcn_alignbyte(w[1], lo, sh);
}

// Bilinear warp sample at Q10 source position (qx, qy), reflect-101 taps.
__device__ __forceinline__ uint32_t warp_sample(const uint8_t *img, int H, int W, int64_t qx, int64_t qy) {
    int x0 = (int)(qx >> kFBits), y0 = (int)(qy >> kFBits);
    const int ax = (int)(qx & (kFOne - 1)), ay = (int)(qy & (kFOne - 1));
    int x1 = x0 + 1, y1 = y0 + 1;
    if (x0 < 0 || x1 >= W) { x0 = reflect101(x0, W); x1 = reflect101(x1, W); }
    if (y0 < 0 || y1 >= H) { y0 = reflect101(y0, H); y1 = reflect101(y1, H); }
    const uint32_t p00 = load_rgb(img + ((size_t)y0 * W + x0) * 3), p01 = load_rgb(img + ((size_t)y0 * W + x1) * 3);
    const uint32_t p10 = load_rgb(img + ((size_t)y1 * W + x0) * 3), p11 = load_rgb(img + ((size_t)y1 * W + x1) * 3);
    return blend_q10<3>(p00, p01, p10, p11, q10_pair(ax), ay);
}

// n / d rounded to nearest, ties to even, for n < 2^16 and 1 <= d <= 255: a
// float estimate (relative error below 2^-22, so at most one off) and one
// correction each way give the exact floor and remainder.
__device__ __forceinline__ uint32_t udiv_he_small(uint32_t n, uint32_t d) {
    uint32_t q = (uint32_t)((float)n * __builtin_amdgcn_rcpf((float)d));
    int r = (int)n - (int)(q * d);
    if (r < 0) {
        --q;
        r += (int)d;
    } else if (r >= (int)d) {
        ++q;
        r -= (int)d;
    }
    return q + ((2 * r > (int)d) | ((2 * r == (int)d) & (q & 1)));
}

// Integer hexcone HSV shift of one RGB pixel (packed R | G<<8 | B<<16).
// The hue's signed quotient t / C with |t| <= 30 C is taken as
// (t + 30 C) / C - 30: shifting by the even integer 30 keeps the
// ties-to-even rounding.
__device__ __forceinline__ uint32_t hsv_shift(uint32_t rgb, int dh, int ds, int dv) {
    const int R = rgb & 255, G = (rgb >> 8) & 255, B = (rgb >> 16) & 255;
    const int V = max(R, max(G, B)), m = min(R, min(G, B)), C = V - m;
    const int S8 = V ? (int)udiv_he_small(255u * (uint32_t)C, (uint32_t)V) : 0;
    int h = 0;
    if (C != 0) {
        const int t = V == R ? G - B : (V == G ? B - R : R - G);
        const int base = V == R ? 0 : (V == G ? 60 : 120);
        h = base + (int)udiv_he_small((uint32_t)(30 * t + 30 * C), (uint32_t)C) - 30;
    }
    int H8 = h % 180;
    if (H8 < 0) H8 += 180;
    int Hs = (H8 + dh) % 180;
    if (Hs < 0) Hs += 180;
    const int Ss = sat8(S8 + ds), Vs = sat8(V + dv);
    const int sector = Hs / 30, r = Hs - 30 * sector;
    const uint32_t pv = udiv_he((uint32_t)(Vs * (7650 - Ss * 30)), 7650u);
    const uint32_t qv = udiv_he((uint32_t)(Vs * (7650 - Ss * r)), 7650u);
    const uint32_t tv = udiv_he((uint32_t)(Vs * (7650 - Ss * (30 - r))), 7650u);
    const uint32_t v = (uint32_t)Vs;
    uint32_t o0, o1, o2;
    switch (sector) {
    case 0: o0 = v;  o1 = tv; o2 = pv; break;
    case 1: o0 = qv; o1 = v;  o2 = pv; break;
    case 2: o0 = pv; o1 = v;  o2 = tv; break;
    case 3: o0 = pv; o1 = qv; o2 = v;  break;
    case 4: o0 = tv; o1 = pv; o2 = v;  break;
    default: o0 = v; o1 = pv; o2 = qv; break;
    }
    return o0 | (o1 << 8) | (o2 << 16);
}

// Reflect-101 of an index within one reflection of [0, n): -(n - 1) <= i <= 2n - 2, n >= 2.
__device__ __forceinline__ int refl1(int i, int n) { return i < 0 ? -i : (i >= n ? 2 * n - 2 - i : i); }

typedef __attribute__((address_space(3))) void *lds_ptr_t;
constexpr int kStageMax = 40 * 1024;  // bytes of staged source per tile
constexpr int kMaxRows = 160;          // staged source rows per tile

// Three bytes of a staged pixel at LDS byte offset o (any alignment).
__device__ __forceinline__ uint32_t lds_rgb(const uint8_t *st, int o) {
    const uint32_t *w = (const uint32_t *)(st + (o & ~3));
    return __builtin_amdgcn_alignbyte(w[1], w[0], o & 3);
}

// Bilinear blend of four packed RGB taps with Q10 weights, one rounding.
__device__ __forceinline__ uint32_t blend4(uint32_t p00, uint32_t p01, uint32_t p10, uint32_t p11, int ax, int ay) {
    return blend_q10<3>(p00, p01, p10, p11, q10_pair(ax), ay);
}

// One workgroup per (image, T x T output tile):
//  1. resize positions of the (T+2) pre-blur rows and columns, and the affine
//     terms of the crop lines their taps touch (a1 Y + a2, a0 X, ... in Q32);
//  2. the source bounding box of every warp tap of the tile (the map is
//     affine, so its extremes are at the corners of the crop-line ranges);
//     when the box lies inside the image (no reflection needed) and fits,
//     its rows are staged into LDS with 16-byte DMA loads;
//  3. each pre-blur pixel evaluates its 2 x 2 warp samples (taps from LDS, or
//     from global memory with reflect-101 for tiles near the border), the
//     resize blend, the HSV shift and the gamma LUT;
//  4. the output: 3x3 blur (or copy) written as aligned dwords.
__global__ __launch_bounds__(kThreads) void k_c2(const uint8_t *__restrict__ in, int H, int W,
                                                 const miaug_c2_record *__restrict__ recs, int crop, int outsz,
                                                 uint8_t *__restrict__ out) {
    __shared__ __align__(16) uint8_t stage[kStageMax + 16];
    __shared__ uint32_t pre[kP][kP];
    __shared__ int32_t rq[kP], cq[kP];
    __shared__ int64_t tyx[kG], tyy[kG], txx[kG], txy[kG];  // affine terms of crop rows / columns
    __shared__ int32_t rowoff[kMaxRows];                       // LDS offset of staged row r's first pixel
    __shared__ int32_t box[6];                                 // bx, by, bw, bh, nch, staged
    __shared__ uint8_t lut[256];

    const int2 lb = xcd_block();  // (output tile, image): an image's tiles share one XCD's L2
    const int img = lb.y, tid = threadIdx.x;
    const miaug_c2_record &R = recs[img];
    const int tiles_x = (outsz + kT - 1) / kT;
    const int y0 = (lb.x / tiles_x) * kT, x0 = (lb.x % tiles_x) * kT;
    const int th = min(kT, outsz - y0), tw = min(kT, outsz - x0);
    const uint8_t *src = in + (size_t)img * H * W * 3;
    const int gh = 2 * (th + 2), gw = 2 * (tw + 2);

    lut[tid] = R.gamma_lut[tid];
    if (tid < th + 2) rq[tid] = resize_q(reflect101(y0 - 1 + tid, outsz), crop, outsz);
    if (tid >= 64 && tid - 64 < tw + 2) cq[tid - 64] = resize_q(reflect101(x0 - 1 + tid - 64, outsz), crop, outsz);
    __syncthreads();
    const int64_t a0 = R.aq[0], a1 = R.aq[1], a2 = R.aq[2], a3 = R.aq[3], a4 = R.aq[4], a5 = R.aq[5];
    if (tid < gh) {
        const int Y = R.crop_y + clampi((rq[tid >> 1] >> kFBits) + (tid & 1), crop);
        tyx[tid] = a1 * Y + a2;
        tyy[tid] = a4 * Y + a5;
    }
    if (tid >= 128 && tid - 128 < gw) {
        const int c = tid - 128, X = R.crop_x + clampi((cq[c >> 1] >> kFBits) + (c & 1), crop);
        txx[c] = a0 * X;
        txy[c] = a3 * X;
    }
    __syncthreads();
    // Source box of the taps.  A position is (row term) + (column term) and the
    // rounding is monotone, so its extremes over the tile are the rounded sums
    // of the extreme terms.  The crop lines grow with the pre-blur index except
    // that a halo line reflected at the output border repeats an inner line, so
    // the extreme terms are among the first and last four lines.
    if (tid == 0) {
        int64_t lo[4], hi[4];  // min / max of txx, tyx, txy, tyy
        const int64_t *t[4] = {txx, tyx, txy, tyy};
        const int len[4] = {gw, gh, gw, gh};
        for (int a = 0; a < 4; ++a) {
            lo[a] = hi[a] = t[a][0];
            for (int k = 0; k < 4; ++k) {
                const int64_t u = t[a][k], v = t[a][len[a] - 1 - k];
                lo[a] = min(lo[a], min(u, v));
                hi[a] = max(hi[a], max(u, v));
            }
        }
        const int xmin = (int)(rshr_he64(lo[0] + lo[1], 32 - kFBits) >> kFBits);
        const int xmax = (int)(rshr_he64(hi[0] + hi[1], 32 - kFBits) >> kFBits) + 1;
        const int ymin = (int)(rshr_he64(lo[2] + lo[3], 32 - kFBits) >> kFBits);
        const int ymax = (int)(rshr_he64(hi[2] + hi[3], 32 - kFBits) >> kFBits) + 1;
        const bool inside = xmin >= 0 && xmax <= W - 1 && ymin >= 0 && ymax <= H - 1;
        // a box that crosses the border by less than the image size: stage the
        // range of image pixels its reflected taps read (form 2)
        const bool once = W >= 2 && H >= 2 && xmin >= 1 - W && xmax <= 2 * W - 2 && ymin >= 1 - H && ymax <= 2 * H - 2;
        int xl = xmin, xh = xmax, yl = ymin, yh = ymax;
        if (!inside && once) {
            xl = min(refl1(xmin, W), refl1(xmax, W));
            xh = max(refl1(xmin, W), refl1(xmax, W));
            if (xmin <= 0 && xmax >= 0) xl = 0;
            if (xmin <= W - 1 && xmax >= W - 1) xh = W - 1;
            yl = min(refl1(ymin, H), refl1(ymax, H));
            yh = max(refl1(ymin, H), refl1(ymax, H));
            if (ymin <= 0 && ymax >= 0) yl = 0;
            if (ymin <= H - 1 && ymax >= H - 1) yh = H - 1;
        }
        const int bw = xh - xl + 1, bh = yh - yl + 1;
        const int nch = (3 * bw + 30) >> 4;
        const bool fits = bh <= kMaxRows && bh * nch * 16 <= kStageMax;
        box[0] = xl; box[1] = yl; box[2] = bw; box[3] = bh; box[4] = nch;
        box[5] = fits ? (inside ? 1 : (once ? 2 : 0)) : 0;
    }
    __syncthreads();
    const int bx = box[0], by = box[1], bh = box[3], nch = box[4];
    const int form = box[5];
    const bool staged = form != 0;
    if (staged) {
        const int bw = box[2];
        if (tid < bh) {
            const uint8_t *g = src + ((size_t)(by + tid) * W + bx) * 3;
            rowoff[tid] = 16 * tid * nch + (int)((uintptr_t)g & 15);
        }
        // chunk it of the box: row it / nch, chunk it % nch of that row's 16-byte aligned span
        const int total = bh * nch, lane = tid & 63;
        const float rn = __builtin_amdgcn_rcpf((float)nch);
        for (int base = tid - lane; base < total; base += kThreads) {
            const int it = base + lane;
            const uint8_t *s = nullptr;
            if (it < total) {
                int r = (int)((float)it * rn), ch;
                ch = it - r * nch;
                if (ch < 0) { r -= 1; ch += nch; } else if (ch >= nch) { r += 1; ch -= nch; }
                const uint8_t *g = src + ((size_t)(by + r) * W + bx) * 3;
                if (ch < span_chunks(g, 3 * bw)) s = (const uint8_t *)((uintptr_t)g & ~(uintptr_t)15) + 16 * ch;
            }
            if (s) __builtin_amdgcn_global_load_lds((const void *)s, (lds_ptr_t)(stage + 16 * base), 16, 0, 0);
        }
        __builtin_amdgcn_s_waitcnt(0);  // LDS-DMA writes are counted by vmcnt
    }
    __syncthreads();

    // pre-blur pixels: 2 x 2 warp samples -> resize blend -> HSV shift -> gamma
    for (int e = tid; e < (th + 2) * (tw + 2); e += kThreads) {
        const int pi = e / (tw + 2), pj = e - pi * (tw + 2);
        uint32_t g[2][2];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int r = 2 * pi + u, c = 2 * pj + v;
                const int64_t qx = rshr_he64(txx[c] + tyx[r], 32 - kFBits);
                const int64_t qy = rshr_he64(txy[c] + tyy[r], 32 - kFBits);
                if (form == 1) {
                    const int sx = (int)(qx >> kFBits) - bx, sy = (int)(qy >> kFBits) - by;
                    const int ax = (int)(qx & (kFOne - 1)), ay = (int)(qy & (kFOne - 1));
                    const int o0 = rowoff[sy] + 3 * sx, o1 = rowoff[sy + 1] + 3 * sx;
                    g[u][v] = blend4(lds_rgb(stage, o0), lds_rgb(stage, o0 + 3), lds_rgb(stage, o1),
                                     lds_rgb(stage, o1 + 3), ax, ay);
                } else if (form == 2) {
                    // every tap reflected on its own (a reflected pair need not be adjacent)
                    const int x0 = (int)(qx >> kFBits), y0 = (int)(qy >> kFBits);
                    const int ax = (int)(qx & (kFOne - 1)), ay = (int)(qy & (kFOne - 1));
                    const int c0 = 3 * (refl1(x0, W) - bx), c1 = 3 * (refl1(x0 + 1, W) - bx);
                    const int r0 = rowoff[refl1(y0, H) - by], r1 = rowoff[refl1(y0 + 1, H) - by];
                    g[u][v] = blend4(lds_rgb(stage, r0 + c0), lds_rgb(stage, r0 + c1), lds_rgb(stage, r1 + c0),
                                     lds_rgb(stage, r1 + c1), ax, ay);
                } else {
                    g[u][v] = warp_sample(src, H, W, qx, qy);
                }
            }
        const int wy = rq[pi] & (kFOne - 1), wx = cq[pj] & (kFOne - 1);
        const uint32_t rgb = blend4(g[0][0], g[0][1], g[1][0], g[1][1], wx, wy);
        const uint32_t h = hsv_shift(rgb, R.dh, R.ds, R.dv);
        pre[pi][pj] = (uint32_t)lut[h & 255] | ((uint32_t)lut[(h >> 8) & 255] << 8) | ((uint32_t)lut[(h >> 16) & 255] << 16);
    }
    __syncthreads();

    // blur (or copy) per output pixel into LDS, all three channels at once: a
    // pre-blur word c0 | c1 << 8 | c2 << 16 splits into c0 | c2 << 16 and c1,
    // whose 16-bit lanes take the 3x3 binomial sums (at most 16 x 255) and the
    // round-half-even shift without carrying into each other
    const bool blur = R.blur != 0;
    uint8_t *ob = stage;  // the staged source is no longer read
    for (int e = tid; e < th * tw; e += kThreads) {
        const int r = e / tw, px = e - r * tw;
        uint32_t v;
        if (blur) {
            uint32_t slo = 0, shi = 0;
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
                const uint32_t *q = &pre[r + dy][px];
                const uint32_t lo = (q[0] & 0x00FF00FFu) + 2 * (q[1] & 0x00FF00FFu) + (q[2] & 0x00FF00FFu);
                const uint32_t hi = ((q[0] >> 8) & 0xFFu) + 2 * ((q[1] >> 8) & 0xFFu) + ((q[2] >> 8) & 0xFFu);
                const uint32_t w = dy == 1 ? 2u : 1u;
                slo += w * lo;
                shi += w * hi;
            }
            slo = ((slo + 0x00070007u + ((slo >> 4) & 0x00010001u)) >> 4) & 0x00FF00FFu;
            shi = ((shi + 7u + ((shi >> 4) & 1u)) >> 4) & 0xFFu;
            v = slo | shi << 8;
        } else {
            v = pre[r + 1][px + 1];
        }
        uint8_t *o = ob + r * (kT * 3) + 3 * px;
        o[0] = (uint8_t)v;
        o[1] = (uint8_t)(v >> 8);
        o[2] = (uint8_t)(v >> 16);
    }
    __syncthreads();

    // output rows from LDS, aligned dword stores
    constexpr int kItems = (kT * 3) / 4 + 8;
    for (int it = tid; it < th * kItems; it += kThreads) {
        const int r = it / kItems, j = it - r * kItems;
        uint8_t *g = out + ((size_t)img * outsz * outsz + (size_t)(y0 + r) * outsz + x0) * 3;
        const int len = tw * 3;
        if (j >= span_items(g, len)) continue;
        const uint8_t *orow = ob + r * (kT * 3);
        store_span_item(g, len, j, [&](int b) -> uint8_t { return orow[b]; });
    }
}

// Reflect-101 of a 64-bit index (a strongly shrinking warp can reach far out).
__device__ __forceinline__ int reflect101_64(int64_t i, int n) {
    if (n == 1) return 0;
    const int64_t p = 2 * (int64_t)n - 2;
    i %= p;
    if (i < 0) i += p;
    return (int)(i >= n ? p - i : i);
}

// Masks of the u8 chain: the same geometry with nearest taps and no colour
// ops.  Output (y, x) takes the nearest resize index of the crop (source
// index (q + 512) >> 10 of the Q10 position, clamped into the crop), shifts
// it by the crop offset and samples the warped mask there: nearest tap of the
// Q32 inverse map rounded to Q10, reflect-101.  One thread per output pixel.
__global__ __launch_bounds__(kThreads) void k_c2_mask(const uint8_t *__restrict__ in, int H, int W,
                                                      const miaug_c2_record *__restrict__ rec, int crop, int outsz,
                                                      uint8_t *__restrict__ out) {
    const int img = blockIdx.y;
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= outsz * outsz) return;
    const int y = e / outsz, x = e - y * outsz;
    const miaug_c2_record &r = rec[img];
    const int ny = min(max((resize_q(y, crop, outsz) + kFOne / 2) >> kFBits, 0), crop - 1) + r.crop_y;
    const int nx = min(max((resize_q(x, crop, outsz) + kFOne / 2) >> kFBits, 0), crop - 1) + r.crop_x;
    const int64_t qx = rshr_he64(r.aq[0] * nx + r.aq[1] * ny + r.aq[2], 32 - kFBits);
    const int64_t qy = rshr_he64(r.aq[3] * nx + r.aq[4] * ny + r.aq[5], 32 - kFBits);
    const int64_t ix = (qx + kFOne / 2) >> kFBits, iy = (qy + kFOne / 2) >> kFBits;
    const int sx = reflect101_64(ix, W), sy = reflect101_64(iy, H);
    out[(size_t)img * outsz * outsz + e] = in[(size_t)img * H * W + (size_t)sy * W + sx];
}

// Boxes of the u8 chain: the forward map of the warp (the inverse of the
// record's Q32 matrix, in double) takes each corner u of a box (continuous
// coordinates, pixel i spans [i, i + 1)) as the index position u - 1/2 to
// F(u - 1/2) + 1/2; the box becomes the bounding box of its four corners,
// clipped to the image, then shifted by the crop offset, clipped to the crop
// and scaled by outsz / crop.  One workgroup per image, a thread per box.
__global__ __launch_bounds__(64) void k_c2_boxes(const float *__restrict__ boxes, const int32_t *__restrict__ box_off,
                                                 int H, int W, const miaug_c2_record *__restrict__ rec, int crop,
                                                 int outsz, float *__restrict__ out) {
    const int img = blockIdx.x;
    const miaug_c2_record &r = rec[img];
    const double q = 4294967296.0;
    const double a0 = r.aq[0] / q, a1 = r.aq[1] / q, a2 = r.aq[2] / q;
    const double a3 = r.aq[3] / q, a4 = r.aq[4] / q, a5 = r.aq[5] / q;
    const double det = a0 * a4 - a1 * a3;
    const double i00 = a4 / det, i01 = -a1 / det, i10 = -a3 / det, i11 = a0 / det;
    const double k = (double)outsz / crop;
    for (int b = box_off[img] + (int)threadIdx.x; b < box_off[img + 1]; b += 64) {
        const float *bx = boxes + 4 * (size_t)b;
        double x1 = 1e300, y1 = 1e300, x2 = -1e300, y2 = -1e300;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double px = (double)bx[(c & 1) ? 2 : 0] - 0.5 - a2, py = (double)bx[(c & 2) ? 3 : 1] - 0.5 - a5;
            const double ox = i00 * px + i01 * py + 0.5, oy = i10 * px + i11 * py + 0.5;
            x1 = fmin(x1, ox); x2 = fmax(x2, ox);
            y1 = fmin(y1, oy); y2 = fmax(y2, oy);
        }
        x1 = fmin(fmax(x1, 0.0), (double)W); x2 = fmin(fmax(x2, 0.0), (double)W);
        y1 = fmin(fmax(y1, 0.0), (double)H); y2 = fmin(fmax(y2, 0.0), (double)H);
        x1 = fmin(fmax(x1 - r.crop_x, 0.0), (double)crop); x2 = fmin(fmax(x2 - r.crop_x, 0.0), (double)crop);
        y1 = fmin(fmax(y1 - r.crop_y, 0.0), (double)crop); y2 = fmin(fmax(y2 - r.crop_y, 0.0), (double)crop);
        float *o = out + 4 * (size_t)b;
        o[0] = (float)(x1 * k);
        o[1] = (float)(y1 * k);
        o[2] = (float)(x2 * k);
        o[3] = (float)(y2 * k);
    }
}

// Standalone ShiftHSV (Table I): the chain's HSV step on a dense RGB batch.
// A lane takes four pixels (12 bytes, three dwords) when every image's bytes
// and the pointers are dword-aligned, else one pixel in bytes.
__global__ __launch_bounds__(256) void k_hsv_u8(const uint8_t *__restrict__ in, int64_t npx,
                                                const int32_t *__restrict__ dhsv, bool quads,
                                                uint8_t *__restrict__ out) {
    const int img = blockIdx.y;
    const int dh = dhsv[3 * img], ds = dhsv[3 * img + 1], dv = dhsv[3 * img + 2];
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const uint8_t *src = in + (size_t)img * npx * 3;
    uint8_t *dst = out + (size_t)img * npx * 3;
    if (quads) {
        if (4 * q + 3 < npx) {
            const uint32_t *w = (const uint32_t *)(src + 12 * q);
            const uint32_t w0 = w[0], w1 = w[1], w2 = w[2];
            const uint32_t o0 = hsv_shift(w0 & 0xFFFFFFu, dh, ds, dv);
            const uint32_t o1 = hsv_shift((w0 >> 24) | ((w1 & 0xFFFFu) << 8), dh, ds, dv);
            const uint32_t o2 = hsv_shift((w1 >> 16) | ((w2 & 0xFFu) << 16), dh, ds, dv);
            const uint32_t o3 = hsv_shift(w2 >> 8, dh, ds, dv);
            uint32_t *o = (uint32_t *)(dst + 12 * q);
            o[0] = o0 | (o1 << 24);
            o[1] = (o1 >> 8) | (o2 << 16);
            o[2] = (o2 >> 16) | (o3 << 8);
            return;
        }
        for (int64_t p = 4 * q; p < npx && p < 4 * q + 4; ++p) {  // the tail of an image
            const uint8_t *a = src + 3 * p;
            const uint32_t o = hsv_shift(a[0] | (a[1] << 8) | (a[2] << 16), dh, ds, dv);
            dst[3 * p] = o & 255;
            dst[3 * p + 1] = (o >> 8) & 255;
            dst[3 * p + 2] = o >> 16;
        }
        return;
    }
    if (q >= npx) return;
    const uint8_t *a = src + 3 * q;
    const uint32_t o = hsv_shift(a[0] | (a[1] << 8) | (a[2] << 16), dh, ds, dv);
    dst[3 * q] = o & 255;
    dst[3 * q + 1] = (o >> 8) & 255;
    dst[3 * q + 2] = o >> 16;
}

}  // namespace

hipError_t launch_c2_mask(const uint8_t *in, int n, int H, int W, const miaug_c2_record *rec, int crop, int outsz,
                          uint8_t *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_c2_mask, dim3((outsz * outsz + kThreads - 1) / kThreads, n), dim3(kThreads), 0, s, in, H, W,
                       rec, crop, outsz, out);
    return hipGetLastError();
}

hipError_t launch_c2_boxes(const float *boxes, const int32_t *box_off, int n, int H, int W,
                           const miaug_c2_record *rec, int crop, int outsz, float *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_c2_boxes, dim3(n), dim3(64), 0, s, boxes, box_off, H, W, rec, crop, outsz, out);
    return hipGetLastError();
}

hipError_t launch_c2(const uint8_t *in, int n, int H, int W, const miaug_c2_record *rec, int crop, int outsz,
                     uint8_t *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int t = (outsz + kT - 1) / kT;
    hipLaunchKernelGGL(k_c2, dim3(t * t, n), dim3(kThreads), 0, s, in, H, W, rec, crop, outsz, out);
    return hipGetLastError();
}

hipError_t launch_hsv_u8(const uint8_t *in, int n, int H, int W, const int32_t *dhsv, uint8_t *out, hipStream_t s) {
    if (n == 0 || H == 0 || W == 0) return hipSuccess;
    const int64_t npx = (int64_t)H * W;
    const bool quads = ((uintptr_t)in & 3) == 0 && ((uintptr_t)out & 3) == 0 && (npx & 3) == 0;
    const int64_t lanes = quads ? (npx + 3) / 4 : npx;
    dim3 grid((unsigned)((lanes + 255) / 256), n);
    hipLaunchKernelGGL(k_hsv_u8, grid, dim3(256), 0, s, in, npx, dhsv, quads, out);
    return hipGetLastError();
}

}  // namespace miaug
