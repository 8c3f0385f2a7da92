// k_c2.hip -- full u8 pipeline in one pass per output tile: shift-scale-rotate
// warp (bilinear, reflect-101) -> crop -> bilinear resize -> integer HSV shift
// -> gamma LUT -> 3x3 binomial blur (Table I ShiftScaleRotate, RandomCrop64,
// ShiftHSV, Gamma; Sec. II colour transforms).
//
// One workgroup per (image, T x T output tile).  The blur needs the pre-blur
// values of a 1-pixel halo, and the resize needs two warp samples per output
// line along each axis, so the tile evaluates, in LDS:
//   1. the resize positions of its (T+2) rows and columns (halo rows/columns
//      reflected at the image border, as the blur reads them);
//   2. the warp samples on the grid of the 2(T+2) x 2(T+2) crop lines those
//      positions touch (each sample: Q32 affine position -> 4 taps -> u8);
//   3. the (T+2)^2 pre-blur pixels: resize blend -> u8 -> HSV8 -> gamma LUT;
//   4. the output: 3x3 blur (or copy) written as aligned dwords.
// Every intermediate is rounded exactly as the sequential definition rounds
// it; only the order of evaluation differs.
#include "dev_common.h"
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
    uint32_t out = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int a00 = (p00 >> (8 * c)) & 255, a01 = (p01 >> (8 * c)) & 255;
        const int a10 = (p10 >> (8 * c)) & 255, a11 = (p11 >> (8 * c)) & 255;
        const int t0 = (a00 << kFBits) + ax * (a01 - a00);
        const int t1 = (a10 << kFBits) + ax * (a11 - a10);
        const int acc = (t0 << kFBits) + ay * (t1 - t0);
        out |= (uint32_t)((acc + 0x7FFFF + ((acc >> 20) & 1)) >> 20) << (8 * c);
    }
    return out;
}

// Integer hexcone HSV shift of one RGB pixel (packed R | G<<8 | B<<16).
__device__ __forceinline__ uint32_t hsv_shift(uint32_t rgb, int dh, int ds, int dv) {
    const int R = rgb & 255, G = (rgb >> 8) & 255, B = (rgb >> 16) & 255;
    const int V = max(R, max(G, B)), m = min(R, min(G, B)), C = V - m;
    const int S8 = V ? (int)udiv_he(255u * (uint32_t)C, (uint32_t)V) : 0;
    int h = 0;
    if (C != 0) {
        if (V == R) h = sdiv_he(30 * (G - B), C);
        else if (V == G) h = 60 + sdiv_he(30 * (B - R), C);
        else h = 120 + sdiv_he(30 * (R - G), C);
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

__global__ __launch_bounds__(kThreads) void k_c2(const uint8_t *__restrict__ in, int H, int W,
                                                 const miaug_c2_record *__restrict__ recs, int crop, int outsz,
                                                 uint8_t *__restrict__ out) {
    __shared__ uint32_t grid[kG][kG];
    __shared__ uint32_t pre[kP][kP];
    __shared__ int32_t rq[kP], cq[kP];
    __shared__ uint8_t lut[256];

    const int img = blockIdx.y, tid = threadIdx.x;
    const miaug_c2_record &R = recs[img];
    const int tiles_x = (outsz + kT - 1) / kT;
    const int y0 = (blockIdx.x / tiles_x) * kT, x0 = (blockIdx.x % tiles_x) * kT;
    const int th = min(kT, outsz - y0), tw = min(kT, outsz - x0);
    const uint8_t *src = in + (size_t)img * H * W * 3;

    lut[tid] = R.gamma_lut[tid];
    if (tid < th + 2) rq[tid] = resize_q(reflect101(y0 - 1 + tid, outsz), crop, outsz);
    if (tid >= 64 && tid - 64 < tw + 2) cq[tid - 64] = resize_q(reflect101(x0 - 1 + tid - 64, outsz), crop, outsz);
    __syncthreads();

    // warp samples on the crop lines the resize taps touch
    const int64_t a0 = R.aq[0], a1 = R.aq[1], a2 = R.aq[2], a3 = R.aq[3], a4 = R.aq[4], a5 = R.aq[5];
    const int gh = 2 * (th + 2), gw = 2 * (tw + 2);
    for (int e = tid; e < gh * gw; e += kThreads) {
        const int gi = e / gw, gj = e - gi * gw;
        const int Y = R.crop_y + clampi((rq[gi >> 1] >> kFBits) + (gi & 1), crop);
        const int X = R.crop_x + clampi((cq[gj >> 1] >> kFBits) + (gj & 1), crop);
        const int64_t qx = rshr_he64(a0 * X + a1 * Y + a2, 32 - kFBits);
        const int64_t qy = rshr_he64(a3 * X + a4 * Y + a5, 32 - kFBits);
        grid[gi][gj] = warp_sample(src, H, W, qx, qy);
    }
    __syncthreads();

    // pre-blur pixels: resize blend -> HSV shift -> gamma
    for (int e = tid; e < (th + 2) * (tw + 2); e += kThreads) {
        const int pi = e / (tw + 2), pj = e - pi * (tw + 2);
        const int wy = rq[pi] & (kFOne - 1), wx = cq[pj] & (kFOne - 1);
        const uint32_t g00 = grid[2 * pi][2 * pj], g01 = grid[2 * pi][2 * pj + 1];
        const uint32_t g10 = grid[2 * pi + 1][2 * pj], g11 = grid[2 * pi + 1][2 * pj + 1];
        uint32_t rgb = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int b00 = (g00 >> (8 * c)) & 255, b01 = (g01 >> (8 * c)) & 255;
            const int b10 = (g10 >> (8 * c)) & 255, b11 = (g11 >> (8 * c)) & 255;
            const int t0 = (b00 << kFBits) + wx * (b01 - b00);
            const int t1 = (b10 << kFBits) + wx * (b11 - b10);
            const int acc = (t0 << kFBits) + wy * (t1 - t0);
            rgb |= (uint32_t)((acc + 0x7FFFF + ((acc >> 20) & 1)) >> 20) << (8 * c);
        }
        const uint32_t h = hsv_shift(rgb, R.dh, R.ds, R.dv);
        pre[pi][pj] = (uint32_t)lut[h & 255] | ((uint32_t)lut[(h >> 8) & 255] << 8) | ((uint32_t)lut[(h >> 16) & 255] << 16);
    }
    __syncthreads();

    // output rows: blur (or copy) from the pre-blur tile, aligned dword stores
    const bool blur = R.blur != 0;
    constexpr int kItems = (kT * 3) / 4 + 8;
    for (int it = tid; it < th * kItems; it += kThreads) {
        const int r = it / kItems, j = it - r * kItems;
        uint8_t *g = out + ((size_t)img * outsz * outsz + (size_t)(y0 + r) * outsz + x0) * 3;
        const int len = tw * 3;
        if (j >= span_items(g, len)) continue;
        auto byte_at = [&](int b) -> uint8_t {
            const int px = b / 3, c = b - 3 * px, sh = 8 * c;
            if (!blur) return (uint8_t)(pre[r + 1][px + 1] >> sh);
            const uint32_t *u = &pre[r][px], *m = &pre[r + 1][px], *d = &pre[r + 2][px];
            const int s = (int)((u[0] >> sh) & 255) + 2 * (int)((u[1] >> sh) & 255) + (int)((u[2] >> sh) & 255) +
                          2 * ((int)((m[0] >> sh) & 255) + 2 * (int)((m[1] >> sh) & 255) + (int)((m[2] >> sh) & 255)) +
                          (int)((d[0] >> sh) & 255) + 2 * (int)((d[1] >> sh) & 255) + (int)((d[2] >> sh) & 255);
            return (uint8_t)((s + 7 + ((s >> 4) & 1)) >> 4);
        };
        store_span_item(g, len, j, byte_at);
    }
}

}  // namespace

hipError_t launch_c2(const uint8_t *in, int n, int H, int W, const miaug_c2_record *rec, int crop, int outsz,
                     uint8_t *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int t = (outsz + kT - 1) / kT;
    hipLaunchKernelGGL(k_c2, dim3(t * t, n), dim3(kThreads), 0, s, in, H, W, rec, crop, outsz, out);
    return hipGetLastError();
}

}  // namespace miaug
