// k_padwarp.hip -- the remaining geometric rows of Table I as single ops on a
// dense u8 batch: PadToSize (identity map plus a border) and a standalone
// affine warp (Rotate; ShiftScaleRotate without crop or resize), both with a
// reflect-101 or constant border.  The pad takes four pixels of four output
// rows per thread (no reuse to stage); the warp stages each output tile's
// source box in LDS.
#include "dev_common.h"
#include "internal.h"

namespace miaug {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int64_t reflect101_64(int64_t i, int64_t n) {
    if (n == 1) return 0;
    const int64_t p = 2 * n - 2;
    i %= p;
    if (i < 0) i += p;
    return i >= n ? p - i : i;
}

// Source index of a tap, or -1 for the constant border outside the image.
// Indices within one reflection of the image take the reflection directly;
// only farther ones need the period.
__device__ __forceinline__ int64_t border_index(int64_t i, int n, int border) {
    if (i >= 0 && i < n) return i;
    if (border == MIAUG_BORDER_CONSTANT) return -1;
    if (n > 1 && i < 0 && i > -n) return -i;
    if (n > 1 && i >= n && i < 2 * (int64_t)n - 1) return 2 * (int64_t)n - 2 - i;
    return reflect101_64(i, n);
}

constexpr int kPadThreads = 128;  // k_pad: 512 output pixels of a row per block and step
constexpr int kPadRows = 4;       // output rows per block: their loads are in flight together

template <int C>
__global__ __launch_bounds__(kPadThreads) void k_pad(const uint8_t *__restrict__ in, int H, int W, int Ho, int Wo,
                                                     int top, int left, int border, int value,
                                                     uint8_t *__restrict__ out) {
    // block (image, group of kPadRows output rows, column block): four pixels
    // of each row per thread, every row's source words loaded before any is stored
    const int groups = (Ho + kPadRows - 1) / kPadRows;
    const int img = (int)(blockIdx.x / (unsigned)groups), y0 = (int)(blockIdx.x - (unsigned)img * groups) * kPadRows;
    int64_t sy[kPadRows];  // source row of each output row (the same for the whole block), -1: constant
#pragma unroll
    for (int r = 0; r < kPadRows; ++r) sy[r] = y0 + r < Ho ? border_index(y0 + r - top, H, border) : -1;
    for (int xb = blockIdx.y; (int64_t)xb * 4 * kPadThreads < Wo; xb += gridDim.y) {
        const int x = (xb * kPadThreads + (int)threadIdx.x) * 4;
        if (x >= Wo) break;
        const int sx0 = x - left, np = min(4, Wo - x);
        const bool cols = np == 4 && sx0 >= 0 && sx0 + 4 <= W;
        uint32_t d[kPadRows][C + 1];
        bool fast[kPadRows];
        int sh[kPadRows];
#pragma unroll
        for (int r = 0; r < kPadRows; ++r) {
            uint8_t *o = out + (((size_t)img * Ho + y0 + r) * Wo + x) * C;
            // four contiguous source pixels: C words (C + 1 when they do not start on
            // a word, the last one holding their last bytes), shifted into C output words
            fast[r] = cols && sy[r] >= 0 && ((uintptr_t)o & 3) == 0;
            sh[r] = 0;
#pragma unroll
            for (int k = 0; k <= C; ++k) d[r][k] = 0u;
            if (fast[r]) {  // only then are the words inside the source row
                const uint8_t *p = in + (((size_t)img * H + sy[r]) * W + sx0) * C;
                sh[r] = (int)((uintptr_t)p & 3);
                const uint32_t *w = (const uint32_t *)(p - sh[r]);
#pragma unroll
                for (int k = 0; k < C; ++k) d[r][k] = w[k];
                if (sh[r]) d[r][C] = w[C];
            }
        }
#pragma unroll
        for (int r = 0; r < kPadRows; ++r) {
            if (y0 + r >= Ho) break;
            uint8_t *o = out + (((size_t)img * Ho + y0 + r) * Wo + x) * C;
            if (fast[r]) {
#pragma unroll
                for (int k = 0; k < C; ++k) ((uint32_t *)o)[k] = __builtin_amdgcn_alignbyte(d[r][k + 1], d[r][k], sh[r]);
                continue;
            }
            const uint8_t *srow = in + ((size_t)img * H + (sy[r] < 0 ? 0 : sy[r])) * W * C;
            for (int j = 0; j < np; ++j) {
                const int64_t sx = border_index(sx0 + j, W, border);
#pragma unroll
                for (int c = 0; c < C; ++c) o[j * C + c] = (sy[r] < 0 || sx < 0) ? (uint8_t)value : srow[sx * C + c];
            }
        }
    }
}

// Output (x, y) samples the source at the Q10 position rshr_he(A (x, y, 1), 22)
// of the record's Q32 inverse matrix A: bilinear (weights (1024 - a, a), one
// round-half-even of the 2^20-scaled sum) or nearest ((q + 512) >> 10).
__device__ __forceinline__ void warp_pos(const int64_t *a, int x, int y, int64_t &qx, int64_t &qy) {
    qx = rshr_he64(a[0] * x + a[1] * y + a[2], 32 - kFBits);
    qy = rshr_he64(a[3] * x + a[4] * y + a[5], 32 - kFBits);
}

// Bilinear value of one channel from four taps (the blend of the u8 chain).
__device__ __forceinline__ uint8_t blend4(int v00, int v01, int v10, int v11, int ax, int ay) {
    const int t0 = (v00 << kFBits) + ax * (v01 - v00);
    const int t1 = (v10 << kFBits) + ax * (v11 - v10);
    const int acc = (t0 << kFBits) + ay * (t1 - t0);
    return (uint8_t)((acc + 0x7FFFF + ((acc >> 20) & 1)) >> 20);
}

// One output pixel straight from global memory (tiles whose source box does
// not fit the stage).
template <int C>
__device__ __forceinline__ void warp_px_direct(const uint8_t *src, int H, int W, const int64_t *a, int interp,
                                               int border, int x, int y, uint8_t *o) {
    int64_t qx, qy;
    warp_pos(a, x, y, qx, qy);
    if (interp == MIAUG_INTERP_NEAREST) {
        const int64_t sy = border_index((qy + kFOne / 2) >> kFBits, H, border);
        const int64_t sx = border_index((qx + kFOne / 2) >> kFBits, W, border);
#pragma unroll
        for (int c = 0; c < C; ++c) o[c] = (sy < 0 || sx < 0) ? 0 : src[((size_t)sy * W + sx) * C + c];
        return;
    }
    const int64_t x0 = qx >> kFBits, y0 = qy >> kFBits;
    const int ax = (int)(qx & (kFOne - 1)), ay = (int)(qy & (kFOne - 1));
    const int64_t xs[2] = {border_index(x0, W, border), border_index(x0 + 1, W, border)};
    const int64_t ys[2] = {border_index(y0, H, border), border_index(y0 + 1, H, border)};
#pragma unroll
    for (int c = 0; c < C; ++c) {
        int v[2][2];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int i = 0; i < 2; ++i)
                v[j][i] = (ys[j] < 0 || xs[i] < 0) ? 0 : src[((size_t)ys[j] * W + xs[i]) * C + c];
        o[c] = blend4(v[0][0], v[0][1], v[1][0], v[1][1], ax, ay);
    }
}

typedef __attribute__((address_space(3))) void *lds_ptr_t;

constexpr int kWarpTile = 32;            // output tile side
constexpr int kWarpStage = 16 * 1024;    // bytes of staged source box per workgroup
constexpr int kWarpRows = 128;           // rows of a box staged in dwords

// floor(e / d) for 0 <= e < 2^20, 1 <= d < 2^12, from a float estimate and
// one correction each way.
__device__ __forceinline__ int small_div(int e, int d, float rd) {
    int q = (int)((float)e * rd);
    if (q * d > e) --q;
    else if ((q + 1) * d <= e) ++q;
    return q;
}

// One workgroup per 32 x 32 output tile.  The affine map is monotone along
// every line, so every tap of the tile lies in the box spanned by the Q10
// positions of its four corners (floor, plus one for the second bilinear tap);
// that box is staged in LDS with the border rule applied per staged pixel
// (reflect-101 index or the constant 0), and the taps read LDS in the box's
// own coordinates.  A box larger than the stage (a strong zoom-out) takes the
// direct path.
template <int C>
__global__ __launch_bounds__(kThreads) void k_warp(const uint8_t *__restrict__ in, int H, int W,
                                                   const int64_t *__restrict__ aq, int interp, int border,
                                                   uint8_t *__restrict__ out) {
    __shared__ __align__(16) uint8_t box[kWarpStage];
    __shared__ int roff[kWarpRows];
    __shared__ __align__(4) uint8_t obuf[kWarpTile * kWarpTile * C];
    const int2 lb = xcd_block();  // (output tile, image): an image's tiles share one XCD's L2
    const int img = lb.y;
    const int ntx = (W + kWarpTile - 1) / kWarpTile;
    const int tx0 = (lb.x % ntx) * kWarpTile, ty0 = (lb.x / ntx) * kWarpTile;
    const int tw = min(kWarpTile, W - tx0), th = min(kWarpTile, H - ty0);
    int64_t a[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) a[k] = aq[6 * img + k];
    const uint8_t *src = in + (size_t)img * H * W * C;
    uint8_t *dst = out + (size_t)img * H * W * C;
    // source box of the tile's taps
    int64_t qx[4], qy[4];
    warp_pos(a, tx0, ty0, qx[0], qy[0]);
    warp_pos(a, tx0 + tw - 1, ty0, qx[1], qy[1]);
    warp_pos(a, tx0, ty0 + th - 1, qx[2], qy[2]);
    warp_pos(a, tx0 + tw - 1, ty0 + th - 1, qx[3], qy[3]);
    int64_t xlo = qx[0], xhi = qx[0], ylo = qy[0], yhi = qy[0];
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        xlo = min(xlo, qx[k]); xhi = max(xhi, qx[k]);
        ylo = min(ylo, qy[k]); yhi = max(yhi, qy[k]);
    }
    const int64_t bx0 = xlo >> kFBits, by0 = ylo >> kFBits;
    const int64_t bw64 = (xhi >> kFBits) + 2 - bx0, bh64 = (yhi >> kFBits) + 2 - by0;
    if (bw64 > kWarpStage || bh64 > kWarpStage || bw64 * bh64 * C > kWarpStage) {  // sides first: no overflow
        for (int p = threadIdx.x; p < tw * th; p += kThreads) {
            const int y = ty0 + p / tw, x = tx0 + p % tw;
            warp_px_direct<C>(src, H, W, a, interp, border, x, y, dst + ((size_t)y * W + x) * C);
        }
        return;
    }
    const int bw = (int)bw64, bh = (int)bh64;
    // A box inside the image is staged in dwords: row r's bytes start at the
    // dword boundary below them (offset o_r = its byte address mod 4) in a row
    // of pitch P; roff[r] = r P + o_r.  Needs a 4-aligned image, and the last
    // row's dwords inside the image.  Other boxes go pixel by pixel with the
    // border rule.
    const int nd = (bw * C + 6) / 4, P = 4 * nd;
    const bool dw = ((uintptr_t)src & 3) == 0 && bx0 >= 0 && by0 >= 0 && bx0 + bw <= W && by0 + bh <= H &&
                    bh <= kWarpRows && bh * P <= kWarpStage &&
                    ((by0 + bh - 1) * (int64_t)W + bx0) * C + P <= (int64_t)H * W * C;
    if (dw) {
        if ((int)threadIdx.x < bh) roff[threadIdx.x] = threadIdx.x * P + (int)(((by0 + threadIdx.x) * W + bx0) * C & 3);
        // dword e = r nd + j of the box lands at box + 4 e: the LDS-DMA's
        // lane-ordered destinations, every dword of a thread in flight at once
        const float rnd = 1.0f / (float)nd;
        const int lane = threadIdx.x & 63;
        for (int b = threadIdx.x - lane; b < bh * nd; b += kThreads) {  // b is uniform in the wave
            const int e = b + lane;
            if (e < bh * nd) {
                const int r = small_div(e, nd, rnd), j = e - r * nd;
                const size_t g4 = (size_t)(((by0 + r) * W + bx0) * C) & ~(size_t)3;
                __builtin_amdgcn_global_load_lds((const void *)(src + g4 + 4 * j), (lds_ptr_t)(box + 4 * b), 4, 0, 0);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);  // LDS-DMA writes are counted by vmcnt
    } else {
        // pixel by pixel with the border rule, kBatch pixels of a thread loaded
        // before any is stored (their loads in flight together)
        constexpr int kBatch = 4;
        const float rbw = 1.0f / (float)bw;
        for (int e0 = threadIdx.x; e0 < bw * bh; e0 += kBatch * kThreads) {
            uint8_t v[kBatch][C];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int e = e0 + u * kThreads;
                const int r = small_div(min(e, bw * bh - 1), bw, rbw), c = min(e, bw * bh - 1) - r * bw;
                const int64_t sy = border_index(by0 + r, H, border), sx = border_index(bx0 + c, W, border);
                const bool in = sy >= 0 && sx >= 0;
                const uint8_t *p = src + (in ? ((size_t)sy * W + sx) * C : 0);
#pragma unroll
                for (int ch = 0; ch < C; ++ch) v[u][ch] = in ? p[ch] : 0;
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int e = e0 + u * kThreads;
                if (e < bw * bh)
#pragma unroll
                    for (int ch = 0; ch < C; ++ch) box[e * C + ch] = v[u][ch];
            }
        }
    }
    __syncthreads();
    // lane (lx, ly0) takes pixels (lx, ly0 + 8 k): the Q32 sums step by 8 a1 / 8 a4
    constexpr int kRows = kThreads / kWarpTile;
    const int lx = threadIdx.x % kWarpTile, ly0 = threadIdx.x / kWarpTile;
    int64_t sxq = a[0] * (tx0 + lx) + a[1] * (ty0 + ly0) + a[2];
    int64_t syq = a[3] * (tx0 + lx) + a[4] * (ty0 + ly0) + a[5];
    const int64_t dx = a[1] * kRows, dy = a[4] * kRows;
#pragma unroll
    for (int k = 0; k < kWarpTile / kRows; ++k, sxq += dx, syq += dy) {
        const int ly = ly0 + kRows * k;
        if (ly >= th || lx >= tw) continue;  // outside the image: taps outside the box; never copied out
        uint8_t *o = obuf + (ly * kWarpTile + lx) * C;
        const int64_t px = rshr_he64(sxq, 32 - kFBits), py = rshr_he64(syq, 32 - kFBits);
        if (interp == MIAUG_INTERP_NEAREST) {
            const int sx = (int)(((px + kFOne / 2) >> kFBits) - bx0), sy = (int)(((py + kFOne / 2) >> kFBits) - by0);
            const uint8_t *b = box + (dw ? roff[sy] : sy * bw * C) + sx * C;
#pragma unroll
            for (int c = 0; c < C; ++c) o[c] = b[c];
            continue;
        }
        const int sx = (int)((px >> kFBits) - bx0), sy = (int)((py >> kFBits) - by0);
        const int ax = (int)(px & (kFOne - 1)), ay = (int)(py & (kFOne - 1));
        const uint8_t *b0 = box + (dw ? roff[sy] : sy * bw * C) + sx * C;
        const uint8_t *b1 = box + (dw ? roff[sy + 1] : (sy + 1) * bw * C) + sx * C;
#pragma unroll
        for (int c = 0; c < C; ++c) o[c] = blend4(b0[c], b0[C + c], b1[c], b1[C + c], ax, ay);
    }
    __syncthreads();
    // the tile's rows out of LDS: dwords when rows are 4-byte aligned, else bytes
    const int rb = tw * C;
    if ((((uintptr_t)dst + ((size_t)ty0 * W + tx0) * C) & 3) == 0 && ((W * C) & 3) == 0 && (rb & 3) == 0) {
        const int nd = rb / 4;
        for (int e = threadIdx.x; e < nd * th; e += kThreads) {
            const int r = e / nd, d = e - r * nd;
            *(uint32_t *)(dst + ((size_t)(ty0 + r) * W + tx0) * C + 4 * d) =
                *(const uint32_t *)(obuf + r * kWarpTile * C + 4 * d);
        }
    } else {
        for (int e = threadIdx.x; e < rb * th; e += kThreads) {
            const int r = e / rb, d = e - r * rb;
            dst[((size_t)(ty0 + r) * W + tx0) * C + d] = obuf[r * kWarpTile * C + d];
        }
    }
}

}  // namespace

hipError_t launch_pad_u8(const uint8_t *in, int n, int H, int W, int C, int Ho, int Wo, int border, int value,
                         uint8_t *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int top = (Ho - H) / 2, left = (Wo - W) / 2;
    const int64_t cb = ((int64_t)Wo + 4 * kPadThreads - 1) / (4 * kPadThreads);
    dim3 grid((unsigned)((int64_t)((Ho + kPadRows - 1) / kPadRows) * n), (unsigned)(cb < 65535 ? cb : 65535));
    if (C == 1) hipLaunchKernelGGL(k_pad<1>, grid, dim3(kPadThreads), 0, s, in, H, W, Ho, Wo, top, left, border, value, out);
    else if (C == 3) hipLaunchKernelGGL(k_pad<3>, grid, dim3(kPadThreads), 0, s, in, H, W, Ho, Wo, top, left, border, value, out);
    else hipLaunchKernelGGL(k_pad<4>, grid, dim3(kPadThreads), 0, s, in, H, W, Ho, Wo, top, left, border, value, out);
    return hipGetLastError();
}

hipError_t launch_warp_u8(const uint8_t *in, int n, int H, int W, int C, const int64_t *aq, int interp, int border,
                          uint8_t *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    dim3 grid((unsigned)(((W + kWarpTile - 1) / kWarpTile) * ((H + kWarpTile - 1) / kWarpTile)), n);
    if (C == 1) hipLaunchKernelGGL(k_warp<1>, grid, dim3(kThreads), 0, s, in, H, W, aq, interp, border, out);
    else if (C == 3) hipLaunchKernelGGL(k_warp<3>, grid, dim3(kThreads), 0, s, in, H, W, aq, interp, border, out);
    else hipLaunchKernelGGL(k_warp<4>, grid, dim3(kThreads), 0, s, in, H, W, aq, interp, border, out);
    return hipGetLastError();
}

}  // namespace miaug
