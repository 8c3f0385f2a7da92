// k_padwarp.hip -- the remaining geometric rows of Table I as single ops on a
// dense u8 batch: PadToSize (identity map plus a border) and a standalone
// affine warp (Rotate; ShiftScaleRotate without crop or resize), both with a
// reflect-101 or constant border.  One thread per output pixel: these ops
// move C bytes per pixel and have no reuse to stage.
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
__device__ __forceinline__ int64_t border_index(int64_t i, int n, int border) {
    if (i >= 0 && i < n) return i;
    return border == MIAUG_BORDER_CONSTANT ? -1 : reflect101_64(i, n);
}

template <int C>
__global__ __launch_bounds__(kThreads) void k_pad(const uint8_t *__restrict__ in, int H, int W, int Ho, int Wo,
                                                  int top, int left, int border, int value,
                                                  uint8_t *__restrict__ out) {
    const int img = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= (int64_t)Ho * Wo) return;
    const int y = (int)(e / Wo), x = (int)(e - (int64_t)y * Wo);
    const int64_t sy = border_index(y - top, H, border), sx = border_index(x - left, W, border);
    const uint8_t *p = in + (size_t)img * H * W * C + ((size_t)sy * W + sx) * C;
    uint8_t *o = out + (size_t)img * Ho * Wo * C + (size_t)e * C;
#pragma unroll
    for (int c = 0; c < C; ++c) o[c] = (sy < 0 || sx < 0) ? (uint8_t)value : p[c];
}

// Output (x, y) samples the source at the Q10 position rshr_he(A (x, y, 1), 22)
// of the record's Q32 inverse matrix A: bilinear (weights (1024 - a, a), one
// round-half-even of the 2^20-scaled sum) or nearest ((q + 512) >> 10).
template <int C>
__global__ __launch_bounds__(kThreads) void k_warp(const uint8_t *__restrict__ in, int H, int W,
                                                   const int64_t *__restrict__ aq, int interp, int border,
                                                   uint8_t *__restrict__ out) {
    const int img = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= (int64_t)H * W) return;
    const int y = (int)(e / W), x = (int)(e - (int64_t)y * W);
    const int64_t *a = aq + 6 * img;
    const int64_t qx = rshr_he64(a[0] * x + a[1] * y + a[2], 32 - kFBits);
    const int64_t qy = rshr_he64(a[3] * x + a[4] * y + a[5], 32 - kFBits);
    const uint8_t *src = in + (size_t)img * H * W * C;
    uint8_t *o = out + (size_t)img * H * W * C + (size_t)e * C;
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
        const int t0 = (v[0][0] << kFBits) + ax * (v[0][1] - v[0][0]);
        const int t1 = (v[1][0] << kFBits) + ax * (v[1][1] - v[1][0]);
        const int acc = (t0 << kFBits) + ay * (t1 - t0);
        o[c] = (uint8_t)((acc + 0x7FFFF + ((acc >> 20) & 1)) >> 20);
    }
}

}  // namespace

hipError_t launch_pad_u8(const uint8_t *in, int n, int H, int W, int C, int Ho, int Wo, int border, int value,
                         uint8_t *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int top = (Ho - H) / 2, left = (Wo - W) / 2;
    dim3 grid((unsigned)(((int64_t)Ho * Wo + kThreads - 1) / kThreads), n);
    if (C == 1) hipLaunchKernelGGL(k_pad<1>, grid, dim3(kThreads), 0, s, in, H, W, Ho, Wo, top, left, border, value, out);
    else if (C == 3) hipLaunchKernelGGL(k_pad<3>, grid, dim3(kThreads), 0, s, in, H, W, Ho, Wo, top, left, border, value, out);
    else hipLaunchKernelGGL(k_pad<4>, grid, dim3(kThreads), 0, s, in, H, W, Ho, Wo, top, left, border, value, out);
    return hipGetLastError();
}

hipError_t launch_warp_u8(const uint8_t *in, int n, int H, int W, int C, const int64_t *aq, int interp, int border,
                          uint8_t *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    dim3 grid((unsigned)(((int64_t)H * W + kThreads - 1) / kThreads), n);
    if (C == 1) hipLaunchKernelGGL(k_warp<1>, grid, dim3(kThreads), 0, s, in, H, W, aq, interp, border, out);
    else if (C == 3) hipLaunchKernelGGL(k_warp<3>, grid, dim3(kThreads), 0, s, in, H, W, aq, interp, border, out);
    else hipLaunchKernelGGL(k_warp<4>, grid, dim3(kThreads), 0, s, in, H, W, aq, interp, border, out);
    return hipGetLastError();
}

}  // namespace miaug
