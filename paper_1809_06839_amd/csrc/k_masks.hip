// k_masks.hip -- multi-channel (instance) masks of the ragged batch: K u8
// channels per pixel, one per instance, take the image's geometry (Dih4
// element, crop window, nearest resize) exactly like the one-channel masks of
// the fused ragged kernel (Sec. II-A: masks follow the image).  A nearest
// resample moves K contiguous bytes per output pixel and has no arithmetic, so
// one thread copies one pixel.
#include "dev_common.h"
#include "internal.h"

namespace miaug {
namespace {

constexpr int kThreads = 256;

// Half-pixel-centre Q10 position of output index j: rdiv_he(((2j+1) Ls - Lo) 2^10, 2 Lo).
__device__ __forceinline__ int32_t resize_q64(int j, int Ls, int Lo) {
    const int64_t D = 2 * (int64_t)Lo;
    const int64_t N = ((2 * (int64_t)j + 1) * Ls - Lo) * kFOne;
    int64_t q = N / D, r = N - q * D;
    if (r < 0) { q -= 1; r += D; }
    return (int32_t)(q + ((2 * r > D) | ((2 * r == D) & (q & 1))));
}

__global__ __launch_bounds__(kThreads) void k_ragged_masks(miaug_ragged_args a, int K, uint8_t *__restrict__ out) {
    const int img = blockIdx.y;
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= a.out_h * a.out_w) return;
    const int H = a.hw[2 * img], W = a.hw[2 * img + 1];
    if (H < 1 || W < 1 || H >= (1 << 20) || W >= (1 << 20)) return;
    const int32_t *fl = a.flags + 4 * img;
    D4Map m = make_d4(H, W, fl[0], fl[1], fl[2], fl[3]);
    if (a.crop && a.crop[4 * img + 2] != 0) {
        const int wy = a.crop[4 * img], wx = a.crop[4 * img + 1], wh = a.crop[4 * img + 2], ww = a.crop[4 * img + 3];
        if (wy < 0 || wx < 0 || wh < 1 || ww < 1 || wh > m.oh - wy || ww > m.ow - wx) return;  // skipped image
        m.cy += m.ay * wy + m.by * wx;
        m.cx += m.ax * wy + m.bx * wx;
        m.oh = wh;
        m.ow = ww;
    }
    const int y = e / a.out_w, x = e - y * a.out_w;
    const int r = min(max((resize_q64(y, m.oh, a.out_h) + kFOne / 2) >> kFBits, 0), m.oh - 1);
    const int c = min(max((resize_q64(x, m.ow, a.out_w) + kFOne / 2) >> kFBits, 0), m.ow - 1);
    const uint8_t *src = a.mask + a.mask_off[img] + ((size_t)m.sy(r, c) * W + m.sx(r, c)) * K;
    uint8_t *dst = out + ((size_t)img * a.out_h * a.out_w + e) * K;
    for (int k = 0; k < K; ++k) dst[k] = src[k];
}

}  // namespace

hipError_t launch_ragged_masks(const miaug_ragged_args *a, int K, uint8_t *out, hipStream_t s) {
    if (a->n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ragged_masks, dim3((a->out_h * a->out_w + kThreads - 1) / kThreads, a->n), dim3(kThreads), 0,
                       s, *a, K, out);
    return hipGetLastError();
}

}  // namespace miaug
