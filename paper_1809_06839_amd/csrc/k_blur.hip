// k_blur.hip -- binomial blur of a dense u8 batch: the outer product of
// [1, 2, 1] (3x3, / 16) or [1, 4, 6, 4, 1] (5x5, / 256), one round-half-even
// division of the integer sum, reflect-101 border, per channel, switched on or
// off per image (the op's probability is drawn by the sampler).
//
// One workgroup per 32 x 32 output tile: the tile and its reflect-101 halo
// are staged in LDS, a horizontal pass writes 16-bit row sums (at most
// 16 x 255), and a vertical pass forms the full sum, which equals the 2-D sum
// exactly (integer arithmetic), and rounds it.
#include "dev_common.h"
#include "internal.h"

namespace miaug {
namespace {

constexpr int kBT = 32;  // output tile side
constexpr int kBThreads = 256;

template <int R>
__device__ __forceinline__ int binom(int i) {
    if (R == 1) return i == 1 ? 2 : 1;
    return i == 2 ? 6 : (i == 1 || i == 3 ? 4 : 1);
}

template <int C, int R>
__global__ __launch_bounds__(kBThreads) void k_blur(const uint8_t *__restrict__ in, int H, int W,
                                                    const int32_t *__restrict__ apply, uint8_t *__restrict__ out) {
    constexpr int S = kBT + 2 * R;  // staged side
    constexpr int kShift = R == 1 ? 4 : 8;
    __shared__ uint8_t st[S * S * C];
    __shared__ uint16_t hs[S * kBT * C];
    const int img = blockIdx.y;
    const int ntx = (W + kBT - 1) / kBT;
    const int tx0 = (int)(blockIdx.x % ntx) * kBT, ty0 = (int)(blockIdx.x / ntx) * kBT;
    const int tw = min(kBT, W - tx0), th = min(kBT, H - ty0);
    const uint8_t *src = in + (size_t)img * H * W * C;
    uint8_t *dst = out + (size_t)img * H * W * C;
    const int rb = tw * C;  // bytes of a tile row
    if (apply && apply[img] == 0) {  // the op was not drawn for this image: copy the tile
        for (int e = threadIdx.x; e < rb * th; e += kBThreads) {
            const int r = e / rb, d = e - r * rb;
            const size_t o = ((size_t)(ty0 + r) * W + tx0) * C + d;
            dst[o] = src[o];
        }
        return;
    }
    for (int e = threadIdx.x; e < S * S; e += kBThreads) {
        const int r = e / S, c = e - r * S;
        const int sy = reflect101(ty0 - R + r, H), sx = reflect101(tx0 - R + c, W);
        const uint8_t *p = src + ((size_t)sy * W + sx) * C;
#pragma unroll
        for (int ch = 0; ch < C; ++ch) st[e * C + ch] = p[ch];
    }
    __syncthreads();
    // horizontal sums: entry (r, d) with d = column * C + channel
    for (int e = threadIdx.x; e < S * kBT * C; e += kBThreads) {
        const int r = e / (kBT * C), d = e - r * (kBT * C);
        const uint8_t *p = st + r * S * C + d;
        int acc = 0;
#pragma unroll
        for (int i = 0; i <= 2 * R; ++i) acc += binom<R>(i) * p[i * C];
        hs[e] = (uint16_t)acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kBT * kBT * C; e += kBThreads) {
        const int r = e / (kBT * C), d = e - r * (kBT * C);
        if (r >= th || d >= rb) continue;
        int acc = 0;
#pragma unroll
        for (int j = 0; j <= 2 * R; ++j) acc += binom<R>(j) * hs[(r + j) * kBT * C + d];
        const int q = acc >> kShift, rem = acc & ((1 << kShift) - 1), half = 1 << (kShift - 1);
        dst[((size_t)(ty0 + r) * W + tx0) * C + d] = (uint8_t)(q + ((rem > half) | ((rem == half) & (q & 1))));
    }
}

template <int R>
hipError_t launch_r(const uint8_t *in, int n, int H, int W, int C, const int32_t *apply, uint8_t *out,
                    hipStream_t s) {
    dim3 grid((unsigned)(((W + kBT - 1) / kBT) * ((H + kBT - 1) / kBT)), n);
    if (C == 1) hipLaunchKernelGGL((k_blur<1, R>), grid, dim3(kBThreads), 0, s, in, H, W, apply, out);
    else if (C == 3) hipLaunchKernelGGL((k_blur<3, R>), grid, dim3(kBThreads), 0, s, in, H, W, apply, out);
    else hipLaunchKernelGGL((k_blur<4, R>), grid, dim3(kBThreads), 0, s, in, H, W, apply, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_blur_u8(const uint8_t *in, int n, int H, int W, int C, int ksize, const int32_t *apply,
                          uint8_t *out, hipStream_t s) {
    if (n == 0 || H == 0 || W == 0) return hipSuccess;
    return ksize == 5 ? launch_r<2>(in, n, H, W, C, apply, out, s) : launch_r<1>(in, n, H, W, C, apply, out, s);
}

}  // namespace miaug
