// k_stats.hip -- per-image, per-channel statistics of u8 images: sum, min,
// max and a 256-bin histogram.  Wavefront reductions (shuffles) and LDS
// histograms per workgroup, then one global atomic per workgroup and value.
#include "dev_common.h"
#include "internal.h"

namespace miaug {
namespace {

constexpr int kThreads = 256;
constexpr int kBlocksPerImage = 64;

__global__ void k_stats_init(int n, int C, uint64_t *sum, int32_t *mn, int32_t *mx, uint32_t *hist) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n * C) {
        if (sum) sum[i] = 0;
        if (mn) mn[i] = 255;
        if (mx) mx[i] = 0;
    }
    if (hist)
        for (int j = i; j < n * C * 256; j += gridDim.x * blockDim.x) hist[j] = 0;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

__global__ __launch_bounds__(kThreads) void k_stats(const uint8_t *__restrict__ img, int64_t npix, int C,
                                                    uint64_t *sum, int32_t *mn, int32_t *mx, uint32_t *hist) {
    __shared__ uint32_t h[4][256];
    __shared__ uint32_t rs[kThreads / 64][4];
    __shared__ int rmn[kThreads / 64][4], rmx[kThreads / 64][4];
    const int im = blockIdx.y;
    for (int e = threadIdx.x; e < 4 * 256; e += kThreads) (&h[0][0])[e] = 0;
    __syncthreads();
    const uint8_t *base = img + (size_t)im * npix * C;
    uint32_t s[4] = {0, 0, 0, 0};
    int lo[4] = {255, 255, 255, 255}, hi[4] = {0, 0, 0, 0};
    for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < npix; p += (int64_t)gridDim.x * kThreads) {
        for (int c = 0; c < C; ++c) {
            const int v = base[p * C + c];
            s[c] += v;
            lo[c] = min(lo[c], v);
            hi[c] = max(hi[c], v);
            if (hist) atomicAdd(&h[c][v], 1u);
        }
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int c = 0; c < C; ++c) {
        const uint32_t ws = wave_sum_u32(s[c]);  // < 2^32: a workgroup sees < 2^24 pixels per image per pass
        const int wl = wave_min(lo[c]), wh = wave_max(hi[c]);
        if (lane == 0) { rs[wave][c] = ws; rmn[wave][c] = wl; rmx[wave][c] = wh; }
    }
    __syncthreads();
    if (threadIdx.x < C) {
        const int c = threadIdx.x;
        uint64_t tot = 0;
        int l = 255, u = 0;
        for (int w = 0; w < kThreads / 64; ++w) { tot += rs[w][c]; l = min(l, rmn[w][c]); u = max(u, rmx[w][c]); }
        if (sum) atomicAdd((unsigned long long *)&sum[im * C + c], (unsigned long long)tot);
        if (mn) atomicMin(&mn[im * C + c], l);
        if (mx) atomicMax(&mx[im * C + c], u);
    }
    if (hist)
        for (int e = threadIdx.x; e < C * 256; e += kThreads) {
            const uint32_t v = h[e >> 8][e & 255];
            if (v) atomicAdd(&hist[((size_t)im * C + (e >> 8)) * 256 + (e & 255)], v);
        }
}

}  // namespace

hipError_t launch_image_stats(const uint8_t *img, int n, int64_t npix, int C, uint64_t *sum, int32_t *mn, int32_t *mx,
                              uint32_t *hist, hipStream_t s) {
    hipLaunchKernelGGL(k_stats_init, dim3((n * C * 256 + 255) / 256), dim3(256), 0, s, n, C, sum, mn, mx, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || npix == 0) return e;
    int blocks = (int)min((int64_t)kBlocksPerImage, (npix + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_stats, dim3(blocks, n), dim3(kThreads), 0, s, img, npix, C, sum, mn, mx, hist);
    return hipGetLastError();
}

}  // namespace miaug
