// k_stats.hip -- per-image, per-channel statistics of u8 images: sum, min,
// max and a 256-bin histogram.  Wavefront reductions (shuffles) and LDS
// histograms per wave, then one global atomic per workgroup and value.
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

// Histogram step of one channel's values v[0..K-1] of a thread: each distinct
// value adds its count once (neighbouring pixels of smooth images are often
// equal, and atomics on one LDS word serialise).
template <int K>
__device__ __forceinline__ void hist_add(uint32_t *h, const int (&v)[K]) {
#pragma unroll
    for (int j = 0; j < K; ++j) {
        bool first = true;
        uint32_t cnt = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (k < j && v[k] == v[j]) first = false;
            cnt += v[k] == v[j];
        }
        if (first) atomicAdd(&h[v[j]], cnt);
    }
}

// quads: a thread takes four consecutive pixels (4 C bytes, C dword loads)
// per step; needs a 4-byte aligned batch and npix a multiple of 4.  Each
// wave keeps its own histograms, summed at the end.
__global__ __launch_bounds__(kThreads) void k_stats(const uint8_t *__restrict__ img, int64_t npix, int C, bool quads,
                                                    uint64_t *sum, int32_t *mn, int32_t *mx, uint32_t *hist) {
    constexpr int kW = kThreads / 64;
    __shared__ uint32_t h[kW][4][256];
    __shared__ uint32_t rs[kW][4];
    __shared__ int rmn[kW][4], rmx[kW][4];
    const int im = blockIdx.y, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int e = threadIdx.x; e < kW * 4 * 256; e += kThreads) (&h[0][0][0])[e] = 0;
    __syncthreads();
    uint32_t(*hw)[256] = h[wave];
    const uint8_t *base = img + (size_t)im * npix * C;
    uint32_t s[4] = {0, 0, 0, 0};
    int lo[4] = {255, 255, 255, 255}, hi[4] = {0, 0, 0, 0};
    const int64_t step = (int64_t)gridDim.x * kThreads;
    if (quads) {
        const int64_t nq = npix / 4;
        for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < nq; q += step) {
            const uint32_t *w = (const uint32_t *)(base + 4 * q * C);
            uint32_t d[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) d[k] = k < C ? w[k] : 0u;
            // byte 4 j + c of the group is pixel j, channel c: byte b sits in word b / 4
            for (int c = 0; c < C; ++c) {
                int v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int b = j * C + c;
                    v[j] = (int)((d[b >> 2] >> (8 * (b & 3))) & 255u);
                    s[c] += v[j];
                    lo[c] = min(lo[c], v[j]);
                    hi[c] = max(hi[c], v[j]);
                }
                if (hist) hist_add<4>(hw[c], v);
            }
        }
    } else {
        for (int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x; p < npix; p += step)
            for (int c = 0; c < C; ++c) {
                const int v = base[p * C + c];
                s[c] += v;
                lo[c] = min(lo[c], v);
                hi[c] = max(hi[c], v);
                if (hist) atomicAdd(&hw[c][v], 1u);
            }
    }
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
        for (int w = 0; w < kW; ++w) { tot += rs[w][c]; l = min(l, rmn[w][c]); u = max(u, rmx[w][c]); }
        if (sum) atomicAdd((unsigned long long *)&sum[im * C + c], (unsigned long long)tot);
        if (mn) atomicMin(&mn[im * C + c], l);
        if (mx) atomicMax(&mx[im * C + c], u);
    }
    if (hist)
        for (int e = threadIdx.x; e < C * 256; e += kThreads) {
            uint32_t v = 0;
#pragma unroll
            for (int w = 0; w < kW; ++w) v += h[w][e >> 8][e & 255];
            if (v) atomicAdd(&hist[((size_t)im * C + (e >> 8)) * 256 + (e & 255)], v);
        }
}

}  // namespace

hipError_t launch_image_stats(const uint8_t *img, int n, int64_t npix, int C, uint64_t *sum, int32_t *mn, int32_t *mx,
                              uint32_t *hist, hipStream_t s) {
    hipLaunchKernelGGL(k_stats_init, dim3((n * C * 256 + 255) / 256), dim3(256), 0, s, n, C, sum, mn, mx, hist);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || npix == 0) return e;
    const bool quads = ((uintptr_t)img & 3) == 0 && (npix & 3) == 0;
    const int64_t items = quads ? npix / 4 : npix;
    int blocks = (int)min((int64_t)kBlocksPerImage, max((int64_t)1, (items + kThreads - 1) / kThreads));
    hipLaunchKernelGGL(k_stats, dim3(blocks, n), dim3(kThreads), 0, s, img, npix, C, quads, sum, mn, mx, hist);
    return hipGetLastError();
}

}  // namespace miaug
