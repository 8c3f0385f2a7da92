// ragged_common.h -- device helpers shared by the ragged-batch kernels
// (k_ragged.hip: tile passes; k_rows.hip: row bands): exact small divisions,
// the half-pixel resize position, normalisation and brightness/contrast LUTs,
// boxes, per-image records, LDS-DMA and the per-XCD work queues.
// Library-internal; not part of the C ABI.
#pragma once
#include "dev_common.h"
#include "internal.h"

namespace miaug {
namespace {

constexpr int kQueues = 8;
constexpr int kCounterStride = 16;  // ints between counters (one 64-byte line each)
constexpr int kMaxSide = 1 << 20;   // images with a side this long or longer are skipped
typedef __attribute__((address_space(3))) void *lds_ptr_t;

// Load of read-only kernel input through the constant address space: with a
// uniform address it becomes a scalar load (counted by lgkmcnt, so it never
// waits behind LDS-DMA traffic counted by vmcnt).
template <class T>
__device__ __forceinline__ T ldc(const T *p) {
    return *(const __attribute__((address_space(4))) T *)p;
}

// floor(A / D) and the remainder for 0 <= A < 2^23, 1 <= D < 2^23, given
// rD = v_rcp_f32(D) (relative error below 2^-22).  The float quotient is
// within 2/D <= 1 of A / D for D >= 2 (exact for D = 1), so its truncation is
// off by at most one (and q D < 2^24 for the full-rate multiply).
__device__ __forceinline__ int fdiv_small(int A, int D, float rD, int &r) {
    int q = (int)((float)A * rD);
    r = A - (int)__umul24(q, D);
    if (r < 0) { q -= 1; r += D; }
    else if (r >= D) { q += 1; r -= D; }
    return q;
}

// floor(A / D) and the remainder for 0 <= A, 1 <= D < 2^23: the float form
// below 2^23, the compiler's integer division above.
__device__ __forceinline__ int udiv_small(int A, int D, int &r) {
    if (A < (1 << 23)) return fdiv_small(A, D, __builtin_amdgcn_rcpf((float)D), r);
    const int q = A / D;
    r = A - q * D;
    return q;
}

// floor(A / D) and the remainder for 2^23 <= A < 2^34 (sides of at least
// about 2^13 pixels); out of line, since it is rarely taken.
__device__ __noinline__ int2 div_wide(int64_t A, int D) {
    const int q = (int)(A / D);
    return make_int2(q, (int)(A - (int64_t)q * D));
}

// Half-pixel-centre position of output index j (Q10):
// rdiv_he(((2j+1) Ls - Lo) 2^10, 2 Lo) for 0 <= j < Lo <= 4096, 1 <= Ls < 2^20.
// A + D = (2j+1) Ls + Lo > 0 is split as qa D + ra, then ra 2^10 = qb D + rb.
__device__ __forceinline__ int32_t resize_q(int j, int Ls, int Lo) {
    const int D = 2 * Lo;
    const float rD = __builtin_amdgcn_rcpf((float)D);
    const int64_t A = (int64_t)(2 * j + 1) * Ls + Lo;
    int qa, ra;
    if (A < (1 << 23)) {
        qa = fdiv_small((int)A, D, rD, ra);
    } else {
        const int2 qr = div_wide(A, D);
        qa = qr.x;
        ra = qr.y;
    }
    qa -= 1;
    int rb;
    const int qb = fdiv_small(ra << kFBits, D, rD, rb);
    const int q = (qa << kFBits) + qb;
    return q + ((2 * rb > D) | ((2 * rb == D) & (q & 1)));
}

// Round-half-even of acc / 2^20 for acc >= 0.
__device__ __forceinline__ int rhe20(int acc) { return (acc + 0x7FFFF + ((acc >> 20) & 1)) >> 20; }

__device__ __forceinline__ void build_norm_lut(const miaug_ragged_args &a, float (&nlut)[3][256]) {
    for (int e = threadIdx.x; e < 3 * 256; e += blockDim.x) {
        int c = e >> 8, v = e & 255;
        nlut[c][v] = (float)((((double)v / 255.0) - (double)a.mean[c]) / (double)a.stdv[c]);
    }
}

__device__ __forceinline__ void build_bc_lut(float alpha, float beta, uint8_t *lut) {
    const int tid = threadIdx.x;
    const double v = (double)alpha * (double)tid + (double)beta;
    lut[tid] = (uint8_t)sat8((int)rint(v));
}

// Boxes of one image: Dih4 ops one after the other, the shift into the crop
// window and the clip to it (when there is one), then the scale to the output
// size, in double.  Called only for images whose window is valid.
template <int NT>
__device__ __forceinline__ void ragged_boxes(const miaug_ragged_args &a, int img) {
    int b0 = ldc(a.box_off + img), b1 = ldc(a.box_off + img + 1);
    const int32_t *fl = a.flags + 4 * img;
    const int f0 = ldc(fl), f1 = ldc(fl + 1), f2 = ldc(fl + 2), f3 = ldc(fl + 3);
    for (int b = b0 + (int)threadIdx.x; b < b1; b += NT) {
        double x1 = a.boxes[4 * b], y1 = a.boxes[4 * b + 1], x2 = a.boxes[4 * b + 2], y2 = a.boxes[4 * b + 3];
        double h = ldc(a.hw + 2 * img), w = ldc(a.hw + 2 * img + 1);
        if (f0) { double u = w - x2, v = w - x1; x1 = u; x2 = v; }
        if (f1) { double u = h - y2, v = h - y1; y1 = u; y2 = v; }
        for (int t = 0; t < (f2 & 3); ++t) {
            double nx1 = y1, ny1 = w - x2, nx2 = y2, ny2 = w - x1;
            x1 = nx1; y1 = ny1; x2 = nx2; y2 = ny2;
            double s = h; h = w; w = s;
        }
        if (f3) {
            double nx1 = y1, ny1 = x1, nx2 = y2, ny2 = x2;
            x1 = nx1; y1 = ny1; x2 = nx2; y2 = ny2;
            double s = h; h = w; w = s;
        }
        if (a.crop && ldc(a.crop + 4 * img + 2) != 0) {  // shift into the crop window and clip to it
            const double wy = ldc(a.crop + 4 * img), wx = ldc(a.crop + 4 * img + 1);
            h = ldc(a.crop + 4 * img + 2);
            w = ldc(a.crop + 4 * img + 3);
            x1 = fmin(fmax(x1 - wx, 0.0), w);
            x2 = fmin(fmax(x2 - wx, 0.0), w);
            y1 = fmin(fmax(y1 - wy, 0.0), h);
            y2 = fmin(fmax(y2 - wy, 0.0), h);
        }
        double sx = (double)a.out_w / w, sy = (double)a.out_h / h;
        a.out_boxes[4 * b] = (float)(x1 * sx);
        a.out_boxes[4 * b + 1] = (float)(y1 * sy);
        a.out_boxes[4 * b + 2] = (float)(x2 * sx);
        a.out_boxes[4 * b + 3] = (float)(y2 * sy);
    }
}

// Per-image inputs a pass plan needs.
struct ImgInfo {
    int H, W, f0, f1, f2, f3;
    int64_t io, mo;  // byte offsets of the image and mask
    float alpha, beta;
    int wy, wx, wh, ww;  // crop window of the Dih4 image (wh = 0: none)
};

// Through scalar loads (uniform img).
__device__ __forceinline__ ImgInfo info_scalar(const miaug_ragged_args &a, int img) {
    ImgInfo r;
    r.H = ldc(a.hw + 2 * img);
    r.W = ldc(a.hw + 2 * img + 1);
    const int32_t *fl = a.flags + 4 * img;
    r.f0 = ldc(fl);
    r.f1 = ldc(fl + 1);
    r.f2 = ldc(fl + 2);
    r.f3 = ldc(fl + 3);
    r.io = ldc(a.img_off + img);
    r.mo = a.mask ? ldc(a.mask_off + img) : 0;
    r.alpha = ldc(a.ab + 2 * img);
    r.beta = ldc(a.ab + 2 * img + 1);
    r.wy = r.wx = r.wh = r.ww = 0;
    if (a.crop) {
        r.wy = ldc(a.crop + 4 * img);
        r.wx = ldc(a.crop + 4 * img + 1);
        r.wh = ldc(a.crop + 4 * img + 2);
        r.ww = ldc(a.crop + 4 * img + 3);
    }
    return r;
}

__device__ __forceinline__ const uint8_t *align16(const uint8_t *g) {
    return (const uint8_t *)((uintptr_t)g & ~(uintptr_t)15);
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// 16 bytes per lane from a buffer (32-bit offset) into LDS at lds + 16 * lane.
__device__ __forceinline__ void dma16(__amdgpu_buffer_rsrc_t rs, uint8_t *lds, uint32_t voff) {
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr_t)lds, 16, voff, 0, 0, 0);
}

// floor(x / d) for 0 <= x < 2^12, 1 <= d < 2^11, given M = ceil(2^32 / d)
// (M = 0 for d = 1): with M d = 2^32 + e, 0 <= e < d, the error term x e is
// below 2^23, far under 2^32, so the high word of x M is the exact quotient.
__device__ __forceinline__ int div_by_m(int x, int d, uint32_t M) { return d == 1 ? x : (int)__umulhi((uint32_t)x, M); }
__device__ __forceinline__ uint32_t div_magic(int d) {
    return d <= 1 ? 0u : (uint32_t)((0x100000000ull + (uint64_t)d - 1) / (uint64_t)d);
}

// Chunked work claiming (thread 0 of a workgroup): one atomic claims K
// consecutive positions of a queue (position u of queue q is tile u mod tiles
// of image (u / tiles) * 8 + q), and the atomic for the next chunk is issued
// as soon as the current one is known, so its latency hides behind a whole
// chunk of tiles.
template <int K>
struct Claimer {
    int tiles, q, tries, raw;

    __device__ __forceinline__ void issue(int *counters) {
        if (tries < kQueues) raw = atomicAdd(&counters[q * kCounterStride], K);
    }
    // Chunk from the atomic issued last: queue, first position and count
    // (count 0 once every queue is exhausted).  Exhausted queues are skipped
    // with further, synchronous atomics.
    __device__ __forceinline__ int3 resolve(const miaug_ragged_args &a, int *counters) {
        while (tries < kQueues) {
            const int total = ((a.n - q + kQueues - 1) / kQueues) * tiles;  // images i with i mod 8 == q
            if (raw < total) return make_int3(q, raw, min(K, total - raw));
            q = (q + 1) % kQueues;
            if (++tries < kQueues) raw = atomicAdd(&counters[q * kCounterStride], K);
        }
        return make_int3(0, 0, 0);
    }
};

// Next item of the claim stream of thread 0 (-1 once every queue is
// exhausted); the atomic for the one after it is issued before returning.
__device__ __forceinline__ int claim_item(Claimer<1> &C, const miaug_ragged_args &a, int *counters) {
    const int3 c = C.resolve(a, counters);
    if (c.z == 0) return -1;
    int ut;
    const int img = udiv_small(c.y, C.tiles, ut) * kQueues + c.x;
    C.issue(counters);
    return img * C.tiles + ut;
}

__global__ void k_zero_counters(int *counters, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) counters[i] = 0;
}

}  // namespace
}  // namespace miaug
