// dev_common.h -- device helpers shared by the libmiaug kernels (gfx950).
//
// Integer rounding, reflect-101 borders, Dih4 index maps and byte-span
// movement between HBM and LDS.  Library-internal; not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace miaug {

constexpr int kFBits = 10;          // sub-pixel bits of every fixed-point position
constexpr int kFOne = 1 << kFBits;

// n / 2^k rounded to nearest, ties to even (arithmetic shift = floor).
__device__ __forceinline__ int32_t rshr_he(int32_t n, int k) {
    int32_t q = n >> k;
    int32_t r = n - (q << k);
    int32_t half = 1 << (k - 1);
    return q + ((r > half) | ((r == half) & (q & 1)));
}

__device__ __forceinline__ int64_t rshr_he64(int64_t n, int k) {
    int64_t q = n >> k;
    int64_t r = n - (q << k);
    int64_t half = int64_t(1) << (k - 1);
    return q + ((r > half) | ((r == half) & (q & 1)));
}

// n / d rounded to nearest, ties to even, d > 0, n >= 0 (unsigned fast path).
__device__ __forceinline__ uint32_t udiv_he(uint32_t n, uint32_t d) {
    uint32_t q = n / d;
    uint32_t r = n - q * d;
    return q + ((2 * r > d) | ((2 * r == d) & (q & 1)));
}

// General signed n / d, ties to even, floor-based remainder, d > 0.
__device__ __forceinline__ int32_t sdiv_he(int32_t n, int32_t d) {
    int32_t q = n / d;
    int32_t r = n - q * d;
    if (r < 0) { q -= 1; r += d; }
    return q + ((2 * r > d) | ((2 * r == d) & (q & 1)));
}

// a * b + c with operands known to fit 24 bits (full-rate v_mad_i32_i24; the
// compiler otherwise widens such products to 64-bit multiply-adds).  ALU-only
// inline asm: no memory operand.
__device__ __forceinline__ int mad24(int a, int b, int c) {
    int d;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// Unsigned form: a * b + c for a, b < 2^24 (v_mad_u32_u24).
__device__ __forceinline__ uint32_t umad24(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t d;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
    return d;
}

// Logical workgroup (x, y) of a 2-D grid (x fastest), remapped for L2
// locality: the hardware deals consecutive workgroups to the 8 XCDs
// round-robin, each XCD with its own L2, so the logical range is cut into 8
// contiguous runs and XCD k takes run k; neighbouring logical workgroups (tiles
// that share source rows) then meet in one L2.  A bijection on the grid.
__device__ __forceinline__ int2 xcd_block() {
    const int gx = gridDim.x, nb = gx * gridDim.y;
    const int b = blockIdx.x + gx * blockIdx.y;
    const int per = nb >> 3, rem = nb & 7, x = b & 7, k = b >> 3;
    const int L = x < rem ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
    return make_int2(L % gx, L / gx);
}

// Buffer resource over [base, base + bytes) for raw buffer stores: 32-bit byte
// offsets, stores outside the range are dropped by the hardware.  Word 3 is
// the gfx9-family default descriptor (32-bit data, no swizzle).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ int sat8(int v) { return v < 0 ? 0 : (v > 255 ? 255 : v); }

__device__ __forceinline__ int clampi(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

// Reflect-101 (edge pixel not repeated); valid for any int i.
__device__ __forceinline__ int reflect101(int i, int n) {
    if (n == 1) return 0;
    int p = 2 * n - 2;
    i %= p;
    if (i < 0) i += p;
    return i >= n ? p - i : i;
}

// Dih4 element as an integer map from D4-space coordinates (r, c) of the
// output of hflip -> vflip -> rot90^k -> transpose to source coordinates:
//   sy = ay r + by c + cy,   sx = ax r + bx c + cx,
// with coefficients in {-1, 0, 1}.  Built by substituting each op's
// coordinate change in turn; oh, ow receive the D4-space shape.
struct D4Map {
    int ay, by, cy, ax, bx, cx;
    int oh, ow;
    __host__ __device__ __forceinline__ bool swaps() const { return by != 0; }
    __host__ __device__ __forceinline__ int sy(int r, int c) const { return ay * r + by * c + cy; }
    __host__ __device__ __forceinline__ int sx(int r, int c) const { return ax * r + bx * c + cx; }
};

__host__ __device__ inline D4Map make_d4(int H, int W, int hflip, int vflip, int k, int transpose) {
    D4Map m{1, 0, 0, 0, 1, 0, H, W};
    int h = H, w = W;
    if (hflip) {  // (r, c) -> (r, w-1-c)
        m.cy += m.by * (w - 1); m.by = -m.by;
        m.cx += m.bx * (w - 1); m.bx = -m.bx;
    }
    if (vflip) {  // (r, c) -> (h-1-r, c)
        m.cy += m.ay * (h - 1); m.ay = -m.ay;
        m.cx += m.ax * (h - 1); m.ax = -m.ax;
    }
    for (int t = 0; t < (k & 3); ++t) {  // (r, c) -> (c, w-1-r), shape (w, h)
        int ay = m.ay, by = m.by, ax = m.ax, bx = m.bx;
        m.cy += by * (w - 1); m.ay = -by; m.by = ay;
        m.cx += bx * (w - 1); m.ax = -bx; m.bx = ax;
        int s = h; h = w; w = s;
    }
    if (transpose) {  // (r, c) -> (c, r), shape (w, h)
        int ay = m.ay, ax = m.ax;
        m.ay = m.by; m.by = ay;
        m.ax = m.bx; m.bx = ax;
        int s = h; h = w; w = s;
    }
    m.oh = h; m.ow = w;
    return m;
}

// Copies global bytes [g, g + len) into LDS with 16-byte aligned vector loads:
// the aligned chunk containing g lands at dst, so byte g[b] is at
// dst[phase + b] with phase = (uintptr_t)g & 15.  Chunks never leave the
// 16-byte aligned blocks that hold valid bytes, so they stay inside mapped
// pages.  Work is spread over `nthr` threads starting at thread `tid`.
__device__ __forceinline__ int span_phase(const uint8_t *g) { return (int)((uintptr_t)g & 15); }

__device__ __forceinline__ void load_span16(const uint8_t *g, int len, uint8_t *dst, int tid, int nthr) {
    const uint8_t *a = (const uint8_t *)((uintptr_t)g & ~(uintptr_t)15);
    int nchunk = (int)((((uintptr_t)g + len + 15) & ~(uintptr_t)15) - (uintptr_t)a) >> 4;
    for (int i = tid; i < nchunk; i += nthr) {
        uint4 v = *(const uint4 *)(a + 16 * i);
        *(uint4 *)(dst + 16 * i) = v;
    }
}

// Byte-span stores: bytes [0, len) produced by byte_at(b) go to global g + b.
// Whole aligned dwords inside the span are written with one store; the edge
// bytes of dwords shared with neighbouring spans are written one by one.  A
// span splits into span_items(g, len) independent items; store_span_item
// performs item j (several threads can share one span, or one thread can do
// items of many spans).
__device__ __forceinline__ int span_items(const uint8_t *g, int len) {
    int head = (int)((4 - ((uintptr_t)g & 3)) & 3);
    if (head > len) head = len;
    int body = (len - head) >> 2;
    return len - 3 * body;  // head + body + tail
}

template <class F>
__device__ __forceinline__ void store_span_item(uint8_t *g, int len, int j, F byte_at) {
    int head = (int)((4 - ((uintptr_t)g & 3)) & 3);
    if (head > len) head = len;
    int body = (len - head) >> 2;
    if (j < head) {
        g[j] = byte_at(j);
    } else if (j < head + body) {
        int b = head + 4 * (j - head);
        uint32_t v = (uint32_t)byte_at(b) | ((uint32_t)byte_at(b + 1) << 8) | ((uint32_t)byte_at(b + 2) << 16) |
                     ((uint32_t)byte_at(b + 3) << 24);
        *(uint32_t *)(g + b) = v;
    } else {
        int b = head + 4 * body + (j - head - body);
        if (b < len) g[b] = byte_at(b);
    }
}

// Number of 16-byte chunks load_span16 moves for span [g, g + len).
__device__ __forceinline__ int span_chunks(const uint8_t *g, int len) {
    return (int)((((uintptr_t)g + len + 15) & ~(uintptr_t)15) - ((uintptr_t)g & ~(uintptr_t)15)) >> 4;
}

// Chunk i of load_span16 for span starting at g (dst as in load_span16).
__device__ __forceinline__ void load_span16_chunk(const uint8_t *g, int i, uint8_t *dst) {
    const uint8_t *a = (const uint8_t *)((uintptr_t)g & ~(uintptr_t)15);
    *(uint4 *)(dst + 16 * i) = *(const uint4 *)(a + 16 * i);
}

}  // namespace miaug
