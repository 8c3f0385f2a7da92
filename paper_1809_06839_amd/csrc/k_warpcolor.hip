// k_warpcolor.hip -- differentiable float32 warp + colour op and its backward
// (training-time form of Table I ShiftScaleRotate + Brightness/contrast +
// Gamma, with gradients w.r.t. the image and the 7 per-sample parameters).
//
// Forward, per image i, channel c, output pixel (x, y):
//   X = x - cx - tx W, Y = y - cy - ty H (c the image centre),
//   sx = (cos X - sin Y) / s + cx,  sy = (sin X + cos Y) / s + cy,
//   w = bilinear(x_ic, sx, sy) (taps outside the image read 0),
//   z = alpha w + beta, y1 = clamp(z, 0, 1), y = y1^gamma (0^gamma = 0).
// Sample positions are evaluated in double, pixel values and the colour ops
// in float32 (no contraction).
//
// Layout of the work:
//   k_wc_fwd      one workgroup per 32 x 32 output tile, four pixels per
//                 thread down a column (rows 8 apart): the fp64 position is
//                 evaluated once per thread and stepped by the constant row
//                 increment.  The tile's source footprint (its bounding box)
//                 is staged in LDS by LDS-DMA with zeros outside the image,
//                 one channel at a time through two slots, the next channel's
//                 DMA in flight while a channel is blended; a footprint too
//                 large for a slot (zoom-out well below 1) gathers its taps
//                 from global memory instead, as 32-bit buffer offsets where a
//                 tap outside the image gets an offset past the end of the
//                 plane, which reads as 0;
//   k_wc_bwd      one workgroup per 32 x 32 source tile: the adjoint of the
//                 bilinear warp as a gather over the output pixels whose cell
//                 has a tap in the tile (grad_x has one writer per element: no
//                 global atomics, no zero-fill, no dL/dw buffer), with the
//                 parameter-gradient terms of the output pixels the tile owns
//                 reduced into one record per workgroup;
//   k_wc_reduce   sums the records of each image in a fixed order (double
//                 accumulators, one wave per image), plus the share of the
//                 output pixels whose cell lies wholly outside the image.
// The parameter gradients are bit-identical across runs.  grad_x is too,
// except where three or more output pixels share one bilinear cell (a
// zoom): the LDS slot order of those entries, and so their summation order,
// follows the order of the count atomics.
// y1^gamma is evaluated as exp2(gamma log2 y1) with the hardware base-2
// exponential and logarithm (a few float32 ulp, well inside the 1e-5
// forward and 1e-4 gradient tolerances).
#include "dev_common.h"
#include "internal.h"

namespace miaug {
namespace {

constexpr int kThreads = 256;
constexpr int kTile = 32;                // output tile of the per-pixel kernels
constexpr int kRowStep = 8;              // rows between a thread's four pixels
constexpr int kPix = kTile * kTile / kThreads;
constexpr int kSrcTile = 32;             // source tile of the adjoint kernel
constexpr int kCells = kSrcTile + 1;     // cells with a tap in the tile, per axis
constexpr int kMaxC = 4;
constexpr uint32_t kOOB = 0x80000000u;   // byte offset past every plane (planes are at most 2^30 bytes)

// Per-image geometry in double.  Sample positions are evaluated in double
// because a float32 position alone carries up to 2^-17 relative error (about
// 1e-5 px at x ~ 200), which the zero border and the gamma curve would turn
// into value errors above 1e-5.  One thread per workgroup computes it.
struct Geo {
    double c, s_, inv_s, cx, cy, ux, uy, scale;
};

__device__ __forceinline__ Geo make_geo(const float *p, int H, int W) {
    Geo g;
    sincospi((double)p[0] / 180.0, &g.s_, &g.c);  // the angle is in degrees: no reduction by pi needed
    g.scale = (double)p[1];
    g.inv_s = 1.0 / g.scale;
    g.cx = 0.5 * (double)(W - 1);
    g.cy = 0.5 * (double)(H - 1);
    g.ux = g.cx + (double)p[2] * (double)W;
    g.uy = g.cy + (double)p[3] * (double)H;
    return g;
}

__device__ __forceinline__ void sample_pos(const Geo &g, int x, int y, double &sx, double &sy) {
    const double X = (double)x - g.ux, Y = (double)y - g.uy;
    sx = (g.c * X - g.s_ * Y) * g.inv_s + g.cx;
    sy = (g.s_ * X + g.c * Y) * g.inv_s + g.cy;
}

// Bilinear cell of a sample point as four tap byte offsets into a plane
// (kOOB for a tap outside the image) and the float32 fractions.
struct Taps {
    uint32_t o00, o01, o10, o11;
    float fx, fy;
};

__device__ __forceinline__ Taps taps_of(double sx, double sy, int H, int W) {
    const double fx0 = floor(sx), fy0 = floor(sy);
    Taps t;
    t.fx = (float)(sx - fx0);
    t.fy = (float)(sy - fy0);
    // corners beyond the image read as outside; clamping first keeps the
    // integer conversion in range
    const uint32_t ux = (uint32_t)(int)fmin(fmax(fx0, -2.0), (double)W);
    const uint32_t uy = (uint32_t)(int)fmin(fmax(fy0, -2.0), (double)H);
    const bool vx0 = ux < (uint32_t)W, vx1 = ux + 1u < (uint32_t)W;
    const bool vy0 = uy < (uint32_t)H, vy1 = uy + 1u < (uint32_t)H;
    const uint32_t b = (uy * (uint32_t)W + ux) * 4u, bw = 4u * (uint32_t)W;  // wraps when unused
    t.o00 = (vx0 && vy0) ? b : kOOB;
    t.o01 = (vx1 && vy0) ? b + 4u : kOOB;
    t.o10 = (vx0 && vy1) ? b + bw : kOOB;
    t.o11 = (vx1 && vy1) ? b + bw + 4u : kOOB;
    return t;
}

__device__ __forceinline__ float ldf(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

__device__ __forceinline__ void stf(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, 0);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float *base, size_t plane, int H, int W) {
    return buffer_rsrc(const_cast<float *>(base) + plane * (size_t)H * W, (uint32_t)H * (uint32_t)W * 4u);
}

struct Quad {
    float p00, p01, p10, p11;
};

__device__ __forceinline__ Quad load_quad(__amdgpu_buffer_rsrc_t r, const Taps &t) {
    return Quad{ldf(r, t.o00), ldf(r, t.o01), ldf(r, t.o10), ldf(r, t.o11)};
}

__device__ __forceinline__ float bilerp(const Quad &q, float fx, float fy) {
    return (1.0f - fy) * ((1.0f - fx) * q.p00 + fx * q.p01) + fy * ((1.0f - fx) * q.p10 + fx * q.p11);
}

// y1^gamma for y1 > 0 (exactly y1 when gamma is 1), given l2 = log2(y1).
__device__ __forceinline__ float pow_pos(float y1, float gamma, float l2) {
    return gamma == 1.0f ? y1 : __builtin_amdgcn_exp2f(gamma * l2);
}

constexpr int kSlotFloats = 3072;  // 12 KB of LDS: one channel of the source footprint of an output tile

// Source box staged in LDS: [h][w] floats per channel from (x0, y0); w = 0
// when the footprint does not fit (the forward then gathers from global memory).
// v4: x0 and w are multiples of 4 and the rows are staged as 16-byte chunks
// (planes 16-byte aligned, W a multiple of 4, so a chunk never straddles the
// image's edge).
struct Box {
    int x0, y0, w, h, v4;
};

// Footprint of the 32 x 32 output tile at (X0, Y0): the cells of its sample
// points, their +1 taps and one pixel of margin on each side for the rounding
// of the stepped per-pixel positions.  With al, widened to whole 16-byte
// chunks when that still fits.
__device__ __forceinline__ Box tile_box(const Geo &g, int X0, int Y0, bool al) {
    double xl = 1e300, xh = -1e300, yl = 1e300, yh = -1e300;
    for (int k = 0; k < 4; ++k) {
        double sx, sy;
        sample_pos(g, X0 + ((k & 1) ? kTile - 1 : 0), Y0 + ((k & 2) ? kTile - 1 : 0), sx, sy);
        xl = fmin(xl, sx);
        xh = fmax(xh, sx);
        yl = fmin(yl, sy);
        yh = fmax(yh, sy);
    }
    Box b{0, 0, 0, 0, 0};
    const double x0 = floor(xl) - 1.0, y0 = floor(yl) - 1.0;
    const double w = floor(xh) + 3.0 - x0, h = floor(yh) + 3.0 - y0;
    if (!(fabs(x0) < 1e9 && fabs(y0) < 1e9 && w <= 64.0 && w * h <= (double)kSlotFloats)) return b;
    b.x0 = (int)x0;
    b.y0 = (int)y0;
    b.w = (int)w;
    b.h = (int)h;
    if (al) {
        const int xa = (b.x0 >> 2) << 2, wa = (((b.x0 + b.w + 3) >> 2) << 2) - xa;  // floor / ceil to 4
        if (wa <= 64 && wa * b.h <= kSlotFloats) {
            b.x0 = xa;
            b.w = wa;
            b.v4 = 1;
        }
    }
    return b;
}

typedef __attribute__((address_space(3))) void *lds_ptr_t;

// Stages box b of plane `plane` of x into lds ([h][w]) through LDS-DMA
// (buffer loads that write LDS directly, so a wave has every row of its share
// in flight at once); pixels outside the image are 0.  A row or column
// outside the image loads through an offset past the end of the plane.  A v4
// box moves 16 bytes per lane: one instruction covers 64 / (w / 4) whole rows
// (the LDS destination of lane i is 16 i bytes on, so rows land w floats
// apart), waves taking consecutive groups of rows in turn.  Otherwise 4 bytes
// per lane: wave w takes rows w, w + 4, ..., lane i column i of the row.  The
// wave issues stage_count(b) instructions and does not wait for them.
__device__ __forceinline__ void stage_plane(const float *x, size_t plane, int H, int W, const Box &b, float *dst) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const __amdgpu_buffer_rsrc_t r = plane_rsrc(x, plane, H, W);
    if (b.v4) {
        const int lpr = b.w >> 2, rpi = 64 / lpr;  // lanes per row, rows per instruction
        const int rl = lane / lpr, col = b.x0 + 4 * (lane - rl * lpr);
        const bool cok = col >= 0 && col < W && rl < rpi;
        for (int r0 = wave * rpi; r0 < b.h; r0 += (kThreads / 64) * rpi) {
            const int row = r0 + rl, sy = b.y0 + row;
            const bool ok = cok && sy >= 0 && sy < H;
            if (rl < rpi && row < b.h)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr_t)(dst + r0 * b.w), 16,
                                                         ok ? ((uint32_t)sy * (uint32_t)W + (uint32_t)col) * 4u : kOOB,
                                                         0, 0, 0);
        }
    } else {
        const int col = b.x0 + lane;
        const uint32_t voff = (col >= 0 && col < W) ? (uint32_t)col * 4u : kOOB;
        for (int row = wave; row < b.h; row += kThreads / 64) {
            const int sy = b.y0 + row;
            const bool ok = sy >= 0 && sy < H;
            if (lane < b.w)  // lane i lands at dst + row w + 4 i bytes
                __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr_t)(dst + row * b.w), 4, ok ? voff : kOOB,
                                                         ok ? sy * W * 4 : 0, 0, 0);
        }
    }
}

// Instructions stage_plane issues in this wave (uniform).
__device__ __forceinline__ int stage_count(const Box &b) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int step = b.v4 ? 64 / (b.w >> 2) : 1, first = wave * step, stride = (kThreads / 64) * step;
    return b.h > first ? (b.h - first + stride - 1) / stride : 0;
}

// Waits until at most n (uniform) of this wave's vector memory instructions
// are outstanding (n rounded down to a bucket: waiting for fewer is safe).
// Vector memory instructions complete in issue order, so the ones issued
// before the last n have then completed.
template <int N>
__device__ __forceinline__ void wait_vm() {
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}
__device__ __forceinline__ void wait_vm_at_most(int n) {
    if (n >= 48) wait_vm<48>();
    else if (n >= 32) wait_vm<32>();
    else if (n >= 24) wait_vm<24>();
    else if (n >= 16) wait_vm<16>();
    else if (n >= 12) wait_vm<12>();
    else if (n >= 8) wait_vm<8>();
    else if (n >= 4) wait_vm<4>();
    else wait_vm<0>();
}

// This thread's four pixels of the 32 x 32 output tile (column ox, rows oy0
// + 8k): bilinear fractions, the pixel's byte offset in a plane (kOOB outside
// the image), and the taps -- LDS box index of tap (0, 0), or global offsets.
struct PixSet {
    int ox, oy0;
    float fx[kPix], fy[kPix];
    uint32_t off[kPix];
    int bi[kPix];
    Taps t[kPix];
};

template <bool LDS>
__device__ __forceinline__ void pix_set(const Geo &g, int H, int W, int tile, const Box &b, PixSet &ps) {
    const int tiles_x = (W + kTile - 1) / kTile;
    const int X0 = (tile % tiles_x) * kTile, Y0 = (tile / tiles_x) * kTile;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    ps.ox = X0 + (lane & 31);
    ps.oy0 = Y0 + 2 * wave + (lane >> 5);
    double sx0, sy0;
    sample_pos(g, ps.ox, ps.oy0, sx0, sy0);
    // one row of output moves the sample point by (-sin, cos) / s
    const double dsx = -g.s_ * g.inv_s * kRowStep, dsy = g.c * g.inv_s * kRowStep;
#pragma unroll
    for (int k = 0; k < kPix; ++k) {
        const int oy = ps.oy0 + k * kRowStep;
        const double sx = sx0 + (double)k * dsx, sy = sy0 + (double)k * dsy;
        ps.off[k] = (ps.ox < W && oy < H) ? ((uint32_t)oy * (uint32_t)W + (uint32_t)ps.ox) * 4u : kOOB;
        if (LDS) {
            const double fx0 = floor(sx), fy0 = floor(sy);
            ps.fx[k] = (float)(sx - fx0);
            ps.fy[k] = (float)(sy - fy0);
            // inside the box by construction; the clamp only guards the LDS range
            const int lx = (int)fmin(fmax(fx0 - (double)b.x0, 0.0), (double)(b.w - 2));
            const int ly = (int)fmin(fmax(fy0 - (double)b.y0, 0.0), (double)(b.h - 2));
            ps.bi[k] = ly * b.w + lx;
        } else {
            ps.t[k] = taps_of(sx, sy, H, W);
            ps.fx[k] = ps.t[k].fx;
            ps.fy[k] = ps.t[k].fy;
        }
    }
}

// Channel c of this thread's four pixels from taps q, written to y.
__device__ __forceinline__ void fwd_store(float *y, size_t plane, int H, int W, const PixSet &ps, const Quad (&q)[kPix],
                                          float alpha, float beta, float gamma) {
    const __amdgpu_buffer_rsrc_t yr = plane_rsrc(y, plane, H, W);
#pragma unroll
    for (int k = 0; k < kPix; ++k) {
        const float w = bilerp(q[k], ps.fx[k], ps.fy[k]);
        const float z = alpha * w + beta;
        const float y1 = fminf(fmaxf(z, 0.0f), 1.0f);
        stf(yr, ps.off[k], y1 > 0.0f ? pow_pos(y1, gamma, __builtin_amdgcn_logf(y1)) : 0.0f);
    }
}

// One channel from a staged slot: the four taps of each pixel from LDS, kPix
// stores.  The LDS reads sit in one asm block that waits for them itself: the
// compiler cannot tell this slot's DMA from the other slot's (their issue
// counts are data-dependent), and would otherwise wait for every DMA in
// flight before the first read.
__device__ __forceinline__ void fwd_slot(float *y, size_t plane, int H, int W, const PixSet &ps, const Box &b,
                                         const float *slot, float alpha, float beta, float gamma) {
    static_assert(kPix == 4, "one asm block reads the taps of four pixels");
    uint32_t a[kPix], u[kPix];
#pragma unroll
    for (int k = 0; k < kPix; ++k) {
        a[k] = (uint32_t)(uintptr_t)(lds_ptr_t)(slot + ps.bi[k]);
        u[k] = a[k] + 4u * (uint32_t)b.w;
    }
    float2 r0, r1, r2, r3, r4, r5, r6, r7;
    asm volatile(
        "ds_read2_b32 %0, %8 offset1:1\n\t"
        "ds_read2_b32 %1, %9 offset1:1\n\t"
        "ds_read2_b32 %2, %10 offset1:1\n\t"
        "ds_read2_b32 %3, %11 offset1:1\n\t"
        "ds_read2_b32 %4, %12 offset1:1\n\t"
        "ds_read2_b32 %5, %13 offset1:1\n\t"
        "ds_read2_b32 %6, %14 offset1:1\n\t"
        "ds_read2_b32 %7, %15 offset1:1\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3), "=&v"(r4), "=&v"(r5), "=&v"(r6), "=&v"(r7)
        : "v"(a[0]), "v"(u[0]), "v"(a[1]), "v"(u[1]), "v"(a[2]), "v"(u[2]), "v"(a[3]), "v"(u[3])
        : "memory");
    const Quad q[kPix] = {Quad{r0.x, r0.y, r1.x, r1.y}, Quad{r2.x, r2.y, r3.x, r3.y}, Quad{r4.x, r4.y, r5.x, r5.y},
                          Quad{r6.x, r6.y, r7.x, r7.y}};
    fwd_store(y, plane, H, W, ps, q, alpha, beta, gamma);
}

// Footprint too large for a slot: taps gathered from global memory.
__device__ __forceinline__ void fwd_tile_global(const float *x, int img, int tile, int C, int H, int W, const float *p,
                                                const Geo &g, float *y) {
    PixSet ps;
    pix_set<false>(g, H, W, tile, Box{0, 0, 0, 0, 0}, ps);
    const float alpha = p[4], beta = p[5], gamma = p[6];
    for (int c = 0; c < C; ++c) {
        const size_t plane = (size_t)img * C + c;
        const __amdgpu_buffer_rsrc_t xr = plane_rsrc(x, plane, H, W);
        Quad q[kPix];
#pragma unroll
        for (int k = 0; k < kPix; ++k) q[k] = load_quad(xr, ps.t[k]);
        fwd_store(y, plane, H, W, ps, q, alpha, beta, gamma);
    }
}

// Geometry and source box of output tile `tile`, in LDS.
__device__ __forceinline__ void tile_setup(const float *p, int tile, int H, int W, bool al, Geo &sg, Box &sb) {
    if (threadIdx.x == 0) {
        const int tiles_x = (W + kTile - 1) / kTile;
        sg = make_geo(p, H, W);
        sb = tile_box(sg, (tile % tiles_x) * kTile, (tile / tiles_x) * kTile, al);
    }
    __syncthreads();
}

// Workgroup barrier without a memory fence (a fence would wait for every
// LDS-DMA in flight): the callers have waited for their own DMA, and for their
// LDS reads, themselves.  The memory clobber keeps the compiler from moving
// memory operations across it.
__device__ __forceinline__ void bare_barrier() { asm volatile("s_barrier" ::: "memory"); }

// Workgroup barrier for LDS written with ordinary stores, without the fence
// that would also wait for every LDS-DMA in flight.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Channels go through two LDS slots in turn: channel c + 1 (and, once its
// slot is free, c + 2) is in flight while channel c is blended and stored.
// The wait before channel c's blend lets the instructions issued after its
// DMA stay outstanding: the stores of channel c - 1 (kPix per thread) and the
// DMA of channel c + 1.  Two separate LDS arrays keep the compiler from
// waiting on the other slot's DMA when it reads one.
__global__ __launch_bounds__(kThreads) void k_wc_fwd(const float *__restrict__ x, int C, int H, int W,
                                                     const float *__restrict__ params, float *__restrict__ y) {
    __shared__ float slot0[kSlotFloats];
    __shared__ float slot1[kSlotFloats];
    __shared__ Geo sg;
    __shared__ Box sb;
    const int2 lb = xcd_block();  // (output tile, image): an image's tiles share one XCD's L2
    const int tile = lb.x, img = lb.y;
    const float *p = params + 7 * img;
    tile_setup(p, tile, H, W, (((uintptr_t)x & 15) | (W & 3)) == 0, sg, sb);
    const Box b = sb;
    if (b.w == 0) {
        fwd_tile_global(x, img, tile, C, H, W, p, sg, y);
        return;
    }
    const size_t pl0 = (size_t)img * C;
    stage_plane(x, pl0, H, W, b, slot0);
    if (C > 1) stage_plane(x, pl0 + 1, H, W, b, slot1);
    PixSet ps;
    pix_set<true>(sg, H, W, tile, b, ps);
    const float alpha = p[4], beta = p[5], gamma = p[6];
    const int n = stage_count(b);
    for (int c = 0; c < C; c += 2) {
        wait_vm_at_most((c > 0 ? kPix : 0) + (c + 1 < C ? n : 0));
        bare_barrier();
        fwd_slot(y, pl0 + c, H, W, ps, b, slot0, alpha, beta, gamma);
        if (c + 2 < C) {
            bare_barrier();  // every wave has read slot 0
            stage_plane(x, pl0 + c + 2, H, W, b, slot0);
        }
        if (c + 1 < C) {
            wait_vm_at_most(kPix + (c + 2 < C ? n : 0));
            bare_barrier();
            fwd_slot(y, pl0 + c + 1, H, W, ps, b, slot1, alpha, beta, gamma);
            if (c + 3 < C) {
                bare_barrier();
                stage_plane(x, pl0 + c + 3, H, W, b, slot1);
            }
        }
    }
}

// Integer span [lo, hi] of t for which a t + b lies in [v0, v1), given
// ia = 1 / a, widened by a hair (1e-6 px: the bounds are rounded products,
// the callers confirm every pixel with its cell) and clamped to [0, n - 1]
// (empty: lo > hi).
__device__ __forceinline__ int2 affine_span(double a, double ia, double b, double v0, double v1, int n) {
    double lo, hi;
    if (a > 0.0) {
        lo = (v0 - b) * ia;
        hi = (v1 - b) * ia;
    } else if (a < 0.0) {
        lo = (v1 - b) * ia;
        hi = (v0 - b) * ia;
    } else {
        if (b < v0 || b >= v1) return make_int2(1, 0);
        return make_int2(0, n - 1);
    }
    const double l = fmax(ceil(lo - 1e-6), 0.0), h = fmin(floor(hi + 1e-6), (double)(n - 1));
    return l > h ? make_int2(1, 0) : make_int2((int)l, (int)h);
}

// Along output row oy the sample point is (A ox + B, Cc ox + D).
struct RowMap {
    double A, iA, Cc, iC;
};

__device__ __forceinline__ RowMap row_map(const Geo &g) {
    RowMap r;
    r.A = g.c * g.inv_s;
    r.Cc = g.s_ * g.inv_s;
    r.iA = r.A != 0.0 ? 1.0 / r.A : 0.0;
    r.iC = r.Cc != 0.0 ? 1.0 / r.Cc : 0.0;
    return r;
}

// Output pixels of row oy whose sample point lies in [x0, x1) x [y0, y1)
// (a hair wider), clamped to the image (empty: .x > .y).
__device__ __forceinline__ int2 row_span(const Geo &g, const RowMap &m, int oy, double x0, double x1, double y0,
                                         double y1, int W) {
    const double Y = (double)oy - g.uy;
    const double B = (-g.c * g.ux - g.s_ * Y) * g.inv_s + g.cx;
    const double D = (-g.s_ * g.ux + g.c * Y) * g.inv_s + g.cy;
    const int2 a = affine_span(m.A, m.iA, B, x0, x1, W);
    const int2 b = affine_span(m.Cc, m.iC, D, y0, y1, W);
    return make_int2(max(a.x, b.x), min(a.y, b.y));
}

// Per-thread sums for the parameter gradients over the pixels a workgroup
// owns: v = {sum (g_sy rx - g_sx ry), sum (g_sx rx + g_sy ry), sum g_sx,
// sum g_sy, dL/dalpha, dL/dbeta, dL/dgamma}, (rx, ry) = (sx - cx, sy - cy).
struct ParAcc {
    float v[7];
};

// One output pixel of the region: dL/dw per channel into gw and, when the
// pixel is owned, its parameter-gradient terms into a.  With g_y = dL/dy and
// y1 in (0, 1]: dL/dgamma += g_y y ln y1; where z lies in (0, 1), with
// g_z = g_y gamma y / y1: dL/dw = g_z alpha, dL/dalpha += g_z w,
// dL/dbeta += g_z, (g_sx, g_sy) += dL/dw (dw/dsx, dw/dsy).
// quad(c) gives the pixel's taps in channel c, gvf(c) its dL/dy; (rx, ry) is
// its sample point relative to the image centre.
template <class QuadF, class GyF>
__device__ __forceinline__ void pixel_adjoint(int C, float fx, float fy, float rx, float ry, float alpha, float beta,
                                              float gamma, bool owned, QuadF quad, GyF gvf, float (&gw)[kMaxC],
                                              ParAcc &a) {
    float gsx = 0.0f, gsy = 0.0f;
#pragma unroll
    for (int c = 0; c < kMaxC; ++c) {
        gw[c] = 0.0f;
        if (c >= C) continue;
        const Quad q = quad(c);
        const float gv = gvf(c);
        const float w = bilerp(q, fx, fy);
        const float z = alpha * w + beta;
        const float y1 = fminf(fmaxf(z, 0.0f), 1.0f);
        if (y1 > 0.0f) {
            const float l2 = __builtin_amdgcn_logf(y1);
            const float yv = pow_pos(y1, gamma, l2);
            if (owned) a.v[6] += gv * yv * (l2 * 0.6931471805599453f);
            if (z < 1.0f) {
                const float gz = gv * gamma * (yv / y1);  // d(y1^gamma)/dy1 = gamma y1^(gamma-1)
                gw[c] = gz * alpha;
                if (owned) {
                    a.v[4] += gz * w;
                    a.v[5] += gz;
                    gsx += gw[c] * ((1.0f - fy) * (q.p01 - q.p00) + fy * (q.p11 - q.p10));
                    gsy += gw[c] * ((1.0f - fx) * (q.p10 - q.p00) + fx * (q.p11 - q.p01));
                }
            }
        }
    }
    if (owned) {
        a.v[0] += gsy * rx - gsx * ry;
        a.v[1] += gsx * rx + gsy * ry;
        a.v[2] += gsx;
        a.v[3] += gsy;
    }
}

constexpr int kEPT = 6;                         // region pixels per thread in the gather form
constexpr int kPoolFloats = 7936;               // 31 KB of sorted entries
constexpr int kMaxRows = 64;                    // region rows of the gather form (one wave scans them)
constexpr int kCellN = kCells * kCells;
constexpr int kScanPT = (kCellN + 1 + kThreads - 1) / kThreads;
constexpr int kRec = 12;                        // floats per workgroup record: 7 parameters, then kMaxC sums, pad

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// The backward, one workgroup per 32 x 32 source tile T at (X0, Y0):
//   0. the sum of dL/dy over the pixels of the output tile at (X0, Y0) (the
//      same grid) whose cell lies wholly outside the image;
//   1. the region -- output pixels whose bilinear cell has a tap in T, i.e.
//      cell corner in [X0-1, X0+31] x [Y0-1, Y0+31] -- row by row from the
//      affine map, flattened over the workgroup;
//   2. per region pixel, from T's taps staged in LDS ([X0-1, X0+32]^2): its
//      cell, fractions and dL/dw (recomputed in registers), counted per cell;
//      and, for the pixels T owns (cell corner in T, the first tile row and
//      column also owning corner -1), the parameter-gradient terms;
//   3. an exclusive scan of the 33 x 33 cell counts, the entries stored in
//      LDS sorted by cell;
//   4. each source pixel sums the entries of the four cells that have it as
//      a tap: two contiguous runs (the two cells of a row are adjacent in
//      the sorted order).  Every grad_x element has one writer: no global
//      atomics, no zero-fill, no dL/dw buffer.
// Output pixels whose cell has no tap in the image (w = 0, z = beta) belong
// to no source tile; their share of dL/dbeta and dL/dgamma depends only on
// the sum of their dL/dy, which step 0 forms over the output tile at the
// same grid position, the record carries, and k_wc_reduce applies.
// A region larger than the LDS pool (scale well above 1) takes its taps from
// global memory and scatters into an LDS accumulator with float atomics.
// With gx NULL only the parameter gradients are formed.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_wc_bwd(const float *__restrict__ x, int C, int H, int W,
                                                     const float *__restrict__ params,
                                                     const float *__restrict__ gy, float *__restrict__ gx,
                                                     float *__restrict__ rec) {
    // pool: T's taps [c][34][34] during step 2; then entries sorted by cell,
    // g[c][cap], fx[cap], fy[cap]; or the scatter form's accumulator [c][32][33]
    __shared__ float pool[kPoolFloats];
    __shared__ int off[kCellN + 1];  // per cell: entry count, then exclusive start
    __shared__ int rxa[kMaxRows], roff[kMaxRows + 1];
    __shared__ int wsum[kThreads / 64];
    __shared__ float red[kThreads / 64][kRec];
    __shared__ Geo sg;
    __shared__ int s_r0, s_nrows, s_total;
    const int2 lb = xcd_block();  // (source tile, image): an image's tiles share one XCD's L2
    const int tile = lb.x, img = lb.y;
    const int tiles_x = (W + kSrcTile - 1) / kSrcTile;
    const int X0 = (tile % tiles_x) * kSrcTile, Y0 = (tile / tiles_x) * kSrcTile;
    const float *p = params + 7 * img;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (threadIdx.x == 0) {
        const Geo g = make_geo(p, H, W);
        sg = g;
        // rows of the forward image of the cell square [X0-1, X0+32] x [Y0-1, Y0+32],
        // p_out = s R (p_src - c) + c + t, plus a margin
        double yl = 1e300, yh = -1e300;
        for (int k = 0; k < 4; ++k) {
            const double px = ((k & 1) ? (double)(X0 + kSrcTile) : (double)(X0 - 1)) - g.cx;
            const double py = ((k & 2) ? (double)(Y0 + kSrcTile) : (double)(Y0 - 1)) - g.cy;
            const double qy = g.scale * (-g.s_ * px + g.c * py) + g.uy;
            yl = fmin(yl, qy);
            yh = fmax(yh, qy);
        }
        const int r0 = (int)fmin(fmax(floor(yl) - 1.0, 0.0), (double)H);
        const int r1 = (int)fmax(fmin(ceil(yh) + 1.0, (double)(H - 1)), -1.0);
        s_r0 = r0;
        s_nrows = max(0, r1 - r0 + 1);
    }
    for (int i = threadIdx.x; i < kCellN + 1; i += kThreads) off[i] = 0;
    __syncthreads();
    const Geo &g = sg;
    const RowMap rm = row_map(g);
    const int r0 = s_r0, nrows = s_nrows;
    // 0. dL/dy summed over the pixels of the output tile at the same grid
    // position whose bilinear cell lies wholly outside the image.  Most tiles
    // have none, and their waves load nothing; a wave that has some loads
    // every channel of its four pixels at once (an offset past the plane reads
    // 0), before the tap DMA is issued, so that waiting for these loads does
    // not wait for the DMA.
    constexpr int kOwnPix = kSrcTile * kSrcTile / kThreads;
    uint32_t oo[kOwnPix];  // byte offset of such a pixel in a plane, else kOOB
    bool any_off = false;
#pragma unroll
    for (int j = 0; j < kOwnPix; ++j) {
        const int e = threadIdx.x + j * kThreads;
        const int u = X0 + (e & (kSrcTile - 1)), v = Y0 + e / kSrcTile;
        double sx, sy;
        sample_pos(g, u, v, sx, sy);
        const double fx0 = floor(sx), fy0 = floor(sy);
        const bool outside = fx0 < -1.0 || fx0 > (double)(W - 1) || fy0 < -1.0 || fy0 > (double)(H - 1);
        oo[j] = (u < W && v < H && outside) ? ((uint32_t)v * (uint32_t)W + (uint32_t)u) * 4u : kOOB;
        any_off |= oo[j] != kOOB;
    }
    float s_off[kMaxC] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (__builtin_amdgcn_ballot_w64(any_off) != 0) {  // uniform in the wave
        float ov[kOwnPix][kMaxC];
#pragma unroll
        for (int j = 0; j < kOwnPix; ++j)
#pragma unroll
            for (int c = 0; c < kMaxC; ++c)
                ov[j][c] = ldf(plane_rsrc(gy, (size_t)img * C + min(c, C - 1), H, W), c < C ? oo[j] : kOOB);
#pragma unroll
        for (int j = 0; j < kOwnPix; ++j)
#pragma unroll
            for (int c = 0; c < kMaxC; ++c) s_off[c] += ov[j][c];
    }
    // the tile's taps (34 x 34 per channel around it): their DMA is in flight
    // through step 1 and the region's positions and dL/dy loads, and waited
    // for before the first tap is read (or before the scatter form reuses the
    // pool); the barriers until then wait for LDS stores only
    constexpr int kXT = kCells + 1;
    {
        const Box tb{X0 - 1, Y0 - 1, kXT, kXT, 0};
        for (int c = 0; c < C; ++c) stage_plane(x, (size_t)img * C + c, H, W, tb, pool + c * kXT * kXT);
    }
    const double tx0 = (double)(X0 - 1), tx1 = (double)(X0 + kSrcTile);
    const double ty0 = (double)(Y0 - 1), ty1 = (double)(Y0 + kSrcTile);
    if (wave == 0) {
        int xa = 0, len = 0;
        if (lane < nrows) {
            const int2 sp = row_span(g, rm, r0 + lane, tx0, tx1, ty0, ty1, W);
            xa = sp.x;
            len = max(0, sp.y - sp.x + 1);
        }
        const int inc = wave_incl_scan(len, lane);
        rxa[lane] = xa;
        roff[lane + 1] = inc;
        if (lane == 0) roff[0] = 0;
        if (lane == 63) s_total = nrows > kMaxRows ? INT_MAX : inc;
    }
    lds_barrier();
    const float alpha = p[4], beta = p[5], gamma = p[6];
    const int total = s_total;
    const int cap = min(kEPT * kThreads, kPoolFloats / (C + 2));
    // owned cell corners, relative to the cell square: [own_x0, own_x1] x [own_y0, own_y1]
    const int own_x0 = X0 == 0 ? 0 : 1, own_x1 = min(kCells - 1, W - X0);
    const int own_y0 = Y0 == 0 ? 0 : 1, own_y1 = min(kCells - 1, H - Y0);
    ParAcc acc;
#pragma unroll
    for (int k = 0; k < 7; ++k) acc.v[k] = 0.0f;
    if (total <= cap) {
        // 2. region pixels: positions and cells first, then every dL/dy load of
        // the thread's pixels in flight together, then the arithmetic
        uint32_t eop[kEPT];  // the pixel's byte offset in a plane; kOOB: no pixel, or a cell outside the square
        int einf[kEPT];      // tap index in the staged tile | cell index << 11 | owned << 22
        float efx[kEPT], efy[kEPT], erx[kEPT], ery[kEPT];
#pragma unroll
        for (int k = 0; k < kEPT; ++k) {
            const int e = threadIdx.x + k * kThreads;
            eop[k] = kOOB;
            einf[k] = 0;
            efx[k] = efy[k] = erx[k] = ery[k] = 0.0f;
            if (e >= total) continue;
            int r = 0;  // the last row whose start is at or before e
#pragma unroll
            for (int st = kMaxRows / 2; st > 0; st >>= 1)
                if (r + st < nrows && roff[r + st] <= e) r += st;
            const int oy = r0 + r, ox = rxa[r] + (e - roff[r]);
            double sx, sy;
            sample_pos(g, ox, oy, sx, sy);
            const double fx0 = floor(sx), fy0 = floor(sy);
            const double dcx = fx0 - tx0, dcy = fy0 - ty0;  // cell relative to the cell square
            if (!(dcx >= 0.0 && dcx < (double)kCells && dcy >= 0.0 && dcy < (double)kCells)) continue;
            const int cx = (int)dcx, cy = (int)dcy;
            const bool owned = cx >= own_x0 && cx <= own_x1 && cy >= own_y0 && cy <= own_y1;
            eop[k] = ((uint32_t)oy * (uint32_t)W + (uint32_t)ox) * 4u;
            einf[k] = (cy * kXT + cx) | ((cy * kCells + cx) << 11) | ((int)owned << 22);
            efx[k] = (float)(sx - fx0);
            efy[k] = (float)(sy - fy0);
            erx[k] = (float)(sx - g.cx);
            ery[k] = (float)(sy - g.cy);
        }
        float egv[kEPT][kMaxC];
#pragma unroll
        for (int k = 0; k < kEPT; ++k)
#pragma unroll
            for (int c = 0; c < kMaxC; ++c)
                egv[k][c] = c < C ? ldf(plane_rsrc(gy, (size_t)img * C + c, H, W), eop[k]) : 0.0f;
        __builtin_amdgcn_s_waitcnt(0);  // this wave's tap DMA and dL/dy loads
        lds_barrier();                  // every wave's taps
        float eg[kEPT][kMaxC];
        int ecs[kEPT];
#pragma unroll
        for (int k = 0; k < kEPT; ++k) {
            ecs[k] = -1;
#pragma unroll
            for (int c = 0; c < kMaxC; ++c) eg[k][c] = 0.0f;
            if (eop[k] == kOOB) continue;
            const int bi = einf[k] & 2047;
            pixel_adjoint(
                C, efx[k], efy[k], erx[k], ery[k], alpha, beta, gamma, (einf[k] >> 22) != 0,
                [&](int c) {
                    const float *q = pool + c * kXT * kXT + bi;
                    return Quad{q[0], q[1], q[kXT], q[kXT + 1]};
                },
                [&](int c) { return egv[k][c]; }, eg[k], acc);
            if (gx) {
                const int ci = (einf[k] >> 11) & 2047;
                ecs[k] = (atomicAdd(&off[ci], 1) << 11) | ci;
            }
        }
        if (gx) {
            __syncthreads();
            // 3. exclusive scan of the cell counts (off[kCellN] becomes the entry count)
            {
                int v[kScanPT], s = 0;
#pragma unroll
                for (int j = 0; j < kScanPT; ++j) {
                    const int i = threadIdx.x * kScanPT + j;
                    v[j] = i < kCellN ? off[i] : 0;
                    s += v[j];
                }
                const int inc = wave_incl_scan(s, lane);
                if (lane == 63) wsum[wave] = inc;
                __syncthreads();
                int base = inc - s;
                for (int w = 0; w < wave; ++w) base += wsum[w];
#pragma unroll
                for (int j = 0; j < kScanPT; ++j) {
                    const int i = threadIdx.x * kScanPT + j;
                    if (i <= kCellN) off[i] = base;
                    base += v[j];
                }
            }
            __syncthreads();
            float *pg = pool, *pfx = pool + C * cap, *pfy = pool + (C + 1) * cap;
#pragma unroll
            for (int k = 0; k < kEPT; ++k) {
                if (ecs[k] < 0) continue;
                const int pos = off[ecs[k] & 2047] + (ecs[k] >> 11);
#pragma unroll
                for (int c = 0; c < kMaxC; ++c)
                    if (c < C) pg[c * cap + pos] = eg[k][c];
                pfx[pos] = efx[k];
                pfy[pos] = efy[k];
            }
            __syncthreads();
            // 4. every source pixel sums the entries of its four cells
#pragma unroll
            for (int j = 0; j < kSrcTile * kSrcTile / kThreads; ++j) {
                const int e = threadIdx.x + j * kThreads;
                const int lu = e & (kSrcTile - 1), lv = e / kSrcTile;
                const int u = X0 + lu, v = Y0 + lv;
                float sum[kMaxC] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int dy = 0; dy < 2; ++dy) {
                    // cell row lv + dy has corner y0 = v - 1 + dy: the pixel is its tap row 1 - dy
                    const int ci = (lv + dy) * kCells + lu;
                    const int a0 = off[ci], mid = off[ci + 1], b0 = off[ci + 2];
                    for (int q = a0; q < b0; ++q) {
                        const float fx = pfx[q], fy = pfy[q];
                        const float wx = q < mid ? fx : 1.0f - fx;  // left cell: corner x0 = u - 1
                        const float wy = dy == 0 ? fy : 1.0f - fy;
                        const float wt = wy * wx;
#pragma unroll
                        for (int c = 0; c < kMaxC; ++c)
                            if (c < C) sum[c] += pg[c * cap + q] * wt;
                    }
                }
                const uint32_t o = (u < W && v < H) ? ((uint32_t)v * (uint32_t)W + (uint32_t)u) * 4u : kOOB;
#pragma unroll
                for (int c = 0; c < kMaxC; ++c)
                    if (c < C) stf(plane_rsrc(gx, (size_t)img * C + c, H, W), o, sum[c]);
            }
        }
    } else {
        // a region beyond the pool: taps from global memory, scatter with LDS float atomics
        float(*accs)[kSrcTile][kSrcTile + 1] = reinterpret_cast<float(*)[kSrcTile][kSrcTile + 1]>(pool);
        __builtin_amdgcn_s_waitcnt(0);  // the tap DMA has landed before the pool is reused
        lds_barrier();
        if (gx)
            for (int e = threadIdx.x; e < kMaxC * kSrcTile * (kSrcTile + 1); e += kThreads) pool[e] = 0.0f;
        __syncthreads();
        for (int oy = r0 + wave; oy < r0 + nrows; oy += kThreads / 64) {
            const int2 sp = row_span(g, rm, oy, tx0, tx1, ty0, ty1, W);
            for (int ox = sp.x + lane; ox <= sp.y; ox += 64) {
                double sx, sy;
                sample_pos(g, ox, oy, sx, sy);
                const double fx0 = floor(sx), fy0 = floor(sy);
                if (!(fx0 >= tx0 && fx0 < tx1 && fy0 >= ty0 && fy0 < ty1)) continue;
                const int cx = (int)(fx0 - tx0), cy = (int)(fy0 - ty0);
                const bool owned = cx >= own_x0 && cx <= own_x1 && cy >= own_y0 && cy <= own_y1;
                const Taps t = taps_of(sx, sy, H, W);
                const uint32_t opix = ((uint32_t)oy * (uint32_t)W + (uint32_t)ox) * 4u;
                float gw[kMaxC];
                pixel_adjoint(
                    C, t.fx, t.fy, (float)(sx - g.cx), (float)(sy - g.cy), alpha, beta, gamma, owned,
                    [&](int c) { return load_quad(plane_rsrc(x, (size_t)img * C + c, H, W), t); },
                    [&](int c) { return ldf(plane_rsrc(gy, (size_t)img * C + c, H, W), opix); }, gw, acc);
                if (!gx) continue;
                const float wt[4] = {(1.0f - t.fy) * (1.0f - t.fx), (1.0f - t.fy) * t.fx, t.fy * (1.0f - t.fx),
                                     t.fy * t.fx};
#pragma unroll
                for (int c = 0; c < kMaxC; ++c) {
                    if (c >= C || gw[c] == 0.0f) continue;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int yy = cy - 1 + (q >> 1), xx = cx - 1 + (q & 1);
                        if (yy >= 0 && yy < kSrcTile && xx >= 0 && xx < kSrcTile)
                            atomicAdd(&accs[c][yy][xx], gw[c] * wt[q]);
                    }
                }
            }
        }
        __syncthreads();
        if (gx)
            for (int e = threadIdx.x; e < C * kSrcTile * kSrcTile; e += kThreads) {
                const int c = e / (kSrcTile * kSrcTile), r = (e / kSrcTile) % kSrcTile, q = e % kSrcTile;
                if (Y0 + r < H && X0 + q < W) gx[(((size_t)img * C + c) * H + Y0 + r) * W + X0 + q] = accs[c][r][q];
            }
    }
    // the workgroup's record: parameter partials, and per channel the dL/dy sum
    // of its output tile's pixels whose cell lies outside the image
#pragma unroll
    for (int k = 0; k < kRec; ++k) {
        float v = 0.0f;
        if (k < 7) v = acc.v[k];
#pragma unroll
        for (int c = 0; c < kMaxC; ++c)
            if (k == 7 + c) v = s_off[c];
        const float t = wave_sum(v);
        if (lane == 0) red[wave][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < kRec) {
        const int t = threadIdx.x;
        auto sum = [&](int k) { return red[0][k] + red[1][k] + red[2][k] + red[3][k]; };
        const float is = (float)g.inv_s, c = (float)g.c, sn = (float)g.s_;
        float o;
        if (t == 0) o = sum(0) * 0.017453292519943295f;                     // angle (degrees)
        else if (t == 1) o = -sum(1) * is;                                 // scale
        else if (t == 2) o = -(c * sum(2) + sn * sum(3)) * is * (float)W;  // tx
        else if (t == 3) o = (sn * sum(2) - c * sum(3)) * is * (float)H;   // ty
        else o = sum(t);                                                   // alpha, beta, gamma, dL/dy sums
        rec[((size_t)img * gridDim.x + tile) * kRec + t] = o;
    }
}

// Sums the workgroup records of one image (lane l takes records l, l + 64,
// ... in order, then a fixed butterfly over the wave, in double) and adds
// the share of the output pixels whose cell has no tap in the image: w = 0,
// z = beta, so with S their dL/dy sum over channels, dL/dgamma gains
// S y ln y1 and, for beta in (0, 1), dL/dbeta gains S gamma y / y1.
__global__ __launch_bounds__(64) void k_wc_reduce(const float *__restrict__ rec, int blocks, int C,
                                                  const float *__restrict__ params, float *__restrict__ gp) {
    const int img = blockIdx.x, lane = threadIdx.x;
    double s[kRec];
#pragma unroll
    for (int k = 0; k < kRec; ++k) s[k] = 0.0;
    for (int b = lane; b < blocks; b += 64) {
        const float *q = rec + ((size_t)img * blocks + b) * kRec;
#pragma unroll
        for (int k = 0; k < kRec; ++k) s[k] += (double)q[k];
    }
#pragma unroll
    for (int k = 0; k < kRec; ++k)
        for (int o = 32; o > 0; o >>= 1) s[k] += __shfl_xor(s[k], o, 64);
    if (lane == 0) {
        double off = 0.0;
#pragma unroll
        for (int c = 0; c < kMaxC; ++c)
            if (c < C) off += s[7 + c];
        const float *p = params + 7 * img;
        const float beta = p[5], gamma = p[6];
        const float y1 = fminf(fmaxf(beta, 0.0f), 1.0f);
        if (y1 > 0.0f) {
            const float l2 = __builtin_amdgcn_logf(y1);
            const float yv = pow_pos(y1, gamma, l2);
            s[6] += off * (double)(yv * (l2 * 0.6931471805599453f));
            if (beta < 1.0f) s[5] += off * (double)(gamma * (yv / y1));
        }
#pragma unroll
        for (int k = 0; k < 7; ++k) gp[img * 7 + k] = (float)s[k];
    }
}

constexpr int kMaxGridY = 65535;

}  // namespace

hipError_t launch_wc_fwd(const float *x, int n, int C, int H, int W, const float *p, float *y, hipStream_t s) {
    const int tiles = ((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
    const size_t img = (size_t)C * H * W;
    for (int i0 = 0; i0 < n; i0 += kMaxGridY) {
        const int m = min(n - i0, kMaxGridY);
        hipLaunchKernelGGL(k_wc_fwd, dim3(tiles, m), dim3(kThreads), 0, s, x + i0 * img, C, H, W, p + 7 * (size_t)i0,
                           y + i0 * img);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t wc_workspace_bytes(int n, int C, int H, int W) {
    (void)C;
    const size_t tiles = (size_t)((W + kSrcTile - 1) / kSrcTile) * ((H + kSrcTile - 1) / kSrcTile);
    return (size_t)n * tiles * kRec * sizeof(float);
}

hipError_t launch_wc_bwd(const float *x, int n, int C, int H, int W, const float *p, const float *gy, float *gx,
                         float *gp, void *ws, hipStream_t s) {
    if (C > kMaxC) return hipErrorInvalidValue;
    const int st = ((W + kSrcTile - 1) / kSrcTile) * ((H + kSrcTile - 1) / kSrcTile);
    const size_t img = (size_t)C * H * W;
    for (int i0 = 0; i0 < n; i0 += kMaxGridY) {
        const int m = min(n - i0, kMaxGridY);
        hipLaunchKernelGGL(k_wc_bwd, dim3(st, m), dim3(kThreads), 0, s, x + i0 * img, C, H, W, p + 7 * (size_t)i0,
                           gy + i0 * img, gx ? gx + i0 * img : nullptr, (float *)ws + (size_t)i0 * st * kRec);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_wc_reduce, dim3(n), dim3(64), 0, s, (const float *)ws, st, C, p, gp);
    return hipGetLastError();
}

}  // namespace miaug
