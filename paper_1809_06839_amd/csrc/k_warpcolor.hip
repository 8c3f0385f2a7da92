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
// in float32 (no contraction); the forward and the backward evaluate the
// positions with the same function, so both see the same bilinear cells.
//
// Backward:
//   k_wc_bwd_pix  one thread per output pixel: dL/dw per channel (stored in
//                 the workspace) and the pixel's contributions to the 7
//                 parameter gradients, reduced over the wavefront (shuffles)
//                 and the workgroup (LDS) into one partial per workgroup;
//   k_wc_bwd_img  the adjoint of the bilinear warp, owned per source tile: a
//                 workgroup scans the output pixels whose sample point can
//                 reach its tile (the forward image of the tile, plus a
//                 margin), accumulates their weighted dL/dw in LDS and stores
//                 the tile once -- every grad_x element has exactly one
//                 writer, so no global atomics and no zero-fill are needed;
//   k_wc_reduce   sums the per-workgroup partials of each image in a fixed
//                 order (double accumulators).
#include "dev_common.h"
#include "internal.h"

namespace miaug {
namespace {

constexpr int kThreads = 256;
constexpr int kTile = 16;                // output tile of the per-pixel kernels is 16 x 16
constexpr int kSrcTile = 32;             // source tile of the adjoint kernel
constexpr int kMaxC = 4;

// Per-image geometry in double.  Sample positions are evaluated in double
// because a float32 position alone carries up to 2^-17 relative error (about
// 1e-5 px at x ~ 200), which the zero border and the gamma curve would turn
// into value errors above 1e-5.  One thread per workgroup computes it.
struct Geo {
    double c, s_, inv_s, cx, cy, ux, uy, scale;
};

__device__ __forceinline__ Geo make_geo(const float *p, int H, int W) {
    Geo g;
    const double th = (double)p[0] * (3.14159265358979323846 / 180.0);
    g.c = cos(th);
    g.s_ = sin(th);
    g.scale = (double)p[1];
    g.inv_s = 1.0 / g.scale;
    g.cx = 0.5 * (double)(W - 1);
    g.cy = 0.5 * (double)(H - 1);
    g.ux = g.cx + (double)p[2] * (double)W;
    g.uy = g.cy + (double)p[3] * (double)H;
    return g;
}

// Bilinear cell and weights of output pixel (x, y); X, Y are its offsets
// from the shifted centre (used by the parameter chain rule).
struct Cell {
    int x0, y0;
    float fx, fy;
    double X, Y;
};

__device__ __forceinline__ Cell cell_of(const Geo &g, int x, int y) {
    Cell k;
    k.X = (double)x - g.ux;
    k.Y = (double)y - g.uy;
    const double sx = (g.c * k.X - g.s_ * k.Y) * g.inv_s + g.cx;
    const double sy = (g.s_ * k.X + g.c * k.Y) * g.inv_s + g.cy;
    const double fx0 = floor(sx), fy0 = floor(sy);
    k.x0 = (int)fx0;
    k.y0 = (int)fy0;
    k.fx = (float)(sx - fx0);
    k.fy = (float)(sy - fy0);
    return k;
}

__device__ __forceinline__ float ztap(const float *img, int H, int W, int yy, int xx) {
    return (yy >= 0 && yy < H && xx >= 0 && xx < W) ? img[(size_t)yy * W + xx] : 0.0f;
}

__global__ __launch_bounds__(kThreads) void k_wc_fwd(const float *__restrict__ x, int C, int H, int W,
                                                     const float *__restrict__ params, float *__restrict__ y) {
    const int img = blockIdx.z;
    const int tiles_x = (W + kTile - 1) / kTile;
    const int ox = (blockIdx.x % tiles_x) * kTile + (threadIdx.x & (kTile - 1));
    const int oy = (blockIdx.x / tiles_x) * kTile + (threadIdx.x / kTile);
    const float *p = params + 7 * img;
    __shared__ Geo sg;
    if (threadIdx.x == 0) sg = make_geo(p, H, W);
    __syncthreads();
    if (ox >= W || oy >= H) return;
    const Cell k = cell_of(sg, ox, oy);
    const int x0 = k.x0, y0 = k.y0;
    const float fx = k.fx, fy = k.fy;
    const float alpha = p[4], beta = p[5], gamma = p[6];
    for (int c = 0; c < C; ++c) {
        const float *xc = x + ((size_t)img * C + c) * H * W;
        const float p00 = ztap(xc, H, W, y0, x0), p01 = ztap(xc, H, W, y0, x0 + 1);
        const float p10 = ztap(xc, H, W, y0 + 1, x0), p11 = ztap(xc, H, W, y0 + 1, x0 + 1);
        const float w = (1.0f - fy) * ((1.0f - fx) * p00 + fx * p01) + fy * ((1.0f - fx) * p10 + fx * p11);
        const float z = alpha * w + beta;
        const float y1 = fminf(fmaxf(z, 0.0f), 1.0f);
        y[(((size_t)img * C + c) * H + oy) * W + ox] = y1 > 0.0f ? (gamma == 1.0f ? y1 : powf(y1, gamma)) : 0.0f;
    }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ __launch_bounds__(kThreads) void k_wc_bwd_pix(const float *__restrict__ x, int C, int H, int W,
                                                         const float *__restrict__ params,
                                                         const float *__restrict__ gy, float *__restrict__ gw,
                                                         float *__restrict__ partial) {
    __shared__ float red[kThreads / 64][8];
    const int img = blockIdx.z;
    const int tiles_x = (W + kTile - 1) / kTile;
    const int ox = (blockIdx.x % tiles_x) * kTile + (threadIdx.x & (kTile - 1));
    const int oy = (blockIdx.x / tiles_x) * kTile + (threadIdx.x / kTile);
    const float *p = params + 7 * img;
    __shared__ Geo sg;
    if (threadIdx.x == 0) sg = make_geo(p, H, W);
    __syncthreads();
    const Geo &g = sg;
    float acc[7] = {0, 0, 0, 0, 0, 0, 0};
    if (ox < W && oy < H) {
        const Cell k = cell_of(g, ox, oy);
        const int x0 = k.x0, y0 = k.y0;
        const float fx = k.fx, fy = k.fy;
        const float alpha = p[4], beta = p[5], gamma = p[6];
        float gsx = 0.0f, gsy = 0.0f;  // dL/dsx, dL/dsy summed over channels
        for (int c = 0; c < C; ++c) {
            const size_t plane = ((size_t)img * C + c) * H * W;
            const float *xc = x + plane;
            const float p00 = ztap(xc, H, W, y0, x0), p01 = ztap(xc, H, W, y0, x0 + 1);
            const float p10 = ztap(xc, H, W, y0 + 1, x0), p11 = ztap(xc, H, W, y0 + 1, x0 + 1);
            const float w = (1.0f - fy) * ((1.0f - fx) * p00 + fx * p01) + fy * ((1.0f - fx) * p10 + fx * p11);
            const float z = alpha * w + beta;
            const float y1 = fminf(fmaxf(z, 0.0f), 1.0f);
            const float gv = gy[plane + (size_t)oy * W + ox];
            float gwv = 0.0f;
            if (y1 > 0.0f) {
                const float yv = gamma == 1.0f ? y1 : powf(y1, gamma);
                acc[6] += gv * yv * logf(y1);
                if (z > 0.0f && z < 1.0f) {
                    const float gz = gv * gamma * (gamma == 1.0f ? 1.0f : powf(y1, gamma - 1.0f));
                    acc[4] += gz * w;
                    acc[5] += gz;
                    gwv = gz * alpha;
                    gsx += gwv * ((1.0f - fy) * (p01 - p00) + fy * (p11 - p10));
                    gsy += gwv * ((1.0f - fx) * (p10 - p00) + fx * (p11 - p01));
                }
            }
            gw[plane + (size_t)oy * W + ox] = gwv;
        }
        // chain through (sx, sy)(angle_deg, scale, tx, ty)
        const float is = (float)g.inv_s, d2r = 0.017453292519943295f, c = (float)g.c, sn = (float)g.s_;
        const float rx = (float)((g.c * k.X - g.s_ * k.Y) * g.inv_s);  // rotated, scaled offsets
        const float ry = (float)((g.s_ * k.X + g.c * k.Y) * g.inv_s);
        acc[0] += (gsx * (-ry) + gsy * rx) * d2r;
        acc[1] += (gsx * (-rx) + gsy * (-ry)) * is;
        acc[2] += (gsx * (-c) + gsy * (-sn)) * is * (float)W;
        acc[3] += (gsx * sn + gsy * (-c)) * is * (float)H;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        const float v = wave_sum(acc[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
        float v = 0.0f;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) v += red[w][threadIdx.x];
        partial[((size_t)img * gridDim.x + blockIdx.x) * 8 + threadIdx.x] = v;
    }
}

// Adjoint of the bilinear warp, one source tile per workgroup (all channels).
__global__ __launch_bounds__(kThreads) void k_wc_bwd_img(int C, int H, int W, const float *__restrict__ params,
                                                         const float *__restrict__ gw, float *__restrict__ gx) {
    __shared__ float acc[kMaxC][kSrcTile][kSrcTile + 1];
    const int img = blockIdx.z;
    const int tiles_x = (W + kSrcTile - 1) / kSrcTile;
    const int X0 = (blockIdx.x % tiles_x) * kSrcTile, Y0 = (blockIdx.x / tiles_x) * kSrcTile;
    const float *p = params + 7 * img;
    __shared__ Geo sg;
    if (threadIdx.x == 0) sg = make_geo(p, H, W);
    for (int e = threadIdx.x; e < kMaxC * kSrcTile * (kSrcTile + 1); e += kThreads) (&acc[0][0][0])[e] = 0.0f;
    __syncthreads();
    const Geo &g = sg;
    // Output pixels that can sample this tile: the forward image of the tile
    // grown by one pixel (bilinear footprint), mapped with the forward map
    // p_out = s R (p_src - c) + c + t, plus a 2-pixel margin for float rounding.
    float bx0 = 1e30f, bx1 = -1e30f, by0 = 1e30f, by1 = -1e30f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float px = (k & 1) ? (float)(X0 + kSrcTile) : (float)(X0 - 1);
        const float py = (k & 2) ? (float)(Y0 + kSrcTile) : (float)(Y0 - 1);
        const float dx = px - (float)g.cx, dy = py - (float)g.cy;
        const float c = (float)g.c, sn = (float)g.s_, sc = (float)g.scale;
        const float qx = sc * (c * dx + sn * dy) + (float)g.ux;
        const float qy = sc * (-sn * dx + c * dy) + (float)g.uy;
        bx0 = fminf(bx0, qx); bx1 = fmaxf(bx1, qx);
        by0 = fminf(by0, qy); by1 = fmaxf(by1, qy);
    }
    const int ox0 = max(0, (int)floorf(bx0) - 2), ox1 = min(W - 1, (int)ceilf(bx1) + 2);
    const int oy0 = max(0, (int)floorf(by0) - 2), oy1 = min(H - 1, (int)ceilf(by1) + 2);
    __syncthreads();
    const int bw = ox1 - ox0 + 1;
    const int cnt = (ox1 >= ox0 && oy1 >= oy0) ? bw * (oy1 - oy0 + 1) : 0;
    for (int e = threadIdx.x; e < cnt; e += kThreads) {
        const int oy = oy0 + e / bw, ox = ox0 + e % bw;
        const Cell k = cell_of(g, ox, oy);
        const int x0 = k.x0 - X0, y0 = k.y0 - Y0;
        if (x0 < -1 || x0 >= kSrcTile || y0 < -1 || y0 >= kSrcTile) continue;
        const float fx = k.fx, fy = k.fy;
        const float wt[4] = {(1.0f - fy) * (1.0f - fx), (1.0f - fy) * fx, fy * (1.0f - fx), fy * fx};
        for (int c = 0; c < C; ++c) {
            const float gv = gw[(((size_t)img * C + c) * H + oy) * W + ox];
            if (gv == 0.0f) continue;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int ty = y0 + (k >> 1), tx = x0 + (k & 1);
                if (ty >= 0 && ty < kSrcTile && tx >= 0 && tx < kSrcTile && Y0 + ty < H && X0 + tx < W)
                    atomicAdd(&acc[c][ty][tx], gv * wt[k]);
            }
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < C * kSrcTile * kSrcTile; e += kThreads) {
        const int c = e / (kSrcTile * kSrcTile), r = (e / kSrcTile) % kSrcTile, q = e % kSrcTile;
        if (Y0 + r < H && X0 + q < W) gx[(((size_t)img * C + c) * H + Y0 + r) * W + X0 + q] = acc[c][r][q];
    }
}

__global__ void k_wc_reduce(const float *__restrict__ partial, int blocks, float *__restrict__ gp) {
    const int img = blockIdx.x, k = threadIdx.x;
    if (k >= 7) return;
    double s = 0.0;
    for (int b = 0; b < blocks; ++b) s += (double)partial[((size_t)img * blocks + b) * 8 + k];
    gp[img * 7 + k] = (float)s;
}

}  // namespace

hipError_t launch_wc_fwd(const float *x, int n, int C, int H, int W, const float *p, float *y, hipStream_t s) {
    const int tiles = ((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_wc_fwd, dim3(tiles, 1, n), dim3(kThreads), 0, s, x, C, H, W, p, y);
    return hipGetLastError();
}

size_t wc_workspace_bytes(int n, int C, int H, int W) {
    const size_t tiles = (size_t)((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
    return (size_t)n * C * H * W * sizeof(float) + (size_t)n * tiles * 8 * sizeof(float);
}

hipError_t launch_wc_bwd(const float *x, int n, int C, int H, int W, const float *p, const float *gy, float *gx,
                         float *gp, void *ws, hipStream_t s) {
    if (C > kMaxC) return hipErrorInvalidValue;
    const int tiles = ((W + kTile - 1) / kTile) * ((H + kTile - 1) / kTile);
    float *gw = (float *)ws;
    float *partial = gw + (size_t)n * C * H * W;
    hipLaunchKernelGGL(k_wc_bwd_pix, dim3(tiles, 1, n), dim3(kThreads), 0, s, x, C, H, W, p, gy, gw, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (gx) {
        const int st = ((W + kSrcTile - 1) / kSrcTile) * ((H + kSrcTile - 1) / kSrcTile);
        hipLaunchKernelGGL(k_wc_bwd_img, dim3(st, 1, n), dim3(kThreads), 0, s, C, H, W, p, gw, gx);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_wc_reduce, dim3(n), dim3(64), 0, s, partial, tiles, gp);
    return hipGetLastError();
}

}  // namespace miaug
