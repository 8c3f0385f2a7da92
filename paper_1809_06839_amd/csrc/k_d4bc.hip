// k_d4bc.hip -- random Dih4 element + colour LUTs on a dense u8 batch
// (Sec. II-B Dih4 transforms; Table I HorizontalFlip, VerticalFlip,
// Brightness, ShiftRGB, Grayscale).
//
// One workgroup per (image, 64x64 output tile).  The tile's source block is
// an axis-aligned rectangle (a Dih4 element maps rectangles to rectangles);
// its rows are staged into LDS with 16-byte LDS-DMA loads (all of a thread's
// chunks in flight at once; rows contiguous in LDS, so the lane-ordered DMA
// destinations tile them), the 256-entry LUT
// is built in LDS in IEEE double, and each thread forms four output pixels
// (each one LDS word read at the Dih4-mapped position, then the LUTs) and
// writes them as C aligned words (flips and transposes become LDS
// addressing).  HBM traffic is one read and one write of every byte.
#include "dev_common.h"
#include "internal.h"

namespace miaug {
namespace {

constexpr int kT = 64;
constexpr int kThreads = 256;
typedef __attribute__((address_space(3))) void *lds_ptr_t;

// FROM_AB: one LUT per image built from (alpha, beta); otherwise C LUTs per
// image read from `luts` ([n][C][256], composed on the host) and, for C = 3,
// an optional per-image grayscale flag applied after them.
template <int C, bool FROM_AB>
__global__ __launch_bounds__(kThreads) void k_d4_bc(const uint8_t *__restrict__ in, int H, int W,
                                                   const int32_t *__restrict__ flags, const float *__restrict__ ab,
                                                   const uint8_t *__restrict__ luts, const int32_t *__restrict__ gray,
                                                   uint8_t *__restrict__ out) {
    constexpr int kChunks = (kT * C + 30) / 16;          // 16-byte chunks per staged row (phase included)
    constexpr int kStride = kChunks * 16;                // LDS bytes per row
    constexpr int kLuts = FROM_AB ? 1 : C;
    __shared__ __align__(16) uint8_t src[kT * kStride + 16];  // + the word past the last pixel a read takes
    __shared__ uint8_t lut[kLuts][256];

    const int img = blockIdx.y;
    const int tid = threadIdx.x;
    const int32_t *fl = flags + 4 * img;
    const D4Map m = make_d4(H, W, fl[0], fl[1], fl[2], fl[3]);
    const int Ho = m.oh, Wo = m.ow;
    const int tiles_x = (Wo + kT - 1) / kT;
    const int r0 = (blockIdx.x / tiles_x) * kT, c0 = (blockIdx.x % tiles_x) * kT;
    if (r0 >= Ho) return;
    const int th = min(kT, Ho - r0), tw = min(kT, Wo - c0);

    const int ya = m.sy(r0, c0), yb = m.sy(r0 + th - 1, c0 + tw - 1);
    const int xa = m.sx(r0, c0), xb = m.sx(r0 + th - 1, c0 + tw - 1);
    const int sr0 = min(ya, yb), nsr = abs(yb - ya) + 1;
    const int sc0 = min(xa, xb), nsc = abs(xb - xa) + 1;
    const size_t plane = (size_t)H * W * C;
    const uint8_t *base = in + (size_t)img * plane;

    // stage source rows [sr0, sr0 + nsr), columns [sc0, sc0 + nsc): chunk it
    // (row it / kChunks of the row's 16-byte aligned span) lands at 16 it
    {
        const int total = nsr * kChunks, lane = tid & 63;
        for (int b = tid - lane; b < total; b += kThreads) {  // b is uniform in the wave
            const int it = b + lane;
            const uint8_t *g = nullptr;
            if (it < total) {
                const int row = it / kChunks, ch = it - row * kChunks;
                const uint8_t *r = base + ((size_t)(sr0 + row) * W + sc0) * C;
                if (ch < span_chunks(r, nsc * C)) g = (const uint8_t *)((uintptr_t)r & ~(uintptr_t)15) + 16 * ch;
            }
            if (g) __builtin_amdgcn_global_load_lds((const void *)g, (lds_ptr_t)(src + 16 * b), 16, 0, 0);
        }
        __builtin_amdgcn_s_waitcnt(0);  // LDS-DMA writes are counted by vmcnt
    }
    if (FROM_AB) {
        double t = (double)ab[2 * img] * (double)tid + (double)ab[2 * img + 1];
        lut[0][tid] = (uint8_t)sat8((int)rint(t));
    } else {  // every channel's entry loaded before any is stored
        static_assert(kThreads == 256, "one LUT entry per thread and channel");
        uint8_t lv[C];
#pragma unroll
        for (int c = 0; c < C; ++c) lv[c] = luts[((size_t)img * C + c) * 256 + tid];
#pragma unroll
        for (int c = 0; c < C; ++c) lut[c][tid] = lv[c];
    }
    const bool to_gray = !FROM_AB && C == 3 && gray && gray[img];
    __syncthreads();

    // four output pixels per item: the Dih4 map, the staged row's phase and the
    // pixel (one LDS word) once per pixel, the LUTs per channel, and C words
    // stored when the four pixels start on a word
    uint8_t *obase = out + (size_t)img * plane;
    constexpr int kQ = kT / 4;
    const uint32_t bphase = (uint32_t)(uintptr_t)base;
    for (int it = tid; it < th * kQ; it += kThreads) {
        const int r = it / kQ, q4 = (it - r * kQ) * 4;
        if (q4 >= tw) continue;
        const int orow = r0 + r, np = min(4, tw - q4);
        uint32_t v[4] = {0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (j >= np) break;
            const int c = c0 + q4 + j;
            const int sy = m.sy(orow, c), sx = m.sx(orow, c);
            const int o = (sy - sr0) * kStride + (int)((bphase + (uint32_t)(sy * W + sc0) * C) & 15) + (sx - sc0) * C;
            const uint32_t *w = (const uint32_t *)(src + (o & ~3));
            const uint32_t pw = __builtin_amdgcn_alignbyte(w[1], w[0], o & 3);
            uint32_t q = 0;
            if (FROM_AB) {
#pragma unroll
                for (int ch = 0; ch < C; ++ch) q |= (uint32_t)lut[0][(pw >> (8 * ch)) & 255] << (8 * ch);
            } else if (!to_gray) {
#pragma unroll
                for (int ch = 0; ch < C; ++ch) q |= (uint32_t)lut[ch][(pw >> (8 * ch)) & 255] << (8 * ch);
            } else {
                // BT.601 luma in Q14 (4899, 9617, 1868), rounded half up, on the LUT'd channels
                const int rr = lut[0][pw & 255], gg = lut[C > 1 ? 1 : 0][(pw >> 8) & 255];
                const int bb = lut[C > 2 ? 2 : 0][(pw >> 16) & 255];
                const uint32_t y = (uint32_t)((4899 * rr + 9617 * gg + 1868 * bb + 8192) >> 14);
#pragma unroll
                for (int ch = 0; ch < C; ++ch) q |= y << (8 * ch);
            }
            v[j] = q;
        }
        uint8_t *g = obase + ((size_t)orow * Wo + c0 + q4) * C;
        if (np == 4 && ((uintptr_t)g & 3) == 0) {
            uint32_t *gw = (uint32_t *)g;
            if (C == 1) {
                gw[0] = v[0] | v[1] << 8 | v[2] << 16 | v[3] << 24;
            } else if (C == 3) {
                gw[0] = v[0] | v[1] << 24;
                gw[1] = v[1] >> 8 | v[2] << 16;
                gw[2] = v[2] >> 16 | v[3] << 8;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) gw[j] = v[j];
            }
        } else {
            for (int j = 0; j < np; ++j)
#pragma unroll
                for (int ch = 0; ch < C; ++ch) g[j * C + ch] = (uint8_t)(v[j] >> (8 * ch));
        }
    }
}

}  // namespace

hipError_t launch_d4_bc_u8(const uint8_t *in, int n, int H, int W, int C, const int32_t *flags, const float *ab,
                           uint8_t *out, hipStream_t s) {
    if (n == 0 || H == 0 || W == 0) return hipSuccess;
    int t = (max(H, W) + kT - 1) / kT;
    dim3 grid(t * t, n);
    const uint8_t *nl = nullptr;
    const int32_t *ng = nullptr;
    if (C == 1) hipLaunchKernelGGL((k_d4_bc<1, true>), grid, dim3(kThreads), 0, s, in, H, W, flags, ab, nl, ng, out);
    else if (C == 3) hipLaunchKernelGGL((k_d4_bc<3, true>), grid, dim3(kThreads), 0, s, in, H, W, flags, ab, nl, ng, out);
    else hipLaunchKernelGGL((k_d4_bc<4, true>), grid, dim3(kThreads), 0, s, in, H, W, flags, ab, nl, ng, out);
    return hipGetLastError();
}

hipError_t launch_d4_lut_u8(const uint8_t *in, int n, int H, int W, int C, const int32_t *flags, const uint8_t *luts,
                            const int32_t *gray, uint8_t *out, hipStream_t s) {
    if (n == 0 || H == 0 || W == 0) return hipSuccess;
    int t = (max(H, W) + kT - 1) / kT;
    dim3 grid(t * t, n);
    const float *na = nullptr;
    if (C == 1) hipLaunchKernelGGL((k_d4_bc<1, false>), grid, dim3(kThreads), 0, s, in, H, W, flags, na, luts, gray, out);
    else if (C == 3) hipLaunchKernelGGL((k_d4_bc<3, false>), grid, dim3(kThreads), 0, s, in, H, W, flags, na, luts, gray, out);
    else hipLaunchKernelGGL((k_d4_bc<4, false>), grid, dim3(kThreads), 0, s, in, H, W, flags, na, luts, gray, out);
    return hipGetLastError();
}

}  // namespace miaug
