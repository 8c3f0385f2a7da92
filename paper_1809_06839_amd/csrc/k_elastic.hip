// k_elastic.hip -- elastic transform and grid distortion (Sec. II-C, Fig. 4;
// the elastic distortion of Simard et al. 2003 cited in Sec. I).
//
// Fields: per image and field, 16-bit Philox noise is smoothed by a separable
// integer Gaussian (Q15 taps, reflect-101):
//   k_field_h2 one workgroup per (row segment of 2560, field, image): noise of
//              the segment and its +-radius halo is generated into LDS as
//              int16, each thread produces 10 consecutive outputs from pairs
//              of noise values and taps (packed 16-bit multiply-adds into
//              int32, exact); k_field_h is the int32 form for taps of 2^15
//              (segments of 1280, 5 outputs per thread);
//   k_field_v2 one workgroup per (32-column strip x 256 rows, field, image): the
//              strip of the H-pass result with its +-radius halo is staged in
//              LDS as pairs of rows, each thread produces 8 consecutive rows of
//              one column the same way, then offsets off = rdiv_he(alpha v,
//              2^20) (Q10 px); a strip with a value outside int16 (possible
//              only when rounding lifts the taps' sum above 2^15) is done
//              with direct int32 sums; taps of 2^15 take the int32 form
//              (k_field_v, strips of 64 rows).
// Remap chain (u8): one workgroup per 32 x 32 output tile.  The tile's grid
// taps read a block of rows and columns (before reflection) of the elastic
// result e, the e-block; the displaced Q10 positions of the e-block read a
// block of the source, which is staged in LDS once (one pixel per word, with
// its mask); the e-block is blended from it into LDS (4 source taps -> u8,
// reflect-101), and the output from the e-block.  Tiles whose blocks do not
// fit, or reach past one reflection of the image, gather their taps from
// global memory instead.  The mask takes the same two maps with nearest
// sampling.  Float copy: the same maps without rounding; its adjoint is
// owner-computes: the grid step as a gather over the inverse grid ranges,
// the elastic step per source tile over the window its largest displacement
// allows, accumulated in LDS (no global float atomics).
#include "dev_common.h"
#include "q10_blend.h"
#include "internal.h"

namespace miaug {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxRadius = 200;  // V-pass strip (64 + 2 radius rows x 32 columns) stays below 64 KiB of LDS

// ---------------------------------------------------------------- Philox4x64-10 (device copy)
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t h0 = __umul64hi(M0, c[0]), l0 = M0 * c[0];
        const uint64_t h1 = __umul64hi(M1, c[2]), l1 = M1 * c[2];
        const uint64_t o0 = h1 ^ c[1] ^ k0, o2 = h0 ^ c[3] ^ k1;
        c[0] = o0; c[1] = l1; c[2] = o2; c[3] = l0;
        k0 += W0; k1 += W1;
    }
}

// ---------------------------------------------------------------- H pass
constexpr int kHPer = 5;                   // consecutive outputs per thread (odd: no LDS bank sharing)
constexpr int kHSeg = kHPer * kThreads;    // outputs per workgroup

// Noise of row y of one field at reflected columns x0 - radius .. x0 + SEG + radius - 1 (as far as needed)
// into noise[0 ..): the segment's own columns x0 .. x0 + m - 1 (m <= SEG) first, where one Philox block
// gives the 16 values of 16 consecutive stream positions; then the reflected halo columns, which are copies
// of columns already generated when the row is covered by this segment and are generated one by one
// otherwise.  Ends with a barrier.
template <int SEG, typename T>
__device__ __forceinline__ void row_noise(uint64_t seed, uint64_t g, int field, int y, int W, int radius, int x0,
                                          T *noise) {
    const int n_need = min(SEG, W - x0) + 2 * radius;
    const int m = min(SEG, W - x0);
    const int64_t e0 = (int64_t)y * W + x0, e1 = e0 + m;
    for (int64_t grp = (e0 >> 4) + threadIdx.x; grp <= ((e1 - 1) >> 4); grp += kThreads) {
        uint64_t c[4] = {(uint64_t)grp, g, (uint64_t)field, 4};
        philox4x64_10(c, seed, 0);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int64_t e = grp * 16 + k;
            if (e >= e0 && e < e1) noise[radius + (int)(e - e0)] = (T)((int32_t)((c[k >> 2] >> (16 * (k & 3))) & 0xFFFFu) - 32768);
        }
    }
    // halo columns of other segments that need no reflection (x in [0, W)): the
    // ranges [x0 - radius, x0) and [x0 + m, x0 + m + radius), in aligned blocks of 16
    const int la = max(0, x0 - radius), lb = x0, ra = x0 + m, rb = min(W, x0 + m + radius);
    const int64_t gl0 = ((int64_t)y * W + la) >> 4, gl1 = ((int64_t)y * W + lb - 1) >> 4;
    const int64_t gr0 = ((int64_t)y * W + ra) >> 4, gr1 = ((int64_t)y * W + rb - 1) >> 4;
    const int nl = lb > la ? (int)(gl1 - gl0 + 1) : 0, nr = rb > ra ? (int)(gr1 - gr0 + 1) : 0;
    for (int t = threadIdx.x; t < nl + nr; t += kThreads) {
        const int64_t grp = t < nl ? gl0 + t : gr0 + (t - nl);
        const int64_t lo = (int64_t)y * W + (t < nl ? la : ra), hi = (int64_t)y * W + (t < nl ? lb : rb);
        uint64_t c[4] = {(uint64_t)grp, g, (uint64_t)field, 4};
        philox4x64_10(c, seed, 0);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int64_t e = grp * 16 + k;
            if (e >= lo && e < hi)
                noise[(int)(e - e0) + radius] = (T)((int32_t)((c[k >> 2] >> (16 * (k & 3))) & 0xFFFFu) - 32768);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_need; i += kThreads) {
        if (i >= radius && i < radius + m) continue;  // own column, generated above
        const int xi = x0 - radius + i;
        if (xi >= 0 && xi < W) continue;               // another segment's column, generated above
        const int xs = reflect101(x0 - radius + i, W);
        if (xs >= x0 && xs < x0 + m) {
            noise[i] = noise[radius + (xs - x0)];
        } else {
            const int64_t e = (int64_t)y * W + xs;
            uint64_t c[4] = {(uint64_t)(e >> 4), g, (uint64_t)field, 4};
            philox4x64_10(c, seed, 0);
            const uint64_t word = c[(e & 15) >> 2];
            noise[i] = (T)((int32_t)((word >> (16 * (e & 3))) & 0xFFFFu) - 32768);
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(kThreads) void k_field_h(uint64_t seed, uint64_t first, int H, int W, int radius,
                                                      const int32_t *__restrict__ taps, int32_t *__restrict__ hout) {
    __shared__ int32_t noise[kHSeg + 2 * kMaxRadius + 16];
    __shared__ int32_t tp[2 * kMaxRadius + 16];  // taps, zero-padded to a multiple of kHPer
    const int segs = (W + kHSeg - 1) / kHSeg;
    const int y = blockIdx.x / segs, x0 = (blockIdx.x % segs) * kHSeg;
    const int field = blockIdx.y, img = blockIdx.z;
    const uint64_t g = first + (uint64_t)img;
    const int nt = 2 * radius + 1, ntp = (nt + kHPer - 1) / kHPer * kHPer;
    for (int k = threadIdx.x; k < ntp; k += kThreads) tp[k] = k < nt ? taps[k] : 0;
    row_noise<kHSeg>(seed, g, field, y, W, radius, x0, noise);
    const int xl = kHPer * threadIdx.x;  // first of this thread's outputs, relative to x0
    if (x0 + xl >= W) return;
    // Register-blocked correlation: per block of kHPer taps, 2 kHPer - 1 noise values and
    // kHPer taps feed kHPer^2 multiply-adds with compile-time register indices.  Operands fit
    // 24 bits (|noise| <= 2^15, taps <= 2^15): full-rate v_mad_i32_i24.  Reads past the noise
    // of the segment meet zero taps.
    int32_t acc[kHPer];
#pragma unroll
    for (int o = 0; o < kHPer; ++o) acc[o] = 0;
    for (int j0 = 0; j0 < ntp; j0 += kHPer) {
        int32_t xv[2 * kHPer - 1], tv[kHPer];
#pragma unroll
        for (int i = 0; i < 2 * kHPer - 1; ++i) xv[i] = noise[xl + j0 + i];
#pragma unroll
        for (int i = 0; i < kHPer; ++i) tv[i] = tp[j0 + i];
#pragma unroll
        for (int jj = 0; jj < kHPer; ++jj)
#pragma unroll
            for (int o = 0; o < kHPer; ++o) acc[o] += __mul24(tv[jj], xv[jj + o]);
    }
    int32_t *row = hout + (((size_t)img * 2 + field) * H + y) * W + x0 + xl;
#pragma unroll
    for (int o = 0; o < kHPer; ++o)
        if (x0 + xl + o < W) row[o] = rshr_he(acc[o], 15);
}

// The same pass with packed 16-bit multiply-adds (v_dot2c_i32_i16: two products and the int32
// accumulator, exact), for taps below 2^15 (every sigma above about 0.4).  Noise is kept as int16 in
// LDS; an even-aligned pair (n[2k], n[2k+1]) is dword k of that array, an odd-aligned pair
// (n[2k+1], n[2k+2]) is formed in registers from dwords k and k + 1 (alignbit), and the taps are packed
// in pairs, so output x + o takes sum_j pair(x + o + 2j) . (t[2j], t[2j+1]).  Ten outputs per thread
// (an odd stride of five dwords between lanes: no bank sharing), four tap pairs per register block.
constexpr int kH2Per = 10;
constexpr int kH2Seg = kH2Per * kThreads;
constexpr int kH2N = kH2Seg + 2 * kMaxRadius + 64;  // int16 noise entries: the segment, its halo, the reads past it

typedef short short2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ int dot2(uint32_t a, uint32_t b, int c) {
    return __builtin_amdgcn_sdot2(__builtin_bit_cast(short2v, a), __builtin_bit_cast(short2v, b), c, false);
}

__global__ __launch_bounds__(kThreads) void k_field_h2(uint64_t seed, uint64_t first, int H, int W, int radius,
                                                       const int32_t *__restrict__ taps, int32_t *__restrict__ hout) {
    __shared__ __align__(16) int16_t noise[kH2N + 2];
    __shared__ uint32_t tp2[kMaxRadius + 8];
    const int segs = (W + kH2Seg - 1) / kH2Seg;
    const int y = blockIdx.x / segs, x0 = (blockIdx.x % segs) * kH2Seg;
    const int field = blockIdx.y, img = blockIdx.z;
    const uint64_t g = first + (uint64_t)img;
    const int nt = 2 * radius + 1, npair = ((nt + 1) / 2 + 3) / 4 * 4;
    for (int j = threadIdx.x; j < npair; j += kThreads) {
        const int t0 = 2 * j < nt ? taps[2 * j] : 0, t1 = 2 * j + 1 < nt ? taps[2 * j + 1] : 0;
        tp2[j] = (uint32_t)(t0 & 0xFFFF) | ((uint32_t)t1 << 16);
    }
    row_noise<kH2Seg>(seed, g, field, y, W, radius, x0, noise);
    const uint32_t *even = (const uint32_t *)noise;
    const int xl = kH2Per * threadIdx.x;  // first of this thread's outputs, relative to x0
    if (x0 + xl >= W) return;
    // Reads past the noise of the segment meet zero taps.
    int32_t acc[kH2Per];
#pragma unroll
    for (int o = 0; o < kH2Per; ++o) acc[o] = 0;
    const int b = xl / 2;
    for (int j0 = 0; j0 < npair; j0 += 4) {
        uint32_t xe[kH2Per / 2 + 4], xo[kH2Per / 2 + 3], tv[4];
#pragma unroll
        for (int i = 0; i < kH2Per / 2 + 4; ++i) xe[i] = even[b + j0 + i];
#pragma unroll
        for (int i = 0; i < kH2Per / 2 + 3; ++i) xo[i] = __builtin_amdgcn_alignbit(xe[i + 1], xe[i], 16);
#pragma unroll
        for (int i = 0; i < 4; ++i) tv[i] = tp2[j0 + i];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
#pragma unroll
            for (int i = 0; i < kH2Per / 2; ++i) {
                acc[2 * i] = dot2(xe[i + jj], tv[jj], acc[2 * i]);
                acc[2 * i + 1] = dot2(xo[i + jj], tv[jj], acc[2 * i + 1]);
            }
    }
    int32_t *row = hout + (((size_t)img * 2 + field) * H + y) * W + x0 + xl;
#pragma unroll
    for (int o = 0; o < kH2Per; ++o)
        if (x0 + xl + o < W) row[o] = rshr_he(acc[o], 15);
}

// ---------------------------------------------------------------- V pass
constexpr int kVCols = 32, kVRows = 64, kVPer = 8;  // 32 columns x (8 threads x 8 rows)

// The int32 form: the strip of the H-pass result with its halo in LDS (smem), each thread 8 rows of one
// column, register-blocked as in the H pass; rows past the strip meet zero taps.
// Rows y0 .. y0 + kVRows - 1 of columns xs0 .. xs0 + kVCols - 1.
__device__ __forceinline__ void field_v_int32(int H, int W, int radius, int alpha, const int32_t *__restrict__ taps,
                                              const int32_t *__restrict__ hin, int32_t *__restrict__ off,
                                              int32_t *smem, int xs0, int y0) {
    const int nt = 2 * radius + 1, ntp = (nt + kVPer - 1) / kVPer * kVPer;
    int32_t *tp = smem;          // taps, zero-padded to ntp
    int32_t *strip = smem + ntp;  // (kVRows + 2 radius + kVPer) x kVCols
    const int field = blockIdx.y, img = blockIdx.z;
    const int32_t *hb = hin + ((size_t)img * 2 + field) * H * W;
    for (int k = threadIdx.x; k < ntp; k += kThreads) tp[k] = k < nt ? taps[k] : 0;
    const int rows = min(kVRows, H - y0) + 2 * radius;
    for (int e = threadIdx.x; e < rows * kVCols; e += kThreads) {
        const int r = e / kVCols, c = e - r * kVCols;
        const int yy = reflect101(y0 - radius + r, H), xx = min(xs0 + c, W - 1);
        strip[e] = hb[(size_t)yy * W + xx];
    }
    __syncthreads();
    const int col = threadIdx.x % kVCols, grp = threadIdx.x / kVCols;
    const int x = xs0 + col, yl = grp * kVPer;
    if (x >= W || y0 + yl >= H) return;
    int32_t acc[kVPer];
#pragma unroll
    for (int o = 0; o < kVPer; ++o) acc[o] = 0;
    for (int j0 = 0; j0 < ntp; j0 += kVPer) {
        int32_t xv[2 * kVPer - 1], tv[kVPer];
#pragma unroll
        for (int i = 0; i < 2 * kVPer - 1; ++i) xv[i] = strip[(yl + j0 + i) * kVCols + col];
#pragma unroll
        for (int i = 0; i < kVPer; ++i) tv[i] = tp[j0 + i];
        // |h| <= 2^15 (1 + 150 / 2^15) and taps <= 2^15 fit 24 bits
#pragma unroll
        for (int jj = 0; jj < kVPer; ++jj)
#pragma unroll
            for (int o = 0; o < kVPer; ++o) acc[o] += __mul24(tv[jj], xv[jj + o]);
    }
    int32_t *ob = off + ((size_t)img * 2 + field) * H * W;
#pragma unroll
    for (int o = 0; o < kVPer; ++o)
        if (y0 + yl + o < H) ob[(size_t)(y0 + yl + o) * W + x] = (int32_t)rshr_he64((int64_t)alpha * acc[o], 30 - kFBits);
}

__global__ __launch_bounds__(kThreads) void k_field_v(int H, int W, int radius, int alpha,
                                                      const int32_t *__restrict__ taps,
                                                      const int32_t *__restrict__ hin, int32_t *__restrict__ off) {
    extern __shared__ int32_t smem[];
    const int strips_x = (W + kVCols - 1) / kVCols;
    field_v_int32(H, W, radius, alpha, taps, hin, off, smem, (blockIdx.x % strips_x) * kVCols,
                  (blockIdx.x / strips_x) * kVRows);
}

// Packed form of the V pass, for strips whose H-pass values all fit int16 (|h| <= the sum of the taps,
// which rounding can lift a little above 2^15): pairs of consecutive rows (2k, 2k + 1) of a column are
// one dword, the odd-aligned pairs are formed in registers as in the H pass, and taps go in pairs, so
// each thread's 8-row blocks take 4 dot2 per tap pair.  Strips of 256 rows, so the 2 radius halo rows
// are staged once per 256 output rows.  A strip with a value outside int16 is done with int32 sums read
// straight from global memory (a uniform branch: the result is the same either way).
constexpr int kV2Blocks = 4;                  // 64-row blocks per strip
constexpr int kV2Rows = kV2Blocks * kVRows;  // rows per strip (each thread kV2Blocks blocks of kVPer rows)
constexpr int kV2Pad = 8;            // pairs read past the strip (zero taps)
__host__ __device__ constexpr int v2_pairs(int radius) { return (kV2Rows + 2 * radius) / 2 + 1 + kV2Pad; }

__global__ __launch_bounds__(kThreads) void k_field_v2(int H, int W, int radius, int alpha,
                                                       const int32_t *__restrict__ taps,
                                                       const int32_t *__restrict__ hin, int32_t *__restrict__ off) {
    extern __shared__ int32_t smem[];
    __shared__ int wide;  // a staged value outside int16
    const int nt = 2 * radius + 1, npair = ((nt + 1) / 2 + 3) / 4 * 4;
    const int np = v2_pairs(radius);
    uint32_t *tp2 = (uint32_t *)smem;
    uint32_t *ev = tp2 + npair;
    const int strips_x = (W + kVCols - 1) / kVCols;
    const int xs0 = (blockIdx.x % strips_x) * kVCols, y0 = (blockIdx.x / strips_x) * kV2Rows;
    const int field = blockIdx.y, img = blockIdx.z;
    const int32_t *hb = hin + ((size_t)img * 2 + field) * H * W;
    if (threadIdx.x == 0) wide = 0;
    for (int j = threadIdx.x; j < npair; j += kThreads) {
        const int t0 = 2 * j < nt ? taps[2 * j] : 0, t1 = 2 * j + 1 < nt ? taps[2 * j + 1] : 0;
        tp2[j] = (uint32_t)(t0 & 0xFFFF) | ((uint32_t)t1 << 16);
    }
    __syncthreads();
    // staged row r is image row reflect(y0 - radius + r); pairs past the needed rows repeat a valid row
    const int rows = min(kV2Rows, H - y0) + 2 * radius;
    bool out16 = false;
    for (int e = threadIdx.x; e < np * kVCols; e += kThreads) {
        const int k = e / kVCols, c = e - k * kVCols;
        const int xx = min(xs0 + c, W - 1);
        int32_t h[2];
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const int r = min(2 * k + d, rows - 1);
            h[d] = hb[(size_t)reflect101(y0 - radius + r, H) * W + xx];
            out16 |= h[d] < -32768 || h[d] > 32767;
        }
        ev[e] = (uint32_t)(h[0] & 0xFFFF) | ((uint32_t)h[1] << 16);
    }
    if (out16) wide = 1;
    __syncthreads();
    if (wide) {  // uniform: int32 sums straight from global memory (no staging, never on a hot path)
        int32_t *ob = off + ((size_t)img * 2 + field) * H * W;
        for (int e = threadIdx.x; e < kV2Rows * kVCols; e += kThreads) {
            const int r = e / kVCols, x = xs0 + e % kVCols, y = y0 + r;
            if (y >= H || x >= W) continue;
            int32_t acc = 0;
            for (int k = 0; k < nt; ++k) acc += taps[k] * hb[(size_t)reflect101(y - radius + k, H) * W + x];
            ob[(size_t)y * W + x] = (int32_t)rshr_he64((int64_t)alpha * acc, 30 - kFBits);
        }
        return;
    }
    const int col = threadIdx.x % kVCols, grp = threadIdx.x / kVCols;
    const int x = xs0 + col;
    if (x >= W) return;
    int32_t *ob = off + ((size_t)img * 2 + field) * H * W;
    for (int blk = 0; blk < kV2Blocks; ++blk) {
        const int yl = blk * kVRows + grp * kVPer;  // yl even: output row yl + o takes pair (yl + o + 2j)
        if (y0 + yl >= H) break;
        int32_t acc[kVPer];
#pragma unroll
        for (int o = 0; o < kVPer; ++o) acc[o] = 0;
        const int b = yl / 2;
        for (int j0 = 0; j0 < npair; j0 += 4) {
            uint32_t xe[kVPer / 2 + 4], xo[kVPer / 2 + 3], tv[4];
#pragma unroll
            for (int i = 0; i < kVPer / 2 + 4; ++i) xe[i] = ev[(b + j0 + i) * kVCols + col];
#pragma unroll
            for (int i = 0; i < kVPer / 2 + 3; ++i) xo[i] = __builtin_amdgcn_alignbit(xe[i + 1], xe[i], 16);
#pragma unroll
            for (int i = 0; i < 4; ++i) tv[i] = tp2[j0 + i];
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
#pragma unroll
                for (int i = 0; i < kVPer / 2; ++i) {
                    acc[2 * i] = dot2(xe[i + jj], tv[jj], acc[2 * i]);
                    acc[2 * i + 1] = dot2(xo[i + jj], tv[jj], acc[2 * i + 1]);
                }
        }
#pragma unroll
        for (int o = 0; o < kVPer; ++o)
            if (y0 + yl + o < H)
                ob[(size_t)(y0 + yl + o) * W + x] = (int32_t)rshr_he64((int64_t)alpha * acc[o], 30 - kFBits);
    }
}

// ---------------------------------------------------------------- box-cascade field (approximate, opt-in)
// Each axis's Gaussian is replaced by three box filters (Wells 1986; widths
// of Kovesi 2010), every pass rounding its mean: pass(x) = rdiv_he(sum over
// |k| <= r of in[refl(x + k)], 2r + 1).  Rows: noise and the three passes in
// LDS, one workgroup per row.  Columns: one pass per launch, each thread
// sliding a window down a segment of rows of one column (of two adjacent
// columns when W is even); the last pass writes the offsets rshr_he(alpha v, 5)
// (Q10 px).
constexpr int kBoxSeg = 64;       // rows per thread in the single-column passes

// rdiv_he(s, w) for odd w and |s| <= 32768 w (w values of the noise range):
// A = s + 32768 w >= 0, A / w <= 65536, so the float quotient (rw = v_rcp_f32(w))
// is within 1/64 of A / w and one correction step makes it exact; w is odd,
// so 2r == w never happens.
__device__ __forceinline__ int box_round(int s, int w, float rw) {
    const int A = s + 32768 * w;
    int q = (int)((float)A * rw);
    int r = A - q * w;
    if (r < 0) { q -= 1; r += w; }
    else if (r >= w) { q += 1; r -= w; }
    return q - 32768 + (2 * r > w);
}

// LDS (dynamic): two lines of W + 2 (r2 + 1) int16 (the noise and every rounded
// box mean lie in the int16 range); the halo offset is hb = r2 + 1.
__global__ __launch_bounds__(kThreads) void k_box_rows(uint64_t seed, uint64_t first, int H, int W, int r0, int r1,
                                                       int r2, int16_t *__restrict__ out) {
    extern __shared__ int16_t lines[];
    const int hb = r2 + 1;  // halo of the widest pass
    int16_t *bufa = lines, *bufb = lines + ((W + 2 * hb + 1) & ~1);  // both lines start on a word
    const int y = blockIdx.x, field = blockIdx.y, img = blockIdx.z;
    const uint64_t g = first + (uint64_t)img;
    const int64_t e0 = (int64_t)y * W, e1 = e0 + W;
    // noise: one Philox block gives the 16 values of 16 consecutive stream positions
    for (int64_t grp = (e0 >> 4) + threadIdx.x; grp <= ((e1 - 1) >> 4); grp += kThreads) {
        uint64_t c[4] = {(uint64_t)grp, g, (uint64_t)field, 4};
        philox4x64_10(c, seed, 0);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int64_t e = grp * 16 + k;
            if (e >= e0 && e < e1)
                bufa[hb + (int)(e - e0)] = (int16_t)((int32_t)((c[k >> 2] >> (16 * (k & 3))) & 0xFFFFu) - 32768);
        }
    }
    int16_t *src = bufa, *dst = bufb;
    // each thread slides over `chunk` consecutive outputs; an odd chunk puts the 64
    // lanes of a wave in 64 different LDS banks (an even one would share few banks)
    const int chunk = ((W + kThreads - 1) / kThreads) | 1, x0 = threadIdx.x * chunk;
    for (int p = 0; p < 3; ++p) {
        const int r = p == 0 ? r0 : (p == 1 ? r1 : r2), w = 2 * r + 1;
        __syncthreads();
        for (int k = threadIdx.x; k <= r; k += kThreads) {  // reflected ends (r left, r + 1 right)
            if (k < r) src[hb - 1 - k] = src[hb + reflect101(-1 - k, W)];
            src[hb + W + k] = src[hb + reflect101(W + k, W)];
        }
        __syncthreads();
        if (x0 < W) {
            const float rw = __builtin_amdgcn_rcpf((float)w);
            // the first window: int16 pairs summed by one packed dot product with (1, 1)
            int s = 0, i = hb + x0 - r;
            const int iend = hb + x0 + r;
            if (i & 1) s += src[i++];
            const uint32_t *pw = (const uint32_t *)(src + i);
            const int np = (iend - i + 1) >> 1;
            for (int k = 0; k < np; ++k) s = dot2(pw[k], 0x00010001u, s);
            if ((iend - i + 1) & 1) s += src[iend];
            const int xe = min(W, x0 + chunk);
            for (int x = x0; x < xe; ++x) {
                dst[hb + x] = (int16_t)box_round(s, w, rw);
                s += src[hb + x + r + 1] - src[hb + x - r];
            }
        }
        int16_t *t = src; src = dst; dst = t;
    }
    __syncthreads();
    int16_t *o = out + (((size_t)img * 2 + field) * H + y) * W;
    for (int x = threadIdx.x; x < W; x += kThreads) o[x] = src[hb + x];
}

// One column pass: in -> out16 (alpha < 0) or in -> offsets rshr_he(alpha v, 5).
__global__ __launch_bounds__(kThreads) void k_box_cols(const int16_t *__restrict__ in, int H, int W, int r, int alpha,
                                                       int16_t *__restrict__ out16, int32_t *__restrict__ off) {
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y0 = (blockIdx.y * 4 + (threadIdx.x >> 6)) * kBoxSeg;
    const size_t plane = ((size_t)blockIdx.z) * H * W;  // (image, field) plane
    if (x >= W || y0 >= H) return;
    const int16_t *col = in + plane + x;
    const int w = 2 * r + 1;
    const float rw = __builtin_amdgcn_rcpf((float)w);
    const int ye = min(H, y0 + kBoxSeg);
    int s = 0;
    auto emit = [&](int y, int v) {
        if (alpha < 0) out16[plane + (size_t)y * W + x] = (int16_t)v;
        else off[plane + (size_t)y * W + x] = (int32_t)rshr_he64((int64_t)alpha * v, 5);
    };
    if (y0 - r >= 0 && ye + r < H && ye - y0 == kBoxSeg) {  // every read inside the column: no reflection
        const int16_t *c = col + (size_t)(y0 - r) * W;
        for (int k = 0; k < w; ++k) s += c[(size_t)k * W];
        const int16_t *add = col + (size_t)(y0 + r + 1) * W, *sub = col + (size_t)(y0 - r) * W;
        for (int y = y0; y < ye; y += 8) {  // the 16 loads of 8 rows are issued together
            int av[8], sv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                av[k] = add[(size_t)k * W];
                sv[k] = sub[(size_t)k * W];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                emit(y + k, box_round(s, w, rw));
                s += av[k] - sv[k];
            }
            add += (size_t)8 * W;
            sub += (size_t)8 * W;
        }
        return;
    }
    for (int k = -r; k <= r; ++k) s += col[(size_t)reflect101(y0 + k, H) * W];
    for (int y = y0; y < ye; ++y) {
        emit(y, box_round(s, w, rw));
        s += col[(size_t)reflect101(y + r + 1, H) * W] - col[(size_t)reflect101(y - r, H) * W];
    }
}

// The same column pass for even W, two or four adjacent columns per lane (one
// 4- or 8-byte load and store per row) and kBoxSeg2 rows per thread; reflected
// rows are wave-uniform, and the loads of 8 rows are issued together (rows past
// the window or the segment repeat a valid row and are not used).
constexpr int kBoxSeg2 = 256;

__device__ __forceinline__ int box_row(int y, int H, bool near) {
    if (near) {  // y in [-(H - 1), 2H - 2]: at most one reflection
        const int a = y < 0 ? -y : y;
        return a >= H ? 2 * H - 2 - a : a;
    }
    return reflect101(y, H);
}

// NC adjacent columns per lane (NC = 2 or 4; W % NC == 0): the NC int16 values
// of a row move as one 4- or 8-byte word.
template <int NC>
struct BoxWord;
template <>
struct BoxWord<2> {
    typedef int32_t T;
    static __device__ __forceinline__ int get(T v, int j) { return j == 0 ? (v << 16) >> 16 : v >> 16; }
};
template <>
struct BoxWord<4> {
    typedef int2 T;
    static __device__ __forceinline__ int get(T v, int j) {
        const int h = j < 2 ? v.x : v.y;
        return (j & 1) ? h >> 16 : (h << 16) >> 16;
    }
};

template <int NC>
__global__ __launch_bounds__(kThreads) void k_box_cols2(const int16_t *__restrict__ in, int H, int W, int r,
                                                        int alpha, int16_t *__restrict__ out16,
                                                        int32_t *__restrict__ off) {
    typedef typename BoxWord<NC>::T T;
    const int x = NC * ((int)blockIdx.x * 64 + ((int)threadIdx.x & 63));
    const int y0 = ((int)blockIdx.y * 4 + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6)) * kBoxSeg2;
    const size_t plane = ((size_t)blockIdx.z) * H * W;  // (image, field) plane
    if (x >= W || y0 >= H) return;
    const T *col = (const T *)(in + plane + x);  // W % NC == 0: every group is aligned to its size
    const int Wp = W / NC;                       // words per row
    const int w = 2 * r + 1;
    const bool near = r <= H - 2;
    const float rw = __builtin_amdgcn_rcpf((float)w);
    const int ye = min(H, y0 + kBoxSeg2);
    int sum[NC];
#pragma unroll
    for (int j = 0; j < NC; ++j) sum[j] = 0;
    for (int k0 = -r; k0 <= r; k0 += 8) {
        T v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = col[(size_t)box_row(y0 + min(k0 + k, r), H, near) * Wp];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k0 + k <= r) {
#pragma unroll
                for (int j = 0; j < NC; ++j) sum[j] += BoxWord<NC>::get(v[k], j);
            }
    }
    for (int y = y0; y < ye; y += 8) {
        T av[8], sv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int yy = min(y + k, ye - 1);
            av[k] = col[(size_t)box_row(yy + r + 1, H, near) * Wp];
            sv[k] = col[(size_t)box_row(yy - r, H, near) * Wp];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (y + k >= ye) break;
            int b[NC];
#pragma unroll
            for (int j = 0; j < NC; ++j) b[j] = box_round(sum[j], w, rw);
            const size_t o = plane + (size_t)(y + k) * W + x;
            if (alpha < 0) {
                if (NC == 2) {
                    *(int32_t *)(out16 + o) = (b[0] & 0xFFFF) | (b[1] << 16);
                } else {
                    int2 q;
                    q.x = (b[0] & 0xFFFF) | (b[1] << 16);
                    q.y = (b[NC - 2] & 0xFFFF) | (b[NC - 1] << 16);
                    *(int2 *)(out16 + o) = q;
                }
            } else {
                if (NC == 2) {
                    int2 q;
                    q.x = (int32_t)rshr_he64((int64_t)alpha * b[0], 5);
                    q.y = (int32_t)rshr_he64((int64_t)alpha * b[1], 5);
                    *(int2 *)(off + o) = q;
                } else {
                    int4 q;
                    q.x = (int32_t)rshr_he64((int64_t)alpha * b[0], 5);
                    q.y = (int32_t)rshr_he64((int64_t)alpha * b[1], 5);
                    q.z = (int32_t)rshr_he64((int64_t)alpha * b[NC - 2], 5);
                    q.w = (int32_t)rshr_he64((int64_t)alpha * b[NC - 1], 5);
                    *(int4 *)(off + o) = q;
                }
            }
#pragma unroll
            for (int j = 0; j < NC; ++j) sum[j] += BoxWord<NC>::get(av[k], j) - BoxWord<NC>::get(sv[k], j);
        }
    }
}

// ---------------------------------------------------------------- grid tables
__global__ void k_grid_tables(const double *__restrict__ grid, int H, int W, int32_t *__restrict__ mapx,
                              int32_t *__restrict__ mapy) {
    const int img = blockIdx.y;
    const int axis = blockIdx.z;  // 0: x (W entries), 1: y (H entries)
    const int n = axis ? H : W;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *d = grid + 10 * img + 5 * axis;
    const double cw = (double)n / 5;
    const double u = i + 0.5;
    int k = (int)floor(u / cw);
    if (k > 4) k = 4;
    double S = 0.0;
    for (int j = 0; j < k; ++j) S = S + cw * d[j];
    const double src = S + (u - k * cw) * d[k] - 0.5;
    (axis ? mapy + (size_t)img * H : mapx + (size_t)img * W)[i] = (int32_t)llrint(src * kFOne);
}

// ---------------------------------------------------------------- u8 remap chain
constexpr int kRT = 32;  // output tile side
constexpr int kRE = 44;  // max side of the e-block held in LDS (grid factors up to ~1.3)
constexpr int kRS = 56;  // max side of the source block the e-block's displaced taps read
// (about 25 KB of LDS: three workgroups in each half of a CU's LDS)
constexpr int kREPer = (kRE * kRE + kThreads - 1) / kThreads;  // e-block entries per thread

// reflect-101 with the in-range case inline and the rest out of line
__device__ __noinline__ int reflect101_far(int i, int n) { return reflect101(i, n); }
__device__ __forceinline__ int refl(int i, int n) { return (unsigned)i < (unsigned)n ? i : reflect101_far(i, n); }
// reflect-101 of i in [-(n - 1), 2n - 2] (at most one reflection), branch-free
__device__ __forceinline__ int refl1(int i, int n) {
    const int a = i < 0 ? -i : i;
    return a >= n ? 2 * n - 2 - a : a;
}
__device__ __forceinline__ bool near_range(int lo, int hi, int n) { return lo >= -(n - 1) && hi <= 2 * n - 2; }

__device__ __forceinline__ uint32_t load_px(const uint8_t *p, int C) {
    if (C == 1) return p[0];
    const int sh = (int)((uintptr_t)p & 3);
    const uint32_t *w = (const uint32_t *)(p - sh);  // pointer arithmetic keeps the global address space
    const uint32_t lo = w[0];
    if (sh + C <= 4) return lo >> (8 * sh);
    return __builtin_amdgcn_alignbyte(w[1], lo, sh);
}

// Displaced Q10 position of the e pixel (Y, X) (inside the image).
__device__ __forceinline__ void displaced(const int32_t *ox, const int32_t *oy, int W, int Y, int X, int &qx,
                                          int &qy) {
    const uint32_t e = (uint32_t)Y * W + X;
    qx = (X << kFBits) + ox[e];
    qy = (Y << kFBits) + oy[e];
}

// Elastic result at the displaced position (qx, qy): four taps read from global memory.
template <int C>
__device__ __noinline__ uint32_t elastic_at(const uint8_t *img, int H, int W, int qx, int qy) {
    const int x0 = qx >> kFBits, y0 = qy >> kFBits;
    const int X0 = refl(x0, W), X1 = refl(x0 + 1, W), Y0 = refl(y0, H), Y1 = refl(y0 + 1, H);
    return blend_q10<C>(load_px(img + ((uint32_t)Y0 * W + X0) * C, C), load_px(img + ((uint32_t)Y0 * W + X1) * C, C),
                       load_px(img + ((uint32_t)Y1 * W + X0) * C, C), load_px(img + ((uint32_t)Y1 * W + X1) * C, C),
                       q10_pair(qx & (kFOne - 1)), qy & (kFOne - 1));
}

__device__ __forceinline__ uint8_t nearest_at(const uint8_t *m, int H, int W, int qx, int qy) {
    return m[(uint32_t)refl((qy + kFOne / 2) >> kFBits, H) * W + refl((qx + kFOne / 2) >> kFBits, W)];
}

// Output pixel at grid position (gx, gy) with every tap from global memory (tiles whose
// e-block does not fit in LDS).
template <int C>
__device__ __noinline__ void remap_direct(const uint8_t *src, const uint8_t *msrc, int H, int W, const int32_t *ox,
                                          const int32_t *oy, int gx, int gy, uint32_t &v, uint32_t &mv) {
    const int cx = gx >> kFBits, cy = gy >> kFBits;
    const int X0 = refl(cx, W), X1 = refl(cx + 1, W), Y0 = refl(cy, H), Y1 = refl(cy + 1, H);
    int q[8];
    displaced(ox, oy, W, Y0, X0, q[0], q[1]);
    displaced(ox, oy, W, Y0, X1, q[2], q[3]);
    displaced(ox, oy, W, Y1, X0, q[4], q[5]);
    displaced(ox, oy, W, Y1, X1, q[6], q[7]);
    v = blend_q10<C>(elastic_at<C>(src, H, W, q[0], q[1]), elastic_at<C>(src, H, W, q[2], q[3]),
                    elastic_at<C>(src, H, W, q[4], q[5]), elastic_at<C>(src, H, W, q[6], q[7]),
                    q10_pair(gx & (kFOne - 1)), gy & (kFOne - 1));
    mv = 0;
    if (msrc) {
        int mqx, mqy;
        displaced(ox, oy, W, refl((gy + kFOne / 2) >> kFBits, H), refl((gx + kFOne / 2) >> kFBits, W), mqx, mqy);
        mv = nearest_at(msrc, H, W, mqx, mqy);
    }
}

// Four packed pixels of C bytes as C little-endian words.
template <int C>
__device__ __forceinline__ void store4(uint8_t *o, const uint32_t v[4]) {
    if (C == 1) {
        *(uint32_t *)o = (v[0] & 255) | (v[1] & 255) << 8 | (v[2] & 255) << 16 | v[3] << 24;
    } else if (C == 3) {
        uint32_t *w = (uint32_t *)o;
        w[0] = (v[0] & 0xFFFFFF) | v[1] << 24;
        w[1] = (v[1] >> 8 & 0xFFFF) | v[2] << 16;
        w[2] = (v[2] >> 16 & 0xFF) | v[3] << 8;
    } else {
        uint4 q;
        q.x = v[0]; q.y = v[1]; q.z = v[2]; q.w = v[3];
        *(uint4 *)o = q;
    }
}

template <int C>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_remap_chain_u8(
    const uint8_t *__restrict__ img, const uint8_t *__restrict__ mask, int H, int W, const int32_t *__restrict__ off,
    const int32_t *__restrict__ mapx, const int32_t *__restrict__ mapy, uint8_t *__restrict__ out,
    uint8_t *__restrict__ out_mask, int img_index, int vec) {
    __shared__ uint32_t ss[kRS * kRS];  // source block, one pixel per word
    __shared__ uint8_t sm[kRS * kRS];   // its mask
    __shared__ uint32_t eb[kRE * kRE];  // e-block
    __shared__ uint8_t em[kRE * kRE];
    __shared__ int32_t qx[kRT], qy[kRT];
    __shared__ int red[kThreads / 64][4];
    __shared__ int rng[2][2];
    const int tid = (int)threadIdx.x;
    const int im = img_index >= 0 ? img_index : (int)blockIdx.y;
    const int tiles_x = (W + kRT - 1) / kRT;
    // Workgroups go round-robin to the 8 XCDs, each with its own L2; neighbouring
    // tiles share cache lines of every plane, so XCD b % 8 takes the b % 8-th
    // contiguous eighth of the tiles (when the count divides by 8).
    const int nt = (int)gridDim.x;
    const int t = (nt & 7) == 0 ? ((int)blockIdx.x & 7) * (nt >> 3) + ((int)blockIdx.x >> 3) : (int)blockIdx.x;
    const int x0 = (t % tiles_x) * kRT, y0 = (t / tiles_x) * kRT;
    const int tw = min(kRT, W - x0), th = min(kRT, H - y0);
    const size_t plane = (size_t)H * W;
    const uint8_t *src = img + (size_t)im * plane * C;
    const uint8_t *msrc = mask ? mask + (size_t)im * plane : nullptr;
    const int32_t *ox = off + (size_t)im * 2 * plane, *oy = ox + plane;
    const int32_t *mx = mapx + (size_t)im * W, *my = mapy + (size_t)im * H;
    // e rows/columns the tile's grid taps read (pre-reflection ranges; the
    // extremes are taken over every entry, so any table is handled): wave 0
    // reduces the tile's columns, wave 1 its rows
    if (tid < 128) {
        const int lane = tid & 63, cnt = tid < 64 ? tw : th;
        int lo = INT_MAX, hi = INT_MIN;
        if (lane < cnt) {
            const int q = tid < 64 ? mx[x0 + lane] : my[y0 + lane];
            (tid < 64 ? qx : qy)[lane] = q;
            lo = hi = q >> kFBits;
        }
        for (int o = 16; o > 0; o >>= 1) {
            lo = min(lo, __shfl_xor(lo, o));
            hi = max(hi, __shfl_xor(hi, o));
        }
        if (lane == 0) {
            rng[tid >> 6][0] = lo;
            rng[tid >> 6][1] = hi;
        }
    }
    __syncthreads();
    const int c_lo = rng[0][0], c_hi = rng[0][1] + 1, r_lo = rng[1][0], r_hi = rng[1][1] + 1;
    const int ew = c_hi - c_lo + 1, eh = r_hi - r_lo + 1;
    // the e-block is held in LDS when it fits and lies within one reflection of the image
    const bool staged = ew <= kRE && eh <= kRE && near_range(c_lo, c_hi, W) && near_range(r_lo, r_hi, H);
    if (staged) {
        // Pass 1, rows of the e-block over the waves (row wave + 4k) and columns
        // over the lanes (lanes past ew repeat the last column; rows past eh the
        // last row): displaced Q10 position of every entry, every load of the
        // phase in flight at once, and the source rows/columns their taps read.
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
        const int ex = refl1(c_lo + min(lane, ew - 1), W);
        int sx[kRE / 4], sy[kRE / 4];
#pragma unroll
        for (int k = 0; k < kRE / 4; ++k) {
            if (4 * k < eh) {
                const int ey = refl1(r_lo + min(wave + 4 * k, eh - 1), H);
                sx[k] = ox[(uint32_t)ey * W + ex];
                sy[k] = oy[(uint32_t)ey * W + ex];
            }
        }
        int lx = INT_MAX, hx = INT_MIN, ly = INT_MAX, hy = INT_MIN;
#pragma unroll
        for (int k = 0; k < kRE / 4; ++k) {
            if (4 * k < eh) {
                const int ey = refl1(r_lo + min(wave + 4 * k, eh - 1), H);
                sx[k] += ex << kFBits;
                sy[k] += ey << kFBits;
                lx = min(lx, sx[k] >> kFBits);
                hx = max(hx, sx[k] >> kFBits);
                ly = min(ly, sy[k] >> kFBits);
                hy = max(hy, sy[k] >> kFBits);
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            lx = min(lx, __shfl_xor(lx, o));
            hx = max(hx, __shfl_xor(hx, o));
            ly = min(ly, __shfl_xor(ly, o));
            hy = max(hy, __shfl_xor(hy, o));
        }
        if (lane == 0) {
            int *rw = red[wave];
            rw[0] = lx; rw[1] = hx; rw[2] = ly; rw[3] = hy;
        }
        __syncthreads();
        lx = min(min(red[0][0], red[1][0]), min(red[2][0], red[3][0]));
        hx = max(max(red[0][1], red[1][1]), max(red[2][1], red[3][1])) + 1;
        ly = min(min(red[0][2], red[1][2]), min(red[2][2], red[3][2]));
        hy = max(max(red[0][3], red[1][3]), max(red[2][3], red[3][3])) + 1;
        const int sw = hx - lx + 1, sh = hy - ly + 1;
        const int ne = ew * eh;
        if (sw <= kRS && sh <= kRS && near_range(lx, hx, W) && near_range(ly, hy, H)) {
            // each entry's taps as one word in eb: source-block index of the top-left
            // tap (12 bits), ax (10 bits), ay (10 bits); the blend pass replaces it
#pragma unroll
            for (int k = 0; k < kRE / 4; ++k) {
                if (4 * k < eh && lane < ew && wave + 4 * k < eh)
                    eb[(wave + 4 * k) * ew + lane] = (uint32_t)(((sy[k] >> kFBits) - ly) * sw + (sx[k] >> kFBits) - lx) |
                                                     (uint32_t)(sx[k] & (kFOne - 1)) << 12 |
                                                     (uint32_t)(sy[k] & (kFOne - 1)) << 22;
            }
            // the source block (pre-reflection rows ly..hy, columns lx..hx), read
            // once with the same row/lane split: all loads, then the LDS writes
            const int mis = (int)((uintptr_t)src & 3);
            const uint32_t *wsrc = (const uint32_t *)(src - mis);
            const uint32_t last_dw = (uint32_t)((plane * C - 1 + mis) >> 2);
            const int sxc = refl1(lx + min(lane, sw - 1), W);
            // the mask byte is loaded unconditionally (from the image when there is
            // no mask), so no branch splits the batch of loads
            const uint8_t *mload = msrc ? msrc : src;
            uint32_t plo[kRS / 4], phi[kRS / 4], mk[kRS / 4];
#pragma unroll
            for (int k = 0; k < kRS / 4; ++k) {  // no branch: rows past sh repeat the last row
                const int syr = refl1(ly + min(wave + 4 * k, sh - 1), H);
                const uint32_t p = (uint32_t)syr * W + sxc, d = (p * C + mis) >> 2;
                plo[k] = wsrc[d];
                if (C == 3) phi[k] = wsrc[min(d + 1, last_dw)];
                mk[k] = mload[p];
            }
            // the pixels are cut out of their words only here, after every load was issued
#pragma unroll
            for (int k = 0; k < kRS / 4; ++k) {
                if (4 * k < sh && lane < sw && wave + 4 * k < sh) {
                    const int syr = refl1(ly + wave + 4 * k, H);
                    const uint32_t sb = ((uint32_t)syr * W + sxc) * C + mis;
                    const int e = (wave + 4 * k) * sw + lane;
                    ss[e] = C == 4 ? plo[k]
                                   : (C == 3 ? __builtin_amdgcn_alignbyte(phi[k], plo[k], sb & 3) : plo[k] >> (8 * (sb & 3)));
                    if (msrc) sm[e] = (uint8_t)mk[k];
                }
            }
            __syncthreads();
            // Pass 2: the e-block from LDS, entries e = tid + k kThreads
#pragma unroll
            for (int k = 0; k < kREPer; ++k) {
                const int e = tid + k * kThreads;
                if (e < ne) {
                    const uint32_t w = eb[e];
                    const int ax = (int)(w >> 12) & (kFOne - 1), ay = (int)(w >> 22);
                    const uint32_t *p = ss + (w & 4095);
                    eb[e] = blend_q10<C>(p[0], p[1], p[sw], p[sw + 1], q10_pair(ax), ay);
                    if (msrc) em[e] = sm[(w & 4095) + (ax >> (kFBits - 1)) + (ay >> (kFBits - 1)) * sw];
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < kRE / 4; ++k) {
                if (4 * k < eh && lane < ew && wave + 4 * k < eh) {
                    const int e = (wave + 4 * k) * ew + lane;
                    eb[e] = elastic_at<C>(src, H, W, sx[k], sy[k]);
                    if (msrc) em[e] = nearest_at(msrc, H, W, sx[k], sy[k]);
                }
            }
        }
        __syncthreads();
    }
    // four consecutive outputs of one row per thread
    const int rr = tid >> 3, c0 = (tid & 7) * 4;
    if (rr >= th || c0 >= tw) return;
    const int gy = qy[rr], cy = gy >> kFBits, ay = gy & (kFOne - 1);
    const int nc = min(4, tw - c0);
    uint32_t v[4] = {0, 0, 0, 0}, mv[4] = {0, 0, 0, 0};
    if (staged) {
        const uint32_t *erow = eb + (cy - r_lo) * ew - c_lo;
        const uint8_t *mrow = em + (((gy + kFOne / 2) >> kFBits) - r_lo) * ew - c_lo;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gx = qx[min(c0 + j, tw - 1)], cx = gx >> kFBits;
            const uint32_t *p = erow + cx;
            v[j] = blend_q10<C>(p[0], p[1], p[ew], p[ew + 1], q10_pair(gx & (kFOne - 1)), ay);
            if (msrc) mv[j] = mrow[(gx + kFOne / 2) >> kFBits];
        }
    } else {
        for (int j = 0; j < nc; ++j) remap_direct<C>(src, msrc, H, W, ox, oy, qx[c0 + j], gy, v[j], mv[j]);
    }
    uint8_t *dst = out + (size_t)im * plane * C;
    uint8_t *mdst = msrc ? out_mask + (size_t)im * plane : nullptr;
    const uint32_t o = (uint32_t)(y0 + rr) * W + x0 + c0;
    if (vec && nc == 4) {  // o is a multiple of 4 (W is)
        store4<C>(dst + o * C, v);
        if (msrc) *(uint32_t *)(mdst + o) = mv[0] | mv[1] << 8 | mv[2] << 16 | mv[3] << 24;
    } else {
        for (int j = 0; j < nc; ++j) {
            for (int ch = 0; ch < C; ++ch) dst[(o + j) * C + ch] = (uint8_t)(v[j] >> (8 * ch));
            if (msrc) mdst[o + j] = (uint8_t)mv[j];
        }
    }
}

// ---------------------------------------------------------------- float copy of the chain
__device__ __forceinline__ int reflect_fast(int i, int n) { return (unsigned)i < (unsigned)n ? i : reflect101(i, n); }

__device__ __forceinline__ void taps_q(int qx, int qy, int H, int W, int xs[2], int ys[2], float wx[2], float wy[2]) {
    const int x0 = qx >> kFBits, y0 = qy >> kFBits;
    const int ax = qx & (kFOne - 1), ay = qy & (kFOne - 1);
    xs[0] = reflect_fast(x0, W); xs[1] = reflect_fast(x0 + 1, W);
    ys[0] = reflect_fast(y0, H); ys[1] = reflect_fast(y0 + 1, H);
    wx[0] = (float)(kFOne - ax) * (1.0f / kFOne); wx[1] = (float)ax * (1.0f / kFOne);
    wy[0] = (float)(kFOne - ay) * (1.0f / kFOne); wy[1] = (float)ay * (1.0f / kFOne);
}

// e = elastic(x) for every pixel (workspace), then y = grid(e).
__global__ void k_chain_f_elastic(const float *__restrict__ x, int C, int H, int W, const int32_t *__restrict__ off,
                                  float *__restrict__ e) {
    const size_t plane = (size_t)H * W;
    const int im = blockIdx.y;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= plane) return;
    // pixel index to (row, column): 32-bit division while the plane fits 32 bits
    const int Y = plane <= 0xFFFFFFFFu ? (int)((uint32_t)p / (uint32_t)W) : (int)(p / W);
    const int X = (int)(p - (size_t)Y * W);
    const int32_t *ox = off + (size_t)im * 2 * plane, *oy = ox + plane;
    int xs[2], ys[2];
    float wx[2], wy[2];
    taps_q((X << kFBits) + ox[p], (Y << kFBits) + oy[p], H, W, xs, ys, wx, wy);
    for (int c = 0; c < C; ++c) {
        const float *xc = x + ((size_t)im * C + c) * plane;
        const float v = wy[0] * (wx[0] * xc[(size_t)ys[0] * W + xs[0]] + wx[1] * xc[(size_t)ys[0] * W + xs[1]]) +
                        wy[1] * (wx[0] * xc[(size_t)ys[1] * W + xs[0]] + wx[1] * xc[(size_t)ys[1] * W + xs[1]]);
        e[((size_t)im * C + c) * plane + p] = v;
    }
}

__global__ void k_chain_f_grid(const float *__restrict__ e, int C, int H, int W, const int32_t *__restrict__ mapx,
                               const int32_t *__restrict__ mapy, float *__restrict__ y) {
    const size_t plane = (size_t)H * W;
    const int im = blockIdx.y;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= plane) return;
    const int r = plane <= 0xFFFFFFFFu ? (int)((uint32_t)p / (uint32_t)W) : (int)(p / W);
    const int c0 = (int)(p - (size_t)r * W);
    int xs[2], ys[2];
    float wx[2], wy[2];
    taps_q(mapx[(size_t)im * W + c0], mapy[(size_t)im * H + r], H, W, xs, ys, wx, wy);
    for (int c = 0; c < C; ++c) {
        const float *ec = e + ((size_t)im * C + c) * plane;
        y[((size_t)im * C + c) * plane + p] =
            wy[0] * (wx[0] * ec[(size_t)ys[0] * W + xs[0]] + wx[1] * ec[(size_t)ys[0] * W + xs[1]]) +
            wy[1] * (wx[0] * ec[(size_t)ys[1] * W + xs[0]] + wx[1] * ec[(size_t)ys[1] * W + xs[1]]);
    }
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, size_t n, uint32_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_fill_u8(uint8_t *__restrict__ p, size_t n, uint8_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}


// ---- adjoint of the float copy, owner-computes (every element has one writer)
// Workspace: ge [n][C][H][W] (dL/de); dmax [n] (the largest |offset| of the
// elastic field, Q10); wide [n]; the inverse grid tables: per source column j
// (row i) the count of output columns (rows) whose nonzero taps land on it,
// then up to kInvK of them with their weights, sorted by output index and
// padded with weight 0.
constexpr int kInvK = 8;

struct ChainWs {
    float *ge;
    int32_t *dmax, *wide, *cx, *cy;  // cx [n][W], cy [n][H]: entry counts
    int32_t *xc, *yc;                // [n][W][kInvK] / [n][H][kInvK] output index of each entry
    float *xw, *yw;                  // its weight
};

__host__ __device__ inline ChainWs chain_ws(void *ws, int n, int C, int H, int W) {
    ChainWs w;
    w.ge = (float *)ws;
    w.dmax = (int32_t *)(w.ge + (size_t)n * C * H * W);
    w.wide = w.dmax + n;
    w.cx = w.wide + n;
    w.cy = w.cx + (size_t)n * W;
    w.xc = w.cy + (size_t)n * H;
    w.yc = w.xc + (size_t)n * W * kInvK;
    w.xw = (float *)(w.yc + (size_t)n * H * kInvK);
    w.yw = w.xw + (size_t)n * W * kInvK;
    return w;
}


// Inverse grid tables, step 1: output column c (row r) appends itself, with
// the weight, to the entries of each source index its nonzero taps land on.
// More than kInvK entries for one index (a map that folds many outputs onto
// one source index) marks the image wide.
__global__ void k_chain_inv(const int32_t *__restrict__ mapx, const int32_t *__restrict__ mapy, int H, int W,
                            ChainWs w) {
    const int im = blockIdx.y, t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int axis = 0; axis < 2; ++axis) {
        const int n = axis ? H : W;
        if (t >= n) continue;
        const int q = (axis ? mapy : mapx)[(size_t)im * n + t];
        const int x0 = q >> kFBits, ax = q & (kFOne - 1);
        const int js[2] = {reflect101(x0, n), reflect101(x0 + 1, n)};
        const float ws[2] = {(float)(kFOne - ax) * (1.0f / kFOne), (float)ax * (1.0f / kFOne)};
        int32_t *cnt = (axis ? w.cy : w.cx) + (size_t)im * n;
        int32_t *oc = (axis ? w.yc : w.xc) + (size_t)im * n * kInvK;
        float *ow = (axis ? w.yw : w.xw) + (size_t)im * n * kInvK;
        for (int k = 0; k < 2; ++k) {
            if (ws[k] == 0.0f) continue;
            const int slot = atomicAdd(cnt + js[k], 1);
            if (slot < kInvK) {
                oc[(size_t)js[k] * kInvK + slot] = t;
                ow[(size_t)js[k] * kInvK + slot] = ws[k];
            } else {
                w.wide[im] = 1;
            }
        }
    }
}

// Step 2: each source index sorts its entries by output index (so sums run
// in a fixed order) and pads the rest with weight 0.
__global__ void k_chain_inv_sort(int H, int W, ChainWs w) {
    const int im = blockIdx.y, t = blockIdx.x * blockDim.x + threadIdx.x;
    for (int axis = 0; axis < 2; ++axis) {
        const int n = axis ? H : W;
        if (t >= n) continue;
        const size_t e = (size_t)im * n + t;
        const int m = min((axis ? w.cy : w.cx)[e], kInvK);
        int32_t *oc = (axis ? w.yc : w.xc) + e * kInvK;
        float *ow = (axis ? w.yw : w.xw) + e * kInvK;
        int c[kInvK];
        float v[kInvK];
#pragma unroll
        for (int k = 0; k < kInvK; ++k) {
            c[k] = k < m ? oc[k] : INT_MAX;
            v[k] = k < m ? ow[k] : 0.0f;
        }
#pragma unroll
        for (int a = 1; a < kInvK; ++a)  // insertion sort as a fixed network of compare-exchanges
#pragma unroll
            for (int b = a; b > 0; --b)
                if (c[b] < c[b - 1]) {
                    const int tc = c[b];
                    c[b] = c[b - 1];
                    c[b - 1] = tc;
                    const float tv = v[b];
                    v[b] = v[b - 1];
                    v[b - 1] = tv;
                }
#pragma unroll
        for (int k = 0; k < kInvK; ++k) {
            oc[k] = k < m ? c[k] : t;  // pads: weight 0 at a valid index
            ow[k] = k < m ? v[k] : 0.0f;
        }
    }
}

// dL/de of one pixel of the grid step from the tables: sum over the entries
// (r, wy) of row i and (c, wx) of column j of wy wx gy(r, c).
__device__ __forceinline__ void ge_pixel_tab(const float *__restrict__ gy, int C, int H, int W, int im, int i, int j,
                                             const ChainWs &w) {
    const size_t plane = (size_t)H * W;
    const size_t ey = ((size_t)im * H + i) * kInvK, ex = ((size_t)im * W + j) * kInvK;
    for (int cb = 0; cb < C; cb += 4) {
        float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int a = 0; a < kInvK; ++a) {
            const float wy = w.yw[ey + a];
            if (wy == 0.0f) break;  // sorted: the pads come last
            const int r = w.yc[ey + a];
            for (int b = 0; b < kInvK; ++b) {
                const float wx = w.xw[ex + b];
                if (wx == 0.0f) break;
                const float wt = wy * wx;
                const float *g = gy + ((size_t)im * C + cb) * plane + (size_t)r * W + w.xc[ex + b];
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (cb + k < C) acc[k] += wt * g[k * plane];
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (cb + k < C) w.ge[((size_t)im * C + cb + k) * plane + (size_t)i * W + j] = acc[k];
    }
}

// Folds the largest |offset| of a workgroup's pixels into dmax (integer max;
// the atomic only when it raises the value, so the workgroups of an image do
// not serialise on the one word).
__device__ __forceinline__ void fold_dmax(int dm, int32_t *dmax, int *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dm = max(dm, __shfl_xor(dm, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = dm;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int v = max(max(red[0], red[1]), max(red[2], red[3]));
        if (v > __hip_atomic_load(dmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(dmax, v);
    }
}

// The largest |offset| of each image (both planes, Q10) into dmax, for the
// elastic adjoint's window: a streaming pass over the offsets, 16 bytes per
// lane when the image's offsets start 16-byte aligned, four loads of a thread
// in flight at a time.
constexpr int kDmaxBlocks = 256;  // workgroups per image

__global__ __launch_bounds__(256) void k_chain_dmax(const int32_t *__restrict__ off, int H, int W, ChainWs w) {
    __shared__ int red[4];
    const int im = blockIdx.y;
    const size_t cnt = 2 * (size_t)H * W, stride = (size_t)gridDim.x * 256;
    const int32_t *o = off + (size_t)im * cnt;
    const size_t first = (size_t)blockIdx.x * 256 + threadIdx.x;
    int dm = 0;
    size_t t0 = 0;  // elements from here on go one at a time
    if (((uintptr_t)o & 15) == 0) {
        const int4 *v = (const int4 *)o;
        const size_t n4 = cnt / 4;
        size_t i = first;
        for (; i + 3 * stride < n4; i += 4 * stride) {
            int4 a[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = v[i + u * stride];
#pragma unroll
            for (int u = 0; u < 4; ++u) dm = max(dm, max(max(abs(a[u].x), abs(a[u].y)), max(abs(a[u].z), abs(a[u].w))));
        }
        for (; i < n4; i += stride) {
            const int4 a = v[i];
            dm = max(dm, max(max(abs(a.x), abs(a.y)), max(abs(a.z), abs(a.w))));
        }
        t0 = n4 * 4;
    }
    for (size_t t = t0 + first; t < cnt; t += stride) dm = max(dm, abs(o[t]));
    fold_dmax(dm, w.dmax + im, red);
}

// dL/de of the grid step, separable: one workgroup per 16 rows x 256 columns
// of ge.  Pass x: for each output row r the tile's rows draw on (at most
// kSepR of them, contiguous), t(r, j) = sum_k xw(j, k) gy(r, xc(j, k)) into
// LDS; pass y: ge(i, j) = sum_k yw(i, k) t(yc(i, k), j).  One channel at a
// time.  A tile whose rows draw on a wider span (a fold at a border) does
// its pixels from the tables one by one; images marked wide are left to the
// scatter form.
constexpr int kSepI = 16, kSepR = 32;

__global__ __launch_bounds__(256) void k_chain_grid_adj_sep(const float *__restrict__ gy, int C, int H, int W,
                                                            ChainWs w) {
    __shared__ float tl[kSepR][256];
    __shared__ int s_r0, s_r1;
    const int im = blockIdx.z, I0 = blockIdx.y * kSepI, j = blockIdx.x * 256 + threadIdx.x;
    const size_t plane = (size_t)H * W;
    const int I1 = min(H, I0 + kSepI);
    if (w.wide[im]) return;
    if (threadIdx.x < 64) {  // output rows the tile draws on (entries of weight != 0)
        int lo = INT_MAX, hi = -1;
        const int i = I0 + (threadIdx.x >> 2);
        if (i < I1)
            for (int k = (threadIdx.x & 3); k < kInvK; k += 4) {
                const size_t e = ((size_t)im * H + i) * kInvK + k;
                if (w.yw[e] != 0.0f) {
                    lo = min(lo, w.yc[e]);
                    hi = max(hi, w.yc[e]);
                }
            }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo = min(lo, __shfl_xor(lo, o, 64));
            hi = max(hi, __shfl_xor(hi, o, 64));
        }
        if (threadIdx.x == 0) {
            s_r0 = lo;
            s_r1 = hi;
        }
    }
    __syncthreads();
    const int r0 = s_r0;
    const long nr = (long)s_r1 - (long)s_r0 + 1;  // <= 0: no entries
    if (nr > kSepR) {
        if (j < W)
            for (int i = I0; i < I1; ++i) ge_pixel_tab(gy, C, H, W, im, i, j, w);
        return;
    }
    int xc[kInvK];
    float xw[kInvK];
#pragma unroll
    for (int k = 0; k < kInvK; ++k) {
        const size_t e = ((size_t)im * W + min(j, W - 1)) * kInvK + k;
        xc[k] = w.xc[e];
        xw[k] = j < W ? w.xw[e] : 0.0f;
    }
    // entries are sorted with the weight-0 pads last: the wave needs only as many as its widest column
    int kx = 0;
#pragma unroll
    for (int k = 0; k < kInvK; ++k) kx += xw[k] != 0.0f;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) kx = max(kx, __shfl_xor(kx, o, 64));
    kx = __builtin_amdgcn_readfirstlane(kx);
    for (int ch = 0; ch < C; ++ch) {
        const float *g = gy + ((size_t)im * C + ch) * plane;
        // pass x, four rows' loads in flight at a time
        for (int q = 0; q < nr; q += 4) {
            float v[4][kInvK];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int k = 0; k < kInvK; ++k)
                    v[u][k] = k < kx && q + u < nr ? g[(size_t)(r0 + q + u) * W + xc[k]] : 0.0f;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                float t = 0.0f;
#pragma unroll
                for (int k = 0; k < kInvK; ++k)
                    if (xw[k] != 0.0f) t += xw[k] * v[u][k];
                if (q + u < nr) tl[q + u][threadIdx.x] = t;
            }
        }
        __syncthreads();
        // pass y
        if (j < W)
            for (int i = I0; i < I1; ++i) {
                float a = 0.0f;
                for (int k = 0; k < kInvK; ++k) {  // row i is uniform: scalar loads, stop at the first pad
                    const size_t e = ((size_t)im * H + i) * kInvK + k;
                    const float yw = w.yw[e];
                    if (yw == 0.0f) break;
                    a += yw * tl[w.yc[e] - r0][threadIdx.x];
                }
                w.ge[((size_t)im * C + ch) * plane + (size_t)i * W + j] = a;
            }
        __syncthreads();
    }
}

// Scatter form of dL/de for images marked wide: zero, then each gy element
// adds its four weighted taps with float atomics (maps that fold more than
// kInvK output indices onto one source index; grid distortions never do).
__global__ void k_chain_ge_zero_wide(int C, int H, int W, ChainWs w) {
    const int im = blockIdx.y;
    if (!w.wide[im]) return;
    const size_t total = (size_t)C * H * W;
    float *g = w.ge + (size_t)im * total;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x)
        g[e] = 0.0f;
}

__global__ void k_chain_grid_scatter_wide(const float *__restrict__ gy, int C, int H, int W,
                                          const int32_t *__restrict__ mapx, const int32_t *__restrict__ mapy,
                                          ChainWs w) {
    const int im = blockIdx.y;
    if (!w.wide[im]) return;
    const size_t plane = (size_t)H * W;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < plane; p += (size_t)gridDim.x * blockDim.x) {
        const int r = (int)(p / W), c0 = (int)(p % W);
        int xs[2], ys[2];
        float wx[2], wy[2];
        taps_q(mapx[(size_t)im * W + c0], mapy[(size_t)im * H + r], H, W, xs, ys, wx, wy);
        for (int c = 0; c < C; ++c) {
            const float g = gy[((size_t)im * C + c) * plane + p];
            float *gc = w.ge + ((size_t)im * C + c) * plane;
#pragma unroll
            for (int k = 0; k < 4; ++k) atomicAdd(&gc[(size_t)ys[k >> 1] * W + xs[k & 1]], wy[k >> 1] * wx[k & 1] * g);
        }
    }
}

// dL/dx of the elastic step.  Every output pixel P whose four taps (reflect-
// 101) reach a source tile T lies within m = ceil(dmax / 2^10) + 1 of T (or of
// T's mirror image at a border, which the window clipped to the image already
// holds).  A 32 x 32 tile is interior when it lies at least m + 2 from every
// border: then no reflected tap reaches it and each contributor reaches it
// through its own bilinear cell.  Interior tiles take the gather of
// k_chain_elastic_gather; the others k_chain_elastic_adj, which owns a 64 x 32
// tile, scans the window, sums w dL/de(P) of the taps inside it in LDS (float
// adds) and stores the tile's pixels that no interior 32 x 32 tile owns.
// Channels in groups of four.
constexpr int kAdjTX = 64, kAdjTY = 32;
constexpr int kAdjU = 4;  // window elements per thread per round
constexpr int kEG = 32;   // tile of the gather form

__device__ __forceinline__ int elastic_margin(const ChainWs &w, int im, int H, int W) {
    return (int)min(((long)w.dmax[im] + kFOne - 1) >> kFBits, (long)(H + W)) + 1;
}

__device__ __forceinline__ bool interior_tile(int X0, int Y0, int m, int H, int W) {
    return X0 >= m + 2 && X0 + kEG <= W - m - 2 && Y0 >= m + 2 && Y0 + kEG <= H - m - 2;
}

__global__ __launch_bounds__(256) void k_chain_elastic_adj(int C, int H, int W, const int32_t *__restrict__ off,
                                                           ChainWs w, float *__restrict__ gx) {
    __shared__ float acc[4][kAdjTY][kAdjTX + 1];
    const int2 lb = xcd_block();  // (source tile, image): an image's tiles share one XCD's L2
    const int im = lb.y;
    const int tiles_x = (W + kAdjTX - 1) / kAdjTX;
    const int X0 = (lb.x % tiles_x) * kAdjTX, Y0 = (lb.x / tiles_x) * kAdjTY;
    const size_t plane = (size_t)H * W;
    const int m = elastic_margin(w, im, H, W);
    const bool in0 = interior_tile(X0, Y0, m, H, W), in1 = interior_tile(X0 + kEG, Y0, m, H, W);
    if (in0 && in1) return;  // both halves belong to the gather form
    const int wx0 = max(0, X0 - m), wx1 = min(W - 1, X0 + kAdjTX - 1 + m);
    const int wy0 = max(0, Y0 - m), wy1 = min(H - 1, Y0 + kAdjTY - 1 + m);
    const int ww = wx1 - wx0 + 1, total = ww * (wy1 - wy0 + 1);
    const int dq = 256 / ww, dr = 256 % ww;
    const int32_t *ox = off + (size_t)im * 2 * plane, *oy = ox + plane;
    for (int cb = 0; cb < C; cb += 4) {
        for (int e = threadIdx.x; e < 4 * kAdjTY * (kAdjTX + 1); e += 256) (&acc[0][0][0])[e] = 0.0f;
        __syncthreads();
        // window element e = tid + 256 k -> row e / ww, column e mod ww, stepped
        // incrementally; kAdjU elements per thread per round with their loads
        // issued together
        int row = threadIdx.x / ww, col = threadIdx.x % ww;
        for (int base = 0; base < total; base += 256 * kAdjU) {
            size_t pp[kAdjU];
            int qx[kAdjU], qy[kAdjU];
#pragma unroll
            for (int u = 0; u < kAdjU; ++u) {
                const bool ok = base + (int)threadIdx.x + 256 * u < total;
                const int Y = wy0 + row, X = wx0 + col;
                pp[u] = ok ? (size_t)Y * W + X : 0;
                qx[u] = ok ? (X << kFBits) + ox[pp[u]] : INT_MIN;  // INT_MIN: no element
                qy[u] = ok ? (Y << kFBits) + oy[pp[u]] : 0;
                col += dr;
                row += dq;
                if (col >= ww) {
                    col -= ww;
                    ++row;
                }
            }
            int xs[kAdjU][2], ys[kAdjU][2];
            bool hit[kAdjU];
#pragma unroll
            for (int u = 0; u < kAdjU; ++u) {
                const int x0 = qx[u] >> kFBits, y0 = qy[u] >> kFBits;
                xs[u][0] = reflect_fast(x0, W) - X0;
                xs[u][1] = reflect_fast(x0 + 1, W) - X0;
                ys[u][0] = reflect_fast(y0, H) - Y0;
                ys[u][1] = reflect_fast(y0 + 1, H) - Y0;
                const bool inx = (unsigned)xs[u][0] < (unsigned)kAdjTX || (unsigned)xs[u][1] < (unsigned)kAdjTX;
                const bool iny = (unsigned)ys[u][0] < (unsigned)kAdjTY || (unsigned)ys[u][1] < (unsigned)kAdjTY;
                hit[u] = qx[u] != INT_MIN && inx && iny;
            }
            float g[kAdjU][4];
#pragma unroll
            for (int u = 0; u < kAdjU; ++u)
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    g[u][k] = hit[u] && cb + k < C ? w.ge[((size_t)im * C + cb + k) * plane + pp[u]] : 0.0f;
#pragma unroll
            for (int u = 0; u < kAdjU; ++u) {
                if (!hit[u]) continue;
                const int ax = qx[u] & (kFOne - 1), ay = qy[u] & (kFOne - 1);
                const float wx[2] = {(float)(kFOne - ax) * (1.0f / kFOne), (float)ax * (1.0f / kFOne)};
                const float wy[2] = {(float)(kFOne - ay) * (1.0f / kFOne), (float)ay * (1.0f / kFOne)};
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int tx = xs[u][t & 1], ty = ys[u][t >> 1];
                    if ((unsigned)tx >= (unsigned)kAdjTX || (unsigned)ty >= (unsigned)kAdjTY) continue;
                    const float wt = wy[t >> 1] * wx[t & 1];
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (cb + k < C) atomicAdd(&acc[k][ty][tx], wt * g[u][k]);
                }
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kAdjTY * kAdjTX; e += 256) {
            const int r = e / kAdjTX, c = e % kAdjTX;
            if (Y0 + r >= H || X0 + c >= W || (c < kEG ? in0 : in1)) continue;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (cb + k < C) gx[((size_t)im * C + cb + k) * plane + (size_t)(Y0 + r) * W + X0 + c] = acc[k][r][c];
        }
        __syncthreads();
    }
}

// Gather form for interior 32 x 32 tiles T: the window's output pixels whose
// bilinear cell (x0, y0) lies in T's 33 x 33 cells [X0-1, X0+31] x [Y0-1, Y0+31]
// are counted per cell (pass A), the counts scanned, and their dL/de values
// and Q10 fractions stored in LDS sorted by cell (pass B, a second count per
// cell giving each its slot); each source pixel then sums the entries of the
// four cells that have it as a tap (two contiguous runs).  No float atomics:
// one integer count per entry and pass.  A tile with more entries than the
// pool takes the float-add form in LDS.
constexpr int kEC = kEG + 1, kECN = kEC * kEC;
constexpr int kEPool = 7168;  // words: kEPoolCap entries x (4 dL/de + packed fractions)
constexpr int kEPoolCap = kEPool / 5;
constexpr int kEScanPT = (kECN + 1 + 255) / 256;

__device__ __forceinline__ int block_incl_scan_w(int v, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__global__ __launch_bounds__(256) void k_chain_elastic_gather(int C, int H, int W, const int32_t *__restrict__ off,
                                                              ChainWs w, float *__restrict__ gx) {
    __shared__ int cnt[kECN + 1], cnt2[kECN];
    __shared__ float pool[kEPool];
    __shared__ int wsum[4];
    const int2 lb = xcd_block();
    const int im = lb.y;
    const int tiles_x = (W + kEG - 1) / kEG;
    const int X0 = (lb.x % tiles_x) * kEG, Y0 = (lb.x / tiles_x) * kEG;
    const int m = elastic_margin(w, im, H, W);
    if (!interior_tile(X0, Y0, m, H, W)) return;
    const size_t plane = (size_t)H * W;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wx0 = X0 - m, wx1 = X0 + kEG - 1 + m, wy0 = Y0 - m, wy1 = Y0 + kEG - 1 + m;  // inside the image
    const int ww = wx1 - wx0 + 1, total = ww * (wy1 - wy0 + 1);
    const int dq = 256 / ww, dr = 256 % ww;
    const int32_t *ox = off + (size_t)im * 2 * plane, *oy = ox + plane;
    // cell index (-1: outside T's cells) and packed fractions of window element e
    auto cell = [&](int Y, int X, int &frac) {
        const size_t p = (size_t)Y * W + X;
        const int qx = (X << kFBits) + ox[p], qy = (Y << kFBits) + oy[p];
        const int cx = (qx >> kFBits) - (X0 - 1), cy = (qy >> kFBits) - (Y0 - 1);
        frac = (qx & (kFOne - 1)) | (qy & (kFOne - 1)) << 16;
        return ((unsigned)cx < (unsigned)kEC && (unsigned)cy < (unsigned)kEC) ? cy * kEC + cx : -1;
    };
    for (int cb = 0; cb < C; cb += 4) {
        for (int i = threadIdx.x; i < kECN; i += 256) {
            cnt[i] = 0;
            cnt2[i] = 0;
        }
        __syncthreads();
        // pass A: counts
        {
            int row = threadIdx.x / ww, col = threadIdx.x % ww;
            for (int base = 0; base < total; base += 256 * kAdjU) {
                int ci[kAdjU];
#pragma unroll
                for (int u = 0; u < kAdjU; ++u) {
                    int fr;
                    ci[u] = base + (int)threadIdx.x + 256 * u < total ? cell(wy0 + row, wx0 + col, fr) : -1;
                    col += dr;
                    row += dq;
                    if (col >= ww) {
                        col -= ww;
                        ++row;
                    }
                }
#pragma unroll
                for (int u = 0; u < kAdjU; ++u)
                    if (ci[u] >= 0) atomicAdd(&cnt[ci[u]], 1);
            }
        }
        __syncthreads();
        // exclusive scan of the counts (cnt[kECN] becomes the entry count)
        {
            int v[kEScanPT], sum = 0;
#pragma unroll
            for (int j = 0; j < kEScanPT; ++j) {
                const int i = threadIdx.x * kEScanPT + j;
                v[j] = i < kECN ? cnt[i] : 0;
                sum += v[j];
            }
            const int inc = block_incl_scan_w(sum, lane);
            if (lane == 63) wsum[wave] = inc;
            __syncthreads();
            int base = inc - sum;
            for (int k = 0; k < wave; ++k) base += wsum[k];
#pragma unroll
            for (int j = 0; j < kEScanPT; ++j) {
                const int i = threadIdx.x * kEScanPT + j;
                if (i <= kECN) cnt[i] = base;
                base += v[j];
            }
        }
        __syncthreads();
        const int entries = cnt[kECN];
        float(*acc)[kEG][kEG + 1] = reinterpret_cast<float(*)[kEG][kEG + 1]>(pool);
        const bool gather = entries <= kEPoolCap;
        if (!gather) {
            for (int e = threadIdx.x; e < 4 * kEG * (kEG + 1); e += 256) pool[e] = 0.0f;
            __syncthreads();
        }
        // pass B: entries in cell order (or, past the pool, float adds into the tile)
        {
            int row = threadIdx.x / ww, col = threadIdx.x % ww;
            for (int base = 0; base < total; base += 256 * kAdjU) {
                int ci[kAdjU], fr[kAdjU];
                size_t pp[kAdjU];
#pragma unroll
                for (int u = 0; u < kAdjU; ++u) {
                    const int Y = wy0 + row, X = wx0 + col;
                    pp[u] = (size_t)Y * W + X;
                    ci[u] = base + (int)threadIdx.x + 256 * u < total ? cell(Y, X, fr[u]) : -1;
                    col += dr;
                    row += dq;
                    if (col >= ww) {
                        col -= ww;
                        ++row;
                    }
                }
                float g[kAdjU][4];
#pragma unroll
                for (int u = 0; u < kAdjU; ++u)
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        g[u][k] = ci[u] >= 0 && cb + k < C ? w.ge[((size_t)im * C + cb + k) * plane + pp[u]] : 0.0f;
#pragma unroll
                for (int u = 0; u < kAdjU; ++u) {
                    if (ci[u] < 0) continue;
                    if (gather) {
                        const int pos = cnt[ci[u]] + atomicAdd(&cnt2[ci[u]], 1);
#pragma unroll
                        for (int k = 0; k < 4; ++k) pool[k * kEPoolCap + pos] = g[u][k];
                        pool[4 * kEPoolCap + pos] = __int_as_float(fr[u]);
                    } else {
                        const int cx = ci[u] % kEC - 1, cy = ci[u] / kEC - 1;  // tap (0, 0) relative to T
                        const int ax = fr[u] & 0xffff, ay = fr[u] >> 16;
                        const float wxs[2] = {(float)(kFOne - ax) * (1.0f / kFOne), (float)ax * (1.0f / kFOne)};
                        const float wys[2] = {(float)(kFOne - ay) * (1.0f / kFOne), (float)ay * (1.0f / kFOne)};
#pragma unroll
                        for (int t = 0; t < 4; ++t) {
                            const int tx = cx + (t & 1), ty = cy + (t >> 1);
                            if ((unsigned)tx >= (unsigned)kEG || (unsigned)ty >= (unsigned)kEG) continue;
                            const float wt = wys[t >> 1] * wxs[t & 1];
#pragma unroll
                            for (int k = 0; k < 4; ++k)
                                if (cb + k < C) atomicAdd(&acc[k][ty][tx], wt * g[u][k]);
                        }
                    }
                }
            }
        }
        __syncthreads();
        // every source pixel of T: the entries of its four cells, or the summed tile
#pragma unroll
        for (int j = 0; j < kEG * kEG / 256; ++j) {
            const int e = threadIdx.x + j * 256;
            const int lu = e % kEG, lv = e / kEG;
            float sum[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (gather) {
#pragma unroll
                for (int dy = 0; dy < 2; ++dy) {
                    // cell row lv + dy has corner y0 = v - 1 + dy: the pixel is its tap row 1 - dy
                    const int ci = (lv + dy) * kEC + lu;
                    const int a0 = cnt[ci], mid = cnt[ci + 1], b0 = cnt[ci + 2];
                    for (int q = a0; q < b0; ++q) {
                        const int fr = __float_as_int(pool[4 * kEPoolCap + q]);
                        const int ax = fr & 0xffff, ay = fr >> 16;
                        const float wx = (float)(q < mid ? ax : kFOne - ax) * (1.0f / kFOne);  // left cell: x0 = u - 1
                        const float wy = (float)(dy == 0 ? ay : kFOne - ay) * (1.0f / kFOne);
                        const float wt = wy * wx;
#pragma unroll
                        for (int k = 0; k < 4; ++k) sum[k] += wt * pool[k * kEPoolCap + q];
                    }
                }
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) sum[k] = acc[k][lv][lu];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (cb + k < C) gx[((size_t)im * C + cb + k) * plane + (size_t)(Y0 + lv) * W + X0 + lu] = sum[k];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- boxes under the distortion
// A box covers the source pixels whose centres lie in [x1, x2) x [y1, y2).
// Output pixel (x, y) takes, on the mask path, the source pixel reached by the
// grid's nearest tap and then the elastic map's nearest tap; the transformed
// box is the bounding box of the output pixels whose source pixel it covers
// (empty: all zeros).  The outputs are first used as int32 accumulators.
constexpr int kBoxChunk = 16;

__global__ __launch_bounds__(64) void k_boxes_distort_init(const int32_t *__restrict__ box_off, int32_t *acc) {
    for (int b = box_off[blockIdx.x] + (int)threadIdx.x; b < box_off[blockIdx.x + 1]; b += 64) {
        acc[4 * (size_t)b] = INT32_MAX;
        acc[4 * (size_t)b + 1] = INT32_MAX;
        acc[4 * (size_t)b + 2] = -1;
        acc[4 * (size_t)b + 3] = -1;
    }
}

constexpr int kBoxPx = 16;  // output pixels per thread

__global__ __launch_bounds__(kThreads) void k_boxes_distort(const float *__restrict__ boxes,
                                                            const int32_t *__restrict__ box_off, int H, int W,
                                                            const int32_t *__restrict__ off,
                                                            const int32_t *__restrict__ mapx,
                                                            const int32_t *__restrict__ mapy, int32_t *acc) {
    __shared__ int red[kBoxChunk][4];
    const int im = blockIdx.y;
    const int b0 = box_off[im], nb = box_off[im + 1] - b0;
    if (nb <= 0) return;
    const size_t plane = (size_t)H * W;
    const int32_t *ox = off + (size_t)im * 2 * plane, *oy = ox + plane;
    // source pixel of each of this thread's output pixels (mask path)
    int sxs[kBoxPx], sys[kBoxPx], xs[kBoxPx], ys[kBoxPx];
    const int64_t e0 = ((int64_t)blockIdx.x * kThreads * kBoxPx) + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kBoxPx; ++k) {
        const int64_t e = e0 + (int64_t)k * kThreads;
        sxs[k] = -1;
        if (e >= (int64_t)plane) continue;
        const int y = (int)(e / W), x = (int)(e - (int64_t)y * W);
        const int X = reflect101((mapx[(size_t)im * W + x] + kFOne / 2) >> kFBits, W);
        const int Y = reflect101((mapy[(size_t)im * H + y] + kFOne / 2) >> kFBits, H);
        const size_t q = (size_t)Y * W + X;
        sxs[k] = reflect101(((X << kFBits) + ox[q] + kFOne / 2) >> kFBits, W);
        sys[k] = reflect101(((Y << kFBits) + oy[q] + kFOne / 2) >> kFBits, H);
        xs[k] = x;
        ys[k] = y;
    }
    for (int c0 = 0; c0 < nb; c0 += kBoxChunk) {
        const int cn = min(kBoxChunk, nb - c0);
        if (threadIdx.x < kBoxChunk * 4) red[threadIdx.x >> 2][threadIdx.x & 3] = (threadIdx.x & 2) ? -1 : INT32_MAX;
        __syncthreads();
        for (int j = 0; j < cn; ++j) {
            const float *bx = boxes + 4 * (size_t)(b0 + c0 + j);
            const float x1 = bx[0], y1 = bx[1], x2 = bx[2], y2 = bx[3];
            int mnx = INT32_MAX, mny = INT32_MAX, mxx = -1, mxy = -1;
#pragma unroll
            for (int k = 0; k < kBoxPx; ++k) {
                if (sxs[k] < 0) continue;
                const float cx = (float)sxs[k] + 0.5f, cy = (float)sys[k] + 0.5f;
                if (cx >= x1 && cx < x2 && cy >= y1 && cy < y2) {
                    mnx = min(mnx, xs[k]);
                    mny = min(mny, ys[k]);
                    mxx = max(mxx, xs[k]);
                    mxy = max(mxy, ys[k]);
                }
            }
            if (mxx >= 0) {
                atomicMin(&red[j][0], mnx);
                atomicMin(&red[j][1], mny);
                atomicMax(&red[j][2], mxx);
                atomicMax(&red[j][3], mxy);
            }
        }
        __syncthreads();
        if (threadIdx.x < cn && red[threadIdx.x][2] >= 0) {
            int32_t *a = acc + 4 * (size_t)(b0 + c0 + threadIdx.x);
            atomicMin(a, red[threadIdx.x][0]);
            atomicMin(a + 1, red[threadIdx.x][1]);
            atomicMax(a + 2, red[threadIdx.x][2]);
            atomicMax(a + 3, red[threadIdx.x][3]);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void k_boxes_distort_final(const int32_t *__restrict__ box_off, int32_t *acc) {
    for (int b = box_off[blockIdx.x] + (int)threadIdx.x; b < box_off[blockIdx.x + 1]; b += 64) {
        int32_t *a = acc + 4 * (size_t)b;
        const bool empty = a[2] < 0;
        float *o = (float *)a;
        const float v0 = empty ? 0.f : (float)a[0], v1 = empty ? 0.f : (float)a[1];
        const float v2 = empty ? 0.f : (float)(a[2] + 1), v3 = empty ? 0.f : (float)(a[3] + 1);
        o[0] = v0;
        o[1] = v1;
        o[2] = v2;
        o[3] = v3;
    }
}

}  // namespace

size_t elastic_workspace_bytes(int n, int H, int W) {
    return (size_t)n * 2 * H * W * sizeof(int32_t) + (2 * kMaxRadius + 1 + 15) * sizeof(int32_t);
}

hipError_t launch_elastic_fields(uint64_t seed, uint64_t first, int n, int H, int W, double sigma, int alpha,
                                 int radius, int32_t *off, void *ws, hipStream_t s) {
    // Q15 taps t_k = rint(2^15 g_k / sum g), g_k = exp(-k^2 / (2 sigma^2)), on the host in double
    int32_t taps[2 * kMaxRadius + 1];
    double sum = 0.0;
    for (int k = -radius; k <= radius; ++k) sum += exp(-(double)k * k / (2.0 * sigma * sigma));
    for (int k = -radius; k <= radius; ++k)
        taps[k + radius] = (int32_t)rint(32768.0 * exp(-(double)k * k / (2.0 * sigma * sigma)) / sum);
    int32_t *hbuf = (int32_t *)ws;
    int32_t *dtaps = hbuf + (size_t)n * 2 * H * W;
    hipError_t e = hipMemcpyAsync(dtaps, taps, sizeof(int32_t) * (2 * radius + 1), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    int tmax = 0;
    for (int k = 0; k < 2 * radius + 1; ++k) tmax = taps[k] > tmax ? taps[k] : tmax;
    if (tmax < 32768) {  // taps fit int16: packed multiply-adds
        const int segs = (W + kH2Seg - 1) / kH2Seg;
        hipLaunchKernelGGL(k_field_h2, dim3((unsigned)H * segs, 2, n), dim3(kThreads), 0, s, seed, first, H, W,
                           radius, dtaps, hbuf);
    } else {
        const int segs = (W + kHSeg - 1) / kHSeg;
        hipLaunchKernelGGL(k_field_h, dim3((unsigned)H * segs, 2, n), dim3(kThreads), 0, s, seed, first, H, W,
                           radius, dtaps, hbuf);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int strips = ((W + kVCols - 1) / kVCols) * ((H + kVRows - 1) / kVRows);
    const int ntp = (2 * radius + 1 + kVPer - 1) / kVPer * kVPer;
    const size_t lds = sizeof(int32_t) * (ntp + (size_t)(kVRows + 2 * radius + kVPer) * kVCols);
    if (tmax < 32768) {  // the packed form
        const int npair = ((2 * radius + 1 + 1) / 2 + 3) / 4 * 4;
        const size_t lds2 = sizeof(uint32_t) * (npair + (size_t)v2_pairs(radius) * kVCols);
        const int strips2 = ((W + kVCols - 1) / kVCols) * ((H + kV2Rows - 1) / kV2Rows);
        hipLaunchKernelGGL(k_field_v2, dim3(strips2, 2, n), dim3(kThreads), lds2, s, H, W, radius, alpha, dtaps, hbuf,
                           off);
    } else {
        hipLaunchKernelGGL(k_field_v, dim3(strips, 2, n), dim3(kThreads), lds, s, H, W, radius, alpha, dtaps, hbuf,
                           off);
    }
    return hipGetLastError();
}

hipError_t launch_grid_tables(const double *grid, int n, int H, int W, int32_t *mapx, int32_t *mapy, hipStream_t s) {
    const int m = max(H, W);
    hipLaunchKernelGGL(k_grid_tables, dim3((m + 255) / 256, n, 2), dim3(256), 0, s, grid, H, W, mapx, mapy);
    return hipGetLastError();
}

hipError_t launch_elastic_grid_u8(const uint8_t *img, const uint8_t *mask, int n, int H, int W, int C,
                                  const int32_t *off, const int32_t *mapx, const int32_t *mapy, uint8_t *out,
                                  uint8_t *out_mask, int per_image, hipStream_t s) {
    if (n == 0 || H == 0 || W == 0) return hipSuccess;
    const int tiles = ((W + kRT - 1) / kRT) * ((H + kRT - 1) / kRT);
    // packed stores of four pixels when every group of four starts on a word
    const int vec = W % 4 == 0 && (uintptr_t)out % 4 == 0 && (uintptr_t)out_mask % 4 == 0;
    auto go = [&](dim3 grid, int index) {
        if (C == 1)
            hipLaunchKernelGGL((k_remap_chain_u8<1>), grid, dim3(kThreads), 0, s, img, mask, H, W, off, mapx, mapy,
                               out, out_mask, index, vec);
        else if (C == 3)
            hipLaunchKernelGGL((k_remap_chain_u8<3>), grid, dim3(kThreads), 0, s, img, mask, H, W, off, mapx, mapy,
                               out, out_mask, index, vec);
        else
            hipLaunchKernelGGL((k_remap_chain_u8<4>), grid, dim3(kThreads), 0, s, img, mask, H, W, off, mapx, mapy,
                               out, out_mask, index, vec);
        return hipGetLastError();
    };
    if (per_image) {
        for (int i = 0; i < n; ++i) {
            hipError_t e = go(dim3(tiles, 1), i);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    return go(dim3(tiles, n), -1);
}

size_t chain_f32_workspace_bytes(int n, int C, int H, int W) {
    return (size_t)n * C * H * W * sizeof(float) +
           (2 * (size_t)n + (size_t)n * (W + H) * (1 + 2 * kInvK)) * sizeof(int32_t);
}

hipError_t launch_chain_f32_fwd(const float *x, int n, int C, int H, int W, const int32_t *off, const int32_t *mapx,
                                const int32_t *mapy, float *y, void *ws, hipStream_t s) {
    const size_t plane = (size_t)H * W;
    const dim3 grid((unsigned)((plane + 255) / 256), n);
    float *e = (float *)ws;
    hipLaunchKernelGGL(k_chain_f_elastic, grid, dim3(256), 0, s, x, C, H, W, off, e);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_chain_f_grid, grid, dim3(256), 0, s, e, C, H, W, mapx, mapy, y);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s);

hipError_t launch_chain_f32_bwd(const float *gy, int n, int C, int H, int W, const int32_t *off, const int32_t *mapx,
                                const int32_t *mapy, float *gx, void *ws, hipStream_t s) {
    const ChainWs w = chain_ws(ws, n, C, H, W);
    // dmax, wide and the entry counts are contiguous: one zero fill
    hipError_t err = launch_fill_u32((uint32_t *)w.dmax, 2 * (size_t)n + (size_t)n * (W + H), 0u, s);
    if (err != hipSuccess) return err;
    const dim3 g1((unsigned)((max(H, W) + 255) / 256), n);
    hipLaunchKernelGGL(k_chain_dmax, dim3(kDmaxBlocks, n), dim3(256), 0, s, off, H, W, w);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(k_chain_inv, g1, dim3(256), 0, s, mapx, mapy, H, W, w);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(k_chain_inv_sort, g1, dim3(256), 0, s, H, W, w);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(k_chain_grid_adj_sep, dim3((unsigned)((W + 255) / 256), (unsigned)((H + kSepI - 1) / kSepI), n),
                       dim3(256), 0, s, gy, C, H, W, w);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(k_chain_ge_zero_wide, dim3(1024, n), dim3(256), 0, s, C, H, W, w);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(k_chain_grid_scatter_wide, dim3(1024, n), dim3(256), 0, s, gy, C, H, W, mapx, mapy, w);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    const int tiles = ((W + kAdjTX - 1) / kAdjTX) * ((H + kAdjTY - 1) / kAdjTY);
    hipLaunchKernelGGL(k_chain_elastic_adj, dim3(tiles, n), dim3(256), 0, s, C, H, W, off, w, gx);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    const int gtiles = ((W + kEG - 1) / kEG) * ((H + kEG - 1) / kEG);
    hipLaunchKernelGGL(k_chain_elastic_gather, dim3(gtiles, n), dim3(256), 0, s, C, H, W, off, w, gx);
    return hipGetLastError();
}

// Fill of n 32-bit words with v (a kernel, so it can sit in a captured graph).
hipError_t launch_fill_u32(uint32_t *p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(1024), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, size_t n, uint8_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u8, dim3(1024), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Box widths of a three-pass cascade for sigma (Kovesi 2010): w_ideal =
// sqrt(4 sigma^2 + 1), wl = largest odd integer <= w_ideal, wu = wl + 2, and
// m = round((12 sigma^2 - 3 wl^2 - 12 wl - 9) / (-4 wl - 4)) passes of wl.
void box_radii(double sigma, int r[3]) {
    const double wi = sqrt(12.0 * sigma * sigma / 3.0 + 1.0);
    int wl = (int)floor(wi);
    if (wl % 2 == 0) wl -= 1;
    const int m = (int)round((12.0 * sigma * sigma - 3.0 * wl * wl - 12.0 * wl - 9.0) / (-4.0 * wl - 4.0));
    for (int i = 0; i < 3; ++i) r[i] = ((i < m) ? wl : wl + 2) / 2;
}

size_t box_workspace_bytes(int n, int H, int W) { return (size_t)n * 2 * H * W * sizeof(int16_t) * 2; }

hipError_t launch_elastic_fields_box(uint64_t seed, uint64_t first, int n, int H, int W, double sigma, int alpha,
                                     int32_t *off, void *ws, hipStream_t s) {
    int r[3];
    box_radii(sigma, r);
    int16_t *a = (int16_t *)ws, *b = a + (size_t)n * 2 * H * W;
    const size_t lds = sizeof(int16_t) * 2 * (((size_t)W + 2 * (r[2] + 1) + 1) & ~(size_t)1);
    hipLaunchKernelGGL(k_box_rows, dim3(H, 2, n), dim3(kThreads), lds, s, seed, first, H, W, r[0], r[1], r[2], a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (W % 4 == 0) {  // four columns per lane
        const dim3 grid4((W / 4 + 63) / 64, (H + 4 * kBoxSeg2 - 1) / (4 * kBoxSeg2), 2 * n);
        hipLaunchKernelGGL(k_box_cols2<4>, grid4, dim3(kThreads), 0, s, a, H, W, r[0], -1, b, (int32_t *)nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_box_cols2<4>, grid4, dim3(kThreads), 0, s, b, H, W, r[1], -1, a, (int32_t *)nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_box_cols2<4>, grid4, dim3(kThreads), 0, s, a, H, W, r[2], alpha, (int16_t *)nullptr,
                           off);
        return hipGetLastError();
    }
    if (W % 2 == 0) {  // column pairs
        const dim3 grid2((W / 2 + 63) / 64, (H + 4 * kBoxSeg2 - 1) / (4 * kBoxSeg2), 2 * n);
        hipLaunchKernelGGL(k_box_cols2<2>, grid2, dim3(kThreads), 0, s, a, H, W, r[0], -1, b, (int32_t *)nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_box_cols2<2>, grid2, dim3(kThreads), 0, s, b, H, W, r[1], -1, a, (int32_t *)nullptr);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(k_box_cols2<2>, grid2, dim3(kThreads), 0, s, a, H, W, r[2], alpha, (int16_t *)nullptr,
                           off);
        return hipGetLastError();
    }
    const dim3 grid((W + 63) / 64, (H + 4 * kBoxSeg - 1) / (4 * kBoxSeg), 2 * n);
    hipLaunchKernelGGL(k_box_cols, grid, dim3(kThreads), 0, s, a, H, W, r[0], -1, b, (int32_t *)nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_box_cols, grid, dim3(kThreads), 0, s, b, H, W, r[1], -1, a, (int32_t *)nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_box_cols, grid, dim3(kThreads), 0, s, a, H, W, r[2], alpha, (int16_t *)nullptr, off);
    return hipGetLastError();
}

hipError_t launch_boxes_distort(const float *boxes, const int32_t *box_off, int n, int H, int W, const int32_t *off,
                                const int32_t *mapx, const int32_t *mapy, float *out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    int32_t *acc = (int32_t *)out;
    hipLaunchKernelGGL(k_boxes_distort_init, dim3(n), dim3(64), 0, s, box_off, acc);
    const int64_t per = (int64_t)kThreads * kBoxPx;
    hipLaunchKernelGGL(k_boxes_distort, dim3((unsigned)(((int64_t)H * W + per - 1) / per), n), dim3(kThreads), 0, s,
                       boxes, box_off, H, W, off, mapx, mapy, acc);
    hipLaunchKernelGGL(k_boxes_distort_final, dim3(n), dim3(64), 0, s, box_off, acc);
    return hipGetLastError();
}

}  // namespace miaug
