// k_gather.hip -- ragged batch with wave-independent row gathers.  Computes
// exactly what k_ragged.hip computes (per image: Dih4 element -> optional crop
// window -> brightness/contrast LUT at every tap -> half-pixel bilinear resize
// -> per-channel normalisation into float32 CHW; masks by the nearest tap;
// boxes through the same geometry; Sec. II-A, Sec. II-B Dih4, Table I
// Brightness), with no LDS staging and no workgroup barrier in the loop.
//
// Line and span axes are those of k_ragged.hip (a line is an output row, or an
// output column when the element swaps the axes).  A work item is an image, a
// band of 16 or 32 output lines and a span segment of 64 positions, and it
// belongs to one wave: lane l takes span position s0 + l.  For every line the
// lane reads the two source rows' taps as one aligned 12-byte window each (the
// six bytes of the two neighbouring column taps) and the mask byte, straight
// from global memory; the 64 windows of a wave cover one run of the source
// row, which the L1 turns into whole 128-byte line requests.  The loads of the
// next seven lines are in flight while a line is blended.  Only the lookup
// tables live in LDS: the normalisation LUT per workgroup and one
// brightness/contrast LUT per wave (rebuilt when its image changes).
//
// Keep-axes elements pass every four blended lines through a per-wave LDS
// tile and store them 16 bytes per lane.  Swapping elements keep the band's
// pixels of each of their output rows in that tile (packed R | G << 8 |
// B << 16 | mask << 24), written a line at a time, and at the band's end read
// it back row-wise so that the stores write whole row runs.
//
// Work items are dealt to the eight per-XCD queues of k_ragged.hip; every wave
// claims its own items, four at a time (the span segments of one band), one
// atomic ahead.
#include "ragged_common.h"

namespace miaug {
namespace {

constexpr int kGWaves = 4;  // waves per workgroup
constexpr int kGThreads = 64 * kGWaves;
constexpr int kGSeg = 64;   // span positions per item: one per lane
constexpr int kGDepth = 7;  // lines whose loads are in flight ahead of the one being blended
constexpr int kGClaim = 4;  // consecutive items claimed per atomic (the span segments of one band)

template <int BAND>
__host__ __device__ __forceinline__ int gather_items_per_image(int OH, int OW) {
    const int a = ((OH + BAND - 1) / BAND) * ((OW + kGSeg - 1) / kGSeg);
    const int b = ((OW + BAND - 1) / BAND) * ((OH + kGSeg - 1) / kGSeg);
    return a > b ? a : b;
}

// Geometry of one item (uniform in the wave).
struct GItem {
    int ok, img, tile, swap;
    int H, W, Ll, Ls, kl, ks, cx, cy, OL, OS, l0, nl, s0, ns;
    int64_t io, mo;
    int iph;  // image base address mod 4 (loads are made from the 4-byte aligned base below it)
    float alpha, beta;
};

template <int BAND>
__device__ __forceinline__ GItem make_gitem(const miaug_ragged_args &a, int img, int tile) {
    const ImgInfo in = info_scalar(a, img);
    GItem it;
    it.img = img;
    it.tile = tile;
    it.H = in.H;
    it.W = in.W;
    it.io = in.io;
    it.mo = in.mo;
    it.alpha = in.alpha;
    it.beta = in.beta;
    bool empty = in.H < 1 || in.W < 1 || in.H >= kMaxSide || in.W >= kMaxSide ||
                 (int64_t)in.H * in.W * 3 >= ((int64_t)1 << 31);
    D4Map m = make_d4(empty ? 1 : in.H, empty ? 1 : in.W, in.f0, in.f1, in.f2, in.f3);
    if (in.wh != 0 && !empty) {
        // crop window (wy, wx, wh, ww) of the Dih4 image; a window that is not
        // inside it skips the image
        if (in.wy < 0 || in.wx < 0 || in.wh < 1 || in.ww < 1 || in.wh > m.oh - in.wy || in.ww > m.ow - in.wx) {
            empty = true;
        } else {
            m.cy += m.ay * in.wy + m.by * in.wx;
            m.cx += m.ax * in.wy + m.bx * in.wx;
            m.oh = in.wh;
            m.ow = in.ww;
        }
    }
    it.swap = m.swaps();
    it.OL = it.swap ? a.out_w : a.out_h;
    it.OS = it.swap ? a.out_h : a.out_w;
    const int nseg = (it.OS + kGSeg - 1) / kGSeg;
    int seg;
    const int band = udiv_small(tile, nseg, seg);
    it.l0 = band * BAND;
    it.s0 = seg * kGSeg;
    if (it.l0 >= it.OL) empty = true;  // spare item of the larger grid
    it.nl = min(BAND, it.OL - it.l0);
    it.ns = min(kGSeg, it.OS - it.s0);
    it.Ll = it.swap ? m.ow : m.oh;
    it.Ls = it.swap ? m.oh : m.ow;
    it.kl = it.swap ? m.by : m.ay;
    it.ks = it.swap ? m.ax : m.bx;
    it.cx = m.cx;
    it.cy = m.cy;
    it.iph = (int)((uintptr_t)(a.img + it.io) & 3);
    it.ok = !empty;
    return it;
}

// The lane's column taps: byte offset in a row of the six-byte window holding
// both column taps (3 min(x0, x1)), whether both taps are the same clamped
// pixel, the Q10 weight and the nearest mask column.
struct GTap {
    int xb, mcol;
    uint32_t w;
    bool same, on;
};

__device__ __forceinline__ GTap gather_tap(const GItem &it) {
    GTap t;
    const int j = (int)(threadIdx.x & 63);
    t.on = j < it.ns;
    const int32_t q = resize_q(it.s0 + (t.on ? j : 0), it.Ls, it.OS);
    const int e0 = clampi(q >> kFBits, it.Ls), e1 = clampi((q >> kFBits) + 1, it.Ls);
    const int en = clampi((q + kFOne / 2) >> kFBits, it.Ls);
    const int x0 = it.ks * e0 + it.cx, x1 = it.ks * e1 + it.cx;
    t.xb = 3 * min(x0, x1);
    t.same = x0 == x1;
    t.w = q & (kFOne - 1);
    t.mcol = it.ks * en + it.cx;
    return t;
}

// One line's source rows (uniform): byte offsets of the two bilinear rows
// from the image's aligned base, of the nearest mask row from the mask's base,
// and the Q10 row weight.
struct GLine {
    int r0, r1, rm;
    uint32_t wy;
};

__device__ __forceinline__ GLine gather_line(const GItem &it, int l) {
    const int32_t q = resize_q(it.l0 + min(l, it.nl - 1), it.Ll, it.OL);
    const int d0 = clampi(q >> kFBits, it.Ll), d1 = clampi((q >> kFBits) + 1, it.Ll);
    const int dn = clampi((q + kFOne / 2) >> kFBits, it.Ll);
    GLine g;
    g.r0 = it.iph + (it.kl * d0 + it.cy) * it.W * 3;
    g.r1 = it.iph + (it.kl * d1 + it.cy) * it.W * 3;
    g.rm = (it.kl * dn + it.cy) * it.W;
    g.wy = q & (kFOne - 1);
    return g;
}

// Line l of the band from the per-lane table (lane l computed line l).
__device__ __forceinline__ GLine line_at(const GLine &tab, int l) {
    GLine g;
    g.r0 = __builtin_amdgcn_readlane(tab.r0, l);
    g.r1 = __builtin_amdgcn_readlane(tab.r1, l);
    g.rm = __builtin_amdgcn_readlane(tab.rm, l);
    g.wy = (uint32_t)__builtin_amdgcn_readlane((int)tab.wy, l);
    return g;
}

typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));

// A line's loads: the two 12-byte windows and the mask byte.
struct GLoads {
    u32x3 a, b;
    uint32_t m;
};

__device__ __forceinline__ GLoads gather_issue(const GLine &g, const GTap &t, __amdgpu_buffer_rsrc_t ri,
                                               __amdgpu_buffer_rsrc_t rm) {
    GLoads L;
    L.a = __builtin_amdgcn_raw_buffer_load_b96(ri, (uint32_t)((g.r0 + t.xb) & ~3), 0, 0);
    L.b = __builtin_amdgcn_raw_buffer_load_b96(ri, (uint32_t)((g.r1 + t.xb) & ~3), 0, 0);
    L.m = __builtin_amdgcn_raw_buffer_load_b8(rm, (uint32_t)(g.rm + t.mcol), 0, 0);
    return L;
}

// The two tap words of one row: the window starts (r + xb) & 3 bytes into the
// loaded dwords; word A holds the pixel at window bytes 0..2, word B the one at
// bytes 3..5.  x0 is A for ks = +1 and B for ks = -1 (the window starts at the
// lower column); a clamped pair is A twice.
__device__ __forceinline__ void row_taps(u32x3 d, int r, const GTap &t, int ks, uint32_t &w0, uint32_t &w1) {
    const uint32_t sh = (uint32_t)((r + t.xb) & 3) * 8;
    const uint32_t lo = __builtin_amdgcn_alignbit(d.y, d.x, sh);
    const uint32_t hi = __builtin_amdgcn_alignbit(d.z, d.y, sh);
    const uint32_t wa = lo, wb = __builtin_amdgcn_alignbit(hi, lo, 24);
    const uint32_t other = t.same ? wa : wb;
    w0 = ks > 0 ? wa : other;
    w1 = ks > 0 ? other : wa;
}

__device__ __forceinline__ uint32_t byte_of(uint32_t w, int c) { return (w >> (8 * c)) & 255u; }

// Blended u8 value of channel c (through the brightness/contrast LUT at every
// tap): px = rhe20(t1 wy + t0 (1024 - wy)) with t_r the row's column blend.
__device__ __forceinline__ void gather_blend(const GLoads &L, const GLine &g, const GTap &t, int ks, const uint8_t *bc,
                                             uint32_t (&px)[3]) {
    uint32_t a0, a1, b0, b1;
    row_taps(L.a, g.r0, t, ks, a0, a1);
    row_taps(L.b, g.r1, t, ks, b0, b1);
    uint32_t v[12];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        v[4 * c] = bc[byte_of(a0, c)];
        v[4 * c + 1] = bc[byte_of(a1, c)];
        v[4 * c + 2] = bc[byte_of(b0, c)];
        v[4 * c + 3] = bc[byte_of(b1, c)];
    }
    const uint32_t ws1 = t.w, ws0 = kFOne - ws1, wl1 = g.wy, wl0 = kFOne - wl1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const uint32_t t0 = umad24(v[4 * c + 1], ws1, __umul24(v[4 * c], ws0));
        const uint32_t t1 = umad24(v[4 * c + 3], ws1, __umul24(v[4 * c + 2], ws0));
        px[c] = rhe20((int)umad24(t1, wl1, __umul24(t0, wl0)));
    }
}

// Word of tile row r, column k: rows of BAND words; the groups of four
// columns are permuted by the row (group g of row r sits at g ^ (r mod 8)), so
// that the 64 lanes' writes of one column spread over the LDS banks while a
// group stays four aligned words for the 16-byte read back.
template <int BAND>
__device__ __forceinline__ int tile_word(int r, int k) {
    return r * BAND + (k ^ ((r & 7 & (BAND / 4 - 1)) << 2));
}

// Band-end store of a swapping element: tile row j holds output row s0 + j,
// columns l0 .. l0 + BAND - 1 (written one line at a time by gather_item).
// The wave reads the tile back as runs of four columns, so that each store
// writes 16 bytes per lane and BAND / 4 lanes cover one output row's BAND
// floats of a plane (whole 64- or 128-byte runs).
template <int BAND>
__device__ __forceinline__ void gather_store_swap(const miaug_ragged_args &a, const GItem &it,
                                                  const float (&nlut)[3][256], const uint32_t *tile) {
    constexpr int LPR = BAND / 4;  // lanes per output row
    constexpr int RPI = 64 / LPR;  // output rows per store
    const int plane = a.out_h * a.out_w;
    const bool has_mask = a.mask != nullptr;
    const int lane = (int)(threadIdx.x & 63);
    __builtin_amdgcn_wave_barrier();
    const __amdgpu_buffer_rsrc_t ro = buffer_rsrc(a.out + (size_t)it.img * 3 * plane, (uint32_t)(12 * plane));
    const __amdgpu_buffer_rsrc_t rmo =
        buffer_rsrc(has_mask ? a.out_mask + (size_t)it.img * plane : a.out_mask, (uint32_t)plane);
    const bool wide = it.nl == BAND && (a.out_w & 3) == 0;
    const int g = lane % LPR;  // column group
#pragma unroll
    for (int r0 = 0; r0 < 64; r0 += RPI) {
        const int r = r0 + lane / LPR;  // row of the tile (output row s0 + r)
        const u32x4 w = *(const u32x4 *)(tile + tile_word<BAND>(r, 4 * g));
        // rows past the segment, and columns past the item, store past the
        // image's outputs (element 3 plane), where the range check drops them
        const int base = r < it.ns ? (it.s0 + r) * a.out_w + it.l0 : 3 * plane;
        if (wide) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                u32x4 v;
                v.x = __float_as_uint(nlut[c][byte_of(w.x, c)]);
                v.y = __float_as_uint(nlut[c][byte_of(w.y, c)]);
                v.z = __float_as_uint(nlut[c][byte_of(w.z, c)]);
                v.w = __float_as_uint(nlut[c][byte_of(w.w, c)]);
                __builtin_amdgcn_raw_buffer_store_b128(v, ro, 4 * (base + 4 * g), 4 * c * plane, 0);
            }
            if (has_mask) {
                const uint32_t mv = (w.x >> 24) | ((w.y >> 24) << 8) | ((w.z >> 24) << 16) | (w.w & 0xff000000u);
                __builtin_amdgcn_raw_buffer_store_b32(mv, rmo, base + 4 * g, 0, 0);
            }
        } else {
            const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = 4 * g + e;
                const int off = k < it.nl ? base + k : 3 * plane;
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(nlut[c][byte_of(ws[e], c)]), ro, 4 * off,
                                                          4 * c * plane, 0);
                if (has_mask) __builtin_amdgcn_raw_buffer_store_b8(ws[e] >> 24, rmo, off, 0, 0);
            }
        }
    }
    __builtin_amdgcn_wave_barrier();  // the tile is rewritten by this wave's next item
}

// Store of four keep-axes lines lf .. lf + 3 of the band from the tile (row
// r = line lf + r, 64 packed pixels): lane j writes line lf + j / 16, span
// positions 4 (j mod 16) .. + 3 -- 16 bytes per plane and 4 mask bytes -- when
// the output rows take 16-byte stores, else one element at a time.  Lines past
// the item and positions past the segment store past the image's outputs
// (element 3 plane), where the buffer range check drops them.
__device__ __forceinline__ void keep_flush(const miaug_ragged_args &a, const GItem &it, const float (&nlut)[3][256],
                                           const uint32_t *tile, int lf, __amdgpu_buffer_rsrc_t ro,
                                           __amdgpu_buffer_rsrc_t rmo) {
    const int plane = a.out_h * a.out_w;
    const bool has_mask = a.mask != nullptr;
    const int lane = (int)(threadIdx.x & 63);
    const int r = lane >> 4, g = lane & 15;
    const u32x4 w = *(const u32x4 *)(tile + r * 64 + 4 * g);
    const int l = lf + r, k = 4 * g;
    const int base = (it.l0 + l) * a.out_w + it.s0;
    if ((a.out_w & 3) == 0 && (it.ns & 3) == 0) {
        const int off = (l < it.nl && k < it.ns) ? base + k : 3 * plane;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            u32x4 v;
            v.x = __float_as_uint(nlut[c][byte_of(w.x, c)]);
            v.y = __float_as_uint(nlut[c][byte_of(w.y, c)]);
            v.z = __float_as_uint(nlut[c][byte_of(w.z, c)]);
            v.w = __float_as_uint(nlut[c][byte_of(w.w, c)]);
            __builtin_amdgcn_raw_buffer_store_b128(v, ro, 4 * off, 4 * c * plane, 0);
        }
        if (has_mask) {
            const uint32_t mv = (w.x >> 24) | ((w.y >> 24) << 8) | ((w.z >> 24) << 16) | (w.w & 0xff000000u);
            __builtin_amdgcn_raw_buffer_store_b32(mv, rmo, off, 0, 0);
        }
    } else {
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int off = (l < it.nl && k + e < it.ns) ? base + k + e : 3 * plane;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(nlut[c][byte_of(ws[e], c)]), ro, 4 * off,
                                                      4 * c * plane, 0);
            if (has_mask) __builtin_amdgcn_raw_buffer_store_b8(ws[e] >> 24, rmo, off, 0, 0);
        }
    }
}

// Boxes of one image by one wave (lane-strided).
__device__ __forceinline__ void gather_boxes(const miaug_ragged_args &a, int img) {
    const int b0 = ldc(a.box_off + img), b1 = ldc(a.box_off + img + 1);
    const int32_t *fl = a.flags + 4 * img;
    const int f0 = ldc(fl), f1 = ldc(fl + 1), f2 = ldc(fl + 2), f3 = ldc(fl + 3);
    for (int b = b0 + (int)(threadIdx.x & 63); b < b1; b += 64) {
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

// One item by one wave: BAND lines, the loads of the next kGDepth lines in
// flight while a line is blended (a ring of kGDepth + 1 load sets, indexed
// statically by unrolling the line loop by that count).  Past the item's last
// line the ring reloads its last line, and such lines store nothing, so every
// iteration issues the same memory instructions.
template <int BAND, bool SWAP>
__device__ __forceinline__ void gather_item(const miaug_ragged_args &a, const GItem &it, const uint8_t *bc,
                                            const float (&nlut)[3][256], uint32_t *tile) {
    constexpr int R = kGDepth + 1;
    static_assert(BAND % R == 0, "the line loop is unrolled by the ring size");
    const int plane = a.out_h * a.out_w;
    const bool has_mask = a.mask != nullptr;
    const GTap tp = gather_tap(it);
    // loads from the 4-byte aligned base below the image; the range ends with
    // the dword that holds the image's last byte (the hardware checks whole
    // dwords), so a window reaching further reads zeros there
    const __amdgpu_buffer_rsrc_t ri =
        buffer_rsrc((void *)(a.img + it.io - it.iph), (uint32_t)((it.iph + it.H * it.W * 3 + 3) & ~3));
    // without masks every mask load is out of range and reads zero
    const __amdgpu_buffer_rsrc_t rm =
        buffer_rsrc(has_mask ? (void *)(a.mask + it.mo) : (void *)a.img, has_mask ? (uint32_t)(it.H * it.W) : 0u);
    const __amdgpu_buffer_rsrc_t ro = buffer_rsrc(a.out + (size_t)it.img * 3 * plane, (uint32_t)(12 * plane));
    const __amdgpu_buffer_rsrc_t rmo =
        buffer_rsrc(has_mask ? a.out_mask + (size_t)it.img * plane : a.out_mask, (uint32_t)plane);
    // the band's line table, lane l holding line l (lines past the item repeat its last)
    const GLine tab = gather_line(it, (int)(threadIdx.x & 63));
    GLoads ring[R];
    GLine lines[R];
#pragma unroll
    for (int u = 0; u < kGDepth; ++u) {
        lines[u] = line_at(tab, min(u, it.nl - 1));
        ring[u] = gather_issue(lines[u], tp, ri, rm);
    }
    for (int l0 = 0; l0 < it.nl; l0 += R) {
#pragma unroll
        for (int u = 0; u < R; ++u) {
            const int l = l0 + u;
            const int ahead = (u + kGDepth) % R;
            lines[ahead] = line_at(tab, min(l + kGDepth, it.nl - 1));
            ring[ahead] = gather_issue(lines[ahead], tp, ri, rm);
            uint32_t px[3];
            gather_blend(ring[u], lines[u], tp, it.ks, bc, px);
            if constexpr (SWAP) {
                // line l of the band is tile column l (lines past the item are never read back)
                tile[tile_word<BAND>((int)(threadIdx.x & 63), l & (BAND - 1))] =
                    px[0] | (px[1] << 8) | (px[2] << 16) | (ring[u].m << 24);
            } else {
                // four lines collect in the tile (row l mod 4) and leave in one
                // store per plane: lane j takes line j / 16, columns 4 (j mod 16) .. + 3
                const int lane = (int)(threadIdx.x & 63);
                tile[(l & 3) * 64 + lane] = px[0] | (px[1] << 8) | (px[2] << 16) | (ring[u].m << 24);
                if ((u & 3) == 3) keep_flush(a, it, nlut, tile, l - 3, ro, rmo);
            }
        }
    }
    if constexpr (SWAP) gather_store_swap<BAND>(a, it, nlut, tile);
}

// The brightness/contrast LUT of image img into this wave's slot.
__device__ __forceinline__ void gather_bc_lut(const GItem &it, uint8_t *bc) {
    const int lane = (int)(threadIdx.x & 63);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = lane + 64 * q;
        bc[e] = (uint8_t)sat8((int)rint((double)it.alpha * (double)e + (double)it.beta));
    }
}

template <int BAND>
__device__ __forceinline__ void gather_run(const miaug_ragged_args &a, int img, int tile, int &bc_img, uint8_t *bc,
                                           const float (&nlut)[3][256], uint32_t *tile_lds) {
    const GItem it = make_gitem<BAND>(a, img, tile);
    if (!it.ok) return;
    if (tile == 0 && a.boxes) gather_boxes(a, img);
    if (bc_img != img) {
        gather_bc_lut(it, bc);
        bc_img = img;
    }
    if (it.swap) gather_item<BAND, true>(a, it, bc, nlut, tile_lds);
    else gather_item<BAND, false>(a, it, bc, nlut, tile_lds);
}

// SYNC = false: every wave claims its own chunks of kGClaim items.  SYNC =
// true: thread 0 claims kGWaves items (the span segments of one band) and wave
// w takes item w, so the four waves read the same source rows at about the
// same time and the 128-byte lines at segment boundaries are fetched once; a
// barrier per band keeps them together.
template <int BAND, bool SYNC>
__global__ __launch_bounds__(kGThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_gather(
    miaug_ragged_args a, int *__restrict__ counters, const int *__restrict__ order) {
    __shared__ float nlut[3][256];
    __shared__ uint8_t bcl[kGWaves][256];
    __shared__ __align__(16) uint32_t tiles[kGWaves][64 * BAND];  // per-wave transpose tile
    __shared__ int3 claim_s;
    build_norm_lut(a, nlut);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    uint8_t *bc = bcl[wave];
    const int per = gather_items_per_image<BAND>(a.out_h, a.out_w);
    int bc_img = -1;
    if constexpr (SYNC) {
        Claimer<kGWaves> C{per, (int)(blockIdx.x % kQueues), 0, 0};  // meaningful in thread 0
        if (threadIdx.x == 0) {
            C.issue(counters);
            claim_s = C.resolve(a, counters);
            C.issue(counters);
        }
        __syncthreads();
        for (;;) {
            const int cq = __builtin_amdgcn_readfirstlane(claim_s.x), cbase = __builtin_amdgcn_readfirstlane(claim_s.y);
            const int cn = __builtin_amdgcn_readfirstlane(claim_s.z);
            if (cn == 0) break;
            if (wave < cn) {
                int tile;
                const int slot = udiv_small(cbase + wave, per, tile) * kQueues + cq;
                const int img = order ? ldc(order + slot) : slot;
                gather_run<BAND>(a, img, tile, bc_img, bc, nlut, tiles[wave]);
            }
            __syncthreads();  // every wave has read claim_s
            if (threadIdx.x == 0) {
                claim_s = C.resolve(a, counters);
                C.issue(counters);  // the next chunk's atomic, in flight during this band
            }
            __syncthreads();
        }
    } else {
        __syncthreads();
        Claimer<kGClaim> C{per, (int)(blockIdx.x % kQueues), 0, 0};  // meaningful in lane 0
        if (lane == 0) C.issue(counters);
        for (;;) {
            int3 ch = make_int3(0, 0, 0);
            if (lane == 0) {
                ch = C.resolve(a, counters);
                C.issue(counters);  // the next chunk's atomic, in flight during this one
            }
            const int cq = __builtin_amdgcn_readfirstlane(ch.x), cbase = __builtin_amdgcn_readfirstlane(ch.y);
            const int cn = __builtin_amdgcn_readfirstlane(ch.z);
            if (cn == 0) break;
            for (int k = 0; k < cn; ++k) {
                int tile;
                const int slot = udiv_small(cbase + k, per, tile) * kQueues + cq;
                const int img = order ? ldc(order + slot) : slot;
                gather_run<BAND>(a, img, tile, bc_img, bc, nlut, tiles[wave]);
            }
        }
    }
}

// Largest-first work order (longest processing time first): image slots
// sorted by an estimate of the source bytes the image's items read --
// min(h, 2 out_h) rows of w pixels (4 bytes with a mask, 3 without) for the
// window (h, w) of its Dih4 image -- in descending order, ties by index, by
// a bitonic sort of (estimate << 32 | ~index) keys in LDS.  Slot j of the
// queues (queue j mod 8, position j / 8) then takes image order[j], so every
// queue starts with its largest images and the last items of the launch are
// small ones.  n <= kLptMax; one workgroup.
__global__ __launch_bounds__(1024) void k_lpt_order(miaug_ragged_args a, int *__restrict__ order) {
    __shared__ uint64_t key[kLptMax];
    const int n = a.n;
    int N = 1;
    while (N < n) N <<= 1;
    for (int i = threadIdx.x; i < N; i += 1024) {
        uint64_t k = 0;
        if (i < n) {
            const bool swap = ((a.flags[4 * i + 2] & 1) ^ (a.flags[4 * i + 3] & 1)) != 0;
            int h = a.hw[2 * i], w = a.hw[2 * i + 1];
            if (swap) {
                const int t = h;
                h = w;
                w = t;
            }
            if (a.crop && a.crop[4 * i + 2] > 0) {
                h = a.crop[4 * i + 2];
                w = a.crop[4 * i + 3];
            }
            const uint64_t rows = (uint64_t)min(max(h, 0), 2 * a.out_h);
            const uint64_t est = min(rows * (uint64_t)max(w, 0) * (a.mask ? 4u : 3u), (uint64_t)0xFFFFFFFFu);
            k = est << 32 | (uint64_t)(0xFFFFFFFFu - (uint32_t)i);
        }
        key[i] = k;
    }
    __syncthreads();
    for (int size = 2; size <= N; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < N / 2; t += 1024) {
                const int lo = 2 * t - (t & (stride - 1)), hi = lo + stride;
                const bool desc = (lo & size) == 0;  // the last merge (size N) is descending throughout
                const uint64_t x = key[lo], y = key[hi];
                if (desc ? x < y : x > y) {
                    key[lo] = y;
                    key[hi] = x;
                }
            }
            __syncthreads();
        }
    for (int i = threadIdx.x; i < n; i += 1024) order[i] = (int)(0xFFFFFFFFu - (uint32_t)key[i]);
}

}  // namespace

hipError_t launch_ragged_gather(const miaug_ragged_args *a, int band, int wg_per_cu, const RaggedLaunch &L,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(256), 0, s, L.counters, kQueues * kCounterStride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int b = band & 63;
    const bool sync = (band & 64) != 0;
    // bit 128: largest images first (index order without a context's order
    // buffer or beyond kLptMax images)
    const int *order = nullptr;
    if ((band & 128) && L.order && a->n <= kLptMax) {
        hipLaunchKernelGGL(k_lpt_order, dim3(1), dim3(1024), 0, s, *a, L.order);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        order = L.order;
    }
    const int per = b == 32 ? gather_items_per_image<32>(a->out_h, a->out_w)
                            : gather_items_per_image<16>(a->out_h, a->out_w);
    int grid = L.num_cu * wg_per_cu;
    const long waves = ((long)a->n * per + kGWaves - 1) / kGWaves;
    if (grid > waves) grid = (int)waves;
    grid = ((grid + kQueues - 1) / kQueues) * kQueues;
    if (b == 32 && sync) hipLaunchKernelGGL((k_gather<32, true>), dim3(grid), dim3(kGThreads), 0, s, *a, L.counters, order);
    else if (b == 32) hipLaunchKernelGGL((k_gather<32, false>), dim3(grid), dim3(kGThreads), 0, s, *a, L.counters, order);
    else if (sync) hipLaunchKernelGGL((k_gather<16, true>), dim3(grid), dim3(kGThreads), 0, s, *a, L.counters, order);
    else hipLaunchKernelGGL((k_gather<16, false>), dim3(grid), dim3(kGThreads), 0, s, *a, L.counters, order);
    return hipGetLastError();
}

}  // namespace miaug
