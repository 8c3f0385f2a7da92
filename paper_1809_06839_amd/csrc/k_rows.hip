// k_rows.hip -- ragged batch in row bands.  Computes exactly what the tile
// passes of k_ragged.hip compute (per image: Dih4 element -> optional crop
// window -> brightness/contrast LUT at every tap -> half-pixel bilinear resize
// -> per-channel normalisation into float32 CHW; masks by the nearest tap;
// boxes through the same geometry; Sec. II-A, Sec. II-B Dih4, Table I
// Brightness), with the work cut so that every staged source segment is a
// whole row of the image (of the crop window), read in full 128-byte lines.
//
// Line and span axes are those of k_ragged.hip: the resize needs two source
// rows per output line (output rows, or output columns when the element swaps
// the axes) and one run of source columns along the span.  A work item is an
// image, a band of up to 16 consecutive output lines and a span segment of up
// to 256 positions (one per worker thread; 224-wide outputs have one segment).
// For a band the workgroup streams, line group by line group ("steps"), the
// source rows the lines' taps read -- each row once per step, so rows shared
// by neighbouring lines of upscaled or mildly downscaled images are staged
// once -- plus each line's nearest mask row, into LDS with LDS-DMA
// (global_load_lds_dwordx4, 16 bytes per lane).  A step holds as many lines
// as fit the stage.
//
// Workgroup: four worker waves and a planning wave, one barrier per step.  In
// step k the planner claims items and builds the tables of step k+2 (row list
// for the DMA, per-line LDS offsets and weights); the workers issue the DMA of
// step k+1 into one of two stages (distinct LDS variables, so the compiler
// keeps the blend's LDS reads of the other stage free of waits on it), then
// blend step k.  Worker thread t owns span position s0 + t for the whole band:
// its two column taps, weight and nearest mask column are computed once per
// item.  When the element keeps the axes a line is an output row and each
// blended line is stored at once (consecutive lanes, consecutive floats).
// When it swaps them, a line is an output column: thread t collects its
// output row's pixels of the band in registers (packed RGB + mask) and writes
// the row's 16 floats per plane, 64 bytes, at the band's end.
//
// An item whose single line does not fit a stage (a source row of more than
// about 2,700 pixels across the span segment) runs on direct global loads.
// Queues, claims, skipped images and boxes are those of k_ragged.hip.
#include "ragged_common.h"

namespace miaug {
namespace {

constexpr int kRW = 256;       // worker threads: thread t owns span position s0 + t
constexpr int kRT = kRW + 64;  // workers + the planning wave
constexpr int kBand = 16;      // output lines per item
constexpr int kSeg = kRW;      // span positions per item
constexpr int kRowSlots = 3 * kBand;  // staged rows per step: 2 image rows + 1 mask row per line, at most

// A stage of CAP 16-byte chunks plus slack.
constexpr int rows_stage_bytes(int cap) { return cap * 16 + 16; }

// Items per image: the band x segment grid depends on whether the element
// swaps the axes; the queue reserves the larger count.
__host__ __device__ __forceinline__ int row_items_per_image(int OH, int OW) {
    const int a = ((OH + kBand - 1) / kBand) * ((OW + kSeg - 1) / kSeg);
    const int b = ((OW + kBand - 1) / kBand) * ((OH + kSeg - 1) / kSeg);
    return a > b ? a : b;
}

// Geometry of one item (planning wave; every value uniform).
struct RowItem {
    int valid, empty, direct;
    int img, tile, swap;
    int W, Ll, Ls, kl, ks, cx, cy, OL, OS, l0, nl, s0, ns;
    int sxlo, nsx, mxlo, nmx, nchi, nchm, ph, mph;
    int64_t io, mo;
    float alpha, beta;
};

template <int CAP>
__device__ __forceinline__ RowItem make_row_item(const miaug_ragged_args &a, int img, int tile) {
    const ImgInfo in = info_scalar(a, img);
    RowItem it;
    it.valid = 1;
    it.img = img;
    it.tile = tile;
    it.W = in.W;
    it.io = in.io;
    it.mo = in.mo;
    it.alpha = in.alpha;
    it.beta = in.beta;
    const int H = in.H, W = in.W;
    it.empty = H < 1 || W < 1 || H >= kMaxSide || W >= kMaxSide || (int64_t)H * W * 3 >= ((int64_t)1 << 31);
    D4Map m = make_d4(it.empty ? 1 : H, it.empty ? 1 : W, in.f0, in.f1, in.f2, in.f3);
    if (in.wh != 0 && !it.empty) {
        // crop window (wy, wx, wh, ww) of the Dih4 image; a window that is not
        // inside it skips the image
        if (in.wy < 0 || in.wx < 0 || in.wh < 1 || in.ww < 1 || in.wh > m.oh - in.wy || in.ww > m.ow - in.wx) {
            it.empty = 1;
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
    const int nseg = (it.OS + kSeg - 1) / kSeg;
    int seg;
    const int band = udiv_small(tile, nseg, seg);
    it.l0 = band * kBand;
    it.s0 = seg * kSeg;
    if (it.l0 >= it.OL) it.empty = 1;  // spare item of the larger grid
    it.nl = min(kBand, it.OL - it.l0);
    it.ns = min(kSeg, it.OS - it.s0);
    it.Ll = it.swap ? m.ow : m.oh;
    it.Ls = it.swap ? m.oh : m.ow;
    it.kl = it.swap ? m.by : m.ay;
    it.ks = it.swap ? m.ax : m.bx;
    it.cx = m.cx;
    it.cy = m.cy;
    it.sxlo = it.nsx = it.mxlo = it.nmx = it.nchi = it.nchm = it.ph = it.mph = 0;
    it.direct = 0;
    if (it.empty) return it;
    const int32_t qf = resize_q(it.s0, it.Ls, it.OS), ql = resize_q(it.s0 + it.ns - 1, it.Ls, it.OS);
    const int dlo = clampi(qf >> kFBits, it.Ls), dhi = clampi((ql >> kFBits) + 1, it.Ls);
    const int xa = it.ks * dlo + it.cx, xb = it.ks * dhi + it.cx;
    it.sxlo = min(xa, xb);
    it.nsx = abs(xb - xa) + 1;
    const int nlo = clampi((qf + kFOne / 2) >> kFBits, it.Ls), nhi = clampi((ql + kFOne / 2) >> kFBits, it.Ls);
    const int mxa = it.ks * nlo + it.cx, mxb = it.ks * nhi + it.cx;
    it.mxlo = min(mxa, mxb);
    it.nmx = abs(mxb - mxa) + 1;
    it.nchi = (3 * it.nsx + 30) >> 4;  // most chunks a row segment of 3 nsx bytes can touch
    it.nchm = a.mask ? (it.nmx + 30) >> 4 : 0;
    it.ph = (int)((uintptr_t)(a.img + it.io) & 15);
    it.mph = a.mask ? (int)((uintptr_t)(a.mask + it.mo) & 15) : 0;
    it.direct = 2 * it.nchi + it.nchm > CAP;
    return it;
}

// Step record in LDS (one int each), written by lane 0 of the planner.
enum {
    R_VALID, R_DIRECT, R_IMG, R_SWAP, R_FIRST, R_LAST, R_NEWIMG, R_BOXES, R_BCSLOT, R_G, R_LREL, R_CROWS, R_MROWS,
    R_NCHI, R_NCHM, R_W, R_LL, R_LS, R_KL, R_KS, R_CX, R_CY, R_OL, R_OS, R_L0, R_NL, R_S0, R_NS, R_SXLO, R_MXLO,
    R_IOFF, R_MOFF = R_IOFF + 2, R_ALPHA = R_MOFF + 2, R_BETA, R_N
};

struct RowStep {
    int valid, direct, img, swap, first, last, newimg, boxes, bcslot, G, lrel, crows, mrows, nchi, nchm;
    int W, Ll, Ls, kl, ks, cx, cy, OL, OS, l0, nl, s0, ns, sxlo, mxlo;
    int64_t io, mo;
    float alpha, beta;
};

__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ RowStep read_step(const int *s) {
    RowStep r;
    r.valid = rfl(s[R_VALID]);
    r.direct = rfl(s[R_DIRECT]);
    r.img = rfl(s[R_IMG]);
    r.swap = rfl(s[R_SWAP]);
    r.first = rfl(s[R_FIRST]);
    r.last = rfl(s[R_LAST]);
    r.newimg = rfl(s[R_NEWIMG]);
    r.boxes = rfl(s[R_BOXES]);
    r.bcslot = rfl(s[R_BCSLOT]);
    r.G = rfl(s[R_G]);
    r.lrel = rfl(s[R_LREL]);
    r.crows = rfl(s[R_CROWS]);
    r.mrows = rfl(s[R_MROWS]);
    r.nchi = rfl(s[R_NCHI]);
    r.nchm = rfl(s[R_NCHM]);
    r.W = rfl(s[R_W]);
    r.Ll = rfl(s[R_LL]);
    r.Ls = rfl(s[R_LS]);
    r.kl = rfl(s[R_KL]);
    r.ks = rfl(s[R_KS]);
    r.cx = rfl(s[R_CX]);
    r.cy = rfl(s[R_CY]);
    r.OL = rfl(s[R_OL]);
    r.OS = rfl(s[R_OS]);
    r.l0 = rfl(s[R_L0]);
    r.nl = rfl(s[R_NL]);
    r.s0 = rfl(s[R_S0]);
    r.ns = rfl(s[R_NS]);
    r.sxlo = rfl(s[R_SXLO]);
    r.mxlo = rfl(s[R_MXLO]);
    r.io = (int64_t)(((uint64_t)(uint32_t)rfl(s[R_IOFF + 1]) << 32) | (uint32_t)rfl(s[R_IOFF]));
    r.mo = (int64_t)(((uint64_t)(uint32_t)rfl(s[R_MOFF + 1]) << 32) | (uint32_t)rfl(s[R_MOFF]));
    r.alpha = __int_as_float(rfl(s[R_ALPHA]));
    r.beta = __int_as_float(rfl(s[R_BETA]));
    return r;
}

// What the workers need of the next step: its DMA and, for a new image, its
// brightness/contrast LUT.
struct RowNext {
    int valid, direct, newimg, bcslot, crows, mrows, nchi, nchm;
    int64_t io, mo;
    float alpha, beta;
};

__device__ __forceinline__ RowNext read_next(const int *s) {
    RowNext r;
    r.valid = rfl(s[R_VALID]);
    r.direct = rfl(s[R_DIRECT]);
    r.newimg = rfl(s[R_NEWIMG]);
    r.bcslot = rfl(s[R_BCSLOT]);
    r.crows = rfl(s[R_CROWS]);
    r.mrows = rfl(s[R_MROWS]);
    r.nchi = rfl(s[R_NCHI]);
    r.nchm = rfl(s[R_NCHM]);
    r.io = (int64_t)(((uint64_t)(uint32_t)rfl(s[R_IOFF + 1]) << 32) | (uint32_t)rfl(s[R_IOFF]));
    r.mo = (int64_t)(((uint64_t)(uint32_t)rfl(s[R_MOFF + 1]) << 32) | (uint32_t)rfl(s[R_MOFF]));
    r.alpha = __int_as_float(rfl(s[R_ALPHA]));
    r.beta = __int_as_float(rfl(s[R_BETA]));
    return r;
}

__device__ __forceinline__ int wave_scan_incl(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Planner: the next step of item `it` from its line `next` (relative to the
// band) into one table set; returns the number of lines it takes.  Lane j
// looks at line next + j.  Along the line axis the resize positions are
// monotone, so the rows a line reads that are not already staged are the ones
// above every row staged before: with C_j the running count of staged rows,
// line j's lower tap is row C_j - 2 of the stage (C_j - 1 when both taps are
// the same clamped row) and its upper tap row C_j - 1; masks likewise with one
// row per line.  The step ends at the last line whose cumulative chunks fit.
template <int CAP>
__device__ __forceinline__ int plan_rows(const miaug_ragged_args &a, const RowItem &it, int next, int *meta,
                                         int2 *rowtab, int4 *linetab) {
    const int lane = threadIdx.x & 63;
    const int rem = it.nl - next;
    const bool live = lane < rem;
    const int l = it.l0 + next + min(lane, rem - 1);
    const int32_t q = resize_q(l, it.Ll, it.OL);
    const int d0 = clampi(q >> kFBits, it.Ll), d1 = clampi((q >> kFBits) + 1, it.Ll);
    const int dn = clampi((q + kFOne / 2) >> kFBits, it.Ll);
    const int pd1 = __shfl_up(d1, 1, 64), pdn = __shfl_up(dn, 1, 64);
    const bool first = lane == 0;
    const int new1 = (first || d1 > pd1) ? 1 : 0;
    const int new0 = (d0 != d1 && (first || d0 > pd1)) ? 1 : 0;
    const bool has_mask = a.mask != nullptr;
    const int mnew = (has_mask && (first || dn > pdn)) ? 1 : 0;
    const int C = wave_scan_incl(new0 + new1);
    const int M = wave_scan_incl(mnew);
    const bool fits = live && C * it.nchi + M * it.nchm <= CAP;
    const int G = max(1, (int)__builtin_popcountll(__ballot(fits)));
    const int Ct = __builtin_amdgcn_readlane(C, G - 1), Mt = __builtin_amdgcn_readlane(M, G - 1);
    if (lane < G) {
        // rows are < 2^31 bytes into the image: 32-bit offsets from its aligned base
        const int r0 = it.ph + ((it.kl * d0 + it.cy) * it.W + it.sxlo) * 3;
        const int r1 = it.ph + ((it.kl * d1 + it.cy) * it.W + it.sxlo) * 3;
        if (new0) rowtab[C - 2] = make_int2(r0 & ~15, ((r0 & 15) + 3 * it.nsx + 15) >> 4);
        if (new1) rowtab[C - 1] = make_int2(r1 & ~15, ((r1 & 15) + 3 * it.nsx + 15) >> 4);
        int mofs = 0;
        if (has_mask) {
            const int rm = it.mph + (it.kl * dn + it.cy) * it.W + it.mxlo;
            if (mnew) rowtab[Ct + M - 1] = make_int2(rm & ~15, ((rm & 15) + it.nmx + 15) >> 4);
            mofs = 16 * (Ct * it.nchi + (M - 1) * it.nchm) + (rm & 15);
        }
        const int s1 = C - 1, s0 = d0 == d1 ? C - 1 : C - 2;
        linetab[lane] = make_int4(16 * it.nchi * s0 + (r0 & 15), 16 * it.nchi * s1 + (r1 & 15), q & (kFOne - 1), mofs);
    }
    if (lane == 0) {
        meta[R_CROWS] = Ct;
        meta[R_MROWS] = Mt;
    }
    return G;
}

// Lane 0 of the planner: the item part of a step record.
__device__ __forceinline__ void write_item_meta(const RowItem &it, int *meta) {
    meta[R_VALID] = 1;
    meta[R_DIRECT] = it.direct;
    meta[R_IMG] = it.img;
    meta[R_SWAP] = it.swap;
    meta[R_NCHI] = it.nchi;
    meta[R_NCHM] = it.nchm;
    meta[R_W] = it.W;
    meta[R_LL] = it.Ll;
    meta[R_LS] = it.Ls;
    meta[R_KL] = it.kl;
    meta[R_KS] = it.ks;
    meta[R_CX] = it.cx;
    meta[R_CY] = it.cy;
    meta[R_OL] = it.OL;
    meta[R_OS] = it.OS;
    meta[R_L0] = it.l0;
    meta[R_NL] = it.nl;
    meta[R_S0] = it.s0;
    meta[R_NS] = it.ns;
    meta[R_SXLO] = it.sxlo;
    meta[R_MXLO] = it.mxlo;
    meta[R_IOFF] = (int)(uint32_t)it.io;
    meta[R_IOFF + 1] = (int)(uint32_t)((uint64_t)it.io >> 32);
    meta[R_MOFF] = (int)(uint32_t)it.mo;
    meta[R_MOFF + 1] = (int)(uint32_t)((uint64_t)it.mo >> 32);
    meta[R_ALPHA] = __float_as_int(it.alpha);
    meta[R_BETA] = __float_as_int(it.beta);
}

// Planning wave state: the current item, its next unplanned line, the image of
// the last planned step and the brightness/contrast LUT slot of that image.
template <int CAP>
struct RowPlanner {
    Claimer<1> C;
    RowItem it;
    int next, prev_img, bcslot;

    // Claims items until a non-empty one (or the end of the stream).
    __device__ __forceinline__ void advance(const miaug_ragged_args &a, int *counters) {
        for (;;) {
            int v = -1;
            if ((threadIdx.x & 63) == 0) v = claim_item(C, a, counters);
            const int item = __builtin_amdgcn_readfirstlane(v);
            if (item < 0) {
                it.valid = 0;
                return;
            }
            int tile;
            const int img = udiv_small(item, C.tiles, tile);
            it = make_row_item<CAP>(a, img, tile);
            if (!it.empty) break;
        }
        next = 0;
    }

    // The next step into one table set.
    __device__ __forceinline__ void plan(const miaug_ragged_args &a, int *counters, int *meta, int2 *rowtab,
                                         int4 *linetab) {
        const int lane = threadIdx.x & 63;
        if (it.valid && next >= it.nl) advance(a, counters);
        if (!it.valid) {
            if (lane == 0) meta[R_VALID] = 0;
            return;
        }
        const bool first = next == 0;
        const bool newimg = first && it.img != prev_img;
        if (newimg) {
            bcslot ^= 1;
            prev_img = it.img;
        }
        const int lrel = next;
        int G;
        if (it.direct) {
            G = it.nl - next;
            if (lane == 0) meta[R_CROWS] = meta[R_MROWS] = 0;
        } else {
            G = plan_rows<CAP>(a, it, next, meta, rowtab, linetab);
        }
        next += G;
        if (lane == 0) {
            write_item_meta(it, meta);
            meta[R_FIRST] = first;
            meta[R_LAST] = next >= it.nl;
            meta[R_NEWIMG] = newimg;
            meta[R_BOXES] = first && it.tile == 0;
            meta[R_BCSLOT] = bcslot;
            meta[R_G] = G;
            meta[R_LREL] = lrel;
        }
    }
};

// Workers: the LDS-DMA of a step.  Chunk c of the step (image rows first, C
// slots of nchi chunks, then M mask slots of nchm chunks) lands at stage byte
// 16 c; 64 lanes of a wave take 64 consecutive chunks (the DMA writes lane l
// at its LDS base + 16 l).  Row-table reads go in groups of four ahead of
// their DMAs.  Completion is counted by vmcnt.
template <int CAP, int N>
__device__ __forceinline__ void rows_dma(const miaug_ragged_args &a, const RowNext &m, const int2 *rowtab,
                                         uint8_t (&st)[N]) {
    constexpr int kIt = (CAP + kRW - 1) / kRW;
    constexpr int kB = 4;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wbase = __builtin_amdgcn_readfirstlane(tid - lane);
    const int items = m.crows * m.nchi;
    auto issue = [&](const __amdgpu_buffer_rsrc_t rs, int n, int d, int r0, int smax, int sbase) {
        const uint32_t M = div_magic(d);
#pragma unroll
        for (int u0 = 0; u0 < kIt; u0 += kB) {
            if (wbase + u0 * kRW >= n) break;  // uniform per wave
            int2 r[kB];
            int ch[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int it = tid + (u0 + u) * kRW;
                const int slot = div_by_m(it, d, M);
                ch[u] = it - slot * d;
                r[u] = rowtab[r0 + min(slot, smax)];
            }
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                if (u0 + u >= kIt || wbase + (u0 + u) * kRW >= n) break;
                const int it = tid + (u0 + u) * kRW;
                if (it < n && ch[u] < r[u].y)
                    dma16(rs, st + 16 * (sbase + wbase + (u0 + u) * kRW), (uint32_t)(r[u].x + 16 * ch[u]));
            }
        }
    };
    issue(buffer_rsrc((void *)align16(a.img + m.io), 0x7fffffffu), items, m.nchi, 0, m.crows - 1, 0);
    if (m.mrows > 0)
        issue(buffer_rsrc((void *)align16(a.mask + m.mo), 0x7fffffffu), m.mrows * m.nchm, m.nchm, m.crows,
              m.mrows - 1, items);
}

// Per-thread span taps of an item: byte offsets of the two column taps inside
// a staged row, the Q10 weight and the nearest mask column; `on` is false for
// threads past the segment (they read offset 0 and store nothing).
struct SpanTaps {
    int c0, c1, w, mc;
    bool on;
};

__device__ __forceinline__ SpanTaps span_taps(const RowStep &m, bool has_mask) {
    SpanTaps t;
    const int j = threadIdx.x;
    t.on = j < m.ns;
    t.c0 = t.c1 = t.w = t.mc = 0;
    if (t.on) {
        const int32_t q = resize_q(m.s0 + j, m.Ls, m.OS);
        const int e0 = clampi(q >> kFBits, m.Ls), e1 = clampi((q >> kFBits) + 1, m.Ls);
        const int en = clampi((q + kFOne / 2) >> kFBits, m.Ls);
        t.c0 = 3 * (m.ks * e0 + m.cx - m.sxlo);
        t.c1 = 3 * (m.ks * e1 + m.cx - m.sxlo);
        t.w = q & (kFOne - 1);
        t.mc = has_mask ? m.ks * en + m.cx - m.mxlo : 0;
    }
    return t;
}

// Blend of a staged step: thread t, every line g of the step, kG lines at a
// time with their LDS reads issued together.  Lines past the step re-read the
// last line and store nothing.  Keep-axes elements store each line's pixel at
// once; swapping elements put it into acc[line within the band] (packed
// R | G << 8 | B << 16 | mask << 24) for the band-end store.
template <int N>
__device__ __forceinline__ void rows_blend(const miaug_ragged_args &a, const RowStep &m, const uint8_t (&st)[N],
                                           const int4 *linetab, const uint8_t *bc, const float (&nlut)[3][256],
                                           const SpanTaps &tp, uint32_t (&acc)[kBand]) {
    const int plane = a.out_h * a.out_w;  // outputs are at most 4096 x 4096
    const bool has_mask = a.mask != nullptr;
    const __amdgpu_buffer_rsrc_t ro = buffer_rsrc(a.out + (size_t)m.img * 3 * plane, (uint32_t)(12 * plane));
    const __amdgpu_buffer_rsrc_t rm =
        buffer_rsrc(has_mask ? a.out_mask + (size_t)m.img * plane : a.out_mask, (uint32_t)plane);
    constexpr int kG = 2;
    const uint32_t ws1 = tp.w, ws0 = kFOne - ws1;
    for (int g0 = 0; g0 < m.G; g0 += kG) {
        uint32_t v[kG][12], mk[kG], wl[kG];
#pragma unroll
        for (int gg = 0; gg < kG; ++gg) {
            const int g = min(g0 + gg, m.G - 1);
            const int4 L = linetab[g];
            const int ax = rfl(L.x), ay = rfl(L.y);
            wl[gg] = rfl(L.z);
            const int o00 = ax + tp.c0, o01 = ax + tp.c1, o10 = ay + tp.c0, o11 = ay + tp.c1;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                v[gg][4 * c] = st[o00 + c];
                v[gg][4 * c + 1] = st[o01 + c];
                v[gg][4 * c + 2] = st[o10 + c];
                v[gg][4 * c + 3] = st[o11 + c];
            }
            mk[gg] = st[rfl(L.w) + tp.mc];
        }
#pragma unroll
        for (int gg = 0; gg < kG; ++gg)
#pragma unroll
            for (int e = 0; e < 12; ++e) v[gg][e] = bc[v[gg][e]];
#pragma unroll
        for (int gg = 0; gg < kG; ++gg) {
            const uint32_t wl1 = wl[gg], wl0 = kFOne - wl1;
            uint32_t px[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint32_t t0 = umad24(v[gg][4 * c + 1], ws1, __umul24(v[gg][4 * c], ws0));
                const uint32_t t1 = umad24(v[gg][4 * c + 3], ws1, __umul24(v[gg][4 * c + 2], ws0));
                px[c] = rhe20((int)umad24(t1, wl1, __umul24(t0, wl0)));
            }
            const int g = g0 + gg;
            if (g >= m.G) break;  // uniform
            const int line = m.lrel + g;
            if (m.swap) {
                acc[line] = px[0] | (px[1] << 8) | (px[2] << 16) | (mk[gg] << 24);
            } else if (tp.on) {
                const int off = (m.l0 + line) * a.out_w + m.s0 + (int)threadIdx.x;
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(nlut[c][px[c]]), ro, 4 * off, 4 * c * plane,
                                                          0);
                if (has_mask) __builtin_amdgcn_raw_buffer_store_b8(mk[gg], rm, off, 0, 0);
            }
        }
    }
}

// Band-end store of a swapping element: thread t writes output row s0 + t,
// columns l0 .. l0 + nl - 1 (16 floats per plane, 64 bytes, when the row is
// 16-byte aligned and the band full).
__device__ __forceinline__ void rows_store_swap(const miaug_ragged_args &a, const RowStep &m,
                                                const float (&nlut)[3][256], const SpanTaps &tp,
                                                const uint32_t (&acc)[kBand]) {
    if (!tp.on) return;
    const int plane = a.out_h * a.out_w;
    const bool has_mask = a.mask != nullptr;
    const __amdgpu_buffer_rsrc_t ro = buffer_rsrc(a.out + (size_t)m.img * 3 * plane, (uint32_t)(12 * plane));
    const __amdgpu_buffer_rsrc_t rm =
        buffer_rsrc(has_mask ? a.out_mask + (size_t)m.img * plane : a.out_mask, (uint32_t)plane);
    const int off = (m.s0 + (int)threadIdx.x) * a.out_w + m.l0;  // element offset of the row segment
    if (m.nl == kBand && (a.out_w & 3) == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int k = 0; k < kBand; k += 4) {
                u32x4 v;
                v.x = __float_as_uint(nlut[c][(acc[k] >> (8 * c)) & 255]);
                v.y = __float_as_uint(nlut[c][(acc[k + 1] >> (8 * c)) & 255]);
                v.z = __float_as_uint(nlut[c][(acc[k + 2] >> (8 * c)) & 255]);
                v.w = __float_as_uint(nlut[c][(acc[k + 3] >> (8 * c)) & 255]);
                __builtin_amdgcn_raw_buffer_store_b128(v, ro, 4 * (off + k), 4 * c * plane, 0);
            }
        }
    } else {
        for (int k = 0; k < m.nl; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(nlut[c][(acc[k] >> (8 * c)) & 255]), ro,
                                                      4 * (off + k), 4 * c * plane, 0);
    }
    if (!has_mask) return;
    if (m.nl == kBand && (a.out_w & 15) == 0) {
        u32x4 v;
        v.x = (acc[0] >> 24) | ((acc[1] >> 24) << 8) | ((acc[2] >> 24) << 16) | (acc[3] & 0xff000000u);
        v.y = (acc[4] >> 24) | ((acc[5] >> 24) << 8) | ((acc[6] >> 24) << 16) | (acc[7] & 0xff000000u);
        v.z = (acc[8] >> 24) | ((acc[9] >> 24) << 8) | ((acc[10] >> 24) << 16) | (acc[11] & 0xff000000u);
        v.w = (acc[12] >> 24) | ((acc[13] >> 24) << 8) | ((acc[14] >> 24) << 16) | (acc[15] & 0xff000000u);
        __builtin_amdgcn_raw_buffer_store_b128(v, rm, off, 0, 0);
    } else {
        for (int k = 0; k < m.nl; ++k) __builtin_amdgcn_raw_buffer_store_b8(acc[k] >> 24, rm, off + k, 0, 0);
    }
}

// An item whose line does not fit a stage: every pixel from global memory
// (thread t, span position s0 + t, every line of the band), stored at once.
__device__ __forceinline__ void rows_direct(const miaug_ragged_args &a, const RowStep &m, const uint8_t *bc,
                                            const float (&nlut)[3][256], const SpanTaps &tp) {
    if (!tp.on) return;
    const size_t plane = (size_t)a.out_h * a.out_w;
    const uint8_t *ib = a.img + m.io;
    const uint8_t *mb = a.mask ? a.mask + m.mo : nullptr;
    const int si = m.s0 + (int)threadIdx.x;
    const int32_t qs = resize_q(si, m.Ls, m.OS);
    const int ws1 = qs & (kFOne - 1);
    const int x0 = m.ks * clampi(qs >> kFBits, m.Ls) + m.cx, x1 = m.ks * clampi((qs >> kFBits) + 1, m.Ls) + m.cx;
    const int mx = m.ks * clampi((qs + kFOne / 2) >> kFBits, m.Ls) + m.cx;
    for (int g = 0; g < m.G; ++g) {
        const int li = m.l0 + m.lrel + g;
        const int32_t ql = resize_q(li, m.Ll, m.OL);
        const int wl1 = ql & (kFOne - 1);
        const int y0 = m.kl * clampi(ql >> kFBits, m.Ll) + m.cy, y1 = m.kl * clampi((ql >> kFBits) + 1, m.Ll) + m.cy;
        const uint8_t *r0 = ib + (size_t)y0 * m.W * 3, *r1 = ib + (size_t)y1 * m.W * 3;
        const int jj = m.swap ? si : li, ii = m.swap ? li : si;
        float *o = a.out + (size_t)m.img * 3 * plane + (size_t)jj * a.out_w + ii;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int p00 = bc[r0[3 * x0 + c]], p01 = bc[r0[3 * x1 + c]];
            const int p10 = bc[r1[3 * x0 + c]], p11 = bc[r1[3 * x1 + c]];
            const int t0 = (p00 << kFBits) + ws1 * (p01 - p00);
            const int t1 = (p10 << kFBits) + ws1 * (p11 - p10);
            o[c * plane] = nlut[c][rhe20((t0 << kFBits) + wl1 * (t1 - t0))];
        }
        if (mb) {
            const int my = m.kl * clampi((ql + kFOne / 2) >> kFBits, m.Ll) + m.cy;
            a.out_mask[(size_t)m.img * plane + (size_t)jj * a.out_w + ii] = mb[(size_t)my * m.W + mx];
        }
    }
}

// One iteration of the workers (step k in stage `cur`, DMA of step k+1 into
// `nxt`): boxes of a new image first (their global loads would otherwise wait
// behind the DMA), the DMA, the LUT of step k+1's image when it changes, then
// the blend of step k.
template <int CAP, int N>
__device__ __forceinline__ void rows_work(const miaug_ragged_args &a, const RowStep &mk, const RowNext &mn,
                                          const int2 *rt_next, const int4 *lt_cur, const uint8_t (&cur)[N],
                                          uint8_t (&nxt)[N], uint8_t (*bc)[256], const float (&nlut)[3][256],
                                          SpanTaps &tp, uint32_t (&acc)[kBand]) {
    if (mk.boxes && a.boxes) ragged_boxes<kRW>(a, mk.img);
    if (mn.valid && !mn.direct) rows_dma<CAP>(a, mn, rt_next, nxt);
    if (mn.valid && mn.newimg) build_bc_lut(mn.alpha, mn.beta, bc[mn.bcslot]);
    if (mk.first) tp = span_taps(mk, a.mask != nullptr);
    if (mk.direct) {
        rows_direct(a, mk, bc[mk.bcslot], nlut, tp);
    } else {
        rows_blend(a, mk, cur, lt_cur, bc[mk.bcslot], nlut, tp, acc);
        if (mk.swap && mk.last) rows_store_swap(a, mk, nlut, tp, acc);
    }
}

template <int CAP>
__global__ __launch_bounds__(kRT) void k_rows(miaug_ragged_args a, int *__restrict__ counters) {
    __shared__ __align__(16) uint8_t st0[rows_stage_bytes(CAP)];  // two distinct variables: see the file comment
    __shared__ __align__(16) uint8_t st1[rows_stage_bytes(CAP)];
    __shared__ __align__(16) int meta[3][R_N];
    __shared__ int2 rowtab[3][kRowSlots];
    __shared__ int4 linetab[3][kBand];
    __shared__ float nlut[3][256];
    __shared__ uint8_t bc[2][256];
    const bool planner = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == kRW / 64;
    if (planner) {
        __builtin_amdgcn_s_setprio(2);
        RowPlanner<CAP> P;
        P.C = Claimer<1>{row_items_per_image(a.out_h, a.out_w), (int)(blockIdx.x % kQueues), 0, 0};
        P.it.valid = 1;
        P.next = 0;
        P.prev_img = -1;
        P.bcslot = 1;
        if ((threadIdx.x & 63) == 0) P.C.issue(counters);
        P.advance(a, counters);
        P.plan(a, counters, meta[0], rowtab[0], linetab[0]);
        P.plan(a, counters, meta[1], rowtab[1], linetab[1]);
        __syncthreads();
        __syncthreads();
        for (int s = 0;; s = s == 2 ? 0 : s + 1) {
            if (!__builtin_amdgcn_readfirstlane(meta[s][R_VALID])) break;
            const int s2 = s == 0 ? 2 : s - 1;  // (s + 2) mod 3
            P.plan(a, counters, meta[s2], rowtab[s2], linetab[s2]);
            __syncthreads();
        }
        return;
    }
    for (int e = threadIdx.x; e < 3 * 256; e += kRW) {  // workers only
        const int c = e >> 8, v = e & 255;
        nlut[c][v] = (float)((((double)v / 255.0) - (double)a.mean[c]) / (double)a.stdv[c]);
    }
    __syncthreads();
    {
        const RowNext m0 = read_next(meta[0]);
        if (m0.valid) {
            build_bc_lut(m0.alpha, m0.beta, bc[m0.bcslot]);
            if (!m0.direct) rows_dma<CAP>(a, m0, rowtab[0], st0);
        }
        __builtin_amdgcn_s_waitcnt(0);  // LDS-DMA writes are counted by vmcnt
    }
    __syncthreads();
    SpanTaps tp{0, 0, 0, 0, false};
    uint32_t acc[kBand];
#pragma unroll
    for (int k = 0; k < kBand; ++k) acc[k] = 0;
    for (int k = 0, s = 0;; ++k, s = s == 2 ? 0 : s + 1) {
        const RowStep mk = read_step(meta[s]);
        if (!mk.valid) break;
        const int s1 = s == 2 ? 0 : s + 1;
        const RowNext mn = read_next(meta[s1]);
        if (k & 1) rows_work<CAP>(a, mk, mn, rowtab[s1], linetab[s], st1, st0, bc, nlut, tp, acc);
        else rows_work<CAP>(a, mk, mn, rowtab[s1], linetab[s], st0, st1, bc, nlut, tp, acc);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_ragged_rows(const miaug_ragged_args *a, int cap_kind, int wg_per_cu, const RaggedLaunch &L,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(256), 0, s, L.counters, kQueues * kCounterStride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int per = row_items_per_image(a->out_h, a->out_w);
    int grid = L.num_cu * wg_per_cu;
    const long items = (long)a->n * per;
    if (grid > items) grid = (int)items;
    grid = ((grid + kQueues - 1) / kQueues) * kQueues;
    if (cap_kind == 1) hipLaunchKernelGGL((k_rows<576>), dim3(grid), dim3(kRT), 0, s, *a, L.counters);
    else if (cap_kind == 2) hipLaunchKernelGGL((k_rows<2304>), dim3(grid), dim3(kRT), 0, s, *a, L.counters);
    else hipLaunchKernelGGL((k_rows<1088>), dim3(grid), dim3(kRT), 0, s, *a, L.counters);
    return hipGetLastError();
}

}  // namespace miaug
