// k_ragged.hip -- ragged batch: Dih4 + brightness/contrast -> bilinear resize
// -> per-channel normalisation into float32 CHW, with masks (nearest) and
// boxes following the same geometry (Sec. II-A: images of uneven size
// transformed together with masks and boxes; Sec. II-B Dih4; Table I
// Brightness).
//
// Work item = (image, output tile of TL lines x TS span positions).  The
// separable resize needs two source rows per output line along the "line"
// axis (output rows, or output columns when the Dih4 element swaps axes) and a
// contiguous span of source columns along the other.  A pass stages the 2 TL
// source row segments of its lines (only the rows the taps touch, so
// downscaled images skip rows in HBM) and TL nearest mask row segments into
// LDS with global_load_lds_dwordx4, then every output pixel reads its 4 taps
// from LDS, applies the brightness/contrast LUT per tap, blends with Q10
// weights, rounds once and looks the result up in the normalisation LUT.
// A tile whose staged footprint does not fit the staging buffer runs as two
// passes over the halves of its span positions; a half that still does not
// fit reads its taps straight from global memory.
//
// The best tile-pass form is a persistent launch in which four worker waves of
// a workgroup stream and blend pass k while a fifth wave claims items and
// plans pass k+1 into a second table set.  Other launch forms are kept as
// autotuner candidates: the same pipeline with the planning done by a rotating
// worker wave, one pass at a time with chunked claims, a flat grid, and a
// streaming form.  This file also holds the launcher and the variant table of
// every batched form, including the row bands of k_rows.hip and the wave
// gathers of k_gather.hip (the default).
//
// The streaming form is a persistent launch in which every workgroup runs a
// three-stage software pipeline over its passes: in one iteration it builds
// the tables of pass k+2, issues the LDS-DMA of pass k+1 into one staging
// buffer and blends pass k from the other.  The two staging buffers are
// distinct LDS variables, so the compiler can tell the DMA in flight from the
// LDS reads of the blend and does not wait for it there.
//
// Scheduling: images are dealt to 8 queues (image i -> queue i mod 8);
// workgroup b starts on queue b mod 8, which is the XCD the hardware dispatches
// it to, so the tiles of one image share that XCD's L2.  A workgroup pops
// tiles with an atomic counter and, when its queue is empty, moves on to the
// next queue; every workgroup ends after at most 8 empty pops.  Counters are
// cleared by a one-block fill kernel enqueued just before, so the pair can be
// captured in a hipGraph.
#include "ragged_common.h"

namespace miaug {
namespace {

constexpr int kThreads = 256;

// Staging buffer of CAP 16-byte chunks plus slack: a tap's two-dword read may
// reach a few bytes past the last chunk.
constexpr int stage_bytes(int cap) { return cap * 16 + 16; }

template <int TS>
constexpr int log2_of() { return TS == 128 ? 7 : TS == 64 ? 6 : TS == 32 ? 5 : TS == 16 ? 4 : 3; }

// Work items per image: the tile grid in line x span coordinates depends on
// whether the element swaps axes, so the queue reserves the larger count.
template <int TL, int TS>
__host__ __device__ __forceinline__ int tiles_per_image(int OH, int OW) {
    const int a = ((OH + TL - 1) / TL) * ((OW + TS - 1) / TS);
    const int b = ((OW + TL - 1) / TL) * ((OH + TS - 1) / TS);
    return a > b ? a : b;
}

// Largest staged footprint (16-byte chunks) of a whole TL x TS tile whose
// source extent along the span axis is up to R / 10 times the output's
// (4.6 by default; 4.3 leaves room for a second table set in 40 KB, which is
// what a workgroup may take for two of them to share one half of the LDS).
template <int TL, int TS, int R = 46>
constexpr int full_cap() {
    return 2 * TL * ((((TS - 1) * R / 10 + 4) * 3 + 30) / 16) + TL * ((((TS - 1) * R / 10 + 4) + 30) / 16);
}

// ---------------------------------------------------------------- passes

// Asynchronous form for a whole wave: lane l < 16 loads field l of image img
// with one vector load (counted by vmcnt, so it can stay in flight across LDS
// work); info_gather() assembles the fields once the load has completed.
__device__ __forceinline__ int info_issue(const miaug_ragged_args &a, int img) {
    const int l = threadIdx.x & 63;
    const int32_t *p = nullptr;
    if (l < 2) p = a.hw + 2 * img + l;
    else if (l < 6) p = a.flags + 4 * img + (l - 2);
    else if (l < 8) p = (const int32_t *)(a.img_off + img) + (l - 6);
    else if (l < 10 && a.mask) p = (const int32_t *)(a.mask_off + img) + (l - 8);
    else if (l >= 10 && l < 12) p = (const int32_t *)(a.ab + 2 * img) + (l - 10);
    else if (l >= 12 && l < 16 && a.crop) p = a.crop + 4 * img + (l - 12);
    return p ? *p : 0;
}

__device__ __forceinline__ ImgInfo info_gather(int v) {
    ImgInfo r;
    r.H = __builtin_amdgcn_readlane(v, 0);
    r.W = __builtin_amdgcn_readlane(v, 1);
    r.f0 = __builtin_amdgcn_readlane(v, 2);
    r.f1 = __builtin_amdgcn_readlane(v, 3);
    r.f2 = __builtin_amdgcn_readlane(v, 4);
    r.f3 = __builtin_amdgcn_readlane(v, 5);
    r.io = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(v, 7) << 32) |
                     (uint32_t)__builtin_amdgcn_readlane(v, 6));
    r.mo = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(v, 9) << 32) |
                     (uint32_t)__builtin_amdgcn_readlane(v, 8));
    r.alpha = __int_as_float(__builtin_amdgcn_readlane(v, 10));
    r.beta = __int_as_float(__builtin_amdgcn_readlane(v, 11));
    r.wy = __builtin_amdgcn_readlane(v, 12);
    r.wx = __builtin_amdgcn_readlane(v, 13);
    r.wh = __builtin_amdgcn_readlane(v, 14);
    r.ww = __builtin_amdgcn_readlane(v, 15);
    return r;
}

// Geometry of one pass, identical in every thread.
struct Pass {
    int img, tile, part;  // part 0: whole tile; 1 / 2: first / second half of its span positions
    bool valid;           // false: end of the work stream
    bool empty;           // image skipped or spare item: nothing to do
    bool staged;          // footprint fits the staging buffer
    bool swap;
    int H, W;
    D4Map m;
    int l0, s0, nl, ns;  // first output line / span position, counts
    int OL, OS, Ll, Ls, kl, ks;
    int sxlo, nsx, mxlo, nmx;          // source column spans of the bilinear / nearest taps
    int nchi, nchm, img_items, total;  // staging layout in 16-byte chunks
    int64_t io, mo;
    float alpha, beta;
};

template <int TL, int TS, int CAP>
__device__ __forceinline__ Pass make_pass(const miaug_ragged_args &a, const ImgInfo &in, int img, int tile,
                                          int part) {
    Pass p;
    p.img = img;
    p.tile = tile;
    p.part = part;
    p.valid = true;
    p.H = in.H;
    p.W = in.W;
    p.io = in.io;
    p.mo = in.mo;
    p.alpha = in.alpha;
    p.beta = in.beta;
    p.empty = p.H < 1 || p.W < 1 || p.H >= kMaxSide || p.W >= kMaxSide || (int64_t)p.H * p.W * 3 >= ((int64_t)1 << 31);
    p.m = make_d4(p.empty ? 1 : p.H, p.empty ? 1 : p.W, in.f0, in.f1, in.f2, in.f3);
    if (in.wh != 0 && !p.empty) {
        // crop window (wy, wx, wh, ww) of the Dih4 image: output (r, c) of the
        // window is (r + wy, c + wx) of that image; a window that is not inside
        // it skips the image
        if (in.wy < 0 || in.wx < 0 || in.wh < 1 || in.ww < 1 || in.wh > p.m.oh - in.wy || in.ww > p.m.ow - in.wx) {
            p.empty = true;
        } else {
            p.m.cy += p.m.ay * in.wy + p.m.by * in.wx;
            p.m.cx += p.m.ax * in.wy + p.m.bx * in.wx;
            p.m.oh = in.wh;
            p.m.ow = in.ww;
        }
    }
    p.swap = p.m.swaps();
    p.OL = p.swap ? a.out_w : a.out_h;
    p.OS = p.swap ? a.out_h : a.out_w;
    const int n_sb = (p.OS + TS - 1) / TS;
    int sb;
    p.l0 = udiv_small(tile, n_sb, sb) * TL;
    p.s0 = sb * TS;
    if (p.l0 >= p.OL) p.empty = true;  // spare item of the larger tile grid
    p.nl = min(TL, p.OL - p.l0);
    int ns = min(TS, p.OS - p.s0);
    if (part == 1) {
        ns = min(ns, TS / 2);
    } else if (part == 2) {
        p.s0 += TS / 2;
        ns -= TS / 2;
    }
    p.ns = ns;
    if (p.nl < 1 || ns < 1) p.empty = true;
    p.Ll = p.swap ? p.m.ow : p.m.oh;
    p.Ls = p.swap ? p.m.oh : p.m.ow;
    p.kl = p.swap ? p.m.by : p.m.ay;
    p.ks = p.swap ? p.m.ax : p.m.bx;
    p.staged = false;
    p.sxlo = p.nsx = p.mxlo = p.nmx = p.nchi = p.nchm = p.img_items = p.total = 0;
    if (p.empty) return p;
    const int32_t qf = resize_q(p.s0, p.Ls, p.OS), ql = resize_q(p.s0 + ns - 1, p.Ls, p.OS);
    const int dlo = clampi(qf >> kFBits, p.Ls), dhi = clampi((ql >> kFBits) + 1, p.Ls);
    const int xa = p.ks * dlo + p.m.cx, xb = p.ks * dhi + p.m.cx;
    p.sxlo = min(xa, xb);
    p.nsx = abs(xb - xa) + 1;
    const int nlo = clampi((qf + kFOne / 2) >> kFBits, p.Ls), nhi = clampi((ql + kFOne / 2) >> kFBits, p.Ls);
    const int mxa = p.ks * nlo + p.m.cx, mxb = p.ks * nhi + p.m.cx;
    p.mxlo = min(mxa, mxb);
    p.nmx = abs(mxb - mxa) + 1;
    p.nchi = (3 * p.nsx + 30) >> 4;  // most chunks a row segment of 3 nsx bytes can touch
    p.nchm = a.mask ? (p.nmx + 30) >> 4 : 0;
    p.img_items = 2 * p.nl * p.nchi;
    p.total = p.img_items + p.nl * p.nchm;
    p.staged = p.total <= CAP;
    return p;
}

// Pass `part` of tile (img, tile); part 0 becomes part 1 when the whole tile's
// footprint does not fit the staging buffer (one call site of make_pass).
template <int TL, int TS, int CAP>
__device__ __forceinline__ Pass plan_pass(const miaug_ragged_args &a, const ImgInfo &in, int img, int tile,
                                          int part) {
    Pass p;
    for (;;) {
        p = make_pass<TL, TS, CAP>(a, in, img, tile, part);
        if (part != 0 || p.empty || p.staged || p.ns <= TS / 2) break;
        part = 1;
    }
    return p;
}

// What later stages of a pass read back from LDS (one int each).
enum { M_VALID, M_EMPTY, M_STAGED, M_IMG, M_TILE, M_PART, M_SWAP, M_J0, M_I0, M_NL, M_NS, M_NCHI, M_NCHM,
       M_ITEMS, M_TOTAL, M_W, M_LL, M_LS, M_KL, M_KS, M_CX, M_CY, M_OL, M_OS, M_L0, M_S0, M_IOFF,
       M_MOFF = M_IOFF + 2, M_ALPHA = M_MOFF + 2, M_BETA, M_N = (M_BETA + 1 + 3) / 4 * 4 };

struct Meta {
    int valid, empty, staged, img, tile, part, swap, j0, i0, nl, ns, nchi, nchm, items, total;
    int W, Ll, Ls, kl, ks, cx, cy, OL, OS, l0, s0;  // geometry for the direct path
    int64_t img_off, mask_off;  // byte offsets of the image and mask in the packed batch
    float alpha, beta;          // brightness/contrast parameters
};

__device__ __forceinline__ Meta read_meta(const int *s) {
    Meta m;
    m.valid = __builtin_amdgcn_readfirstlane(s[M_VALID]);
    m.empty = __builtin_amdgcn_readfirstlane(s[M_EMPTY]);
    m.staged = __builtin_amdgcn_readfirstlane(s[M_STAGED]);
    m.img = __builtin_amdgcn_readfirstlane(s[M_IMG]);
    m.tile = __builtin_amdgcn_readfirstlane(s[M_TILE]);
    m.part = __builtin_amdgcn_readfirstlane(s[M_PART]);
    m.swap = __builtin_amdgcn_readfirstlane(s[M_SWAP]);
    m.j0 = __builtin_amdgcn_readfirstlane(s[M_J0]);
    m.i0 = __builtin_amdgcn_readfirstlane(s[M_I0]);
    m.nl = __builtin_amdgcn_readfirstlane(s[M_NL]);
    m.ns = __builtin_amdgcn_readfirstlane(s[M_NS]);
    m.nchi = __builtin_amdgcn_readfirstlane(s[M_NCHI]);
    m.nchm = __builtin_amdgcn_readfirstlane(s[M_NCHM]);
    m.items = __builtin_amdgcn_readfirstlane(s[M_ITEMS]);
    m.total = __builtin_amdgcn_readfirstlane(s[M_TOTAL]);
    m.W = __builtin_amdgcn_readfirstlane(s[M_W]);
    m.Ll = __builtin_amdgcn_readfirstlane(s[M_LL]);
    m.Ls = __builtin_amdgcn_readfirstlane(s[M_LS]);
    m.kl = __builtin_amdgcn_readfirstlane(s[M_KL]);
    m.ks = __builtin_amdgcn_readfirstlane(s[M_KS]);
    m.cx = __builtin_amdgcn_readfirstlane(s[M_CX]);
    m.cy = __builtin_amdgcn_readfirstlane(s[M_CY]);
    m.OL = __builtin_amdgcn_readfirstlane(s[M_OL]);
    m.OS = __builtin_amdgcn_readfirstlane(s[M_OS]);
    m.l0 = __builtin_amdgcn_readfirstlane(s[M_L0]);
    m.s0 = __builtin_amdgcn_readfirstlane(s[M_S0]);
    m.img_off = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(s[M_IOFF + 1]) << 32) |
                          (uint32_t)__builtin_amdgcn_readfirstlane(s[M_IOFF]));
    m.mask_off = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane(s[M_MOFF + 1]) << 32) |
                           (uint32_t)__builtin_amdgcn_readfirstlane(s[M_MOFF]));
    m.alpha = __int_as_float(__builtin_amdgcn_readfirstlane(s[M_ALPHA]));
    m.beta = __int_as_float(__builtin_amdgcn_readfirstlane(s[M_BETA]));
    return m;
}


template <int TL, int TS>
__device__ __forceinline__ void table_entry(const miaug_ragged_args &a, const Pass &p, const D4Map &m, bool isl,
                                            int idx, int64_t io, int64_t mo, int4 *ln, int4 *cl, int2 *rw);

// Tables of a pass, built by wave 0 alone (the other waves only read them
// after a barrier):
//   ln[l]  = LDS byte offsets of the two tap rows of line l, its Q10 weight and
//            the LDS byte offset of its nearest mask row;
//   cl[s]  = byte offsets of the two taps of span position s inside a staged
//            row, its weight, and the nearest mask tap's offset;
//   rw[r]  = per staged row r (2 per line, then 1 mask row per line): offset of
//            its first 16-byte chunk from the image's (mask's) aligned base,
//            and its chunk count;
//   meta   = what the DMA and blend stages need.
// Entry l < TL is line l, entry TL + s span position s (lane e takes entries
// e, e + 64, ...), with one shared evaluation of the resize position.
template <int TL, int TS>
__device__ __forceinline__ void pass_tables(const miaug_ragged_args &a, const Pass &p, int4 *ln, int4 *cl, int2 *rw,
                                            int *meta) {

    const int lane = threadIdx.x & 63;
    const bool live = p.valid && !p.empty;
    const int64_t io = live ? p.io : 0;
    const int64_t mo = live && a.mask ? p.mo : 0;
    if (lane == 0) {
        meta[M_VALID] = p.valid;
        meta[M_EMPTY] = p.empty;
        meta[M_STAGED] = p.staged;
        meta[M_IMG] = p.img;
        meta[M_TILE] = p.tile;
        meta[M_PART] = p.part;
        meta[M_SWAP] = p.swap;
        meta[M_J0] = p.swap ? p.s0 : p.l0;
        meta[M_I0] = p.swap ? p.l0 : p.s0;
        meta[M_NL] = p.nl;
        meta[M_NS] = p.ns;
        meta[M_NCHI] = p.nchi;
        meta[M_NCHM] = p.nchm;
        meta[M_ITEMS] = p.img_items;
        meta[M_TOTAL] = p.total;
        meta[M_W] = p.W;
        meta[M_LL] = p.Ll;
        meta[M_LS] = p.Ls;
        meta[M_KL] = p.kl;
        meta[M_KS] = p.ks;
        meta[M_CX] = p.m.cx;
        meta[M_CY] = p.m.cy;
        meta[M_OL] = p.OL;
        meta[M_OS] = p.OS;
        meta[M_L0] = p.l0;
        meta[M_S0] = p.s0;
        meta[M_IOFF] = (int)(uint32_t)io;
        meta[M_IOFF + 1] = (int)(uint32_t)((uint64_t)io >> 32);
        meta[M_MOFF] = (int)(uint32_t)mo;
        meta[M_MOFF + 1] = (int)(uint32_t)((uint64_t)mo >> 32);
        meta[M_ALPHA] = __float_as_int(p.alpha);
        meta[M_BETA] = __float_as_int(p.beta);
    }
    if (!live || !p.staged) return;
    const D4Map &m = p.m;
    for (int e = lane; e < TL + TS; e += 64) {
        const bool isl = e < TL;  // entries 0..TL-1: lines; TL..TL+TS-1: span positions
        const int idx = isl ? e : e - TL;
        if (idx >= (isl ? p.nl : p.ns)) continue;
        table_entry<TL, TS>(a, p, m, isl, idx, io, mo, ln, cl, rw);
    }
}

template <int TL, int TS>
__device__ __forceinline__ void table_entry(const miaug_ragged_args &a, const Pass &p, const D4Map &m, bool isl,
                                            int idx, int64_t io, int64_t mo, int4 *ln, int4 *cl, int2 *rw) {
    const int Lsrc = isl ? p.Ll : p.Ls;
    const int q = resize_q(isl ? p.l0 + idx : p.s0 + idx, Lsrc, isl ? p.OL : p.OS);
    const int d0 = clampi(q >> kFBits, Lsrc), d1 = clampi((q >> kFBits) + 1, Lsrc);
    const int dn = clampi((q + kFOne / 2) >> kFBits, Lsrc);
    if (isl) {
        // rows are < 2^31 bytes into the image: 32-bit offsets from its aligned base
        const int ph = (int)((uintptr_t)(a.img + io) & 15);
        const int r0 = ph + ((p.kl * d0 + m.cy) * p.W + p.sxlo) * 3;
        const int r1 = ph + ((p.kl * d1 + m.cy) * p.W + p.sxlo) * 3;
        rw[2 * idx] = make_int2(r0 & ~15, ((r0 & 15) + 3 * p.nsx + 15) >> 4);
        rw[2 * idx + 1] = make_int2(r1 & ~15, ((r1 & 15) + 3 * p.nsx + 15) >> 4);
        int mof = 0;
        if (a.mask) {
            const int mph = (int)((uintptr_t)(a.mask + mo) & 15);
            const int rm = mph + (p.kl * dn + m.cy) * p.W + p.mxlo;
            rw[2 * p.nl + idx] = make_int2(rm & ~15, ((rm & 15) + p.nmx + 15) >> 4);
            mof = 16 * (p.img_items + idx * p.nchm) + (rm & 15);
        }
        ln[idx] = make_int4(16 * (2 * idx) * p.nchi + (r0 & 15), 16 * (2 * idx + 1) * p.nchi + (r1 & 15),
                            q & (kFOne - 1), mof);
    } else {
        cl[idx] = make_int4(3 * (p.ks * d0 + m.cx - p.sxlo), 3 * (p.ks * d1 + m.cx - p.sxlo), q & (kFOne - 1),
                            p.ks * dn + m.cx - p.mxlo);
    }
}


// Issues the LDS-DMA of a staged pass: chunk `it` of the pass (image rows
// first, 2 nl slots of nchi chunks, then nl mask slots of nchm chunks) lands
// at stage byte 16 it.  Image and mask chunks are issued in two loops, each
// through a buffer resource of its own base (32-bit offsets); the 64 lanes of
// a wave take 64 consecutive chunks, which is the DMA's lane layout (LDS base
// in M0 + 16 * lane); threads 0..NT-1 take part.  Row-table reads go in
// groups of four ahead of their DMAs, so their LDS latencies overlap (a wave
// that has run out of chunks reads clamped entries and issues nothing).
// Completion is counted by vmcnt.
template <int NT, int CAP, int N>
__device__ __forceinline__ void pass_dma(const miaug_ragged_args &a, const Meta &mt, const int2 *rw,
                                         uint8_t (&st)[N]) {
    constexpr int kIt = (CAP + NT - 1) / NT;
    constexpr int kB = 4;  // row-table reads issued together
    if (!mt.valid || mt.empty || !mt.staged) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wbase = __builtin_amdgcn_readfirstlane(tid - lane);
    const int items = mt.items, nmask = mt.total - mt.items, nl = mt.nl;
    // chunks [0, n) of slots of d chunks each, rows rw[r0 + slot] (slot clamped
    // to smax), landing at stage byte 16 (sbase + chunk)
    auto issue = [&](const __amdgpu_buffer_rsrc_t rs, int n, int d, int r0, int smax, int sbase) {
        const uint32_t M = div_magic(d);
#pragma unroll
        for (int u0 = 0; u0 < kIt; u0 += kB) {
            if (wbase + u0 * NT >= n) break;  // uniform per wave
            int2 r[kB];
            int ch[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const int it = tid + (u0 + u) * NT;
                const int slot = div_by_m(it, d, M);
                ch[u] = it - slot * d;
                r[u] = rw[r0 + min(slot, smax)];
            }
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                if (u0 + u >= kIt || wbase + (u0 + u) * NT >= n) break;
                const int it = tid + (u0 + u) * NT;
                if (it < n && ch[u] < r[u].y)
                    dma16(rs, st + 16 * (sbase + wbase + (u0 + u) * NT), (uint32_t)(r[u].x + 16 * ch[u]));
            }
        }
    };
    issue(buffer_rsrc((void *)align16(a.img + mt.img_off), 0x7fffffffu), items, mt.nchi, 0, 2 * nl - 1, 0);
    if (nmask > 0)
        issue(buffer_rsrc((void *)align16(a.mask + mt.mask_off), 0x7fffffffu), nmask, mt.nchm, 2 * nl, nl - 1,
              items);
}

// Register staging of a pass: the same chunks as pass_dma, loaded into VGPRs
// (16 bytes each; chunk j = tid + u NT of the pass, image chunks first, then
// mask chunks), so that the loads can be in flight while the previous pass is
// blended out of the single LDS stage; pass_stage then writes them to stage
// byte 16 j.  Bit u of the returned mask marks the chunks loaded.
template <int NT, int CAP>
constexpr int chunks_per_lane() {
    return (CAP + NT - 1) / NT;
}

template <int NT, int CAP>
__device__ __forceinline__ uint32_t pass_load(const miaug_ragged_args &a, const Meta &mt, const int2 *rw,
                                              u32x4 (&R)[chunks_per_lane<NT, CAP>()]) {
    constexpr int kIt = chunks_per_lane<NT, CAP>();
    constexpr int kB = 4;  // row-table reads issued together
    static_assert(kIt <= 32, "one bit per chunk");
    uint32_t okm = 0;
    if (!mt.valid || mt.empty || !mt.staged) return okm;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wbase = __builtin_amdgcn_readfirstlane(tid - lane);
    const int items = mt.items, total = mt.total, nl = mt.nl;
    const int di = mt.nchi, dm = mt.nchm;
    const uint32_t Mi = div_magic(di), Mm = div_magic(dm);
    const __amdgpu_buffer_rsrc_t ri = buffer_rsrc((void *)align16(a.img + mt.img_off), 0x7fffffffu);
    const __amdgpu_buffer_rsrc_t rm =
        buffer_rsrc((void *)(a.mask ? align16(a.mask + mt.mask_off) : a.img), 0x7fffffffu);
#pragma unroll
    for (int u0 = 0; u0 < kIt; u0 += kB) {
        if (wbase + u0 * NT >= total) break;  // uniform per wave
        int2 r[kB];
        int ch[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int j = tid + (u0 + u) * NT;
            const bool im = j < items;
            const int jj = im ? j : j - items;
            const int d = im ? di : dm;
            const int slot = div_by_m(jj, d, im ? Mi : Mm);
            ch[u] = jj - slot * d;
            r[u] = rw[im ? min(slot, 2 * nl - 1) : 2 * nl + min(slot, nl - 1)];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            if (u0 + u >= kIt || wbase + (u0 + u) * NT >= total) break;
            const int j = tid + (u0 + u) * NT;
            if (j < total && ch[u] < r[u].y) {
                const uint32_t off = (uint32_t)(r[u].x + 16 * ch[u]);
                if (j < items) R[u0 + u] = __builtin_amdgcn_raw_buffer_load_b128(ri, off, 0, 0);
                else R[u0 + u] = __builtin_amdgcn_raw_buffer_load_b128(rm, off, 0, 0);
                okm |= 1u << (u0 + u);
            }
        }
    }
    return okm;
}

template <int NT, int CAP, int N>
__device__ __forceinline__ void pass_stage(const u32x4 (&R)[chunks_per_lane<NT, CAP>()], uint32_t okm,
                                           uint8_t (&st)[N]) {
    constexpr int kIt = chunks_per_lane<NT, CAP>();
#pragma unroll
    for (int u = 0; u < kIt; ++u)
        if (okm & (1u << u)) *(u32x4 *)(st + 16 * (threadIdx.x + u * NT)) = R[u];
}

// One lane's blended pixels of a pass, held in registers until stored.
template <int K>
struct BlendOut {
    float f[K][3];
    uint32_t m[K];
    int off[K];  // element offset within the image's output plane
    bool ok[K];
};

template <int TL, int TS, int NT>
constexpr int pix_per_lane() {
    return (TL * TS + NT - 1) / NT;
}

// Blend and normalise a staged pass into registers (store_out writes them;
// blend_px does both).  Each tap byte is one ds_read_u8
// (the channel is the instruction's immediate offset) whose result indexes
// the brightness/contrast LUT directly.  The separable blend uses full-rate
// 24-bit multiplies (weights <= 1024, partial sums < 2^18, total < 2^28).
// Stores take per-channel scalar offsets.  A lane's pixels go in groups of up
// to four whose tap, LUT and normalisation reads are issued together, so a
// wave waits for three LDS round trips per group rather than per pixel.
// Lanes take output row segments when the element keeps the axes (consecutive
// lanes read consecutive columns of the same two staged rows), and 8 x 8
// blocks when it swaps them (consecutive lanes would otherwise read the same
// column of many staged rows, which share few LDS banks).
template <int TL, int TS, int NT, bool SWAP, int N>
__device__ __forceinline__ void blend_keep(const miaug_ragged_args &a, const Meta &mt, const uint8_t (&st)[N],
                                           const int4 *ln, const int4 *cl, const uint8_t *bc,
                                           const float (&nlut)[3][256], BlendOut<pix_per_lane<TL, TS, NT>()> &o) {
    constexpr int kPix = pix_per_lane<TL, TS, NT>();
    constexpr int G = kPix < 4 ? kPix : 4;  // pixels per lane whose LDS reads are issued together
    static_assert(NT % 64 == 0 && (TL * TS) % NT == 0 && kPix % G == 0, "whole waves, whole tiles, whole groups");
    const int tid = threadIdx.x;
    const int OW = a.out_w;
    const int wlog = mt.part ? log2_of<TS>() - 1 : log2_of<TS>();
    const int npx = TL << wlog;  // a multiple of NT
    const int base = mt.j0 * OW + mt.i0;
#pragma unroll
    for (int k0 = 0; k0 < kPix; k0 += G) {
        if (k0 * NT >= npx) {
#pragma unroll
            for (int g = 0; g < G; ++g) o.ok[k0 + g] = false;
            continue;
        }
        uint32_t wl[G], ws[G];
        uint32_t v[G][12];
        int4 Lg[G], Cg[G];
        // table entries of the whole group
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int p = tid + (k0 + g) * NT;
            int l, si;  // line and span position within the pass
            if (!SWAP) {
                l = p >> wlog;
                si = p & ((1 << wlog) - 1);
            } else {
                const int lane = p & 63, blk = p >> 6;  // 8 x 8 blocks
                l = 8 * (blk % (TL / 8)) + (lane & 7);
                si = 8 * (blk / (TL / 8)) + (lane >> 3);
            }
            o.ok[k0 + g] = l < mt.nl && si < mt.ns;
            if (!o.ok[k0 + g]) l = si = 0;  // read table entries that exist; nothing is stored
            Lg[g] = ln[l];
            Cg[g] = cl[si];
            o.off[k0 + g] = base + (SWAP ? umad24(si, OW, l) : umad24(l, OW, si));
        }
        // taps (and the mask byte) of the whole group
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int4 L = Lg[g], C = Cg[g];
            ws[g] = C.z;
            wl[g] = L.z;
            const int o00 = L.x + C.x, o01 = L.x + C.y, o10 = L.y + C.x, o11 = L.y + C.y;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                v[g][4 * c] = st[o00 + c];
                v[g][4 * c + 1] = st[o01 + c];
                v[g][4 * c + 2] = st[o10 + c];
                v[g][4 * c + 3] = st[o11 + c];
            }
            o.m[k0 + g] = st[L.w + C.w];  // inside the stage even without a mask (offsets 0 and < nmx then)
        }
        // brightness / contrast of every tap
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
            for (int e = 0; e < 12; ++e) v[g][e] = bc[v[g][e]];
        // separable blend and normalisation
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const uint32_t ws1 = ws[g], ws0 = kFOne - ws1, wl1 = wl[g], wl0 = kFOne - wl1;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const uint32_t t0 = umad24(v[g][4 * c + 1], ws1, __umul24(v[g][4 * c], ws0));
                const uint32_t t1 = umad24(v[g][4 * c + 3], ws1, __umul24(v[g][4 * c + 2], ws0));
                o.f[k0 + g][c] = nlut[c][rhe20((int)umad24(t1, wl1, __umul24(t0, wl0)))];
            }
        }
    }
}

template <int K>
__device__ __forceinline__ void store_out(const miaug_ragged_args &a, int img, const BlendOut<K> &o) {
    const int plane = a.out_h * a.out_w;  // outputs are at most 4096 x 4096
    const bool has_mask = a.mask != nullptr;
    const __amdgpu_buffer_rsrc_t ro = buffer_rsrc(a.out + (size_t)img * 3 * plane, (uint32_t)(12 * plane));
    const __amdgpu_buffer_rsrc_t rm =
        buffer_rsrc(has_mask ? a.out_mask + (size_t)img * plane : a.out_mask, (uint32_t)plane);
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (!o.ok[k]) continue;
#pragma unroll
        for (int c = 0; c < 3; ++c)  // the b32 store takes the bit pattern: pass the float's bits
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(o.f[k][c]), ro, 4 * o.off[k], 4 * c * plane, 0);
        if (has_mask) __builtin_amdgcn_raw_buffer_store_b8(o.m[k], rm, o.off[k], 0, 0);
    }
}

template <int TL, int TS, int NT, bool SWAP, int N>
__device__ __forceinline__ void blend_px(const miaug_ragged_args &a, const Meta &mt, const uint8_t (&st)[N],
                                         const int4 *ln, const int4 *cl, const uint8_t *bc,
                                         const float (&nlut)[3][256]) {
    BlendOut<pix_per_lane<TL, TS, NT>()> o;
    blend_keep<TL, TS, NT, SWAP>(a, mt, st, ln, cl, bc, nlut, o);
    store_out(a, mt.img, o);
}

template <int TL, int TS, int NT, int N>
__device__ __forceinline__ void pass_blend(const miaug_ragged_args &a, const Meta &mt, const uint8_t (&st)[N],
                                           const int4 *ln, const int4 *cl, const uint8_t *bc,
                                           const float (&nlut)[3][256]) {
    if (mt.swap) blend_px<TL, TS, NT, true>(a, mt, st, ln, cl, bc, nlut);
    else blend_px<TL, TS, NT, false>(a, mt, st, ln, cl, bc, nlut);
}

// A pass whose footprint does not fit the staging buffer (the source is more
// than about 4.6 / 9 times the output along the span axis for a whole / half
// tile): the same arithmetic on direct global loads.
template <int NT>
__device__ __forceinline__ void pass_direct(const miaug_ragged_args &a, const Meta &p, const uint8_t *bc,
                                            const float (&nlut)[3][256]) {
    const int tid = threadIdx.x;
    const size_t plane = (size_t)a.out_h * a.out_w;
    const uint8_t *ib = a.img + p.img_off;
    const uint8_t *mb = a.mask ? a.mask + p.mask_off : nullptr;
    for (int e = tid; e < p.nl * p.ns; e += NT) {
        const int l = e / p.ns, si = e - l * p.ns;
        const int jj = p.swap ? p.s0 + si : p.l0 + l, ii = p.swap ? p.l0 + l : p.s0 + si;
        const int32_t ql = resize_q(p.l0 + l, p.Ll, p.OL), qs = resize_q(p.s0 + si, p.Ls, p.OS);
        const int wl1 = ql & (kFOne - 1), ws1 = qs & (kFOne - 1);
        const int x0 = p.ks * clampi(qs >> kFBits, p.Ls) + p.cx, x1 = p.ks * clampi((qs >> kFBits) + 1, p.Ls) + p.cx;
        const int y0 = p.kl * clampi(ql >> kFBits, p.Ll) + p.cy, y1 = p.kl * clampi((ql >> kFBits) + 1, p.Ll) + p.cy;
        const uint8_t *r0 = ib + (size_t)y0 * p.W * 3, *r1 = ib + (size_t)y1 * p.W * 3;
        float *o = a.out + (size_t)p.img * 3 * plane + (size_t)jj * a.out_w + ii;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int p00 = bc[r0[3 * x0 + c]], p01 = bc[r0[3 * x1 + c]];
            const int p10 = bc[r1[3 * x0 + c]], p11 = bc[r1[3 * x1 + c]];
            const int t0 = (p00 << kFBits) + ws1 * (p01 - p00);
            const int t1 = (p10 << kFBits) + ws1 * (p11 - p10);
            o[c * plane] = nlut[c][rhe20((t0 << kFBits) + wl1 * (t1 - t0))];
        }
        if (mb) {
            const int mx = p.ks * clampi((qs + kFOne / 2) >> kFBits, p.Ls) + p.cx;
            const int my = p.kl * clampi((ql + kFOne / 2) >> kFBits, p.Ll) + p.cy;
            a.out_mask[(size_t)p.img * plane + (size_t)jj * a.out_w + ii] = mb[(size_t)my * p.W + mx];
        }
    }
}

// One work item, its passes one after the other (single staging buffer).
// One wave plans the pass and builds its tables; after a barrier every wave
// reads the plan back.
template <int TL, int TS, int CAP, int N>
__device__ __forceinline__ void run_item(const miaug_ragged_args &a, int item, int tiles, uint8_t (&st)[N], int4 *ln,
                                         int4 *cl, int2 *rw, int *meta, uint8_t *bc, int &bc_img,
                                         const float (&nlut)[3][256], int &planner) {
    int tile;
    const int img = udiv_small(item, tiles, tile);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int part = 0;
    for (;;) {
        if (wave == (planner++ & 3)) {  // the planning wave rotates, so no SIMD gets all of it
            const Pass p = plan_pass<TL, TS, CAP>(a, info_scalar(a, img), img, tile, part);
            pass_tables<TL, TS>(a, p, ln, cl, rw, meta);
        }
        __syncthreads();
        const Meta mt = read_meta(meta);
        if (!mt.empty) {
            if (bc_img != mt.img) {
                build_bc_lut(mt.alpha, mt.beta, bc);
                bc_img = mt.img;
            }
            if (mt.tile == 0 && mt.part <= 1 && a.boxes) ragged_boxes<kThreads>(a, mt.img);
        }
        pass_dma<kThreads, CAP>(a, mt, rw, st);
        __builtin_amdgcn_s_waitcnt(0);  // LDS-DMA writes are counted by vmcnt
        __syncthreads();
        if (!mt.empty) {
            if (mt.staged) pass_blend<TL, TS, kThreads>(a, mt, st, ln, cl, bc, nlut);
            else pass_direct<kThreads>(a, mt, bc, nlut);
        }
        __syncthreads();  // tables and stage are rewritten next
        if (mt.part != 1) break;
        part = 2;
    }
}


// Persistent form: chunks of K tiles, one pass at a time.
template <int TL, int TS, int CAP, int K>
__global__ __launch_bounds__(kThreads) void k_ragged_persistent(miaug_ragged_args a, int *__restrict__ counters) {
    __shared__ __align__(16) uint8_t st[stage_bytes(CAP)];
    __shared__ int4 ln[TL];
    __shared__ int4 cl[TS];
    __shared__ int2 rw[3 * TL];
    __shared__ __align__(16) int meta[M_N];
    __shared__ float nlut[3][256];
    __shared__ uint8_t bc[256];
    __shared__ int3 chunk_s;
    const int tiles = tiles_per_image<TL, TS>(a.out_h, a.out_w);
    Claimer<K> C{tiles, (int)(blockIdx.x % kQueues), 0, 0};  // meaningful in thread 0
    if (threadIdx.x == 0) {
        C.issue(counters);
        chunk_s = C.resolve(a, counters);
        C.issue(counters);  // next chunk, in flight
    }
    build_norm_lut(a, nlut);
    int bc_img = -1, planner = 0;
    __syncthreads();
    for (;;) {
        const int cq = __builtin_amdgcn_readfirstlane(chunk_s.x);
        const int cbase = __builtin_amdgcn_readfirstlane(chunk_s.y);
        const int cn = __builtin_amdgcn_readfirstlane(chunk_s.z);
        if (cn == 0) break;
        for (int t = 0; t < cn; ++t) {
            const int u = cbase + t;
            int ut;
            const int img = udiv_small(u, tiles, ut) * kQueues + cq;
            run_item<TL, TS, CAP>(a, img * tiles + ut, tiles, st, ln, cl, rw, meta, bc, bc_img, nlut, planner);
        }
        if (threadIdx.x == 0) {  // run_item ended with a barrier: chunk_s is free
            chunk_s = C.resolve(a, counters);
            C.issue(counters);
        }
        __syncthreads();
    }
}


// Plans pass `part` of work item `item` (-1: end of the stream) into one set
// of tables (one wave).
template <int TL, int TS, int CAP>
__device__ __forceinline__ void plan_item(const miaug_ragged_args &a, int item, int part, int tiles, int4 *ln,
                                          int4 *cl, int2 *rw, int *meta) {
    if (item < 0) {
        if ((threadIdx.x & 63) == 0) meta[M_VALID] = 0;
        return;
    }
    int tile;
    const int img = udiv_small(item, tiles, tile);
    const Pass p = plan_pass<TL, TS, CAP>(a, info_scalar(a, img), img, tile, part);
    pass_tables<TL, TS>(a, p, ln, cl, rw, meta);
}

// Persistent form in which the next pass is planned while the current one's
// LDS-DMA is in flight: the tables (and the plan) are double-buffered, the
// staging buffer is not.  Per pass: every wave issues its share of the DMA,
// one wave (rotating) then plans the next pass into the other table set, all
// wait for their DMA, a barrier, blend, a barrier.  Thread 0 claims items one
// ahead: `nx` holds the next unplanned item and is refilled after the barrier
// that follows the planner's read of it.
template <int TL, int TS, int CAP>
__global__ __launch_bounds__(kThreads) void k_ragged_pipe(miaug_ragged_args a, int *__restrict__ counters) {
    __shared__ __align__(16) uint8_t st[stage_bytes(CAP)];
    __shared__ int4 ln[2][TL];
    __shared__ int4 cl[2][TS];
    __shared__ int2 rw[2][3 * TL];
    __shared__ __align__(16) int meta[2][M_N];
    __shared__ float nlut[3][256];
    __shared__ uint8_t bc[256];
    __shared__ int nx;
    const int tiles = tiles_per_image<TL, TS>(a.out_h, a.out_w);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    Claimer<1> C{tiles, (int)(blockIdx.x % kQueues), 0, 0};  // meaningful in thread 0
    int first = -1;
    if (threadIdx.x == 0) {
        C.issue(counters);
        first = claim_item(C, a, counters);
        nx = claim_item(C, a, counters);
    }
    first = __builtin_amdgcn_readfirstlane(first);  // lane 0 of wave 0
    if (wave == 0) plan_item<TL, TS, CAP>(a, first, 0, tiles, ln[0], cl[0], rw[0], meta[0]);
    build_norm_lut(a, nlut);
    int bc_img = -1, planner = 1, b = 0;
    __syncthreads();
    for (;;) {
        const Meta mt = read_meta(meta[b]);
        if (!mt.valid) break;
        if (!mt.empty) {
            if (bc_img != mt.img) {
                build_bc_lut(mt.alpha, mt.beta, bc);
                bc_img = mt.img;
            }
            if (mt.tile == 0 && mt.part <= 1 && a.boxes) ragged_boxes<kThreads>(a, mt.img);
        }
        pass_dma<kThreads, CAP>(a, mt, rw[b], st);
        const bool consume = mt.part != 1;  // the next pass starts a new item
        if (wave == (planner++ & 3)) {
            const int item = consume ? __builtin_amdgcn_readfirstlane(nx) : mt.img * tiles + mt.tile;
            plan_item<TL, TS, CAP>(a, item, consume ? 0 : 2, tiles, ln[b ^ 1], cl[b ^ 1], rw[b ^ 1], meta[b ^ 1]);
        }
        __builtin_amdgcn_s_waitcnt(0);  // LDS-DMA writes are counted by vmcnt
        __syncthreads();
        if (threadIdx.x == 0 && consume) nx = claim_item(C, a, counters);
        if (!mt.empty) {
            if (mt.staged) pass_blend<TL, TS, kThreads>(a, mt, st, ln[b], cl[b], bc, nlut);
            else pass_direct<kThreads>(a, mt, bc, nlut);
        }
        __syncthreads();  // the stage and this table set are rewritten next
        b ^= 1;
    }
}

// The same pipeline with a fifth, dedicated planning wave: it claims items
// (one atomic ahead) and plans pass k+1 into the other table set while the
// four worker waves stream and blend pass k, so neither planning nor claiming
// sits in a worker's path.  Two barriers per pass, as above.
template <int TL, int TS, int CAP>
__global__ __launch_bounds__(kThreads + 64) __attribute__((amdgpu_waves_per_eu(5))) void k_ragged_pipe5(
    miaug_ragged_args a, int *__restrict__ counters) {
    __shared__ __align__(16) uint8_t st[stage_bytes(CAP)];
    __shared__ int4 ln[2][TL];
    __shared__ int4 cl[2][TS];
    __shared__ int2 rw[2][3 * TL];
    __shared__ __align__(16) int meta[2][M_N];
    __shared__ float nlut[3][256];
    __shared__ uint8_t bc[256];
    const int tiles = tiles_per_image<TL, TS>(a.out_h, a.out_w);
    const bool planner = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == kThreads / 64;
    build_norm_lut(a, nlut);
    int b = 0;
    if (planner) {
        __builtin_amdgcn_s_setprio(2);
        const int lane = threadIdx.x & 63;
        Claimer<1> C{tiles, (int)(blockIdx.x % kQueues), 0, 0};  // meaningful in lane 0
        int v = -1;
        if (lane == 0) {
            C.issue(counters);
            v = claim_item(C, a, counters);
        }
        plan_item<TL, TS, CAP>(a, __builtin_amdgcn_readfirstlane(v), 0, tiles, ln[0], cl[0], rw[0], meta[0]);
        __syncthreads();
        for (;;) {
            const int valid = __builtin_amdgcn_readfirstlane(meta[b][M_VALID]);
            if (!valid) break;
            const int part = __builtin_amdgcn_readfirstlane(meta[b][M_PART]);
            int item;
            if (part == 1) {
                item = __builtin_amdgcn_readfirstlane(meta[b][M_IMG]) * tiles +
                       __builtin_amdgcn_readfirstlane(meta[b][M_TILE]);
            } else {
                v = -1;
                if (lane == 0) v = claim_item(C, a, counters);
                item = __builtin_amdgcn_readfirstlane(v);
            }
            plan_item<TL, TS, CAP>(a, item, part == 1 ? 2 : 0, tiles, ln[b ^ 1], cl[b ^ 1], rw[b ^ 1], meta[b ^ 1]);
            __syncthreads();
            __syncthreads();
            b ^= 1;
        }
        return;
    }
    int bc_img = -1;
    __syncthreads();
    for (;;) {
        const Meta mt = read_meta(meta[b]);
        if (!mt.valid) break;
        if (!mt.empty) {
            if (bc_img != mt.img) {
                build_bc_lut(mt.alpha, mt.beta, bc);
                bc_img = mt.img;
            }
            if (mt.tile == 0 && mt.part <= 1 && a.boxes) ragged_boxes<kThreads>(a, mt.img);
        }
        pass_dma<kThreads, CAP>(a, mt, rw[b], st);
        __builtin_amdgcn_s_waitcnt(0);  // LDS-DMA writes are counted by vmcnt
        __syncthreads();
        if (!mt.empty) {
            if (mt.staged) pass_blend<TL, TS, kThreads>(a, mt, st, ln[b], cl[b], bc, nlut);
            else pass_direct<kThreads>(a, mt, bc, nlut);
        }
        __syncthreads();  // the stage and this table set are rewritten next
        b ^= 1;
    }
}

// Pipelined form with a double-buffered stage: the four worker waves issue the
// LDS-DMA of pass k+1 into one stage and then blend pass k out of the other,
// so every workgroup keeps loads in flight while it computes.  The planning
// wave runs two passes ahead into a third table set (pass k+2 while pass k is
// blended and pass k+1 streamed).  The two stages are separate LDS variables
// and the loop is unrolled by two, so each blend's LDS reads carry no wait on
// the other stage's DMA.  One barrier per pass; the brightness/contrast LUT is
// double-buffered by pass parity and built one pass ahead.  Both sides leave
// the loop at the first invalid pass, after the same number of barriers.
// Two stages do not fit in 40 KB with a useful footprint, so this form runs
// two workgroups per CU; it measured slower than the single-stage form at
// three (1.10 against 0.81 ms on the 2048-image batch).
template <int TL, int TS, int CAP, int N>
__device__ __forceinline__ bool pipe6_step(const miaug_ragged_args &a, int k, int4 (*ln)[TL], int4 (*cl)[TS],
                                           int2 (*rw)[3 * TL], int (*meta)[M_N], uint8_t (*bc)[256],
                                           const float (&nlut)[3][256], uint8_t (&cur)[N], uint8_t (&nxt)[N]) {
    const int t = k % 3, t1 = (k + 1) % 3;
    if (!__builtin_amdgcn_readfirstlane(meta[t][M_VALID])) return false;
    if (a.boxes && !__builtin_amdgcn_readfirstlane(meta[t][M_EMPTY]) &&
        __builtin_amdgcn_readfirstlane(meta[t][M_TILE]) == 0 && __builtin_amdgcn_readfirstlane(meta[t][M_PART]) <= 1)
        ragged_boxes<kThreads>(a, __builtin_amdgcn_readfirstlane(meta[t][M_IMG]));  // before the DMA: its loads
                                                                                   // would wait for it
    {
        const Meta mn = read_meta(meta[t1]);
        if (mn.valid && !mn.empty) build_bc_lut(mn.alpha, mn.beta, bc[(k + 1) & 1]);
        pass_dma<kThreads, CAP>(a, mn, rw[t1], nxt);
    }
    const Meta mc = read_meta(meta[t]);
    if (!mc.empty) {
        if (mc.staged) pass_blend<TL, TS, kThreads>(a, mc, cur, ln[t], cl[t], bc[k & 1], nlut);
        else pass_direct<kThreads>(a, mc, bc[k & 1], nlut);
    }
    __builtin_amdgcn_s_waitcnt(0);  // the next pass's LDS-DMA writes are counted by vmcnt
    __syncthreads();
    return true;
}

template <int TL, int TS, int CAP>
__global__ __launch_bounds__(kThreads + 64) void k_ragged_pipe6(miaug_ragged_args a, int *__restrict__ counters) {
    __shared__ __align__(16) uint8_t st0[stage_bytes(CAP)];
    __shared__ __align__(16) uint8_t st1[stage_bytes(CAP)];
    __shared__ int4 ln[3][TL];
    __shared__ int4 cl[3][TS];
    __shared__ int2 rw[3][3 * TL];
    __shared__ __align__(16) int meta[3][M_N];
    __shared__ float nlut[3][256];
    __shared__ uint8_t bc[2][256];
    const int tiles = tiles_per_image<TL, TS>(a.out_h, a.out_w);
    const bool planner = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == kThreads / 64;
    build_norm_lut(a, nlut);
    if (planner) {
        __builtin_amdgcn_s_setprio(2);
        const int lane = threadIdx.x & 63;
        Claimer<1> C{tiles, (int)(blockIdx.x % kQueues), 0, 0};  // meaningful in lane 0
        // item and part of pass k + 1 (from pass k's plan)
        auto next_of = [&](const int *m, int &item, int &part) {
            if (!__builtin_amdgcn_readfirstlane(m[M_VALID])) {
                item = -1;
                part = 0;
            } else if (__builtin_amdgcn_readfirstlane(m[M_PART]) == 1) {
                item = __builtin_amdgcn_readfirstlane(m[M_IMG]) * tiles + __builtin_amdgcn_readfirstlane(m[M_TILE]);
                part = 2;
            } else {
                int v = -1;
                if (lane == 0) v = claim_item(C, a, counters);
                item = __builtin_amdgcn_readfirstlane(v);
                part = 0;
            }
        };
        int v = -1;
        if (lane == 0) {
            C.issue(counters);
            v = claim_item(C, a, counters);
        }
        plan_item<TL, TS, CAP>(a, __builtin_amdgcn_readfirstlane(v), 0, tiles, ln[0], cl[0], rw[0], meta[0]);
        int item, part;
        next_of(meta[0], item, part);
        plan_item<TL, TS, CAP>(a, item, part, tiles, ln[1], cl[1], rw[1], meta[1]);
        __syncthreads();  // tables of passes 0 and 1
        __syncthreads();  // pass 0 staged
        for (int k = 0;; ++k) {
            if (!__builtin_amdgcn_readfirstlane(meta[k % 3][M_VALID])) break;
            next_of(meta[(k + 1) % 3], item, part);
            const int t2 = (k + 2) % 3;
            plan_item<TL, TS, CAP>(a, item, part, tiles, ln[t2], cl[t2], rw[t2], meta[t2]);
            __syncthreads();
        }
        return;
    }
    __syncthreads();  // tables of passes 0 and 1
    {
        const Meta m0 = read_meta(meta[0]);
        if (m0.valid && !m0.empty) build_bc_lut(m0.alpha, m0.beta, bc[0]);
        pass_dma<kThreads, CAP>(a, m0, rw[0], st0);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();  // pass 0 staged
    for (int k = 0;; k += 2) {
        if (!pipe6_step<TL, TS, CAP>(a, k, ln, cl, rw, meta, bc, nlut, st0, st1)) break;
        if (!pipe6_step<TL, TS, CAP>(a, k + 1, ln, cl, rw, meta, bc, nlut, st1, st0)) break;
    }
}

// Pipelined form with register staging: the four worker waves load pass k+1
// into VGPRs, blend pass k out of the single LDS stage into registers, and
// only after a barrier write the loaded chunks into the stage and store pass
// k's pixels, so the loads are in flight during the blend and the stores
// during the next pass, with one stage of LDS (two do not fit in the 40 KB a
// workgroup may take).  The planning wave runs two passes ahead into a third
// table set; two barriers per pass; both sides leave the loop at the first
// invalid pass, after the same number of barriers.
template <int TL, int TS, int CAP>
__global__ __launch_bounds__(kThreads + 64) __attribute__((amdgpu_waves_per_eu(4))) void k_ragged_pipe7(miaug_ragged_args a, int *__restrict__ counters) {
    __shared__ __align__(16) uint8_t st[stage_bytes(CAP)];
    __shared__ int4 ln[3][TL];
    __shared__ int4 cl[3][TS];
    __shared__ int2 rw[3][3 * TL];
    __shared__ __align__(16) int meta[3][M_N];
    __shared__ float nlut[3][256];
    __shared__ uint8_t bc[256];
    constexpr int kIt = chunks_per_lane<kThreads, CAP>();
    const int tiles = tiles_per_image<TL, TS>(a.out_h, a.out_w);
    const bool planner = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == kThreads / 64;
    build_norm_lut(a, nlut);
    if (planner) {
        __builtin_amdgcn_s_setprio(2);
        const int lane = threadIdx.x & 63;
        Claimer<1> C{tiles, (int)(blockIdx.x % kQueues), 0, 0};  // meaningful in lane 0
        auto next_of = [&](const int *m, int &item, int &part) {  // item and part of the pass after m's
            if (!__builtin_amdgcn_readfirstlane(m[M_VALID])) {
                item = -1;
                part = 0;
            } else if (__builtin_amdgcn_readfirstlane(m[M_PART]) == 1) {
                item = __builtin_amdgcn_readfirstlane(m[M_IMG]) * tiles + __builtin_amdgcn_readfirstlane(m[M_TILE]);
                part = 2;
            } else {
                int v = -1;
                if (lane == 0) v = claim_item(C, a, counters);
                item = __builtin_amdgcn_readfirstlane(v);
                part = 0;
            }
        };
        int v = -1;
        if (lane == 0) {
            C.issue(counters);
            v = claim_item(C, a, counters);
        }
        plan_item<TL, TS, CAP>(a, __builtin_amdgcn_readfirstlane(v), 0, tiles, ln[0], cl[0], rw[0], meta[0]);
        int item, part;
        next_of(meta[0], item, part);
        plan_item<TL, TS, CAP>(a, item, part, tiles, ln[1], cl[1], rw[1], meta[1]);
        __syncthreads();  // tables of passes 0 and 1
        __syncthreads();  // pass 0 staged
        for (int k = 0;; ++k) {
            if (!__builtin_amdgcn_readfirstlane(meta[k % 3][M_VALID])) break;
            next_of(meta[(k + 1) % 3], item, part);
            const int t2 = (k + 2) % 3;
            plan_item<TL, TS, CAP>(a, item, part, tiles, ln[t2], cl[t2], rw[t2], meta[t2]);
            __syncthreads();
            __syncthreads();
        }
        return;
    }
    __syncthreads();  // tables of passes 0 and 1
    {
        const Meta m0 = read_meta(meta[0]);
        u32x4 R[kIt];
        const uint32_t okm = pass_load<kThreads, CAP>(a, m0, rw[0], R);
        pass_stage<kThreads, CAP>(R, okm, st);
        if (m0.valid && !m0.empty) build_bc_lut(m0.alpha, m0.beta, bc);
    }
    __syncthreads();  // pass 0 staged
    for (int k = 0;; ++k) {
        const int t = k % 3, t1 = (k + 1) % 3;
        if (!__builtin_amdgcn_readfirstlane(meta[t][M_VALID])) break;
        if (a.boxes && !__builtin_amdgcn_readfirstlane(meta[t][M_EMPTY]) &&
            __builtin_amdgcn_readfirstlane(meta[t][M_TILE]) == 0 && __builtin_amdgcn_readfirstlane(meta[t][M_PART]) <= 1)
            ragged_boxes<kThreads>(a, __builtin_amdgcn_readfirstlane(meta[t][M_IMG]));  // before the loads: its
                                                                                       // loads would wait for them
        const Meta mn = read_meta(meta[t1]);
        u32x4 R[kIt];
        const uint32_t okm = pass_load<kThreads, CAP>(a, mn, rw[t1], R);
        const Meta mc = read_meta(meta[t]);
        BlendOut<pix_per_lane<TL, TS, kThreads>()> o;
        const bool keep = !mc.empty && mc.staged;
        if (keep) {
            if (mc.swap) blend_keep<TL, TS, kThreads, true>(a, mc, st, ln[t], cl[t], bc, nlut, o);
            else blend_keep<TL, TS, kThreads, false>(a, mc, st, ln[t], cl[t], bc, nlut, o);
        } else if (!mc.empty) {
            pass_direct<kThreads>(a, mc, bc, nlut);
        }
        __syncthreads();  // the stage and the LUT are free
        pass_stage<kThreads, CAP>(R, okm, st);
        if (mn.valid && !mn.empty) build_bc_lut(mn.alpha, mn.beta, bc);
        if (keep) store_out(a, mc.img, o);
        __syncthreads();  // pass k+1 staged
    }
}

// Flat grid: one workgroup per item, XCD-aware: workgroup b runs on XCD b mod 8
// and takes item b / 8 of queue b mod 8.
template <int TL, int TS, int CAP>
__global__ __launch_bounds__(kThreads) void k_ragged_flat(miaug_ragged_args a) {
    __shared__ __align__(16) uint8_t st[stage_bytes(CAP)];
    __shared__ int4 ln[TL];
    __shared__ int4 cl[TS];
    __shared__ int2 rw[3 * TL];
    __shared__ __align__(16) int meta[M_N];
    __shared__ float nlut[3][256];
    __shared__ uint8_t bc[256];
    const int tiles = tiles_per_image<TL, TS>(a.out_h, a.out_w);
    const int q = blockIdx.x % kQueues, idx = blockIdx.x / kQueues;
    const int img = (idx / tiles) * kQueues + q;
    if (img >= a.n) return;
    build_norm_lut(a, nlut);
    int bc_img = -1;
    int planner = 0;
    run_item<TL, TS, CAP>(a, img * tiles + idx % tiles, tiles, st, ln, cl, rw, meta, bc, bc_img, nlut, planner);
}

// One image per launch (the comparison form): workgroup b = tile b.
template <int TL, int TS, int CAP>
__global__ __launch_bounds__(kThreads) void k_ragged_one(miaug_ragged_args a, int img) {
    __shared__ __align__(16) uint8_t st[stage_bytes(CAP)];
    __shared__ int4 ln[TL];
    __shared__ int4 cl[TS];
    __shared__ int2 rw[3 * TL];
    __shared__ __align__(16) int meta[M_N];
    __shared__ float nlut[3][256];
    __shared__ uint8_t bc[256];
    const int tiles = tiles_per_image<TL, TS>(a.out_h, a.out_w);
    build_norm_lut(a, nlut);
    int bc_img = -1;
    int planner = 0;
    run_item<TL, TS, CAP>(a, img * tiles + (int)blockIdx.x, tiles, st, ln, cl, rw, meta, bc, bc_img, nlut, planner);
}

// ---------------------------------------------------------------- streaming pipeline
// Per-workgroup pass stream, followed by the planner wave.  Its first thread
// (the owner) keeps items two ahead in a 4-entry ring: when a pass consumes an
// item it issues the atomic for a later one and only reads the result after
// the next s_waitcnt vmcnt(0), so the atomic's latency overlaps a whole
// iteration.
template <int TL, int TS, int CAP>
struct Stream {
    int tiles;
    int r;                    // ring index of the next item (all threads of the planner wave)
    int q, tries, raw, slot;  // owner thread: queue state, atomic in flight (slot < 0: none)

    __device__ __forceinline__ void issue(int *counters) {
        if (tries < kQueues) raw = atomicAdd(&counters[q * kCounterStride], 1);
    }
    // Item from the atomic issued last (owner, after its result arrived);
    // exhausted queues are skipped with further, synchronous atomics.
    __device__ __forceinline__ int resolve(const miaug_ragged_args &a, int *counters) {
        while (tries < kQueues) {
            const int nq = (a.n - q + kQueues - 1) / kQueues;  // images i with i mod 8 == q
            if (raw < nq * tiles) return ((raw / tiles) * kQueues + q) * tiles + raw % tiles;
            q = (q + 1) % kQueues;
            if (++tries < kQueues) raw = atomicAdd(&counters[q * kCounterStride], 1);
        }
        return -1;
    }
    // Issues the atomic a consumed ring entry asked for (after the table
    // stage's global loads, so that none of them waits for it).
    __device__ __forceinline__ void issue_as_owner(int *counters) {
        if (slot >= 0) issue(counters);
    }
    __device__ __forceinline__ void publish_as_owner(const miaug_ragged_args &a, int *counters, int *ring) {
        if (slot >= 0) {
            ring[slot] = resolve(a, counters);
            slot = -1;
        }
    }
    // The pass after `prev` (the last planned pass): its second half, or the
    // first pass of the next item in the ring.  Every thread of the planner
    // wave takes the same decision; valid = false at the end of the work.
    __device__ __forceinline__ bool next_as(const Meta &prev, const int *ring, int &img, int &tile, int &part,
                                            bool owner) {
        if (!prev.valid) return false;
        if (prev.part == 1) {
            img = prev.img;
            tile = prev.tile;
            part = 2;
            return true;
        }
        const int item = __builtin_amdgcn_readfirstlane(ring[r & 3]);
        if (owner) slot = (r + 2) & 3;  // its atomic is issued by issue_as_owner()
        ++r;
        if (item < 0) return false;
        img = udiv_small(item, tiles, tile);
        part = 0;
        return true;
    }
};

// Boxes and brightness/contrast LUT of a pass about to be staged, by threads
// 0..NT-1 (NT >= 256).  Their global loads come before the pass's DMA is
// issued, so they never wait behind it.
template <int NT>
__device__ __forceinline__ void pass_side(const miaug_ragged_args &a, const Meta &m, uint8_t *bc, int &bc_img) {
    if (!m.valid || m.empty) return;
    if (m.tile == 0 && m.part <= 1 && a.boxes) ragged_boxes<NT>(a, m.img);
    if (bc_img != m.img) {
        if (threadIdx.x < 256) build_bc_lut(m.alpha, m.beta, bc);
        bc_img = m.img;
    }
}

// Streaming pipeline: NC waves stage and blend, one more wave plans.
// Iteration k (pass P_k in staging buffer k mod 2, table set k mod 3), after
// a barrier that publishes P_k's DMA, the tables of P_{k+1} and the item ring:
//   planner wave: decide P_{k+2}, plan it and write its tables (set k+2);
//                 thread 0 issues the queue atomic for a later item;
//   other waves:  LUT and boxes of P_{k+1}, DMA of P_{k+1} into the other
//                 buffer, blend of P_k (its LDS reads touch only variables the
//                 DMA does not write, so they do not wait for it).
// Two warm-up passes that do nothing fill the pipeline.
template <int TL, int TS, int CAP, int NC>
__global__ __launch_bounds__(64 * (NC + 1)) void k_ragged_stream(miaug_ragged_args a, int *__restrict__ counters) {
    constexpr int NT = 64 * NC;  // staging and blending threads
    __shared__ __align__(16) uint8_t st0[stage_bytes(CAP)];  // two distinct variables: see the file comment
    __shared__ __align__(16) uint8_t st1[stage_bytes(CAP)];
    __shared__ int4 ln[3][TL];
    __shared__ int4 cl[3][TS];
    __shared__ int2 rw[3][3 * TL];
    __shared__ __align__(16) int meta[3][M_N];
    __shared__ float nlut[3][256];
    __shared__ uint8_t bc[2][256];
    __shared__ int ring[4];
    const int tid = threadIdx.x;
    const bool planner = __builtin_amdgcn_readfirstlane(tid >> 6) == NC;
    // The planner's serial chain sets the pace of every iteration: let the
    // SIMD's arbiter prefer its instructions over the blend waves'.
    if (planner) __builtin_amdgcn_s_setprio(3);
    Stream<TL, TS, CAP> S;
    S.tiles = tiles_per_image<TL, TS>(a.out_h, a.out_w);
    S.r = 0;
    S.q = blockIdx.x % kQueues;
    S.tries = 0;
    S.raw = 0;
    S.slot = -1;
    if (tid == NT) {  // thread 0 of the planner wave owns the queue state
        for (int i = 0; i < 2; ++i) {
            S.slot = i;
            S.issue(counters);
            S.publish_as_owner(a, counters, ring);
        }
    }
    if (tid < 2 * M_N) meta[tid / M_N][tid % M_N] = (tid % M_N == M_VALID || tid % M_N == M_EMPTY) ? 1 : 0;
    build_norm_lut(a, nlut);
    int bc_img[2] = {-1, -1};
    int set = 0, B = 0;
    int info_img = -1, info_raw = 0;  // planner wave: image whose record is in (or on its way to) info_raw
    __syncthreads();
    Meta mnext = read_meta(meta[0]);  // warm-up pass 0
    for (;;) {
        __builtin_amdgcn_s_waitcnt(0);  // P_k's LDS-DMA, the stores before it, the owner's atomic
        if (tid == NT) S.publish_as_owner(a, counters, ring);
        __syncthreads();
        const int s1 = set == 2 ? 0 : set + 1, s2 = s1 == 2 ? 0 : s1 + 1;
        const Meta mk = mnext;  // P_k's plan, read last iteration
        if (!mk.valid) break;
        const Meta m1 = read_meta(meta[s1]);
        mnext = m1;
        if (planner) {
            int img2 = 0, tile2 = 0, part2 = 0;
            const bool v2 = S.next_as(m1, ring, img2, tile2, part2, tid == NT);
            if (v2 && img2 != info_img) {  // not prefetched: load now
                info_raw = info_issue(a, img2);
                info_img = img2;
            }
            const ImgInfo in = info_gather(info_raw);
            Pass p2 = plan_pass<TL, TS, CAP>(a, in, img2, tile2, part2);
            p2.valid = v2;
            pass_tables<TL, TS>(a, p2, ln[s2], cl[s2], rw[s2], meta[s2]);
            // prefetch the image of the next ring entry; it arrives by the next iteration's wait
            const int nitem = v2 ? __builtin_amdgcn_readfirstlane(ring[S.r & 3]) : -1;
            if (nitem >= 0) {
                int t;
                const int nimg = udiv_small(nitem, S.tiles, t);
                if (nimg != info_img) {
                    info_raw = info_issue(a, nimg);
                    info_img = nimg;
                }
            }
            if (tid == NT) S.issue_as_owner(counters);
        } else {
            pass_side<NT>(a, m1, bc[B ^ 1], bc_img[B ^ 1]);
            if (B == 0) {
                pass_dma<NT, CAP>(a, m1, rw[s1], st1);
                if (!mk.empty && mk.staged) pass_blend<TL, TS, NT>(a, mk, st0, ln[set], cl[set], bc[0], nlut);
            } else {
                pass_dma<NT, CAP>(a, m1, rw[s1], st0);
                if (!mk.empty && mk.staged) pass_blend<TL, TS, NT>(a, mk, st1, ln[set], cl[set], bc[1], nlut);
            }
            if (!mk.empty && !mk.staged) pass_direct<NT>(a, mk, bc[B], nlut);
        }
        set = s1;
        B ^= 1;
    }
}


struct Variant {
    int tl, ts;
    int mode;       // 0 streaming pipeline, 1 persistent one pass at a time, 2 flat grid, 3 persistent with
                    // the next pass planned during the current pass's DMA, 4 the same with a planning wave,
                    // 5 double-buffered stage with the planning wave two passes ahead, 6 register-staged loads,
                    // 7 row bands (k_rows.hip), 8 wave-independent row gathers (k_gather.hip)
    int wg_per_cu;  // workgroups per CU of the persistent modes
    int chunk;      // tiles claimed per atomic (persistent mode); stage size of the row-band form
    const char *name;
};
// Variant 0 is the default: the wave-gather form of k_gather.hip with one
// band per workgroup (0.66-0.68 ms per 2048-image batch against 0.76 ms for
// the best tile-pass form, which follows it).  Workgroups per CU are chosen
// against the LDS as measured on gfx950: a workgroup above about 40 KB runs as
// if only one fits in each 80 KB half of the 160 KB (three 42.5 KB workgroups
// per CU run like two), so the staged forms keep a workgroup at or under
// 40 KB; the tile passes run three per CU (four measured the same).
const Variant kVariants[] = {
    {0, 0, 8, 4, 32 + 64, "wave row gathers, 32 lines x 64 per item, band per workgroup, 4 wg/CU"},
    {0, 0, 8, 6, 32 + 64, "wave row gathers, 32 lines x 64 per item, band per workgroup, 6 wg/CU"},
    {0, 0, 8, 4, 16 + 64, "wave row gathers, 16 lines x 64 per item, band per workgroup, 4 wg/CU"},
    {0, 0, 8, 4, 32, "wave row gathers, 32 lines x 64 per item, 4 wg/CU"},
    {32, 32, 4, 3, 1, "tile 32x32, persistent 3 wg/CU, 4 worker waves + a planning wave"},
    {32, 32, 3, 4, 1, "tile 32x32, persistent 4 wg/CU, next pass planned during the DMA"},
    {32, 32, 5, 2, 1, "tile 32x32, persistent 2 wg/CU, double-buffered stage, planning wave two passes ahead"},
    {32, 32, 6, 3, 1, "tile 32x32, persistent 3 wg/CU, register-staged loads, planning wave two passes ahead"},
    {32, 32, 1, 4, 1, "tile 32x32, persistent 4 wg/CU, chunks of 1"},
    {32, 32, 1, 4, 4, "tile 32x32, persistent 4 wg/CU, chunks of 4"},
    {32, 32, 1, 4, 8, "tile 32x32, persistent 4 wg/CU, chunks of 8"},
    {16, 32, 1, 8, 8, "tile 16x32, persistent 8 wg/CU, chunks of 8"},
    {16, 32, 4, 6, 1, "tile 16x32, persistent 6 wg/CU, 4 worker waves + a planning wave"},
    {32, 32, 2, 0, 1, "tile 32x32, flat grid"},
    {32, 32, 0, 2, 1, "tile 32x32, streaming pipeline 8+1 waves, 2 wg/CU"},
    {16, 64, 4, 4, 1, "tile 16x64, persistent 4 wg/CU, 4 worker waves + a planning wave"},
    {8, 128, 4, 4, 1, "tile 8x128, persistent 4 wg/CU, 4 worker waves + a planning wave"},
    {0, 0, 7, 3, 0, "off: row bands of 16 lines, whole source rows, 17 KB stages x 2, 3 wg/CU"},
    {0, 0, 7, 4, 0, "off: row bands of 16 lines, whole source rows, 17 KB stages x 2, 4 wg/CU"},
    {0, 0, 7, 6, 1, "off: row bands of 16 lines, whole source rows, 9 KB stages x 2, 6 wg/CU"},
    {0, 0, 7, 2, 2, "off: row bands of 16 lines, whole source rows, 36 KB stages x 2, 2 wg/CU"},
    {0, 0, 8, 4, 32 + 64 + 128, "wave row gathers, 32 lines x 64 per item, band per workgroup, 4 wg/CU, largest images first"},
    {0, 0, 8, 6, 32 + 64 + 128, "wave row gathers, 32 lines x 64 per item, band per workgroup, 6 wg/CU, largest images first"},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <int TL, int TS, int K>
hipError_t launch_chunked(const miaug_ragged_args *a, int grid, int *counters, hipStream_t s) {
    hipLaunchKernelGGL((k_ragged_persistent<TL, TS, full_cap<TL, TS>(), K>), dim3(grid), dim3(kThreads), 0, s, *a,
                       counters);
    return hipGetLastError();
}

template <int TL, int TS>
hipError_t launch_t(const miaug_ragged_args *a, const Variant &v, const RaggedLaunch &L, int per_image,
                    hipStream_t s) {
    constexpr int kFull = full_cap<TL, TS>();
    const int tiles = tiles_per_image<TL, TS>(a->out_h, a->out_w);
    if (per_image) {
        for (int i = 0; i < a->n; ++i) {
            hipLaunchKernelGGL((k_ragged_one<TL, TS, kFull>), dim3(tiles), dim3(kThreads), 0, s, *a, i);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    if (v.mode == 2) {
        const int per_q = (a->n + kQueues - 1) / kQueues;
        hipLaunchKernelGGL((k_ragged_flat<TL, TS, kFull>), dim3(kQueues * per_q * tiles), dim3(kThreads), 0, s, *a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(256), 0, s, L.counters, kQueues * kCounterStride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int grid = L.num_cu * v.wg_per_cu;
    const long items = (long)a->n * tiles;
    if (grid > items) grid = (int)items;
    grid = ((grid + kQueues - 1) / kQueues) * kQueues;
    if (v.mode == 0) {
        hipLaunchKernelGGL((k_ragged_stream<TL, TS, kFull, 8>), dim3(grid), dim3(64 * 9), 0, s, *a, L.counters);
        return hipGetLastError();
    }
    if (v.mode == 3) {
        hipLaunchKernelGGL((k_ragged_pipe<TL, TS, full_cap<TL, TS, 43>()>), dim3(grid), dim3(kThreads), 0, s,
                           *a, L.counters);
        return hipGetLastError();
    }
    if (v.mode == 4) {
        hipLaunchKernelGGL((k_ragged_pipe5<TL, TS, full_cap<TL, TS, 43>()>), dim3(grid), dim3(kThreads + 64), 0, s,
                           *a, L.counters);
        return hipGetLastError();
    }
    if (v.mode == 6) {
        hipLaunchKernelGGL((k_ragged_pipe7<TL, TS, full_cap<TL, TS, 41>()>), dim3(grid), dim3(kThreads + 64), 0, s,
                           *a, L.counters);
        return hipGetLastError();
    }
    if (v.mode == 5) {
        hipLaunchKernelGGL((k_ragged_pipe6<TL, TS, full_cap<TL, TS, 26>()>), dim3(grid), dim3(kThreads + 64), 0, s,
                           *a, L.counters);
        return hipGetLastError();
    }
    if (v.chunk >= 8) return launch_chunked<TL, TS, 8>(a, grid, L.counters, s);
    if (v.chunk >= 4) return launch_chunked<TL, TS, 4>(a, grid, L.counters, s);
    return launch_chunked<TL, TS, 1>(a, grid, L.counters, s);
}

// Tile shapes that only the planning-wave form runs.
template <int TL, int TS>
hipError_t launch_pipe5_only(const miaug_ragged_args *a, const Variant &v, const RaggedLaunch &L, hipStream_t s) {
    if (v.mode != 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(256), 0, s, L.counters, kQueues * kCounterStride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int tiles = tiles_per_image<TL, TS>(a->out_h, a->out_w);
    int grid = L.num_cu * v.wg_per_cu;
    const long items = (long)a->n * tiles;
    if (grid > items) grid = (int)items;
    grid = ((grid + kQueues - 1) / kQueues) * kQueues;
    hipLaunchKernelGGL((k_ragged_pipe5<TL, TS, full_cap<TL, TS, 43>()>), dim3(grid), dim3(kThreads + 64), 0, s, *a,
                       L.counters);
    return hipGetLastError();
}

}  // namespace

int ragged_variant_count() { return kNumVariants; }
// The row-band forms (k_rows.hip) are switched off: in one run of the parity
// tests one of them wrote a wrong image for one batch with unaligned starts,
// while a rerun and every earlier run were exact; the cause is not found.
// They were never the fastest form.  Their indices stay (names "off: ...").
bool ragged_variant_enabled(int v) { return v >= 0 && v < kNumVariants && kVariants[v].mode != 7; }
const char *ragged_variant_name(int v) { return (v >= 0 && v < kNumVariants) ? kVariants[v].name : nullptr; }
int ragged_default_variant() { return 0; }
int ragged_counter_ints() { return kQueues * kCounterStride; }

hipError_t launch_ragged(const miaug_ragged_args *a, const RaggedLaunch &L, int per_image, hipStream_t s) {
    if (a->n == 0) return hipSuccess;
    const Variant &v = kVariants[(L.variant >= 0 && L.variant < kNumVariants) ? L.variant : 0];
    if (!per_image && v.mode == 7) return launch_ragged_rows(a, v.chunk, v.wg_per_cu, L, s);
    if (!per_image && v.mode == 8) return launch_ragged_gather(a, v.chunk, v.wg_per_cu, L, s);
    if (per_image || v.tl == 32) return launch_t<32, 32>(a, v, L, per_image, s);
    if (v.ts == 64) return launch_pipe5_only<16, 64>(a, v, L, s);
    if (v.ts == 128) return launch_pipe5_only<8, 128>(a, v, L, s);
    return launch_t<16, 32>(a, v, L, per_image, s);
}

}  // namespace miaug
