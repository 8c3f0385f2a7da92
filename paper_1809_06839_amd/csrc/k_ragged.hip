// k_ragged.hip -- ragged batch: Dih4 + brightness/contrast -> bilinear resize
// -> per-channel normalisation into float32 CHW, with masks (nearest) and
// boxes following the same geometry (Sec. II-A: images of uneven size
// transformed together with masks and boxes; Sec. II-B Dih4; Table I
// Brightness).
//
// Work item = (image, output tile of T x T).  The separable resize needs two
// source lines per output line along one output axis (the "line" axis: output
// rows, or output columns when the Dih4 element swaps axes) and a contiguous
// span of source columns along the other.  A tile therefore stages 2*T
// source row segments into LDS with 16-byte loads (only the rows the taps
// touch, so downscaled images skip rows in HBM), then every output pixel reads
// its 4 taps from LDS, applies the brightness/contrast LUT per tap, blends
// with Q10 weights, rounds once and looks the result up in the normalisation
// LUT.  Output stores are float rows of T (coalesced per channel plane).
//
// Scheduling: the batched form is one persistent launch.  Images are dealt to
// 8 queues (image i -> queue i mod 8); workgroup b starts on queue b mod 8,
// which is the XCD the hardware dispatches it to, so the tiles of one image
// share that XCD's L2.  A workgroup pops tiles with an atomic counter and,
// when its queue is empty, moves on to the next queue; every workgroup ends
// after at most 8 empty pops.  Counters are cleared by a one-block fill kernel
// enqueued just before, so the pair can be captured in a hipGraph.
#include "dev_common.h"
#include "internal.h"

namespace miaug {
namespace {

constexpr int kThreads = 256;
constexpr int kQueues = 8;
constexpr int kCounterStride = 16;  // ints between counters (one 64-byte line each)
typedef __attribute__((address_space(3))) void *lds_ptr_t;

// Half-pixel-centre position of output index j (Q10):
// rdiv_he(((2j+1) Ls - Lo) 2^10, 2 Lo), evaluated with two 32-bit floor
// divisions: A = (2j+1) Ls - Lo = qa D + ra (D = 2 Lo), then ra 2^10 = qb D + rb.
__device__ __forceinline__ int32_t resize_q(int j, int Ls, int Lo) {
    const int D = 2 * Lo;
    const int A = (2 * j + 1) * Ls - Lo;
    int qa = A / D, ra = A - qa * D;
    if (ra < 0) { qa -= 1; ra += D; }
    const int B = ra << kFBits;
    const int qb = B / D, rb = B - qb * D;
    const int q = (qa << kFBits) + qb;
    return q + ((2 * rb > D) | ((2 * rb == D) & (q & 1)));
}

// Round-half-even of acc / 2^20 for acc >= 0.
__device__ __forceinline__ int rhe20(int acc) { return (acc + 0x7FFFF + ((acc >> 20) & 1)) >> 20; }

// A tile covers TL output lines (the axis whose taps select source rows) by
// TS span positions (the axis whose taps select source columns).
template <int TL, int TS>
struct Cfg {
    static constexpr int kMaxSpanPx = (TS - 1) * 46 / 10 + 4;        // staged span: scale factors up to 4.6
    static constexpr int kChunks = (kMaxSpanPx * 3 + 30) / 16;       // 16-byte chunks per image slot
    static constexpr int kStride = kChunks * 16;
    static constexpr int kMChunks = (kMaxSpanPx + 30) / 16;
    static constexpr int kMStride = kMChunks * 16;
    static constexpr int kPix = (TL * TS + kThreads - 1) / kThreads;  // output pixels per thread
    static_assert(TL <= 64 && TS <= 64 && TL % 8 == 0 && TS % 8 == 0, "tile sides are multiples of 8, at most 64");
};

// Work items per image: the tile grid in line x span coordinates depends on
// whether the element swaps axes, so the queue reserves the larger count.
template <int TL, int TS>
__host__ __device__ __forceinline__ int tiles_per_image(int OH, int OW) {
    const int a = ((OH + TL - 1) / TL) * ((OW + TS - 1) / TS);
    const int b = ((OW + TL - 1) / TL) * ((OH + TS - 1) / TS);
    return a > b ? a : b;
}

// LDS of a workgroup with NB staging buffers (1: plain, 2: pipelined).
template <int TL, int TS, int NB>
struct __align__(16) Smem {
    // staging buffer b: image slot s at byte 16*s*nchi, mask slot s at byte
    // 16*(2*nl*nchi + s*nchm) (nchi, nchm: 16-byte chunks per slot of the tile)
    uint8_t stage[NB][2 * TL * Cfg<TL, TS>::kStride + TL * Cfg<TL, TS>::kMStride + 16];
    int4 line[NB][TL];  // per output line: LDS offsets of the two tap rows and the nearest mask row, weight
    int4 col[NB][TS];   // per span position: byte offsets of the two taps in a row, weight, mask offset
    int32_t qline[NB][TL], qspan[NB][TS];
    float nlut[3][256];
    uint8_t bclut[NB][256];
    int item[4];
};

template <int TL, int TS, int NB>
__device__ __forceinline__ void build_norm_lut(const miaug_ragged_args &a, Smem<TL, TS, NB> &S) {
    for (int e = threadIdx.x; e < 3 * 256; e += kThreads) {
        int c = e >> 8, v = e & 255;
        S.nlut[c][v] = (float)((((double)v / 255.0) - (double)a.mean[c]) / (double)a.stdv[c]);
    }
}

// Boxes of one image: Dih4 ops one after the other, then the scale to the
// output size, in double.
__device__ __forceinline__ void ragged_boxes(const miaug_ragged_args &a, int img) {
    int b0 = a.box_off[img], b1 = a.box_off[img + 1];
    const int32_t *fl = a.flags + 4 * img;
    for (int b = b0 + (int)threadIdx.x; b < b1; b += kThreads) {
        double x1 = a.boxes[4 * b], y1 = a.boxes[4 * b + 1], x2 = a.boxes[4 * b + 2], y2 = a.boxes[4 * b + 3];
        double h = a.hw[2 * img], w = a.hw[2 * img + 1];
        if (fl[0]) { double u = w - x2, v = w - x1; x1 = u; x2 = v; }
        if (fl[1]) { double u = h - y2, v = h - y1; y1 = u; y2 = v; }
        for (int t = 0; t < (fl[2] & 3); ++t) {
            double nx1 = y1, ny1 = w - x2, nx2 = y2, ny2 = w - x1;
            x1 = nx1; y1 = ny1; x2 = nx2; y2 = ny2;
            double s = h; h = w; w = s;
        }
        if (fl[3]) {
            double nx1 = y1, ny1 = x1, nx2 = y2, ny2 = x2;
            x1 = nx1; y1 = ny1; x2 = nx2; y2 = ny2;
            double s = h; h = w; w = s;
        }
        double sx = (double)a.out_w / w, sy = (double)a.out_h / h;
        a.out_boxes[4 * b] = (float)(x1 * sx);
        a.out_boxes[4 * b + 1] = (float)(y1 * sy);
        a.out_boxes[4 * b + 2] = (float)(x2 * sx);
        a.out_boxes[4 * b + 3] = (float)(y2 * sy);
    }
}

// Geometry of one work item, identical in every thread.
struct Tile {
    int img, tile;
    int H, W;
    D4Map m;
    bool swap, staged, empty;
    int j0, i0, th, tw, nl, ns, Ll, Ls, kl, ks;
    int nchi, nchm, img_items;
    int sxlo, nsx, mxlo, nmx;  // source column span of the bilinear taps / of the nearest taps
};

template <int TL, int TS>
__device__ __forceinline__ Tile tile_geometry(const miaug_ragged_args &a, int img, int tile) {
    Tile t;
    t.img = img;
    t.tile = tile;
    t.H = a.hw[2 * img];
    t.W = a.hw[2 * img + 1];
    // images that are empty or not addressable with 32-bit byte offsets are
    // skipped (their outputs are left untouched)
    t.empty = t.H < 1 || t.W < 1 || (int64_t)t.H * t.W * 3 >= ((int64_t)1 << 31);
    const int32_t *fl = a.flags + 4 * img;
    t.m = make_d4(max(t.H, 1), max(t.W, 1), fl[0], fl[1], fl[2], fl[3]);
    t.swap = t.m.swaps();
    // line axis: output rows, or output columns when the element swaps axes
    const int OL = t.swap ? a.out_w : a.out_h, OS = t.swap ? a.out_h : a.out_w;
    const int n_sb = (OS + TS - 1) / TS;
    const int l0 = (tile / n_sb) * TL, s0 = (tile % n_sb) * TS;
    if (l0 >= OL) t.empty = true;  // spare item of the larger tile grid
    t.nl = min(TL, OL - l0);
    t.ns = min(TS, OS - s0);
    t.j0 = t.swap ? s0 : l0;
    t.i0 = t.swap ? l0 : s0;
    t.th = t.swap ? t.ns : t.nl;
    t.tw = t.swap ? t.nl : t.ns;
    t.Ll = t.swap ? t.m.ow : t.m.oh;
    t.Ls = t.swap ? t.m.oh : t.m.ow;
    t.kl = t.swap ? t.m.by : t.m.ay;
    t.ks = t.swap ? t.m.ax : t.m.bx;
    return t;
}

// Phase 1 of a work item into buffer b: resize positions of its lines and
// span positions, the brightness/contrast LUT, the boxes (first tile of an
// image), then -- after one barrier -- the LDS-DMA of the source rows and the
// per-line / per-column tables.  The DMA completes asynchronously (vmcnt);
// compute_tile may read buffer b only after s_waitcnt vmcnt(0) + a barrier.
template <int TL, int TS, int NB>
__device__ __forceinline__ void prepare_tile(const miaug_ragged_args &a, Tile &t, int b, Smem<TL, TS, NB> &S,
                                             int &lut_img) {
    using C = Cfg<TL, TS>;
    const int tid = threadIdx.x;
    if (t.empty) {
        __syncthreads();
        t.staged = false;
        return;
    }
    const int OL = t.swap ? a.out_w : a.out_h, OS = t.swap ? a.out_h : a.out_w;
    const int l0 = t.swap ? t.i0 : t.j0, s0 = t.swap ? t.j0 : t.i0;
    static_assert(TL <= 64 && TS <= 64, "line and span positions are computed by threads 0..63 and 64..127");
    if (lut_img != t.img) {
        if (tid < 256) {
            const double v = (double)a.ab[2 * t.img] * (double)tid + (double)a.ab[2 * t.img + 1];
            S.bclut[b][tid] = (uint8_t)sat8((int)rint(v));
        }
        lut_img = t.img;
    }
    if (tid < t.nl) S.qline[b][tid] = resize_q(l0 + tid, t.Ll, OL);
    if (tid >= 64 && tid - 64 < t.ns) S.qspan[b][tid - 64] = resize_q(s0 + tid - 64, t.Ls, OS);
    if (t.tile == 0 && a.boxes) ragged_boxes(a, t.img);
    __syncthreads();

    // source column span of the tile (bilinear taps) and of its nearest taps
    const D4Map &m = t.m;
    const int W = t.W, Ll = t.Ll, Ls = t.Ls, kl = t.kl, ks = t.ks, nl = t.nl;
    const int32_t qs_first = S.qspan[b][0], qs_last = S.qspan[b][t.ns - 1];
    const int dlo = clampi(qs_first >> kFBits, Ls), dhi = clampi((qs_last >> kFBits) + 1, Ls);
    const int xa = ks * dlo + m.cx, xb = ks * dhi + m.cx;
    const int sxlo = min(xa, xb), nsx = abs(xb - xa) + 1;
    const int nlo = clampi((qs_first + kFOne / 2) >> kFBits, Ls), nhi = clampi((qs_last + kFOne / 2) >> kFBits, Ls);
    const int mxa = ks * nlo + m.cx, mxb = ks * nhi + m.cx;
    const int mxlo = min(mxa, mxb), nmx = abs(mxb - mxa) + 1;
    t.staged = nsx <= C::kMaxSpanPx;
    const uint8_t *ibase = a.img + a.img_off[t.img];
    const uint8_t *mbase = a.mask ? a.mask + a.mask_off[t.img] : nullptr;

    // Staging: item `it` (a 16-byte chunk of an image or mask slot) is copied
    // straight from HBM to LDS byte 16*it with global_load_lds_dwordx4.  The 64
    // lanes of a wave take 64 consecutive items, which is the DMA's lane layout
    // (LDS base in M0 + 16 * lane), so no registers hold the data and a
    // workgroup has its whole footprint in flight at once.
    t.nchi = (nsx * 3 + 30) >> 4;
    t.nchm = mbase ? (nmx + 30) >> 4 : 0;
    t.img_items = 2 * nl * t.nchi;
    if (!t.staged) return;
    const int nchi = t.nchi, nchm = t.nchm, img_items = t.img_items;
    const int total = img_items + nl * nchm;
    const uint32_t inv_i = ((1u << 20) + nchi - 1) / nchi;            // it / nchi = (it * inv) >> 20
    const uint32_t inv_m = nchm ? ((1u << 20) + nchm - 1) / nchm : 0;  // (exact for it < 4096)
    const int lane = tid & 63;
    uint8_t *stage = S.stage[b];
    for (int base = tid - lane; base < total; base += kThreads) {
        const int it = base + lane;
        const uint8_t *src = nullptr;
        if (it < total) {
            const uint8_t *g;
            int len, ch;
            if (it < img_items) {
                const int slot = (int)(((uint32_t)it * inv_i) >> 20);
                ch = it - slot * nchi;
                const int d = clampi((S.qline[b][slot >> 1] >> kFBits) + (slot & 1), Ll);
                g = ibase + (uint32_t)(((kl * d + m.cy) * W + sxlo) * 3);  // images are < 2^31 bytes
                len = nsx * 3;
            } else {
                const int it2 = it - img_items, slot = (int)(((uint32_t)it2 * inv_m) >> 20);
                ch = it2 - slot * nchm;
                const int d = clampi((S.qline[b][slot] + kFOne / 2) >> kFBits, Ll);
                g = mbase + (uint32_t)((kl * d + m.cy) * W + mxlo);
                len = nmx;
            }
            if (ch < span_chunks(g, len)) src = (const uint8_t *)((uintptr_t)g & ~(uintptr_t)15) + 16 * ch;
        }
        if (src) __builtin_amdgcn_global_load_lds((const void *)src, (lds_ptr_t)(stage + 16 * base), 16, 0, 0);
    }
    // per-line and per-column tables
    if (tid < nl) {
        const int q = S.qline[b][tid];
        const int d0 = clampi(q >> kFBits, Ll), d1 = clampi((q >> kFBits) + 1, Ll);
        const uint8_t *g0 = ibase + ((size_t)(kl * d0 + m.cy) * W + sxlo) * 3;
        const uint8_t *g1 = ibase + ((size_t)(kl * d1 + m.cy) * W + sxlo) * 3;
        int mb = 0;
        if (mbase) {
            const int dn = clampi((q + kFOne / 2) >> kFBits, Ll);
            mb = 16 * (img_items + tid * nchm) + span_phase(mbase + (size_t)(kl * dn + m.cy) * W + mxlo);
        }
        S.line[b][tid] = make_int4(16 * (2 * tid) * nchi + span_phase(g0), 16 * (2 * tid + 1) * nchi + span_phase(g1),
                                   q & (kFOne - 1), mb);
    }
    if (tid >= 64 && tid - 64 < t.ns) {
        const int si = tid - 64, q = S.qspan[b][si];
        const int e0 = clampi(q >> kFBits, Ls), e1 = clampi((q >> kFBits) + 1, Ls);
        const int en = clampi((q + kFOne / 2) >> kFBits, Ls);
        S.col[b][si] = make_int4(3 * (ks * e0 + m.cx - sxlo), 3 * (ks * e1 + m.cx - sxlo), q & (kFOne - 1),
                                 ks * en + m.cx - mxlo);
    }
}

// Phase 2: blend, normalise and store the tile from buffer b (staged), or
// from global memory when the span was too wide for the staging buffer.
// Three bytes of a staged pixel at LDS byte offset o (any alignment): one
// ds_read2_b32 of the two dwords that hold it, then a byte-aligned funnel shift.
__device__ __forceinline__ uint32_t lds_rgb(const uint8_t *st, int o) {
    const uint32_t *w = (const uint32_t *)(st + (o & ~3));
    return __builtin_amdgcn_alignbyte(w[1], w[0], o & 3);
}

template <int TL, int TS, int NB>
__device__ __forceinline__ void compute_tile(const miaug_ragged_args &a, const Tile &t, int b,
                                             Smem<TL, TS, NB> &S) {
    using C = Cfg<TL, TS>;
    if (t.empty) return;
    const int tid = threadIdx.x;
    const size_t plane = (size_t)a.out_h * a.out_w;
    const int OW = a.out_w;
    const bool has_mask = a.mask != nullptr;
    if (t.staged) {
        // Uniform per-channel bases + 32-bit per-pixel offsets keep address
        // arithmetic scalar.  Lanes take a 32-wide output row segment when the
        // element keeps the axes (consecutive lanes read consecutive columns of
        // the same two staged rows), and an 8 x 8 block when it swaps them
        // (consecutive lanes would otherwise read the same column of 32
        // different staged rows, which share few LDS banks).
        const __amdgpu_buffer_rsrc_t ro = buffer_rsrc(a.out + (size_t)t.img * 3 * plane, (uint32_t)(12 * plane));
        const __amdgpu_buffer_rsrc_t rm =
            buffer_rsrc(has_mask ? a.out_mask + (size_t)t.img * plane : a.out_mask, (uint32_t)plane);
        const int base = t.j0 * OW + t.i0;
        const uint8_t *st = S.stage[b];
#pragma unroll
        for (int k = 0; k < C::kPix; ++k) {
            const int p = tid + k * kThreads;
            int l, si;  // line and span position within the tile
            if (!t.swap) {
                l = p / TS;
                si = p - l * TS;
            } else {
                const int lane = p & 63, blk = p >> 6;  // 8 x 8 blocks
                l = 8 * (blk % (TL / 8)) + (lane & 7);
                si = 8 * (blk / (TL / 8)) + (lane >> 3);
            }
            if (p >= TL * TS || l >= t.nl || si >= t.ns) continue;
            const int jj = t.swap ? si : l, ii = t.swap ? l : si;
            const int4 L = S.line[b][l];
            const int4 Cc = S.col[b][si];
            const uint32_t q00 = lds_rgb(st, L.x + Cc.x), q01 = lds_rgb(st, L.x + Cc.y);
            const uint32_t q10 = lds_rgb(st, L.y + Cc.x), q11 = lds_rgb(st, L.y + Cc.y);
            const int wl1 = L.z, ws1 = Cc.z;
            int v[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int p00 = S.bclut[b][(q00 >> (8 * c)) & 255], p01 = S.bclut[b][(q01 >> (8 * c)) & 255];
                const int p10 = S.bclut[b][(q10 >> (8 * c)) & 255], p11 = S.bclut[b][(q11 >> (8 * c)) & 255];
                // (1024-ws1) p00 + ws1 p01 = 1024 p00 + ws1 (p01 - p00), exactly; same for rows.
                // Every product has operands below 2^24 in magnitude: full-rate 24-bit multiplies.
                const int t0 = mad24(ws1, p01 - p00, p00 << kFBits);
                const int t1 = mad24(ws1, p11 - p10, p10 << kFBits);
                v[c] = rhe20(mad24(wl1, t1 - t0, t0 << kFBits));
            }
            const int off = base + jj * OW + ii;
            // the b32 store takes the bit pattern: pass the float's bits, not its value
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(S.nlut[0][v[0]]), ro, 4 * off, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(S.nlut[1][v[1]]), ro, 4 * (off + (int)plane), 0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(S.nlut[2][v[2]]), ro, 4 * (off + 2 * (int)plane), 0,
                                                  0);
            if (has_mask) __builtin_amdgcn_raw_buffer_store_b8(st[L.w + Cc.w], rm, off, 0, 0);
        }
        return;
    }
    // Fallback for spans wider than the staging buffer (source more than 4.6x
    // the output along the span axis): the same arithmetic on direct loads.
    const D4Map &m = t.m;
    const uint8_t *ibase = a.img + a.img_off[t.img];
    const uint8_t *mbase = has_mask ? a.mask + a.mask_off[t.img] : nullptr;
#pragma unroll
    for (int k = 0; k < C::kPix; ++k) {
        const int p = tid + k * kThreads;
        const int l = p / TS, si = p - l * TS;
        if (p >= TL * TS || l >= t.nl || si >= t.ns) continue;
        const int jj = t.swap ? si : l, ii = t.swap ? l : si;
        const int32_t ql = S.qline[b][l], qs = S.qspan[b][si];
        const int wl1 = ql & (kFOne - 1), ws1 = qs & (kFOne - 1);
        const int x0 = t.ks * clampi(qs >> kFBits, t.Ls) + m.cx, x1 = t.ks * clampi((qs >> kFBits) + 1, t.Ls) + m.cx;
        const int y0 = t.kl * clampi(ql >> kFBits, t.Ll) + m.cy, y1 = t.kl * clampi((ql >> kFBits) + 1, t.Ll) + m.cy;
        const uint8_t *r0 = ibase + (size_t)y0 * t.W * 3, *r1 = ibase + (size_t)y1 * t.W * 3;
        float *o = a.out + (size_t)t.img * 3 * plane + (size_t)(t.j0 + jj) * OW + (t.i0 + ii);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int p00 = S.bclut[b][r0[3 * x0 + c]], p01 = S.bclut[b][r0[3 * x1 + c]];
            const int p10 = S.bclut[b][r1[3 * x0 + c]], p11 = S.bclut[b][r1[3 * x1 + c]];
            const int t0 = (p00 << kFBits) + ws1 * (p01 - p00);
            const int t1 = (p10 << kFBits) + ws1 * (p11 - p10);
            o[c * plane] = S.nlut[c][rhe20((t0 << kFBits) + wl1 * (t1 - t0))];
        }
        if (mbase) {
            const int mx = t.ks * clampi((qs + kFOne / 2) >> kFBits, t.Ls) + m.cx;
            const int my = t.kl * clampi((ql + kFOne / 2) >> kFBits, t.Ll) + m.cy;
            a.out_mask[(size_t)t.img * plane + (size_t)(t.j0 + jj) * OW + (t.i0 + ii)] = mbase[(size_t)my * t.W + mx];
        }
    }
}

// One work item, not pipelined.
template <int TL, int TS, int NB>
__device__ __forceinline__ void run_tile(const miaug_ragged_args &a, int img, int tile, Smem<TL, TS, NB> &S,
                                         int &lut_img) {
    Tile t = tile_geometry<TL, TS>(a, img, tile);
    prepare_tile<TL, TS, NB>(a, t, 0, S, lut_img);
    __builtin_amdgcn_s_waitcnt(0);  // LDS-DMA writes are counted by vmcnt
    __syncthreads();
    compute_tile<TL, TS, NB>(a, t, 0, S);
}

// Work-item queue: images are dealt to 8 queues (image i -> queue i mod 8);
// pop() hands out (image, tile) items of queue q in order and moves on to the
// next queue when q is empty.  Returns -1 once all 8 queues are exhausted.
__device__ __forceinline__ int pop_item(const miaug_ragged_args &a, int *counters, int tiles, int &q, int &tries) {
    while (tries < kQueues) {
        const int nq = (a.n - q + kQueues - 1) / kQueues;  // images i with i mod 8 == q
        const int idx = atomicAdd(&counters[q * kCounterStride], 1);
        if (idx < nq * tiles) return ((idx / tiles) * kQueues + q) * tiles + idx % tiles;
        q = (q + 1) % kQueues;
        ++tries;
    }
    return -1;
}

// ---------------------------------------------------------------- register-prefetch pipeline
// The next tile's source rows are loaded into registers (ordinary 16-byte
// global loads) while the current tile is blended from LDS; after a barrier
// the registers are written to the single LDS stage.  Unlike an LDS-DMA into
// a second buffer, register loads do not make the compiler wait for them
// before the current tile's LDS reads, so load latency overlaps compute while
// the workgroup keeps one stage buffer (4 workgroups per CU at 32 x 32).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int TL, int TS>
struct Prefetch {
    static constexpr int kPer = (2 * TL * Cfg<TL, TS>::kChunks + TL * Cfg<TL, TS>::kMChunks + kThreads - 1) / kThreads;
    u32x4 v[kPer];
    int d[kPer];  // LDS byte offset in the stage, -1: nothing
};

// Resize positions of a tile's lines and span positions into ql / qs, the
// boxes of the image's first tile.  Readers need a barrier.
template <int TL, int TS>
__device__ __forceinline__ void tile_positions(const miaug_ragged_args &a, const Tile &t, int32_t *ql, int32_t *qs) {
    if (t.empty) return;
    const int tid = threadIdx.x;
    const int OL = t.swap ? a.out_w : a.out_h, OS = t.swap ? a.out_h : a.out_w;
    const int l0 = t.swap ? t.i0 : t.j0, s0 = t.swap ? t.j0 : t.i0;
    if (tid < t.nl) ql[tid] = resize_q(l0 + tid, t.Ll, OL);
    if (tid >= 64 && tid - 64 < t.ns) qs[tid - 64] = resize_q(s0 + tid - 64, t.Ls, OS);
    if (t.tile == 0 && a.boxes) ragged_boxes(a, t.img);
}

// Source column spans of a tile from its span positions (uniform).
template <int TL, int TS>
__device__ __forceinline__ void tile_span(const miaug_ragged_args &a, Tile &t, const int32_t *qs) {
    using C = Cfg<TL, TS>;
    if (t.empty) {
        t.staged = false;
        return;
    }
    const D4Map &m = t.m;
    const int32_t qs_first = qs[0], qs_last = qs[t.ns - 1];
    const int dlo = clampi(qs_first >> kFBits, t.Ls), dhi = clampi((qs_last >> kFBits) + 1, t.Ls);
    const int xa = t.ks * dlo + m.cx, xb = t.ks * dhi + m.cx;
    t.sxlo = min(xa, xb);
    t.nsx = abs(xb - xa) + 1;
    const int nlo = clampi((qs_first + kFOne / 2) >> kFBits, t.Ls), nhi = clampi((qs_last + kFOne / 2) >> kFBits, t.Ls);
    const int mxa = t.ks * nlo + m.cx, mxb = t.ks * nhi + m.cx;
    t.mxlo = min(mxa, mxb);
    t.nmx = abs(mxb - mxa) + 1;
    t.staged = t.nsx <= C::kMaxSpanPx;
    t.nchi = (t.nsx * 3 + 30) >> 4;
    t.nchm = a.mask ? (t.nmx + 30) >> 4 : 0;
    t.img_items = 2 * t.nl * t.nchi;
}

// Issues the 16-byte loads of a staged tile into registers (item it -> LDS
// byte 16*it, the same layout as the DMA path).
template <int TL, int TS>
__device__ __forceinline__ void tile_loads(const miaug_ragged_args &a, const Tile &t, const int32_t *ql,
                                           Prefetch<TL, TS> &pf) {
    const int tid = threadIdx.x;
    const bool on = !t.empty && t.staged;
    const int total = on ? t.img_items + t.nl * t.nchm : 0;
    const uint32_t inv_i = on ? ((1u << 20) + t.nchi - 1) / t.nchi : 0;
    const uint32_t inv_m = t.nchm ? ((1u << 20) + t.nchm - 1) / t.nchm : 0;
    const uint8_t *ibase = a.img + (on ? a.img_off[t.img] : 0);
    const uint8_t *mbase = (on && a.mask) ? a.mask + a.mask_off[t.img] : nullptr;
    const D4Map &m = t.m;
#pragma unroll
    for (int u = 0; u < Prefetch<TL, TS>::kPer; ++u) {
        const int it = tid + u * kThreads;
        pf.d[u] = -1;
        if (it < total) {
            const uint8_t *g;
            int len, ch;
            if (it < t.img_items) {
                const int slot = (int)(((uint32_t)it * inv_i) >> 20);
                ch = it - slot * t.nchi;
                const int d = clampi((ql[slot >> 1] >> kFBits) + (slot & 1), t.Ll);
                g = ibase + (uint32_t)(((t.kl * d + m.cy) * t.W + t.sxlo) * 3);
                len = t.nsx * 3;
            } else {
                const int it2 = it - t.img_items, slot = (int)(((uint32_t)it2 * inv_m) >> 20);
                ch = it2 - slot * t.nchm;
                const int d = clampi((ql[slot] + kFOne / 2) >> kFBits, t.Ll);
                g = mbase + (uint32_t)((t.kl * d + m.cy) * t.W + t.mxlo);
                len = t.nmx;
            }
            if (ch < span_chunks(g, len)) {
                pf.v[u] = *(const u32x4 *)((const uint8_t *)((uintptr_t)g & ~(uintptr_t)15) + 16 * ch);
                pf.d[u] = 16 * it;
            }
        }
    }
}

// Writes the prefetched registers to the stage and builds the tile's tables
// and brightness/contrast LUT.  Readers need a barrier.
template <int TL, int TS>
__device__ __forceinline__ void tile_commit(const miaug_ragged_args &a, const Tile &t, const Prefetch<TL, TS> &pf,
                                            const int32_t *ql, const int32_t *qs, Smem<TL, TS, 1> &S, int &lut_img) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int u = 0; u < Prefetch<TL, TS>::kPer; ++u)
        if (pf.d[u] >= 0) *(u32x4 *)(S.stage[0] + pf.d[u]) = pf.v[u];
    if (t.empty) return;
    if (lut_img != t.img) {
        if (tid < 256) {
            const double v = (double)a.ab[2 * t.img] * (double)tid + (double)a.ab[2 * t.img + 1];
            S.bclut[0][tid] = (uint8_t)sat8((int)rint(v));
        }
        lut_img = t.img;
    }
    // positions for the fallback path, tables for the staged path
    if (tid < t.nl) S.qline[0][tid] = ql[tid];
    if (tid >= 64 && tid - 64 < t.ns) S.qspan[0][tid - 64] = qs[tid - 64];
    if (!t.staged) return;
    const D4Map &m = t.m;
    const uint8_t *ibase = a.img + a.img_off[t.img];
    const uint8_t *mbase = a.mask ? a.mask + a.mask_off[t.img] : nullptr;
    if (tid < t.nl) {
        const int q = ql[tid];
        const int d0 = clampi(q >> kFBits, t.Ll), d1 = clampi((q >> kFBits) + 1, t.Ll);
        const uint8_t *g0 = ibase + (uint32_t)(((t.kl * d0 + m.cy) * t.W + t.sxlo) * 3);
        const uint8_t *g1 = ibase + (uint32_t)(((t.kl * d1 + m.cy) * t.W + t.sxlo) * 3);
        int mb = 0;
        if (mbase) {
            const int dn = clampi((q + kFOne / 2) >> kFBits, t.Ll);
            mb = 16 * (t.img_items + tid * t.nchm) + span_phase(mbase + (uint32_t)((t.kl * dn + m.cy) * t.W + t.mxlo));
        }
        S.line[0][tid] = make_int4(16 * (2 * tid) * t.nchi + span_phase(g0),
                                   16 * (2 * tid + 1) * t.nchi + span_phase(g1), q & (kFOne - 1), mb);
    }
    if (tid >= 64 && tid - 64 < t.ns) {
        const int si = tid - 64, q = qs[si];
        const int e0 = clampi(q >> kFBits, t.Ls), e1 = clampi((q >> kFBits) + 1, t.Ls);
        const int en = clampi((q + kFOne / 2) >> kFBits, t.Ls);
        S.col[0][si] = make_int4(3 * (t.ks * e0 + m.cx - t.sxlo), 3 * (t.ks * e1 + m.cx - t.sxlo),
                                 q & (kFOne - 1), t.ks * en + m.cx - t.mxlo);
    }
}

template <int TL, int TS>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_ragged_prefetch(miaug_ragged_args a, int *__restrict__ counters) {
    __shared__ Smem<TL, TS, 1> S;
    __shared__ int32_t pql[2][TL], pqs[2][TS];  // positions of the prefetched tile (alternating)
    const int tiles = tiles_per_image<TL, TS>(a.out_h, a.out_w);
    build_norm_lut(a, S);
    int lut_img = -1;
    int q = blockIdx.x % kQueues, tries = 0;  // thread 0 only
    if (threadIdx.x == 0) {
        S.item[0] = pop_item(a, counters, tiles, q, tries);
        S.item[1] = pop_item(a, counters, tiles, q, tries);
    }
    __syncthreads();
    int nxt = S.item[0], after = S.item[1];
    if (nxt < 0) return;
    Prefetch<TL, TS> pf;
    Tile tn = tile_geometry<TL, TS>(a, nxt / tiles, nxt % tiles);
    tile_positions<TL, TS>(a, tn, pql[0], pqs[0]);
    __syncthreads();
    tile_span<TL, TS>(a, tn, pqs[0]);
    tile_loads<TL, TS>(a, tn, pql[0], pf);
    int pb = 0;      // position buffer of the prefetched tile
    int slot = 2;    // item ring slot the next pop writes
    for (;;) {
        // the prefetched tile becomes current
        const Tile tc = tn;
        tile_commit<TL, TS>(a, tc, pf, pql[pb], pqs[pb], S, lut_img);
        const int cur_next = after;
        if (cur_next >= 0) {
            if (threadIdx.x == 0) S.item[slot] = pop_item(a, counters, tiles, q, tries);
            tn = tile_geometry<TL, TS>(a, cur_next / tiles, cur_next % tiles);
            tile_positions<TL, TS>(a, tn, pql[pb ^ 1], pqs[pb ^ 1]);
        }
        __syncthreads();  // stage, tables, LUT of tc; positions of tn; S.item[slot]
        if (cur_next >= 0) {
            after = S.item[slot];
            slot = (slot + 1) & 3;
            tile_span<TL, TS>(a, tn, pqs[pb ^ 1]);
            tile_loads<TL, TS>(a, tn, pql[pb ^ 1], pf);
        }
        compute_tile<TL, TS, 1>(a, tc, 0, S);
        if (cur_next < 0) break;
        pb ^= 1;
        __syncthreads();  // every thread is done reading the stage before it is overwritten
    }
}

// Persistent form, not pipelined: one item at a time.
template <int TL, int TS>
__global__ __launch_bounds__(kThreads) void k_ragged_persistent(miaug_ragged_args a, int *__restrict__ counters) {
    __shared__ Smem<TL, TS, 1> S;
    const int tiles = tiles_per_image<TL, TS>(a.out_h, a.out_w);
    build_norm_lut(a, S);
    int lut_img = -1;
    int q = blockIdx.x % kQueues, tries = 0;  // thread 0 only
    for (;;) {
        if (threadIdx.x == 0) S.item[0] = pop_item(a, counters, tiles, q, tries);
        __syncthreads();
        const int item = S.item[0];
        if (item < 0) break;
        run_tile<TL, TS, 1>(a, item / tiles, item % tiles, S, lut_img);
        __syncthreads();
    }
}

// Persistent, software-pipelined form: while tile k is blended from LDS
// buffer k mod 2, the rows of tile k+1 are already streaming into the other
// buffer and the index of tile k+2 is being fetched, so the HBM and atomic
// latencies of one item hide behind the arithmetic of the previous one.
template <int TL, int TS>
__global__ __launch_bounds__(kThreads) void k_ragged_pipe(miaug_ragged_args a, int *__restrict__ counters) {
    __shared__ Smem<TL, TS, 2> S;
    const int tiles = tiles_per_image<TL, TS>(a.out_h, a.out_w);
    build_norm_lut(a, S);
    int lut0 = -1, lut1 = -1;  // image whose brightness/contrast LUT sits in buffer 0 / 1
    int q = blockIdx.x % kQueues, tries = 0;  // thread 0 only
    if (threadIdx.x == 0) {
        S.item[0] = pop_item(a, counters, tiles, q, tries);
        S.item[1] = pop_item(a, counters, tiles, q, tries);
    }
    __syncthreads();
    int cur = S.item[0], nxt = S.item[1];
    if (cur < 0) return;
    Tile tc = tile_geometry<TL, TS>(a, cur / tiles, cur % tiles);
    prepare_tile<TL, TS, 2>(a, tc, 0, S, lut0);
    int b = 0;
    for (;;) {
        __builtin_amdgcn_s_waitcnt(0);  // tile `cur` is in buffer b (LDS-DMA counted by vmcnt)
        __syncthreads();
        Tile tn = tc;
        if (nxt >= 0) {
            if (threadIdx.x == 0) S.item[2] = pop_item(a, counters, tiles, q, tries);
            tn = tile_geometry<TL, TS>(a, nxt / tiles, nxt % tiles);
            int li = b ? lut0 : lut1;
            prepare_tile<TL, TS, 2>(a, tn, b ^ 1, S, li);  // its barrier publishes S.item[2]
            if (b) lut0 = li; else lut1 = li;
        }
        compute_tile<TL, TS, 2>(a, tc, b, S);
        if (nxt < 0) break;
        const int nn = S.item[2];
        cur = nxt;
        nxt = nn;
        tc = tn;
        b ^= 1;
    }
}

// Flat grid: one workgroup per item, XCD-aware: workgroup b runs on XCD b mod 8
// and takes item b / 8 of queue b mod 8.
template <int TL, int TS>
__global__ __launch_bounds__(kThreads) void k_ragged_flat(miaug_ragged_args a) {
    __shared__ Smem<TL, TS, 1> S;
    const int tiles = tiles_per_image<TL, TS>(a.out_h, a.out_w);
    const int q = blockIdx.x % kQueues, idx = blockIdx.x / kQueues;
    const int img = (idx / tiles) * kQueues + q;
    if (img >= a.n) return;
    build_norm_lut(a, S);
    int lut_img = -1;
    run_tile<TL, TS, 1>(a, img, idx % tiles, S, lut_img);
}

// One image per launch (the comparison form): workgroup b = tile b.
template <int TL, int TS>
__global__ __launch_bounds__(kThreads) void k_ragged_one(miaug_ragged_args a, int img) {
    __shared__ Smem<TL, TS, 1> S;
    build_norm_lut(a, S);
    int lut_img = -1;
    run_tile<TL, TS, 1>(a, img, blockIdx.x, S, lut_img);
}

__global__ void k_zero_counters(int *counters, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) counters[i] = 0;
}

struct Variant {
    int tl, ts;     // lines x span positions per tile
    int mode;       // 0 persistent, 1 persistent pipelined (LDS-DMA), 2 flat grid, 3 persistent register prefetch
    int wg_per_cu;  // workgroups per CU of the persistent modes
    const char *name;
};
const Variant kVariants[] = {
    {32, 32, 3, 4, "tile 32x32, register-prefetch persistent 4 wg/CU"},
    {32, 32, 0, 4, "tile 32x32, persistent 4 wg/CU"},
    {32, 32, 2, 0, "tile 32x32, flat grid"},
    {16, 32, 3, 7, "tile 16x32, register-prefetch persistent 7 wg/CU"},
    {16, 32, 0, 8, "tile 16x32, persistent 8 wg/CU"},
    {16, 32, 2, 0, "tile 16x32, flat grid"},
    {32, 32, 1, 2, "tile 32x32, LDS-DMA double-buffered persistent 2 wg/CU"},
    {16, 16, 2, 0, "tile 16x16, flat grid"},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <int TL, int TS>
hipError_t launch_t(const miaug_ragged_args *a, const Variant &v, const RaggedLaunch &L, int per_image,
                    hipStream_t s) {
    const int tiles = tiles_per_image<TL, TS>(a->out_h, a->out_w);
    if (per_image) {
        for (int i = 0; i < a->n; ++i) {
            hipLaunchKernelGGL((k_ragged_one<TL, TS>), dim3(tiles), dim3(kThreads), 0, s, *a, i);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    if (v.mode == 2) {
        const int per_q = (a->n + kQueues - 1) / kQueues;
        hipLaunchKernelGGL((k_ragged_flat<TL, TS>), dim3(kQueues * per_q * tiles), dim3(kThreads), 0, s, *a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(256), 0, s, L.counters, kQueues * kCounterStride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int grid = L.num_cu * v.wg_per_cu;
    const long items = (long)a->n * tiles;
    if (grid > items) grid = (int)items;
    grid = ((grid + kQueues - 1) / kQueues) * kQueues;
    if (v.mode == 1)
        hipLaunchKernelGGL((k_ragged_pipe<TL, TS>), dim3(grid), dim3(kThreads), 0, s, *a, L.counters);
    else if (v.mode == 3)
        hipLaunchKernelGGL((k_ragged_prefetch<TL, TS>), dim3(grid), dim3(kThreads), 0, s, *a, L.counters);
    else
        hipLaunchKernelGGL((k_ragged_persistent<TL, TS>), dim3(grid), dim3(kThreads), 0, s, *a, L.counters);
    return hipGetLastError();
}

}  // namespace

int ragged_variant_count() { return kNumVariants; }
const char *ragged_variant_name(int v) { return (v >= 0 && v < kNumVariants) ? kVariants[v].name : nullptr; }
int ragged_default_variant() { return 0; }

hipError_t launch_ragged(const miaug_ragged_args *a, const RaggedLaunch &L, int per_image, hipStream_t s) {
    if (a->n == 0) return hipSuccess;
    const Variant &v = kVariants[(L.variant >= 0 && L.variant < kNumVariants) ? L.variant : 0];
    if (v.tl == 32) return launch_t<32, 32>(a, v, L, per_image, s);
    if (v.ts == 16) return launch_t<16, 16>(a, v, L, per_image, s);
    return launch_t<16, 32>(a, v, L, per_image, s);
}

}  // namespace miaug
