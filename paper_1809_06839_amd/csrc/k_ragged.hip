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

template <int T>
struct Cfg {
    static constexpr int kMaxSpanPx = (T - 1) * 46 / 10 + 4;       // staged span: scale factors up to 4.6
    static constexpr int kChunks = (kMaxSpanPx * 3 + 30) / 16;      // 16-byte chunks per image slot
    static constexpr int kStride = kChunks * 16;
    static constexpr int kMChunks = (kMaxSpanPx + 30) / 16;
    static constexpr int kMStride = kMChunks * 16;
    static constexpr int kPix = (T * T + kThreads - 1) / kThreads;  // output pixels per thread
};

template <int T>
struct __align__(16) Smem {
    // staging buffer: image slot s at byte 16*s*nchi, mask slot s at byte
    // 16*(2*nl*nchi + s*nchm) (nchi, nchm: 16-byte chunks per slot of the tile)
    uint8_t stage[2 * T * Cfg<T>::kStride + T * Cfg<T>::kMStride];
    float nlut[3][256];
    int32_t qline[T], qspan[T];
    int4 line[T];  // per output line: LDS offsets of the two tap rows and the nearest mask row, weight
    int4 col[T];   // per span position: byte offsets of the two taps in a row, weight, mask offset
    uint8_t bclut[256];
    int item;
};

template <int T>
__device__ __forceinline__ void build_norm_lut(const miaug_ragged_args &a, Smem<T> &S) {
    for (int e = threadIdx.x; e < 3 * 256; e += kThreads) {
        int c = e >> 8, v = e & 255;
        S.nlut[c][v] = (float)((((double)v / 255.0) - (double)a.mean[c]) / (double)a.stdv[c]);
    }
}

template <int T>
__device__ __forceinline__ void build_bc_lut(const miaug_ragged_args &a, int img, Smem<T> &S) {
    int v = threadIdx.x;
    if (v < 256) {
        double t = (double)a.ab[2 * img] * (double)v + (double)a.ab[2 * img + 1];
        S.bclut[v] = (uint8_t)sat8((int)rint(t));
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

// One (image, tile) work item.  Contains two __syncthreads; callers must
// synchronise before LDS is reused.  `lut_img` is the image whose
// brightness/contrast LUT is currently in LDS (-1: none).
template <int T>
__device__ __forceinline__ void ragged_tile(const miaug_ragged_args &a, int img, int tile, Smem<T> &S, int &lut_img) {
    using C = Cfg<T>;
    const int tid = threadIdx.x;
    const int H = a.hw[2 * img], W = a.hw[2 * img + 1];
    if (H < 1 || W < 1) return;  // empty image: nothing to read, outputs left untouched (uniform per block)
    const int32_t *fl = a.flags + 4 * img;
    const D4Map m = make_d4(H, W, fl[0], fl[1], fl[2], fl[3]);
    const bool swap = m.swaps();
    const int OH = a.out_h, OW = a.out_w;
    const int tiles_x = (OW + T - 1) / T;
    const int j0 = (tile / tiles_x) * T, i0 = (tile % tiles_x) * T;
    const int th = min(T, OH - j0), tw = min(T, OW - i0);
    // line axis: its taps select source rows; span axis: contiguous source columns
    const int nl = swap ? tw : th, ns = swap ? th : tw;
    const int l0 = swap ? i0 : j0, s0 = swap ? j0 : i0;
    const int Ll = swap ? m.ow : m.oh, Ls = swap ? m.oh : m.ow;
    const int OL = swap ? OW : OH, OS = swap ? OH : OW;
    const int kl = swap ? m.by : m.ay, ks = swap ? m.ax : m.bx;

    if (lut_img != img) {
        build_bc_lut(a, img, S);
        lut_img = img;
    }
    if (tid < nl) S.qline[tid] = resize_q(l0 + tid, Ll, OL);
    if (tid >= 64 && tid - 64 < ns) S.qspan[tid - 64] = resize_q(s0 + tid - 64, Ls, OS);
    const uint8_t *ibase = a.img + a.img_off[img];
    const uint8_t *mbase = a.mask ? a.mask + a.mask_off[img] : nullptr;
    if (tile == 0 && a.boxes) ragged_boxes(a, img);
    __syncthreads();

    // source column span of the tile (bilinear taps) and of its nearest taps
    const int32_t qs_first = S.qspan[0], qs_last = S.qspan[ns - 1];
    const int dlo = clampi(qs_first >> kFBits, Ls), dhi = clampi((qs_last >> kFBits) + 1, Ls);
    const int xa = ks * dlo + m.cx, xb = ks * dhi + m.cx;
    const int sxlo = min(xa, xb), nsx = abs(xb - xa) + 1;
    const int nlo = clampi((qs_first + kFOne / 2) >> kFBits, Ls), nhi = clampi((qs_last + kFOne / 2) >> kFBits, Ls);
    const int mxa = ks * nlo + m.cx, mxb = ks * nhi + m.cx;
    const int mxlo = min(mxa, mxb), nmx = abs(mxb - mxa) + 1;
    const bool staged = nsx <= C::kMaxSpanPx;

    // Staging: item `it` (a 16-byte chunk of an image or mask slot) is copied
    // straight from HBM to LDS byte 16*it with global_load_lds_dwordx4.  The 64
    // lanes of a wave take 64 consecutive items, which is the DMA's lane layout
    // (LDS base in M0 + 16 * lane), so no registers hold the data and a
    // workgroup has its whole footprint in flight at once.
    const int nchi = (nsx * 3 + 30) >> 4, nchm = mbase ? (nmx + 30) >> 4 : 0;
    const int img_items = 2 * nl * nchi, total = img_items + nl * nchm;
    const size_t plane = (size_t)OH * OW;
    if (staged) {
        const uint32_t inv_i = ((1u << 20) + nchi - 1) / nchi;            // it / nchi = (it * inv) >> 20
        const uint32_t inv_m = nchm ? ((1u << 20) + nchm - 1) / nchm : 0;  // (exact for it < 4096)
        const int lane = tid & 63;
        for (int base = tid - lane; base < total; base += kThreads) {
            const int it = base + lane;
            const uint8_t *src = nullptr;
            if (it < total) {
                const uint8_t *g;
                int len, ch;
                if (it < img_items) {
                    const int slot = (int)(((uint32_t)it * inv_i) >> 20);
                    ch = it - slot * nchi;
                    const int d = clampi((S.qline[slot >> 1] >> kFBits) + (slot & 1), Ll);
                    g = ibase + ((size_t)(kl * d + m.cy) * W + sxlo) * 3;
                    len = nsx * 3;
                } else {
                    const int it2 = it - img_items, slot = (int)(((uint32_t)it2 * inv_m) >> 20);
                    ch = it2 - slot * nchm;
                    const int d = clampi((S.qline[slot] + kFOne / 2) >> kFBits, Ll);
                    g = mbase + (size_t)(kl * d + m.cy) * W + mxlo;
                    len = nmx;
                }
                if (ch < span_chunks(g, len)) src = (const uint8_t *)((uintptr_t)g & ~(uintptr_t)15) + 16 * ch;
            }
            if (src)
                __builtin_amdgcn_global_load_lds((const void *)src, (lds_ptr_t)(S.stage + 16 * base), 16, 0, 0);
        }
        // per-line and per-column tables (the same addresses, from the registers of phase A)
        if (tid < nl) {
            const int q = S.qline[tid];
            const int d0 = clampi(q >> kFBits, Ll), d1 = clampi((q >> kFBits) + 1, Ll);
            const uint8_t *g0 = ibase + ((size_t)(kl * d0 + m.cy) * W + sxlo) * 3;
            const uint8_t *g1 = ibase + ((size_t)(kl * d1 + m.cy) * W + sxlo) * 3;
            int mb = 0;
            if (mbase) {
                const int dn = clampi((q + kFOne / 2) >> kFBits, Ll);
                mb = 16 * (img_items + tid * nchm) + span_phase(mbase + (size_t)(kl * dn + m.cy) * W + mxlo);
            }
            S.line[tid] = make_int4(16 * (2 * tid) * nchi + span_phase(g0), 16 * (2 * tid + 1) * nchi + span_phase(g1),
                                    q & (kFOne - 1), mb);
        }
        if (tid >= 64 && tid - 64 < ns) {
            const int si = tid - 64, q = S.qspan[si];
            const int e0 = clampi(q >> kFBits, Ls), e1 = clampi((q >> kFBits) + 1, Ls);
            const int en = clampi((q + kFOne / 2) >> kFBits, Ls);
            S.col[si] = make_int4(3 * (ks * e0 + m.cx - sxlo), 3 * (ks * e1 + m.cx - sxlo), q & (kFOne - 1),
                                  ks * en + m.cx - mxlo);
        }
        __builtin_amdgcn_s_waitcnt(0);  // LDS-DMA writes are counted by vmcnt
        __syncthreads();

#pragma unroll
        for (int k = 0; k < C::kPix; ++k) {
            const int p = tid + k * kThreads;
            const int jj = p / T, ii = p - jj * T;
            if (p >= T * T || jj >= th || ii >= tw) continue;
            const int4 L = S.line[swap ? ii : jj];
            const int4 Cc = S.col[swap ? jj : ii];
            const uint8_t *r0 = S.stage + L.x, *r1 = S.stage + L.y;
            const int wl1 = L.z, ws1 = Cc.z;
            float *o = a.out + (size_t)img * 3 * plane + (size_t)(j0 + jj) * OW + (i0 + ii);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int p00 = S.bclut[r0[Cc.x + c]], p01 = S.bclut[r0[Cc.y + c]];
                const int p10 = S.bclut[r1[Cc.x + c]], p11 = S.bclut[r1[Cc.y + c]];
                // (1024-ws1) p00 + ws1 p01 = 1024 p00 + ws1 (p01 - p00), exactly; same for rows
                const int t0 = (p00 << kFBits) + ws1 * (p01 - p00);
                const int t1 = (p10 << kFBits) + ws1 * (p11 - p10);
                o[c * plane] = S.nlut[c][rhe20((t0 << kFBits) + wl1 * (t1 - t0))];
            }
            if (mbase) a.out_mask[(size_t)img * plane + (size_t)(j0 + jj) * OW + (i0 + ii)] = S.stage[L.w + Cc.w];
        }
        return;
    }

    // Fallback for spans wider than the staging buffer (source more than 4.6x
    // the output along the span axis): the same arithmetic on direct loads.
    __syncthreads();
#pragma unroll
    for (int k = 0; k < C::kPix; ++k) {
        const int p = tid + k * kThreads;
        const int jj = p / T, ii = p - jj * T;
        if (p >= T * T || jj >= th || ii >= tw) continue;
        const int l = swap ? ii : jj, si = swap ? jj : ii;
        const int32_t ql = S.qline[l], qs = S.qspan[si];
        const int wl1 = ql & (kFOne - 1), ws1 = qs & (kFOne - 1);
        const int x0 = ks * clampi(qs >> kFBits, Ls) + m.cx, x1 = ks * clampi((qs >> kFBits) + 1, Ls) + m.cx;
        const int y0 = kl * clampi(ql >> kFBits, Ll) + m.cy, y1 = kl * clampi((ql >> kFBits) + 1, Ll) + m.cy;
        const uint8_t *r0 = ibase + (size_t)y0 * W * 3, *r1 = ibase + (size_t)y1 * W * 3;
        float *o = a.out + (size_t)img * 3 * plane + (size_t)(j0 + jj) * OW + (i0 + ii);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int p00 = S.bclut[r0[3 * x0 + c]], p01 = S.bclut[r0[3 * x1 + c]];
            const int p10 = S.bclut[r1[3 * x0 + c]], p11 = S.bclut[r1[3 * x1 + c]];
            const int t0 = (p00 << kFBits) + ws1 * (p01 - p00);
            const int t1 = (p10 << kFBits) + ws1 * (p11 - p10);
            o[c * plane] = S.nlut[c][rhe20((t0 << kFBits) + wl1 * (t1 - t0))];
        }
        if (mbase) {
            const int mx = ks * clampi((qs + kFOne / 2) >> kFBits, Ls) + m.cx;
            const int my = kl * clampi((ql + kFOne / 2) >> kFBits, Ll) + m.cy;
            a.out_mask[(size_t)img * plane + (size_t)(j0 + jj) * OW + (i0 + ii)] = mbase[(size_t)my * W + mx];
        }
    }
}

template <int T>
__global__ __launch_bounds__(kThreads) void k_ragged_persistent(miaug_ragged_args a, int *__restrict__ counters) {
    __shared__ Smem<T> S;
    const int tiles = ((a.out_h + T - 1) / T) * ((a.out_w + T - 1) / T);
    build_norm_lut(a, S);
    int lut_img = -1;
    int q = blockIdx.x % kQueues, tries = 0;  // thread 0 only
    for (;;) {
        if (threadIdx.x == 0) {
            int item = -1;
            while (tries < kQueues) {
                const int nq = (a.n - q + kQueues - 1) / kQueues;  // images i with i mod 8 == q
                const int idx = atomicAdd(&counters[q * kCounterStride], 1);
                if (idx < nq * tiles) {
                    item = ((idx / tiles) * kQueues + q) * tiles + idx % tiles;
                    break;
                }
                q = (q + 1) % kQueues;
                ++tries;
            }
            S.item = item;
        }
        __syncthreads();
        const int item = S.item;
        if (item < 0) break;
        ragged_tile<T>(a, item / tiles, item % tiles, S, lut_img);
        __syncthreads();
    }
}

// Flat grid: one workgroup per item, XCD-aware: workgroup b runs on XCD b mod 8
// and takes item b / 8 of queue b mod 8.
template <int T>
__global__ __launch_bounds__(kThreads) void k_ragged_flat(miaug_ragged_args a) {
    __shared__ Smem<T> S;
    const int tiles = ((a.out_h + T - 1) / T) * ((a.out_w + T - 1) / T);
    const int q = blockIdx.x % kQueues, idx = blockIdx.x / kQueues;
    const int img = (idx / tiles) * kQueues + q;
    if (img >= a.n) return;
    build_norm_lut(a, S);
    int lut_img = -1;
    ragged_tile<T>(a, img, idx % tiles, S, lut_img);
}

// One image per launch (the comparison form): workgroup b = tile b.
template <int T>
__global__ __launch_bounds__(kThreads) void k_ragged_one(miaug_ragged_args a, int img) {
    __shared__ Smem<T> S;
    build_norm_lut(a, S);
    int lut_img = -1;
    ragged_tile<T>(a, img, blockIdx.x, S, lut_img);
}

__global__ void k_zero_counters(int *counters, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) counters[i] = 0;
}

struct Variant {
    int tile;       // 16 or 32
    int wg_per_cu;  // persistent workgroups per CU; 0 = flat grid
    const char *name;
};
const Variant kVariants[] = {
    {32, 4, "tile 32x32, persistent 4 wg/CU"}, {32, 2, "tile 32x32, persistent 2 wg/CU"},
    {32, 8, "tile 32x32, persistent 8 wg/CU"}, {32, 0, "tile 32x32, flat grid"},
    {16, 4, "tile 16x16, persistent 4 wg/CU"}, {16, 8, "tile 16x16, persistent 8 wg/CU"},
    {16, 16, "tile 16x16, persistent 16 wg/CU"}, {16, 0, "tile 16x16, flat grid"},
};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <int T>
hipError_t launch_t(const miaug_ragged_args *a, const Variant &v, const RaggedLaunch &L, int per_image,
                    hipStream_t s) {
    const int tiles = ((a->out_h + T - 1) / T) * ((a->out_w + T - 1) / T);
    if (per_image) {
        for (int i = 0; i < a->n; ++i) {
            hipLaunchKernelGGL(k_ragged_one<T>, dim3(tiles), dim3(kThreads), 0, s, *a, i);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    if (v.wg_per_cu == 0) {
        const int per_q = (a->n + kQueues - 1) / kQueues;
        hipLaunchKernelGGL(k_ragged_flat<T>, dim3(kQueues * per_q * tiles), dim3(kThreads), 0, s, *a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(256), 0, s, L.counters, kQueues * kCounterStride);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int grid = L.num_cu * v.wg_per_cu;
    const long items = (long)a->n * tiles;
    if (grid > items) grid = (int)items;
    grid = ((grid + kQueues - 1) / kQueues) * kQueues;
    hipLaunchKernelGGL(k_ragged_persistent<T>, dim3(grid), dim3(kThreads), 0, s, *a, L.counters);
    return hipGetLastError();
}

}  // namespace

int ragged_variant_count() { return kNumVariants; }
const char *ragged_variant_name(int v) { return (v >= 0 && v < kNumVariants) ? kVariants[v].name : nullptr; }
int ragged_default_variant() { return 0; }

hipError_t launch_ragged(const miaug_ragged_args *a, const RaggedLaunch &L, int per_image, hipStream_t s) {
    if (a->n == 0) return hipSuccess;
    const Variant &v = kVariants[(L.variant >= 0 && L.variant < kNumVariants) ? L.variant : 0];
    return v.tile == 32 ? launch_t<32>(a, v, L, per_image, s) : launch_t<16>(a, v, L, per_image, s);
}

}  // namespace miaug
