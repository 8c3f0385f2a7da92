// api.cpp -- the C ABI of libmiaug: argument validation, contexts, graphs
// and the ragged-batch autotuner.  Every image operation is
// executed by the HIP kernels behind the launch_* functions.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "internal.h"

using namespace miaug;

struct miaug_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

namespace {

int begin_call() {
    clear_error();
    return MIAUG_OK;
}

// Launch variant of a context: MIAUG_FORCE_VARIANT when set and in range.
int ctx_variant(const miaug_ctx *c) {
    const int f = env().force_variant;
    return ragged_variant_enabled(f) ? f : c->variant;
}

// Bookkeeping of a context call whose arguments were accepted; returns st.
// (Argument errors return before it: a context pointer is only trusted once
// the rest of the call checks out.)
int ctx_done(miaug_ctx *c, int st) {
    if (c) {
        c->stats.calls++;
        c->stats.last_status = st;
        if (st < 0) c->stats.errors++;
    }
    if (st < 0) log_msg(1, "error %d: %s", st, miaug_last_error());
    return st;
}

// Status of a ragged argument block (sizes of each image are validated on
// the device side only through clamping; H, W must be >= 1 by contract).
int ragged_check(const miaug_ragged_args *a) {
    if (!a) return set_error(MIAUG_EINVAL, "ragged: args is NULL");
    if (a->n < 0) return set_error(MIAUG_EINVAL, "ragged: n < 0");
    if (a->out_h < 1 || a->out_w < 1 || a->out_h > 4096 || a->out_w > 4096)
        return set_error(MIAUG_ESHAPE, "ragged: output size %dx%d outside 1..4096", a->out_h, a->out_w);
    if (a->n == 0) return MIAUG_OK;
    if (!a->img || !a->img_off || !a->hw || !a->flags || !a->ab || !a->out)
        return set_error(MIAUG_EINVAL, "ragged: a required pointer is NULL");
    if (a->mask && (!a->mask_off || !a->out_mask)) return set_error(MIAUG_EINVAL, "ragged: mask without offsets/output");
    if (a->boxes && (!a->box_off || !a->out_boxes)) return set_error(MIAUG_EINVAL, "ragged: boxes without offsets/output");
    for (int c = 0; c < 3; ++c)
        if (!(a->stdv[c] != 0.0f)) return set_error(MIAUG_EINVAL, "ragged: std[%d] is zero", c);
    return MIAUG_OK;
}

}  // namespace

extern "C" {


int miaug_ctx_create(int device, const char *tune_cache_path, miaug_ctx **out) {
    begin_call();
    if (!out) return set_error(MIAUG_EINVAL, "ctx_create: out is NULL");
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return set_error(MIAUG_EDEVICE, "ctx_create: no HIP device");
    if (device < 0 || device >= ndev) return set_error(MIAUG_EINVAL, "ctx_create: device %d of %d", device, ndev);
    int prev = 0;
    hipGetDevice(&prev);
    int st = hip_status(hipSetDevice(device), "hipSetDevice");
    if (st) return st;
    hipDeviceProp_t prop;
    st = hip_status(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    miaug_ctx *c = nullptr;
    if (!st) {
        c = new (std::nothrow) miaug_ctx();
        if (!c) st = set_error(MIAUG_ENOMEM, "ctx_create: host allocation");
    }
    if (!st) {
        c->device = device;
        c->num_cu = prop.multiProcessorCount;
        c->variant = ragged_default_variant();
        c->counters = nullptr;
        c->arch = prop.gcnArchName;
        c->tune_cache = tune_cache_path ? tune_cache_path : env().tune_cache;
        memset(&c->stats, 0, sizeof(c->stats));
        st = dev_alloc((void **)&c->counters, (256 + kLptMax) * sizeof(int), "ctx_create: queue counters");
        if (!st) st = hip_status(hipMemset(c->counters, 0, (256 + kLptMax) * sizeof(int)), "hipMemset counters");
    }
    hipSetDevice(prev);
    if (st) {
        if (c && c->counters) hipFree(c->counters);
        delete c;
        return st;
    }
    log_msg(2, "context on device %d (%s, %d CUs), tune cache %s", device, c->arch.c_str(), c->num_cu,
         c->tune_cache.empty() ? "(none)" : c->tune_cache.c_str());
    *out = c;
    return MIAUG_OK;
}

int miaug_ctx_destroy(miaug_ctx *c) {
    begin_call();
    if (!c) return MIAUG_OK;
    if (c->counters) hipFree(c->counters);
    delete c;
    return MIAUG_OK;
}

int miaug_ctx_stats(const miaug_ctx *c, miaug_stats *out) {
    begin_call();
    if (!c || !out) return set_error(MIAUG_EINVAL, "ctx_stats: NULL pointer");
    *out = c->stats;
    out->variant = ctx_variant(c);
    return MIAUG_OK;
}

int miaug_tune_cache_lookup(const char *path, const char *key, int *variant, float *ms, char *name, size_t name_len) {
    begin_call();
    if (!path || !key) return set_error(MIAUG_EINVAL, "tune_cache_lookup: NULL path or key");
    TuneEntry e;
    const int st = tune_cache_get(path, key, &e);
    if (st == MIAUG_EUNSUPPORTED) return set_error(st, "tune_cache_lookup: %s has no entry %s", path, key);
    if (st) return st;
    if (variant) *variant = e.variant;
    if (ms) *ms = e.ms;
    if (name && name_len) {
        strncpy(name, e.name.c_str(), name_len - 1);
        name[name_len - 1] = 0;
    }
    return MIAUG_OK;
}

int miaug_tune_cache_store(const char *path, const char *key, int variant, const char *name, float ms) {
    begin_call();
    if (!path || !key) return set_error(MIAUG_EINVAL, "tune_cache_store: NULL path or key");
    TuneEntry e;
    e.key = key;
    e.variant = variant;
    e.name = name ? name : "";
    e.ms = ms;
    return tune_cache_put(path, e);
}

int miaug_debug_fail_alloc_after(long after) {
    begin_call();
    arm_alloc_failure(after);
    return MIAUG_OK;
}

int miaug_debug_alloc_probe(size_t bytes) {
    begin_call();
    void *p = nullptr;
    const int st = dev_alloc(&p, bytes, "alloc_probe");
    if (p) hipFree(p);
    return st;
}

int miaug_d4_bc_u8(const uint8_t *in, int n, int H, int W, int C, const int32_t *flags, const float *ab,
                   uint8_t *out, void *stream) {
    begin_call();
    if (n < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "d4_bc_u8: negative size");
    if (C != 1 && C != 3 && C != 4) return set_error(MIAUG_ESHAPE, "d4_bc_u8: C=%d (1, 3 or 4)", C);
    if (n == 0 || H == 0 || W == 0) return MIAUG_OK;
    if (!in || !flags || !ab || !out) return set_error(MIAUG_EINVAL, "d4_bc_u8: NULL pointer");
    if ((long long)H * W * C > (1ll << 31) - 1) return set_error(MIAUG_ESHAPE, "d4_bc_u8: image too large");
    return hip_status(launch_d4_bc_u8(in, n, H, W, C, flags, ab, out, as_stream(stream)), "d4_bc_u8 launch");
}

int miaug_d4_lut_u8(const uint8_t *in, int n, int H, int W, int C, const int32_t *flags, const uint8_t *luts,
                    const int32_t *gray, uint8_t *out, void *stream) {
    begin_call();
    if (n < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "d4_lut_u8: negative size");
    if (C != 1 && C != 3 && C != 4) return set_error(MIAUG_ESHAPE, "d4_lut_u8: C=%d (1, 3 or 4)", C);
    if (gray && C != 3) return set_error(MIAUG_ESHAPE, "d4_lut_u8: grayscale needs C = 3");
    if (n == 0 || H == 0 || W == 0) return MIAUG_OK;
    if (!in || !flags || !luts || !out) return set_error(MIAUG_EINVAL, "d4_lut_u8: NULL pointer");
    if ((long long)H * W * C > (1ll << 31) - 1) return set_error(MIAUG_ESHAPE, "d4_lut_u8: image too large");
    return hip_status(launch_d4_lut_u8(in, n, H, W, C, flags, luts, gray, out, as_stream(stream)), "d4_lut_u8 launch");
}

int miaug_pad_u8(const uint8_t *in, int n, int H, int W, int C, int min_h, int min_w, int border, int value,
                 uint8_t *out, void *stream) {
    begin_call();
    if (n < 0 || H < 1 || W < 1 || min_h < 0 || min_w < 0) return set_error(MIAUG_EINVAL, "pad_u8: bad size");
    if (C != 1 && C != 3 && C != 4) return set_error(MIAUG_ESHAPE, "pad_u8: C=%d (1, 3 or 4)", C);
    if (border != MIAUG_BORDER_REFLECT101 && border != MIAUG_BORDER_CONSTANT)
        return set_error(MIAUG_EINVAL, "pad_u8: border %d", border);
    if (value < 0 || value > 255) return set_error(MIAUG_EINVAL, "pad_u8: value %d", value);
    const int Ho = H > min_h ? H : min_h, Wo = W > min_w ? W : min_w;
    if ((long long)Ho * Wo * C > (1ll << 31) - 1) return set_error(MIAUG_ESHAPE, "pad_u8: output too large");
    if (n == 0) return MIAUG_OK;
    if (!in || !out) return set_error(MIAUG_EINVAL, "pad_u8: NULL pointer");
    return hip_status(launch_pad_u8(in, n, H, W, C, Ho, Wo, border, value, out, as_stream(stream)), "pad_u8 launch");
}

int miaug_blur_u8(const uint8_t *in, int n, int H, int W, int C, int ksize, const int32_t *apply, uint8_t *out,
                  void *stream) {
    begin_call();
    if (n < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "blur_u8: negative size");
    if (C != 1 && C != 3 && C != 4) return set_error(MIAUG_ESHAPE, "blur_u8: C=%d (1, 3 or 4)", C);
    if (ksize != 3 && ksize != 5) return set_error(MIAUG_EINVAL, "blur_u8: ksize %d (3 or 5)", ksize);
    if (H > 65535 || W > 65535) return set_error(MIAUG_ESHAPE, "blur_u8: %dx%d image too large", H, W);
    if (n == 0 || H == 0 || W == 0) return MIAUG_OK;
    if (!in || !out) return set_error(MIAUG_EINVAL, "blur_u8: NULL pointer");
    const size_t bytes = (size_t)n * H * W * C;
    if ((uintptr_t)out < (uintptr_t)in + bytes && (uintptr_t)in < (uintptr_t)out + bytes)
        return set_error(MIAUG_EINVAL, "blur_u8: out overlaps in (tiles read their neighbours)");
    return hip_status(launch_blur_u8(in, n, H, W, C, ksize, apply, out, as_stream(stream)), "blur_u8 launch");
}

int miaug_hsv_shift_u8(const uint8_t *in, int n, int H, int W, const int32_t *dhsv, uint8_t *out, void *stream) {
    begin_call();
    if (n < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "hsv_shift_u8: negative size");
    if ((long long)H * W * 3 > (1ll << 40)) return set_error(MIAUG_ESHAPE, "hsv_shift_u8: image too large");
    if (n == 0 || H == 0 || W == 0) return MIAUG_OK;
    if (!in || !out || !dhsv) return set_error(MIAUG_EINVAL, "hsv_shift_u8: NULL pointer");
    return hip_status(launch_hsv_u8(in, n, H, W, dhsv, out, as_stream(stream)), "hsv_shift_u8 launch");
}

int miaug_warp_affine_u8(const uint8_t *in, int n, int H, int W, int C, const int64_t *aq, int interp, int border,
                         uint8_t *out, void *stream) {
    begin_call();
    if (n < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "warp_affine_u8: negative size");
    if (C != 1 && C != 3 && C != 4) return set_error(MIAUG_ESHAPE, "warp_affine_u8: C=%d (1, 3 or 4)", C);
    if (interp != MIAUG_INTERP_BILINEAR && interp != MIAUG_INTERP_NEAREST)
        return set_error(MIAUG_EINVAL, "warp_affine_u8: interp %d", interp);
    if (border != MIAUG_BORDER_REFLECT101 && border != MIAUG_BORDER_CONSTANT)
        return set_error(MIAUG_EINVAL, "warp_affine_u8: border %d", border);
    if (n == 0 || H == 0 || W == 0) return MIAUG_OK;
    if (!in || !aq || !out) return set_error(MIAUG_EINVAL, "warp_affine_u8: NULL pointer");
    if ((long long)H * W * C > (1ll << 31) - 1 || H > 16384 || W > 16384)
        return set_error(MIAUG_ESHAPE, "warp_affine_u8: image too large");
    return hip_status(launch_warp_u8(in, n, H, W, C, aq, interp, border, out, as_stream(stream)),
                      "warp_affine_u8 launch");
}

int miaug_ssr_crop_resize_hsv_gamma_blur_u8(const uint8_t *in, int n, int H, int W, const miaug_c2_record *rec,
                                            int crop, int outsz, uint8_t *out, void *stream) {
    begin_call();
    if (n < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "c2: negative size");
    if (n == 0) return MIAUG_OK;
    if (!in || !rec || !out) return set_error(MIAUG_EINVAL, "c2: NULL pointer");
    if (H < 1 || W < 1 || crop < 1 || crop > H || crop > W || outsz < 1 || outsz > 4096 || H > 16384 || W > 16384)
        return set_error(MIAUG_ESHAPE, "c2: H=%d W=%d crop=%d outsz=%d", H, W, crop, outsz);
    return hip_status(launch_c2(in, n, H, W, rec, crop, outsz, out, as_stream(stream)), "c2 launch");
}

int miaug_ssr_crop_resize_mask_u8(const uint8_t *in, int n, int H, int W, const miaug_c2_record *rec, int crop,
                                  int outsz, uint8_t *out, void *stream) {
    clear_error();
    if (n < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "c2 mask: negative size");
    if (n == 0) return MIAUG_OK;
    if (!in || !rec || !out) return set_error(MIAUG_EINVAL, "c2 mask: NULL pointer");
    if (crop < 1 || crop > H || crop > W || outsz < 1 || outsz > 4096 || H > 16384 || W > 16384)
        return set_error(MIAUG_ESHAPE, "c2 mask: H=%d W=%d crop=%d outsz=%d", H, W, crop, outsz);
    return hip_status(launch_c2_mask(in, n, H, W, rec, crop, outsz, out, as_stream(stream)), "c2 mask launch");
}

int miaug_boxes_ssr_crop_resize(const float *boxes, const int32_t *box_off, int n, int H, int W,
                                const miaug_c2_record *rec, int crop, int outsz, float *out, void *stream) {
    clear_error();
    if (n < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "c2 boxes: negative size");
    if (n == 0) return MIAUG_OK;
    if (!boxes || !box_off || !rec || !out) return set_error(MIAUG_EINVAL, "c2 boxes: NULL pointer");
    if (crop < 1 || crop > H || crop > W || outsz < 1 || outsz > 4096)
        return set_error(MIAUG_ESHAPE, "c2 boxes: H=%d W=%d crop=%d outsz=%d", H, W, crop, outsz);
    return hip_status(launch_c2_boxes(boxes, box_off, n, H, W, rec, crop, outsz, out, as_stream(stream)),
                      "c2 boxes launch");
}

int miaug_ragged_apply(miaug_ctx *ctx, const miaug_ragged_args *a, void *stream) {
    begin_call();
    if (!ctx) return set_error(MIAUG_EINVAL, "ragged_apply: ctx is NULL");
    if (int st = ragged_check(a)) return st;
    RaggedLaunch L{ctx_variant(ctx), ctx->num_cu, ctx->counters, ctx->counters + 256};
    log_msg(3, "ragged_apply: %d images, variant %d (%s)", a->n, L.variant, ragged_variant_name(L.variant));
    const int st = hip_status(launch_ragged(a, L, 0, as_stream(stream)), "ragged_apply launch");
    if (!st && a->n > 0) ctx->stats.launches++;
    return ctx_done(ctx, st);
}

int miaug_ragged_masks_u8(const miaug_ragged_args *a, int channels, uint8_t *out, void *stream) {
    begin_call();
    if (!a) return set_error(MIAUG_EINVAL, "ragged_masks: args is NULL");
    if (a->n < 0) return set_error(MIAUG_EINVAL, "ragged_masks: n < 0");
    if (channels < 1 || channels > 256) return set_error(MIAUG_ESHAPE, "ragged_masks: channels %d outside 1..256", channels);
    if (a->out_h < 1 || a->out_w < 1 || a->out_h > 4096 || a->out_w > 4096)
        return set_error(MIAUG_ESHAPE, "ragged_masks: output size %dx%d outside 1..4096", a->out_h, a->out_w);
    if (a->n == 0) return MIAUG_OK;
    if (!a->mask || !a->mask_off || !a->hw || !a->flags || !out)
        return set_error(MIAUG_EINVAL, "ragged_masks: a required pointer is NULL");
    return hip_status(launch_ragged_masks(a, channels, out, as_stream(stream)), "ragged_masks launch");
}

int miaug_ragged_apply_per_image(miaug_ctx *ctx, const miaug_ragged_args *a, void *stream) {
    begin_call();
    if (!ctx) return set_error(MIAUG_EINVAL, "ragged_apply_per_image: ctx is NULL");
    if (int st = ragged_check(a)) return st;
    RaggedLaunch L{ctx_variant(ctx), ctx->num_cu, ctx->counters, ctx->counters + 256};
    const int st = hip_status(launch_ragged(a, L, 1, as_stream(stream)), "ragged_apply_per_image launch");
    if (!st && a->n > 0) ctx->stats.launches++;
    return ctx_done(ctx, st);
}

int miaug_ragged_graph_create(miaug_ctx *ctx, const miaug_ragged_args *a, void *stream, miaug_graph **out) {
    begin_call();
    if (!ctx || !out) return set_error(MIAUG_EINVAL, "graph_create: NULL ctx or out");
    *out = nullptr;
    if (int st = ragged_check(a)) return st;
    if (!stream) return set_error(MIAUG_EINVAL, "graph_create: capture needs a non-null stream");
    hipStream_t s = as_stream(stream);
    int st = hip_status(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (st) return ctx_done(ctx, st);
    ctx->stats.calls++;
    RaggedLaunch L{ctx_variant(ctx), ctx->num_cu, ctx->counters, ctx->counters + 256};
    hipError_t le = launch_ragged(a, L, 0, s);
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(s, &g);
    if (le != hipSuccess || ee != hipSuccess) {
        if (g) hipGraphDestroy(g);
        return hip_status(le != hipSuccess ? le : ee, "graph capture");
    }
    hipGraphExec_t ex = nullptr;
    st = hip_status(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (st) {
        hipGraphDestroy(g);
        return st;
    }
    miaug_graph *G = new (std::nothrow) miaug_graph{g, ex};
    if (!G) {
        hipGraphExecDestroy(ex);
        hipGraphDestroy(g);
        return set_error(MIAUG_ENOMEM, "graph_create: host allocation");
    }
    *out = G;
    return MIAUG_OK;
}

int miaug_graph_launch(miaug_graph *g, void *stream) {
    begin_call();
    if (!g) return set_error(MIAUG_EINVAL, "graph_launch: NULL graph");
    return hip_status(hipGraphLaunch(g->exec, as_stream(stream)), "hipGraphLaunch");
}

int miaug_graph_destroy(miaug_graph *g) {
    begin_call();
    if (!g) return MIAUG_OK;
    hipGraphExecDestroy(g->exec);
    hipGraphDestroy(g->graph);
    delete g;
    return MIAUG_OK;
}

// Device scratch of miaug_ragged_apply_noalloc: the queue counters of the
// persistent ragged kernel, one copy per GPU (the runtime loads the array into
// every device the library runs on; each copy lives until the process ends).
// Host code never passes `scratch` itself to a kernel or a copy: on the host
// the name stands for a host-side shadow, not a device address.  It resolves
// the device address once per device with hipGetSymbolAddress and uses that.
static __device__ __align__(256) int scratch[MIAUG_NOALLOC_SCRATCH_BYTES / sizeof(int)];

namespace {
constexpr int kMaxDevices = 64;
struct NoAllocSlot {
    std::once_flag once;
    int status = MIAUG_OK;
    int *ptr = nullptr;  // device address of this device's `scratch`
    int num_cu = 0;
    char err[256] = "";
};
NoAllocSlot g_noalloc[kMaxDevices];

// Set-up of device `dev` (current at the call): the address of its copy of
// `scratch` and its compute-unit count.  Runs once per device.
void noalloc_setup(NoAllocSlot &S, int dev) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        S.status = MIAUG_EDEVICE;
        snprintf(S.err, sizeof(S.err), "ragged_apply_noalloc: hipGetSymbolAddress(scratch) on device %d: %s", dev,
                 hipGetErrorString(e));
        return;
    }
    int cu = 0;
    e = hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess || cu < 1) {
        S.status = MIAUG_EDEVICE;
        snprintf(S.err, sizeof(S.err), "ragged_apply_noalloc: compute-unit count of device %d: %s", dev,
                 hipGetErrorString(e));
        return;
    }
    S.ptr = (int *)p;
    S.num_cu = cu;
}
}  // namespace

int miaug_ragged_apply_noalloc(const miaug_ragged_args *a, int variant, void *stream) {
    begin_call();
    if (int st = ragged_check(a)) return st;
    if (variant < -1 || variant >= ragged_variant_count())
        return set_error(MIAUG_EINVAL, "ragged_apply_noalloc: variant %d out of range", variant);
    if (variant >= 0 && !ragged_variant_enabled(variant))
        return set_error(MIAUG_EUNSUPPORTED, "ragged_apply_noalloc: variant %d is switched off", variant);
    const size_t need = (size_t)ragged_counter_ints() * sizeof(int);
    if (need > MIAUG_NOALLOC_SCRATCH_BYTES)
        return set_error(MIAUG_ECAPACITY, "ragged_apply_noalloc: needs %zu bytes of scratch, the static array holds %d",
                         need, MIAUG_NOALLOC_SCRATCH_BYTES);
    if (a->n == 0) return MIAUG_OK;
    int dev = -1;
    if (int st = hip_status(hipGetDevice(&dev), "hipGetDevice")) return st;
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(MIAUG_EUNSUPPORTED, "ragged_apply_noalloc: device %d (at most %d devices)", dev, kMaxDevices);
    NoAllocSlot &S = g_noalloc[dev];
    std::call_once(S.once, noalloc_setup, std::ref(S), dev);
    if (S.status != MIAUG_OK) return set_error(S.status, "%s", S.err);
    RaggedLaunch L{variant < 0 ? ragged_default_variant() : variant, S.num_cu, S.ptr};
    return hip_status(launch_ragged(a, L, 0, as_stream(stream)), "ragged_apply_noalloc launch");
}

int miaug_ragged_variant_count(void) { return ragged_variant_count(); }
const char *miaug_ragged_variant_name(int v) { return ragged_variant_name(v); }

int miaug_ragged_set_variant(miaug_ctx *ctx, int v) {
    begin_call();
    if (!ctx) return set_error(MIAUG_EINVAL, "set_variant: NULL ctx");
    if (v < -1 || v >= ragged_variant_count()) return set_error(MIAUG_EINVAL, "set_variant: %d out of range", v);
    if (v >= 0 && !ragged_variant_enabled(v)) return set_error(MIAUG_EUNSUPPORTED, "set_variant: variant %d is switched off", v);
    ctx->variant = v < 0 ? ragged_default_variant() : v;
    return ctx_done(ctx, MIAUG_OK);
}

namespace {

// Cache key of a ragged batch: GPU architecture, chain options, output size
// and buckets (powers of two) of the image count, the mean image area and the
// longest side, plus the size of the variant table.
int ragged_tune_key(const miaug_ctx *ctx, const miaug_ragged_args *a, hipStream_t s, std::string &key) {
    std::vector<int32_t> hw((size_t)2 * a->n);
    int st = hip_status(hipMemcpyAsync(hw.data(), a->hw, hw.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s),
                        "autotune: copy sizes");
    if (!st) st = hip_status(hipStreamSynchronize(s), "sync");
    if (st) return st;
    double area = 0;
    int side = 1;
    for (int i = 0; i < a->n; ++i) {
        area += (double)hw[2 * i] * hw[2 * i + 1];
        side = hw[2 * i] > side ? hw[2 * i] : side;
        side = hw[2 * i + 1] > side ? hw[2 * i + 1] : side;
    }
    auto lg = [](double v) { int k = 0; while (v > 1.5 && k < 62) { v /= 2; ++k; } return k; };
    char buf[256];
    snprintf(buf, sizeof(buf), "%s|ragged|o%dx%d|m%db%dc%d|n%d|p%d|s%d|v%d", ctx->arch.c_str(), a->out_h, a->out_w,
             a->mask != nullptr, a->boxes != nullptr, a->crop != nullptr, lg((double)a->n), lg(area / a->n),
             lg((double)side), ragged_variant_count());
    key = buf;
    return MIAUG_OK;
}

int ragged_autotune_run(miaug_ctx *ctx, const miaug_ragged_args *a, int reps, hipStream_t s, int *chosen, float *ms,
                        float *times) {
    const size_t out_words = (size_t)a->n * 3 * a->out_h * a->out_w;
    const size_t out_bytes = out_words * sizeof(float);
    const size_t mask_bytes = a->mask ? (size_t)a->n * a->out_h * a->out_w : 0;
    int nbox = 0;
    int st = MIAUG_OK;
    if (a->boxes) {
        st = hip_status(hipMemcpyAsync(&nbox, a->box_off + a->n, sizeof(int), hipMemcpyDeviceToHost, s), "copy");
        if (!st) st = hip_status(hipStreamSynchronize(s), "sync");
        if (st) return st;
        if (nbox < 0) return set_error(MIAUG_EINVAL, "autotune: box_off[n] = %d", nbox);
    }
    const size_t box_bytes = (size_t)nbox * 4 * sizeof(float);
    std::vector<char> ref(out_bytes), got(out_bytes), mref(mask_bytes), mgot(mask_bytes), bref(box_bytes),
        bgot(box_bytes);
    // Every run starts from the same sentinel in all three outputs, so images
    // a launch skips (their outputs stay untouched) compare equal, and a form
    // that leaves a mask or box unwritten does not.
    auto fill = [&]() {
        int e = hip_status(launch_fill_u32((uint32_t *)a->out, out_words, 0x7fc0a5a5u, s), "autotune fill");
        if (!e && mask_bytes) e = hip_status(launch_fill_u8(a->out_mask, mask_bytes, 0xa5, s), "autotune fill");
        if (!e && box_bytes)
            e = hip_status(launch_fill_u32((uint32_t *)a->out_boxes, (size_t)nbox * 4, 0x7fc0a5a5u, s), "autotune fill");
        return e;
    };
    auto fetch = [&](std::vector<char> &o, std::vector<char> &mo, std::vector<char> &bo) {
        int e = hip_status(hipMemcpyAsync(o.data(), a->out, out_bytes, hipMemcpyDeviceToHost, s), "copy");
        if (!e && mask_bytes)
            e = hip_status(hipMemcpyAsync(mo.data(), a->out_mask, mask_bytes, hipMemcpyDeviceToHost, s), "copy");
        if (!e && box_bytes)
            e = hip_status(hipMemcpyAsync(bo.data(), a->out_boxes, box_bytes, hipMemcpyDeviceToHost, s), "copy");
        if (!e) e = hip_status(hipStreamSynchronize(s), "sync");
        return e;
    };
    RaggedLaunch L{0, ctx->num_cu, ctx->counters, ctx->counters + 256};
    st = fill();
    if (!st) st = hip_status(launch_ragged(a, L, 1, s), "autotune reference");
    if (!st) st = fetch(ref, mref, bref);
    if (st) return st;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    int best = -1;
    float best_ms = 0.f;
    for (int v = 0; v < ragged_variant_count() && !st; ++v) {
        L.variant = v;
        if (times) times[v] = -1.f;
        if (!ragged_variant_enabled(v)) continue;
        st = fill();
        if (!st) st = hip_status(launch_ragged(a, L, 0, s), "autotune candidate");
        if (!st) st = fetch(got, mgot, bgot);
        if (st) break;
        if (memcmp(ref.data(), got.data(), out_bytes) != 0 || memcmp(mref.data(), mgot.data(), mask_bytes) != 0 ||
            memcmp(bref.data(), bgot.data(), box_bytes) != 0)
            continue;  // parity gate: only variants identical to the per-image form compete
        // untimed launches first: the parity copy above leaves the GPU idle, and
        // its clocks need some back-to-back work to come up again
        for (int r = 0; r < 2 * reps && !st; ++r) st = hip_status(launch_ragged(a, L, 0, s), "autotune warm-up");
        hipEventRecord(e0, s);
        for (int r = 0; r < reps && !st; ++r) st = hip_status(launch_ragged(a, L, 0, s), "autotune timing");
        hipEventRecord(e1, s);
        if (!st) st = hip_status(hipEventSynchronize(e1), "sync");
        float t = 0.f;
        hipEventElapsedTime(&t, e0, e1);
        t /= reps;
        if (times) times[v] = t;
        if (best < 0 || t < best_ms) {
            best = v;
            best_ms = t;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st) return st;
    if (best < 0) return set_error(MIAUG_EDEVICE, "autotune: no variant matched the per-image output");
    ctx->variant = best;
    if (chosen) *chosen = best;
    if (ms) *ms = best_ms;
    return MIAUG_OK;
}

}  // namespace

int miaug_ragged_autotune(miaug_ctx *ctx, const miaug_ragged_args *a, int reps, void *stream, int *chosen, float *ms,
                          float *times) {
    begin_call();
    if (!ctx) return set_error(MIAUG_EINVAL, "autotune: NULL ctx");
    if (int st = ragged_check(a)) return st;
    if (reps < 1) return set_error(MIAUG_EINVAL, "autotune: reps < 1");
    if (a->n == 0) {
        if (chosen) *chosen = ctx->variant;
        if (ms) *ms = 0.f;
        return ctx_done(ctx, MIAUG_OK);
    }
    hipStream_t s = as_stream(stream);
    std::string key;
    if (!ctx->tune_cache.empty()) {
        if (int st = ragged_tune_key(ctx, a, s, key)) return ctx_done(ctx, st);
        TuneEntry e;
        const int cst = tune_cache_get(ctx->tune_cache, key, &e);
        const char *nm = ragged_variant_name(e.variant);
        if (cst == MIAUG_OK && nm && e.name == nm && ragged_variant_enabled(e.variant)) {
            ctx->variant = e.variant;
            if (chosen) *chosen = e.variant;
            if (ms) *ms = e.ms;
            if (times)
                for (int v = 0; v < ragged_variant_count(); ++v) times[v] = v == e.variant ? e.ms : -1.f;
            ctx->stats.tune_cache_hits++;
            log_msg(2, "autotune: %s from the cache: variant %d (%s), %.4f ms", key.c_str(), e.variant, nm, (double)e.ms);
            clear_error();
            return ctx_done(ctx, MIAUG_OK);
        }
        clear_error();  // a missing or stale entry is not an error
    }
    int v = -1;
    float t = 0.f;
    int st = ragged_autotune_run(ctx, a, reps, s, &v, &t, times);
    if (st) return ctx_done(ctx, st);
    ctx->stats.tune_runs++;
    log_msg(2, "autotune: variant %d (%s), %.4f ms", v, ragged_variant_name(v), (double)t);
    if (!key.empty()) {
        TuneEntry e;
        e.key = key;
        e.variant = v;
        e.name = ragged_variant_name(v);
        e.ms = t;
        st = tune_cache_put(ctx->tune_cache, e);  // the choice stands even if the file cannot be written
        if (st) log_msg(1, "autotune: %s", miaug_last_error());
        clear_error();
    }
    if (chosen) *chosen = v;
    if (ms) *ms = t;
    return ctx_done(ctx, MIAUG_OK);
}

int miaug_warpcolor_fwd(const float *x, int n, int C, int H, int W, const float *params, float *y, void *stream) {
    begin_call();
    if (n < 0 || C < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "warpcolor_fwd: negative size");
    if (n == 0 || C == 0 || H == 0 || W == 0) return MIAUG_OK;
    if (!x || !params || !y) return set_error(MIAUG_EINVAL, "warpcolor_fwd: NULL pointer");
    if (H > 16384 || W > 16384) return set_error(MIAUG_ESHAPE, "warpcolor_fwd: %dx%d too large", H, W);
    return hip_status(launch_wc_fwd(x, n, C, H, W, params, y, as_stream(stream)), "warpcolor_fwd launch");
}

size_t miaug_warpcolor_workspace_bytes(int n, int C, int H, int W) {
    if (n <= 0 || C <= 0 || H <= 0 || W <= 0) return 0;
    return wc_workspace_bytes(n, C, H, W);
}

int miaug_warpcolor_bwd(const float *x, int n, int C, int H, int W, const float *params, const float *gy,
                        float *grad_x, float *grad_params, void *ws, size_t ws_bytes, void *stream) {
    begin_call();
    if (n < 0 || C < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "warpcolor_bwd: negative size");
    if (n == 0 || C == 0 || H == 0 || W == 0) return MIAUG_OK;
    if (!x || !params || !gy || !grad_params) return set_error(MIAUG_EINVAL, "warpcolor_bwd: NULL pointer");
    if (C > 4) return set_error(MIAUG_ESHAPE, "warpcolor_bwd: C=%d (at most 4 channels)", C);
    if (H > 16384 || W > 16384) return set_error(MIAUG_ESHAPE, "warpcolor_bwd: %dx%d too large", H, W);
    size_t need = wc_workspace_bytes(n, C, H, W);
    if (!ws || ws_bytes < need)
        return set_error(MIAUG_ECAPACITY, "warpcolor_bwd: workspace %zu < %zu bytes", ws_bytes, need);
    return hip_status(launch_wc_bwd(x, n, C, H, W, params, gy, grad_x, grad_params, ws, as_stream(stream)),
                      "warpcolor_bwd launch");
}

size_t miaug_elastic_workspace_bytes(int n, int H, int W) {
    if (n <= 0 || H <= 0 || W <= 0) return 0;
    return elastic_workspace_bytes(n, H, W);
}

int miaug_elastic_fields(uint64_t seed, uint64_t first, int n, int H, int W, double sigma, int alpha, int radius,
                         int32_t *off, void *ws, size_t ws_bytes, void *stream) {
    begin_call();
    if (n < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "elastic_fields: negative size");
    if (n == 0 || H == 0 || W == 0) return MIAUG_OK;
    if (!off) return set_error(MIAUG_EINVAL, "elastic_fields: NULL off");
    if (radius < 1 || radius > 200 || !(sigma > 0.0) || alpha < 0 || alpha > 65535)
        return set_error(MIAUG_ESHAPE, "elastic_fields: radius=%d sigma=%g alpha=%d", radius, sigma, alpha);
    if ((long long)H * W > (1ll << 30)) return set_error(MIAUG_ESHAPE, "elastic_fields: image too large");
    size_t need = elastic_workspace_bytes(n, H, W);
    if (!ws || ws_bytes < need)
        return set_error(MIAUG_ECAPACITY, "elastic_fields: workspace %zu < %zu bytes", ws_bytes, need);
    return hip_status(launch_elastic_fields(seed, first, n, H, W, sigma, alpha, radius, off, ws, as_stream(stream)),
                      "elastic_fields launch");
}

size_t miaug_elastic_box_workspace_bytes(int n, int H, int W) {
    return (n > 0 && H > 0 && W > 0) ? box_workspace_bytes(n, H, W) : 0;
}

int miaug_elastic_fields_box(uint64_t seed, uint64_t first, int n, int H, int W, double sigma, int alpha,
                             int32_t *off, void *ws, size_t ws_bytes, void *stream) {
    begin_call();
    if (n < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "elastic_fields_box: negative size");
    if (n == 0 || H == 0 || W == 0) return MIAUG_OK;
    if (!off) return set_error(MIAUG_EINVAL, "elastic_fields_box: NULL off");
    if (!(sigma > 0.0) || alpha < 0 || alpha > 65535)
        return set_error(MIAUG_ESHAPE, "elastic_fields_box: sigma=%g alpha=%d", sigma, alpha);
    int r[3];
    box_radii(sigma, r);
    if (r[0] < 0 || r[2] > 255) return set_error(MIAUG_ESHAPE, "elastic_fields_box: sigma %g gives box radius %d > 255", sigma, r[2]);
    if (W > 7168 || (long long)H * W > (1ll << 30))
        return set_error(MIAUG_ESHAPE, "elastic_fields_box: rows longer than 7168 or image too large");
    const size_t need = box_workspace_bytes(n, H, W);
    if (!ws || ws_bytes < need)
        return set_error(MIAUG_ECAPACITY, "elastic_fields_box: workspace %zu < %zu bytes", ws_bytes, need);
    return hip_status(launch_elastic_fields_box(seed, first, n, H, W, sigma, alpha, off, ws, as_stream(stream)),
                      "elastic_fields_box launch");
}

int miaug_grid_tables(const double *grid, int n, int H, int W, int32_t *mapx, int32_t *mapy, void *stream) {
    begin_call();
    if (n < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "grid_tables: negative size");
    if (n == 0 || H == 0 || W == 0) return MIAUG_OK;
    if (!grid || !mapx || !mapy) return set_error(MIAUG_EINVAL, "grid_tables: NULL pointer");
    if (H > 1000000 || W > 1000000) return set_error(MIAUG_ESHAPE, "grid_tables: size too large");
    return hip_status(launch_grid_tables(grid, n, H, W, mapx, mapy, as_stream(stream)), "grid_tables launch");
}

int miaug_elastic_grid_u8(const uint8_t *img, const uint8_t *mask, int n, int H, int W, int C, const int32_t *off,
                          const int32_t *mapx, const int32_t *mapy, uint8_t *out, uint8_t *out_mask, int per_image,
                          void *stream) {
    begin_call();
    if (n < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "elastic_grid_u8: negative size");
    if (C != 1 && C != 3 && C != 4) return set_error(MIAUG_ESHAPE, "elastic_grid_u8: C=%d", C);
    if (n == 0 || H == 0 || W == 0) return MIAUG_OK;
    if (!img || !off || !mapx || !mapy || !out || (mask && !out_mask))
        return set_error(MIAUG_EINVAL, "elastic_grid_u8: NULL pointer");
    if ((long long)H * W * C > (1ll << 31) - 1) return set_error(MIAUG_ESHAPE, "elastic_grid_u8: image too large");
    return hip_status(launch_elastic_grid_u8(img, mask, n, H, W, C, off, mapx, mapy, out, out_mask, per_image,
                                             as_stream(stream)),
                      "elastic_grid_u8 launch");
}

int miaug_boxes_elastic_grid(const float *boxes, const int32_t *box_off, int n, int H, int W, const int32_t *off,
                             const int32_t *mapx, const int32_t *mapy, float *out, void *stream) {
    begin_call();
    if (n < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "boxes_elastic_grid: negative size");
    if (n == 0 || H == 0 || W == 0) return MIAUG_OK;
    if (!boxes || !box_off || !off || !mapx || !mapy || !out)
        return set_error(MIAUG_EINVAL, "boxes_elastic_grid: NULL pointer");
    if ((long long)H * W > (1ll << 30) || H > 16384 || W > 16384)
        return set_error(MIAUG_ESHAPE, "boxes_elastic_grid: image too large");
    return hip_status(launch_boxes_distort(boxes, box_off, n, H, W, off, mapx, mapy, out, as_stream(stream)),
                      "boxes_elastic_grid launch");
}

size_t miaug_chain_f32_workspace_bytes(int n, int C, int H, int W) {
    if (n <= 0 || C <= 0 || H <= 0 || W <= 0) return 0;
    return chain_f32_workspace_bytes(n, C, H, W);
}

int miaug_elastic_grid_f32_fwd(const float *x, int n, int C, int H, int W, const int32_t *off, const int32_t *mapx,
                               const int32_t *mapy, float *y, void *ws, size_t ws_bytes, void *stream) {
    begin_call();
    if (n < 0 || C < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "chain_f32_fwd: negative size");
    if (n == 0 || C == 0 || H == 0 || W == 0) return MIAUG_OK;
    if (!x || !off || !mapx || !mapy || !y) return set_error(MIAUG_EINVAL, "chain_f32_fwd: NULL pointer");
    if ((long long)H * W > (1ll << 30) || H >= (1 << 20) || W >= (1 << 20) || n > 65535)
        return set_error(MIAUG_ESHAPE, "chain_f32_fwd: n=%d, %dx%d out of range", n, H, W);
    size_t need = chain_f32_workspace_bytes(n, C, H, W);
    if (!ws || ws_bytes < need)
        return set_error(MIAUG_ECAPACITY, "chain_f32_fwd: workspace %zu < %zu bytes", ws_bytes, need);
    return hip_status(launch_chain_f32_fwd(x, n, C, H, W, off, mapx, mapy, y, ws, as_stream(stream)),
                      "chain_f32_fwd launch");
}

int miaug_elastic_grid_f32_bwd(const float *gy, int n, int C, int H, int W, const int32_t *off, const int32_t *mapx,
                               const int32_t *mapy, float *gx, void *ws, size_t ws_bytes, void *stream) {
    begin_call();
    if (n < 0 || C < 0 || H < 0 || W < 0) return set_error(MIAUG_EINVAL, "chain_f32_bwd: negative size");
    if (n == 0 || C == 0 || H == 0 || W == 0) return MIAUG_OK;
    if (!gy || !off || !mapx || !mapy || !gx) return set_error(MIAUG_EINVAL, "chain_f32_bwd: NULL pointer");
    if ((long long)H * W > (1ll << 30) || H >= (1 << 20) || W >= (1 << 20) || n > 65535)
        return set_error(MIAUG_ESHAPE, "chain_f32_bwd: n=%d, %dx%d out of range", n, H, W);
    size_t need = chain_f32_workspace_bytes(n, C, H, W);
    if (!ws || ws_bytes < need)
        return set_error(MIAUG_ECAPACITY, "chain_f32_bwd: workspace %zu < %zu bytes", ws_bytes, need);
    return hip_status(launch_chain_f32_bwd(gy, n, C, H, W, off, mapx, mapy, gx, ws, as_stream(stream)),
                      "chain_f32_bwd launch");
}

int miaug_image_stats_u8(const uint8_t *img, int n, int64_t npix, int C, uint64_t *sum, int32_t *mn, int32_t *mx,
                         uint32_t *hist, void *stream) {
    begin_call();
    if (n < 0 || npix < 0) return set_error(MIAUG_EINVAL, "image_stats: negative size");
    if (C < 1 || C > 4) return set_error(MIAUG_ESHAPE, "image_stats: C=%d", C);
    if (n == 0) return MIAUG_OK;
    if (!img && npix > 0) return set_error(MIAUG_EINVAL, "image_stats: NULL image");
    if (npix > (1ll << 40)) return set_error(MIAUG_ESHAPE, "image_stats: too many pixels");
    return hip_status(launch_image_stats(img, n, npix, C, sum, mn, mx, hist, as_stream(stream)), "image_stats launch");
}

}  // extern "C"
