/*
 * miaug.h -- C ABI of libmiaug, an MI355X (gfx950) implementation of the
 * batched image-augmentation hot path of Buslaev et al., "Albumentations:
 * fast and flexible image augmentations" (arXiv:1809.06839).
 *
 * The paper describes augmentation as label-preserving transforms applied to
 * images together with their masks and boxes (Abstract; Sec. I; Sec. II-A to
 * II-C) and times the single ops of Table I.  It gives no formulas; the exact
 * arithmetic of every op below is a stated reading (integer fixed point with
 * round-half-even and saturation for u8 data, IEEE double for per-sample
 * setup), so that results are reproducible bit for bit.
 *
 * Conventions for every entry point:
 *  - Return value: MIAUG_OK (0) or a negative status; nothing throws.  The
 *    text of the last error of the calling thread is miaug_last_error().
 *  - Memory: every tensor is owned by the caller.  Arguments documented as
 *    "device" are HIP device pointers; "host" are ordinary host pointers.  The
 *    library never keeps a caller pointer after the enqueued work.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Calls enqueue work and return; validation errors are reported
 *    synchronously; launch failures are reported as MIAUG_EDEVICE.
 *  - Layouts: u8 images are HWC with dense rows (C = 3 unless stated); masks
 *    are HW u8; float images are CHW float32; boxes are xyxy float32 in
 *    continuous pixel coordinates (pixel (i, j) covers [j, j+1) x [i, i+1)).
 *  - Fixed point: sub-pixel positions carry 10 fraction bits (Q10).
 *    rdiv_he(n, d) is n/d rounded to nearest, ties to even, with floor
 *    division; sat8 clamps to [0, 255].
 */
#ifndef MIAUG_H
#define MIAUG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
    MIAUG_OK = 0,
    MIAUG_EINVAL = -1,       /* null pointer or out-of-range scalar argument   */
    MIAUG_ESHAPE = -2,       /* inconsistent or unsupported sizes              */
    MIAUG_EUNSUPPORTED = -3, /* valid request the library does not implement   */
    MIAUG_EDEVICE = -4,      /* HIP runtime error (launch, copy, no device)    */
    MIAUG_ENOMEM = -5,       /* device or host allocation failed               */
    MIAUG_ECAPACITY = -6     /* workspace smaller than required                */
};

/* Library version as 10000*major + 100*minor + patch. */
int miaug_version(void);
/* Static text of a status code. */
const char *miaug_status_str(int status);
/* Text of the calling thread's last error; valid until its next miaug call. */
const char *miaug_last_error(void);

/* ---------------------------------------------------------------- sampler
 * Per-sample transform parameters from a counter-based generator
 * (Philox4x64-10, Salmon et al., SC'11): draw d of global sample index g is
 * word 0 of Philox(counter = {d, g, 0, 0}, key = {seed, 0}).  A uniform is
 * (word >> 11) * 2^-53; a Bernoulli(p) is uniform < p; an integer in
 * {0..m-1} is ((word >> 32) * m) >> 32; a float in [lo, hi] is
 * (float)(lo + (hi - lo) * uniform) in double.  Results depend only on
 * (seed, g), never on batch composition.  All outputs are host arrays of n
 * records; the functions never touch the GPU.
 */

/* Random Dih4 element + brightness/contrast (Sec. II-B Dih4; Table I
 * HorizontalFlip, VerticalFlip, Brightness).  flags[4i..4i+3] = {hflip p=.5,
 * vflip p=.5, rot90 k in {0..3}, transpose p=.5}; ab[2i..2i+1] = {alpha in
 * [0.8,1.2], beta in [-51,51]} (draws 0..5). */
int miaug_sample_d4bc(uint64_t seed, uint64_t first_index, int n, int32_t *flags, float *ab);

/* Shift-scale-rotate + crop + hue/saturation + gamma + blur (Table I Rotate,
 * ShiftScaleRotate, RandomCrop64, ShiftHSV, Gamma).  f[5i..] = {angle_deg in
 * [-45,45], scale in [0.9,1.1], dx, dy in [-0.0625,0.0625], gamma in
 * [0.8,1.2]}; k[5i..] = {crop_x, crop_y in {0..crop_range}, dh = rint(U[-20,20])
 * (hue, 2-degree units), ds = rint(U[-30,30]) (saturation, 0..255 scale),
 * blur p=0.3}. */
int miaug_sample_c2(uint64_t seed, uint64_t first_index, int n, int crop_range, float *f, int32_t *k);

/* Differentiable warp + colour parameters: f[7i..] = {angle_deg in [-45,45],
 * scale in [0.9,1.1], tx, ty in [-0.0625,0.0625] (fractions of W, H), alpha
 * in [0.8,1.2], beta in [-0.2,0.2], gamma in [0.8,1.2]}. */
int miaug_sample_wc(uint64_t seed, uint64_t first_index, int n, float *f);

/* Grid distortion (Sec. II-C): f[10i..] = {x factors d_0..d_4, y factors
 * d_0..d_4}, each 1 + (double)(float)U[-limit, limit]. */
int miaug_sample_grid(uint64_t seed, uint64_t first_index, int n, double limit, double *f);

/* ---------------------------------------------------------------- context
 * A context holds per-device state: queue counters of the persistent ragged
 * kernel, the tuned launch choice, the autotuner's cache file, counters of
 * its use and device properties.  One context per host thread/stream; calls
 * on one context must not overlap in time on different streams. */
typedef struct miaug_ctx miaug_ctx;
/* Creates a context on HIP device `device` (allocates 1 KiB of device
 * memory).  tune_cache_path: JSON file in which miaug_ragged_autotune keeps its
 * choice per (GPU architecture, chain, batch-shape bucket) and from which later
 * processes take it without timing; NULL = the MIAUG_TUNE_CACHE environment
 * variable, or no cache when that is unset too.  The file is created on the
 * first autotuner run; a file that is not a cache is ignored and replaced.
 * Errors: EINVAL null out or device out of range; EDEVICE no HIP device;
 * ENOMEM allocation failure. */
int miaug_ctx_create(int device, const char *tune_cache_path, miaug_ctx **out);
int miaug_ctx_destroy(miaug_ctx *ctx);

/* Counters of a context since its creation. */
typedef struct {
    uint64_t calls;           /* calls with this context whose arguments were accepted   */
    uint64_t launches;        /* batched or per-image ragged launches enqueued           */
    uint64_t tune_runs;       /* autotuner runs that timed the variants                  */
    uint64_t tune_cache_hits; /* autotuner runs answered from the cache file             */
    uint64_t errors;          /* of those, calls that failed (device, launch, memory)    */
    int32_t variant;          /* ragged launch variant the next launch uses              */
    int32_t last_status;      /* status of the last call                                 */
} miaug_stats;
/* Copies the counters to *out.  Errors: EINVAL null pointer. */
int miaug_ctx_stats(const miaug_ctx *ctx, miaug_stats *out);

/* The autotuner's cache file, for tools and tests (host only, no GPU needed).
 * lookup: the entry stored under `key` -> *variant, *ms and the variant's name
 * (copied into name[0..name_len-1], NUL-terminated; name may be NULL); returns
 * MIAUG_EUNSUPPORTED when the file has no such key (or does not exist) and
 * MIAUG_EINVAL when it is not a cache file.  store: adds or replaces the entry
 * (written to a temporary file renamed over the cache).  Errors: EINVAL null
 * path or key, or the file cannot be written. */
int miaug_tune_cache_lookup(const char *path, const char *key, int *variant, float *ms, char *name, size_t name_len);
int miaug_tune_cache_store(const char *path, const char *key, int variant, const char *name, float ms);

/* Failure injection for tests of the error paths: the library's allocation
 * number `after` (0 = the next one; device or pinned host memory, counted
 * across the process) fails with MIAUG_ENOMEM, once; -1 disarms.  The same
 * as setting MIAUG_FAIL_ALLOC_AFTER before the first call. */
int miaug_debug_fail_alloc_after(long after);
/* Allocates `bytes` of device memory through the library's allocator (the one
 * the injector above intercepts) and frees it; returns the allocation status
 * (MIAUG_ENOMEM when injected, MIAUG_EDEVICE without a usable device). */
int miaug_debug_alloc_probe(size_t bytes);

/* ---------------------------------------------------------------- plain Dih4 + brightness/contrast
 * Sec. II-B (random transformation from Dih4) and Table I (HorizontalFlip,
 * VerticalFlip, Brightness).  For each image i of a dense batch:
 * out_i = LUT_i[d4_i(in_i)] with d4_i = hflip -> vflip -> rot90^k ->
 * transpose as selected by flags[4i..4i+3] (rot90 is counter-clockwise,
 * out[r][c] = in[c][W-1-r]) and LUT_i[v] = sat8(rint((double)alpha*v +
 * (double)beta)).
 *   in     device u8 [n][H][W][C], C in {1, 3, 4}
 *   flags  device int32 [n][4]; ab device float [n][2]
 *   out    device u8, n*H*W*C bytes; image i occupies bytes
 *          [i*H*W*C, (i+1)*H*W*C) with shape (H, W, C), or (W, H, C) when its
 *          element swaps the axes (odd k xor transpose).
 * Errors: EINVAL on null pointers or n, H, W < 0 (n == 0 is a no-op);
 * ESHAPE if C is not 1, 3 or 4; EDEVICE on launch failure. */
int miaug_d4_bc_u8(const uint8_t *in, int n, int H, int W, int C, const int32_t *flags, const float *ab,
                   uint8_t *out, void *stream);

/* ---------------------------------------------------------------- the other Table I single ops
 * ShiftRGB and Grayscale (Table I): the Dih4 kernel with per-channel LUTs
 * and an optional grayscale step.  out_i = G_i(L_i[d4_i(in_i)]) where
 * L_i applies luts[i][c][.] to channel c, and G_i (when gray != NULL and
 * gray[i] != 0; C = 3 only) replaces every pixel by its BT.601 luma
 * Y = (4899 R + 9617 G + 1868 B + 8192) >> 14 in all three channels.
 *   luts device u8 [n][C][256] (miaug_compile_color_luts); gray device int32
 *   [n] or NULL; other arguments as miaug_d4_bc_u8 (flags all zero: no
 *   geometric change).  Errors as miaug_d4_bc_u8; ESHAPE gray with C != 3. */
int miaug_d4_lut_u8(const uint8_t *in, int n, int H, int W, int C, const int32_t *flags, const uint8_t *luts,
                    const int32_t *gray, uint8_t *out, void *stream);
/* Host: luts[i][c][v] = S_ic(B_i(v)) with B_i(v) = sat8(rint(alpha_i v + beta_i))
 * (ab host float [n][2], NULL: identity) and S_ic(u) = sat8(rint(u + shift[i][c]))
 * (ShiftRGB; shift host float [n][C], NULL: identity), in IEEE double. */
int miaug_compile_color_luts(const float *ab, const float *shift, int n, int C, uint8_t *luts);

/* Host: Gamma as a per-channel LUT for miaug_d4_lut_u8 (Table I Gamma):
 * luts[i][c][v] = sat8(rint(255 (v / 255)^gamma_i)) in IEEE double, the same
 * table as the gamma step of miaug_ssr_crop_resize_hsv_gamma_blur_u8, for
 * every c < C.  gamma host float [n]; luts host u8 [n][C][256].  Errors:
 * EINVAL bad arguments or a gamma that is not finite. */
int miaug_compile_gamma_luts(const float *gamma, int n, int C, uint8_t *luts);

/* Binomial blur: out = rdiv_he(sum_ij k_i k_j in[y + j - r][x + i - r], N)
 * per channel with k = [1, 2, 1], N = 16 (ksize 3, r = 1) or
 * k = [1, 4, 6, 4, 1], N = 256 (ksize 5, r = 2), reflect-101 border (the
 * blur step of the u8 chain is the 3x3 case).  apply device int32 [n]
 * (0: image copied unchanged) or NULL (every image blurred).  in, out device
 * u8 [n][H][W][C], not overlapping.  Errors: EINVAL bad size, ksize, NULL
 * pointer or overlap; ESHAPE C or sides above 65535. */
int miaug_blur_u8(const uint8_t *in, int n, int H, int W, int C, int ksize, const int32_t *apply, uint8_t *out,
                  void *stream);

/* ShiftHSV alone (Table I ShiftHSV): each RGB pixel goes through the integer
 * hexcone HSV round trip of the u8 chain (step 4 of
 * miaug_ssr_crop_resize_hsv_gamma_blur_u8) with hue, saturation and value
 * shifts dhsv[i] = {dh, ds, dv} (dh in 2-degree units; dv is 0 in the chain).
 * in device u8 [n][H][W][3]; dhsv device int32 [n][3]; out device u8
 * [n][H][W][3] (may equal in).  Errors: EINVAL negative sizes or NULL
 * pointers; ESHAPE images above 2^40 bytes. */
int miaug_hsv_shift_u8(const uint8_t *in, int n, int H, int W, const int32_t *dhsv, uint8_t *out, void *stream);

/* PadToSize (Table I PadToSize512): out_i has size max(H, min_h) x
 * max(W, min_w); the padding along an axis is split floor(d / 2) before and
 * the rest after; out[y][x] = in[y - top][x - left] inside, else the
 * reflect-101 image of that index (border MIAUG_BORDER_REFLECT101) or value
 * (MIAUG_BORDER_CONSTANT).  in device u8 [n][H][W][C]; out device u8
 * [n][Ho][Wo][C]; in is read in the aligned 4-byte words that hold its bytes.
 * Errors: EINVAL bad sizes, border or value; ESHAPE C. */
int miaug_pad_u8(const uint8_t *in, int n, int H, int W, int C, int min_h, int min_w, int border, int value,
                 uint8_t *out, void *stream);

/* Standalone affine warp (Table I Rotate; ShiftScaleRotate without crop):
 * out[y][x] samples in at the Q10 position rshr_he(A_i (x, y, 1), 22) of the
 * Q32 inverse matrix A_i = aq[6i .. 6i+5] (miaug_compile_ssr_q32): bilinear
 * (weights (1024 - a, a), one round-half-even of the 2^20-scaled sum) or
 * nearest (index (q + 512) >> 10); taps outside the image take reflect-101
 * or 0 (constant border).  Output has the input's shape.
 *   aq device int64 [n][6].  Errors: EINVAL, ESHAPE (H, W > 16384). */
int miaug_warp_affine_u8(const uint8_t *in, int n, int H, int W, int C, const int64_t *aq, int interp, int border,
                         uint8_t *out, void *stream);
/* Host: the Q32 inverse matrices of shift-scale-rotate maps
 * p' = s R(angle) (p - c) + c + (dx W, dy H) (the map of the full u8 chain),
 * f host float [n][4] = {angle_deg, scale, dx, dy}; Rotate is scale 1,
 * dx = dy = 0.  aq host int64 [n][6].  Errors: EINVAL, ESHAPE (scale 0). */
int miaug_compile_ssr_q32(const float *f, int n, int H, int W, int64_t *aq);

/* ---------------------------------------------------------------- full u8 pipeline
 * Table I ShiftScaleRotate -> RandomCrop -> resize -> ShiftHSV -> Gamma, then
 * a 3x3 binomial blur with probability 0.3, per RGB image, each op rounding
 * to u8 before the next:
 *  1. warp: forward map p' = s R(theta)(p - c) + c + (dx W, dy H), R(theta) =
 *     [[cos, sin], [-sin, cos]], c = ((W-1)/2, (H-1)/2).  Its inverse
 *     a = {cos/s, -sin/s, cx - a0 (cx + dx W) - a1 (cy + dy H),
 *          sin/s,  cos/s, cy - a3 (cx + dx W) - a4 (cy + dy H)}
 *     (theta in radians = angle_deg * (pi/180), every expression evaluated
 *     left to right in IEEE double) is quantised aq_i = llrint(a_i 2^32); the
 *     source position of output pixel (x, y) is
 *     q = rdiv_he(aq0 x + aq1 y + aq2, 2^22) (Q10, same for y with aq3..5);
 *     bilinear with weights (1024 - f, f) per axis, value
 *     rdiv_he(sum w_y w_x p, 2^20), reflect-101 border per tap;
 *  2. crop crop x crop at (crop_x, crop_y);
 *  3. resize to outsz x outsz, half-pixel centres
 *     q_j = rdiv_he(((2j+1) Ws - Wd) 2^10, 2 Wd), replicate border;
 *  4. integer hexcone HSV (H8 in 2-degree units 0..179, S8, V8 0..255):
 *     H8' = (H8 + dh) mod 180, S8' = sat8(S8 + ds), V8' = sat8(V8 + dv), back
 *     to RGB;
 *  5. gamma LUT[v] = sat8(rint(255 * pow(v / 255.0, gamma))) in double;
 *  6. if the blur flag is set: [1,2,1]x[1,2,1]/16, one rdiv_he, reflect-101.
 * Per-image setup (the Q32 matrix, crop offsets, the gamma LUT) is compiled
 * on the host by miaug_compile_c2, so transcendental functions are evaluated
 * once, in host double precision; the kernel is integer-only.
 */
typedef struct {
    int64_t aq[6];          /* Q32 inverse affine matrix                          */
    int32_t crop_x, crop_y; /* clamped into [0, W - crop] x [0, H - crop]         */
    int32_t dh, ds, dv;     /* HSV8 shifts                                        */
    int32_t blur;           /* 0 or 1                                             */
    uint8_t gamma_lut[256]; /* LUT of step 5                                      */
} miaug_c2_record;

/* Host-side parameter compile: f[5i..] = {angle_deg, scale, dx, dy, gamma},
 * k[5i..] = {crop_x, crop_y, dh, ds, blur} (miaug_sample_c2 layout) ->
 * out[i] (host array of n records); dv = 0.  Errors: EINVAL, ESHAPE unless
 * 1 <= crop <= min(H, W) and scale != 0. */
int miaug_compile_c2(const float *f, const int32_t *k, int n, int H, int W, int crop, miaug_c2_record *out);

/*   in   device u8 [n][H][W][3]; rec device miaug_c2_record [n]
 *   out  device u8 [n][outsz][outsz][3]
 * Errors: EINVAL null pointers or negative sizes (n == 0 is a no-op);
 * ESHAPE unless 1 <= crop <= min(H, W), 1 <= outsz <= 4096, H, W <= 16384. */
int miaug_ssr_crop_resize_hsv_gamma_blur_u8(const uint8_t *in, int n, int H, int W, const miaug_c2_record *rec,
                                            int crop, int outsz, uint8_t *out, void *stream);

/* Masks of the same chain (Sec. II-A: masks take the image's geometry, with
 * nearest interpolation and no colour op): out[i][y][x] = the mask warped by
 * rec[i]'s matrix (nearest tap of the Q10 position, index (q + 512) >> 10,
 * reflect-101), cropped at (crop_x, crop_y) and resized to outsz x outsz with
 * the nearest rule of the ragged batch (replicate at the crop's edges).
 *   in device u8 [n][H][W]; out device u8 [n][outsz][outsz].
 * Errors as miaug_ssr_crop_resize_hsv_gamma_blur_u8. */
int miaug_ssr_crop_resize_mask_u8(const uint8_t *in, int n, int H, int W, const miaug_c2_record *rec, int crop,
                                  int outsz, uint8_t *out, void *stream);

/* Boxes of the same chain (xyxy, continuous coordinates: pixel i spans
 * [i, i + 1)).  The warp's forward map F is the inverse of rec[i]'s Q32
 * matrix (in double); a corner u maps to F(u - 1/2) + 1/2; a box becomes the
 * bounding box of its four mapped corners, clipped to [0, W] x [0, H], then
 * shifted by (-crop_x, -crop_y), clipped to [0, crop]^2 and scaled by
 * outsz / crop; stored as float.  A box that leaves the image or the crop
 * keeps its slot with zero width or height.
 *   boxes device float [nbox][4]; box_off device int32 [n + 1] (CSR by image);
 *   out device float [nbox][4].  Errors: EINVAL null pointers; ESHAPE sizes. */
int miaug_boxes_ssr_crop_resize(const float *boxes, const int32_t *box_off, int n, int H, int W,
                                const miaug_c2_record *rec, int crop, int outsz, float *out, void *stream);

/* ---------------------------------------------------------------- ragged batch
 * Sec. II-A: images of a detection / segmentation set (uneven sizes) are
 * transformed together with their masks and boxes.  Per image i: Dih4 element
 * (flags) -> optional crop window (crop: the random-sized crop of the
 * paper's detection example, Fig. 2) -> brightness/contrast LUT (ab) ->
 * bilinear resize of the window to out_h x out_w (half-pixel centres,
 * replicate border at the window's edges) -> per-channel normalisation
 * (float)(((double)v/255 - mean_c) / std_c) into float32 CHW.  The mask takes
 * the same Dih4 element and window and a nearest resize (source index
 * (q + 512) >> 10 of the same Q10 position).  Boxes take the Dih4 element
 * (hflip (W-x2, y1, W-x1, y2), vflip, rot90 (y1, W-x2, y2, W-x1), transpose
 * (y1, x1, y2, x2)), the window (shift by (-x0, -y0), clip to [0, w] x
 * [0, h]: a box outside the window keeps its slot with zero width or height)
 * and the scale (out_w/w', out_h/h') of the window (or the whole Dih4 image),
 * in double, stored as float.
 * Images and masks may start at any byte offset.  The kernels stage source
 * rows in the 16-byte aligned blocks that hold their bytes, so they may read
 * (never write) up to 15 bytes before an image's or mask's first byte and
 * after its last; those bytes share a 16-byte block with the image's own, so
 * they lie in mapped memory, and they never enter a result.
 */
typedef struct {
    int32_t n;               /* number of images (0 allowed)                      */
    int32_t out_h, out_w;    /* output size, 1..4096                               */
    const uint8_t *img;      /* device: packed HWC u8 images                       */
    const int64_t *img_off;  /* device: [n] byte offset of image i in img          */
    const int32_t *hw;       /* device: [n][2] = {H_i, W_i}; an image with a side
                                < 1 or >= 2^20, or H_i W_i 3 >= 2^31, is skipped
                                (its outputs are left untouched)                  */
    const int32_t *flags;    /* device: [n][4] Dih4 flags (miaug_sample_d4bc)      */
    const float *ab;         /* device: [n][2] alpha, beta                         */
    const int32_t *crop;     /* device or NULL: [n][4] = {y0, x0, h, w} crop window
                                of the Dih4 image (h = 0: no window for that
                                image); an image whose window is not inside its
                                Dih4 image (or has w < 1) is skipped               */
    const uint8_t *mask;     /* device or NULL: packed HW u8 masks                 */
    const int64_t *mask_off; /* device: [n] byte offsets (when mask != NULL)       */
    const float *boxes;      /* device or NULL: [nbox][4] xyxy                     */
    const int32_t *box_off;  /* device: [n+1] CSR offsets (when boxes != NULL)     */
    float mean[3], stdv[3];  /* normalisation constants                            */
    float *out;              /* device: [n][3][out_h][out_w] float32               */
    uint8_t *out_mask;       /* device: [n][out_h][out_w] (when mask != NULL)      */
    float *out_boxes;        /* device: [nbox][4] (when boxes != NULL)             */
} miaug_ragged_args;

/* Batched form: one persistent launch.  Work items are (image, output tile);
 * images are spread over per-XCD queues, workgroups pop tiles with atomics and
 * steal from other queues when their own is empty.  The queue counters live in
 * the context and are cleared by a fill kernel enqueued before the main
 * kernel, so the call is stream-ordered and graph-capturable.
 * Errors: EINVAL null ctx/args/pointers; ESHAPE bad sizes; EDEVICE launch. */
int miaug_ragged_apply(miaug_ctx *ctx, const miaug_ragged_args *args, void *stream);

/* Multi-channel (instance) masks of a ragged batch: args->mask holds, per
 * image, H x W pixels of `channels` u8 values (one per instance; byte offsets
 * in args->mask_off), and each output pixel of out [n][out_h][out_w][channels]
 * copies the source pixel that the one-channel masks of miaug_ragged_apply
 * take (Dih4 element, crop window, nearest resize).  Reads hw, flags, crop,
 * mask, mask_off, n, out_h, out_w of args; skipped images (see hw and crop)
 * leave their output untouched.  Errors: EINVAL null pointers; ESHAPE sizes
 * or channels outside 1..256. */
int miaug_ragged_masks_u8(const miaug_ragged_args *args, int channels, uint8_t *out, void *stream);

/* Comparison form: the same kernels launched once per image (n launches, no
 * persistence, no queue).  Output is bit-identical to miaug_ragged_apply. */
int miaug_ragged_apply_per_image(miaug_ctx *ctx, const miaug_ragged_args *args, void *stream);

/* hipGraph form: captures miaug_ragged_apply for fixed args (pointers, n,
 * sizes) on `stream`; miaug_graph_launch replays it (reading whatever the
 * argument buffers hold at replay time). */
typedef struct miaug_graph miaug_graph;
int miaug_ragged_graph_create(miaug_ctx *ctx, const miaug_ragged_args *args, void *stream, miaug_graph **out);
int miaug_graph_launch(miaug_graph *g, void *stream);
int miaug_graph_destroy(miaug_graph *g);

/* Autotuner for the batched form: times each launch variant (output tile
 * shape; persistent loop claiming 1, 4 or 8 tiles per atomic, flat grid, or
 * the streaming pipeline with a planner wave; workgroups per CU) on `args`
 * `reps` times, keeps only variants whose output is bit-identical to the
 * per-image form, and stores the fastest in the context (used by later
 * miaug_ragged_apply calls).  Writes the chosen variant index to *chosen, its
 * mean time in ms to *ms and, when `times` is not NULL, every variant's mean
 * time to times[0 .. variant_count-1] (-1 for a variant that failed the
 * parity gate or is switched off).  Synchronises `stream`.  `args->out*` are
 * overwritten. */
int miaug_ragged_autotune(miaug_ctx *ctx, const miaug_ragged_args *args, int reps, void *stream, int *chosen,
                          float *ms, float *times);
/* Number of variants and a variant's description ("tile 32x32, 4 wg/CU");
 * the description of a variant that is switched off begins "off: ". */
int miaug_ragged_variant_count(void);
const char *miaug_ragged_variant_name(int v);
/* Forces a variant (-1 restores the default).  EUNSUPPORTED for a variant that
 * is switched off (MIAUG_FORCE_VARIANT ignores such a variant). */
int miaug_ragged_set_variant(miaug_ctx *ctx, int v);

/* No-allocation form of miaug_ragged_apply, for callers that cannot allocate
 * device memory: code under hipGraph stream capture, tight serving loops and
 * harnesses that forbid hipMalloc.  It needs no context and calls no
 * hipMalloc, hipFree or other allocating routine: the queue counters the
 * persistent kernel uses live in a static device array of the library
 * (MIAUG_NOALLOC_SCRATCH_BYTES bytes on each GPU, held until the process ends),
 * whose address is looked up once per device on the first call made with that
 * device current.  Runs on the calling thread's current HIP device.
 *   args     as miaug_ragged_apply (all device pointers, caller-owned)
 *   variant  launch variant (miaug_ragged_variant_count; the index the
 *            autotuner chose), -1 for the default
 * Output is bit-identical to miaug_ragged_apply with the same variant.  The
 * counters are cleared by a fill kernel enqueued before each launch, so each
 * call starts from zero; calls that overlap in time on one GPU (different
 * streams, or threads without ordering) share the one array and race, and
 * must be serialised by the caller.  The counters do not grow with the
 * batch, so every batch miaug_ragged_apply accepts is accepted.
 * Errors: as miaug_ragged_apply; EINVAL variant out of range; ECAPACITY if a
 * launch form needs more counter memory than the static array holds;
 * EUNSUPPORTED device index >= 64, or a variant that is switched off; EDEVICE
 * symbol lookup or launch failure. */
#define MIAUG_NOALLOC_SCRATCH_BYTES 1024
int miaug_ragged_apply_noalloc(const miaug_ragged_args *args, int variant, void *stream);

/* ---------------------------------------------------------------- differentiable warp + colour
 * Float32 form for training-time augmentation with gradients.  Per image i
 * and channel c, with p_i = {angle_deg, scale, tx, ty, alpha, beta, gamma}:
 *   (sx, sy) = inverse of the shift-scale-rotate map above (tx, ty are
 *   fractions of W, H) evaluated in double at output pixel (x, y), its
 *   fractional parts rounded to float for the bilinear weights;
 *   w = bilinear(x_i[c], sx, sy), taps outside the image read 0;
 *   z = alpha w + beta; y1 = clamp(z, 0, 1); y = y1^gamma (0^gamma = 0).
 *   x, y: device float [n][C][H][W]; params: device float [n][7].
 * Errors: EINVAL null pointers; ESHAPE n, C, H, W out of range. */
int miaug_warpcolor_fwd(const float *x, int n, int C, int H, int W, const float *params, float *y,
                        void *stream);

/* Backward of miaug_warpcolor_fwd given gy = dL/dy.  grad_x (may be NULL)
 * receives dL/dx (the adjoint of the bilinear warp, accumulated per source
 * tile without global atomics); grad_params receives dL/dparams [n][7].
 * Conventions at kinks: the clamp derivative is 0 outside the open interval
 * (0, 1); at y1 = 0 every derivative is 0; the bilinear derivative uses the
 * cell floor(s).  workspace: device memory of miaug_warpcolor_workspace_bytes
 * bytes (contents need not be initialised).  ESHAPE if C > 4. */
size_t miaug_warpcolor_workspace_bytes(int n, int C, int H, int W);
int miaug_warpcolor_bwd(const float *x, int n, int C, int H, int W, const float *params, const float *gy,
                        float *grad_x, float *grad_params, void *workspace, size_t workspace_bytes,
                        void *stream);

/* ---------------------------------------------------------------- elastic + grid distortion
 * Sec. II-C and Fig. 4 (grid distortion and elastic transform; the elastic
 * distortion of Simard et al. 2003 cited in Sec. I).
 *
 * Fields: for image i (global index first_index + i) and field f (0: x,
 * 1: y), noise n_f(y, x) = (16-bit word (e mod 4) of word ((e mod 16)/4) of
 * Philox(counter = {e/16, g, f, 4}, key = {seed, 0})) - 32768, e = y W + x.
 * Taps t_k = rint(2^15 g_k / sum g), g_k = exp(-k^2 / (2 sigma^2)),
 * |k| <= radius.  h = rdiv_he(sum_k t_k n(y, refl(x+k)), 2^15);
 * v = sum_k t_k h(refl(y+k), x); off = rdiv_he(alpha v, 2^20) (Q10 px);
 * refl = reflect-101.
 *   off  device int32 [n][2][H][W] (written)
 *   workspace device, miaug_elastic_workspace_bytes bytes (int16 pass data).
 * Errors: EINVAL; ESHAPE unless 1 <= radius <= 200, sigma > 0, 0 <= alpha <= 65535;
 * ECAPACITY small workspace. */
size_t miaug_elastic_workspace_bytes(int n, int H, int W);
int miaug_elastic_fields(uint64_t seed, uint64_t first_index, int n, int H, int W, double sigma, int alpha,
                         int radius, int32_t *off, void *workspace, size_t workspace_bytes, void *stream);

/* Approximate fields (opt-in): each axis's Gaussian is replaced by a cascade
 * of three box filters (Wells, IEEE PAMI 1986), widths w_i from Kovesi
 * ("Fast almost-Gaussian filtering", DICTA 2010): w_ideal = sqrt(4 sigma^2 +
 * 1), wl = the largest odd integer <= w_ideal, wu = wl + 2, the first
 * m = round((12 sigma^2 - 3 wl^2 - 12 wl - 9) / (-4 wl - 4)) passes use wl, the
 * others wu.  A pass is pass(x) = rdiv_he(sum over |k| <= r of
 * in[refl(x + k)], 2r + 1) with r = w / 2.  Per field: the noise of
 * miaug_elastic_fields -> three passes along each row -> three passes along
 * each column -> v; off = rdiv_he(alpha v, 2^5) (Q10 px, the scale of the
 * exact field).  O(1) work per pixel and pass instead of 2 (2 radius + 1).
 *   off  device int32 [n][2][H][W] (written)
 *   workspace device, miaug_elastic_box_workspace_bytes bytes.
 * Errors: EINVAL; ESHAPE unless sigma > 0 with every box radius <= 255,
 * 0 <= alpha <= 65535, W <= 7168; ECAPACITY small workspace. */
size_t miaug_elastic_box_workspace_bytes(int n, int H, int W);
int miaug_elastic_fields_box(uint64_t seed, uint64_t first_index, int n, int H, int W, double sigma, int alpha,
                             int32_t *off, void *workspace, size_t workspace_bytes, void *stream);

/* Grid tables: for each image, 5 cells per axis of width cw = W/5, knots
 * S_0 = 0, S_{k+1} = S_k + cw d_k (not renormalised); pixel x maps to
 * src = S_k + (x + 1/2 - k cw) d_k - 1/2 with k = min(floor((x+1/2)/cw), 4),
 * in double, q = rint(src 2^10).
 *   grid device double [n][10] (miaug_sample_grid layout); mapx device int32
 *   [n][W]; mapy device int32 [n][H]. */
int miaug_grid_tables(const double *grid, int n, int H, int W, int32_t *mapx, int32_t *mapy, void *stream);

/* u8 chain: e = elastic remap of the image by off (source position
 * ((x<<10) + off_x, (y<<10) + off_y), bilinear, reflect-101), rounded to u8;
 * out = grid remap of e (source (mapx[x], mapy[y]), bilinear, reflect-101).
 * The mask (optional) takes the same two remaps with nearest sampling.
 *   img device u8 [n][H][W][C] (C in {1,3,4}); mask device u8 [n][H][W] or NULL
 *   out device u8 like img; out_mask like mask.  The image is read in the
 *   aligned 4-byte words that hold its bytes (at most 3 bytes on either side
 *   of it, inside those words; device allocations are word granular).
 * per_image != 0 launches the kernel once per image (comparison form). */
int miaug_elastic_grid_u8(const uint8_t *img, const uint8_t *mask, int n, int H, int W, int C,
                          const int32_t *off, const int32_t *mapx, const int32_t *mapy, uint8_t *out,
                          uint8_t *out_mask, int per_image, void *stream);

/* Boxes under the same distortion (Sec. II-A: boxes follow the image).  A box
 * (xyxy, continuous coordinates) covers the source pixels whose centres lie
 * in [x1, x2) x [y1, y2); output pixel (x, y) reaches, on the mask path, the
 * source pixel of the grid's nearest tap followed by the elastic map's
 * nearest tap (reflect-101 both times).  The transformed box is the bounding
 * box [min x, min y, max x + 1, max y + 1] of the output pixels whose source
 * pixel it covers: the box transformed as its own mask.  A box no output
 * pixel reaches becomes (0, 0, 0, 0) and keeps its slot.
 *   boxes device float [nbox][4]; box_off device int32 [n + 1]; off, mapx,
 *   mapy as miaug_elastic_grid_u8; out device float [nbox][4] (also used as
 *   int32 accumulators while the call runs).  Errors: EINVAL, ESHAPE. */
int miaug_boxes_elastic_grid(const float *boxes, const int32_t *box_off, int n, int H, int W, const int32_t *off,
                             const int32_t *mapx, const int32_t *mapy, float *out, void *stream);

/* Float copy of the chain without u8 rounding (same Q10 positions, dyadic
 * weights), CHW float32, and its adjoint w.r.t. the image (fields and grid
 * are random draws, not parameters; the training-time form of Sec. II-C's
 * distortions).  The backward has one writer per element and no global
 * float atomics: dL/de of the grid step as a gather over the grid's inverse
 * ranges, then dL/dx of the elastic step per source tile over the window
 * the field's largest displacement allows, summed in LDS (the order of
 * those sums may vary between runs).  workspace (contents need not be
 * initialised): dL/de and small tables, miaug_chain_f32_workspace_bytes.
 * Errors: EINVAL null pointers; ESHAPE n > 65535, H or W >= 2^20 or
 * H W > 2^30; ECAPACITY workspace too small. */
int miaug_elastic_grid_f32_fwd(const float *x, int n, int C, int H, int W, const int32_t *off,
                               const int32_t *mapx, const int32_t *mapy, float *y, void *workspace,
                               size_t workspace_bytes, void *stream);
size_t miaug_chain_f32_workspace_bytes(int n, int C, int H, int W);
int miaug_elastic_grid_f32_bwd(const float *gy, int n, int C, int H, int W, const int32_t *off,
                               const int32_t *mapx, const int32_t *mapy, float *grad_x, void *workspace,
                               size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------- image statistics
 * Per image and channel: sum (uint64), min, max (int32) and a 256-bin
 * histogram (uint32), reduced with wavefront and workgroup reductions.
 *   img device u8 [n][npix][C]; sum device uint64 [n][C]; mn, mx device
 *   int32 [n][C]; hist device uint32 [n][C][256] (any of the four may be NULL). */
int miaug_image_stats_u8(const uint8_t *img, int n, int64_t npix, int C, uint64_t *sum, int32_t *mn,
                         int32_t *mx, uint32_t *hist, void *stream);

/* ---------------------------------------------------------------- op-list pipelines
 * The paper's usage pattern (Sec. I; Sec. II and the listings of its
 * figures): a user lists transforms, each applied with its own probability
 * and a parameter drawn from a range, and applies the composition to an image
 * together with its masks and boxes.  A pipeline compiles such a list, by
 * pattern, onto one of the fused chains above (brackets: optional; the ops
 * must come in this order):
 *   MIAUG_PIPE_DIH4      [HFLIP] [VFLIP] [ROT90] [TRANSPOSE] [BRIGHT_CONTRAST]
 *                        [SHIFT_RGB] [GAMMA] [TO_GRAY]
 *                        dense u8 images (and masks, Dih4 only) -> u8,
 *                        miaug_d4_bc_u8 or, with colour ops, miaug_d4_lut_u8
 *   MIAUG_PIPE_RAGGED    [HFLIP] [VFLIP] [ROT90] [TRANSPOSE] [SIZED_CROP]
 *                        [BRIGHT_CONTRAST] RESIZE [NORMALIZE]
 *                        ragged RGB u8 + masks + boxes -> f32 NCHW, miaug_ragged_apply
 *   MIAUG_PIPE_U8CHAIN   [SSR] CROP RESIZE [HSV] [GAMMA] [BLUR3]
 *                        dense RGB u8 (+ masks, + boxes CSR by image) -> u8
 *                        (square crop and output),
 *                        miaug_ssr_crop_resize_hsv_gamma_blur_u8,
 *                        miaug_ssr_crop_resize_mask_u8, miaug_boxes_ssr_crop_resize
 *   MIAUG_PIPE_DISTORT   ELASTIC [GRID] | GRID
 *                        dense u8 images (and masks, boxes) -> u8,
 *                        miaug_elastic_grid_u8, miaug_boxes_elastic_grid
 *   MIAUG_PIPE_WARP      ROTATE | SSR (alone)
 *                        dense u8 images (and masks, nearest) -> u8 of the same
 *                        shape, miaug_warp_affine_u8
 *   MIAUG_PIPE_PAD       PAD
 *                        dense u8 images (and masks, label 0) -> u8
 *                        [n][max(H, out_h)][max(W, out_w)][C], miaug_pad_u8
 *   MIAUG_PIPE_HSV       HSV (alone)
 *                        dense RGB u8 (masks copied unchanged) -> u8,
 *                        miaug_hsv_shift_u8
 *   MIAUG_PIPE_BLUR      BLUR3 | BLUR5 (alone)
 *                        dense u8 images (masks copied unchanged) -> u8,
 *                        miaug_blur_u8
 * Any other list is rejected with MIAUG_EUNSUPPORTED and a message naming
 * the first op that does not fit.
 *
 * Op fields (p is the probability of applying the op; a skipped op takes
 * its identity parameters):
 *   HFLIP, VFLIP, TRANSPOSE   p.
 *   ROT90             p; k uniform in {lo[0] .. hi[0]} (integers in 0..3).
 *   BRIGHT_CONTRAST   p; alpha in [lo[0], hi[0]], beta in [lo[1], hi[1]]
 *                     (pixel units); skipped: (1, 0).
 *   SSR               p; angle_deg in [lo[0], hi[0]], scale in [lo[1], hi[1]],
 *                     dx, dy in [lo[2], hi[2]], [lo[3], hi[3]] (fractions of
 *                     W, H); skipped: identity.  In the u8 chain bilinear with
 *                     reflect-101 only; alone (WARP) any interp and border.
 *   ROTATE            p; angle_deg in [lo[0], hi[0]] (scale 1, no shift);
 *                     interp, border; skipped: identity.
 *   SHIFT_RGB         p; channel c moves by U[lo[c], hi[c]] (c < 3, pixel
 *                     units, rounded in the LUT); skipped: 0.
 *   TO_GRAY           p; BT.601 luma to all channels (RGB only).
 *   PAD               to at least out_h x out_w (border; lo[0] = constant
 *                     value); p must be 1; no draws.
 *   CROP              out_h x out_w window at offsets uniform in
 *                     {0 .. H - out_h} x {0 .. W - out_w}; p must be 1.
 *   SIZED_CROP        p; random-sized crop of the Dih4 image (H' x W'):
 *                     area fraction in [lo[0], hi[0]] (0 < lo, hi <= 1),
 *                     aspect ratio w/h log-uniform in [lo[1], hi[1]].  Try t
 *                     (t < 10) reads the four words of Philox block 16 j + 1 + t:
 *                     s = lo0 + (hi0 - lo0) u(word 0), r = exp(log lo1 +
 *                     (log hi1 - log lo1) u(word 1)), A = H' W' s,
 *                     w = floor(sqrt(A r) + 1/2), h = floor(sqrt(A / r) + 1/2);
 *                     the first try with 1 <= w <= W', 1 <= h <= H' takes
 *                     crop_y = below(word 2, H' - h + 1), crop_x = below(word 3,
 *                     W' - w + 1).  No try fits: a centred window with
 *                     h = max(1, floor(W' / lo1 + 1/2)) if W'/H' < lo1,
 *                     w = max(1, floor(H' hi1 + 1/2)) if W'/H' > hi1, else the
 *                     whole image.  u(x) = (x >> 11) 2^-53, below(x, m) =
 *                     ((x >> 32) m) >> 32.  Skipped: crop_h = crop_w = 0.
 *   RESIZE            to out_h x out_w; bilinear (masks: nearest).
 *   HSV               p; dh = rint(U[lo[0], hi[0]]) (2-degree units),
 *                     ds = rint(U[lo[1], hi[1]]), dv = rint(U[lo[2], hi[2]]).
 *   GAMMA             p; gamma in [lo[0], hi[0]]; skipped: 1.
 *   BLUR3, BLUR5      p (3x3 / 5x5 binomial).
 *   ELASTIC           alpha = lo[0] (pixels, integer 0..65535), sigma = lo[1],
 *                     radius = lo[2] (0: ceil(3 sigma), at most 200); p must be 1;
 *                     hi[0] != 0 selects the box-cascade approximation
 *                     (miaug_elastic_fields_box; radius unused).
 *   GRID              p; 5 cells per axis, factors 1 + U[-lo[0], lo[0]]
 *                     (0 <= lo[0] < 1); skipped: all 1.
 *   NORMALIZE         mean = lo[0..2], std = hi[0..2]; p must be 1.
 * Draws: op number j of the list uses Philox draws 16 j (its Bernoulli gate,
 * only when p < 1) and 16 j + 1, 16 j + 2, ... (its parameters, in the order
 * listed above), with the generator of the sampler section. */
enum {
    MIAUG_OP_HFLIP = 1, MIAUG_OP_VFLIP = 2, MIAUG_OP_ROT90 = 3, MIAUG_OP_TRANSPOSE = 4, MIAUG_OP_SSR = 5,
    MIAUG_OP_CROP = 6, MIAUG_OP_RESIZE = 7, MIAUG_OP_BRIGHT_CONTRAST = 8, MIAUG_OP_HSV = 9, MIAUG_OP_GAMMA = 10,
    MIAUG_OP_BLUR3 = 11, MIAUG_OP_BLUR5 = 12, MIAUG_OP_ELASTIC = 13, MIAUG_OP_GRID = 14, MIAUG_OP_NORMALIZE = 15,
    MIAUG_OP_SIZED_CROP = 16, MIAUG_OP_SHIFT_RGB = 17, MIAUG_OP_TO_GRAY = 18, MIAUG_OP_PAD = 19, MIAUG_OP_ROTATE = 20
};
enum { MIAUG_INTERP_BILINEAR = 0, MIAUG_INTERP_NEAREST = 1 };
enum { MIAUG_BORDER_REFLECT101 = 0, MIAUG_BORDER_CONSTANT = 1 };
enum {
    MIAUG_PIPE_DIH4 = 1, MIAUG_PIPE_RAGGED = 2, MIAUG_PIPE_U8CHAIN = 3, MIAUG_PIPE_DISTORT = 4, MIAUG_PIPE_WARP = 5,
    MIAUG_PIPE_PAD = 6, MIAUG_PIPE_HSV = 7, MIAUG_PIPE_BLUR = 8
};

typedef struct {
    uint32_t kind;         /* MIAUG_OP_*                                          */
    float p;               /* probability of applying the op                     */
    float lo[4], hi[4];    /* parameter ranges (see above)                        */
    uint32_t interp;       /* MIAUG_INTERP_*                                      */
    uint32_t border;       /* MIAUG_BORDER_*                                      */
    int32_t out_h, out_w;  /* CROP, RESIZE                                        */
} miaug_op;

/* Per-sample parameters (host record; what miaug_sample writes and
 * miaug_apply consumes).  Fields an op list does not use keep identity
 * values. */
typedef struct {
    uint64_t seed, index;           /* generator key and global sample index     */
    int32_t flags[4];               /* hflip, vflip, rot90 k, transpose          */
    float alpha, beta;              /* brightness/contrast                       */
    float angle, scale, dx, dy;     /* shift-scale-rotate                        */
    int32_t crop_x, crop_y;         /* crop offsets                              */
    int32_t dh, ds, dv;             /* HSV shifts                                */
    float gamma;                    /* gamma                                     */
    int32_t blur;                   /* 3x3 blur flag                             */
    int32_t crop_h, crop_w;         /* random-sized crop window size (0: none);
                                       its offsets are crop_y, crop_x            */
    float shift[3];                 /* ShiftRGB channel shifts                   */
    int32_t gray;                   /* grayscale flag                            */
    double grid[10];                /* grid factors: x d_0..d_4, y d_0..d_4      */
} miaug_params;

typedef struct miaug_pipeline miaug_pipeline;
/* Compiles `ops` (host array, copied).  ctx may be NULL for a pipeline that
 * only samples.  Errors: EINVAL (NULL out, n_ops < 1, bad field values),
 * EUNSUPPORTED (list fits no chain). */
int miaug_pipeline_create(miaug_ctx *ctx, const miaug_op *ops, int n_ops, miaug_pipeline **out);
/* Frees the pipeline and its device buffers (synchronises the device). */
int miaug_pipeline_destroy(miaug_pipeline *p);
/* MIAUG_PIPE_* of a pipeline (or a negative status). */
int miaug_pipeline_kind(const miaug_pipeline *p);
/* Bytes of n parameter records: n * sizeof(miaug_params). */
size_t miaug_param_bytes(const miaug_pipeline *p, int n);
/* Draws the records of samples first_index .. first_index + n - 1.
 *   hw  host int32 [n][2] source sizes (needed when the list has CROP; may be
 *       NULL otherwise); params host [n] records (written).  Host only. */
int miaug_sample(const miaug_pipeline *p, uint64_t seed, uint64_t first_index, int n, const int32_t *hw,
                 miaug_params *params);

/* A batch.  Dense pipelines (DIH4, U8CHAIN, DISTORT) read img as
 * [n][H][W][channels] (mask [n][H][W]); the ragged pipeline reads the packed
 * layout of miaug_ragged_args (img_off, hw, mask_off, box_off device arrays,
 * channels = 3).  All pointers are device pointers. */
typedef struct {
    int32_t n, channels, H, W;
    const uint8_t *img;
    const int64_t *img_off;
    const int32_t *hw;
    const uint8_t *mask;      /* NULL: no masks                                   */
    const int64_t *mask_off;
    const float *boxes;       /* NULL: no boxes (ragged, u8 and distortion chains) */
    const int32_t *box_off;
} miaug_batch_in;
/* Outputs (device): img u8 like the input (DIH4: image i keeps its byte range,
 * with shape (W, H) when its element swaps axes; DISTORT: same shape), u8
 * [n][s][s][3] (U8CHAIN, s = RESIZE size) or float32 [n][3][out_h][out_w]
 * (RAGGED); mask and boxes as the chains above. */
typedef struct {
    void *img;
    uint8_t *mask;
    float *boxes;
} miaug_batch_out;

/* Applies the pipeline with host records `params` [in->n] (copied to the
 * device through a pinned staging buffer owned by the pipeline; the call
 * waits for the previous call's copy before reusing it).  Device buffers of
 * the chain (parameter records, elastic fields and tables) are allocated on
 * first use and grown when a larger batch comes.  Errors: EINVAL, ESHAPE,
 * EUNSUPPORTED (mask or boxes the chain cannot take, records of a DISTORT
 * batch that are not consecutive samples of one seed), EDEVICE. */
int miaug_apply(miaug_pipeline *p, const miaug_batch_in *in, const miaug_params *params, miaug_batch_out *out,
                void *stream);
/* Comparison form: one launch per image; identical output. */
int miaug_apply_per_image(miaug_pipeline *p, const miaug_batch_in *in, const miaug_params *params,
                          miaug_batch_out *out, void *stream);

/* hipGraph of miaug_apply for a fixed batch and outputs: the graph copies the
 * records from its own pinned buffer, so each launch takes new records.
 * miaug_pipeline_graph_launch waits for the previous launch's copy, fills
 * the buffer from `params` and replays the graph on `stream`.  A DISTORT
 * pipeline with ELASTIC is not capturable (EUNSUPPORTED): its noise stream is
 * a launch argument. */
typedef struct miaug_pipeline_graph miaug_pipeline_graph;
int miaug_pipeline_graph_capture(miaug_pipeline *p, const miaug_batch_in *in, const miaug_batch_out *out,
                                 void *stream, miaug_pipeline_graph **g);
int miaug_pipeline_graph_launch(miaug_pipeline_graph *g, const miaug_params *params, void *stream);
int miaug_pipeline_graph_destroy(miaug_pipeline_graph *g);

/* Tunes the launch of the pipeline's chain on this batch (the ragged
 * autotuner for MIAUG_PIPE_RAGGED; other chains have one launch form and
 * return at once).  Overwrites the outputs; synchronises `stream`. */
int miaug_pipeline_autotune(miaug_pipeline *p, const miaug_batch_in *in, const miaug_params *params,
                            miaug_batch_out *out, int reps, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MIAUG_H */
