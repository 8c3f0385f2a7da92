/*
 * oracle.c -- plain, slow, single-threaded CPU oracle for the batched image
 * augmentation hot path (Buslaev et al., "Albumentations: fast and flexible
 * image augmentations", arXiv:1809.06839).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark may load this library.  The product path (the HIP
 * library under paper_1809_06839_amd/) shares no code, header, table or
 * constant generator with this file and never calls it.
 *
 * The paper names the operations (Abstract; Sec. I; Sec. II and its
 * subsections A-C; Table I) and states that masks and boxes follow the
 * geometry of the image (Sec. II-A, Sec. II-B), but it gives no formula.  Every
 * arithmetic definition below is therefore a stated reading: integer
 * fixed-point resampling with round-half-even and saturation, so that an
 * independent GPU implementation can be compared bit for bit.  Floating point
 * appears only where a reading fixes it (IEEE double for parameter setup and
 * LUT construction, and the fp64 differentiable path).
 *
 * Style rules: every op is its own function that materialises its output;
 * nothing is fused, tiled or reordered; coordinates are int64; this file is
 * compiled with -O2 -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define F_BITS 10                 /* sub-pixel bits of every fixed-point coordinate */
#define F_ONE (1 << F_BITS)

/* ------------------------------------------------------------------------ */
/* Rounding and border primitives                                            */
/* ------------------------------------------------------------------------ */

/* Nearest integer to n/d (d > 0), ties to even, built on floor division. */
int64_t or_rdiv_he(int64_t n, int64_t d)
{
    int64_t q = n / d;
    int64_t r = n % d;
    if (r < 0) { q -= 1; r += d; }          /* make q = floor(n/d), 0 <= r < d */
    if (2 * r > d || (2 * r == d && (q & 1))) q += 1;
    return q;
}

int64_t or_rshr_he(int64_t n, int k) { return or_rdiv_he(n, (int64_t)1 << k); }

static int sat8(int64_t v) { return v < 0 ? 0 : (v > 255 ? 255 : (int)v); }

/* Reflect-101 border (the edge pixel is not repeated). */
int64_t or_reflect101(int64_t i, int64_t n)
{
    if (n == 1) return 0;
    int64_t p = 2 * n - 2;
    i = ((i % p) + p) % p;
    if (i >= n) i = p - i;
    return i;
}

static int64_t clampi(int64_t i, int64_t n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

static int64_t floor_shift(int64_t q, int k) { return (q - (((q % (1 << k)) + (1 << k)) % (1 << k))) / (1 << k); }
static int64_t frac_bits(int64_t q, int k) { return ((q % (1 << k)) + (1 << k)) % (1 << k); }

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the sampler         */
/* ------------------------------------------------------------------------ */

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(0xD2E7470EE14C6C93ULL, c0, &hi0, &lo0);
        mulhilo64(0xCA5A826395121157ULL, c2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B97F4A7C15ULL;
        k1 += 0xBB67AE8584CAA73BULL;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Streams of the counter word 3. */
#define STREAM_PARAMS 0u
#define STREAM_NOISE 4u

/* Raw 64-bit draw number `draw` of sample `index` in stream `stream`. */
uint64_t or_draw_u64(uint64_t seed, uint64_t stream, uint64_t index, uint64_t draw)
{
    uint64_t ctr[4] = {draw, index, 0, stream};
    uint64_t key[2] = {seed, 0};
    uint64_t out[4];
    or_philox4x64_10(ctr, key, out);
    return out[0];
}

static double draw_uniform(uint64_t seed, uint64_t index, uint64_t draw)
{
    uint64_t x = or_draw_u64(seed, STREAM_PARAMS, index, draw);
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);        /* [0, 1) */
}

static int draw_bern(uint64_t seed, uint64_t index, uint64_t draw, double p)
{
    return draw_uniform(seed, index, draw) < p;
}

static int32_t draw_int(uint64_t seed, uint64_t index, uint64_t draw, uint32_t n)
{
    uint64_t x = or_draw_u64(seed, STREAM_PARAMS, index, draw);
    return (int32_t)(((x >> 32) * (uint64_t)n) >> 32);
}

static float draw_range(uint64_t seed, uint64_t index, uint64_t draw, double lo, double hi)
{
    return (float)(lo + (hi - lo) * draw_uniform(seed, index, draw));
}

/* Dih4 + brightness/contrast parameters (the small plain pipeline and the
 * ragged pipeline): flags[i] = {hflip, vflip, rot90 k, transpose},
 * ab[i] = {alpha, beta}. */
void or_sample_d4bc(uint64_t seed, uint64_t first, int n, int32_t *flags, float *ab)
{
    for (int i = 0; i < n; ++i) {
        uint64_t g = first + (uint64_t)i;
        flags[4 * i + 0] = draw_bern(seed, g, 0, 0.5);
        flags[4 * i + 1] = draw_bern(seed, g, 1, 0.5);
        flags[4 * i + 2] = draw_int(seed, g, 2, 4);
        flags[4 * i + 3] = draw_bern(seed, g, 3, 0.5);
        ab[2 * i + 0] = draw_range(seed, g, 4, 0.8, 1.2);
        ab[2 * i + 1] = draw_range(seed, g, 5, -51.0, 51.0);
    }
}

/* Full u8 pipeline parameters: f[i] = {angle_deg, scale, dx, dy, gamma},
 * k[i] = {crop_x, crop_y, dh, ds, blur}. */
void or_sample_c2(uint64_t seed, uint64_t first, int n, int crop_range, float *f, int32_t *k)
{
    for (int i = 0; i < n; ++i) {
        uint64_t g = first + (uint64_t)i;
        f[5 * i + 0] = draw_range(seed, g, 0, -45.0, 45.0);
        f[5 * i + 1] = draw_range(seed, g, 1, 0.9, 1.1);
        f[5 * i + 2] = draw_range(seed, g, 2, -0.0625, 0.0625);
        f[5 * i + 3] = draw_range(seed, g, 3, -0.0625, 0.0625);
        k[5 * i + 0] = draw_int(seed, g, 4, (uint32_t)(crop_range + 1));
        k[5 * i + 1] = draw_int(seed, g, 5, (uint32_t)(crop_range + 1));
        k[5 * i + 2] = (int32_t)rint((double)draw_range(seed, g, 6, -20.0, 20.0));
        k[5 * i + 3] = (int32_t)rint((double)draw_range(seed, g, 7, -30.0, 30.0));
        f[5 * i + 4] = draw_range(seed, g, 8, 0.8, 1.2);
        k[5 * i + 4] = draw_bern(seed, g, 9, 0.3);
    }
}

/* Differentiable pipeline parameters: f[i] = {angle_deg, scale, tx, ty,
 * alpha, beta, gamma}. */
void or_sample_wc(uint64_t seed, uint64_t first, int n, float *f)
{
    for (int i = 0; i < n; ++i) {
        uint64_t g = first + (uint64_t)i;
        f[7 * i + 0] = draw_range(seed, g, 0, -45.0, 45.0);
        f[7 * i + 1] = draw_range(seed, g, 1, 0.9, 1.1);
        f[7 * i + 2] = draw_range(seed, g, 2, -0.0625, 0.0625);
        f[7 * i + 3] = draw_range(seed, g, 3, -0.0625, 0.0625);
        f[7 * i + 4] = draw_range(seed, g, 4, 0.8, 1.2);
        f[7 * i + 5] = draw_range(seed, g, 5, -0.2, 0.2);
        f[7 * i + 6] = draw_range(seed, g, 6, 0.8, 1.2);
    }
}

/* Grid-distortion factors: f[i] = {x factors d_0..d_4, y factors d_0..d_4},
 * each 1 + U[-limit, limit]. */
void or_sample_grid(uint64_t seed, uint64_t first, int n, double limit, double *f)
{
    for (int i = 0; i < n; ++i) {
        uint64_t g = first + (uint64_t)i;
        for (int j = 0; j < 10; ++j)
            f[10 * i + j] = 1.0 + (double)draw_range(seed, g, (uint64_t)j, -limit, limit);
    }
}

/* Elastic noise value of field `field` (0: x, 1: y) at element e = y*W + x. */
int32_t or_noise16(uint64_t seed, uint64_t index, int field, int64_t e)
{
    uint64_t ctr[4] = {(uint64_t)(e / 16), index, (uint64_t)field, STREAM_NOISE};
    uint64_t key[2] = {seed, 0};
    uint64_t out[4];
    or_philox4x64_10(ctr, key, out);
    uint64_t word = out[(e % 16) / 4];
    return (int32_t)((word >> (16 * (e % 4))) & 0xFFFFu) - 32768;
}

/* ------------------------------------------------------------------------ */
/* Dih4 geometry (Sec. II-B: random element of the dihedral group; Table I   */
/* HorizontalFlip / VerticalFlip).  Each op materialises a new array.        */
/* ------------------------------------------------------------------------ */

void or_hflip(const uint8_t *in, int H, int W, int C, uint8_t *out)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < C; ++c)
                out[((int64_t)y * W + x) * C + c] = in[((int64_t)y * W + (W - 1 - x)) * C + c];
}

void or_vflip(const uint8_t *in, int H, int W, int C, uint8_t *out)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < C; ++c)
                out[((int64_t)y * W + x) * C + c] = in[((int64_t)(H - 1 - y) * W + x) * C + c];
}

/* One counter-clockwise quarter turn: output shape (W, H), out[i][j] = in[j][W-1-i]. */
void or_rot90(const uint8_t *in, int H, int W, int C, uint8_t *out)
{
    for (int i = 0; i < W; ++i)
        for (int j = 0; j < H; ++j)
            for (int c = 0; c < C; ++c)
                out[((int64_t)i * H + j) * C + c] = in[((int64_t)j * W + (W - 1 - i)) * C + c];
}

/* Transpose: output shape (W, H), out[i][j] = in[j][i]. */
void or_transpose(const uint8_t *in, int H, int W, int C, uint8_t *out)
{
    for (int i = 0; i < W; ++i)
        for (int j = 0; j < H; ++j)
            for (int c = 0; c < C; ++c)
                out[((int64_t)i * H + j) * C + c] = in[((int64_t)j * W + i) * C + c];
}

/* hflip -> vflip -> rot90^k -> transpose, applied one after the other.
 * out must hold H*W*C bytes; *Ho, *Wo receive the output shape. */
void or_d4(const uint8_t *in, int H, int W, int C, int hflip, int vflip, int k, int transpose,
           uint8_t *out, int *Ho, int *Wo)
{
    size_t n = (size_t)H * W * C;
    uint8_t *a = (uint8_t *)malloc(n), *b = (uint8_t *)malloc(n);
    memcpy(a, in, n);
    int h = H, w = W;
    if (hflip) { or_hflip(a, h, w, C, b); uint8_t *t = a; a = b; b = t; }
    if (vflip) { or_vflip(a, h, w, C, b); uint8_t *t = a; a = b; b = t; }
    for (int r = 0; r < (k & 3); ++r) {
        or_rot90(a, h, w, C, b); uint8_t *t = a; a = b; b = t;
        int s = h; h = w; w = s;
    }
    if (transpose) {
        or_transpose(a, h, w, C, b); uint8_t *t = a; a = b; b = t;
        int s = h; h = w; w = s;
    }
    memcpy(out, a, n);
    *Ho = h; *Wo = w;
    free(a); free(b);
}

/* Boxes (xyxy, continuous pixel coordinates) follow the same Dih4 ops and a
 * final resize to (Hd, Wd) (Sec. II-A: boxes follow spatial transforms). */
/* One box (double xyxy, in place) under the Dih4 ops one after the other;
 * (*h, *w) go from the source size to the Dih4 image's size. */
static void box_d4(double *x1, double *y1, double *x2, double *y2, double *h, double *w, int hflip, int vflip,
                   int k, int transpose)
{
    if (hflip) { double a = *w - *x2, b = *w - *x1; *x1 = a; *x2 = b; }
    if (vflip) { double a = *h - *y2, b = *h - *y1; *y1 = a; *y2 = b; }
    for (int r = 0; r < (k & 3); ++r) {
        double nx1 = *y1, ny1 = *w - *x2, nx2 = *y2, ny2 = *w - *x1;
        *x1 = nx1; *y1 = ny1; *x2 = nx2; *y2 = ny2;
        double s = *h; *h = *w; *w = s;
    }
    if (transpose) {
        double nx1 = *y1, ny1 = *x1, nx2 = *y2, ny2 = *x2;
        *x1 = nx1; *y1 = ny1; *x2 = nx2; *y2 = ny2;
        double s = *h; *h = *w; *w = s;
    }
}

void or_boxes_d4_resize(const float *boxes, int nb, int H, int W, int hflip, int vflip, int k,
                        int transpose, int Hd, int Wd, float *out)
{
    for (int i = 0; i < nb; ++i) {
        double x1 = boxes[4 * i + 0], y1 = boxes[4 * i + 1], x2 = boxes[4 * i + 2], y2 = boxes[4 * i + 3];
        double h = H, w = W;
        box_d4(&x1, &y1, &x2, &y2, &h, &w, hflip, vflip, k, transpose);
        double sx = (double)Wd / w, sy = (double)Hd / h;
        out[4 * i + 0] = (float)(x1 * sx);
        out[4 * i + 1] = (float)(y1 * sy);
        out[4 * i + 2] = (float)(x2 * sx);
        out[4 * i + 3] = (float)(y2 * sy);
    }
}

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Boxes under Dih4, then a crop window win = {y0, x0, h, w} of the Dih4 image
 * (the random-sized crop of Fig. 2's detection pipeline), then a resize of the
 * window to (Hd, Wd).  The crop shifts the box by (-x0, -y0) and clips it to
 * the window; a box outside the window becomes one of zero width or height
 * (it keeps its slot, so the box count per image is unchanged). */
void or_boxes_d4_crop_resize(const float *boxes, int nb, int H, int W, int hflip, int vflip, int k,
                             int transpose, const int32_t *win, int Hd, int Wd, float *out)
{
    for (int i = 0; i < nb; ++i) {
        double x1 = boxes[4 * i + 0], y1 = boxes[4 * i + 1], x2 = boxes[4 * i + 2], y2 = boxes[4 * i + 3];
        double h = H, w = W;
        box_d4(&x1, &y1, &x2, &y2, &h, &w, hflip, vflip, k, transpose);
        if (win) {
            h = win[2];
            w = win[3];
            x1 = clampd(x1 - win[1], 0.0, w);
            x2 = clampd(x2 - win[1], 0.0, w);
            y1 = clampd(y1 - win[0], 0.0, h);
            y2 = clampd(y2 - win[0], 0.0, h);
        }
        double sx = (double)Wd / w, sy = (double)Hd / h;
        out[4 * i + 0] = (float)(x1 * sx);
        out[4 * i + 1] = (float)(y1 * sy);
        out[4 * i + 2] = (float)(x2 * sx);
        out[4 * i + 3] = (float)(y2 * sy);
    }
}

/* ------------------------------------------------------------------------ */
/* Point ops: brightness/contrast, gamma (Table I Brightness, Gamma rows;    */
/* Sec. II colour/contrast/brightness), normalisation.                       */
/* ------------------------------------------------------------------------ */

/* LUT[v] = sat8(rint(alpha*v + beta)) in IEEE double. */
void or_bc_lut(float alpha, float beta, uint8_t *lut)
{
    for (int v = 0; v < 256; ++v) {
        double t = (double)alpha * (double)v + (double)beta;
        lut[v] = (uint8_t)sat8((int64_t)rint(t));
    }
}

/* LUT[v] = sat8(rint(255 * (v/255)^gamma)) in IEEE double. */
void or_gamma_lut(float gamma, uint8_t *lut)
{
    for (int v = 0; v < 256; ++v) {
        double t = 255.0 * pow((double)v / 255.0, (double)gamma);
        lut[v] = (uint8_t)sat8((int64_t)rint(t));
    }
}

void or_apply_lut(const uint8_t *in, int64_t n, const uint8_t *lut, uint8_t *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = lut[in[i]];
}

/* ShiftRGB (Table I): channel c of every pixel moves by shift[c] (pixel
 * units), rounded half to even and saturated: lut[c*256 + v] =
 * sat8(rint(v + shift_c)) in IEEE double. */
void or_shift_rgb_lut(const float *shift, int C, uint8_t *lut)
{
    for (int c = 0; c < C; ++c)
        for (int v = 0; v < 256; ++v)
            lut[c * 256 + v] = (uint8_t)sat8((int64_t)rint((double)v + (double)shift[c]));
}

/* Per-channel LUT on an interleaved image: out[p*C + c] = lut[c*256 + in[p*C + c]]. */
void or_apply_lut_c(const uint8_t *in, int64_t npix, int C, const uint8_t *lut, uint8_t *out)
{
    for (int64_t p = 0; p < npix; ++p)
        for (int c = 0; c < C; ++c) out[p * C + c] = lut[c * 256 + in[p * C + c]];
}

/* Grayscale (Table I): BT.601 luma with the weights 0.299, 0.587, 0.114
 * quantised to Q14 (4899, 9617, 1868; they sum to 2^14, so a grey pixel
 * keeps its value), rounded half up; the luma goes to all three channels. */
void or_gray_u8(const uint8_t *in, int64_t npix, uint8_t *out)
{
    for (int64_t p = 0; p < npix; ++p) {
        int64_t y = (4899 * (int64_t)in[3 * p] + 9617 * (int64_t)in[3 * p + 1] + 1868 * (int64_t)in[3 * p + 2] +
                     8192) >> 14;
        out[3 * p] = out[3 * p + 1] = out[3 * p + 2] = (uint8_t)y;
    }
}

/* lut[c*256 + v] = (float)((v/255 - mean_c) / std_c) in IEEE double. */
void or_normalize_lut(const float *mean, const float *stdv, int C, float *lut)
{
    for (int c = 0; c < C; ++c)
        for (int v = 0; v < 256; ++v)
            lut[c * 256 + v] = (float)((((double)v / 255.0) - (double)mean[c]) / (double)stdv[c]);
}

/* HWC u8 -> CHW f32 through the per-channel normalisation LUT. */
void or_normalize_chw(const uint8_t *in, int H, int W, int C, const float *lut, float *out)
{
    for (int c = 0; c < C; ++c)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x)
                out[((int64_t)c * H + y) * W + x] = lut[c * 256 + in[((int64_t)y * W + x) * C + c]];
}

/* ------------------------------------------------------------------------ */
/* Resampling core shared by every geometric op of this file: given a        */
/* fixed-point source position (qx, qy) in Q10 pixel-centre coordinates,     */
/* bilinear = rshr_he(sum w_y*w_x*p, 20) with per-axis weights (1024-a, a);  */
/* nearest = the pixel (q + 512) >> 10.  Border: 0 reflect-101, 1 constant   */
/* zero (decided per tap), 2 replicate.                                      */
/* ------------------------------------------------------------------------ */

enum { OR_REFLECT101 = 0, OR_CONSTANT = 1, OR_REPLICATE = 2 };
enum { OR_BILINEAR = 0, OR_NEAREST = 1 };

static int tap(const uint8_t *in, int H, int W, int C, int64_t y, int64_t x, int c, int border)
{
    if (border == OR_CONSTANT) {
        if (y < 0 || y >= H || x < 0 || x >= W) return 0;
    } else if (border == OR_REFLECT101) {
        y = or_reflect101(y, H); x = or_reflect101(x, W);
    } else {
        y = clampi(y, H); x = clampi(x, W);
    }
    return in[((int64_t)y * W + x) * C + c];
}

static int sample_q(const uint8_t *in, int H, int W, int C, int64_t qx, int64_t qy, int c,
                    int interp, int border)
{
    if (interp == OR_NEAREST) {
        int64_t ix = floor_shift(qx + F_ONE / 2, F_BITS);
        int64_t iy = floor_shift(qy + F_ONE / 2, F_BITS);
        return tap(in, H, W, C, iy, ix, c, border);
    }
    int64_t x0 = floor_shift(qx, F_BITS), ax = frac_bits(qx, F_BITS);
    int64_t y0 = floor_shift(qy, F_BITS), ay = frac_bits(qy, F_BITS);
    int64_t wx[2] = {F_ONE - ax, ax}, wy[2] = {F_ONE - ay, ay};
    int64_t acc = 0;
    for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 2; ++i)
            acc += wy[j] * wx[i] * tap(in, H, W, C, y0 + j, x0 + i, c, border);
    return sat8(or_rshr_he(acc, 2 * F_BITS));
}

/* ------------------------------------------------------------------------ */
/* Resize with half-pixel centres (Sec. II-A random sized crop; Sec. II-B    */
/* scaling).  Position of output j: q_j = rdiv_he(((2j+1)Ws - Wd) 2^F, 2Wd). */
/* ------------------------------------------------------------------------ */

int64_t or_resize_q(int j, int Ws, int Wd)
{
    return or_rdiv_he(((int64_t)(2 * j + 1) * Ws - Wd) * F_ONE, 2 * (int64_t)Wd);
}

void or_resize_u8(const uint8_t *in, int Hs, int Ws, int C, uint8_t *out, int Hd, int Wd, int interp)
{
    for (int y = 0; y < Hd; ++y)
        for (int x = 0; x < Wd; ++x)
            for (int c = 0; c < C; ++c)
                out[((int64_t)y * Wd + x) * C + c] = (uint8_t)sample_q(
                    in, Hs, Ws, C, or_resize_q(x, Ws, Wd), or_resize_q(y, Hs, Hd), c, interp, OR_REPLICATE);
}

/* ------------------------------------------------------------------------ */
/* ShiftScaleRotate / Rotate (Table I rows Rotate, ShiftScaleRotate).        */
/* Forward map p' = s R(theta) (p - c) + c + (dx W, dy H), c the image       */
/* centre; the inverse is evaluated in double and quantised to Q32.          */
/* ------------------------------------------------------------------------ */

void or_ssr_inverse(float angle_deg, float scale, float dx, float dy, int H, int W, double *a)
{
    double t = (double)angle_deg * (3.14159265358979323846 / 180.0);
    double cs = cos(t), sn = sin(t), s = (double)scale;
    double cx = (W - 1) * 0.5, cy = (H - 1) * 0.5;
    double tx = (double)dx * W, ty = (double)dy * H;
    a[0] = cs / s;  a[1] = -sn / s;
    a[3] = sn / s;  a[4] = cs / s;
    a[2] = cx - a[0] * (cx + tx) - a[1] * (cy + ty);
    a[5] = cy - a[3] * (cx + tx) - a[4] * (cy + ty);
}

void or_ssr_matrix_q32(float angle_deg, float scale, float dx, float dy, int H, int W, int64_t *aq)
{
    double a[6];
    or_ssr_inverse(angle_deg, scale, dx, dy, H, W, a);
    for (int i = 0; i < 6; ++i) aq[i] = (int64_t)llrint(a[i] * 4294967296.0);
}

/* Boxes under shift-scale-rotate, then a crop (offset crop_x, crop_y, size
 * crop x crop) and a resize to outsz x outsz.  The SSR forward map, from the
 * definition above: a source pixel index p goes to s R(-t) (p - c) + c + T
 * (c the image centre, T = (dx W, dy H)).  A box corner u in continuous
 * coordinates (pixel i spans [i, i + 1)) is the index position u - 1/2, so
 * it maps to F(u - 1/2) + 1/2.  The box becomes the bounding box of its four
 * mapped corners, clipped to the image [0, W] x [0, H] (the warp keeps the
 * image size); the crop shifts and clips it to [0, crop]^2; the resize scales
 * it by outsz / crop.  All in double, stored as float. */
void or_boxes_ssr_crop_resize(const float *boxes, int nb, int H, int W, float angle_deg, float scale, float dx,
                              float dy, int crop_x, int crop_y, int crop, int outsz, float *out)
{
    double t = (double)angle_deg * (3.14159265358979323846 / 180.0);
    double cs = cos(t), sn = sin(t), s = (double)scale;
    double cx = (W - 1) * 0.5, cy = (H - 1) * 0.5;
    double tx = (double)dx * W, ty = (double)dy * H;
    for (int i = 0; i < nb; ++i) {
        double ux[4] = {boxes[4 * i + 0], boxes[4 * i + 2], boxes[4 * i + 0], boxes[4 * i + 2]};
        double uy[4] = {boxes[4 * i + 1], boxes[4 * i + 1], boxes[4 * i + 3], boxes[4 * i + 3]};
        double x1 = 1e300, y1 = 1e300, x2 = -1e300, y2 = -1e300;
        for (int k = 0; k < 4; ++k) {
            double px = ux[k] - 0.5 - cx, py = uy[k] - 0.5 - cy;
            double ox = s * (cs * px + sn * py) + cx + tx + 0.5;
            double oy = s * (-sn * px + cs * py) + cy + ty + 0.5;
            x1 = ox < x1 ? ox : x1; x2 = ox > x2 ? ox : x2;
            y1 = oy < y1 ? oy : y1; y2 = oy > y2 ? oy : y2;
        }
        x1 = clampd(x1, 0.0, W); x2 = clampd(x2, 0.0, W);
        y1 = clampd(y1, 0.0, H); y2 = clampd(y2, 0.0, H);
        x1 = clampd(x1 - crop_x, 0.0, crop); x2 = clampd(x2 - crop_x, 0.0, crop);
        y1 = clampd(y1 - crop_y, 0.0, crop); y2 = clampd(y2 - crop_y, 0.0, crop);
        double k = (double)outsz / crop;
        out[4 * i + 0] = (float)(x1 * k);
        out[4 * i + 1] = (float)(y1 * k);
        out[4 * i + 2] = (float)(x2 * k);
        out[4 * i + 3] = (float)(y2 * k);
    }
}

/* Affine warp with a Q32 inverse matrix: sx_q = a0 x + a1 y + a2 (exact),
 * then rshr_he(., 32 - F).  Output has the input's shape. */
void or_warp_affine_u8(const uint8_t *in, int H, int W, int C, const int64_t *aq, int interp,
                       int border, uint8_t *out)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int64_t qx = or_rshr_he(aq[0] * x + aq[1] * y + aq[2], 32 - F_BITS);
            int64_t qy = or_rshr_he(aq[3] * x + aq[4] * y + aq[5], 32 - F_BITS);
            for (int c = 0; c < C; ++c)
                out[((int64_t)y * W + x) * C + c] = (uint8_t)sample_q(in, H, W, C, qx, qy, c, interp, border);
        }
}

/* PadToSize (Table I PadToSize512): an image smaller than Hmin x Wmin along
 * an axis is padded to that size, the padding split as floor(d / 2) before
 * and the rest after; border OR_REFLECT101 (reflect-101 of the source index)
 * or OR_CONSTANT (value).  Larger axes are left as they are.  *Ho x *Wo is
 * the output size. */
void or_pad_u8(const uint8_t *in, int H, int W, int C, int Hmin, int Wmin, int border, int value, uint8_t *out,
               int *Ho, int *Wo)
{
    int ho = H > Hmin ? H : Hmin, wo = W > Wmin ? W : Wmin;
    int top = (ho - H) / 2, left = (wo - W) / 2;
    for (int y = 0; y < ho; ++y)
        for (int x = 0; x < wo; ++x)
            for (int c = 0; c < C; ++c) {
                int64_t sy = y - top, sx = x - left;
                int v;
                if (sy >= 0 && sy < H && sx >= 0 && sx < W) v = in[(sy * W + sx) * C + c];
                else if (border == OR_CONSTANT) v = value;
                else v = in[(or_reflect101(sy, H) * W + or_reflect101(sx, W)) * C + c];
                out[((int64_t)y * wo + x) * C + c] = (uint8_t)v;
            }
    *Ho = ho;
    *Wo = wo;
}

/* Crop (Table I RandomCrop64; Sec. II-B cropping): out = in[oy:oy+Hc, ox:ox+Wc]. */
void or_crop_u8(const uint8_t *in, int H, int W, int C, int ox, int oy, int Hc, int Wc, uint8_t *out)
{
    (void)H;
    for (int y = 0; y < Hc; ++y)
        for (int x = 0; x < Wc; ++x)
            for (int c = 0; c < C; ++c)
                out[((int64_t)y * Wc + x) * C + c] = in[((int64_t)(y + oy) * W + (x + ox)) * C + c];
}

/* ------------------------------------------------------------------------ */
/* ShiftHSV (Table I): integer hexcone HSV with hue in 2-degree units        */
/* (0..179), saturation and value on 0..255.                                 */
/* ------------------------------------------------------------------------ */

void or_rgb_to_hsv8(int R, int G, int B, int *H8, int *S8, int *V8)
{
    int V = R > G ? (R > B ? R : B) : (G > B ? G : B);
    int m = R < G ? (R < B ? R : B) : (G < B ? G : B);
    int Cc = V - m;
    *V8 = V;
    *S8 = V ? (int)or_rdiv_he(255 * (int64_t)Cc, V) : 0;
    int h;
    if (Cc == 0) h = 0;
    else if (V == R) h = (int)or_rdiv_he(30 * (int64_t)(G - B), Cc);
    else if (V == G) h = 60 + (int)or_rdiv_he(30 * (int64_t)(B - R), Cc);
    else h = 120 + (int)or_rdiv_he(30 * (int64_t)(R - G), Cc);
    *H8 = ((h % 180) + 180) % 180;
}

void or_hsv8_to_rgb(int H8, int S8, int V8, int *R, int *G, int *B)
{
    int sector = H8 / 30, r = H8 % 30;
    int pv = (int)or_rdiv_he((int64_t)V8 * (7650 - S8 * 30), 7650);
    int qv = (int)or_rdiv_he((int64_t)V8 * (7650 - S8 * r), 7650);
    int tv = (int)or_rdiv_he((int64_t)V8 * (7650 - S8 * (30 - r)), 7650);
    int v = V8;
    switch (sector) {
    case 0: *R = v;  *G = tv; *B = pv; break;
    case 1: *R = qv; *G = v;  *B = pv; break;
    case 2: *R = pv; *G = v;  *B = tv; break;
    case 3: *R = pv; *G = qv; *B = v;  break;
    case 4: *R = tv; *G = pv; *B = v;  break;
    default: *R = v; *G = pv; *B = qv; break;
    }
}

void or_hsv_shift_u8(const uint8_t *in, int64_t npix, int dh, int ds, int dv, uint8_t *out)
{
    for (int64_t i = 0; i < npix; ++i) {
        int h, s, v, r, g, b;
        or_rgb_to_hsv8(in[3 * i], in[3 * i + 1], in[3 * i + 2], &h, &s, &v);
        h = (((h + dh) % 180) + 180) % 180;
        s = sat8(s + ds);
        v = sat8(v + dv);
        or_hsv8_to_rgb(h, s, v, &r, &g, &b);
        out[3 * i] = (uint8_t)r; out[3 * i + 1] = (uint8_t)g; out[3 * i + 2] = (uint8_t)b;
    }
}

/* ------------------------------------------------------------------------ */
/* Binomial blur: 3x3 = [1,2,1]x[1,2,1]/16, 5x5 = [1,4,6,4,1]x[..]/256,      */
/* one rdiv_he, reflect-101 border, per channel.                             */
/* ------------------------------------------------------------------------ */

void or_blur_u8(const uint8_t *in, int H, int W, int C, int ksize, uint8_t *out)
{
    static const int k3[3] = {1, 2, 1};
    static const int k5[5] = {1, 4, 6, 4, 1};
    const int *k = ksize == 5 ? k5 : k3;
    int r = ksize / 2, norm = ksize == 5 ? 256 : 16;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < C; ++c) {
                int64_t acc = 0;
                for (int j = -r; j <= r; ++j)
                    for (int i = -r; i <= r; ++i)
                        acc += (int64_t)k[j + r] * k[i + r] *
                               in[(or_reflect101(y + j, H) * W + or_reflect101(x + i, W)) * C + c];
                out[((int64_t)y * W + x) * C + c] = (uint8_t)sat8(or_rdiv_he(acc, norm));
            }
}

/* ------------------------------------------------------------------------ */
/* Elastic transform (Sec. II-C, Fig. 4; the Simard et al. 2003 reference of */
/* Sec. I): uniform noise fields smoothed by a Gaussian, scaled by alpha.    */
/* ------------------------------------------------------------------------ */

/* Q15 taps t_k = rint(2^15 g_k / sum g), g_k = exp(-k^2 / (2 sigma^2)), |k| <= radius. */
void or_gauss_taps_q15(double sigma, int radius, int32_t *taps)
{
    double sum = 0.0;
    for (int k = -radius; k <= radius; ++k) sum += exp(-(double)k * k / (2.0 * sigma * sigma));
    for (int k = -radius; k <= radius; ++k)
        taps[k + radius] = (int32_t)rint(32768.0 * exp(-(double)k * k / (2.0 * sigma * sigma)) / sum);
}

/* Horizontal pass of one field over rows [y0, y1): h = rshr_he(sum t n, 15). */
void or_elastic_hpass(uint64_t seed, uint64_t index, int field, int H, int W, const int32_t *taps,
                      int radius, int y0, int y1, int32_t *h)
{
    (void)H;
    int32_t *row = (int32_t *)malloc(sizeof(int32_t) * (size_t)W);
    for (int y = y0; y < y1; ++y) {
        for (int x = 0; x < W; ++x) row[x] = or_noise16(seed, index, field, (int64_t)y * W + x);
        for (int x = 0; x < W; ++x) {
            int64_t acc = 0;
            for (int k = -radius; k <= radius; ++k) acc += (int64_t)taps[k + radius] * row[or_reflect101(x + k, W)];
            h[(int64_t)(y - y0) * W + x] = (int32_t)or_rshr_he(acc, 15);
        }
    }
    free(row);
}

/* Full-image displacement fields in Q10 pixels: off = rshr_he(alpha v, 20),
 * v the vertical pass (Q15) of the horizontal pass. */
void or_elastic_field(uint64_t seed, uint64_t index, int H, int W, double sigma, int alpha, int radius,
                      int32_t *offx, int32_t *offy)
{
    int32_t *taps = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * radius + 1));
    or_gauss_taps_q15(sigma, radius, taps);
    int32_t *h = (int32_t *)malloc(sizeof(int32_t) * (size_t)H * W);
    for (int field = 0; field < 2; ++field) {
        int32_t *off = field == 0 ? offx : offy;
        or_elastic_hpass(seed, index, field, H, W, taps, radius, 0, H, h);
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                int64_t v = 0;
                for (int k = -radius; k <= radius; ++k)
                    v += (int64_t)taps[k + radius] * h[or_reflect101(y + k, H) * W + x];
                off[(int64_t)y * W + x] = (int32_t)or_rshr_he((int64_t)alpha * v, 30 - F_BITS);
            }
    }
    free(h); free(taps);
}

/* Approximate elastic field (opt-in): the Gaussian of each axis is replaced by
 * a cascade of three box filters (Wells, IEEE PAMI 1986), with the widths of
 * Kovesi ("Fast almost-Gaussian filtering", DICTA 2010): w_ideal =
 * sqrt(12 sigma^2 / n + 1) for n = 3 passes, wl = the largest odd integer not
 * above w_ideal, wu = wl + 2, m = round((12 sigma^2 - n wl^2 - 4 n wl - 3 n) /
 * (-4 wl - 4)) (half away from zero); the first m passes use wl, the rest wu.
 * widths[] receives the three widths. */
void or_box_widths(double sigma, int *widths)
{
    const int n = 3;
    double w_ideal = sqrt(12.0 * sigma * sigma / n + 1.0);
    int wl = (int)floor(w_ideal);
    if (wl % 2 == 0) wl -= 1;
    int wu = wl + 2;
    double m_ideal = (12.0 * sigma * sigma - n * wl * wl - 4.0 * n * wl - 3.0 * n) / (-4.0 * wl - 4.0);
    int m = (int)round(m_ideal);
    for (int i = 0; i < n; ++i) widths[i] = i < m ? wl : wu;
}

/* One box pass along a line of n values: out[i] = rdiv_he(sum over |k| <= r of
 * in[reflect101(i + k)], 2r + 1). */
void or_box_pass(const int32_t *in, int n, int r, int32_t *out)
{
    for (int i = 0; i < n; ++i) {
        int64_t s = 0;
        for (int k = -r; k <= r; ++k) s += in[or_reflect101(i + k, n)];
        out[i] = (int32_t)or_rdiv_he(s, 2 * r + 1);
    }
}

/* Per field: noise (as in the exact field) -> three box passes along each row
 * -> three box passes along each column -> v (noise units) -> offset
 * rshr_he(alpha v, 5), the Q10 scale of the exact field (whose v carries 15
 * more fraction bits). */
void or_elastic_field_box(uint64_t seed, uint64_t index, int H, int W, double sigma, int alpha,
                          int32_t *offx, int32_t *offy)
{
    int widths[3];
    or_box_widths(sigma, widths);
    int L = H > W ? H : W;
    int32_t *a = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
    int32_t *b = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
    int32_t *f = (int32_t *)malloc(sizeof(int32_t) * (size_t)H * W);
    for (int field = 0; field < 2; ++field) {
        int32_t *off = field == 0 ? offx : offy;
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) a[x] = or_noise16(seed, index, field, (int64_t)y * W + x);
            for (int p = 0; p < 3; ++p) {
                or_box_pass(a, W, widths[p] / 2, b);
                memcpy(a, b, sizeof(int32_t) * (size_t)W);
            }
            memcpy(f + (size_t)y * W, a, sizeof(int32_t) * (size_t)W);
        }
        for (int x = 0; x < W; ++x) {
            for (int y = 0; y < H; ++y) a[y] = f[(size_t)y * W + x];
            for (int p = 0; p < 3; ++p) {
                or_box_pass(a, H, widths[p] / 2, b);
                memcpy(a, b, sizeof(int32_t) * (size_t)H);
            }
            for (int y = 0; y < H; ++y) off[(size_t)y * W + x] = (int32_t)or_rshr_he((int64_t)alpha * a[y], 5);
        }
    }
    free(a); free(b); free(f);
}

/* The same field value at one pixel, computed from the definition alone
 * (used to check sampled pixels of full-size images). */
void or_elastic_field_at(uint64_t seed, uint64_t index, int H, int W, double sigma, int alpha,
                         int radius, int y, int x, int32_t *offx, int32_t *offy)
{
    int32_t *taps = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * radius + 1));
    or_gauss_taps_q15(sigma, radius, taps);
    for (int field = 0; field < 2; ++field) {
        int64_t v = 0;
        for (int k = -radius; k <= radius; ++k) {
            int64_t yy = or_reflect101(y + k, H);
            int64_t acc = 0;
            for (int j = -radius; j <= radius; ++j)
                acc += (int64_t)taps[j + radius] * or_noise16(seed, index, field, yy * W + or_reflect101(x + j, W));
            v += (int64_t)taps[k + radius] * or_rshr_he(acc, 15);
        }
        int32_t o = (int32_t)or_rshr_he((int64_t)alpha * v, 30 - F_BITS);
        if (field == 0) *offx = o; else *offy = o;
    }
    free(taps);
}

/* Remap by a displacement field: source of (y, x) is ((x<<F)+offx, (y<<F)+offy). */
void or_remap_field_u8(const uint8_t *in, int H, int W, int C, const int32_t *offx, const int32_t *offy,
                       int interp, uint8_t *out)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            int64_t qx = ((int64_t)x << F_BITS) + offx[(int64_t)y * W + x];
            int64_t qy = ((int64_t)y << F_BITS) + offy[(int64_t)y * W + x];
            for (int c = 0; c < C; ++c)
                out[((int64_t)y * W + x) * C + c] = (uint8_t)sample_q(in, H, W, C, qx, qy, c, interp, OR_REFLECT101);
        }
}

/* ------------------------------------------------------------------------ */
/* Grid distortion (Sec. II-C, Fig. 4): 5 cells per axis, cell k stretched   */
/* by d_k; knots S_0 = 0, S_{k+1} = S_k + cw d_k (not renormalised).          */
/* ------------------------------------------------------------------------ */

void or_grid_table(const double *d, int ncell, int n, int32_t *q)
{
    double cw = (double)n / ncell;
    double *S = (double *)malloc(sizeof(double) * (size_t)(ncell + 1));
    S[0] = 0.0;
    for (int k = 0; k < ncell; ++k) S[k + 1] = S[k] + cw * d[k];
    for (int x = 0; x < n; ++x) {
        double u = x + 0.5;
        int k = (int)floor(u / cw);
        if (k > ncell - 1) k = ncell - 1;
        double src = S[k] + (u - k * cw) * d[k] - 0.5;
        q[x] = (int32_t)llrint(src * F_ONE);
    }
    free(S);
}

void or_grid_remap_u8(const uint8_t *in, int H, int W, int C, const int32_t *mapx, const int32_t *mapy,
                      int interp, uint8_t *out)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int c = 0; c < C; ++c)
                out[((int64_t)y * W + x) * C + c] =
                    (uint8_t)sample_q(in, H, W, C, mapx[x], mapy[y], c, interp, OR_REFLECT101);
}

/* ------------------------------------------------------------------------ */
/* Image statistics: per channel sum, min, max and 256-bin histogram.        */
/* ------------------------------------------------------------------------ */

void or_image_stats_u8(const uint8_t *in, int64_t npix, int C, uint64_t *sum, int32_t *mn, int32_t *mx,
                       uint32_t *hist)
{
    for (int c = 0; c < C; ++c) {
        sum[c] = 0; mn[c] = 255; mx[c] = 0;
        for (int v = 0; v < 256; ++v) hist[c * 256 + v] = 0;
    }
    for (int64_t i = 0; i < npix; ++i)
        for (int c = 0; c < C; ++c) {
            int v = in[i * C + c];
            sum[c] += (uint64_t)v;
            if (v < mn[c]) mn[c] = v;
            if (v > mx[c]) mx[c] = v;
            hist[c * 256 + v] += 1;
        }
}

/* ------------------------------------------------------------------------ */
/* Composed pipelines (Sec. II: combinations of transforms; every value-     */
/* producing op rounds to u8 before the next op runs).                       */
/* ------------------------------------------------------------------------ */

/* Small plain pipeline: Dih4 element then brightness/contrast, n images of
 * H x W x C (HWC, dense).  Output image i has shape d4(H, W). */
void or_pipe_d4bc(const uint8_t *imgs, int n, int H, int W, int C, const int32_t *flags, const float *ab,
                  uint8_t *out)
{
    size_t sz = (size_t)H * W * C;
    uint8_t *t = (uint8_t *)malloc(sz);
    uint8_t lut[256];
    for (int i = 0; i < n; ++i) {
        int ho, wo;
        or_d4(imgs + i * sz, H, W, C, flags[4 * i], flags[4 * i + 1], flags[4 * i + 2], flags[4 * i + 3], t, &ho, &wo);
        or_bc_lut(ab[2 * i], ab[2 * i + 1], lut);
        or_apply_lut(t, (int64_t)sz, lut, out + i * sz);
    }
    free(t);
}

/* Full u8 pipeline for one RGB image: shift-scale-rotate (bilinear,
 * reflect-101) -> crop (crop x crop) -> resize to out x out (bilinear) ->
 * hue/saturation shift -> gamma LUT -> 3x3 blur when the blur flag is set.
 * f = {angle_deg, scale, dx, dy, gamma}, k = {crop_x, crop_y, dh, ds, blur}. */
void or_pipe_c2_one(const uint8_t *img, int H, int W, const float *f, const int32_t *k, int crop, int outsz,
                    uint8_t *out)
{
    int64_t aq[6];
    uint8_t lut[256];
    uint8_t *warp = (uint8_t *)malloc((size_t)H * W * 3);
    uint8_t *cr = (uint8_t *)malloc((size_t)crop * crop * 3);
    uint8_t *rs = (uint8_t *)malloc((size_t)outsz * outsz * 3);
    uint8_t *hs = (uint8_t *)malloc((size_t)outsz * outsz * 3);
    or_ssr_matrix_q32(f[0], f[1], f[2], f[3], H, W, aq);
    or_warp_affine_u8(img, H, W, 3, aq, OR_BILINEAR, OR_REFLECT101, warp);
    or_crop_u8(warp, H, W, 3, k[0], k[1], crop, crop, cr);
    or_resize_u8(cr, crop, crop, 3, rs, outsz, outsz, OR_BILINEAR);
    or_hsv_shift_u8(rs, (int64_t)outsz * outsz, k[2], k[3], 0, hs);
    or_gamma_lut(f[4], lut);
    if (k[4]) {
        or_apply_lut(hs, (int64_t)outsz * outsz * 3, lut, rs);
        or_blur_u8(rs, outsz, outsz, 3, 3, out);
    } else {
        or_apply_lut(hs, (int64_t)outsz * outsz * 3, lut, out);
    }
    free(warp); free(cr); free(rs); free(hs);
}

/* Ragged-batch pipeline for one image (Sec. II-A: image, masks and boxes
 * transformed together): Dih4 -> [crop window] -> brightness/contrast ->
 * resize (Hd x Wd, bilinear) -> normalise to CHW f32; the mask takes Dih4 ->
 * [crop] -> nearest resize; boxes take Dih4 -> [crop: shift, clip] -> scale.
 * win (NULL: none) = {y0, x0, h, w} inside the Dih4 image; mask/boxes may be
 * NULL. */
void or_pipe_ragged_one(const uint8_t *img, const uint8_t *mask, int H, int W, const int32_t *flags,
                        const float *ab, const int32_t *win, const float *boxes, int nb, const float *mean,
                        const float *stdv, int Hd, int Wd, float *out, uint8_t *out_mask, float *out_boxes)
{
    int ho, wo;
    uint8_t lut[256];
    float nlut[3 * 256];
    uint8_t *d = (uint8_t *)malloc((size_t)H * W * 3);
    uint8_t *c = (uint8_t *)malloc((size_t)H * W * 3);
    uint8_t *l = (uint8_t *)malloc((size_t)H * W * 3);
    uint8_t *r = (uint8_t *)malloc((size_t)Hd * Wd * 3);
    or_d4(img, H, W, 3, flags[0], flags[1], flags[2], flags[3], d, &ho, &wo);
    int hc = ho, wc = wo;
    if (win) {  /* crop window {y0, x0, h, w} of the Dih4 image */
        or_crop_u8(d, ho, wo, 3, win[1], win[0], win[2], win[3], c);
        hc = win[2];
        wc = win[3];
    } else {
        memcpy(c, d, (size_t)H * W * 3);
    }
    or_bc_lut(ab[0], ab[1], lut);
    or_apply_lut(c, (int64_t)hc * wc * 3, lut, l);
    or_resize_u8(l, hc, wc, 3, r, Hd, Wd, OR_BILINEAR);
    or_normalize_lut(mean, stdv, 3, nlut);
    or_normalize_chw(r, Hd, Wd, 3, nlut, out);
    if (mask && out_mask) {
        uint8_t *md = (uint8_t *)malloc((size_t)H * W);
        uint8_t *mc = (uint8_t *)malloc((size_t)H * W);
        or_d4(mask, H, W, 1, flags[0], flags[1], flags[2], flags[3], md, &ho, &wo);
        if (win) or_crop_u8(md, ho, wo, 1, win[1], win[0], win[2], win[3], mc);
        else memcpy(mc, md, (size_t)H * W);
        or_resize_u8(mc, hc, wc, 1, out_mask, Hd, Wd, OR_NEAREST);
        free(md); free(mc);
    }
    if (boxes && out_boxes && nb > 0)
        or_boxes_d4_crop_resize(boxes, nb, H, W, flags[0], flags[1], flags[2], flags[3], win, Hd, Wd, out_boxes);
    free(d); free(c); free(l); free(r);
}

/* Large-tile pipeline for one image: elastic (bilinear image, nearest mask,
 * reflect-101) then grid distortion on the u8 result.  grid = {x d_0..d_4,
 * y d_0..d_4}.  mask may be NULL. */
void or_pipe_elastic_grid_one(const uint8_t *img, const uint8_t *mask, int H, int W, int C, uint64_t seed,
                              uint64_t index, double sigma, int alpha, int radius, const double *grid,
                              uint8_t *out, uint8_t *out_mask)
{
    int32_t *offx = (int32_t *)malloc(sizeof(int32_t) * (size_t)H * W);
    int32_t *offy = (int32_t *)malloc(sizeof(int32_t) * (size_t)H * W);
    int32_t *mx = (int32_t *)malloc(sizeof(int32_t) * (size_t)W);
    int32_t *my = (int32_t *)malloc(sizeof(int32_t) * (size_t)H);
    uint8_t *e = (uint8_t *)malloc((size_t)H * W * C);
    or_elastic_field(seed, index, H, W, sigma, alpha, radius, offx, offy);
    or_grid_table(grid, 5, W, mx);
    or_grid_table(grid + 5, 5, H, my);
    or_remap_field_u8(img, H, W, C, offx, offy, OR_BILINEAR, e);
    or_grid_remap_u8(e, H, W, C, mx, my, OR_BILINEAR, out);
    if (mask && out_mask) {
        or_remap_field_u8(mask, H, W, 1, offx, offy, OR_NEAREST, e);
        or_grid_remap_u8(e, H, W, 1, mx, my, OR_NEAREST, out_mask);
    }
    free(offx); free(offy); free(mx); free(my); free(e);
}

/* ------------------------------------------------------------------------ */
/* Differentiable fp64 warp + colour (one CHW image).  Continuous affine     */
/* map with the shift-scale-rotate parameterisation above (tx, ty are        */
/* fractions of W, H), bilinear with zero border decided per tap, then       */
/* z = alpha w + beta, y1 = clamp(z, 0, 1), y = y1^gamma (0^gamma = 0).      */
/* p = {angle_deg, scale, tx, ty, alpha, beta, gamma}.                       */
/* ------------------------------------------------------------------------ */

static double ztap(const float *x, int H, int W, int64_t yy, int64_t xx)
{
    if (yy < 0 || yy >= H || xx < 0 || xx >= W) return 0.0;
    return (double)x[yy * W + xx];
}

static void wc_coords(const double *p, int H, int W, int x, int y, double *sx, double *sy, double dsx[4],
                      double dsy[4])
{
    double d2r = 3.14159265358979323846 / 180.0;
    double t = p[0] * d2r, s = p[1];
    double cs = cos(t), sn = sin(t);
    double cx = (W - 1) * 0.5, cy = (H - 1) * 0.5;
    double X = x - cx - p[2] * W, Y = y - cy - p[3] * H;
    *sx = (cs * X - sn * Y) / s + cx;
    *sy = (sn * X + cs * Y) / s + cy;
    /* d/d angle_deg, d/d scale, d/d tx, d/d ty */
    dsx[0] = (-sn * X - cs * Y) / s * d2r;
    dsy[0] = (cs * X - sn * Y) / s * d2r;
    dsx[1] = -(cs * X - sn * Y) / (s * s);
    dsy[1] = -(sn * X + cs * Y) / (s * s);
    dsx[2] = -cs * W / s;
    dsy[2] = -sn * W / s;
    dsx[3] = sn * H / s;
    dsy[3] = -cs * H / s;
}

void or_wc_forward(const float *x, int C, int H, int W, const double *p, double *y)
{
    for (int c = 0; c < C; ++c)
        for (int oy = 0; oy < H; ++oy)
            for (int ox = 0; ox < W; ++ox) {
                double sx, sy, dsx[4], dsy[4];
                wc_coords(p, H, W, ox, oy, &sx, &sy, dsx, dsy);
                const float *xc = x + (int64_t)c * H * W;
                double fx0 = floor(sx), fy0 = floor(sy);
                int64_t x0 = (int64_t)fx0, y0 = (int64_t)fy0;
                double fx = sx - fx0, fy = sy - fy0;
                double w = (1 - fy) * ((1 - fx) * ztap(xc, H, W, y0, x0) + fx * ztap(xc, H, W, y0, x0 + 1)) +
                           fy * ((1 - fx) * ztap(xc, H, W, y0 + 1, x0) + fx * ztap(xc, H, W, y0 + 1, x0 + 1));
                double z = p[4] * w + p[5];
                double y1 = z < 0 ? 0 : (z > 1 ? 1 : z);
                y[((int64_t)c * H + oy) * W + ox] = y1 > 0 ? pow(y1, p[6]) : 0.0;
            }
}

/* Analytic adjoint of or_wc_forward: gx (may be NULL) receives dL/dx, gp the
 * seven parameter gradients, given gy = dL/dy. */
void or_wc_backward(const float *x, int C, int H, int W, const double *p, const double *gy, double *gx,
                    double *gp)
{
    for (int i = 0; i < 7; ++i) gp[i] = 0.0;
    if (gx) for (int64_t i = 0; i < (int64_t)C * H * W; ++i) gx[i] = 0.0;
    for (int c = 0; c < C; ++c)
        for (int oy = 0; oy < H; ++oy)
            for (int ox = 0; ox < W; ++ox) {
                double sx, sy, dsx[4], dsy[4];
                wc_coords(p, H, W, ox, oy, &sx, &sy, dsx, dsy);
                const float *xc = x + (int64_t)c * H * W;
                double fx0 = floor(sx), fy0 = floor(sy);
                int64_t x0 = (int64_t)fx0, y0 = (int64_t)fy0;
                double fx = sx - fx0, fy = sy - fy0;
                double p00 = ztap(xc, H, W, y0, x0), p01 = ztap(xc, H, W, y0, x0 + 1);
                double p10 = ztap(xc, H, W, y0 + 1, x0), p11 = ztap(xc, H, W, y0 + 1, x0 + 1);
                double w = (1 - fy) * ((1 - fx) * p00 + fx * p01) + fy * ((1 - fx) * p10 + fx * p11);
                double z = p[4] * w + p[5];
                double y1 = z < 0 ? 0 : (z > 1 ? 1 : z);
                double g = gy[((int64_t)c * H + oy) * W + ox];
                if (y1 <= 0.0) continue;                     /* y = 0 and all derivatives are 0 */
                double yv = pow(y1, p[6]);
                gp[6] += g * yv * log(y1);
                if (!(z > 0.0 && z < 1.0)) continue;         /* clamp derivative is 0 */
                double gz = g * p[6] * pow(y1, p[6] - 1.0);
                gp[4] += gz * w;
                gp[5] += gz;
                double gw = gz * p[4];
                double dwdx = (1 - fy) * (p01 - p00) + fy * (p11 - p10);
                double dwdy = (1 - fx) * (p10 - p00) + fx * (p11 - p01);
                for (int k = 0; k < 4; ++k) gp[k] += gw * (dwdx * dsx[k] + dwdy * dsy[k]);
                if (gx) {
                    double *gc = gx + (int64_t)c * H * W;
                    double wt[4] = {(1 - fy) * (1 - fx), (1 - fy) * fx, fy * (1 - fx), fy * fx};
                    int64_t ty[4] = {y0, y0, y0 + 1, y0 + 1}, tx[4] = {x0, x0 + 1, x0, x0 + 1};
                    for (int k = 0; k < 4; ++k)
                        if (ty[k] >= 0 && ty[k] < H && tx[k] >= 0 && tx[k] < W) gc[ty[k] * W + tx[k]] += gw * wt[k];
                }
            }
}

/* ------------------------------------------------------------------------ */
/* Float copy of the large-tile chain (no u8 rounding): elastic remap then   */
/* grid remap with the same Q10 coordinates and dyadic bilinear weights,     */
/* reflect-101 border.  One CHW image; fp64 result, and its adjoint.         */
/* ------------------------------------------------------------------------ */

static void dyadic_taps(int64_t qx, int64_t qy, int W, int H, int64_t tyx[4][2], double wt[4])
{
    int64_t x0 = floor_shift(qx, F_BITS), ax = frac_bits(qx, F_BITS);
    int64_t y0 = floor_shift(qy, F_BITS), ay = frac_bits(qy, F_BITS);
    double wx[2] = {(double)(F_ONE - ax) / F_ONE, (double)ax / F_ONE};
    double wy[2] = {(double)(F_ONE - ay) / F_ONE, (double)ay / F_ONE};
    for (int j = 0; j < 2; ++j)
        for (int i = 0; i < 2; ++i) {
            tyx[2 * j + i][0] = or_reflect101(y0 + j, H);
            tyx[2 * j + i][1] = or_reflect101(x0 + i, W);
            wt[2 * j + i] = wy[j] * wx[i];
        }
}

void or_chain_f_forward(const float *x, int C, int H, int W, const int32_t *offx, const int32_t *offy,
                        const int32_t *mapx, const int32_t *mapy, double *y)
{
    double *e = (double *)malloc(sizeof(double) * (size_t)H * W);
    for (int c = 0; c < C; ++c) {
        const float *xc = x + (int64_t)c * H * W;
        for (int yy = 0; yy < H; ++yy)
            for (int xx = 0; xx < W; ++xx) {
                int64_t t[4][2]; double wt[4];
                dyadic_taps(((int64_t)xx << F_BITS) + offx[(int64_t)yy * W + xx],
                            ((int64_t)yy << F_BITS) + offy[(int64_t)yy * W + xx], W, H, t, wt);
                double acc = 0;
                for (int k = 0; k < 4; ++k) acc += wt[k] * (double)xc[t[k][0] * W + t[k][1]];
                e[(int64_t)yy * W + xx] = acc;
            }
        for (int yy = 0; yy < H; ++yy)
            for (int xx = 0; xx < W; ++xx) {
                int64_t t[4][2]; double wt[4];
                dyadic_taps(mapx[xx], mapy[yy], W, H, t, wt);
                double acc = 0;
                for (int k = 0; k < 4; ++k) acc += wt[k] * e[t[k][0] * W + t[k][1]];
                y[((int64_t)c * H + yy) * W + xx] = acc;
            }
    }
    free(e);
}

void or_chain_f_backward(int C, int H, int W, const int32_t *offx, const int32_t *offy, const int32_t *mapx,
                         const int32_t *mapy, const double *gy, double *gx)
{
    double *ge = (double *)malloc(sizeof(double) * (size_t)H * W);
    for (int c = 0; c < C; ++c) {
        double *gc = gx + (int64_t)c * H * W;
        for (int64_t i = 0; i < (int64_t)H * W; ++i) { ge[i] = 0; gc[i] = 0; }
        for (int yy = 0; yy < H; ++yy)
            for (int xx = 0; xx < W; ++xx) {
                int64_t t[4][2]; double wt[4];
                dyadic_taps(mapx[xx], mapy[yy], W, H, t, wt);
                double g = gy[((int64_t)c * H + yy) * W + xx];
                for (int k = 0; k < 4; ++k) ge[t[k][0] * W + t[k][1]] += wt[k] * g;
            }
        for (int yy = 0; yy < H; ++yy)
            for (int xx = 0; xx < W; ++xx) {
                int64_t t[4][2]; double wt[4];
                dyadic_taps(((int64_t)xx << F_BITS) + offx[(int64_t)yy * W + xx],
                            ((int64_t)yy << F_BITS) + offy[(int64_t)yy * W + xx], W, H, t, wt);
                double g = ge[(int64_t)yy * W + xx];
                for (int k = 0; k < 4; ++k) gc[t[k][0] * W + t[k][1]] += wt[k] * g;
            }
    }
    free(ge);
}
