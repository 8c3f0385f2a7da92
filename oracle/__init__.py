"""CPU oracle for the batched image-augmentation hot path (arXiv:1809.06839).

TEST INFRASTRUCTURE ONLY: the test-suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  The product path
(``paper_1809_06839_amd``) never imports this package and shares no code with
it.

This module is a ctypes wrapper around ``oracle.c`` (plain C99, fp64 / exact
integer arithmetic, single-threaded, built with ``-O2 -ffp-contract=off``).
The paper fixes which operations exist (Abstract; Sec. I; Sec. II-A..C;
Table I) and that masks and boxes follow the image geometry (Sec. II-A,
Sec. II-B) but gives no formula, so each function implements a stated reading;
each wrapper names the passage that introduces its operation.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
against numpy / scipy / colorsys / exact rational arithmetic / closed forms,
except agreement with the paper's own library outputs, which the paper does
not contain (parity unpinned against the original library).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_SANITIZE=1 builds and loads an AddressSanitizer + UndefinedBehaviorSanitizer
# copy instead (the process must preload the sanitizer runtimes)
_SANITIZE = os.environ.get("ORACLE_SANITIZE", "") == "1"
_LIB_PATH = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")

BILINEAR, NEAREST = 0, 1
REFLECT101, CONSTANT, REPLICATE = 0, 1, 2
F_BITS = 10

IMAGENET_MEAN = np.array([0.485, 0.456, 0.406], dtype=np.float32)
IMAGENET_STD = np.array([0.229, 0.224, 0.225], dtype=np.float32)


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (no GPU involved)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        san = ["-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"] if _SANITIZE else []
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99",
                               "-Wall", "-Wextra"] + san + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None

_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i, _i64, _u64, _f, _d = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float, ctypes.c_double
_ip = ctypes.POINTER(ctypes.c_int)

_SIGS = {
    "or_rdiv_he": (_i64, [_i64, _i64]),
    "or_rshr_he": (_i64, [_i64, _i]),
    "or_reflect101": (_i64, [_i64, _i64]),
    "or_philox4x64_10": (None, [_u64p, _u64p, _u64p]),
    "or_draw_u64": (_u64, [_u64, _u64, _u64, _u64]),
    "or_sample_d4bc": (None, [_u64, _u64, _i, _i32p, _f32p]),
    "or_sample_c2": (None, [_u64, _u64, _i, _i, _f32p, _i32p]),
    "or_sample_wc": (None, [_u64, _u64, _i, _f32p]),
    "or_sample_grid": (None, [_u64, _u64, _i, _d, _f64p]),
    "or_noise16": (ctypes.c_int32, [_u64, _u64, _i, _i64]),
    "or_hflip": (None, [_u8p, _i, _i, _i, _u8p]),
    "or_vflip": (None, [_u8p, _i, _i, _i, _u8p]),
    "or_rot90": (None, [_u8p, _i, _i, _i, _u8p]),
    "or_transpose": (None, [_u8p, _i, _i, _i, _u8p]),
    "or_d4": (None, [_u8p, _i, _i, _i, _i, _i, _i, _i, _u8p, _ip, _ip]),
    "or_boxes_d4_resize": (None, [_f32p, _i, _i, _i, _i, _i, _i, _i, _i, _i, _f32p]),
    "or_bc_lut": (None, [_f, _f, _u8p]),
    "or_gamma_lut": (None, [_f, _u8p]),
    "or_apply_lut": (None, [_u8p, _i64, _u8p, _u8p]),
    "or_normalize_lut": (None, [_f32p, _f32p, _i, _f32p]),
    "or_normalize_chw": (None, [_u8p, _i, _i, _i, _f32p, _f32p]),
    "or_resize_q": (_i64, [_i, _i, _i]),
    "or_resize_u8": (None, [_u8p, _i, _i, _i, _u8p, _i, _i, _i]),
    "or_ssr_inverse": (None, [_f, _f, _f, _f, _i, _i, _f64p]),
    "or_ssr_matrix_q32": (None, [_f, _f, _f, _f, _i, _i, _i64p]),
    "or_warp_affine_u8": (None, [_u8p, _i, _i, _i, _i64p, _i, _i, _u8p]),
    "or_crop_u8": (None, [_u8p, _i, _i, _i, _i, _i, _i, _i, _u8p]),
    "or_pad_u8": (None, [_u8p, _i, _i, _i, _i, _i, _i, _i, _u8p, ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "or_shift_rgb_lut": (None, [_f32p, _i, _u8p]),
    "or_apply_lut_c": (None, [_u8p, ctypes.c_int64, _i, _u8p, _u8p]),
    "or_gray_u8": (None, [_u8p, ctypes.c_int64, _u8p]),
    "or_rgb_to_hsv8": (None, [_i, _i, _i, _ip, _ip, _ip]),
    "or_hsv8_to_rgb": (None, [_i, _i, _i, _ip, _ip, _ip]),
    "or_hsv_shift_u8": (None, [_u8p, _i64, _i, _i, _i, _u8p]),
    "or_blur_u8": (None, [_u8p, _i, _i, _i, _i, _u8p]),
    "or_gauss_taps_q15": (None, [_d, _i, _i32p]),
    "or_elastic_hpass": (None, [_u64, _u64, _i, _i, _i, _i32p, _i, _i, _i, _i32p]),
    "or_elastic_field": (None, [_u64, _u64, _i, _i, _d, _i, _i, _i32p, _i32p]),
    "or_box_widths": (None, [_d, _i32p]),
    "or_box_pass": (None, [_i32p, _i, _i, _i32p]),
    "or_elastic_field_box": (None, [_u64, _u64, _i, _i, _d, _i, _i32p, _i32p]),
    "or_elastic_field_at": (None, [_u64, _u64, _i, _i, _d, _i, _i, _i, _i, _ip, _ip]),
    "or_remap_field_u8": (None, [_u8p, _i, _i, _i, _i32p, _i32p, _i, _u8p]),
    "or_grid_table": (None, [_f64p, _i, _i, _i32p]),
    "or_grid_remap_u8": (None, [_u8p, _i, _i, _i, _i32p, _i32p, _i, _u8p]),
    "or_image_stats_u8": (None, [_u8p, _i64, _i, _u64p, _i32p, _i32p, _u32p]),
    "or_pipe_d4bc": (None, [_u8p, _i, _i, _i, _i, _i32p, _f32p, _u8p]),
    "or_pipe_c2_one": (None, [_u8p, _i, _i, _f32p, _i32p, _i, _i, _u8p]),
    "or_pipe_ragged_one": (None, [_u8p, ctypes.c_void_p, _i, _i, _i32p, _f32p, ctypes.c_void_p, ctypes.c_void_p,
                                  _i, _f32p, _f32p, _i, _i, _f32p, ctypes.c_void_p, ctypes.c_void_p]),
    "or_boxes_d4_crop_resize": (None, [_f32p, _i, _i, _i, _i, _i, _i, _i, ctypes.c_void_p, _i, _i, _f32p]),
    "or_boxes_ssr_crop_resize": (None, [_f32p, _i, _i, _i, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_float, _i, _i, _i, _i, _f32p]),
    "or_pipe_elastic_grid_one": (None, [_u8p, ctypes.c_void_p, _i, _i, _i, _u64, _u64, _d, _i, _i,
                                        _f64p, _u8p, ctypes.c_void_p]),
    "or_wc_forward": (None, [_f32p, _i, _i, _i, _f64p, _f64p]),
    "or_wc_backward": (None, [_f32p, _i, _i, _i, _f64p, _f64p, ctypes.c_void_p, _f64p]),
    "or_chain_f_forward": (None, [_f32p, _i, _i, _i, _i32p, _i32p, _i32p, _i32p, _f64p]),
    "or_chain_f_backward": (None, [_i, _i, _i, _i32p, _i32p, _i32p, _i32p, _f64p, _f64p]),
}


def lib():
    """Load (building first when needed) the oracle shared library."""
    global _lib
    if _lib is None:
        path = build()
        L = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------- primitives
def rdiv_he(n: int, d: int) -> int:
    return lib().or_rdiv_he(n, d)


def rshr_he(n: int, k: int) -> int:
    return lib().or_rshr_he(n, k)


def reflect101(i: int, n: int) -> int:
    return lib().or_reflect101(i, n)


def philox4x64_10(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint64)
    lib().or_philox4x64_10(_c(ctr, np.uint64), _c(key, np.uint64), out)
    return out


def draw_u64(seed, stream, index, draw) -> int:
    return lib().or_draw_u64(seed, stream, index, draw)


def noise16(seed, index, field, e) -> int:
    return lib().or_noise16(seed, index, field, e)


# ---------------------------------------------------------------- sampler
def sample_d4bc(seed: int, first: int, n: int):
    """Dih4 flags {hflip, vflip, k, transpose} and {alpha, beta} per sample."""
    flags = np.zeros((n, 4), np.int32)
    ab = np.zeros((n, 2), np.float32)
    lib().or_sample_d4bc(seed, first, n, flags, ab)
    return flags, ab


def sample_c2(seed: int, first: int, n: int, crop_range: int = 64):
    f = np.zeros((n, 5), np.float32)
    k = np.zeros((n, 5), np.int32)
    lib().or_sample_c2(seed, first, n, crop_range, f, k)
    return f, k


def sample_wc(seed: int, first: int, n: int):
    f = np.zeros((n, 7), np.float32)
    lib().or_sample_wc(seed, first, n, f)
    return f


def sample_grid(seed: int, first: int, n: int, limit: float = 0.3):
    f = np.zeros((n, 10), np.float64)
    lib().or_sample_grid(seed, first, n, limit, f)
    return f


def _unit(word) -> float:
    return (int(word) >> 11) * 2.0 ** -53


def _below(word, m: int) -> int:
    return ((int(word) >> 32) * m) >> 32


def sized_crop_window(seed, index, draw0, H, W, scale=(0.08, 1.0), ratio=(0.75, 4.0 / 3.0), attempts=10):
    """Window {y0, x0, h, w} of the random-sized crop (Sec. II and Fig. 2's detection
    pipeline name a random-sized crop; the sampler is the usual area / aspect-ratio
    scheme, written out here as this library reads it).

    Try t (0 <= t < attempts) reads the four words of Philox block
    {draw0 + t, index, 0, 0} under key {seed, 0}: word 0 gives the area fraction
    s = lo + (hi - lo) u0, word 1 the aspect ratio r = exp(log lo_r + (log hi_r - log lo_r) u1);
    with A = H W s, w = floor(sqrt(A r) + 1/2) and h = floor(sqrt(A / r) + 1/2).  The first
    try with 1 <= w <= W and 1 <= h <= H wins, at y0 = below(word 2, H - h + 1),
    x0 = below(word 3, W - w + 1).  When no try fits, the window is centred and keeps the
    image's aspect ratio clamped into [lo_r, hi_r] (the full image if it is inside)."""
    lo_s, hi_s = float(scale[0]), float(scale[1])
    lo_r, hi_r = float(ratio[0]), float(ratio[1])
    llo, lhi = math.log(lo_r), math.log(hi_r)
    for t in range(attempts):
        w4 = philox4x64_10([draw0 + t, index, 0, 0], [seed, 0])
        s = lo_s + (hi_s - lo_s) * _unit(w4[0])
        r = math.exp(llo + (lhi - llo) * _unit(w4[1]))
        area = float(H) * float(W) * s
        w = int(math.floor(math.sqrt(area * r) + 0.5))
        h = int(math.floor(math.sqrt(area / r) + 0.5))
        if 1 <= w <= W and 1 <= h <= H:
            return np.array([_below(w4[2], H - h + 1), _below(w4[3], W - w + 1), h, w], np.int32)
    in_r = float(W) / float(H)
    if in_r < lo_r:
        w, h = W, max(1, int(math.floor(W / lo_r + 0.5)))
    elif in_r > hi_r:
        h, w = H, max(1, int(math.floor(H * hi_r + 0.5)))
    else:
        h, w = H, W
    return np.array([(H - h) // 2, (W - w) // 2, h, w], np.int32)


# ---------------------------------------------------------------- geometry
def _hwc(img):
    img = _c(img, np.uint8)
    if img.ndim == 2:
        return img, img.shape[0], img.shape[1], 1
    return img, img.shape[0], img.shape[1], img.shape[2]


def _like(img, H, W, C):
    return np.zeros((H, W) if img.ndim == 2 else (H, W, C), np.uint8)


def hflip(img):
    img, H, W, C = _hwc(img); out = _like(img, H, W, C); lib().or_hflip(img, H, W, C, out); return out


def vflip(img):
    img, H, W, C = _hwc(img); out = _like(img, H, W, C); lib().or_vflip(img, H, W, C, out); return out


def rot90(img):
    img, H, W, C = _hwc(img); out = _like(img, W, H, C); lib().or_rot90(img, H, W, C, out); return out


def transpose(img):
    img, H, W, C = _hwc(img); out = _like(img, W, H, C); lib().or_transpose(img, H, W, C, out); return out


def d4(img, hflip_, vflip_, k, transpose_):
    """Sec. II-B: element of Dih4 built as hflip -> vflip -> rot90^k -> transpose."""
    img, H, W, C = _hwc(img)
    buf = np.zeros(H * W * C, np.uint8)
    ho, wo = ctypes.c_int(), ctypes.c_int()
    lib().or_d4(img, H, W, C, int(hflip_), int(vflip_), int(k), int(transpose_), buf,
                ctypes.byref(ho), ctypes.byref(wo))
    return buf.reshape((ho.value, wo.value) if img.ndim == 2 else (ho.value, wo.value, C))


def boxes_d4_resize(boxes, H, W, flags, Hd, Wd):
    boxes = _c(boxes, np.float32).reshape(-1, 4)
    out = np.zeros_like(boxes)
    if len(boxes):
        lib().or_boxes_d4_resize(boxes, len(boxes), H, W, int(flags[0]), int(flags[1]), int(flags[2]),
                                 int(flags[3]), Hd, Wd, out)
    return out


def boxes_d4_crop_resize(boxes, H, W, flags, win, Hd, Wd):
    boxes = _c(boxes, np.float32).reshape(-1, 4)
    out = np.zeros_like(boxes)
    win = None if win is None else _c(win, np.int32)
    if len(boxes):
        lib().or_boxes_d4_crop_resize(boxes, len(boxes), H, W, int(flags[0]), int(flags[1]), int(flags[2]),
                                      int(flags[3]), _ptr(win), Hd, Wd, out)
    return out


def boxes_ssr_crop_resize(boxes, H, W, f, crop_x, crop_y, crop_, outsz):
    """f = (angle_deg, scale, dx, dy) as float32 values."""
    boxes = _c(boxes, np.float32).reshape(-1, 4)
    out = np.zeros_like(boxes)
    if len(boxes):
        lib().or_boxes_ssr_crop_resize(boxes, len(boxes), H, W, float(f[0]), float(f[1]), float(f[2]), float(f[3]),
                                       int(crop_x), int(crop_y), int(crop_), int(outsz), out)
    return out


def resize_q(j, Ws, Wd):
    return lib().or_resize_q(j, Ws, Wd)


def resize(img, Hd, Wd, interp=BILINEAR):
    img, H, W, C = _hwc(img); out = _like(img, Hd, Wd, C)
    lib().or_resize_u8(img, H, W, C, out, Hd, Wd, interp)
    return out


def ssr_inverse(angle, scale, dx, dy, H, W):
    a = np.zeros(6, np.float64)
    lib().or_ssr_inverse(angle, scale, dx, dy, H, W, a)
    return a


def ssr_matrix_q32(angle, scale, dx, dy, H, W):
    a = np.zeros(6, np.int64)
    lib().or_ssr_matrix_q32(angle, scale, dx, dy, H, W, a)
    return a


def warp_affine(img, aq, interp=BILINEAR, border=REFLECT101):
    img, H, W, C = _hwc(img); out = _like(img, H, W, C)
    lib().or_warp_affine_u8(img, H, W, C, _c(aq, np.int64), interp, border, out)
    return out


def crop(img, ox, oy, Hc, Wc):
    img, H, W, C = _hwc(img); out = _like(img, Hc, Wc, C)
    lib().or_crop_u8(img, H, W, C, ox, oy, Hc, Wc, out)
    return out


def pad(img, Hmin, Wmin, border=REFLECT101, value=0):
    img, H, W, C = _hwc(img)
    ho, wo = max(H, Hmin), max(W, Wmin)
    out = _like(img, ho, wo, C)
    a, b = ctypes.c_int(), ctypes.c_int()
    lib().or_pad_u8(img, H, W, C, Hmin, Wmin, border, value, out, ctypes.byref(a), ctypes.byref(b))
    assert (a.value, b.value) == (ho, wo)
    return out


# ---------------------------------------------------------------- point ops
def shift_rgb_lut(shift):
    shift = _c(shift, np.float32)
    lut = np.zeros((len(shift), 256), np.uint8)
    lib().or_shift_rgb_lut(shift, len(shift), lut)
    return lut


def apply_lut_c(img, lut):
    """Per-channel LUT (lut [C, 256]) on an HWC image."""
    img, H, W, C = _hwc(img)
    out = _like(img, H, W, C)
    lib().or_apply_lut_c(img, H * W, C, _c(lut, np.uint8), out)
    return out


def gray(img):
    img, H, W, C = _hwc(img)
    assert C == 3
    out = _like(img, H, W, C)
    lib().or_gray_u8(img, H * W, out)
    return out


def bc_lut(alpha, beta):
    lut = np.zeros(256, np.uint8); lib().or_bc_lut(alpha, beta, lut); return lut


def gamma_lut(gamma):
    lut = np.zeros(256, np.uint8); lib().or_gamma_lut(gamma, lut); return lut


def apply_lut(img, lut):
    img = _c(img, np.uint8); out = np.zeros_like(img)
    lib().or_apply_lut(img.reshape(-1), img.size, _c(lut, np.uint8), out.reshape(-1))
    return out


def normalize_lut(mean=IMAGENET_MEAN, std=IMAGENET_STD):
    mean = _c(mean, np.float32); std = _c(std, np.float32)
    lut = np.zeros(len(mean) * 256, np.float32)
    lib().or_normalize_lut(mean, std, len(mean), lut)
    return lut.reshape(len(mean), 256)


def normalize_chw(img, mean=IMAGENET_MEAN, std=IMAGENET_STD):
    img, H, W, C = _hwc(img)
    lut = normalize_lut(mean, std)
    out = np.zeros((C, H, W), np.float32)
    lib().or_normalize_chw(img, H, W, C, _c(lut, np.float32).reshape(-1), out)
    return out


def rgb_to_hsv8(r, g, b):
    """Integer hexcone RGB -> (H8 in 2-degree units, S8, V8)."""
    h, s, v = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    lib().or_rgb_to_hsv8(r, g, b, ctypes.byref(h), ctypes.byref(s), ctypes.byref(v))
    return h.value, s.value, v.value


def hsv8_to_rgb(h, s, v):
    r, g, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    lib().or_hsv8_to_rgb(h, s, v, ctypes.byref(r), ctypes.byref(g), ctypes.byref(b))
    return r.value, g.value, b.value


def hsv_shift(img, dh, ds, dv=0):
    """Table I ShiftHSV: integer hexcone HSV shift of an RGB u8 image."""
    img = _c(img, np.uint8); out = np.zeros_like(img)
    lib().or_hsv_shift_u8(img.reshape(-1), img.size // 3, dh, ds, dv, out.reshape(-1))
    return out


def blur(img, ksize=3):
    img, H, W, C = _hwc(img); out = _like(img, H, W, C)
    lib().or_blur_u8(img, H, W, C, ksize, out)
    return out


# ---------------------------------------------------------------- elastic / grid
def gauss_taps_q15(sigma=50.0, radius=150):
    t = np.zeros(2 * radius + 1, np.int32); lib().or_gauss_taps_q15(sigma, radius, t); return t


def elastic_hpass(seed, index, field, H, W, sigma=50.0, radius=150, y0=0, y1=None):
    y1 = H if y1 is None else y1
    taps = gauss_taps_q15(sigma, radius)
    h = np.zeros((y1 - y0, W), np.int32)
    lib().or_elastic_hpass(seed, index, field, H, W, taps, radius, y0, y1, h)
    return h


def elastic_field(seed, index, H, W, sigma=50.0, alpha=1000, radius=150):
    ox = np.zeros((H, W), np.int32); oy = np.zeros((H, W), np.int32)
    lib().or_elastic_field(seed, index, H, W, sigma, alpha, radius, ox, oy)
    return ox, oy


def box_widths(sigma):
    w = np.zeros(3, np.int32)
    lib().or_box_widths(sigma, w)
    return tuple(int(v) for v in w)


def box_pass(line, r):
    line = _c(line, np.int32)
    out = np.zeros_like(line)
    lib().or_box_pass(line, len(line), r, out)
    return out


def elastic_field_box(seed, index, H, W, sigma=50.0, alpha=1000):
    """Box-cascade approximation of the elastic field: (offx, offy) int32 [H, W]."""
    ox = np.zeros((H, W), np.int32); oy = np.zeros((H, W), np.int32)
    lib().or_elastic_field_box(seed, index, H, W, sigma, alpha, ox, oy)
    return ox, oy


def elastic_field_at(seed, index, H, W, y, x, sigma=50.0, alpha=1000, radius=150):
    ox, oy = ctypes.c_int(), ctypes.c_int()
    lib().or_elastic_field_at(seed, index, H, W, sigma, alpha, radius, y, x, ctypes.byref(ox), ctypes.byref(oy))
    return ox.value, oy.value


def remap_field(img, offx, offy, interp=BILINEAR):
    img, H, W, C = _hwc(img); out = _like(img, H, W, C)
    lib().or_remap_field_u8(img, H, W, C, _c(offx, np.int32), _c(offy, np.int32), interp, out)
    return out


def grid_table(d, n, ncell=5):
    q = np.zeros(n, np.int32); lib().or_grid_table(_c(d, np.float64), ncell, n, q); return q


def grid_remap(img, mapx, mapy, interp=BILINEAR):
    img, H, W, C = _hwc(img); out = _like(img, H, W, C)
    lib().or_grid_remap_u8(img, H, W, C, _c(mapx, np.int32), _c(mapy, np.int32), interp, out)
    return out


def boxes_distort(boxes, H, W, offx, offy, mapx, mapy):
    """Boxes under elastic then grid distortion, as the masks see them: each box is
    rasterised (pixels whose centres lie in [x1, x2) x [y1, y2)), the 0/1 mask goes through
    the nearest elastic remap and the nearest grid remap of the oracle, and the result's
    bounding box [min x, min y, max x + 1, max y + 1] is the transformed box (empty: zeros)."""
    boxes = _c(boxes, np.float32).reshape(-1, 4)
    out = np.zeros_like(boxes)
    cx = np.arange(W, dtype=np.float32) + np.float32(0.5)
    cy = np.arange(H, dtype=np.float32) + np.float32(0.5)
    for i, (x1, y1, x2, y2) in enumerate(boxes):
        inx = (cx >= x1) & (cx < x2)
        iny = (cy >= y1) & (cy < y2)
        mask = (iny[:, None] & inx[None, :]).astype(np.uint8)
        e = remap_field(mask, offx, offy, NEAREST)
        g = grid_remap(e, mapx, mapy, NEAREST)
        ys, xs = np.nonzero(g)
        if len(xs):
            out[i] = (xs.min(), ys.min(), xs.max() + 1, ys.max() + 1)
    return out


def image_stats(img, C=3):
    img = _c(img, np.uint8)
    s = np.zeros(C, np.uint64); mn = np.zeros(C, np.int32); mx = np.zeros(C, np.int32)
    h = np.zeros(C * 256, np.uint32)
    lib().or_image_stats_u8(img.reshape(-1), img.size // C, C, s, mn, mx, h)
    return s, mn, mx, h.reshape(C, 256)


# ---------------------------------------------------------------- pipelines
def pipe_d4bc(imgs, flags, ab):
    """Sec. II-B Dih4 element + Table I Brightness, per image of a dense batch."""
    imgs = _c(imgs, np.uint8)
    n, H, W, C = imgs.shape
    out = np.zeros(n * H * W * C, np.uint8)
    lib().or_pipe_d4bc(imgs, n, H, W, C, _c(flags, np.int32), _c(ab, np.float32), out)
    if H == W:
        return out.reshape(n, H, W, C)
    return out  # caller reshapes per image (shape depends on the element)


def pipe_c2_one(img, f, k, crop_=448, outsz=224):
    img = _c(img, np.uint8); H, W = img.shape[:2]
    out = np.zeros((outsz, outsz, 3), np.uint8)
    lib().or_pipe_c2_one(img, H, W, _c(f, np.float32), _c(k, np.int32), crop_, outsz, out)
    return out


def pipe_ragged_one(img, mask, flags, ab, boxes=None, Hd=224, Wd=224, mean=IMAGENET_MEAN, std=IMAGENET_STD,
                    win=None):
    """win: None or {y0, x0, h, w}, a crop window of the Dih4 image."""
    img = _c(img, np.uint8); H, W = img.shape[:2]
    win = None if win is None else _c(win, np.int32)
    out = np.zeros((3, Hd, Wd), np.float32)
    om = np.zeros((Hd, Wd), np.uint8) if mask is not None else None
    mask = _c(mask, np.uint8) if mask is not None else None
    nb = 0 if boxes is None else len(boxes)
    boxes = _c(boxes, np.float32).reshape(-1, 4) if nb else None
    ob = np.zeros((nb, 4), np.float32) if nb else None
    lib().or_pipe_ragged_one(img, _ptr(mask), H, W, _c(flags, np.int32), _c(ab, np.float32), _ptr(win), _ptr(boxes), nb,
                             _c(mean, np.float32), _c(std, np.float32), Hd, Wd, out, _ptr(om), _ptr(ob))
    return out, om, (ob if nb else np.zeros((0, 4), np.float32))


def pipe_elastic_grid_one(img, mask, seed, index, grid, sigma=50.0, alpha=1000, radius=150):
    img, H, W, C = _hwc(img)
    out = _like(img, H, W, C)
    mask = _c(mask, np.uint8) if mask is not None else None
    om = np.zeros((H, W), np.uint8) if mask is not None else None
    lib().or_pipe_elastic_grid_one(img, _ptr(mask), H, W, C, seed, index, sigma, alpha, radius,
                                   _c(grid, np.float64), out, _ptr(om))
    return out, om


def wc_forward(x, p):
    """fp64 forward of the differentiable warp + colour op on one CHW image."""
    x = _c(x, np.float32); C, H, W = x.shape
    y = np.zeros((C, H, W), np.float64)
    lib().or_wc_forward(x, C, H, W, _c(p, np.float64), y)
    return y


def wc_backward(x, p, gy, want_gx=True):
    x = _c(x, np.float32); C, H, W = x.shape
    gx = np.zeros((C, H, W), np.float64) if want_gx else None
    gp = np.zeros(7, np.float64)
    lib().or_wc_backward(x, C, H, W, _c(p, np.float64), _c(gy, np.float64), _ptr(gx), gp)
    return gx, gp


def chain_f_forward(x, offx, offy, mapx, mapy):
    x = _c(x, np.float32); C, H, W = x.shape
    y = np.zeros((C, H, W), np.float64)
    lib().or_chain_f_forward(x, C, H, W, _c(offx, np.int32), _c(offy, np.int32), _c(mapx, np.int32),
                             _c(mapy, np.int32), y)
    return y


def chain_f_backward(gy, offx, offy, mapx, mapy):
    gy = _c(gy, np.float64); C, H, W = gy.shape
    gx = np.zeros((C, H, W), np.float64)
    lib().or_chain_f_backward(C, H, W, _c(offx, np.int32), _c(offy, np.int32), _c(mapx, np.int32),
                              _c(mapy, np.int32), gy, gx)
    return gx
