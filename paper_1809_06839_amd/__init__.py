"""MI355X (gfx950) batched image augmentation: a thin Python binding of
libmiaug, the HIP implementation of the augmentation hot path of
Buslaev et al., "Albumentations: fast and flexible image augmentations"
(arXiv:1809.06839).

Every function marshals torch tensors (device memory) and the current HIP
stream into the C ABI declared in ``include/miaug.h``; all image work runs in
the library's HIP kernels.  There is no CPU fallback: if ``libmiaug.so`` is
not built, loading raises ``RuntimeError``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loaded first so that libmiaug binds to the HIP runtime torch uses

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libmiaug.so")

OK, EINVAL, ESHAPE, EUNSUPPORTED, EDEVICE, ENOMEM, ECAPACITY = 0, -1, -2, -3, -4, -5, -6

IMAGENET_MEAN = (0.485, 0.456, 0.406)
IMAGENET_STD = (0.229, 0.224, 0.225)


class MiaugError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("miaug status %d (%s): %s" % (status, _status_str(status), msg))
        self.status = status


_vp, _i, _i64, _u64, _d, _sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t


class RaggedArgs(ctypes.Structure):
    """Mirror of miaug_ragged_args (include/miaug.h)."""
    _fields_ = [("n", ctypes.c_int32), ("out_h", ctypes.c_int32), ("out_w", ctypes.c_int32),
                ("img", _vp), ("img_off", _vp), ("hw", _vp), ("flags", _vp), ("ab", _vp), ("crop", _vp),
                ("mask", _vp), ("mask_off", _vp), ("boxes", _vp), ("box_off", _vp),
                ("mean", ctypes.c_float * 3), ("stdv", ctypes.c_float * 3),
                ("out", _vp), ("out_mask", _vp), ("out_boxes", _vp)]


class C2Record(ctypes.Structure):
    """Mirror of miaug_c2_record (include/miaug.h)."""
    _fields_ = [("aq", ctypes.c_int64 * 6), ("crop_x", ctypes.c_int32), ("crop_y", ctypes.c_int32),
                ("dh", ctypes.c_int32), ("ds", ctypes.c_int32), ("dv", ctypes.c_int32), ("blur", ctypes.c_int32),
                ("gamma_lut", ctypes.c_uint8 * 256)]


class Op(ctypes.Structure):
    """Mirror of miaug_op (include/miaug.h)."""
    _fields_ = [("kind", ctypes.c_uint32), ("p", ctypes.c_float), ("lo", ctypes.c_float * 4),
                ("hi", ctypes.c_float * 4), ("interp", ctypes.c_uint32), ("border", ctypes.c_uint32),
                ("out_h", ctypes.c_int32), ("out_w", ctypes.c_int32)]


class Params(ctypes.Structure):
    """Mirror of miaug_params (include/miaug.h): one sample's parameters."""
    _fields_ = [("seed", ctypes.c_uint64), ("index", ctypes.c_uint64), ("flags", ctypes.c_int32 * 4),
                ("alpha", ctypes.c_float), ("beta", ctypes.c_float), ("angle", ctypes.c_float),
                ("scale", ctypes.c_float), ("dx", ctypes.c_float), ("dy", ctypes.c_float),
                ("crop_x", ctypes.c_int32), ("crop_y", ctypes.c_int32), ("dh", ctypes.c_int32),
                ("ds", ctypes.c_int32), ("dv", ctypes.c_int32), ("gamma", ctypes.c_float),
                ("blur", ctypes.c_int32), ("crop_h", ctypes.c_int32), ("crop_w", ctypes.c_int32),
                ("shift", ctypes.c_float * 3), ("gray", ctypes.c_int32), ("grid", ctypes.c_double * 10)]


class BatchIn(ctypes.Structure):
    """Mirror of miaug_batch_in (include/miaug.h)."""
    _fields_ = [("n", ctypes.c_int32), ("channels", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("img", _vp), ("img_off", _vp), ("hw", _vp), ("mask", _vp), ("mask_off", _vp), ("boxes", _vp),
                ("box_off", _vp)]


class BatchOut(ctypes.Structure):
    """Mirror of miaug_batch_out (include/miaug.h)."""
    _fields_ = [("img", _vp), ("mask", _vp), ("boxes", _vp)]


_SIGS = {
    "miaug_compile_c2": (_i, [_vp, _vp, _i, _i, _i, _i, _vp]),
    "miaug_version": (_i, []),
    "miaug_status_str": (ctypes.c_char_p, [_i]),
    "miaug_last_error": (ctypes.c_char_p, []),
    "miaug_sample_d4bc": (_i, [_u64, _u64, _i, _vp, _vp]),
    "miaug_sample_c2": (_i, [_u64, _u64, _i, _i, _vp, _vp]),
    "miaug_sample_wc": (_i, [_u64, _u64, _i, _vp]),
    "miaug_sample_grid": (_i, [_u64, _u64, _i, _d, _vp]),
    "miaug_ctx_create": (_i, [_i, ctypes.c_char_p, ctypes.POINTER(_vp)]),
    "miaug_ctx_stats": (_i, [_vp, ctypes.c_void_p]),
    "miaug_tune_cache_lookup": (_i, [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(_i), ctypes.POINTER(ctypes.c_float),
                                     ctypes.c_char_p, _sz]),
    "miaug_tune_cache_store": (_i, [ctypes.c_char_p, ctypes.c_char_p, _i, ctypes.c_char_p, ctypes.c_float]),
    "miaug_debug_fail_alloc_after": (_i, [ctypes.c_long]),
    "miaug_debug_alloc_probe": (_i, [_sz]),
    "miaug_ctx_destroy": (_i, [_vp]),
    "miaug_d4_bc_u8": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _vp, _vp]),
    "miaug_ssr_crop_resize_hsv_gamma_blur_u8": (_i, [_vp, _i, _i, _i, _vp, _i, _i, _vp, _vp]),
    "miaug_ssr_crop_resize_mask_u8": (_i, [_vp, _i, _i, _i, _vp, _i, _i, _vp, _vp]),
    "miaug_d4_lut_u8": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp]),
    "miaug_boxes_elastic_grid": (_i, [_vp, _vp, _i, _i, _i, _vp, _vp, _vp, _vp, _vp]),
    "miaug_ragged_masks_u8": (_i, [ctypes.POINTER(RaggedArgs), _i, _vp, _vp]),
    "miaug_compile_color_luts": (_i, [_vp, _vp, _i, _i, _vp]),
    "miaug_pad_u8": (_i, [_vp, _i, _i, _i, _i, _i, _i, _i, _i, _vp, _vp]),
    "miaug_compile_gamma_luts": (_i, [_vp, _i, _i, _vp]),
    "miaug_hsv_shift_u8": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp]),
    "miaug_blur_u8": (_i, [_vp, _i, _i, _i, _i, _i, _vp, _vp, _vp]),
    "miaug_warp_affine_u8": (_i, [_vp, _i, _i, _i, _i, _vp, _i, _i, _vp, _vp]),
    "miaug_compile_ssr_q32": (_i, [_vp, _i, _i, _i, _vp]),
    "miaug_boxes_ssr_crop_resize": (_i, [_vp, _vp, _i, _i, _i, _vp, _i, _i, _vp, _vp]),
    "miaug_ragged_apply": (_i, [_vp, ctypes.POINTER(RaggedArgs), _vp]),
    "miaug_ragged_apply_per_image": (_i, [_vp, ctypes.POINTER(RaggedArgs), _vp]),
    "miaug_ragged_graph_create": (_i, [_vp, ctypes.POINTER(RaggedArgs), _vp, ctypes.POINTER(_vp)]),
    "miaug_graph_launch": (_i, [_vp, _vp]),
    "miaug_graph_destroy": (_i, [_vp]),
    "miaug_ragged_autotune": (_i, [_vp, ctypes.POINTER(RaggedArgs), _i, _vp, ctypes.POINTER(_i),
                                   ctypes.POINTER(ctypes.c_float), _vp]),
    "miaug_ragged_variant_count": (_i, []),
    "miaug_ragged_variant_name": (ctypes.c_char_p, [_i]),
    "miaug_ragged_set_variant": (_i, [_vp, _i]),
    "miaug_ragged_apply_noalloc": (_i, [ctypes.POINTER(RaggedArgs), _i, _vp]),
    "miaug_warpcolor_fwd": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _vp]),
    "miaug_warpcolor_workspace_bytes": (_sz, [_i, _i, _i, _i]),
    "miaug_warpcolor_bwd": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "miaug_elastic_workspace_bytes": (_sz, [_i, _i, _i]),
    "miaug_elastic_fields": (_i, [_u64, _u64, _i, _i, _i, _d, _i, _i, _vp, _vp, _sz, _vp]),
    "miaug_elastic_box_workspace_bytes": (_sz, [_i, _i, _i]),
    "miaug_elastic_fields_box": (_i, [_u64, _u64, _i, _i, _i, _d, _i, _vp, _vp, _sz, _vp]),
    "miaug_grid_tables": (_i, [_vp, _i, _i, _i, _vp, _vp, _vp]),
    "miaug_elastic_grid_u8": (_i, [_vp, _vp, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _i, _vp]),
    "miaug_chain_f32_workspace_bytes": (_sz, [_i, _i, _i, _i]),
    "miaug_elastic_grid_f32_fwd": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "miaug_elastic_grid_f32_bwd": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "miaug_image_stats_u8": (_i, [_vp, _i, _i64, _i, _vp, _vp, _vp, _vp, _vp]),
    "miaug_pipeline_create": (_i, [_vp, ctypes.POINTER(Op), _i, ctypes.POINTER(_vp)]),
    "miaug_pipeline_destroy": (_i, [_vp]),
    "miaug_pipeline_kind": (_i, [_vp]),
    "miaug_param_bytes": (_sz, [_vp, _i]),
    "miaug_sample": (_i, [_vp, _u64, _u64, _i, _vp, _vp]),
    "miaug_apply": (_i, [_vp, ctypes.POINTER(BatchIn), _vp, ctypes.POINTER(BatchOut), _vp]),
    "miaug_apply_per_image": (_i, [_vp, ctypes.POINTER(BatchIn), _vp, ctypes.POINTER(BatchOut), _vp]),
    "miaug_pipeline_graph_capture": (_i, [_vp, ctypes.POINTER(BatchIn), ctypes.POINTER(BatchOut), _vp,
                                          ctypes.POINTER(_vp)]),
    "miaug_pipeline_graph_launch": (_i, [_vp, _vp, _vp]),
    "miaug_pipeline_graph_destroy": (_i, [_vp]),
    "miaug_pipeline_autotune": (_i, [_vp, ctypes.POINTER(BatchIn), _vp, ctypes.POINTER(BatchOut), _i, _vp]),
}

_lib = None


def lib():
    """The loaded libmiaug (raises RuntimeError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmiaug.so is not built (%s); run __graft_entry__.build() or "
                               "python paper_1809_06839_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _status_str(s):
    try:
        return lib().miaug_status_str(s).decode()
    except Exception:
        return "?"


def _check(status):
    if status != OK:
        raise MiaugError(status, lib().miaug_last_error().decode())
    return status


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


# ---------------------------------------------------------------- sampler (host)
def sample_d4bc(seed: int, first: int, n: int):
    flags = np.zeros((n, 4), np.int32); ab = np.zeros((n, 2), np.float32)
    _check(lib().miaug_sample_d4bc(seed, first, n, flags.ctypes.data, ab.ctypes.data))
    return flags, ab


def sample_c2(seed: int, first: int, n: int, crop_range: int = 64):
    f = np.zeros((n, 5), np.float32); k = np.zeros((n, 5), np.int32)
    _check(lib().miaug_sample_c2(seed, first, n, crop_range, f.ctypes.data, k.ctypes.data))
    return f, k


def sample_wc(seed: int, first: int, n: int):
    f = np.zeros((n, 7), np.float32)
    _check(lib().miaug_sample_wc(seed, first, n, f.ctypes.data))
    return f


def sample_grid(seed: int, first: int, n: int, limit: float = 0.3):
    f = np.zeros((n, 10), np.float64)
    _check(lib().miaug_sample_grid(seed, first, n, limit, f.ctypes.data))
    return f


# ---------------------------------------------------------------- context
class Stats(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_uint64), ("launches", ctypes.c_uint64), ("tune_runs", ctypes.c_uint64),
                ("tune_cache_hits", ctypes.c_uint64), ("errors", ctypes.c_uint64), ("variant", ctypes.c_int32),
                ("last_status", ctypes.c_int32)]


class Context:
    """Per-device state (queue counters, tuned variant, autotuner cache file) of the ragged kernels."""

    def __init__(self, device: int = 0, tune_cache: str | None = None):
        h = ctypes.c_void_p()
        _check(lib().miaug_ctx_create(device, tune_cache.encode() if tune_cache else None, ctypes.byref(h)))
        self.handle = h

    def stats(self) -> dict:
        st = Stats()
        _check(lib().miaug_ctx_stats(self.handle, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in Stats._fields_}

    def close(self):
        if self.handle:
            lib().miaug_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_variant(self, v: int):
        _check(lib().miaug_ragged_set_variant(self.handle, v))


def tune_cache_lookup(path: str, key: str):
    """(variant, ms, name) stored under key in an autotuner cache file, or None."""
    v, ms, name = ctypes.c_int(), ctypes.c_float(), ctypes.create_string_buffer(256)
    st = lib().miaug_tune_cache_lookup(path.encode(), key.encode(), ctypes.byref(v), ctypes.byref(ms), name, 256)
    if st == EUNSUPPORTED:
        return None
    _check(st)
    return v.value, ms.value, name.value.decode()


def tune_cache_store(path: str, key: str, variant: int, name: str, ms: float):
    _check(lib().miaug_tune_cache_store(path.encode(), key.encode(), variant, name.encode(), ms))


def debug_fail_alloc_after(after: int):
    """The library's allocation number `after` from now fails with MIAUG_ENOMEM, once (-1 disarms)."""
    _check(lib().miaug_debug_fail_alloc_after(after))


def ragged_variants():
    L = lib()
    return [L.miaug_ragged_variant_name(i).decode() for i in range(L.miaug_ragged_variant_count())]


# ---------------------------------------------------------------- plain Dih4 + brightness/contrast
def d4_bc_u8(img, flags, ab, out=None, stream=None):
    """img [n, H, W, C] u8 -> out (same byte size; image i has shape (H, W, C) or (W, H, C))."""
    _dev(img, torch.uint8, "img"); _dev(flags, torch.int32, "flags"); _dev(ab, torch.float32, "ab")
    n, H, W, C = img.shape
    if out is None:
        out = torch.empty_like(img)
    _dev(out, torch.uint8, "out")
    _check(lib().miaug_d4_bc_u8(_p(img), n, H, W, C, _p(flags), _p(ab), _p(out), _stream(stream)))
    return out


# ---------------------------------------------------------------- full u8 pipeline
def compile_c2(f, k, H, W, crop=448):
    """Host parameter compile: returns an (n, 328) uint8 array of miaug_c2_record."""
    f = np.ascontiguousarray(f, np.float32); k = np.ascontiguousarray(k, np.int32)
    n = len(f)
    rec = (C2Record * max(n, 1))()
    _check(lib().miaug_compile_c2(f.ctypes.data, k.ctypes.data, n, H, W, crop, ctypes.addressof(rec)))
    return np.frombuffer(bytes(rec), dtype=np.uint8).reshape(max(n, 1), ctypes.sizeof(C2Record))[:n].copy()


def ssr_crop_resize_hsv_gamma_blur_u8(img, rec, crop=448, outsz=224, out=None, stream=None):
    """img [n, H, W, 3] u8; rec: device uint8 [n, sizeof(miaug_c2_record)] from compile_c2."""
    _dev(img, torch.uint8, "img"); _dev(rec, torch.uint8, "rec")
    n, H, W, C = img.shape
    if C != 3:
        raise ValueError("RGB images expected")
    if rec.numel() != n * ctypes.sizeof(C2Record):
        raise ValueError("rec must hold n records")
    if out is None:
        out = torch.empty((n, outsz, outsz, 3), dtype=torch.uint8, device=img.device)
    _check(lib().miaug_ssr_crop_resize_hsv_gamma_blur_u8(_p(img), n, H, W, _p(rec), crop, outsz, _p(out),
                                                         _stream(stream)))
    return out


def ssr_crop_resize_mask_u8(mask, rec, crop=448, outsz=224, out=None, stream=None):
    """Masks [n, H, W] u8 under the same records (nearest, no colour ops)."""
    _dev(mask, torch.uint8, "mask"); _dev(rec, torch.uint8, "rec")
    n, H, W = mask.shape
    if rec.numel() != n * ctypes.sizeof(C2Record):
        raise ValueError("rec must hold n records")
    if out is None:
        out = torch.empty((n, outsz, outsz), dtype=torch.uint8, device=mask.device)
    _check(lib().miaug_ssr_crop_resize_mask_u8(_p(mask), n, H, W, _p(rec), crop, outsz, _p(out), _stream(stream)))
    return out


def boxes_ssr_crop_resize(boxes, box_off, H, W, rec, crop=448, outsz=224, out=None, stream=None):
    """Boxes float [nbox, 4] (CSR by image: box_off int32 [n + 1]) under the same records."""
    _dev(boxes, torch.float32, "boxes"); _dev(box_off, torch.int32, "box_off"); _dev(rec, torch.uint8, "rec")
    n = box_off.numel() - 1
    if rec.numel() != n * ctypes.sizeof(C2Record):
        raise ValueError("rec must hold n records")
    if out is None:
        out = torch.empty_like(boxes)
    _check(lib().miaug_boxes_ssr_crop_resize(_p(boxes), _p(box_off), n, H, W, _p(rec), crop, outsz, _p(out),
                                             _stream(stream)))
    return out


def compile_color_luts(ab=None, shift=None, n=None, C=3):
    """Host u8 [n, C, 256]: brightness/contrast (ab [n, 2]) then ShiftRGB (shift [n, C]) LUTs."""
    abh = None if ab is None else np.ascontiguousarray(ab, np.float32)
    sh = None if shift is None else np.ascontiguousarray(shift, np.float32)
    n = n if n is not None else (len(abh) if abh is not None else len(sh))
    luts = np.zeros((n, C, 256), np.uint8)
    _check(lib().miaug_compile_color_luts(None if abh is None else abh.ctypes.data,
                                          None if sh is None else sh.ctypes.data, n, C, luts.ctypes.data))
    return luts


def d4_lut_u8(img, flags, luts, gray=None, out=None, stream=None):
    """img [n, H, W, C] u8; flags [n, 4] int32; luts [n, C, 256] u8; gray [n] int32 or None (device)."""
    _dev(img, torch.uint8, "img"); _dev(flags, torch.int32, "flags"); _dev(luts, torch.uint8, "luts")
    if gray is not None:
        _dev(gray, torch.int32, "gray")
    n, H, W = img.shape[:3]
    C = img.shape[3] if img.dim() == 4 else 1
    if out is None:
        out = torch.empty_like(img)
    _check(lib().miaug_d4_lut_u8(_p(img), n, H, W, C, _p(flags), _p(luts), None if gray is None else _p(gray),
                                 _p(out), _stream(stream)))
    return out


def compile_gamma_luts(gamma, C=3):
    """Host u8 [n, C, 256]: the Gamma LUT of each image (gamma [n]) for every channel."""
    g = np.ascontiguousarray(gamma, np.float32)
    luts = np.zeros((len(g), C, 256), np.uint8)
    _check(lib().miaug_compile_gamma_luts(g.ctypes.data, len(g), C, luts.ctypes.data))
    return luts


def blur_u8(img, ksize=3, apply=None, out=None, stream=None):
    """img [n, H, W(, C)] u8; ksize 3 or 5; apply [n] int32 (device) or None (every image)."""
    _dev(img, torch.uint8, "img")
    if apply is not None:
        _dev(apply, torch.int32, "apply")
    n, H, W = img.shape[:3]
    C = img.shape[3] if img.dim() == 4 else 1
    if out is None:
        out = torch.empty_like(img)
    _check(lib().miaug_blur_u8(_p(img), n, H, W, C, ksize, None if apply is None else _p(apply), _p(out),
                               _stream(stream)))
    return out


def hsv_shift_u8(img, dhsv, out=None, stream=None):
    """img [n, H, W, 3] u8; dhsv [n, 3] int32 (dh, ds, dv), both on the device."""
    _dev(img, torch.uint8, "img"); _dev(dhsv, torch.int32, "dhsv")
    if img.dim() != 4 or img.shape[3] != 3:
        raise MiaugError(ESHAPE, "hsv_shift_u8: img must be [n, H, W, 3]")
    n, H, W = img.shape[:3]
    if out is None:
        out = torch.empty_like(img)
    _check(lib().miaug_hsv_shift_u8(_p(img), n, H, W, _p(dhsv), _p(out), _stream(stream)))
    return out


def pad_u8(img, min_h, min_w, border=0, value=0, out=None, stream=None):
    _dev(img, torch.uint8, "img")
    n, H, W = img.shape[:3]
    C = img.shape[3] if img.dim() == 4 else 1
    Ho, Wo = max(H, min_h), max(W, min_w)
    if out is None:
        out = torch.empty((n, Ho, Wo) + ((C,) if img.dim() == 4 else ()), dtype=torch.uint8, device=img.device)
    _check(lib().miaug_pad_u8(_p(img), n, H, W, C, min_h, min_w, border, value, _p(out), _stream(stream)))
    return out


def compile_ssr_q32(f, H, W):
    """Host int64 [n, 6] Q32 inverse matrices of f [n, 4] = {angle_deg, scale, dx, dy}."""
    fh = np.ascontiguousarray(f, np.float32).reshape(-1, 4)
    aq = np.zeros((len(fh), 6), np.int64)
    _check(lib().miaug_compile_ssr_q32(fh.ctypes.data, len(fh), H, W, aq.ctypes.data))
    return aq


def warp_affine_u8(img, aq, interp=0, border=0, out=None, stream=None):
    """img [n, H, W(, C)] u8; aq device int64 [n, 6]."""
    _dev(img, torch.uint8, "img"); _dev(aq, torch.int64, "aq")
    n, H, W = img.shape[:3]
    C = img.shape[3] if img.dim() == 4 else 1
    if out is None:
        out = torch.empty_like(img)
    _check(lib().miaug_warp_affine_u8(_p(img), n, H, W, C, _p(aq), interp, border, _p(out), _stream(stream)))
    return out


# ---------------------------------------------------------------- ragged batch
class Ragged:
    """Device-side ragged batch + outputs, packed into one miaug_ragged_args."""

    def __init__(self, img, img_off, hw, flags, ab, out_h=224, out_w=224, mask=None, mask_off=None, boxes=None,
                 box_off=None, mean=IMAGENET_MEAN, std=IMAGENET_STD, out=None, out_mask=None, out_boxes=None,
                 crop=None):
        n = hw.shape[0]
        dev = img.device
        _dev(img, torch.uint8, "img"); _dev(img_off, torch.int64, "img_off"); _dev(hw, torch.int32, "hw")
        _dev(flags, torch.int32, "flags"); _dev(ab, torch.float32, "ab")
        if crop is not None:
            _dev(crop, torch.int32, "crop")
        self.out = out if out is not None else torch.empty((n, 3, out_h, out_w), dtype=torch.float32, device=dev)
        self.out_mask = None
        self.out_boxes = None
        if mask is not None:
            _dev(mask, torch.uint8, "mask"); _dev(mask_off, torch.int64, "mask_off")
            self.out_mask = out_mask if out_mask is not None else torch.empty((n, out_h, out_w), dtype=torch.uint8,
                                                                              device=dev)
        if boxes is not None:
            _dev(boxes, torch.float32, "boxes"); _dev(box_off, torch.int32, "box_off")
            self.out_boxes = out_boxes if out_boxes is not None else torch.empty_like(boxes)
        self.keep = (img, img_off, hw, flags, ab, mask, mask_off, boxes, box_off, crop)
        a = RaggedArgs()
        a.n, a.out_h, a.out_w = n, out_h, out_w
        a.img, a.img_off, a.hw, a.flags, a.ab = (t.data_ptr() for t in (img, img_off, hw, flags, ab))
        a.crop = crop.data_ptr() if crop is not None else None
        a.mask = mask.data_ptr() if mask is not None else None
        a.mask_off = mask_off.data_ptr() if mask is not None else None
        a.boxes = boxes.data_ptr() if boxes is not None and boxes.numel() > 0 else None
        a.box_off = box_off.data_ptr() if a.boxes else None
        a.mean = (ctypes.c_float * 3)(*mean)
        a.stdv = (ctypes.c_float * 3)(*std)
        a.out = self.out.data_ptr()
        a.out_mask = self.out_mask.data_ptr() if self.out_mask is not None else None
        a.out_boxes = self.out_boxes.data_ptr() if a.boxes else None
        self.args = a

    @classmethod
    def from_host(cls, batch, flags, ab, device="cuda", crop=None, **kw):
        """Uploads a synth.RaggedBatch-like host batch and host parameters
        (crop: optional host int32 [n][4] windows {y0, x0, h, w})."""
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dtype=dt).to(device)
        has_mask = batch.mask is not None
        has_boxes = batch.boxes is not None and len(batch.boxes) > 0
        return cls(t(batch.img, torch.uint8), t(batch.img_off, torch.int64), t(batch.hw, torch.int32),
                   t(flags, torch.int32), t(ab, torch.float32),
                   mask=t(batch.mask, torch.uint8) if has_mask else None,
                   mask_off=t(batch.mask_off, torch.int64) if has_mask else None,
                   boxes=t(batch.boxes, torch.float32) if has_boxes else None,
                   box_off=t(batch.box_off, torch.int32) if has_boxes else None,
                   crop=t(crop, torch.int32) if crop is not None else None, **kw)


def ragged_apply(ctx: Context, r: Ragged, stream=None):
    _check(lib().miaug_ragged_apply(ctx.handle, ctypes.byref(r.args), _stream(stream)))
    return r


def ragged_apply_noalloc(r: Ragged, variant: int = -1, stream=None):
    """ragged_apply without a context or any device allocation (static counters)."""
    _check(lib().miaug_ragged_apply_noalloc(ctypes.byref(r.args), variant, _stream(stream)))
    return r


def ragged_masks_u8(r: Ragged, channels: int, out=None, stream=None):
    """Multi-channel masks of a Ragged whose mask buffer holds `channels` bytes per pixel."""
    a = r.args
    if out is None:
        out = torch.empty((a.n, a.out_h, a.out_w, channels), dtype=torch.uint8, device=r.out.device)
    _check(lib().miaug_ragged_masks_u8(ctypes.byref(a), channels, _p(out), _stream(stream)))
    return out


def ragged_apply_per_image(ctx: Context, r: Ragged, stream=None):
    _check(lib().miaug_ragged_apply_per_image(ctx.handle, ctypes.byref(r.args), _stream(stream)))
    return r


def ragged_autotune(ctx: Context, r: Ragged, reps: int = 3, stream=None, return_times=False):
    """Times every launch variant (parity-gated); returns (chosen, ms) or (chosen, ms, times)."""
    v, ms = ctypes.c_int(), ctypes.c_float()
    times = np.zeros(lib().miaug_ragged_variant_count(), np.float32)
    _check(lib().miaug_ragged_autotune(ctx.handle, ctypes.byref(r.args), reps, _stream(stream), ctypes.byref(v),
                                       ctypes.byref(ms), times.ctypes.data))
    return (v.value, ms.value, times.tolist()) if return_times else (v.value, ms.value)


class Graph:
    """A captured hipGraph of ragged_apply for fixed buffers."""

    def __init__(self, ctx: Context, r: Ragged, stream):
        h = ctypes.c_void_p()
        _check(lib().miaug_ragged_graph_create(ctx.handle, ctypes.byref(r.args), _stream(stream), ctypes.byref(h)))
        self.handle, self.r = h, r

    def launch(self, stream=None):
        _check(lib().miaug_graph_launch(self.handle, _stream(stream)))

    def close(self):
        if self.handle:
            lib().miaug_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- differentiable warp + colour
def warpcolor_fwd(x, params, out=None, stream=None):
    """x [n, C, H, W] float32, params [n, 7] float32 -> y."""
    _dev(x, torch.float32, "x"); _dev(params, torch.float32, "params")
    n, C, H, W = x.shape
    y = out if out is not None else torch.empty_like(x)
    _check(lib().miaug_warpcolor_fwd(_p(x), n, C, H, W, _p(params), _p(y), _stream(stream)))
    return y


def warpcolor_bwd(x, params, gy, want_gx=True, stream=None):
    _dev(x, torch.float32, "x"); _dev(params, torch.float32, "params"); _dev(gy, torch.float32, "gy")
    n, C, H, W = x.shape
    ws = torch.empty(max(1, lib().miaug_warpcolor_workspace_bytes(n, C, H, W)), dtype=torch.uint8, device=x.device)
    gx = torch.empty_like(x) if want_gx else None
    gp = torch.empty_like(params)
    _check(lib().miaug_warpcolor_bwd(_p(x), n, C, H, W, _p(params), _p(gy), _p(gx), _p(gp), _p(ws), ws.numel(),
                                     _stream(stream)))
    return gx, gp


class WarpColor(torch.autograd.Function):
    """y = clamp(alpha * warp(x; angle, scale, tx, ty) + beta, 0, 1) ** gamma with
    hand-written HIP backward kernels for x and the [n, 7] parameters."""

    @staticmethod
    def forward(ctx, x, params):
        x = x.contiguous(); params = params.contiguous()
        ctx.save_for_backward(x, params)
        return warpcolor_fwd(x, params)

    @staticmethod
    def backward(ctx, gy):
        x, params = ctx.saved_tensors
        gx, gp = warpcolor_bwd(x, params, gy.contiguous(), want_gx=ctx.needs_input_grad[0])
        return gx, gp


def warp_color(x, params):
    return WarpColor.apply(x, params)


# ---------------------------------------------------------------- elastic + grid distortion
def elastic_fields(seed, first, n, H, W, sigma=50.0, alpha=1000, radius=150, device="cuda", stream=None):
    """Q10 displacement fields [n, 2, H, W] int32 (field 0: x, field 1: y)."""
    off = torch.empty((n, 2, H, W), dtype=torch.int32, device=device)
    ws = torch.empty(max(1, lib().miaug_elastic_workspace_bytes(n, H, W)), dtype=torch.uint8, device=device)
    _check(lib().miaug_elastic_fields(seed, first, n, H, W, sigma, alpha, radius, _p(off), _p(ws), ws.numel(),
                                      _stream(stream)))
    return off


def elastic_fields_box(seed, first, n, H, W, sigma=50.0, alpha=1000, device="cuda", stream=None):
    """Box-cascade approximation of elastic_fields: Q10 offsets [n, 2, H, W] int32."""
    off = torch.empty((n, 2, H, W), dtype=torch.int32, device=device)
    ws = torch.empty(max(1, lib().miaug_elastic_box_workspace_bytes(n, H, W)), dtype=torch.uint8, device=device)
    _check(lib().miaug_elastic_fields_box(seed, first, n, H, W, sigma, alpha, _p(off), _p(ws), ws.numel(),
                                          _stream(stream)))
    return off


def grid_tables(grid, H, W, stream=None):
    """grid: device float64 [n, 10] -> (mapx [n, W], mapy [n, H]) int32 Q10 tables."""
    _dev(grid, torch.float64, "grid")
    n = grid.shape[0]
    mapx = torch.empty((n, W), dtype=torch.int32, device=grid.device)
    mapy = torch.empty((n, H), dtype=torch.int32, device=grid.device)
    _check(lib().miaug_grid_tables(_p(grid), n, H, W, _p(mapx), _p(mapy), _stream(stream)))
    return mapx, mapy


def elastic_grid_u8(img, off, mapx, mapy, mask=None, per_image=False, stream=None):
    """img [n, H, W, C] u8 (+ mask [n, H, W] u8) -> elastic then grid distortion."""
    _dev(img, torch.uint8, "img"); _dev(off, torch.int32, "off")
    _dev(mapx, torch.int32, "mapx"); _dev(mapy, torch.int32, "mapy")
    n, H, W, C = img.shape
    out = torch.empty_like(img)
    om = torch.empty_like(mask) if mask is not None else None
    if mask is not None:
        _dev(mask, torch.uint8, "mask")
    _check(lib().miaug_elastic_grid_u8(_p(img), _p(mask), n, H, W, C, _p(off), _p(mapx), _p(mapy), _p(out), _p(om),
                                       int(per_image), _stream(stream)))
    return out, om


def elastic_grid_f32_fwd(x, off, mapx, mapy, stream=None):
    _dev(x, torch.float32, "x")
    n, C, H, W = x.shape
    y = torch.empty_like(x)
    ws = torch.empty(max(1, lib().miaug_chain_f32_workspace_bytes(n, C, H, W)), dtype=torch.uint8, device=x.device)
    _check(lib().miaug_elastic_grid_f32_fwd(_p(x), n, C, H, W, _p(off), _p(mapx), _p(mapy), _p(y), _p(ws),
                                            ws.numel(), _stream(stream)))
    return y


def elastic_grid_f32_bwd(gy, off, mapx, mapy, stream=None):
    _dev(gy, torch.float32, "gy")
    n, C, H, W = gy.shape
    gx = torch.empty_like(gy)
    ws = torch.empty(max(1, lib().miaug_chain_f32_workspace_bytes(n, C, H, W)), dtype=torch.uint8, device=gy.device)
    _check(lib().miaug_elastic_grid_f32_bwd(_p(gy), n, C, H, W, _p(off), _p(mapx), _p(mapy), _p(gx), _p(ws),
                                            ws.numel(), _stream(stream)))
    return gx


class ElasticGridF32(torch.autograd.Function):
    """Float copy of the elastic + grid chain; gradient w.r.t. the image only
    (the fields and grid tables are random draws, not parameters)."""

    @staticmethod
    def forward(ctx, x, off, mapx, mapy):
        ctx.save_for_backward(off, mapx, mapy)
        return elastic_grid_f32_fwd(x.contiguous(), off, mapx, mapy)

    @staticmethod
    def backward(ctx, gy):
        off, mapx, mapy = ctx.saved_tensors
        return elastic_grid_f32_bwd(gy.contiguous(), off, mapx, mapy), None, None, None


# ---------------------------------------------------------------- statistics
def image_stats_u8(img, C=None, stream=None):
    """img [n, ..., C] u8 -> (sum [n, C] uint64 as int64, min, max [n, C] int32, hist [n, C, 256] int32)."""
    _dev(img, torch.uint8, "img")
    n = img.shape[0]
    C = C or img.shape[-1]
    npix = img[0].numel() // C
    dev = img.device
    s = torch.empty((n, C), dtype=torch.int64, device=dev)
    mn = torch.empty((n, C), dtype=torch.int32, device=dev)
    mx = torch.empty((n, C), dtype=torch.int32, device=dev)
    h = torch.empty((n, C, 256), dtype=torch.int32, device=dev)
    _check(lib().miaug_image_stats_u8(_p(img), n, npix, C, _p(s), _p(mn), _p(mx), _p(h), _stream(stream)))
    return s, mn, mx, h


# ---------------------------------------------------------------- op-list pipelines
OP = {"HFLIP": 1, "VFLIP": 2, "ROT90": 3, "TRANSPOSE": 4, "SSR": 5, "CROP": 6, "RESIZE": 7, "BRIGHT_CONTRAST": 8,
      "HSV": 9, "GAMMA": 10, "BLUR3": 11, "BLUR5": 12, "ELASTIC": 13, "GRID": 14, "NORMALIZE": 15,
      "SIZED_CROP": 16, "SHIFT_RGB": 17, "TO_GRAY": 18, "PAD": 19, "ROTATE": 20}
PIPE = {1: "DIH4", 2: "RAGGED", 3: "U8CHAIN", 4: "DISTORT", 5: "WARP", 6: "PAD", 7: "HSV", 8: "BLUR"}
INTERP_BILINEAR, INTERP_NEAREST = 0, 1
BORDER_REFLECT101, BORDER_CONSTANT = 0, 1


def op(kind, p=1.0, lo=(0, 0, 0, 0), hi=(0, 0, 0, 0), interp=INTERP_BILINEAR, border=BORDER_REFLECT101,
       out=(0, 0)):
    """One miaug_op; `kind` is a name of OP or its value; lo, hi take up to 4 values."""
    o = Op()
    o.kind = OP[kind] if isinstance(kind, str) else int(kind)
    o.p = p
    lo = list(lo) + [0] * (4 - len(lo))
    hi = list(hi) + [0] * (4 - len(hi))
    for i in range(4):
        o.lo[i] = lo[i]
        o.hi[i] = hi[i]
    o.interp, o.border = interp, border
    o.out_h, o.out_w = out
    return o


class Pipeline:
    """An op list compiled onto one fused chain (miaug_pipeline_create)."""

    def __init__(self, ctx, ops):
        self.ops = (Op * len(ops))(*ops)
        h = _vp()
        _check(lib().miaug_pipeline_create(ctx.handle if ctx is not None else None, self.ops, len(ops),
                                           ctypes.byref(h)))
        self.handle = h

    @property
    def kind(self):
        return PIPE[lib().miaug_pipeline_kind(self.handle)]

    def sample(self, seed, first, n, hw=None):
        """n parameter records (a ctypes array of Params); hw: host int32 [n, 2] when the list has CROP."""
        recs = (Params * max(n, 1))()
        hwa = None if hw is None else np.ascontiguousarray(hw, dtype=np.int32)
        _check(lib().miaug_sample(self.handle, seed, first, n, None if hwa is None else hwa.ctypes.data,
                                  ctypes.byref(recs)))
        return recs

    @staticmethod
    def batch(img=None, mask=None, ragged=None, boxes=None, box_off=None):
        """miaug_batch_in / miaug_batch_out for a dense batch (img [n, H, W, C] u8, mask [n, H, W] u8, boxes
        float [nbox, 4] with box_off int32 [n + 1]) or a Ragged (its packed inputs and outputs).  Returns
        (batch_in, batch_out, outputs); the caller sets the output pointers of a dense batch."""
        bi, bo = BatchIn(), BatchOut()
        if ragged is not None:
            a = ragged.args
            bi.n, bi.channels, bi.H, bi.W = a.n, 3, 0, 0
            bi.img, bi.img_off, bi.hw = a.img, a.img_off, a.hw
            bi.mask, bi.mask_off, bi.boxes, bi.box_off = a.mask, a.mask_off, a.boxes, a.box_off
            bo.img, bo.mask, bo.boxes = a.out, a.out_mask, a.out_boxes
            return bi, bo, ragged
        _dev(img, torch.uint8, "img")
        n, H, W = img.shape[:3]
        bi.n, bi.channels, bi.H, bi.W = n, (img.shape[3] if img.dim() == 4 else 1), H, W
        bi.img = img.data_ptr()
        if mask is not None:
            _dev(mask, torch.uint8, "mask")
            bi.mask = mask.data_ptr()
        if boxes is not None:
            _dev(boxes, torch.float32, "boxes"); _dev(box_off, torch.int32, "box_off")
            bi.boxes, bi.box_off = boxes.data_ptr(), box_off.data_ptr()
        return bi, bo, None

    def apply(self, bi, bo, params, stream=None, per_image=False):
        f = lib().miaug_apply_per_image if per_image else lib().miaug_apply
        _check(f(self.handle, ctypes.byref(bi), ctypes.byref(params), ctypes.byref(bo), _stream(stream)))

    def autotune(self, bi, bo, params, reps=3, stream=None):
        _check(lib().miaug_pipeline_autotune(self.handle, ctypes.byref(bi), ctypes.byref(params), ctypes.byref(bo),
                                             reps, _stream(stream)))

    def graph(self, bi, bo, stream):
        return PipelineGraph(self, bi, bo, stream)

    def close(self):
        if self.handle:
            lib().miaug_pipeline_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PipelineGraph:
    """miaug_pipeline_graph: a captured pipeline launch that takes new records at every replay."""

    def __init__(self, pipe, bi, bo, stream):
        self.pipe = pipe
        h = _vp()
        _check(lib().miaug_pipeline_graph_capture(pipe.handle, ctypes.byref(bi), ctypes.byref(bo),
                                                  ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h

    def launch(self, params, stream):
        _check(lib().miaug_pipeline_graph_launch(self.handle, ctypes.byref(params),
                                                 ctypes.c_void_p(stream.cuda_stream)))

    def close(self):
        if self.handle:
            lib().miaug_pipeline_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
