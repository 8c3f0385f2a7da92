"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds none of the augmentation arithmetic: it only draws images,
masks, boxes and weights with the shapes and value structure of the paper's
workloads (natural-looking images for Table I; street-view images with masks
and boxes, Sec. II-A; satellite tiles and non-rigid medical images,
Sec. II-B/II-C).  The paper's datasets are not available, so smooth value
noise stands in for their content.

* smooth noise: v = sum_o 2^-o VN_o / sum_o 2^-o over 4 octaves, VN_o bilinear
  value noise with lattice spacing 64 / 2^o px and lattice values U[0, 1);
  u8 = min(255, floor(256 v)); the float variant returns v.
* blob masks: label = min(K - 1, floor(K * VN)) with one octave of spacing
  `spacing` px.
* boxes: count ~ U{0..max}; x1 ~ U[0, W-1), width ~ U[1, W - x1], same for y.

Lattices come from a CPU torch.Generator seeded per call, so the values are
identical on every machine; interpolation runs on `device` (CPU or GPU).
"""
from __future__ import annotations

import math

import numpy as np
import torch
import torch.nn.functional as F


def _value_noise(gen, n, C, H, W, spacing, device):
    lh, lw = math.ceil(H / spacing) + 1, math.ceil(W / spacing) + 1
    lat = torch.rand((n, C, lh, lw), generator=gen, dtype=torch.float32).to(device)
    up = F.interpolate(lat, size=((lh - 1) * spacing + 1, (lw - 1) * spacing + 1), mode="bilinear",
                       align_corners=True)
    return up[:, :, :H, :W]


def smooth_noise(seed: int, n: int, H: int, W: int, C: int = 3, device="cpu", octaves: int = 4):
    """Float smooth noise in [0, 1), shape [n, C, H, W]."""
    gen = torch.Generator().manual_seed(int(seed))
    acc = torch.zeros((n, C, H, W), dtype=torch.float32, device=device)
    tot = 0.0
    for o in range(octaves):
        wgt = 2.0 ** -o
        acc += wgt * _value_noise(gen, n, C, H, W, max(1, 64 >> o), device)
        tot += wgt
    return (acc / tot).clamp_(0.0, 0.99999994)


def smooth_u8_hwc(seed: int, n: int, H: int, W: int, C: int = 3, device="cpu"):
    """u8 smooth-noise images, shape [n, H, W, C] (HWC, dense rows)."""
    v = smooth_noise(seed, n, H, W, C, device)
    return torch.clamp(torch.floor(v * 256.0), max=255).to(torch.uint8).permute(0, 2, 3, 1).contiguous()


def blob_masks(seed: int, n: int, H: int, W: int, K: int, spacing: int, device="cpu"):
    gen = torch.Generator().manual_seed(int(seed))
    vn = _value_noise(gen, n, 1, H, W, spacing, device)[:, 0]
    return torch.clamp(torch.floor(vn * K), max=K - 1).to(torch.uint8).contiguous()


def uniform_u8(seed: int, n: int, H: int, W: int, C: int = 3):
    gen = torch.Generator().manual_seed(int(seed))
    return torch.randint(0, 256, (n, H, W, C), generator=gen, dtype=torch.uint8)


def random_boxes(seed: int, H: int, W: int, max_boxes: int = 16):
    rng = np.random.default_rng(seed)
    nb = int(rng.integers(0, max_boxes + 1))
    out = np.zeros((nb, 4), np.float32)
    for i in range(nb):
        x1 = rng.uniform(0, W - 1); w = rng.uniform(1, W - x1)
        y1 = rng.uniform(0, H - 1); h = rng.uniform(1, H - y1)
        out[i] = (x1, y1, x1 + w, y1 + h)
    return out


class RaggedBatch:
    """Packed ragged batch: images HWC u8 and HW u8 masks, each image starting
    at a 256-byte aligned offset; boxes in CSR form (box_off has n + 1 entries)."""

    def __init__(self, hw, img, img_off, mask, mask_off, boxes, box_off):
        self.hw, self.img, self.img_off = hw, img, img_off
        self.mask, self.mask_off, self.boxes, self.box_off = mask, mask_off, boxes, box_off

    @property
    def n(self):
        return len(self.hw)

    def image(self, i):
        H, W = (int(v) for v in self.hw[i])
        o = int(self.img_off[i])
        return self.img[o:o + H * W * 3].reshape(H, W, 3)

    def mask_of(self, i):
        H, W = (int(v) for v in self.hw[i])
        o = int(self.mask_off[i])
        return self.mask[o:o + H * W].reshape(H, W)

    def boxes_of(self, i):
        return self.boxes[int(self.box_off[i]):int(self.box_off[i + 1])]


def ragged_batch(seed: int, n: int, lo: int = 128, hi: int = 1024, K: int = 21, mask_spacing: int = 128,
                 max_boxes: int = 16, device="cpu", sizes=None, canvases: int = 16, phases=None) -> RaggedBatch:
    """n RGB images with H, W ~ U{lo..hi}, blob masks with K labels, 0..max_boxes boxes.

    Content: `canvases` smooth-noise canvases (and blob-mask canvases) of the
    largest size are drawn once; image i is the H x W window of canvas i mod
    `canvases` at a random offset, so every image is smooth noise with the same
    statistics while generation costs a few kernel launches.  Image and mask
    starts are 256-byte aligned, or, with `phases` (a list of byte offsets),
    image i and its mask start phases[i % len(phases)] bytes after a 256-byte
    boundary.  Returns host-side (numpy) buffers."""
    rng = np.random.default_rng(seed)
    hw = np.asarray(sizes, np.int32) if sizes is not None else rng.integers(lo, hi + 1, size=(n, 2)).astype(np.int32)
    CH, CW = int(hw[:, 0].max()), int(hw[:, 1].max())
    nc = min(canvases, n)
    canvas = smooth_u8_hwc(seed * 7919 + 1, nc, CH, CW, 3, device).cpu().numpy()
    mcanvas = blob_masks(seed * 7919 + 2, nc, CH, CW, K, mask_spacing, device).cpu().numpy()
    align = 256
    img_off = np.zeros(n, np.int64); mask_off = np.zeros(n, np.int64)
    io = mo = 0
    for i, (H, W) in enumerate(hw):
        ph = int(phases[i % len(phases)]) if phases else 0
        img_off[i] = io + ph; mask_off[i] = mo + ph
        io += -(-(int(H) * int(W) * 3 + ph) // align) * align
        mo += -(-(int(H) * int(W) + ph) // align) * align
    img = np.zeros(io, np.uint8); mask = np.zeros(mo, np.uint8)
    boxes, box_off = [], [0]
    for i, (H, W) in enumerate(hw):
        H, W = int(H), int(W)
        oy, ox = int(rng.integers(0, CH - H + 1)), int(rng.integers(0, CW - W + 1))
        c = i % nc
        img[img_off[i]:img_off[i] + H * W * 3] = canvas[c, oy:oy + H, ox:ox + W].reshape(-1)
        mask[mask_off[i]:mask_off[i] + H * W] = mcanvas[c, oy:oy + H, ox:ox + W].reshape(-1)
        b = random_boxes(seed * 7919 + i, H, W, max_boxes)
        boxes.append(b); box_off.append(box_off[-1] + len(b))
    boxes = np.concatenate(boxes) if boxes else np.zeros((0, 4), np.float32)
    return RaggedBatch(hw, img, img_off, mask, mask_off, boxes.astype(np.float32), np.asarray(box_off, np.int32))
