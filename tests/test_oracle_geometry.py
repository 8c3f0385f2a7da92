"""Pins of the oracle's geometric ops: Dih4, resize, affine warp, crop, boxes.

References used: numpy flips/rot90/transpose, exact rational arithmetic for
bilinear weights and rounding, scipy.ndimage.affine_transform and torch's
bilinear interpolation as independent float references (to +-1), and group
identities (Sec. II-B, the dihedral group Dih4).
"""
from fractions import Fraction
import itertools

import numpy as np
import pytest

import oracle
from tests.test_oracle_primitives import round_half_even


def rand_img(rng, H, W, C=3):
    return rng.integers(0, 256, size=(H, W, C) if C else (H, W), dtype=np.uint8)


# ------------------------------------------------------------------ Dih4
@pytest.mark.parametrize("shape", [(4, 4), (3, 5), (1, 7), (6, 1), (17, 9)])
def test_single_d4_ops_match_numpy(shape):
    rng = np.random.default_rng(0)
    img = rand_img(rng, *shape)
    assert np.array_equal(oracle.hflip(img), img[:, ::-1])
    assert np.array_equal(oracle.vflip(img), img[::-1])
    assert np.array_equal(oracle.rot90(img), np.rot90(img, 1, axes=(0, 1)))
    assert np.array_equal(oracle.transpose(img), img.transpose(1, 0, 2))


def test_d4_compositions_match_numpy_for_all_32_draws():
    rng = np.random.default_rng(1)
    img = rand_img(rng, 5, 7)
    seen = set()
    for hf, vf, k, tr in itertools.product((0, 1), (0, 1), range(4), (0, 1)):
        ref = img
        if hf: ref = ref[:, ::-1]
        if vf: ref = ref[::-1]
        ref = np.rot90(ref, k, axes=(0, 1))
        if tr: ref = ref.transpose(1, 0, 2)
        out = oracle.d4(img, hf, vf, k, tr)
        assert np.array_equal(out, ref)
        seen.add(out.tobytes() + bytes(out.shape))
    assert len(seen) == 8  # the 32 draws cover exactly the 8 elements of Dih4


def test_d4_group_relations():
    rng = np.random.default_rng(2)
    img = rand_img(rng, 6, 6)
    x = img
    for _ in range(4):
        x = oracle.rot90(x)
    assert np.array_equal(x, img)
    assert np.array_equal(oracle.hflip(oracle.hflip(img)), img)
    assert np.array_equal(oracle.vflip(oracle.vflip(img)), img)
    assert np.array_equal(oracle.transpose(oracle.transpose(img)), img)
    assert np.array_equal(oracle.transpose(img), oracle.vflip(oracle.rot90(img)))


# ------------------------------------------------------------------ resize
def exact_resize_q(j, Ws, Wd):
    # continuous half-pixel-centre map (j + 1/2) Ws / Wd - 1/2, in Q10, ties to even
    return round_half_even((Fraction(2 * j + 1, 2) * Ws / Wd - Fraction(1, 2)) * 1024)


def exact_bilinear(img, H, W, qx, qy, c, border):
    x0, ax = qx >> 10, qx & 1023
    y0, ay = qy >> 10, qy & 1023
    acc = Fraction(0)
    for j, wy in ((0, Fraction(1024 - ay, 1024)), (1, Fraction(ay, 1024))):
        for i, wx in ((0, Fraction(1024 - ax, 1024)), (1, Fraction(ax, 1024))):
            yy, xx = border(y0 + j, H), border(x0 + i, W)
            acc += wy * wx * (0 if yy is None or xx is None else int(img[yy, xx, c]))
    return max(0, min(255, round_half_even(acc)))


def replicate(i, n):
    return min(max(i, 0), n - 1)


@pytest.mark.parametrize("src,dst", [((4, 4), (3, 3)), ((4, 4), (2, 2)), ((3, 5), (7, 2)), ((5, 3), (5, 3)),
                                     ((1, 6), (4, 3)), ((9, 13), (4, 6))])
def test_resize_bilinear_brute_force_exact(src, dst):
    rng = np.random.default_rng(3)
    img = rand_img(rng, *src)
    out = oracle.resize(img, *dst)
    for y in range(dst[0]):
        for x in range(dst[1]):
            qy, qx = exact_resize_q(y, src[0], dst[0]), exact_resize_q(x, src[1], dst[1])
            assert oracle.resize_q(x, src[1], dst[1]) == qx
            for c in range(3):
                assert out[y, x, c] == exact_bilinear(img, src[0], src[1], qx, qy, c, replicate)


def test_resize_identity_and_two_to_one_closed_form():
    rng = np.random.default_rng(4)
    img = rand_img(rng, 10, 14)
    assert np.array_equal(oracle.resize(img, 10, 14), img)
    half = oracle.resize(img, 5, 7)
    s = img.reshape(5, 2, 7, 2, 3).astype(np.int64).sum(axis=(1, 3))
    ref = np.vectorize(lambda v: oracle.rdiv_he(int(v), 4))(s)
    assert np.array_equal(half, ref)


def test_resize_one_to_two_uses_quarter_weights():
    img = np.array([[[0], [100]]], dtype=np.uint8)  # 1 x 2
    out = oracle.resize(img[..., 0], 1, 4)
    # positions -1/4, 1/4, 3/4, 5/4 -> replicate, (3/4,1/4), (1/4,3/4), replicate
    assert out.tolist() == [[0, 25, 75, 100]]


def test_resize_bilinear_agrees_with_torch_to_one_level():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    for (H, W), (h, w) in [((37, 53), (224, 224)), ((300, 611), (224, 224)), ((128, 1024), (224, 224))]:
        img = rand_img(rng, H, W)
        out = oracle.resize(img, h, w).astype(np.int32)
        t = torch.from_numpy(img).permute(2, 0, 1)[None].double()
        ref = torch.nn.functional.interpolate(t, size=(h, w), mode="bilinear", align_corners=False,
                                              antialias=False)[0].permute(1, 2, 0).numpy()
        # final rounding (1/2) + Q10 position quantisation (<= 2^-11 px per axis, times a
        # neighbour difference of at most 255, on two axes)
        assert np.abs(out - ref).max() <= 0.5 + 2 * 255 / 2048 + 1e-9


@pytest.mark.parametrize("Ws,Wd", [(128, 224), (224, 224), (300, 224), (1024, 224), (577, 224), (5, 3), (3, 8)])
def test_resize_nearest_is_floor_of_scaled_centre(Ws, Wd):
    rng = np.random.default_rng(6)
    row = rng.integers(0, 256, size=(1, Ws), dtype=np.uint8)
    out = oracle.resize(row, 1, Wd, oracle.NEAREST)
    idx = np.minimum(((2 * np.arange(Wd) + 1) * Ws) // (2 * Wd), Ws - 1)
    assert np.array_equal(out[0], row[0, idx])


def test_resize_nearest_mask_labels_are_a_subset():
    rng = np.random.default_rng(7)
    m = rng.integers(0, 21, size=(333, 517), dtype=np.uint8)
    out = oracle.resize(m, 224, 224, oracle.NEAREST)
    assert set(np.unique(out)) <= set(np.unique(m))


# ------------------------------------------------------------------ affine warp
def test_ssr_identity_is_identity():
    rng = np.random.default_rng(8)
    img = rand_img(rng, 12, 9)
    aq = oracle.ssr_matrix_q32(0.0, 1.0, 0.0, 0.0, 12, 9)
    assert aq.tolist() == [2**32, 0, 0, 0, 2**32, 0]
    assert np.array_equal(oracle.warp_affine(img, aq), img)


def test_ssr_integer_shift_is_an_exact_shift_with_border_fill():
    rng = np.random.default_rng(9)
    img = rand_img(rng, 16, 16)
    # dx * W = 4 px: p' = p + 4, so out[y][x] = in[y][x - 4]
    aq = oracle.ssr_matrix_q32(0.0, 1.0, 4.0 / 16, 0.0, 16, 16)
    out = oracle.warp_affine(img, aq, border=oracle.CONSTANT)
    assert np.array_equal(out[:, 4:], img[:, :-4])
    assert not out[:, :4].any()
    out_r = oracle.warp_affine(img, aq, border=oracle.REFLECT101)
    assert np.array_equal(out_r[:, :4], img[:, 4:0:-1])


def test_ssr_quarter_and_half_turns_are_exact_dih4_elements():
    rng = np.random.default_rng(10)
    img = rand_img(rng, 11, 11)
    a90 = oracle.ssr_matrix_q32(90.0, 1.0, 0.0, 0.0, 11, 11)
    assert np.array_equal(oracle.warp_affine(img, a90), np.rot90(img, 1, axes=(0, 1)))
    a180 = oracle.ssr_matrix_q32(180.0, 1.0, 0.0, 0.0, 11, 11)
    assert np.array_equal(oracle.warp_affine(img, a180), img[::-1, ::-1])
    img2 = rand_img(rng, 6, 10)
    a180b = oracle.ssr_matrix_q32(180.0, 1.0, 0.0, 0.0, 6, 10)
    assert np.array_equal(oracle.warp_affine(img2, a180b), img2[::-1, ::-1])


def test_ssr_scale_two_closed_form():
    # s = 2 about the centre of an odd image: out[y][x] samples in at c + (p - c)/2.
    img = np.arange(81, dtype=np.uint8).reshape(9, 9) * 3
    aq = oracle.ssr_matrix_q32(0.0, 2.0, 0.0, 0.0, 9, 9)
    out = oracle.warp_affine(img, aq)
    for y in range(9):
        for x in range(9):
            sy, sx = Fraction(4) + Fraction(y - 4, 2), Fraction(4) + Fraction(x - 4, 2)
            y0, x0 = int(sy), int(sx)
            fy, fx = sy - y0, sx - x0
            v = (1 - fy) * ((1 - fx) * int(img[y0, x0]) + fx * int(img[y0, min(x0 + 1, 8)])) + \
                fy * ((1 - fx) * int(img[min(y0 + 1, 8), x0]) + fx * int(img[min(y0 + 1, 8), min(x0 + 1, 8)]))
            assert out[y, x] == round_half_even(v)


def test_warp_brute_force_exact_with_both_borders():
    rng = np.random.default_rng(11)
    img = rand_img(rng, 4, 5)
    for angle, scale, dx, dy in [(17.0, 1.05, 0.03, -0.02), (-44.0, 0.91, -0.06, 0.06), (90.5, 1.0, 0.0, 0.0)]:
        aq = [int(v) for v in oracle.ssr_matrix_q32(angle, scale, dx, dy, 4, 5)]
        for border, bfun in ((oracle.REFLECT101, lambda i, n: oracle.reflect101(i, n)),
                             (oracle.CONSTANT, lambda i, n: i if 0 <= i < n else None)):
            out = oracle.warp_affine(img, np.array(aq, np.int64), border=border)
            for y in range(4):
                for x in range(5):
                    qx = round_half_even(Fraction(aq[0] * x + aq[1] * y + aq[2], 2**22))
                    qy = round_half_even(Fraction(aq[3] * x + aq[4] * y + aq[5], 2**22))
                    for c in range(3):
                        assert out[y, x, c] == exact_bilinear(img, 4, 5, qx, qy, c, bfun)


def test_ssr_matrix_matches_the_inverse_of_the_forward_map():
    H, W = 512, 512
    a = oracle.ssr_inverse(30.0, 1.1, 0.05, -0.03, H, W)
    t = np.deg2rad(30.0)
    R = np.array([[np.cos(t), np.sin(t)], [-np.sin(t), np.cos(t)]])
    c = np.array([(W - 1) / 2, (H - 1) / 2])
    rng = np.random.default_rng(12)
    for _ in range(20):
        p = rng.uniform(0, 512, 2)
        fwd = 1.1 * R @ (p - c) + c + np.array([0.05 * W, -0.03 * H])
        back = np.array([a[0] * fwd[0] + a[1] * fwd[1] + a[2], a[3] * fwd[0] + a[4] * fwd[1] + a[5]])
        assert np.allclose(back, p, atol=1e-9)


def test_warp_agrees_with_scipy_affine_transform_to_one_level():
    ndimage = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(13)
    yy, xx = np.mgrid[0:64, 0:80]
    img = (127 + 100 * np.sin(xx / 7.0) * np.cos(yy / 5.0)).astype(np.uint8)
    for angle, scale, dx, dy in [(23.0, 0.95, 0.02, 0.01), (-40.0, 1.08, -0.05, 0.04)]:
        aq = oracle.ssr_matrix_q32(angle, scale, dx, dy, 64, 80)
        out = oracle.warp_affine(img, aq).astype(np.float64)
        a = oracle.ssr_inverse(angle, scale, dx, dy, 64, 80)
        # scipy uses (row, col) order: [sy, sx] = M [y, x] + off
        M = np.array([[a[4], a[3]], [a[1], a[0]]])
        ref = ndimage.affine_transform(img.astype(np.float64), M, offset=[a[5], a[2]], order=1, mode="mirror")
        assert np.abs(out - ref).max() <= 1.0


def test_crop_is_numpy_slicing():
    rng = np.random.default_rng(14)
    img = rand_img(rng, 30, 40)
    assert np.array_equal(oracle.crop(img, 7, 3, 20, 25), img[3:23, 7:32])


# ------------------------------------------------------------------ boxes
def rasterize(box, H, W):
    m = np.zeros((H, W), np.uint8)
    x1, y1, x2, y2 = [int(v) for v in box]
    m[y1:y2, x1:x2] = 1
    return m


def bbox_of(m):
    ys, xs = np.nonzero(m)
    return [xs.min(), ys.min(), xs.max() + 1, ys.max() + 1]


def test_boxes_follow_d4_exactly_like_their_masks():
    rng = np.random.default_rng(15)
    H, W = 23, 31
    for hf, vf, k, tr in itertools.product((0, 1), (0, 1), range(4), (0, 1)):
        x1, y1 = int(rng.integers(0, W - 2)), int(rng.integers(0, H - 2))
        box = [x1, y1, int(rng.integers(x1 + 1, W + 1)), int(rng.integers(y1 + 1, H + 1))]
        m = oracle.d4(rasterize(box, H, W), hf, vf, k, tr)
        Ho, Wo = m.shape
        out = oracle.boxes_d4_resize(np.array([box], np.float32), H, W, (hf, vf, k, tr), Ho, Wo)
        assert out[0].tolist() == [float(v) for v in bbox_of(m)]


def test_boxes_follow_resize_within_one_pixel_of_the_mask():
    rng = np.random.default_rng(16)
    for H, W in [(300, 500), (1000, 200), (150, 150)]:
        x1, y1 = int(rng.integers(0, W // 2)), int(rng.integers(0, H // 2))
        box = [x1, y1, x1 + W // 3, y1 + H // 3]
        flags = (1, 0, 1, 1)
        m = oracle.d4(rasterize(box, H, W), *flags)
        mr = oracle.resize(m, 224, 224, oracle.NEAREST)
        out = oracle.boxes_d4_resize(np.array([box], np.float32), H, W, flags, 224, 224)
        assert np.abs(np.array(bbox_of(mr)) - out[0]).max() <= 1.0


# ---------------------------------------------------------------- boxes under shift-scale-rotate
def test_ssr_boxes_quarter_turns_match_the_dih4_element_of_the_image():
    # the warp by 90 / 180 degrees of a square image is rot90 / a half turn (pinned above);
    # its boxes must be the Dih4 element's boxes exactly
    rng = np.random.default_rng(17)
    n = 11
    for _ in range(20):
        x1, y1 = int(rng.integers(0, n - 1)), int(rng.integers(0, n - 1))
        box = np.array([[x1, y1, int(rng.integers(x1 + 1, n + 1)), int(rng.integers(y1 + 1, n + 1))]], np.float32)
        b90 = oracle.boxes_ssr_crop_resize(box, n, n, (90.0, 1.0, 0.0, 0.0), 0, 0, n, n)
        m90 = oracle.warp_affine(rasterize(box[0].astype(int).tolist(), n, n), oracle.ssr_matrix_q32(90.0, 1, 0, 0, n, n),
                                 oracle.NEAREST)
        assert np.allclose(b90[0], bbox_of(m90), atol=1e-9)
        b180 = oracle.boxes_ssr_crop_resize(box, n, n, (180.0, 1.0, 0.0, 0.0), 0, 0, n, n)
        ref = oracle.boxes_d4_resize(box, n, n, (1, 1, 0, 0), n, n)
        assert np.allclose(b180, ref, atol=1e-9)


def test_ssr_boxes_identity_shift_and_crop_closed_form():
    box = np.array([[10.0, 20.0, 40.0, 30.0]], np.float32)
    # identity warp, crop at (5, 8) of size 50, resize to 100: shift then scale by 2
    out = oracle.boxes_ssr_crop_resize(box, 60, 70, (0.0, 1.0, 0.0, 0.0), 5, 8, 50, 100)
    assert np.allclose(out[0], [10.0, 24.0, 70.0, 44.0])
    # a shift by dx W = +7 pixels (W = 70, dx = 0.1) moves the box right by 7, clipped at the image edge
    out = oracle.boxes_ssr_crop_resize(np.array([[60.0, 1.0, 68.0, 2.0]], np.float32), 60, 70,
                                       (0.0, 1.0, np.float32(0.1), 0.0), 10, 0, 60, 60)
    assert np.allclose(out[0], [57.0, 1.0, 60.0, 2.0], atol=1e-5)  # 67..70 (clipped at W), minus the crop offset
    # scale 2 about the centre c = ((W-1)/2, (H-1)/2) maps continuous u to 2 (u - 1/2 - c) + c + 1/2
    out = oracle.boxes_ssr_crop_resize(np.array([[30.0, 25.0, 35.0, 30.0]], np.float32), 60, 70,
                                       (0.0, 2.0, 0.0, 0.0), 0, 0, 60, 60)
    c = np.array([34.5, 29.5])
    ref = [2 * (30 - 0.5 - c[0]) + c[0] + 0.5, 2 * (25 - 0.5 - c[1]) + c[1] + 0.5,
           2 * (35 - 0.5 - c[0]) + c[0] + 0.5, 2 * (30 - 0.5 - c[1]) + c[1] + 0.5]
    assert np.allclose(out[0], ref, atol=1e-5)


def test_ssr_boxes_contain_the_warped_mask_of_the_box():
    # the bounding box of the four mapped corners contains every pixel the warped box mask covers
    # (up to one pixel for nearest sampling), at arbitrary angles
    rng = np.random.default_rng(18)
    H, W = 64, 80
    for _ in range(12):
        angle, scale = float(rng.uniform(-45, 45)), float(rng.uniform(0.9, 1.1))
        dx, dy = float(rng.uniform(-0.06, 0.06)), float(rng.uniform(-0.06, 0.06))
        f = np.float32([angle, scale, dx, dy])
        x1, y1 = int(rng.integers(16, 40)), int(rng.integers(16, 30))
        box = [x1, y1, x1 + int(rng.integers(4, 20)), y1 + int(rng.integers(4, 18))]
        m = oracle.warp_affine(rasterize(box, H, W), oracle.ssr_matrix_q32(*f, H, W), oracle.NEAREST, oracle.CONSTANT)
        got = oracle.boxes_ssr_crop_resize(np.array([box], np.float32), H, W, f, 0, 0, min(H, W), min(H, W))[0]
        mb = bbox_of(m)
        assert got[0] <= mb[0] + 1 and got[1] <= mb[1] + 1 and got[2] >= mb[2] - 1 and got[3] >= mb[3] - 1
        # and is not much larger: at most the rotation's corner overhang plus a pixel
        assert (got[2] - got[0]) <= (mb[2] - mb[0]) + 2 and (got[3] - got[1]) <= (mb[3] - mb[1]) + 2


# ---------------------------------------------------------------- PadToSize (Table I PadToSize512)
@pytest.mark.parametrize("H,W,Hm,Wm", [(5, 7, 9, 12), (1, 1, 4, 3), (6, 6, 6, 6), (10, 3, 4, 8), (3, 10, 8, 4)])
def test_pad_matches_numpy_reflect_and_constant(H, W, Hm, Wm):
    rng = np.random.default_rng(H * 100 + W)
    img = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
    ho, wo = max(H, Hm), max(W, Wm)
    top, left = (ho - H) // 2, (wo - W) // 2
    pw = ((top, ho - H - top), (left, wo - W - left), (0, 0))
    if H > 1 and W > 1 and max(pw[0]) < H and max(pw[1]) < W:  # numpy's single reflection
        assert np.array_equal(oracle.pad(img, Hm, Wm, oracle.REFLECT101), np.pad(img, pw, mode="reflect"))
    assert np.array_equal(oracle.pad(img, Hm, Wm, oracle.CONSTANT, 17), np.pad(img, pw, constant_values=17))


def test_pad_reflects_repeatedly_for_large_pads():
    img = np.arange(3, dtype=np.uint8).reshape(1, 3)
    out = oracle.pad(img, 1, 11, oracle.REFLECT101)
    # reflect-101 of 0 1 2 has period 4: ... 2 1 0 1 2 1 0 ...
    assert out[0].tolist() == [0, 1, 2, 1, 0, 1, 2, 1, 0, 1, 2]
