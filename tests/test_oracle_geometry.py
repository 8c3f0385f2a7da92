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
