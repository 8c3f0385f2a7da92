"""The oracle's composed pipelines equal the step-by-step composition of its
pinned single ops (Sec. II: transforms are combined; each op rounds to u8
before the next one)."""
import numpy as np

import oracle


def test_d4bc_pipeline_is_d4_then_lut():
    rng = np.random.default_rng(50)
    imgs = rng.integers(0, 256, (6, 8, 8, 3), dtype=np.uint8)
    flags, ab = oracle.sample_d4bc(99, 0, 6)
    out = oracle.pipe_d4bc(imgs, flags, ab)
    for i in range(6):
        ref = oracle.apply_lut(oracle.d4(imgs[i], *flags[i]), oracle.bc_lut(*ab[i]))
        assert np.array_equal(out[i], ref)


def test_c2_pipeline_is_the_op_sequence():
    rng = np.random.default_rng(51)
    img = rng.integers(0, 256, (40, 40, 3), dtype=np.uint8)
    f, k = oracle.sample_c2(7, 0, 4, crop_range=8)
    for i in range(4):
        out = oracle.pipe_c2_one(img, f[i], k[i], crop_=32, outsz=16)
        aq = oracle.ssr_matrix_q32(*f[i][:4], 40, 40)
        t = oracle.warp_affine(img, aq)
        t = oracle.crop(t, k[i][0], k[i][1], 32, 32)
        t = oracle.resize(t, 16, 16)
        t = oracle.hsv_shift(t, k[i][2], k[i][3])
        t = oracle.apply_lut(t, oracle.gamma_lut(f[i][4]))
        if k[i][4]:
            t = oracle.blur(t, 3)
        assert np.array_equal(out, t)


def test_ragged_pipeline_is_the_op_sequence():
    rng = np.random.default_rng(52)
    img = rng.integers(0, 256, (37, 53, 3), dtype=np.uint8)
    mask = rng.integers(0, 21, (37, 53), dtype=np.uint8)
    boxes = np.array([[1.5, 2.0, 30.0, 20.25], [0, 0, 53, 37]], np.float32)
    flags, ab = oracle.sample_d4bc(3, 0, 8)
    for i in range(8):
        out, om, ob = oracle.pipe_ragged_one(img, mask, flags[i], ab[i], boxes, 24, 20)
        t = oracle.apply_lut(oracle.d4(img, *flags[i]), oracle.bc_lut(*ab[i]))
        t = oracle.resize(t, 24, 20)
        assert np.array_equal(out, oracle.normalize_chw(t))
        m = oracle.resize(oracle.d4(mask, *flags[i]), 24, 20, oracle.NEAREST)
        assert np.array_equal(om, m)
        h, w = oracle.d4(mask, *flags[i]).shape
        assert np.array_equal(ob, oracle.boxes_d4_resize(boxes, 37, 53, flags[i], 24, 20))


# ---------------------------------------------------------------- random-sized crop
def test_ragged_crop_of_the_whole_image_is_no_crop():
    rng = np.random.default_rng(53)
    img = rng.integers(0, 256, (29, 41, 3), dtype=np.uint8)
    mask = rng.integers(0, 21, (29, 41), dtype=np.uint8)
    boxes = np.array([[1.5, 2.0, 30.0, 20.25], [0, 0, 41, 29]], np.float32)
    flags, ab = oracle.sample_d4bc(5, 0, 8)
    for i in range(8):
        h, w = oracle.d4(mask, *flags[i]).shape
        a = oracle.pipe_ragged_one(img, mask, flags[i], ab[i], boxes, 16, 24)
        b = oracle.pipe_ragged_one(img, mask, flags[i], ab[i], boxes, 16, 24, win=(0, 0, h, w))
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_ragged_crop_at_output_size_is_numpy_slicing():
    # a window of exactly the output size makes the resize the identity (Q10 positions land on
    # pixel centres), so the output is the normalised LUT image of the sliced Dih4 image
    rng = np.random.default_rng(54)
    img = rng.integers(0, 256, (40, 31, 3), dtype=np.uint8)
    mask = rng.integers(0, 21, (40, 31), dtype=np.uint8)
    flags, ab = oracle.sample_d4bc(6, 0, 8)
    for i in range(8):
        d, dm = oracle.d4(img, *flags[i]), oracle.d4(mask, *flags[i])
        y0, x0 = (3, 5) if d.shape[0] > d.shape[1] else (5, 3)
        out, om, _ = oracle.pipe_ragged_one(img, mask, flags[i], ab[i], None, 17, 12, win=(y0, x0, 17, 12))
        ref = oracle.bc_lut(*ab[i])[d[y0:y0 + 17, x0:x0 + 12]]
        assert np.array_equal(out, oracle.normalize_chw(ref))
        assert np.array_equal(om, dm[y0:y0 + 17, x0:x0 + 12])


def test_boxes_under_a_crop_are_shifted_clipped_and_scaled():
    boxes = np.array([[12, 14, 30, 20], [0, 0, 5, 5], [35, 8, 60, 40], [45, 45, 50, 50]], np.float32)
    win = (10, 10, 25, 30)  # y0, x0, h, w in a 50 x 60 image, identity Dih4
    out = oracle.boxes_d4_crop_resize(boxes, 50, 60, (0, 0, 0, 0), win, 50, 120)
    sy, sx = 50 / 25, 120 / 30
    ref = np.array([[2 * sx, 4 * sy, 20 * sx, 10 * sy],       # inside: shifted and scaled
                    [0, 0, 0, 0],                             # left of and above the window
                    [25 * sx, 0, 30 * sx, 25 * sy],           # straddles two edges: clipped
                    [30 * sx, 25 * sy, 30 * sx, 25 * sy]],    # below and right: zero area at the corner
                   np.float32)
    assert np.allclose(out, ref, rtol=0, atol=1e-5)


def test_crop_windows_lie_in_the_image_and_respect_the_ranges():
    import math
    for (H, W) in [(128, 1024), (1024, 128), (500, 500), (37, 300)]:
        for i in range(300):
            y0, x0, h, w = (int(v) for v in oracle.sized_crop_window(11, i, 1, H, W))
            assert 0 <= y0 and y0 + h <= H and 0 <= x0 and x0 + w <= W and h >= 1 and w >= 1
            # a window from a successful try has area fraction in [0.08, 1] and aspect in [3/4, 4/3],
            # up to the rounding of w and h; a fallback window is centred with clamped aspect
            frac, ar = h * w / (H * W), w / h
            fits = (0.08 * (1 - 2 / min(h, w)) - 1e-12 <= frac <= 1 + 1e-12
                    and 0.75 * (1 - 1 / min(h, w)) <= ar <= 4 / 3 * (1 + 1 / min(h, w)))
            centred = y0 == (H - h) // 2 and x0 == (W - w) // 2
            assert fits or centred


def test_crop_window_statistics_follow_the_ranges():
    # scale U[0.3, 0.7], log-ratio U[log 0.9, log 1.1] on a large square image: every try fits
    n = 3000
    win = np.array([oracle.sized_crop_window(12, i, 1, 1000, 1000, (0.3, 0.7), (0.9, 1.1)) for i in range(n)])
    frac = win[:, 2] * win[:, 3] / 1e6
    lr = np.log(win[:, 3] / win[:, 2])
    assert abs(frac.mean() - 0.5) < 4 * 0.4 / np.sqrt(12 * n)
    assert abs(lr.mean()) < 4 * (2 * np.log(1.1)) / np.sqrt(12 * n) + 1e-3
    assert frac.min() > 0.299 and frac.max() < 0.701
    # offsets are uniform over the free range: their mean is half of it
    assert abs((win[:, 0] / (1000 - win[:, 2])).mean() - 0.5) < 0.03


def test_crop_window_fallbacks_closed_form():
    # aspect range far above a square image's: no try fits, centred window of width W, height W / lo_r
    assert tuple(oracle.sized_crop_window(1, 0, 1, 1000, 1000, (0.5, 1.0), (5.0, 6.0))) == (400, 0, 200, 1000)
    # far below: height H, width H hi_r
    assert tuple(oracle.sized_crop_window(1, 0, 1, 1000, 1000, (0.5, 1.0), (0.1, 0.2))) == (0, 400, 1000, 200)
    # ratio 1 on a non-square image at full area never fits: a centred square of the short side
    assert tuple(oracle.sized_crop_window(1, 0, 1, 100, 160, (1.0, 1.0), (1.0, 1.0))) == (0, 30, 100, 100)
    # the whole image when scale and ratio are both exactly 1 on a square image
    assert tuple(oracle.sized_crop_window(1, 0, 1, 64, 64, (1.0, 1.0), (1.0, 1.0))) == (0, 0, 64, 64)
