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
