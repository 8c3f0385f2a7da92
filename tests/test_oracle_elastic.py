"""Pins of the oracle's elastic transform and grid distortion (Sec. II-C and
Fig. 4; the Simard et al. 2003 elastic distortion cited in Sec. I).

References: scipy.ndimage.correlate1d with mirror borders (= reflect-101) on
exact int64 data, numpy Philox, closed-form shifts and piecewise-linear maps.
"""
import numpy as np
import pytest

import oracle


def test_gauss_taps_are_symmetric_normalised_q15():
    t = oracle.gauss_taps_q15(50.0, 150)
    assert len(t) == 301
    assert np.array_equal(t, t[::-1])
    assert abs(int(t.sum()) - 32768) <= 150  # per-tap rounding, at most 1/2 each
    k = np.arange(-150, 151)
    g = np.exp(-k.astype(np.float64) ** 2 / (2 * 50.0 ** 2))
    assert np.abs(t - 32768 * g / g.sum()).max() <= 0.5 + 1e-9


def test_hpass_equals_scipy_mirror_correlation_then_rshr():
    ndimage = pytest.importorskip("scipy.ndimage")
    H, W, r = 5, 37, 9
    taps = oracle.gauss_taps_q15(3.0, r)
    h = np.zeros((H, W), np.int32)
    oracle.lib().or_elastic_hpass(11, 2, 0, H, W, taps, r, 0, H, h)
    noise = np.array([[oracle.noise16(11, 2, 0, y * W + x) for x in range(W)] for y in range(H)], np.int64)
    ref = ndimage.correlate1d(noise, taps.astype(np.int64), axis=1, mode="mirror")
    ref = np.vectorize(lambda v: oracle.rshr_he(int(v), 15))(ref)
    assert np.array_equal(h, ref)


def test_field_equals_scipy_separable_reference_and_pointwise_definition():
    ndimage = pytest.importorskip("scipy.ndimage")
    H, W, r, sigma, alpha = 23, 29, 7, 2.5, 40
    ox, oy = oracle.elastic_field(3, 1, H, W, sigma, alpha, r)
    taps = oracle.gauss_taps_q15(sigma, r).astype(np.int64)
    for field, off in ((0, ox), (1, oy)):
        noise = np.array([[oracle.noise16(3, 1, field, y * W + x) for x in range(W)] for y in range(H)], np.int64)
        h = ndimage.correlate1d(noise, taps, axis=1, mode="mirror")
        h = np.vectorize(lambda v: oracle.rshr_he(int(v), 15))(h).astype(np.int64)
        v = ndimage.correlate1d(h, taps, axis=0, mode="mirror")
        ref = np.vectorize(lambda t: oracle.rshr_he(alpha * int(t), 20))(v)
        assert np.array_equal(off, ref)
    for (y, x) in [(0, 0), (5, 28), (22, 13)]:
        assert oracle.elastic_field_at(3, 1, H, W, y, x, sigma, alpha, r) == (ox[y, x], oy[y, x])


def test_field_statistics_at_the_large_tile_setting():
    # sigma = 50, alpha = 1000: displacement std ~ alpha * std(U[-1,1]) / (2 sqrt(pi) sigma) ~ 3.3 px
    H = W = 256
    ox, oy = oracle.elastic_field(1809068395, 0, H, W, 50.0, 1000, 150)
    sd = np.concatenate([ox.ravel(), oy.ravel()]).std() / 1024
    assert 1.0 < sd < 8.0


def test_zero_alpha_is_identity_and_constant_field_is_a_shift():
    rng = np.random.default_rng(30)
    img = rng.integers(0, 256, (16, 20, 3), dtype=np.uint8)
    ox, oy = oracle.elastic_field(9, 0, 16, 20, 3.0, 0, 5)
    assert not ox.any() and not oy.any()
    assert np.array_equal(oracle.remap_field(img, ox, oy), img)
    sx, sy = 3, -2
    fx = np.full((16, 20), sx * 1024, np.int32)
    fy = np.full((16, 20), sy * 1024, np.int32)
    out = oracle.remap_field(img, fx, fy)
    ys = [oracle.reflect101(y + sy, 16) for y in range(16)]
    xs = [oracle.reflect101(x + sx, 20) for x in range(20)]
    assert np.array_equal(out, img[np.ix_(ys, xs)])
    outn = oracle.remap_field(img, fx, fy, oracle.NEAREST)
    assert np.array_equal(outn, img[np.ix_(ys, xs)])


def test_grid_identity_table_and_monotone_and_single_cell_closed_form():
    for n in (7, 100, 4096):
        q = oracle.grid_table(np.ones(5), n)
        assert np.array_equal(q, np.arange(n) * 1024)
    rng = np.random.default_rng(31)
    d = 1 + rng.uniform(-0.3, 0.3, 5)
    q = oracle.grid_table(d, 500)
    assert np.all(np.diff(q) > 0)
    # only cell 2 stretched: inside it, src = S_2 + (u - 2 cw) d_2 - 1/2 with S_2 = 2 cw
    d = np.array([1.0, 1.0, 1.25, 1.0, 1.0])
    q = oracle.grid_table(d, 100)
    for x in range(40, 60):
        u = x + 0.5
        assert q[x] == round((40 + (u - 40) * 1.25 - 0.5) * 1024)
    for x in range(0, 40):
        assert q[x] == x * 1024
    for x in range(60, 100):  # later cells are shifted by the stretch of cell 2 (not renormalised)
        assert q[x] == (x + 5) * 1024


def test_grid_remap_identity_tables_are_identity():
    rng = np.random.default_rng(32)
    img = rng.integers(0, 256, (9, 13, 3), dtype=np.uint8)
    assert np.array_equal(oracle.grid_remap(img, np.arange(13) * 1024, np.arange(9) * 1024), img)


def test_elastic_grid_pipeline_composes_the_two_ops():
    rng = np.random.default_rng(33)
    img = rng.integers(0, 256, (40, 36, 3), dtype=np.uint8)
    mask = rng.integers(0, 8, (40, 36), dtype=np.uint8)
    g = oracle.sample_grid(7, 3, 1)[0]
    out, om = oracle.pipe_elastic_grid_one(img, mask, 7, 3, g, sigma=4.0, alpha=60, radius=12)
    ox, oy = oracle.elastic_field(7, 3, 40, 36, 4.0, 60, 12)
    mx, my = oracle.grid_table(g[:5], 36), oracle.grid_table(g[5:], 40)
    e = oracle.remap_field(img, ox, oy)
    assert np.array_equal(out, oracle.grid_remap(e, mx, my))
    em = oracle.remap_field(mask, ox, oy, oracle.NEAREST)
    assert np.array_equal(om, oracle.grid_remap(em, mx, my, oracle.NEAREST))
    assert set(np.unique(om)) <= set(np.unique(mask))


# ---------------------------------------------------------------- box-cascade field (opt-in approximation)
def _cascade_variance(widths):
    return sum((w * w - 1) / 12.0 for w in widths)


@pytest.mark.parametrize("sigma", [0.8, 1.0, 2.5, 6.0, 20.0, 50.0, 77.7])
def test_box_widths_are_odd_and_give_the_closest_cascade_variance(sigma):
    w = oracle.box_widths(sigma)
    assert all(v % 2 == 1 for v in w) and w[0] <= w[1] <= w[2] and w[2] - w[0] in (0, 2)
    wl = w[0] if w[2] != w[0] else None
    # among cascades of three odd widths from {wl, wl + 2} (any split), the chosen one is nearest to sigma^2
    base = w[0] if w[0] == w[2] else wl
    cands = [[base] * k + [base + 2] * (3 - k) for k in range(4)] + [[base - 2] * k + [base] * (3 - k) for k in range(4)]
    cands = [c for c in cands if min(c) >= 1]
    best = min(abs(_cascade_variance(c) - sigma ** 2) for c in cands)
    assert abs(_cascade_variance(w) - sigma ** 2) <= best + 1e-9


def test_box_pass_equals_scipy_mirror_sum_then_rounded_division():
    ndimage = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(5)
    for n, r in [(37, 4), (9, 6), (1, 3), (200, 50), (3, 1)]:
        line = rng.integers(-32768, 32768, n).astype(np.int64)
        s = ndimage.correlate1d(line, np.ones(2 * r + 1, np.int64), mode="mirror")
        ref = np.array([oracle.rdiv_he(int(v), 2 * r + 1) for v in s], np.int32)
        assert np.array_equal(oracle.box_pass(line.astype(np.int32), r), ref), (n, r)


def test_box_field_is_the_row_then_column_cascade():
    ndimage = pytest.importorskip("scipy.ndimage")
    H, W, sigma, alpha = 19, 23, 2.0, 300
    radii = [w // 2 for w in oracle.box_widths(sigma)]
    ox, oy = oracle.elastic_field_box(9, 4, H, W, sigma, alpha)

    def cascade(a, axis):
        for r in radii:
            s = ndimage.correlate1d(a, np.ones(2 * r + 1, np.int64), axis=axis, mode="mirror")
            a = np.vectorize(lambda v, r=r: oracle.rdiv_he(int(v), 2 * r + 1))(s).astype(np.int64)
        return a

    for field, off in ((0, ox), (1, oy)):
        noise = np.array([[oracle.noise16(9, 4, field, y * W + x) for x in range(W)] for y in range(H)], np.int64)
        v = cascade(cascade(noise, 1), 0)
        ref = np.vectorize(lambda t: oracle.rshr_he(alpha * int(t), 5))(v)
        assert np.array_equal(off, ref), field


def test_box_field_tracks_the_gaussian_field_and_zero_alpha_is_zero():
    H, W, sigma, alpha = 64, 80, 6.0, 300
    ex, ey = oracle.elastic_field(1, 0, H, W, sigma, alpha, 18)
    bx, by = oracle.elastic_field_box(1, 0, H, W, sigma, alpha)
    for e, b in ((ex, bx), (ey, by)):
        assert np.corrcoef(e.ravel(), b.ravel())[0, 1] > 0.99
        assert 0.9 < b.std() / e.std() < 1.1
    zx, zy = oracle.elastic_field_box(1, 0, H, W, sigma, 0)
    assert not zx.any() and not zy.any()


# ---------------------------------------------------------------- boxes under the distortion
def _ident_tables(H, W):
    return (np.arange(W, dtype=np.int32) * 1024, np.arange(H, dtype=np.int32) * 1024)


def test_distort_boxes_identity_and_integer_shift():
    H, W = 40, 56
    z = np.zeros((H, W), np.int32)
    mx, my = _ident_tables(H, W)
    boxes = np.array([[10, 5, 30, 20], [10.2, 5.7, 29.5, 20.5], [0, 0, 56, 40]], np.float32)
    out = oracle.boxes_distort(boxes, H, W, z, z, mx, my)
    # pixels whose centres lie in [x1, x2): 10.2 -> first centre 10.5, 29.5 -> last centre 28.5
    assert out.tolist() == [[10, 5, 30, 20], [10, 6, 29, 20], [0, 0, 56, 40]]
    # every output pixel samples the source 5 px to the right and 3 px down: the box moves left and up
    out = oracle.boxes_distort(boxes[:1], H, W, z + 5 * 1024, z + 3 * 1024, mx, my)
    assert out.tolist() == [[5, 2, 25, 17]]


def test_distort_boxes_follow_separable_grid_tables():
    H, W = 48, 64
    rng = np.random.default_rng(21)
    d = 1 + rng.uniform(-0.3, 0.3, 10)
    mx, my = oracle.grid_table(d[:5], W), oracle.grid_table(d[5:], H)
    z = np.zeros((H, W), np.int32)
    box = np.array([[13.0, 9.0, 41.0, 30.0]], np.float32)
    out = oracle.boxes_distort(box, H, W, z, z, mx, my)[0]
    # brute force on the tables: output column x reaches source column reflect((mapx[x] + 512) >> 10)
    def src(q, n):
        i = (q.astype(np.int64) + 512) >> 10
        p = 2 * n - 2
        i = np.mod(i, p)
        return np.where(i >= n, p - i, i)
    sx, sy = src(mx, W), src(my, H)
    xs = np.nonzero((sx + 0.5 >= 13) & (sx + 0.5 < 41))[0]
    ys = np.nonzero((sy + 0.5 >= 9) & (sy + 0.5 < 30))[0]
    assert out.tolist() == [xs.min(), ys.min(), xs.max() + 1, ys.max() + 1]


def test_distort_boxes_match_the_transformed_mask_of_a_blob():
    # a box drawn around a blob of labels stays around the blob after the distortion
    H, W = 64, 80
    ox, oy = oracle.elastic_field(3, 0, H, W, sigma=6.0, alpha=300, radius=18)
    d = 1 + np.random.default_rng(22).uniform(-0.3, 0.3, 10)
    mx, my = oracle.grid_table(d[:5], W), oracle.grid_table(d[5:], H)
    m = np.zeros((H, W), np.uint8); m[20:35, 30:50] = 1
    out = oracle.boxes_distort(np.array([[30, 20, 50, 35]], np.float32), H, W, ox, oy, mx, my)[0]
    g = oracle.grid_remap(oracle.remap_field(m, ox, oy, oracle.NEAREST), mx, my, oracle.NEAREST)
    ys, xs = np.nonzero(g)
    assert out.tolist() == [xs.min(), ys.min(), xs.max() + 1, ys.max() + 1]
