"""Pins of the oracle's fp64 differentiable paths: the warp + colour op and
the float copy of the elastic + grid chain.

References: central finite differences in fp64 (h = 1e-4) on the oracle's
own forward (an independent check of the hand-derived adjoint), the
dot-product (adjoint) identity <A x, y> = <x, A^T y>, and identity cases.
"""
import numpy as np
import pytest

import oracle


def smooth_image(rng, C, H, W):
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    out = np.zeros((C, H, W))
    for c in range(C):
        a, b, p = rng.uniform(0.05, 0.3, 3)
        out[c] = 0.5 + 0.4 * np.sin(a * xx + p) * np.cos(b * yy - p)
    return out.astype(np.float32)


def test_wc_identity_parameters_give_the_image():
    rng = np.random.default_rng(40)
    x = smooth_image(rng, 3, 12, 10)
    y = oracle.wc_forward(x, [0.0, 1.0, 0.0, 0.0, 1.0, 0.0, 1.0])
    assert np.abs(y - x).max() < 1e-12


def test_wc_image_adjoint_dot_product():
    rng = np.random.default_rng(41)
    C, H, W = 2, 16, 14
    # alpha = 1, beta = 0, gamma = 1 and values in (0, 1): the op is linear in x
    p = np.array([23.0, 1.07, 0.03, -0.05, 1.0, 0.0, 1.0])
    x = rng.uniform(0.1, 0.4, (C, H, W)).astype(np.float32)
    g = rng.uniform(-1, 1, (C, H, W))
    y = oracle.wc_forward(x, p)
    gx, _ = oracle.wc_backward(x, p, g)
    assert abs((y * g).sum() - (x.astype(np.float64) * gx).sum()) < 1e-12 * max(1.0, abs((y * g).sum()))


def _loss(x, p, w):
    return (oracle.wc_forward(x, p) * w).sum()


def _fd(x, p, w, k, h):
    pp, pm = np.array(p, np.float64), np.array(p, np.float64)
    pp[k] += h
    pm[k] -= h
    return (_loss(x, pp, w) - _loss(x, pm, w)) / (2 * h)


def test_wc_colour_gradients_match_central_differences_h1e4_without_kinks():
    # Parameters chosen so that no pixel meets a clamp or the zero border within +-1e-4:
    # z stays inside (0, 1) and every tap stays inside the image.  The loss is then
    # smooth in alpha, beta and gamma, and h = 1e-4 reproduces their gradients to 1e-7.
    # (In the geometric parameters the bilinear sample is only piecewise linear in
    # position: a step of 1e-4 moves sample points across cell edges, so those are
    # checked at h = 1e-6 below.)
    rng = np.random.default_rng(42)
    C, H, W = 3, 40, 36
    x = (0.25 + 0.5 * smooth_image(rng, C, H, W)).astype(np.float32)
    w = rng.uniform(-1, 1, (C, H, W))
    for p in ([3.0, 1.1, 0.005, -0.005, 1.1, 0.05, 0.9], [-2.5, 1.12, -0.004, 0.006, 0.85, -0.02, 1.15]):
        _, gp = oracle.wc_backward(x, p, w, want_gx=False)
        for k in (4, 5, 6):
            fd = _fd(x, p, w, k, 1e-4)
            assert abs(fd - gp[k]) <= 1e-7 * max(1.0, abs(gp[k])), (p, k, fd, gp[k])


def test_wc_parameter_gradients_match_central_differences_at_sampled_parameters():
    # Sampled parameters hit the clamp and the zero border; a step of 1e-4 then crosses
    # kinks on a few percent of pixels (the beta derivative moves by ~8%), so the tight
    # check uses h = 1e-6, where the fp64 difference quotient has converged.
    rng = np.random.default_rng(42)
    C, H, W = 3, 24, 20
    x = smooth_image(rng, C, H, W)
    w = rng.uniform(-1, 1, (C, H, W))
    checked = 0
    for trial in range(6):
        f = oracle.sample_wc(1809068394, trial, 1)[0].astype(np.float64)
        _, gp = oracle.wc_backward(x, f, w, want_gx=False)
        for k in range(7):
            fd = _fd(x, f, w, k, 1e-6)
            assert abs(fd - gp[k]) <= 1e-6 * max(1.0, abs(gp[k])), (trial, k, fd, gp[k])
            checked += 1
    assert checked == 42


def test_wc_image_gradient_matches_central_differences():
    rng = np.random.default_rng(43)
    C, H, W = 1, 14, 12
    x = smooth_image(rng, C, H, W)
    w = rng.uniform(-1, 1, (C, H, W))
    p = np.array([-31.0, 0.93, -0.04, 0.02, 1.1, 0.05, 0.9])
    gx, _ = oracle.wc_backward(x, p, w)
    for (yy, xx) in [(3, 4), (7, 7), (10, 2), (0, 11), (13, 0)]:
        # the oracle takes f32 images, so difference with a step exactly representable
        h = 2.0 ** -10
        xp, xm = x.copy(), x.copy()
        xp[0, yy, xx] += h; xm[0, yy, xx] -= h
        fd = (_loss(xp, p, w) - _loss(xm, p, w)) / (2 * h)
        assert abs(fd - gx[0, yy, xx]) <= 1e-6 + 1e-4 * abs(gx[0, yy, xx]), (yy, xx, fd, gx[0, yy, xx])


def test_chain_f_identity_and_adjoint():
    rng = np.random.default_rng(44)
    C, H, W = 2, 18, 15
    x = rng.uniform(0, 1, (C, H, W)).astype(np.float32)
    z = np.zeros((H, W), np.int32)
    ix, iy = np.arange(W, dtype=np.int32) * 1024, np.arange(H, dtype=np.int32) * 1024
    assert np.abs(oracle.chain_f_forward(x, z, z, ix, iy) - x).max() == 0
    ox, oy = oracle.elastic_field(5, 2, H, W, 2.0, 40, 6)
    g = oracle.sample_grid(5, 2, 1)[0]
    mx, my = oracle.grid_table(g[:5], W), oracle.grid_table(g[5:], H)
    y = oracle.chain_f_forward(x, ox, oy, mx, my)
    gy = rng.uniform(-1, 1, (C, H, W))
    gx = oracle.chain_f_backward(gy, ox, oy, mx, my)
    assert abs((y * gy).sum() - (x.astype(np.float64) * gx).sum()) < 1e-10


def test_chain_f_matches_the_u8_chain_before_rounding():
    # On an image whose values are integers, the float chain rounded once after each
    # remap reproduces the u8 chain (the u8 chain rounds after each op).
    rng = np.random.default_rng(45)
    H, W = 20, 22
    img = rng.integers(0, 256, (H, W, 1), dtype=np.uint8)
    ox, oy = oracle.elastic_field(8, 0, H, W, 2.0, 30, 6)
    g = oracle.sample_grid(8, 0, 1)[0]
    mx, my = oracle.grid_table(g[:5], W), oracle.grid_table(g[5:], H)
    e = oracle.remap_field(img, ox, oy)
    ef = oracle.chain_f_forward(img[..., 0][None].astype(np.float32), ox, oy,
                                np.arange(W, dtype=np.int32) * 1024, np.arange(H, dtype=np.int32) * 1024)
    from tests.test_oracle_primitives import round_half_even
    from fractions import Fraction
    r = np.vectorize(lambda v: round_half_even(Fraction(v)))(ef[0])
    assert np.array_equal(r, e[..., 0])
