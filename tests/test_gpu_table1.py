"""GPU parity of the remaining Table I single ops (ShiftRGB, Grayscale,
PadToSize, Rotate and a standalone shift-scale-rotate warp) against the
oracle, bit-exact, called through the C ABI."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m(dev):
    import paper_1809_06839_amd as m
    m.lib()
    return m


def test_color_luts_compose_brightness_then_shift(m):
    # host compile against the oracle's two LUTs applied one after the other
    rng = np.random.default_rng(1)
    ab = np.stack([rng.uniform(0.8, 1.2, 5), rng.uniform(-51, 51, 5)], 1).astype(np.float32)
    sh = rng.uniform(-20, 20, (5, 3)).astype(np.float32)
    luts = m.compile_color_luts(ab, sh)
    for i in range(5):
        s = oracle.shift_rgb_lut(sh[i])
        b = oracle.bc_lut(*ab[i])
        for c in range(3):
            assert np.array_equal(luts[i, c], s[c][b])


@pytest.mark.parametrize("C", [1, 3, 4])
def test_d4_luts_and_gray_bit_exact(m, C):
    import torch
    rng = np.random.default_rng(C)
    n, H, W = 8, 70, 45
    imgs = rng.integers(0, 256, (n, H, W, C), dtype=np.uint8)
    flags, ab = m.sample_d4bc(C, 0, n)
    sh = rng.uniform(-20, 20, (n, C)).astype(np.float32)
    luts = m.compile_color_luts(ab, sh, C=C)
    gray = (np.arange(n) % 2).astype(np.int32) if C == 3 else None
    out = m.d4_lut_u8(torch.from_numpy(imgs).cuda(), torch.from_numpy(flags).cuda(), torch.from_numpy(luts).cuda(),
                      None if gray is None else torch.from_numpy(gray).cuda())
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(-1)
    size = H * W * C
    for i in range(n):
        ref = oracle.apply_lut_c(oracle.d4(imgs[i], *flags[i]), luts[i])
        if gray is not None and gray[i]:
            ref = oracle.gray(ref)
        assert np.array_equal(got[i * size:(i + 1) * size], ref.reshape(-1)), i


@pytest.mark.parametrize("H,W,Hm,Wm,C", [(500, 380, 512, 512, 3), (512, 512, 512, 512, 3), (7, 600, 512, 512, 1),
                                         (1, 1, 5, 9, 4), (300, 700, 512, 512, 3)])
def test_pad_bit_exact_both_borders(m, H, W, Hm, Wm, C):
    import torch
    rng = np.random.default_rng(H + W)
    n = 3
    imgs = rng.integers(0, 256, (n, H, W, C), dtype=np.uint8)
    x = torch.from_numpy(imgs).cuda()
    for border, value in ((0, 0), (1, 77)):
        out = m.pad_u8(x, Hm, Wm, border, value).cpu().numpy()
        for i in range(n):
            ref = oracle.pad(imgs[i], Hm, Wm, oracle.REFLECT101 if border == 0 else oracle.CONSTANT, value)
            assert np.array_equal(out[i], ref), (i, border)


@pytest.mark.parametrize("interp,border", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_rotate_and_warp_bit_exact(m, interp, border):
    import torch
    n, H, W, C = 6, 61, 90, 3
    imgs = synth.smooth_u8_hwc(interp * 2 + border, n, H, W).numpy()
    f = np.array([[a, 1.0, 0.0, 0.0] for a in (-45.0, -12.5, 0.0, 30.0, 90.0)] + [[17.0, 1.07, 0.05, -0.03]],
                 np.float32)
    aq = m.compile_ssr_q32(f, H, W)
    for i in range(n):
        assert np.array_equal(aq[i], oracle.ssr_matrix_q32(*f[i], H, W))
    out = m.warp_affine_u8(torch.from_numpy(imgs).cuda(), torch.from_numpy(aq).cuda(), interp, border).cpu().numpy()
    for i in range(n):
        ref = oracle.warp_affine(imgs[i], aq[i], oracle.NEAREST if interp else oracle.BILINEAR,
                                 oracle.CONSTANT if border else oracle.REFLECT101)
        assert np.array_equal(out[i], ref), i
