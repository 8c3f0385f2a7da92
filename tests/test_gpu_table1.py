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
                                         (1, 1, 5, 9, 4), (300, 700, 512, 512, 3),
                                         # output rows of 123 bytes: most pixel groups start off a word
                                         (5, 37, 9, 41, 3)])
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


@pytest.mark.parametrize("C", [1, 4])
@pytest.mark.parametrize("interp,border", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_warp_tiles_channels_and_zoom_bit_exact(m, C, interp, border):
    # ragged 32x32 tiles (100 x 77), identity, rotations, a zoom-in and a strong
    # zoom-out whose source boxes do not fit the stage (the direct path)
    import torch
    rng = np.random.default_rng(C * 10 + interp * 2 + border)
    H, W = 100, 77
    f = np.array([[0.0, 1.0, 0.0, 0.0], [33.0, 1.0, 0.0, 0.0], [-90.0, 1.0, 0.0, 0.0], [12.0, 3.0, 0.1, -0.05],
                  [25.0, 0.3, 0.0, 0.0], [-160.0, 0.45, 0.2, 0.2], [45.0, 1.1, -0.06, 0.06]], np.float32)
    n = len(f)
    imgs = rng.integers(0, 256, (n, H, W, C), dtype=np.uint8)
    aq = m.compile_ssr_q32(f, H, W)
    x = torch.from_numpy(imgs).cuda()
    if C == 1:
        x = x[..., 0].contiguous()
    out = m.warp_affine_u8(x, torch.from_numpy(aq).cuda(), interp, border).cpu().numpy().reshape(n, H, W, C)
    for i in range(n):
        ref = oracle.warp_affine(imgs[i], aq[i], oracle.NEAREST if interp else oracle.BILINEAR,
                                 oracle.CONSTANT if border else oracle.REFLECT101).reshape(H, W, C)
        assert np.array_equal(out[i], ref), i


def test_rotate_full_table1_size_bit_exact(m):
    # the Table I size, 512 x 512 x 3, whole images
    import torch
    n, H, W = 4, 512, 512
    imgs = synth.smooth_u8_hwc(99, n, H, W).numpy()
    f = np.array([[a, 1.0, 0.0, 0.0] for a in (-45.0, 7.5, 44.9)] + [[-21.0, 0.93, 0.0625, -0.0625]], np.float32)
    aq = m.compile_ssr_q32(f, H, W)
    out = m.warp_affine_u8(torch.from_numpy(imgs).cuda(), torch.from_numpy(aq).cuda(), 0, 0).cpu().numpy()
    for i in range(n):
        assert np.array_equal(out[i], oracle.warp_affine(imgs[i], aq[i], oracle.BILINEAR, oracle.REFLECT101)), i


def test_gamma_luts_match_the_chain_gamma(m):
    g = np.array([0.8, 1.0, 1.2, 0.93], np.float32)
    luts = m.compile_gamma_luts(g, C=3)
    for i in range(len(g)):
        ref = oracle.gamma_lut(g[i])
        for c in range(3):
            assert np.array_equal(luts[i, c], ref)


def test_gamma_via_lut_kernel_bit_exact(m):
    import torch
    n, H, W = 3, 130, 97
    imgs = synth.smooth_u8_hwc(5, n, H, W).numpy()
    g = np.array([0.8, 1.17, 1.0], np.float32)
    luts = torch.from_numpy(m.compile_gamma_luts(g)).cuda()
    fl = torch.zeros((n, 4), dtype=torch.int32, device="cuda")
    out = m.d4_lut_u8(torch.from_numpy(imgs).cuda(), fl, luts).cpu().numpy()
    for i in range(n):
        assert np.array_equal(out[i], oracle.gamma_lut(g[i])[imgs[i]]), i


def test_hsv_shift_every_rgb_colour_bit_exact(m):
    # all 2^24 RGB colours as one 4096 x 4096 image per shift set (quads path)
    import torch
    v = np.arange(1 << 24, dtype=np.uint32)
    img = np.stack([v & 255, (v >> 8) & 255, v >> 16], -1).astype(np.uint8).reshape(1, 4096, 4096, 3)
    x = torch.from_numpy(img).cuda()
    for dh, ds, dv in ((0, 0, 0), (-20, 30, 0), (179, -255, 17)):
        d = torch.tensor([[dh, ds, dv]], dtype=torch.int32, device="cuda")
        out = m.hsv_shift_u8(x, d).cpu().numpy()
        assert np.array_equal(out[0], oracle.hsv_shift(img[0], dh, ds, dv)), (dh, ds, dv)


@pytest.mark.parametrize("H,W", [(7, 9), (1, 1), (33, 65), (512, 512)])
def test_hsv_shift_shapes_and_tails_bit_exact(m, H, W):
    # odd pixel counts take the byte path, multiples of four the dword path
    import torch
    rng = np.random.default_rng(H * W)
    n = 3
    imgs = rng.integers(0, 256, (n, H, W, 3), dtype=np.uint8)
    d = rng.integers(-40, 41, (n, 3)).astype(np.int32)
    out = m.hsv_shift_u8(torch.from_numpy(imgs).cuda(), torch.from_numpy(d).cuda()).cpu().numpy()
    for i in range(n):
        assert np.array_equal(out[i], oracle.hsv_shift(imgs[i], int(d[i, 0]), int(d[i, 1]), int(d[i, 2]))), i


@pytest.mark.parametrize("k", [3, 5])
@pytest.mark.parametrize("H,W,C", [(1, 1, 3), (2, 3, 1), (31, 33, 3), (64, 96, 4), (100, 77, 1), (512, 512, 3)])
def test_blur_bit_exact(m, k, H, W, C):
    # tiles with ragged edges, images smaller than the halo, per-image on/off
    import torch
    rng = np.random.default_rng(k * 1000 + H + W + C)
    n = 3
    imgs = rng.integers(0, 256, (n, H, W, C), dtype=np.uint8)
    apply = torch.tensor([1, 0, 1], dtype=torch.int32, device="cuda")
    x = torch.from_numpy(imgs).cuda()
    if C == 1:
        x = x[..., 0].contiguous()
    out = m.blur_u8(x, k, apply).cpu().numpy().reshape(n, H, W, C)
    for i in range(n):
        ref = oracle.blur(imgs[i], k).reshape(H, W, C) if i != 1 else imgs[i]
        assert np.array_equal(out[i], ref), i
    out_all = m.blur_u8(x, k).cpu().numpy().reshape(n, H, W, C)
    assert np.array_equal(out_all[1], oracle.blur(imgs[1], k).reshape(H, W, C))


def test_blur_rejects_overlap_and_bad_ksize(m):
    import torch
    x = torch.zeros((1, 8, 8, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(m.MiaugError):
        m.blur_u8(x, 3, out=x)
    with pytest.raises(m.MiaugError):
        m.blur_u8(x, 7)
