"""GPU parity of the elastic + grid-distortion path: fields and grid tables
bit-exact, the u8 chain (images and masks) bit-exact, batched == per-image,
and the float copy forward (<= 1e-6) and adjoint (<= 1e-5 of max) against the
fp64 oracle, including sampled pixels of a 4096 x 4096 image."""
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


@pytest.mark.parametrize("H,W,sigma,alpha,radius", [(40, 36, 4.0, 60, 12), (1, 50, 3.0, 100, 7), (67, 1, 2.0, 30, 5),
                                                    (130, 1100, 50.0, 1000, 150), (3, 3, 1.0, 500, 1),
                                                    # rows wider than one horizontal-pass segment (2560 outputs)
                                                    (3, 5200, 50.0, 1000, 150), (2, 2561, 10.0, 500, 30),
                                                    # a centre tap of 2^15: the int32 multiply-add pass
                                                    (4, 40, 0.2, 100, 1)])
def test_fields_bit_exact(m, H, W, sigma, alpha, radius):
    off = m.elastic_fields(7, 3, 2, H, W, sigma, alpha, radius).cpu().numpy()
    for i in range(2):
        ox, oy = oracle.elastic_field(7, 3 + i, H, W, sigma, alpha, radius)
        assert np.array_equal(off[i, 0], ox) and np.array_equal(off[i, 1], oy), i


@pytest.mark.parametrize("n,H,W,sigma,alpha", [(2, 40, 36, 2.0, 60), (1, 1, 50, 3.0, 100), (1, 67, 1, 2.0, 30),
                                               (2, 96, 130, 6.0, 300), (1, 3, 3, 5.0, 500), (1, 512, 2048, 50.0, 1000)])
def test_box_fields_bit_exact(m, n, H, W, sigma, alpha):
    off = m.elastic_fields_box(7, 3, n, H, W, sigma, alpha).cpu().numpy()
    for i in range(n):
        ox, oy = oracle.elastic_field_box(7, 3 + i, H, W, sigma, alpha)
        assert np.array_equal(off[i, 0], ox) and np.array_equal(off[i, 1], oy), i


def test_grid_tables_bit_exact(m):
    import torch
    g = m.sample_grid(5, 0, 4)
    mx, my = m.grid_tables(torch.from_numpy(g).cuda(), 77, 4096)
    mx, my = mx.cpu().numpy(), my.cpu().numpy()
    for i in range(4):
        assert np.array_equal(mx[i], oracle.grid_table(g[i, :5], 4096))
        assert np.array_equal(my[i], oracle.grid_table(g[i, 5:], 77))


@pytest.mark.parametrize("H,W,C", [(64, 80, 3), (33, 47, 1), (100, 37, 4), (5, 300, 3)])
def test_u8_chain_bit_exact_and_batched_equals_per_image(m, H, W, C):
    import torch
    n = 3
    img = synth.smooth_u8_hwc(H * W + C, n, H, W, C)
    mask = synth.blob_masks(H + W, n, H, W, 8, 16)
    off = m.elastic_fields(3, 0, n, H, W, 4.0, 80, 12)
    g = m.sample_grid(3, 0, n)
    mx, my = m.grid_tables(torch.from_numpy(g).cuda(), H, W)
    out, om = m.elastic_grid_u8(img.cuda(), off, mx, my, mask.cuda())
    out2, om2 = m.elastic_grid_u8(img.cuda(), off, mx, my, mask.cuda(), per_image=True)
    torch.cuda.synchronize()
    assert torch.equal(out, out2) and torch.equal(om, om2)
    out, om = out.cpu().numpy(), om.cpu().numpy()
    for i in range(n):
        ref, rm = oracle.pipe_elastic_grid_one(img[i].numpy(), mask[i].numpy(), 3, i, g[i], 4.0, 80, 12)
        assert np.array_equal(out[i], ref), i
        assert np.array_equal(om[i], rm), i


@pytest.mark.parametrize("H,W,C,sigma,alpha,radius,limit", [
    (130, 260, 3, 50.0, 1000, 150, 0.3),   # the large-image field: every source block staged
    (70, 96, 4, 1.5, 300, 5, 0.3),         # rough, large displacements: source blocks too wide for LDS
    (70, 96, 4, 3.0, 150, 9, 0.3),         # source blocks of both kinds, some exactly 64 rows
    (150, 170, 3, 4.0, 80, 12, 0.95),      # grid steps up to 1.95x: e-blocks too wide for LDS, all three paths
    (37, 44, 1, 3.0, 60, 9, 0.6),          # W % 4 == 0 with a ragged last tile
])
def test_u8_chain_staging_paths_bit_exact(m, H, W, C, sigma, alpha, radius, limit):
    import torch
    n = 2
    img = synth.smooth_u8_hwc(H + 7 * W + C, n, H, W, C)
    mask = synth.blob_masks(H * W, n, H, W, 8, 16)
    off = m.elastic_fields(5, 0, n, H, W, sigma, alpha, radius)
    g = m.sample_grid(5, 0, n, limit)
    mx, my = m.grid_tables(torch.from_numpy(g).cuda(), H, W)
    out, om = m.elastic_grid_u8(img.cuda(), off, mx, my, mask.cuda())
    out2, _ = m.elastic_grid_u8(img.cuda(), off, mx, my, None)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    out, om = out.cpu().numpy(), om.cpu().numpy()
    for i in range(n):
        ref, rm = oracle.pipe_elastic_grid_one(img[i].numpy(), mask[i].numpy(), 5, i, g[i], sigma, alpha, radius)
        assert np.array_equal(out[i], ref), i
        assert np.array_equal(om[i], rm), i


def test_f32_chain_forward_and_adjoint(m):
    import torch
    n, C, H, W = 2, 3, 48, 40
    x = synth.smooth_noise(4, n, H, W, C)
    off = m.elastic_fields(4, 0, n, H, W, 4.0, 80, 12)
    g = m.sample_grid(4, 0, n)
    mx, my = m.grid_tables(torch.from_numpy(g).cuda(), H, W)
    y = m.elastic_grid_f32_fwd(x.cuda(), off, mx, my).cpu().numpy()
    gy = np.random.default_rng(3).uniform(-1, 1, (n, C, H, W)).astype(np.float32)
    gx = m.elastic_grid_f32_bwd(torch.from_numpy(gy).cuda(), off, mx, my).cpu().numpy()
    o, mxx, myy = off.cpu().numpy(), mx.cpu().numpy(), my.cpu().numpy()
    for i in range(n):
        yr = oracle.chain_f_forward(x[i].numpy(), o[i, 0], o[i, 1], mxx[i], myy[i])
        assert np.abs(y[i] - yr).max() <= 1e-6
        gr = oracle.chain_f_backward(gy[i].astype(np.float64), o[i, 0], o[i, 1], mxx[i], myy[i])
        assert np.abs(gx[i] - gr).max() <= 1e-5 * np.abs(gr).max()


def test_f32_adjoint_with_arbitrary_maps_and_far_offsets(m):
    # maps that are not monotonic and reach outside the image, offsets beyond
    # the image size (several reflect-101 folds), five channels (two channel
    # groups), and in image 1 a column map that folds every output onto two
    # source columns: the adjoint (table and scatter forms) against the oracle
    import torch
    n, C, H, W = 2, 5, 37, 53
    rng = np.random.default_rng(8)
    x = rng.uniform(0, 1, (n, C, H, W)).astype(np.float32)
    o = rng.integers(-70 * 1024, 70 * 1024, (n, 2, H, W)).astype(np.int32)
    mxx = rng.integers(-W * 1024, 2 * W * 1024, (n, W)).astype(np.int32)
    myy = rng.integers(-H * 1024, 2 * H * 1024, (n, H)).astype(np.int32)
    mxx[1] = 5 * 1024 + 512  # every output column samples x = 5.5: more than 8 outputs per source index (scatter form)
    off, mx, my = (torch.from_numpy(a).cuda() for a in (o, mxx, myy))
    y = m.elastic_grid_f32_fwd(torch.from_numpy(x).cuda(), off, mx, my).cpu().numpy()
    gy = rng.uniform(-1, 1, (n, C, H, W)).astype(np.float32)
    gx = m.elastic_grid_f32_bwd(torch.from_numpy(gy).cuda(), off, mx, my).cpu().numpy()
    for i in range(n):
        yr = oracle.chain_f_forward(x[i], o[i, 0], o[i, 1], mxx[i], myy[i])
        assert np.abs(y[i] - yr).max() <= 1e-6
        gr = oracle.chain_f_backward(gy[i].astype(np.float64), o[i, 0], o[i, 1], mxx[i], myy[i])
        assert np.abs(gx[i] - gr).max() <= 1e-5 * np.abs(gr).max(), i


def test_large_tile_sampled_pixels_against_the_definition(m):
    # one 4096 x 4096 image (sigma 50, alpha 1000, radius 150, 5x5 grid with limit 0.3):
    # sampled field values and output pixels recomputed by the oracle one by one
    import torch
    H = W = 4096
    img = synth.smooth_u8_hwc(1809068395, 1, H, W, 3, device="cuda")
    mask = synth.blob_masks(1809068396, 1, H, W, 8, 512, device="cuda")
    off = m.elastic_fields(1809068395, 0, 1, H, W)
    g = m.sample_grid(1809068395, 0, 1)
    mx, my = m.grid_tables(torch.from_numpy(g).cuda(), H, W)
    out, om = m.elastic_grid_u8(img, off, mx, my, mask)
    torch.cuda.synchronize()
    offn, imgn, mxn, myn = off.cpu().numpy()[0], img.cpu().numpy()[0], mx.cpu().numpy()[0], my.cpu().numpy()[0]
    rng = np.random.default_rng(6)
    pts = [(0, 0), (H - 1, W - 1), (0, W - 1)] + [tuple(v) for v in rng.integers(0, H, (5, 2))]
    for (yy, xx) in pts:
        assert oracle.elastic_field_at(1809068395, 0, H, W, yy, xx) == (offn[0, yy, xx], offn[1, yy, xx]), (yy, xx)
    # output pixels: grid taps of e, each e pixel from its own displaced taps
    assert np.array_equal(mxn, oracle.grid_table(g[0, :5], W)) and np.array_equal(myn, oracle.grid_table(g[0, 5:], H))
    outn = out.cpu().numpy()[0]
    for (yy, xx) in [tuple(v) for v in rng.integers(0, H, (200, 2))]:
        qx, qy = int(mxn[xx]), int(myn[yy])
        x0, y0, ax, ay = qx >> 10, qy >> 10, qx & 1023, qy & 1023
        e = {}
        for dy in (0, 1):
            for dx in (0, 1):
                Y, X = oracle.reflect101(y0 + dy, H), oracle.reflect101(x0 + dx, W)
                ex, ey = (X << 10) + int(offn[0, Y, X]), (Y << 10) + int(offn[1, Y, X])
                bx, by, fx, fy = ex >> 10, ey >> 10, ex & 1023, ey & 1023
                taps = [[imgn[oracle.reflect101(by + j, H), oracle.reflect101(bx + i, W)].astype(np.int64)
                         for i in (0, 1)] for j in (0, 1)]
                acc = (1024 - fy) * ((1024 - fx) * taps[0][0] + fx * taps[0][1]) + fy * ((1024 - fx) * taps[1][0] + fx * taps[1][1])
                e[(dy, dx)] = np.array([oracle.rshr_he(int(v), 20) for v in acc], np.int64)
        acc = (1024 - ay) * ((1024 - ax) * e[(0, 0)] + ax * e[(0, 1)]) + ay * ((1024 - ax) * e[(1, 0)] + ax * e[(1, 1)])
        ref = np.array([oracle.rshr_he(int(v), 20) for v in acc], np.uint8)
        assert np.array_equal(outn[yy, xx], ref), (yy, xx)
    # masks: the nearest grid tap of the elastic result, whose pixel is the
    # mask's nearest displaced tap; the field at that pixel from the oracle
    omn, maskn = om.cpu().numpy()[0], mask.cpu().numpy()[0]
    for (yy, xx) in [tuple(v) for v in rng.integers(0, H, (200, 2))] + [(0, 0), (H - 1, W - 1)]:
        Y = oracle.reflect101((int(myn[yy]) + 512) >> 10, H)
        X = oracle.reflect101((int(mxn[xx]) + 512) >> 10, W)
        ox, oy = oracle.elastic_field_at(1809068395, 0, H, W, Y, X)
        sy = oracle.reflect101(((Y << 10) + oy + 512) >> 10, H)
        sx = oracle.reflect101(((X << 10) + ox + 512) >> 10, W)
        assert omn[yy, xx] == maskn[sy, sx], (yy, xx)


def test_f32_chain_at_1024_against_the_oracle(m):
    # one 3 x 1024 x 1024 float image through the elastic (sigma 50, alpha 1000)
    # and grid maps the oracle computes; forward and adjoint against its fp64 chain
    import torch
    H = W = 1024
    x = synth.smooth_noise(9, 1, H, W, 3)
    ox, oy = oracle.elastic_field(9, 0, H, W)
    g = oracle.sample_grid(9, 0, 1)
    mx, my = oracle.grid_table(g[0, :5], W), oracle.grid_table(g[0, 5:], H)
    off = torch.from_numpy(np.stack([ox, oy])[None].copy()).cuda()
    mxt, myt = torch.from_numpy(mx[None].copy()).cuda(), torch.from_numpy(my[None].copy()).cuda()
    y = m.elastic_grid_f32_fwd(x.cuda(), off, mxt, myt).cpu().numpy()[0]
    yr = oracle.chain_f_forward(x[0].numpy(), ox, oy, mx, my)
    assert np.abs(y - yr).max() <= 1e-6
    gy = np.random.default_rng(4).uniform(-1, 1, (1, 3, H, W)).astype(np.float32)
    gx = m.elastic_grid_f32_bwd(torch.from_numpy(gy).cuda(), off, mxt, myt).cpu().numpy()[0]
    gr = oracle.chain_f_backward(gy[0].astype(np.float64), ox, oy, mx, my)
    assert np.abs(gx - gr).max() <= 1e-5 * np.abs(gr).max()


@pytest.mark.parametrize("n,H,W,C,smooth", [(3, 33, 17, 1, False), (2, 64, 64, 4, True), (2, 31, 31, 3, False),
                                            (2, 128, 128, 2, False), (3, 96, 80, 3, True), (2, 1, 6, 4, False)])
def test_image_stats_shapes_and_smooth_images(m, n, H, W, C, smooth):
    # four-pixel groups (npix a multiple of 4) and single pixels, 1-4 channels;
    # smooth images put many equal values in one group and on one histogram bin
    img = synth.smooth_u8_hwc(5 + H, n, H, W, C) if smooth else synth.uniform_u8(7 + H, n, H, W, C)
    s, mn, mx, h = m.image_stats_u8(img.cuda())
    for i in range(n):
        rs, rmn, rmx, rh = oracle.image_stats(img[i].cpu().numpy(), C)
        assert s[i].cpu().numpy().astype(np.uint64).tolist() == rs.tolist()
        assert mn[i].tolist() == rmn.tolist() and mx[i].tolist() == rmx.tolist()
        assert np.array_equal(h[i].cpu().numpy().astype(np.uint32), rh)


def test_image_stats_match_oracle(m):
    import torch
    img = synth.uniform_u8(3, 5, 70, 90, 3)
    s, mn, mx, h = m.image_stats_u8(img.cuda())
    for i in range(5):
        rs, rmn, rmx, rh = oracle.image_stats(img[i].numpy())
        assert s[i].cpu().numpy().astype(np.uint64).tolist() == rs.tolist()
        assert mn[i].tolist() == rmn.tolist() and mx[i].tolist() == rmx.tolist()
        assert np.array_equal(h[i].cpu().numpy().astype(np.uint32), rh)
    empty = torch.zeros((2, 0, 3), dtype=torch.uint8, device="cuda")
    s, mn, mx, h = m.image_stats_u8(empty)
    assert s.sum().item() == 0 and (mn == 255).all() and (mx == 0).all() and h.sum().item() == 0
