"""Op-list pipelines (miaug_pipeline_*): matching of op lists onto the fused
chains, the per-op sampler (checked against the oracle's Philox), and on the
GPU each chain against a composition of the oracle's single ops, the direct
entry points, the per-image form and graph replays."""
import numpy as np
import pytest

import oracle
import synth

m = pytest.importorskip("paper_1809_06839_amd")
op = m.op


def uniform(seed, index, draw):
    return (oracle.draw_u64(seed, 0, index, draw) >> 11) * 2.0 ** -53


def f32_range(seed, index, draw, lo, hi):
    # op ranges are float fields: the bounds enter the double expression as float values
    lo, hi = float(np.float32(lo)), float(np.float32(hi))
    return np.float32(lo + (hi - lo) * uniform(seed, index, draw))


def below(seed, index, draw, mcount):
    return ((oracle.draw_u64(seed, 0, index, draw) >> 32) * mcount) >> 32


# ---------------------------------------------------------------- matching
def kind_of(ops):
    return m.Pipeline(None, ops).kind


def test_op_lists_map_onto_their_chains():
    assert kind_of([op("HFLIP", 0.5), op("VFLIP", 0.5), op("ROT90", 1, (0,), (3,)), op("TRANSPOSE", 0.5),
                    op("BRIGHT_CONTRAST", 1, (0.8, -51), (1.2, 51))]) == "DIH4"
    assert kind_of([op("BRIGHT_CONTRAST", 1, (0.8, -51), (1.2, 51))]) == "DIH4"
    assert kind_of([op("HFLIP", 0.5), op("RESIZE", out=(224, 224)),
                    op("NORMALIZE", 1, (0.485, 0.456, 0.406), (0.229, 0.224, 0.225))]) == "RAGGED"
    assert kind_of([op("RESIZE", out=(64, 32))]) == "RAGGED"
    assert kind_of([op("SSR", 1, (-45, 0.9, -0.0625, -0.0625), (45, 1.1, 0.0625, 0.0625)), op("CROP", out=(448, 448)),
                    op("RESIZE", out=(224, 224)), op("HSV", 1, (-20, -30), (20, 30)), op("GAMMA", 1, (0.8,), (1.2,)),
                    op("BLUR3", 0.3)]) == "U8CHAIN"
    assert kind_of([op("CROP", out=(8, 8)), op("RESIZE", out=(4, 4))]) == "U8CHAIN"
    assert kind_of([op("ELASTIC", 1, (1000, 50, 150)), op("GRID", 1, (0.3,))]) == "DISTORT"
    assert kind_of([op("GRID", 1, (0.3,))]) == "DISTORT"


@pytest.mark.parametrize("ops, status", [
    ([op("RESIZE", out=(8, 8)), op("HFLIP")], m.MiaugError),            # order
    ([op("HFLIP"), op("HFLIP")], m.MiaugError),                          # repeated op
    ([op("BLUR3"), op("BLUR5")], m.MiaugError),                          # no chain takes both
    ([op("HSV", 1, (-20, -30), (20, 30)), op("BLUR3", 0.3)], m.MiaugError),  # u8 chain without crop/resize
    ([op("HFLIP", 1.5)], m.MiaugError),                                  # p outside [0, 1]
    ([op("ROT90", 1, (0,), (4,))], m.MiaugError),                        # k outside 0..3
    ([op("SSR", 1, (0, 1, 0, 0), (0, 1, 0, 0), border=1), op("CROP", out=(4, 4)), op("RESIZE", out=(4, 4))],
     m.MiaugError),                                                      # constant border not in the u8 chain
])
def test_unsupported_or_invalid_lists_are_rejected(ops, status):
    with pytest.raises(status):
        m.Pipeline(None, ops)


def test_rejection_names_the_offending_op():
    with pytest.raises(m.MiaugError) as e:
        m.Pipeline(None, [op("HFLIP"), op("GAMMA", 1, (0.8,), (1.2,)), op("VFLIP")])
    assert "GAMMA" in str(e.value) or "VFLIP" in str(e.value)


# ---------------------------------------------------------------- sampling
def test_sampled_draws_follow_the_documented_layout():
    seed = 1809068391
    ops = [op("HFLIP", 0.5), op("ROT90", 1, (1,), (3,)), op("BRIGHT_CONTRAST", 0.7, (0.8, -51), (1.2, 51))]
    p = m.Pipeline(None, ops)
    recs = p.sample(seed, 100, 64)
    for i in range(64):
        g = 100 + i
        r = recs[i]
        assert r.seed == seed and r.index == g
        assert r.flags[0] == int(uniform(seed, g, 0) < 0.5)               # op 0 gate: draw 0
        assert r.flags[2] == 1 + below(seed, g, 16 + 1, 3)                # op 1 (p = 1, no gate): draw 17
        on = uniform(seed, g, 32) < 0.7                                    # op 2 gate: draw 32
        if on:
            assert r.alpha == f32_range(seed, g, 33, 0.8, 1.2)
            assert r.beta == f32_range(seed, g, 34, -51, 51)
        else:
            assert (r.alpha, r.beta) == (1.0, 0.0)
        assert r.flags[1] == 0 and r.flags[3] == 0                         # ops not in the list: identity


def test_samples_do_not_depend_on_batch_composition():
    p = m.Pipeline(None, [op("SSR", 1, (-45, 0.9, -0.0625, -0.0625), (45, 1.1, 0.0625, 0.0625)),
                          op("CROP", out=(448, 448)), op("RESIZE", out=(224, 224)),
                          op("HSV", 0.5, (-20, -30, -10), (20, 30, 10)), op("GAMMA", 1, (0.8,), (1.2,)),
                          op("BLUR3", 0.3)])
    hw = np.full((12, 2), 512, np.int32)
    a = p.sample(7, 0, 12, hw)
    b = p.sample(7, 5, 4, hw[:4])
    for i in range(4):
        assert bytes(a[5 + i]) == bytes(b[i])


def test_skipped_ops_take_identity_and_frequencies_match_p():
    p = m.Pipeline(None, [op("SSR", 0.25, (-45, 0.9, -0.1, -0.1), (45, 1.1, 0.1, 0.1)), op("CROP", out=(16, 16)),
                          op("RESIZE", out=(8, 8)), op("GAMMA", 0.5, (0.8,), (1.2,)), op("BLUR3", 0.3)])
    n = 4000
    hw = np.tile(np.array([[20, 24]], np.int32), (n, 1))
    recs = p.sample(3, 0, n, hw)
    ssr = np.array([(r.angle, r.scale, r.dx, r.dy) != (0.0, 1.0, 0.0, 0.0) for r in recs])
    gam = np.array([r.gamma != 1.0 for r in recs])
    blur = np.array([r.blur for r in recs])
    for frac, pp in ((ssr.mean(), 0.25), (gam.mean(), 0.5), (blur.mean(), 0.3)):
        assert abs(frac - pp) < 4 * np.sqrt(pp * (1 - pp) / n)
    cx = np.array([r.crop_x for r in recs]); cy = np.array([r.crop_y for r in recs])
    assert cx.min() == 0 and cx.max() == 24 - 16 and cy.min() == 0 and cy.max() == 20 - 16
    assert all(0.8 <= r.gamma <= 1.2 for r in recs)


def test_crop_needs_source_sizes_and_fitting_images():
    p = m.Pipeline(None, [op("CROP", out=(16, 16)), op("RESIZE", out=(8, 8))])
    with pytest.raises(m.MiaugError):
        p.sample(1, 0, 2)
    with pytest.raises(m.MiaugError):
        p.sample(1, 0, 1, np.array([[8, 40]], np.int32))


def test_param_record_size():
    p = m.Pipeline(None, [op("HFLIP")])
    assert m.lib().miaug_param_bytes(p.handle, 3) == 3 * 192


# ---------------------------------------------------------------- GPU
@pytest.fixture(scope="module")
def ctx(dev):
    m.lib()
    return m.Context(0)


def host_flags(recs, n):
    flags = np.array([[recs[i].flags[k] for k in range(4)] for i in range(n)], np.int32)
    ab = np.array([[recs[i].alpha, recs[i].beta] for i in range(n)], np.float32)
    return flags, ab


@pytest.mark.gpu
def test_dih4_pipeline_matches_the_oracle_ops_and_masks_follow(ctx):
    import torch
    n, H, W = 7, 37, 53
    p = m.Pipeline(ctx, [op("HFLIP", 0.5), op("VFLIP", 0.5), op("ROT90", 1, (0,), (3,)), op("TRANSPOSE", 0.5),
                         op("BRIGHT_CONTRAST", 0.8, (0.8, -51), (1.2, 51))])
    imgs = synth.uniform_u8(11, n, H, W).numpy()
    masks = np.ascontiguousarray(synth.uniform_u8(12, n, H, W, 1).numpy()[..., 0])
    recs = p.sample(99, 0, n)
    x = torch.from_numpy(imgs).cuda(); xm = torch.from_numpy(masks).cuda()
    out = torch.empty_like(x); om = torch.empty_like(xm)
    bi, bo, _ = p.batch(img=x, mask=xm)
    bo.img, bo.mask = out.data_ptr(), om.data_ptr()
    p.apply(bi, bo, recs)
    got = out.cpu().numpy().reshape(n, -1); gm = om.cpu().numpy().reshape(n, -1)
    flags, ab = host_flags(recs, n)
    for i in range(n):
        ref = oracle.apply_lut(oracle.d4(imgs[i], *flags[i]), oracle.bc_lut(*ab[i]))
        assert np.array_equal(got[i], ref.reshape(-1)), i
        assert np.array_equal(gm[i], oracle.d4(masks[i], *flags[i]).reshape(-1)), i
    # per-image form
    out2 = torch.empty_like(x); om2 = torch.empty_like(xm)
    bo.img, bo.mask = out2.data_ptr(), om2.data_ptr()
    p.apply(bi, bo, recs, per_image=True)
    assert torch.equal(out, out2) and torch.equal(om, om2)


@pytest.mark.gpu
def test_ragged_pipeline_equals_the_direct_entry_point_and_the_oracle(ctx):
    sizes = [(1, 1), (300, 41), (129, 1000), (224, 224), (57, 91), (640, 480)]
    b = synth.ragged_batch(21, len(sizes), sizes=sizes)
    p = m.Pipeline(ctx, [op("HFLIP", 0.5), op("VFLIP", 0.5), op("ROT90", 1, (0,), (3,)), op("TRANSPOSE", 0.5),
                         op("BRIGHT_CONTRAST", 1, (0.8, -51), (1.2, 51)), op("RESIZE", out=(224, 224)),
                         op("NORMALIZE", 1, m.IMAGENET_MEAN, m.IMAGENET_STD)])
    recs = p.sample(5, 1000, b.n)
    flags, ab = host_flags(recs, b.n)
    r1 = m.Ragged.from_host(b, flags, ab)
    m.ragged_apply(ctx, r1)
    r2 = m.Ragged.from_host(b, flags, ab)
    bi, bo, _ = p.batch(ragged=r2)
    p.apply(bi, bo, recs)
    import torch
    torch.cuda.synchronize()
    assert np.array_equal(r1.out.cpu().numpy().view(np.uint32), r2.out.cpu().numpy().view(np.uint32))
    assert np.array_equal(r1.out_mask.cpu().numpy(), r2.out_mask.cpu().numpy())
    for i in (0, 2, 5):
        ref, rm, _ = oracle.pipe_ragged_one(b.image(i), b.mask_of(i), flags[i], ab[i], b.boxes_of(i), 224, 224)
        assert np.array_equal(r2.out.cpu().numpy()[i].view(np.uint32), ref.view(np.uint32)), i
        assert np.array_equal(r2.out_mask.cpu().numpy()[i], rm), i


@pytest.mark.gpu
def test_ragged_pipeline_graph_takes_new_records_each_replay(ctx):
    import torch
    b = synth.ragged_batch(22, 5, sizes=[(100, 200), (333, 77), (64, 64), (500, 300), (31, 17)])
    p = m.Pipeline(ctx, [op("HFLIP", 0.5), op("ROT90", 1, (0,), (3,)), op("BRIGHT_CONTRAST", 1, (0.8, -51), (1.2, 51)),
                         op("RESIZE", out=(48, 40))])
    recs0 = p.sample(1, 0, b.n)
    flags, ab = host_flags(recs0, b.n)
    r = m.Ragged.from_host(b, flags, ab, out_h=48, out_w=40)
    bi, bo, _ = p.batch(ragged=r)
    s = torch.cuda.Stream()
    g = p.graph(bi, bo, s)
    for rep in range(3):
        recs = p.sample(1, 100 * rep, b.n)
        g.launch(recs, s)
        s.synchronize()
        got = r.out.cpu().numpy().copy()
        fl, a2 = host_flags(recs, b.n)
        for i in range(b.n):
            ref, _, _ = oracle.pipe_ragged_one(b.image(i), b.mask_of(i), fl[i], a2[i], b.boxes_of(i), 48, 40,
                                               mean=(0.0, 0.0, 0.0), std=(1 / 255.0,) * 3)
            assert np.array_equal(got[i].view(np.uint32), ref.view(np.uint32)), (rep, i)
    g.close()


@pytest.mark.gpu
@pytest.mark.parametrize("ops", [
    [("BLUR5", 0.5)],
    [("HSV", 0.7, (-20, -30, -10), (20, 30, 10))],
    [("HFLIP", 0.5), ("BRIGHT_CONTRAST", 0.8, (0.8, -51), (1.2, 51)), ("GAMMA", 0.8, (0.7,), (1.4,))],
])
def test_new_chains_graph_replays_take_new_records(ctx, ops):
    # captured once, replayed with fresh records (eager work and a synchronisation between
    # replays); every replay equals the eager apply of the same records, masks included
    import torch
    n, H, W = 4, 35, 52
    rng = np.random.default_rng(len(ops))
    imgs = rng.integers(0, 256, (n, H, W, 3), dtype=np.uint8)
    masks = rng.integers(0, 9, (n, H, W), dtype=np.uint8)
    p = m.Pipeline(ctx, [op(*o) for o in ops])
    x, xm = torch.from_numpy(imgs).cuda(), torch.from_numpy(masks).cuda()
    out, om = torch.empty_like(x), torch.empty_like(xm)
    bi, bo, _ = p.batch(img=x, mask=xm)
    bo.img, bo.mask = out.data_ptr(), om.data_ptr()
    s = torch.cuda.Stream()
    g = p.graph(bi, bo, s)
    ref, rm = torch.empty_like(out), torch.empty_like(om)
    bo2 = type(bo).from_buffer_copy(bo)
    bo2.img, bo2.mask = ref.data_ptr(), rm.data_ptr()
    for rep in range(3):
        recs = p.sample(40 + rep, 0, n)
        g.launch(recs, s)
        s.synchronize()
        p.apply(bi, bo2, recs)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
        assert torch.equal(om, rm), rep
        out.zero_()
        om.zero_()
        torch.cuda.synchronize()
    g.close()


@pytest.mark.gpu
def test_u8_chain_pipeline_matches_the_oracle_ops_including_value_shift(ctx):
    import torch
    n, H, W, crop, outsz = 5, 96, 80, 64, 40
    p = m.Pipeline(ctx, [op("SSR", 1, (-45, 0.9, -0.0625, -0.0625), (45, 1.1, 0.0625, 0.0625)),
                         op("CROP", out=(crop, crop)), op("RESIZE", out=(outsz, outsz)),
                         op("HSV", 1, (-20, -30, -15), (20, 30, 15)), op("GAMMA", 1, (0.8,), (1.2,)),
                         op("BLUR3", 0.5)])
    imgs = synth.smooth_u8_hwc(31, n, H, W).numpy()
    recs = p.sample(8, 0, n, np.tile(np.array([[H, W]], np.int32), (n, 1)))
    x = torch.from_numpy(imgs).cuda()
    out = torch.empty((n, outsz, outsz, 3), dtype=torch.uint8, device="cuda")
    bi, bo, _ = p.batch(img=x)
    bo.img = out.data_ptr()
    p.apply(bi, bo, recs)
    got = out.cpu().numpy()
    for i in range(n):
        r = recs[i]
        aq = oracle.ssr_matrix_q32(r.angle, r.scale, r.dx, r.dy, H, W)
        y = oracle.warp_affine(imgs[i], aq)
        y = oracle.crop(y, r.crop_x, r.crop_y, crop, crop)
        y = oracle.resize(y, outsz, outsz)
        y = oracle.hsv_shift(y, r.dh, r.ds, r.dv)
        y = oracle.apply_lut(y, oracle.gamma_lut(r.gamma))
        if r.blur:
            y = oracle.blur(y, 3)
        assert np.array_equal(got[i], y), (i, r.dv, r.blur)
    out2 = torch.empty_like(out)
    bo.img = out2.data_ptr()
    p.apply(bi, bo, recs, per_image=True)
    assert torch.equal(out, out2)


@pytest.mark.gpu
def test_distortion_pipeline_matches_the_oracle_chain(ctx):
    import torch
    n, H, W = 3, 72, 96
    p = m.Pipeline(ctx, [op("ELASTIC", 1, (300, 6, 18)), op("GRID", 1, (0.3,))])
    imgs = synth.smooth_u8_hwc(41, n, H, W).numpy()
    masks = synth.blob_masks(42, n, H, W, 8, 32).numpy()
    recs = p.sample(77, 10, n)
    x = torch.from_numpy(imgs).cuda(); xm = torch.from_numpy(masks).cuda()
    out = torch.empty_like(x); om = torch.empty_like(xm)
    bi, bo, _ = p.batch(img=x, mask=xm)
    bo.img, bo.mask = out.data_ptr(), om.data_ptr()
    p.apply(bi, bo, recs)
    got, gm = out.cpu().numpy(), om.cpu().numpy()
    for i in range(n):
        grid = np.array(list(recs[i].grid), np.float64)
        ref, rm = oracle.pipe_elastic_grid_one(imgs[i], masks[i], 77, 10 + i, grid, sigma=6.0, alpha=300, radius=18)
        assert np.array_equal(got[i], ref), i
        assert np.array_equal(gm[i], rm), i
    # grid only: zero offsets
    pg = m.Pipeline(ctx, [op("GRID", 1, (0.3,))])
    recs = pg.sample(5, 0, n)
    pg.apply(bi, bo, recs)
    got = out.cpu().numpy()
    for i in range(n):
        d = np.array(list(recs[i].grid), np.float64)
        ref = oracle.grid_remap(imgs[i], oracle.grid_table(d[:5], W), oracle.grid_table(d[5:], H))
        assert np.array_equal(got[i], ref), i


@pytest.mark.gpu
def test_distortion_pipeline_with_the_box_field(ctx):
    import torch
    n, H, W = 2, 64, 90
    p = m.Pipeline(ctx, [op("ELASTIC", 1, (300, 6, 0), (1, 0, 0)), op("GRID", 1, (0.3,))])
    imgs = synth.smooth_u8_hwc(43, n, H, W).numpy()
    recs = p.sample(78, 0, n)
    x = torch.from_numpy(imgs).cuda()
    out = torch.empty_like(x)
    bi, bo, _ = p.batch(img=x)
    bo.img = out.data_ptr()
    p.apply(bi, bo, recs)
    got = out.cpu().numpy()
    for i in range(n):
        d = np.array(list(recs[i].grid), np.float64)
        ox, oy = oracle.elastic_field_box(78, i, H, W, 6.0, 300)
        e = oracle.remap_field(imgs[i], ox, oy)
        ref = oracle.grid_remap(e, oracle.grid_table(d[:5], W), oracle.grid_table(d[5:], H))
        assert np.array_equal(got[i], ref), i


# ---------------------------------------------------------------- random-sized crop
def test_sized_crop_sampler_matches_the_oracle_windows():
    seed = 1809068395
    scale, ratio = (0.08, 1.0), (0.75, 4 / 3)
    ops = [op("HFLIP", 0.5), op("ROT90", 1, (0,), (3,)), op("TRANSPOSE", 0.5),
           op("SIZED_CROP", 0.9, (scale[0], ratio[0]), (scale[1], ratio[1])),
           op("RESIZE", out=(224, 224))]
    p = m.Pipeline(None, ops)
    assert p.kind == "RAGGED"
    rng = np.random.default_rng(3)
    n = 200
    hw = np.stack([rng.integers(1, 1025, n), rng.integers(1, 1025, n)], 1).astype(np.int32)
    recs = p.sample(seed, 50, n, hw)
    f32 = lambda v: float(np.float32(v))
    for i in range(n):
        r, g = recs[i], 50 + i
        on = uniform(seed, g, 48) < 0.9                                   # op 3 gate: draw 48
        if not on:
            assert (r.crop_h, r.crop_w) == (0, 0)
            continue
        swap = (r.flags[2] & 1) != (r.flags[3] != 0)
        H, W = (hw[i][1], hw[i][0]) if swap else (hw[i][0], hw[i][1])
        ref = oracle.sized_crop_window(seed, g, 48 + 1, int(H), int(W), (f32(scale[0]), f32(scale[1])),
                                       (f32(ratio[0]), f32(ratio[1])))
        assert (r.crop_y, r.crop_x, r.crop_h, r.crop_w) == tuple(int(v) for v in ref), i
    with pytest.raises(m.MiaugError):
        p.sample(seed, 0, 2)  # source sizes are needed


@pytest.mark.gpu
def test_ragged_pipeline_with_sized_crop_matches_the_oracle(ctx):
    import torch
    sizes = [(1, 1), (300, 41), (129, 1000), (224, 224), (57, 91), (640, 480), (1024, 128)]
    b = synth.ragged_batch(23, len(sizes), sizes=sizes)
    p = m.Pipeline(ctx, [op("HFLIP", 0.5), op("VFLIP", 0.5), op("ROT90", 1, (0,), (3,)), op("TRANSPOSE", 0.5),
                         op("SIZED_CROP", 0.8, (0.08, 0.75), (1.0, 4 / 3)),
                         op("BRIGHT_CONTRAST", 1, (0.8, -51), (1.2, 51)), op("RESIZE", out=(96, 128)),
                         op("NORMALIZE", 1, m.IMAGENET_MEAN, m.IMAGENET_STD)])
    recs = p.sample(9, 0, b.n, np.asarray(b.hw, np.int32))
    flags, ab = host_flags(recs, b.n)
    r = m.Ragged.from_host(b, flags, ab, out_h=96, out_w=128)
    bi, bo, _ = p.batch(ragged=r)
    p.apply(bi, bo, recs)
    torch.cuda.synchronize()
    out, om = r.out.cpu().numpy(), r.out_mask.cpu().numpy()
    ob = r.out_boxes.cpu().numpy() if r.out_boxes is not None else None
    for i in range(b.n):
        win = None if recs[i].crop_h == 0 else (recs[i].crop_y, recs[i].crop_x, recs[i].crop_h, recs[i].crop_w)
        ref, rm, rb = oracle.pipe_ragged_one(b.image(i), b.mask_of(i), flags[i], ab[i], b.boxes_of(i), 96, 128,
                                             win=win)
        assert np.array_equal(out[i].view(np.uint32), ref.view(np.uint32)), i
        assert np.array_equal(om[i], rm), i
        if len(rb):
            got = ob[b.box_off[i]:b.box_off[i + 1]]
            assert np.all(np.abs(got - rb) <= 1e-5 * np.maximum(1.0, np.abs(rb))), i


@pytest.mark.gpu
def test_u8_chain_pipeline_takes_masks_and_boxes(ctx):
    import torch
    n, H, W, crop, outsz = 4, 96, 80, 64, 40
    p = m.Pipeline(ctx, [op("SSR", 1, (-45, 0.9, -0.0625, -0.0625), (45, 1.1, 0.0625, 0.0625)),
                         op("CROP", out=(crop, crop)), op("RESIZE", out=(outsz, outsz)), op("GAMMA", 1, (0.8,), (1.2,))])
    imgs = synth.smooth_u8_hwc(32, n, H, W).numpy()
    masks = np.ascontiguousarray(synth.blob_masks(33, n, H, W, 8, 16).numpy())
    boxes = np.array([[5, 6, 40, 50], [0, 0, 80, 96], [30, 30, 31, 31], [70, 2, 79, 90], [10, 80, 60, 95]], np.float32)
    off = np.array([0, 2, 2, 4, 5], np.int32)
    recs = p.sample(10, 0, n, np.tile(np.array([[H, W]], np.int32), (n, 1)))
    x, xm = torch.from_numpy(imgs).cuda(), torch.from_numpy(masks).cuda()
    bxd, offd = torch.from_numpy(boxes).cuda(), torch.from_numpy(off).cuda()
    out = torch.empty((n, outsz, outsz, 3), dtype=torch.uint8, device="cuda")
    om = torch.empty((n, outsz, outsz), dtype=torch.uint8, device="cuda")
    ob = torch.empty_like(bxd)
    bi, bo, _ = p.batch(img=x, mask=xm, boxes=bxd, box_off=offd)
    bo.img, bo.mask, bo.boxes = out.data_ptr(), om.data_ptr(), ob.data_ptr()
    p.apply(bi, bo, recs)
    torch.cuda.synchronize()
    gm, gb = om.cpu().numpy(), ob.cpu().numpy()
    for i in range(n):
        r = recs[i]
        aq = oracle.ssr_matrix_q32(r.angle, r.scale, r.dx, r.dy, H, W)
        ref = oracle.resize(oracle.crop(oracle.warp_affine(masks[i], aq, oracle.NEAREST), r.crop_x, r.crop_y, crop, crop),
                            outsz, outsz, oracle.NEAREST)
        assert np.array_equal(gm[i], ref), i
        rb = oracle.boxes_ssr_crop_resize(boxes[off[i]:off[i + 1]], H, W, (r.angle, r.scale, r.dx, r.dy), r.crop_x,
                                          r.crop_y, crop, outsz)
        assert np.all(np.abs(gb[off[i]:off[i + 1]] - rb) <= 1e-5 * np.maximum(1.0, np.abs(rb))), i
    om2 = torch.empty_like(om)
    bo.mask = om2.data_ptr()
    p.apply(bi, bo, recs, per_image=True)
    assert torch.equal(om, om2)


# ---------------------------------------------------------------- the other Table I ops
def test_table1_op_lists_map_onto_their_chains():
    assert kind_of([op("HFLIP", 0.5), op("BRIGHT_CONTRAST", 1, (0.8, -51), (1.2, 51)),
                    op("SHIFT_RGB", 0.5, (-20, -20, -20), (20, 20, 20)), op("TO_GRAY", 0.3)]) == "DIH4"
    assert kind_of([op("SHIFT_RGB", 1, (-20, -20, -20), (20, 20, 20))]) == "DIH4"
    assert kind_of([op("ROTATE", 1, (-45,), (45,))]) == "WARP"
    assert kind_of([op("SSR", 1, (-45, 0.9, -0.06, -0.06), (45, 1.1, 0.06, 0.06), border=1)]) == "WARP"
    assert kind_of([op("PAD", out=(512, 512))]) == "PAD"
    with pytest.raises(m.MiaugError):
        m.Pipeline(None, [op("TO_GRAY"), op("SHIFT_RGB")])  # order
    with pytest.raises(m.MiaugError):
        m.Pipeline(None, [op("PAD", 0.5, out=(8, 8))])      # PAD has p = 1
    # Gamma as a LUT step of the Dih4 chain; ShiftHSV alone
    assert kind_of([op("GAMMA", 1, (0.8,), (1.2,))]) == "DIH4"
    assert kind_of([op("HFLIP", 0.5), op("BRIGHT_CONTRAST", 1, (0.8, -51), (1.2, 51)), op("SHIFT_RGB", 0.5, (-9,) * 3,
                    (9,) * 3), op("GAMMA", 0.5, (0.8,), (1.2,)), op("TO_GRAY", 0.3)]) == "DIH4"
    assert kind_of([op("HSV", 1, (-20, -30, 0), (20, 30, 0))]) == "HSV"
    assert kind_of([op("BLUR3", 0.3)]) == "BLUR" and kind_of([op("BLUR5", 0.3)]) == "BLUR"
    assert kind_of([op("CROP", out=(64, 64)), op("RESIZE", out=(64, 64)), op("HSV", 1, (-20, -30, 0), (20, 30, 0)),
                    op("GAMMA", 1, (0.8,), (1.2,))]) == "U8CHAIN"
    with pytest.raises(m.MiaugError):
        m.Pipeline(None, [op("TO_GRAY"), op("GAMMA", 1, (0.8,), (1.2,))])  # order
    with pytest.raises(m.MiaugError):
        m.Pipeline(None, [op("HSV", 1, (-20, -30, 0), (20, 30, 0)), op("GAMMA", 1, (0.8,), (1.2,))])


def test_table1_sampler_draws():
    seed = 1809068396
    p = m.Pipeline(None, [op("SHIFT_RGB", 0.5, (-20, -10, 0), (20, 10, 5)), op("TO_GRAY", 0.3)])
    recs = p.sample(seed, 7, 300)
    for i in range(300):
        r, g = recs[i], 7 + i
        if uniform(seed, g, 0) < 0.5:
            for c, (lo, hi) in enumerate(((-20, 20), (-10, 10), (0, 5))):
                assert r.shift[c] == f32_range(seed, g, 1 + c, lo, hi)
        else:
            assert list(r.shift) == [0.0, 0.0, 0.0]
        assert r.gray == int(uniform(seed, g, 16) < 0.3)
    p = m.Pipeline(None, [op("ROTATE", 0.7, (-45,), (45,))])
    recs = p.sample(seed, 0, 100)
    for i in range(100):
        on = uniform(seed, i, 0) < 0.7
        assert recs[i].angle == (f32_range(seed, i, 1, -45, 45) if on else 0.0)
        assert recs[i].scale == 1.0 and recs[i].dx == 0.0 and recs[i].dy == 0.0


@pytest.mark.gpu
def test_color_chain_pipeline_matches_the_oracle(ctx):
    import torch
    n, H, W = 6, 37, 52
    rng = np.random.default_rng(11)
    imgs = rng.integers(0, 256, (n, H, W, 3), dtype=np.uint8)
    masks = rng.integers(0, 21, (n, H, W), dtype=np.uint8)
    p = m.Pipeline(ctx, [op("HFLIP", 0.5), op("ROT90", 1, (0,), (3,)), op("BRIGHT_CONTRAST", 0.8, (0.8, -51), (1.2, 51)),
                         op("SHIFT_RGB", 0.7, (-20, -20, -20), (20, 20, 20)), op("TO_GRAY", 0.5)])
    recs = p.sample(12, 0, n)
    x, xm = torch.from_numpy(imgs).cuda(), torch.from_numpy(masks).cuda()
    out, om = torch.empty_like(x), torch.empty_like(xm)
    bi, bo, _ = p.batch(img=x, mask=xm)
    bo.img, bo.mask = out.data_ptr(), om.data_ptr()
    p.apply(bi, bo, recs)
    torch.cuda.synchronize()
    got, gm = out.cpu().numpy().reshape(n, -1), om.cpu().numpy().reshape(n, -1)
    for i in range(n):
        r = recs[i]
        fl = [r.flags[k] for k in range(4)]
        y = oracle.apply_lut(oracle.d4(imgs[i], *fl), oracle.bc_lut(r.alpha, r.beta))
        y = oracle.apply_lut_c(y, oracle.shift_rgb_lut(list(r.shift)))
        if r.gray:
            y = oracle.gray(y)
        assert np.array_equal(got[i], y.reshape(-1)), i
        assert np.array_equal(gm[i], oracle.d4(masks[i], *fl).reshape(-1)), i
    out2 = torch.empty_like(out)
    bo.img = out2.data_ptr()
    p.apply(bi, bo, recs, per_image=True)
    assert torch.equal(out, out2)


@pytest.mark.gpu
def test_gamma_in_the_color_chain_matches_the_oracle(ctx):
    import torch
    n, H, W = 6, 41, 29
    rng = np.random.default_rng(21)
    imgs = rng.integers(0, 256, (n, H, W, 3), dtype=np.uint8)
    p = m.Pipeline(ctx, [op("VFLIP", 0.5), op("BRIGHT_CONTRAST", 0.8, (0.8, -51), (1.2, 51)),
                         op("SHIFT_RGB", 0.7, (-20, -20, -20), (20, 20, 20)), op("GAMMA", 0.8, (0.7,), (1.4,)),
                         op("TO_GRAY", 0.4)])
    recs = p.sample(22, 0, n)
    x = torch.from_numpy(imgs).cuda()
    out = torch.empty_like(x)
    bi, bo, _ = p.batch(img=x)
    bo.img = out.data_ptr()
    p.apply(bi, bo, recs)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(n, -1)
    for i in range(n):
        r = recs[i]
        y = oracle.apply_lut(oracle.d4(imgs[i], *[r.flags[k] for k in range(4)]), oracle.bc_lut(r.alpha, r.beta))
        y = oracle.apply_lut_c(y, oracle.shift_rgb_lut(list(r.shift)))
        y = oracle.apply_lut(y, oracle.gamma_lut(r.gamma))
        if r.gray:
            y = oracle.gray(y)
        assert np.array_equal(got[i], y.reshape(-1)), i


@pytest.mark.gpu
@pytest.mark.parametrize("kind,k", [("BLUR3", 3), ("BLUR5", 5)])
def test_blur_pipeline_matches_the_oracle(ctx, kind, k):
    import torch
    n, H, W = 7, 37, 70
    rng = np.random.default_rng(k)
    imgs = rng.integers(0, 256, (n, H, W, 3), dtype=np.uint8)
    masks = rng.integers(0, 9, (n, H, W), dtype=np.uint8)
    p = m.Pipeline(ctx, [op(kind, 0.5)])
    recs = p.sample(25 + k, 0, n)
    assert 0 < sum(r.blur for r in recs) < n  # both branches
    x, xm = torch.from_numpy(imgs).cuda(), torch.from_numpy(masks).cuda()
    out, om = torch.empty_like(x), torch.empty_like(xm)
    bi, bo, _ = p.batch(img=x, mask=xm)
    bo.img, bo.mask = out.data_ptr(), om.data_ptr()
    p.apply(bi, bo, recs)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for i in range(n):
        ref = oracle.blur(imgs[i], k) if recs[i].blur else imgs[i]
        assert np.array_equal(got[i], ref), i
    assert np.array_equal(om.cpu().numpy(), masks)


@pytest.mark.gpu
def test_hsv_pipeline_matches_the_oracle(ctx):
    import torch
    n, H, W = 5, 33, 48
    rng = np.random.default_rng(23)
    imgs = rng.integers(0, 256, (n, H, W, 3), dtype=np.uint8)
    masks = rng.integers(0, 9, (n, H, W), dtype=np.uint8)
    p = m.Pipeline(ctx, [op("HSV", 0.7, (-20, -30, -10), (20, 30, 10))])
    recs = p.sample(24, 0, n)
    x, xm = torch.from_numpy(imgs).cuda(), torch.from_numpy(masks).cuda()
    out, om = torch.empty_like(x), torch.empty_like(xm)
    bi, bo, _ = p.batch(img=x, mask=xm)
    bo.img, bo.mask = out.data_ptr(), om.data_ptr()
    p.apply(bi, bo, recs)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for i in range(n):
        r = recs[i]
        assert np.array_equal(got[i], oracle.hsv_shift(imgs[i], r.dh, r.ds, r.dv)), i
    assert np.array_equal(om.cpu().numpy(), masks)
    out2 = torch.empty_like(out)
    bo.img = out2.data_ptr()
    p.apply(bi, bo, recs, per_image=True)
    assert torch.equal(out, out2)


@pytest.mark.gpu
@pytest.mark.parametrize("interp,border", [(0, 0), (1, 1)])
def test_rotate_and_pad_pipelines_match_the_oracle(ctx, interp, border):
    import torch
    n, H, W = 5, 45, 60
    imgs = synth.smooth_u8_hwc(13, n, H, W).numpy()
    masks = np.ascontiguousarray(synth.blob_masks(14, n, H, W, 8, 16).numpy())
    x, xm = torch.from_numpy(imgs).cuda(), torch.from_numpy(masks).cuda()
    p = m.Pipeline(ctx, [op("ROTATE", 0.8, (-45,), (45,), interp=interp, border=border)])
    recs = p.sample(15, 0, n)
    out, om = torch.empty_like(x), torch.empty_like(xm)
    bi, bo, _ = p.batch(img=x, mask=xm)
    bo.img, bo.mask = out.data_ptr(), om.data_ptr()
    p.apply(bi, bo, recs)
    torch.cuda.synchronize()
    bor = oracle.CONSTANT if border else oracle.REFLECT101
    for i in range(n):
        aq = oracle.ssr_matrix_q32(recs[i].angle, 1.0, 0.0, 0.0, H, W)
        ref = oracle.warp_affine(imgs[i], aq, oracle.NEAREST if interp else oracle.BILINEAR, bor)
        assert np.array_equal(out.cpu().numpy()[i], ref), i
        assert np.array_equal(om.cpu().numpy()[i], oracle.warp_affine(masks[i], aq, oracle.NEAREST, bor)), i
    p = m.Pipeline(ctx, [op("PAD", 1, (33,), out=(64, 80), border=border)])
    recs = p.sample(16, 0, n)
    out = torch.empty((n, 64, 80, 3), dtype=torch.uint8, device="cuda")
    om = torch.empty((n, 64, 80), dtype=torch.uint8, device="cuda")
    bi, bo, _ = p.batch(img=x, mask=xm)
    bo.img, bo.mask = out.data_ptr(), om.data_ptr()
    p.apply(bi, bo, recs)
    torch.cuda.synchronize()
    for i in range(n):
        assert np.array_equal(out.cpu().numpy()[i], oracle.pad(imgs[i], 64, 80, bor, 33)), i
        assert np.array_equal(om.cpu().numpy()[i], oracle.pad(masks[i], 64, 80, bor, 0)), i


@pytest.mark.gpu
def test_distortion_pipeline_transforms_boxes_like_their_masks(ctx):
    import torch
    n, H, W = 3, 72, 96
    p = m.Pipeline(ctx, [op("ELASTIC", 1, (300, 6, 18)), op("GRID", 1, (0.3,))])
    imgs = synth.smooth_u8_hwc(44, n, H, W).numpy()
    boxes = np.array([[10, 5, 40, 30], [0, 0, 96, 72], [50.5, 40.2, 70.7, 71.9], [90, 60, 96, 72], [20, 20, 20.2, 20.2],
                      [33, 11, 34, 12]], np.float32)
    off = np.array([0, 2, 5, 6], np.int32)
    recs = p.sample(79, 3, n)
    x = torch.from_numpy(imgs).cuda()
    bxd, offd = torch.from_numpy(boxes).cuda(), torch.from_numpy(off).cuda()
    out = torch.empty_like(x)
    ob = torch.full_like(bxd, -7.0)
    bi, bo, _ = p.batch(img=x, boxes=bxd, box_off=offd)
    bo.img, bo.boxes = out.data_ptr(), ob.data_ptr()
    p.apply(bi, bo, recs)
    torch.cuda.synchronize()
    gb = ob.cpu().numpy()
    for i in range(n):
        ox, oy = oracle.elastic_field(79, 3 + i, H, W, sigma=6.0, alpha=300, radius=18)
        d = np.array(list(recs[i].grid), np.float64)
        ref = oracle.boxes_distort(boxes[off[i]:off[i + 1]], H, W, ox, oy, oracle.grid_table(d[:5], W),
                                   oracle.grid_table(d[5:], H))
        assert np.array_equal(gb[off[i]:off[i + 1]], ref), (i, gb[off[i]:off[i + 1]], ref)
