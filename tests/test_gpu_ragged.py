"""GPU parity of the ragged-batch kernels (batched persistent, flat, per-image,
hipGraph, autotuned) against the oracle: bit-exact float32 images (the u8
resize result goes through the same normalisation LUT), bit-exact masks, and
boxes within 1e-5 relative."""
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


@pytest.fixture(scope="module")
def ctx(m):
    return m.Context(0)


SMALL_SIZES = [(1, 1), (1, 300), (300, 1), (2, 3), (128, 1024), (1024, 128), (224, 224), (223, 225), (57, 91),
               (449, 448), (1000, 999), (150, 700), (31, 17), (640, 480), (333, 77), (96, 96), (512, 900),
               (129, 130), (7, 400), (260, 261), (40, 2500), (2500, 40)]


def oracle_image(b, i, flags, ab, OH=224, OW=224):
    return oracle.pipe_ragged_one(b.image(i), b.mask_of(i), flags[i], ab[i], b.boxes_of(i), OH, OW)


def check_outputs(m, b, r, flags, ab, idx, OH=224, OW=224):
    out = r.out.cpu().numpy()
    om = r.out_mask.cpu().numpy()
    ob = r.out_boxes.cpu().numpy() if r.out_boxes is not None else None
    for i in idx:
        ref, rm, rb = oracle_image(b, i, flags, ab, OH, OW)
        assert np.array_equal(out[i].view(np.uint32), ref.view(np.uint32)), ("image", i, tuple(b.hw[i]), flags[i])
        assert np.array_equal(om[i], rm), ("mask", i, tuple(b.hw[i]))
        if len(rb):
            got = ob[b.box_off[i]:b.box_off[i + 1]]
            assert np.all(np.abs(got - rb) <= 1e-5 * np.maximum(1.0, np.abs(rb))), ("boxes", i)


@pytest.fixture(scope="module")
def small(m):
    b = synth.ragged_batch(11, len(SMALL_SIZES), sizes=SMALL_SIZES)
    flags, ab = m.sample_d4bc(11, 0, len(SMALL_SIZES))
    flags[:8] = [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 2, 0), (0, 0, 3, 0), (0, 0, 0, 1),
                 (1, 1, 1, 1)]
    return b, flags, ab


@pytest.mark.parametrize("variant", range(24))
def test_small_ragged_all_variants_bit_exact(m, ctx, small, variant):
    if variant >= len(m.ragged_variants()):
        pytest.skip("the library has fewer variants")
    if m.ragged_variants()[variant].startswith("off: "):
        pytest.skip("launch form switched off in the library: an intermittent wrong image, cause not found")
    b, flags, ab = small
    ctx.set_variant(variant)
    r = m.Ragged.from_host(b, flags, ab)
    m.ragged_apply(ctx, r)
    check_outputs(m, b, r, flags, ab, range(b.n))
    ctx.set_variant(-1)


def test_small_ragged_per_image_form(m, ctx, small):
    b, flags, ab = small
    r = m.Ragged.from_host(b, flags, ab)
    m.ragged_apply_per_image(ctx, r)
    check_outputs(m, b, r, flags, ab, range(b.n))


def test_other_output_sizes(m, ctx):
    b = synth.ragged_batch(12, 6, sizes=[(50, 70), (300, 20), (1, 1), (64, 64), (99, 1), (200, 333)])
    flags, ab = m.sample_d4bc(12, 0, 6)
    for OH, OW in [(17, 45), (64, 64), (1, 1), (300, 100)]:
        r = m.Ragged.from_host(b, flags, ab, out_h=OH, out_w=OW)
        m.ragged_apply(ctx, r)
        check_outputs(m, b, r, flags, ab, range(b.n), OH, OW)


def test_graph_replays_match_eager(m, ctx, small):
    import torch
    b, flags, ab = small
    r = m.Ragged.from_host(b, flags, ab)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = m.Graph(ctx, r, s)
        for rep in range(4):
            r.out.zero_(); r.out_mask.zero_()
            g.launch(s)
            s.synchronize()
            check_outputs(m, b, r, flags, ab, range(b.n))
    g.close()


# ---------------------------------------------------------------- image and mask starts at any byte offset
@pytest.fixture(scope="module")
def unaligned(m):
    # image and mask i start 1, 7 or 13 bytes past a 256-byte boundary, so the
    # 16-byte chunks the kernels stage straddle each image's first and last byte
    b = synth.ragged_batch(13, len(SMALL_SIZES), sizes=SMALL_SIZES, phases=(1, 7, 13))
    assert set(int(o) % 16 for o in b.img_off) == {1, 7, 13}
    assert set(int(o) % 16 for o in b.mask_off) == {1, 7, 13}
    flags, ab = m.sample_d4bc(13, 0, len(SMALL_SIZES))
    flags[:8] = [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 2, 0), (0, 0, 3, 0), (0, 0, 0, 1),
                 (1, 1, 1, 1)]
    return b, flags, ab


@pytest.mark.parametrize("variant", range(24))
def test_unaligned_starts_all_variants_bit_exact(m, ctx, unaligned, variant):
    if variant >= len(m.ragged_variants()):
        pytest.skip("the library has fewer variants")
    if m.ragged_variants()[variant].startswith("off: "):
        pytest.skip("launch form switched off in the library: an intermittent wrong image, cause not found")
    b, flags, ab = unaligned
    ctx.set_variant(variant)
    r = m.Ragged.from_host(b, flags, ab)
    m.ragged_apply(ctx, r)
    check_outputs(m, b, r, flags, ab, range(b.n))
    win = crop_windows(b, flags, 79)
    rc = m.Ragged.from_host(b, flags, ab, crop=win)
    m.ragged_apply(ctx, rc)
    check_crop_outputs(b, rc, flags, ab, win, range(b.n))
    ctx.set_variant(-1)


def test_unaligned_starts_per_image_and_graph(m, ctx, unaligned):
    import torch
    b, flags, ab = unaligned
    r = m.Ragged.from_host(b, flags, ab)
    m.ragged_apply_per_image(ctx, r)
    check_outputs(m, b, r, flags, ab, range(b.n))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = m.Graph(ctx, r, s)
        for rep in range(3):
            r.out.zero_(); r.out_mask.zero_()
            g.launch(s)
            s.synchronize()
            check_outputs(m, b, r, flags, ab, range(b.n))
    g.close()


def test_empty_ragged_batch(m, ctx):
    import torch
    z = lambda *s, dt=torch.int32: torch.zeros(s, dtype=dt, device="cuda")
    r = m.Ragged(z(16, dt=torch.uint8), z(0, dt=torch.int64), z(0, 2), z(0, 4), z(0, 2, dt=torch.float32))
    m.ragged_apply(ctx, r)
    m.ragged_apply_per_image(ctx, r)


def test_full_size_batch_sampled_against_oracle(m, ctx):
    # 2048 images with H, W ~ U{128..1024}, in the launch configuration the bench times
    import torch
    b = synth.ragged_batch(1809068393, 2048, device="cuda")
    flags, ab = m.sample_d4bc(1809068393, 0, 2048)
    r = m.Ragged.from_host(b, flags, ab)
    v, ms = m.ragged_autotune(ctx, r, reps=2)
    r.out.zero_()
    m.ragged_apply(ctx, r)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    check_outputs(m, b, r, flags, ab, sorted(rng.choice(2048, 48, replace=False)))
    # batched == per-image on every image
    out_b = r.out.clone(); m_b = r.out_mask.clone()
    m.ragged_apply_per_image(ctx, r)
    torch.cuda.synchronize()
    assert torch.equal(out_b, r.out) and torch.equal(m_b, r.out_mask)


# ---------------------------------------------------------------- crop windows (random-sized crop)
def d4_shape(h, w, fl):
    swap = (int(fl[2]) & 1) != int(fl[3] != 0)
    return (w, h) if swap else (h, w)


def crop_windows(b, flags, seed, scale=(0.08, 1.0), ratio=(0.75, 4 / 3)):
    win = np.zeros((b.n, 4), np.int32)
    for i in range(b.n):
        H, W = d4_shape(int(b.hw[i][0]), int(b.hw[i][1]), flags[i])
        win[i] = oracle.sized_crop_window(seed, i, 1, H, W, scale, ratio)
    return win


def check_crop_outputs(b, r, flags, ab, win, idx, OH=224, OW=224):
    out, om = r.out.cpu().numpy(), r.out_mask.cpu().numpy()
    ob = r.out_boxes.cpu().numpy() if r.out_boxes is not None else None
    for i in idx:
        ref, rm, rb = oracle.pipe_ragged_one(b.image(i), b.mask_of(i), flags[i], ab[i], b.boxes_of(i), OH, OW,
                                             win=win[i])
        assert np.array_equal(out[i].view(np.uint32), ref.view(np.uint32)), ("image", i, tuple(win[i]))
        assert np.array_equal(om[i], rm), ("mask", i, tuple(win[i]))
        if len(rb):
            got = ob[b.box_off[i]:b.box_off[i + 1]]
            assert np.all(np.abs(got - rb) <= 1e-5 * np.maximum(1.0, np.abs(rb))), ("boxes", i)


@pytest.mark.parametrize("variant", range(24))
def test_crop_windows_all_variants_bit_exact(m, ctx, small, variant):
    if variant >= len(m.ragged_variants()):
        pytest.skip("the library has fewer variants")
    if m.ragged_variants()[variant].startswith("off: "):
        pytest.skip("launch form switched off in the library: an intermittent wrong image, cause not found")
    b, flags, ab = small
    win = crop_windows(b, flags, 77)
    win[3] = (0, 0, *d4_shape(int(b.hw[3][0]), int(b.hw[3][1]), flags[3]))  # the whole image
    ctx.set_variant(variant)
    r = m.Ragged.from_host(b, flags, ab, crop=win)
    m.ragged_apply(ctx, r)
    check_crop_outputs(b, r, flags, ab, win, range(b.n))
    ctx.set_variant(-1)


def test_crop_window_per_image_form_and_skips(m, ctx, small):
    import torch
    b, flags, ab = small
    win = crop_windows(b, flags, 78, scale=(0.3, 0.9))
    win[5, 2] = 0          # h = 0: no window for image 5
    bad = [1, 6]
    win[1] = (0, 0, 2, 400)  # wider than the image
    win[6] = (-1, 0, 1, 1)   # negative offset
    r = m.Ragged.from_host(b, flags, ab, crop=win)
    r.out.fill_(7.0); r.out_mask.fill_(9)
    m.ragged_apply_per_image(ctx, r)
    torch.cuda.synchronize()
    full = [i for i in range(b.n) if i not in bad]
    w2 = win.copy(); w2[5] = (0, 0, *d4_shape(int(b.hw[5][0]), int(b.hw[5][1]), flags[5]))
    check_crop_outputs(b, r, flags, ab, w2, full)
    out, om = r.out.cpu().numpy(), r.out_mask.cpu().numpy()
    for i in bad:  # skipped images: outputs untouched
        assert np.all(out[i] == 7.0) and np.all(om[i] == 9), i


def test_autotune_gate_with_skipped_images(m, small):
    # images whose window is invalid are skipped (outputs untouched) by every
    # form alike, so every variant passes the parity gate
    b, flags, ab = small
    win = crop_windows(b, flags, 78, scale=(0.3, 0.9))
    win[1] = (0, 0, 2, 400)
    win[6] = (-1, 0, 1, 1)
    c2 = m.Context(0)
    r = m.Ragged.from_host(b, flags, ab, crop=win)
    v, ms, times = m.ragged_autotune(c2, r, reps=1, return_times=True)
    names = m.ragged_variants()
    assert all((t > 0) != names[i].startswith("off: ") for i, t in enumerate(times)), times  # off: -1
    full = [i for i in range(b.n) if i not in (1, 6)]
    m.ragged_apply(c2, r)
    check_crop_outputs(b, r, flags, ab, win, full)
    c2.close()


def test_full_size_batch_with_crop_windows_sampled_against_oracle(m, ctx):
    import torch
    b = synth.ragged_batch(1809068394, 2048, device="cuda")
    flags, ab = m.sample_d4bc(1809068394, 0, 2048)
    win = crop_windows(b, flags, 1809068394)
    r = m.Ragged.from_host(b, flags, ab, crop=win)
    m.ragged_apply(ctx, r)
    torch.cuda.synchronize()
    rng = np.random.default_rng(6)
    check_crop_outputs(b, r, flags, ab, win, sorted(rng.choice(2048, 32, replace=False)))


# ---------------------------------------------------------------- multi-channel instance masks
@pytest.mark.parametrize("K", [1, 3, 7])
def test_multichannel_instance_masks_follow_the_one_channel_masks(m, ctx, small, K):
    import torch
    b, flags, ab = small
    win = crop_windows(b, flags, 80 + K)
    win[::3, 2] = 0  # no window for every third image
    parts, offs, o = [], [], 0
    for i in range(b.n):
        lab = b.mask_of(i)
        mc = np.stack([(lab % K == k).astype(np.uint8) * (k + 1) for k in range(K)], -1)  # instance k -> value k + 1
        parts.append(mc.reshape(-1)); offs.append(o); o += mc.size
    packed = np.concatenate(parts) if parts else np.zeros(1, np.uint8)
    r = m.Ragged.from_host(b, flags, ab, crop=win, out_h=48, out_w=40)
    r1 = m.Ragged(r.keep[0], r.keep[1], r.keep[2], r.keep[3], r.keep[4], out_h=48, out_w=40,
                  mask=torch.from_numpy(packed).cuda(), mask_off=torch.tensor(offs, dtype=torch.int64).cuda(),
                  crop=r.keep[9])
    got = m.ragged_masks_u8(r1, K).cpu().numpy()
    for i in range(b.n):
        H, W = int(b.hw[i][0]), int(b.hw[i][1])
        mc = parts[i].reshape(H, W, K)
        d = oracle.d4(mc, *flags[i])
        if win[i][2]:
            y0, x0, h, w = (int(v) for v in win[i])
            d = oracle.crop(d, x0, y0, h, w)
        ref = oracle.resize(d, 48, 40, oracle.NEAREST)
        assert np.array_equal(got[i], ref), (i, K)
    if K == 1:  # on the real one-channel labels: the same pixels as the fused kernel's masks
        m.ragged_apply(ctx, r)
        torch.cuda.synchronize()
        assert torch.equal(m.ragged_masks_u8(r, 1)[..., 0], r.out_mask)
