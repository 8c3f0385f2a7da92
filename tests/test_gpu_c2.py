"""GPU parity of the full u8 pipeline (shift-scale-rotate -> crop -> resize ->
HSV shift -> gamma -> blur) against the oracle, bit-exact, called through the
C ABI; parameters from the library's sampler and host compile."""
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


def run(m, imgs, f, k, crop, outsz):
    import torch
    n, H, W, _ = imgs.shape
    rec = torch.from_numpy(m.compile_c2(f, k, H, W, crop)).cuda()
    out = m.ssr_crop_resize_hsv_gamma_blur_u8(torch.from_numpy(imgs).cuda(), rec, crop, outsz)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(imgs, f, k, crop, outsz, got, idx=None):
    n, H, W, _ = imgs.shape
    for i in (range(n) if idx is None else idx):
        kk = k[i].copy()
        kk[0] = min(max(kk[0], 0), W - crop); kk[1] = min(max(kk[1], 0), H - crop)
        ref = oracle.pipe_c2_one(imgs[i], f[i], kk, crop, outsz)
        assert np.array_equal(got[i], ref), ("image", i, f[i], k[i])


def test_small_batch_sampled_parameters(m):
    imgs = synth.smooth_u8_hwc(3, 12, 96, 80).numpy()
    f, k = m.sample_c2(3, 0, 12, crop_range=16)
    got = run(m, imgs, f, k, 64, 40)
    check(imgs, f, k, 64, 40, got)


@pytest.mark.parametrize("angle,scale,dx,dy", [(90.0, 1.0, 0.0, 0.0), (180.0, 1.0, 0.0, 0.0), (45.0, 0.9, 0.0625, -0.0625),
                                               (-45.0, 1.1, -0.0625, 0.0625), (0.0, 1.0, 0.0, 0.0), (13.7, 0.95, 0.01, 0.02)])
def test_edge_parameters_and_both_blur_states(m, angle, scale, dx, dy):
    rng = np.random.default_rng(int(abs(angle) * 10 + scale * 100))
    imgs = rng.integers(0, 256, (4, 70, 70, 3), dtype=np.uint8)
    f = np.array([[angle, scale, dx, dy, g] for g in (0.8, 1.0, 1.2, 0.93)], np.float32)
    k = np.array([[0, 0, 20, 30, 1], [6, 3, -20, -30, 0], [6, 6, 0, 0, 1], [2, 5, 180, 7, 0]], np.int32)
    got = run(m, imgs, f, k, 64, 64)
    check(imgs, f, k, 64, 64, got)


@pytest.mark.parametrize("H,W,crop,outsz", [(33, 47, 20, 50), (64, 64, 64, 1), (100, 37, 37, 19), (129, 131, 128, 96)])
def test_shapes_tails_and_upsampling(m, H, W, crop, outsz):
    imgs = synth.smooth_u8_hwc(H * W, 3, H, W).numpy()
    f, k = m.sample_c2(H + W, 0, 3, crop_range=max(H, W))
    got = run(m, imgs, f, k, crop, outsz)
    check(imgs, f, k, crop, outsz, got)


def test_full_size_batch_sampled_against_oracle(m):
    # 256 smooth-noise images 512x512 -> crop 448 -> 224, as the bench launches it
    import torch
    imgs_t = synth.smooth_u8_hwc(1809068392, 256, 512, 512, device="cuda")
    f, k = m.sample_c2(1809068392, 0, 256)
    rec = torch.from_numpy(m.compile_c2(f, k, 512, 512, 448)).cuda()
    out = m.ssr_crop_resize_hsv_gamma_blur_u8(imgs_t, rec, 448, 224)
    torch.cuda.synchronize()
    imgs = imgs_t.cpu().numpy()
    got = out.cpu().numpy()
    rng = np.random.default_rng(8)
    check(imgs, f, k, 448, 224, got, sorted(rng.choice(256, 10, replace=False)))


# ---------------------------------------------------------------- masks and boxes of the u8 chain
def rand_boxes(rng, n, H, W, per=(0, 9)):
    counts = rng.integers(per[0], per[1], n)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    x1 = rng.uniform(-5, W, off[-1]); y1 = rng.uniform(-5, H, off[-1])
    bx = np.stack([x1, y1, x1 + rng.uniform(0.5, W / 2, off[-1]), y1 + rng.uniform(0.5, H / 2, off[-1])], 1)
    return bx.astype(np.float32), off


@pytest.mark.parametrize("H,W,crop,outsz", [(96, 80, 64, 40), (70, 70, 70, 70), (61, 130, 50, 96), (512, 512, 448, 224)])
def test_masks_and_boxes_follow_the_image_geometry(m, H, W, crop, outsz):
    import torch
    rng = np.random.default_rng(H * 1000 + W)
    n = 6
    masks = np.ascontiguousarray(synth.blob_masks(H * 7 + W, n, H, W, 8, 16).numpy())
    f, k = m.sample_c2(H + W, 0, n, crop_range=max(1, min(H, W) - crop + 1))
    f[0] = (90.0, 1.0, 0.0, 0.0, 1.0)
    f[1] = (0.0, 1.0, 0.0, 0.0, 1.0)
    rec = torch.from_numpy(m.compile_c2(f, k, H, W, crop)).cuda()
    om = m.ssr_crop_resize_mask_u8(torch.from_numpy(masks).cuda(), rec, crop, outsz)
    bx, off = rand_boxes(rng, n, H, W)
    ob = m.boxes_ssr_crop_resize(torch.from_numpy(bx).cuda(), torch.from_numpy(off).cuda(), H, W, rec, crop, outsz)
    torch.cuda.synchronize()
    om, ob = om.cpu().numpy(), ob.cpu().numpy()
    for i in range(n):
        kx, ky = min(max(int(k[i][0]), 0), W - crop), min(max(int(k[i][1]), 0), H - crop)
        aq = oracle.ssr_matrix_q32(*f[i][:4], H, W)
        ref = oracle.resize(oracle.crop(oracle.warp_affine(masks[i], aq, oracle.NEAREST), kx, ky, crop, crop),
                            outsz, outsz, oracle.NEAREST)
        assert np.array_equal(om[i], ref), ("mask", i)
        rb = oracle.boxes_ssr_crop_resize(bx[off[i]:off[i + 1]], H, W, f[i][:4], kx, ky, crop, outsz)
        got = ob[off[i]:off[i + 1]]
        assert np.all(np.abs(got - rb) <= 1e-5 * np.maximum(1.0, np.abs(rb))), ("boxes", i, np.abs(got - rb).max())
