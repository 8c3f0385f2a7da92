"""GPU parity of the differentiable warp + colour op: the float32 forward
against the fp64 oracle (|y - y_ref| <= 1e-5 max(1, |y_ref|)), the HIP backward
against the oracle's analytic fp64 adjoint (image gradient within 1e-4 of
max|g_ref|; each parameter gradient within 1e-4 (|g_ref| + median |g_ref|)
over the batch: a float32 sum of ~150 K terms that nearly cancel has no
relative bound, the median sets its scale), and torch.autograd plumbing.  The
full-size test checks all 128 images and prints the errors reached, pure
relative ones included."""
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


def compare(m, x, p, w, check_gx=True, n_check=None):
    """Checks the HIP forward and backward against the oracle on images n_check
    (default all) and returns the errors reached: forward max |dy| and max
    |dy| / |y_ref| over |y_ref| >= 1e-3; grad_x max |dg| / max |g_ref| per
    image; parameter gradients max |dg| / |g_ref| (pure relative) and max of
    |dg| / (|g_ref| + median |g_ref|) (the mixed bar)."""
    import torch
    xt, pt, wt = (torch.from_numpy(a).cuda() for a in (x, p, w))
    y = m.warpcolor_fwd(xt, pt)
    gx, gp = m.warpcolor_bwd(xt, pt, wt)
    torch.cuda.synchronize()
    y, gx, gp = y.cpu().numpy(), gx.cpu().numpy(), gp.cpu().numpy()
    n = x.shape[0]
    idx = range(n) if n_check is None else n_check
    ref_gp = np.zeros((n, 7))
    st = {"fwd_abs": 0.0, "fwd_rel": 0.0, "gx_rel_to_max": 0.0}
    for i in idx:
        yr = oracle.wc_forward(x[i], p[i].astype(np.float64))
        d = np.abs(y[i] - yr)
        assert np.all(d <= 1e-5 * np.maximum(1.0, np.abs(yr))), ("forward", i)
        big = np.abs(yr) >= 1e-3
        st["fwd_abs"] = max(st["fwd_abs"], float(d.max()))
        st["fwd_rel"] = max(st["fwd_rel"], float((d[big] / np.abs(yr[big])).max()) if big.any() else 0.0)
        gxr, gpr = oracle.wc_backward(x[i], p[i].astype(np.float64), w[i].astype(np.float64), want_gx=check_gx)
        ref_gp[i] = gpr
        if check_gx:
            e = np.abs(gx[i] - gxr).max() / max(np.abs(gxr).max(), 1e-300)
            st["gx_rel_to_max"] = max(st["gx_rel_to_max"], float(e))
            assert e <= 1e-4, ("grad_x", i, e)
    idx = list(idx)
    med = np.median(np.abs(ref_gp[idx]), axis=0)
    err = np.abs(gp[idx] - ref_gp[idx])
    tol = 1e-4 * (np.abs(ref_gp[idx]) + med)
    st["gp_mixed"] = float((err / np.maximum(tol, 1e-300)).max()) * 1e-4
    st["gp_rel"] = float((err / np.maximum(np.abs(ref_gp[idx]), 1e-300)).max())
    st["gp_rel_over_1e-4"] = int((err > 1e-4 * np.abs(ref_gp[idx])).sum())
    assert np.all(err <= tol), (err / np.maximum(tol, 1e-30)).max()
    return st


def test_small_batch_matches_oracle(m):
    n, C, H, W = 6, 3, 40, 36
    x = synth.smooth_noise(11, n, H, W, C).numpy()
    p = m.sample_wc(11, 0, n)
    w = np.random.default_rng(1).uniform(-1, 1, (n, C, H, W)).astype(np.float32)
    compare(m, x, p, w)


@pytest.mark.parametrize("C,H,W", [(1, 17, 29), (4, 33, 8), (3, 1, 5), (2, 64, 65), (4, 31, 45), (1, 48, 64),
                                   (3, 50, 52)])
def test_odd_shapes_and_channel_counts(m, C, H, W):
    n = 3
    x = synth.smooth_noise(C * H * W, n, H, W, C).numpy()
    p = m.sample_wc(C + H, 0, n)
    p[0] = [0.0, 1.0, 0.0, 0.0, 1.0, 0.0, 1.0]  # identity
    w = np.random.default_rng(2).uniform(-1, 1, (n, C, H, W)).astype(np.float32)
    compare(m, x, p, w)


def test_far_scales_take_the_other_kernel_forms(m):
    # a zoom-out whose source footprint is too wide for the LDS box (the forward
    # and parameter kernels then gather from global memory) and zoom-ins whose
    # adjoint region exceeds the sorted LDS entries (scatter form)
    n, C, H, W = 4, 3, 80, 72
    x = synth.smooth_noise(21, n, H, W, C).numpy()
    p = m.sample_wc(21, 0, n)
    p[:, 1] = [0.4, 0.6, 1.7, 2.5]
    w = np.random.default_rng(3).uniform(-1, 1, (n, C, H, W)).astype(np.float32)
    compare(m, x, p, w)


def test_forward_same_from_an_unaligned_base(m):
    # rows are staged as 16-byte chunks only when the planes start 16-byte
    # aligned and W is a multiple of 4; a base 4 bytes off takes the 4-byte
    # form, which must give the same bits
    import torch
    n, C, H, W = 5, 3, 96, 100
    x = synth.smooth_noise(31, n, H, W, C).cuda()
    p = torch.from_numpy(m.sample_wc(31, 0, n)).cuda()
    buf = torch.empty(x.numel() + 1, device="cuda")
    xu = buf[1:].view(n, C, H, W)
    xu.copy_(x)
    assert xu.data_ptr() % 16 != 0
    assert torch.equal(m.warpcolor_fwd(xu, p), m.warpcolor_fwd(x, p))


def test_identity_forward_is_exact(m):
    import torch
    x = synth.smooth_noise(3, 2, 20, 24, 3).cuda()
    p = torch.tensor([[0.0, 1.0, 0.0, 0.0, 1.0, 0.0, 1.0]] * 2, device="cuda")
    assert torch.equal(m.warpcolor_fwd(x, p), x)


def test_full_size_batch_all_images(m):
    # 128 x 3 x 224 x 224 float32 in [0, 1], loss weights U[-1, 1]
    import torch
    n, C, H, W = 128, 3, 224, 224
    x = synth.smooth_noise(1809068394, n, H, W, C, device="cuda")
    p = m.sample_wc(1809068394, 0, n)
    g = torch.Generator().manual_seed(5)
    w = (torch.rand((n, C, H, W), generator=g) * 2 - 1)
    st = compare(m, x.cpu().numpy(), p, w.numpy(), check_gx=True)
    print("\nwarpcolor parity, 128 x 3 x 224 x 224: " + ", ".join("%s=%.3g" % kv for kv in st.items()))


def test_autograd_function(m):
    import torch
    n, C, H, W = 4, 3, 32, 32
    x = synth.smooth_noise(9, n, H, W, C).cuda().requires_grad_(True)
    p = torch.from_numpy(m.sample_wc(9, 0, n)).cuda().requires_grad_(True)
    w = torch.rand((n, C, H, W), device="cuda") * 2 - 1
    loss = (m.warp_color(x, p) * w).sum()
    loss.backward()
    gx, gp = m.warpcolor_bwd(x.detach(), p.detach(), w)
    # parameter gradients use fixed-order reductions (bit-identical across runs); the
    # image gradient accumulates with LDS float atomics, whose order may vary
    assert torch.equal(p.grad, gp)
    assert (x.grad - gx).abs().max().item() <= 1e-6 * gx.abs().max().item()
