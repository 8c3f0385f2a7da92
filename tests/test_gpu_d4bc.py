"""GPU parity of the plain Dih4 + brightness/contrast kernel against the oracle
(bit-exact u8), called through the C ABI."""
import itertools

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


def run(m, imgs_np, flags, ab):
    import torch
    img = torch.from_numpy(imgs_np).cuda()
    out = m.d4_bc_u8(img, torch.from_numpy(flags).cuda(), torch.from_numpy(ab).cuda())
    torch.cuda.synchronize()
    return out.cpu().numpy()


def oracle_batch(imgs, flags, ab):
    n, H, W, C = imgs.shape
    outs = []
    for i in range(n):
        o = oracle.apply_lut(oracle.d4(imgs[i], *flags[i]), oracle.bc_lut(*ab[i]))
        outs.append(o.reshape(-1))
    return np.stack(outs)


def test_small_plain_config_bit_exact(m):
    # 64 RGB images 256x256, pixels U[0,255], parameters from the sampler
    imgs = synth.uniform_u8(1809068391, 64, 256, 256).numpy()
    flags, ab = m.sample_d4bc(1809068391, 0, 64)
    got = run(m, imgs, flags, ab).reshape(64, -1)
    assert np.array_equal(got, oracle_batch(imgs, flags, ab))


@pytest.mark.parametrize("shape", [(2, 37, 53, 3), (2, 70, 130, 1), (2, 1, 7, 4), (1, 129, 65, 3), (1, 5, 1, 3),
                                   (1, 1, 1, 3), (1, 200, 3, 4)])
def test_all_dih4_elements_odd_shapes(m, shape):
    n, H, W, C = shape
    rng = np.random.default_rng(H * 1000 + W)
    combos = list(itertools.product((0, 1), (0, 1), range(4), (0, 1)))
    imgs = rng.integers(0, 256, (len(combos) * n, H, W, C), dtype=np.uint8)
    flags = np.array([c for c in combos for _ in range(n)], np.int32)
    ab = np.stack([rng.uniform(0.8, 1.2, len(flags)), rng.uniform(-51, 51, len(flags))], 1).astype(np.float32)
    got = run(m, imgs, flags, ab).reshape(len(flags), -1)
    assert np.array_equal(got, oracle_batch(imgs, flags, ab))


def test_empty_batch_is_a_no_op(m):
    import torch
    img = torch.zeros((0, 8, 8, 3), dtype=torch.uint8, device="cuda")
    out = m.d4_bc_u8(img, torch.zeros((0, 4), dtype=torch.int32, device="cuda"),
                     torch.zeros((0, 2), dtype=torch.float32, device="cuda"))
    assert out.shape == (0, 8, 8, 3)
