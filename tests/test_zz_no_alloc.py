"""The no-allocation ragged entry point (static device counters) against
miaug_ragged_apply: bit-identical outputs on two calls in a row, the second
with a smaller batch, on the default and a second launch variant."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def m(dev):
    import paper_1809_06839_amd as m
    m.lib()
    return m


def _fill(r):
    r.out.fill_(-7.0)
    r.out_mask.fill_(0xA5)
    if r.out_boxes is not None:
        r.out_boxes.fill_(-9.0)


def _same(a, b):
    assert torch.equal(a.out.view(torch.int32), b.out.view(torch.int32))
    assert torch.equal(a.out_mask, b.out_mask)
    if a.out_boxes is not None:
        assert torch.equal(a.out_boxes.view(torch.int32), b.out_boxes.view(torch.int32))


@pytest.mark.parametrize("variant", [-1, 4])
def test_noalloc_matches_ctx_form_two_calls(m, variant):
    ctx = m.Context(0)
    if variant >= 0:
        ctx.set_variant(variant)
    big = synth.ragged_batch(71, 40, sizes=None, lo=128, hi=700)
    small = synth.ragged_batch(72, 5, sizes=[(1, 1), (300, 40), (224, 224), (77, 513), (640, 129)])
    for b, seed in ((big, 71), (small, 72)):
        flags, ab = m.sample_d4bc(seed, 0, b.n)
        print("noalloc: variant", variant, "n", b.n, flush=True)
        ref = m.Ragged.from_host(b, flags, ab)
        got = m.Ragged.from_host(b, flags, ab)
        _fill(ref)
        _fill(got)
        m.ragged_apply(ctx, ref)
        m.ragged_apply_noalloc(got, variant)
        torch.cuda.synchronize()
        _same(ref, got)
    ctx.close()


def test_noalloc_rejects_bad_variant(m):
    b = synth.ragged_batch(73, 2, sizes=[(10, 10), (20, 30)])
    flags, ab = m.sample_d4bc(73, 0, b.n)
    r = m.Ragged.from_host(b, flags, ab)
    with pytest.raises(m.MiaugError):
        m.ragged_apply_noalloc(r, 10 ** 6)
