"""Host runtime on the GPU: the autotuner's choice persisted in its cache file
and reused by a second process without timing, an injected allocation failure
that leaves the context usable, and the context's counters."""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIZES = [(1, 1), (300, 41), (129, 1000), (224, 224), (57, 91), (640, 480), (1024, 128), (77, 513)]


@pytest.fixture(scope="module")
def m(dev):
    import paper_1809_06839_amd as m
    m.lib()
    return m


def _batch(m):
    b = synth.ragged_batch(31, len(SIZES), sizes=SIZES)
    flags, ab = m.sample_d4bc(31, 0, b.n)
    return b, flags, ab


SECOND = r"""
import json, sys
sys.path.insert(0, %(root)r)
import paper_1809_06839_amd as m, synth
b = synth.ragged_batch(31, %(n)d, sizes=%(sizes)r)
flags, ab = m.sample_d4bc(31, 0, b.n)
ctx = m.Context(0, tune_cache=%(path)r)
r = m.Ragged.from_host(b, flags, ab)
v, ms = m.ragged_autotune(ctx, r, reps=1)
print(json.dumps({"variant": v, "ms": ms, "stats": ctx.stats()}))
"""


def test_autotune_choice_is_persisted_and_reused_by_a_second_process(m, tmp_path):
    path = str(tmp_path / "tune.json")
    b, flags, ab = _batch(m)
    ctx = m.Context(0, tune_cache=path)
    r = m.Ragged.from_host(b, flags, ab)
    v, ms = m.ragged_autotune(ctx, r, reps=1)
    st = ctx.stats()
    assert st["tune_runs"] == 1 and st["tune_cache_hits"] == 0 and st["variant"] == v
    assert os.path.exists(path)
    ctx.close()
    code = SECOND % {"root": ROOT, "n": len(SIZES), "sizes": SIZES, "path": path}
    print("second process", flush=True)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    import json
    out = json.loads(res.stdout.strip().splitlines()[-1])
    assert out["variant"] == v and out["stats"]["tune_cache_hits"] == 1 and out["stats"]["tune_runs"] == 0
    assert out["ms"] == pytest.approx(ms, rel=1e-5)


def test_injected_allocation_failure_leaves_the_context_usable(m):
    import torch
    b, flags, ab = _batch(m)
    ctx = m.Context(0)
    p = m.Pipeline(ctx, [m.op("HFLIP", 0.5), m.op("ROT90", 1, (0,), (3,)),
                         m.op("BRIGHT_CONTRAST", 1, (0.8, -51), (1.2, 51)), m.op("RESIZE", out=(224, 224)),
                         m.op("NORMALIZE", 1, m.IMAGENET_MEAN, m.IMAGENET_STD)])
    recs = p.sample(5, 0, b.n)
    flags = np.array([[recs[i].flags[k] for k in range(4)] for i in range(b.n)], np.int32)
    ab = np.array([[recs[i].alpha, recs[i].beta] for i in range(b.n)], np.float32)
    r = m.Ragged.from_host(b, flags, ab)
    bi, bo, _ = p.batch(ragged=r)
    m.debug_fail_alloc_after(0)  # the next allocation (the pipeline's staging) fails
    with pytest.raises(m.MiaugError) as e:
        p.apply(bi, bo, recs)
    assert e.value.status == m.ENOMEM
    r.out.fill_(-1.0)
    p.apply(bi, bo, recs)  # the same pipeline and context, now allocating normally
    m.ragged_apply(ctx, r)
    torch.cuda.synchronize()
    out, om = r.out.cpu().numpy(), r.out_mask.cpu().numpy()
    for i in range(b.n):
        ref, rm, _ = oracle.pipe_ragged_one(b.image(i), b.mask_of(i), flags[i], ab[i], b.boxes_of(i), 224, 224)
        assert np.array_equal(out[i].view(np.uint32), ref.view(np.uint32)), i
        assert np.array_equal(om[i], rm), i
    m.debug_fail_alloc_after(0)  # a context that cannot get its counters is not created
    with pytest.raises(m.MiaugError) as e:
        m.Context(0)
    assert e.value.status == m.ENOMEM
    p.close()
    ctx.close()


def test_context_counters(m):
    b, flags, ab = _batch(m)
    ctx = m.Context(0)
    r = m.Ragged.from_host(b, flags, ab)
    m.ragged_apply(ctx, r)
    m.ragged_apply(ctx, r)
    m.ragged_apply_per_image(ctx, r)
    ctx.set_variant(1)
    st = ctx.stats()
    assert st["launches"] == 3 and st["calls"] == 4 and st["errors"] == 0 and st["variant"] == 1
    assert st["last_status"] == 0
