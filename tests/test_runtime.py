"""Host runtime of the library, on the CPU: the autotuner's cache file (round
trip, replacement, escaping, malformed files) and the allocation-failure
injector (one-shot MIAUG_ENOMEM, also armed from MIAUG_FAIL_ALLOC_AFTER)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def m():
    import paper_1809_06839_amd as m
    m.lib()
    return m


def test_tune_cache_round_trip_and_replacement(m, tmp_path):
    path = str(tmp_path / "tune.json")
    assert m.tune_cache_lookup(path, "gfx950|ragged|o224x224") is None  # no file yet
    m.tune_cache_store(path, "gfx950|ragged|o224x224", 17, "wave row gathers", 0.75)
    m.tune_cache_store(path, "gfx950|ragged|o64x64", 3, "tile 32x32", 0.125)
    assert m.tune_cache_lookup(path, "gfx950|ragged|o224x224") == (17, pytest.approx(0.75), "wave row gathers")
    assert m.tune_cache_lookup(path, "gfx950|ragged|o64x64") == (3, pytest.approx(0.125), "tile 32x32")
    m.tune_cache_store(path, "gfx950|ragged|o224x224", 5, "other", 1.5)  # replaces, keeps the other key
    assert m.tune_cache_lookup(path, "gfx950|ragged|o224x224") == (5, pytest.approx(1.5), "other")
    assert m.tune_cache_lookup(path, "gfx950|ragged|o64x64")[0] == 3
    doc = json.load(open(path))  # the file is plain JSON
    assert doc["version"] == 1 and len(doc["entries"]) == 2
    assert not [f for f in os.listdir(tmp_path) if ".tmp" in f]  # no temporary left behind


def test_tune_cache_escapes_and_tolerates_unknown_fields(m, tmp_path):
    path = str(tmp_path / "tune.json")
    key = 'arch "x"\\y|ragged'
    m.tune_cache_store(path, key, 2, 'name with "quotes"', 0.5)
    assert json.load(open(path))["entries"][0]["key"] == key
    assert m.tune_cache_lookup(path, key) == (2, pytest.approx(0.5), 'name with "quotes"')
    doc = {"version": 1, "comment": [1, {"a": None}], "entries": [
        {"key": "k", "variant": 4, "ms": 2.0, "name": "n", "extra": {"x": [True, False]}}]}
    open(path, "w").write(json.dumps(doc))
    assert m.tune_cache_lookup(path, "k") == (4, pytest.approx(2.0), "n")


@pytest.mark.parametrize("text", ["", "not json", '{"entries": [', '{"entries": [{"key": 1}]}', "[1, 2]",
                                  '{"entries": [{"key": "k", "variant": -3}]}'])
def test_tune_cache_malformed_file_is_reported_then_replaced(m, tmp_path, text):
    path = str(tmp_path / "tune.json")
    open(path, "w").write(text)
    with pytest.raises(m.MiaugError) as e:
        m.tune_cache_lookup(path, "k")
    assert e.value.status == m.EINVAL
    m.tune_cache_store(path, "k", 1, "one", 0.25)
    assert m.tune_cache_lookup(path, "k") == (1, pytest.approx(0.25), "one")


def test_alloc_failure_injector_is_one_shot(m):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible (the GPU test covers this)")
    # without a device the allocator reports EDEVICE; an armed failure comes first
    assert m.lib().miaug_debug_alloc_probe(4096) == m.EDEVICE
    m.debug_fail_alloc_after(1)
    assert m.lib().miaug_debug_alloc_probe(4096) == m.EDEVICE  # allocation 0 passes on
    assert m.lib().miaug_debug_alloc_probe(4096) == m.ENOMEM   # allocation 1 is the armed one
    assert "injected" in m.lib().miaug_last_error().decode()
    assert m.lib().miaug_debug_alloc_probe(4096) == m.EDEVICE  # disarmed again
    m.debug_fail_alloc_after(-1)


def test_alloc_failure_injector_from_the_environment():
    code = ("import paper_1809_06839_amd as m; L = m.lib(); "
            "print(L.miaug_debug_alloc_probe(64), L.miaug_debug_alloc_probe(64), L.miaug_debug_alloc_probe(64))")
    env = dict(os.environ, MIAUG_FAIL_ALLOC_AFTER="1", MIAUG_LOG="2", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    first, second, third = (int(v) for v in r.stdout.split())
    assert second == -5 and first != -5 and third != -5  # MIAUG_ENOMEM once, at allocation 1
    assert "injected allocation failure" in r.stderr      # MIAUG_LOG=2 reports it
