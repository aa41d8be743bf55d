"""GPU checks of the autotuner: it records one of its candidate choices per
(length, window) bucket, applying the cache changes no result, and the cache
survives a save/load round trip."""
import json

import numpy as np
import pytest
import torch

import gen
import paper_2010_05371_amd as eap

pytestmark = pytest.mark.gpu


@pytest.fixture
def autotune_on():
    old = eap.get_option("autotune")
    eap.set_option("autotune", 1)
    yield
    eap.set_option("autotune", old)


@pytest.mark.parametrize("m,w", [(128, 0), (128, 13), (256, 52), (300, 100), (200, 199)])
def test_autotune_choice_and_same_results(m, w, autotune_on):
    g = gen.rng(4100, m + w)
    x = torch.from_numpy(gen.as_f32(gen.random_walk(100_000, g))).cuda()
    q = torch.from_numpy(gen.as_f32(gen.random_walk(m, g))).cuda()
    eap.set_option("autotune", 0)
    plain = eap.nn_search(q, x, w)
    t = eap.autotune(q, x, w, sample_n=30_000)
    assert t["ms"] > 0 and t["rows_per_group"] in (0, 2, 4, 8) and t["border"] in (0, 1)
    assert t["check_interval"] in (0, 1, 4) and t["wide_rows"] in (0, 32, 64)
    assert t["lanes"] in (0, 1) and (t["lanes"] == 0 or (m % 4 == 0 and 1 <= min(w, m - 1) <= 64))
    assert eap.tune_get(m, w) == t
    eap.set_option("autotune", 1)
    assert eap.nn_search(q, x, w) == plain
    d_plain = None
    eap.set_option("autotune", 0)
    d_plain = eap.nn_dists(q, x[:20_000], w).cpu().numpy()
    eap.set_option("autotune", 1)
    d_tuned = eap.nn_dists(q, x[:20_000], w).cpu().numpy()
    assert np.array_equal(d_plain.view(np.uint32), d_tuned.view(np.uint32))


def test_batch_autotune_same_results(autotune_on):
    g = gen.rng(4101)
    x = torch.from_numpy(gen.as_f32(gen.random_walk(60_000, g))).cuda()
    qs = [(torch.from_numpy(gen.as_f32(gen.random_walk(m, g))).cuda(), w)
          for m, w in ((64, 4), (150, 30), (400, 70), (90, 0), (333, 50))]
    eap.set_option("autotune", 0)
    plain = eap.nn_search_batch(qs, x)
    eap.set_option("autotune", 1)
    tuned = eap.nn_search_batch(qs, x)   # tunes the missing buckets first
    assert tuned == plain
    for q, w in qs:
        assert eap.tune_get(q.numel(), w) is not None
    assert eap.nn_search_batch(qs, x) == plain   # replay with the tuned choices


def test_tune_save_load_round_trip(tmp_path, autotune_on):
    g = gen.rng(4102)
    x = torch.from_numpy(gen.as_f32(gen.random_walk(80_000, g))).cuda()
    q = torch.from_numpy(gen.as_f32(gen.random_walk(100, g))).cuda()
    t = eap.autotune(q, x, 10, sample_n=20_000)
    p = tmp_path / "tune.json"
    eap.tune_save(p)
    d = json.loads(p.read_text())
    assert d["arch"] == "gfx950"
    assert any(e["bucket"] == eap.tune_bucket(100, 10) for e in d["entries"])
    eap.tune_load(p)
    assert eap.tune_get(100, 10) == pytest.approx(t)
    # an entry written without the lanes field still loads (lanes 0)
    old = tmp_path / "old.json"
    old.write_text('{"arch": "gfx950", "entries": [\n  {"bucket": 7, "rows_per_group": 4, '
                   '"border": 1, "check_interval": 0, "wide_rows": 0, "ms": 1.5}\n]}\n')
    eap.tune_load(old)
    bad = tmp_path / "bad.json"
    bad.write_text('{"arch": "gfx942", "entries": []}')
    with pytest.raises(eap.EapdtwError):
        eap.tune_load(bad)
