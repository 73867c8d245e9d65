"""Host logic of the batch autotuner (no GPU): it times every candidate in
the start mode it is told (cold: warm_start = 0), keeps the fastest, caches
the choice under a key that depends on the multiset of shapes and the
precision, and answers from the cache without timing again."""
import json
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


@pytest.fixture()
def tuner(monkeypatch):
    from paper_1306_0645_amd import autotune
    calls = []

    def fake_time(shapes, hs, params, fields, dts, reps):
        calls.append((params.tile_z, params.nu_pre, params.nu_post, params.warm_start))
        # a made-up cost surface with its minimum at tile depth 4, V(2,2)
        return 1.0 + abs(params.tile_z - 4) * 0.1 + (0.0 if params.nu_pre == 2 else 0.05)

    monkeypatch.setattr(autotune, "_time_batch", fake_time)
    return autotune, calls


def test_tuner_picks_the_fastest_and_caches_it(tuner, tmp_path):
    autotune, calls = tuner
    import paper_1306_0645_amd as fld
    base = fld.fld_default_params(3e10, 1e22, precision=fld.FLD_PREC_MIXED, warm_start=2)
    shapes = [(32, 32, 32), (64, 64, 64), (48, 48, 48)]
    hs = [(1.0, 1.0, 1.0)] * 3
    cache = str(tmp_path / "tune.json")
    p, rep = autotune.tune_batch(shapes, hs, base, None, [1.0] * 3, cache_path=cache)
    assert not rep["cached"]
    assert (p.tile_z, p.nu_pre, p.nu_post) == (4, 2, 2)
    # every candidate timed once, each with cold starts
    assert len(calls) == len(autotune.CANDIDATES)
    assert {c[3] for c in calls} == {0}
    # the returned parameters keep the caller's own warm start
    assert p.warm_start == 2 and p.precision == fld.FLD_PREC_MIXED
    with open(cache) as f:
        stored = json.load(f)
    assert rep["key"] in stored and stored[rep["key"]]["best"] == rep["best"]
    # the same multiset of shapes in another order: answered from the cache
    calls.clear()
    p2, rep2 = autotune.tune_batch(list(reversed(shapes)), hs, base, None, [1.0] * 3,
                                   cache_path=cache)
    assert rep2["cached"] and not calls
    assert (p2.tile_z, p2.nu_pre) == (4, 2)
    # another precision or another set of shapes is tuned anew
    b64 = fld.fld_default_params(3e10, 1e22, precision=fld.FLD_PREC_FP64)
    _, rep3 = autotune.tune_batch(shapes, hs, b64, None, [1.0] * 3, cache_path=cache)
    assert not rep3["cached"] and calls
    calls.clear()
    _, rep4 = autotune.tune_batch(shapes[:2], hs[:2], base, None, [1.0] * 2,
                                  cache_path=cache)
    assert not rep4["cached"] and calls
    assert len({rep["key"], rep3["key"], rep4["key"]}) == 3


def test_tuner_skips_failing_candidates(tuner, tmp_path, monkeypatch):
    autotune, calls = tuner
    import paper_1306_0645_amd as fld

    def fail_fused(shapes, hs, params, fields, dts, reps):
        # candidates whose batch step failed report inf and must never win
        return float("inf") if params.nu_pre == 1 else 2.0 - 0.01 * params.tile_z

    monkeypatch.setattr(autotune, "_time_batch", fail_fused)
    base = fld.fld_default_params(3e10, 1e22, precision=fld.FLD_PREC_MIXED)
    p, rep = autotune.tune_batch([(32, 32, 32)], [(1.0, 1.0, 1.0)], base, None, [1.0],
                                 cache_path=str(tmp_path / "t.json"))
    assert p.nu_pre == 2 and p.tile_z == 8
