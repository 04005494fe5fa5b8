"""The seeded input generators shared by the GPU tests, the bench and the
oracle check: the serving stream's draws and its stratified sample."""
import numpy as np

import workloads as W


def test_serving_stream_is_seeded_and_in_range():
    a1, r1 = W.serving_stream(512, 40.0, 12345)
    a2, r2 = W.serving_stream(512, 40.0, 12345)
    assert np.array_equal(a1, a2) and r1 == r2
    assert a1[0] == 0.0 and np.all(np.diff(a1) >= 0)
    assert all(8 <= r["n"] <= 64 and 2 <= r["p"] <= 10 for r in r1)
    grad = [r for r in r1 if r["kind"] == "gradient"]
    assert 0.15 < len(grad) / len(r1) < 0.35
    assert all(0.2 <= r["phi_const"] <= 0.5 for r in grad)
    # each request's draws depend on its own seed only: a shorter stream is a prefix
    _, r3 = W.serving_stream(24, 40.0, 12345)
    assert r3 == r1[:24]


def test_stratified_sample_covers_every_stratum_with_its_smallest_meshes():
    _, reqs = W.serving_stream(512, 40.0, 12345)
    idx = W.stratified_sample(reqs, per_stratum=4)
    assert idx == sorted(set(idx))
    strata = {}
    for i, r in enumerate(reqs):
        strata.setdefault(W.serving_strata(r), []).append(i)
    assert len(strata) == 9   # 3 kinds x 3 degree bands
    chosen = {}
    for i in idx:
        chosen.setdefault(W.serving_strata(reqs[i]), []).append(i)
    assert set(chosen) == set(strata)
    for key, members in strata.items():
        got = chosen[key]
        assert len(got) == min(4, len(members))
        # no request outside the sample is smaller (n, then index) than a chosen one
        worst = max((reqs[i]["n"], i) for i in got)
        assert all((reqs[i]["n"], i) >= worst for i in members if i not in got)
    assert len(idx) >= 32
