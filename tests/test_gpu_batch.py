"""GPU tests of the fused batch path: the hipGraph-captured plan replays,
in-place regeneration between replays, and the autotuner."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    assert torch.cuda.is_available()
    import paper_1203_3415_amd as pm
    pm.lib()
    return pm


def _ensemble(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        n = int(rng.integers(60, 400))
        out.append(gg.chung_lu(n, int(n * rng.uniform(2, 4)), 2.3, 2.3, 0.05, seed=seed * 100 + t))
    return out


@pytest.mark.parametrize("k", [3, 4, 5])
def test_plan_replays_match_eager(pm, k):
    import torch
    graphs = _ensemble(12 if k < 5 else 6, 40 + k)
    dev = [(*pm.to_device(g.out_off, g.out_idx), g.n) for g in graphs]
    eager = pm.census_batch(dev, k)
    plan = pm.BatchPlan(dev, k)
    assert np.array_equal(plan.hists(), eager)
    other = gg.chung_lu(300, 1200, 2.2, 2.2, 0.1, seed=9)
    oo, oi = pm.to_device(other.out_off, other.out_idx)
    for r in range(3):
        print(f"[case] plan replay k={k} round {r}", flush=True)
        pm.census(oo, oi, other.n, 4)          # eager work between replays
        torch.cuda.synchronize()
        plan.out.fill_(0)
        plan.run()
        assert np.array_equal(plan.hists(), eager), f"replay {r}"
    plan.close()


def test_plan_sees_in_place_regeneration(pm):
    import torch
    base = gg.chung_lu(300, 1200, 2.3, 2.3, 0.05, seed=5)
    first = gg.arc_switch_many(base, 20 * base.m, [1, 2, 3, 4])
    second = gg.arc_switch_many(base, 20 * base.m, [5, 6, 7, 8])
    dev = [(*pm.to_device(g.out_off, g.out_idx), g.n) for g in [base] + first]
    plan = pm.BatchPlan(dev, 4)
    for i, g in enumerate([base] + first):
        assert np.array_equal(plan.hists()[i], oracle.census(g, 4))
    # write new randomisations (same n and m per slot) into the same buffers
    for (off_t, idx_t, _), g in zip(dev[1:], second):
        off_t.copy_(torch.as_tensor(g.out_off, device=off_t.device))
        idx_t.copy_(torch.as_tensor(g.out_idx, device=idx_t.device))
    torch.cuda.synchronize()
    plan.run()
    for i, g in enumerate([base] + second):
        assert np.array_equal(plan.hists()[i], oracle.census(g, 4)), i
    plan.close()


def test_plan_rejects_invalid_batch(pm):
    off, idx = pm.to_device(np.array([0, 1, 1], np.int32), np.array([0], np.int32))
    with pytest.raises(pm.MotifError) as e:
        pm.BatchPlan([(off, idx, 2)], 3)
    assert e.value.name == "ESELFLOOP"


def test_autotune_keeps_results(pm, tmp_path):
    graphs = _ensemble(10, 77)
    dev = [(*pm.to_device(g.out_off, g.out_idx), g.n) for g in graphs]
    saved = pm.get_tuning(4)
    try:
        print("[case] autotune k=4 on 10 graphs", flush=True)
        best = pm.autotune(dev, 4)
        assert best["block"] in (256, 512, 1024)
        assert 1 <= best["solo_deg"] <= 64 and 1 <= best["light_deg"] <= 256
        hb = pm.census_batch(dev, 4)
        for i, g in enumerate(graphs):
            assert np.array_equal(hb[i], oracle.census(g, 4))
        # the cache survives a save / clear / load round trip
        path = str(tmp_path / "tune.txt")
        pm.tune_cache_save(path)
        text = open(path).read()
        assert "gfx950" in text
        pm.set_tuning(4, **saved)          # drops the cached entries of k = 4
        assert pm.tune_cache_load(path) >= 1
        hb2 = pm.census_batch(dev, 4)
        assert np.array_equal(hb2, hb)
    finally:
        pm.set_tuning(4, **saved)


def test_placement_limits_keep_results(pm):
    # The work-placement limits only move work between waves and workgroups.
    g = gg.chung_lu(3000, 24000, 2.1, 2.1, 0.2, seed=31)
    off, idx = pm.to_device(g.out_off, g.out_idx)
    # the method reference (pinned against ESU): ESU needs minutes on these graphs
    want4 = oracle.method_census(g, 4)
    saved4, saved5 = pm.get_tuning(4), pm.get_tuning(5)
    try:
        for solo, light in ((1, 1), (16, 96), (64, 256), (40, 200)):
            print(f"[case] k=4 solo={solo} light={light}", flush=True)
            pm.set_tuning(4, solo_deg=solo, light_deg=light)
            assert np.array_equal(pm.census(off, idx, g.n, 4), want4)
        h = gg.chung_lu(700, 3500, 2.2, 2.5, 0.1, seed=32)
        ho, hi = pm.to_device(h.out_off, h.out_idx)
        want5 = oracle.method_census(h, 5)
        for light5 in (1, 64, 767):
            print(f"[case] k=5 light5={light5}", flush=True)
            pm.set_tuning(5, light5=light5)
            assert np.array_equal(pm.census(ho, hi, h.n, 5), want5)
    finally:
        pm.set_tuning(4, **saved4)
        pm.set_tuning(5, **saved5)
