"""Full-size parity in the launch configuration bench.py times.

Where the oracle could enumerate the workload, the GPU histogram must equal
the stored oracle golden bit for bit (tests/golden/*.json, written by
tests/golden/make_golden.py, which calls only the oracle).  Where it cannot
(the n = 1e5, m = 1e6 power-law graph at k = 4: about 4e12 connected 4-sets;
the n = 2e4 graph at k = 5), properties that hold at any size are checked:
invariance under vertex relabelling, additivity over a disjoint union with a
graph the oracle censuses, and batch = single."""
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def pm():
    import torch
    assert torch.cuda.is_available()
    import paper_1203_3415_amd as pm
    pm.lib()
    return pm


def _golden(name):
    path = os.path.join(HERE, "golden", name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"golden {name} not generated")
    d = json.load(open(path))
    h = np.zeros(oracle.N_CLASSES[d["k"]], np.uint64)
    for c, v in d["hist"].items():
        h[int(c)] = v
    g = getattr(gg, d["generator"])(**d["params"])
    assert g.sha256() == d["sha256"], "generator changed since the golden was written"
    return g, d["k"], h


@pytest.mark.parametrize("name", ["gnm_n1000_k3", "gnm_n1000_k4", "gnm_n1000_k5", "chunglu_n2000_m8000_k4",
                                  "chunglu_n1e5_m1e6_k3"])
def test_golden(pm, name):
    g, k, want = _golden(name)
    print(f"[case] golden {name} n={g.n} m={g.m} k={k}", flush=True)
    off, idx = pm.to_device(g.out_off, g.out_idx)
    got = pm.census(off, idx, g.n, k)
    assert np.array_equal(got, want)


@pytest.fixture(scope="module")
def big():
    return gg.chung_lu(100_000, 1_000_000, 2.1, 2.1, 0.2, seed=2)


def test_bench_graph_k4_invariants(pm, big):
    k = 4
    off, idx = pm.to_device(big.out_off, big.out_idx)
    print("[case] n=1e5 m=1e6 k=4 base", flush=True)
    h = pm.census(off, idx, big.n, k)
    assert int(h.sum()) > 0
    print("[case] relabelled", flush=True)
    r = gg.relabel(big, seed=77)
    ro, ri = pm.to_device(r.out_off, r.out_idx)
    assert np.array_equal(pm.census(ro, ri, r.n, k), h)
    print("[case] union with an oracle-censused graph", flush=True)
    small = gg.chung_lu(300, 1500, 2.2, 2.2, 0.2, seed=78)
    u = gg.disjoint_union(big, small)
    uo, ui = pm.to_device(u.out_off, u.out_idx)
    assert np.array_equal(pm.census(uo, ui, u.n, k), h + oracle.census(small, k))
    print("[case] batch of two", flush=True)
    so, si = pm.to_device(small.out_off, small.out_idx)
    hb = pm.census_batch([(off, idx, big.n), (so, si, small.n)], k)
    assert np.array_equal(hb[0], h)


def test_k5_workload_invariants(pm):
    g = gg.chung_lu(20_000, 100_000, 2.2, 2.5, 0.1, seed=4)
    off, idx = pm.to_device(g.out_off, g.out_idx)
    print("[case] n=2e4 m=1e5 k=5 base", flush=True)
    h = pm.census(off, idx, g.n, 5)
    r = gg.relabel(g, seed=5)
    ro, ri = pm.to_device(r.out_off, r.out_idx)
    print("[case] relabelled", flush=True)
    assert np.array_equal(pm.census(ro, ri, r.n, 5), h)
    small = gg.random_small(30, 0.3, 0.4, seed=6)
    u = gg.disjoint_union(g, small)
    uo, ui = pm.to_device(u.out_off, u.out_idx)
    print("[case] union", flush=True)
    assert np.array_equal(pm.census(uo, ui, u.n, 5), h + oracle.census(small, 5))
