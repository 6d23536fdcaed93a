"""Full-size parity in the launch configuration bench.py times.

Every workload is compared bit for bit with a stored CPU golden
(tests/golden/*.json, written by tests/golden/make_golden.py, which calls only
the oracle package):
* "esu" goldens: the plain definition (ESU enumeration), for the workloads it
  finishes -- the n = 1e3 G(n, m) graph (k = 3, 4, 5), the null-model base
  (k = 4), the bench graph at k = 3, the bench workloads scaled to n/20 and a
  graph of 74 planted hubs of degree >= 256 with mixed arc types;
* "method_ref" goldens: the paper's method written out on the CPU, pinned
  against ESU (tests/test_method_ref.py), for the bench graph at k = 4
  (4.25e12 connected 4-sets) and the n = 2e4 graph at k = 5.
The k = 4 bench golden also stores the undirected skeleton counts of
Algorithm "und4" / Table "ept"; the GPU's 199 classes summed by skeleton
must reproduce them.  Small goldens are also re-run padded with isolated
vertices to the bench sizes, so that the kernel instances of the bench
workloads (label tables sized for n = 1e5 at k = 4, 2e4 at k = 5) see them,
and the default core-reuse kernels are compared with the per-anchor kernels
at full size."""
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from skeleton import project

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def pm():
    import torch
    assert torch.cuda.is_available()
    import paper_1203_3415_amd as pm
    pm.lib()
    return pm


_GRAPHS = {}


def _golden(name):
    path = os.path.join(HERE, "golden", name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"golden {name} not generated")
    d = json.load(open(path))
    undirected = d.get("route", "esu").endswith("_undirected")
    size = len(oracle.undirected_class_table(d["k"])[0]) if undirected else oracle.N_CLASSES[d["k"]]
    h = np.zeros(size, np.uint64)
    for c, v in d["hist"].items():
        h[int(c)] = v
    key = (d["generator"], json.dumps(d["params"], sort_keys=True))
    if key not in _GRAPHS:
        _GRAPHS.clear()  # keep one large graph at a time
        _GRAPHS[key] = getattr(gg, d["generator"])(**d["params"])
    g = _GRAPHS[key]
    assert g.sha256() == d["sha256"], "generator changed since the golden was written"
    return g, d["k"], h, d


def _diff(got, want):
    bad = np.flatnonzero(got != want)
    return f"{len(bad)} classes differ, first {bad[:6].tolist()}: gpu {got[bad[:6]].tolist()} " \
           f"cpu {want[bad[:6]].tolist()}"


GOLDENS = ["gnm_n1000_k3", "gnm_n1000_k4", "gnm_n1000_k5", "chunglu_n2000_m8000_k4", "chunglu_n5000_m5e4_k4",
           "chunglu_n1000_m5000_k5", "hubs_n6000_k4", "chunglu_n1e5_m1e6_k3", "chunglu_n1e5_m1e6_k4",
           "chunglu_n2e4_m1e5_k5"]


@pytest.mark.parametrize("name", GOLDENS)
def test_golden(pm, name):
    g, k, want, d = _golden(name)
    print(f"[case] golden {name} ({d.get('route', 'esu')}) n={g.n} m={g.m} k={k}", flush=True)
    off, idx = pm.to_device(g.out_off, g.out_idx)
    got = pm.census(off, idx, g.n, k)
    assert np.array_equal(got, want), _diff(got, want)


def test_bench_step_matches_goldens(pm):
    # The call bench.py times: k = 3 and 4 over one build, out- and in-CSR.
    g, _, want4, d4 = _golden("chunglu_n1e5_m1e6_k4")
    _, _, want3, _ = _golden("chunglu_n1e5_m1e6_k3")
    print("[case] bench step: census_multi k=(3,4) with in-CSR", flush=True)
    off, idx = pm.to_device(g.out_off, g.out_idx)
    io, ii = pm.to_device(*g.in_csr())
    h3, h4 = pm.census_multi(off, idx, g.n, (3, 4), in_off=io, in_idx=ii)
    assert np.array_equal(h3, want3), _diff(h3, want3)
    assert np.array_equal(h4, want4), _diff(h4, want4)
    # the undirected skeleton (Algorithm "und4", Table "ept"), computed on the
    # CPU by a different algorithm from the directed one
    assert project(h4).tolist() == [d4["undirected4"][s] for s in oracle.UNDIRECTED4]


@pytest.mark.parametrize("name,n_total", [("gnm_n1000_k4", 100_000), ("chunglu_n2000_m8000_k4", 100_000),
                                          ("hubs_n6000_k4", 100_000), ("gnm_n1000_k5", 20_000),
                                          ("chunglu_n1000_m5000_k5", 20_000)])
def test_golden_padded_to_bench_size(pm, name, n_total):
    g, k, want, _ = _golden(name)
    p = gg.pad_relabel(g, n_total, seed=n_total + g.n)
    print(f"[case] padded {name} to n={n_total} k={k}", flush=True)
    off, idx = pm.to_device(p.out_off, p.out_idx)
    got = pm.census(off, idx, p.n, k)
    assert np.array_equal(got, want), _diff(got, want)


@pytest.mark.parametrize("name", ["chunglu_n1e5_m1e6_k4", "chunglu_n2e4_m1e5_k5", "hubs_n6000_k4"])
def test_per_anchor_kernels_at_full_size(pm, name):
    # The per-anchor kernels (the paper's scheme, one anchor at a time) and the
    # default core-reuse kernels, each against the same golden.
    g, k, want, _ = _golden(name)
    off, idx = pm.to_device(g.out_off, g.out_idx)
    saved = pm.get_tuning(k)
    try:
        pm.set_tuning(k, heavy=2)
        print(f"[case] per-anchor {name} k={k}", flush=True)
        got = pm.census(off, idx, g.n, k)
    finally:
        pm.set_tuning(k, **saved)
    assert np.array_equal(got, want), _diff(got, want)


def test_undirected_census_at_full_size(pm):
    # k = 4: the bench graph's undirected version against Algorithm "und4" /
    # Table "ept" (stored with the k = 4 golden); k = 5: the n = 2e4 graph
    # against the method reference on its symmetric version; k = 5 on the
    # n = 1e3 graph against ESU.
    g, _, _, d4 = _golden("chunglu_n1e5_m1e6_k4")
    off, idx = pm.to_device(g.out_off, g.out_idx)
    print("[case] undirected k=4 n=1e5", flush=True)
    h = pm.census_undirected(off, idx, g.n, 4)
    canon = oracle.undirected_class_table(4)[0]
    name = {7: "claw", 13: "P4", 15: "tailed_triangle", 30: "C4", 31: "diamond", 63: "K4"}
    assert {name[int(c)]: int(h[i]) for i, c in enumerate(canon)} == d4["undirected4"]
    for gname in ("chunglu_n2e4_m1e5_und5", "gnm_n1000_und5"):
        g, k, want, _ = _golden(gname)
        off, idx = pm.to_device(g.out_off, g.out_idx)
        print(f"[case] undirected {gname}", flush=True)
        got = pm.census_undirected(off, idx, g.n, k)
        assert np.array_equal(got, want), _diff(got, want)


def test_bench_graph_k4_invariants(pm):
    g, k, want, _ = _golden("chunglu_n1e5_m1e6_k4")
    print("[case] n=1e5 m=1e6 k=4 relabelled", flush=True)
    r = gg.relabel(g, seed=77)
    ro, ri = pm.to_device(r.out_off, r.out_idx)
    assert np.array_equal(pm.census(ro, ri, r.n, k), want)
    print("[case] union with an oracle-censused graph, and a batch of two", flush=True)
    small = gg.chung_lu(300, 1500, 2.2, 2.2, 0.2, seed=78)
    u = gg.disjoint_union(g, small)
    uo, ui = pm.to_device(u.out_off, u.out_idx)
    hs = oracle.census(small, k)
    assert np.array_equal(pm.census(uo, ui, u.n, k), want + hs)
    off, idx = pm.to_device(g.out_off, g.out_idx)
    so, si = pm.to_device(small.out_off, small.out_idx)
    hb = pm.census_batch([(off, idx, g.n), (so, si, small.n)], k)
    assert np.array_equal(hb[0], want) and np.array_equal(hb[1], hs)
