"""GPU tests of the k = 6 census (the anchor method with connected 4-set
anchors) against the CPU oracle, which counts the connected 6-sets by ESU and
names each class by its canonical code (minimum over the 720 relabellings).

The device-built class table is pinned by its counts (1,530,843 weakly
connected digraphs on 6 vertices), by the oracle's canonical form and
multiplicity on sampled classes, and the census by exact equality with the
oracle on seeded random, power-law and structured graphs."""
import math

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


@pytest.fixture(scope="module")
def codes(pm):
    print("[case] k=6 class table", flush=True)
    return pm.class6_codes()


def _by_code(pm, codes, g):
    off, idx = pm.to_device(g.out_off, g.out_idx)
    h = pm.census6(off, idx, g.n)
    nz = np.flatnonzero(h)
    return {int(codes[c]): int(h[c]) for c in nz}


def test_class_table(pm, codes):
    assert codes.size == oracle.N_CLASSES6 == pm.NUM_CLASSES6
    assert np.all(np.diff(codes.astype(np.int64)) > 0)
    mult = pm.class6_multiplicities()
    assert mult.min() >= 1 and mult.max() == 15
    rng = np.random.default_rng(6)
    for c in np.r_[0, 1, codes.size - 1, rng.integers(0, codes.size, 300)]:
        x = int(codes[c])
        assert oracle.canon6(x) == x
        assert int(mult[c]) == oracle.multiplicity(6, x)
    assert codes[-1] == (1 << 30) - 1          # the complete digraph is the largest code


@pytest.mark.parametrize("seed", range(6))
def test_random_graphs(pm, codes, seed):
    rng = np.random.default_rng(660 + seed)
    n = int(rng.integers(20, 60))
    g = gg.gnm_reciprocal(n, int(rng.integers(2 * n, 4 * n)), float(rng.uniform(0, 0.4)), seed=seed)
    print(f"[case] k=6 random seed={seed} n={g.n} m={g.m}", flush=True)
    assert _by_code(pm, codes, g) == oracle.census6(g)


@pytest.mark.parametrize("n,m,seed", [(150, 450, 61), (300, 700, 62), (120, 600, 63)])
def test_power_law(pm, codes, n, m, seed):
    g = gg.chung_lu(n, m, 2.3, 2.4, 0.2, seed=seed)
    print(f"[case] k=6 power law n={n} m={m}", flush=True)
    assert _by_code(pm, codes, g) == oracle.census6(g)


def test_closed_forms(pm, codes):
    full = (1 << 30) - 1
    kn = np.array([(a, b) for a in range(9) for b in range(9) if a != b])
    assert _by_code(pm, codes, gg.from_arcs(9, kn)) == {full: math.comb(9, 6)}
    star = np.array([(0, i) for i in range(1, 12)])
    assert sum(_by_code(pm, codes, gg.from_arcs(12, star)).values()) == math.comb(11, 5)
    cyc = np.array([(i, (i + 1) % 40) for i in range(40)])
    assert list(_by_code(pm, codes, gg.from_arcs(40, cyc)).values()) == [40]
    assert _by_code(pm, codes, gg.from_arcs(30, np.zeros((0, 2), np.int64))) == {}


def test_errors(pm):
    off, idx = pm.to_device(np.array([0, 1, 2], np.int32), np.array([1, 1], np.int32))
    with pytest.raises(pm.MotifError) as e:
        pm.census6(off, idx, 2)
    assert e.value.name == "ESELFLOOP"


def test_in_csr_checked(pm, codes):
    g = gg.chung_lu(60, 150, 2.3, 2.3, 0.2, seed=64)
    off, idx = pm.to_device(g.out_off, g.out_idx)
    ioff, iidx = pm.to_device(*g.in_csr())
    h = pm.census6(off, idx, g.n, in_off=ioff, in_idx=iidx)
    assert {int(codes[c]): int(h[c]) for c in np.flatnonzero(h)} == oracle.census6(g)
    # one in-arc replaced by an arc that is not in the graph
    ioff_h, iidx_h = g.in_csr()
    t = int(np.flatnonzero(np.diff(ioff_h))[0])
    row = set(iidx_h[ioff_h[t]:ioff_h[t + 1]].tolist())
    bad = iidx_h.copy()
    bad[ioff_h[t]] = next(x for x in range(g.n) if x not in row and x != t)
    ioff2, iidx2 = pm.to_device(ioff_h, bad)
    with pytest.raises(pm.MotifError) as e:
        pm.census6(off, idx, g.n, in_off=ioff2, in_idx=iidx2)
    assert e.value.name == "ETRANSPOSE"


def test_too_big_anchor_edge(pm):
    # a star with 1,100 leaves: every anchor edge has more than 1,024 members
    star = np.array([(0, i) for i in range(1, 1101)])
    g = gg.from_arcs(1101, star)
    off, idx = pm.to_device(g.out_off, g.out_idx)
    with pytest.raises(pm.MotifError) as e:
        pm.census6(off, idx, g.n)
    assert e.value.name == "ETOOBIG"
