"""GPU tests of the on-device null model: degree-preserving arc-switch
randomisation in place (plain, and keeping reciprocated pairs), and the fused
randomise + census + z-score job.

For every seed the generated graphs are copied back and checked on the host:
out- and in-degrees preserved (and the numbers of reciprocated and one-way
neighbours for the mutual-preserving switch), no self-loops, no repeated
arcs, most arcs moved.  On tiny graphs, thousands of independent chains must
land on the graphs the switches can reach (enumerated on the host) uniformly.
The census of the generated graphs (copied back) must equal the CPU oracle on
those same graphs, and the device z-scores must equal the host's
exact-integer z-scores of the same histograms."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from switch_space import reachable

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    assert torch.cuda.is_available()
    import paper_1203_3415_amd as pm
    pm.lib()
    return pm


def _host(g, idx_t):
    """The randomised graph as a Digraph (rows sorted), from its device targets."""
    idx = idx_t.cpu().numpy()
    src = np.repeat(np.arange(g.n), np.diff(g.out_off))
    return gg.from_arcs(g.n, np.stack([src, idx], axis=1))   # rejects loops and repeated arcs


def _reciprocated(g):
    """Per arc: is its reverse present?"""
    a = g.arcs().astype(np.int64)
    key = a[:, 0] * g.n + a[:, 1]
    return np.isin(a[:, 1] * g.n + a[:, 0], key)


def _check_same_degrees(base, r, mutual=False):
    a0, a = base.arcs(), r.arcs()
    assert np.array_equal(np.diff(r.out_off), np.diff(base.out_off))
    assert np.array_equal(np.bincount(a[:, 1], minlength=base.n), np.bincount(a0[:, 1], minlength=base.n))
    if mutual:   # reciprocated, one-way out and one-way in neighbours of every vertex
        def sig(g, arcs):
            rec = _reciprocated(g)
            return [np.bincount(arcs[rec, 0], minlength=base.n), np.bincount(arcs[~rec, 0], minlength=base.n),
                    np.bincount(arcs[~rec, 1], minlength=base.n)]
        for x, y in zip(sig(base, a0), sig(r, a)):
            assert np.array_equal(x, y)
    moved = 1.0 - len(set(map(tuple, a.tolist())) & set(map(tuple, a0.tolist()))) / base.m
    return moved


@pytest.mark.parametrize("mutual", [False, True])
@pytest.mark.parametrize("shape", ["nullbase_n2000", "uneven_n5000", "global_n20000"])
def test_randomize_keeps_degrees_and_simplicity(pm, shape, mutual):
    import torch
    base = {"nullbase_n2000": lambda: gg.chung_lu(2000, 8000, 2.3, 2.3, 0.05, seed=3),
            "uneven_n5000": lambda: gg.chung_lu(5000, 20000, 2.3, 2.3, 0.3, seed=4),
            # too large for one workgroup's LDS: switched in global memory
            "global_n20000": lambda: gg.chung_lu(20000, 60000, 2.2, 2.2, 0.1, seed=5)}[shape]()
    off, idx = pm.to_device(base.out_off, base.out_idx)
    copies = [idx.clone() for _ in range(4)]
    print(f"[case] randomise {shape} n={base.n} m={base.m} mutual={mutual}", flush=True)
    pm.null_randomize([(off, c, base.n) for c in copies], 100, seed=11, mutual=mutual)
    torch.cuda.synchronize()
    outs = []
    rec0 = _reciprocated(base)
    for c in copies:
        r = _host(base, c)
        moved = _check_same_degrees(base, r, mutual)
        assert moved > 0.5, moved
        if mutual:   # the reciprocated pairs moved too
            a0, a = base.arcs()[rec0], r.arcs()[_reciprocated(r)]
            assert len(set(map(tuple, a.tolist())) & set(map(tuple, a0.tolist()))) < 0.5 * len(a0)
        outs.append(c.cpu().numpy())
    assert not np.array_equal(outs[0], outs[1])           # one stream per graph
    again = idx.clone()
    pm.null_randomize([(off, copies[0].clone(), base.n), (off, again, base.n)], 100, seed=11, mutual=mutual)
    torch.cuda.synchronize()
    assert np.array_equal(again.cpu().numpy(), outs[1])   # a function of (input, seed, graph index)


@pytest.mark.parametrize("mutual", [False, True])
def test_randomize_mixed_sizes(pm, mutual):
    """One call over graphs of every placement: small enough for two
    workgroups per CU, needing a CU's whole LDS, and switched in global
    memory (three launches, each list largest first).  Every graph keeps its
    degrees and stays simple, and the call is a function of its inputs."""
    import torch
    bases = [gg.chung_lu(1500, 6000, 2.3, 2.3, 0.05, seed=21),    # fits in half the LDS
             gg.chung_lu(5000, 20000, 2.3, 2.3, 0.3, seed=22),    # needs all of it
             gg.chung_lu(20000, 60000, 2.2, 2.2, 0.1, seed=23),   # global memory
             gg.chung_lu(800, 3200, 2.3, 2.3, 0.05, seed=24)]     # half again, smaller
    devs = [pm.to_device(b.out_off, b.out_idx) for b in bases]
    outs = []
    for rep in range(2):
        print(f"[case] randomise mixed sizes mutual={mutual} rep={rep}", flush=True)
        copies = [idx.clone() for _, idx in devs]
        pm.null_randomize([(off, c, b.n) for (off, _), c, b in zip(devs, copies, bases)], 100, seed=31, mutual=mutual)
        torch.cuda.synchronize()
        outs.append([c.cpu().numpy() for c in copies])
    for b, c0, c1 in zip(bases, outs[0], outs[1]):
        assert np.array_equal(c0, c1)
        assert _check_same_degrees(b, _host(b, torch.from_numpy(c0)), mutual) > 0.5


# Tiny start graphs with 73 graphs reachable by plain switches and 48 by
# mutual-preserving ones (enumerated by switch_space.reachable).
UNIFORM = {False: (5, [(0, 1), (1, 0), (2, 3), (3, 2), (0, 2), (1, 3), (4, 0), (2, 4)]),
           True: (6, [(0, 1), (1, 0), (2, 3), (3, 2), (4, 5), (5, 4), (0, 4), (2, 1), (5, 3)])}


@pytest.mark.parametrize("mutual", [False, True])
def test_switch_chain_is_uniform(pm, mutual):
    # Every round is a symmetric move, so each chain's state tends to the
    # uniform distribution over the graphs it can reach: 8,192 chains (one
    # random stream each) must land only on reachable graphs, each about
    # equally often (chi-square against uniform, p > 0.001; seeded, so the
    # outcome is fixed).
    import torch
    from scipy.stats import chi2
    n, arcs = UNIFORM[mutual]
    space = reachable(arcs, mutual)
    assert len(space) == (48 if mutual else 73)
    g = gg.from_arcs(n, np.array(arcs))
    off, idx = pm.to_device(g.out_off, g.out_idx)
    count = 8192
    flat = idx.repeat(count)
    views = [flat[i * g.m:(i + 1) * g.m] for i in range(count)]
    print(f"[case] uniformity mutual={mutual} states={len(space)} chains={count}", flush=True)
    pm.null_randomize([(off, v, n) for v in views], 40_000, seed=5, mutual=mutual)   # about 300 rounds
    torch.cuda.synchronize()
    got = flat.cpu().numpy().reshape(count, g.m)
    src = np.repeat(np.arange(n), np.diff(g.out_off))
    seen = {}
    for row in got:
        key = frozenset(zip(src.tolist(), row.tolist()))
        assert key in space
        seen[key] = seen.get(key, 0) + 1
    obs = np.array([seen.get(x, 0) for x in space], np.float64)
    exp = count / len(space)
    stat = float(((obs - exp) ** 2 / exp).sum())
    assert chi2.sf(stat, len(space) - 1) > 1e-3, (stat, obs.min(), obs.max())


def test_randomize_rejects_bad_offsets(pm):
    import torch
    off, idx = pm.to_device(np.array([0, 2, 1, 3], np.int32), np.array([1, 2, 0], np.int32))
    before = idx.clone()
    with pytest.raises(pm.MotifError) as e:
        pm.null_randomize([(off, idx, 3)], 10, seed=1)
    assert e.value.name == "EINVAL_SHAPE"
    torch.cuda.synchronize()
    assert torch.equal(idx, before)


@pytest.mark.parametrize("targets,name", [([1, 3, 0], "EINDEX"), ([1, -1, 0], "EINDEX"), ([1, 1, 0], "ESELFLOOP")])
def test_randomize_rejects_bad_targets(pm, targets, name):
    import torch
    # rows 0: {1}, 1: {x}, 2: {0} beside a valid 3-cycle; nothing is rewritten, in either mode
    good_off, good_idx = pm.to_device(np.array([0, 1, 2, 3], np.int32), np.array([1, 2, 0], np.int32))
    off, idx = pm.to_device(np.array([0, 1, 2, 3], np.int32), np.array(targets, np.int32))
    keep = good_idx.clone()
    for mutual in (False, True):
        with pytest.raises(pm.MotifError) as e:
            pm.null_randomize([(good_off, good_idx, 3), (off, idx, 3)], 10, seed=1, mutual=mutual)
        assert e.value.name == name
        torch.cuda.synchronize()
        assert idx.cpu().tolist() == targets and torch.equal(good_idx, keep)


@pytest.mark.parametrize("k,count,mutual", [(3, 24, False), (4, 16, False), (5, 6, False), (4, 16, True)])
def test_null_model_matches_oracle_on_generated_graphs(pm, k, count, mutual):
    import torch
    real = gg.chung_lu(300 if k < 5 else 150, 1200 if k < 5 else 500, 2.3, 2.3, 0.3 if mutual else 0.1, seed=40 + k)
    off, idx = pm.to_device(real.out_off, real.out_idx)
    print(f"[case] null model k={k} count={count} mutual={mutual}", flush=True)
    hists, z = pm.null_model(off, idx, real.n, count, k, switches_per_arc=50, seed=7, mutual=mutual)
    assert np.array_equal(hists[0], oracle.census(real, k))
    # the same randomisations, made by the in-place call, copied back and censused on the CPU
    copies = [idx.clone() for _ in range(count)]
    pm.null_randomize([(off, c, real.n) for c in copies], 50, seed=7, mutual=mutual)
    torch.cuda.synchronize()
    for i, c in enumerate(copies):
        r = _host(real, c)
        _check_same_degrees(real, r, mutual)
        assert np.array_equal(hists[i + 1], oracle.census(r, k)), i
    want = pm.zscores(hists)
    fin = np.isfinite(want)
    assert np.array_equal(fin, np.isfinite(z))
    assert np.allclose(z[fin], want[fin], rtol=1e-12, atol=0)


def test_null_model_c3_shape(pm):
    # The null-model workload: base n = 2000, m = 8000, 100 m switches per
    # copy; the fused census equals the batch census of the copies made in place.
    import torch
    real = gg.chung_lu(2000, 8000, 2.3, 2.3, 0.05, seed=3)
    off, idx = pm.to_device(real.out_off, real.out_idx)
    count = 64
    print("[case] null model n=2000 m=8000 k=4 x64", flush=True)
    hists, z = pm.null_model(off, idx, real.n, count, 4, switches_per_arc=100, seed=1000)
    copies = [idx.clone() for _ in range(count)]
    pm.null_randomize([(off, c, real.n) for c in copies], 100, seed=1000)
    hb = pm.census_batch([(off, idx, real.n)] + [(off, c, real.n) for c in copies], 4)
    assert np.array_equal(hists, hb)
    # spot-check two copies against the method reference (pinned against ESU)
    for i in (0, count - 1):
        r = _host(real, copies[i])
        assert np.array_equal(hists[i + 1], oracle.method_census(r, 4))
    assert np.isfinite(z).sum() > 20
