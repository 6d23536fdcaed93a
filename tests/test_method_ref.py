"""Pins for the CPU method reference (oracle/method_ref.c), no GPU.

The method reference writes out the paper's combinatorial census (Algorithms
"Count 3/4/5 Sized Patterns", and Algorithm "und4" with Table "ept" for the
undirected skeleton).  Before it may stand in for the ESU oracle on workloads
too large to enumerate, it must agree with ESU bit for bit: on many seeded
small graphs, on the closed forms, and on every stored ESU golden, including
the n/20-scaled versions of the full-size workloads.  The census_timed pin is
here too: with a deadline it never reaches it equals census_roots.
"""
import json
import math
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from skeleton import project

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def _check(g, k, label):
    got = oracle.method_census(g, k)
    want = oracle.census(g, k)
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError(f"{label} k={k}: classes {bad[:6].tolist()} method {got[bad[:6]].tolist()} "
                             f"esu {want[bad[:6]].tolist()}")


@pytest.mark.parametrize("k", [3, 4, 5])
def test_matches_esu_on_120_small_graphs(k):
    rng = np.random.default_rng(900 + k)
    for t in range(120):
        n = int(rng.integers(k, 14 if k < 5 else 12))
        g = gg.random_small(n, float(rng.uniform(0.05, 0.8)), float(rng.uniform(0, 1)), seed=7000 * k + t)
        _check(g, k, f"random_small#{t}")


@pytest.mark.parametrize("k", [3, 4, 5])
def test_matches_esu_on_power_law_graphs(k):
    # heavy tails, reciprocity, isolated vertices, ragged rows
    sizes = {3: [(300, 1500), (800, 6000)], 4: [(200, 900), (400, 2000)], 5: [(120, 400), (180, 600)]}[k]
    for i, (n, m) in enumerate(sizes):
        for gam, r in ((2.1, 0.3), (2.6, 0.0)):
            g = gg.chung_lu(n, m, gam, gam + 0.2, r, seed=40 * k + 3 * i + int(10 * r))
            _check(g, k, f"chung_lu n={n} gamma={gam}")
    _check(gg.disjoint_union(gg.star(3, 2, 4), gg.gnm_reciprocal(40, 120, 0.4, seed=5)), k, "union")


@pytest.mark.parametrize("k", [3, 4, 5])
def test_closed_forms(k):
    n = 9
    for g, arcs in ((gg.complete_digraph(n), [(i, j) for i in range(k) for j in range(k) if i != j]),
                    (gg.transitive_tournament(n), [(i, j) for i in range(k) for j in range(i + 1, k)])):
        h = oracle.method_census(g, k)
        assert h[oracle.class_of(k, arcs)] == math.comb(n, k) == h.sum()
    path_cls = oracle.class_of(k, [(i, i + 1) for i in range(k - 1)])
    h = oracle.method_census(gg.directed_cycle(11), k)
    assert h[path_cls] == 11 == h.sum()
    h = oracle.method_census(gg.directed_cycle(k), k)
    assert h[oracle.class_of(k, [(i, (i + 1) % k) for i in range(k)])] == 1 == h.sum()
    h = oracle.method_census(gg.directed_path(10), k)
    assert h[path_cls] == 10 - k + 1 == h.sum()
    assert oracle.method_census(gg.from_arcs(7, []), k).sum() == 0
    assert oracle.method_census(gg.complete_digraph(k - 1), k).sum() == 0
    # the paper's star example (Figure "star"): C(13, k-1) sets, all at the centre
    assert oracle.method_census(gg.star(4, 4, 5), k).sum() == math.comb(13, k - 1)


def _esu_goldens():
    out = []
    for f in sorted(os.listdir(GOLDEN)):
        if f.endswith(".json"):
            d = json.load(open(os.path.join(GOLDEN, f)))
            if d.get("route", "esu") == "esu" and d["n"] <= 10_000:
                out.append(f)
    return out


@pytest.mark.parametrize("fname", _esu_goldens())
def test_matches_stored_esu_goldens(fname):
    # Includes the n/20-scaled bench workloads and the planted-hub graph.
    d = json.load(open(os.path.join(GOLDEN, fname)))
    g = getattr(gg, d["generator"])(**d["params"])
    assert g.sha256() == d["sha256"]
    h = oracle.method_census(g, d["k"])
    want = np.zeros(len(h), np.uint64)
    for c, v in d["hist"].items():
        want[int(c)] = v
    assert np.array_equal(h, want)


# -- the undirected skeleton (Algorithm "und4", Table "ept") -------------------

def test_undirected4_matches_esu_projection():
    rng = np.random.default_rng(31)
    for t in range(60):
        n = int(rng.integers(4, 13))
        g = gg.random_small(n, float(rng.uniform(0.1, 0.7)), float(rng.uniform(0, 1)), seed=8100 + t)
        assert np.array_equal(oracle.undirected4(g), project(oracle.census(g, 4))), t
    for g in (gg.chung_lu(300, 1500, 2.2, 2.4, 0.2, seed=4), gg.gnm_reciprocal(200, 900, 0.2, seed=6)):
        assert np.array_equal(oracle.undirected4(g), project(oracle.census(g, 4)))


def test_undirected4_closed_forms():
    # K_n: only K4; a chordless cycle: n paths P4; C_4 itself; a star S_n: claws
    und = lambda n, es: gg.from_arcs(n, [(a, b) for a, b in es] + [(b, a) for a, b in es])  # noqa: E731
    kn = und(8, [(i, j) for i in range(8) for j in range(i + 1, 8)])
    assert oracle.undirected4(kn).tolist() == [0, 0, 0, 0, 0, math.comb(8, 4)]
    assert oracle.undirected4(und(9, [(i, (i + 1) % 9) for i in range(9)])).tolist() == [9, 0, 0, 0, 0, 0]
    assert oracle.undirected4(und(4, [(i, (i + 1) % 4) for i in range(4)])).tolist() == [0, 0, 0, 1, 0, 0]
    assert oracle.undirected4(gg.star(2, 3, 2)).tolist() == [0, 0, math.comb(7, 3), 0, 0, 0]
    # orientation does not matter: one direction only, the same skeleton
    tt = gg.transitive_tournament(8)
    assert oracle.undirected4(tt).tolist() == [0, 0, 0, 0, 0, math.comb(8, 4)]


def test_method_reports_inexact_division():
    # A wrong multiplicity must surface as an error, not a rounded count.
    import ctypes
    g = gg.chung_lu(80, 300, 2.2, 2.2, 0.2, seed=3)
    cls, canon, _, _ = oracle.class_table(4)
    mult = oracle.multiplicities(4).copy()
    h = oracle.census(g, 4)
    c = int(np.flatnonzero(h)[0])
    mult[c] = 7 if (int(h[c]) * int(mult[c])) % 7 else 11
    hist = np.zeros(len(canon), np.uint64)
    off = np.ascontiguousarray(g.out_off, np.int32)
    idx = np.ascontiguousarray(g.out_idx, np.int32)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    rc = oracle._lib().mref_census(g.n, P(off), P(idx), 4, P(cls), P(mult), len(canon), P(hist), 0)
    assert rc == -3 and hist.sum() == 0


# -- census_timed ---------------------------------------------------------------

@pytest.mark.parametrize("k", [3, 4])
def test_census_timed_with_unreached_deadline_equals_roots(k):
    g = gg.chung_lu(300, 1500, 2.2, 2.4, 0.2, seed=17)
    roots = np.random.default_rng(5).permutation(g.n)[:120]
    full = oracle.census_roots(g, k, roots)
    timed = oracle.census_timed(g, k, roots, seconds=1e6)
    assert np.array_equal(timed, full)
    # a deadline already passed stops early: at most the full count, per class
    early = oracle.census_timed(g, k, roots, seconds=1e-9)
    assert (early <= full).all()
