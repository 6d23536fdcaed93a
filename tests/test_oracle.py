"""Pins for the CPU oracle (no GPU).

Each test ties the oracle to something other than itself: the paper's class
counts and worked example, closed forms, multiplicities the paper states, an
independent pure-Python all-subsets checker, and invariants of the census.
"""
import itertools
import math
import os
from collections import Counter

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import brute

HERE = os.path.dirname(os.path.abspath(__file__))


# -- class tables -----------------------------------------------------------

@pytest.mark.parametrize("k,conn_classes,all_classes,conn_codes", [
    (3, 13, 16, 54),        # Problem Motifs-3: 13 classes
    (4, 199, 218, 3834),    # Problem Motifs-4: 199 classes
    (5, 9364, 9608, 1027080),  # Problem Motifs-5: 9364 classes
])
def test_class_counts(k, conn_classes, all_classes, conn_codes):
    # Connected counts: the paper's problem statements.  All-digraph counts and
    # labelled weakly connected digraph counts: the standard enumerations of
    # unlabelled digraphs and of labelled weakly connected digraphs on k nodes.
    cls, canon, n_all, n_codes = oracle.class_table(k)
    assert len(canon) == conn_classes
    assert n_all == all_classes
    assert n_codes == conn_codes
    assert int((cls != 0xFFFF).sum()) == conn_codes
    assert list(canon) == sorted(canon)
    # every class id is hit and each canonical code maps to its own class
    assert set(np.unique(cls[cls != 0xFFFF]).tolist()) == set(range(conn_classes))
    for c, code in enumerate(canon[:50]):
        assert cls[code] == c


def test_class_table_matches_python_canonical_k3_k4():
    for k in (3, 4):
        cls, canon, _, _ = oracle.class_table(k)
        nb = k * (k - 1)
        for code in range(0, 1 << nb, 7 if k == 4 else 1):
            arcs = [(i, j) for i in range(k) for j in range(k) if i != j
                    and code >> (i * (k - 1) + (j if j < i else j - 1)) & 1]
            c = cls[code]
            if c != 0xFFFF:
                assert canon[c] == brute.canonical(k, arcs)


# -- multiplicities (anchors that see a pattern) ------------------------------

def _mult(k, arcs):
    return oracle.multiplicity(k, oracle.code_of(k, arcs))


def test_multiplicity_k3():
    # Each triangle is a v-Pattern of its three corners; an open wedge only of
    # its centre (division by 3 in Algorithm "Count 3 Sized Patterns").
    assert _mult(3, [(0, 1), (1, 2)]) == 1
    assert _mult(3, [(0, 1), (1, 2), (2, 0)]) == 3


def test_multiplicity_k4_fact_correction():
    # Fact "correction": P4 1, S3 3, tailed triangle 3, C4 4, K4\e 5, K4 6.
    assert _mult(4, [(0, 1), (1, 2), (2, 3)]) == 1
    assert _mult(4, [(0, 1), (0, 2), (0, 3)]) == 3
    assert _mult(4, [(0, 1), (1, 2), (2, 0), (2, 3)]) == 3
    assert _mult(4, [(0, 1), (1, 2), (2, 3), (3, 0)]) == 4
    assert _mult(4, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 2)]) == 5
    assert _mult(4, [(i, j) for i in range(4) for j in range(i + 1, 4)]) == 6
    # orientation does not matter: all-bidirected K4 too
    assert _mult(4, [(i, j) for i in range(4) for j in range(4) if i != j]) == 6


def test_multiplicity_k5():
    # Figure "correction:five": C5 is counted by 5 connected triples.
    assert _mult(5, [(i, (i + 1) % 5) for i in range(5)]) == 5
    assert _mult(5, [(i, i + 1) for i in range(4)]) == 1                     # P5: only the middle triple
    assert _mult(5, [(0, j) for j in range(1, 5)]) == math.comb(4, 2)       # K1,4
    assert _mult(5, [(i, j) for i in range(5) for j in range(i + 1, 5)]) == math.comb(5, 3)


# -- the paper's worked example ---------------------------------------------

def _read_star_fixture():
    rows = []
    with open(os.path.join(HERE, "golden", "star_k3.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            sizes, arcs, freq = [p.strip() for p in line.split("|")]
            na, nb, nc = map(int, sizes.split())
            arcs = [tuple(map(int, a.split(">"))) for a in arcs.split(",")]
            rows.append(((na, nb, nc), arcs, int(freq)))
    return rows


def test_star_worked_example():
    rows = _read_star_fixture()
    na, nb, nc = rows[0][0]
    hist = oracle.census(gg.star(na, nb, nc), 3)
    expect = np.zeros(13, np.uint64)
    for _, arcs, freq in rows:
        expect[oracle.class_of(3, arcs)] += freq
    assert (hist == expect).all()
    assert int(hist.sum()) == math.comb(na + nb + nc, 2) == 78


@pytest.mark.parametrize("k", [3, 4, 5])
@pytest.mark.parametrize("na,nb,nc", [(4, 4, 5), (0, 3, 2), (3, 0, 0), (2, 2, 2)])
def test_star_multinomial(k, na, nb, nc):
    # Only sets containing the centre are connected; the class depends only on
    # the multiset of leaf types: C(na,i) C(nb,j) C(nc,l) sets for i+j+l = k-1.
    hist = oracle.census(gg.star(na, nb, nc), k)
    expect = np.zeros(len(hist), np.uint64)
    for i in range(k):
        for j in range(k - i):
            l = k - 1 - i - j
            cnt = math.comb(na, i) * math.comb(nb, j) * math.comb(nc, l)
            if cnt == 0:
                continue
            arcs, leaf = [], 1
            for _ in range(i):
                arcs += [(0, leaf), (leaf, 0)]; leaf += 1
            for _ in range(j):
                arcs.append((0, leaf)); leaf += 1
            for _ in range(l):
                arcs.append((leaf, 0)); leaf += 1
            expect[oracle.class_of(k, arcs)] += cnt
    assert (hist == expect).all()


# -- closed forms -----------------------------------------------------------

@pytest.mark.parametrize("k", [3, 4, 5])
def test_closed_forms(k):
    n = 8
    h = oracle.census(gg.complete_digraph(n), k)
    c = oracle.class_of(k, [(i, j) for i in range(k) for j in range(k) if i != j])
    assert h[c] == math.comb(n, k) and h.sum() == math.comb(n, k)

    h = oracle.census(gg.transitive_tournament(n), k)
    c = oracle.class_of(k, [(i, j) for i in range(k) for j in range(i + 1, k)])
    assert h[c] == math.comb(n, k) and h.sum() == math.comb(n, k)

    path_cls = oracle.class_of(k, [(i, i + 1) for i in range(k - 1)])
    h = oracle.census(gg.directed_cycle(9), k)
    assert h[path_cls] == 9 and h.sum() == 9
    h = oracle.census(gg.directed_cycle(k), k)
    assert h[oracle.class_of(k, [(i, (i + 1) % k) for i in range(k)])] == 1 and h.sum() == 1
    h = oracle.census(gg.directed_path(10), k)
    assert h[path_cls] == 10 - k + 1 and h.sum() == 10 - k + 1

    assert oracle.census(gg.from_arcs(6, []), k).sum() == 0
    assert oracle.census(gg.complete_digraph(k - 1), k).sum() == 0
    assert oracle.census(gg.from_arcs(0, []), k).sum() == 0


# -- brute force on tiny inputs ------------------------------------------------

def _by_canon(k, hist):
    _, canon, _, _ = oracle.class_table(k)
    return Counter({int(canon[c]): int(v) for c, v in enumerate(hist) if v})


@pytest.mark.parametrize("k", [3, 4, 5])
def test_esu_matches_all_subsets(k):
    rng = np.random.default_rng(100 + k)
    cases = 12 if k < 5 else 6
    for t in range(cases):
        n = int(rng.integers(k, 10 if k < 5 else 9))
        g = gg.random_small(n, float(rng.uniform(0.1, 0.6)), float(rng.uniform(0, 1)), seed=1000 * k + t)
        got = _by_canon(k, oracle.census(g, k))
        want = brute.census_by_canon(g.n, g.arcs(), k)
        assert got == want, (k, t, n)


# -- invariants ---------------------------------------------------------------

def _undirected(g):
    a = g.arcs()
    s = set()
    for u, v in a:
        s.add((min(u, v), max(u, v)))
    return s


def test_k3_sum_identity():
    # Sum over classes = connected 3-subsets = sum_v C(d*(v),2) - 2 T(G*).
    g = gg.chung_lu(400, 2400, 2.3, 2.3, 0.2, seed=7)
    e = _undirected(g)
    adj = [set() for _ in range(g.n)]
    for u, v in e:
        adj[u].add(v); adj[v].add(u)
    wedges = sum(math.comb(len(a), 2) for a in adj)
    tri = sum(len(adj[u] & adj[v]) for u, v in e) // 3
    h = oracle.census(g, 3)
    assert int(h.sum()) == wedges - 2 * tri
    # triangles: classes whose skeleton is a triangle hold exactly T
    _, canon, _, _ = oracle.class_table(3)
    closed = 0
    for c, code in enumerate(canon):
        und = set()
        for i in range(3):
            for j in range(3):
                if i != j and code >> (i * 2 + (j if j < i else j - 1)) & 1:
                    und.add((min(i, j), max(i, j)))
        if len(und) == 3:
            closed += int(h[c])
    assert closed == tri


@pytest.mark.parametrize("k", [3, 4, 5])
def test_relabel_union_reverse(k):
    g = gg.chung_lu(60, 200, 2.2, 2.4, 0.2, seed=11)
    h = oracle.census(g, k)
    assert (oracle.census(gg.relabel(g, 5), k) == h).all()
    g2 = gg.gnm_reciprocal(40, 90, 0.3, seed=12)
    h2 = oracle.census(g2, k)
    assert (oracle.census(gg.disjoint_union(g, g2), k) == h + h2).all()
    # reversing every arc maps each class to the class of its transpose
    cls, canon, _, _ = oracle.class_table(k)
    hr = oracle.census(gg.reverse(g), k)
    expect = np.zeros_like(h)
    for c, code in enumerate(canon):
        arcs = [(i, j) for i in range(k) for j in range(k) if i != j
                and code >> (i * (k - 1) + (j if j < i else j - 1)) & 1]
        expect[oracle.class_of(k, [(j, i) for i, j in arcs])] += h[c]
    assert (hr == expect).all()


def test_esu_count_small_random_sum():
    # Sum of the histogram equals the number of connected k-subsets found by
    # the independent checker (count only; classes compared elsewhere).
    g = gg.random_small(11, 0.25, 0.3, seed=3)
    for k in (3, 4, 5):
        want = sum(brute.census_by_canon(g.n, g.arcs(), k).values())
        assert int(oracle.census(g, k).sum()) == want


@pytest.mark.parametrize("k", [3, 4, 5])
def test_root_partition_sums_to_census(k):
    # ESU emits each connected set from its smallest vertex, so censuses over
    # a partition of the roots add up to the full census.
    g = gg.chung_lu(120, 500, 2.2, 2.4, 0.2, seed=13)
    rng = np.random.default_rng(4)
    perm = rng.permutation(g.n)
    parts = np.array_split(perm, 3)
    total = sum(oracle.census_roots(g, k, p) for p in parts)
    assert (total == oracle.census(g, k)).all()
