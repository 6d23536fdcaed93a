"""Pins of the switch-chain helper (host only): the reachable graphs are
realisations of the same degrees, equal to the brute-force list where the
chain is known to connect them, and smaller where it is known not to (a
directed triangle cannot be reversed by 2-switches)."""
import pytest

from switch_space import all_realisations, reachable, signature


def test_triangle_reversal_is_unreachable():
    tri = [(0, 1), (1, 2), (2, 0)]
    assert reachable(tri) == {frozenset(tri)}
    assert all_realisations(tri, 3) == {frozenset(tri), frozenset([(1, 0), (2, 1), (0, 2)])}


def test_permutations_without_fixed_points():
    # out- and in-degree 1 on 4 vertices: the 9 fixed-point-free permutations
    # (derangements of 4), all joined by switches
    cyc = [(0, 1), (1, 2), (2, 3), (3, 0)]
    assert len(all_realisations(cyc, 4)) == 9
    assert reachable(cyc) == all_realisations(cyc, 4)


@pytest.mark.parametrize("mutual", [False, True])
def test_reachable_keeps_signature(mutual):
    g = [(0, 1), (1, 0), (2, 3), (3, 2), (0, 2), (1, 3), (4, 0), (2, 4)]
    r = reachable(g, mutual)
    assert frozenset(g) in r
    assert all(signature(x, 5, mutual) == signature(g, 5, mutual) for x in r)
    assert r <= all_realisations(g, 5, mutual)
    if not mutual:
        assert len(r) == 73
    else:
        # reciprocated pairs {0,1}, {2,3} may become {0,3}, {2,1}; one-way arcs follow
        assert 1 < len(r) < 73


def test_mutual_switch_keeps_pairs_together():
    g = [(0, 1), (1, 0), (2, 3), (3, 2)]
    r = reachable(g, True)
    assert r == {frozenset(g), frozenset([(0, 3), (3, 0), (2, 1), (1, 2)]),
                 frozenset([(0, 2), (2, 0), (1, 3), (3, 1)])}
    assert len(reachable(g, False)) > len(r)
