"""The graphs an arc-switch chain can reach from a start graph (test helper,
host only, for tiny graphs), and a brute-force list of every simple digraph
with the same degree sequences to pin it.

A switch takes two arcs a->b, c->d (a != c) and makes them a->d, c->b; it is
valid when that makes no self-loop and no repeated arc.  With mutual=True the
two arcs must be of one kind: both one-way (then no arc may join a and d, or c
and b, in either direction) or both reciprocated (a<->b, c<->d become a<->d,
c<->b, under the same condition)."""
import itertools


def _moves(arcs, mutual):
    A = set(arcs)
    for (a, b), (c, d) in itertools.permutations(sorted(A), 2):
        if a == c or a == d or c == b or b == d:
            continue
        if (a, d) in A or (c, b) in A:
            continue
        if not mutual:
            yield frozenset((A - {(a, b), (c, d)}) | {(a, d), (c, b)})
            continue
        if (d, a) in A or (b, c) in A:
            continue
        ri, rj = (b, a) in A, (d, c) in A
        if ri != rj:
            continue
        if ri:
            yield frozenset((A - {(a, b), (b, a), (c, d), (d, c)}) | {(a, d), (d, a), (c, b), (b, c)})
        else:
            yield frozenset((A - {(a, b), (c, d)}) | {(a, d), (c, b)})


def reachable(arcs, mutual=False):
    """Every graph (a frozenset of arcs) reachable from `arcs` by valid switches."""
    start = frozenset(map(tuple, arcs))
    seen, todo = {start}, [start]
    while todo:
        for y in _moves(todo.pop(), mutual):
            if y not in seen:
                seen.add(y)
                todo.append(y)
    return seen


def signature(arcs, n, mutual=False):
    """Per vertex (out-degree, in-degree), or with mutual=True (reciprocated,
    one-way out, one-way in) neighbour counts."""
    A = set(map(tuple, arcs))
    if not mutual:
        return tuple((sum(1 for a, _ in A if a == v), sum(1 for _, b in A if b == v)) for v in range(n))
    rec = [sum(1 for a, b in A if a == v and (b, a) in A) for v in range(n)]
    out1 = [sum(1 for a, b in A if a == v and (b, a) not in A) for v in range(n)]
    in1 = [sum(1 for a, b in A if b == v and (b, a) not in A) for v in range(n)]
    return tuple(zip(rec, out1, in1))


def all_realisations(arcs, n, mutual=False):
    """Brute force: every simple digraph on n vertices with the signature of `arcs`."""
    want = signature(arcs, n, mutual)
    pairs = [(a, b) for a in range(n) for b in range(n) if a != b]
    m = len(set(map(tuple, arcs)))
    return {frozenset(c) for c in itertools.combinations(pairs, m) if signature(c, n, mutual) == want}
