"""Graph generators (inputs only; no census arithmetic lives here).

Shapes follow the workloads the paper measures on (biological and complex
networks, Section "Results and Discussion"): sparse, heavy-tailed degree
distributions with a fraction of reciprocated arcs.  The recipes:

* ``gnm_reciprocal``: uniform G(n, m0) digraph, then the reverse of a seeded
  fraction of its arcs is added (those reverses not already present).
* ``chung_lu``: arc (u, v) drawn with u ~ w_out, v ~ w_in where
  w_i = (i+1)^(-1/(gamma-1)) and the in-weights are independently permuted;
  self-loops and repeats rejected until m(1 - r/2) distinct arcs exist, then
  the reverse of round(m r / 2) arcs whose reverse is absent is added, giving
  exactly m arcs with reciprocated fraction about r.
* ``arc_switch``: degree-preserving randomisation; each attempted switch picks
  two arcs a->b, c->d and rewires to a->d, c->b unless that creates a loop or
  a repeated arc.  In- and out-degrees are preserved exactly.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Digraph:
    """Simple digraph in out-CSR form: arcs u->out_idx[out_off[u]:out_off[u+1]]."""

    n: int
    out_off: np.ndarray  # int32 [n+1]
    out_idx: np.ndarray  # int32 [m], each row sorted ascending

    @property
    def m(self) -> int:
        return int(self.out_off[-1])

    def arcs(self) -> np.ndarray:
        """(m, 2) int64 array of (tail, head), sorted by (tail, head)."""
        deg = np.diff(self.out_off.astype(np.int64))
        src = np.repeat(np.arange(self.n, dtype=np.int64), deg)
        return np.stack([src, self.out_idx.astype(np.int64)], axis=1)

    def in_csr(self) -> tuple[np.ndarray, np.ndarray]:
        """Transpose as (in_off, in_idx), rows sorted ascending."""
        a = self.arcs()
        order = np.lexsort((a[:, 0], a[:, 1]))
        heads = a[order, 1]
        tails = a[order, 0]
        cnt = np.bincount(heads, minlength=self.n) if self.n else np.zeros(0, np.int64)
        off = np.zeros(self.n + 1, dtype=np.int64)
        np.cumsum(cnt, out=off[1:])
        return off.astype(np.int32), tails.astype(np.int32)

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.out_off, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(self.out_idx, dtype=np.int32).tobytes())
        return h.hexdigest()


def from_arcs(n: int, arcs) -> Digraph:
    """Build a Digraph from an iterable/array of (tail, head) pairs.

    Rejects self-loops and repeated arcs (the census is defined on simple
    digraphs)."""
    a = np.asarray(arcs, dtype=np.int64).reshape(-1, 2)
    if a.size and (a.min() < 0 or a.max() >= n):
        raise ValueError("arc endpoint out of range")
    if np.any(a[:, 0] == a[:, 1]):
        raise ValueError("self-loop")
    key = a[:, 0] * max(n, 1) + a[:, 1]
    order = np.argsort(key, kind="stable")
    key = key[order]
    if key.size and np.any(key[1:] == key[:-1]):
        raise ValueError("repeated arc")
    a = a[order]
    cnt = np.bincount(a[:, 0], minlength=n) if n else np.zeros(0, np.int64)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt, out=off[1:])
    return Digraph(n, off.astype(np.int32), a[:, 1].astype(np.int32))


def _keys_to_graph(n: int, keys: np.ndarray) -> Digraph:
    keys = np.unique(keys)
    return from_arcs(n, np.stack([keys // n, keys % n], axis=1))


def _add_reciprocals(n: int, keys: np.ndarray, n_add: int, rng) -> np.ndarray:
    """Add the reverse of n_add distinct arcs (chosen uniformly among those
    whose reverse is absent)."""
    keys = np.unique(keys)
    rev = (keys % n) * n + keys // n
    absent = ~np.isin(rev, keys)
    cand = np.flatnonzero(absent)
    n_add = min(n_add, cand.size)
    pick = rng.choice(cand, size=n_add, replace=False) if n_add else np.zeros(0, np.int64)
    return np.unique(np.concatenate([keys, rev[pick]]))


def gnm_reciprocal(n: int, m0: int, frac: float, seed: int) -> Digraph:
    """m0 distinct uniform arcs (no loops), then the reverse of round(frac*m0)
    of them added (chosen among arcs whose reverse is absent)."""
    rng = np.random.default_rng(seed)
    if m0 > n * (n - 1):
        raise ValueError("too many arcs")
    keys = np.zeros(0, dtype=np.int64)
    while keys.size < m0:
        need = m0 - keys.size
        u = rng.integers(0, n, size=2 * need + 16)
        v = rng.integers(0, n, size=2 * need + 16)
        ok = u != v
        k = np.unique(u[ok] * n + v[ok])
        k = k[~np.isin(k, keys)]
        k = rng.permutation(k)[:need]
        keys = np.concatenate([keys, k])
    keys = _add_reciprocals(n, keys, int(round(frac * m0)), rng)
    return _keys_to_graph(n, keys)


def chung_lu(n: int, m: int, gamma_out: float, gamma_in: float, r: float, seed: int) -> Digraph:
    """Directed Chung-Lu power-law digraph with exactly m arcs and reciprocity ~r."""
    rng = np.random.default_rng(seed)
    idx = np.arange(n, dtype=np.float64)
    w_out = (idx + 1.0) ** (-1.0 / (gamma_out - 1.0))
    w_in = (idx + 1.0) ** (-1.0 / (gamma_in - 1.0))
    w_in = w_in[rng.permutation(n)]
    p_out = w_out / w_out.sum()
    p_in = w_in / w_in.sum()
    n_rec = int(round(m * r / 2.0))
    m_base = m - n_rec
    keys = np.zeros(0, dtype=np.int64)
    while keys.size < m_base:
        need = m_base - keys.size
        batch = int(need * 1.3) + 64
        u = rng.choice(n, size=batch, p=p_out)
        v = rng.choice(n, size=batch, p=p_in)
        ok = u != v
        k = u[ok].astype(np.int64) * n + v[ok]
        k, first = np.unique(k, return_index=True)
        k = k[np.argsort(first)]  # keep draw order among new keys
        k = k[~np.isin(k, keys)]
        keys = np.concatenate([keys, k[:need]])
    keys = _add_reciprocals(n, keys, n_rec, rng)
    if keys.size != m:
        # Not enough arcs with an absent reverse (tiny dense graphs): top up.
        while keys.size < m:
            u = rng.choice(n, p=p_out)
            v = rng.choice(n, p=p_in)
            if u != v:
                keys = np.unique(np.append(keys, np.int64(u) * n + v))
    return _keys_to_graph(n, keys)


def arc_switch(g: Digraph, attempts: int, seed: int) -> Digraph:
    """Degree-preserving randomisation by `attempts` attempted arc switches."""
    rng = np.random.default_rng(seed)
    a = g.arcs()
    n, m = g.n, a.shape[0]
    if m < 2:
        return g
    src = a[:, 0].copy()
    dst = a[:, 1].copy()
    present = set((src * n + dst).tolist())
    picks = rng.integers(0, m, size=(attempts, 2))
    for i, j in picks:
        if i == j:
            continue
        s1, d1, s2, d2 = src[i], dst[i], src[j], dst[j]
        if s1 == d2 or s2 == d1:
            continue
        k1, k2 = s1 * n + d2, s2 * n + d1
        if k1 in present or k2 in present:
            continue
        present.discard(s1 * n + d1)
        present.discard(s2 * n + d2)
        present.add(k1)
        present.add(k2)
        dst[i], dst[j] = d2, d1
    return from_arcs(n, np.stack([src, dst], axis=1))


_SWITCH_LIB = None


def _switch_lib():
    """gcc-built helper for many randomisations (compiled on first use)."""
    global _SWITCH_LIB
    if _SWITCH_LIB is None:
        import ctypes
        import os
        import subprocess
        here = os.path.dirname(os.path.abspath(__file__))
        src, lib = os.path.join(here, "switch.c"), os.path.join(here, "libswitch.so")
        if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
            subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", lib + ".tmp", src])
            os.replace(lib + ".tmp", lib)
        L = ctypes.CDLL(lib)
        P = ctypes.c_void_p
        L.gg_arc_switch_many.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, ctypes.c_int64, P, ctypes.c_int32, P, P]
        L.gg_arc_switch_many.restype = ctypes.c_int
        _SWITCH_LIB = L
    return _SWITCH_LIB


def arc_switch_many(g: Digraph, attempts: int, seeds) -> list:
    """Independent degree-preserving randomisations of g (one per seed), each
    by `attempts` attempted arc switches (C helper, splitmix64 per seed)."""
    import ctypes
    a = g.arcs()
    m = a.shape[0]
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    if m < 2:
        return [g for _ in seeds]
    src = np.ascontiguousarray(a[:, 0], dtype=np.int32)
    dst = np.ascontiguousarray(a[:, 1], dtype=np.int32)
    out = np.empty((len(seeds), m), dtype=np.int32)
    acc = np.zeros(len(seeds), dtype=np.int64)
    P = lambda x: x.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    _switch_lib().gg_arc_switch_many(g.n, m, P(src), P(dst), int(attempts), P(seeds), len(seeds), P(out), P(acc))
    return [from_arcs(g.n, np.stack([src, out[i]], axis=1)) for i in range(len(seeds))]


def planted_hubs(n: int, m_bg: int, n_hubs: int, hub_deg: int, hub_links: int, r: float, seed: int) -> Digraph:
    """Chung-Lu background (gamma 2.1 in and out, reciprocity r, m_bg arcs)
    plus n_hubs planted hubs: each hub is joined to hub_deg vertices drawn
    uniformly (so hubs share some neighbours) and to hub_links other hubs, by
    an arc out of the hub, into it or both ways (both with probability r, the
    other two equally likely).  Gives many vertices of large degree with
    mixed arc types at a modest number of connected small subgraphs."""
    rng = np.random.default_rng(seed)
    g = chung_lu(n, m_bg, 2.1, 2.1, r, seed)
    keys = [g.arcs()[:, 0] * n + g.arcs()[:, 1]]
    hubs = rng.choice(n, size=n_hubs, replace=False)

    def join(h, others):
        kind = rng.random(others.size)
        out = kind < (1 - r) / 2
        inn = (kind >= (1 - r) / 2) & (kind < 1 - r)
        both = kind >= 1 - r
        ks = [h * n + others[out | both], others[inn | both] * n + h]
        return np.concatenate(ks)

    for h in hubs:
        nb = rng.choice(n, size=hub_deg, replace=False)
        nb = nb[nb != h].astype(np.int64)
        keys.append(join(np.int64(h), nb))
        hl = rng.choice(hubs, size=min(hub_links, n_hubs - 1) + 1, replace=False)
        hl = hl[hl != h][:hub_links].astype(np.int64)
        keys.append(join(np.int64(h), hl))
    return _keys_to_graph(n, np.concatenate(keys))


def pad_relabel(g: Digraph, n_total: int, seed: int) -> Digraph:
    """g plus n_total - g.n isolated vertices, all relabelled by a seeded
    permutation.  Isolated vertices belong to no connected k-set, so the
    census is unchanged; only the vertex-id range grows."""
    if n_total < g.n:
        raise ValueError("n_total below g.n")
    perm = np.random.default_rng(seed).permutation(n_total)
    a = g.arcs()
    return from_arcs(n_total, perm[a])


def directed_cycle(n: int) -> Digraph:
    return from_arcs(n, [(i, (i + 1) % n) for i in range(n)] if n >= 2 else [])


def directed_path(n: int) -> Digraph:
    return from_arcs(n, [(i, i + 1) for i in range(n - 1)])


def complete_digraph(n: int) -> Digraph:
    return from_arcs(n, [(i, j) for i in range(n) for j in range(n) if i != j])


def transitive_tournament(n: int) -> Digraph:
    return from_arcs(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def star(n_bi: int, n_out: int, n_in: int) -> Digraph:
    """Centre 0 with n_bi bidirected, n_out outgoing-only and n_in incoming-only
    leaves (the paper's star example, Figure "star")."""
    arcs = []
    leaf = 1
    for _ in range(n_bi):
        arcs += [(0, leaf), (leaf, 0)]
        leaf += 1
    for _ in range(n_out):
        arcs.append((0, leaf))
        leaf += 1
    for _ in range(n_in):
        arcs.append((leaf, 0))
        leaf += 1
    return from_arcs(leaf, arcs)


def disjoint_union(*gs: Digraph) -> Digraph:
    arcs, base = [], 0
    for g in gs:
        a = g.arcs()
        arcs.append(a + base)
        base += g.n
    return from_arcs(base, np.concatenate(arcs) if arcs else np.zeros((0, 2), np.int64))


def relabel(g: Digraph, seed: int) -> Digraph:
    perm = np.random.default_rng(seed).permutation(g.n)
    a = g.arcs()
    return from_arcs(g.n, perm[a])


def reverse(g: Digraph) -> Digraph:
    a = g.arcs()
    return from_arcs(g.n, a[:, ::-1])


def random_small(n: int, p_arc: float, p_recip: float, seed: int) -> Digraph:
    """Small dense-ish random digraph for exhaustive parity tests: each ordered
    pair carries an arc with probability p_arc, and each arc's reverse is
    forced with probability p_recip."""
    rng = np.random.default_rng(seed)
    adj = rng.random((n, n)) < p_arc
    np.fill_diagonal(adj, False)
    force = rng.random((n, n)) < p_recip
    adj = adj | (adj.T & force.T)
    np.fill_diagonal(adj, False)
    u, v = np.nonzero(adj)
    return from_arcs(n, np.stack([u, v], axis=1))
