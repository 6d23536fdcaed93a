"""CPU oracle for the exact directed motif census -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It computes the census from its plain
definition (paper, Section "Problem statement": count the weakly connected
induced k-subgraphs, k = 3, 4, 5, grouped by isomorphism class) by ESU
enumeration plus canonical labelling over all k! vertex permutations, and it
shares no code with the GPU library.

Class ids: rank of the canonical code (minimum over all k! relabellings of the
k(k-1)-bit adjacency code, arc i->j at bit i*(k-1) + (j<i ? j : j-1)) among the
weakly connected classes, ascending.  The paper leaves the numbering free
("arbitrarily associated", "hard coded").

Parity: every function here is pinned in ``tests/test_oracle.py`` against the
paper's class counts, its star worked example, its multiplicities and closed
forms, and against the independent pure-Python all-subsets checker in
``oracle/brute.py``.

``method_census`` and ``undirected4`` (``method_ref.c``) are a second CPU
route: the paper's own combinatorial method (Algorithms "Count 3/4/5 Sized
Patterns", and Algorithm "und4" with Table "ept" on the undirected version),
written out step by step.  They are pinned against the ESU census above in
``tests/test_method_ref.py`` and serve for the workloads too large for ESU.
"""
from __future__ import annotations

import ctypes
import functools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "method_ref.c")]
_LIB = os.path.join(_HERE, "liboracle.so")

N_CLASSES = {3: 13, 4: 199, 5: 9364}


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or any(os.path.getmtime(_LIB) < os.path.getmtime(s) for s in _SRCS):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, *_SRCS])
        os.replace(tmp, _LIB)
    return _LIB


@functools.lru_cache(maxsize=1)
def _lib():
    lib = ctypes.CDLL(build())
    P = ctypes.c_void_p
    lib.oracle_class_table.argtypes = [ctypes.c_int, P, P, P, P, P]
    lib.oracle_class_table.restype = ctypes.c_int
    lib.oracle_multiplicity.argtypes = [ctypes.c_int, ctypes.c_uint32]
    lib.oracle_multiplicity.restype = ctypes.c_int
    lib.oracle_census.argtypes = [ctypes.c_int32, P, P, ctypes.c_int32, P, ctypes.c_int32, P, ctypes.c_int32]
    lib.oracle_census.restype = ctypes.c_int
    lib.oracle_census_roots.argtypes = [ctypes.c_int32, P, P, ctypes.c_int32, P, ctypes.c_int32, P, ctypes.c_int32,
                                        P, ctypes.c_int32]
    lib.oracle_census_roots.restype = ctypes.c_int
    lib.oracle_census_timed.argtypes = [ctypes.c_int32, P, P, ctypes.c_int32, P, ctypes.c_int32, P, ctypes.c_int32,
                                        P, ctypes.c_int32, ctypes.c_double]
    lib.oracle_census_timed.restype = ctypes.c_int
    lib.mref_census.argtypes = [ctypes.c_int32, P, P, ctypes.c_int32, P, P, ctypes.c_int32, P, ctypes.c_int32]
    lib.mref_census.restype = ctypes.c_int
    lib.mref_census_sample.argtypes = [ctypes.c_int32, P, P, ctypes.c_int32, P, ctypes.c_int32, P, ctypes.c_int32,
                                       ctypes.c_int64]
    lib.mref_census_sample.restype = ctypes.c_int
    lib.mref_undirected4.argtypes = [ctypes.c_int32, P, P, P, ctypes.c_int32]
    lib.mref_undirected4.restype = ctypes.c_int
    lib.oracle_canon6.argtypes = [ctypes.c_uint32]
    lib.oracle_canon6.restype = ctypes.c_uint32
    lib.oracle_census6.argtypes = [ctypes.c_int32, P, P, ctypes.c_int32, P, P, ctypes.c_int64, P]
    lib.oracle_census6.restype = ctypes.c_int
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@functools.lru_cache(maxsize=4)
def class_table(k: int):
    """(cls_of_code uint16[2^(k(k-1))], canon_of_class uint32[C], n_all_classes,
    n_connected_codes) computed by brute force over all codes and permutations."""
    lib = _lib()
    nb = k * (k - 1)
    cls = np.empty(1 << nb, dtype=np.uint16)
    canon = np.zeros(16384, dtype=np.uint32)
    nc = np.zeros(1, np.int32)
    na = np.zeros(1, np.int32)
    ncodes = np.zeros(1, np.int64)
    rc = lib.oracle_class_table(k, _ptr(cls), _ptr(canon), _ptr(nc), _ptr(na), _ptr(ncodes))
    if rc != 0:
        raise RuntimeError(f"oracle_class_table failed: {rc}")
    cls.setflags(write=False)
    c = canon[: int(nc[0])].copy()
    c.setflags(write=False)
    return cls, c, int(na[0]), int(ncodes[0])


def multiplicity(k: int, code: int) -> int:
    """Number of connected (k-2)-subsets dominating the other two vertices."""
    return int(_lib().oracle_multiplicity(k, code))


def census(g, k: int, threads: int = 0) -> np.ndarray:
    """uint64 histogram over the classes for graph ``g`` (graphgen.Digraph or
    anything with n, out_off, out_idx)."""
    cls, canon, _, _ = class_table(k)
    hist = np.zeros(len(canon), dtype=np.uint64)
    off = np.ascontiguousarray(g.out_off, dtype=np.int32)
    idx = np.ascontiguousarray(g.out_idx, dtype=np.int32)
    if idx.size == 0:
        idx = np.zeros(1, np.int32)
    rc = _lib().oracle_census(int(g.n), _ptr(off), _ptr(idx), k, _ptr(cls), len(canon), _ptr(hist), threads)
    if rc != 0:
        raise RuntimeError(f"oracle_census failed: {rc}")
    return hist


def census_roots(g, k: int, roots, threads: int = 0) -> np.ndarray:
    """Histogram of the connected k-sets whose smallest vertex is in `roots`."""
    cls, canon, _, _ = class_table(k)
    hist = np.zeros(len(canon), dtype=np.uint64)
    off = np.ascontiguousarray(g.out_off, dtype=np.int32)
    idx = np.ascontiguousarray(g.out_idx, dtype=np.int32)
    if idx.size == 0:
        idx = np.zeros(1, np.int32)
    r = np.ascontiguousarray(roots, dtype=np.int32)
    rc = _lib().oracle_census_roots(int(g.n), _ptr(off), _ptr(idx), k, _ptr(cls), len(canon), _ptr(hist), threads,
                                    _ptr(r), int(r.size))
    if rc != 0:
        raise RuntimeError(f"oracle_census_roots failed: {rc}")
    return hist


def census_timed(g, k: int, roots, seconds: float, threads: int = 0) -> np.ndarray:
    """Sets emitted by ESU from `roots` (in order) within `seconds` of wall time."""
    cls, canon, _, _ = class_table(k)
    hist = np.zeros(len(canon), dtype=np.uint64)
    off = np.ascontiguousarray(g.out_off, dtype=np.int32)
    idx = np.ascontiguousarray(g.out_idx, dtype=np.int32)
    if idx.size == 0:
        idx = np.zeros(1, np.int32)
    r = np.ascontiguousarray(roots, dtype=np.int32)
    rc = _lib().oracle_census_timed(int(g.n), _ptr(off), _ptr(idx), k, _ptr(cls), len(canon), _ptr(hist), threads,
                                    _ptr(r), int(r.size), float(seconds))
    if rc != 0:
        raise RuntimeError(f"oracle_census_timed failed: {rc}")
    return hist


@functools.lru_cache(maxsize=4)
def multiplicities(k: int) -> np.ndarray:
    """int32 [C]: the oracle's multiplicity of every class (anchors that see
    one occurrence)."""
    _, canon, _, _ = class_table(k)
    lib = _lib()
    m = np.array([lib.oracle_multiplicity(k, int(c)) for c in canon], dtype=np.int32)
    m.setflags(write=False)
    return m


def _csr(g):
    off = np.ascontiguousarray(g.out_off, dtype=np.int32)
    idx = np.ascontiguousarray(g.out_idx, dtype=np.int32)
    if idx.size == 0:
        idx = np.zeros(1, np.int32)
    return off, idx


def method_census(g, k: int, threads: int = 0) -> np.ndarray:
    """uint64 histogram by the paper's combinatorial method (method_ref.c):
    per-anchor set sizes, m-variables and closed forms, then the exact
    division by the class multiplicities."""
    cls, canon, _, _ = class_table(k)
    mult = multiplicities(k)
    hist = np.zeros(len(canon), dtype=np.uint64)
    off, idx = _csr(g)
    rc = _lib().mref_census(int(g.n), _ptr(off), _ptr(idx), k, _ptr(cls), _ptr(mult), len(canon), _ptr(hist),
                            threads)
    if rc != 0:
        raise RuntimeError(f"mref_census failed: {rc}")
    return hist


def method_census_sample(g, k: int, stride: int, threads: int = 0) -> None:
    """Timing only: the method's per-anchor work on a pseudo-random 1/stride
    of the anchor units (no division, result discarded)."""
    cls, canon, _, _ = class_table(k)
    hist = np.zeros(len(canon), dtype=np.uint64)
    off, idx = _csr(g)
    rc = _lib().mref_census_sample(int(g.n), _ptr(off), _ptr(idx), k, _ptr(cls), len(canon), _ptr(hist), threads,
                                   int(stride))
    if rc != 0:
        raise RuntimeError(f"mref_census_sample failed: {rc}")


UNDIRECTED4 = ("P4", "tailed_triangle", "claw", "C4", "diamond", "K4")


def undirected4(g, threads: int = 0) -> np.ndarray:
    """uint64 [6]: induced connected 4-vertex subgraphs of the undirected
    version G*, by skeleton (P4, tailed triangle, claw, C4, K4 minus an edge,
    K4), by Algorithm "und4" and Table "ept"."""
    out = np.zeros(6, dtype=np.uint64)
    off, idx = _csr(g)
    rc = _lib().mref_undirected4(int(g.n), _ptr(off), _ptr(idx), _ptr(out), threads)
    if rc != 0:
        raise RuntimeError(f"mref_undirected4 failed: {rc}")
    return out


# -- undirected censuses --------------------------------------------------------

def und_bit(k: int, i: int, j: int) -> int:
    """Bit of the edge {i, j} (i < j) in a k-vertex undirected code."""
    return i * (2 * k - i - 1) // 2 + (j - i - 1)


def _und_connected(k: int, code: int) -> bool:
    adj = [[False] * k for _ in range(k)]
    for i in range(k):
        for j in range(i + 1, k):
            if code >> und_bit(k, i, j) & 1:
                adj[i][j] = adj[j][i] = True
    seen, stack = {0}, [0]
    while stack:
        a = stack.pop()
        for b in range(k):
            if adj[a][b] and b not in seen:
                seen.add(b)
                stack.append(b)
    return len(seen) == k


@functools.lru_cache(maxsize=4)
def undirected_class_table(k: int):
    """(canon: sorted canonical codes of the connected undirected graphs on k
    vertices, cls_of_code: dict code -> class id for every connected code,
    n_all_classes, n_connected_codes), by brute force over all
    2^(k(k-1)/2) codes and all k! relabellings."""
    import itertools
    perms = list(itertools.permutations(range(k)))
    nb = k * (k - 1) // 2
    canon_of = {}
    for code in range(1 << nb):
        best = None
        for p in perms:
            c = 0
            for i in range(k):
                for j in range(i + 1, k):
                    if code >> und_bit(k, i, j) & 1:
                        a, b = min(p[i], p[j]), max(p[i], p[j])
                        c |= 1 << und_bit(k, a, b)
            best = c if best is None else min(best, c)
        canon_of[code] = best
    classes = sorted({c for x, c in canon_of.items() if _und_connected(k, x)})
    rank = {c: i for i, c in enumerate(classes)}
    cls = {x: rank[c] for x, c in canon_of.items() if c in rank}
    return tuple(classes), cls, len(set(canon_of.values())), len(cls)


def census_undirected(g, k: int, threads: int = 0, method: bool = False) -> np.ndarray:
    """uint64 histogram over the undirected classes: the connected induced
    k-subgraphs of the undirected version G* of g, by ESU on G* read as a
    symmetric digraph (every pattern then has all arcs reciprocated), each
    class mapped to the undirected class of its skeleton.  method=True takes
    the method reference instead of ESU for the directed census (for sizes
    ESU cannot finish)."""
    a = np.asarray(g.arcs())
    sym = np.unique(np.concatenate([a, a[:, ::-1]]), axis=0) if a.size else a.reshape(0, 2)

    class _G:
        pass
    h = _G()
    h.n = g.n
    cnt = np.bincount(sym[:, 0], minlength=g.n) if sym.size else np.zeros(g.n, np.int64)
    h.out_off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)
    h.out_idx = sym[:, 1].astype(np.int32) if sym.size else np.zeros(0, np.int32)
    hd = method_census(h, k, threads=threads) if method else census(h, k, threads=threads)
    _, canon, _, _ = class_table(k)
    _, ucls, _, _ = undirected_class_table(k)
    out = np.zeros(len(undirected_class_table(k)[0]), np.uint64)
    for c in np.flatnonzero(hd):
        code = int(canon[c])
        u = 0
        for i in range(k):
            for j in range(i + 1, k):
                if code >> (i * (k - 1) + (j - 1)) & 1:
                    u |= 1 << und_bit(k, i, j)
        out[ucls[u]] += hd[c]
    return out


def code_of(k: int, arcs) -> int:
    """Adjacency code of a k-vertex pattern given as (i, j) arcs."""
    code = 0
    for i, j in arcs:
        code |= 1 << (i * (k - 1) + (j if j < i else j - 1))
    return code


def class_of(k: int, arcs) -> int:
    """Class id of the k-vertex pattern with these arcs (0xFFFF if disconnected)."""
    return int(class_table(k)[0][code_of(k, arcs)])


# ---------------------------------------------------------------- k = 6 --
# The paper's stated extension to larger motifs (Section "Our approach").
# 2^30 codes are too many for a class table here, so k = 6 classes are named
# by their canonical code (minimum over the 720 relabellings).

N_CLASSES6 = 1_530_843  # weakly connected digraphs on 6 vertices


def canon6(code: int) -> int:
    """Canonical code of a 6-vertex code (minimum over all 720 relabellings)."""
    return int(_lib().oracle_canon6(ctypes.c_uint32(code)))


def census6(g, threads: int = 0) -> dict:
    """Connected 6-sets of the digraph g by ESU, as {canonical code: count}."""
    cap = N_CLASSES6 + 1
    codes = np.zeros(cap, np.uint32)
    counts = np.zeros(cap, np.uint64)
    nout = np.zeros(1, np.int64)
    off = np.ascontiguousarray(g.out_off, np.int32)
    idx = np.ascontiguousarray(g.out_idx, np.int32)
    rc = _lib().oracle_census6(int(g.n), _ptr(off), _ptr(idx), int(threads), _ptr(codes), _ptr(counts), cap,
                               _ptr(nout))
    if rc:
        raise RuntimeError(f"oracle_census6 failed: {rc}")
    k = int(nout[0])
    return {int(c): int(v) for c, v in zip(codes[:k], counts[:k])}
