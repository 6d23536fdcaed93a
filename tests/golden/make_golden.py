"""Write golden histograms computed by the CPU oracle package only.

Usage: python tests/golden/make_golden.py NAME [THREADS]

Each golden file records the generator recipe, the input's SHA-256, which
CPU route computed it and the histogram (class id -> count; class ids as
defined by the oracle's canonical-code numbering):

* "esu": the plain definition, ESU enumeration of every connected k-set
  (oracle.census).
* "method_ref": the paper's combinatorial method written out on the CPU
  (oracle.method_census), for the workloads too large to enumerate.  It is
  pinned against ESU on many small graphs and on the n/20-scaled versions of
  these same workloads (tests/test_method_ref.py), which are "esu" goldens.
  k = 4 method goldens also store the undirected skeleton counts of
  Algorithm "und4" (oracle.undirected4), an independent projection check.
* "esu_undirected" / "method_ref_undirected": the undirected census of the
  graph's undirected version (oracle.census_undirected), its directed
  census of the symmetric digraph taken by ESU or by the method reference.

Nothing here calls the GPU library.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

CL = "chung_lu"
RECIPES = {
    # name: (generator, params, k, route)
    "chunglu_n1e5_m1e6_k3": (CL, dict(n=100_000, m=1_000_000, gamma_out=2.1, gamma_in=2.1, r=0.2, seed=2), 3, "esu"),
    "gnm_n1000_k3": ("gnm_reciprocal", dict(n=1000, m0=5000, frac=0.1, seed=1), 3, "esu"),
    "gnm_n1000_k4": ("gnm_reciprocal", dict(n=1000, m0=5000, frac=0.1, seed=1), 4, "esu"),
    "gnm_n1000_k5": ("gnm_reciprocal", dict(n=1000, m0=5000, frac=0.1, seed=1), 5, "esu"),
    "chunglu_n2000_m8000_k4": (CL, dict(n=2000, m=8000, gamma_out=2.3, gamma_in=2.3, r=0.05, seed=3), 4, "esu"),
    # the bench workloads scaled to n/20 (same generator, density and exponents)
    "chunglu_n5000_m5e4_k4": (CL, dict(n=5000, m=50_000, gamma_out=2.1, gamma_in=2.1, r=0.2, seed=2), 4, "esu"),
    "chunglu_n1000_m5000_k5": (CL, dict(n=1000, m=5000, gamma_out=2.2, gamma_in=2.5, r=0.1, seed=4), 5, "esu"),
    # 74 vertices of degree >= 256 with mixed arc types
    "hubs_n6000_k4": ("planted_hubs", dict(n=6000, m_bg=12_000, n_hubs=70, hub_deg=260, hub_links=8, r=0.2, seed=5),
                      4, "esu"),
    # full-size bench workloads, beyond ESU
    "chunglu_n1e5_m1e6_k4": (CL, dict(n=100_000, m=1_000_000, gamma_out=2.1, gamma_in=2.1, r=0.2, seed=2), 4,
                             "method_ref"),
    "chunglu_n2e4_m1e5_k5": (CL, dict(n=20_000, m=100_000, gamma_out=2.2, gamma_in=2.5, r=0.1, seed=4), 5,
                             "method_ref"),
    # undirected censuses (21 classes for k = 5) of the same workloads' undirected versions
    "chunglu_n2e4_m1e5_und5": (CL, dict(n=20_000, m=100_000, gamma_out=2.2, gamma_in=2.5, r=0.1, seed=4), 5,
                               "method_ref_undirected"),
    "gnm_n1000_und5": ("gnm_reciprocal", dict(n=1000, m0=5000, frac=0.1, seed=1), 5, "esu_undirected"),
}


def graph_of(name):
    gen, kw, k, _ = RECIPES[name]
    return getattr(gg, gen)(**kw), k


def make(name, threads=0):
    gen, kw, k, route = RECIPES[name]
    g = getattr(gg, gen)(**kw)
    t = time.time()
    if route == "esu":
        h = oracle.census(g, k, threads=threads)
    elif route == "method_ref":
        h = oracle.method_census(g, k, threads=threads)
    else:  # undirected census (classes of oracle.undirected_class_table)
        h = oracle.census_undirected(g, k, threads=threads, method=route == "method_ref_undirected")
    dt = time.time() - t
    out = {"name": name, "generator": gen, "params": kw, "k": k, "n": g.n, "m": g.m, "sha256": g.sha256(),
           "route": route, "oracle_seconds": round(dt, 1), "total": int(h.sum()),
           "hist": {str(c): int(v) for c, v in enumerate(h) if v}}
    if k == 4 and route == "method_ref":
        u = oracle.undirected4(g, threads=threads)
        out["undirected4"] = dict(zip(oracle.UNDIRECTED4, (int(x) for x in u)))
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=0)
    print(name, route, "done in", round(dt, 1), "s", flush=True)


if __name__ == "__main__":
    make(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 0)
