"""Write full-size golden histograms computed by the CPU oracle only.

Usage: python tests/golden/make_golden.py NAME [THREADS]

Each golden file records the generator recipe, the input's SHA-256 and the
oracle histogram (class id -> count; class ids as defined by the oracle's
canonical-code numbering).  Nothing here calls the GPU library.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

RECIPES = {
    "chunglu_n1e5_m1e6_k3": ("chung_lu", dict(n=100_000, m=1_000_000, gamma_out=2.1, gamma_in=2.1, r=0.2, seed=2), 3),
    "gnm_n1000_k3": ("gnm_reciprocal", dict(n=1000, m0=5000, frac=0.1, seed=1), 3),
    "gnm_n1000_k4": ("gnm_reciprocal", dict(n=1000, m0=5000, frac=0.1, seed=1), 4),
    "gnm_n1000_k5": ("gnm_reciprocal", dict(n=1000, m0=5000, frac=0.1, seed=1), 5),
    "chunglu_n2000_m8000_k4": ("chung_lu", dict(n=2000, m=8000, gamma_out=2.3, gamma_in=2.3, r=0.05, seed=3), 4),
}


def make(name, threads=0):
    gen, kw, k = RECIPES[name]
    g = getattr(gg, gen)(**kw)
    t = time.time()
    h = oracle.census(g, k, threads=threads)
    dt = time.time() - t
    out = {"name": name, "generator": gen, "params": kw, "k": k, "n": g.n, "m": g.m, "sha256": g.sha256(),
           "oracle_seconds": round(dt, 1), "total": int(h.sum()),
           "hist": {str(c): int(v) for c, v in enumerate(h) if v}}
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=0)
    print(name, "done in", round(dt, 1), "s", flush=True)


if __name__ == "__main__":
    make(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 0)
