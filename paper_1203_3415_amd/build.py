"""Build the HIP shared library libmotif.so for gfx950 with hipcc.

Every source under csrc/ is compiled in place (no JIT cache), so the built
library sits next to the Python binding and travels with the source tree.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmotif.so")
SOURCES = ["classes.cpp", "graph.hip", "census.hip", "census6.hip", "nullmodel.hip", "api.cpp", "server.cpp",
           "ingest.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed fp32 instructions are kept out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-variable",
]


def build(verbose: bool = False) -> str:
    """Compile every source and link libmotif.so; returns its path."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with tempfile.TemporaryDirectory(prefix="motif_build_") as tmp:
        objs = []
        procs = []
        for src in srcs:
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
            if src.endswith(".cpp"):
                cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
            objs.append(obj)
        failed = []
        for src, p in procs:
            out, _ = p.communicate()
            text = out.decode(errors="replace")
            if p.returncode != 0:
                failed.append((src, text))
            elif verbose and text.strip():
                print(text)
        if failed:
            for src, text in failed:
                sys.stderr.write(f"--- {src}\n{text}\n")
            raise RuntimeError("hipcc failed for: " + ", ".join(s for s, _ in failed))
        tmp_lib = LIB + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp_lib, *objs, "-lpthread"]
        subprocess.check_call(cmd)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
