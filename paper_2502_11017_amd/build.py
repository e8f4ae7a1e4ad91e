"""Build libcur.so (HIP, gfx950) and the microbenchmark library libcurbench.so
in-tree with hipcc.

Usage: python -m paper_2502_11017_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcur.so")
BENCH_LIB = os.path.join(HERE, "libcurbench.so")  # the microbenchmarks (not part of the selection ABI)
BENCH_SOURCES = ["microbench.hip"]
SOURCES = ["api.hip", "select.hip", "pass.hip", "assemble.hip", "residual.hip", "residual_mp.hip", "greedy.hip",
           "propose.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Every decision of the selection is taken on explicitly written fma() chains;
# -ffp-contract=off keeps the compiler from fusing anything else.  Packed FP32
# instructions are disabled for every device pass.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-munsafe-fp-atomics", "-Wno-unused-result", "-I" + os.path.join(ROOT, "include")]


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compiles libcur.so and libcurbench.so; returns the path of libcur.so."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    all_src = SOURCES + BENCH_SOURCES
    objs = [os.path.join(objdir, src.replace(".hip", ".o")) for src in all_src]
    failed = []

    def finish(src, p, log):
        p.wait()
        log.seek(0)
        out = log.read()
        log.close()
        if p.returncode != 0:
            failed.append((src, out.decode(errors="replace")))
        elif verbose and out:
            sys.stdout.write(out.decode(errors="replace"))

    running = []  # at most `jobs` compilers at a time, each drained when it ends
    for src, obj in zip(all_src, objs):
        while len(running) >= jobs:
            done = [sp for sp in running if sp[1].poll() is not None]
            if not done:
                running[0][1].wait()
                continue
            for sp in done:
                finish(*sp)
                running.remove(sp)
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        log = tempfile.TemporaryFile()  # a file, not a pipe: a chatty compiler cannot block on it
        running.append((src, subprocess.Popen(cmd, stdout=log, stderr=subprocess.STDOUT), log))
    for sp in running:
        finish(*sp)
    if failed:
        for src, out in failed:
            sys.stderr.write(f"--- {src}\n{out}\n")
        raise RuntimeError("hipcc failed for " + ", ".join(s for s, _ in failed))
    for lib, o in ((LIB, objs[:len(SOURCES)]), (BENCH_LIB, objs[len(SOURCES):])):
        tmp = lib + ".tmp"
        subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *o])
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
