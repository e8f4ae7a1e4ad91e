"""Strong scaling of one selection over compute units, after the scalability
experiment of Sec. 3.2 (a 16384 x 16384 matrix, there over 2-64 processes).  On
one GPU the resource that grows is the number of compute units the process
may use; the ROCm runtime restricts every queue of a process to a set of them
when HSA_CU_MASK is set before it starts, so each count runs in a child
process of its own.

    python -m paper_2502_11017_amd.cusweep [--n 16384] [--r 64] [--cus 32 64 128 256] [--steps 3]

The matrix is the spectral construction of the 8192 x 8192 workload at size
n (singular values 0.9^i for i < 64, then 1e-6; N(0, 1e-7) noise), FP64,
built once on the GPU by a first child and handed to the others through a
file.  Each child runs the library's selection (column blocks of 64, default
options), warm calls first, and reports the mean wall time of the timed
calls and a digest of I and J, which must not depend on the compute units.
The parent never initialises the GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import tempfile


def _child_gen(path: str, n: int, seed: int) -> None:
    import numpy as np

    from paper_2502_11017_amd import workloads as W

    print(f"building {n} x {n}", flush=True)
    A = W.c2(seed=seed, device="cuda:0", n=n)
    np.save(path, A.cpu().numpy())
    print("saved", flush=True)


def _child_run(path: str, r: int, steps: int, warmup: int) -> None:
    import numpy as np
    import torch

    import paper_2502_11017_amd as cur

    A = torch.from_numpy(np.load(path)).to("cuda:0")
    for _ in range(warmup):  # warm-up calls also let the launch autotuner settle
        res = cur.select(A, r)
    torch.cuda.synchronize()
    ms = []
    for _ in range(steps):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        res = cur.select(A, r)
        t1.record()
        torch.cuda.synchronize()
        ms.append(t0.elapsed_time(t1))
    h = hashlib.sha256(res["I"].cpu().numpy().tobytes() + res["J"].cpu().numpy().tobytes()).hexdigest()[:16]
    print(json.dumps({"ms": sum(ms) / len(ms), "ms_all": ms, "status": res["status"], "swaps": res["swaps"],
                      "digest": h}), flush=True)


def _spawn(args, env=None, timeout=600) -> str:
    """Run a child, echo its lines as they come, return its stdout."""
    cmd = [sys.executable, "-u", "-m", "paper_2502_11017_amd.cusweep", *args]
    p = subprocess.Popen(cmd, env=env, stdout=subprocess.PIPE, text=True)
    lines = []
    for ln in p.stdout:
        lines.append(ln)
        if not ln.startswith("{"):
            print("  " + ln.rstrip(), flush=True)
    rc = p.wait(timeout=timeout)
    if rc != 0:
        raise RuntimeError(f"child {' '.join(args)} exited with {rc}")
    return "".join(lines)


def sweep(n=16384, r=64, cus=(32, 64, 128, 256), steps=3, warmup=3, seed=2, workdir=None):
    """Rows {cus, ms, status, swaps, digest} of one selection per CU count."""
    own = workdir is None
    workdir = workdir or tempfile.mkdtemp(prefix="cusweep_")
    path = os.path.join(workdir, f"c2_{n}.npy")
    if not os.path.exists(path):
        print(f"generating {n} x {n}", flush=True)
        _spawn(["--child-gen", path, "--n", str(n), "--seed", str(seed)])
    rows = []
    for k in cus:
        env = dict(os.environ)
        env["HSA_CU_MASK"] = f"0:0-{k - 1}"
        out = _spawn(["--child-run", path, "--r", str(r), "--steps", str(steps), "--warmup", str(warmup)], env=env)
        d = json.loads([ln for ln in out.splitlines() if ln.startswith("{")][-1])
        d["cus"] = k
        rows.append(d)
        print(f"cus {k:>4}  {d['ms']:9.2f} ms  status {d['status']}  swaps {d['swaps']}  I,J {d['digest']}",
              flush=True)
    os.remove(path)
    if own:
        os.rmdir(workdir)
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(prog="cusweep")
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--r", type=int, default=64)
    ap.add_argument("--cus", type=int, nargs="+", default=[32, 64, 128, 256])
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--workdir", default=None)
    ap.add_argument("--child-gen", default=None)
    ap.add_argument("--child-run", default=None)
    a = ap.parse_args(argv)
    if a.child_gen:
        _child_gen(a.child_gen, a.n, a.seed)
        return 0
    if a.child_run:
        _child_run(a.child_run, a.r, a.steps, a.warmup)
        return 0
    rows = sweep(a.n, a.r, a.cus, a.steps, a.warmup, a.seed, a.workdir)
    base = rows[0]
    out = {"n": a.n, "r": a.r, "rows": rows,
           "speedup_vs_first": [base["ms"] / x["ms"] for x in rows],
           "same_selection": len({x["digest"] for x in rows}) == 1}
    print(json.dumps(out), flush=True)
    return 0 if out["same_selection"] else 1


if __name__ == "__main__":
    sys.exit(main())
