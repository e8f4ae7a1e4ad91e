#!/usr/bin/env python3
"""Benchmark of the CUR hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): the C2 matrix,
8192 x 8192 FP64, A = Q1 diag(s) Q2^T + noise with s_i = 0.9^i for i < 64, a
flat 1e-6 floor afterwards, i.i.d. Gaussian noise of standard deviation 1e-7,
Q1/Q2 Haar (QR of seeded Gaussians); rank r = 64; leaf column blocks of 64
(128 leaves, 7 merge levels).  Synthetic data, generated on the GPU.

One step = the whole path on that matrix: cur_select (leaf ACA, maxvol swap
loops, binary merge tree) + cur_assemble (C, U, R) + cur_residual (Chebyshev
and Frobenius error).  The matrix is resident in HBM before timing starts.

Printed: ONE JSON line with the metric (CUR selections per second), the
swap-loop HBM GB/s (algorithmic bytes of the streaming pass kernel over its
summed HIP-event durations, each measured on the stream it was issued on),
the roofline record of that kernel, the CPU oracle timed on the same matrix, and the volume ratio of the GPU selection to
the oracle's.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 (vector and matrix)
TRAFFIC_FILE = {"pass": os.path.join(ROOT, "profiles", "pass_c2_traffic.json"),
                "fresh": os.path.join(ROOT, "profiles", "fresh_c2_traffic.json")}
PASS_SOURCE = os.path.join(ROOT, "paper_2502_11017_amd", "csrc", "pass.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kind):
    """HBM bytes per launch of the pass (kind "pass") or fresh-B ("fresh")
    kernel from the committed rocprofv3 counter summary, or None when their
    source changed since it was taken."""
    try:
        with open(TRAFFIC_FILE[kind]) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256_16") != source_hash(PASS_SOURCE):
        return None
    return t.get("bytes_per_launch")


def bench_e1(cur, W, torch, dev, reps=3):
    """Residual of the tall FP32 workload (1,048,576 x 1024, rank-128 Gaussian
    product + N(0, 1e-4) noise, r = 128) in the three precisions.  The FP32
    selection and assembly run once (untimed here); each residual is timed
    over `reps` calls.  The error of the BF16x3 and FP8 forms is taken against
    the native form (FP64 arithmetic on the FP32 data), which agrees with the
    FP64 oracle to 1e-10 ||A||_C (tests/test_gpu_mixed.py checks all three
    forms against the oracle at a reduced height)."""
    m, n, r = 1 << 20, 1024, 128
    log(f"e1: generating the tall FP32 workload {m}x{n} on the GPU")
    A = W.c4(seed=4, device=dev, m=m, n=n, k=128)
    torch.cuda.synchronize()
    a = time.perf_counter()
    res = cur.select(A, r)
    torch.cuda.synchronize()
    t_sel = time.perf_counter() - a
    C, U, R = cur.assemble(A, res["I"], res["J"])
    out = {"workload": f"{m}x{n} FP32, rank-128 Gaussian product + N(0,1e-4) noise, r={r}",
           "select_ms": 1e3 * t_sel, "select_status": res["status"], "forms": {}}
    ref = None
    for name, prec in (("native_fp64_arith", cur.PREC_NATIVE), ("bf16x3", cur.PREC_BF16X3), ("fp8", cur.PREC_FP8)):
        cur.residual(A, C, U, R, prec)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            cheb, fro = cur.residual(A, C, U, R, prec)
        torch.cuda.synchronize()
        t = (time.perf_counter() - a) / reps
        if ref is None:
            ref = (cheb, fro)
        f = {"ms": 1e3 * t, "cheb": cheb, "fro_rel": fro,
             "tflops": 2.0 * m * n * r / t / 1e12,
             "a_stream_gbs": m * n * 4 / t / 1e9,
             "cheb_rel_err_vs_native": abs(cheb - ref[0]) / ref[0],
             "fro_rel_err_vs_native": abs(fro - ref[1]) / ref[1]}
        out["forms"][name] = f
        log(f"e1 {name}: {1e3 * t:.2f} ms, cheb {cheb:.6e}, fro {fro:.6e}")
    del A, C, U, R
    torch.cuda.empty_cache()
    return out


def bench_e2(cur, W, torch, dev, reps=2):
    """The batched uneven form: 256 independent FP32 matrices, m and n uniform
    in [256, 4096], r in {8, 16, 32, 64}, geometric spectra with ratio uniform
    in [0.8, 0.95] (seeded).  All trees in one batched call, against the same
    matrices selected one call at a time; the per-item index sets of the two
    must agree."""
    specs = W.c3_specs()
    log(f"e2: generating {len(specs)} FP32 matrices")
    As = [W.c3_matrix(sp, device=dev, dtype=torch.float32) for sp in specs]
    rs = [sp[2] for sp in specs]
    torch.cuda.synchronize()
    for _ in range(3):  # the launch autotuner tries its candidates on each level shape
        cur.select_batched(As, rs)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(reps):
        outs, rc = cur.select_batched(As, rs)
    torch.cuda.synchronize()
    t_b = (time.perf_counter() - a) / reps
    a = time.perf_counter()
    # one call per matrix (every shape seen once, one node group per level)
    singles = [cur.select(A, r, groups=1) for A, r in zip(As, rs)]
    torch.cuda.synchronize()
    t_s = time.perf_counter() - a
    same = sum(int(torch.equal(I, g["I"]) and torch.equal(J, g["J"]) and st == g["status"])
               for (I, J, st), g in zip(outs, singles))
    short = sum(int(st == cur.ERR_RANK) for _, _, st in outs)
    elems = sum(A.numel() for A in As)
    out = {"workload": "256 FP32 matrices, m,n ~ U[256,4096], r in {8,16,32,64}, spectra ratio ~ U[0.8,0.95]",
           "matrices": len(As), "elements": elems,
           "batched_ms": 1e3 * t_b, "batched_selections_per_s": len(As) / t_b,
           "one_at_a_time_ms": 1e3 * t_s, "one_at_a_time_selections_per_s": len(As) / t_s,
           "speedup": t_s / t_b, "items_equal_single": same, "items_rank_short": short, "status_worst": rc}
    log(f"e2: batched {1e3 * t_b:.1f} ms, one at a time {1e3 * t_s:.1f} ms, equal {same}/{len(As)}")
    del As
    torch.cuda.empty_cache()
    return out


def bench_f1(cur, torch, A, r, res_maxvol, reps=3):
    """The paper's literal norm-greedy selection (Alg. 2 with Alg. 3, rows and
    columns independently) on the same C2 matrix; its cross volume against
    the maximal-volume selection's (log|det| of the r x r crosses, host LU)."""
    import numpy as np

    cur.select(A, r, method=cur.METHOD_GREEDY)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(reps):
        g = cur.select(A, r, method=cur.METHOD_GREEDY)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - a) / reps

    def logvol(I, J):
        G = A[I][:, J].double().cpu().numpy()
        return float(np.linalg.slogdet(G)[1])

    lg, lm = logvol(g["I"], g["J"]), logvol(res_maxvol["I"], res_maxvol["J"])
    out = {"workload": "C2 (same matrix), rows and columns by the norm-greedy rule, FP64",
           "select_ms": 1e3 * dt, "selections_per_s": 1.0 / dt, "status": g["status"],
           "logvol_greedy": lg, "logvol_maxvol": lm, "volume_ratio_greedy_over_maxvol": float(np.exp(lg - lm))}
    log(f"f1: norm-greedy {1e3 * dt:.1f} ms, volume ratio to the maximal-volume cross {out['volume_ratio_greedy_over_maxvol']:.3e}")
    return out


def bench_f2_polish(cur, torch, A, r, res_plain, t_plain, reps=3):
    """The optional whole-matrix polish on the same C2 matrix: the selection
    with one more node that runs the swap loop over all columns from the
    root's cross, its time against the plain selection's, and the volume it
    gains (the polished cross is dominant over the whole matrix)."""
    import numpy as np

    cur.select(A, r, polish=True)
    if t_plain is None:
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            cur.select(A, r)
        torch.cuda.synchronize()
        t_plain = (time.perf_counter() - a) / reps
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(reps):
        g = cur.select(A, r, polish=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - a) / reps
    out = {"workload": "C2 (same matrix), selection then the swap loop over all 8192 columns from the root's cross",
           "select_ms": 1e3 * dt, "plain_select_ms": 1e3 * t_plain, "status": g["status"],
           "polish_swaps": g["swaps"] - res_plain["swaps"], "nodes": g["nodes"],
           "volume_ratio_vs_plain": float(np.exp(g["logvol"] - res_plain["logvol"]))}
    log(f"f2: polished selection {1e3 * dt:.1f} ms (plain {1e3 * t_plain:.1f} ms), {out['polish_swaps']} more swaps, "
        f"volume ratio to the plain cross {out['volume_ratio_vs_plain']:.3e}")
    return out


def bench_e4(cur, torch, A, r, res_plain, t_plain, reps=3):
    """The learned candidate proposal on the same C2 matrix: the selection
    time with the shipped weights (features, scores, restricted starts and
    the verifying swap loops included), the feature pass alone, and the
    volume of the cross it ends with against the plain selection's."""
    import numpy as np

    from paper_2502_11017_amd import learn

    blob = learn.load_blob(device=A.device)
    if t_plain is None:
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            cur.select(A, r)
        torch.cuda.synchronize()
        t_plain = (time.perf_counter() - a) / reps
    cur.select(A, r, mlp=blob, seed=7)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(reps):
        g = cur.select(A, r, mlp=blob, seed=7)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - a) / reps
    a = time.perf_counter()
    for _ in range(reps):
        cur.mlp_features(A, r, seed=7)
    torch.cuda.synchronize()
    tf = (time.perf_counter() - a) / reps
    out = {"workload": "C2 (same matrix), learned proposal with the shipped weights, FP64",
           "select_ms": 1e3 * dt, "plain_select_ms": 1e3 * t_plain, "features_ms": 1e3 * tf,
           "speedup_vs_plain": t_plain / dt, "status": g["status"], "swaps": g["swaps"],
           "swaps_plain": res_plain["swaps"], "volume_ratio_vs_plain": float(np.exp(g["logvol"] - res_plain["logvol"]))}
    log(f"e4: learned {1e3 * dt:.1f} ms (plain {1e3 * t_plain:.1f} ms, features {1e3 * tf:.2f} ms), "
        f"volume ratio to the plain cross {out['volume_ratio_vs_plain']:.3f}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3,
                    help="untimed steps; the first three also let the launch autotuner try its candidates")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f32", action="store_true")
    ap.add_argument("--no-stages", action="store_true", help="skip the per-stage breakdown")
    ap.add_argument("--host-matrix", action="store_true",
                    help="build the C2 matrix on the host and copy it over (for counter runs)")
    ap.add_argument("--no-e1", action="store_true",
                    help="skip the reduced-precision residual figures on the tall FP32 workload")
    ap.add_argument("--no-e2", action="store_true", help="skip the batched uneven-workload figures")
    ap.add_argument("--no-e4", action="store_true", help="skip the learned-proposal figures")
    ap.add_argument("--no-f1", action="store_true", help="skip the norm-greedy (paper-literal) selection figures")
    ap.add_argument("--no-f2", action="store_true", help="skip the whole-matrix polish figures")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of the launch autotuner cache: loaded before the run when it exists, "
                         "written at the end (profiling runs reuse the tuned launch shapes)")
    ap.add_argument("--groups", type=int, default=0,
                    help="node groups (streams) per tree level of the C2 selection: 0 autotuned, 1 one stream "
                         "(a single-stream kernel timeline), 2 or 3")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="one untimed device copy of this size, the calibration of the byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding of the merge tree is a design note only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2502_11017_amd as cur
    from paper_2502_11017_amd import workloads as W

    dev = torch.device("cuda:0")
    if args.tune_cache and os.path.exists(args.tune_cache):
        with open(args.tune_cache) as f:
            cur.tune_import(json.load(f))
        log(f"autotuner cache loaded from {args.tune_cache}")
    m = n = 8192
    r = 64
    if args.host_matrix:
        log(f"generating C2 {m}x{n} seed {args.seed} on the host")
        A = W.c2(args.seed, device="cpu", n=n).to(dev)
    else:
        log(f"generating C2 {m}x{n} seed {args.seed} on the GPU")
        A = W.c2(args.seed, device=dev, n=n)
    torch.cuda.synchronize()
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {src.numel() * 8} bytes read and written")
        del src, dst

    def step(Ax):
        res = cur.select(Ax, r, groups=args.groups)
        C, U, R = cur.assemble(Ax, res["I"], res["J"])
        cheb, fro = cur.residual(Ax, C, U, R)
        return res, cheb, fro

    for k in range(args.warmup):
        log(f"warmup {k + 1}/{args.warmup}")
        step(A)
    torch.cuda.synchronize()

    # The roofline's HIP events (a pair around every pass and fresh launch, on
    # the launch's own stream, read back after each selection: ~4.7 ms of host
    # work per C2 selection) are taken in the last timed step only; its 600+
    # pass launches give the per-launch average.
    prof_steps = 1
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    t0 = time.perf_counter()
    for k in range(args.steps):
        if k == args.steps - prof_steps:
            cur.profile_enable(2)
        res, cheb, fro = step(A)
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = cur.profile_read()
    cur.profile_enable(False)
    total_s = max(t1 - t0, ev0.elapsed_time(ev1) * 1e-3)
    ms_per_step = 1e3 * total_s / args.steps
    sel_per_s = args.steps / total_s
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step")

    # per-stage breakdown (separate, untimed for the metric)
    def timed(fn, reps=3):
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - a) / reps, out

    if args.no_stages:
        t_sel = t_asm = t_res = None
        C, U, R = cur.assemble(A, res["I"], res["J"])
        res_tflops = None
    else:
        t_sel, res = timed(lambda: cur.select(A, r))
        t_asm, (C, U, R) = timed(lambda: cur.assemble(A, res["I"], res["J"]))
        t_res, (cheb, fro) = timed(lambda: cur.residual(A, C, U, R))
        res_tflops = 2.0 * m * n * r / t_res / 1e12

    def roof(kind):
        """Roofline record of one row kernel over the timed region: achieved =
        the in-place algorithm's bytes (an elimination step reads and writes
        the active columns, a row swap the m x r matrix B, a fresh B reads
        A(:, J) and writes B) / the summed HIP-event time of its launches; the
        bytes this implementation moves (lazy row swaps) beside it."""
        pre = "fresh_" if kind == "fresh" else ""
        sec, n_l = prof[pre + "seconds"], max(prof[pre + "launches"], 1)
        b_model, b_impl = prof[pre + "bytes_inplace"], prof[pre + "bytes"]
        ach = b_model / sec / 1e9 if sec > 0 else 0.0
        return {"bound": "hbm",
                "kernel": ("k_fresh (fresh interpolation matrix B = A(:,J) A(I,J)^-1)" if kind == "fresh"
                           else "k_pass (streaming row pass: ACA updates, row swaps)"),
                "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "algorithmic_bytes_per_launch": b_model / n_l,
                "implementation_bytes_per_launch": b_impl / n_l,
                "achieved_implementation_bytes_gbs": b_impl / sec / 1e9 if sec > 0 else 0.0,
                "launches_per_step": prof[pre + "launches"] / prof_steps,
                "busy_launches_per_step": prof[pre + "busy"] / prof_steps,
                "avg_launch_us": 1e6 * sec / n_l,
                # context: the same bytes over the busy launches only (a
                # launch that finds no node in its state returns at once)
                "achieved_busy_launches_gbs": (b_model / prof[pre + "busy_seconds"] / 1e9
                                               if prof[pre + "busy_seconds"] > 0 else 0.0),
                "avg_busy_launch_us": 1e6 * prof[pre + "busy_seconds"] / max(prof[pre + "busy"], 1),
                "timed_steps_with_events": prof_steps}

    roof_pass, roof_fresh = roof("pass"), roof("fresh")
    pass_gbs = roof_pass["achieved"]
    roof_pass["traffic"] = measured_traffic("pass")
    roof_fresh["traffic"] = measured_traffic("fresh")

    I = res["I"].cpu().numpy()
    J = res["J"].cpu().numpy()
    Ah = None
    cpu = None
    vol_ratio = None
    exact = None
    if not args.no_cpu_baseline:
        from oracle import oracle as orc

        Ah = A.cpu().numpy()
        log("cpu_baseline: oracle selection on the same matrix (single thread)")
        a = time.perf_counter()
        o = orc.select(Ah, r)
        t_orc = time.perf_counter() - a
        cpu = {"value": 1.0 / t_orc, "unit": "selections/s", "cores": 1, "kind": "oracle",
               "sample": f"one full C2 selection (8192x8192 FP64, r=64, 128 leaves), {t_orc:.1f} s "
                         "on one host core; assembly and residual not included"}
        exact = bool(np.array_equal(I, o["I"]) and np.array_equal(J, o["J"]))
        vol_ratio = float(np.exp(orc.logvol(Ah, I, J) - orc.logvol(Ah, o["I"], o["J"])))
        log(f"oracle {t_orc:.1f} s; indices equal: {exact}; volume ratio {vol_ratio:.6f}")

    f32 = None
    if not args.no_f32:
        A32 = A.to(torch.float32)
        for _ in range(3):  # autotuner candidates on this shape
            cur.select(A32, r)
        t32, r32 = timed(lambda: cur.select(A32, r))
        f32 = {"select_ms": 1e3 * t32, "selections_per_s": 1.0 / t32, "status": r32["status"]}
        if Ah is not None:
            from oracle import oracle as orc

            A32h = A32.cpu().numpy().astype(np.float64)
            f32["volume_ratio_vs_f64_selection"] = float(np.exp(
                orc.logvol(A32h, r32["I"].cpu().numpy(), r32["J"].cpu().numpy())
                - orc.logvol(A32h, I, J)))
        del A32

    f1 = None
    if not args.no_f1:
        f1 = bench_f1(cur, torch, A, r, res)
    f2 = None
    if not args.no_f2:
        f2 = bench_f2_polish(cur, torch, A, r, res, t_sel)
    e1 = None
    if not args.no_e1:
        e1 = bench_e1(cur, W, torch, dev)
    e2 = None
    if not args.no_e2:
        e2 = bench_e2(cur, W, torch, dev)
    e4 = None
    if not args.no_e4:
        e4 = bench_e4(cur, torch, A, r, res, t_sel)

    out = {
        "metric": "CUR selections/sec + swap-loop HBM GB/s at volume ratio >=0.99 vs FP64 oracle",
        "value": sel_per_s,
        "unit": "selections/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "C2: 8192x8192 FP64, s_i=0.9^i (i<64) then 1e-6, noise std 1e-7, "
                               "r=64, column blocks of 64 (128 leaves), select+assemble+residual",
                   "m": m, "n": n, "r": r, "col_block": 64, "seed": args.seed},
        "swap_loop_gbs": pass_gbs,
        "volume_ratio": vol_ratio,
        "indices_equal_oracle": exact,
        "roofline": roof_pass,
        "roofline_fresh": roof_fresh,
        "stages_ms": None if args.no_stages else {"select": 1e3 * t_sel, "assemble": 1e3 * t_asm,
                                                  "residual": 1e3 * t_res},
        "residual": {"cheb": cheb, "fro_rel": fro, "tflops": res_tflops,
                     "frac_fp64_peak": None if res_tflops is None else res_tflops / FP64_PEAK_TFLOPS},
        "selection": {"status": res["status"], "swaps": res["swaps"], "phases": res["phases"],
                      "refreshes": res["refreshes"], "nodes": res["nodes"], "logvol": res["logvol"]},
        "f32": f32,
        "e1_reduced_precision_residual": e1,
        "e2_batched_uneven": e2,
        "f1_paper_greedy": f1,
        "f2_polish": f2,
        "e4_learned_proposal": e4,
        "cpu_baseline": cpu,
    }
    if args.tune_cache:
        with open(args.tune_cache, "w") as f:
            json.dump(cur.tune_export(), f)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
