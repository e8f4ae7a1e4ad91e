"""HBM and MFMA microbenchmarks on the current GPU (libcurbench.so).

    python -m paper_2502_11017_amd.microbench [--gib 4] [--reps 5]

Prints one line per probe and a JSON record: streaming read, write and copy
bandwidth over buffers of --gib GiB (bytes read plus written per second), and
dense MFMA throughput for the three instruction shapes the kernels use
(v_mfma_f64_16x16x4f64, v_mfma_f32_16x16x32_bf16, v_mfma_f32_16x16x32_fp8_fp8),
each against MI355X's published peak.  These are the measured ceilings beside
the published ones that the roofline fractions are quoted against.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PEAK = {"hbm": 8000.0, "fp64": 78.6, "bf16": 2500.0, "fp8": 5000.0}


def lib():
    path = os.path.join(HERE, "libcurbench.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2502_11017_amd.build")
    L = ctypes.CDLL(path)
    d = ctypes.POINTER(ctypes.c_double)
    L.curbench_stream.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int, d, d]
    L.curbench_mfma.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, d, d]
    return L


def run(gib=4.0, reps=5, cus=256):
    L = lib()
    out = {"stream": {}, "mfma": {}}
    v, t = ctypes.c_double(), ctypes.c_double()
    for kind, name in enumerate(("read", "write", "copy")):
        if L.curbench_stream(kind, int(gib * (1 << 30)), reps, ctypes.byref(v), ctypes.byref(t)) != 0:
            raise RuntimeError(f"stream {name} failed")
        out["stream"][name] = {"gbs": v.value, "ms": t.value, "frac_of_8000": v.value / PEAK["hbm"]}
        print(f"HBM {name:5s} {v.value:8.1f} GB/s ({v.value / PEAK['hbm']:.3f} of 8 TB/s), {t.value:.3f} ms", flush=True)
    for kind, (name, iters) in enumerate((("fp64", 10000), ("bf16", 20000), ("fp8", 20000))):
        blocks = 8 * cus
        if L.curbench_mfma(kind, iters, blocks, reps, ctypes.byref(v), ctypes.byref(t)) != 0:
            raise RuntimeError(f"mfma {name} failed")
        out["mfma"][name] = {"tflops": v.value, "ms": t.value, "peak": PEAK[name], "frac": v.value / PEAK[name],
                             "iters": iters, "blocks": blocks}
        print(f"MFMA {name:4s} {v.value:8.1f} TFLOP/s ({v.value / PEAK[name]:.3f} of {PEAK[name]:.1f}), "
              f"{t.value:.3f} ms", flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(prog="microbench")
    ap.add_argument("--gib", type=float, default=4.0)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args(argv)
    print(json.dumps(run(a.gib, a.reps)), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
