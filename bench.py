"""Throughput of the IBM-HT step on one MI355X.

One "step" is one pass of the whole hot path -- predictor, marker interpolation /
forcing / spreading, pressure set-up, pressure CG to convergence, correction -- on
the 2D heated-cylinder workload (1024^2 cells over [-4,12]x[-8,8], 400 candidate
markers, Re 100, Ma 0.2, Tw/Tinf 0.8), with all inputs resident in HBM.

Prints ONE JSON line: Mcell-steps/s, per-kernel roofline of the dominant kernel
(HIP events on the library's stream over the timed region), and the FP64 CPU
oracle timed on a bounded sample of the same workload.
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_words(cls: str, dim: int) -> int:
    """Algorithmic cell-array words each kernel class must move per cell (each
    distinct array element read or written once; face arrays counted as one word
    per cell and direction)."""
    return {
        "predictor": (2 * dim + 2) + (dim + 2),          # rho, m, E, F -> rho*, m*, E*
        "setup": (dim + 3) + (dim + 2) + (dim + 3) + (dim + 3),
        "cg_a": 3 + 2,                                    # r, p_old, psi -> p, q
        "cg_b": 4 + 2,                                    # x, p, r, q -> x, r
        "correct": (2 * dim + 4) + (2 * dim + 2),
    }[cls]


def traffic_entry(kernel: str, precision: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, when it was
    taken on the current kernel source; None otherwise."""
    path = os.path.join(ROOT, "profiles", "traffic_cylinder1024.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    src = os.path.join(ROOT, "paper_2301_09349_amd", "csrc", "ibm_grid.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    ent = rec.get(precision, {}).get(kernel)
    if not ent or ent.get("source_sha") != h:
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(case, steps: int):
    """The oracle as it stands, single-threaded, on `steps` steps of the workload."""
    from oracle.oracle import Oracle
    from paper_2301_09349_amd import inputs

    o = Oracle(case)
    rho, u, th = inputs.initial_fields(case)
    o.init_primitive(rho, u, th)
    X, Ud, Tw, dA = inputs.markers(case)
    o.set_markers(X, Ud, Tw, dA, dedupe=True)
    o.step(1)  # warm-up
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    ncell = 1
    for v in case["n"][: case["dim"]]:
        ncell *= v
    return {"value": ncell * steps / dt / 1e6, "unit": "Mcell-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} steps of the same 1024^2 workload after 1 warm-up step "
                      f"({dt:.1f} s, single thread, -O2 FP64)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--workload", default="cfg2a")
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the step runs on one MI355X); "
              "--gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2301_09349_amd import inputs
    from paper_2301_09349_amd.solver import IBMSolver

    case = inputs.case(args.workload, cg_rtol=1e-10)
    dim = case["dim"]
    N = int(np.prod(case["n"][:dim]))
    dev = torch.device("cuda:0")
    s = IBMSolver(case, args.precision, max_markers=case["ns"])
    rho, u, th = inputs.initial_fields(case)
    s.init_primitive(rho, u, th)
    X, Ud, Tw, dA = inputs.markers(case)
    s.set_markers(X, Ud, Tw, dA, dedupe=True)
    if case.get("motion"):
        m = case["motion"]
        s.set_motion(m["axis"], m["amp"], m["freq"])
    hist = torch.zeros((max(args.steps, args.warmup, 1), 4), dtype=torch.float64, device=dev)
    log(f"bench: {args.workload} {case['n']} {args.precision}, dt={s.dt:.4e}, "
        f"warmup {args.warmup}, steps {args.steps}")
    if args.warmup:
        s.step(args.warmup, hist_out=hist)
    torch.cuda.synchronize()
    s.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = s.step(args.steps, hist_out=hist)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = s.profile_read()
    s.profile(False)
    ids, _ = s.markers_in_use()
    value = N * args.steps / elapsed / 1e6
    ms_per_step = 1e3 * elapsed / args.steps
    cg_per_step = info["cg_iters_total"] / max(args.steps, 1)
    w = 4 if args.precision == "fp32" else 8
    per_kernel = {}
    for cls, (ms, n) in prof.items():
        if n == 0:
            continue
        ent = {"total_ms": ms, "launches": n, "avg_us": 1e3 * ms / n}
        if cls in ("predictor", "setup", "cg_a", "cg_b", "correct"):
            # the CG vectors stay FP64 in both precision forms
            ww = 8 if cls in ("cg_a", "cg_b") else w
            b = kernel_words(cls, dim) * ww * N
            ent["alg_bytes_per_launch"] = b
            ent["GBps"] = b / (ms / n * 1e-3) / 1e9
        per_kernel[cls] = ent
    dom = max((k for k in per_kernel if "GBps" in per_kernel[k]),
              key=lambda k: per_kernel[k]["total_ms"])
    d = per_kernel[dom]
    traffic = traffic_entry(dom, args.precision)
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(d["GBps"], 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(d["GBps"] / HBM_PEAK_GBS, 4),
            "traffic": traffic}
    log("bench: per-kernel " + json.dumps({k: {kk: (round(vv, 2) if isinstance(vv, float) else vv)
                                                 for kk, vv in v.items()}
                                             for k, v in per_kernel.items()}))
    out = {
        "metric": "Mcell-steps/s (fwd, FP32 vs FP64 at stated err) + adjoint/forward time ratio",
        "value": round(value, 2),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "2D heated cylinder, 1024x1024 cells over [-4,12]x[-8,8], "
                               "400 candidate markers (check routine keeps %d), Re 100, Ma 0.2, "
                               "Tw/Tinf 0.8, dt %.4e, CG rtol 1e-10" % (ids.shape[0], s.dt),
                   "cells": N, "precision": args.precision,
                   "cg_iters_per_step": round(cg_per_step, 2)},
        "roofline": roof,
        "kernels": {k: {"avg_us": round(v["avg_us"], 2), "launches": v["launches"],
                        **({"GBps": round(v["GBps"], 1)} if "GBps" in v else {})}
                    for k, v in per_kernel.items()},
    }
    if not args.no_cpu:
        log(f"bench: timing the oracle on {args.cpu_steps} steps ...")
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
