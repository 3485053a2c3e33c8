"""Throughput of the IBM-HT step on one MI355X.

One "step" is one pass of the whole hot path -- predictor, marker interpolation /
forcing / spreading, pressure set-up, pressure CG to convergence, correction -- on
the 3D heated-sphere workload (256^3 cells over [-2.5,7.5]x[-4,4]^2, 3200 Fibonacci
candidate markers, Re 300, Ma 0.3, Tw/Tinf 1.5), with all inputs resident in HBM.

Prints ONE JSON line: FP64 Mcell-steps/s (``value``), the FP32 form's throughput and
its error against the FP64 run (per result: velocity, temperature, Nusselt number,
drag; over full-length runs of the 1024^2 cylinder and the 256^3 sphere), the
adjoint/forward time ratio on the gradient workload (512^2 cylinder, van Leer
convection, 200 markers, checkpoints every 50), the roofline of the dominant kernel
(HIP events on the library's stream over the timed region), other workloads as
extra legs, and the FP64 CPU oracle timed on a bounded sample of the same workload.

``--summarize DIR`` (no GPU) turns rocprofv3 output of this script into the text
summaries kept under profiles/.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
CALIB_ELEMS = 1 << 26  # float64 elements of the copy-kernel calibration (512 MiB)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def refine32(dim: int, precision: str) -> bool:
    """Whether the FP32 form solves by refinement around an FP32 inner CG: the
    library's default in 3D, IBM_FP32_SOLVE=refine|fp64 overriding it."""
    if precision != "fp32":
        return False
    env = os.environ.get("IBM_FP32_SOLVE", "")
    return env == "refine" or (env != "fp64" and dim == 3)


def kernel_bytes(cls: str, dim: int, precision: str = "fp64", scheme: int = 0) -> int:
    """Algorithmic bytes each kernel class must move per cell (each distinct array
    element read or written once; face arrays counted as one value per cell and
    direction). State-type arrays take s bytes (8 FP64, 4 FP32); the pressure x, the
    right-hand side b and the FP64 CG vectors take 8 in both forms. The FP32 form's
    solve by refinement has FP32 CG vectors (an inner iteration's figure is given
    for its launches) and its set-up leaves the CG start to the solve."""
    s = 8 if precision == "fp64" else 4
    if scheme == 0 and refine32(dim, precision):
        if cls == "setup":
            # rho^n, m^, psi, F^ (FP32), x, b (FP64), the start residual (FP32)
            return 4 * (2 * dim + 2) + 8 * 2 + 4
        if cls == "cg":
            # inner iteration: psi, r, w, s_old, p, d -> r', w', s, p, d, all FP32
            return 4 * 11
    if scheme == 1:  # density-based step
        if cls == "predictor":
            # inviscid: rho, m, E -> rho*, (rho u)**, (rho e_t)**, face mass flux;
            # viscous: rho*, (rho u)**, (rho e_t)** -> m*, E*
            return s * (3 * (dim + 2) + dim + dim + 1)
        if cls == "correct":
            # rho*, m**, E** -> the new state
            return s * 2 * (dim + 2)
        raise KeyError(cls)
    if cls == "predictor":
        # rho, m, E, F and the three previous E (four-point extrapolated start) ->
        # rho*, m*, E*, m^, psi, the kept E^{n-1}, E^{n-2} (state type) and x (FP64)
        return s * ((2 * dim + 5) + (2 * dim + 5)) + 8
    if cls == "setup":
        # rho^n, m^, psi, F^ (state type), x, b, r0 (FP64); then the CG start
        # psi, r0 -> w0 (both forms run the FP64 CG)
        return s * (2 * dim + 2) + 8 * 3 + s + 8 * 2
    if cls == "correct":
        # rho*, E*, m^, F^, rho^n, x -> F, m, rho, E
        return s * ((2 * dim + 3) + (2 * dim + 2)) + 8
    if cls == "cg":
        # single-reduction CG: r, w, s_old, p, x, psi -> r', w', s, p, x; the vectors
        # FP64 in both forms, psi in the state type
        return 8 * 10 + s
    raise KeyError(cls)


# kernel symbol prefix -> kernel class of the library's event timing
KERNEL_CLASS = [("k_predictor", "predictor"), ("k_setup", "setup"), ("k_cg_start", "setup"),
                ("k_cg_iter", "cg"), ("k_mcg_iter", "cg"),
                # the column CG's start (template argument 0) belongs to the set-up
                ("k_cg_col<0", "setup"), ("k_cg_col", "cg"), ("k_mcg_col", "cg"),
                ("k_correct", "correct"), ("k_interp_force", "markers"), ("k_spread", "markers"),
                ("k_totals", "markers"), ("k_markers_fused", "markers"),
                ("k_dsys", "diffusion"), ("k_diff_coef", "diffusion"),
                ("k_dens_inviscid", "predictor"),
                ("k_dens_viscous", "predictor"),
                ("k_dens_finish", "correct"),
                ("k_rebuild_small", "rebuild"), ("k_eps_cg_wave", "rebuild")]


def kernel_class(name: str):
    """Class of a kernel from its demangled name (``void ibmk::k_setup2<2, double>(...)``)."""
    m = re.search(r"ibmk::(\w+)(<[^>]*>)?", name)
    if not m:
        return None
    sym = m.group(1) + (m.group(2) or "")
    for key, cls in KERNEL_CLASS:
        if sym.startswith(key):
            return cls
    return None


def source_sha() -> str:
    h = hashlib.sha256()
    for f in ("ibm_grid.hip", "ibm_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2301_09349_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


WORKLOAD_LABEL = {"cfg1": "cylinder128", "cfg2a": "cylinder1024", "cfg2b": "cylinder1024",
                  "cfg2": "cylinder1024", "cfg3": "sphere256", "cfg4": "moving512",
                  "cfg5": "gradient512", "osc1": "oscillating512", "osc2": "oscillating512"}


def traffic_entry(label: str, kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this
    workload and precision (profiles/traffic_<label>.json), when it was taken on the
    current kernel source; None otherwise."""
    path = os.path.join(ROOT, "profiles", f"traffic_{label}.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    ent = rec.get("classes", {}).get(kernel)
    if not ent or rec.get("source_sha") != source_sha():
        return None
    return ent.get("bytes_per_launch")


def host_info():
    """CPU model and logical CPU count of the host (lscpu, os.cpu_count)."""
    model = ""
    try:
        import subprocess

        for line in subprocess.run(["lscpu"], capture_output=True, text=True).stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    return {"cpu": model, "nproc": os.cpu_count()}


def cpu_baseline(case, steps: int):
    """The oracle as it stands (plain FP64 loops, one thread; built here with -O3
    -march=native, still without FMA contraction) on `steps` steps of the workload
    after its set-up (grid, markers, quadrature solve; not timed)."""
    from oracle import oracle as orc
    from paper_2301_09349_amd import inputs

    orc.use_native()
    o = orc.Oracle(case)
    rho, u, th = inputs.initial_fields(case)
    o.init_primitive(rho, u, th)
    X, Ud, Tw, dA = inputs.markers(case)
    o.set_markers(X, Ud, Tw, dA, dedupe=True)
    t0 = time.perf_counter()
    h = o.step(steps)
    dt = time.perf_counter() - t0
    ncell = 1
    for v in case["n"][: case["dim"]]:
        ncell *= v
    cells = "x".join(str(v) for v in case["n"][: case["dim"]])
    return {"value": round(ncell * steps / dt / 1e6, 3), "unit": "Mcell-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} step(s) of the same workload ({cells} cells, "
                      f"{int(h[:, 5].sum())} CG iterations) after its set-up, {dt:.1f} s; one "
                      "thread, g++ -O3 -march=native -ffp-contract=off, FP64",
            "host": host_info()}


def make_solver(case, precision, tape_steps=0):
    from paper_2301_09349_amd import inputs
    from paper_2301_09349_amd.solver import IBMSolver

    s = IBMSolver(case, precision, max_markers=case["ns"], tape_steps=tape_steps)
    rho, u, th = inputs.initial_fields(case)
    s.init_primitive(rho, u, th)
    X, Ud, Tw, dA = inputs.markers(case)
    s.set_markers(X, Ud, Tw, dA, dedupe=True, no_heat=bool(case.get("no_heat", False)))
    if case.get("motion"):
        m = case["motion"]
        s.set_motion(m["axis"], m["amp"], m["freq"])
    return s


def run_forward(case, precision, steps, warmup):
    """Times `steps` steps after `warmup` with kernel timing off (the throughput),
    then `steps` more with the library's per-class HIP events on its stream (the
    kernel durations; the events slow the step a little)."""
    import numpy as np
    import torch

    dim = case["dim"]
    N = int(np.prod(case["n"][:dim]))
    s = make_solver(case, precision)
    hist = torch.zeros((max(steps, warmup, 1), 4), dtype=torch.float64, device="cuda:0")
    log(f"bench: {case['n']} {precision}, dt={s.dt:.4e}, warmup {warmup}, steps {steps}")
    it_all = 0
    if warmup:
        _, wi = s.step(warmup, hist_out=hist)
        it_all += wi["cg_iters_total"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, info = s.step(steps, hist_out=hist)
    it_all += info["cg_iters_total"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    h_timed = hist[:steps].clone()
    s.profile(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, pi = s.step(steps, hist=False)
    it_all += pi["cg_iters_total"]
    torch.cuda.synchronize()
    elapsed_prof = time.perf_counter() - t1
    prof = s.profile_read()
    s.profile(False)
    per_kernel = {}
    for cls, (ms, n) in prof.items():
        if n == 0:
            continue
        ent = {"total_ms": ms, "launches": n, "avg_us": 1e3 * ms / n,
               "ms_per_step": ms / steps}
        if cls in (("predictor", "correct") if case.get("scheme", 0) == 1 else
                   ("predictor", "setup", "cg", "correct")):
            b = kernel_bytes(cls, dim, precision, case.get("scheme", 0)) * N
            ent["alg_bytes_per_launch"] = b
            ent["GBps"] = b / (ms / n * 1e-3) / 1e9
        per_kernel[cls] = ent
    return {"solver": s, "N": N, "elapsed": elapsed, "info": info, "per_kernel": per_kernel,
            "hist": h_timed, "value": N * steps / elapsed / 1e6,
            "ms_per_step": 1e3 * elapsed / steps,
            "ms_per_step_profiled": 1e3 * elapsed_prof / steps, "cg_iters_all": it_all}


def fp32_error(r64, r32):
    """Error of the FP32 form against the FP64 run after the same steps: velocity and
    temperature (relative L2; temperature as theta - 1), and the time-averaged drag
    and heat (relative)."""
    import torch

    def prim(s):
        r, m, e, _ = s.get_state()
        r, m, e = r.double(), m.double(), e.double()
        cv = 1.0 / (s.case["gamma"] * s.case["Ma"] ** 2) / (s.case["gamma"] - 1.0)
        return m / r, e / (r * cv)

    u64, t64 = prim(r64["solver"])
    u32, t32 = prim(r32["solver"])
    h64, h32 = r64["hist"], r32["hist"]
    rel = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
    return {"u": rel(u32, u64), "theta_minus_1": rel(t32 - 1.0, t64 - 1.0),
            "drag_mean": abs(float(h32[:, 0].mean() / h64[:, 0].mean()) - 1.0),
            "heat_mean": abs(float(h32[:, 3].mean() / h64[:, 3].mean()) - 1.0)}


def run_adjoint(steps: int, checkpoint: int, warmup: int, precision: str = "fp64"):
    """Adjoint/forward time ratio on the gradient workload. forward = `steps` plain
    steps; backward = what the gradient costs beyond them: the rollout's forward pass
    (checkpoints, and its last segment recorded on the tape) less the plain steps,
    then the reverse pass (each earlier segment re-run with the tape on, one adjoint
    step per step). Also with a tape of all the steps (nothing re-run)."""
    import numpy as np
    import torch

    from paper_2301_09349_amd import inputs
    from paper_2301_09349_amd.adjoint import (Rollout, nusselt_scale, _set_state_vector,
                                              _state_vector)

    case = inputs.case("cfg5")
    out = {"workload": "2D heated cylinder, 512x512 over [-4,12]x[-8,8], 200 candidate "
                       "markers, Re 100, Ma 0.2, Tw 1.3, van Leer convection, CG rtol 1e-13; "
                       "gradient of the time-averaged Nusselt number w.r.t. T_w",
           "steps": steps, "checkpoint": checkpoint, "precision": precision}
    for label, ckpt in (("", checkpoint), ("_tape_all_steps", steps)):
        s = make_solver(case, precision, tape_steps=ckpt)
        if warmup:
            s.step(warmup)
        x0 = _state_vector(s)
        step0 = warmup
        _set_state_vector(s, x0, step0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps, hist=False)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        _set_state_vector(s, x0, step0)
        roll = Rollout(s, steps, ckpt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        roll.forward()
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        ob = np.zeros((steps, 4))
        ob[:, 3] = nusselt_scale(case) / steps
        # the reverse pass of Rollout.reverse, with its two parts timed apart
        sb = torch.zeros(s.state_size, dtype=torch.float64, device="cuda:0")
        sb2 = torch.empty_like(sb)
        Tw_bar = torch.zeros(s.nc, dtype=torch.float64, device="cuda:0")
        t_rec = t_adj = 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for idx in reversed(range(len(roll.segs))):
            start, k, ck, st_step = roll.segs[idx]
            ta = time.perf_counter()
            if idx != roll.taped or s.tape_length() != k:
                _set_state_vector(s, ck, st_step)
                s.step(k, hist=False, record=True)
            roll.taped = None
            torch.cuda.synchronize()
            tb = time.perf_counter()
            for i in reversed(range(k)):
                s.adjoint_step(i, sb, sb2, ob[start + i], Tw_bar)
                sb, sb2 = sb2, sb
            torch.cuda.synchronize()
            tc = time.perf_counter()
            t_rec += tb - ta
            t_adj += tc - tb
        t_rev = time.perf_counter() - t0
        t_back = (t_fwd - t_plain) + t_rev
        ent = {"forward_ms_per_step": round(1e3 * t_plain / steps, 4),
               "rollout_forward_ms_per_step": round(1e3 * t_fwd / steps, 4),
               "backward_ms_per_step": round(1e3 * t_back / steps, 4),
               "recompute_ms_per_step": round(1e3 * t_rec / steps, 4),
               "adjoint_step_ms": round(1e3 * t_adj / steps, 4),
               "ratio": round(t_back / t_plain, 3),
               "ratio_adjoint_step_only": round(t_adj / t_plain, 3),
               "grad_norm": float(torch.linalg.norm(Tw_bar))}
        if label:
            out["tape_all_steps"] = {k: v for k, v in ent.items()
                                     if k in ("backward_ms_per_step", "ratio", "grad_norm")}
        else:
            out.update(ent)
        del s, roll
        torch.cuda.empty_cache()
    return out


def run_cylinder(steps: int, warmup: int):
    """The 2D workload (1024^2 heated cylinder, 400 candidate markers, Re 100, Ma 0.2,
    Tw 0.8) in both forms. Its FP64 working set (~250 MB) fits the 256 MB Infinity
    Cache, so its kernels' GB/s are not HBM figures."""
    from paper_2301_09349_amd import inputs

    case = inputs.case("cfg2a", cg_rtol=1e-10)
    res = {"steps": steps}
    for prec in ("fp64", "fp32"):
        r = run_forward(case, prec, steps, warmup)
        if "workload" not in res:
            kept = r["solver"].markers_in_use()[0].shape[0]
            res["workload"] = workload_text(case, kept, r["solver"].dt)
        res[prec] = {"value": round(r["value"], 2), "ms_per_step": round(r["ms_per_step"], 4),
                     "dt": r["solver"].dt,
                     "cg_iters_per_step": round(r["info"]["cg_iters_total"] / steps, 2),
                     "kernels": {k: {"avg_us": round(v["avg_us"], 2),
                                     **({"GBps": round(v["GBps"], 1)} if "GBps" in v else {})}
                                 for k, v in r["per_kernel"].items()}}
        del r
    return res


def fp32_errors_full(runs):
    """The FP32 form against the FP64 GPU path (itself pinned to the oracle) over
    full-length runs of the same workload from the same start: velocity and
    temperature at the end (relative L2; temperature as theta - 1), and the
    time-averaged Nusselt number and drag coefficient (relative). `runs` lists
    (workload name, overrides, steps)."""
    import numpy as np
    import torch

    from paper_2301_09349_amd import inputs

    out = {}
    for name, over, steps in runs:
        case = inputs.case(name, cg_rtol=1e-10, **over)
        res = {}
        for prec in ("fp64", "fp32"):
            s = make_solver(case, prec)
            hist = torch.zeros((steps, 4), dtype=torch.float64, device="cuda:0")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(steps, hist_out=hist)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            r, m, e, _ = s.get_state()
            r, m, e = r.double(), m.double(), e.double()
            cv = 1.0 / (case["gamma"] * case["Ma"] ** 2) / (case["gamma"] - 1.0)
            res[prec] = (m / r, e / (r * cv), hist.cpu().numpy(), el)
            del s
        u64, t64, h64, e64 = res["fp64"]
        u32, t32, h32, e32 = res["fp32"]
        rel = lambda a, b: float(torch.linalg.norm(a - b) / torch.linalg.norm(b))  # noqa: E731
        nu = abs(h32[:, 3].mean() / h64[:, 3].mean() - 1.0)
        cd = abs(h32[:, 0].mean() / h64[:, 0].mean() - 1.0)
        key = name + "".join(f"_{k}{v}" for k, v in over.items())
        out[key] = {"steps": steps, "u": float("%.3g" % rel(u32, u64)),
                    "theta_minus_1": float("%.3g" % rel(t32 - 1.0, t64 - 1.0)),
                    "nusselt_mean": float("%.3g" % nu), "drag_mean": float("%.3g" % cd),
                    "ms_per_step_fp64": round(1e3 * e64 / steps, 4),
                    "ms_per_step_fp32": round(1e3 * e32 / steps, 4)}
        log(f"bench: FP32 vs FP64 on {key}: {out[key]}")
        torch.cuda.empty_cache()
    return out


def shedding_frequency(scheme: int, t_end: float = 250.0, window: float = 100.0):
    """Sec. 5's preliminary run: the cylinder of the oscillating cases held fixed (512^2,
    200 candidate markers, Re 100, Ma 0.3, Tw/Tinf 1, FP64) from the perturbed free
    stream to t_end D/U on the given step (0 pressure-based, 1 density-based); the
    shedding frequency f_0 from the lift coefficient C_l = 2 F_y / (rho U^2 D) over
    the last `window` time units: the mean period between upward zero crossings of C_l
    minus its mean (each crossing located by linear interpolation), with the FFT peak
    of the same window (Hann window, parabolic interpolation of the log magnitude) and
    its three strongest peaks as checks."""
    import numpy as np
    import torch
    from paper_2301_09349_amd import inputs

    case = inputs.case("osc1", cg_rtol=1e-10, scheme=scheme)
    case["motion"] = None
    case["dt_u_max"] = 0.0
    s = make_solver(case, "fp64")
    dt = s.dt
    n = int(math.ceil(t_end / dt))
    chunk = 20000
    hist = torch.zeros((chunk, 4), dtype=torch.float64, device="cuda:0")
    cl = np.empty(n)
    cd = np.empty(n)
    log(f"bench: fixed cylinder for f_0 (scheme {scheme}), {n} steps of dt {dt:.4e}")
    t0 = time.perf_counter()
    done = 0
    while done < n:
        k = min(chunk, n - done)
        s.step(k, hist_out=hist)
        h = hist[:k].cpu().numpy()
        cd[done:done + k] = 2.0 * h[:, 0]
        cl[done:done + k] = 2.0 * h[:, 1]
        done += k
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    del s
    t = dt * (np.arange(n) + 1)
    sel = t >= t_end - window
    tw, c = t[sel], cl[sel] - cl[sel].mean()
    up = np.nonzero((c[:-1] < 0.0) & (c[1:] >= 0.0))[0]
    tc = tw[up] - c[up] * (tw[up + 1] - tw[up]) / (c[up + 1] - c[up])
    per = np.diff(tc)
    f0 = 1.0 / per.mean() if len(per) > 1 else float("nan")
    spec = np.abs(np.fft.rfft(c * np.hanning(len(c))))
    freqs = np.fft.rfftfreq(len(c), dt)
    i = 1 + int(np.argmax(spec[1:]))
    la, lb, lc = np.log(spec[i - 1:i + 2])
    f_fft = freqs[i] + 0.5 * (la - lc) / (la - 2.0 * lb + lc) * (freqs[1] - freqs[0])
    top = np.argsort(spec[1:])[::-1][:3] + 1
    return {"scheme": "density-based" if scheme == 1 else "pressure-based",
            "f0": round(float(f0), 5), "St": round(float(f0), 5), "f0_fft": round(float(f_fft), 5),
            "period_rel_std": round(float(per.std() / per.mean()), 4) if len(per) > 1 else None,
            "fft_peaks": [[round(float(freqs[j]), 4), round(float(spec[j] / spec[i]), 3)]
                          for j in top],
            "cl_amplitude": round(float(0.5 * (c.max() - c.min())), 4),
            "cl_std": round(float(c.std()), 4), "cd_mean": round(float(cd[sel].mean()), 4),
            "periods": int(len(per)), "t_end": t_end, "window": window, "steps": n, "dt": dt,
            "wall_s": round(wall, 2),
            "workload": "fixed cylinder of osc1 (512^2 over [-4,12]x[-8,8], 200 candidate "
                        "markers, Re 100, Ma 0.3, Tw/Tinf 1, FP64)"}


def run_moving(steps: int, warmup: int):
    """The moving bodies on 512^2 grids, markers re-placed, re-selected and re-weighted
    every step, in both forms: the streamwise-oscillating cylinder of Sec. 5 on the
    density-based step (200 candidate markers, x = 0.14 D sin(2 pi f_c t) with
    f_c = 2 f_0 and f_0 measured first from the lift of the fixed cylinder on the
    pressure-based step, Re 100, Ma 0.3, Tw/Tinf 1 and 2) and the transversely
    oscillating one on the pressure-based step
    (200 candidate markers, y = 0.2 D sin(2 pi 0.2 t), Re 100, Ma 0.2, Tw/Tinf 1.2).
    Per kernel class, "markers" is the marker work on the step's own stream
    (interpolation, forcing, totals, spreading, and the set-up of the first step of a
    call) and "rebuild" a later step's marker set-up on one of the library's side
    streams, which overlaps the steps."""
    from paper_2301_09349_amd import inputs

    # f_0 from the pressure-based step: on the density-based one the fixed cylinder's
    # lift is dominated by the closed box's acoustic modes (reflecting sides; the
    # density-based run is recorded alongside)
    out = {"shedding_fixed": shedding_frequency(0),
           "shedding_fixed_density": shedding_frequency(1)}
    f0 = out["shedding_fixed"]["f0"]
    for name in ("osc1", "osc2", "cfg4"):
        case = inputs.case(name, cg_rtol=1e-10)
        if name.startswith("osc") and math.isfinite(f0):
            m = dict(case["motion"], freq=2.0 * f0)
            case["motion"] = m
            case["dt_u_max"] = 2.0 * math.pi * m["freq"] * m["amp"]
        res = {"steps": steps}
        for prec in ("fp64", "fp32"):
            r = run_forward(case, prec, steps, warmup)
            if "workload" not in res:
                kept = r["solver"].markers_in_use()[0].shape[0]
                res["workload"] = workload_text(case, kept, r["solver"].dt)
            res[prec] = {"value": round(r["value"], 2), "ms_per_step": round(r["ms_per_step"], 4),
                         "cg_iters_per_step": round(r["info"]["cg_iters_total"] / steps, 2),
                         "kernels_ms_per_step": {k: round(v["ms_per_step"], 4)
                                                 for k, v in r["per_kernel"].items()}}
            del r
        out[name] = res
    return out


def run_implicit(case, steps: int, warmup: int, explicit: dict):
    """The main workload with the compact viscous and conductive fluxes implicit
    (backward Euler; the step from convection alone): ms per step, the step, and
    simulated time per wall-clock second against the explicit runs in `explicit`
    ({precision: (dt, ms_per_step)})."""
    res = {"steps": steps}
    for prec, (dt_e, ms_e) in explicit.items():
        r = run_forward(dict(case, diffusion=1), prec, steps, warmup)
        dt_i = r["solver"].dt
        ent = {"value": round(r["value"], 2), "ms_per_step": round(r["ms_per_step"], 4),
               "dt": dt_i, "dt_explicit": dt_e, "dt_ratio": round(dt_i / dt_e, 3),
               "cg_iters_per_step": round(r["info"]["cg_iters_total"] / steps, 2),
               "diffusion_iters_per_step": round(r["info"]["diff_iters_total"] / steps, 2),
               "sim_time_per_s": round(dt_i / (r["ms_per_step"] * 1e-3), 4),
               "sim_time_per_s_explicit": round(dt_e / (ms_e * 1e-3), 4),
               "kernels_ms_per_step": {k: round(v["ms_per_step"], 4)
                                       for k, v in r["per_kernel"].items()}}
        ent["sim_time_speedup"] = round(ent["sim_time_per_s"] / ent["sim_time_per_s_explicit"], 3)
        res[prec] = ent
        del r
    # the same grid at Re 20, where conduction limits the explicit step far more
    low = dict(case, Re=20.0)
    re_ = run_forward(low, "fp64", steps, warmup)
    ri = run_forward(dict(low, diffusion=1), "fp64", steps, warmup)
    dt_e, ms_e = re_["solver"].dt, re_["ms_per_step"]
    dt_i, ms_i = ri["solver"].dt, ri["ms_per_step"]
    res["fp64_re20"] = {"ms_per_step": round(ms_i, 4), "ms_per_step_explicit": round(ms_e, 4),
                        "dt": dt_i, "dt_explicit": dt_e, "dt_ratio": round(dt_i / dt_e, 3),
                        "diffusion_iters_per_step": round(ri["info"]["diff_iters_total"] / steps, 2),
                        "cg_iters_per_step": round(ri["info"]["cg_iters_total"] / steps, 2),
                        "sim_time_speedup": round((dt_i / ms_i) / (dt_e / ms_e), 3)}
    del re_, ri
    return res


def run_outer(case, steps: int, warmup: int):
    """The main workload in FP64 with 1, 2 and 3 outer passes per step (App. A step
    3 repeated) at half the default step (CFL 0.25: the passes are a fixed-point
    iteration that converges only where dt |lambda| < 1, and at the default step
    an even pass count is unstable): ms per step and CG iterations per step."""
    res = {"steps": steps, "cfl": 0.25}
    one = None
    for K in (1, 2, 3):
        r = run_forward(dict(case, n_outer=K, cfl=0.25), "fp64", steps, warmup)
        ms = r["ms_per_step"]
        one = one or ms
        res[f"n_outer_{K}"] = {
            "ms_per_step": round(ms, 4), "cost_vs_one_pass": round(ms / one, 3),
            "dt": r["solver"].dt,
            "cg_iters_per_step": round(r["info"]["cg_iters_total"] / steps, 2),
            "kernels_ms_per_step": {k: round(v["ms_per_step"], 4)
                                    for k, v in r["per_kernel"].items()}}
        del r
    return res


def run_density(steps: int, warmup: int):
    """The density-based step (App. B; explicit, its step limited by the sound
    speed) on the 1024^2 cylinder and the 256^3 sphere at Ma 0.8, both forms:
    throughput and the per-kernel achieved bandwidth."""
    from paper_2301_09349_amd import inputs

    res = {}
    for name, wl, st, wu in (("cylinder1024", "cfg2a", steps, warmup), ("sphere256", "cfg3", 30, 10)):
        case = inputs.case(wl, Ma=0.8, scheme=1)
        ent = {"steps": st}
        for prec in ("fp64", "fp32"):
            r = run_forward(case, prec, st, wu)
            if "workload" not in ent:
                kept = r["solver"].markers_in_use()[0].shape[0]
                ent["workload"] = workload_text(case, kept, r["solver"].dt)
            ent[prec] = {"value": round(r["value"], 2), "ms_per_step": round(r["ms_per_step"], 4),
                         "kernels": {k: {"avg_us": round(v["avg_us"], 2),
                                         **({"GBps": round(v["GBps"], 1),
                                             "frac": round(v["GBps"] / HBM_PEAK_GBS, 4)}
                                            if "GBps" in v else {})}
                                     for k, v in r["per_kernel"].items()}}
            del r
        res[name] = ent
    return res


def run_grid_convergence(t_end: float = 40.0, t_avg: float = 10.0):
    """The grid-convergence study of App. C: the cylinder at Ma 2.5, Re 250 without
    heat exchange on h = D/10, D/15, D/25, D/50 (28, 39, 62, 104 markers), the
    density-based step from an impulsive start to t_end; C_D = 2 F_x / (rho U^2 D)
    averaged over the last t_avg; errors against the finest grid and the order of
    their least-squares fit in log h."""
    import numpy as np
    import torch
    from paper_2301_09349_amd import inputs

    res, cd = {"t_end": t_end, "t_average": t_avg, "grids": {}}, {}
    for r in (10, 15, 25, 50):
        case = inputs.case("sup%d" % r)
        s = make_solver(case, "fp64")
        steps = int(round(t_end / s.dt))
        navg = int(round(t_avg / s.dt))
        hist = torch.zeros((steps, 4), dtype=torch.float64, device="cuda:0")
        log(f"bench: grid convergence D/{r}: {case['n']}, {steps} steps")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps, hist_out=hist)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        h = hist.cpu().numpy()
        cd[r] = float(2.0 * h[-navg:, 0].mean())
        res["grids"]["D/%d" % r] = {"cells": int(np.prod(case["n"][:2])),
                                    "markers_kept": int(s.markers_in_use()[0].shape[0]),
                                    "dt": s.dt, "steps": steps, "C_D": round(cd[r], 6),
                                    "ms_per_step": round(1e3 * el / steps, 4)}
        del s
    coarse = (10, 15, 25)
    err = [abs(cd[r] - cd[50]) for r in coarse]
    res["error_vs_finest"] = {"D/%d" % r: float("%.4g" % e) for r, e in zip(coarse, err)}
    if all(e > 0 for e in err):
        res["observed_order"] = round(float(np.polyfit(np.log([1.0 / r for r in coarse]),
                                                       np.log(err), 1)[0]), 3)
    return res


def calibrate_copy():
    """A plain streaming kernel of known size for scaling the HBM counters: negation
    of CALIB_ELEMS float64 values (8 B read + 8 B written each), three launches."""
    import torch

    a = torch.ones(CALIB_ELEMS, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    del a, b


# ------------------------------------------------------------ rocprofv3 summaries
def _rows(pattern):
    files = sorted(glob.glob(pattern, recursive=True))
    if not files:
        raise SystemExit(f"no file matches {pattern}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def summarize(directory: str, label: str, command: str):
    """Reads rocprofv3 output under `directory` -- kernel_stats from a --kernel-trace
    --stats run (stats/), counter_collection from --pmc FETCH_SIZE (fetch/) and --pmc
    WRITE_SIZE (write/) runs, and each run's JSON line (stats.json) -- and writes
    profiles/kernels_<label>.md and, with counters, profiles/traffic_<label>.json."""
    out_md = os.path.join(ROOT, "profiles", f"kernels_{label}.md")
    bj = json.loads(open(os.path.join(directory, "stats.json")).read().strip().splitlines()[-1])
    total_steps = bj["warmup"] + 2 * bj["steps"]
    # CG iterations per step over every step of the profiled run (warm-up included)
    iters = bj.get("cg_iters_all_steps", bj["config"]["cg_iters_per_step"] * total_steps)
    iters = iters / total_steps
    prec = bj["config"]["precision"]
    lines = [f"# rocprofv3 summary: {label}", "", "Commands (from the repository root):", ""]
    for c in command.split(";;"):
        lines.append(f"    {c.strip()}")
    lines += ["", f"The profiled program runs {bj['warmup']} warm-up steps, {bj['steps']} steps "
              f"without and {bj['steps']} steps with the library's event timing "
              f"({total_steps} steps, {iters:.2f} CG iterations per step); per-step figures divide "
              "the kernel totals by the steps.", "",
              "## Kernel trace (--kernel-trace --stats)", "",
              "| kernel | class | calls | avg us | total ms | % |", "|---|---|---|---|---|---|"]
    stats = _rows(os.path.join(directory, "stats", "**", "*kernel_stats.csv"))
    cls_ns = {}
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
        name = r["Name"]
        cls = kernel_class(name)
        if cls:
            cls_ns[cls] = cls_ns.get(cls, 0.0) + float(r["TotalDurationNs"])
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:25]:
        name = r["Name"]
        lines.append(f"| `{name.split('(')[0][:70]}` | {kernel_class(name) or ''} | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['TotalDurationNs']) / 1e6:.3f} "
                     f"| {float(r['Percentage']):.1f} |")
    lines += ["", "## Kernel time per step: kernel trace against the HIP events of the same run",
              "", "| class | trace us/step | events us/step | trace us per launch or CG iteration "
              "| events us per launch or CG iteration |", "|---|---|---|---|---|"]
    for cls, ns in sorted(cls_ns.items(), key=lambda kv: -kv[1]):
        ev = bj["kernels"].get(cls)
        tr_step = ns / 1e3 / total_steps
        per = tr_step / iters if cls == "cg" else None
        if ev:
            ev_step = 1e3 * ev["ms_per_step"]
            ev_per = ev["avg_us"]
            lines.append(f"| {cls} | {tr_step:.2f} | {ev_step:.2f} | "
                         f"{(per if per else tr_step):.2f} | {ev_per:.2f} |")
    traffic = {}
    have_pmc = all(glob.glob(os.path.join(directory, d, "**", "*counter_collection.csv"),
                             recursive=True) for d in ("fetch", "write"))
    if have_pmc:
        per = {}
        for d, counter in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
            acc = {}
            for r in _rows(os.path.join(directory, d, "**", "*counter_collection.csv")):
                if r.get("Counter_Name") != counter:
                    continue
                key = r["Kernel_Name"]
                disp = r.get("Dispatch_Id") or r.get("Correlation_Id")
                acc.setdefault(key, {}).setdefault(disp, 0.0)
                acc[key][disp] += float(r["Counter_Value"])
            for k, v in acc.items():
                per.setdefault(k, {})[counter + "_total"] = sum(v.values())  # KiB
                per[k][counter] = sum(v.values()) / len(v)                    # KiB per dispatch
                per[k]["dispatches_" + d] = len(v)
        calib = [k for k in per if "neg_kernel" in k]
        if not calib:
            raise SystemExit("the copy calibration kernel was not found in the counters")
        c = per[calib[0]]
        nominal_kib = CALIB_ELEMS * 8 / 1024.0
        f_fetch = c.get("FETCH_SIZE", 0.0) / nominal_kib
        f_write = c.get("WRITE_SIZE", 0.0) / nominal_kib
        lines += ["", "## HBM traffic (--pmc FETCH_SIZE, then --pmc WRITE_SIZE)", "",
                  f"Copy calibration: negation of {CALIB_ELEMS} float64 values (512 MiB read, "
                  f"512 MiB written) reads FETCH_SIZE x{f_fetch:.4f} and WRITE_SIZE "
                  f"x{f_write:.4f} of the nominal bytes; the figures below are divided by "
                  "these factors.", "",
                  "| kernel | class | dispatches | fetch MB/dispatch | write MB/dispatch | "
                  "total MB/dispatch |", "|---|---|---|---|---|---|"]
        cls_bytes = {}
        for k, v in sorted(per.items(), key=lambda kv: -(kv[1].get("FETCH_SIZE", 0)
                                                         + kv[1].get("WRITE_SIZE", 0))):
            fb = v.get("FETCH_SIZE", 0.0) * 1024 / max(f_fetch, 1e-12)
            wb = v.get("WRITE_SIZE", 0.0) * 1024 / max(f_write, 1e-12)
            cls = kernel_class(k)
            lines.append(f"| `{k.split('(')[0][:70]}` | {cls or ''} | "
                         f"{v.get('dispatches_fetch', 0)} | {fb / 1e6:.2f} | {wb / 1e6:.2f} | "
                         f"{(fb + wb) / 1e6:.2f} |")
            if cls:
                tot = (v.get("FETCH_SIZE_total", 0.0) * 1024 / max(f_fetch, 1e-12)
                       + v.get("WRITE_SIZE_total", 0.0) * 1024 / max(f_write, 1e-12))
                cls_bytes[cls] = cls_bytes.get(cls, 0.0) + tot
        lines += ["", "Per class, as the bench line uses them (bytes per step; per CG iteration "
                  "for the CG):", "", "| class | MB |", "|---|---|"]
        for cls, tot in sorted(cls_bytes.items()):
            units = total_steps * (iters if cls == "cg" else 1)
            traffic[cls] = {"bytes_per_launch": tot / units}
            lines.append(f"| {cls} | {tot / units / 1e6:.2f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")
    log(f"wrote {out_md}")
    if traffic:
        path = os.path.join(ROOT, "profiles", f"traffic_{label}.json")
        rec = {"source_sha": source_sha(), "precision": prec, "classes": traffic,
               "note": "HBM bytes per launch (per CG iteration for the CG) from FETCH_SIZE + "
                       "WRITE_SIZE scaled by the copy calibration; see kernels_%s.md" % label}
        json.dump(rec, open(path, "w"), indent=1, sort_keys=True)
        log(f"wrote {path}")


def workload_text(case, kept: int, dt: float) -> str:
    dim = case["dim"]
    body = "2D heated cylinder" if dim == 2 else "3D heated sphere"
    m = case.get("motion")
    if m:
        body = "2D cylinder oscillating along %s, %g sin(2 pi %g t)" % (
            "xyz"[m["axis"]], m["amp"], m["freq"])
    cells = "x".join(str(v) for v in case["n"][:dim])
    box = "x".join("[%g,%g]" % (case["lo"][d], case["hi"][d]) for d in range(dim))
    step = ("density-based step" if case.get("scheme", 0) == 1
            else "pressure-based step, CG rtol 1e-10")
    return ("%s, %s cells over %s, %d candidate markers (check routine keeps %d), Re %g, "
            "Ma %g, Tw/Tinf %g, dt %.4e, %s"
            % (body, cells, box, case["ns"], kept, case["Re"], case["Ma"], case["Tw"], dt, step))


# SQ and GRBM counters of the three --pmc passes that --summarize-counters reads
COUNTER_PASSES = [
    "SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_SALU "
    "SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_TRANS_F64",
    "SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_LDS SQ_ACTIVE_INST_VALU "
    "SQ_ACTIVE_INST_LDS SQ_LDS_BANK_CONFLICT SQ_ACTIVE_INST_ANY",
    "SQ_INSTS_VALU_INT32 SQ_INSTS_VALU_INT64 SQ_INSTS_VALU_ADD_F64 SQ_INSTS_VALU_MUL_F64 "
    "SQ_INSTS_VALU_CVT SQ_INSTS_BRANCH SQ_INSTS_SMEM GRBM_GUI_ACTIVE",
]


def summarize_counters(directory: str, label: str, command: str, cells: int):
    """Reads the counter_collection files of the --pmc passes in COUNTER_PASSES (the
    sub-directories pmc0, pmc1, pmc2 of `directory`) and the kernel trace of the same
    program (stats/), and writes profiles/counters_<label>.md: per kernel and dispatch
    the counters summed over the device, and derived figures with their formulas."""
    stats = _rows(os.path.join(directory, "stats", "**", "*kernel_stats.csv"))
    dur = {r["Name"]: float(r["AverageNs"]) for r in stats}
    per = {}
    for i in range(len(COUNTER_PASSES)):
        acc = {}
        for r in _rows(os.path.join(directory, f"pmc{i}", "**", "*counter_collection.csv")):
            key = r["Kernel_Name"]
            disp = r.get("Dispatch_Id") or r.get("Correlation_Id")
            c = r["Counter_Name"]
            acc.setdefault(key, {}).setdefault(c, {}).setdefault(disp, 0.0)
            acc[key][c][disp] += float(r["Counter_Value"])
        for k, cs in acc.items():
            for c, v in cs.items():
                per.setdefault(k, {})[c] = sum(v.values()) / len(v)
    lines = [f"# rocprofv3 counters: {label}", "", "Commands (from the repository root):", ""]
    for c in command.split(";;"):
        lines.append(f"    {c.strip()}")
    lines += ["", "Counters per dispatch (averaged over the dispatches of each kernel, each summed "
              "over the device). Passes: " + "; ".join(f"`{p}`" for p in COUNTER_PASSES) + ".",
              "", "Derived, per kernel (cells = %d; a wave-instruction serves 64 cells, so "
              "`X per cell` = X / (cells / 64) is the count per cell and lane):" % cells, "",
              "- VALU, LDS, VMEM (read + write), SALU, FP64 FMA, FP64 transcendental "
              "instructions per cell;",
              "- `valu/wave`, `lds/wave`, `wait/wave`, `ldswait/wave`: SQ_ACTIVE_INST_VALU, "
              "SQ_ACTIVE_INST_LDS, SQ_WAIT_ANY, SQ_WAIT_INST_LDS over SQ_WAVE_CYCLES (the share "
              "of the waves' resident time spent issuing VALU or LDS work, waiting on a counter, "
              "waiting to issue LDS);",
              "- `bank conflict`: SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS (stall cycles per "
              "cycle of LDS work);",
              "- `waves/CU`: 4 SQ_WAVE_CYCLES / (GRBM_GUI_ACTIVE / 8) / 256, the mean number "
              "of resident waves per CU over the kernel (SQ_WAVE_CYCLES counts quad-cycles "
              "summed over all waves; GRBM_GUI_ACTIVE counts the kernel's cycles summed over "
              "the 8 XCDs);",
              "- INT32, INT64, ADD64, MUL64, CVT: VALU instructions of those kinds per cell;",
              "- `us`: mean duration from the kernel trace of the same program.", "",
              "| kernel | us | VALU/cell | LDS/cell | VMEM/cell | SALU/cell | FMA64/cell | "
              "TRANS64/cell | INT32 | INT64 | ADD64 | MUL64 | CVT | valu/wave | lds/wave | "
              "wait/wave | ldswait/wave | bank conflict | waves/CU |", "|---|" + "---|" * 18]
    wcell = cells / 64.0

    def g(v, c):
        return v.get(c, float("nan"))

    rows = sorted(per.items(), key=lambda kv: -dur.get(kv[0], 0.0))
    for k, v in rows:
        if k not in dur or dur[k] < 20000:  # kernels of at least 20 us
            continue
        wc = g(v, "SQ_WAVE_CYCLES")
        lines.append(
            f"| `{k.split('(')[0][:60]}` | {dur[k] / 1e3:.1f} | {g(v, 'SQ_INSTS_VALU') / wcell:.0f} | "
            f"{g(v, 'SQ_INSTS_LDS') / wcell:.1f} | "
            f"{(g(v, 'SQ_INSTS_VMEM_RD') + g(v, 'SQ_INSTS_VMEM_WR')) / wcell:.1f} | "
            f"{g(v, 'SQ_INSTS_SALU') / wcell:.0f} | {g(v, 'SQ_INSTS_VALU_FMA_F64') / wcell:.0f} | "
            f"{g(v, 'SQ_INSTS_VALU_TRANS_F64') / wcell:.1f} | "
            f"{g(v, 'SQ_INSTS_VALU_INT32') / wcell:.0f} | {g(v, 'SQ_INSTS_VALU_INT64') / wcell:.0f} | "
            f"{g(v, 'SQ_INSTS_VALU_ADD_F64') / wcell:.0f} | "
            f"{g(v, 'SQ_INSTS_VALU_MUL_F64') / wcell:.0f} | {g(v, 'SQ_INSTS_VALU_CVT') / wcell:.0f} | "
            f"{g(v, 'SQ_ACTIVE_INST_VALU') / wc:.3f} | {g(v, 'SQ_ACTIVE_INST_LDS') / wc:.3f} | "
            f"{g(v, 'SQ_WAIT_ANY') / wc:.3f} | {g(v, 'SQ_WAIT_INST_LDS') / wc:.3f} | "
            f"{g(v, 'SQ_LDS_BANK_CONFLICT') / max(g(v, 'SQ_ACTIVE_INST_LDS'), 1.0):.3f} | "
            f"{4.0 * wc / max(g(v, 'GRBM_GUI_ACTIVE') / 8.0, 1.0) / 256:.2f} |")
    lines += ["", "Raw counters per dispatch:", "", "| kernel | counter | value |",
              "|---|---|---|"]
    for k, v in rows:
        if k not in dur or dur[k] < 20000:
            continue
        for c in sorted(v):
            lines.append(f"| `{k.split('(')[0][:60]}` | {c} | {v[c]:.6g} |")
    out_md = os.path.join(ROOT, "profiles", f"counters_{label}.md")
    open(out_md, "w").write("\n".join(lines) + "\n")
    log(f"wrote {out_md}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"],
                    help="precision of the headline value (the other form is run too)")
    ap.add_argument("--workload", default="cfg3",
                    help="headline workload (default cfg3, the 256^3 heated sphere)")
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-fp32-errors", action="store_true",
                    help="skip the full-length FP32-vs-FP64 error runs")
    ap.add_argument("--adjoint-steps", type=int, default=100)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-2d", action="store_true", help="skip the 1024^2 cylinder figures")
    ap.add_argument("--no-implicit", action="store_true",
                    help="skip the implicit-diffusion figures")
    ap.add_argument("--no-outer", action="store_true", help="skip the outer-pass figures")
    ap.add_argument("--diffusion", default="explicit", choices=["explicit", "implicit"],
                    help="viscous and conductive terms of the main workload (profiling)")
    ap.add_argument("--scheme", default="pressure", choices=["pressure", "density"],
                    help="step of the main workload (profiling; density: at Ma 0.8)")
    ap.add_argument("--no-density", action="store_true",
                    help="skip the density-based figures")
    ap.add_argument("--no-convergence", action="store_true",
                    help="skip the grid-convergence study of App. C")
    ap.add_argument("--no-moving", action="store_true",
                    help="skip the moving-body figures")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="launch the copy kernel used to scale HBM counters first")
    ap.add_argument("--summarize", metavar="DIR", help="summarize rocprofv3 output (no GPU)")
    ap.add_argument("--label", default="sphere256_fp64",
                    help="summary name: <workload>_<precision>, e.g. sphere256_fp32")
    ap.add_argument("--command", default="")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="summarize the SQ counter passes of this script (no GPU)")
    ap.add_argument("--cells", type=int, default=256 ** 3,
                    help="cells of the profiled workload (--summarize-counters)")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.label, args.command, args.cells)
        return
    if args.summarize:
        summarize(args.summarize, args.label, args.command)
        return
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (the step runs on one MI355X); "
              "--gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2301_09349_amd import inputs

    if args.calibrate_copy:
        calibrate_copy()
    case = inputs.case(args.workload, cg_rtol=1e-10,
                       diffusion=1 if args.diffusion == "implicit" else 0)
    if args.scheme == "density":
        case = dict(case, scheme=1, Ma=0.8)
    main_p = args.precision
    other = "fp32" if main_p == "fp64" else "fp64"
    r = run_forward(case, main_p, args.steps, args.warmup)
    ro = None if args.no_fp32 else run_forward(case, other, args.steps, args.warmup)
    per_kernel = r["per_kernel"]
    dom = max((k for k in per_kernel if "GBps" in per_kernel[k]),
              key=lambda k: per_kernel[k]["total_ms"])
    d = per_kernel[dom]
    label = "%s%s%s_%s" % (WORKLOAD_LABEL.get(args.workload, args.workload),
                           "_implicit" if args.diffusion == "implicit" else "",
                           "_density" if args.scheme == "density" else "", main_p)
    traffic = traffic_entry(label, dom)
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(d["GBps"], 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(d["GBps"] / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "alg_bytes_per_launch": d["alg_bytes_per_launch"],
            "avg_us": round(d["avg_us"], 3),
            "timing": "HIP events on the library stream over a second run of the same "
                      "steps (the throughput run is untimed per kernel)"}
    log("bench: per-kernel " + json.dumps({k: {kk: (round(vv, 2) if isinstance(vv, float) else vv)
                                                 for kk, vv in v.items()}
                                             for k, v in per_kernel.items()}))
    ids, eps_used = r["solver"].markers_in_use()
    out = {
        "metric": "Mcell-steps/s (fwd, FP32 vs FP64 at stated err) + adjoint/forward time ratio",
        "value": round(r["value"], 2),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_p == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": workload_text(case, ids.shape[0], r["solver"].dt),
                   "cells": r["N"], "precision": main_p,
                   "cg_iters_per_step": round(r["info"]["cg_iters_total"] / args.steps, 2),
                   # the quadrature weights of the markers in use (Eqs. (8)-(9))
                   "eps_range": [round(float(eps_used.min()), 4), round(float(eps_used.max()), 4)],
                   "eps_negative": int((eps_used < 0).sum())},
        "roofline": roof,
        "kernels": {k: {"avg_us": round(v["avg_us"], 2), "launches": v["launches"],
                        "ms_per_step": round(v["ms_per_step"], 4),
                        **({"GBps": round(v["GBps"], 1),
                            "frac": round(v["GBps"] / HBM_PEAK_GBS, 4)} if "GBps" in v else {})}
                    for k, v in per_kernel.items()},
        "ms_per_step_profiled": round(r["ms_per_step_profiled"], 4),
        "cg_iters_all_steps": r["cg_iters_all"],
    }
    if ro is not None:
        r64, r32 = (r, ro) if main_p == "fp64" else (ro, r)
        out[other] = {"value": round(ro["value"], 2), "ms_per_step": round(ro["ms_per_step"], 4),
                      "cg_iters_per_step": round(ro["info"]["cg_iters_total"] / args.steps, 2),
                      "speedup_fp32_over_fp64": round(r64["ms_per_step"] / r32["ms_per_step"], 3),
                      "kernels": {k: {"avg_us": round(v["avg_us"], 2),
                                      **({"GBps": round(v["GBps"], 1)} if "GBps" in v else {})}
                                  for k, v in ro["per_kernel"].items()}}
        out["fp32_error_vs_fp64"] = {k: float("%.3g" % v) for k, v in fp32_error(r64, r32).items()}
        del ro
    del r
    torch.cuda.empty_cache()
    if not args.no_fp32 and not args.no_fp32_errors:
        log("bench: FP32 form against FP64 over full runs ...")
        out["fp32_errors_full_runs"] = fp32_errors_full(
            [("cfg2a", {}, 2000), ("cfg2b", {}, 2000), ("cfg3", {}, 500)])
    if not args.no_2d:
        log("bench: 1024^2 cylinder ...")
        out["cylinder1024"] = run_cylinder(args.steps, args.warmup)
        torch.cuda.empty_cache()
    cyl_case = inputs.case("cfg2a", cg_rtol=1e-10)
    if not args.no_implicit:
        log("bench: implicit diffusion ...")
        if "cylinder1024" in out:
            base = {p: (out["cylinder1024"][p]["dt"], out["cylinder1024"][p]["ms_per_step"])
                    for p in ("fp64", "fp32")}
        else:
            base = {}
            for prec in ("fp64", "fp32"):
                rb = run_forward(cyl_case, prec, args.steps, args.warmup)
                base[prec] = (rb["solver"].dt, rb["ms_per_step"])
                del rb
        out["implicit_diffusion"] = run_implicit(cyl_case, args.steps, args.warmup, base)
        torch.cuda.empty_cache()
    if not args.no_outer:
        log("bench: outer passes ...")
        out["outer_passes"] = run_outer(cyl_case, args.steps, args.warmup)
        torch.cuda.empty_cache()
    if not args.no_density:
        log("bench: density-based step ...")
        out["density_based"] = run_density(args.steps, args.warmup)
        torch.cuda.empty_cache()
    if not args.no_convergence:
        log("bench: grid convergence (App. C) ...")
        out["grid_convergence"] = run_grid_convergence()
        torch.cuda.empty_cache()
    if not args.no_moving:
        log("bench: moving bodies ...")
        out["moving512"] = run_moving(100, 10)
        torch.cuda.empty_cache()
    if not args.no_adjoint:
        log(f"bench: adjoint leg, {args.adjoint_steps} steps ...")
        out["adjoint"] = run_adjoint(args.adjoint_steps, 50, 10)
        a32 = run_adjoint(args.adjoint_steps, 50, 10, "fp32")
        out["adjoint_fp32"] = {k: a32[k] for k in ("forward_ms_per_step", "backward_ms_per_step",
                                                   "ratio", "grad_norm", "tape_all_steps")}
    if not args.no_cpu:
        log(f"bench: timing the oracle on {args.cpu_steps} step(s) ...")
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
