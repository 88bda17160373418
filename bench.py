"""Throughput of the semi-implicit BTE step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision mixed_fp32|mixed_bf16|fp64]

Workload (synthetic, seeded): Nx = 256 Chebyshev points, Nr = 64 B-splines,
Ntheta = 32 ordinates (n = 2048 unknowns per point), argon-like analytic cross
sections, RF field E0 sin(2 pi f t)(1 + x/2), dt = 1e-3 RF period.  A step is one
pass of X(dt/2) -> field -> V(dt) -> X(dt/2) over all 256 points, inputs resident
in HBM.  Prints one JSON line; ``value`` is steps/s of the selected precision
(default: the mixed FP32 + FP64-refinement form), and the FP64 step is timed
beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MI355X_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}


def _update_flops(npad: int, nb: int, nmat: int) -> float:
    """Algorithmic flops of all trailing-update launches of one factorization."""
    tot = 0.0
    for k0 in range(0, npad, nb):
        m = npad - k0 - nb
        if m > 0:
            tot += 2.0 * m * m * nb
    return tot * nmat


def run_gpu(cfg, precision, steps, warmup, torch, lu_streams=None):
    from paper_2502_16555_amd import Solver, _lib
    t0 = time.time()
    s = Solver(cfg, precision=precision)
    setup_s = time.time() - t0
    if lu_streams is not None:
        s.set_tuning(_lib.TUNE_LU_STREAMS, lu_streams)
    import workloads
    ne = workloads.density_profile(s.xhat(), cfg["ic"]["ne_peak"])
    F = s.initial_state(torch.as_tensor(ne, device="cuda:0"), cfg["ic"]["Te_eV"])
    dt = cfg["dt_s"]
    n = 0
    for _ in range(warmup):
        s.step(F, n * dt)
        n += 1
    torch.cuda.synchronize()
    code, sweeps, resid = s.status()
    if code != 0:
        raise RuntimeError(f"{precision}: device status {code} after warm-up")
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        s.step(F, n * dt)
        n += 1
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1) / steps
    code, sweeps, resid = s.status()
    if code != 0:
        raise RuntimeError(f"{precision}: device status {code} in the timed steps")
    mom = s.moments(F).cpu().numpy()
    # kernel-level breakdown (separate, instrumented steps)
    s.set_timing(True)
    nt = 3
    for _ in range(nt):
        s.step(F, n * dt)
        n += 1
    tm = s.timing()
    s.set_timing(False)
    out = {"ms_per_step": ms, "wall_s": wall, "setup_s": setup_s, "refine_sweeps": sweeps, "refine_resid": resid,
           "moments": mom, "t_final": n * dt,
           "ms_update": tm[0] / nt, "ms_panel": tm[1] / nt, "ms_vwall": tm[2] / nt, "ms_x": tm[4] / nt,
           "update_launches": tm[3] / nt, "lu_streams": s.get_tuning(_lib.TUNE_LU_STREAMS),
           "info": s.info}
    s.close()
    return out


def cpu_baseline(cfg, budget_s=20.0):
    """The FP64 oracle on the host cores, on a bounded sample of one step's work:
    one full X(dt/2) plus as many of the per-point V solves as fit the budget;
    the step time is 2 t_X + Nx t_V."""
    import oracle
    from oracle import semi_implicit as S
    import workloads
    ops = oracle.build_operators(cfg)
    F = S.initial_state(ops, workloads.density_profile(ops.xhat, cfg["ic"]["ne_peak"]), cfg["ic"]["Te_eV"])
    t = time.perf_counter()
    Fh = S.x_half_step(ops, F)
    tx = time.perf_counter() - t
    E = S.field_half(ops, 0.0)
    nv = 0
    t = time.perf_counter()
    while nv < ops.nx and (time.perf_counter() - t) < max(budget_s - tx, 1.0):
        S.v_step(ops, Fh, E, xs=[nv])
        nv += 1
    tv = (time.perf_counter() - t) / nv
    step_s = 2 * tx + ops.nx * tv
    threads = int(os.environ.get("OPENBLAS_NUM_THREADS", os.cpu_count() or 1))
    return {"value": 1.0 / step_s, "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"one X(dt/2) over all {ops.nx} points ({tx:.2f} s) + {nv} of {ops.nx} V solves "
                      f"({tv:.3f} s each), scaled to one step = 2 t_X + Nx t_V"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="mixed_fp32", choices=["mixed_fp32", "mixed_bf16", "fp64"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--lu-streams", type=int, default=None, help="concurrent factorization groups (library default 2)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the hot path is single-GPU in this build",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    cfg = workloads.config("C2")
    if args.nx != 256:
        cfg = dict(cfg, nx=args.nx, nx_per=[args.nx])
    main_run = run_gpu(cfg, args.precision, args.steps, args.warmup, torch, args.lu_streams)
    fp64 = None
    if not args.no_fp64 and args.precision != "fp64":
        fp64 = run_gpu(cfg, "fp64", max(args.steps // 2, 5), args.warmup, torch, args.lu_streams)
    info = main_run["info"]
    nx_total, n = info.nx_total, info.n
    npad = ((n + 127) // 128) * 128
    dtype = {"fp64": "f64", "mixed_fp32": "f32+f64", "mixed_bf16": "bf16+f32+f64"}[args.precision]
    mfma = {"fp64": "fp64", "mixed_fp32": "fp32", "mixed_bf16": "bf16"}[args.precision]
    # update flops of one step over the summed durations of its update launches
    upd_flops = _update_flops(npad, 128, nx_total)
    n_upd_launches = main_run["update_launches"]
    achieved = upd_flops / (main_run["ms_update"] * 1e-3) / 1e12
    peak = MI355X_PEAK_TFLOPS[mfma]
    value = 1000.0 / main_run["ms_per_step"]
    line = {
        "metric": "BTE steps/s at Nx256 Nr64 Ntheta32 (mixed precision step; FP64 step timed beside it)",
        "value": value, "unit": "steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": dtype, "data": "synthetic",
        "config": {"workload": f"Nx={cfg['nx']} CGL, Nr=64 B-splines (f(vmax)=0), Ntheta=32 GL, n=2048 per point, "
                               f"argon-like sigma, RF E0={cfg['field']['E0']:.1f} V/m, dt=1e-3 T_rf",
                   "precision": args.precision, "nx": cfg["nx"], "nr": 64, "ntheta": 32},
        "roofline": {"bound": "mfma", "kernel": "k_update (LU trailing update)", "achieved": achieved,
                     "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "launches_per_step": n_upd_launches,
                     "avg_launch_ms": main_run["ms_update"] / n_upd_launches},
        "breakdown_ms": {"lu_update_launches": main_run["ms_update"], "lu_panel_u12_launches": main_run["ms_panel"],
                         "v_step_wall": main_run["ms_vwall"], "x_and_field_wall": main_run["ms_x"],
                         "lu_streams": main_run["lu_streams"]},
        "lu_tflops_step": info.lu_flops_per_step / (main_run["ms_per_step"] * 1e-3) / 1e12,
        "refine": {"sweeps": main_run["refine_sweeps"], "resid": main_run["refine_resid"]},
    }
    if fp64 is not None:
        line["fp64"] = {"steps_per_s": 1000.0 / fp64["ms_per_step"], "ms_per_step": fp64["ms_per_step"],
                        "speedup_mixed_over_fp64": fp64["ms_per_step"] / main_run["ms_per_step"],
                        "ms_update": fp64["ms_update"], "ms_panel": fp64["ms_panel"],
                        "update_tflops": _update_flops(npad, 128, nx_total) / (fp64["ms_update"] * 1e-3) / 1e12}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(cfg)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
