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
MI355X_PEAK_HBM_GBS = 8000.0

# HBM bytes of the FP32 trailing update (k_update<float, 16, ...>, K = 128 to 512)
# per launch, averaged over the 15 launches of one factorization at this workload
# (statically pivoted panels in groups of four: 3 launches of K = 512 beyond a
# group, and 4 each of K = 128, 256, 384 on the next panel's columns and top rows),
# from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by what the same
# counters read for a 1 GiB copy (x2.0 and x1.0).  Valid for the sources it was
# taken on (hash of kernels_update.hip, the kernels, then kernels_lu.hip, the
# launch schedule); reported as null once either has changed.
KUPDATE_TRAFFIC = {"source_sha256_16": "5fec9a410800504f", "fetch_bytes": 1.3351e+09, "write_bytes": 4.5187e+08,
                   "fetch_scale": 2.0, "write_scale": 1.0}


def _update_traffic():
    import hashlib
    h = hashlib.sha256()
    try:
        for name in ("kernels_update.hip", "kernels_lu.hip"):
            h.update(open(os.path.join(ROOT, "paper_2502_16555_amd", "csrc", name), "rb").read())
    except OSError:
        return None
    if h.hexdigest()[:16] != KUPDATE_TRAFFIC["source_sha256_16"]:
        return None
    return KUPDATE_TRAFFIC["fetch_bytes"] + KUPDATE_TRAFFIC["write_bytes"]


def _update_launches(npad: int, nb: int, group: int = 2):
    """(flops, elements moved) of each trailing-update launch of one
    factorization, with the panels taken singly (group 1), in pairs (2) or in
    groups of four (4, statically pivoted dense factors).  In a group, a panel
    other than the last updates only the next panel's columns with the group's
    panels so far (K = 128 j: that column block read and written, the L rows and
    U columns read), and the last applies the whole group to the columns beyond
    (K = group nb, A22 read and written once); the panels after the last full
    group go singly (K = nb; pairs: the last two).  In groups of four the same
    launch also updates the next panel's top rows beyond it (one tile row, in
    place; its L rows are the column block's first); for pairs that update is
    part of the second panel's U12 pre-update, not of these launches."""
    npan = npad // nb
    out = []
    for p in range(npan):
        m = npad - p * nb - nb
        if group == 4:
            g0 = p // 4 * 4
            j = p - g0 if g0 + 4 <= npan else -1
        elif group == 2:
            j = p % 2 if (p % 2 == 0 and p + 2 < npan) or (p % 2 == 1 and p + 1 < npan) else -1
        else:
            j = -1
        if j >= 0 and j < group - 1:
            k = (j + 1) * nb
            if m > 0:
                fl, el = 2.0 * m * nb * k, 2 * m * nb + m * k + k * nb
                if group == 4 and m > nb:
                    # groups of four: the same launch updates the next panel's
                    # top rows beyond it too (in place)
                    w = m - nb
                    fl, el = fl + 2.0 * nb * w * k, el + 2 * nb * w + k * w
                out.append((fl, el))
        elif j == group - 1:
            k = group * nb
            if m > 0:
                out.append((2.0 * m * m * k, 2 * m * m + 2 * m * k))
        elif m > 0:
            out.append((2.0 * m * m * nb, 2 * m * m + 2 * m * nb))
    return out


def _update_bytes(npad: int, nb: int, nmat: int, elt: int, group: int = 2) -> float:
    """Algorithmic bytes of one average update launch (see _update_launches)."""
    ls = _update_launches(npad, nb, group)
    return sum(b for _, b in ls) * elt * nmat / len(ls)


def _update_flops(npad: int, nb: int, nmat: int, group: int = 2) -> float:
    """Algorithmic flops of all trailing-update launches of one factorization."""
    return sum(f for f, _ in _update_launches(npad, nb, group)) * nmat


def _panel_group(run) -> int:
    """Panels per deferred-update group of a timed run: groups of four need
    statically pivoted factors (otherwise the setting 2 takes pairs)."""
    pp = run["panel_pairs"]
    return 4 if pp == 2 and run["static_pivoting"] else (2 if pp else 1)


KRYLOV = dict(n_bins=128, bin_scale=100.0, restart=12, cycles=3, rtol=1e-12, factor_precision="mixed_fp32")


def run_gpu(cfg, precision, steps, warmup, torch, lu_streams=None, one_step=False, krylov=False, banded=False,
            pairs=None, vsolver=None, static_piv=None):
    from paper_2502_16555_amd import Solver, _lib
    t0 = time.time()
    s = Solver(cfg, precision=precision)
    if krylov:
        s.set_vsolver("gmres", **KRYLOV)
    if banded:
        s.set_vsolver("banded")
    if vsolver is not None:
        s.set_vsolver(vsolver)
    setup_s = time.time() - t0
    if lu_streams is not None:
        s.set_tuning(_lib.TUNE_LU_STREAMS, lu_streams)
    if pairs is not None:
        s.set_tuning(_lib.TUNE_PANEL_PAIRS, pairs)
    if static_piv is not None:
        s.set_tuning(_lib.TUNE_STATIC_PIVOTING, static_piv)
    import workloads
    ne = workloads.density_profile(s.xhat(), cfg["ic"]["ne_peak"])
    F = s.initial_state(torch.as_tensor(ne, device="cuda:0"), cfg["ic"]["Te_eV"])
    dt = cfg["dt_s"]
    first = None
    n = 0
    for _ in range(warmup):
        s.step(F, n * dt)
        n += 1
        if n == 1 and one_step:
            first = s.moments(F).cpu().numpy()
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
    n_end = n
    # kernel-level breakdown (separate, instrumented steps), then the phase
    # walls alone (no events inside the factorization to lengthen them)
    s.set_timing(True)
    nt = 3
    for _ in range(nt):
        s.step(F, n * dt)
        n += 1
    tm = s.timing()
    s.set_timing(True, walls_only=True)
    ntw = 10
    for _ in range(ntw):
        s.step(F, n * dt)
        n += 1
    tw = s.timing()
    s.set_timing(False)
    out = {"ms_per_step": ms, "wall_s": wall, "setup_s": setup_s, "refine_sweeps": sweeps, "refine_resid": resid,
           "moments": mom, "n_end": n_end, "first_step_moments": first,
           "ms_update": tm[0] / nt, "ms_panel": tm[1] / nt, "ms_vwall": tw[2] / ntw, "ms_x": tw[4] / ntw,
           "ms_vwall_kernel_timing": tm[2] / nt,
           "update_launches": tm[3] / nt, "lu_streams": s.get_tuning(_lib.TUNE_LU_STREAMS),
           "panel_pairs": s.get_tuning(_lib.TUNE_PANEL_PAIRS),
           "static_pivoting": s.get_tuning(_lib.TUNE_STATIC_PIVOTING),
           "info": s.info}
    s.close()
    return out


def rel_err(a, b, mask=None):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if mask is not None:
        a, b = a[mask], b[mask]
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def moment_errors(got, ref):
    """Relative max-norm errors per result: density, mean energy (on points with
    n_e > 1e-3 max n_e; the walls have n_e -> 0), energy density, k_i n_e."""
    mask = ref[0] > 1e-3 * ref[0].max()
    return {"n_e": rel_err(got[0], ref[0]), "mean_energy": rel_err(got[1], ref[1], mask),
            "energy_density": rel_err(got[0] * got[1], ref[0] * ref[1]),
            "k_i_n_e": rel_err(got[0] * got[2], ref[0] * ref[2])}


def golden_check(cfg, precision, torch, name="C2", n_steps=100):
    """Untimed: the first n_steps steps of the RF cycle from the initial state,
    compared every stored step with the stored FP64 oracle run of the same
    workload (tests/golden/<name>_oracle_<n_steps>.npz, written by the oracle
    alone); returns the largest relative error per result over the stored steps,
    or None when the file is absent or belongs to another workload."""
    path = os.path.join(ROOT, "tests", "golden", f"{name.lower()}_oracle_{n_steps}.npz")
    if not os.path.exists(path):
        return None
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import make_golden
    import workloads
    from paper_2502_16555_amd import Solver
    g = np.load(path, allow_pickle=False)
    if str(g["config_hash"]) != make_golden.config_hash(cfg):
        return None
    s = Solver(cfg, precision=precision)
    ne = workloads.density_profile(s.xhat(), cfg["ic"]["ne_peak"])
    F = s.initial_state(torch.as_tensor(ne, device="cuda:0"), cfg["ic"]["Te_eV"])
    every = int(g["every"])
    worst = {}
    for n in range(n_steps):
        s.step(F, n * cfg["dt_s"])
        if (n + 1) % every == 0:
            e = moment_errors(s.moments(F).cpu().numpy(), g["moments"][(n + 1) // every])
            for k, v in e.items():
                worst[k] = max(worst.get(k, 0.0), v)
    worst["final_state"] = rel_err(F.cpu().numpy(), g["F"])
    worst["steps"] = n_steps
    code = s.status()[0]
    s.close()
    if code != 0:
        raise RuntimeError(f"{precision}: device status {code} in the stored-run comparison")
    return worst


def run_hybrid(cfg, steps, warmup, torch):
    """The hybrid model's step at the bench grid: heavies' update (eq. fluid_step)
    with E^n from the Poisson field (V0 = 100 V), then the electron step with the
    Poisson field of the new ion density; mixed precision.  Times the whole step
    and, separately, the ion update alone."""
    import copy
    import workloads
    from paper_2502_16555_amd import Solver
    hc = copy.deepcopy(cfg)
    hc["field"] = {"kind": "poisson", "V0": 100.0, "freq_hz": workloads.RF_FREQ_HZ}
    s = Solver(hc, precision="mixed_fp32")
    ne = workloads.density_profile(s.xhat(), hc["ic"]["ne_peak"])
    F = s.initial_state(torch.as_tensor(ne, device="cuda:0"), hc["ic"]["Te_eV"])
    ni = torch.as_tensor(ne, device="cuda:0").clone()
    dt = hc["dt_s"]
    for k in range(warmup):
        s.hybrid_step(F, ni, k * dt)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        s.hybrid_step(F, ni, (warmup + k) * dt)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    out = torch.empty_like(ni)
    n_ion = 20
    e0.record()
    for k in range(n_ion):
        s.ion_step(F, ni, out, 0.0)
    e1.record()
    torch.cuda.synchronize()
    ms_ion = e0.elapsed_time(e1) / n_ion
    code = s.status()[0]
    if code != 0:
        raise RuntimeError(f"hybrid: device status {code}")
    mom = s.moments(F).cpu().numpy()
    res = {"workload": f"Nx={hc['nx']}, Nr={hc['nr']}, Ntheta={hc['ntheta']}, Poisson field V0=100 V, "
                       "ions: n0 mu_i = 4.65e21, n0 D_i = 2.07e20, mixed precision",
           "steps_per_s": 1000.0 / ms, "ms_per_step": ms, "ms_ion_update": ms_ion,
           "ni_range": [float(ni.min()), float(ni.max())], "ne_max": float(mom[0].max()),
           "finite": bool(np.isfinite(mom).all() and torch.isfinite(ni).all())}
    s.close()
    return res


def run_implicit(cfg, torch, runs=((0, 1.0), (1, 1.0), (0, 10.0))):
    """The fully implicit step at the bench grid (RF field, mixed-precision
    preconditioner): wall time per step, Newton and GMRES iterations, and the
    simulated time advanced per wall second against the semi-implicit step's,
    for each (preconditioner, step multiple) in runs: preconditioner 0 the V
    solve then the full-step x solve, 1 the semi-implicit step."""
    import copy
    import workloads
    from paper_2502_16555_amd import Solver
    opts = dict(newton_rtol=1e-8, gmres_rtol=1e-4, restart=60, max_gmres=1500, max_newton=8)
    names = {0: "V solve then x solve over dt", 1: "semi-implicit step X(dt/2) V(dt) X(dt/2)"}
    out = {"workload": f"Nx={cfg['nx']}, Nr={cfg['nr']}, Ntheta={cfg['ntheta']}, RF field, Newton-GMRES "
                       "with a mixed-precision operator-split preconditioner, one step from the initial state",
           "options": opts, "steps": []}
    for pk, mult in runs:
        c = copy.deepcopy(cfg)
        c["dt_s"] = cfg["dt_s"] * mult
        s = Solver(c, precision="mixed_fp32")
        ne = workloads.density_profile(s.xhat(), c["ic"]["ne_peak"])
        F = s.initial_state(torch.as_tensor(ne, device="cuda:0"), c["ic"]["Te_eV"])
        # first use: kernels loaded, workspace and the full-step x inverses built
        s.implicit_step(F.clone(), 0.0, max_newton=1, max_gmres=2, precond=pk, raise_on_noconv=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = s.implicit_step(F, 0.0, raise_on_noconv=False, precond=pk, **opts)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out["steps"].append({"preconditioner": names[pk], "dt_over_T_rf": c["dt_s"] / c["T_rf_s"],
                             "ms_per_step": wall * 1e3,
                             "newton_iters": st["newton_iters"], "gmres_iters": st["gmres_iters"],
                             "converged": st["status"] == 0, "residual_rel": st["residual"] / st["residual0"],
                             "simulated_s_per_wall_s": c["dt_s"] / wall})
        s.close()
    return out


def run_adjoint(torch, n_steps=1000, every=50):
    """Adjoint cost on the differentiation workload (Nx=128, Nr=64, Ntheta=32,
    8 bins x 3 processes + E0, FP64, one RF cycle of 1000 steps, checkpoints
    every 50): time of the checkpointed forward pass vs forward + reverse pass,
    operators set up beforehand."""
    import workloads
    from paper_2502_16555_amd import Solver
    from paper_2502_16555_amd.autograd import forward_cycle, reverse_cycle
    cfg = workloads.config("C4")
    s = Solver(cfg, precision="fp64")
    ne = workloads.density_profile(s.xhat(), cfg["ic"]["ne_peak"])
    F0 = s.initial_state(torch.as_tensor(ne, device="cuda:0"), cfg["ic"]["Te_eV"])
    forward_cycle(s, F0, 2, 0)               # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    nbar, ckpts = forward_cycle(s, F0, n_steps, every)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t
    g = 2.0 * (nbar - 1.05 * nbar.detach()) / 1e32
    t = time.perf_counter()
    gs, gE0, _ = reverse_cycle(s, ckpts, g, n_steps)
    torch.cuda.synchronize()
    t_rev = time.perf_counter() - t
    s.close()
    return {"workload": f"Nx=128, Nr=64, Ntheta=32, FP64, {s.n_params} scalings + E0, {n_steps} steps, "
                        f"checkpoint every {every}",
            "forward_s": t_fwd, "reverse_s": t_rev, "cost_ratio": (t_fwd + t_rev) / t_fwd,
            "grad_finite": bool(torch.isfinite(gs).all() and torch.isfinite(gE0).all())}


def run_ensemble(torch, steps=3):
    """Batching form: 64 discharges (Nx ~ U{32..200}, 0.1-2 Torr, E0 ~ U[1e3, 1e4]
    V/m, seed 1), mixed precision, all discharges in the same launches; the
    steps are captured once into a HIP graph and replayed."""
    import workloads
    from paper_2502_16555_amd import Solver
    cfg = workloads.config("C3")
    t = time.time()
    s = Solver(cfg, precision="mixed_fp32")
    setup_s = time.time() - t
    xh = s.xhat()
    ne = np.concatenate([workloads.density_profile(xh[o:o + n], cfg["ic"]["ne_peak"])
                         for o, n in zip(np.cumsum([0] + cfg["nx_per"][:-1]), cfg["nx_per"])])
    F = s.initial_state(torch.as_tensor(ne, device="cuda:0"), cfg["ic"]["Te_eV"])
    from paper_2502_16555_amd.autotune import autotune
    t = time.time()
    tuned = autotune(s, F, "mixed_fp32", steps=1)
    tune_s = time.time() - t
    t = time.time()
    s.graph_capture(F, 0.0, steps)
    capture_s = time.time() - t
    s.graph_launch()                      # warm-up replay
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    s.graph_launch()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    code = s.status()[0]
    info = s.info
    s.close()
    if code != 0:
        raise RuntimeError(f"ensemble: device status {code}")
    return {"workload": f"{info.n_discharges} discharges, sum Nx = {info.nx_total}, Nr=64, Ntheta=32, mixed FP32",
            "steps_per_s": 1000.0 / ms, "ms_per_step": ms, "point_steps_per_s": info.nx_total * 1000.0 / ms,
            "graph_steps": steps, "setup_s": setup_s, "capture_s": capture_s, "autotune_s": tune_s,
            "tuned": {"lu_streams": tuned["settings"][1 - 1], "update_kc": tuned["settings"][1],
                      "form_xpb": tuned["settings"][2], "trials": tuned["trials"],
                      "ms_per_step_tuned": tuned["ms_per_step"]},
            "device_GB": info.bytes_device / 1e9}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def paper_grid(torch, steps):
    """The grid of the paper's timed semi-implicit runs (table of the hybrid
    solver's performance: Nr = 64, Ntheta = 16, Nl = 3, Nx = 100, dt f = 5e-5),
    with this repository's synthetic RF physics, by every V solver here.  The
    paper's own time for that grid (GMRES V solver, 1 A100 + 1 CPU core, its
    LXCat physics) is quoted as context only."""
    import workloads
    cfg = dict(workloads.config("C1"), nx=100, nx_per=[100], ntheta=16, nl=3)
    cfg["dt_s"] = 5e-5 * cfg["T_rf_s"]
    out = {"workload": "Nx=100 CGL, Nr=64, Ntheta=16, Nl=3, dt = 5e-5 T_rf, RF E0=6732.7 V/m",
           "paper_context": {"s_per_step": 3.53e-2, "hardware": "1x A100 + 1 EPYC 7763 core",
                             "solver": "semi-implicit step, GMRES V solver (table of the hybrid solver's performance)"},
           "solvers": {}}
    for name, prec, vs in (("lu_fp64", "fp64", None), ("lu_mixed_fp32", "mixed_fp32", None),
                           ("banded_fp64", "fp64", "banded"), ("hessenberg_fp64", "fp64", "hessenberg")):
        r = run_gpu(cfg, prec, steps, 3, torch, vsolver=vs)
        out["solvers"][name] = {"ms_per_step": r["ms_per_step"], "steps_per_s": 1000.0 / r["ms_per_step"],
                                "setup_s": r["setup_s"]}
    out["implicit"] = paper_grid_implicit(cfg, torch, out["solvers"]["lu_mixed_fp32"]["ms_per_step"])
    return out


def paper_grid_implicit(cfg, torch, semi_ms, mult=4, n_steps=5):
    """The paper's comparison on its timed grid: the fully implicit step at
    mult = 4 times the semi-implicit dt (dt f = 2e-4 against 5e-5 in the table of
    the hybrid solver's performance), mixed-precision preconditioner, n_steps
    consecutive steps from the initial state, with each preconditioner.  The
    overall speedup is the semi-implicit time for the same simulated time over
    the fully implicit one (the table's last column)."""
    import copy
    import workloads
    from paper_2502_16555_amd import Solver
    opts = dict(newton_rtol=1e-8, gmres_rtol=1e-4, restart=60, max_gmres=1500, max_newton=8)
    c = copy.deepcopy(cfg)
    c["dt_s"] = cfg["dt_s"] * mult
    out = {"dt_over_T_rf": c["dt_s"] / c["T_rf_s"], "steps": n_steps, "options": opts,
           "semi_implicit_ms_per_step": semi_ms, "runs": []}
    for pk, name in ((0, "V solve then x solve over dt"), (1, "semi-implicit step X(dt/2) V(dt) X(dt/2)")):
        s = Solver(c, precision="mixed_fp32")
        ne = workloads.density_profile(s.xhat(), c["ic"]["ne_peak"])
        F = s.initial_state(torch.as_tensor(ne, device="cuda:0"), c["ic"]["Te_eV"])
        s.implicit_step(F.clone(), 0.0, max_newton=1, max_gmres=2, precond=pk, raise_on_noconv=False)
        torch.cuda.synchronize()
        newton = gmres = 0
        ok = True
        t0 = time.perf_counter()
        for k in range(n_steps):
            st = s.implicit_step(F, k * c["dt_s"], raise_on_noconv=False, precond=pk, **opts)
            newton += st["newton_iters"]
            gmres += st["gmres_iters"]
            ok = ok and st["status"] == 0
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / n_steps
        out["runs"].append({"preconditioner": name, "ms_per_step": ms, "newton_per_step": newton / n_steps,
                            "gmres_per_step": gmres / n_steps, "converged": ok,
                            "speedup_over_semi_implicit": mult * semi_ms / ms})
        s.close()
    return out


def cpu_baseline(cfg):
    """The FP64 oracle on the host cores: one full step from the initial state
    (both X half-steps and all Nx velocity-space solves).  Returns the timing and
    the moments after the step (the reference of the one-step accuracy check).
    ``cores`` is the number of BLAS threads the oracle's LAPACK calls ran on (read
    from the loaded BLAS library), beside the host's CPU model and logical CPUs."""
    import oracle
    from oracle import semi_implicit as S
    import workloads
    ops = oracle.build_operators(cfg)
    F = S.initial_state(ops, workloads.density_profile(ops.xhat, cfg["ic"]["ne_peak"]), cfg["ic"]["Te_eV"])
    t = time.perf_counter()
    F1 = S.step(ops, F, 0.0)
    step_s = time.perf_counter() - t
    try:
        from threadpoolctl import threadpool_info
        threads = max(int(p["num_threads"]) for p in threadpool_info() if p.get("user_api") == "blas")
    except Exception:
        threads = int(os.environ.get("OPENBLAS_NUM_THREADS", os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    res = {"value": 1.0 / step_s, "unit": "steps/s", "cores": threads, "kind": "oracle",
           "sample": f"one full step (t=0, from the initial state) at Nx={ops.nx}: {step_s:.1f} s",
           "cpu_model": _cpu_model(), "logical_cpus": os.cpu_count()}
    return res, S.moments(ops, F1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="mixed_fp32", choices=["mixed_fp32", "mixed_bf16x3", "mixed_bf16", "fp64"])
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--lu-streams", type=int, default=None, help="concurrent factorization groups (library default 1)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint-cost leg")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 64-discharge batching form")
    ap.add_argument("--no-krylov", action="store_true", help="skip the GMRES V-solver leg")
    ap.add_argument("--no-partial", action="store_true",
                    help="skip the mixed step with partially pivoted FP32 factors")
    ap.add_argument("--no-banded", action="store_true", help="skip the banded harmonic-basis V-solver leg")
    ap.add_argument("--no-hybrid", action="store_true", help="skip the hybrid-model (ions + electrons) leg")
    ap.add_argument("--no-hessenberg", action="store_true", help="skip the Hessenberg-form V-solver leg")
    ap.add_argument("--no-paper-grid", action="store_true", help="skip the legs at the paper's timed grid")
    ap.add_argument("--no-implicit", action="store_true", help="skip the fully implicit step leg")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16 variants (split and plain operands)")
    ap.add_argument("--no-golden", action="store_true",
                    help="skip the comparison of the first 100 steps with the stored oracle run")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy a 1 GiB buffer 3 times (reference kernel for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the step is measured on a single GPU",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        n = (1 << 30) // 4
        src = torch.rand(n, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read_per_copy": 4 * n, "bytes_written_per_copy": 4 * n,
                                               "copies": 3}}), flush=True)
        return
    cfg = workloads.config("C2")
    if args.nx != 256:
        cfg = dict(cfg, nx=args.nx, nx_per=[args.nx])
    warm = max(args.warmup, 1)
    main_run = run_gpu(cfg, args.precision, args.steps, warm, torch, args.lu_streams, one_step=True)
    fp64 = None
    if not args.no_fp64 and args.precision != "fp64":
        # same number of steps from the same state, so the final moments compare
        fp64 = run_gpu(cfg, "fp64", args.steps, warm, torch, args.lu_streams, one_step=True)
    info = main_run["info"]
    nx_total, n = info.nx_total, info.n
    npad = ((n + 127) // 128) * 128
    dtype = {"fp64": "f64", "mixed_fp32": "f32+f64", "mixed_bf16": "bf16+f32+f64", "mixed_bf16x3": "bf16x3+f32+f64"}[args.precision]
    mfma = {"fp64": "fp64", "mixed_fp32": "fp32", "mixed_bf16": "bf16", "mixed_bf16x3": "bf16"}[args.precision]
    # update flops of one step over the summed durations of its update launches
    group = _panel_group(main_run)
    upd_flops = _update_flops(npad, 128, nx_total, group)
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
                     "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": _update_traffic() if args.precision == "mixed_fp32" and npad == 2048 and nx_total == 256
                     else None,
                     "algorithmic_bytes_per_launch": _update_bytes(npad, 128, nx_total,
                                                                   8 if args.precision == "fp64" else 4, group),
                     "panels_per_update_group": group,
                     "launches_per_step": n_upd_launches,
                     "avg_launch_ms": main_run["ms_update"] / n_upd_launches},
        "v_solve_roofline": {"bound": "mfma", "what": "whole velocity-space solve: formation, factorization, "
                                                      "solves and FP64 refinement, wall time",
                             "lu_flops": info.lu_flops_per_step, "ms": main_run["ms_vwall"],
                             "achieved": info.lu_flops_per_step / (main_run["ms_vwall"] * 1e-3) / 1e12,
                             "peak": peak, "unit": "TFLOP/s",
                             "frac": info.lu_flops_per_step / (main_run["ms_vwall"] * 1e-3) / 1e12 / peak},
        "breakdown_ms": {"lu_update_launches": main_run["ms_update"], "lu_panel_u12_launches": main_run["ms_panel"],
                         "v_step_wall": main_run["ms_vwall"], "x_and_field_wall": main_run["ms_x"],
                         "v_step_wall_with_launch_events": main_run["ms_vwall_kernel_timing"],
                         "lu_streams": main_run["lu_streams"]},
        "lu_tflops_step": info.lu_flops_per_step / (main_run["ms_per_step"] * 1e-3) / 1e12,
        "refine": {"sweeps": main_run["refine_sweeps"], "resid": main_run["refine_resid"]},
        "pivoting": ("static (no interchanges; E < 0 points factored as their angular mirror image)"
                     if main_run["static_pivoting"] else "partial"),
    }
    if fp64 is not None:
        line["fp64"] = {"steps_per_s": 1000.0 / fp64["ms_per_step"], "ms_per_step": fp64["ms_per_step"],
                        "speedup_mixed_over_fp64": fp64["ms_per_step"] / main_run["ms_per_step"],
                        "ms_update": fp64["ms_update"], "ms_panel": fp64["ms_panel"], "ms_vwall": fp64["ms_vwall"],
                        "v_solve_frac_fp64_peak": info.lu_flops_per_step / (fp64["ms_vwall"] * 1e-3) / 1e12
                        / MI355X_PEAK_TFLOPS["fp64"],
                        "update_tflops": _update_flops(npad, 128, nx_total, _panel_group(fp64))
                        / (fp64["ms_update"] * 1e-3) / 1e12,
                        "update_frac_fp64_peak": _update_flops(npad, 128, nx_total, _panel_group(fp64))
                        / (fp64["ms_update"] * 1e-3)
                        / 1e12 / MI355X_PEAK_TFLOPS["fp64"]}
        line["accuracy"] = {
            "mixed_vs_fp64_gpu": dict(moment_errors(main_run["moments"], fp64["moments"]),
                                      steps=main_run["n_end"])}
    if not args.no_partial and args.precision != "fp64":
        # the same mixed step with partially pivoted FP32 factors (128 pivot
        # searches per panel), for comparison with the statically pivoted default
        pp = run_gpu(cfg, args.precision, args.steps, warm, torch, args.lu_streams, static_piv=0)
        line["partial_pivoting"] = {"steps_per_s": 1000.0 / pp["ms_per_step"], "ms_per_step": pp["ms_per_step"],
                                    "ms_update": pp["ms_update"], "ms_panel": pp["ms_panel"],
                                    "ms_vwall": pp["ms_vwall"],
                                    "refine": {"sweeps": pp["refine_sweeps"], "resid": pp["refine_resid"]},
                                    "static_over_partial_speedup": pp["ms_per_step"] / main_run["ms_per_step"]}
        if fp64 is not None:
            line["partial_pivoting"]["vs_fp64_gpu"] = dict(moment_errors(pp["moments"], fp64["moments"]),
                                                           steps=pp["n_end"])
    if not args.no_krylov:
        kr = run_gpu(cfg, "fp64", args.steps, warm, torch, args.lu_streams, krylov=True)
        line["krylov"] = {"solver": "restarted GMRES per point, FP64, field-binned preconditioner "
                                    "(Alg. vspace_action_precon), bins factored and stored in FP32",
                          "settings": KRYLOV, "steps_per_s": 1000.0 / kr["ms_per_step"],
                          "ms_per_step": kr["ms_per_step"], "iterations_last_step": kr["refine_sweeps"],
                          "resid_estimate": kr["refine_resid"]}
        if fp64 is not None:
            line["krylov"]["speedup_over_fp64_lu"] = fp64["ms_per_step"] / kr["ms_per_step"]
            line["krylov"]["vs_fp64_lu"] = dict(moment_errors(kr["moments"], fp64["moments"]), steps=kr["n_end"])
    bf = None
    if not args.no_bf16 and args.precision != "mixed_bf16x3":
        # the BF16 variant of the precision form: trailing updates with split bf16
        # operands (three products), same FP64 refinement
        bf = run_gpu(cfg, "mixed_bf16x3", args.steps, warm, torch, args.lu_streams, one_step=True)
        nup = bf["update_launches"]
        line["bf16x3"] = {"steps_per_s": 1000.0 / bf["ms_per_step"], "ms_per_step": bf["ms_per_step"],
                          "ms_update": bf["ms_update"], "ms_panel": bf["ms_panel"], "ms_vwall": bf["ms_vwall"],
                          "update_hbm_frac": (_update_bytes(npad, 128, nx_total, 4, _panel_group(bf))
                                              / (bf["ms_update"] / nup * 1e-3))
                          / (MI355X_PEAK_HBM_GBS * 1e9),
                          "refine": {"sweeps": bf["refine_sweeps"], "resid": bf["refine_resid"]}}
        if fp64 is not None:
            line["bf16x3"]["speedup_over_fp64"] = fp64["ms_per_step"] / bf["ms_per_step"]
            line["bf16x3"]["vs_fp64_gpu"] = dict(moment_errors(bf["moments"], fp64["moments"]), steps=bf["n_end"])
    bfp = None
    if not args.no_bf16 and args.precision != "mixed_bf16":
        # plain bf16 operands in the trailing updates (one product), same FP64 refinement
        bfp = run_gpu(cfg, "mixed_bf16", args.steps, warm, torch, args.lu_streams, one_step=True)
        nup = bfp["update_launches"]
        line["bf16"] = {"steps_per_s": 1000.0 / bfp["ms_per_step"], "ms_per_step": bfp["ms_per_step"],
                        "ms_update": bfp["ms_update"], "ms_panel": bfp["ms_panel"], "ms_vwall": bfp["ms_vwall"],
                        "update_hbm_frac": (_update_bytes(npad, 128, nx_total, 4, _panel_group(bfp))
                                            / (bfp["ms_update"] / nup * 1e-3)) / (MI355X_PEAK_HBM_GBS * 1e9),
                        "refine": {"sweeps": bfp["refine_sweeps"], "resid": bfp["refine_resid"]}}
        if fp64 is not None:
            line["bf16"]["speedup_over_fp64"] = fp64["ms_per_step"] / bfp["ms_per_step"]
            line["bf16"]["vs_fp64_gpu"] = dict(moment_errors(bfp["moments"], fp64["moments"]), steps=bfp["n_end"])
    if not args.no_golden and args.nx == 256:
        vs = {}
        for prec in dict.fromkeys([args.precision, "fp64", "mixed_bf16x3", "mixed_bf16"]):
            r = golden_check(cfg, prec, torch)
            if r is None:
                break
            vs[prec] = r
        if vs:
            line.setdefault("accuracy", {})["vs_oracle_stored_run"] = vs
    if not args.no_banded:
        bd = run_gpu(cfg, "fp64", args.steps, warm, torch, args.lu_streams, banded=True)
        line["banded"] = {"solver": "FP64 batched LU of the harmonic-basis systems restricted to their band "
                                    "(half-bandwidth 2 Nr - 1, eq. f_expansion)",
                          "steps_per_s": 1000.0 / bd["ms_per_step"], "ms_per_step": bd["ms_per_step"],
                          "ms_update": bd["ms_update"], "ms_panel": bd["ms_panel"], "ms_vwall": bd["ms_vwall"]}
        if fp64 is not None:
            line["banded"]["speedup_over_fp64_lu"] = fp64["ms_per_step"] / bd["ms_per_step"]
            line["banded"]["vs_fp64_lu"] = dict(moment_errors(bd["moments"], fp64["moments"]), steps=bd["n_end"])
    if not args.no_hessenberg:
        hs = run_gpu(cfg, "fp64", args.steps, warm, torch, args.lu_streams, vsolver="hessenberg")
        line["hessenberg"] = {"solver": "harmonic-basis systems in Hessenberg form (one Householder reduction per "
                                        "discharge at setup, one O(n^2) Givens solve per point and step), FP64",
                              "steps_per_s": 1000.0 / hs["ms_per_step"], "ms_per_step": hs["ms_per_step"],
                              "ms_vwall": hs["ms_vwall"], "setup_s": hs["setup_s"]}
        if fp64 is not None:
            line["hessenberg"]["speedup_over_fp64_lu"] = fp64["ms_per_step"] / hs["ms_per_step"]
            line["hessenberg"]["vs_fp64_lu"] = dict(moment_errors(hs["moments"], fp64["moments"]), steps=hs["n_end"])
    if not args.no_paper_grid:
        line["paper_grid"] = paper_grid(torch, min(args.steps, 20))
    if not args.no_hybrid:
        line["hybrid"] = run_hybrid(cfg, min(args.steps, 20), 2, torch)
    if not args.no_implicit:
        line["implicit"] = run_implicit(cfg, torch)
        line["implicit"]["semi_implicit_simulated_s_per_wall_s"] = cfg["dt_s"] / (main_run["ms_per_step"] * 1e-3)
    if not args.no_adjoint:
        line["adjoint"] = run_adjoint(torch)
    if not args.no_ensemble:
        line["ensemble"] = run_ensemble(torch)
        line["ensemble"]["point_steps_per_s_single_discharge"] = nx_total * value
    if not args.no_cpu:
        cb, mom1 = cpu_baseline(cfg)
        line["cpu_baseline"] = cb
        acc = line.setdefault("accuracy", {})
        acc["vs_oracle_one_step"] = {args.precision: moment_errors(main_run["first_step_moments"], mom1)}
        if fp64 is not None:
            acc["vs_oracle_one_step"]["fp64"] = moment_errors(fp64["first_step_moments"], mom1)
        if bf is not None:
            acc["vs_oracle_one_step"]["mixed_bf16x3"] = moment_errors(bf["first_step_moments"], mom1)
        if bfp is not None:
            acc["vs_oracle_one_step"]["mixed_bf16"] = moment_errors(bfp["first_step_moments"], mom1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
