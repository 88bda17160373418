"""Launch-shape autotuner for the batched step.

The library exposes launch shapes that do not change results (bte_set_tuning):
the number of concurrent factorization groups, the K chunk of the trailing
update tiles, the number of matrices per formation block and the look-ahead
of the statically pivoted panels.  The best shape
depends on the size class of the problem (unknowns per point, number of points,
precision), e.g. a 64-discharge ensemble of 7000+ points against a single
discharge of 9.  ``autotune`` times a few steps per candidate by coordinate
descent on a scratch copy of the state and keeps the fastest; results are cached
per size class in a JSON file so that later handles of the same class reuse them.
"""
from __future__ import annotations

import json
import os

from . import _lib


def candidates(precision: str) -> dict:
    """Candidate values per tuning key (the first one is the library default)."""
    kc = [16, 8] if precision == "fp64" else [16, 32]
    if precision in ("mixed_bf16", "mixed_bf16x3"):
        kc = [32]   # the bf16 updates have a fixed chunk
    c = {_lib.TUNE_LU_STREAMS: [1, 2], _lib.TUNE_UPDATE_KC: kc, _lib.TUNE_FORM_XPB: [8, 4, 16, 32]}
    if precision != "fp64":
        c[_lib.TUNE_LOOK_AHEAD] = [0, 1]   # the statically pivoted panels on a side stream
    return c


def size_class(n: int, nx_total: int, precision: str) -> str:
    """Points are bucketed by powers of two (the launch grids scale with them)."""
    b = 1
    while b < nx_total:
        b *= 2
    return f"n{n}-x{b}-{precision}"


def _time_steps(solver, F, t0, steps):
    import torch
    Fs = F.clone()
    dt = solver.cfg["dt_s"]
    solver.step(Fs, t0)                         # warm the shape once
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for k in range(steps):
        solver.step(Fs, t0 + (k + 1) * dt)
    e1.record()
    torch.cuda.synchronize()
    code = solver.status()[0]
    if code != _lib.BTE_OK:
        raise _lib.BteError(code, "autotune")
    return e0.elapsed_time(e1) / steps


def coordinate_descent(apply, measure, cands: dict, rounds: int = 1):
    """Minimize measure() over the product of candidate lists, one key at a time.

    apply(key, value) sets a value; measure() returns a cost for the values set.
    Returns (best settings {key: value}, best cost, trials [(settings, cost)])."""
    best = {k: v[0] for k, v in cands.items()}
    for k, v in best.items():
        apply(k, v)
    best_cost = measure()
    trials = [(dict(best), best_cost)]
    for _ in range(rounds):
        for k, vals in cands.items():
            for v in vals:
                if v == best[k]:
                    continue
                apply(k, v)
                c = measure()
                trial = dict(best)
                trial[k] = v
                trials.append((trial, c))
                if c < best_cost:
                    best_cost, best[k] = c, v
            apply(k, best[k])
    return best, best_cost, trials


def autotune(solver, F, precision: str, t0: float = 0.0, steps: int = 2, cache_path: str | None = None,
             measure=None) -> dict:
    """Pick and apply the fastest launch shapes for ``solver`` (state F is not modified).

    Returns {"class": ..., "settings": {key: value}, "ms_per_step": best, "trials": n, "cached": bool}."""
    cls = size_class(solver.n, solver.nx_total, precision)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    if cls in cache:
        settings = {int(k): int(v) for k, v in cache[cls]["settings"].items()}
        for k, v in settings.items():
            solver.set_tuning(k, v)
        return {"class": cls, "settings": settings, "ms_per_step": cache[cls]["ms_per_step"], "trials": 0,
                "cached": True}
    if measure is None:
        def measure():
            return _time_steps(solver, F, t0, steps)
    best, cost, trials = coordinate_descent(solver.set_tuning, measure, candidates(precision))
    if cache_path:
        cache[cls] = {"settings": {str(k): v for k, v in best.items()}, "ms_per_step": cost}
        d = os.path.dirname(os.path.abspath(cache_path))
        os.makedirs(d, exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return {"class": cls, "settings": best, "ms_per_step": cost, "trials": len(trials), "cached": False}
