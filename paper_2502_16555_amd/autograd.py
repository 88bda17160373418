"""Differentiation through a run of semi-implicit steps (torch.autograd).

The forward pass advances F with ``bte_step`` and keeps a checkpoint of the
state every K steps; the reverse pass recomputes one segment at a time from its
checkpoint and walks it backwards with the hand-written transposed step
``bte_adjoint_step`` (X^T, then A^-T with the factors of the recomputed step,
then X^T), which also accumulates the gradients with respect to the
collision-operator scalings of eq. (c_en_mat_1d) per (process, energy bin) and
the field of eq. (bte_semi_implicit_efield).  Only the state of one segment is
held at a time, so memory is O(K + N/K) states for N steps.

The differentiated quantity is the cycle-mean density profile
    nbar_x = (1/N) sum_{n=1..N} u^T F^n_x,
as a function of the scalings ``scal`` [n_proc, n_bins], the RF amplitude
factor ``e0_scale`` (E0 -> e0_scale * E0) and the initial state F^0; a loss
built on it in torch (e.g. a weighted misfit to a target profile) chains
through ``backward``.
"""
from __future__ import annotations

import copy

import numpy as np

from . import _lib
from .solver import Solver


def param_config(cfg: dict, scal, e0_scale: float) -> dict:
    """``cfg`` with collision scalings ``scal`` and the field amplitude(s) times ``e0_scale``."""
    c = copy.copy(cfg)
    nb = int(cfg.get("n_bins", 1))
    c["scal"] = np.asarray(scal, dtype=np.float64).reshape(len(cfg["processes"]), nb)
    c["field"] = dict(cfg["field"], E0=float(cfg["field"].get("E0", 0.0)) * float(e0_scale))
    if "E0_per" in cfg:
        c["E0_per"] = [float(e) * float(e0_scale) for e in cfg["E0_per"]]
    return c


def forward_cycle(solver: Solver, F0, n_steps: int, every: int, t0: float = 0.0):
    """Advance n_steps from F0 (not modified).  Returns (nbar [sum Nx], checkpoints {step: F})."""
    import torch
    dt = solver.cfg["dt_s"]
    F = F0.detach().clone().contiguous()
    ckpts = {0: F.clone()}
    mom = torch.empty((3, solver.nx_total), dtype=torch.float64, device=F.device)
    acc = torch.zeros(solver.nx_total, dtype=torch.float64, device=F.device)
    for n in range(n_steps):
        solver.step(F, t0 + n * dt)
        solver.moments(F, out=mom)
        acc += mom[0]
        if every and (n + 1) % every == 0 and n + 1 < n_steps:
            ckpts[n + 1] = F.clone()
    code = solver.status()[0]
    if code != _lib.BTE_OK:
        raise _lib.BteError(code, "forward_cycle")
    return acc / n_steps, ckpts


def reverse_cycle(solver: Solver, ckpts: dict, g, n_steps: int, t0: float = 0.0):
    """Reverse pass for a cotangent g [sum Nx] of nbar.

    Returns (grad_scal [n_params], grad_E0 [n_discharges] = dL/dE0_d in 1/(V/m),
    dL/dF^0)."""
    import torch
    dt = solver.cfg["dt_s"]
    dev = ckpts[0].device
    nxt = solver.nx_total
    gbar = torch.zeros((3, nxt), dtype=torch.float64, device=dev)
    gbar[0] = g.to(device=dev, dtype=torch.float64) / n_steps
    lam = torch.zeros_like(ckpts[0])
    grad_scal = torch.zeros(max(solver.n_params, 1), dtype=torch.float64, device=dev)
    grad_E0 = torch.zeros(max(solver.n_discharges, 1), dtype=torch.float64, device=dev)
    starts = sorted(ckpts)
    for si in range(len(starts) - 1, -1, -1):
        a = starts[si]
        b = starts[si + 1] if si + 1 < len(starts) else n_steps
        states = [ckpts[a]]
        for n in range(a, b):                       # recompute the segment
            F = states[-1].clone()
            solver.step(F, t0 + n * dt)
            states.append(F)
        for n in range(b, a, -1):                   # lam: dL/dF^n -> dL/dF^{n-1}
            solver.moments_vjp(states[n - a], gbar, lam)
            solver.adjoint_step(states[n - 1 - a], t0 + (n - 1) * dt, lam, grad_scal, grad_E0)
        del states
    code = solver.status()[0]
    if code != _lib.BTE_OK:
        raise _lib.BteError(code, "reverse_cycle")
    return grad_scal[:solver.n_params], grad_E0[:solver.n_discharges], lam


def _function():
    import torch

    class CycleMeanDensity(torch.autograd.Function):
        """nbar = CycleMeanDensity.apply(scal, e0_scale, F0, cfg, n_steps, every, precision, t0)."""

        @staticmethod
        def forward(ctx, scal, e0_scale, F0, cfg, n_steps, every, precision, t0):
            c = param_config(cfg, scal.detach().cpu().numpy(), float(e0_scale))
            solver = Solver(c, precision=precision)
            try:
                nbar, ckpts = forward_cycle(solver, F0, n_steps, every, t0)
            except Exception:
                solver.close()
                raise
            ctx.solver, ctx.ckpts = solver, ckpts
            ctx.meta = (n_steps, t0, scal.shape, scal.dtype, scal.device)
            ctx.E0_base = np.asarray(cfg.get("E0_per", [cfg["field"].get("E0", 0.0)]), dtype=np.float64)
            if int(cfg.get("n_discharges", 1)) == 1:
                ctx.E0_base = np.array([cfg["field"].get("E0", 0.0)], dtype=np.float64)
            return nbar

        @staticmethod
        def backward(ctx, g):
            n_steps, t0, shape, dtype, device = ctx.meta
            try:
                gs, gE0, lam0 = reverse_cycle(ctx.solver, ctx.ckpts, g, n_steps, t0)
            finally:
                ctx.solver.close()
                ctx.ckpts = None
            g_scal = gs.to(device=device, dtype=dtype).reshape(shape)
            g_e0 = (gE0.cpu() * torch.as_tensor(ctx.E0_base, dtype=torch.float64)).sum()
            return g_scal, g_e0.to(dtype=dtype), lam0, None, None, None, None, None

    return CycleMeanDensity


_FN = None


def cycle_mean_density(scal, e0_scale, F0, cfg: dict, n_steps: int, every: int = 50, precision: str = "fp64",
                       t0: float = 0.0):
    """Differentiable cycle-mean density profile [sum Nx] (see the module docstring).

    scal: tensor [n_proc, n_bins] (CPU), e0_scale: 0-d tensor (CPU), F0: device
    state [sum Nx][Nr][Ntheta].  Gradients flow to all three."""
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN.apply(scal, e0_scale, F0, cfg, n_steps, every, precision, t0)
