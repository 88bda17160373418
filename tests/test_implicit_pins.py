"""Pins of the oracle's fully implicit step (eq. bte_fully_implicit), CPU only.

Against: central differences of the residual (exact for its quadratic field
coupling), an independent Kronecker assembly of the linear (specified-field)
system, and the O(dt^2) per-step agreement with the semi-implicit step."""
import numpy as np
import pytest

import oracle
import workloads
from oracle import implicit as I
from oracle import semi_implicit as S


def _cfg(nx=5, nr=4, nth=4, kind="poisson"):
    cfg = workloads.small_config(nx=nx, nr=nr, nth=nth, kinds=("elastic", "ionization"), E=4e3,
                                 field_kind="const")
    if kind == "poisson":
        cfg["field"] = {"kind": "poisson", "V0": 80.0, "freq_hz": workloads.RF_FREQ_HZ}
    return cfg


def _state(ops, seed=1):
    F = S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 2.0)
    rng = np.random.default_rng(seed)
    F = F * (1.0 + 0.1 * rng.standard_normal(F.shape))
    F[I.inflow_mask(ops)] = 0.0
    return F


def test_jacobian_matches_central_differences():
    """The residual is quadratic in F (the field is affine in F), so central
    differences reproduce the Jacobian up to rounding."""
    ops = oracle.build_operators(_cfg())
    F = _state(ops)
    ni = 1.2 * S.moments(ops, F)[0]
    t1 = 0.3 * workloads.rf_period_s()
    J = I.jacobian(ops, F, t1, ni)
    h = 1e-3 * np.abs(F).max()
    N = F.size
    Jfd = np.zeros((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = h
        Rp = I.residual(ops, F + e.reshape(F.shape), F, t1, ni)
        Rm = I.residual(ops, F - e.reshape(F.shape), F, t1, ni)
        Jfd[:, c] = (Rp - Rm).ravel() / (2 * h)
    assert np.abs(J - Jfd).max() <= 1e-7 * np.abs(J).max()
    # the E(X) . F coupling is present (it is what the semi-implicit step leaves out)
    El = I.field(ops, F, t1, linear=True)
    assert np.abs(El).max() > 0


def test_linear_case_against_kronecker_assembly():
    """Specified (constant) field: one linear system, assembled here from
    Kronecker products in the x-major (x, k, a) ordering."""
    ops = oracle.build_operators(_cfg(kind="const"))
    F = _state(ops, 2)
    got, its = I.implicit_step(ops, F, 0.0)
    assert its <= 2
    nx, n = ops.nx, ops.nr * ops.nth
    MinvG = np.linalg.solve(ops.M, ops.G)
    Ax = np.kron(MinvG, np.diag(ops.mu))
    E = ops.cfg["field"]["E0"]
    K = (np.eye(nx * n) + ops.dt * np.kron(ops.Dx, Ax)
         - ops.dt * np.kron(np.eye(nx), ops.n0 * ops.Cord + E * ops.Aord))
    m = I.inflow_mask(ops).ravel()
    K[m, :] = 0.0
    K[m, m] = 1.0
    rhs = F.ravel().copy()
    rhs[m] = 0.0
    want = np.linalg.solve(K, rhs).reshape(F.shape)
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()


def test_agrees_with_semi_implicit_to_second_order():
    """Both schemes are first-order consistent: their one-step difference from
    the same smooth state shrinks like dt^2."""
    diffs = []
    for dt_frac in (2e-4, 1e-4):
        cfg = _cfg(nx=9, nr=6, nth=4, kind="const")
        cfg["dt_s"] = dt_frac * workloads.rf_period_s()
        ops = oracle.build_operators(cfg)
        F = S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 2.0)
        F[I.inflow_mask(ops)] = 0.0
        Fi, _ = I.implicit_step(ops, F, 0.0)
        Fs = S.step(ops, F, 0.0)
        diffs.append(np.abs(Fi - Fs).max() / np.abs(F).max())
    ratio = diffs[0] / diffs[1]
    assert 3.0 < ratio < 5.0, (diffs, ratio)
