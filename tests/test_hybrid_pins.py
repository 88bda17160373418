"""Pins of the oracle's hybrid step (ion fluid update of eq. fluid_step), CPU only.

Each pin checks the oracle against something other than itself: exact
derivatives of polynomials (manufactured solutions), the closed-form decay of a
Neumann cosine mode under implicit Euler, a uniform source, and the moments."""
import math

import numpy as np
import numpy.polynomial.polynomial as P
import pytest

import oracle
import workloads
from oracle import hybrid as H
from oracle import semi_implicit as S


def _ops(nx=24):
    cfg = workloads.small_config(nx=nx, nr=6, nth=4, kinds=("elastic", "ionization"))
    cfg["field"] = {"kind": "poisson", "V0": 100.0, "freq_hz": workloads.RF_FREQ_HZ}
    return oracle.build_operators(cfg)


@pytest.mark.parametrize("signs", [(1.0, 1.0), (-1.0, -1.0), (-1.0, 1.0)])
def test_ion_matrix_manufactured_polynomials(signs):
    """M n = b with b from exact derivatives: n of degree 5 and E of degree 4 in x
    (their product is below the collocation degree, so D_x is exact on them).
    The wall rows follow the outflow condition for every sign of E at the walls."""
    ops = _ops(24)
    L, dt = ops.L, ops.dt
    x = 0.5 * L * (ops.xhat + 1.0)
    s0, sL = signs
    # n > 0; E = linear from s0 * 2e3 at x = 0 to sL * 3e3 at x = L, plus bumps that
    # vanish at both walls (x (x - L) and x^2 (x - L)^2)
    cn = np.array([1.0, 0.3, -0.2, 0.1, 0.05, -0.02]) * 1e16 / L ** np.arange(6)
    wall = np.array([0.0, -L, 1.0])                                  # x (x - L)
    ce = P.polyadd([s0 * 2e3, (sL * 3e3 - s0 * 2e3) / L],
                   P.polyadd(500.0 / L ** 2 * wall, -800.0 / L ** 4 * P.polymul(wall, wall)))
    mu, D = H.ion_coefficients(ops)
    n = P.polyval(x, cn)
    E = P.polyval(x, ce)
    flux = P.polysub(mu * P.polymul(ce, cn), D * P.polyder(cn))      # J = mu E n - D n'
    b = n / dt + P.polyval(x, P.polyder(flux))
    J0, JL = P.polyval(0.0, flux), P.polyval(L, flux)
    b[0] = -J0 - max(0.0, -mu * E[0]) * n[0]
    b[-1] = JL - max(0.0, mu * E[-1]) * n[-1]
    M = H.ion_matrix(ops, E, mu, D)
    assert np.abs(M @ n - b).max() <= 1e-9 * np.abs(b).max()
    assert np.abs(H.ion_solve(ops, M, b) - n).max() <= 1e-10 * np.abs(n).max()


def test_ion_neumann_cosine_decay():
    """E = 0, no source: the walls reduce to zero diffusive flux and
    1 + cos(pi x / L) decays as 1 + cos(pi x / L) / (1 + dt D (pi / L)^2)
    (spectral accuracy at 40 nodes; dt = 1 ms, so that the decay is about 10%)."""
    cfg = workloads.small_config(nx=40, nr=6, nth=4, kinds=("elastic",))
    cfg["field"] = {"kind": "poisson", "V0": 0.0, "freq_hz": workloads.RF_FREQ_HZ}
    cfg["dt_s"] = 1e-3
    ops = oracle.build_operators(cfg)
    L, dt = ops.L, ops.dt
    x = 0.5 * L * (ops.xhat + 1.0)
    mu, D = H.ion_coefficients(ops)
    n = 1e16 * (1.0 + np.cos(math.pi * x / L))
    got = H.ion_solve(ops, H.ion_matrix(ops, np.zeros(ops.nx), mu, D), H.ion_rhs(ops, n, np.zeros(ops.nx)))
    want = 1e16 * (1.0 + np.cos(math.pi * x / L) / (1.0 + dt * D * (math.pi / L) ** 2))
    assert np.abs(got - want).max() <= 1e-9 * 1e16
    assert np.abs(want - n).max() > 5e14          # the decay is resolved


def test_ion_uniform_source():
    """E = 0 and a uniform n and source: n^{n+1} = n + dt S exactly (the walls
    impose zero flux, which a uniform state satisfies)."""
    ops = _ops(17)
    mu, D = H.ion_coefficients(ops)
    n = np.full(ops.nx, 3e15)
    Sx = np.full(ops.nx, 2e20)
    got = H.ion_solve(ops, H.ion_matrix(ops, np.zeros(ops.nx), mu, D), H.ion_rhs(ops, n, Sx))
    assert np.abs(got - (n + ops.dt * Sx)).max() <= 1e-12 * n.max()


def test_ion_source_and_field_readings():
    """The source is n0 k_i n_e with k_i, n_e the moments of F; E^n is the
    Poisson field of the step's electron solve evaluated at t_n instead of t_n + dt/2."""
    ops = _ops(12)
    F = S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 2.0)
    mom = S.moments(ops, F)
    assert np.allclose(H.ion_source(ops, F), ops.n0 * mom[2] * mom[0], rtol=1e-13, atol=0)
    ni = 1.1 * mom[0]
    t = 0.37 * workloads.rf_period_s()
    assert np.allclose(H.field_at(ops, t, F, ni), S.field_half(ops, t - 0.5 * ops.dt, F, ni=ni),
                       rtol=1e-13, atol=1e-9)


def test_hybrid_step_is_ion_update_then_electron_step():
    ops = _ops(10)
    F = S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 2.0)
    ni = S.moments(ops, F)[0].copy()
    t = 0.1 * workloads.rf_period_s()
    F1, ni1 = H.hybrid_step(ops, F, ni, t)
    assert np.array_equal(ni1, H.ion_step(ops, ni, F, t))
    assert np.array_equal(F1, S.step(ops, F, t, ni=ni1))
    assert np.all(np.isfinite(ni1)) and ni1.min() > 0
