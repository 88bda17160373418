"""The hybrid RF glow-discharge step: ion fluid update, then the semi-implicit
electron step (test infrastructure only).

Operator split of the hybrid model (eq. glow_hybrid), "Hybrid solver time
integration": for a state (n_i^n, F^n) at t_n,

  heavies   (n_i^{n+1} - n_i^n)/dt + D_x J_i(E^n, n_i^{n+1}) = (k_i^T F^n) n0 (u^T F^n)
            (eq. fluid_step), with the drift-diffusion flux J_i = mu_i n_i E - D_i D_x n_i
            (eq. hybrid_cnt_a_flux) and E^n = L (n_i^n - u^T F^n) (the Poisson operator of
            eq. hybrid_cnt_c with the voltage of eq. voltage_bc at t_n), E frozen;
  electrons the semi-implicit step (eq. bte_semi_implicit) with the field
            E^{1/2} = L (n_i^{n+1} - u^T F^{n+1/2}).

The ion coefficients are the constant ones of the table of modeling parameters:
n0 mu_i = 4.65e21 /(V m s), n0 D_i = 2.07e20 /(m s).

Readings (restated in the design notes):
* Source: k_i^T F^n is the ionization rate coefficient of the normalized EDF, so
  (k_i^T F^n) n0 (u^T F^n) = n0 times the unnormalized ionization integral of F^n.
* Walls (eq. fl_ion_bc): with the outward normal, ions leave by drift and none
  enter, J_i . n = n_i max(0, mu_i E . n).  The printed sign is read as an
  inward-normal convention (with the outward normal it would make ions enter
  the gap where the field pushes them out).  The condition replaces the ion
  equation at the two wall nodes (collocation), with E frozen at E^n.
"""
from __future__ import annotations

import math

import numpy as np

from .operators import E_CHARGE, EPS0, Operators
from .semi_implicit import step

ION_N0_MU = 4.65e21   # n0 mu_i [1/(V m s)]
ION_N0_D = 2.07e20    # n0 D_i [1/(m s)]


def ion_coefficients(ops: Operators, n0: float | None = None) -> tuple[float, float]:
    """(mu_i, D_i) at the gas density n0 (table of modeling parameters)."""
    n0 = ops.n0 if n0 is None else n0
    return ION_N0_MU / n0, ION_N0_D / n0


def field_at(ops: Operators, t: float, F: np.ndarray, ni: np.ndarray) -> np.ndarray:
    """E^n = L (n_i - u^T F) with V(0) = V0 sin(2 pi f t), V(L) = 0 (eq. hybrid_cnt_c,
    eq. voltage_bc), at the start of the step (the heavies' update uses E^n)."""
    fld = ops.cfg["field"]
    ne = F.reshape(ops.nx, -1) @ ops.u_ord
    rhs = -(E_CHARGE / EPS0) * (np.asarray(ni, dtype=np.float64) - ne)
    rhs[0] = fld["V0"] * math.sin(2 * math.pi * fld["freq_hz"] * t)
    rhs[-1] = 0.0
    return ops.Poisson @ rhs


def ion_source(ops: Operators, F: np.ndarray) -> np.ndarray:
    """(k_i^T F) n0 (u^T F) at every point: n0 times the ionization integral of F."""
    return ops.n0 * (F.reshape(ops.nx, -1) @ ops.ki_ord)


def ion_matrix(ops: Operators, E: np.ndarray, mu: float, D: float) -> np.ndarray:
    """Collocation matrix of eq. fluid_step for n_i^{n+1}: I/dt + D_x diag(mu E) - D D_x D_x
    in the interior; at the wall nodes the outflow condition (module docstring)
    written as a linear condition on n_i^{n+1}."""
    nx, dt, Dx = ops.nx, ops.dt, ops.Dx
    M = np.eye(nx) / dt + Dx @ np.diag(mu * E) - D * (Dx @ Dx)
    # x = L (last node), outward normal +x:  mu E n - D n' - max(0, mu E) n = 0
    M[-1, :] = -D * Dx[-1, :]
    M[-1, -1] += mu * E[-1] - max(0.0, mu * E[-1])
    # x = 0 (first node), outward normal -x: -(mu E n - D n') - max(0, -mu E) n = 0
    M[0, :] = D * Dx[0, :]
    M[0, 0] += -mu * E[0] - max(0.0, -mu * E[0])
    return M


def ion_rhs(ops: Operators, ni: np.ndarray, S: np.ndarray) -> np.ndarray:
    b = np.asarray(ni, dtype=np.float64) / ops.dt + S
    b[0] = 0.0
    b[-1] = 0.0
    return b


def ion_solve(ops: Operators, M: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Dense LU solve of the ion system.  The two wall rows (flux conditions, of
    size D_i |D_x|) are first scaled to the size of the interior rows (1/dt): an
    equilibration that leaves the solution unchanged and keeps the wall values
    as accurate as the interior ones."""
    M = M.copy()
    b = np.array(b, dtype=np.float64)
    for r in (0, ops.nx - 1):
        s = 1.0 / (ops.dt * np.abs(M[r]).max())
        M[r] *= s
        b[r] *= s
    return np.linalg.solve(M, b)


def ion_step(ops: Operators, ni: np.ndarray, F: np.ndarray, t: float) -> np.ndarray:
    """n_i^{n+1} by eq. fluid_step (one dense LU solve)."""
    mu, D = ion_coefficients(ops)
    E = field_at(ops, t, F, ni)
    M = ion_matrix(ops, E, mu, D)
    return ion_solve(ops, M, ion_rhs(ops, ni, ion_source(ops, F)))


def hybrid_step(ops: Operators, F: np.ndarray, ni: np.ndarray, t: float):
    """(F^{n+1}, n_i^{n+1}): the heavies' update, then the electron step with n_i^{n+1}."""
    ni1 = ion_step(ops, ni, F, t)
    return step(ops, F, t, ni=ni1), ni1
