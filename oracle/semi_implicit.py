"""The semi-implicit step, moments and the adjoint step (test infrastructure only).

State layout: F[x, k, a] -- spatial point x (ascending CGL nodes), B-spline k,
ordinate a (ascending cos theta_a); f(x_i, v, theta_a) = sum_k F[i, k, a] phi_k(v).
This is the paper's EDF matrix of eq. (bte_1d_discrete) stored transposed
(x-major), with the (k, a) row index ordered v outer, theta inner.

Semi-implicit scheme (eq. bte_semi_implicit, Strang order):
    X(dt/2)  -- eq. bte_semi_implicit_xspace0 via Alg. bte_spatial_adv
    E^{1/2}  -- eq. bte_semi_implicit_efield (or a specified field at t + dt/2)
    V(dt)    -- eq. vspace_batched_system, one dense system per spatial point
    X(dt/2)  -- eq. bte_semi_implicit_xspace1

The oracle solves every linear system directly (LU with partial pivoting) and
never forms an explicit inverse.  Zero-inflow walls (eq. hybrid_cnt_b_bdy)
enter the X systems mode by mode: for cos theta_a > 0 the equation at
xhat = -1 is replaced by "value = 0", for cos theta_a < 0 the one at xhat = +1
(valid because the eigenvector change of basis acts on speed only).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.special as ssp

from .basis import bspline_basis, composite_gauss
from .operators import E_CHARGE, EPS0, M_ELECTRON, N_GAUSS, Operators


# --- spatial advection -------------------------------------------------------------------
def _x_system(ops: Operators, i: int, a: int, dt_half: float):
    """B_ia = I + dt_half * lam_i * cos(theta_a) * D_x with the inflow row replaced.

    Returns (B, inflow index or None)."""
    nx = ops.nx
    B = np.eye(nx) + dt_half * ops.lam[i] * ops.mu[a] * ops.Dx
    if ops.mu[a] > 0:
        b = 0
    elif ops.mu[a] < 0:
        b = nx - 1
    else:
        return np.eye(nx), None
    B[b, :] = 0.0
    B[b, b] = 1.0
    return B, b


def x_half_step(ops: Operators, F: np.ndarray, dt_half: float | None = None) -> np.ndarray:
    """Alg. bte_spatial_adv: contract with U^-1 over speed, solve every (eigen-speed,
    ordinate) Chebyshev system, contract back with U."""
    if dt_half is None:
        dt_half = 0.5 * ops.dt
    Y = np.einsum("ik,xka->xia", ops.Uinv, F)
    for i in range(ops.nr):
        for a in range(ops.nth):
            B, b = _x_system(ops, i, a, dt_half)
            rhs = Y[:, i, a].copy()
            if b is not None:
                rhs[b] = 0.0
            Y[:, i, a] = sla.lu_solve(sla.lu_factor(B), rhs)
    return np.einsum("ki,xia->xka", ops.U, Y)


def x_half_step_T(ops: Operators, lam: np.ndarray, dt_half: float | None = None) -> np.ndarray:
    """Transpose of ``x_half_step`` (same linear map, transposed factor by factor)."""
    if dt_half is None:
        dt_half = 0.5 * ops.dt
    Z = np.einsum("ki,xka->xia", ops.U, lam)
    for i in range(ops.nr):
        for a in range(ops.nth):
            B, b = _x_system(ops, i, a, dt_half)
            z = sla.lu_solve(sla.lu_factor(B), Z[:, i, a], trans=1)
            if b is not None:
                z[b] = 0.0
            Z[:, i, a] = z
    return np.einsum("ik,xia->xka", ops.Uinv, Z)


# --- electric field ------------------------------------------------------------------------
def field_half(ops: Operators, t: float, F_half: np.ndarray | None = None, ni=None, V_left=None,
               E0=None) -> np.ndarray:
    """Field at t + dt/2 on the x grid.

    'const': E = E0 everywhere.  'rf': E = E0 sin(2 pi f (t + dt/2)) (1 + a1 xhat).
    'poisson': eq. bte_semi_implicit_efield -- Delta V = -(e/eps0)(n_i - n_e) with
    V(0) = V_left, V(L) = 0 and E = -dV/dx, n_e taken from F^{n+1/2}.
    """
    fld = ops.cfg["field"]
    th = t + 0.5 * ops.dt
    if fld["kind"] == "poisson":
        ne = np.einsum("xj,j->x", F_half.reshape(ops.nx, -1), ops.u_ord)
        rhs = -(E_CHARGE / EPS0) * (np.asarray(ni) - ne)
        rhs[0] = V_left if V_left is not None else fld["V0"] * math.sin(2 * math.pi * fld["freq_hz"] * th)
        rhs[-1] = 0.0
        return ops.Poisson @ rhs
    E0 = fld["E0"] if E0 is None else E0
    if fld["kind"] == "const":
        return np.full(ops.nx, float(E0))
    return E0 * math.sin(2 * math.pi * fld["freq_hz"] * th) * (1.0 + fld["a1"] * ops.xhat)


def field_dE0(ops: Operators, t: float) -> np.ndarray:
    """d E^{1/2} / d E0 for the specified-field modes."""
    fld = ops.cfg["field"]
    if fld["kind"] == "const":
        return np.ones(ops.nx)
    th = t + 0.5 * ops.dt
    return math.sin(2 * math.pi * fld["freq_hz"] * th) * (1.0 + fld["a1"] * ops.xhat)


# --- velocity space ------------------------------------------------------------------------
def v_matrix(ops: Operators, Ex: float, n0: float | None = None) -> np.ndarray:
    """I - dt P_O (n0 C_en + E_x A_v) P_S (eq. vspace_batched_system)."""
    n0 = ops.n0 if n0 is None else n0
    n = ops.nr * ops.nth
    return np.eye(n) - ops.dt * (n0 * ops.Cord + Ex * ops.Aord)


def v_step(ops: Operators, F: np.ndarray, E: np.ndarray, xs=None) -> np.ndarray:
    """Solve the decoupled velocity-space systems at every spatial point (or at ``xs``)."""
    out = F.copy()
    for x in (range(ops.nx) if xs is None else xs):
        A = v_matrix(ops, E[x])
        out[x] = sla.lu_solve(sla.lu_factor(A), F[x].ravel()).reshape(ops.nr, ops.nth)
    return out


def step(ops: Operators, F: np.ndarray, t: float, ni=None, V_left=None) -> np.ndarray:
    """One semi-implicit step F^n -> F^{n+1} (eq. bte_semi_implicit)."""
    Fh = x_half_step(ops, F)
    E = field_half(ops, t, Fh, ni=ni, V_left=V_left)
    Fs = v_step(ops, Fh, E)
    return x_half_step(ops, Fs)


# --- moments --------------------------------------------------------------------------------
def moments(ops: Operators, F: np.ndarray) -> np.ndarray:
    """[3, nx]: n_e [m^-3] (u^T F, eq. hybrid_discrete_c), mean energy [eV] and the
    ionization rate coefficient k_i [m^3/s] (hybrid model, k_i = int |v| sigma_i f / n_e)."""
    Fm = F.reshape(ops.nx, -1)
    ne = Fm @ ops.u_ord
    en = Fm @ ops.e_ord
    ki = Fm @ ops.ki_ord
    safe = np.where(ne != 0.0, ne, 1.0)
    return np.stack([ne, np.where(ne != 0.0, en / safe, 0.0), np.where(ne != 0.0, ki / safe, 0.0)])


def maxwellian_coeffs(ops: Operators, Te_eV: float) -> np.ndarray:
    """Galerkin (v^2-weighted) projection of the unit-density Maxwellian at Te onto the
    B-splines: M c = b, b_p = int v^2 phi_p f_M dv,
    f_M = exp(-v^2/vth^2) / (pi^{3/2} vth^3), vth = sqrt(2 e Te / m_e)."""
    vth = math.sqrt(2.0 * E_CHARGE * Te_eV / M_ELECTRON)
    x, w = composite_gauss(ops.knots, 2 * N_GAUSS)
    P = bspline_basis(ops.knots, x, ops.nr)
    fM = np.exp(-(x / vth) ** 2) / (math.pi ** 1.5 * vth ** 3)
    b = P.T @ (w * x ** 2 * fM)
    return np.linalg.solve(ops.M, b)


def initial_state(ops: Operators, ne_x: np.ndarray, Te_eV: float) -> np.ndarray:
    """Isotropic Maxwellian times the density profile (same value on every ordinate)."""
    c = maxwellian_coeffs(ops, Te_eV)
    return np.asarray(ne_x)[:, None, None] * c[None, :, None] * np.ones((1, 1, ops.nth))


def truncated_maxwellian_moments(Te_eV: float, vmax: float):
    """Closed forms of the Maxwellian truncated at vmax: (number fraction, mean energy eV)."""
    vth = math.sqrt(2.0 * E_CHARGE * Te_eV / M_ELECTRON)
    z2 = (vmax / vth) ** 2
    frac = ssp.gammainc(1.5, z2)
    mean = 1.5 * Te_eV * ssp.gammainc(2.5, z2) / ssp.gammainc(1.5, z2)
    return frac, mean


# --- adjoint ------------------------------------------------------------------------------
def adjoint_step(ops: Operators, F_n: np.ndarray, t: float, lam_next: np.ndarray):
    """Transpose of one step with a specified field, and the parameter gradients.

    With F* = A^-1 X F^n and mu = A^-T X^T lam (block-wise over x):
      lam^n            = X^T mu
      dL/dscal[s,b]   += dt n0 sum_x mu_x^T C^(s,b)_ord F*_x
      dL/dE^{1/2}_x    = dt mu_x^T A_ord F*_x
    Returns (lam_n, grad_scal [n_proc * n_bins], grad_E [nx]).
    """
    Y = x_half_step(ops, F_n)
    E = field_half(ops, t, Y)
    Z = x_half_step_T(ops, lam_next)
    n = ops.nr * ops.nth
    Fs = np.zeros_like(Y)
    Mu = np.zeros_like(Z)
    for x in range(ops.nx):
        lu = sla.lu_factor(v_matrix(ops, E[x]))
        Fs[x] = sla.lu_solve(lu, Y[x].ravel()).reshape(ops.nr, ops.nth)
        Mu[x] = sla.lu_solve(lu, Z[x].ravel(), trans=1).reshape(ops.nr, ops.nth)
    Fm = Fs.reshape(ops.nx, n)
    Mm = Mu.reshape(ops.nx, n)
    grad_scal = np.array([ops.dt * ops.n0 * np.einsum("xi,ij,xj->", Mm, C, Fm) for C in ops.Cord_sb])
    grad_E = ops.dt * np.einsum("xi,ij,xj->x", Mm, ops.Aord, Fm)
    return x_half_step_T(ops, Mu), grad_scal, grad_E


def run(ops: Operators, F0: np.ndarray, n_steps: int, t0: float = 0.0, every: int = 0, callback=None):
    """Advance n_steps; optionally call callback(n, F) every ``every`` steps."""
    F = F0.copy()
    for n in range(n_steps):
        F = step(ops, F, t0 + n * ops.dt)
        if callback is not None and every and (n + 1) % every == 0:
            callback(n + 1, F)
    return F


def cycle_mean_density(ops: Operators, F0: np.ndarray, n_steps: int, t0: float = 0.0) -> np.ndarray:
    """Mean over the step-end states F^1..F^N of the density n_e = u^T F (per x)."""
    F = F0.copy()
    acc = np.zeros(ops.nx)
    for n in range(n_steps):
        F = step(ops, F, t0 + n * ops.dt)
        acc += F.reshape(ops.nx, -1) @ ops.u_ord
    return acc / n_steps


def cycle_mean_density_vjp(ops: Operators, F0: np.ndarray, n_steps: int, g: np.ndarray, t0: float = 0.0):
    """Reverse-mode derivative of ``cycle_mean_density`` for a cotangent g [nx].

    All states are kept (no checkpointing): lam^N = (1/N) u g, and for n = N-1..0
    lam^n = S_n^T lam^{n+1} (+ (1/N) u g for n >= 1), with the parameter
    gradients of every transposed step summed.  The field derivative is chained
    to the amplitude E0 of the specified field.
    Returns (grad_scal [n_proc * n_bins], dL/dE0, dL/dF^0).
    """
    states = [F0.copy()]
    for n in range(n_steps):
        states.append(step(ops, states[-1], t0 + n * ops.dt))
    direct = np.outer(g / n_steps, ops.u_ord).reshape(F0.shape)
    lam = np.zeros_like(F0)
    grad_scal = np.zeros(len(ops.Cord_sb))
    grad_E0 = 0.0
    for n in range(n_steps, 0, -1):
        lam = lam + direct
        t = t0 + (n - 1) * ops.dt
        lam, gs, gE = adjoint_step(ops, states[n - 1], t, lam)
        grad_scal += gs
        grad_E0 += float(gE @ field_dE0(ops, t))
    return grad_scal, grad_E0, lam
