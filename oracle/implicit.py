"""The fully implicit electron step (test infrastructure only).

eq. bte_fully_implicit: F^{n+1} solves

    (F^{n+1} - F^n)/dt = -A_x F^{n+1} D_x^T + P_O C_en P_S F^{n+1} + P_O A_v P_S (E(F^{n+1}) . F^{n+1}),
    E(F) = L (n_i - u^T F),

with A_x = (M_v^-1 G_v) (x) diag(cos theta) acting on speed and angle and D_x on
x; in the state layout F[x, k, a] the term A_x F D_x^T is
sum_j (M^-1 G)[k, j] cos(theta_a) (D_x F[:, j, a])[x].  P_O C_en P_S and
P_O A_v P_S are the ordinate operators C_ord (times n0) and A_ord.

Readings (restated in the design notes):
* Walls: the zero-inflow condition of eq. hybrid_cnt_b_bdy replaces the
  equation at the inflow entries (x = 0 for cos theta > 0, x = L for
  cos theta < 0): F = 0 there, as in the X step of the semi-implicit scheme.
* Field: E(F) takes the electrode voltage at t_{n+1} (the time the implicit
  equation is written at); with a specified field (const / RF) E is that field
  at t_{n+1} and the equation is linear.
* Solver: Newton's method on the residual R(F) (full steps; the Jacobian is the
  linearization of eq. 1dbte_jac_action, assembled densely column by column and
  factored by LU), from F^n, until ||R||_inf <= 1e-13 max(||F^n||_inf, 1).
"""
from __future__ import annotations

import math

import numpy as np

from .operators import E_CHARGE, EPS0, Operators


def inflow_mask(ops: Operators) -> np.ndarray:
    """Boolean [nx, nr, nth]: the entries whose equation is the wall condition."""
    m = np.zeros((ops.nx, ops.nr, ops.nth), dtype=bool)
    pos = ops.mu > 0
    m[0, :, pos] = True
    m[-1, :, ~pos] = True
    return m


def x_operator(ops: Operators, F: np.ndarray) -> np.ndarray:
    """A_x F D_x^T (eq. A_x): speed-angle factor M^-1 G (x) diag(cos theta), x derivative."""
    MinvG = np.linalg.solve(ops.M, ops.G)
    dF = np.einsum("xy,yka->xka", ops.Dx, F)
    return np.einsum("kj,xja,a->xka", MinvG, dF, ops.mu)


def field(ops: Operators, F: np.ndarray, t: float, ni=None, linear: bool = False) -> np.ndarray:
    """E(F) at t.  linear=True: the derivative of the affine map F -> E(F) (no ions,
    no electrode voltage), used by the Jacobian; for specified fields it is 0."""
    fld = ops.cfg["field"]
    if fld["kind"] != "poisson":
        if linear:
            return np.zeros(ops.nx)
        E0 = fld["E0"]
        if fld["kind"] == "const":
            return np.full(ops.nx, float(E0))
        return E0 * math.sin(2 * math.pi * fld["freq_hz"] * t) * (1.0 + fld["a1"] * ops.xhat)
    ne = F.reshape(ops.nx, -1) @ ops.u_ord
    ion = 0.0 if linear else np.asarray(ni, dtype=np.float64)
    rhs = -(E_CHARGE / EPS0) * (ion - ne)
    rhs[0] = 0.0 if linear else fld["V0"] * math.sin(2 * math.pi * fld["freq_hz"] * t)
    rhs[-1] = 0.0
    return ops.Poisson @ rhs


def v_operator(ops: Operators, F: np.ndarray, E: np.ndarray, n0: float | None = None) -> np.ndarray:
    """P_O (n0 C_en + E_x A_v) P_S F at every point."""
    n0 = ops.n0 if n0 is None else n0
    Fm = F.reshape(ops.nx, -1)
    out = n0 * Fm @ ops.Cord.T + E[:, None] * (Fm @ ops.Aord.T)
    return out.reshape(F.shape)


def residual(ops: Operators, F: np.ndarray, Fn: np.ndarray, t1: float, ni=None) -> np.ndarray:
    """R(F) = F - F^n + dt A_x F D_x^T - dt P_O (C_en + E(F) A_v) P_S F; R = F at the inflow entries."""
    E = field(ops, F, t1, ni)
    R = F - Fn + ops.dt * x_operator(ops, F) - ops.dt * v_operator(ops, F, E)
    m = inflow_mask(ops)
    R[m] = F[m]
    return R


def jacobian_action(ops: Operators, F: np.ndarray, X: np.ndarray, t1: float, ni=None) -> np.ndarray:
    """J_F X: eq. 1dbte_jac_action in residual form,
    X + dt A_x X D_x^T - dt [C X + A (E(F) . X) + A (E_lin(X) . F)]; X at the inflow entries."""
    E = field(ops, F, t1, ni)
    El = field(ops, X, t1, linear=True)
    J = (X + ops.dt * x_operator(ops, X) - ops.dt * v_operator(ops, X, E)
         - ops.dt * v_operator(ops, F, El, n0=0.0))
    m = inflow_mask(ops)
    J[m] = X[m]
    return J


def jacobian(ops: Operators, F: np.ndarray, t1: float, ni=None) -> np.ndarray:
    """Dense J_F, one column per unit vector."""
    N = F.size
    J = np.zeros((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        J[:, c] = jacobian_action(ops, F, e.reshape(F.shape), t1, ni).ravel()
    return J


def implicit_step(ops: Operators, Fn: np.ndarray, t: float, ni=None, max_newton: int = 30):
    """F^{n+1} of eq. bte_fully_implicit by Newton's method; returns (F, iterations)."""
    t1 = t + ops.dt
    F = Fn.copy()
    tol = 1e-13 * max(np.abs(Fn).max(), 1.0)
    for it in range(max_newton):
        R = residual(ops, F, Fn, t1, ni)
        if np.abs(R).max() <= tol:
            return F, it
        J = jacobian(ops, F, t1, ni)
        F = F - np.linalg.solve(J, R.ravel()).reshape(F.shape)
    R = residual(ops, F, Fn, t1, ni)
    if np.abs(R).max() > tol:
        raise RuntimeError(f"Newton did not converge: |R| = {np.abs(R).max():.3e}")
    return F, max_newton
