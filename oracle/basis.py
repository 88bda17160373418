"""Grids and basis functions of the oracle (test infrastructure only).

Follows the discretization of the "Hybrid fluid-BTE solver" section:
Chebyshev collocation in x, cubic B-splines on a regular grid in speed
(eq. f_expansion), real spherical harmonics with m = 0 (eq. sph_harmonics) and
discrete ordinates in the polar angle (eq. proj_ops).
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as npleg


# --- x: Chebyshev-Gauss-Lobatto collocation ------------------------------------
def cgl_nodes(nx: int) -> np.ndarray:
    """Ascending CGL nodes xhat_i = -cos(pi i / (nx-1)) on [-1, 1]."""
    i = np.arange(nx)
    return -np.cos(np.pi * i / (nx - 1))


def cheb_diff(nx: int) -> np.ndarray:
    """Collocation derivative on the CGL nodes (Lagrange interpolant derivative).

    Barycentric form: D_ij = (w_j / w_i) / (x_i - x_j) for i != j, with the
    Chebyshev-Lobatto weights w_j = (-1)^j delta_j (delta = 1/2 at both ends);
    the diagonal is the negative row sum (derivative of a constant is zero).
    """
    x = cgl_nodes(nx)
    w = np.where(np.arange(nx) % 2 == 0, 1.0, -1.0)
    w[0] *= 0.5
    w[-1] *= 0.5
    D = np.zeros((nx, nx))
    for i in range(nx):
        for j in range(nx):
            if i != j:
                D[i, j] = (w[j] / w[i]) / (x[i] - x[j])
        D[i, i] = -np.sum(D[i, :])
    return D


# --- polar angle: Gauss-Legendre ordinates and spherical harmonics --------------
def gl_nodes(n: int):
    """Gauss-Legendre nodes mu_a (ascending) and weights w_a on [-1, 1]."""
    mu, w = npleg.leggauss(n)
    return mu, w


def sph_harm_m0(l: int, mu: np.ndarray) -> np.ndarray:
    """Y_l0 = sqrt((2l+1)/(4 pi)) P_l(cos theta) (eq. sph_harmonics with m = 0)."""
    c = np.zeros(l + 1)
    c[l] = 1.0
    return math.sqrt((2 * l + 1) / (4 * math.pi)) * npleg.legval(mu, c)


def sph_harm_m0_deriv(l: int, mu: np.ndarray) -> np.ndarray:
    """d Y_l0 / d mu."""
    c = np.zeros(l + 1)
    c[l] = 1.0
    return math.sqrt((2 * l + 1) / (4 * math.pi)) * npleg.legval(mu, npleg.legder(c))


# --- speed: clamped cubic B-splines on a uniform grid ----------------------------
def bspline_knots(nr: int, vmax: float, v_bc: str = "natural") -> np.ndarray:
    """Clamped knot vector on a uniform grid of [0, vmax].

    ``natural``: nr cubic B-splines on nr-3 intervals, no condition at either end.
    ``zero_vmax``: nr+1 clamped splines on nr-2 intervals of which the last one (the
    only spline non-zero at vmax) is dropped, i.e. f(vmax) = 0 is imposed.
    """
    nint = nr - 3 if v_bc == "natural" else nr - 2
    inner = np.linspace(0.0, vmax, nint + 1)
    return np.concatenate([[0.0] * 3, inner, [vmax] * 3])


def _cox_de_boor(t: np.ndarray, nbasis: int, deg: int, x: np.ndarray) -> np.ndarray:
    """All B-splines of degree ``deg`` on knots ``t`` evaluated at x -> (len(x), nbasis).

    Plain Cox-de Boor recursion.  Half-open intervals [t_j, t_j+1), except that
    the right end of the domain belongs to the last non-empty interval.
    """
    x = np.asarray(x, dtype=np.float64)
    nk = len(t)
    B = np.zeros((x.size, nk - 1))
    last = np.max(np.nonzero(t[1:] > t[:-1])[0])
    for j in range(nk - 1):
        if t[j + 1] > t[j]:
            inside = (x >= t[j]) & (x < t[j + 1])
            if j == last:
                inside |= x == t[j + 1]
            B[:, j] = inside
    for d in range(1, deg + 1):
        Bn = np.zeros((x.size, nk - 1 - d))
        for j in range(nk - 1 - d):
            a = t[j + d] - t[j]
            b = t[j + d + 1] - t[j + 1]
            term = np.zeros(x.size)
            if a > 0:
                term += (x - t[j]) / a * B[:, j]
            if b > 0:
                term += (t[j + d + 1] - x) / b * B[:, j + 1]
            Bn[:, j] = term
        B = Bn
    return B[:, :nbasis]


def bspline_basis(knots: np.ndarray, v: np.ndarray, nr: int | None = None) -> np.ndarray:
    """phi_k(v) for the first nr splines on ``knots``: array (len(v), nr).  Zero outside [0, vmax]."""
    nr = len(knots) - 4 if nr is None else nr
    return _cox_de_boor(knots, len(knots) - 4, 3, v)[:, :nr]


def bspline_basis_deriv(knots: np.ndarray, v: np.ndarray, nr: int | None = None) -> np.ndarray:
    """d phi_k / dv from the standard derivative formula of B-splines:
    B'_{j,3} = 3 [B_{j,2} / (t_{j+3}-t_j) - B_{j+1,2} / (t_{j+4}-t_{j+1})]."""
    nr = len(knots) - 4 if nr is None else nr
    B2 = _cox_de_boor(knots, len(knots) - 3, 2, v)
    out = np.zeros((np.size(v), nr))
    for j in range(nr):
        a = knots[j + 3] - knots[j]
        b = knots[j + 4] - knots[j + 1]
        if a > 0:
            out[:, j] += 3.0 * B2[:, j] / a
        if b > 0 and j + 1 < B2.shape[1]:
            out[:, j] -= 3.0 * B2[:, j + 1] / b
    return out


# --- composite Gauss-Legendre quadrature -------------------------------------------
def composite_gauss(breaks: np.ndarray, npts: int):
    """Nodes/weights of npts-point Gauss-Legendre rules on every [breaks_i, breaks_i+1]."""
    g, w = npleg.leggauss(npts)
    br = np.unique(np.asarray(breaks, dtype=np.float64))
    a, b = br[:-1], br[1:]
    keep = b > a
    a, b = a[keep], b[keep]
    half = 0.5 * (b - a)
    mid = 0.5 * (b + a)
    x = (mid[:, None] + half[:, None] * g[None, :]).ravel()
    wx = (half[:, None] * w[None, :]).ravel()
    return x, wx
