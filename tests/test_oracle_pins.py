"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test pins one part of the oracle to something other than itself: closed
forms, exact invariants, library routines for textbook special cases, brute
force on tiny inputs and the values the paper prints.  They run on the CPU.
"""
import math

import numpy as np
import pytest
import scipy.integrate as sint
import scipy.interpolate as sinterp
import scipy.linalg as sla

import oracle
import workloads
from oracle import basis as B
from oracle import operators as O
from oracle import semi_implicit as S


def small(nx=6, nr=8, nth=4, kinds=("elastic",), E=2e3, v_bc="natural", **kw):
    cfg = workloads.small_config(nx=nx, nr=nr, nth=nth, kinds=kinds, E=E, **kw)
    cfg["v_bc"] = v_bc
    return cfg


# --- P1: Chebyshev collocation derivative is exact on polynomials of degree < Nx ------------
@pytest.mark.parametrize("nx", [4, 9, 16, 33])
def test_cheb_diff_exact_on_polynomials(nx):
    x = B.cgl_nodes(nx)
    D = B.cheb_diff(nx)
    assert np.all(np.diff(x) > 0) and x[0] == -1.0 and abs(x[-1] - 1.0) < 1e-15
    for k in range(nx):
        err = np.abs(D @ x ** k - (k * x ** (k - 1) if k > 0 else 0 * x)).max()
        assert err <= 1e-12 * nx ** 2 * max(1, k), (k, err)


# --- P2: Gauss-Legendre ordinates integrate Legendre polynomials exactly ----------------------
@pytest.mark.parametrize("n", [2, 4, 8, 32])
def test_gauss_legendre_and_projections(n):
    mu, w = B.gl_nodes(n)
    for l in range(2 * n):
        c = np.zeros(l + 1)
        c[l] = 1.0
        val = np.sum(w * np.polynomial.legendre.legval(mu, c))
        assert abs(val - (2.0 if l == 0 else 0.0)) < 1e-13, (l, val)
    _, _, T_O, T_S, a, b = O.angular_parts(n, n)
    assert np.abs(T_S @ T_O - np.eye(n)).max() < 1e-13
    assert np.abs(T_O @ T_S - np.eye(n)).max() < 1e-12


def test_angular_couplings_closed_form():
    """<Y_q|mu|Y_l> and <Y_q|(1-mu^2)d/dmu|Y_l> against the Legendre recurrences."""
    n = 12
    _, _, _, _, a, b = O.angular_parts(n, n)
    A_ref = np.zeros((n, n))
    B_ref = np.zeros((n, n))
    for l in range(n):
        if l >= 1:
            A_ref[l - 1, l] = l / math.sqrt(4 * l * l - 1)
            B_ref[l - 1, l] = l * (l + 1) / math.sqrt(4 * l * l - 1)
        if l + 1 < n:
            A_ref[l + 1, l] = (l + 1) / math.sqrt((2 * l + 1) * (2 * l + 3))
            B_ref[l + 1, l] = -l * (l + 1) / math.sqrt((2 * l + 1) * (2 * l + 3))
    assert np.abs(a - A_ref).max() < 1e-13
    assert np.abs(b - B_ref).max() < 1e-12
    # collocation identity: T_O a T_S = diag(mu) (P_N vanishes at the nodes)
    mu, _, T_O, T_S, _, _ = O.angular_parts(n, n)
    assert np.abs(T_O @ a @ T_S - np.diag(mu)).max() < 1e-13


# --- P3: B-splines ------------------------------------------------------------------------------
@pytest.mark.parametrize("v_bc", ["natural", "zero_vmax"])
def test_bspline_against_library_and_exact_integrals(v_bc):
    nr, vmax = 10, 3.0
    t = B.bspline_knots(nr, vmax, v_bc)
    v = np.linspace(0, vmax, 301)
    P = B.bspline_basis(t, v, nr)
    dP = B.bspline_basis_deriv(t, v, nr)
    for k in range(nr):
        c = np.zeros(len(t) - 4)
        c[k] = 1.0
        spl = sinterp.BSpline(t, c, 3, extrapolate=False)
        ref = np.nan_to_num(spl(v))
        dref = np.nan_to_num(spl.derivative()(v))
        assert np.abs(P[:, k] - ref).max() < 1e-14
        assert np.abs(dP[:-1, k] - dref[:-1]).max() < 1e-12
    if v_bc == "natural":
        assert np.abs(P.sum(1) - 1.0).max() < 1e-14        # partition of unity
    else:
        assert np.abs(P[-1]).max() == 0.0                    # f(vmax) = 0 imposed
    # exact integrals: for polynomials g = v^i, h = v^j (i, j <= 3, natural basis reproduces them)
    if v_bc == "natural":
        M = O.mass_like(t, nr, 2)
        G = O.mass_like(t, nr, 3)
        vs = np.linspace(0, vmax, 57)
        Ps = B.bspline_basis(t, vs, nr)
        for i in range(4):
            for j in range(4):
                ci = np.linalg.lstsq(Ps, vs ** i, rcond=None)[0]
                cj = np.linalg.lstsq(Ps, vs ** j, rcond=None)[0]
                for Mx, pw in ((M, 2), (G, 3)):
                    exact = vmax ** (i + j + pw + 1) / (i + j + pw + 1)
                    assert abs(ci @ Mx @ cj - exact) < 1e-12 * exact


@pytest.mark.parametrize("v_bc", ["natural", "zero_vmax"])
def test_advection_eigenvalues_in_range(v_bc):
    cfg = small(nr=16, v_bc=v_bc)
    ops = oracle.build_operators(cfg)
    assert ops.lam.min() > 0 and ops.lam.max() <= ops.vmax * (1 + 1e-14)
    assert np.abs(ops.U.T @ ops.M @ ops.U - np.eye(16)).max() < 1e-10
    assert np.abs(ops.Uinv @ ops.U - np.eye(16)).max() < 1e-10


# --- P4 / P5: particle conservation of elastic and excitation, ionization growth -----------------
def test_elastic_and_temperature_term_conserve_number():
    cfg = small(nr=16, nth=4, kinds=("elastic",))
    ops = oracle.build_operators(cfg)
    C = ops.Cord
    rel = np.abs(ops.u_ord @ C) / (np.abs(ops.u_ord) @ np.abs(C))
    assert rel.max() < 1e-12
    # C_T alone (differences of the operator with and without gas temperature)
    cfg0 = dict(cfg)
    cfg0["T0_K"] = 0.0
    C0 = oracle.build_operators(cfg0).Cord
    CT = C - C0
    assert np.abs(CT).max() > 0
    rel = np.abs(ops.u_ord @ CT) / (np.abs(ops.u_ord) @ np.abs(CT))
    assert rel.max() < 1e-10


def test_ionization_growth_and_excitation_conservation():
    cfg = small(nr=16, nth=4, kinds=("elastic", "excitation", "ionization"))
    ops = oracle.build_operators(cfg)
    el, ex, io = ops.Cord_sb
    scale = np.abs(ops.u_ord) @ np.abs(io)
    assert (np.abs(ops.u_ord @ ex) / (np.abs(ops.u_ord) @ np.abs(ex) + 1e-300)).max() < 1e-12
    # every ionization adds one electron: u^T C_ion = k_i^T (pins the gain multiplicity 2
    # and the v^3 weight of the collision integrals against the rate definition)
    assert (np.abs(ops.u_ord @ io - ops.ki_ord) / (scale + 1e-300)).max() < 1e-12


def test_inelastic_gain_quadrature_against_adaptive():
    """Gain entries (integrated in the post-collision speed) against scipy.integrate.quad in v."""
    cfg = small(nr=12, nth=2, kinds=("ionization",))
    ops = oracle.build_operators(cfg)
    proc = cfg["processes"][0]
    knots = ops.knots
    edges = O.speed_of(cfg["bin_edges_eV"])
    _, Gain, _ = O.collision_parts(knots, 12, proc, edges, cfg["T0_K"])[0]
    vI = float(O.speed_of(proc["threshold_eV"]))

    def u_of(v):
        return math.sqrt(max(v * v - vI * vI, 0.0) / 2.0)

    for p, k in [(0, 9), (1, 10), (2, 11), (0, 11)]:
        def f(v):
            return (v ** 3 * O.sigma_of_speed(proc, v) * B.bspline_basis(knots, np.array([v]), 12)[0, k]
                    * B.bspline_basis(knots, np.array([u_of(v)]), 12)[0, p])
        cand = list(knots) + [math.sqrt(2 * q * q + vI * vI) for q in knots]
        cand += list(O.speed_of(proc["eps_eV"]))
        pts = sorted(set(float(q) for q in cand if vI < q < ops.vmax))
        # split the integral at every breakpoint; each piece is smooth except for the
        # square-root behaviour of u(v) at the threshold, which QAGS extrapolates away
        edges = [vI] + pts + [ops.vmax]
        ref = sum(sint.quad(f, a, b, limit=200, epsabs=0, epsrel=1e-13)[0] for a, b in zip(edges[:-1], edges[1:]))
        assert abs(Gain[p, k] - ref) <= 1e-9 * abs(ref) + 1e-300, (p, k, Gain[p, k], ref)


# --- P6: relaxation to the gas Maxwellian ------------------------------------------------------
def test_relaxation_to_gas_maxwellian():
    """With E = 0 and elastic collisions, the null state is the Maxwellian at T0 and its
    mean energy is 3/2 k_B T0 (pins the sign and size of the gas-temperature term)."""
    errs = []
    kT_eV = O.K_BOLTZMANN * 300.0 / O.E_CHARGE
    for nr in (8, 16, 32):
        cfg = small(nr=nr, nth=2, kinds=("elastic",), v_bc="natural")
        cfg["eps_max_eV"] = 25 * kT_eV
        ops = oracle.build_operators(cfg)
        n = nr * 2
        K = ops.n0 * ops.Cord
        w, V = np.linalg.eig(K)
        f = np.real(V[:, np.argmin(np.abs(w))])
        f /= f @ ops.u_ord
        ref = S.initial_state(ops, np.array([1.0]), kT_eV).ravel()
        ref /= ref @ ops.u_ord
        errs.append(np.abs(f - ref).max() / np.abs(ref).max())
        mean = (f @ ops.e_ord) / (f @ ops.u_ord)
        if nr >= 16:
            assert abs(mean - 1.5 * kT_eV) < 1e-4 * kT_eV, (nr, mean, 1.5 * kT_eV)
    # converges with Nr down to the O(m_e/m0) difference between the discrete energy-shift
    # collision model and its Fokker-Planck limit
    assert errs[0] > 10 * errs[1] > 100 * errs[2] and errs[2] < 1e-4, errs


# --- P7: acceleration identities (number, momentum, Joule heating) -----------------------------
def test_acceleration_identities():
    nr, nth = 16, 6
    cfg = small(nr=nr, nth=nth, v_bc="natural")
    ops = oracle.build_operators(cfg)
    A = ops.Aord                          # d f / dt = E * A f for unit field
    W = 2 * math.pi * ops.w
    m1 = O.moment_vector(ops.knots, nr, 3)                       # int v^3 phi_k
    mom = np.kron(m1, W * ops.mu)                                # int v cos(theta) f d^3v
    # number: u^T A f is only the flux through vmax -> zero for f vanishing near vmax
    rng = np.random.default_rng(0)
    f = rng.standard_normal((nr, nth))
    f[-4:, :] = 0.0
    f = f.ravel()
    e_over_m = O.E_CHARGE / O.M_ELECTRON
    scale = e_over_m * (np.abs(ops.u_ord) @ np.abs(f)) / ops.vmax
    assert abs(ops.u_ord @ (A @ f)) < 1e-12 * scale
    # momentum: d<v_z>/dt = -(e/m) E n_e  (force -eE on electrons)
    assert abs(mom @ (A @ f) + e_over_m * (ops.u_ord @ f)) < 1e-11 * scale * ops.vmax
    # Joule: d/dt int 1/2 m v^2 f = -e E int v_z f   (energy functional in eV: e_ord)
    lhs = (ops.e_ord @ (A @ f)) * O.E_CHARGE
    rhs = -O.E_CHARGE * (mom @ f)
    assert abs(lhs - rhs) < 1e-11 * abs(rhs) + 1e-300


def test_acceleration_against_bruteforce_quadrature():
    """A (harmonic, before mass scaling) against a 2D quadrature of the weak form in (v, mu)."""
    nr, nl = 7, 4
    cfg = small(nr=nr, nth=nl, v_bc="natural")
    ops = oracle.build_operators(cfg)
    t = ops.knots
    xv, wv = B.composite_gauss(t, 10)
    mu, wm = np.polynomial.legendre.leggauss(20)
    P = B.bspline_basis(t, xv, nr)
    dP = B.bspline_basis_deriv(t, xv, nr)
    Y = np.stack([B.sph_harm_m0(l, mu) for l in range(nl)], 1)
    dY = np.stack([B.sph_harm_m0_deriv(l, mu) for l in range(nl)], 1)
    Aref = np.zeros((nr * nl, nr * nl))
    for p in range(nr):
        for q in range(nl):
            for k in range(nr):
                for l in range(nl):
                    # integrand of phi_p Y_q (mu d_v + (1-mu^2)/v d_mu)(phi_k Y_l) v^2
                    g = (np.outer(P[:, p] * dP[:, k] * xv ** 2, Y[:, q] * mu * Y[:, l])
                         + np.outer(P[:, p] * P[:, k] * xv, Y[:, q] * (1 - mu ** 2) * dY[:, l]))
                    Aref[p * nl + q, k * nl + l] = 2 * math.pi * wv @ g @ wm
    Aref *= O.E_CHARGE / O.M_ELECTRON
    Minv = np.linalg.inv(ops.M)
    Aord_ref = O.ordinate(Minv, ops.T_O, ops.T_S, Aref)
    assert np.abs(Aord_ref - ops.Aord).max() < 1e-11 * np.abs(ops.Aord).max()


# --- P9 / P10: dense brute-force step and mirror symmetry ------------------------------------
def _x_step_dense(ops):
    """X(dt/2) as one dense phase-space system, without eigen-decomposition:
    (I + dt/2 (D_x (x) M^-1 G (x) diag(mu))) with the zero-inflow rows replaced."""
    nx, nr, nth = ops.nx, ops.nr, ops.nth
    Gs = np.linalg.solve(ops.M, ops.G)
    Big = np.eye(nx * nr * nth) + 0.5 * ops.dt * np.kron(ops.Dx, np.kron(Gs, np.diag(ops.mu)))
    keep = np.ones(nx * nr * nth, dtype=bool)
    for a in range(nth):
        b = 0 if ops.mu[a] > 0 else nx - 1
        for k in range(nr):
            r = (b * nr + k) * nth + a
            Big[r, :] = 0.0
            Big[r, r] = 1.0
            keep[r] = False
    return Big, keep


def test_dense_bruteforce_step_nx4():
    cfg = small(nx=4, nr=6, nth=4, kinds=("elastic", "ionization"), E=3e3, field_kind="rf")
    ops = oracle.build_operators(cfg)
    rng = np.random.default_rng(3)
    F = rng.standard_normal((4, 6, 4))
    Big, keep = _x_step_dense(ops)
    n = 6 * 4
    t = 0.3 * ops.cfg["T_rf_s"]
    E = S.field_half(ops, t)
    Vblk = sla.block_diag(*[np.eye(n) - ops.dt * (ops.n0 * ops.Cord + E[x] * ops.Aord) for x in range(4)])
    P = np.diag(keep.astype(float))                  # zero right-hand side on inflow rows
    X = np.linalg.solve(Big, P)
    Sdense = X @ np.linalg.solve(Vblk, X)
    ref = (Sdense @ F.ravel()).reshape(F.shape)
    got = S.step(ops, F, t)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    Xh = S.x_half_step(ops, F)
    assert np.abs(Xh - (X @ F.ravel()).reshape(F.shape)).max() < 1e-12 * np.abs(Xh).max()


def test_mirror_symmetry_of_x_systems():
    cfg = small(nx=9, nr=5, nth=6)
    ops = oracle.build_operators(cfg)
    J = np.eye(9)[::-1]
    for i in range(5):
        for a in range(3):
            B1, _ = S._x_system(ops, i, a, 0.5 * ops.dt)
            B2, _ = S._x_system(ops, i, 5 - a, 0.5 * ops.dt)
            Q1 = np.linalg.inv(B1)
            Q2 = np.linalg.inv(B2)
            assert np.abs(J @ Q1 @ J - Q2).max() < 1e-11 * np.abs(Q1).max()


# --- P11: adjoint -----------------------------------------------------------------------------
def test_adjoint_dot_product_and_fd():
    cfg = small(nx=5, nr=6, nth=4, kinds=("elastic", "ionization"), E=4e3, field_kind="rf", n_bins=2)
    ops = oracle.build_operators(cfg)
    rng = np.random.default_rng(7)
    F = rng.standard_normal((5, 6, 4))
    lam = rng.standard_normal((5, 6, 4))
    t = 0.2 * cfg["T_rf_s"]
    # X^T
    d = rng.standard_normal(F.shape)
    assert abs(np.vdot(S.x_half_step(ops, d), lam) - np.vdot(d, S.x_half_step_T(ops, lam))) < 1e-12 * np.abs(lam).sum() * np.abs(d).max()
    lam_n, gs, gE = S.adjoint_step(ops, F, t, lam)
    lhs = np.vdot(S.step(ops, d, t), lam)
    rhs = np.vdot(d, lam_n)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # gradients: central differences of L = <lam, S(F)>
    h = 1e-6
    for j in range(ops.scal.size):
        sp = ops.scal.copy().ravel()
        sm = sp.copy()
        sp[j] += h
        sm[j] -= h
        opp = oracle.build_operators(cfg, scal=sp.reshape(ops.scal.shape))
        opm = oracle.build_operators(cfg, scal=sm.reshape(ops.scal.shape))
        fd = (np.vdot(lam, S.step(opp, F, t)) - np.vdot(lam, S.step(opm, F, t))) / (2 * h)
        assert abs(fd - gs[j]) < 1e-6 * (abs(fd) + 1e-3 * np.abs(gs).max()), (j, fd, gs[j])
    E0 = cfg["field"]["E0"]
    dE = S.field_dE0(ops, t)
    cp = dict(cfg)
    cm = dict(cfg)
    cp["field"] = dict(cfg["field"], E0=E0 * (1 + h))
    cm["field"] = dict(cfg["field"], E0=E0 * (1 - h))
    fd = (np.vdot(lam, S.step(oracle.build_operators(cp), F, t))
          - np.vdot(lam, S.step(oracle.build_operators(cm), F, t))) / (2 * h * E0)
    assert abs(fd - gE @ dE) < 1e-6 * abs(fd)


def test_cycle_density_gradient_against_central_differences():
    """Reverse-mode gradient of the cycle-mean density (the differentiation
    workload's loss ingredient) against central differences of the forward
    oracle: per-(process, bin) scalings, the RF amplitude and the initial state."""
    cfg = small(nx=5, nr=6, nth=4, kinds=("elastic", "excitation", "ionization"), E=6e3, field_kind="rf", n_bins=2)
    cfg["dt_s"] = 0.02 * cfg["T_rf_s"]
    ops = oracle.build_operators(cfg)
    rng = np.random.default_rng(3)
    F0 = S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 1.0)
    n_steps = 6
    g = rng.standard_normal(ops.nx)
    t0 = 0.1 * cfg["T_rf_s"]
    gs, gE0, lam0 = S.cycle_mean_density_vjp(ops, F0, n_steps, g, t0=t0)

    def loss(o, F=F0):
        return float(g @ S.cycle_mean_density(o, F, n_steps, t0=t0))

    h = 1e-6
    for j in range(ops.scal.size):
        sp = ops.scal.copy().ravel()
        sm = sp.copy()
        sp[j] += h
        sm[j] -= h
        fd = (loss(oracle.build_operators(cfg, scal=sp.reshape(ops.scal.shape)))
              - loss(oracle.build_operators(cfg, scal=sm.reshape(ops.scal.shape)))) / (2 * h)
        assert abs(fd - gs[j]) < 1e-6 * (abs(fd) + 1e-3 * np.abs(gs).max()), (j, fd, gs[j])
    E0 = cfg["field"]["E0"]
    cp = dict(cfg, field=dict(cfg["field"], E0=E0 * (1 + h)))
    cm = dict(cfg, field=dict(cfg["field"], E0=E0 * (1 - h)))
    fd = (loss(oracle.build_operators(cp)) - loss(oracle.build_operators(cm))) / (2 * h * E0)
    assert abs(fd - gE0) < 1e-6 * abs(fd), (fd, gE0)
    d = rng.standard_normal(F0.shape) * np.abs(F0).max()
    fd = (loss(ops, F0 + h * d) - loss(ops, F0 - h * d)) / (2 * h)
    assert abs(fd - np.vdot(lam0, d)) < 1e-6 * abs(fd)


# --- P12 / P13: printed constants ---------------------------------------------------------------
def test_neutral_densities_match_paper():
    printed = {0.1: 0.322e22, 0.5: 1.61e22, 1.0: 3.22e22, 2.0: 6.44e22}
    for p, n0 in printed.items():
        assert abs(workloads.n0_ideal_gas(p) - n0) / n0 < 5e-3


def test_rf_period_matches_paper():
    assert abs(workloads.rf_period_s() - 7.374e-8) / 7.374e-8 < 1e-4


# --- P14: moments of the projected initial condition ------------------------------------------
@pytest.mark.parametrize("v_bc", ["natural", "zero_vmax"])
def test_initial_condition_moments(v_bc):
    cfg = workloads.config("C0")
    cfg["v_bc"] = v_bc
    ops = oracle.build_operators(cfg)
    ne = workloads.density_profile(ops.xhat, 1e16)
    F0 = S.initial_state(ops, ne, 1.0)
    m = S.moments(ops, F0)
    frac, mean = S.truncated_maxwellian_moments(1.0, ops.vmax)
    tol = 1e-10 if v_bc == "natural" else 1e-6
    assert np.abs(m[0] - frac * ne).max() < tol * 1e16
    inner = ne > 0
    assert np.abs(m[1][inner] - mean).max() < tol * 10


# --- V-step invariants --------------------------------------------------------------------
def test_vstep_conserves_number_and_ionization_identity():
    cfg = small(nx=3, nr=10, nth=4, kinds=("elastic",), E=0.0, v_bc="natural")
    ops = oracle.build_operators(cfg)
    rng = np.random.default_rng(1)
    F = np.abs(rng.standard_normal((3, 10, 4)))
    Fs = S.v_step(ops, F, np.zeros(3))
    assert np.abs(S.moments(ops, Fs)[0] - S.moments(ops, F)[0]).max() < 1e-12 * S.moments(ops, F)[0].max()
    cfg = small(nx=3, nr=10, nth=4, kinds=("ionization",), E=0.0, v_bc="natural")
    ops = oracle.build_operators(cfg)
    Fs = S.v_step(ops, F, np.zeros(3))
    Fm = Fs.reshape(3, -1)
    lhs = Fm @ ops.u_ord - F.reshape(3, -1) @ ops.u_ord
    rhs = ops.dt * ops.n0 * (Fm @ ops.ki_ord)
    assert np.abs(lhs - rhs).max() < 1e-10 * np.abs(rhs).max()


def test_poisson_field_closed_form():
    """Uniform net charge: V'' = -(e/eps0) rho0 with V(0)=V0, V(L)=0 has the closed form
    E(x) = V0/L + (e rho0/eps0)(x - L/2)."""
    cfg = small(nx=12)
    cfg["field"] = {"kind": "poisson", "V0": 100.0, "freq_hz": workloads.RF_FREQ_HZ}
    ops = oracle.build_operators(cfg)
    F = np.zeros((12, ops.nr, ops.nth))
    ni = np.full(12, 3e15)
    E = S.field_half(ops, 0.0, F, ni=ni, V_left=100.0)
    x = 0.5 * ops.L * (ops.xhat + 1)
    ref = 100.0 / ops.L + O.E_CHARGE * 3e15 / O.EPS0 * (x - ops.L / 2)
    assert np.abs(E - ref).max() < 1e-9 * np.abs(ref).max()


def test_blocked_lu_restatement_matches_lapack():
    """The NumPy restatement of the device's blocked LU (used to localize device
    errors) solves the V systems like LAPACK, with and without interchanges, in
    both storage conventions (single panels, and panels in pairs whose second
    interchanges also reach the first panel's L rows); a random matrix makes
    interchanges in every panel, including the rows across a pair."""
    import lu_reference as LR
    cfg = workloads.small_config(nx=3, nr=20, nth=20, kinds=("elastic", "ionization"))
    ops = oracle.build_operators(cfg)
    rng = np.random.default_rng(0)
    mats = [LR.pad(S.v_matrix(ops, E)) for E in (0.0, 1.2e4, -1.4e4)]
    mats.append(rng.standard_normal((512, 512)) + 0.1 * np.eye(512))
    for M in mats:
        b = rng.standard_normal(len(M))
        want = np.linalg.solve(M, b)
        for IB in (8, 16):
            for pairs in (False, True):
                LU, ip = LR.factor(M, IB, pairs=pairs)
                x = LR.solve(LU, ip, b, pairs=pairs)
                assert np.abs(x - want).max() < 1e-10 * np.abs(want).max(), (IB, pairs)
    # the conventions differ exactly in the first panel's L rows of a pair
    M = mats[-1]
    a, ip_a = LR.factor(M, 16)
    b_, ip_b = LR.factor(M, 16, pairs=True)
    assert np.array_equal(ip_a, ip_b)
    assert not np.array_equal(a[128:, :128], b_[128:, :128])
    assert np.allclose(a[:, 128:], b_[:, 128:], rtol=0, atol=1e-12 * np.abs(a).max())


def test_static_restatement_is_an_exact_lu_of_the_velocity_systems():
    """The no-interchange restatement (test helper for the statically pivoted
    FP32 factors) on the velocity-space systems, whose pivots stay well above
    the replacement bound: L U reproduces the matrix to rounding and the pivots
    are the identity.  A matrix with an exactly zero leading pivot gets the
    bound in its place (and is then no longer an exact LU of it)."""
    import lu_reference as LR
    cfg = workloads.small_config(nx=3, nr=20, nth=20, kinds=("elastic", "ionization"))
    ops = oracle.build_operators(cfg)
    for E in (0.0, 1.2e4, -1.4e4):
        M = LR.pad(S.v_matrix(ops, E))
        LU, ip = LR.factor_static(M)
        L = np.tril(LU, -1) + np.eye(len(M))
        U = np.triu(LU)
        assert np.array_equal(ip, np.arange(len(M)))
        assert np.abs(L @ U - M).max() < 1e-12 * np.abs(M).max(), E
    Z = np.eye(256)
    Z[0, 0] = 0.0
    Z[0, 1] = Z[1, 0] = 1.0
    LU, _ = LR.factor_static(Z)
    assert LU[0, 0] == 2.0 ** -20


def test_ionization_rate_is_sensitive_to_speed_mode_rounding():
    """Why k_i agrees less closely than n_e between two FP64 evaluations of a
    step.  k_i weights only the splines above the 15.76 eV threshold, where the
    1 eV initial Maxwellian is below 5e-7 of its bulk.  The X half-step changes
    basis through the eigenvectors U of (G_v, M_v) (Alg. bte_spatial_adv),
    which are global in speed (cond(U) ~ 1e3), so rounding of order eps times
    the bulk lands on the tail coefficients.  An exact identity, U (U^-1 F) = F,
    evaluated in FP64 already moves k_i n_e by about 4e-9 while n_e moves by
    rounding only.  Two correct FP64 implementations of the step (different
    summation orders) therefore differ by this much in k_i n_e after one step
    from the initial state, and the parity bar for k_i is set from it."""
    cfg = workloads.config("C1")
    ops = oracle.build_operators(cfg)
    F = S.initial_state(ops, workloads.density_profile(ops.xhat, cfg["ic"]["ne_peak"]), cfg["ic"]["Te_eV"])
    c = F[ops.nx // 2, :, 0]
    assert np.abs(c[np.flatnonzero(ops.ki_ord.reshape(ops.nr, ops.nth)[:, 0])]).max() < 1e-6 * np.abs(c).max()
    Fr = np.einsum("ki,xia->xka", ops.U, np.einsum("ik,xka->xia", ops.Uinv, F))
    m0, mr = S.moments(ops, F), S.moments(ops, Fr)
    rel = lambda a, b: np.abs(a - b).max() / np.abs(b).max()
    d_ne = rel(mr[0], m0[0])
    d_ki = rel(mr[0] * mr[2], m0[0] * m0[2])
    assert d_ne < 1e-14
    assert 1e-10 < d_ki < 1e-7, d_ki


def test_reduced_harmonic_basis_vstep():
    """Fewer harmonics than ordinates (Nl < Ntheta; the paper's timed runs use
    Nl = 3 with Ntheta = 16).  With T_S T_O = I_Nl (Gauss-Legendre quadrature is
    exact for Y_q Y_l) P = P_O P_S is a projector of rank Nr Nl, the ordinate
    operators P_O X P_S vanish on its complement, so the V step leaves
    (I - P) F unchanged and conserves nothing it should not touch; and the
    oracle's direct solve of the full Nr Ntheta system equals the exact
    reduction to Nr Nl unknowns,
        (I - P_O K P_S)^-1 b = (I - P_O P_S) b + P_O (I - P_S K' P_O)^-1 P_S b,
    K' = dt (n0 C + E A) in ordinate form, solved here as a separate small system."""
    cfg = dict(workloads.small_config(nx=4, nr=8, nth=8, kinds=("elastic", "excitation", "ionization"),
                                      E=8e3, field_kind="rf"), nl=3)
    ops = oracle.build_operators(cfg)
    nr, nth, nl = ops.nr, ops.nth, ops.nl
    assert np.abs(ops.T_S @ ops.T_O - np.eye(nl)).max() < 1e-13
    PS = np.kron(np.eye(nr), ops.T_S)          # [k][a] -> [k][l]
    PO = np.kron(np.eye(nr), ops.T_O)          # [k][l] -> [k][a]
    P = PO @ PS
    Q = np.eye(nr * nth) - P
    assert np.abs(P @ P - P).max() < 1e-13
    for X in (ops.Cord, ops.Aord):
        sc = np.abs(X).max()
        assert np.abs(X @ Q).max() < 1e-12 * sc and np.abs(Q @ X).max() < 1e-12 * sc
    rng = np.random.default_rng(31)
    F = rng.standard_normal((ops.nx, nr, nth))
    E = np.array([0.0, 5e3, -1.2e4, 2e4])
    Fs = S.v_step(ops, F, E)
    for x in range(ops.nx):
        b = F[x].ravel()
        got = Fs[x].ravel()
        assert np.abs(Q @ (got - b)).max() < 1e-12 * np.abs(b).max()
        Kp = ops.dt * (ops.n0 * PS @ ops.Cord @ PO + E[x] * PS @ ops.Aord @ PO)
        red = Q @ b + PO @ np.linalg.solve(np.eye(nr * nl) - Kp, PS @ b)
        assert np.abs(red - got).max() < 1e-12 * np.abs(got).max()
    # the number functional ignores the complement (only l = 0 carries density)
    assert np.abs(ops.u_ord @ Q).max() < 1e-13 * np.abs(ops.u_ord).max()
