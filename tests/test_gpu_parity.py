"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Tolerances (relative, max-norm over the compared array):
* X(dt/2): the library applies precomputed inverses Q, the oracle LU-solves;
  both are rounding-level apart times cond(B) <= ~1e4  -> 1e-11.
* V(dt) in FP64: LU with partial pivoting on both sides; the difference is
  bounded by cond(I - dt(n0 C + E A)) * eps * growth; cond <= ~3e4 for |E| <=
  1.5e4 V/m at n = 2048 -> 1e-10 (1e-12 for the small cases, cond < 1e3).
* V(dt) mixed: FP32 factors refined in FP64 until max|r| <= 1e-14 max|b|, so
  the error is <= cond * 1e-14 -> 1e-9 at full size, 1e-11 small.
* full runs: the per-step differences above accumulate linearly -> 1e-9 / 1e-8.
"""
import math
import os
import sys

import numpy as np
import pytest

import oracle
import workloads
from oracle import semi_implicit as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2502_16555_amd import _lib
    _lib.load()          # the built library is required: no fallback
    return _t


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def close(a, b, tol, what=""):
    e = rel(a, b)
    if not e < tol:
        raise AssertionError(f"{what}: max relative difference {e:.3e} >= {tol:.1e}")


def cuda(torch, a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")


def solver(cfg, **kw):
    from paper_2502_16555_amd import Solver
    return Solver(cfg, **kw)


CASES = {
    # name: (config factory, tolerance scale)
    "C0": lambda: workloads.config("C0"),
    # ragged: n = 60 is padded to 128, nx odd, three processes, two energy bins
    "ragged": lambda: workloads.small_config(nx=9, nr=10, nth=6, kinds=("elastic", "excitation", "ionization"),
                                             E=5e3, field_kind="rf", n_bins=2),
    # two panels with a ragged tail: n = 12 * 16 = 192 -> padded to 256
    "panels": lambda: workloads.small_config(nx=7, nr=12, nth=16, kinds=("elastic", "ionization"), E=8e3,
                                             field_kind="rf"),
    # four panels: n = 20 * 20 = 400 -> padded to 512
    "panels4": lambda: workloads.small_config(nx=5, nr=20, nth=20, kinds=("elastic", "excitation", "ionization"),
                                              E=1.2e4, field_kind="rf"),
}

# banded V solver: many l blocks of a narrow radial basis -> the band ends well
# inside the matrix (n = 8 * 48 = 384, half-bandwidth 15)
BANDED_CASES = {
    "wide_band": lambda: workloads.small_config(nx=5, nr=8, nth=48, kinds=("elastic", "excitation", "ionization"),
                                                E=1e4, field_kind="rf"),
    # fewer harmonics than ordinates: Nr Nl = 36 harmonic unknowns, n = 192 ordinate unknowns
    "reduced_nl": lambda: dict(workloads.small_config(nx=5, nr=12, nth=16, kinds=("elastic", "excitation",
                                                                                  "ionization"),
                                                      E=1.2e4, field_kind="rf"), nl=3),
}


def _state(ops, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((ops.nx, ops.nr, ops.nth)) * 1e3


def test_device_operators_equal_host_assembly(torch):
    from paper_2502_16555_amd import host_operator
    cfg = CASES["ragged"]()
    s = solver(cfg)
    n = s.n
    assert np.array_equal(s.operator(0, n * n), host_operator(cfg, 0, n * n))
    assert np.array_equal(s.operator(1, n * n), host_operator(cfg, 1, n * n))
    s.close()


@pytest.mark.parametrize("case", sorted(CASES))
def test_xstep_matches_oracle(torch, case):
    cfg = CASES[case]()
    ops = oracle.build_operators(cfg)
    s = solver(cfg)
    F = _state(ops, 1)
    Fg = cuda(torch, F)
    s.xstep(Fg)
    got = Fg.cpu().numpy()
    close(got, S.x_half_step(ops, F), 1e-11, '')
    # transpose: against the oracle and the dot-product identity
    L = _state(ops, 2)
    Lg = cuda(torch, L)
    s.xstep_T(Lg)
    gotT = Lg.cpu().numpy()
    close(gotT, S.x_half_step_T(ops, L), 1e-11, '')
    lhs = np.vdot(got, L)
    rhs = np.vdot(F, gotT)
    assert abs(lhs - rhs) < 1e-11 * np.abs(got).max() * np.abs(L).sum()
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3", "mixed_bf16"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_vstep_matches_oracle(torch, case, prec):
    cfg = CASES[case]()
    ops = oracle.build_operators(cfg)
    s = solver(cfg, precision=prec)
    F = _state(ops, 3)
    rng = np.random.default_rng(4)
    E = rng.uniform(-1.5e4, 1.5e4, size=ops.nx)
    Fg = cuda(torch, F)
    s.vstep(Fg, cuda(torch, E))
    code, sweeps, resid = s.status()
    assert code == 0, (code, sweeps, resid)
    ref = S.v_step(ops, F, E)
    close(Fg.cpu().numpy(), ref, (1e-11 if prec == "fp64" else 1e-10), '')
    if prec != "fp64":
        assert resid <= 1e-14 and sweeps >= 1
    s.close()


# the V solvers as the benchmark runs them: (precision, solver settings, tolerance)
FULL_SIZE = {
    "mixed_fp32": ("mixed_fp32", None, 1e-10),
    "fp64": ("fp64", None, 1e-11),
    # GMRES stops at 1e-12 ||b||: the error is bounded by cond * 1e-12
    "krylov": ("fp64", dict(n_bins=128, bin_scale=100.0, restart=12, cycles=3, rtol=1e-12,
                            factor_precision="mixed_fp32"), 1e-9),
    "banded": ("fp64", "banded", 1e-10),
    "hessenberg": ("fp64", "hessenberg", 1e-10),
    "mixed_fp32_partial": ("mixed_fp32", "partial", 1e-10),
}


@pytest.mark.parametrize("variant", sorted(FULL_SIZE))
def test_full_size_substeps_at_sampled_points(torch, variant):
    """The benchmark's workload at full size (Nx = 256, Nr = 64, Ntheta = 32:
    256 systems of order 2048, sixteen panels in pairs) in the launch
    configuration the benchmark times (the mixed and FP64 LU, and the Krylov and
    banded V solvers with the benchmark's settings).  X(dt/2) and the field are
    checked at every point; V(dt), whose oracle costs one dense solve per point, at points
    spread over the domain (both walls included), each solved by the oracle on
    its own.  The field is taken near its RF peak, where the systems are least
    diagonally dominant."""
    prec, vsolver, tol = FULL_SIZE[variant]
    cfg = workloads.config("C2")
    ops = oracle.build_operators(cfg)
    s = solver(cfg, precision=prec)
    if vsolver in ("banded", "hessenberg"):
        s.set_vsolver(vsolver)
    elif vsolver == "partial":
        from paper_2502_16555_amd import _lib
        s.set_tuning(_lib.TUNE_STATIC_PIVOTING, 0)
    elif vsolver is not None:
        s.set_vsolver("gmres", **vsolver)
    ne = workloads.density_profile(ops.xhat, cfg["ic"]["ne_peak"])
    rng = np.random.default_rng(21)
    F = S.initial_state(ops, ne, cfg["ic"]["Te_eV"]) * (1.0 + 0.1 * rng.standard_normal((ops.nx, ops.nr, ops.nth)))
    t = 0.25 / workloads.RF_FREQ_HZ - 0.5 * ops.dt
    Fg = cuda(torch, F)
    s.xstep(Fg)
    Fh = S.x_half_step(ops, F)
    close(Fg.cpu().numpy(), Fh, 1e-11, 'X(dt/2)')
    E = torch.empty(s.nx_total, dtype=torch.float64, device="cuda:0")
    s.field(cuda(torch, Fh), t, E)
    Eo = S.field_half(ops, t, Fh)
    close(E.cpu().numpy(), Eo, 1e-12, 'field')
    assert np.abs(Eo).max() > 0.9 * cfg["field"]["E0"]
    Fv = cuda(torch, Fh)
    s.vstep(Fv, cuda(torch, Eo))
    code, sweeps, resid = s.status()
    assert code == 0, (code, sweeps, resid)
    if variant in ("mixed_fp32", "mixed_fp32_partial"):
        assert resid <= 1e-14 and sweeps >= 1
    if variant == "krylov":
        assert resid <= 1e-12, (sweeps, resid)
    xs = [0, 1, 37, 128, 200, 254, 255]
    ref = S.v_step(ops, Fh, Eo, xs=xs)
    got = Fv.cpu().numpy()
    for x in xs:
        close(got[x], ref[x], tol, f'V(dt) at x = {x}')
    s.close()


@pytest.mark.parametrize("case", sorted(CASES))
def test_initial_state_and_moments(torch, case):
    cfg = CASES[case]()
    ops = oracle.build_operators(cfg)
    s = solver(cfg)
    ne = workloads.density_profile(s.xhat(), 1e16)
    Fg = s.initial_state(cuda(torch, ne), 1.0)
    F0 = S.initial_state(ops, ne, 1.0)
    close(Fg.cpu().numpy(), F0, 1e-12, '')
    F = np.abs(_state(ops, 5))
    m = s.moments(cuda(torch, F)).cpu().numpy()
    mo = S.moments(ops, F)
    for q in range(3):
        if np.abs(mo[q]).max() > 0:
            close(m[q], mo[q], 1e-12, q)
    s.close()


def test_c0_full_run_matches_oracle(torch):
    """The tiny plain case run to the end (100 steps) on both sides."""
    cfg = workloads.config("C0")
    ops = oracle.build_operators(cfg)
    s = solver(cfg)
    ne = workloads.density_profile(ops.xhat, 1e16)
    F = S.initial_state(ops, ne, 1.0)
    Fg = cuda(torch, F)
    for n in range(cfg["n_steps"]):
        t = n * ops.dt
        F = S.step(ops, F, t)
        s.step(Fg, t)
        if (n + 1) % 10 == 0:
            mg = s.moments(Fg).cpu().numpy()
            mo = S.moments(ops, F)
            close(mg[0], mo[0], 1e-10, n)
            inner = mo[0] > 1e-3 * mo[0].max()
            close(mg[1][inner], mo[1][inner], 1e-10, n)
    close(Fg.cpu().numpy(), F, 1e-10, '')
    assert s.status()[0] == 0
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_step_is_the_composition_of_substeps(torch, prec):
    cfg = CASES["panels"]()
    ops = oracle.build_operators(cfg)
    s = solver(cfg, precision=prec)
    F = _state(ops, 6)
    A = cuda(torch, F)
    B = cuda(torch, F)
    t = 0.37 * cfg["T_rf_s"]
    s.step(A, t)
    E = torch.empty(s.nx_total, dtype=torch.float64, device="cuda:0")
    s.xstep(B)
    s.field(B, t, E)
    s.vstep(B, E)
    s.xstep(B)
    assert torch.equal(A, B)
    # and the field kernel matches the specified RF form
    Eo = S.field_half(ops, t)
    close(E.cpu().numpy(), Eo, 1e-14, '')
    s.close()


@pytest.mark.parametrize("prec,x_fp32,tol", [("fp64", False, 1e-10), ("mixed_fp32", False, 1e-10),
                                             ("mixed_fp32", True, 2e-5)])
def test_rf_steps_match_oracle(torch, prec, x_fp32, tol):
    """A few full steps of the realistic case with ionization and excitation.
    With Q streamed in FP32 every X(dt/2) rounds Q to 2^-24 relative, which after
    amplification by the Chebyshev systems measured ~2e-7 per half-step."""
    cfg = CASES["ragged"]()
    ops = oracle.build_operators(cfg)
    if True:
        s = solver(cfg, precision=prec, x_fp32=x_fp32)
        F = S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 1.0)
        Fg = cuda(torch, F)
        for n in range(5):
            t = (n + 200) * ops.dt
            F = S.step(ops, F, t)
            s.step(Fg, t)
        close(Fg.cpu().numpy(), F, tol, prec)
        s.close()


def test_poisson_field_matches_oracle(torch):
    cfg = CASES["ragged"]()
    cfg["field"] = {"kind": "poisson", "V0": 100.0, "freq_hz": workloads.RF_FREQ_HZ}
    ops = oracle.build_operators(cfg)
    s = solver(cfg)
    F = np.abs(_state(ops, 8)) * 1e-3
    ni = np.full(ops.nx, 2e15)
    t = 0.1 * cfg["T_rf_s"]
    E = torch.empty(s.nx_total, dtype=torch.float64, device="cuda:0")
    s.field(cuda(torch, F), t, E, ni=cuda(torch, ni))
    V_left = 100.0 * math.sin(2 * math.pi * workloads.RF_FREQ_HZ * (t + 0.5 * ops.dt))
    Eo = S.field_half(ops, t, F, ni=ni, V_left=V_left)
    close(E.cpu().numpy(), Eo, 1e-11, '')
    s.close()


@pytest.mark.parametrize("nx,tol", [(130, 1e-11), (256, 1e-11), (700, 1e-10), (1024, 1e-10)])
def test_poisson_field_large_nx_matches_oracle(torch, nx, tol):
    """The Poisson field at large Nx, in a state where n_i - n_e changes sign
    across the gap.  Its operator (D_x^2 with Dirichlet rows) has a condition
    number of order Nx^4: the library forms and inverts it in 80-bit arithmetic,
    the oracle inverts it in double (LAPACK), whose rounding sets the
    agreement: measured 2e-13 (Nx = 130), 2e-12 (256), 8e-12 (700), 3e-11
    (1024).  An inverse by Gauss-Jordan in double was 1000x further off."""
    cfg = _hybrid_cfg(nx)
    ops = oracle.build_operators(cfg)
    s = solver(cfg)
    F = S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 2.0)
    ni = 0.8 * S.moments(ops, F)[0] + 3e14 * (1.0 + ops.xhat)
    t = 0.3 * cfg["T_rf_s"]
    E = torch.empty(s.nx_total, dtype=torch.float64, device="cuda:0")
    s.field(cuda(torch, F), t, E, ni=cuda(torch, ni))
    V_left = 150.0 * math.sin(2 * math.pi * workloads.RF_FREQ_HZ * (t + 0.5 * ops.dt))
    Eo = S.field_half(ops, t, F, ni=ni, V_left=V_left)
    close(E.cpu().numpy(), Eo, tol, f"Poisson field nx={nx}")
    s.close()


@pytest.mark.parametrize("nx", [9, 256, 1024])
def test_poisson_field_exact_for_a_quadratic_potential(torch, nx):
    """A closed form, independent of the oracle: with no electrons and a uniform
    ion density n_i, eq. (voltage_bc) with V(0) = V_left, V(L) = 0 has the
    quadratic solution V = V_left (1 - s) + a s (1 - s), s = x / L, with
    a = e n_i L^2 / (2 eps0), so E = -V' = (V_left - a (1 - 2 s)) / L.
    Collocation on the CGL nodes is exact for it, which leaves rounding: the
    field must hold to 1e-11 of its largest value even at Nx = 1024."""
    cfg = _hybrid_cfg(nx, V0=100.0)
    s = solver(cfg)
    xhat = s.xhat()
    L = cfg["L_m"]
    ni = np.full(nx, 1e15)
    t = 0.1 * cfg["T_rf_s"]
    E = torch.empty(s.nx_total, dtype=torch.float64, device="cuda:0")
    F = torch.zeros((nx, cfg["nr"], cfg["ntheta"]), dtype=torch.float64, device="cuda:0")
    s.field(F, t, E, ni=cuda(torch, ni))
    V_left = 100.0 * math.sin(2 * math.pi * workloads.RF_FREQ_HZ * (t + 0.5 * cfg["dt_s"]))
    a = 1.602176634e-19 * 1e15 * L * L / (2 * 8.8541878128e-12)
    sx = 0.5 * (np.asarray(xhat) + 1.0)
    close(E.cpu().numpy(), (V_left - a * (1.0 - 2.0 * sx)) / L, 1e-11, f"quadratic potential nx={nx}")
    s.close()


def _hybrid_cfg(nx=9, V0=150.0):
    cfg = workloads.small_config(nx=nx, nr=10, nth=6, kinds=("elastic", "excitation", "ionization"), E=5e3,
                                 field_kind="rf", n_bins=2)
    cfg["field"] = {"kind": "poisson", "V0": V0, "freq_hz": workloads.RF_FREQ_HZ}
    return cfg


@pytest.mark.parametrize("nx", [9, 37, 130, 256, 700, 1024])
def test_ion_step_matches_oracle(torch, nx):
    """Heavies' update of the hybrid model (eq. fluid_step) against the oracle's
    dense solve: ragged Nx (130 spans more than two 64-row wavefronts), the
    benchmark's Nx = 256, and the 8-column panels above Nx = 512 (700, ragged,
    and the largest Nx, 1024).  With its wall rows equilibrated the system's
    condition number stays below 100 up to Nx = 1024."""
    from oracle import hybrid as H
    cfg = _hybrid_cfg(nx)
    ops = oracle.build_operators(cfg)
    s = solver(cfg)
    F = S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 2.0)
    ni = 0.8 * S.moments(ops, F)[0] + 3e14 * (1.0 + ops.xhat)
    t = 0.3 * cfg["T_rf_s"]
    out = torch.empty(s.nx_total, dtype=torch.float64, device="cuda:0")
    s.ion_step(cuda(torch, F), cuda(torch, ni), out, t)
    assert s.status()[0] == 0
    close(out.cpu().numpy(), H.ion_step(ops, ni, F, t), 1e-10, f"ion step nx={nx}")
    s.close()


def test_hybrid_steps_match_oracle(torch):
    """Five hybrid steps (ions, then electrons with the Poisson field of the new
    ion density) against the oracle, F and n_i."""
    from oracle import hybrid as H
    cfg = _hybrid_cfg(9)
    ops = oracle.build_operators(cfg)
    s = solver(cfg)
    F0 = S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 2.0)
    ni0 = S.moments(ops, F0)[0] * 1.05
    F = cuda(torch, F0)
    ni = cuda(torch, ni0)
    Fo, nio = F0, ni0
    t0 = 0.15 * cfg["T_rf_s"]
    for k in range(5):
        s.hybrid_step(F, ni, t0 + k * ops.dt)
        Fo, nio = H.hybrid_step(ops, Fo, nio, t0 + k * ops.dt)
    assert s.status()[0] == 0
    close(ni.cpu().numpy(), nio, 1e-10, "n_i")
    close(F.cpu().numpy(), Fo, 1e-10, "F")
    s.close()


@pytest.mark.parametrize("nx_per", [(5, 9, 7), (5, 600, 9)])
def test_hybrid_ensemble_per_discharge(torch, nx_per):
    """The hybrid step of an uneven ensemble (three sizes and pressures) against
    the oracle per discharge; with Nx = 600 in it, every discharge of the launch
    takes the ion elimination's 8-column panels."""
    from oracle import hybrid as H
    cfg, members = _ensemble_case(nx_per)
    fld = {"kind": "poisson", "V0": 120.0, "freq_hz": workloads.RF_FREQ_HZ}
    cfg["field"] = fld
    for m in members:
        m["field"] = dict(fld)
    ops = [oracle.build_operators(m) for m in members]
    F0 = [S.initial_state(o, workloads.density_profile(o.xhat, 1e16), 1.0) for o in ops]
    ni0 = [S.moments(o, f)[0] * 0.9 for o, f in zip(ops, F0)]
    s = solver(cfg)
    F = cuda(torch, np.concatenate(F0))
    ni = cuda(torch, np.concatenate(ni0))
    t0 = 0.4 * cfg["T_rf_s"]
    ref = list(zip(F0, ni0))
    for k in range(3):
        s.hybrid_step(F, ni, t0 + k * cfg["dt_s"])
        ref = [H.hybrid_step(o, f, n, t0 + k * cfg["dt_s"]) for o, (f, n) in zip(ops, ref)]
    assert s.status()[0] == 0
    got_F, got_n = F.cpu().numpy(), ni.cpu().numpy()
    o = 0
    for d, (f, n) in enumerate(ref):
        close(got_n[o:o + n.shape[0]], n, 1e-10, f"discharge {d} n_i")
        close(got_F[o:o + f.shape[0]], f, 1e-10, f"discharge {d} F")
        o += n.shape[0]
    s.close()


@pytest.mark.parametrize("kind,prec,dt_mult,precond", [
    ("const", "fp64", 1.0, 0), ("rf", "mixed_fp32", 1.0, 0), ("poisson", "fp64", 1.0, 0),
    ("poisson", "mixed_fp32", 1.0, 0), ("rf", "mixed_fp32", 10.0, 0), ("poisson", "mixed_fp32", 10.0, 0),
    ("rf", "mixed_fp32", 1.0, 1), ("poisson", "fp64", 1.0, 1), ("rf", "mixed_fp32", 10.0, 1)])
def test_implicit_step_matches_oracle(torch, kind, prec, dt_mult, precond):
    """Fully implicit step (Newton-Krylov, preconditioned by the V-then-x split
    (precond 0) or by the semi-implicit step (precond 1)) against the oracle's
    Newton iteration with a dense Jacobian: specified and Poisson fields, FP64
    and mixed preconditioners, and steps ten times the semi-implicit one (with
    the Poisson field, Newton from F^n with a monotone line search stalls there:
    the full first step overshoots ||R|| a hundredfold; the frozen-field first
    step does not)."""
    from oracle import implicit as I
    cfg = workloads.small_config(nx=9, nr=10, nth=6, kinds=("elastic", "excitation", "ionization"), E=5e3,
                                 field_kind="rf" if kind == "rf" else "const", n_bins=2)
    if kind == "poisson":
        cfg["field"] = {"kind": "poisson", "V0": 100.0, "freq_hz": workloads.RF_FREQ_HZ}
    cfg["dt_s"] *= dt_mult
    ops = oracle.build_operators(cfg)
    F0 = S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 2.0)
    ni = 1.1 * S.moments(ops, F0)[0] if kind == "poisson" else None
    t = 0.2 * cfg["T_rf_s"]
    s = solver(cfg, precision=prec)
    F = cuda(torch, F0)
    st = s.implicit_step(F, t, ni=cuda(torch, ni) if ni is not None else None, newton_rtol=1e-13,
                         gmres_rtol=1e-11, restart=40, max_gmres=400, precond=precond)
    assert st["status"] == 0 and st["residual"] <= 1e-13 * np.linalg.norm(F0) * 1.0001, st
    assert s.status()[0] == 0
    got = F.cpu().numpy()
    if kind == "poisson" and dt_mult > 1.0:
        # the quadratic equations have more than one root at this step: the
        # oracle's full-step Newton from F^n lands on another one, so the check
        # is that this result solves the oracle's equations
        r = I.residual(ops, got, F0, t + ops.dt, ni)
        assert np.linalg.norm(r) <= 1e-11 * np.linalg.norm(F0), np.linalg.norm(r)
    else:
        ref, its = I.implicit_step(ops, F0, t, ni)
        close(got, ref, 1e-10, f"implicit {kind} {prec} x{dt_mult} precond {precond}")
    s.close()


def test_implicit_split_preconditioner_beats_semi_implicit(torch):
    """On a grid whose x modes are stiff over the step (Nx = 96), the V-then-x
    split leaves GMRES far fewer iterations than the semi-implicit step as
    preconditioner (whose inverse misses J by dt^2 X^2 / 4 on those modes), and
    both reach the same Newton solution."""
    cfg = workloads.small_config(nx=96, nr=12, nth=8, kinds=("elastic", "excitation", "ionization"), E=5e3,
                                 field_kind="rf", n_bins=1)
    ops = oracle.build_operators(cfg)
    F0 = S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 2.0)
    t = 0.2 * cfg["T_rf_s"]
    out, its = [], []
    for pk in (0, 1):
        s = solver(cfg, precision="fp64")
        F = cuda(torch, F0)
        st = s.implicit_step(F, t, newton_rtol=1e-12, gmres_rtol=1e-8, restart=60, max_gmres=600, precond=pk)
        assert st["status"] == 0, (pk, st)
        out.append(F.cpu().numpy())
        its.append(st["gmres_iters"])
        s.close()
    assert its[0] * 3 <= its[1], its
    close(out[0], out[1], 1e-10, "split vs semi-implicit preconditioner")


@pytest.mark.parametrize("precond", [0, 1])
def test_implicit_ensemble_matches_oracle_per_discharge(torch, precond):
    """The fully implicit step over an uneven ensemble (Nx = 5, 9, 7; different
    pressures and amplitudes) in one Krylov space: each discharge's part
    against the oracle's Newton iteration for that discharge alone."""
    from oracle import implicit as I
    cfg, members = _ensemble_case()
    ops = [oracle.build_operators(m) for m in members]
    F0 = [S.initial_state(o, workloads.density_profile(o.xhat, 1e16), 1.0) for o in ops]
    t = 0.3 * cfg["T_rf_s"]
    s = solver(cfg, precision="mixed_fp32")
    F = cuda(torch, np.concatenate(F0))
    st = s.implicit_step(F, t, newton_rtol=1e-13, gmres_rtol=1e-11, restart=40, max_gmres=400, precond=precond)
    assert st["status"] == 0, st
    assert s.status()[0] == 0
    got = F.cpu().numpy()
    o = 0
    for d, (op, f0) in enumerate(zip(ops, F0)):
        ref, _ = I.implicit_step(op, f0, t)
        close(got[o:o + f0.shape[0]], ref, 1e-10, f"discharge {d} precond {precond}")
        o += f0.shape[0]
    s.close()


@pytest.mark.parametrize("precond", [0, 1])
def test_implicit_step_with_reduced_harmonics(torch, precond):
    """The fully implicit step with Nl = 3 < Ntheta = 16 (the operator part of the
    V systems has rank Nr Nl; the rest of the state moves by advection only)
    against the oracle's Newton iteration, at four times the semi-implicit dt."""
    from oracle import implicit as I
    cfg = BANDED_CASES["reduced_nl"]()
    cfg["dt_s"] *= 4
    ops = oracle.build_operators(cfg)
    F0 = S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 2.0)
    t = 0.15 * cfg["T_rf_s"]
    s = solver(cfg, precision="mixed_fp32")
    F = cuda(torch, F0)
    st = s.implicit_step(F, t, newton_rtol=1e-13, gmres_rtol=1e-11, restart=40, max_gmres=400, precond=precond)
    assert st["status"] == 0, st
    assert s.status()[0] == 0
    ref, _ = I.implicit_step(ops, F0, t)
    close(F.cpu().numpy(), ref, 1e-10, f"reduced harmonics precond {precond}")
    s.close()


def test_implicit_step_at_largest_nx_solves_oracle_equations(torch):
    """Nx = 1024, the largest the library takes (the forward x operator's eight
    mode rows then fill exactly 64 KB of LDS), with a tiny velocity grid: the
    oracle's residual of eq. bte_fully_implicit at the result is within the
    Newton tolerance (a dense oracle Newton solve is out of reach at this size)."""
    from oracle import implicit as I
    cfg = workloads.small_config(nx=1024, nr=4, nth=2, kinds=("elastic",), E=2e3, field_kind="const", n_bins=1)
    ops = oracle.build_operators(cfg)
    F0 = S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 2.0)
    s = solver(cfg, precision="fp64")
    F = cuda(torch, F0)
    st = s.implicit_step(F, 0.0, newton_rtol=1e-12, gmres_rtol=1e-10, restart=60, max_gmres=600)
    assert st["status"] == 0, st
    r = I.residual(ops, F.cpu().numpy(), F0, ops.dt)
    assert np.linalg.norm(r) <= 1e-11 * np.linalg.norm(F0), (np.linalg.norm(r), st)
    s.close()


def test_implicit_rejects_unknown_preconditioner(torch):
    cfg = workloads.small_config(nx=9, nr=10, nth=6, field_kind="rf")
    ops = oracle.build_operators(cfg)
    s = solver(cfg, precision="fp64")
    F = cuda(torch, S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 2.0))
    with pytest.raises(Exception, match="invalid argument"):
        s.implicit_step(F, 0.0, precond=2, raise_on_noconv=False)
    s.close()


def test_adjoint_step_matches_oracle(torch):
    cfg = CASES["ragged"]()
    ops = oracle.build_operators(cfg)
    s = solver(cfg)
    F = _state(ops, 9)
    L = _state(ops, 10)
    t = 0.21 * cfg["T_rf_s"]
    lam_o, gs_o, gE_o = S.adjoint_step(ops, F, t, L)
    Lg = cuda(torch, L)
    gs = torch.zeros(s.n_params, dtype=torch.float64, device="cuda:0")
    gE0 = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    gE = torch.zeros(s.nx_total, dtype=torch.float64, device="cuda:0")
    s.adjoint_step(cuda(torch, F), t, Lg, gs, gE0, gE)
    close(Lg.cpu().numpy(), lam_o, 1e-10, '')
    close(gs.cpu().numpy(), gs_o, 1e-10, '')
    close(gE.cpu().numpy(), gE_o, 1e-10, '')
    assert abs(gE0.item() - gE_o @ S.field_dE0(ops, t)) < 1e-10 * np.abs(gE_o).sum()
    s.close()


def test_adjoint_step_is_bitwise_reproducible(torch):
    """The gradient contractions sum their per-block partials in a fixed order
    (no floating-point atomics), so repeated adjoint steps from the same inputs
    give the same bits: lambda, the scaling gradients, dL/dE0 and dL/dE, on an
    ensemble whose points span several 32-point blocks."""
    cfg, _ = _ensemble_case((37, 41, 29))
    rng = np.random.default_rng(17)
    Fn = rng.standard_normal((sum(cfg["nx_per"]), cfg["nr"], cfg["ntheta"]))
    lam0 = rng.standard_normal(Fn.shape)
    t = 0.3 * cfg["T_rf_s"]
    s = solver(cfg)
    outs = []
    for rep in range(3):
        lam = cuda(torch, lam0)
        gs = torch.zeros(s.n_params, dtype=torch.float64, device="cuda:0")
        gE0 = torch.zeros(3, dtype=torch.float64, device="cuda:0")
        gE = torch.zeros(s.nx_total, dtype=torch.float64, device="cuda:0")
        s.adjoint_step(cuda(torch, Fn), t, lam, gs, gE0, gE)
        outs.append([a.cpu().numpy() for a in (lam, gs, gE0, gE)])
    assert s.status()[0] == 0
    for rep in (1, 2):
        for a, b in zip(outs[rep], outs[0]):
            assert np.array_equal(a, b), rep
    s.close()


def test_nonfinite_state_is_reported(torch):
    from paper_2502_16555_amd import _lib
    cfg = workloads.config("C0")
    s = solver(cfg)
    F = s.new_state()
    F[3, 2, 1] = float("nan")
    s.step(F, 0.0)
    assert s.status()[0] == _lib.BTE_ENONFINITE
    assert s.status()[0] == 0          # latched status is cleared once read
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_nonfinite_field_is_reported(torch, prec):
    """A NaN field makes whole pivot columns NaN: the factorization keeps every
    row index in range (no interchange) and reports the non-finite value."""
    from paper_2502_16555_amd import _lib
    cfg = CASES["panels"]()
    s = solver(cfg, precision=prec, field_mode="given")
    ops = oracle.build_operators(cfg)
    F = cuda(torch, _state(ops, 5))
    E = torch.full((s.nx_total,), 1e3, dtype=torch.float64, device="cuda:0")
    E[2] = float("nan")
    s.vstep(F, E)
    assert s.status()[0] == _lib.BTE_ENONFINITE
    E[2] = 1e3
    F = cuda(torch, _state(ops, 5))
    s.vstep(F, E)                      # the handle stays usable
    assert s.status()[0] == 0
    s.close()


def _golden_run(torch, name, n_file_steps, mode, tol, tol_ki=None):
    """Run the stored oracle workload ``name`` on the GPU from its initial state
    and compare n_e, the mean energy (everywhere, and on points with n_e above
    1e-3 of its peak), the energy density and k_i n_e (to tol_ki, default tol)
    at every stored step, and the final state."""
    tol_ki = tol if tol_ki is None else tol_ki
    path = os.path.join(ROOT, "tests", "golden", f"{name.lower()}_oracle_{n_file_steps}.npz")
    if not os.path.exists(path):
        pytest.skip(f"golden file {os.path.basename(path)} not generated")
    g = np.load(path, allow_pickle=False)
    cfg = workloads.config(name)
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import make_golden
    assert str(g["config_hash"]) == make_golden.config_hash(cfg), f"{name} workload changed since the golden run"
    partial = mode.endswith("_partial")   # mixed precision with partially pivoted FP32 factors
    prec = mode[:-len("_partial")] if partial else mode
    s = solver(cfg, precision="fp64" if mode in ("banded", "hessenberg") else prec)
    if mode in ("banded", "hessenberg"):
        s.set_vsolver(mode)
    if partial:
        from paper_2502_16555_amd import _lib
        s.set_tuning(_lib.TUNE_STATIC_PIVOTING, 0)
    ne = workloads.density_profile(s.xhat(), cfg["ic"]["ne_peak"])
    Fg = s.initial_state(cuda(torch, ne), cfg["ic"]["Te_eV"])
    every = int(g["every"])
    worst = {}
    for n in range(int(g["n_steps"])):
        s.step(Fg, n * cfg["dt_s"])
        if (n + 1) % every == 0:
            mg = s.moments(Fg).cpu().numpy()
            mo = g["moments"][(n + 1) // every]
            inner = mo[0] > 1e-3 * mo[0].max()
            for what, a, b in (("n_e", mg[0], mo[0]), ("mean energy", mg[1], mo[1]),
                               ("mean energy (n_e > 1e-3 max)", mg[1][inner], mo[1][inner]),
                               ("energy density", mg[0] * mg[1], mo[0] * mo[1]),
                               ("k_i n_e", mg[0] * mg[2], mo[0] * mo[2])):
                worst[what] = max(worst.get(what, 0.0), rel(a, b))
                close(a, b, tol_ki if what == "k_i n_e" else tol, f"{mode} {what} at step {n + 1}")
    worst["final state"] = rel(Fg.cpu().numpy(), g["F"])
    print(f"{name} {mode}: " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()))
    close(Fg.cpu().numpy(), g["F"], tol, f"{mode} final state")
    assert s.status()[0] == 0
    s.close()


GOLDEN_MODES = ["fp64", "mixed_fp32", "mixed_bf16x3", "mixed_bf16", "mixed_fp32_partial", "banded", "hessenberg"]


@pytest.mark.parametrize("mode", GOLDEN_MODES)
def test_c1_golden_cycle(torch, mode):
    """Realistic RF case (Nx=64, Nr=64, Ntheta=32), one full cycle of 1000 steps on
    the GPU against the stored oracle (written by tests/golden/make_golden.py,
    which calls only the oracle), every 100 steps and at the end, for every
    V solver and precision: FP64 LU, FP32 / split-bf16 / bf16 factors with FP64
    refinement, and the banded harmonic-basis LU.

    Tolerance 2e-10 for all of them, n_e, mean energy and k_i alike: the
    refinement brings the mixed steps to the FP64 backward error, so every
    path carries the FP64 rounding of the X step (Chebyshev systems of
    condition ~1e4) and of the V solve, which adds up about linearly over the
    steps: measured 1.6e-12 per 100 steps, 1.8e-11 after the cycle for every
    mode and result.  (One step from the initial Maxwellian, k_i n_e agrees to
    only ~1e-8, see test_ionization_rate_is_sensitive_to_speed_mode_rounding; by
    step 100 the field has filled the tail and the gap is gone.)"""
    _golden_run(torch, "C1", 1000, mode, 2e-10)


@pytest.mark.parametrize("mode", [m for m in GOLDEN_MODES if m not in ("banded", "hessenberg")])
def test_c2_golden_run(torch, mode):
    """The benchmark workload itself (Nx=256, Nr=64, Ntheta=32: 256 systems of
    order 2048 per step) for the first 100 steps of the RF cycle against the
    stored oracle run (every 10 steps and the final state), in FP64 and in the
    three mixed forms of the precision workload (FP32, split-bf16 and bf16
    trailing updates, each with FP64 refinement).  The target for the mixed
    step is 1e-6 relative on n_e and the mean energy; the test holds n_e, the
    mean energy and the energy density to 1e-9 (the FP64 rounding of the steps,
    as for C1), and k_i n_e to that same 1e-6: in the first tens of steps the
    ionization tail is still the initial Maxwellian's, below 1e-6 of the bulk,
    where FP64 rounding of the speed-mode transforms shows (measured 6e-8 at
    step 10; test_ionization_rate_is_sensitive_to_speed_mode_rounding)."""
    _golden_run(torch, "C2", 100, mode, 1e-9, tol_ki=1e-6)


def test_refinement_nonconvergence_is_latched_and_the_handle_recovers(torch):
    """With one refinement sweep and an unreachable stop (rtol 1e-30) the mixed
    V step latches BTE_ENOCONV; the state holds the last iterate (finite, and
    one sweep from the FP32 factors already agrees with the oracle to 1e-9).
    After restoring the default stop the same handle steps cleanly and matches
    the oracle to the mixed tolerance."""
    from paper_2502_16555_amd import _lib
    cfg = CASES["panels"]()
    ops = oracle.build_operators(cfg)
    s = solver(cfg, precision="mixed_fp32")
    F0 = _state(ops, 13)
    t = 0.3 * cfg["T_rf_s"]
    ref = S.step(ops, F0, t)
    s.set_refine(1, 1e-30)
    Fg = cuda(torch, F0)
    s.step(Fg, t)
    code, sweeps, resid = s.status()
    assert code == _lib.BTE_ENOCONV and sweeps == 1 and resid > 0, (code, sweeps, resid)
    assert s.status()[0] == 0                  # read once, then cleared
    got = Fg.cpu().numpy()
    assert np.isfinite(got).all()
    close(got, ref, 1e-9, "last iterate after one sweep")
    s.set_refine(0, 0.0)                       # defaults: 10 sweeps, 1e-14
    Fg = cuda(torch, F0)
    s.step(Fg, t)
    code, sweeps, resid = s.status()
    assert code == 0 and 1 <= sweeps <= 10 and resid <= 1e-14, (code, sweeps, resid)
    close(Fg.cpu().numpy(), ref, 1e-10, "after recovery")
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3", "mixed_bf16"])
def test_device_factors_match_blocked_restatement(torch, prec):
    """Device LU factors and pivots against the NumPy restatement of the same blocked
    algorithm with partial pivoting: identical pivots, factors equal to rounding
    (FP32: 1e-4 relative)."""
    import lu_reference as LR
    from paper_2502_16555_amd import _lib
    cfg = CASES["panels4"]()
    ops = oracle.build_operators(cfg)
    s = solver(cfg, precision=prec)
    if prec != "fp64":
        s.set_tuning(_lib.TUNE_STATIC_PIVOTING, 0)   # the partially pivoted FP32 factors
    E = np.array([0.0, 1.2e4, -1.4e4, 3e3, -6e3])[:ops.nx]
    Eg = cuda(torch, E)
    IB = 8 if prec == "fp64" else 16
    for x in (0, 1, 2):
        lu, piv = s.factor_export(Eg, x)
        M = LR.pad(S.v_matrix(ops, E[x]))
        if prec != "fp64":
            M = M.astype(np.float32).astype(np.float64)
        ref, ip = LR.factor(M, IB, pairs=True)   # dense factors take the panels in pairs
        nb = LR.NB
        # FP32 factors: 1e-4; bf16 products split in three terms keep ~16 bits of
        # each operand (2e-3 after the updates); plain bf16 operands keep 8 bits
        tol = {"fp64": 1e-12, "mixed_fp32": 1e-4, "mixed_bf16x3": 2e-3, "mixed_bf16": 5e-2}[prec]
        for k0 in range(0, len(M), nb):
            blk = slice(k0, k0 + nb)
            close(lu[k0:, blk], ref[k0:, blk], tol, (x, "L panel", k0))
            close(lu[blk, k0:], ref[blk, k0:], tol, (x, "U rows", k0))
        if prec == "fp64":
            assert np.array_equal(piv, ip), x
    s.close()


@pytest.mark.parametrize("prec", ["mixed_fp32", "mixed_bf16x3", "mixed_bf16"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_partial_pivoting_vstep_matches_oracle(torch, case, prec):
    """The mixed precisions factor without row interchanges by default (static
    pivoting, covered by test_vstep_matches_oracle); the partially pivoted FP32
    factors, still selectable, refine to the same solution and backward error,
    for fields up to 1.5e4 V/m of either sign."""
    from paper_2502_16555_amd import _lib
    cfg = CASES[case]()
    ops = oracle.build_operators(cfg)
    s = solver(cfg, precision=prec)
    assert s.get_tuning(_lib.TUNE_STATIC_PIVOTING) == 1
    s.set_tuning(_lib.TUNE_STATIC_PIVOTING, 0)
    assert s.get_tuning(_lib.TUNE_STATIC_PIVOTING) == 0
    F = _state(ops, 3)
    rng = np.random.default_rng(4)
    E = rng.uniform(-1.5e4, 1.5e4, size=ops.nx)
    Fg = cuda(torch, F)
    s.vstep(Fg, cuda(torch, E))
    code, sweeps, resid = s.status()
    assert code == 0, (code, sweeps, resid)
    assert resid <= 1e-14 and sweeps >= 1
    close(Fg.cpu().numpy(), S.v_step(ops, F, E), 1e-10, f"{case} partial pivoting")
    s.close()


def test_static_pivoting_factors_match_restatement(torch):
    """The device factors with static pivoting against the NumPy restatement
    (no interchanges; each diagonal block's tiny pivots replaced; L21 through
    U11^-1), a negative field's point factored as its angular mirror image:
    identity pivots, factors equal to FP32 rounding."""
    import lu_reference as LR
    from paper_2502_16555_amd import _lib
    cfg = CASES["panels4"]()
    ops = oracle.build_operators(cfg)
    s = solver(cfg, precision="mixed_fp32")
    assert s.get_tuning(_lib.TUNE_STATIC_PIVOTING) == 1   # the default for mixed precisions
    E = np.array([0.0, 1.2e4, -1.4e4, 3e3, -6e3])[:ops.nx]
    Eg = cuda(torch, E)
    for x in (0, 1, 2):
        lu, piv = s.factor_export(Eg, x)
        # a negative field is factored as its angular mirror image, M(|E|) = J M(E) J
        M = LR.pad(S.v_matrix(ops, abs(E[x]))).astype(np.float32).astype(np.float64)
        ref, ip = LR.factor_static(M)
        assert np.array_equal(piv, ip), x
        for k0 in range(0, len(M), LR.NB):
            blk = slice(k0, k0 + LR.NB)
            close(lu[k0:, blk], ref[k0:, blk], 1e-4, (x, "L panel", k0))
            close(lu[blk, k0:], ref[blk, k0:], 1e-4, (x, "U rows", k0))
    s.close()


def test_static_pivoting_is_rejected_for_fp64(torch):
    from paper_2502_16555_amd import _lib
    s = solver(CASES["ragged"](), precision="fp64")
    with pytest.raises(Exception):
        s.set_tuning(_lib.TUNE_STATIC_PIVOTING, 1)
    assert s.get_tuning(_lib.TUNE_STATIC_PIVOTING) == 0
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32", "mixed_bf16x3"])
def test_factorization_schedule_does_not_change_results(torch, prec):
    """Factoring the points in 1..4 concurrent groups, with or without the
    look-ahead of the statically pivoted panels and the overlap of the formation
    with the first pair (both off by default), gives bit-identical steps,
    with the panels in pairs (K = 256 trailing updates) and singly; the two
    forms round the trailing updates differently and agree to rounding (four
    panels: one pair, then two single panels)."""
    from paper_2502_16555_amd import _lib
    cfg = CASES["panels4"]()
    ops = oracle.build_operators(cfg)
    F0 = _state(ops, 11)
    res = {}
    for pairs in (1, 0):
        outs = []
        for g in (1, 2, 3, 4):
            s = solver(cfg, precision=prec)
            s.set_tuning(_lib.TUNE_LU_STREAMS, g)
            s.set_tuning(_lib.TUNE_PANEL_PAIRS, pairs)
            assert s.get_tuning(_lib.TUNE_LU_STREAMS) == g
            assert s.get_tuning(_lib.TUNE_PANEL_PAIRS) == pairs
            F = cuda(torch, F0)
            for n in range(3):
                s.step(F, n * cfg["dt_s"])
            assert s.status()[0] == 0
            outs.append(F.cpu().numpy())
            s.close()
        for g, o in enumerate(outs[1:], start=2):
            assert np.array_equal(o, outs[0]), f"pairs={pairs}: {g} groups differ from 1"
        if prec != "fp64":
            # one group with the look-ahead of the statically pivoted panels and
            # the formation overlap (both off by default)
            for ahead, fover in ((1, 1), (0, 1), (1, 0)):
                s = solver(cfg, precision=prec)
                s.set_tuning(_lib.TUNE_PANEL_PAIRS, pairs)
                assert s.get_tuning(_lib.TUNE_LOOK_AHEAD) == 0
                assert s.get_tuning(_lib.TUNE_FORM_OVERLAP) == 0
                s.set_tuning(_lib.TUNE_LOOK_AHEAD, ahead)
                s.set_tuning(_lib.TUNE_FORM_OVERLAP, fover)
                F = cuda(torch, F0)
                for n in range(3):
                    s.step(F, n * cfg["dt_s"])
                assert s.status()[0] == 0
                assert np.array_equal(F.cpu().numpy(), outs[0]), \
                    f"pairs={pairs}: look-ahead {ahead} / formation overlap {fover} change the result"
                s.close()
        res[pairs] = outs[0]
    tol = 1e-12 if prec == "fp64" else 1e-13   # mixed: refined to the FP64 backward error
    close(res[1], res[0], tol, "pairs vs single panels")


@pytest.mark.parametrize("case", ["panels4", "panels6"])
@pytest.mark.parametrize("prec", ["mixed_fp32", "mixed_bf16x3", "mixed_bf16"])
def test_panel_groups_of_four_match_pairs(torch, prec, case):
    """Statically pivoted factors in groups of four panels (BTE_TUNE_PANEL_PAIRS
    = 2: the next panel's columns take the group's earlier panels' updates at
    depth 128 j, its top rows the same in the U12 pre-update, and the columns
    beyond the group one depth-512 update) against pairs: the same steps to
    rounding, with one and two factorization groups; partially pivoted factors
    take pairs for the value 2 (bit-identical).  Four panels (one group) and six
    (a group, then two single panels)."""
    from paper_2502_16555_amd import _lib
    cfg = CASES["panels4"]() if case == "panels4" else \
        workloads.small_config(nx=5, nr=24, nth=28, kinds=("elastic", "excitation", "ionization"), E=1.2e4,
                               field_kind="rf")
    ops = oracle.build_operators(cfg)
    F0 = _state(ops, 13)
    out = {}
    for pairs, g, stat in ((1, 1, 1), (2, 1, 1), (2, 2, 1), (1, 1, 0), (2, 1, 0)):
        s = solver(cfg, precision=prec)
        s.set_tuning(_lib.TUNE_PANEL_PAIRS, pairs)
        s.set_tuning(_lib.TUNE_LU_STREAMS, g)
        s.set_tuning(_lib.TUNE_STATIC_PIVOTING, stat)
        assert s.get_tuning(_lib.TUNE_PANEL_PAIRS) == pairs
        F = cuda(torch, F0)
        for n in range(3):
            s.step(F, n * cfg["dt_s"])
        assert s.status()[0] == 0, (pairs, g, stat, s.status())
        out[(pairs, g, stat)] = F.cpu().numpy()
        s.close()
    assert np.array_equal(out[(2, 2, 1)], out[(2, 1, 1)])
    assert np.array_equal(out[(2, 1, 0)], out[(1, 1, 0)])
    close(out[(2, 1, 1)], out[(1, 1, 1)], 1e-13, f"groups of four vs pairs ({prec}, {case})")
    S_ref = F0
    for n in range(3):
        S_ref = S.step(ops, S_ref, n * cfg["dt_s"])
    close(out[(2, 1, 1)], S_ref, 1e-10, f"groups of four vs the oracle ({prec}, {case})")


def _grad_case():
    cfg = workloads.small_config(nx=5, nr=6, nth=4, kinds=("elastic", "excitation", "ionization"), E=6e3,
                                 field_kind="rf", n_bins=2)
    cfg["dt_s"] = 0.02 * cfg["T_rf_s"]
    return cfg


def test_cycle_gradient_matches_oracle_adjoint(torch):
    """autograd through bte_step / bte_adjoint_step with checkpoints (every 4 of
    10 steps, a ragged last segment) against the oracle's reverse-mode gradient."""
    from paper_2502_16555_amd.autograd import cycle_mean_density
    cfg = _grad_case()
    ops = oracle.build_operators(cfg)
    F0 = S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 1.0)
    n_steps, t0 = 10, 0.1 * cfg["T_rf_s"]
    g = np.random.default_rng(3).standard_normal(ops.nx)
    ref_s, ref_e0, ref_lam = S.cycle_mean_density_vjp(ops, F0, n_steps, g, t0=t0)
    ref_nbar = S.cycle_mean_density(ops, F0, n_steps, t0=t0)
    scal = torch.ones(ops.scal.shape, dtype=torch.float64, requires_grad=True)
    e0 = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    F0d = cuda(torch, F0).requires_grad_(True)
    nbar = cycle_mean_density(scal, e0, F0d, cfg, n_steps, every=4, precision="fp64", t0=t0)
    close(nbar.detach().cpu().numpy(), ref_nbar, 1e-10, "cycle-mean density")
    (torch.as_tensor(g, device="cuda:0") * nbar).sum().backward()
    close(scal.grad.numpy().ravel(), ref_s, 1e-9, "dL/dscal")
    close([float(e0.grad)], [ref_e0 * cfg["field"]["E0"]], 1e-9, "dL/de0_scale")
    close(F0d.grad.cpu().numpy(), ref_lam, 1e-9, "dL/dF0")


def test_cycle_gradient_matches_central_differences(torch):
    """Tied scalings (one per energy bin across the processes) and the RF
    amplitude, differentiated by the adjoint and by central differences of the
    GPU forward (h = 1e-6 relative): agreement to 1e-5."""
    from paper_2502_16555_amd.autograd import cycle_mean_density
    cfg = workloads.small_config(nx=7, nr=12, nth=16, kinds=("elastic", "excitation", "ionization"), E=8e3,
                                 field_kind="rf", n_bins=3)
    ops = oracle.build_operators(cfg)
    F0 = cuda(torch, S.initial_state(ops, workloads.density_profile(ops.xhat, 1e16), 1.0))
    n_steps, every = 24, 10
    w = torch.as_tensor(np.random.default_rng(4).uniform(0.5, 1.5, ops.nx), device="cuda:0")
    target = 1.05e16 * torch.as_tensor(workloads.density_profile(ops.xhat, 1.0), device="cuda:0")

    def loss(theta):
        scal = theta[:3].reshape(1, 3).expand(3, 3)   # bins tied across the processes
        nbar = cycle_mean_density(scal, theta[3], F0, cfg, n_steps, every=every)
        return (w * (nbar - target) ** 2).sum() / 1e32

    theta = torch.tensor([1.0, 1.1, 0.9, 1.0], dtype=torch.float64, requires_grad=True)
    L = loss(theta)
    L.backward()
    grad = theta.grad.numpy()
    h = 1e-6
    fd = np.zeros(4)
    with torch.no_grad():
        for j in range(4):
            tp = theta.detach().clone()
            tm = theta.detach().clone()
            tp[j] *= 1 + h
            tm[j] *= 1 - h
            fd[j] = float(loss(tp) - loss(tm)) / (2 * h * float(theta[j]))
    scale = np.abs(fd).max()
    assert np.abs(grad - fd).max() < 1e-5 * scale, (grad, fd)


def _ensemble_case(nx_per=(5, 9, 7)):
    """Three discharges of different size, pressure and amplitude (the batching
    form at test size): Nx = 5, 9, 7 by default; 0.3, 1, 2 Torr; E0 = 3e3, 8e3,
    1.2e4 V/m."""
    base = workloads.small_config(nx=nx_per[0], nr=10, nth=6, kinds=("elastic", "excitation", "ionization"),
                                  E=3e3, field_kind="rf", n_bins=2)
    nx_per = list(nx_per)
    p = [0.3, 1.0, 2.0]
    E0 = [3e3, 8e3, 1.2e4]
    ens = dict(base, n_discharges=3, nx_per=nx_per, n0_per=[workloads.n0_ideal_gas(q) for q in p], E0_per=E0)
    members = [dict(base, nx=nx_per[d], nx_per=[nx_per[d]], n0_m3=workloads.n0_ideal_gas(p[d]),
                    field=dict(base["field"], E0=E0[d])) for d in range(3)]
    return ens, members


@pytest.mark.parametrize("prec", ["fp64", "mixed_fp32"])
def test_ensemble_steps_match_oracle_per_discharge(torch, prec):
    cfg, members = _ensemble_case()
    ops = [oracle.build_operators(m) for m in members]
    F0 = [S.initial_state(o, workloads.density_profile(o.xhat, 1e16), 1.0) for o in ops]
    s = solver(cfg, precision=prec)
    assert s.nx_total == sum(cfg["nx_per"]) and s.n_discharges == 3
    close(s.xhat(), np.concatenate([o.xhat for o in ops]), 1e-15, "ensemble grid")
    F = cuda(torch, np.concatenate(F0))
    t0 = 0.2 * cfg["T_rf_s"]
    ref = list(F0)
    for k in range(3):
        s.step(F, t0 + k * cfg["dt_s"])
        ref = [S.step(o, r, t0 + k * cfg["dt_s"]) for o, r in zip(ops, ref)]
    assert s.status()[0] == 0
    got = F.cpu().numpy()
    o = 0
    for d, r in enumerate(ref):
        nx = r.shape[0]
        close(got[o:o + nx], r, 1e-10, f"discharge {d} ({prec})")
        o += nx
    mom = s.moments(F).cpu().numpy()
    ref_mom = np.concatenate([S.moments(op, r) for op, r in zip(ops, ref)], axis=1)
    close(mom[0], ref_mom[0], 1e-10, "ensemble n_e")
    close(mom[1], ref_mom[1], 1e-10, "ensemble mean energy")
    s.close()


def test_ensemble_adjoint_matches_oracle_per_discharge(torch):
    """Per-discharge E0 gradients and shared scaling gradients of an ensemble."""
    cfg, members = _ensemble_case()
    ops = [oracle.build_operators(m) for m in members]
    rng = np.random.default_rng(9)
    Fn = [rng.standard_normal((o.nx, o.nr, o.nth)) for o in ops]
    lam = [rng.standard_normal((o.nx, o.nr, o.nth)) for o in ops]
    t = 0.3 * cfg["T_rf_s"]
    s = solver(cfg)
    lam_d = cuda(torch, np.concatenate(lam))
    gs = torch.zeros(s.n_params, dtype=torch.float64, device="cuda:0")
    gE0 = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    s.adjoint_step(cuda(torch, np.concatenate(Fn)), t, lam_d, gs, gE0)
    ref_lam, ref_gs, ref_gE0 = [], np.zeros(s.n_params), np.zeros(3)
    for d, (o, f, l) in enumerate(zip(ops, Fn, lam)):
        ln, g, gE = S.adjoint_step(o, f, t, l)
        ref_lam.append(ln)
        ref_gs += g
        ref_gE0[d] = gE @ S.field_dE0(o, t)
    close(lam_d.cpu().numpy(), np.concatenate(ref_lam), 1e-10, "ensemble lambda")
    close(gs.cpu().numpy(), ref_gs, 1e-10, "ensemble dL/dscal")
    close(gE0.cpu().numpy(), ref_gE0, 1e-10, "ensemble dL/dE0")
    s.close()


@pytest.mark.parametrize("prec,groups", [("fp64", 1), ("mixed_fp32", 1), ("mixed_fp32", 2)])
def test_graph_replays_match_eager_steps(torch, prec, groups):
    """A captured run of 3 steps, replayed 3 times with eager work of the same
    handle in between, equals the eager steps bit for bit after every replay."""
    from paper_2502_16555_amd import _lib
    cfg = CASES["panels"]()
    ops = oracle.build_operators(cfg)
    s = solver(cfg, precision=prec)
    s.set_tuning(_lib.TUNE_LU_STREAMS, groups)
    F0 = _state(ops, 21)
    Fg = cuda(torch, F0)
    Fe = cuda(torch, F0)
    t0 = 0.1 * cfg["T_rf_s"]
    s.graph_capture(Fg, t0, 3)
    assert np.array_equal(Fg.cpu().numpy(), F0)          # capture runs nothing
    for rep in range(3):
        s.graph_launch()
        for k in range(3):
            s.step(Fe, t0 + k * cfg["dt_s"])
        s.moments(Fe)                                     # unrelated eager work between replays
        torch.cuda.synchronize()
        assert s.status()[0] == 0
        assert np.array_equal(Fg.cpu().numpy(), Fe.cpu().numpy()), f"replay {rep}"
    s.close()


def test_step_timing_levels(torch):
    """Timing level 1 times the LU launch groups and the phases; level 2 only
    the phases, with the steps' events read when the sums are asked for (more
    steps than the 64-step event ring included).  Neither changes the steps,
    and an unknown level is rejected."""
    cfg = CASES["panels"]()
    ops = oracle.build_operators(cfg)
    s = solver(cfg, precision="mixed_fp32")
    F0 = _state(ops, 31)
    Fa = cuda(torch, F0)
    Fb = cuda(torch, F0)
    t0 = 0.1 * cfg["T_rf_s"]
    for k in range(70):
        s.step(Fa, t0 + k * cfg["dt_s"])
    s.set_timing(True)
    for k in range(3):
        s.step(Fb, t0 + k * cfg["dt_s"])
    t1 = s.timing()
    assert t1[5] == 3 and t1[0] > 0 and t1[1] > 0 and t1[2] > 0 and t1[3] > 0
    s.set_timing(True, walls_only=True)
    for k in range(3, 70):
        s.step(Fb, t0 + k * cfg["dt_s"])
    t2 = s.timing()
    assert t2[5] == 67 and t2[0] == 0 and t2[1] == 0 and t2[3] == 0
    assert t2[2] > 0 and t2[4] > 0
    s.set_timing(False)
    torch.cuda.synchronize()
    assert s.status()[0] == 0
    assert np.array_equal(Fa.cpu().numpy(), Fb.cpu().numpy())
    with pytest.raises(Exception):
        _raw_set_timing(s, 3)
    s.close()


def _raw_set_timing(s, level):
    from paper_2502_16555_amd._lib import check
    check(s.lib.bte_set_timing(s.h, level), "bte_set_timing")


def test_autotuned_shapes_leave_results_unchanged(torch, tmp_path):
    """The autotuner picks launch shapes by timing; the steps after tuning equal
    the default-shape steps bit for bit, for FP64 and mixed precision."""
    from paper_2502_16555_amd import _lib
    from paper_2502_16555_amd.autotune import autotune
    cfg = CASES["panels4"]()
    ops = oracle.build_operators(cfg)
    F0 = _state(ops, 8)
    for prec in ("fp64", "mixed_fp32"):
        s = solver(cfg, precision=prec)
        Fa = cuda(torch, F0)
        for k in range(2):
            s.step(Fa, k * cfg["dt_s"])
        r = autotune(s, cuda(torch, F0), prec, steps=1, cache_path=str(tmp_path / "tune.json"))
        keys = {_lib.TUNE_LU_STREAMS, _lib.TUNE_UPDATE_KC, _lib.TUNE_FORM_XPB}
        if prec != "fp64":   # look-ahead of the statically pivoted panels
            keys.add(_lib.TUNE_LOOK_AHEAD)
        assert set(r["settings"]) == keys
        for k, v in r["settings"].items():
            assert s.get_tuning(k) == v
        # every candidate shape once more, explicitly
        for kc in ((16, 8) if prec == "fp64" else (32, 16)):
            for xpb in (1, 4, 16):
                s.set_tuning(_lib.TUNE_UPDATE_KC, kc)
                s.set_tuning(_lib.TUNE_FORM_XPB, xpb)
                Fb = cuda(torch, F0)
                for k in range(2):
                    s.step(Fb, k * cfg["dt_s"])
                assert s.status()[0] == 0
                assert np.array_equal(Fb.cpu().numpy(), Fa.cpu().numpy()), (prec, kc, xpb)
        s.close()


@pytest.mark.parametrize("fprec", ["fp64", "mixed_fp32", "fp16_factors"])
@pytest.mark.parametrize("case", ["ragged", "panels", "panels4"])
def test_krylov_vstep_matches_oracle(torch, case, fprec):
    """Batched GMRES with the field-binned preconditioner (bin factors in FP64
    or FP32) against the oracle's direct solves: the GMRES stop at
    ||r|| <= 1e-13 ||b|| bounds the error by cond * 1e-13."""
    cfg = CASES[case]()
    ops = oracle.build_operators(cfg)
    s = solver(cfg, precision="fp64")
    s.set_vsolver("gmres", n_bins=32, E_bound=1.5e4, restart=30, cycles=3, rtol=1e-13, factor_precision=fprec)
    F = _state(ops, 3)
    rng = np.random.default_rng(4)
    E = rng.uniform(-1.5e4, 1.5e4, size=ops.nx)
    E[0] = 1.6e4                       # outside the bound: the end bin
    Fg = cuda(torch, F)
    s.vstep(Fg, cuda(torch, E))
    code, iters, resid = s.status()
    assert code == 0 and 1 <= iters <= 90 and resid <= 1e-13, (code, iters, resid)
    close(Fg.cpu().numpy(), S.v_step(ops, F, E), 1e-10, f"{case} gmres {fprec}")
    s.close()


@pytest.mark.parametrize("case", ["ragged", "panels", "panels4", "wide_band", "reduced_nl"])
def test_banded_vstep_matches_oracle(torch, case):
    """The V step solved in the harmonic basis by the banded LU (half-bandwidth
    2 Nr - 1 of the l-major ordering, fill of the interchanges included) against
    the oracle's dense ordinate-space solves; switching back to the dense LU
    reproduces the dense path bit for bit."""
    cfg = BANDED_CASES[case]() if case in BANDED_CASES else CASES[case]()
    ops = oracle.build_operators(cfg)
    s = solver(cfg, precision="fp64")
    F = _state(ops, 3)
    rng = np.random.default_rng(5)
    E = rng.uniform(-2e4, 2e4, size=ops.nx)
    Fd = cuda(torch, F)
    s.vstep(Fd, cuda(torch, E))
    s.set_vsolver("banded")
    Fb = cuda(torch, F)
    s.vstep(Fb, cuda(torch, E))
    assert s.status()[0] == 0
    close(Fb.cpu().numpy(), S.v_step(ops, F, E), 1e-10, f"{case} banded")
    s.set_vsolver("lu")
    Fd2 = cuda(torch, F)
    s.vstep(Fd2, cuda(torch, E))
    assert np.array_equal(Fd2.cpu().numpy(), Fd.cpu().numpy())
    s.close()


def paper_grid_config(nx=100):
    """The grid of the paper's timed semi-implicit runs (table of the hybrid
    solver's performance): Nr = 64, Ntheta = 16, Nl = 3, Nx = 100, with the
    realistic RF physics of the other workloads."""
    cfg = workloads.config("C1")
    return dict(cfg, nx=nx, nx_per=[nx], ntheta=16, nl=3)


@pytest.mark.parametrize("prec,vsolver", [("fp64", "lu"), ("mixed_fp32", "lu"), ("fp64", "banded"),
                                          ("fp64", "hessenberg")])
def test_reduced_harmonics_at_paper_grid(torch, prec, vsolver):
    """Nl = 3 < Ntheta = 16 at the paper's timed grid (n = 1024 ordinate unknowns,
    Nr Nl = 192 harmonic ones): the dense LU of the ordinate systems and the
    exact reduction to the harmonic systems (I - P_O P_S + P_O (I - K)^-1 P_S)
    against the oracle's direct solves at sampled points, with the field at its
    RF peak, then five full steps against the oracle at every point."""
    cfg = paper_grid_config()
    ops = oracle.build_operators(cfg)
    s = solver(cfg, precision=prec)
    if vsolver != "lu":
        s.set_vsolver(vsolver)
    rng = np.random.default_rng(41)
    ne = workloads.density_profile(ops.xhat, cfg["ic"]["ne_peak"])
    F = S.initial_state(ops, ne, cfg["ic"]["Te_eV"]) * (1.0 + 0.1 * rng.standard_normal((ops.nx, ops.nr, ops.nth)))
    E = cfg["field"]["E0"] * (1.0 + 0.5 * ops.xhat)
    Fv = cuda(torch, F)
    s.vstep(Fv, cuda(torch, E))
    code, sweeps, resid = s.status()
    assert code == 0, (code, sweeps, resid)
    xs = [0, 1, 50, 98, 99]
    ref = S.v_step(ops, F, E, xs=xs)
    got = Fv.cpu().numpy()
    for x in xs:
        close(got[x], ref[x], 1e-10, f"V(dt) at x = {x}")
    F0 = S.initial_state(ops, ne, cfg["ic"]["Te_eV"])
    Fg, Fo = cuda(torch, F0), F0
    t0 = 0.2 * cfg["T_rf_s"]
    for k in range(5):
        s.step(Fg, t0 + k * ops.dt)
        Fo = S.step(ops, Fo, t0 + k * ops.dt)
    assert s.status()[0] == 0
    close(Fg.cpu().numpy(), Fo, 1e-10, "five steps")
    s.close()


@pytest.mark.parametrize("case", ["ragged", "panels", "panels4", "wide_band", "reduced_nl"])
def test_hessenberg_vstep_matches_oracle(torch, case):
    """The V step by the Hessenberg form of the harmonic-basis systems (one
    Householder reduction per discharge at setup, one Givens solve per point)
    against the oracle's dense ordinate-space solves, fields up to 2e4 V/m of
    either sign, ragged sizes, a wide band and Nl < Ntheta."""
    cfg = BANDED_CASES[case]() if case in BANDED_CASES else CASES[case]()
    ops = oracle.build_operators(cfg)
    s = solver(cfg, precision="fp64")
    s.set_vsolver("hessenberg")
    F = _state(ops, 3)
    rng = np.random.default_rng(5)
    E = rng.uniform(-2e4, 2e4, size=ops.nx)
    Fh = cuda(torch, F)
    s.vstep(Fh, cuda(torch, E))
    assert s.status()[0] == 0
    close(Fh.cpu().numpy(), S.v_step(ops, F, E), 1e-10, f"{case} hessenberg")
    s.close()


def test_hessenberg_steps_ensemble(torch):
    """Full RF steps of an uneven ensemble (three pressures: three Hessenberg
    forms) against the oracle per discharge."""
    cfg, members = _ensemble_case()
    ops = [oracle.build_operators(m) for m in members]
    F0 = [S.initial_state(o, workloads.density_profile(o.xhat, 1e16), 1.0) for o in ops]
    s = solver(cfg, precision="fp64")
    s.set_vsolver("hessenberg")
    t0 = 0.2 * cfg["T_rf_s"]
    F = cuda(torch, np.concatenate(F0))
    ref = list(F0)
    for k in range(3):
        s.step(F, t0 + k * cfg["dt_s"])
        ref = [S.step(o, r, t0 + k * cfg["dt_s"]) for o, r in zip(ops, ref)]
    assert s.status()[0] == 0
    got = F.cpu().numpy()
    o = 0
    for d, r in enumerate(ref):
        close(got[o:o + r.shape[0]], r, 1e-10, f"discharge {d} hessenberg")
        o += r.shape[0]
    s.close()


def test_banded_steps_ensemble_and_graph(torch):
    """Full RF steps of an uneven ensemble with the banded V solver against the
    oracle per discharge, and a captured run of them against the eager steps."""
    cfg, members = _ensemble_case()
    ops = [oracle.build_operators(m) for m in members]
    F0 = [S.initial_state(o, workloads.density_profile(o.xhat, 1e16), 1.0) for o in ops]
    s = solver(cfg, precision="mixed_fp32")
    s.set_vsolver("banded")
    t0 = 0.2 * cfg["T_rf_s"]
    F = cuda(torch, np.concatenate(F0))
    Fg = cuda(torch, np.concatenate(F0))
    ref = list(F0)
    for k in range(3):
        s.step(F, t0 + k * cfg["dt_s"])
        ref = [S.step(o, r, t0 + k * cfg["dt_s"]) for o, r in zip(ops, ref)]
    assert s.status()[0] == 0
    got = F.cpu().numpy()
    o = 0
    for d, r in enumerate(ref):
        close(got[o:o + r.shape[0]], r, 1e-10, f"discharge {d} banded")
        o += r.shape[0]
    s.graph_capture(Fg, t0, 3)
    s.graph_launch()
    torch.cuda.synchronize()
    assert s.status()[0] == 0
    assert np.array_equal(Fg.cpu().numpy(), got)
    s.close()


def test_krylov_steps_ensemble_and_graph(torch):
    """Full RF steps of an uneven ensemble with the Krylov V solver against the
    oracle per discharge, and a captured run of them against the eager steps."""
    cfg, members = _ensemble_case()
    ops = [oracle.build_operators(m) for m in members]
    F0 = [S.initial_state(o, workloads.density_profile(o.xhat, 1e16), 1.0) for o in ops]
    s = solver(cfg, precision="mixed_fp32")
    s.set_vsolver("gmres", n_bins=32, restart=30, cycles=2, rtol=1e-13)
    t0 = 0.2 * cfg["T_rf_s"]
    F = cuda(torch, np.concatenate(F0))
    Fg = cuda(torch, np.concatenate(F0))
    ref = list(F0)
    for k in range(3):
        s.step(F, t0 + k * cfg["dt_s"])
        ref = [S.step(o, r, t0 + k * cfg["dt_s"]) for o, r in zip(ops, ref)]
    assert s.status()[0] == 0
    got = F.cpu().numpy()
    o = 0
    for d, r in enumerate(ref):
        close(got[o:o + r.shape[0]], r, 1e-10, f"discharge {d} gmres")
        o += r.shape[0]
    s.graph_capture(Fg, t0, 3)
    s.graph_launch()
    torch.cuda.synchronize()
    assert s.status()[0] == 0
    assert np.array_equal(Fg.cpu().numpy(), got)
    s.close()


def test_c3_ensemble_at_size(torch):
    """The batching workload at its full size: 64 discharges (Nx ~ U{32..200},
    7255 points, 0.1-2 Torr, E0 ~ U[1e3, 1e4] V/m, seed 1) in the same
    launches, mixed precision, as the benchmark runs it.  Inputs are built on
    the oracle side (CGL nodes and the projected Maxwellian of every
    discharge).  Checked against the oracle per discharge:
    * the smallest discharge over two full steps, every point;
    * a median-size and the largest discharge: X(dt/2) and the field at every
      point, V(dt) at three points (both walls and the middle), each solved by
      the oracle alone, from the oracle's own half-step and field."""
    from oracle import basis as OB
    cfg = workloads.config("C3")
    nx_per = list(cfg["nx_per"])
    nd = len(nx_per)
    offs = np.concatenate([[0], np.cumsum(nx_per)]).astype(int)
    order = np.argsort(nx_per, kind="stable")
    d_small, d_mid, d_big = int(order[0]), int(order[nd // 2]), int(order[-1])

    def member(d):
        return dict(cfg, n_discharges=1, nx=nx_per[d], nx_per=[nx_per[d]], n0_m3=cfg["n0_per"][d],
                    n0_per=[cfg["n0_per"][d]], E0_per=[cfg["E0_per"][d]], field=dict(cfg["field"], E0=cfg["E0_per"][d]))

    ops = {d: oracle.build_operators(member(d)) for d in (d_small, d_mid, d_big)}
    ne = np.concatenate([workloads.density_profile(OB.cgl_nodes(nx_per[d]), cfg["ic"]["ne_peak"]) for d in range(nd)])
    F0 = S.initial_state(ops[d_small], ne, cfg["ic"]["Te_eV"])       # same speed basis for every discharge
    s = solver(cfg, precision="mixed_fp32")
    assert s.nx_total == offs[-1] == 7255 and s.n_discharges == 64
    close(s.xhat()[offs[d_big]:offs[d_big + 1]], ops[d_big].xhat, 1e-15, "grid of the largest discharge")
    dt, t0 = cfg["dt_s"], 0.2 * cfg["T_rf_s"]
    Fg = cuda(torch, F0)
    for k in range(2):
        s.step(Fg, t0 + k * dt)
    code, sweeps, resid = s.status()
    assert code == 0 and resid <= 1e-14, (code, sweeps, resid)
    got = Fg.cpu().numpy()
    assert np.isfinite(got).all()
    sl = slice(offs[d_small], offs[d_small + 1])
    ref = F0[sl]
    for k in range(2):
        ref = S.step(ops[d_small], ref, t0 + k * dt)
    close(got[sl], ref, 1e-10, f"discharge {d_small} (Nx={nx_per[d_small]}) after two steps")
    # sub-steps of the larger discharges
    Fx = cuda(torch, F0)
    s.xstep(Fx)
    gx = Fx.cpu().numpy()
    E = torch.empty(s.nx_total, dtype=torch.float64, device="cuda:0")
    t = 0.25 * cfg["T_rf_s"] - 0.5 * dt                               # field at its RF peak
    s.field(Fx, t, E)
    gE = E.cpu().numpy()
    Fv_in, E_in = gx.copy(), gE.copy()
    refs = {}
    for d in (d_mid, d_big):
        sl = slice(offs[d], offs[d + 1])
        Fh = S.x_half_step(ops[d], F0[sl])
        close(gx[sl], Fh, 1e-11, f"X(dt/2) of discharge {d} (Nx={nx_per[d]})")
        Eo = S.field_half(ops[d], t, Fh)
        close(gE[sl], Eo, 1e-13, f"field of discharge {d}")
        Fv_in[sl], E_in[sl] = Fh, Eo
        xs = [0, nx_per[d] // 2, nx_per[d] - 1]
        refs[d] = (xs, S.v_step(ops[d], Fh, Eo, xs=xs))
    Fv = cuda(torch, Fv_in)
    s.vstep(Fv, cuda(torch, E_in))
    code, sweeps, resid = s.status()
    assert code == 0 and resid <= 1e-14, (code, sweeps, resid)
    gv = Fv.cpu().numpy()
    for d, (xs, rv) in refs.items():
        for x in xs:
            close(gv[offs[d] + x], rv[x], 1e-10, f"V(dt) of discharge {d} at x = {x}")
    s.close()


@pytest.mark.slow
def test_c4_cycle_gradient_against_central_differences(torch):
    """The differentiation workload at its size: Nx = 128, Nr = 64, Ntheta = 32,
    one RF cycle of 1000 steps, checkpoints every 50, nine parameters (eight
    energy-bin scalings tied across the three processes, and the RF amplitude).
    The loss is the weighted misfit of the cycle-mean density to the profile of
    the same solver at seeded +-10% perturbed parameters.  The adjoint gradient
    (autograd through bte_adjoint_step) against central differences of the
    forward run with h = 1e-6 relative, on the amplitude and two bins (the bulk
    and the ionization tail): agreement to 1e-5.  The steps are the mixed form
    (FP32 factors refined to the FP64 backward error), which keeps the eight
    cycles of the test within two minutes."""
    import time
    from paper_2502_16555_amd import Solver
    from paper_2502_16555_amd.autograd import cycle_mean_density
    cfg = workloads.config("C4")
    nb = cfg["n_bins"]
    s = Solver(cfg, precision="mixed_fp32")
    ne = workloads.density_profile(s.xhat(), cfg["ic"]["ne_peak"])
    F0 = s.initial_state(cuda(torch, ne), cfg["ic"]["Te_eV"])
    s.close()
    n_steps, every = cfg["n_steps"], cfg["checkpoint_every"]
    w = torch.as_tensor(np.random.default_rng(4).uniform(0.5, 1.5, cfg["nx"]), device="cuda:0")

    def nbar_of(theta):
        scal = theta[:nb].reshape(1, nb).expand(len(cfg["processes"]), nb)
        return cycle_mean_density(scal, theta[nb], F0, cfg, n_steps, every=every, precision="mixed_fp32")

    theta_t = torch.as_tensor(workloads.perturbed_scalings(nb + 1, seed=2), dtype=torch.float64)
    with torch.no_grad():
        target = nbar_of(theta_t)

    def loss(theta):
        return (w * (nbar_of(theta) - target) ** 2).sum() / 1e30

    theta = torch.ones(nb + 1, dtype=torch.float64, requires_grad=True)
    t = time.perf_counter()
    L = loss(theta)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t
    t = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t_rev = time.perf_counter() - t
    grad = theta.grad.numpy()
    h = 1e-6
    fd = {}
    with torch.no_grad():
        for j in (nb, 0, 5):
            tp, tm = theta.detach().clone(), theta.detach().clone()
            tp[j] *= 1 + h
            tm[j] *= 1 - h
            fd[j] = float(loss(tp) - loss(tm)) / (2 * h)
    print(f"C4 cycle: forward {t_fwd:.1f} s, reverse {t_rev:.1f} s, ratio {(t_fwd + t_rev) / t_fwd:.2f}; "
          + ", ".join(f"theta[{j}]: adjoint {grad[j]:.6e} fd {fd[j]:.6e}" for j in fd))
    for j, f in fd.items():
        assert abs(grad[j] - f) <= 1e-5 * abs(f), (j, grad[j], f)
