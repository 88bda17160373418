"""Seeded synthetic workloads for the 1D-space electron BTE step.

This module only *describes inputs*: grid sizes, physical parameters, tabulated
cross sections, seeded random draws and synthetic states.  It holds none of the
solver's arithmetic (no basis functions, no operators, no time stepping), so
that both the FP64 CPU oracle and the GPU library can consume the same inputs
without sharing any code of the method.

Workloads (all use the paper's RF glow-discharge parameters, "Glow discharge"
section, Table of modeling parameters: L = 2.54 cm, T0 = 300 K, 13.56 MHz):

* ``C0`` tiny plain FP64 case: Nx=16, Nr=16, Ntheta=8, elastic-only constant
  momentum-transfer cross section, uniform E = 100 V/m, 100 steps.
* ``C1`` realistic RF case: Nx=64, Nr=64, Ntheta=32, argon-like analytic cross
  sections (elastic, one excitation, ionization), E = E0 sin(2 pi t)(1+x/2).
* ``C2`` the same physics at Nx=256 (the throughput workload).
* ``C3`` uneven ensemble of 64 discharges (Nx in 32..200, 0.1..2 Torr).
* ``C4`` differentiation case at Nx=128 with 8 energy bins per process.

The analytic cross sections stand in for the LXCat argon data the paper uses,
which are not available here.
"""
from __future__ import annotations

import math

import numpy as np

# --- physical constants (CODATA 2018 exact / recommended values) -------------
K_BOLTZMANN = 1.380649e-23          # J/K
TORR_PA = 101325.0 / 760.0          # Pa per Torr
RF_FREQ_HZ = 13.56e6                # driving frequency (paper: 13.56 MHz)
GAP_M = 2.54e-2                     # electrode gap L
GAS_T_K = 300.0                     # background gas temperature
MASS_RATIO = 1.36e-5                # electron / argon mass ratio used by the workloads

KIND_ELASTIC = 0
KIND_EXCITATION = 1
KIND_IONIZATION = 2


def n0_ideal_gas(p_torr: float, T_K: float = GAS_T_K) -> float:
    """Neutral number density [m^-3] from the ideal-gas law n0 = p / (k_B T)."""
    return p_torr * TORR_PA / (K_BOLTZMANN * T_K)


def rf_period_s() -> float:
    return 1.0 / RF_FREQ_HZ


# --- tabulated cross sections (inputs; piecewise linear in energy) -----------
def _table_grid(eps_max_eV: float, threshold_eV: float, d_eps: float) -> np.ndarray:
    hi = eps_max_eV * 1.2 + 1.0
    if threshold_eV > 0.0:
        pts = np.arange(threshold_eV, hi + d_eps, d_eps)
        return np.concatenate([[0.0], pts])
    return np.arange(0.0, hi + d_eps, d_eps)


def sigma_table_constant(value_m2: float, eps_max_eV: float):
    eps = np.array([0.0, eps_max_eV * 1.2 + 1.0])
    return eps, np.full_like(eps, value_m2)


def sigma_table_elastic_argon_like(eps_max_eV: float, d_eps: float = 0.05):
    """sigma_el(eps) = 7e-20 (1 + eps / 10 eV)^-1/2 m^2, tabulated."""
    eps = _table_grid(eps_max_eV, 0.0, d_eps)
    return eps, 7e-20 / np.sqrt(1.0 + eps / 10.0)


def sigma_table_lotz(threshold_eV: float, peak_m2: float, eps_max_eV: float, d_eps: float = 0.05):
    """Lotz-type form sigma = s * (I/eps) ln(eps/I) for eps > I, zero below.

    The form peaks at eps = e*I with value s/e; ``s`` is chosen so the peak equals
    ``peak_m2``.  Tabulated with the threshold as an exact breakpoint.
    """
    eps = _table_grid(eps_max_eV, threshold_eV, d_eps)
    s = peak_m2 * math.e
    sig = np.zeros_like(eps)
    above = eps > threshold_eV
    sig[above] = s * (threshold_eV / eps[above]) * np.log(eps[above] / threshold_eV)
    return eps, sig


def _proc(kind, threshold_eV, eps, sig, mass_ratio=MASS_RATIO):
    return {"kind": int(kind), "threshold_eV": float(threshold_eV), "mass_ratio": float(mass_ratio),
            "eps_eV": np.asarray(eps, dtype=np.float64), "sigma_m2": np.asarray(sig, dtype=np.float64)}


def argon_like_processes(eps_max_eV: float):
    e1, s1 = sigma_table_elastic_argon_like(eps_max_eV)
    e2, s2 = sigma_table_lotz(11.55, 1.5e-21, eps_max_eV)
    e3, s3 = sigma_table_lotz(15.76, 3.0e-20, eps_max_eV)
    return [_proc(KIND_ELASTIC, 0.0, e1, s1), _proc(KIND_EXCITATION, 11.55, e2, s2),
            _proc(KIND_IONIZATION, 15.76, e3, s3)]


# --- workloads ----------------------------------------------------------------
def draw_E0(seed: int = 0) -> float:
    """E0 ~ U[1e3, 1e4] V/m from numpy's PCG64 generator."""
    rng = np.random.default_rng(seed)
    return float(1e3 + 9e3 * rng.uniform())


def _base(nx, nr, nth, procs, E0, field_kind, n_steps, precision="fp64", p_torr=1.0, n_bins=1):
    eps_max = 30.0
    return {
        "nx": nx, "nr": nr, "ntheta": nth, "nl": nth,
        "L_m": GAP_M, "eps_max_eV": eps_max, "v_bc": "zero_vmax", "n0_m3": n0_ideal_gas(p_torr), "T0_K": GAS_T_K,
        "T_rf_s": rf_period_s(), "dt_s": 1e-3 * rf_period_s(), "n_steps": n_steps,
        "processes": procs,
        "n_bins": n_bins, "bin_edges_eV": np.linspace(0.0, eps_max, n_bins + 1),
        "field": {"kind": field_kind, "E0": E0, "a1": 0.5, "freq_hz": RF_FREQ_HZ},
        "ic": {"ne_peak": 1e16, "Te_eV": 1.0},
        "precision": precision,
        "n_discharges": 1, "nx_per": [nx], "n0_per": [n0_ideal_gas(p_torr)], "E0_per": [E0],
    }


def config(name: str) -> dict:
    """Return the named workload as a plain dict (see module docstring)."""
    if name == "C0":
        e, s = sigma_table_constant(1e-19, 30.0)
        return _base(16, 16, 8, [_proc(KIND_ELASTIC, 0.0, e, s)], 100.0, "const", 100)
    if name in ("C1", "C2"):
        nx = 64 if name == "C1" else 256
        return _base(nx, 64, 32, argon_like_processes(30.0), draw_E0(0), "rf", 1000,
                     precision="fp64" if name == "C1" else "mixed_fp32")
    if name == "C3":
        return ensemble_config(64, seed=1)
    if name == "C4":
        cfg = _base(128, 64, 32, argon_like_processes(30.0), draw_E0(0), "rf", 1000, n_bins=8)
        cfg["checkpoint_every"] = 50
        return cfg
    raise KeyError(name)


def small_config(nx=8, nr=8, nth=4, kinds=("elastic",), E=2e3, field_kind="const", n_bins=1,
                 n_steps=4, dt_frac=1e-3) -> dict:
    """Reduced-size variant of the realistic physics for fast tests."""
    procs = argon_like_processes(30.0)
    sel = {"elastic": procs[0], "excitation": procs[1], "ionization": procs[2]}
    cfg = _base(nx, nr, nth, [sel[k] for k in kinds], E, field_kind, n_steps, n_bins=n_bins)
    cfg["dt_s"] = dt_frac * rf_period_s()
    return cfg


def ensemble_config(n_discharges: int = 64, seed: int = 1, nx_lo: int = 32, nx_hi: int = 200) -> dict:
    """Uneven ensemble: Nx ~ U{nx_lo..nx_hi}, p log-uniform in [0.1, 2] Torr, E0 ~ U[1e3, 1e4]."""
    rng = np.random.default_rng(seed)
    nx_per = rng.integers(nx_lo, nx_hi + 1, size=n_discharges).tolist()
    p = np.exp(rng.uniform(math.log(0.1), math.log(2.0), size=n_discharges))
    E0 = (1e3 + 9e3 * rng.uniform(size=n_discharges)).tolist()
    cfg = _base(nx_per[0], 64, 32, argon_like_processes(30.0), E0[0], "rf", 1000, precision="mixed_fp32")
    cfg.update({"n_discharges": n_discharges, "nx_per": nx_per,
                "n0_per": [n0_ideal_gas(float(pi)) for pi in p], "E0_per": E0, "p_torr_per": p.tolist()})
    return cfg


def perturbed_scalings(n_params: int, seed: int = 2, rel: float = 0.1) -> np.ndarray:
    """Target parameters theta*(1 + rel*U[-1,1]) around theta = 1 (differentiation workload)."""
    rng = np.random.default_rng(seed)
    return 1.0 + rel * rng.uniform(-1.0, 1.0, size=n_params)


def synthetic_state(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded random FP64 array (used as a generic right-hand side / cotangent)."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(size=shape)


def density_profile(xhat: np.ndarray, ne_peak: float) -> np.ndarray:
    """Initial density n_e(x) = ne_peak (1 - xhat^2) on the caller's grid."""
    return ne_peak * (1.0 - np.asarray(xhat) ** 2)
