"""Python binding of the C-ABI: device memory and streams come from torch, every
step of the computation runs in libbte.so.  Argument marshalling only."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import check


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _Config:
    """bte_config plus the host arrays it points into (kept alive)."""

    def __init__(self, cfg: dict, precision=None, field_mode=None, refine_max_iter=0, refine_rtol=0.0,
                 x_fp32=False):
        self.keep = []
        procs = cfg["processes"]
        P = (_lib.bte_process * len(procs))()
        for i, p in enumerate(procs):
            e = np.ascontiguousarray(p["eps_eV"], dtype=np.float64)
            s = np.ascontiguousarray(p["sigma_m2"], dtype=np.float64)
            self.keep += [e, s]
            P[i] = _lib.bte_process(int(p["kind"]), float(p["threshold_eV"]), float(p["mass_ratio"]), len(e),
                                    _dptr(e), _dptr(s))
        self.keep.append(P)
        nb = int(cfg.get("n_bins", 1))
        edges = np.ascontiguousarray(cfg.get("bin_edges_eV", np.linspace(0, cfg["eps_max_eV"], nb + 1)),
                                     dtype=np.float64)
        scal = cfg.get("scal")
        scal = None if scal is None else np.ascontiguousarray(scal, dtype=np.float64).ravel()
        nd = int(cfg.get("n_discharges", 1))
        nx_per = np.ascontiguousarray(cfg.get("nx_per", [cfg["nx"]]), dtype=np.int32)
        n0 = np.ascontiguousarray(cfg.get("n0_per", [cfg["n0_m3"]]), dtype=np.float64)
        fld = cfg["field"]
        E0 = np.ascontiguousarray(cfg.get("E0_per", [fld.get("E0", 0.0)]), dtype=np.float64)
        if nd == 1:
            n0 = np.array([cfg["n0_m3"]], dtype=np.float64)
            E0 = np.array([fld.get("E0", 0.0)], dtype=np.float64)
            nx_per = np.array([cfg["nx"]], dtype=np.int32)
        self.keep += [edges, nx_per, n0, E0]
        if scal is not None:
            self.keep.append(scal)
        prec = _lib.PRECISION[precision or cfg.get("precision", "fp64")]
        fm = _lib.FIELD[field_mode or fld["kind"]]
        self.c = _lib.bte_config(
            nx=int(cfg["nx"]), nr=int(cfg["nr"]), ntheta=int(cfg["ntheta"]), nl=int(cfg["nl"]),
            v_bc=_lib.VBC[cfg.get("v_bc", "natural")], L_m=float(cfg["L_m"]), eps_max_eV=float(cfg["eps_max_eV"]),
            T0_K=float(cfg["T0_K"]), dt_s=float(cfg["dt_s"]), n_proc=len(procs), proc=P, n_bins=nb,
            bin_edges_eV=_dptr(edges), scal=_dptr(scal) if scal is not None else None, precision=prec,
            refine_max_iter=int(refine_max_iter), refine_rtol=float(refine_rtol), field_mode=fm,
            field_freq_hz=float(fld.get("freq_hz", 0.0)), field_a1=float(fld.get("a1", 0.0)),
            poisson_V0=float(fld.get("V0", 0.0)), n_discharges=nd, nx_per=nx_per.ctypes.data_as(C.POINTER(C.c_int32)),
            n0_per=_dptr(n0), E0_per=_dptr(E0), x_fp32=1 if x_fp32 else 0)


def make_config(cfg: dict, **kw) -> _Config:
    return _Config(cfg, **kw)


def host_operator(cfg: dict, which: int, size: int) -> np.ndarray:
    """Operator ``which`` (see bte_get_operator) assembled on the host, no device needed."""
    lib = _lib.load()
    c = _Config(cfg)
    out = np.zeros(size, dtype=np.float64)
    check(lib.bte_host_operator(C.byref(c.c), which, _dptr(out)), "bte_host_operator")
    return out


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.dtype.is_floating_point and t.is_contiguous(), "need a contiguous CUDA tensor"
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Solver:
    """One setup of the operators (bte_setup_operators) and the step calls on it."""

    def __init__(self, cfg: dict, device: int = 0, precision: str | None = None, field_mode: str | None = None,
                 refine_max_iter: int = 0, refine_rtol: float = 0.0, x_fp32: bool = False):
        self.lib = _lib.load()
        self.cfg = cfg
        self.device = device
        self._c = _Config(cfg, precision=precision, field_mode=field_mode, refine_max_iter=refine_max_iter,
                          refine_rtol=refine_rtol, x_fp32=x_fp32)
        h = C.c_void_p()
        check(self.lib.bte_setup_operators(C.byref(self._c.c), device, C.byref(h)), "bte_setup_operators")
        self.h = h
        info = _lib.bte_info()
        check(self.lib.bte_get_info(self.h, C.byref(info)), "bte_get_info")
        self.info = info
        self.nx_total, self.n = info.nx_total, info.n
        self.nr, self.nth = int(cfg["nr"]), int(cfg["ntheta"])
        self.n_params = info.n_params
        self.n_discharges = info.n_discharges

    # ---- helpers -------------------------------------------------------------------
    def new_state(self):
        import torch
        return torch.zeros((self.nx_total, self.nr, self.nth), dtype=torch.float64, device=f"cuda:{self.device}")

    def xhat(self) -> np.ndarray:
        out = np.zeros(self.nx_total)
        check(self.lib.bte_get_operator(self.h, 6, _dptr(out)), "bte_get_operator")
        return out

    def operator(self, which: int, size: int) -> np.ndarray:
        out = np.zeros(size)
        check(self.lib.bte_get_operator(self.h, which, _dptr(out)), "bte_get_operator")
        return out

    @staticmethod
    def _field(E_half=None, ni=None):
        return _lib.bte_field(_ptr(E_half), _ptr(ni))

    # ---- the C-ABI calls ----------------------------------------------------------------
    def step(self, F, t, E_half=None, ni=None, stream=None):
        check(self.lib.bte_step(self.h, _ptr(F), float(t), self._field(E_half, ni), _stream(stream)), "bte_step")

    def set_vsolver(self, kind: str = "lu", n_bins: int = 32, E_bound: float = 0.0, bin_scale: float = 0.0,
                    restart: int = 20, cycles: int = 2, rtol: float = 1e-12, factor_precision: str = "mixed_fp32"):
        """Select the velocity-space solver: "lu" (batched factorization), "gmres"
        (restarted GMRES with the field-binned preconditioner, factored here),
        "banded" (banded LU of the harmonic-basis systems) or "hessenberg" (the
        harmonic-basis systems in Hessenberg form, reduced here)."""
        k = {"lu": _lib.VSOLVER_LU, "gmres": _lib.VSOLVER_GMRES, "banded": _lib.VSOLVER_BANDED,
             "hessenberg": _lib.VSOLVER_HESSENBERG}[kind]
        check(self.lib.bte_set_vsolver(self.h, k, int(n_bins), float(E_bound), float(bin_scale), int(restart),
                                       int(cycles), float(rtol), _lib.PRECISION[factor_precision]),
              "bte_set_vsolver")

    def graph_capture(self, F, t0, n_steps, E_half=None, ni=None):
        """Capture n_steps steps of F from t0 into the handle's HIP graph (nothing runs)."""
        check(self.lib.bte_graph_capture(self.h, _ptr(F), float(t0), int(n_steps), self._field(E_half, ni)),
              "bte_graph_capture")

    def graph_launch(self, stream=None):
        check(self.lib.bte_graph_launch(self.h, _stream(stream)), "bte_graph_launch")

    def xstep(self, F, stream=None):
        check(self.lib.bte_xstep(self.h, _ptr(F), _stream(stream)), "bte_xstep")

    def xstep_T(self, F, stream=None):
        check(self.lib.bte_xstep_T(self.h, _ptr(F), _stream(stream)), "bte_xstep_T")

    def ion_step(self, F, ni_in, ni_out, t, stream=None):
        """Heavies' update of the hybrid model (bte_ion_step): ni_out <- n_i^{n+1}."""
        check(self.lib.bte_ion_step(self.h, _ptr(F), _ptr(ni_in), _ptr(ni_out), float(t), _stream(stream)),
              "bte_ion_step")

    def ion_step_noalloc(self, F, ni_in, ni_out, t, stream=None):
        """bte_ion_step with its scratch in the library's fixed device array (no allocation)."""
        check(self.lib.bte_ion_step_noalloc(self.h, _ptr(F), _ptr(ni_in), _ptr(ni_out), float(t), _stream(stream)),
              "bte_ion_step_noalloc")

    def hybrid_step(self, F, ni, t, stream=None):
        """One hybrid step (bte_hybrid_step): ions, then electrons; F and ni in place."""
        check(self.lib.bte_hybrid_step(self.h, _ptr(F), _ptr(ni), float(t), _stream(stream)), "bte_hybrid_step")

    def implicit_step(self, F, t, ni=None, newton_rtol=0.0, max_newton=0, gmres_rtol=0.0, restart=0,
                      max_gmres=0, precond=0, stream=None, raise_on_noconv=True) -> dict:
        """Fully implicit step (bte_implicit_step), F in place; returns the iteration counts
        and residual norms.  Zero options take the library defaults."""
        opts = _lib.bte_implicit_opts(float(newton_rtol), int(max_newton), float(gmres_rtol), int(restart),
                                      int(max_gmres), int(precond))
        st = _lib.bte_implicit_stats()
        code = self.lib.bte_implicit_step(self.h, _ptr(F), _ptr(ni), float(t), opts, C.byref(st), _stream(stream))
        if code != _lib.BTE_OK and (raise_on_noconv or code != _lib.BTE_ENOCONV):
            check(code, "bte_implicit_step")
        return {"status": code, "newton_iters": st.newton_iters, "gmres_iters": st.gmres_iters,
                "residual": st.residual, "residual0": st.residual0}

    def vstep(self, F, E, stream=None):
        check(self.lib.bte_vstep(self.h, _ptr(F), _ptr(E), _stream(stream)), "bte_vstep")

    def field(self, F_half, t, E_out, E_half=None, ni=None, stream=None):
        check(self.lib.bte_field_eval(self.h, _ptr(F_half), float(t), self._field(E_half, ni), _ptr(E_out),
                                      _stream(stream)), "bte_field_eval")

    def moments(self, F, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty((3, self.nx_total), dtype=torch.float64, device=F.device)
        check(self.lib.bte_moments(self.h, _ptr(F), _ptr(out), _stream(stream)), "bte_moments")
        return out

    def moments_vjp(self, F, gbar, lam, stream=None):
        check(self.lib.bte_moments_vjp(self.h, _ptr(F), _ptr(gbar), _ptr(lam), _stream(stream)), "bte_moments_vjp")

    def initial_state(self, ne, Te_eV, F=None, stream=None):
        if F is None:
            F = self.new_state()
        check(self.lib.bte_initial_maxwellian(self.h, _ptr(ne), float(Te_eV), _ptr(F), _stream(stream)),
              "bte_initial_maxwellian")
        return F

    def adjoint_step(self, F_n, t, lam, grad_scal, grad_E0=None, grad_E=None, E_half=None, stream=None):
        check(self.lib.bte_adjoint_step(self.h, _ptr(F_n), float(t), self._field(E_half, None), _ptr(lam),
                                        _ptr(grad_scal), _ptr(grad_E0), _ptr(grad_E), _stream(stream)),
              "bte_adjoint_step")

    def factor_export(self, E, x: int):
        """Factors (npad x npad, FP64) and pivots of point x after factoring with field E."""
        npad = ((self.n + 127) // 128) * 128
        lu = np.zeros((npad, npad))
        piv = np.zeros(npad, dtype=np.int32)
        check(self.lib.bte_factor_export(self.h, _ptr(E), int(x), _dptr(lu), piv.ctypes.data_as(C.POINTER(C.c_int32))),
              "bte_factor_export")
        return lu.T.copy(), piv   # stored column-major

    def status(self):
        it = C.c_int32()
        r = C.c_double()
        code = self.lib.bte_get_status(self.h, C.byref(it), C.byref(r))
        return code, it.value, r.value

    def set_refine(self, max_iter: int = 0, rtol: float = 0.0):
        """Refinement sweeps and stop of the mixed-precision V step (bte_set_refine)."""
        check(self.lib.bte_set_refine(self.h, int(max_iter), float(rtol)), "bte_set_refine")

    def set_timing(self, on, walls_only: bool = False):
        """Kernel-level timing of step() (on: events around every LU launch
        group too; walls_only: around the step's phases only)."""
        check(self.lib.bte_set_timing(self.h, (2 if walls_only else 1) if on else 0), "bte_set_timing")

    def timing(self):
        out = (C.c_double * 6)()
        check(self.lib.bte_get_timing(self.h, out), "bte_get_timing")
        return list(out)

    def set_tuning(self, key: int, value: int):
        check(self.lib.bte_set_tuning(self.h, int(key), int(value)), "bte_set_tuning")

    def get_tuning(self, key: int) -> int:
        v = C.c_int32()
        check(self.lib.bte_get_tuning(self.h, int(key), C.byref(v)), "bte_get_tuning")
        return v.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.bte_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
