"""The allocation-free ion step (bte_ion_step_noalloc) against bte_ion_step,
through the C-ABI: two calls in a row on different handles, the second with a
smaller input, each bit for bit equal to the allocating entry point (same
kernels, same order of operations); the smaller one also against the oracle;
and an input beyond the fixed scratch rejected as an argument error."""
import numpy as np
import pytest

import oracle
import workloads
from oracle import hybrid as H
from oracle import semi_implicit as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2502_16555_amd import _lib
    _lib.load()
    return _t


def _poisson_cfg(nx_per, nr=10, nth=6):
    base = workloads.small_config(nx=nx_per[0], nr=nr, nth=nth, kinds=("elastic", "excitation", "ionization"),
                                  E=5e3, field_kind="rf", n_bins=2)
    p = [0.3, 1.0, 2.0] * ((len(nx_per) + 2) // 3)
    nd = len(nx_per)
    n0 = [workloads.n0_ideal_gas(q) for q in p[:nd]]
    cfg = dict(base, n_discharges=nd, nx_per=list(nx_per), n0_per=n0, n0_m3=n0[0], E0_per=[5e3] * nd)
    cfg["field"] = {"kind": "poisson", "V0": 150.0, "freq_hz": workloads.RF_FREQ_HZ}
    return cfg


def _inputs(cfg, seed):
    """Projected Maxwellian states times a density, and an ion density that
    differs from n_e (oracle-side inputs on the CGL nodes of every discharge)."""
    from oracle import basis as OB
    member = dict(cfg, n_discharges=1, nx=cfg["nx_per"][0], nx_per=[cfg["nx_per"][0]], n0_m3=cfg["n0_per"][0],
                  n0_per=cfg["n0_per"][:1], E0_per=cfg["E0_per"][:1])
    ops = oracle.build_operators(member)
    xh = np.concatenate([OB.cgl_nodes(nx) for nx in cfg["nx_per"]])
    ne = workloads.density_profile(xh, 1e16)
    F = S.initial_state(ops, ne, 2.0)
    rng = np.random.default_rng(seed)
    ni = 0.8 * ne + 3e14 * (1.0 + xh) * rng.uniform(0.9, 1.1, size=xh.shape)
    return ops, F, ni


def test_ion_step_noalloc_equals_ion_step(torch):
    from paper_2502_16555_amd import Solver
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")
    t = 0.3 * workloads.rf_period_s()
    for k, nx_per in enumerate([(130, 256, 9), (37,)]):     # second call: a smaller input
        cfg = _poisson_cfg(nx_per)
        ops, F, ni = _inputs(cfg, 5 + k)
        s = Solver(cfg)
        Fd, nid = dev(F), dev(ni)
        ref = torch.empty_like(nid)
        got = torch.full_like(nid, float("nan"))
        s.ion_step(Fd, nid, ref, t)
        s.ion_step_noalloc(Fd, nid, got, t)
        torch.cuda.synchronize()
        assert s.status()[0] == 0
        assert torch.equal(got, ref), f"call {k} (Nx = {nx_per}): differs from bte_ion_step"
        if len(nx_per) == 1:
            want = H.ion_step(ops, ni, F, t)
            err = np.abs(got.cpu().numpy() - want).max() / np.abs(want).max()
            assert err < 1e-10, err
        s.close()


def test_ion_step_noalloc_rejects_inputs_beyond_its_scratch(torch):
    """40 discharges of Nx = 230 need 40 * 230^2 + 3 * 9200 doubles of scratch,
    more than the fixed 2^21: an argument error, and the handle stays usable."""
    from paper_2502_16555_amd import Solver, _lib
    cfg = _poisson_cfg([230] * 40, nr=6, nth=2)
    need = sum(nx * nx for nx in cfg["nx_per"]) + 3 * sum(cfg["nx_per"])
    assert need > _lib.ION_SCRATCH_DOUBLES
    s = Solver(cfg)
    F = s.new_state()
    ni = torch.full((s.nx_total,), 1e15, dtype=torch.float64, device="cuda:0")
    out = torch.empty_like(ni)
    code = s.lib.bte_ion_step_noalloc(s.h, F.data_ptr(), ni.data_ptr(), out.data_ptr(), 0.0, None)
    assert code == _lib.BTE_EINVAL
    s.ion_step(F, ni, out, 0.0)
    torch.cuda.synchronize()
    assert s.status()[0] == 0 and bool(torch.isfinite(out).all())
    s.close()
