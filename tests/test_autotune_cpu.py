"""Host logic of the launch-shape autotuner (no GPU: a fake handle and cost)."""
import json

from paper_2502_16555_amd import _lib
from paper_2502_16555_amd import autotune as AT


class FakeSolver:
    def __init__(self, n=2048, nx_total=300):
        self.n, self.nx_total = n, nx_total
        self.settings = {}
        self.log = []

    def set_tuning(self, k, v):
        self.settings[k] = v
        self.log.append((k, v))


def test_coordinate_descent_finds_separable_minimum():
    s = FakeSolver()
    cost = {_lib.TUNE_LU_STREAMS: {1: 3.0, 2: 1.0}, _lib.TUNE_UPDATE_KC: {32: 0.5, 16: 2.0},
            _lib.TUNE_FORM_XPB: {16: 1.0, 4: 4.0, 8: 0.25, 32: 2.0}, _lib.TUNE_LOOK_AHEAD: {0: 0.5, 1: 0.25}}

    def measure():
        return sum(cost[k][s.settings[k]] for k in cost)

    best, c, trials = AT.coordinate_descent(s.set_tuning, measure, AT.candidates("mixed_fp32"))
    assert best == {_lib.TUNE_LU_STREAMS: 2, _lib.TUNE_UPDATE_KC: 32, _lib.TUNE_FORM_XPB: 8,
                    _lib.TUNE_LOOK_AHEAD: 1}
    assert c == measure() == 2.0
    assert len(trials) == 1 + 1 + 1 + 3 + 1
    assert s.settings == best          # the handle is left at the best settings


def test_size_classes_and_cache(tmp_path):
    assert AT.size_class(2048, 256, "mixed_fp32") == "n2048-x256-mixed_fp32"
    assert AT.size_class(2048, 7255, "mixed_fp32") == "n2048-x8192-mixed_fp32"
    assert AT.candidates("mixed_bf16")[_lib.TUNE_UPDATE_KC] == [32]
    path = tmp_path / "tune.json"
    s = FakeSolver()
    calls = []

    def measure():
        calls.append(dict(s.settings))
        return 1.0 + 0.1 * s.settings[_lib.TUNE_FORM_XPB] / 16

    r = AT.autotune(s, None, "fp64", cache_path=str(path), measure=measure)
    assert not r["cached"] and r["settings"][_lib.TUNE_FORM_XPB] == 4
    stored = json.loads(path.read_text())
    assert r["class"] in stored
    s2 = FakeSolver()
    r2 = AT.autotune(s2, None, "fp64", cache_path=str(path), measure=None)
    assert r2["cached"] and s2.settings == r["settings"]
