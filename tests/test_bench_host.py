"""Host-side checks of the benchmark's roofline arithmetic (no GPU): the
whole-solve bound is the sum over phases of max(executed flops / peak,
algorithmic bytes / HBM peak), worked here by hand for the production mesh
at lmax 32."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


class _Plan:
    """The attributes solve_bound reads, for the production mesh: 512 shells x
    128 x 256 cells, lmax 32, 4 x 4 blocks (2048 per shell) in 32 shells and
    29696 blocks per shell in the other 480."""
    nr, shape, lmax = 512, (512, 128, 256), 32

    def __init__(self, separable):
        cells = 512 * 128 * 256
        nam = 33 * 33
        if separable:
            f = 2.0 * 512 * 128 * 256 * 65
            self._work = (f, f, 16.0 * cells)
        else:
            f = 2.0 * (32 * 2048 + 480 * 29696) * nam
            self._work = (f, f, 16.0 * cells + 8.0 * (2048 + 29696) * nam)

    def work(self):
        return self._work


def test_dense_bf16x3_bound_by_hand():
    b = _bench()
    r = b.solve_bound(_Plan(False), "bf16x3", 0.6)
    cells, nam = 512 * 128 * 256, 1089
    blocks = 32 * 2048 + 480 * 29696
    flops = 2.0 * blocks * nam
    table = 6.0 * (2048 + 29696) * nam
    pack = (8.0 * cells + 6.0 * blocks) / 8e12
    contraction = max(6 * flops / 2.5e15, (6.0 * blocks + table) / 8e12)
    expand = max(6 * flops / 2.5e15, (table + 8.0 * cells) / 8e12)
    scan = 8.0 * nam * (512 + 3 * 513) / 8e12
    want = (pack + contraction + scan + expand) * 1e3
    assert r["bound_ms"] == pytest.approx(want, rel=1e-12)
    assert r["frac"] == pytest.approx(want / 0.6, rel=1e-12)
    # both contractions are MFMA-bound at six products: 74.9 us each
    assert r["phase_bound_ms"]["moment"] == pytest.approx(6 * flops / 2.5e15 * 1e3, rel=1e-12)
    assert 0.17 < r["bound_ms"] < 0.19


def test_fp64_bound_uses_the_f64_peak():
    b = _bench()
    r = b.solve_bound(_Plan(False), "fp64", 1.0)
    flops = 2.0 * (32 * 2048 + 480 * 29696) * 1089
    assert r["phase_bound_ms"]["moment"] == pytest.approx(flops / 78.6e12 * 1e3, rel=1e-12)


def test_separable_bound_is_hbm_bound():
    b = _bench()
    r = b.solve_bound(_Plan(True), "bf16x3sep", 0.2)
    cells = 512 * 128 * 256
    inter = 8.0 * 65 * 512 * 128
    assert r["phase_bound_ms"]["phi_analysis"] == pytest.approx((8.0 * cells + inter) / 8e12 * 1e3, rel=1e-12)
    assert r["phase_bound_ms"]["phi_synthesis"] == pytest.approx((8.0 * cells + inter) / 8e12 * 1e3, rel=1e-12)
    assert set(r["phase_bound_ms"]) == {"phi_analysis", "theta_analysis", "scan", "theta_synthesis", "phi_synthesis"}
