"""Host parity of the library's GenASiS mesh builder (mpole_genasis_shape /
mpole_genasis_build, Sec. 2.1) with the oracle's: edges, block maps,
classes and coarsening factors are bit-identical; parameters are validated;
the arrays feed plan creation directly.  No GPU needed (no HIP call)."""
import numpy as np
import pytest

from oracle import genasis as og
from paper_2602_02507_amd import mpole
from paper_2602_02507_amd import workloads as wl

PARAMS = [
    (32, 1.0, 1.0, 3, 0.0, 0.0),
    (64, 0.25, 3.68, 3, 0.0, 0.0),
    (128, 0.25, 3.68, 2, 0.0, 0.0),
    (192, 16.0, 5.9, 3, 0.0, 0.0),
    (256, 0.25, 3.68, 3, 0.0, 0.0),
    (48, 0.25, 3.68, 3, 0.0, 0.0),      # 48 = 16 x 3: groups capped at 16 / 32
    (24, 2.0, 2.0, 3, 1.5, 0.0),        # another core ratio (N_core = 16)
    (40, 1.0, 1.5, 3, 0.0, 0.2),        # wider coarsening width
    (64, 1.0, 2.0, 1, 0.0, 0.0),        # 1D: no angular cells to group
    (20, 1.0, 2.3, 2, 0.0, 0.0),        # 2.3 * 20 = 45.99999...: the guard keeps 46 shells
]


@pytest.mark.parametrize("p", PARAMS, ids=[str(p) for p in PARAMS])
def test_library_mesh_is_bit_identical_to_oracle(p):
    nt, rc, rr, dims, ratio, drc = p
    got = mpole.genasis_mesh(nt, rc, rr, dims=dims, core_ratio=ratio, dr_coarsen=drc)
    ref = og.mesh(nt, rc, rr, dims=dims, core_ratio=ratio if ratio > 0 else og.PAPER_CORE_RATIO, dr_coarsen=drc)
    assert got["ncore"] == ref["ncore"]
    for k in ("r_edges", "theta_edges", "phi_edges", "shell_class", "class_block", "c_theta", "c_phi"):
        assert got[k].shape == ref[k].shape, k
        assert (got[k] == ref[k]).all(), k


def test_guarded_shell_count():
    assert mpole.genasis_mesh(20, 1.0, 2.3, dims=2)["r_edges"].size - 1 == 46


@pytest.mark.parametrize("kw", [
    dict(dims=0), dict(dims=4), dict(ntheta=0), dict(ntheta=70000), dict(r_core=0.0), dict(r_core=float("nan")),
    dict(r_radial=-1.0), dict(core_ratio=-1.0), dict(dr_coarsen=-0.1), dict(core_ratio=1e9),
])
def test_invalid_parameters_rejected(kw):
    args = dict(ntheta=32, r_core=1.0, r_radial=2.0, dims=3)
    args.update(kw)
    with pytest.raises(mpole.MpoleError) as e:
        mpole.genasis_mesh(**args)
    assert e.value.code == 1


def test_outer_radius_overflow_is_a_range_error():
    with pytest.raises(mpole.MpoleError) as e:
        mpole.genasis_mesh(4, 1.0, 250000.0, dims=1, core_ratio=4.0)   # N_core = 1: doubling per shell
    assert e.value.code == 2


def test_genasis_mesh_feeds_plan_creation():
    g = mpole.genasis_mesh(32, 0.25, 3.68, dims=3)
    m = wl.Mesh(g["r_edges"], g["theta_edges"], g["phi_edges"], 12, g["shell_class"], g["class_block"])
    sizes = {}
    for prec in ("fp64", "bf16x3", "fp64sep"):
        p = mpole.HostPlan.from_mesh(m, precision=prec)
        assert p.nmodes == 169
        sizes[prec] = p.workspace_bytes
    # the separable path keeps no per-class kernel tables
    assert sizes["fp64sep"] < sizes["fp64"]
