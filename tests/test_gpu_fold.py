"""GPU parity of the mirror fold of the dense contractions.

On a mesh symmetric about the equator the dense paths run over block pairs
(a block and its mirror image) with even and odd mode sums; the result is
the same sums reordered.  Each case is solved folded and unfolded
(MPOLE_FOLD=0 at plan creation) and both are checked against the oracle:
potential per cell, angular moments and edge moments, at 1e-12 (FP64) and
1e-6 (BF16 x3, FP16 x2); the two FP64 solves agree to 1e-13 of max|Phi|.
Cases: a coarsened production-like mesh, an odd theta count (the equator
row is its own mirror), 4 x 4 blocks that straddle the equator (their own
mirrors), and a GenASiS mesh (blocks of up to a whole shell)."""
import numpy as np
import pytest

from paper_2602_02507_amd import workloads as wl
from test_gpu_parity import check_against_oracle

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "bf16x3": 1e-6, "fp16x2": 1e-6}


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def fold_meshes():
    a = wl.production_mesh(12, nr=96, ntheta=32, nphi=64)
    a.shell_class, a.class_block = wl.production_merge(96, 32, 64, inner_shells=16, polar_rows=4)
    b = wl.production_mesh(9, nr=40, ntheta=33, nphi=24, merged=False)
    c = wl.production_mesh(10, nr=50, ntheta=36, nphi=72)
    c.shell_class, c.class_block = wl.production_merge(50, 36, 72, inner_shells=12, polar_rows=4)
    from oracle import genasis as og
    g = og.mesh(32, 0.25, 1.5, dims=3)
    d = wl.Mesh(g["r_edges"], g["theta_edges"], g["phi_edges"], 8, g["shell_class"], g["class_block"])
    return [("coarsened", a), ("odd_theta", b), ("straddling", c), ("genasis", d)]


CASES = fold_meshes()


@pytest.mark.parametrize("precision", ["fp64", "bf16x3", "fp16x2"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fold_matches_unfolded_and_oracle(case, precision, monkeypatch):
    torch = _torch()
    from paper_2602_02507_amd import mpole
    name, m = case
    rho_h = wl.production_density(m, seed=31) * (1.0 + 0.3 * wl.random_density(32, m.shape))
    rho = torch.from_numpy(np.ascontiguousarray(rho_h)).cuda()
    print("%s: %d x %d x %d lmax %d %s" % (name, m.nr, m.ntheta, m.nphi, m.lmax, precision), flush=True)
    folded = mpole.Plan.from_mesh(m, precision=precision)
    assert folded.folded
    got_f = {k: v.cpu().numpy() for k, v in folded.solve(rho).items()}
    monkeypatch.setenv("MPOLE_FOLD", "0")
    plain = mpole.Plan.from_mesh(m, precision=precision)
    assert not plain.folded
    got_u = {k: v.cpu().numpy() for k, v in plain.solve(rho).items()}
    torch.cuda.synchronize()
    check_against_oracle(m, rho_h, got_f, tol=TOL[precision])
    check_against_oracle(m, rho_h, got_u, tol=TOL[precision])
    if precision == "fp64":
        d = np.abs(got_f["phi"] - got_u["phi"]).max() / np.abs(got_u["phi"]).max()
        assert d <= 1e-13, d


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_fold_signed_density(precision):
    """A signed density with odd and even parts of equal size (no mirror
    symmetry in the source itself) on the folded production-like mesh."""
    torch = _torch()
    from paper_2602_02507_amd import mpole
    m = CASES[0][1]
    rho_h = wl.random_density(33, m.shape, positive=False)
    plan = mpole.Plan.from_mesh(m, precision=precision)
    assert plan.folded
    got = {k: v.cpu().numpy() for k, v in plan.solve(torch.from_numpy(rho_h).cuda()).items()}
    check_against_oracle(m, rho_h, got, tol=TOL[precision], signed=True)
