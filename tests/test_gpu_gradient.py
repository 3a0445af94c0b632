"""GPU parity of the centred-difference gradient (Sec. 3 source terms)
against the oracle: ragged non-uniform meshes with and without a closed phi
circle, single-cell dimensions, and the production mesh in full on the
potential the library itself computed."""
import numpy as np
import pytest

import oracle
from paper_2602_02507_amd import workloads as wl

pytestmark = pytest.mark.gpu
TOL = 1e-13


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def check(mesh, phi_h):
    torch = _torch()
    from paper_2602_02507_amd import mpole
    plan = mpole.Plan.from_mesh(mesh, precision="fp64")
    got = [g.cpu().numpy() for g in plan.gradient(torch.from_numpy(np.ascontiguousarray(phi_h)).cuda())]
    want = oracle.gradient(mesh.r_edges, mesh.theta_edges, mesh.phi_edges, phi_h)
    for name, g, w in zip(("r", "theta", "phi"), got, want):
        scale = max(np.abs(w).max(), 1e-300)
        err = np.abs(g - w).max() / scale
        assert err <= TOL, (name, err)


@pytest.mark.parametrize("shape", [(37, 11, 23), (5, 1, 9), (1, 6, 1), (3, 4, 2), (64, 33, 65)])
def test_gradient_random_mesh(shape):
    nr, nt, npf = shape
    m = wl.random_mesh(sum(shape), nr, nt, npf, 4, r0=0.01)
    phi = wl.random_density(sum(shape) + 1, m.shape, positive=False)
    check(m, phi)


def test_gradient_open_phi_range():
    m = wl.random_mesh(9, 20, 10, 16, 4, r0=0.0)
    m.phi_edges = np.linspace(0.0, 3.0, 17)      # does not close the circle: one-sided seam
    phi = wl.random_density(10, m.shape, positive=False)
    check(m, phi)


def test_gradient_of_production_potential():
    torch = _torch()
    from paper_2602_02507_amd import mpole
    m, rho = wl.workload("production")
    plan = mpole.Plan.from_mesh(m, precision="fp64")
    phi = plan.solve(torch.from_numpy(rho).cuda(), ang=False, interior=False, exterior=False)["phi"]
    got = [g.cpu().numpy() for g in plan.gradient(phi)]
    want = oracle.gradient(m.r_edges, m.theta_edges, m.phi_edges, phi.cpu().numpy())
    for g, w in zip(got, want):
        assert np.abs(g - w).max() <= TOL * np.abs(w).max()
    # physics: outside the core (r > 0.1) the monopole dominates, so the
    # radial derivative is positive (near the origin the l = 1 part of the 1 %
    # perturbation, a uniform field, can win and flip it)
    rc = 0.5 * (m.r_edges[1:] + m.r_edges[:-1])
    outer = (rc > 0.1) & (np.arange(m.nr) < m.nr - 1)
    assert (got[0][outer] > 0).all()
