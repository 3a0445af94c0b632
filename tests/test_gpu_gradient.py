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


@pytest.mark.parametrize("shape", [(37, 11, 23), (5, 1, 9), (1, 6, 1), (3, 4, 2), (64, 33, 65), (17, 9, 128),
                                   (16, 7, 129), (9, 5, 64)])
def test_gradient_random_mesh(shape):
    nr, nt, npf = shape
    m = wl.random_mesh(sum(shape), nr, nt, npf, 4, r0=0.01)
    phi = wl.random_density(sum(shape) + 1, m.shape, positive=False)
    check(m, phi)


@pytest.mark.parametrize("nphi", [16, 130])
def test_gradient_open_phi_range(nphi):
    m = wl.random_mesh(9, 20, 10, nphi, 4, r0=0.0)
    m.phi_edges = np.linspace(0.0, 3.0, nphi + 1)      # does not close the circle: one-sided seam
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


SRC_CASES = [((37, 11, 23), (True, True, True)), ((5, 1, 9), (True, False, True)), ((3, 4, 2), (False, False, False)),
             ((64, 33, 65), (True, True, False)), ((1, 6, 1), (False, True, False)),
             ((17, 9, 128), (True, True, True)), ((16, 7, 129), (False, True, True))]


@pytest.mark.parametrize("shape,vel", SRC_CASES, ids=[str(c[0]) for c in SRC_CASES])
def test_gravity_sources_match_oracle(shape, vel):
    """-rho grad Phi and -rho v . grad Phi in one pass (missing velocity
    components count as zero) against the oracle, on ragged meshes with
    single-cell dimensions; a null output is not written."""
    torch = _torch()
    from paper_2602_02507_amd import mpole
    nr, nt, npf = shape
    seed = sum(shape) + 7
    m = wl.random_mesh(seed, nr, nt, npf, 4, r0=0.01)
    phi = wl.random_density(seed + 1, m.shape, positive=False)
    rho = wl.random_density(seed + 2, m.shape)
    v = [wl.random_density(seed + 3 + k, m.shape, positive=False) if on else None for k, on in enumerate(vel)]
    plan = mpole.Plan.from_mesh(m, precision="fp64")
    cu = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()
    got = [g.cpu().numpy() for g in plan.gravity_sources(cu(phi), cu(rho), tuple(cu(x) for x in v))]
    want = oracle.gravity_sources(m.r_edges, m.theta_edges, m.phi_edges, phi, rho, *v)
    for name, g, w in zip(("s_r", "s_theta", "s_phi", "s_energy"), got, want):
        scale = max(np.abs(w).max(), 1e-300)
        assert np.abs(g - w).max() <= TOL * scale or np.abs(w).max() == 0 and np.abs(g).max() == 0, name
    # outputs left out are not written
    keep = torch.full(m.shape, 7.0, dtype=torch.float64, device="cuda")
    out = (None, keep, None, None)
    plan.gravity_sources(cu(phi), cu(rho), tuple(cu(x) for x in v), out=out)
    torch.cuda.synchronize()
    assert np.abs(keep.cpu().numpy() - want[1]).max() <= TOL * max(np.abs(want[1]).max(), 1e-300) or \
        np.abs(want[1]).max() == 0


def test_gradient_and_sources_replay_from_a_graph():
    """Both launches captured in one HIP graph (the entry points promise
    capture): every replay, with eager work on the same buffers between
    replays, equals the eager results bitwise."""
    torch = _torch()
    from paper_2602_02507_amd import mpole
    m = wl.random_mesh(41, 19, 12, 128, 4, r0=0.01)
    plan = mpole.Plan.from_mesh(m, precision="fp64")
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    phi = cu(wl.random_density(42, m.shape, positive=False))
    rho = cu(wl.random_density(43, m.shape))
    vel = tuple(cu(wl.random_density(44 + k, m.shape, positive=False)) for k in range(3))
    grads = tuple(torch.empty_like(phi) for _ in range(3))
    srcs = tuple(torch.empty_like(phi) for _ in range(4))
    plan.gradient(phi, *grads)
    plan.gravity_sources(phi, rho, vel, out=srcs)
    torch.cuda.synchronize()
    eager = [t.clone() for t in grads + srcs]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.gradient(phi, *grads)
            plan.gravity_sources(phi, rho, vel, out=srcs)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(3):
        for t in grads + srcs:
            t.fill_(7.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert all(torch.equal(t, e) for t, e in zip(grads + srcs, eager))
