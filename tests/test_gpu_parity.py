"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle,
element by element, on the same seeded inputs.

Bars (FP64 path):
  * potential: |dPhi| <= 1e-12 |Phi| per cell (positive densities; Phi < 0),
    or <= 1e-12 max|Phi| for signed densities;
  * angular moments: |dA[i][n]| <= 1e-12 x (sum over the shell of |dOmega S| x
    max|kernel|), i.e. relative to the size of the terms being summed;
  * edge moments: |dM[e][n]| <= 1e-12 x sum_i |J_l(i)| x (terms of shell i)
    x kernel bound, the size of the increments being summed;
  * kernel tables: |dT| <= 1e-13 x sqrt((2l+1)/4pi) (the bound of P~_l^m).
"""
import zlib

import numpy as np
import pytest

import oracle
from paper_2602_02507_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def gpu_solve(mesh, rho, precision="fp64"):
    torch = _torch()
    from paper_2602_02507_amd import mpole
    plan = mpole.Plan.from_mesh(mesh, precision=precision)
    r = torch.from_numpy(np.ascontiguousarray(rho)).to("cuda")
    out = plan.solve(r)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}, plan


def check_against_oracle(mesh, rho, got, tol=1e-12, signed=False):
    ref = oracle.solve(rho=rho, **mesh.oracle_kwargs())
    # potential
    d = np.abs(got["phi"] - ref["phi"])
    if signed:
        assert d.max() <= tol * np.abs(ref["phi"]).max(), d.max()
    else:
        rel = d / np.abs(ref["phi"])
        assert rel.max() <= tol, (rel.max(), np.unravel_index(rel.argmax(), rel.shape))
    # angular moments, relative to the size of the summed terms of each shell:
    # sum_cells 4 pi |G| dOmega |rho| times the kernel bound sqrt((2l+1)/4pi)
    th, ph = mesh.theta_edges, mesh.phi_edges
    dom = (np.cos(th[:-1]) - np.cos(th[1:]))[:, None] * np.diff(ph)[None, :]
    terms = 4 * np.pi * abs(mesh.G) * (np.abs(rho) * dom[None]).reshape(mesh.nr, -1).sum(1)
    da = np.abs(got["ang"] - ref["ang"]) / np.maximum(terms[:, None] * lbound(mesh.lmax)[None, :], 1e-300)
    assert da.max() <= tol, (da.max(), np.unravel_index(da.argmax(), da.shape))
    # edge moments, relative to the summed size of their increments, bounded by
    # |J_l(i)| x (terms of shell i) x kernel bound, with J the shell integrals
    ls = np.concatenate([[l] * (2 * l + 1) for l in range(mesh.lmax + 1)])
    rad = [oracle.radial(mesh.lmax, mesh.r_edges[i], mesh.r_edges[i + 1]) for i in range(mesh.nr)]
    for key, idx in (("interior", 0), ("exterior", 1)):
        J = np.abs(np.array([r[idx] for r in rad]))[:, ls]            # [nr][nAM]
        scale = (J * terms[:, None] * lbound(mesh.lmax)[None, :]).sum(0)
        de = np.abs(got[key] - ref[key]) / np.maximum(scale, 1e-300)[None, :]
        assert de.max() <= tol, (key, de.max(), np.unravel_index(de.argmax(), de.shape))
    return ref


def block_table(mesh, cls):
    T = oracle.angular_tables(mesh.theta_edges, mesh.phi_edges, mesh.lmax)
    dom = T["domega"].reshape(-1)
    A = T["akern"].reshape(dom.size, -1)
    if mesh.class_block is None:
        return A
    cb = mesh.class_block[cls]
    nb = cb.max() + 1
    num = np.zeros((nb, A.shape[1]))
    np.add.at(num, cb, dom[:, None] * A)
    den = np.bincount(cb, weights=dom)
    return num / den[:, None]


def lbound(lmax):
    ls = np.concatenate([[l] * (2 * l + 1) for l in range(lmax + 1)])
    return np.sqrt((2 * ls + 1) / (4 * np.pi))


@pytest.mark.parametrize("merged", [False, True])
def test_kernel_tables_match_oracle(merged):
    torch = _torch()
    from paper_2602_02507_amd import mpole
    m = wl.random_mesh(21, 5, 11, 14, 12, r0=0.01)
    if merged:
        m.shell_class, m.class_block = wl.random_merge(22, 5, 11, 14)
    plan = mpole.Plan.from_mesh(m)
    torch.cuda.synchronize()
    ncls = 1 if m.class_block is None else m.class_block.shape[0]
    for c in range(ncls):
        got = plan.table(c)
        ref = block_table(m, c)
        assert got.shape == ref.shape
        err = np.abs(got - ref) / lbound(m.lmax)[None, :]
        assert err.max() <= 1e-13, (c, err.max())


CASES = [
    # name, nr, ntheta, nphi, lmax, r0, merged
    ("tiny", 3, 2, 3, 2, 0.1, False),
    ("ragged", 70, 13, 26, 10, 0.02, False),
    ("ragged_merged", 130, 12, 24, 16, 0.01, True),
    ("origin_shell", 33, 8, 16, 6, 0.0, False),
    ("monopole_only", 17, 5, 7, 0, 0.05, False),
    ("single_angle", 9, 1, 1, 4, 0.1, False),
    ("axisymmetric", 20, 16, 1, 8, 0.1, False),
    ("high_l", 40, 24, 48, 32, 0.05, True),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_solve_matches_oracle(case):
    name, nr, nt, npf, L, r0, merged = case
    seed = zlib.crc32(name.encode()) % 1000
    m = wl.random_mesh(seed, nr, nt, npf, L, r0=r0)
    if merged:
        m.shell_class, m.class_block = wl.random_merge(seed + 1, nr, nt, npf)
    rho = wl.random_density(seed + 2, m.shape)
    got, _ = gpu_solve(m, rho)
    check_against_oracle(m, rho, got)


def test_signed_density_and_G():
    m = wl.random_mesh(31, 50, 10, 20, 8, r0=0.05)
    m.G = 6.674e-8
    rho = wl.random_density(32, m.shape, positive=False)
    got, _ = gpu_solve(m, rho)
    check_against_oracle(m, rho, got, signed=True)


def test_spheroid_workload_full():
    """Homogeneous oblate spheroid (a1 = 1, a3 = 0.5) on 64 x 32 x 64, lmax 8."""
    import closed_forms as cf
    m, rho = wl.workload("spheroid")
    got, _ = gpu_solve(m, rho)
    check_against_oracle(m, rho, got)
    r = 0.5 * (m.r_edges[1:] + m.r_edges[:-1])
    th = 0.5 * (m.theta_edges[1:] + m.theta_edges[:-1])
    R, T = np.meshgrid(r, th, indexing="ij")
    exact = cf.spheroid_potential(R * np.sin(T), R * np.cos(T), 1.0, 0.5, 1.0)
    rel = np.abs(got["phi"] - exact[:, :, None]) / np.abs(exact[:, :, None])
    assert rel.max() < 1e-2


def test_production_workload_full():
    """512 log shells x 128 x 256, lmax 16, coarsened near origin and poles."""
    m, rho = wl.workload("production")
    got, _ = gpu_solve(m, rho)
    check_against_oracle(m, rho, got)


def test_optional_outputs_and_determinism():
    torch = _torch()
    from paper_2602_02507_amd import mpole
    m = wl.production_mesh(8, nr=96, ntheta=32, nphi=64)
    rho = wl.production_density(m)
    plan = mpole.Plan.from_mesh(m)
    r = torch.from_numpy(rho).cuda()
    a = plan.solve(r)
    b = plan.solve(r)
    only_phi = plan.empty_outputs(ang=False, interior=False, exterior=False)
    plan.solve_into(r, **only_phi)
    only_ang = plan.empty_outputs(phi=False, interior=False, exterior=False)
    plan.solve_into(r, **only_ang)
    torch.cuda.synchronize()
    for k in a:
        assert torch.equal(a[k], b[k]), k
    assert torch.equal(only_phi["phi"], a["phi"])
    assert torch.equal(only_ang["ang"], a["ang"])


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_phase_timing_and_merged_block_broadcast(precision):
    """Per-phase timing reports every phase of a dense solve; on a coarsened
    mesh (merged blocks in theta bands) the broadcast phase runs and every
    member cell of a merged block carries its block's value; without merged
    blocks the broadcast phase has no launch."""
    torch = _torch()
    from paper_2602_02507_amd import mpole
    for merged in (True, False):
        mesh = wl.production_mesh(6, nr=40, ntheta=32, nphi=64, merged=merged)
        rho = torch.from_numpy(wl.production_density(mesh, seed=11)).cuda()
        plan = mpole.Plan.from_mesh(mesh, precision=precision)
        plan.set_timing(True)
        plan.phase_ms()
        phi = plan.solve(rho)["phi"]
        ph = plan.phase_ms()
        plan.set_timing(False)
        assert set(ph) == set(mpole.PHASES)
        for k in ("pack", "moment", "reduce", "scan", "expand"):
            assert ph[k][1] == 1 and ph[k][0] > 0, (k, ph[k])
        assert ph["bcast"][1] == (1 if merged else 0), ph["bcast"]
        if merged:
            got = phi.cpu().numpy()
            blocks = np.asarray(mesh.class_block)
            cls = np.asarray(mesh.shell_class)
            for i in (0, 5, 39):
                ids = blocks[cls[i]].reshape(mesh.ntheta, mesh.nphi)
                row = got[i]
                for b in np.unique(ids)[:200]:
                    v = row[ids == b]
                    assert np.all(v == v[0]), (i, b)
