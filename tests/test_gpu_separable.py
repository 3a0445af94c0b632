"""GPU parity of the separable FP64 path (phi transform + per-m theta
transforms; the same sums as the dense contractions, reordered) against the
oracle, to the FP64 bar of 1e-12: ragged and degenerate meshes, arbitrary
(non-rectangular) block maps, the spheroid, the production mesh in full, and
lmax 64 on the 256 x 512 angular mesh; plus graph replay."""
import numpy as np
import pytest

import oracle
from paper_2602_02507_amd import workloads as wl

pytestmark = pytest.mark.gpu
TOL = 1e-12


def run(mesh, rho, precision="fp64sep"):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_02507_amd import mpole
    plan = mpole.Plan.from_mesh(mesh, precision=precision)
    out = plan.solve(torch.from_numpy(np.ascontiguousarray(rho)).cuda())
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def compare(mesh, rho, got, ref):
    rel = np.max(np.abs(got["phi"] - ref["phi"]) / np.max(np.abs(ref["phi"])))
    dom = (np.cos(mesh.theta_edges[:-1]) - np.cos(mesh.theta_edges[1:]))[:, None] * np.diff(mesh.phi_edges)[None, :]
    terms = 4 * np.pi * abs(mesh.G) * (np.abs(rho) * dom[None]).reshape(mesh.nr, -1).sum(1)
    ls = np.concatenate([[l] * (2 * l + 1) for l in range(mesh.lmax + 1)])
    bound = np.sqrt((2 * ls + 1) / (4 * np.pi))
    ang = np.max(np.abs(got["ang"] - ref["ang"]) / np.maximum(terms[:, None] * bound[None, :], 1e-300))
    return rel, ang


CASES = [
    ("ragged", 70, 13, 26, 10, 0.02, False),
    ("ragged_merged", 130, 12, 24, 16, 0.01, True),
    ("origin_shell", 33, 8, 16, 6, 0.0, True),
    ("high_l", 40, 24, 48, 32, 0.05, True),
    ("thin", 5, 1, 1, 0, 0.1, False),
    ("one_theta", 9, 1, 12, 4, 0.1, False),
    ("one_phi", 9, 10, 1, 5, 0.1, False),
    # 128 and 256 theta rows (the whole-K theta transforms), shells past the
    # last 64-shell tile
    ("theta128_l8", 70, 128, 8, 8, 0.02, False),
    ("theta128_l16", 70, 128, 8, 16, 0.02, True),
    ("theta128_l32", 70, 128, 8, 32, 0.0, True),
    ("theta256_l12", 37, 256, 8, 12, 0.02, True),
    ("theta256_l3", 130, 256, 4, 3, 0.0, False),
    ("theta128_l35", 20, 128, 4, 35, 0.02, False),   # the most k steps of the synthesis form
    ("theta128_l47", 20, 128, 4, 47, 0.02, True),    # the most column blocks of the analysis form
    # 64-row, 64-column tiles (the whole-K phi synthesis) at three k-step counts
    ("phi64_l12", 21, 64, 64, 12, 0.02, True),
    ("phi128_l24", 9, 64, 128, 24, 0.0, False),
    ("phi64_l40", 7, 128, 64, 40, 0.02, True),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_separable_matches_oracle(case):
    name, nr, nt, npf, L, r0, merged = case
    seed = sum(map(ord, name))
    m = wl.random_mesh(seed, nr, nt, npf, L, r0=r0)
    if merged:
        m.shell_class, m.class_block = wl.random_merge(seed + 1, nr, nt, npf)
    rho = wl.random_density(seed + 2, m.shape, positive=False)
    got = run(m, rho)
    ref = oracle.solve(rho=rho, **m.oracle_kwargs())
    ephi, eang = compare(m, rho, got, ref)
    print(name, "phi %.3e ang %.3e" % (ephi, eang))
    assert ephi <= TOL and eang <= TOL, (ephi, eang)
    for k in ("interior", "exterior"):
        # relative to the largest edge moment (modes that vanish identically
        # on this mesh sit at rounding level on both sides)
        scale = np.abs(ref[k]).max() + 1e-300
        assert np.max(np.abs(got[k] - ref[k])) / scale <= TOL, k


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_separable_bf16x3_matches_oracle(case):
    """The separable form with BF16 x3 phi transforms on the same meshes
    (degenerate ones included: one shell row, one theta row, one phi cell,
    lmax 0), to the mixed-precision bar of 1e-6 of the largest potential."""
    name, nr, nt, npf, L, r0, merged = case
    seed = sum(map(ord, name))
    m = wl.random_mesh(seed, nr, nt, npf, L, r0=r0)
    if merged:
        m.shell_class, m.class_block = wl.random_merge(seed + 1, nr, nt, npf)
    rho = wl.random_density(seed + 2, m.shape, positive=False)
    got = run(m, rho, "bf16x3sep")
    ref = oracle.solve(rho=rho, **m.oracle_kwargs())
    ephi, eang = compare(m, rho, got, ref)
    print(name, "bf16x3sep phi %.3e ang %.3e" % (ephi, eang))
    assert ephi <= 1e-6 and eang <= 1e-6, (ephi, eang)


def test_separable_bf16x3_unaligned_density_and_odd_phi():
    """The BF16 x3 phi analysis loads 16 bytes at a time only from 16-byte
    aligned rows: a density view starting one double into its storage, and a
    mesh with an odd phi count, take the element-wise loads and give the
    aligned result bitwise; both against the oracle at 1e-6."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_02507_amd import mpole
    for npf in (26, 27):
        m = wl.random_mesh(77 + npf, 40, 20, npf, 12, r0=0.01)
        m.shell_class, m.class_block = wl.random_merge(78, 40, 20, npf)
        rho = wl.random_density(79, m.shape, positive=False)
        plan = mpole.Plan.from_mesh(m, precision="bf16x3sep")
        a = plan.solve(torch.from_numpy(rho).cuda())["phi"]
        store = torch.zeros(rho.size + 1, dtype=torch.float64, device="cuda")
        view = store[1:].view(m.shape)
        view.copy_(torch.from_numpy(rho).cuda())
        assert view.data_ptr() % 16 == 8
        b = plan.solve(view)["phi"]
        torch.cuda.synchronize()
        assert torch.equal(a, b), npf
        ref = oracle.solve(rho=rho, **m.oracle_kwargs())["phi"]
        rel = np.max(np.abs(a.cpu().numpy() - ref)) / np.max(np.abs(ref))
        assert rel <= 1e-6, (npf, rel)


@pytest.mark.parametrize("blk,npf", [(2, 64), (4, 64), (8, 64), (4, 96)])
def test_separable_bf16x3_whole_step_analysis_equals_general(blk, npf):
    """The whole-step form of the BF16 x3 phi analysis (nphi a multiple of 32,
    16-byte aligned density) does the arithmetic of the general form in the
    same order: on production-rule meshes whose polar rows hold 1 x blk blocks
    (averaged inside the transforms) and whose inner shells hold blk x blk
    blocks, the aligned density (whole-step form) and a view one double into
    its storage (general form) give bitwise the same potential; both against
    the oracle at 1e-6.  nphi 96: three tile pairs per row, spread over
    chunks of the synthesis grid."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_02507_amd import mpole
    nr, nt = 24, 64
    m = wl.Mesh(wl.log_edges(1e-3, 1.0, nr), wl.uniform_edges(0.0, np.pi, nt), wl.uniform_edges(0.0, 2 * np.pi, npf), 12)
    m.shell_class, m.class_block = wl.production_merge(nr, nt, npf, inner_shells=6, polar_rows=8, blk=blk)
    rho = wl.random_density(900 + blk + npf, m.shape, positive=True)
    plan = mpole.Plan.from_mesh(m, precision="bf16x3sep")
    a = plan.solve(torch.from_numpy(rho).cuda())["phi"]
    store = torch.zeros(rho.size + 1, dtype=torch.float64, device="cuda")
    view = store[1:].view(m.shape)
    view.copy_(torch.from_numpy(rho).cuda())
    assert view.data_ptr() % 16 == 8
    b = plan.solve(view)["phi"]
    torch.cuda.synchronize()
    assert torch.equal(a, b), (blk, npf)
    ref = oracle.solve(rho=rho, **m.oracle_kwargs())["phi"]
    rel = np.max(np.abs(a.cpu().numpy() - ref)) / np.max(np.abs(ref))
    assert rel <= 1e-6, (blk, npf, rel)


@pytest.mark.parametrize("name", ["spheroid", "production"])
def test_separable_workloads_full(name):
    m, rho = wl.workload(name)
    got = run(m, rho)
    ref = oracle.solve(rho=rho, **m.oracle_kwargs())
    rel = np.max(np.abs(got["phi"] - ref["phi"]) / np.abs(ref["phi"]))
    print(name, "max rel %.3e" % rel)
    assert rel <= TOL, rel


def test_separable_equals_dense_fp64_path():
    m, rho = wl.workload("production_l32")
    a = run(m, rho, "fp64sep")["phi"]
    b = run(m, rho, "fp64")["phi"]
    assert np.max(np.abs(a - b) / np.abs(b)) <= 1e-13


def test_separable_lmax64_large_angular_mesh():
    m = wl.large_mesh(nr=40)
    m.shell_class, m.class_block = wl.production_merge(40, 256, 512, inner_shells=32)
    c = wl.real_ylm_coeffs(wl.LARGE_LPERT, wl.LARGE_SEED)
    rho = np.ascontiguousarray(wl.radial_profile(m)[:, None, None]
                               * wl.rotated_angular_factor(m, wl.rotation_sequence(2)[2], c)[None])
    got = run(m, rho)
    ref = oracle.solve(rho=rho, **m.oracle_kwargs())
    rel = np.max(np.abs(got["phi"] - ref["phi"]) / np.abs(ref["phi"]))
    assert rel <= TOL, rel


def test_separable_graph_replay_and_restrictions():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_02507_amd import mpole
    m, rho_h = wl.workload("production")
    plan = mpole.Plan.from_mesh(m, precision="fp64sep")
    rho = torch.from_numpy(rho_h).cuda()
    phi = torch.empty_like(rho)
    plan.solve_into(rho, phi=phi)
    torch.cuda.synchronize()
    eager = phi.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.solve_into(rho, phi=phi)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(3):
        phi.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(phi, eager)
    with pytest.raises(mpole.MpoleError):
        plan.table(0)


@pytest.mark.parametrize("precision,tol", [("fp64sep", TOL), ("bf16x3sep", 1e-6)])
def test_separable_batch_equals_single_plans_and_graph_replay(precision, tol):
    """A batch of separable fields (uneven meshes, lmax, merged blocks)
    gives each field's single-plan result bitwise, eagerly and replayed from
    a HIP graph, and reports per-field completion times."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_02507_amd import mpole
    meshes = wl.batch_meshes(6, seed0=7100, nr=(8, 40), ntheta=(8, 24), lmax=(2, 12))
    rhos = [torch.from_numpy(r).cuda() for r in wl.batch_densities(meshes, seed0=7100)]
    b = mpole.Batch(meshes, precision=precision, rho=rhos)
    b.solve()
    torch.cuda.synchronize()
    for m, r, phi in zip(meshes, rhos, b.phi):
        single = mpole.Plan.from_mesh(m, precision=precision).solve(r)["phi"]
        torch.cuda.synchronize()
        assert torch.equal(phi, single)
        ref = oracle.solve(rho=r.cpu().numpy(), **m.oracle_kwargs())["phi"]
        assert np.max(np.abs(phi.cpu().numpy() - ref) / np.abs(ref)) <= tol
    eager = [p.clone() for p in b.phi]
    ms = b.field_ms()
    assert all(0.0 < t for t in ms) and max(ms) < 1e4
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            b.solve()
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(3):
        for p in b.phi:
            p.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert all(torch.equal(p, e) for p, e in zip(b.phi, eager))


def uniform_phi_mesh(seed, nr, nt, nph, L, merged=False, jitter_phi=False):
    m = wl.random_mesh(seed, nr, nt, nph, L, r0=0.05)
    m.phi_edges = wl.uniform_edges(0.3, 0.3 + 2 * np.pi, nph)
    if jitter_phi:   # still closing the circle, no longer uniform: the MFMA transforms
        m.phi_edges = m.phi_edges.copy()
        m.phi_edges[nph // 2] += 1e-3
    if merged:
        m.shell_class, m.class_block = wl.random_merge(seed + 1, nr, nt, nph)
    return m


UNIFORM_PHI_CASES = [
    ("nphi16_lmax7", 9, 6, 16, 7, False, False),
    ("nphi64_lmax31_merged", 7, 5, 64, 31, True, False),
    ("nphi1024", 5, 3, 1024, 20, False, False),
    ("offset_merged", 11, 8, 32, 12, True, False),
    ("nonuniform", 11, 8, 32, 12, True, True),
]


@pytest.mark.parametrize("case", UNIFORM_PHI_CASES, ids=[c[0] for c in UNIFORM_PHI_CASES])
def test_separable_uniform_phi_rows(case):
    """Uniform phi cells closing the circle (lmax up to nphi/2 - 1, nphi up
    to 1024, phi starting off zero, merged blocks) and a nudged edge: the
    phi transforms match the oracle at the FP64 bar."""
    name, nr, nt, nph, L, merged, jit = case
    seed = sum(map(ord, name))
    m = uniform_phi_mesh(seed, nr, nt, nph, L, merged, jit)
    rho = wl.random_density(seed + 2, m.shape, positive=False)
    got = run(m, rho)
    ref = oracle.solve(rho=rho, **m.oracle_kwargs())
    ephi, eang = compare(m, rho, got, ref)
    print(name, "phi %.3e ang %.3e" % (ephi, eang))
    assert ephi <= TOL and eang <= TOL, (ephi, eang)
