"""GPU tests of the batched solve: uneven fields in one launch per phase.

* every field of a batch equals the single-plan solve of that field, bitwise
  when both use the same split-K configuration (the same kernels run the same
  tiles), and matches the FP64 oracle (1e-12 FP64, 1e-6 BF16 x3);
* a HIP graph capture of the batch solve, replayed several times with eager
  work in between, reproduces the eager result every time;
* per-field completion times are positive and ordered within the batch.
"""
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


def small_batch(n=6, seed0=77):
    return wl.batch_meshes(n, seed0=seed0, nr=(20, 90), ntheta=(8, 24), lmax=(2, 12))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("bf16x3", 1e-6)])
def test_batch_matches_single_plans_and_oracle(precision, tol):
    torch = _torch()
    from paper_2602_02507_amd import mpole
    meshes = small_batch()
    rho = [torch.from_numpy(r).cuda() for r in wl.batch_densities(meshes, seed0=77)]
    wgs = [5, 1, 3, 8, 2, 4]
    batch = mpole.Batch(meshes, precision=precision, rho=rho, moment_wgs=wgs)
    batch.solve()
    torch.cuda.synchronize()
    for f, m in enumerate(meshes):
        plan = mpole.Plan.from_mesh(m, precision=precision, moment_wgs=wgs[f])
        single = plan.solve(rho[f])["phi"]
        torch.cuda.synchronize()
        assert torch.equal(single, batch.phi[f]), f
        ref = oracle.solve(rho=rho[f].cpu().numpy(), **m.oracle_kwargs())["phi"]
        rel = np.max(np.abs(batch.phi[f].cpu().numpy() - ref) / np.abs(ref))
        assert rel <= tol, (f, rel)


@pytest.mark.parametrize("precision,tol", [("bf16x3", 1e-6), ("fp16x2", 1e-6)])
def test_batch_with_mixed_tile_heights(precision, tol):
    """Per-field launch tunings (as the autotuner picks them) in one batch:
    each field equals its single-plan solve under the same tuning, bitwise."""
    torch = _torch()
    from paper_2602_02507_amd import mpole
    meshes = small_batch(6, seed0=123)
    rho = [torch.from_numpy(r).cuda() for r in wl.batch_densities(meshes, seed0=123)]
    tun = [{"moment_wgs": w, "moment_tile_m": hm, "expand_tile_m": he}
           for w, hm, he in [(3, 64, 64), (1, 128, 64), (6, 64, 128), (2, 128, 128), (9, 64, 64), (4, 128, 64)]]
    batch = mpole.Batch(meshes, precision=precision, rho=rho, tunings=tun)
    batch.solve()
    torch.cuda.synchronize()
    for f, m in enumerate(meshes):
        plan = mpole.Plan.from_mesh(m, precision=precision, tuning=tun[f])
        single = plan.solve(rho[f])["phi"]
        torch.cuda.synchronize()
        assert torch.equal(single, batch.phi[f]), f
        ref = oracle.solve(rho=rho[f].cpu().numpy(), **m.oracle_kwargs())["phi"]
        rel = np.max(np.abs(batch.phi[f].cpu().numpy() - ref) / np.abs(ref))
        assert rel <= tol, (f, rel)


def test_batch_graph_replay_matches_eager():
    torch = _torch()
    from paper_2602_02507_amd import mpole
    meshes = small_batch(5, seed0=91)
    rho = [torch.from_numpy(r).cuda() for r in wl.batch_densities(meshes, seed0=91)]
    batch = mpole.Batch(meshes, precision="bf16x3", rho=rho)
    batch.solve()
    torch.cuda.synchronize()
    eager = [p.clone() for p in batch.phi]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):          # warm the capture stream
        batch.solve()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.solve()
    for rep in range(4):
        for p in batch.phi:              # eager work between replays
            p.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for f in range(len(meshes)):
            assert torch.equal(batch.phi[f], eager[f]), (rep, f)
    ms = batch.field_ms()
    assert all(x > 0 for x in ms), ms


def test_batch_field_times_after_eager_solve():
    torch = _torch()
    from paper_2602_02507_amd import mpole
    meshes = small_batch(4, seed0=5)
    rho = [torch.from_numpy(r).cuda() for r in wl.batch_densities(meshes, seed0=5)]
    batch = mpole.Batch(meshes, precision="fp64", rho=rho)
    batch.solve()
    torch.cuda.synchronize()
    ms = batch.field_ms()
    assert len(ms) == 4 and all(0 < x < 1e3 for x in ms), ms


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("bf16x3", 1e-6), ("fp64sep", 1e-12), ("bf16x3sep", 1e-6)])
def test_batch_of_genasis_meshes(precision, tol):
    """GenASiS meshes (automatic coarsening: many classes, blocks up to whole
    shells) mixed with a production-rule mesh in one batch: the per-field
    block sums and broadcasts of the large blocks run around the batched
    launches; every field equals its single-plan solve bitwise and the
    oracle to the precision's bar."""
    torch = _torch()
    from oracle import genasis as og
    from paper_2602_02507_amd import mpole
    meshes = []
    for nt, rr, L in ((16, 2.5, 6), (32, 1.5, 10)):
        g = og.mesh(nt, 0.25, rr, dims=3)
        meshes.append(wl.Mesh(g["r_edges"], g["theta_edges"], g["phi_edges"], L, g["shell_class"],
                              g["class_block"]))
    meshes += small_batch(1, seed0=91)
    rho = [torch.from_numpy(wl.production_density(m, seed=5)).cuda() for m in meshes]
    wgs = [7, 3, 5]   # the same split-K on both sides
    batch = mpole.Batch(meshes, precision=precision, rho=rho, moment_wgs=wgs)
    batch.solve()
    torch.cuda.synchronize()
    for f, m in enumerate(meshes):
        single = mpole.Plan.from_mesh(m, precision=precision, moment_wgs=wgs[f]).solve(rho[f])["phi"]
        torch.cuda.synchronize()
        assert torch.equal(single, batch.phi[f]), f
        ref = oracle.solve(rho=rho[f].cpu().numpy(), **m.oracle_kwargs())["phi"]
        rel = np.max(np.abs(batch.phi[f].cpu().numpy() - ref) / np.abs(ref))
        assert rel <= tol, (f, rel)


# fields of the 64-field uneven workload (seeds 4000 + f): the smallest, a
# mid-sized one, the one with the most cells (and theta rows), the one with
# the most shells and one at the largest lmax
CONFIG4_FIELDS = (58, 24, 5, 44, 51)


@pytest.mark.parametrize("precision", ["bf16x3", "fp16x2"])
def test_batch_real_uneven_draws_match_oracle(precision):
    """Five real draws of the 64-field workload (up to 933 x 240 x 480 cells,
    1020 shells, lmax 32) solved as one batch: every cell of every field
    within 1e-6 of the oracle, and each field bitwise equal to its
    single-plan solve under the same launch tuning."""
    torch = _torch()
    from paper_2602_02507_amd import mpole
    allm = wl.batch_meshes(64)
    # the workload's densities use seed 4000 + f
    dens = [wl.production_density(allm[f], seed=4000 + f) for f in CONFIG4_FIELDS]
    meshes = [allm[f] for f in CONFIG4_FIELDS]
    rho = [torch.from_numpy(r).cuda() for r in dens]
    batch = mpole.Batch(meshes, precision=precision, rho=rho)
    batch.solve()
    torch.cuda.synchronize()
    tunings = batch.tunings()
    for f, m in enumerate(meshes):
        print("field %d: %d x %d x %d lmax %d" % (CONFIG4_FIELDS[f], m.nr, m.ntheta, m.nphi, m.lmax), flush=True)
        single = mpole.Plan.from_mesh(m, precision=precision, tuning=tunings[f]).solve(rho[f])["phi"]
        torch.cuda.synchronize()
        assert torch.equal(single, batch.phi[f]), f
        del single
        ref = oracle.solve(rho=dens[f], **m.oracle_kwargs())["phi"]
        rel = np.max(np.abs(batch.phi[f].cpu().numpy() - ref) / np.abs(ref))
        print("  max rel err vs oracle %.3e" % rel, flush=True)
        assert rel <= 1e-6, (f, rel)


def test_batch_of_1100_tiny_fields():
    """More fields than a workgroup has threads (the completion stamps are
    reset by a grid of workgroups): 1100 tiny fields in one batch, each
    bitwise equal to its single-plan solve (sampled) and the completion times
    all recorded."""
    torch = _torch()
    from paper_2602_02507_amd import mpole
    n = 1100
    base = wl.Mesh(wl.log_edges(0.1, 1.0, 4), wl.uniform_edges(0.0, np.pi, 4), wl.uniform_edges(0.0, 2 * np.pi, 8), 2)
    meshes = [base.with_lmax(1 + f % 3) for f in range(n)]
    rho = [torch.from_numpy(wl.random_density(f, base.shape) + 0.5).cuda() for f in range(n)]
    batch = mpole.Batch(meshes, precision="fp64", rho=rho)
    batch.solve()
    torch.cuda.synchronize()
    tun = batch.tunings()
    for f in (0, 1, 511, 1023, 1024, n - 1):
        single = mpole.Plan.from_mesh(meshes[f], precision="fp64", tuning=tun[f]).solve(rho[f])["phi"]
        torch.cuda.synchronize()
        assert torch.equal(single, batch.phi[f]), f
    ms = batch.field_ms()
    assert len(ms) == n and all(x > 0 for x in ms), min(ms)
