"""GPU tests of the persistent batched launch (one launch, per-XCD work queues).

* every field equals the per-phase launch of the same batch and its
  single-plan solve, bitwise (the items run the per-phase kernels' device
  code on the same tiles), and matches the FP64 oracle;
* a HIP graph capture of the persistent solve, replayed with eager work in
  between, reproduces the eager result every time;
* on a batch of many uneven fields, small fields complete well before the
  batch does (per-field completion stamps);
* a dependency-wait budget too small for the batch makes the launch give up
  its waits, end normally and report MPOLE_ERR_DEVICE through check(); the
  next solve with the default budget is again bitwise right.
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


def _batch_pair(meshes, rho, precision, **kw):
    from paper_2602_02507_amd import mpole
    per = mpole.Batch(meshes, precision=precision, rho=rho, launch="forced", **kw)
    ph = mpole.Batch(meshes, precision=precision, rho=rho, launch="phases", **kw)
    assert per.launch == "persistent", per.launch_note
    assert ph.launch == "phases"
    return per, ph


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("bf16x3", 1e-6), ("fp16x2", 1e-6)])
def test_persistent_matches_phases_single_and_oracle(precision, tol):
    torch = _torch()
    from paper_2602_02507_amd import mpole
    meshes = wl.batch_meshes(11, seed0=301, nr=(20, 90), ntheta=(8, 24), lmax=(2, 12))
    rho = [torch.from_numpy(r).cuda() for r in wl.batch_densities(meshes, seed0=301)]
    per, ph = _batch_pair(meshes, rho, precision)
    print("persistent %s: %d fields" % (precision, len(meshes)), flush=True)
    per.solve()
    ph.solve()
    per.check()
    torch.cuda.synchronize()
    tun = per.tunings()
    for f, m in enumerate(meshes):
        assert torch.equal(per.phi[f], ph.phi[f]), f
        single = mpole.Plan.from_mesh(m, precision=precision, tuning=tun[f]).solve(rho[f])["phi"]
        torch.cuda.synchronize()
        assert torch.equal(single, per.phi[f]), f
        ref = oracle.solve(rho=rho[f].cpu().numpy(), **m.oracle_kwargs())["phi"]
        rel = np.max(np.abs(per.phi[f].cpu().numpy() - ref) / np.abs(ref))
        assert rel <= tol, (f, rel)


def test_persistent_mixed_tiles_and_signed_density():
    """Per-field tile heights and split-K targets and a signed density with
    zero-mean fields, through the persistent launch: bitwise the per-phase
    launch."""
    torch = _torch()
    meshes = wl.batch_meshes(9, seed0=17, nr=(16, 70), ntheta=(8, 20), lmax=(1, 16))
    dens = wl.batch_densities(meshes, seed0=17)
    dens = [d - d.mean() if f % 2 else d - 0.5 * d.mean() for f, d in enumerate(dens)]
    rho = [torch.from_numpy(np.ascontiguousarray(d)).cuda() for d in dens]
    hs = [(64, 64), (128, 64), (64, 128), (128, 128)]
    tun = [{"moment_wgs": 1 + 3 * f % 7, "moment_tile_m": hs[f % 4][0], "expand_tile_m": hs[f % 4][1]}
           for f in range(len(meshes))]
    per, ph = _batch_pair(meshes, rho, "bf16x3", tunings=tun)
    for _ in range(2):
        per.solve()
        ph.solve()
    per.check()
    torch.cuda.synchronize()
    for f in range(len(meshes)):
        assert torch.equal(per.phi[f], ph.phi[f]), f


def test_persistent_graph_replay_matches_eager():
    torch = _torch()
    from paper_2602_02507_amd import mpole
    meshes = wl.batch_meshes(16, seed0=92, nr=(20, 90), ntheta=(8, 24), lmax=(2, 12))
    rho = [torch.from_numpy(r).cuda() for r in wl.batch_densities(meshes, seed0=92)]
    batch = mpole.Batch(meshes, precision="bf16x3", rho=rho, launch="forced")
    assert batch.launch == "persistent", batch.launch_note
    batch.solve()
    batch.check()
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
        batch.check()
        for f in range(len(meshes)):
            assert torch.equal(batch.phi[f], eager[f]), (rep, f)
    ms = batch.field_ms()
    assert all(x > 0 for x in ms), ms


def test_persistent_small_fields_finish_early():
    """64 uneven fields (the size mix of the 64-field workload, scaled down):
    the persistent launch is the default, and the median field completes
    well before the batch."""
    torch = _torch()
    from paper_2602_02507_amd import mpole
    meshes = wl.batch_meshes(64, seed0=4000, nr=(40, 200), ntheta=(8, 48), lmax=(4, 24))
    rho = [torch.from_numpy(r).cuda() for r in wl.batch_densities(meshes, seed0=4000)]
    batch = mpole.Batch(meshes, precision="bf16x3", rho=rho)
    assert batch.launch == "persistent", batch.launch_note
    for _ in range(3):
        batch.solve()
    batch.check()
    torch.cuda.synchronize()
    ms = np.array(batch.field_ms())
    assert np.all(ms > 0), ms
    p50, last = np.median(ms), ms.max()
    print("fields %d: p50 %.3f ms, last %.3f ms" % (len(ms), p50, last), flush=True)
    assert p50 < 0.75 * last, (p50, last)


def test_persistent_wait_budget_exhausted_is_reported():
    """A one-poll dependency-wait budget: waits give up, the launch ends
    normally and check() reports MPOLE_ERR_DEVICE; with the default budget
    the next solve is bitwise the per-phase launch again."""
    torch = _torch()
    from paper_2602_02507_amd import mpole
    meshes = wl.batch_meshes(12, seed0=55, nr=(60, 120), ntheta=(16, 32), lmax=(8, 16))
    rho = [torch.from_numpy(r).cuda() for r in wl.batch_densities(meshes, seed0=55)]
    per, ph = _batch_pair(meshes, rho, "bf16x3")
    ph.solve()
    per.set_launch("forced", wait_polls=1)
    per.solve()
    with pytest.raises(mpole.MpoleError) as ei:
        per.check()
    assert "MPOLE_ERR_DEVICE" in str(ei.value) and "gave up" in str(ei.value)
    per.set_launch("forced")
    per.solve()
    per.check()
    torch.cuda.synchronize()
    for f in range(len(meshes)):
        assert torch.equal(per.phi[f], ph.phi[f]), f
