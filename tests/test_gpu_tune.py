"""GPU test of the autotuner: it returns a valid tuning, caches it per mesh
shape, and the tuned plan solves to the same bar as the default one."""
import numpy as np
import pytest

import oracle
from paper_2602_02507_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_tune_plan_caches_and_stays_exact(tmp_path, monkeypatch):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_02507_amd import mpole, tune
    monkeypatch.setenv(tune.CACHE_ENV, str(tmp_path / "tune.json"))
    m = wl.random_mesh(5, 150, 16, 32, 12, r0=0.01)
    m.shell_class, m.class_block = wl.random_merge(6, 150, 16, 32)
    t = tune.tune_plan(m, "bf16x3", "cuda")
    assert t["moment_tile_m"] in (64, 128) and t["expand_tile_m"] in (64, 128) and t["moment_wgs"] > 0
    cache = tune.load_cache()
    assert len(cache) == 1
    (entry,) = cache.values()
    assert entry["tuning"] == t and entry["moment_ms"] > 0 and entry["expand_ms"] > 0
    assert tune.tune_plan(m, "bf16x3", "cuda") == t   # from the cache
    rho = wl.random_density(7, m.shape) + 0.5
    plan = mpole.Plan.from_mesh(m, precision="bf16x3", tuning=t)
    phi = plan.solve(torch.from_numpy(rho).cuda())["phi"].cpu().numpy()
    ref = oracle.solve(rho=rho, **m.oracle_kwargs())["phi"]
    assert np.max(np.abs(phi - ref) / np.abs(ref)) <= 1e-6


def test_tune_batch_returns_one_tuning_per_field(tmp_path, monkeypatch):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_02507_amd import mpole, tune
    monkeypatch.setenv(tune.CACHE_ENV, str(tmp_path / "tune.json"))
    meshes = wl.batch_meshes(4, seed0=300, nr=(20, 80), ntheta=(8, 20), lmax=(2, 10))
    rho = [torch.from_numpy(r).cuda() for r in wl.batch_densities(meshes, seed0=300)]
    tun, info = tune.tune_batch(meshes, "bf16x3", "cuda", rho=rho)
    assert len(tun) == 4 and info["field_shapes_tuned"] >= 1
    b = mpole.Batch(meshes, precision="bf16x3", rho=rho, tunings=tun)
    b.solve()
    torch.cuda.synchronize()
    for f, m in enumerate(meshes):
        ref = oracle.solve(rho=rho[f].cpu().numpy(), **m.oracle_kwargs())["phi"]
        assert np.max(np.abs(b.phi[f].cpu().numpy() - ref) / np.abs(ref)) <= 1e-6
