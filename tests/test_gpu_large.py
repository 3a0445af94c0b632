"""GPU tests of the repeated-solve workload (2048 x 256 x 512, lmax 64,
FP16 x2 in one HIP graph): its device density generator against the host
recipe, the lmax = 64 path on its full angular mesh against the oracle, and a
short graph of consecutive solves on the advected density against eager
solves and the FP64 path."""
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


def test_rotated_density_kernel_matches_host():
    torch = _torch()
    from paper_2602_02507_amd import devicegen
    m = wl.large_mesh(nr=5, ntheta=64, nphi=128, lmax=8)
    c = wl.real_ylm_coeffs(wl.LARGE_LPERT, wl.LARGE_SEED)
    rots = wl.rotation_sequence(7)
    gen = devicegen.RotatedDensity(m, c, rots, wl.LARGE_EPS)
    rho = torch.empty(m.shape, dtype=torch.float64, device="cuda")
    radial = wl.radial_profile(m)
    for step in (0, 3, 7):
        gen.write(rho, step)
        torch.cuda.synchronize()
        got = rho.cpu().numpy()
        want = radial[:, None, None] * wl.rotated_angular_factor(m, rots[step], c)[None]
        assert np.max(np.abs(got - want) / np.abs(want)) < 1e-13, step
    with pytest.raises(IndexError):
        gen.write(rho, 8)


def test_lmax64_full_angular_mesh_matches_oracle():
    """40 log shells of the 256 x 512 angular mesh at lmax = 64 (4225 modes),
    coarsened: FP64 path to 1e-12, FP16 x2 to 1e-6, every cell."""
    torch = _torch()
    from paper_2602_02507_amd import mpole
    m = wl.large_mesh(nr=40)
    m.shell_class, m.class_block = wl.production_merge(40, 256, 512, inner_shells=32)
    c = wl.real_ylm_coeffs(wl.LARGE_LPERT, wl.LARGE_SEED)
    rho = wl.radial_profile(m)[:, None, None] * wl.rotated_angular_factor(m, wl.rotation_sequence(2)[2], c)[None]
    rho = np.ascontiguousarray(rho)
    ref = oracle.solve(rho=rho, **m.oracle_kwargs())["phi"]
    for precision, tol in (("fp64", 1e-12), ("fp16x2", 1e-6)):
        plan = mpole.Plan.from_mesh(m, precision=precision)
        phi = plan.solve(torch.from_numpy(rho).cuda())["phi"].cpu().numpy()
        err = np.max(np.abs(phi - ref) / np.abs(ref))
        print(precision, "max rel err %.3e" % err)
        assert err <= tol, (precision, err)
        del plan
        torch.cuda.empty_cache()


def test_graph_of_advected_solves_matches_eager_and_fp64():
    """Ten steps (density update + FP16 x2 solve) captured in one graph with a
    snapshot of the potential every fifth step; each snapshot equals the eager
    solve of the same step bitwise and the FP64 solve to 1e-6."""
    torch = _torch()
    from paper_2602_02507_amd import devicegen, mpole
    m = wl.large_mesh(nr=96, ntheta=64, nphi=128, lmax=24)
    c = wl.real_ylm_coeffs(wl.LARGE_LPERT, wl.LARGE_SEED)
    steps, every = 10, 5
    rots = wl.rotation_sequence(steps)
    gen = devicegen.RotatedDensity(m, c, rots, wl.LARGE_EPS)
    dev = torch.device("cuda")
    rho = torch.empty(m.shape, dtype=torch.float64, device=dev)
    plan = mpole.Plan.from_mesh(m, precision="fp16x2")
    phi = torch.empty_like(rho)
    snaps = [torch.empty_like(rho) for _ in range(steps // every)]
    gen.write(rho, 0)
    plan.solve_into(rho, phi=phi)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for t in range(1, steps + 1):
                gen.write(rho, t)
                plan.solve_into(rho, phi=phi)
                if t % every == 0:
                    snaps[t // every - 1].copy_(phi)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(2):
        phi.zero_()
        g.replay()
        torch.cuda.synchronize()
        p64 = mpole.Plan.from_mesh(m, precision="fp64")
        for k, snap in enumerate(snaps):
            t = (k + 1) * every
            gen.write(rho, t)
            eager = plan.solve(rho)["phi"]
            ref = p64.solve(rho)["phi"]
            torch.cuda.synchronize()
            assert torch.equal(eager, snap), (rep, t)
            err = float((snap - ref).abs().div(ref.abs()).max())
            assert err <= 1e-6, (rep, t, err)
        del p64
