"""The allocation-free entry point mpole_solve_static through the C ABI.

It must give exactly what mpole_solve gives for the same bound plan and
inputs (the same kernels run; only where the intermediates live differs):
every output bitwise equal, on two static solves in a row, the second on a
smaller plan, so that the static array still holds the first solve's
intermediates when the second starts.  Also: the oversize error, and a
static solve between two ordinary ones of the same plan."""
import ctypes

import numpy as np
import pytest

from paper_2602_02507_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def meshes(precision):
    big = wl.random_mesh(501, 130, 16, 32, 14, r0=0.01)
    big.shell_class, big.class_block = wl.random_merge(502, 130, 16, 32)
    small = wl.production_mesh(6, nr=40, ntheta=8, nphi=16)
    small.shell_class, small.class_block = wl.production_merge(40, 8, 16, inner_shells=8, polar_rows=2)
    return big, small


def static_solve(plan, rho, out, stream):
    from paper_2602_02507_amd import mpole
    rc = mpole.lib().mpole_solve_static(plan.handle, _ptr(rho), _ptr(out["phi"]), _ptr(out["ang"]),
                                        _ptr(out["interior"]), _ptr(out["exterior"]), ctypes.c_void_p(stream))
    assert rc == 0, mpole.lib().mpole_last_error()


@pytest.mark.parametrize("precision", ["fp64", "bf16x3", "fp16x2", "fp64sep", "bf16x3sep"])
def test_static_solve_equals_solve_two_calls_shrinking(precision):
    torch = _torch()
    from paper_2602_02507_amd import mpole
    stream = torch.cuda.current_stream().cuda_stream
    plans, rhos, refs = [], [], []
    for k, m in enumerate(meshes(precision)):
        print("mesh %d: %d x %d x %d lmax %d %s" % (k, m.nr, m.ntheta, m.nphi, m.lmax, precision), flush=True)
        plan = mpole.Plan.from_mesh(m, precision=precision)
        rho = torch.from_numpy(wl.random_density(600 + k, m.shape, positive=False) + 0.2).cuda()
        ref = plan.solve(rho)
        plans.append(plan)
        rhos.append(rho)
        refs.append(ref)
    torch.cuda.synchronize()
    for plan, rho, ref in zip(plans, rhos, refs):   # larger plan first, then the smaller one
        out = plan.empty_outputs()
        for v in out.values():
            v.fill_(-7.0)
        static_solve(plan, rho, out, stream)
        torch.cuda.synchronize()
        for key in ("phi", "ang", "interior", "exterior"):
            assert torch.equal(out[key], ref[key]), key


def test_static_between_workspace_solves_and_repeated():
    """Static and workspace solves of one plan interleaved, and a static solve
    repeated: all bitwise equal."""
    torch = _torch()
    from paper_2602_02507_amd import mpole
    stream = torch.cuda.current_stream().cuda_stream
    m, _ = meshes("bf16x3")
    plan = mpole.Plan.from_mesh(m, precision="bf16x3")
    rho = torch.from_numpy(wl.random_density(700, m.shape) + 0.5).cuda()
    a = plan.solve(rho)
    b = plan.empty_outputs()
    static_solve(plan, rho, b, stream)
    c = plan.solve(rho)
    d = plan.empty_outputs()
    static_solve(plan, rho, d, stream)
    torch.cuda.synchronize()
    for key in a:
        assert torch.equal(a[key], b[key]) and torch.equal(a[key], c[key]) and torch.equal(a[key], d[key]), key


def test_static_rejects_oversize_and_unbound():
    """A plan whose intermediates exceed the static array is rejected before
    anything is launched (no device pointer is touched)."""
    _torch()
    from paper_2602_02507_amd import mpole
    big = mpole.HostPlan.from_mesh(wl.production_mesh(64, nr=2048, ntheta=256, nphi=512), precision="bf16x3")
    fake = ctypes.c_void_p(1 << 20)
    L = mpole.lib()
    assert L.mpole_solve_static(big.handle, fake, fake, None, None, None, None) == 5
    assert b"static array" in L.mpole_last_error()
    small = mpole.HostPlan.from_mesh(meshes("fp64")[1])
    assert L.mpole_solve_static(small.handle, fake, fake, None, None, None, None) == 3
