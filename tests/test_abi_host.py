"""Host-side checks of the C ABI: the library loads, exports every entry point
the header declares, and plan creation validates meshes (no GPU needed:
mpole_plan_create makes no HIP call)."""
import os
import re

import numpy as np
import pytest

from paper_2602_02507_amd import mpole
from paper_2602_02507_amd import workloads as wl

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mpole.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mpole_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert set(names) == set(mpole.EXPORTS)
    L = mpole.lib()
    for n in names:
        assert hasattr(L, n), n
    assert L.mpole_abi_version() == 2


def test_plan_sizes():
    m = wl.production_mesh(16)
    p = mpole.HostPlan.from_mesh(m)
    assert p.nmodes == 289
    # tables + packed source of both classes dominate; stays far below HBM size
    assert 1e8 < p.workspace_bytes < 1e9


def mk(**kw):
    base = dict(r_edges=[0.0, 0.5, 1.0], theta_edges=[0.0, np.pi / 2, np.pi], phi_edges=[0.0, np.pi, 2 * np.pi],
                lmax=2)
    base.update(kw)
    return base


@pytest.mark.parametrize("kw,code", [
    (dict(r_edges=[0.0, 1.0, 0.5]), mpole.MpoleError),
    (dict(r_edges=[-0.1, 1.0]), mpole.MpoleError),
    (dict(r_edges=[0.0, np.nan]), mpole.MpoleError),
    (dict(theta_edges=[0.0, 4.0]), mpole.MpoleError),
    (dict(phi_edges=[0.0, 7.0]), mpole.MpoleError),
    (dict(lmax=-1), mpole.MpoleError),
])
def test_invalid_meshes_rejected(kw, code):
    with pytest.raises(mpole.MpoleError) as e:
        mpole.HostPlan(**mk(**kw))
    assert e.value.code == 1


def test_unsupported_and_range_codes():
    with pytest.raises(mpole.MpoleError) as e:
        mpole.HostPlan(**mk(lmax=65))
    assert e.value.code == 5
    with pytest.raises(mpole.MpoleError) as e:
        mpole.HostPlan(**mk(r_edges=[1e-30, 1.0], lmax=10))
    assert e.value.code == 2
    with pytest.raises(mpole.MpoleError) as e:
        mpole.HostPlan(**mk(precision=7))
    assert e.value.code == 5


def test_block_maps_validated():
    sc = np.zeros(2, np.int32)
    good = np.array([[0, 0, 1, 1]], np.int32)
    mpole.HostPlan(**mk(), shell_class=sc, class_block=good)
    for bad in ([[0, 0, 2, 2]], [[0, -1, 1, 1]]):
        with pytest.raises(mpole.MpoleError):
            mpole.HostPlan(**mk(), shell_class=sc, class_block=np.array(bad, np.int32))
    with pytest.raises(mpole.MpoleError):
        mpole.HostPlan(**mk(), shell_class=np.array([0, 1], np.int32), class_block=good)


def test_degenerate_meshes_accepted():
    mpole.HostPlan([0.0, 1.0], [0.0, np.pi], [0.0, 2 * np.pi], 0)
    mpole.HostPlan(wl.log_edges(1e-3, 1, 5), [0.0, np.pi], wl.uniform_edges(0, 2 * np.pi, 3), 64)


def test_error_message_is_per_call():
    with pytest.raises(mpole.MpoleError):
        mpole.HostPlan(**mk(lmax=-1))
    assert mpole.lib().mpole_last_error().decode() != ""
    mpole.HostPlan(**mk())
    assert mpole.lib().mpole_last_error().decode() == ""


def test_tuning_knobs_validated_and_reported():
    m = wl.production_mesh(16)
    p = mpole.HostPlan.from_mesh(m, precision="bf16x3")
    t0 = p.tuning()
    assert t0["moment_tile_m"] == 128 and t0["expand_tile_m"] == 128 and t0["moment_wgs"] > 0
    w0 = p.moment_wgs
    lib = mpole.lib()
    t = mpole.Tuning(0, 64, 64)
    assert lib.mpole_plan_tune(p.handle, t) == 0
    assert p.tuning() == {"moment_wgs": t0["moment_wgs"], "moment_tile_m": 64, "expand_tile_m": 64}
    # half-height tiles double the moment tiles at the same split count or more
    assert lib.mpole_plan_moment_wgs(p.handle) >= w0
    for bad in (mpole.Tuning(0, 32, 0), mpole.Tuning(0, 0, 256), mpole.Tuning(-1, 0, 0)):
        rc = lib.mpole_plan_tune(p.handle, bad)
        assert rc in (1, 5), rc
        assert lib.mpole_last_error()
    # FP64 tiles are 64 high only
    q = mpole.HostPlan.from_mesh(m, precision="fp64")
    assert lib.mpole_plan_tune(q.handle, mpole.Tuning(0, 128, 0)) == 5
    assert lib.mpole_plan_tune(q.handle, mpole.Tuning(2048, 64, 64)) == 0
    assert q.tuning()["moment_wgs"] == 2048


def test_split_chunk_cap_bounds_accumulation_chains(monkeypatch):
    # one workgroup requested: the split precisions still split K into chunks of
    # at most 2048 pairs (FP32 accumulators), FP64 does not
    m = wl.production_mesh(16)
    outer_blocks = 128 * 256 - 16 * 256 + 16 * 256 // 4   # outer class: 8 polar rows per pole merged 1x4 in phi
    ru = lambda x, k: -(-x // k) * k
    # folded (the production mesh is mirror-symmetric): pairs of blocks, and
    # moment columns = even modes padded to the tile width + odd modes
    b = mpole.HostPlan.from_mesh(m, precision="bf16x3", tuning={"moment_wgs": 1})
    f = mpole.HostPlan.from_mesh(m, precision="fp64", tuning={"moment_wgs": 1})
    assert b.folded and f.folded
    n_even, n_odd = 153, 136                                # l + m even / odd for lmax 16
    n_tiles = -(-(ru(n_even, 128) + ru(n_odd, 16)) // 128)
    assert b.moment_wgs >= 4 * n_tiles * -(-(outer_blocks // 2) // 2048)
    n_tiles64 = -(-(ru(n_even, 64) + ru(n_odd, 16)) // 64)
    assert f.moment_wgs == -(-480 // 64) * n_tiles64 + 1 * n_tiles64   # FP64: one split per 64 x 64 tile
    # unfolded: blocks and natural mode order
    monkeypatch.setenv("MPOLE_FOLD", "0")
    b = mpole.HostPlan.from_mesh(m, precision="bf16x3", tuning={"moment_wgs": 1})
    f = mpole.HostPlan.from_mesh(m, precision="fp64", tuning={"moment_wgs": 1})
    assert not b.folded and not f.folded
    n_tiles = (289 + 127) // 128
    assert b.moment_wgs >= 4 * n_tiles * -(-outer_blocks // 2048)
    assert f.moment_wgs == -(-480 // 64) * 5 + 1 * 5


def test_fold_detection():
    """The mirror fold needs theta edges symmetric about the equator and a
    block map that maps onto itself under theta -> pi - theta (blocks that
    straddle the equator are their own mirrors); dense precisions only."""
    prod = wl.production_mesh(8, nr=40, ntheta=36, nphi=72)   # 4 x 4 blocks straddle the equator (rows 16-19)
    prod.shell_class, prod.class_block = wl.production_merge(40, 36, 72, inner_shells=8, polar_rows=4)
    assert mpole.HostPlan.from_mesh(prod, precision="bf16x3").folded
    odd = wl.production_mesh(6, nr=12, ntheta=33, nphi=16, merged=False)   # equator row is its own mirror
    assert mpole.HostPlan.from_mesh(odd).folded
    assert not mpole.HostPlan.from_mesh(odd, precision="fp64sep").folded
    assert not mpole.HostPlan.from_mesh(wl.random_mesh(3, 12, 8, 16, 4)).folded   # jittered theta edges
    asym = wl.production_mesh(6, nr=12, ntheta=8, nphi=16, merged=False)
    cb = np.arange(8 * 16, dtype=np.int32)
    cb[16:18] = 16                  # a 1 x 2 block in row 1 whose mirror row (6) stays single cells
    cb = np.unique(cb, return_inverse=True)[1].astype(np.int32)
    asym.shell_class, asym.class_block = np.zeros(12, np.int32), cb[None, :]
    assert not mpole.HostPlan.from_mesh(asym).folded


def test_workload_library_exports_its_header():
    from paper_2602_02507_amd import devicegen
    text = open(os.path.join(os.path.dirname(HEADER), "mpole_workload.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(mpole_[a-z_0-9]+)\s*\(", text))
    assert names == {"mpole_wl_rotated_density"}
    L = devicegen.lib()
    for n in names:
        assert hasattr(L, n), n
    # invalid arguments are rejected before any launch (no GPU touched)
    assert L.mpole_wl_rotated_density(0, 1, 1, 1, 1, 1, 0, 1, 0.0, 1, 1, None) == 1
    assert L.mpole_wl_rotated_density(1, 1, 1, 1, 1, 1, 17, 1, 0.0, 1, 1, None) == 1
    assert L.mpole_wl_rotated_density(1, 1, 1, None, 1, 1, 0, 1, 0.0, 1, 1, None) == 1


def test_gradient_rejects_unbound_plan():
    m = wl.production_mesh(4, nr=8, ntheta=8, nphi=8, merged=False)
    p = mpole.HostPlan.from_mesh(m)
    L = mpole.lib()
    assert L.mpole_gradient(None, 1, 1, 1, 1, None) == 1
    assert L.mpole_gradient(p.handle, 1, 1, 1, 1, None) == 1      # not bound: nothing launched
    assert b"not bound" in L.mpole_last_error()


def test_bf16x3_separable_plan_host_side():
    """MPOLE_BF16X3_SEPARABLE plans like the FP64 separable path, plus the
    bind-time fragment-order trig tables: 64 lanes x 16 bytes per (K step,
    16-row tile, plane), 3 planes; no launch knobs, no block x mode table."""
    m = wl.production_mesh(32)
    a = mpole.HostPlan.from_mesh(m, precision="fp64sep")
    b = mpole.HostPlan.from_mesh(m, precision="bf16x3sep")
    ks_a, mt_a = -(-m.nphi // 32), -(-2 * m.lmax // 16)
    ks_s, nt_s = -(-2 * m.lmax // 32), -(-m.nphi // 16)
    frag = 3 * 64 * 16
    align = lambda x: -(-x // 256) * 256
    extra = align(frag * ks_a * mt_a) + align(frag * ks_s * nt_s)
    assert b.workspace_bytes == a.workspace_bytes + extra, (b.workspace_bytes, a.workspace_bytes, extra)
    lib = mpole.lib()
    assert lib.mpole_plan_tune(b.handle, mpole.Tuning(0, 128, 0)) == 5
    assert lib.mpole_plan_copy_table(b.handle, 0, None, None, None) == 5
    # lmax 0: no m >= 1 rows, empty fragment tables
    m0 = wl.production_mesh(0)
    a0 = mpole.HostPlan.from_mesh(m0, precision="fp64sep")
    b0 = mpole.HostPlan.from_mesh(m0, precision="bf16x3sep")
    assert b0.workspace_bytes == a0.workspace_bytes


def test_workspace_errors_before_any_device_work():
    """Every MPOLE_ERR_WORKSPACE path is decided on the host before a HIP call:
    a null, misaligned or undersized workspace at bind (plan and batch), and
    solves, table copies, field times and launch checks of an unbound plan or
    batch; an unknown batch launch is MPOLE_ERR_INVALID.  The
    fake device addresses below are never dereferenced."""
    import ctypes
    L = mpole.lib()
    m = wl.production_mesh(4, nr=8, ntheta=8, nphi=8, merged=False)
    p = mpole.HostPlan.from_mesh(m)
    need = p.workspace_bytes
    fake = ctypes.c_void_p(1 << 20)            # 256-byte aligned, never touched
    assert L.mpole_plan_bind(p.handle, None, need, None) == 3
    assert b"null" in L.mpole_last_error()
    assert L.mpole_plan_bind(p.handle, ctypes.c_void_p((1 << 20) + 8), need, None) == 3
    assert b"aligned" in L.mpole_last_error()
    assert L.mpole_plan_bind(p.handle, fake, need - 1, None) == 3
    assert b"needs" in L.mpole_last_error()
    assert L.mpole_solve(p.handle, fake, fake, None, None, None, None) == 3
    assert b"no bound workspace" in L.mpole_last_error()
    out = np.zeros((64, p.nmodes))
    n = ctypes.c_int64()
    assert L.mpole_plan_copy_table(p.handle, 0, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n), None) == 3
    # batches
    descs = (mpole.MeshC * 2)()
    keep = []
    for f in range(2):
        d, k = mpole.make_mesh(m.r_edges, m.theta_edges, m.phi_edges, 2 + f)
        descs[f] = d
        keep.append(k)
    h = ctypes.c_void_p()
    assert L.mpole_batch_create(2, descs, ctypes.byref(h)) == 0
    bneed = L.mpole_batch_workspace_bytes(h)
    ptrs = (ctypes.c_void_p * 2)(1 << 20, 1 << 21)
    assert L.mpole_batch_bind(h, None, bneed, ptrs, ptrs, None) == 3
    assert L.mpole_batch_bind(h, ctypes.c_void_p((1 << 20) + 64), bneed, ptrs, ptrs, None) == 3
    assert L.mpole_batch_bind(h, fake, bneed - 256, ptrs, ptrs, None) == 3
    assert L.mpole_batch_solve(h, None) == 3
    ms = (ctypes.c_double * 2)()
    assert L.mpole_batch_field_ms(h, ms) == 3
    # launch selection: decided on the host; an unbound batch has no launch yet
    assert L.mpole_batch_set_launch(h, 3, 0) == 1
    assert b"unknown launch" in L.mpole_last_error()
    assert L.mpole_batch_set_launch(h, mpole.LAUNCH_PERSISTENT_FORCED, 5) == 0
    assert L.mpole_batch_set_launch(h, mpole.LAUNCH_PHASES, 0) == 0
    assert L.mpole_batch_launch(h) == -1
    assert L.mpole_batch_launch_note(h) == b""
    assert L.mpole_batch_check(h, None) == 3
    assert L.mpole_batch_set_launch(None, 1, 0) == 1
    assert L.mpole_batch_launch(None) == -1
    assert L.mpole_batch_launch_note(None) == b""
    assert L.mpole_batch_check(None, None) == 1
    assert L.mpole_batch_destroy(h) == 0


def test_batch_field_count_limits():
    """Batches of 1..4096 fields are accepted (the per-field completion stamps
    are reset by a grid of 256-thread workgroups, so 1024 fields and more
    launch too); 0 and 4097 are rejected."""
    import ctypes
    L = mpole.lib()
    m = wl.production_mesh(1, nr=2, ntheta=2, nphi=2, merged=False)
    d, keep = mpole.make_mesh(m.r_edges, m.theta_edges, m.phi_edges, 1)
    h = ctypes.c_void_p()
    descs = (mpole.MeshC * 4097)(*([d] * 4097))
    assert L.mpole_batch_create(0, descs, ctypes.byref(h)) == 1
    assert L.mpole_batch_create(4097, descs, ctypes.byref(h)) == 1
    assert L.mpole_batch_create(4096, descs, ctypes.byref(h)) == 0
    t = (mpole.Tuning * 4096)()
    assert L.mpole_batch_get_tuning(h, t) == 0
    assert all(t[f].moment_wgs >= 1 for f in range(4096))
    assert L.mpole_batch_destroy(h) == 0
