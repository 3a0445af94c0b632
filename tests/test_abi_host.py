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
    assert L.mpole_abi_version() == 1


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
