"""Pins of the oracle's GenASiS mesh, automatic coarsening and block volume
average (Sec. 2.1, Sec. 2.3, Sec. 3) against numbers the paper prints, group
sizes worked by hand, and properties the rule guarantees."""
import json
import math
import os

import numpy as np
import pytest

from oracle import genasis as og

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "genasis_mesh.json")


@pytest.fixture(scope="module")
def gold():
    with open(GOLDEN) as f:
        return json.load(f)


def test_worked_meshes_reproduce_printed_rout_and_drmin(gold):
    for c in gold["worked_meshes"]["cases"]:
        r, th, ph, ncore = og.edges(c["ntheta"], c["r_core"], c["r_radial"])
        assert abs(c["r_core"] / ncore - c["dr_min"]) <= c["dr_tol"]
        assert abs(r[-1] - c["r_out"]) <= c["r_out_tol"], (c, r[-1])
        # the core is uniform with width dr_min and ends exactly at r_core
        dr = np.diff(r[:ncore + 1])
        np.testing.assert_allclose(dr, c["r_core"] / ncore, rtol=1e-12)
        assert r[ncore] == c["r_core"]


def test_aspect_ratio_at_core_and_constant_outside(gold):
    g = gold["aspect"]
    r, th, ph, ncore = og.edges(256, 0.25, 3.68)
    dth = th[1] - th[0]
    dr_min = 0.25 / ncore
    assert abs(0.25 * dth / dr_min - g["value"]) <= g["tol"]
    outer = np.arange(ncore, r.size - 1)
    ratio = r[outer] * dth / (r[outer + 1] - r[outer])
    np.testing.assert_allclose(ratio, 0.25 * dth / dr_min, rtol=1e-9)


def test_timestep_gain_of_coarsening(gold):
    """The paper's gains reproduce with the first cell centre at dr_min / 2,
    theta_min = dtheta / 2 and dphi = dtheta (phi cells = 2 theta cells)."""
    g = gold["timestep_gain"]
    for dims, key, tol in ((2, "gain_2d", "tol_2d"), (3, "gain_3d", "tol_3d")):
        m = og.mesh(g["ntheta"], g["r_core"], g["r_radial"], dims=dims)
        r, th, ph = m["r_edges"], m["theta_edges"], m["phi_edges"]
        rmin = 0.5 * (r[0] + r[1])
        dr_min = m["dr_min"]
        if dims == 2:
            gain = dr_min / (rmin * (th[1] - th[0]))
            assert ph.size == 2
        else:
            gain = dr_min / (rmin * math.sin(0.5 * (th[0] + th[1])) * (ph[1] - ph[0]))
            assert ph.size - 1 == 2 * (th.size - 1)
        assert abs(gain - g[key]) <= g[tol], (dims, gain)
        # the innermost cell is coarsened up to the cap, so its factors are the
        # full theta (and phi) extents of the shell
        assert m["c_theta"][0] == og.pow2_cap(th.size - 1)


def test_tiny_mesh_group_sizes_worked_by_hand(gold):
    t = gold["tiny_mesh"]
    m = og.mesh(t["ntheta"], t["r_core"], t["r_radial"], dims=t["dims"])
    assert m["r_edges"].size - 1 == t["nr"] and m["ncore"] == t["ncore"]
    assert m["phi_edges"].size - 1 == t["nphi"]
    assert m["c_theta"].tolist() == t["c_theta"]
    assert m["c_phi"][12].tolist() == t["c_phi_shell12"]
    assert m["c_phi"][5].tolist() == t["c_phi_shell5"]
    assert m["class_block"][m["shell_class"][0]].max() + 1 == t["shell0_blocks"]


def _check_rule(m):
    r, th, ph = m["r_edges"], m["theta_edges"], m["phi_edges"]
    nr, nt, nph = r.size - 1, th.size - 1, ph.size - 1
    dr = m["dr_min"]
    cap_t, cap_p = og.pow2_cap(nt), og.pow2_cap(nph)
    dth, dph = math.pi / nt, 2 * math.pi / nph
    cb = m["class_block"].reshape(-1, nt, nph)
    for i in range(nr):
        rc = 0.5 * (r[i] + r[i + 1])
        ct = int(m["c_theta"][i])
        # sufficient (unless capped) and minimal
        assert ct * rc * dth >= dr or ct == cap_t
        assert ct == 1 or (ct // 2) * rc * dth < dr
        blk = cb[m["shell_class"][i]]
        for j0 in range(0, nt, ct):
            cps = set(m["c_phi"][i, j0:j0 + ct].tolist())
            assert len(cps) == 1
            cp = cps.pop()
            w = [rc * math.sin(0.5 * (th[j] + th[j + 1])) * dph for j in range(j0, j0 + ct)]
            assert cp == cap_p or all(cp * x >= dr for x in w)
            assert cp == 1 or any((cp // 2) * x < dr for x in w)
            # blocks are aligned ct x cp rectangles with one id each
            for k0 in range(0, nph, cp):
                ids = blk[j0:j0 + ct, k0:k0 + cp]
                assert (ids == ids[0, 0]).all()
        # distinct rectangles carry distinct ids, numbered by first member
        flat = blk.ravel()
        first = {}
        for q, b in enumerate(flat):
            first.setdefault(int(b), q)
        assert sorted(first) == list(range(len(first)))
        assert [first[b] for b in range(len(first))] == sorted(first.values())
        assert len(first) == sum(nph // int(m["c_phi"][i, j0]) for j0 in range(0, nt, ct))


@pytest.mark.parametrize("ntheta,dims", [(64, 3), (128, 2), (48, 3)])
def test_coarsening_rule_sufficient_minimal_and_tiling(ntheta, dims):
    m = og.mesh(ntheta, 0.25, 3.68, dims=dims)
    _check_rule(m)
    # outside the core r dtheta / dr_min >= pi N_core / N_theta ~ 2.45 > 1:
    # no polar grouping there
    assert (m["c_theta"][m["ncore"]:] == 1).all()
    # shells of one class share one pattern, distinct classes differ
    pats = {}
    for i, c in enumerate(m["shell_class"]):
        pats.setdefault(int(c), set()).add((int(m["c_theta"][i]), tuple(m["c_phi"][i].tolist())))
    assert all(len(v) == 1 for v in pats.values())
    assert len({next(iter(v)) for v in pats.values()}) == len(pats)


def test_one_dimensional_mesh_is_not_coarsened():
    m = og.mesh(64, 1.0, 2.0, dims=1)
    assert m["theta_edges"].size == 2 and m["phi_edges"].size == 2
    assert m["class_block"].shape == (1, 1) and (m["shell_class"] == 0).all()


def test_coarsening_threshold_override_changes_only_the_width():
    a = og.mesh(32, 1.0, 2.0, dr_coarsen=0.0)
    b = og.mesh(32, 1.0, 2.0, dr_coarsen=a["dr_min"])
    assert (a["c_phi"] == b["c_phi"]).all() and (a["c_theta"] == b["c_theta"]).all()
    c = og.mesh(32, 1.0, 2.0, dr_coarsen=4 * a["dr_min"])
    assert (c["c_theta"] >= a["c_theta"]).all() and (c["c_theta"] > a["c_theta"]).any()


# ---- block volume average ---------------------------------------------------

def _brute_coarsen(f, m):
    """Direct loops: for each shell and block, scan every cell for members."""
    r, th, ph = m["r_edges"], m["theta_edges"], m["phi_edges"]
    nr, nt, nph = f.shape
    out = np.empty_like(f)
    for i in range(nr):
        blk = m["class_block"][m["shell_class"][i]].reshape(nt, nph)
        for b in range(blk.max() + 1):
            num = den = 0.0
            cells = []
            for j in range(nt):
                for k in range(nph):
                    if blk[j, k] == b:
                        v = (r[i + 1] ** 3 - r[i] ** 3) / 3 * (math.cos(th[j]) - math.cos(th[j + 1])) * (ph[k + 1] - ph[k])
                        num += v * f[i, j, k]
                        den += v
                        cells.append((j, k))
            for j, k in cells:
                out[i, j, k] = num / den
    return out


def _field(m, seed=7):
    rng = np.random.default_rng(seed)
    shape = (m["r_edges"].size - 1, m["theta_edges"].size - 1, m["phi_edges"].size - 1)
    return rng.standard_normal(shape)


def test_coarsen_matches_brute_force_on_tiny_mesh():
    m = og.mesh(8, 1.0, 1.5, dims=3)
    f = _field(m)
    got = og.coarsen(f, m["r_edges"], m["theta_edges"], m["phi_edges"], m["shell_class"], m["class_block"])
    np.testing.assert_allclose(got, _brute_coarsen(f, m), rtol=1e-13, atol=1e-13)


def test_coarsen_conserves_leaves_constants_and_is_idempotent():
    m = og.mesh(32, 1.0, 1.5, dims=3)
    args = (m["r_edges"], m["theta_edges"], m["phi_edges"], m["shell_class"], m["class_block"])
    f = _field(m, 3)
    g = og.coarsen(f, *args)
    V = og.cell_volumes(m["r_edges"], m["theta_edges"], m["phi_edges"])
    # conservation of the volume integral, shell by shell
    np.testing.assert_allclose((V * g).sum(axis=(1, 2)), (V * f).sum(axis=(1, 2)), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(og.coarsen(g, *args), g, rtol=1e-13, atol=1e-14)
    c = np.full_like(f, 2.5)
    np.testing.assert_allclose(og.coarsen(c, *args), c, rtol=1e-14)
    # cells that are blocks of their own keep their value (to rounding of V f / V)
    for i in range(f.shape[0]):
        ids = m["class_block"][m["shell_class"][i]]
        counts = np.bincount(ids)
        single = (counts[ids] == 1).reshape(f.shape[1:])
        np.testing.assert_allclose(g[i][single], f[i][single], rtol=4e-16, atol=0)
    # the mean is volume-weighted, not a plain cell mean: a block spanning
    # theta rows of unequal solid angle gives a different value
    i = 1
    blk = m["class_block"][m["shell_class"][i]].reshape(f.shape[1:])
    rows = np.unique(np.nonzero(blk == blk[0, 0])[0])
    assert rows.size > 1
    members = blk == blk[0, 0]
    assert abs(g[i][members][0] - f[i][members].mean()) > 1e-6
