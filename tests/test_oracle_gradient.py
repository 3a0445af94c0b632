"""Pins of the oracle's centred-difference gradient (Sec. 3 source terms):
exact on linear functions on any mesh (interior and one-sided edges), exact on
quadratics in the interior of a uniform mesh, the closed form of the centred
difference of cos(phi) across the periodic seam, zero in single-cell
dimensions, and second-order convergence of dPhi/dr to GM/r^2 outside a
uniform sphere solved by the oracle itself."""
import numpy as np

import oracle


def centres(e):
    return 0.5 * (e[1:] + e[:-1])


def grid(r, th, ph):
    return np.meshgrid(centres(r), centres(th), centres(ph), indexing="ij")


def test_linear_function_exact_everywhere_on_nonuniform_mesh():
    rng = np.random.default_rng(11)
    r = np.cumsum(np.r_[0.05, rng.random(9) + 0.1])
    th = np.sort(np.r_[0.0, rng.random(7) * np.pi, np.pi])
    ph = np.sort(np.r_[0.0, rng.random(5) * 4.0, 4.0])   # does not close the circle: one-sided seam
    R, T, P = grid(r, th, ph)
    dr, dth, dph = oracle.gradient(r, th, ph, 1.5 * R - 0.25 * T + 3.0 * P + 7.0)
    assert np.abs(dr - 1.5).max() < 1e-13
    assert np.abs(dth + 0.25).max() < 1e-13
    assert np.abs(dph - 3.0).max() < 1e-13


def test_quadratic_in_radius_on_uniform_mesh():
    r = np.linspace(0.0, 2.0, 17)
    th = np.linspace(0.0, np.pi, 5)
    ph = np.linspace(0.0, 2 * np.pi, 7)
    R, T, P = grid(r, th, ph)
    dr, dth, dph = oracle.gradient(r, th, ph, R ** 2)
    rc = centres(r)
    # interior: centred difference of a quadratic is exact
    assert np.abs(dr[1:-1] - 2 * R[1:-1]).max() < 1e-13
    # edges: one-sided difference (r1^2 - r0^2)/(r1 - r0) = r1 + r0
    assert np.abs(dr[0] - (rc[0] + rc[1])).max() < 1e-13
    assert np.abs(dr[-1] - (rc[-1] + rc[-2])).max() < 1e-13
    assert np.abs(dth).max() == 0.0 and np.abs(dph).max() == 0.0


def test_periodic_seam_closed_form():
    nphi = 12
    r = np.array([1.0, 2.0])
    th = np.array([0.0, np.pi])
    ph = np.linspace(0.0, 2 * np.pi, nphi + 1)
    R, T, P = grid(r, th, ph)
    _, _, dph = oracle.gradient(r, th, ph, np.cos(P))
    h = 2 * np.pi / nphi
    want = -np.sin(P) * np.sin(h) / h     # (cos(x+h) - cos(x-h)) / 2h
    assert np.abs(dph - want).max() < 1e-14


def test_single_cell_dimensions_have_zero_derivative():
    r = np.array([0.5, 1.0])
    th = np.array([0.0, np.pi])
    ph = np.array([0.0, 2 * np.pi])
    d = oracle.gradient(r, th, ph, np.full((1, 1, 1), 3.0))
    assert all(np.all(x == 0.0) for x in d)


def test_radial_gradient_outside_uniform_sphere_converges_to_gm_over_r2():
    # oracle potential of a uniform sphere of radius 1 (density 1, G = 1):
    # outside, dPhi/dr -> G M / r^2 with the second-order centred difference
    errs = []
    for nr in (40, 80):
        r = np.linspace(0.0, 2.0, nr + 1)
        th = np.linspace(0.0, np.pi, 5)
        ph = np.linspace(0.0, 2 * np.pi, 5)
        rc = centres(r)
        rho = np.zeros((nr, 4, 4))
        rho[r[1:] <= 1.0] = 1.0
        mass = 4 * np.pi / 3 * (r[1:][r[1:] <= 1.0][-1]) ** 3
        sol = oracle.solve(r, th, ph, 0, rho)
        dr, _, _ = oracle.gradient(r, th, ph, sol["phi"])
        out = (rc > 1.2) & (np.arange(nr) < nr - 1)
        errs.append(np.max(np.abs(dr[out, 0, 0] - mass / rc[out] ** 2) / (mass / rc[out] ** 2)))
    assert errs[1] < errs[0] / 3.0, errs
    assert errs[1] < 1e-3, errs


def test_gravity_sources_definition_and_closed_forms():
    """-rho grad Phi and -rho v . grad Phi: on a potential linear in r,
    theta and phi the sources are -rho times the slopes (exactly), the
    energy source is -rho (v^r a + v^theta b + v^phi c); a velocity along
    the level sets of Phi (v . grad Phi = 0) gives no energy source, and a
    missing velocity component counts as zero."""
    rng = np.random.default_rng(5)
    r = np.cumsum(np.r_[0.1, rng.random(6) + 0.2])
    th = np.sort(np.r_[0.0, rng.random(5) * np.pi, np.pi])
    ph = np.linspace(0.0, 3.0, 6)
    R, T, P = grid(r, th, ph)
    a, b, c = 0.7, -1.3, 0.4
    phi = a * R + b * T + c * P
    rho = 1.0 + rng.random(R.shape)
    vr, vt, vp = rng.standard_normal((3,) + R.shape)
    sr, st, sp, se = oracle.gravity_sources(r, th, ph, phi, rho, vr, vt, vp)
    assert np.abs(sr + rho * a).max() < 1e-12
    assert np.abs(st + rho * b).max() < 1e-12
    assert np.abs(sp + rho * c).max() < 1e-12
    assert np.abs(se + rho * (vr * a + vt * b + vp * c)).max() < 1e-12
    # v^r = -b s, v^theta = a s: tangent to the level sets of a r + b theta
    s = rng.random(R.shape)
    _, _, _, se0 = oracle.gravity_sources(r, th, ph, a * R + b * T, rho, -b * s, a * s, None)
    assert np.abs(se0).max() < 1e-12
    _, _, _, se1 = oracle.gravity_sources(r, th, ph, phi, rho, None, None, None)
    assert (se1 == 0).all()
