"""CPU checks of the input recipes that are not plain draws: the rotation
sequence of the repeated-solve workload and the host value of its rotated
perturbation (the reference for the device generator)."""
import numpy as np

from paper_2602_02507_amd import workloads as wl


def test_rotation_sequence_is_orthonormal_and_seeded():
    R = wl.rotation_sequence(50)
    assert R.shape == (51, 3, 3)
    assert np.allclose(R[0], np.eye(3))
    for t in (1, 25, 50):
        assert np.abs(R[t] @ R[t].T - np.eye(3)).max() < 1e-14
        assert abs(np.linalg.det(R[t]) - 1.0) < 1e-14
    # each step turns by at most the maximum angle
    for t in range(1, 51):
        Q = R[t] @ R[t - 1].T
        ang = np.arccos(np.clip((np.trace(Q) - 1) / 2, -1, 1))
        assert ang <= wl.LARGE_MAX_ANGLE + 1e-12
    assert np.array_equal(R, wl.rotation_sequence(50))


def test_rotated_factor_of_a_dipole_is_the_rotated_axis():
    # Y_10 = sqrt(3/4pi) z, so at R^T u it is sqrt(3/4pi) (R e_z) . u
    m = wl.production_mesh(2, nr=2, ntheta=12, nphi=24, merged=False)
    c = np.zeros(4)
    c[1] = 1.0   # (l, m) = (1, 0): index l^2
    R = wl.axis_angle(np.array([1.0, 2.0, 2.0]) / 3.0, 0.7)
    got = wl.rotated_angular_factor(m, R, c, lpert=1, eps=1.0) - 1.0
    th = 0.5 * (m.theta_edges[:-1] + m.theta_edges[1:])
    ph = 0.5 * (m.phi_edges[:-1] + m.phi_edges[1:])
    tt, pp = np.meshgrid(th, ph, indexing="ij")
    u = np.stack([np.sin(tt) * np.cos(pp), np.sin(tt) * np.sin(pp), np.cos(tt)], axis=-1)
    want = np.sqrt(3 / (4 * np.pi)) * (u @ (R @ np.array([0.0, 0.0, 1.0])))
    assert np.abs(got - want).max() < 1e-14


def test_rotation_preserves_the_perturbation_power():
    # rotations mix m within each l: sum over the sphere of the squared
    # perturbation (a rotation invariant) is unchanged, to quadrature accuracy
    m = wl.production_mesh(2, nr=2, ntheta=96, nphi=192, merged=False)
    c = wl.real_ylm_coeffs(4, 3)
    dom = (np.cos(m.theta_edges[:-1]) - np.cos(m.theta_edges[1:]))[:, None] * np.diff(m.phi_edges)[None, :]
    p0 = ((wl.rotated_angular_factor(m, np.eye(3), c, 4, 1.0) - 1) ** 2 * dom).sum()
    p1 = ((wl.rotated_angular_factor(m, wl.rotation_sequence(3)[3], c, 4, 1.0) - 1) ** 2 * dom).sum()
    assert abs(p0 - (c ** 2).sum()) < 2e-3 * p0
    assert abs(p1 - p0) < 2e-3 * p0
