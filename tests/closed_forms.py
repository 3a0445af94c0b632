"""Closed-form potentials used to pin the oracle (test-side only, G = 1 units
unless a G argument is given).

* Homogeneous oblate spheroid, interior and exterior (the paper's Sec. 3.1,
  Eq. SpheroidPotential with the I, A1, A3 and lambda definitions that follow
  it), with the uniform sphere as its e -> 0 special case.
* The exterior multipole series of the same spheroid,
  Phi = -G M / r sum_n (-1)^n 3 (a1 e / r)^(2n) P_2n(cos th) / ((2n+1)(2n+3)),
  an independent textbook expansion used to check the closed form.
"""
import numpy as np
from scipy.special import eval_legendre


def spheroid_coeffs(e):
    """I, A1, A3 of the paper's spheroid formula.

    Below e = 1e-2 the closed forms cancel badly in double precision, so they
    are evaluated with 50-digit mpmath arithmetic instead (same formulas)."""
    e = float(e)
    if e == 0.0:
        return 2.0, 2.0 / 3.0, 2.0 / 3.0
    if e < 1e-2:
        import mpmath as mp
        with mp.workdps(50):
            E = mp.mpf(e)
            s = mp.sqrt(1 - E * E)
            ase = mp.asin(E) / E
            return (float(2 * s * ase), float(s / E ** 2 * (ase - s)),
                    float(2 * s / E ** 2 * (1 / s - ase)))
    s = np.sqrt(1.0 - e * e)
    ase = np.arcsin(e) / e
    I = 2.0 * s * ase
    A1 = s / e ** 2 * (ase - s)
    A3 = 2.0 * s / e ** 2 * (1.0 / s - ase)
    return I, A1, A3


def spheroid_lambda(rp2, z2, a1, a3):
    """Positive root of rp2/(a1^2+l) + z2/(a3^2+l) = 1 (exterior points)."""
    b = a1 ** 2 + a3 ** 2 - rp2 - z2
    c = a1 ** 2 * a3 ** 2 - rp2 * a3 ** 2 - z2 * a1 ** 2
    disc = np.sqrt(np.maximum(b * b - 4.0 * c, 0.0))
    # larger root of l^2 + b l + c = 0, evaluated without cancellation
    return np.where(b > 0, 2.0 * (-c) / (b + disc), 0.5 * (-b + disc))


def spheroid_potential(rp, z, a1, a3, rho, G=1.0):
    """Potential of a homogeneous oblate spheroid (a1 >= a3) at cylindrical (rp, z)."""
    rp = np.asarray(rp, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    rp2, z2 = rp * rp, z * z
    inside = rp2 / a1 ** 2 + z2 / a3 ** 2 <= 1.0
    e = np.sqrt(1.0 - a3 ** 2 / a1 ** 2)
    I, A1, A3 = spheroid_coeffs(e)
    out = np.empty(np.broadcast(rp, z).shape)
    phin = -np.pi * G * rho * (I * a1 ** 2 - A1 * rp2 - A3 * z2)
    lam = spheroid_lambda(rp2, z2, a1, a3)
    ap1 = np.sqrt(a1 ** 2 + lam)
    ap3 = np.sqrt(a3 ** 2 + lam)
    phout = np.empty_like(out)
    flat_ap1, flat_ap3 = np.broadcast_to(ap1, out.shape).ravel(), np.broadcast_to(ap3, out.shape).ravel()
    frp2, fz2 = np.broadcast_to(rp2, out.shape).ravel(), np.broadcast_to(z2, out.shape).ravel()
    po = phout.ravel()
    for q in range(po.size):
        b1, b3 = flat_ap1[q], flat_ap3[q]
        ep = np.sqrt(max(1.0 - b3 * b3 / (b1 * b1), 0.0))
        Ip, A1p, A3p = spheroid_coeffs(ep)
        po[q] = -np.pi * G * rho * a1 ** 2 * a3 / (b1 ** 2 * b3) * (Ip * b1 ** 2 - A1p * frp2[q] - A3p * fz2[q])
    return np.where(inside, phin, phout)


def sphere_potential(r, R, rho, G=1.0):
    r = np.asarray(r, dtype=np.float64)
    return np.where(r <= R, -2.0 * np.pi * G * rho * (R * R - r * r / 3.0),
                    -4.0 * np.pi * G * rho * R ** 3 / (3.0 * np.maximum(r, 1e-300)))


def spheroid_mass(a1, a3, rho):
    return 4.0 / 3.0 * np.pi * rho * a1 * a1 * a3


def spheroid_axes_from_mass(M, rho, e):
    """Semi-axes (a1, a3) of a spheroid of mass M, density rho, eccentricity e."""
    s = np.sqrt(1.0 - e * e)
    a1 = (3.0 * M / (4.0 * np.pi * rho * s)) ** (1.0 / 3.0)
    return a1, a1 * s


def spheroid_exterior_series(r, theta, a1, a3, rho, nmax, G=1.0):
    """Exterior multipole series of the homogeneous spheroid, terms n = 0..nmax."""
    e = np.sqrt(1.0 - a3 ** 2 / a1 ** 2)
    M = spheroid_mass(a1, a3, rho)
    x = np.cos(theta)
    s = np.zeros(np.broadcast(r, theta).shape)
    for n in range(nmax + 1):
        s = s + (-1) ** n * 3.0 * (a1 * e / r) ** (2 * n) * eval_legendre(2 * n, x) / ((2 * n + 1) * (2 * n + 3))
    return -G * M / r * s
