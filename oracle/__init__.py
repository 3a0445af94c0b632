"""FP64 CPU oracle for the multipole Poisson solve -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never calls it and shares no code with
it.  The arithmetic lives in mpole_oracle.c (plain C, FP64, sums in ascending
index order); this module only marshals numpy arrays through ctypes.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        c_int, c_double = ctypes.c_int, ctypes.c_double
        L.oracle_legendre.argtypes = [c_int, c_double, dp]
        L.oracle_theta_average.argtypes = [c_int, c_double, c_double, dp]
        L.oracle_theta_average.restype = c_int
        L.oracle_phi_average.argtypes = [c_int, c_double, c_double, dp, dp]
        L.oracle_radial.argtypes = [c_int, c_double, c_double, dp, dp, dp]
        L.oracle_angular_tables.argtypes = [c_int, c_int, c_int, dp, dp, dp, dp, dp, dp, dp]
        L.oracle_angular_tables.restype = c_int
        L.oracle_mode_index.argtypes = [c_int, c_int, c_int]
        L.oracle_mode_index.restype = c_int
        L.oracle_solve.argtypes = [c_int, c_int, c_int, c_int, dp, dp, dp, c_double, c_int, ip, ip,
                                   dp, dp, dp, dp, dp, dp, dp]
        L.oracle_solve.restype = c_int
        L.oracle_gradient.argtypes = [c_int, c_int, c_int, dp, dp, dp, dp, dp, dp, dp]
        L.oracle_set_threads.argtypes = [c_int]
        L.oracle_set_threads.restype = c_int
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def n_modes(lmax):
    return (lmax + 1) ** 2


def plm_index(l, m):
    return l * (l + 1) // 2 + m


def mode_index(l, m, a):
    """Collapsed index of (l, m, a), a = 0 cosine / 1 sine."""
    return lib().oracle_mode_index(l, m, a)


def legendre(lmax, theta):
    """P~_l^m(cos theta) for all 0 <= m <= l <= lmax, triangular order."""
    out = np.zeros((lmax + 1) * (lmax + 2) // 2)
    lib().oracle_legendre(lmax, float(theta), _dp(out))
    return out


def theta_average(lmax, th0, th1):
    out = np.zeros((lmax + 1) * (lmax + 2) // 2)
    k = lib().oracle_theta_average(lmax, float(th0), float(th1), _dp(out))
    return out, k


def phi_average(lmax, ph0, ph1):
    c = np.zeros(lmax + 1)
    s = np.zeros(lmax + 1)
    lib().oracle_phi_average(lmax, float(ph0), float(ph1), _dp(c), _dp(s))
    return c, s


def radial(lmax, r0, r1):
    JR = np.zeros(lmax + 1)
    JI = np.zeros(lmax + 1)
    V3 = np.zeros(1)
    lib().oracle_radial(lmax, float(r0), float(r1), _dp(JR), _dp(JI), _dp(V3))
    return JR, JI, float(V3[0])


def angular_tables(theta_edges, phi_edges, lmax):
    th = np.ascontiguousarray(theta_edges, dtype=np.float64)
    ph = np.ascontiguousarray(phi_edges, dtype=np.float64)
    nt, npf = th.size - 1, ph.size - 1
    np_ = (lmax + 1) * (lmax + 2) // 2
    pavg = np.zeros((nt, np_))
    cavg = np.zeros((npf, lmax + 1))
    savg = np.zeros((npf, lmax + 1))
    dom = np.zeros((nt, npf))
    ak = np.zeros((nt, npf, n_modes(lmax)))
    k = lib().oracle_angular_tables(nt, npf, lmax, _dp(th), _dp(ph), _dp(pavg), _dp(cavg),
                                    _dp(savg), _dp(dom), _dp(ak))
    return dict(pavg=pavg, cavg=cavg, savg=savg, domega=dom, akern=ak, romberg_levels=k)


def solve(r_edges, theta_edges, phi_edges, lmax, rho, G=1.0, shell_class=None, class_block=None):
    """Full FP64 solve.  Returns dict(phi, ang, interior, exterior, coef, seconds);
    seconds = (table construction, solve proper) wall times."""
    r = np.ascontiguousarray(r_edges, dtype=np.float64)
    th = np.ascontiguousarray(theta_edges, dtype=np.float64)
    ph = np.ascontiguousarray(phi_edges, dtype=np.float64)
    nr, nt, npf = r.size - 1, th.size - 1, ph.size - 1
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    assert rho.shape == (nr, nt, npf)
    nam = n_modes(lmax)
    if class_block is not None:
        cb = np.ascontiguousarray(class_block, dtype=np.int32).reshape(-1, nt * npf)
        sc = np.ascontiguousarray(shell_class, dtype=np.int32)
        assert sc.shape == (nr,)
        ncls = cb.shape[0]
    else:
        cb = sc = None
        ncls = 0
    phi = np.zeros((nr, nt, npf))
    ang = np.zeros((nr, nam))
    itr = np.zeros((nr + 1, nam))
    ext = np.zeros((nr + 1, nam))
    coef = np.zeros((nr, nam))
    sec = np.zeros(2)
    lib().oracle_solve(nr, nt, npf, lmax, _dp(r), _dp(th), _dp(ph), float(G), ncls, _ip(sc), _ip(cb),
                       _dp(rho), _dp(phi), _dp(ang), _dp(itr), _dp(ext), _dp(coef), _dp(sec))
    return dict(phi=phi, ang=ang, interior=itr, exterior=ext, coef=coef, seconds=(sec[0], sec[1]))


def gradient(r_edges, theta_edges, phi_edges, phi):
    """Centred-difference coordinate derivatives (dPhi/dr, dPhi/dtheta,
    dPhi/dphi) at cell centres, each [nr][ntheta][nphi] (Sec. 3 source terms)."""
    r = np.ascontiguousarray(r_edges, dtype=np.float64)
    th = np.ascontiguousarray(theta_edges, dtype=np.float64)
    ph = np.ascontiguousarray(phi_edges, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    shape = (r.size - 1, th.size - 1, ph.size - 1)
    assert phi.shape == shape
    out = [np.zeros(shape) for _ in range(3)]
    lib().oracle_gradient(shape[0], shape[1], shape[2], _dp(r), _dp(th), _dp(ph), _dp(phi), *[_dp(o) for o in out])
    return tuple(out)


def gravity_sources(r_edges, theta_edges, phi_edges, phi, rho, v_r=None, v_theta=None, v_phi=None):
    """Gravitational sources of the balance equations (Sec. 3): the momentum
    covector source -rho grad Phi, i.e. -rho dPhi/dx^i for x = (r, theta,
    phi), and the energy source -rho v . grad Phi = -rho sum_i v^i dPhi/dx^i
    with v the contravariant velocity components (a missing component is
    zero); the derivatives are the centred differences of gradient()."""
    g = gradient(r_edges, theta_edges, phi_edges, phi)
    rho = np.asarray(rho, dtype=np.float64)
    s = tuple(-rho * gi for gi in g)
    e = np.zeros_like(rho)
    for v, gi in zip((v_r, v_theta, v_phi), g):
        if v is not None:
            e = e + np.asarray(v, dtype=np.float64) * gi
    return s + (-rho * e,)


def threads():
    """OpenMP threads the oracle's parallel regions use."""
    return lib().oracle_set_threads(0)


def set_threads(n):
    """Set the oracle's OpenMP thread count (n >= 1); returns the count in effect."""
    return lib().oracle_set_threads(int(n))
