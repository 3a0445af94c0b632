"""Seeded synthetic inputs: meshes, coarsening-block maps and density fields.

This module holds no arithmetic of the solve itself.  It only builds the
inputs that the GPU library and the CPU oracle both consume: edge arrays,
block-id maps and densities.  Densities that need spherical harmonics take
them from SciPy, never from either implementation.

Workloads (all dimensionless, G = 1):

* ``spheroid`` -- 64 uniform shells on r in [0, 2], 32 x 64 uniform angular
  cells, lmax = 8; density 1 inside the homogeneous oblate spheroid with
  semi-axes a1 = 1 (equatorial) and a3 = 0.5 (polar), 0 outside, smoothed at
  the surface by the volume fraction of 4^3 coordinate sub-cells (the
  sub-grid smoothing of the paper's homogeneous-spheroid test, Sec. 3 and
  Sec. 3.1).
* ``production`` -- 512 log-spaced shells on [1e-3, 1], 128 x 256 angular
  cells, lmax = 16; density (1 + (r/0.05)^2)^-1.5 (1 + 0.01 sum_{l<=4} c Y),
  c ~ N(0, 1) from a seeded generator, Y the real orthonormal harmonics;
  coarsening blocks 4 x 4 in angle within 32 shells of the origin and 1 x 4
  (four phi cells) in the 8 theta rows next to each pole further out
  (the angular coarsening of Sec. 2.1, with a fixed rule).
* ``production_l32`` -- the same mesh and density with lmax = 32.
"""
import numpy as np

__all__ = [
    "Mesh", "uniform_edges", "log_edges", "spheroid_mesh", "spheroid_density",
    "production_mesh", "production_density", "production_merge", "real_ylm_coeffs",
    "random_mesh", "random_merge", "workload",
]


class Mesh:
    """Edges, lmax and optional coarsening maps of one spherical mesh."""

    def __init__(self, r_edges, theta_edges, phi_edges, lmax, shell_class=None, class_block=None,
                 G=1.0, name=""):
        self.r_edges = np.ascontiguousarray(r_edges, dtype=np.float64)
        self.theta_edges = np.ascontiguousarray(theta_edges, dtype=np.float64)
        self.phi_edges = np.ascontiguousarray(phi_edges, dtype=np.float64)
        self.lmax = int(lmax)
        self.shell_class = None if shell_class is None else np.ascontiguousarray(shell_class, np.int32)
        self.class_block = None if class_block is None else np.ascontiguousarray(class_block, np.int32)
        self.G = float(G)
        self.name = name

    @property
    def nr(self):
        return self.r_edges.size - 1

    @property
    def ntheta(self):
        return self.theta_edges.size - 1

    @property
    def nphi(self):
        return self.phi_edges.size - 1

    @property
    def shape(self):
        return (self.nr, self.ntheta, self.nphi)

    @property
    def ncells(self):
        return self.nr * self.ntheta * self.nphi

    @property
    def nmodes(self):
        return (self.lmax + 1) ** 2

    def with_lmax(self, lmax):
        return Mesh(self.r_edges, self.theta_edges, self.phi_edges, lmax, self.shell_class,
                    self.class_block, self.G, self.name)

    def oracle_kwargs(self):
        return dict(r_edges=self.r_edges, theta_edges=self.theta_edges, phi_edges=self.phi_edges,
                    lmax=self.lmax, G=self.G, shell_class=self.shell_class,
                    class_block=self.class_block)


def uniform_edges(lo, hi, n):
    return np.linspace(lo, hi, n + 1)


def log_edges(lo, hi, n):
    return lo * (hi / lo) ** (np.arange(n + 1) / n)


def spheroid_mesh(nr=64, ntheta=32, nphi=64, rmax=2.0, lmax=8):
    return Mesh(uniform_edges(0.0, rmax, nr), uniform_edges(0.0, np.pi, ntheta),
                uniform_edges(0.0, 2 * np.pi, nphi), lmax, name="spheroid")


def spheroid_density(mesh, a1=1.0, a3=0.5, rho0=1.0, nsub=4):
    """rho0 times the volume fraction of each cell inside r_perp^2/a1^2 + z^2/a3^2 < 1.

    Each cell is split into nsub equal coordinate intervals per dimension; a
    sub-cell counts as inside when its coordinate midpoint is strictly inside,
    and is weighted by its exact volume.
    """
    r, th, ph = mesh.r_edges, mesh.theta_edges, mesh.phi_edges
    t = (np.arange(nsub) + 0.5) / nsub
    s = np.arange(nsub + 1) / nsub

    def sub(edges):
        lo, hi = edges[:-1, None], edges[1:, None]
        mids = lo + (hi - lo) * t[None, :]
        sedges = lo + (hi - lo) * s[None, :]
        return mids, sedges

    rm, re = sub(r)
    tm, te = sub(th)
    pm, pe = sub(ph)
    vr = (re[:, 1:] ** 3 - re[:, :-1] ** 3) / 3.0            # [nr][nsub]
    vt = np.cos(te[:, :-1]) - np.cos(te[:, 1:])              # [nt][nsub]
    vp = pe[:, 1:] - pe[:, :-1]                              # [np][nsub]
    # inside test depends on r and theta only (axisymmetric body)
    R = rm[:, None, :, None]
    T = tm[None, :, None, :]
    rp2 = (R * np.sin(T)) ** 2
    z2 = (R * np.cos(T)) ** 2
    inside = (rp2 / a1 ** 2 + z2 / a3 ** 2) < 1.0           # [nr][nt][nsub_r][nsub_t]
    w = vr[:, None, :, None] * vt[None, :, None, :]
    frac_rt = (inside * w).sum(axis=(2, 3)) / w.sum(axis=(2, 3))
    # the phi sub-cells all share the same inside flag, so the fraction is phi independent
    rho = np.repeat(frac_rt[:, :, None], mesh.nphi, axis=2) * rho0
    return np.ascontiguousarray(rho)


def real_ylm(l, m, a, theta, phi):
    """Orthonormal real harmonic with the Condon-Shortley phase (SciPy)."""
    from scipy.special import sph_harm_y
    y = sph_harm_y(l, m, theta, phi)
    if m == 0:
        return y.real
    return np.sqrt(2.0) * (y.real if a == 0 else y.imag)


def real_ylm_coeffs(lmax, seed):
    """N(0,1) coefficients in collapsed (l, m, a) order: l^2, then (m, cos), (m, sin)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((lmax + 1) ** 2)


def _modes(lmax):
    out = []
    for l in range(lmax + 1):
        out.append((l, 0, 0))
        for m in range(1, l + 1):
            out.append((l, m, 0))
            out.append((l, m, 1))
    return out


def perturbation(theta_c, phi_c, coeffs, lmax):
    tt, pp = np.meshgrid(theta_c, phi_c, indexing="ij")
    s = np.zeros_like(tt)
    for c, (l, m, a) in zip(coeffs, _modes(lmax)):
        s += c * real_ylm(l, m, a, tt, pp)
    return s


def production_mesh(lmax=16, nr=512, ntheta=128, nphi=256, merged=True):
    mesh = Mesh(log_edges(1e-3, 1.0, nr), uniform_edges(0.0, np.pi, ntheta),
                uniform_edges(0.0, 2 * np.pi, nphi), lmax, name="production")
    if merged:
        mesh.shell_class, mesh.class_block = production_merge(nr, ntheta, nphi)
    return mesh


def production_merge(nr, ntheta, nphi, inner_shells=32, polar_rows=8, blk=4):
    """Coarsening blocks: class 0 (shells < inner_shells) groups blk x blk angular
    cells aligned at multiples of blk; class 1 groups blk phi cells in the
    polar_rows theta rows next to each pole and leaves the others single.
    Block ids are numbered in row-major order of each block's first cell."""
    assert ntheta % blk == 0 and nphi % blk == 0
    shell_class = np.where(np.arange(nr) < inner_shells, 0, 1).astype(np.int32)
    j = np.arange(ntheta)[:, None]
    k = np.arange(nphi)[None, :]
    key0 = (j // blk) * (nphi // blk) + (k // blk)
    polar = (j < polar_rows) | (j >= ntheta - polar_rows)
    key1 = np.where(polar, j * nphi + (k // blk) * blk, j * nphi + k)
    cb = np.stack([_renumber(key0), _renumber(key1)])
    return shell_class, cb.reshape(2, ntheta * nphi)


def _renumber(key):
    """Dense block ids 0.. in order of each block's first cell."""
    flat = key.reshape(-1)
    uniq, first, inv = np.unique(flat, return_index=True, return_inverse=True)
    rank = np.empty(uniq.size, np.int64)
    rank[np.argsort(first)] = np.arange(uniq.size)
    return rank[inv].astype(np.int32).reshape(key.shape)


def production_density(mesh, seed=2, lpert=4, eps=0.01, rc=0.05):
    r = 0.5 * (mesh.r_edges[:-1] + mesh.r_edges[1:])
    th = 0.5 * (mesh.theta_edges[:-1] + mesh.theta_edges[1:])
    ph = 0.5 * (mesh.phi_edges[:-1] + mesh.phi_edges[1:])
    radial = (1.0 + (r / rc) ** 2) ** -1.5
    ang = 1.0 + eps * perturbation(th, ph, real_ylm_coeffs(lpert, seed), lpert)
    return np.ascontiguousarray(radial[:, None, None] * ang[None, :, :])


def random_mesh(seed, nr, ntheta, nphi, lmax, r0=0.0, r1=1.0, jitter=0.3):
    """Non-uniform but monotone edges covering [r0, r1] x [0, pi] x [0, 2 pi]."""
    rng = np.random.default_rng(seed)

    def edges(lo, hi, n):
        w = 1.0 + jitter * (2 * rng.random(n) - 1)
        e = np.concatenate([[0.0], np.cumsum(w)])
        e = lo + (hi - lo) * e / e[-1]
        e[0], e[-1] = lo, hi
        return e

    return Mesh(edges(r0, r1, nr), edges(0.0, np.pi, ntheta), edges(0.0, 2 * np.pi, nphi), lmax,
                name="random%d" % seed)


def random_merge(seed, nr, ntheta, nphi, nclasses=3, max_group=5):
    """Arbitrary (non-rectangular) coarsening blocks: each class groups runs of
    up to max_group consecutive cells in flattened angular order."""
    rng = np.random.default_rng(seed)
    ncell = ntheta * nphi
    cb = np.empty((nclasses, ncell), np.int32)
    for c in range(nclasses):
        if c == 0:
            cb[c] = np.arange(ncell)
            continue
        sizes = rng.integers(1, max_group + 1, size=ncell)
        ids = np.repeat(np.arange(ncell), sizes)[:ncell]
        cb[c] = ids
    shell_class = rng.integers(0, nclasses, size=nr).astype(np.int32)
    return shell_class, cb


def random_density(seed, shape, positive=True):
    rng = np.random.default_rng(seed)
    x = rng.random(shape)
    return np.ascontiguousarray(x if positive else x - 0.5)


def batch_meshes(nfields=64, seed0=4000, nr=(128, 1024), ntheta=(32, 256), lmax=(8, 32), merged=True):
    """Uneven meshes of a batched solve: per field f (seed seed0 + f) draws, in
    this order, nr ~ U{nr}, ntheta ~ U over multiples of 4 in ntheta,
    nphi = 2 ntheta, lmax ~ U{lmax}; log-spaced shells on [1e-3, 1]; the
    production coarsening rule (shells < 32 and 8 polar rows, scaled down
    for small meshes)."""
    meshes = []
    for f in range(nfields):
        rng = np.random.default_rng(seed0 + f)
        n_r = int(rng.integers(nr[0], nr[1] + 1))
        n_t = 4 * int(rng.integers(ntheta[0] // 4, ntheta[1] // 4 + 1))
        L = int(rng.integers(lmax[0], lmax[1] + 1))
        m = Mesh(log_edges(1e-3, 1.0, n_r), uniform_edges(0.0, np.pi, n_t), uniform_edges(0.0, 2 * np.pi, 2 * n_t),
                 L, name="field%d" % f)
        if merged:
            m.shell_class, m.class_block = production_merge(n_r, n_t, 2 * n_t, inner_shells=min(32, n_r),
                                                            polar_rows=min(8, n_t // 4))
        meshes.append(m)
    return meshes


def batch_densities(meshes, seed0=4000):
    return [production_density(m, seed=seed0 + f) for f, m in enumerate(meshes)]


def large_mesh(nr=2048, ntheta=256, nphi=512, lmax=64):
    """Mesh of the repeated-solve workload: log-spaced shells on [1e-3, 1],
    uniform angles, the production coarsening rule."""
    mesh = Mesh(log_edges(1e-3, 1.0, nr), uniform_edges(0.0, np.pi, ntheta), uniform_edges(0.0, 2 * np.pi, nphi),
                lmax, name="large")
    mesh.shell_class, mesh.class_block = production_merge(nr, ntheta, nphi)
    return mesh


LARGE_LPERT, LARGE_SEED, LARGE_EPS, LARGE_RC, LARGE_MAX_ANGLE = 8, 5, 0.01, 0.05, 0.05


def radial_profile(mesh, rc=0.05):
    r = 0.5 * (mesh.r_edges[:-1] + mesh.r_edges[1:])
    return np.ascontiguousarray((1.0 + (r / rc) ** 2) ** -1.5)


def axis_angle(axis, angle):
    """Rotation matrix by `angle` about the unit vector `axis` (Rodrigues)."""
    x, y, z = axis
    K = np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])
    return np.eye(3) + np.sin(angle) * K + (1.0 - np.cos(angle)) * (K @ K)


def rotation_sequence(nsteps, seed=LARGE_SEED, max_angle=LARGE_MAX_ANGLE):
    """R_0 = I and R_t = Q_t R_{t-1} for t = 1..nsteps, Q_t a rotation by an
    angle ~ U[0, max_angle] about an axis uniform on the sphere (normalised
    Gaussian triple), all drawn from one seeded generator in step order.
    Returns [nsteps+1][3][3]."""
    rng = np.random.default_rng(seed + 1)
    R = np.eye(3)
    out = [R]
    for _ in range(nsteps):
        a = rng.standard_normal(3)
        a /= np.linalg.norm(a)
        R = axis_angle(a, rng.uniform(0.0, max_angle)) @ R
        out.append(R)
    return np.ascontiguousarray(np.array(out))


def perturbation_at(theta, phi, coeffs, lmax):
    """sum_n coeffs[n] Y_n(theta, phi) at arbitrary points (arrays of one shape)."""
    s = np.zeros_like(theta, dtype=np.float64)
    for c, (l, m, a) in zip(coeffs, _modes(lmax)):
        s += c * real_ylm(l, m, a, theta, phi)
    return s


def rotated_angular_factor(mesh, R, coeffs, lpert=LARGE_LPERT, eps=LARGE_EPS):
    """Host value of 1 + eps * perturbation(R^T u) at every cell centre
    direction u, [ntheta][nphi] (the angular factor of the repeated-solve
    density at rotation R)."""
    th = 0.5 * (mesh.theta_edges[:-1] + mesh.theta_edges[1:])
    ph = 0.5 * (mesh.phi_edges[:-1] + mesh.phi_edges[1:])
    tt, pp = np.meshgrid(th, ph, indexing="ij")
    u = np.stack([np.sin(tt) * np.cos(pp), np.sin(tt) * np.sin(pp), np.cos(tt)], axis=-1)
    v = u @ R          # rows of u times R = (R^T u)^T
    t2 = np.arccos(np.clip(v[..., 2], -1.0, 1.0))
    p2 = np.arctan2(v[..., 1], v[..., 0])
    return 1.0 + eps * perturbation_at(t2, p2, coeffs, lpert)


def workload(name):
    """(mesh, rho) of a named workload."""
    if name == "spheroid":
        m = spheroid_mesh()
        return m, spheroid_density(m)
    if name == "production":
        m = production_mesh(16)
        return m, production_density(m)
    if name == "production_l32":
        m = production_mesh(32)
        return m, production_density(m)
    raise KeyError(name)
