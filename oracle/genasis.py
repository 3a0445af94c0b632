"""GenASiS mesh, automatic angular coarsening and the block volume average --
TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  The GPU library never calls it and shares no code with
it.  Plain Python and numpy in FP64, written for checking by eye.

What it follows:

* Sec. 2.1 ("Mesh"): a core r < r_core of N_core shells of uniform width
  dr_min = r_core / N_core; outside it dr is proportional to r, so the
  polar/radial aspect ratio r dtheta / dr keeps the value it has at r_core;
  N_theta / N_core is a fixed ratio (32/25 in the paper) and the ratio
  R_radial = N_r / N_theta fixes the shell count.  Angular cells narrower
  than dr_min are grouped, per shell, into blocks of 2, 4, 8, ... cells along
  a dimension until the block is at least that wide: along theta by
  comparing r dtheta with dr_min, along phi by comparing r sin(theta) dphi.
* Sec. 2.3 ("Fluid Dynamics of Baryonic Matter"): the coarsening operation
  replaces the value of every cell of a block by the volume-weighted mean of
  the block, sum_j V_j K_j / sum_j V_j; the coarsening factor c_i of a cell
  in dimension i is the block's cell count in that dimension.
* Sec. 3 ("Tests"): the worked mesh parameters (r_core, N_theta, R_radial)
  and the resulting r_out, dr_min and time-step gains that pin this module.

Readings where the paper leaves a choice:

* N_core = N_theta / core_ratio rounded to the nearest integer (as
  floor(x + 0.5) of the FP64 quotient); N_r = floor(R_radial N_theta),
  evaluated as floor(R_radial * N_theta + 1e-9) so that products like
  2.3 * 100 do not lose a shell to rounding.
* Core edges r_i = r_core i / N_core; outer edges
  r_i = r_core (1 + 1/N_core)^(i - N_core), i.e. dr = r_inner / N_core.
* theta: N_theta uniform cells on [0, pi] (one cell in 1D); phi: 2 N_theta
  uniform cells on [0, 2 pi] in 3D, so dphi = dtheta (one cell otherwise).
* Widths are taken at the cell centre (coordinate midpoints, the reading
  under which the paper's time-step gains reproduce).
* A group size is the smallest power of two c with c * width >= dr_min,
  capped at the largest power of two that divides the cell count of that
  dimension (so blocks tile the shell).
* theta group sizes depend on the shell only (dtheta is uniform); the phi
  group size of a theta block is the largest any of its rows needs, i.e. it
  is set by the row nearest the axis, so that every member cell's coarsened
  azimuthal width reaches dr_min (each cell of a block uses the block's
  factors in the time-step bound of Sec. 2.3).
* Shells with the same block pattern form one class, numbered in order of
  their first shell; blocks are numbered in order of their first member cell
  (row-major j * nphi + k).
"""
import math

import numpy as np

PAPER_CORE_RATIO = 32.0 / 25.0


def sizes(ntheta, r_core, r_radial, dims=3, core_ratio=PAPER_CORE_RATIO):
    """(N_r, N_core, mesh theta cells, mesh phi cells)."""
    ncore = int(math.floor(ntheta / core_ratio + 0.5))
    nr = int(math.floor(r_radial * ntheta + 1e-9))
    nt = ntheta if dims >= 2 else 1
    nph = 2 * ntheta if dims == 3 else 1
    return nr, ncore, nt, nph


def edges(ntheta, r_core, r_radial, dims=3, core_ratio=PAPER_CORE_RATIO):
    """r, theta and phi edges of the mesh, and N_core."""
    nr, ncore, nt, nph = sizes(ntheta, r_core, r_radial, dims, core_ratio)
    r = []
    for i in range(nr + 1):
        if i <= ncore:
            r.append(r_core * i / ncore)
        else:
            r.append(r_core * (1.0 + 1.0 / ncore) ** (i - ncore))
    th = [math.pi * j / nt for j in range(nt + 1)]
    ph = [2.0 * math.pi * k / nph for k in range(nph + 1)]
    return np.array(r), np.array(th), np.array(ph), ncore


def pow2_cap(n):
    """Largest power of two dividing n."""
    c = 1
    while n % (2 * c) == 0:
        c *= 2
    return c


def group_size(width, dr, cap):
    """Smallest power of two c with c * width >= dr, at most cap."""
    c = 1
    while c * width < dr and c < cap:
        c *= 2
    return c


def shell_pattern(rc, nt, nph, dr):
    """Group sizes of one shell with centre radius rc: (c_theta, [c_phi of
    each theta block])."""
    dth = math.pi / nt
    dph = 2.0 * math.pi / nph
    c_theta = group_size(rc * dth, dr, pow2_cap(nt))
    c_phi = []
    for j0 in range(0, nt, c_theta):
        need = 1
        for j in range(j0, j0 + c_theta):
            thc = 0.5 * (math.pi * j / nt + math.pi * (j + 1) / nt)
            need = max(need, group_size(rc * math.sin(thc) * dph, dr, pow2_cap(nph)))
        c_phi.append(need)
    return c_theta, c_phi


def block_map(nt, nph, c_theta, c_phi):
    """[nt][nph] block ids of one pattern, numbered by first member cell."""
    m = np.full((nt, nph), -1, dtype=np.int32)
    nb = 0
    for jb, j0 in enumerate(range(0, nt, c_theta)):
        for k0 in range(0, nph, c_phi[jb]):
            m[j0:j0 + c_theta, k0:k0 + c_phi[jb]] = nb
            nb += 1
    return m


def mesh(ntheta, r_core, r_radial, dims=3, core_ratio=PAPER_CORE_RATIO, dr_coarsen=0.0):
    """The whole mesh: dict with r_edges, theta_edges, phi_edges, ncore,
    dr_min, shell_class [nr], class_block [nclasses][nt*nph], c_theta [nr],
    c_phi [nr][nt] (the phi factor of the block holding each row)."""
    r, th, ph, ncore = edges(ntheta, r_core, r_radial, dims, core_ratio)
    nr, nt, nph = r.size - 1, th.size - 1, ph.size - 1
    dr_min = r_core / ncore
    dr = dr_coarsen if dr_coarsen > 0 else dr_min
    classes = {}
    maps = []
    shell_class = np.zeros(nr, dtype=np.int32)
    c_theta = np.zeros(nr, dtype=np.int32)
    c_phi = np.zeros((nr, nt), dtype=np.int32)
    for i in range(nr):
        rc = 0.5 * (r[i] + r[i + 1])
        ct, cp = shell_pattern(rc, nt, nph, dr)
        key = (ct, tuple(cp))
        if key not in classes:
            classes[key] = len(maps)
            maps.append(block_map(nt, nph, ct, cp).ravel())
        shell_class[i] = classes[key]
        c_theta[i] = ct
        for jb, j0 in enumerate(range(0, nt, ct)):
            c_phi[i, j0:j0 + ct] = cp[jb]
    return dict(r_edges=r, theta_edges=th, phi_edges=ph, ncore=ncore, dr_min=dr_min,
                shell_class=shell_class, class_block=np.stack(maps).astype(np.int32),
                c_theta=c_theta, c_phi=c_phi)


def cell_volumes(r_edges, theta_edges, phi_edges):
    """[nr][nt][nph] exact cell volumes (r^3/3 times cos difference times dphi)."""
    r = np.asarray(r_edges)
    th = np.asarray(theta_edges)
    ph = np.asarray(phi_edges)
    vr = (r[1:] ** 3 - r[:-1] ** 3) / 3.0
    vt = np.cos(th[:-1]) - np.cos(th[1:])
    vp = ph[1:] - ph[:-1]
    return vr[:, None, None] * vt[None, :, None] * vp[None, None, :]


def coarsen(field, r_edges, theta_edges, phi_edges, shell_class, class_block):
    """Block volume average (Sec. 2.3): each cell of a block gets
    sum_j V_j K_j / sum_j V_j over the block's members j in its shell."""
    f = np.asarray(field, dtype=np.float64)
    nr, nt, nph = f.shape
    V = cell_volumes(r_edges, theta_edges, phi_edges)
    out = np.empty_like(f)
    cb = np.asarray(class_block).reshape(-1, nt * nph)
    for i in range(nr):
        ids = cb[shell_class[i]]
        w = V[i].ravel()
        num = np.bincount(ids, weights=w * f[i].ravel())
        den = np.bincount(ids, weights=w)
        out[i] = (num / den)[ids].reshape(nt, nph)
    return out
