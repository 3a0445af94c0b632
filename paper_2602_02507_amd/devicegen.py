"""Binding of the device input generator (libmpole_workload.so,
include/mpole_workload.h): the rotated-perturbation density of the
repeated-solve workload, written on the GPU so that a sequence of solves on
an advected density can be captured in one HIP graph."""
import ctypes
import os

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.WL_LIB):
            _build.build()
        L = ctypes.CDLL(_build.WL_LIB)
        i32, vp = ctypes.c_int32, ctypes.c_void_p
        L.mpole_wl_rotated_density.argtypes = [i32, i32, i32, vp, vp, vp, i32, vp, ctypes.c_double, vp, vp, vp]
        L.mpole_wl_rotated_density.restype = ctypes.c_int
        _lib = L
    return _lib


class RotatedDensity:
    """rho = radial(r) * (1 + eps * sum_n coef[n] Y_n(R^T u)) on a mesh, with the
    rotations R of a sequence held on the device ([nsteps+1][3][3])."""

    def __init__(self, mesh, coef, rotations, eps, rc=0.05, device="cuda"):
        import numpy as np
        import torch
        from . import workloads as wl
        self.shape = (mesh.nr, mesh.ntheta, mesh.nphi)
        self.lpert = int(round(np.sqrt(len(coef)))) - 1
        assert (self.lpert + 1) ** 2 == len(coef)
        dev = torch.device(device)
        th = 0.5 * (mesh.theta_edges[:-1] + mesh.theta_edges[1:])
        ph = 0.5 * (mesh.phi_edges[:-1] + mesh.phi_edges[1:])
        f64 = dict(dtype=torch.float64, device=dev)
        self.radial = torch.tensor(wl.radial_profile(mesh, rc), **f64)
        self.theta_c = torch.tensor(th, **f64)
        self.phi_c = torch.tensor(ph, **f64)
        self.coef = torch.tensor(np.asarray(coef, np.float64), **f64)
        self.rot = torch.tensor(np.ascontiguousarray(rotations, np.float64).reshape(-1, 9), **f64)
        self.eps = float(eps)
        self.device = dev

    def write(self, rho, step, stream=None):
        """Enqueue rho (float64 [nr][ntheta][nphi], device) for rotation `step`."""
        import torch
        if tuple(rho.shape) != self.shape or rho.dtype != torch.float64 or not rho.is_contiguous():
            raise ValueError("rho must be contiguous float64 of shape %s" % (self.shape,))
        if not 0 <= step < self.rot.shape[0]:
            raise IndexError("rotation step %d outside [0, %d)" % (step, self.rot.shape[0]))
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        nr, nt, npf = self.shape
        rc = lib().mpole_wl_rotated_density(nr, nt, npf, self.radial.data_ptr(), self.theta_c.data_ptr(),
                                            self.phi_c.data_ptr(), self.lpert, self.coef.data_ptr(), self.eps,
                                            self.rot[step].data_ptr(), rho.data_ptr(), ctypes.c_void_p(s))
        if rc != 0:
            raise RuntimeError("mpole_wl_rotated_density failed with status %d" % rc)
