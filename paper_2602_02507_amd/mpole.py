"""Python binding of the mpole C ABI (include/mpole.h).

Argument marshalling only: every step of the solve runs in the gfx950 HIP
kernels of libmpole.so.  PyTorch supplies device memory (the workspace and
output tensors) and the HIP stream; nothing here computes any part of the
method, and there is no CPU fallback -- without the built library or a GPU
every call raises.
"""
import ctypes
import os

import numpy as np

from . import build as _build

FP64, BF16X3, FP16X2, FP64_SEPARABLE, BF16X3_SEPARABLE = 0, 1, 2, 3, 4
_PRECISIONS = {"fp64": FP64, "bf16x3": BF16X3, "fp16x2": FP16X2, "fp64sep": FP64_SEPARABLE,
               "bf16x3sep": BF16X3_SEPARABLE}

STATUS = {0: "MPOLE_OK", 1: "MPOLE_ERR_INVALID", 2: "MPOLE_ERR_RANGE", 3: "MPOLE_ERR_WORKSPACE",
          4: "MPOLE_ERR_DEVICE", 5: "MPOLE_ERR_UNSUPPORTED"}

# every entry point include/mpole.h declares
EXPORTS = ("mpole_abi_version", "mpole_last_error", "mpole_plan_create", "mpole_plan_workspace_bytes",
           "mpole_plan_nmodes", "mpole_plan_folded", "mpole_plan_bind", "mpole_solve", "mpole_solve_static", "mpole_plan_copy_table",
           "mpole_plan_set_timing", "mpole_plan_phase_ms", "mpole_plan_work", "mpole_gradient", "mpole_gravity_sources", "mpole_coarsen",
           "mpole_genasis_shape", "mpole_genasis_build", "mpole_plan_tune",
           "mpole_plan_get_tuning", "mpole_plan_configure", "mpole_plan_moment_wgs", "mpole_plan_destroy",
           "mpole_batch_create", "mpole_batch_tune", "mpole_batch_configure", "mpole_batch_get_tuning",
           "mpole_batch_workspace_bytes",
           "mpole_batch_bind",
           "mpole_batch_solve", "mpole_batch_field_ms", "mpole_batch_destroy", "mpole_batch_set_launch",
           "mpole_batch_launch", "mpole_batch_launch_note", "mpole_batch_check")
LAUNCH_PHASES, LAUNCH_PERSISTENT, LAUNCH_PERSISTENT_FORCED = 0, 1, 2
PHASES = ("pack", "moment", "reduce", "scan", "split", "expand", "bcast")


class Tuning(ctypes.Structure):
    """Launch tuning of the two contractions (mpole_tuning); zeros mean defaults."""
    _fields_ = [("moment_wgs", ctypes.c_int32), ("moment_tile_m", ctypes.c_int32),
                ("expand_tile_m", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}

    @classmethod
    def of(cls, t):
        """Tuning from a Tuning, a dict with some of the three keys, or None (defaults)."""
        if isinstance(t, cls):
            return t
        t = dict(t or {})
        return cls(int(t.get("moment_wgs", 0)), int(t.get("moment_tile_m", 0)), int(t.get("expand_tile_m", 0)))


class MpoleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code


class GenasisC(ctypes.Structure):
    """GenASiS mesh parameters (mpole_genasis)."""
    _fields_ = [("dims", ctypes.c_int32), ("ntheta", ctypes.c_int32), ("r_core", ctypes.c_double),
                ("core_ratio", ctypes.c_double), ("r_radial", ctypes.c_double), ("dr_coarsen", ctypes.c_double)]


class MeshC(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("ntheta", ctypes.c_int32), ("nphi", ctypes.c_int32),
                ("lmax", ctypes.c_int32),
                ("r_edges", ctypes.POINTER(ctypes.c_double)),
                ("theta_edges", ctypes.POINTER(ctypes.c_double)),
                ("phi_edges", ctypes.POINTER(ctypes.c_double)),
                ("nclasses", ctypes.c_int32),
                ("shell_class", ctypes.POINTER(ctypes.c_int32)),
                ("class_block", ctypes.POINTER(ctypes.c_int32)),
                ("G", ctypes.c_double), ("precision", ctypes.c_int32)]


_lib = None


def library_path():
    """The library to load: $MPOLE_LIBRARY when set (e.g. a host-sanitized
    build of the same sources), else the in-tree libmpole.so."""
    return os.environ.get("MPOLE_LIBRARY") or _build.LIB


def lib():
    """Load libmpole.so (building it first only if it is absent)."""
    global _lib
    if _lib is None:
        path = library_path()
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        L.mpole_abi_version.restype = ctypes.c_int
        L.mpole_last_error.restype = ctypes.c_char_p
        L.mpole_plan_create.argtypes = [ctypes.POINTER(MeshC), ctypes.POINTER(vp)]
        L.mpole_plan_workspace_bytes.argtypes = [vp]
        L.mpole_plan_workspace_bytes.restype = sz
        L.mpole_plan_nmodes.argtypes = [vp]
        L.mpole_plan_folded.argtypes = [vp]
        L.mpole_plan_bind.argtypes = [vp, vp, sz, vp]
        L.mpole_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.mpole_solve_static.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.mpole_plan_copy_table.argtypes = [vp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_int64), vp]
        L.mpole_plan_set_timing.argtypes = [vp, ctypes.c_int]
        L.mpole_plan_phase_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        dptr = ctypes.POINTER(ctypes.c_double)
        L.mpole_plan_work.argtypes = [vp, dptr, dptr, dptr]
        L.mpole_gradient.argtypes = [vp, vp, vp, vp, vp, vp]
        L.mpole_coarsen.argtypes = [vp, vp, vp, vp]
        L.mpole_gravity_sources.argtypes = [vp] + [vp] * 10
        ip = ctypes.POINTER(ctypes.c_int32)
        L.mpole_genasis_shape.argtypes = [ctypes.POINTER(GenasisC), ip, ip, ip, ip, ip]
        L.mpole_genasis_build.argtypes = [ctypes.POINTER(GenasisC), dptr, dptr, dptr, ip, ip, ip, ip]
        L.mpole_plan_tune.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.mpole_plan_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.mpole_plan_configure.argtypes = [vp, ctypes.c_int32]
        L.mpole_plan_moment_wgs.argtypes = [vp]
        L.mpole_plan_destroy.argtypes = [vp]
        L.mpole_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(MeshC), ctypes.POINTER(vp)]
        L.mpole_batch_tune.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.mpole_batch_configure.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
        L.mpole_batch_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.mpole_batch_workspace_bytes.argtypes = [vp]
        L.mpole_batch_workspace_bytes.restype = sz
        L.mpole_batch_bind.argtypes = [vp, vp, sz, ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
        L.mpole_batch_solve.argtypes = [vp, vp]
        L.mpole_batch_field_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.mpole_batch_destroy.argtypes = [vp]
        L.mpole_batch_set_launch.argtypes = [vp, ctypes.c_int32, ctypes.c_uint32]
        L.mpole_batch_launch.argtypes = [vp]
        L.mpole_batch_launch_note.argtypes = [vp]
        L.mpole_batch_launch_note.restype = ctypes.c_char_p
        L.mpole_batch_check.argtypes = [vp, vp]
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise MpoleError(rc, lib().mpole_last_error().decode())


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype)) if a is not None else None


def _dev_ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def genasis_mesh(ntheta, r_core, r_radial, dims=3, core_ratio=0.0, dr_coarsen=0.0):
    """GenASiS mesh with automatic angular coarsening (mpole_genasis_build).
    Returns a dict of host arrays: r_edges, theta_edges, phi_edges,
    shell_class, class_block [nclasses][ntheta*nphi], c_theta [nr],
    c_phi [nr][ntheta], and the core shell count ncore."""
    g = GenasisC(int(dims), int(ntheta), float(r_core), float(core_ratio), float(r_radial), float(dr_coarsen))
    n = [ctypes.c_int32() for _ in range(5)]
    _check(lib().mpole_genasis_shape(ctypes.byref(g), *[ctypes.byref(x) for x in n]))
    nr, nt, nph, ncore, ncls = (x.value for x in n)
    out = dict(r_edges=np.empty(nr + 1), theta_edges=np.empty(nt + 1), phi_edges=np.empty(nph + 1),
               shell_class=np.empty(nr, np.int32), class_block=np.empty((ncls, nt * nph), np.int32),
               c_theta=np.empty(nr, np.int32), c_phi=np.empty((nr, nt), np.int32))
    d, i = ctypes.c_double, ctypes.c_int32
    _check(lib().mpole_genasis_build(ctypes.byref(g), _ptr(out["r_edges"], d), _ptr(out["theta_edges"], d),
                                     _ptr(out["phi_edges"], d), _ptr(out["shell_class"], i),
                                     _ptr(out["class_block"], i), _ptr(out["c_theta"], i), _ptr(out["c_phi"], i)))
    out["ncore"] = ncore
    return out


def make_mesh(r_edges, theta_edges, phi_edges, lmax, shell_class=None, class_block=None, G=1.0,
              precision="fp64"):
    """(MeshC, arrays to keep alive) for the C mesh descriptor."""
    keep = [np.ascontiguousarray(r_edges, np.float64), np.ascontiguousarray(theta_edges, np.float64),
            np.ascontiguousarray(phi_edges, np.float64)]
    r, th, ph = keep
    m = MeshC()
    m.nr, m.ntheta, m.nphi, m.lmax = r.size - 1, th.size - 1, ph.size - 1, int(lmax)
    m.r_edges, m.theta_edges, m.phi_edges = _ptr(r, ctypes.c_double), _ptr(th, ctypes.c_double), _ptr(ph, ctypes.c_double)
    if class_block is not None:
        cb = np.ascontiguousarray(class_block, np.int32).reshape(-1, m.ntheta * m.nphi)
        sc = np.ascontiguousarray(shell_class, np.int32)
        keep += [cb, sc]
        m.nclasses = cb.shape[0]
        m.shell_class, m.class_block = _ptr(sc, ctypes.c_int32), _ptr(cb, ctypes.c_int32)
    else:
        m.nclasses = 0
    m.G = float(G)
    m.precision = _PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return m, keep


class HostPlan:
    """A validated plan without device state (mpole_plan_create only)."""

    def __init__(self, r_edges, theta_edges, phi_edges, lmax, shell_class=None, class_block=None,
                 G=1.0, precision="fp64", moment_wgs=0, tuning=None):
        m, self._keep = make_mesh(r_edges, theta_edges, phi_edges, lmax, shell_class, class_block, G, precision)
        self.nr, self.ntheta, self.nphi, self.lmax = m.nr, m.ntheta, m.nphi, m.lmax
        self._mesh = m
        h = ctypes.c_void_p()
        _check(lib().mpole_plan_create(ctypes.byref(m), ctypes.byref(h)))
        self.handle = h
        self.nmodes = lib().mpole_plan_nmodes(h)
        self.folded = bool(lib().mpole_plan_folded(h))
        if moment_wgs:
            _check(lib().mpole_plan_configure(h, int(moment_wgs)))
        if tuning is not None:
            t = Tuning.of(tuning)
            _check(lib().mpole_plan_tune(h, ctypes.byref(t)))
        self.workspace_bytes = lib().mpole_plan_workspace_bytes(h)
        self.moment_wgs = lib().mpole_plan_moment_wgs(h)

    @classmethod
    def from_mesh(cls, mesh, precision="fp64", tuning=None):
        return cls(mesh.r_edges, mesh.theta_edges, mesh.phi_edges, mesh.lmax, mesh.shell_class,
                   mesh.class_block, mesh.G, precision, tuning=tuning)

    def tuning(self):
        """The plan's launch tuning in use, as a dict."""
        t = Tuning()
        _check(lib().mpole_plan_get_tuning(self.handle, ctypes.byref(t)))
        return t.as_dict()

    def work(self):
        """(moment flops, expansion flops, minimum HBM bytes) of one solve."""
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().mpole_plan_work(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def set_timing(self, enable):
        _check(lib().mpole_plan_set_timing(self.handle, int(bool(enable))))

    def phase_ms(self):
        """{phase: (total ms, launches)} since timing was enabled or last read."""
        ms = (ctypes.c_double * len(PHASES))()
        n = (ctypes.c_int64 * len(PHASES))()
        _check(lib().mpole_plan_phase_ms(self.handle, ms, n))
        return {PHASES[k]: (ms[k], n[k]) for k in range(len(PHASES))}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.mpole_plan_destroy(h)
            self.handle = None


class Plan(HostPlan):
    """Plan bound to a device workspace on a torch CUDA (HIP) device."""

    def __init__(self, *args, device="cuda", **kw):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("mpole needs a ROCm GPU; none is visible to torch")
        super().__init__(*args, **kw)
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device(dev.type, torch.cuda.current_device())
        self.device = dev
        self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().mpole_plan_bind(self.handle, ctypes.c_void_p(self._ws_ptr), self.workspace_bytes,
                                     ctypes.c_void_p(stream)))

    @classmethod
    def from_mesh(cls, mesh, precision="fp64", device="cuda", moment_wgs=0, tuning=None):
        return cls(mesh.r_edges, mesh.theta_edges, mesh.phi_edges, mesh.lmax, mesh.shell_class,
                   mesh.class_block, mesh.G, precision=precision, device=device, moment_wgs=moment_wgs,
                   tuning=tuning)

    @property
    def shape(self):
        return (self.nr, self.ntheta, self.nphi)

    def empty_outputs(self, phi=True, ang=True, interior=True, exterior=True):
        import torch
        f = lambda shp, want: torch.empty(shp, dtype=torch.float64, device=self.device) if want else None
        return dict(phi=f(self.shape, phi), ang=f((self.nr, self.nmodes), ang),
                    interior=f((self.nr + 1, self.nmodes), interior),
                    exterior=f((self.nr + 1, self.nmodes), exterior))

    def _check_tensor(self, t, shape, name):
        import torch
        if t is None:
            return
        if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.device:
            raise ValueError("%s must be a contiguous float64 tensor on %s" % (name, self.device))
        if tuple(t.shape) != tuple(shape):
            raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))

    def solve_into(self, rho, phi=None, ang=None, interior=None, exterior=None, stream=None):
        """Enqueue one solve writing into caller-provided tensors (any may be None but rho)."""
        import torch
        self._check_tensor(rho, self.shape, "rho")
        self._check_tensor(phi, self.shape, "phi")
        self._check_tensor(ang, (self.nr, self.nmodes), "ang")
        self._check_tensor(interior, (self.nr + 1, self.nmodes), "interior")
        self._check_tensor(exterior, (self.nr + 1, self.nmodes), "exterior")
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().mpole_solve(self.handle, _dev_ptr(rho), _dev_ptr(phi), _dev_ptr(ang), _dev_ptr(interior),
                                 _dev_ptr(exterior), ctypes.c_void_p(s)))

    def solve(self, rho, **want):
        out = self.empty_outputs(**want)
        self.solve_into(rho, **out)
        return out

    def gradient(self, phi, d_r=None, d_theta=None, d_phi=None, stream=None):
        """Centred-difference (dPhi/dr, dPhi/dtheta, dPhi/dphi) of a potential on
        this mesh (mpole_gradient); outputs allocated when not given."""
        import torch
        self._check_tensor(phi, self.shape, "phi")
        outs = []
        for t in (d_r, d_theta, d_phi):
            if t is None:
                t = torch.empty(self.shape, dtype=torch.float64, device=self.device)
            self._check_tensor(t, self.shape, "gradient output")
            outs.append(t)
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().mpole_gradient(self.handle, _dev_ptr(phi), *[_dev_ptr(t) for t in outs], ctypes.c_void_p(s)))
        return tuple(outs)

    def gravity_sources(self, phi, rho, v=(None, None, None), out=None, stream=None):
        """(-rho dPhi/dr, -rho dPhi/dtheta, -rho dPhi/dphi, -rho v . grad Phi)
        of a potential (mpole_gravity_sources); v = contravariant velocity
        components (None: zero); outputs allocated when out is None."""
        import torch
        self._check_tensor(phi, self.shape, "phi")
        self._check_tensor(rho, self.shape, "rho")
        for t in v:
            if t is not None:
                self._check_tensor(t, self.shape, "velocity")
        if out is None:
            out = tuple(torch.empty(self.shape, dtype=torch.float64, device=self.device) for _ in range(4))
        for t in out:
            if t is not None:
                self._check_tensor(t, self.shape, "source output")
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().mpole_gravity_sources(self.handle, _dev_ptr(phi), _dev_ptr(rho), *[_dev_ptr(t) for t in v],
                                           *[_dev_ptr(t) for t in out], ctypes.c_void_p(s)))
        return out

    def coarsen(self, field, out=None, stream=None):
        """Block volume average of a cell field over this mesh's coarsening
        blocks (mpole_coarsen); out may be field itself (in place)."""
        import torch
        self._check_tensor(field, self.shape, "field")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        self._check_tensor(out, self.shape, "coarsen output")
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().mpole_coarsen(self.handle, _dev_ptr(field), _dev_ptr(out), ctypes.c_void_p(s)))
        return out

    def table(self, cls=0):
        """FP64 block-mean kernel table of a coarsening class, [nblocks][nAM] (host numpy)."""
        import torch
        n = ctypes.c_int64()
        s = torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().mpole_plan_copy_table(self.handle, cls, None, ctypes.byref(n), ctypes.c_void_p(s)))
        out = np.empty((n.value, self.nmodes))
        _check(lib().mpole_plan_copy_table(self.handle, cls, out.ctypes.data_as(ctypes.c_void_p),
                                           ctypes.byref(n), ctypes.c_void_p(s)))
        return out


class Batch:
    """Many fields (uneven meshes, same precision) solved together: one
    persistent launch over per-XCD work queues where the batch allows it,
    else one launch per phase (`launch`: "persistent", "phases", or "forced" for
    persistent also on unbalanced queues).

    `meshes` are workloads.Mesh-like objects; rho/phi are per-field float64
    device tensors (phi allocated here when not given).  `solve()` enqueues one
    batch solve on the current stream (graph-capturable); `field_ms()` gives
    each field's completion time within the last solve after a sync;
    `check()` synchronises and raises if a dependency wait of the persistent
    launch gave up."""

    def __init__(self, meshes, precision="bf16x3", rho=None, device="cuda", moment_wgs=None, tunings=None,
                 launch="persistent", wait_polls=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("mpole needs a ROCm GPU; none is visible to torch")
        self.n = len(meshes)
        descs = (MeshC * self.n)()
        self._keep = []
        for f, mesh in enumerate(meshes):
            m, keep = make_mesh(mesh.r_edges, mesh.theta_edges, mesh.phi_edges, mesh.lmax, mesh.shell_class,
                                mesh.class_block, mesh.G, precision)
            descs[f] = m
            self._keep.append(keep)
        h = ctypes.c_void_p()
        _check(lib().mpole_batch_create(self.n, descs, ctypes.byref(h)))
        self.handle = h
        if moment_wgs is not None:
            arr = (ctypes.c_int32 * self.n)(*[int(x) for x in moment_wgs])
            _check(lib().mpole_batch_configure(h, arr))
        if tunings is not None:
            if len(tunings) != self.n:
                raise ValueError("one tuning per field")
            arr = (Tuning * self.n)(*[Tuning.of(t) for t in tunings])
            _check(lib().mpole_batch_tune(h, arr))
        self.set_launch(launch, wait_polls)
        dev = torch.device(device)
        if dev.index is None:
            dev = torch.device(dev.type, torch.cuda.current_device())
        self.device = dev
        self.shapes = [(m.nr, m.ntheta, m.nphi) for m in meshes]
        self.rho = rho if rho is not None else [torch.empty(s, dtype=torch.float64, device=dev) for s in self.shapes]
        self.phi = [torch.empty(s, dtype=torch.float64, device=dev) for s in self.shapes]
        for t, s in zip(self.rho, self.shapes):
            if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != s:
                raise ValueError("rho tensors must be contiguous float64 of the mesh shapes")
        self.workspace_bytes = lib().mpole_batch_workspace_bytes(h)
        self.workspace = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=dev)
        ws = (self.workspace.data_ptr() + 255) & ~255
        rp = (ctypes.c_void_p * self.n)(*[t.data_ptr() for t in self.rho])
        pp = (ctypes.c_void_p * self.n)(*[t.data_ptr() for t in self.phi])
        stream = torch.cuda.current_stream(dev).cuda_stream
        _check(lib().mpole_batch_bind(h, ctypes.c_void_p(ws), self.workspace_bytes, rp, pp, ctypes.c_void_p(stream)))

    def solve(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().mpole_batch_solve(self.handle, ctypes.c_void_p(s)))

    def set_launch(self, launch="persistent", wait_polls=0):
        """Launch of later solves ("persistent", "phases" or "forced": persistent
        also on unbalanced queues) and the dependency-wait budget of the
        persistent launch in polls (0: the library default)."""
        mode = {"phases": LAUNCH_PHASES, "persistent": LAUNCH_PERSISTENT, "forced": LAUNCH_PERSISTENT_FORCED}[launch]
        _check(lib().mpole_batch_set_launch(self.handle, mode, int(wait_polls)))

    @property
    def launch(self):
        """The launch the next solve runs: "persistent" or "phases"."""
        return "persistent" if lib().mpole_batch_launch(self.handle) == LAUNCH_PERSISTENT else "phases"

    @property
    def launch_note(self):
        """Why the batch does not launch persistent when asked to ("" if it does)."""
        return lib().mpole_batch_launch_note(self.handle).decode()

    def check(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().mpole_batch_check(self.handle, ctypes.c_void_p(s)))

    def tunings(self):
        """Per-field launch tunings in use, as dicts."""
        arr = (Tuning * self.n)()
        _check(lib().mpole_batch_get_tuning(self.handle, arr))
        return [t.as_dict() for t in arr]

    def field_ms(self):
        out = (ctypes.c_double * self.n)()
        _check(lib().mpole_batch_field_ms(self.handle, out))
        return list(out)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.mpole_batch_destroy(h)
            self.handle = None
