"""ctypes binding of libisoadv.so: argument marshalling only.

Every step of the advection runs in the HIP kernels behind the C interface
(include/isoadv.h).  PyTorch supplies device memory and the current HIP stream.
If the library is not built this module raises at load time; there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libisoadv.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "isoadv.h")

ISO_OK, ISO_EINVAL, ISO_ENOMEM, ISO_EDEVICE, ISO_ENOSPACE, ISO_ECOURANT, ISO_EMESH, ISO_EUNSUPPORTED = range(8)
PATCH_WALL, PATCH_EMPTY, PATCH_INOUT, PATCH_CYCLIC = range(4)

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_vp = C.c_void_p


class IsoOptions(C.Structure):
    _fields_ = [("eps_surf", C.c_double), ("flat_tol", C.c_double), ("bound_tol", C.c_double),
                ("max_courant", C.c_double), ("root_max_iter", C.c_int32), ("n_bound_iter", C.c_int32),
                ("clip", C.c_int32), ("check_inputs", C.c_int32), ("block_cells", C.c_int32),
                ("surface_blocks", C.c_int32), ("max_surface", C.c_int32), ("surface_waves", C.c_int32),
                ("bound_blocks", C.c_int32), ("us_mode", C.c_int32), ("root_tol", C.c_double),
                ("full_slots", C.c_int32)]


class IsoStepStats(C.Structure):
    _fields_ = [("n_surface", C.c_int64), ("n_flat", C.c_int64), ("n_nonconverged", C.c_int64),
                ("n_bound_active", C.c_int64), ("max_root_iter", C.c_int32), ("reserved", C.c_int32),
                ("vol_before", C.c_double), ("vol_after", C.c_double), ("vol_boundary_flux", C.c_double),
                ("vol_clipped", C.c_double), ("alpha_min", C.c_double), ("alpha_max", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class IsoRelaxZone(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("direction", C.c_double * 3), ("length", C.c_double)]


class IsoTrace(C.Structure):
    _fields_ = [("vert_alpha", _vp), ("kind", _vp), ("iso", _vp), ("rec", _vp), ("dV", _vp),
                ("alpha_raw", _vp), ("iters", _vp)]


class IsoError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"isoadv error {status}: {message}")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        # PyTorch carries its own HIP runtime.  Loading it first lets the library's libamdhip64.so.7
        # dependency bind to that same runtime (matched by soname), so device pointers and streams
        # of torch tensors are valid in the library.  Two runtimes in one process do not work.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        _check_single_runtime()
        L.iso_options_default.argtypes = [C.POINTER(IsoOptions)]
        L.iso_options_default.restype = None
        L.iso_status_string.argtypes = [C.c_int]
        L.iso_status_string.restype = C.c_char_p
        L.iso_last_error.argtypes = []
        L.iso_last_error.restype = C.c_char_p
        L.iso_mesh_create.argtypes = [C.c_int32, _dp, _dp, _dp, C.c_int32, _ip, _ip, _ip, C.c_int32, _ip, C.c_int32,
                                      C.c_int32, _ip, _ip, _ip, _ip, _dp, _dp, C.POINTER(_vp)]
        L.iso_mesh_create.restype = C.c_int
        L.iso_mesh_destroy.argtypes = [_vp]
        L.iso_mesh_destroy.restype = None
        L.iso_mesh_info.argtypes = [_vp, C.POINTER(C.c_int64)]
        L.iso_mesh_info.restype = C.c_int
        L.iso_mesh_cell_points.argtypes = [_vp, _ip]
        L.iso_mesh_cell_points.restype = C.c_int
        L.iso_mesh_geometry.argtypes = [_vp, _dp, _dp]
        L.iso_mesh_geometry.restype = C.c_int
        L.iso_plan_create.argtypes = [_vp, C.POINTER(IsoOptions), _vp, C.POINTER(_vp)]
        L.iso_plan_create.restype = C.c_int
        L.iso_plan_set_stream.argtypes = [_vp, _vp]
        L.iso_plan_set_stream.restype = C.c_int
        L.iso_plan_destroy.argtypes = [_vp]
        L.iso_plan_destroy.restype = None
        L.iso_advect_step.argtypes = [_vp, _vp, _vp, _vp, C.c_double, _vp, C.POINTER(IsoStepStats)]
        L.iso_advect_step.restype = C.c_int
        L.iso_plan_run.argtypes = [_vp, _vp, _vp, C.c_int64, _vp, C.c_int64, C.c_double, C.c_int32]
        L.iso_plan_run.restype = C.c_int
        L.iso_advect_step_traced.argtypes = [_vp, _vp, _vp, _vp, C.c_double, _vp, C.POINTER(IsoStepStats),
                                             C.POINTER(IsoTrace)]
        L.iso_advect_step_traced.restype = C.c_int
        L.iso_advect_step_avg.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, C.c_double, _vp, C.POINTER(IsoStepStats)]
        L.iso_advect_step_avg.restype = C.c_int
        L.iso_advect_step_noalloc.argtypes = [_vp, C.POINTER(IsoOptions), _vp, _vp, _vp, _vp, C.c_double, _vp]
        L.iso_advect_step_noalloc.restype = C.c_int
        L.iso_gfm_faces.argtypes = [_vp, _vp, _vp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                    _vp, _vp, _vp, _vp, _vp]
        L.iso_gfm_faces.restype = C.c_int
        L.iso_plan_set_relaxation.argtypes = [_vp, C.c_int32, C.POINTER(IsoRelaxZone), C.POINTER(C.c_int64)]
        L.iso_plan_set_relaxation.restype = C.c_int
        L.iso_relax_blend.argtypes = [_vp, _vp, _vp]
        L.iso_relax_blend.restype = C.c_int
        L.iso_advect_step_adjoint.argtypes = [_vp, _vp, _vp, _vp, C.c_double, C.POINTER(IsoTrace), _vp, _vp, _vp]
        L.iso_advect_step_adjoint.restype = C.c_int
        L.iso_plan_set_timing.argtypes = [_vp, C.c_int32]
        L.iso_plan_set_timing.restype = C.c_int
        L.iso_plan_timing.argtypes = [_vp, _dp, C.POINTER(C.c_int32)]
        L.iso_plan_timing.restype = C.c_int
        L.iso_batch_create.argtypes = [C.POINTER(_vp), C.c_int32, C.POINTER(IsoOptions), _vp, C.POINTER(_vp)]
        L.iso_batch_create.restype = C.c_int
        L.iso_batch_destroy.argtypes = [_vp]
        L.iso_batch_destroy.restype = None
        L.iso_batch_layout.argtypes = [_vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.iso_batch_layout.restype = C.c_int
        L.iso_batch_advect.argtypes = [_vp, _vp, _vp, C.c_int64, _vp, C.c_int64, _dp, C.c_int32]
        L.iso_batch_advect.restype = C.c_int
        L.iso_batch_config.argtypes = [_vp, _ip]
        L.iso_batch_config.restype = C.c_int
        L.iso_batch_set_config.argtypes = [_vp, _ip]
        L.iso_batch_set_config.restype = C.c_int
        L.iso_batch_tune.argtypes = [_vp, _vp, _vp, _vp, _dp, C.c_int32, C.c_char_p, _dp]
        L.iso_batch_tune.restype = C.c_int
        _lib = L
    return _lib


def _check_single_runtime():
    try:
        maps = open("/proc/self/maps").read()
    except OSError:
        return
    paths = set(re.findall(r"\S*/libamdhip64\.so\S*", maps))
    if len(paths) > 1:
        raise RuntimeError("two HIP runtimes are loaded in this process: " + ", ".join(sorted(paths)))


def header_functions():
    """Names of the functions declared in include/isoadv.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(iso_[a-z_]+)\s*\(", txt)))


def check(status):
    if status != ISO_OK:
        msg = lib().iso_last_error().decode()
        raise IsoError(status, msg or lib().iso_status_string(status).decode())


def default_options(**kw) -> IsoOptions:
    o = IsoOptions()
    lib().iso_options_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _check(t, n=None, dtype="f64", name="tensor"):
    """With n, the tensor must hold exactly n elements of dtype ("f64" float64, "i32" int32): the
    kernels behind the C interface trust the sizes the mesh implies, so a short or mistyped
    buffer is refused here."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor")
    if n is not None:
        want = torch.float64 if dtype == "f64" else torch.int32
        if t.dtype != want:
            raise ValueError(f"{name}: expected {want}, got {t.dtype}")
        if t.numel() != int(n):
            raise ValueError(f"{name}: expected {int(n)} elements, got {t.numel()}")


def _ptrs(*specs):
    """Device pointers of (tensor, n, dtype, name) specs: every size is checked before any device."""
    for sp in specs:
        _check(*sp)
    return [_ptr(sp[0], name=sp[3]) for sp in specs]


def _ptr(t, n=None, dtype="f64", name="tensor"):
    """Device pointer of a contiguous CUDA (HIP) tensor (checked as in _check first)."""
    _check(t, n, dtype, name)
    if not t.is_cuda:
        raise ValueError(f"{name}: expected a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Mesh:
    """A face-based hexahedral mesh uploaded to the device (iso_mesh_create).

    ``points`` (n,3) float64; ``face_ptr``/``face_pts`` the face point lists; ``owner``
    per face; ``neighbour`` per interior face; patches as parallel arrays.
    """

    def __init__(self, points, face_ptr, face_pts, owner, neighbour, n_cells, patch_start, patch_size, patch_kind,
                 patch_partner, patch_translation, patch_alpha_in):
        L = lib()
        pts = np.ascontiguousarray(points, dtype=np.float64)
        px, py, pz = (np.ascontiguousarray(pts[:, i]) for i in range(3))
        arrs = dict(face_ptr=np.ascontiguousarray(face_ptr, dtype=np.int32),
                    face_pts=np.ascontiguousarray(face_pts, dtype=np.int32),
                    owner=np.ascontiguousarray(owner, dtype=np.int32),
                    neighbour=np.ascontiguousarray(neighbour if len(neighbour) else np.zeros(1), dtype=np.int32),
                    ps=np.ascontiguousarray(patch_start, dtype=np.int32),
                    pn=np.ascontiguousarray(patch_size, dtype=np.int32),
                    pk=np.ascontiguousarray(patch_kind, dtype=np.int32),
                    pp=np.ascontiguousarray(patch_partner, dtype=np.int32))
        pt = np.ascontiguousarray(patch_translation, dtype=np.float64).reshape(-1)
        pa = np.ascontiguousarray(patch_alpha_in, dtype=np.float64)
        h = _vp()
        ip = lambda a: a.ctypes.data_as(_ip)
        dp = lambda a: a.ctypes.data_as(_dp)
        n_faces = len(arrs["owner"])
        st = L.iso_mesh_create(len(pts), dp(px), dp(py), dp(pz), n_faces, ip(arrs["face_ptr"]), ip(arrs["face_pts"]),
                               ip(arrs["owner"]), len(neighbour), ip(arrs["neighbour"]), int(n_cells),
                               len(arrs["ps"]), ip(arrs["ps"]), ip(arrs["pn"]), ip(arrs["pk"]), ip(arrs["pp"]),
                               dp(pt), dp(pa), C.byref(h))
        check(st)
        self.h = h
        self.n_cells = int(n_cells)
        self.n_faces = n_faces
        self.n_points = len(pts)

    @classmethod
    def from_arrays(cls, m):
        """From any object with the attributes of a face-based mesh (points, face_ptr, face_pts, owner,
        neighbour, n_cells, patch_arrays())."""
        ps, pn, pk, pp, pt, pa = m.patch_arrays()
        return cls(m.points, m.face_ptr, m.face_pts, m.owner, m.neighbour, m.n_cells, ps, pn, pk, pp, pt, pa)

    def info(self):
        out = (C.c_int64 * 8)()
        check(lib().iso_mesh_info(self.h, out))
        keys = ["n_cells", "n_points", "n_faces", "n_flux_faces", "n_point_classes", "slots", "device_bytes",
                "wide_slots"]
        return {k: int(out[i]) for i, k in enumerate(keys)}

    def cell_points(self):
        out = np.zeros(8 * self.n_cells, dtype=np.int32)
        check(lib().iso_mesh_cell_points(self.h, out.ctypes.data_as(_ip)))
        return out.reshape(-1, 8)

    def geometry(self):
        vol = np.zeros(self.n_cells)
        xc = np.zeros(3 * self.n_cells)
        check(lib().iso_mesh_geometry(self.h, vol.ctypes.data_as(_dp), xc.ctypes.data_as(_dp)))
        return vol, xc.reshape(-1, 3)

    def close(self):
        if getattr(self, "h", None):
            lib().iso_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def advect_step_noalloc(mesh, alpha, phi, U, dt, out, options: IsoOptions | None = None, stream=None):
    """One step without a plan and without any device allocation (iso_advect_step_noalloc): out is
    written on the given (default: current) stream.  The library's fixed workspace limits the mesh
    to about 24 B per cell plus 60 B per face within 64 MiB."""
    nc, nf = mesh.n_cells, mesh.n_faces
    pa, pp, pu, po = _ptrs((alpha, nc, "f64", "alpha"), (phi, nf, "f64", "phi"), (U, 3 * nc, "f64", "U"),
                           (out, nc, "f64", "out"))
    check(lib().iso_advect_step_noalloc(mesh.h, C.byref(options) if options is not None else None,
                                        _stream_handle(stream), pa, pp, pu, float(dt), po))
    return out


class Plan:
    """Options + workspace + stream for stepping one mesh (iso_plan_create)."""

    def __init__(self, mesh: Mesh, options: IsoOptions | None = None, stream=None):
        self.mesh = mesh
        self.options = options or default_options()
        h = _vp()
        check(lib().iso_plan_create(mesh.h, C.byref(self.options), _stream_handle(stream), C.byref(h)))
        self.h = h

    def set_stream(self, stream):
        check(lib().iso_plan_set_stream(self.h, _stream_handle(stream)))

    def run(self, alpha, phi, U, dt, n_steps, phi_stride=0, U_stride=0):
        """In place: alpha (device, float64 [n_cells]) after n_steps steps (iso_plan_run, replayed as a
        captured graph while its arguments stay the same).  phi/U: one step's fields (strides 0) or
        n_steps of them at the given element strides."""
        import torch
        m = self.mesh
        last = max(int(n_steps) - 1, 0)
        for t, name in ((phi, "phi"), (U, "U")):
            if not isinstance(t, torch.Tensor) or t.dtype != torch.float64:
                raise ValueError(f"{name}: expected a float64 torch tensor")
        if phi.numel() < m.n_faces + last * int(phi_stride):
            raise ValueError(f"phi: expected at least {m.n_faces + last * int(phi_stride)} elements")
        if U.numel() < 3 * m.n_cells + last * int(U_stride):
            raise ValueError(f"U: expected at least {3 * m.n_cells + last * int(U_stride)} elements")
        check(lib().iso_plan_run(self.h, _ptr(alpha, m.n_cells, name="alpha"), _ptr(phi, name="phi"),
                                 int(phi_stride), _ptr(U, name="U"), int(U_stride), float(dt), int(n_steps)))
        return alpha

    def step(self, alpha, phi, U, dt, out=None, stats=False, trace=None, phi1=None, U1=None):
        """alpha_new = isoAdvector step (device tensors, float64).  Returns (alpha_new, stats dict or None).
        phi1, U1: the fields' estimates at t + dt of an outer iteration; the step then uses the
        averages (phi + phi1)/2 and (U + U1)/2 (iso_advect_step_avg; no trace)."""
        import torch
        if out is None:
            out = torch.empty_like(alpha)
        st = IsoStepStats() if stats else None
        if (phi1 is None) != (U1 is None):
            raise ValueError("phi1 and U1 go together")
        nc, nf = self.mesh.n_cells, self.mesh.n_faces
        specs = [(alpha, nc, "f64", "alpha"), (phi, nf, "f64", "phi"), (U, 3 * nc, "f64", "U"),
                 (out, nc, "f64", "out")]
        if phi1 is not None:
            specs += [(phi1, nf, "f64", "phi1"), (U1, 3 * nc, "f64", "U1")]
        pa, pp, pu, po, *p1 = _ptrs(*specs)
        self.set_stream(None)
        if phi1 is not None:
            if trace is not None:
                raise ValueError("the averaged-field step takes no trace")
            check(lib().iso_advect_step_avg(self.h, pa, pp, p1[0], pu, p1[1], float(dt), po,
                                            C.byref(st) if st is not None else None))
        elif trace is None:
            check(lib().iso_advect_step(self.h, pa, pp, pu, float(dt), po, C.byref(st) if st is not None else None))
        else:
            tr = self._trace(trace, self.TRACE_KEYS)
            check(lib().iso_advect_step_traced(self.h, pa, pp, pu, float(dt), po,
                                               C.byref(st) if st is not None else None, C.byref(tr)))
        return out, (st.as_dict() if st is not None else None)

    def _trace(self, trace, keys):
        """iso_trace of the given device tensors, each checked against its size in the header."""
        nc, nf = self.mesh.n_cells, self.mesh.n_faces
        sizes = {"vert_alpha": (8 * nc, "f64"), "kind": (nc, "i32"), "iso": (nc, "f64"), "rec": (7 * nc, "f64"),
                 "dV": (nf, "f64"), "alpha_raw": (nc, "f64"), "iters": (nc, "i32")}
        specs = [(trace[k], *sizes[k], f"trace[{k}]") for k in self.TRACE_KEYS
                 if k in keys and trace.get(k) is not None]
        got = dict(zip([sp[3] for sp in specs], _ptrs(*specs)))
        return IsoTrace(*[got[f"trace[{k}]"].value if f"trace[{k}]" in got else None for k in self.TRACE_KEYS])

    TRACE_KEYS = ("vert_alpha", "kind", "iso", "rec", "dV", "alpha_raw", "iters")

    def set_relaxation(self, zones):
        """Relaxation zones (iso_plan_set_relaxation): a list of (origin[3], direction[3], length).
        Returns the number of zone cells."""
        arr = (IsoRelaxZone * max(len(zones), 1))()
        for i, (o, d, ln) in enumerate(zones):
            arr[i].origin[:] = [float(v) for v in o]
            arr[i].direction[:] = [float(v) for v in d]
            arr[i].length = float(ln)
        n = C.c_int64(0)
        check(lib().iso_plan_set_relaxation(self.h, len(zones), arr, C.byref(n)))
        return n.value

    def relax_blend(self, alpha, alpha_target):
        """alpha (device tensor) blended in place towards alpha_target in the plan's zones."""
        nc = self.mesh.n_cells
        pa, pt = _ptrs((alpha, nc, "f64", "alpha"), (alpha_target, nc, "f64", "alpha_target"))
        self.set_stream(None)
        check(lib().iso_relax_blend(self.h, pa, pt))
        return alpha
    GFM_KEYS = ("lambda", "jump", "beta_w", "ghost_own", "ghost_nbr")

    def gfm_faces(self, alpha, p_d, rho_heavy, rho_light, g, out=None):
        """Ghost-fluid face data (iso_gfm_faces): dict of lambda, jump, beta_w, ghost_own and
        ghost_nbr, each a float64 device tensor [n_faces] (``out`` supplies them)."""
        import torch
        if out is None:
            out = {k: torch.empty(self.mesh.n_faces, dtype=torch.float64, device=alpha.device) for k in self.GFM_KEYS}
        gx, gy, gz = (float(v) for v in g)
        nc, nf = self.mesh.n_cells, self.mesh.n_faces
        pa, pd, *ptrs = _ptrs((alpha, nc, "f64", "alpha"), (p_d, nc, "f64", "p_d"),
                              *[(out[k], nf, "f64", f"out[{k}]") for k in self.GFM_KEYS])
        self.set_stream(None)
        check(lib().iso_gfm_faces(self.h, pa, pd, float(rho_heavy), float(rho_light), gx, gy, gz, *ptrs))
        return out

    def adjoint(self, alpha, phi, U, dt, alpha_new_bar, trace=None, alpha_bar=None, phi_bar=None):
        """(alpha_bar, phi_bar) of the step alpha_new = step(alpha, phi, U, dt) for the given alpha_new_bar.
        ``trace``: the dict of device tensors a traced step of the same inputs wrote (vert_alpha, kind,
        iso, dV, alpha_raw), or None to recompute the forward step inside."""
        import torch
        if alpha_bar is None:
            alpha_bar = torch.empty_like(alpha)
        if phi_bar is None:
            phi_bar = torch.empty_like(phi)
        nc, nf = self.mesh.n_cells, self.mesh.n_faces
        ptrs = _ptrs((alpha, nc, "f64", "alpha"), (phi, nf, "f64", "phi"), (U, 3 * nc, "f64", "U"),
                     (alpha_new_bar, nc, "f64", "alpha_new_bar"), (alpha_bar, nc, "f64", "alpha_bar"),
                     (phi_bar, nf, "f64", "phi_bar"))
        tr = self._trace(trace, ("vert_alpha", "kind", "iso", "dV", "alpha_raw")) if trace is not None else None
        args, bars = ptrs[:3], ptrs[3:]
        self.set_stream(None)
        check(lib().iso_advect_step_adjoint(self.h, *args, float(dt), C.byref(tr) if tr is not None else None,
                                            *bars))
        return alpha_bar, phi_bar

    KERNELS = ("find_surface", "surface", "update", "bound")

    def set_timing(self, max_steps):
        check(lib().iso_plan_set_timing(self.h, int(max_steps)))

    def timing(self):
        """Summed per-kernel milliseconds over the recorded steps, and the number of steps."""
        ms = (C.c_double * 4)()
        n = C.c_int32(0)
        check(lib().iso_plan_timing(self.h, ms, C.byref(n)))
        return {k: ms[i] for i, k in enumerate(self.KERNELS)}, n.value

    def close(self):
        if getattr(self, "h", None):
            lib().iso_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent meshes advanced together (iso_batch_create): one launch per kernel for all
    members and a captured HIP graph per multi-step run.  The state and fields are concatenated
    by member; ``layout()`` gives the offsets.  U is structure of arrays over the concatenated
    cells (all Ux, then all Uy, then all Uz)."""

    CONFIG_KEYS = ("block_cells", "surface_blocks", "surface_waves", "bound_blocks")

    def __init__(self, meshes, options: IsoOptions | None = None, stream=None):
        self.meshes = list(meshes)  # kept alive only for the caller's convenience; the batch copies them
        self.options = options or default_options()
        arr = (_vp * len(self.meshes))(*[m.h.value for m in self.meshes])
        h = _vp()
        check(lib().iso_batch_create(arr, len(self.meshes), C.byref(self.options), _stream_handle(stream), C.byref(h)))
        self.h = h
        co = (C.c_int64 * (len(self.meshes) + 1))()
        fo = (C.c_int64 * (len(self.meshes) + 1))()
        check(lib().iso_batch_layout(self.h, co, fo))
        self.cell_off = np.array(co[:], dtype=np.int64)
        self.face_off = np.array(fo[:], dtype=np.int64)
        self.n_cells = int(self.cell_off[-1])
        self.n_faces = int(self.face_off[-1])

    def layout(self):
        return self.cell_off.copy(), self.face_off.copy()

    def concat_cells(self, per_member):
        """Concatenate per-member cell arrays (numpy) into the batch layout."""
        return np.concatenate([np.asarray(a, dtype=np.float64) for a in per_member])

    def concat_U(self, per_member):
        """Concatenate per-member SoA velocity arrays [3 n_d] into the batch SoA layout [3 N]."""
        parts = [np.asarray(u, dtype=np.float64).reshape(3, -1) for u in per_member]
        return np.concatenate([np.concatenate([p[k] for p in parts]) for k in range(3)])

    def split_cells(self, a):
        a = np.asarray(a)
        return [a[self.cell_off[d]:self.cell_off[d + 1]] for d in range(len(self.meshes))]

    def advect(self, alpha, phi, U, dt, n_steps, phi_stride=0, U_stride=0, stream=None):
        """In place: alpha (device, float64 [N]) after n_steps steps.  phi/U: device tensors holding one
        step's fields (strides 0) or several steps' fields at the given element strides."""
        dts = np.ascontiguousarray(dt, dtype=np.float64)
        if dts.shape != (len(self.meshes),):
            raise ValueError("dt needs one time step per member")
        pa, pp, pu = self._fields(alpha, phi, U, n_steps, phi_stride, U_stride)
        check(lib().iso_batch_advect(self.h, pa, pp, int(phi_stride), pu, int(U_stride), dts.ctypes.data_as(_dp),
                                     int(n_steps)))
        return alpha

    def _fields(self, alpha, phi, U, n_steps, phi_stride=0, U_stride=0):
        """Pointers of the concatenated state and fields, each checked to hold what the steps read:
        one step's fields (stride 0) or n_steps of them at the given element strides."""
        import torch
        last = max(int(n_steps) - 1, 0)
        for t, name in ((phi, "phi"), (U, "U")):
            if not isinstance(t, torch.Tensor) or t.dtype != torch.float64:
                raise ValueError(f"{name}: expected a float64 torch tensor")
        need_phi = self.n_faces + last * int(phi_stride)
        need_U = 3 * self.n_cells + last * int(U_stride)
        if phi.numel() < need_phi:
            raise ValueError(f"phi: expected at least {need_phi} elements, got {phi.numel()}")
        if U.numel() < need_U:
            raise ValueError(f"U: expected at least {need_U} elements, got {U.numel()}")
        return _ptr(alpha, self.n_cells, name="alpha"), _ptr(phi, name="phi"), _ptr(U, name="U")

    def config(self):
        c = (C.c_int32 * 4)()
        check(lib().iso_batch_config(self.h, c))
        return dict(zip(self.CONFIG_KEYS, c[:]))

    def set_config(self, **kw):
        cur = self.config()
        cur.update(kw)
        c = (C.c_int32 * 4)(*[int(cur[k]) for k in self.CONFIG_KEYS])
        check(lib().iso_batch_set_config(self.h, c))

    def tune(self, alpha, phi, U, dt, n_trial=3, cache_path=None):
        """Autotune the launch shapes on n_trial steps (alpha is not modified).  Returns (config, ms/step)."""
        dts = np.ascontiguousarray(dt, dtype=np.float64)
        if dts.shape != (len(self.meshes),):
            raise ValueError("dt needs one time step per member")
        best = C.c_double(0.0)
        pa, pp, pu = self._fields(alpha, phi, U, 1)
        check(lib().iso_batch_tune(self.h, pa, pp, pu, dts.ctypes.data_as(_dp), int(n_trial),
                                   cache_path.encode() if cache_path else None, C.byref(best)))
        return self.config(), best.value

    def close(self):
        if getattr(self, "h", None):
            lib().iso_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
