"""ctypes front end of the CPU oracle (isoadv_oracle.c).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg use this module; the GPU library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "isoadv_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# a prebuilt oracle variant can be named here (used by the mutation test to load planted mistakes)
_ALT_LIB = os.environ.get("ISOADV_ORACLE_LIB")

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


class Opts(C.Structure):
    _fields_ = [("eps_surf", C.c_double), ("flat_tol", C.c_double), ("bound_tol", C.c_double),
                ("n_bound_iter", C.c_int), ("clip", C.c_int), ("max_bisect", C.c_int), ("us_mode", C.c_int)]


class Trace(C.Structure):
    _fields_ = [("a_pts", _dp), ("kind", _ip), ("iso", _dp), ("rec", _dp), ("dV", _dp),
                ("alpha_raw", _dp), ("iters", _ip)]


class Stats(C.Structure):
    _fields_ = [("n_surface", C.c_int64), ("n_flat", C.c_int64), ("n_bound_active", C.c_int64),
                ("max_iter", C.c_int32), ("vol_before", C.c_double), ("vol_after", C.c_double),
                ("vol_boundary", C.c_double), ("vol_clipped", C.c_double), ("alpha_min", C.c_double),
                ("alpha_max", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def compile_oracle(src: str, out: str) -> str:
    """gcc build of an oracle source file (no FMA contraction, so rounding follows the source)."""
    tmp = f"{out}.tmp{os.getpid()}"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
                           "-shared", "-Wall", "-Wno-unused-function", "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile the oracle next to its source."""
    if _ALT_LIB:
        return _ALT_LIB
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        compile_oracle(SRC, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        L.or_mesh_create.restype = C.c_void_p
        L.or_mesh_create.argtypes = [C.c_int, _dp, C.c_int, _ip, _ip, _ip, C.c_int, _ip, C.c_int, C.c_int,
                                     _ip, _ip, _ip, _ip, _dp, _dp, C.c_char_p, C.c_int]
        L.or_mesh_free.argtypes = [C.c_void_p]
        L.or_mesh_geometry.argtypes = [C.c_void_p, _dp, _dp]
        L.or_point_values.argtypes = [C.c_void_p, _dp, _dp]
        L.or_cell_isovalue.restype = C.c_double
        L.or_cell_isovalue.argtypes = [C.c_void_p, C.c_int, _dp, C.c_double, C.c_int, _ip]
        L.or_cell_cut_flat.argtypes = [C.c_void_p, C.c_int, _dp, C.c_double, _dp]
        L.or_tri_integral.restype = C.c_double
        L.or_tri_integral.argtypes = [_dp, _dp, _dp, C.c_double, C.c_double]
        L.or_tri_wet_fraction.restype = C.c_double
        L.or_tri_wet_fraction.argtypes = [_dp, _dp, _dp, C.c_double, C.c_double]
        L.or_face_integral.restype = C.c_double
        L.or_face_integral.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp, _dp, C.c_double, C.c_double]
        L.or_default_opts.argtypes = [C.POINTER(Opts)]
        L.or_step.argtypes = [C.c_void_p, C.POINTER(Opts), _dp, _dp, _dp, C.c_double, _dp, C.POINTER(Trace),
                              C.POINTER(Stats)]
        L.or_run.argtypes = [C.c_void_p, C.POINTER(Opts), _dp, _dp, _dp, C.c_double, C.c_int]
        L.or_step_tlm.argtypes = [C.c_void_p, C.POINTER(Opts), _dp, _dp, _dp, C.c_double, _dp, _dp, _dp, _dp]
        L.or_step_tlm.restype = C.c_int
        L.or_cell_point_velocity.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp]
        L.or_relax_blend.argtypes = [C.c_void_p, C.c_int, _dp, _dp, _dp, _dp]
        L.or_relax_blend.restype = C.c_int
        L.or_relax_weight.argtypes = [C.c_double]
        L.or_relax_weight.restype = C.c_double
        L.or_set_threads.argtypes = [C.c_int]
        L.or_set_threads.restype = None
        L.or_get_threads.argtypes = []
        L.or_get_threads.restype = C.c_int
        L.or_gfm_faces.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (results do not depend on the count)."""
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().or_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def relax_weight(chi) -> float:
    """Blending weight of a relaxation zone at the zone coordinate chi (reading R17)."""
    return lib().or_relax_weight(float(chi))


def tri_integral(x9, xS, nS, un, dt) -> float:
    x9 = np.ascontiguousarray(x9, dtype=np.float64).ravel()
    xS = np.ascontiguousarray(xS, dtype=np.float64)
    nS = np.ascontiguousarray(nS, dtype=np.float64)
    return lib().or_tri_integral(_d(x9), _d(xS), _d(nS), float(un), float(dt))


def tri_wet_fraction(x9, xS, nS, un, tau) -> float:
    x9 = np.ascontiguousarray(x9, dtype=np.float64).ravel()
    xS = np.ascontiguousarray(xS, dtype=np.float64)
    nS = np.ascontiguousarray(nS, dtype=np.float64)
    return lib().or_tri_wet_fraction(_d(x9), _d(xS), _d(nS), float(un), float(tau))


class OracleMesh:
    """The oracle's own view of a face-based mesh (geometry, periodic classes, stencils)."""

    def __init__(self, mesh):
        L = lib()
        self.mesh = mesh
        self._keep = []

        def keep(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a

        pts = keep(mesh.points.reshape(-1), np.float64)
        fptr = keep(mesh.face_ptr, np.int32)
        fpts = keep(mesh.face_pts, np.int32)
        own = keep(mesh.owner, np.int32)
        nbr = keep(mesh.neighbour if mesh.n_internal else np.zeros(1), np.int32)
        start, size, kind, partner, trans, ain = mesh.patch_arrays()
        start, size, kind, partner = (keep(x, np.int32) for x in (start, size, kind, partner))
        trans, ain = keep(trans, np.float64), keep(ain, np.float64)
        err = C.create_string_buffer(512)
        h = L.or_mesh_create(mesh.n_points, _d(pts), mesh.n_faces, _i(fptr), _i(fpts), _i(own), mesh.n_internal,
                             _i(nbr), mesh.n_cells, len(mesh.patches), _i(start), _i(size), _i(kind),
                             _i(partner), _d(trans), _d(ain), err, 512)
        if not h:
            raise ValueError("oracle mesh: " + err.value.decode())
        self.h = C.c_void_p(h)
        self.n_cells = mesh.n_cells
        self.n_points = mesh.n_points
        self.n_faces = mesh.n_faces

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().or_mesh_free(self.h)
                self.h = None
        except Exception:
            pass

    def geometry(self):
        xc = np.zeros(3 * self.n_cells)
        V = np.zeros(self.n_cells)
        lib().or_mesh_geometry(self.h, _d(xc), _d(V))
        return xc.reshape(-1, 3), V

    def point_values(self, alpha):
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        out = np.zeros(self.n_points)
        lib().or_point_values(self.h, _d(alpha), _d(out))
        return out

    def isovalue(self, c, a_pts, alpha_c, max_iter=200):
        a_pts = np.ascontiguousarray(a_pts, dtype=np.float64)
        it = C.c_int(0)
        r = lib().or_cell_isovalue(self.h, int(c), _d(a_pts), float(alpha_c), int(max_iter), C.byref(it))
        return r, it.value

    def cut(self, c, a_pts, iso):
        """vsub, S (3), xS (3), Swet (3), n_cut of cell c cut at isovalue iso."""
        a_pts = np.ascontiguousarray(a_pts, dtype=np.float64)
        out = np.zeros(11)
        lib().or_cell_cut_flat(self.h, int(c), _d(a_pts), float(iso), _d(out))
        return {"vsub": out[0], "S": out[1:4].copy(), "xS": out[4:7].copy(), "Swet": out[7:10].copy(),
                "n_cut": int(out[10])}

    def cell_point_velocity(self, c, U, x):
        """Velocity at x in cell c by cell-point interpolation (reading R15), U as [3 n_cells] SoA."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros(3)
        lib().or_cell_point_velocity(self.h, int(c), _d(U), _d(x), _d(out))
        return out

    def relax_blend(self, zones, alpha, target):
        """alpha blended towards target in relaxation zones (reading R17).  zones: list of
        (origin[3], direction[3], length).  Raises ValueError for invalid or overlapping zones."""
        z = np.ascontiguousarray([list(o) + list(d) + [ln] for o, d, ln in zones], dtype=np.float64).ravel()
        if z.size == 0:
            z = np.zeros(1)
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        target = np.ascontiguousarray(target, dtype=np.float64)
        out = np.zeros(self.n_cells)
        if lib().or_relax_blend(self.h, len(zones), _d(z), _d(alpha), _d(target), _d(out)) != 0:
            raise ValueError("invalid or overlapping relaxation zones")
        return out

    def gfm_faces(self, alpha, p_d, rho_heavy, rho_light, g):
        """Ghost-fluid face data (Eqs. 12-20, reading R16) per face: dict of lambda, jump, beta_w,
        ghost_own and ghost_nbr, each [n_faces]."""
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        p_d = np.ascontiguousarray(p_d, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        out = {k: np.zeros(self.n_faces) for k in ("lambda", "jump", "beta_w", "ghost_own", "ghost_nbr")}
        lib().or_gfm_faces(self.h, _d(alpha), _d(p_d), float(rho_heavy), float(rho_light), _d(g),
                           *(_d(out[k]) for k in ("lambda", "jump", "beta_w", "ghost_own", "ghost_nbr")))
        return out

    def face_integral(self, f, c, xS, nS, un, dt):
        xS = np.ascontiguousarray(xS, dtype=np.float64)
        nS = np.ascontiguousarray(nS, dtype=np.float64)
        return lib().or_face_integral(self.h, int(f), int(c), _d(xS), _d(nS), float(un), float(dt))

    def step(self, alpha, phi, U, dt, opts=None, trace=False):
        """One advection step.  Returns alpha_new, stats dict and (if trace) the intermediates."""
        opts = opts or default_opts()
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        U = np.ascontiguousarray(U, dtype=np.float64)
        out = np.zeros(self.n_cells)
        st = Stats()
        tr = None
        arrays = None
        if trace:
            arrays = {"a_pts": np.zeros(self.n_points), "kind": np.zeros(self.n_cells, dtype=np.int32),
                      "iso": np.full(self.n_cells, np.nan), "rec": np.full(7 * self.n_cells, np.nan),
                      "dV": np.zeros(self.n_faces), "alpha_raw": np.zeros(self.n_cells),
                      "iters": np.zeros(self.n_cells, dtype=np.int32)}
            tr = Trace(_d(arrays["a_pts"]), _i(arrays["kind"]), _d(arrays["iso"]), _d(arrays["rec"]),
                       _d(arrays["dV"]), _d(arrays["alpha_raw"]), _i(arrays["iters"]))
        lib().or_step(self.h, C.byref(opts), _d(alpha), _d(phi), _d(U), float(dt), _d(out),
                      C.byref(tr) if tr is not None else None, C.byref(st))
        if trace:
            arrays["rec"] = arrays["rec"].reshape(-1, 7)
            return out, st.as_dict(), arrays
        return out, st.as_dict()

    def step_tlm(self, alpha, phi, U, dt, dalpha=None, dphi=None, opts=None):
        """One step and its derivative along (dalpha, dphi) (complex step): (alpha_new, dalpha_new)."""
        opts = opts or default_opts()
        alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        U = np.ascontiguousarray(U, dtype=np.float64)
        da = np.ascontiguousarray(np.zeros(self.n_cells) if dalpha is None else dalpha, dtype=np.float64)
        dp = np.ascontiguousarray(np.zeros(self.n_faces) if dphi is None else dphi, dtype=np.float64)
        out = np.zeros(self.n_cells)
        dout = np.zeros(self.n_cells)
        if lib().or_step_tlm(self.h, C.byref(opts), _d(alpha), _d(phi), _d(U), float(dt), _d(da), _d(dp), _d(out),
                             _d(dout)) != 0:
            raise ValueError("the tangent follows U_S = U_P only (us_mode 0)")
        return out, dout

    def gradient(self, alpha, phi, U, dt, alpha_new_bar, cells=None, faces=None, opts=None):
        """Components of the step's vector-Jacobian product (d alpha_new / d input)^T alpha_new_bar,
        each computed as one tangent along a unit input direction (slow, exact): returns
        (alpha_bar[cells], phi_bar[faces])."""
        cells = range(self.n_cells) if cells is None else cells
        faces = range(self.n_faces) if faces is None else faces
        ab = np.asarray(alpha_new_bar, dtype=np.float64)
        ga, gp = [], []
        for c in cells:
            e = np.zeros(self.n_cells)
            e[c] = 1.0
            ga.append(float(ab @ self.step_tlm(alpha, phi, U, dt, dalpha=e, opts=opts)[1]))
        for f in faces:
            e = np.zeros(self.n_faces)
            e[f] = 1.0
            gp.append(float(ab @ self.step_tlm(alpha, phi, U, dt, dphi=e, opts=opts)[1]))
        return np.array(ga), np.array(gp)

    def run(self, alpha, phi, U, dt, n_steps, opts=None):
        opts = opts or default_opts()
        a = np.array(alpha, dtype=np.float64, copy=True)
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        U = np.ascontiguousarray(U, dtype=np.float64)
        lib().or_run(self.h, C.byref(opts), _d(a), _d(phi), _d(U), float(dt), int(n_steps))
        return a
