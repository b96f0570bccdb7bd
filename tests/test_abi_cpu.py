"""Host-side checks of the C interface that need no GPU: the library loads, exports every
function the header declares, and rejects bad meshes before touching the device."""
import ctypes as C

import numpy as np
import pytest

import wavegen as W
from paper_1804_01130_amd import binding as B


def test_library_exports_every_declared_function():
    L = B.lib()
    names = B.header_functions()
    assert "iso_advect_step" in names and "iso_mesh_create" in names and "iso_plan_create" in names
    for name in names:
        assert hasattr(L, name), name


def test_status_strings_and_defaults():
    L = B.lib()
    for s in range(8):
        assert L.iso_status_string(s)
    o = B.default_options()
    assert o.eps_surf == 1e-8 and o.n_bound_iter == 3 and o.clip == 1 and o.root_max_iter == 100
    assert o.us_mode == 0  # U_S = U_P unless cell-point interpolation is asked for
    assert o.root_tol == 0.0 and o.full_slots == 0  # round-off search; the update's slot words
    # the binding's structure ends where the header's does: its size is what the library fills
    assert C.sizeof(B.IsoOptions) == 88  # sizeof(iso_options) from the C compiler, padding included


def test_bench_refuses_more_than_one_gpu():
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _create(m, **over):
    ps, pn, pk, pp, pt, pa = m.patch_arrays()
    a = dict(points=m.points, face_ptr=m.face_ptr, face_pts=m.face_pts, owner=m.owner, neighbour=m.neighbour,
             n_cells=m.n_cells, ps=ps, pn=pn, pk=pk, pp=pp, pt=pt, pa=pa)
    a.update(over)
    return B.Mesh(a["points"], a["face_ptr"], a["face_pts"], a["owner"], a["neighbour"], a["n_cells"], a["ps"],
                  a["pn"], a["pk"], a["pp"], a["pt"], a["pa"])


def test_mesh_validation_errors_before_device():
    m = W.cosine_uniform(nx=4, ny=3).mesh
    bad_owner = m.owner.copy()
    bad_owner[0] = m.n_cells + 5
    with pytest.raises(B.IsoError) as e:
        _create(m, owner=bad_owner)
    assert e.value.status == B.ISO_EMESH
    ps, pn, pk, pp, pt, pa = m.patch_arrays()
    pp2 = pp.copy()
    pp2[0] = 2  # cyclic patch pointing at a wall
    with pytest.raises(B.IsoError) as e:
        _create(m, pp=pp2)
    assert e.value.status == B.ISO_EMESH
    with pytest.raises(B.IsoError) as e:  # a face of seventeen points
        fp = m.face_pts.copy()
        fptr = np.concatenate([[0], np.cumsum([17] + [4] * (m.n_faces - 1))]).astype(np.int32)
        fp = np.concatenate([fp[:4], np.repeat(fp[:1], 13), fp[4:]])
        _create(m, face_ptr=fptr, face_pts=fp)
    assert e.value.status == B.ISO_EUNSUPPORTED
    with pytest.raises(B.IsoError) as e:  # a cell whose faces do not close it
        fp = m.face_pts.copy()
        fptr = np.concatenate([[0], np.cumsum([3] + [4] * (m.n_faces - 1))]).astype(np.int32)
        fp = np.concatenate([fp[:3], fp[4:]])
        _create(m, face_ptr=fptr, face_pts=fp)
    assert e.value.status == B.ISO_EMESH


def _merged(xs, ys, zs, periodic_x=True):
    """2 x 2 hexahedra joined into one cell wherever i and j are even: 18 points, 16 faces."""
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    return W.merged_block(xs, ys, zs, merge_xy=[(i, j, k) for k in range(nz) for j in range(0, ny - 1, 2)
                                                for i in range(0, nx - 1, 2)], periodic_x=periodic_x)


@pytest.mark.parametrize("build", [W.tet_block, W.prism_block, W.pyramid_block, _merged])
def test_cells_other_than_hexahedra_pass_the_host_checks(build):
    """Tetrahedra, prisms, pyramids and polyhedra of merged hexahedra are taken: without a GPU the
    only failure left is the device one, after every host-side check."""
    m = build(np.linspace(0, 2, 5), np.linspace(0, 1, 3), np.linspace(0, 1, 3), periodic_x=True)
    with pytest.raises(B.IsoError) as e:
        _create(m)
    assert e.value.status == B.ISO_EDEVICE, e.value


def test_cyclic_mismatch_detected():
    m = W.cosine_uniform(nx=4, ny=3).mesh
    ps, pn, pk, pp, pt, pa = m.patch_arrays()
    pt2 = pt.copy()
    pt2[0] += 0.25  # wrong translation
    with pytest.raises(B.IsoError) as e:
        _create(m, pt=pt2)
    assert e.value.status in (B.ISO_EMESH, B.ISO_EDEVICE)


def test_batch_entry_points_reject_null_arguments():
    """Ensemble calls check their arguments before any device work."""
    L = B.lib()
    h = C.c_void_p()
    assert L.iso_batch_create(None, 0, None, None, C.byref(h)) == B.ISO_EINVAL
    assert L.iso_batch_create(None, 2, None, None, None) == B.ISO_EINVAL
    dt = (C.c_double * 1)(1.0)
    assert L.iso_batch_advect(None, None, None, 0, None, 0, dt, 1) == B.ISO_EINVAL
    cfg = (C.c_int32 * 4)()
    assert L.iso_batch_config(None, cfg) == B.ISO_EINVAL
    assert L.iso_batch_set_config(None, cfg) == B.ISO_EINVAL
    assert L.iso_batch_tune(None, None, None, None, dt, 1, None, None) == B.ISO_EINVAL
    assert L.iso_batch_layout(None, None, None) == B.ISO_EINVAL


class _FakePlan:
    """Stands in for a plan on the host: the binding checks buffers against the mesh's sizes
    before it touches the library, so these checks run without a device."""

    def __init__(self, nc, nf):
        self.mesh = type("M", (), {"n_cells": nc, "n_faces": nf})()

    _trace = B.Plan._trace
    TRACE_KEYS = B.Plan.TRACE_KEYS
    GFM_KEYS = B.Plan.GFM_KEYS


def test_binding_rejects_mistyped_or_short_buffers():
    """A buffer of the wrong dtype or length is refused before its pointer reaches the C interface
    (the kernels size their accesses from the mesh, so such a buffer would be read out of bounds)."""
    import torch
    nc, nf = 12, 30
    p = _FakePlan(nc, nf)
    f64 = dict(dtype=torch.float64)
    ok = dict(alpha=torch.zeros(nc, **f64), phi=torch.zeros(nf, **f64), U=torch.zeros(3 * nc, **f64),
              out=torch.zeros(nc, **f64))
    bad = {"alpha": torch.zeros(nc, dtype=torch.float32), "phi": torch.zeros(nf - 1, **f64),
           "U": torch.zeros(nc, **f64), "out": torch.zeros(nc + 1, **f64)}
    for k, t in bad.items():
        args = dict(ok, **{k: t})
        with pytest.raises(ValueError, match=k):
            B.Plan.step(p, args["alpha"], args["phi"], args["U"], 0.1, out=args["out"])
    # correct sizes and dtypes get as far as the device check
    with pytest.raises(ValueError, match="device tensor"):
        B.Plan.step(p, ok["alpha"], ok["phi"], ok["U"], 0.1, out=ok["out"])
    with pytest.raises(ValueError, match="kind"):
        p._trace({"kind": torch.zeros(nc, dtype=torch.int64)}, B.Plan.TRACE_KEYS)
    with pytest.raises(ValueError, match="vert_alpha"):
        p._trace({"vert_alpha": torch.zeros(nc, **f64)}, B.Plan.TRACE_KEYS)
    with pytest.raises(ValueError, match="p_d"):
        B.Plan.gfm_faces(p, ok["alpha"], torch.zeros(nc - 1, **f64), 1000.0, 1.2, (0, 0, -9.81),
                         out={k: torch.zeros(nf, **f64) for k in B.Plan.GFM_KEYS})
    with pytest.raises(ValueError, match="alpha_target"):
        B.Plan.relax_blend(p, ok["alpha"], torch.zeros(nc, dtype=torch.float32))
    with pytest.raises(ValueError, match="phi_bar"):
        B.Plan.adjoint(p, ok["alpha"], ok["phi"], ok["U"], 0.1, ok["alpha"], alpha_bar=ok["out"],
                       phi_bar=torch.zeros(nc, **f64))
