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
