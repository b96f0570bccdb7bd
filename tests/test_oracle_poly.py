"""Pins of the oracle on tetrahedra, triangular prisms, square pyramids and polyhedra made of merged
hexahedra (split faces, up to 18 points and 16 faces, or the shared faces joined into polygons of 6
and 8 points), against what elementary geometry and the
method's invariants fix:

* linear vertex data cut at an isovalue is exactly a plane clip of the cell (convex hull of the
  clipped vertices), and the isoface is the plane section (normal, area, centroid);
* every reconstructed cell's isoface cuts off alpha_P V_P to 1e-12 after whole steps;
* the flux form conserves volume to round-off and chopping keeps 0 <= alpha <= 1;
* each flux of an interface cell is phi times the exact space-time integral of the face's
  submerged area below the moving isoface (triangles clipped exactly, checked against dense
  sampling).
"""
import numpy as np
import pytest

import wavegen as W
from tests import geomref as R


def _refined(v):
    v = list(v)
    return [v[0], 0.5 * (v[0] + v[1]), v[1]] if len(v) == 2 else v


def merged_x(xs, ys, zs, **kw):
    """Hexahedra (i, j, k), i even, joined with (i+1, j, k): 12 points, 10 faces."""
    xs = _refined(xs)
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    return W.merged_block(xs, ys, zs, merge_x=[(i, j, k) for k in range(nz) for j in range(ny)
                                              for i in range(0, nx - 1, 2)], **kw)


def merged_xy(xs, ys, zs, **kw):
    """2 x 2 hexahedra joined from every (i, j, k) with i, j even: 18 points, 16 faces."""
    xs, ys = _refined(xs), _refined(ys)
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    return W.merged_block(xs, ys, zs, merge_xy=[(i, j, k) for k in range(nz) for j in range(0, ny - 1, 2)
                                                for i in range(0, nx - 1, 2)], **kw)


def merged_joined(xs, ys, zs, **kw):
    """Pairs along x merged in every row, the two quadrilaterals that neighbouring pairs share
    joined into one face of 6 points: 12 points and 9 faces per cell."""
    xs, ys = _refined(xs), _refined(ys)
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    return W.merged_block(xs, ys, zs, merge_x=[(i, j, k) for k in range(nz) for j in range(ny)
                                              for i in range(0, nx - 1, 2)], join=True, **kw)


BUILDERS = {"tet": W.tet_block, "prism": W.prism_block, "pyramid": W.pyramid_block, "merged_x": merged_x,
            "merged_xy": merged_xy, "merged_joined": merged_joined}


def _cell_faces(mesh, c):
    out = []
    for f in range(mesh.n_faces):
        if mesh.owner[f] == c or (f < mesh.n_internal and mesh.neighbour[f] == c):
            out.append(mesh.face_pts[mesh.face_ptr[f]:mesh.face_ptr[f + 1]])
    return out


def _cell_verts_edges(mesh, c):
    faces = _cell_faces(mesh, c)
    ids = sorted({int(p) for f in faces for p in f})
    loc = {p: i for i, p in enumerate(ids)}
    edges = set()
    for f in faces:
        for a in range(len(f)):
            e = (loc[int(f[a])], loc[int(f[(a + 1) % len(f)])])
            edges.add((min(e), max(e)))
    return ids, mesh.points[ids], sorted(edges)


def _sheared(kind):
    M = np.array([[1.0, 0.3, 0.1], [0.0, 0.8, 0.25], [0.1, 0.0, 1.2]])
    m = BUILDERS[kind]([0.0, 1.0], [0.0, 1.0], [0.0, 1.0])
    m.points = np.ascontiguousarray(m.points @ M.T)
    return m


@pytest.mark.parametrize("kind", list(BUILDERS))
def test_subvolume_of_linear_data_is_plane_clip(oracle_lib, kind):
    mesh = _sheared(kind)
    om = oracle_lib.OracleMesh(mesh)
    _, V = om.geometry()
    rng = np.random.default_rng(31)
    for c in range(mesh.n_cells):
        ids, verts, edges = _cell_verts_edges(mesh, c)
        vol_total, _ = R.clipped_hull_volume_and_section(list(verts), edges, np.array([0.0, 0.0, 1.0]), 1e9)
        assert abs(V[c] - vol_total) <= 1e-13 * vol_total
        for _ in range(12):
            g = rng.normal(size=3)
            c0 = 0.37
            a_pts = c0 - mesh.points @ g
            av = c0 - verts @ g
            iso = rng.uniform(av.min(), av.max())
            cut = om.cut(c, a_pts, iso)
            ref, _ = R.clipped_hull_volume_and_section(list(verts), edges, g, c0 - iso)
            assert abs(cut["vsub"] - ref) <= 1e-12 * vol_total, (kind, c, cut["vsub"], ref)
            assert np.abs(cut["S"] + cut["Swet"]).max() <= 1e-13


@pytest.mark.parametrize("kind", list(BUILDERS))
def test_isoface_of_linear_data(oracle_lib, kind):
    mesh = _sheared(kind)
    om = oracle_lib.OracleMesh(mesh)
    rng = np.random.default_rng(32)
    for c in range(mesh.n_cells):
        ids, verts, edges = _cell_verts_edges(mesh, c)
        for _ in range(8):
            g = rng.normal(size=3)
            a_pts = 1.0 - mesh.points @ g
            av = 1.0 - verts @ g
            iso = rng.uniform(av.min() + 0.1 * np.ptp(av), av.max() - 0.1 * np.ptp(av))
            cut = om.cut(c, a_pts, iso)
            S = cut["S"]
            assert np.abs(S / np.linalg.norm(S) - g / np.linalg.norm(g)).max() <= 1e-12
            _, sec = R.clipped_hull_volume_and_section(list(verts), edges, g, 1.0 - iso)
            cen, area = R.section_centroid(sec, g)
            assert abs(np.linalg.norm(S) - area) <= 1e-12 * max(area, 1e-3)
            assert np.abs(cut["xS"] - cen).max() <= 1e-12


def _workloads():
    return [W.poly_violent("tet", nx=8, ny=4, nz=4, steps=6), W.poly_violent("prism", nx=8, ny=4, nz=4, steps=6),
            W.poly_violent("merged", nx=16, ny=8, nz=8, steps=6),
            W.poly_violent("merged_joined", nx=16, ny=8, nz=8, steps=6),
            W.poly_airy("prism", 32, 16, steps=6), W.poly_airy("tet", 24, 12, steps=6)]


def test_isovalue_meets_volume_fraction(oracle_lib):
    for w in _workloads():
        om = oracle_lib.OracleMesh(w.mesh)
        _, V = om.geometry()
        phi, U = w.phi_U(0)
        _, st, tr = om.step(w.alpha0, phi, U, w.dt, trace=True)
        cells = np.nonzero(tr["kind"] == 1)[0]
        assert len(cells) > 20, w.name
        for c in cells:
            cut = om.cut(c, tr["a_pts"], tr["iso"][c])
            assert abs(cut["vsub"] / V[c] - w.alpha0[c]) <= 1e-12, (w.name, c)


def test_conservation_and_bounds(oracle_lib):
    for w in _workloads():
        om = oracle_lib.OracleMesh(w.mesh)
        _, V = om.geometry()
        phi, U = w.phi_U(0)
        a = w.alpha0.copy()
        for _ in range(w.n_steps):
            a, st = om.step(a, phi, U, w.dt, oracle_lib.default_opts(clip=0))
        m0 = (w.alpha0 * V).sum()
        assert abs((a * V).sum() - m0) <= 1e-14 * m0, w.name
        a = w.alpha0.copy()
        for _ in range(w.n_steps):
            a, st = om.step(a, phi, U, w.dt)
            assert a.min() >= 0.0 and a.max() <= 1.0


@pytest.mark.parametrize("kind", ["tet", "prism", "pyramid", "merged_x", "merged_joined"])
def test_surface_face_fluxes_brute_force(oracle_lib, kind):
    """A smooth field on a 3x3x3 block of cells of one kind: every flux of an interface cell equals
    phi times the exact space-time integral of the submerged part of the face (each face fanned
    about its vertex mean, triangles clipped exactly), which dense sampling confirms."""
    mesh = BUILDERS[kind](np.linspace(0, 1, 4), np.linspace(0, 1, 4), np.linspace(0, 1, 4))
    om = oracle_lib.OracleMesh(mesh)
    cen, _ = om.geometry()
    alpha = np.clip(0.5 + 2.2 * (0.55 - cen[:, 2] - 0.3 * cen[:, 0] + 0.2 * cen[:, 1]), 0, 1)
    rng = np.random.default_rng(5)
    U = np.concatenate([rng.uniform(-1, 1, mesh.n_cells) for _ in range(3)])
    phi = np.zeros(mesh.n_faces)
    phi[:mesh.n_internal] = rng.uniform(-0.02, 0.02, mesh.n_internal)
    dt = 0.15
    _, _, tr = om.step(alpha, phi, U, dt, trace=True)
    checked = 0
    for f in range(mesh.n_internal):
        up = mesh.owner[f] if phi[f] > 0 else mesh.neighbour[f]
        if tr["kind"][up] != 1:
            continue
        xS, nS, un = tr["rec"][up, :3], tr["rec"][up, 3:6], tr["rec"][up, 6]
        pts = mesh.points[mesh.face_pts[mesh.face_ptr[f]:mesh.face_ptr[f + 1]]]
        apex = pts.mean(axis=0)
        I, Af = 0.0, 0.0
        for k in range(len(pts)):
            tri = np.array([apex, pts[k], pts[(k + 1) % len(pts)]])
            Ai = R.polygon_area(tri)
            I += Ai * R.wet_integral_exact(tri, xS, nS, un, dt)
            Af += Ai
        I /= Af
        # dense sampling of the face (fan triangles) in space and time
        gx = (np.arange(30) + 0.5) / 30
        uu, vv = np.meshgrid(gx, gx, indexing="ij")
        keep = (uu + vv) < 1.0
        samp, wsum = 0.0, 0.0
        s = (np.arange(30) + 0.5) / 30 * dt
        for k in range(len(pts)):
            a0, a1, a2 = apex, pts[k], pts[(k + 1) % len(pts)]
            q = a0 + uu[keep][:, None] * (a1 - a0) + vv[keep][:, None] * (a2 - a0)
            d = (q - xS) @ nS
            Ai = R.polygon_area(np.array([a0, a1, a2]))
            samp += Ai * (d[None, :] <= un * s[:, None]).mean() * dt
            wsum += Ai
        assert abs(samp / wsum - I) <= 0.05 * dt
        assert abs(tr["dV"][f] - phi[f] * I) <= 1e-13 * abs(phi[f]) * dt, (f, tr["dV"][f], phi[f] * I)
        checked += 1
    assert checked >= 5, checked


def test_point_wet_alone(oracle_lib):
    """One point wet alone, on four pairs of hexahedra merged along x whose shared faces are
    joined in y and in z.  A point with only two edges in its cell (where two joined faces meet)
    bounds a sliver: the two faces at it hold the same wet triangle with opposite orientation, so
    the sub-volume and the isoface area vector are exactly zero.  A point whose edges lie in one
    plane bounds a flat region: zero sub-volume, an isoface of non-zero area.  Otherwise a corner
    of positive volume is cut off."""
    xs, ys, zs = [0.0, 0.5, 1.0], [0.0, 0.5, 1.0], [0.0, 0.5, 1.0]
    mesh = W.merged_block(xs, ys, zs, merge_x=[(0, j, k) for k in range(2) for j in range(2)], join=True)
    om = oracle_lib.OracleMesh(mesh)
    seen = {"sliver": 0, "flat": 0, "corner": 0}
    for c in range(mesh.n_cells):
        ids, verts, edges = _cell_verts_edges(mesh, c)
        for i, p in enumerate(ids):
            dirs = np.array([verts[b] - verts[a] for a, b in edges if i in (a, b)])
            a_pts = np.zeros(mesh.n_points)
            a_pts[p] = 1.0
            cut = om.cut(c, a_pts, 0.5)
            if len(dirs) == 2:
                assert cut["vsub"] == 0.0 and np.all(cut["S"] == 0.0), (c, p)
                seen["sliver"] += 1
            elif np.linalg.matrix_rank(dirs, tol=1e-12) == 2:
                assert abs(cut["vsub"]) <= 1e-15 and np.linalg.norm(cut["S"]) > 1e-3, (c, p)
                seen["flat"] += 1
            else:
                assert cut["vsub"] > 1e-4 and np.linalg.norm(cut["S"]) > 1e-3, (c, p)
                seen["corner"] += 1
    assert seen["sliver"] >= 4 and seen["flat"] >= 8 and seen["corner"] >= 16, seen
