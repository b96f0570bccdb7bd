"""Pins of the CPU oracle against what the paper and elementary mathematics fix.

Nothing here compares the oracle with itself: every expected value comes from a
closed form, an independent geometric construction (tests/geomref.py), brute-force
sampling, an exactness statement of the paper, or a hand-derived fixture.
"""
import json
import math
import os

import numpy as np
import pytest

import wavegen as W
from tests import geomref as R

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def single_cell_mesh(M=None, lo=(0, 0, 0), hi=(1, 1, 1)):
    m = W.hex_block([lo[0], hi[0]], [lo[1], hi[1]], [lo[2], hi[2]], periodic_x=False)
    if M is not None:
        m.points = np.ascontiguousarray(m.points @ np.asarray(M, float).T)
    return m


HEX_EDGES_LOCAL = [(0, 1), (1, 2), (2, 3), (3, 0), (4, 5), (5, 6), (6, 7), (7, 4), (0, 4), (1, 5), (2, 6), (3, 7)]


def hex_cell_vertices(mesh):
    """The 8 points of a single-cell block in local hex order (points are (i,j,k) ordered)."""
    P = mesh.points
    order = [0, 1, 3, 2, 4, 5, 7, 6]  # (0,0,0),(1,0,0),(1,1,0),(0,1,0),(0,0,1),(1,0,1),(1,1,1),(0,1,1)
    return P[order]


# ---------------------------------------------------------------------- one triangle (Eqs. tv .. intaplus)
def test_triangle_golden(oracle_lib):
    cases = json.load(open(os.path.join(GOLD, "triangle_sweeps.json")))["cases"]
    for cs in cases:
        got = oracle_lib.tri_integral(cs["tri"], cs["xS"], cs["nS"], cs["un"], cs["dt"])
        assert abs(got - cs["expected"]) <= 1e-14 * max(1.0, cs["dt"]), (cs["name"], got, cs["expected"])


def _random_tri(rng):
    tri = rng.normal(size=(3, 3))
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    return tri, n


def test_triangle_mean_arrival_closed_form(oracle_lib):
    """Window containing all arrival times: integral = dt - mean arrival time."""
    rng = np.random.default_rng(11)
    for _ in range(300):
        tri, n = _random_tri(rng)
        d = tri @ n
        un = rng.uniform(0.2, 3.0)
        xS = (d.min() - rng.uniform(0.01, 1.0)) * n  # plane reaches the triangle after the start
        t = (tri - xS) @ n / un
        dt = t.max() * rng.uniform(1.0, 2.0)
        got = oracle_lib.tri_integral(tri, xS, n, un, dt)
        assert abs(got - (dt - t.mean())) <= 1e-13 * dt


def test_triangle_vs_exact_clip_integral(oracle_lib):
    """Random triangles, planes, speeds of either sign and windows: piecewise-exact quadrature of clipped areas."""
    rng = np.random.default_rng(12)
    for i in range(400):
        tri, n = _random_tri(rng)
        d = tri @ n
        un = rng.choice([-1, 1]) * rng.uniform(0.05, 2.0)
        if i % 25 == 0:
            un = 0.0
        xS = rng.uniform(d.min() - 1.0, d.max() + 1.0) * n + rng.normal(size=3) * 0.1
        xS -= (np.dot(xS, n) - np.dot(xS, n)) * n
        dt = rng.uniform(0.1, 3.0)
        got = oracle_lib.tri_integral(tri, xS, n, un, dt)
        ref = R.wet_integral_exact(tri, xS, n, un, dt)
        assert abs(got - ref) <= 1e-12 * dt, (i, got, ref)


def test_triangle_area_fraction_pieces(oracle_lib):
    """Eq. aplus1 and the corrected Eq. aplus2 against exact clipped areas at many times,
    including just before/after t2 (continuity) and at t3 (value 1)."""
    rng = np.random.default_rng(13)
    for _ in range(100):
        tri, n = _random_tri(rng)
        un = rng.uniform(0.3, 2.0)
        xS = (tri @ n).min() * n - 0.2 * n
        t = np.sort((tri - xS) @ n / un)
        taus = list(rng.uniform(t[0] - 0.1, t[2] + 0.1, size=12)) + [t[1] - 1e-9, t[1], t[1] + 1e-9, t[2]]
        for tau in taus:
            got = oracle_lib.tri_wet_fraction(tri, xS, n, un, tau)
            ref = R.wet_fraction_exact(tri, xS, n, un, tau)
            assert abs(got - ref) <= 1e-11, (tau, got, ref)
        assert oracle_lib.tri_wet_fraction(tri, xS, n, un, t[2]) == pytest.approx(1.0, abs=1e-14)


def test_triangle_parallel_to_the_plane_up_to_rounding(oracle_lib):
    """A triangle whose plane is parallel to the isoface only up to rounding (its vertex distances
    agree to a few ulps): all of it arrives at once, so the integral is the step's closed form
    dt - t (or t for a receding plane), never a 0/0 from Eq. x_41's ratio of projections."""
    rng = np.random.default_rng(12)
    n = np.array([-1.0, 1.0, 0.0]) / np.sqrt(2.0)
    for _ in range(200):
        c = rng.uniform(-1, 1)
        p = rng.uniform(-1, 1, (3, 2))
        tri = np.array([[x, x + c, z] for x, z in p])  # on the plane y - x = c
        d0 = rng.uniform(-0.3, 0.3)
        xS = tri.mean(axis=0) - d0 * n
        for un in (0.7, -0.7):
            dt = 0.5
            got = oracle_lib.tri_integral(tri, xS, n, un, dt)
            t = ((tri - xS) @ n).mean() / un
            ref = (dt - min(max(t, 0.0), dt)) if un > 0 else min(max(t, 0.0), dt)
            assert np.isfinite(got) and abs(got - ref) <= 1e-12, (got, ref, t)


def test_printed_aplus2_would_jump():
    """Documents the reading of Eq. aplus2: the printed bracket [1-(1-(tau-t3)/(t2-t3))^2]
    equals 1 at tau=t2, so alpha+ would jump by A234/A there and return to alpha+(t2) at t3."""
    t2, t3 = 1.0, 2.0
    printed = lambda tau: 1 - (1 - (tau - t3) / (t2 - t3)) ** 2
    used = lambda tau: 1 - ((t3 - tau) / (t3 - t2)) ** 2
    assert printed(t2) == 1.0 and printed(t3) == 0.0
    assert used(t2) == 0.0 and used(t3) == 1.0


def test_triangle_brute_force_sampling(oracle_lib):
    """Dense sampling in space (barycentric grid) and time (midpoints)."""
    rng = np.random.default_rng(14)
    K, M = 160, 160
    ii, jj = np.meshgrid(np.arange(K), np.arange(K), indexing="ij")
    mask = ii + jj < K
    b1 = ((ii + 1.0 / 3) / K)[mask]
    b2 = ((jj + 1.0 / 3) / K)[mask]
    for _ in range(6):
        tri, n = _random_tri(rng)
        un = rng.choice([-1, 1]) * rng.uniform(0.2, 1.0)
        xS = np.mean(tri, axis=0) + rng.normal(size=3) * 0.2
        dt = rng.uniform(0.5, 2.0)
        pts = tri[0] + b1[:, None] * (tri[1] - tri[0]) + b2[:, None] * (tri[2] - tri[0])
        dpt = (pts - xS) @ n
        s = (np.arange(M) + 0.5) / M * dt
        wet = (dpt[None, :] <= un * s[:, None]).mean()
        got = oracle_lib.tri_integral(tri, xS, n, un, dt)
        assert abs(got - wet * dt) <= 2e-2 * dt


def test_triangle_limits(oracle_lib):
    """u_n -> 0 tends to the static fraction; coincident arrival times; face parallel to the plane."""
    tri = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0]])
    n = np.array([0.6, 0.8, 0.0])
    xS = np.array([0.3, 0.2, 0.0])
    static = oracle_lib.tri_integral(tri, xS, n, 0.0, 1.0)
    for un in (1e-12, -1e-12, 1e-200):
        assert abs(oracle_lib.tri_integral(tri, xS, n, un, 1.0) - static) <= 1e-10
    # plane parallel to the triangle: it is submerged from its (single) arrival time on
    nz = np.array([0.0, 0, 1])
    assert oracle_lib.tri_integral(tri, np.array([0, 0, -0.5]), nz, 1.0, 2.0) == pytest.approx(1.5, abs=1e-15)
    assert oracle_lib.tri_integral(tri, np.array([0, 0, -0.5]), nz, -1.0, 2.0) == 0.0
    # two vertices arriving together (t1 == t2 and t2 == t3)
    for tri2, nn in ((tri, np.array([0.0, 1, 0])), (tri, np.array([1.0, 1, 0]) / np.sqrt(2))):
        xS2 = -0.1 * nn
        ref = R.wet_integral_exact(tri2, xS2, nn, 1.0, 2.0)
        assert abs(oracle_lib.tri_integral(tri2, xS2, nn, 1.0, 2.0) - ref) <= 1e-13


# ---------------------------------------------------------------------- sub-cell volume and isoface
@pytest.mark.parametrize("shape", ["box", "sheared"])
def test_subvolume_linear_data_is_plane_clip(oracle_lib, shape):
    """Linear vertex data cut at alpha0 is exactly a plane clip of the cell (edge interpolation is exact).
    Box: inclusion-exclusion closed form. Sheared parallelepiped: convex hull of the clipped vertices."""
    M = None if shape == "box" else np.array([[1.0, 0.3, 0.1], [0.0, 0.8, 0.25], [0.1, 0.0, 1.2]])
    lo, hi = (0.2, -0.1, 0.5), (1.3, 0.6, 1.4)
    mesh = single_cell_mesh(M, lo, hi)
    om = oracle_lib.OracleMesh(mesh)
    _, V = om.geometry()
    verts = hex_cell_vertices(mesh)
    rng = np.random.default_rng(21)
    for _ in range(40):
        g = rng.normal(size=3)
        c0 = 0.37
        a_pts = c0 - mesh.points @ g
        av = c0 - verts @ g
        iso = rng.uniform(av.min(), av.max())
        cut = om.cut(0, a_pts, iso)
        # wet iff a > iso  <=>  g.x < c0 - iso
        if shape == "box":
            ref = R.box_below_plane_volume(lo, hi, g, c0 - iso)
            vol_total = np.prod(np.subtract(hi, lo))
        else:
            ref, _ = R.clipped_hull_volume_and_section(list(verts), HEX_EDGES_LOCAL, g, c0 - iso)
            vol_total = abs(np.linalg.det(M)) * np.prod(np.subtract(hi, lo))
        assert abs(V[0] - vol_total) <= 1e-13 * vol_total
        assert abs(cut["vsub"] - ref) <= 1e-12 * vol_total, (cut["vsub"], ref)
        # the isoface closes the wet part
        assert np.abs(cut["S"] + cut["Swet"]).max() <= 1e-13


def test_isoface_of_linear_data(oracle_lib):
    """Normal = g/|g| (away from the heavy side), centre = area centroid of the plane section."""
    M = np.array([[1.0, 0.2, 0.0], [0.1, 0.9, 0.3], [0.0, 0.2, 1.1]])
    mesh = single_cell_mesh(M, (0, 0, 0), (1, 1, 1))
    om = oracle_lib.OracleMesh(mesh)
    verts = hex_cell_vertices(mesh)
    rng = np.random.default_rng(22)
    for _ in range(30):
        g = rng.normal(size=3)
        a_pts = 1.0 - mesh.points @ g
        av = 1.0 - verts @ g
        iso = rng.uniform(av.min() + 0.05 * np.ptp(av), av.max() - 0.05 * np.ptp(av))
        cut = om.cut(0, a_pts, iso)
        S = cut["S"]
        nS = S / np.linalg.norm(S)
        assert np.abs(nS - g / np.linalg.norm(g)).max() <= 1e-13
        _, sec = R.clipped_hull_volume_and_section(list(verts), HEX_EDGES_LOCAL, g, 1.0 - iso)
        cen, area = R.section_centroid(sec, g)
        assert abs(np.linalg.norm(S) - area) <= 1e-13 * max(area, 1e-3)
        assert np.abs(cut["xS"] - cen).max() <= 1e-13
        assert abs(np.dot(g, cut["xS"]) - (1.0 - iso)) <= 1e-13


def test_isovalue_meets_volume_fraction(oracle_lib):
    """Every reconstructed cell's isoface cuts off alpha_P V_P to 1e-12 (2D cosine and a 3D case)."""
    w2 = W.cosine_uniform()
    w3 = W.violent_3d(nx=16, ny=8, nz=8, steps=1)
    for w in (w2, w3):
        om = oracle_lib.OracleMesh(w.mesh)
        _, V = om.geometry()
        phi, U = w.phi_U(0)
        _, st, tr = om.step(w.alpha0, phi, U, w.dt, trace=True)
        cells = np.nonzero(tr["kind"] == 1)[0]
        assert len(cells) > 10
        for c in cells:
            cut = om.cut(c, tr["a_pts"], tr["iso"][c])
            assert abs(cut["vsub"] / V[c] - w.alpha0[c]) <= 1e-12
            assert np.abs(cut["S"] + cut["Swet"]).max() <= 1e-14 * max(1.0, V[c] ** (2 / 3) * 1e14)


# ---------------------------------------------------------------------- vertex interpolation
def test_idw_golden(oracle_lib):
    g = json.load(open(os.path.join(GOLD, "idw_two_cells.json")))
    mesh = W.hex_block(g["xs"], g["ys"], g["zs"], periodic_x=False)
    om = oracle_lib.OracleMesh(mesh)
    a = om.point_values(np.array(g["alpha"]))
    p = int(np.nonzero(np.all(mesh.points == np.array(g["point"]), axis=1))[0][0])
    assert abs(a[p] - g["expected"]) <= 1e-15


def test_idw_partition_of_unity_and_periodic(oracle_lib):
    w = W.cosine_uniform(nx=8, ny=6)
    om = oracle_lib.OracleMesh(w.mesh)
    a = om.point_values(np.full(w.mesh.n_cells, 0.3))
    assert np.abs(a - 0.3).max() <= 1e-15
    rng = np.random.default_rng(3)
    alpha = rng.uniform(size=w.mesh.n_cells)
    a = om.point_values(alpha)
    nx, ny, _ = w.mesh.shape
    A = alpha.reshape(ny, nx)
    P = a.reshape(2, ny + 1, nx + 1)
    # interior points of a uniform slab: mean of the 4 cells around them
    for j in range(1, ny):
        for i in range(1, nx):
            ref = 0.25 * (A[j - 1, i - 1] + A[j - 1, i] + A[j, i - 1] + A[j, i])
            assert abs(P[0, j, i] - ref) <= 1e-15 and abs(P[1, j, i] - P[0, j, i]) <= 1e-15
        # periodic seam: x=0 and x=L copies equal, mean of the cells on both sides
        ref = 0.25 * (A[j - 1, nx - 1] + A[j - 1, 0] + A[j, nx - 1] + A[j, 0])
        assert abs(P[0, j, 0] - ref) <= 1e-15 and P[0, j, nx] == P[0, j, 0]
    # wall points: mean of the two cells above
    assert abs(P[0, 0, 3] - 0.5 * (A[0, 2] + A[0, 3])) <= 1e-15


# ---------------------------------------------------------------------- whole steps
def band_slab(nx, ny, ya, yb, u, v, co):
    """Doubly periodic uniform slab holding a band of heavy fluid ya < y < yb, uniform velocity (u, v)."""
    h = 1.0 / nx
    mesh = W.hex_block(np.linspace(0, 1, nx + 1), np.linspace(0, ny * h, ny + 1), [0.0, h], periodic_x=True,
                       periodic_y=True, kinds={"zmin": W.PATCH_EMPTY, "zmax": W.PATCH_EMPTY})
    phi = W.fluxes_from_edge_integral(mesh, lambda x, y, z0, z1: (u * y - v * x) * (z1 - z0))
    U = np.concatenate([np.full(mesh.n_cells, u), np.full(mesh.n_cells, v), np.zeros(mesh.n_cells)])
    dt = W.courant_dt(mesh, phi, co)
    return mesh, phi, U, dt


def band_alpha(mesh, ya, yb):
    return W.alpha_cosine_2d(mesh, yb, 0.0, 1.0) - W.alpha_cosine_2d(mesh, ya, 0.0, 1.0)


@pytest.mark.parametrize("u,v", [(0.0, 1.0), (0.0, -1.0), (0.7, 0.6), (-0.4, -0.9), (1.0, 0.3)])
def test_planar_interface_transport_is_exact(oracle_lib, u, v):
    """Planar interfaces in uniform flow on a periodic uniform mesh: the reconstruction is exact and the
    modelled fluxes are exact (planar face, planar interface, constant velocity), or cancel by
    x-translation invariance, so alpha equals the exact cell integral at every step."""
    nx, ny = 16, 24
    ya, yb = 0.3137, 0.9021 * ny / nx / 1.6
    mesh, phi, U, dt = band_slab(nx, ny, ya, yb, u, v, 0.45)
    om = oracle_lib.OracleMesh(mesh)
    a = band_alpha(mesh, ya, yb)
    for n in range(1, 9):
        a, st = om.step(a, phi, U, dt, oracle_lib.default_opts(clip=0))
        exact = band_alpha(mesh, ya + v * n * dt, yb + v * n * dt)
        assert np.abs(a - exact).max() <= 1e-12, (n, np.abs(a - exact).max())
        assert st["n_bound_active"] == 0


def test_45_degree_line_reconstruction(oracle_lib):
    """Cell fractions of x + y < c on a uniform grid depend on i+j only, so vertex values do too, and the
    isoface is the exact line: normal (1,1,0)/sqrt2 and centre on the line."""
    n = 14
    h = 1.0 / n
    mesh = W.hex_block(np.linspace(0, 1, n + 1), np.linspace(0, 1, n + 1), [0.0, h], periodic_x=False,
                       kinds={"zmin": W.PATCH_EMPTY, "zmax": W.PATCH_EMPTY})
    c = 0.97
    s = (c - (np.arange(n)[None, :] + np.arange(n)[:, None]) * h) / h
    frac = np.where(s <= 0, 0.0, np.where(s <= 1, 0.5 * s * s, np.where(s <= 2, 1 - 0.5 * (2 - s) ** 2, 1.0)))
    alpha = frac.ravel()
    om = oracle_lib.OracleMesh(mesh)
    phi = np.zeros(mesh.n_faces)
    U = np.zeros(3 * mesh.n_cells)
    _, _, tr = om.step(alpha, phi, U, 1e-3, trace=True)
    checked = 0
    for cell in np.nonzero(tr["kind"] == 1)[0]:
        j, i = divmod(cell, n)
        if not (1 <= i < n - 1 and 1 <= j < n - 1):
            continue
        xS, nS = tr["rec"][cell, :3], tr["rec"][cell, 3:6]
        assert np.abs(nS - np.array([1, 1, 0]) / np.sqrt(2)).max() <= 1e-13
        assert abs(xS[0] + xS[1] - c) <= 1e-13
        checked += 1
    assert checked >= 8


def test_conservation_and_bounds(oracle_lib):
    """Flux form conserves total volume to round-off without chopping; with chopping 0<=alpha<=1."""
    w = W.airy_slab(128, 64, 32, 0.09, 0.5, 10, "airy_small")
    om = oracle_lib.OracleMesh(w.mesh)
    _, V = om.geometry()
    a0 = w.alpha0
    a = a0.copy()
    for n in range(10):
        phi, U = w.phi_U(n)
        a, st = om.step(a, phi, U, w.dt, oracle_lib.default_opts(clip=0))
    assert abs((a * V).sum() - (a0 * V).sum()) <= 1e-14 * (a0 * V).sum()
    a = a0.copy()
    for n in range(10):
        phi, U = w.phi_U(n)
        a, st = om.step(a, phi, U, w.dt)
        assert a.min() >= 0.0 and a.max() <= 1.0


def test_bounding_redistributes_conservatively(oracle_lib):
    """At a Courant number beyond the method's comfort zone the redistribution is active; it moves
    volume between cells without creating or destroying any, and reduces the excursions."""
    w = W.airy_slab(64, 32, 16, 0.1, 0.95, 6, "airy_stressed")
    om = oracle_lib.OracleMesh(w.mesh)
    _, V = om.geometry()
    a = w.alpha0.copy()
    active = 0
    for n in range(6):
        phi, U = w.phi_U(n)
        b0, st0, tr = om.step(a, phi, U, w.dt, oracle_lib.default_opts(clip=0, n_bound_iter=0), trace=True)
        b3, st3 = om.step(a, phi, U, w.dt, oracle_lib.default_opts(clip=0, n_bound_iter=3))
        active += st3["n_bound_active"]
        assert abs((b3 * V).sum() - (b0 * V).sum()) <= 1e-15 * (a * V).sum() + 1e-18
        exc0 = np.maximum(b0 - 1, 0).sum() + np.maximum(-b0, 0).sum()
        exc3 = np.maximum(b3 - 1, 0).sum() + np.maximum(-b3, 0).sum()
        assert exc3 <= exc0 + 1e-15
        a = b3
    assert active > 0


def test_always_wet_and_dry_faces(oracle_lib):
    """Faces in the bulk carry phi*dt (wet) or 0 (dry) (the special cases of Eq. dVdef)."""
    w = W.cosine_uniform()
    om = oracle_lib.OracleMesh(w.mesh)
    phi, U = w.phi_U(0)
    _, _, tr = om.step(w.alpha0, phi, U, w.dt, trace=True)
    m = w.mesh
    for f in range(m.n_internal):
        o, nb = m.owner[f], m.neighbour[f]
        up = o if phi[f] > 0 else nb
        if phi[f] != 0 and w.alpha0[up] == 1.0:
            assert tr["dV"][f] == phi[f] * w.dt
        if phi[f] != 0 and w.alpha0[up] == 0.0:
            assert tr["dV"][f] == 0.0


def test_surface_face_fluxes_brute_force_tiny_mesh(oracle_lib):
    """On a 3x3x3 mesh with a smooth field, every flux of an interface cell equals phi times the
    space-time integral of the submerged area of the face below the moving isoface, computed here
    triangle by triangle with exact clipping and checked against dense sampling."""
    mesh = W.hex_block(np.linspace(0, 1, 4), np.linspace(0, 1, 4), np.linspace(0, 1, 4), periodic_x=False)
    cen = mesh.cell_centres_structured()
    alpha = np.clip(0.5 + 2.2 * (0.55 - cen[:, 2] - 0.3 * cen[:, 0] + 0.2 * cen[:, 1]), 0, 1)
    om = oracle_lib.OracleMesh(mesh)
    rng = np.random.default_rng(5)
    U = np.concatenate([rng.uniform(-1, 1, mesh.n_cells) for _ in range(3)])
    phi = np.zeros(mesh.n_faces)
    phi[:mesh.n_internal] = rng.uniform(-0.05, 0.05, mesh.n_internal)
    dt = 0.15
    _, _, tr = om.step(alpha, phi, U, dt, trace=True)
    fp = mesh.face_pts.reshape(-1, 4)
    checked = 0
    for f in range(mesh.n_internal):
        up = mesh.owner[f] if phi[f] > 0 else mesh.neighbour[f]
        if tr["kind"][up] != 1:
            continue
        xS, nS, un = tr["rec"][up, :3], tr["rec"][up, 3:6], tr["rec"][up, 6]
        pts = mesh.points[fp[f]]
        apex = pts.mean(axis=0)
        I, Af, samp = 0.0, 0.0, 0.0
        for k in range(4):
            tri = np.array([apex, pts[k], pts[(k + 1) % 4]])
            Ai = R.polygon_area(tri)
            I += Ai * R.wet_integral_exact(tri, xS, nS, un, dt)
            Af += Ai
        I /= Af
        # sampling check of the exact reference
        gx = (np.arange(40) + 0.5) / 40
        uu, vv = np.meshgrid(gx, gx, indexing="ij")
        q = (pts[0][None, None] * ((1 - uu) * (1 - vv))[..., None] + pts[1][None, None] * (uu * (1 - vv))[..., None]
             + pts[2][None, None] * (uu * vv)[..., None] + pts[3][None, None] * ((1 - uu) * vv)[..., None])
        d = (q.reshape(-1, 3) - xS) @ nS
        s = (np.arange(40) + 0.5) / 40 * dt
        samp = (d[None, :] <= un * s[:, None]).mean() * dt
        assert abs(samp - I) <= 0.05 * dt
        assert abs(tr["dV"][f] - phi[f] * I) <= 1e-13 * abs(phi[f]) * dt, (f, tr["dV"][f], phi[f] * I)
        checked += 1
    assert checked >= 5


def test_face_integral_on_trapezoidal_faces(oracle_lib):
    """A frustum cell has trapezoidal side faces, whose four centre-fan triangles differ in area.  The
    face integral must equal the exact submerged space-time integral of the face, computed here on
    an independent two-triangle split of each planar face."""
    mesh = single_cell_mesh()
    P = mesh.points.copy()
    top = P[:, 2] > 0.5
    P[top, 0] = 0.2 + 0.6 * P[top, 0]
    P[top, 1] = 0.1 + 0.5 * P[top, 1]
    mesh.points = np.ascontiguousarray(P)
    om = oracle_lib.OracleMesh(mesh)
    rng = np.random.default_rng(8)
    fp = mesh.face_pts.reshape(-1, 4)
    for _ in range(20):
        nS = rng.normal(size=3)
        nS /= np.linalg.norm(nS)
        xS = np.array([0.5, 0.4, 0.5]) + 0.2 * rng.normal(size=3)
        un = rng.choice([-1, 1]) * rng.uniform(0.1, 1.0)
        dt = rng.uniform(0.2, 1.0)
        for f in range(mesh.n_faces):
            q = mesh.points[fp[f]]
            t1, t2 = q[[0, 1, 2]], q[[0, 2, 3]]
            A1, A2 = R.polygon_area(t1), R.polygon_area(t2)
            ref = (A1 * R.wet_integral_exact(t1, xS, nS, un, dt) + A2 * R.wet_integral_exact(t2, xS, nS, un, dt)) \
                / (A1 + A2)
            got = om.face_integral(f, mesh.owner[f], xS, nS, un, dt)
            assert abs(got - ref) <= 1e-13 * dt, (f, got, ref)


def test_subvolume_and_isoface_continuous_across_vertex_ties(oracle_lib):
    """Away from saddle faces (diagonal wet corners), the cut points that merge or split when the
    isovalue crosses a vertex value must not move the sub-volume or the isoface centre: both are
    continuous there.  Vertex data = a linear field plus a perturbation (non-planar isofaces)."""
    mesh = single_cell_mesh(np.array([[1.0, 0.2, 0.1], [0.0, 0.9, 0.2], [0.1, 0.0, 1.1]]))
    om = oracle_lib.OracleMesh(mesh)
    _, V = om.geometry()
    rng = np.random.default_rng(31)
    worst_v, worst_x, ties = 0.0, 0.0, 0
    fp = mesh.face_pts.reshape(-1, 4)

    def saddle(a_pts, iso):
        w = a_pts[fp] > iso
        return np.any((w[:, 0] == w[:, 2]) & (w[:, 1] == w[:, 3]) & (w[:, 0] != w[:, 1]))

    for _ in range(300):
        g = rng.normal(size=3)
        a_pts = 0.5 - mesh.points @ g
        a_pts = a_pts + 0.08 * np.ptp(a_pts) * rng.uniform(-1, 1, mesh.n_points)
        s = np.sort(a_pts)
        for tie in s[1:-1]:
            d = 1e-10
            if saddle(a_pts, tie - d) or saddle(a_pts, tie + d):
                continue
            # a jump keeps its size as the gap closes; a continuous function's difference shrinks with it
            jv, jx = [], []
            for dd in (d, 0.01 * d):
                lo = om.cut(0, a_pts, tie - dd)
                hi = om.cut(0, a_pts, tie + dd)
                jv.append(abs(lo["vsub"] - hi["vsub"]) / V[0])
                jx.append(np.abs(lo["xS"] - hi["xS"]).max())
            if jv[0] > 1e-12 and jv[1] > 0.1 * jv[0]:
                worst_v = max(worst_v, jv[0])
            if jx[0] > 1e-12 and jx[1] > 0.1 * jx[0]:
                worst_x = max(worst_x, jx[0])
            ties += 1
    assert ties > 1000
    assert worst_v == 0.0 and worst_x == 0.0, (worst_v, worst_x)


def test_isovalue_is_root_or_jump(oracle_lib):
    """The sub-volume is non-increasing in the isovalue; with arbitrary vertex data (saddle faces) it can
    jump at a vertex value.  The isovalue is the root where the volume fraction is continuous, and the
    vertex value itself where the volume fraction jumps across alpha_P."""
    mesh = single_cell_mesh(np.array([[1.0, 0.2, 0.1], [0.0, 0.9, 0.2], [0.1, 0.0, 1.1]]))
    om = oracle_lib.OracleMesh(mesh)
    _, V = om.geometry()
    rng = np.random.default_rng(32)
    jumps = 0
    for _ in range(300):
        a_pts = rng.uniform(0, 1, mesh.n_points)
        grid = np.linspace(a_pts.min(), a_pts.max(), 41)
        vs = [om.cut(0, a_pts, x)["vsub"] for x in grid]
        assert np.all(np.diff(vs) <= 1e-14 * V[0])
        alpha = rng.uniform(0.02, 0.98)
        iso, _ = om.isovalue(0, a_pts, alpha)
        f = om.cut(0, a_pts, iso)["vsub"] / V[0] - alpha
        if abs(f) > 1e-12:
            jumps += 1
            assert np.any(a_pts == iso)
            assert f < 0 and om.cut(0, a_pts, np.nextafter(iso, -1))["vsub"] / V[0] - alpha > 0
    assert jumps > 0


# ---------------------------------------------------------------------- R15: isoface velocity
def _uniform_box(n=(6, 5, 5)):
    xs, ys, zs = (np.linspace(0.0, 1.0, k + 1) for k in n)
    return W.hex_block(xs, ys, zs, periodic_x=False), n


def _box_cell(n, c):
    nx, ny, _ = n
    return c % nx, (c // nx) % ny, c // (nx * ny)


def _interior(n, c):
    i, j, k = _box_cell(n, c)
    return all(1 <= q <= m - 2 for q, m in zip((i, j, k), n))


def test_cell_point_velocity_constant_field(oracle_lib):
    """A uniform velocity is reproduced anywhere in any cell (weights sum to one at every stage)."""
    m, n = _uniform_box()
    om = oracle_lib.OracleMesh(m)
    xc, _ = om.geometry()
    u0 = np.array([0.3, -0.2, 0.7])
    U = np.repeat(u0, m.n_cells)
    rng = np.random.default_rng(5)
    for c in rng.choice(m.n_cells, 40, replace=False):
        x = xc[c] + rng.uniform(-0.45, 0.45, 3) * 0.2
        assert np.abs(om.cell_point_velocity(c, U, x) - u0).max() <= 1e-15


def test_cell_point_velocity_linear_field_interior(oracle_lib):
    """U = a + G x sampled at the cell centres: in cells whose points are all interior to a uniform
    box (where the inverse-distance point values of a linear field are exact by symmetry) the
    interpolant is exact at every point of the cell."""
    m, n = _uniform_box()
    om = oracle_lib.OracleMesh(m)
    xc, _ = om.geometry()
    rng = np.random.default_rng(6)
    a = rng.normal(size=3)
    G = rng.normal(size=(3, 3))
    Uc = a + xc @ G.T
    U = np.ascontiguousarray(Uc.T.ravel())
    cells = [c for c in range(m.n_cells) if _interior(n, c)]
    assert len(cells) >= 20
    h = np.array([1.0 / q for q in n])
    for c in cells:
        for _ in range(5):
            x = xc[c] + rng.uniform(-0.5, 0.5, 3) * h
            assert np.abs(om.cell_point_velocity(c, U, x) - (a + G @ x)).max() <= 1e-13


def test_cell_point_velocity_centre_and_points(oracle_lib):
    """At the cell centre the interpolant is U_P; at a point of the cell it is that point's
    inverse-distance value (R1), whatever the field."""
    m, n = _uniform_box()
    om = oracle_lib.OracleMesh(m)
    xc, _ = om.geometry()
    rng = np.random.default_rng(7)
    U = rng.normal(size=3 * m.n_cells)
    pts = np.stack([om.point_values(U[d * m.n_cells:(d + 1) * m.n_cells]) for d in range(3)], axis=1)
    nx, ny, _ = n
    for c in rng.choice(m.n_cells, 25, replace=False):
        Up = U[[c, m.n_cells + c, 2 * m.n_cells + c]]
        assert np.abs(om.cell_point_velocity(c, U, xc[c]) - Up).max() <= 1e-14
        i, j, k = _box_cell(n, c)
        for di, dj, dk in ((0, 0, 0), (1, 0, 1), (1, 1, 1), (0, 1, 0)):
            p = (i + di) + (nx + 1) * ((j + dj) + (ny + 1) * (k + dk))
            assert np.abs(om.cell_point_velocity(c, U, m.points[p]) - pts[p]).max() <= 1e-14


def test_step_isoface_velocity_modes(oracle_lib):
    """The step's U_S . n_S (trace) with us_mode 1 is the linear field at the isoface centre in the
    interior cells of a uniform box; with us_mode 0 it is U_P . n_S."""
    m, n = _uniform_box()
    om = oracle_lib.OracleMesh(m)
    xc, _ = om.geometry()
    rng = np.random.default_rng(8)
    a = rng.normal(size=3)
    G = 0.3 * rng.normal(size=(3, 3))
    U = np.ascontiguousarray((a + xc @ G.T).T.ravel())
    alpha = np.clip(0.5 + 0.9 * (xc[:, 2] - 0.5) + 0.4 * (xc[:, 0] - 0.5) + 0.2 * (xc[:, 1] - 0.5), 0.02, 0.98)
    phi = np.zeros(m.n_faces)
    dt = 1e-3
    checked = 0
    for mode in (0, 1):
        _, _, tr = om.step(alpha, phi, U, dt, oracle_lib.default_opts(us_mode=mode), trace=True)
        for c in np.nonzero(tr["kind"] == 1)[0]:
            xS, nS, un = tr["rec"][c, :3], tr["rec"][c, 3:6], tr["rec"][c, 6]
            if mode == 0:
                assert abs(un - U[[c, m.n_cells + c, 2 * m.n_cells + c]] @ nS) <= 1e-15
            elif _interior(n, c):
                assert abs(un - (a + G @ xS) @ nS) <= 1e-13
                checked += 1
    assert checked >= 10


def test_cell_point_velocity_stays_within_nodal_values(oracle_lib):
    """Inside a (convex) cell the interpolant is a convex combination of U_P, the face means and the
    point values, so each component lies within their range: picking a tetrahedron that does not
    contain x would extrapolate."""
    m, n = _uniform_box()
    om = oracle_lib.OracleMesh(m)
    xc, _ = om.geometry()
    rng = np.random.default_rng(9)
    U = rng.normal(size=3 * m.n_cells)
    pts = np.stack([om.point_values(U[d * m.n_cells:(d + 1) * m.n_cells]) for d in range(3)], axis=1)
    nx, ny, _ = n
    h = np.array([1.0 / q for q in n])
    for c in rng.choice(m.n_cells, 30, replace=False):
        i, j, k = _box_cell(n, c)
        ids = [(i + di) + (nx + 1) * ((j + dj) + (ny + 1) * (k + dk)) for di in (0, 1) for dj in (0, 1) for dk in (0, 1)]
        nodal = np.vstack([pts[ids], U[[c, m.n_cells + c, 2 * m.n_cells + c]][None, :]])
        lo, hi = nodal.min(axis=0) - 1e-14, nodal.max(axis=0) + 1e-14
        for _ in range(10):
            x = xc[c] + rng.uniform(-0.49, 0.49, 3) * h
            u = om.cell_point_velocity(c, U, x)
            assert np.all(u >= lo) and np.all(u <= hi), (c, x, u, lo, hi)
