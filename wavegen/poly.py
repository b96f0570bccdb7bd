"""Meshes of tetrahedra and triangular prisms in face-based (owner/neighbour) form, and face fluxes
on meshes whose edges need not be vertical.

Like the rest of the package this only produces inputs of the advection method (its polyhedral
control volumes, Section 3): a block of hexahedra cut into prisms (each hexahedron split along one
diagonal of its xy projection, a 2D triangle mesh when the block is one cell thick) or into six
tetrahedra (the Kuhn split along the main diagonal, conforming between neighbours and identical
on opposite periodic sides).

Conventions are those of wavegen.mesh: interior faces first in upper-triangular order, boundary
faces patch after patch (xmin, xmax, ymin, ymax, zmin, zmax), the points of a face counter-clockwise
seen from outside its owner, face n of a cyclic patch matching face n of its partner.
"""
from __future__ import annotations

import itertools

import numpy as np

from .mesh import PATCH_CYCLIC, PATCH_WALL, Mesh, Patch


def _grid_points(xs, ys, zs):
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def mesh_from_cells(points, cells, xs, ys, zs, kinds=None, periodic_x=False, periodic_y=False, alpha_in=None):
    """Face-based mesh from cells given as lists of faces, each face a tuple of point ids
    counter-clockwise seen from outside the cell.  Boundary faces go to the patch of the block side
    they lie on (xs, ys, zs: the block's node coordinates)."""
    kinds = dict(kinds or {})
    if periodic_x:
        kinds["xmin"] = kinds["xmax"] = PATCH_CYCLIC
    if periodic_y:
        kinds["ymin"] = kinds["ymax"] = PATCH_CYCLIC
    for key in ("xmin", "xmax", "ymin", "ymax", "zmin", "zmax"):
        kinds.setdefault(key, PATCH_WALL)
    alpha_in = dict(alpha_in or {})
    seen = {}
    internal = []
    for c, faces in enumerate(cells):
        for fp in faces:
            key = tuple(sorted(fp))
            if key in seen:
                own, pts = seen.pop(key)
                internal.append((own, c, pts))
            else:
                seen[key] = (c, tuple(fp))
    internal.sort(key=lambda t: (t[0], t[1]))
    P = np.asarray(points, dtype=np.float64)
    lo = np.array([xs[0], ys[0], zs[0]])
    hi = np.array([xs[-1], ys[-1], zs[-1]])
    span = hi - lo
    sides = {"xmin": (0, 0), "xmax": (0, 1), "ymin": (1, 0), "ymax": (1, 1), "zmin": (2, 0), "zmax": (2, 1)}
    groups = {k: [] for k in sides}
    for own, pts in seen.values():
        cen = P[list(pts)].mean(axis=0)
        name = None
        for k, (ax, end) in sides.items():
            ref = hi[ax] if end else lo[ax]
            if np.all(np.abs(P[list(pts), ax] - ref) <= 1e-12 * max(1.0, span[ax])):
                name = k
                break
        if name is None:
            raise ValueError(f"boundary face {pts} lies on no side of the block")
        groups[name].append((own, pts, cen))
    # order each side by the transverse coordinates of the face centroids, so that the faces of
    # opposite sides match one to one
    for k, (ax, _) in sides.items():
        tr = [a for a in range(3) if a != ax]
        groups[k].sort(key=lambda t: (round(t[2][tr[1]], 9), round(t[2][tr[0]], 9)))
    owner = [t[0] for t in internal]
    neighbour = [t[1] for t in internal]
    fpts = [t[2] for t in internal]
    patches = []
    start = len(internal)
    for k in ("xmin", "xmax", "ymin", "ymax", "zmin", "zmax"):
        g = groups[k]
        patches.append(Patch(k, kinds[k], start, len(g), alpha_in=float(alpha_in.get(k, 0.0))))
        owner += [t[0] for t in g]
        fpts += [t[1] for t in g]
        start += len(g)
    if periodic_x:
        L = float(xs[-1] - xs[0])
        patches[0].partner, patches[0].translation = 1, (L, 0.0, 0.0)
        patches[1].partner, patches[1].translation = 0, (-L, 0.0, 0.0)
    if periodic_y:
        L = float(ys[-1] - ys[0])
        patches[2].partner, patches[2].translation = 3, (0.0, L, 0.0)
        patches[3].partner, patches[3].translation = 2, (0.0, -L, 0.0)
    face_ptr = np.concatenate([[0], np.cumsum([len(f) for f in fpts])]).astype(np.int32)
    face_pts = np.array([p for f in fpts for p in f], dtype=np.int32)
    return Mesh(points=P, face_ptr=face_ptr, face_pts=face_pts, owner=np.array(owner, dtype=np.int32),
                neighbour=np.array(neighbour, dtype=np.int32), n_cells=len(cells), patches=patches,
                shape=(len(xs) - 1, len(ys) - 1, len(zs) - 1))


def prism_block(xs, ys, zs, kinds=None, periodic_x=False, periodic_y=False):
    """Each hexahedron (i, j, k) of the block cut into two triangular prisms along the diagonal from
    (x_i, y_j) to (x_i+1, y_j+1): cell 2 c (the lower-right triangle) and 2 c + 1, c the hexahedron's
    number in wavegen.mesh.hex_block."""
    xs, ys, zs = (np.asarray(v, dtype=np.float64) for v in (xs, ys, zs))
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1

    def P(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    cells = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for tri in (((i, j), (i + 1, j), (i + 1, j + 1)), ((i, j), (i + 1, j + 1), (i, j + 1))):
                    bot = [P(a, b, k) for a, b in tri]
                    top = [P(a, b, k + 1) for a, b in tri]
                    faces = [tuple(reversed(bot)), tuple(top)]
                    for e in range(3):
                        a, b = e, (e + 1) % 3
                        faces.append((bot[a], bot[b], top[b], top[a]))
                    cells.append(faces)
    return mesh_from_cells(_grid_points(xs, ys, zs), cells, xs, ys, zs, kinds, periodic_x, periodic_y)


def pyramid_block(xs, ys, zs, kinds=None, periodic_x=False, periodic_y=False):
    """Each hexahedron of the block cut into six square pyramids with their apex at its centre (one
    extra point per hexahedron, numbered after the grid points): cells 6 c .. 6 c + 5, bases on the
    -x, +x, -y, +y, -z, +z sides."""
    xs, ys, zs = (np.asarray(v, dtype=np.float64) for v in (xs, ys, zs))
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    pts = [_grid_points(xs, ys, zs)]
    n0 = len(pts[0])

    def P(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    cells, centres = [], []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                apex = n0 + len(centres)
                centres.append([0.5 * (xs[i] + xs[i + 1]), 0.5 * (ys[j] + ys[j + 1]), 0.5 * (zs[k] + zs[k + 1])])
                for q in _hex_quads(P, i, j, k):
                    # base outward as on the hexahedron; each side triangle outward from the pyramid
                    cells.append([q] + [(q[(a + 1) % 4], q[a], apex) for a in range(4)])
    pts = np.concatenate([pts[0], np.array(centres, dtype=np.float64)])
    return mesh_from_cells(pts, cells, xs, ys, zs, kinds, periodic_x, periodic_y)


def _hex_quads(P, i, j, k):
    """The six faces of hexahedron (i, j, k) counter-clockwise from outside (as in hex_block):
    -x, +x, -y, +y, -z, +z."""
    return [(P(i, j + 1, k), P(i, j, k), P(i, j, k + 1), P(i, j + 1, k + 1)),
            (P(i + 1, j, k), P(i + 1, j + 1, k), P(i + 1, j + 1, k + 1), P(i + 1, j, k + 1)),
            (P(i, j, k), P(i + 1, j, k), P(i + 1, j, k + 1), P(i, j, k + 1)),
            (P(i + 1, j + 1, k), P(i, j + 1, k), P(i, j + 1, k + 1), P(i + 1, j + 1, k + 1)),
            (P(i, j, k), P(i, j + 1, k), P(i + 1, j + 1, k), P(i + 1, j, k)),
            (P(i, j, k + 1), P(i + 1, j, k + 1), P(i + 1, j + 1, k + 1), P(i, j + 1, k + 1))]


def mixed_block(xs, ys, zs, split_from, kinds=None, periodic_x=False, periodic_y=False):
    """Hexahedra in the columns i < split_from, and each hexahedron of the columns i >= split_from
    cut into two prisms as in prism_block (they meet the hexahedra on whole quadrilaterals)."""
    xs, ys, zs = (np.asarray(v, dtype=np.float64) for v in (xs, ys, zs))
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1

    def P(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    cells = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if i < split_from:
                    cells.append(_hex_quads(P, i, j, k))
                    continue
                for tri in (((i, j), (i + 1, j), (i + 1, j + 1)), ((i, j), (i + 1, j + 1), (i, j + 1))):
                    bot = [P(a, b, k) for a, b in tri]
                    top = [P(a, b, k + 1) for a, b in tri]
                    faces = [tuple(reversed(bot)), tuple(top)]
                    for e in range(3):
                        a, b = e, (e + 1) % 3
                        faces.append((bot[a], bot[b], top[b], top[a]))
                    cells.append(faces)
    return mesh_from_cells(_grid_points(xs, ys, zs), cells, xs, ys, zs, kinds, periodic_x, periodic_y)


def _join_loop(quads):
    """One polygon from faces that tile it, all oriented alike: the edges they share cancel, the
    rest is walked from the smallest point id."""
    edges = set()
    for q in quads:
        for a in range(len(q)):
            e = (q[a], q[(a + 1) % len(q)])
            if (e[1], e[0]) in edges:
                edges.remove((e[1], e[0]))
            else:
                edges.add(e)
    nxt = dict(edges)
    if len(nxt) != len(edges):
        raise ValueError("the joined faces do not bound one polygon")
    start = min(nxt)
    loop = [start]
    p = nxt[start]
    while p != start:
        loop.append(p)
        p = nxt[p]
    if len(loop) != len(edges):
        raise ValueError("the joined faces do not bound one polygon")
    return tuple(loop)


def merged_block(xs, ys, zs, kinds=None, periodic_x=False, periodic_y=False, merge_x=(), merge_xy=(), join=False):
    """Hexahedra, some of them merged into polyhedra whose sides are split faces: each (i, j, k) in
    merge_x joins hexahedra (i, j, k) and (i+1, j, k) into one cell of 12 points and 10
    quadrilateral faces; each (i, j, k) in merge_xy joins the 2 x 2 hexahedra from (i, j, k) into
    one cell of 18 points and 16 faces.  The neighbours keep their faces, so the mesh conforms.
    With join, the quadrilaterals that two merged cells share become one polygon (6 points for two
    of them, 8 for a 2 x 2 patch, whose middle point then belongs to no face)."""
    xs, ys, zs = (np.asarray(v, dtype=np.float64) for v in (xs, ys, zs))
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1

    def P(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    owner_of = {}
    groups = []
    for (i, j, k) in merge_xy:
        g = [(i, j, k), (i + 1, j, k), (i, j + 1, k), (i + 1, j + 1, k)]
        groups.append(g)
    for (i, j, k) in merge_x:
        groups.append([(i, j, k), (i + 1, j, k)])
    for gi, g in enumerate(groups):
        for h in g:
            if h in owner_of:
                raise ValueError(f"hexahedron {h} merged twice")
            owner_of[h] = gi
    cells = []
    done = set()
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                h = (i, j, k)
                if h in owner_of:
                    gi = owner_of[h]
                    if gi in done:
                        continue
                    done.add(gi)
                    faces = {}
                    for hh in groups[gi]:
                        for q in _hex_quads(P, *hh):
                            key = tuple(sorted(q))
                            if key in faces:
                                del faces[key]  # shared inside the merged cell
                            else:
                                faces[key] = q
                    cells.append(list(faces.values()))
                else:
                    cells.append(_hex_quads(P, i, j, k))
    if join:
        where = {}
        for c, faces in enumerate(cells):
            for q in faces:
                where.setdefault(tuple(sorted(q)), []).append(c)
        for c, faces in enumerate(cells):
            by_nbr, keep = {}, []
            for q in faces:
                cs = where[tuple(sorted(q))]
                if len(cs) == 2:
                    by_nbr.setdefault(cs[0] if cs[1] == c else cs[1], []).append(q)
                else:
                    keep.append(q)
            for qs in by_nbr.values():
                keep += [_join_loop(qs)] if len(qs) > 1 else qs
            cells[c] = keep
    return mesh_from_cells(_grid_points(xs, ys, zs), cells, xs, ys, zs, kinds, periodic_x, periodic_y)


def tet_block(xs, ys, zs, kinds=None, periodic_x=False, periodic_y=False):
    """Each hexahedron of the block cut into six tetrahedra along its main diagonal (Kuhn): cells
    6 c .. 6 c + 5, one per ordering of the axes."""
    xs, ys, zs = (np.asarray(v, dtype=np.float64) for v in (xs, ys, zs))
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    pts = _grid_points(xs, ys, zs)

    def P(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    # corner offsets of each tetrahedron's path, ordered for a positive volume (the coordinates
    # increase along every axis, so one orientation test per ordering of the axes holds for all)
    paths = []
    for perm in itertools.permutations(range(3)):
        v = [0, 0, 0]
        path = [(0, 0, 0)]
        for ax in perm:
            v[ax] += 1
            path.append(tuple(v))
        o = np.array(path, dtype=np.float64)
        if np.dot(o[1] - o[0], np.cross(o[2] - o[0], o[3] - o[0])) < 0:
            path[1], path[2] = path[2], path[1]
        paths.append(path)
    cells = []
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for path in paths:
                    a, b, c, d = (P(i + di, j + dj, k + dk) for di, dj, dk in path)
                    cells.append([(a, c, b), (a, b, d), (a, d, c), (b, c, d)])
    return mesh_from_cells(pts, cells, xs, ys, zs, kinds, periodic_x, periodic_y)


def _face_groups(mesh):
    """Faces grouped by their number of points: {n: (face ids, (len, n) point ids)}."""
    cnt = np.diff(mesh.face_ptr)
    out = {}
    for n in np.unique(cnt):
        f = np.nonzero(cnt == n)[0]
        idx = mesh.face_ptr[f][:, None] + np.arange(n)[None, :]
        out[int(n)] = (f, mesh.face_pts[idx])
    return out


def cell_geometry(mesh):
    """Cell volumes and centroids of any mesh with planar faces (faces fanned about their vertex
    mean, cells about the mean of their faces' vertex means)."""
    P = mesh.points
    groups = _face_groups(mesh)
    ref = np.zeros((mesh.n_cells, 3))
    cnt = np.zeros(mesh.n_cells)
    for n, (f, pts) in groups.items():
        m = P[pts].mean(axis=1)
        inner = f < mesh.n_internal
        cells = np.concatenate([mesh.owner[f], mesh.neighbour[f[inner]]])
        np.add.at(ref, cells, np.concatenate([m, m[inner]]))
        np.add.at(cnt, cells, 1.0)
    ref /= cnt[:, None]
    vol = np.zeros(mesh.n_cells)
    mom = np.zeros((mesh.n_cells, 3))
    for n, (f, pts) in groups.items():
        q = P[pts]
        ap = q.mean(axis=1)
        inner = f < mesh.n_internal
        cells = np.concatenate([mesh.owner[f], mesh.neighbour[f[inner]]])
        sgn = np.concatenate([np.ones(len(f)), -np.ones(int(inner.sum()))])
        qq = np.concatenate([q, q[inner]])
        aa = np.concatenate([ap, ap[inner]])
        r = ref[cells]
        for a in range(n):
            qa, qb = qq[:, a], qq[:, (a + 1) % n]
            tv = sgn * np.einsum("ij,ij->i", aa - r, np.cross(qa - r, qb - r)) / 6.0
            np.add.at(vol, cells, tv)
            np.add.at(mom, cells, (tv * 0.25)[:, None] * (r + aa + qa + qb))
    return vol, mom / vol[:, None]


def fluxes_from_potential(mesh, psi, n_gauss=8):
    """phi_f = circulation of the vector potential (0, 0, psi) around face f (Stokes), each edge's
    line integral of psi dz computed once (Gauss-Legendre with n_gauss points along the straight
    edge) and shared with opposite sign, so that every cell's fluxes sum to zero up to round-off.
    Wall and empty patches carry exactly zero flux."""
    P = mesh.points
    gx, gw = np.polynomial.legendre.leggauss(n_gauss)
    s = 0.5 * (gx + 1.0)
    w = 0.5 * gw
    fa, pa, pb = [], [], []
    for n, (f, pts) in _face_groups(mesh).items():
        for a in range(n):
            fa.append(f)
            pa.append(pts[:, a])
            pb.append(pts[:, (a + 1) % n])
    fa, pa, pb = np.concatenate(fa), np.concatenate(pa), np.concatenate(pb)
    lo, hi = np.minimum(pa, pb), np.maximum(pa, pb)
    keys, inv = np.unique(lo.astype(np.int64) * (len(P) + 1) + hi, return_inverse=True)
    ka, kb = keys // (len(P) + 1), keys % (len(P) + 1)
    xa, xb = P[ka], P[kb]
    val = np.zeros(len(keys))
    for q in range(n_gauss):
        x = xa + s[q] * (xb - xa)
        val += w[q] * psi(x[:, 0], x[:, 1], x[:, 2])
    val *= xb[:, 2] - xa[:, 2]
    val[xb[:, 2] == xa[:, 2]] = 0.0
    e = val[inv]
    e = np.where(pa == lo, e, -e)
    phi = np.zeros(mesh.n_faces)
    np.add.at(phi, fa, e)
    for p in mesh.patches:
        if p.kind in (0, 1):
            phi[p.start:p.start + p.size] = 0.0
    return phi


def _lattice(order):
    """Barycentric points (4 weights) of the interior of a tetrahedral lattice of the given order:
    equal-weight sample points of a tetrahedron."""
    pts = []
    for i in range(order):
        for j in range(order - i):
            for k in range(order - i - j):
                l = order - 1 - i - j - k
                pts.append((i + 0.25, j + 0.25, k + 0.25, l + 0.25))
    b = np.array(pts, dtype=np.float64)
    return b / b.sum(axis=1, keepdims=True)


def alpha_sampled(mesh, wet, order=6, chunk=20000):
    """Volume fractions of the region wet(x, y, z) > 0 per cell, by equal-weight sampling of the
    tetrahedra that fan each cell about its centroid over its face triangles (an input generator:
    a sharp field with fractional values near the surface, not an exact integral)."""
    vol, cen = cell_geometry(mesh)
    bary = _lattice(order)
    P = mesh.points
    acc = np.zeros(mesh.n_cells)
    for n, (f, pts) in _face_groups(mesh).items():
        q = P[pts]
        ap = q.mean(axis=1)
        inner = f < mesh.n_internal
        cells = np.concatenate([mesh.owner[f], mesh.neighbour[f[inner]]])
        qq = np.concatenate([q, q[inner]])
        aa = np.concatenate([ap, ap[inner]])
        for a in range(n):
            for lo in range(0, len(cells), chunk):
                sl = slice(lo, lo + chunk)
                t = np.stack([cen[cells[sl]], aa[sl], qq[sl, a], qq[sl, (a + 1) % n]], axis=1)
                tv = np.abs(np.einsum("ij,ij->i", t[:, 1] - t[:, 0],
                                      np.cross(t[:, 2] - t[:, 0], t[:, 3] - t[:, 0]))) / 6.0
                x = np.matmul(bary[None, :, :], t)
                fr = (wet(x[..., 0], x[..., 1], x[..., 2]) > 0).mean(axis=1)
                np.add.at(acc, cells[sl], tv * fr)
    return np.clip(acc / vol, 0.0, 1.0)


class PolyWorkload:
    """A steady flow on a tetrahedral or prismatic mesh: mesh, alpha0, phi_U(n), dt, n_steps."""

    def __init__(self, name, mesh, alpha0, phi, U, dt, n_steps):
        self.name, self.mesh, self.alpha0, self.dt, self.n_steps = name, mesh, alpha0, dt, n_steps
        self._phi, self._U = phi, U
        self.steady = True

    def phi_U(self, n):
        return self._phi, self._U


def poly_violent(kind="tet", nx=12, ny=6, nz=6, steps=8, co=0.5, perturb=0.0, seed=4):
    """The violent 3D workload's ingredients on tetrahedra, prisms, pyramids, hexahedra and prisms
    side by side ("mixed"), or hexahedra among merged polyhedra ("merged", "merged_joined",
    "merged_sparse"), with the interior points optionally moved at random: the box [0,2]x[0,1]x[0,1],
    periodic in x, a water column {x < 0.3, z < 0.6} joined to a wavy layer
    {z < 0.45 + 0.02 cos 4 pi x cos 4 pi y}, and the uniform + Taylor-Green flow (its fluxes from the
    vector potential along the straight edges)."""
    from .fields import UniformPlusTaylorGreen
    xs, ys, zs = np.linspace(0, 2, nx + 1), np.linspace(0, 1, ny + 1), np.linspace(0, 1, nz + 1)
    if kind == "mixed":
        mesh = mixed_block(xs, ys, zs, nx // 2, periodic_x=True)
    elif kind in ("merged", "merged_joined", "merged_sparse"):
        # polyhedra: pairs along x in every fourth column, 2 x 2 blocks in another; "merged_joined"
        # makes the faces two of them share one polygon of 6 or 8 points; "merged_sparse" keeps
        # only pairs in every eighth column (polyhedra a minority of the cells)
        mx = [(i, j, k) for k in range(nz) for j in range(ny) for i in range(1, nx - 1, 4)]
        mxy = [(i, j, k) for k in range(nz) for j in range(0, ny - 1, 2) for i in range(3, nx - 1, 4)]
        if kind == "merged_sparse":
            mx, mxy = [(i, j, k) for k in range(nz) for j in range(ny) for i in range(1, nx - 1, 8)], []
        mesh = merged_block(xs, ys, zs, periodic_x=True, merge_x=mx, merge_xy=mxy, join=kind == "merged_joined")
    else:
        build = {"tet": tet_block, "prism": prism_block, "pyramid": pyramid_block}[kind]
        mesh = build(xs, ys, zs, periodic_x=True)
    if perturb > 0.0:
        # move the interior grid points by up to perturb cell sizes (seeded), which bends the
        # quadrilaterals out of plane; the boundary stays flat, so the periodic sides still match
        P = mesh.points
        h = np.array([2.0 / nx, 1.0 / ny, 1.0 / nz])
        inner = np.all((P > 1e-12) & (P < np.array([2.0, 1.0, 1.0]) - 1e-12), axis=1)
        rng = np.random.default_rng(seed)
        P[inner] += rng.uniform(-perturb, perturb, (int(inner.sum()), 3)) * h
    flow = UniformPlusTaylorGreen(0.5, 1.0, 0.25)
    wet = lambda x, y, z: np.maximum(0.45 + 0.02 * np.cos(4 * np.pi * x) * np.cos(4 * np.pi * y) - z,
                                     np.minimum(0.3 - x, 0.6 - z))
    a0 = alpha_sampled(mesh, wet)
    phi = fluxes_from_potential(mesh, flow.psi)
    vol, cen = cell_geometry(mesh)
    U = flow.velocity_at(cen)
    from .fields import courant_dt
    dt = courant_dt(mesh, phi, co, volumes=vol)
    return PolyWorkload(f"violent_{kind}_{nx}x{ny}x{nz}", mesh, a0, phi, U, dt, steps)


def poly_airy(kind="prism", nx=64, ny=32, steps=8, co=0.5, steepness=0.07):
    """A linear Airy wave (as wavegen.configs.airy_slab) on a one-cell-thick slab of triangular
    prisms (kind "prism") or tetrahedra, [0, 2] x [0, 1], periodic in x, wavelength 1."""
    from .fields import AiryWave, courant_dt
    from .mesh import PATCH_EMPTY
    h = 1.0 / ny
    xs, ys, zs = np.linspace(0, 2, nx + 1), np.linspace(0, 1, ny + 1), np.array([0.0, h])
    build = prism_block if kind == "prism" else tet_block
    mesh = build(xs, ys, zs, kinds={"zmin": PATCH_EMPTY, "zmax": PATCH_EMPTY}, periodic_x=True)
    wave = AiryWave(1.0, steepness, 0.5, 1.0)
    wet = lambda x, y, z: 0.5 + 0.5 * steepness * np.cos(2 * np.pi * x) - y
    a0 = alpha_sampled(mesh, wet)
    vol, cen = cell_geometry(mesh)
    phi = fluxes_from_potential(mesh, lambda x, y, z: wave.psi(x, y, 0.0))
    u, v = wave.velocity(cen[:, 0], cen[:, 1], 0.0)
    U = np.ascontiguousarray(np.concatenate([u, v, np.zeros_like(u)]))
    dt = courant_dt(mesh, phi, co, volumes=vol)
    return PolyWorkload(f"airy_{kind}_{nx}x{ny}", mesh, a0, phi, U, dt, steps)
