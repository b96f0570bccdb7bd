"""Structured hexahedral meshes written out in face-based (owner/neighbour) form.

The finite-volume mesh of the method is an arbitrary polyhedral mesh in which
every face knows the cell that owns it and, for interior faces, the neighbouring
cell (paper, Section 3, the polyhedral control volume figure).  This module only
produces such meshes for block-structured grids; it holds no part of the
advection arithmetic.

Conventions of the produced mesh
--------------------------------
* points: (n_points, 3) float64.  Point (i, j, k) has id ``i + (nx+1)*(j + (ny+1)*k)``;
  a periodic direction keeps both the x=0 and the x=L copies of its points.
* cells: cell (i, j, k) has id ``i + nx*(j + ny*k)``.
* faces: interior faces first, in upper-triangular order (sorted by owner, then
  by neighbour); then the boundary faces patch after patch.  The points of a face
  are listed counter-clockwise seen from outside its owner, so the right-hand
  normal points from owner to neighbour (or out of the domain).
* patches: WALL and EMPTY faces carry no flux; INOUT faces carry flux with a
  prescribed inflow volume fraction; CYCLIC patches come in pairs: face n of a
  cyclic patch coincides with face n of its partner after the patch translation
  (x_partner = x_this + translation).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PATCH_WALL = 0
PATCH_EMPTY = 1
PATCH_INOUT = 2
PATCH_CYCLIC = 3


@dataclass
class Patch:
    name: str
    kind: int
    start: int
    size: int
    partner: int = -1
    translation: tuple = (0.0, 0.0, 0.0)
    alpha_in: float = 0.0


@dataclass
class Mesh:
    points: np.ndarray
    face_ptr: np.ndarray
    face_pts: np.ndarray
    owner: np.ndarray
    neighbour: np.ndarray
    n_cells: int
    patches: list = field(default_factory=list)
    # structured-grid metadata (for generators and diagnostics only)
    shape: tuple = (0, 0, 0)
    xs: np.ndarray | None = None
    ys: np.ndarray | None = None
    zs: np.ndarray | None = None

    @property
    def n_points(self) -> int:
        return int(self.points.shape[0])

    @property
    def n_faces(self) -> int:
        return int(self.owner.shape[0])

    @property
    def n_internal(self) -> int:
        return int(self.neighbour.shape[0])

    def patch_arrays(self):
        """Patch table as flat arrays, in the order the C interfaces take them."""
        n = len(self.patches)
        start = np.array([p.start for p in self.patches], dtype=np.int32)
        size = np.array([p.size for p in self.patches], dtype=np.int32)
        kind = np.array([p.kind for p in self.patches], dtype=np.int32)
        partner = np.array([p.partner for p in self.patches], dtype=np.int32)
        trans = np.array([p.translation for p in self.patches], dtype=np.float64).reshape(n, 3)
        ain = np.array([p.alpha_in for p in self.patches], dtype=np.float64)
        return start, size, kind, partner, np.ascontiguousarray(trans.reshape(-1)), ain

    def cell_centres_structured(self) -> np.ndarray:
        """Box centres of a structured mesh, (n_cells, 3), cell-id order."""
        xc = 0.5 * (self.xs[1:] + self.xs[:-1])
        yc = 0.5 * (self.ys[1:] + self.ys[:-1])
        zc = 0.5 * (self.zs[1:] + self.zs[:-1])
        Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
        return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def cell_volumes_structured(self) -> np.ndarray:
        dx = np.diff(self.xs)
        dy = np.diff(self.ys)
        dz = np.diff(self.zs)
        Z, Y, X = np.meshgrid(dz, dy, dx, indexing="ij")
        return (X * Y * Z).ravel()


def graded_halves(n_half: int, lo: float, mid: float, ratio: float) -> np.ndarray:
    """Node coordinates of a grid graded geometrically towards ``mid``.

    ``2*n_half`` cells span [lo, 2*mid-lo]; the cell widths shrink geometrically
    from lo to mid, the largest being ``ratio`` times the smallest, and the upper
    half mirrors the lower one.
    """
    r = ratio ** (-1.0 / (n_half - 1)) if n_half > 1 else 1.0
    w = r ** np.arange(n_half)
    w *= (mid - lo) / w.sum()
    lower = lo + np.concatenate([[0.0], np.cumsum(w)])
    lower[-1] = mid
    upper = (2.0 * mid - lower[::-1])[1:]
    upper[-1] = 2.0 * mid - lo
    return np.concatenate([lower, upper])


def hex_block(xs, ys, zs, kinds=None, periodic_x=True, alpha_in=None, periodic_y=False) -> Mesh:
    """Build a block of (nx, ny, nz) hexahedra with node coordinates xs, ys, zs.

    ``kinds`` maps each of 'xmin','xmax','ymin','ymax','zmin','zmax' to a patch
    kind; with ``periodic_x`` (``periodic_y``) the two x (y) patches become a cyclic pair.
    """
    xs = np.asarray(xs, dtype=np.float64)
    ys = np.asarray(ys, dtype=np.float64)
    zs = np.asarray(zs, dtype=np.float64)
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    kinds = dict(kinds or {})
    if periodic_x:
        kinds["xmin"] = PATCH_CYCLIC
        kinds["xmax"] = PATCH_CYCLIC
    if periodic_y:
        kinds["ymin"] = PATCH_CYCLIC
        kinds["ymax"] = PATCH_CYCLIC
    for key in ("xmin", "xmax", "ymin", "ymax", "zmin", "zmax"):
        kinds.setdefault(key, PATCH_WALL)
    alpha_in = dict(alpha_in or {})

    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    points = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def P(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    def C(i, j, k):
        return i + nx * (j + ny * k)

    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i = i.ravel(); j = j.ravel(); k = k.ravel()
    cid = C(i, j, k)

    # canonical local faces of cell (i,j,k), listed counter-clockwise from outside
    def face_xp(i, j, k):  # +x
        return np.stack([P(i + 1, j, k), P(i + 1, j + 1, k), P(i + 1, j + 1, k + 1), P(i + 1, j, k + 1)], 1)

    def face_xm(i, j, k):  # -x
        return np.stack([P(i, j + 1, k), P(i, j, k), P(i, j, k + 1), P(i, j + 1, k + 1)], 1)

    def face_yp(i, j, k):  # +y
        return np.stack([P(i + 1, j + 1, k), P(i, j + 1, k), P(i, j + 1, k + 1), P(i + 1, j + 1, k + 1)], 1)

    def face_ym(i, j, k):  # -y
        return np.stack([P(i, j, k), P(i + 1, j, k), P(i + 1, j, k + 1), P(i, j, k + 1)], 1)

    def face_zp(i, j, k):  # +z
        return np.stack([P(i, j, k + 1), P(i + 1, j, k + 1), P(i + 1, j + 1, k + 1), P(i, j + 1, k + 1)], 1)

    def face_zm(i, j, k):  # -z
        return np.stack([P(i, j, k), P(i, j + 1, k), P(i + 1, j + 1, k), P(i + 1, j, k)], 1)

    own_l, nbr_l, pts_l = [], [], []
    m = i < nx - 1
    own_l.append(cid[m]); nbr_l.append(C(i[m] + 1, j[m], k[m])); pts_l.append(face_xp(i[m], j[m], k[m]))
    m = j < ny - 1
    own_l.append(cid[m]); nbr_l.append(C(i[m], j[m] + 1, k[m])); pts_l.append(face_yp(i[m], j[m], k[m]))
    m = k < nz - 1
    own_l.append(cid[m]); nbr_l.append(C(i[m], j[m], k[m] + 1)); pts_l.append(face_zp(i[m], j[m], k[m]))
    own = np.concatenate(own_l)
    nbr = np.concatenate(nbr_l)
    fpts = np.concatenate(pts_l)
    order = np.lexsort((nbr, own))
    own, nbr, fpts = own[order], nbr[order], fpts[order]

    patches = []
    b_own, b_pts = [], []
    start = own.shape[0]

    def add_patch(name, mask, facefn):
        nonlocal start
        ii, jj, kk = i[mask], j[mask], k[mask]
        b_own.append(C(ii, jj, kk))
        b_pts.append(facefn(ii, jj, kk))
        n = int(mask.sum())
        patches.append(Patch(name, kinds[name], start, n, alpha_in=float(alpha_in.get(name, 0.0))))
        start += n

    add_patch("xmin", i == 0, face_xm)
    add_patch("xmax", i == nx - 1, face_xp)
    add_patch("ymin", j == 0, face_ym)
    add_patch("ymax", j == ny - 1, face_yp)
    add_patch("zmin", k == 0, face_zm)
    add_patch("zmax", k == nz - 1, face_zp)
    if periodic_x:
        L = float(xs[-1] - xs[0])
        patches[0].partner = 1
        patches[0].translation = (L, 0.0, 0.0)
        patches[1].partner = 0
        patches[1].translation = (-L, 0.0, 0.0)
    if periodic_y:
        Ly = float(ys[-1] - ys[0])
        patches[2].partner = 3
        patches[2].translation = (0.0, Ly, 0.0)
        patches[3].partner = 2
        patches[3].translation = (0.0, -Ly, 0.0)

    owner = np.concatenate([own] + b_own).astype(np.int32)
    face_pts4 = np.concatenate([fpts] + b_pts).astype(np.int32)
    n_faces = owner.shape[0]
    face_ptr = (4 * np.arange(n_faces + 1)).astype(np.int32)
    return Mesh(points=points, face_ptr=face_ptr, face_pts=np.ascontiguousarray(face_pts4.ravel()),
                owner=owner, neighbour=nbr.astype(np.int32), n_cells=nx * ny * nz, patches=patches,
                shape=(nx, ny, nz), xs=xs, ys=ys, zs=zs)


def face_vertical_edges(mesh: Mesh):
    """Vertical (z-directed) edges of every face, for flux evaluation by Stokes' theorem.

    Returns (face index, x, y, z_from, z_to) arrays for every pair of consecutive
    face points that share x and y; walking the face counter-clockwise from
    outside gives the edge direction.  Cached on the mesh.
    """
    cached = getattr(mesh, "_vertical_edges", None)
    if cached is not None:
        return cached
    mesh._vertical_edges = _face_vertical_edges(mesh)
    return mesh._vertical_edges


def _face_vertical_edges(mesh: Mesh):
    nf = mesh.n_faces
    fp = mesh.face_pts.reshape(nf, 4)
    P = mesh.points
    fidx, xe, ye, z0, z1 = [], [], [], [], []
    for a in range(4):
        pa = fp[:, a]
        pb = fp[:, (a + 1) % 4]
        same = (P[pa, 0] == P[pb, 0]) & (P[pa, 1] == P[pb, 1]) & (P[pa, 2] != P[pb, 2])
        idx = np.nonzero(same)[0]
        fidx.append(idx)
        xe.append(P[pa[idx], 0]); ye.append(P[pa[idx], 1])
        z0.append(P[pa[idx], 2]); z1.append(P[pb[idx], 2])
    return (np.concatenate(fidx), np.concatenate(xe), np.concatenate(ye),
            np.concatenate(z0), np.concatenate(z1))
