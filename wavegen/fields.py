"""Initial volume fractions, face fluxes and cell velocities for the synthetic workloads.

Nothing here is part of the advection method: these functions only produce its
inputs (alpha at the start, the volumetric face fluxes phi_f and the cell
velocities U_P that the method takes, paper Section 3.2 problem statement).

* Volume fractions are the exact (2D) or quadrature (3D) cell integrals of the
  region below a prescribed free surface.
* Face fluxes come from a vector potential A = (0, 0, psi): by Stokes' theorem the
  flux through a face is the circulation of A around its edges, and only the
  vertical edges contribute.  Every edge integral is computed once per edge
  direction and shared, so each cell's fluxes sum to zero up to round-off.
"""
from __future__ import annotations

import numpy as np

from .mesh import Mesh, face_vertical_edges

G = 9.81


# --------------------------------------------------------------------------------------
# exact cell integrals below eta(x) = eta0 + amp*cos(kx*x + ph)
# --------------------------------------------------------------------------------------
def _cos_crossings(level, x0, x1, eta0, amp, kx, ph):
    """Candidate abscissae in (x0, x1) where eta(x) == level (masked to x1 when absent)."""
    out = []
    with np.errstate(invalid="ignore", divide="ignore"):
        r = (level - eta0) / amp
        ok = np.abs(r) < 1.0
        ac = np.arccos(np.clip(r, -1.0, 1.0))
    n0 = np.floor((kx * x0 + ph) / (2.0 * np.pi)) - 1.0
    for dn in range(4):
        n = n0 + dn
        for sgn in (1.0, -1.0):
            x = (sgn * ac + 2.0 * np.pi * n - ph) / kx
            good = ok & (x > x0) & (x < x1)
            out.append(np.where(good, x, x1))
    return out


def cell_fraction_below_cosine(x0, x1, y0, y1, eta0, amp, kx, ph=0.0):
    """(1/(dx*dy)) * integral over [x0,x1] of clamp(eta(x)-y0, 0, y1-y0) dx, exactly.

    All arguments are broadcastable arrays; eta(x) = eta0 + amp*cos(kx*x + ph).
    The integrand is split at the crossings of eta with y0 and y1 and each piece
    is integrated in closed form.
    """
    x0, x1, y0, y1, eta0, amp = np.broadcast_arrays(*[np.asarray(v, dtype=np.float64)
                                                     for v in (x0, x1, y0, y1, eta0, amp)])
    shape = x0.shape
    x0, x1, y0, y1, eta0, amp = (v.ravel() for v in (x0, x1, y0, y1, eta0, amp))
    if np.isscalar(kx) or np.ndim(kx) == 0:
        kx = np.full(x0.shape, float(kx))
    else:
        kx = np.broadcast_to(np.asarray(kx, dtype=np.float64), shape).ravel()
    if np.isscalar(ph) or np.ndim(ph) == 0:
        ph = np.full(x0.shape, float(ph))
    else:
        ph = np.broadcast_to(np.asarray(ph, dtype=np.float64), shape).ravel()
    amp_safe = np.where(amp == 0.0, 1.0, amp)
    cands = [x0] + _cos_crossings(y0, x0, x1, eta0, amp_safe, kx, ph) \
        + _cos_crossings(y1, x0, x1, eta0, amp_safe, kx, ph) + [x1]
    cands = np.stack(cands, axis=1)
    cands.sort(axis=1)
    a = cands[:, :-1]
    b = cands[:, 1:]
    mid = 0.5 * (a + b)
    eta_mid = eta0[:, None] + amp[:, None] * np.cos(kx[:, None] * mid + ph[:, None])
    dy = (y1 - y0)[:, None]
    full = eta_mid >= y1[:, None]
    part = (eta_mid > y0[:, None]) & ~full
    lin = (eta0 - y0)[:, None] * (b - a) + (amp / kx)[:, None] * (
        np.sin(kx[:, None] * b + ph[:, None]) - np.sin(kx[:, None] * a + ph[:, None]))
    area = np.where(full, dy * (b - a), np.where(part, lin, 0.0)).sum(axis=1)
    frac = area / ((x1 - x0) * (y1 - y0))
    return np.clip(frac, 0.0, 1.0).reshape(shape)


def alpha_cosine_2d(mesh: Mesh, eta0, amp, kx, ph=0.0):
    """Cell volume fractions of the region y < eta0 + amp*cos(kx*x + ph) (2D slab mesh)."""
    xs, ys = mesh.xs, mesh.ys
    nx, ny, nz = mesh.shape
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    fr = cell_fraction_below_cosine(xs[I], xs[I + 1], ys[J], ys[J + 1], eta0, amp, kx, ph)
    return np.ascontiguousarray(np.tile(fr.ravel(), nz))


# --------------------------------------------------------------------------------------
# fluxes from a vector potential (0, 0, psi)
# --------------------------------------------------------------------------------------
def fluxes_from_edge_integral(mesh: Mesh, edge_integral):
    """phi_f = sum over the face's vertical edges of integral psi dz (Stokes).

    ``edge_integral(x, y, z_lo, z_hi)`` returns the integral of psi along the
    vertical edge from z_lo to z_hi (z_lo < z_hi).  It is evaluated once per edge
    in the upward direction and negated for downward traversals, so the two faces
    sharing an edge use bitwise-opposite values.
    """
    fidx, xe, ye, z0, z1 = face_vertical_edges(mesh)
    up = z1 > z0
    lo = np.where(up, z0, z1)
    hi = np.where(up, z1, z0)
    val = edge_integral(xe, ye, lo, hi)
    val = np.where(up, val, -val)
    phi = np.zeros(mesh.n_faces)
    np.add.at(phi, fidx, val)
    # wall / empty patches carry no flux by construction of the potentials used here;
    # force exact zeros so that round-off never leaks through a closed boundary
    for p in mesh.patches:
        if p.kind in (0, 1):
            phi[p.start:p.start + p.size] = 0.0
    return phi


def courant_dt(mesh: Mesh, phi, co, volumes=None):
    """dt giving max cell Courant number ``co``, Co_P = 0.5*dt*sum_f |phi_f| / V_P."""
    V = mesh.cell_volumes_structured() if volumes is None else volumes
    s = np.zeros(mesh.n_cells)
    a = np.abs(phi)
    np.add.at(s, mesh.owner, a)
    ni = mesh.n_internal
    np.add.at(s, mesh.neighbour, a[:ni])
    # owner side of every face, neighbour side of interior faces: each cell counts each of its
    # faces once (both faces of a cyclic pair are boundary faces of their own cells)
    return float(co / np.max(0.5 * s / V))


# --------------------------------------------------------------------------------------
# linear (Airy) progressive wave, mirrored into the air above the surface
# --------------------------------------------------------------------------------------
class AiryWave:
    """Linear progressive wave eta = d + (H/2) cos(k x - w t) in a box [x0,x1]x[0,h].

    Stream function psi = (H/2)(w/k) f(y) cos(k x - w t) with f = sinh(k y)/sinh(k d)
    in the water and f = sinh(k (h - y))/sinh(k (h - d)) in the air, so that the
    bottom and the lid are streamlines.  Velocity u = d(psi)/dy, v = -d(psi)/dx.
    """

    def __init__(self, wavelength, height, depth, top):
        self.k = 2.0 * np.pi / wavelength
        self.H = float(height)
        self.d = float(depth)
        self.h = float(top)
        self.w = float(np.sqrt(G * self.k * np.tanh(self.k * self.d)))

    def _f(self, y):
        k, d, h = self.k, self.d, self.h
        water = np.sinh(k * y) / np.sinh(k * d)
        air = np.sinh(k * (h - y)) / np.sinh(k * (h - d))
        return np.where(y <= d, water, air)

    def _fy(self, y):
        k, d, h = self.k, self.d, self.h
        water = k * np.cosh(k * y) / np.sinh(k * d)
        air = -k * np.cosh(k * (h - y)) / np.sinh(k * (h - d))
        return np.where(y <= d, water, air)

    def psi(self, x, y, t):
        return 0.5 * self.H * (self.w / self.k) * self._f(y) * np.cos(self.k * x - self.w * t)

    def velocity(self, x, y, t):
        c = 0.5 * self.H * (self.w / self.k)
        u = c * self._fy(y) * np.cos(self.k * x - self.w * t)
        v = c * self.k * self._f(y) * np.sin(self.k * x - self.w * t)
        return u, v

    def fluxes(self, mesh: Mesh, t):
        return fluxes_from_edge_integral(mesh, lambda x, y, z0, z1: self.psi(x, y, t) * (z1 - z0))

    def cell_velocity(self, mesh: Mesh, t):
        c = mesh.cell_centres_structured()
        u, v = self.velocity(c[:, 0], c[:, 1], t)
        return np.ascontiguousarray(np.concatenate([u, v, np.zeros_like(u)]))

    def alpha0(self, mesh: Mesh):
        return alpha_cosine_2d(mesh, self.d, 0.5 * self.H, self.k, 0.0)


# --------------------------------------------------------------------------------------
# uniform stream + Taylor-Green vortex (3D, w = 0)
# --------------------------------------------------------------------------------------
class UniformPlusTaylorGreen:
    """U = (u0, 0, 0) + A (sin kx cos ky cos kz, -cos kx sin ky cos kz, 0).

    Vector potential (0, 0, psi) with psi = u0*y + (A/k) sin kx sin ky cos kz.
    """

    def __init__(self, u0, amp, period):
        self.u0 = float(u0)
        self.A = float(amp)
        self.k = 2.0 * np.pi / period

    def edge_integral(self, x, y, z0, z1):
        k, A = self.k, self.A
        return self.u0 * y * (z1 - z0) + (A / k) * np.sin(k * x) * np.sin(k * y) * (
            np.sin(k * z1) - np.sin(k * z0)) / k

    def fluxes(self, mesh: Mesh):
        return fluxes_from_edge_integral(mesh, self.edge_integral)

    def psi(self, x, y, z):
        k, A = self.k, self.A
        return self.u0 * y + (A / k) * np.sin(k * x) * np.sin(k * y) * np.cos(k * z)

    def velocity_at(self, c):
        """Cell velocities (SoA) at the points c (n, 3)."""
        k, A = self.k, self.A
        x, y, z = c[:, 0], c[:, 1], c[:, 2]
        u = self.u0 + A * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
        v = -A * np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
        return np.ascontiguousarray(np.concatenate([u, v, np.zeros_like(u)]))

    def cell_velocity(self, mesh: Mesh):
        c = mesh.cell_centres_structured()
        k, A = self.k, self.A
        x, y, z = c[:, 0], c[:, 1], c[:, 2]
        u = self.u0 + A * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
        v = -A * np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
        return np.ascontiguousarray(np.concatenate([u, v, np.zeros_like(u)]))


def alpha_column_plus_wave_3d(mesh: Mesh, col_x, col_top, eta0, amp, kw, n_gauss=16):
    """Volume fractions of {z < eta(x,y)} U {x < col_x and z < col_top}, z vertical.

    eta(x, y) = eta0 + amp cos(kw x) cos(kw y).  In each cell the fraction is
    integrated exactly in y (eta is a cosine in y for fixed x) and by
    ``n_gauss``-point Gauss-Legendre in x, on the parts of the cell left and right
    of x = col_x.  Cells that the wave surface cannot reach are classified directly.
    """
    xs, ys, zs = mesh.xs, mesh.ys, mesh.zs
    nx, ny, nz = mesh.shape
    alpha = np.zeros((nz, ny, nx))
    eta_lo, eta_hi = eta0 - abs(amp), eta0 + abs(amp)
    dz = np.diff(zs)
    gx, gw = np.polynomial.legendre.leggauss(n_gauss)
    for kk in range(nz):
        z0, z1 = zs[kk], zs[kk + 1]
        # column part (x < col_x): h = max(eta, col_top) = col_top there
        col_frac_z = np.clip((col_top - z0) / dz[kk], 0.0, 1.0)
        # wave part
        if z1 <= eta_lo:
            wave = np.ones((ny, nx))
        elif z0 >= eta_hi:
            wave = np.zeros((ny, nx))
        else:
            wave = np.zeros((ny, nx))
            for ii in range(nx):
                xa, xb = xs[ii], xs[ii + 1]
                xq = 0.5 * (xa + xb) + 0.5 * (xb - xa) * gx
                wq = 0.5 * gw  # weights for the mean over [xa, xb]
                a_y = amp * np.cos(kw * xq)  # amplitude of the y-cosine at each x node
                Y0 = ys[:-1][:, None]
                Y1 = ys[1:][:, None]
                fr = cell_fraction_below_cosine(Y0, Y1, z0, z1, eta0, a_y[None, :], kw)
                wave[:, ii] = fr @ wq
        # combine: left of col_x the region is full up to col_top (>= eta everywhere)
        frac_left = np.clip((col_x - xs[:-1]) / np.diff(xs), 0.0, 1.0)  # share of cell with x<col_x
        cell_has_col = frac_left > 0.0
        out = wave.copy()
        if np.any(cell_has_col):
            # cells fully left: column dominates (col_top >= eta_hi); split cells: mix
            ii_split = np.nonzero(cell_has_col & (frac_left < 1.0))[0]
            ii_full = np.nonzero(frac_left >= 1.0)[0]
            out[:, ii_full] = col_frac_z
            for ii in ii_split:
                xa, xb = xs[ii], col_x
                xq = 0.5 * (xa + xb) + 0.5 * (xb - xa) * gx
                # left part: column fraction; right part: wave part integrated on [col_x, x1]
                xa2, xb2 = col_x, xs[ii + 1]
                xq2 = 0.5 * (xa2 + xb2) + 0.5 * (xb2 - xa2) * gx
                a_y = amp * np.cos(kw * xq2)
                if z1 <= eta_lo:
                    wr = np.ones(ny)
                elif z0 >= eta_hi:
                    wr = np.zeros(ny)
                else:
                    fr = cell_fraction_below_cosine(ys[:-1][:, None], ys[1:][:, None], z0, z1,
                                                    eta0, a_y[None, :], kw)
                    wr = fr @ (0.5 * gw)
                fl = frac_left[ii]
                out[:, ii] = fl * col_frac_z + (1.0 - fl) * wr
        alpha[kk] = out
    return np.ascontiguousarray(np.clip(alpha, 0.0, 1.0).ravel())


# --------------------------------------------------------------------------------------
# dynamic pressure for the ghost-fluid face data
# --------------------------------------------------------------------------------------
def dynamic_pressure(xc, alpha, rho_heavy, rho_light, g, level, seed, noise=0.02, p_atm=1.0e5):
    """A synthetic dynamic pressure p_d = p - rho g . x per cell, an input of the ghost-fluid face
    data: hydrostatic about a flat free surface through the point ``level`` (p = p_atm there), the
    fluid of each cell chosen by alpha > 1/2, plus seeded normal noise of relative size ``noise``
    of rho_heavy |g| times the extent of the cell centres (a stand-in for the flow's dynamic part).
    xc: (n_cells, 3) cell centres."""
    xc = np.asarray(xc, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    rho = np.where(np.asarray(alpha) > 0.5, rho_heavy, rho_light)
    base = p_atm - rho * float(g @ np.asarray(level, dtype=np.float64))
    ext = float(np.ptp(xc, axis=0).max())
    rng = np.random.default_rng(seed)
    return base + noise * rho_heavy * float(np.linalg.norm(g)) * ext * rng.standard_normal(len(rho))
