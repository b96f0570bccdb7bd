"""The five synthetic workloads of the advection step, seeded and reproducible.

Each builder returns a ``Workload``: a mesh, the initial volume fraction, and a
function giving (phi, U) for step n.  Random draws use numpy's PCG64
(``numpy.random.default_rng(seed)``) in the order written in each builder.

The paper's own cases (a progressive wave in a 2D tank, green water on a deck in
3D; Section 4) need its full flow solver; these workloads reproduce their shapes
(wave steepness, cells per wavelength, graded hexahedra, a violent 3D surface)
with analytic, divergence-free velocity fields instead.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable

import numpy as np

from .fields import AiryWave, UniformPlusTaylorGreen, alpha_column_plus_wave_3d, alpha_cosine_2d, \
    courant_dt, fluxes_from_edge_integral
from .mesh import PATCH_EMPTY, PATCH_INOUT, PATCH_WALL, Mesh, graded_halves, hex_block


@dataclass
class Workload:
    name: str
    mesh: Mesh
    alpha0: np.ndarray
    dt: float
    n_steps: int
    fields: Callable  # fields(n) -> (phi[n_faces], U[3*n_cells]) for step n
    steady: bool = False
    meta: dict = field(default_factory=dict)

    def phi_U(self, n):
        return self.fields(n)


def slab_mesh(nx, ny, x1, y1):
    """One-cell-thick 2D slab [0,x1]x[0,y1]x[0,dz], dz = dx; periodic x, walls y, empty z."""
    xs = np.linspace(0.0, x1, nx + 1)
    ys = np.linspace(0.0, y1, ny + 1)
    dz = x1 / nx
    zs = np.array([0.0, dz])
    return hex_block(xs, ys, zs, kinds={"ymin": PATCH_WALL, "ymax": PATCH_WALL,
                                        "zmin": PATCH_EMPTY, "zmax": PATCH_EMPTY}, periodic_x=True)


def cosine_uniform(nx=64, ny=32, steps=20, co=0.25) -> Workload:
    """64x32x1 on [0,2]x[0,1], alpha below 0.5 + 0.05 cos(2 pi x), U = (1,0,0)."""
    mesh = slab_mesh(nx, ny, 2.0, 1.0)
    alpha0 = alpha_cosine_2d(mesh, 0.5, 0.05, 2.0 * np.pi)
    phi = fluxes_from_edge_integral(mesh, lambda x, y, z0, z1: y * (z1 - z0))
    U = np.concatenate([np.ones(mesh.n_cells), np.zeros(mesh.n_cells), np.zeros(mesh.n_cells)])
    dt = courant_dt(mesh, phi, co)
    return Workload("cosine_2d_64x32", mesh, alpha0, dt, steps, lambda n: (phi, U), steady=True,
                    meta={"eta0": 0.5, "amp": 0.05, "kx": 2.0 * np.pi, "u": 1.0})


def airy_slab(nx, ny, wavelength_cells, steepness, co, steps, name) -> Workload:
    """Linear Airy wave in a slab of nx x ny square cells, depth = half the height."""
    dx = 1.0 / wavelength_cells  # one wavelength = 1 length unit
    x1 = nx * dx
    y1 = ny * dx
    mesh = slab_mesh(nx, ny, x1, y1)
    wave = AiryWave(wavelength=1.0, height=steepness * 1.0, depth=0.5 * y1, top=y1)
    alpha0 = wave.alpha0(mesh)
    phi0 = wave.fluxes(mesh, 0.0)
    dt = courant_dt(mesh, phi0, co)

    def fields(n):
        t = (n + 0.5) * dt
        return wave.fluxes(mesh, t), wave.cell_velocity(mesh, t)

    return Workload(name, mesh, alpha0, dt, steps, fields,
                    meta={"steepness": steepness, "co": co, "omega": wave.w, "k": wave.k,
                          "depth": wave.d, "top": wave.h})


def airy_1024x256(seed=0, steps=200) -> Workload:
    rng = np.random.default_rng(seed)
    steep = float(rng.uniform(0.02, 0.08))
    return airy_slab(1024, 256, 256, steep, 0.5, steps, "airy_2d_1024x256")


def violent_3d(nx=256, ny=128, nz=128, steps=100, co=0.5) -> Workload:
    """256x128x128 graded (4:1 towards z=0.5) box [0,2]x[0,1]x[0,1], z vertical.

    Water column (x<0.3, z<0.6) plus a 3D wave z < 0.45 + 0.02 cos(4 pi x) cos(4 pi y);
    steady flux field of U = (0.5,0,0) + Taylor-Green vortex (amplitude 1, period 0.25).
    """
    xs = np.linspace(0.0, 2.0, nx + 1)
    ys = np.linspace(0.0, 1.0, ny + 1)
    zs = graded_halves(nz // 2, 0.0, 0.5, 4.0)
    mesh = hex_block(xs, ys, zs, kinds={"ymin": PATCH_WALL, "ymax": PATCH_WALL,
                                        "zmin": PATCH_WALL, "zmax": PATCH_WALL}, periodic_x=True)
    alpha0 = alpha_column_plus_wave_3d(mesh, 0.3, 0.6, 0.45, 0.02, 4.0 * np.pi)
    flow = UniformPlusTaylorGreen(0.5, 1.0, 0.25)
    phi = flow.fluxes(mesh)
    U = flow.cell_velocity(mesh)
    dt = courant_dt(mesh, phi, co)
    return Workload(f"violent_3d_{nx}x{ny}x{nz}", mesh, alpha0, dt, steps, lambda n: (phi, U),
                    steady=True)


def airy_ensemble(n_domains=64, seed=1, steps=100):
    """Independent Airy domains: nx = 32*U{4..32}, ny = 16*U{4..16}, lambda = nx/4 cells,
    steepness ~ U[0.02,0.10], Courant ~ U[0.3,0.5]; drawn per domain in that order."""
    rng = np.random.default_rng(seed)
    out = []
    for d in range(n_domains):
        nx = 32 * int(rng.integers(4, 33))
        ny = 16 * int(rng.integers(4, 17))
        steep = float(rng.uniform(0.02, 0.10))
        co = float(rng.uniform(0.3, 0.5))
        out.append(airy_slab(nx, ny, nx // 4, steep, co, steps, f"airy_member{d}_{nx}x{ny}"))
    return out


def adjoint_case(seed=2, steps=50):
    """256x128x1 Airy wave (lambda = 64 cells) and the target from a perturbed steepness."""
    rng = np.random.default_rng(seed)
    steep = float(rng.uniform(0.02, 0.08))
    delta = float(rng.uniform(-0.1, 0.1))
    base = airy_slab(256, 128, 64, steep, 0.5, steps, "airy_2d_256x128")
    target = airy_slab(256, 128, 64, steep * (1.0 + delta), 0.5, steps, "airy_2d_256x128_target")
    base.meta["delta"] = delta
    return base, target


def tiny_slab(nx=4, ny=4, steps=3):
    """Small cosine case for quick parity checks."""
    return cosine_uniform(nx=nx, ny=ny, steps=steps)


def perturbed_box(nx=10, ny=7, nz=6, amp=0.15, seed=3, steps=8, co=0.4) -> Workload:
    """A hexahedral box [0,1]^3 whose interior points are displaced at random by up to ``amp``
    times the spacing (seeded), so that its faces are not planar; in/out patches at x = 0
    (inflow with alpha = 1) and x = 1, walls elsewhere.  alpha, fluxes and velocities are those of
    the undisplaced box (a column plus a wave, a uniform stream plus a Taylor-Green vortex): they
    are inputs of the step here, not a flow of the displaced geometry."""
    rng = np.random.default_rng(seed)
    xs = np.linspace(0.0, 1.0, nx + 1)
    ys = np.linspace(0.0, 1.0, ny + 1)
    zs = np.linspace(0.0, 1.0, nz + 1)
    box = hex_block(xs, ys, zs, kinds={"xmin": PATCH_INOUT, "xmax": PATCH_INOUT}, periodic_x=False,
                    alpha_in={"xmin": 1.0})
    alpha0 = alpha_column_plus_wave_3d(box, 0.3, 0.6, 0.45, 0.08, 2.0 * np.pi)
    flow = UniformPlusTaylorGreen(0.5, 0.8, 0.5)
    phi = flow.fluxes(box)
    U = flow.cell_velocity(box)
    P = box.points.copy()
    h = np.array([xs[1] - xs[0], ys[1] - ys[0], zs[1] - zs[0]])
    inner = np.all((P > 1e-12) & (P < 1.0 - 1e-12), axis=1)
    P[inner] += amp * h * rng.uniform(-1.0, 1.0, size=(int(inner.sum()), 3))
    mesh = Mesh(P, box.face_ptr, box.face_pts, box.owner, box.neighbour, box.n_cells, box.patches, box.shape,
                box.xs, box.ys, box.zs)
    dt = courant_dt(box, phi, co)
    return Workload(f"perturbed_box_{nx}x{ny}x{nz}", mesh, alpha0, dt, steps, lambda n: (phi, U), steady=True,
                    meta={"amp": amp})
