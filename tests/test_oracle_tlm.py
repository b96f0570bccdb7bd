"""Pins of the oracle's tangent of the step (complex step, implicit isovalue derivative).

Each pin ties the derivative to something other than the tangent code: central differences of
the real oracle step, the exact derivative of planar-interface transport, exact volume
conservation, and the transpose identity of the gradient assembled from tangents.  Directions
avoid topology changes: alpha moves only in cells strictly inside (0, 1), and flux
perturbations are divergence-free (from a stream function), so no bulk cell crosses a bound.
"""
import numpy as np
import pytest

import wavegen as W


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def _psi_slab(mesh, rng):
    L = mesh.xs[-1] - mesh.xs[0]
    H = mesh.ys[-1] - mesh.ys[0]
    c = rng.standard_normal(3)
    return lambda x, y, z0, z1: np.sin(np.pi * y / H) * (c[0] * np.cos(2 * np.pi * x / L) + c[1] * np.sin(
        4 * np.pi * x / L) + c[2] * np.cos(6 * np.pi * x / L)) * (z1 - z0)


def _psi_box(mesh, rng):
    """Vector potential (0, 0, psi) of a flow with no flux through the y and z walls."""
    L = mesh.xs[-1] - mesh.xs[0]
    c = rng.standard_normal(3)

    def edge(x, y, z0, z1):
        g = c[0] * np.cos(2 * np.pi * x / L) + c[1] * np.sin(2 * np.pi * x / L)
        # integral of sin(pi y) g(x) (1 + c2 cos(pi z)) dz
        return np.sin(np.pi * y) * g * ((z1 - z0) + c[2] * (np.sin(np.pi * z1) - np.sin(np.pi * z0)) / np.pi)
    return edge


def _directions(w, rng, psi):
    a0 = w.alpha0
    inner = (a0 > 1e-4) & (a0 < 1 - 1e-4)
    da = rng.standard_normal(w.mesh.n_cells) * inner
    phi, _ = w.phi_U(0)
    dp = W.fluxes_from_edge_integral(w.mesh, psi(w.mesh, rng))
    dp *= np.abs(phi).max() / np.abs(dp).max()
    return da, dp


@pytest.mark.parametrize("case", ["airy_32x16", "violent_12x9x8"])
def test_tangent_matches_central_differences(O, case):
    """Central differences with a step small enough to stay clear of the nearest kink (a cut point
    reaching a vertex lies within 1e-5 of the 3D state) agree to 1e-6 relative, the bar the
    adjoint is held to.  The 3D box has 9 cells in y so that no face lies on a zero of the
    Taylor-Green flux, where the upwind cell would switch with the sign of the perturbation."""
    rng = np.random.default_rng(11)
    if case == "airy_32x16":
        w, psi = W.airy_slab(32, 16, 16, 0.07, 0.45, 3, case), _psi_slab
    else:
        w, psi = W.violent_3d(nx=12, ny=9, nz=8, steps=3), _psi_box
    om = O.OracleMesh(w.mesh)
    phi, U = w.phi_U(0)
    checked = 0
    for trial in range(3):
        da, dp = _directions(w, rng, psi)
        _, t = om.step_tlm(w.alpha0, phi, U, w.dt, da, dp)
        eps = 1e-7
        ap, _ = om.step(w.alpha0 + eps * da, phi + eps * dp, U, w.dt)
        am, _ = om.step(w.alpha0 - eps * da, phi - eps * dp, U, w.dt)
        fd = (ap - am) / (2 * eps)
        assert np.abs(t).max() > 0
        assert np.abs(fd - t).max() <= 1e-6 * np.abs(t).max(), (trial, np.abs(fd - t).max(), np.abs(t).max())
        checked += 1
    assert checked == 3


def test_tangent_of_band_shift_is_exact(O):
    """A flat band in uniform oblique flow is transported exactly, so moving its upper edge by ds
    moves the result's upper edge by ds: in the cut row d alpha/ds = 1/dy before and after."""
    ny, H = 24, 1.5
    mesh = W.hex_block(np.linspace(0, 1, 17), np.linspace(0, H, ny + 1), [0.0, 1 / 16], periodic_x=True,
                       periodic_y=True, kinds={"zmin": W.PATCH_EMPTY, "zmax": W.PATCH_EMPTY})
    phi = W.fluxes_from_edge_integral(mesh, lambda x, y, z0, z1: (0.7 * y - 0.6 * x) * (z1 - z0))
    U = np.concatenate([np.full(mesh.n_cells, 0.7), np.full(mesh.n_cells, 0.6), np.zeros(mesh.n_cells)])
    dt = W.courant_dt(mesh, phi, 0.45)
    s1, s0 = 0.9021, 0.3137
    a0 = W.alpha_cosine_2d(mesh, s1, 0.0, 1.0) - W.alpha_cosine_2d(mesh, s0, 0.0, 1.0)
    dy = H / ny
    yc = mesh.cell_centres_structured()[:, 1]
    row = lambda s: np.abs(yc - (np.floor(s / dy) + 0.5) * dy) < 0.25 * dy
    assert np.floor(s1 / dy) == np.floor((s1 + 0.6 * dt) / dy)  # the edge stays in its row
    da = row(s1) / dy
    om = O.OracleMesh(mesh)
    a1, t = om.step_tlm(a0, phi, U, dt, da, None)
    exact = W.alpha_cosine_2d(mesh, s1 + 0.6 * dt, 0.0, 1.0) - W.alpha_cosine_2d(mesh, s0 + 0.6 * dt, 0.0, 1.0)
    assert np.abs(a1 - exact).max() <= 1e-12
    assert np.abs(t - row(s1 + 0.6 * dt) / dy).max() <= 1e-9 / dy


def test_tangent_conserves_volume_without_chopping(O):
    """Without chopping the step conserves the total volume exactly for any inputs (closed
    domain), so the tangent of sum V alpha_new equals that of sum V alpha, for any flux direction."""
    w = W.airy_slab(32, 16, 16, 0.08, 0.5, 3, "t")
    om = O.OracleMesh(w.mesh)
    _, V = om.geometry()
    phi, U = w.phi_U(1)
    rng = np.random.default_rng(5)
    inner = (w.alpha0 > 1e-4) & (w.alpha0 < 1 - 1e-4)
    da = rng.standard_normal(w.mesh.n_cells) * inner
    dp = rng.standard_normal(w.mesh.n_faces) * np.abs(phi).max()
    opts = O.default_opts(clip=0)
    _, t = om.step_tlm(w.alpha0, phi, U, w.dt, da, dp, opts=opts)
    assert abs(V @ t - V @ da) <= 1e-12 * (np.abs(V * t).sum() + np.abs(V * da).sum())


def test_gradient_is_transpose_of_tangent(O):
    """The per-component gradient assembly satisfies <g, d> = <abar, tangent(d)> for any d."""
    w = W.airy_slab(16, 8, 8, 0.08, 0.5, 3, "t")
    om = O.OracleMesh(w.mesh)
    phi, U = w.phi_U(0)
    rng = np.random.default_rng(9)
    abar = rng.standard_normal(w.mesh.n_cells)
    ga, gp = om.gradient(w.alpha0, phi, U, w.dt, abar)
    for _ in range(3):
        da = rng.standard_normal(w.mesh.n_cells)
        dp = rng.standard_normal(w.mesh.n_faces) * np.abs(phi).max()
        _, t = om.step_tlm(w.alpha0, phi, U, w.dt, da, dp)
        lhs, rhs = ga @ da + gp @ dp, abar @ t
        assert abs(lhs - rhs) <= 1e-11 * (np.abs(ga * da).sum() + np.abs(gp * dp).sum() + 1e-300)


def test_tangent_on_nonplanar_faces_matches_central_differences(O):
    """Randomly displaced interior points (non-planar faces, in/out patches): alpha directions in
    cells strictly inside (0, 1), central differences of the real oracle step."""
    w = W.perturbed_box(nx=8, ny=7, nz=6, steps=2)
    om = O.OracleMesh(w.mesh)
    phi, U = w.phi_U(0)
    rng = np.random.default_rng(21)
    inner = (w.alpha0 > 1e-4) & (w.alpha0 < 1 - 1e-4)
    for trial in range(3):
        da = rng.standard_normal(w.mesh.n_cells) * inner
        _, t = om.step_tlm(w.alpha0, phi, U, w.dt, da, None)
        eps = 1e-7
        ap, _ = om.step(w.alpha0 + eps * da, phi, U, w.dt)
        am, _ = om.step(w.alpha0 - eps * da, phi, U, w.dt)
        fd = (ap - am) / (2 * eps)
        assert np.abs(t).max() > 0
        assert np.abs(fd - t).max() <= 1e-6 * np.abs(t).max(), (trial, np.abs(fd - t).max(), np.abs(t).max())
