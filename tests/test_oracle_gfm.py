"""Pins of the oracle's ghost-fluid face data (Eqs. 12-20, reading R16) against fields whose
answer the physics fixes, never against the formulas themselves:

* a hydrostatic state (continuous pressure, Eq. 3) with the free surface on a tilted plane: the
  dynamic pressure is constant in each fluid, so the heavy fluid's value extended to a dry cell is
  the heavy constant and the light fluid's extended to a wet cell is the light constant;
* a two-fluid field that is linear on each side of the surface, with the jump of Eq. 7 and the
  continuous beta grad p_d of Eq. 8: the one-sided extrapolations are exact, and so is the flux
  through the face that beta_w implies;
* a cyclic face against the same geometry unrolled into an internal face;
* equal densities (no jump: the plain values) and faces away from the surface.

rho^+ is the heavy fluid's density, rho^- the light fluid's; a cell is wet iff alpha > 1/2.
"""
import numpy as np
import pytest

import wavegen as W

RHO_H, RHO_L = 1000.0, 1.2


def _graded(n, lo, hi, ratio, rng):
    """n cells over [lo, hi] with widths drawn in [1, ratio] (seeded)."""
    w = rng.uniform(1.0, ratio, n)
    return lo + (hi - lo) * np.concatenate([[0.0], np.cumsum(w) / w.sum()])


def _crossing(alpha, own, nbr):
    return (alpha[own] > 0.5) != (alpha[nbr] > 0.5)


def test_hydrostatic_state_is_reproduced(oracle_lib):
    """Free surface on the plane ghat . (x - x0) = 0 for a tilted gravity g; alpha linear in
    ghat . x so that Eq. 13 puts x_Gamma on that plane; p_d = p0 - rho g . x0 in each fluid."""
    rng = np.random.default_rng(5)
    xs, ys, zs = _graded(9, 0.0, 1.0, 3.0, rng), _graded(7, 0.0, 0.8, 2.0, rng), _graded(8, 0.0, 0.9, 2.5, rng)
    mesh = W.hex_block(xs, ys, zs, periodic_x=False)
    g = np.array([1.3, -2.1, -9.4])
    gh = g / np.linalg.norm(g)
    x0 = np.array([0.45, 0.37, 0.52])
    xc = mesh.cell_centres_structured()
    alpha = 0.5 + (xc - x0) @ gh / 4.0  # heavy fluid lies along g; no clipping needed
    assert alpha.min() > 0.0 and alpha.max() < 1.0
    p0 = 1.0e5
    c_heavy, c_light = p0 - RHO_H * g @ x0, p0 - RHO_L * g @ x0
    wet = alpha > 0.5
    p_d = np.where(wet, c_heavy, c_light)
    out = oracle_lib.OracleMesh(mesh).gfm_faces(alpha, p_d, RHO_H, RHO_L, g)

    own, nbr = mesh.owner, mesh.neighbour
    ni = mesh.n_internal
    cross = _crossing(alpha, own[:ni], nbr)
    assert cross.sum() > 50
    f = np.nonzero(cross)[0]
    tol = 1e-12 * p0
    dry_side = np.where(wet[own[f]], out["ghost_nbr"][f], out["ghost_own"][f])
    wet_side = np.where(wet[own[f]], out["ghost_own"][f], out["ghost_nbr"][f])
    assert np.abs(dry_side - c_heavy).max() <= tol
    assert np.abs(wet_side - c_light).max() <= tol
    assert np.abs(out["jump"][f] - (c_light - c_heavy)).max() <= tol
    assert np.all((out["lambda"][f] >= 0.0) & (out["lambda"][f] <= 1.0))
    # faces away from the surface and boundary faces carry the plain values
    g_f = np.nonzero(~cross)[0]
    assert np.all(out["lambda"][g_f] == -1.0) and np.all(out["jump"][g_f] == 0.0)
    assert np.array_equal(out["ghost_own"][g_f], p_d[own[g_f]])
    assert np.array_equal(out["ghost_nbr"][g_f], p_d[nbr[g_f]])
    b = np.arange(ni, mesh.n_faces)
    assert np.all(out["lambda"][b] == -1.0)
    assert np.array_equal(out["ghost_own"][b], p_d[own[b]]) and np.array_equal(out["ghost_nbr"][b], p_d[own[b]])


@pytest.mark.parametrize("heavy_right", [True, False])
def test_piecewise_linear_two_fluid_field_is_reproduced(oracle_lib, heavy_right):
    """alpha depends on x alone and crosses 1/2 at x = xg; on each row (y, z) the dynamic pressure
    is linear in x on each side, with slopes s+ / rho+ = s- / rho- (Eq. 8) and the jump
    p_d^- - p_d^+ = (rho+ - rho-) g . x_Gamma at x_Gamma = (xg, y, z) (Eq. 7)."""
    rng = np.random.default_rng(7 if heavy_right else 8)
    xs = _graded(14, 0.0, 1.4, 4.0, rng)
    ys, zs = _graded(3, 0.0, 0.3, 2.0, rng), _graded(4, 0.0, 0.4, 2.0, rng)
    mesh = W.hex_block(xs, ys, zs, periodic_x=False)
    xc = mesh.cell_centres_structured()
    sgn = 1.0 if heavy_right else -1.0
    g = np.array([sgn * 7.0, 2.5, -5.0])
    xg = 0.5 * (xc[:, 0].min() + xc[:, 0].max()) + 0.013
    alpha = 0.5 + sgn * (xc[:, 0] - xg) / 3.0
    wet = alpha > 0.5
    s_h = 830.0
    s_l = s_h * RHO_L / RHO_H
    a_row = 2.0e4 + 1.0e3 * xc[:, 1] - 3.0e3 * xc[:, 2]  # p_d^+ at x_Gamma, per row
    xgam = np.stack([np.full(len(xc), xg), xc[:, 1], xc[:, 2]], 1)
    h_row = (RHO_H - RHO_L) * xgam @ g
    p_heavy = a_row + s_h * (xc[:, 0] - xg)
    p_light = a_row + h_row + s_l * (xc[:, 0] - xg)
    p_d = np.where(wet, p_heavy, p_light)
    out = oracle_lib.OracleMesh(mesh).gfm_faces(alpha, p_d, RHO_H, RHO_L, g)

    own, nbr = mesh.owner, mesh.neighbour
    f = np.nonzero(_crossing(alpha, own[:mesh.n_internal], nbr))[0]
    assert len(f) == 12  # one crossing per row
    P, N = own[f], nbr[f]
    wP = wet[P]
    W_, D = np.where(wP, P, N), np.where(wP, N, P)
    tol = 1e-11 * 2.0e4
    ghost_at_dry = np.where(wP, out["ghost_nbr"][f], out["ghost_own"][f])
    ghost_at_wet = np.where(wP, out["ghost_own"][f], out["ghost_nbr"][f])
    assert np.abs(ghost_at_dry - p_heavy[D]).max() <= tol
    assert np.abs(ghost_at_wet - p_light[W_]).max() <= tol
    assert np.abs(out["jump"][f] - h_row[P]).max() <= tol
    # Eq. 13 from the owner: x_Gamma at xg
    lam = out["lambda"][f]
    assert np.abs(xc[P, 0] + lam * (xc[N, 0] - xc[P, 0]) - xg).max() <= 1e-13
    # the flux through the face implied by beta_w equals the exact beta grad p_d
    bh, bl = 1.0 / RHO_H, 1.0 / RHO_L
    flux = bh * bl * (p_d[D] - p_d[W_] - out["jump"][f]) / ((xc[D, 0] - xc[W_, 0]) * out["beta_w"][f])
    assert np.abs(flux - bh * s_h).max() <= 1e-12 * bh * s_h


def test_cyclic_face_matches_the_unrolled_internal_face(oracle_lib):
    """A row periodic in x whose free surface crosses the cyclic face, with gravity along x
    (g . translation != 0), against the same cells unrolled: the far cell's image placed before
    the first cell makes the pair an internal face of a plain block."""
    rng = np.random.default_rng(9)
    xs = _graded(10, 0.0, 1.0, 2.0, rng)
    ys, zs = np.array([0.0, 0.2, 0.5]), np.array([0.0, 0.3])
    per = W.hex_block(xs, ys, zs, periodic_x=True)
    nx = len(xs) - 1
    unrolled = W.hex_block(np.concatenate([[xs[0] - (xs[-1] - xs[-2])], xs]), ys, zs, periodic_x=False)
    g = np.array([4.0, -1.0, -9.0])
    a_per = np.tile(np.array([0.83, 0.7, 0.55, 0.4, 0.2, 0.1, 0.05, 0.12, 0.3, 0.37]), 2)  # wet at the start
    p_per = rng.normal(1.0e4, 300.0, per.n_cells)
    # unrolled cell 0 of each row is the image of the row's last cell
    ny = 2
    a_un = np.concatenate([[a_per[r * nx + nx - 1]] + list(a_per[r * nx:(r + 1) * nx]) for r in range(ny)])
    p_un = np.concatenate([[p_per[r * nx + nx - 1]] + list(p_per[r * nx:(r + 1) * nx]) for r in range(ny)])
    o_per = oracle_lib.OracleMesh(per).gfm_faces(a_per, p_per, RHO_H, RHO_L, g)
    o_un = oracle_lib.OracleMesh(unrolled).gfm_faces(a_un, p_un, RHO_H, RHO_L, g)

    xmin = per.patches[0]
    for r in range(ny):
        fp = xmin.start + r  # cyclic flux face owned by the row's first cell
        assert per.owner[fp] == r * nx
        cu = r * (nx + 1)  # the image cell of the unrolled row
        fu = np.nonzero((unrolled.owner[:unrolled.n_internal] == cu) & (unrolled.neighbour == cu + 1))[0]
        assert len(fu) == 1
        fu = fu[0]
        assert o_per["lambda"][fp] >= 0.0
        # owner and neighbour trade places between the two
        assert abs(o_per["lambda"][fp] - (1.0 - o_un["lambda"][fu])) <= 1e-14
        for k in ("jump", "beta_w"):
            assert abs(o_per[k][fp] - o_un[k][fu]) <= 1e-12 * max(1.0, abs(o_un[k][fu])), k
        assert abs(o_per["ghost_own"][fp] - o_un["ghost_nbr"][fu]) <= 1e-11 * 1.0e4
        assert abs(o_per["ghost_nbr"][fp] - o_un["ghost_own"][fu]) <= 1e-11 * 1.0e4
        # the partner face on the other patch carries nothing of its own
        fs = per.patches[1].start + r
        assert o_per["lambda"][fs] == -1.0 and o_per["jump"][fs] == 0.0
    # the internal crossings are the same points in both
    jp, ju = np.sort(o_per["jump"][o_per["lambda"] >= 0]), np.sort(o_un["jump"][o_un["lambda"] >= 0])
    assert len(jp) == len(ju) == 2 * ny and np.abs(jp - ju).max() <= 1e-12 * np.abs(ju).max()


def test_equal_densities_carry_no_jump(oracle_lib):
    rng = np.random.default_rng(10)
    w = W.perturbed_box(steps=1)
    a = rng.uniform(0.0, 1.0, w.mesh.n_cells)
    p = rng.normal(0.0, 10.0, w.mesh.n_cells)
    out = oracle_lib.OracleMesh(w.mesh).gfm_faces(a, p, 998.0, 998.0, np.array([0.3, -0.2, -9.81]))
    ni = w.mesh.n_internal
    own, nbr = w.mesh.owner[:ni], w.mesh.neighbour
    f = np.nonzero(_crossing(a, own, nbr))[0]
    assert len(f) > 100
    assert np.all(out["jump"][f] == 0.0)
    assert np.abs(out["beta_w"][f] - 1.0 / 998.0).max() <= 1e-18
    assert np.abs(out["ghost_own"][:ni] - p[own]).max() <= 1e-13 * 10
    assert np.abs(out["ghost_nbr"][:ni] - p[nbr]).max() <= 1e-13 * 10
