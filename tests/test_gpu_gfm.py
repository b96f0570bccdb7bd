"""Ghost-fluid face data (Eqs. 12-20, reading R16) on the GPU against the oracle, through the C
interface (iso_gfm_faces).  Same seeded inputs on both sides: volume fractions from the workload
generators (the initial fields, seeded random fields, and states the oracle advected), dynamic
pressures from wavegen.dynamic_pressure.

lambda and beta_w depend on the volume fractions alone and are computed by the same IEEE
operations in the same order on both sides (no fused multiply-add): bit for bit.  The jump and the
ghost values also use the cell centroids, which the library and the oracle compute each in their
own summation order; they agree to a few ulps of the centroids, amplified by at most the
coefficients of Eq. 20 and its mirror (beta/beta_w, up to the density ratio):
    |jump_gpu - jump_oracle|   <= 1e-13 |rho^+ - rho^-| |g| max|x|
    |ghost_gpu - ghost_oracle| <= 1e-13 (1 + max(beta^+, beta^-)/beta_w) (max|p_d| + |rho^+ - rho^-| |g| max|x|)
"""
import numpy as np
import pytest

import wavegen as W
from tests.gpuutil import say, to_dev

pytestmark = pytest.mark.gpu

RHO_H, RHO_L = 1000.0, 1.2
KEYS = ("lambda", "jump", "beta_w", "ghost_own", "ghost_nbr")


def _gpu(mesh, alpha, p_d, g, rho_h=RHO_H, rho_l=RHO_L):
    import torch
    from paper_1804_01130_amd import Mesh, Plan, default_options
    gm = Mesh.from_arrays(mesh)
    plan = Plan(gm, default_options())
    out = plan.gfm_faces(to_dev(alpha), to_dev(p_d), rho_h, rho_l, g)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    plan.close()
    return res


def _centres(O, mesh):
    return O.OracleMesh(mesh).geometry()[0]


def _compare(got, exp, p_d, g, xc, rho_h=RHO_H, rho_l=RHO_L):
    assert np.array_equal(got["lambda"], exp["lambda"])
    assert np.array_equal(got["beta_w"], exp["beta_w"])
    hscale = abs(rho_h - rho_l) * np.linalg.norm(g) * np.abs(xc).max()
    dj = np.abs(got["jump"] - exp["jump"])
    assert dj.max() <= 1e-13 * hscale, dj.max()
    bw = np.where(exp["beta_w"] > 0, exp["beta_w"], np.inf)
    amp = 1.0 + max(1.0 / rho_h, 1.0 / rho_l) / bw
    tol = 1e-13 * amp * (np.abs(p_d).max() + hscale)
    worst = 0.0
    for k in ("ghost_own", "ghost_nbr"):
        d = np.abs(got[k] - exp[k])
        assert np.all(d <= tol), (k, int(np.argmax(d - tol)), d.max())
        worst = max(worst, float((d / tol).max()))
    exact = all(np.array_equal(got[k], exp[k]) for k in KEYS)
    n_if = int((exp["lambda"] >= 0).sum())
    say(f"[gpu]   {n_if} interface faces; max |d jump| = {dj.max():.2e}; ghosts at {worst:.2e} of the "
        f"tolerance; bit for bit: {exact}")
    return n_if


def _oracle_state(O, w, steps):
    om = O.OracleMesh(w.mesh)
    a = np.array(w.alpha0, copy=True)
    for n in range(steps):
        phi, U = w.phi_U(n)
        a, _ = om.step(a, phi, U, w.dt)
    return a


CASES = {
    # name: (workload, oracle steps before, gravity, still-water level)
    "airy_128x64": (lambda: W.airy_slab(128, 64, 32, 0.07, 0.5, 8, "airy_128x64"), 4, (0.0, -9.81, 0.0),
                    (0.0, 0.5, 0.0)),
    "airy_128x64_tilted_g": (lambda: W.airy_slab(128, 64, 32, 0.07, 0.5, 8, "airy_128x64"), 0, (1.7, -9.6, 0.0),
                             (0.0, 0.5, 0.0)),
    "violent_32x16x16": (lambda: W.violent_3d(nx=32, ny=16, nz=16, steps=4), 3, (0.0, 0.0, -9.81),
                         (0.0, 0.0, 0.5)),
    "perturbed_10x7x6": (lambda: W.perturbed_box(steps=4), 2, (0.4, -0.3, -9.7), (0.0, 0.0, 0.5)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_gfm_faces_match_oracle(oracle_lib, name):
    make, steps, g, level = CASES[name]
    w = make()
    say(f"[gpu] ghost-fluid face data: {name} cells={w.mesh.n_cells} after {steps} oracle steps")
    a = _oracle_state(oracle_lib, w, steps)
    xc = _centres(oracle_lib, w.mesh)
    p = W.dynamic_pressure(xc, a, RHO_H, RHO_L, g, level, seed=21)
    got = _gpu(w.mesh, a, p, g)
    exp = oracle_lib.OracleMesh(w.mesh).gfm_faces(a, p, RHO_H, RHO_L, np.array(g))
    assert _compare(got, exp, p, g, xc) > 20


@pytest.mark.parametrize("seed", [31, 32])
def test_gfm_faces_random_fields(oracle_lib, seed):
    """alpha ~ U[0, 1] per cell (seeded) on the graded box: about half of all faces are interface
    faces, with lambda anywhere in [0, 1], including ties at alpha = 1/2 exactly."""
    w = W.violent_3d(nx=16, ny=12, nz=10, steps=1)
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 1.0, w.mesh.n_cells)
    a[rng.integers(0, w.mesh.n_cells, 40)] = 0.5
    g = (0.3, 0.2, -9.81)
    xc = _centres(oracle_lib, w.mesh)
    p = W.dynamic_pressure(xc, a, RHO_H, RHO_L, g, (0.0, 0.0, 0.5), seed=seed)
    say(f"[gpu] ghost-fluid face data, random field: seed={seed}")
    got = _gpu(w.mesh, a, p, g)
    exp = oracle_lib.OracleMesh(w.mesh).gfm_faces(a, p, RHO_H, RHO_L, np.array(g))
    assert _compare(got, exp, p, g, xc) > 0.3 * w.mesh.n_internal


def test_gfm_faces_across_cyclic_pairs(oracle_lib):
    """Rows periodic in x whose free surface crosses the cyclic faces, gravity with a component
    along the translation (the partner cell's centre must be moved into the owner's frame), and
    the reversed density ratio."""
    rng = np.random.default_rng(41)
    xs = np.concatenate([[0.0], np.cumsum(rng.uniform(1.0, 2.0, 12))])
    mesh = W.hex_block(xs, np.linspace(0.0, 0.6, 5), np.linspace(0.0, 0.4, 3), periodic_x=True, periodic_y=True)
    row = np.array([0.83, 0.7, 0.55, 0.4, 0.2, 0.1, 0.05, 0.12, 0.3, 0.37, 0.45, 0.49])
    a = np.tile(row, mesh.n_cells // 12) + rng.uniform(-0.02, 0.02, mesh.n_cells)
    g = (4.0, -1.0, -9.0)
    xc = _centres(oracle_lib, mesh)
    for rho_h, rho_l in ((RHO_H, RHO_L), (1.0, 1025.0)):
        p = W.dynamic_pressure(xc, a, rho_h, rho_l, g, (0.5, 0.0, 0.0), seed=42)
        say(f"[gpu] ghost-fluid face data across cyclic pairs: rho = {rho_h}, {rho_l}")
        got = _gpu(mesh, a, p, g, rho_h, rho_l)
        exp = oracle_lib.OracleMesh(mesh).gfm_faces(a, p, rho_h, rho_l, np.array(g))
        _compare(got, exp, p, g, xc, rho_h, rho_l)
        n_cyc = int((exp["lambda"][mesh.n_internal:] >= 0).sum())
        assert n_cyc >= 8, n_cyc


def test_gfm_faces_hydrostatic_state():
    """A still free surface on a tilted plane with hydrostatic pressure: each fluid's p_d is
    constant, and the GPU's ghost values are the other fluid's constant (no oracle involved)."""
    w = W.violent_3d(nx=24, ny=16, nz=12, steps=1)
    xc = w.mesh.cell_centres_structured()
    g = np.array([1.3, -2.1, -9.4])
    x0 = np.array([0.5, 0.5, 0.45])
    a = 0.5 + (xc - x0) @ (g / np.linalg.norm(g)) / 4.0
    p0 = 1.0e5
    ch, cl = p0 - RHO_H * g @ x0, p0 - RHO_L * g @ x0
    wet = a > 0.5
    p = np.where(wet, ch, cl)
    say("[gpu] ghost-fluid face data, hydrostatic state")
    got = _gpu(w.mesh, a, p, g)
    ni = w.mesh.n_internal
    own, nbr = w.mesh.owner[:ni], w.mesh.neighbour
    f = np.nonzero(wet[own] != wet[nbr])[0]
    assert len(f) > 100
    at_dry = np.where(wet[own[f]], got["ghost_nbr"][f], got["ghost_own"][f])
    at_wet = np.where(wet[own[f]], got["ghost_own"][f], got["ghost_nbr"][f])
    assert np.abs(at_dry - ch).max() <= 1e-12 * p0 and np.abs(at_wet - cl).max() <= 1e-12 * p0


def test_gfm_faces_full_size(oracle_lib):
    """The graded 3D box at its full size (4.19M cells, 12.7M faces): the state after one step of
    the oracle; every face against the oracle."""
    w = W.violent_3d()
    say(f"[gpu] ghost-fluid face data at full size: {w.mesh.n_cells} cells")
    om = oracle_lib.OracleMesh(w.mesh)
    phi, U = w.phi_U(0)
    a, _ = om.step(w.alpha0, phi, U, w.dt)
    xc = om.geometry()[0]
    g = (0.0, 0.0, -9.81)
    p = W.dynamic_pressure(xc, a, RHO_H, RHO_L, g, (0.0, 0.0, 0.5), seed=51)
    got = _gpu(w.mesh, a, p, g)
    exp = om.gfm_faces(a, p, RHO_H, RHO_L, np.array(g))
    assert _compare(got, exp, p, g, xc) > 10000


def test_gfm_faces_argument_errors():
    import torch
    from paper_1804_01130_amd import IsoError, Mesh, Plan, default_options
    w = W.violent_3d(nx=8, ny=6, nz=6, steps=1)
    plan = Plan(Mesh.from_arrays(w.mesh), default_options())
    a = to_dev(w.alpha0)
    p = torch.zeros_like(a)
    with pytest.raises(IsoError):
        plan.gfm_faces(a, p, 0.0, 1.0, (0, 0, -9.81))
    with pytest.raises(IsoError):
        plan.gfm_faces(a, p, 1000.0, float("nan"), (0, 0, -9.81))
    with pytest.raises(IsoError):
        plan.gfm_faces(a, p, 1000.0, 1.0, (0, float("inf"), -9.81))
    buf = torch.empty(w.mesh.n_faces, dtype=torch.float64, device=a.device)
    with pytest.raises(IsoError):  # two outputs in one buffer
        plan.gfm_faces(a, p, 1000.0, 1.0, (0, 0, -9.81), out={k: buf for k in KEYS})
    plan.close()


@pytest.mark.parametrize("fill", [0.0, 0.5, 1.0])
def test_gfm_faces_without_interface(fill):
    """A uniform field (all dry, exactly 1/2 everywhere, all wet): no face lies on the surface, so
    every face carries lambda = -1, no jump, and the plain cell values, bit for bit."""
    w = W.violent_3d(nx=12, ny=8, nz=6, steps=1)
    a = np.full(w.mesh.n_cells, fill)
    p = np.random.default_rng(81).normal(1.0e5, 50.0, w.mesh.n_cells)
    got = _gpu(w.mesh, a, p, (0.0, 0.0, -9.81))
    ni = w.mesh.n_internal
    own, nbr = w.mesh.owner, w.mesh.neighbour
    assert np.all(got["lambda"] == -1.0) and np.all(got["jump"] == 0.0) and np.all(got["beta_w"] == 0.0)
    assert np.array_equal(got["ghost_own"], p[own])
    assert np.array_equal(got["ghost_nbr"][:ni], p[nbr])
