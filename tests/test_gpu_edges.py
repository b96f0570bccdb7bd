"""Edge cases of the step on the GPU against the oracle.

A field with no interface cell, a step with no flux, a field whose cells are all flat, and random
fields in which every cell is an interface cell with arbitrary vertex values: saddle faces, cells
with more than two of them (the interval solve hands those to the generic one), vertex-value
jumps, and bounding in about one cell in twenty.  Same seeded inputs on both sides;
|delta alpha| <= 1e-10.
"""
import numpy as np
import pytest

import wavegen as W
from tests.gpuutil import gpu_plan, gpu_traced_step, say, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _gpu_run(plan, a0, phi, U, dt, steps):
    import torch
    a = to_dev(a0)
    b = torch.empty_like(a)
    tphi, tU = to_dev(phi), to_dev(U)
    for _ in range(steps):
        plan.step(a, tphi, tU, dt, out=b)
        a, b = b, a
    torch.cuda.synchronize()
    return a.cpu().numpy()


def _oracle_run(om, a0, phi, U, dt, steps):
    a = np.array(a0, copy=True)
    for _ in range(steps):
        a, _ = om.step(a, phi, U, dt)
    return a


def test_no_interface_cell(oracle_lib):
    """Water below the face plane z = 1/2 of the graded box: the first step has no interface cell,
    so every face carries alpha_up phi dt; the following steps grow an interface."""
    w = W.violent_3d(nx=12, ny=8, nz=8, steps=4)
    say(f"[gpu] no interface cell: {w.name}")
    a0 = (w.mesh.cell_centres_structured()[:, 2] < 0.5).astype(np.float64)
    phi, U = w.phi_U(0)
    gm, plan = gpu_plan(w.mesh)
    _, st, _ = gpu_traced_step(plan, gm, a0, phi, U, w.dt)
    assert st["n_surface"] == 0
    om = oracle_lib.OracleMesh(w.mesh)
    err = np.abs(_gpu_run(plan, a0, phi, U, w.dt, 4) - _oracle_run(om, a0, phi, U, w.dt, 4)).max()
    say(f"[gpu]   max |gpu - oracle| = {err:.3e}")
    assert err <= TOL


def test_no_flux_leaves_alpha_unchanged():
    """phi = 0 and U = 0: every dV is zero and alpha_new is alpha, bit for bit."""
    w = W.violent_3d(nx=12, ny=8, nz=8, steps=4)
    say(f"[gpu] no flux: {w.name}")
    phi = np.zeros(w.mesh.n_faces)
    U = np.zeros(3 * w.mesh.n_cells)
    gm, plan = gpu_plan(w.mesh)
    out, st, _ = gpu_traced_step(plan, gm, w.alpha0, phi, U, w.dt)
    assert st["n_surface"] > 0
    assert np.array_equal(out, w.alpha0)


def test_all_cells_flat(oracle_lib):
    """alpha = 1/2 everywhere: every cell is an interface cell whose vertex values coincide, so
    each is treated as a bulk cell."""
    w = W.violent_3d(nx=12, ny=8, nz=8, steps=4)
    say(f"[gpu] all cells flat: {w.name}")
    a0 = np.full(w.mesh.n_cells, 0.5)
    phi, U = w.phi_U(0)
    gm, plan = gpu_plan(w.mesh)
    _, st, _ = gpu_traced_step(plan, gm, a0, phi, U, w.dt)
    assert st["n_flat"] > 0
    om = oracle_lib.OracleMesh(w.mesh)
    err = np.abs(_gpu_run(plan, a0, phi, U, w.dt, 3) - _oracle_run(om, a0, phi, U, w.dt, 3)).max()
    say(f"[gpu]   max |gpu - oracle| = {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("mesh,seed", [("graded", 11), ("graded", 12), ("perturbed", 13)])
def test_random_fields(oracle_lib, mesh, seed):
    """alpha ~ U[0.02, 0.98] per cell (seeded): every cell is an interface cell, vertex patterns
    are arbitrary, and bounding flags about one cell in twenty.  Planar hexahedra (graded box)
    and non-planar ones (perturbed box)."""
    w = (W.violent_3d(nx=16, ny=12, nz=10, steps=4) if mesh == "graded"
         else W.perturbed_box(nx=10, ny=8, nz=7, steps=4))
    say(f"[gpu] random field: {w.name} seed={seed}")
    a0 = np.random.default_rng(seed).uniform(0.02, 0.98, w.mesh.n_cells)
    phi, U = w.phi_U(0)
    gm, plan = gpu_plan(w.mesh)
    _, st, _ = gpu_traced_step(plan, gm, a0, phi, U, w.dt)
    say(f"[gpu]   interface cells {st['n_surface']}, flagged for bounding {st['n_bound_active']}, "
        f"max rounds {st['max_root_iter']}, not converged {st['n_nonconverged']}")
    assert st["n_surface"] > 0.5 * w.mesh.n_cells
    assert st["n_nonconverged"] == 0
    om = oracle_lib.OracleMesh(w.mesh)
    err = np.abs(_gpu_run(plan, a0, phi, U, w.dt, 3) - _oracle_run(om, a0, phi, U, w.dt, 3)).max()
    say(f"[gpu]   max |gpu - oracle| after 3 steps = {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("mesh,seed", [("graded", 21), ("perturbed", 22)])
def test_isovalue_of_every_cell_near_its_extreme_vertices(oracle_lib, mesh, seed):
    """Cells with alpha close to 0 or 1 next to cells far from it put the isovalue in the lowest or
    highest interval of their sorted vertex values (next to one vertex).  Every reconstructed cell's
    isovalue, not a sample of them, must cut off alpha V to 1e-12 by the oracle's sub-volume, or sit
    at the same vertex value where the sub-volume jumps across alpha V."""
    w = (W.violent_3d(nx=16, ny=12, nz=10, steps=1) if mesh == "graded"
         else W.perturbed_box(nx=10, ny=8, nz=7, steps=1))
    n = w.mesh.n_cells
    rng = np.random.default_rng(seed)
    pick = rng.uniform(size=n)
    a0 = np.where(pick < 0.45, rng.uniform(1e-6, 0.03, n),
                  np.where(pick < 0.9, rng.uniform(0.97, 1.0 - 1e-6, n), rng.uniform(0.0, 1.0, n)))
    say(f"[gpu] isovalue of every cell, roots next to extreme vertices: {w.name} seed={seed}")
    phi, U = w.phi_U(0)
    gm, plan = gpu_plan(w.mesh)
    _, g_st, g = gpu_traced_step(plan, gm, a0, phi, U, w.dt)
    om = oracle_lib.OracleMesh(w.mesh)
    _, _, o = om.step(a0, phi, U, w.dt, trace=True)
    _, V = om.geometry()
    assert np.array_equal(g["kind"], o["kind"])
    cp = gm.cell_points()
    rec = np.nonzero(o["kind"] == 1)[0]
    end_intervals = 0
    for c in rec:
        s = np.sort(o["a_pts"][cp[c]])
        end_intervals += int(o["iso"][c] < s[1] or o["iso"][c] > s[6])
        fo = om.cut(c, o["a_pts"], o["iso"][c])["vsub"] / V[c] - a0[c]
        if abs(fo) <= 1e-12:
            err = abs(om.cut(c, o["a_pts"], g["iso"][c])["vsub"] / V[c] - a0[c])
            assert err <= 1e-12, (c, a0[c], g["iso"][c], o["iso"][c], s)
        else:
            assert abs(g["iso"][c] - o["iso"][c]) <= 8 * np.finfo(float).eps, (c, g["iso"][c], o["iso"][c], s)
    say(f"[gpu]   {len(rec)} reconstructed cells, {end_intervals} with the root in the lowest or highest interval")
    assert end_intervals >= 50
