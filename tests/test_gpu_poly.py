"""Cells other than hexahedra on the GPU: tetrahedra, square pyramids, triangular prisms,
hexahedra next to prisms in one mesh, and polyhedra of merged hexahedra (10 or 16 faces, 12 or 18
points, split faces; or the faces two of them share joined into polygons of 6 and 8 points) among
hexahedra, against the oracle.  Same seeded inputs on both sides (the
workloads of wavegen.poly); |delta alpha| <= 1e-10 after the whole run, per-face dV of one traced
step within 1e-13 of max|phi| dt, interface cells the same on both sides.
"""
import numpy as np
import pytest

import wavegen as W
from tests.gpuutil import gpu_plan, gpu_traced_step, say, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _cases():
    return {
        "tet_12x6x6": W.poly_violent("tet", nx=12, ny=6, nz=6, steps=8),
        "prism_16x8x8": W.poly_violent("prism", nx=16, ny=8, nz=8, steps=8),
        "pyramid_8x4x4": W.poly_violent("pyramid", nx=8, ny=4, nz=4, steps=8),
        "mixed_16x8x8": W.poly_violent("mixed", nx=16, ny=8, nz=8, steps=8),
        "airy_prism_64x32": W.poly_airy("prism", 64, 32, steps=12),
        # bent quadrilaterals: those prisms and hexahedra take the generic search
        "prism_perturbed_12x6x6": W.poly_violent("prism", nx=12, ny=6, nz=6, steps=8, perturb=0.15),
        "mixed_perturbed_12x6x6": W.poly_violent("mixed", nx=12, ny=6, nz=6, steps=8, perturb=0.15),
        # general polyhedra: the one-thread-per-cell kernel, flat and bent faces
        "merged_16x8x8": W.poly_violent("merged", nx=16, ny=8, nz=8, steps=8),
        "merged_perturbed_16x8x8": W.poly_violent("merged", nx=16, ny=8, nz=8, steps=8, perturb=0.1),
        # faces of 6 and 8 points: the kernel's general face loops
        "merged_joined_16x8x8": W.poly_violent("merged_joined", nx=16, ny=8, nz=8, steps=8),
        "merged_joined_perturbed_16x8x8": W.poly_violent("merged_joined", nx=16, ny=8, nz=8, steps=8, perturb=0.1),
        # polyhedra a minority: the eight-lane kernel and the polyhedron kernel side by side (two
        # streams); the meshes above are mostly polyhedra, whose plans send every cell to the latter
        "merged_sparse_16x8x8": W.poly_violent("merged_sparse", nx=16, ny=8, nz=8, steps=8),
        "merged_sparse_perturbed_16x8x8": W.poly_violent("merged_sparse", nx=16, ny=8, nz=8, steps=8, perturb=0.1),
    }


CASES = _cases()


def _gpu_run(plan, w, steps, alpha0=None):
    import torch
    a = to_dev(w.alpha0 if alpha0 is None else alpha0)
    b = torch.empty_like(a)
    phi, U = w.phi_U(0)
    tphi, tU = to_dev(phi), to_dev(U)
    for _ in range(steps):
        plan.step(a, tphi, tU, w.dt, out=b)
        a, b = b, a
    torch.cuda.synchronize()
    return a.cpu().numpy()


def _oracle_run(om, w, steps, alpha0=None):
    phi, U = w.phi_U(0)
    return om.run(np.array(w.alpha0 if alpha0 is None else alpha0, copy=True), phi, U, w.dt, steps)


@pytest.mark.parametrize("name", list(CASES))
def test_trajectory_matches_oracle(oracle_lib, name):
    w = CASES[name]
    say(f"[gpu] cells with triangular faces, trajectory: {name} cells={w.mesh.n_cells} steps={w.n_steps}")
    gm, plan = gpu_plan(w.mesh)
    g = _gpu_run(plan, w, w.n_steps)
    o = _oracle_run(oracle_lib.OracleMesh(w.mesh), w, w.n_steps)
    err = np.abs(g - o).max()
    say(f"[gpu]   max |gpu - oracle| = {err:.3e}")
    assert err <= TOL
    assert g.min() >= 0.0 and g.max() <= 1.0


@pytest.mark.parametrize("name", ["tet_12x6x6", "pyramid_8x4x4", "mixed_16x8x8", "merged_16x8x8",
                                  "merged_perturbed_16x8x8", "merged_joined_16x8x8",
                                  "merged_joined_perturbed_16x8x8", "merged_sparse_16x8x8"])
def test_traced_step_matches_oracle(oracle_lib, name):
    w = CASES[name]
    phi, U = w.phi_U(0)
    say(f"[gpu] cells with triangular faces, one traced step: {name}")
    gm, plan = gpu_plan(w.mesh)
    out, st, tr = gpu_traced_step(plan, gm, w.alpha0, phi, U, w.dt)
    o_new, o_st, otr = oracle_lib.OracleMesh(w.mesh).step(w.alpha0, phi, U, w.dt, trace=True)
    assert st["n_surface"] == o_st["n_surface"] and st["n_surface"] > 20
    assert np.array_equal(tr["kind"] == 1, otr["kind"] == 1)
    flux_faces = ~np.isnan(tr["dV"])  # the trace leaves faces that carry no flux untouched
    assert flux_faces[:w.mesh.n_internal].all()
    ddv = np.abs(tr["dV"][flux_faces] - otr["dV"][flux_faces]).max()
    say(f"[gpu]   interface cells {st['n_surface']}; max |d dV| = {ddv:.3e}; max |d alpha| = "
        f"{np.abs(out - o_new).max():.3e}")
    assert ddv <= 1e-13 * np.abs(phi).max() * w.dt
    assert np.abs(out - o_new).max() <= 1e-13


@pytest.mark.parametrize("kind,seed,perturb", [("tet", 61, 0.0), ("tet", 62, 0.0), ("merged", 63, 0.0),
                                               ("merged", 64, 0.0), ("merged_joined", 65, 0.0),
                                               ("merged_joined", 66, 0.1), ("merged_sparse", 67, 0.1)])
def test_random_fields(oracle_lib, kind, seed, perturb):
    """alpha ~ U[0.02, 0.98] per cell: every cell an interface cell, arbitrary vertex patterns on
    triangular faces and on the many faces of the merged polyhedra, flat or bent."""
    w = W.poly_violent(kind, nx=8, ny=4, nz=4, steps=3, perturb=perturb)
    a0 = np.random.default_rng(seed).uniform(0.02, 0.98, w.mesh.n_cells)
    say(f"[gpu] random field on {kind} cells: seed={seed}")
    gm, plan = gpu_plan(w.mesh)
    g = _gpu_run(plan, w, 3, a0)
    o = _oracle_run(oracle_lib.OracleMesh(w.mesh), w, 3, a0)
    err = np.abs(g - o).max()
    say(f"[gpu]   max |gpu - oracle| = {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("name", ["mixed_16x8x8", "merged_16x8x8", "merged_joined_16x8x8", "merged_sparse_16x8x8"])
def test_launch_shapes_give_the_same_bits(name):
    w = CASES[name]
    ref = None
    for opts in ({}, {"block_cells": 64}, {"surface_waves": 1}, {"surface_blocks": 7, "bound_blocks": 3}):
        gm, plan = gpu_plan(w.mesh, **opts)
        g = _gpu_run(plan, w, 4)
        if ref is None:
            ref = g
        assert np.array_equal(g, ref), opts


@pytest.mark.parametrize("name", ["mixed_16x8x8", "merged_16x8x8", "merged_joined_perturbed_16x8x8",
                                  "merged_sparse_16x8x8"])
def test_capped_searches_are_counted_once_per_cell(name):
    """With root_max_iter too small for the isovalue searches to finish, n_nonconverged counts each
    capped cell once, in the eight-lane kernel and in the sixteen-lane polyhedron kernel alike: at
    least one, and no more than the reconstructed cells whose trace shows the cap reached."""
    w = CASES[name]
    phi, U = w.phi_U(0)
    cap = 4
    gm, plan = gpu_plan(w.mesh, root_max_iter=cap)
    _, st, tr = gpu_traced_step(plan, gm, w.alpha0, phi, U, w.dt)
    capped = int(np.count_nonzero((tr["kind"] == 1) & (tr["iters"] >= cap)))
    say(f"[gpu] root_max_iter {cap}: {name}: not converged {st['n_nonconverged']}, cells at the cap {capped}, "
        f"interface cells {st['n_surface']}")
    assert 1 <= st["n_nonconverged"] <= capped


def test_ghost_fluid_faces_and_relaxation_on_prisms(oracle_lib):
    """The face and cell kernels after the step need no hexahedra: ghost-fluid face data and the
    relaxation blend on the prism mesh against the oracle."""
    import torch
    w = CASES["prism_16x8x8"]
    om = oracle_lib.OracleMesh(w.mesh)
    xc = om.geometry()[0]
    phi, U = w.phi_U(0)
    a, _ = om.step(w.alpha0, phi, U, w.dt)
    g = (0.0, 0.0, -9.81)
    p = W.dynamic_pressure(xc, a, 1000.0, 1.2, g, (0.0, 0.0, 0.5), seed=71)
    gm, plan = gpu_plan(w.mesh)
    got = plan.gfm_faces(to_dev(a), to_dev(p), 1000.0, 1.2, g)
    torch.cuda.synchronize()
    exp = om.gfm_faces(a, p, 1000.0, 1.2, np.array(g))
    assert np.array_equal(got["lambda"].cpu().numpy(), exp["lambda"])
    assert np.abs(got["ghost_nbr"].cpu().numpy() - exp["ghost_nbr"]).max() <= 1e-13 * 1e4 * 1e3
    zones = [((0.3003, 0.0, 0.0), (-1.0, 0.0, 0.0), 0.3)]
    plan.set_relaxation(zones)
    x = to_dev(a)
    plan.relax_blend(x, to_dev(w.alpha0))
    torch.cuda.synchronize()
    assert np.abs(x.cpu().numpy() - om.relax_blend(zones, a, w.alpha0)).max() <= 1e-13


def _merged_pair(xs, ys, zs, **kw):
    """2 x 2 x 1 hexahedra merged along x into two cells of 12 points that share one face of 6
    points; every other face on the boundary."""
    xs, ys = [xs[0], 0.5 * (xs[0] + xs[1]), xs[1]], [ys[0], 0.5 * (ys[0] + ys[1]), ys[1]]
    return W.merged_block(xs, ys, zs, merge_x=[(0, 0, 0), (0, 1, 0)], join=True, **kw)


def _merged_one(xs, ys, zs, **kw):
    """2 x 2 x 1 hexahedra merged into one cell of 18 points and 16 faces, all on the boundary."""
    xs, ys = [xs[0], 0.5 * (xs[0] + xs[1]), xs[1]], [ys[0], 0.5 * (ys[0] + ys[1]), ys[1]]
    return W.merged_block(xs, ys, zs, merge_xy=[(0, 0, 0)], **kw)


@pytest.mark.parametrize("build", ["tet", "pyramid", "prism", "merged_pair", "merged_one"])
def test_one_block_of_cells(oracle_lib, build):
    """The smallest meshes: one hexahedron's worth of tetrahedra, pyramids or prisms (6, 6 and 2
    cells), two polyhedra sharing one joined face, or one polyhedron alone; every cell touches the
    boundary; a steep field and a uniform flow, 4 steps."""
    b = {"tet": W.tet_block, "pyramid": W.pyramid_block, "prism": W.prism_block, "merged_pair": _merged_pair,
         "merged_one": _merged_one}[build]
    mesh = b([0.0, 1.0], [0.0, 1.0], [0.0, 1.0], kinds={"xmin": W.PATCH_INOUT, "xmax": W.PATCH_INOUT},
             periodic_x=False)
    om = oracle_lib.OracleMesh(mesh)
    xc, V = om.geometry()
    a0 = np.clip(0.5 + 1.5 * (0.45 - xc[:, 2] + 0.3 * (xc[:, 0] - 0.5) + 0.4 * (xc[:, 1] - 0.5)), 0.0, 1.0)
    phi = W.fluxes_from_potential(mesh, lambda x, y, z: 0.3 * y * np.ones_like(z))
    U = np.concatenate([np.full(mesh.n_cells, 0.3), np.zeros(mesh.n_cells), np.zeros(mesh.n_cells)])
    dt = 0.2
    gm, plan = gpu_plan(mesh)
    import torch
    a = to_dev(a0)
    bb = torch.empty_like(a)
    o = a0.copy()
    for _ in range(4):
        plan.step(a, to_dev(phi), to_dev(U), dt, out=bb)
        a, bb = bb, a
        o, _ = om.step(o, phi, U, dt)
    torch.cuda.synchronize()
    err = np.abs(a.cpu().numpy() - o).max()
    say(f"[gpu] one block of {build} cells: max |gpu - oracle| = {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("name", ["prism_16x8x8", "merged_16x8x8", "merged_joined_perturbed_16x8x8",
                                  "merged_sparse_16x8x8"])
def test_averaged_fields_on_other_cells(oracle_lib, name):
    """The step with a second time level of the fields (phi1 = 0.7 phi, U1 = 0.7 U + a seeded
    perturbation) is bit for bit the step with the averaged fields, on the eight-lane and the
    polyhedron kernels, and its trajectory matches the oracle fed the averages."""
    import torch
    w = CASES[name]
    phi, U = w.phi_U(0)
    phi1 = 0.7 * phi
    U1 = 0.7 * U + np.random.default_rng(81).uniform(-0.05, 0.05, U.shape)
    say(f"[gpu] averaged fields on {name}")
    gm, plan = gpu_plan(w.mesh)
    a = to_dev(w.alpha0)
    b, c = torch.empty_like(a), torch.empty_like(a)
    tp, tu, tp1, tu1 = to_dev(phi), to_dev(U), to_dev(phi1), to_dev(U1)
    tpa, tua = to_dev(0.5 * (phi + phi1)), to_dev(0.5 * (U + U1))
    for n in range(6):
        plan.step(a, tp, tu, w.dt, out=b, phi1=tp1, U1=tu1)
        plan.step(a, tpa, tua, w.dt, out=c)
        torch.cuda.synchronize()
        assert torch.equal(b, c), n
        a, b = b, a
    om = oracle_lib.OracleMesh(w.mesh)
    o = om.run(np.array(w.alpha0, copy=True), 0.5 * (phi + phi1), 0.5 * (U + U1), w.dt, 6)
    err = np.abs(a.cpu().numpy() - o).max()
    say(f"[gpu]   max |gpu - oracle| = {err:.3e}")
    assert err <= TOL


@pytest.mark.parametrize("kind", ["merged", "merged_joined"])
def test_polyhedra_at_the_bench_size(oracle_lib, kind):
    """The polyhedral bench meshes themselves (64x32x32 hexahedra, mostly merged: 26,112 cells),
    in the launch configuration the bench times: 4 steps, every cell against the oracle."""
    w = W.poly_violent(kind, nx=64, ny=32, nz=32, steps=4)
    say(f"[gpu] polyhedra at the bench size: {w.name} cells={w.mesh.n_cells}")
    gm, plan = gpu_plan(w.mesh)
    g = _gpu_run(plan, w, 4)
    o = _oracle_run(oracle_lib.OracleMesh(w.mesh), w, 4)
    err = np.abs(g - o).max()
    say(f"[gpu]   max |gpu - oracle| = {err:.3e}")
    assert err <= TOL
