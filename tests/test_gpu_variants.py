"""Variants of the step on the GPU against the oracle: the isoface velocity by cell-point
interpolation (us_mode 1, reading R15) and the time-averaged fields of an outer iteration
(Crank-Nicolson, reading R14; iso_advect_step_avg).  Same seeded inputs on both sides,
|delta alpha| <= 1e-10 after the whole run.
"""
import numpy as np
import pytest

import wavegen as W
from tests.gpuutil import gpu_plan, gpu_traced_step, gpu_trajectory, say, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _cases():
    return {
        "cosine_64x32": W.cosine_uniform(steps=12),
        "airy_128x64": W.airy_slab(128, 64, 32, 0.07, 0.5, 16, "airy_128x64"),
        "violent_32x16x16": W.violent_3d(nx=32, ny=16, nz=16, steps=8),
        "perturbed_10x7x6": W.perturbed_box(steps=8),
    }


CASES = _cases()


def _oracle_run(O, w, steps, opts, averaged=False):
    om = O.OracleMesh(w.mesh)
    a = np.array(w.alpha0, copy=True)
    for n in range(steps):
        phi, U = w.phi_U(n)
        if averaged:
            phi1, U1 = w.phi_U(n + 1)
            phi, U = 0.5 * (phi + phi1), 0.5 * (U + U1)
        a, _ = om.step(a, phi, U, w.dt, opts)
    return a


@pytest.mark.parametrize("name", list(CASES))
def test_interpolated_isoface_velocity(oracle_lib, name):
    w = CASES[name]
    say(f"[gpu] us_mode 1 trajectory: {name} steps={w.n_steps}")
    gm, plan = gpu_plan(w.mesh, us_mode=1)
    g = gpu_trajectory(plan, w, w.n_steps)
    o = _oracle_run(oracle_lib, w, w.n_steps, oracle_lib.default_opts(us_mode=1))
    err = np.abs(g - o).max()
    # the interpolation must matter on these flows (else the test would not see it)
    o0 = _oracle_run(oracle_lib, w, w.n_steps, oracle_lib.default_opts(us_mode=0))
    say(f"[gpu]   max |gpu - oracle| = {err:.3e}; us_mode 1 vs 0 in the oracle: {np.abs(o - o0).max():.3e}")
    assert err <= TOL
    if name != "cosine_64x32":  # uniform flow: U_S = U_P exactly
        assert np.abs(o - o0).max() > 1e-8


@pytest.mark.parametrize("kind,perturb", [("tet", 0.0), ("pyramid", 0.0), ("prism", 0.15), ("mixed", 0.0),
                                          ("merged", 0.1), ("merged_joined", 0.0), ("merged_sparse", 0.1)])
def test_interpolated_isoface_velocity_on_other_cells(oracle_lib, kind, perturb):
    """us_mode 1 on tetrahedra, pyramids, bent prisms, hexahedra next to prisms and general polyhedra
    (mostly polyhedra, one kernel, bent; joined faces of 6 and 8 points; a minority of polyhedra
    beside the eight-lane kernel, bent): every face is fanned about the mean of its points, as in
    the oracle.  (Bent faces of 6 or 8 points give fans that overlap their neighbours', where the
    choice of tetrahedron is discontinuous and rounding can flip it: one step of such a mesh is
    compared in the next test.)"""
    w = W.poly_violent(kind, nx=12, ny=6, nz=6, steps=8, perturb=perturb)
    say(f"[gpu] us_mode 1 trajectory on {kind} (perturb {perturb}): {w.mesh.n_cells} cells, {w.n_steps} steps")
    gm, plan = gpu_plan(w.mesh, us_mode=1)
    g = gpu_trajectory(plan, w, w.n_steps)
    o = _oracle_run(oracle_lib, w, w.n_steps, oracle_lib.default_opts(us_mode=1))
    o0 = _oracle_run(oracle_lib, w, w.n_steps, oracle_lib.default_opts(us_mode=0))
    err = np.abs(g - o).max()
    say(f"[gpu]   max |gpu - oracle| = {err:.3e}; us_mode 1 vs 0 in the oracle: {np.abs(o - o0).max():.3e}")
    assert err <= TOL
    assert np.abs(o - o0).max() > 1e-8


def test_interpolated_isoface_velocity_on_bent_joined_polyhedra(oracle_lib):
    """One step of bent polyhedra with joined faces of 6 and 8 points from the same state: every
    cell's U_S . n_S and the new state against the oracle's."""
    w = W.poly_violent("merged_joined", nx=12, ny=6, nz=6, steps=8, perturb=0.1)
    gm, plan = gpu_plan(w.mesh, us_mode=1)
    phi, U = w.phi_U(0)
    g_new, _, tr = gpu_traced_step(plan, gm, w.alpha0, phi, U, w.dt)
    o_new, _, otr = oracle_lib.OracleMesh(w.mesh).step(w.alpha0, phi, U, w.dt, oracle_lib.default_opts(us_mode=1),
                                                       trace=True)
    rec = (tr["kind"] == 1) & (otr["kind"] == 1)
    assert rec.sum() > 20
    du = np.abs(tr["rec"][rec, 6] - otr["rec"][rec, 6]).max()
    say(f"[gpu] us_mode 1, bent joined polyhedra, one step: max |un gpu - un oracle| = {du:.3e} over "
        f"{rec.sum()} cells, max |alpha gpu - oracle| = {np.abs(g_new - o_new).max():.3e}")
    assert du <= 1e-11 * np.abs(U).max()
    assert np.abs(g_new - o_new).max() <= 1e-13


def test_interpolated_isoface_velocity_in_the_trace(oracle_lib):
    """One step from the same state: the GPU's U_S . n_S per interface cell against the oracle's."""
    w = CASES["violent_32x16x16"]
    gm, plan = gpu_plan(w.mesh, us_mode=1)
    phi, U = w.phi_U(0)
    _, _, tr = gpu_traced_step(plan, gm, w.alpha0, phi, U, w.dt)
    _, _, otr = oracle_lib.OracleMesh(w.mesh).step(w.alpha0, phi, U, w.dt, oracle_lib.default_opts(us_mode=1),
                                                   trace=True)
    rec = (tr["kind"] == 1) & (otr["kind"] == 1)
    assert rec.sum() > 100
    du = np.abs(tr["rec"][rec, 6] - otr["rec"][rec, 6]).max()
    say(f"[gpu]   max |un gpu - un oracle| = {du:.3e} over {rec.sum()} cells")
    assert du <= 1e-11 * np.abs(U).max()


@pytest.mark.parametrize("name,us_mode", [("airy_128x64", 0), ("violent_32x16x16", 0), ("airy_128x64", 1),
                                          ("perturbed_10x7x6", 1)])
def test_averaged_fields(oracle_lib, name, us_mode):
    """iso_advect_step_avg(phi(t), phi(t+dt), U(t), U(t+dt)) is bit for bit the step with the averaged
    fields, and its trajectory matches the oracle fed the averages."""
    import torch
    w = CASES[name]
    steps = min(w.n_steps, 8)
    say(f"[gpu] averaged fields: {name} us_mode={us_mode} steps={steps}")
    gm, plan = gpu_plan(w.mesh, us_mode=us_mode)
    a = to_dev(w.alpha0)
    b = torch.empty_like(a)
    c = torch.empty_like(a)
    for n in range(steps):
        p0, u0 = w.phi_U(n)
        p1, u1 = w.phi_U(n + 1)
        plan.step(a, to_dev(p0), to_dev(u0), w.dt, out=b, phi1=to_dev(p1), U1=to_dev(u1))
        plan.step(a, to_dev(0.5 * (p0 + p1)), to_dev(0.5 * (u0 + u1)), w.dt, out=c)
        torch.cuda.synchronize()
        assert torch.equal(b, c), n
        a, b = b, a
    g = a.cpu().numpy()
    o = _oracle_run(oracle_lib, w, steps, oracle_lib.default_opts(us_mode=us_mode), averaged=True)
    err = np.abs(g - o).max()
    say(f"[gpu]   max |gpu - oracle| = {err:.3e}")
    assert err <= TOL


def test_interpolated_velocity_in_an_ensemble():
    """Ensemble members with us_mode 1 compute bit for bit what each computes alone."""
    import torch
    from paper_1804_01130_amd import Batch, Mesh, Plan, default_options
    ws = [W.airy_slab(64, 32, 16, 0.07, 0.45, 4, "m0"), W.violent_3d(nx=12, ny=8, nz=8, steps=4),
          W.perturbed_box(steps=4)]
    meshes = [Mesh.from_arrays(w.mesh) for w in ws]
    batch = Batch(meshes, default_options(us_mode=1))
    S = 4
    phi = torch.stack([torch.cat([to_dev(w.phi_U(n)[0]) for w in ws]) for n in range(S)]).contiguous()
    U = torch.stack([to_dev(batch.concat_U([w.phi_U(n)[1] for w in ws])) for n in range(S)]).contiguous()
    a = to_dev(batch.concat_cells([w.alpha0 for w in ws]))
    batch.advect(a, phi, U, np.array([w.dt for w in ws]), S, phi_stride=phi.shape[1], U_stride=U.shape[1])
    torch.cuda.synchronize()
    got = batch.split_cells(a.cpu().numpy())
    for d, (w, m) in enumerate(zip(ws, meshes)):
        plan = Plan(m, default_options(us_mode=1))
        x = to_dev(w.alpha0)
        y = torch.empty_like(x)
        for n in range(S):
            p, u = w.phi_U(n)
            plan.step(x, to_dev(p), to_dev(u), w.dt, out=y)
            x, y = y, x
        torch.cuda.synchronize()
        assert np.array_equal(got[d], x.cpu().numpy()), d
        plan.close()


def test_variant_argument_errors():
    import torch
    from paper_1804_01130_amd import IsoError
    w = CASES["airy_128x64"]
    gm, plan = gpu_plan(w.mesh, us_mode=1)
    phi, U = w.phi_U(0)
    a = to_dev(w.alpha0)
    with pytest.raises(IsoError):  # the adjoint follows U_S = U_P only
        plan.adjoint(a, to_dev(phi), to_dev(U), w.dt, torch.ones_like(a))
    with pytest.raises(ValueError):
        plan.step(a, to_dev(phi), to_dev(U), w.dt, phi1=to_dev(phi))
    with pytest.raises(IsoError):
        gpu_plan(w.mesh, us_mode=2)
