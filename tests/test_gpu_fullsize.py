"""Parity at the full sizes of the workloads, in the launch configuration the benchmark times."""
import numpy as np
import pytest

import wavegen as W
from tests.gpuutil import gpu_plan, gpu_trajectory, oracle_trajectory, say, to_dev

pytestmark = pytest.mark.gpu


def test_airy_1024x256_full_trajectory(oracle_lib):
    """Linear Airy wave, 262,144 cells, 200 steps at Courant 0.5, time-varying fluxes: every cell
    within 1e-10 of the oracle after the whole run."""
    w = W.airy_1024x256()
    say(f"[gpu] {w.name}: {w.mesh.n_cells} cells x {w.n_steps} steps")
    gm, plan = gpu_plan(w.mesh)
    g = gpu_trajectory(plan, w, w.n_steps)
    say("[gpu]   oracle trajectory")
    om = oracle_lib.OracleMesh(w.mesh)
    o = oracle_trajectory(om, w, w.n_steps)
    err = np.abs(g - o).max()
    say(f"[gpu]   max |gpu - oracle| = {err:.3e}")
    assert err <= 1e-10
    assert g.min() >= 0.0 and g.max() <= 1.0


def test_violent_3d_full_size_steps(oracle_lib):
    """4.19M-cell graded 3D box: six steps from the initial field on each side; every cell within
    1e-10 of the oracle after the first step and after the sixth."""
    import torch
    w = W.violent_3d()
    say(f"[gpu] {w.name}: {w.mesh.n_cells} cells")
    gm, plan = gpu_plan(w.mesh)
    om = oracle_lib.OracleMesh(w.mesh)
    phi, U = w.phi_U(0)
    tphi, tU = to_dev(phi), to_dev(U)
    a = to_dev(w.alpha0)
    b = torch.empty_like(a)
    o = np.array(w.alpha0, copy=True)
    for n in range(6):
        plan.step(a, tphi, tU, w.dt, out=b)
        a, b = b, a
        o, _ = om.step(o, phi, U, w.dt)
        if n in (0, 5):
            err = np.abs(a.cpu().numpy() - o).max()
            say(f"[gpu]   step {n + 1}: max |gpu - oracle| = {err:.3e}")
            assert err <= 1e-10


def test_airy_ensemble_full_size_sampled_members(oracle_lib):
    """The 64-member Airy ensemble at its full size (5.86M cells) through the batched path the
    benchmark times (one launch per kernel over all members, a captured graph), 4 steps of
    host-generated fields: the smallest and the largest member and three seeded others against
    the oracle, every cell within 1e-10."""
    import torch
    from paper_1804_01130_amd import Batch, Mesh, default_options
    S = 4
    ws = W.airy_ensemble(64, seed=1, steps=S)
    meshes = [Mesh.from_arrays(w.mesh) for w in ws]
    batch = Batch(meshes, default_options())
    say(f"[gpu] full-size ensemble: {len(ws)} members, {batch.n_cells} cells, {S} steps")
    phi = torch.stack([torch.cat([to_dev(w.phi_U(n)[0]) for w in ws]) for n in range(S)]).contiguous()
    U = torch.stack([to_dev(batch.concat_U([w.phi_U(n)[1] for w in ws])) for n in range(S)]).contiguous()
    a = to_dev(batch.concat_cells([w.alpha0 for w in ws]))
    batch.advect(a, phi, U, np.array([w.dt for w in ws]), S, phi_stride=phi.shape[1], U_stride=U.shape[1])
    torch.cuda.synchronize()
    got = batch.split_cells(a.cpu().numpy())
    sizes = [w.mesh.n_cells for w in ws]
    pick = {int(np.argmin(sizes)), int(np.argmax(sizes))} | set(
        int(d) for d in np.random.default_rng(5).choice(len(ws), 3, replace=False))
    for d in sorted(pick):
        w = ws[d]
        ref = oracle_trajectory(oracle_lib.OracleMesh(w.mesh), w, S)
        err = np.abs(got[d] - ref).max()
        say(f"[gpu]   member {d} ({w.name}): max |gpu - oracle| = {err:.3e}")
        assert err <= 1e-10
    batch.close()
