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


def _flips(g, o, eps=1e-8):
    """Cells classified differently (interface cell or not) by the two states: branch flips."""
    return int(np.count_nonzero(((g > eps) & (g < 1 - eps)) != ((o > eps) & (o < 1 - eps))))


def test_violent_3d_full_trajectory(oracle_lib):
    """4.19M-cell graded 3D box, all 100 steps of the workload, each side advancing its own state
    (the benchmark times a window of this run): every cell within 1e-10 of the oracle at every
    tenth step, where the count of cells classified differently (branch flips) is reported too."""
    import torch
    w = W.violent_3d()
    say(f"[gpu] {w.name}: {w.mesh.n_cells} cells x {w.n_steps} steps, oracle on {oracle_lib.get_threads()} threads")
    gm, plan = gpu_plan(w.mesh)
    om = oracle_lib.OracleMesh(w.mesh)
    phi, U = w.phi_U(0)
    tphi, tU = to_dev(phi), to_dev(U)
    a = to_dev(w.alpha0)
    b = torch.empty_like(a)
    o = np.array(w.alpha0, copy=True)
    worst = 0.0
    for n in range(w.n_steps):
        plan.step(a, tphi, tU, w.dt, out=b)
        a, b = b, a
        o, st = om.step(o, phi, U, w.dt)
        if n % 10 == 9:
            g = a.cpu().numpy()
            err = float(np.abs(g - o).max())
            worst = max(worst, err)
            say(f"[gpu]   step {n + 1}: max |gpu - oracle| = {err:.3e}, branch flips {_flips(g, o)}, "
                f"interface cells {st['n_surface']}")
            assert err <= 1e-10, (n + 1, err)
    say(f"[gpu]   worst over the run {worst:.3e}")


def test_airy_ensemble_full_length_sampled_members(oracle_lib):
    """The 64-member Airy ensemble at its full size (5.86M cells) through the batched path the
    benchmark times (one launch per kernel over all members, a captured graph per run of steps),
    all 100 steps with per-step fields generated on the device; the smallest and the largest
    member and three seeded others are stepped by the oracle with the same field values copied
    to the host: every cell within 1e-10 at every twentieth step."""
    import torch
    from paper_1804_01130_amd import Batch, Mesh, default_options
    from wavegen.device import EnsembleAiryFields
    S, chunk = 100, 10
    ws = W.airy_ensemble(64, seed=1, steps=S)
    meshes = [Mesh.from_arrays(w.mesh) for w in ws]
    batch = Batch(meshes, default_options())
    N, F = batch.n_cells, batch.n_faces
    co, fo = batch.layout()
    say(f"[gpu] full-length ensemble: {len(ws)} members, {N} cells, {S} steps")
    ef = EnsembleAiryFields(ws, torch.device("cuda:0"))
    sizes = [w.mesh.n_cells for w in ws]
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes))} | set(
        int(d) for d in np.random.default_rng(5).choice(len(ws), 3, replace=False)))
    oms = {d: oracle_lib.OracleMesh(ws[d].mesh) for d in pick}
    ref = {d: np.array(ws[d].alpha0, copy=True) for d in pick}
    dts = np.array([w.dt for w in ws])
    a = to_dev(batch.concat_cells([w.alpha0 for w in ws]))
    phi = torch.empty((chunk, F), dtype=torch.float64, device=a.device)
    U = torch.empty((chunk, 3 * N), dtype=torch.float64, device=a.device)
    for n0 in range(0, S, chunk):
        for k in range(chunk):
            ef.fields(n0 + k, phi[k], U[k])
        batch.advect(a, phi, U, dts, chunk, phi_stride=F, U_stride=3 * N)
        ph = phi.cpu().numpy()
        uh = U.cpu().numpy()
        for d in pick:
            for k in range(chunk):
                u = np.concatenate([uh[k, j * N + co[d]:j * N + co[d + 1]] for j in range(3)])
                ref[d], _ = oms[d].step(ref[d], ph[k, fo[d]:fo[d + 1]], u, dts[d])
        if (n0 + chunk) % 20 == 0:
            got = batch.split_cells(a.cpu().numpy())
            errs = {d: float(np.abs(got[d] - ref[d]).max()) for d in pick}
            say(f"[gpu]   step {n0 + chunk}: max |gpu - oracle| per sampled member "
                + ", ".join(f"{d}: {e:.2e}" for d, e in errs.items()))
            assert max(errs.values()) <= 1e-10
    batch.close()
