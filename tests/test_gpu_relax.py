"""Relaxation-zone blending (reading R17) on the GPU against the oracle, through the C interface
(iso_plan_set_relaxation, iso_relax_blend).  Same seeded inputs on both sides: volume fractions
from the workload generators and from the oracle's own steps; the target is the workload's initial
field (a stand-in for the incident wave's).

The weights are computed on the host by both sides with the same operations in the same order;
they can differ only through the cell centroids, which each side sums in its own order (a few
ulps), and the blend is rounded operation by operation on both sides.  Bar: |d alpha| <= 1e-13 per
blend, and 1e-10 over a trajectory of steps and blends.  No zone edge passes within 1e-9 of a
cell centre in these cases, so both sides find the same zone cells.
"""
import numpy as np
import pytest

import wavegen as W
from tests.gpuutil import gpu_plan, say, to_dev

pytestmark = pytest.mark.gpu


def _chi_ok(xc, zones):
    """Zone cells by the definition (numpy), and the distance of the nearest centre to an edge."""
    inside = np.zeros(len(xc), dtype=bool)
    margin = np.inf
    for o, d, ln in zones:
        e = np.asarray(d, float) / np.linalg.norm(d)
        q = (xc - np.asarray(o, float)) @ e / ln
        inside |= (q >= 0) & (q <= 1)
        margin = min(margin, np.abs(q).min() * ln, np.abs(q - 1).min() * ln)
    return inside, margin


def _gpu_blend(plan, a, t):
    import torch
    x = to_dev(a)
    plan.relax_blend(x, to_dev(t))
    torch.cuda.synchronize()
    return x.cpu().numpy()


CASES = {
    "airy_128x64": (lambda: W.airy_slab(128, 64, 32, 0.07, 0.5, 8, "airy_128x64"),
                    [((0.61, 0.0, 0.0), (-1.0, 0.0, 0.0), 0.6), ((3.37, 0.0, 0.0), (1.0, 0.0, 0.0), 0.55)]),
    "violent_32x16x16_oblique": (lambda: W.violent_3d(nx=32, ny=16, nz=16, steps=4),
                                 [((0.41, 0.2, 0.0), (-1.0, -0.3, 0.0), 0.4), ((1.63, 0.5, 0.5), (1.0, 0.2, 0.1), 0.33)]),
    "perturbed_10x7x6": (lambda: W.perturbed_box(steps=4), [((0.33, 0.0, 0.0), (-1.0, 0.0, 0.0), 0.5)]),
}


@pytest.mark.parametrize("name", list(CASES))
def test_relax_blend_matches_oracle(oracle_lib, name):
    make, zones = CASES[name]
    w = make()
    om = oracle_lib.OracleMesh(w.mesh)
    xc = om.geometry()[0]
    inside, margin = _chi_ok(xc, zones)
    assert margin > 1e-9 and inside.sum() > 10
    phi, U = w.phi_U(0)
    a, _ = om.step(w.alpha0, phi, U, w.dt)
    a, _ = om.step(a, phi, U, w.dt)
    say(f"[gpu] relaxation blend: {name} cells={w.mesh.n_cells} zone cells={inside.sum()}")
    gm, plan = gpu_plan(w.mesh)
    assert plan.set_relaxation(zones) == inside.sum()
    got = _gpu_blend(plan, a, w.alpha0)
    exp = om.relax_blend(zones, a, w.alpha0)
    err = np.abs(got - exp).max()
    say(f"[gpu]   max |gpu - oracle| = {err:.3e}; bit for bit: {np.array_equal(got, exp)}")
    assert err <= 1e-13
    assert np.array_equal(got[~inside], a[~inside])


def test_advect_then_blend_trajectory(oracle_lib):
    """The paper's order within a time step: the advection step, then the blend; 16 steps on each
    side."""
    import torch
    w = W.airy_slab(128, 64, 32, 0.07, 0.5, 16, "airy_128x64")
    zones = CASES["airy_128x64"][1]
    gm, plan = gpu_plan(w.mesh)
    plan.set_relaxation(zones)
    om = oracle_lib.OracleMesh(w.mesh)
    tgt = to_dev(w.alpha0)
    a = to_dev(w.alpha0)
    b = torch.empty_like(a)
    o = np.array(w.alpha0, copy=True)
    for n in range(w.n_steps):
        phi, U = w.phi_U(n)
        plan.step(a, to_dev(phi), to_dev(U), w.dt, out=b)
        plan.relax_blend(b, tgt)
        a, b = b, a
        o, _ = om.step(o, phi, U, w.dt)
        o = om.relax_blend(zones, o, w.alpha0)
    torch.cuda.synchronize()
    err = np.abs(a.cpu().numpy() - o).max()
    say(f"[gpu] advect + blend, {w.n_steps} steps: max |gpu - oracle| = {err:.3e}")
    assert err <= 1e-10


def test_relax_full_size(oracle_lib):
    """The graded 3D box at full size with zones 0.3 long at both ends of x (30 % of the cells)."""
    w = W.violent_3d()
    zones = [((0.3003, 0.0, 0.0), (-1.0, 0.0, 0.0), 0.3), ((1.6997, 0.0, 0.0), (1.0, 0.0, 0.0), 0.3)]
    om = oracle_lib.OracleMesh(w.mesh)
    xc = om.geometry()[0]
    inside, margin = _chi_ok(xc, zones)
    assert margin > 1e-9
    phi, U = w.phi_U(0)
    a, _ = om.step(w.alpha0, phi, U, w.dt)
    say(f"[gpu] relaxation blend at full size: {w.mesh.n_cells} cells, {inside.sum()} in zones")
    gm, plan = gpu_plan(w.mesh)
    assert plan.set_relaxation(zones) == inside.sum()
    got = _gpu_blend(plan, a, w.alpha0)
    exp = om.relax_blend(zones, a, w.alpha0)
    err = np.abs(got - exp).max()
    say(f"[gpu]   max |gpu - oracle| = {err:.3e}")
    assert err <= 1e-13


def test_relax_edge_cases_and_errors():
    import torch
    from paper_1804_01130_amd import IsoError
    w = W.violent_3d(nx=8, ny=6, nz=6, steps=1)
    gm, plan = gpu_plan(w.mesh)
    a = to_dev(w.alpha0)
    t = torch.zeros_like(a)
    ref = a.clone()
    plan.relax_blend(a, t)  # no zones: nothing happens
    assert plan.set_relaxation([((5.0, 0, 0), (1, 0, 0), 1.0)]) == 0  # a zone outside the mesh
    plan.relax_blend(a, t)
    torch.cuda.synchronize()
    assert torch.equal(a, ref)
    with pytest.raises(IsoError):
        plan.set_relaxation([((0, 0, 0), (0, 0, 0), 1.0)])
    with pytest.raises(IsoError):
        plan.set_relaxation([((0, 0, 0), (1, 0, 0), -1.0)])
    with pytest.raises(IsoError):  # overlapping zones
        plan.set_relaxation([((0, 0, 0), (1, 0, 0), 1.0), ((1.5, 0, 0), (-1, 0, 0), 1.0)])
    n = plan.set_relaxation([((0.5, 0, 0), (-1, 0, 0), 0.5)])
    assert n > 0
    with pytest.raises(IsoError):  # alpha and target overlap
        plan.relax_blend(a, a)
    plan.set_relaxation([])  # cleared
    plan.relax_blend(a, t)
    torch.cuda.synchronize()
    assert torch.equal(a, ref)
