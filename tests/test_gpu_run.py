"""Multi-step runs of one mesh (iso_plan_run): the same bits as the same number of single steps;
the captured graph replayed with other device work in between and checked against the single
steps each time; steady and per-step fields; polyhedra among hexahedra (whose kernel runs on the
plan's side stream inside the capture); and the argument checks."""
import numpy as np
import pytest

import wavegen as W
from tests.gpuutil import gpu_plan, say, to_dev

pytestmark = pytest.mark.gpu


def _single_steps(plan, a0, dt, steps, fields):
    import torch
    a = a0.clone()
    b = torch.empty_like(a)
    for n in range(steps):
        p, u = fields(n)
        plan.step(a, p, u, dt, out=b)
        a, b = b, a
    torch.cuda.synchronize()
    return a.cpu().numpy()


@pytest.mark.parametrize("name,steps", [("violent", 5), ("violent", 6), ("merged_sparse", 5)])
def test_run_matches_single_steps(name, steps):
    import torch
    w = (W.violent_3d(nx=24, ny=13, nz=16, steps=steps) if name == "violent" else
         W.poly_violent("merged_sparse", nx=16, ny=8, nz=8, steps=steps, perturb=0.1))
    say(f"[gpu] run of {steps} steps vs single steps: {w.name} ({w.mesh.n_cells} cells)")
    gm, plan = gpu_plan(w.mesh)
    phi, U = (to_dev(x) for x in w.phi_U(0))
    a0 = to_dev(w.alpha0)
    ref = _single_steps(plan, a0, w.dt, steps, lambda n: (phi, U))
    assert not np.array_equal(ref, w.alpha0)
    a = a0.clone()
    other = torch.ones(1 << 20, dtype=torch.float64, device=a.device)
    for rep in range(3):  # the capture, then two replays with other work in between
        a.copy_(a0)
        plan.run(a, phi, U, w.dt, steps)
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), ref), rep
        other.mul_(1.5).add_(1.0)
        torch.cuda.synchronize()
    plan.close()


def test_run_with_per_step_fields():
    import torch
    steps = 7
    w = W.airy_slab(128, 64, 32, 0.08, 0.5, steps, "airy_128x64")
    say(f"[gpu] run with per-step fields: {w.name}")
    gm, plan = gpu_plan(w.mesh)
    phis = torch.stack([to_dev(w.phi_U(n)[0]) for n in range(steps)]).contiguous()
    Us = torch.stack([to_dev(w.phi_U(n)[1]) for n in range(steps)]).contiguous()
    a0 = to_dev(w.alpha0)
    ref = _single_steps(plan, a0, w.dt, steps, lambda n: (phis[n], Us[n]))
    a = a0.clone()
    plan.run(a, phis, Us, w.dt, steps, phi_stride=phis.shape[1], U_stride=Us.shape[1])
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy(), ref)
    # a different step count is captured again
    a.copy_(a0)
    plan.run(a, phis, Us, w.dt, 3, phi_stride=phis.shape[1], U_stride=Us.shape[1])
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy(), _single_steps(plan, a0, w.dt, 3, lambda n: (phis[n], Us[n])))
    plan.close()


def test_long_run_is_launched_step_by_step():
    """More than 256 steps are not captured: the run launches them one by one, with the same bits."""
    import torch
    steps = 300
    w = W.cosine_uniform(nx=32, ny=16, steps=steps)
    say(f"[gpu] run of {steps} steps (no capture): {w.name}")
    gm, plan = gpu_plan(w.mesh)
    phi, U = (to_dev(x) for x in w.phi_U(0))
    a0 = to_dev(w.alpha0)
    ref = _single_steps(plan, a0, w.dt, steps, lambda n: (phi, U))
    a = a0.clone()
    plan.run(a, phi, U, w.dt, steps)
    torch.cuda.synchronize()
    assert np.array_equal(a.cpu().numpy(), ref)
    assert not np.array_equal(ref, w.alpha0)
    plan.close()


def test_run_argument_errors():
    import torch
    from paper_1804_01130_amd import IsoError
    from paper_1804_01130_amd.binding import ISO_EINVAL, ISO_EUNSUPPORTED
    w = W.cosine_uniform(nx=16, ny=8, steps=2)
    gm, plan = gpu_plan(w.mesh)
    phi, U = (to_dev(x) for x in w.phi_U(0))
    a = to_dev(w.alpha0)
    with pytest.raises(IsoError) as e:
        plan.run(a, phi, U, w.dt, -1)
    assert e.value.status == ISO_EINVAL
    two = torch.cat([phi, phi])  # room for the binding's size check; the stride is still too short
    with pytest.raises(IsoError) as e:
        plan.run(a, two, U, w.dt, 2, phi_stride=1)
    assert e.value.status == ISO_EINVAL
    with pytest.raises(ValueError):  # fields shorter than the steps read: refused before the call
        plan.run(a, phi, U, w.dt, 2, phi_stride=gm.n_faces)
    with pytest.raises(IsoError) as e:
        plan.run(a, phi, U, -w.dt, 2)
    assert e.value.status == ISO_EINVAL
    big = torch.zeros(max(gm.n_cells, gm.n_faces), dtype=torch.float64, device=a.device)
    with pytest.raises(IsoError) as e:  # the state inside the fields
        plan.run(big[:gm.n_cells], big[:gm.n_faces], U, w.dt, 2)
    assert e.value.status == ISO_EINVAL
    plan.close()
    _, small = gpu_plan(w.mesh, max_surface=8)
    with pytest.raises(IsoError) as e:
        small.run(a, phi, U, w.dt, 2)
    assert e.value.status == ISO_EUNSUPPORTED
    small.close()
    _, checked = gpu_plan(w.mesh, check_inputs=1)
    with pytest.raises(IsoError) as e:
        checked.run(a, phi, U, w.dt, 2)
    assert e.value.status == ISO_EINVAL
    checked.close()
