"""The step for callers that cannot allocate (iso_advect_step_noalloc) against the plan's step
(iso_advect_step): the same kernels, so the same bits, on consecutive calls that share the
library's fixed workspace, the second with a smaller mesh."""
import numpy as np
import pytest

import wavegen as W
from tests.gpuutil import say, to_dev

pytestmark = pytest.mark.gpu


def _both(w, steps, **opts):
    """alpha after each of `steps` steps through the plan and through the no-allocation entry."""
    import torch
    from paper_1804_01130_amd import Mesh, Plan, default_options
    from paper_1804_01130_amd.binding import advect_step_noalloc
    gm = Mesh.from_arrays(w.mesh)
    o = default_options(**opts)
    plan = Plan(gm, o)
    a = to_dev(w.alpha0)
    b = to_dev(w.alpha0)
    ref, got = [], []
    for n in range(steps):
        phi, U = w.phi_U(n)
        tphi, tU = to_dev(phi), to_dev(U)
        a, _ = plan.step(a, tphi, tU, w.dt)
        b = advect_step_noalloc(gm, b, tphi, tU, w.dt, torch.empty_like(b), options=o)
        torch.cuda.synchronize()
        ref.append(a.cpu().numpy())
        got.append(b.cpu().numpy())
    plan.close()
    return ref, got


def test_no_alloc_step_matches_the_plan_step_bit_for_bit():
    cases = [(W.violent_3d(nx=24, ny=13, nz=16, steps=6), 6, {}),          # 3D, bounding active
             (W.airy_slab(128, 64, 32, 0.08, 0.5, 6, "airy_128x64"), 6, {}),
             (W.cosine_uniform(nx=32, ny=16, steps=4), 4, {"n_bound_iter": 1, "clip": 0})]
    for w, steps, opts in cases:  # each call after the first reuses the workspace at a smaller size
        say(f"[gpu] no-allocation step vs plan step: {w.name} ({w.mesh.n_cells} cells, {steps} steps, {opts})")
        ref, got = _both(w, steps, **opts)
        for n in range(steps):
            assert np.array_equal(ref[n], got[n]), (w.name, n, np.abs(ref[n] - got[n]).max())
        assert not np.array_equal(ref[0], w.alpha0)


def test_no_alloc_step_on_cells_other_than_hexahedra():
    # polyhedra among hexahedra: the plan runs the polyhedron kernel on its side stream, this entry
    # on the caller's stream; then polyhedra only, then tetrahedra and pyramids, each mesh smaller
    cases = [W.poly_violent("merged_sparse", nx=16, ny=8, nz=8, steps=4, perturb=0.1),
             W.poly_violent("merged_joined", nx=12, ny=6, nz=6, steps=4, perturb=0.1),
             W.poly_violent("mixed", nx=12, ny=6, nz=6, steps=4),
             W.poly_violent("tet", nx=8, ny=4, nz=4, steps=4)]
    for w in cases:
        say(f"[gpu] no-allocation step vs plan step: {w.name} ({w.mesh.n_cells} cells, 4 steps)")
        ref, got = _both(w, 4)
        for n in range(4):
            assert np.array_equal(ref[n], got[n]), (w.name, n, np.abs(ref[n] - got[n]).max())
        assert not np.array_equal(ref[0], w.alpha0)


def test_no_alloc_step_refuses_what_it_cannot_hold():
    import torch
    from paper_1804_01130_amd import IsoError, Mesh, default_options
    from paper_1804_01130_amd.binding import ISO_EINVAL, ISO_ENOSPACE, advect_step_noalloc
    w = W.violent_3d(nx=128, ny=64, nz=64, steps=1)  # 524k cells, 1.6M faces: ~107 MB of workspace
    say(f"[gpu] no-allocation step beyond its workspace: {w.mesh.n_cells} cells")
    gm = Mesh.from_arrays(w.mesh)
    phi, U = w.phi_U(0)
    a = to_dev(w.alpha0)
    with pytest.raises(IsoError) as e:
        advect_step_noalloc(gm, a, to_dev(phi), to_dev(U), w.dt, torch.empty_like(a))
    assert e.value.status == ISO_ENOSPACE
    small = W.cosine_uniform(nx=8, ny=4, steps=1)
    sm = Mesh.from_arrays(small.mesh)
    p, u = (to_dev(x) for x in small.phi_U(0))
    b = to_dev(small.alpha0)
    with pytest.raises(IsoError) as e:
        advect_step_noalloc(sm, b, p, u, small.dt, b)  # output aliases the input
    assert e.value.status == ISO_EINVAL
    with pytest.raises(IsoError) as e:
        advect_step_noalloc(sm, b, p, u, small.dt, torch.empty_like(b), options=default_options(check_inputs=1))
    assert e.value.status == ISO_EINVAL
