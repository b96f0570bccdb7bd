"""The adjoint step (iso_advect_step_adjoint) and the checkpointed multi-step gradient on the GPU.

One step: every component of alpha_bar and phi_bar against the oracle's gradient, each component
of which is one exact tangent (complex step) of the oracle's step.  One step of the 256x128 Airy
case: the dot-product identity <alpha_bar, da> + <phi_bar, dphi> = <alpha_new_bar, tangent(da, dphi)>
against the oracle tangent.  Fifty steps: the gradient of a misfit loss through checkpoints against
central differences of the GPU forward along directions that stay clear of topology changes
(interior-cell alpha, divergence-free fluxes), at 1e-6 relative.
"""
import numpy as np
import pytest

import wavegen as W
from tests.gpuutil import gpu_plan, gpu_traced_step, say, to_dev

pytestmark = pytest.mark.gpu


def _adjoint(plan, w, alpha, phi, U, abar_new):
    import torch
    ab, pb = plan.adjoint(to_dev(alpha), to_dev(phi), to_dev(U), w.dt, to_dev(abar_new))
    torch.cuda.synchronize()
    return ab.cpu().numpy(), pb.cpu().numpy()


def _state_after(O, w, steps):
    om = O.OracleMesh(w.mesh)
    a = np.array(w.alpha0, copy=True)
    for n in range(steps):
        phi, U = w.phi_U(n)
        a, _ = om.step(a, phi, U, w.dt)
    return a


@pytest.mark.parametrize("name", ["airy_16x8", "cosine_16x8", "violent_6x5x4", "perturbed_5x4x4"])
def test_one_step_adjoint_matches_oracle_gradient(oracle_lib, name):
    O = oracle_lib
    w = {"airy_16x8": lambda: W.airy_slab(16, 8, 8, 0.09, 0.5, 4, name),
         "cosine_16x8": lambda: W.cosine_uniform(nx=16, ny=8, steps=4, co=0.5),
         "violent_6x5x4": lambda: W.violent_3d(nx=6, ny=5, nz=4, steps=4),
         "perturbed_5x4x4": lambda: W.perturbed_box(nx=5, ny=4, nz=4, steps=4)}[name]()
    say(f"[gpu] one-step adjoint vs oracle gradient: {name} cells={w.mesh.n_cells}")
    a = _state_after(O, w, 2)  # a state with some history (bounding active in places)
    phi, U = w.phi_U(2)
    rng = np.random.default_rng(3)
    abar_new = rng.standard_normal(w.mesh.n_cells)
    gm, plan = gpu_plan(w.mesh)
    ga, gp = _adjoint(plan, w, a, phi, U, abar_new)
    om = O.OracleMesh(w.mesh)
    oa, op = om.gradient(a, phi, U, w.dt, abar_new)
    scale_a = max(np.abs(oa).max(), 1e-300)
    scale_p = max(np.abs(op).max(), 1e-300)
    assert np.abs(ga - oa).max() <= 1e-9 * scale_a, (np.argmax(np.abs(ga - oa)), np.abs(ga - oa).max(), scale_a)
    assert np.abs(gp - op).max() <= 1e-9 * scale_p, (np.argmax(np.abs(gp - op)), np.abs(gp - op).max(), scale_p)


@pytest.mark.parametrize("n_iter,clip", [(0, True), (0, False), (1, True), (2, False), (3, True), (5, True)])
def test_adjoint_through_every_bounding_schedule(oracle_lib, n_iter, clip):
    """The bounding adjoint (tape replay, then reversed sweeps, grid-wide) against the oracle's
    gradient with the same options: no sweep (the final clip alone, or nothing), one sweep, several,
    and more sweeps than the three rotating correction buffers; on a state where cells are out of
    bounds after the update, through two calls in a row on one plan (its buffers must come back
    clean)."""
    O = oracle_lib
    w = W.violent_3d(nx=8, ny=6, nz=6, steps=6)
    opts = dict(n_bound_iter=n_iter, clip=clip)
    a = _state_after(O, w, 3)
    phi, U = w.phi_U(3)
    om = O.OracleMesh(w.mesh)
    _, st = om.step(a, phi, U, w.dt, opts=O.default_opts(**opts))
    say(f"[gpu] adjoint through bounding: sweeps={n_iter} clip={clip} cells out of bounds {st['n_bound_active']}")
    assert st["n_bound_active"] > 0
    gm, plan = gpu_plan(w.mesh, **opts)
    # the oracle's Jacobian, one exact tangent per input component, then two adjoint seeds
    n, nf = w.mesh.n_cells, w.mesh.n_faces
    oo = O.default_opts(**opts)
    ja = np.array([om.step_tlm(a, phi, U, w.dt, dalpha=np.eye(1, n, k)[0], opts=oo)[1] for k in range(n)])
    jp = np.array([om.step_tlm(a, phi, U, w.dt, dphi=np.eye(1, nf, f)[0], opts=oo)[1] for f in range(nf)])
    seeds = [np.ones(n), np.random.default_rng(11).standard_normal(n)]
    for bar in seeds:
        ra, rp = ja @ bar, jp @ bar
        ga, gp = _adjoint(plan, w, a, phi, U, bar)
        # relative to the sum of the magnitudes the products add up (with the seed of ones and no
        # clip, the flux gradient of the conserved total is zero up to round-off)
        sa = max((np.abs(ja) @ np.abs(bar)).max(), 1e-300)
        sp = max((np.abs(jp) @ np.abs(bar)).max(), 1e-300)
        assert np.abs(ga - ra).max() <= 1e-9 * sa, (np.argmax(np.abs(ga - ra)), np.abs(ga - ra).max(), sa)
        assert np.abs(gp - rp).max() <= 1e-9 * sp, (np.argmax(np.abs(gp - rp)), np.abs(gp - rp).max(), sp)


@pytest.mark.parametrize("kind,perturb", [("tet", 0.0), ("pyramid", 0.0), ("prism", 0.0), ("prism", 0.15),
                                          ("mixed", 0.0), ("merged", 0.0), ("merged", 0.1),
                                          ("merged_joined", 0.1), ("merged_sparse", 0.1)])
def test_adjoint_on_cells_other_than_hexahedra(oracle_lib, kind, perturb):
    """Tetrahedra, pyramids, prisms (flat, or with bent quadrilaterals), hexahedra next to prisms and
    general polyhedra (mostly polyhedra, flat or bent; joined faces of 6 and 8 points; a minority
    beside the eight-lane kernels): every component of the adjoint against the oracle's Jacobian
    (one exact tangent per input component), for two seeds."""
    O = oracle_lib
    w = W.poly_violent(kind, nx=8, ny=4, nz=4, steps=4, perturb=perturb)
    n, nf = w.mesh.n_cells, w.mesh.n_faces
    a = _state_after(O, w, 2)
    phi, U = w.phi_U(2)
    om = O.OracleMesh(w.mesh)
    _, st = om.step(a, phi, U, w.dt)
    say(f"[gpu] adjoint on {kind} (perturb {perturb}): {n} cells, {st['n_surface']} interface cells")
    assert st["n_surface"] > 10
    ja = np.array([om.step_tlm(a, phi, U, w.dt, dalpha=np.eye(1, n, k)[0])[1] for k in range(n)])
    jp = np.array([om.step_tlm(a, phi, U, w.dt, dphi=np.eye(1, nf, f)[0])[1] for f in range(nf)])
    gm, plan = gpu_plan(w.mesh)
    for bar in (np.ones(n), np.random.default_rng(13).standard_normal(n)):
        ga, gp = _adjoint(plan, w, a, phi, U, bar)
        ra, rp = ja @ bar, jp @ bar
        sa = max((np.abs(ja) @ np.abs(bar)).max(), 1e-300)
        sp = max((np.abs(jp) @ np.abs(bar)).max(), 1e-300)
        assert np.abs(ga - ra).max() <= 1e-9 * sa, (np.argmax(np.abs(ga - ra)), np.abs(ga - ra).max(), sa)
        assert np.abs(gp - rp).max() <= 1e-9 * sp, (np.argmax(np.abs(gp - rp)), np.abs(gp - rp).max(), sp)


def test_adjoint_keeps_each_rate_at_exact_ties(oracle_lib):
    """The small violent case is mirror-symmetric about y = 1/2: in the middle row of cells both
    ends of every y-edge carry the same value, so the distances of a face's vertices from the
    isoface come in pairs that tie exactly or differ by round-off, depending on the last bit of the
    isovalue.  Each vertex's rate must survive either way: the gradient with every traced isovalue
    moved one ulp up, or one ulp down, is the oracle's."""
    import torch
    O = oracle_lib
    w = W.violent_3d(nx=6, ny=5, nz=4, steps=4)
    say(f"[gpu] adjoint with the isovalues moved by one ulp: {w.name} cells={w.mesh.n_cells}")
    a = _state_after(O, w, 2)
    phi, U = w.phi_U(2)
    abar_new = np.random.default_rng(3).standard_normal(w.mesh.n_cells)
    gm, plan = gpu_plan(w.mesh)
    _, _, tr = gpu_traced_step(plan, gm, a, phi, U, w.dt)
    oa, op = O.OracleMesh(w.mesh).gradient(a, phi, U, w.dt, abar_new)
    rec = tr["kind"] == 1
    assert rec.sum() > 10
    for towards in (np.inf, -np.inf):
        iso = tr["iso"].copy()
        iso[rec] = np.nextafter(iso[rec], towards)
        dev_tr = {"vert_alpha": to_dev(tr["vert_alpha"].reshape(-1)), "iso": to_dev(iso), "dV": to_dev(tr["dV"]),
                  "alpha_raw": to_dev(tr["alpha_raw"]),
                  "kind": torch.tensor(tr["kind"], dtype=torch.int32, device="cuda:0")}
        ab, pb = plan.adjoint(to_dev(a), to_dev(phi), to_dev(U), w.dt, to_dev(abar_new), trace=dev_tr)
        torch.cuda.synchronize()
        ab, pb = ab.cpu().numpy(), pb.cpu().numpy()
        assert np.abs(ab - oa).max() <= 1e-9 * np.abs(oa).max(), (towards, np.argmax(np.abs(ab - oa)))
        assert np.abs(pb - op).max() <= 1e-9 * np.abs(op).max(), (towards, np.argmax(np.abs(pb - op)))


def test_adjoint_dot_product_against_oracle_tangent(oracle_lib):
    O = oracle_lib
    base, _ = W.adjoint_case()
    say(f"[gpu] adjoint dot-product test: {base.name} cells={base.mesh.n_cells}")
    a = _state_after(O, base, 3)
    phi, U = base.phi_U(3)
    om = O.OracleMesh(base.mesh)
    rng = np.random.default_rng(4)
    abar_new = rng.standard_normal(base.mesh.n_cells)
    gm, plan = gpu_plan(base.mesh)
    ga, gp = _adjoint(plan, base, a, phi, U, abar_new)
    for k in range(6):
        da = rng.standard_normal(base.mesh.n_cells)
        dp = rng.standard_normal(base.mesh.n_faces) * np.abs(phi).max()
        _, t = om.step_tlm(a, phi, U, base.dt, da, dp)
        lhs, rhs = ga @ da + gp @ dp, abar_new @ t
        assert abs(lhs - rhs) <= 1e-9 * (np.abs(ga * da).sum() + np.abs(gp * dp).sum()), (k, lhs, rhs)


@pytest.fixture(scope="module")
def misfit():
    """The adjoint workload: 50 steps, loss sum (alpha_T - alpha_target)^2, target from a run with a
    perturbed steepness; fields resident on the device."""
    import torch
    base, target = W.adjoint_case()
    S = base.n_steps
    phis = torch.stack([to_dev(base.phi_U(n)[0]) for n in range(S)]).contiguous()
    Us = torch.stack([to_dev(base.phi_U(n)[1]) for n in range(S)]).contiguous()
    gm, plan = gpu_plan(base.mesh)
    tphis = torch.stack([to_dev(target.phi_U(n)[0]) for n in range(S)]).contiguous()
    tUs = torch.stack([to_dev(target.phi_U(n)[1]) for n in range(S)]).contiguous()
    gt, tplan = gpu_plan(target.mesh)
    a = to_dev(target.alpha0)
    b = torch.empty_like(a)
    for n in range(S):
        tplan.step(a, tphis[n], tUs[n], target.dt, out=b)
        a, b = b, a
    torch.cuda.synchronize()
    return dict(w=base, plan=plan, gm=gm, phis=phis, Us=Us, alpha_target=a.clone(), S=S)


def _loss_and_grad(M, alpha0, phis, every=10, grad=True):
    import torch
    from paper_1804_01130_amd.autograd import advect
    a0 = alpha0.clone().requires_grad_(grad)
    ph = phis.clone().requires_grad_(grad)
    aT = advect(a0, ph, M["plan"], M["Us"], M["w"].dt, checkpoint_every=every)
    L = ((aT - M["alpha_target"]) ** 2).sum()
    if not grad:
        return L.item(), None, None
    L.backward()
    torch.cuda.synchronize()
    return L.item(), a0.grad.clone(), ph.grad.clone()


def _psi_direction(mesh, rng):
    L = mesh.xs[-1] - mesh.xs[0]
    H = mesh.ys[-1] - mesh.ys[0]
    c = rng.standard_normal(3)
    return lambda x, y, z0, z1: np.sin(np.pi * y / H) * (c[0] * np.cos(2 * np.pi * x / L) + c[1] * np.sin(
        4 * np.pi * x / L) + c[2] * np.cos(6 * np.pi * x / L)) * (z1 - z0)


def test_gradient_of_fifty_steps_against_central_differences(misfit):
    import torch
    M = misfit
    w = M["w"]
    say(f"[gpu] 50-step gradient vs central differences: {w.name}")
    alpha0 = to_dev(w.alpha0)
    L0, ga, gp = _loss_and_grad(M, alpha0, M["phis"])
    say(f"[gpu]   loss {L0:.12e}")
    rng = np.random.default_rng(8)
    inner = (w.alpha0 > 1e-4) & (w.alpha0 < 1 - 1e-4)
    checked = 0
    for k in range(6):
        da = to_dev(rng.standard_normal(w.mesh.n_cells) * inner)
        dp1 = W.fluxes_from_edge_integral(w.mesh, _psi_direction(w.mesh, rng))
        dp1 *= np.abs(w.phi_U(0)[0]).max() / np.abs(dp1).max()
        dp = to_dev(dp1)[None, :].expand_as(M["phis"]).contiguous()
        pred = float((ga * da).sum() + (gp * dp).sum())

        def L(e):
            return _loss_and_grad(M, alpha0 + e * da, M["phis"] + e * dp, grad=False)[0]
        # over 50 steps the loss has many small kinks (cut points crossing vertices, sweep
        # breakpoints reaching the ends of the step): a direction counts as smooth at this scale when
        # central differences with two small steps agree to 1e-6, and the adjoint must then agree
        # with the smaller one to 1e-6
        fd = [(L(h) - L(-h)) / (2 * h) for h in (2.5e-7, 5e-7, 1e-6)]
        if abs(fd[0] - fd[1]) > 1e-6 * max(abs(fd[0]), 1e-300):
            say(f"[gpu]   direction {k}: kink within 5e-7, skipped ({fd} adjoint {pred:.9e})")
            continue
        say(f"[gpu]   direction {k}: adjoint {pred:.12e} central differences {fd}")
        assert abs(pred - fd[0]) <= 1e-6 * max(abs(fd[0]), abs(pred)), (k, pred, fd)
        checked += 1
    assert checked >= 3


def test_checkpoint_interval_does_not_change_the_gradient(misfit):
    """The adjoint sums in a fixed order (no atomics), and the recomputed segments repeat the
    forward bit for bit: the gradient is the same bits for every checkpoint interval, and on a
    second run."""
    import torch
    M = misfit
    alpha0 = to_dev(M["w"].alpha0)
    ref = _loss_and_grad(M, alpha0, M["phis"], every=10)
    for every in (1, 7, 50, 10):
        say(f"[gpu] checkpoint interval {every}")
        got = _loss_and_grad(M, alpha0, M["phis"], every=every)
        assert got[0] == ref[0]
        for g, r in ((got[1], ref[1]), (got[2], ref[2])):
            assert torch.equal(g, r), float((g - r).abs().max())


def test_adjoint_argument_errors():
    import torch
    from paper_1804_01130_amd import IsoError, Plan, default_options
    w = W.cosine_uniform(nx=8, ny=4, steps=1)
    gm, plan = gpu_plan(w.mesh)
    phi, U = w.phi_U(0)
    a, p, u = to_dev(w.alpha0), to_dev(phi), to_dev(U)
    with pytest.raises(IsoError):
        plan.adjoint(a, p, u, -1.0, torch.zeros_like(a))
    with pytest.raises(IsoError):
        plan.adjoint(a, p, u, w.dt, torch.zeros_like(a), alpha_bar=a)  # output overlaps an input
    with pytest.raises(IsoError):
        plan.adjoint(a, p, u, w.dt, torch.zeros_like(a), trace={"kind": torch.zeros(gm.n_cells, dtype=torch.int32,
                                                                                       device=a.device)})
    many = Plan(gm, default_options(n_bound_iter=40))
    with pytest.raises(IsoError):
        many.adjoint(a, p, u, w.dt, torch.zeros_like(a))


def test_advect_leaves_the_callers_state_alone(misfit):
    """The differentiable multi-step advection steps on its own buffers: the caller's initial state
    (a leaf that requires grad) is unchanged after forward and backward."""
    import torch
    from paper_1804_01130_amd.autograd import advect
    M = misfit
    say("[gpu] advect keeps alpha0 unchanged")
    a0 = to_dev(M["w"].alpha0).requires_grad_(True)
    before = a0.detach().clone()
    aT = advect(a0, M["phis"][:4].clone().requires_grad_(True), M["plan"], M["Us"][:4], M["w"].dt,
                checkpoint_every=2)
    ((aT - M["alpha_target"]) ** 2).sum().backward()
    torch.cuda.synchronize()
    assert torch.equal(a0.detach(), before)
    assert not torch.equal(aT.detach(), before)
