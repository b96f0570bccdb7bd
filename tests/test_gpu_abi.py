"""Error paths, statistics and restart behaviour of the C interface on the device."""
import numpy as np
import pytest

import wavegen as W
from paper_1804_01130_amd import binding as B
from tests.gpuutil import gpu_plan, gpu_trajectory, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    return W.airy_slab(128, 64, 32, 0.07, 0.5, 12, "airy_128x64")


def test_argument_errors(case):
    import torch
    say("[gpu] argument errors")
    gm, plan = gpu_plan(case.mesh)
    phi, U = case.phi_U(0)
    a, tphi, tU = to_dev(case.alpha0), to_dev(phi), to_dev(U)
    with pytest.raises(B.IsoError) as e:
        plan.step(a, tphi, tU, case.dt, out=a)  # output aliases the input
    assert e.value.status == B.ISO_EINVAL
    for dt in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(B.IsoError) as e:
            plan.step(a, tphi, tU, dt)
        assert e.value.status == B.ISO_EINVAL
    torch.cuda.synchronize()


def test_input_checks(case):
    say("[gpu] input checks")
    gm, plan = gpu_plan(case.mesh, check_inputs=1, max_courant=0.6)
    phi, U = case.phi_U(0)
    a = case.alpha0.copy()
    a[17] = np.nan
    with pytest.raises(B.IsoError) as e:
        plan.step(to_dev(a), to_dev(phi), to_dev(U), case.dt)
    assert e.value.status == B.ISO_EINVAL
    with pytest.raises(B.IsoError) as e:
        plan.step(to_dev(case.alpha0), to_dev(phi), to_dev(U), 2.0 * case.dt)  # Courant 1.0 > 0.6
    assert e.value.status == B.ISO_ECOURANT
    out, st = plan.step(to_dev(case.alpha0), to_dev(phi), to_dev(U), case.dt, stats=True)
    assert st["n_surface"] > 0


def test_capacity_exceeded_is_reported(case):
    say("[gpu] interface-cell capacity")
    gm, plan = gpu_plan(case.mesh, max_surface=8)
    phi, U = case.phi_U(0)
    with pytest.raises(B.IsoError) as e:
        plan.step(to_dev(case.alpha0), to_dev(phi), to_dev(U), case.dt)
    assert e.value.status == B.ISO_ENOSPACE


def test_stats_and_conservation(case, oracle_lib):
    say("[gpu] statistics")
    gm, plan = gpu_plan(case.mesh, clip=0)
    om = oracle_lib.OracleMesh(case.mesh)
    phi, U = case.phi_U(0)
    out, st = plan.step(to_dev(case.alpha0), to_dev(phi), to_dev(U), case.dt, stats=True)
    _, ost = om.step(case.alpha0, phi, U, case.dt, oracle_lib.default_opts(clip=0))
    assert st["n_surface"] == ost["n_surface"]
    assert st["n_bound_active"] == ost["n_bound_active"]
    assert abs(st["vol_after"] - st["vol_before"]) <= 1e-14 * st["vol_before"]
    assert abs(st["vol_before"] - ost["vol_before"]) <= 1e-14 * ost["vol_before"]


def test_restart_from_host_copy_is_bit_identical(case):
    """alpha is the whole state: stopping, copying to the host and back, and continuing gives the same bits."""
    say("[gpu] restart")
    gm, plan = gpu_plan(case.mesh)
    full = gpu_trajectory(plan, case, 12)
    half = gpu_trajectory(plan, case, 6)
    w2 = W.Workload(case.name, case.mesh, half, case.dt, 6, lambda n: case.phi_U(n + 6))
    rest = gpu_trajectory(plan, w2, 6)
    assert np.array_equal(rest, full)


@pytest.mark.parametrize("name", ["perturbed", "stressed_wave", "violent"])
def test_stats_against_the_oracle_with_chopping(oracle_lib, name):
    """Every statistic of a step with the chop on against the oracle's, on cases where the chop and
    the redistribution act and (perturbed box) volume enters and leaves through in/out patches; on
    both sides vol_after = vol_before - vol_boundary_flux + vol_clipped."""
    w = {"perturbed": lambda: W.perturbed_box(steps=4),
         "stressed_wave": lambda: W.airy_slab(64, 32, 16, 0.1, 0.95, 4, "airy_stressed"),
         "violent": lambda: W.violent_3d(nx=24, ny=13, nz=16, steps=4)}[name]()
    say(f"[gpu] statistics with chopping: {w.name}")
    gm, plan = gpu_plan(w.mesh)
    om = oracle_lib.OracleMesh(w.mesh)
    a = w.alpha0.copy()
    seen_clip = seen_bound = 0
    for n in range(w.n_steps):
        phi, U = w.phi_U(n)
        out, st = plan.step(to_dev(a), to_dev(phi), to_dev(U), w.dt, stats=True)
        o_out, ost = om.step(a, phi, U, w.dt)
        tot = max(abs(ost["vol_before"]), 1e-300)
        for k in ("n_surface", "n_flat", "n_bound_active"):
            assert st[k] == ost[k], (n, k, st[k], ost[k])
        for k, o_k in (("vol_before", "vol_before"), ("vol_after", "vol_after"),
                       ("vol_boundary_flux", "vol_boundary"), ("vol_clipped", "vol_clipped")):
            assert abs(st[k] - ost[o_k]) <= 1e-12 * tot, (n, k, st[k], ost[o_k])
        assert st["alpha_min"] == float(o_out.min()) or abs(st["alpha_min"] - o_out.min()) <= 1e-13
        assert st["alpha_max"] == float(o_out.max()) or abs(st["alpha_max"] - o_out.max()) <= 1e-13
        bal = st["vol_before"] - st["vol_boundary_flux"] + st["vol_clipped"]
        assert abs(st["vol_after"] - bal) <= 1e-12 * tot, (n, st)
        seen_clip += st["vol_clipped"] != 0.0
        seen_bound += st["n_bound_active"] > 0
        a = out.cpu().numpy()
    say(f"[gpu]   steps with clipped volume {seen_clip}, with redistribution {seen_bound}")
    assert seen_bound > 0
