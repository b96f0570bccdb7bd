"""GPU path (through the C interface) against the CPU oracle, element by element.

Bar: 1e-10 per cell in FP64 for whole trajectories; intermediates of one step from identical
inputs are compared tighter (they differ only by rounding order).  Interface classification and
cell kinds must agree exactly.
"""
import numpy as np
import pytest

import wavegen as W
from tests.gpuutil import gpu_plan, gpu_traced_step, gpu_trajectory, oracle_trajectory, say, to_dev

pytestmark = pytest.mark.gpu

TOL_TRAJ = 1e-10


def small_cases():
    band_mesh = W.hex_block(np.linspace(0, 1, 17), np.linspace(0, 1.5, 25), [0.0, 1 / 16], periodic_x=True,
                            periodic_y=True, kinds={"zmin": W.PATCH_EMPTY, "zmax": W.PATCH_EMPTY})
    phi_b = W.fluxes_from_edge_integral(band_mesh, lambda x, y, z0, z1: (0.7 * y - 0.6 * x) * (z1 - z0))
    U_b = np.concatenate([np.full(band_mesh.n_cells, 0.7), np.full(band_mesh.n_cells, 0.6), np.zeros(band_mesh.n_cells)])
    a_b = W.alpha_cosine_2d(band_mesh, 0.9021, 0.0, 1.0) - W.alpha_cosine_2d(band_mesh, 0.3137, 0.0, 1.0)
    band = W.Workload("band_periodic", band_mesh, a_b, W.courant_dt(band_mesh, phi_b, 0.45), 8,
                      lambda n: (phi_b, U_b), steady=True)
    return {
        "cosine_64x32": W.cosine_uniform(),
        "airy_128x64": W.airy_slab(128, 64, 32, 0.07, 0.5, 30, "airy_128x64"),
        "violent_32x16x16": W.violent_3d(nx=32, ny=16, nz=16, steps=10),
        "band_periodic": band,
        # non-planar faces (randomly displaced interior points), in/out patches with inflow alpha
        "perturbed_10x7x6": W.perturbed_box(),
    }


CASES = small_cases()


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


@pytest.mark.parametrize("name", list(CASES))
def test_one_step_intermediates(O, name):
    w = CASES[name]
    say(f"[gpu] one-step intermediates: {name} cells={w.mesh.n_cells}")
    gm, plan = gpu_plan(w.mesh)
    om = O.OracleMesh(w.mesh)
    phi, U = w.phi_U(0)
    g_new, g_st, g = gpu_traced_step(plan, gm, w.alpha0, phi, U, w.dt)
    o_new, o_st, o = om.step(w.alpha0, phi, U, w.dt, trace=True)
    _, V = om.geometry()
    vol, _ = gm.geometry()
    assert np.abs(vol - V).max() <= 1e-15 * V.max()
    # classification
    assert np.array_equal(g["kind"], o["kind"]), np.nonzero(g["kind"] != o["kind"])[0][:10]
    assert g_st["n_surface"] == o_st["n_surface"]
    surf = np.nonzero(o["kind"] > 0)[0]
    rec = np.nonzero(o["kind"] == 1)[0]
    assert len(rec) > 0
    # vertex values of interface cells (inverse-distance interpolation)
    cp = gm.cell_points()
    # normalised weights vs. sum-then-divide: a few ulps of a value <= 1
    assert np.abs(g["vert_alpha"][surf] - o["a_pts"][cp[surf]]).max() <= 16 * np.finfo(float).eps
    # the GPU isovalue cuts off alpha V to 1e-12, judged by the oracle's sub-volume; where the
    # sub-volume jumps across alpha V at a vertex value, both sides take that vertex value
    for c in rec[:: max(1, len(rec) // 40)]:
        fo = om.cut(c, o["a_pts"], o["iso"][c])["vsub"] / V[c] - w.alpha0[c]
        if abs(fo) <= 1e-12:
            cut = om.cut(c, o["a_pts"], g["iso"][c])
            assert abs(cut["vsub"] / V[c] - w.alpha0[c]) <= 1e-12
        else:
            assert abs(g["iso"][c] - o["iso"][c]) <= 8 * np.finfo(float).eps
    # isoface centre, normal, normal speed
    h = np.cbrt(V[rec])[:, None]
    assert np.abs(g["rec"][rec, 0:3] - o["rec"][rec, 0:3]).max() <= 1e-11 * h.max()
    assert np.abs(g["rec"][rec, 3:6] - o["rec"][rec, 3:6]).max() <= 1e-11
    assert np.abs(g["rec"][rec, 6] - o["rec"][rec, 6]).max() <= 1e-11 * max(1.0, np.abs(U).max())
    # face volumes
    fl = np.abs(phi).max() * w.dt
    flux_faces = ~np.isnan(g["dV"])
    assert np.abs(g["dV"][flux_faces] - o["dV"][flux_faces]).max() <= 1e-13 * fl
    # update and bounding
    assert np.abs(g["alpha_raw"] - o["alpha_raw"]).max() <= 1e-13
    assert np.abs(g_new - o_new).max() <= 1e-13
    assert g_st["n_bound_active"] == o_st["n_bound_active"]


@pytest.mark.parametrize("name", list(CASES))
def test_trajectory(O, name):
    w = CASES[name]
    say(f"[gpu] trajectory: {name} steps={w.n_steps}")
    gm, plan = gpu_plan(w.mesh)
    om = O.OracleMesh(w.mesh)
    g = gpu_trajectory(plan, w, w.n_steps)
    o = oracle_trajectory(om, w, w.n_steps)
    err = np.abs(g - o).max()
    say(f"[gpu]   max |gpu - oracle| = {err:.3e}")
    assert err <= TOL_TRAJ


@pytest.mark.parametrize("name", ["airy_128x64", "violent_32x16x16", "perturbed_10x7x6"])
def test_root_tolerance_bounds_the_volume_error(O, name):
    """root_tol (Section 3.2 leaves the isovalue's tolerance to the user): at 1e-6 the sub-volume
    the oracle computes at each GPU isovalue meets alpha_P within 1e-6, the searches take fewer
    rounds than at round-off, none fails to converge, and the step moves by at most a few times
    the tolerance from the oracle's round-off step (each face's swept volume moves by at most
    about the tolerance times the cell volume)."""
    w = CASES[name]
    say(f"[gpu] root_tol 1e-6: {name} cells={w.mesh.n_cells}")
    gm, plan = gpu_plan(w.mesh, root_tol=1e-6)
    _, plan0 = gpu_plan(w.mesh)
    om = O.OracleMesh(w.mesh)
    phi, U = w.phi_U(0)
    g_new, g_st, g = gpu_traced_step(plan, gm, w.alpha0, phi, U, w.dt)
    _, _, g0 = gpu_traced_step(plan0, gm, w.alpha0, phi, U, w.dt)
    o_new, _, o = om.step(w.alpha0, phi, U, w.dt, trace=True)
    _, V = om.geometry()
    assert np.array_equal(g["kind"], o["kind"])
    rec = np.nonzero(o["kind"] == 1)[0]
    worst, at_jump = 0.0, 0
    for c in rec:
        fo = om.cut(c, o["a_pts"], o["iso"][c])["vsub"] / V[c] - w.alpha0[c]
        if abs(fo) > 1e-12:  # the sub-volume jumps across alpha V: both sides take the vertex value
            assert abs(g["iso"][c] - o["iso"][c]) <= 8 * np.finfo(float).eps
            at_jump += 1
            continue
        e = abs(om.cut(c, o["a_pts"], g["iso"][c])["vsub"] / V[c] - w.alpha0[c])
        worst = max(worst, e)
        assert e <= 1e-6 + 1e-12, (c, e)
    rounds, rounds0 = int(g["iters"][rec].sum()), int(g0["iters"][rec].sum())
    err = float(np.abs(g_new - o_new).max())
    say(f"[gpu]   worst |V_sub/V - alpha| {worst:.2e} over {len(rec)} cells ({at_jump} at a jump); "
        f"rounds {rounds} vs {rounds0} at round-off; max |alpha_new - oracle| {err:.2e}")
    assert g_st["n_nonconverged"] == 0
    assert rounds < rounds0
    assert err <= 1e-5


@pytest.mark.parametrize("n_iter,clip", [(0, 1), (0, 0), (1, 1), (2, 0), (5, 1)])
def test_bounding_sweep_counts(O, n_iter, clip):
    """Every bounding schedule against the oracle with the same options: no sweep (chop only, or
    nothing), one sweep (its phase A runs inside the update), and more sweeps than the three
    rotating counter slots; with and without the final chop."""
    import torch
    w = CASES["violent_32x16x16"]
    say(f"[gpu] bounding sweeps={n_iter} clip={clip}: {w.name}")
    gm, plan = gpu_plan(w.mesh, n_bound_iter=n_iter, clip=clip)
    om = O.OracleMesh(w.mesh)
    steps = 12
    phi, U = w.phi_U(0)
    tphi, tU = to_dev(phi), to_dev(U)
    a = to_dev(w.alpha0)
    b = torch.empty_like(a)
    active = 0
    for _ in range(steps):
        _, st = plan.step(a, tphi, tU, w.dt, out=b, stats=True)
        active += st["n_bound_active"]
        a, b = b, a
    g = a.cpu().numpy()
    o = oracle_trajectory(om, w, steps, opts=O.default_opts(n_bound_iter=n_iter, clip=clip))
    err = np.abs(g - o).max()
    say(f"[gpu]   cells flagged for bounding over the run: {active}; max |gpu - oracle| = {err:.3e}")
    assert active > 0
    assert err <= TOL_TRAJ


def test_planar_transport_exact_on_gpu(O):
    """The exactness pin of the oracle holds for the GPU path too (clip off)."""
    w = CASES["band_periodic"]
    say("[gpu] planar band transport")
    gm, plan = gpu_plan(w.mesh, clip=0)
    a = gpu_trajectory(plan, w, 8)
    exact = W.alpha_cosine_2d(w.mesh, 0.9021 + 0.6 * 8 * w.dt, 0.0, 1.0) - \
        W.alpha_cosine_2d(w.mesh, 0.3137 + 0.6 * 8 * w.dt, 0.0, 1.0)
    assert np.abs(a - exact).max() <= 1e-12


def _slot_word_cases():
    # (workload, flux slots expected to be read from the full tables: the cyclic pair in x of each
    # row of the box, the inflow and outflow faces of the perturbed box; None: not checked)
    v = W.violent_3d(nx=24, ny=13, nz=16, steps=5)
    p = W.perturbed_box()
    return {"violent_24x13x16": (v, 2 * 13 * 16), "perturbed_10x7x6": (p, 2 * 7 * 6),
            "airy_128x64": (CASES["airy_128x64"], None),
            "tet_12x6x6": (W.poly_violent("tet", nx=12, ny=6, nz=6, steps=5), None),
            "mixed_16x8x8": (W.poly_violent("mixed", nx=16, ny=8, nz=8, steps=5), None),
            "merged_16x8x8": (W.poly_violent("merged", nx=16, ny=8, nz=8, steps=5), None)}


SLOT_WORD_CASES = _slot_word_cases()


@pytest.mark.parametrize("name", list(SLOT_WORD_CASES))
def test_slot_words_give_the_same_bits_as_the_full_tables(name):
    w, wide = SLOT_WORD_CASES[name]
    say(f"[gpu] update through 32-bit slot words vs the full tables: {name} ({w.mesh.n_cells} cells)")
    gm, plan = gpu_plan(w.mesh)
    info = gm.info()
    say(f"[gpu]   slots per cell {info['slots']}, slots read from the full tables {info['wide_slots']}")
    assert info["wide_slots"] >= 0  # every mesh here has the words
    if wide is not None:
        assert info["wide_slots"] == wide
    a = gpu_trajectory(plan, w, 5)
    plan.close()
    _, full = gpu_plan(w.mesh, full_slots=1)
    b = gpu_trajectory(full, w, 5)
    full.close()
    assert np.array_equal(a, b)
    assert not np.array_equal(a, w.alpha0)


def _flipped(w, frac=0.04, seed=11):
    """The workload with a seeded fraction of its internal faces turned around (owner and
    neighbour swapped, the point loop reversed, the flux negated): the same flow on the same
    cells, with those faces' owners numbered above their neighbours."""
    import dataclasses
    m = w.mesh
    ni = m.n_internal
    rng = np.random.default_rng(seed)
    flip = np.zeros(m.n_faces, bool)
    flip[:ni] = rng.random(ni) < frac
    owner, neighbour = m.owner.copy(), m.neighbour.copy()
    owner[:ni][flip[:ni]], neighbour[flip[:ni]] = m.neighbour[flip[:ni]], m.owner[:ni][flip[:ni]]
    pts = m.face_pts.copy()
    for f in np.flatnonzero(flip):
        a, b = m.face_ptr[f], m.face_ptr[f + 1]
        pts[a:b] = m.face_pts[a:b][::-1]
    mesh = dataclasses.replace(m, face_pts=pts, owner=owner, neighbour=neighbour)
    sign = np.where(flip, -1.0, 1.0)
    fields = lambda n: (sign * w.phi_U(n)[0], w.phi_U(n)[1])
    return dataclasses.replace(w, name=w.name + "_flipped", mesh=mesh, fields=fields), int(flip.sum())


def test_slot_words_with_faces_owned_by_the_higher_cell(oracle_lib):
    """Internal faces whose owner is numbered above the neighbour do not fit the slot words: those
    slots (two per face) are read from the full tables, the others from the words, with the same
    bits as the full tables alone and the oracle's trajectory."""
    base = W.violent_3d(nx=24, ny=13, nz=16, steps=6)
    w, n_flip = _flipped(base)
    say(f"[gpu] slot words with {n_flip} faces turned around: {w.name} ({w.mesh.n_cells} cells)")
    gm, plan = gpu_plan(w.mesh)
    info = gm.info()
    assert info["wide_slots"] == 2 * n_flip + 2 * 13 * 16  # the turned faces and the cyclic pairs
    a = gpu_trajectory(plan, w, 6)
    plan.close()
    _, full = gpu_plan(w.mesh, full_slots=1)
    b = gpu_trajectory(full, w, 6)
    full.close()
    assert np.array_equal(a, b)
    ref = oracle_trajectory(oracle_lib.OracleMesh(w.mesh), w, 6)
    err = np.abs(a - ref).max()
    say(f"[gpu]   max |gpu - oracle| = {err:.3e}")
    assert err <= 1e-10
    # the turned mesh is the same flow on the same cells: its trajectory is the original's
    _, orig = gpu_plan(base.mesh)
    c = gpu_trajectory(orig, base, 6)
    orig.close()
    assert np.abs(a - c).max() <= 1e-12


def test_no_slot_words_where_neighbours_lie_too_far_apart():
    """A box two cells high whose z-neighbours are 256 x 130 = 33280 cells apart: a fifth of the
    flux slots (both sides of every z-face, and the cyclic pairs) cannot take the words, more than
    the tenth allowed, so the mesh gets none and the update reads the full tables."""
    w = W.violent_3d(nx=256, ny=130, nz=2, steps=2)
    say(f"[gpu] slot words refused: {w.name} ({w.mesh.n_cells} cells)")
    gm, plan = gpu_plan(w.mesh)
    assert gm.info()["wide_slots"] == -1
    a = gpu_trajectory(plan, w, 2)
    plan.close()
    assert not np.array_equal(a, w.alpha0)


def test_determinism_across_launch_shapes():
    w = CASES["violent_32x16x16"]
    say("[gpu] determinism across block sizes")
    outs = []
    # 32 and 100 threads per work-group leave the update kernel's waves partly filled
    for bc, sw in ((256, 2), (64, 3), (128, 4), (32, 1), (100, 2)):
        gm, plan = gpu_plan(w.mesh, block_cells=bc, surface_waves=sw)
        outs.append(gpu_trajectory(plan, w, 5))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
