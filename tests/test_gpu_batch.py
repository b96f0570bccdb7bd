"""Ensembles (iso_batch_*) through the C interface: every member of a batched run must equal, bit
for bit, the same member stepped alone by its own plan, and match the oracle at 1e-10.  Graph
replays are checked against eager runs with other device work in between."""
import numpy as np
import pytest

import wavegen as W
from tests.gpuutil import dev, oracle_trajectory, say, to_dev

pytestmark = pytest.mark.gpu

STEPS = 9  # odd: the run ends in the ensemble's second state buffer and is copied back


def members():
    """Mixed 2D (4 flux slots) and 3D (6 slots) members of uneven sizes, time-dependent fields."""
    return [W.airy_slab(96, 48, 24, 0.07, 0.45, STEPS, "m0"),
            W.cosine_uniform(nx=40, ny=20, steps=STEPS),
            W.violent_3d(nx=16, ny=8, nz=8, steps=STEPS),
            W.airy_slab(64, 32, 32, 0.05, 0.35, STEPS, "m3"),
            W.airy_slab(128, 32, 32, 0.09, 0.5, STEPS, "m4")]


def members_of_all_cells():
    """Tetrahedra, pyramids, bent prisms, hexahedra next to prisms and general polyhedra (mostly
    polyhedra with faces of at most 4 points; joined faces of 6 and 8 points, which take the other
    instantiation of the polyhedron kernel; a minority of bent polyhedra), beside meshes of
    hexahedra (2D and 3D)."""
    return [W.poly_violent("tet", nx=8, ny=4, nz=4, steps=STEPS),
            W.airy_slab(64, 32, 32, 0.05, 0.35, STEPS, "h1"),
            W.poly_violent("prism", nx=12, ny=6, nz=6, steps=STEPS, perturb=0.15),
            W.poly_violent("merged", nx=12, ny=6, nz=6, steps=STEPS),
            W.violent_3d(nx=16, ny=8, nz=8, steps=STEPS),
            W.poly_violent("merged_joined", nx=12, ny=6, nz=6, steps=STEPS),
            W.poly_violent("pyramid", nx=8, ny=4, nz=4, steps=STEPS),
            W.poly_violent("merged_sparse", nx=16, ny=8, nz=8, steps=STEPS, perturb=0.1),
            W.poly_violent("mixed", nx=12, ny=6, nz=6, steps=STEPS)]


def _build(ws, **opts):
    import torch
    from paper_1804_01130_amd import Batch, Mesh, Plan, default_options
    meshes = [Mesh.from_arrays(w.mesh) for w in ws]
    batch = Batch(meshes, default_options(**opts))
    S = STEPS
    phi = torch.stack([torch.cat([to_dev(w.phi_U(n)[0]) for w in ws]) for n in range(S)]).contiguous()
    U = torch.stack([to_dev(batch.concat_U([w.phi_U(n)[1] for w in ws])) for n in range(S)]).contiguous()
    alpha0 = to_dev(batch.concat_cells([w.alpha0 for w in ws]))
    dts = np.array([w.dt for w in ws])
    # each member alone, eagerly, through its own plan
    alone = []
    for w, m in zip(ws, meshes):
        plan = Plan(m, default_options(**opts))
        a = to_dev(w.alpha0)
        b = torch.empty_like(a)
        for n in range(S):
            p, u = w.phi_U(n)
            plan.step(a, to_dev(p), to_dev(u), w.dt, out=b)
            a, b = b, a
        torch.cuda.synchronize()
        alone.append(a.cpu().numpy())
        plan.close()
    return dict(ws=ws, meshes=meshes, batch=batch, phi=phi, U=U, alpha0=alpha0, dts=dts, alone=alone)


@pytest.fixture(scope="module")
def ensemble():
    return _build(members())


def _run(E, steps=STEPS, alpha=None):
    a = (E["alpha0"] if alpha is None else alpha).clone()
    F, N3 = E["phi"].shape[1], E["U"].shape[1]
    E["batch"].advect(a, E["phi"], E["U"], E["dts"], steps, phi_stride=F, U_stride=N3)
    import torch
    torch.cuda.synchronize()
    return a


def test_batch_equals_members_alone_bitwise(ensemble):
    E = ensemble
    say(f"[gpu] ensemble of {len(E['ws'])} members, {E['batch'].n_cells} cells, {STEPS} steps")
    got = E["batch"].split_cells(_run(E).cpu().numpy())
    for d, (g, ref) in enumerate(zip(got, E["alone"])):
        assert np.array_equal(g, ref), (d, np.abs(g - ref).max())


def test_members_sharing_blocks_of_64_cells():
    """Members of a few dozen cells: three of them meet in the first 64-cell block of the union's
    slot-word records (there the update finds each cell's member by a search), and two have no
    slot words of their own (more than a tenth of their slots are cyclic or inflow faces), so
    every slot of theirs is read from the full tables; the same bits as each member alone, with
    the words and without them."""
    ws = [W.cosine_uniform(nx=8, ny=4, steps=STEPS), W.violent_3d(nx=4, ny=2, nz=2, steps=STEPS),
          W.cosine_uniform(nx=6, ny=4, steps=STEPS), W.poly_violent("tet", nx=3, ny=2, nz=2, steps=STEPS),
          W.airy_slab(16, 8, 4, 0.07, 0.45, STEPS, "s4"), W.perturbed_box(nx=4, ny=3, nz=3, steps=STEPS)]
    off = np.cumsum([0] + [w.mesh.n_cells for w in ws])
    assert off[2] < 64  # members 0, 1 and 2 in the first block
    runs = []
    for full in (0, 1):
        say(f"[gpu] ensemble of {len(ws)} small members ({off[-1]} cells), full_slots={full}")
        E = _build(ws, full_slots=full)
        wide = [m.info()["wide_slots"] for m in E["meshes"]]
        assert min(wide) < 0 <= max(wide), wide  # members with words and members without
        got = E["batch"].split_cells(_run(E).cpu().numpy())
        for d, (g, ref) in enumerate(zip(got, E["alone"])):
            assert np.array_equal(g, ref), (full, d, np.abs(g - ref).max())
        runs.append(got)
        E["batch"].close()
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


def test_batch_members_match_oracle(ensemble, oracle_lib):
    E = ensemble
    got = E["batch"].split_cells(_run(E).cpu().numpy())
    for d, w in enumerate(E["ws"]):
        say(f"[gpu] ensemble member {d} vs oracle: {w.name}")
        ref = oracle_trajectory(oracle_lib.OracleMesh(w.mesh), w, STEPS)
        assert np.abs(got[d] - ref).max() <= 1e-10, (d, np.abs(got[d] - ref).max())


@pytest.mark.parametrize("us_mode", [0, 1])
def test_members_of_every_cell_type(oracle_lib, us_mode):
    """Members of every cell type: the generic interface kernel over the whole ensemble (the
    hexahedral members with their faces in the hexahedron kernel's edge directions), and the
    polyhedron kernel once per instantiation its members take alone, on the side stream inside the
    captured graph: every member still equals itself stepped alone, bit for bit, and matches the
    oracle."""
    E = _build(members_of_all_cells(), us_mode=us_mode)
    say(f"[gpu] ensemble of every cell type, us_mode {us_mode}: {len(E['ws'])} members, "
        f"{E['batch'].n_cells} cells, {STEPS} steps")
    got = E["batch"].split_cells(_run(E).cpu().numpy())
    for d, (g, ref) in enumerate(zip(got, E["alone"])):
        assert np.array_equal(g, ref), (d, np.abs(g - ref).max())
    for d, w in enumerate(E["ws"]):
        ref = oracle_trajectory(oracle_lib.OracleMesh(w.mesh), w, STEPS,
                                opts=oracle_lib.default_opts(us_mode=us_mode))
        assert np.abs(got[d] - ref).max() <= 1e-10, (d, np.abs(got[d] - ref).max())
    E["batch"].close()


def test_graph_replays_with_work_in_between(ensemble):
    """The same run replayed from a captured graph several times, with eager device work and
    synchronisations between replays; every replay equals the members run alone."""
    import torch
    E = ensemble
    ref = np.concatenate(E["alone"])
    a = E["alpha0"].clone()
    F, N3 = E["phi"].shape[1], E["U"].shape[1]
    for r in range(3):
        say(f"[gpu] graph replay {r}")
        a.copy_(E["alpha0"])
        junk = torch.randn(1 << 16, device=dev(), dtype=torch.float64)
        _ = (junk * 2.0).sum().item()  # eager work between replays
        E["batch"].advect(a, E["phi"], E["U"], E["dts"], STEPS, phi_stride=F, U_stride=N3)
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), ref), r
    # an even step count (no final copy) and steady fields (strides 0) through a new capture
    b = E["alpha0"].clone()
    E["batch"].advect(b, E["phi"][0].contiguous(), E["U"][0].contiguous(), E["dts"], 4)
    torch.cuda.synchronize()
    assert np.isfinite(b.cpu().numpy()).all()


def test_autotuner_choices_do_not_change_results(ensemble, tmp_path):
    E = ensemble
    ref = np.concatenate(E["alone"])
    cache = str(tmp_path / "tune.txt")
    cfg, ms = E["batch"].tune(E["alpha0"], E["phi"][0].contiguous(), E["U"][0].contiguous(), E["dts"], n_trial=2,
                              cache_path=cache)
    say(f"[gpu] tuned {cfg} {ms:.3f} ms/step")
    assert ms > 0 and open(cache).read().strip()
    assert np.array_equal(_run(E).cpu().numpy(), ref)
    # the cache answers the second time without trials
    cfg2, ms2 = E["batch"].tune(E["alpha0"], E["phi"][0].contiguous(), E["U"][0].contiguous(), E["dts"],
                                n_trial=2, cache_path=cache)
    assert cfg2 == cfg and ms2 == pytest.approx(ms, rel=1e-4)
    for shape in ({"block_cells": 64, "surface_blocks": 7, "surface_waves": 1, "bound_blocks": 3},
                  {"block_cells": 512, "surface_blocks": 2048, "surface_waves": 3, "bound_blocks": 1024}):
        E["batch"].set_config(**shape)
        assert np.array_equal(_run(E).cpu().numpy(), ref), shape


def test_batch_argument_errors(ensemble):
    from paper_1804_01130_amd import IsoError
    E = ensemble
    a = E["alpha0"].clone()
    F = E["phi"].shape[1]
    with pytest.raises(IsoError):
        E["batch"].advect(a, E["phi"], E["U"], -E["dts"], 1)
    with pytest.raises(IsoError):
        E["batch"].advect(a, E["phi"], E["U"], E["dts"], 2, phi_stride=F - 1)
    with pytest.raises(ValueError):
        E["batch"].advect(a, E["phi"], E["U"], E["dts"][:2], 1)
    with pytest.raises(IsoError):
        E["batch"].set_config(surface_waves=9)
