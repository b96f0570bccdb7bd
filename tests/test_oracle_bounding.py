"""Pins of the oracle's bounding step, inflow boundary value and cell centres.

Expected values are hand-derived (tests/golden/bounding_channels.json, each case with its working)
or closed forms of elementary solids; none is produced by the oracle.
"""
import ast
import json
import operator
import os

import numpy as np
import pytest

import wavegen as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
_PATCH = {"xmin": 0, "xmax": 1, "ymin": 2, "ymax": 3, "zmin": 4, "zmax": 5}
_OPS = {ast.Add: operator.add, ast.Sub: operator.sub, ast.Mult: operator.mul, ast.Pow: operator.pow,
        ast.Div: operator.truediv}


def num(x):
    """A fixture number: a plain number, or a string of +, -, * and ** over literals (exact in FP64)."""
    if not isinstance(x, str):
        return float(x)

    def ev(n):
        if isinstance(n, ast.Expression):
            return ev(n.body)
        if isinstance(n, ast.Constant) and isinstance(n.value, (int, float)):
            return float(n.value)
        if isinstance(n, ast.UnaryOp) and isinstance(n.op, ast.USub):
            return -ev(n.operand)
        if isinstance(n, ast.BinOp) and type(n.op) in _OPS:
            return _OPS[type(n.op)](ev(n.left), ev(n.right))
        raise ValueError(f"unsupported fixture expression {x!r}")

    return ev(ast.parse(x, mode="eval"))


def channel_case(case):
    """Mesh, alpha and phi of one fixture case."""
    ms = case["mesh"]
    kinds = {k: W.PATCH_INOUT for k in ms["inout"]}
    mesh = W.hex_block(ms["xs"], ms["ys"], ms["zs"], kinds=kinds, periodic_x=False, alpha_in=ms["alpha_in"])
    phi = np.zeros(mesh.n_faces)
    for fl in case["fluxes"]:
        if "neighbour" in fl:
            hit = np.nonzero((mesh.owner[:mesh.n_internal] == fl["owner"]) & (mesh.neighbour == fl["neighbour"]))[0]
        else:
            p = mesh.patches[_PATCH[fl["patch"]]]
            faces = np.arange(p.start, p.start + p.size)
            hit = faces[mesh.owner[faces] == fl["owner"]]
        assert hit.size == 1, fl
        phi[hit[0]] = num(fl["phi"])
    alpha = np.array([num(a) for a in case["alpha"]])
    return mesh, alpha, phi


def _cases():
    data = json.load(open(os.path.join(GOLD, "bounding_channels.json")))
    for case in data["cases"]:
        for k, run in enumerate(case["runs"]):
            yield pytest.param(case, run, id=f"{case['name']}-{k}")


@pytest.mark.parametrize("case,run", list(_cases()))
def test_bounding_and_inflow_golden(oracle_lib, case, run):
    mesh, alpha, phi = channel_case(case)
    om = oracle_lib.OracleMesh(mesh)
    xc, V = om.geometry()
    # the oracle's volumes are pyramid sums: 1 to a few ulps, which is why values carry 1e-14
    assert np.allclose(V, 1.0, rtol=0, atol=1e-15)
    U = np.zeros(3 * mesh.n_cells)
    opts = oracle_lib.default_opts(n_bound_iter=run["n_bound_iter"], clip=run["clip"])
    out, st = om.step(alpha, phi, U, 1.0, opts)
    expected = np.array([num(x) for x in run["expected"]])
    assert np.abs(out - expected).max() <= 1e-14, (out, expected)
    assert abs(st["vol_clipped"] - num(run["vol_clipped"])) <= 1e-14, st["vol_clipped"]
    if "n_bound_active" in run:
        assert st["n_bound_active"] == run["n_bound_active"]
    assert abs(st["vol_boundary"] - num(run["vol_boundary"])) <= 1e-14, st["vol_boundary"]
    # the step's volume balance: what is there after is what was there, less what left through
    # the boundary, plus what the chop added
    bal = st["vol_before"] - st["vol_boundary"] + st["vol_clipped"]
    assert abs(st["vol_after"] - bal) <= 1e-14, (st["vol_after"], bal)
    # every cell is flat (equal vertex values), so none is reconstructed
    assert st["n_flat"] == st["n_surface"]


def _single_hex(points8):
    """One hexahedral cell with the given corners in (i, j, k) point order (i fastest)."""
    m = W.hex_block([0, 1], [0, 1], [0, 1], periodic_x=False)
    m.points = np.ascontiguousarray(np.asarray(points8, dtype=np.float64))
    return m


def test_cell_centre_is_the_volume_centroid_of_a_frustum(oracle_lib):
    """A square frustum, base 2x2 at z=0 and top 1x1 at z=1: V = (1/3)(4 + 1 + 2) = 7/3 and the
    centroid height is (A1 + 2 sqrt(A1 A2) + 3 A2) / (4 (A1 + sqrt(A1 A2) + A2)) = 11/28, while the
    mean of the corners sits at 1/2.  The cell centre is the volume centroid (Section 3: x_P of the
    collocated polyhedral control volume)."""
    pts = []
    for k, half in ((0, 1.0), (1, 0.5)):
        for j in (0, 1):
            for i in (0, 1):
                pts.append([(2 * i - 1) * half, (2 * j - 1) * half, float(k)])
    om = oracle_lib.OracleMesh(_single_hex(pts))
    xc, V = om.geometry()
    assert abs(V[0] - 7.0 / 3.0) <= 1e-14
    assert np.abs(xc[0] - np.array([0.0, 0.0, 11.0 / 28.0])).max() <= 1e-14


def test_cell_centre_of_a_ramp(oracle_lib):
    """The unit square extruded up to the plane z = 1 + x: V = 3/2; the centroid is
    x = (1/2 + 1/3)/V = 5/9, y = 1/2, z = (1/2) (1 + 1 + 1/3)/V = 7/9 (the corners' mean is
    (1/2, 1/2, 3/4))."""
    pts = []
    for k in (0, 1):
        for j in (0, 1):
            for i in (0, 1):
                pts.append([float(i), float(j), float(k) * (1.0 + i)])
    om = oracle_lib.OracleMesh(_single_hex(pts))
    xc, V = om.geometry()
    assert abs(V[0] - 1.5) <= 1e-14
    assert np.abs(xc[0] - np.array([5.0 / 9.0, 0.5, 7.0 / 9.0])).max() <= 1e-14


def test_vertex_value_uses_the_volume_centroid(oracle_lib):
    """The unit cube next to the ramp [1,2]x[0,1] under z = x (its low side on the shared face
    x = 1).  The ramp's centroid is (1 + 5/9, 1/2, 7/9) (the ramp of the previous test, moved by 1
    in x), so the shared corner (1, 0, 0) is sqrt(3)/2 from the cube's centre and
    sqrt(25/81 + 1/4 + 49/81) = sqrt(377)/18 from the ramp's; with weights 1/distance the vertex
    value is (0.2 / d0 + 0.7 / d1) / (1 / d0 + 1 / d1).  The corners' mean of the ramp,
    (3/2, 1/2, 3/4), would give another value."""
    m = W.hex_block([0, 1, 2], [0, 1], [0, 1], periodic_x=False)
    P = m.points.copy()
    P[:, 2] = np.where((P[:, 2] == 1.0) & (P[:, 0] == 2.0), 2.0, P[:, 2])
    m.points = np.ascontiguousarray(P)
    om = oracle_lib.OracleMesh(m)
    xc, V = om.geometry()
    assert abs(V[0] - 1.0) <= 1e-14 and abs(V[1] - 1.5) <= 1e-14
    assert np.abs(xc[1] - [14 / 9, 0.5, 7 / 9]).max() <= 1e-14
    a_pts = om.point_values(np.array([0.2, 0.7]))
    p = int(np.nonzero((P[:, 0] == 1.0) & (P[:, 1] == 0.0) & (P[:, 2] == 0.0))[0][0])
    d0, d1 = np.sqrt(3.0) / 2.0, np.sqrt(377.0) / 18.0
    assert abs(a_pts[p] - (0.2 / d0 + 0.7 / d1) / (1 / d0 + 1 / d1)) <= 1e-15
