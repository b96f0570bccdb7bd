"""Pins of the oracle's relaxation-zone blending (reading R17) against what fixes it independently
of its formula: the weight keeps the computed solution at a zone's inner edge and imposes the
target at its outer edge, leaves the inner edge like chi^3.5 / (e - 1) (measured from the weight's
values, not retyped), decreases monotonically, and the blend acts only on the cells whose centres
lie in a zone, as a convex combination."""
import math

import numpy as np
import pytest

import wavegen as W


def test_weight_end_points(oracle_lib):
    assert oracle_lib.relax_weight(0.0) == 1.0
    assert abs(oracle_lib.relax_weight(1.0)) <= 1e-16


def test_weight_leaves_the_inner_edge_like_a_power(oracle_lib):
    """Slope of log(1 - w) against log chi near 0 is the exponent, and (1 - w)(e - 1) / chi^p -> 1
    fixes the normalisation."""
    c1, c2 = 1e-3, 2e-3
    d1, d2 = 1.0 - oracle_lib.relax_weight(c1), 1.0 - oracle_lib.relax_weight(c2)
    p = math.log(d2 / d1) / math.log(c2 / c1)
    assert abs(p - 3.5) <= 1e-6, p
    assert abs(d1 * (math.e - 1.0) / c1 ** p - 1.0) <= 1e-6


def test_weight_is_monotone(oracle_lib):
    chi = np.linspace(0.0, 1.0, 2001)
    w = np.array([oracle_lib.relax_weight(c) for c in chi])
    assert np.all(np.diff(w) < 0.0) and w.min() >= 0.0 and w.max() <= 1.0


def _row_mesh(nx=40):
    xs = np.linspace(0.0, 5.0, nx + 1)  # centres at 0.0625 + 0.125 i
    return W.hex_block(xs, [0.0, 0.125, 0.25], [0.0, 0.125], periodic_x=False), xs


def test_blend_acts_on_zone_cells_only(oracle_lib):
    """Two zones at the ends of a row, pointing outwards: alpha = 1, target = 0 gives the weight at
    each zone cell's coordinate, 1 at the inner edge, the target at the outer edge, and alpha
    everywhere else."""
    mesh, xs = _row_mesh()
    x = mesh.cell_centres_structured()[:, 0]
    om = oracle_lib.OracleMesh(mesh)
    # left zone from the centre 1.0625 down to just past the centre 0.0625; right zone from 3.9375
    # up to just past 4.9375 (a centre exactly on an outer edge would sit on the zone's boundary)
    L = 1.0 + 1e-6
    zones = [((1.0625, 0.0, 0.0), (-2.0, 0.0, 0.0), L), ((3.9375, 0.3, 0.1), (1.0, 0.0, 0.0), L)]
    one = np.ones(mesh.n_cells)
    out = om.relax_blend(zones, one, np.zeros(mesh.n_cells))
    chi = np.where(x <= 2.5, 1.0625 - x, x - 3.9375) / L
    inside = (chi > 1e-9) & (chi < 1.0)
    outside = chi < -1e-9
    assert inside.sum() == 2 * 8 * 2 and outside.sum() == (40 - 18) * 2
    assert np.array_equal(out[outside], one[outside])
    ref = np.array([oracle_lib.relax_weight(c) for c in chi[inside]])
    assert np.abs(out[inside] - ref).max() <= 1e-12
    assert np.abs(out[np.isclose(x, 0.0625)]).max() <= 1e-4  # close to the target at the outer edge
    assert np.abs(out[np.isclose(x, 4.9375)]).max() <= 1e-4
    assert np.abs(out[np.isclose(x, 1.0625)] - 1.0).max() <= 1e-12  # alpha, at the inner edge
    assert np.abs(out[np.isclose(x, 3.9375)] - 1.0).max() <= 1e-12


def test_blend_is_a_convex_combination(oracle_lib):
    mesh, _ = _row_mesh()
    rng = np.random.default_rng(3)
    a, t = rng.uniform(0, 1, mesh.n_cells), rng.uniform(0, 1, mesh.n_cells)
    om = oracle_lib.OracleMesh(mesh)
    zones = [((0.0, 0.0, 0.0), (1.0, 0.0, 0.0), 5.0)]
    out = om.relax_blend(zones, a, t)
    lo, hi = np.minimum(a, t), np.maximum(a, t)
    assert np.all(out >= lo - 1e-16) and np.all(out <= hi + 1e-16)
    # the direction's length does not matter
    out2 = om.relax_blend([((0.0, 0.0, 0.0), (4.0, 0.0, 0.0), 5.0)], a, t)
    assert np.array_equal(out, out2)
    # swapping alpha and target mirrors the weight: out(a, t) + out(t, a) = a + t
    out3 = om.relax_blend(zones, t, a)
    assert np.abs(out + out3 - (a + t)).max() <= 1e-15
    # near the inner edge the result leans to alpha, near the outer edge to the target
    first, last = 0, 39
    assert abs(out[first] - a[first]) < abs(out[first] - t[first])
    assert abs(out[last] - t[last]) < abs(out[last] - a[last])


def test_invalid_zones(oracle_lib):
    mesh, _ = _row_mesh()
    om = oracle_lib.OracleMesh(mesh)
    a = np.zeros(mesh.n_cells)
    for zones in ([((0, 0, 0), (0, 0, 0), 1.0)], [((0, 0, 0), (1, 0, 0), 0.0)],
                  [((0, 0, 0), (1, 0, 0), 1.0), ((1.5, 0, 0), (-1, 0, 0), 1.0)]):
        with pytest.raises(ValueError):
            om.relax_blend(zones, a, a)
