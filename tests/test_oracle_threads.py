"""The oracle's parallel loops: every result and statistic is bit for bit the same on one thread
and on several (per-cell work is independent, and sums keep the serial cell order)."""
import numpy as np

import wavegen as W


def _run(O, w, steps, threads):
    O.set_threads(threads)
    om = O.OracleMesh(w.mesh)
    a = w.alpha0.copy()
    out = []
    for n in range(steps):
        phi, U = w.phi_U(n)
        a, st, tr = om.step(a, phi, U, w.dt, trace=True)
        out.append((a.copy(), st, tr))
    return out


def test_results_do_not_depend_on_the_thread_count(oracle_lib):
    O = oracle_lib
    before = O.get_threads()
    try:
        for w in (W.violent_3d(nx=24, ny=13, nz=16, steps=3), W.perturbed_box(steps=3),
                  W.airy_slab(64, 32, 16, 0.1, 0.95, 3, "airy_stressed")):
            one = _run(O, w, 3, 1)
            many = _run(O, w, 3, 4)
            for (a1, s1, t1), (a4, s4, t4) in zip(one, many):
                assert np.array_equal(a1, a4), w.name
                assert s1 == s4, (w.name, s1, s4)
                for k in t1:
                    assert np.array_equal(t1[k], t4[k], equal_nan=True), (w.name, k)
            assert sum(s["n_bound_active"] for _, s, _ in one) > 0 or w.name.startswith("perturbed")
    finally:
        O.set_threads(before)
