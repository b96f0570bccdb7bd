"""The pins must be able to fail: plant plausible mistakes in a copy of the oracle, on the CPU,
and check that the pin suite rejects every one of them."""
import os
import subprocess
import sys

import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (name, snippet of the oracle, planted mistake); every snippet must occur exactly once
MUTANTS = [
    ("idw_inverse_square", "double w = 1.0 / v_norm(e);", "double w = 1.0 / v_dot(e, e);"),
    ("cut_from_wrong_end", "double lam = (iso - aw) / (ad - aw);", "double lam = (iso - ad) / (aw - ad);"),
    ("printed_aplus2", "return sw->c1 + sw->c2 * (1.0 - q * q);",
     "return sw->c1 + sw->c2 * (1.0 - (1.0 - q) * (1.0 - q));"),
    ("first_piece_integral_factor", "I += sw->c1 * (b - a) * (ra * ra + ra * rb + rb * rb) / 3.0;",
     "I += sw->c1 * (b - a) * (ra * ra + ra * rb + rb * rb) / 2.0;"),
    ("no_dry_fraction_for_receding_plane", "return un > 0 ? I : dt - I;", "return I;"),
    ("update_sign", "sum += m->ce_sign[e] * dV[m->ce_flux[e]];", "sum -= m->ce_sign[e] * dV[m->ce_flux[e]];"),
    ("bulk_flux_ignores_alpha", "dV[fid] = alpha[c] * ph * dt;", "dV[fid] = ph * dt;"),
    ("x41_ratio_inverted", "double r = (sw->t2 - sw->t1) / (sw->t3 - sw->t1);",
     "double r = (sw->t3 - sw->t1) / (sw->t2 - sw->t1);"),
    ("equal_triangle_weights", "double Ai = 0.5 * v_norm(cr);", "double Ai = 0.5;"),
    ("isoface_centre_is_vertex_mean", "for (int d = 0; d < 3; ++d) out->xS[d] = xs[d] / wsum;",
     "for (int d = 0; d < 3; ++d) out->xS[d] = o[d] + 0.0 * xs[d] / wsum;"),
    ("isoface_edges_reversed",
     "for (int d = 0; d < 3; ++d) { seg_a[nseg][d] = cp[d]; seg_b[nseg][d] = last_exit[d]; }",
     "for (int d = 0; d < 3; ++d) { seg_b[nseg][d] = cp[d]; seg_a[nseg][d] = last_exit[d]; }"),
    ("isoface_apex_mean_of_cut_points", "perimeter_centroid(seg_a, seg_b, nseg, 0, o);",
     "perimeter_centroid(seg_a, seg_a, nseg, 0, o);"),
    ("velocity_components_swapped", "double Uc[3] = {U[c], U[nc + c], U[2 * nc + c]};",
     "double Uc[3] = {U[c], U[2 * nc + c], U[nc + c]};"),
    ("cell_point_face_value_not_mean", "for (int d = 0; d < 3; ++d) Uf[d] /= n;",
     "for (int d = 0; d < 3; ++d) Uf[d] /= n + 1;"),
    ("cell_point_centre_carries_face_value", "out[d] = l0 * Up[d] + l1 * Uf[d]", "out[d] = l0 * Uf[d] + l1 * Uf[d]"),
    ("cell_point_tet_least_inside", "if (mn > best) {", "if (-mn > best) {"),
]

# planted mistakes in the tangent of the step, which its own pins must reject
TANGENT_MUTANTS = [
    ("tangent_isovalue_fixed", "return x + (-g_dot / g_x) * OR_CSTEP * _Complex_I;", "return x;"),
    ("tangent_volume_target_sign", "double g_dot = cimag(cut.vsub / m->V[c] - alpha_c) / OR_CSTEP;",
     "double g_dot = cimag(cut.vsub / m->V[c] + alpha_c) / OR_CSTEP;"),
    ("tangent_bounding_need_sign", "cplx need = over ? (a - 1.0) * m->V[c] : -a * m->V[c];",
     "cplx need = over ? (1.0 - a) * m->V[c] : -a * m->V[c];"),
]

# planted mistakes in the ghost-fluid face data (Eqs. 12-20), which its own pins must reject
GFM_MUTANTS = [
    ("gfm_jump_sign_as_printed", "double H = (rho_heavy - rho_light) * v_dot(g, xG);",
     "double H = (rho_light - rho_heavy) * v_dot(g, xG);"),
    ("gfm_lambda_from_neighbour", "double lam = (aP - 0.5) / (aP - aN);", "double lam = (aN - 0.5) / (aN - aP);"),
    ("gfm_weight_from_owner", "double lw = wetP ? lam : 1.0 - lam;", "double lw = lam;"),
    ("gfm_beta_weights_swapped", "double bw = lw * bm + (1.0 - lw) * bp;", "double bw = lw * bp + (1.0 - lw) * bm;"),
    ("gfm_cyclic_translation_sign", "for (int d = 0; d < 3; ++d) xN[d] -= m->ptrans[3 * p + d];",
     "for (int d = 0; d < 3; ++d) xN[d] += m->ptrans[3 * p + d];"),
    ("gfm_ghosts_on_wrong_cells", "ghost_nbr[f] = wetP ? to_dry : to_wet;", "ghost_nbr[f] = wetP ? to_wet : to_dry;"),
    ("gfm_mirror_jump_sign", "+ (bp / bw) * H;  /* its mirror */", "- (bp / bw) * H;  /* its mirror */"),
]

# planted mistakes in the relaxation-zone blending, which its own pins must reject
RELAX_MUTANTS = [
    ("relax_exponent_three", "return 1.0 - (exp(pow(chi, 3.5)) - 1.0) / (exp(1.0) - 1.0);",
     "return 1.0 - (exp(pow(chi, 3.0)) - 1.0) / (exp(1.0) - 1.0);"),
    ("relax_normalised_by_e", "return 1.0 - (exp(pow(chi, 3.5)) - 1.0) / (exp(1.0) - 1.0);",
     "return 1.0 - (exp(pow(chi, 3.5)) - 1.0) / exp(1.0);"),
    ("relax_blend_reversed", "out[c] = w * alpha[c] + (1.0 - w) * target[c];",
     "out[c] = w * target[c] + (1.0 - w) * alpha[c];"),
    ("relax_direction_not_normalised", "e[3] = {d[0] / n, d[1] / n, d[2] / n}", "e[3] = {d[0], d[1], d[2]}"),
    ("relax_overlap_accepted", "if (hit >= 0) return -1;", "if (hit >= 0) continue;"),
]

# mistakes that only cells other than hexahedra show: checked against the pins on tetrahedra,
# prisms, pyramids and merged polyhedra
POLY_MUTANTS = [
    ("face_walk_wraparound_pair_dropped", "if (pending && first_is_entry) {", "if (0 && pending && first_is_entry) {"),
    ("face_fan_about_first_point",
     "double x9[9] = {ap[0], ap[1], ap[2], p0[0], p0[1], p0[2], p1[0], p1[1], p1[2]};",
     "double x9[9] = {m->P[3 * fp[0]], m->P[3 * fp[0] + 1], m->P[3 * fp[0] + 2], p0[0], p0[1], p0[2], p1[0], p1[1], p1[2]};"),
]


# planted mistakes in the bounding step (R13), the inflow boundary value (R11), the round-off chop
# and the cell centre (the volume centroid), which the hand-derived channel states and the closed
# forms of tests/test_oracle_bounding.py must reject.  A snippet may be a list of (old, new) pairs,
# and "*" before old replaces every occurrence of it (the two capacity loops of a sweep).
BOUNDING_MUTANTS = [
    ("excess_capacity_is_outflow_volume", "*double cap = over ? outphi * dt - outv : outv;",
     "double cap = over ? outv : outv;"),
    ("redistribution_ratio_uncapped", "if (r > 1.0) r = 1.0;", "if (0) r = 1.0;"),
    ("excess_spread_equally", [("if (cap > 0) sumcap += cap;", "if (cap > 0) sumcap += 1.0;"),
                               ("double d = cap * r;", "double d = fmin(cap, need / sumcap);")], None),
    ("first_sweep_halved", "double d = cap * r;", "double d = cap * r * (it == 0 ? 0.5 : 1.0);"),
    ("capacity_sum_doubled", "if (cap > 0) sumcap += cap;", "if (cap > 0) sumcap += 2.0 * cap;"),
    ("inflow_alpha_dropped", "dV[fid] = m->palpha[p] * ph * dt;", "dV[fid] = 0.0 * m->palpha[p] * ph * dt;"),
    ("cell_centre_is_vertex_mean", "for (int d = 0; d < 3; ++d) m->xc[3 * c + d] = mom[d] / vol;",
     "for (int d = 0; d < 3; ++d) m->xc[3 * c + d] = xr[d] + 0.0 * mom[d] / vol;"),
    ("roundoff_tolerance_raised", "double tol = opt->bound_tol;", "double tol = 1e-6 + 0.0 * opt->bound_tol;"),
    ("boundary_volume_before_redistribution", "s.vol_boundary += m->ce_sign[e] * dVc[m->ce_flux[e]];",
     "s.vol_boundary += m->ce_sign[e] * dV[m->ce_flux[e]];"),
]

TANGENT_HEADER = "Tangent of the step (directional derivative"


def _plant(name, old, new, tangent):
    """The oracle source with `old` replaced by `new` in the step (before the tangent section) or
    in the tangent section, where the snippet must occur exactly once (every occurrence, and at
    least one, if it starts with "*").  `old` may also be a list of (old, new) pairs."""
    src = open(O.SRC).read()
    cut = src.index(TANGENT_HEADER)
    head, tail = src[:cut], src[cut:]
    part = tail if tangent else head
    pairs = old if isinstance(old, list) else [(old, new)]
    for o, n in pairs:
        every = o.startswith("*")
        o = o[1:] if every else o
        k = part.count(o)
        assert (k >= 1 if every else k == 1), f"snippet for mutant {name} no longer matches the oracle"
        part = part.replace(o, n)
    return head + part if tangent else part + tail


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_reject_planted_mistake(tmp_path, name, old, new):
    mutant_src = tmp_path / "mutant.c"
    mutant_src.write_text(_plant(name, old, new, tangent=False))
    lib = O.compile_oracle(str(mutant_src), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, ISOADV_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name,old,new", POLY_MUTANTS, ids=[m[0] for m in POLY_MUTANTS])
def test_poly_pins_reject_planted_mistake(tmp_path, name, old, new):
    mutant_src = tmp_path / "mutant.c"
    mutant_src.write_text(_plant(name, old, new, tangent=False))
    lib = O.compile_oracle(str(mutant_src), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, ISOADV_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_poly.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name,old,new", TANGENT_MUTANTS, ids=[m[0] for m in TANGENT_MUTANTS])
def test_tangent_pins_reject_planted_mistake(tmp_path, name, old, new):
    mutant_src = tmp_path / "mutant.c"
    mutant_src.write_text(_plant(name, old, new, tangent=True))
    lib = O.compile_oracle(str(mutant_src), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, ISOADV_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_tlm.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name,old,new", GFM_MUTANTS, ids=[m[0] for m in GFM_MUTANTS])
def test_gfm_pins_reject_planted_mistake(tmp_path, name, old, new):
    mutant_src = tmp_path / "mutant.c"
    mutant_src.write_text(_plant(name, old, new, tangent=False))
    lib = O.compile_oracle(str(mutant_src), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, ISOADV_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_gfm.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name,old,new", RELAX_MUTANTS, ids=[m[0] for m in RELAX_MUTANTS])
def test_relax_pins_reject_planted_mistake(tmp_path, name, old, new):
    mutant_src = tmp_path / "mutant.c"
    mutant_src.write_text(_plant(name, old, new, tangent=False))
    lib = O.compile_oracle(str(mutant_src), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, ISOADV_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_relax.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name,old,new", BOUNDING_MUTANTS, ids=[m[0] for m in BOUNDING_MUTANTS])
def test_bounding_pins_reject_planted_mistake(tmp_path, name, old, new):
    mutant_src = tmp_path / "mutant.c"
    mutant_src.write_text(_plant(name, old, new, tangent=False))
    lib = O.compile_oracle(str(mutant_src), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, ISOADV_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_bounding.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
