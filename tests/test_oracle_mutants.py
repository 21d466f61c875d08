"""The pins must catch plausible mistakes in the oracle.

Each case plants one mistake in a temporary copy of ``oracle/mg_oracle.c``
(a dropped term, a wrong sign, a wrong index or operand), builds it on the
CPU, and runs the pin that is meant to catch it against that build; the pin
must fail.  The committed oracle is never modified.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mg_oracle.c")

CF = "tests/test_oracle_closed_forms.py::"
RNG = "tests/test_oracle_rng.py::"
RS = "tests/test_oracle_root_slots.py::"
INV = "tests/test_oracle_invariants.py::"
SEQ = "tests/test_oracle_split_sequences.py::"
SRCS = "tests/test_oracle_sources.py::"
MIR = "tests/test_oracle_mirror.py::"
COEF = "tests/test_oracle_coefficients.py::"
WZ = "tests/test_oracle_wentzell.py::"

MUTANTS = {
    "drift_sign": (
        [("const double mu = drift_at(g, e, x);",
          "const double mu = -drift_at(g, e, x);")],
        CF + "test_linear_drift_ar1_law"),
    "drift_uses_full_dt": (
        [("const double xt = fma(gsd, w, fma(mu, h, x));",
          "const double xt = fma(gsd, w, fma(mu, dt, x));")],
        CF + "test_exit_law_matches_renewal_equation"),
    "diffusion_uses_full_dt": (
        [("const double gsd = sigma_at(g, e, x) * sqrt(h);",
          "const double gsd = sigma_at(g, e, x) * sqrt(dt);")],
        CF + "test_exit_law_matches_renewal_equation"),
    "remaining_time_uses_u": (
        [("h = fma(-alpha, h, h);", "h = fma(-u, h, h);")],
        CF + "test_exit_law_matches_renewal_equation"),
    "term_end_in_init_frame": (
        [("const double A = hit_init ? mu * h : -(mu * h);", "const double A = mu * h;"),
         ("const double B = hit_init ? gsd * w : -(gsd * w);", "const double B = gsd * w;")],
        CF + "test_star_quadratic_potential_stays_stationary"),
    "term_vertex_points_outward": (
        [("else if (x == L) w = -fabs(w);", "else if (x == L) w = fabs(w);")],
        CF + "test_path_graph_with_terminal_entries"),
    "entry_always_at_zero": (
        [("x = g->slot_orient[s] ? g->length[e] : 0.0;", "x = 0.0;")],
        CF + "test_path_graph_with_terminal_entries"),
    "slot_ignores_b": (
        [("if ((uint64_t)r < thr[s]) return s;",
          "if ((uint64_t)r < ((((uint64_t)(s - s0 + 1)) << 32) / (uint64_t)(s1 - s0))) return s;")],
        RS + "test_slot_draw_frequencies_in_simulation"),
    "box_muller_scale": (
        [("double r = sqrt(-2.0 * log(u1));", "double r = sqrt(-log(u1));")],
        RNG + "test_main_normals_standard_normal"),
    "main_normal_reused": (
        [("return (n & 1u) ? ws : wc;", "return wc;")],
        RNG + "test_main_normals_independent_across_steps"),
    "hit_draw_reused": (
        [("hit_draw(p, n, (uint32_t)k, tag, seed, &r, &w_next);",
          "hit_draw(p, n, 1u, tag, seed, &r, &w_next);")],
        CF + "test_exit_law_matches_renewal_equation"),
    "exit_counted_every_hit": (
        [("if (k >= 1 && alive) cnt->exit_slot[last_slot]++;", "(void)0;"),
         ("last_slot = s;\n", "last_slot = s;\n      cnt->exit_slot[s]++;\n")],
        CF + "test_exit_law_matches_renewal_equation"),
    "absorption_ignored": (
        [("if (killed || (g->vtx_kind && g->vtx_kind[v] == 1)) {", "if (killed) {")],
        CF + "test_absorbing_vertex_survival"),
    "philox_multiplier": (
        [("#define OR_PHILOX_M1 0xCD9E8D57u", "#define OR_PHILOX_M1 0xCD9E8D59u")],
        RNG + "test_philox_matches_rocrand"),
    "philox_key_schedule": (
        [("if (round > 0) {", "if (round > 1) {")],
        RNG + "test_philox_matches_rocrand"),
    "histogram_ignores_span": (
        [("const double inv = (double)nb / g->bin_span[e];", "const double inv = (double)nb;")],
        INV + "test_mass_histogram_and_hits_consistency"),
    "root_takes_larger": (
        [("u = lo > 0.0 ? lo : hi;", "u = hi;")],
        RS + "test_root_random_well_conditioned"),
    "init_position_not_scaled": (
        [("x[i] = g->length[e] * unit_open(o[1]);", "x[i] = unit_open(o[1]);")],
        INV + "test_init_laws"),
    "vertex_normal_not_folded": (
        [("if (x == 0.0) w = fabs(w);", "if (0) w = fabs(w);")],
        CF + "test_first_vertex_substep_closed_form"),
    "remaining_time_kept": (
        [("h = fma(-alpha, h, h);", "h = h;")],
        SEQ + "test_split_sequences_match_exact_law"),
    "source_slot_from_source_word": (
        [("const int32_t s = pick_slot(g, thr, v, o[1]);",
          "const int32_t s = pick_slot(g, thr, v, o[0]);")],
        SRCS + "test_sources_law"),
    "drift_cubic_term_dropped": (
        [("return coef(g->drift_c2, g->drift_c3, e, g->drift_a[e], g->drift_c[e], x);",
          "return coef(g->drift_c2, NULL, e, g->drift_a[e], g->drift_c[e], x);")],
        COEF + "test_one_step_gaussian_with_frozen_coefficients"),
    "sigma_frozen_at_edge_start": (
        [("const double gsd = sigma_at(g, e, x) * sqrt(h);",
          "const double gsd = sigma_at(g, e, 0.0) * sqrt(h);")],
        COEF + "test_one_step_gaussian_with_frozen_coefficients"),
    "sigma_linear_term_dropped": (
        [("const double s1 = g->sigma_c1 ? g->sigma_c1[e] : 0.0;", "const double s1 = 0.0;")],
        COEF + "test_stationary_law_with_cubic_drift_and_diffusion"),
    "mirror_skipped": (
        [("if (g->vtx_kind && g->vtx_kind[v] == 2) {", "if (0) {")],
        MIR + "test_one_step_is_the_folded_normal"),
    "mirror_far_image_wrong": (
        [("const double xr = hit_init ? -xt : 2.0 * L - xt;",
          "const double xr = hit_init ? -xt : L - xt;")],
        MIR + "test_one_step_is_the_folded_normal"),
    "mirror_image_not_checked": (
        [("if (xr > 0.0 && xr < L) {", "if (xr > 0.0) {")],
        MIR + "test_image_outside_the_edge_splits"),
    "wentzell_gamma_unnormalised": (
        [("wz->gamma[v] = (g->vtx_sticky ? g->vtx_sticky[v] : 0.0) / beta;",
          "wz->gamma[v] = (g->vtx_sticky ? g->vtx_sticky[v] : 0.0);")],
        WZ + "test_sticky_halfline_from_vertex"),
    "wentzell_kill_ignores_move": (
        [("lt = o + c * sqrt(h);", "lt = o;")],
        WZ + "test_robin_segment_survival"),
    "wentzell_overshoot_dropped": (
        [("const double o = hit_init ? -xt : xt - L;", "const double o = 0.0;")],
        WZ + "test_robin_segment_survival"),
    "wentzell_sigma_v_ignored": (
        [("sig += (g->slot_jump_prob[s] / beta) * sigma_at(g, e, at);",
          "sig += g->slot_jump_prob[s] / beta;")],
        WZ + "test_killing_halfline_from_vertex"),
    "wentzell_owed_dropped": (
        [("*owed = gam * o - h;", "*owed = 0.0;")],
        WZ + "test_sticky_halfline_from_vertex"),
    "wentzell_move_stay_dropped": (
        [("const double b = gam * c, r = h - gam * o;", "const double b = 0.0, r = h - gam * o;")],
        WZ + "test_sticky_star_stationary_atom"),
    "table_derivative_unscaled": (
        [("return h00 * v[k0 + j] + h10 * h * d[k0 + j] + h01 * v[k0 + j + 1] + h11 * h * d[k0 + j + 1];",
          "return h00 * v[k0 + j] + h10 * d[k0 + j] + h01 * v[k0 + j + 1] + h11 * d[k0 + j + 1];")],
        COEF + "test_table_of_a_cubic_is_the_cubic"),
    "table_coordinate_in_length_units": (
        [("const double t = s - (double)j;", "const double t = x - (double)j * h;")],
        COEF + "test_table_of_a_cubic_is_the_cubic"),
    "table_basis_swapped": (
        [("const double h10 = t3 - 2.0 * t2 + t;", "const double h10 = t3 - t2;"),
         ("const double h11 = t3 - t2;", "const double h11 = t3 - 2.0 * t2 + t;")],
        COEF + "test_table_stationary_law_of_non_polynomial_coefficients"),
    "far_end_not_checked": (
        [("if (xt > 0.0 && xt < L) {", "if (xt > 0.0) {")],
        CF + "test_radial_reflected_heat_kernel_converges"),
}


def _run_mutant(name, tmpdir):
    edits, target = MUTANTS[name]
    src = open(SRC).read()
    for old, new in edits:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    cfile = os.path.join(tmpdir, f"{name}.c")
    so = os.path.join(tmpdir, f"{name}.so")
    with open(cfile, "w") as f:
        f.write(src)
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                    "-shared", "-o", so, cfile, "-lm"], check=True, capture_output=True)
    env = dict(os.environ, MG_ORACLE_LIB=so, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", target, "-x", "-q",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


@pytest.fixture(scope="module")
def mutant_results():
    with tempfile.TemporaryDirectory() as d:
        with ThreadPoolExecutor(max_workers=4) as ex:
            futs = {n: ex.submit(_run_mutant, n, d) for n in MUTANTS}
            yield {n: f.result() for n, f in futs.items()}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pin_catches_mutant(name, mutant_results):
    rc, out = mutant_results[name]
    # pytest exit code 1 = a test failed (not a crash or a collection error)
    assert rc == 1, f"mutant {name} survived its pin (rc={rc}):\n{out}"
