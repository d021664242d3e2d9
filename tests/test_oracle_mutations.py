"""The oracle's pins must catch plausible mistakes (CPU only).

Each case plants one mistake in a copy of the oracle's C source, builds it in
a temporary directory, points the oracle wrapper at it and runs the pin that
should catch it; the pin must fail.  Nothing here touches the GPU.
"""
import ctypes
import os
import subprocess
import tempfile

import pytest

import oracle
from tests import test_oracle_pins as pins
from tests import test_oracle_replay as rp

SRC = os.path.join(os.path.dirname(oracle.__file__), "pulda_oracle.c")

MUTATIONS = [
    # (name, original text, planted mistake, pins that must fail)
    ("philox_wrong_half", "uint32_t n0 = hi1 ^ c1 ^ k0;", "uint32_t n0 = hi0 ^ c1 ^ k0;",
     [pins.test_philox_matches_rocrand]),
    ("vose_residual", "p[g] = (p[g] + p[s]) - 1.0;", "p[g] = p[g] - p[s];",
     [lambda: pins.test_vose_induced_law("random")]),
    ("poisson_support_short", "ceil(lam + 10.0 * sqrt(lam) + 10.0)", "ceil(lam + 1.0 * sqrt(lam) + 1.0)",
     [pins.test_pois_tables_exact_law]),
    ("gaussian_no_rounding", "floor(lam + sqrt(lam) * g + 0.5)", "floor(lam + sqrt(lam) * g)",
     [lambda: pins.test_rounded_gaussian_closed_form(150)]),
    ("prior_rate_inverted", "double e = -log(1.0 - u53(r[0], r[1])) / bv;",
     "double e = -log(1.0 - u53(r[0], r[1])) * (1.0 / (2.0 * bv));",
     [pins.test_prior_marks_binomial_and_uniform]),
    ("prior_marks_overwrite_counted", "if (n[(size_t)pos * V + v] == 0) gam[(size_t)pos * V + v] = x;",
     "if (1) gam[(size_t)pos * V + v] = x;",
     [pins.test_prior_marks_ignore_counted_cells]),
    ("no_alpha_part", "double sa = M->sigma_a[v];", "double sa = 0.0;",
     [lambda: pins.test_token_law_enumeration("overlap")]),
    ("b_part_transposed", "double b = (double)M->phi[(size_t)k * V + v] * (double)m[k];\n        if (b > 0.0) {\n            c += b;\n            last = k;",
     "double b = (double)M->phi[(size_t)k * V + (v + 1) % V] * (double)m[k];\n        if (b > 0.0) {\n            c += b;\n            last = k;",
     [lambda: pins.test_token_law_enumeration("overlap")]),
    ("token_not_removed", "if (--m[kold] == 0) kd--;", "(void)0;",
     [pins.test_within_document_chain_stationary_law]),
    ("loglik_sign", "word -= lgamma((double)nk[k] + Vb);", "word += lgamma((double)nk[k] + Vb);",
     [pins.test_loglik_independent_evaluation, pins.test_loglik_closed_form_uniform_priors]),
    ("foldin_theta_no_prior", "theta[k] = (float)(((double)acc[k] / (double)(S - burn_in) + alpha[k])",
     "theta[k] = (float)(((double)acc[k] / (double)(S - burn_in))",
     [pins.test_foldin_outputs_definition]),
    ("gamma_d_offset", "const double d = a1 - 1.0 / 3.0;", "const double d = a1 - 1.0 / 2.0;",
     [lambda: pins.test_gamma_draw_law(2.5)]),
    ("gamma_boost_power", "exp(log(u32o(boost)) / a)", "exp(log(u32o(boost)) * a)",
     [lambda: pins.test_gamma_draw_law(0.3)]),
    ("gamma_normal_variance", "sqrt(-2.0 * log(u32o(r[0])))", "sqrt(-1.0 * log(u32o(r[0])))",
     [lambda: pins.test_gamma_draw_law(2.5)]),
    ("dirichlet_shape_prior", "or_gamma_draw((beta_v ? beta_v[v] : beta) + (double)n[",
     "or_gamma_draw((beta_v ? beta_v[v] : 2.0 * beta) + (double)n[",
     [lambda: pins.test_phi_dirichlet_moments(0.5)]),
    ("dirichlet_row_sum_skips", "double s = 0.0;\n        for (int32_t v = 0; v < V; v++) s += gam[",
     "double s = 0.0;\n        for (int32_t v = 1; v < V; v++) s += gam[",
     [lambda: pins.test_phi_dirichlet_moments(0.5)]),
    ("ltr_no_redraws", "for (int32_t q = 0; q < n; q++) {\n                mr[zr[q]]--;",
     "for (int32_t q = 0; q < 0; q++) {\n                mr[zr[q]]--;",
     [pins.test_ltr_third_token_expectation]),
    ("ltr_token_kept_in_counts", "                mr[zr[q]]--;\n                draw4(seed, (uint32_t)q,",
     "                draw4(seed, (uint32_t)q,",
     [pins.test_ltr_third_token_expectation]),
    ("ltr_denominator", "sum += Z / ((double)n + A);", "sum += Z / ((double)n + 1.0 + A);",
     [pins.test_ltr_single_token_closed_form]),
    ("vector_mark_not_added", "else if (beta_v) gam[(size_t)pos * V + v] += x;",
     "else if (0) gam[(size_t)pos * V + v] += x;",
     [pins.test_vector_beta_cell_law]),
    ("vector_tables_keep_beta", "const double tb = beta_v ? 0.0 : beta;", "const double tb = beta;",
     [pins.test_vector_beta_cell_law]),
    ("vector_loglik_prior_sum", "for (int32_t v = 0; v < V; v++) Vb += beta_v[v];",
     "for (int32_t v = 0; v < V; v++) Vb += beta;",
     [pins.test_vector_beta_loglik_and_dirichlet]),
    ("replay_wrong_scale", "double rel = dist / Z;", "double rel = dist / sa;",
     [lambda: rp.test_replay_constructed_tie("b"), lambda: rp.test_replay_constructed_tie("a")]),
    ("replay_every_mismatch_a_tie", "if (rel <= tol) out[1]++;", "if (1) out[1]++;",
     [rp.test_replay_wrong_neighbour_far_from_boundary_is_bad, rp.test_replay_wrong_topic_is_bad]),
    ("replay_interval_counts_token", "double b = (double)phi[(size_t)k * V + v] * (double)m[k];\n                if (b > 0.0) {\n                    lo = c;",
     "double b = (double)phi[(size_t)k * V + v] * (double)(m[k] + (k == kold));\n                if (b > 0.0) {\n                    lo = c;",
     [lambda: rp.test_replay_constructed_tie("b")]),
    ("replay_interval_upper_edge", "double dd = x < lo ? lo - x : (x >= c ? x - c : 0.0);",
     "double dd = x < lo ? lo - x : 0.0;",
     [rp.test_replay_wrong_neighbour_far_from_boundary_is_bad]),
    ("sparse_column_descending", "for (int64_t e = c0; e < c0 + nv; e++) {\n                        int32_t k = topic[e];",
     "for (int64_t e = c0 + nv - 1; e >= c0; e--) {\n                        int32_t k = topic[e];",
     [lambda: rp.test_sparse_mode_bit_identical(300, 500, 400, 0.6)]),
    ("sparse_list_insert_unsorted", "while (j > 0 && lst[j - 1] > knew) { lst[j] = lst[j - 1]; j--; }",
     "(void)0;",
     [lambda: rp.test_sparse_mode_bit_identical(50, 200, 60, 0.3)]),
    ("normalise_wrong_row", "phi[(size_t)k * V + v] = g > 0 ? (float)((double)g / (double)s) : 0.0f;",
     "phi[(size_t)k * V + v] = g > 0 ? (float)((double)g / (double)(s + 1)) : 0.0f;",
     [pins.test_phi_normalise_definition]),
]


@pytest.mark.parametrize("name,old,new,checks", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_mutation(name, old, new, checks, monkeypatch):
    src = open(SRC).read()
    assert old in src, name
    d = tempfile.mkdtemp(prefix="oracle_mut_")
    c_path = os.path.join(d, "m.c")
    so_path = os.path.join(d, "m.so")
    with open(c_path, "w") as f:
        f.write(src.replace(old, new, 1))
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", so_path, c_path, "-lm"])
    lib = ctypes.CDLL(so_path)
    oracle._declare(lib)
    monkeypatch.setattr(oracle, "_lib", lib)
    for check in checks:
        with pytest.raises(AssertionError):
            check()
