"""The oracle pins catch plausible mistakes.

Each case applies one textual mutation to a copy of the oracle's C source
(a dropped term, a flipped sign, a wrong normaliser or index, a changed
order), builds it on the CPU, and runs the pins against it: at least one pin
must fail.  The repository's oracle itself is never modified.
"""
import os
import subprocess

import pytest

import tests.test_oracle_kruskal as kpins
import tests.test_oracle_momentum as mpins
import tests.test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "stdecomp_oracle.c")

MUTANTS = {
    "core_drops_lambda": ("double grad = -sum_rh[lin] / (double)m + lam_G * G[lin];",
                          "double grad = -sum_rh[lin] / (double)m;"),
    "core_wrong_average": ("double grad = -sum_rh[lin] / (double)m + lam_G * G[lin];",
                           "double grad = -sum_rh[lin] / (double)(m + 1) + lam_G * G[lin];"),
    "core_residual_sign": ("sum_rh[lin] += r * h;", "sum_rh[lin] -= r * h;"),
    "row_residual_sign": ("F[jn] += -r[p] * E[(int64_t)p * Jn + jn];", "F[jn] += r[p] * E[(int64_t)p * Jn + jn];"),
    "row_normaliser_m": ("a[jn] -= gam_A * (F[jn] / (double)c + lam_A * a[jn]);",
                         "a[jn] -= gam_A * (F[jn] / (double)m + lam_A * a[jn]);"),
    "row_drops_lambda": ("a[jn] -= gam_A * (F[jn] / (double)c + lam_A * a[jn]);",
                         "a[jn] -= gam_A * (F[jn] / (double)c);"),
    "E_wrong_index": ("E[p * Jn + j[n]] += s;", "E[p * Jn + j[0] % Jn] += s;"),
    "E_includes_own_mode": ("if (k != n) s *= row_of", "if (k != n || 1) s *= row_of"),
    "unfold_mode_order": ("for (int k = 0; k < N; k++) {\n        if (k == n) continue;",
                          "for (int k = N - 1; k >= 0; k--) {\n        if (k == n) continue;"),
    "feistel_three_rounds": ("for (int r = 0; r < 4; r++) {\n        uint64_t F = orc_sm64(R ^ key[r]) & mask;",
                             "for (int r = 0; r < 3; r++) {\n        uint64_t F = orc_sm64(R ^ key[r]) & mask;"),
    "segment_order_desc": ("return pa < pb ? -1 : (pa > pb ? 1 : 0);", "return pa < pb ? 1 : (pa > pb ? -1 : 0);"),
    "modes_before_core": ("int rc = orc_core_step(N, dims, ranks, A, G, m, idx, x, gam_G, lam_G);\n    for (int n = 0; rc == ORC_OK && n < N; n++)\n        rc = orc_mode_step(N, dims, ranks, A, G, m, idx, x, n, gam_A, lam_A);",
                          "int rc = ORC_OK;\n    for (int n = 0; rc == ORC_OK && n < N; n++)\n        rc = orc_mode_step(N, dims, ranks, A, G, m, idx, x, n, gam_A, lam_A);\n    if (rc == ORC_OK) rc = orc_core_step(N, dims, ranks, A, G, m, idx, x, gam_G, lam_G);"),
    "ragged_batch_dropped": ("int64_t m = (T - b0 < M) ? (T - b0) : M;\n            for (int64_t p = 0; p < m; p++) {\n                int64_t t = order[b0 + p];\n                for (int k = 0; k < N; k++) bidx[k * m + p] = idx[k * T + t];\n                bx[p] = vals[t];\n            }\n            rc = orc_step(",
                             "int64_t m = M; if (T - b0 < M) break;\n            for (int64_t p = 0; p < m; p++) {\n                int64_t t = order[b0 + p];\n                for (int k = 0; k < N; k++) bidx[k * m + p] = idx[k * T + t];\n                bx[p] = vals[t];\n            }\n            rc = orc_step("),
    # Kruskal core
    "kruskal_drops_lambda": ("Bn[a * R + c] -= gam_B * (V[a] / (double)m + lam_B * Bn[a * R + c]);",
                             "Bn[a * R + c] -= gam_B * (V[a] / (double)m);"),
    "kruskal_wrong_average": ("Bn[a * R + c] -= gam_B * (V[a] / (double)m + lam_B * Bn[a * R + c]);",
                              "Bn[a * R + c] -= gam_B * (V[a] / (double)(m + 1) + lam_B * Bn[a * R + c]);"),
    "kruskal_residual_keeps_own_column": ("                if (r == c) continue;\n", ""),
    "kruskal_stale_C_term": ("for (int b = 0; b < Jn; b++) v += C[a * Jn + b] * Bn[b * R + c];", ""),
    "kruskal_q_includes_own_mode": ("if (k != n) qv *= B[boff[k] + (int64_t)j[k] * R + r];",
                                    "qv *= B[boff[k] + (int64_t)j[k] * R + r];"),
    "kruskal_vec_order": ("const int64_t v = j[n] + (int64_t)Jn * col;", "const int64_t v = col + K * j[n];"),
    "kruskal_modes_reversed": ("for (int n = 0; n < N && rc == ORC_OK; n++)\n        rc = kruskal_columns(",
                               "for (int n = N - 1; n >= 0 && rc == ORC_OK; n--)\n        rc = kruskal_columns("),
    # heavy-ball momentum
    "momentum_row_velocity_not_carried": ("v[jn] = mu * v[jn] + (F[jn] / (double)c + lam_A * a[jn]);",
                                          "v[jn] = (F[jn] / (double)c + lam_A * a[jn]);"),
    "momentum_row_normaliser_m": ("v[jn] = mu * v[jn] + (F[jn] / (double)c + lam_A * a[jn]);",
                                  "v[jn] = mu * v[jn] + (F[jn] / (double)m + lam_A * a[jn]);"),
    "momentum_row_steps_on_gradient": ("a[jn] -= gam_A * v[jn];",
                                       "a[jn] -= gam_A * (F[jn] / (double)c + lam_A * a[jn]);"),
    "momentum_core_velocity_not_carried": ("VG[lin] = mu * VG[lin] + grad;", "VG[lin] = grad;"),
    "momentum_core_velocity_squared_mu": ("VG[lin] = mu * VG[lin] + grad;", "VG[lin] = mu * mu * VG[lin] + grad;"),
    "momentum_core_step_sign": ("G[lin] -= gam_G * VG[lin];", "G[lin] += gam_G * VG[lin];"),
    "kruskal_core_not_formed": ("    if (rc == ORC_OK) rc = orc_kruskal_core(N, ranks, R, B, G);\n    return rc;\n}",
                                "    return rc;\n}"),
}


def _pin_calls():
    return [
        (pins.test_perm_frozen_vectors, {}),
        (pins.test_unfolding_columns_paper_example, {}),
        (pins.test_segments_paper_example, {}),
        (pins.test_predict_matches_dense_tucker, {"dims": (3, 4, 2, 3), "ranks": (2, 1, 2, 3)}),
        (pins.test_unfolding_kronecker_identity, {"n": 1}),
        (pins.test_core_step_is_gradient_of_fC, {"dims": (4, 3, 5), "ranks": (2, 3, 2)}),
        (pins.test_mode_step_is_gradient_of_row_objective, {"n": 0}),
        (pins.test_mode_step_is_gradient_of_row_objective, {"n": 2}),
        (pins.test_step_order_core_then_modes, {}),
        (pins.test_matrix_factorisation_exact, {}),
        (pins.test_run_uses_sampler_and_ragged_last_batch, {}),
        (kpins.test_kruskal_core_is_sum_of_outer_products, {"ranks": (2, 3, 4), "R": 2}),
        (kpins.test_W_closed_form_and_prediction, {"dims": (5, 4, 6), "ranks": (2, 3, 2), "R": 3}),
        (kpins.test_column_step_is_gradient, {"dims": (5, 4, 6), "ranks": (2, 3, 2), "R": 3, "n": 0, "r": 1}),
        (kpins.test_core_step_is_cyclic_over_modes_then_columns, {}),
        (kpins.test_matrix_factorisation_exact_kruskal, {}),
        (kpins.test_kruskal_step_then_factor_steps, {}),
        (mpins.test_mu_zero_is_the_plain_method, {}),
        (mpins.test_heavy_ball_matrix_factorisation_exact, {}),
        (mpins.test_heavy_ball_core_exact, {}),
        (mpins.test_unsampled_rows_keep_row_and_velocity, {}),
    ]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(oracle_mod, tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not found: " + name
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    lib = tmp_path / ("lib_%s.so" % name)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", str(lib), str(mpath), "-lm"])
    oracle_mod.use_library(str(lib))
    failed = []
    try:
        for fn, kw in _pin_calls():
            try:
                fn(oracle_mod, **kw)
            except (AssertionError, oracle_mod.OracleError, ValueError, IndexError):
                failed.append(fn.__name__)
    finally:
        oracle_mod.use_library(None)
    assert failed, "no pin caught mutant " + name
