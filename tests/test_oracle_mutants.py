"""Every plausible mistake planted in a copy of the oracle must trip at least
one pin.  Each mutant is the oracle's C source with one textual edit (a wrong
sign, a dropped term, a transposed operand, a wrong index), compiled with the
oracle's own flags into a temporary library; the pins then run against it.
Planted mistakes live only in these temporary copies, on the CPU."""
import os

import pytest

import oracle
import pins

MUTATIONS = {
    "update_sign": ("y[i] = y[i] - colk[i] * xk", "y[i] = y[i] + colk[i] * xk"),
    "dropped_alpha": ("y[i] = alpha * y[i];", "y[i] = y[i];"),
    "transposed_L": ("y[i] = y[i] - colk[i] * xk", "y[i] = y[i] - A[k + i * lda] * xk"),
    "skipped_subdiagonal": ("for (int64_t i = k + 1; i < m; ++i) y[i] = y[i] - colk[i] * xk;",
                            "for (int64_t i = k + 2; i < m; ++i) y[i] = y[i] - colk[i] * xk;"),
    "wrong_diag_index": ("y[k] = y[k] / A[k + k * lda];", "y[k] = y[k] / A[k + (k > 0 ? k - 1 : 0) * lda + (k > 0)];"),
    "diag_multiplied": ("y[k] = y[k] / A[k + k * lda];", "y[k] = y[k] * A[k + k * lda];"),
    "unit_diag_read": ("if (!unit) y[k] = y[k] / A[k + k * lda];", "y[k] = y[k] / A[k + k * lda];"),
    "alpha_zero_reads_inputs": ("    if (alpha == 0.0) {\n        for (int64_t j = 0; j < n; ++j)\n            for (int64_t i = 0; i < m; ++i) B[i + j * ldb] = 0.0;\n        return;\n    }\n#pragma omp parallel for schedule(dynamic, 1)\n    for (int64_t j = 0; j < n; ++j)\n        d_solve_column",
                                "#pragma omp parallel for schedule(dynamic, 1)\n    for (int64_t j = 0; j < n; ++j)\n        d_solve_column"),
    "complex_mul_sign": ("*cr = ar * br - ai * bi;", "*cr = ar * br + ai * bi;"),
    "complex_mul_swap": ("*ci = ar * bi + ai * br;", "*ci = ar * br + ai * bi;"),
    "complex_div_conj": ("const double ni = xi * dr - xr * di;", "const double ni = xi * dr + xr * di;"),
    "complex_div_modulus": ("const double den = dr * dr + di * di;", "const double den = dr * dr - di * di;"),
    "complex_update_imag": ("y[2 * i + 1] = y[2 * i + 1] - pi;", "y[2 * i + 1] = y[2 * i + 1] + pi;"),
    "complex_L_conjugated": ("z_mul(colk[2 * i], colk[2 * i + 1], xr, xi, &pr, &pi);",
                             "z_mul(colk[2 * i], -colk[2 * i + 1], xr, xi, &pr, &pi);"),
    "complex_alpha_conj": ("z_mul(alpha[0], alpha[1], y[2 * i], y[2 * i + 1], &r, &s);",
                           "z_mul(alpha[0], -alpha[1], y[2 * i], y[2 * i + 1], &r, &s);"),
    "rowform_index": ("for (int64_t k = 0; k < i; ++k) s = s - A[i + k * lda] * x[k];",
                      "for (int64_t k = 0; k < i; ++k) s = s - A[k + i * lda] * x[k];"),
    "residual_alpha_sign": ("dot2_add_prod(&acc, -alpha, B0[i + j * ldb]);",
                            "dot2_add_prod(&acc, alpha, B0[i + j * ldb]);"),
    "residual_dropped_diag": ("dot2_add_prod(&acc, unit ? 1.0 : A[i + i * lda], x[i]);", ""),
    "norm_of_X_wrong": ("d_norm_inf_lower(unit, m, A, lda) * d_norm_inf_general(m, n, X, ldx)",
                        "d_norm_inf_lower(unit, m, A, lda) * d_norm_inf_general(m, n, B0, ldb)"),
    # the general solver (either side, either triangle, op(A) = A, A^T, A^H)
    "general_transpose_ignored": ("return trans ? A[c + r * lda] : A[r + c * lda];",
                                  "return A[r + c * lda];"),
    "general_conj_dropped": ("*im = trans == 2 ? -a[1] : a[1];", "*im = a[1];"),
    "general_upper_rule": ("return (uplo == 1) == (trans == 0);", "return uplo == 1;"),
    "general_left_direction": ("const int64_t i = upper ? m - 1 - t : t;\n                double s",
                               "const int64_t i = upper ? t : m - 1 - t;\n                double s"),
    "general_right_direction": ("const int64_t j = upper ? t : n - 1 - t;\n                double s",
                                "const int64_t j = upper ? n - 1 - t : t;\n                double s"),
    "general_right_operand_index": ("s = s - B[i + k * ldb] * d_op(trans, A, lda, k, j);",
                                    "s = s - B[i + k * ldb] * d_op(trans, A, lda, j, k);"),
    "general_unit_read": ("x[i] = unit ? s : s / d_op(trans, A, lda, i, i);",
                          "x[i] = s / d_op(trans, A, lda, i, i);"),
    "general_left_skips_last": ("for (int64_t k = i + 1; k < m; ++k) s = s - d_op(trans, A, lda, i, k) * x[k];",
                                "for (int64_t k = i + 2; k < m; ++k) s = s - d_op(trans, A, lda, i, k) * x[k];"),
    "general_z_right_update_sign": ("                    sr = sr - pr;\n                    si = si - pi;\n                }\n                if (unit) {\n                    b[0] = sr;",
                                    "                    sr = sr + pr;\n                    si = si - pi;\n                }\n                if (unit) {\n                    b[0] = sr;"),
    "general_z_alpha_conj": ("z_mul(alpha[0], alpha[1], b[0], b[1], &sr, &si);",
                             "z_mul(alpha[0], -alpha[1], b[0], b[1], &sr, &si);"),
    "general_residual_right_index": ("OPEL(k, j, ar, ai);", "OPEL(j, k, ar, ai);"),
    "general_residual_conj": ("dot2_add_prod(&im, ai, xr);\n                }", "dot2_add_prod(&im, -ai, xr);\n                }"),
    "general_norm_of_op": ("s += cx ? hypot(ar, ai) : fabs(ar);", "s += cx ? hypot(ar, ai) : ar;"),
    # the Cholesky factorization
    "cholesky_pivot_sign": ("for (int64_t k = 0; k < j; ++k) s = s - A[j + k * lda] * A[j + k * lda];",
                            "for (int64_t k = 0; k < j; ++k) s = s + A[j + k * lda] * A[j + k * lda];"),
    "cholesky_row_index": ("for (int64_t k = 0; k < j; ++k) t = t - A[i + k * lda] * A[j + k * lda];",
                           "for (int64_t k = 0; k < j; ++k) t = t - A[i + k * lda] * A[i + k * lda];"),
    "cholesky_no_sqrt": ("const double d = sqrt(s);\n        A[j + j * lda] = d;",
                         "const double d = s;\n        A[j + j * lda] = d;"),
    "cholesky_conj_dropped": ("z_mul(a[0], a[1], b[0], -b[1], &pr, &pi);",
                              "z_mul(a[0], a[1], b[0], b[1], &pr, &pi);"),
    "cholesky_info_off_by_one": ("if (!(s > 0.0)) return (int)(j + 1);\n        const double d = sqrt(s);\n        A[j + j * lda] = d;\n        for",
                                 "if (!(s > 0.0)) return (int)(j);\n        const double d = sqrt(s);\n        A[j + j * lda] = d;\n        for"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTATIONS[name]
    src = oracle.source_text()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutated = src.replace(old, new, 1)
    so = oracle.compile_variant(mutated, os.path.join(str(tmp_path), f"mut_{name}.so"))
    orc = oracle.OracleLib(so)
    failed = []
    for pin in pins.ALL_PINS:
        try:
            pin(orc)
        except (AssertionError, ValueError, FloatingPointError):
            failed.append(pin.__name__)
            break               # caught; the remaining pins need not run
    assert failed, f"no pin catches the planted mistake {name}"
