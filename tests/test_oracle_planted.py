"""Planted mistakes: each mutation of the oracle source must make some pin fail.

The mutated copy is compiled into a temporary directory on the CPU; the oracle
source itself is never modified.
"""
import os
import tempfile

import pytest

import oracle
import test_oracle_pins as P

MUTATIONS = [
    ("getrf update sign",
     "for (int i = j + 1; i < n; ++i) EL(A, lda, i, c) -= EL(A, lda, i, j) * u;",
     "for (int i = j + 1; i < n; ++i) EL(A, lda, i, c) += EL(A, lda, i, j) * u;",
     [P.test_getrf_matches_lapack]),
    ("fig4 line 13 and->or",
     "if (delta > tol && delta > tol * fmax",
     "if (delta > tol || delta > tol * fmax",
     [P.test_likely_sympd_conditions]),
    ("fig4 line 15 >= -> >",
     "if (fabs(a_ij) >= max_diag) return 0;",
     "if (fabs(a_ij) > max_diag) return 0;",
     [P.test_likely_sympd_conditions]),
    ("fig4 line 15 tests the upper element",
     "if (fabs(a_ij) >= max_diag) return 0;",
     "if (fabs(a_ji) >= max_diag) return 0;",
     [P.test_likely_sympd_conditions]),
    ("fig4 line 16 >= -> >",
     "if ((fabs(a_ij) + fabs(a_ji)) >= (EL(A, lda, i, i) + EL(A, lda, j, j))) return 0;",
     "if ((fabs(a_ij) + fabs(a_ji)) > (EL(A, lda, i, i) + EL(A, lda, j, j))) return 0;",
     [P.test_likely_sympd_conditions]),
    ("band scan off by one",
     "if (last >= 0 && last - j > kl) kl = last - j;\n  }\n  *kl_out",
     "if (last >= 0 && last - j > kl) kl = last - j + 1;\n  }\n  *kl_out",
     [P.test_band_scan_all_4x4_patterns]),
    ("25% rule equality",
     "return 4 * nnz <= n * n;",
     "return 4 * nnz < n * n;",
     [P.test_band_rule_counts_positions_exactly]),
    ("trsv transposed operand",
     "  if (lower_system) {\n    for (int i = 0; i < n; ++i) {\n      double s = x[i];\n      for (int j = 0; j < i; ++j) {\n        const double a = trans ? EL(T, ldt, j, i) : EL(T, ldt, i, j);",
     "  if (lower_system) {\n    for (int i = 0; i < n; ++i) {\n      double s = x[i];\n      for (int j = 0; j < i; ++j) {\n        const double a = trans ? EL(T, ldt, i, j) : EL(T, ldt, j, i);",
     [P.test_trsv_matches_lapack]),
    ("potrf skips the diagonal update",
     "for (int i = c; i < n; ++i) EL(A, lda, i, c) -= EL(A, lda, i, j) * l_cj;",
     "for (int i = c + 1; i < n; ++i) EL(A, lda, i, c) -= EL(A, lda, i, j) * l_cj;",
     [P.test_potrf_matches_lapack_and_failure_column]),
    ("gbtrf fill extent too short",
     "const int ju = imin(n - 1, j + kl + ku);",
     "const int ju = imin(n - 1, j + ku);",
     [P.test_band_lu_equals_dense_lu]),
    ("estimator uses inv(A) where inv(A)^T is due",
     "  apply(ctx, 2, x); ++ns;\n  {\n    int j = iamax(n, x);",
     "  apply(ctx, 1, x); ++ns;\n  {\n    int j = iamax(n, x);",
     [P.test_rcond_against_lapack_estimators]),
    ("rcond drops the matrix norm",
     "return (1.0 / ainvnm) / anorm;",
     "return (1.0 / ainvnm);",
     [P.test_rcond_is_lower_bound_and_close]),
    ("getrs transposed solves in the wrong order",
     "      orc_trsv(1, 1, 0, n, LU, lda, b);\n      orc_trsv(0, 1, 1, n, LU, lda, b);",
     "      orc_trsv(0, 1, 1, n, LU, lda, b);\n      orc_trsv(1, 1, 0, n, LU, lda, b);",
     [P.test_getrf_matches_lapack]),
    ("jacobi rotation sign",
     "EL(U, ldu, i, p) = c * up - s * uq;",
     "EL(U, ldu, i, p) = c * up + s * uq;",
     [P.test_jacobi_prescribed_singular_values]),
    ("svd truncation level",
     "const double cut = ORC_EPS * smax;",
     "const double cut = 1e-3 * smax;",
     [P.test_svd_lstsq_min_norm_matches_lapack]),
    ("rule <= instead of <",
     "  if (failed) res->fallback = 1;\n  else if (res->rcond != res->rcond) res->fallback = 3;\n  else if (res->rcond < thr) res->fallback = 2;\n  if (res->fallback) {\n    if (no_approx) {",
     "  if (failed) res->fallback = 1;\n  else if (res->rcond != res->rcond) res->fallback = 3;\n  else if (res->rcond <= thr) res->fallback = 2;\n  if (res->fallback) {\n    if (no_approx) {",
     [P.test_rule_threshold_is_half_eps]),
    ("berr drops ||b||",
     "  const double den = anorm_inf * xn + bn;\n  return den > 0.0",
     "  const double den = anorm_inf * xn;\n  return den > 0.0",
     [P.test_berr_definition]),
    ("berr residual drops the low part of the products",
     "*lo = al * bl - (((*hi - ah * bh) - al * bh) - ah * bl);",
     "*lo = 0.0;",
     [P.test_berr_exact_rational]),
    ("berr residual drops the summation's compensation",
     "    for (int i = 0; i < n; ++i) r[i] = acc[i].s + acc[i].c;",
     "    for (int i = 0; i < n; ++i) r[i] = acc[i].s;",
     [P.test_berr_exact_rational]),
    ("band berr reads the wrong band row",
     "exact_product(AB[(size_t)(ku + i - j) + (size_t)j * ldab], x[j], &hi, &lo);",
     "exact_product(AB[(size_t)(ku + j - i) + (size_t)j * ldab], x[j], &hi, &lo);",
     [P.test_berr_band_hand_and_against_dense]),
    ("bunch-kaufman alpha", "BK_ALPHA = 0.64038820320220756872767623199676;", "BK_ALPHA = 0.5;",
     [P.test_sytrf_bk_matches_lapack_ldl, P.test_sytrf_bk_pivot_rules_by_hand]),
    ("bunch-kaufman rowmax takes the diagonal",
     "if (i != r && fabs(EL(S, n, r, i)) > rowmax)",
     "if (fabs(EL(S, n, r, i)) > rowmax)",
     [P.test_sytrf_bk_matches_lapack_ldl, P.test_sytrf_bk_pivot_rules_by_hand]),
    ("bunch-kaufman interchange leaves the formed L rows",
     "      for (int c = 0; c < j; ++c) {\n        const double t = EL(A, lda, swap_from, c);",
     "      for (int c = 0; c < 0; ++c) {\n        const double t = EL(A, lda, swap_from, c);",
     [P.test_sytrf_bk_factorisation_identities]),
    ("bunch-kaufman 2x2 inverse sign",
     "EL(A, lda, i, j) = (s0 * c2 - s1 * b) / det;",
     "EL(A, lda, i, j) = (s0 * c2 + s1 * b) / det;",
     [P.test_sytrf_bk_factorisation_identities]),
    ("sytrs skips the 2x2 coupling",
     "y[j] = (c2 * y0 - bb * y1) / det;",
     "y[j] = (c2 * y0) / det;",
     [P.test_sytrs_and_rcond_sym_against_lapack]),
    ("gttrf drops the second super-diagonal",
     "du2[i] = du[i + 1];",
     "du2[i] = 0.0;",
     [P.test_gttrf_matches_lapack_bitwise]),
    ("gttrs transposed L step",
     "          b[i + 1] = b[i] - dl[i] * t;",
     "          b[i + 1] = b[i] + dl[i] * t;",
     [P.test_gttrs_both_directions_and_rcond]),
]


@pytest.mark.parametrize("name,old,new,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, old, new, pins):
    src = open(oracle.SRC_PATH).read()
    assert src.count(old) == 1, f"mutation anchor not unique: {name}"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mut.c")
        with open(path, "w") as f:
            f.write(src.replace(old, new))
        hdr = os.path.join(os.path.dirname(oracle.SRC_PATH), "ada_oracle.h")
        with open(os.path.join(d, "ada_oracle.h"), "w") as f:
            f.write(open(hdr).read())
        so = oracle.build(src=path, out=os.path.join(d, "libmut.so"))
        mutant = oracle.Oracle(so)
        caught = False
        for pin in pins:
            try:
                pin(o=mutant)
            except (AssertionError, Exception):
                caught = True
        assert caught, f"no pin caught the planted mistake: {name}"
