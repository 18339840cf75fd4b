/*
 * sanitize_check.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A driver that runs the oracle's public entry points over every class, route and option on small
 * deterministic inputs, built with AddressSanitizer and UndefinedBehaviorSanitizer by the CPU test
 * suite: any out-of-bounds access, use of freed memory, signed overflow or similar in the oracle
 * ends the run with a report and a non-zero status. The inputs come from a 64-bit linear
 * congruential generator (Knuth's MMIX constants), so every run sees the same matrices.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ada_oracle.h"

static unsigned long long g_state = 88172645463325252ull;
static double unif(void) { /* uniform in [-1, 1) */
  g_state = g_state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(g_state >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

enum { DENSE, SPD, UPPER, LOWER, BANDED, SYMINDEF, RANKDEF, NKIND };

static void make(int kind, int n, double* A) {
  memset(A, 0, sizeof(double) * n * n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      double v = unif();
      switch (kind) {
        case UPPER: if (i > j) v = 0.0; break;
        case LOWER: if (i < j) v = 0.0; break;
        case BANDED: if (i - j > 2 || j - i > 1) v = 0.0; break;
        default: break;
      }
      A[i + j * n] = v;
    }
  if (kind == SPD || kind == SYMINDEF) {
    for (int j = 0; j < n; ++j)
      for (int i = j + 1; i < n; ++i) A[j + i * n] = A[i + j * n];
  }
  for (int i = 0; i < n; ++i) {
    if (kind == SPD) A[i + i * n] = fabs(A[i + i * n]) + n;
    else if (kind == SYMINDEF) A[i + i * n] = (i & 1) ? 0.01 : 0.02;
    else if (kind != RANKDEF) A[i + i * n] += (A[i + i * n] >= 0 ? 4.0 : -4.0);
  }
  if (kind == RANKDEF && n > 1) /* two equal columns: exactly singular, the fallback must run */
    for (int i = 0; i < n; ++i) A[i + (n - 1) * n] = A[i];
}

/* lstsq: the system is inconsistent (rank deficient), so only a finite backward error is asked for */
static int check(const char* what, int n, const orc_result_t* r, int lstsq) {
  if (r->status != ORC_OK && r->status != ORC_ERR_SINGULAR) {
    fprintf(stderr, "%s n=%d: status %d\n", what, n, r->status);
    return 1;
  }
  if (r->status == ORC_OK && !(lstsq ? isfinite(r->berr) : r->berr <= 1e-8)) {
    fprintf(stderr, "%s n=%d: backward error %g\n", what, n, r->berr);
    return 1;
  }
  return 0;
}

int main(void) {
  static const int sizes[] = {1, 2, 3, 5, 17, 40};
  int bad = 0;
  for (size_t s = 0; s < sizeof(sizes) / sizeof(sizes[0]); ++s) {
    const int n = sizes[s], nrhs = 3;
    double* A = malloc(sizeof(double) * n * n);
    double* B = malloc(sizeof(double) * n * nrhs);
    double* X = malloc(sizeof(double) * n * nrhs);
    for (int kind = 0; kind < NKIND; ++kind) {
      make(kind, n, A);
      for (int e = 0; e < n * nrhs; ++e) B[e] = unif();
      orc_result_t r;
      orc_solve(n, nrhs, A, n, B, n, X, n, 0, -1.0, 0, &r);
      bad |= check("solve", n, &r, kind == RANKDEF);
      orc_solve(n, nrhs, A, n, B, n, X, n, 0, -1.0, 1, &r);
      bad |= check("solve force_general", n, &r, kind == RANKDEF);
      orc_solve(n, nrhs, A, n, B, n, X, n, 1, -1.0, 0, &r);
      bad |= check("solve no_approx", n, &r, kind == RANKDEF);
      orc_solve_ext(n, nrhs, A, n, B, n, X, n, 0, -1.0, 0, ORC_EXT_SYM | ORC_EXT_TRIDIAG, &r);
      bad |= check("solve_ext", n, &r, kind == RANKDEF);
      orc_detect_t d;
      orc_detect(n, A, n, &d);
      if (kind == BANDED && n >= 3) { /* the same matrix in band layout, kl = 2, ku = 1, ldab = 5 */
        const int kl = 2, ku = 1, ldab = kl + ku + 2;
        double* AB = calloc((size_t)ldab * n, sizeof(double));
        for (int j = 0; j < n; ++j)
          for (int i = j - ku; i <= j + kl; ++i)
            if (i >= 0 && i < n) AB[ku + i - j + j * ldab] = A[i + j * n];
        orc_solve_band(n, kl, ku, nrhs, AB, ldab, B, n, X, n, 0, -1.0, 4096, &r);
        bad |= check("solve_band", n, &r, 0);
        orc_solve_band_ext(n, kl, ku, nrhs, AB, ldab, B, n, X, n, 0, -1.0, 4096, ORC_EXT_TRIDIAG, &r);
        bad |= check("solve_band_ext", n, &r, 0);
        const double eb = orc_berr_band(n, kl, ku, nrhs, AB, ldab, B, n, X, n);
        bad |= !(eb >= 0.0);
        free(AB);
      }
    }
    /* a non-finite input is reported, not solved */
    A[0] = NAN;
    orc_result_t r;
    orc_solve(n, nrhs, A, n, B, n, X, n, 0, -1.0, 0, &r);
    bad |= r.status != ORC_ERR_NONFINITE;
    free(A);
    free(B);
    free(X);
  }
  printf(bad ? "FAILED\n" : "OK\n");
  return bad;
}
