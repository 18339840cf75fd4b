/*
 * ada_oracle.c -- TEST INFRASTRUCTURE ONLY (see ada_oracle.h).
 *
 * Plain FP64 reference of the adaptive solver of Sanderson & Curtin,
 * arXiv 2007.11208. Every routine states the passage of the paper it follows.
 * No LAPACK/BLAS is linked; loops are written out. OpenMP is used only to run
 * independent columns (or right-hand sides) of one step side by side, which
 * does not change any arithmetic.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared -o libada_oracle.so ada_oracle.c -lm
 */
#include "ada_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EL(M, ld, i, j) (M)[(size_t)(i) + (size_t)(j) * (size_t)(ld)]

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int imin(int a, int b) { return a < b ? a : b; }
static int imax(int a, int b) { return a > b ? a : b; }

/* machine epsilon: gap between 1 and the next double (Section II-C footnote) */
static const double ORC_EPS = DBL_EPSILON;

/* ======================================================================
 * Section II-A: band-width scan over a column-major matrix.
 * For every column j the rows from the top down to the diagonal are walked
 * and the first non-zero row r gives j - r super-diagonals; the rows from the
 * diagonal down to the bottom are walked and the last non-zero row r gives
 * r - j sub-diagonals. The widths are the maxima over all columns. A column
 * with no non-zero in a half contributes 0. "Non-zero" is the IEEE test
 * a != 0 (so -0.0 counts as zero).
 * ==================================================================== */
void orc_band_scan(int n, const double* A, int lda, int* kl_out, int* ku_out) {
  int kl = 0, ku = 0;
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i <= j; ++i) {
      if (EL(A, lda, i, j) != 0.0) {
        if (j - i > ku) ku = j - i;
        break;
      }
    }
    int last = -1;
    for (int i = j; i < n; ++i)
      if (EL(A, lda, i, j) != 0.0) last = i;
    if (last >= 0 && last - j > kl) kl = last - j;
  }
  *kl_out = kl;
  *ku_out = ku;
}

/* Section II-A: the matrix is deemed non-banded once the band implied by kl/ku
 * holds more than 25% of the n*n elements. The band holds exactly
 * n(kl+ku+1) - kl(kl+1)/2 - ku(ku+1)/2 positions; equality counts as banded. */
int orc_is_banded(int64_t n, int64_t kl, int64_t ku) {
  int64_t nnz = n * (kl + ku + 1) - kl * (kl + 1) / 2 - ku * (ku + 1) / 2;
  return 4 * nnz <= n * n;
}

/* Fig. 4 (Section II-C): likely_sympd, transcribed in the paper's order with
 * its early returns. tol = 100*eps. */
int orc_likely_sympd(int n, const double* A, int lda) {
  const double tol = 100.0 * ORC_EPS;
  double max_diag = 0.0;
  for (int j = 0; j < n; ++j) {
    const double d = EL(A, lda, j, j);
    if (d <= 0.0) return 0;
    if (d > max_diag) max_diag = d;
  }
  for (int j = 0; j + 1 < n; ++j) {
    for (int i = j + 1; i < n; ++i) {
      const double a_ij = EL(A, lda, i, j);
      const double a_ji = EL(A, lda, j, i);
      const double delta = fabs(a_ij - a_ji);
      if (delta > tol && delta > tol * fmax(fabs(a_ij), fabs(a_ji))) return 0;
      if (fabs(a_ij) >= max_diag) return 0;
      if ((fabs(a_ij) + fabs(a_ji)) >= (EL(A, lda, i, i) + EL(A, lda, j, j))) return 0;
    }
  }
  return 1;
}

/* Section II: detection order banded -> upper/lower triangular -> sympd,
 * first match wins. A diagonal matrix that is not banded (n <= 3) is both
 * upper and lower triangular; upper is taken first. */
void orc_detect(int n, const double* A, int lda, orc_detect_t* out) {
  int kl, ku;
  orc_band_scan(n, A, lda, &kl, &ku);
  out->kl = kl;
  out->ku = ku;
  out->banded = orc_is_banded(n, kl, ku);
  out->likely_sympd = 0;
  if (out->banded) { out->cls = ORC_BANDED; return; }
  if (kl == 0) { out->cls = ORC_TRI_UPPER; return; }
  if (ku == 0) { out->cls = ORC_TRI_LOWER; return; }
  out->likely_sympd = orc_likely_sympd(n, A, lda);
  out->cls = out->likely_sympd ? ORC_SYMPD : ORC_GENERAL;
}

/* ======================================================================
 * Section II-D: LU with partial pivoting, A = P L U, L unit lower.
 * Right-looking elimination; the pivot is the first row holding the largest
 * modulus in the current column. An exact zero pivot records info (first
 * such column, 1-based) and the column is skipped.
 * ==================================================================== */
int orc_getrf(int n, double* A, int lda, int* ipiv) {
  int info = 0;
  for (int j = 0; j < n; ++j) {
    int p = j;
    double best = fabs(EL(A, lda, j, j));
    for (int i = j + 1; i < n; ++i) {
      const double v = fabs(EL(A, lda, i, j));
      if (v > best) { best = v; p = i; }
    }
    ipiv[j] = p;
    if (EL(A, lda, p, j) == 0.0) {
      if (info == 0) info = j + 1;
      continue;
    }
    if (p != j) {
      for (int c = 0; c < n; ++c) {
        const double t = EL(A, lda, j, c);
        EL(A, lda, j, c) = EL(A, lda, p, c);
        EL(A, lda, p, c) = t;
      }
    }
    const double piv = EL(A, lda, j, j);
    for (int i = j + 1; i < n; ++i) EL(A, lda, i, j) /= piv;
#pragma omp parallel for schedule(static) if (n - j > 256)
    for (int c = j + 1; c < n; ++c) {
      const double u = EL(A, lda, j, c);
      for (int i = j + 1; i < n; ++i) EL(A, lda, i, c) -= EL(A, lda, i, j) * u;
    }
  }
  return info;
}

/* Triangular substitution, eq. (3) of Section II-B and its mirror image.
 * upper/trans pick the system: T x = b or T^T x = b; unit means an implicit
 * unit diagonal. Each x_i is b_i minus the already-known terms, divided by
 * the diagonal entry. */
void orc_trsv(int upper, int trans, int unit, int n, const double* T, int ldt, double* x) {
  const int lower_system = (!upper && !trans) || (upper && trans); /* effective matrix is lower */
  if (lower_system) {
    for (int i = 0; i < n; ++i) {
      double s = x[i];
      for (int j = 0; j < i; ++j) {
        const double a = trans ? EL(T, ldt, j, i) : EL(T, ldt, i, j);
        s -= a * x[j];
      }
      x[i] = unit ? s : s / EL(T, ldt, i, i);
    }
  } else {
    for (int i = n - 1; i >= 0; --i) {
      double s = x[i];
      for (int j = i + 1; j < n; ++j) {
        const double a = trans ? EL(T, ldt, j, i) : EL(T, ldt, i, j);
        s -= a * x[j];
      }
      x[i] = unit ? s : s / EL(T, ldt, i, i);
    }
  }
}

/* Section II-D, eq. (4): solve with the LU factors. trans=0: A x = b is
 * L y = P b then U x = y. trans=1: A^T x = b is U^T z = b, L^T w = z, x = P^T w. */
void orc_getrs(int trans, int n, int nrhs, const double* LU, int lda, const int* ipiv, double* B, int ldb) {
#pragma omp parallel for schedule(static) if (nrhs > 1)
  for (int r = 0; r < nrhs; ++r) {
    double* b = B + (size_t)r * ldb;
    if (!trans) {
      for (int j = 0; j < n; ++j) {
        const int p = ipiv[j];
        if (p != j) { const double t = b[j]; b[j] = b[p]; b[p] = t; }
      }
      orc_trsv(0, 0, 1, n, LU, lda, b);
      orc_trsv(1, 0, 0, n, LU, lda, b);
    } else {
      orc_trsv(1, 1, 0, n, LU, lda, b);
      orc_trsv(0, 1, 1, n, LU, lda, b);
      for (int j = n - 1; j >= 0; --j) {
        const int p = ipiv[j];
        if (p != j) { const double t = b[j]; b[j] = b[p]; b[p] = t; }
      }
    }
  }
}

/* Section II-C: Cholesky A = L L^T from the lower triangle. The factorisation
 * fails (the matrix is then taken not to be sympd) when a pivot
 * A_jj - sum_k L_jk^2 is not positive or is NaN; info = j+1. */
int orc_potrf_lower(int n, double* A, int lda) {
  for (int j = 0; j < n; ++j) {
    double d = EL(A, lda, j, j);
    if (!(d > 0.0)) return j + 1;
    d = sqrt(d);
    EL(A, lda, j, j) = d;
    for (int i = j + 1; i < n; ++i) EL(A, lda, i, j) /= d;
#pragma omp parallel for schedule(static) if (n - j > 256)
    for (int c = j + 1; c < n; ++c) {
      const double l_cj = EL(A, lda, c, j);
      for (int i = c; i < n; ++i) EL(A, lda, i, c) -= EL(A, lda, i, j) * l_cj;
    }
  }
  return 0;
}

void orc_potrs_lower(int n, int nrhs, const double* L, int lda, double* B, int ldb) {
#pragma omp parallel for schedule(static) if (nrhs > 1)
  for (int r = 0; r < nrhs; ++r) {
    double* b = B + (size_t)r * ldb;
    orc_trsv(0, 0, 0, n, L, lda, b);
    orc_trsv(0, 1, 0, n, L, lda, b);
  }
}

/* ======================================================================
 * Section II-A: banded LU with partial pivoting in the compact band format
 * (each diagonal one row of a dense array, plus kl rows of room for the
 * fill that row interchanges create). Element (i,j) lives at
 * AB[kl+ku+i-j + j*ldab], ldab >= 2kl+ku+1, and the top kl rows start zero.
 * The pivot is searched among the kl+1 rows at and below the diagonal.
 * ==================================================================== */
#define BND(i, j) AB[(size_t)(kl + ku + (i) - (j)) + (size_t)(j) * (size_t)ldab]
#define BNDC(i, j) AB[(size_t)(kl + ku + (i) - (j)) + (size_t)(j) * (size_t)ldab]

int orc_gbtrf(int n, int kl, int ku, double* AB, int ldab, int* ipiv) {
  int info = 0;
  for (int j = 0; j < n; ++j) {
    const int lm = imin(kl, n - 1 - j);
    int p = j;
    double best = fabs(BND(j, j));
    for (int i = j + 1; i <= j + lm; ++i) {
      const double v = fabs(BND(i, j));
      if (v > best) { best = v; p = i; }
    }
    ipiv[j] = p;
    if (BND(p, j) == 0.0) {
      if (info == 0) info = j + 1;
      continue;
    }
    const int ju = imin(n - 1, j + kl + ku);
    if (p != j) {
      for (int c = j; c <= ju; ++c) {
        const double t = BND(j, c);
        BND(j, c) = BND(p, c);
        BND(p, c) = t;
      }
    }
    const double piv = BND(j, j);
    for (int i = j + 1; i <= j + lm; ++i) BND(i, j) /= piv;
    for (int c = j + 1; c <= ju; ++c) {
      const double u = BND(j, c);
      for (int i = j + 1; i <= j + lm; ++i) BND(i, c) -= BND(i, j) * u;
    }
  }
  return info;
}

void orc_gbtrs(int trans, int n, int kl, int ku, int nrhs, const double* AB, int ldab, const int* ipiv,
               double* B, int ldb) {
  const int kd = kl + ku; /* U has kl+ku super-diagonals after interchanges */
#pragma omp parallel for schedule(static) if (nrhs > 1)
  for (int r = 0; r < nrhs; ++r) {
    double* b = B + (size_t)r * ldb;
    if (!trans) {
      for (int j = 0; j + 1 < n; ++j) {
        const int lm = imin(kl, n - 1 - j);
        const int p = ipiv[j];
        if (p != j) { const double t = b[j]; b[j] = b[p]; b[p] = t; }
        for (int i = j + 1; i <= j + lm; ++i) b[i] -= BNDC(i, j) * b[j];
      }
      for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int j = i + 1; j <= imin(n - 1, i + kd); ++j) s -= BNDC(i, j) * b[j];
        b[i] = s / BNDC(i, i);
      }
    } else {
      for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int j = imax(0, i - kd); j < i; ++j) s -= BNDC(j, i) * b[j];
        b[i] = s / BNDC(i, i);
      }
      for (int j = n - 2; j >= 0; --j) {
        const int lm = imin(kl, n - 1 - j);
        double s = b[j];
        for (int i = j + 1; i <= j + lm; ++i) s -= BNDC(i, j) * b[i];
        b[j] = s;
        const int p = ipiv[j];
        if (p != j) { const double t = b[j]; b[j] = b[p]; b[p] = t; }
      }
    }
  }
}

/* ======================================================================
 * 1-norms (maximum absolute column sum) of the original matrix, as the
 * condition estimate of each route needs.
 * ==================================================================== */
double orc_norm1_general(int n, const double* A, int lda) {
  double best = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += fabs(EL(A, lda, i, j));
    if (s > best || s != s) best = s;
  }
  return best;
}

double orc_norm1_tri(int upper, int n, const double* A, int lda) {
  double best = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    if (upper)
      for (int i = 0; i <= j; ++i) s += fabs(EL(A, lda, i, j));
    else
      for (int i = j; i < n; ++i) s += fabs(EL(A, lda, i, j));
    if (s > best || s != s) best = s;
  }
  return best;
}

double orc_norm1_sym_lower(int n, const double* A, int lda) {
  double best = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = 0; i < j; ++i) s += fabs(EL(A, lda, j, i));
    for (int i = j; i < n; ++i) s += fabs(EL(A, lda, i, j));
    if (s > best || s != s) best = s;
  }
  return best;
}

double orc_norm1_band(int n, int kl, int ku, const double* AB, int ldab, int off) {
  double best = 0.0;
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = imax(0, j - ku); i <= imin(n - 1, j + kl); ++i) s += fabs(AB[(size_t)(off + i - j) + (size_t)j * ldab]);
    if (s > best || s != s) best = s;
  }
  return best;
}

/* ======================================================================
 * Reciprocal condition number (Section II: every solver estimates it).
 * The 1-norm of inv(A) is estimated with Hager's method as refined by Higham
 * (ACM TOMS 14(4), 1988): at most five iterations of the sign-vector / unit-
 * vector power step, stopping on a repeated sign vector, on no growth of the
 * estimate, or when the previous index still attains the maximum; then the
 * alternating vector x_i = (-1)^i (1 + i/(n-1)) gives a second lower bound
 * 2||inv(A) x||_1 / (3n). sign(0) = +1; argmax ties go to the lowest index.
 * ==================================================================== */
static double asum(int n, const double* x) {
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += fabs(x[i]);
  return s;
}
static int iamax(int n, const double* x) {
  int j = 0;
  double b = fabs(x[0]);
  for (int i = 1; i < n; ++i)
    if (fabs(x[i]) > b) { b = fabs(x[i]); j = i; }
  return j;
}
static double sgn(double v) { return v >= 0.0 ? 1.0 : -1.0; }

double orc_inv_norm1_est(int n, orc_apply_fn apply, void* ctx, int* nsolves) {
  int ns = 0;
  double* x = (double*)malloc(sizeof(double) * (size_t)n);
  double* xi = (double*)malloc(sizeof(double) * (size_t)n);
  double est;
  for (int i = 0; i < n; ++i) x[i] = 1.0 / n;
  apply(ctx, 1, x); ++ns;
  if (n == 1) {
    est = fabs(x[0]);
    goto done;
  }
  est = asum(n, x);
  for (int i = 0; i < n; ++i) xi[i] = sgn(x[i]);
  for (int i = 0; i < n; ++i) x[i] = xi[i];
  apply(ctx, 2, x); ++ns;
  {
    int j = iamax(n, x);
    int iter = 2;
    for (;;) {
      for (int i = 0; i < n; ++i) x[i] = 0.0;
      x[j] = 1.0;
      apply(ctx, 1, x); ++ns;
      const double est_old = est;
      est = asum(n, x);
      int same = 1;
      for (int i = 0; i < n; ++i)
        if (sgn(x[i]) != xi[i]) { same = 0; break; }
      if (same) break;
      if (est <= est_old) break;
      for (int i = 0; i < n; ++i) xi[i] = sgn(x[i]);
      for (int i = 0; i < n; ++i) x[i] = xi[i];
      apply(ctx, 2, x); ++ns;
      const int jlast = j;
      j = iamax(n, x);
      if (fabs(x[jlast]) != fabs(x[j]) && iter < 5) {
        ++iter;
        continue;
      }
      break;
    }
  }
  /* alternating-sign test vector */
  for (int i = 0; i < n; ++i) x[i] = (i % 2 ? -1.0 : 1.0) * (1.0 + (double)i / (double)(n - 1));
  apply(ctx, 1, x); ++ns;
  {
    const double temp = 2.0 * (asum(n, x) / (3.0 * n));
    if (temp > est) est = temp;
  }
done:
  free(x);
  free(xi);
  if (nsolves) *nsolves = ns;
  return est;
}

static double rcond_from(double anorm, double ainvnm) {
  if (anorm == 0.0) return 0.0;
  if (ainvnm != ainvnm) return ainvnm; /* NaN propagates */
  if (ainvnm == 0.0) return 0.0;
  return (1.0 / ainvnm) / anorm;
}

typedef struct { int n; const double* LU; int lda; const int* ipiv; } ge_ctx;
static void ge_apply(void* c, int kase, double* x) {
  ge_ctx* g = (ge_ctx*)c;
  orc_getrs(kase == 2, g->n, 1, g->LU, g->lda, g->ipiv, x, g->n);
}
double orc_rcond_general(int n, const double* LU, int lda, const int* ipiv, double anorm, int* nsolves) {
  ge_ctx g = {n, LU, lda, ipiv};
  if (anorm == 0.0) { if (nsolves) *nsolves = 0; return 0.0; }
  return rcond_from(anorm, orc_inv_norm1_est(n, ge_apply, &g, nsolves));
}

typedef struct { int n; const double* L; int lda; } po_ctx;
static void po_apply(void* c, int kase, double* x) {
  (void)kase; /* inv(A) is symmetric: both directions are the same solve */
  po_ctx* p = (po_ctx*)c;
  orc_potrs_lower(p->n, 1, p->L, p->lda, x, p->n);
}
double orc_rcond_chol(int n, const double* L, int lda, double anorm, int* nsolves) {
  po_ctx p = {n, L, lda};
  if (anorm == 0.0) { if (nsolves) *nsolves = 0; return 0.0; }
  return rcond_from(anorm, orc_inv_norm1_est(n, po_apply, &p, nsolves));
}

typedef struct { int upper, n; const double* T; int ldt; } tr_ctx;
static void tr_apply(void* c, int kase, double* x) {
  tr_ctx* t = (tr_ctx*)c;
  orc_trsv(t->upper, kase == 2, 0, t->n, t->T, t->ldt, x);
}
double orc_rcond_tri(int upper, int n, const double* T, int ldt, double anorm, int* nsolves) {
  tr_ctx t = {upper, n, T, ldt};
  if (anorm == 0.0) { if (nsolves) *nsolves = 0; return 0.0; }
  return rcond_from(anorm, orc_inv_norm1_est(n, tr_apply, &t, nsolves));
}

typedef struct { int n, kl, ku; const double* AB; int ldab; const int* ipiv; } gb_ctx;
static void gb_apply(void* c, int kase, double* x) {
  gb_ctx* g = (gb_ctx*)c;
  orc_gbtrs(kase == 2, g->n, g->kl, g->ku, 1, g->AB, g->ldab, g->ipiv, x, g->n);
}
double orc_rcond_band(int n, int kl, int ku, const double* AB, int ldab, const int* ipiv, double anorm,
                      int* nsolves) {
  gb_ctx g = {n, kl, ku, AB, ldab, ipiv};
  if (anorm == 0.0) { if (nsolves) *nsolves = 0; return 0.0; }
  return rcond_from(anorm, orc_inv_norm1_est(n, gb_apply, &g, nsolves));
}

/* ======================================================================
 * Section V (the future work it names): plain symmetric matrices.
 * Reading: symmetric-indefinite LDL^T with Bunch-Kaufman partial pivoting
 * (Bunch & Kaufman, Math. Comp. 31(137), 1977), P A P^T = L D L^T with L unit
 * lower triangular and D block diagonal with 1x1 and 2x2 blocks.
 * Written on a full symmetric copy S of the current Schur complement so that
 * every step can be checked by eye. At column j (alpha = (1 + sqrt 17)/8):
 *   colmax = largest |S(i,j)|, i > j, first such row r;
 *   both |S(j,j)| and colmax zero: D(j) = 0, info = j+1 (first), nothing moves;
 *   |S(j,j)| >= alpha colmax: 1x1 pivot, no interchange;
 *   otherwise rowmax = largest off-diagonal |S(r,i)|, i >= j, i != r, and
 *     |S(j,j)| rowmax >= alpha colmax^2: 1x1, no interchange;
 *     |S(r,r)| >= alpha rowmax: 1x1, interchange j <-> r;
 *     else: 2x2 pivot on (j, j+1), interchange j+1 <-> r.
 * An interchange swaps rows and columns of S, rows of the L columns already
 * formed and the entries of perm (so that P is one permutation at the end).
 * Output: L strictly below the diagonal of A (L(j+1,j) = 0 at a 2x2 block),
 * d[j] = D(j,j), e[j] = D(j+1,j) at the first column of a 2x2 block (else 0),
 * perm[i] = the row of A that goes to position i. Returns info.
 * ==================================================================== */
static const double BK_ALPHA = 0.64038820320220756872767623199676; /* (1 + sqrt(17)) / 8 */

static void sym_swap(int n, double* S, int a, int b) {
  for (int c = 0; c < n; ++c) { const double t = EL(S, n, a, c); EL(S, n, a, c) = EL(S, n, b, c); EL(S, n, b, c) = t; }
  for (int c = 0; c < n; ++c) { const double t = EL(S, n, c, a); EL(S, n, c, a) = EL(S, n, c, b); EL(S, n, c, b) = t; }
}

int orc_sytrf_bk(int n, double* A, int lda, double* d, double* e, int* perm) {
  double* S = (double*)malloc(sizeof(double) * (size_t)n * n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) EL(S, n, i, j) = i >= j ? EL(A, lda, i, j) : EL(A, lda, j, i);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) EL(A, lda, i, j) = 0.0; /* becomes L (strict lower part) */
  for (int i = 0; i < n; ++i) { perm[i] = i; d[i] = 0.0; e[i] = 0.0; }
  int info = 0;
  int j = 0;
  while (j < n) {
    int r = j;
    double colmax = 0.0;
    for (int i = j + 1; i < n; ++i)
      if (fabs(EL(S, n, i, j)) > colmax) { colmax = fabs(EL(S, n, i, j)); r = i; }
    const double absjj = fabs(EL(S, n, j, j));
    int size = 1, swap_from = -1, swap_to = -1;
    if (absjj == 0.0 && colmax == 0.0) {
      if (info == 0) info = j + 1;
      d[j] = 0.0;
      ++j;
      continue;
    }
    if (absjj < BK_ALPHA * colmax) {
      double rowmax = 0.0;
      for (int i = j; i < n; ++i)
        if (i != r && fabs(EL(S, n, r, i)) > rowmax) rowmax = fabs(EL(S, n, r, i));
      if (absjj * rowmax >= BK_ALPHA * colmax * colmax) {
        /* 1x1, no interchange */
      } else if (fabs(EL(S, n, r, r)) >= BK_ALPHA * rowmax) {
        swap_from = j;
        swap_to = r;
      } else {
        size = 2;
        swap_from = j + 1;
        swap_to = r;
      }
    }
    if (swap_to >= 0 && swap_to != swap_from) {
      sym_swap(n, S, swap_from, swap_to);
      for (int c = 0; c < j; ++c) {
        const double t = EL(A, lda, swap_from, c);
        EL(A, lda, swap_from, c) = EL(A, lda, swap_to, c);
        EL(A, lda, swap_to, c) = t;
      }
      const int t = perm[swap_from];
      perm[swap_from] = perm[swap_to];
      perm[swap_to] = t;
    }
    if (size == 1) {
      const double dj = EL(S, n, j, j);
      d[j] = dj;
      for (int i = j + 1; i < n; ++i) EL(A, lda, i, j) = EL(S, n, i, j) / dj;
#pragma omp parallel for schedule(static) if (n - j > 256)
      for (int c = j + 1; c < n; ++c)
        for (int i = j + 1; i < n; ++i) EL(S, n, i, c) -= EL(A, lda, i, j) * dj * EL(A, lda, c, j);
      j += 1;
    } else {
      const double a = EL(S, n, j, j), b = EL(S, n, j + 1, j), c2 = EL(S, n, j + 1, j + 1);
      const double det = a * c2 - b * b;
      d[j] = a;
      d[j + 1] = c2;
      e[j] = b;
      /* [l_i0 l_i1] = [s_i0 s_i1] D^{-1}, D^{-1} = [c2 -b; -b a] / det */
      for (int i = j + 2; i < n; ++i) {
        const double s0 = EL(S, n, i, j), s1 = EL(S, n, i, j + 1);
        EL(A, lda, i, j) = (s0 * c2 - s1 * b) / det;
        EL(A, lda, i, j + 1) = (s1 * a - s0 * b) / det;
      }
#pragma omp parallel for schedule(static) if (n - j > 256)
      for (int c = j + 2; c < n; ++c)
        for (int i = j + 2; i < n; ++i)
          EL(S, n, i, c) -= EL(A, lda, i, j) * EL(S, n, c, j) + EL(A, lda, i, j + 1) * EL(S, n, c, j + 1);
      j += 2;
    }
  }
  free(S);
  return info;
}

/* x = P^T L^{-T} D^{-1} L^{-1} P b for every right-hand side */
void orc_sytrs_bk(int n, int nrhs, const double* L, int lda, const double* d, const double* e, const int* perm,
                  double* B, int ldb) {
#pragma omp parallel for schedule(static) if (nrhs > 1)
  for (int r = 0; r < nrhs; ++r) {
    double* b = B + (size_t)r * ldb;
    double* y = (double*)malloc(sizeof(double) * (size_t)n);
    for (int i = 0; i < n; ++i) y[i] = b[perm[i]];
    orc_trsv(0, 0, 1, n, L, lda, y);
    for (int j = 0; j < n;) {
      if (j + 1 < n && e[j] != 0.0) {
        const double a = d[j], bb = e[j], c2 = d[j + 1], det = a * c2 - bb * bb;
        const double y0 = y[j], y1 = y[j + 1];
        y[j] = (c2 * y0 - bb * y1) / det;
        y[j + 1] = (a * y1 - bb * y0) / det;
        j += 2;
      } else {
        y[j] /= d[j];
        j += 1;
      }
    }
    orc_trsv(0, 1, 1, n, L, lda, y);
    for (int i = 0; i < n; ++i) b[perm[i]] = y[i];
    free(y);
  }
}

typedef struct { int n; const double* L; int lda; const double *d, *e; const int* perm; } sy_ctx;
static void sy_apply(void* c, int kase, double* x) {
  (void)kase; /* inv(A) is symmetric */
  sy_ctx* q = (sy_ctx*)c;
  orc_sytrs_bk(q->n, 1, q->L, q->lda, q->d, q->e, q->perm, x, q->n);
}
double orc_rcond_sym_bk(int n, const double* L, int lda, const double* d, const double* e, const int* perm,
                        double anorm, int* nsolves) {
  sy_ctx q = {n, L, lda, d, e, perm};
  if (anorm == 0.0) { if (nsolves) *nsolves = 0; return 0.0; }
  return rcond_from(anorm, orc_inv_norm1_est(n, sy_apply, &q, nsolves));
}

/* ======================================================================
 * Section V (future work): tridiagonal matrices, the banded case kl = ku = 1.
 * Reading: Gaussian elimination with partial pivoting in tridiagonal storage
 * (dl: sub-, dm: main, du: super-diagonal). At row i the pivot is row i unless
 * |dl_i| > |dm_i| (ties keep row i); an interchange brings a second
 * super-diagonal du2 into U. L is unit lower bidiagonal (multipliers in dl),
 * U upper triangular with the diagonals dm, du, du2. ipiv[i] = i or i+1.
 * ==================================================================== */
int orc_gttrf(int n, double* dl, double* dm, double* du, double* du2, int* ipiv) {
  int info = 0;
  for (int i = 0; i < n; ++i) ipiv[i] = i;
  for (int i = 0; i < n - 2; ++i) du2[i] = 0.0;
  for (int i = 0; i < n - 1; ++i) {
    if (fabs(dm[i]) >= fabs(dl[i])) {
      /* no interchange: eliminate dl[i] */
      if (dm[i] != 0.0) {
        const double f = dl[i] / dm[i];
        dl[i] = f;
        dm[i + 1] -= f * du[i];
      }
    } else {
      /* interchange rows i and i+1 */
      const double f = dm[i] / dl[i];
      dm[i] = dl[i];
      dl[i] = f;
      const double t = du[i];
      du[i] = dm[i + 1];
      dm[i + 1] = t - f * dm[i + 1];
      if (i < n - 2) {
        du2[i] = du[i + 1];
        du[i + 1] = -f * du[i + 1];
      }
      ipiv[i] = i + 1;
    }
  }
  for (int i = 0; i < n; ++i)
    if (dm[i] == 0.0) { info = i + 1; break; }
  return info;
}

/* trans = 0: A x = b ; trans = 1: A^T x = b, with the factors of orc_gttrf */
void orc_gttrs(int trans, int n, int nrhs, const double* dl, const double* dm, const double* du, const double* du2,
               const int* ipiv, double* B, int ldb) {
  for (int r = 0; r < nrhs; ++r) {
    double* b = B + (size_t)r * ldb;
    if (!trans) {
      /* L y = P b, applied row by row */
      for (int i = 0; i < n - 1; ++i) {
        if (ipiv[i] == i) {
          b[i + 1] -= dl[i] * b[i];
        } else {
          const double t = b[i];
          b[i] = b[i + 1];
          b[i + 1] = t - dl[i] * b[i];
        }
      }
      /* U x = y */
      for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        if (i + 1 < n) s -= du[i] * b[i + 1];
        if (i + 2 < n) s -= du2[i] * b[i + 2];
        b[i] = s / dm[i];
      }
    } else {
      /* U^T z = b */
      for (int i = 0; i < n; ++i) {
        double s = b[i];
        if (i >= 1) s -= du[i - 1] * b[i - 1];
        if (i >= 2) s -= du2[i - 2] * b[i - 2];
        b[i] = s / dm[i];
      }
      /* L^T then P^T, from the last row up */
      for (int i = n - 2; i >= 0; --i) {
        if (ipiv[i] == i) {
          b[i] -= dl[i] * b[i + 1];
        } else {
          const double t = b[i + 1];
          b[i + 1] = b[i] - dl[i] * t;
          b[i] = t;
        }
      }
    }
  }
}

typedef struct { int n; const double *dl, *dm, *du, *du2; const int* ipiv; } gt_ctx;
static void gt_apply(void* c, int kase, double* x) {
  gt_ctx* g = (gt_ctx*)c;
  orc_gttrs(kase == 2, g->n, 1, g->dl, g->dm, g->du, g->du2, g->ipiv, x, g->n);
}
double orc_rcond_gt(int n, const double* dl, const double* dm, const double* du, const double* du2, const int* ipiv,
                    double anorm, int* nsolves) {
  gt_ctx g = {n, dl, dm, du, du2, ipiv};
  if (anorm == 0.0) { if (nsolves) *nsolves = 0; return 0.0; }
  return rcond_from(anorm, orc_inv_norm1_est(n, gt_apply, &g, nsolves));
}

/* ======================================================================
 * Section II-E: SVD-based minimum-norm least-squares fallback.
 * One-sided (Hestenes) Jacobi on the columns of U (initially A), cyclic by
 * rows over the pairs p<q. A pair is rotated when its inner product exceeds
 * n*eps times the product of the column norms. The rotation uses
 * Rutishauser's formulas: zeta = (beta-alpha)/(2 gamma),
 * t = sign(zeta)/(|zeta| + sqrt(1+zeta^2)), c = 1/sqrt(1+t^2), s = c t.
 * V accumulates the rotations. Stops after a sweep without rotation.
 * On return column i of U is sigma_i * u_i and sigma_i = ||U(:,i)||_2.
 * ==================================================================== */
int orc_jacobi_svd(int n, double* U, int ldu, double* V, int ldv, double* sigma, int max_sweeps) {
  const double tol = (double)n * ORC_EPS;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) EL(V, ldv, i, j) = (i == j) ? 1.0 : 0.0;
  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    int rotated = 0;
    for (int p = 0; p + 1 < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double alpha = 0.0, beta = 0.0, gamma = 0.0;
        for (int i = 0; i < n; ++i) {
          const double up = EL(U, ldu, i, p), uq = EL(U, ldu, i, q);
          alpha += up * up;
          beta += uq * uq;
          gamma += up * uq;
        }
        if (!(fabs(gamma) > tol * sqrt(alpha) * sqrt(beta))) continue;
        rotated = 1;
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double s = c * t;
        for (int i = 0; i < n; ++i) {
          const double up = EL(U, ldu, i, p), uq = EL(U, ldu, i, q);
          EL(U, ldu, i, p) = c * up - s * uq;
          EL(U, ldu, i, q) = s * up + c * uq;
        }
        for (int i = 0; i < n; ++i) {
          const double vp = EL(V, ldv, i, p), vq = EL(V, ldv, i, q);
          EL(V, ldv, i, p) = c * vp - s * vq;
          EL(V, ldv, i, q) = s * vp + c * vq;
        }
      }
    }
    if (!rotated) { ++sweep; break; }
  }
  for (int j = 0; j < n; ++j) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += EL(U, ldu, i, j) * EL(U, ldu, i, j);
    sigma[j] = sqrt(s);
  }
  return sweep;
}

/* x = sum over kept i of v_i (u_i^T b) / sigma_i, keeping sigma_i > eps*sigma_max
 * (the truncation of a minimum-norm least-squares solver at machine precision).
 * Returns the number of kept singular values. */
int orc_svd_lstsq(int n, int nrhs, const double* A, int lda, const double* B, int ldb, double* X, int ldx,
                  double* sigma_out, int* sweeps_out) {
  double* U = (double*)malloc(sizeof(double) * (size_t)n * n);
  double* V = (double*)malloc(sizeof(double) * (size_t)n * n);
  double* sg = (double*)malloc(sizeof(double) * (size_t)n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) U[(size_t)i + (size_t)j * n] = EL(A, lda, i, j);
  const int sweeps = orc_jacobi_svd(n, U, n, V, n, sg, 30);
  double smax = 0.0;
  for (int i = 0; i < n; ++i)
    if (sg[i] > smax) smax = sg[i];
  const double cut = ORC_EPS * smax;
  int rank = 0;
  for (int i = 0; i < n; ++i)
    if (sg[i] > cut) ++rank;
  for (int r = 0; r < nrhs; ++r) {
    double* x = X + (size_t)r * ldx;
    const double* b = B + (size_t)r * ldb;
    for (int i = 0; i < n; ++i) x[i] = 0.0;
    for (int k = 0; k < n; ++k) {
      if (!(sg[k] > cut)) continue;
      double d = 0.0;
      for (int i = 0; i < n; ++i) d += U[(size_t)i + (size_t)k * n] * b[i];
      const double coef = d / (sg[k] * sg[k]);
      for (int i = 0; i < n; ++i) x[i] += V[(size_t)i + (size_t)k * n] * coef;
    }
  }
  if (sigma_out) memcpy(sigma_out, sg, sizeof(double) * (size_t)n);
  if (sweeps_out) *sweeps_out = sweeps;
  free(U);
  free(V);
  free(sg);
  return rank;
}

/* ======================================================================
 * Accuracy metric (not part of the paper): normwise backward error
 * eta = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf), per column.
 *
 * The residual of a backward-stable solution is as small as the rounding of
 * a plain FP64 evaluation of b - A x, so the residual entries are formed
 * accurately here: every product a*x is split exactly into hi + lo by
 * Dekker's algorithm (Veltkamp splitting, no fused multiply-add: this file
 * is compiled with -ffp-contract=off), and the 2n+1 terms of each entry are
 * summed with Neumaier's compensated summation (Numer. Math. 1974), whose
 * error is at most 2u|sum| + O(n u^2) sum|terms|: eta is exact to a few
 * units in its last place. Valid while |a|, |x| < 2^996 (the splitting
 * constant times a must not overflow).
 * ==================================================================== */
typedef struct {
  double s, c;
} orc_nsum_t;

static void nsum_add(orc_nsum_t* a, double t) {
  const double u = a->s + t;
  if (fabs(a->s) >= fabs(t))
    a->c += (a->s - u) + t;
  else
    a->c += (t - u) + a->s;
  a->s = u;
}

/* exact product: a*b = hi + lo (Dekker 1971) */
static void exact_product(double a, double b, double* hi, double* lo) {
  const double split = 134217729.0; /* 2^27 + 1 */
  double t = split * a;
  const double ah = t - (t - a), al = a - ah;
  t = split * b;
  const double bh = t - (t - b), bl = b - bh;
  *hi = a * b;
  *lo = al * bl - (((*hi - ah * bh) - al * bh) - ah * bl);
}

static double eta_of(int n, const double* r, const double* x, const double* b, double anorm_inf) {
  double rn = 0.0, xn = 0.0, bn = 0.0;
  for (int i = 0; i < n; ++i) {
    if (fabs(r[i]) > rn || r[i] != r[i]) rn = fabs(r[i]);
    if (fabs(x[i]) > xn || x[i] != x[i]) xn = fabs(x[i]);
    if (fabs(b[i]) > bn) bn = fabs(b[i]);
  }
  const double den = anorm_inf * xn + bn;
  return den > 0.0 ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
}

double orc_berr(int n, int nrhs, const double* A, int lda, const double* B, int ldb, const double* X, int ldx,
                double* per_rhs) {
  double anorm_inf = 0.0;
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += fabs(EL(A, lda, i, j));
    if (s > anorm_inf) anorm_inf = s;
  }
  double worst = 0.0;
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  orc_nsum_t* acc = (orc_nsum_t*)malloc(sizeof(orc_nsum_t) * (size_t)n);
  for (int k = 0; k < nrhs; ++k) {
    const double* x = X + (size_t)k * ldx;
    const double* b = B + (size_t)k * ldb;
    for (int i = 0; i < n; ++i) {
      acc[i].s = b[i];
      acc[i].c = 0.0;
    }
    /* rows are independent: blocks of rows side by side, columns in order within each */
#pragma omp parallel for schedule(static) if (n > 512)
    for (int i0 = 0; i0 < n; i0 += 256) {
      const int i1 = i0 + 256 < n ? i0 + 256 : n;
      for (int j = 0; j < n; ++j)
        for (int i = i0; i < i1; ++i) {
          double hi, lo;
          exact_product(EL(A, lda, i, j), x[j], &hi, &lo);
          nsum_add(&acc[i], -hi);
          nsum_add(&acc[i], -lo);
        }
    }
    for (int i = 0; i < n; ++i) r[i] = acc[i].s + acc[i].c;
    const double eta = eta_of(n, r, x, b, anorm_inf);
    if (per_rhs) per_rhs[k] = eta;
    if (eta > worst || eta != eta) worst = eta;
  }
  free(acc);
  free(r);
  return worst;
}

/* band-layout version: A(i,j) = AB[ku + i - j + j*ldab], the same accurate residual */
double orc_berr_band(int n, int kl, int ku, int nrhs, const double* AB, int ldab, const double* B, int ldb,
                     const double* X, int ldx) {
  double anorm_inf = 0.0;
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = imax(0, i - kl); j <= imin(n - 1, i + ku); ++j) s += fabs(AB[(size_t)(ku + i - j) + (size_t)j * ldab]);
    if (s > anorm_inf) anorm_inf = s;
  }
  double worst = 0.0;
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  for (int k = 0; k < nrhs; ++k) {
    const double* x = X + (size_t)k * ldx;
    const double* b = B + (size_t)k * ldb;
    for (int i = 0; i < n; ++i) {
      orc_nsum_t a = {b[i], 0.0};
      for (int j = imax(0, i - kl); j <= imin(n - 1, i + ku); ++j) {
        double hi, lo;
        exact_product(AB[(size_t)(ku + i - j) + (size_t)j * ldab], x[j], &hi, &lo);
        nsum_add(&a, -hi);
        nsum_add(&a, -lo);
      }
      r[i] = a.s + a.c;
    }
    const double eta = eta_of(n, r, x, b, anorm_inf);
    if (eta > worst || eta != eta) worst = eta;
  }
  free(r);
  return worst;
}

/* ======================================================================
 * The adaptive driver (Section II and the Fig. 2 caption):
 *   detect -> banded LU | triangular substitution | Cholesky (failure -> LU)
 *          | LU;  every route estimates rcond;
 *   solver failure, rcond < threshold or rcond NaN -> SVD least squares on the
 *   original A, unless the fallback is disabled.
 * Readings where the paper is silent: non-finite input is rejected; the
 * default threshold is 0.5*eps with a strict "<"; a non-finite x from a
 * route counts as a solver failure.
 * ==================================================================== */
static int all_finite(int rows, int cols, const double* M, int ld) {
  for (int j = 0; j < cols; ++j)
    for (int i = 0; i < rows; ++i)
      if (!isfinite(EL(M, ld, i, j))) return 0;
  return 1;
}

static void copy_mat(int rows, int cols, const double* S, int lds, double* D, int ldd) {
  for (int j = 0; j < cols; ++j) memcpy(D + (size_t)j * ldd, S + (size_t)j * lds, sizeof(double) * (size_t)rows);
}

/* routes the system and fills X, info, rcond; returns 1 if the solver failed */
static int exactly_symmetric(int n, const double* A, int lda) {
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i)
      if (!(EL(A, lda, i, j) == EL(A, lda, j, i))) return 0;
  return 1;
}

/* LDL^T route (Section V future work, Bunch-Kaufman reading); returns 1 on failure */
static int route_ldlt(int n, int nrhs, const double* A, int lda, double* X, int ldx, orc_result_t* res) {
  double* F = (double*)malloc(sizeof(double) * (size_t)n * n);
  double* d = (double*)malloc(sizeof(double) * (size_t)n);
  double* e = (double*)malloc(sizeof(double) * (size_t)n);
  int* perm = (int*)malloc(sizeof(int) * (size_t)n);
  copy_mat(n, n, A, lda, F, n);
  res->route = ORC_ROUTE_LDLT;
  res->info = orc_sytrf_bk(n, F, n, d, e, perm);
  int failed = res->info != 0;
  if (!failed) {
    orc_sytrs_bk(n, nrhs, F, n, d, e, perm, X, ldx);
    res->rcond = orc_rcond_sym_bk(n, F, n, d, e, perm, orc_norm1_sym_lower(n, A, lda), NULL);
  }
  free(F);
  free(d);
  free(e);
  free(perm);
  return failed;
}

/* tridiagonal route (Section V future work): the three diagonals of A(i,j) = get(i,j) */
static int route_gt(int n, int nrhs, const double* dl0, const double* dm0, const double* du0, double* X, int ldx,
                    orc_result_t* res) {
  double* dl = (double*)calloc((size_t)n + 1, sizeof(double));
  double* dm = (double*)calloc((size_t)n + 1, sizeof(double));
  double* du = (double*)calloc((size_t)n + 1, sizeof(double));
  double* du2 = (double*)calloc((size_t)n + 1, sizeof(double));
  int* ipiv = (int*)malloc(sizeof(int) * (size_t)n);
  memcpy(dm, dm0, sizeof(double) * (size_t)n);
  if (n > 1) {
    memcpy(dl, dl0, sizeof(double) * (size_t)(n - 1));
    memcpy(du, du0, sizeof(double) * (size_t)(n - 1));
  }
  /* ||A||_1: column j holds du(j-1), dm(j), dl(j) */
  double anorm = 0.0;
  for (int j = 0; j < n; ++j) {
    double c = fabs(dm0[j]);
    if (j > 0) c += fabs(du0[j - 1]);
    if (j < n - 1) c += fabs(dl0[j]);
    if (c > anorm || c != c) anorm = c;
  }
  res->route = ORC_ROUTE_GT;
  res->info = orc_gttrf(n, dl, dm, du, du2, ipiv);
  const int failed = res->info != 0;
  if (!failed) {
    orc_gttrs(0, n, nrhs, dl, dm, du, du2, ipiv, X, ldx);
    res->rcond = orc_rcond_gt(n, dl, dm, du, du2, ipiv, anorm, NULL);
  }
  free(dl);
  free(dm);
  free(du);
  free(du2);
  free(ipiv);
  return failed;
}

static int run_route(int n, int nrhs, const double* A, int lda, const double* B, int ldb, double* X, int ldx,
                     int ext, orc_result_t* res) {
  copy_mat(n, nrhs, B, ldb, X, ldx);
  int failed = 0;
  res->info = 0;
  res->rcond = NAN;
  if (res->cls == ORC_BANDED && (ext & ORC_EXT_TRIDIAG) && res->kl == 1 && res->ku == 1) {
    double* dg = (double*)calloc(3 * (size_t)n, sizeof(double));
    for (int i = 0; i < n; ++i) {
      dg[n + i] = EL(A, lda, i, i);
      if (i + 1 < n) {
        dg[i] = EL(A, lda, i + 1, i);
        dg[2 * n + i] = EL(A, lda, i, i + 1);
      }
    }
    failed = route_gt(n, nrhs, dg, dg + n, dg + 2 * n, X, ldx, res);
    free(dg);
  } else if (res->cls == ORC_SYM) {
    failed = route_ldlt(n, nrhs, A, lda, X, ldx, res);
  } else if (res->cls == ORC_BANDED) {
    const int kl = res->kl, ku = res->ku, ldab = 2 * kl + ku + 1;
    double* AB = (double*)calloc((size_t)ldab * n, sizeof(double));
    int* ipiv = (int*)malloc(sizeof(int) * (size_t)n);
    for (int j = 0; j < n; ++j)
      for (int i = imax(0, j - ku); i <= imin(n - 1, j + kl); ++i)
        AB[(size_t)(kl + ku + i - j) + (size_t)j * ldab] = EL(A, lda, i, j);
    const double anorm = orc_norm1_band(n, kl, ku, AB, ldab, kl + ku);
    res->route = ORC_ROUTE_BAND_LU;
    res->info = orc_gbtrf(n, kl, ku, AB, ldab, ipiv);
    if (res->info) failed = 1;
    else {
      orc_gbtrs(0, n, kl, ku, nrhs, AB, ldab, ipiv, X, ldx);
      res->rcond = orc_rcond_band(n, kl, ku, AB, ldab, ipiv, anorm, NULL);
    }
    free(AB);
    free(ipiv);
  } else if (res->cls == ORC_TRI_UPPER || res->cls == ORC_TRI_LOWER) {
    const int upper = res->cls == ORC_TRI_UPPER;
    res->route = ORC_ROUTE_TRI;
    for (int i = 0; i < n; ++i)
      if (EL(A, lda, i, i) == 0.0) { res->info = i + 1; break; }
    if (res->info) failed = 1;
    else {
      for (int r = 0; r < nrhs; ++r) orc_trsv(upper, 0, 0, n, A, lda, X + (size_t)r * ldx);
      res->rcond = orc_rcond_tri(upper, n, A, lda, orc_norm1_tri(upper, n, A, lda), NULL);
    }
  } else {
    double* F = (double*)malloc(sizeof(double) * (size_t)n * n);
    int general = res->cls == ORC_GENERAL;
    if (res->cls == ORC_SYMPD) {
      copy_mat(n, n, A, lda, F, n);
      const int info = orc_potrf_lower(n, F, n);
      if (info) {
        res->chol_failed = 1;
        res->info = info; /* replaced below by the LU's own info */
        general = 1;
        if ((ext & ORC_EXT_SYM) && exactly_symmetric(n, A, lda)) {
          /* with the symmetric-indefinite extension, LDL^T instead of LU */
          general = 0;
          failed = route_ldlt(n, nrhs, A, lda, X, ldx, res);
        }
      } else {
        res->route = ORC_ROUTE_CHOL;
        orc_potrs_lower(n, nrhs, F, n, X, ldx);
        res->rcond = orc_rcond_chol(n, F, n, orc_norm1_sym_lower(n, A, lda), NULL);
      }
    }
    if (general) {
      int* ipiv = (int*)malloc(sizeof(int) * (size_t)n);
      copy_mat(n, n, A, lda, F, n);
      res->route = ORC_ROUTE_LU;
      res->info = orc_getrf(n, F, n, ipiv);
      if (res->info) failed = 1;
      else {
        orc_getrs(0, n, nrhs, F, n, ipiv, X, ldx);
        res->rcond = orc_rcond_general(n, F, n, ipiv, orc_norm1_general(n, A, lda), NULL);
      }
      free(ipiv);
    }
    free(F);
  }
  if (!failed && !all_finite(n, nrhs, X, ldx)) failed = 1;
  return failed;
}

void orc_solve(int n, int nrhs, const double* A, int lda, const double* B, int ldb, double* X, int ldx,
               int no_approx, double rcond_threshold, int force_general, orc_result_t* res) {
  orc_solve_ext(n, nrhs, A, lda, B, ldb, X, ldx, no_approx, rcond_threshold, force_general, 0, res);
}

void orc_solve_ext(int n, int nrhs, const double* A, int lda, const double* B, int ldb, double* X, int ldx,
                   int no_approx, double rcond_threshold, int force_general, int ext, orc_result_t* res) {
  memset(res, 0, sizeof(*res));
  res->rcond = NAN;
  res->berr = NAN;
  res->kl = res->ku = -1;
  if (n < 1 || nrhs < 1 || lda < n || ldb < n || ldx < n || !A || !B || !X) { res->status = ORC_ERR_ARG; return; }
  if (!all_finite(n, n, A, lda) || !all_finite(n, nrhs, B, ldb)) { res->status = ORC_ERR_NONFINITE; return; }
  const double thr = rcond_threshold < 0.0 ? 0.5 * ORC_EPS : rcond_threshold;
  if (force_general) {
    res->cls = ORC_GENERAL;
  } else {
    orc_detect_t d;
    orc_detect(n, A, lda, &d);
    res->cls = d.cls;
    res->kl = d.kl;
    res->ku = d.ku;
    /* extension: a plain symmetric matrix (equal to its transpose, failing the Fig. 4 test) */
    if (res->cls == ORC_GENERAL && (ext & ORC_EXT_SYM) && exactly_symmetric(n, A, lda)) res->cls = ORC_SYM;
  }
  res->rank = n;
  const int failed = run_route(n, nrhs, A, lda, B, ldb, X, ldx, ext, res);
  if (failed) res->fallback = 1;
  else if (res->rcond != res->rcond) res->fallback = 3;
  else if (res->rcond < thr) res->fallback = 2;
  if (res->fallback) {
    if (no_approx) {
      res->status = ORC_ERR_SINGULAR;
    } else {
      res->route = ORC_ROUTE_SVD;
      res->rank = orc_svd_lstsq(n, nrhs, A, lda, B, ldb, X, ldx, NULL, &res->sweeps);
    }
  }
  res->berr = orc_berr(n, nrhs, A, lda, B, ldb, X, ldx, NULL);
}

/* ======================================================================
 * Band-layout input (the dense copy of a very large banded system does not
 * fit in memory). Detection finds the true kl/ku inside the stored band; a
 * system that is not banded under the 25% rule is expanded to dense and takes
 * the dense path, as does the SVD fallback when n*n <= dense_limit; beyond
 * that the fallback is infeasible.
 * ==================================================================== */
void orc_solve_band(int n, int kl_in, int ku_in, int nrhs, const double* ABin, int ldab_in, const double* B,
                    int ldb, double* X, int ldx, int no_approx, double rcond_threshold, int64_t dense_limit,
                    orc_result_t* res) {
  orc_solve_band_ext(n, kl_in, ku_in, nrhs, ABin, ldab_in, B, ldb, X, ldx, no_approx, rcond_threshold, dense_limit, 0,
                     res);
}

void orc_solve_band_ext(int n, int kl_in, int ku_in, int nrhs, const double* ABin, int ldab_in, const double* B,
                        int ldb, double* X, int ldx, int no_approx, double rcond_threshold, int64_t dense_limit,
                        int ext, orc_result_t* res) {
  memset(res, 0, sizeof(*res));
  res->rcond = NAN;
  res->berr = NAN;
  res->kl = res->ku = -1;
  if (n < 1 || nrhs < 1 || kl_in < 0 || ku_in < 0 || kl_in >= n || ku_in >= n || ldab_in < kl_in + ku_in + 1 ||
      ldb < n || ldx < n || !ABin || !B || !X) {
    res->status = ORC_ERR_ARG;
    return;
  }
  for (int j = 0; j < n; ++j)
    for (int i = imax(0, j - ku_in); i <= imin(n - 1, j + kl_in); ++i)
      if (!isfinite(ABin[(size_t)(ku_in + i - j) + (size_t)j * ldab_in])) { res->status = ORC_ERR_NONFINITE; return; }
  if (!all_finite(n, nrhs, B, ldb)) { res->status = ORC_ERR_NONFINITE; return; }
  const double thr = rcond_threshold < 0.0 ? 0.5 * ORC_EPS : rcond_threshold;
  /* Section II-A scan restricted to the stored rows (everything else is zero) */
  int kl = 0, ku = 0;
  for (int j = 0; j < n; ++j) {
    for (int i = imax(0, j - ku_in); i <= j; ++i)
      if (ABin[(size_t)(ku_in + i - j) + (size_t)j * ldab_in] != 0.0) { if (j - i > ku) ku = j - i; break; }
    int last = -1;
    for (int i = j; i <= imin(n - 1, j + kl_in); ++i)
      if (ABin[(size_t)(ku_in + i - j) + (size_t)j * ldab_in] != 0.0) last = i;
    if (last >= 0 && last - j > kl) kl = last - j;
  }
  res->kl = kl;
  res->ku = ku;
  const int64_t nn = (int64_t)n * n;
  if (!orc_is_banded(n, kl, ku)) {
    if (nn > dense_limit) { res->status = ORC_ERR_FALLBACK_INFEASIBLE; return; }
    double* A = (double*)calloc((size_t)nn, sizeof(double));
    for (int j = 0; j < n; ++j)
      for (int i = imax(0, j - ku_in); i <= imin(n - 1, j + kl_in); ++i)
        A[(size_t)i + (size_t)j * n] = ABin[(size_t)(ku_in + i - j) + (size_t)j * ldab_in];
    orc_solve_ext(n, nrhs, A, n, B, ldb, X, ldx, no_approx, rcond_threshold, 0, ext, res);
    free(A);
    return;
  }
  res->cls = ORC_BANDED;
  res->route = ORC_ROUTE_BAND_LU;
  res->rank = n;
  int failed = 0;
  copy_mat(n, nrhs, B, ldb, X, ldx);
  if ((ext & ORC_EXT_TRIDIAG) && kl == 1 && ku == 1) {
    double* dg = (double*)calloc(3 * (size_t)n, sizeof(double));
    for (int i = 0; i < n; ++i) {
      dg[n + i] = ABin[(size_t)ku_in + (size_t)i * ldab_in];
      if (i + 1 < n) {
        dg[i] = ABin[(size_t)(ku_in + 1) + (size_t)i * ldab_in];
        dg[2 * n + i] = ABin[(size_t)(ku_in - 1) + (size_t)(i + 1) * ldab_in];
      }
    }
    failed = route_gt(n, nrhs, dg, dg + n, dg + 2 * n, X, ldx, res);
    free(dg);
  } else {
    const int ldab = 2 * kl + ku + 1;
    double* AB = (double*)calloc((size_t)ldab * n, sizeof(double));
    int* ipiv = (int*)malloc(sizeof(int) * (size_t)n);
    for (int j = 0; j < n; ++j)
      for (int i = imax(0, j - ku); i <= imin(n - 1, j + kl); ++i)
        AB[(size_t)(kl + ku + i - j) + (size_t)j * ldab] = ABin[(size_t)(ku_in + i - j) + (size_t)j * ldab_in];
    const double anorm = orc_norm1_band(n, kl, ku, AB, ldab, kl + ku);
    res->info = orc_gbtrf(n, kl, ku, AB, ldab, ipiv);
    if (res->info) failed = 1;
    else {
      orc_gbtrs(0, n, kl, ku, nrhs, AB, ldab, ipiv, X, ldx);
      res->rcond = orc_rcond_band(n, kl, ku, AB, ldab, ipiv, anorm, NULL);
    }
    free(AB);
    free(ipiv);
  }
  if (!failed && !all_finite(n, nrhs, X, ldx)) failed = 1;
  if (failed) res->fallback = 1;
  else if (res->rcond != res->rcond) res->fallback = 3;
  else if (res->rcond < thr) res->fallback = 2;
  if (res->fallback) {
    if (no_approx) res->status = ORC_ERR_SINGULAR;
    else if (nn > dense_limit) {
      res->status = ORC_ERR_FALLBACK_INFEASIBLE;
      return;
    } else {
      double* A = (double*)calloc((size_t)nn, sizeof(double));
      for (int j = 0; j < n; ++j)
        for (int i = imax(0, j - ku_in); i <= imin(n - 1, j + kl_in); ++i)
          A[(size_t)i + (size_t)j * n] = ABin[(size_t)(ku_in + i - j) + (size_t)j * ldab_in];
      res->route = ORC_ROUTE_SVD;
      res->rank = orc_svd_lstsq(n, nrhs, A, n, B, ldb, X, ldx, NULL, &res->sweeps);
      free(A);
    }
  }
  res->berr = orc_berr_band(n, kl_in, ku_in, nrhs, ABin, ldab_in, B, ldb, X, ldx);
}
