/*
 * ada_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of the adaptive
 * solve of A x = b described in Sanderson & Curtin, "An Adaptive Solver for
 * Systems of Linear Equations" (arXiv 2007.11208), Sections II-A .. II-E.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this code. The GPU library shares no code, header,
 * table or constant with it.
 *
 * All matrices are column-major FP64; element (i,j) of a matrix with leading
 * dimension ld is M[i + j*ld] (zero-based, as in Fig. 4 of the paper).
 */
#ifndef ADA_ORACLE_H
#define ADA_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* structure classes (Section II, detection order banded -> triangular -> sympd) */
enum { ORC_GENERAL = 0, ORC_BANDED = 1, ORC_TRI_UPPER = 2, ORC_TRI_LOWER = 3, ORC_SYMPD = 4,
       ORC_SYM = 5 /* extension only: plain symmetric */ };
/* solver whose x is returned */
enum { ORC_ROUTE_NONE = 0, ORC_ROUTE_BAND_LU = 1, ORC_ROUTE_TRI = 2, ORC_ROUTE_CHOL = 3,
       ORC_ROUTE_LU = 4, ORC_ROUTE_SVD = 5, ORC_ROUTE_LDLT = 6, ORC_ROUTE_GT = 7 };
/* extensions named as future work in Section V (off by default: the paper's classes and routes):
   ORC_EXT_SYM: a matrix equal to its transpose that fails the Fig. 4 test (or whose Cholesky fails)
   is solved by LDL^T with Bunch-Kaufman pivoting; ORC_EXT_TRIDIAG: a banded matrix with
   kl = ku = 1 is solved by tridiagonal LU with partial pivoting. */
enum { ORC_EXT_SYM = 1, ORC_EXT_TRIDIAG = 2 };
/* status codes */
enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_NONFINITE = -2, ORC_ERR_SINGULAR = -3,
       ORC_ERR_FALLBACK_INFEASIBLE = -6 };

typedef struct {
  int32_t kl, ku;          /* exact band widths (Section II-A) */
  int32_t banded;          /* 25% rule */
  int32_t likely_sympd;    /* Fig. 4 (only evaluated when reached) */
  int32_t cls;             /* ORC_* class */
} orc_detect_t;

typedef struct {
  int32_t status;
  int32_t cls, kl, ku;
  int32_t route, chol_failed, fallback; /* fallback: 0 none, 1 solver failure, 2 rcond<thr, 3 rcond NaN */
  int32_t info;                          /* 1-based column of the first failing pivot, 0 if none */
  int32_t rank;                          /* SVD route: number of kept singular values; else n */
  int32_t sweeps;                        /* SVD route: Jacobi sweeps used */
  double rcond;                          /* from the routed factorisation; NaN if none */
  double berr;                           /* max over right-hand sides of the normwise backward error */
} orc_result_t;

/* ---- detection (Section II-A, II-B, II-C / Fig. 4) ---- */
void orc_band_scan(int n, const double* A, int lda, int* kl, int* ku);
int orc_is_banded(int64_t n, int64_t kl, int64_t ku);
int orc_likely_sympd(int n, const double* A, int lda);
void orc_detect(int n, const double* A, int lda, orc_detect_t* out);

/* ---- factorisations and solves ---- */
int orc_getrf(int n, double* A, int lda, int* ipiv);                 /* returns info */
void orc_getrs(int trans, int n, int nrhs, const double* LU, int lda, const int* ipiv, double* B, int ldb);
int orc_potrf_lower(int n, double* A, int lda);                     /* returns info */
void orc_potrs_lower(int n, int nrhs, const double* L, int lda, double* B, int ldb);
void orc_trsv(int upper, int trans, int unit, int n, const double* T, int ldt, double* x);
int orc_gbtrf(int n, int kl, int ku, double* AB, int ldab, int* ipiv);    /* AB: 2kl+ku+1 rows */
void orc_gbtrs(int trans, int n, int kl, int ku, int nrhs, const double* AB, int ldab, const int* ipiv,
               double* B, int ldb);

/* ---- norms and condition estimate ---- */
double orc_norm1_general(int n, const double* A, int lda);
double orc_norm1_tri(int upper, int n, const double* A, int lda);
double orc_norm1_sym_lower(int n, const double* A, int lda);
double orc_norm1_band(int n, int kl, int ku, const double* AB, int ldab, int off); /* A(i,j)=AB[off+i-j + j*ldab] */
typedef void (*orc_apply_fn)(void* ctx, int kase, double* x); /* kase 1: x <- inv(A) x ; 2: x <- inv(A)^T x */
double orc_inv_norm1_est(int n, orc_apply_fn apply, void* ctx, int* nsolves);
double orc_rcond_general(int n, const double* LU, int lda, const int* ipiv, double anorm, int* nsolves);
double orc_rcond_chol(int n, const double* L, int lda, double anorm, int* nsolves);
double orc_rcond_tri(int upper, int n, const double* T, int ldt, double anorm, int* nsolves);
double orc_rcond_band(int n, int kl, int ku, const double* AB, int ldab, const int* ipiv, double anorm, int* nsolves);

/* ---- Section V extensions: symmetric indefinite (Bunch-Kaufman) and tridiagonal ---- */
int orc_sytrf_bk(int n, double* A, int lda, double* d, double* e, int* perm);   /* returns info */
void orc_sytrs_bk(int n, int nrhs, const double* L, int lda, const double* d, const double* e, const int* perm,
                  double* B, int ldb);
double orc_rcond_sym_bk(int n, const double* L, int lda, const double* d, const double* e, const int* perm,
                        double anorm, int* nsolves);
int orc_gttrf(int n, double* dl, double* dm, double* du, double* du2, int* ipiv); /* returns info */
void orc_gttrs(int trans, int n, int nrhs, const double* dl, const double* dm, const double* du, const double* du2,
               const int* ipiv, double* B, int ldb);
double orc_rcond_gt(int n, const double* dl, const double* dm, const double* du, const double* du2, const int* ipiv,
                    double anorm, int* nsolves);

/* ---- SVD fallback (Section II-E) ---- */
int orc_jacobi_svd(int n, double* U, int ldu, double* V, int ldv, double* sigma, int max_sweeps);
int orc_svd_lstsq(int n, int nrhs, const double* A, int lda, const double* B, int ldb, double* X, int ldx,
                  double* sigma_out, int* sweeps_out);

/* ---- metric: normwise backward error per right-hand side ---- */
double orc_berr(int n, int nrhs, const double* A, int lda, const double* B, int ldb, const double* X, int ldx,
                double* per_rhs);
double orc_berr_band(int n, int kl, int ku, int nrhs, const double* AB, int ldab, const double* B, int ldb,
                     const double* X, int ldx);

/* ---- the adaptive driver (Fig. 2 as described in the text) ---- */
void orc_solve(int n, int nrhs, const double* A, int lda, const double* B, int ldb, double* X, int ldx,
               int no_approx, double rcond_threshold, int force_general, orc_result_t* res);
/* band-layout input: AB holds A(i,j) at AB[ku_in + i - j + j*ldab], ldab >= kl_in+ku_in+1 */
void orc_solve_band(int n, int kl_in, int ku_in, int nrhs, const double* AB, int ldab, const double* B, int ldb,
                    double* X, int ldx, int no_approx, double rcond_threshold, int64_t dense_limit,
                    orc_result_t* res);

/* the same with the Section V extensions ORC_EXT_* switched on */
void orc_solve_ext(int n, int nrhs, const double* A, int lda, const double* B, int ldb, double* X, int ldx,
                   int no_approx, double rcond_threshold, int force_general, int ext, orc_result_t* res);
void orc_solve_band_ext(int n, int kl_in, int ku_in, int nrhs, const double* AB, int ldab, const double* B, int ldb,
                        double* X, int ldx, int no_approx, double rcond_threshold, int64_t dense_limit, int ext,
                        orc_result_t* res);

int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
