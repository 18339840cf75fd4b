// Structure detection (Section II-A band scan and 25% rule inputs, Section II-B
// triangular test inputs, Section II-C / Fig. 4 likely_sympd) in ONE pass over A.
//
// The paper walks each column from both ends and runs Fig. 4 with early exits.
// Here every quantity those walks decide is computed as a map-reduce that gives
// the same values: kl = max{i-j : A_ij != 0, i > j}, ku = max{j-i : A_ij != 0,
// i < j} (the first non-zero from the top of a column and the last one from the
// bottom give exactly these maxima), and Fig. 4 is a conjunction of per-pair
// tests plus one test against the largest diagonal entry, which is
// order-independent: max_{i>j}|A_ij| < max_diag. The pass also rejects
// non-finite input and produces deterministic partial column/row sums for the
// 1-norm (condition estimate) and inf-norm (backward error).
#include "ada_internal.h"

#include <climits>

namespace ada {

__global__ void k_fill_int(int* p, int v, size_t count) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  size_t s = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += s) p[i] = v;
}

hipError_t launch_fill_int(int* p, int v, size_t count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  int blocks = (int)((count + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_int, dim3(blocks), dim3(256), 0, st, p, v, count);
  return hipGetLastError();
}

__global__ void k_init_rec(DevRec* rec) {
  // zero everything, then set the sentinels
  int* w = reinterpret_cast<int*>(rec);
  const int words = (int)(sizeof(DevRec) / sizeof(int));
  for (int i = threadIdx.x; i < words; i += blockDim.x) w[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    rec->diag_zero_first = INT_MAX;
    rec->info = INT_MAX;
    rec->chol_info = INT_MAX;
    rec->rcond = __longlong_as_double(0x7ff8000000000000LL);  // NaN until computed
    rec->berr = __longlong_as_double(0x7ff8000000000000LL);
  }
}

hipError_t launch_init_rec(DevRec* rec, hipStream_t st) {
  hipLaunchKernelGGL(k_init_rec, dim3(1), dim3(256), 0, st, rec);
  return hipGetLastError();
}

// One workgroup per tile pair (I, J), I >= J, of 64x64 tiles: tile X = (I,J)
// (on or below the diagonal) and its mirror Y = (J,I). Thread (r, q) handles
// row r of X and the 16 columns q*16..q*16+15; the mirror element of X(r,c) is
// Y(c,r), staged in LDS.
__global__ __launch_bounds__(256) void k_detect_dense(int n, const double* __restrict__ A, int lda, DevRec* rec,
                                                      double* __restrict__ pcol, double* __restrict__ prow,
                                                      double* __restrict__ col_lo_diag,
                                                      double* __restrict__ row_lo_diag, double* __restrict__ diag) {
  const long b = blockIdx.x;
  int I = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
  while ((long)I * (I + 1) / 2 > b) --I;
  while ((long)(I + 1) * (I + 2) / 2 <= b) ++I;
  const int J = (int)(b - (long)I * (I + 1) / 2);
  const bool dtile = (I == J);

  __shared__ double sY[64][65];
  __shared__ double sdI[64], sdJ[64];
  __shared__ double s_rowX[4][64], s_colY[4][64];
  __shared__ int s_red[4][8];
  __shared__ double s_redd[4][2];

  const int t = threadIdx.x;
  const int r = t & 63;
  const int q = t >> 6;
  const double tol = 100.0 * kEps;

  // stage the mirror tile Y = (J, I): sY[rr][cc] = A(J*64+rr, I*64+cc)
  {
    const int gi = J * 64 + r;
#pragma unroll 4
    for (int cc = 0; cc < 16; ++cc) {
      const int c = q * 16 + cc;
      const int gj = I * 64 + c;
      sY[r][c] = (gi < n && gj < n) ? A[(size_t)gi + (size_t)gj * lda] : 0.0;
    }
  }
  if (t < 64) {
    const int gi = I * 64 + t, gj = J * 64 + t;
    sdI[t] = gi < n ? A[(size_t)gi + (size_t)gi * lda] : 0.0;
    sdJ[t] = gj < n ? A[(size_t)gj + (size_t)gj * lda] : 0.0;
  }
  __syncthreads();

  __shared__ double s_cs[64], s_rs[64];
  int kl_c = 0, ku_c = 0, nonfin = 0, bad = 0, asym = 0;
  double maxlow = 0.0;
  double rowX = 0.0;  // row i = I*64+r over this thread's 16 columns (strictly lower part for the diag tile)
  double colY = 0.0;  // column i = I*64+r from the mirror elements (strictly upper part)
  const int gi = I * 64 + r;
  const double dii = sdI[r];
  for (int cc = 0; cc < 16; ++cc) {
    const int c = q * 16 + cc;
    const int gj = J * 64 + c;
    const bool valid = gi < n && gj < n && (!dtile || r > c);
    double a = 0.0, bm = 0.0;
    if (valid) {
      a = dtile ? sY[r][c] : A[(size_t)gi + (size_t)gj * lda];
      bm = sY[c][r];
      const double aa = fabs(a), ab = fabs(bm);
      nonfin |= !isfinite(a) || !isfinite(bm);
      if (a != 0.0) kl_c = max(kl_c, gi - gj);
      if (bm != 0.0) ku_c = max(ku_c, gi - gj);
      if (a != bm) asym = 1;                                           // exact symmetry
      const double delta = fabs(a - bm);
      if (delta > tol && delta > tol * fmax(aa, ab)) bad = 1;          // Fig. 4 lines 12-14
      if ((aa + ab) >= (dii + sdJ[c])) bad = 1;                        // Fig. 4 line 16
      maxlow = fmax(maxlow, aa);                                       // Fig. 4 line 15 (vs max_diag later)
      rowX += aa;
      colY += ab;
    }
    // column gj of X over the 64 rows of this wave; row gj of the mirror Y over its 64 columns
    const double cs = wave_sum(valid ? fabs(a) : 0.0);
    const double rs = wave_sum(valid ? fabs(bm) : 0.0);
    if (r == 0) { s_cs[c] = cs; s_rs[c] = rs; }
  }
  s_rowX[q][r] = rowX;
  s_colY[q][r] = colY;
  __syncthreads();
  if (t < 64) {
    const double rx = s_rowX[0][t] + s_rowX[1][t] + s_rowX[2][t] + s_rowX[3][t];
    const double cy = s_colY[0][t] + s_colY[1][t] + s_colY[2][t] + s_colY[3][t];
    const double cs = s_cs[t], rs = s_rs[t];
    if (!dtile) {
      const int gj = J * 64 + t;
      // tile X = (I,J): column partial of column gj (rows of tile I); row partial of row gi (columns of tile J)
      // tile Y = (J,I): row partial of row gj (columns of tile I); column partial of column gi (rows of tile J)
      if (gj < n) { pcol[(size_t)I * n + gj] = cs; prow[(size_t)I * n + gj] = rs; }
      if (gi < n) { prow[(size_t)J * n + gi] = rx; pcol[(size_t)J * n + gi] = cy; }
    } else if (gi < n) {
      const double d = sdI[t];
      const double ad = fabs(d);
      col_lo_diag[gi] = cs + ad;                      // column gi: strict lower + diagonal
      pcol[(size_t)I * n + gi] = (cs + ad) + cy;      //   + strict upper
      row_lo_diag[gi] = rx;                           // row gi: strict lower
      prow[(size_t)I * n + gi] = (rx + ad) + rs;      //   + diagonal + strict upper
      diag[gi] = d;
    }
  }
  // diagonal statistics (Fig. 4 lines 7-9) and the zero-diagonal test of the triangular route
  int dnonpos = 0, dzero = INT_MAX;
  double dmax = 0.0;
  if (dtile && t < 64 && gi < n) {
    const double d = sdI[t];
    nonfin |= !isfinite(d);
    if (!(d > 0.0)) dnonpos = 1;
    if (d == 0.0) dzero = gi + 1;
    dmax = fmax(dmax, d);
  }
  // reduce the flags over the workgroup
  kl_c = wave_max_int(kl_c);
  ku_c = wave_max_int(ku_c);
  nonfin = wave_or(nonfin);
  bad = wave_or(bad);
  asym = wave_or(asym);
  dnonpos = wave_or(dnonpos);
  dzero = wave_min_int(dzero);
  maxlow = wave_max(maxlow);
  dmax = wave_max(dmax);
  const int w = t >> 6;
  if (r == 0) {
    s_red[w][0] = kl_c; s_red[w][1] = ku_c; s_red[w][2] = nonfin; s_red[w][3] = bad;
    s_red[w][4] = dnonpos; s_red[w][5] = dzero; s_red[w][6] = asym;
    s_redd[w][0] = maxlow; s_redd[w][1] = dmax;
  }
  __syncthreads();
  if (t == 0) {
    int k0 = 0, k1 = 0, nf = 0, bd = 0, dn = 0, dz = INT_MAX, as = 0;
    double ml = 0.0, dm = 0.0;
    for (int i = 0; i < 4; ++i) {
      k0 = max(k0, s_red[i][0]); k1 = max(k1, s_red[i][1]); nf |= s_red[i][2]; bd |= s_red[i][3];
      dn |= s_red[i][4]; dz = min(dz, s_red[i][5]); as |= s_red[i][6];
      ml = fmax(ml, s_redd[i][0]); dm = fmax(dm, s_redd[i][1]);
    }
    if (k0) atomicMax(&rec->kl, k0);
    if (k1) atomicMax(&rec->ku, k1);
    if (nf) atomicOr(&rec->nonfinite, 1);
    if (bd) atomicOr(&rec->sym_bad, 1);
    if (as) atomicOr(&rec->asym, 1);
    if (dn) atomicOr(&rec->diag_nonpos, 1);
    if (dz != INT_MAX) atomicMin(&rec->diag_zero_first, dz);
    if (ml > 0.0) atomicMax(&rec->max_lower_bits, dbits(ml));
    if (dtile && dm > 0.0) atomicMax(&rec->max_diag_bits, dbits(dm));
  }
}

hipError_t launch_detect_dense(int n, const double* A, int lda, DevRec* rec, double* pcol, double* prow,
                               double* col_lo_diag, double* row_lo_diag, double* diag, hipStream_t st) {
  const long T = (n + 63) / 64;
  const long pairs = T * (T + 1) / 2;
  hipLaunchKernelGGL(k_detect_dense, dim3((unsigned)pairs), dim3(256), 0, st, n, A, lda, rec, pcol, prow,
                     col_lo_diag, row_lo_diag, diag);
  return hipGetLastError();
}

__global__ void k_check_finite(int rows, int cols, const double* __restrict__ M, int ld, DevRec* rec) {
  const size_t total = (size_t)rows * cols;
  int bad = 0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e % rows, j = e / rows;
    bad |= !isfinite(M[i + j * ld]);
  }
  bad = wave_or(bad);
  if ((threadIdx.x & 63) == 0 && bad) atomicOr(&rec->nonfinite, 1);
}

hipError_t launch_check_finite(int rows, int cols, const double* M, int ld, DevRec* rec, hipStream_t st) {
  size_t total = (size_t)rows * cols;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_check_finite, dim3(blocks), dim3(256), 0, st, rows, cols, M, ld, rec);
  return hipGetLastError();
}

// Deterministic reduction of the per-tile partial sums.
__global__ void k_norms_reduce(int n, const double* __restrict__ pcol, const double* __restrict__ prow,
                               const double* __restrict__ col_lo_diag, const double* __restrict__ row_lo_diag,
                               double* col_total, double* col_sym, double* row_total) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const int T = (n + 63) / 64;
  const int tx = x / 64;
  double ct = 0.0, cl = 0.0, rt = 0.0, rl = 0.0;
  for (int R = 0; R < T; ++R) {
    const double pc = pcol[(size_t)R * n + x];
    const double pr = prow[(size_t)R * n + x];
    ct += pc;
    rt += pr;
    if (R > tx) cl += pc;   // column x: tiles strictly below the diagonal tile
    if (R < tx) rl += pr;   // row x: tiles strictly left of the diagonal tile
  }
  col_total[x] = ct;
  row_total[x] = rt;
  // symmetric 1-norm read from the lower triangle: column x lower part + row x strict lower part
  col_sym[x] = (cl + col_lo_diag[x]) + (rl + row_lo_diag[x]);
}

hipError_t launch_norms_reduce(int n, const double* pcol, const double* prow, const double* col_lo_diag,
                               const double* row_lo_diag, double* col_total, double* col_sym, double* row_total,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_norms_reduce, dim3((n + 255) / 256), dim3(256), 0, st, n, pcol, prow, col_lo_diag,
                     row_lo_diag, col_total, col_sym, row_total);
  return hipGetLastError();
}

__global__ __launch_bounds__(1024) void k_anorm(int n, const double* __restrict__ col_total,
                                                const double* __restrict__ col_sym,
                                                const double* __restrict__ row_total, int mode, DevRec* rec) {
  __shared__ double s1[16], s2[16];
  double m1 = 0.0, m2 = 0.0;
  const double* c = mode == 1 ? col_sym : col_total;
  for (int x = threadIdx.x; x < n; x += blockDim.x) {
    m1 = fmax(m1, c[x]);
    m2 = fmax(m2, row_total[x]);
  }
  m1 = wave_max(m1);
  m2 = wave_max(m2);
  if ((threadIdx.x & 63) == 0) { s1[threadIdx.x >> 6] = m1; s2[threadIdx.x >> 6] = m2; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) { a = fmax(a, s1[i]); b = fmax(b, s2[i]); }
    rec->anorm1 = a;
    rec->anorm_inf = b;
  }
}

hipError_t launch_anorm(int n, const double* col_total, const double* col_sym, const double* row_total, int mode,
                        DevRec* rec, hipStream_t st) {
  hipLaunchKernelGGL(k_anorm, dim3(1), dim3(1024), 0, st, n, col_total, col_sym, row_total, mode, rec);
  return hipGetLastError();
}

// Band-layout input: the scan of Section II-A restricted to the stored rows (everything outside the
// stored band is zero by definition of the layout). The storage is read as one flat array, coalesced:
// element e is row r = e mod ldab of column j = e / ldab, entry (j + r - ku_in, j) of A (rows r >
// kl_in + ku_in, and entries outside the matrix, are not part of it). Each thread keeps (j, r) of its
// element and advances them by the grid stride.
__global__ __launch_bounds__(256) void k_detect_band(int n, int kl_in, int ku_in, const double* __restrict__ AB,
                                                     int ldab, DevRec* rec) {
  int kl_c = 0, ku_c = 0, nonfin = 0;
  const long long total = (long long)n * ldab;
  const long long e0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  const int sj = (int)(stride / ldab), sr = (int)(stride % ldab);
  int j = (int)(e0 / ldab), r = (int)(e0 % ldab);
  for (long long e = e0; e < total; e += stride) {
    const int i = j + r - ku_in;
    if (r <= kl_in + ku_in && i >= 0 && i < n) {
      const double v = AB[e];
      nonfin |= !isfinite(v);
      if (v != 0.0) {
        if (i < j) ku_c = max(ku_c, j - i);
        if (i > j) kl_c = max(kl_c, i - j);
      }
    }
    j += sj;
    r += sr;
    if (r >= ldab) {
      r -= ldab;
      ++j;
    }
  }
  kl_c = wave_max_int(kl_c);
  ku_c = wave_max_int(ku_c);
  nonfin = wave_or(nonfin);
  if ((threadIdx.x & 63) == 0) {
    if (kl_c) atomicMax(&rec->kl, kl_c);
    if (ku_c) atomicMax(&rec->ku, ku_c);
    if (nonfin) atomicOr(&rec->nonfinite, 1);
  }
}

hipError_t launch_detect_band(int n, int kl_in, int ku_in, const double* AB, int ldab, DevRec* rec,
                              hipStream_t st) {
  const long long total = (long long)n * ldab;
  long long blocks = (total + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_detect_band, dim3((unsigned)blocks), dim3(256), 0, st, n, kl_in, ku_in, AB, ldab, rec);
  return hipGetLastError();
}

}  // namespace ada
