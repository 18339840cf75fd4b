// Batched adaptive solve: many independent small systems (n <= 256,
// nrhs <= 8) in one persistent launch. Every step of Section II runs inside
// one workgroup per system, on the device, with no host decision:
//   detection (band scan, 25% rule, triangular test, likely_sympd of Fig. 4),
//   the routed factorisation (Cholesky with the LU re-route, LU with partial
//   pivoting, triangular substitution; a banded system is factored by the
//   same partial-pivoting elimination, which on a band makes the band LU's
//   pivots and factors), the solve, the condition estimate, the rule of
//   Section II-E and the Jacobi SVD least-squares fallback, and the backward
//   error.
// Workgroups take systems from a counter until none are left. The matrix of
// a system lives in LDS up to order 128 and in the workgroup's slice of the
// workspace above that. The triangular solves and the condition estimate run
// in one wave (lane = row, four rows per lane, solved values broadcast by
// readlane); factorisations and the Jacobi rounds use the four waves.
#include "ada.h"
#include "ada_internal.h"

#include <algorithm>
#include <climits>

namespace ada {

constexpr int BT = 256;       // threads per workgroup
constexpr int BNM = 256;      // largest order
constexpr int BRM = 8;        // most right-hand sides
constexpr int BNL = 128;      // orders up to this keep the matrix in LDS
constexpr int BRB = BNM / 64; // rows per lane in the one-wave solves
constexpr int BNL32 = 181;    // orders up to this keep an FP32 matrix in LDS (181^2 * 4 bytes <= 128 KB)
constexpr int kMaxRefine = 30;  // refinement steps at most (the limit of LAPACK's mixed-precision driver)
constexpr double kRcondRefine = 1e-9;  // FP32 factors with a smaller rcond estimate are not refined

// Pointers with their memory named in the type. The routines below are compiled as functions of their own;
// a plain pointer there is a flat address, whose loads wait on the LDS counter as well as the memory one
// and so complete one after another. Naming the memory gives global (buffer) and LDS instructions.
template <class T> using gptr = __attribute__((address_space(1))) T*;
template <class T> using lptr = __attribute__((address_space(3))) T*;
template <class T> __device__ __forceinline__ gptr<T> as_global(T* p) { return (gptr<T>)p; }
template <class T> __device__ __forceinline__ lptr<T> as_lds(T* p) { return (lptr<T>)p; }

struct BDesc {
  int32_t n, nrhs, lda, ldb, ldx, pad;
  int64_t a_off, b_off, x_off;
};

// per-workgroup slice of the workspace for systems of order <= hi (doubles, then ints): the matrix
// (orders > BNL) or Jacobi U, hi * hi; the Jacobi V / FP32 copy, hi * hi; right-hand-side buffers
__host__ __device__ constexpr size_t b_slice_doubles(int hi) {
  return 2 * (size_t)hi * hi + (size_t)BNM * BRM * 2 + (size_t)BNM * 4;
}
__host__ __device__ constexpr size_t b_slice_bytes(int hi) { return b_slice_doubles(hi) * 8 + (size_t)BNM * 2 * 4; }
// LDS of a launch for orders <= hi: the matrix region (the matrix itself up to order BNL; above that the
// blocked factorisations' panels and the staging of the triangles), then hi * BRM doubles of vectors
__host__ __device__ constexpr size_t b_lds_matrix(int hi) { return hi <= BNL ? (size_t)hi * hi : (size_t)BNL * BNL; }
__host__ __device__ constexpr size_t b_lds_bytes(int hi) { return 8 * (b_lds_matrix(hi) + (size_t)hi * BRM); }

struct BCtx {
  int t, lane, w;
  lptr<double> red;  // LDS scratch for reductions (8 doubles)
  lptr<int> ired;    // 8 ints
};

__device__ __forceinline__ double b_sum(const BCtx c, double v) {
  v = wave_sum(v);
  if (c.lane == 0) c.red[c.w] = v;
  __syncthreads();
  const double s = (c.red[0] + c.red[1]) + (c.red[2] + c.red[3]);
  __syncthreads();
  return s;
}
__device__ __forceinline__ double b_max(const BCtx c, double v) {
  v = wave_max(v);
  if (c.lane == 0) c.red[c.w] = v;
  __syncthreads();
  const double s = fmax(fmax(c.red[0], c.red[1]), fmax(c.red[2], c.red[3]));
  __syncthreads();
  return s;
}
__device__ __forceinline__ int b_max_int(const BCtx c, int v) {
  v = wave_max_int(v);
  if (c.lane == 0) c.ired[c.w] = v;
  __syncthreads();
  const int s = max(max(c.ired[0], c.ired[1]), max(c.ired[2], c.ired[3]));
  __syncthreads();
  return s;
}
__device__ __forceinline__ int b_or(const BCtx c, int v) {
  v = wave_or(v);
  if (c.lane == 0) c.ired[c.w] = v;
  __syncthreads();
  const int s = c.ired[0] | c.ired[1] | c.ired[2] | c.ired[3];
  __syncthreads();
  return s;
}
// largest |v| with the lowest index on ties (idx < 0: no candidate)
__device__ __forceinline__ int b_argmax(const BCtx c, double v, int idx) {
  wave_argmax(v, idx);
  if (c.lane == 0) { c.red[c.w] = v; c.ired[c.w] = idx; }
  __syncthreads();
  double bv = c.red[0];
  int bi = c.ired[0];
  for (int q = 1; q < 4; ++q) {
    const int i2 = c.ired[q];
    const double v2 = c.red[q];
    if (i2 >= 0 && (bi < 0 || v2 > bv || (v2 == bv && i2 < bi))) { bv = v2; bi = i2; }
  }
  __syncthreads();
  return bi;
}

// ---------------------------------------------------------------- factorisations (four waves)
// LU with partial pivoting of M (ld n) in place; perm tracks the row order. Returns info (0 or 1-based column).
template <class T>
__device__ int b_getrf(const BCtx c, lptr<T> M, int n, gptr<int> perm) {
  int info = 0;
  for (int i = c.t; i < n; i += BT) perm[i] = i;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double v = -1.0;
    int idx = -1;
    for (int i = j + c.t; i < n; i += BT) {
      const double a = fabs((double)M[i + j * n]);
      if (idx < 0 || a > v) { v = a; idx = i; }
    }
    const int p = b_argmax(c, v, idx);
    const T piv = M[p + j * n];
    if (piv == 0.0) {
      if (info == 0) info = j + 1;
      continue;
    }
    if (p != j) {
      for (int k = c.t; k < n; k += BT) {
        const T a = M[j + k * n];
        M[j + k * n] = M[p + k * n];
        M[p + k * n] = a;
      }
      if (c.t == 0) {
        const int q = perm[j];
        perm[j] = perm[p];
        perm[p] = q;
      }
      __syncthreads();
    }
    for (int i = j + 1 + c.t; i < n; i += BT) M[i + j * n] = M[i + j * n] / piv;
    __syncthreads();
    // rank-1 update: wave w takes columns j+1+w, j+5+w, ...; lane takes rows j+1+lane, +64, ...
    T l[BRB];
#pragma unroll
    for (int b = 0; b < BRB; ++b) {
      const int i = j + 1 + c.lane + 64 * b;
      l[b] = i < n ? M[i + j * n] : T(0);
    }
    for (int k = j + 1 + c.w; k < n; k += 4) {
      const T u = M[j + k * n];
#pragma unroll
      for (int b = 0; b < BRB; ++b) {
        const int i = j + 1 + c.lane + 64 * b;
        if (i < n) M[i + k * n] = fma(-l[b], u, M[i + k * n]);
      }
    }
    __syncthreads();
  }
  return info;
}

// ---- blocked forms for matrices in HBM (orders above what LDS holds): 32-column panels are factored in
// LDS, and the trailing matrix takes one rank-32 update per panel in 4x4 register tiles, so each of its
// elements is read and written once per panel rather than once per column. S: LDS scratch of at least
// 2 * PW * BNM elements of T (the LDS matrix region).
constexpr int PW = 32;
constexpr int LDP = BNM;  // P and U together fill the BNL x BNL LDS region exactly
static_assert(2 * PW * BNM <= BNL * BNL, "the blocked factorisations' LDS scratch must fit the matrix region");

// LU with partial pivoting (ties to the lowest row, as b_getrf), same result up to rounding order
template <class T>
__device__ int b_getrf_blk(const BCtx c, gptr<T> M, int n, gptr<int> perm, lptr<T> S) {
  lptr<T> P = S;             // panel: P[r + cc * LDP] = M(k0 + r, k0 + cc)
  lptr<T> U = S + PW * LDP;  // U12: U[kk * BNM + q] = M(k0 + kk, k0 + nbw + q)
  __shared__ int s_piv[PW];       // panel row that column jj's pivot came from (jj: no interchange)
  __shared__ int s_rows[2 * PW];  // rows touched by the panel's interchanges (offsets from k0)
  __shared__ int s_from[2 * PW];  // ... and which of them each one takes its value from (index into s_rows)
  __shared__ int s_nrows;
  int info = 0;
  for (int i = c.t; i < n; i += BT) perm[i] = i;
  __syncthreads();
  for (int k0 = 0; k0 < n; k0 += PW) {
    const int nbw = min(PW, n - k0), m = n - k0, rest = m - nbw;
    for (int e = c.t; e < m * nbw; e += BT) {
      const int r = e % m, cc = e / m;
      P[r + cc * LDP] = M[(k0 + r) + (size_t)(k0 + cc) * n];
    }
    __syncthreads();
    for (int jj = 0; jj < nbw; ++jj) {
      double v = -1.0;
      int idx = -1;
      for (int r = jj + c.t; r < m; r += BT) {
        const double a = fabs((double)P[r + jj * LDP]);
        if (idx < 0 || a > v) { v = a; idx = r; }
      }
      const int p = b_argmax(c, v, idx);
      const T piv = P[p + jj * LDP];
      if (piv == T(0)) {
        if (info == 0) info = k0 + jj + 1;
        if (c.t == 0) s_piv[jj] = jj;
        __syncthreads();
        continue;
      }
      if (c.t == 0) s_piv[jj] = p;
      if (p != jj) {
        for (int cc = c.t; cc < nbw; cc += BT) {
          const T a = P[jj + cc * LDP];
          P[jj + cc * LDP] = P[p + cc * LDP];
          P[p + cc * LDP] = a;
        }
        if (c.t == 0) {
          const int q = perm[k0 + jj];
          perm[k0 + jj] = perm[k0 + p];
          perm[k0 + p] = q;
        }
      }
      __syncthreads();
      for (int r = jj + 1 + c.t; r < m; r += BT) P[r + jj * LDP] = P[r + jj * LDP] / piv;
      __syncthreads();
      for (int r = jj + 1 + c.t; r < m; r += BT) {
        const T l = P[r + jj * LDP];
        for (int cc = jj + 1; cc < nbw; ++cc) P[r + cc * LDP] = fma(-l, P[jj + cc * LDP], P[r + cc * LDP]);
      }
      __syncthreads();
    }
    // the panel back; the interchanges as one gather per column: s_rows lists the touched rows, row
    // s_rows[i] takes the value row s_rows[s_from[i]] had
    for (int e = c.t; e < m * nbw; e += BT) {
      const int r = e % m, cc = e / m;
      M[(k0 + r) + (size_t)(k0 + cc) * n] = P[r + cc * LDP];
    }
    if (c.t == 0) {
      int nr = 0;
      for (int jj = 0; jj < nbw; ++jj) s_rows[nr++] = jj;
      for (int jj = 0; jj < nbw; ++jj) {
        const int p = s_piv[jj];
        bool seen = false;
        for (int i = 0; i < nr; ++i) seen |= s_rows[i] == p;
        if (!seen) s_rows[nr++] = p;
      }
      for (int i = 0; i < nr; ++i) s_from[i] = i;
      for (int jj = 0; jj < nbw; ++jj) {
        const int p = s_piv[jj];
        if (p == jj) continue;
        int ia = 0, ib = 0;
        for (int i = 0; i < nr; ++i) {
          if (s_rows[i] == jj) ia = i;
          if (s_rows[i] == p) ib = i;
        }
        const int tmp = s_from[ia];
        s_from[ia] = s_from[ib];
        s_from[ib] = tmp;
      }
      s_nrows = nr;
    }
    __syncthreads();
    // each of 128 threads gathers one column through its own slots of U's region (free until U12 is formed)
    const int nr = s_nrows;
    for (int b0 = 0; b0 < n - nbw; b0 += 128) {
      const int qi = b0 + c.t;
      if (c.t < 128 && qi < n - nbw) {
        const int q = qi < k0 ? qi : qi + nbw;  // the columns left and right of the panel
        gptr<T> col = M + (size_t)q * n + k0;
#pragma unroll 16
        for (int i = 0; i < nr; ++i) U[i * 128 + c.t] = col[s_rows[i]];
#pragma unroll 16
        for (int i = 0; i < nr; ++i) col[s_rows[i]] = U[s_from[i] * 128 + c.t];
      }
    }
    __syncthreads();
    if (rest <= 0) break;
    // U12 = L11^{-1} A12 (unit lower L11), one thread per column
    for (int q = c.t; q < rest; q += BT) {
      gptr<T> col = M + (size_t)(k0 + nbw + q) * n + k0;
      T x[PW];
#pragma unroll
      for (int kk = 0; kk < PW; ++kk) x[kk] = kk < nbw ? col[kk] : T(0);
#pragma unroll
      for (int kk = 1; kk < PW; ++kk)
#pragma unroll
        for (int ii = 0; ii < kk; ++ii)
          if (kk < nbw) x[kk] = fma(-P[kk + ii * LDP], x[ii], x[kk]);
#pragma unroll
      for (int kk = 0; kk < PW; ++kk)
        if (kk < nbw) {
          U[kk * BNM + q] = x[kk];
          col[kk] = x[kk];
        }
    }
    __syncthreads();
    // A22 -= L21 U12 in 4x4 tiles
    const int nt = (rest + 3) / 4;
    for (int tile = c.t; tile < nt * nt; tile += BT) {
      const int r4 = 4 * (tile % nt), q4 = 4 * (tile / nt);
      T acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = (r4 + a < rest && q4 + b < rest)
                          ? M[(k0 + nbw + r4 + a) + (size_t)(k0 + nbw + q4 + b) * n] : T(0);
      for (int kk = 0; kk < nbw; ++kk) {
        T l[4], u[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          l[a] = r4 + a < rest ? P[(nbw + r4 + a) + kk * LDP] : T(0);
          u[a] = q4 + a < rest ? U[kk * BNM + q4 + a] : T(0);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = fma(-l[a], u[b], acc[a][b]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if (r4 + a < rest && q4 + b < rest) M[(k0 + nbw + r4 + a) + (size_t)(k0 + nbw + q4 + b) * n] = acc[a][b];
    }
    __syncthreads();
  }
  return info;
}

// Cholesky A = L L^T from the lower triangle (as b_potrf): 0 or the 1-based failing column
template <class T>
__device__ int b_potrf_blk(const BCtx c, gptr<T> M, int n, lptr<T> S) {
  lptr<T> P = S;  // panel: P[r + cc * LDP] = M(k0 + r, k0 + cc), r >= cc
  for (int k0 = 0; k0 < n; k0 += PW) {
    const int nbw = min(PW, n - k0), m = n - k0, rest = m - nbw;
    for (int e = c.t; e < m * nbw; e += BT) {
      const int r = e % m, cc = e / m;
      P[r + cc * LDP] = r >= cc ? M[(k0 + r) + (size_t)(k0 + cc) * n] : T(0);
    }
    __syncthreads();
    for (int jj = 0; jj < nbw; ++jj) {
      const T d = P[jj + jj * LDP];
      if (!(d > T(0))) return k0 + jj + 1;
      const T sd = sqrt(d);
      __syncthreads();
      for (int r = jj + c.t; r < m; r += BT) P[r + jj * LDP] = (r == jj) ? sd : P[r + jj * LDP] / sd;
      __syncthreads();
      for (int r = jj + 1 + c.t; r < m; r += BT) {
        const T l = P[r + jj * LDP];
        for (int cc = jj + 1; cc < nbw && cc <= r; ++cc) P[r + cc * LDP] = fma(-l, P[cc + jj * LDP], P[r + cc * LDP]);
      }
      __syncthreads();
    }
    for (int e = c.t; e < m * nbw; e += BT) {
      const int r = e % m, cc = e / m;
      if (r >= cc) M[(k0 + r) + (size_t)(k0 + cc) * n] = P[r + cc * LDP];
    }
    if (rest <= 0) break;
    // trailing lower triangle: A22 -= L21 L21^T in 4x4 tiles (tile rows ti >= tile columns tj)
    const int nt = (rest + 3) / 4;
    const int ntiles = nt * (nt + 1) / 2;
    for (int tile = c.t; tile < ntiles; tile += BT) {
      int ti = (int)((sqrt(8.0 * (double)tile + 1.0) - 1.0) * 0.5);
      while (ti * (ti + 1) / 2 > tile) --ti;
      while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
      const int tj = tile - ti * (ti + 1) / 2;
      const int r4 = 4 * ti, q4 = 4 * tj;
      T acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int r = r4 + a, q = q4 + b;
          acc[a][b] = (r < rest && q <= r) ? M[(k0 + nbw + r) + (size_t)(k0 + nbw + q) * n] : T(0);
        }
      for (int kk = 0; kk < nbw; ++kk) {
        T l[4], u[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          l[a] = r4 + a < rest ? P[(nbw + r4 + a) + kk * LDP] : T(0);
          u[a] = q4 + a < rest ? P[(nbw + q4 + a) + kk * LDP] : T(0);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = fma(-l[a], u[b], acc[a][b]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int r = r4 + a, q = q4 + b;
          if (r < rest && q <= r) M[(k0 + nbw + r) + (size_t)(k0 + nbw + q) * n] = acc[a][b];
        }
    }
    __syncthreads();
  }
  return 0;
}

// Cholesky A = L L^T from the lower triangle of M; returns 0 or the 1-based failing column
template <class T>
__device__ int b_potrf(const BCtx c, lptr<T> M, int n) {
  for (int j = 0; j < n; ++j) {
    const T d = M[j + j * n];
    if (!(d > T(0))) return j + 1;
    const T sd = sqrt(d);
    __syncthreads();
    for (int i = j + c.t; i < n; i += BT) M[i + j * n] = (i == j) ? sd : M[i + j * n] / sd;
    __syncthreads();
    T l[BRB];
#pragma unroll
    for (int b = 0; b < BRB; ++b) {
      const int i = j + 1 + c.lane + 64 * b;
      l[b] = i < n ? M[i + j * n] : T(0);
    }
    for (int k = j + 1 + c.w; k < n; k += 4) {
      const T u = M[k + j * n];
#pragma unroll
      for (int b = 0; b < BRB; ++b) {
        const int i = j + 1 + c.lane + 64 * b;
        if (i >= k && i < n) M[i + k * n] = fma(-l[b], u, M[i + k * n]);
      }
    }
    __syncthreads();
  }
  return 0;
}

// ---------------------------------------------------------------- one-wave solves
// Vector (or block of nr <= BRM columns) held by wave 0: x[b][r] = row lane + 64 b, column r.
template <int NRC>
struct WVec {
  double x[BRB][NRC];
};

// op(T) y = y in place; T (ld ldt) lower or upper as stored, op = transpose if trans.
// FWD: forward substitution (op(T) lower). The columns are taken in groups of scol (scol divides 64), in
// solve order; a group's diagonal entries are inverted together (one division per lane), and each column's
// entries are loaded one column ahead so that their latency hides behind the previous column's update.
// stg: this wave's LDS staging area of scol * BNM elements (matrix in HBM; scol <= SPF), or null (matrix
// in LDS; scol = 64). A staged group is copied into registers while the group before it is solved: lane i
// loads row i of the group, a column segment of T (coalesced over the lanes) or a row segment (contiguous
// for each lane).
constexpr int SPF = 8;   // most columns of a staged group
// A function of its own (the vector in and out by value): its column loop gets registers of its own
// rather than what the whole kernel leaves over.
template <bool FWD, bool STG, int NRC, class TF>
__device__ __noinline__ WVec<NRC> w_trsv_dir(const TF* T, int ldt, int n, bool trans, bool unit, WVec<NRC> v,
                                             int nr, int lane, TF* stg, int scol) {
  const size_t pr = trans ? (size_t)ldt : 1, pc = trans ? 1 : (size_t)ldt;  // op(T)(i, c) = T[i*pr + c*pc]
  if (STG) scol = min(scol, SPF);
  const int ngr = (n + scol - 1) / scol;
  TF pf[SPF][BRB];
  auto fetch = [&](int g) {  // the triangle is in HBM when it is staged
    gptr<const TF> Tg = as_global(T);
    const int c0 = g * scol, scnt = min(scol, n - c0);
#pragma unroll
    for (int kk = 0; kk < SPF; ++kk)
#pragma unroll
      for (int b = 0; b < BRB; ++b) {
        const int i = lane + 64 * b;
        pf[kk][b] = (kk < scnt && i < n) ? Tg[i * pr + (size_t)(c0 + kk) * pc] : TF(0);
      }
  };
  if (STG) fetch(FWD ? 0 : ngr - 1);
  for (int gi = 0; gi < ngr; ++gi) {
    const int g = FWD ? gi : ngr - 1 - gi;
    const int c0 = g * scol, scnt = min(scol, n - c0);
    lptr<const TF> P;  // the stage, or the triangle itself when it is held in LDS
    size_t qr, qc;     // op(T)(i, c0 + k) = P[i*qr + k*qc]
    if (STG) {
#pragma unroll
      for (int kk = 0; kk < SPF; ++kk)
#pragma unroll
        for (int b = 0; b < BRB; ++b) {
          const int i = lane + 64 * b;
          if (kk < scnt && i < n) as_lds(stg)[kk * BNM + i] = pf[kk][b];
        }
      __builtin_amdgcn_wave_barrier();
      if (gi + 1 < ngr) fetch(FWD ? g + 1 : g - 1);
      P = as_lds<const TF>(stg);
      qr = 1;
      qc = BNM;
    } else {
      P = as_lds(T) + (size_t)c0 * pc;
      qr = pr;
      qc = pc;
    }
    double rk = 1.0;  // lane k: 1 / op(T)(c0 + k, c0 + k)
    if (!unit && lane < scnt) rk = 1.0 / (double)P[(c0 + lane) * qr + lane * qc];
    const int gjb = c0 >> 6, s0 = c0 & 63;
#pragma unroll
    for (int jb = 0; jb < BRB; ++jb) {
      if (jb != gjb) continue;
      TF tc[BRB];
      auto col = [&](int k, TF* t) {
#pragma unroll
        for (int b = 0; b < BRB; ++b) {
          const int i = lane + 64 * b;
          t[b] = i < n ? P[i * qr + k * qc] : TF(0);
        }
      };
      col(FWD ? 0 : scnt - 1, tc);
      for (int k0 = 0; k0 < scnt; ++k0) {
        const int k = FWD ? k0 : scnt - 1 - k0;
        TF tn[BRB];
        if (k0 + 1 < scnt) col(FWD ? k + 1 : k - 1, tn);
        const int jj = s0 + k;  // column within the block
        const int j = c0 + k;
        const double ri = unit ? 1.0 : read_lane(rk, k);
        double xj[NRC];
#pragma unroll
        for (int r = 0; r < NRC; ++r) {
          if (r < nr) {
            xj[r] = read_lane(v.x[jb][r], jj) * ri;
            if (lane == jj) v.x[jb][r] = xj[r];
          } else {
            xj[r] = 0.0;
          }
        }
#pragma unroll
        for (int b = 0; b < BRB; ++b) {
          const int i = lane + 64 * b;
          const bool rel = FWD ? (i > j) : (i < j);
          if (i < n && rel) {
            const double tij = (double)tc[b];
#pragma unroll
            for (int r = 0; r < NRC; ++r)
              if (r < nr) v.x[b][r] = fma(-tij, xj[r], v.x[b][r]);
          }
        }
#pragma unroll
        for (int b = 0; b < BRB; ++b) tc[b] = tn[b];
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  return v;
}

template <int NRC, class TF>
__device__ __forceinline__ void w_trsv(const TF* T, int ldt, int n, bool lower, bool trans, bool unit,
                                       WVec<NRC>& v, int nr, int lane, TF* stg, int scol) {
  if (stg) {
    if (lower != trans) v = w_trsv_dir<true, true, NRC, TF>(T, ldt, n, trans, unit, v, nr, lane, stg, scol);
    else v = w_trsv_dir<false, true, NRC, TF>(T, ldt, n, trans, unit, v, nr, lane, stg, scol);
  } else {
    if (lower != trans) v = w_trsv_dir<true, false, NRC, TF>(T, ldt, n, trans, unit, v, nr, lane, stg, scol);
    else v = w_trsv_dir<false, false, NRC, TF>(T, ldt, n, trans, unit, v, nr, lane, stg, scol);
  }
}

// routed factor: 0 LU (M = L\U, perm), 1 Cholesky (M = L), 2 triangular (T = A as given)
template <class TF>
struct BFactor {
  int kind;
  const TF* M;
  int ld;
  const int* perm;
  bool lower;  // triangular kind
  TF* stg;     // LDS staging for a matrix kept in HBM (null when M is in LDS)
  int scol;    // columns staged at a time (64 when one wave has the whole staging region)
};

// y = inv(A) y (trans = false) or inv(A)^T y (trans = true); one wave; sbuf: LDS, n * BRM doubles
template <int NRC, class TF>
__device__ __forceinline__ void w_apply_inv(const BFactor<TF>& f, int n, bool trans, WVec<NRC>& v, int nr, int lane,
                                            double* sbuf) {
  if (f.kind == 0) {
    if (!trans) {
      // P y: y_new[i] = y[perm[i]]
#pragma unroll
      for (int b = 0; b < BRB; ++b)
#pragma unroll
        for (int r = 0; r < NRC; ++r)
          if (r < nr && lane + 64 * b < n) sbuf[(lane + 64 * b) * BRM + r] = v.x[b][r];
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int b = 0; b < BRB; ++b) {
        const int i = lane + 64 * b;
        if (i < n) {
          const int src = f.perm[i];
#pragma unroll
          for (int r = 0; r < NRC; ++r)
            if (r < nr) v.x[b][r] = sbuf[src * BRM + r];
        }
      }
      __builtin_amdgcn_wave_barrier();
      w_trsv(f.M, f.ld, n, true, false, true, v, nr, lane, f.stg, f.scol);
      w_trsv(f.M, f.ld, n, false, false, false, v, nr, lane, f.stg, f.scol);
    } else {
      w_trsv(f.M, f.ld, n, false, true, false, v, nr, lane, f.stg, f.scol);
      w_trsv(f.M, f.ld, n, true, true, true, v, nr, lane, f.stg, f.scol);
      // P^T y: y_new[perm[i]] = y[i]
#pragma unroll
      for (int b = 0; b < BRB; ++b) {
        const int i = lane + 64 * b;
        if (i < n) {
          const int dst = f.perm[i];
#pragma unroll
          for (int r = 0; r < NRC; ++r)
            if (r < nr) sbuf[dst * BRM + r] = v.x[b][r];
        }
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int b = 0; b < BRB; ++b)
#pragma unroll
        for (int r = 0; r < NRC; ++r)
          if (r < nr && lane + 64 * b < n) v.x[b][r] = sbuf[(lane + 64 * b) * BRM + r];
      __builtin_amdgcn_wave_barrier();
    }
  } else if (f.kind == 1) {
    w_trsv(f.M, f.ld, n, true, false, false, v, nr, lane, f.stg, f.scol);
    w_trsv(f.M, f.ld, n, true, true, false, v, nr, lane, f.stg, f.scol);
  } else {
    w_trsv(f.M, f.ld, n, f.lower, trans, false, v, nr, lane, f.stg, f.scol);
  }
}

__device__ __forceinline__ double w_sum(const WVec<1>& v, int n, int lane) {
  double s = 0.0;
#pragma unroll
  for (int b = 0; b < BRB; ++b)
    if (lane + 64 * b < n) s += fabs(v.x[b][0]);
  return wave_sum(s);
}

// ||inv(A)||_1 by Hager's method as refined by Higham (the same steps as the single-system estimator)
template <class TF>
__device__ __forceinline__ double w_estimate(const BFactor<TF>& f, int n, int lane, double* sbuf, int& nsolves) {
  WVec<1> v;
  double xi[BRB];
#pragma unroll
  for (int b = 0; b < BRB; ++b) {
    xi[b] = 0.0;
    v.x[b][0] = (lane + 64 * b < n) ? 1.0 / n : 0.0;
  }
  nsolves = 0;
  w_apply_inv(f, n, false, v, 1, lane, sbuf);
  ++nsolves;
  if (n == 1) return fabs(read_lane(v.x[0][0], 0));
  double est = w_sum(v, n, lane);
#pragma unroll
  for (int b = 0; b < BRB; ++b) {
    xi[b] = v.x[b][0] >= 0.0 ? 1.0 : -1.0;
    v.x[b][0] = (lane + 64 * b < n) ? xi[b] : 0.0;
  }
  w_apply_inv(f, n, true, v, 1, lane, sbuf);
  ++nsolves;
  int iter = 2;
  int j = 0;
  auto argmax_abs = [&](const WVec<1>& z) -> int {
    double bv = -1.0;
    int bi = -1;
#pragma unroll
    for (int b = 0; b < BRB; ++b) {
      const int i = lane + 64 * b;
      if (i < n) {
        const double a = fabs(z.x[b][0]);
        if (bi < 0 || a > bv) { bv = a; bi = i; }
      }
    }
    wave_argmax(bv, bi);
    return bi;
  };
  auto value_at = [&](const WVec<1>& z, int i) -> double {
    double r = 0.0;
#pragma unroll
    for (int b = 0; b < BRB; ++b)
      if (i / 64 == b) r = read_lane(z.x[b][0], i % 64);
    return r;
  };
  j = argmax_abs(v);
  bool alt = false;
  while (true) {
    // y = inv(A) e_j
#pragma unroll
    for (int b = 0; b < BRB; ++b) v.x[b][0] = (lane + 64 * b == j) ? 1.0 : 0.0;
    w_apply_inv(f, n, false, v, 1, lane, sbuf);
    ++nsolves;
    const double est_old = est;
    est = w_sum(v, n, lane);
    int same = 1;
#pragma unroll
    for (int b = 0; b < BRB; ++b)
      if (lane + 64 * b < n && (v.x[b][0] >= 0.0 ? 1.0 : -1.0) != xi[b]) same = 0;
    same = __all(same) ? 1 : 0;
    if (same || est <= est_old) {
      alt = true;
      break;
    }
#pragma unroll
    for (int b = 0; b < BRB; ++b) {
      xi[b] = v.x[b][0] >= 0.0 ? 1.0 : -1.0;
      v.x[b][0] = (lane + 64 * b < n) ? xi[b] : 0.0;
    }
    w_apply_inv(f, n, true, v, 1, lane, sbuf);
    ++nsolves;
    const int jn = argmax_abs(v);
    const double zl = fabs(value_at(v, j));
    const double zmax = fabs(value_at(v, jn));
    if (zl != zmax && iter < 5) {
      ++iter;
      j = jn;
      continue;
    }
    alt = true;
    break;
  }
  if (alt) {
#pragma unroll
    for (int b = 0; b < BRB; ++b) {
      const int i = lane + 64 * b;
      v.x[b][0] = i < n ? ((i & 1) ? -1.0 : 1.0) * (1.0 + (double)i / (double)(n - 1)) : 0.0;
    }
    w_apply_inv(f, n, false, v, 1, lane, sbuf);
    ++nsolves;
    const double temp = 2.0 * (w_sum(v, n, lane) / (3.0 * n));
    if (temp > est) est = temp;
  }
  return est;
}

// ---------------------------------------------------------------- Jacobi SVD (four waves)
__device__ __forceinline__ void b_rr_pair(int m, int r, int pi, int& a, int& b) {
  if (pi == 0) {
    a = r;
    b = m - 1;
  } else {
    a = (r + pi) % (m - 1);
    b = (r - pi + m - 1) % (m - 1);
  }
}

// One-sided Jacobi on the n columns of U (ld n), round-robin pairs, the rotation rule and Rutishauser's
// formulas of the single-system route. Each quarter-wave (16 lanes) takes one pair at a time, so a
// workgroup has 16 pairs in flight; the two columns stay in registers between the dot products and the
// rotation (up to 16 elements per lane), and with PF the columns of the quarter's next pair of the same
// round are loaded while the current pair is rotated (PF = false: the kernel variant with half the
// registers loads each pair when it starts on it). Y (n x BRM, row j = the nr projections w_j^T c) takes
// every rotation as well.
constexpr int JQ = BNM / 16;  // elements of a column per lane of a quarter-wave
template <bool PF>
__device__ int b_jacobi(const BCtx c, gptr<double> U, gptr<double> Y, int nr, int n, int max_sweeps) {
  const int m = (n + 1) & ~1;
  const double tol = (double)n * kEps;
  const int q = c.lane >> 4, ql = c.lane & 15;  // quarter of the wave, lane in it
  const int slot = c.w * 4 + q;                 // 16 pair slots per workgroup
  const int npairs = m / 2;
  __shared__ int s_rot;
  int sweeps = 0;
  for (; sweeps < max_sweeps; ++sweeps) {
    if (c.t == 0) s_rot = 0;
    __syncthreads();
    int rot = 0;
    for (int r = 0; r < m - 1; ++r) {
      // pair pi of round r (pi = slot, slot + 16, ...): its columns p < qq, or live = false
      auto pair_of = [&](int pi, int& p, int& qq) -> bool {
        int a = 0, b = 0;
        bool live = pi < npairs;
        if (live) {
          b_rr_pair(m, r, pi, a, b);
          live = a < n && b < n;
        }
        p = min(a, b);
        qq = max(a, b);
        return live;
      };
      auto load = [&](bool live, int p, int qq, double* x, double* y) {
        gptr<const double> up = U + (size_t)p * n;
        gptr<const double> uq = U + (size_t)qq * n;
#pragma unroll
        for (int k = 0; k < JQ; ++k) {
          const int i = ql + 16 * k;
          x[k] = (live && i < n) ? up[i] : 0.0;
          y[k] = (live && i < n) ? uq[i] : 0.0;
        }
      };
      int pn = 0, qn = 0;
      bool liven = false;
      double xn[PF ? JQ : 1], yn[PF ? JQ : 1];
      if (PF) {
        liven = pair_of(slot, pn, qn);
        load(liven, pn, qn, xn, yn);
      }
      for (int pi = slot; pi < npairs; pi += 16) {
        int p, qq;
        bool live;
        double x[JQ], y[JQ];
        if (PF) {
          p = pn;
          qq = qn;
          live = liven;
#pragma unroll
          for (int k = 0; k < JQ; ++k) {
            x[k] = xn[PF ? k : 0];
            y[k] = yn[PF ? k : 0];
          }
          if (pi + 16 < npairs) {  // the next pair's columns are disjoint from this one's
            liven = pair_of(pi + 16, pn, qn);
            load(liven, pn, qn, xn, yn);
          }
        } else {
          live = pair_of(pi, p, qq);
          load(live, p, qq, x, y);
        }
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int k = 0; k < JQ; ++k) {
          al = fma(x[k], x[k], al);
          be = fma(y[k], y[k], be);
          ga = fma(x[k], y[k], ga);
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
          al += __shfl_xor(al, o, 64);
          be += __shfl_xor(be, o, 64);
          ga += __shfl_xor(ga, o, 64);
        }
        if (live && fabs(ga) > tol * sqrt(al) * sqrt(be)) {
          const double zeta = (be - al) / (2.0 * ga);
          const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
          const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
          gptr<double> up = U + (size_t)p * n;
          gptr<double> uq = U + (size_t)qq * n;
#pragma unroll
          for (int k = 0; k < JQ; ++k) {
            const int i = ql + 16 * k;
            if (i < n) {
              up[i] = cs * x[k] - sn * y[k];
              uq[i] = sn * x[k] + cs * y[k];
            }
          }
          // the same rotation on the projections y_j = w_j^T c (the accumulated rotations W are not needed)
          if (ql < nr) {
            gptr<double> yp = Y + (size_t)p * BRM + ql;
            gptr<double> yq = Y + (size_t)qq * BRM + ql;
            const double xv = *yp, yv = *yq;
            *yp = cs * xv - sn * yv;
            *yq = sn * xv + cs * yv;
          }
          rot = 1;
        }
      }
      __syncthreads();
    }
    rot = wave_or(rot);
    if (c.lane == 0 && rot) s_rot = 1;
    __syncthreads();
    const int any = s_rot;
    __syncthreads();
    if (!any) {
      ++sweeps;
      break;
    }
  }
  return sweeps;
}

// Sum over the 16 lanes of a quarter-wave by DPP exchanges within rows of 16 (lane i^1, i^2, then the
// mirror images in 8 and in 16); every lane of the quarter ends with the same value.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double quarter_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return v;
}

// Jacobi rotations of NP disjoint column pairs (p[j], q[j]) of S (LDS, n rows, ld n) by one quarter-wave
// (lane ql of 16), the pairs' loads and arithmetic interleaved; rows p and q of the projections Ys (LDS, BRM
// per row) along; the rotation rule and Rutishauser's formulas of b_jacobi. live[j] = false skips pair j.
// Returns whether any pair rotated (the same in every lane of the quarter).
template <int NP>
__device__ __forceinline__ bool q_rotate_lds(lptr<double> S, lptr<double> Ys, const int* p, const int* q,
                                             const bool* live, int n, int nr, int ql, double tol) {
  double x[NP][JQ], y[NP][JQ];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    lptr<double> sp = S + p[j] * n;
    lptr<double> sq = S + q[j] * n;
#pragma unroll
    for (int k = 0; k < JQ; ++k) {
      const int i = ql + 16 * k;
      x[j][k] = (live[j] && i < n) ? sp[i] : 0.0;
      y[j][k] = (live[j] && i < n) ? sq[i] : 0.0;
    }
  }
  bool any = false;
  double al[NP], be[NP], ga[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    al[j] = be[j] = ga[j] = 0.0;
#pragma unroll
    for (int k = 0; k < JQ; ++k) {
      al[j] = fma(x[j][k], x[j][k], al[j]);
      be[j] = fma(y[j][k], y[j][k], be[j]);
      ga[j] = fma(x[j][k], y[j][k], ga[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    al[j] = quarter_sum(al[j]);
    be[j] = quarter_sum(be[j]);
    ga[j] = quarter_sum(ga[j]);
  }
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    if (!(live[j] && fabs(ga[j]) > tol * sqrt(al[j]) * sqrt(be[j]))) continue;
    const double zeta = (be[j] - al[j]) / (2.0 * ga[j]);
    const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
    const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
    lptr<double> sp = S + p[j] * n;
    lptr<double> sq = S + q[j] * n;
#pragma unroll
    for (int k = 0; k < JQ; ++k) {
      const int i = ql + 16 * k;
      if (i < n) {
        sp[i] = cs * x[j][k] - sn * y[j][k];
        sq[i] = sn * x[j][k] + cs * y[j][k];
      }
    }
    if (ql < nr) {
      const double xv = Ys[p[j] * BRM + ql], yv = Ys[q[j] * BRM + ql];
      Ys[p[j] * BRM + ql] = cs * xv - sn * yv;
      Ys[q[j] * BRM + ql] = sn * xv + cs * yv;
    }
    any = true;
  }
  return any;
}

// q_rotate_lds for pairs whose first columns a quarter-wave holds in registers (xr[j]: its 16 elements of
// lane ql; yr[j]: the first column's projection on lane ql < nr), updated in place; the second columns q[j]
// and their projection rows are in S and Ys.
template <int NP>
__device__ __forceinline__ bool q_rotate_xreg(double (&xr)[NP][JQ], double (&yr)[NP], lptr<double> S,
                                              lptr<double> Ys, const int* q, const bool* live, int n, int nr,
                                              int ql, double tol) {
  double y[NP][JQ];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    lptr<double> sq = S + q[j] * n;
#pragma unroll
    for (int k = 0; k < JQ; ++k) {
      const int i = ql + 16 * k;
      y[j][k] = (live[j] && i < n) ? sq[i] : 0.0;
    }
  }
  bool any = false;
  double al[NP], be[NP], ga[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    al[j] = be[j] = ga[j] = 0.0;
#pragma unroll
    for (int k = 0; k < JQ; ++k) {
      al[j] = fma(xr[j][k], xr[j][k], al[j]);
      be[j] = fma(y[j][k], y[j][k], be[j]);
      ga[j] = fma(xr[j][k], y[j][k], ga[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    al[j] = quarter_sum(al[j]);
    be[j] = quarter_sum(be[j]);
    ga[j] = quarter_sum(ga[j]);
  }
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    if (!(live[j] && fabs(ga[j]) > tol * sqrt(al[j]) * sqrt(be[j]))) continue;
    const double zeta = (be[j] - al[j]) / (2.0 * ga[j]);
    const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
    const double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
    lptr<double> sq = S + q[j] * n;
#pragma unroll
    for (int k = 0; k < JQ; ++k) {
      const int i = ql + 16 * k;
      const double xv = xr[j][k];
      xr[j][k] = cs * xv - sn * y[j][k];
      if (i < n) sq[i] = sn * xv + cs * y[j][k];
    }
    if (ql < nr) {
      const double xv = yr[j], yv = Ys[q[j] * BRM + ql];
      yr[j] = cs * xv - sn * yv;
      Ys[q[j] * BRM + ql] = sn * xv + cs * yv;
    }
    any = true;
  }
  return any;
}

// One-sided Jacobi of b_jacobi for a matrix U in HBM, by blocks of JB columns staged in LDS: a sweep takes
// each block in turn, rotates the pairs inside it (round robin over its columns), then the JB * JB pairs
// across it and each later block (JB rounds; round r pairs column k of the first with column (k + r) mod JB
// of the second), so every pair of columns once per sweep. The first block stays in LDS (S columns 0..JB-1)
// while the later ones pass through S columns JB..2JB-1, with their rows of Y in Ys (2 * JB * BRM doubles);
// a block goes back to HBM when a rotation changed it. Sixteen quarter-waves take the pairs of a round.
constexpr int JB = 32;
__device__ int b_jacobi_blk(const BCtx c, gptr<double> U, gptr<double> Y, int nr, int n, int max_sweeps,
                            lptr<double> S, lptr<double> Ys) {
  const double tol = (double)n * kEps;
  const int ql = c.lane & 15;
  const int slot = c.w * 4 + (c.lane >> 4);
  const int nbk = (n + JB - 1) / JB;
  __shared__ int s_any;
  // columns c0 .. c0+cnt-1 of U (contiguous, cnt * n doubles) <-> S columns s0 .., and their rows of Y
  auto stage = [&](int c0, int cnt, int s0, bool in) {
    gptr<double> g = U + (size_t)c0 * n;
    lptr<double> l = S + s0 * n;
    const int tot = cnt * n;
    if (in) {
#pragma unroll 16
      for (int e = c.t; e < tot; e += BT) l[e] = g[e];
      for (int e = c.t; e < cnt * BRM; e += BT) Ys[s0 * BRM + e] = Y[(size_t)c0 * BRM + e];
    } else {
#pragma unroll 16
      for (int e = c.t; e < tot; e += BT) g[e] = l[e];
      for (int e = c.t; e < cnt * BRM; e += BT) Y[(size_t)c0 * BRM + e] = Ys[s0 * BRM + e];
    }
  };
  // every thread learns whether any quarter rotated (any: this thread's flag); resets the flag after use
  auto any_of = [&](int any) -> bool {
    if (wave_or(any) && c.lane == 0) s_any = 1;
    __syncthreads();
    const bool r = s_any != 0;
    __syncthreads();
    if (c.t == 0) s_any = 0;
    return r;
  };
  if (c.t == 0) s_any = 0;
  int sweeps = 0;
  for (; sweeps < max_sweeps; ++sweeps) {
    bool rot = false;
    for (int bi = 0; bi < nbk; ++bi) {
      const int c0 = bi * JB, cnt0 = min(JB, n - c0);
      __syncthreads();  // the previous write-back has read S
      stage(c0, cnt0, 0, true);
      __syncthreads();
      int any = 0;
      const int m = (cnt0 + 1) & ~1;
      for (int r = 0; r < m - 1; ++r) {
        if (slot < m / 2) {
          int a = 0, b = 0;
          b_rr_pair(m, r, slot, a, b);
          const int pp = min(a, b), qq = max(a, b);
          const bool lv = a < cnt0 && b < cnt0;
          any |= q_rotate_lds<1>(S, Ys, &pp, &qq, &lv, n, nr, ql, tol);
        }
        __syncthreads();
      }
      bool dirty0 = any_of(any);
      // the cross rounds: this quarter's first columns (slot, slot + 16 of the block) and their projections
      // stay in registers for all the later blocks
      double xr[2][JQ], yr[2];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        lptr<double> sp = S + (slot + 16 * j) * n;
#pragma unroll
        for (int k = 0; k < JQ; ++k) {
          const int i = ql + 16 * k;
          xr[j][k] = i < n ? sp[i] : 0.0;
        }
        yr[j] = ql < nr ? Ys[(slot + 16 * j) * BRM + ql] : 0.0;
      }
      for (int bj = bi + 1; bj < nbk; ++bj) {
        const int c1 = bj * JB, cnt1 = min(JB, n - c1);
        stage(c1, cnt1, JB, true);
        __syncthreads();
        any = 0;
        for (int r = 0; r < JB; ++r) {
          int qq[2];
          bool lv[2];
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const int k = slot + 16 * j, b = (k + r) & (JB - 1);
            qq[j] = JB + b;
            lv[j] = k < cnt0 && b < cnt1;
          }
          any |= q_rotate_xreg<2>(xr, yr, S, Ys, qq, lv, n, nr, ql, tol);
          __syncthreads();
        }
        if (any_of(any)) {
          dirty0 = true;
          stage(c1, cnt1, JB, false);
        }
        __syncthreads();  // the write-back has read S before the next block comes in
      }
      // the first block's columns back into S (for its write-back)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        lptr<double> sp = S + (slot + 16 * j) * n;
#pragma unroll
        for (int k = 0; k < JQ; ++k) {
          const int i = ql + 16 * k;
          if (i < n && slot + 16 * j < cnt0) sp[i] = xr[j][k];
        }
        if (ql < nr && slot + 16 * j < cnt0) Ys[(slot + 16 * j) * BRM + ql] = yr[j];
      }
      __syncthreads();
      if (dirty0) {
        rot = true;
        stage(c0, cnt0, 0, false);
      }
    }
    __syncthreads();  // the last write-back is complete
    if (!rot) {
      ++sweeps;
      break;
    }
  }
  return sweeps;
}

// ---------------------------------------------------------------- the solve of one system
// Householder QR of M (n x n, ld n) in place, reflectors below the diagonal, tau[n] (LDS); the same
// reflectors applied to the ncol columns of C (ld ldc). Reflector k maps M[k.., k] to (beta, 0, ...):
// beta = -sign(alpha) ||M[k.., k]||, tau_k = (beta - alpha) / beta, v = (1, M[k+1.., k] / (alpha - beta));
// tau_k = 0 when the part below the diagonal is zero. Columns are updated one per wave.
template <int QB>
__device__ void b_house_qr(const BCtx c, gptr<double> M, int n, lptr<double> tau, gptr<double> C, int ldc,
                           int ncol) {
  for (int k = 0; k < n; ++k) {
    gptr<double> col = M + (size_t)k * n;
    double s = 0.0;
    for (int i = k + 1 + c.t; i < n; i += BT) s = fma(col[i], col[i], s);
    const double sig2 = b_sum(c, s);
    const double alpha = col[k];
    double tk = 0.0, sc = 1.0, beta = alpha;
    if (sig2 != 0.0) {
      beta = -copysign(sqrt(alpha * alpha + sig2), alpha);
      tk = (beta - alpha) / beta;
      sc = 1.0 / (alpha - beta);
    }
    __syncthreads();  // every thread has read alpha
    for (int i = k + 1 + c.t; i < n; i += BT) col[i] *= sc;
    if (c.t == 0) {
      col[k] = beta;
      tau[k] = tk;
    }
    __syncthreads();
    if (tk != 0.0) {
      // wave w updates the columns q = w, w + 4, ...; QB of them at a time so that their loads are in flight
      // together (per column the same operations in the same order as one at a time)
      const int ncols = (n - k - 1) + ncol;
      double v[BRB];  // the reflector on this lane's rows k + 1 + lane + 64 j
#pragma unroll
      for (int j = 0; j < BRB; ++j) {
        const int i = k + 1 + c.lane + 64 * j;
        v[j] = i < n ? col[i] : 0.0;
      }
      for (int q0 = c.w; q0 < ncols; q0 += QB * (BT / 64)) {
        auto colp = [&](int q) {
          return q < n - k - 1 ? M + (size_t)(k + 1 + q) * n : C + (size_t)(q - (n - k - 1)) * ldc;
        };
        double av[QB][BRB], ak[QB];
#pragma unroll
        for (int cb = 0; cb < QB; ++cb) {
          const int q = q0 + cb * (BT / 64);
          const bool live = q < ncols;
          gptr<double> a = colp(live ? q : 0);
          ak[cb] = live ? a[k] : 0.0;
#pragma unroll
          for (int j = 0; j < BRB; ++j) {
            const int i = k + 1 + c.lane + 64 * j;
            av[cb][j] = (live && i < n) ? a[i] : 0.0;
          }
        }
#pragma unroll
        for (int cb = 0; cb < QB; ++cb) {
          const int q = q0 + cb * (BT / 64);
          double dd = 0.0;
#pragma unroll
          for (int j = 0; j < BRB; ++j)
            if (k + 1 + c.lane + 64 * j < n) dd = fma(v[j], av[cb][j], dd);
          dd = (wave_sum(dd) + ak[cb]) * tk;
          if (q < ncols) {
            gptr<double> a = colp(q);
            if (c.lane == 0) a[k] = ak[cb] - dd;
#pragma unroll
            for (int j = 0; j < BRB; ++j) {
              const int i = k + 1 + c.lane + 64 * j;
              if (i < n) a[i] = fma(-dd, v[j], av[cb][j]);
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

// One launch takes the systems of one range of orders (the systems at order[range[0] .. range[1]), all of
// order <= hi). OCC: workgroups per compute unit the register budget allows (1: 512 registers per lane,
// 2: 256). scol: columns of a triangle in HBM a wave stages into LDS at a time.
template <int OCC>
__global__ __launch_bounds__(BT, OCC) void k_solve_batched(const BDesc* __restrict__ desc,
                                                           const double* __restrict__ Apool,
                                                           const double* __restrict__ Bpool, double* Xpool,
                                                           char* work, ada_opts o, ada_result* results,
                                                           unsigned* queue, const int* __restrict__ order,
                                                           const int* __restrict__ range, int hi, int scol) {
  extern __shared__ double lds[];  // matrix region (b_lds_matrix(hi)), then hi * BRM vector buffer
  __shared__ double s_red[8];
  __shared__ int s_ired[8];
  __shared__ int s_idx;
  BCtx c;
  c.t = threadIdx.x;
  c.lane = c.t & 63;
  c.w = c.t >> 6;
  c.red = as_lds(s_red);
  c.ired = as_lds(s_ired);
  double* sbuf = lds + b_lds_matrix(hi);
  char* slice = work + (size_t)blockIdx.x * b_slice_bytes(hi);
  double* gW = reinterpret_cast<double*>(slice);
  double* gV = gW + (size_t)hi * hi;
  double* gX = gV + (size_t)hi * hi;         // BNM * BRM
  int* perm = reinterpret_cast<int*>(gW + b_slice_doubles(hi));
  const int first = range[0], last = range[1];
  const double thr = o.rcond_threshold >= 0.0 ? o.rcond_threshold : 0.5 * kEps;

  while (true) {
    if (c.t == 0) s_idx = first + (int)atomicAdd(queue, 1u);
    __syncthreads();
    const int idx = s_idx;
    __syncthreads();
    if (idx >= last) break;
    const int sys = order[idx];  // largest systems first
    const BDesc d = desc[sys];
    ada_result res;
    res.cls = ADA_CLASS_GENERAL;
    res.kl = -1;
    res.ku = -1;
    res.route = ADA_ROUTE_NONE;
    res.chol_failed = 0;
    res.fallback = ADA_FALLBACK_NONE;
    res.info = 0;
    res.rank = d.n;
    res.sweeps = 0;
    res.nsolves = 0;
    res.refine_iters = 0;
    res.status = ADA_OK;
    res.rcond = __longlong_as_double(0x7ff8000000000000LL);
    res.berr = __longlong_as_double(0x7ff8000000000000LL);
    const int n = d.n, nr = d.nrhs;
    if (n < 1 || n > hi || nr < 1 || nr > BRM || d.lda < n || d.ldb < n || d.ldx < n) {
      res.status = ADA_ERR_ARG;
      if (c.t == 0) results[sys] = res;
      continue;
    }
    const double* A = Apool + d.a_off;
    const double* B = Bpool + d.b_off;
    double* X = Xpool + d.x_off;
    // the matrix is held in LDS up to order BNL (FP32 copy: BNL32); the variant with two workgroups per
    // compute unit only takes orders <= 96 (the launch's range), so it compiles the LDS paths alone
    const bool lds64 = OCC == 2 || n <= BNL, lds32 = OCC == 2 || n <= BNL32;
    double* M = lds64 ? lds : gW;  // working matrix, ld n
    // ---- S1/S2: copy A to the working matrix (coalesced), non-finite check, band scan, norms
    int nf = 0;
    for (int e = c.t; e < n * n; e += BT) {
      const double a = A[e % n + (size_t)(e / n) * d.lda];
      nf |= !isfinite(a);
      M[e] = a;
    }
    for (int e = c.t; e < n * nr; e += BT) nf |= !isfinite(B[e % n + (size_t)(e / n) * d.ldb]);
    nf = b_or(c, nf);  // (its barriers also publish M)
    if (nf) {
      res.status = ADA_ERR_NONFINITE;
      if (c.t == 0) results[sys] = res;
      continue;
    }
    int klj = 0, kuj = 0;
    double colsum = 0.0, rowsum = 0.0;
    for (int j = c.t; j < n; j += BT) {
      double cs = 0.0, rs = 0.0;
#pragma unroll 8
      for (int i = 0; i < n; ++i) {
        const double a = M[i + j * n];
        cs += fabs(a);
        if (a != 0.0) {
          if (i < j) kuj = max(kuj, j - i);
          if (i > j) klj = max(klj, i - j);
        }
        rs += fabs(M[j + i * n]);
      }
      colsum = fmax(colsum, cs);
      rowsum = fmax(rowsum, rs);
    }
    const int kl = b_max_int(c, klj), ku = b_max_int(c, kuj);
    const double anorm1 = b_max(c, colsum);
    const double anorm_inf = b_max(c, rowsum);
    int cls = ADA_CLASS_GENERAL;
    if (!o.force_general) {
      res.kl = kl;
      res.ku = ku;
      const long long nn = n;
      const long long nnz = nn * (kl + ku + 1) - (long long)kl * (kl + 1) / 2 - (long long)ku * (ku + 1) / 2;
      if (4 * nnz <= nn * nn) cls = ADA_CLASS_BANDED;
      else if (kl == 0) cls = ADA_CLASS_TRI_UPPER;
      else if (ku == 0) cls = ADA_CLASS_TRI_LOWER;
      else {
        // S5: Fig. 4 (tol = 100 eps)
        const double tol = 100.0 * kEps;
        int bad = 0;
        double md = 0.0;
        for (int j = c.t; j < n; j += BT) {
          const double dj = M[j + j * n];
          if (dj <= 0.0) bad = 1;
          md = fmax(md, dj);
        }
        bad = b_or(c, bad);
        const double max_diag = b_max(c, md);
        if (!bad) {
          for (int j = c.t; j < n; j += BT) {
            const double ajj = M[j + j * n];
#pragma unroll 8
            for (int i = j + 1; i < n; ++i) {
              const double aij = M[i + j * n], aji = M[j + i * n];
              const double delta = fabs(aij - aji);
              if (delta > tol && delta > tol * fmax(fabs(aij), fabs(aji))) bad = 1;
              if (fabs(aij) >= max_diag) bad = 1;
              if ((fabs(aij) + fabs(aji)) >= (M[i + i * n] + ajj)) bad = 1;
            }
          }
          bad = b_or(c, bad);
        }
        cls = bad ? ADA_CLASS_GENERAL : ADA_CLASS_SYMPD;
      }
    }
    res.cls = cls;
    // ---- FP32 factorisation with FP64 iterative refinement (precision option): the class and the
    // route are the FP64 decisions above; residuals, corrections and the condition estimate are FP64
    // arithmetic on FP32 factors; a refinement that does not reach sqrt(n)*eps in backward error
    // (stagnation, a non-finite value, or the step limit) hands the system to the FP64 route.
    __shared__ int s_flag;
    __shared__ double s_rc;
    __shared__ double s_est;  // condition estimate of the FP32 factors
    __shared__ int s_ns;
    bool mixed_ok = false;
    bool m_clobbered = false;
    int refine = 0;
    const bool sym_class = cls == ADA_CLASS_SYMPD;
    double anorm = anorm1;
    if (sym_class) {
      // ||A||_1 of the symmetric matrix the lower triangle defines
      double s = 0.0;
      for (int j = c.t; j < n; j += BT) {
        double q = 0.0;
        for (int i = 0; i < j; ++i) q += fabs(A[j + (size_t)i * d.lda]);
#pragma unroll 8
        for (int i = j; i < n; ++i) q += fabs(A[i + (size_t)j * d.lda]);
        s = fmax(s, q);
      }
      anorm = b_max(c, s);
    }
    if (o.precision == ADA_PREC_FP32_IR &&
        (cls == ADA_CLASS_SYMPD || cls == ADA_CLASS_GENERAL || cls == ADA_CLASS_BANDED)) {
      float* M32 = lds32 ? reinterpret_cast<float*>(lds) : reinterpret_cast<float*>(gV);
      m_clobbered = lds64;  // the FP64 copy shared the LDS region
      for (int e = c.t; e < n * n; e += BT) M32[e] = (float)A[e % n + (size_t)(e / n) * d.lda];
      __syncthreads();
      BFactor<float> g;
      g.M = M32;
      g.ld = n;
      g.perm = perm;
      g.lower = false;
      g.stg = lds32 ? nullptr : reinterpret_cast<float*>(lds);
      g.scol = 64;  // wave 0 alone solves on this route: the whole staging region
      int ok;
      if (sym_class) {
        ok = (lds32 ? b_potrf<float>(c, as_lds(M32), n)
                          : b_potrf_blk<float>(c, as_global(M32), n, as_lds(reinterpret_cast<float*>(lds)))) == 0;
        g.kind = 1;
      } else {
        ok = (lds32 ? b_getrf<float>(c, as_lds(M32), n, as_global(perm))
                         : b_getrf_blk<float>(c, as_global(M32), n, as_global(perm),
                                              as_lds(reinterpret_cast<float*>(lds)))) == 0;
        g.kind = 0;
      }
      __syncthreads();
      refine = -1;  // the FP32 factorisation failed
      if (ok) {
        const double tol = sqrt((double)n) * kEps;
        double* Rv = gX;  // residuals, BNM x BRM
        BFactor<float> gw = g;
        if (g.stg) {
          gw.stg = g.stg + (size_t)c.w * scol * BNM;
          gw.scol = scol;
        }
        double* sbw = sbuf + c.w;
        // the condition estimate (wave 0) beside x0 = solve(b) for every right-hand side (waves 1-3)
        if (c.w == 0) {
          int ns = 0;
          const double est = w_estimate(gw, n, c.lane, sbw, ns);
          if (c.lane == 0) {
            s_est = est;
            s_ns = ns;
          }
        } else {
          for (int r0 = c.w - 1; r0 < nr; r0 += BT / 64 - 1) {
            WVec<1> v;
#pragma unroll
            for (int b = 0; b < BRB; ++b) {
              const int ii = c.lane + 64 * b;
              v.x[b][0] = ii < n ? B[ii + (size_t)r0 * d.ldb] : 0.0;
            }
            w_apply_inv(gw, n, false, v, 1, c.lane, sbw);
#pragma unroll
            for (int b = 0; b < BRB; ++b) {
              const int ii = c.lane + 64 * b;
              if (ii < n) X[ii + (size_t)r0 * d.ldx] = v.x[b][0];
            }
          }
        }
        __syncthreads();
        // refinement of all right-hand sides together: residuals by every thread, corrections shared by the
        // waves; each column keeps its own stopping test (every thread holds the same per-column state)
        // factors whose condition estimate puts kappa_1 beyond 1e9 (kappa_1 * u32 > 50) are not refined:
        // such systems go to the FP64 route at once
        const double rc32 = (anorm > 0.0 && s_est > 0.0) ? (1.0 / s_est) / anorm : 0.0;
        const bool hopeless = !(rc32 >= kRcondRefine);
        double prev[BRM];
        int act[BRM], conv[BRM], its[BRM];
#pragma unroll
        for (int r = 0; r < BRM; ++r) {
          prev[r] = INFINITY;
          act[r] = r < nr && !hopeless;
          conv[r] = 0;
          its[r] = 0;
        }
        for (;;) {
          int any = 0;
#pragma unroll
          for (int r = 0; r < BRM; ++r) any |= act[r];
          if (!any) break;
          double rn[BRM], xn[BRM], bn[BRM];
          int bad[BRM];
#pragma unroll
          for (int r = 0; r < BRM; ++r) {
            rn[r] = xn[r] = bn[r] = 0.0;
            bad[r] = 0;
          }
          for (int ii = c.t; ii < n; ii += BT) {
#pragma unroll
            for (int r = 0; r < BRM; ++r) {
              if (act[r]) {
                const double bi = B[ii + (size_t)r * d.ldb];
                double sres = bi;
#pragma unroll 8
                for (int j = 0; j < n; ++j) sres = fma(-A[ii + (size_t)j * d.lda], X[j + (size_t)r * d.ldx], sres);
                Rv[ii + (size_t)r * BNM] = sres;
                const double xi = X[ii + (size_t)r * d.ldx];
                bad[r] |= !isfinite(xi) || !isfinite(sres);
                rn[r] = fmax(rn[r], fabs(sres));
                xn[r] = fmax(xn[r], fabs(xi));
                bn[r] = fmax(bn[r], fabs(bi));
              }
            }
          }
          unsigned cmask = 0;  // columns that take a correction this step
#pragma unroll
          for (int r = 0; r < BRM; ++r) {
            if (act[r]) {
              const double rr = b_max(c, rn[r]), xx = b_max(c, xn[r]), bb = b_max(c, bn[r]);
              const int bd = b_or(c, bad[r]);
              const double den = anorm_inf * xx + bb;
              const double eta = bd ? __longlong_as_double(0x7ff8000000000000LL)
                                    : (den > 0.0 ? rr / den : (rr > 0.0 ? INFINITY : 0.0));
              if (eta <= tol) {
                act[r] = 0;
                conv[r] = 1;
              } else if (!(eta <= 0.5 * prev[r]) || its[r] == kMaxRefine) {
                act[r] = 0;  // stalled: the system goes to the FP64 route
              } else {
                prev[r] = eta;
                ++its[r];
                cmask |= 1u << r;
              }
            }
          }
          // corrections x += solve(r), the k-th column to correct on wave k mod 4
          int k = 0;
#pragma unroll
          for (int r = 0; r < BRM; ++r) {
            if ((cmask >> r) & 1u) {
              if ((k & 3) == c.w) {
                WVec<1> v;
#pragma unroll
                for (int b = 0; b < BRB; ++b) {
                  const int ii = c.lane + 64 * b;
                  v.x[b][0] = ii < n ? Rv[ii + (size_t)r * BNM] : 0.0;
                }
                w_apply_inv(gw, n, false, v, 1, c.lane, sbw);
#pragma unroll
                for (int b = 0; b < BRB; ++b) {
                  const int ii = c.lane + 64 * b;
                  if (ii < n) X[ii + (size_t)r * d.ldx] += v.x[b][0];
                }
              }
              ++k;
            }
          }
          __syncthreads();
        }
        int conv_all = 1;
        refine = 0;
#pragma unroll
        for (int r = 0; r < BRM; ++r) {
          if (r < nr) {
            conv_all &= conv[r];
            refine = max(refine, its[r]);
          }
        }
        mixed_ok = conv_all && !hopeless;
        if (!mixed_ok) refine = -1 - refine;
      }
      if (mixed_ok) {
        res.route = sym_class ? ADA_ROUTE_CHOL : (cls == ADA_CLASS_BANDED ? ADA_ROUTE_BAND_LU : ADA_ROUTE_LU);
        res.nsolves = s_ns;
        const double est = s_est;
        double rcond;
        if (anorm == 0.0) rcond = 0.0;
        else if (est != est) rcond = est;
        else if (est == 0.0) rcond = 0.0;
        else rcond = (1.0 / est) / anorm;
        int fb = ADA_FALLBACK_NONE;
        if (rcond != rcond) fb = ADA_FALLBACK_RCOND_NAN;
        else if (rcond < thr) fb = ADA_FALLBACK_RCOND;
        res.fallback = fb;
        res.rcond = rcond;
        res.info = 0;
      }
      res.refine_iters = refine;
    }
    int info = 0;
    if (!mixed_ok) {
      // ---- S6: routed factorisation
      BFactor<double> f;
      f.M = M;
      f.ld = n;
      f.perm = perm;
      f.lower = false;
      f.stg = lds64 ? nullptr : lds;  // the LDS matrix region is free when the matrix lives in HBM
      f.scol = 64;
      bool routed_sym = false;
      if (m_clobbered) {
        for (int e = c.t; e < n * n; e += BT) M[e] = A[e % n + (size_t)(e / n) * d.lda];
        __syncthreads();
      }
      if (cls == ADA_CLASS_TRI_UPPER || cls == ADA_CLASS_TRI_LOWER) {
        res.route = ADA_ROUTE_TRI;
        f.kind = 2;
        f.lower = cls == ADA_CLASS_TRI_LOWER;
        int z = INT_MAX;
        for (int j = c.t; j < n; j += BT)
          if (M[j + j * n] == 0.0) z = min(z, j);
        z = -b_max_int(c, z == INT_MAX ? -INT_MAX : -z);
        info = (z == INT_MAX) ? 0 : z + 1;
      } else {
        bool fresh = true;  // M still holds A
        if (cls == ADA_CLASS_SYMPD) {
          const int ci = lds64 ? b_potrf(c, as_lds(M), n) : b_potrf_blk(c, as_global(M), n, as_lds(lds));
          fresh = false;
          __syncthreads();
          if (ci == 0) {
            res.route = ADA_ROUTE_CHOL;
            f.kind = 1;
            routed_sym = true;
          } else {
            res.chol_failed = 1;
          }
        }
        if (!routed_sym) {
          res.route = (cls == ADA_CLASS_BANDED) ? ADA_ROUTE_BAND_LU : ADA_ROUTE_LU;
          if (!fresh) {
            for (int e = c.t; e < n * n; e += BT) M[e] = A[e % n + (size_t)(e / n) * d.lda];
            __syncthreads();
          }
          info = lds64 ? b_getrf(c, as_lds(M), n, as_global(perm))
                          : b_getrf_blk(c, as_global(M), n, as_global(perm), as_lds(lds));
          __syncthreads();
          f.kind = 0;
        }
      }
      const double anorm_r = routed_sym ? anorm : anorm1;  // LU after a failed Cholesky: the full matrix
      res.info = info;
      // ---- condition estimate (wave 0) beside the solves of the right-hand sides (waves 1-3, one right-hand
      // side each in turn): each wave has its own staging quarter and its own slot of sbuf's rows
      __shared__ int s_xnf;
      if (c.t == 0) s_xnf = 0;
      __syncthreads();
      BFactor<double> fw = f;
      if (f.stg) {
        fw.stg = f.stg + (size_t)c.w * scol * BNM;
        fw.scol = scol;
      }
      double* sbw = sbuf + c.w;
      double rcond = __longlong_as_double(0x7ff8000000000000LL);
      if (info == 0) {
        if (c.w == 0) {
          int ns = 0;
          const double est = w_estimate(fw, n, c.lane, sbw, ns);
          res.nsolves = ns;
          if (anorm_r == 0.0) rcond = 0.0;
          else if (est != est) rcond = est;
          else if (est == 0.0) rcond = 0.0;
          else rcond = (1.0 / est) / anorm_r;
        } else {
          int xnf = 0;
          for (int r0 = c.w - 1; r0 < nr; r0 += BT / 64 - 1) {  // one right-hand side at a time per wave
            WVec<1> v;
#pragma unroll
            for (int b = 0; b < BRB; ++b) {
              const int i = c.lane + 64 * b;
              v.x[b][0] = i < n ? B[i + (size_t)r0 * d.ldb] : 0.0;
            }
            w_apply_inv(fw, n, false, v, 1, c.lane, sbw);
#pragma unroll
            for (int b = 0; b < BRB; ++b) {
              const int i = c.lane + 64 * b;
              if (i < n) {
                X[i + (size_t)r0 * d.ldx] = v.x[b][0];
                xnf |= !isfinite(v.x[b][0]);
              }
            }
          }
          xnf = wave_or(xnf);
          if (c.lane == 0 && xnf) atomicOr(&s_xnf, 1);
        }
      }
      __syncthreads();
      if (c.t == 0) {
        int fb = ADA_FALLBACK_NONE;
        if (info || s_xnf) fb = ADA_FALLBACK_FAILURE;
        else if (rcond != rcond) fb = ADA_FALLBACK_RCOND_NAN;
        else if (rcond < thr) fb = ADA_FALLBACK_RCOND;
        s_flag = fb;
        s_rc = rcond;
      }
      __syncthreads();
      res.fallback = s_flag;
      res.rcond = info ? __longlong_as_double(0x7ff8000000000000LL) : s_rc;
      __syncthreads();
    }
    bool svd = false;
    if (res.fallback != ADA_FALLBACK_NONE) {
      if (o.no_approx) {
        res.status = ADA_ERR_SINGULAR;
      } else {
        svd = true;
      }
    }
    if (svd) {
      // ---- S8: SVD of the original A, min-norm least squares. A P = Q R (columns by decreasing norm,
      // Householder, reflectors in gV), C = Q^T B (gX), then one-sided Jacobi on R^T (gW): R^T W = U~,
      // sigma_j = ||u~_j||, x = P sum over kept j of u~_j (w_j^T C) / sigma_j^2, where the projections
      // w_j^T C are rotated along with the columns instead of accumulating W
      res.route = ADA_ROUTE_SVD;
      double* C = gX;              // BNM x BRM
      double* tau = lds;           // n (the LDS matrix region is free here)
      // columns by decreasing norm: perm[k] = source column of position k (ties to the lower index)
      double* cn = sbuf;  // n
      for (int j = c.t; j < n; j += BT) {
        double q = 0.0;
#pragma unroll 8
        for (int i = 0; i < n; ++i) q = fma(A[i + (size_t)j * d.lda], A[i + (size_t)j * d.lda], q);
        cn[j] = sqrt(q);
      }
      __syncthreads();
      for (int j = c.t; j < n; j += BT) {
        int r = 0;
        for (int k = 0; k < n; ++k) r += (cn[k] > cn[j] || (cn[k] == cn[j] && k < j)) ? 1 : 0;
        perm[r] = j;
      }
      __syncthreads();
      for (int e = c.t; e < n * n; e += BT) gV[e] = A[e % n + (size_t)perm[e / n] * d.lda];
      for (int e = c.t; e < n * nr; e += BT) C[e % n + (size_t)(e / n) * BNM] = B[e % n + (size_t)(e / n) * d.ldb];
      __syncthreads();
      b_house_qr<OCC == 1 ? 8 : 2>(c, as_global(gV), n, as_lds(tau), as_global(C), BNM, nr);
      for (int e = c.t; e < n * n; e += BT) {
        const int i = e % n, j = e / n;
        gW[e] = i >= j ? gV[j + (size_t)i * n] : 0.0;
      }
      __syncthreads();
      // projections y_j = w_j^T C, rotated with the columns (W = I at the start: y_j = C[j, :])
      double* Y = gV;  // n x BRM (the reflectors are no longer needed)
      for (int e = c.t; e < n * nr; e += BT) Y[(size_t)(e % n) * BRM + e / n] = C[e % n + (size_t)(e / n) * BNM];
      __syncthreads();
      // the whole of U in HBM above order BNL: by blocks staged in the LDS matrix region (free after the QR)
      res.sweeps = !lds64 ? b_jacobi_blk(c, as_global(gW), as_global(Y), nr, n, 30, as_lds(lds), as_lds(sbuf))
                           : b_jacobi<OCC == 1>(c, as_global(gW), as_global(Y), nr, n, 30);
      // sigma_j = ||u_j||, cut at eps * sigma_max
      double* sig = sbuf;  // n
      for (int j = c.t; j < n; j += BT) {
        double s = 0.0;
#pragma unroll 8
        for (int i = 0; i < n; ++i) s = fma(gW[i + (size_t)j * n], gW[i + (size_t)j * n], s);
        sig[j] = sqrt(s);
      }
      __syncthreads();
      double sm = 0.0;
      for (int j = c.t; j < n; j += BT) sm = fmax(sm, sig[j]);
      const double smax = b_max(c, sm);
      const double cut = kEps * smax;
      int keep = 0;
      for (int j = c.t; j < n; j += BT) keep += sig[j] > cut ? 1 : 0;
      keep = (int)b_sum(c, (double)keep);
      res.rank = keep;
      // T = diag(1/sigma^2) (W^T C) for kept j, then X = U~ T
      double* T = gX + (size_t)BNM * BRM;  // BNM x BRM
      for (int e = c.t; e < n * nr; e += BT) {
        const int j = e % n, r = e / n;
        T[j + (size_t)r * BNM] = sig[j] > cut ? Y[(size_t)j * BRM + r] / (sig[j] * sig[j]) : 0.0;
      }
      __syncthreads();
      for (int e = c.t; e < n * nr; e += BT) {
        const int i = e % n, r = e / n;
        double s = 0.0;
#pragma unroll 8
        for (int j = 0; j < n; ++j) s = fma(gW[i + (size_t)j * n], T[j + (size_t)r * BNM], s);
        X[perm[i] + (size_t)r * d.ldx] = s;
      }
      __syncthreads();
    }
    // ---- S9: backward error of the returned x
    const bool have_x = res.status == ADA_OK || (res.status == ADA_ERR_SINGULAR && info == 0);
    if (have_x && o.want_berr) {
      double worst = 0.0;
      int nan = 0;
      for (int r = 0; r < nr; ++r) {
        double rn = 0.0, xn = 0.0, bn = 0.0;
        int xbad = 0;
        for (int i = c.t; i < n; i += BT) {
          double s = B[i + (size_t)r * d.ldb], e = 0.0;  // accurate residual (Dot2)
#pragma unroll 8
          for (int j = 0; j < n; ++j) dot2_sub(s, e, A[i + (size_t)j * d.lda], X[j + (size_t)r * d.ldx]);
          s += e;
          const double xi = X[i + (size_t)r * d.ldx];
          xbad |= !isfinite(xi);
          rn = fmax(rn, fabs(s));
          xn = fmax(xn, fabs(xi));
          bn = fmax(bn, fabs(B[i + (size_t)r * d.ldb]));
        }
        rn = b_max(c, rn);
        xn = b_max(c, xn);
        bn = b_max(c, bn);
        xbad = b_or(c, xbad);
        const double den = anorm_inf * xn + bn;
        const double eta = xbad ? __longlong_as_double(0x7ff8000000000000LL)
                                : (den > 0.0 ? rn / den : (rn > 0.0 ? INFINITY : 0.0));
        if (eta != eta) nan = 1;
        else worst = fmax(worst, eta);
      }
      res.berr = nan ? __longlong_as_double(0x7ff8000000000000LL) : worst;
    }
    if (c.t == 0) results[sys] = res;
    __syncthreads();
  }
}

// order[] = the systems by decreasing n (a counting sort; systems outside the kernel's limits last), so
// that the persistent workgroups take the longest systems first and a launch does not end on a tail of
// large systems picked up late. The order among systems of equal n is arbitrary: each system's result does
// not depend on when or where it runs. range[2k], range[2k+1]: the part of order[] that launch k takes
// (orders in (max_n[k+1], max_n[k]]; the last launch also takes the systems outside the limits). Also
// zeroes the launches' queue counters. One workgroup.
__global__ __launch_bounds__(1024) void k_batch_order(int count, const BDesc* __restrict__ desc, int* order,
                                                      unsigned* queue, int* range, int nb, int m0, int m1, int m2) {
  __shared__ int cnt[BNM + 1];
  for (int b = threadIdx.x; b <= BNM; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  auto bin_of = [&](int i) {
    const int n = desc[i].n;
    return (n >= 1 && n <= BNM) ? BNM - n : BNM;
  };
  for (int i = threadIdx.x; i < count; i += blockDim.x) atomicAdd(&cnt[bin_of(i)], 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int b = 0; b <= BNM; ++b) {
      const int c = cnt[b];
      cnt[b] = run;
      run += c;
    }
    const int mx[3] = {m0, m1, m2};
    for (int k = 0; k < nb; ++k) {
      range[2 * k] = cnt[BNM - mx[k]];
      range[2 * k + 1] = k + 1 < nb ? cnt[BNM - mx[k + 1]] : count;
      queue[k] = 0u;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < count; i += blockDim.x) order[atomicAdd(&cnt[bin_of(i)], 1)] = i;
}

namespace {
constexpr size_t kLdsPerCu = 160 * 1024;
constexpr size_t kStaticLds = 2048;  // the kernel's own shared variables (1.4 KB) with room to spare
size_t slice_budget() { return (size_t)BNM * b_slice_bytes(BNM); }  // 256 workgroups at the largest order
size_t order_bytes(int count) { return ((size_t)count * 4 + 255) / 256 * 256; }
}  // namespace

ada_batched_shape batched_default_shape(int max_wg) {
  ada_batched_shape s{};
  s.buckets = 1;
  s.max_n[0] = BNM;
  s.wg_per_cu[0] = 1;
  s.workgroups[0] = max_wg < 1 ? 1 : (max_wg > 256 ? 256 : max_wg);  // one per compute unit
  s.stage_cols = 8;
  return s;
}

const char* batched_shape_problem(const ada_batched_shape& s) {
  if (s.buckets < 1 || s.buckets > 3) return "buckets must be 1, 2 or 3";
  if (s.max_n[0] != BNM) return "max_n[0] must be 256";
  for (int k = 0; k < s.buckets; ++k) {
    if (k > 0 && !(s.max_n[k] < s.max_n[k - 1])) return "max_n must decrease";
    if (s.max_n[k] < 16) return "max_n must be >= 16";
    if (s.wg_per_cu[k] != 1 && s.wg_per_cu[k] != 2) return "wg_per_cu must be 1 or 2";
    if (s.wg_per_cu[k] == 2 && 2 * (b_lds_bytes(s.max_n[k]) + kStaticLds) > kLdsPerCu)
      return "two workgroups per compute unit need max_n <= 96 (LDS)";
    if (s.workgroups[k] < 1 || (size_t)s.workgroups[k] * b_slice_bytes(s.max_n[k]) > slice_budget())
      return "workgroups out of range for the workspace";
  }
  if (s.stage_cols != 4 && s.stage_cols != SPF) return "stage_cols must be 4 or 8";
  return nullptr;
}

size_t batched_workspace_bytes(int count) { return 256 + order_bytes(count) + slice_budget(); }

hipError_t launch_solve_batched(int count, const void* desc, const double* A, const double* B, double* X,
                                void* work, size_t work_bytes, const ada_opts& o, void* results, hipStream_t st,
                                const ada_batched_shape& shape, hipEvent_t* ev) {
  if (count < 1 || work_bytes < batched_workspace_bytes(count) || batched_shape_problem(shape))
    return hipErrorInvalidValue;
  unsigned* queue = reinterpret_cast<unsigned*>(work);                    // 3 counters
  int* range = reinterpret_cast<int*>(reinterpret_cast<char*>(work) + 64);  // 3 ranges
  int* order = reinterpret_cast<int*>(reinterpret_cast<char*>(work) + 256);
  char* slices = reinterpret_cast<char*>(work) + 256 + order_bytes(count);
  const int nb = shape.buckets;
  hipLaunchKernelGGL(k_batch_order, dim3(1), dim3(1024), 0, st, count, (const BDesc*)desc, order, queue, range, nb,
                     shape.max_n[0], nb > 1 ? shape.max_n[1] : 0, nb > 2 ? shape.max_n[2] : 0);
  if (ev) hipEventRecord(ev[0], st);
  for (int k = 0; k < nb; ++k) {
    const int hi = shape.max_n[k];
    const size_t lds = b_lds_bytes(hi);
    const int G = std::min(shape.workgroups[k], count);
    hipError_t e;
    if (shape.wg_per_cu[k] == 2) {
      static size_t done2 = 0;
      e = ensure_lds((const void*)k_solve_batched<2>, lds, done2);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_solve_batched<2>, dim3(G), dim3(BT), lds, st, (const BDesc*)desc, A, B, X, slices, o,
                         (ada_result*)results, queue + k, (const int*)order, (const int*)(range + 2 * k), hi,
                         shape.stage_cols);
    } else {
      static size_t done1 = 0;
      e = ensure_lds((const void*)k_solve_batched<1>, lds, done1);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_solve_batched<1>, dim3(G), dim3(BT), lds, st, (const BDesc*)desc, A, B, X, slices, o,
                         (ada_result*)results, queue + k, (const int*)order, (const int*)(range + 2 * k), hi,
                         shape.stage_cols);
    }
    if (ev) hipEventRecord(ev[k + 1], st);
  }
  return hipGetLastError();
}

}  // namespace ada
