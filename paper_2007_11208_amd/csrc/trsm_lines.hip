// Block triangular solves inside the blocked factorisations:
//   LU (Section II-D)         U12 = L11^{-1} A12, L11 unit lower: every column of A12 is a line
//                             (k_trsm_cols below);
//   Cholesky (Section II-C)   L21 = A21 L11^{-T}: every row of A21 is a line, x L11^T = a
//                             (k_trsm_lines; it can also take columns as lines).
// Both are forward substitution with the lower-triangular L11 on each line:
//   for i: v_i *= 1 / L(i,i) (non-unit only); v_r -= L(r,i) v_i for r > i.
// The non-unit solve multiplies by the reciprocals of the diagonal (computed once per workgroup, as
// LAPACK's triangular solve does it), so that a step is as short as the unit one and the whole loop
// unrolls with constant register indices.
// k_trsm_lines: eight threads share a line (thread g holds elements g, g+8, ..., g+120 in
// registers), 32 lines per workgroup, so a 128 x 8064 block fills the chip;
// L11's lower triangle sits in LDS packed by columns (66 KB, so that a workgroup fits beside one of the
// trailing update's: the Cholesky's block solve runs while that update is in flight), the solved v_i goes
// to the line's other threads with one cross-lane read, and the loop over i is
// unrolled so that every register index is a constant. Lanes are laid out so
// that the loads and stores of the block are coalesced: consecutive lanes hold
// consecutive rows of the matrix in both cases.
#include "ada_internal.h"

#include <climits>

namespace ada {

constexpr int TLB = 128;           // block width (the factorisation's panel width)
constexpr int TLG = 8;             // threads per line
constexpr int TLK = TLB / TLG;     // elements per thread
constexpr int TLL = 256 / TLG;     // lines per workgroup
// start of column i of the packed lower triangle (columns of TLB - i entries)
__host__ __device__ constexpr int tri_col(int i) { return i * TLB - i * (i - 1) / 2; }
constexpr int TLPACK = tri_col(TLB);  // 8256 doubles

template <bool LINE_IS_ROW, bool UNIT>
__global__ __launch_bounds__(256) void k_trsm_lines(int k0, int nbw, int first, int nlines, double* __restrict__ W,
                                                    int ldw, const DevRec* rec) {
  if (rec->stop) return;
  extern __shared__ double sL[];  // sL[tri_col(i) + r - i] = L11(r, i), r >= i; identity padding past nbw
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int g = LINE_IS_ROW ? (lane >> 3) : (lane & 7);
  const int li = LINE_IS_ROW ? (lane & 7) : (lane >> 3);
  const int line = blockIdx.x * TLL + w * 8 + li;
  const bool live = line < nlines;
  // 16 loads in flight per thread
  for (int e0 = t; e0 < TLB * TLB; e0 += 256 * 16) {
    double tmp[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + 256 * u, r = e % TLB, i = e / TLB;
      double x = (r == i) ? 1.0 : 0.0;
      if (r >= i && r < nbw && i < nbw) x = W[(size_t)(k0 + r) + (size_t)(k0 + i) * ldw];
      tmp[u] = x;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + 256 * u, r = e % TLB, i = e / TLB;
      if (r >= i) sL[tri_col(i) + r - i] = tmp[u];
    }
  }
  // element i of this line
  auto at = [&](int i) -> double* {
    return LINE_IS_ROW ? W + (size_t)(k0 + nbw + first + line) + (size_t)(k0 + i) * ldw
                       : W + (size_t)(k0 + i) + (size_t)(k0 + nbw + first + line) * ldw;
  };
  __shared__ double s_rd[TLB];  // 1 / L11(i, i) (non-unit)
  if (!UNIT && t < TLB) s_rd[t] = t < nbw ? 1.0 / W[(size_t)(k0 + t) + (size_t)(k0 + t) * ldw] : 1.0;
  double v[TLK];
#pragma unroll
  for (int k = 0; k < TLK; ++k) {
    const int i = g + TLG * k;
    v[k] = (live && i < nbw) ? *at(i) : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < TLB; ++i) {
    const int ki = i / TLG, gi = i % TLG;
    double xi = v[ki];
    if (!UNIT) {
      xi = xi * s_rd[i];
      v[ki] = (g == gi) ? xi : v[ki];
    }
    const int src = LINE_IS_ROW ? (li + 8 * gi) : (gi + 8 * li);
    xi = __shfl(xi, src, 64);
    // column i from row 0 on: the rows above i that the lanes below read there belong to column i - 1,
    // and their products are discarded (g <= gi in the first element block)
    const double* Li = sL + tri_col(i) - i;
#pragma unroll
    for (int k = ki; k < TLK; ++k) {
      const double l = Li[g + TLG * k];
      if (k == ki) v[k] = (g > gi) ? fma(-l, xi, v[k]) : v[k];
      else v[k] = fma(-l, xi, v[k]);
    }
  }
  if (!live) return;
#pragma unroll
  for (int k = 0; k < TLK; ++k) {
    const int i = g + TLG * k;
    if (i < nbw) *at(i) = v[k];
  }
}

// LU's U12 = L11^{-1} A12 (unit lower): a column of A12 is contiguous, so sixteen threads share one, a
// whole 16-lane row of the wave (thread g holds elements g, g+16, ..., g+112), and the solved v_i reaches
// the other fifteen by a DPP row broadcast instead of a cross-lane read through the LDS crossbar: the
// step's latency is a register move, not an LDS round trip. The steps are a template recursion so that
// each broadcast's source lane is a constant.
constexpr int TCG = 16;           // threads per column
constexpr int TCK = TLB / TCG;    // elements per thread
constexpr int TCL = 256 / TCG;    // columns per workgroup

// lane G of each 16-lane row, to the whole row
template <int G>
__device__ __forceinline__ double row_bcast(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x150 + G, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x150 + G, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int I>
__device__ __forceinline__ void cols_step(double (&v)[TCK], int g, const double* sL) {
  if constexpr (I < TLB) {
    constexpr int ki = I / TCG, gi = I % TCG;
    const double xi = row_bcast<gi>(v[ki]);
    const double* Li = sL + tri_col(I) - I;  // as in k_trsm_lines: rows above I are discarded
#pragma unroll
    for (int k = ki; k < TCK; ++k) {
      const double l = Li[g + TCG * k];
      if (k == ki) v[k] = (g > gi) ? fma(-l, xi, v[k]) : v[k];
      else v[k] = fma(-l, xi, v[k]);
    }
    cols_step<I + 1>(v, g, sL);
  }
}

// SWAP: the workgroup first applies the panel's row moves (count, then (destination, source) pairs) to
// its own columns, and workgroup 0 to the permutation vector, so that the next block column's
// interchanges and its block row of U are one launch (a workgroup owns whole columns: no other
// workgroup's moves are waited for).
template <bool SWAP>
__global__ __launch_bounds__(256) void k_trsm_cols(int k0, int nbw, int first, int ncols, double* __restrict__ W,
                                                   int ldw, const int* __restrict__ moves, int* __restrict__ perm,
                                                   DevRec* rec) {
  if (rec->stop) return;
  extern __shared__ double sL[];  // packed L11 as in k_trsm_lines
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int g = lane & 15;
  const int col = blockIdx.x * TCL + w * 4 + (lane >> 4);
  const bool live = col < ncols;
  if constexpr (SWAP) {
    if (rec->info != INT_MAX) {
      // the panel met an exact zero pivot: the routed solve has failed; later kernels skip
      if (blockIdx.x == 0 && t == 0) rec->stop = 1;
      return;
    }
    __shared__ double s_mv[2 * TLB][TCL + 1];
    __shared__ int s_pv[2 * TLB];
    const int cnt = moves[0];
    const int cb = blockIdx.x * TCL;
    for (int e = t; e < cnt * TCL; e += 256) {
      const int mi = e / TCL, c = e % TCL;
      if (cb + c < ncols) s_mv[mi][c] = W[(size_t)moves[2 + 2 * mi] + (size_t)(k0 + nbw + first + cb + c) * ldw];
    }
    if (blockIdx.x == 0)
      for (int mi = t; mi < cnt; mi += 256) s_pv[mi] = perm[moves[2 + 2 * mi]];
    __syncthreads();
    for (int e = t; e < cnt * TCL; e += 256) {
      const int mi = e / TCL, c = e % TCL;
      if (cb + c < ncols) W[(size_t)moves[1 + 2 * mi] + (size_t)(k0 + nbw + first + cb + c) * ldw] = s_mv[mi][c];
    }
    if (blockIdx.x == 0)
      for (int mi = t; mi < cnt; mi += 256) perm[moves[1 + 2 * mi]] = s_pv[mi];
    __syncthreads();  // the moved rows are read below (and L11 is not among them: the panel's own columns)
  }
  for (int e0 = t; e0 < TLB * TLB; e0 += 256 * 16) {
    double tmp[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + 256 * u, r = e % TLB, i = e / TLB;
      double x = (r == i) ? 1.0 : 0.0;
      if (r >= i && r < nbw && i < nbw) x = W[(size_t)(k0 + r) + (size_t)(k0 + i) * ldw];
      tmp[u] = x;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + 256 * u, r = e % TLB, i = e / TLB;
      if (r >= i) sL[tri_col(i) + r - i] = tmp[u];
    }
  }
  double* x = W + k0 + (size_t)(k0 + nbw + first + (live ? col : 0)) * ldw;
  double v[TCK];
#pragma unroll
  for (int k = 0; k < TCK; ++k) {
    const int i = g + TCG * k;
    v[k] = (live && i < nbw) ? x[i] : 0.0;
  }
  __syncthreads();
  cols_step<0>(v, g, sL);  // every lane of a row takes part (a row is one column, live or not)
  if (!live) return;
#pragma unroll
  for (int k = 0; k < TCK; ++k) {
    const int i = g + TCG * k;
    if (i < nbw) x[i] = v[k];
  }
}

template <bool LINE_IS_ROW, bool UNIT>
static hipError_t launch_lines(int k0, int nbw, int first, int nlines, double* W, int ldw, const DevRec* rec,
                               hipStream_t st) {
  if (nlines <= 0) return hipSuccess;
  if (nbw > TLB) return hipErrorInvalidValue;
  const size_t lds = (size_t)TLPACK * sizeof(double);
  static size_t done = 0;
  hipError_t e = ensure_lds((const void*)k_trsm_lines<LINE_IS_ROW, UNIT>, lds, done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_trsm_lines<LINE_IS_ROW, UNIT>), dim3((nlines + TLL - 1) / TLL), dim3(256), lds, st, k0, nbw,
                     first, nlines, W, ldw, rec);
  return hipGetLastError();
}

hipError_t launch_trsm_llnu(int k0, int nbw, int first, int ncols, double* W, int ldw, const DevRec* rec,
                            hipStream_t st) {
  if (ncols <= 0) return hipSuccess;
  if (nbw > TLB) return hipErrorInvalidValue;
  const size_t lds = (size_t)TLPACK * sizeof(double);
  static size_t done = 0;
  hipError_t e = ensure_lds((const void*)k_trsm_cols<false>, lds, done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_trsm_cols<false>, dim3((ncols + TCL - 1) / TCL), dim3(256), lds, st, k0, nbw, first, ncols, W,
                     ldw, (const int*)nullptr, (int*)nullptr, const_cast<DevRec*>(rec));
  return hipGetLastError();
}

hipError_t launch_swap_trsm_llnu(int k0, int nbw, int ncols, double* W, int ldw, const int* moves, int* perm,
                                 DevRec* rec, hipStream_t st) {
  if (ncols <= 0) return hipSuccess;
  if (nbw > TLB) return hipErrorInvalidValue;
  const size_t lds = (size_t)TLPACK * sizeof(double);
  static size_t done = 0;
  hipError_t e = ensure_lds((const void*)k_trsm_cols<true>, lds, done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_trsm_cols<true>, dim3((ncols + TCL - 1) / TCL), dim3(256), lds, st, k0, nbw, 0, ncols, W, ldw,
                     moves, perm, rec);
  return hipGetLastError();
}

hipError_t launch_trsm_rltn(int k0, int nbw, int mrows, double* W, int ldw, const DevRec* rec, hipStream_t st) {
  return launch_lines<true, false>(k0, nbw, 0, mrows, W, ldw, rec, st);
}

}  // namespace ada
