// Symmetric indefinite LDL^T with Bunch-Kaufman partial pivoting: the route the paper's
// conclusion (Section V) names as future work for plain symmetric matrices (symmetric but
// not positive definite). Off by default; selected with the symmetric extension option.
//
// P A P^T = L D L^T, L unit lower triangular, D block diagonal with 1x1 and 2x2 blocks
// (Bunch & Kaufman, Math. Comp. 31(137), 1977, pivot threshold alpha = (1 + sqrt 17) / 8).
// Blocked and right-looking between panels: a panel of up to b columns is factored by one
// workgroup that keeps the trailing matrix unchanged and forms each column it needs as
// "raw column minus the panel's contribution so far" (the delayed update); the trailing
// matrix then takes one symmetric rank-kb update A22 -= L21 (L21 D)^T on the FP64 MFMA GEMM.
//
// The permutation is kept whole (every interchange also swaps the rows of L already formed),
// so the solve is x = P^T L^{-T} D^{-1} L^{-1} P b with the library's triangular solves.
#include "ada_internal.h"

namespace ada {

constexpr int SP_T = 1024;  // threads of the panel workgroup
constexpr int SP_W = SP_T / 64;
constexpr int SP_BMAX = 64;  // widest panel
constexpr double kBkAlpha = 0.64038820320220756872767623199676;  // (1 + sqrt(17)) / 8

// workgroup argmax of (v, idx): larger v wins, ties to the lower index; idx < 0 = none
__device__ void block_argmax(double& v, int& idx, double* sv, int* si) {
  wave_argmax(v, idx);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) { sv[w] = v; si[w] = idx; }
  __syncthreads();
  v = -1.0;
  idx = -1;
  for (int q = 0; q < SP_W; ++q)
    if (si[q] >= 0 && (idx < 0 || sv[q] > v || (sv[q] == v && si[q] < idx))) { v = sv[q]; idx = si[q]; }
}

// Rows i = i0 + q*SP_T (q < 4) of "raw column minus the panel's contribution": v_q = raw(i) -
// sum_{c < jj} L(i, k0+c) s[c], with raw(i) = W(i, col) below the diagonal position `mirror` and
// W(mirror, i) above it (mirror < 0: always W(i, col)). Four rows and four panel columns per step
// keep sixteen loads in flight per thread (the panel's L columns stream from L2). Rows past the
// end are clamped to n-1 (valid addresses, results unused).
__device__ __forceinline__ void panel_rows(int n, int i0, int col, int mirror, int k0, int jj,
                                           const double* __restrict__ W, int ldw, const double* s, double v[4]) {
  int ir[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ir[q] = min(i0 + q * SP_T, n - 1);
    v[q] = (mirror >= 0 && ir[q] < mirror) ? W[mirror + (size_t)ir[q] * ldw] : W[ir[q] + (size_t)col * ldw];
  }
  // 32-bit offsets from the uniform panel base (n <= 16384: the panel spans < 2^31 elements)
  const double* L = W + (size_t)k0 * ldw;
  int c = 0;
  for (; c + 4 <= jj; c += 4) {
    double l[4][4];
    const int cb = c * ldw;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) l[u][q] = L[ir[q] + cb + u * ldw];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = fma(-l[u][q], s[c + u], v[q]);
  }
  for (; c < jj; ++c) {
    const double sc = s[c];
    const int cb = c * ldw;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = fma(-L[ir[q] + cb], sc, v[q]);
  }
}

// kind of pivot: 0 zero column, 1 1x1 in place, 2 1x1 with j <-> r, 3 2x2 with j+1 <-> r
__global__ __launch_bounds__(SP_T) void k_sytrf_panel(int n, int k0, int b, double* __restrict__ W, int ldw,
                                                      double* __restrict__ Wp, int ldp, int* __restrict__ swp,
                                                      double* __restrict__ dd, double* __restrict__ ee,
                                                      DevRec* rec) {
  __shared__ double s_wj[SP_BMAX], s_wr[SP_BMAX];
  __shared__ double s_rv[SP_W];
  __shared__ int s_ri[SP_W];
  __shared__ double s_val[8];
  const int t = threadIdx.x;
  const bool last = n - k0 <= b;
  // panels start every b-1 columns; when the previous panel's last pivot was a 2x2 block it has
  // already factored position k0 (delta = 1): its L.D column here is zero, so the delayed updates and
  // the trailing update of this panel take nothing from it
  const int delta = rec->ldlt_delta;
  if (delta)
    for (int i = k0 + t; i < n; i += SP_T) Wp[i] = 0.0;
  __syncthreads();
  int jj = delta;
  while (true) {
    const int j = k0 + jj;
    if (j >= n || (!last && jj >= b - 1)) break;
    // ---- updated column j: A(i,j) - sum_c L(i,k0+c) Wp(j,c), rows i >= j
    if (t < jj) s_wj[t] = Wp[j + (size_t)t * ldp];
    __syncthreads();
    double best = -1.0;
    int bi = -1;
    for (int i0 = j + t; i0 < n; i0 += 4 * SP_T) {
      double v[4];
      panel_rows(n, i0, j, -1, k0, jj, W, ldw, s_wj, v);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + q * SP_T;
        if (i >= n) break;
        Wp[i + (size_t)jj * ldp] = v[q];
        if (i == j) s_val[0] = v[q];
        else if (fabs(v[q]) > best) { best = fabs(v[q]); bi = i; }
      }
    }
    block_argmax(best, bi, s_rv, s_ri);
    const double colmax = bi >= 0 ? best : 0.0;
    const int r = bi;
    const double wjj = s_val[0];
    const double absjj = fabs(wjj);
    int kind;
    if (absjj == 0.0 && colmax == 0.0) kind = 0;
    else if (absjj >= kBkAlpha * colmax) kind = 1;
    else {
      // ---- updated column r (row r left of the diagonal, column r below it), into Wp(:, jj+1)
      __syncthreads();
      if (t < jj) s_wr[t] = Wp[r + (size_t)t * ldp];
      __syncthreads();
      double rb = -1.0;
      int ri = -1;
      for (int i0 = j + t; i0 < n; i0 += 4 * SP_T) {
        double v[4];
        panel_rows(n, i0, r, r, k0, jj, W, ldw, s_wr, v);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = i0 + q * SP_T;
          if (i >= n) break;
          Wp[i + (size_t)(jj + 1) * ldp] = v[q];
          if (i == r) s_val[1] = v[q];
          else if (fabs(v[q]) > rb) { rb = fabs(v[q]); ri = i; }
        }
      }
      block_argmax(rb, ri, s_rv, s_ri);
      const double rowmax = rb;
      const double wrr = s_val[1];
      if (absjj * rowmax >= kBkAlpha * colmax * colmax) kind = 1;
      else if (fabs(wrr) >= kBkAlpha * rowmax) kind = 2;
      else kind = 3;
    }
    __syncthreads();
    if (kind >= 2) {
      const int p = kind == 2 ? j : j + 1;
      // the values that cross rows: w(p), w(r) of column j and w2(p), w2(r) of column r
      if (t == 0) {
        s_val[2] = Wp[p + (size_t)jj * ldp];
        s_val[3] = Wp[r + (size_t)jj * ldp];
        s_val[4] = Wp[p + (size_t)(jj + 1) * ldp];
        s_val[5] = Wp[r + (size_t)(jj + 1) * ldp];
      }
      // rows p and r of the L and Wp columns this panel already formed
      if (p != r && t < jj) {
        double* lc = W + (size_t)(k0 + t) * ldw;
        double x = lc[p];
        lc[p] = lc[r];
        lc[r] = x;
        double* wc = Wp + (size_t)t * ldp;
        x = wc[p];
        wc[p] = wc[r];
        wc[r] = x;
      }
      // the raw column p moves to position r (the raw column and row r were consumed into w2)
      if (p != r) {
        if (t == 0) W[r + (size_t)r * ldw] = W[p + (size_t)p * ldw];
#pragma unroll 4
        for (int i = p + 1 + t; i < n; i += SP_T) {
          if (i < r) W[r + (size_t)i * ldw] = W[i + (size_t)p * ldw];
          else if (i > r) W[i + (size_t)r * ldw] = W[i + (size_t)p * ldw];
        }
      }
      __syncthreads();
      if (kind == 2) {
        // new column j = w2 with entries j and r exchanged
#pragma unroll 4
        for (int i = j + t; i < n; i += SP_T) {
          const double v = i == j ? s_val[5] : (i == r ? s_val[4] : Wp[i + (size_t)(jj + 1) * ldp]);
          Wp[i + (size_t)jj * ldp] = v;
        }
      } else {
        // new columns j, j+1 = w, w2 with entries j+1 and r exchanged
        if (p != r) {
          if (t == 0) {
            Wp[p + (size_t)jj * ldp] = s_val[3];
            Wp[r + (size_t)jj * ldp] = s_val[2];
            Wp[p + (size_t)(jj + 1) * ldp] = s_val[5];
            Wp[r + (size_t)(jj + 1) * ldp] = s_val[4];
          }
        }
      }
      __syncthreads();
    }
    if (t == 0) {
      swp[j] = kind == 2 ? r : j;
      if (kind == 3) swp[j + 1] = r;
      if (kind == 0) atomicMin(&rec->info, j + 1);
    }
    // ---- L columns and D
    if (kind <= 2) {
      const double dj = kind == 2 ? s_val[5] : wjj;
#pragma unroll 4
      for (int i = j + 1 + t; i < n; i += SP_T)
        W[i + (size_t)j * ldw] = kind == 0 ? 0.0 : Wp[i + (size_t)jj * ldp] / dj;
      if (t == 0) {
        W[j + (size_t)j * ldw] = dj;
        dd[j] = dj;
        ee[j] = 0.0;
      }
      jj += 1;
    } else {
      const double a = wjj, bb = s_val[3], c2 = s_val[5];
      const double det = a * c2 - bb * bb;
#pragma unroll 4
      for (int i = j + 2 + t; i < n; i += SP_T) {
        const double s0 = Wp[i + (size_t)jj * ldp], s1 = Wp[i + (size_t)(jj + 1) * ldp];
        W[i + (size_t)j * ldw] = (s0 * c2 - s1 * bb) / det;
        W[i + (size_t)(j + 1) * ldw] = (s1 * a - s0 * bb) / det;
      }
      if (t == 0) {
        W[j + (size_t)j * ldw] = a;
        W[(j + 1) + (size_t)j * ldw] = 0.0;
        W[(j + 1) + (size_t)(j + 1) * ldw] = c2;
        dd[j] = a;
        dd[j + 1] = c2;
        ee[j] = bb;
        ee[j + 1] = 0.0;
      }
      jj += 2;
    }
    __syncthreads();
  }
  int next_delta = 0;
  if (!last && jj == b - 1) {
    // position k0+b-1 is left to the next panel: it takes this panel's update here (the trailing update
    // covers the rows and columns from k0+b on), and its L.D column stays zero
    const int j = k0 + b - 1;
    if (t < jj) s_wj[t] = Wp[j + (size_t)t * ldp];
    __syncthreads();
    for (int i0 = j + t; i0 < n; i0 += 4 * SP_T) {
      double v[4];
      panel_rows(n, i0, j, -1, k0, jj, W, ldw, s_wj, v);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + q * SP_T;
        if (i >= n) break;
        W[i + (size_t)j * ldw] = v[q];
        Wp[i + (size_t)jj * ldp] = 0.0;
      }
    }
  } else if (!last) {
    next_delta = 1;  // a 2x2 block ended on position k0+b-1
  }
  if (t == 0) {
    rec->ldlt_first = k0 + delta;
    rec->ldlt_kb = jj - delta;
    rec->ldlt_delta = next_delta;
  }
}

hipError_t launch_sytrf_panel(int n, int k0, int b, double* W, int ldw, double* Wp, int ldp, int* swp, double* d,
                              double* e, DevRec* rec, hipStream_t st) {
  if (b < 3 || b > SP_BMAX || k0 < 0 || k0 >= n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sytrf_panel, dim3(1), dim3(SP_T), 0, st, n, k0, b, W, ldw, Wp, ldp, swp, d, e, rec);
  return hipGetLastError();
}

// one thread per column c < k0 walks the interchanges of the positions the last panel factored
// (rec->ldlt_first .. +ldlt_kb) in order; thread 0 of workgroup 0 also carries them into perm
__global__ __launch_bounds__(256) void k_ldlt_swap_left(int n, int k0, double* __restrict__ W, int ldw,
                                                        const int* __restrict__ swp, int* __restrict__ perm,
                                                        const DevRec* rec) {
  const int q0 = rec->ldlt_first, q1 = q0 + rec->ldlt_kb;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < k0) {
    double* col = W + (size_t)c * ldw;
    for (int q = q0; q < q1; ++q) {
      const int r = swp[q];
      if (r != q) {
        const double x = col[q];
        col[q] = col[r];
        col[r] = x;
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int q = q0; q < q1; ++q) {
      const int r = swp[q];
      if (r != q) {
        const int x = perm[q];
        perm[q] = perm[r];
        perm[r] = x;
      }
    }
  }
}

hipError_t launch_ldlt_swap_left(int n, int k0, double* W, int ldw, const int* swp, int* perm, const DevRec* rec,
                                 hipStream_t st) {
  const int blocks = k0 > 0 ? (k0 + 255) / 256 : 1;
  hipLaunchKernelGGL(k_ldlt_swap_left, dim3(blocks), dim3(256), 0, st, n, k0, W, ldw, swp, perm, rec);
  return hipGetLastError();
}

// the first row of a 2x2 block solves both of its rows; the second row's thread skips
__global__ __launch_bounds__(256) void k_ldlt_dsolve(int n, int nrhs, const double* __restrict__ d,
                                                     const double* __restrict__ e, double* __restrict__ X, int ldx,
                                                     const int* pred, int pred_val) {
  if (pred && *pred != pred_val) return;
  const size_t total = (size_t)n * nrhs;
  for (size_t g = blockIdx.x * (size_t)blockDim.x + threadIdx.x; g < total; g += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(g % n), c = (int)(g / n);
    double* x = X + (size_t)c * ldx;
    if (i + 1 < n && e[i] != 0.0) {
      const double a = d[i], b = e[i], c2 = d[i + 1], det = a * c2 - b * b;
      const double y0 = x[i], y1 = x[i + 1];
      x[i] = (c2 * y0 - b * y1) / det;
      x[i + 1] = (a * y1 - b * y0) / det;
    } else if (!(i > 0 && e[i - 1] != 0.0)) {
      x[i] = x[i] / d[i];
    }
  }
}

hipError_t launch_ldlt_dsolve(int n, int nrhs, const double* d, const double* e, double* X, int ldx,
                              const int* pred, int pred_val, hipStream_t st) {
  size_t total = (size_t)n * nrhs;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_ldlt_dsolve, dim3(blocks), dim3(256), 0, st, n, nrhs, d, e, X, ldx, pred, pred_val);
  return hipGetLastError();
}

}  // namespace ada
