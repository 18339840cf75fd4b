// Cholesky A = L L^T from the lower triangle (Section II-C), right-looking,
// blocked by 128 columns. Per block column k0:
//   k_potrf_diag   factor the diagonal block in LDS (one workgroup); a pivot
//                  that is not positive (or NaN) ends the factorisation: the
//                  matrix is then not taken to be sympd and the system is
//                  re-solved by LU on the original A (Section II-C);
//   k_trsm_rltn    L21 = A21 L11^{-T} (rows are independent: one thread per row,
//                  forward substitution in registers, L11 broadcast from LDS);
//   k_gemm_sub     A22 -= L21 L21^T on the matrix cores, lower tiles only.
#include "ada_internal.h"

#include <climits>

namespace ada {

__global__ __launch_bounds__(256) void k_potrf_diag(int k0, int nbw, double* __restrict__ W, int ldw, DevRec* rec) {
  if (rec->stop) return;
  extern __shared__ double sA[];  // sA[c * ld + r], ld = nbw + 1
  const int ld = nbw + 1;
  const int t = threadIdx.x;
  for (int e = t; e < nbw * nbw; e += blockDim.x) {
    const int r = e % nbw, c = e / nbw;
    if (r >= c) sA[c * ld + r] = W[(size_t)(k0 + r) + (size_t)(k0 + c) * ldw];
  }
  __shared__ int s_fail;
  if (t == 0) s_fail = 0;
  __syncthreads();
  for (int j = 0; j < nbw; ++j) {
    const double d = sA[j * ld + j];
    if (!(d > 0.0)) {
      if (t == 0) {
        atomicMin(&rec->chol_info, k0 + j + 1);
        rec->stop = 1;
        s_fail = 1;
      }
      break;
    }
    const double sd = sqrt(d);
    __syncthreads();
    if (t == 0) sA[j * ld + j] = sd;
    for (int r = j + 1 + t; r < nbw; r += blockDim.x) sA[j * ld + r] /= sd;
    __syncthreads();
    // trailing update of the lower part: sA[c][r] -= L[r][j] * L[c][j], j < c <= r
    const int rem = nbw - j - 1;
    const int tot = rem * rem;
    for (int e = t; e < tot; e += blockDim.x) {
      const int r = j + 1 + e % rem, c = j + 1 + e / rem;
      if (r >= c) sA[c * ld + r] = fma(-sA[j * ld + r], sA[j * ld + c], sA[c * ld + r]);
    }
    __syncthreads();
  }
  __syncthreads();
  if (s_fail) return;
  for (int e = t; e < nbw * nbw; e += blockDim.x) {
    const int r = e % nbw, c = e / nbw;
    if (r >= c) W[(size_t)(k0 + r) + (size_t)(k0 + c) * ldw] = sA[c * ld + r];
  }
}

hipError_t launch_potrf_diag(int k0, int nbw, double* W, int ldw, DevRec* rec, hipStream_t st) {
  const size_t lds = (size_t)nbw * (nbw + 1) * sizeof(double);
  static size_t done = 0;
  hipError_t e = ensure_lds((const void*)k_potrf_diag, lds, done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), lds, st, k0, nbw, W, ldw, rec);
  return hipGetLastError();
}

// rows k0+nbw .. k0+nbw+mrows-1 of the block column: x L11^T = a  <=>  L11 x^T = a^T
__global__ __launch_bounds__(256) void k_trsm_rltn(int k0, int nbw, int mrows, double* __restrict__ W, int ldw,
                                                   const DevRec* rec) {
  if (rec->stop) return;
  extern __shared__ double sL[];  // sL[c * nbw + r] = L11(r, c)
  const int t = threadIdx.x;
  for (int e = t; e < nbw * nbw; e += blockDim.x) {
    const int r = e % nbw, c = e / nbw;
    sL[e] = (r >= c) ? W[(size_t)(k0 + r) + (size_t)(k0 + c) * ldw] : 0.0;
  }
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + t;
  if (i >= mrows) return;
  double* row = W + (size_t)(k0 + nbw + i) + (size_t)k0 * ldw;  // row[c * ldw] = A21(i, c)
  const int nch = (nbw + 31) / 32;
  for (int ch = 0; ch < nch; ++ch) {
    const int c0 = ch * 32;
    double x[32];
#pragma unroll
    for (int c = 0; c < 32; ++c) x[c] = (c0 + c < nbw) ? row[(size_t)(c0 + c) * ldw] : 0.0;
    for (int p = 0; p < ch; ++p) {
      const int p0 = p * 32;
      double y[32];
#pragma unroll
      for (int pc = 0; pc < 32; ++pc) y[pc] = row[(size_t)(p0 + pc) * ldw];  // solved entries, loaded together
#pragma unroll
      for (int pc = 0; pc < 32; ++pc) {
        const double* lc = sL + (size_t)(p0 + pc) * nbw + c0;  // L11(c0+c, p0+pc)
#pragma unroll
        for (int c = 0; c < 32; ++c)
          if (c0 + c < nbw) x[c] = fma(-lc[c], y[pc], x[c]);
      }
    }
#pragma unroll
    for (int c = 0; c < 32; ++c) {
      if (c0 + c < nbw) {
        x[c] = x[c] / sL[(size_t)(c0 + c) * nbw + (c0 + c)];
        const double* lc = sL + (size_t)(c0 + c) * nbw + c0;
#pragma unroll
        for (int r = c + 1; r < 32; ++r)
          if (c0 + r < nbw) x[r] = fma(-lc[r], x[c], x[r]);
      }
    }
#pragma unroll
    for (int c = 0; c < 32; ++c)
      if (c0 + c < nbw) row[(size_t)(c0 + c) * ldw] = x[c];
  }
}

hipError_t launch_trsm_rltn(int k0, int nbw, int mrows, double* W, int ldw, const DevRec* rec, hipStream_t st) {
  if (mrows <= 0) return hipSuccess;
  const size_t lds = (size_t)nbw * nbw * sizeof(double);
  static size_t done = 0;
  hipError_t e = ensure_lds((const void*)k_trsm_rltn, lds, done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_trsm_rltn, dim3((mrows + 255) / 256), dim3(256), lds, st, k0, nbw, mrows, W, ldw, rec);
  return hipGetLastError();
}

}  // namespace ada
