// Cholesky A = L L^T from the lower triangle (Section II-C), right-looking,
// blocked by 128 columns. Per block column k0:
//   k_potrf_diag   factor the diagonal block in LDS (one workgroup); a pivot
//                  that is not positive (or NaN) ends the factorisation: the
//                  matrix is then not taken to be sympd and the system is
//                  re-solved by LU on the original A (Section II-C);
//   k_trsm_lines   L21 = A21 L11^{-T} (rows are independent; trsm_lines.hip);
//   k_gemm_sub     A22 -= L21 L21^T on the matrix cores, lower tiles only.
#include "ada_internal.h"

#include <climits>

namespace ada {

// Diagonal block (nbw <= 128) in LDS, column by column. Thread t works on row
// r = t % 128 and on every other column of the update (parity t / 128), so
// each step is one broadcast read of L(c, j) and one read-modify-write of
// A(r, c) per column, with no index arithmetic beyond the loop.
__global__ __launch_bounds__(256) void k_potrf_diag(int k0, int nbw, double* __restrict__ W, int ldw, DevRec* rec) {
  if (rec->stop) return;
  extern __shared__ double sA[];  // sA[c * ld + r], ld = nbw + 1
  const int ld = nbw + 1;
  const int t = threadIdx.x;
  const int r = t & 127, half = t >> 7;
  for (int e = t; e < nbw * nbw; e += blockDim.x) {
    const int rr = e % nbw, c = e / nbw;
    if (rr >= c) sA[c * ld + rr] = W[(size_t)(k0 + rr) + (size_t)(k0 + c) * ldw];
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
    double lrj = 0.0;
    if (r > j && r < nbw) lrj = sA[j * ld + r] / sd;
    __syncthreads();  // every thread has read column j
    if (half == 0 && r >= j && r < nbw) sA[j * ld + r] = (r == j) ? sd : lrj;
    __syncthreads();  // column j of L is in place
    if (r > j && r < nbw) {
      for (int c = j + 1 + half; c <= r; c += 2) sA[c * ld + r] = fma(-lrj, sA[j * ld + c], sA[c * ld + r]);
    }
    __syncthreads();
  }
  __syncthreads();
  if (s_fail) return;
  for (int e = t; e < nbw * nbw; e += blockDim.x) {
    const int rr = e % nbw, c = e / nbw;
    if (rr >= c) W[(size_t)(k0 + rr) + (size_t)(k0 + c) * ldw] = sA[c * ld + rr];
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

}  // namespace ada
