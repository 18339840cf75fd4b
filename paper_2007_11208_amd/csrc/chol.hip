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

// Diagonal block (nbw <= 128) in LDS, in sub-blocks of 32 columns:
//   1. wave 0 factors the 32x32 diagonal sub-block with lane = row and the
//      row in registers (the column-j values of other rows come by readlane,
//      so the 32 steps need no barrier);
//   2. the rows below solve x L_kk^T = a (one thread per row, L_kk from LDS);
//   3. the trailing lower triangle takes the symmetric rank-32 update (4x4 register tiles).
// A pivot that is not positive (or NaN) ends the factorisation: the matrix is
// then not taken to be sympd and the system is re-solved by LU on the
// original A (Section II-C).
constexpr int PB = 32;
__global__ __launch_bounds__(256) void k_potrf_diag(int k0, int nbw, double* __restrict__ W, int ldw, DevRec* rec) {
  if (rec->stop) return;
  extern __shared__ double sA[];  // sA[c * ld + r], ld = nbw + 1 (lower triangle used)
  const int ld = nbw + 1;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // 16 loads in flight per thread
  for (int e0 = t; e0 < nbw * nbw; e0 += 256 * 16) {
    double tmp[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + 256 * u, rr = e % nbw, c = e / nbw;
      tmp[u] = (e < nbw * nbw && rr >= c) ? W[(size_t)(k0 + rr) + (size_t)(k0 + c) * ldw] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + 256 * u, rr = e % nbw, c = e / nbw;
      if (e < nbw * nbw && rr >= c) sA[c * ld + rr] = tmp[u];
    }
  }
  __shared__ int s_fail;
  if (t == 0) s_fail = 0;
  __syncthreads();
  for (int kb = 0; kb < nbw; kb += PB) {
    const int cb = min(PB, nbw - kb);
    // 1. diagonal sub-block
    if (w == 0) {
      double v[PB];
#pragma unroll
      for (int j = 0; j < PB; ++j) v[j] = (lane < cb && j <= lane) ? sA[(kb + j) * ld + kb + lane] : 0.0;
      int fail = 0;
#pragma unroll
      for (int j = 0; j < PB; ++j) {
        if (j < cb && !fail) {
          const double dj = read_lane(v[j], j);
          if (!(dj > 0.0)) {
            fail = j + 1;
          } else {
            const double sd = sqrt(dj);
            v[j] = (lane == j) ? sd : (lane > j ? v[j] / sd : v[j]);
#pragma unroll
            for (int k = j + 1; k < PB; ++k) {
              const double lkj = read_lane(v[j], k);
              if (lane >= k && k < cb) v[k] = fma(-v[j], lkj, v[k]);
            }
          }
        }
      }
      if (fail) {
        if (lane == 0) {
          atomicMin(&rec->chol_info, k0 + kb + fail);
          rec->stop = 1;
          s_fail = 1;
        }
      } else if (lane < cb) {
#pragma unroll
        for (int j = 0; j < PB; ++j)
          if (j <= lane) sA[(kb + j) * ld + kb + lane] = v[j];
      }
    }
    __syncthreads();
    if (s_fail) break;
    const int r0 = kb + cb, rest = nbw - r0;
    if (rest <= 0) break;
    // 2. rows below: x L_kk^T = a
    for (int i = t; i < rest; i += blockDim.x) {
      const int r = r0 + i;
      double x[PB];
#pragma unroll
      for (int j = 0; j < PB; ++j) x[j] = j < cb ? sA[(kb + j) * ld + r] : 0.0;
#pragma unroll
      for (int j = 0; j < PB; ++j) {
        if (j < cb) {
          x[j] = x[j] / sA[(kb + j) * ld + kb + j];
#pragma unroll
          for (int k = j + 1; k < PB; ++k)
            if (k < cb) x[k] = fma(-x[j], sA[(kb + j) * ld + kb + k], x[k]);
        }
      }
#pragma unroll
      for (int j = 0; j < PB; ++j)
        if (j < cb) sA[(kb + j) * ld + r] = x[j];
    }
    __syncthreads();
    // 3. trailing lower triangle: A(r, c) -= sum_j L(r, j) L(c, j), r >= c >= r0, in 4x4 register tiles
    //    (tile rows ti >= tile columns tj, dealt evenly over the threads; 8 LDS reads per 16 FMAs)
    {
      const int nt = (rest + 3) / 4;
      const int ntiles = nt * (nt + 1) / 2;
      for (int tile = t; tile < ntiles; tile += blockDim.x) {
        int ti = (int)((sqrt(8.0 * (double)tile + 1.0) - 1.0) * 0.5);
        while (ti * (ti + 1) / 2 > tile) --ti;
        while ((ti + 1) * (ti + 2) / 2 <= tile) ++ti;
        const int tj = tile - ti * (ti + 1) / 2;
        const int rb = r0 + 4 * ti, cb0 = r0 + 4 * tj;
        double acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int r = rb + a, c = cb0 + b;
            acc[a][b] = (r < nbw && c <= r) ? sA[c * ld + r] : 0.0;
          }
        for (int j = 0; j < cb; ++j) {
          const double* lj = sA + (kb + j) * ld;
          double lr[4], lc[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            lr[a] = rb + a < nbw ? lj[rb + a] : 0.0;
            lc[a] = cb0 + a < nbw ? lj[cb0 + a] : 0.0;
          }
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = fma(-lr[a], lc[b], acc[a][b]);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int r = rb + a, c = cb0 + b;
            if (r < nbw && c <= r) sA[c * ld + r] = acc[a][b];
          }
      }
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
