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
//   1. wave 0 factors the 32x32 diagonal sub-block, one lane per row with its
//      32 columns in registers: the pivot of column j comes by readlane, the
//      scaled column through LDS as broadcast reads (the 32 steps need no
//      barrier of the workgroup); the reciprocals of the diagonal go to LDS
//      for step 2;
//   2. the rows below solve x L_kk^T = a (one thread per row, L_kk and the
//      reciprocals of its diagonal from LDS, as LAPACK's triangular solve
//      does it: multiply by the reciprocal);
//   3. the trailing lower triangle takes the symmetric rank-32 update (4x4 register tiles).
// A pivot that is not positive (or NaN) ends the factorisation: the matrix is
// then not taken to be sympd and the system is re-solved by LU on the
// original A (Section II-C).
// A zero the compiler cannot see through: added to an LDS index it makes the
// broadcast loads of steps 1 and 2 per-lane values, so that the compiler keeps
// them in vector registers instead of hoisting hundreds of them into scalar
// registers (and spilling those).
__device__ __forceinline__ int opaque_zero() {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return z;
}
// the same once v is known: loads indexed with it cannot be issued before v is computed
__device__ __forceinline__ int zero_after(double v) {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z) : "v"(v));
  return z;
}

constexpr int PB = 32;
constexpr int PLD = 129;  // LDS column stride of the diagonal block (nbw <= 128)
// Row r of the rows below a 32-column diagonal sub-block at column kb: x L_kk^T = a, L_kk and the
// reciprocals of its diagonal in LDS (stride PLD), x in registers, as LAPACK's triangular solve does it
// (multiply by the reciprocal). FULL: cb == 32, no column bounds.
template <bool FULL>
__device__ __forceinline__ void trsm_row(double* sA, int kb, int r, int cb, const double* s_rinv) {
  double x[PB];
#pragma unroll
  for (int j = 0; j < PB; ++j) x[j] = (FULL || j < cb) ? sA[(kb + j) * PLD + r] : 0.0;
  // column j's entries of L are loaded once x[j-1] is known (a data dependence through an opaque
  // zero), so they are not all hoisted to the start and kept in registers
  int z = opaque_zero();
#pragma unroll
  for (int j = 0; j < PB; ++j) {
    if (FULL || j < cb) {
      x[j] = x[j] * s_rinv[j + z];
      const int zn = zero_after(x[j]);
#pragma unroll
      for (int k = j + 1; k < PB; ++k)
        if (FULL || k < cb) x[k] = fma(-x[j], sA[(kb + j) * PLD + kb + k + z], x[k]);
      z = zn;
    }
  }
#pragma unroll
  for (int j = 0; j < PB; ++j)
    if (FULL || j < cb) sA[(kb + j) * PLD + r] = x[j];
}

__global__ __launch_bounds__(256) void k_potrf_diag(int k0, int nbw, double* __restrict__ W, int ldw, DevRec* rec) {
  if (rec->stop) return;
  extern __shared__ double sA[];  // sA[c * ld + r] (lower triangle used)
  constexpr int ld = PLD;         // a constant stride: every LDS offset below is an immediate
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // 16 loads in flight per thread; element e of the 128 x 128 frame is row e % 128 of column e / 128
  for (int e0 = t; e0 < PB * 4 * PB * 4; e0 += 256 * 16) {
    double tmp[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + 256 * u, rr = e & 127, c = e >> 7;
      tmp[u] = (rr < nbw && c < nbw && rr >= c) ? W[(size_t)(k0 + rr) + (size_t)(k0 + c) * ldw] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = e0 + 256 * u, rr = e & 127, c = e >> 7;
      if (rr < nbw && c < nbw && rr >= c) sA[c * ld + rr] = tmp[u];
    }
  }
  __shared__ int s_fail;
  __shared__ double s_rinv[PB];  // reciprocals of the sub-block's diagonal (step 2)
  __shared__ double s_col[PB];   // the column being scaled (step 1)
  if (t == 0) s_fail = 0;
  __syncthreads();
  for (int kb = 0; kb < nbw; kb += PB) {
    const int cb = min(PB, nbw - kb);
    // 1. diagonal sub-block: wave 0, lane i < 32 holding row i's 32 columns (lanes 32-63 repeat rows 0-31
    //    and store nothing): A(i, c) -= L(i, j) L(c, j) for c > j, L(c, j) read from LDS where lane c
    //    wrote it. Entries right of a row's diagonal take the same arithmetic and are never stored.
    if (w == 0) {
      const int i = lane & 31;
      double v[PB];
#pragma unroll
      for (int c = 0; c < PB; ++c) v[c] = (i < cb && c <= i) ? sA[(kb + c) * ld + kb + i] : 0.0;
      int fail = 0;
#pragma unroll
      for (int j = 0; j < PB; ++j) {
        if (j < cb && !fail) {
          const double dj = read_lane(v[j], j);
          if (!(dj > 0.0)) {
            fail = j + 1;
          } else {
            // 1/sqrt(dj) by the hardware estimate and two Newton steps (each doubles the correct bits of the
            // estimate; the second ends at rounding level), so the step's dependent chain is a few FMAs
            // instead of a correctly rounded square root followed by a division; sqrt(dj) = dj / sqrt(dj).
            // Pivots below 1e-300 (where the estimate loses range) take the square root and the division.
            double ri, sd;
            if (dj >= 1e-300) {
              ri = __builtin_amdgcn_rsq(dj);
#pragma unroll
              for (int it = 0; it < 2; ++it) ri = fma(0.5 * ri, fma(-dj * ri, ri, 1.0), ri);
              sd = dj * ri;
            } else {
              sd = sqrt(dj);
              ri = 1.0 / sd;
            }
            const double l = (i == j) ? sd : (i > j ? v[j] * ri : v[j]);
            v[j] = l;
            if (lane == 0) s_rinv[j] = ri;
            s_col[i] = l;  // lanes i and i + 32 write the same value
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int c = j + 1; c < PB; ++c) v[c] = fma(-l, s_col[c], v[c]);
            __builtin_amdgcn_wave_barrier();
          }
        }
      }
      if (fail) {
        if (lane == 0) {
          atomicMin(&rec->chol_info, k0 + kb + fail);
          rec->stop = 1;
          s_fail = 1;
        }
      } else if (lane < 32 && i < cb) {
#pragma unroll
        for (int c = 0; c < PB; ++c)
          if (c <= i) sA[(kb + c) * ld + kb + i] = v[c];
      }
    }
    __syncthreads();
    if (s_fail) break;
    const int r0 = kb + cb, rest = nbw - r0;
    if (rest <= 0) break;
    // 2. rows below: x L_kk^T = a (a full 32-column sub-block needs no column bounds)
    if (cb == PB) {
      for (int i = t; i < rest; i += blockDim.x) trsm_row<true>(sA, kb, r0 + i, PB, s_rinv);
    } else {
      for (int i = t; i < rest; i += blockDim.x) trsm_row<false>(sA, kb, r0 + i, cb, s_rinv);
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
  for (int e = t; e < PB * 4 * PB * 4; e += blockDim.x) {
    const int rr = e & 127, c = e >> 7;
    if (rr < nbw && c < nbw && rr >= c) W[(size_t)(k0 + rr) + (size_t)(k0 + c) * ldw] = sA[c * ld + rr];
  }
}

hipError_t launch_potrf_diag(int k0, int nbw, double* W, int ldw, DevRec* rec, hipStream_t st) {
  if (nbw > PLD - 1) return hipErrorInvalidValue;
  const size_t lds = (size_t)nbw * PLD * sizeof(double);
  static size_t done = 0;
  hipError_t e = ensure_lds((const void*)k_potrf_diag, lds, done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), lds, st, k0, nbw, W, ldw, rec);
  return hipGetLastError();
}

}  // namespace ada
