// Trailing-matrix update C -= A * op(B) in FP64 on the CDNA4 matrix cores
// (v_mfma_f64_16x16x4_f64). This is the O(n^3) part of the LU (Section II-D)
// and Cholesky (Section II-C) factorisations.
//
// Tiling: 128x128 C tile per 256-thread workgroup (4 waves, 64x64 each =
// 4x4 MFMA blocks of 16x16), K staged through LDS in chunks of 16, double
// buffered. Narrow updates (the next block column of the look-ahead, a few
// dozen 128x128 tiles) take 64x64 tiles instead (4 waves of 32x32), so that
// they spread over four times as many compute units. The accumulators are loaded from C first and the A operand is
// negated, so the matrix cores form C - A op(B) directly. The MFMA is issued
// as D = B^T A^T so that the accumulator layout
// (lane l, register r -> row 4r + l/16, column l%16 of D) puts 16 consecutive
// rows of C in consecutive lanes: the read-modify-write of C is coalesced.
// Tile ids are spread so that each XCD (workgroups are dealt round-robin to
// the 8 XCDs) owns a contiguous range of tiles and its L2 keeps the shared
// A/B panels.
#include "ada_internal.h"

namespace ada {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BK = 16, PADK = 4;

template <bool TRANSB, int TM = 128>
__global__ __launch_bounds__(256, 2) void k_gemm_sub(int m, int n, int k, const double* __restrict__ A, int lda,
                                                  const double* __restrict__ B, int ldb, double* __restrict__ C,
                                                  int ldc, int lower, int tiles_m, int ntiles,
                                                  const int* __restrict__ skip) {
  constexpr int TN = TM, WT = TM / 2, MB = WT / 16;  // wave tile WT x WT = MB x MB blocks of 16x16
  constexpr int EA = TM * BK / 256;                  // elements of A (and of B) per thread and K chunk
  if (skip && *skip) return;
  const int per = gridDim.x >> 3;
  const int lin = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (lin >= ntiles) return;
  int ti, tj;
  if (lower) {
    // column-major enumeration of the tiles with ti >= tj
    int rem = lin;
    tj = 0;
    while (rem >= tiles_m - tj) { rem -= tiles_m - tj; ++tj; }
    ti = tj + rem;
  } else {
    ti = lin % tiles_m;
    tj = lin / tiles_m;
  }
  const int row0 = ti * TM, col0 = tj * TN;

  __shared__ double As[2][BK][TM + PADK];
  __shared__ double Bs[2][BK][TN + PADK];

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int wm = w & 1, wn = w >> 1;

  // global->LDS load assignment
  const int a_kk = t >> 4, a_ii = (t & 15) * EA;                          // A: EA consecutive rows of one k
  const int bn_jj = t / (BK / EA), bn_kh = (t % (BK / EA)) * EA;           // B (NN): EA consecutive k of one column
  const int bt_kk = t >> 4, bt_jj = (t & 15) * EA;                         // B (NT): EA consecutive columns of one k

  double ra[EA], rb[EA];
  auto load_regs = [&](int k0) {
    {
      const int kk = k0 + a_kk;
#pragma unroll
      for (int e = 0; e < EA; ++e) {
        const int i = row0 + a_ii + e;
        ra[e] = (i < m && kk < k) ? A[(size_t)i + (size_t)kk * lda] : 0.0;
      }
    }
    if (!TRANSB) {
      const int j = col0 + bn_jj;
#pragma unroll
      for (int e = 0; e < EA; ++e) {
        const int kk = k0 + bn_kh + e;
        rb[e] = (j < n && kk < k) ? B[(size_t)kk + (size_t)j * ldb] : 0.0;
      }
    } else {
      const int kk = k0 + bt_kk;
#pragma unroll
      for (int e = 0; e < EA; ++e) {
        const int j = col0 + bt_jj + e;
        rb[e] = (j < n && kk < k) ? B[(size_t)j + (size_t)kk * ldb] : 0.0;
      }
    }
  };
  auto store_lds = [&](int buf) {
#pragma unroll
    for (int e = 0; e < EA; ++e) As[buf][a_kk][a_ii + e] = ra[e];
    if (!TRANSB) {
#pragma unroll
      for (int e = 0; e < EA; ++e) Bs[buf][bn_kh + e][bn_jj] = rb[e];
    } else {
#pragma unroll
      for (int e = 0; e < EA; ++e) Bs[buf][bt_kk][bt_jj + e] = rb[e];
    }
  };

  // the accumulators start from C (loads in flight beside the first K chunk's) and the matrix cores
  // subtract A * op(B) from them, so the epilogue is a store
  const int lr = lane & 15, lk = lane >> 4;
  d4 acc[MB][MB];
#pragma unroll
  for (int bi = 0; bi < MB; ++bi) {
    const int i = row0 + wm * WT + bi * 16 + lr;
#pragma unroll
    for (int bj = 0; bj < MB; ++bj) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = col0 + wn * WT + bj * 16 + 4 * r + lk;
        acc[bi][bj][r] = (i < m && j < n) ? C[(size_t)i + (size_t)j * ldc] : 0.0;
      }
    }
  }

  const int nch = (k + BK - 1) / BK;
  load_regs(0);
  store_lds(0);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) load_regs((c + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double af[MB], bf[MB];
#pragma unroll
      for (int bi = 0; bi < MB; ++bi) af[bi] = -As[buf][kk + lk][wm * WT + bi * 16 + lr];
#pragma unroll
      for (int bj = 0; bj < MB; ++bj) bf[bj] = Bs[buf][kk + lk][wn * WT + bj * 16 + lr];
#pragma unroll
      for (int bi = 0; bi < MB; ++bi)
#pragma unroll
        for (int bj = 0; bj < MB; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[bj], af[bi], acc[bi][bj], 0, 0, 0);
    }
    if (c + 1 < nch) store_lds(buf ^ 1);
    __syncthreads();
  }
  // acc[bi][bj][r] = (C - A*op(B))[row0+wm*WT+bi*16+lr][col0+wn*WT+bj*16+4r+lk]
#pragma unroll
  for (int bi = 0; bi < MB; ++bi) {
    const int i = row0 + wm * WT + bi * 16 + lr;
    if (i >= m) continue;
#pragma unroll
    for (int bj = 0; bj < MB; ++bj) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = col0 + wn * WT + bj * 16 + 4 * r + lk;
        if (j < n) C[(size_t)i + (size_t)j * ldc] = acc[bi][bj][r];
      }
    }
  }
}

hipError_t launch_gemm_sub(int m, int n, int k, const double* A, int lda, const double* B, int ldb, bool transB,
                           double* C, int ldc, bool lower, const int* skip_if_nonzero, hipStream_t st,
                           hipEvent_t ev0, hipEvent_t ev1) {
  if (m <= 0 || n <= 0 || k <= 0) return hipSuccess;
  // a rectangular update of fewer than 256 tiles of 128 x 128 takes 64 x 64 tiles
  const bool small = !lower && (size_t)((m + 127) / 128) * ((n + 127) / 128) < 256;
  const int tm = small ? 64 : 128;
  const int tiles_m = (m + tm - 1) / tm, tiles_n = (n + tm - 1) / tm;
  int ntiles;
  if (lower) {
    // square update (m == n): tiles on or below the diagonal
    ntiles = tiles_m * (tiles_m + 1) / 2;
  } else {
    ntiles = tiles_m * tiles_n;
  }
  const int grid = ((ntiles + 7) / 8) * 8;
  if (ev0) hipEventRecord(ev0, st);
  if (small) {
    if (transB)
      hipLaunchKernelGGL((k_gemm_sub<true, 64>), dim3(grid), dim3(256), 0, st, m, n, k, A, lda, B, ldb, C, ldc, 0,
                         tiles_m, ntiles, skip_if_nonzero);
    else
      hipLaunchKernelGGL((k_gemm_sub<false, 64>), dim3(grid), dim3(256), 0, st, m, n, k, A, lda, B, ldb, C, ldc, 0,
                         tiles_m, ntiles, skip_if_nonzero);
  } else if (transB) {
    hipLaunchKernelGGL(k_gemm_sub<true>, dim3(grid), dim3(256), 0, st, m, n, k, A, lda, B, ldb, C, ldc,
                       (int)lower, tiles_m, ntiles, skip_if_nonzero);
  } else {
    hipLaunchKernelGGL(k_gemm_sub<false>, dim3(grid), dim3(256), 0, st, m, n, k, A, lda, B, ldb, C, ldc,
                       (int)lower, tiles_m, ntiles, skip_if_nonzero);
  }
  if (ev1) hipEventRecord(ev1, st);
  return hipGetLastError();
}

}  // namespace ada
