// Trailing-matrix update C -= A * op(B) with low-precision operands on the CDNA4
// matrix cores and FP32 accumulation; C stays FP64 and the subtraction is FP64.
// This is the O(n^3) part of the LU (Section II-D) and Cholesky (Section II-C)
// factorisations in the mixed-precision solve: the factors it produces carry an
// error of the operand precision's order, which FP64 iterative refinement removes.
//
//   FP32: v_mfma_f32_16x16x4_f32, K staged through LDS in chunks of 16 (as FP32);
//   BF16: v_mfma_f32_16x16x32_bf16, K staged in chunks of 32 (as BF16, rounded
//         to nearest even from FP64 through FP32).
//
// Tiling as in the FP64 kernel: a 128x128 C tile per 256-thread workgroup, four
// waves of 64x64 (4x4 blocks of 16x16), the MFMA issued as D = B^T A^T so that 16
// consecutive rows of C sit in consecutive lanes (coalesced read-modify-write of C),
// and tile ids dealt so that each XCD owns a contiguous range of tiles.
//
// FP32-output 16x16 MFMA accumulator layout: lane l, register r holds
// D[4 (l / 16) + r][l % 16].
#include "ada_internal.h"

namespace ada {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

namespace {

constexpr int TM = 128, TN = 128;

__device__ __forceinline__ void tile_of(int lin, int lower, int tiles_m, int& ti, int& tj) {
  if (lower) {
    // column-major enumeration of the tiles with ti >= tj
    int rem = lin;
    tj = 0;
    while (rem >= tiles_m - tj) {
      rem -= tiles_m - tj;
      ++tj;
    }
    ti = tj + rem;
  } else {
    ti = lin % tiles_m;
    tj = lin / tiles_m;
  }
}

// C[row0 + wm*64 + bi*16 + (l%16)][col0 + wn*64 + bj*16 + 4 (l/16) + r] -= acc[bi][bj][r]
__device__ __forceinline__ void store_sub(const f4 (&acc)[4][4], int m, int n, double* C, int ldc, int row0, int col0,
                                          int wm, int wn, int lane) {
  const int lr = lane & 15, lg = lane >> 4;
#pragma unroll
  for (int bi = 0; bi < 4; ++bi) {
    const int i = row0 + wm * 64 + bi * 16 + lr;
    if (i >= m) continue;
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = col0 + wn * 64 + bj * 16 + 4 * lg + r;
        if (j < n) {
          double* p = C + (size_t)i + (size_t)j * ldc;
          *p = *p - (double)acc[bi][bj][r];
        }
      }
    }
  }
}

// ---------------------------------------------------------------- FP32 operands
constexpr int BK32 = 16, PAD32 = 4;

template <bool TRANSB>
__global__ __launch_bounds__(256) void k_gemm_sub_f32(int m, int n, int k, const double* __restrict__ A, int lda,
                                                      const double* __restrict__ B, int ldb, double* __restrict__ C,
                                                      int ldc, int lower, int tiles_m, int ntiles,
                                                      const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int per = gridDim.x >> 3;
  const int lin = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (lin >= ntiles) return;
  int ti, tj;
  tile_of(lin, lower, tiles_m, ti, tj);
  const int row0 = ti * TM, col0 = tj * TN;

  __shared__ float As[2][BK32][TM + PAD32];
  __shared__ float Bs[2][BK32][TN + PAD32];

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int wm = w & 1, wn = w >> 1;
  const int a_kk = t >> 4, a_ii = (t & 15) * 8;   // A: 8 consecutive rows of one k
  const int bn_jj = t >> 1, bn_kh = (t & 1) * 8;  // B (NN): 8 consecutive k of one column
  const int bt_kk = t >> 4, bt_jj = (t & 15) * 8; // B (NT): 8 consecutive columns of one k

  double ra[8], rb[8];
  auto load_regs = [&](int k0) {
    {
      const int kk = k0 + a_kk;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int i = row0 + a_ii + e;
        ra[e] = (i < m && kk < k) ? A[(size_t)i + (size_t)kk * lda] : 0.0;
      }
    }
    if (!TRANSB) {
      const int j = col0 + bn_jj;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int kk = k0 + bn_kh + e;
        rb[e] = (j < n && kk < k) ? B[(size_t)kk + (size_t)j * ldb] : 0.0;
      }
    } else {
      const int kk = k0 + bt_kk;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int j = col0 + bt_jj + e;
        rb[e] = (j < n && kk < k) ? B[(size_t)j + (size_t)kk * ldb] : 0.0;
      }
    }
  };
  auto store_lds = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; ++e) As[buf][a_kk][a_ii + e] = (float)ra[e];
    if (!TRANSB) {
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[buf][bn_kh + e][bn_jj] = (float)rb[e];
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) Bs[buf][bt_kk][bt_jj + e] = (float)rb[e];
    }
  };

  f4 acc[4][4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = f4{0.f, 0.f, 0.f, 0.f};

  const int nch = (k + BK32 - 1) / BK32;
  load_regs(0);
  store_lds(0);
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) load_regs((c + 1) * BK32);
#pragma unroll
    for (int kk = 0; kk < BK32; kk += 4) {
      float af[4], bf[4];
#pragma unroll
      for (int bi = 0; bi < 4; ++bi) af[bi] = As[buf][kk + lk][wm * 64 + bi * 16 + lr];
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) bf[bj] = Bs[buf][kk + lk][wn * 64 + bj * 16 + lr];
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32(bf[bj], af[bi], acc[bi][bj], 0, 0, 0);
    }
    if (c + 1 < nch) store_lds(buf ^ 1);
    __syncthreads();
  }
  store_sub(acc, m, n, C, ldc, row0, col0, wm, wn, lane);
}

// ---------------------------------------------------------------- BF16 operands
// LDS holds each tile row (of A) or tile column (of op(B)) with its 32 k values
// contiguous, so that a lane's 8 consecutive k are one 16-byte read.
constexpr int BK16 = 32, PAD16 = 8;

__device__ __forceinline__ void put16(__bf16* dst, const double* v) {
  bf8 lo, hi;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    lo[e] = (__bf16)(float)v[e];
    hi[e] = (__bf16)(float)v[8 + e];
  }
  *reinterpret_cast<bf8*>(dst) = lo;
  *reinterpret_cast<bf8*>(dst + 8) = hi;
}

template <bool TRANSB>
__global__ __launch_bounds__(256) void k_gemm_sub_bf16(int m, int n, int k, const double* __restrict__ A, int lda,
                                                       const double* __restrict__ B, int ldb, double* __restrict__ C,
                                                       int ldc, int lower, int tiles_m, int ntiles,
                                                       const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int per = gridDim.x >> 3;
  const int lin = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (lin >= ntiles) return;
  int ti, tj;
  tile_of(lin, lower, tiles_m, ti, tj);
  const int row0 = ti * TM, col0 = tj * TN;

  __shared__ __attribute__((aligned(16))) __bf16 As[2][TM][BK16 + PAD16];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][TN][BK16 + PAD16];

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int wm = w & 1, wn = w >> 1;
  // A and op(B) with rows along memory (A; B^T stored, NT): row t % 128, k half t / 128
  const int r_i = t & 127, r_kh = (t >> 7) * 16;
  // B (NN) with k along memory: column t / 2, k half t % 2
  const int c_j = t >> 1, c_kh = (t & 1) * 16;

  double ra[16], rb[16];
  auto load_regs = [&](int k0) {
    {
      const int i = row0 + r_i;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int kk = k0 + r_kh + e;
        ra[e] = (i < m && kk < k) ? A[(size_t)i + (size_t)kk * lda] : 0.0;
      }
    }
    if (!TRANSB) {
      const int j = col0 + c_j;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int kk = k0 + c_kh + e;
        rb[e] = (j < n && kk < k) ? B[(size_t)kk + (size_t)j * ldb] : 0.0;
      }
    } else {
      const int j = col0 + r_i;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int kk = k0 + r_kh + e;
        rb[e] = (j < n && kk < k) ? B[(size_t)j + (size_t)kk * ldb] : 0.0;
      }
    }
  };
  auto store_lds = [&](int buf) {
    put16(&As[buf][r_i][r_kh], ra);
    if (!TRANSB) put16(&Bs[buf][c_j][c_kh], rb);
    else put16(&Bs[buf][r_i][r_kh], rb);
  };

  f4 acc[4][4];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = f4{0.f, 0.f, 0.f, 0.f};

  const int nch = (k + BK16 - 1) / BK16;
  load_regs(0);
  store_lds(0);
  __syncthreads();
  const int lr = lane & 15, lk = (lane >> 4) * 8;
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) load_regs((c + 1) * BK16);
    bf8 af[4], bf[4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) af[bi] = *reinterpret_cast<const bf8*>(&As[buf][wm * 64 + bi * 16 + lr][lk]);
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) bf[bj] = *reinterpret_cast<const bf8*>(&Bs[buf][wn * 64 + bj * 16 + lr][lk]);
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < 4; ++bj)
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bf[bj], af[bi], acc[bi][bj], 0, 0, 0);
    if (c + 1 < nch) store_lds(buf ^ 1);
    __syncthreads();
  }
  store_sub(acc, m, n, C, ldc, row0, col0, wm, wn, lane);
}

}  // namespace

hipError_t launch_gemm_sub_lp(int prec, int m, int n, int k, const double* A, int lda, const double* B, int ldb,
                              bool transB, double* C, int ldc, bool lower, const int* skip_if_nonzero,
                              hipStream_t st) {
  if (m <= 0 || n <= 0 || k <= 0) return hipSuccess;
  if (prec != ADA_PREC_FP32_IR && prec != ADA_PREC_BF16_IR) return hipErrorInvalidValue;
  const int tiles_m = (m + TM - 1) / TM, tiles_n = (n + TN - 1) / TN;
  const int ntiles = lower ? tiles_m * (tiles_m + 1) / 2 : tiles_m * tiles_n;
  const int grid = ((ntiles + 7) / 8) * 8;
  const int lo = (int)lower;
  if (prec == ADA_PREC_FP32_IR) {
    if (transB)
      hipLaunchKernelGGL(k_gemm_sub_f32<true>, dim3(grid), dim3(256), 0, st, m, n, k, A, lda, B, ldb, C, ldc, lo,
                         tiles_m, ntiles, skip_if_nonzero);
    else
      hipLaunchKernelGGL(k_gemm_sub_f32<false>, dim3(grid), dim3(256), 0, st, m, n, k, A, lda, B, ldb, C, ldc, lo,
                         tiles_m, ntiles, skip_if_nonzero);
  } else {
    if (transB)
      hipLaunchKernelGGL(k_gemm_sub_bf16<true>, dim3(grid), dim3(256), 0, st, m, n, k, A, lda, B, ldb, C, ldc, lo,
                         tiles_m, ntiles, skip_if_nonzero);
    else
      hipLaunchKernelGGL(k_gemm_sub_bf16<false>, dim3(grid), dim3(256), 0, st, m, n, k, A, lda, B, ldb, C, ldc, lo,
                         tiles_m, ntiles, skip_if_nonzero);
  }
  return hipGetLastError();
}

}  // namespace ada
