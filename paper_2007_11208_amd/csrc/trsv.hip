// Triangular solve op(T) X = B in place (X holds B on entry), used for the
// triangular route (Section II-B, eq. 3), the LU solve (eq. 4), the Cholesky
// solve and every solve of the condition estimate.
//
// One kernel launch per solve. The rows are cut into 64-row blocks; each
// workgroup takes the next block in solve order from a ticket counter, stages
// the 64x64 tiles of its block row through LDS, subtracts the contribution of
// every earlier block as soon as that block's flag shows it is finished, then
// runs substitution on its own diagonal block and publishes its rows with a
// release store of the flag. Tickets follow start order, so a workgroup only
// waits for workgroups that started before it: no deadlock, whatever the grid.
// Waits are bounded.
#include "ada_internal.h"

namespace ada {

constexpr int TB = 64;

__global__ __launch_bounds__(256) void k_trsm_dec(int n, int nrhs, const double* __restrict__ T, int ldt, int lower,
                                                  int trans, int unit, double* X, int ldx, int* flags, int epoch,
                                                  unsigned* ticket, DevRec* rec, const int* pred, int pred_val) {
  if (pred && *pred != pred_val) return;
  const int t = threadIdx.x;
  const int nblk = (n + TB - 1) / TB;
  __shared__ int s_tk;
  if (t == 0) s_tk = (int)atomicAdd(ticket, 1u);
  __syncthreads();
  const int tk = s_tk;
  if (tk >= nblk) return;
  const bool eff_lower = (lower != 0) != (trans != 0);
  const int bi = eff_lower ? tk : (nblk - 1 - tk);
  const int r0 = bi * TB;
  const int rows = min(TB, n - r0);

  extern __shared__ double sm[];
  double* acc = sm;                    // acc[c * TB + r]
  double* tile = acc + TB * nrhs;      // tile[k * (TB + 1) + r] = op(T)(r0 + r, c0 + k)
  double* xj = tile + TB * (TB + 1);   // xj[c * TB + k]

  for (int e = t; e < TB * nrhs; e += blockDim.x) {
    const int r = e % TB, c = e / TB;
    acc[e] = (r < rows) ? X[(size_t)(r0 + r) + (size_t)c * ldx] : 0.0;
  }

  auto stage_tile = [&](int c0, int cols) {
    if (!trans) {
      for (int e = t; e < TB * TB; e += blockDim.x) {
        const int r = e % TB, k = e / TB;
        tile[k * (TB + 1) + r] = (r < rows && k < cols) ? T[(size_t)(r0 + r) + (size_t)(c0 + k) * ldt] : 0.0;
      }
    } else {
      for (int e = t; e < TB * TB; e += blockDim.x) {
        const int k = e % TB, r = e / TB;
        tile[k * (TB + 1) + r] = (r < rows && k < cols) ? T[(size_t)(c0 + k) + (size_t)(r0 + r) * ldt] : 0.0;
      }
    }
  };

  for (int q = 0; q < tk; ++q) {
    const int bj = eff_lower ? q : (nblk - 1 - q);
    const int c0 = bj * TB;
    const int cols = min(TB, n - c0);
    stage_tile(c0, cols);
    if (t == 0) {
      long spins = 0;
      while (agent_load(&flags[bj]) != epoch) {
        if (++spins > kSpinLimit) {
          atomicOr(&rec->timeout, 1);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __syncthreads();
    for (int e = t; e < TB * nrhs; e += blockDim.x) {
      const int k = e % TB, c = e / TB;
      xj[e] = (k < cols) ? X[(size_t)(c0 + k) + (size_t)c * ldx] : 0.0;
    }
    __syncthreads();
    {
      const int r = t & 63;
      for (int c = t >> 6; c < nrhs; c += 4) {
        double s = 0.0;
        const double* xc = xj + c * TB;
#pragma unroll 16
        for (int k = 0; k < TB; ++k) s = fma(tile[k * (TB + 1) + r], xc[k], s);
        acc[c * TB + r] -= s;
      }
    }
    __syncthreads();
  }

  // diagonal block: substitution
  stage_tile(r0, rows);
  __syncthreads();
  if (nrhs <= 4) {
    // wave w solves column w; lane = row
    const int w = t >> 6, lane = t & 63;
    if (w < nrhs) {
      double a = acc[w * TB + lane];
      if (eff_lower) {
        for (int i = 0; i < rows; ++i) {
          double xi = unit ? a : a / tile[i * (TB + 1) + i];
          xi = __shfl(xi, i, 64);
          if (lane == i) a = xi;
          if (lane > i) a = fma(-tile[i * (TB + 1) + lane], xi, a);
        }
      } else {
        for (int i = rows - 1; i >= 0; --i) {
          double xi = unit ? a : a / tile[i * (TB + 1) + i];
          xi = __shfl(xi, i, 64);
          if (lane == i) a = xi;
          if (lane < i) a = fma(-tile[i * (TB + 1) + lane], xi, a);
        }
      }
      acc[w * TB + lane] = a;
    }
  } else {
    // thread c solves column c
    for (int c = t; c < nrhs; c += blockDim.x) {
      double* a = acc + c * TB;
      if (eff_lower) {
        for (int i = 0; i < rows; ++i) {
          const double xi = unit ? a[i] : a[i] / tile[i * (TB + 1) + i];
          a[i] = xi;
          for (int r = i + 1; r < rows; ++r) a[r] = fma(-tile[i * (TB + 1) + r], xi, a[r]);
        }
      } else {
        for (int i = rows - 1; i >= 0; --i) {
          const double xi = unit ? a[i] : a[i] / tile[i * (TB + 1) + i];
          a[i] = xi;
          for (int r = 0; r < i; ++r) a[r] = fma(-tile[i * (TB + 1) + r], xi, a[r]);
        }
      }
    }
  }
  __syncthreads();
  for (int e = t; e < TB * nrhs; e += blockDim.x) {
    const int r = e % TB, c = e / TB;
    if (r < rows) X[(size_t)(r0 + r) + (size_t)c * ldx] = acc[e];
  }
  __threadfence();
  __syncthreads();
  if (t == 0) __hip_atomic_store(&flags[bi], epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

hipError_t launch_trsm_dec(int n, int nrhs, const double* T, int ldt, bool lower, bool trans, bool unit, double* X,
                           int ldx, int* flags, int epoch, unsigned* ticket, DevRec* rec, const int* pred,
                           int pred_val, hipStream_t st) {
  if (nrhs < 1 || nrhs > 64) return hipErrorInvalidValue;
  const int nblk = (n + TB - 1) / TB;
  const size_t lds = sizeof(double) * ((size_t)TB * nrhs * 2 + (size_t)TB * (TB + 1));
  static size_t done = 0;
  hipError_t e = ensure_lds((const void*)k_trsm_dec, lds, done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_trsm_dec, dim3(nblk), dim3(256), lds, st, n, nrhs, T, ldt, (int)lower, (int)trans,
                     (int)unit, X, ldx, flags, epoch, ticket, rec, pred, pred_val);
  return hipGetLastError();
}

}  // namespace ada
