// Copies, row permutations, the residual R = B - A X and the normwise
// backward error max_k ||r_k||_inf / (||A||_inf ||x_k||_inf + ||b_k||_inf)
// (an accuracy metric; the paper does not define one).
#include "ada_internal.h"

namespace ada {

__global__ void k_copy(int rows, int cols, const double* __restrict__ S, int lds, double* __restrict__ D, int ldd) {
  const size_t total = (size_t)rows * cols;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e % rows, j = e / rows;
    D[i + j * ldd] = S[i + j * lds];
  }
}

hipError_t launch_copy(int rows, int cols, const double* S, int lds, double* D, int ldd, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  size_t total = (size_t)rows * cols;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, st, rows, cols, S, lds, D, ldd);
  return hipGetLastError();
}

__global__ void k_iota(int* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = i;
}

hipError_t launch_iota(int* p, int n, hipStream_t st) {
  int blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_iota, dim3(blocks), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

// D[i,:] = S[perm[i],:]  (P b, perm[i] = original row now at position i)
__global__ void k_gather_rows(int n, int nrhs, const int* __restrict__ perm, const double* __restrict__ S, int lds,
                              double* __restrict__ D, int ldd, const int* pred, int pred_val) {
  if (pred && *pred != pred_val) return;
  const size_t total = (size_t)n * nrhs;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), c = (int)(e / n);
    D[(size_t)i + (size_t)c * ldd] = S[(size_t)perm[i] + (size_t)c * lds];
  }
}

// D[perm[i],:] = S[i,:]  (P^T w)
__global__ void k_scatter_rows(int n, int nrhs, const int* __restrict__ perm, const double* __restrict__ S, int lds,
                               double* __restrict__ D, int ldd, const int* pred, int pred_val) {
  if (pred && *pred != pred_val) return;
  const size_t total = (size_t)n * nrhs;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), c = (int)(e / n);
    D[(size_t)perm[i] + (size_t)c * ldd] = S[(size_t)i + (size_t)c * lds];
  }
}

hipError_t launch_gather_rows(int n, int nrhs, const int* perm, const double* S, int lds, double* D, int ldd,
                              const int* pred, int pred_val, hipStream_t st) {
  size_t total = (size_t)n * nrhs;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_gather_rows, dim3(blocks), dim3(256), 0, st, n, nrhs, perm, S, lds, D, ldd, pred, pred_val);
  return hipGetLastError();
}

hipError_t launch_scatter_rows(int n, int nrhs, const int* perm, const double* S, int lds, double* D, int ldd,
                               const int* pred, int pred_val, hipStream_t st) {
  size_t total = (size_t)n * nrhs;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_scatter_rows, dim3(blocks), dim3(256), 0, st, n, nrhs, perm, S, lds, D, ldd, pred, pred_val);
  return hipGetLastError();
}

// R = B - A X, accurately (Dot2: every product split exactly, the sums
// compensated), for right-hand sides in groups of 8 (blockIdx.z): rows over
// threads, the n columns of A split into chunks over blockIdx.y; each chunk's
// compensated partial sum (s, c) goes to P[group][chunk][c][i] and k_resid_sum
// adds them in chunk order, again compensated (deterministic).
constexpr int RCH = 512;  // columns of A per chunk
__global__ __launch_bounds__(256) void k_resid_part(int n, int nrhs, const double* __restrict__ A, int lda,
                                                    const double* __restrict__ X, int ldx, double* __restrict__ P) {
  __shared__ double sx[64][8];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int g0 = blockIdx.z * 8, ng = min(8, nrhs - g0);
  const int nch = gridDim.y;
  const int j0 = blockIdx.y * RCH, j1 = min(n, j0 + RCH);
  double s[8], c[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) s[q] = c[q] = 0.0;
  for (int jb = j0; jb < j1; jb += 64) {
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 8; e += blockDim.x) {
      const int jj = e / 8, q = e % 8;
      sx[jj][q] = (jb + jj < j1 && q < ng) ? X[(size_t)(jb + jj) + (size_t)(g0 + q) * ldx] : 0.0;
    }
    __syncthreads();
    if (i < n) {
      const int jn = min(64, j1 - jb);
      for (int jj = 0; jj < jn; ++jj) {
        const double a = A[(size_t)i + (size_t)(jb + jj) * lda];
#pragma unroll
        for (int q = 0; q < 8; ++q) dot2_sub(s[q], c[q], a, sx[jj][q]);
      }
    }
  }
  if (i < n) {
    double* Pg = P + (size_t)blockIdx.z * nch * 8 * 2 * n;
    for (int q = 0; q < ng; ++q) {
      Pg[(((size_t)blockIdx.y * 8 + q) * 2 + 0) * n + i] = s[q];
      Pg[(((size_t)blockIdx.y * 8 + q) * 2 + 1) * n + i] = c[q];
    }
  }
}

__global__ void k_resid_sum(int n, int nrhs, int nch, const double* __restrict__ B, int ldb,
                            const double* __restrict__ P, double* __restrict__ R, int ldr) {
  const size_t total = (size_t)n * nrhs;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), col = (int)(e / n);
    const int g = col / 8, q = col % 8;
    const double* Pg = P + (size_t)g * nch * 8 * 2 * n;
    double s = B[(size_t)i + (size_t)col * ldb], c = 0.0;
    for (int ch = 0; ch < nch; ++ch) {
      two_sum_acc(s, c, Pg[(((size_t)ch * 8 + q) * 2 + 0) * n + i]);
      c += Pg[(((size_t)ch * 8 + q) * 2 + 1) * n + i];
    }
    R[(size_t)i + (size_t)col * ldr] = s + c;
  }
}

size_t resid_partial_doubles(int n, int nrhs) {
  const size_t nch = (size_t)((n + RCH - 1) / RCH);
  return (size_t)((nrhs + 7) / 8) * nch * 8 * 2 * (size_t)n;
}

// P must hold resid_partial_doubles(n, nrhs) doubles.
hipError_t launch_resid_gemv(int n, int nrhs, const double* A, int lda, const double* B, int ldb, const double* X,
                             int ldx, double* R, int ldr, double* P, hipStream_t st) {
  const int nch = (n + RCH - 1) / RCH;
  const int groups = (nrhs + 7) / 8;
  if (groups > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_resid_part, dim3((n + 255) / 256, nch, groups), dim3(256), 0, st, n, nrhs, A, lda, X, ldx, P);
  size_t total = (size_t)n * nrhs;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_resid_sum, dim3(blocks), dim3(256), 0, st, n, nrhs, nch, B, ldb, P, R, ldr);
  return hipGetLastError();
}

// eta_c = ||r_c||_inf / (||A||_inf ||x_c||_inf + ||b_c||_inf) per right-hand side, then the maximum.
// The three maxima of each column are formed by a grid of workgroups with
// atomic maxima on the bit patterns (non-negative doubles order like their bits),
// so the result does not depend on the order.
__global__ void k_berr_zero(int nrhs, unsigned long long* acc) {
  for (int e = threadIdx.x; e < 4 * nrhs; e += blockDim.x) acc[e] = 0ull;
}

__global__ __launch_bounds__(256) void k_berr_part(int n, const double* __restrict__ R, int ldr,
                                                   const double* __restrict__ B, int ldb,
                                                   const double* __restrict__ X, int ldx,
                                                   unsigned long long* acc) {
  const int c = blockIdx.y;
  double rn = 0.0, xn = 0.0, bn = 0.0;
  int nf = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double r = R[(size_t)i + (size_t)c * ldr];
    const double x = X[(size_t)i + (size_t)c * ldx];
    const double b = B[(size_t)i + (size_t)c * ldb];
    nf |= !isfinite(x);
    rn = fmax(rn, fabs(r));
    xn = fmax(xn, fabs(x));
    bn = fmax(bn, fabs(b));
  }
  rn = wave_max(rn);
  xn = wave_max(xn);
  bn = wave_max(bn);
  nf = wave_or(nf);
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&acc[4 * c + 0], dbits(rn));
    atomicMax(&acc[4 * c + 1], dbits(xn));
    atomicMax(&acc[4 * c + 2], dbits(bn));
    if (nf) atomicOr(&acc[4 * c + 3], 1ull);
  }
}

__global__ void k_berr_max(int nrhs, const unsigned long long* acc, DevRec* rec) {
  double m = 0.0;
  bool nan = false, nonfinite = false;
  const double an = rec->anorm_inf;
  for (int c = 0; c < nrhs; ++c) {
    const double rn = __longlong_as_double((long long)acc[4 * c + 0]);
    const double xn = __longlong_as_double((long long)acc[4 * c + 1]);
    const double bn = __longlong_as_double((long long)acc[4 * c + 2]);
    if (acc[4 * c + 3]) nonfinite = true;
    const double den = an * xn + bn;
    double v = den > 0.0 ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
    if (acc[4 * c + 3]) v = __longlong_as_double(0x7ff8000000000000LL);
    if (v != v) nan = true;
    else m = fmax(m, v);
  }
  if (nonfinite) rec->x_nonfinite = 1;
  rec->berr = nan ? __longlong_as_double(0x7ff8000000000000LL) : m;
}

hipError_t launch_berr(int n, int nrhs, const double* R, int ldr, const double* B, int ldb, const double* X,
                       int ldx, double* per_col, DevRec* rec, hipStream_t st) {
  unsigned long long* acc = reinterpret_cast<unsigned long long*>(per_col);  // 4 * nrhs words
  hipLaunchKernelGGL(k_berr_zero, dim3(1), dim3(256), 0, st, nrhs, acc);
  int gx = (n + 2047) / 2048;
  gx = gx < 1 ? 1 : (gx > 256 ? 256 : gx);
  hipLaunchKernelGGL(k_berr_part, dim3(gx, nrhs), dim3(256), 0, st, n, R, ldr, B, ldb, X, ldx, acc);
  hipLaunchKernelGGL(k_berr_max, dim3(1), dim3(1), 0, st, nrhs, acc, rec);
  return hipGetLastError();
}

// X += D (n x nrhs), the correction step of iterative refinement
__global__ void k_add_to(int n, int nrhs, const double* __restrict__ D, int ldd, double* __restrict__ X, int ldx) {
  const size_t total = (size_t)n * nrhs;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e % n, c = e / n;
    X[i + c * ldx] += D[i + c * ldd];
  }
}

hipError_t launch_add_to(int n, int nrhs, const double* D, int ldd, double* X, int ldx, hipStream_t st) {
  const size_t total = (size_t)n * nrhs;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_add_to, dim3(blocks), dim3(256), 0, st, n, nrhs, D, ldd, X, ldx);
  return hipGetLastError();
}

// x finiteness only (used when the backward error is not requested)
__global__ void k_x_finite(int n, int nrhs, const double* __restrict__ X, int ldx, DevRec* rec) {
  const size_t total = (size_t)n * nrhs;
  int bad = 0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e % n, c = e / n;
    bad |= !isfinite(X[i + c * ldx]);
  }
  bad = wave_or(bad);
  if ((threadIdx.x & 63) == 0 && bad) atomicOr(&rec->x_nonfinite, 1);
}

hipError_t launch_x_finite(int n, int nrhs, const double* X, int ldx, DevRec* rec, hipStream_t st) {
  size_t total = (size_t)n * nrhs;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_x_finite, dim3(blocks), dim3(256), 0, st, n, nrhs, X, ldx, rec);
  return hipGetLastError();
}

__global__ void k_set_identity(int n, double* V, int ldv) {
  const size_t total = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e % n, j = e / n;
    V[i + j * ldv] = (i == j) ? 1.0 : 0.0;
  }
}

hipError_t launch_set_identity(int n, double* V, int ldv, hipStream_t st) {
  size_t total = (size_t)n * n;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_set_identity, dim3(blocks), dim3(256), 0, st, n, V, ldv);
  return hipGetLastError();
}

// mark the routed solve as failed when the factorisation reported a zero pivot
__global__ void k_mark_stop(DevRec* rec) {
  if (rec->info != 0x7fffffff) rec->stop = 1;
}

hipError_t launch_mark_stop(DevRec* rec, hipStream_t st) {
  hipLaunchKernelGGL(k_mark_stop, dim3(1), dim3(1), 0, st, rec);
  return hipGetLastError();
}

}  // namespace ada
