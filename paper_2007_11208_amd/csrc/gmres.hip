// Column-wise vector kernels of GMRES-based iterative refinement (the correction equation of the
// mixed-precision solve, Section II-D's LU and Section II-C's Cholesky in low precision used as the
// preconditioner): every right-hand side j has a Krylov basis of its own, the basis vectors of all
// right-hand sides are stored together, V_i = V + i * vstride (n x nrhs, ld n). All arithmetic FP64.
#include "ada_internal.h"

namespace ada {

namespace {
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += red[q];
  return s;
}
}  // namespace

// h[i + j * ldh] = V_i(:, j) . W(:, j) for i < kk (grid kk x nrhs); sum in a fixed order
__global__ __launch_bounds__(256) void k_col_dots(int n, const double* __restrict__ V, size_t vstride,
                                                  const double* __restrict__ W, int ldw, double* h, int ldh) {
  __shared__ double red[4];
  const int i = blockIdx.x, j = blockIdx.y;
  const double* v = V + (size_t)i * vstride + (size_t)j * n;
  const double* w = W + (size_t)j * ldw;
  double s = 0.0;
  for (int r = threadIdx.x; r < n; r += 256) s = fma(v[r], w[r], s);
  s = block_sum(s, red);
  if (threadIdx.x == 0) h[i + (size_t)j * ldh] = s;
}

// W(:, j) += sign * sum_{i < kk} h[i + j * ldh] V_i(:, j)
__global__ __launch_bounds__(256) void k_col_axpy(int n, int nrhs, int kk, const double* __restrict__ V,
                                                  size_t vstride, const double* __restrict__ h, int ldh,
                                                  double sign, double* W, int ldw) {
  const int j = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n || j >= nrhs) return;
  double acc = W[r + (size_t)j * ldw];
  for (int i = 0; i < kk; ++i) acc = fma(sign * h[i + (size_t)j * ldh], V[(size_t)i * vstride + r + (size_t)j * n], acc);
  W[r + (size_t)j * ldw] = acc;
}

// D(:, j) = S(:, j) * s_j with s_j = sign / sqrt(nrm2[j * ldn]) (0 when the norm is 0)
__global__ __launch_bounds__(256) void k_col_normalize(int n, int nrhs, const double* __restrict__ S, int lds,
                                                       const double* __restrict__ nrm2, int ldn, double sign,
                                                       double* D, int ldd) {
  const int j = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n || j >= nrhs) return;
  const double q = nrm2[(size_t)j * ldn];
  const double sc = q > 0.0 ? sign / sqrt(q) : 0.0;
  D[r + (size_t)j * ldd] = S[r + (size_t)j * lds] * sc;
}

hipError_t launch_col_dots(int n, int nrhs, int kk, const double* V, size_t vstride, const double* W, int ldw,
                           double* h, int ldh, hipStream_t st) {
  if (kk < 1 || nrhs < 1) return hipSuccess;
  hipLaunchKernelGGL(k_col_dots, dim3(kk, nrhs), dim3(256), 0, st, n, V, vstride, W, ldw, h, ldh);
  return hipGetLastError();
}

hipError_t launch_col_axpy(int n, int nrhs, int kk, const double* V, size_t vstride, const double* h, int ldh,
                           double sign, double* W, int ldw, hipStream_t st) {
  if (kk < 1 || nrhs < 1) return hipSuccess;
  hipLaunchKernelGGL(k_col_axpy, dim3((n + 255) / 256, nrhs), dim3(256), 0, st, n, nrhs, kk, V, vstride, h, ldh,
                     sign, W, ldw);
  return hipGetLastError();
}

hipError_t launch_col_normalize(int n, int nrhs, const double* S, int lds, const double* nrm2, int ldn, double sign,
                                double* D, int ldd, hipStream_t st) {
  hipLaunchKernelGGL(k_col_normalize, dim3((n + 255) / 256, nrhs), dim3(256), 0, st, n, nrhs, S, lds, nrm2, ldn,
                     sign, D, ldd);
  return hipGetLastError();
}

}  // namespace ada
