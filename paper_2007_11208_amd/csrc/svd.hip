// SVD-based minimum-norm least-squares fallback (Section II-E) by one-sided
// (Hestenes) Jacobi with V accumulating the rotations. Pairs are visited in
// round-robin (tournament) order, so the n/2 pairs of a round are disjoint and
// are rotated in parallel. A pair is rotated when
// |u_p^T u_q| > n*eps*||u_p|| ||u_q||, with Rutishauser's formulas.
//
// Preconditioning (Drmac and Veselic's QR-preconditioned one-sided Jacobi):
// the columns of A are ordered by decreasing norm (A P), A P = Q R by
// Householder reflectors, and the Jacobi runs on R^T, whose columns are graded:
// the sweeps drop from the cap of 30 (dense log-spaced spectra, triangular
// matrices with N(0,1) entries) to about 10. With R^T W = U~ (columns of norm
// sigma_j): A P = (Q W) Sigma (U~ Sigma^{-1})^T, so
// x = P sum_{sigma_j > eps*sigma_max} u~_j (w_j^T Q^T b) / sigma_j^2.
#include "ada_internal.h"

namespace ada {

__device__ __forceinline__ void rr_pair(int m, int r, int pi, int& a, int& b) {
  if (pi == 0) {
    a = r;
    b = m - 1;
  } else {
    a = (r + pi) % (m - 1);
    b = (r - pi + m - 1) % (m - 1);
  }
}

__device__ __forceinline__ void rotation(double alpha, double beta, double gamma, double& c, double& s) {
  const double zeta = (beta - alpha) / (2.0 * gamma);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
  c = 1.0 / sqrt(1.0 + t * t);
  s = c * t;
}

// whole algorithm in one workgroup (small n); U, V stay in L2
__global__ __launch_bounds__(1024) void k_jacobi_small(int n, double* U, int ldu, double* V, int ldv, double* Y,
                                                       int ldy, int ny, int max_sweeps, DevRec* rec) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = blockDim.x >> 6;
  const int m = (n + 1) & ~1;
  const double tol = (double)n * kEps;
  __shared__ int s_rot;
  int sweeps = 0;
  for (; sweeps < max_sweeps; ++sweeps) {
    if (t == 0) s_rot = 0;
    __syncthreads();
    for (int r = 0; r < m - 1; ++r) {
      for (int pi = w; pi < m / 2; pi += nw) {
        int a, b;
        rr_pair(m, r, pi, a, b);
        if (a >= n || b >= n) continue;
        const int p = min(a, b), q = max(a, b);
        double* up = U + (size_t)p * ldu;
        double* uq = U + (size_t)q * ldu;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int i = lane; i < n; i += 64) {
          const double x = up[i], y = uq[i];
          al = fma(x, x, al);
          be = fma(y, y, be);
          ga = fma(x, y, ga);
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (!(fabs(ga) > tol * sqrt(al) * sqrt(be))) continue;
        double c, s;
        rotation(al, be, ga, c, s);
        for (int i = lane; i < n; i += 64) {
          const double x = up[i], y = uq[i];
          up[i] = c * x - s * y;
          uq[i] = s * x + c * y;
        }
        if (V) {
          double* vp = V + (size_t)p * ldv;
          double* vq = V + (size_t)q * ldv;
          for (int i = lane; i < n; i += 64) {
            const double x = vp[i], y = vq[i];
            vp[i] = c * x - s * y;
            vq[i] = s * x + c * y;
          }
        }
        for (int k = lane; k < ny; k += 64) {
          const double x = Y[p + (size_t)k * ldy], y = Y[q + (size_t)k * ldy];
          Y[p + (size_t)k * ldy] = c * x - s * y;
          Y[q + (size_t)k * ldy] = s * x + c * y;
        }
        if (lane == 0) s_rot = 1;
      }
      __syncthreads();
    }
    const int rot = s_rot;
    __syncthreads();
    if (!rot) { ++sweeps; break; }
  }
  if (t == 0) rec->sweeps = sweeps;
}

hipError_t launch_jacobi_small(int n, double* U, int ldu, double* V, int ldv, double* Y, int ldy, int ny,
                               int max_sweeps, DevRec* rec, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_small, dim3(1), dim3(1024), 0, st, n, U, ldu, V, ldv, Y, ldy, ny, max_sweeps, rec);
  return hipGetLastError();
}

// one round of the tournament, one pair per workgroup
__global__ __launch_bounds__(256) void k_jacobi_round(int n, int m, int round, double* U, int ldu, double* V, int ldv,
                                                      double* Y, int ldy, int ny, DevRec* rec) {
  int a, b;
  rr_pair(m, round, blockIdx.x, a, b);
  if (a >= n || b >= n) return;
  const int p = min(a, b), q = max(a, b);
  const int t = threadIdx.x;
  double* up = U + (size_t)p * ldu;
  double* uq = U + (size_t)q * ldu;
  double al = 0.0, be = 0.0, ga = 0.0;
  for (int i = t; i < n; i += blockDim.x) {
    const double x = up[i], y = uq[i];
    al = fma(x, x, al);
    be = fma(y, y, be);
    ga = fma(x, y, ga);
  }
  al = wave_sum(al);
  be = wave_sum(be);
  ga = wave_sum(ga);
  __shared__ double s[3][4];
  const int w = t >> 6;
  if ((t & 63) == 0) { s[0][w] = al; s[1][w] = be; s[2][w] = ga; }
  __syncthreads();
  al = s[0][0] + s[0][1] + s[0][2] + s[0][3];
  be = s[1][0] + s[1][1] + s[1][2] + s[1][3];
  ga = s[2][0] + s[2][1] + s[2][2] + s[2][3];
  const double tol = (double)n * kEps;
  if (!(fabs(ga) > tol * sqrt(al) * sqrt(be))) return;
  double c, sn;
  rotation(al, be, ga, c, sn);
  for (int i = t; i < n; i += blockDim.x) {
    const double x = up[i], y = uq[i];
    up[i] = c * x - sn * y;
    uq[i] = sn * x + c * y;
  }
  if (V) {
    double* vp = V + (size_t)p * ldv;
    double* vq = V + (size_t)q * ldv;
    for (int i = t; i < n; i += blockDim.x) {
      const double x = vp[i], y = vq[i];
      vp[i] = c * x - sn * y;
      vq[i] = sn * x + c * y;
    }
  }
  for (int r = t; r < ny; r += blockDim.x) {
    const double x = Y[p + (size_t)r * ldy], y = Y[q + (size_t)r * ldy];
    Y[p + (size_t)r * ldy] = c * x - sn * y;
    Y[q + (size_t)r * ldy] = sn * x + c * y;
  }
  if (t == 0) atomicOr(&rec->jacobi_rotated, 1);
}

hipError_t launch_jacobi_round(int n, int m, int round, double* U, int ldu, double* V, int ldv, double* Y, int ldy,
                               int ny, DevRec* rec, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_round, dim3(m / 2), dim3(256), 0, st, n, m, round, U, ldu, V, ldv, Y, ldy, ny, rec);
  return hipGetLastError();
}

// Blocked form of the same cyclic one-sided Jacobi for 1024 < n <= 4096: the columns form blocks of
// four; one workgroup holds two blocks (eight columns, rows spread over 1024 threads, four rows per
// thread) in registers and applies the ordinary two-column rotations to every pair that crosses the
// two blocks (four rounds of four disjoint pairs), or, in the intra step, to the six pairs inside
// one block. A sweep is one intra step and a round-robin over block pairs, so every column pair is
// visited once per sweep as in the per-pair form, while U streams through HBM about n/4 times per
// sweep instead of n. The right-hand sides' projections (rows of Y) turn with their columns.
constexpr int JB_T = 1024;
constexpr int JB_R = 4;       // rows per thread (n <= 4096)
constexpr int JB_YMAX = 64;   // projections held in LDS (columns of Y)

// slots of the pairs of round rd: intra {(0,1),(2,3)}, {(0,2),(1,3)}, {(0,3),(1,2)}; cross (k, 4+(k+rd)%4)
template <bool INTRA>
__device__ __forceinline__ constexpr int blk_pa(int rd, int k) {
  return INTRA ? (k == 0 ? 0 : (rd == 0 ? 2 : 1)) : k;
}
template <bool INTRA>
__device__ __forceinline__ constexpr int blk_pb(int rd, int k) {
  return INTRA ? (k == 0 ? rd + 1 : (rd == 2 ? 2 : 3)) : 4 + ((k + rd) & 3);
}

template <bool INTRA>
__global__ __launch_bounds__(JB_T) void k_jacobi_blk(int n, int nbm, int round, double* __restrict__ U, int ldu,
                                                     double* __restrict__ Y, int ldy, int ny, DevRec* rec) {
  const bool intra = INTRA;
  const int nblk = (n + 3) / 4;
  int ba, bb;
  if (intra) {
    ba = blockIdx.x;
    bb = -1;
  } else {
    rr_pair(nbm, round, blockIdx.x, ba, bb);
    if (ba >= nblk || bb >= nblk) return;
  }
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int nslot = intra ? 4 : 8;
  __shared__ double sy[8][JB_YMAX];
  __shared__ double sred[JB_T / 64][12];
  __shared__ double stot[12];
  __shared__ int s_any;
  int col[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) col[k] = k < 4 ? ba * 4 + k : (bb >= 0 ? bb * 4 + (k - 4) : n);
  double u[8][JB_R];
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int q = 0; q < JB_R; ++q) {
      const int row = t + q * JB_T;
      u[k][q] = (k < nslot && col[k] < n && row < n) ? U[row + (size_t)col[k] * ldu] : 0.0;
    }
  for (int e = t; e < nslot * ny; e += JB_T) {
    const int k = e / ny, c = e % ny;
    sy[k][c] = col[k] < n ? Y[col[k] + (size_t)c * ldy] : 0.0;
  }
  if (t == 0) s_any = 0;
  __syncthreads();
  const double tol = (double)n * kEps;
  constexpr int nrounds = INTRA ? 3 : 4;
  constexpr int np = INTRA ? 2 : 4;
#pragma unroll
  for (int rd = 0; rd < nrounds; ++rd) {
    double part[12];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double al = 0.0, be = 0.0, ga = 0.0;
      if (k < np) {
#pragma unroll
        for (int q = 0; q < JB_R; ++q) {
          const double x = u[blk_pa<INTRA>(rd, k)][q], y = u[blk_pb<INTRA>(rd, k)][q];
          al = fma(x, x, al);
          be = fma(y, y, be);
          ga = fma(x, y, ga);
        }
      }
      part[3 * k] = wave_sum(al);
      part[3 * k + 1] = wave_sum(be);
      part[3 * k + 2] = wave_sum(ga);
    }
    if (lane == 0)
#pragma unroll
      for (int k = 0; k < 12; ++k) sred[w][k] = part[k];
    __syncthreads();
    if (t < 12) {
      double sum = 0.0;
      for (int q = 0; q < JB_T / 64; ++q) sum += sred[q][t];
      stot[t] = sum;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (k >= np) continue;
      const int sa = blk_pa<INTRA>(rd, k), sb = blk_pb<INTRA>(rd, k);
      if (col[sa] >= n || col[sb] >= n) continue;
      // the first column of the pair is the lower index (the per-pair form's convention)
      const bool swap = col[sa] > col[sb];
      const double al = swap ? stot[3 * k + 1] : stot[3 * k], be = swap ? stot[3 * k] : stot[3 * k + 1];
      const double ga = stot[3 * k + 2];
      if (!(fabs(ga) > tol * sqrt(al) * sqrt(be))) continue;
      double c, sn;
      rotation(al, be, ga, c, sn);
      const int sp = swap ? sb : sa, sq = swap ? sa : sb;
      if (!swap) {
#pragma unroll
        for (int q = 0; q < JB_R; ++q) {
          const double x = u[sa][q], y = u[sb][q];
          u[sa][q] = c * x - sn * y;
          u[sb][q] = sn * x + c * y;
        }
      } else {
#pragma unroll
        for (int q = 0; q < JB_R; ++q) {
          const double x = u[sb][q], y = u[sa][q];
          u[sb][q] = c * x - sn * y;
          u[sa][q] = sn * x + c * y;
        }
      }
      for (int cc = t; cc < ny; cc += JB_T) {
        const double x = sy[sp][cc], y = sy[sq][cc];
        sy[sp][cc] = c * x - sn * y;
        sy[sq][cc] = sn * x + c * y;
      }
      if (t == 0) s_any = 1;
    }
    __syncthreads();
  }
  if (!s_any) return;  // nothing turned: U and Y unchanged
#pragma unroll
  for (int k = 0; k < 8; ++k)
#pragma unroll
    for (int q = 0; q < JB_R; ++q) {
      const int row = t + q * JB_T;
      if (k < nslot && col[k] < n && row < n) U[row + (size_t)col[k] * ldu] = u[k][q];
    }
  for (int e = t; e < nslot * ny; e += JB_T) {
    const int k = e / ny, c = e % ny;
    if (col[k] < n) Y[col[k] + (size_t)c * ldy] = sy[k][c];
  }
  if (t == 0) atomicOr(&rec->jacobi_rotated, 1);
}

// below about a thousand columns the per-pair rounds are cheaper (U sits in L2; measured on the MI355X)
bool jacobi_blocked_fits(int n, int ny) { return n > 1024 && n <= JB_T * JB_R && ny <= JB_YMAX; }

hipError_t launch_jacobi_blk(int n, int round, bool intra, double* U, int ldu, double* Y, int ldy, int ny,
                             DevRec* rec, hipStream_t st) {
  if (!jacobi_blocked_fits(n, ny)) return hipErrorInvalidValue;
  const int nblk = (n + 3) / 4, nbm = (nblk + 1) & ~1;
  if (intra)
    hipLaunchKernelGGL(k_jacobi_blk<true>, dim3(nblk), dim3(JB_T), 0, st, n, nbm, round, U, ldu, Y, ldy, ny, rec);
  else
    hipLaunchKernelGGL(k_jacobi_blk<false>, dim3(nbm / 2), dim3(JB_T), 0, st, n, nbm, round, U, ldu, Y, ldy, ny, rec);
  return hipGetLastError();
}

__global__ void k_clear_rotated(DevRec* rec) { rec->jacobi_rotated = 0; }

hipError_t launch_clear_rotated(DevRec* rec, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_rotated, dim3(1), dim3(1), 0, st, rec);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_colnorms(int n, const double* U, int ldu, double* sigma) {
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double x = U[(size_t)i + (size_t)j * ldu];
    s = fma(x, x, s);
  }
  s = wave_sum(s);
  __shared__ double sh[4];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) sigma[j] = sqrt(sh[0] + sh[1] + sh[2] + sh[3]);
}

__global__ __launch_bounds__(1024) void k_sigma_stats(int n, const double* sigma, DevRec* rec) {
  __shared__ double sm[16];
  __shared__ int sc[16];
  double m = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) m = fmax(m, sigma[j]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  double mx = 0.0;
  for (int q = 0; q < (int)(blockDim.x >> 6); ++q) mx = fmax(mx, sm[q]);
  const double cut = kEps * mx;
  int cnt = 0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) cnt += sigma[j] > cut ? 1 : 0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sc[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) tot += sc[q];
    rec->sigma_max = mx;
    rec->rank = tot;
  }
}

// T[k][c] = (u_k^T b_c) / sigma_k^2 for kept k, else 0 ; one workgroup per k
__global__ __launch_bounds__(256) void k_utb(int n, int nrhs, const double* U, int ldu, const double* B, int ldb,
                                             const double* sigma, const DevRec* rec, double* T) {
  const int k = blockIdx.x;
  const double sk = sigma[k];
  const bool keep = sk > kEps * rec->sigma_max;
  __shared__ double sh[4];
  for (int c = 0; c < nrhs; ++c) {
    double s = 0.0;
    if (keep) {
      if (U) {
        for (int i = threadIdx.x; i < n; i += blockDim.x)
          s = fma(U[(size_t)i + (size_t)k * ldu], B[(size_t)i + (size_t)c * ldb], s);
      } else if (threadIdx.x == 0) {
        s = B[(size_t)k + (size_t)c * ldb];  // identity: the projection is the entry itself
      }
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) T[(size_t)k + (size_t)c * n] = keep ? (sh[0] + sh[1] + sh[2] + sh[3]) / (sk * sk) : 0.0;
    __syncthreads();
  }
}

// X = V T, eight right-hand sides per pass
__global__ __launch_bounds__(256) void k_vt(int n, int nrhs, int c0, const double* V, int ldv, const double* T,
                                            double* X, int ldx, const int* perm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  __shared__ double st[64][8];
  double acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = 0.0;
  const int nc = min(8, nrhs - c0);
  for (int kb = 0; kb < n; kb += 64) {
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 8; e += blockDim.x) {
      const int kk = e / 8, c = e % 8;
      st[kk][c] = (kb + kk < n && c < nc) ? T[(size_t)(kb + kk) + (size_t)(c0 + c) * n] : 0.0;
    }
    __syncthreads();
    if (i < n) {
      const int kn = min(64, n - kb);
      for (int kk = 0; kk < kn; ++kk) {
        const double v = V[(size_t)i + (size_t)(kb + kk) * ldv];
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = fma(v, st[kk][c], acc[c]);
      }
    }
  }
  if (i < n) {
    const int row = perm ? perm[i] : i;
    for (int c = 0; c < nc; ++c) X[(size_t)row + (size_t)(c0 + c) * ldx] = acc[c];
  }
}

hipError_t launch_svd_apply(int n, int nrhs, const double* Ut, int ldu, const double* W, int ldw, const double* C,
                            int ldc, double* X, int ldx, const int* perm, double* sigma, double* T, DevRec* rec,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_colnorms, dim3(n), dim3(256), 0, st, n, Ut, ldu, sigma);
  hipLaunchKernelGGL(k_sigma_stats, dim3(1), dim3(1024), 0, st, n, sigma, rec);
  hipLaunchKernelGGL(k_utb, dim3(n), dim3(256), 0, st, n, nrhs, W, ldw, C, ldc, sigma, rec, T);
  for (int c0 = 0; c0 < nrhs; c0 += 8)
    hipLaunchKernelGGL(k_vt, dim3((n + 255) / 256), dim3(256), 0, st, n, nrhs, c0, Ut, ldu, T, X, ldx, perm);
  return hipGetLastError();
}

// ---- column order by decreasing norm: perm[k] = the column of A that goes to position k (ties to the
// lower index), then Q = A P
__global__ void k_norm_rank(int n, const double* norm, int* perm) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double s = norm[j];
  int r = 0;
  for (int k = 0; k < n; ++k) {
    const double t = norm[k];
    r += (t > s || (t == s && k < j)) ? 1 : 0;
  }
  perm[r] = j;
}

__global__ void k_gather_cols(int n, const double* A, int lda, const int* perm, double* Q, int ldq) {
  const size_t total = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), k = (int)(e / n);
    Q[(size_t)i + (size_t)k * ldq] = A[(size_t)i + (size_t)perm[k] * lda];
  }
}

hipError_t launch_order_columns(int n, const double* A, int lda, double* norm, int* perm, double* Q, int ldq,
                                hipStream_t st) {
  hipLaunchKernelGGL(k_colnorms, dim3(n), dim3(256), 0, st, n, A, lda, norm);
  hipLaunchKernelGGL(k_norm_rank, dim3((n + 255) / 256), dim3(256), 0, st, n, norm, perm);
  size_t total = (size_t)n * n;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_gather_cols, dim3(blocks), dim3(256), 0, st, n, A, lda, perm, Q, ldq);
  return hipGetLastError();
}

// ---- Householder QR (the preconditioner)
// Reflector k: H_k = I - tau_k v v^T with v = (1, v_{k+1..n-1}) stored below the diagonal of column k,
// chosen so that H_k maps Q[k..n-1, k] to (beta, 0, ..., 0); beta = -sign(alpha) ||Q[k..n-1, k]||,
// tau_k = (beta - alpha) / beta, v_i = Q[i, k] / (alpha - beta); tau_k = 0 (H_k = I) when the part
// below the diagonal is zero.
__global__ __launch_bounds__(256) void k_house_gen(int n, int k, double* Q, int ldq, double* tau) {
  double* col = Q + (size_t)k * ldq;
  double s = 0.0;
  for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) s = fma(col[i], col[i], s);
  s = wave_sum(s);
  __shared__ double sh[4];
  __shared__ double s_scale;
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double sig2 = sh[0] + sh[1] + sh[2] + sh[3];
    const double alpha = col[k];
    if (sig2 == 0.0) {
      tau[k] = 0.0;
      s_scale = 1.0;
    } else {
      const double beta = -copysign(sqrt(alpha * alpha + sig2), alpha);
      tau[k] = (beta - alpha) / beta;
      s_scale = 1.0 / (alpha - beta);
      col[k] = beta;
    }
  }
  __syncthreads();
  const double sc = s_scale;
  for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) col[i] *= sc;
}

// apply H_k to columns k+1..n-1 of Q (when with_q) and to the ncol columns of C; one wave per column
__global__ __launch_bounds__(256) void k_house_apply(int n, int k, const double* Q, int ldq, double* Qw, int with_q,
                                                     const double* tau, double* C, int ldc, int ncol) {
  const int lane = threadIdx.x & 63;
  const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int nq = with_q ? n - k - 1 : 0;
  if (col >= nq + ncol) return;
  const double t = tau[k];
  if (t == 0.0) return;
  double* a = col < nq ? Qw + (size_t)(k + 1 + col) * ldq : C + (size_t)(col - nq) * ldc;
  const double* v = Q + (size_t)k * ldq;
  double d = 0.0;
  for (int i = k + 1 + lane; i < n; i += 64) d = fma(v[i], a[i], d);
  d = wave_sum(d) + a[k];
  d *= t;
  if (lane == 0) a[k] -= d;
  for (int i = k + 1 + lane; i < n; i += 64) a[i] = fma(-d, v[i], a[i]);
}

// X = R^T (R: upper triangle of Q), zero above the diagonal
__global__ void k_rt(int n, const double* Q, int ldq, double* X, int ldx) {
  const size_t total = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    X[(size_t)i + (size_t)j * ldx] = i >= j ? Q[(size_t)j + (size_t)i * ldq] : 0.0;
  }
}

hipError_t launch_house_qr(int n, double* Q, int ldq, double* tau, double* C, int ldc, int ncol, hipStream_t st) {
  for (int k = 0; k < n; ++k) {
    hipLaunchKernelGGL(k_house_gen, dim3(1), dim3(256), 0, st, n, k, Q, ldq, tau);
    const int cols = (n - k - 1) + ncol;
    if (cols > 0)
      hipLaunchKernelGGL(k_house_apply, dim3((cols + 3) / 4), dim3(256), 0, st, n, k, Q, ldq, Q, 1, tau, C, ldc,
                         ncol);
  }
  return hipGetLastError();
}

hipError_t launch_house_qt(int n, const double* Q, int ldq, const double* tau, double* C, int ldc, int ncol,
                           hipStream_t st) {
  for (int k = 0; k < n; ++k)
    hipLaunchKernelGGL(k_house_apply, dim3((ncol + 3) / 4), dim3(256), 0, st, n, k, Q, ldq, nullptr, 0, tau, C, ldc,
                       ncol);
  return hipGetLastError();
}

hipError_t launch_rt(int n, const double* Q, int ldq, double* X, int ldx, hipStream_t st) {
  size_t total = (size_t)n * n;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_rt, dim3(blocks), dim3(256), 0, st, n, Q, ldq, X, ldx);
  return hipGetLastError();
}

}  // namespace ada
