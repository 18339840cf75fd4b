// Reciprocal condition number (Section II: every route estimates it; the
// fallback of Section II-E fires when it is below the threshold).
//
// ||inv(A)||_1 is estimated with Hager's method as refined by Higham (ACM TOMS
// 14(4), 1988): x = e/n, y = inv(A) x, xi = sign(y), z = inv(A)^T xi, then up
// to four more rounds of y = inv(A) e_j with j = argmax|z| (lowest index on
// ties), stopping on a repeated sign vector, on no growth, or when the previous
// index still attains max|z|; finally the alternating vector
// x_i = (-1)^i (1 + i/(n-1)) gives the second bound 2||inv(A) x||_1/(3n).
//
// The control flow runs on the device: the host enqueues the longest possible
// sequence (inv(A), inv(A)^T alternating, eleven solves) once; each solve
// kernel and each k_est_step is predicated on est_phase, so steps the
// algorithm does not take cost only an empty launch and no host round trip.
#include "ada_internal.h"

namespace ada {

__global__ void k_est_init(int n, double* v, DevRec* rec) {
  const bool live = rec->stop == 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) v[i] = 1.0 / n;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    rec->est_phase = live ? 1 : 0;
    rec->est_stage = 0;
    rec->est_nsolves = 0;
    rec->est = 0.0;
  }
}

hipError_t launch_est_init(int n, double* v, DevRec* rec, hipStream_t st) {
  int blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_est_init, dim3(blocks), dim3(256), 0, st, n, v, rec);
  return hipGetLastError();
}

__device__ __forceinline__ double sgn1(double v) { return v >= 0.0 ? 1.0 : -1.0; }

// One workgroup. `result` holds the vector the preceding solve produced,
// `next_in` receives the next right-hand side (may alias `result`).
__global__ __launch_bounds__(1024) void k_est_step(int n, int slot_type, const double* result, double* next_in,
                                                   double* xi, DevRec* rec) {
  if (rec->est_phase != slot_type) return;
  const int t = threadIdx.x;
  const int nw = blockDim.x >> 6;
  __shared__ double s_d[16];
  __shared__ int s_i[16];
  __shared__ double s_sum, s_zl;
  __shared__ int s_same, s_j;
  const int stage = rec->est_stage;

  // reductions over the result: sum|y|, argmax|y| (lowest index on ties), sign agreement with xi
  double sum = 0.0;
  double best = -1.0;
  int bi = -1;
  int same = 1;
  for (int i = t; i < n; i += blockDim.x) {
    const double y = result[i];
    sum += fabs(y);
    const double a = fabs(y);
    if (bi < 0 || a > best) { best = a; bi = i; }
    if (stage == 2 && sgn1(y) != xi[i]) same = 0;
  }
  // (a strided loop visits indices in increasing order per thread, so the per-thread
  // argmax already holds the lowest index among its ties)
  sum = wave_sum(sum);
  wave_argmax(best, bi);
  same = __all(same) ? 1 : 0;
  const int lane = t & 63, w = t >> 6;
  __shared__ int s_same_w[16];
  if (lane == 0) { s_d[w] = best; s_i[w] = bi; s_same_w[w] = same; }
  __shared__ double s_sum_w[16];
  if (lane == 0) s_sum_w[w] = sum;
  __syncthreads();
  if (t == 0) {
    double tot = 0.0, b = -1.0;
    int ib = -1, sm = 1;
    for (int q = 0; q < nw; ++q) {
      tot += s_sum_w[q];
      const int i2 = s_i[q];
      const double v2 = s_d[q];
      if (i2 >= 0 && (ib < 0 || v2 > b || (v2 == b && i2 < ib))) { b = v2; ib = i2; }
      sm &= s_same_w[q];
    }
    s_sum = tot;
    s_j = ib;
    s_same = sm;
    s_zl = (stage == 3) ? fabs(result[rec->est_j]) : 0.0;
  }
  __syncthreads();
  const double ysum = s_sum;
  const int jmax = s_j;
  // decide (thread 0), then write the next right-hand side (all threads)
  __shared__ int s_next;  // 0 done, 1 sign vector, 2 unit vector e_j, 3 alternating vector
  if (t == 0) {
    rec->est_nsolves += 1;
    int next = 0;
    if (stage == 0) {
      if (n == 1) {
        rec->est = fabs(result[0]);
        next = 0;
      } else {
        rec->est = ysum;
        next = 1;
        rec->est_phase = 2;
        rec->est_stage = 1;
      }
    } else if (stage == 1) {
      rec->est_j = jmax;
      rec->est_iter = 2;
      next = 2;
      rec->est_phase = 1;
      rec->est_stage = 2;
    } else if (stage == 2) {
      const double est_old = rec->est;
      rec->est = ysum;
      if (s_same || ysum <= est_old) {
        next = 3;
        rec->est_phase = 1;
        rec->est_stage = 4;
      } else {
        next = 1;
        rec->est_phase = 2;
        rec->est_stage = 3;
      }
    } else if (stage == 3) {
      const double zl = s_zl;             // |z| at the previous index
      const double zmax = fabs(result[jmax]);
      if (zl != zmax && rec->est_iter < 5) {
        rec->est_iter += 1;
        rec->est_j = jmax;
        next = 2;
        rec->est_phase = 1;
        rec->est_stage = 2;
      } else {
        next = 3;
        rec->est_phase = 1;
        rec->est_stage = 4;
      }
    } else {
      const double temp = 2.0 * (ysum / (3.0 * n));
      if (temp > rec->est) rec->est = temp;
      next = 0;
    }
    if (next == 0) rec->est_phase = 0;
    s_next = next;
  }
  __syncthreads();
  const int next = s_next;
  if (next == 1) {
    for (int i = t; i < n; i += blockDim.x) {
      const double s = sgn1(result[i]);
      xi[i] = s;
    }
    __syncthreads();
    for (int i = t; i < n; i += blockDim.x) next_in[i] = xi[i];
  } else if (next == 2) {
    const int j = rec->est_j;
    __syncthreads();
    for (int i = t; i < n; i += blockDim.x) next_in[i] = (i == j) ? 1.0 : 0.0;
  } else if (next == 3) {
    __syncthreads();
    for (int i = t; i < n; i += blockDim.x)
      next_in[i] = ((i & 1) ? -1.0 : 1.0) * (1.0 + (double)i / (double)(n - 1));
  }
}

hipError_t launch_est_step(int n, int slot_type, const double* result, double* next_in, double* xi, DevRec* rec,
                           hipStream_t st) {
  hipLaunchKernelGGL(k_est_step, dim3(1), dim3(1024), 0, st, n, slot_type, result, next_in, xi, rec);
  return hipGetLastError();
}

// rcond = (1/est)/||A||_1 as the condition routines of the paper's LAPACK mapping form it;
// 0 when ||A||_1 or est is 0; NaN propagates.
__global__ void k_finalize_rcond(DevRec* rec) {
  if (rec->stop) return;
  const double anorm = rec->anorm1, est = rec->est;
  double r;
  if (anorm == 0.0) r = 0.0;
  else if (est != est) r = est;
  else if (est == 0.0) r = 0.0;
  else r = (1.0 / est) / anorm;
  rec->rcond = r;
}

hipError_t launch_finalize_rcond(DevRec* rec, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize_rcond, dim3(1), dim3(1), 0, st, rec);
  return hipGetLastError();
}

}  // namespace ada
