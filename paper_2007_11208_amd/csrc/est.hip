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

// One estimator step in two launches. k_est_reduce: every workgroup reduces
// its part of the result (sum |y|, argmax |y| with the lowest index on ties,
// agreement of sign(y) with the previous sign vector) into a partial record;
// the last workgroup to finish (a counter) combines the partials in
// workgroup order and takes the decision. k_est_write: every workgroup writes
// its part of the next right-hand side the decision asks for. `result` holds
// the vector the preceding solve produced; `next_in` receives the next
// right-hand side (may alias `result`: each element is read and written by
// the same thread).
constexpr int EST_WG = 256;   // threads per workgroup
constexpr int EST_MAXG = 256; // workgroups at most

struct EstPart {
  double sum, best;
  int bi, same;
};

__global__ __launch_bounds__(EST_WG) void k_est_reduce(int n, int slot_type, int tag, const double* result,
                                                       const double* xi, DevRec* rec, EstPart* part,
                                                       unsigned* counter) {
  if (rec->est_phase != slot_type) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int G = gridDim.x, g = blockIdx.x;
  const int stage = rec->est_stage;
  // contiguous range of this workgroup, strided by thread inside it (increasing indices per thread)
  const int per = (n + G - 1) / G;
  const int i0 = g * per, i1 = min(n, i0 + per);
  double sum = 0.0, best = -1.0;
  int bi = -1, same = 1;
  for (int i = i0 + t; i < i1; i += EST_WG) {
    const double y = result[i];
    const double a = fabs(y);
    sum += a;
    if (bi < 0 || a > best) { best = a; bi = i; }
    if (stage == 2 && sgn1(y) != xi[i]) same = 0;
  }
  sum = wave_sum(sum);
  wave_argmax(best, bi);
  same = __all(same) ? 1 : 0;
  __shared__ double s_sum[EST_WG / 64], s_best[EST_WG / 64];
  __shared__ int s_bi[EST_WG / 64], s_same[EST_WG / 64];
  __shared__ int s_last;
  if (lane == 0) { s_sum[w] = sum; s_best[w] = best; s_bi[w] = bi; s_same[w] = same; }
  __syncthreads();
  if (t == 0) {
    double tot = 0.0, b = -1.0;
    int ib = -1, sm = 1;
    for (int q = 0; q < EST_WG / 64; ++q) {
      tot += s_sum[q];
      if (s_bi[q] >= 0 && (ib < 0 || s_best[q] > b || (s_best[q] == b && s_bi[q] < ib))) { b = s_best[q]; ib = s_bi[q]; }
      sm &= s_same[q];
    }
    relaxed_store(&part[g].sum, tot);
    relaxed_store(&part[g].best, b);
    relaxed_store(&part[g].bi, ib);
    relaxed_store(&part[g].same, sm);
    wait_stores_done();
    const unsigned old = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (old == (unsigned)(G - 1));
  }
  __syncthreads();
  if (!s_last || t != 0) return;
  // the last workgroup: combine the partials in workgroup order, then decide
  double ysum = 0.0, b = -1.0;
  int jmax = -1, sm = 1;
  for (int q = 0; q < G; ++q) {
    ysum += relaxed_load(&part[q].sum);
    const double bq = relaxed_load(&part[q].best);
    const int iq = relaxed_load(&part[q].bi);
    if (iq >= 0 && (jmax < 0 || bq > b || (bq == b && iq < jmax))) { b = bq; jmax = iq; }
    sm &= relaxed_load(&part[q].same);
  }
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
    if (sm || ysum <= est_old) {
      next = 3;
      rec->est_phase = 1;
      rec->est_stage = 4;
    } else {
      next = 1;
      rec->est_phase = 2;
      rec->est_stage = 3;
    }
  } else if (stage == 3) {
    const double zl = fabs(result[rec->est_j]);  // |z| at the previous index
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
  rec->est_next = next;
  rec->est_next_tag = tag;
}

__global__ __launch_bounds__(EST_WG) void k_est_write(int n, int tag, const double* result, double* next_in,
                                                      double* xi, const DevRec* rec) {
  if (rec->est_next_tag != tag) return;
  const int next = rec->est_next;
  if (next == 0) return;
  const int j = rec->est_j;
  for (int i = blockIdx.x * EST_WG + threadIdx.x; i < n; i += gridDim.x * EST_WG) {
    if (next == 1) {
      const double s = sgn1(result[i]);
      xi[i] = s;
      next_in[i] = s;
    } else if (next == 2) {
      next_in[i] = (i == j) ? 1.0 : 0.0;
    } else {
      next_in[i] = ((i & 1) ? -1.0 : 1.0) * (1.0 + (double)i / (double)(n - 1));
    }
  }
}

size_t est_part_bytes() { return sizeof(EstPart) * EST_MAXG; }

hipError_t launch_est_step(int n, int slot_type, int tag, const double* result, double* next_in, double* xi,
                           DevRec* rec, void* part, unsigned* counter, hipStream_t st) {
  int G = (n + 4 * EST_WG - 1) / (4 * EST_WG);
  G = G < 1 ? 1 : (G > EST_MAXG ? EST_MAXG : G);
  hipLaunchKernelGGL(k_est_reduce, dim3(G), dim3(EST_WG), 0, st, n, slot_type, tag, result, xi, rec,
                     (EstPart*)part, counter);
  int Gw = (n + EST_WG - 1) / EST_WG;
  Gw = Gw > 1024 ? 1024 : Gw;
  hipLaunchKernelGGL(k_est_write, dim3(Gw), dim3(EST_WG), 0, st, n, tag, result, next_in, xi, rec);
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
