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

// Several right-hand sides (2..64). The tiles of earlier blocks stream through two LDS buffers (the next
// tile's loads are in flight while the current one is applied to all columns); the diagonal block is solved
// by the four waves, each taking every fourth column, lane = row, the lane's row of the diagonal tile scaled
// by the reciprocal of its diagonal entry in registers, the solved values broadcast by readlane; a wave runs
// two of its columns at a time, interleaved step by step, so their broadcasts overlap.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void k_trsm_dec(
    int n, int nrhs, const double* __restrict__ T, int ldt, int lower,
                                                  int trans, int unit, double* X, int ldx, int* flags, int epoch,
                                                  unsigned* ticket, DevRec* rec, const int* pred, int pred_val) {
  if (pred && *pred != pred_val) return;
  constexpr int LD = TB + 1;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int nblk = (n + TB - 1) / TB;
  __shared__ int s_tk;
  if (t == 0) s_tk = (int)atomicAdd(ticket, 1u);
  __syncthreads();
  const int tk = s_tk;
  if (tk >= nblk) return;
  const bool eff_lower = (lower != 0) != (trans != 0);
  auto blk = [&](int q) { return eff_lower ? q : (nblk - 1 - q); };
  const int bi = blk(tk);
  const int r0 = bi * TB;
  const int rows = min(TB, n - r0);

  extern __shared__ double sm[];
  double* acc = sm;                  // acc[c * TB + r]
  double* xj = acc + TB * nrhs;      // xj[c * TB + k]
  double* tb0 = xj + TB * nrhs;      // tb[k * LD + r] = op(T)(r0 + r, c0 + k)
  double* tb1 = tb0 + TB * LD;

  for (int e = t; e < TB * nrhs; e += blockDim.x) {
    const int r = e % TB, c = e / TB;
    acc[e] = (r < rows) ? X[(size_t)(r0 + r) + (size_t)c * ldx] : 0.0;
  }
  // thread t stages 16 elements of a 64x64 tile (coalesced in memory)
  double st[16];
  auto load_tile = [&](int c0, int cols) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = t + 256 * u;
      const int a = e % TB, b = e / TB;  // a runs along memory
      const int r = trans ? b : a, k = trans ? a : b;
      st[u] = (r < rows && k < cols) ? (trans ? T[(size_t)(c0 + k) + (size_t)(r0 + r) * ldt]
                                               : T[(size_t)(r0 + r) + (size_t)(c0 + k) * ldt])
                                     : 0.0;
    }
  };
  auto store_tile = [&](double* dst) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = t + 256 * u;
      const int a = e % TB, b = e / TB;
      const int r = trans ? b : a, k = trans ? a : b;
      dst[k * LD + r] = st[u];
    }
  };
  if (tk > 0) {
    const int c0 = blk(0) * TB;
    load_tile(c0, min(TB, n - c0));
    store_tile(tb0);
  }
  __syncthreads();
  for (int q = 0; q < tk; ++q) {
    double* cur = (q & 1) ? tb1 : tb0;
    double* nxt = (q & 1) ? tb0 : tb1;
    if (q + 1 < tk) {
      const int c1 = blk(q + 1) * TB;
      load_tile(c1, min(TB, n - c1));
    }
    const int bj = blk(q), c0 = bj * TB, cols = min(TB, n - c0);
    if (t == 0) {
      long spins = 0;
      while (relaxed_load(&flags[bj]) != epoch) {
        if (++spins > kSpinLimit) {
          atomicOr(&rec->timeout, 1);
          break;
        }
        __builtin_amdgcn_s_sleep(0);
      }
    }
    __syncthreads();
    for (int e = t; e < TB * nrhs; e += blockDim.x) {
      const int k = e % TB, c = e / TB;
      xj[e] = (k < cols) ? relaxed_load(X + (size_t)(c0 + k) + (size_t)c * ldx) : 0.0;
    }
    __syncthreads();
    for (int c = w; c < nrhs; c += 4) {
      double sacc = 0.0;
      const double* xc = xj + c * TB;
#pragma unroll 16
      for (int k = 0; k < TB; ++k) sacc = fma(cur[k * LD + lane], xc[k], sacc);
      acc[c * TB + lane] -= sacc;
    }
    if (q + 1 < tk) store_tile(nxt);
    __syncthreads();
  }

  // diagonal block
  double* td = (tk & 1) ? tb1 : tb0;
  load_tile(r0, rows);
  store_tile(td);
  __syncthreads();
  {
    // the row scaled by the reciprocal of its diagonal entry (as in k_trsv1): a step is a readlane and
    // an FMA per column
    const double rd = (lane < rows && !unit) ? 1.0 / td[lane * LD + lane] : 1.0;
    double trow[TB];
#pragma unroll
    for (int i = 0; i < TB; ++i) trow[i] = td[i * LD + lane] * rd;
    // the wave's columns c = w, w + 4, ..., two per pass (their steps interleave)
    for (int c = w; c < nrhs; c += 8) {
      const bool two = c + 4 < nrhs;  // wave-uniform
      double a0 = acc[c * TB + lane] * rd;
      double a1 = two ? acc[(c + 4) * TB + lane] * rd : 0.0;
      if (eff_lower) {
#pragma unroll
        for (int i = 0; i < TB; ++i) {
          const double x0 = read_lane(a0, i);
          const double x1 = read_lane(a1, i);
          a0 = (lane > i) ? fma(-trow[i], x0, a0) : a0;
          a1 = (lane > i) ? fma(-trow[i], x1, a1) : a1;
        }
      } else {
#pragma unroll
        for (int i = TB - 1; i >= 0; --i) {
          const double x0 = read_lane(a0, i);
          const double x1 = read_lane(a1, i);
          a0 = (lane < i) ? fma(-trow[i], x0, a0) : a0;
          a1 = (lane < i) ? fma(-trow[i], x1, a1) : a1;
        }
      }
      if (lane < rows) {
        relaxed_store(X + (size_t)(r0 + lane) + (size_t)c * ldx, a0);
        if (two) relaxed_store(X + (size_t)(r0 + lane) + (size_t)(c + 4) * ldx, a1);
      }
    }
  }
  wait_stores_done();
  __syncthreads();
  if (t == 0) relaxed_store(&flags[bi], epoch);
}

// One right-hand side (the routed 1-RHS solves and every solve of the
// condition estimate). The same decoupled scheme with the critical path cut
// down: the tiles of earlier blocks are streamed through two LDS buffers
// (the next tile's loads are in flight while the current one is used); the
// tile next to the diagonal and the diagonal tile itself are staged, and the
// reciprocals of the diagonal formed, before the wait for the block that
// precedes this one, so that after the wait only that block's x (64 values),
// one 64x64 product and the substitution remain. The substitution runs in one
// wave with lane = row, the row of the diagonal tile in registers and the
// solved value broadcast by readlane, fully unrolled. The solved
// block and its flag are handed over with agent-scope relaxed accesses (the
// flag is stored once the block's stores are complete), so no cache
// write-back or invalidation sits on the chain.
__global__ __launch_bounds__(256) void k_trsv1(int n, const double* __restrict__ T, int ldt, int lower, int trans,
                                               int unit, double* x, int* flags, int epoch, unsigned* ticket,
                                               DevRec* rec, const int* pred, int pred_val) {
  if (pred && *pred != pred_val) return;
  constexpr int LD = TB + 1;
  const int t = threadIdx.x, lane = t & 63, cq = t >> 6;
  const int nblk = (n + TB - 1) / TB;
  __shared__ int s_tk;
  if (t == 0) s_tk = (int)atomicAdd(ticket, 1u);
  __syncthreads();
  const int tk = s_tk;
  if (tk >= nblk) return;
  const bool eff_lower = (lower != 0) != (trans != 0);
  auto blk = [&](int q) { return eff_lower ? q : (nblk - 1 - q); };
  const int bi = blk(tk);
  const int r0 = bi * TB;
  const int rows = min(TB, n - r0);

  extern __shared__ double sm[];
  double* tb0 = sm;             // [64][65]: tb[k * LD + r] = op(T)(r0 + r, c0 + k)
  double* tb1 = tb0 + TB * LD;
  double* td = tb1 + TB * LD;   // diagonal tile
  double* sx = td + TB * LD;    // x of the block being applied
  double* sacc = sx + TB;       // [4][64] partial sums

  // thread t stages 16 elements of a 64x64 tile: k = t / 4 * ... (coalesced in memory)
  double st[16];
  auto load_tile = [&](int c0, int cols) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = t + 256 * u;
      const int a = e % TB, b = e / TB;  // a runs along memory
      const int r = trans ? b : a, k = trans ? a : b;
      st[u] = (r < rows && k < cols) ? (trans ? T[(size_t)(c0 + k) + (size_t)(r0 + r) * ldt]
                                               : T[(size_t)(r0 + r) + (size_t)(c0 + k) * ldt])
                                     : 0.0;
    }
  };
  auto store_tile = [&](double* dst) {
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int e = t + 256 * u;
      const int a = e % TB, b = e / TB;
      const int r = trans ? b : a, k = trans ? a : b;
      dst[k * LD + r] = st[u];
    }
  };
  auto wait_flag = [&](int b) {
    if (t == 0) {
      long spins = 0;
      while (relaxed_load(&flags[b]) != epoch) {
        if (++spins > kSpinLimit) {
          atomicOr(&rec->timeout, 1);
          break;
        }
        __builtin_amdgcn_s_sleep(0);
      }
    }
    __syncthreads();
  };

  const double bval = (cq == 0 && lane < rows) ? x[r0 + lane] : 0.0;
  double acc = 0.0;
  const int nfar = tk > 0 ? tk - 1 : 0;
  if (nfar > 0) {
    const int c0 = blk(0) * TB;
    load_tile(c0, min(TB, n - c0));
    store_tile(tb0);
  }
  __syncthreads();
  for (int q = 0; q < nfar; ++q) {
    double* cur = (q & 1) ? tb1 : tb0;
    double* nxt = (q & 1) ? tb0 : tb1;
    if (q + 1 < nfar) {
      const int c1 = blk(q + 1) * TB;
      load_tile(c1, min(TB, n - c1));
    }
    const int bj = blk(q), c0 = bj * TB, cols = min(TB, n - c0);
    wait_flag(bj);
    if (t < TB) sx[t] = t < cols ? relaxed_load(x + c0 + t) : 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc = fma(cur[(16 * cq + k) * LD + lane], sx[16 * cq + k], acc);
    if (q + 1 < nfar) store_tile(nxt);
    __syncthreads();
  }
  // the tile next to the diagonal and the diagonal tile, before the wait
  double* near = (nfar & 1) ? tb1 : tb0;
  int bn = -1, cn = 0, coln = 0;
  if (tk > 0) {
    bn = blk(tk - 1);
    cn = bn * TB;
    coln = min(TB, n - cn);
    load_tile(cn, coln);
    store_tile(near);
  }
  load_tile(r0, rows);
  store_tile(td);
  __syncthreads();
  // before the wait: the near tile's 16 values of this thread, and for wave 0 its row of the diagonal
  // tile and the reciprocal of its diagonal entry, all in registers
  double nr[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) nr[k] = (tk > 0) ? near[(16 * cq + k) * LD + lane] : 0.0;
  // The row is scaled by the reciprocal of its diagonal entry here, so that the substitution's dependent
  // chain is a readlane and an FMA per step (no multiply by the reciprocal on it).
  double trow[TB];
  double rd = 1.0;
  if (cq == 0) {
    rd = (lane < rows && !unit) ? 1.0 / td[lane * LD + lane] : 1.0;
#pragma unroll
    for (int i = 0; i < TB; ++i) trow[i] = td[i * LD + lane] * rd;
  }
  if (tk > 0) {
    wait_flag(bn);
    if (t < TB) sx[t] = t < coln ? relaxed_load(x + cn + t) : 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc = fma(nr[k], sx[16 * cq + k], acc);
  }
  sacc[cq * TB + lane] = acc;
  __syncthreads();
  if (cq == 0) {
    // substitution, lane = row; padded rows (past `rows`) hold zeros and stay zero
    // a = (b - sum) / T(lane, lane); lane i holds x_i once the steps before i have been applied
    double a = (bval - ((sacc[lane] + sacc[TB + lane]) + (sacc[2 * TB + lane] + sacc[3 * TB + lane]))) * rd;
    if (eff_lower) {
#pragma unroll
      for (int i = 0; i < TB; ++i) {
        const double xi = read_lane(a, i);
        a = (lane > i) ? fma(-trow[i], xi, a) : a;
      }
    } else {
#pragma unroll
      for (int i = TB - 1; i >= 0; --i) {
        const double xi = read_lane(a, i);
        a = (lane < i) ? fma(-trow[i], xi, a) : a;
      }
    }
    if (lane < rows) relaxed_store(x + r0 + lane, a);
    wait_stores_done();
    // wave 0 wrote the block: its lane 0 raises the flag once the stores are complete
    if (lane == 0) relaxed_store(&flags[bi], epoch);
  }
}

hipError_t launch_trsm_dec(int n, int nrhs, const double* T, int ldt, bool lower, bool trans, bool unit, double* X,
                           int ldx, int* flags, int epoch, unsigned* ticket, DevRec* rec, const int* pred,
                           int pred_val, hipStream_t st) {
  if (nrhs < 1 || nrhs > 64) return hipErrorInvalidValue;
  const int nblk = (n + TB - 1) / TB;
  if (nrhs == 1) {
    const size_t lds1 = sizeof(double) * ((size_t)3 * TB * (TB + 1) + (size_t)5 * TB);
    static size_t done1 = 0;
    hipError_t e1 = ensure_lds((const void*)k_trsv1, lds1, done1);
    if (e1 != hipSuccess) return e1;
    hipLaunchKernelGGL(k_trsv1, dim3(nblk), dim3(256), lds1, st, n, T, ldt, (int)lower, (int)trans, (int)unit, X,
                       flags, epoch, ticket, rec, pred, pred_val);
    return hipGetLastError();
  }
  const size_t lds = sizeof(double) * ((size_t)TB * nrhs * 2 + (size_t)2 * TB * (TB + 1));
  static size_t done = 0;
  hipError_t e = ensure_lds((const void*)k_trsm_dec, lds, done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_trsm_dec, dim3(nblk), dim3(256), lds, st, n, nrhs, T, ldt, (int)lower, (int)trans,
                     (int)unit, X, ldx, flags, epoch, ticket, rec, pred, pred_val);
  return hipGetLastError();
}

}  // namespace ada
