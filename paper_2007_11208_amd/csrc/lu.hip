// LU with partial pivoting (Section II-D), right-looking and blocked by 128
// columns. Per block column k0:
//   k_getrf_panel    factor the m x nb panel W[k0:n, k0:k0+nb] with partial
//                    pivoting (ties to the lowest row), rows spread over P
//                    workgroups that keep the panel in registers;
//   k_laswp_moves    apply the panel's row interchanges to every other column
//                    (and to the permutation vector used by the solves);
//   k_trsm_lines     U12 = L11^{-1} A12 (unit lower; trsm_lines.hip);
//   k_gemm_sub       A22 -= L21 U12 on the matrix cores (gemm.hip).
//
// The panel needs one cross-workgroup exchange per column (the pivot search
// spans all m rows): every workgroup publishes its best candidate and that
// candidate's row, then all of them meet at a counter; every workgroup then
// picks the same winner (largest modulus, lowest row on ties) and applies the
// swap and the rank-1 update to the rows it holds. All waits are bounded.
#include "ada_internal.h"

#include <climits>

namespace ada {

constexpr int PNB = 128;    // panel width
constexpr int PROWS = 256;  // panel rows per workgroup = threads per workgroup (one row per thread)

__device__ void grid_wait(unsigned* counter, unsigned target, DevRec* rec) {
  long spins = 0;
  while (agent_load(counter) < target) {
    if (++spins > kSpinLimit) {
      atomicOr(&rec->timeout, 1);
      break;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Each panel row is held in registers by four threads (32 columns each). The
// part that holds the current column rotates its registers left
// by one after every column step, so the current column is always its d[0] and
// every register index is a constant. Row interchanges are not moved through
// memory: each row carries its current position `pos`; the pivot row takes
// position s and the row that sat at s takes the pivot's old position, exactly
// as an explicit interchange would. Rows are written to their final positions
// at the end and the list of moved rows is handed to k_laswp_moves.
constexpr int HC = 32;                 // columns per thread
constexpr int PTH = (PNB / HC) * PROWS;  // 1024 threads: part h = t / PROWS holds columns HC*h .. HC*h+HC-1
__global__ __launch_bounds__(PTH) void k_getrf_panel(int n, int k0, int nbw, double* __restrict__ W, int ldw,
                                                     int* __restrict__ ipiv, DevRec* rec, unsigned* counter,
                                                     PanelScratch ps) {
  if (rec->stop) return;
  const int m = n - k0;
  const int P = gridDim.x;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int h = t / PROWS, r = t % PROWS;
  const int wg = blockIdx.x;
  const int prow = wg * PROWS + r;
  const bool rvalid = prow < m;
  int pos = rvalid ? prow : INT_MAX;

  __shared__ double s_u[PNB];
  __shared__ double s_l[PROWS];
  __shared__ double s_cv[4];
  __shared__ int s_cp[4];
  __shared__ int s_bp, s_win_pos, s_win_wg;
  __shared__ double s_bv;
  extern __shared__ double s_rows[];  // P x PNB candidate rows (P > 1)

  if (wg == 0 && t == 0) __hip_atomic_store(ps.moves, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

  double d[HC];
  {
    // column pointers are uniform per wave, the row offset is per thread: one register per address
    const int row = k0 + min(prow, m - 1);
#pragma unroll
    for (int c = 0; c < HC; ++c) {
      const double* colp = W + (size_t)(k0 + min(HC * h + c, nbw - 1)) * ldw;
      d[c] = colp[row];
    }
#pragma unroll
    for (int c = 0; c < HC; ++c)
      if (!rvalid || HC * h + c >= nbw) d[c] = 0.0;
  }

  for (int s = 0; s < nbw; ++s) {
    const int par = s & 1;
    const int hc = s / HC;          // half holding column s (its d[0])
    const int sl = s % HC;          // rotations that half has done so far
    const bool cur = (h == hc);
    // 1. this workgroup's candidate: largest |A(row, s)| over rows at positions >= s, lowest position on ties
    if (cur) {
      double v = -1.0;
      int key = -1;
      if (rvalid && pos >= s) {
        v = fabs(d[0]);
        key = pos;
      }
      wave_argmax(v, key);
      if (lane == 0) { s_cv[w - 4 * hc] = v; s_cp[w - 4 * hc] = key; }
    }
    __syncthreads();
    if (t == 0) {
      double bv = s_cv[0];
      int bp = s_cp[0];
      for (int q = 1; q < 4; ++q) {
        const int k2 = s_cp[q];
        const double v2 = s_cv[q];
        if (k2 >= 0 && (bp < 0 || v2 > bv || (v2 == bv && k2 < bp))) { bv = v2; bp = k2; }
      }
      s_bv = bv;
      s_bp = bp;
    }
    __syncthreads();
    const int bp = s_bp;
    if (P == 1) {
      if (rvalid && pos == bp) {
#pragma unroll
        for (int c = 0; c < HC; ++c) s_u[HC * h + c] = d[c];
      }
      if (t == 0) s_win_pos = bp;
      __syncthreads();
    } else {
      // 2. publish (value, position) and the candidate row, then meet at the counter
      double* myslot = ps.slot_rows + ((size_t)par * 64 + wg) * PNB;
      if (rvalid && pos == bp) {
#pragma unroll
        for (int c = 0; c < HC; ++c) relaxed_store(myslot + HC * h + c, d[c]);
        __threadfence();
      }
      if (t == 0) {
        relaxed_store(ps.slot_val + par * 64 + wg, s_bv);
        __hip_atomic_store(ps.slot_row + par * 64 + wg, bp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
      if (t == 0) {
        __threadfence();
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        grid_wait(counter, (unsigned)(s + 1) * (unsigned)P, rec);
      }
      __syncthreads();
      // 3. read every candidate (value, position, row) in one round trip; all workgroups pick the same winner
      for (int e = t; e < P * PNB; e += PTH) s_rows[e] = relaxed_load(ps.slot_rows + (size_t)par * 64 * PNB + e);
      if (t < 64) {
        double cv = -1.0;
        int ck = -1, cw = t;
        if (t < P) {
          cv = relaxed_load(ps.slot_val + par * 64 + t);
          ck = __hip_atomic_load(ps.slot_row + par * 64 + t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const double v2 = __shfl_xor(cv, o, 64);
          const int k2 = __shfl_xor(ck, o, 64);
          const int w2 = __shfl_xor(cw, o, 64);
          if (k2 >= 0 && (ck < 0 || v2 > cv || (v2 == cv && k2 < ck))) { cv = v2; ck = k2; cw = w2; }
        }
        if (t == 0) { s_win_pos = ck; s_win_wg = cw; }
      }
      __syncthreads();
      if (t < PNB) s_u[t] = s_rows[s_win_wg * PNB + t];
      __syncthreads();
    }
    const int p = s_win_pos;
    if (wg == 0 && t == 0) ipiv[k0 + s] = k0 + p;
    // 4. the interchange of positions s and p (bookkeeping only)
    const bool is_win = rvalid && pos == p;
    if (rvalid && pos == s && !is_win) pos = p;
    if (is_win) pos = s;
    // s_u holds the pivot row in the frames of the two halves: half hc rotated by sl, the others not
    const double piv = s_u[HC * hc];
    if (piv == 0.0 && wg == 0 && t == 0) atomicMin(&rec->info, k0 + s + 1);  // exact zero pivot: failure
    // 5. multiplier (current part) and rank-1 update of this row; straight-line selects keep d[] in place
    const bool active = piv != 0.0 && rvalid && pos > s;
    double l = 0.0;
    if (cur) {
      l = active ? d[0] / piv : 0.0;
      d[0] = active ? l : d[0];
      s_l[r] = l;
    }
    __syncthreads();
    l = s_l[r];
    {
      // current part: columns s+1.. sit in d[1 .. live-1]; later parts: every column below nbw
      const int live = cur ? min(HC - sl, nbw - s) : (nbw - HC * h);
      const int first = cur ? 1 : 0;
      const bool upd = active && h >= hc;
#pragma unroll
      for (int c = 0; c < HC; ++c) {
        const double nv = fma(-l, s_u[HC * h + c], d[c]);
        d[c] = (upd && c >= first && c < live) ? nv : d[c];
      }
    }
    // 6. rotate the current part: the finished column moves to the back
    {
      const double f = d[0];
#pragma unroll
      for (int c = 0; c < HC - 1; ++c) d[c] = cur ? d[c + 1] : d[c];
      d[HC - 1] = cur ? f : d[HC - 1];
    }
    __syncthreads();
  }
  // half h was rotated rot times (HC rotations restore the order): d[c] holds column HC*h + (c + rot) % HC
  if (rvalid) {
    const int rot = max(0, min(HC, nbw - HC * h)) % HC;
    const int row = k0 + pos;
#pragma unroll
    for (int c = 0; c < HC; ++c) {
      const int col = HC * h + (c + rot) % HC;
      if (col < nbw) W[(size_t)(k0 + col) * ldw + row] = d[c];
    }
    if (h == 0 && pos != prow) {
      const int idx = atomicAdd(ps.moves, 1);
      ps.moves[1 + 2 * idx] = k0 + pos;   // destination row
      ps.moves[2 + 2 * idx] = k0 + prow;  // source row
    }
  }
}

hipError_t launch_getrf_panel(int n, int k0, int nbw, double* W, int ldw, int* ipiv, DevRec* rec,
                              unsigned* counter, PanelScratch ps, hipStream_t st) {
  const int m = n - k0;
  const int P = (m + PROWS - 1) / PROWS;
  if (P > 64) return hipErrorInvalidValue;  // n - k0 <= 16384 per panel
  const size_t lds = P > 1 ? (size_t)P * PNB * sizeof(double) : 0;
  hipLaunchKernelGGL(k_getrf_panel, dim3(P), dim3(PTH), lds, st, n, k0, nbw, W, ldw, ipiv, rec, counter, ps);
  return hipGetLastError();
}

// Apply the panel's row moves to all columns outside the panel (32 per
// workgroup) and, in workgroup 0, to the permutation vector.
__global__ __launch_bounds__(256) void k_laswp_moves(int n, int k0, int nbw, double* __restrict__ W, int ldw,
                                                     const int* __restrict__ moves, int* __restrict__ perm,
                                                     DevRec* rec) {
  if (rec->stop) return;
  if (rec->info != INT_MAX) {
    // the panel met an exact zero pivot: the routed solve has failed; later kernels skip
    if (blockIdx.x == 0 && threadIdx.x == 0) rec->stop = 1;
    return;
  }
  const int cnt = moves[0];
  if (cnt == 0) return;
  __shared__ double sv[2 * PNB][33];
  __shared__ int sp[2 * PNB];
  const int t = threadIdx.x;
  const int outside = n - nbw;
  const int c0 = blockIdx.x * 32;
  if (c0 < outside) {
    for (int mi = t; mi < cnt; mi += blockDim.x) {
      const int src = moves[2 + 2 * mi];
      for (int c = 0; c < 32; ++c) {
        const int oc = c0 + c;
        if (oc >= outside) break;
        const int col = oc < k0 ? oc : oc + nbw;
        sv[mi][c] = W[(size_t)src + (size_t)col * ldw];
      }
    }
  }
  if (blockIdx.x == 0)
    for (int mi = t; mi < cnt; mi += blockDim.x) sp[mi] = perm[moves[2 + 2 * mi]];
  __syncthreads();
  if (c0 < outside) {
    for (int mi = t; mi < cnt; mi += blockDim.x) {
      const int dst = moves[1 + 2 * mi];
      for (int c = 0; c < 32; ++c) {
        const int oc = c0 + c;
        if (oc >= outside) break;
        const int col = oc < k0 ? oc : oc + nbw;
        W[(size_t)dst + (size_t)col * ldw] = sv[mi][c];
      }
    }
  }
  if (blockIdx.x == 0)
    for (int mi = t; mi < cnt; mi += blockDim.x) perm[moves[1 + 2 * mi]] = sp[mi];
}

hipError_t launch_laswp_moves(int n, int k0, int nbw, double* W, int ldw, const int* moves, int* perm,
                              DevRec* rec, hipStream_t st) {
  const int outside = n - nbw;
  int grid = (outside + 31) / 32;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_laswp_moves, dim3(grid), dim3(256), 0, st, n, k0, nbw, W, ldw, moves, perm, rec);
  return hipGetLastError();
}

// U12 = L11^{-1} A12 with L11 the unit lower nbw x nbw block at W(k0,k0) and
}  // namespace ada
