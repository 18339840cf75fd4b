// LU with partial pivoting (Section II-D), right-looking and blocked by 128
// columns. Per block column k0:
//   k_getrf_panel    factor the m x nb panel W[k0:n, k0:k0+nb] with partial
//                    pivoting (ties to the lowest row), rows spread over P
//                    workgroups that keep the panel in registers;
//   k_trsm_cols      the next block column: the panel's row interchanges, then
//                    U12 = L11^{-1} A12 (unit lower; trsm_lines.hip);
//   k_gemm_sub       its A22 -= L21 U12 on the matrix cores (gemm.hip);
//   and on a second stream, beside the next panel: k_laswp_moves (the
//   interchanges of every other column, and of columns left of the panel),
//   k_trsm_cols and k_gemm_sub for the rest of the trailing matrix.
//
// The panel needs one cross-workgroup exchange per column (the pivot search
// spans all m rows): every workgroup publishes its best candidate and that
// candidate's row, then a record of it (below); every workgroup then picks
// the same winner (largest modulus, lowest row on ties) and applies the swap
// and the rank-1 update to the rows it holds. All waits are bounded.
#include "ada_internal.h"

#include <climits>

namespace ada {

constexpr int PNB = 128;    // panel width
constexpr int PROWS = 256;  // panel rows per workgroup = threads per workgroup (one row per thread)


// Each panel row is held in registers by four threads, one per column
// quarter (quarter h = waves 4h .. 4h+3, 32 columns each, d[c] = column
// 32h + c), so whatever depends on the current column's quarter is uniform
// across a wave: the current column is picked out of the registers by a
// uniform branch on its index and the update of a quarter starts at its first
// live column by a uniform jump into straight-line code. Row interchanges are
// not moved through memory: each row carries its current position `pos`; the
// pivot row takes position s and the row that sat at s takes the pivot's old
// position, exactly as an explicit interchange would. Rows are written to
// their final positions at the end and the list of moved rows is handed to
// k_laswp_moves.
//
// With several workgroups, every column needs one exchange: each workgroup
// publishes its best candidate's row and, once those stores have completed, a
// 16-byte record: word 0 = the bits of the candidate's modulus with a toggle in
// bit 63 (the sign bit of a non-negative double is free), word 1 = its position
// and the column's epoch. Each word is written and read as one 64-bit
// agent-scope atomic, so a reader that sees the current epoch in word 1 and the
// current toggle in word 0 has the current candidate: the toggle flips between
// successive uses of a record, and a reader has already seen the previous use
// (or the reset state, whose toggle is the opposite of the first use's), so
// word 0 cannot be older than that. Wave 0 of every workgroup polls all the
// records at once (one lane per workgroup, no read-modify-write on a shared
// counter), picks the winner (largest modulus, lowest position on ties) and
// stages the winner's row, complete before its record was written, in LDS.
// The hand-off uses agent-scope relaxed accesses and a wait for store
// completion (no cache write-back or invalidation). All waits are bounded;
// once one gives up (rec->timeout) the others stop waiting too.
constexpr int HC = 32;                   // columns per thread
constexpr int PTH = (PNB / HC) * PROWS;  // 1024 threads

// d[i] for a wave-uniform i (a branch tree, no register indexing)
__device__ __forceinline__ double get_col(const double (&d)[HC], int i) {
  double v = 0.0;
  switch (i) {
#define ADA_CASE(K) case K: v = d[K]; break;
    ADA_CASE(0) ADA_CASE(1) ADA_CASE(2) ADA_CASE(3) ADA_CASE(4) ADA_CASE(5) ADA_CASE(6) ADA_CASE(7)
    ADA_CASE(8) ADA_CASE(9) ADA_CASE(10) ADA_CASE(11) ADA_CASE(12) ADA_CASE(13) ADA_CASE(14) ADA_CASE(15)
    ADA_CASE(16) ADA_CASE(17) ADA_CASE(18) ADA_CASE(19) ADA_CASE(20) ADA_CASE(21) ADA_CASE(22) ADA_CASE(23)
    ADA_CASE(24) ADA_CASE(25) ADA_CASE(26) ADA_CASE(27) ADA_CASE(28) ADA_CASE(29) ADA_CASE(30) ADA_CASE(31)
#undef ADA_CASE
  }
  return v;
}
__device__ __forceinline__ void set_col(double (&d)[HC], int i, double v) {
  switch (i) {
#define ADA_CASE(K) case K: d[K] = v; break;
    ADA_CASE(0) ADA_CASE(1) ADA_CASE(2) ADA_CASE(3) ADA_CASE(4) ADA_CASE(5) ADA_CASE(6) ADA_CASE(7)
    ADA_CASE(8) ADA_CASE(9) ADA_CASE(10) ADA_CASE(11) ADA_CASE(12) ADA_CASE(13) ADA_CASE(14) ADA_CASE(15)
    ADA_CASE(16) ADA_CASE(17) ADA_CASE(18) ADA_CASE(19) ADA_CASE(20) ADA_CASE(21) ADA_CASE(22) ADA_CASE(23)
    ADA_CASE(24) ADA_CASE(25) ADA_CASE(26) ADA_CASE(27) ADA_CASE(28) ADA_CASE(29) ADA_CASE(30) ADA_CASE(31)
#undef ADA_CASE
  }
}
// d[c] -= l * u[c] for c = first .. HC-1 (first wave-uniform): a jump into straight-line code
__device__ __forceinline__ void update_from(double (&d)[HC], int first, double l, const double* u) {
  switch (first) {
#define ADA_CASE(K) case K: d[K] = fma(-l, u[K], d[K]); [[fallthrough]];
    ADA_CASE(0) ADA_CASE(1) ADA_CASE(2) ADA_CASE(3) ADA_CASE(4) ADA_CASE(5) ADA_CASE(6) ADA_CASE(7)
    ADA_CASE(8) ADA_CASE(9) ADA_CASE(10) ADA_CASE(11) ADA_CASE(12) ADA_CASE(13) ADA_CASE(14) ADA_CASE(15)
    ADA_CASE(16) ADA_CASE(17) ADA_CASE(18) ADA_CASE(19) ADA_CASE(20) ADA_CASE(21) ADA_CASE(22) ADA_CASE(23)
    ADA_CASE(24) ADA_CASE(25) ADA_CASE(26) ADA_CASE(27) ADA_CASE(28) ADA_CASE(29) ADA_CASE(30)
    case 31: d[31] = fma(-l, u[31], d[31]);
#undef ADA_CASE
    default: break;
  }
}

__device__ __forceinline__ unsigned long long relaxed_load_u64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void relaxed_store_u64(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr unsigned kNoCand = 0xffffffffu;  // position word of a workgroup without a candidate

__global__ __launch_bounds__(PTH) void k_getrf_panel(int n, int k0, int nbw, double* __restrict__ W, int ldw,
                                                     int* __restrict__ ipiv, DevRec* rec, PanelScratch ps) {
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
  __shared__ double s_x[2][PROWS];  // column s of every row, from the quarter holding it (by column parity)
  __shared__ double s_cv[4];
  __shared__ int s_cp[4];
  __shared__ int s_win;

  if (wg == 0 && t == 0) __hip_atomic_store(ps.moves, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

  double d[HC];
  {
    const int row = k0 + min(prow, m - 1);
    const double* base = W + (size_t)(k0 + HC * h) * ldw + row;
#pragma unroll
    for (int c = 0; c < HC; ++c) d[c] = (rvalid && HC * h + c < nbw) ? base[(size_t)c * ldw] : 0.0;
  }
  // columns of quarter h that exist (the last panel may be narrower)
  const int ncols = max(0, min(HC, nbw - HC * h));

  for (int s = 0; s < nbw; ++s) {
    const int par = s & 1;
    const int hc = s / HC;  // quarter holding column s
    const int sl = s % HC;  // its register
    const bool cur = (h == hc);
    // 1. candidate of each wave of the current quarter: largest |A(row, s)| at positions >= s, lowest position on ties
    if (cur) {
      double v = -1.0;
      int key = -1;
      const double x = get_col(d, sl);
      s_x[par][r] = x;  // read by every quarter after the exchange's barrier: each forms the multiplier itself
      if (rvalid && pos >= s) {
        v = fabs(x);
        key = pos;
      }
      wave_argmax(v, key);
      if (lane == 0) { s_cv[w - 4 * hc] = v; s_cp[w - 4 * hc] = key; }
    }
    __syncthreads();
    // the workgroup's candidate (every thread, same order)
    double bv = s_cv[0];
    int bp = s_cp[0];
#pragma unroll
    for (int q = 1; q < 4; ++q) {
      const int k2 = s_cp[q];
      const double v2 = s_cv[q];
      if (k2 >= 0 && (bp < 0 || v2 > bv || (v2 == bv && k2 < bp))) { bv = v2; bp = k2; }
    }
    const bool holder = rvalid && pos == bp;
    int p;
    if (P == 1) {
      if (holder) {
#pragma unroll
        for (int c = 0; c < HC; ++c) s_u[HC * h + c] = d[c];
      }
      __syncthreads();
      p = bp;
    } else {
      // 2. publish the candidate row, then (once those stores have completed) the candidate's record
      const unsigned G = (unsigned)(k0 + s);  // column of the factorisation: contiguous over panels
      const unsigned epoch = G + 1;
      const unsigned long long toggle = (unsigned long long)((G >> 1) & 1u) << 63;
      double* myslot = ps.slot_rows + ((size_t)par * 64 + wg) * PNB;
      if (holder) {
        // only the columns s.. of the row are read (the pivot and the update's row): the quarters left of
        // column s publish nothing
        if (HC * h + HC > s) {
#pragma unroll
          for (int c = 0; c < HC; ++c) relaxed_store(myslot + HC * h + c, d[c]);
        }
        wait_stores_done();
      }
      __syncthreads();
      if (t == 0) {
        unsigned long long* myrec = ps.recs + ((size_t)par * 64 + wg) * 2;
        relaxed_store_u64(myrec, (bp >= 0 ? dbits(bv) : 0ull) | toggle);
        relaxed_store_u64(myrec + 1, ((unsigned long long)epoch << 32) | (bp >= 0 ? (unsigned)bp : kNoCand));
      }
      // 3. wave 0: every workgroup's record (lane q reads workgroup q's), the winner, its row into LDS
      if (w == 0) {
        double cv = -1.0;
        int ck = -1;
        if (lane < P) {
          const unsigned long long* rp = ps.recs + ((size_t)par * 64 + lane) * 2;
          unsigned long long w0 = 0, w1 = 0;
          long spins = 0;
          for (;;) {
            w0 = relaxed_load_u64(rp);
            w1 = relaxed_load_u64(rp + 1);
            if ((unsigned)(w1 >> 32) == epoch && (w0 & (1ull << 63)) == toggle) break;
            if (++spins > kSpinLimit || ((spins & 1023) == 0 && relaxed_load(&rec->timeout))) {
              atomicOr(&rec->timeout, 1);
              w1 = kNoCand;
              break;
            }
            __builtin_amdgcn_s_sleep(0);
          }
          if ((unsigned)(w1 & 0xffffffffull) != kNoCand) {
            cv = __longlong_as_double((long long)(w0 & ~(1ull << 63)));
            ck = (int)(unsigned)(w1 & 0xffffffffull);
          }
        }
        int cw = lane;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          const double v2 = __shfl_xor(cv, o, 64);
          const int k2 = __shfl_xor(ck, o, 64);
          const int w2 = __shfl_xor(cw, o, 64);
          if (k2 >= 0 && (ck < 0 || v2 > cv || (v2 == cv && k2 < ck))) { cv = v2; ck = k2; cw = w2; }
        }
        const double* win = ps.slot_rows + ((size_t)par * 64 + cw) * PNB;
        s_u[lane] = relaxed_load(win + lane);  // (columns left of s: stale, never read)
        s_u[lane + 64] = relaxed_load(win + lane + 64);
        if (lane == 0) s_win = ck;
      }
      __syncthreads();
      p = s_win;
    }
    if (wg == 0 && t == 0) ipiv[k0 + s] = k0 + p;
    // 4. the interchange of positions s and p (bookkeeping only)
    const bool is_win = rvalid && pos == p;
    if (rvalid && pos == s && !is_win) pos = p;
    if (is_win) pos = s;
    const double piv = s_u[s];
    if (piv == 0.0 && wg == 0 && t == 0) atomicMin(&rec->info, k0 + s + 1);  // exact zero pivot: failure
    // 5. multiplier (every quarter forms it from column s of its row, written before the barriers above),
    //    rank-1 update; the next column's LDS writes are separated from these reads by its first barrier
    //    (s_u, s_cv) or go to the other parity's buffer (s_x)
    const bool active = piv != 0.0 && rvalid && pos > s;
    const double l = active ? s_x[par][r] / piv : 0.0;  // 0 for rows that are not updated: exact no-op
    if (cur && active) set_col(d, sl, l);
    if (h > hc) update_from(d, 0, l, s_u + HC * h);
    else if (cur && sl + 1 < HC) update_from(d, sl + 1, l, s_u + HC * h);
  }
  if (rvalid) {
    const int row = k0 + pos;
#pragma unroll
    for (int c = 0; c < HC; ++c)
      if (c < ncols) W[(size_t)(k0 + HC * h + c) * ldw + row] = d[c];
    if (h == 0 && pos != prow) {
      const int idx = atomicAdd(ps.moves, 1);
      ps.moves[1 + 2 * idx] = k0 + pos;   // destination row
      ps.moves[2 + 2 * idx] = k0 + prow;  // source row
    }
  }
}

hipError_t launch_getrf_panel(int n, int k0, int nbw, double* W, int ldw, int* ipiv, DevRec* rec, PanelScratch ps,
                              hipStream_t st) {
  const int m = n - k0;
  const int P = (m + PROWS - 1) / PROWS;
  if (P > 64 || nbw > PNB || nbw > m) return hipErrorInvalidValue;  // n - k0 <= 16384 per panel
  hipLaunchKernelGGL(k_getrf_panel, dim3(P), dim3(PTH), 0, st, n, k0, nbw, W, ldw, ipiv, rec, ps);
  return hipGetLastError();
}

// Resets the panel records before a factorisation: epochs 0 (they count the
// factorisation's columns from 1) and the toggle of every record 1, the
// opposite of its first use's toggle (columns 0 and 1), so that a reader can
// never take the initial word 0 for a current one.
__global__ void k_panel_reset(PanelScratch ps) {
  const int t = threadIdx.x;
  if (t < 2 * 64) {
    ps.recs[2 * t] = 1ull << 63;
    ps.recs[2 * t + 1] = 0ull;
  }
}

hipError_t launch_panel_reset(PanelScratch ps, hipStream_t st) {
  hipLaunchKernelGGL(k_panel_reset, dim3(1), dim3(128), 0, st, ps);
  return hipGetLastError();
}

// Apply the panel's row moves to the columns [a0, a1) and [b0, b1) (LCW per workgroup; the panel's own
// columns are never among them) and, when `with_perm`, in workgroup 0 to the permutation vector. The
// next block column and the rest are separate launches, so that only the former sits between two panels.
constexpr int LCW = 8;  // columns per workgroup: the next block column alone spreads over 16 workgroups
__global__ __launch_bounds__(256) void k_laswp_moves(int a0, int a1, int b0, int b1, int with_perm,
                                                     double* __restrict__ W, int ldw, const int* __restrict__ moves,
                                                     int* __restrict__ perm, DevRec* rec) {
  if (rec->stop) return;
  if (rec->info != INT_MAX) {
    // the panel met an exact zero pivot: the routed solve has failed; later kernels skip
    if (blockIdx.x == 0 && threadIdx.x == 0) rec->stop = 1;
    return;
  }
  const int cnt = moves[0];
  if (cnt == 0) return;
  __shared__ double sv[2 * PNB][LCW + 1];
  __shared__ int sp[2 * PNB];
  const int t = threadIdx.x;
  const int na = a1 - a0, outside = na + (b1 - b0);
  const int c0 = blockIdx.x * LCW;
  if (c0 < outside) {
    for (int mi = t; mi < cnt; mi += blockDim.x) {
      const int src = moves[2 + 2 * mi];
      for (int c = 0; c < LCW; ++c) {
        const int oc = c0 + c;
        if (oc >= outside) break;
        const int col = oc < na ? a0 + oc : b0 + (oc - na);
        sv[mi][c] = W[(size_t)src + (size_t)col * ldw];
      }
    }
  }
  if (with_perm && blockIdx.x == 0)
    for (int mi = t; mi < cnt; mi += blockDim.x) sp[mi] = perm[moves[2 + 2 * mi]];
  __syncthreads();
  if (c0 < outside) {
    for (int mi = t; mi < cnt; mi += blockDim.x) {
      const int dst = moves[1 + 2 * mi];
      for (int c = 0; c < LCW; ++c) {
        const int oc = c0 + c;
        if (oc >= outside) break;
        const int col = oc < na ? a0 + oc : b0 + (oc - na);
        W[(size_t)dst + (size_t)col * ldw] = sv[mi][c];
      }
    }
  }
  if (with_perm && blockIdx.x == 0)
    for (int mi = t; mi < cnt; mi += blockDim.x) perm[moves[1 + 2 * mi]] = sp[mi];
}

hipError_t launch_laswp_moves(int a0, int a1, int b0, int b1, bool with_perm, double* W, int ldw, const int* moves,
                              int* perm, DevRec* rec, hipStream_t st) {
  if (a1 < a0 || b1 < b0) return hipErrorInvalidValue;
  const int outside = (a1 - a0) + (b1 - b0);
  if (outside == 0 && !with_perm) return hipSuccess;
  int grid = (outside + LCW - 1) / LCW;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(k_laswp_moves, dim3(grid), dim3(256), 0, st, a0, a1, b0, b1, (int)with_perm, W, ldw, moves, perm,
                     rec);
  return hipGetLastError();
}

// U12 = L11^{-1} A12 with L11 the unit lower nbw x nbw block at W(k0,k0) and
}  // namespace ada
