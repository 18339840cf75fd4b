// Band solves for long bands (Section II-A route), parallel over the rows.
//
// Each sweep of a band solve (L with interchanges forward, U backward, U^T
// forward, L^T with interchanges backward) is a linear recurrence on a short
// state vector: the S values later rows still need (S = kl for the L sweeps,
// kl+ku for the U sweeps). Cut the n steps into chunks of LC steps; a chunk
// maps its entry state s to its exit state Phi s + phi. So
//   phase 1  every chunk computes Phi (propagating the S unit vectors with zero
//            input) and phi (propagating the right-hand side from a zero
//            state), all chunks in parallel;
//   phase 2  one short sequential scan over the chunks gives every chunk its
//            true entry state;
//   phase 3  every chunk replays its steps from that state and writes its rows.
// A sweep reads one buffer and writes another (chunks read rows that a
// neighbouring chunk writes). The band data is staged through LDS in pieces.
#include "ada_internal.h"

namespace ada {

constexpr int CPW = 4;   // chunks per workgroup (one group of 64 threads each)
constexpr int NCB = 16;  // right-hand sides per launch of phases 1 and 3
constexpr size_t kLdsMax = 160 * 1024;

__host__ __device__ inline int sweep_state(int kind, int kl, int ku) {
  return (kind == SW_L || kind == SW_LT) ? kl : kl + ku;
}
__host__ __device__ inline bool sweep_fwd(int kind) { return kind == SW_L || kind == SW_UT; }

struct Stage {
  double* col;  // [piece + 2*halo][ldgb]
  int* piv;     // [piece + 2*halo]
  int base;     // first staged column
};

// One step of a sweep. st: state; in: value entering at this step; returns the
// value finalised by the step in `out` and its row in `outpos` (-1 for none).
template <int KIND, int SM>
__device__ __forceinline__ void band_step(double (&st)[SM], int S, double in, int j, int n, int kl, int kd,
                                          int ldgb, const Stage& sg, double& out, int& outpos) {
  const double* colj = sg.col + (size_t)(j - sg.base) * ldgb;
  if (KIND == SW_L) {
    // window: positions j .. j+kl-1 (state) and b_{j+kl} (in); interchange, emit y_j, eliminate
    double w[SM + 1];
#pragma unroll
    for (int r = 0; r < SM; ++r) w[r] = st[r];
    w[SM] = 0.0;
#pragma unroll
    for (int r = 0; r <= SM; ++r)
      if (r == kl) w[r] = in;
    const int p = sg.piv[j - sg.base] - j;
#pragma unroll
    for (int r = 1; r <= SM; ++r) {
      const bool sw = (r == p);
      const double a = w[0], b = w[r];
      w[0] = sw ? b : a;
      w[r] = sw ? a : b;
    }
    out = w[0];
    outpos = j;
    const int lm = min(kl, n - 1 - j);
#pragma unroll
    for (int r = 1; r <= SM; ++r)
      if (r <= lm) w[r] = fma(-colj[kd + r], w[0], w[r]);
#pragma unroll
    for (int r = 0; r < SM; ++r) st[r] = (r < S) ? w[r + 1] : 0.0;
  } else if (KIND == SW_U) {
    // x_j = (y_j - sum_k U(j, j+k) x_{j+k}) / U(j,j); st[k-1] = x_{j+k}
    double s = in;
#pragma unroll
    for (int k = 1; k <= SM; ++k)
      if (k <= kd && j + k < n) s = fma(-sg.col[(size_t)(j + k - sg.base) * ldgb + kd - k], st[k - 1], s);
    s = s / colj[kd];
    out = s;
    outpos = j;
#pragma unroll
    for (int k = SM - 1; k >= 1; --k) st[k] = st[k - 1];
    st[0] = s;
  } else if (KIND == SW_UT) {
    // z_j = (b_j - sum_k U(j-k, j) z_{j-k}) / U(j,j); st[k-1] = z_{j-k}
    double s = in;
#pragma unroll
    for (int k = 1; k <= SM; ++k)
      if (k <= kd && j - k >= 0) s = fma(-colj[kd - k], st[k - 1], s);
    s = s / colj[kd];
    out = s;
    outpos = j;
#pragma unroll
    for (int k = SM - 1; k >= 1; --k) st[k] = st[k - 1];
    st[0] = s;
  } else {
    // window: z_j (in) and positions j+1 .. j+kl (state). w_j = z_j - sum_r L(j+r, j) w_{j+r};
    // interchange j <-> ipiv[j]; position j+kl is then final.
    double w[SM + 1];
    w[0] = in;
#pragma unroll
    for (int r = 1; r <= SM; ++r) w[r] = st[r - 1];
    const int lm = min(kl, n - 1 - j);
    double s = w[0];
#pragma unroll
    for (int r = 1; r <= SM; ++r)
      if (r <= lm) s = fma(-colj[kd + r], w[r], s);
    w[0] = s;
    const int p = sg.piv[j - sg.base] - j;
#pragma unroll
    for (int r = 1; r <= SM; ++r) {
      const bool sw = (r == p);
      const double a = w[0], b = w[r];
      w[0] = sw ? b : a;
      w[r] = sw ? a : b;
    }
    out = 0.0;
#pragma unroll
    for (int r = 0; r <= SM; ++r)
      if (r == kl) out = w[r];
    outpos = (j + kl < n) ? j + kl : -1;
#pragma unroll
    for (int r = 0; r < SM; ++r) st[r] = (r < S) ? w[r] : 0.0;
  }
}

// Physical chunk handled by group g of this workgroup (scan order -> rows).
__device__ __forceinline__ int phys_chunk(int kind, int nchunks, int scan_idx) {
  return sweep_fwd(kind) ? scan_idx : nchunks - 1 - scan_idx;
}

// All threads of the workgroup call this together; group g (threads 64g..64g+63)
// runs scan chunk blockIdx.x*CPW+g, thread v of it right-hand side c0+v (v < nc)
// in modes 1 and 2. mode 0: homogeneous (no input, no output); mode 1:
// particular (input, no output); mode 2: replay (input and output). The band
// columns, pivots and inputs of each piece are staged through LDS together.
template <int KIND, int SM>
__device__ void run_chunk(const BandSweep& B, int nchunks, bool live, int S, double (&st)[SM], int mode,
                          const double* X, int ldx, int c0, int nc, double* xout, int xstride, double* lds) {
  const int n = B.n, kl = B.kl, kd = B.kl + B.ku, ldgb = B.ldgb;
  const bool fwd = sweep_fwd(KIND);
  const int halo = kd + 1;
  const int piece = B.piece;
  const int span = piece + 2 * halo;
  const int g = threadIdx.x / 64, v = threadIdx.x % 64;
  const int ioff = (KIND == SW_L) ? kl : 0;  // the input row of step j is j + ioff
  double* gcol = lds;                                     // CPW x span x ldgb
  double* gx = lds + (size_t)CPW * span * ldgb;           // CPW x NCB x piece
  int* gpiv = reinterpret_cast<int*>(gx + (size_t)CPW * NCB * piece);  // CPW x span
  const int sc = blockIdx.x * CPW + g;
  const int ph = phys_chunk(KIND, nchunks, sc < nchunks ? sc : nchunks - 1);
  const int s0 = ph * LC, s1 = min(n, s0 + LC);
  for (int pc = 0; pc < LC; pc += piece) {
    __syncthreads();
    for (int gg = 0; gg < CPW; ++gg) {
      const int scg = blockIdx.x * CPW + gg;
      if (scg >= nchunks) break;
      const int pg = phys_chunk(KIND, nchunks, scg);
      const int g0 = pg * LC, g1 = min(n, g0 + LC);
      const int base = fwd ? (g0 + pc - halo) : (g1 - pc - piece - halo);
      double* dc = gcol + (size_t)gg * span * ldgb;
      int* dp = gpiv + gg * span;
      // the band columns base .. base+span-1 are contiguous in memory: 8 loads in flight per thread
      for (int e0 = threadIdx.x; e0 < span * ldgb; e0 += 256 * 8) {
        double tmp[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + 256 * u, c = base + e / ldgb;
          tmp[u] = (e < span * ldgb && c >= 0 && c < n) ? B.GB[(size_t)base * ldgb + e] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (e0 + 256 * u < span * ldgb) dc[e0 + 256 * u] = tmp[u];
      }
      for (int e = threadIdx.x; e < span; e += blockDim.x) {
        const int c = base + e;
        dp[e] = (c >= 0 && c < n) ? B.ipiv[c] : c;
      }
      if (mode != 0) {
        double* dx = gx + (size_t)gg * NCB * piece;
        for (int e = threadIdx.x; e < nc * piece; e += blockDim.x) {
          const int cc = e / piece, k = e % piece;
          const int j = fwd ? (g0 + pc + k) : (g1 - 1 - pc - k);
          const int row = j + ioff;
          dx[e] = (j >= g0 && j < g1 && row < n) ? X[(size_t)row + (size_t)(c0 + cc) * ldx] : 0.0;
        }
      }
    }
    __syncthreads();
    if (!live) continue;
    Stage sg;
    sg.col = gcol + (size_t)g * span * ldgb;
    sg.piv = gpiv + g * span;
    sg.base = fwd ? (s0 + pc - halo) : (s1 - pc - piece - halo);
    const double* xs = gx + (size_t)g * NCB * piece + (size_t)(v < nc ? v : 0) * piece;
    for (int k = 0; k < piece; ++k) {
      const int j = fwd ? (s0 + pc + k) : (s1 - 1 - pc - k);
      if (j < s0 || j >= s1) break;
      const double in = (mode != 0) ? xs[k] : 0.0;
      double out;
      int outpos;
      band_step<KIND, SM>(st, S, in, j, n, kl, kd, ldgb, sg, out, outpos);
      if (xout && outpos >= 0) xout[(size_t)outpos * xstride] = out;
    }
  }
  // the L^T sweep ends with positions 0 .. kl-1 in the state of the chunk holding row 0
  if (KIND == SW_LT && mode == 2 && live && ph == 0)
#pragma unroll
    for (int r = 0; r < SM; ++r)
      if (r < S && r < n) xout[(size_t)r * xstride] = st[r];
}

// phase 1: mode 0 -> Phi (thread v of a group propagates unit vector e_v, v < S) and, when H is given,
//          the response of every output position to e_v: H[pos * S + v];
//          mode 1 -> phi for right-hand sides c0 .. c0+nc-1 (thread v handles c0+v) and, when Xout is
//          given, the outputs of the chunk from a zero entry state (the particular part).
template <int KIND, int SM>
__global__ __launch_bounds__(256) void k_band_phase1(BandSweep B, int nchunks, int mode, int c0, int nc,
                                                     const double* X, int ldx, double* Phi, double* phi, double* H,
                                                     double* Xout, int ldo, const int* pred, int pred_val) {
  if (pred && *pred != pred_val) return;
  extern __shared__ double lds[];
  const int S = sweep_state(KIND, B.kl, B.ku);
  const int g = threadIdx.x / 64, v = threadIdx.x % 64;
  const int sc = blockIdx.x * CPW + g;
  const bool live = sc < nchunks && (mode == 0 ? v < S : v < nc);
  double st[SM];
#pragma unroll
  for (int r = 0; r < SM; ++r) st[r] = (mode == 0 && r == v) ? 1.0 : 0.0;
  double* xo = nullptr;
  int xs = 1;
  if (mode == 0 && H) {
    xo = H + (v < S ? v : 0);
    xs = S;
  } else if (mode == 1 && Xout) {
    xo = Xout + (size_t)(c0 + (v < nc ? v : 0)) * ldo;
  }
  run_chunk<KIND, SM>(B, nchunks, live, S, st, mode, X, ldx, c0, nc, xo, xs, lds);
  if (!live) return;
  if (mode == 0) {
#pragma unroll
    for (int r = 0; r < SM; ++r)
      if (r < S) Phi[((size_t)sc * S + r) * S + v] = st[r];
  } else {
#pragma unroll
    for (int r = 0; r < SM; ++r)
      if (r < S) phi[((size_t)sc * B.nrhs_all + c0 + v) * S + r] = st[r];
  }
}

// The outputs are affine in the chunk's entry state e: x(pos) = particular(pos) + H(pos, :) e.
// One thread per (position, right-hand side) adds the homogeneous part to the particular outputs
// phase 1 wrote; the L^T sweep's first kl positions are the exit state of the chunk holding row 0,
// Phi e + phi of that chunk.
template <int KIND, int SM>
__global__ __launch_bounds__(256) void k_band_combine(BandSweep B, int nchunks, const double* H, const double* Phi,
                                                      const double* phi, const double* entry, double* Xout, int ldo,
                                                      const int* pred, int pred_val) {
  if (pred && *pred != pred_val) return;
  const int S = sweep_state(KIND, B.kl, B.ku);
  const int n = B.n, nr = B.nrhs_all;
  const size_t total = (size_t)n * nr;
  for (size_t gi = blockIdx.x * (size_t)blockDim.x + threadIdx.x; gi < total; gi += (size_t)gridDim.x * blockDim.x) {
    const int p = (int)(gi % n), c = (int)(gi / n);
    if (KIND == SW_LT && p < B.kl) {
      const int sc0 = nchunks - 1;  // the chunk holding row 0 comes last in the backward scan
      const double* e = entry + ((size_t)sc0 * nr + c) * S;
      double x = phi[((size_t)sc0 * nr + c) * S + p];
#pragma unroll
      for (int v = 0; v < SM; ++v)
        if (v < S) x = fma(Phi[((size_t)sc0 * S + p) * S + v], e[v], x);
      Xout[(size_t)p + (size_t)c * ldo] = x;
      continue;
    }
    const int step = (KIND == SW_LT) ? p - B.kl : p;
    const int ph = step / LC;
    const int sc = sweep_fwd(KIND) ? ph : nchunks - 1 - ph;
    const double* e = entry + ((size_t)sc * nr + c) * S;
    const double* h = H + (size_t)p * S;
    double x = Xout[(size_t)p + (size_t)c * ldo];
#pragma unroll
    for (int v = 0; v < SM; ++v)
      if (v < S) x = fma(h[v], e[v], x);
    Xout[(size_t)p + (size_t)c * ldo] = x;
  }
}

// phase 2: entry state of every chunk, in three short launches over groups of
// G consecutive chunks (scan order):
//   2a  every group composes its chunk maps: M = Phi_last ... Phi_first (once per
//       factor, k_band_compose), and m_c = the group's exit state from a zero
//       entry, per right-hand side (k_band_vec_chain);
//   2b  one wave per right-hand side chains the groups (lane r holds component
//       r of the state);
//   2c  every group replays its chunk maps from its entry and writes every
//       chunk's entry state (k_band_vec_chain).
template <int KIND, int SM>
// part: 1 the maps M (depend on the factor only), 2 the particular parts m (per right-hand side), 3 both
__global__ __launch_bounds__(64) void k_band_compose(BandSweep B, int nchunks, int G, int part, const double* Phi,
                                                     const double* phi, double* Msup, double* msup,
                                                     const int* pred, int pred_val) {
  if (pred && *pred != pred_val) return;
  const int S = sweep_state(KIND, B.kl, B.ku);
  const int sg = blockIdx.x, t = threadIdx.x;
  const int nr = B.nrhs_all;
  const int c = (part & 2) ? blockIdx.y * 64 + t : nr;  // right-hand side of this lane (none for part 1)
  const bool mats = (part & 1) && blockIdx.y == 0;
  const int q0 = sg * G, q1 = min(nchunks, q0 + G);
  __shared__ double sP[SM * SM], sM[2][SM * SM];
  for (int e = t; e < S * S; e += 64) sM[0][e] = (e / S == e % S) ? 1.0 : 0.0;
  int cur = 0;
  double m[SM], pf[SM];
#pragma unroll
  for (int r = 0; r < SM; ++r) {
    m[r] = 0.0;
    pf[r] = (c < nr && r < S && q0 < q1) ? phi[((size_t)q0 * nr + c) * S + r] : 0.0;
  }
  constexpr int PE = (SM * SM + 63) / 64;  // map entries per thread
  double pre[PE];                           // the next chunk's map, loaded one step ahead
#pragma unroll
  for (int u = 0; u < PE; ++u) {
    const int e = t + 64 * u;
    pre[u] = (q0 < q1 && e < S * S) ? Phi[(size_t)q0 * S * S + e] : 0.0;
  }
  for (int q = q0; q < q1; ++q) {
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PE; ++u) {
      const int e = t + 64 * u;
      if (e < S * S) sP[e] = pre[u];
      pre[u] = (q + 1 < q1 && e < S * S) ? Phi[(size_t)(q + 1) * S * S + e] : 0.0;
    }
    __syncthreads();
    if (mats) {
#pragma unroll
      for (int u = 0; u < PE; ++u) {
        const int e = t + 64 * u;
        if (e < S * S) {
          const int r = e / S, k = e % S;
          double a = 0.0;
#pragma unroll
          for (int v = 0; v < SM; ++v)
            if (v < S) a = fma(sP[r * S + v], sM[cur][v * S + k], a);
          sM[cur ^ 1][e] = a;
        }
      }
      cur ^= 1;
    }
    double a[SM];
#pragma unroll
    for (int r = 0; r < SM; ++r) {
      double x = pf[r];
#pragma unroll
      for (int u = 0; u < SM; ++u)
        if (r < S && u < S) x = fma(sP[r * S + u], m[u], x);
      a[r] = x;
    }
#pragma unroll
    for (int r = 0; r < SM; ++r) {
      m[r] = a[r];
      pf[r] = (c < nr && r < S && q + 1 < q1) ? phi[((size_t)(q + 1) * nr + c) * S + r] : 0.0;
    }
  }
  __syncthreads();
  if (mats)
    for (int e = t; e < S * S; e += 64) Msup[(size_t)sg * S * S + e] = sM[cur][e];
  if (c < nr) {
#pragma unroll
    for (int r = 0; r < SM; ++r)
      if (r < S) msup[((size_t)sg * nr + c) * S + r] = m[r];
  }
}

template <int KIND, int SM>
__global__ __launch_bounds__(64) void k_band_chain(BandSweep B, int nsup, const double* X, int ldx,
                                                   const double* Msup, const double* msup, double* esup,
                                                   const int* pred, int pred_val) {
  if (pred && *pred != pred_val) return;
  const int S = sweep_state(KIND, B.kl, B.ku);
  const int c = blockIdx.x, r = threadIdx.x;
  const int nr = B.nrhs_all;
  double cur = (KIND == SW_L && r < S && r < B.n) ? X[(size_t)r + (size_t)c * ldx] : 0.0;
  const int rr = r < S ? r : 0;
  double pm[SM], pa;
#pragma unroll
  for (int u = 0; u < SM; ++u) pm[u] = (u < S && nsup > 0) ? Msup[(size_t)rr * S + u] : 0.0;
  pa = nsup > 0 ? msup[(size_t)c * S + rr] : 0.0;
  for (int sg = 0; sg < nsup; ++sg) {
    if (r < S) esup[((size_t)sg * nr + c) * S + r] = cur;
    double a = pa;
#pragma unroll
    for (int u = 0; u < SM; ++u)
      if (u < S) a = fma(pm[u], read_lane(cur, u), a);
    // the next group's row of M and particular part, loaded before they are needed
    if (sg + 1 < nsup) {
      const double* M = Msup + (size_t)(sg + 1) * S * S + (size_t)rr * S;
#pragma unroll
      for (int u = 0; u < SM; ++u) pm[u] = u < S ? M[u] : 0.0;
      pa = msup[((size_t)(sg + 1) * nr + c) * S + rr];
    }
    cur = r < S ? a : 0.0;
  }
}

// The per-right-hand-side chains of phase 2 over the chunks of one scan group: e <- Phi_q e + phi_q.
// One wave per (group, right-hand side); lane r holds component r of the state, the next chunk's row r
// of Phi and phi are loaded one step ahead, and the other components come by readlane, so a step
// costs S fused multiply-adds and no barrier. mode 0 (composition): start from zero, write the
// group's exit state to msup; mode 1 (fill): start from the group's entry state esup and write every
// chunk's entry state. The sums run in the same order as the matrix form (phi first, then u = 0..S-1).
template <int KIND, int SM>
__global__ __launch_bounds__(64) void k_band_vec_chain(BandSweep B, int nchunks, int G, int mode, const double* Phi,
                                                       const double* phi, const double* esup, double* msup,
                                                       double* entry, const int* pred, int pred_val) {
  if (pred && *pred != pred_val) return;
  const int S = sweep_state(KIND, B.kl, B.ku);
  const int sg = blockIdx.x, c = blockIdx.y, r = threadIdx.x;
  const int nr = B.nrhs_all;
  const int q0 = sg * G, q1 = min(nchunks, q0 + G);
  const bool act = r < S;
  const int rr = act ? r : 0;
  double e = (mode == 1 && act) ? esup[((size_t)sg * nr + c) * S + r] : 0.0;
  double prow[SM], pf = 0.0;
#pragma unroll
  for (int u = 0; u < SM; ++u) prow[u] = (u < S && q0 < q1) ? Phi[((size_t)q0 * S + rr) * S + u] : 0.0;
  if (q0 < q1) pf = phi[((size_t)q0 * nr + c) * S + rr];
  for (int q = q0; q < q1; ++q) {
    if (mode == 1 && act) entry[((size_t)q * nr + c) * S + r] = e;
    double a = pf;
#pragma unroll
    for (int u = 0; u < SM; ++u)
      if (u < S) a = fma(prow[u], read_lane(e, u), a);
    if (q + 1 < q1) {
#pragma unroll
      for (int u = 0; u < SM; ++u) prow[u] = u < S ? Phi[((size_t)(q + 1) * S + rr) * S + u] : 0.0;
      pf = phi[((size_t)(q + 1) * nr + c) * S + rr];
    }
    e = act ? a : 0.0;
  }
  if (mode == 0 && act) msup[((size_t)sg * nr + c) * S + r] = e;
}

// phase 3: replay every chunk from its entry state (right-hand sides c0 .. c0+nc-1).
template <int KIND, int SM>
__global__ __launch_bounds__(256) void k_band_phase3(BandSweep B, int nchunks, int c0, int nc, const double* Xin,
                                                     int ldi, double* Xout, int ldo, const double* entry,
                                                     const int* pred, int pred_val) {
  if (pred && *pred != pred_val) return;
  extern __shared__ double lds[];
  const int S = sweep_state(KIND, B.kl, B.ku);
  const int g = threadIdx.x / 64, v = threadIdx.x % 64;
  const int sc = blockIdx.x * CPW + g;
  const bool live = sc < nchunks && v < nc;
  double st[SM];
#pragma unroll
  for (int r = 0; r < SM; ++r) st[r] = (live && r < S) ? entry[((size_t)sc * B.nrhs_all + c0 + v) * S + r] : 0.0;
  const int c = c0 + (v < nc ? v : 0);
  run_chunk<KIND, SM>(B, nchunks, live, S, st, 2, Xin, ldi, c0, nc, Xout + (size_t)c * ldo, 1, lds);
}

// LDS of the phase 1 / phase 3 kernels for a given piece length
static size_t chunk_lds(int piece, int kd, int ldgb) {
  const size_t span = (size_t)piece + 2 * (size_t)(kd + 1);
  return (size_t)CPW * span * ldgb * sizeof(double) + (size_t)CPW * NCB * piece * sizeof(double) +
         (size_t)CPW * span * sizeof(int) + 16;
}

// chunks per group of the two-level scan
static int scan_group(int nchunks) {
  int G = 1;
  while (G * G < nchunks) ++G;
  return G;
}

template <int KIND, int SM>
static hipError_t sweep(const BandSweep& B, const double* Xin, int ldi, double* Xout, int ldo, BandScratch sc,
                        const int* pred, int pred_val, const int* map_pred, int map_pred_val, bool maps_ready,
                        hipStream_t st) {
  const int nchunks = (B.n + LC - 1) / LC;
  const int S = sweep_state(KIND, B.kl, B.ku);
  const size_t lds13 = chunk_lds(B.piece, B.kl + B.ku, B.ldgb);
  static size_t done1 = 0, done3 = 0;
  hipError_t e = ensure_lds((const void*)k_band_phase1<KIND, SM>, lds13, done1);
  if (e != hipSuccess) return e;
  e = ensure_lds((const void*)k_band_phase3<KIND, SM>, lds13, done3);
  if (e != hipSuccess) return e;
  const int grid = (nchunks + CPW - 1) / CPW;
  if (S > 0) {
    double* Phi = sc.Phi + (size_t)KIND * sc.map_stride;
    double* Msup = sc.Msup + (size_t)KIND * sc.sup_stride;
    const int G = scan_group(nchunks);
    const int nsup = (nchunks + G - 1) / G;
    double* H = sc.H + (size_t)KIND * sc.h_stride;
    if (!maps_ready) {
      // the factor's own maps: Phi per chunk with the outputs' responses H, then the maps' products
      // per scan group
      hipLaunchKernelGGL((k_band_phase1<KIND, SM>), dim3(grid), dim3(256), lds13, st, B, nchunks, 0, 0, 0, Xin, ldi,
                         Phi, sc.phi, H, (double*)nullptr, 0, map_pred, map_pred_val);
      hipLaunchKernelGGL((k_band_compose<KIND, SM>), dim3(nsup, 1), dim3(64), 0, st, B, nchunks, G, 1, Phi, sc.phi,
                         Msup, sc.msup, map_pred, map_pred_val);
    }
    for (int c0 = 0; c0 < B.nrhs_all; c0 += NCB) {
      const int nc = B.nrhs_all - c0 < NCB ? B.nrhs_all - c0 : NCB;
      hipLaunchKernelGGL((k_band_phase1<KIND, SM>), dim3(grid), dim3(256), lds13, st, B, nchunks, 1, c0, nc, Xin,
                         ldi, Phi, sc.phi, (double*)nullptr, Xout, ldo, pred, pred_val);
    }
    hipLaunchKernelGGL((k_band_vec_chain<KIND, SM>), dim3(nsup, B.nrhs_all), dim3(64), 0, st, B, nchunks, G, 0,
                       Phi, sc.phi, sc.esup, sc.msup, sc.entry, pred, pred_val);
    hipLaunchKernelGGL((k_band_chain<KIND, SM>), dim3(B.nrhs_all), dim3(64), 0, st, B, nsup, Xin, ldi, Msup,
                       sc.msup, sc.esup, pred, pred_val);
    hipLaunchKernelGGL((k_band_vec_chain<KIND, SM>), dim3(nsup, B.nrhs_all), dim3(64), 0, st, B, nchunks, G, 1,
                       Phi, sc.phi, sc.esup, sc.msup, sc.entry, pred, pred_val);
    // outputs = the particular part phase 1 wrote + H times the chunk's entry state
    const size_t total = (size_t)B.n * B.nrhs_all;
    const int cblocks = (int)((total + 255) / 256 < 8192 ? (total + 255) / 256 : 8192);
    hipLaunchKernelGGL((k_band_combine<KIND, SM>), dim3(cblocks), dim3(256), 0, st, B, nchunks, H, Phi, sc.phi,
                       sc.entry, Xout, ldo, pred, pred_val);
    return hipGetLastError();
  }
  // no state (kl = 0 for the L sweeps): every chunk starts from the empty state and replays its rows
  for (int c0 = 0; c0 < B.nrhs_all; c0 += NCB) {
    const int nc = B.nrhs_all - c0 < NCB ? B.nrhs_all - c0 : NCB;
    hipLaunchKernelGGL((k_band_phase3<KIND, SM>), dim3(grid), dim3(256), lds13, st, B, nchunks, c0, nc, Xin, ldi,
                       Xout, ldo, sc.entry, pred, pred_val);
  }
  return hipGetLastError();
}

template <int KIND>
static hipError_t sweep_any(const BandSweep& B, const double* Xin, int ldi, double* Xout, int ldo, BandScratch sc,
                            const int* pred, int pred_val, const int* map_pred, int map_pred_val,
                            unsigned* maps_ready, hipStream_t st) {
  const int S = sweep_state(KIND, B.kl, B.ku);
  const bool ready = maps_ready && ((*maps_ready >> KIND) & 1u);
  hipError_t e;
  if (S <= 8) e = sweep<KIND, 8>(B, Xin, ldi, Xout, ldo, sc, pred, pred_val, map_pred, map_pred_val, ready, st);
  else if (S <= 16) e = sweep<KIND, 16>(B, Xin, ldi, Xout, ldo, sc, pred, pred_val, map_pred, map_pred_val, ready, st);
  else e = sweep<KIND, 32>(B, Xin, ldi, Xout, ldo, sc, pred, pred_val, map_pred, map_pred_val, ready, st);
  if (e == hipSuccess && maps_ready) *maps_ready |= 1u << KIND;
  return e;
}

hipError_t launch_gbtrs_chunked(int n, int kl, int ku, int nrhs, const double* GB, int ldgb, const int* ipiv,
                                bool trans, double* X, int ldx, double* T, int ldt, BandScratch sc, const int* pred,
                                int pred_val, const int* map_pred, int map_pred_val, unsigned* maps_ready,
                                int piece_hint, hipStream_t st) {
  if (kl + ku > 31 || nrhs < 1) return hipErrorInvalidValue;
  // rows staged through LDS per step of a chunk: short pieces keep the LDS of a workgroup small, so
  // that more chunks run side by side (measured: 16 beats 8, 32 and 64 at kl + ku = 10); the
  // autotuner may name another one for a band width (the results do not depend on it)
  int piece = piece_hint > 0 ? piece_hint : 16;
  while (piece > 8 && chunk_lds(piece, kl + ku, ldgb) > kLdsMax) piece /= 2;
  if (chunk_lds(piece, kl + ku, ldgb) > kLdsMax) return hipErrorInvalidValue;
  BandSweep B{GB, ldgb, kl, ku, n, ipiv, nrhs, piece};
  hipError_t e;
  if (!trans) {
    e = sweep_any<SW_L>(B, X, ldx, T, ldt, sc, pred, pred_val, map_pred, map_pred_val, maps_ready, st);
    if (e != hipSuccess) return e;
    return sweep_any<SW_U>(B, T, ldt, X, ldx, sc, pred, pred_val, map_pred, map_pred_val, maps_ready, st);
  }
  e = sweep_any<SW_UT>(B, X, ldx, T, ldt, sc, pred, pred_val, map_pred, map_pred_val, maps_ready, st);
  if (e != hipSuccess) return e;
  return sweep_any<SW_LT>(B, T, ldt, X, ldx, sc, pred, pred_val, map_pred, map_pred_val, maps_ready, st);
}

bool band_piece_fits(int piece, int kl, int ku) {
  return piece >= 8 && chunk_lds(piece, kl + ku, 2 * kl + ku + 1) <= kLdsMax;
}

__global__ void k_band_tune_fill(int n, int kl, int ku, double* GB, int ldgb, int* ipiv, double* X, int nrhs) {
  const size_t total = (size_t)n * ldgb;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % ldgb), j = (int)(e / ldgb);
    double v = 0.0;
    if (r == kl + ku) v = 4.0;
    else if (r >= kl) {
      // a fixed hash of the position, mapped to [-0.25, 0.25]
      unsigned h = (unsigned)e * 2654435761u;
      h ^= h >> 15;
      v = ((double)(h & 0xffff) / 65535.0 - 0.5) * 0.5;
    }
    (void)j;
    GB[e] = v;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    ipiv[i] = i;
    for (int c = 0; c < nrhs; ++c) X[(size_t)i + (size_t)c * n] = 1.0;
  }
}

hipError_t launch_band_tune_fill(int n, int kl, int ku, double* GB, int ldgb, int* ipiv, double* X, int nrhs,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_band_tune_fill, dim3(1024), dim3(256), 0, st, n, kl, ku, GB, ldgb, ipiv, X, nrhs);
  return hipGetLastError();
}

size_t band_chunked_scratch_doubles(int n, int kl, int ku, int nrhs) {
  const size_t nchunks = (size_t)(n + LC - 1) / LC;
  const size_t S = (size_t)(kl + ku) > 1 ? (size_t)(kl + ku) : 1;
  const size_t G = (size_t)scan_group((int)nchunks), nsup = (nchunks + G - 1) / G;
  return 4 * nchunks * S * S + 4 * nsup * S * S + 4 * (size_t)n * S + 2 * nchunks * (size_t)nrhs * S +
         2 * nsup * (size_t)nrhs * S + 64;
}

BandScratch band_chunked_scratch(double* base, int n, int kl, int ku, int nrhs) {
  const size_t nchunks = (size_t)(n + LC - 1) / LC;
  const size_t S = (size_t)(kl + ku) > 1 ? (size_t)(kl + ku) : 1;
  const size_t G = (size_t)scan_group((int)nchunks), nsup = (nchunks + G - 1) / G;
  BandScratch sc;
  sc.map_stride = nchunks * S * S;
  sc.sup_stride = nsup * S * S;
  sc.h_stride = (size_t)n * S;
  sc.Phi = base;
  sc.Msup = sc.Phi + 4 * sc.map_stride;
  sc.H = sc.Msup + 4 * sc.sup_stride;
  sc.phi = sc.H + 4 * sc.h_stride;
  sc.entry = sc.phi + nchunks * (size_t)nrhs * S;
  sc.msup = sc.entry + nchunks * (size_t)nrhs * S;
  sc.esup = sc.msup + nsup * (size_t)nrhs * S;
  return sc;
}

}  // namespace ada
