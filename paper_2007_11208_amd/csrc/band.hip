// Banded route (Section II-A): the compact band format (one diagonal per row
// of a dense array, with kl extra rows for the fill of row interchanges), LU
// with partial pivoting restricted to the kl+1 candidate rows of each column,
// the band solves, and the band norms.
//
// Element (i,j) of the working band lives at GB[(kl+ku) + i - j + j*ldgb],
// ldgb >= 2kl+ku+1. Partial pivoting makes the factorisation a chain of n
// dependent column steps; it runs in one compute wave that keeps the active
// (kl+1) x (kl+ku+1) window in registers (lane = column of the window), while
// three loader waves stream the next chunks of the band into an LDS ring, so
// the chain never waits on HBM. The solves use the same scheme with lane =
// right-hand side.
#include "ada_internal.h"

#include <climits>

namespace ada {


__global__ void k_band_pack_dense(int n, int kl, int ku, const double* __restrict__ A, int lda,
                                  double* __restrict__ GB, int ldgb) {
  const int kd = kl + ku;
  const size_t total = (size_t)ldgb * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % ldgb), j = (int)(e / ldgb);
    const int i = r - kd + j;  // row of this storage slot
    double v = 0.0;
    if (r >= kl && i >= 0 && i < n && i - j <= kl) v = A[(size_t)i + (size_t)j * lda];
    GB[e] = v;
  }
}

hipError_t launch_band_pack_dense(int n, int kl, int ku, const double* A, int lda, double* GB, int ldgb,
                                  hipStream_t st) {
  size_t total = (size_t)ldgb * n;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_band_pack_dense, dim3(blocks), dim3(256), 0, st, n, kl, ku, A, lda, GB, ldgb);
  return hipGetLastError();
}

// from LAPACK band storage AB[ku_in + i - j + j*ldab] (any stored width >= the true one)
__global__ void k_band_pack_band(int n, int kl, int ku, const double* __restrict__ AB, int ldab, int ku_in,
                                 double* __restrict__ GB, int ldgb) {
  const int kd = kl + ku;
  const size_t total = (size_t)ldgb * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int r = (int)(e % ldgb), j = (int)(e / ldgb);
    const int i = r - kd + j;
    double v = 0.0;
    if (r >= kl && i >= 0 && i < n && i - j <= kl) v = AB[(size_t)(ku_in + i - j) + (size_t)j * ldab];
    GB[e] = v;
  }
}

hipError_t launch_band_pack_band(int n, int kl, int ku, const double* AB, int ldab, int ku_in, double* GB,
                                 int ldgb, hipStream_t st) {
  size_t total = (size_t)ldgb * n;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_band_pack_band, dim3(blocks), dim3(256), 0, st, n, kl, ku, AB, ldab, ku_in, GB, ldgb);
  return hipGetLastError();
}

__global__ void k_band_to_dense(int n, int kl_in, int ku_in, const double* __restrict__ AB, int ldab,
                                double* __restrict__ A, int lda) {
  const size_t total = (size_t)n * n;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % n), j = (int)(e / n);
    double v = 0.0;
    if (i - j <= kl_in && j - i <= ku_in) v = AB[(size_t)(ku_in + i - j) + (size_t)j * ldab];
    A[(size_t)i + (size_t)j * lda] = v;
  }
}

hipError_t launch_band_to_dense(int n, int kl_in, int ku_in, const double* AB, int ldab, double* A, int lda,
                                hipStream_t st) {
  size_t total = (size_t)n * n;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_band_to_dense, dim3(blocks), dim3(256), 0, st, n, kl_in, ku_in, AB, ldab, A, lda);
  return hipGetLastError();
}

// ||A||_1 (max column sum) and ||A||_inf (max row sum) of the band before factorisation. A workgroup
// copies the band storage of its BNT columns and the kl + ku columns around them into LDS (one contiguous
// stretch of the layout, read coalesced), then threads 0..BNT-1 sum columns and BNT..2BNT-1 sum rows from
// LDS, each in increasing row / column order.
constexpr int BNT = 128;
__global__ __launch_bounds__(256) void k_band_norms(int n, int kl, int ku, const double* __restrict__ GB, int ldgb,
                                                    DevRec* rec) {
  extern __shared__ double tile[];  // columns lo .. hi-1 of the band storage
  const int kd = kl + ku, t = threadIdx.x;
  const int c0 = blockIdx.x * BNT;
  const int lo = max(0, c0 - kl), hi = min(n, c0 + BNT + ku);
  const int cnt = (hi - lo) * ldgb;
  const double* src = GB + (size_t)lo * ldgb;
  for (int e = t; e < cnt; e += 256) tile[e] = src[e];
  __syncthreads();
  double c1 = 0.0, ri = 0.0;
  if (t < BNT) {
    const int x = c0 + t;  // column x: rows x - ku .. x + kl
    if (x < n) {
      double s = 0.0;
      for (int d = 0; d <= kd; ++d) {
        const int i = x - ku + d;
        if (i >= 0 && i < n) s += fabs(tile[(x - lo) * ldgb + kd + i - x]);
      }
      c1 = s;
    }
  } else {
    const int x = c0 + t - BNT;  // row x: columns x - kl .. x + ku
    if (x < n) {
      double r = 0.0;
      for (int d = 0; d <= kd; ++d) {
        const int j = x - kl + d;
        if (j >= 0 && j < n) r += fabs(tile[(j - lo) * ldgb + kd + x - j]);
      }
      ri = r;
    }
  }
  c1 = wave_max(c1);
  ri = wave_max(ri);
  if ((t & 63) == 0) {
    if (c1 > 0.0) atomicMax(reinterpret_cast<unsigned long long*>(&rec->anorm1), dbits(c1));
    if (ri > 0.0) atomicMax(reinterpret_cast<unsigned long long*>(&rec->anorm_inf), dbits(ri));
  }
}

hipError_t launch_band_norms(int n, int kl, int ku, const double* GB, int ldgb, DevRec* rec, hipStream_t st) {
  if (kl + ku > 31 || ldgb < 2 * kl + ku + 1 || ldgb > 63) return hipErrorInvalidValue;
  const size_t lds = (size_t)(BNT + kl + ku) * ldgb * sizeof(double);  // <= 159 * 63 * 8 bytes
  static size_t done = 0;
  hipError_t e = ensure_lds((const void*)k_band_norms, lds, done);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_band_norms, dim3((n + BNT - 1) / BNT), dim3(256), lds, st, n, kl, ku, GB, ldgb, rec);
  return hipGetLastError();
}

// ---------------------------------------------------------------- factorisation
// Band kernels need kl + ku <= BAND_KD_MAX (the window spans one lane per column).
constexpr int BAND_KD_MAX = 31;
constexpr int BCH2 = 32;  // chunk length; the LDS rings hold 4 chunks

// Window of the band LU at step j: columns j .. j+kd, rows j .. j+kl. Lane c
// (c < W = kd+1) permanently owns the columns congruent to c modulo W, so the
// window advances without moving data between lanes: the lane whose column is
// finished takes the column that enters on the right. Each lane keeps rows
// j .. j+kl of its column in registers; the scalars the step broadcasts (pivot
// index, pivot, multipliers) are read with readlane. LDS ring: 4 chunks of
// `chf` columns, streamed by three loader waves two chunks ahead.
template <int KLM>
__global__ __launch_bounds__(256) void k_gbtrf(int n, int kl, int ku, double* __restrict__ GB, int ldgb,
                                               int* __restrict__ ipiv, DevRec* rec, int chf) {
  const int kd = kl + ku, W = kd + 1;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int SL = 4 * chf;
  extern __shared__ double ring[];  // ring[(col % SL) * ldgb + r] = original GB column
  const int nch = (n + chf - 1) / chf;
  auto load_chunk = [&](int q) {
    if (q < 0 || q >= nch) return;
    const int c0 = q * chf, c1 = min(n, c0 + chf);
    const int cnt = (c1 - c0) * ldgb;
    for (int e = t - 64; e < cnt; e += 192) {
      const int r = e % ldgb, c = c0 + e / ldgb;
      ring[(size_t)(c % SL) * ldgb + r] = GB[(size_t)r + (size_t)c * ldgb];
    }
  };
  auto R = [&](int off, int col) -> double { return ring[(size_t)(col % SL) * ldgb + off]; };

  if (w >= 1) { load_chunk(0); load_chunk(1); }
  __syncthreads();
  double v[KLM + 1];
#pragma unroll
  for (int r = 0; r <= KLM; ++r) v[r] = 0.0;
  if (w == 0 && lane < W && lane < n) {
#pragma unroll
    for (int r = 0; r <= KLM; ++r)
      if (r <= kl && r < n) v[r] = R(kd + r - lane, lane);
  }
  int info = INT_MAX;
  int cl = 0;  // lane holding column j
  for (int q = 0; q < nch; ++q) {
    if (w >= 1) load_chunk(q + 2);
    if (w == 0) {
      const int jend = min(n, (q + 1) * chf);
      for (int j = q * chf; j < jend; ++j) {
        int o = lane - cl;  // this lane's column is j + o
        if (o < 0) o += W;
        const int mycol = j + o;
        // the entry that joins this lane's registers for step j+1 (prefetched now, off the chain)
        const int o1 = (o == 0) ? kd : o - 1;  // offset of this lane's column at step j+1
        const int col1 = j + 1 + o1;
        const int row1 = j + 1 + kl;
        const double nxt = (lane < W && row1 < n && col1 < n) ? R(kd + kl - o1, col1) : 0.0;
        const int lm = min(kl, n - 1 - j);
        // pivot search in the lane of column j (first maximum)
        int p = 0;
        if (lane == cl) {
          double best = fabs(v[0]);
#pragma unroll
          for (int r = 1; r <= KLM; ++r) {
            const double a = fabs(v[r]);
            const bool take = (r <= lm) && (a > best);
            best = take ? a : best;
            p = take ? r : p;
          }
          ipiv[j] = j + p;
        }
        p = __builtin_amdgcn_readlane(p, cl);
#pragma unroll
        for (int r = 1; r <= KLM; ++r) {
          const bool sw = (r == p);
          const double a = v[0], b = v[r];
          v[0] = sw ? b : a;
          v[r] = sw ? a : b;
        }
        const double piv = read_lane(v[0], cl);
        if (piv == 0.0) {
          if (info == INT_MAX) info = j + 1;
        } else {
          const double rp = 1.0 / piv;
          if (lane == cl) {
#pragma unroll
            for (int r = 1; r <= KLM; ++r)
              if (r <= lm) v[r] *= rp;
          }
          double l[KLM + 1];
#pragma unroll
          for (int r = 1; r <= KLM; ++r) l[r] = read_lane(v[r], cl);
          if (lane < W && o >= 1 && mycol < n) {
#pragma unroll
            for (int r = 1; r <= KLM; ++r)
              if (r <= lm) v[r] = fma(-l[r], v[0], v[r]);
          }
        }
        // column j is final (U(j,j) and the multipliers); row j of U is final in every other lane
        if (lane == cl) {
#pragma unroll
          for (int r = 0; r <= KLM; ++r)
            if (r <= lm) GB[(size_t)(kd + r) + (size_t)j * ldgb] = v[r];
        } else if (lane < W && mycol < n) {
          GB[(size_t)(kd - o) + (size_t)mycol * ldgb] = v[0];
        }
        // advance: rows move up one register; the finished lane starts column j+W (fill rows are zero)
#pragma unroll
        for (int r = 0; r < KLM; ++r) v[r] = (lane == cl) ? 0.0 : v[r + 1];
        v[KLM] = 0.0;
#pragma unroll
        for (int r = 0; r <= KLM; ++r)
          if (r == kl) v[r] = nxt;
        cl = (cl + 1 == W) ? 0 : cl + 1;
      }
    }
    __syncthreads();
  }
  if (w == 0 && lane == 0 && info != INT_MAX) {
    atomicMin(&rec->info, info);
    rec->stop = 1;
  }
}

// Band LU for 1 <= kl <= 8 with the band width a compile-time constant,
// out of place (reads the packed band `in`, writes the factor `out`).
//
// Step j of the factorisation depends on the earlier steps only through the
// active window (rows j .. j+kl of columns j .. j+kl+ku), so the chain can be
// cut into chunks of L steps that run at once:
//   mode 0  every chunk starts from a guess of its entry window (the original
//           entries, i.e. no influence of the rows above) and runs its L steps,
//           keeping snapshots of the window at its first group starts and its
//           exit window;
//   mode 1  chunk c (c >= 1) restarts from the exit window of chunk c-1 and
//           compares its window, bit for bit, with chunk c's mode-0 snapshots;
//           once they agree, every later step of chunk c is what mode 0
//           computed, so it stops. A chunk whose window does not agree within
//           the snapshots, or any zero pivot, marks the speculation failed;
//   mode 2  the plain sequential factorisation, launched in every case and
//           predicated on that mark.
// When the speculation holds, the result is bit-identical to the sequential
// one: chunk 0 starts exact, and by induction every chunk's mode-0 exit window
// is exact once its successor's check has passed. On diagonally dominant
// bands the window forgets its entry state within a few dozen steps.
//
// Within a chunk, one wave runs the chain (lane = window column, rows j ..
// j+KL in registers); the register holding row 0 at step j becomes row KL at
// step j+1, so the loop is unrolled KL+1 times with the register names
// rotated at compile time; the usual case, no interchange, is told by one
// comparison and one ballot; three loader waves stream the band into an LDS
// ring.
struct GbSpec {
  const double* in;
  double* out;
  int* ipiv;
  DevRec* rec;
  double* snap;    // [chunk][nsnap][KL+1][64]
  double* exitst;  // [chunk][KL+1][64]
  int L;           // steps per chunk (a multiple of the ring chunk)
  int nsnap;       // snapshots per chunk (at group starts)
  int mode;
  const int* pred;  // mode 2: run only when *pred != 0 (null: always)
};

template <int KL>
struct GbWave {
  static constexpr int R = KL + 1;
  double v[R];
  int o;        // column offset of this lane's column from the current step j
  int slot;     // ring offset (doubles) of this lane's column
  int cl;       // lane holding column j (uniform)
  int bad;      // a zero pivot was met (uniform)
  int kd, W, ldgb, RS, n, lane;
  const double* ring;
  double* out;
  int* ipiv;

  template <int S>
  __device__ __forceinline__ void step(int j) {
#define VR(r) v[((r) + S) % R]
    // pivot: first maximum of |column j| over rows j .. j+KL (rows past n hold zeros)
    bool ge = true;
#pragma unroll
    for (int r = 1; r <= KL; ++r) ge = ge && (fabs(VR(0)) >= fabs(VR(r)));
    const unsigned long long keep = __ballot(ge);
    int p = 0;
    if (!((keep >> cl) & 1ull)) {
      double best = fabs(VR(0));
      int pp = 0;
#pragma unroll
      for (int r = 1; r <= KL; ++r) {
        const double a = fabs(VR(r));
        const bool take = a > best;
        best = take ? a : best;
        pp = take ? r : pp;
      }
      p = __builtin_amdgcn_readlane(pp, cl);
#pragma unroll
      for (int r = 1; r <= KL; ++r) {
        if (p == r) {
          const double a = VR(0);
          VR(0) = VR(r);
          VR(r) = a;
        }
      }
    }
    if (lane == 0) ipiv[j] = j + p;
    const double piv = read_lane(VR(0), cl);
    double rp = 0.0;
    if (piv == 0.0) {
      bad = min(bad, j + 1);
    } else {
      rp = 1.0 / piv;
    }
    double l[R];
#pragma unroll
    for (int r = 1; r <= KL; ++r) l[r] = read_lane(VR(r), cl) * rp;
#pragma unroll
    for (int r = 1; r <= KL; ++r) VR(r) = fma(-l[r], VR(0), VR(r));
    // row j of U (U(j,j) from lane cl), then the multipliers of column j
    if (lane < W && j + o < n) out[(size_t)(kd - o) + (size_t)(j + o) * ldgb] = VR(0);
    if (lane == cl) {
      double* col = out + (size_t)j * ldgb + kd;
#pragma unroll
      for (int r = 1; r <= KL; ++r) col[r] = l[r];
    }
    // advance: lane cl takes column j+W (rows j+1 .. j+KL of it are zero); every lane
    // receives the entry of row j+1+KL of its column
    const bool fin = lane == cl;
    const int o2 = fin ? kd : o - 1;
    int s2 = slot + W * ldgb;
    s2 = s2 >= RS ? s2 - RS : s2;
    slot = fin ? s2 : slot;
    o = o2;
    double nx = 0.0;
    if (j + 1 + KL < n && lane < W) nx = ring[slot + kd + KL - o2];
    if (fin) {
#pragma unroll
      for (int r = 1; r <= KL; ++r) VR(r) = 0.0;
    }
    VR(0) = nx;
    cl = __builtin_amdgcn_readfirstlane((cl + 1 == W) ? 0 : cl + 1);
#undef VR
  }
};

template <int KL, int S>
struct GbUnroll {
  __device__ __forceinline__ static void run(GbWave<KL>& g, int j, int jend) {
    if (j + S >= jend) return;
    g.template step<S>(j + S);
    GbUnroll<KL, S + 1>::run(g, j, jend);
  }
};
template <int KL>
struct GbUnroll<KL, KL + 1> {
  __device__ __forceinline__ static void run(GbWave<KL>&, int, int) {}
};

template <int KL>
__global__ __launch_bounds__(256) void k_gbtrf_k(int n, int ku, int ldgb, int chf, GbSpec sp) {
  constexpr int R = KL + 1;
  if (sp.pred && *sp.pred == 0) return;
  const int kd = KL + ku, W = kd + 1;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int c = sp.mode == 1 ? blockIdx.x + 1 : blockIdx.x;  // chunk
  const int s0 = c * sp.L, s1 = min(n, s0 + sp.L);
  const bool last = s1 == n;
  const int SL = 4 * chf;
  extern __shared__ double ring[];  // ring[((col - s0) % SL) * ldgb + r] = original band column col
  __shared__ int s_done;
  const int nq = (s1 - s0 + chf - 1) / chf;
  auto load_chunk = [&](int q) {
    if (q < 0 || q > nq + 1) return;
    const int c0 = s0 + q * chf;
    const int cnt = chf * ldgb;
    for (int e = t - 64; e < cnt; e += 192) {
      const int r = e % ldgb, cc = c0 + e / ldgb;
      ring[(size_t)((cc - s0) % SL) * ldgb + r] = cc < n ? sp.in[(size_t)r + (size_t)cc * ldgb] : 0.0;
    }
  };
  if (t == 0) s_done = 0;
  if (w >= 1) { load_chunk(0); load_chunk(1); }
  __syncthreads();
  GbWave<KL> g;
  g.kd = kd; g.W = W; g.ldgb = ldgb; g.RS = SL * ldgb; g.n = n; g.lane = lane; g.ring = ring;
  g.out = sp.out; g.ipiv = sp.ipiv;
  g.cl = 0; g.bad = INT_MAX;
  g.o = lane < W ? lane : 0;
  g.slot = lane < W ? lane * ldgb : 0;
  double* snapc = sp.snap + (size_t)c * sp.nsnap * R * 64;
  if (sp.mode == 1) {
    const double* ex = sp.exitst + (size_t)(c - 1) * R * 64;
#pragma unroll
    for (int r = 0; r < R; ++r) g.v[r] = ex[r * 64 + lane];
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
      g.v[r] = (lane < W && s0 + lane < n && s0 + r < n) ? ring[lane * ldgb + kd + r - lane] : 0.0;
  }
  double sn[R];  // mode 1: the snapshot due at the next group start
#pragma unroll
  for (int r = 0; r < R; ++r) sn[r] = (sp.mode == 1) ? snapc[r * 64 + lane] : 0.0;
  int grp = 0;
  for (int q = 0; q < nq; ++q) {
    if (w >= 1) {
      load_chunk(q + 2);
    } else {
      const int jend = min(s1, s0 + (q + 1) * chf);
      bool stop = false;
      for (int j = s0 + q * chf; j < jend; j += R) {
        if (sp.mode == 0 && grp < sp.nsnap) {
          double* d = snapc + (size_t)grp * R * 64;
#pragma unroll
          for (int r = 0; r < R; ++r) d[r * 64 + lane] = g.v[r];
        } else if (sp.mode == 1) {
          if (grp < sp.nsnap) {
            bool eq = true;
#pragma unroll
            for (int r = 0; r < R; ++r) eq = eq && (__double_as_longlong(g.v[r]) == __double_as_longlong(sn[r]));
            if (__ballot(eq) == ~0ull) { stop = true; break; }
            if (grp + 1 < sp.nsnap) {
              const double* d = snapc + (size_t)(grp + 1) * R * 64;
#pragma unroll
              for (int r = 0; r < R; ++r) sn[r] = d[r * 64 + lane];
            }
          } else if (!last) {
            // no agreement within the snapshots: the speculation does not hold here
            if (lane == 0) atomicOr(&sp.rec->band_spec_bad, 1);
            stop = true;
            break;
          }
        }
        GbUnroll<KL, 0>::run(g, j, jend);
        ++grp;
      }
      if (stop && lane == 0) s_done = 1;
    }
    __syncthreads();
    if (s_done) break;
  }
  if (w == 0) {
    if (sp.mode == 2) {
      if (lane == 0 && g.bad != INT_MAX) {
        atomicMin(&sp.rec->info, g.bad);
        sp.rec->stop = 1;
      }
    } else {
      if (lane == 0 && g.bad != INT_MAX) atomicOr(&sp.rec->band_spec_bad, 1);
      if (sp.mode == 0 && !last) {
        // exit window in the order of the next chunk's start: column s1 + o at position o
        double* ex = sp.exitst + (size_t)c * R * 64;
        const int at = lane < W ? g.o : lane;
#pragma unroll
        for (int r = 0; r < R; ++r) ex[r * 64 + at] = g.v[r];
      }
    }
  }
}

// ring chunk length: a multiple of kl+1 (whole unrolled groups) and > kl+ku+1 (the window spans two chunks)
static int gbtrf_chf(int kl, int ldgb) { return (kl + 1) * ((ldgb <= 32 ? 128 : 64) / (kl + 1)); }
constexpr int kGbSpecChunks = 16;    // ring chunks per speculative chunk (at least)
constexpr int kGbSpecSteps = 256;    // steps covered by the snapshots

GbSpecPlan gbtrf_spec_plan(int n, int kl, int ku) {
  GbSpecPlan p{};
  if (kl < 1 || kl > 8 || kl + ku > BAND_KD_MAX) return p;
  const int ldgb = 2 * kl + ku + 1;
  const int chf = gbtrf_chf(kl, ldgb);
  int q = (n + chf * 512 - 1) / (chf * 512);  // about 512 chunks at most
  if (q < kGbSpecChunks / 4) q = kGbSpecChunks / 4;
  p.L = chf * q;
  p.nchunks = (n + p.L - 1) / p.L;
  if (p.nchunks < 2) return GbSpecPlan{};
  p.nsnap = (kGbSpecSteps + kl) / (kl + 1);
  p.snap_doubles = (size_t)p.nchunks * p.nsnap * (kl + 1) * 64;
  p.exit_doubles = (size_t)p.nchunks * (kl + 1) * 64;
  return p;
}

hipError_t launch_gbtrf(int n, int kl, int ku, const double* GBin, double* GB, int ldgb, int* ipiv, DevRec* rec,
                        double* spec_scratch, size_t spec_doubles, hipStream_t st) {
  const int kd = kl + ku;
  if (kd > BAND_KD_MAX) return hipErrorInvalidValue;
  if (kl >= 1 && kl <= 8) {
    const int chf = gbtrf_chf(kl, ldgb);
    const size_t lds = (size_t)4 * chf * ldgb * sizeof(double);
    GbSpecPlan sp = gbtrf_spec_plan(n, kl, ku);
    const bool spec = sp.nchunks >= 2 && spec_scratch && sp.snap_doubles + sp.exit_doubles <= spec_doubles;
    GbSpec a{GBin, GB, ipiv, rec, spec_scratch, spec ? spec_scratch + sp.snap_doubles : nullptr, spec ? sp.L : n,
             sp.nsnap, 2, nullptr};
#define ADA_GBTRF_K(K)                                                                                  \
  case K: {                                                                                             \
    static size_t done = 0;                                                                             \
    hipError_t e = ensure_lds((const void*)k_gbtrf_k<K>, lds, done);                                   \
    if (e != hipSuccess) return e;                                                                      \
    if (spec) {                                                                                         \
      a.mode = 0;                                                                                       \
      hipLaunchKernelGGL(k_gbtrf_k<K>, dim3(sp.nchunks), dim3(256), lds, st, n, ku, ldgb, chf, a);     \
      a.mode = 1;                                                                                       \
      hipLaunchKernelGGL(k_gbtrf_k<K>, dim3(sp.nchunks - 1), dim3(256), lds, st, n, ku, ldgb, chf, a); \
      a.mode = 2;                                                                                       \
      a.L = n;                                                                                          \
      a.pred = &rec->band_spec_bad;                                                                     \
    }                                                                                                   \
    hipLaunchKernelGGL(k_gbtrf_k<K>, dim3(1), dim3(256), lds, st, n, ku, ldgb, chf, a);                \
    return hipGetLastError();                                                                           \
  }
    switch (kl) {
      ADA_GBTRF_K(1)
      ADA_GBTRF_K(2)
      ADA_GBTRF_K(3)
      ADA_GBTRF_K(4)
      ADA_GBTRF_K(5)
      ADA_GBTRF_K(6)
      ADA_GBTRF_K(7)
      ADA_GBTRF_K(8)
    }
#undef ADA_GBTRF_K
  }
  // other widths: the general in-place kernel on a copy of the band
  if (GB != GBin) {
    hipError_t e = hipMemcpyAsync(GB, GBin, sizeof(double) * (size_t)ldgb * n, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  const int chf = ldgb <= 32 ? 128 : 64;  // chunk length > kd + 1 keeps the window inside two chunks
  const size_t lds = (size_t)4 * chf * ldgb * sizeof(double);
#define ADA_GBTRF(K)                                                                                         \
  do {                                                                                                       \
    static size_t done = 0;                                                                                  \
    hipError_t e = ensure_lds((const void*)k_gbtrf<K>, lds, done);                                          \
    if (e != hipSuccess) return e;                                                                           \
    hipLaunchKernelGGL(k_gbtrf<K>, dim3(1), dim3(256), lds, st, n, kl, ku, GB, ldgb, ipiv, rec, chf);       \
  } while (0)
  if (kl <= 4) ADA_GBTRF(4);
  else if (kl <= 8) ADA_GBTRF(8);
  else if (kl <= 16) ADA_GBTRF(16);
  else ADA_GBTRF(32);
#undef ADA_GBTRF
  return hipGetLastError();
}

// ---------------------------------------------------------------- solves
// trans = 0: A x = b with A = P0 L0 P1 L1 ... U: forward (interchange, unit
//            lower band) then backward with U (kl+ku super-diagonals);
// trans = 1: A^T x = b: U^T forward, then L^T backward with the interchanges
//            applied in reverse order.
// One compute wave, lane = right-hand side (nrhs <= 32 per launch). Band
// columns, pivots and the right-hand-side rows are streamed through LDS rings
// by three loader waves two chunks ahead of the compute wave.
template <int KW>
__global__ __launch_bounds__(256) void k_gbtrs(int n, int kl, int ku, int nrhs, const double* __restrict__ GB,
                                               int ldgb, const int* __restrict__ ipiv, int trans, double* X, int ldx,
                                               const int* pred, int pred_val) {
  if (pred && *pred != pred_val) return;
  const int kd = kl + ku;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  constexpr int SL = 4 * BCH2;
  extern __shared__ double lds[];
  double* ring = lds;                                     // [SL][ldgb]
  double* xr = ring + (size_t)SL * ldgb;                  // [SL][nrhs]
  int* pring = reinterpret_cast<int*>(xr + (size_t)SL * nrhs);  // [SL]
  const int nch = (n + BCH2 - 1) / BCH2;
  const bool active = w == 0 && lane < nrhs;
  double* x = X + (size_t)lane * ldx;

  auto load_chunk = [&](int q) {
    if (q < 0 || q >= nch) return;
    const int c0 = q * BCH2, c1 = min(n, c0 + BCH2);
    const int cnt = (c1 - c0) * ldgb;
    for (int e = t - 64; e < cnt; e += 192) {
      const int r = e % ldgb, c = c0 + e / ldgb;
      ring[(size_t)(c % SL) * ldgb + r] = GB[(size_t)r + (size_t)c * ldgb];
    }
    const int xc = (c1 - c0) * nrhs;
    for (int e = t - 64; e < xc; e += 192) {
      const int cc = e % nrhs, row = c0 + e / nrhs;
      xr[(size_t)(row % SL) * nrhs + cc] = X[(size_t)row + (size_t)cc * ldx];
    }
    for (int c = c0 + t - 64; c < c1; c += 192) pring[c % SL] = ipiv[c];
  };
  auto R = [&](int off, int col) -> double { return ring[(size_t)(col % SL) * ldgb + off]; };
  auto XR = [&](int row) -> double { return xr[(size_t)(row % SL) * nrhs + lane]; };

  double win[KW + 1];
  // ------------------------------------------------ pass 1: rows in increasing order
  if (w >= 1) { load_chunk(0); load_chunk(1); }
  __syncthreads();
#pragma unroll
  for (int r = 0; r <= KW; ++r) win[r] = 0.0;
  if (!trans && active) {
#pragma unroll
    for (int r = 0; r <= KW; ++r)
      if (r <= kl && r < n) win[r] = XR(r);
  }
  for (int q = 0; q < nch; ++q) {
    if (w >= 1) load_chunk(q + 2);
    if (active) {
      const int jend = min(n, (q + 1) * BCH2);
      for (int j = q * BCH2; j < jend; ++j) {
        if (!trans) {
          // y = L^{-1} P b; window win[r] = b_{j+r}
          const int lm = min(kl, n - 1 - j);
          const int p = pring[j % SL] - j;
          if (p != 0) {
#pragma unroll
            for (int r = 1; r <= KW; ++r)
              if (r == p) { const double tmp = win[0]; win[0] = win[r]; win[r] = tmp; }
          }
#pragma unroll
          for (int r = 1; r <= KW; ++r)
            if (r <= lm) win[r] = fma(-R(kd + r, j), win[0], win[r]);
          x[j] = win[0];
#pragma unroll
          for (int r = 0; r < KW; ++r) win[r] = win[r + 1];
          win[KW] = 0.0;
          const int nr = j + 1 + kl;
          const double nv = nr < n ? XR(nr) : 0.0;
#pragma unroll
          for (int r = 0; r <= KW; ++r)
            if (r == kl) win[r] = nv;
        } else {
          // z = U^{-T} b: z_j = (b_j - sum_k U(j-k, j) z_{j-k}) / U(j,j); win[k-1] = z_{j-k}
          double s = XR(j);
#pragma unroll
          for (int k = 1; k <= KW; ++k)
            if (k <= kd && j - k >= 0) s = fma(-R(kd - k, j), win[k - 1], s);
          s = s / R(kd, j);
          x[j] = s;
#pragma unroll
          for (int k = KW; k >= 1; --k) win[k] = win[k - 1];
          win[0] = s;
        }
      }
    }
    __syncthreads();
  }
  // ------------------------------------------------ pass 2: rows in decreasing order
  if (w >= 1) { load_chunk(nch - 1); load_chunk(nch - 2); }
  __syncthreads();
#pragma unroll
  for (int r = 0; r <= KW; ++r) win[r] = 0.0;
  if (trans && active) win[0] = XR(n - 1);
  for (int q = nch - 1; q >= 0; --q) {
    if (w >= 1) load_chunk(q - 2);
    if (active) {
      const int jbeg = q * BCH2;
      for (int j = min(n, (q + 1) * BCH2) - 1; j >= jbeg; --j) {
        if (!trans) {
          // x_j = (y_j - sum_k U(j, j+k) x_{j+k}) / U(j,j); win[k-1] = x_{j+k}
          double s = XR(j);
#pragma unroll
          for (int k = 1; k <= KW; ++k)
            if (k <= kd && j + k < n) s = fma(-R(kd - k, j + k), win[k - 1], s);
          s = s / R(kd, j);
          x[j] = s;
#pragma unroll
          for (int k = KW; k >= 1; --k) win[k] = win[k - 1];
          win[0] = s;
        } else {
          // w_j = z_j - sum_r L(j+r, j) w_{j+r}, then interchange j <-> ipiv[j].
          // win[r] = current value at position j+r; position j+kl becomes final after this step.
          const int lm = min(kl, n - 1 - j);
          double s = win[0];
#pragma unroll
          for (int r = 1; r <= KW; ++r)
            if (r <= lm) s = fma(-R(kd + r, j), win[r], s);
          win[0] = s;
          const int p = pring[j % SL] - j;
          if (p != 0) {
#pragma unroll
            for (int r = 1; r <= KW; ++r)
              if (r == p) { const double tmp = win[0]; win[0] = win[r]; win[r] = tmp; }
          }
          if (j + kl < n) {
            double out = 0.0;
#pragma unroll
            for (int r = 0; r <= KW; ++r)
              if (r == kl) out = win[r];
            x[j + kl] = out;
          }
          if (j > 0) {
#pragma unroll
            for (int r = KW; r >= 1; --r) win[r] = win[r - 1];
            win[0] = XR(j - 1);
          } else {
#pragma unroll
            for (int r = 0; r < KW; ++r)
              if (r < kl && r < n) x[r] = win[r];
          }
        }
      }
    }
    __syncthreads();
  }
}

hipError_t launch_gbtrs(int n, int kl, int ku, int nrhs, const double* GB, int ldgb, const int* ipiv, bool trans,
                        double* X, int ldx, const int* pred, int pred_val, hipStream_t st) {
  const int kd = kl + ku;
  if (nrhs < 1 || kd > BAND_KD_MAX) return hipErrorInvalidValue;
  for (int c0 = 0; c0 < nrhs; c0 += 32) {
    const int nr = nrhs - c0 < 32 ? nrhs - c0 : 32;
    const size_t lds = (size_t)4 * BCH2 * ldgb * sizeof(double) + (size_t)4 * BCH2 * nr * sizeof(double) +
                       (size_t)4 * BCH2 * sizeof(int);
    double* Xc = X + (size_t)c0 * ldx;
#define ADA_GBTRS(K)                                                                                         \
  do {                                                                                                       \
    static size_t done = 0;                                                                                  \
    hipError_t e = ensure_lds((const void*)k_gbtrs<K>, lds, done);                                          \
    if (e != hipSuccess) return e;                                                                           \
    hipLaunchKernelGGL(k_gbtrs<K>, dim3(1), dim3(256), lds, st, n, kl, ku, nr, GB, ldgb, ipiv, (int)trans, Xc, \
                       ldx, pred, pred_val);                                                                 \
  } while (0)
    const int kw = kd > kl ? kd : kl;
    if (kw <= 8) ADA_GBTRS(8);
    else if (kw <= 16) ADA_GBTRS(16);
    else ADA_GBTRS(32);
#undef ADA_GBTRS
  }
  return hipGetLastError();
}

// R = B - A X for band-layout input (AB[ku_in + i - j + j*ldab])
__global__ void k_band_resid(int n, int kl, int ku, int nrhs, const double* __restrict__ AB, int ldab, int ku_in,
                             const double* __restrict__ B, int ldb, const double* __restrict__ X, int ldx,
                             double* __restrict__ R, int ldr) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    for (int c = 0; c < nrhs; ++c) {
      double s = B[(size_t)i + (size_t)c * ldb], e = 0.0;  // accurate residual (Dot2)
      for (int j = max(0, i - kl); j <= min(n - 1, i + ku); ++j)
        dot2_sub(s, e, AB[(size_t)(ku_in + i - j) + (size_t)j * ldab], X[(size_t)j + (size_t)c * ldx]);
      R[(size_t)i + (size_t)c * ldr] = s + e;
    }
  }
}

hipError_t launch_band_resid(int n, int kl, int ku, int nrhs, const double* AB, int ldab, int ku_in,
                             const double* B, int ldb, const double* X, int ldx, double* R, int ldr,
                             hipStream_t st) {
  int blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_band_resid, dim3(blocks), dim3(256), 0, st, n, kl, ku, nrhs, AB, ldab, ku_in, B, ldb, X, ldx,
                     R, ldr);
  return hipGetLastError();
}

}  // namespace ada
