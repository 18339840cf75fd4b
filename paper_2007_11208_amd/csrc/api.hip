// C ABI of libada: argument checks, workspace layout and the host side of the
// adaptive solve (Section II of Sanderson & Curtin): detection pass -> route
// -> condition estimate -> fallback rule -> SVD least squares. The host reads
// the device record twice per solve (after detection, to pick the route, and
// at the end); everything between is stream-ordered device work, with the
// condition estimate's control flow kept on the device.
#include <cfloat>
#include <climits>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ada.h"
#include "ada_internal.h"

using namespace ada;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(ADA_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kNB = 128;          // LU / Cholesky block width
constexpr int kMovesInts = 1 + 2 * 256;  // a panel's row-move list: count, then (destination, source) pairs
constexpr int kDenseMax = 16384;  // dense routes: the panel kernel spreads at most 64 x 256 rows
constexpr int kBandKdMax = 31;    // band kernels: kl + ku
constexpr int kBandDenseMax = 4096;  // band-layout input expanded to dense when needed (not banded / SVD)
constexpr int kJacobiSmall = 256;    // one-workgroup Jacobi up to this n
constexpr int kBandChunkMin = 2 * LC;  // band solves parallel over the rows from this n on
constexpr int kGmresM = 50;             // Krylov dimension of one GMRES correction solve

struct Plan {
  size_t total = 0;
  // offsets (bytes)
  size_t rec, pcol, prow, cld, rld, diag, ctot, csym, rtot, W, V, ipiv, perm, flags, ev, et, exi, recs,
      slot_rows, moves, R, P, percol, T, sigma, Adense, bsc, gb0, gbspec, estpart, Q, tau, gmV, gmW, gmH;
  size_t bsc_doubles, gbspec_doubles;
  int n, nrhs, ldw, T64, nflags;
  bool dense, band, band_dense;
};

size_t take(size_t& cur, size_t bytes) {
  size_t off = align_up(cur, 256);
  cur = off + align_up(bytes, 256);
  return off;
}

bool make_plan(int n, int nrhs, const ada_opts& o, Plan& p) {
  if (n < 1 || nrhs < 1) return false;
  p = Plan();
  p.n = n;
  p.nrhs = nrhs;
  p.band = o.layout == ADA_LAYOUT_BAND;
  p.dense = !p.band || n <= kBandDenseMax;
  p.band_dense = p.band && p.dense;
  const size_t N = (size_t)n;
  p.ldw = n;
  p.T64 = (n + 63) / 64;
  p.nflags = p.T64;
  size_t cur = 0;
  p.rec = take(cur, sizeof(DevRec));
  p.ipiv = take(cur, N * 4);
  p.perm = take(cur, N * 4);
  p.flags = take(cur, (size_t)p.nflags * 4);
  p.ev = take(cur, N * 8);
  p.et = take(cur, N * 8);
  p.exi = take(cur, N * 8);
  p.R = take(cur, N * nrhs * 8);
  p.T = take(cur, N * nrhs * 8);
  p.percol = take(cur, (size_t)nrhs * 8 * 4);
  p.estpart = take(cur, est_part_bytes());
  {
    // scratch of the row-parallel band solves: the band width of band-layout
    // input, the widest band the kernels take otherwise
    const int kd = p.band ? (o.kl_in + o.ku_in) : kBandKdMax;
    p.bsc_doubles = band_chunked_scratch_doubles(n, kd, 0, nrhs);
    p.bsc = take(cur, p.bsc_doubles * 8);
  }
  if (p.dense) p.P = take(cur, resid_partial_doubles(n, nrhs) * 8);
  // W: dense working copy (LU/Cholesky factor, Jacobi U) and/or the band factor (2kl+ku+1 rows)
  size_t wrows = (size_t)n;
  if (p.band) {
    const size_t ldgb = (size_t)(2 * o.kl_in + o.ku_in + 1);
    wrows = p.dense ? (ldgb > N ? ldgb : N) : ldgb;
  }
  p.W = take(cur, wrows * N * 8);
  {
    // band LU: the packed band it reads (the factor goes to W) and the scratch of its chunked form
    const int kl = p.band ? o.kl_in : 8, ku = p.band ? o.ku_in : kBandKdMax - 8;
    const size_t ldgb = (size_t)(2 * kl + ku + 1);
    // the detected widths may be narrower than the stored ones: size for the largest need
    p.gbspec_doubles = 0;
    for (int a = 1; a <= (kl < 8 ? kl : 8); ++a)
      for (int b = 0; b <= ku && a + b <= kBandKdMax; ++b) {
        GbSpecPlan sp = gbtrf_spec_plan(n, a, b);
        const size_t d = sp.nchunks >= 2 ? sp.snap_doubles + sp.exit_doubles : 0;
        if (d > p.gbspec_doubles) p.gbspec_doubles = d;
      }
    p.gbspec = take(cur, p.gbspec_doubles * 8 + 8);
    if (p.band && !p.dense) p.gb0 = take(cur, ldgb * N * 8);
  }
  if (p.dense) {
    const size_t T = (size_t)p.T64;
    p.pcol = take(cur, T * N * 8);
    p.prow = take(cur, T * N * 8);
    p.cld = take(cur, N * 8);
    p.rld = take(cur, N * 8);
    p.diag = take(cur, N * 8);
    p.ctot = take(cur, N * 8);
    p.csym = take(cur, N * 8);
    p.rtot = take(cur, N * 8);
    p.V = take(cur, (N > 64 ? N : 64) * N * 8);
    if (!(p.band && !p.dense)) p.gb0 = p.V;  // the Jacobi V is not in use on the band route
    p.sigma = take(cur, N * 8);
    p.Q = take(cur, N * N * 8);  // Householder reflectors of the SVD route's QR preconditioner
    p.tau = take(cur, N * 8);
    p.recs = take(cur, 2 * 64 * 2 * 8);
    p.slot_rows = take(cur, (size_t)2 * 64 * 128 * 8);
    p.moves = take(cur, 2 * kMovesInts * 4);
    if (p.band) p.Adense = take(cur, N * N * 8);  // dense expansion of band-layout input
    if (o.precision == ADA_PREC_BF16_IR) {
      // GMRES correction solves: the Krylov bases of every right-hand side, the work vectors, the
      // Arnoldi coefficients (two Gram-Schmidt passes and the norm) and the combination weights
      p.gmV = take(cur, (size_t)(kGmresM + 1) * N * nrhs * 8);
      p.gmW = take(cur, N * nrhs * 8);
      p.gmH = take(cur, (size_t)(3 * (kGmresM + 2)) * nrhs * 8);
    }
  }
  p.total = cur + 256;
  return true;
}

ada_opts defaults() {
  ada_opts o;
  memset(&o, 0, sizeof(o));
  o.struct_size = sizeof(ada_opts);
  o.rcond_threshold = -1.0;
  o.layout = ADA_LAYOUT_DENSE;
  o.want_berr = 1;
  return o;
}

bool read_opts(const ada_opts* in, ada_opts& o) {
  o = defaults();
  if (!in) return true;
  if (in->struct_size < sizeof(uint32_t) || in->struct_size > sizeof(ada_opts)) return false;
  memcpy(&o, in, in->struct_size);
  return true;
}

int ilog2(int n) {
  int b = 0;
  while (b < 31 && (2LL << b) <= n) ++b;
  return b;
}

bool is_banded(int64_t n, int64_t kl, int64_t ku) {
  const int64_t nnz = n * (kl + ku + 1) - kl * (kl + 1) / 2 - ku * (ku + 1) / 2;
  return 4 * nnz <= n * n;
}

double bits_to_double(unsigned long long b) {
  double d;
  memcpy(&d, &b, 8);
  return d;
}

}  // namespace

struct ada_ctx_s {
  int device = 0;
  DevRec* host_rec = nullptr;  // pinned
  std::mutex mu;
  // look-ahead: the bulk of each trailing update runs on a second stream while
  // the next panel / diagonal block is factored (fork and join by events)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // per-family launch timing (instrumentation)
  bool prof = false;
  unsigned prof_mask = ~0u;  // kernel families timed while prof is on
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  struct Pending {
    int kind;
    double flops, bytes;
    size_t e0, e1;
  };
  std::vector<Pending> pending;
  struct Acc {
    int64_t launches = 0;
    double ms = 0.0, flops = 0.0, bytes = 0.0;
  } acc[ADA_KF_COUNT];
  // autotuned LDS staging piece of the row-parallel band solve, by kl + ku, one / several right-hand
  // sides and floor(log2 n) (the best piece depends on how many chunks compete for the compute units);
  // 0 = the built-in choice
  int band_piece[32][2][32] = {};
  // device address of this GPU's fixed scratch of ada_solve_noalloc (from hipGetSymbolAddress)
  void* noalloc_scratch = nullptr;
  // set during ada_solve_noalloc: instrumentation records events only from the existing pool
  bool no_grow = false;
  // launch shape of the batched solve, by precision (0: FP64, 1: FP32 factors with FP64 refinement)
  ada_batched_shape bshape[2] = {ada::batched_default_shape(), ada::batched_default_shape()};
};

namespace {

// Everything one solve needs on the host side.
struct Solve {
  ada_ctx ctx;
  hipStream_t st;
  Plan p;
  char* base;
  DevRec* rec;
  int n, nrhs;
  int counter_idx = 0;
  int epoch = 0;
  int lowp = ADA_PREC_FP64;  // operand precision of the trailing-matrix updates
  bool keep_factors = false; // the factors left in the workspace serve later right-hand sides
  unsigned band_maps = 0;     // sweep kinds whose chunk maps the current band factor already has

  template <class T>
  T* at(size_t off) const { return reinterpret_cast<T*>(base + off); }
  unsigned* next_counter() {
    if (counter_idx >= 512) return nullptr;
    return &rec->counters[counter_idx++];
  }
  // index of a recorded event in the pool, or -1 (profiling off / no event)
  long ev_record(hipStream_t on) {
    if (!ctx->prof) return -1;
    if (ctx->ev_used >= ctx->ev_pool.size()) {
      if (ctx->no_grow) return -1;
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return -1;
      ctx->ev_pool.push_back(e);
    }
    if (hipEventRecord(ctx->ev_pool[ctx->ev_used], on) != hipSuccess) return -1;
    return (long)ctx->ev_used++;
  }
  // run `launch` (returns hipError_t); when profiling, bracket it with events of family `kind` on stream `on`
  template <class F>
  hipError_t timed(int kind, double flops, double bytes, F&& launch, hipStream_t on = nullptr) {
    if (kind < 0 || !ctx->prof || !((ctx->prof_mask >> kind) & 1u)) return launch();
    if (!on) on = st;
    const long e0 = ev_record(on);
    const hipError_t e = launch();
    const long e1 = ev_record(on);
    if (e0 >= 0 && e1 >= 0) ctx->pending.push_back({kind, flops, bytes, (size_t)e0, (size_t)e1});
    return e;
  }
  int gemm(int m, int nn, int k, const double* A, int lda, const double* B, int ldb, bool transB, double* C, int ldc,
           bool lower, hipStream_t on = nullptr) {
    if (!on) on = st;
    // algorithmic flops: the lower triangle only for the symmetric update
    const double fl = lower ? 2.0 * (double)k * ((double)m * (m + 1) / 2.0) : 2.0 * (double)m * nn * k;
    const double by = 8.0 * ((double)m * k + (double)nn * k + 2.0 * (lower ? (double)m * (m + 1) / 2.0 : (double)m * nn));
    HIPCHK(timed(ADA_KF_GEMM, fl, by, [&] {
      if (lowp != ADA_PREC_FP64)
        return launch_gemm_sub_lp(lowp, m, nn, k, A, lda, B, ldb, transB, C, ldc, lower, &rec->stop, on);
      return launch_gemm_sub(m, nn, k, A, lda, B, ldb, transB, C, ldc, lower, &rec->stop, on, nullptr, nullptr);
    }, on));
    return ADA_OK;
  }
  // the side stream starts after everything enqueued on st so far
  int fork() {
    HIPCHK(hipEventRecord(ctx->ev_fork, st));
    HIPCHK(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0));
    return ADA_OK;
  }
  // st continues after everything enqueued on the side stream so far
  int join() {
    HIPCHK(hipEventRecord(ctx->ev_join, ctx->side));
    HIPCHK(hipStreamWaitEvent(st, ctx->ev_join, 0));
    return ADA_OK;
  }
  // op(T) X = X, nrhs <= 64 per launch (split otherwise)
  int trsm(const double* T, int ldt, bool lower, bool trans, bool unit, double* X, int ldx, int nr, const int* pred,
           int pv) {
    for (int c0 = 0; c0 < nr; c0 += 64) {
      const int cnt = nr - c0 < 64 ? nr - c0 : 64;
      unsigned* tk = next_counter();
      if (!tk) return fail(ADA_ERR_ARG, "too many device synchronisation counters for this size");
      const double nn = (double)n;
      const int ep = ++epoch;
      // estimator solves are predicated on the estimator's state (some do not run): not timed
      const int kind = pred == &rec->est_phase ? -1 : ADA_KF_TRSV;
      HIPCHK(timed(kind, nn * nn * cnt, 8.0 * (nn * (nn + 1) / 2.0 + 2.0 * nn * cnt), [&] {
        return launch_trsm_dec(n, cnt, T, ldt, lower, trans, unit, X + (size_t)c0 * ldx, ldx, at<int>(p.flags), ep,
                               tk, rec, pred, pv, st);
      }));
    }
    return ADA_OK;
  }
  int sync_read() {
    HIPCHK(hipMemcpyAsync(ctx->host_rec, rec, sizeof(DevRec), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return ADA_OK;
  }
};

#define TRY(expr)               \
  do {                          \
    int r_ = (expr);            \
    if (r_ != ADA_OK) return r_; \
  } while (0)

// ---------------------------------------------------------------- routes
// Each route leaves X = the routed solution (when the factorisation succeeded),
// rec->info / rec->stop, rec->anorm1, and runs the condition estimate.

// op(A) X = X with the band LU in GB (in place; T: n x nrhs scratch)
int band_solve(Solve& s, const double* GB, int kl, int ku, bool trans, double* X, int ldx, int nrhs, double* T,
               int ldt, const int* pred, int pred_val) {
  const int n = s.n, ldgb = 2 * kl + ku + 1;
  const int* ipiv = s.at<int>(s.p.ipiv);
  // algorithmic: 2 flops per factor entry (kl of L, kl+ku+1 of U per column) per right-hand side;
  // reads the factor rows and pivots, reads and writes X
  const double nn = (double)n, fe = nn * (2.0 * kl + ku + 1);
  const double fl = 2.0 * fe * nrhs, by = 8.0 * fe + 4.0 * nn + 16.0 * nn * nrhs;
  const int kind = pred == &s.rec->est_phase ? -1 : ADA_KF_GBTRS;
  if (n >= kBandChunkMin) {
    if (band_chunked_scratch_doubles(n, kl, ku, nrhs) > s.p.bsc_doubles)
      return fail(ADA_ERR_ARG, "band scratch smaller than the band width needs");
    BandScratch sc = band_chunked_scratch(s.at<double>(s.p.bsc), n, kl, ku, nrhs);
    HIPCHK(s.timed(kind, fl, by, [&] {
      return launch_gbtrs_chunked(n, kl, ku, nrhs, GB, ldgb, ipiv, trans, X, ldx, T, ldt, sc, pred, pred_val,
                                  &s.rec->stop, 0, &s.band_maps, s.ctx->band_piece[kl + ku][nrhs > 1 ? 1 : 0][ilog2(n)],
                                  s.st);
    }));
  } else {
    HIPCHK(s.timed(kind, fl, by, [&] {
      return launch_gbtrs(n, kl, ku, nrhs, GB, ldgb, ipiv, trans, X, ldx, pred, pred_val, s.st);
    }));
  }
  return ADA_OK;
}

int estimate(Solve& s, int route_kind, const double* F, int ldf, bool tri_lower, int kl, int ku) {
  // route_kind: 0 LU (F = LU, perm), 1 Cholesky (F = L), 2 triangular (F = A), 3 band (F = GB),
  // 4 LDL^T (F = L, perm, D)
  const int n = s.n;
  double* v = s.at<double>(s.p.ev);
  double* t = s.at<double>(s.p.et);
  double* xi = s.at<double>(s.p.exi);
  int* phase = &s.rec->est_phase;
  HIPCHK(launch_est_init(n, v, s.rec, s.st));
  for (int slot = 0; slot < 11; ++slot) {
    const int type = (slot % 2 == 0) ? 1 : 2;
    const double* result = v;
    if (route_kind == 0) {
      const int* perm = s.at<int>(s.p.perm);
      if (type == 1) {
        HIPCHK(launch_gather_rows(n, 1, perm, v, n, t, n, phase, 1, s.st));
        TRY(s.trsm(F, ldf, true, false, true, t, n, 1, phase, 1));
        TRY(s.trsm(F, ldf, false, false, false, t, n, 1, phase, 1));
      } else {
        TRY(s.trsm(F, ldf, false, true, false, v, n, 1, phase, 2));
        TRY(s.trsm(F, ldf, true, true, true, v, n, 1, phase, 2));
        HIPCHK(launch_scatter_rows(n, 1, perm, v, n, t, n, phase, 2, s.st));
      }
      result = t;
    } else if (route_kind == 1) {
      TRY(s.trsm(F, ldf, true, false, false, v, n, 1, phase, type));
      TRY(s.trsm(F, ldf, true, true, false, v, n, 1, phase, type));
    } else if (route_kind == 2) {
      TRY(s.trsm(F, ldf, tri_lower, type == 2, false, v, n, 1, phase, type));
    } else if (route_kind == 4) {
      // inv(A) is symmetric: both directions are the same solve
      const int* perm = s.at<int>(s.p.perm);
      HIPCHK(launch_gather_rows(n, 1, perm, v, n, t, n, phase, type, s.st));
      TRY(s.trsm(F, ldf, true, false, true, t, n, 1, phase, type));
      HIPCHK(launch_ldlt_dsolve(n, 1, s.at<double>(s.p.tau), s.at<double>(s.p.sigma), t, n, phase, type, s.st));
      TRY(s.trsm(F, ldf, true, true, true, t, n, 1, phase, type));
      HIPCHK(launch_scatter_rows(n, 1, perm, t, n, v, n, phase, type, s.st));
    } else {
      TRY(band_solve(s, F, kl, ku, type == 2, v, n, 1, t, n, phase, type));
    }
    unsigned* ctr = s.next_counter();
    if (!ctr) return fail(ADA_ERR_ARG, "too many device synchronisation counters for this size");
    HIPCHK(launch_est_step(n, type, slot + 1, result, v, xi, s.rec, s.at<char>(s.p.estpart), ctr, s.st));
  }
  HIPCHK(launch_finalize_rcond(s.rec, s.st));
  return ADA_OK;
}

int route_lu(Solve& s, const double* A, int lda, const double* B, int ldb, double* X, int ldx) {
  const int n = s.n, ldw = s.p.ldw;
  double* W = s.at<double>(s.p.W);
  int* ipiv = s.at<int>(s.p.ipiv);
  int* perm = s.at<int>(s.p.perm);
  HIPCHK(launch_copy(n, n, A, lda, W, ldw, s.st));
  HIPCHK(launch_iota(perm, n, s.st));
  PanelScratch ps{s.at<unsigned long long>(s.p.recs), s.at<double>(s.p.slot_rows),
                  s.at<int>(s.p.moves)};
  HIPCHK(launch_panel_reset(ps, s.st));
  // look-ahead: after panel k, only the next block column takes its interchanges, its block row of U
  // and its trailing update on st, ahead of panel k+1; the interchanges, the block row of U and the
  // trailing update of every other column go on the side stream alongside panel k+1 (disjoint
  // columns), which st joins after panel k+1. The panels' row-move lists alternate between two
  // buffers, so that panel k+1 does not overwrite the list the side stream is still reading.
  bool pending = false;
  int kb = 0;
  for (int k0 = 0; k0 < n; k0 += kNB, ++kb) {
    const int nbw = n - k0 < kNB ? n - k0 : kNB;
    const double m = (double)(n - k0), b = (double)nbw;
    PanelScratch pk = ps;
    pk.moves = ps.moves + (kb & 1) * kMovesInts;
    // panel: sum over its columns s of 2 (m - s - 1)(b - s - 1) + (m - s - 1); reads and writes m x b
    const double pfl = b * (b - 1) * (3.0 * m - b - 1) / 3.0 + b * m - b * (b + 1) / 2.0;
    HIPCHK(s.timed(ADA_KF_PANEL, pfl, 16.0 * m * b,
                   [&] { return launch_getrf_panel(n, k0, nbw, W, ldw, ipiv, s.rec, pk, s.st); }));
    if (pending) TRY(s.join());
    pending = false;
    const int rest = n - k0 - nbw;
    const int nb2 = rest < kNB ? rest : kNB;
    const int c1 = k0 + nbw, c2 = c1 + nb2;  // the next block column: [c1, c2)
    const double* L21 = W + c1 + (size_t)k0 * ldw;
    if (rest == 0) {
      // last panel: only the permutation takes the moves
      HIPCHK(s.timed(ADA_KF_LASWP, 0.0, 0.0, [&] {
        return launch_laswp_moves(c1, c2, 0, 0, true, W, ldw, pk.moves, perm, s.rec, s.st);
      }));
    } else {
      // the next block column's interchanges and its block row of U in one launch
      HIPCHK(s.timed(ADA_KF_TRSM_BLOCK, b * b * nb2, 8.0 * (b * b / 2.0 + 2.0 * b * nb2) + 32.0 * b * nb2, [&] {
        return launch_swap_trsm_llnu(k0, nbw, nb2, W, ldw, pk.moves, perm, s.rec, s.st);
      }));
      TRY(s.gemm(rest, nb2, nbw, L21, ldw, W + k0 + (size_t)c1 * ldw, ldw, false, W + c1 + (size_t)c1 * ldw, ldw,
                 false));
    }
    TRY(s.fork());
    HIPCHK(s.timed(ADA_KF_LASWP, 0.0, 32.0 * b * (n - nbw - nb2), [&] {
      return launch_laswp_moves(0, k0, c2, n, false, W, ldw, pk.moves, perm, s.rec, s.ctx->side);
    }, s.ctx->side));
    pending = true;
    if (rest > 0) {
      if (rest > nb2) {
        const double r2 = (double)(rest - nb2);
        HIPCHK(s.timed(ADA_KF_TRSM_BLOCK, b * b * r2, 8.0 * (b * b / 2.0 + 2.0 * b * r2), [&] {
          return launch_trsm_llnu(k0, nbw, nb2, rest - nb2, W, ldw, s.rec, s.ctx->side);
        }, s.ctx->side));
        TRY(s.gemm(rest, rest - nb2, nbw, L21, ldw, W + k0 + (size_t)c2 * ldw, ldw, false,
                   W + c1 + (size_t)c2 * ldw, ldw, false, s.ctx->side));
      }
    }
  }
  if (pending) TRY(s.join());
  // X = U^{-1} L^{-1} P B
  int* stop = &s.rec->stop;
  HIPCHK(launch_gather_rows(n, s.nrhs, perm, B, ldb, X, ldx, stop, 0, s.st));
  TRY(s.trsm(W, ldw, true, false, true, X, ldx, s.nrhs, stop, 0));
  TRY(s.trsm(W, ldw, false, false, false, X, ldx, s.nrhs, stop, 0));
  return estimate(s, 0, W, ldw, false, 0, 0);
}

int route_chol(Solve& s, const double* A, int lda, const double* B, int ldb, double* X, int ldx) {
  const int n = s.n, ldw = s.p.ldw;
  double* W = s.at<double>(s.p.W);
  HIPCHK(launch_copy(n, n, A, lda, W, ldw, s.st));
  // look-ahead: the update of the next block column runs on st ahead of its diagonal block, the rest
  // of the trailing triangle on the side stream alongside the next diagonal block and its column
  bool pending = false;
  for (int k0 = 0; k0 < n; k0 += kNB) {
    const int nbw = n - k0 < kNB ? n - k0 : kNB;
    const double b = (double)nbw;
    HIPCHK(s.timed(ADA_KF_POTRF, b * b * b / 3.0, 8.0 * b * b,
                   [&] { return launch_potrf_diag(k0, nbw, W, ldw, s.rec, s.st); }));
    const int rest = n - k0 - nbw;
    if (rest > 0) {
      HIPCHK(s.timed(ADA_KF_TRSM_BLOCK, b * b * rest, 8.0 * (b * b / 2.0 + 2.0 * b * rest),
                     [&] { return launch_trsm_rltn(k0, nbw, rest, W, ldw, s.rec, s.st); }));
      if (pending) TRY(s.join());
      pending = false;
      const double* L21 = W + (k0 + nbw) + (size_t)k0 * ldw;
      double* A22 = W + (k0 + nbw) + (size_t)(k0 + nbw) * ldw;
      const int nb2 = rest < kNB ? rest : kNB;
      // next block column (all rows below, rectangular; its upper part is never read)
      TRY(s.gemm(rest, nb2, nbw, L21, ldw, L21, ldw, true, A22, ldw, false));
      if (rest > nb2) {
        TRY(s.fork());
        TRY(s.gemm(rest - nb2, rest - nb2, nbw, L21 + nb2, ldw, L21 + nb2, ldw, true,
                   A22 + nb2 + (size_t)nb2 * ldw, ldw, true, s.ctx->side));
        pending = true;
      }
    }
  }
  if (pending) TRY(s.join());
  int* stop = &s.rec->stop;
  HIPCHK(launch_copy(n, s.nrhs, B, ldb, X, ldx, s.st));
  TRY(s.trsm(W, ldw, true, false, false, X, ldx, s.nrhs, stop, 0));
  TRY(s.trsm(W, ldw, true, true, false, X, ldx, s.nrhs, stop, 0));
  return estimate(s, 1, W, ldw, false, 0, 0);
}

int route_tri(Solve& s, const double* A, int lda, bool lower, const double* B, int ldb, double* X, int ldx) {
  int* stop = &s.rec->stop;
  HIPCHK(launch_copy(s.n, s.nrhs, B, ldb, X, ldx, s.st));
  TRY(s.trsm(A, lda, lower, false, false, X, ldx, s.nrhs, stop, 0));
  return estimate(s, 2, A, lda, lower, 0, 0);
}

constexpr int kSyPanel = 16;  // LDL^T panel width (panels start every kSyPanel - 1 columns)

// Symmetric indefinite route (Section V future work): Bunch-Kaufman LDL^T. Panels start at fixed
// positions every kSyPanel - 1 columns; whether a 2x2 pivot crossed a panel edge is decided and read
// on the device, so the host enqueues the whole factorisation and reads the record once at the end.
int route_ldlt(Solve& s, const double* A, int lda, const double* B, int ldb, double* X, int ldx) {
  const int n = s.n, ldw = s.p.ldw, b = kSyPanel;
  double* W = s.at<double>(s.p.W);
  double* Wp = s.at<double>(s.p.V);
  int* swp = s.at<int>(s.p.ipiv);
  int* perm = s.at<int>(s.p.perm);
  double* d = s.at<double>(s.p.tau);
  double* e = s.at<double>(s.p.sigma);
  HIPCHK(launch_copy(n, n, A, lda, W, ldw, s.st));
  HIPCHK(launch_iota(perm, n, s.st));
  DevRec& h = *s.ctx->host_rec;
  for (int k0 = 0; k0 < n; k0 += b - 1) {
    const double m = (double)(n - k0), bb = (double)(b < n - k0 ? b : n - k0);
    // delayed updates of the panel's columns: sum over its columns of 2 m c flops; reads m x b twice
    HIPCHK(s.timed(ADA_KF_PANEL, m * bb * bb, 16.0 * m * bb, [&] {
      return launch_sytrf_panel(n, k0, b, W, ldw, Wp, n, swp, d, e, s.rec, s.st);
    }));
    HIPCHK(launch_ldlt_swap_left(n, k0, W, ldw, swp, perm, s.rec, s.st));
    const int rest = n - k0 - b;
    if (rest <= 0) break;
    const double* L21 = W + (k0 + b) + (size_t)k0 * ldw;
    const double* W21 = Wp + (k0 + b);
    double* A22 = W + (k0 + b) + (size_t)(k0 + b) * ldw;
    TRY(s.gemm(rest, rest, b, L21, ldw, W21, n, true, A22, ldw, true));
  }
  TRY(s.sync_read());
  if (h.info != INT_MAX) {
    HIPCHK(launch_mark_stop(s.rec, s.st));
    return ADA_OK;
  }
  // X = P^T L^{-T} D^{-1} L^{-1} P B
  int* stop = &s.rec->stop;
  double* T = s.at<double>(s.p.T);
  HIPCHK(launch_gather_rows(n, s.nrhs, perm, B, ldb, T, n, stop, 0, s.st));
  TRY(s.trsm(W, ldw, true, false, true, T, n, s.nrhs, stop, 0));
  HIPCHK(launch_ldlt_dsolve(n, s.nrhs, d, e, T, n, stop, 0, s.st));
  TRY(s.trsm(W, ldw, true, true, true, T, n, s.nrhs, stop, 0));
  HIPCHK(launch_scatter_rows(n, s.nrhs, perm, T, n, X, ldx, stop, 0, s.st));
  return estimate(s, 4, W, ldw, false, 0, 0);
}

int route_band(Solve& s, const double* GB0, double* GB, int kl, int ku, const double* B, int ldb, double* X,
               int ldx) {
  // GB0: the packed band (its norms already recorded); the factor goes to GB
  const int n = s.n, ldgb = 2 * kl + ku + 1;
  s.band_maps = 0;  // a new factor: its chunk maps are formed at the first solve of each kind
  {
    // algorithmic: per column kl multipliers and a kl x (kl + ku) update; reads the kl+ku+1 band rows,
    // writes the 2kl+ku+1 factor rows and the pivots
    const double nn = (double)n;
    const double fl = nn * ((double)kl + 2.0 * kl * (kl + ku));
    const double by = 8.0 * nn * (kl + ku + 1) + 8.0 * nn * ldgb + 4.0 * nn;
    HIPCHK(s.timed(ADA_KF_GBTRF, fl, by, [&] {
      return launch_gbtrf(n, kl, ku, GB0, GB, ldgb, s.at<int>(s.p.ipiv), s.rec, s.at<double>(s.p.gbspec),
                          s.p.gbspec_doubles, s.st);
    }));
  }
  int* stop = &s.rec->stop;
  HIPCHK(launch_copy(n, s.nrhs, B, ldb, X, ldx, s.st));
  TRY(band_solve(s, GB, kl, ku, false, X, ldx, s.nrhs, s.at<double>(s.p.T), n, stop, 0));
  return estimate(s, 3, GB, ldgb, false, kl, ku);
}

int route_svd(Solve& s, const double* A, int lda, const double* B, int ldb, double* X, int ldx, double* Wbuf,
              double* Vbuf, double* Tbuf) {
  // W (the accumulated rotations) is kept only when the factors serve later right-hand sides; otherwise the
  // rotations go to the projections C = Q^T B directly (half the Jacobi's memory traffic)
  const bool keep_w = s.keep_factors;
  const int n = s.n;
  // A P = Q R (columns by decreasing norm); C = Q^T B (in R's slot: the residual is formed after the solve);
  // one-sided Jacobi on R^T, each rotation applied to W (started at I) or to the rows of C
  double* Q = s.at<double>(s.p.Q);
  double* tau = s.at<double>(s.p.tau);
  double* C = s.at<double>(s.p.R);
  int* perm = s.at<int>(s.p.perm);
  HIPCHK(launch_order_columns(n, A, lda, s.at<double>(s.p.sigma), perm, Q, n, s.st));
  HIPCHK(launch_copy(n, s.nrhs, B, ldb, C, n, s.st));
  HIPCHK(launch_house_qr(n, Q, n, tau, C, n, s.nrhs, s.st));
  HIPCHK(launch_rt(n, Q, n, Wbuf, n, s.st));
  if (keep_w) HIPCHK(launch_set_identity(n, Vbuf, n, s.st));
  double* V = keep_w ? Vbuf : nullptr;
  double* Y = keep_w ? nullptr : C;
  const int ny = keep_w ? 0 : s.nrhs;
  if (n <= kJacobiSmall) {
    HIPCHK(launch_jacobi_small(n, Wbuf, n, V, n, Y, n, ny, 30, s.rec, s.st));
  } else if (!keep_w && jacobi_blocked_fits(n, ny)) {
    // blocks of four columns: one intra-block step and a round-robin over block pairs per sweep
    const int nblk = (n + 3) / 4, nbm = (nblk + 1) & ~1;
    int sweeps = 0;
    for (; sweeps < 30; ++sweeps) {
      HIPCHK(launch_clear_rotated(s.rec, s.st));
      HIPCHK(launch_jacobi_blk(n, 0, true, Wbuf, n, Y, n, ny, s.rec, s.st));
      for (int r = 0; r < nbm - 1; ++r) HIPCHK(launch_jacobi_blk(n, r, false, Wbuf, n, Y, n, ny, s.rec, s.st));
      TRY(s.sync_read());
      if (!s.ctx->host_rec->jacobi_rotated) { ++sweeps; break; }
    }
    s.ctx->host_rec->sweeps = sweeps;
    HIPCHK(hipMemcpyAsync(&s.rec->sweeps, &s.ctx->host_rec->sweeps, sizeof(int), hipMemcpyHostToDevice, s.st));
  } else {
    const int m = (n + 1) & ~1;
    int sweeps = 0;
    for (; sweeps < 30; ++sweeps) {
      HIPCHK(launch_clear_rotated(s.rec, s.st));
      for (int r = 0; r < m - 1; ++r) HIPCHK(launch_jacobi_round(n, m, r, Wbuf, n, V, n, Y, n, ny, s.rec, s.st));
      TRY(s.sync_read());
      if (!s.ctx->host_rec->jacobi_rotated) { ++sweeps; break; }
    }
    s.ctx->host_rec->sweeps = sweeps;
    HIPCHK(hipMemcpyAsync(&s.rec->sweeps, &s.ctx->host_rec->sweeps, sizeof(int), hipMemcpyHostToDevice, s.st));
  }
  HIPCHK(launch_svd_apply(n, s.nrhs, Wbuf, n, V, n, C, n, X, ldx, perm, s.at<double>(s.p.sigma), Tbuf, s.rec,
                          s.st));
  return ADA_OK;
}

int backward_error_dense(Solve& s, const double* A, int lda, const double* B, int ldb, const double* X, int ldx) {
  const int n = s.n, nrhs = s.nrhs;
  double* R = s.at<double>(s.p.R);
  HIPCHK(launch_resid_gemv(n, nrhs, A, lda, B, ldb, X, ldx, R, n, s.at<double>(s.p.P), s.st));
  HIPCHK(launch_berr(n, nrhs, R, n, B, ldb, X, ldx, s.at<double>(s.p.percol), s.rec, s.st));
  return ADA_OK;
}

constexpr int kMaxRefine = 30;  // refinement steps at most (as LAPACK's mixed-precision drivers)
// low-precision factors with a smaller rcond estimate are not refined (kappa_1 * u_FP32 > 50; the BF16
// factors are refined by GMRES, whose reach does not end at kappa_1 * u_BF16 = 1)
constexpr double kRcondRefine = 1e-9;

// FP64 iterative refinement of X with the factors in W (chol: L of the Cholesky route; else the LU
// route's LU and row permutation): r = B - A X, stop when the backward error of every column is at
// most sqrt(n) eps (converged) or has not halved since the last step, or after kMaxRefine steps;
// otherwise X += solve(r). On return rec->berr is the backward error of X.
int refine(Solve& s, bool chol, const double* A, int lda, const double* B, int ldb, double* X, int ldx, bool& conv,
           int& steps) {
  const int n = s.n, nrhs = s.nrhs, ldw = s.p.ldw;
  const double tol = std::sqrt((double)n) * DBL_EPSILON;
  double* R = s.at<double>(s.p.R);
  double* T = s.at<double>(s.p.T);
  const double* W = s.at<double>(s.p.W);
  const int* perm = s.at<int>(s.p.perm);
  int* stop = &s.rec->stop;
  double prev = INFINITY;
  conv = false;
  for (steps = 0;; ++steps) {
    TRY(backward_error_dense(s, A, lda, B, ldb, X, ldx));
    TRY(s.sync_read());
    const double eta = s.ctx->host_rec->berr;
    if (eta <= tol) {
      conv = true;
      return ADA_OK;
    }
    if (!(eta <= 0.5 * prev) || steps == kMaxRefine) return ADA_OK;
    prev = eta;
    if (chol) {
      TRY(s.trsm(W, ldw, true, false, false, R, n, nrhs, stop, 0));
      TRY(s.trsm(W, ldw, true, true, false, R, n, nrhs, stop, 0));
      HIPCHK(launch_add_to(n, nrhs, R, n, X, ldx, s.st));
    } else {
      HIPCHK(launch_gather_rows(n, nrhs, perm, R, n, T, n, stop, 0, s.st));
      TRY(s.trsm(W, ldw, true, false, true, T, n, nrhs, stop, 0));
      TRY(s.trsm(W, ldw, false, false, false, T, n, nrhs, stop, 0));
      HIPCHK(launch_add_to(n, nrhs, T, n, X, ldx, s.st));
    }
  }
}

// D = M^{-1} S with the low-precision factors in W (the preconditioner of the GMRES correction solves):
// Cholesky: L L^T; LU: the row permutation, then L (unit) and U
int precondition(Solve& s, bool chol, const double* S, int lds, double* D) {
  const int n = s.n, nrhs = s.nrhs, ldw = s.p.ldw;
  const double* W = s.at<double>(s.p.W);
  int* stop = &s.rec->stop;
  if (chol) {
    HIPCHK(launch_copy(n, nrhs, S, lds, D, n, s.st));
    TRY(s.trsm(W, ldw, true, false, false, D, n, nrhs, stop, 0));
    TRY(s.trsm(W, ldw, true, true, false, D, n, nrhs, stop, 0));
  } else {
    HIPCHK(launch_gather_rows(n, nrhs, s.at<int>(s.p.perm), S, lds, D, n, stop, 0, s.st));
    TRY(s.trsm(W, ldw, true, false, true, D, n, nrhs, stop, 0));
    TRY(s.trsm(W, ldw, false, false, false, D, n, nrhs, stop, 0));
  }
  return ADA_OK;
}

// Iterative refinement whose correction equation A d = r is solved by GMRES preconditioned with the
// low-precision factors (left preconditioning, M^{-1} A d = M^{-1} r), every right-hand side with its own
// Krylov basis: Arnoldi with two classical Gram-Schmidt passes, the small least-squares problems by Givens
// rotations on the host, at most kGmresM steps or until the preconditioned residual of every column has
// dropped by kGmresTol; x += V y. The outer loop and its stopping rules are those of refine(). This is the
// refinement of the BF16 factors, whose error is too large for the plain correction x += M^{-1} r.
constexpr double kGmresTol = 1e-10;
int refine_gmres(Solve& s, bool chol, const double* A, int lda, const double* B, int ldb, double* X, int ldx,
                 bool& conv, int& steps) {
  const int n = s.n, nrhs = s.nrhs, m = kGmresM, ldh = kGmresM + 2;
  const double tol = std::sqrt((double)n) * DBL_EPSILON;
  double* R = s.at<double>(s.p.R);
  double* T = s.at<double>(s.p.T);
  double* V = s.at<double>(s.p.gmV);
  double* Wv = s.at<double>(s.p.gmW);
  double* H1 = s.at<double>(s.p.gmH);       // ldh x nrhs
  double* H2 = H1 + (size_t)ldh * nrhs;     // ldh x nrhs
  double* H3 = H2 + (size_t)ldh * nrhs;     // norms, then the weights y
  const size_t vs = (size_t)n * nrhs;
  const int cbase = s.counter_idx;  // the synchronisation counters the corrections reuse
  std::vector<double> h1((size_t)ldh * nrhs), h2((size_t)ldh * nrhs), h3((size_t)ldh * nrhs);
  std::vector<double> Hh((size_t)(m + 1) * m * nrhs), cs((size_t)m * nrhs), sn((size_t)m * nrhs),
      g((size_t)(m + 1) * nrhs), beta(nrhs), y((size_t)ldh * nrhs);
  auto fetch = [&](const double* d, std::vector<double>& hv, size_t cnt) -> int {
    HIPCHK(hipMemcpyAsync(hv.data(), d, cnt * sizeof(double), hipMemcpyDeviceToHost, s.st));
    HIPCHK(hipStreamSynchronize(s.st));
    return ADA_OK;
  };
  double prev = INFINITY;
  conv = false;
  for (steps = 0;; ++steps) {
    TRY(backward_error_dense(s, A, lda, B, ldb, X, ldx));
    TRY(s.sync_read());
    const double eta = s.ctx->host_rec->berr;
    if (eta <= tol) {
      conv = true;
      return ADA_OK;
    }
    if (!(eta <= 0.5 * prev) || steps == kMaxRefine) return ADA_OK;
    prev = eta;
    if (s.counter_idx > cbase) {  // the kernels that used them have completed (the stream was synchronised)
      HIPCHK(hipMemsetAsync(&s.rec->counters[cbase], 0, sizeof(unsigned) * (s.counter_idx - cbase), s.st));
      s.counter_idx = cbase;
    }
    // z0 = M^{-1} r, beta = ||z0||, V_0 = z0 / beta
    TRY(precondition(s, chol, R, n, T));
    HIPCHK(launch_col_dots(n, nrhs, 1, T, 0, T, n, H3, 1, s.st));
    HIPCHK(launch_col_normalize(n, nrhs, T, n, H3, 1, 1.0, V, n, s.st));
    TRY(fetch(H3, h3, nrhs));
    for (int j = 0; j < nrhs; ++j) {
      beta[j] = std::sqrt(h3[j]);
      g[(size_t)j * (m + 1)] = beta[j];
      for (int i = 1; i <= m; ++i) g[(size_t)j * (m + 1) + i] = 0.0;
    }
    int kd = 0;  // Arnoldi steps taken
    for (int k = 0; k < m; ++k) {
      // T = -M^{-1} A V_k (the MFMA update subtracts A V_k from zero)
      HIPCHK(hipMemsetAsync(Wv, 0, vs * sizeof(double), s.st));
      HIPCHK(launch_gemm_sub(n, nrhs, n, A, lda, V + (size_t)k * vs, n, false, Wv, n, false, nullptr, s.st, nullptr,
                             nullptr));
      TRY(precondition(s, chol, Wv, n, T));
      // two Gram-Schmidt passes against V_0..V_k (on -w: h = -(H1 + H2)), the norm, V_{k+1} = w / ||w||
      HIPCHK(launch_col_dots(n, nrhs, k + 1, V, vs, T, n, H1, ldh, s.st));
      HIPCHK(launch_col_axpy(n, nrhs, k + 1, V, vs, H1, ldh, -1.0, T, n, s.st));
      HIPCHK(launch_col_dots(n, nrhs, k + 1, V, vs, T, n, H2, ldh, s.st));
      HIPCHK(launch_col_axpy(n, nrhs, k + 1, V, vs, H2, ldh, -1.0, T, n, s.st));
      HIPCHK(launch_col_dots(n, nrhs, 1, T, 0, T, n, H3, 1, s.st));
      HIPCHK(launch_col_normalize(n, nrhs, T, n, H3, 1, -1.0, V + (size_t)(k + 1) * vs, n, s.st));
      TRY(fetch(H1, h1, (size_t)ldh * nrhs));
      TRY(fetch(H2, h2, (size_t)ldh * nrhs));
      TRY(fetch(H3, h3, nrhs));
      bool all = true;
      for (int j = 0; j < nrhs; ++j) {
        double* hc = &Hh[((size_t)j * m + k) * (m + 1)];  // column k of column j's Hessenberg matrix
        for (int i = 0; i <= k; ++i) hc[i] = -(h1[i + (size_t)j * ldh] + h2[i + (size_t)j * ldh]);
        hc[k + 1] = std::sqrt(h3[j]);
        for (int i = 0; i < k; ++i) {  // the earlier rotations
          const double c = cs[(size_t)j * m + i], sg = sn[(size_t)j * m + i];
          const double a = hc[i], b = hc[i + 1];
          hc[i] = c * a + sg * b;
          hc[i + 1] = -sg * a + c * b;
        }
        const double a = hc[k], b = hc[k + 1];
        const double rr = std::hypot(a, b);
        const double c = rr > 0.0 ? a / rr : 1.0, sg = rr > 0.0 ? b / rr : 0.0;
        cs[(size_t)j * m + k] = c;
        sn[(size_t)j * m + k] = sg;
        hc[k] = rr;
        hc[k + 1] = 0.0;
        double* gj = &g[(size_t)j * (m + 1)];
        gj[k + 1] = -sg * gj[k];
        gj[k] = c * gj[k];
        if (!(std::fabs(gj[k + 1]) <= kGmresTol * beta[j])) all = false;
      }
      kd = k + 1;
      if (all) break;
    }
    // y = H^{-1} g (upper triangular after the rotations), x += V y
    for (int j = 0; j < nrhs; ++j) {
      for (int i = kd - 1; i >= 0; --i) {
        double t = g[(size_t)j * (m + 1) + i];
        for (int l = i + 1; l < kd; ++l) t -= Hh[((size_t)j * m + l) * (m + 1) + i] * y[l + (size_t)j * ldh];
        const double d = Hh[((size_t)j * m + i) * (m + 1) + i];
        y[i + (size_t)j * ldh] = d != 0.0 ? t / d : 0.0;
      }
    }
    HIPCHK(hipMemcpyAsync(H3, y.data(), (size_t)ldh * nrhs * sizeof(double), hipMemcpyHostToDevice, s.st));
    HIPCHK(launch_col_axpy(n, nrhs, kd, V, vs, H3, ldh, 1.0, X, ldx, s.st));
  }
}

void fill_result(ada_result* r, const DevRec& h, int cls, int kl, int ku, int route, int chol_failed, int fallback,
                 int n) {
  memset(r, 0, sizeof(*r));
  r->cls = cls;
  r->kl = kl;
  r->ku = ku;
  r->route = route;
  r->chol_failed = chol_failed;
  r->fallback = fallback;
  r->info = 0;
  r->rank = n;
  r->rcond = h.rcond;
  r->berr = h.berr;
  r->nsolves = h.est_nsolves;
}

// The workspace of ada_solve_noalloc: one fixed array per GPU (each device that
// loads the library holds its own copy until the process ends). In host code
// `scratch` only names the symbol; its device address on each GPU comes from
// hipGetSymbolAddress with that GPU current, taken once per device when a
// context is created there, and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[ADA_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// device address of the current device's scratch (the device is `device`, already current)
hipError_t noalloc_scratch_address(int device, void** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch_addr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[device] = ptr;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

}  // namespace

extern "C" {

int ada_create(ada_ctx* out, int device) {
  if (!out) return fail(ADA_ERR_ARG, "out is NULL");
  *out = nullptr;
  int count = 0;
  HIPCHK(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(ADA_ERR_ARG, "device out of range");
  ada_ctx c = new (std::nothrow) ada_ctx_s();
  if (!c) return fail(ADA_ERR_NOMEM, "context allocation");
  c->device = device;
  HIPCHK(hipSetDevice(device));
  hipError_t e = hipHostMalloc((void**)&c->host_rec, sizeof(DevRec), hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming);
  if (e == hipSuccess) e = noalloc_scratch_address(device, &c->noalloc_scratch);
  if (e != hipSuccess) {
    ada_destroy(c);
    return fail(ADA_ERR_HIP, std::string("context set-up: ") + hipGetErrorString(e));
  }
  *out = c;
  return ADA_OK;
}

void ada_destroy(ada_ctx ctx) {
  if (!ctx) return;
  if (ctx->side) (void)hipStreamSynchronize(ctx->side);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  if (ctx->side) (void)hipStreamDestroy(ctx->side);
  for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->host_rec) (void)hipHostFree(ctx->host_rec);
  delete ctx;
}

const char* ada_last_error(void) { return g_err.c_str(); }

void ada_opts_default(ada_opts* o) {
  if (o) *o = defaults();
}

size_t ada_workspace_size(int n, int nrhs, const ada_opts* opts) {
  ada_opts o;
  if (!read_opts(opts, o)) return 0;
  Plan p;
  if (!make_plan(n, nrhs, o, p)) return 0;
  return p.total;
}

size_t ada_batched_workspace_size(int count) {
  if (count < 1) return 0;
  return batched_workspace_bytes(count);
}

namespace {
int batched_prec_index(int precision) {
  return precision == ADA_PREC_FP64 ? 0 : (precision == ADA_PREC_FP32_IR ? 1 : -1);
}
// arguments of ada_solve_batched and ada_autotune_batched
int check_batched_args(ada_ctx ctx, int count, const ada_desc* d_desc, const double* A_pool, const double* B_pool,
                       double* X_pool, void* work, size_t work_bytes, const ada_opts* opts, ada_result* d_results,
                       ada_opts& o) {
  if (!ctx) return fail(ADA_ERR_ARG, "ctx is NULL");
  if (count < 1) return fail(ADA_ERR_ARG, "count must be >= 1");
  if (!d_desc || !A_pool || !B_pool || !X_pool || !work || !d_results)
    return fail(ADA_ERR_ARG, "NULL descriptor, pool, workspace or result pointer");
  if (!read_opts(opts, o)) return fail(ADA_ERR_ARG, "opts->struct_size is not a known size");
  if (o.layout != ADA_LAYOUT_DENSE) return fail(ADA_ERR_ARG, "batched solves take dense input only");
  if (batched_prec_index(o.precision) < 0)
    return fail(ADA_ERR_ARG, "batched solves take precision ADA_PREC_FP64 or ADA_PREC_FP32_IR");
  if (o.extensions != 0) return fail(ADA_ERR_ARG, "batched solves take the paper's routes only (extensions = 0)");
  if ((reinterpret_cast<uintptr_t>(work) & 255) != 0) return fail(ADA_ERR_ARG, "work must be 256-byte aligned");
  if (work_bytes < ada_batched_workspace_size(count)) return fail(ADA_ERR_ARG, "workspace too small");
  return ADA_OK;
}
}  // namespace

int ada_set_batched_shape(ada_ctx ctx, int precision, const ada_batched_shape* shape) {
  if (!ctx) return fail(ADA_ERR_ARG, "ctx is NULL");
  const int pi = batched_prec_index(precision);
  if (pi < 0) return fail(ADA_ERR_ARG, "precision must be ADA_PREC_FP64 or ADA_PREC_FP32_IR");
  ada_batched_shape sh = shape ? *shape : batched_default_shape();
  if (const char* why = batched_shape_problem(sh)) return fail(ADA_ERR_ARG, std::string("batched shape: ") + why);
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->bshape[pi] = sh;
  return ADA_OK;
}

int ada_get_batched_shape(ada_ctx ctx, int precision, ada_batched_shape* shape) {
  if (!ctx || !shape) return fail(ADA_ERR_ARG, "ctx or shape is NULL");
  const int pi = batched_prec_index(precision);
  if (pi < 0) return fail(ADA_ERR_ARG, "precision must be ADA_PREC_FP64 or ADA_PREC_FP32_IR");
  std::lock_guard<std::mutex> lk(ctx->mu);
  *shape = ctx->bshape[pi];
  return ADA_OK;
}

int ada_solve_batched(ada_ctx ctx, int count, const ada_desc* d_desc, const double* A_pool, const double* B_pool,
                      double* X_pool, void* work, size_t work_bytes, const ada_opts* opts, ada_result* d_results,
                      void* stream) {
  ada_opts o;
  if (int rc = check_batched_args(ctx, count, d_desc, A_pool, B_pool, X_pool, work, work_bytes, opts, d_results, o))
    return rc;
  std::lock_guard<std::mutex> lk(ctx->mu);
  HIPCHK(hipSetDevice(ctx->device));
  HIPCHK(launch_solve_batched(count, d_desc, A_pool, B_pool, X_pool, work, work_bytes, o, d_results,
                              static_cast<hipStream_t>(stream), ctx->bshape[batched_prec_index(o.precision)]));
  return ADA_OK;
}

int ada_autotune_batched(ada_ctx ctx, int count, const ada_desc* d_desc, const double* A_pool, const double* B_pool,
                         double* X_pool, void* work, size_t work_bytes, const ada_opts* opts, ada_result* d_results,
                         void* stream, ada_batched_shape* shape_out, double* ms_out) {
  ada_opts o;
  if (int rc = check_batched_args(ctx, count, d_desc, A_pool, B_pool, X_pool, work, work_bytes, opts, d_results, o))
    return rc;
  std::lock_guard<std::mutex> lk(ctx->mu);
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t ev[4] = {};
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      for (auto& f : ev)
        if (f) (void)hipEventDestroy(f);
      return fail(ADA_ERR_HIP, "autotune: event creation failed");
    }
  int rc = ADA_OK;
  // runs the batch under shape s and returns the time of each of its launches (ms)
  auto run = [&](const ada_batched_shape& s, float* ms) -> bool {
    if (launch_solve_batched(count, d_desc, A_pool, B_pool, X_pool, work, work_bytes, o, d_results, st, s, ev) !=
            hipSuccess ||
        hipEventSynchronize(ev[s.buckets]) != hipSuccess)
      return false;
    for (int k = 0; k < s.buckets; ++k)
      if (hipEventElapsedTime(&ms[k], ev[k], ev[k + 1]) != hipSuccess) return false;
    return true;
  };
  // the splits (largest order of each range after the first) and the per-range variants
  static const int splits[][2] = {{0, 0}, {128, 0}, {96, 0}, {64, 0}, {128, 64}, {96, 48}};
  struct Variant { int wg_per_cu, stage_cols; };
  static const Variant variants[] = {{1, 8}, {1, 4}, {2, 8}};
  ada_batched_shape best = batched_default_shape();
  double best_ms = 1e300;
  float ms[3];
  if (!run(best, ms)) rc = fail(ADA_ERR_HIP, "autotune: warm-up launch failed");
  for (const auto& sp : splits) {
    if (rc != ADA_OK) break;
    ada_batched_shape base = batched_default_shape();
    base.buckets = 1 + (sp[0] > 0) + (sp[1] > 0);
    base.max_n[1] = sp[0];
    base.max_n[2] = sp[1];
    // fastest variant of each range under this split
    double range_ms[3] = {1e300, 1e300, 1e300};
    ada_batched_shape pick = base;
    for (const auto& v : variants) {
      ada_batched_shape s = base;
      bool any = v.wg_per_cu == 1;  // a two-per-unit variant only where some range can take it
      for (int k = 0; k < s.buckets; ++k) {
        const bool two = v.wg_per_cu == 2 && s.max_n[k] <= 96;
        s.wg_per_cu[k] = two ? 2 : 1;
        s.workgroups[k] = two ? 512 : 256;
        any |= two;
      }
      s.stage_cols = v.stage_cols;
      if (!any || batched_shape_problem(s)) continue;
      if (!run(s, ms)) {
        rc = fail(ADA_ERR_HIP, "autotune: launch failed");
        break;
      }
      for (int k = 0; k < s.buckets; ++k)
        if (ms[k] < range_ms[k]) {
          range_ms[k] = ms[k];
          pick.wg_per_cu[k] = s.wg_per_cu[k];
          pick.workgroups[k] = s.workgroups[k];
          if (k == 0) pick.stage_cols = s.stage_cols;  // only the first range holds orders above 128
        }
    }
    double total = 0.0;
    for (int k = 0; k < base.buckets; ++k) total += range_ms[k];
    if (rc == ADA_OK && total < best_ms && !batched_shape_problem(pick)) {
      best_ms = total;
      best = pick;
    }
  }
  if (rc == ADA_OK) {
    if (!run(best, ms)) {
      rc = fail(ADA_ERR_HIP, "autotune: launch failed");
    } else {
      double t = 0.0;
      for (int k = 0; k < best.buckets; ++k) t += ms[k];
      ctx->bshape[batched_prec_index(o.precision)] = best;
      if (shape_out) *shape_out = best;
      if (ms_out) *ms_out = t;
    }
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  return rc;
}

int ada_profile_enable(ada_ctx ctx, int on) {
  if (!ctx) return fail(ADA_ERR_ARG, "ctx is NULL");
  ctx->prof = on != 0;
  return ADA_OK;
}

int ada_profile_families(ada_ctx ctx, unsigned mask) {
  if (!ctx) return fail(ADA_ERR_ARG, "ctx is NULL");
  ctx->prof_mask = mask;
  return ADA_OK;
}

int ada_autotune_band(ada_ctx ctx, int n, int kl, int ku, int nrhs, void* stream, int* piece_out,
                      double* ms_out) {
  if (!ctx) return fail(ADA_ERR_ARG, "ctx is NULL");
  if (kl < 0 || ku < 0 || kl + ku < 1 || kl + ku > 31 || nrhs < 1 || nrhs > 64 || n < kBandChunkMin || n > (1 << 26))
    return fail(ADA_ERR_ARG, "autotune: need 1 <= kl + ku <= 31, 1 <= nrhs <= 64 and 512 <= n <= 2^26");
  std::lock_guard<std::mutex> lock(ctx->mu);
  HIPCHK(hipSetDevice(ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int ldgb = 2 * kl + ku + 1;
  const size_t scd = band_chunked_scratch_doubles(n, kl, ku, nrhs);
  const size_t bytes = ((size_t)n * ldgb + 2 * (size_t)n * nrhs + scd) * sizeof(double) + (size_t)n * sizeof(int) + 1024;
  char* buf = nullptr;
  if (hipMalloc(&buf, bytes) != hipSuccess) return fail(ADA_ERR_NOMEM, "autotune: device allocation failed");
  double* GB = reinterpret_cast<double*>(buf);
  double* X = GB + (size_t)n * ldgb;
  double* T = X + (size_t)n * nrhs;
  double* scb = T + (size_t)n * nrhs;
  int* ipiv = reinterpret_cast<int*>(scb + scd);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = ADA_OK;
  int best = 0;
  double best_ms = INFINITY;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      launch_band_tune_fill(n, kl, ku, GB, ldgb, ipiv, X, nrhs, st) != hipSuccess) {
    rc = fail(ADA_ERR_HIP, "autotune: set-up failed");
  }
  const BandScratch sc = band_chunked_scratch(scb, n, kl, ku, nrhs);
  for (int k = 0; rc == ADA_OK && k < 4; ++k) {
    const int piece = kBandPieces[k];
    if (!band_piece_fits(piece, kl, ku)) continue;
    unsigned maps = 0;
    // first solve forms the maps (not timed); then the best of three solves with the maps kept
    auto one = [&]() {
      return launch_gbtrs_chunked(n, kl, ku, nrhs, GB, ldgb, ipiv, false, X, n, T, n, sc, nullptr, 0, nullptr, 0,
                                  &maps, piece, st);
    };
    if (one() != hipSuccess) { rc = fail(ADA_ERR_HIP, "autotune: band solve launch failed"); break; }
    double ms = INFINITY;
    for (int rep = 0; rep < 3; ++rep) {
      float t = 0.0f;
      if (hipEventRecord(e0, st) != hipSuccess || one() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
          hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
        rc = fail(ADA_ERR_HIP, "autotune: timing failed");
        break;
      }
      ms = std::min(ms, (double)t);
    }
    if (rc == ADA_OK && ms < best_ms) { best_ms = ms; best = piece; }
  }
  if (hipStreamSynchronize(st) != hipSuccess && rc == ADA_OK) rc = fail(ADA_ERR_HIP, "autotune: stream failed");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  if (rc != ADA_OK) return rc;
  ctx->band_piece[kl + ku][nrhs > 1 ? 1 : 0][ilog2(n)] = best;
  if (piece_out) *piece_out = best;
  if (ms_out) *ms_out = best_ms;
  return ADA_OK;
}

int ada_profile_reset(ada_ctx ctx) {
  if (!ctx) return fail(ADA_ERR_ARG, "ctx is NULL");
  for (auto& a : ctx->acc) a = ada_ctx_s::Acc();
  return ADA_OK;
}

int ada_profile_read(ada_ctx ctx, int kind, int64_t* launches, double* total_ms, double* total_flops,
                     double* total_bytes) {
  if (!ctx) return fail(ADA_ERR_ARG, "ctx is NULL");
  if (kind < 0 || kind >= ADA_KF_COUNT) return fail(ADA_ERR_ARG, "kind is not an ADA_KF_* value");
  const auto& a = ctx->acc[kind];
  if (launches) *launches = a.launches;
  if (total_ms) *total_ms = a.ms;
  if (total_flops) *total_flops = a.flops;
  if (total_bytes) *total_bytes = a.bytes;
  return ADA_OK;
}

// fold the timed launches of the finished part of a solve into the per-family totals
static void collect_profile(ada_ctx ctx) {
  if (!ctx->prof) return;
  for (const auto& q : ctx->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev_pool[q.e0], ctx->ev_pool[q.e1]) != hipSuccess) continue;
    auto& a = ctx->acc[q.kind];
    a.launches += 1;
    a.ms += ms;
    a.flops += q.flops;
    a.bytes += q.bytes;
  }
  ctx->pending.clear();
}

static int solve_impl(ada_ctx ctx, int n, int nrhs, const double* A, int lda, const double* B, int ldb, double* X,
                      int ldx, void* work, size_t work_bytes, const ada_opts& o, ada_result* result,
                      hipStream_t st, int plan_nrhs, bool keep_factors) {
  Plan p;
  if (plan_nrhs < nrhs) return fail(ADA_ERR_ARG, "plan_nrhs < nrhs");
  if (!make_plan(n, plan_nrhs, o, p)) return fail(ADA_ERR_ARG, "n and nrhs must be >= 1");
  if (!work || work_bytes < p.total)
    return fail(ADA_ERR_ARG, "workspace too small: need " + std::to_string(p.total) + " bytes");
  if (((uintptr_t)work & 255) != 0) return fail(ADA_ERR_ARG, "workspace must be 256-byte aligned");
  Solve s;
  s.ctx = ctx;
  s.st = st;
  s.p = p;
  s.base = static_cast<char*>(work);
  s.rec = s.at<DevRec>(p.rec);
  s.n = n;
  s.nrhs = nrhs;
  s.keep_factors = keep_factors;
  DevRec& h = *ctx->host_rec;
  ctx->ev_used = 0;
  ctx->pending.clear();
  const double thr = o.rcond_threshold < 0.0 ? 0.5 * DBL_EPSILON : o.rcond_threshold;

  HIPCHK(launch_init_rec(s.rec, st));
  HIPCHK(launch_fill_int(s.at<int>(p.flags), 0, (size_t)p.nflags, st));

  int cls = ADA_CLASS_GENERAL, kl = -1, ku = -1;
  int route = ADA_ROUTE_NONE, chol_failed = 0, fallback = 0, info = 0;
  const double* Ad = A;  // dense view of A (band-layout input: expanded copy when needed)
  int ldad = lda;
  bool band_route_from_band_layout = false;
  bool exact_sym = false;  // A == A^T exactly (dense detection)
  int bkl = 0, bku = 0;

  if (o.layout == ADA_LAYOUT_BAND) {
    if (o.kl_in < 0 || o.ku_in < 0 || o.kl_in >= n || o.ku_in >= n || lda < o.kl_in + o.ku_in + 1)
      return fail(ADA_ERR_ARG, "band layout: need 0 <= kl_in, ku_in < n and lda >= kl_in + ku_in + 1");
    HIPCHK(launch_detect_band(n, o.kl_in, o.ku_in, A, lda, s.rec, st));
    HIPCHK(launch_check_finite(n, nrhs, B, ldb, s.rec, st));
    TRY(s.sync_read());
    if (h.nonfinite) return fail(ADA_ERR_NONFINITE, "A or B holds NaN or Inf");
    kl = h.kl;
    ku = h.ku;
    if (o.force_general || !is_banded(n, kl, ku) || kl + ku > kBandKdMax) {
      if (!p.dense) {
        return fail(o.force_general || !is_banded(n, kl, ku) ? ADA_ERR_FALLBACK_INFEASIBLE : ADA_ERR_ARG,
                    "band-layout system needs the dense path but n exceeds the dense expansion limit");
      }
      double* Ax = s.at<double>(p.Adense);
      HIPCHK(launch_band_to_dense(n, o.kl_in, o.ku_in, A, lda, Ax, n, st));
      Ad = Ax;
      ldad = n;
      HIPCHK(launch_init_rec(s.rec, st));
    } else {
      band_route_from_band_layout = true;
      cls = ADA_CLASS_BANDED;
      bkl = kl;
      bku = ku;
    }
  }

  if (!band_route_from_band_layout) {
    if (n > kDenseMax) return fail(ADA_ERR_ARG, "dense routes support n <= 16384");
    HIPCHK(s.timed(ADA_KF_DETECT, 0.0, 8.0 * (double)n * n, [&] {
      return launch_detect_dense(n, Ad, ldad, s.rec, s.at<double>(p.pcol), s.at<double>(p.prow), s.at<double>(p.cld),
                               s.at<double>(p.rld), s.at<double>(p.diag), st);
    }));
    HIPCHK(launch_check_finite(n, nrhs, B, ldb, s.rec, st));
    HIPCHK(launch_norms_reduce(n, s.at<double>(p.pcol), s.at<double>(p.prow), s.at<double>(p.cld),
                               s.at<double>(p.rld), s.at<double>(p.ctot), s.at<double>(p.csym), s.at<double>(p.rtot),
                               st));
    TRY(s.sync_read());
    if (h.nonfinite) return fail(ADA_ERR_NONFINITE, "A or B holds NaN or Inf");
    exact_sym = !h.asym;
    if (o.force_general) {
      cls = ADA_CLASS_GENERAL;
      kl = ku = -1;
    } else {
      kl = h.kl;
      ku = h.ku;
      if (is_banded(n, kl, ku)) cls = ADA_CLASS_BANDED;
      else if (kl == 0) cls = ADA_CLASS_TRI_UPPER;
      else if (ku == 0) cls = ADA_CLASS_TRI_LOWER;
      else {
        const double max_diag = bits_to_double(h.max_diag_bits);
        const double max_lower = bits_to_double(h.max_lower_bits);
        const bool sympd = !h.diag_nonpos && !h.sym_bad && (max_lower < max_diag);
        cls = sympd ? ADA_CLASS_SYMPD : ADA_CLASS_GENERAL;
        if (cls == ADA_CLASS_GENERAL && (o.extensions & ADA_EXT_SYM) && exact_sym) cls = ADA_CLASS_SYM;
      }
    }
  }

  // ---------------- route
  double* W = s.at<double>(p.W);
  const int norm_mode = (cls == ADA_CLASS_SYMPD) ? 1 : 0;
  if (!band_route_from_band_layout)
    HIPCHK(launch_anorm(n, s.at<double>(p.ctot), s.at<double>(p.csym), s.at<double>(p.rtot), norm_mode, s.rec, st));
  // mixed precision (LU and Cholesky routes): low-precision trailing updates, FP64 refinement; the
  // FP64 route below runs when the factorisation fails or the refinement does not converge
  bool mixed_done = false;
  int refine_iters = 0;
  if (o.precision != ADA_PREC_FP64 && (cls == ADA_CLASS_GENERAL || cls == ADA_CLASS_SYMPD)) {
    const bool chol = cls == ADA_CLASS_SYMPD;
    s.lowp = o.precision;
    TRY(chol ? route_chol(s, Ad, ldad, B, ldb, X, ldx) : route_lu(s, Ad, ldad, B, ldb, X, ldx));
    s.lowp = ADA_PREC_FP64;
    TRY(s.sync_read());
    if (h.timeout) return fail(ADA_ERR_HIP, "a bounded device wait timed out");
    const bool fact_ok = chol ? h.chol_info == INT_MAX : h.info == INT_MAX;
    const bool refinable =
        fact_ok && h.rcond >= kRcondRefine;
    bool conv = false;
    int steps = 0;
    if (refinable) {
      if (o.precision == ADA_PREC_BF16_IR) TRY(refine_gmres(s, chol, Ad, ldad, B, ldb, X, ldx, conv, steps));
      else TRY(refine(s, chol, Ad, ldad, B, ldb, X, ldx, conv, steps));
    }
    if (conv) {
      mixed_done = true;
      route = chol ? ADA_ROUTE_CHOL : ADA_ROUTE_LU;
      refine_iters = steps;
    } else {
      refine_iters = refinable ? -1 - steps : -1;
      HIPCHK(launch_init_rec(s.rec, st));
      HIPCHK(launch_anorm(n, s.at<double>(p.ctot), s.at<double>(p.csym), s.at<double>(p.rtot), norm_mode, s.rec, st));
    }
  }
  if (mixed_done) {
    // x, rcond (of the low-precision factors) and the backward error come from the refinement
  } else if (cls == ADA_CLASS_GENERAL) {
    route = ADA_ROUTE_LU;
    TRY(route_lu(s, Ad, ldad, B, ldb, X, ldx));
  } else if (cls == ADA_CLASS_SYM) {
    route = ADA_ROUTE_LDLT;
    TRY(route_ldlt(s, Ad, ldad, B, ldb, X, ldx));
  } else if (cls == ADA_CLASS_SYMPD) {
    route = ADA_ROUTE_CHOL;
    TRY(route_chol(s, Ad, ldad, B, ldb, X, ldx));
    TRY(s.sync_read());
    if (h.timeout) return fail(ADA_ERR_HIP, "a bounded device wait timed out");
    if (h.chol_info != INT_MAX) {
      // Cholesky failed: not sympd after all -> LU on the original A (LDL^T with the symmetric extension)
      chol_failed = 1;
      const bool ldlt = (o.extensions & ADA_EXT_SYM) && exact_sym;
      route = ldlt ? ADA_ROUTE_LDLT : ADA_ROUTE_LU;
      HIPCHK(launch_init_rec(s.rec, st));
      HIPCHK(launch_anorm(n, s.at<double>(p.ctot), s.at<double>(p.csym), s.at<double>(p.rtot), 0, s.rec, st));
      TRY(ldlt ? route_ldlt(s, Ad, ldad, B, ldb, X, ldx) : route_lu(s, Ad, ldad, B, ldb, X, ldx));
    }
  } else if (cls == ADA_CLASS_TRI_UPPER || cls == ADA_CLASS_TRI_LOWER) {
    route = ADA_ROUTE_TRI;
    if (h.diag_zero_first != INT_MAX) {
      info = h.diag_zero_first;  // zero on the diagonal: the triangular solver fails
    } else {
      TRY(route_tri(s, Ad, ldad, cls == ADA_CLASS_TRI_LOWER, B, ldb, X, ldx));
    }
  } else {  // banded
    route = ADA_ROUTE_BAND_LU;
    if (!band_route_from_band_layout) {
      bkl = kl;
      bku = ku;
      if (bkl + bku > kBandKdMax) return fail(ADA_ERR_ARG, "band kernels support kl + ku <= 31");
    }
    const int ldgb = 2 * bkl + bku + 1;
    double* G0 = s.at<double>(p.gb0);
    if (band_route_from_band_layout)
      HIPCHK(launch_band_pack_band(n, bkl, bku, A, lda, o.ku_in, G0, ldgb, st));
    else
      HIPCHK(launch_band_pack_dense(n, bkl, bku, Ad, ldad, G0, ldgb, st));
    HIPCHK(launch_band_norms(n, bkl, bku, G0, ldgb, s.rec, st));
    TRY(route_band(s, G0, W, bkl, bku, B, ldb, X, ldx));
  }
  // backward error of the routed x (also flags a non-finite x)
  if (info == 0 && !mixed_done) {
    if (band_route_from_band_layout) {
      HIPCHK(launch_band_resid(n, o.kl_in, o.ku_in, nrhs, A, lda, o.ku_in, B, ldb, X, ldx, s.at<double>(p.R), n, st));
      HIPCHK(launch_berr(n, nrhs, s.at<double>(p.R), n, B, ldb, X, ldx, s.at<double>(p.percol), s.rec, st));
    } else if (o.want_berr) {
      TRY(backward_error_dense(s, Ad, ldad, B, ldb, X, ldx));
    } else {
      HIPCHK(launch_x_finite(n, nrhs, X, ldx, s.rec, st));
    }
  }
  TRY(s.sync_read());
  if (h.timeout) return fail(ADA_ERR_HIP, "a bounded device wait timed out");
  if (info == 0 && h.info != INT_MAX) info = h.info;
  const double rcond = info ? NAN : h.rcond;
  if (info || h.x_nonfinite) fallback = ADA_FALLBACK_FAILURE;
  else if (rcond != rcond) fallback = ADA_FALLBACK_RCOND_NAN;
  else if (rcond < thr) fallback = ADA_FALLBACK_RCOND;

  collect_profile(ctx);

  fill_result(result, h, cls, kl, ku, route, chol_failed, fallback, n);
  result->refine_iters = refine_iters;
  result->info = info;
  result->rcond = rcond;
  result->berr = (o.want_berr || band_route_from_band_layout || mixed_done) && info == 0 ? h.berr : NAN;
  if (!fallback) return ADA_OK;
  if (o.no_approx) return fail(ADA_ERR_SINGULAR, "the fallback is due (solver failure or rcond below threshold) "
                                                 "but no_approx is set");
  // ---------------- SVD least-squares fallback on the original A
  if (!p.dense) return fail(ADA_ERR_FALLBACK_INFEASIBLE, "SVD fallback of a band-layout system this large");
  if (o.layout == ADA_LAYOUT_BAND && Ad == A) {
    double* Ax = s.at<double>(p.Adense);
    HIPCHK(launch_band_to_dense(n, o.kl_in, o.ku_in, A, lda, Ax, n, st));
    Ad = Ax;
    ldad = n;
  }
  double* Ws = W;
  double* Vs = s.at<double>(p.V);
  double* Ts = s.at<double>(p.T);
  TRY(route_svd(s, Ad, ldad, B, ldb, X, ldx, Ws, Vs, Ts));
  if (o.want_berr || o.layout == ADA_LAYOUT_BAND) {
    if (o.layout == ADA_LAYOUT_BAND) {
      HIPCHK(launch_band_resid(n, o.kl_in, o.ku_in, nrhs, A, lda, o.ku_in, B, ldb, X, ldx, s.at<double>(p.R), n, st));
      HIPCHK(launch_berr(n, nrhs, s.at<double>(p.R), n, B, ldb, X, ldx, s.at<double>(p.percol), s.rec, st));
    } else {
      TRY(backward_error_dense(s, Ad, ldad, B, ldb, X, ldx));
    }
  }
  TRY(s.sync_read());
  collect_profile(ctx);
  result->route = ADA_ROUTE_SVD;
  result->rank = h.rank;
  result->sweeps = h.sweeps;
  result->berr = (o.want_berr || o.layout == ADA_LAYOUT_BAND) ? h.berr : NAN;
  return ADA_OK;
}

int ada_solve(ada_ctx ctx, int n, int nrhs, const double* A, int lda, const double* B, int ldb, double* X, int ldx,
              void* work, size_t work_bytes, const ada_opts* opts, ada_result* result, void* stream) {
  if (!ctx) return fail(ADA_ERR_ARG, "ctx is NULL");
  if (!A || !B || !X || !result) return fail(ADA_ERR_ARG, "NULL matrix or result pointer");
  ada_opts o;
  if (!read_opts(opts, o)) return fail(ADA_ERR_ARG, "opts->struct_size is not a known size");
  if (o.layout != ADA_LAYOUT_DENSE && o.layout != ADA_LAYOUT_BAND) return fail(ADA_ERR_ARG, "unknown layout");
  if (o.precision != ADA_PREC_FP64 && o.precision != ADA_PREC_FP32_IR && o.precision != ADA_PREC_BF16_IR)
    return fail(ADA_ERR_ARG, "unknown precision");
  if (o.extensions & ~ADA_EXT_SYM) return fail(ADA_ERR_ARG, "unknown extension bits");
  if (n < 1 || nrhs < 1) return fail(ADA_ERR_ARG, "n and nrhs must be >= 1");
  if (o.layout == ADA_LAYOUT_DENSE && lda < n) return fail(ADA_ERR_ARG, "lda < n");
  if (ldb < n || ldx < n) return fail(ADA_ERR_ARG, "ldb or ldx < n");
  std::lock_guard<std::mutex> lock(ctx->mu);
  HIPCHK(hipSetDevice(ctx->device));
  return solve_impl(ctx, n, nrhs, A, lda, B, ldb, X, ldx, work, work_bytes, o, result,
                    static_cast<hipStream_t>(stream), nrhs, false);
}

int ada_solve_noalloc(ada_ctx ctx, int n, int nrhs, const double* A, int lda, const double* B, int ldb, double* X,
                      int ldx, const ada_opts* opts, ada_result* result, void* stream) {
  if (!ctx) return fail(ADA_ERR_ARG, "ctx is NULL");
  if (!A || !B || !X || !result) return fail(ADA_ERR_ARG, "NULL matrix or result pointer");
  ada_opts o;
  if (!read_opts(opts, o)) return fail(ADA_ERR_ARG, "opts->struct_size is not a known size");
  if (o.layout != ADA_LAYOUT_DENSE && o.layout != ADA_LAYOUT_BAND) return fail(ADA_ERR_ARG, "unknown layout");
  if (o.precision != ADA_PREC_FP64 && o.precision != ADA_PREC_FP32_IR && o.precision != ADA_PREC_BF16_IR)
    return fail(ADA_ERR_ARG, "unknown precision");
  if (o.extensions & ~ADA_EXT_SYM) return fail(ADA_ERR_ARG, "unknown extension bits");
  if (n < 1 || nrhs < 1) return fail(ADA_ERR_ARG, "n and nrhs must be >= 1");
  if (o.layout == ADA_LAYOUT_DENSE && lda < n) return fail(ADA_ERR_ARG, "lda < n");
  if (ldb < n || ldx < n) return fail(ADA_ERR_ARG, "ldb or ldx < n");
  Plan p;
  if (!make_plan(n, nrhs, o, p)) return fail(ADA_ERR_ARG, "invalid shape");
  if (p.total > (size_t)ADA_NOALLOC_SCRATCH_BYTES)
    return fail(ADA_ERR_ARG, "ada_solve_noalloc: this shape needs " + std::to_string(p.total) +
                                 " bytes of workspace, more than the fixed scratch of " +
                                 std::to_string((size_t)ADA_NOALLOC_SCRATCH_BYTES) + " bytes");
  if (!ctx->noalloc_scratch) return fail(ADA_ERR_HIP, "ada_solve_noalloc: no scratch address for this device");
  std::lock_guard<std::mutex> lock(ctx->mu);
  HIPCHK(hipSetDevice(ctx->device));
  struct NoGrow {
    ada_ctx c;
    ~NoGrow() { c->no_grow = false; }
  } guard{ctx};
  ctx->no_grow = true;
  return solve_impl(ctx, n, nrhs, A, lda, B, ldb, X, ldx, ctx->noalloc_scratch, (size_t)ADA_NOALLOC_SCRATCH_BYTES, o,
                    result, static_cast<hipStream_t>(stream), nrhs, false);
}

}  // extern "C"

namespace ada {

void set_last_error(const std::string& msg) { g_err = msg; }
int context_device(ada_ctx ctx) { return ctx ? ctx->device : -1; }
std::string last_error_string() { return g_err; }

int solve_internal(ada_ctx ctx, int n, int nrhs, int plan_nrhs, const double* A, int lda, const double* B, int ldb,
                   double* X, int ldx, void* work, size_t work_bytes, const ada_opts& o, ada_result* result,
                   hipStream_t st, bool keep_factors) {
  if (!ctx || !A || !B || !X || !result) return fail(ADA_ERR_ARG, "NULL context, matrix or result pointer");
  if (n < 1 || nrhs < 1 || lda < n || ldb < n || ldx < n) return fail(ADA_ERR_ARG, "bad n, nrhs or leading dimension");
  std::lock_guard<std::mutex> lock(ctx->mu);
  HIPCHK(hipSetDevice(ctx->device));
  return solve_impl(ctx, n, nrhs, A, lda, B, ldb, X, ldx, work, work_bytes, o, result, st, plan_nrhs, keep_factors);
}

int solve_factored(ada_ctx ctx, int n, int nrhs, int plan_nrhs, const double* A, int lda, const double* B, int ldb,
                   double* X, int ldx, void* work, size_t work_bytes, const ada_opts& o, const ada_result& orig,
                   ada_result* result, hipStream_t st) {
  if (!ctx || !A || !B || !X || !result) return fail(ADA_ERR_ARG, "NULL context, matrix or result pointer");
  if (n < 1 || nrhs < 1 || nrhs > plan_nrhs || lda < n || ldb < n || ldx < n)
    return fail(ADA_ERR_ARG, "bad n, nrhs or leading dimension for the kept factors");
  if (o.layout != ADA_LAYOUT_DENSE) return fail(ADA_ERR_ARG, "kept factors of dense input only");
  std::lock_guard<std::mutex> lock(ctx->mu);
  HIPCHK(hipSetDevice(ctx->device));
  Plan p;
  if (!make_plan(n, plan_nrhs, o, p) || work_bytes < p.total) return fail(ADA_ERR_ARG, "workspace of the kept factors");
  Solve s;
  s.ctx = ctx;
  s.st = st;
  s.p = p;
  s.base = static_cast<char*>(work);
  s.rec = s.at<DevRec>(p.rec);
  s.n = n;
  s.nrhs = nrhs;
  DevRec& h = *ctx->host_rec;
  ctx->ev_used = 0;
  ctx->pending.clear();
  // fresh record (counters, flags, stop), then the norms from the column/row totals detection left
  HIPCHK(launch_init_rec(s.rec, st));
  HIPCHK(launch_fill_int(s.at<int>(p.flags), 0, (size_t)p.nflags, st));
  const int norm_mode = orig.route == ADA_ROUTE_CHOL ? 1 : 0;
  HIPCHK(launch_anorm(n, s.at<double>(p.ctot), s.at<double>(p.csym), s.at<double>(p.rtot), norm_mode, s.rec, st));
  double* W = s.at<double>(p.W);
  int* stop = &s.rec->stop;
  switch (orig.route) {
    case ADA_ROUTE_LU:
      HIPCHK(launch_gather_rows(n, nrhs, s.at<int>(p.perm), B, ldb, X, ldx, stop, 0, st));
      TRY(s.trsm(W, p.ldw, true, false, true, X, ldx, nrhs, stop, 0));
      TRY(s.trsm(W, p.ldw, false, false, false, X, ldx, nrhs, stop, 0));
      break;
    case ADA_ROUTE_CHOL:
      HIPCHK(launch_copy(n, nrhs, B, ldb, X, ldx, st));
      TRY(s.trsm(W, p.ldw, true, false, false, X, ldx, nrhs, stop, 0));
      TRY(s.trsm(W, p.ldw, true, true, false, X, ldx, nrhs, stop, 0));
      break;
    case ADA_ROUTE_LDLT: {
      const int* perm = s.at<int>(p.perm);
      double* T = s.at<double>(p.T);
      HIPCHK(launch_gather_rows(n, nrhs, perm, B, ldb, T, n, stop, 0, st));
      TRY(s.trsm(W, p.ldw, true, false, true, T, n, nrhs, stop, 0));
      HIPCHK(launch_ldlt_dsolve(n, nrhs, s.at<double>(p.tau), s.at<double>(p.sigma), T, n, stop, 0, st));
      TRY(s.trsm(W, p.ldw, true, true, true, T, n, nrhs, stop, 0));
      HIPCHK(launch_scatter_rows(n, nrhs, perm, T, n, X, ldx, stop, 0, st));
      break;
    }
    case ADA_ROUTE_TRI:
      HIPCHK(launch_copy(n, nrhs, B, ldb, X, ldx, st));
      TRY(s.trsm(A, lda, orig.cls == ADA_CLASS_TRI_LOWER, false, false, X, ldx, nrhs, stop, 0));
      break;
    case ADA_ROUTE_BAND_LU:
      HIPCHK(launch_copy(n, nrhs, B, ldb, X, ldx, st));
      TRY(band_solve(s, W, orig.kl, orig.ku, false, X, ldx, nrhs, s.at<double>(p.T), n, stop, 0));
      break;
    case ADA_ROUTE_SVD: {
      double* C = s.at<double>(p.R);
      HIPCHK(launch_copy(n, nrhs, B, ldb, C, n, st));
      HIPCHK(launch_house_qt(n, s.at<double>(p.Q), n, s.at<double>(p.tau), C, n, nrhs, st));
      HIPCHK(launch_svd_apply(n, nrhs, W, n, s.at<double>(p.V), n, C, n, X, ldx, s.at<int>(p.perm),
                              s.at<double>(p.sigma), s.at<double>(p.T), s.rec, st));
      break;
    }
    default:
      return fail(ADA_ERR_ARG, "no kept factors (the solve did not route)");
  }
  int refine_iters = 0;
  if (orig.refine_iters > 0 && (orig.route == ADA_ROUTE_LU || orig.route == ADA_ROUTE_CHOL)) {
    bool conv = false;
    int steps = 0;
    TRY(refine(s, orig.route == ADA_ROUTE_CHOL, A, lda, B, ldb, X, ldx, conv, steps));
    refine_iters = conv ? steps : -1 - steps;
  } else if (o.want_berr) {
    TRY(backward_error_dense(s, A, lda, B, ldb, X, ldx));
  } else {
    HIPCHK(launch_x_finite(n, nrhs, X, ldx, s.rec, st));
  }
  TRY(s.sync_read());
  if (h.timeout) return fail(ADA_ERR_HIP, "a bounded device wait timed out");
  *result = orig;
  result->refine_iters = refine_iters;
  result->berr = (o.want_berr || orig.refine_iters > 0) ? h.berr : NAN;
  result->status = ADA_OK;
  if (h.x_nonfinite) return fail(ADA_ERR_NONFINITE, "the solve with the kept factors produced a non-finite x");
  return ADA_OK;
}

}  // namespace ada
