// Internal declarations of libada (HIP, gfx950). Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "ada.h"
#include <stdint.h>
#include <stddef.h>

namespace ada {

constexpr double kEps = 2.220446049250313080847e-16;  // 2^-52, gap between 1 and the next double
constexpr int kWave = 64;
constexpr long kSpinLimit = 1L << 22;  // bounded waits: every spinning wave eventually exits

// Device-side record of one solve. Lives at the start of the workspace.
struct DevRec {
  // ---- detection (one pass over A) ----
  int kl, ku;                 // exact band widths (atomicMax)
  int nonfinite;              // any NaN/Inf in A or B
  int sym_bad;                // a pair violated Fig. 4 line 13 or line 16
  int diag_nonpos;            // some A_jj <= 0 (Fig. 4 line 8)
  int diag_zero_first;        // first j with A_jj == 0, +1 (INT_MAX if none)
  unsigned long long max_diag_bits;   // max diagonal entry (bit pattern; valid when all > 0)
  unsigned long long max_lower_bits;  // max |A_ij|, i > j (bit pattern of a non-negative double)
  // ---- factorisation ----
  int info;                   // first failing pivot column, 1-based (INT_MAX if none)
  int chol_info;              // Cholesky failure column (INT_MAX if none)
  int stop;                   // 1 once the routed factorisation has failed: later kernels skip their work
  int timeout;                // a bounded device wait gave up
  // ---- condition estimate (state machine of Hager/Higham) ----
  int est_phase;              // 0 done, 1 = inv(A) solve due, 2 = inv(A)^T solve due
  int est_stage;              // position in the algorithm
  int est_iter;               // iteration counter (starts at 2 after the first transposed solve)
  int est_j;                  // current unit-vector index
  int est_nsolves;
  int est_next;               // right-hand side the last decision asks for (0 none, 1 signs, 2 e_j, 3 alternating)
  int est_next_tag;           // slot that decision belongs to
  int pad1;
  int band_spec_bad;          // the chunked band LU's speculation failed (zero pivot or no agreement)
  double est;                 // current estimate of ||inv(A)||_1
  double anorm1;              // ||A||_1 of the routed matrix
  double anorm_inf;           // ||A||_inf (backward error)
  double rcond;
  // ---- result ----
  int x_nonfinite;
  int rank;
  double berr;
  double sigma_max;
  int jacobi_rotated;         // a rotation happened in the current sweep
  int sweeps;                 // Jacobi sweeps used
  int asym;                   // some A_ij != A_ji exactly (the LDL^T extension needs A = A^T)
  int ldlt_kb;                // columns the last LDL^T panel factored, from position ldlt_first
  int ldlt_first;
  int ldlt_delta;             // 1: the next LDL^T panel's first position is already factored (2x2 block)
  // ---- synchronisation counters (zeroed per solve) ----
  unsigned int counters[512];  // grid barriers / tickets, one per launch that needs one
};

// Raise a kernel's dynamic-LDS limit when a launch needs more than the default
// 64 KB (static LDS counts against the same 160 KB). `done` caches the largest
// value already granted for that kernel.
inline hipError_t ensure_lds(const void* fn, size_t bytes, size_t& done) {
  if (bytes <= 65536 || bytes <= done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) done = bytes;
  else (void)hipGetLastError();
  return e;
}

// Size-class helpers
__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// -------- device helpers --------
// value of v in lane l (l uniform across the wave)
__device__ __forceinline__ double read_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}
// argmax of |v| with ties to the lowest index (the IxAMAX convention); idx < 0 marks "no candidate"
__device__ __forceinline__ void wave_argmax(double& v, int& idx) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double v2 = __shfl_xor(v, o, 64);
    int i2 = __shfl_xor(idx, o, 64);
    bool take = (i2 >= 0) && (idx < 0 || v2 > v || (v2 == v && i2 < idx));
    if (take) { v = v2; idx = i2; }
  }
}

__device__ __forceinline__ unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }

// Accurate residual entries (the backward error of a backward-stable solution
// is as small as the rounding of a plain evaluation of b - A x): Dot2 of
// Ogita, Rump and Oishi (Accurate sum and dot product, SIAM J. Sci. Comput.
// 26(6), 2005). Each product is split exactly by a fused multiply-add
// (TwoProduct), the running sum by Knuth's TwoSum, and both errors gather in c;
// s + c is as accurate as a sum formed in twice the working precision. The
// bodies must not be contracted into other fused operations.
__device__ __forceinline__ void two_sum_acc(double& s, double& c, double p) {
#pragma clang fp contract(off)
  const double t = s + p;
  const double z = t - s;
  c += (s - (t - z)) + (p - z);
  s = t;
}
// (s, c) += -(a * x)
__device__ __forceinline__ void dot2_sub(double& s, double& c, double a, double x) {
#pragma clang fp contract(off)
  const double p = -a * x;
  const double h = fma(-a, x, -p);
  two_sum_acc(s, c, p);
  c += h;
}

__device__ __forceinline__ unsigned agent_load(const unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int agent_load(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double relaxed_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void relaxed_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int relaxed_load(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void relaxed_store(int* p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Hand-off between workgroups without cache maintenance: the data and the flag
// are written and read with agent-scope relaxed atomics (coherent across the
// chip's L2s, no write-back or invalidation of whole caches), and the writer
// waits until its data stores are complete before the flag store is issued.
// A reader that has seen the flag then reads the data with agent-scope loads.
__device__ __forceinline__ void wait_stores_done() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): every earlier load/store of this wave has completed
}

// ---------------------------------------------------------------- launchers
// Every launcher enqueues on `st` and returns hipGetLastError().

// detection
hipError_t launch_fill_int(int* p, int v, size_t count, hipStream_t st);
hipError_t launch_init_rec(DevRec* rec, hipStream_t st);
hipError_t launch_detect_dense(int n, const double* A, int lda, DevRec* rec, double* pcol, double* prow,
                               double* col_lo_diag, double* row_lo_diag, double* diag, hipStream_t st);
hipError_t launch_check_finite(int rows, int cols, const double* M, int ld, DevRec* rec, hipStream_t st);
hipError_t launch_norms_reduce(int n, const double* pcol, const double* prow, const double* col_lo_diag,
                               const double* row_lo_diag, double* col_total, double* col_sym, double* row_total,
                               hipStream_t st);
// mode: 0 general (max col_total), 1 symmetric from the lower triangle (max col_sym); also sets anorm_inf
hipError_t launch_anorm(int n, const double* col_total, const double* col_sym, const double* row_total, int mode,
                        DevRec* rec, hipStream_t st);
hipError_t launch_detect_band(int n, int kl_in, int ku_in, const double* AB, int ldab, DevRec* rec,
                              hipStream_t st);

// dense copies and permutations
hipError_t launch_copy(int rows, int cols, const double* S, int lds, double* D, int ldd, hipStream_t st);
hipError_t launch_iota(int* p, int n, hipStream_t st);
hipError_t launch_gather_rows(int n, int nrhs, const int* perm, const double* S, int lds, double* D, int ldd,
                              const int* pred, int pred_val, hipStream_t st);
hipError_t launch_scatter_rows(int n, int nrhs, const int* perm, const double* S, int lds, double* D, int ldd,
                               const int* pred, int pred_val, hipStream_t st);

// FP64 MFMA GEMM: C -= A * op(B); op(B) = B (k x n) or B^T (B is n x k); lower: only tiles meeting i >= j
// C -= A * op(B) with FP32 (prec = ADA_PREC_FP32_IR) or BF16 (ADA_PREC_BF16_IR) operands, FP32 accumulation
hipError_t launch_gemm_sub_lp(int prec, int m, int n, int k, const double* A, int lda, const double* B, int ldb,
                              bool transB, double* C, int ldc, bool lower, const int* skip_if_nonzero,
                              hipStream_t st);
hipError_t launch_gemm_sub(int m, int n, int k, const double* A, int lda, const double* B, int ldb, bool transB,
                           double* C, int ldc, bool lower, const int* skip_if_nonzero, hipStream_t st,
                           hipEvent_t ev0, hipEvent_t ev1);

// LU
struct PanelScratch {
  unsigned long long* recs;  // [2][64][2]: each workgroup's candidate record, by column parity
  double* slot_rows;         // [2][64][128]: each workgroup's candidate row
  int* moves;                // [2*256+1]: count, then (dst,src) pairs
};
hipError_t launch_getrf_panel(int n, int k0, int nbw, double* W, int ldw, int* ipiv, DevRec* rec, PanelScratch ps,
                              hipStream_t st);
hipError_t launch_panel_reset(PanelScratch ps, hipStream_t st);
// the panel's row moves applied to columns [a0, a1) and [b0, b1); with_perm: to the permutation too
hipError_t launch_laswp_moves(int a0, int a1, int b0, int b1, bool with_perm, double* W, int ldw, const int* moves,
                              int* perm, DevRec* rec, hipStream_t st);
// U12 = L11^{-1} A12 for the ncols columns starting first columns right of the panel
hipError_t launch_trsm_llnu(int k0, int nbw, int first, int ncols, double* W, int ldw, const DevRec* rec,
                            hipStream_t st);
// the next block column: the panel's row moves on its columns (and on perm), then U12 = L11^{-1} A12
hipError_t launch_swap_trsm_llnu(int k0, int nbw, int ncols, double* W, int ldw, const int* moves, int* perm,
                                 DevRec* rec, hipStream_t st);

// Cholesky
hipError_t launch_potrf_diag(int k0, int nbw, double* W, int ldw, DevRec* rec, hipStream_t st);
hipError_t launch_trsm_rltn(int k0, int nbw, int mrows, double* W, int ldw, const DevRec* rec, hipStream_t st);

// triangular solve, decoupled blocks. Solves op(T) X = X in place, T n x n (ldt).
//  lower: T is lower triangular (else upper); trans: use T^T; unit: implicit unit diagonal.
//  flags: >= ceil(n/64) ints, epoch: value that marks a finished block in this launch;
//  ticket: a zeroed counter; pred/pred_val: run only when *pred == pred_val (pred may be NULL).
hipError_t launch_trsm_dec(int n, int nrhs, const double* T, int ldt, bool lower, bool trans, bool unit, double* X,
                           int ldx, int* flags, int epoch, unsigned* ticket, DevRec* rec, const int* pred,
                           int pred_val, hipStream_t st);

// band
hipError_t launch_band_pack_dense(int n, int kl, int ku, const double* A, int lda, double* GB, int ldgb,
                                  hipStream_t st);
hipError_t launch_band_pack_band(int n, int kl, int ku, const double* AB, int ldab, int ku_in, double* GB,
                                 int ldgb, hipStream_t st);
hipError_t launch_band_norms(int n, int kl, int ku, const double* GB, int ldgb, DevRec* rec, hipStream_t st);
// band LU: GBin packed band (read only), GB factor (may equal GBin only for kl = 0 or kl > 8);
// spec_scratch: doubles for the chunked speculative factorisation (see gbtrf_spec_plan), may be null
struct GbSpecPlan {
  int L, nchunks, nsnap;
  size_t snap_doubles, exit_doubles;
};
GbSpecPlan gbtrf_spec_plan(int n, int kl, int ku);
hipError_t launch_gbtrf(int n, int kl, int ku, const double* GBin, double* GB, int ldgb, int* ipiv, DevRec* rec,
                        double* spec_scratch, size_t spec_doubles, hipStream_t st);
hipError_t launch_gbtrs(int n, int kl, int ku, int nrhs, const double* GB, int ldgb, const int* ipiv, bool trans,
                        double* X, int ldx, const int* pred, int pred_val, hipStream_t st);
// batched solve of many small systems (n <= 256, nrhs <= 8): one persistent launch per range of orders of
// the shape (the default: one launch of at most max_wg workgroups, one per compute unit). The workspace
// size covers every valid shape.
ada_batched_shape batched_default_shape(int max_wg = 256);
const char* batched_shape_problem(const ada_batched_shape& s);  // null when the shape is valid
size_t batched_workspace_bytes(int count);
hipError_t launch_solve_batched(int count, const void* desc, const double* A, const double* B, double* X,
                                void* work, size_t work_bytes, const ada_opts& o, void* results, hipStream_t st,
                                const ada_batched_shape& shape, hipEvent_t* ev = nullptr);
// ev (optional): ev[0] is recorded after the ordering kernel, ev[k + 1] after launch k
// band solves parallel over the rows (long bands); T: n x nrhs scratch (ldt); sc: see band_chunked_scratch_doubles.
// The chunk maps of a sweep kind (bit 1<<kind of *maps_ready) are computed at its first use after the
// factorisation, predicated on map_pred == map_pred_val only (not on the solve's own predicate), and
// reused while the bit stays set; the caller clears *maps_ready when the factor changes.
enum { SW_L = 0, SW_U = 1, SW_UT = 2, SW_LT = 3 };
constexpr int LC = 256;  // steps per chunk of the parallel band sweeps
struct BandSweep {
  const double* GB;
  int ldgb, kl, ku, n;
  const int* ipiv;
  int nrhs_all;
  int piece;  // steps staged in LDS at a time
};
struct BandScratch {
  // the homogeneous parts depend on the factor only: one set per sweep kind, kept across the solves
  // of one factorisation (the four Phi sets, the four Msup sets, the four H sets, whatever nrhs is)
  double* Phi;    // chunk maps (homogeneous part), nchunks x S x S, kind k at Phi + k * map_stride
  double* Msup;   // composed maps of the scan groups, kind k at Msup + k * sup_stride
  double* H;      // response of every output position to the chunk's entry state, n x S, kind k at H + k * h_stride
  size_t map_stride, sup_stride, h_stride;
  double* phi;    // chunk maps (particular part), nchunks x nrhs x S
  double* entry;  // entry state of every chunk, nchunks x nrhs x S
  double* msup;
  double* esup;   // entry state of every scan group
};
BandScratch band_chunked_scratch(double* base, int n, int kl, int ku, int nrhs);
hipError_t launch_gbtrs_chunked(int n, int kl, int ku, int nrhs, const double* GB, int ldgb, const int* ipiv,
                                bool trans, double* X, int ldx, double* T, int ldt, BandScratch sc, const int* pred,
                                int pred_val, const int* map_pred, int map_pred_val, unsigned* maps_ready,
                                int piece_hint, hipStream_t st);
// rows of a chunk staged through LDS at a time that the band solve may take (the autotuner's candidates)
constexpr int kBandPieces[4] = {8, 16, 32, 64};
bool band_piece_fits(int piece, int kl, int ku);
// a synthetic band factor for timing: diagonal 4, other band entries in [-0.25, 0.25], no interchanges
hipError_t launch_band_tune_fill(int n, int kl, int ku, double* GB, int ldgb, int* ipiv, double* X, int nrhs,
                                 hipStream_t st);
size_t band_chunked_scratch_doubles(int n, int kl, int ku, int nrhs);
hipError_t launch_band_resid(int n, int kl, int ku, int nrhs, const double* AB, int ldab, int ku_in,
                             const double* B, int ldb, const double* X, int ldx, double* R, int ldr,
                             hipStream_t st);
hipError_t launch_band_to_dense(int n, int kl_in, int ku_in, const double* AB, int ldab, double* A, int lda,
                                hipStream_t st);

// condition estimate
hipError_t launch_est_init(int n, double* v, DevRec* rec, hipStream_t st);
// tag: 1-based slot index, unique within one estimate; part: est_part_bytes() of scratch; counter: zeroed
hipError_t launch_est_step(int n, int slot_type, int tag, const double* result, double* next_in, double* xi,
                           DevRec* rec, void* part, unsigned* counter, hipStream_t st);
size_t est_part_bytes();
hipError_t launch_finalize_rcond(DevRec* rec, hipStream_t st);

// column-wise vectors of the GMRES correction solve (gmres.hip): V_i = V + i * vstride, n x nrhs, ld n
hipError_t launch_col_dots(int n, int nrhs, int kk, const double* V, size_t vstride, const double* W, int ldw,
                           double* h, int ldh, hipStream_t st);  // h[i + j ldh] = V_i(:,j) . W(:,j), i < kk
hipError_t launch_col_axpy(int n, int nrhs, int kk, const double* V, size_t vstride, const double* h, int ldh,
                           double sign, double* W, int ldw, hipStream_t st);  // W(:,j) += sign sum_i h_ij V_i(:,j)
hipError_t launch_col_normalize(int n, int nrhs, const double* S, int lds, const double* nrm2, int ldn, double sign,
                                double* D, int ldd, hipStream_t st);  // D(:,j) = sign S(:,j) / sqrt(nrm2_j)

// residual and backward error
// X += D (n x nrhs)
hipError_t launch_add_to(int n, int nrhs, const double* D, int ldd, double* X, int ldx, hipStream_t st);
size_t resid_partial_doubles(int n, int nrhs);  // scratch of launch_resid_gemv
hipError_t launch_resid_gemv(int n, int nrhs, const double* A, int lda, const double* B, int ldb, const double* X,
                             int ldx, double* R, int ldr, double* P, hipStream_t st);
hipError_t launch_x_finite(int n, int nrhs, const double* X, int ldx, DevRec* rec, hipStream_t st);
hipError_t launch_mark_stop(DevRec* rec, hipStream_t st);
hipError_t launch_berr(int n, int nrhs, const double* R, int ldr, const double* B, int ldb, const double* X,
                       int ldx, double* per_col, DevRec* rec, hipStream_t st);

// Jacobi SVD least squares
hipError_t launch_set_identity(int n, double* V, int ldv, hipStream_t st);
// One-sided Jacobi on U's columns (n <= 256: all sweeps in one workgroup; otherwise one launch per round of the
// round-robin order). Each rotation is applied to V's columns when V is not null (the accumulated rotations) and
// to rows p and q of the ny columns of Y (ld ldy) when ny > 0 (projections w_j^T c, carried instead of V).
hipError_t launch_jacobi_small(int n, double* U, int ldu, double* V, int ldv, double* Y, int ldy, int ny,
                               int max_sweeps, DevRec* rec, hipStream_t st);
hipError_t launch_jacobi_round(int n, int m, int round, double* U, int ldu, double* V, int ldv, double* Y, int ldy,
                               int ny, DevRec* rec, hipStream_t st);
hipError_t launch_clear_rotated(DevRec* rec, hipStream_t st);
// blocked sweep step (blocks of four columns, two blocks per workgroup): intra = the pairs inside
// each block, else round `round` of the round-robin over block pairs; Y (ny <= 64 columns) turns
// with U; no V. jacobi_blocked_fits says whether (n, ny) can take it.
bool jacobi_blocked_fits(int n, int ny);
hipError_t launch_jacobi_blk(int n, int round, bool intra, double* U, int ldu, double* Y, int ldy, int ny,
                             DevRec* rec, hipStream_t st);
// x = P sum over kept j of Ut_j (W_j^T C) / sigma_j^2, sigma_j = ||Ut_j|| (after the Jacobi on R^T: Ut = R^T W, W
// the accumulated rotations, C = Q^T B, P the column order, row i of the sum goes to row perm[i] of X; perm NULL:
// identity); W NULL: C already holds the projections W^T Q^T B (rotated along with the columns); also sets
// rec->sigma_max and rec->rank
// ---- symmetric indefinite LDL^T, Bunch-Kaufman pivoting (ldlt.hip) ----
// One panel from nominal position k0 (one workgroup; panels start every b-1 positions): it factors
// positions k0+delta .. up to k0+b-2, or k0+b-1 when its last pivot is a 2x2 block (delta = 1 when
// the previous panel's block took position k0), writes L to W, the updated columns (L D) to Wp
// (n x b, ld ldp; columns of positions it does not factor are zero), the interchange partner of each
// factored position to swp, D to d (diagonal) and e (sub-diagonal of 2x2 blocks), and applies its
// update to position k0+b-1 when it leaves that one to the next panel; the range it factored and
// the next delta go to rec, a zero pivot column to rec->info. The trailing update then always covers
// rows and columns from k0+b with the b columns of W and Wp from k0.
hipError_t launch_sytrf_panel(int n, int k0, int b, double* W, int ldw, double* Wp, int ldp, int* swp, double* d,
                              double* e, DevRec* rec, hipStream_t st);
// the interchanges of the range the last panel factored, applied to the rows of the columns left of
// k0 and to perm
hipError_t launch_ldlt_swap_left(int n, int k0, double* W, int ldw, const int* swp, int* perm, const DevRec* rec,
                                 hipStream_t st);
// X = D^{-1} X for the block diagonal D (predicated like the triangular solves)
hipError_t launch_ldlt_dsolve(int n, int nrhs, const double* d, const double* e, double* X, int ldx,
                              const int* pred, int pred_val, hipStream_t st);

hipError_t launch_svd_apply(int n, int nrhs, const double* Ut, int ldu, const double* W, int ldw, const double* C,
                            int ldc, double* X, int ldx, const int* perm, double* sigma, double* T, DevRec* rec,
                            hipStream_t st);
// Q = A P with the columns of A in order of decreasing 2-norm (ties to the lower index): perm[k] = source column
// of Q's column k; norm: n doubles of scratch
hipError_t launch_order_columns(int n, const double* A, int lda, double* norm, int* perm, double* Q, int ldq,
                                hipStream_t st);
// Householder QR of Q in place (reflectors below the diagonal, tau[n]), applying Q^T to the ncol columns of C
hipError_t launch_house_qr(int n, double* Q, int ldq, double* tau, double* C, int ldc, int ncol, hipStream_t st);
// C = Q^T C with the reflectors launch_house_qr left
hipError_t launch_house_qt(int n, const double* Q, int ldq, const double* tau, double* C, int ldc, int ncol,
                           hipStream_t st);
// X = R^T from the upper triangle of Q
hipError_t launch_rt(int n, const double* Q, int ldq, double* X, int ldx, hipStream_t st);

// ---- host entry points shared by the C ABI and the solve server
// ada_solve with the workspace planned for up to plan_nrhs right-hand sides (plan_nrhs >= nrhs), so that the
// factors it leaves in `work` can serve later solves of up to plan_nrhs columns (solve_factored)
// (keep_factors: the SVD route also keeps its accumulated rotations, which solve_factored needs)
int solve_internal(ada_ctx ctx, int n, int nrhs, int plan_nrhs, const double* A, int lda, const double* B, int ldb,
                   double* X, int ldx, void* work, size_t work_bytes, const ada_opts& o, ada_result* result,
                   hipStream_t st, bool keep_factors);
// X = A^{-1} B with the factors a completed solve_internal (same n, plan_nrhs, opts) left in `work`; A is the
// matrix it solved (for the triangular route and the backward error); `orig` its result
int solve_factored(ada_ctx ctx, int n, int nrhs, int plan_nrhs, const double* A, int lda, const double* B, int ldb,
                   double* X, int ldx, void* work, size_t work_bytes, const ada_opts& o, const ada_result& orig,
                   ada_result* result, hipStream_t st);
// the device a context is bound to
int context_device(ada_ctx ctx);
// the calling thread's ada_last_error() message
void set_last_error(const std::string& msg);
std::string last_error_string();

}  // namespace ada
