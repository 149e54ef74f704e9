// Internal launcher API shared by the kernel files and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace rsvd {

// ---------------------------------------------------------------- sketch --
// Omega[i * ldo + j] = normal number j*n + i of Philox stream `sid`
// (rows i < n, columns j < l); columns l..ldo-1 are set to zero.
hipError_t launch_sketch(bool f32, uint64_t seed, uint32_t sid, uint32_t batch, int64_t n,
                         int64_t l, void* Omega, int64_t ldo, hipStream_t s);
// raw Philox words: out[4*i + r] = word r of counter first+i of stream sid
hipError_t launch_philox_words(uint64_t seed, uint32_t sid, uint32_t batch, uint64_t first,
                               int64_t count, uint32_t* out, hipStream_t s);

// ------------------------------------------------------------------ gemm --
enum GemmTypes {      // element types A, X, compute, C
  GEMM_DDDD = 0,
  GEMM_FFFF = 1,
  GEMM_FFDD = 2,
  GEMM_FDDF = 3,
  GEMM_DDDF = 4,
  GEMM_FDDD = 5,
  GEMM_DFDD = 6,
};
struct GemmPlan {
  int64_t nrt, nct, KI, U, G;
  int cbw, bm, bn;
};
GemmPlan plan_gemm(int64_t M, int64_t K, int64_t L, int ncu, int force_G);
size_t gemm_part_bytes(const GemmPlan& p, size_t tc_size);
hipError_t launch_gemm(GemmTypes ty, bool trans, const void* A, int64_t lda, const void* X,
                       int64_t ldx, void* C, int64_t ldc, int64_t M, int64_t K, int64_t L,
                       const GemmPlan& p, void* part, size_t part_cap, hipStream_t s);

// Narrow passes (L <= 64) in FP32 / FP64, A streamed from HBM straight into
// the matrix-core operands: usable when lda is a multiple of 16 bytes' worth
// of elements and A is 16-byte aligned; work: narrow_work_bytes bytes
// (256-byte aligned).  C = op(A) X in A's type.
bool narrow_applies(bool f32, int64_t lda, const void* A, int64_t L);
size_t narrow_work_bytes(bool f32, bool trans, int64_t M, int64_t K, int64_t L, int ncu);
hipError_t launch_narrow(bool f32, bool trans, const void* A, int64_t lda, const void* X,
                         int64_t ldx, void* C, int64_t ldc, int64_t M, int64_t K, int64_t L,
                         int ncu, void* work, size_t work_bytes, hipStream_t s);

// BF16 passes: C (FP32) = op(A) X with A in BF16 (lda % 8 == 0, 16-byte
// aligned) and Xt = X^T in BF16 (L x ldx, ldx = rup(K, 8)); L <= 256.
GemmPlan plan_gemm_bf16(int64_t M, int64_t K, int64_t L, int ncu);
size_t gemm_bf16_part_bytes(const GemmPlan& p);
hipError_t launch_gemm_bf16(bool trans, const uint16_t* A, int64_t lda, const uint16_t* Xt,
                            int64_t ldx, float* C, int64_t ldc, int64_t M, int64_t K, int64_t L,
                            const GemmPlan& p, void* part, size_t part_cap, hipStream_t s);
// the same, adding to C
hipError_t launch_gemm_bf16_acc(bool trans, const uint16_t* A, int64_t lda, const uint16_t* Xt,
                                int64_t ldx, float* C, int64_t ldc, int64_t M, int64_t K,
                                int64_t L, const GemmPlan& p, void* part, size_t part_cap,
                                hipStream_t s);
// FP8 passes: C (FP32) = op(A8) X' with A8 FP8 E4M3 codes (lda % 16 == 0,
// 16-byte aligned) and Xt the E4M3 codes of X' transposed (L x ldx, ldx =
// rup(K, 16)), scaled in the epilogue by the column scales of X' (xscale, L)
// and, for the transposed pass, by row scales (rscale, M; may be null).
GemmPlan plan_gemm_f8(int64_t M, int64_t K, int64_t L, int ncu);
size_t gemm_f8_part_bytes(const GemmPlan& p);
hipError_t launch_gemm_f8(bool trans, const uint8_t* A, int64_t lda, const uint8_t* Xt,
                          int64_t ldx, const float* xscale, const float* rscale, float* C,
                          int64_t ldc, int64_t M, int64_t K, int64_t L, const GemmPlan& p,
                          void* part, size_t part_cap, bool accumulate, hipStream_t s);
// Xt[c][k] = e4m3(X'(k, c) / t[c]), t[c] = max_k |X'(k, c)| / 448, with X'(k, c)
// = rowscale[k] X(k, c) (rowscale may be null), or with prev (the codes of a
// first term, ld ldp, scales t0) the residual X'(k, c) - t0[c] dec(prev[c][k]).
// tmax: cols words of scratch.
hipError_t launch_quant_x_f8(bool x_f32, const void* X, int64_t ldx, int64_t rows, int cols,
                             const float* rowscale, const uint8_t* prev, int64_t ldp,
                             const float* t0, uint8_t* Xt, int64_t ldo, float* t, uint32_t* tmax,
                             hipStream_t s);
// Storage formats from an FP64 A: BF16 bit patterns (nearest, ties to even)
// and FP8 E4M3 codes with per-column FP32 scales.
hipError_t launch_quantize_bf16(const double* A, int64_t lda, int64_t m, int64_t n, uint16_t* Q,
                                int64_t ldq, hipStream_t s);
hipError_t launch_quantize_e4m3(const double* A, int64_t lda, int64_t m, int64_t n, uint8_t* Q,
                                int64_t ldq, float* scale, hipStream_t s);
// Xt[c * ldo + k] = bf16(X[k * ldi + c]) (round to nearest even), zero for k >= rows
hipError_t launch_convert_bf16(bool in_f32, const void* X, int64_t ldi, int64_t rows, int cols,
                               uint16_t* Xt, int64_t ldo, hipStream_t s);
// Xt = bf16(X - bf16(X)), the low part of a two-term split of an FP32 X
hipError_t launch_bf16_residual(const float* X, int64_t ldx, int64_t rows, int cols,
                                uint16_t* Xt, int64_t ldo, hipStream_t s);

}  // namespace rsvd

namespace rsvd {

// ------------------------------------------------------------------ orth --
// One Cholesky factorization of an lp x lp Gram matrix (lp <= 256, lp % 16 == 0,
// only rows/columns < l are read).  R upper triangular (zero below), Rdinv the
// inverses of its 16x16 diagonal blocks (lp/16 blocks of 256 doubles), dep[j]
// = 1 for columns declared dependent (pivot <= eta * G_jj).  With ni_part
// (lp/16 doubles of scratch), G is first taken as I + E: R = I + Phi(E) is
// written by one workgroup per 16 rows together with the parts of
// ||E||_F^2, and the full factorization returns at once when their sum is
// below a quarter of the unit roundoff (and otherwise overwrites R).
hipError_t launch_chol(const double* G, int64_t ldg, int l, int lp, double eta, double* R,
                       int64_t ldr, double* Rdinv, int32_t* dep, int32_t* info, hipStream_t s,
                       double* ni_part = nullptr);
// G = Y^T Y (upper 16x16 tiles of an lp x lp matrix) in FP64 for a tall Y,
// sized for ncu compute units; `part` holds gram_part_bytes(lp, ncu_cap)
// bytes for any ncu <= ncu_cap.
size_t gram_part_bytes(int lp, int ncu_cap);
hipError_t launch_gram(bool y_f32, const void* Y, int64_t ldy, int64_t rows, int l, int lp,
                       double* Gm, int64_t ldg, double* part, int ncu, hipStream_t s);
// Q = Y R^{-1} (M x l); Y and Q may be FP32 or FP64; arithmetic in FP64.
// With skip_part (the lp/16 parts of ||Y^T Y - I||_F^2 left by the
// near-identity Cholesky), Q = Y when their sum is at most 2^-60.
hipError_t launch_trsm(bool y_f32, bool q_f32, const void* Y, int64_t ldy, int64_t M, int l,
                       int lp, const double* R, int64_t ldr, const double* Rdinv, void* Q,
                       int64_t ldq, hipStream_t s, const double* skip_part = nullptr);
// overwrite the columns j with dep[j] != 0 of Q (M rows) by N(0, 1/M) values
hipError_t launch_replace(bool q_f32, void* Q, int64_t ldq, int64_t M, int l, const int32_t* dep,
                          uint64_t seed, uint32_t call, hipStream_t s);
// C = A B for upper-triangular lp x lp matrices; rows k of B with bdep[k] != 0
// (bdep may be null) are taken as zero
hipError_t launch_trmm_upper(const double* A, int64_t lda, const double* B, int64_t ldb,
                             const int32_t* bdep, double* C, int64_t ldc, int lp, hipStream_t s);
hipError_t launch_set_word(int32_t* w, int32_t v, hipStream_t s);
// T = Y - T (rows x cols; Y FP32 or FP64, T FP64)
hipError_t launch_rsub(bool y_f32, const void* Y, int64_t ldy, double* T, int64_t ldt,
                       int64_t rows, int cols, hipStream_t s);
// rows j < l of R with dep[j] != 0 set to zero (R lp x lp)
hipError_t launch_zero_dep_rows(double* R, int64_t ldr, int l, int lp, const int32_t* dep,
                                hipStream_t s);

// ---------------------------------------------------------------- jacobi --
// work: jacobi_work_bytes(l) bytes; sweeps_out (device int, may be null)
// receives the number of sweeps of the block iteration.  The block iteration
// (l > 64) waits across at most 8 workgroups of one ordinary launch (bounded
// spins, INFO_BARRIER on give-up): the caller keeps that many CUs free of
// other waiting kernels.  giveup_test: every cross-workgroup wait waits for a
// value no workgroup posts, with a small spin cap (failure-handling tests).
size_t jacobi_work_bytes(int l);
hipError_t launch_jacobi(const double* Rh, int64_t ldr, int l, int k, double* work, double* S,
                         double* Uh, int64_t lduh, double* Vh, int64_t ldvh, int max_sweeps,
                         int32_t* info, int32_t* sweeps_out, bool giveup_test, hipStream_t s);

// ------------------------------------------------------------------ cpqr --
struct CpqrPlan {
  int G;
  int64_t cs;
  int rp, rpl;                       // LDS column stride, rows per lane / 16
  size_t lds;
  int64_t slot_len;
  bool ok;
};
CpqrPlan plan_cpqr(int r, int64_t c, int k, int ncu);
size_t cpqr_work_bytes(const CpqrPlan& p);
// The p.G workgroups of one ordinary launch wait for each other at every step
// (bounded spins, INFO_BARRIER on give-up): p.G must fit in CUs not held by
// other waiting kernels (one workgroup per CU).  giveup_test as for
// launch_jacobi.
hipError_t launch_cpqr(bool b_f32, const void* Bt, int64_t ldb, int r, int64_t c, int k,
                       const CpqrPlan& p, void* work, int64_t* J, double* S11t, double* S12t,
                       int64_t lds, double* pivn, int32_t* info, bool giveup_test,
                       hipStream_t s);
// X = S^{-1} B by back substitution (k <= 256); a zero pivot S_ii gives x_i = 0
hipError_t launch_backsub(const double* S, int64_t s_r, int64_t s_c, const double* Bm,
                          int64_t b_r, int64_t b_c, int k, int64_t nrhs, double* X, int64_t x_r,
                          int64_t x_c, hipStream_t s);

// --------------------------------------------------------------- lowrank --
// P = sum_t X_t W_t^T over count terms (X_t m x l, W_t n x l, row-major with
// leading dimensions ldx / ldw; columns >= l are not read), FP64.
constexpr int LR_MAX = 18;       // 2q + 2 terms of the derivative for q <= 8
struct LowRank {
  const double* X[LR_MAX];
  const double* W[LR_MAX];
  int64_t ldx, ldw;
  int count, l;
};
// number of partial sums written by the norm modes (the size of `part`)
int64_t lowrank_tiles(int64_t m, int64_t n);
// out = P + 2 dres[0] A (the A term only when dres is not null); out m x n
hipError_t launch_lowrank_out(const LowRank& t, int64_t m, int64_t n, const double* A,
                              int64_t lda, const double* dres, double* out, int64_t ldo,
                              hipStream_t st);
// *norm2 = ||A - P||_F^2, with A = A - P written when store is true
hipError_t launch_lowrank_sub(const LowRank& t, int64_t m, int64_t n, double* A, int64_t lda,
                              bool store, double* part, double* norm2, hipStream_t st);

// -------------------------------------------------------------------- qb --
// A -= Q Bt^T (A m x n in place, Q m x b, Bt n x b; b <= 256) and
// *norm2 = ||A||_F^2 of the result; part holds qb_update_tiles(m, n) doubles.
int64_t qb_update_tiles(int64_t m, int64_t n);
hipError_t launch_qb_update(double* A, int64_t lda, int64_t m, int64_t n, const double* Q,
                            int64_t ldq, const double* Bt, int64_t ldbt, int b, double* part,
                            double* norm2, hipStream_t s);
// *norm2 = ||A - Q Bt^T||_F^2 without writing A (part as above)
hipError_t launch_resid2(const double* A, int64_t lda, int64_t m, int64_t n, const double* Q,
                         int64_t ldq, const double* Bt, int64_t ldbt, int b, double* part,
                         double* norm2, hipStream_t s);
// B[t][c] = Bt[c][t] (t < b, c < n)
hipError_t launch_transpose(const double* Bt, int64_t ldbt, int64_t n, int b, double* B,
                            int64_t ldb, hipStream_t s);
// X -= Y (rows x cols)
hipError_t launch_sub(double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t rows,
                      int cols, hipStream_t s);

// ------------------------------------------------------------------ grad --
// Reverse-mode pieces of the randomized SVD (FP64).
// out = (F o (Pu - Pu^T)) S + diag(ds) + S (F o (Pv - Pv^T)), F_ij = 1/(s_j^2 - s_i^2),
// ds_i = dS_i (i < k; dS may be null) - 2 dres[0] s_i (dres, a device scalar, may be null)
hipError_t launch_svd_inner(const double* Pu, const double* Pv, int64_t ldp, const double* s,
                            const double* dS, int k, const double* dres, int l, double* out,
                            int64_t ldo, hipStream_t st);
// Mc = copyltu(-P + Qm) (Qm may be NULL), l x l, P and Qm with leading dimension ld
hipError_t launch_copyltu(const double* P, const double* Qm, int64_t ld, int l, double* Mc,
                          int64_t ldm, hipStream_t st);
// X = 0 (rows x cols)
hipError_t launch_zero(double* X, int64_t ldx, int64_t rows, int cols, hipStream_t st);
// X += Y (rows x cols)
hipError_t launch_add(double* X, int64_t ldx, const double* Y, int64_t ldy, int64_t rows,
                      int cols, hipStream_t st);

// ----------------------------------------------------------------- batch --
// Batched randomized SVD of small FP32 matrices, one workgroup per matrix in
// one persistent launch.
constexpr int BATCH_MAX_LP = 80;     // l = min(k + p, m, n) <= 80
constexpr int BATCH_VARIANTS = 3;    // pass shapes of the batch kernel
struct BatchDesc {
  int64_t m, n, lda;                 // A_i: m x n row-major, lda % 4 == 0
  int64_t a_off, u_off, v_off, s_off;   // element offsets in the packed A, U, V, S
  int32_t k, l, lp, index;           // index: position in the caller's list
  int32_t variant, pad;              // pass shape (0 .. BATCH_VARIANTS - 1)
};
struct BatchArgs {
  const BatchDesc* desc;             // in work-queue order
  int64_t count;
  int32_t* counter;                  // work-queue head (reset by the launcher)
  const float* A;
  float* U;
  double* S;
  float* V;
  char* scratch;                     // one slot of slot_bytes per workgroup
  int64_t slot_bytes;
  int64_t off_om, off_y, off_q, off_z, off_zq, off_t, off_qh, off_uh, off_vh;
  uint32_t k0, k1;                   // seed words
  int q;
  int32_t* info;
};
hipError_t launch_batch_rsvd(const BatchArgs& g, int grid, hipStream_t st);

// ------------------------------------------------------------------- cur --
// atype: element type of A, 0 FP64, 1 FP32, 2 BF16
hipError_t launch_gather_cols(int atype, const void* A, int64_t lda, int64_t m, int64_t n,
                              const int64_t* J, int k, double* Crow, int64_t ldc, hipStream_t s);
hipError_t launch_gather_rows_t(int atype, const void* A, int64_t lda, int64_t m, int64_t n,
                                const int64_t* Jr, int k, double* Rt, int64_t ldr, hipStream_t s);
// indices outside [0, in_rows) give zero rows (defensive; they never occur
// when the pivoted QR succeeded)
hipError_t launch_pick_rows(const double* In, int64_t ldi, int64_t in_rows, const int64_t* J,
                            int64_t rows, int cols, double* Out, int64_t ldo, bool add,
                            hipStream_t s);
hipError_t launch_convert(const float* in, int64_t ldi, int64_t rows, int cols, double* out,
                          int64_t ldo, hipStream_t s);

}  // namespace rsvd
