/* rsvd.h -- randomized SVD, interpolative (ID) and CUR decompositions on one
 * AMD Instinct MI355X (gfx950), after Voronin & Martinsson, "RSVDPACK:
 * Implementations of randomized algorithms for computing the singular value,
 * interpolative, and CUR decompositions of matrices on multi-core and GPU
 * architectures" (arXiv:1502.05366).
 *
 * Entry points: the decompositions (rsvd_svd, rsvd_id, rsvd_id_left, rsvd_cur,
 * rsvd_decompose, rsvd_qb), the reverse-mode derivative of the randomized
 * SVD (rsvd_svd_grad), the batched randomized SVD of many small FP32
 * matrices (rsvd_batch_*), and single steps of the path (rsvd_sketch,
 * rsvd_philox, rsvd_pass, rsvd_orth, rsvd_small_svd, rsvd_cpqr).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All matrix pointers are DEVICE pointers; the caller allocates every
 *   input, output and workspace buffer.  The library allocates nothing per
 *   call.  The handle holds per-device facts and a second stream with two
 *   events, on which rsvd_decompose runs the SVD post-processing beside the
 *   ID / CUR post-processing (forked from and joined back into `stream`); a
 *   handle must not be used by two host threads at once.
 * - Matrices are row-major: element (i, j) of an r x c matrix X with leading
 *   dimension ldx (>= c) is X[i * ldx + j].  Index outputs are 0-based int64.
 * - `dtype` selects the storage and pass precision of A (and of the
 *   range-finder matrices): RSVD_F64, RSVD_F32, or RSVD_BF16 (mixed
 *   precision: A holds BF16 bit patterns (uint16), lda % 8 == 0 and A
 *   16-byte aligned; the passes run on the BF16 matrix cores with FP32
 *   accumulation, the range-finder matrices and U, V are FP32, and the last
 *   projection B^T = A^T Q applies Q as the sum of two BF16 terms).  Gram
 *   matrices, Cholesky factors, the small SVD and the pivoted QR always run
 *   in FP64.  The step entry points other than rsvd_pass take F64 / F32.
 * - All work is enqueued on `stream` (a hipStream_t, may be NULL for the null
 *   stream); nothing synchronizes with the host.  Buffers must stay valid
 *   until the stream has passed the call.
 * - Return value (synchronous): RSVD_OK, -i when the i-th argument is invalid
 *   (1-based, LAPACK convention), or a positive RSVD_ERR_* code.
 * - Numerical status (asynchronous) goes to the device words info[0..1]:
 *   info[0] is a bit set of RSVD_INFO_*, info[1] the numerical rank found by
 *   the pivoted QR when RSVD_INFO_RANK is set.  Each call resets both words.
 * - l = min(k + p, m, n) is the sample size: l <= 576 for the randomized SVD
 *   and its steps (orth works on column blocks of at most 256 above 256),
 *   l <= 256 when the ID or CUR is requested, for the derivative and the
 *   blocked QB, l <= 80 in a batch.  p >= 0, q >= 0, 1 <= k <= min(m, n).
 * - Co-residency: the pivoted QR (ID, CUR) and the block Jacobi (l > 64) run
 *   as ordinary launches of up to one workgroup per compute unit whose
 *   workgroups wait for each other with bounded spins.  They assume the
 *   call's kernels are not starved of compute units by concurrent kernels on
 *   other streams; if a wait gives up, the call reports RSVD_INFO_BARRIER and
 *   its outputs are invalid.  rsvd_decompose with both the SVD and the ID or
 *   CUR runs the Jacobi beside the pivoted QRs and keeps 8 compute units for
 *   it, so it needs the whole device.
 * - The Gaussian test matrix is drawn from Philox4x32-10 (key = seed) with
 *   Box-Muller normals: sketch entry (i, j) is normal number j*n + i of
 *   stream 0 (see rsvd_sketch).
 */
#ifndef RSVD_H_
#define RSVD_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { RSVD_F64 = 0, RSVD_F32 = 1, RSVD_BF16 = 2, RSVD_F8E4M3 = 3 } rsvd_dtype_t;

enum {
  RSVD_OK = 0,
  RSVD_ERR_HIP = 1,         /* a HIP call failed (launch or device query)       */
  RSVD_ERR_WORKSPACE = 2,   /* work_bytes smaller than the workspace query      */
  RSVD_ERR_UNSUPPORTED = 3, /* valid arguments outside what this build supports */
  RSVD_ERR_NO_DEVICE = 4,   /* no HIP device with the requested index           */
  RSVD_ERR_SCRATCH = 5      /* the call needs more than RSVD_NOALLOC_MAX_BYTES  */
};

enum {
  RSVD_INFO_ORTH_FALLBACK = 1, /* orth met a numerically dependent column and
                                  replaced it by a random one (rank-deficient Y) */
  RSVD_INFO_JACOBI_CAP = 2,    /* the Jacobi SVD stopped at its sweep cap        */
  RSVD_INFO_RANK = 4,          /* pivoted QR residual fell below the rank
                                  tolerance before step k; info[1] = that step   */
  RSVD_INFO_NONFINITE = 8,     /* NaN or Inf met in a Gram matrix                */
  RSVD_INFO_BARRIER = 16       /* internal: a grid barrier hit its spin cap      */
};

typedef struct rsvd_handle_s* rsvd_handle_t;
typedef struct rsvd_batch_s* rsvd_batch_t;

/* Operation selector of rsvd_workspace_bytes. */
enum { RSVD_OP_SVD = 1, RSVD_OP_ID = 2, RSVD_OP_CUR = 4 };

/* Create a handle for HIP device `device` (queries its compute-unit count).
 * Returns RSVD_ERR_NO_DEVICE if it does not exist. */
int rsvd_create(rsvd_handle_t* handle, int device);
int rsvd_destroy(rsvd_handle_t handle);
const char* rsvd_status_string(int code);

/* Options of a handle, for the calls made through it afterwards:
 *   RSVD_OPT_JACOBI_MAX_SWEEPS (1..1000, default 40): sweep cap of the Jacobi
 *     SVD of the small factor; stopping at the cap sets RSVD_INFO_JACOBI_CAP.
 *   RSVD_OPT_TEST_WAIT_GIVEUP (0 or 1, default 0): failure-handling test
 *     mode.  The kernels whose workgroups wait for each other (the pivoted QR
 *     and the block Jacobi, l > 64) then wait for a value that no workgroup
 *     posts, with a small spin cap, so every wait gives up: the kernels run
 *     to their end, the call reports RSVD_INFO_BARRIER and its outputs are
 *     invalid (J then lists the columns in order).
 * Returns -2 for an unknown option, -3 for a value out of range. */
enum { RSVD_OPT_JACOBI_MAX_SWEEPS = 1, RSVD_OPT_TEST_WAIT_GIVEUP = 2 };
int rsvd_set_option(rsvd_handle_t h, int option, int value);

/* Bytes of device workspace needed by rsvd_decompose (and rsvd_svd, rsvd_id,
 * rsvd_cur) for the outputs selected by `ops` (a bit set of RSVD_OP_*).
 * Pure host function of its arguments; 0 for invalid arguments. */
size_t rsvd_workspace_bytes(int ops, int dtype, int64_t m, int64_t n, int k, int p, int q);

/* Rank-k randomized SVD, Alg. 5 of the paper (RSVD Version II) with the
 * power scheme of Sec. 3.2 re-orthonormalized after every product (s = 1):
 *   Y = A Omega;  q times { Q = orth(Y); Z = A^T Q; Z = orth(Z); Y = A Z };
 *   Q = orth(Y);  B^T = A^T Q;  [Qh, Rh] = qr(B^T);  Rh = Uh diag(S) Vh^T;
 *   U = Q Vh(:, 1:k),  V = Qh Uh(:, 1:k).
 * A: m x n (lda >= n).  U: m x k (ldu >= k), V: n x k (ldv >= k), both of the
 * type of A (FP32 for RSVD_BF16).  S: k FP64 values, descending.
 * A ~ U diag(S) V^T. */
int rsvd_svd(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
             uint64_t seed, const void* A, int64_t lda, void* U, int64_t ldu, double* S,
             void* V, int64_t ldv, void* work, size_t work_bytes, int32_t* info,
             void* stream);

/* rsvd_svd with the two additions of the mixed-precision path (Alg. 5; the
 * re-orthonormalization of Sec. 3.2 between the narrow passes):
 *  - dtype RSVD_F8E4M3: A holds FP8 E4M3 codes (uint8, lda % 16 == 0, A
 *    16-byte aligned) and a_col_scale the n FP32 column scales s_j, so that A
 *    stands for A8 diag(s) (rsvd_quantize makes both from an FP64 A).  For the
 *    products Y = A X the scales are folded into X before X is quantized to
 *    E4M3 per column; for Z = A^T X they scale the rows of the result.  The
 *    passes run on the FP8 matrix cores (FP32 accumulation) and the last
 *    projection B^T = A^T Q applies Q as the sum of two E4M3 terms.
 *    a_col_scale must be NULL for the other dtypes (else -11).
 *  - Qb (optional, m x l with ldqb >= l, type FP64 for RSVD_F64 and FP32
 *    otherwise): the orthonormal basis Q of the range finder (Alg. 5 up to
 *    Q = orth(Y)), from which B = Q^T A.
 * RSVD_F8E4M3 is accepted only here (rsvd_svd_ex) and by rsvd_pass_f8; the
 * workspace is rsvd_workspace_bytes(RSVD_OP_SVD, dtype, ...). */
int rsvd_svd_ex(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
                uint64_t seed, const void* A, int64_t lda, const float* a_col_scale, void* U,
                int64_t ldu, double* S, void* V, int64_t ldv, void* Qb, int64_t ldqb, void* work,
                size_t work_bytes, int32_t* info, void* stream);

/* The storage formats of the mixed-precision path, from an FP64 A (m x n,
 * lda >= n) into Aq (ldq >= n):
 *  - RSVD_BF16: Aq (uint16) holds each entry rounded to the nearest BF16
 *    value, ties to even, directly from FP64 (col_scale unused, may be NULL);
 *  - RSVD_F8E4M3: col_scale[j] = fl32(max_i |A_ij| / 448) (1 for a zero
 *    column) and Aq (uint8) the E4M3 code of the FP64 quotient A_ij /
 *    col_scale[j], nearest with ties to even, saturated to +-448 (the OCP
 *    E4M3 format: no infinities, largest finite 448).
 * Both are exact decisions on FP64 values (bit-reproducible). */
int rsvd_quantize(rsvd_handle_t h, int dtype, int64_t m, int64_t n, const double* A, int64_t lda,
                  void* Aq, int64_t ldq, float* col_scale, void* stream);

/* rsvd_svd without a workspace argument, for callers that cannot allocate
 * device memory (code under stream capture, tight serving loops): the call
 * allocates nothing and uses a static scratch array of RSVD_NOALLOC_MAX_BYTES
 * (64 MiB) in device memory instead, one copy per device that loads the
 * library, held until the process ends.  Same arguments (without work,
 * work_bytes), outputs and errors as rsvd_svd, plus RSVD_ERR_SCRATCH when the
 * problem needs more scratch than that: rsvd_svd_noalloc_bytes(...) returns
 * the need (0 for invalid sizes).  Every call on a device shares that device's
 * scratch and leaves its contents behind, so calls that overlap on one device
 * (two streams, two host threads) race and must not be issued. */
#define RSVD_NOALLOC_MAX_BYTES ((size_t)64 << 20)
size_t rsvd_svd_noalloc_bytes(int dtype, int64_t m, int64_t n, int k, int p, int q);
int rsvd_svd_noalloc(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
                     uint64_t seed, const void* A, int64_t lda, void* U, int64_t ldu, double* S,
                     void* V, int64_t ldv, int32_t* info, void* stream);

/* Rank-k column ID computed from B = Q^T A (Sec. 3.5, last part; Alg. 1 on B):
 * k steps of column-pivoted QR of B give the skeleton J[0..k) (pivot order)
 * and T = S11^{-1} S12 (Sec. 2.4).  J: n int64, J[k..n) are the remaining
 * columns in ascending order.  T: k x (n-k) FP64 (ldt >= n-k), its column j
 * belongs to column J[k+j] of A.  With V = P [I_k; T^T] (V[J[i], :] = e_i,
 * V[J[k+j], :] = T(:, j)^T), A ~ A(:, J[0..k)) V^T.  When the numerical rank
 * is below k (RSVD_INFO_RANK), an exactly zero pivot of S11 gives a zero row
 * of T. */
int rsvd_id(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
            uint64_t seed, const void* A, int64_t lda, int64_t* J, double* T, int64_t ldt,
            void* work, size_t work_bytes, int32_t* info, void* stream);

/* Rank-k column ID with the Gaussian sketch on the left (Sec. 3.5, Alg. 6):
 * the sample Y = Omega~ A (A^T A)^q of eq. (Ypower), (k+p) x n, formed with the
 * columns orthonormalized before every product (the listing after that
 * equation):  Y^T = A^T Omega~^T;  q times { Y^T = A orth(Y^T);
 * Y^T = A^T orth(Y^T) };  then k steps of column-pivoted QR of Y and
 * T = S11^{-1} S12.  Omega~^T (m x (k+p)) holds normal number j*m + i of
 * Philox stream 6 at (i, j).  Arguments, outputs (J, T) and errors as for
 * rsvd_id; the workspace is rsvd_id_left_workspace_bytes(...) bytes.  Passes
 * over A: 2q + 1. */
size_t rsvd_id_left_workspace_bytes(int dtype, int64_t m, int64_t n, int k, int p, int q);
int rsvd_id_left(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
                 uint64_t seed, const void* A, int64_t lda, int64_t* J, double* T, int64_t ldt,
                 void* work, size_t work_bytes, int32_t* info, void* stream);

/* Blocked adaptive QB decomposition (Sec. 3.3, Alg. 7), FP64 only.  For
 * block i = 0, 1, ..: Omega_i (n x b) = normal numbers of Philox stream 5
 * with batch index i (Omega_i[r][j] = number j*n + r);
 *   Q_i = orth(A Omega_i);  q times { Q_i = orth(A^T Q_i); Q_i = orth(A Q_i) };
 *   Q_i = orth(Q_i - Qbar Qbar^T Q_i)  (Qbar = Q_0 .. Q_{i-1});
 *   B_i = Q_i^T A;  A = A - Q_i B_i;
 * and the loop stops after block i when ||A||_F < tol, or after M blocks.
 * A (m x n, lda >= n) is overwritten by the deflated residual A - Q B.
 * Q: m x (b*M) (ldq >= b*M) and B: (b*M) x n (ldb >= n), FP64; their first
 * b * (*nblocks) columns / rows hold the result, A_in ~ Q B.
 * *nblocks (host) = blocks used; *resid (host, may be NULL) = ||A - Q B||_F.
 * 1 <= b <= 256, b*M <= min(m, n), q >= 0, tol >= 0.  The call synchronizes
 * `stream` once per block to test the stopping rule.  Workspace:
 * rsvd_qb_workspace_bytes(...) bytes (0 for invalid sizes); FP32 and BF16
 * return RSVD_ERR_UNSUPPORTED. */
size_t rsvd_qb_workspace_bytes(int dtype, int64_t m, int64_t n, int b, int M, int q);
int rsvd_qb(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int b, int M, int q, double tol,
            uint64_t seed, void* A, int64_t lda, double* Q, int64_t ldq, double* B, int64_t ldb,
            int32_t* nblocks, double* resid, void* work, size_t work_bytes, int32_t* info,
            void* stream);

/* Reverse-mode derivative of the rank-k randomized SVD with the Gaussian sketch
 * held fixed (FP64 only; q <= 8).  The forward map is the one of rsvd_svd
 * (Alg. 5, re-orthonormalization after every product as in Sec. 3.2; the small
 * SVD from the QR of B^T as in Sec. 3.4): the call recomputes it, keeping its
 * bases and triangular factors in the workspace, so a caller stores only A.
 *
 * Cotangents (device pointers, each may be NULL for zero): dU (m x k, lddu),
 * dS (k), dV (n x k, lddv), dres (one double: the cotangent of
 * resid2 = ||A - Q Q^T A||_F^2, Q the basis of the range finder).  With dA
 * non-NULL (m x n, ldda >= n) the call writes
 *   dA = d/dA [ <dU, U> + <dS, S> + <dV, V> + dres * resid2 ],
 * the adjoint of every product with A (dA += dC X^T, dX = A^T dC), of every
 * thin QR Y = Q R (dY = (dQ + Q copyltu(R dR^T - dQ^T Q)) R^{-T}) and of the
 * SVD of the l x l factor (the 1 / (s_j^2 - s_i^2) formula).  The map is
 * differentiable where the Y's have full rank and the l singular values of the
 * small factor are distinct and non-zero; elsewhere dA is not finite.
 * Forward outputs, each optional: U (m x k, ldu), S (k), V (n x k, ldv) (the
 * same values as rsvd_svd with this seed) and resid2 (one double, formed as
 * the sum of squares of A - Q B).  At least one of dA, U, S, V, resid2 must
 * be non-NULL.  A is not modified; it must not overlap dA.
 * F32 / BF16: RSVD_ERR_UNSUPPORTED.  Workspace: rsvd_svd_grad_workspace_bytes
 * (0 for invalid sizes). */
size_t rsvd_svd_grad_workspace_bytes(int dtype, int64_t m, int64_t n, int k, int p, int q);
int rsvd_svd_grad(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
                  uint64_t seed, const double* A, int64_t lda, const double* dU, int64_t lddu,
                  const double* dS, const double* dV, int64_t lddv, const double* dres,
                  double* dA, int64_t ldda, double* U, int64_t ldu, double* S, double* V,
                  int64_t ldv, double* resid2, void* work, size_t work_bytes, int32_t* info,
                  void* stream);

/* Batched randomized SVD: `count` independent FP32 matrices A_i (m_i x n_i,
 * rank k_i, the same p and q), each decomposed as by rsvd_svd (Alg. 5 with
 * re-orthonormalization after every product, Sec. 3.2; the small SVD from the
 * QR of B_i^T) in one persistent launch: the workgroups take matrices from a
 * work queue in decreasing order of work, one matrix per workgroup at a time
 * (the matrices are independent, as the blocks of Alg. 8 are).  Omega_i is
 * Philox stream 0 with batch index i under the call's seed.  Limits:
 * l_i = min(k_i + p, m_i, n_i) <= 80.  Products on the FP32 matrix cores
 * (FP32 accumulation); orth (CholeskyQR2), the Jacobi SVD and U, V in FP64.
 * A column that the orth finds dependent (Cholesky pivot below 1e-13 G_jj)
 * is replaced by a fresh Gaussian column (Philox stream 7) before the second
 * CholeskyQR pass, as in rsvd_orth, and sets info bit 1; a non-finite pivot
 * sets info bit 8.
 *
 * rsvd_batch_create: host arrays m, n (int64) and k (int32) of `count`
 *   entries; the plan keeps its own copy.  Codes: -i for an invalid i-th
 *   argument, RSVD_ERR_UNSUPPORTED when some l_i exceeds 80.
 * rsvd_batch_layout: the packed layouts (host outputs, each may be NULL):
 *   A_i at element a_off[i] of one FP32 buffer, row-major with leading
 *   dimension lda[i] = n_i rounded up to a multiple of 4 (the buffer must be
 *   16-byte aligned); U_i (m_i x k_i FP32, ld k_i) at u_off[i]; S_i (k_i FP64,
 *   descending) at s_off[i]; V_i (n_i x k_i FP32, ld k_i) at v_off[i]; the
 *   totals in a_elems, u_elems, s_elems, v_elems.
 * rsvd_batch_prepare: copies the plan's descriptor table into the workspace
 *   (rsvd_batch_workspace_bytes bytes, 256-byte aligned) and synchronizes the
 *   stream; once per workspace, outside any stream capture.
 * rsvd_batch_svd: launches only kernels (a queue reset and the persistent
 *   kernel), so it may be captured into a graph and replayed; calls that
 *   share a workspace must not overlap.  `work` must be the workspace last
 *   passed to rsvd_batch_prepare for this plan (-7 otherwise).  info (2
 *   int32, device) as for the other calls. */
int rsvd_batch_create(rsvd_handle_t h, int64_t count, const int64_t* m, const int64_t* n,
                      const int32_t* k, int p, int q, rsvd_batch_t* plan);
int rsvd_batch_destroy(rsvd_batch_t plan);
int rsvd_batch_layout(rsvd_batch_t plan, int64_t* a_elems, int64_t* u_elems, int64_t* s_elems,
                      int64_t* v_elems, int64_t* a_off, int64_t* lda, int64_t* u_off,
                      int64_t* s_off, int64_t* v_off);
size_t rsvd_batch_workspace_bytes(rsvd_batch_t plan);
/*
 * rsvd_batch_set_variants: the shape of the passes over A for each matrix
 *   (host int32 array of `count`, caller order), each in
 *   0 .. RSVD_BATCH_VARIANTS - 1: 0 = 128-row tiles of A with 64-deep chunks,
 *   1 = 256-row tiles with 32-deep chunks, 2 = 128-row tiles with 32-deep
 *   chunks (A^T passes: columns).  A shape changes only the order of the FP32
 *   sums of the passes.  Plans start at shape 0; the package's autotuner
 *   measures the shapes per (m, n, l) bucket and stores the fastest in a
 *   table that its BatchPlan applies.  The descriptors travel with
 *   rsvd_batch_prepare, so call it again afterwards (rsvd_batch_svd returns
 *   -7 until then).  Returns -2 on a NULL array or a value out of range.
 */
#define RSVD_BATCH_VARIANTS 3
int rsvd_batch_set_variants(rsvd_batch_t plan, const int32_t* variant);
int rsvd_batch_prepare(rsvd_batch_t plan, void* work, size_t work_bytes, void* stream);
int rsvd_batch_svd(rsvd_batch_t plan, uint64_t seed, const float* A, float* U, double* S, float* V,
                   void* work, size_t work_bytes, int32_t* info, void* stream);

/* Rank-k CUR from the two-sided ID (Sec. 2.5, Alg. 3; Sec. 3.6): Jc = skeleton
 * columns of the ID above, Jr = the k rows chosen by k steps of column-pivoted
 * QR of C^T (C = A(:, Jc)), and Ucur = V^T R^dagger (k x k FP64, lduc >= k),
 * the least-squares solution of Ucur R = V^T with R = A(Jr, :):
 * A ~ A(:, Jc) Ucur A(Jr, :). */
int rsvd_cur(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
             uint64_t seed, const void* A, int64_t lda, int64_t* Jc, int64_t* Jr,
             double* Ucur, int64_t lduc, void* work, size_t work_bytes, int32_t* info,
             void* stream);

/* One range finder, then any of the three decompositions of the same B.
 * Output groups may be NULL to skip them: (U, S, V) for the SVD, (J, T) for
 * the ID, (Jr, Ucur) for the CUR (the CUR needs the ID, which is then computed
 * into the workspace when J/T are NULL; Jc = J[0..k)).  The workspace query
 * must be made with the same set of ops.  With the SVD and the ID / CUR both
 * requested, the Jacobi runs on the handle's second stream beside the pivoted
 * QRs, and the two wait-across-workgroup kernels together hold every compute
 * unit: no other work may run on the device meanwhile (see co-residency). */
int rsvd_decompose(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
                   uint64_t seed, const void* A, int64_t lda, void* U, int64_t ldu,
                   double* S, void* V, int64_t ldv, int64_t* J, double* T, int64_t ldt,
                   int64_t* Jr, double* Ucur, int64_t lduc, void* work, size_t work_bytes,
                   int32_t* info, void* stream);

/* ------------------------------------------------------------------------
 * Single steps of the path, exposed so that each can be checked on its own.
 * ------------------------------------------------------------------------ */

/* The n x l Gaussian test matrix (Fig. 1 step 1): Omega[i * ldo + j] = normal
 * number j*n + i of stream 0, rounded to dtype; columns l..ldo-1 are zeroed. */
int rsvd_sketch(rsvd_handle_t h, int dtype, uint64_t seed, int64_t n, int64_t l, void* Omega,
                int64_t ldo, void* stream);

/* Raw Philox4x32-10 words: out[4*i + r] = word r for counter
 * (first + i, stream_id, batch) under key = seed.  out: 4*count uint32. */
int rsvd_philox(rsvd_handle_t h, uint64_t seed, uint32_t stream_id, uint32_t batch,
                uint64_t first, int64_t count, uint32_t* out, void* stream);

/* One pass over A on the matrix cores: Y = A X (trans = 0; X n x l, Y m x l)
 * or Y = A^T X (trans = 1; X m x l, Y n x l).  A, X, Y of type dtype; with
 * RSVD_BF16, A is BF16 (lda % 8 == 0, 16-byte aligned, else argument 8 is
 * reported), X and Y are FP32, X is rounded to BF16 in the workspace and
 * l <= 256. */
size_t rsvd_pass_workspace_bytes(int dtype, int trans, int64_t m, int64_t n, int64_t l);
int rsvd_pass(rsvd_handle_t h, int dtype, int trans, int64_t m, int64_t n, int64_t l,
              const void* A, int64_t lda, const void* X, int64_t ldx, void* Y, int64_t ldy,
              void* work, size_t work_bytes, void* stream);

/* orth (Sec. 2.1): Q (rows x l, type dtype) with orthonormal columns and
 * Y = Q R, by CholeskyQR2 in FP64; R (l x l FP64, upper triangular with a
 * positive diagonal, zero below; may be NULL).  A column of Y that depends on
 * the columns before it gets a fresh random direction in Q
 * (RSVD_INFO_ORTH_FALLBACK) and a zero diagonal in R, so Y = Q R still holds
 * to rounding.  rows >= l, l <= 256. */
/* One pass over an FP8 A with column scales (see rsvd_svd_ex): Y = A X
 * (trans = 0; X n x l, Y m x l) or Y = A^T X (trans = 1; X m x l, Y n x l),
 * X and Y FP32, A ~ A8 diag(a_col_scale).  split = 1 applies X as the sum of
 * two E4M3 terms (the second holding the rounding residual of the first).
 * l <= 576. */
size_t rsvd_pass_f8_workspace_bytes(int trans, int64_t m, int64_t n, int64_t l);
int rsvd_pass_f8(rsvd_handle_t h, int trans, int64_t m, int64_t n, int64_t l, const uint8_t* A,
                 int64_t lda, const float* a_col_scale, const float* X, int64_t ldx, float* Y,
                 int64_t ldy, int split, void* work, size_t work_bytes, void* stream);

size_t rsvd_orth_workspace_bytes(int dtype, int64_t rows, int64_t l);
int rsvd_orth(rsvd_handle_t h, int dtype, int64_t rows, int64_t l, const void* Y, int64_t ldy,
              void* Q, int64_t ldq, double* R, int64_t ldr, uint64_t seed, void* work,
              size_t work_bytes, int32_t* info, void* stream);

/* Small SVD of Alg. 5: one-sided Jacobi on an l x l FP64 matrix Rh,
 * Rh = Uh diag(S) Vh^T; the k largest singular values (descending) and the
 * matching columns Uh (l x k, lduh >= k) and Vh (l x k, ldvh >= k). */
size_t rsvd_small_svd_workspace_bytes(int64_t l);
int rsvd_small_svd(rsvd_handle_t h, int64_t l, int k, const double* Rh, int64_t ldr, double* S,
                   double* Uh, int64_t lduh, double* Vh, int64_t ldvh, void* work,
                   size_t work_bytes, int32_t* info, void* stream);

/* k steps of column-pivoted QR of an r x c matrix B given by columns:
 * column j of B is Bcols[j * ldb .. j * ldb + r) (type dtype), i.e. B^T in
 * row-major.  Outputs as in rsvd_id: J (c), T (k x (c-k), ldt), and the pivot
 * norms pivn (k FP64, may be NULL).  k <= min(r, c, 256). */
size_t rsvd_cpqr_workspace_bytes(int64_t r, int64_t c, int k);
int rsvd_cpqr(rsvd_handle_t h, int dtype, int64_t r, int64_t c, int k, const void* Bcols,
              int64_t ldb, int64_t* J, double* T, int64_t ldt, double* pivn, void* work,
              size_t work_bytes, int32_t* info, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RSVD_H_ */
