// C-ABI of the randomized SVD / ID / CUR library: argument checks, workspace
// layout and the order of kernel launches on the caller's stream.
//
// The path (Alg. 5 of the paper with s = 1, then the ID from B of Sec. 3.5 and
// the CUR of Sec. 2.5 / 3.6):
//   Omega = sketch(seed)                      Philox4x32-10 + Box-Muller
//   Y = A Omega                               pass over A
//   q times: Q = orth(Y); Z = A^T Q;          orth = CholeskyQR2 in FP64
//            Zq = orth(Z); Y = A Zq
//   Q = orth(Y); B^T = A^T Q
//   SVD:  [Qh, Rh] = orth(B^T) (keep R); Jacobi: Rh = Uh S Vh^T;
//         U = Q Vh_k, V = Qh Uh_k
//   ID:   k-step CPQR of B -> J, S11, S12; T = S11^{-1} S12
//   CUR:  C = A(:, J_k); k-step CPQR of C^T -> Jr; R = A(Jr, :);
//         R^T = Qt Rt; U = (Qt(J_k, :) + T Qt(J_res, :)) Rt^{-T}
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "rsvd.h"
#include "common.h"
#include "internal.h"

struct rsvd_handle_s {
  int device;
  int ncu;
  // second stream and fork / join events: the SVD post-processing runs
  // beside the ID / CUR post-processing inside rsvd_decompose
  hipStream_t aux;
  hipEvent_t ev_fork, ev_join;
  // options (rsvd_set_option)
  int jacobi_max_sweeps;
  bool giveup_test;
  // this device's copy of the static scratch of rsvd_svd_noalloc
  void* scratch;
};

// Host side of a batch: the per-matrix descriptors in work-queue order and
// the packed layouts of A, U, S, V in the caller's order.
struct rsvd_batch_s {
  rsvd_handle_s* h;
  int64_t count;
  int p, q;
  std::vector<rsvd::BatchDesc> desc;     // queue order (decreasing work)
  std::vector<int64_t> a_off, lda, u_off, s_off, v_off;   // caller order
  int64_t a_elems, u_elems, s_elems, v_elems;
  int64_t mmax, nmax;
  int grid;
  // workspace layout
  int64_t desc_off, slot_off, slot_bytes;
  int64_t off_om, off_y, off_q, off_z, off_zq, off_t, off_qh, off_uh, off_vh;
  size_t work_bytes;
  const void* prepared;                  // the workspace that holds the descriptors
};

// Scratch of rsvd_svd_noalloc: a fixed array in device memory, one copy per
// device that loads the library, held until the process ends.  In host code
// its name is only a stand-in: kernels get the device address that
// hipGetSymbolAddress returns on each device (scratch_addr).
static __device__ __align__(256) char scratch[RSVD_NOALLOC_MAX_BYTES];

namespace rsvd {
namespace {

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_dev[MAX_DEVICES];

// The address of `scratch` on the current device `device`, looked up once per
// device (nullptr when the lookup fails).
void* scratch_addr(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> g(scratch_mu);
  if (!scratch_dev[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    scratch_dev[device] = p;
  }
  return scratch_dev[device];
}

constexpr int MAX_L = 256;          // ID / CUR, derivative, blocked QB
constexpr int MAX_L_SVD = 576;      // randomized SVD and its steps (block Jacobi limit)
constexpr int ORTH_BLOCK = 256;     // orth works on column blocks of at most this many
constexpr int NCU_CAP = 256;          // workspace is sized for at most this many CUs
constexpr double ETA_ORTH = 1e-13;    // Cholesky pivot / G_jj below which a column is dependent
constexpr int JACOBI_MAX_SWEEPS = 40;

struct Arena {
  char* base;
  size_t off;
  explicit Arena(void* b) : base(static_cast<char*>(b)), off(0) {}
  template <typename T> T* take(size_t count) {
    const size_t o = (off + 255) & ~(size_t)255;
    off = o + count * sizeof(T) + 256;
    return base ? reinterpret_cast<T*>(base + o) : nullptr;
  }
};

struct Shape {
  int64_t m, n;
  int k, p, q, l, lp, kp;
  bool f32;       // skinny matrices (Omega, Y, Q, Z) in FP32 (FP32 and BF16 inputs)
  bool bf16;      // A in BF16: passes on the BF16 matrix cores
  bool f8;        // A in FP8 E4M3 with column scales: passes on the FP8 matrix cores
  int atype;      // element type of A: 0 FP64, 1 FP32, 2 BF16
  size_t dsz;
  int ops;
};

Shape make_shape(int ops, int dtype, int64_t m, int64_t n, int k, int p, int q) {
  Shape s;
  s.m = m; s.n = n; s.k = k; s.p = p; s.q = q;
  int64_t l = (int64_t)k + p;
  l = std::min<int64_t>(l, std::min(m, n));
  s.l = (int)l;
  s.lp = (int)rup(l, 16);
  s.kp = (int)rup(k, 16);
  s.bf16 = dtype == RSVD_BF16;
  s.f8 = dtype == RSVD_F8E4M3;
  s.f32 = dtype == RSVD_F32 || s.bf16 || s.f8;
  s.atype = dtype == RSVD_F64 ? 0 : (dtype == RSVD_F32 ? 1 : (dtype == RSVD_BF16 ? 2 : 3));
  s.dsz = s.f32 ? 4 : 8;
  s.ops = ops;
  return s;
}

// FP8 A: its column scales and the buffers of the quantized skinny operand
struct F8Bufs {
  const float* ascale = nullptr;   // n column scales of A
  uint8_t* xt = nullptr;           // 2 x lp x rup(max(m, n), 16) codes (two terms)
  float* t = nullptr;              // 2 x lp column scales of the two terms
  uint32_t* tmax = nullptr;        // lp words
};

// buffers of one orth (CholeskyQR2) call
struct OrthBufs {
  double *G = nullptr, *R1 = nullptr, *R2 = nullptr, *Rd1 = nullptr, *Rd2 = nullptr,
         *Qa = nullptr;
  int32_t *dep = nullptr, *dep2 = nullptr;
  double* nip = nullptr;  // lp/16 parts of ||G - I||_F^2 of the second Gram matrix
  void* part = nullptr;
  size_t part_bytes = 0;
  double* gpart = nullptr;  // partial Gram tiles, gram_part_bytes(lp, NCU_CAP)
  // l > ORTH_BLOCK (column blocks): the projected block T (rows x ORTH_BLOCK) and
  // the coefficients W, W2 and W2 R1 (lp x ORTH_BLOCK)
  double *T = nullptr, *W = nullptr, *W2 = nullptr, *P2 = nullptr;
};

struct Bufs {
  void *Om, *Y, *Q, *Z, *Zq;
  uint16_t* Xt;            // BF16 passes: the skinny operand, rounded and transposed
  F8Bufs f8;               // FP8 passes (ascale set per call)
  double *Qh, *Rh, *Wj, *Uh, *Vh;
  OrthBufs ob;
  // ID
  void* cq_work;
  int64_t* J;
  double *S11t, *S12t, *pivn, *T;
  // CUR (its orth and small products run beside the SVD branch: own buffers)
  OrthBufs ob2;
  double* Crow;
  void* cq2_work;
  int64_t* J2;
  double *S11t2, *S12t2, *pivn2, *Rt, *Qt, *Rtt, *Qres, *Mb;
};

// partial tiles of the products of the block orth of a rows x l matrix
size_t orth_block_part_bytes(int64_t rows, int l) {
  if (l <= ORTH_BLOCK) return 0;
  const int nblk = (int)cdiv(l, ORTH_BLOCK);
  const int bs = (int)rup(cdiv(l, nblk), 16);
  size_t b = 0;
  for (int c0 = bs; c0 < l; c0 += bs) {
    const int bj = std::min(bs, l - c0);
    b = std::max(b, gemm_part_bytes(plan_gemm(c0, rows, bj, NCU_CAP, 0), 8));
    b = std::max(b, gemm_part_bytes(plan_gemm(rows, c0, bj, NCU_CAP, 0), 8));
    b = std::max(b, gemm_part_bytes(plan_gemm(c0, bj, bj, NCU_CAP, 0), 8));
  }
  return b;
}

size_t max_part(const Shape& s) {
  const int ncu = NCU_CAP;
  size_t b = std::max(orth_block_part_bytes(s.m, s.l), orth_block_part_bytes(s.n, s.l));
  auto upd = [&](int64_t M, int64_t K, int64_t L) {
    if (M <= 0 || K <= 0 || L <= 0) return;
    b = std::max(b, gemm_part_bytes(plan_gemm(M, K, L, ncu, 0), 8));
  };
  upd(s.m, s.n, s.l);
  upd(s.n, s.m, s.l);
  if (!s.bf16 && !s.f8) {
    b = std::max(b, narrow_work_bytes(s.f32, false, s.m, s.n, s.l, ncu));
    b = std::max(b, narrow_work_bytes(s.f32, true, s.n, s.m, s.l, ncu));
  }
  if (s.bf16) {
    b = std::max(b, gemm_bf16_part_bytes(plan_gemm_bf16(s.m, s.n, s.l, ncu)));
    b = std::max(b, gemm_bf16_part_bytes(plan_gemm_bf16(s.n, s.m, s.l, ncu)));
  }
  if (s.f8) {
    b = std::max(b, gemm_f8_part_bytes(plan_gemm_f8(s.m, s.n, s.l, ncu)));
    b = std::max(b, gemm_f8_part_bytes(plan_gemm_f8(s.n, s.m, s.l, ncu)));
  }
  upd(s.m, s.l, s.k);
  upd(s.n, s.l, s.k);
  upd(s.k, s.n - s.k, s.k);
  return b;
}

OrthBufs take_orth(Arena& a, int64_t rows, int lp, size_t part_bytes) {
  OrthBufs ob;
  ob.G = a.take<double>((size_t)lp * lp);
  ob.R1 = a.take<double>((size_t)lp * lp);
  ob.R2 = a.take<double>((size_t)lp * lp);
  ob.Rd1 = a.take<double>((size_t)lp * 16);
  ob.Rd2 = a.take<double>((size_t)lp * 16);
  ob.Qa = a.take<double>((size_t)rows * lp);
  ob.dep = a.take<int32_t>(lp);
  ob.dep2 = a.take<int32_t>(lp);
  ob.nip = a.take<double>(16);
  ob.part_bytes = part_bytes;
  ob.part = a.take<char>(part_bytes);
  ob.gpart = a.take<double>(gram_part_bytes(lp, NCU_CAP) / sizeof(double));
  if (lp > ORTH_BLOCK) {
    ob.T = a.take<double>((size_t)rows * ORTH_BLOCK);
    ob.W = a.take<double>((size_t)lp * ORTH_BLOCK);
    ob.W2 = a.take<double>((size_t)lp * ORTH_BLOCK);
    ob.P2 = a.take<double>((size_t)lp * ORTH_BLOCK);
  }
  return ob;
}

size_t layout(const Shape& s, void* base, Bufs* out) {
  Arena a(base);
  Bufs b;
  std::memset(&b, 0, sizeof(b));
  const int64_t rmax = std::max(s.m, s.n);
  b.Om = a.take<char>((size_t)s.n * s.lp * s.dsz);
  b.Y = a.take<char>((size_t)s.m * s.lp * s.dsz);
  b.Q = a.take<char>((size_t)s.m * s.lp * s.dsz);
  b.Z = a.take<char>((size_t)s.n * s.lp * s.dsz);
  b.Zq = a.take<char>((size_t)s.n * s.lp * s.dsz);
  if (s.bf16) b.Xt = a.take<uint16_t>((size_t)s.lp * rup(std::max(s.m, s.n), 32));
  if (s.f8) {
    b.f8.xt = a.take<uint8_t>((size_t)2 * s.lp * rup(std::max(s.m, s.n), 16));
    b.f8.t = a.take<float>((size_t)2 * s.lp);
    b.f8.tmax = a.take<uint32_t>((size_t)s.lp);
  }
  b.ob = take_orth(a, rmax, s.lp, max_part(s));
  if (s.ops & RSVD_OP_SVD) {
    b.Qh = a.take<double>((size_t)s.n * s.lp);
    b.Rh = a.take<double>((size_t)s.lp * s.lp);
    b.Wj = a.take<double>(jacobi_work_bytes(s.l) / sizeof(double) + 1);
    b.Uh = a.take<double>((size_t)s.lp * s.kp);
    b.Vh = a.take<double>((size_t)s.lp * s.kp);
  }
  if (s.ops & (RSVD_OP_ID | RSVD_OP_CUR)) {
    const CpqrPlan cp = plan_cpqr(s.l, s.n, s.k, NCU_CAP);
    b.cq_work = a.take<char>(cpqr_work_bytes(cp));
    b.J = a.take<int64_t>(s.n);
    b.S11t = a.take<double>((size_t)s.k * s.kp);
    b.S12t = a.take<double>((size_t)(s.n - s.k + 1) * s.kp);
    b.pivn = a.take<double>(s.k);
    b.T = a.take<double>((size_t)s.k * (s.n - s.k + 1));
  }
  if (s.ops & RSVD_OP_CUR) {
    const CpqrPlan cp2 = plan_cpqr(s.k, s.m, s.k, NCU_CAP);
    b.Crow = a.take<double>((size_t)s.m * s.kp);
    b.cq2_work = a.take<char>(cpqr_work_bytes(cp2));
    b.J2 = a.take<int64_t>(s.m);
    b.S11t2 = a.take<double>((size_t)s.k * s.kp);
    b.S12t2 = a.take<double>((size_t)(s.m - s.k + 1) * s.kp);
    b.pivn2 = a.take<double>(s.k);
    b.Rt = a.take<double>((size_t)s.n * s.kp);
    b.Qt = a.take<double>((size_t)s.n * s.kp);
    b.Rtt = a.take<double>((size_t)s.lp * s.lp);
    b.Qres = a.take<double>((size_t)(s.n - s.k + 1) * s.kp);
    b.Mb = a.take<double>((size_t)s.kp * s.kp);
    const int64_t nk = std::max<int64_t>(s.n - s.k, 1);
    b.ob2 = take_orth(a, s.n, s.kp, gemm_part_bytes(plan_gemm(s.k, nk, s.k, NCU_CAP, 0), 8));
  }
  if (out) *out = b;
  return a.off;
}

struct Ctx {
  hipStream_t st;
  int ncu;
  int32_t* info;
  uint64_t seed;
  uint32_t orth_calls;
  rsvd_handle_s* h;
  F8Bufs f8 = F8Bufs();
};

// CUs kept free for the block Jacobi (at most 8 workgroups) while the
// pivoted QR runs beside it
constexpr int JACOBI_CU_RESERVE = 8;

#define RSVD_TRY(x)                         \
  do {                                      \
    hipError_t e_ = (x);                    \
    if (e_ != hipSuccess) return e_;        \
  } while (0)

// First CholeskyQR pass of orth (l <= ORTH_BLOCK): G = Y^T Y = R1^T R1,
// Qa = Y R1^{-1} (FP64, ld rup(l, 16)), dependent columns of Qa replaced.
hipError_t orth_p1(Ctx& c, const OrthBufs& ob, bool y_f32, const void* Y, int64_t ldy,
                   int64_t rows, int l) {
  const int lp = (int)rup(l, 16);
  const int gG = std::min(c.ncu, NCU_CAP);
  RSVD_TRY(launch_gram(y_f32, Y, ldy, rows, l, lp, ob.G, lp, ob.gpart, gG, c.st));
  RSVD_TRY(launch_chol(ob.G, lp, l, lp, ETA_ORTH, ob.R1, lp, ob.Rd1, ob.dep, c.info, c.st));
  RSVD_TRY(launch_trsm(y_f32, false, Y, ldy, rows, l, lp, ob.R1, lp, ob.Rd1, ob.Qa, lp, c.st));
  return launch_replace(false, ob.Qa, lp, rows, l, ob.dep, c.seed, c.orth_calls++, c.st);
}

// Second pass: Qa = Q R2.  An FP32 basis is the first pass rounded to FP32
// when that pass is already orthonormal far below the FP32 rounding (the
// near-identity parts decide).
hipError_t orth_p2(Ctx& c, const OrthBufs& ob, int64_t rows, int l, void* Q, bool q_f32,
                   int64_t ldq) {
  const int lp = (int)rup(l, 16);
  const int gG = std::min(c.ncu, NCU_CAP);
  RSVD_TRY(launch_gram(false, ob.Qa, lp, rows, l, lp, ob.G, lp, ob.gpart, gG, c.st));
  RSVD_TRY(launch_chol(ob.G, lp, l, lp, ETA_ORTH, ob.R2, lp, ob.Rd2, ob.dep2, c.info, c.st,
                       ob.nip));
  return launch_trsm(false, q_f32, ob.Qa, lp, rows, l, lp, ob.R2, lp, ob.Rd2, Q, ldq, c.st,
                     q_f32 ? ob.nip : nullptr);
}

// Q = orth(Y) by CholeskyQR2 (rows x l, l <= ORTH_BLOCK); optionally
// R = R2 R1 (rup(l, 16) square, ldr).
hipError_t orth_small(Ctx& c, const OrthBufs& ob, bool y_f32, const void* Y, int64_t ldy,
                      int64_t rows, int l, void* Q, bool q_f32, int64_t ldq, double* Rout,
                      int64_t ldr) {
  const int lp = (int)rup(l, 16);
  RSVD_TRY(orth_p1(c, ob, y_f32, Y, ldy, rows, l));
  RSVD_TRY(orth_p2(c, ob, rows, l, Q, q_f32, ldq));
  if (Rout) RSVD_TRY(launch_trmm_upper(ob.R2, lp, ob.R1, lp, ob.dep, Rout, ldr, lp, c.st));
  return hipSuccess;
}

// Q = orth(Y) for l > ORTH_BLOCK: block Gram-Schmidt over column blocks Y_j of
// at most ORTH_BLOCK columns, each block projected against the columns
// before it (Qb) and factored by one CholeskyQR pass, twice:
//   T = Y_j - Qb (Qb^T Y_j) = Qa R1;  Qa - Qb (Qb^T Qa) = Q_j R2
// so Y_j = Qb (W1 + W2 R1) + Q_j (R2 R1), with W1 = Qb^T Y_j, W2 = Qb^T Qa
// (a replaced dependent column of Qa is projected in the second pass too).
// The result is the QR factorization of Y with a positive diagonal (the
// same Q and R as one CholeskyQR2 of all l columns, to rounding).
hipError_t orth_blocks(Ctx& c, const OrthBufs& ob, bool y_f32, const void* Y, int64_t ldy,
                       int64_t rows, int l, void* Q, bool q_f32, int64_t ldq, double* Rout,
                       int64_t ldr) {
  const int nblk = (int)cdiv(l, ORTH_BLOCK);
  const int bs = (int)rup(cdiv(l, nblk), 16);
  const int lp = (int)rup(l, 16);
  const size_t ysz = y_f32 ? 4 : 8, qsz = q_f32 ? 4 : 8;
  const int ncu = std::min(c.ncu, NCU_CAP);
  const int64_t ldw = ORTH_BLOCK;
  const GemmTypes ty = q_f32 ? (y_f32 ? GEMM_FFDD : GEMM_FDDD) : (y_f32 ? GEMM_DFDD : GEMM_DDDD);
  const GemmTypes tq = q_f32 ? GEMM_FDDD : GEMM_DDDD;
  if (Rout) RSVD_TRY(launch_zero(Rout, ldr, lp, lp, c.st));
  for (int j = 0; j < nblk; ++j) {
    const int c0 = j * bs;
    const int bj = std::min(bs, l - c0);
    const int lpj = (int)rup(bj, 16);
    const void* Yj = static_cast<const char*>(Y) + c0 * ysz;
    void* Qj = static_cast<char*>(Q) + c0 * qsz;
    double* Rjj = Rout ? Rout + (int64_t)c0 * ldr + c0 : nullptr;
    if (j == 0) {
      RSVD_TRY(orth_small(c, ob, y_f32, Yj, ldy, rows, bj, Qj, q_f32, ldq, Rjj, ldr));
      continue;
    }
    const GemmPlan pw = plan_gemm(c0, rows, bj, ncu, 0);     // Qb^T X  (c0 x bj)
    const GemmPlan pp = plan_gemm(rows, c0, bj, ncu, 0);     // Qb W    (rows x bj)
    double* W1 = Rout ? Rout + c0 : ob.W;                    // R(0:c0, block) holds W1
    const int64_t ldw1 = Rout ? ldr : ldw;
    // pass 1
    RSVD_TRY(launch_gemm(ty, true, Q, ldq, Yj, ldy, W1, ldw1, c0, rows, bj, pw, ob.part,
                         ob.part_bytes, c.st));
    RSVD_TRY(launch_gemm(tq, false, Q, ldq, W1, ldw1, ob.T, ldw, rows, c0, bj, pp, ob.part,
                         ob.part_bytes, c.st));
    RSVD_TRY(launch_rsub(y_f32, Yj, ldy, ob.T, ldw, rows, bj, c.st));
    RSVD_TRY(orth_p1(c, ob, false, ob.T, ldw, rows, bj));
    // pass 2
    RSVD_TRY(launch_gemm(tq, true, Q, ldq, ob.Qa, lpj, ob.W2, ldw, c0, rows, bj, pw, ob.part,
                         ob.part_bytes, c.st));
    RSVD_TRY(launch_gemm(tq, false, Q, ldq, ob.W2, ldw, ob.T, ldw, rows, c0, bj, pp, ob.part,
                         ob.part_bytes, c.st));
    RSVD_TRY(launch_sub(ob.Qa, lpj, ob.T, ldw, rows, bj, c.st));
    RSVD_TRY(orth_p2(c, ob, rows, bj, Qj, q_f32, ldq));
    if (Rout) {
      // the unit rows of dependent columns are not part of Y_j = Qb W1 + Qa R1
      RSVD_TRY(launch_zero_dep_rows(ob.R1, lpj, bj, lpj, ob.dep, c.st));
      const GemmPlan pr = plan_gemm(c0, bj, bj, ncu, 0);
      RSVD_TRY(launch_gemm(GEMM_DDDD, false, ob.W2, ldw, ob.R1, lpj, ob.P2, ldw, c0, bj, bj, pr,
                           ob.part, ob.part_bytes, c.st));
      RSVD_TRY(launch_add(W1, ldw1, ob.P2, ldw, c0, bj, c.st));
      RSVD_TRY(launch_trmm_upper(ob.R2, lpj, ob.R1, lpj, ob.dep, Rjj, ldr, lpj, c.st));
    }
  }
  return hipSuccess;
}

// Q = orth(Y) (rows x l); optionally R (rup(l, 16) square, ldr) with Y = Q R.
hipError_t orth(Ctx& c, const OrthBufs& ob, bool y_f32, const void* Y, int64_t ldy,
                int64_t rows, int l, void* Q, bool q_f32, int64_t ldq, double* Rout,
                int64_t ldr) {
  if (l <= ORTH_BLOCK) return orth_small(c, ob, y_f32, Y, ldy, rows, l, Q, q_f32, ldq, Rout, ldr);
  return orth_blocks(c, ob, y_f32, Y, ldy, rows, l, Q, q_f32, ldq, Rout, ldr);
}

// One pass over A: Y = A X (trans false) or Y = A^T X (trans true).  atype 0 / 1:
// X and Y in A's type; atype 2 (BF16 A): X and Y in FP32, X rounded to BF16
// into xt (l x rup(K, 32), zero past K) first.  With split, X = X_hi + X_lo is applied as
// two BF16 passes whose FP32 results are added (X kept to ~16 bits).
hipError_t pass(Ctx& c, int atype, bool trans, int64_t m, int64_t n, int l, const void* A,
                int64_t lda, const void* X, int64_t ldx, void* Y, int64_t ldy, void* part,
                size_t part_bytes, uint16_t* xt = nullptr, bool split = false) {
  const int64_t M = trans ? n : m, K = trans ? m : n;
  if (atype == 3) {
    // FP8 A ~ A8 diag(s): Y = A8 (diag(s) X) or Z = diag(s) (A8^T X); X' is
    // quantized per column; with split a second term holds its residual
    const int64_t ldt = rup(K, 16);
    const int lp = (int)rup(l, 16);
    const GemmPlan pg = plan_gemm_f8(M, K, l, std::min(c.ncu, NCU_CAP));
    const float* xs = trans ? nullptr : c.f8.ascale;     // folded into X' for Y = A X
    const float* rs = trans ? c.f8.ascale : nullptr;     // epilogue row scale for A^T X
    uint8_t* x0 = c.f8.xt;
    uint8_t* x1 = c.f8.xt + (size_t)lp * ldt;
    RSVD_TRY(launch_quant_x_f8(true, X, ldx, K, l, xs, nullptr, 0, nullptr, x0, ldt, c.f8.t,
                               c.f8.tmax, c.st));
    RSVD_TRY(launch_gemm_f8(trans, static_cast<const uint8_t*>(A), lda, x0, ldt, c.f8.t, rs,
                            static_cast<float*>(Y), ldy, M, K, l, pg, part, part_bytes, false,
                            c.st));
    if (!split) return hipSuccess;
    RSVD_TRY(launch_quant_x_f8(true, X, ldx, K, l, xs, x0, ldt, c.f8.t, x1, ldt, c.f8.t + lp,
                               c.f8.tmax, c.st));
    return launch_gemm_f8(trans, static_cast<const uint8_t*>(A), lda, x1, ldt, c.f8.t + lp, rs,
                          static_cast<float*>(Y), ldy, M, K, l, pg, part, part_bytes, true, c.st);
  }
  if (atype < 2 && narrow_applies(atype == 1, lda, A, l) &&
      narrow_work_bytes(atype == 1, trans, M, K, l, std::min(c.ncu, NCU_CAP)) <= part_bytes)
    return launch_narrow(atype == 1, trans, A, lda, X, ldx, Y, ldy, M, K, l,
                         std::min(c.ncu, NCU_CAP), part, part_bytes, c.st);
  if (atype != 2) {
    const GemmPlan pg = plan_gemm(M, K, l, std::min(c.ncu, NCU_CAP), 0);
    return launch_gemm(atype == 1 ? GEMM_FFFF : GEMM_DDDD, trans, A, lda, X, ldx, Y, ldy, M, K, l,
                       pg, part, part_bytes, c.st);
  }
  const int64_t ldt = rup(K, 32);   // (the BF16 passes read whole 32-deep k-steps of Xt)
  const GemmPlan pg = plan_gemm_bf16(M, K, l, std::min(c.ncu, NCU_CAP));
  RSVD_TRY(launch_convert_bf16(true, X, ldx, K, l, xt, ldt, c.st));
  RSVD_TRY(launch_gemm_bf16(trans, static_cast<const uint16_t*>(A), lda, xt, ldt,
                            static_cast<float*>(Y), ldy, M, K, l, pg, part, part_bytes, c.st));
  if (!split) return hipSuccess;
  // X_lo = X - bf16(X), then Y += A X_lo
  RSVD_TRY(launch_bf16_residual(static_cast<const float*>(X), ldx, K, l, xt, ldt, c.st));
  return launch_gemm_bf16_acc(trans, static_cast<const uint16_t*>(A), lda, xt, ldt,
                              static_cast<float*>(Y), ldy, M, K, l, pg, part, part_bytes, c.st);
}

struct Outs {
  void* U; int64_t ldu; double* S; void* V; int64_t ldv;
  int64_t* J; double* T; int64_t ldt;
  int64_t* Jc; int64_t* Jr; double* Ucur; int64_t lduc;
  void* Qb; int64_t ldqb;          // optional copy of the range finder's basis Q
};

hipError_t run_decompose(Ctx& c, const Shape& s, const Bufs& b, const void* A, int64_t lda,
                         const Outs& o) {
  const bool f32 = s.f32;
  const int l = s.l, lp = s.lp, k = s.k;
  const int64_t m = s.m, n = s.n;
  RSVD_TRY(launch_set_word(c.info, 0, c.st));
  RSVD_TRY(launch_set_word(c.info + 1, 0, c.st));
  // range finder
  const int at = s.atype;
  RSVD_TRY(launch_sketch(f32, c.seed, 0, 0, n, l, b.Om, lp, c.st));
  RSVD_TRY(pass(c, at, false, m, n, l, A, lda, b.Om, lp, b.Y, lp, b.ob.part, b.ob.part_bytes,
                b.Xt));
  for (int j = 0; j < s.q; ++j) {
    RSVD_TRY(orth(c, b.ob, f32, b.Y, lp, m, l, b.Q, f32, lp, nullptr, 0));
    RSVD_TRY(pass(c, at, true, m, n, l, A, lda, b.Q, lp, b.Z, lp, b.ob.part, b.ob.part_bytes,
                  b.Xt));
    RSVD_TRY(orth(c, b.ob, f32, b.Z, lp, n, l, b.Zq, f32, lp, nullptr, 0));
    RSVD_TRY(pass(c, at, false, m, n, l, A, lda, b.Zq, lp, b.Y, lp, b.ob.part, b.ob.part_bytes,
                  b.Xt));
  }
  RSVD_TRY(orth(c, b.ob, f32, b.Y, lp, m, l, b.Q, f32, lp, nullptr, 0));
  if (o.Qb)
    RSVD_TRY(hipMemcpy2DAsync(o.Qb, o.ldqb * s.dsz, b.Q, lp * s.dsz, l * s.dsz, m,
                              hipMemcpyDeviceToDevice, c.st));
  // B^T = A^T Q; with a BF16 A the basis enters this last product in two
  // BF16 parts, so B keeps ~16 bits of Q
  RSVD_TRY(pass(c, at, true, m, n, l, A, lda, b.Q, lp, b.Z, lp, b.ob.part, b.ob.part_bytes, b.Xt,
                true));
  const int ncu = std::min(c.ncu, NCU_CAP);
  // With both the SVD and the ID / CUR requested, the SVD's Jacobi (a few
  // workgroups) and its two products run on the handle's second stream while
  // the pivoted QRs run here on all but JACOBI_CU_RESERVE CUs; the cross-
  // workgroup waits of the two kernels then never compete for CUs.
  const bool fork = o.U && (o.J || o.Jr) && ncu >= 4 * JACOBI_CU_RESERVE;
  if (o.U) {
    // [Qh, Rh] = qr(B^T); Rh = Uh S Vh^T; U = Q Vh_k; V = Qh Uh_k
    RSVD_TRY(orth(c, b.ob, f32, b.Z, lp, n, l, b.Qh, false, lp, b.Rh, lp));
    hipStream_t s1 = c.st;
    if (fork) {
      RSVD_TRY(hipEventRecord(c.h->ev_fork, c.st));
      RSVD_TRY(hipStreamWaitEvent(c.h->aux, c.h->ev_fork, 0));
      s1 = c.h->aux;
    }
    RSVD_TRY(launch_jacobi(b.Rh, lp, l, k, b.Wj, o.S, b.Uh, s.kp, b.Vh, s.kp,
                           c.h->jacobi_max_sweeps, c.info, nullptr, c.h->giveup_test, s1));
    const GemmPlan pu = plan_gemm(m, l, k, ncu, 0);
    RSVD_TRY(launch_gemm(f32 ? GEMM_FDDF : GEMM_DDDD, false, b.Q, lp, b.Vh, s.kp, o.U, o.ldu, m, l,
                         k, pu, b.ob.part, b.ob.part_bytes, s1));
    const GemmPlan pv = plan_gemm(n, l, k, ncu, 0);
    RSVD_TRY(launch_gemm(f32 ? GEMM_DDDF : GEMM_DDDD, false, b.Qh, lp, b.Uh, s.kp, o.V, o.ldv, n,
                         l, k, pv, b.ob.part, b.ob.part_bytes, s1));
    if (fork) RSVD_TRY(hipEventRecord(c.h->ev_join, s1));
  }
  if (o.J || o.Jr) {
    const int ncq = fork ? ncu - JACOBI_CU_RESERVE : ncu;
    int64_t* J = o.J ? o.J : b.J;
    double* T = o.T ? o.T : b.T;
    const int64_t ldt = o.T ? o.ldt : (n - k);
    const CpqrPlan cp = plan_cpqr(l, n, k, ncq);
    RSVD_TRY(launch_cpqr(f32, b.Z, lp, l, n, k, cp, b.cq_work, J, b.S11t, b.S12t, s.kp, b.pivn,
                         c.info, c.h->giveup_test, c.st));
    RSVD_TRY(launch_backsub(b.S11t, 1, s.kp, b.S12t, 1, s.kp, k, n - k, T, ldt, 1, c.st));
    if (o.Jr) {
      // row selection on C^T = A(:, J_k)^T
      RSVD_TRY(launch_gather_cols(s.atype, A, lda, m, n, J, k, b.Crow, s.kp, c.st));
      const CpqrPlan cp2 = plan_cpqr(k, m, k, ncq);
      RSVD_TRY(launch_cpqr(false, b.Crow, s.kp, k, m, k, cp2, b.cq2_work, b.J2, b.S11t2, b.S12t2,
                           s.kp, b.pivn2, c.info, c.h->giveup_test, c.st));
      // R^T = A(Jr, :)^T = Qt Rt
      RSVD_TRY(launch_gather_rows_t(s.atype, A, lda, m, n, b.J2, k, b.Rt, s.kp, c.st));
      RSVD_TRY(orth(c, b.ob2, false, b.Rt, s.kp, n, k, b.Qt, false, s.kp, b.Rtt, s.kp));
      // M = T Qt(J_res, :) + Qt(J_k, :)
      RSVD_TRY(launch_pick_rows(b.Qt, s.kp, n, J + k, n - k, k, b.Qres, s.kp, false, c.st));
      if (n > k) {
        const GemmPlan pm = plan_gemm(k, n - k, k, ncu, 0);
        RSVD_TRY(launch_gemm(GEMM_DDDD, false, T, ldt, b.Qres, s.kp, b.Mb, s.kp, k, n - k, k, pm,
                             b.ob2.part, b.ob2.part_bytes, c.st));
        RSVD_TRY(launch_pick_rows(b.Qt, s.kp, n, J, k, k, b.Mb, s.kp, true, c.st));
      } else {
        RSVD_TRY(launch_pick_rows(b.Qt, s.kp, n, J, k, k, b.Mb, s.kp, false, c.st));
      }
      // U Rt^T = M  <=>  Rt U^T = M^T
      RSVD_TRY(launch_backsub(b.Rtt, s.kp, 1, b.Mb, 1, s.kp, k, k, o.Ucur, 1, o.lduc, c.st));
      RSVD_TRY(hipMemcpyAsync(o.Jr, b.J2, sizeof(int64_t) * k, hipMemcpyDeviceToDevice, c.st));
      if (o.Jc)
        RSVD_TRY(hipMemcpyAsync(o.Jc, J, sizeof(int64_t) * k, hipMemcpyDeviceToDevice, c.st));
    }
  }
  if (fork) RSVD_TRY(hipStreamWaitEvent(c.st, c.h->ev_join, 0));
  return hipSuccess;
}

// ---- left-sketch ID (Alg. 6 with the power scheme of eq. (Ypower)) -------
constexpr uint32_t STREAM_LEFT = 6;   // Philox stream of Omega~^T

struct LeftBufs {
  void *Ot, *Yt, *Ym, *Qm, *Qn;
  uint16_t* Xt;
  OrthBufs ob;
  void* cq_work;
  double *S11t, *S12t, *pivn;
};

size_t layout_left(const Shape& s, void* base, LeftBufs* out) {
  Arena a(base);
  LeftBufs b;
  const int64_t rmax = std::max(s.m, s.n);
  b.Ot = a.take<char>((size_t)s.m * s.lp * s.dsz);
  b.Yt = a.take<char>((size_t)s.n * s.lp * s.dsz);
  b.Ym = a.take<char>((size_t)s.m * s.lp * s.dsz);
  b.Qm = a.take<char>((size_t)s.m * s.lp * s.dsz);
  b.Qn = a.take<char>((size_t)s.n * s.lp * s.dsz);
  b.Xt = s.bf16 ? a.take<uint16_t>((size_t)s.lp * rup(rmax, 32)) : nullptr;
  b.ob = take_orth(a, rmax, s.lp, max_part(s));
  b.cq_work = a.take<char>(cpqr_work_bytes(plan_cpqr(s.l, s.n, s.k, NCU_CAP)));
  b.S11t = a.take<double>((size_t)s.k * s.kp);
  b.S12t = a.take<double>((size_t)(s.n - s.k + 1) * s.kp);
  b.pivn = a.take<double>(s.k);
  if (out) *out = b;
  return a.off;
}

// Y^T = A^T Omega~^T;  q times { Y^T = A orth(Y^T);  Y^T = A^T orth(Y^T) };
// k steps of column-pivoted QR of Y (its columns are the rows of Y^T);
// T = S11^{-1} S12.
hipError_t run_id_left(Ctx& c, const Shape& s, const LeftBufs& b, const void* A, int64_t lda,
                       int64_t* J, double* T, int64_t ldt) {
  const bool f32 = s.f32;
  const int l = s.l, lp = s.lp, k = s.k, at = s.atype;
  const int64_t m = s.m, n = s.n;
  RSVD_TRY(launch_set_word(c.info, 0, c.st));
  RSVD_TRY(launch_set_word(c.info + 1, 0, c.st));
  RSVD_TRY(launch_sketch(f32, c.seed, STREAM_LEFT, 0, m, l, b.Ot, lp, c.st));
  RSVD_TRY(pass(c, at, true, m, n, l, A, lda, b.Ot, lp, b.Yt, lp, b.ob.part, b.ob.part_bytes,
                b.Xt));
  for (int j = 0; j < s.q; ++j) {
    RSVD_TRY(orth(c, b.ob, f32, b.Yt, lp, n, l, b.Qn, f32, lp, nullptr, 0));
    RSVD_TRY(pass(c, at, false, m, n, l, A, lda, b.Qn, lp, b.Ym, lp, b.ob.part,
                  b.ob.part_bytes, b.Xt));
    RSVD_TRY(orth(c, b.ob, f32, b.Ym, lp, m, l, b.Qm, f32, lp, nullptr, 0));
    // with a BF16 A the last basis enters in two BF16 parts, as for B^T
    RSVD_TRY(pass(c, at, true, m, n, l, A, lda, b.Qm, lp, b.Yt, lp, b.ob.part, b.ob.part_bytes,
                  b.Xt, j == s.q - 1));
  }
  const CpqrPlan cp = plan_cpqr(l, n, k, std::min(c.ncu, NCU_CAP));
  RSVD_TRY(launch_cpqr(f32, b.Yt, lp, l, n, k, cp, b.cq_work, J, b.S11t, b.S12t, s.kp, b.pivn,
                       c.info, c.h->giveup_test, c.st));
  return launch_backsub(b.S11t, 1, s.kp, b.S12t, 1, s.kp, k, n - k, T, ldt, 1, c.st);
}

// ---- blocked adaptive QB (Alg. 7) -----------------------------------------
constexpr uint32_t STREAM_QB = 5;     // Philox stream of Omega_i (batch = block index)

struct QbBufs {
  double *Om, *Ya, *Za, *Zb, *Yb, *W, *P, *Bt, *part, *norm2;
  OrthBufs ob;
};

size_t qb_gemm_part_bytes(int64_t m, int64_t n, int b, int M) {
  const int ncu = NCU_CAP;
  const int64_t ib = std::max<int64_t>((int64_t)b * (M - 1), 1);
  size_t r = 0;
  r = std::max(r, gemm_part_bytes(plan_gemm(m, n, b, ncu, 0), 8));
  r = std::max(r, gemm_part_bytes(plan_gemm(n, m, b, ncu, 0), 8));
  r = std::max(r, gemm_part_bytes(plan_gemm(ib, m, b, ncu, 0), 8));
  r = std::max(r, gemm_part_bytes(plan_gemm(m, ib, b, ncu, 0), 8));
  return r;
}

size_t layout_qb(int64_t m, int64_t n, int b, int M, void* base, QbBufs* out) {
  Arena a(base);
  QbBufs q;
  const int bp = (int)rup(b, 16);
  q.Om = a.take<double>((size_t)n * bp);
  q.Ya = a.take<double>((size_t)m * bp);
  q.Za = a.take<double>((size_t)n * bp);
  q.Zb = a.take<double>((size_t)n * bp);
  q.Yb = a.take<double>((size_t)m * bp);
  q.W = a.take<double>((size_t)b * M * bp);
  q.P = a.take<double>((size_t)m * bp);
  q.Bt = a.take<double>((size_t)n * bp);
  q.part = a.take<double>((size_t)qb_update_tiles(m, n));
  q.norm2 = a.take<double>(1);
  q.ob = take_orth(a, std::max(m, n), bp, qb_gemm_part_bytes(m, n, b, M));
  if (out) *out = q;
  return a.off;
}

// Block i: Omega_i; Q_i = orth(A Omega_i); q times { Q_i = orth(A^T Q_i);
// Q_i = orth(A Q_i) }; Q_i = orth(Q_i - Qbar (Qbar^T Q_i)); B_i = Q_i^T A;
// A -= Q_i B_i; stop when ||A||_F < tol.  The host reads ||A||_F^2 after
// every block (one stream synchronization per block).
hipError_t run_qb(Ctx& c, const QbBufs& w, int64_t m, int64_t n, int b, int M, int q, double tol,
                  double* A, int64_t lda, double* Q, int64_t ldq, double* B, int64_t ldb,
                  int32_t* nblocks, double* resid) {
  const int bp = (int)rup(b, 16);
  const int ncu = std::min(c.ncu, NCU_CAP);
  const OrthBufs& ob = w.ob;
  RSVD_TRY(launch_set_word(c.info, 0, c.st));
  RSVD_TRY(launch_set_word(c.info + 1, 0, c.st));
  int nb = 0;
  double r2 = 0.0;
  for (int i = 0; i < M; ++i) {
    double* Qi = Q + (int64_t)i * b;                 // columns i*b .. of Q
    RSVD_TRY(launch_sketch(false, c.seed, STREAM_QB, (uint32_t)i, n, b, w.Om, bp, c.st));
    RSVD_TRY(pass(c, 0, false, m, n, b, A, lda, w.Om, bp, w.Ya, bp, ob.part, ob.part_bytes));
    RSVD_TRY(orth(c, ob, false, w.Ya, bp, m, b, w.Yb, false, bp, nullptr, 0));
    for (int j = 0; j < q; ++j) {
      RSVD_TRY(pass(c, 0, true, m, n, b, A, lda, w.Yb, bp, w.Za, bp, ob.part, ob.part_bytes));
      RSVD_TRY(orth(c, ob, false, w.Za, bp, n, b, w.Zb, false, bp, nullptr, 0));
      RSVD_TRY(pass(c, 0, false, m, n, b, A, lda, w.Zb, bp, w.Ya, bp, ob.part, ob.part_bytes));
      RSVD_TRY(orth(c, ob, false, w.Ya, bp, m, b, w.Yb, false, bp, nullptr, 0));
    }
    if (i > 0) {
      // Yb -= Qbar (Qbar^T Yb), Qbar = the first i*b columns of Q
      const int64_t ib = (int64_t)i * b;
      const GemmPlan pw = plan_gemm(ib, m, b, ncu, 0);
      RSVD_TRY(launch_gemm(GEMM_DDDD, true, Q, ldq, w.Yb, bp, w.W, bp, ib, m, b, pw, ob.part,
                           ob.part_bytes, c.st));
      const GemmPlan pp = plan_gemm(m, ib, b, ncu, 0);
      RSVD_TRY(launch_gemm(GEMM_DDDD, false, Q, ldq, w.W, bp, w.P, bp, m, ib, b, pp, ob.part,
                           ob.part_bytes, c.st));
      RSVD_TRY(launch_sub(w.Yb, bp, w.P, bp, m, b, c.st));
    }
    RSVD_TRY(orth(c, ob, false, w.Yb, bp, m, b, Qi, false, ldq, nullptr, 0));
    // B_i^T = A^T Q_i (n x b), B_i = its transpose, A -= Q_i B_i
    RSVD_TRY(pass(c, 0, true, m, n, b, A, lda, Qi, ldq, w.Bt, bp, ob.part, ob.part_bytes));
    RSVD_TRY(launch_transpose(w.Bt, bp, n, b, B + (int64_t)i * b * ldb, ldb, c.st));
    RSVD_TRY(launch_qb_update(A, lda, m, n, Qi, ldq, w.Bt, bp, b, w.part, w.norm2, c.st));
    RSVD_TRY(hipMemcpyAsync(&r2, w.norm2, sizeof(double), hipMemcpyDeviceToHost, c.st));
    RSVD_TRY(hipStreamSynchronize(c.st));
    nb = i + 1;
    if (std::sqrt(r2) < tol) break;
  }
  if (nblocks) *nblocks = nb;
  if (resid) *resid = std::sqrt(r2);
  return hipSuccess;
}

// ---- reverse-mode derivative of the randomized SVD (sketch fixed) --------
// The forward map is recomputed with its bases and triangular factors kept
// (the caller stores only A): Y_0 = A Omega; for j < q: Qy_j Ry_j = Y_j,
// Z_j = A^T Qy_j, Qz_j Rz_j = Z_j, Y_{j+1} = A Qz_j; Q Rq = Y_q; B^T = A^T Q;
// Qh Rh = B^T; Rh = Uh diag(s) Vh^T (all l values).  The adjoint then walks
// these steps backwards; dA collects one rank-l term per product with A.
constexpr int GRAD_MAX_Q = (LR_MAX - 2) / 2;

struct GradBufs {
  double *Om, *Yt, *Zt, *Q, *Rq, *Qh, *Rh, *Wj, *sv, *Uh, *Vh;
  double *Qy[GRAD_MAX_Q], *Ry[GRAD_MAX_Q], *Qz[GRAD_MAX_Q], *Rz[GRAD_MAX_Q];
  double *dQ, *dQh, *dBt, *dY[GRAD_MAX_Q + 1], *dZ[GRAD_MAX_Q], *Cm, *G;
  double *dUh, *dVh, *Pu, *Pv, *inner, *T1, *T2, *dRh, *Pm, *Rm, *Mc;
  double *rpart;
  OrthBufs ob;
};

size_t grad_part_bytes(const Shape& s) {
  const int ncu = NCU_CAP;
  size_t r = max_part(s);
  auto upd = [&](int64_t M, int64_t K, int64_t L) {
    if (M > 0 && K > 0 && L > 0) r = std::max(r, gemm_part_bytes(plan_gemm(M, K, L, ncu, 0), 8));
  };
  for (int64_t rows : {s.m, s.n}) {
    upd(rows, s.k, s.l);      // dQ = dU Vh_k^T, dQh = dV Uh_k^T
    upd(s.l, rows, s.k);      // Q^T dU, Qh^T dV
    upd(s.l, rows, s.l);      // dQ^T Q
    upd(rows, s.l, s.l);      // Q Mc
    upd(rows, s.l, s.k);      // U = Q Vh_k, V = Qh Uh_k
  }
  upd(s.l, s.l, s.l);
  return r;
}

size_t layout_grad(const Shape& s, void* base, GradBufs* out) {
  Arena a(base);
  GradBufs g;
  std::memset(&g, 0, sizeof(g));
  const int64_t m = s.m, n = s.n, lp = s.lp, rmax = std::max(m, n);
  const size_t sq = (size_t)lp * lp;
  g.Om = a.take<double>((size_t)n * lp);
  g.Yt = a.take<double>((size_t)m * lp);
  g.Zt = a.take<double>((size_t)n * lp);
  for (int j = 0; j < s.q; ++j) {
    g.Qy[j] = a.take<double>((size_t)m * lp);
    g.Qz[j] = a.take<double>((size_t)n * lp);
    g.Ry[j] = a.take<double>(sq);
    g.Rz[j] = a.take<double>(sq);
    g.dZ[j] = a.take<double>((size_t)n * lp);
  }
  for (int j = 0; j <= s.q; ++j) g.dY[j] = a.take<double>((size_t)m * lp);
  g.Q = a.take<double>((size_t)m * lp);
  g.Rq = a.take<double>(sq);
  g.Qh = a.take<double>((size_t)n * lp);
  g.Rh = a.take<double>(sq);
  g.Wj = a.take<double>(jacobi_work_bytes(s.l) / sizeof(double) + 1);
  g.sv = a.take<double>(lp);
  g.Uh = a.take<double>(sq);
  g.Vh = a.take<double>(sq);
  g.dQ = a.take<double>((size_t)m * lp);
  g.dQh = a.take<double>((size_t)n * lp);
  g.dBt = a.take<double>((size_t)n * lp);
  g.Cm = a.take<double>((size_t)rmax * lp);
  g.G = a.take<double>((size_t)rmax * lp);
  for (double** t : {&g.dUh, &g.dVh, &g.Pu, &g.Pv, &g.inner, &g.T1, &g.T2, &g.dRh, &g.Pm, &g.Rm,
                     &g.Mc})
    *t = a.take<double>(sq);
  g.rpart = a.take<double>((size_t)qb_update_tiles(m, n) + 1);
  g.ob = take_orth(a, rmax, s.lp, grad_part_bytes(s));
  if (out) *out = g;
  return a.off;
}

// C (M x L) = op(A) X for the small FP64 products of the adjoint
hipError_t small_gemm(Ctx& c, const OrthBufs& ob, bool trans, const double* A, int64_t lda,
                      const double* X, int64_t ldx, double* C, int64_t ldc, int64_t M, int64_t K,
                      int64_t L) {
  const GemmPlan p = plan_gemm(M, K, L, std::min(c.ncu, NCU_CAP), 0);
  return launch_gemm(GEMM_DDDD, trans, A, lda, X, ldx, C, ldc, M, K, L, p, ob.part, ob.part_bytes,
                     c.st);
}

// Adjoint of the thin QR Y = Qm R (rows x l):
// dY = (dQm + Qm copyltu(R dR^T - dQm^T Qm)) R^{-T}   (dR may be null)
hipError_t qr_adjoint(Ctx& c, const GradBufs& g, int lp, const double* Qm, const double* R,
                      const double* dQm, const double* dR, int64_t rows, int l, double* dY) {
  const OrthBufs& ob = g.ob;
  RSVD_TRY(small_gemm(c, ob, true, dQm, lp, Qm, lp, g.Pm, lp, l, rows, l));   // dQm^T Qm
  if (dR) {
    RSVD_TRY(launch_transpose(dR, lp, l, l, g.T2, lp, c.st));
    RSVD_TRY(small_gemm(c, ob, false, R, lp, g.T2, lp, g.Rm, lp, l, l, l));      // R dR^T
  }
  RSVD_TRY(launch_copyltu(g.Pm, dR ? g.Rm : nullptr, lp, l, g.Mc, lp, c.st));
  RSVD_TRY(small_gemm(c, ob, false, Qm, lp, g.Mc, lp, g.Cm, lp, rows, l, l));
  RSVD_TRY(launch_add(g.Cm, lp, dQm, lp, rows, l, c.st));
  // dY R^T = Cm  <=>  R dY^T = Cm^T
  return launch_backsub(R, lp, 1, g.Cm, 1, lp, l, rows, dY, 1, lp, c.st);
}

struct GradIO {
  const double *dU, *dS, *dV, *dres;
  int64_t lddu, lddv;
  double* dA; int64_t ldda;
  double *U, *S, *V, *resid2;
  int64_t ldu, ldv;
};

hipError_t run_grad(Ctx& c, const Shape& s, const GradBufs& g, const double* A, int64_t lda,
                    const GradIO& io) {
  const int l = s.l, lp = s.lp, k = s.k, q = s.q;
  const int64_t m = s.m, n = s.n;
  const OrthBufs& ob = g.ob;
  RSVD_TRY(launch_set_word(c.info, 0, c.st));
  RSVD_TRY(launch_set_word(c.info + 1, 0, c.st));
  // forward, with the bases and factors kept
  RSVD_TRY(launch_sketch(false, c.seed, 0, 0, n, l, g.Om, lp, c.st));
  RSVD_TRY(pass(c, 0, false, m, n, l, A, lda, g.Om, lp, g.Yt, lp, ob.part, ob.part_bytes));
  for (int j = 0; j < q; ++j) {
    RSVD_TRY(orth(c, ob, false, g.Yt, lp, m, l, g.Qy[j], false, lp, g.Ry[j], lp));
    RSVD_TRY(pass(c, 0, true, m, n, l, A, lda, g.Qy[j], lp, g.Zt, lp, ob.part, ob.part_bytes));
    RSVD_TRY(orth(c, ob, false, g.Zt, lp, n, l, g.Qz[j], false, lp, g.Rz[j], lp));
    RSVD_TRY(pass(c, 0, false, m, n, l, A, lda, g.Qz[j], lp, g.Yt, lp, ob.part, ob.part_bytes));
  }
  RSVD_TRY(orth(c, ob, false, g.Yt, lp, m, l, g.Q, false, lp, g.Rq, lp));
  RSVD_TRY(pass(c, 0, true, m, n, l, A, lda, g.Q, lp, g.Zt, lp, ob.part, ob.part_bytes));
  RSVD_TRY(orth(c, ob, false, g.Zt, lp, n, l, g.Qh, false, lp, g.Rh, lp));
  RSVD_TRY(launch_jacobi(g.Rh, lp, l, l, g.Wj, g.sv, g.Uh, lp, g.Vh, lp, c.h->jacobi_max_sweeps,
                         c.info, nullptr, c.h->giveup_test, c.st));
  if (io.U) RSVD_TRY(small_gemm(c, ob, false, g.Q, lp, g.Vh, lp, io.U, io.ldu, m, l, k));
  if (io.V) RSVD_TRY(small_gemm(c, ob, false, g.Qh, lp, g.Uh, lp, io.V, io.ldv, n, l, k));
  if (io.S)
    RSVD_TRY(hipMemcpyAsync(io.S, g.sv, sizeof(double) * k, hipMemcpyDeviceToDevice, c.st));
  if (io.resid2)
    RSVD_TRY(launch_resid2(A, lda, m, n, g.Q, lp, g.Zt, lp, l, g.rpart, io.resid2, c.st));
  if (!io.dA) return hipSuccess;

  // U_k = Q Vh_k, V_k = Qh Uh_k
  RSVD_TRY(launch_zero(g.dVh, lp, l, l, c.st));
  RSVD_TRY(launch_zero(g.dUh, lp, l, l, c.st));
  if (io.dU) {
    RSVD_TRY(launch_transpose(g.Vh, lp, l, k, g.T1, lp, c.st));                  // Vh_k^T
    RSVD_TRY(small_gemm(c, ob, false, io.dU, io.lddu, g.T1, lp, g.dQ, lp, m, k, l));
    RSVD_TRY(small_gemm(c, ob, true, g.Q, lp, io.dU, io.lddu, g.dVh, lp, l, m, k));
  } else {
    RSVD_TRY(launch_zero(g.dQ, lp, m, l, c.st));
  }
  if (io.dV) {
    RSVD_TRY(launch_transpose(g.Uh, lp, l, k, g.T1, lp, c.st));                  // Uh_k^T
    RSVD_TRY(small_gemm(c, ob, false, io.dV, io.lddv, g.T1, lp, g.dQh, lp, n, k, l));
    RSVD_TRY(small_gemm(c, ob, true, g.Qh, lp, io.dV, io.lddv, g.dUh, lp, l, n, k));
  } else {
    RSVD_TRY(launch_zero(g.dQh, lp, n, l, c.st));
  }
  // Rh = Uh S Vh^T
  RSVD_TRY(small_gemm(c, ob, true, g.Uh, lp, g.dUh, lp, g.Pu, lp, l, l, l));
  RSVD_TRY(small_gemm(c, ob, true, g.Vh, lp, g.dVh, lp, g.Pv, lp, l, l, l));
  RSVD_TRY(launch_svd_inner(g.Pu, g.Pv, lp, g.sv, io.dS, k, io.dres, l, g.inner, lp, c.st));
  RSVD_TRY(small_gemm(c, ob, false, g.Uh, lp, g.inner, lp, g.T1, lp, l, l, l));
  RSVD_TRY(launch_transpose(g.Vh, lp, l, l, g.T2, lp, c.st));
  RSVD_TRY(small_gemm(c, ob, false, g.T1, lp, g.T2, lp, g.dRh, lp, l, l, l));
  // B^T = Qh Rh
  RSVD_TRY(qr_adjoint(c, g, lp, g.Qh, g.Rh, g.dQh, g.dRh, n, l, g.dBt));
  // B^T = A^T Q: dA += Q dBt^T, dQ += A dBt
  LowRank t;
  std::memset(&t, 0, sizeof(t));
  t.ldx = lp; t.ldw = lp; t.l = l;
  auto term = [&](const double* X, const double* W) {
    t.X[t.count] = X;
    t.W[t.count] = W;
    ++t.count;
  };
  term(g.Q, g.dBt);
  RSVD_TRY(pass(c, 0, false, m, n, l, A, lda, g.dBt, lp, g.G, lp, ob.part, ob.part_bytes));
  RSVD_TRY(launch_add(g.dQ, lp, g.G, lp, m, l, c.st));
  // Y_q = Q Rq
  RSVD_TRY(qr_adjoint(c, g, lp, g.Q, g.Rq, g.dQ, nullptr, m, l, g.dY[q]));
  for (int j = q - 1; j >= 0; --j) {
    // Y_{j+1} = A Qz_j
    term(g.dY[j + 1], g.Qz[j]);
    RSVD_TRY(pass(c, 0, true, m, n, l, A, lda, g.dY[j + 1], lp, g.G, lp, ob.part,
                  ob.part_bytes));
    // Z_j = Qz_j Rz_j
    RSVD_TRY(qr_adjoint(c, g, lp, g.Qz[j], g.Rz[j], g.G, nullptr, n, l, g.dZ[j]));
    // Z_j = A^T Qy_j
    term(g.Qy[j], g.dZ[j]);
    RSVD_TRY(pass(c, 0, false, m, n, l, A, lda, g.dZ[j], lp, g.G, lp, ob.part, ob.part_bytes));
    // Y_j = Qy_j Ry_j
    RSVD_TRY(qr_adjoint(c, g, lp, g.Qy[j], g.Ry[j], g.G, nullptr, m, l, g.dY[j]));
  }
  // Y_0 = A Omega
  term(g.dY[0], g.Om);
  return launch_lowrank_out(t, m, n, A, lda, io.dres, io.dA, io.ldda, c.st);
}

int check_common(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q) {
  if (!h) return -1;
  if (dtype == RSVD_F8E4M3) return RSVD_ERR_UNSUPPORTED;   // needs column scales: rsvd_svd_ex
  if (dtype != RSVD_F64 && dtype != RSVD_F32 && dtype != RSVD_BF16) return -2;
  if (m < 1) return -3;
  if (n < 1) return -4;
  if (k < 1 || k > std::min(m, n)) return -5;
  if (p < 0) return -6;
  if (q < 0) return -7;
  return 0;
}

int finish(hipError_t e) { return e == hipSuccess ? RSVD_OK : RSVD_ERR_HIP; }

// workspace of the orth step: R (lp x lp) and the buffers of one orth
size_t orth_step_layout(int64_t rows, int l, void* base, OrthBufs* ob, double** Rfull) {
  const int lp = (int)rup(l, 16);
  const size_t part = orth_block_part_bytes(rows, l);
  Arena a(base);
  double* R = a.take<double>((size_t)lp * lp);
  const OrthBufs o = take_orth(a, rows, lp, part);
  if (ob) *ob = o;
  if (Rfull) *Rfull = R;
  return a.off;
}


}  // namespace
}  // namespace rsvd

using namespace rsvd;

extern "C" {

int rsvd_create(rsvd_handle_t* handle, int device) {
  if (!handle) return -1;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
    return RSVD_ERR_NO_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return RSVD_ERR_HIP;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess)
    return RSVD_ERR_HIP;
  rsvd_handle_s* h = new rsvd_handle_s;
  h->device = device;
  h->ncu = prop.multiProcessorCount;
  h->aux = nullptr;
  h->ev_fork = h->ev_join = nullptr;
  h->jacobi_max_sweeps = JACOBI_MAX_SWEEPS;
  h->giveup_test = false;
  h->scratch = scratch_addr(device);   // with `device` current
  const bool ok = h->scratch != nullptr &&
                  hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) == hipSuccess &&
                  hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming) == hipSuccess;
  (void)hipSetDevice(prev);
  if (!ok) {
    rsvd_destroy(h);
    return RSVD_ERR_HIP;
  }
  *handle = h;
  return RSVD_OK;
}

int rsvd_destroy(rsvd_handle_t handle) {
  if (!handle) return RSVD_OK;
  if (handle->ev_join) (void)hipEventDestroy(handle->ev_join);
  if (handle->ev_fork) (void)hipEventDestroy(handle->ev_fork);
  if (handle->aux) (void)hipStreamDestroy(handle->aux);
  delete handle;
  return RSVD_OK;
}

int rsvd_set_option(rsvd_handle_t h, int option, int value) {
  if (!h) return -1;
  switch (option) {
    case RSVD_OPT_JACOBI_MAX_SWEEPS:
      if (value < 1 || value > 1000) return -3;
      h->jacobi_max_sweeps = value;
      return RSVD_OK;
    case RSVD_OPT_TEST_WAIT_GIVEUP:
      if (value != 0 && value != 1) return -3;
      h->giveup_test = value != 0;
      return RSVD_OK;
    default:
      return -2;
  }
}

const char* rsvd_status_string(int code) {
  if (code < 0) return "invalid argument";
  switch (code) {
    case RSVD_OK: return "ok";
    case RSVD_ERR_HIP: return "HIP error";
    case RSVD_ERR_WORKSPACE: return "workspace too small";
    case RSVD_ERR_UNSUPPORTED: return "unsupported by this build";
    case RSVD_ERR_NO_DEVICE: return "no such device";
    case RSVD_ERR_SCRATCH: return "needs more than the static scratch of the no-allocation call";
    default: return "unknown status";
  }
}

size_t rsvd_workspace_bytes(int ops, int dtype, int64_t m, int64_t n, int k, int p, int q) {
  if ((dtype != RSVD_F64 && dtype != RSVD_F32 && dtype != RSVD_BF16 && dtype != RSVD_F8E4M3) ||
      m < 1 || n < 1 || k < 1 || k > std::min(m, n) || p < 0 || q < 0 || (ops & 7) == 0)
    return 0;
  if (dtype == RSVD_F8E4M3 && ops != RSVD_OP_SVD) return 0;
  if (ops & RSVD_OP_CUR) ops |= RSVD_OP_ID;
  const Shape s = make_shape(ops, dtype, m, n, k, p, q);
  return layout(s, nullptr, nullptr);
}

int rsvd_decompose(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
                   uint64_t seed, const void* A, int64_t lda, void* U, int64_t ldu, double* S,
                   void* V, int64_t ldv, int64_t* J, double* T, int64_t ldt, int64_t* Jr,
                   double* Ucur, int64_t lduc, void* work, size_t work_bytes, int32_t* info,
                   void* stream) {
  int rc = check_common(h, dtype, m, n, k, p, q);
  if (rc) return rc;
  if (!A) return -9;
  if (lda < n) return -10;
  if (dtype == RSVD_BF16 && (lda % 8 || (reinterpret_cast<uintptr_t>(A) & 15))) return -10;
  const bool svd = U || S || V;
  if (svd) {
    if (!U) return -11;
    if (ldu < k) return -12;
    if (!S) return -13;
    if (!V) return -14;
    if (ldv < k) return -15;
  }
  const bool id = J || T;
  if (id) {
    if (!J) return -16;
    if (!T) return -17;
    if (ldt < n - k) return -18;
  }
  const bool cur = Jr || Ucur;
  if (cur) {
    if (!Jr) return -19;
    if (!Ucur) return -20;
    if (lduc < k) return -21;
  }
  if (!svd && !id && !cur) return -11;
  if (!work) return -22;
  if (!info) return -24;
  int ops = (svd ? RSVD_OP_SVD : 0) | (id ? RSVD_OP_ID : 0) | (cur ? RSVD_OP_CUR : 0);
  if (cur) ops |= RSVD_OP_ID;
  const Shape s = make_shape(ops, dtype, m, n, k, p, q);
  if (s.l > MAX_L_SVD) return RSVD_ERR_UNSUPPORTED;
  if ((id || cur) && !plan_cpqr(s.l, n, k, NCU_CAP).ok) return RSVD_ERR_UNSUPPORTED;
  if (cur && !plan_cpqr(k, m, k, NCU_CAP).ok) return RSVD_ERR_UNSUPPORTED;
  Bufs b;
  const size_t need = layout(s, work, &b);
  if (work_bytes < need) return RSVD_ERR_WORKSPACE;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  Ctx c{static_cast<hipStream_t>(stream), h->ncu, info, seed, 0, h};
  Outs o;
  std::memset(&o, 0, sizeof(o));
  o.U = U; o.ldu = ldu; o.S = S; o.V = V; o.ldv = ldv;
  o.J = J; o.T = T; o.ldt = ldt;
  o.Jr = Jr; o.Ucur = Ucur; o.lduc = lduc;
  return finish(run_decompose(c, s, b, A, lda, o));
}

int rsvd_svd(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
             uint64_t seed, const void* A, int64_t lda, void* U, int64_t ldu, double* S,
             void* V, int64_t ldv, void* work, size_t work_bytes, int32_t* info,
             void* stream) {
  int rc = check_common(h, dtype, m, n, k, p, q);
  if (rc) return rc;
  if (!A) return -9;
  if (lda < n) return -10;
  if (dtype == RSVD_BF16 && (lda % 8 || (reinterpret_cast<uintptr_t>(A) & 15))) return -10;
  if (!U) return -11;
  if (ldu < k) return -12;
  if (!S) return -13;
  if (!V) return -14;
  if (ldv < k) return -15;
  if (!work) return -16;
  if (!info) return -18;
  const Shape s = make_shape(RSVD_OP_SVD, dtype, m, n, k, p, q);
  if (s.l > MAX_L_SVD) return RSVD_ERR_UNSUPPORTED;
  Bufs b;
  const size_t need = layout(s, work, &b);
  if (work_bytes < need) return RSVD_ERR_WORKSPACE;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  Ctx c{static_cast<hipStream_t>(stream), h->ncu, info, seed, 0, h};
  Outs o;
  std::memset(&o, 0, sizeof(o));
  o.U = U; o.ldu = ldu; o.S = S; o.V = V; o.ldv = ldv;
  return finish(run_decompose(c, s, b, A, lda, o));
}

int rsvd_svd_ex(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
                uint64_t seed, const void* A, int64_t lda, const float* a_col_scale, void* U,
                int64_t ldu, double* S, void* V, int64_t ldv, void* Qb, int64_t ldqb, void* work,
                size_t work_bytes, int32_t* info, void* stream) {
  const bool f8 = dtype == RSVD_F8E4M3;
  int rc = check_common(h, f8 ? RSVD_BF16 : dtype, m, n, k, p, q);
  if (rc) return rc;
  if (!A) return -9;
  if (lda < n) return -10;
  if (dtype == RSVD_BF16 && (lda % 8 || (reinterpret_cast<uintptr_t>(A) & 15))) return -10;
  if (f8 && (lda % 16 || (reinterpret_cast<uintptr_t>(A) & 15))) return -10;
  if (f8 != (a_col_scale != nullptr)) return -11;
  if (!U) return -12;
  if (ldu < k) return -13;
  if (!S) return -14;
  if (!V) return -15;
  if (ldv < k) return -16;
  const Shape s = make_shape(RSVD_OP_SVD, dtype, m, n, k, p, q);
  if (Qb && ldqb < s.l) return -18;
  if (!work) return -19;
  if (!info) return -21;
  if (s.l > MAX_L_SVD) return RSVD_ERR_UNSUPPORTED;
  Bufs b;
  const size_t need = layout(s, work, &b);
  if (work_bytes < need) return RSVD_ERR_WORKSPACE;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  Ctx c{static_cast<hipStream_t>(stream), h->ncu, info, seed, 0, h};
  c.f8 = b.f8;
  c.f8.ascale = a_col_scale;
  Outs o;
  std::memset(&o, 0, sizeof(o));
  o.U = U; o.ldu = ldu; o.S = S; o.V = V; o.ldv = ldv;
  o.Qb = Qb; o.ldqb = ldqb;
  return finish(run_decompose(c, s, b, A, lda, o));
}

int rsvd_quantize(rsvd_handle_t h, int dtype, int64_t m, int64_t n, const double* A, int64_t lda,
                  void* Aq, int64_t ldq, float* col_scale, void* stream) {
  if (!h) return -1;
  if (dtype != RSVD_BF16 && dtype != RSVD_F8E4M3) return -2;
  if (m < 1) return -3;
  if (n < 1) return -4;
  if (!A) return -5;
  if (lda < n) return -6;
  if (!Aq) return -7;
  if (ldq < n) return -8;
  if (dtype == RSVD_F8E4M3 && !col_scale) return -9;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == RSVD_BF16)
    return finish(launch_quantize_bf16(A, lda, m, n, static_cast<uint16_t*>(Aq), ldq, st));
  return finish(launch_quantize_e4m3(A, lda, m, n, static_cast<uint8_t*>(Aq), ldq, col_scale, st));
}

size_t rsvd_svd_noalloc_bytes(int dtype, int64_t m, int64_t n, int k, int p, int q) {
  return rsvd_workspace_bytes(RSVD_OP_SVD, dtype, m, n, k, p, q);
}

int rsvd_svd_noalloc(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
                     uint64_t seed, const void* A, int64_t lda, void* U, int64_t ldu, double* S,
                     void* V, int64_t ldv, int32_t* info, void* stream) {
  int rc = check_common(h, dtype, m, n, k, p, q);
  if (rc) return rc;
  if (!A) return -9;
  if (lda < n) return -10;
  if (dtype == RSVD_BF16 && (lda % 8 || (reinterpret_cast<uintptr_t>(A) & 15))) return -10;
  if (!U) return -11;
  if (ldu < k) return -12;
  if (!S) return -13;
  if (!V) return -14;
  if (ldv < k) return -15;
  if (!info) return -16;
  const Shape s = make_shape(RSVD_OP_SVD, dtype, m, n, k, p, q);
  if (s.l > MAX_L_SVD) return RSVD_ERR_UNSUPPORTED;
  if (layout(s, nullptr, nullptr) > RSVD_NOALLOC_MAX_BYTES) return RSVD_ERR_SCRATCH;
  Bufs b;
  layout(s, h->scratch, &b);
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  Ctx c{static_cast<hipStream_t>(stream), h->ncu, info, seed, 0, h};
  Outs o;
  std::memset(&o, 0, sizeof(o));
  o.U = U; o.ldu = ldu; o.S = S; o.V = V; o.ldv = ldv;
  return finish(run_decompose(c, s, b, A, lda, o));
}

int rsvd_id(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
            uint64_t seed, const void* A, int64_t lda, int64_t* J, double* T, int64_t ldt,
            void* work, size_t work_bytes, int32_t* info, void* stream) {
  int rc = check_common(h, dtype, m, n, k, p, q);
  if (rc) return rc;
  if (!A) return -9;
  if (lda < n) return -10;
  if (dtype == RSVD_BF16 && (lda % 8 || (reinterpret_cast<uintptr_t>(A) & 15))) return -10;
  if (!J) return -11;
  if (!T) return -12;
  if (ldt < n - k || ldt < 1) return -13;
  if (!work) return -14;
  if (!info) return -16;
  const Shape s = make_shape(RSVD_OP_ID, dtype, m, n, k, p, q);
  if (s.l > MAX_L || !plan_cpqr(s.l, n, k, NCU_CAP).ok) return RSVD_ERR_UNSUPPORTED;
  Bufs b;
  const size_t need = layout(s, work, &b);
  if (work_bytes < need) return RSVD_ERR_WORKSPACE;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  Ctx c{static_cast<hipStream_t>(stream), h->ncu, info, seed, 0, h};
  Outs o;
  std::memset(&o, 0, sizeof(o));
  o.J = J; o.T = T; o.ldt = ldt;
  return finish(run_decompose(c, s, b, A, lda, o));
}

size_t rsvd_id_left_workspace_bytes(int dtype, int64_t m, int64_t n, int k, int p, int q) {
  if ((dtype != RSVD_F64 && dtype != RSVD_F32 && dtype != RSVD_BF16) || m < 1 || n < 1 || k < 1 ||
      k > std::min(m, n) || p < 0 || q < 0)
    return 0;
  return layout_left(make_shape(RSVD_OP_ID, dtype, m, n, k, p, q), nullptr, nullptr);
}

int rsvd_id_left(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
                 uint64_t seed, const void* A, int64_t lda, int64_t* J, double* T, int64_t ldt,
                 void* work, size_t work_bytes, int32_t* info, void* stream) {
  int rc = check_common(h, dtype, m, n, k, p, q);
  if (rc) return rc;
  if (!A) return -9;
  if (lda < n) return -10;
  if (dtype == RSVD_BF16 && (lda % 8 || (reinterpret_cast<uintptr_t>(A) & 15))) return -10;
  if (!J) return -11;
  if (!T) return -12;
  if (ldt < n - k || ldt < 1) return -13;
  if (!work) return -14;
  if (!info) return -16;
  const Shape s = make_shape(RSVD_OP_ID, dtype, m, n, k, p, q);
  if (s.l > MAX_L || !plan_cpqr(s.l, n, k, NCU_CAP).ok) return RSVD_ERR_UNSUPPORTED;
  LeftBufs b;
  const size_t need = layout_left(s, work, &b);
  if (work_bytes < need) return RSVD_ERR_WORKSPACE;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  Ctx c{static_cast<hipStream_t>(stream), h->ncu, info, seed, 0, h};
  return finish(run_id_left(c, s, b, A, lda, J, T, ldt));
}

size_t rsvd_qb_workspace_bytes(int dtype, int64_t m, int64_t n, int b, int M, int q) {
  if (dtype != RSVD_F64 || m < 1 || n < 1 || b < 1 || b > MAX_L || M < 1 || q < 0 ||
      (int64_t)b * M > std::min(m, n))
    return 0;
  return layout_qb(m, n, b, M, nullptr, nullptr);
}

int rsvd_qb(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int b, int M, int q, double tol,
            uint64_t seed, void* A, int64_t lda, double* Q, int64_t ldq, double* B, int64_t ldb,
            int32_t* nblocks, double* resid, void* work, size_t work_bytes, int32_t* info,
            void* stream) {
  if (!h) return -1;
  if (dtype != RSVD_F64) return dtype == RSVD_F32 || dtype == RSVD_BF16 ? RSVD_ERR_UNSUPPORTED : -2;
  if (m < 1) return -3;
  if (n < 1) return -4;
  if (b < 1 || b > MAX_L) return -5;
  if (M < 1 || (int64_t)b * M > std::min(m, n)) return -6;
  if (q < 0) return -7;
  if (!(tol >= 0.0)) return -8;
  if (!A) return -10;
  if (lda < n) return -11;
  if (!Q) return -12;
  if (ldq < (int64_t)b * M) return -13;
  if (!B) return -14;
  if (ldb < n) return -15;
  if (!nblocks) return -16;
  if (!work) return -18;
  if (!info) return -20;
  QbBufs w;
  const size_t need = layout_qb(m, n, b, M, work, &w);
  if (work_bytes < need) return RSVD_ERR_WORKSPACE;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  Ctx c{static_cast<hipStream_t>(stream), h->ncu, info, seed, 0, h};
  return finish(run_qb(c, w, m, n, b, M, q, tol, static_cast<double*>(A), lda, Q, ldq, B, ldb,
                       nblocks, resid));
}

size_t rsvd_svd_grad_workspace_bytes(int dtype, int64_t m, int64_t n, int k, int p, int q) {
  if (dtype != RSVD_F64 || m < 1 || n < 1 || k < 1 || k > std::min(m, n) || p < 0 || q < 0 ||
      q > GRAD_MAX_Q)
    return 0;
  return layout_grad(make_shape(RSVD_OP_SVD, dtype, m, n, k, p, q), nullptr, nullptr);
}

int rsvd_svd_grad(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
                  uint64_t seed, const double* A, int64_t lda, const double* dU, int64_t lddu,
                  const double* dS, const double* dV, int64_t lddv, const double* dres,
                  double* dA, int64_t ldda, double* U, int64_t ldu, double* S, double* V,
                  int64_t ldv, double* resid2, void* work, size_t work_bytes, int32_t* info,
                  void* stream) {
  if (!h) return -1;
  if (dtype != RSVD_F64) return dtype == RSVD_F32 || dtype == RSVD_BF16 ? RSVD_ERR_UNSUPPORTED : -2;
  if (m < 1) return -3;
  if (n < 1) return -4;
  if (k < 1 || k > std::min(m, n)) return -5;
  if (p < 0) return -6;
  if (q < 0) return -7;
  if (q > GRAD_MAX_Q) return RSVD_ERR_UNSUPPORTED;
  if (!A) return -9;
  if (lda < n) return -10;
  if (dU && lddu < k) return -12;
  if (dV && lddv < k) return -15;
  if (dA && ldda < n) return -18;
  if (U && ldu < k) return -20;
  if (V && ldv < k) return -23;
  if (!dA && !U && !S && !V && !resid2) return -17;
  if (!work) return -25;
  if (!info) return -27;
  const Shape s = make_shape(RSVD_OP_SVD, dtype, m, n, k, p, q);
  if (s.l > MAX_L) return RSVD_ERR_UNSUPPORTED;
  GradBufs g;
  const size_t need = layout_grad(s, work, &g);
  if (work_bytes < need) return RSVD_ERR_WORKSPACE;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  Ctx c{static_cast<hipStream_t>(stream), h->ncu, info, seed, 0, h};
  GradIO io;
  io.dU = dU; io.dS = dS; io.dV = dV; io.dres = dres; io.lddu = lddu; io.lddv = lddv;
  io.dA = dA; io.ldda = ldda;
  io.U = U; io.S = S; io.V = V; io.resid2 = resid2; io.ldu = ldu; io.ldv = ldv;
  return finish(run_grad(c, s, g, A, lda, io));
}

int rsvd_batch_create(rsvd_handle_t h, int64_t count, const int64_t* m, const int64_t* n,
                      const int32_t* k, int p, int q, rsvd_batch_t* plan) {
  using namespace rsvd;
  if (!h) return -1;
  if (count < 1) return -2;
  if (!m) return -3;
  if (!n) return -4;
  if (!k) return -5;
  if (p < 0) return -6;
  if (q < 0) return -7;
  if (!plan) return -8;
  for (int64_t i = 0; i < count; ++i) {
    if (m[i] < 1) return -3;
    if (n[i] < 1) return -4;
    if (k[i] < 1 || k[i] > std::min(m[i], n[i])) return -5;
    const int64_t l = std::min<int64_t>((int64_t)k[i] + p, std::min(m[i], n[i]));
    if (rup(l, 16) > BATCH_MAX_LP) return RSVD_ERR_UNSUPPORTED;
  }
  rsvd_batch_s* b = new rsvd_batch_s;
  b->h = h;
  b->count = count;
  b->p = p;
  b->q = q;
  b->a_off.resize(count); b->lda.resize(count); b->u_off.resize(count);
  b->s_off.resize(count); b->v_off.resize(count);
  int64_t ao = 0, uo = 0, so = 0, vo = 0;
  b->mmax = b->nmax = 0;
  std::vector<BatchDesc> d(count);
  for (int64_t i = 0; i < count; ++i) {
    const int64_t ld = rup(n[i], 4);
    b->a_off[i] = ao; b->lda[i] = ld; b->u_off[i] = uo; b->s_off[i] = so; b->v_off[i] = vo;
    BatchDesc& e = d[i];
    e.m = m[i]; e.n = n[i]; e.lda = ld;
    e.a_off = ao; e.u_off = uo; e.v_off = vo; e.s_off = so;
    e.k = k[i];
    e.l = (int32_t)std::min<int64_t>((int64_t)k[i] + p, std::min(m[i], n[i]));
    e.lp = (int32_t)rup(e.l, 16);
    e.index = (int32_t)i;
    e.variant = 0;
    e.pad = 0;
    ao += m[i] * ld;
    uo += m[i] * k[i];
    so += k[i];
    vo += n[i] * k[i];
    b->mmax = std::max(b->mmax, m[i]);
    b->nmax = std::max(b->nmax, n[i]);
  }
  b->a_elems = ao; b->u_elems = uo; b->s_elems = so; b->v_elems = vo;
  // queue order: decreasing work (passes 2 (2q+2) m n l), ties by index
  std::vector<int64_t> ord(count);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) {
    return d[x].m * d[x].n * d[x].l > d[y].m * d[y].n * d[y].l;
  });
  b->desc.resize(count);
  for (int64_t i = 0; i < count; ++i) b->desc[i] = d[ord[i]];
  b->grid = (int)std::min<int64_t>(h->ncu, count);
  // workspace: [queue head][descriptors][one slot per workgroup]
  const int64_t lpm = BATCH_MAX_LP;
  const int64_t rmax = std::max(b->mmax, b->nmax);
  auto r256 = [](int64_t x) { return (x + 255) & ~(int64_t)255; };
  int64_t o = 0;
  b->off_om = o; o = r256(o + b->nmax * lpm * 4);
  b->off_y = o;  o = r256(o + b->mmax * lpm * 4);
  b->off_q = o;  o = r256(o + b->mmax * lpm * 4);
  b->off_z = o;  o = r256(o + b->nmax * lpm * 4);
  b->off_zq = o; o = r256(o + b->nmax * lpm * 4);
  b->off_t = o;  o = r256(o + rmax * lpm * 8);
  b->off_qh = o; o = r256(o + b->nmax * lpm * 8);
  b->off_uh = o; o = r256(o + lpm * lpm * 8);
  b->off_vh = o; o = r256(o + lpm * lpm * 8);
  b->slot_bytes = o;
  b->desc_off = 256;
  b->slot_off = r256(b->desc_off + count * (int64_t)sizeof(BatchDesc));
  b->work_bytes = (size_t)(b->slot_off + b->grid * b->slot_bytes);
  b->prepared = nullptr;
  *plan = b;
  return RSVD_OK;
}

int rsvd_batch_destroy(rsvd_batch_t plan) {
  delete plan;
  return RSVD_OK;
}

int rsvd_batch_layout(rsvd_batch_t b, int64_t* a_elems, int64_t* u_elems, int64_t* s_elems,
                      int64_t* v_elems, int64_t* a_off, int64_t* lda, int64_t* u_off,
                      int64_t* s_off, int64_t* v_off) {
  if (!b) return -1;
  if (a_elems) *a_elems = b->a_elems;
  if (u_elems) *u_elems = b->u_elems;
  if (s_elems) *s_elems = b->s_elems;
  if (v_elems) *v_elems = b->v_elems;
  const size_t nb = sizeof(int64_t) * (size_t)b->count;
  if (a_off) std::memcpy(a_off, b->a_off.data(), nb);
  if (lda) std::memcpy(lda, b->lda.data(), nb);
  if (u_off) std::memcpy(u_off, b->u_off.data(), nb);
  if (s_off) std::memcpy(s_off, b->s_off.data(), nb);
  if (v_off) std::memcpy(v_off, b->v_off.data(), nb);
  return RSVD_OK;
}

size_t rsvd_batch_workspace_bytes(rsvd_batch_t b) { return b ? b->work_bytes : 0; }

static_assert(RSVD_BATCH_VARIANTS == rsvd::BATCH_VARIANTS, "pass shape count");

int rsvd_batch_set_variants(rsvd_batch_t b, const int32_t* variant) {
  if (!b) return -1;
  if (!variant) return -2;
  for (int64_t i = 0; i < b->count; ++i)
    if (variant[i] < 0 || variant[i] >= rsvd::BATCH_VARIANTS) return -2;
  for (auto& d : b->desc) d.variant = variant[d.index];
  b->prepared = nullptr;   // the device copy of the descriptors is stale
  return RSVD_OK;
}

int rsvd_batch_prepare(rsvd_batch_t b, void* work, size_t work_bytes, void* stream) {
  if (!b) return -1;
  if (!work) return -2;
  if (work_bytes < b->work_bytes) return RSVD_ERR_WORKSPACE;
  if (hipSetDevice(b->h->device) != hipSuccess) return RSVD_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(work);
  if (hipMemcpyAsync(w + b->desc_off, b->desc.data(), sizeof(rsvd::BatchDesc) * b->count,
                     hipMemcpyHostToDevice, st) != hipSuccess)
    return RSVD_ERR_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return RSVD_ERR_HIP;
  b->prepared = work;
  return RSVD_OK;
}

int rsvd_batch_svd(rsvd_batch_t b, uint64_t seed, const float* A, float* U, double* S, float* V,
                   void* work, size_t work_bytes, int32_t* info, void* stream) {
  using namespace rsvd;
  if (!b) return -1;
  if (!A || (reinterpret_cast<uintptr_t>(A) & 15)) return -3;
  if (!U) return -4;
  if (!S) return -5;
  if (!V) return -6;
  if (!work || (reinterpret_cast<uintptr_t>(work) & 255)) return -7;
  if (work_bytes < b->work_bytes) return RSVD_ERR_WORKSPACE;
  if (work != b->prepared) return -7;   // the descriptors are not in this workspace
  if (!info) return -9;
  if (hipSetDevice(b->h->device) != hipSuccess) return RSVD_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(work);
  BatchArgs g;
  g.desc = reinterpret_cast<const BatchDesc*>(w + b->desc_off);
  g.count = b->count;
  g.counter = reinterpret_cast<int32_t*>(w);
  g.A = A; g.U = U; g.S = S; g.V = V;
  g.scratch = w + b->slot_off;
  g.slot_bytes = b->slot_bytes;
  g.off_om = b->off_om; g.off_y = b->off_y; g.off_q = b->off_q; g.off_z = b->off_z;
  g.off_zq = b->off_zq; g.off_t = b->off_t; g.off_qh = b->off_qh; g.off_uh = b->off_uh;
  g.off_vh = b->off_vh;
  g.k0 = (uint32_t)seed; g.k1 = (uint32_t)(seed >> 32);
  g.q = b->q;
  g.info = info;
  hipError_t e = launch_set_word(info, 0, st);
  if (e == hipSuccess) e = launch_set_word(info + 1, 0, st);
  if (e == hipSuccess) e = launch_batch_rsvd(g, b->grid, st);
  return finish(e);
}

int rsvd_cur(rsvd_handle_t h, int dtype, int64_t m, int64_t n, int k, int p, int q,
             uint64_t seed, const void* A, int64_t lda, int64_t* Jc, int64_t* Jr,
             double* Ucur, int64_t lduc, void* work, size_t work_bytes, int32_t* info,
             void* stream) {
  int rc = check_common(h, dtype, m, n, k, p, q);
  if (rc) return rc;
  if (!A) return -9;
  if (lda < n) return -10;
  if (dtype == RSVD_BF16 && (lda % 8 || (reinterpret_cast<uintptr_t>(A) & 15))) return -10;
  if (!Jc) return -11;
  if (!Jr) return -12;
  if (!Ucur) return -13;
  if (lduc < k) return -14;
  if (!work) return -15;
  if (!info) return -17;
  const Shape s = make_shape(RSVD_OP_CUR | RSVD_OP_ID, dtype, m, n, k, p, q);
  if (s.l > MAX_L || !plan_cpqr(s.l, n, k, NCU_CAP).ok || !plan_cpqr(k, m, k, NCU_CAP).ok)
    return RSVD_ERR_UNSUPPORTED;
  Bufs b;
  const size_t need = layout(s, work, &b);
  if (work_bytes < need) return RSVD_ERR_WORKSPACE;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  Ctx c{static_cast<hipStream_t>(stream), h->ncu, info, seed, 0, h};
  Outs o;
  std::memset(&o, 0, sizeof(o));
  o.Jc = Jc; o.Jr = Jr; o.Ucur = Ucur; o.lduc = lduc;
  return finish(run_decompose(c, s, b, A, lda, o));
}

// ---------------------------------------------------------------- stages --

int rsvd_sketch(rsvd_handle_t h, int dtype, uint64_t seed, int64_t n, int64_t l, void* Omega,
                int64_t ldo, void* stream) {
  if (!h) return -1;
  if (dtype != RSVD_F64 && dtype != RSVD_F32) return -2;
  if (n < 0) return -4;
  if (l < 0) return -5;
  if (!Omega && n * l > 0) return -6;
  if (ldo < l) return -7;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  return finish(launch_sketch(dtype == RSVD_F32, seed, 0, 0, n, l, Omega, ldo,
                              static_cast<hipStream_t>(stream)));
}

int rsvd_philox(rsvd_handle_t h, uint64_t seed, uint32_t stream_id, uint32_t batch,
                uint64_t first, int64_t count, uint32_t* out, void* stream) {
  if (!h) return -1;
  if (count < 0) return -6;
  if (!out && count > 0) return -7;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  return finish(launch_philox_words(seed, stream_id, batch, first, count, out,
                                    static_cast<hipStream_t>(stream)));
}

size_t rsvd_pass_workspace_bytes(int dtype, int trans, int64_t m, int64_t n, int64_t l) {
  if ((dtype != RSVD_F64 && dtype != RSVD_F32 && dtype != RSVD_BF16) || m < 1 || n < 1 || l < 1)
    return 0;
  const int64_t M = trans ? n : m, K = trans ? m : n;
  if (dtype == RSVD_BF16) {
    if (l > MAX_L_SVD) return 0;
    return gemm_bf16_part_bytes(plan_gemm_bf16(M, K, l, NCU_CAP)) + 256 +
           (size_t)rup(l, 16) * rup(K, 32) * sizeof(uint16_t) + 256;
  }
  return std::max(gemm_part_bytes(plan_gemm(M, K, l, NCU_CAP, 0), 8),
                  narrow_work_bytes(dtype == RSVD_F32, trans != 0, M, K, l, NCU_CAP)) + 256;
}

size_t f8_pass_layout(int trans, int64_t m, int64_t n, int64_t l, void* base, F8Bufs* f,
                      void** part, size_t* part_bytes) {
  const int64_t M = trans ? n : m, K = trans ? m : n;
  const int lp = (int)rup(l, 16);
  const size_t pb = gemm_f8_part_bytes(plan_gemm_f8(M, K, l, NCU_CAP));
  Arena a(base);
  F8Bufs b;
  b.xt = a.take<uint8_t>((size_t)2 * lp * rup(K, 16));
  b.t = a.take<float>((size_t)2 * lp);
  b.tmax = a.take<uint32_t>((size_t)lp);
  void* pp = a.take<char>(pb);
  if (f) *f = b;
  if (part) *part = pp;
  if (part_bytes) *part_bytes = pb;
  return a.off;
}

size_t rsvd_pass_f8_workspace_bytes(int trans, int64_t m, int64_t n, int64_t l) {
  if ((trans != 0 && trans != 1) || m < 1 || n < 1 || l < 1 || l > MAX_L_SVD) return 0;
  return f8_pass_layout(trans, m, n, l, nullptr, nullptr, nullptr, nullptr);
}

int rsvd_pass_f8(rsvd_handle_t h, int trans, int64_t m, int64_t n, int64_t l, const uint8_t* A,
                 int64_t lda, const float* a_col_scale, const float* X, int64_t ldx, float* Y,
                 int64_t ldy, int split, void* work, size_t work_bytes, void* stream) {
  if (!h) return -1;
  if (trans != 0 && trans != 1) return -2;
  if (m < 1) return -3;
  if (n < 1) return -4;
  if (l < 1) return -5;
  if (l > MAX_L_SVD) return RSVD_ERR_UNSUPPORTED;
  if (!A) return -6;
  if (lda < n || lda % 16 || (reinterpret_cast<uintptr_t>(A) & 15)) return -7;
  if (!a_col_scale) return -8;
  if (!X) return -9;
  if (ldx < l) return -10;
  if (!Y) return -11;
  if (ldy < l) return -12;
  if (split != 0 && split != 1) return -13;
  if (!work) return -14;
  if (work_bytes < rsvd_pass_f8_workspace_bytes(trans, m, n, l)) return RSVD_ERR_WORKSPACE;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  Ctx c{static_cast<hipStream_t>(stream), h->ncu, nullptr, 0, 0, h};
  void* part = nullptr;
  size_t pb = 0;
  f8_pass_layout(trans, m, n, l, work, &c.f8, &part, &pb);
  c.f8.ascale = a_col_scale;
  return finish(pass(c, 3, trans == 1, m, n, (int)l, A, lda, X, ldx, Y, ldy, part, pb, nullptr,
                     split == 1));
}

int rsvd_pass(rsvd_handle_t h, int dtype, int trans, int64_t m, int64_t n, int64_t l,
              const void* A, int64_t lda, const void* X, int64_t ldx, void* Y, int64_t ldy,
              void* work, size_t work_bytes, void* stream) {
  if (!h) return -1;
  if (dtype != RSVD_F64 && dtype != RSVD_F32 && dtype != RSVD_BF16) return -2;
  if (trans != 0 && trans != 1) return -3;
  if (m < 1) return -4;
  if (n < 1) return -5;
  if (l < 1) return -6;
  if (!A) return -7;
  if (lda < n) return -8;
  if (dtype == RSVD_BF16 && (lda % 8 || (reinterpret_cast<uintptr_t>(A) & 15))) return -8;
  if (!X) return -9;
  if (ldx < l) return -10;
  if (!Y) return -11;
  if (ldy < l) return -12;
  if (work_bytes < rsvd_pass_workspace_bytes(dtype, trans, m, n, l)) return RSVD_ERR_WORKSPACE;
  if (work_bytes > 256 && !work) return -13;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  Ctx c{static_cast<hipStream_t>(stream), h->ncu, nullptr, 0, 0, h};
  if (dtype == RSVD_BF16) {
    if (l > MAX_L_SVD) return RSVD_ERR_UNSUPPORTED;
    const int64_t K = trans ? m : n;
    const size_t xt_bytes = (size_t)rup(l, 16) * rup(K, 32) * sizeof(uint16_t) + 256;
    char* wb = static_cast<char*>(work);
    uint16_t* xt = reinterpret_cast<uint16_t*>(wb);
    return finish(pass(c, 2, trans == 1, m, n, (int)l, A, lda, X, ldx, Y, ldy, wb + xt_bytes,
                       work_bytes - xt_bytes, xt));
  }
  return finish(pass(c, dtype == RSVD_F32 ? 1 : 0, trans == 1, m, n, (int)l, A, lda, X, ldx, Y,
                     ldy, work, work ? work_bytes : 0));
}

size_t rsvd_orth_workspace_bytes(int dtype, int64_t rows, int64_t l) {
  if ((dtype != RSVD_F64 && dtype != RSVD_F32) || l < 1 || rows < l || l > MAX_L_SVD) return 0;
  return orth_step_layout(rows, (int)l, nullptr, nullptr, nullptr);
}

int rsvd_orth(rsvd_handle_t h, int dtype, int64_t rows, int64_t l, const void* Y, int64_t ldy,
              void* Q, int64_t ldq, double* R, int64_t ldr, uint64_t seed, void* work,
              size_t work_bytes, int32_t* info, void* stream) {
  if (!h) return -1;
  if (dtype != RSVD_F64 && dtype != RSVD_F32) return -2;
  if (rows < 1) return -3;
  if (l < 1 || l > rows) return -4;
  if (l > MAX_L_SVD) return RSVD_ERR_UNSUPPORTED;
  if (!Y) return -5;
  if (ldy < l) return -6;
  if (!Q) return -7;
  if (ldq < l) return -8;
  if (R && ldr < l) return -10;
  if (!work) return -12;
  if (work_bytes < rsvd_orth_workspace_bytes(dtype, rows, l)) return RSVD_ERR_WORKSPACE;
  if (!info) return -14;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  const int lp = (int)rup(l, 16);
  OrthBufs ob;
  double* Rfull = nullptr;
  orth_step_layout(rows, (int)l, work, &ob, &Rfull);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Ctx c{st, h->ncu, info, seed, 0, h};
  hipError_t e = launch_set_word(info, 0, st);
  if (e == hipSuccess) e = launch_set_word(info + 1, 0, st);
  const bool f32 = dtype == RSVD_F32;
  if (e == hipSuccess)
    e = orth(c, ob, f32, Y, ldy, rows, (int)l, Q, f32, ldq, R ? Rfull : nullptr, lp);
  if (e == hipSuccess && R)
    e = hipMemcpy2DAsync(R, ldr * sizeof(double), Rfull, lp * sizeof(double), l * sizeof(double),
                         l, hipMemcpyDeviceToDevice, st);
  return finish(e);
}

size_t rsvd_small_svd_workspace_bytes(int64_t l) {
  if (l < 1 || l > MAX_L_SVD) return 0;
  return jacobi_work_bytes((int)l) + sizeof(int32_t) + 256;
}

int rsvd_small_svd(rsvd_handle_t h, int64_t l, int k, const double* Rh, int64_t ldr, double* S,
                   double* Uh, int64_t lduh, double* Vh, int64_t ldvh, void* work,
                   size_t work_bytes, int32_t* info, void* stream) {
  if (!h) return -1;
  if (l < 1) return -2;
  if (l > MAX_L_SVD) return RSVD_ERR_UNSUPPORTED;
  if (k < 1 || k > l) return -3;
  if (!Rh) return -4;
  if (ldr < l) return -5;
  if (!S) return -6;
  if (!Uh) return -7;
  if (lduh < k) return -8;
  if (!Vh) return -9;
  if (ldvh < k) return -10;
  if (!work) return -11;
  if (work_bytes < rsvd_small_svd_workspace_bytes(l)) return RSVD_ERR_WORKSPACE;
  if (!info) return -13;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Arena a(work);
  double* jw = a.take<double>(jacobi_work_bytes((int)l) / sizeof(double) + 1);
  hipError_t e = launch_set_word(info, 0, st);
  if (e == hipSuccess) e = launch_set_word(info + 1, 0, st);
  if (e == hipSuccess)
    e = launch_jacobi(Rh, ldr, (int)l, k, jw, S, Uh, lduh, Vh, ldvh, h->jacobi_max_sweeps, info,
                      nullptr, h->giveup_test, st);
  return finish(e);
}

size_t rsvd_cpqr_workspace_bytes(int64_t r, int64_t c, int k) {
  if (r < 1 || c < 1 || k < 1 || k > std::min<int64_t>(std::min(r, c), 256)) return 0;
  const CpqrPlan p = plan_cpqr((int)r, c, k, NCU_CAP);
  if (!p.ok) return 0;
  const int kp = (int)rup(k, 16);
  Arena a(nullptr);
  a.take<char>(cpqr_work_bytes(p));
  a.take<double>((size_t)k * kp);
  a.take<double>((size_t)(c - k + 1) * kp);
  a.take<double>(k);
  return a.off;
}

int rsvd_cpqr(rsvd_handle_t h, int dtype, int64_t r, int64_t c, int k, const void* Bcols,
              int64_t ldb, int64_t* J, double* T, int64_t ldt, double* pivn, void* work,
              size_t work_bytes, int32_t* info, void* stream) {
  if (!h) return -1;
  if (dtype != RSVD_F64 && dtype != RSVD_F32) return -2;
  if (r < 1 || r > 65536) return -3;
  if (c < 1) return -4;
  if (k < 1 || k > std::min(r, c)) return -5;
  if (k > 256) return RSVD_ERR_UNSUPPORTED;
  if (!Bcols) return -6;
  if (ldb < r) return -7;
  if (!J) return -8;
  if (!T && c > k) return -9;
  if (ldt < c - k) return -10;
  if (!work) return -12;
  const CpqrPlan p = plan_cpqr((int)r, c, k, NCU_CAP);
  if (!p.ok) return RSVD_ERR_UNSUPPORTED;
  if (work_bytes < rsvd_cpqr_workspace_bytes(r, c, k)) return RSVD_ERR_WORKSPACE;
  if (!info) return -14;
  if (hipSetDevice(h->device) != hipSuccess) return RSVD_ERR_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int kp = (int)rup(k, 16);
  Arena a(work);
  void* cw = a.take<char>(cpqr_work_bytes(p));
  double* S11t = a.take<double>((size_t)k * kp);
  double* S12t = a.take<double>((size_t)(c - k + 1) * kp);
  double* pv = a.take<double>(k);
  const CpqrPlan pr = plan_cpqr((int)r, c, k, std::min(h->ncu, NCU_CAP));
  hipError_t e = launch_set_word(info, 0, st);
  if (e == hipSuccess) e = launch_set_word(info + 1, 0, st);
  if (e == hipSuccess)
    e = launch_cpqr(dtype == RSVD_F32, Bcols, ldb, (int)r, c, k, pr, cw, J, S11t, S12t, kp, pv,
                    info, h->giveup_test, st);
  if (e == hipSuccess && c > k)
    e = launch_backsub(S11t, 1, kp, S12t, 1, kp, k, c - k, T, ldt, 1, st);
  if (e == hipSuccess && pivn)
    e = hipMemcpyAsync(pivn, pv, sizeof(double) * k, hipMemcpyDeviceToDevice, st);
  return finish(e);
}

}  // extern "C"
