// Internal declarations shared by the libicur translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "icur.h"

namespace icur {

// Error plumbing: every host wrapper returns an icur_status; the message of the last
// failure of the calling thread is kept for icur_last_error().
void set_error(const std::string& msg);
const char* last_error();

#define ICUR_HIP(call)                                                         \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      ::icur::set_error(std::string(#call) + ": " + hipGetErrorString(e_));    \
      return ICUR_ERR_HIP;                                                     \
    }                                                                          \
  } while (0)

#define ICUR_TRY(expr)        \
  do {                        \
    int s_ = (expr);          \
    if (s_ < 0) return s_;    \
  } while (0)

inline int arg_error(const std::string& msg) {
  set_error(msg);
  return ICUR_ERR_ARG;
}

inline int hip_error(hipError_t e, const std::string& where) {
  set_error(where + ": " + hipGetErrorString(e));
  return ICUR_ERR_HIP;
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Device properties of the current device (cached).
struct DeviceInfo {
  int device;
  int num_cus;
};
int device_info(DeviceInfo* out);

// ----- sketch operator (icur_rng.hip) -----
// G is c x m BF16 bit patterns, row-major with leading dimension ldg >= m.
int launch_gaussian_G(uint64_t seed, int64_t c, int64_t m, uint16_t* G, int64_t ldg, hipStream_t st);
// Same values, entry (r, i) stored at G[r * sr + i * si] (si = ldgt, sr = 1: transposed).
int launch_gaussian_G_strided(uint64_t seed, int64_t c, int64_t m, uint16_t* G, int64_t sr, int64_t si,
                              hipStream_t st);
int launch_sparse_sign(uint64_t seed, int64_t c, int64_t m, int zeta, uint8_t* rows,
                       uint8_t* signs, uint16_t* G_dense, int64_t ldg, hipStream_t st);
// SRTT operator (c <= m): kept rows (c int64, increasing) and, when G is given, the
// dense c x ldg FP32 operator.  mark: m bytes of scratch.
int launch_srtt(uint64_t seed, int64_t c, int64_t m, float* G, int64_t ldg, int64_t* rows, uint8_t* mark,
                hipStream_t st);

// ----- wide products (icur_gemm.hip, icur_wide_*.hip) -----
// OUT(M x N) = X - W(M x K) B(K x N) (subtract) or W B.  X and OUT are FP32, or FP64 when
// out64.  W is FP32 (wterms == 0; BF16 bit patterns widened to FP32 when w_bf16) or
// `wterms` BF16 pieces stored as consecutive M x ldw planes of uint16.  B is FP32, split
// on the fly into `bterms` BF16 pieces; products of pieces (i, j) with i + j <
// max(wterms, bterms) are summed.  Chunks of 32 K rows are summed on the matrix cores
// and accumulated in FP64.  norm_partials (device, may be null) receives per-block FP64
// partial sums of OUT^2; the number written is returned in *nparts.
struct WideGemm {
  const void* X;
  int64_t ldx;
  const void* W;
  int64_t ldw;
  int wterms;    // -1: FP64 W and B on FP64 matrix cores (needs out64)
  bool w_bf16;
  const void* B;
  int64_t ldb;
  int bterms;
  int64_t M, K, N;
  bool subtract;
  bool out64;
  void* OUT;
  int64_t ldo;
  double* norm_partials;
  int* nparts;
};
int wide_gemm(const WideGemm& g, void* workspace, size_t workspace_bytes, hipStream_t st);

// ----- the sketch product (icur_sketch.hip) -----
// X0 (c x n, FP64, ld ldx) = G A with G the c x m BF16 sketch (leading dimension ldg, a
// multiple of 8, 16-byte aligned) and A the m x n FP32 input, each element of A split into
// `terms` (1..3) BF16 pieces; FP32 sums over 128-row blocks are accumulated in FP64
// (over 32-row chunks when precise, which needs terms 3); per-block FP64 partial sums of
// X0^2 land in norm_partials (count in *nparts).  Returns ICUR_ERR_UNSUPPORTED for
// shapes outside its fast path (misaligned A or G, terms 0, very long rows) before
// launching anything; the caller then uses wide_gemm.  ev_begin / ev_end (may be null)
// are recorded around the first slice's sketch kernel.
int sketch_product(const uint16_t* G, int64_t ldg, int64_t c, const float* A, int64_t m, int64_t n,
                   int64_t lda, int terms, bool precise, double* X0, int64_t ldx, double* norm_partials,
                   int* nparts, void* workspace, size_t workspace_bytes, hipStream_t st, hipEvent_t ev_begin,
                   hipEvent_t ev_end);
size_t sketch_workspace_bytes(int64_t c, int64_t m, int64_t n, int num_cus);
// dst (FP32, ld ldd) = src (FP64 M x N, ld N), with per-block partial sums of dst^2
// (at most 1024 blocks; count in *nparts).
int convert_f64_f32_norm(const double* src, int64_t M, int64_t N, float* dst, int64_t ldd, double* norm_partials,
                         int* nparts, hipStream_t st);
int sketch_max_norm_partials(int64_t c, int64_t n);
size_t wide_gemm_workspace_bytes(int64_t M, int64_t K, int64_t N, int num_cus);
int max_norm_partials(int64_t M, int64_t N);

// FP64 -> BF16 pieces (terms planes) or FP32 (terms == 0), optionally transposed.
// src is rows x cols with leading dimension lds; dst is (trans ? cols x rows : rows x
// cols) with leading dimension ldd (elements), planes of stride plane.
int launch_split_f64(const double* src, int64_t rows, int64_t cols, int64_t lds, bool trans,
                     int terms, void* dst, int64_t ldd, int64_t plane, hipStream_t st);

// Sum of per-block partials into out (device double, written in a fixed order).
int launch_reduce_partials(const double* partials, int n, double* out, hipStream_t st);

// Sketch accumulation: FP32 sums over 128 rows of A give X0 a relative noise near
// sqrt(128) 2^-24; the column residual subtracts X0(:,J) times interpolation coefficients
// whose norm reaches tens on ill-conditioned crosses, which puts a floor near 1e-5 under
// rho.  Below this tolerance the sums are widened to FP64 after every 32 rows.
constexpr double kSketchChunkFlushBelow = 1e-4;
// BF16 pieces per FP32 operand of the split form for a tolerance (icur_api.hip).
int terms_for_tol(double tol);
// BF16 pieces per operand of the split form's FP32-factor residual products.
int residual_terms_for_tol(double tol);
// Bytes of the G buffer form_sketch needs (BF16 operators: c x ldg x 2; SRTT: the FP32
// operator, its kept rows and m bytes of scratch).
size_t sketch_G_bytes(int kind, int64_t c, int64_t m, int64_t ldg);
// G drawn from (kind, seed, zeta) into G (c x ldg BF16), X0 = G A into S (c x n FP64,
// leading dimension n) and ||X0||_F^2 into *normsq_dev (device).  terms: BF16 pieces of A
// (1..3) or 0 for FP32 matrix cores; precise: FP64 flush every 32 rows.  partials holds
// the norm partials (at least max(sketch_max_norm_partials, max_norm_partials)), ws the
// product workspace.  ev_begin / ev_end (may be null) bracket the product kernel;
// *used_kernel (may be null) tells whether the dedicated sketch kernel ran (else the
// general product).
int form_sketch(int kind, uint64_t seed, int64_t c, int64_t m, int64_t n, const float* A, int64_t lda, int zeta,
                int terms, bool precise, uint16_t* G, int64_t ldg, double* S, double* partials, void* ws,
                size_t ws_bytes, double* normsq_dev, hipStream_t st, hipEvent_t ev_begin, hipEvent_t ev_end,
                bool* used_kernel = nullptr);

// ----- sparse input (icur_csr.hip) -----
struct CsrMatrix {
  const int64_t* rowptr;  // m + 1
  const int32_t* colind;  // nnz, sorted and unique within each row
  const float* vals;      // nnz
  int64_t m, n, nnz;
};
struct CscCopy {
  int64_t* colptr;          // n + 1
  unsigned long long* ent;  // nnz entries (row << 32) | FP32 bits, rows increasing within each column
};
// Device flag (bit 0 rowptr, bit 1 column range, bit 2 order within a row); 0 = valid.
int csr_validate(const CsrMatrix& A, unsigned* flag_dev, hipStream_t st);
size_t csc_workspace_bytes(int64_t nnz, int64_t n);
int csc_build(const CsrMatrix& A, CscCopy* out, void* ws, size_t ws_bytes, hipStream_t st);
// X0 (c x n FP64, ld ldx) = G A from the CSC copy, G drawn here from (kind, seed, zeta);
// per-block norm partials (count in *nparts).  aux: csr_sketch_aux_bytes(m, c).
size_t csr_sketch_aux_bytes(int64_t m, int64_t c);
int csr_sketch(const CscCopy& csc, int64_t m, int64_t n, int64_t c, int kind, uint64_t seed, int zeta, double* X0,
               int64_t ldx, double* norm_partials, int* nparts, void* aux, hipStream_t st);
int csr_max_norm_partials(int64_t n);
// Dense gathers: Ct row t = A(:, cols[t]); R row t = A(rows[t], :); M = A(I, J) (FP64).
int csc_gather_cols_T(const CscCopy& csc, int64_t m, const int64_t* cols, int64_t k, float* Ct, int64_t ldct,
                      hipStream_t st);
int csc_gather_cols_T(const CscCopy& csc, int64_t m, const int64_t* cols, int64_t k, double* Ct, int64_t ldct,
                      hipStream_t st);
int csr_gather_rows(const CsrMatrix& A, const int64_t* rows, int64_t k, float* R, int64_t ldr, hipStream_t st);
int csr_gather_rows(const CsrMatrix& A, const int64_t* rows, int64_t k, double* R, int64_t ldr, hipStream_t st);
int csr_gather_cross(const CsrMatrix& A, const int64_t* I, int64_t rk, const int64_t* J, int64_t ck, double* M,
                     int64_t ldm, hipStream_t st);

// ----- selection (icur_lupp.hip) -----
struct LuppWork {
  double* L;          // steps_cap x N_cap multipliers
  double* P;          // 16 x N_cap: the current panel
  double* U;          // steps_cap x steps_cap: extended pivot rows
  uint8_t* chosen;    // N_cap flags
  void* slots;        // 2 * max_groups slot records
  unsigned* ctl;      // barrier counter and status words, cleared by every call
  int* status;        // [0] npiv, [1] fault flag, [2] ended early (inside ctl)
  unsigned long long* ref;  // |first pivot| bit pattern (inside ctl)
  int64_t steps_cap, N_cap;
  int max_groups;     // > 0: cap on the panel grid's workgroups (0: one per CU)
};
size_t lupp_workspace_bytes(int64_t steps, int64_t N);
// Candidates one panel grid of at most max_groups workgroups holds.
int64_t lupp_max_candidates(int max_groups);
int lupp_bind_workspace(void* base, int64_t steps, int64_t N, LuppWork* w);
// Pivots of LUPP on T = X^T (see icur_lupp); X is FP32, or FP64 when x64.  piv is
// device; the pivot count and a fault flag land in w.status.  rel_cut > 0 also ends the
// selection at a pivot |p| <= rel_cut * |first pivot| (numerically zero Schur complement).
int lupp_launch(const void* X, bool x64, int64_t K, int64_t N, int64_t ldx, int steps,
                const uint8_t* excluded, int64_t* piv, const LuppWork& w, hipStream_t st, double rel_cut = 0.0);

// Pivots of QR with column pivoting on T = X^T (icur_qrcp.hip), same status words as
// lupp_launch (status[0] pivots found); ws holds qrcp_workspace_bytes(K, N, 4 CUs).
size_t qrcp_workspace_bytes(int64_t K, int64_t N, int groups);
int qrcp_launch(const void* X, bool x64, int64_t K, int64_t N, int64_t ldx, int steps, const uint8_t* excluded,
                int64_t* piv, int* status, void* ws, size_t ws_bytes, hipStream_t st, double rel_cut = 0.0);

// ----- gathers and small FP64 kernels (icur_gather.hip) -----
int launch_gather_cols_T(const float* A, int64_t m, int64_t n, int64_t lda, const int64_t* cols,
                         int64_t k, float* Ct, int64_t ldct, hipStream_t st);
int launch_gather_cols_T(const float* A, int64_t m, int64_t n, int64_t lda, const int64_t* cols,
                         int64_t k, double* Ct, int64_t ldct, hipStream_t st);
int launch_gather_rows(const float* A, int64_t m, int64_t n, int64_t lda, const int64_t* rows,
                       int64_t k, float* R, int64_t ldr, hipStream_t st);
int launch_gather_rows(const float* A, int64_t m, int64_t n, int64_t lda, const int64_t* rows,
                       int64_t k, double* R, int64_t ldr, hipStream_t st);
// dst(rk x ck, FP64, ld ldd) = src[rows[i]][cols[j]] (FP32 src with leading dim lds);
// rows/cols null means identity offset (i or j).  trans: dst(j, i) instead.
int launch_gather_f64(const float* src, int64_t lds, const int64_t* rows, int64_t rk,
                      const int64_t* cols, int64_t ck, bool trans, double* dst, int64_t ldd,
                      hipStream_t st);
// Same with an FP64 source.
int launch_gather_f64(const double* src, int64_t lds, const int64_t* rows, int64_t rk,
                      const int64_t* cols, int64_t ck, bool trans, double* dst, int64_t ldd,
                      hipStream_t st);
// colmask[Jk[t]] = rowmask[Ik[t]] = 1 and Jall[t] = Jk[t], Iall[t] = Ik[t] for t < k.
// Device segments copied into host-mapped pinned memory (host_dev: its device address).
constexpr int kMaxHostSegs = 4;
struct HostSeg {
  const void* src;
  int64_t bytes;
  int64_t dst_off;
};
struct HostSegs {
  HostSeg seg[kMaxHostSegs];
  int n;
};
int launch_to_host(const HostSegs& segs, void* host_dev, hipStream_t st);
// The end of a loop iteration in one launch: *norm_out = the sum of nparts partials (in
// the order of launch_reduce_partials), the commit of k selected indices (as
// launch_commit_block), then rec (rec_bytes, holding norm_out) copied to host_dev and,
// when flag_dev is given, seq published there after the copy is visible.
int launch_iteration_end(const double* partials, int nparts, double* norm_out, uint8_t* colmask, uint8_t* rowmask,
                         const int64_t* Jk, const int64_t* Ik, int64_t k, int64_t* Jall, int64_t* Iall,
                         const void* rec, int64_t rec_bytes, void* host_dev, unsigned* flag_dev, unsigned seq,
                         hipStream_t st);
// One workgroup; writes seq to *flag_dev (host-mapped) after the segments are visible.
int launch_to_host_flag(const HostSegs& segs, void* host_dev, unsigned* flag_dev, unsigned seq, hipStream_t st);

int launch_commit_block(uint8_t* colmask, uint8_t* rowmask, const int64_t* Jk, const int64_t* Ik, int64_t k,
                        int64_t* Jall, int64_t* Iall, hipStream_t st);
int launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t st);
// Per-workgroup FP64 partial sums of squares of an m x n FP32 matrix (ld lda): at most
// kSumsqMaxParts partials (count in *nparts), summed by launch_reduce_partials.
constexpr int kSumsqMaxParts = 1024;
int launch_sumsq_f32(const float* A, int64_t m, int64_t n, int64_t lda, double* partials, int* nparts,
                     hipStream_t st);
int launch_fill_u32(unsigned* p, int64_t n, unsigned v, hipStream_t st);

// ----- FP64 dense kernels (icur_core.hip) -----
// C(M x N) = alpha * A(M x K) B(K x N) + beta * C with element strides:
// A(i,k) = A[i*sa0 + k*sa1], B(k,j) = B[k*sb0 + j*sb1], C(i,j) = C[i*ldc + j].
// Destroys the library GEMM handles (icur_release).
void release_blas_handles();
int dgemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t sa0,
          int64_t sa1, const double* B, int64_t sb0, int64_t sb1, double beta, double* C,
          int64_t ldc, hipStream_t st);
// In-place inverse of the k x k matrix N (ld k) by Gauss-Jordan elimination with
// partial pivoting in FP64; *info = 0 on success, 1 on an exactly zero pivot.  norms
// (device, may be null) receives ||N||_1 and ||N^-1||_1 (max column sums).
int launch_small_inverse(double* N, int64_t k, double* work, int* info, double* norms,
                         hipStream_t st);
// Inverse of a k x k block whose rows are in partial-pivoting order (the pivot block of a
// row selection, or a Schur complement of the cross in selection order): elimination on
// the diagonal without a pivot search (k <= 128; larger k use launch_small_inverse).
int launch_inorder_inverse(double* N, int64_t k, double* work, int* info, hipStream_t st);
size_t small_inverse_work_bytes(int64_t k);
// OUT (M x N, ld ldo) = X + alpha W B (X may be null, or equal to OUT with ldx == ldo), all
// FP64 row-major, on the FP64 matrix cores (icur_group_kernels.hip).
int gemm_f64_native(int64_t M, int64_t N, int64_t K, double alpha, const double* W, int64_t ldw, const double* B,
                    int64_t ldb, const double* X, int64_t ldx, double* OUT, int64_t ldo, hipStream_t st);
int dcopy2d(int64_t M, int64_t N, double alpha, const double* src, int64_t lds, double* dst,
            int64_t ldd, hipStream_t st);
// Grow the core inverse U (ld ldu) from r x r to (r+k) x (r+k) by the block inverse of
// the bordered matrix (see icur_core.hip).  Y is r x k (ld ldy), A21 k x r (ld r), A22
// k x k (ld k).  ws holds core_update_ws_doubles(r, k) doubles.  info/norms are device.
int core_update(double* U, int64_t ldu, int64_t r, int64_t k, const double* Y, int64_t ldy,
                const double* A21, const double* A22, double* ws, int* info, double* norms,
                hipStream_t st);
size_t core_update_ws_doubles(int64_t r, int64_t k);
// U = A(I,J)^{-1} from the gathered cross M (r x r, ld r, overwritten): block LU in the
// selection order, then block triangular solves on the identity.  info has one entry
// per block (0 = regular).  ws: core_inverse_ws_doubles(r, bmax) doubles.  D0inv, when
// given, is the inverse of the first diagonal block M(0:b0, 0:b0) (b0 = blocks[0], ld b0),
// already formed by the same kernel on the same values; it is used instead of inverting
// that block again, and with a single block U is a copy of it.
int core_block_inverse(double* M, int64_t r, const int64_t* blocks, int64_t nblocks, int64_t bmax, double* U,
                       double* ws, int* info, double* norms, hipStream_t st, const double* D0inv = nullptr);
size_t core_inverse_ws_doubles(int64_t r, int64_t bmax);
// Newton steps U <- U + U (I - M U) on the core (M = A(I,J), r x r, ld r): up to three,
// while max |I - M U| converges and exceeds floor (read by the host before each).  ws:
// core_refine_ws_doubles(r) doubles.
int core_refine(const double* M, double* U, int64_t r, double floor, double* ws, hipStream_t st);
size_t core_refine_ws_doubles(int64_t r);
int launch_fill_f64_identity(double* U, int64_t r, hipStream_t st);

}  // namespace icur
