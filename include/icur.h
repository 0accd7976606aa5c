/*
 * libicur: IterativeCUR on one MI355X (gfx950).
 *
 * IterativeCUR (Pritchard, Park, Nakatsukasa, Martinsson, "Fast Rank Adaptive CUR via a
 * Recycled Small Sketch", arXiv 2509.21963) builds A ~ C U R with C = A(:,J), R = A(I,:),
 * U = A(I,J)^+ by adding b columns and b rows per iteration until the sketched relative
 * residual rho = ||G (A - C U R)||_F / ||G A||_F falls to the tolerance (Alg. 1; notation
 * of §1.1; estimator of §3.3).  G is a c x m random sketch, c = floor(1.1 b), drawn once
 * and recycled in every iteration.
 *
 * Conventions for every entry point:
 *   - Matrices are row-major with 0-based indices.  A "device" pointer is memory the
 *     caller allocated on the current HIP device (hipMalloc or a torch CUDA tensor);
 *     a "host" pointer is ordinary CPU memory.  The library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *   - Calls are synchronous: they return after every output has been written (host
 *     outputs copied back, device outputs complete on `stream`).
 *   - Return value: ICUR_OK (0), a positive warning (outputs valid) or a negative error.
 *     Arguments are validated before any device work; on an argument error nothing is
 *     written.  icur_last_error() returns a message describing the last failure of the
 *     calling thread.
 *   - The library keeps a per-device workspace cache between calls; icur_release()
 *     frees it.  Calls on one device from several host threads are serialised
 *     internally.
 */
#ifndef ICUR_H
#define ICUR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum icur_status {
  ICUR_OK = 0,
  ICUR_MAXRANK = 1,          /* |J| reached max_rank with rho > tolerance; outputs valid */
  ICUR_STALLED = 2,          /* a block selected no index (exactly-zero residual pivots) */
  ICUR_ERR_ARG = -1,         /* invalid argument */
  ICUR_ERR_NONFINITE = -2,   /* ||G A||_F is not finite (A holds Inf/NaN) */
  ICUR_ERR_NOMEM = -3,       /* device allocation failed */
  ICUR_ERR_HIP = -4,         /* a HIP runtime call failed, or a kernel reported a fault */
  ICUR_ERR_UNSUPPORTED = -5  /* shape outside what the kernels support (see each call) */
};

enum icur_sketch_kind {
  ICUR_SKETCH_GAUSSIAN = 0,     /* N(0,1) entries rounded to BF16 (§3.4: Gaussian) */
  ICUR_SKETCH_SPARSE_SIGN = 1,  /* zeta entries +-1 per column of G (§2.1, §3.4) */
  ICUR_SKETCH_SRTT = 2          /* subsampled randomized trigonometric transform (§3.4, for
                                   very large m): sqrt(m/c) R F D with the orthonormal
                                   DCT-II F, random signs D and c kept rows R; dense input
                                   only, needs c <= m; applied in FP32 */
};

enum icur_precision {
  ICUR_FP32 = 0,       /* plain form: FP32 products and accumulation */
  ICUR_BF16_SPLIT = 1  /* BF16 matrix-core products of split hi/lo pieces, FP32 accumulate */
};

typedef struct icur_opts {
  int32_t precision;    /* icur_precision; default ICUR_FP32 */
  int32_t zeta;         /* nonzeros per column of a sparse-sign G; 0 -> 8 (clamped to c) */
  int64_t max_rank;     /* cap on |J|; 0 -> min(m, n) */
  void*   stream;       /* hipStream_t or NULL */
  double  alpha;        /* risk-aware stopping (§3.3, Corollary): 0 = off, else in (0,1);
                           Gaussian sketch only (the Corollary's hypothesis).  With
                           ICUR_DENOM_A the stop rho <= xi tol bounds the true error by
                           (1 + delta) tol with probability >= 1 - alpha; with the default
                           denominator xi is applied to rho as a heuristic */
  double  delta;        /* allowed deviation, >= 0 (used when alpha > 0) */
  int32_t split_terms;  /* BF16_SPLIT only: pieces per FP32 operand, 0 = from tol, 1..3 */
  int32_t sketch_fp32;  /* FP32 form only: 1 = form G A on FP32 matrix cores; 0 (default) =
                           exact products of three BF16 pieces of A with the BF16-valued G */
  int32_t residual_fp64; /* residual-form factors: 0 (default) or 1 = FP64 on the FP64
                            matrix cores; -1 = FP32 (plain form) or BF16 pieces (split form),
                            which round N_k^-1 before it multiplies, so the estimate can be
                            off by about cond(N_k) 2^-24: only for well-conditioned blocks */
  int32_t batch_workers; /* icur_run_batched only: 0 (default) the grouped form; 1..16
                            the worker form with that many concurrent matrices; ignored
                            by the single-matrix calls */
  int32_t denominator;  /* estimate's denominator: ICUR_DENOM_GA (0, default, Alg. 1) or
                           ICUR_DENOM_A (1): rho = ||S^col||_F / (s_G ||A||_F), the quantity
                           the §3.3 Corollary bounds (s_G^2 = c for the Gaussian G, min(zeta,c)
                           for the sparse-sign G); costs one extra read of A */
  int32_t selection;    /* index selection of both steps: ICUR_SELECT_LUPP (0, default) or
                           ICUR_SELECT_QRCP (1), Alg. 1's alternative (§5.3) */
  int32_t device_outputs; /* 0 (default): the index and core outputs (I, J, U, or the
                             batched call's pools) are host memory; 1: device memory of the
                             current device, written in stream order (no copy over PCIe).
                             rank, est_err and status stay host memory either way */
  int32_t pad_opts;
} icur_opts;

enum icur_selection {
  ICUR_SELECT_LUPP = 0,  /* LU with partial pivoting (§3.2.1, §3.2.2) */
  ICUR_SELECT_QRCP = 1   /* QR with column pivoting (Alg. 1; §5.3) */
};

enum icur_denominator {
  ICUR_DENOM_GA = 0,  /* rho = ||S^col||_F / ||G A||_F (Alg. 1); rho starts at 1 */
  ICUR_DENOM_A = 1    /* rho = ||S^col||_F / (s_G ||A||_F) (§3.3 Corollary; §5 footnote) */
};

/* Per-call statistics of the calling thread's last icur_run*/
typedef struct icur_info {
  int32_t iterations;
  int32_t split_terms;        /* BF16 pieces used (0 in the FP32 form) */
  double  sketch_norm;        /* ||G A||_F */
  double  threshold;          /* tolerance actually applied (xi * tol) */
  double  ms_total;           /* wall time of the call, host clock */
  double  ms_sketch;          /* G generation + G A + its norm (device events) */
  double  ms_select;          /* both LUPP selections, all iterations */
  double  ms_residual;        /* gathers, N_k^-1 and the residual-form products */
  double  ms_core;            /* FP64 assembly of U = A(I,J)^-1 after the loop */
  double  ms_sketch_product;  /* the G A product kernel(s) alone (device events) */
  int32_t n_rho;              /* entries written to rho[] and block_sizes[] (<= 512) */
  int32_t pad;
  double  rho[512];           /* rho after each iteration */
  int32_t block_sizes[512];   /* indices added by each iteration (b, or fewer when a
                                 block is cut short); I and J are these blocks in order */
  /* icur_run_batched, grouped form: ms_sketch above is the batch's sketch phase,
     ms_select the device time of its grouped selections, ms_residual the host clock of
     the grouped iterations and ms_core the device time of the closing core products
     (ms_sketch_product is 0); and: */
  double  ms_products;        /* device time of the grouped FP64 product launches */
  double  product_bytes;      /* their algorithmic bytes: the nonzero parts of the operands
                                 read once, the output written once */
  int32_t product_launches;
  int32_t group_iterations;   /* grouped iterations (the longest matrix's count) */
  double  ms_setup;           /* host clock of the per-matrix buffer set-up */
  double  ms_results;         /* host clock of the copies to the caller's pools after the loop */
  double  ms_stage[5];        /* device time of the product stages: row residual (P1), new-row
                                 residual and (Q^-1)^T block (P2), row factors and P^-1 block
                                 (P3), column update (P4), core products (FIN) */
  int32_t tiles[4];           /* tile shapes used for P1, P2, P3, FIN (0..5: workgroup tiles
                                 16x128, 32x128, 48x128, 64x128, 32x256, 64x256; 6..8: wave
                                 tiles 32x32, 16x64, 32x64; 9..11: workgroup tiles with more
                                 chunks in flight, 32x128 (2), 64x128 (2), 32x128 (3)) */
  int32_t sketch_kernel;      /* 1 when G A ran on the dedicated sketch kernel, 0 when on the
                                 general product (SRTT, FP32 matrix cores, shapes outside
                                 the kernel's fast path); batched: the count of matrices */
  int32_t residual_terms;     /* BF16 pieces per operand of the residual products: -1 for
                                 FP64 factors, 0 for FP32 factors on the FP32 matrix cores,
                                 2 or 3 in the precision form */
  double  stage_bytes[5];     /* grouped batched call: algorithmic bytes of the product stages
                                 of ms_stage (nonzero operand parts read once, output written
                                 once) */
  int32_t graph_iterations;   /* grouped batched call: iterations run as a replay of the
                                 captured hipGraph of one iteration (all but the first with
                                 ICUR_BATCH_GRAPH=1, else none; the stage times above are
                                 not measured in replays) */
  int32_t pad3;
} icur_info;

/*
 * icur_run: Alg. 1 on a dense FP32 matrix.
 *   A        device, m x n, row-major, leading dimension lda >= n; read only.
 *   tol      finite, > 0: stop when rho <= tol (times xi when opts->alpha > 0).
 *   block    b, 1 <= b <= min(m, n) and b <= 512; c = (11 b) / 10 sketch rows.
 *   sketch_kind, seed: G of icur_sketch_kind drawn from Philox4x32-10 keyed by seed.
 *   opts     may be NULL (all defaults).
 *   I, J     host (device with opts->device_outputs), capacity max_rank each: selected
 *            row / column indices in selection order (block by block, pivot order
 *            within a block).
 *   U        host (device with opts->device_outputs), capacity max_rank * max_rank
 *            doubles: the rank x rank core
 *            A(I,J)^{-1} (row-major, leading dimension rank), so A ~ A(:,J) U A(I,:).
 *   rank     host: |I| = |J|.
 *   est_err  host: the final rho.
 * Returns ICUR_OK, ICUR_MAXRANK, ICUR_STALLED or an error.  A zero matrix returns
 * ICUR_OK with rank 0 and est_err 0.
 */
int icur_run(const float* A, int64_t m, int64_t n, int64_t lda, double tol, int32_t block,
             int32_t sketch_kind, uint64_t seed, const icur_opts* opts, int64_t* I,
             int64_t* J, double* U, int64_t* rank, double* est_err);

/*
 * icur_run_csr: Alg. 1 on a sparse m x n matrix in CSR form (the paper's sparse test
 * matrices, §5; sparse inputs are where the cost of the sketch matters, §3.4).
 *   rowptr   device, m + 1 int64: row i holds entries rowptr[i] .. rowptr[i+1]-1,
 *            rowptr[0] = 0, rowptr[m] = nnz.
 *   colind   device, nnz int32: column indices, strictly increasing within each row.
 *   vals     device, nnz FP32.
 *   nnz      0 <= nnz < 2^31.
 * The other arguments and the outputs are those of icur_run (opts->sketch_fp32 does not
 * apply: the sparse sketch accumulates in FP64).  The CSR arrays are checked on the
 * device first; a non-canonical matrix returns ICUR_ERR_ARG before any other work.  The
 * call builds a column-compressed copy (8 bytes per entry plus n + 1 offsets) in the
 * cached workspace.  Needs c = floor(1.1 b) <= 256.
 */
int icur_run_csr(const int64_t* rowptr, const int32_t* colind, const float* vals, int64_t m,
                 int64_t n, int64_t nnz, double tol, int32_t block, int32_t sketch_kind,
                 uint64_t seed, const icur_opts* opts, int64_t* I, int64_t* J, double* U,
                 int64_t* rank, double* est_err);

/*
 * icur_run_batched: Alg. 1 on `count` independent dense FP32 matrices of uneven sizes and
 * tolerances (many small CUR problems at once; each follows Alg. 1 on its own).
 *   Grouped form (opts->batch_workers == 0, the default): every matrix with max(m, n) <=
 *   8192 (with block <= 64, LUPP selection and FP64 residual factors) advances together
 *   with the others, one launch per step of Alg. 1 for all of them, on the caller's
 *   stream; its rank-sized buffers come from one device arena that the call keeps for
 *   the next one (icur_release frees it), and its results are copied to the pools by a
 *   helper thread while the others go on.  Each matrix's arithmetic is its own (the
 *   result does not depend on the rest of the batch); its pivots are icur_run's
 *   wherever the selection is not decided by rounding, its core is A(I,J)^{-1} formed
 *   from the two block-triangular factors of A(I,J).  Its residual factors are FP64 in
 *   both forms (the precision form changes only its sketch there).
 *   Worker form (batch_workers 1..16), and matrices the grouped form does not take: the
 *   matrices run concurrently, batch_workers (16 for the rest of a grouped call) at a
 *   time, each on a worker stream with its own cached workspace, largest first; each
 *   gets exactly the result icur_run returns for it (same kernels, same arithmetic).
 * The caller's stream (opts->stream) is waited on before any matrix starts.
 *   count        >= 0 (0 returns ICUR_OK at once).
 *   A, m, n, lda host arrays of count entries: device pointer, rows, columns and leading
 *                dimension of each matrix (row-major, lda[i] >= n[i]).
 *   tol, seed    host arrays of count entries: tolerance and sketch seed per matrix.
 *   block, sketch_kind, opts: shared by all matrices as in icur_run (opts->stream is
 *                the caller's stream; opts->max_rank caps every matrix).
 *   cap_offsets  host, count + 1 nondecreasing entries, cap_offsets[0] = 0.  Matrix i
 *                owns I_pool / J_pool entries cap_offsets[i] .. cap_offsets[i+1]-1; this
 *                capacity must be at least min(m[i], n[i], max_rank).
 *   I_pool, J_pool  host int64 (device with opts->device_outputs), cap_offsets[count]
 *                entries each.
 *   U_pool       host doubles (device with opts->device_outputs), sum of cap_i^2
 *                entries: matrix i's core (rank_i x rank_i,
 *                leading dimension rank_i) starts at sum_{j<i} cap_j^2.
 *   rank, est_err, status  host arrays of count entries: per-matrix rank, final rho and
 *                return code of that matrix's run.
 * Every argument of every matrix is checked before any device work.  Returns ICUR_OK when
 * no matrix failed (warnings such as ICUR_MAXRANK are in status[]), else the error code of
 * the lowest-numbered failed matrix, with icur_last_error naming it.
 */
int icur_run_batched(int32_t count, const float* const* A, const int64_t* m, const int64_t* n,
                     const int64_t* lda, const double* tol, int32_t block, int32_t sketch_kind,
                     const uint64_t* seed, const icur_opts* opts, int64_t* I_pool, int64_t* J_pool,
                     double* U_pool, const int64_t* cap_offsets, int64_t* rank, double* est_err,
                     int32_t* status);

/* Statistics of the calling thread's most recent icur_run (copied into *info). */
int icur_last_info(icur_info* info);

/* Message describing the calling thread's most recent failure ("" if none). */
const char* icur_last_error(void);

/* Free the calling process's cached device workspaces and batched arenas (all devices). */
int icur_release(void);

/* ------------------------------------------------------------------------------------
 * Step entry points.  Each runs one step of Alg. 1 on caller-provided device buffers;
 * icur_run is built from the same kernels.
 * ---------------------------------------------------------------------------------- */

/*
 * icur_make_sketch: the recycled sketch operator G (c x m) of Alg. 1 ("Generate a sketch
 * matrix"; G is c x m, see §1.1).  Entry G[r][i] is defined from Philox4x32-10 with
 * counter (lo32(i), hi32(i), r, 0x47415553) and key (lo32(seed), hi32(seed)): Box-Muller
 * on the two 53-bit uniforms of the block, rounded FP64 -> FP32 -> BF16.  For the
 * sparse-sign kind, column i holds min(zeta, c) entries +-1 at distinct rows chosen by
 * Floyd's algorithm from counters (lo32(i), hi32(i), t, 0x53505253).
 *   G_bf16   device, c x m uint16 BF16 bit patterns (dense, zeros included), or NULL.
 *   rows     device, m x min(zeta,c) uint8 row indices (sparse-sign only), or NULL.
 *   signs    device, m uint8 sign bit masks, bit t set = entry t is -1 (sparse-sign
 *            only), or NULL.
 * c <= 255 for the sparse-sign kind.
 */
int icur_make_sketch(uint64_t seed, int64_t c, int64_t m, int32_t sketch_kind, int32_t zeta,
                     uint16_t* G_bf16, uint8_t* rows, uint8_t* signs, void* stream);

/*
 * icur_make_srtt: the SRTT sketch operator (ICUR_SKETCH_SRTT; §3.4): G = sqrt(m/c) R F D,
 * F the orthonormal DCT-II of length m, D = diag(d_i) with d_i = -1 when bit 0 of word 0
 * of Philox4x32-10 counter (lo32(i), hi32(i), 0, 0x53525444) is set, R the c distinct
 * rows drawn by Floyd's algorithm (draw t from counter (t, 0, 0, 0x53525452), value
 * (word1 * 2^32 + word0) mod (m - c + t + 1)), kept in increasing order; key (lo32(seed),
 * hi32(seed)).  G[k][i] = d_i sqrt(m/c) s_r cos(pi r (2i+1) / (2m)), r = rows[k], s_0 =
 * sqrt(1/m), s_r = sqrt(2/m), evaluated in FP64 and rounded to FP32.
 *   G     device, c x m FP32 (leading dimension m), or NULL (rows only).
 *   rows  device, c int64: the kept rows, increasing.
 * 1 <= c <= m.  Allocates m bytes of device scratch for the call.
 */
int icur_make_srtt(uint64_t seed, int64_t c, int64_t m, float* G, int64_t* rows, void* stream);

/*
 * icur_sketch: X0 = G A (Alg. 1, initial sketch S_0^col; §3.4 cost item 4) and
 * ||X0||_F^2 accumulated in FP64.
 *   G_bf16   device, c x m BF16 bit patterns (from icur_make_sketch).
 *   A        device, m x n, lda >= n.
 *   terms    0: FP32 matrix-core products (plain form); 1..3: A split into that many
 *            BF16 pieces on BF16 matrix cores (3 pieces reproduce every FP32 product).
 *   X0       device, c x n FP32 output, leading dimension n.
 *   normsq   host, may be NULL: ||X0||_F^2.
 */
int icur_sketch(const uint16_t* G_bf16, int64_t c, const float* A, int64_t m, int64_t n,
                int64_t lda, int32_t terms, float* X0, double* normsq, void* stream);

/*
 * icur_lupp: pivot order of LU with partial pivoting (§3.2.1 column selection, §3.2.2
 * row selection) applied to T = X^T, an N x K matrix whose rows are the candidates.
 *   X        device, K x N FP32, leading dimension ldx >= N: X[t*ldx + i] = T[i][t].
 *   steps    number of pivots wanted, 1 <= steps <= K.
 *   excluded device, N bytes (nonzero = candidate not eligible), or NULL.
 *   piv      device, capacity steps: chosen candidate indices in pivot order.
 *   npiv     host: number of pivots found (< steps when the candidates run out or the
 *            best remaining entry is exactly zero).
 * Arithmetic is FP64 with the textbook right-looking update (product rounded, then
 * subtracted); ties go to the lowest index.  K <= 4096, N <= 524288.
 */
int icur_lupp(const float* X, int64_t K, int64_t N, int64_t ldx, int32_t steps,
              const uint8_t* excluded, int64_t* piv, int32_t* npiv, void* stream);

/*
 * icur_qrcp: pivot order of QR with column pivoting (Alg. 1's alternative selection;
 * §5.3) applied to X, whose N columns are the candidates (the same candidates as
 * icur_lupp: T = X^T has one row per candidate).  Step t picks the candidate whose
 * component orthogonal to the ones already chosen has the largest 2-norm (ties to the
 * lowest index); FP64, residual vectors orthogonalised explicitly (no norm downdating).
 *   X, K, N, ldx, steps, excluded, piv, npiv: as icur_lupp (npiv < steps when every
 *   remaining candidate has an exactly zero residual).  K <= 4096, N < 2^31.
 */
int icur_qrcp(const float* X, int64_t K, int64_t N, int64_t ldx, int32_t steps,
              const uint8_t* excluded, int64_t* piv, int32_t* npiv, void* stream);

/*
 * icur_residual: OUT = X - W B (the column residual G A - (G C) U R of Alg. 1 with
 * W = (G C) U and B = R, and the row residual A(:,J_k)^T - (U A(I,J_k))^T C^T with
 * W = Y^T and B = C^T), plus ||OUT||_F^2 in FP64.
 *   X        device, M x N FP32, leading dimension ldx (may equal OUT for in place), or
 *            NULL for X = 0.
 *   W        device, M x K FP64, leading dimension ldw.
 *   B        device, K x N FP32, leading dimension ldb.
 *   terms    0: FP32 matrix-core products; 1..3: W and B split into that many BF16
 *            pieces, products of pieces (i, j) with i + j < terms.
 *   OUT      device, M x N FP32, leading dimension ldo.
 *   normsq   host, may be NULL.
 * M <= 4096; K may be 0 (OUT = X).
 */
int icur_residual(const float* X, int64_t ldx, const double* W, int64_t ldw, const float* B,
                  int64_t ldb, int64_t M, int64_t K, int64_t N, int32_t terms, float* OUT,
                  int64_t ldo, double* normsq, void* stream);

/*
 * icur_residual_f64: the residual-form products of the loop in FP64, routed exactly as
 * icur_run routes them (the recurrence of §4.2: the row residual S^row = A(:,J_k) -
 * Lc Ur(:,J_k), the residual at the new rows, Ur_k = N_k^{-1} S(I_k,:) and the column
 * residual S^col <- S^col - S^col(:,J_k) Ur_k).
 *   X        device, M x N FP64, leading dimension ldx: OUT = X - W B; X may equal OUT
 *            (in place).  NULL: OUT = W B.
 *   W        device, M x K FP64 (ldw); B device, K x N FP64 (ldb); OUT device, M x N
 *            FP64 (ldo).
 *   normsq   host, may be NULL: ||OUT||_F^2 (FP64 partial sums).
 * Products of at least 96 rows at depth >= 256 (>= 64 on rows of >= 16384 columns), in
 * place or plain, run on the library FP64 GEMM; all others on the short-M FP64
 * matrix-core kernel.  M <= 4096; K may be 0.
 */
int icur_residual_f64(const double* X, int64_t ldx, const double* W, int64_t ldw, const double* B,
                      int64_t ldb, int64_t M, int64_t K, int64_t N, double* OUT, int64_t ldo,
                      double* normsq, void* stream);

/*
 * icur_gather: the CUR factor gathers of Alg. 1 (C = A(:,J), R = A(I,:)).
 *   cols     device, k indices < n, or NULL: Ct[t][i] = A[i][cols[t]] (Ct is k x m,
 *            leading dimension ldct), i.e. C stored transposed.
 *   rows     device, k indices < m, or NULL: Rout[t][j] = A[rows[t]][j] (k x n,
 *            leading dimension ldr).
 * Exactly one of (cols, Ct) and (rows, Rout) is given.  Indices are not validated on
 * the device beyond being clamped into range; callers pass indices from icur_lupp.
 */
int icur_gather(const float* A, int64_t m, int64_t n, int64_t lda, const int64_t* cols,
                const int64_t* rows, int64_t k, float* Ct, int64_t ldct, float* Rout,
                int64_t ldr, void* stream);

/*
 * icur_core_update: the core U = A(I,J)^{-1} of Alg. 1 grown by one block through the
 * block inverse of the residual-recurrence lemma (§4.2): with Y = U A(I,J_k),
 * N = A(I_k,J_k) - A(I_k,J) Y and Z = A(I_k,J) U,
 *   U_new = [[U + Y N^-1 Z, -Y N^-1], [-N^-1 Z, N^-1]].
 * All FP64, device.
 *   U      r x r on entry (leading dimension ldu >= r + k), (r+k) x (r+k) on exit.
 *   Y      r x k,  A21 = A(I_k, J) k x r,  A22 = A(I_k, J_k) k x k (all row-major,
 *          leading dimensions = their column counts).
 *   rcond  host, may be NULL: 1 / (||N||_1 ||N^-1||_1) of the new block.
 * Returns ICUR_ERR_ARG when N is exactly singular.  k <= 512.
 */
int icur_core_update(double* U, int64_t ldu, int64_t r, int64_t k, const double* Y,
                     const double* A21, const double* A22, double* rcond, void* stream);

/* ------------------------------------------------------------------------------------
 * Entry point that allocates nothing.
 * ---------------------------------------------------------------------------------- */

/*
 * icur_lupp_noalloc: icur_lupp for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, arithmetic, kernels and results as icur_lupp; its workspace is a fixed
 * 48 MiB device array inside the library (one copy per device, held until the process
 * ends) instead of the allocated workspace cache, and the call makes no device or
 * pinned-host allocation.
 *   Limits: steps <= 256 and lupp_workspace(steps, N) <= 48 MiB, where the workspace is
 *   about 8 (steps + 16) N bytes plus 80 KB (b = 100 pivots over N = 40000 candidates
 *   takes 37.3 MB).  Larger requests return ICUR_ERR_ARG with a message.
 *   Concurrency: every call on one device uses that device's one array, so calls that
 *   overlap on one device (several host threads, or several streams) race and give
 *   wrong pivots; serialise them.  Nothing needs clearing between calls: each call
 *   rewrites every word it later reads.
 *   Set-up: icur_init_noalloc() looks up the array's device address on the current
 *   device (call it once per device, with that device current, before any capture);
 *   icur_lupp_noalloc does the same look-up itself on its first call on a device.
 */
int icur_init_noalloc(void);
int icur_lupp_noalloc(const float* X, int64_t K, int64_t N, int64_t ldx, int32_t steps,
                      const uint8_t* excluded, int64_t* piv, int32_t* npiv, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ICUR_H */
