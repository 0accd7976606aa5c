// Grouped kernels of the batched loop: every step of Alg. 1 for all unfinished matrices in
// one launch.  A plan kernel turns the matrices' current state (rank r, pivots found nJ,
// nI) into lists of products and gathers; persistent kernels walk those lists, so their
// launch configuration never depends on the data (the same launches every iteration).
//
// Products are OUT(M x N) = beta X + alpha W(M x K) B(K x N) in FP64 on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64): tiles of 16 TR rows x 128 WN columns (shape chosen per
// stage, 32 x 128 by default), the depth K per tile in 16-deep chunks that start at fixed
// multiples (W staged through LDS, B straight to registers), so the result of every
// element is a fixed-order FP64 sum that depends neither on the grouping nor on the tile
// shape.  Products with a block-triangular operand skip the depth range where that
// operand is zero.
//
// The core A(I,J)^{-1} is carried as two block-triangular inverses (A(I,J) = P Q with
// P = Lc(I,:), Q = Ur(:,J); see BatchMat): each iteration appends one block row to
// (Q^{-1})^T and to P^{-1}, reading only their nonzero halves, and one product after the
// loop forms Q^{-1} P^{-1}.
#include <algorithm>
#include <climits>
#include <cstring>
#include <vector>

#include "icur_batched.h"
#include "icur_gj.h"

namespace icur {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int kPT = 256;           // threads of the product and gather kernels
constexpr int kGatherCols = 256;   // gather tile: one row x 256 columns
constexpr int kGatherTrCols = 64;  // column-gather tile: every row (<= 64) x 64 columns
constexpr int kKC = kGemmKChunk;   // product depth chunk

struct GemmOp {
  const double* X;  // may be null (beta = 0)
  int64_t ldx;
  const double* W;
  int64_t ldw;
  const double* B;
  int64_t ldb;
  double* OUT;
  int64_t ldo;
  int M, K, N, tiles_n;
  double alpha;
  double* normp;    // per-tile sums of OUT^2 (indexed by the op's local tile), or null
  int tile0, pad;   // pad: the op's tile count while the plan is built
  int wt;           // W stored transposed: W(row, k) at W[k * ldw + row]
  int kskip;        // bit 0: W(row, k) = 0 for k < row - kband; bit 1: B(k, col) = 0 for
                    // k < col - kband (block-triangular operands, blocks of <= kband + 1)
  int kband, pad2;
};

struct GatherOp {
  const void* src;  // FP32 when f32, else FP64; null: the identity (times scale)
  int64_t rs, cs;   // src element strides per row index / column index
  const int64_t* ridx;
  const int64_t* cidx;
  double* dst;
  int64_t ldd;
  int rows, cols, tiles_c, f32;
  double scale;
  int tile0, pad;
  int tr, pad2;     // tr: column gather on the transposed tile (see gather_kernel)   // pad: the op's tile count while the plan is built
};

// Stage lists of one iteration.  Phase 0 (after the column selection): gathers GA and
// the row-residual product P1.  Phase 1 (after the row selection): gathers GB, products
// P2, P3, P4 (residual form and the two inverses' new block rows), copies GC (their
// diagonal blocks).  Phase 2, once after the loop: the core products FIN.
enum Stage { kGA, kP1, kGB, kP2, kP3, kP4, kGC, kFin, kNumStages };
constexpr int kOpsPerMat = 4;
// Tile shapes of the grouped product (selected per stage by the host).  Workgroup tiles
// (wave = 0): rows 16 TR, columns 128 WN, four waves of 32 WN columns sharing W through
// LDS.  Wave tiles (wave = 1): rows 16 TR, columns 32 WN, each wave on its own tile with
// W and B straight to registers (no LDS, no barrier).
// pd: chunks in flight ahead of the one being multiplied (workgroup tiles).
struct TileShape {
  int tr, wn, wave, pd;
};
constexpr TileShape kShapes[kGemmShapes] = {{1, 1, 0, 1}, {2, 1, 0, 1}, {3, 1, 0, 1}, {4, 1, 0, 1},
                                            {2, 2, 0, 1}, {4, 2, 0, 1}, {2, 1, 1, 1}, {1, 2, 1, 1},
                                            {2, 2, 1, 1}, {2, 1, 0, 2}, {4, 1, 0, 2}, {2, 1, 0, 3}};

struct Plan {
  GemmOp* gemm[kNumStages];
  GatherOp* gather[kNumStages];
  int* nops;      // per stage
  int* ntiles;    // per stage, followed by the per-stage tile counters of gemm_kernel
  double* bytes;  // per stage: algorithmic bytes of the products so far (the call's total)
  int rt[kNumStages], ct[kNumStages];  // product tile rows / columns of each stage
};

__device__ __forceinline__ int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Ops occupy fixed slots (matrix i, slot k -> entry i * kOpsPerMat + k); an unused slot has
// no tiles.  tile0 is filled in afterwards by a scan over the entries.
__device__ __forceinline__ double tri_sum(int64_t j) { return j > 0 ? 0.5 * static_cast<double>(j) * (j + 1) : 0.0; }

__device__ __forceinline__ void set_gemm(const Plan& pl, int stage, int i, int k, const double* X, int64_t ldx,
                                         const double* W, int64_t ldw, const double* B, int64_t ldb, double* OUT,
                                         int64_t ldo, int M, int K, int N, double alpha, double* normp,
                                         bool count_bytes = true, int kskip = 0, int kband = 0, int wt = 0) {
  GemmOp& o = pl.gemm[stage][i * kOpsPerMat + k];
  double* bytes = count_bytes ? pl.bytes + stage : nullptr;
  const int rt = pl.rt[stage], ct = pl.ct[stage];
  // algorithmic bytes: the nonzero parts of W and B read once, OUT written once, X read
  // once when given
  if (bytes && M > 0 && N > 0) {
    const double wnz = static_cast<double>(M) * K - ((kskip & 1) ? tri_sum(M - 1 - kband) : 0.0);
    const double bnz = static_cast<double>(K) * N - ((kskip & 2) ? tri_sum(N - 1 - kband) : 0.0);
    atomicAdd(bytes, 8.0 * (wnz + bnz + static_cast<double>(M) * N * (X ? 2.0 : 1.0)));
  }
  o.X = X;
  o.ldx = ldx;
  o.W = W;
  o.ldw = ldw;
  o.B = B;
  o.ldb = ldb;
  o.OUT = OUT;
  o.ldo = ldo;
  o.M = M;
  o.K = K;
  o.N = N;
  o.tiles_n = (M > 0 && N > 0) ? ceil_div(N, ct) : 0;
  o.alpha = alpha;
  o.normp = normp;
  o.pad = (M > 0 && N > 0) ? ceil_div(M, rt) * o.tiles_n : 0;  // tiles (until the scan)
  o.wt = wt;
  o.kskip = kskip;
  o.kband = kband;
}

__device__ __forceinline__ void no_gemm(const Plan& pl, int stage, int i, int k) {
  set_gemm(pl, stage, i, k, nullptr, 0, nullptr, 0, nullptr, 0, nullptr, 0, 0, 0, 0, 0.0, nullptr, false);
}

__device__ __forceinline__ void set_gather(GatherOp* ops, int i, int k, const void* src, bool f32, int64_t rs,
                                           int64_t cs, const int64_t* ridx, const int64_t* cidx, double* dst,
                                           int64_t ldd, int rows, int cols, double scale) {
  GatherOp& o = ops[i * kOpsPerMat + k];
  o.src = src;
  o.f32 = f32 ? 1 : 0;
  o.rs = rs;
  o.cs = cs;
  o.ridx = ridx;
  o.cidx = cidx;
  o.dst = dst;
  o.ldd = ldd;
  o.rows = rows;
  o.cols = cols;
  // dst row t = column ridx[t] of a row-major source: taken on tiles of every row x
  // kGatherTrCols columns, which read along the source's rows
  o.tr = (src && rs == 1 && ridx && !cidx && cs > 1 && rows <= 64) ? 1 : 0;
  o.tiles_c = (rows > 0 && cols > 0) ? ceil_div(cols, o.tr ? kGatherTrCols : kGatherCols) : 0;
  o.scale = scale;
  o.pad = rows > 0 ? (o.tr ? o.tiles_c : rows * o.tiles_c) : 0;
}

__device__ __forceinline__ void no_gather(GatherOp* ops, int i, int k) {
  set_gather(ops, i, k, nullptr, false, 0, 0, nullptr, nullptr, nullptr, 0, 0, 0, 0.0);
}

// Exclusive scan of the per-slot tile counts (held in .pad) into .tile0, and the total.
template <typename OP>
__device__ void scan_tiles(OP* ops, int n, int* total, int* nops, int* warp_sums) {
  const int tid = threadIdx.x, nt = blockDim.x;
  int carry = 0;
  for (int base = 0; base < n; base += nt) {
    const int e = base + tid;
    const int v = e < n ? ops[e].pad : 0;
    // inclusive scan within the workgroup: waves by shuffles, then the wave totals
    int x = v;
    const int lane = tid & 63, w = tid >> 6;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    __syncthreads();
    if (lane == 63) warp_sums[w] = x;
    __syncthreads();
    int before = 0;
    for (int q = 0; q < w; ++q) before += warp_sums[q];
    int chunk_total = 0;
    for (int q = 0; q < nt / 64; ++q) chunk_total += warp_sums[q];
    if (e < n) ops[e].tile0 = carry + before + x - v;
    carry += chunk_total;
  }
  if (tid == 0) {
    *total = carry;
    *nops = n;
    total[kNumStages] = 0;  // the stage's tile counter (see gemm_kernel)
  }
}

// The lists of a phase, from every matrix's state.  Phase 0 (after the column selection):
// GA, P1.  Phase 1 (after the row selection): GB, P2, P3, P4, GC.  Phase 2 (after the
// loop): FIN.
__global__ __launch_bounds__(1024) void plan_kernel(BatchMat* __restrict__ mats, int count, int c, int b, int phase,
                                                    Plan plan) {
  __shared__ int warp_sums[16];
  const int band = b - 1;
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    BatchMat& bm = mats[i];
    const bool on = bm.s != 0;
    const int r = bm.r, m = bm.m, n = bm.n, cap = bm.cap;
    if (phase == 0) {
      const int nJ = on ? bm.nJ : 0;
      double* Lk = bm.LcT + static_cast<int64_t>(r) * m;
      // GA: A(:, J_k)^T -> the next rows of LcT; Ur(:, J_k)^T -> Wa
      set_gather(plan.gather[kGA], i, 0, bm.A, true, 1, bm.lda, bm.Jk, nullptr, Lk, m, nJ, m, 1.0);
      set_gather(plan.gather[kGA], i, 1, bm.Ur, false, 1, n, bm.Jk, nullptr, bm.Wa, cap, nJ, r, 1.0);
      for (int k = 2; k < kOpsPerMat; ++k) no_gather(plan.gather[kGA], i, k);
      // P1: row residual S^row = A(:, J_k) - Lc Ur(:, J_k), stored transposed
      set_gemm(plan, kP1, i, 0, Lk, m, bm.Wa, cap, bm.LcT, m, Lk, m, r > 0 ? nJ : 0, r, m, -1.0, nullptr);
      for (int k = 1; k < kOpsPerMat; ++k) no_gemm(plan, kP1, i, k);
    } else if (phase == 1) {
      const int nI = on ? bm.nI : 0;
      const int nR = nI > 0 ? r : 0;   // products with the old blocks, from the second block on
      const int mR = nR > 0 ? nI : 0;  // their row count
      const double* Lk = bm.LcT + static_cast<int64_t>(r) * m;
      double* Urk = bm.Ur + static_cast<int64_t>(r) * n;
      double* QTk = bm.QT + static_cast<int64_t>(r) * cap;  // new block rows of (Q^{-1})^T, P^{-1}
      double* Pik = bm.Pi + static_cast<int64_t>(r) * cap;
      // GB: N_k = S(I_k, J_k); A(I_k, :); Lc(I_k, :); S(:, J_k)
      set_gather(plan.gather[kGB], i, 0, Lk, false, 1, m, bm.Ik, nullptr, bm.Nk, nI, nI, nI, 1.0);
      set_gather(plan.gather[kGB], i, 1, bm.A, true, bm.lda, 1, bm.Ik, nullptr, bm.Sr, n, nI, n, 1.0);
      set_gather(plan.gather[kGB], i, 2, bm.LcT, false, 1, m, bm.Ik, nullptr, bm.Wl, cap, nI, nR, 1.0);
      set_gather(plan.gather[kGB], i, 3, bm.S, false, n, 1, nullptr, bm.Jk, bm.Wc, nI, nI > 0 ? c : 0, nI, 1.0);
      // P2: residual at the new rows Sr -= Lc(I_k,:) Ur; the new block row of (Q^{-1})^T,
      // -Ur(:, J_k)^T (Q^{-1})^T (bordering Q with the block column Ur(:, J_k)); and
      // Wp = N_k^{-1} Lc(I_k, :)
      set_gemm(plan, kP2, i, 0, bm.Sr, n, bm.Wl, cap, bm.Ur, n, bm.Sr, n, mR, r, n, -1.0, nullptr);
      set_gemm(plan, kP2, i, 1, nullptr, 0, bm.Wa, cap, bm.QT, cap, QTk, cap, mR, r, r, -1.0, nullptr,
               true, 2, band);
      set_gemm(plan, kP2, i, 2, nullptr, 0, bm.Nk, nI, bm.Wl, cap, bm.Wp, cap, mR, nI, r, 1.0, nullptr);
      no_gemm(plan, kP2, i, 3);
      // P3: new row factors Ur_k = N_k^{-1} Sr; the new block row of P^{-1}, -Wp P^{-1}
      // (bordering P with the block row Lc(I_k, :) and the diagonal block N_k)
      set_gemm(plan, kP3, i, 0, nullptr, 0, bm.Nk, nI, bm.Sr, n, Urk, n, nI, nI, n, 1.0, nullptr);
      set_gemm(plan, kP3, i, 1, nullptr, 0, bm.Wp, cap, bm.Pi, cap, Pik, cap, mR, r, r, -1.0, nullptr,
               true, 2, band);
      for (int k = 2; k < kOpsPerMat; ++k) no_gemm(plan, kP3, i, k);
      // P4: column residual S -= S(:, J_k) Ur_k, with its norm partials
      set_gemm(plan, kP4, i, 0, bm.S, n, bm.Wc, nI, Urk, n, bm.S, n, nI > 0 ? c : 0, nI, n, -1.0, bm.normp);
      for (int k = 1; k < kOpsPerMat; ++k) no_gemm(plan, kP4, i, k);
      bm.nparts = plan.gemm[kP4][i * kOpsPerMat].pad;
      // GC: the diagonal blocks (identity in (Q^{-1})^T, N_k^{-1} in P^{-1}) and zeros to
      // their right
      const int wq = nI > 0 ? min(cap - r, nI + kBandCols) : 0;
      const int wp = nI > 0 ? min(cap - r - nI, kBandCols) : 0;
      set_gather(plan.gather[kGC], i, 0, nullptr, false, 0, 0, nullptr, nullptr, QTk + r, cap, nI, wq, 1.0);
      set_gather(plan.gather[kGC], i, 1, bm.Nk, false, nI, 1, nullptr, nullptr, Pik + r, cap, nI, nI, 1.0);
      set_gather(plan.gather[kGC], i, 2, nullptr, false, 0, 0, nullptr, nullptr, Pik + r + nI, cap, wp > 0 ? nI : 0,
                 wp, 0.0);
      no_gather(plan.gather[kGC], i, 3);
    } else {
      // FIN, for the matrices that stopped in this iteration: A(I,J)^{-1} = Q^{-1} P^{-1}
      // into LcT (leading dimension r), depth skipped on both triangular factors
      const bool due = bm.s == 0 && bm.fin == 0;
      const int rf = (due && bm.info == 0 && bm.cap > 0) ? r : 0;
      if (due) bm.fin = 1;
      set_gemm(plan, kFin, i, 0, nullptr, 0, bm.QT, cap, bm.Pi, cap, bm.LcT, rf, rf, rf, rf, 1.0, nullptr,
               true, 3, band, 1);
      for (int k = 1; k < kOpsPerMat; ++k) no_gemm(plan, kFin, i, k);
    }
  }
  __syncthreads();
  const int n = count * kOpsPerMat;
  if (phase == 0) {
    scan_tiles(plan.gather[kGA], n, plan.ntiles + kGA, plan.nops + kGA, warp_sums);
    scan_tiles(plan.gemm[kP1], n, plan.ntiles + kP1, plan.nops + kP1, warp_sums);
  } else if (phase == 1) {
    scan_tiles(plan.gather[kGB], n, plan.ntiles + kGB, plan.nops + kGB, warp_sums);
    scan_tiles(plan.gemm[kP2], n, plan.ntiles + kP2, plan.nops + kP2, warp_sums);
    scan_tiles(plan.gemm[kP3], n, plan.ntiles + kP3, plan.nops + kP3, warp_sums);
    scan_tiles(plan.gemm[kP4], n, plan.ntiles + kP4, plan.nops + kP4, warp_sums);
    scan_tiles(plan.gather[kGC], n, plan.ntiles + kGC, plan.nops + kGC, warp_sums);
  } else {
    scan_tiles(plan.gemm[kFin], n, plan.ntiles + kFin, plan.nops + kFin, warp_sums);
  }
}

template <typename OP>
__device__ __forceinline__ int find_op(const OP* ops, int nops, int tile) {
  int lo = 0, hi = nops - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ops[mid].tile0 <= tile) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// The loads of one column-gather tile (see gather_kernel): v[q] = src[(j0 + w + 4 q) cs + ct],
// all issued before any is used.  Source rows past the tile are clamped to its last one,
// so every load is in bounds and none sits under a branch; those values are never
// written out.
template <int Q, typename T>
__device__ __forceinline__ void gather_tr_loads(const T* __restrict__ src, int64_t cs, int64_t ct, int j0, int nj,
                                                int w, double (&v)[Q]) {
  T x[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int jl = min(w + (kPT / 64) * q, nj - 1);
    x[q] = src[static_cast<int64_t>(j0 + jl) * cs + ct];
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) v[q] = static_cast<double>(x[q]);
}

// dst[i][j] = scale * src[ridx[i] rs + cidx[j] cs] (identity where an index list is null);
// with no src, dst[i][j] = scale * (i == j).
// Column gathers (tr: rs = 1, row indices, no column indices, at most 64 rows) run on
// tiles of every row x kGatherTrCols columns: wave w reads source rows j0 + w + 4 q, lane t
// the entry of column ridx[t], so a wave's loads stay in one source row; the tile is
// turned in LDS and written one destination row (64 contiguous entries) per wave step.
// The one-row tiles read a column of the source per wave, one source row per lane.
__global__ __launch_bounds__(kPT) void gather_kernel(const GatherOp* __restrict__ ops, const int* __restrict__ pnops,
                                                     const int* __restrict__ pntiles) {
  constexpr int kQ = kGatherTrCols / (kPT / 64);  // source rows per wave and tile
  __shared__ double tb[64][kGatherTrCols + 1];
  const int nops = *pnops, ntiles = *pntiles;
  for (int g = blockIdx.x; g < ntiles; g += gridDim.x) {
    const GatherOp& o = ops[find_op(ops, nops, g)];
    const int lt = g - o.tile0;
    if (o.tr) {
      const int j0 = lt * kGatherTrCols;
      const int nj = min(kGatherTrCols, o.cols - j0);
      const int t = threadIdx.x & 63, w = threadIdx.x >> 6;
      // lanes past the last row read row 0's column (in bounds; never written out)
      const int64_t ct = o.ridx[t < o.rows ? t : 0];
      double v[kQ];
      if (o.f32)
        gather_tr_loads<kQ>(static_cast<const float*>(o.src), o.cs, ct, j0, nj, w, v);
      else
        gather_tr_loads<kQ>(static_cast<const double*>(o.src), o.cs, ct, j0, nj, w, v);
      __syncthreads();  // the previous tile's reads of tb are done
#pragma unroll
      for (int q = 0; q < kQ; ++q) tb[t][w + (kPT / 64) * q] = v[q];
      __syncthreads();
      const int jl = threadIdx.x & 63;
      if (jl < nj)
        for (int tt = w; tt < o.rows; tt += kPT / 64)
          o.dst[static_cast<int64_t>(tt) * o.ldd + j0 + jl] = o.scale * tb[tt][jl];
      continue;
    }
    const int i = lt / o.tiles_c;
    const int j = (lt % o.tiles_c) * kGatherCols + threadIdx.x;
    double* d = o.dst + static_cast<int64_t>(i) * o.ldd;
    if (!o.src) {
      for (int jj = j; jj < min(o.cols, j + kGatherCols); jj += kPT) d[jj] = jj == i ? o.scale : 0.0;
      continue;
    }
    const int64_t ri = o.ridx ? o.ridx[i] : i;
    for (int jj = j; jj < min(o.cols, j + kGatherCols); jj += kPT) {
      const int64_t cj = o.cidx ? o.cidx[jj] : jj;
      const int64_t e = ri * o.rs + cj * o.cs;
      const double v = o.f32 ? static_cast<double>(static_cast<const float*>(o.src)[e])
                             : static_cast<const double*>(o.src)[e];
      d[jj] = o.scale * v;
    }
  }
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kPT / 64; ++w) s += red[w];
  return s;
}

// FP64 products on workgroup tiles of 16 TR rows x 128 WN columns.  Lane (lr, lg) of wave
// w, MFMA step j of a chunk starting at k0: A operand W[row lr][k0 + 4 lg + j] (from LDS),
// B operand B[k0 + 4 lg + j][column], accumulator slot v = row 4 v + lg (every shape and
// both tile kinds use this k order, so the sums are the same).  The wave owns 32 WN
// columns of the tile in pairs: 16-column sub-tile s holds the columns n0 + 32 (s / 2) +
// 2 lr + s % 2, so a lane reads the two columns of a pair of B (and of X and OUT) with one
// 16-byte access.  The depth runs in chunks of kKC: W of the next chunk and B of the next
// chunk are loaded into registers while the current one is multiplied, W through two LDS
// buffers (one barrier per chunk).  gemm_wg_tile is one tile; gemm_kernel walks a list of
// ops (persistent), gemm_one_kernel the tiles of one op.
template <int TR, int WN, int PD = 1>
__device__ __forceinline__ void gemm_wg_tile(const GemmOp& o, int lt, double (*wl)[kKC * (16 * TR + 2)],
                                             double* red) {
  constexpr int RT = 16 * TR;          // tile rows
  constexpr int CT = 128 * WN;         // tile columns
  constexpr int S = 2 * WN;            // 16-column sub-tiles per wave
  constexpr int kStride = RT + 2;      // LDS row stride of the transposed W chunk
  constexpr int WPT = RT * kKC / kPT;  // W entries per thread per chunk
  static_assert(WPT * kPT == RT * kKC, "W chunk must split evenly over the threads");
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int M = o.M, K = o.K, N = o.N;
  const int m0 = (lt / o.tiles_n) * RT;
  const int n0t = (lt % o.tiles_n) * CT;
  const int n0 = n0t + wave * 32 * WN;
  const double* __restrict__ W = o.W;
  const double* __restrict__ B = o.B;
  const int64_t ldw = o.ldw, ldb = o.ldb;
  const bool wt = o.wt != 0;
  // 16-byte accesses where the pair is aligned: even leading dimension, aligned base
  const bool bvec = ((ldb & 1) == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
  int col[S];
#pragma unroll
  for (int s2 = 0; s2 < S; ++s2) col[s2] = n0 + 32 * (s2 >> 1) + 2 * lr + (s2 & 1);
  // depth range: block-triangular operands are zero below kbeg for the whole tile; it
  // starts at a chunk boundary so the grouping of the sums does not depend on the tile
  int kbeg = 0;
  if (o.kskip & 1) kbeg = max(kbeg, m0 - o.kband);
  if (o.kskip & 2) kbeg = max(kbeg, n0t - o.kband);
  kbeg = (kbeg / kKC) * kKC;
  const int nch = kbeg < K ? (K - kbeg + kKC - 1) / kKC : 0;

  doublex4 acc[TR][S];
#pragma unroll
  for (int t = 0; t < TR; ++t)
#pragma unroll
    for (int s2 = 0; s2 < S; ++s2) acc[t][s2] = doublex4{0.0, 0.0, 0.0, 0.0};
  constexpr int NJ = kKC / 4;  // MFMA steps per chunk
  constexpr int NS = PD + 1;   // register slots: the chunk being multiplied and PD in flight
  double b[NS][NJ][S];
  double wr[NS][WPT];
  auto load_b = [&](double (&bb)[NJ][S], int k0) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int k = k0 + 4 * lg + j;
      const bool kok = k < K;
      const double* row = B + static_cast<int64_t>(kok ? k : 0) * ldb;
#pragma unroll
      for (int p = 0; p < WN; ++p) {
        const int c0 = col[2 * p];
        if (bvec && kok && c0 + 1 < N) {
          const double2 v = *reinterpret_cast<const double2*>(row + c0);
          bb[j][2 * p] = v.x;
          bb[j][2 * p + 1] = v.y;
        } else {
          bb[j][2 * p] = (kok && c0 < N) ? row[c0] : 0.0;
          bb[j][2 * p + 1] = (kok && c0 + 1 < N) ? row[c0 + 1] : 0.0;
        }
      }
    }
  };
  auto load_w = [&](double (&ww)[WPT], int k0) {
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      const int e = tid + kPT * q;
      int row, kk;
      if (wt) {
        kk = e / RT;
        row = e % RT;
      } else {
        row = e / kKC;
        kk = e % kKC;
      }
      const int gr = m0 + row, gk = k0 + kk;
      const bool ok = gr < M && gk < K;
      ww[q] = ok ? (wt ? W[static_cast<int64_t>(gk) * ldw + gr] : W[static_cast<int64_t>(gr) * ldw + gk]) : 0.0;
    }
  };
  auto store_w = [&](const double (&ww)[WPT], int buf) {
#pragma unroll
    for (int q = 0; q < WPT; ++q) {
      const int e = tid + kPT * q;
      const int row = wt ? e % RT : e / kKC;
      const int kk = wt ? e / RT : e % kKC;
      wl[buf][kk * kStride + row] = ww[q];
    }
  };
  auto multiply = [&](const double (&bb)[NJ][S], int buf) {
#pragma unroll
    for (int t = 0; t < TR; ++t) {
      double a[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) a[j] = wl[buf][(4 * lg + j) * kStride + t * 16 + lr];
#pragma unroll
      for (int s2 = 0; s2 < S; ++s2)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[t][s2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j], bb[j][s2], acc[t][s2], 0, 0, 0);
    }
  };
  // prologue: chunks 0 .. PD-1 into register slots 0 .. PD-1, chunk 0's W into LDS
  gj_static_for<PD>([&](auto q_) __attribute__((always_inline)) {
    constexpr int q = decltype(q_)::value;
    if (q < nch) {
      load_w(wr[q], kbeg + q * kKC);
      load_b(b[q], kbeg + q * kKC);
    }
  });
  __syncthreads();  // the previous tile's readers of the LDS buffers are done
  if (nch > 0) store_w(wr[0], 0);
  __syncthreads();
  // chunk ch sits in slot ch % NS; the loop is unrolled by NS so every slot index is static
  for (int base = 0; base < nch; base += NS) {
    gj_static_for<NS>([&](auto s_) __attribute__((always_inline)) {
      constexpr int sl = decltype(s_)::value;
      const int ch = base + sl;
      if (ch >= nch) return;  // uniform over the workgroup
      constexpr int ahead = (sl + PD) % NS;
      constexpr int next = (sl + 1) % NS;
      if (ch + PD < nch) {
        load_w(wr[ahead], kbeg + (ch + PD) * kKC);
        load_b(b[ahead], kbeg + (ch + PD) * kKC);
      }
      multiply(b[sl], ch & 1);
      if (ch + 1 < nch) store_w(wr[next], (ch + 1) & 1);
      __syncthreads();
    });
  }
  // epilogue: OUT = X + alpha acc, pairs of columns per lane
  const bool ovec = ((o.ldo & 1) == 0) && ((reinterpret_cast<uintptr_t>(o.OUT) & 15) == 0) &&
                    (!o.X || (((o.ldx & 1) == 0) && ((reinterpret_cast<uintptr_t>(o.X) & 15) == 0)));
  double sq = 0.0;
#pragma unroll
  for (int t = 0; t < TR; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = m0 + t * 16 + 4 * v + lg;
      if (row >= M) continue;
      double* orow = o.OUT + static_cast<int64_t>(row) * o.ldo;
      const double* xrow = o.X ? o.X + static_cast<int64_t>(row) * o.ldx : nullptr;
#pragma unroll
      for (int p = 0; p < WN; ++p) {
        const int c0 = col[2 * p];
        double y0 = o.alpha * acc[t][2 * p][v];
        double y1 = o.alpha * acc[t][2 * p + 1][v];
        if (ovec && c0 + 1 < N) {
          if (xrow) {
            const double2 x = *reinterpret_cast<const double2*>(xrow + c0);
            y0 = x.x + y0;
            y1 = x.y + y1;
          }
          *reinterpret_cast<double2*>(orow + c0) = double2{y0, y1};
          sq += y0 * y0 + y1 * y1;
        } else {
          if (c0 < N) {
            if (xrow) y0 = xrow[c0] + y0;
            orow[c0] = y0;
            sq += y0 * y0;
          }
          if (c0 + 1 < N) {
            if (xrow) y1 = xrow[c0 + 1] + y1;
            orow[c0 + 1] = y1;
            sq += y1 * y1;
          }
        }
      }
    }
  if (o.normp) {
    const double tot = block_sum(sq, red);
    if (tid == 0) o.normp[lt] = tot;
  }
}

// ROLE only names the instance (0: the loop's products, 1: the closing core products), so
// that a kernel trace tells the two apart.
// Tiles are taken from a device counter (next to the stage's tile count, cleared by the
// plan kernel), one at a time: a workgroup that drew shallow tiles takes more of them, so
// the tiles' uneven depths (each matrix's rank) do not leave a tail of a few workgroups
// with several deep tiles.  No lane-divergent branch may sit in this loop: with the draw
// under `threadIdx.x == 0` and the exit on a plain LDS read, the compiler structured the
// loop so that the drawing lane left it while the rest of its wave went on through the
// barriers, which then never saw a new index.  So the draw is taken by the whole first
// wave under a wave-uniform branch (lane 0 adds 1, the others 0, and every lane keeps lane
// 0's old value), and the exit compares a readfirstlane value.
template <int TR, int WN, int ROLE = 0, int PD = 1>
__global__ __launch_bounds__(kPT) void gemm_kernel(const GemmOp* __restrict__ ops, const int* __restrict__ pnops,
                                                   int* __restrict__ pntiles) {
  __shared__ double wl[2][kKC * (16 * TR + 2)];
  __shared__ double red[kPT / 64];
  __shared__ int g_sh;
  const int nops = *pnops, ntiles = *pntiles;
  int* next = pntiles + kNumStages;
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
  for (;;) {
    if (wave == 0) g_sh = __builtin_amdgcn_readfirstlane(atomicAdd(next, threadIdx.x == 0 ? 1 : 0));
    __syncthreads();
    const int g = __builtin_amdgcn_readfirstlane(g_sh);
    __syncthreads();  // every wave has read g_sh before the next draw overwrites it
    if (g >= ntiles) break;
    const GemmOp& o = ops[find_op(ops, nops, g)];
    gemm_wg_tile<TR, WN, PD>(o, g - o.tile0, wl, red);
  }
}

// One product OUT = X + alpha W B (the op passed by value; tiles_n set by the caller),
// persistent over its tiles.
template <int TR, int WN>
__global__ __launch_bounds__(kPT) void gemm_one_kernel(const GemmOp o) {
  __shared__ double wl[2][kKC * (16 * TR + 2)];
  __shared__ double red[kPT / 64];
  const int ntiles = ((o.M + 16 * TR - 1) / (16 * TR)) * o.tiles_n;
  for (int g = blockIdx.x; g < ntiles; g += gridDim.x) gemm_wg_tile<TR, WN>(o, g, wl, red);
}

// Persistent FP64 product over a list of ops, one tile of 16 TR rows x 32 WN columns per
// wave: each wave walks its own tiles with W and B loaded straight into registers (the
// next chunk's while the current one is multiplied), no LDS and no barrier.  Lane (lr, lg)
// and the k order as in gemm_kernel; its four W entries of a step are contiguous in a row
// of W (one 32-byte read).  Ops with norm partials are not taken (gemm_kernel does those).
template <int TR, int WN, int ROLE = 0>
__global__ __launch_bounds__(kPT) void gemm_wave_kernel(const GemmOp* __restrict__ ops, const int* __restrict__ pnops,
                                                        const int* __restrict__ pntiles) {
  constexpr int RT = 16 * TR;
  constexpr int CT = 32 * WN;
  constexpr int S = 2 * WN;
  constexpr int NJ = kKC / 4;
  static_assert(NJ == 4, "W reads assume four steps per chunk");
  const int nops = *pnops, ntiles = *pntiles;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int nwaves = gridDim.x * (kPT / 64);
  for (int g = blockIdx.x * (kPT / 64) + wave; g < ntiles; g += nwaves) {
    const GemmOp& o = ops[find_op(ops, nops, g)];
    const int lt = g - o.tile0;
    const int M = o.M, K = o.K, N = o.N;
    const int m0 = (lt / o.tiles_n) * RT;
    const int n0 = (lt % o.tiles_n) * CT;
    const double* __restrict__ W = o.W;
    const double* __restrict__ B = o.B;
    const int64_t ldw = o.ldw, ldb = o.ldb;
    const bool wt = o.wt != 0;
    const bool bvec = ((ldb & 1) == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
    const bool wvec = !wt && ((ldw & 1) == 0) && ((reinterpret_cast<uintptr_t>(W) & 15) == 0);
    int col[S];
#pragma unroll
    for (int s2 = 0; s2 < S; ++s2) col[s2] = n0 + 32 * (s2 >> 1) + 2 * lr + (s2 & 1);
    int kbeg = 0;
    if (o.kskip & 1) kbeg = max(kbeg, m0 - o.kband);
    if (o.kskip & 2) kbeg = max(kbeg, n0 - o.kband);
    kbeg = (kbeg / kKC) * kKC;
    const int nch = kbeg < K ? (K - kbeg + kKC - 1) / kKC : 0;
    doublex4 acc[TR][S];
#pragma unroll
    for (int t = 0; t < TR; ++t)
#pragma unroll
      for (int s2 = 0; s2 < S; ++s2) acc[t][s2] = doublex4{0.0, 0.0, 0.0, 0.0};
    double b[NJ][S], w[TR][NJ];
    auto load = [&](int k0) {
      const int kl = k0 + 4 * lg;  // this lane's four k: kl .. kl + 3
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int k = kl + j;
        const bool kok = k < K;
        const double* row = B + static_cast<int64_t>(kok ? k : 0) * ldb;
#pragma unroll
        for (int p = 0; p < WN; ++p) {
          const int c0 = col[2 * p];
          if (bvec && kok && c0 + 1 < N) {
            const double2 v = *reinterpret_cast<const double2*>(row + c0);
            b[j][2 * p] = v.x;
            b[j][2 * p + 1] = v.y;
          } else {
            b[j][2 * p] = (kok && c0 < N) ? row[c0] : 0.0;
            b[j][2 * p + 1] = (kok && c0 + 1 < N) ? row[c0 + 1] : 0.0;
          }
        }
      }
#pragma unroll
      for (int t = 0; t < TR; ++t) {
        const int r = m0 + 16 * t + lr;
        const bool rok = r < M;
        if (wt) {
#pragma unroll
          for (int j = 0; j < NJ; ++j) w[t][j] = (rok && kl + j < K) ? W[static_cast<int64_t>(kl + j) * ldw + r] : 0.0;
        } else if (wvec && rok && kl + 3 < K) {
          const double* wr = W + static_cast<int64_t>(r) * ldw + kl;
          const double2 v0 = *reinterpret_cast<const double2*>(wr);
          const double2 v1 = *reinterpret_cast<const double2*>(wr + 2);
          w[t][0] = v0.x;
          w[t][1] = v0.y;
          w[t][2] = v1.x;
          w[t][3] = v1.y;
        } else {
          const double* wr = W + static_cast<int64_t>(rok ? r : 0) * ldw;
#pragma unroll
          for (int j = 0; j < NJ; ++j) w[t][j] = (rok && kl + j < K) ? wr[kl + j] : 0.0;
        }
      }
    };
    if (nch > 0) load(kbeg);
    for (int ch = 0; ch < nch; ++ch) {
      double bc[NJ][S], wc[TR][NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
#pragma unroll
        for (int s2 = 0; s2 < S; ++s2) bc[j][s2] = b[j][s2];
#pragma unroll
        for (int t = 0; t < TR; ++t) wc[t][j] = w[t][j];
      }
      if (ch + 1 < nch) load(kbeg + (ch + 1) * kKC);
#pragma unroll
      for (int t = 0; t < TR; ++t)
#pragma unroll
        for (int s2 = 0; s2 < S; ++s2)
#pragma unroll
          for (int j = 0; j < NJ; ++j)
            acc[t][s2] = __builtin_amdgcn_mfma_f64_16x16x4f64(wc[t][j], bc[j][s2], acc[t][s2], 0, 0, 0);
    }
    const bool ovec = ((o.ldo & 1) == 0) && ((reinterpret_cast<uintptr_t>(o.OUT) & 15) == 0) &&
                      (!o.X || (((o.ldx & 1) == 0) && ((reinterpret_cast<uintptr_t>(o.X) & 15) == 0)));
#pragma unroll
    for (int t = 0; t < TR; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + t * 16 + 4 * v + lg;
        if (row >= M) continue;
        double* orow = o.OUT + static_cast<int64_t>(row) * o.ldo;
        const double* xrow = o.X ? o.X + static_cast<int64_t>(row) * o.ldx : nullptr;
#pragma unroll
        for (int p = 0; p < WN; ++p) {
          const int c0 = col[2 * p];
          double y0 = o.alpha * acc[t][2 * p][v];
          double y1 = o.alpha * acc[t][2 * p + 1][v];
          if (ovec && c0 + 1 < N) {
            if (xrow) {
              const double2 x = *reinterpret_cast<const double2*>(xrow + c0);
              y0 = x.x + y0;
              y1 = x.y + y1;
            }
            *reinterpret_cast<double2*>(orow + c0) = double2{y0, y1};
          } else {
            if (c0 < N) orow[c0] = xrow ? xrow[c0] + y0 : y0;
            if (c0 + 1 < N) orow[c0 + 1] = xrow ? xrow[c0 + 1] + y1 : y1;
          }
        }
      }
  }
}

// Pivot blocks N_k of every unfinished matrix inverted in place (rows already in
// partial-pivoting order), one workgroup each.
__global__ __launch_bounds__(256) void batch_inverse_kernel(BatchMat* __restrict__ mats, int count) {
  if (static_cast<int>(blockIdx.x) >= count) return;
  BatchMat* bm = mats + blockIdx.x;
  if (bm->s == 0 || bm->nI == 0) return;
  gj_inorder_tile(bm->Nk, bm->nI, &bm->info);
}

// End of an iteration, one workgroup per matrix: the column-residual norm (its tile
// partials summed in a fixed order), the commit of the block, the stopping decision and
// the record for the host.
__global__ __launch_bounds__(256) void batch_end_kernel(BatchMat* __restrict__ mats, int count, int b,
                                                        BatchRec* __restrict__ rec) {
  __shared__ double red[4];
  if (static_cast<int>(blockIdx.x) >= count) return;
  BatchMat* bm = mats + blockIdx.x;
  if (bm->s != 0) {
    const int nJ = bm->nJ, nI = bm->nI;
    if (nJ == 0 || nI == 0) {
      if (threadIdx.x == 0) {
        bm->status = ICUR_STALLED;
        bm->s = 0;
      }
    } else if (bm->info != 0) {
      if (threadIdx.x == 0) {
        bm->status = ICUR_ERR_HIP;
        bm->s = 0;
      }
    } else {
      double v = 0.0;
      for (int q = threadIdx.x; q < bm->nparts; q += 256) v += bm->normp[q];
      const double tot = block_sum(v, red);
      const int r = bm->r;
      for (int t = threadIdx.x; t < nI; t += 256) {
        const int64_t j = bm->Jk[t], i = bm->Ik[t];
        bm->colmask[j] = 1;
        bm->rowmask[i] = 1;
        bm->Jall[r + t] = j;
        bm->Iall[r + t] = i;
      }
      if (threadIdx.x == 0) {
        const double rho = sqrt(tot / bm->denom2);
        const int rn = r + nI;
        bm->rho = rho;
        bm->r = rn;
        bm->iters += 1;
        if (rho <= bm->thr) {
          bm->status = ICUR_OK;
          bm->s = 0;
        } else if (rn >= bm->rmax) {
          bm->status = ICUR_MAXRANK;
          bm->s = 0;
        } else {
          bm->s = min(b, bm->rmax - rn);
        }
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    BatchRec& o = rec[blockIdx.x];
    o.r = bm->r;
    o.s = bm->s;
    o.status = bm->status;
    o.info = bm->info;
    o.iters = bm->iters;
    o.rho = bm->rho;
  }
}

}  // namespace

// ------------------------------------------------------------------ host wrappers
size_t batch_plan_bytes(int count) {
  const size_t per = static_cast<size_t>(count) * kOpsPerMat;
  return kNumStages * per * (sizeof(GemmOp) + sizeof(GatherOp)) + 128 + kNumStages * sizeof(double) + 512;
}

namespace {
Plan bind_plan(void* ws, int count, const int* shape_of_stage = nullptr) {
  Plan p;
  for (int s = 0; s < kNumStages; ++s) {
    const int sh = shape_of_stage ? shape_of_stage[s] : 1;
    p.rt[s] = 16 * kShapes[sh].tr;
    p.ct[s] = (kShapes[sh].wave ? 32 : 128) * kShapes[sh].wn;
  }
  char* q = static_cast<char*>(ws);
  const size_t per = static_cast<size_t>(count) * kOpsPerMat;
  for (int s = 0; s < kNumStages; ++s) {
    p.gemm[s] = reinterpret_cast<GemmOp*>(q);
    q += per * sizeof(GemmOp);
    p.gather[s] = reinterpret_cast<GatherOp*>(q);
    q += per * sizeof(GatherOp);
  }
  p.nops = reinterpret_cast<int*>(q);
  p.ntiles = p.nops + kNumStages;
  p.bytes = reinterpret_cast<double*>(q + 128);
  return p;
}

template <typename KERNEL>
int gemm_launch(KERNEL kernel, int* per_cu, const Plan& p, int s, hipStream_t st) {
  // persistent grid: as many workgroups as fit on the device at once
  if (*per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kPT, 0) != hipSuccess || nb < 1) {
      (void)hipGetLastError();
      nb = 1;
    }
    *per_cu = std::min(nb, 8);
  }
  DeviceInfo dev;
  ICUR_TRY(device_info(&dev));
  hipLaunchKernelGGL(kernel, dim3(*per_cu * dev.num_cus), dim3(kPT), 0, st, p.gemm[s], p.nops + s, p.ntiles + s);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

template <int ROLE>
int gemm_stage_role(const Plan& p, int s, int shape, hipStream_t st) {
  static int per_cu[kGemmShapes] = {};
  switch (shape) {
    case 0: return gemm_launch(gemm_kernel<1, 1, ROLE>, &per_cu[0], p, s, st);
    case 1: return gemm_launch(gemm_kernel<2, 1, ROLE>, &per_cu[1], p, s, st);
    case 2: return gemm_launch(gemm_kernel<3, 1, ROLE>, &per_cu[2], p, s, st);
    case 3: return gemm_launch(gemm_kernel<4, 1, ROLE>, &per_cu[3], p, s, st);
    case 4: return gemm_launch(gemm_kernel<2, 2, ROLE>, &per_cu[4], p, s, st);
    case 5: return gemm_launch(gemm_kernel<4, 2, ROLE>, &per_cu[5], p, s, st);
    case 6: return gemm_launch(gemm_wave_kernel<2, 1, ROLE>, &per_cu[6], p, s, st);
    case 7: return gemm_launch(gemm_wave_kernel<1, 2, ROLE>, &per_cu[7], p, s, st);
    case 8: return gemm_launch(gemm_wave_kernel<2, 2, ROLE>, &per_cu[8], p, s, st);
    case 9: return gemm_launch(gemm_kernel<2, 1, ROLE, 2>, &per_cu[9], p, s, st);
    case 10: return gemm_launch(gemm_kernel<4, 1, ROLE, 2>, &per_cu[10], p, s, st);
    case 11: return gemm_launch(gemm_kernel<2, 1, ROLE, 3>, &per_cu[11], p, s, st);
    default: return arg_error("grouped product: unknown tile shape");
  }
}

int gemm_stage(const Plan& p, int s, int shape, hipStream_t st) {
  return s == kFin ? gemm_stage_role<1>(p, s, shape, st) : gemm_stage_role<0>(p, s, shape, st);
}

// One product on the workgroup tiles of 32 x 128: persistent grid over its tiles.
int gemm_one(const GemmOp& o, hipStream_t st) {
  static int per_cu = 0;
  if (per_cu == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, gemm_one_kernel<2, 1>, kPT, 0) != hipSuccess || nb < 1) {
      (void)hipGetLastError();
      nb = 1;
    }
    per_cu = std::min(nb, 8);
  }
  DeviceInfo dev;
  ICUR_TRY(device_info(&dev));
  const int64_t tiles = ((o.M + 31) / 32) * static_cast<int64_t>(o.tiles_n);
  const int grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(tiles, per_cu * dev.num_cus)));
  hipLaunchKernelGGL((gemm_one_kernel<2, 1>), dim3(grid), dim3(kPT), 0, st, o);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

int gather_stage(const Plan& p, int s, int grid, hipStream_t st) {
  hipLaunchKernelGGL(gather_kernel, dim3(grid), dim3(kPT), 0, st, p.gather[s], p.nops + s, p.ntiles + s);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}
}  // namespace

// One iteration of Alg. 1 (residual form, with the core's two inverses) for every
// unfinished matrix: 13 launches whose configuration depends only on count and the device.
double* batch_plan_bytes_ptr(void* plan_ws, int count) { return bind_plan(plan_ws, count).bytes; }

int batch_plan_stages() { return kNumStages; }

// OUT (M x N, ld ldo) = X + alpha W B (X may be null, or equal to OUT with ldx == ldo), all
// FP64 row-major, on the FP64 matrix cores (the grouped product's workgroup tile).
int gemm_f64_native(int64_t M, int64_t N, int64_t K, double alpha, const double* W, int64_t ldw, const double* B,
                    int64_t ldb, const double* X, int64_t ldx, double* OUT, int64_t ldo, hipStream_t st) {
  if (M < 0 || N < 0 || K < 0 || M > INT_MAX || N > INT_MAX || K > INT_MAX)
    return arg_error("native product: sizes out of range");
  if (M == 0 || N == 0) return ICUR_OK;
  GemmOp o;
  std::memset(&o, 0, sizeof(o));
  o.X = X;
  o.ldx = ldx;
  o.W = W;
  o.ldw = ldw;
  o.B = B;
  o.ldb = ldb;
  o.OUT = OUT;
  o.ldo = ldo;
  o.M = static_cast<int>(M);
  o.K = static_cast<int>(K);
  o.N = static_cast<int>(N);
  o.tiles_n = static_cast<int>((N + 127) / 128);
  o.alpha = alpha;
  return gemm_one(o, st);
}
int batch_plan_final_stage() { return kFin; }
std::vector<int> batch_plan_product_stages() { return {kP1, kP2, kP3, kP4, kFin}; }

// Shape of each product stage: P1, P2, P3 and FIN as given; P4, whose tiles carry the
// norm partials, always the one that fits c rows (so rho does not depend on the tuning).
void stage_shapes(const GemmTiles& t, int c, int* out) {
  for (int s = 0; s < kNumStages; ++s) out[s] = 1;
  out[kP1] = t.p1;
  out[kP2] = t.p2;
  out[kP3] = t.p3;
  out[kFin] = t.fin;
  out[kP4] = c <= 16 ? 0 : c <= 32 ? 1 : c <= 48 ? 2 : 3;
}

int check_tiles(const GemmTiles& t) {
  for (int v : {t.p1, t.p2, t.p3, t.fin})
    if (v < 0 || v >= kGemmShapes) return arg_error("grouped product: tile shape out of range");
  return ICUR_OK;
}

int launch_batch_iteration(BatchMat* mats, int count, int c, int b, double row_cut, void* plan_ws, BatchRec* rec,
                           const GemmTiles& tiles, int grid, hipStream_t st, hipEvent_t* ev) {
  ICUR_TRY(check_tiles(tiles));
  int sh[kNumStages];
  stage_shapes(tiles, c, sh);
  const Plan p = bind_plan(plan_ws, count, sh);
  auto mark = [&](int k) -> int {
    if (ev) ICUR_HIP(hipEventRecord(ev[k], st));
    return ICUR_OK;
  };
  ICUR_TRY(mark(0));
  ICUR_TRY(launch_batch_lupp(mats, count, false, 0.0, st));
  ICUR_TRY(mark(1));
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, st, mats, count, c, b, 0, p);
  ICUR_HIP(hipGetLastError());
  ICUR_TRY(gather_stage(p, kGA, grid, st));
  ICUR_TRY(mark(4));
  ICUR_TRY(gemm_stage(p, kP1, sh[kP1], st));
  ICUR_TRY(mark(5));
  ICUR_TRY(mark(2));
  ICUR_TRY(launch_batch_lupp(mats, count, true, row_cut, st));
  ICUR_TRY(mark(3));
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, st, mats, count, c, b, 1, p);
  ICUR_HIP(hipGetLastError());
  ICUR_TRY(gather_stage(p, kGB, grid, st));
  hipLaunchKernelGGL(batch_inverse_kernel, dim3(count), dim3(256), 0, st, mats, count);
  ICUR_HIP(hipGetLastError());
  ICUR_TRY(mark(6));
  ICUR_TRY(gemm_stage(p, kP2, sh[kP2], st));
  ICUR_TRY(mark(7));
  ICUR_TRY(mark(8));
  ICUR_TRY(gemm_stage(p, kP3, sh[kP3], st));
  ICUR_TRY(mark(9));
  ICUR_TRY(mark(10));
  ICUR_TRY(gemm_stage(p, kP4, sh[kP4], st));
  ICUR_TRY(mark(11));
  ICUR_TRY(gather_stage(p, kGC, grid, st));
  hipLaunchKernelGGL(batch_end_kernel, dim3(count), dim3(256), 0, st, mats, count, b, rec);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

// At the end of an iteration: the core A(I,J)^{-1} = Q^{-1} P^{-1} of every matrix that
// stopped in it, into its LcT buffer (r x r, leading dimension r), one launch for all.
int launch_batch_final(BatchMat* mats, int count, int c, int b, void* plan_ws, const GemmTiles& tiles,
                       hipStream_t st) {
  ICUR_TRY(check_tiles(tiles));
  int sh[kNumStages];
  stage_shapes(tiles, c, sh);
  const Plan p = bind_plan(plan_ws, count, sh);
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, st, mats, count, c, b, 2, p);
  ICUR_HIP(hipGetLastError());
  return gemm_stage(p, kFin, sh[kFin], st);
}

}  // namespace icur
