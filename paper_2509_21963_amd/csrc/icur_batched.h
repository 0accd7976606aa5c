// Grouped kernels of the batched form: many independent matrices advanced together, one
// launch per step of Alg. 1 for all of them (icur_group_*.hip), driven by
// icur_batched.hip.
#pragma once

#include <string>
#include <vector>

#include "icur_internal.h"

namespace icur {

// ----- limits of the grouped path
constexpr int kGMaxN = 8192;     // candidates per selection (one workgroup holds them all)
constexpr int kGMaxSteps = 64;   // pivots per selection (so block <= 64, c <= 70)

// ----- the grouped FP64 product
constexpr int kGemmShapes = 12;    // tile shapes (rows x columns): workgroup tiles 16x128,
                                   // 32x128, 48x128, 64x128, 32x256, 64x256; wave tiles
                                   // 32x32, 16x64, 32x64; workgroup tiles with two or three
                                   // chunks in flight 32x128/2, 64x128/2, 32x128/3
constexpr int kGemmMaxCols = 256;  // widest tile
constexpr int kGemmKChunk = 16;    // depth chunk; chunks start at multiples of it, so an
                                   // element's sum does not depend on the tile shape
// Columns right of a new diagonal block of the core's inverses that are written with it
// (identity or zeros), so that every entry a depth-skipping product reads is defined: a
// tile whose columns start at n0 reads rows k >= n0 - (b - 1) rounded down to a chunk, so
// entries up to k + b + kGemmMaxCols + kGemmKChunk - 2 to the right of the diagonal.
constexpr int kBandCols = kGMaxSteps + kGemmMaxCols + kGemmKChunk;

// One LUPP selection: pivots of T = X^T (N candidates x K >= *steps columns), FP64,
// textbook right-looking rounding (the pivots of icur_lupp on the same values).
struct GroupLuppJob {
  const double* X;        // K x N, leading dimension ldx: X[t * ldx + i] = T[i][t]
  int64_t ldx;
  int N;                  // candidates, <= kGMaxN
  int pad;
  const int* steps;       // device: pivots wanted (<= kGMaxSteps); 0 skips the job
  const uint8_t* excl;    // N flags or null
  double* L;              // scratch, *steps x N doubles
  int64_t* piv;           // out: pivot indices in order
  int* npiv;              // out: pivots found
  double rel_cut;         // > 0: stop at a pivot <= rel_cut * |first pivot|
};
int launch_group_lupp(const GroupLuppJob* jobs_dev, int njobs, hipStream_t st);

// ----- per-matrix state of the batched loop (device array, one entry per matrix)
struct BatchMat {
  // input and fixed buffers
  const float* A;
  int64_t lda;
  int m, n;
  double* S;          // c x n: X0, then the sketched column residual
  double* Lsel;       // b x max(m, n): selection multipliers
  double* Sr;         // b x n: residual at the new rows, A(I_k,:) - Lc(I_k,:) Ur
  double* Wc;         // c x b: S(:, J_k)
  double* Nk;         // b x b: pivot block N_k = S(I_k, J_k), inverted in place
  double* normp;      // norm partials of the column-residual update
  uint8_t* colmask;   // n
  uint8_t* rowmask;   // m
  int64_t* Jk;        // b
  int64_t* Ik;        // b
  // rank-sized buffers (capacity cap, grown by the host between iterations).  The core
  // A(I,J)^{-1} is kept factored: A(I,J) = P Q with P = Lc(I,:) block lower triangular
  // (diagonal blocks N_k) and Q = Ur(:,J) block upper triangular with identity diagonal
  // blocks, so A(I,J)^{-1} = Q^{-1} P^{-1}; both inverses grow by one block per iteration
  // and are multiplied out once, after the loop.
  double* LcT;        // cap x m: column factors (row t = S^{(k-1)}(:, J_k[t])^T); after the
                      // loop the core A(I,J)^{-1}, r x r, leading dimension r
  double* Ur;         // cap x n: row factors (N_k^{-1} S^{(k-1)}(I_k, :))
  double* QT;         // cap x cap: (Q^{-1})^T, block lower triangular, identity diagonal blocks
  double* Pi;         // cap x cap: P^{-1}, block lower triangular, diagonal blocks N_k^{-1}
  double* Wa;         // b x cap: Ur(:, J_k)^T, the new block column of Q (transposed)
  double* Wl;         // b x cap: Lc(I_k, :), the new block row of P
  double* Wp;         // b x cap: N_k^{-1} Lc(I_k, :)
  int64_t* Jall;      // cap
  int64_t* Iall;      // cap
  int cap;
  int rmax;           // rank bound, min(m, n, max_rank)
  // loop state
  int r;              // indices selected so far
  int s;              // column pivots wanted this iteration; 0 = finished
  int nJ, nI;         // pivots found by this iteration's selections
  int info;           // nonzero: N_k exactly singular
  int status;         // ICUR_OK, ICUR_MAXRANK or ICUR_STALLED once finished
  int iters;
  double denom2;      // squared denominator of rho
  double thr;         // stopping threshold xi * tol
  double rho;
  int nparts;         // norm partials written by the last update
  int fin;            // the core has been multiplied out (set once the matrix stops)
};

// The column (rows = false) or row selection of every unfinished matrix, one workgroup
// each: writes Jk / nJ or Ik / nI.
int launch_batch_lupp(BatchMat* mats_dev, int count, bool rows, double rel_cut, hipStream_t st);

// Tile shapes (indices into the shape table above) of the grouped product stages: the
// row residual P1, the new-row residual and (Q^{-1})^T block P2, the row factors and P^{-1}
// block P3, and the core products FIN.  The column update's shape follows c.  Every
// choice gives the same results: only the speed differs.
struct GemmTiles {
  int p1 = 9, p2 = 9, p3 = 9, fin = 9;
};

// The tile shapes for block size b: defaults, the tune file's entry for b, and the
// ICUR_BATCH_TILES override, in that order.
GemmTiles batch_tiles(int b);

// Per-matrix record copied to host-mapped memory at the end of every iteration.
struct BatchRec {
  int r, s, status, info, iters, pad;
  double rho;
};

// Arguments of one icur_run_batched call as the grouped driver sees them (host arrays
// indexed by matrix; checked by the caller).
struct BatchedCall {
  int count;
  const float* const* A;
  const int64_t* m;
  const int64_t* n;
  const int64_t* lda;
  const double* tol;
  int block;
  int kind;
  const uint64_t* seed;
  const icur_opts* opts;  // defaults applied
  double xi;              // risk-aware factor (1 when off)
  double row_cut;         // relative cut of the row selection
  int64_t* I_pool;
  int64_t* J_pool;
  double* U_pool;
  const int64_t* cap_offsets;
  const int64_t* uoff;    // start of each matrix's core in U_pool
  int64_t* rank;
  double* est;
  int32_t* status;
  std::string* errs;      // per-matrix messages of failed matrices
  int iterations;         // out: grouped iterations run
  double ms_sketch;       // out: the sketch phase (host clock, all sketch streams drained)
  double ms_select;       // out: device time of the grouped selections
  double ms_products;     // out: device time of the grouped product launches
  double product_bytes;   // out: their algorithmic bytes (W, B and X read once, OUT written once)
  int product_launches;   // out
  double ms_alloc;        // out: host clock of the buffer set-up after the sketch
  double ms_loop;         // out: host clock of the grouped iterations
  double ms_final;        // out: device time of the closing core products Q^{-1} P^{-1}
  double ms_stage[5];     // out: device time of the product stages P1, P2, P3, P4, FIN
  double stage_bytes[5];  // out: their algorithmic bytes (nonzero operand parts read once,
                          // output written once)
  int tiles[4];           // out: tile shapes used for P1, P2, P3, FIN
  int sketch_kernel;      // out: matrices whose G A ran on the dedicated sketch kernel
  int graph_iterations;   // out: iterations run as a replay of the captured iteration graph
  double ms_results;      // out: host clock of the copies to the caller's pools
};

// Alg. 1 on the matrices listed in `which` (each with max(m, n) <= kGMaxN, block <=
// kGMaxSteps), all advanced together; results into the call's pools.  Per-matrix
// failures go to status / errs; the return value is an error only when the whole group
// could not run.
int run_batched_grouped(const std::vector<int>& which, BatchedCall& a, hipStream_t st);

// Frees the device arenas the grouped calls keep between calls (all devices).
void release_batch_arenas();

}  // namespace icur
