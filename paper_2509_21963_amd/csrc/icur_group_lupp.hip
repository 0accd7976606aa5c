// Grouped LUPP selection: one workgroup per selection, many selections per launch (the
// column and row selections of §3.2.1 / §3.2.2 for every active matrix of a batch).
//
// Each workgroup holds all N <= kGMaxN candidates of its selection (kGR rows per thread
// on kGT threads), so no step needs a grid exchange: the pivot search is a workgroup
// argmax and the pivot row goes through LDS.  The pivot columns are processed in panels
// of kGPW: a panel's entries of every live candidate are formed left-looking from the
// multipliers of the earlier panels (kept in global scratch, read once per panel), the
// panel's steps run on registers, and the new pivot rows are then extended to every later
// column (their triangular recurrence, held in LDS).
//
// Exactness is that of icur_lupp.hip: FP64, contraction off, and every element receives
// the textbook right-looking updates x <- x - (l * u) in step order, so the pivots equal
// those of a plain FP64 LUPP (ties to the lowest index), whatever the grouping.
#include <algorithm>
#include <climits>
#include <utility>

#include "icur_batched.h"
#include "icur_wave.h"

#pragma clang fp contract(off)

namespace icur {
namespace {

constexpr int kGT = 1024;                 // threads per workgroup
constexpr int kGR = kGMaxN / kGT;         // candidate rows per thread
constexpr int kGPW = 4;                   // panel width

template <class F, int... I>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

__device__ __forceinline__ void lupp_wg(const GroupLuppJob& jb) {
  const int steps = jb.steps ? *jb.steps : 0;
  if (steps <= 0) {
    if (threadIdx.x == 0 && jb.npiv) *jb.npiv = 0;
    return;
  }
  __shared__ double Us[kGMaxSteps * kGMaxSteps];  // Us[s * kGMaxSteps + c]: pivot row s at column c
  __shared__ double Lp[kGPW * kGMaxSteps];         // multipliers of the panel's pivot rows
  __shared__ long long pidx[kGMaxSteps];
  __shared__ double prow[kGPW];
  __shared__ Red red[kGT / 64];

  const int tid = threadIdx.x;
  const int N = jb.N;
  const double* X = jb.X;
  const int64_t ldx = jb.ldx;
  double* L = jb.L;

  unsigned alive = 0;
#pragma unroll
  for (int r = 0; r < kGR; ++r) {
    const int i = r * kGT + tid;
    if (i < N && !(jb.excl && jb.excl[i])) alive |= 1u << r;
  }
  int found = 0;
  bool stop = false;
  unsigned long long ref_key = 0ull;

  for (int t0 = 0; t0 < steps && !stop; t0 += kGPW) {
    const int pw = min(kGPW, steps - t0);
    // (1) the panel's entries of every live candidate, all t0 earlier updates applied in
    // step order (left-looking: multipliers from L, pivot rows from Us)
    double x[kGR][kGPW];
#pragma unroll
    for (int r = 0; r < kGR; ++r) {
      const int i = r * kGT + tid;
      const bool live = (alive >> r) & 1u;
#pragma unroll
      for (int jj = 0; jj < kGPW; ++jj) x[r][jj] = (live && jj < pw) ? X[static_cast<int64_t>(t0 + jj) * ldx + i] : 0.0;
    }
    // one step of multipliers per round for all rows (kGR loads in flight per thread,
    // sixteen waves per CU)
    for (int s0 = 0; s0 < t0; ++s0) {
      double l[kGR];
#pragma unroll
      for (int r = 0; r < kGR; ++r) {
        const int i = r * kGT + tid;
        l[r] = ((alive >> r) & 1u) ? L[static_cast<int64_t>(s0) * N + i] : 0.0;
      }
      double u[kGPW];
#pragma unroll
      for (int jj = 0; jj < kGPW; ++jj) u[jj] = Us[s0 * kGMaxSteps + t0 + jj];
#pragma unroll
      for (int r = 0; r < kGR; ++r)
#pragma unroll
        for (int jj = 0; jj < kGPW; ++jj) {
          const double prod = l[r] * u[jj];
          x[r][jj] = x[r][jj] - prod;
        }
    }
    const unsigned alive0 = alive;
    unsigned cstep = 0;  // 4 bits per row: panel step at which row r became a pivot
    // (2) the panel's steps
    sfor<kGPW>([&](auto ttc) {
      constexpr int tt = decltype(ttc)::value;
      if (stop || tt >= pw) return;
      const int t = t0 + tt;
      double bv = -1.0;
      int bi = INT_MAX, br = -1;
#pragma unroll
      for (int r = 0; r < kGR; ++r) {
        const double v = fabs(x[r][tt]);
        const int i = r * kGT + tid;
        if (((alive >> r) & 1u) && better(v, i, bv, bi)) {
          bv = v;
          bi = i;
          br = r;
        }
      }
      unsigned long long gk;
      int gi, gw;
      block_argmax<kGT>(cand_key(bv), bi, 0, red, &gk, &gi, &gw);
      // the owner's row from column tt on, into LDS (selected with masks, no run-time
      // register indexing)
      if (gk != 0ull && br >= 0 && bi == gi) {
#pragma unroll
        for (int jj = tt; jj < kGPW; ++jj) {
          unsigned long long w = 0ull;
#pragma unroll
          for (int r = 0; r < kGR; ++r)
            w |= static_cast<unsigned long long>(__double_as_longlong(x[r][jj])) & (r == br ? ~0ull : 0ull);
          prow[jj] = __longlong_as_double(static_cast<long long>(w));
        }
      }
      if (gk == 0ull) stop = true;
      if (t == 0) ref_key = gk;
      if (jb.rel_cut > 0.0 && t > 0 &&
          gk <= static_cast<unsigned long long>(
                    __double_as_longlong(jb.rel_cut * __longlong_as_double(static_cast<long long>(ref_key)))))
        stop = true;
      __syncthreads();  // prow visible; red free again after this step's reads
      if (stop) return;
      found = t + 1;
      if (tid == 0) pidx[t] = gi;
      if (tid < kGPW && tid >= tt && tid < pw) Us[t * kGMaxSteps + t0 + tid] = prow[tid];
      const double upiv = prow[tt];
      double uu[kGPW];
#pragma unroll
      for (int jj = tt + 1; jj < kGPW; ++jj) uu[jj] = prow[jj];
#pragma unroll
      for (int r = 0; r < kGR; ++r) {
        const int i = r * kGT + tid;
        if (((alive >> r) & 1u) && i == gi) {
          alive &= ~(1u << r);
          cstep |= static_cast<unsigned>(tt) << (4 * r);
        }
        const double l = x[r][tt] / upiv;
        x[r][tt] = l;
#pragma unroll
        for (int jj = tt + 1; jj < kGPW; ++jj) {
          const double prod = l * uu[jj];
          x[r][jj] = x[r][jj] - prod;
        }
      }
      __syncthreads();  // prow is rewritten by the next step's owner
    });
    // (3) multipliers of this panel to L: every step for rows still live, the steps
    // before their own for the rows chosen here
    const int done = found - t0;
#pragma unroll
    for (int r = 0; r < kGR; ++r) {
      if ((alive0 >> r) & 1u) {
        const int i = r * kGT + tid;
        const bool piv_row = !((alive >> r) & 1u);
        const int nl = piv_row ? static_cast<int>((cstep >> (4 * r)) & 15u) : done;
#pragma unroll
        for (int jj = 0; jj < kGPW; ++jj)
          if (jj < nl) L[static_cast<int64_t>(t0 + jj) * N + i] = x[r][jj];
      }
    }
    if (stop || found >= steps) break;
    __syncthreads();  // L of this panel visible to the workgroup
    // (4) extend this panel's pivot rows to every later column: row t at column c is
    // X[c][p_t] minus its updates by the pivot rows of steps 0 .. t-1, in step order
    for (int e = tid; e < done * t0 + done * done; e += kGT) {
      // stage the multipliers L[q][p_t], q < t, of the panel's pivot rows
      const int tt = e / (t0 + done), q = e % (t0 + done);
      const int t = t0 + tt;
      if (q < t) Lp[tt * kGMaxSteps + q] = L[static_cast<int64_t>(q) * N + pidx[t]];
    }
    __syncthreads();
    const int c = t0 + kGPW + tid;
    if (c < steps) {
      for (int tt = 0; tt < done; ++tt) {
        const int t = t0 + tt;
        double acc = X[static_cast<int64_t>(c) * ldx + pidx[t]];
        for (int q = 0; q < t; ++q) {
          const double prod = Lp[tt * kGMaxSteps + q] * Us[q * kGMaxSteps + c];
          acc = acc - prod;
        }
        Us[t * kGMaxSteps + c] = acc;
      }
    }
    __syncthreads();
  }
  if (tid < found) jb.piv[tid] = pidx[tid];
  if (tid == 0) *jb.npiv = found;
}

__global__ __launch_bounds__(kGT, 1) void group_lupp_kernel(const GroupLuppJob* __restrict__ jobs, int njobs) {
  if (static_cast<int>(blockIdx.x) >= njobs) return;
  lupp_wg(jobs[blockIdx.x]);
}

// The selections of the batched loop, built from each matrix's state: the column
// selection on (S^col)^T (s pivots, columns of J masked), or the row selection on the
// iteration's row residual (rows r .. r + nJ - 1 of LcT, nJ pivots, rows of I masked,
// ended early at a numerically zero pivot).
__global__ __launch_bounds__(kGT, 1) void batch_lupp_kernel(BatchMat* __restrict__ mats, int count, int rows,
                                                            double rel_cut) {
  if (static_cast<int>(blockIdx.x) >= count) return;
  BatchMat* bm = mats + blockIdx.x;
  if (bm->s == 0) return;  // finished
  GroupLuppJob jb;
  if (!rows) {
    jb.X = bm->S;
    jb.ldx = bm->n;
    jb.N = bm->n;
    jb.steps = &bm->s;
    jb.excl = bm->colmask;
    jb.piv = bm->Jk;
    jb.npiv = &bm->nJ;
    jb.rel_cut = 0.0;
  } else {
    jb.X = bm->LcT + static_cast<int64_t>(bm->r) * bm->m;
    jb.ldx = bm->m;
    jb.N = bm->m;
    jb.steps = &bm->nJ;
    jb.excl = bm->rowmask;
    jb.piv = bm->Ik;
    jb.npiv = &bm->nI;
    jb.rel_cut = rel_cut;
  }
  jb.L = bm->Lsel;
  lupp_wg(jb);
}

}  // namespace

int launch_batch_lupp(BatchMat* mats_dev, int count, bool rows, double rel_cut, hipStream_t st) {
  if (count <= 0) return ICUR_OK;
  hipLaunchKernelGGL(batch_lupp_kernel, dim3(static_cast<unsigned>(count)), dim3(kGT), 0, st, mats_dev, count,
                     rows ? 1 : 0, rel_cut);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

int launch_group_lupp(const GroupLuppJob* jobs_dev, int njobs, hipStream_t st) {
  if (njobs <= 0) return ICUR_OK;
  hipLaunchKernelGGL(group_lupp_kernel, dim3(static_cast<unsigned>(njobs)), dim3(kGT), 0, st, jobs_dev, njobs);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

}  // namespace icur
