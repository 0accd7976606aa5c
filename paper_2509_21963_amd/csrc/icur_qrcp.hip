// Index selection by QR with column pivoting, Alg. 1's alternative to LUPP for both
// selections (§5.3 compares the two): the candidates are the rows of T = X^T (N
// candidates of K coordinates each), the pivot of step t is the candidate whose component
// orthogonal to the ones already chosen has the largest norm.
//
// The residual vectors are kept explicitly (FP64, one column of a K x N working copy per
// candidate) and orthogonalised against each new direction, modified Gram-Schmidt style:
// s_i = q . x_i, x_i <- x_i - s_i q, and the norm is recomputed from the updated vector
// (no downdating, so small residual norms keep their relative accuracy).  In exact
// arithmetic these are the trailing norms of Householder QR with column pivoting, so
// the pivots equal LAPACK geqp3's wherever the norms are not tied to rounding.
//
// Per step two launches: the update of every live candidate with its workgroup's
// argmax, then a one-workgroup pick of the pivot and its normalised direction.  A step
// whose best norm is zero (or, with a relative cut, at most cut times the first pivot's)
// ends the selection; the later launches return at once.
#include <algorithm>
#include <climits>

#include "icur_internal.h"
#include "icur_wave.h"

namespace icur {
namespace {

constexpr int kQT = 256;
constexpr int kMaxK = 4096;

struct QrcpArgs {
  const void* X;  // K x N (FP32 or FP64), leading dimension ldx
  int64_t ldx;
  int K, N, t;
  const uint8_t* excl;
  double* Xw;     // K x N working copy
  double* q;      // K
  double* pval;   // per-workgroup best norm^2
  int* pidx;
  uint8_t* chosen;
  int* status;    // [0] pivots, [1] fault flag (unused here), [2] ended
  double* ref;    // first pivot's norm^2
  int64_t* piv;
  double rel_cut2;  // squared relative cut (0: none)
};

template <int X64>
__global__ __launch_bounds__(kQT) void qrcp_update(const QrcpArgs a) {
  __shared__ double qs[kMaxK];
  __shared__ Red red[kQT / 64];
  if (a.t > 0 && a.status[2] != 0) return;
  const int K = a.K, N = a.N;
  if (a.t > 0)
    for (int k = threadIdx.x; k < K; k += kQT) qs[k] = a.q[k];
  __syncthreads();
  double bv = -1.0;
  int bi = INT_MAX;
  for (int i = blockIdx.x * kQT + threadIdx.x; i < N; i += gridDim.x * kQT) {
    if (a.t == 0) a.chosen[i] = 0;
    if ((a.excl && a.excl[i]) || (a.t > 0 && a.chosen[i])) continue;
    double d = 0.0;
    if (a.t == 0) {
      for (int k = 0; k < K; ++k) {
        const double v = X64 ? static_cast<const double*>(a.X)[k * a.ldx + i]
                             : static_cast<double>(static_cast<const float*>(a.X)[k * a.ldx + i]);
        a.Xw[static_cast<int64_t>(k) * N + i] = v;
        d += v * v;
      }
    } else {
      double s = 0.0;
      for (int k = 0; k < K; ++k) s += qs[k] * a.Xw[static_cast<int64_t>(k) * N + i];
      for (int k = 0; k < K; ++k) {
        const double v = a.Xw[static_cast<int64_t>(k) * N + i] - s * qs[k];
        a.Xw[static_cast<int64_t>(k) * N + i] = v;
        d += v * v;
      }
    }
    if (d > bv || (d == bv && i < bi)) {
      bv = d;
      bi = i;
    }
  }
  unsigned long long gk;
  int gi, gw;
  block_argmax<kQT>(cand_key(bv), bi, 0, red, &gk, &gi, &gw);
  if (threadIdx.x == 0) {
    a.pval[blockIdx.x] = __longlong_as_double(static_cast<long long>(gk));
    a.pidx[blockIdx.x] = gi;
  }
}

__global__ __launch_bounds__(kQT) void qrcp_pick(const QrcpArgs a, int groups) {
  __shared__ Red red[kQT / 64];
  __shared__ double inv;
  if (a.t > 0 && a.status[2] != 0) return;
  unsigned long long k = 0ull;
  int i = INT_MAX;
  for (int g = threadIdx.x; g < groups; g += kQT) {
    const unsigned long long kg = static_cast<unsigned long long>(__double_as_longlong(a.pval[g]));
    const int ig = a.pidx[g];
    if (kg > k || (kg == k && ig < i)) {
      k = kg;
      i = ig;
    }
  }
  unsigned long long gk;
  int gi, gw;
  block_argmax<kQT>(k, i, 0, red, &gk, &gi, &gw);
  const double best = __longlong_as_double(static_cast<long long>(gk));
  bool stop = gk == 0ull;
  if (!stop && a.t > 0 && a.rel_cut2 > 0.0 && best <= a.rel_cut2 * *a.ref) stop = true;
  if (stop) {
    if (threadIdx.x == 0) {
      a.status[2] = 1;
      a.status[0] = a.t;
    }
    return;
  }
  if (threadIdx.x == 0) {
    if (a.t == 0) *a.ref = best;
    a.piv[a.t] = gi;
    a.chosen[gi] = 1;
    a.status[0] = a.t + 1;
    inv = 1.0 / sqrt(best);
  }
  __syncthreads();
  for (int kk = threadIdx.x; kk < a.K; kk += kQT) a.q[kk] = a.Xw[static_cast<int64_t>(kk) * a.N + gi] * inv;
}

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

size_t qrcp_workspace_bytes(int64_t K, int64_t N, int groups) {
  return al256(static_cast<size_t>(K) * N * 8) + al256(static_cast<size_t>(K) * 8) + al256(groups * 8) +
         al256(groups * 4) + al256(static_cast<size_t>(N)) + 256;
}

int qrcp_launch(const void* X, bool x64, int64_t K, int64_t N, int64_t ldx, int steps, const uint8_t* excluded,
                int64_t* piv, int* status, void* ws, size_t ws_bytes, hipStream_t st, double rel_cut) {
  if (steps < 1 || steps > K) return arg_error("qrcp: need 1 <= steps <= K");
  if (K > kMaxK) return arg_error("qrcp: K above 4096 is not supported");
  if (N < 1 || ldx < N || N > INT_MAX) return arg_error("qrcp: need 1 <= N < 2^31 and ldx >= N");
  if (!(rel_cut >= 0.0 && rel_cut < 1.0)) return arg_error("qrcp: need 0 <= rel_cut < 1");
  DeviceInfo dev;
  ICUR_TRY(device_info(&dev));
  const int groups = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((N + kQT - 1) / kQT, 4 * dev.num_cus)));
  if (qrcp_workspace_bytes(K, N, groups) > ws_bytes) return arg_error("qrcp: workspace too small");
  char* p = static_cast<char*>(ws);
  QrcpArgs a;
  a.X = X;
  a.ldx = ldx;
  a.K = static_cast<int>(K);
  a.N = static_cast<int>(N);
  a.excl = excluded;
  a.Xw = reinterpret_cast<double*>(p);
  p += al256(static_cast<size_t>(K) * N * 8);
  a.q = reinterpret_cast<double*>(p);
  p += al256(static_cast<size_t>(K) * 8);
  a.pval = reinterpret_cast<double*>(p);
  p += al256(groups * 8);
  a.pidx = reinterpret_cast<int*>(p);
  p += al256(groups * 4);
  a.chosen = reinterpret_cast<uint8_t*>(p);
  p += al256(static_cast<size_t>(N));
  a.ref = reinterpret_cast<double*>(p);
  a.status = status;
  a.piv = piv;
  a.rel_cut2 = rel_cut * rel_cut;
  ICUR_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(status), 3, 0u, st));
  for (int t = 0; t < steps; ++t) {
    a.t = t;
    if (x64)
      hipLaunchKernelGGL(qrcp_update<1>, dim3(groups), dim3(kQT), 0, st, a);
    else
      hipLaunchKernelGGL(qrcp_update<0>, dim3(groups), dim3(kQT), 0, st, a);
    hipLaunchKernelGGL(qrcp_pick, dim3(1), dim3(kQT), 0, st, a, groups);
  }
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

}  // namespace icur
