// Gauss-Jordan inverse of a pivot block whose rows are in partial-pivoting order, as a
// device function for one workgroup of 256 threads (shared by the single-matrix core
// kernels and the grouped kernels of the batched form).
#pragma once

#include <hip/hip_runtime.h>

#include <utility>

namespace icur {

template <class F, int... I>
__device__ __forceinline__ void gj_static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void gj_static_for(F&& f) {
  gj_static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Inverse of a k x k block, k <= 128, whose rows are already in partial-pivoting order: the
// pivot block N_k of a row selection (rows I_k in selection order, columns J_k) is the
// leading part of an LU with partial pivoting, so eliminating on the diagonal in order
// keeps every multiplier within 1 and needs no pivot search.  Per step the tile column
// and the tile row holding column and row j publish them, one barrier, then the update.
// A zero pivot reports info = 1.
__device__ __forceinline__ void gj_inorder_tile(double* __restrict__ Ng, int k, int* __restrict__ info) {
  __shared__ double colj[2][128];
  __shared__ double prow[2][128];
  const int tid = threadIdx.x;
  const int tr = tid >> 4, tc = tid & 15;
  const int r0 = 8 * tr, c0 = 8 * tc;
  double a[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const int r = r0 + i, c = c0 + jj;
      a[i][jj] = (r < k && c < k) ? Ng[r * k + c] : 0.0;
    }
  for (int j0 = 0; j0 < k; j0 += 8) {
    const int tj = j0 >> 3;
    bool fail = false;
    gj_static_for<8>([&](auto jcc) __attribute__((always_inline)) {
      constexpr int jc = decltype(jcc)::value;
      const int j = j0 + jc;
      if (fail || j >= k) return;
      const int b = j & 1;
      if (tc == tj) {
#pragma unroll
        for (int i = 0; i < 8; ++i) colj[b][r0 + i] = a[i][jc];
      }
      if (tr == tj) {
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) prow[b][c0 + jj] = a[jc][jj];
      }
      __syncthreads();
      const double piv = colj[b][j];
      if (piv == 0.0) {  // uniform: every thread read the same word
        fail = true;
        return;
      }
      const double rinv = 1.0 / piv;
      double pr[8], f[8];
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) pr[jj] = prow[b][c0 + jj] * rinv;
#pragma unroll
      for (int i = 0; i < 8; ++i) f[i] = colj[b][r0 + i];
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) a[i][jj] = a[i][jj] - f[i] * pr[jj];
      if (tc == tj) {
#pragma unroll
        for (int i = 0; i < 8; ++i) a[i][jc] = -f[i] * rinv;
      }
      if (tr == tj) {
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) a[jc][jj] = pr[jj];
        if (tc == tj) a[jc][jc] = rinv;
      }
    });
    if (fail) {
      if (tid == 0) *info = 1;
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const int r = r0 + i, c = c0 + jj;
      if (r < k && c < k) Ng[r * k + c] = a[i][jj];
    }
  if (tid == 0) *info = 0;
}


}  // namespace icur
