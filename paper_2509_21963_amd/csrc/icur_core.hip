// FP64 kernels for the core U = A(I,J)^{-1} of Alg. 1 and the small products around it.
//
// The core is grown block by block with the block inverse used in the proof of the
// residual-recurrence lemma (§4.2): with the old core A11 = A(I,J) (inverse U known),
// the new block A12 = A(I,J_k), A21 = A(I_k,J), A22 = A(I_k,J_k), Y = U A12,
// Z = A21 U and the Schur complement N = A22 - A21 Y (the residual at the new rows and
// columns),
//     [A11 A12; A21 A22]^{-1} = [U + Y N^-1 Z, -Y N^-1; -N^-1 Z, N^-1].
// This costs O(r^2 b) per iteration instead of refactorising the r x r core (the paper
// notes the update alternative in §3.4).  N^-1 comes from Gauss-Jordan elimination with
// partial pivoting in one workgroup.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include <utility>

#include <map>
#include <memory>
#include <mutex>

#include <rocblas/rocblas.h>

#include "icur_internal.h"
#include "icur_gj.h"
#include "icur_wave.h"

namespace icur {
namespace {

constexpr int kTM = 64, kTN = 64, kTK = 16;

// C = alpha A B + beta C, 64x64 tiles, 256 threads each computing a 4x4 block.
__global__ __launch_bounds__(256) void dgemm_kernel(int64_t M, int64_t N, int64_t K, double alpha,
                                                    const double* __restrict__ A, int64_t sa0,
                                                    int64_t sa1, const double* __restrict__ B,
                                                    int64_t sb0, int64_t sb1, double beta,
                                                    double* __restrict__ C, int64_t ldc) {
  __shared__ double As[kTK][kTM + 1];
  __shared__ double Bs[kTK][kTN + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int64_t row0 = static_cast<int64_t>(blockIdx.y) * kTM;
  const int64_t col0 = static_cast<int64_t>(blockIdx.x) * kTN;
  double acc[4][4] = {};
  for (int64_t k0 = 0; k0 < K; k0 += kTK) {
    for (int e = threadIdx.x; e < kTM * kTK; e += 256) {
      // A tile: choose the mapping that walks A's unit-stride dimension across threads
      int i, kk;
      if (sa1 == 1) {
        i = e / kTK;
        kk = e % kTK;
      } else {
        kk = e / kTM;
        i = e % kTM;
      }
      const int64_t gi = row0 + i, gk = k0 + kk;
      As[kk][i] = (gi < M && gk < K) ? A[gi * sa0 + gk * sa1] : 0.0;
    }
    for (int e = threadIdx.x; e < kTK * kTN; e += 256) {
      int kk, j;
      if (sb1 == 1) {
        kk = e / kTN;
        j = e % kTN;
      } else {
        j = e / kTK;
        kk = e % kTK;
      }
      const int64_t gk = k0 + kk, gj = col0 + j;
      Bs[kk][j] = (gk < K && gj < N) ? B[gk * sb0 + gj * sb1] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kTK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[kk][ty + 16 * u];
        b[u] = Bs[kk][tx + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t gi = row0 + ty + 16 * u;
    if (gi >= M) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t gj = col0 + tx + 16 * v;
      if (gj >= N) continue;
      double* c = C + gi * ldc + gj;
      *c = alpha * acc[u][v] + (beta == 0.0 ? 0.0 : beta * *c);
    }
  }
}

__global__ void identity_kernel(double* U, int64_t r) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e < r * r) U[e] = (e / r == e % r) ? 1.0 : 0.0;
}

__global__ void dcopy2d_kernel(int64_t M, int64_t N, double alpha, const double* __restrict__ src,
                               int64_t lds, double* __restrict__ dst, int64_t ldd) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  const int64_t i = e / N, j = e % N;
  dst[i * ldd + j] = alpha * src[i * lds + j];
}

// In-place inverse of the k x k matrix N by Gauss-Jordan elimination with partial
// pivoting (row interchanges, undone as column interchanges at the end).  One workgroup
// of 1024 threads: thread t owns column t % k of the rows t / k, t / k + g, ... (g row
// groups), so every elimination sweep is coalesced in LDS and needs no division.
__global__ __launch_bounds__(1024) void gj_inverse_kernel(double* __restrict__ Ng, int k, int use_lds,
                                                          double* __restrict__ work,
                                                          int* __restrict__ info,
                                                          double* __restrict__ norms) {
  extern __shared__ double sm[];
  __shared__ int perm[512];
  __shared__ double fcol[512];
  __shared__ double prow[512];
  __shared__ double red_v[16];
  __shared__ int red_i[16];
  __shared__ int bp;
  __shared__ double bpv;
  double* a = use_lds ? sm : work;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  const int ng = nt / k;                      // row groups (>= 2 for k <= 512)
  const int col = tid % k, grp = tid / k;     // this thread's column and row group
  const bool active = grp < ng;
  for (int e = tid; e < k * k; e += nt) a[e] = Ng[e];
  __syncthreads();
  auto colnorm_max = [&](int slot) {
    if (norms == nullptr) return;  // uniform
    double cs = 0.0;
    if (tid < k) {
      double s = 0.0;
      for (int i = 0; i < k; ++i) s += fabs(a[i * k + tid]);
      cs = s;
    }
    for (int off = 32; off > 0; off >>= 1) cs = fmax(cs, __shfl_xor(cs, off, 64));
    if (lane == 0) red_v[wave] = cs;
    __syncthreads();
    if (tid == 0) {
      double m = 0.0;
      for (int w = 0; w < nw; ++w) m = fmax(m, red_v[w]);
      norms[slot] = m;
    }
    __syncthreads();
  };
  colnorm_max(0);
  for (int j = 0; j < k; ++j) {
    // pivot: largest |a[i][j]| over rows i >= j, lowest index on ties
    double bv = -1.0;
    int bi = 0x7fffffff;
    for (int i = j + tid; i < k; i += nt) {
      const double v = fabs(a[i * k + j]);
      if (v > bv || (v == bv && i < bi)) {
        bv = v;
        bi = i;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_xor(bv, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      red_v[wave] = bv;
      red_i[wave] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double gv = red_v[0];
      int gi = red_i[0];
      for (int w = 1; w < nw; ++w)
        if (red_v[w] > gv || (red_v[w] == gv && red_i[w] < gi)) {
          gv = red_v[w];
          gi = red_i[w];
        }
      bp = gi;
      bpv = gv;
      perm[j] = gi;
    }
    __syncthreads();
    if (!(bpv > 0.0)) {
      if (tid == 0) *info = 1;
      return;
    }
    const int p = bp;
    // swap rows j and p, then scale the pivot row; keep column j and the pivot row
    if (tid < k) {
      double rj = a[j * k + tid], rp = a[p * k + tid];
      if (p != j) {
        a[j * k + tid] = rp;
        a[p * k + tid] = rj;
        rj = rp;
      }
      prow[tid] = rj;
    }
    __syncthreads();
    const double pinv = 1.0 / prow[j];
    if (tid < k) {
      fcol[tid] = (tid == j) ? 0.0 : a[tid * k + j];
      const double v = (tid == j) ? pinv : prow[tid] * pinv;
      a[j * k + tid] = v;
    }
    __syncthreads();
    if (tid < k) prow[tid] = a[j * k + tid];
    __syncthreads();
    // eliminate column j from every other row
    if (active) {
      const double pc = prow[col];
      const bool isj = (col == j);
      for (int i = grp; i < k; i += ng) {
        if (i == j) continue;
        const double f = fcol[i];
        double* e = a + i * k + col;
        *e = isj ? -f * pc : *e - f * pc;
      }
    }
    __syncthreads();
  }
  for (int j = k - 1; j >= 0; --j) {
    const int p = perm[j];
    if (p != j)
      for (int i = tid; i < k; i += nt) {
        const double t = a[i * k + j];
        a[i * k + j] = a[i * k + p];
        a[i * k + p] = t;
      }
    __syncthreads();
  }
  for (int e = tid; e < k * k; e += nt) Ng[e] = a[e];
  colnorm_max(1);
  if (tid == 0) *info = 0;
}

template <class F, int... I>
__device__ __forceinline__ void tile_static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void tile_static_for(F&& f) {
  tile_static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Gauss-Jordan inverse of a k x k block, k <= 128, in one workgroup of four waves (one
// per SIMD, so no wave repeats another's work on a shared SIMD).  Thread (tr, tc) of a
// 16 x 16 grid holds the 8 x 8 tile at rows 8 tr, columns 8 tc in registers.  Pivoting
// is implicit (no row swaps): step j takes the unused row p with the largest |a(p, j)|,
// lowest index on ties, and eliminates column j from every other row; the final write
// undoes the permutation (inverse(j, p_c) = storage(p_j, c)).  Per step the tile column
// holding column j publishes that column and its per-tile best rows, every wave reduces
// the 16 candidates, the tile row holding row p publishes that row, and every thread
// updates its tile: two barriers per step.
__global__ __launch_bounds__(256) void gj_inverse_tile_kernel(double* __restrict__ Ng, int k, int* __restrict__ info) {
  __shared__ double colj[2][128];
  __shared__ double prow[2][128];
  __shared__ Red red[2][16];
  __shared__ int perm[128];  // perm[j] = p_j
  __shared__ int pinv[128];  // pinv[p_j] = j
  const int tid = threadIdx.x, lane = tid & 63;
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
  unsigned used = 0;  // bit i: row r0 + i was a pivot
  // Steps go eight at a time so that the column inside a tile is a compile-time index;
  // the pivot row inside its tile is wave-uniform, so it is chosen by uniform branches.
  for (int j0 = 0; j0 < k; j0 += 8) {
    const int tj = j0 >> 3;
    bool fail = false;
    tile_static_for<8>([&](auto jcc) __attribute__((always_inline)) {
      constexpr int jc = decltype(jcc)::value;
      const int j = j0 + jc;
      if (fail || j >= k) return;
      const int b = j & 1;
      // (1) tile column tj publishes column j and its best unused row
      if (tc == tj) {
        unsigned long long bk = 0ull;
        int bi = INT_MAX;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const double v = a[i][jc];
          colj[b][r0 + i] = v;
          const unsigned long long kk = (((used >> i) & 1u) || r0 + i >= k) ? 0ull : cand_key(fabs(v));
          if (kk > bk) {  // rows increase with i: ties keep the lower row
            bk = kk;
            bi = r0 + i;
          }
        }
        red[b][tr] = Red{bk, bi, 0};
      }
      __syncthreads();
      // (2) every wave reduces the 16 candidates (lane l < 16 reads slot l)
      unsigned long long sk = 0ull;
      int si = INT_MAX;
      if (lane < 16) {
        const Red rr = red[b][lane];
        sk = rr.k;
        si = rr.i;
      }
      unsigned long long gk;
      int p, gw;
      wave_argmax(sk, si, 0, &gk, &p, &gw);
      if (gk == 0ull) {  // uniform: every wave reduced the same slots
        fail = true;
        return;
      }
      const int tp = p >> 3, ip = p & 7;
      if (tr == tp) {
        switch (ip) {
#define ICUR_GJ_PUB(I)                                                    \
  case I:                                                                 \
    for (int jj = 0; jj < 8; ++jj) prow[b][c0 + jj] = a[I][jj];           \
    break;
          ICUR_GJ_PUB(0) ICUR_GJ_PUB(1) ICUR_GJ_PUB(2) ICUR_GJ_PUB(3)
          ICUR_GJ_PUB(4) ICUR_GJ_PUB(5) ICUR_GJ_PUB(6) ICUR_GJ_PUB(7)
#undef ICUR_GJ_PUB
        }
        used |= 1u << ip;
      }
      if (tid == 0) {
        perm[j] = p;
        pinv[p] = j;
      }
      __syncthreads();
      // (3) a(i, c) -= a(i, j) a(p, c) / piv for all rows; then column j becomes
      //     -a(i, j) / piv and row p becomes a(p, c) / piv (1 / piv at column j)
      const double rinv = 1.0 / colj[b][p];
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
      if (tr == tp) {
        switch (ip) {
#define ICUR_GJ_ROW(I)                                                    \
  case I:                                                                 \
    for (int jj = 0; jj < 8; ++jj) a[I][jj] = pr[jj];                     \
    if (tc == tj) a[I][jc] = rinv;                                        \
    break;
          ICUR_GJ_ROW(0) ICUR_GJ_ROW(1) ICUR_GJ_ROW(2) ICUR_GJ_ROW(3)
          ICUR_GJ_ROW(4) ICUR_GJ_ROW(5) ICUR_GJ_ROW(6) ICUR_GJ_ROW(7)
#undef ICUR_GJ_ROW
        }
      }
    });
    if (fail) {
      if (tid == 0) *info = 1;
      return;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int jj = 0; jj < 8; ++jj) {
      const int r = r0 + i, c = c0 + jj;
      if (r < k && c < k) Ng[pinv[r] * k + perm[c]] = a[i][jj];
    }
  if (tid == 0) *info = 0;
}

// The in-order Gauss-Jordan inverse (icur_gj.h) for one block.
__global__ __launch_bounds__(256) void gj_inverse_inorder_kernel(double* __restrict__ Ng, int k,
                                                                 int* __restrict__ info) {
  gj_inorder_tile(Ng, k, info);
}

// The same, leaving *info alone unless the block is singular (the blocked inverse runs
// several and reports any failure).
__global__ __launch_bounds__(256) void gj_inverse_inorder_sticky_kernel(double* __restrict__ Ng, int k,
                                                                        int* __restrict__ info) {
  __shared__ int flag;
  gj_inorder_tile(Ng, k, &flag);
  __syncthreads();
  if (threadIdx.x == 0 && flag != 0) *info = 1;
}

}  // namespace

namespace {
// rocBLAS handles, one per (device, stream), kept for the life of the process (or until
// icur_release): the batched workers reuse theirs call after call.  Each handle has a
// mutex held across set_stream and the product, so threads sharing a stream cannot
// interleave on it.  Atomics off so that every product is reproducible run to run.
struct BlasEntry {
  rocblas_handle h = nullptr;
  std::mutex mu;
};
std::mutex g_blas_mu;
std::map<std::pair<int, hipStream_t>, std::unique_ptr<BlasEntry>> g_blas;

int blas_entry(hipStream_t st, BlasEntry** out) {
  int dev = 0;
  ICUR_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_blas_mu);
  auto& e = g_blas[{dev, st}];
  if (!e) {
    std::unique_ptr<BlasEntry> ne(new BlasEntry());
    if (rocblas_create_handle(&ne->h) != rocblas_status_success) {
      g_blas.erase({dev, st});
      set_error("rocblas_create_handle failed");
      return ICUR_ERR_HIP;
    }
    rocblas_set_atomics_mode(ne->h, rocblas_atomics_not_allowed);
    e = std::move(ne);
  }
  *out = e.get();
  return ICUR_OK;
}
}  // namespace

void release_blas_handles() {
  std::lock_guard<std::mutex> g(g_blas_mu);
  for (auto& kv : g_blas) {
    std::lock_guard<std::mutex> l(kv.second->mu);
    if (kv.second->h) rocblas_destroy_handle(kv.second->h);
    kv.second->h = nullptr;
  }
  g_blas.clear();
}

int dgemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t sa0,
          int64_t sa1, const double* B, int64_t sb0, int64_t sb1, double beta, double* C,
          int64_t ldc, hipStream_t st) {
  if (M <= 0 || N <= 0) return ICUR_OK;
  // ICUR_NATIVE_GEMM=1: the row-major products on this library's own FP64 matrix-core
  // kernel instead of rocBLAS (about 20% slower on the deep residual products of the
  // 30000^2 rank-2000 run: 12.1 ms against 10.0 ms per call)
  const char* nat = std::getenv("ICUR_NATIVE_GEMM");
  if (nat && nat[0] == '1' && sa1 == 1 && sb1 == 1 && K > 0 && (beta == 0.0 || beta == 1.0))
    return gemm_f64_native(M, N, K, alpha, A, sa0, B, sb0, beta == 1.0 ? C : nullptr, ldc, C, ldc, st);
  // Row-major operands with unit column strides are a plain library GEMM: the
  // column-major product C^T = alpha B^T A^T + beta C^T on FP64 matrix cores.
  if (sa1 == 1 && sb1 == 1 && K > 0 && M <= INT32_MAX && N <= INT32_MAX && K <= INT32_MAX && sa0 <= INT32_MAX &&
      sb0 <= INT32_MAX && ldc <= INT32_MAX) {
    BlasEntry* be;
    ICUR_TRY(blas_entry(st, &be));
    std::lock_guard<std::mutex> l(be->mu);
    rocblas_handle h = be->h;
    if (rocblas_set_stream(h, st) != rocblas_status_success ||
        rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, static_cast<rocblas_int>(N),
                      static_cast<rocblas_int>(M), static_cast<rocblas_int>(K), &alpha, B,
                      static_cast<rocblas_int>(sb0), A, static_cast<rocblas_int>(sa0), &beta, C,
                      static_cast<rocblas_int>(ldc)) != rocblas_status_success) {
      set_error("rocblas_dgemm failed");
      return ICUR_ERR_HIP;
    }
    return ICUR_OK;
  }
  if ((N + kTN - 1) / kTN > 0x7fffffff || (M + kTM - 1) / kTM > 65535)
    return arg_error("dgemm: matrix too large");
  dim3 grid(static_cast<unsigned>((N + kTN - 1) / kTN), static_cast<unsigned>((M + kTM - 1) / kTM));
  hipLaunchKernelGGL(dgemm_kernel, grid, dim3(256), 0, st, M, N, K, alpha, A, sa0, sa1, B, sb0, sb1,
                     beta, C, ldc);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

int dcopy2d(int64_t M, int64_t N, double alpha, const double* src, int64_t lds, double* dst,
            int64_t ldd, hipStream_t st) {
  if (M <= 0 || N <= 0) return ICUR_OK;
  const int64_t total = M * N;
  hipLaunchKernelGGL(dcopy2d_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, st,
                     M, N, alpha, src, lds, dst, ldd);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

int launch_fill_f64_identity(double* U, int64_t r, hipStream_t st) {
  if (r <= 0) return ICUR_OK;
  const int64_t total = r * r;
  hipLaunchKernelGGL(identity_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, st, U, r);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

// max |R| over an r x r matrix into *out (zeroed by the caller): non-negative doubles
// order as their bit patterns, so an integer atomic max of the bits is the maximum.
__global__ __launch_bounds__(256) void maxabs_kernel(const double* __restrict__ R, int64_t total,
                                                     unsigned long long* __restrict__ out) {
  double m = 0.0;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * 256)
    m = fmax(m, fabs(R[e]));
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, static_cast<unsigned long long>(__double_as_longlong(m)));
}

// U += T when the refinement converges (max |I - M U| below 1/2), else U is left alone.
__global__ __launch_bounds__(256) void refine_apply_kernel(double* __restrict__ U, const double* __restrict__ T,
                                                           int64_t total, const unsigned long long* __restrict__ rmax) {
  if (__longlong_as_double(static_cast<long long>(*rmax)) >= 0.5) return;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * 256)
    U[e] += T[e];
}

// The general kernel's work (k^2) and the blocked in-order inverse's (under 3 k^2).
size_t small_inverse_work_bytes(int64_t k) { return 3 * static_cast<size_t>(k) * k * sizeof(double); }

int launch_small_inverse(double* N, int64_t k, double* work, int* info, double* norms,
                         hipStream_t st) {
  if (k < 1 || k > 512) return arg_error("inverse: block size must be in 1..512");
  if (k <= 128 && norms == nullptr) {
    hipLaunchKernelGGL(gj_inverse_tile_kernel, dim3(1), dim3(256), 0, st, N, static_cast<int>(k), info);
    ICUR_HIP(hipGetLastError());
    return ICUR_OK;
  }
  const bool use_lds = k <= 128;
  const size_t shmem = use_lds ? static_cast<size_t>(k) * k * sizeof(double) : 0;
  if (shmem > 64 * 1024)
    ICUR_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(gj_inverse_kernel),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shmem)));
  hipLaunchKernelGGL(gj_inverse_kernel, dim3(1), dim3(1024), shmem, st, N, static_cast<int>(k),
                     use_lds ? 1 : 0, work, info, norms);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

// In-order inverse of a k x k block (rows in partial-pivoting order, ld k) for k > 128:
// 2 x 2 block elimination on a leading block of 128 (the in-order Gauss-Jordan tile),
// the trailing Schur complement S = D - C A^{-1} B inverted the same way (it is the next
// stage of the same LU), and the four blocks of the inverse formed by FP64 products:
// [A^{-1} + A^{-1} B S^{-1} C A^{-1}, -A^{-1} B S^{-1}; -S^{-1} C A^{-1}, S^{-1}].
// work: under 3 k^2 doubles.  *info must be 0 on entry; set to 1 on a zero pivot.
int blocked_inorder_inverse(double* N, int64_t k, double* work, int* info, hipStream_t st) {
  constexpr int64_t h = 128;
  const int64_t t = k - h;
  double* Ai = work;         // h x h: A^{-1}
  double* X = Ai + h * h;    // t x h: C A^{-1}
  double* S = X + t * h;     // t x t: D - X B, then its inverse
  double* Y = S + t * t;     // h x t: A^{-1} B
  double* Z = Y + h * t;     // t x h: S^{-1} X
  double* rest = Z + t * h;  // the trailing inverse's own work
  ICUR_TRY(dcopy2d(h, h, 1.0, N, k, Ai, h, st));
  hipLaunchKernelGGL(gj_inverse_inorder_sticky_kernel, dim3(1), dim3(256), 0, st, Ai, static_cast<int>(h), info);
  ICUR_HIP(hipGetLastError());
  ICUR_TRY(gemm_f64_native(t, h, h, 1.0, N + h * k, k, Ai, h, nullptr, 0, X, h, st));
  ICUR_TRY(gemm_f64_native(t, t, h, -1.0, X, h, N + h, k, N + h * k + h, k, S, t, st));
  if (t <= h) {
    hipLaunchKernelGGL(gj_inverse_inorder_sticky_kernel, dim3(1), dim3(256), 0, st, S, static_cast<int>(t), info);
    ICUR_HIP(hipGetLastError());
  } else {
    ICUR_TRY(blocked_inorder_inverse(S, t, rest, info, st));
  }
  ICUR_TRY(gemm_f64_native(h, t, h, 1.0, Ai, h, N + h, k, nullptr, 0, Y, t, st));
  ICUR_TRY(gemm_f64_native(t, h, t, 1.0, S, t, X, h, nullptr, 0, Z, h, st));
  ICUR_TRY(gemm_f64_native(h, h, t, 1.0, Y, t, Z, h, Ai, h, N, k, st));
  ICUR_TRY(gemm_f64_native(h, t, t, -1.0, Y, t, S, t, nullptr, 0, N + h, k, st));
  ICUR_TRY(dcopy2d(t, h, -1.0, Z, h, N + h * k, k, st));
  ICUR_TRY(dcopy2d(t, t, 1.0, S, t, N + h * k + h, k, st));
  return ICUR_OK;
}

int launch_inorder_inverse(double* N, int64_t k, double* work, int* info, hipStream_t st) {
  if (k >= 1 && k <= 128) {
    hipLaunchKernelGGL(gj_inverse_inorder_kernel, dim3(1), dim3(256), 0, st, N, static_cast<int>(k), info);
    ICUR_HIP(hipGetLastError());
    return ICUR_OK;
  }
  if (k < 1 || k > 512) return arg_error("inverse: block size must be in 1..512");
  ICUR_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(info), 1, 0u, st));
  return blocked_inorder_inverse(N, k, work, info, st);
}

// U (ldu) grows from r x r to (r+k) x (r+k).  ws must hold k*k + 2*k*r + k*k doubles.
int core_update(double* U, int64_t ldu, int64_t r, int64_t k, const double* Y, int64_t ldy,
                const double* A21, const double* A22, double* ws, int* info, double* norms,
                hipStream_t st) {
  double* Nw = ws;                // k x k
  double* Z = Nw + k * k;         // k x r
  double* V = Z + k * r;          // r x k
  double* gjw = V + r * k;        // k x k (Gauss-Jordan work when k > 128)
  ICUR_TRY(dcopy2d(k, k, 1.0, A22, k, Nw, k, st));
  if (r > 0) ICUR_TRY(dgemm(k, k, r, -1.0, A21, r, 1, Y, ldy, 1, 1.0, Nw, k, st));
  ICUR_TRY(launch_small_inverse(Nw, k, gjw, info, norms, st));
  if (r > 0) {
    ICUR_TRY(dgemm(k, r, r, 1.0, A21, r, 1, U, ldu, 1, 0.0, Z, r, st));      // Z = A21 U
    ICUR_TRY(dgemm(r, k, k, 1.0, Y, ldy, 1, Nw, k, 1, 0.0, V, k, st));      // V = Y N^-1
    ICUR_TRY(dgemm(r, r, k, 1.0, V, k, 1, Z, r, 1, 1.0, U, ldu, st));       // U += V Z
    ICUR_TRY(dcopy2d(r, k, -1.0, V, k, U + r, ldu, st));                    // U12 = -V
    ICUR_TRY(dgemm(k, r, k, -1.0, Nw, k, 1, Z, r, 1, 0.0, U + r * ldu, ldu, st));  // U21
  }
  ICUR_TRY(dcopy2d(k, k, 1.0, Nw, k, U + r * ldu + r, ldu, st));            // U22 = N^-1
  return ICUR_OK;
}

size_t core_update_ws_doubles(int64_t r, int64_t k) { return 2 * k * k + 2 * k * r; }

// U = M^{-1} for the r x r cross M = A(I,J) (FP64, ld r, overwritten), by block LU in the
// selection order (diagonal blocks are the Schur complements N_k the row selection
// pivoted on, each inverted by Gauss-Jordan with partial pivoting) followed by block
// forward and back substitution on the identity.  U (ld r) receives the inverse.
// ws holds core_inverse_ws_doubles(r, bmax) doubles.
int core_block_inverse(double* M, int64_t r, const int64_t* blocks, int64_t nblocks, int64_t bmax, double* U,
                       double* ws, int* info, double* norms, hipStream_t st, const double* D0inv) {
  double* Dinv = ws;                           // r x bmax: the diagonal block inverses, stacked
  double* T = Dinv + r * bmax;                 // bmax x r temporary
  double* gjw = T + bmax * r;                  // bmax x bmax Gauss-Jordan work
  if (D0inv && nblocks == 1 && norms == nullptr) {
    ICUR_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(info), 1, 0u, st));
    ICUR_HIP(hipMemcpyAsync(U, D0inv, static_cast<size_t>(r) * r * 8, hipMemcpyDeviceToDevice, st));
    return ICUR_OK;
  }
  // block LU: M = L~ U~ with L~ unit block lower (stored below the diagonal blocks)
  int64_t q = 0;
  for (int64_t k = 0; k < nblocks; ++k) {
    const int64_t nk = blocks[k];
    double* Dk = Dinv + q * bmax;              // nk x nk, ld nk
    if (k == 0 && D0inv && norms == nullptr) {
      ICUR_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(info), 1, 0u, st));
      ICUR_HIP(hipMemcpyAsync(Dk, D0inv, static_cast<size_t>(nk) * nk * 8, hipMemcpyDeviceToDevice, st));
    } else {
      ICUR_TRY(dcopy2d(nk, nk, 1.0, M + q * r + q, r, Dk, nk, st));
      // the diagonal blocks are Schur complements in selection order: partial-pivoting
      // order already (unless a norm estimate is asked for, which the general kernel makes)
      if (norms == nullptr)
        ICUR_TRY(launch_inorder_inverse(Dk, nk, gjw, info + k, st));
      else
        ICUR_TRY(launch_small_inverse(Dk, nk, gjw, info + k, norms, st));
    }
    const int64_t rest = r - q - nk;
    if (rest > 0) {
      // L~ panel: M[q+nk:, q:q+nk] <- M[q+nk:, q:q+nk] D_k^{-1}   (via T, rest x nk)
      ICUR_TRY(dgemm(rest, nk, nk, 1.0, M + (q + nk) * r + q, r, 1, Dk, nk, 1, 0.0, T, nk, st));
      ICUR_TRY(dcopy2d(rest, nk, 1.0, T, nk, M + (q + nk) * r + q, r, st));
      // trailing update: M[q+nk:, q+nk:] -= L~ panel * M[q:q+nk, q+nk:]
      ICUR_TRY(dgemm(rest, rest, nk, -1.0, M + (q + nk) * r + q, r, 1, M + q * r + q + nk, r, 1, 1.0,
                     M + (q + nk) * r + q + nk, r, st));
    }
    q += nk;
  }
  // forward: U <- L~^{-1} (block unit lower), row block by row block
  ICUR_TRY(launch_fill_f64_identity(U, r, st));
  q = 0;
  for (int64_t k = 0; k < nblocks; ++k) {
    const int64_t nk = blocks[k];
    if (q > 0)
      ICUR_TRY(dgemm(nk, q, q, -1.0, M + q * r, r, 1, U, r, 1, 0.0, U + q * r, r, st));
    q += nk;
  }
  // back: U <- U~^{-1} U, row blocks from the last
  for (int64_t k = nblocks - 1; k >= 0; --k) {
    const int64_t nk = blocks[k];
    q -= nk;
    const int64_t rest = r - q - nk;
    ICUR_TRY(dcopy2d(nk, r, 1.0, U + q * r, r, T, r, st));
    if (rest > 0)
      ICUR_TRY(dgemm(nk, r, rest, -1.0, M + q * r + q + nk, r, 1, U + (q + nk) * r, r, 1, 1.0, T, r, st));
    ICUR_TRY(dgemm(nk, r, nk, 1.0, Dinv + q * bmax, nk, 1, T, r, 1, 0.0, U + q * r, r, st));
  }
  return ICUR_OK;
}

// Newton steps on the core: U <- U + U (I - M U), M the cross A(I,J) (ld r).  The block
// LU in selection order pivots only within the blocks, so on ill-conditioned crosses its
// inverse can carry far more error than a fully pivoted one (the CUR error with it can
// exceed the tolerance while A(I,J)^+ meets it).  The residual R = I - M U squares with
// every step, down to its own rounding (near cond 2^-52).  Up to three steps, each taken
// only while max |R| is below 1/2 (convergence), above `floor` (still worth a step: the
// CUR error it can add is about max |R| relative) and at most half the previous one
// (still shrinking); the host reads max |R| before each.  ws: 2 r^2 + 1 doubles.
int core_refine(const double* M, double* U, int64_t r, double floor, double* ws, hipStream_t st) {
  if (r <= 0) return ICUR_OK;
  double* R = ws;
  double* T = ws + r * r;
  unsigned long long* rmax = reinterpret_cast<unsigned long long*>(T + r * r);
  const int64_t total = r * r;
  const unsigned blocks = static_cast<unsigned>(std::min<int64_t>((total + 255) / 256, 1024));
  double prev = 1.0;
  for (int step = 0; step < 3; ++step) {
    ICUR_TRY(launch_fill_f64_identity(R, r, st));
    ICUR_TRY(dgemm(r, r, r, -1.0, M, r, 1, U, r, 1, 1.0, R, r, st));
    ICUR_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(rmax), 2, 0u, st));
    hipLaunchKernelGGL(maxabs_kernel, dim3(blocks), dim3(256), 0, st, R, total, rmax);
    ICUR_HIP(hipGetLastError());
    unsigned long long bits = 0;
    ICUR_HIP(hipMemcpyAsync(&bits, rmax, sizeof(bits), hipMemcpyDeviceToHost, st));
    ICUR_HIP(hipStreamSynchronize(st));
    double v;
    std::memcpy(&v, &bits, sizeof(v));
    if (!(v < 0.5) || v <= floor || v > 0.5 * prev) break;
    prev = v;
    ICUR_TRY(dgemm(r, r, r, 1.0, U, r, 1, R, r, 1, 0.0, T, r, st));
    hipLaunchKernelGGL(refine_apply_kernel, dim3(blocks), dim3(256), 0, st, U, T, total, rmax);
    ICUR_HIP(hipGetLastError());
  }
  return ICUR_OK;
}

size_t core_refine_ws_doubles(int64_t r) { return 2 * r * r + 1; }

size_t core_inverse_ws_doubles(int64_t r, int64_t bmax) { return r * bmax + bmax * r + 3 * bmax * bmax; }

}  // namespace icur
