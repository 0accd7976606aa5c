// Host side of the wide products OUT(M x N) = X - W(M x K) B(K x N) (kernels in
// icur_wide_kernel.h).  All dense contractions of the IterativeCUR loop have this shape:
//   initial sketch             G A                        M = c, K = m, N = n
//   row residual (transposed)  A(:,J_k)^T - Ur(:,J_k)^T Lc^T     M = b, K = r, N = m
//   residual at the new rows   A(I_k,:) - Lc(I_k,:) Ur    M = b, K = r, N = n
//   new row factors            N_k^{-1} S(I_k,:)          M = b, K = b, N = n
//   sketched residual update   S - S(:,J_k) Ur_k          M = c, K = b, N = n
// With FP64 factors (tight tolerances) the same products run on the FP64 matrix cores.
// This file chooses the tile (rows per tile group, columns per workgroup) and the split
// of K across workgroups, and launches the fixed-order reduction of the split partials.
#include <algorithm>

#include "icur_internal.h"
#include "icur_wide_kernel.h"

namespace icur {
namespace {

using wide::kKC;
using wide::kMaxMT;
using wide::kWaves;

constexpr int64_t kMinColsPerBlock = 16 * 1 * kWaves;

int64_t cols_per_block(int mt, bool f64) { return 16 * wide::ns_for(mt, f64) * kWaves; }

// Split-K factor: enough workgroups to cover the chip ~4 times, each split a multiple of
// the K chunk with at least 8 chunks, at most 64 splits.
int choose_splits(int64_t K, int64_t N, int num_cus, int64_t cpb) {
  const int64_t nblk = (N + cpb - 1) / cpb;
  const int64_t chunks = (K + kKC - 1) / kKC;
  int64_t want = (4 * static_cast<int64_t>(num_cus) + nblk - 1) / nblk;
  want = std::min<int64_t>(want, std::max<int64_t>(1, chunks / 8));
  want = std::min<int64_t>(want, 64);
  return static_cast<int>(std::max<int64_t>(1, want));
}

__global__ __launch_bounds__(256) void reduce_partials_kernel(const double* partials, int n, double* out) {
  __shared__ double red[4];
  double s = 0.0;
  // fixed assignment and order: thread t sums partials t, t+256, ...
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += partials[i];
  s = wide::block_sum_f64(s, red);
  if (threadIdx.x == 0) *out = s;
}

__global__ void split_f64_kernel(const double* __restrict__ src, int64_t rows, int64_t cols, int64_t lds,
                                 int trans, int terms, void* dst, int64_t ldd, int64_t plane) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t i = e / cols, j = e % cols;
  const double x = src[i * lds + j];
  const int64_t o = trans ? (j * ldd + i) : (i * ldd + j);
  if (terms == 0) {
    static_cast<float*>(dst)[o] = static_cast<float>(x);
    return;
  }
  uint16_t* d = static_cast<uint16_t*>(dst);
  double r = x;
  for (int q = 0; q < terms; ++q) {
    const __bf16 h = static_cast<__bf16>(static_cast<float>(r));
    d[q * plane + o] = __builtin_bit_cast(uint16_t, h);
    r = r - static_cast<double>(static_cast<float>(h));
  }
}

}  // namespace

size_t wide_gemm_workspace_bytes(int64_t M, int64_t K, int64_t N, int num_cus) {
  const int64_t mslice = std::min<int64_t>(M, kMaxMT * 16);
  int s = 1;
  for (int mt = 1; mt <= kMaxMT; ++mt)
    for (int f = 0; f < 2; ++f) s = std::max(s, choose_splits(K, N, num_cus, cols_per_block(mt, f != 0)));
  return s > 1 ? static_cast<size_t>(s) * mslice * N * sizeof(double) : 0;
}

int max_norm_partials(int64_t M, int64_t N) {
  const int64_t nblk = (N + kMinColsPerBlock - 1) / kMinColsPerBlock;
  const int64_t slices = (M + kMaxMT * 16 - 1) / (kMaxMT * 16);
  return static_cast<int>(std::max<int64_t>(nblk, 1024) * std::max<int64_t>(slices, 1));
}

int wide_gemm(const WideGemm& g, void* workspace, size_t workspace_bytes, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) {
    if (g.nparts) *g.nparts = 0;
    return ICUR_OK;
  }
  if (g.K < 0) return arg_error("negative K");
  const bool f64 = (g.wterms < 0);
  if (f64 ? (g.bterms >= 0 || !g.out64)
          : (g.wterms > 3 || g.bterms < 0 || g.bterms > 3 || ((g.wterms == 0) != (g.bterms == 0))))
    return arg_error("invalid piece counts");
  DeviceInfo dev;
  ICUR_TRY(device_info(&dev));
  const size_t osz = g.out64 ? sizeof(double) : sizeof(float);
  int parts = 0;
  // M is processed in slices of at most 160 rows (10 tiles of 16).
  for (int64_t m0 = 0; m0 < g.M; m0 += kMaxMT * 16) {
    const int64_t Ms = std::min<int64_t>(g.M - m0, kMaxMT * 16);
    const int mt = static_cast<int>((Ms + 15) / 16);
    wide::Params p;
    p.X = g.X ? static_cast<const char*>(g.X) + m0 * g.ldx * osz : nullptr;
    p.ldx = g.ldx;
    if (f64)
      p.W = static_cast<const double*>(g.W) + m0 * g.ldw;
    else if (g.wterms == 0 && !g.w_bf16)
      p.W = static_cast<const float*>(g.W) + m0 * g.ldw;
    else
      p.W = static_cast<const uint16_t*>(g.W) + m0 * g.ldw;
    p.w_bf16 = g.w_bf16 ? 1 : 0;
    p.ldw = g.ldw;
    p.wplane = g.M * g.ldw;
    p.B = g.B;
    p.ldb = g.ldb;
    p.M = Ms;
    p.K = g.K;
    p.N = g.N;
    p.subtract = g.subtract ? 1 : 0;
    p.OUT = static_cast<char*>(g.OUT) + m0 * g.ldo * osz;
    p.ldo = g.ldo;
    p.norm_partials = g.norm_partials ? g.norm_partials + parts : nullptr;
    const int64_t cpb = cols_per_block(mt, f64);
    const int64_t nblk = (g.N + cpb - 1) / cpb;
    auto reduce = g.out64 ? wide::launch_reduce_f64 : wide::launch_reduce_f32;
    if (g.K == 0) {
      // OUT = X (subtract) or 0: the reduce kernel with zero splits
      const int blocks = static_cast<int>(std::min<int64_t>((Ms * g.N + 255) / 256, 1024));
      ICUR_TRY(reduce(nullptr, 0, Ms, g.N, p.X, g.ldx, p.subtract, p.OUT, g.ldo, p.norm_partials, blocks, st));
      parts += blocks;
      continue;
    }
    int nsplit = choose_splits(g.K, g.N, dev.num_cus, cpb);
    const size_t need = static_cast<size_t>(nsplit) * Ms * g.N * sizeof(double);
    if (nsplit > 1 && (workspace == nullptr || need > workspace_bytes)) nsplit = 1;
    const int64_t chunks = (g.K + kKC - 1) / kKC;
    p.k_per_split = ((chunks + nsplit - 1) / nsplit) * kKC;
    nsplit = static_cast<int>((g.K + p.k_per_split - 1) / p.k_per_split);
    p.partial = static_cast<double*>(workspace);
    wide::KernelFn fn = g.out64 ? wide::pick_kernel_f64(mt, g.wterms, g.bterms)
                                : wide::pick_kernel_f32(mt, g.wterms, g.bterms);
    if (!fn) return arg_error("unsupported tile configuration");
    hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(nblk), static_cast<unsigned>(nsplit)), dim3(wide::kThreads),
                       0, st, p);
    ICUR_HIP(hipGetLastError());
    if (nsplit > 1) {
      const int blocks = static_cast<int>(std::min<int64_t>((Ms * g.N + 255) / 256, 1024));
      ICUR_TRY(reduce(p.partial, nsplit, Ms, g.N, p.X, g.ldx, p.subtract, p.OUT, g.ldo, p.norm_partials, blocks,
                      st));
      parts += blocks;
    } else {
      parts += static_cast<int>(nblk);
    }
  }
  if (g.nparts) *g.nparts = parts;
  return ICUR_OK;
}

int launch_split_f64(const double* src, int64_t rows, int64_t cols, int64_t lds, bool trans, int terms, void* dst,
                     int64_t ldd, int64_t plane, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return ICUR_OK;
  const int64_t total = rows * cols;
  hipLaunchKernelGGL(split_f64_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, st, src,
                     rows, cols, lds, trans ? 1 : 0, terms, dst, ldd, plane);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

int launch_reduce_partials(const double* partials, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3(1), dim3(256), 0, st, partials, n, out);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

}  // namespace icur
