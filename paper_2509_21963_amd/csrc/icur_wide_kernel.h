// Wide product kernel template (included by icur_wide_f32.hip and icur_wide_f64.hip,
// which instantiate it for FP32 and FP64 outputs).
//
// OUT(M x N) = X - W(M x K) B(K x N)   or   OUT = W B
// with a short M (the sketch size c or the block size b) and a long, row-major N.  All
// dense contractions of the IterativeCUR loop have this shape (see icur_gemm.hip).
//
// Layout.  One workgroup (4 waves) owns a 16*NS*4-column strip of OUT and all M rows;
// each wave owns 16*NS columns.  B is read straight from HBM into registers in the operand
// layout of the 16x16 matrix-core instructions (lane l takes column l%16 at K offsets
// 4*(l/16) or 8*(l/16)), so every B element is loaded once per launch.  W is staged
// through LDS one 32-deep K chunk at a time and shared by the four waves.  Long K is split
// across workgroups; the FP64 partial planes are summed in a fixed order by a second
// kernel, so results are deterministic.
//
// Accuracy.  Each 32-deep chunk of a 16x16 output tile is summed on the matrix cores into
// a fresh FP32 accumulator and then added into an FP64 accumulator, so rounding grows
// with the chunk length, not with K.  Long sums (the sketch runs over all m rows of A)
// therefore stay at FP32-product accuracy.
//
// Arithmetic modes:
//   WT = BT = -1 v_mfma_f64_16x16x4f64 on FP64 W and FP64 B, FP64 accumulation (the
//                residual factors at tight tolerances);
//   WT = BT = 0  v_mfma_f32_16x16x4f32 on FP32 operands (the plain form);
//   WT, BT > 0   v_mfma_f32_16x16x32_bf16 on BF16 pieces: each FP32 value of B is split
//                in registers into BT pieces hi + lo + lo2 (hi = RNE(x), lo = RNE(x-hi),
//                ...); W arrives split into WT pieces.  Products of pieces (i, j) with
//                i + j < max(WT, BT) are summed.  Three pieces of B times a BF16-exact W
//                (the sketch G) reproduce every FP32 product exactly.
#pragma once

#include <type_traits>

#include "icur_internal.h"

namespace icur {
namespace wide {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kKC = 32;  // K rows per chunk
constexpr int kMaxMT = 10;

// Columns per wave (x16): fewer for tall M so the FP64 accumulators fit two waves per SIMD
// (the FP64 mode also holds its B operands in FP64).
constexpr int ns_for(int mt, bool f64) { return f64 ? (mt <= 1 ? 4 : (mt <= 2 ? 2 : 1)) : (mt <= 2 ? 4 : 2); }

struct Params {
  const void* X;  // OutT, may be null
  int64_t ldx;
  const void* W;
  int64_t ldw;
  int64_t wplane;  // elements between BF16 pieces of W
  int w_bf16;      // FP32 mode: W holds BF16 bit patterns
  const void* B;   // FP32, or FP64 in the FP64 mode
  int64_t ldb;
  int64_t M, K, N;
  int64_t k_per_split;  // multiple of kKC
  int subtract;
  void* OUT;  // OutT (single split)
  int64_t ldo;
  double* partial;  // nsplit x M x N planes (several splits)
  double* norm_partials;
};

using KernelFn = void (*)(const Params);

__device__ __forceinline__ double block_sum_f64(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) s += red[w];
  return s;  // valid in thread 0
}

template <int MT, int NS, int WT, int BT, typename OutT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void wide_kernel(const Params p) {
  constexpr bool kF64 = (WT < 0);
  constexpr bool kF32 = (WT == 0);
  constexpr bool kScalarW = kF64 || kF32;  // one W value per lane per MFMA (K = 4)
  using BT_t = typename std::conditional<kF64, double, float>::type;
  constexpr int T = (WT > BT ? WT : BT);
  constexpr int kRows = MT * 16;
  // LDS: FP32/FP64 W chunk stored transposed [k][row]; BF16 pieces stored [piece][row][k].
  constexpr int kF32Stride = kRows + 4;
  constexpr int kBfStride = kKC + 8;  // bf16 elements per row (80 bytes)
  constexpr int kLdsBytes = kF64 ? kKC * kF32Stride * 8
                                 : (kF32 ? kKC * kF32Stride * 4 : (WT > 0 ? WT : 1) * kRows * kBfStride * 2);
  __shared__ __attribute__((aligned(16))) unsigned char lds[kLdsBytes];
  __shared__ double red[kWaves];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int lr = lane & 15;  // column (B) / row (W) inside a 16-wide tile
  const int lg = lane >> 4;  // K group 0..3
  const int64_t col0 = static_cast<int64_t>(blockIdx.x) * (16 * NS * kWaves) + wave * 16 * NS;
  const int64_t kbeg = static_cast<int64_t>(blockIdx.y) * p.k_per_split;
  const int64_t kend = min(p.K, kbeg + p.k_per_split);

  bool colok[NS];
  int64_t colidx[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    colidx[s] = col0 + s * 16 + lr;
    colok[s] = colidx[s] < p.N;
    if (!colok[s]) colidx[s] = 0;
  }

  double acc[MT][NS][4];
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[t][s][v] = 0.0;

  // K row that register slot j of this lane holds for a chunk starting at k0.
  auto krow = [&](int64_t k0, int j) -> int64_t { return kScalarW ? (k0 + 4 * j + lg) : (k0 + 8 * lg + j); };

  auto load_b = [&](BT_t (&b)[8][NS], int64_t k0) {
    const bool full = (k0 + kKC <= kend);
    const BT_t* B = static_cast<const BT_t*>(p.B);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t k = krow(k0, j);
      const bool kok = full || k < kend;
      const BT_t* row = B + (kok ? k : 0) * p.ldb;
#pragma unroll
      for (int s = 0; s < NS; ++s)
        b[j][s] = (kok && colok[s]) ? __builtin_nontemporal_load(row + colidx[s]) : BT_t(0);
    }
  };

  auto stage_w = [&](int64_t k0) {
    if constexpr (kF64) {
      double* wl = reinterpret_cast<double*>(lds);
      const double* W = static_cast<const double*>(p.W);
      for (int e = threadIdx.x; e < kRows * kKC; e += kThreads) {
        const int row = e / kKC, kk = e % kKC;
        const int64_t k = k0 + kk;
        wl[kk * kF32Stride + row] = (row < p.M && k < kend) ? W[row * p.ldw + k] : 0.0;
      }
    } else if constexpr (kF32) {
      float* wl = reinterpret_cast<float*>(lds);
      for (int e = threadIdx.x; e < kRows * kKC; e += kThreads) {
        const int row = e / kKC, kk = e % kKC;
        const int64_t k = k0 + kk;
        float v = 0.f;
        if (row < p.M && k < kend) {
          if (p.w_bf16)
            v = __uint_as_float(static_cast<uint32_t>(static_cast<const uint16_t*>(p.W)[row * p.ldw + k]) << 16);
          else
            v = static_cast<const float*>(p.W)[row * p.ldw + k];
        }
        wl[kk * kF32Stride + row] = v;
      }
    } else {
      uint16_t* wl = reinterpret_cast<uint16_t*>(lds);
      const uint16_t* W = static_cast<const uint16_t*>(p.W);
      const bool vec = (k0 + kKC <= kend) && ((p.ldw & 7) == 0) && ((p.wplane & 7) == 0) &&
                       ((reinterpret_cast<uintptr_t>(W) & 15) == 0);
      if (vec) {
        for (int e = threadIdx.x; e < WT * kRows * 4; e += kThreads) {
          const int piece = e / (kRows * 4);
          const int rem = e % (kRows * 4);
          const int row = rem >> 2, q = rem & 3;
          uint4 v = {0u, 0u, 0u, 0u};
          if (row < p.M) v = *reinterpret_cast<const uint4*>(W + piece * p.wplane + row * p.ldw + k0 + 8 * q);
          *reinterpret_cast<uint4*>(wl + (piece * kRows + row) * kBfStride + 8 * q) = v;
        }
      } else {
        for (int e = threadIdx.x; e < WT * kRows * kKC; e += kThreads) {
          const int piece = e / (kRows * kKC);
          const int rem = e % (kRows * kKC);
          const int row = rem / kKC, kk = rem % kKC;
          const int64_t k = k0 + kk;
          uint16_t v = 0;
          if (row < p.M && k < kend) v = W[piece * p.wplane + row * p.ldw + k];
          wl[(piece * kRows + row) * kBfStride + kk] = v;
        }
      }
    }
  };

  // One chunk: each 16x16 tile is summed into a fresh FP32 accumulator on the matrix
  // cores, then added into the FP64 accumulator.
  auto compute = [&](const BT_t (&b)[8][NS]) {
    if constexpr (kF64) {
      // FP64 matrix cores accumulate in FP64 directly; the accumulator layout differs
      // from FP32 (slot v holds row 4v + l/16), which the epilogue accounts for.
      const double* wl = reinterpret_cast<const double*>(lds);
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        double a[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = wl[(4 * j + lg) * kF32Stride + t * 16 + lr];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          doublex4 c = {acc[t][s][0], acc[t][s][1], acc[t][s][2], acc[t][s][3]};
#pragma unroll
          for (int j = 0; j < 8; ++j) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[j], b[j][s], c, 0, 0, 0);
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[t][s][v] = c[v];
        }
      }
    } else if constexpr (kF32) {
      const float* wl = reinterpret_cast<const float*>(lds);
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        float a[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = wl[(4 * j + lg) * kF32Stride + t * 16 + lr];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int j = 0; j < 8; ++j) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[j], b[j][s], c, 0, 0, 0);
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[t][s][v] += static_cast<double>(c[v]);
        }
      }
    } else {
      const uint16_t* wl = reinterpret_cast<const uint16_t*>(lds);
      bf16x8 bp[NS][BT];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          float r = b[j][s];
#pragma unroll
          for (int q = 0; q < BT; ++q) {
            const __bf16 h = static_cast<__bf16>(r);
            bp[s][q][j] = h;
            r = r - static_cast<float>(h);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        bf16x8 a[WT];
#pragma unroll
        for (int i = 0; i < WT; ++i)
          a[i] = *reinterpret_cast<const bf16x8*>(wl + (i * kRows + t * 16 + lr) * kBfStride + 8 * lg);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int i = 0; i < WT; ++i)
#pragma unroll
            for (int q = 0; q < BT; ++q)
              if (i + q < T) c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bp[s][q], c, 0, 0, 0);
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[t][s][v] += static_cast<double>(c[v]);
        }
      }
    }
  };

  BT_t bA[8][NS], bB[8][NS];
  if (kbeg < kend) load_b(bA, kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += 2 * kKC) {
    __syncthreads();
    stage_w(k0);
    __syncthreads();
    if (k0 + kKC < kend) load_b(bB, k0 + kKC);
    compute(bA);
    if (k0 + kKC >= kend) break;
    __syncthreads();
    stage_w(k0 + kKC);
    __syncthreads();
    if (k0 + 2 * kKC < kend) load_b(bA, k0 + 2 * kKC);
    compute(bB);
  }

  // Epilogue: lane holds rows t*16 + 4*lg + v (FP64 mode: t*16 + 4*v + lg), columns
  // colidx[s].
  const bool split = (gridDim.y > 1);
  const OutT* X = static_cast<const OutT*>(p.X);
  OutT* OUT = static_cast<OutT*>(p.OUT);
  double sq = 0.0;
#pragma unroll
  for (int t = 0; t < MT; ++t) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = kF64 ? (t * 16 + 4 * v + lg) : (t * 16 + 4 * lg + v);
      if (row >= p.M) continue;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (!colok[s]) continue;
        const double a = acc[t][s][v];
        if (split) {
          p.partial[(static_cast<int64_t>(blockIdx.y) * p.M + row) * p.N + colidx[s]] = a;
        } else {
          double o = a;
          if (p.subtract) o = (X ? static_cast<double>(X[row * p.ldx + colidx[s]]) : 0.0) - a;
          const OutT ov = static_cast<OutT>(o);
          OUT[row * p.ldo + colidx[s]] = ov;
          sq += static_cast<double>(ov) * static_cast<double>(ov);
        }
      }
    }
  }
  if (!split && p.norm_partials) {
    const double s = block_sum_f64(sq, red);
    if (threadIdx.x == 0) p.norm_partials[blockIdx.x] = s;
  }
}

// OUT = X - sum over splits (or the sum), FP64 partials added in split order, plus
// per-block partial sums of OUT^2.
template <typename OutT>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(const double* __restrict__ partial, int nsplit,
                                                            int64_t M, int64_t N, const OutT* X, int64_t ldx,
                                                            int subtract, OutT* OUT, int64_t ldo,
                                                            double* norm_partials) {
  __shared__ double red[4];
  const int64_t total = M * N;
  double sq = 0.0;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t row = e / N, col = e % N;
    double s = 0.0;
    for (int q = 0; q < nsplit; ++q) s += partial[q * total + e];
    double o = s;
    if (subtract) o = (X ? static_cast<double>(X[row * ldx + col]) : 0.0) - s;
    const OutT ov = static_cast<OutT>(o);
    OUT[row * ldo + col] = ov;
    sq += static_cast<double>(ov) * static_cast<double>(ov);
  }
  if (norm_partials) {
    const double s = block_sum_f64(sq, red);
    if (threadIdx.x == 0) norm_partials[blockIdx.x] = s;
  }
}

template <typename OutT, int MT>
KernelFn pick_mode(int wt, int bt) {
  constexpr int NS = ns_for(MT, false);
  if constexpr (std::is_same<OutT, double>::value) {
    if (wt < 0) return wide_kernel<MT, ns_for(MT, true), -1, -1, OutT>;
  }
  if (wt < 0) return nullptr;
  if (wt == 0) return wide_kernel<MT, NS, 0, 0, OutT>;
  if (wt == 1 && bt == 1) return wide_kernel<MT, NS, 1, 1, OutT>;
  if (wt == 1 && bt == 2) return wide_kernel<MT, NS, 1, 2, OutT>;
  if (wt == 1 && bt == 3) return wide_kernel<MT, NS, 1, 3, OutT>;
  if (wt == 2 && bt == 2) return wide_kernel<MT, NS, 2, 2, OutT>;
  if (wt == 3 && bt == 3) return wide_kernel<MT, NS, 3, 3, OutT>;
  return nullptr;
}

template <typename OutT>
KernelFn pick_kernel_t(int mt, int wt, int bt) {
  switch (mt) {
    case 1: return pick_mode<OutT, 1>(wt, bt);
    case 2: return pick_mode<OutT, 2>(wt, bt);
    case 3: return pick_mode<OutT, 3>(wt, bt);
    case 4: return pick_mode<OutT, 4>(wt, bt);
    case 5: return pick_mode<OutT, 5>(wt, bt);
    case 6: return pick_mode<OutT, 6>(wt, bt);
    case 7: return pick_mode<OutT, 7>(wt, bt);
    case 8: return pick_mode<OutT, 8>(wt, bt);
    case 9: return pick_mode<OutT, 9>(wt, bt);
    case 10: return pick_mode<OutT, 10>(wt, bt);
    default: return nullptr;
  }
}

// Defined in icur_wide_f32.hip / icur_wide_f64.hip.
KernelFn pick_kernel_f32(int mt, int wt, int bt);
KernelFn pick_kernel_f64(int mt, int wt, int bt);
int launch_reduce_f32(const double* partial, int nsplit, int64_t M, int64_t N, const void* X, int64_t ldx,
                      int subtract, void* OUT, int64_t ldo, double* norm_partials, int blocks, hipStream_t st);
int launch_reduce_f64(const double* partial, int nsplit, int64_t M, int64_t N, const void* X, int64_t ldx,
                      int subtract, void* OUT, int64_t ldo, double* norm_partials, int blocks, hipStream_t st);

}  // namespace wide
}  // namespace icur
