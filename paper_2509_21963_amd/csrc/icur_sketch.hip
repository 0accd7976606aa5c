// The initial sketch X0 = G A of Alg. 1 (the recycled sketch of §3.2.1, taken once, and
// its norm ||G A||_F, the denominator of the estimator of §3.3).
//
// This is the one pass over all of A that the method makes, so it is bound by HBM
// bandwidth: 4 m n bytes of A for 2 c m n useful flops (c = 110 gives 55 flop/byte, far
// below the BF16 matrix-core ridge).  The kernel is built to stream A once at full
// bandwidth and keep every other cost under it:
//
//   * A is read straight from HBM into registers, a 128-row block ahead of its use: lane
//     (g, l) of a wave owns column l of the wave's 16-column strip and K rows 8g .. 8g+7
//     of each 32-row chunk, which is the B-operand layout of v_mfma_f32_16x16x32_bf16, so
//     no transposition is needed; the 16 lanes of a row read 64 contiguous bytes and the
//     two waves of neighbouring strips complete each 128-byte line.  Addresses are a
//     uniform chunk base plus eight fixed 32-bit lane offsets.  Eight waves (two per
//     SIMD) keep about 64 KB of A in flight per CU.
//   * Each FP32 element of A is split in registers into `terms` BF16 pieces
//     (hi = RNE(x), mid = RNE(x - hi), lo = RNE(x - hi - mid)); G holds BF16-exact values,
//     so three pieces reproduce every product G_ri A_ij exactly in the FP32 accumulator.
//   * G is staged through LDS, 128 K rows at a time, double buffered (one barrier per
//     block), and shared by the eight waves of a workgroup.
//   * The FP32 accumulators of a 128-row block (of each 32-row chunk in the precise
//     variant, for tight tolerances) are added into FP64 accumulators, so rounding grows
//     with the block length, not with m.
//   * Long m is split across workgroups to balance the grid over the CUs; the FP64
//     partial planes are summed in split order by a second kernel (deterministic).
#include <algorithm>

#include "icur_internal.h"
#include "icur_wide_kernel.h"

namespace icur {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kWaves = 8;             // two waves per SIMD
constexpr int kThreads = 64 * kWaves;
constexpr int kKC = 32;               // K rows per matrix-core chunk
constexpr int kCPB = 4;               // chunks per block
constexpr int kKB = kKC * kCPB;       // K rows per block (G staging, FP64 flush)
constexpr int kColsWave = 16;
constexpr int kColsWG = kColsWave * kWaves;
constexpr int kWStride = kKB + 8;     // BF16 elements per LDS row of G (272 bytes)
constexpr int kMaxMT = 10;            // up to 160 rows of G per launch
constexpr int kBufferWord3 = 0x00020000;  // buffer resource word 3 on gfx9: 32-bit data, raw

struct Params {
  const uint16_t* G;  // rows of this slice, BF16 bit patterns
  int64_t ldg;
  const float* A;
  int64_t lda;
  int64_t M, K, N;
  int64_t k_per_split;  // multiple of kKB
  double* out;          // single split: X0 slice (FP64)
  int64_t ldo;
  double* partial;      // several splits: nsplit planes of M x N
  double* norm_partials;
};

template <int MT>
constexpr size_t lds_bytes() {
  return 2ull * MT * 16 * kWStride * sizeof(uint16_t);
}

// CPF: chunks summed in FP32 before each FP64 flush (4 = once per block; 1 = after
// every 32-row chunk, for tight tolerances).
template <int MT, int BT, int CPF>
__global__ __launch_bounds__(kThreads, 1) void sketch_kernel(const Params p) {
  static_assert(kCPB % CPF == 0, "flushes divide the block");
  constexpr int kRows = MT * 16;
  constexpr int kGPieces = kRows * (kKB / 8);                   // 16-byte pieces of a G block
  constexpr int kGVec = (kGPieces + kThreads - 1) / kThreads;   // per thread
  extern __shared__ __attribute__((aligned(16))) uint16_t wl[];  // 2 x kRows x kWStride
  __shared__ double red[kWaves];

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int lr = lane & 15;
  const int lg = lane >> 4;
  const int64_t col = static_cast<int64_t>(blockIdx.x) * kColsWG + wave * kColsWave + lr;
  const bool colok = col < p.N;
  const int64_t kbeg = static_cast<int64_t>(blockIdx.y) * p.k_per_split;
  const int64_t kend = min(p.K, kbeg + p.k_per_split);
  const unsigned lda4 = static_cast<unsigned>(p.lda) * 4u;  // the host keeps 128 rows below 2^31 bytes

  floatx4 acc32[MT];
  double acc64[MT][4];
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    acc32[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < 4; ++v) acc64[t][v] = 0.0;
  }

  // Block loads go through buffer resources: a uniform base per block, one fixed lane
  // offset and a uniform row offset, so no per-load address arithmetic.  A: lane offset
  // of row 8 lg, column col clamped into the matrix (a lane past column N only feeds its
  // own output column, which is never stored).  G: the thread's 16-byte pieces of a
  // block; pieces in rows past M fall outside the resource and read zero.
  const unsigned a_voff = static_cast<unsigned>(8 * lg) * lda4 + static_cast<unsigned>(min(col, p.N - 1)) * 4u;
  unsigned g_off[kGVec];
  unsigned g_live = 0;  // bit e: piece e exists and lies in a row of G
#pragma unroll
  for (int e = 0; e < kGVec; ++e) {
    const int idx = e * kThreads + threadIdx.x;
    const int row = idx / (kKB / 8), q = idx % (kKB / 8);
    g_off[e] = static_cast<unsigned>((row * static_cast<int>(p.ldg) + 8 * q) * 2);
    if (idx < kGPieces && row < p.M) g_live |= 1u << e;
  }

  // A block of 128 rows from kb, all inside [kbeg, kend).
  auto load_a = [&](float (&b)[kCPB][8], int64_t kb) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(p.A + kb * p.lda), 0, static_cast<int>(kKB * lda4), kBufferWord3);
#pragma unroll
    for (int q = 0; q < kCPB; ++q)
#pragma unroll
      for (int j = 0; j < 8; ++j)
        b[q][j] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                rs, a_voff, static_cast<int>((q * kKC + j) * lda4), 0));
  };

  // The last, partial block of the range: rows from kend on read as zero.
  auto load_a_tail = [&](float (&b)[kCPB][8], int64_t kb) {
    const int64_t cc = min(col, p.N - 1);
#pragma unroll
    for (int q = 0; q < kCPB; ++q)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t k = kb + q * kKC + 8 * lg + j;
        b[q][j] = k < kend ? p.A[k * p.lda + cc] : 0.f;
      }
  };

  auto load_g = [&](uint4 (&w)[kGVec], int64_t kb) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint16_t*>(p.G + kb), 0, static_cast<int>(p.M * p.ldg * 2), kBufferWord3);
#pragma unroll
    for (int e = 0; e < kGVec; ++e) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, g_off[e], 0, 0);
      w[e] = ((g_live >> e) & 1u) ? uint4{v[0], v[1], v[2], v[3]} : uint4{0u, 0u, 0u, 0u};
    }
  };
  auto load_g_tail = [&](uint4 (&w)[kGVec], int64_t kb) {
#pragma unroll
    for (int e = 0; e < kGVec; ++e) {
      const int idx = e * kThreads + threadIdx.x;
      const int row = idx / (kKB / 8), q = idx % (kKB / 8);
      unsigned h[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int64_t k = kb + 8 * q + i;
        h[i] = (((g_live >> e) & 1u) && k < kend) ? p.G[row * p.ldg + k] : 0u;
      }
      w[e] = uint4{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16)};
    }
  };
  auto store_g = [&](const uint4 (&w)[kGVec], int buf) {
    uint16_t* dst = wl + buf * kRows * kWStride;
#pragma unroll
    for (int e = 0; e < kGVec; ++e) {
      const int idx = e * kThreads + threadIdx.x;
      const int row = idx / (kKB / 8), q = idx % (kKB / 8);
      if (idx < kGPieces) *reinterpret_cast<uint4*>(dst + row * kWStride + 8 * q) = w[e];
    }
  };

  auto compute = [&](const float (&b)[kCPB][8], int buf) {
    const uint16_t* wb = wl + buf * kRows * kWStride;
#pragma unroll
    for (int q = 0; q < kCPB; ++q) {
      bf16x8 bp[BT];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        float r = b[q][j];
#pragma unroll
        for (int i = 0; i < BT; ++i) {
          const __bf16 h = static_cast<__bf16>(r);
          bp[i][j] = h;
          if (i + 1 < BT) r = r - static_cast<float>(h);
        }
      }
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(wb + (t * 16 + lr) * kWStride + q * kKC + 8 * lg);
#pragma unroll
        for (int i = 0; i < BT; ++i) acc32[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bp[i], acc32[t], 0, 0, 0);
      }
      if ((q + 1) % CPF == 0) {
#pragma unroll
        for (int t = 0; t < MT; ++t) {
#pragma unroll
          for (int v = 0; v < 4; ++v) acc64[t][v] += static_cast<double>(acc32[t][v]);
          acc32[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
      }
      // keep the next chunk's LDS reads and splitting below this point: hoisting them
      // for all four chunks would need more registers than two waves per SIMD have
      __builtin_amdgcn_sched_barrier(0);
    }
  };

  // Full blocks, pipelined: while block i is multiplied, block i+1 of A and of G is in
  // flight into registers; G then goes to the other LDS buffer (one barrier per block).
  const int64_t kfull = kbeg + (kend - kbeg) / kKB * kKB;
  {
    float bA[kCPB][8], bB[kCPB][8];
    uint4 wr[kGVec];
    if (kbeg < kfull) {
      load_a(bA, kbeg);
      load_g(wr, kbeg);
      store_g(wr, 0);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t kb = kbeg; kb < kfull; kb += 2 * kKB) {
      const int64_t k1 = kb + kKB;
      if (k1 < kfull) {
        load_a(bB, k1);
        load_g(wr, k1);
      }
      compute(bA, buf);
      if (k1 >= kfull) break;
      store_g(wr, buf ^ 1);  // that buffer was last read before the previous barrier
      __syncthreads();
      buf ^= 1;
      const int64_t k2 = k1 + kKB;
      if (k2 < kfull) {
        load_a(bA, k2);
        load_g(wr, k2);
      }
      compute(bB, buf);
      if (k2 >= kfull) break;
      store_g(wr, buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
  if (kfull < kend) {
    float bt[kCPB][8];
    uint4 wt[kGVec];
    load_a_tail(bt, kfull);
    load_g_tail(wt, kfull);
    __syncthreads();  // every wave is done with both G buffers
    store_g(wt, 0);
    __syncthreads();
    compute(bt, 0);
  }

  // Epilogue: lane holds rows 16 t + 4 lg + v of column col.
  const bool split = (gridDim.y > 1);
  double sq = 0.0;
  if (colok) {
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = t * 16 + 4 * lg + v;
        if (row >= p.M) continue;
        const double x = acc64[t][v];
        if (split)
          p.partial[(static_cast<int64_t>(blockIdx.y) * p.M + row) * p.N + col] = x;
        else
          p.out[row * p.ldo + col] = x;
        sq += x * x;
      }
  }
  if (!split && p.norm_partials) {
    const double s = wide::block_sum_f64(sq, red);
    if (threadIdx.x == 0) p.norm_partials[blockIdx.x] = s;
  }
}

using SketchFn = void (*)(const Params);

template <int MT>
SketchFn pick_bt(int bt, bool precise) {
  // the per-chunk flush needs more registers; above 96 rows the general product serves
  if (precise) {
    if constexpr (MT <= 6) return bt == 3 ? sketch_kernel<MT, 3, 1> : nullptr;
    return nullptr;
  }
  switch (bt) {
    case 1: return sketch_kernel<MT, 1, kCPB>;
    case 2: return sketch_kernel<MT, 2, kCPB>;
    case 3: return sketch_kernel<MT, 3, kCPB>;
    default: return nullptr;
  }
}

SketchFn pick(int mt, int bt, bool precise, size_t* lds) {
  switch (mt) {
#define ICUR_SK_CASE(X) \
  case X:               \
    *lds = lds_bytes<X>(); \
    return pick_bt<X>(bt, precise);
    ICUR_SK_CASE(1)
    ICUR_SK_CASE(2)
    ICUR_SK_CASE(3)
    ICUR_SK_CASE(4)
    ICUR_SK_CASE(5)
    ICUR_SK_CASE(6)
    ICUR_SK_CASE(7)
    ICUR_SK_CASE(8)
    ICUR_SK_CASE(9)
    ICUR_SK_CASE(10)
#undef ICUR_SK_CASE
    default: return nullptr;
  }
}

// Splits of m: the grid has one workgroup per CU at a time, so pick the split count
// (at most 8, each split at least 8 blocks of 128 rows) whose number of workgroups best
// fills whole rounds of the CUs; ties go to fewer splits.
int choose_sketch_splits(int64_t m, int64_t n, int num_cus) {
  const int64_t tiles = (n + kColsWG - 1) / kColsWG;
  const int64_t blocks = (m + kKB - 1) / kKB;
  int best = 1;
  double best_eff = 0.0;
  for (int s = 1; s <= 8; ++s) {
    if (s > 1 && blocks / s < 8) break;
    const int64_t wg = tiles * s;
    const int64_t rounds = (wg + num_cus - 1) / num_cus;
    const double eff = static_cast<double>(wg) / static_cast<double>(rounds * num_cus);
    if (eff > best_eff + 0.02) {
      best_eff = eff;
      best = s;
    }
  }
  return best;
}

}  // namespace

int convert_f64_f32_norm(const double* src, int64_t M, int64_t N, float* dst, int64_t ldd, double* norm_partials,
                         int* nparts, hipStream_t st) {
  const int blocks = static_cast<int>(std::min<int64_t>((M * N + 255) / 256, 1024));
  ICUR_TRY(wide::launch_reduce_f32(src, 1, M, N, nullptr, 0, 0, dst, ldd, norm_partials, blocks, st));
  if (nparts) *nparts = blocks;
  return ICUR_OK;
}

size_t sketch_workspace_bytes(int64_t c, int64_t m, int64_t n, int num_cus) {
  const int s = choose_sketch_splits(m, n, num_cus);
  const int64_t slice = std::min<int64_t>(c, kMaxMT * 16);
  return s > 1 ? static_cast<size_t>(s) * slice * n * sizeof(double) : 0;
}

int sketch_max_norm_partials(int64_t c, int64_t n) {
  const int64_t tiles = (n + kColsWG - 1) / kColsWG;
  const int64_t slices = (c + kMaxMT * 16 - 1) / (kMaxMT * 16);
  return static_cast<int>(std::max<int64_t>(tiles, 1024) * std::max<int64_t>(slices, 1));
}

int sketch_product(const uint16_t* G, int64_t ldg, int64_t c, const float* A, int64_t m, int64_t n,
                   int64_t lda, int terms, bool precise, double* X0, int64_t ldx, double* norm_partials,
                   int* nparts, void* workspace, size_t workspace_bytes, hipStream_t st, hipEvent_t ev_begin,
                   hipEvent_t ev_end) {
  if (terms < 1 || terms > 3) return ICUR_ERR_UNSUPPORTED;
  if (reinterpret_cast<uintptr_t>(A) & 3) return ICUR_ERR_UNSUPPORTED;
  if ((ldg & 7) || (reinterpret_cast<uintptr_t>(G) & 15)) return ICUR_ERR_UNSUPPORTED;
  // 32-bit offsets inside a block: A rows of a 128-row block, G rows of a 160-row slice
  if (static_cast<int64_t>(kKB) * lda * 4 + 4 * n >= (int64_t(1) << 31)) return ICUR_ERR_UNSUPPORTED;
  if (static_cast<int64_t>(kMaxMT * 16) * ldg * 2 >= (int64_t(1) << 31)) return ICUR_ERR_UNSUPPORTED;
  if (c < 1 || m < 1 || n < 1) return ICUR_ERR_UNSUPPORTED;
  DeviceInfo dev;
  ICUR_TRY(device_info(&dev));
  int nsplit = choose_sketch_splits(m, n, dev.num_cus);
  const int64_t slice_max = std::min<int64_t>(c, kMaxMT * 16);
  if (nsplit > 1 && (workspace == nullptr ||
                     static_cast<size_t>(nsplit) * slice_max * n * sizeof(double) > workspace_bytes))
    nsplit = 1;
  const int64_t blocks = (m + kKB - 1) / kKB;
  const int64_t k_per_split = ((blocks + nsplit - 1) / nsplit) * kKB;
  nsplit = static_cast<int>((m + k_per_split - 1) / k_per_split);
  const int64_t tiles = (n + kColsWG - 1) / kColsWG;
  for (int64_t r0 = 0; r0 < c; r0 += kMaxMT * 16) {  // every slice has a kernel: check first
    size_t lds = 0;
    if (!pick(static_cast<int>((std::min<int64_t>(c - r0, kMaxMT * 16) + 15) / 16), terms, precise, &lds))
      return ICUR_ERR_UNSUPPORTED;
  }
  int parts = 0;
  for (int64_t r0 = 0; r0 < c; r0 += kMaxMT * 16) {
    const int64_t Ms = std::min<int64_t>(c - r0, kMaxMT * 16);
    const int mt = static_cast<int>((Ms + 15) / 16);
    size_t lds = 0;
    SketchFn fn = pick(mt, terms, precise, &lds);
    Params p;
    p.G = G + r0 * ldg;
    p.ldg = ldg;
    p.A = A;
    p.lda = lda;
    p.M = Ms;
    p.K = m;
    p.N = n;
    p.k_per_split = k_per_split;
    p.out = X0 + r0 * ldx;
    p.ldo = ldx;
    p.partial = static_cast<double*>(workspace);
    p.norm_partials = norm_partials ? norm_partials + parts : nullptr;
    if (lds > 64 * 1024)
      ICUR_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   static_cast<int>(lds)));
    if (r0 == 0 && ev_begin) ICUR_HIP(hipEventRecord(ev_begin, st));
    hipLaunchKernelGGL(fn, dim3(static_cast<unsigned>(tiles), static_cast<unsigned>(nsplit)), dim3(kThreads),
                       lds, st, p);
    ICUR_HIP(hipGetLastError());
    if (r0 == 0 && ev_end) ICUR_HIP(hipEventRecord(ev_end, st));
    if (nsplit > 1) {
      const int rblocks = static_cast<int>(std::min<int64_t>((Ms * n + 255) / 256, 1024));
      ICUR_TRY(wide::launch_reduce_f64(p.partial, nsplit, Ms, n, nullptr, 0, 0, p.out, ldx, p.norm_partials,
                                       rblocks, st));
      parts += rblocks;
    } else {
      parts += static_cast<int>(tiles);
    }
  }
  if (nparts) *nparts = parts;
  return ICUR_OK;
}

}  // namespace icur
