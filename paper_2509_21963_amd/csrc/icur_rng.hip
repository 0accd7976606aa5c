// The recycled sketch operator G (c x m) of Alg. 1, generated on the device.
//
// The paper draws G once and reuses it in every iteration (Alg. 1; §3.2.1); it uses
// Gaussian entries in its experiments and names the sparse-sign matrix as a cheaper
// alternative (§2.1, §3.4).  Entries come from the counter-based generator
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), so every entry is a pure function
// of (seed, row, column) and any thread can produce any entry:
//   Gaussian G[r][i]: counter (lo32(i), hi32(i), r, 'GAUS'), Box-Muller on the two
//     53-bit uniforms of the block in FP64, rounded to FP32 then to BF16 (nearest even);
//   sparse-sign column i: Floyd's sampling of min(zeta, c) distinct rows, the t-th draw
//     from counter (lo32(i), hi32(i), t, 'SPRS'): row = word0 mod (c - z + t + 1),
//     replaced by c - z + t when already taken; sign negative when bit 0 of word1 is 1.
//   SRTT (the subsampled randomized trigonometric transform of §3.4): G = sqrt(m/c) R F D
//     with F the orthonormal DCT-II of length m, D = diag(d_i), d_i = -1 when bit 0 of
//     word0 of counter (lo32(i), hi32(i), 0, 'SRTD') is set, and R keeping c distinct rows
//     of F D chosen by Floyd's algorithm (draw t from counter (t, 0, 0, 'SRTR'),
//     v = (word1 * 2^32 + word0) mod (m - c + t + 1)), listed in increasing order.
//     G[k][i] = d_i sqrt(m/c) s_r cos(pi r (2 i + 1) / (2 m)) for kept row r = R[k]
//     (s_0 = sqrt(1/m), s_r = sqrt(2/m)), the angle reduced exactly as q = r (2i+1) mod 4m.
#include "icur_internal.h"

namespace icur {
namespace {

constexpr uint32_t kTagGauss = 0x47415553u;
constexpr uint32_t kTagSign = 0x53505253u;
constexpr uint32_t kTagSrttSign = 0x53525444u;
constexpr uint32_t kTagSrttRows = 0x53525452u;

struct U32x4 {
  uint32_t x0, x1, x2, x3;
};

__device__ __forceinline__ U32x4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
    const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return {c0, c1, c2, c3};
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  const uint32_t u = __float_as_uint(f);
  return static_cast<uint16_t>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__global__ void gaussian_G_kernel(uint64_t seed, int64_t c, int64_t m, uint16_t* __restrict__ G, int64_t sr,
                                  int64_t si) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (i >= m || r >= c) return;
  const uint64_t ui = static_cast<uint64_t>(i);
  const U32x4 w = philox4x32_10(static_cast<uint32_t>(ui), static_cast<uint32_t>(ui >> 32),
                                static_cast<uint32_t>(r), kTagGauss,
                                static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  const uint64_t a = ((static_cast<uint64_t>(w.x1) << 32) | w.x0) >> 11;
  const uint64_t b = ((static_cast<uint64_t>(w.x3) << 32) | w.x2) >> 11;
  const double u1 = (static_cast<double>(a) + 1.0) * 0x1.0p-53;  // (0, 1]
  const double u2 = static_cast<double>(b) * 0x1.0p-53;          // [0, 1)
  const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  G[r * sr + i * si] = f32_to_bf16_rne(static_cast<float>(z));
}

// One thread per column i of G (row i of A).  Writes the pattern and, when G_dense is
// given, the column's nonzeros as BF16 bit patterns (its zeros are written first by a
// separate fill).
__global__ void sparse_sign_kernel(uint64_t seed, int c, int64_t m, int z,
                                   uint8_t* __restrict__ rows, uint8_t* __restrict__ signs,
                                   uint16_t* __restrict__ G, int64_t ldg) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint64_t ui = static_cast<uint64_t>(i);
  int chosen[8];
  uint32_t sbits = 0;
  for (int t = 0; t < z; ++t) {
    const U32x4 w = philox4x32_10(static_cast<uint32_t>(ui), static_cast<uint32_t>(ui >> 32),
                                  static_cast<uint32_t>(t), kTagSign,
                                  static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    const int j = c - z + t;
    int v = static_cast<int>(w.x0 % static_cast<uint32_t>(j + 1));
    bool taken = false;
    for (int s = 0; s < t; ++s) taken |= (chosen[s] == v);
    chosen[t] = taken ? j : v;
    sbits |= (w.x1 & 1u) << t;
  }
  if (rows) {
    for (int t = 0; t < z; ++t) rows[i * z + t] = static_cast<uint8_t>(chosen[t]);
  }
  if (signs) signs[i] = static_cast<uint8_t>(sbits);
  if (G) {  // the column's zeros were written by zero_columns_kernel
    for (int t = 0; t < z; ++t)
      G[static_cast<int64_t>(chosen[t]) * ldg + i] = ((sbits >> t) & 1u) ? 0xBF80u : 0x3F80u;  // -1 / +1
  }
}

// Zeros in columns 0 .. m-1 of every row of a c x ldg BF16 matrix.
__global__ void zero_columns_kernel(uint16_t* __restrict__ G, int64_t m, int64_t ldg) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < m) G[static_cast<int64_t>(blockIdx.y) * ldg + i] = 0;
}

// Floyd's sampling of the c kept rows into a bitmap of m bytes (zeroed before): one thread,
// c draws; the value j = m - c + t is never taken before draw t.
__global__ void srtt_floyd_kernel(uint64_t seed, int64_t c, int64_t m, uint8_t* __restrict__ mark) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int64_t t = 0; t < c; ++t) {
    const U32x4 w = philox4x32_10(static_cast<uint32_t>(t), 0u, 0u, kTagSrttRows, static_cast<uint32_t>(seed),
                                  static_cast<uint32_t>(seed >> 32));
    const uint64_t j = static_cast<uint64_t>(m - c + t);
    const uint64_t v = ((static_cast<uint64_t>(w.x1) << 32) | w.x0) % (j + 1);
    if (mark[v]) mark[j] = 1;
    else mark[v] = 1;
  }
}

// The marked rows in increasing order: one workgroup scans the bitmap in chunks.
__global__ __launch_bounds__(1024) void srtt_compact_kernel(const uint8_t* __restrict__ mark, int64_t m,
                                                            int64_t* __restrict__ rows) {
  __shared__ int wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int64_t base_out = 0;
  for (int64_t base = 0; base < m; base += 1024) {
    const int64_t i = base + tid;
    const int v = (i < m && mark[i]) ? 1 : 0;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    __syncthreads();
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int before = 0, total = 0;
    for (int q = 0; q < 16; ++q) {
      before += q < w ? wsum[q] : 0;
      total += wsum[q];
    }
    if (v) rows[base_out + before + x - 1] = i;
    base_out += total;
  }
}

__global__ void srtt_G_kernel(uint64_t seed, int64_t c, int64_t m, const int64_t* __restrict__ rows,
                              float* __restrict__ G, int64_t ldg) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t k = blockIdx.y;
  if (i >= m || k >= c) return;
  const uint64_t ui = static_cast<uint64_t>(i);
  const U32x4 w = philox4x32_10(static_cast<uint32_t>(ui), static_cast<uint32_t>(ui >> 32), 0u, kTagSrttSign,
                                static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  const double d = (w.x0 & 1u) ? -1.0 : 1.0;
  const int64_t r = rows[k];
  const int64_t q = (r * (2 * i + 1)) % (4 * m);
  const double scale = (r == 0 ? sqrt(1.0 / static_cast<double>(m)) : sqrt(2.0 / static_cast<double>(m))) *
                       sqrt(static_cast<double>(m) / static_cast<double>(c));
  const double v = d * scale * cos(3.141592653589793 * static_cast<double>(q) / (2.0 * static_cast<double>(m)));
  G[k * ldg + i] = static_cast<float>(v);
}

}  // namespace

int launch_srtt(uint64_t seed, int64_t c, int64_t m, float* G, int64_t ldg, int64_t* rows, uint8_t* mark,
                hipStream_t st) {
  if (c <= 0 || m <= 0) return ICUR_OK;
  if (c > m) return arg_error("SRTT sketch needs c <= m");
  if (c > 65535) return arg_error("sketch rows c exceed 65535");
  if (G && ldg < m) return arg_error("sketch: need ldg >= m");
  if (m > (int64_t(1) << 40)) return arg_error("SRTT sketch: m too large");
  ICUR_TRY(launch_fill_u8(mark, m, 0, st));
  hipLaunchKernelGGL(srtt_floyd_kernel, dim3(1), dim3(64), 0, st, seed, c, m, mark);
  hipLaunchKernelGGL(srtt_compact_kernel, dim3(1), dim3(1024), 0, st, mark, m, rows);
  if (G) {
    dim3 grid(static_cast<unsigned>((m + 255) / 256), static_cast<unsigned>(c));
    hipLaunchKernelGGL(srtt_G_kernel, grid, dim3(256), 0, st, seed, c, m, rows, G, ldg);
  }
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

int launch_gaussian_G(uint64_t seed, int64_t c, int64_t m, uint16_t* G, int64_t ldg, hipStream_t st) {
  if (c <= 0 || m <= 0) return ICUR_OK;
  if (ldg < m) return arg_error("sketch: need ldg >= m");
  if (c > 65535) return arg_error("sketch rows c exceed 65535");
  dim3 grid(static_cast<unsigned>((m + 255) / 256), static_cast<unsigned>(c));
  hipLaunchKernelGGL(gaussian_G_kernel, grid, dim3(256), 0, st, seed, c, m, G, ldg, int64_t(1));
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

int launch_gaussian_G_strided(uint64_t seed, int64_t c, int64_t m, uint16_t* G, int64_t sr, int64_t si,
                              hipStream_t st) {
  if (c <= 0 || m <= 0) return ICUR_OK;
  if (c > 65535) return arg_error("sketch rows c exceed 65535");
  dim3 grid(static_cast<unsigned>((m + 255) / 256), static_cast<unsigned>(c));
  hipLaunchKernelGGL(gaussian_G_kernel, grid, dim3(256), 0, st, seed, c, m, G, sr, si);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

int launch_sparse_sign(uint64_t seed, int64_t c, int64_t m, int zeta, uint8_t* rows,
                       uint8_t* signs, uint16_t* G_dense, int64_t ldg, hipStream_t st) {
  if (c <= 0 || m <= 0) return ICUR_OK;
  if (G_dense && ldg < m) return arg_error("sketch: need ldg >= m");
  if (c > 255) return arg_error("sparse-sign sketch needs c <= 255");
  const int z = zeta < c ? zeta : static_cast<int>(c);
  if (z < 1 || z > 8) return arg_error("sparse-sign zeta must be in 1..8");
  if (G_dense) {
    hipLaunchKernelGGL(zero_columns_kernel, dim3(static_cast<unsigned>((m + 255) / 256), static_cast<unsigned>(c)),
                       dim3(256), 0, st, G_dense, m, ldg);
    ICUR_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(sparse_sign_kernel, dim3(static_cast<unsigned>((m + 255) / 256)), dim3(256),
                     0, st, seed, static_cast<int>(c), m, z, rows, signs, G_dense, ldg);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

}  // namespace icur
