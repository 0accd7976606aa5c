// Sparse input (CSR) for Alg. 1: the initial sketch X0 = G A and the gathers of columns,
// rows and the cross A(I,J) straight from the compressed matrix.  The loop itself (both
// selections, the residual-form products, the core) is the dense path's: its operands
// are the dense gathered columns and rows.
//
// Columns are needed twice (the sketch accumulates X0(:, j) over column j's entries; the
// column selection gathers A(:, J_k)), so a CSC copy is built once per call with a
// stable radix sort of the column indices: within a column the entries keep increasing
// row order, which fixes the summation order of the sketch (results are deterministic).
//
// Sketch, one wave per column j, FP64 accumulation.  Lane l owns output rows l, l + 64,
// l + 128, l + 192 (c <= 256).  For each entry (i, a) of the column, in row order:
//   sparse-sign G: column i of G has zeta nonzeros +-1; it is precomputed as 64-bit row
//     masks and sign masks (one pair per 64 rows), so the lane's coefficient is one bit
//     test and acc += +-a is exact FP64 arithmetic (fma with +-1);
//   Gaussian G: the lane reads G(r, i) from a transposed copy (m x c, the c values of
//     column i contiguous) and accumulates acc += G(r, i) a in FP64.
#include <algorithm>

#include <hipcub/hipcub.hpp>

#include "icur_internal.h"

namespace icur {
namespace {

constexpr int kSkWaves = 4;
constexpr int kMaxWords = 4;  // c <= 256 rows of G

// ---------------------------------------------------------------- validation
// flag bit 0: rowptr not monotone or wrong ends; bit 1: column out of range; bit 2:
// columns not strictly increasing within a row.
// One wave per row (wave m checks rowptr[m]); lanes stride over the row's entries, each
// comparing its column with the previous entry's.
__global__ void csr_validate_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                                    int64_t m, int64_t n, int64_t nnz, unsigned* flag) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i > m) return;
  if (i == m) {
    if (lane == 0 && (rowptr[0] != 0 || rowptr[m] != nnz)) atomicOr(flag, 1u);
    return;
  }
  const int64_t b = rowptr[i], e = rowptr[i + 1];
  if (e < b || b < 0 || e > nnz) {
    if (lane == 0) atomicOr(flag, 1u);
    return;
  }
  unsigned bad = 0;
  for (int64_t p = b + lane; p < e; p += 64) {
    const int64_t j = colind[p];
    if (j < 0 || j >= n) bad |= 2u;
    if (p > b && j <= static_cast<int64_t>(colind[p - 1])) bad |= 4u;
  }
  if (bad) atomicOr(flag, bad);
}

// ---------------------------------------------------------------- CSC copy
// Every entry packed as (row << 32) | FP32 bits of its value, in CSR order: one wave per
// row, lanes striding over the row's entries.
__global__ void pack_entries_kernel(const int64_t* __restrict__ rowptr, const float* __restrict__ vals, int64_t m,
                                    unsigned long long* __restrict__ ent) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= m) return;
  const unsigned long long hi = static_cast<unsigned long long>(i) << 32;
  for (int64_t p = rowptr[i] + (threadIdx.x & 63); p < rowptr[i + 1]; p += 64)
    ent[p] = hi | __float_as_uint(vals[p]);
}

// colptr[j] = first position of column j in the sorted column indices
__global__ void colptr_kernel(const int32_t* __restrict__ sorted, int64_t nnz, int64_t n, int64_t* __restrict__ colptr) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j > n) return;
  int64_t lo = 0, hi = nnz;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (sorted[mid] < j) lo = mid + 1; else hi = mid;
  }
  colptr[j] = lo;
}

// ---------------------------------------------------------------- sketch
// Row masks of the sparse-sign pattern: for row i of A (column i of G), word w bit b set
// when G(64 w + b, i) != 0; sign word bit set when that entry is -1.
__global__ void sign_masks_kernel(const uint8_t* __restrict__ rows, const uint8_t* __restrict__ signs, int64_t m,
                                  int z, int words, unsigned long long* __restrict__ masks) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  unsigned long long mk[kMaxWords] = {0, 0, 0, 0}, sg[kMaxWords] = {0, 0, 0, 0};
  const unsigned sb = signs[i];
  for (int t = 0; t < z; ++t) {
    const int r = rows[i * z + t];
    mk[r >> 6] |= 1ull << (r & 63);
    if ((sb >> t) & 1u) sg[r >> 6] |= 1ull << (r & 63);
  }
  for (int w = 0; w < words; ++w) {
    masks[(i * words + w) * 2] = mk[w];
    masks[(i * words + w) * 2 + 1] = sg[w];
  }
}

__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long v, int t) {
  const unsigned lo = __builtin_amdgcn_readlane(static_cast<unsigned>(v), t);
  const unsigned hi = __builtin_amdgcn_readlane(static_cast<unsigned>(v >> 32), t);
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

__device__ __forceinline__ double readlane_f64(double v, int t) {
  return __longlong_as_double(static_cast<long long>(readlane_u64(static_cast<unsigned long long>(__double_as_longlong(v)), t)));
}

// One wave per column j of A; lane l accumulates sketch row 64 w + l.  The column's
// entries are taken 64 at a time: each lane loads one entry (row index, value and, for
// the sparse-sign kind, the masks of that row of A) so that the 64 loads are in flight
// together, then the wave walks the 64 entries in order, each broadcast from its lane.
// Every row's sum runs over the entries in column order, one FP64 fma per entry.
template <int W, bool SIGN>
__global__ __launch_bounds__(64 * kSkWaves) void csc_sketch_kernel(
    const int64_t* __restrict__ colptr, const unsigned long long* __restrict__ ent,
    int64_t n, int c, const unsigned long long* __restrict__ masks, const uint16_t* __restrict__ Gt, int64_t ldgt,
    double* __restrict__ X0, int64_t ldx, double* __restrict__ norm_partials) {
  __shared__ double red[kSkWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * kSkWaves + wave;
  double acc[W];
#pragma unroll
  for (int w = 0; w < W; ++w) acc[w] = 0.0;
  if (j < n) {
    const int64_t b = colptr[j], e = colptr[j + 1];
    for (int64_t p0 = b; p0 < e; p0 += 64) {
      const int64_t p = p0 + lane;
      const bool valid = p < e;
      const unsigned long long en = valid ? ent[p] : 0ull;
      const int64_t i = static_cast<int64_t>(en >> 32);
      const double a = static_cast<double>(__uint_as_float(static_cast<unsigned>(en)));
      const int cnt = static_cast<int>(e - p0 < 64 ? e - p0 : 64);
      if constexpr (SIGN) {
        unsigned long long mk[W], sg[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
          mk[w] = valid ? masks[(i * W + w) * 2] : 0ull;
          sg[w] = valid ? masks[(i * W + w) * 2 + 1] : 0ull;
        }
        for (int t = 0; t < cnt; ++t) {
          const double at = readlane_f64(a, t);
#pragma unroll
          for (int w = 0; w < W; ++w) {
            const unsigned long long mt = readlane_u64(mk[w], t);
            const unsigned long long st = readlane_u64(sg[w], t);
            const double coef = ((mt >> lane) & 1ull) ? (((st >> lane) & 1ull) ? -1.0 : 1.0) : 0.0;
            acc[w] = fma(coef, at, acc[w]);
          }
        }
      } else {
        // 8 entries per round: their G rows are loaded before any of them is used
        for (int t0 = 0; t0 < cnt; t0 += 8) {
          double g[8][W], av[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int t = t0 + u < cnt ? t0 + u : t0;  // beyond the count: a repeat, weighted 0
            const int64_t it = static_cast<int64_t>(__builtin_amdgcn_readlane(static_cast<int>(i), t));
            av[u] = t0 + u < cnt ? readlane_f64(a, t) : 0.0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
              const int r = 64 * w + lane;
              g[u][w] = r < c ? static_cast<double>(__uint_as_float(static_cast<unsigned>(Gt[it * ldgt + r]) << 16))
                              : 0.0;
            }
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            if (t0 + u < cnt) {
#pragma unroll
              for (int w = 0; w < W; ++w) acc[w] = fma(g[u][w], av[u], acc[w]);
            }
          }
        }
      }
    }
  }
  double sq = 0.0;
  if (j < n) {
#pragma unroll
    for (int w = 0; w < W; ++w) {
      const int r = 64 * w + lane;
      if (r < c) {
        X0[r * ldx + j] = acc[w];
        sq += acc[w] * acc[w];
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
  if (lane == 0) red[wave] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kSkWaves; ++w) s += red[w];
    norm_partials[blockIdx.x] = s;
  }
}

// Sparse-sign sketch with lane-private accumulators in LDS, for c <= 128.  One wave per
// column j.  Lane l owns a private FP64 vector of the c sketch rows (LDS, row stride 65
// so that lanes stay on separate banks).  It walks the column's entries l, l+64, ... in
// order and adds +-a into the z rows its entry's row of A maps to (z <= 8 distinct
// rows, so each entry costs z read-add-writes instead of a pass over all c rows).  At
// the end lane r sums row r over the 64 private vectors in lane order.  Every sum has a
// fixed order, so the result is deterministic.
constexpr int kLdsStride = 65;

__global__ void csc_sketch_sign_lds_kernel(const int64_t* __restrict__ colptr, const unsigned long long* __restrict__ ent,
                                           int64_t n, int c,
                                           const uint8_t* __restrict__ rows, const uint8_t* __restrict__ signs, int z,
                                           double* __restrict__ X0, int64_t ldx, double* __restrict__ norm_partials) {
  extern __shared__ double sk_lds[];
  __shared__ double red[kSkWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int waves = blockDim.x >> 6;
  double* acc = sk_lds + static_cast<int64_t>(wave) * c * kLdsStride;
  const int64_t j = static_cast<int64_t>(blockIdx.x) * waves + wave;
  for (int r = 0; r < c; ++r) acc[r * kLdsStride + lane] = 0.0;
  if (j < n) {
    const int64_t b = colptr[j], e = colptr[j + 1];
    // software pipeline over this lane's entries: the row pattern of the next entry and
    // the index of the one after are loaded while the current entry is added in
    auto pattern = [&](int64_t i, unsigned long long* rr, unsigned* sb) {
      if (z == 8) {
        *rr = *reinterpret_cast<const unsigned long long*>(rows + i * 8);
      } else {
        unsigned long long v = 0;
        for (int t = 0; t < z; ++t) v |= static_cast<unsigned long long>(rows[i * z + t]) << (8 * t);
        *rr = v;
      }
      *sb = signs[i];
    };
    int64_t p0 = b + lane;
    int64_t i0 = 0, i1 = 0;
    double a0 = 0.0, a1 = 0.0;
    unsigned long long rr0 = 0;
    unsigned sb0 = 0;
    if (p0 < e) {
      {
        const unsigned long long en = ent[p0];
        i0 = static_cast<int64_t>(en >> 32);
        a0 = static_cast<double>(__uint_as_float(static_cast<unsigned>(en)));
      }
      pattern(i0, &rr0, &sb0);
    }
    int64_t p1 = p0 + 64;
    if (p1 < e) {
      {
        const unsigned long long en = ent[p1];
        i1 = static_cast<int64_t>(en >> 32);
        a1 = static_cast<double>(__uint_as_float(static_cast<unsigned>(en)));
      }
    }
    while (p0 < e) {
      unsigned long long rr1 = 0;
      unsigned sb1 = 0;
      if (p1 < e) pattern(i1, &rr1, &sb1);
      const int64_t p2 = p1 + 64;
      int64_t i2 = 0;
      double a2 = 0.0;
      if (p2 < e) {
        const unsigned long long en = ent[p2];
        i2 = static_cast<int64_t>(en >> 32);
        a2 = static_cast<double>(__uint_as_float(static_cast<unsigned>(en)));
      }
      for (int t = 0; t < z; ++t) {
        const int r = static_cast<int>((rr0 >> (8 * t)) & 0xFFu);
        // an LDS add on a slot only this lane touches: in program order, no result wait
        __hip_atomic_fetch_add(acc + r * kLdsStride + lane, ((sb0 >> t) & 1u) ? -a0 : a0, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
      }
      p0 = p1;
      a0 = a1;
      rr0 = rr1;
      sb0 = sb1;
      p1 = p2;
      i1 = i2;
      a1 = a2;
    }
  }
  // lane-private slots were written by their own lane only; the row sums read every lane
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  double sq = 0.0;
  if (j < n) {
    for (int r = lane; r < c; r += 64) {
      const double* row = acc + r * kLdsStride;
      double s = 0.0;
      for (int q = 0; q < 64; ++q) s += row[q];
      X0[r * ldx + j] = s;
      sq += s * s;
    }
  }
  for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
  if (lane == 0) red[wave] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < waves; ++w) s += red[w];
    norm_partials[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------- gathers
// Ct row t = column cols[t] of A (dense, length m); Ct is cleared first by the caller.
template <typename DstT>
__global__ void csc_scatter_cols_kernel(const int64_t* __restrict__ colptr, const unsigned long long* __restrict__ ent,
                                        const int64_t* __restrict__ cols, DstT* __restrict__ Ct, int64_t ldct) {
  const int t = blockIdx.y;
  const int64_t j = cols[t];
  const int64_t b = colptr[j], e = colptr[j + 1];
  for (int64_t p = b + static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; p < e;
       p += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const unsigned long long en = ent[p];
    Ct[t * ldct + static_cast<int64_t>(en >> 32)] = static_cast<DstT>(__uint_as_float(static_cast<unsigned>(en)));
  }
}

// R row t = row rows[t] of A (dense, length n); R is cleared first by the caller.
template <typename DstT>
__global__ void csr_scatter_rows_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                                        const float* __restrict__ vals, const int64_t* __restrict__ rows,
                                        DstT* __restrict__ R, int64_t ldr) {
  const int t = blockIdx.y;
  const int64_t i = rows[t];
  const int64_t b = rowptr[i], e = rowptr[i + 1];
  for (int64_t p = b + static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; p < e;
       p += static_cast<int64_t>(gridDim.x) * blockDim.x)
    R[t * ldr + colind[p]] = static_cast<DstT>(vals[p]);
}

// M(t, u) = A(I[t], J[u]) in FP64: binary search of column J[u] in row I[t]
__global__ void csr_cross_kernel(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
                                 const float* __restrict__ vals, const int64_t* __restrict__ I, int64_t rk,
                                 const int64_t* __restrict__ J, int64_t ck, double* __restrict__ M, int64_t ldm) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= rk * ck) return;
  const int64_t t = e / ck, u = e % ck;
  const int64_t i = I[t];
  const int32_t j = static_cast<int32_t>(J[u]);
  int64_t lo = rowptr[i], hi = rowptr[i + 1];
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (colind[mid] < j) lo = mid + 1; else hi = mid;
  }
  M[t * ldm + u] = (lo < rowptr[i + 1] && colind[lo] == j) ? static_cast<double>(vals[lo]) : 0.0;
}

template <typename T>
__global__ void zero_kernel(T* p, int64_t count) {
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
       e += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[e] = T(0);
}

template <typename T>
int zero(T* p, int64_t count, hipStream_t st) {
  if (count <= 0) return ICUR_OK;
  const int blocks = static_cast<int>(std::min<int64_t>((count + 255) / 256, 4096));
  hipLaunchKernelGGL(zero_kernel<T>, dim3(blocks), dim3(256), 0, st, p, count);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

int sort_bits(int64_t n) {
  int b = 1;
  while ((int64_t(1) << b) < n) ++b;
  return b;
}

}  // namespace

int csr_validate(const CsrMatrix& A, unsigned* flag_dev, hipStream_t st) {
  ICUR_TRY(launch_fill_u32(flag_dev, 1, 0u, st));
  const int64_t waves = A.m + 1;
  hipLaunchKernelGGL(csr_validate_kernel, dim3(static_cast<unsigned>((waves + 3) / 4)), dim3(256), 0, st, A.rowptr,
                     A.colind, A.m, A.n, A.nnz, flag_dev);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

size_t csc_workspace_bytes(int64_t nnz, int64_t n) {
  size_t tmp = 0;
  const int64_t cnt = std::max<int64_t>(nnz, 1);
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, static_cast<const int32_t*>(nullptr),
                                           static_cast<int32_t*>(nullptr),
                                           static_cast<const unsigned long long*>(nullptr),
                                           static_cast<unsigned long long*>(nullptr), static_cast<int>(cnt), 0, 31);
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  // colptr, packed entries, then scratch: sorted keys, packed entries in CSR order, sort temp
  return al((n + 1) * 8) + al(cnt * 8) + al(cnt * 4) + al(cnt * 8) + al(tmp);
}

int csc_build(const CsrMatrix& A, CscCopy* out, void* ws, size_t ws_bytes, hipStream_t st) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  if (ws_bytes < csc_workspace_bytes(A.nnz, A.n)) return arg_error("csc: workspace too small");
  const int64_t cnt = std::max<int64_t>(A.nnz, 1);
  char* p = static_cast<char*>(ws);
  out->colptr = reinterpret_cast<int64_t*>(p);
  p += al((A.n + 1) * 8);
  unsigned long long* ent_sorted = reinterpret_cast<unsigned long long*>(p);
  out->ent = ent_sorted;
  p += al(cnt * 8);
  int32_t* keys = reinterpret_cast<int32_t*>(p);
  p += al(cnt * 4);
  unsigned long long* ent_rows = reinterpret_cast<unsigned long long*>(p);
  p += al(cnt * 8);
  void* tmp = p;
  size_t tmp_bytes = ws_bytes - static_cast<size_t>(p - static_cast<char*>(ws));
  if (A.nnz > 0) {
    // pack (row, value) in CSR order, then a stable sort by column carries the packed
    // entries along: rows stay increasing within each column
    hipLaunchKernelGGL(pack_entries_kernel, dim3(static_cast<unsigned>((A.m + 3) / 4)), dim3(256), 0, st, A.rowptr,
                       A.vals, A.m, ent_rows);
    ICUR_HIP(hipGetLastError());
    ICUR_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, A.colind, keys, ent_rows, ent_sorted,
                                                static_cast<int>(A.nnz), 0, sort_bits(A.n), st));
  }
  hipLaunchKernelGGL(colptr_kernel, dim3(static_cast<unsigned>((A.n + 1 + 255) / 256)), dim3(256), 0, st, keys,
                     A.nnz, A.n, out->colptr);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

size_t csr_sketch_aux_bytes(int64_t m, int64_t c) {
  const int64_t words = (c + 63) / 64;
  return std::max<size_t>(static_cast<size_t>(m) * words * 16, static_cast<size_t>(m) * ((c + 7) / 8 * 8) * 2) +
         static_cast<size_t>(m) * 9 + 256;
}

int csr_sketch(const CscCopy& csc, int64_t m, int64_t n, int64_t c, int kind, uint64_t seed, int zeta, double* X0,
               int64_t ldx, double* norm_partials, int* nparts, void* aux, hipStream_t st) {
  if (c > kMaxWords * 64) return arg_error("CSR sketch needs c <= 256");
  const int W = static_cast<int>((c + 63) / 64);
  const unsigned blocks = static_cast<unsigned>((n + kSkWaves - 1) / kSkWaves);
  char* p = static_cast<char*>(aux);
  if (kind == ICUR_SKETCH_SPARSE_SIGN && c <= 128) {
    const int z = std::min<int>(zeta, static_cast<int>(c));
    uint8_t* rows = reinterpret_cast<uint8_t*>(p);
    uint8_t* signs = rows + static_cast<size_t>(m) * 8;
    ICUR_TRY(launch_sparse_sign(seed, c, m, zeta, rows, signs, nullptr, 0, st));
    const size_t per_wave = static_cast<size_t>(c) * kLdsStride * sizeof(double);
    const int waves = static_cast<int>(std::max<size_t>(1, std::min<size_t>(kSkWaves, (160 * 1024) / per_wave)));
    const size_t lds = per_wave * waves;
    if (lds > 64 * 1024)
      ICUR_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(csc_sketch_sign_lds_kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
    const unsigned lblocks = static_cast<unsigned>((n + waves - 1) / waves);
    hipLaunchKernelGGL(csc_sketch_sign_lds_kernel, dim3(lblocks), dim3(64 * waves), lds, st, csc.colptr, csc.ent, n,
                       static_cast<int>(c), rows, signs, z, X0, ldx, norm_partials);
    ICUR_HIP(hipGetLastError());
    if (nparts) *nparts = static_cast<int>(lblocks);
    return ICUR_OK;
  }
  if (kind == ICUR_SKETCH_SPARSE_SIGN) {
    const int z = std::min<int>(zeta, static_cast<int>(c));
    unsigned long long* masks = reinterpret_cast<unsigned long long*>(p);
    uint8_t* rows = reinterpret_cast<uint8_t*>(p + static_cast<size_t>(m) * W * 16);
    uint8_t* signs = rows + static_cast<size_t>(m) * 8;
    ICUR_TRY(launch_sparse_sign(seed, c, m, zeta, rows, signs, nullptr, 0, st));
    hipLaunchKernelGGL(sign_masks_kernel, dim3(static_cast<unsigned>((m + 255) / 256)), dim3(256), 0, st, rows, signs,
                       m, z, W, masks);
    ICUR_HIP(hipGetLastError());
    switch (W) {
#define ICUR_CSR_SIGN(X)                                                                                        \
  case X:                                                                                                       \
    hipLaunchKernelGGL((csc_sketch_kernel<X, true>), dim3(blocks), dim3(64 * kSkWaves), 0, st, csc.colptr,       \
                       csc.ent, n, static_cast<int>(c), masks, nullptr, 0, X0, ldx, norm_partials);           \
    break;
      ICUR_CSR_SIGN(1)
      ICUR_CSR_SIGN(2)
      ICUR_CSR_SIGN(3)
      ICUR_CSR_SIGN(4)
#undef ICUR_CSR_SIGN
    }
  } else {
    const int64_t ldgt = (c + 7) / 8 * 8;
    uint16_t* Gt = reinterpret_cast<uint16_t*>(p);
    ICUR_TRY(launch_gaussian_G_strided(seed, c, m, Gt, 1, ldgt, st));
    switch (W) {
#define ICUR_CSR_GAUSS(X)                                                                                       \
  case X:                                                                                                       \
    hipLaunchKernelGGL((csc_sketch_kernel<X, false>), dim3(blocks), dim3(64 * kSkWaves), 0, st, csc.colptr,      \
                       csc.ent, n, static_cast<int>(c), nullptr, Gt, ldgt, X0, ldx, norm_partials);           \
    break;
      ICUR_CSR_GAUSS(1)
      ICUR_CSR_GAUSS(2)
      ICUR_CSR_GAUSS(3)
      ICUR_CSR_GAUSS(4)
#undef ICUR_CSR_GAUSS
    }
  }
  ICUR_HIP(hipGetLastError());
  if (nparts) *nparts = static_cast<int>(blocks);
  return ICUR_OK;
}

int csr_max_norm_partials(int64_t n) { return static_cast<int>(n); }  // one wave per block at most

template <typename DstT>
int csc_gather_cols_T_t(const CscCopy& csc, int64_t m, const int64_t* cols, int64_t k, DstT* Ct, int64_t ldct,
                        hipStream_t st) {
  if (k <= 0) return ICUR_OK;
  if (ldct == m) {
    ICUR_TRY(zero(Ct, k * m, st));
  } else {
    for (int64_t t = 0; t < k; ++t) ICUR_TRY(zero(Ct + t * ldct, m, st));
  }
  hipLaunchKernelGGL(csc_scatter_cols_kernel<DstT>, dim3(8, static_cast<unsigned>(k)), dim3(256), 0, st, csc.colptr,
                     csc.ent, cols, Ct, ldct);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}
int csc_gather_cols_T(const CscCopy& csc, int64_t m, const int64_t* cols, int64_t k, float* Ct, int64_t ldct,
                      hipStream_t st) {
  return csc_gather_cols_T_t(csc, m, cols, k, Ct, ldct, st);
}
int csc_gather_cols_T(const CscCopy& csc, int64_t m, const int64_t* cols, int64_t k, double* Ct, int64_t ldct,
                      hipStream_t st) {
  return csc_gather_cols_T_t(csc, m, cols, k, Ct, ldct, st);
}

template <typename DstT>
int csr_gather_rows_t(const CsrMatrix& A, const int64_t* rows, int64_t k, DstT* R, int64_t ldr, hipStream_t st) {
  if (k <= 0) return ICUR_OK;
  if (ldr == A.n) {
    ICUR_TRY(zero(R, k * A.n, st));
  } else {
    for (int64_t t = 0; t < k; ++t) ICUR_TRY(zero(R + t * ldr, A.n, st));
  }
  hipLaunchKernelGGL(csr_scatter_rows_kernel<DstT>, dim3(4, static_cast<unsigned>(k)), dim3(256), 0, st, A.rowptr,
                     A.colind, A.vals, rows, R, ldr);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}
int csr_gather_rows(const CsrMatrix& A, const int64_t* rows, int64_t k, float* R, int64_t ldr, hipStream_t st) {
  return csr_gather_rows_t(A, rows, k, R, ldr, st);
}
int csr_gather_rows(const CsrMatrix& A, const int64_t* rows, int64_t k, double* R, int64_t ldr, hipStream_t st) {
  return csr_gather_rows_t(A, rows, k, R, ldr, st);
}

int csr_gather_cross(const CsrMatrix& A, const int64_t* I, int64_t rk, const int64_t* J, int64_t ck, double* M,
                     int64_t ldm, hipStream_t st) {
  if (rk <= 0 || ck <= 0) return ICUR_OK;
  const int64_t total = rk * ck;
  hipLaunchKernelGGL(csr_cross_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, st, A.rowptr,
                     A.colind, A.vals, I, rk, J, ck, M, ldm);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

}  // namespace icur
