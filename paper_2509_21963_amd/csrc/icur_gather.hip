// Gathers of the CUR factors C = A(:,J), R = A(I,:) and of the small blocks of the core
// (Alg. 1 update step; §1.1 Notation), plus mask and fill helpers.
//
// C is kept transposed (C^T: one contiguous row of length m per selected column), so the
// row residual reads it with the same coalesced layout as every other wide product.  A
// column of a row-major A is a strided gather: each element costs one cache line, which
// is inherent to the layout; the writes are coalesced.  Rows of A are copied with 16-byte
// loads when alignment allows.
#include <algorithm>

#include "icur_internal.h"

namespace icur {
namespace {

template <typename DstT>
__global__ void gather_cols_T_kernel(const float* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                     const int64_t* __restrict__ cols, int64_t k,
                                     DstT* __restrict__ Ct, int64_t ldct) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t t = blockIdx.y;
  if (i >= m || t >= k) return;
  int64_t j = cols[t];
  j = j < 0 ? 0 : (j >= n ? n - 1 : j);
  Ct[t * ldct + i] = static_cast<DstT>(A[i * lda + j]);
}

__global__ void gather_rows_kernel(const float* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                   const int64_t* __restrict__ rows, int64_t k,
                                   float* __restrict__ R, int64_t ldr, int vec4) {
  const int64_t t = blockIdx.y;
  if (t >= k) return;
  int64_t i = rows[t];
  i = i < 0 ? 0 : (i >= m ? m - 1 : i);
  const float* src = A + i * lda;
  float* dst = R + t * ldr;
  if (vec4) {
    const int64_t n4 = n / 4;
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < n4;
         j += static_cast<int64_t>(gridDim.x) * blockDim.x)
      reinterpret_cast<float4*>(dst)[j] = reinterpret_cast<const float4*>(src)[j];
    for (int64_t j = 4 * n4 + static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < n;
         j += static_cast<int64_t>(gridDim.x) * blockDim.x)
      dst[j] = src[j];
  } else {
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < n;
         j += static_cast<int64_t>(gridDim.x) * blockDim.x)
      dst[j] = src[j];
  }
}

__global__ void gather_rows_f64_kernel(const float* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                       const int64_t* __restrict__ rows, int64_t k, double* __restrict__ R,
                                       int64_t ldr) {
  const int64_t t = blockIdx.y;
  if (t >= k) return;
  int64_t i = rows[t];
  i = i < 0 ? 0 : (i >= m ? m - 1 : i);
  const float* src = A + i * lda;
  double* dst = R + t * ldr;
  for (int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < n;
       j += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[j] = static_cast<double>(src[j]);
}

template <typename SrcT>
__global__ void gather_f64_kernel(const SrcT* __restrict__ src, int64_t lds,
                                  const int64_t* __restrict__ rows, int64_t rk,
                                  const int64_t* __restrict__ cols, int64_t ck, int trans,
                                  double* __restrict__ dst, int64_t ldd) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= rk * ck) return;
  // consecutive threads walk the source's contiguous dimension when no column index list
  // is given, else the destination's
  const int64_t i = e / ck, j = e % ck;
  const int64_t si = rows ? rows[i] : i;
  const int64_t sj = cols ? cols[j] : j;
  const double v = static_cast<double>(src[si * lds + sj]);
  if (trans)
    dst[j * ldd + i] = v;
  else
    dst[i * ldd + j] = v;
}

// The end of an iteration: the k new columns and rows are masked out of later selections
// and appended to J and I.
__global__ void commit_block_kernel(uint8_t* colmask, uint8_t* rowmask, const int64_t* Jk, const int64_t* Ik,
                                    int64_t k, int64_t* Jall, int64_t* Iall) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < k) {
    const int64_t j = Jk[t], i = Ik[t];
    colmask[j] = 1;
    rowmask[i] = 1;
    Jall[t] = j;
    Iall[t] = i;
  }
}

__global__ void fill_u8_kernel(uint8_t* p, int64_t n, uint8_t v) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

__global__ void fill_u32_kernel(unsigned* p, int64_t n, unsigned v) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

unsigned blocks_for(int64_t n, int64_t per = 256, int64_t cap = 4096) {
  int64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return static_cast<unsigned>(b);
}

}  // namespace

template <typename DstT>
int gather_cols_T_t(const float* A, int64_t m, int64_t n, int64_t lda, const int64_t* cols, int64_t k, DstT* Ct,
                    int64_t ldct, hipStream_t st) {
  if (k <= 0 || m <= 0) return ICUR_OK;
  if (k > 65535) return arg_error("gather: more than 65535 columns at once");
  dim3 grid(static_cast<unsigned>((m + 255) / 256), static_cast<unsigned>(k));
  hipLaunchKernelGGL(gather_cols_T_kernel<DstT>, grid, dim3(256), 0, st, A, m, n, lda, cols, k, Ct, ldct);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

int launch_gather_cols_T(const float* A, int64_t m, int64_t n, int64_t lda, const int64_t* cols,
                         int64_t k, float* Ct, int64_t ldct, hipStream_t st) {
  return gather_cols_T_t(A, m, n, lda, cols, k, Ct, ldct, st);
}

int launch_gather_cols_T(const float* A, int64_t m, int64_t n, int64_t lda, const int64_t* cols,
                         int64_t k, double* Ct, int64_t ldct, hipStream_t st) {
  return gather_cols_T_t(A, m, n, lda, cols, k, Ct, ldct, st);
}

int launch_gather_rows(const float* A, int64_t m, int64_t n, int64_t lda, const int64_t* rows,
                       int64_t k, double* R, int64_t ldr, hipStream_t st) {
  if (k <= 0 || n <= 0) return ICUR_OK;
  if (k > 65535) return arg_error("gather: more than 65535 rows at once");
  const unsigned bx = blocks_for(n, 256, 64);
  hipLaunchKernelGGL(gather_rows_f64_kernel, dim3(bx, static_cast<unsigned>(k)), dim3(256), 0, st, A, m, n, lda,
                     rows, k, R, ldr);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

int launch_gather_rows(const float* A, int64_t m, int64_t n, int64_t lda, const int64_t* rows,
                       int64_t k, float* R, int64_t ldr, hipStream_t st) {
  if (k <= 0 || n <= 0) return ICUR_OK;
  if (k > 65535) return arg_error("gather: more than 65535 rows at once");
  const int vec4 = ((lda & 3) == 0) && ((ldr & 3) == 0) &&
                   ((reinterpret_cast<uintptr_t>(A) & 15) == 0) &&
                   ((reinterpret_cast<uintptr_t>(R) & 15) == 0);
  const unsigned bx = blocks_for(vec4 ? (n + 3) / 4 : n, 256, 64);
  hipLaunchKernelGGL(gather_rows_kernel, dim3(bx, static_cast<unsigned>(k)), dim3(256), 0, st, A, m,
                     n, lda, rows, k, R, ldr, vec4);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

template <typename SrcT>
int gather_f64_t(const SrcT* src, int64_t lds, const int64_t* rows, int64_t rk, const int64_t* cols,
                 int64_t ck, bool trans, double* dst, int64_t ldd, hipStream_t st) {
  if (rk <= 0 || ck <= 0) return ICUR_OK;
  const int64_t total = rk * ck;
  hipLaunchKernelGGL(gather_f64_kernel<SrcT>, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0,
                     st, src, lds, rows, rk, cols, ck, trans ? 1 : 0, dst, ldd);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

int launch_gather_f64(const float* src, int64_t lds, const int64_t* rows, int64_t rk,
                      const int64_t* cols, int64_t ck, bool trans, double* dst, int64_t ldd,
                      hipStream_t st) {
  return gather_f64_t(src, lds, rows, rk, cols, ck, trans, dst, ldd, st);
}

int launch_gather_f64(const double* src, int64_t lds, const int64_t* rows, int64_t rk,
                      const int64_t* cols, int64_t ck, bool trans, double* dst, int64_t ldd,
                      hipStream_t st) {
  return gather_f64_t(src, lds, rows, rk, cols, ck, trans, dst, ldd, st);
}

int launch_commit_block(uint8_t* colmask, uint8_t* rowmask, const int64_t* Jk, const int64_t* Ik, int64_t k,
                        int64_t* Jall, int64_t* Iall, hipStream_t st) {
  if (k <= 0) return ICUR_OK;
  hipLaunchKernelGGL(commit_block_kernel, dim3(static_cast<unsigned>((k + 255) / 256)), dim3(256), 0, st, colmask,
                     rowmask, Jk, Ik, k, Jall, Iall);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

namespace {
// The read-backs of a call (status words, scalars, results) as stores into host-mapped
// pinned memory, all segments in one launch; sizes and offsets are multiples of 4 bytes.
__global__ void to_host_kernel(const HostSegs segs, unsigned* __restrict__ dst) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int s = 0; s < segs.n; ++s) {
    const unsigned* src = static_cast<const unsigned*>(segs.seg[s].src);
    unsigned* d = dst + segs.seg[s].dst_off / 4;
    const int64_t words = segs.seg[s].bytes / 4;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < words; e += stride)
      d[e] = src[e];
  }
}
// Small read-backs: one workgroup copies, then publishes `seq` in a host-visible flag
// after its stores, so the host can poll the flag instead of waiting for the stream.
__global__ __launch_bounds__(256) void to_host_flag_kernel(const HostSegs segs, unsigned* __restrict__ dst,
                                                          unsigned* flag, unsigned seq) {
  for (int s = 0; s < segs.n; ++s) {
    const unsigned* src = static_cast<const unsigned*>(segs.seg[s].src);
    unsigned* d = dst + segs.seg[s].dst_off / 4;
    const int64_t words = segs.seg[s].bytes / 4;
    for (int64_t e = threadIdx.x; e < words; e += blockDim.x) d[e] = src[e];
  }
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}
// End of an iteration in one workgroup: the column-residual norm from its partials (the
// fixed order of the plain partial reduction: thread t sums partials t, t + 256, ..., then
// a butterfly within each wave and the four waves in order), the commit of the block's
// indices, and the scalar record copied to host-mapped memory with an optional flag.
__global__ __launch_bounds__(256) void iteration_end_kernel(const double* partials, int nparts, double* norm_out,
                                                            uint8_t* colmask, uint8_t* rowmask, const int64_t* Jk,
                                                            const int64_t* Ik, int64_t k, int64_t* Jall,
                                                            int64_t* Iall, const unsigned* rec, int rec_words,
                                                            unsigned* host_dst, unsigned* flag, unsigned seq) {
  __shared__ double red[4];
  const int tid = threadIdx.x;
  double v = 0.0;
  for (int i = tid; i < nparts; i += blockDim.x) v += partials[i];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  for (int64_t t = tid; t < k; t += blockDim.x) {
    const int64_t j = Jk[t], i = Ik[t];
    colmask[j] = 1;
    rowmask[i] = 1;
    Jall[t] = j;
    Iall[t] = i;
  }
  if (tid == 0) {
    double sum = 0.0;
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) sum += red[w];
    *norm_out = sum;
    // the record holds norm_out: thread 0 reads its own store back
    for (int e = 0; e < rec_words; ++e) host_dst[e] = rec[e];
    if (flag) {
      __threadfence_system();
      __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}
}  // namespace

int launch_iteration_end(const double* partials, int nparts, double* norm_out, uint8_t* colmask, uint8_t* rowmask,
                         const int64_t* Jk, const int64_t* Ik, int64_t k, int64_t* Jall, int64_t* Iall,
                         const void* rec, int64_t rec_bytes, void* host_dev, unsigned* flag_dev, unsigned seq,
                         hipStream_t st) {
  if (rec_bytes % 4 != 0 || rec_bytes > 4096) return arg_error("iteration end: bad record size");
  if (k < 0 || nparts < 0) return arg_error("iteration end: negative size");
  hipLaunchKernelGGL(iteration_end_kernel, dim3(1), dim3(256), 0, st, partials, nparts, norm_out, colmask, rowmask,
                     Jk, Ik, k, Jall, Iall, static_cast<const unsigned*>(rec), static_cast<int>(rec_bytes / 4),
                     static_cast<unsigned*>(host_dev), flag_dev, seq);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

int launch_to_host_flag(const HostSegs& segs, void* host_dev, unsigned* flag_dev, unsigned seq, hipStream_t st) {
  if (segs.n < 1 || segs.n > kMaxHostSegs) return arg_error("to_host: bad segment list");
  for (int s = 0; s < segs.n; ++s)
    if (segs.seg[s].bytes % 4 != 0 || segs.seg[s].dst_off % 4 != 0) return arg_error("to_host: unaligned segment");
  hipLaunchKernelGGL(to_host_flag_kernel, dim3(1), dim3(256), 0, st, segs, static_cast<unsigned*>(host_dev), flag_dev,
                     seq);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

int launch_to_host(const HostSegs& segs, void* host_dev, hipStream_t st) {
  int64_t words = 0;
  for (int s = 0; s < segs.n; ++s) {
    if (segs.seg[s].bytes % 4 != 0 || segs.seg[s].dst_off % 4 != 0) return arg_error("to_host: unaligned segment");
    words = std::max<int64_t>(words, segs.seg[s].bytes / 4);
  }
  if (segs.n < 1 || segs.n > kMaxHostSegs || words == 0) return arg_error("to_host: bad segment list");
  const unsigned blocks = static_cast<unsigned>(std::min<int64_t>((words + 255) / 256, 256));
  hipLaunchKernelGGL(to_host_kernel, dim3(blocks), dim3(256), 0, st, segs, static_cast<unsigned*>(host_dev));
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

namespace {
// Per-workgroup FP64 partial sums of a^2 over an m x n FP32 matrix (leading dimension
// lda): workgroup g takes rows g, g + G, ...; threads stride the row with 4-element
// loads where the row is aligned.  One partial per workgroup, in a fixed order.
__global__ __launch_bounds__(256) void sumsq_f32_kernel(const float* __restrict__ A, int64_t m, int64_t n,
                                                        int64_t lda, double* __restrict__ partials) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
    const float* row = A + i * lda;
    const int64_t head = (reinterpret_cast<uintptr_t>(row) & 15) ? std::min<int64_t>(n, (16 - (reinterpret_cast<uintptr_t>(row) & 15)) / 4) : 0;
    for (int64_t j = threadIdx.x; j < head; j += blockDim.x) acc += static_cast<double>(row[j]) * row[j];
    const int64_t nv = (n - head) / 4;
    const float4* v4 = reinterpret_cast<const float4*>(row + head);
    for (int64_t j = threadIdx.x; j < nv; j += blockDim.x) {
      const float4 v = v4[j];
      acc += static_cast<double>(v.x) * v.x + static_cast<double>(v.y) * v.y + static_cast<double>(v.z) * v.z +
             static_cast<double>(v.w) * v.w;
    }
    for (int64_t j = head + nv * 4 + threadIdx.x; j < n; j += blockDim.x) acc += static_cast<double>(row[j]) * row[j];
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}
}  // namespace

int launch_sumsq_f32(const float* A, int64_t m, int64_t n, int64_t lda, double* partials, int* nparts,
                     hipStream_t st) {
  if (m < 0 || n < 0 || (m > 0 && lda < n)) return arg_error("sum of squares: bad shape");
  const int blocks = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(m, kSumsqMaxParts)));
  hipLaunchKernelGGL(sumsq_f32_kernel, dim3(blocks), dim3(256), 0, st, A, m, n, lda, partials);
  ICUR_HIP(hipGetLastError());
  *nparts = blocks;
  return ICUR_OK;
}

int launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t st) {
  if (n <= 0) return ICUR_OK;
  hipLaunchKernelGGL(fill_u8_kernel, dim3(blocks_for(n)), dim3(256), 0, st, p, n, v);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

int launch_fill_u32(unsigned* p, int64_t n, unsigned v, hipStream_t st) {
  if (n <= 0) return ICUR_OK;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(n)), dim3(256), 0, st, p, n, v);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

}  // namespace icur
