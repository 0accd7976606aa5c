// Instantiates the wide product kernels with FP32 outputs (the CUR factors).
#include "icur_wide_kernel.h"

namespace icur {
namespace wide {

KernelFn pick_kernel_f32(int mt, int wt, int bt) { return pick_kernel_t<float>(mt, wt, bt); }

int launch_reduce_f32(const double* partial, int nsplit, int64_t M, int64_t N, const void* X, int64_t ldx,
                      int subtract, void* OUT, int64_t ldo, double* norm_partials, int blocks, hipStream_t st) {
  hipLaunchKernelGGL(splitk_reduce_kernel<float>, dim3(blocks), dim3(256), 0, st, partial, nsplit, M, N,
                     static_cast<const float*>(X), ldx, subtract, static_cast<float*>(OUT), ldo, norm_partials);
  ICUR_HIP(hipGetLastError());
  return ICUR_OK;
}

}  // namespace wide
}  // namespace icur
