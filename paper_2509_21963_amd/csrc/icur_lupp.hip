// Index selection by LU with partial pivoting (§3.2.1 column selection on the sketched
// residual, §3.2.2 row selection on the row residual): the pivot order of LUPP applied to
// T = X^T (N candidates x K), first `steps` pivots only.
//
// Exactness.  The arithmetic is FP64 and each candidate entry receives the textbook
// right-looking updates T[i][j] <- T[i][j] - (l_i * u_j), product rounded before the
// subtraction (this file is compiled with contraction off), in step order.  The schedule
// below is blocked and deferred, but every element sees exactly the same sequence of
// rounded operations as the unblocked algorithm, so the pivots equal those of a plain
// FP64 LUPP on the same input, ties going to the lowest index.
//
// Schedule.  One persistent cooperative grid (<= one workgroup per CU).  Candidate rows
// are spread over the grid, R rows per thread, and the current 16-column panel of each
// row lives in registers.  Each pivot step is
//   local argmax (wave shuffle + LDS)  ->  publish (|value|, index, panel row) into a
//   per-workgroup slot  ->  one grid barrier  ->  every workgroup reduces the slots
//   itself, reads the winner's panel row and applies the rank-one update.
// At a panel boundary each workgroup rebuilds the previous pivots' rows restricted to the
// new panel (a right-looking triangular recurrence in LDS, same operation order) and
// applies all previous updates to its own rows, reading the stored multipliers.
#include <algorithm>
#include <utility>

#include "icur_internal.h"

#pragma clang fp contract(off)

namespace icur {
namespace {

constexpr int kPW = 16;          // panel width
constexpr int kLT = 256;         // threads per workgroup
constexpr int kMaxSteps = 1024;  // LDS holds the previous pivot rows of one panel
constexpr unsigned kSpinLimit = 1u << 22;

struct Slot {
  double val;  // |best entry| of the workgroup, -1 if it has no eligible candidate
  long long idx;
  double row[kPW];
};

struct Args {
  const void* X;  // FP32 or FP64 (InT)
  int64_t ldx;
  int K;
  int N;
  int steps;
  const uint8_t* excl;
  double* L;  // steps x N multipliers
  Slot* slots;  // 2 x gridDim.x
  unsigned* bar;
  int* status;  // [0] pivots found, [1] fault flag
  int64_t* piv;
};

// Calls f(std::integral_constant<int, 0>) ... f(std::integral_constant<int, N-1>): the
// step index is a compile-time constant in every call, so per-step register indexing
// stays static whatever the compiler decides about loop unrolling.
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

// Returns false when the barrier could not complete (fault); all threads agree.  The
// arrival is a release add and the wait an acquire, both at device scope, so the slot
// writes before the barrier are visible to every workgroup after it.
__device__ bool grid_barrier(unsigned* bar, unsigned target, int* fault, int* flag_lds) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    int ok = 1;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 255u) == 0 &&
          __hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        ok = 0;
        break;
      }
      if (spins > kSpinLimit) {
        atomicExch(fault, 1);
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *flag_lds = ok;
  }
  __syncthreads();
  return *flag_lds != 0;
}

template <int R, typename InT>
__global__ __launch_bounds__(kLT, 1) void lupp_kernel(const Args a) {
  const InT* Xin = static_cast<const InT*>(a.X);
  extern __shared__ double dyn[];
  double* Upan = dyn;                                               // steps x kPW
  int* pivs = reinterpret_cast<int*>(dyn + static_cast<size_t>(a.steps) * kPW);  // steps
  __shared__ double red_v[kLT / 64];
  __shared__ int red_i[kLT / 64];
  __shared__ int red_w[kLT / 64];
  __shared__ double u_sh[kPW];
  __shared__ int bcast_i;
  __shared__ int bcast_w;
  __shared__ double bcast_v;
  __shared__ int flag;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int G = gridDim.x;
  const int N = a.N;

  int rowid[R];
  unsigned alive = 0;  // bit r: row r is a valid, eligible, not yet chosen candidate
#pragma unroll
  for (int r = 0; r < R; ++r) {
    rowid[r] = (static_cast<int>(blockIdx.x) * R + r) * kLT + tid;
    if (rowid[r] < N && !(a.excl && a.excl[rowid[r]])) alive |= 1u << r;
  }
  double x[R][kPW];
  unsigned epoch = 0;
  int found = 0;
  bool stop = false;

  for (int t0 = 0; t0 < a.steps && !stop; t0 += kPW) {
    const int pw = min(kPW, a.steps - t0);
    // (1) previous pivot rows restricted to this panel, rebuilt in LDS with the same
    //     sequence of rounded updates they received in the unblocked algorithm.
    if (t0 > 0) {
      for (int e = tid; e < t0 * kPW; e += kLT) {
        const int k = e / kPW, jj = e % kPW;
        Upan[e] = (jj < pw) ? static_cast<double>(Xin[static_cast<int64_t>(t0 + jj) * a.ldx + pivs[k]]) : 0.0;
      }
      __syncthreads();
      for (int kp = 0; kp + 1 < t0; ++kp) {
        const int rows_left = t0 - kp - 1;
        for (int e = tid; e < rows_left * pw; e += kLT) {
          const int k = kp + 1 + e / pw, jj = e % pw;
          const double l = a.L[static_cast<int64_t>(kp) * N + pivs[k]];
          const double prod = l * Upan[kp * kPW + jj];
          Upan[k * kPW + jj] = Upan[k * kPW + jj] - prod;
        }
        __syncthreads();
      }
    }
    // (2) own rows: load the panel and apply all previous updates in step order.
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const bool live = (alive >> r) & 1u;
#pragma unroll
      for (int jj = 0; jj < kPW; ++jj)
        x[r][jj] = (live && jj < pw) ? static_cast<double>(Xin[static_cast<int64_t>(t0 + jj) * a.ldx + rowid[r]]) : 0.0;
    }
    for (int kp = 0; kp < t0; ++kp) {
      double u[kPW];
#pragma unroll
      for (int jj = 0; jj < kPW; ++jj) u[jj] = Upan[kp * kPW + jj];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const bool live = (alive >> r) & 1u;
        const double l = live ? a.L[static_cast<int64_t>(kp) * N + rowid[r]] : 0.0;
#pragma unroll
        for (int jj = 0; jj < kPW; ++jj) {
          const double prod = l * u[jj];
          x[r][jj] = x[r][jj] - prod;
        }
      }
    }
    // (3) the pivot steps of this panel (every register index is static).
    static_for<kPW>([&](auto ttc) {
      constexpr int tt = decltype(ttc)::value;
      if (!stop && tt < pw) {
        const int t = t0 + tt;
        // (a) local argmax
        double bv = -1.0;
        int bi = 0x7fffffff;
        int br = -1;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double v = fabs(x[r][tt]);
          if (((alive >> r) & 1u) && better(v, rowid[r], bv, bi)) {
            bv = v;
            bi = rowid[r];
            br = r;
          }
        }
        double wv = bv;
        int wi = bi;
        for (int off = 32; off > 0; off >>= 1) {
          const double ov = __shfl_xor(wv, off, 64);
          const int oi = __shfl_xor(wi, off, 64);
          if (better(ov, oi, wv, wi)) {
            wv = ov;
            wi = oi;
          }
        }
        if (lane == 0) {
          red_v[wave] = wv;
          red_i[wave] = wi;
        }
        __syncthreads();
        if (tid == 0) {
          double gv = red_v[0];
          int gi = red_i[0];
          for (int w = 1; w < kLT / 64; ++w)
            if (better(red_v[w], red_i[w], gv, gi)) {
              gv = red_v[w];
              gi = red_i[w];
            }
          bcast_v = gv;
          bcast_i = gi;
        }
        __syncthreads();
        // (b) publish: the owner writes its panel row, thread 0 the header.
        Slot* slot = a.slots + (t & 1) * G + blockIdx.x;
        if (bcast_v >= 0.0 && br >= 0 && bi == bcast_i) {
          // select row br with bit masks (an indexed read x[br] would force x into memory)
          unsigned long long pub[kPW];
#pragma unroll
          for (int jj = 0; jj < kPW; ++jj) pub[jj] = 0ull;
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const unsigned long long mask = (r == br) ? ~0ull : 0ull;
#pragma unroll
            for (int jj = 0; jj < kPW; ++jj)
              pub[jj] |= static_cast<unsigned long long>(__double_as_longlong(x[r][jj])) & mask;
          }
#pragma unroll
          for (int jj = 0; jj < kPW; ++jj) slot->row[jj] = __longlong_as_double(static_cast<long long>(pub[jj]));
          __threadfence();
        }
        __syncthreads();
        if (tid == 0) {
          slot->val = bcast_v;
          slot->idx = bcast_i;
        }
        // (c) one grid barrier per pivot step
        ++epoch;
        if (!grid_barrier(a.bar, epoch * static_cast<unsigned>(G), a.status + 1, &flag)) stop = true;
        if (!stop) {
          // (d) every workgroup reduces the published candidates itself
          double cv = -1.0;
          int ci = 0x7fffffff, cw = -1;
          for (int w = tid; w < G; w += kLT) {
            const Slot* s = a.slots + (t & 1) * G + w;
            const double v = __hip_atomic_load(&s->val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int i = static_cast<int>(__hip_atomic_load(&s->idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            if (v >= 0.0 && better(v, i, cv, ci)) {
              cv = v;
              ci = i;
              cw = w;
            }
          }
          for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(cv, off, 64);
            const int oi = __shfl_xor(ci, off, 64);
            const int ow = __shfl_xor(cw, off, 64);
            if (ow >= 0 && (cw < 0 || better(ov, oi, cv, ci))) {
              cv = ov;
              ci = oi;
              cw = ow;
            }
          }
          if (lane == 0) {
            red_v[wave] = cv;
            red_i[wave] = ci;
            red_w[wave] = cw;
          }
          __syncthreads();
          if (tid == 0) {
            double gv = -1.0;
            int gi = 0x7fffffff, gw = -1;
            for (int w = 0; w < kLT / 64; ++w)
              if (red_w[w] >= 0 && (gw < 0 || better(red_v[w], red_i[w], gv, gi))) {
                gv = red_v[w];
                gi = red_i[w];
                gw = red_w[w];
              }
            bcast_v = gv;
            bcast_i = gi;
            bcast_w = gw;
          }
          __syncthreads();
          if (bcast_w < 0 || !(bcast_v > 0.0)) stop = true;  // none left, or exact zero
        }
        if (!stop) {
          if (tid < kPW) {
            const Slot* s = a.slots + (t & 1) * G + bcast_w;
            u_sh[tid] = __hip_atomic_load(&s->row[tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
          if (tid == 0) {
            pivs[t] = bcast_i;
            if (blockIdx.x == 0) a.piv[t] = bcast_i;
          }
          __syncthreads();
          found = t + 1;
          const int p = bcast_i;
          // (e) rank-one update of the remaining panel columns; store the multipliers
          const double upiv = u_sh[tt];
          double u[kPW];
#pragma unroll
          for (int jj = tt + 1; jj < kPW; ++jj) u[jj] = u_sh[jj];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            if (((alive >> r) & 1u) && rowid[r] == p) alive &= ~(1u << r);
            if ((alive >> r) & 1u) {
              const double l = x[r][tt] / upiv;
              a.L[static_cast<int64_t>(t) * N + rowid[r]] = l;
#pragma unroll
              for (int jj = tt + 1; jj < kPW; ++jj) {
                const double prod = l * u[jj];
                x[r][jj] = x[r][jj] - prod;
              }
            }
          }
        }
      }
    });
    __syncthreads();
  }
  if (blockIdx.x == 0 && tid == 0) a.status[0] = found;
}

using LuppFn = void (*)(const Args);

template <typename InT>
LuppFn pick_t(int R) {
  switch (R) {
    case 1: return lupp_kernel<1, InT>;
    case 2: return lupp_kernel<2, InT>;
    case 4: return lupp_kernel<4, InT>;
    case 8: return lupp_kernel<8, InT>;
    default: return nullptr;
  }
}

}  // namespace

size_t lupp_workspace_bytes(int64_t steps, int64_t N) {
  const size_t L = static_cast<size_t>(steps) * N * sizeof(double);
  const size_t slots = 2 * 1024 * sizeof(Slot);
  return ((L + 255) & ~size_t(255)) + ((slots + 255) & ~size_t(255)) + 256 + 256;
}

int lupp_bind_workspace(void* base, int64_t steps, int64_t N, LuppWork* w) {
  char* p = static_cast<char*>(base);
  const size_t L = static_cast<size_t>(steps) * N * sizeof(double);
  w->L = reinterpret_cast<double*>(p);
  p += (L + 255) & ~size_t(255);
  w->slots = p;
  p += (2 * 1024 * sizeof(Slot) + 255) & ~size_t(255);
  w->barrier = reinterpret_cast<unsigned*>(p);
  p += 256;
  w->status = reinterpret_cast<int*>(p);
  w->steps_cap = steps;
  w->N_cap = N;
  return ICUR_OK;
}

int lupp_launch(const void* X, bool x64, int64_t K, int64_t N, int64_t ldx, int steps,
                const uint8_t* excluded, int64_t* piv, const LuppWork& w, hipStream_t st) {
  if (steps < 1 || steps > K) return arg_error("lupp: need 1 <= steps <= K");
  if (steps > kMaxSteps) return arg_error("lupp: steps above 1024 are not supported");
  if (N < 1 || ldx < N) return arg_error("lupp: need N >= 1 and ldx >= N");
  if (steps > w.steps_cap || N > w.N_cap) return arg_error("lupp: workspace too small");
  DeviceInfo dev;
  ICUR_TRY(device_info(&dev));
  // Rows per thread: the grid barrier's cost grows with the number of workgroups, so
  // pack up to 8 candidate rows per thread and aim for about 16 workgroups.
  int R = 1;
  while (R < 8 && static_cast<int64_t>(R) * kLT * 16 < N) R *= 2;
  while (R <= 8 && static_cast<int64_t>(R) * kLT * dev.num_cus < N) R *= 2;
  if (R > 8) {
    set_error("lupp: N exceeds the candidates one grid can hold in registers");
    return ICUR_ERR_UNSUPPORTED;
  }
  const int groups = static_cast<int>((N + static_cast<int64_t>(R) * kLT - 1) / (static_cast<int64_t>(R) * kLT));
  ICUR_TRY(launch_fill_u32(w.barrier, 1, 0u, st));
  ICUR_TRY(launch_fill_u32(reinterpret_cast<unsigned*>(w.status), 2, 0u, st));
  Args a;
  a.X = X;
  a.ldx = ldx;
  a.K = static_cast<int>(K);
  a.N = static_cast<int>(N);
  a.steps = steps;
  a.excl = excluded;
  a.L = w.L;
  a.slots = static_cast<Slot*>(w.slots);
  a.bar = w.barrier;
  a.status = w.status;
  a.piv = piv;
  void* params[] = {&a};
  const size_t shmem = static_cast<size_t>(steps) * kPW * sizeof(double) + static_cast<size_t>(steps) * sizeof(int);
  LuppFn fn = x64 ? pick_t<double>(R) : pick_t<float>(R);
  if (shmem > 64 * 1024) ICUR_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       static_cast<int>(shmem)));
  ICUR_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(fn), dim3(groups), dim3(kLT),
                                      params, static_cast<unsigned>(shmem), st));
  return ICUR_OK;
}

}  // namespace icur
