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
// Schedule, per panel of 16 pivot columns [t0, t0 + 16):
//   prep kernel (all CUs)  every live candidate row gets the panel's 16 entries with all
//       t0 previous updates applied (left-looking, multipliers read from L), written to
//       the panel buffer P.  The pivot rows of the previous panel are first extended to
//       every later column (a 16-row triangular recurrence per column, kept in U), so
//       that the previous pivot rows restricted to this panel are available in LDS.
//   panel kernel (one persistent grid, <= one workgroup per CU)  the 16 pivot steps on
//       P held in registers, R rows per thread:
//         local argmax (DPP within waves, LDS across them)  ->  the owner publishes
//         (|value|, index, panel row) into its workgroup's slot for this step with
//         device-coherent stores  ->  every workgroup polls all slots of the step
//         (device-coherent loads) until each word it needs has arrived, and reduces them
//         itself  ->  rank-one update.  A slot word holds the bitwise complement of its
//         value and the slots are cleared to zero before the panel, so a nonzero word
//         is a complete, current value: the exchange needs no counter, no ordering of
//         the stores and no L2 write-back or invalidation, and a step costs the stores'
//         trip to the coherence point plus one polling round trip.
//       The multipliers replace the consumed panel entries in registers and are
//       written to L once, at the end of the panel.
// The panel grid is an ordinary dispatch (a cooperative launch costs about 10 us more
// per panel): at most one workgroup per CU, each within one CU's resources, so every
// workgroup is resident once dispatched, and work of other streams only delays that.
// Every wait is bounded; a wait that runs out sets a fault flag that ends the call
// with an error instead of a hang.
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <utility>

#include "icur_internal.h"
#include "icur_wave.h"

#pragma clang fp contract(off)

namespace icur {
namespace {

constexpr int kPW = 16;          // panel width
constexpr int kPT = 256;         // threads per workgroup of the prep kernel (= 16 x 16)
constexpr int kRowsPrep = kPT / 2;  // candidate rows per prep workgroup (two threads per row)
constexpr int kLC = 64;          // pivot-row multipliers staged in LDS per round (prep)
constexpr int kMaxSteps = 1024;  // LDS of the prep kernel holds (t0 + 64) x 16 doubles
constexpr int kMaxGroups = 256;  // panel-kernel workgroups (one per CU at most)
constexpr unsigned kSpinLimit = 1u << 22;
constexpr size_t kCtlBytes = 256;  // status words (byte 128), first pivot (byte 192)

// Exchange slot of one workgroup at one panel step: kSlotWords 64-bit words, each the
// bitwise complement of its value (zero = not yet written; no value published here has
// all bits set): the key of the workgroup's best |entry| (0 if it has no candidate with
// a nonzero entry), its index (INT_MAX if none), then the pivot-row candidate's panel
// entries (those before the step are not read).  Slots are laid out [step][workgroup].
constexpr int kSlotWords = 2 + kPW;
constexpr int kPoll = 8;  // slot words a thread loads together
constexpr size_t kSlotBytes = static_cast<size_t>(kPW) * kMaxGroups * kSlotWords * sizeof(unsigned long long);

// Device view of the workspace.
struct Work {
  double* L;        // steps x N: row t holds the multipliers of step t
  double* P;        // kPW x N: the current panel with all previous updates applied
  double* U;        // steps x steps: row k = pivot row of step k at the columns after its panel
  uint8_t* chosen;  // N: 1 once the candidate has been chosen as a pivot
  unsigned long long* xs;  // exchange slots, kPW x groups x kSlotWords words
  int groups;       // workgroups of the panel grid
  unsigned* ctl;    // control words
  int* status;      // [0] pivots found, [1] fault flag, [2] ended early
  unsigned long long* ref;  // |first pivot| of the call (bit pattern), set by panel 0
  int64_t* piv;     // steps
};

struct PrepArgs {
  const void* X;
  int64_t ldx;
  int N;
  int steps;
  int t0;
  int ncand;  // workgroups that prepare candidate rows; the rest extend pivot rows
  const uint8_t* excl;
  Work w;
};

struct PanelArgs {
  int N;
  int steps;
  int t0;
  double rel_cut;  // > 0: a pivot at or below rel_cut * |first pivot| ends the selection
  const uint8_t* excl;
  Work w;
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
__device__ __forceinline__ bool better_key(unsigned long long k, int i, unsigned long long bk, int bi) {
  return k > bk || (k == bk && i < bi);
}

// ---------------------------------------------------------------------------------
// prep kernel
// ---------------------------------------------------------------------------------
template <typename InT>
__global__ __launch_bounds__(kPT) void lupp_prep(const PrepArgs a) {
  // clear this panel's exchange slots (the previous panel kernel has finished with them;
  // the end of this kernel makes the zeros visible to every workgroup of the next one)
  if (a.w.groups > 1) {
    const int words = kPW * a.w.groups * kSlotWords;
    for (int e = static_cast<int>(blockIdx.x) * kPT + threadIdx.x; e < words; e += static_cast<int>(gridDim.x) * kPT)
      a.w.xs[e] = 0ull;
  }
  if (a.t0 == 0) {
    // first panel of a call: clear the control words (status, first pivot) for the
    // panel kernels that follow on the stream
    if (blockIdx.x == 0 && threadIdx.x < kCtlBytes / sizeof(unsigned)) a.w.ctl[threadIdx.x] = 0u;
  } else if (a.w.status[1] != 0 || a.w.status[2] != 0) {
    return;  // fault, or no pivots left
  }
  const InT* X = static_cast<const InT*>(a.X);
  // t0 x kPW: pivot rows 0..t0-1 at the 16 columns, then kLC x kPW staged multipliers
  extern __shared__ double Upan[];
  const int tid = threadIdx.x;
  const int N = a.N, t0 = a.t0, steps = a.steps;
  const bool cand = static_cast<int>(blockIdx.x) < a.ncand;
  const int col0 = cand ? t0 : t0 + kPW * (static_cast<int>(blockIdx.x) - a.ncand + 1);

  if (t0 > 0) {
    const int nb = t0 - kPW;  // the previous panel's pivots are steps nb .. t0-1
    double* Lst = Upan + static_cast<size_t>(t0) * kPW;
    // (1) older pivot rows at these columns, extended by earlier launches
    for (int e = tid; e < nb * kPW; e += kPT) {
      const int k = e / kPW, jj = e % kPW;
      const int col = col0 + jj;
      Upan[e] = col < steps ? a.w.U[static_cast<int64_t>(k) * steps + col] : 0.0;
    }
    // (2) the previous panel's pivot rows at these columns.  Thread (jj, q) owns column
    // col0 + jj of the pivot row of step nb + q; the 16 rows of one column sit in one
    // wave, so the recurrence among them runs on shuffles without block barriers.  The
    // multipliers of the 16 pivot rows at the older steps are staged in LDS, kLC steps
    // per round, all loads of a round in flight together.
    const int jj = tid >> 4, q = tid & 15;
    const int lane = tid & 63;
    const int col = col0 + jj;
    const int64_t p = a.w.piv[nb + q];
    double acc = col < steps ? static_cast<double>(X[static_cast<int64_t>(col) * a.ldx + p]) : 0.0;
    double lq[kPW - 1];
#pragma unroll
    for (int qq = 0; qq < kPW - 1; ++qq)
      lq[qq] = (qq < q && col < steps) ? a.w.L[static_cast<int64_t>(nb + qq) * N + p] : 0.0;
    for (int kb = 0; kb < nb; kb += kLC) {
#pragma unroll
      for (int u = 0; u < kLC / kPW; ++u) {
        const int k = kb + jj + kPW * u;  // thread (jj, q) stages its own pivot row
        Lst[(jj + kPW * u) * kPW + q] = k < nb ? a.w.L[static_cast<int64_t>(k) * N + p] : 0.0;
      }
      __syncthreads();  // also orders (1) before the first round
      const int kn = min(kLC, nb - kb);
      if (col < steps) {
        for (int kk = 0; kk < kn; ++kk) {
          const double prod = Lst[kk * kPW + q] * Upan[(kb + kk) * kPW + jj];
          acc = acc - prod;
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int qq = 0; qq < kPW - 1; ++qq) {
      const double u = __shfl(acc, (lane & 48) | qq, 64);  // row nb + qq, final by now
      if (q > qq) {
        const double prod = lq[qq] * u;
        acc = acc - prod;
      }
    }
    Upan[(nb + q) * kPW + jj] = acc;
    if (!cand && col < steps) a.w.U[static_cast<int64_t>(nb + q) * steps + col] = acc;
    __syncthreads();
  }
  if (!cand) return;

  // (3) candidate rows: the panel entries with all t0 previous updates, in step order.
  // Two neighbouring lanes per row, eight panel columns each.  Of each block of 16 steps'
  // multipliers each lane loads every other one and takes the rest from its partner (a
  // DPP exchange), so the multipliers are read from memory once; they are fetched three
  // blocks ahead of their use (t0 is a multiple of 16).
  constexpr int kHalf = kPW / 2;
  const int h = tid & 1;
  const int i = static_cast<int>(blockIdx.x) * kRowsPrep + (tid >> 1);
  // both lanes of a pair hold the same row, so they leave (or stay) together
  if (i >= N) return;
  if (t0 == 0 && h == 0) a.w.chosen[i] = 0;
  if ((a.excl && a.excl[i]) || (t0 > 0 && a.w.chosen[i])) return;
  const int pw = min(kPW, steps - t0);
  double x[kHalf];
#pragma unroll
  for (int j2 = 0; j2 < kHalf; ++j2) {
    const int jj = kHalf * h + j2;
    x[j2] = jj < pw ? static_cast<double>(X[static_cast<int64_t>(t0 + jj) * a.ldx + i]) : 0.0;
  }
  // this lane's half of the multipliers of steps k0 .. k0+15: steps k0 + 2q + h
  auto load_half = [&](int k0, double (&out)[kHalf]) {
#pragma unroll
    for (int q = 0; q < kHalf; ++q) out[q] = a.w.L[static_cast<int64_t>(k0 + 2 * q + h) * N + i];
  };
  // blocks kb .. kb + 3 of multipliers in flight (l0 is the block being applied)
  double l0[kHalf], l1[kHalf], l2[kHalf], l3[kHalf];
  if (t0 > 0) load_half(0, l0);
  if (t0 > kPW) load_half(kPW, l1);
  if (t0 > 2 * kPW) load_half(2 * kPW, l2);
  for (int kb = 0; kb < t0; kb += kPW) {
    if (kb + 3 * kPW < t0) load_half(kb + 3 * kPW, l3);
    double l[kPW];
#pragma unroll
    for (int q = 0; q < kHalf; ++q) {
      const double other = __longlong_as_double(static_cast<long long>(
          dpp_u64<0xB1>(static_cast<unsigned long long>(__double_as_longlong(l0[q])))));  // quad_perm [1,0,3,2]
      l[2 * q] = h ? other : l0[q];
      l[2 * q + 1] = h ? l0[q] : other;
    }
    const double* up = Upan + kb * kPW + kHalf * h;
#pragma unroll
    for (int u = 0; u < kPW; ++u) {
#pragma unroll
      for (int j2 = 0; j2 < kHalf; ++j2) {
        const double prod = l[u] * up[u * kPW + j2];
        x[j2] = x[j2] - prod;
      }
    }
#pragma unroll
    for (int q = 0; q < kHalf; ++q) {
      l0[q] = l1[q];
      l1[q] = l2[q];
      l2[q] = l3[q];
    }
  }
#pragma unroll
  for (int j2 = 0; j2 < kHalf; ++j2) a.w.P[static_cast<int64_t>(kHalf * h + j2) * N + i] = x[j2];
}

// ---------------------------------------------------------------------------------
// panel kernel
// ---------------------------------------------------------------------------------

template <int R, int LT>
__global__ __launch_bounds__(LT, 1) void lupp_panel(const PanelArgs a) {
  __shared__ Red red[LT / 64];  // workgroup argmax scratch
  __shared__ double rows_sh[kMaxGroups * kPW];  // published panel rows of all workgroups
  __shared__ unsigned long long key_sh[kMaxGroups];
  __shared__ unsigned long long pub_sh[kSlotWords];  // the slot being published
  __shared__ int idx_sh[kMaxGroups];
  __shared__ long long piv_sh[kPW];

  // A previous panel ended the factorization (or faulted): every workgroup reads the
  // same values, so the whole grid leaves together.
  if (a.w.status[1] != 0 || a.w.status[2] != 0) return;
  const int tid = threadIdx.x;
  const int G = gridDim.x;
  const int N = a.N, t0 = a.t0;
  const int pw = min(kPW, a.steps - t0);

  int rowid[R];
  unsigned alive = 0;  // bit r: row r is a valid, eligible, not yet chosen candidate
#pragma unroll
  for (int r = 0; r < R; ++r) {
    rowid[r] = (static_cast<int>(blockIdx.x) * R + r) * LT + tid;
    if (rowid[r] < N && !(a.excl && a.excl[rowid[r]]) && !a.w.chosen[rowid[r]]) alive |= 1u << r;
  }
  const unsigned alive0 = alive;
  unsigned cstep = 0;  // 4 bits per row: the panel step at which row r became a pivot
  double x[R][kPW];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const bool live = (alive >> r) & 1u;
#pragma unroll
    for (int jj = 0; jj < kPW; ++jj)
      x[r][jj] = (live && jj < pw) ? a.w.P[static_cast<int64_t>(jj) * N + rowid[r]] : 0.0;
  }
  int found = t0;
  bool stop = false;
  // reference for the relative cut: |first pivot of the call| (known from panel 0 on)
  unsigned long long ref_key = t0 > 0 ? *a.w.ref : 0ull;

  static_for<kPW>([&](auto ttc) {
    constexpr int tt = decltype(ttc)::value;
    if (!stop && tt < pw) {
      const int t = t0 + tt;
      // (a) local argmax, then the workgroup's best
      double bv = -1.0;
      int bi = INT_MAX;
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
      unsigned long long gk;
      int gi, gw;
      block_argmax<LT>(cand_key(bv), bi, 0, red, &gk, &gi, &gw);
      const bool owner = gk != 0ull && br >= 0 && bi == gi;
      // the owner's row from column tt on, selected with bit masks (a read x[br] with a
      // run-time index would force x into scratch memory)
      auto owner_row = [&](unsigned long long (&pub)[kPW]) {
#pragma unroll
        for (int jj = tt; jj < kPW; ++jj) pub[jj] = 0ull;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const unsigned long long mask = (r == br) ? ~0ull : 0ull;
#pragma unroll
          for (int jj = tt; jj < kPW; ++jj)
            pub[jj] |= static_cast<unsigned long long>(__double_as_longlong(x[r][jj])) & mask;
        }
      };
      // the pivot (key gk, row gi): none left, an exact zero column, or (with the relative
      // cut) a Schur complement that is rounding noise of the input's precision ends it
      auto accept = [&]() {
        if (gk == 0ull) stop = true;
        if (t == 0) ref_key = gk;
        if (a.rel_cut > 0.0 && t > 0 &&
            gk <= static_cast<unsigned long long>(__double_as_longlong(a.rel_cut * __longlong_as_double(
                      static_cast<long long>(ref_key)))))
          stop = true;
      };
      if (G == 1) {
        // one workgroup holds every candidate: the pivot row goes through LDS, no grid
        // exchange (rows_sh was last read before the barrier inside block_argmax above)
        if (owner) {
          unsigned long long pub[kPW];
          owner_row(pub);
#pragma unroll
          for (int jj = tt; jj < kPW; ++jj) rows_sh[jj] = __longlong_as_double(static_cast<long long>(pub[jj]));
        }
        __syncthreads();
        gw = 0;
        accept();
      } else {
        // (b) the owner (or thread 0 when the workgroup has no candidate) publishes the
        // workgroup's slot of this step, header and the row from column tt on: it stages
        // the words in LDS and its wave stores them with one vector store, so they travel
        // together instead of as 2 + 16 - tt stores of one thread
        unsigned long long* xs = a.w.xs + static_cast<size_t>(tt) * G * kSlotWords;
        const bool writer = owner || (gk == 0ull && tid == 0);
        if (__ballot(writer) != 0ull) {  // the writer's wave (uniform within it)
          if (writer) {
            unsigned long long pub[kPW];
            if (owner) {
              owner_row(pub);
            } else {
#pragma unroll
              for (int jj = tt; jj < kPW; ++jj) pub[jj] = 0ull;
            }
            pub_sh[0] = ~gk;
            pub_sh[1] = ~static_cast<unsigned long long>(owner ? gi : INT_MAX);
#pragma unroll
            for (int jj = tt; jj < kPW; ++jj) pub_sh[2 + jj] = ~pub[jj];
          }
          // the words were written by one lane of this wave and are read by the others
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          const int ln = tid & 63;
          if (ln < kSlotWords && (ln < 2 || ln - 2 >= tt))
            __hip_atomic_store(xs + static_cast<size_t>(blockIdx.x) * kSlotWords + ln, pub_sh[ln], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        // (c) every word of every slot this step reads.  A thread's words are loaded
        // kPoll at a time, all in flight together, and the ones that had not arrived are
        // loaded again, again all together (bounded; a fault anywhere ends every
        // workgroup's wait): one round trip when the slots are complete, one more per
        // round of late words.
        bool ok = true;
        const int per = kSlotWords - tt;  // header and row entries tt .. kPW-1
        const int total = G * per;
        for (int base = 0; base < total && ok; base += LT * kPoll) {
          const unsigned long long* src[kPoll];
          unsigned long long v[kPoll];
#pragma unroll
          for (int q = 0; q < kPoll; ++q) {
            const int e = base + q * LT + tid;
            src[q] = nullptr;
            v[q] = 1ull;  // no word here: nothing to wait for
            if (e < total) {
              const int g = e / per, w = e % per;
              src[q] = xs + static_cast<size_t>(g) * kSlotWords + (w < 2 ? w : w + tt);
              v[q] = __hip_atomic_load(src[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
          }
          unsigned spins = 0;
          for (;;) {
            bool missing = false;
#pragma unroll
            for (int q = 0; q < kPoll; ++q) missing |= (v[q] == 0ull);
            if (!missing) break;
            __builtin_amdgcn_s_sleep(1);
            if ((++spins & 255u) == 0 &&
                __hip_atomic_load(a.w.status + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
              ok = false;
              break;
            }
            if (spins > kSpinLimit) {
              atomicExch(a.w.status + 1, 1);
              ok = false;
              break;
            }
#pragma unroll
            for (int q = 0; q < kPoll; ++q)
              if (v[q] == 0ull) v[q] = __hip_atomic_load(src[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
#pragma unroll
          for (int q = 0; q < kPoll; ++q) {
            const int e = base + q * LT + tid;
            if (e >= total) continue;
            const int g = e / per, w = e % per;
            const unsigned long long x = ~v[q];
            if (w == 0)
              key_sh[g] = x;
            else if (w == 1)
              idx_sh[g] = static_cast<int>(x);
            else
              rows_sh[g * kPW + w + tt - 2] = __longlong_as_double(static_cast<long long>(x));
          }
        }
        if (__syncthreads_or(ok ? 0 : 1)) {
          stop = true;
        } else {
          // (d) reduce the slots: every wave on its own (the same keys give every wave the
          // same winner), so no further barrier
          unsigned long long ck = 0ull;
          int ci = INT_MAX, cw = -1;
          for (int g = tid & 63; g < G; g += 64) {
            if (better_key(key_sh[g], idx_sh[g], ck, ci)) {
              ck = key_sh[g];
              ci = idx_sh[g];
              cw = g;
            }
          }
          wave_argmax(ck, ci, cw, &gk, &gi, &gw);
          accept();
        }
      }
      if (!stop) {
        if (tid == 0) piv_sh[tt] = gi;
        found = t + 1;
        const int p = gi;
        // (e) rank-one update of the remaining panel columns; the multiplier replaces
        // the consumed entry x[r][tt]
        const double* u = rows_sh + gw * kPW;
        const double upiv = u[tt];
        double uu[kPW];
#pragma unroll
        for (int jj = tt + 1; jj < kPW; ++jj) uu[jj] = u[jj];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (((alive >> r) & 1u) && rowid[r] == p) {
            alive &= ~(1u << r);
            cstep |= static_cast<unsigned>(tt) << (4 * r);
          }
          // Unconditional (no register selects): on a row that is not live the update
          // only touches entries that are never read again (its multipliers before the
          // step it was chosen at stay as they are; rows that never were live hold 0).
          const double l = x[r][tt] / upiv;
          x[r][tt] = l;
#pragma unroll
          for (int jj = tt + 1; jj < kPW; ++jj) {
            const double prod = l * uu[jj];
            x[r][jj] = x[r][jj] - prod;
          }
        }
      }
      // rows_sh, key_sh, idx_sh and pub_sh are rewritten by the next step only after the
      // barrier inside its first block_argmax, which every thread reaches after finishing
      // this update and its slot reduction; red only after the barrier of (c)
    }
  });

  // multipliers of this panel: every step for live rows, the steps before their own
  // for the rows chosen as pivots here
  const int done = found - t0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if ((alive0 >> r) & 1u) {
      const bool piv_row = !((alive >> r) & 1u);
      const int nl = piv_row ? static_cast<int>((cstep >> (4 * r)) & 15u) : done;
#pragma unroll
      for (int jj = 0; jj < kPW; ++jj)
        if (jj < nl) a.w.L[static_cast<int64_t>(t0 + jj) * N + rowid[r]] = x[r][jj];
      if (piv_row) a.w.chosen[rowid[r]] = 1;
    }
  }
  if (blockIdx.x == 0) {
    __syncthreads();
    if (tid < done) a.w.piv[t0 + tid] = piv_sh[tid];
    if (tid == 0) {
      a.w.status[0] = found;
      if (stop) a.w.status[2] = 1;
      if (t0 == 0) *a.w.ref = ref_key;
    }
  }
}

using PanelFn = void (*)(const PanelArgs);

// Candidate rows per workgroup = R * LT: 256, 512, 1024, then 2048 (four rows per thread
// on 512 threads, two waves per SIMD, which keeps each wave within 256 registers).
struct PanelShape {
  int R, LT;
  PanelFn fn;
};
constexpr int kShapes = 4;
const PanelShape kShape[kShapes] = {{1, 256, lupp_panel<1, 256>},
                                    {2, 256, lupp_panel<2, 256>},
                                    {4, 256, lupp_panel<4, 256>},
                                    {4, 512, lupp_panel<4, 512>}};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

size_t lupp_workspace_bytes(int64_t steps, int64_t N) {
  return align256(static_cast<size_t>(steps) * N * sizeof(double)) +      // L
         align256(static_cast<size_t>(kPW) * N * sizeof(double)) +        // P
         align256(static_cast<size_t>(steps) * steps * sizeof(double)) +  // U
         align256(static_cast<size_t>(N)) +                               // chosen
         align256(kSlotBytes) +                                           // exchange slots
         kCtlBytes;                                                       // status
}

int lupp_bind_workspace(void* base, int64_t steps, int64_t N, LuppWork* w) {
  char* p = static_cast<char*>(base);
  w->L = reinterpret_cast<double*>(p);
  p += align256(static_cast<size_t>(steps) * N * sizeof(double));
  w->P = reinterpret_cast<double*>(p);
  p += align256(static_cast<size_t>(kPW) * N * sizeof(double));
  w->U = reinterpret_cast<double*>(p);
  p += align256(static_cast<size_t>(steps) * steps * sizeof(double));
  w->chosen = reinterpret_cast<uint8_t*>(p);
  p += align256(static_cast<size_t>(N));
  w->slots = p;
  p += align256(kSlotBytes);
  // control words, cleared by every call: the status words and the first pivot
  w->ctl = reinterpret_cast<unsigned*>(p);
  w->status = reinterpret_cast<int*>(p + 128);
  w->ref = reinterpret_cast<unsigned long long*>(p + 192);
  w->steps_cap = steps;
  w->N_cap = N;
  w->max_groups = 0;
  return ICUR_OK;
}

int64_t lupp_max_candidates(int max_groups) {
  const PanelShape& big = kShape[kShapes - 1];
  return static_cast<int64_t>(std::min(max_groups, kMaxGroups)) * big.R * big.LT;
}

int lupp_launch(const void* X, bool x64, int64_t K, int64_t N, int64_t ldx, int steps,
                const uint8_t* excluded, int64_t* piv, const LuppWork& w, hipStream_t st, double rel_cut) {
  if (!(rel_cut >= 0.0 && rel_cut < 1.0)) return arg_error("lupp: need 0 <= rel_cut < 1");
  if (steps < 1 || steps > K) return arg_error("lupp: need 1 <= steps <= K");
  if (steps > kMaxSteps) return arg_error("lupp: steps above 1024 are not supported");
  if (N < 1 || ldx < N) return arg_error("lupp: need N >= 1 and ldx >= N");
  if (N > INT_MAX) return arg_error("lupp: N must be below 2^31");
  if (steps > w.steps_cap || N > w.N_cap) return arg_error("lupp: workspace too small");
  DeviceInfo dev;
  ICUR_TRY(device_info(&dev));
  // Rows per workgroup: up to 2048 candidates fit one workgroup, which needs no grid
  // exchange.  Beyond that a step's exchange grows slowly with the workgroup count (about
  // 1.1 us at 8 workgroups, 1.7 us at 30) while its argmax and update shrink with fewer
  // rows per thread: the smallest shape that needs at most 64 workgroups (measured best
  // of 16, 32, 64, 128 on 30000 and 40000 candidates).
  const int max_groups = std::min(std::min(dev.num_cus, kMaxGroups), w.max_groups > 0 ? w.max_groups : kMaxGroups);
  int sh = 0;
  if (N <= static_cast<int64_t>(kShape[kShapes - 1].R) * kShape[kShapes - 1].LT) {
    // one workgroup holds them all: no grid exchange at all (the pivot row goes through LDS)
    while (static_cast<int64_t>(kShape[sh].R) * kShape[sh].LT < N) ++sh;
  } else {
    // ICUR_LUPP_GROUPS: the workgroup count aimed for (default 64)
    int target = 64;
    if (const char* e = std::getenv("ICUR_LUPP_GROUPS")) target = std::max(1, std::atoi(e));
    while (sh + 1 < kShapes && static_cast<int64_t>(kShape[sh].R) * kShape[sh].LT * target < N) ++sh;
    // under a workgroup cap (concurrent selections), larger shapes until the grid fits
    while (sh + 1 < kShapes && static_cast<int64_t>(kShape[sh].R) * kShape[sh].LT * max_groups < N) ++sh;
  }
  const int64_t per_group = static_cast<int64_t>(kShape[sh].R) * kShape[sh].LT;
  if (per_group * max_groups < N) {
    set_error("lupp: N exceeds the candidates one grid can hold in registers");
    return ICUR_ERR_UNSUPPORTED;
  }
  const int groups = static_cast<int>((N + per_group - 1) / per_group);
  // the control words are cleared by the first prep launch, the exchange slots by every
  // prep launch

  Work wk;
  wk.L = w.L;
  wk.P = w.P;
  wk.U = w.U;
  wk.chosen = w.chosen;
  wk.xs = static_cast<unsigned long long*>(w.slots);
  wk.groups = groups;
  wk.ctl = w.ctl;
  wk.ref = w.ref;
  wk.status = w.status;
  wk.piv = piv;

  PrepArgs pa;
  pa.X = X;
  pa.ldx = ldx;
  pa.N = static_cast<int>(N);
  pa.steps = steps;
  pa.ncand = static_cast<int>((N + kRowsPrep - 1) / kRowsPrep);
  pa.excl = excluded;
  pa.w = wk;
  PanelArgs qa;
  qa.N = static_cast<int>(N);
  qa.steps = steps;
  qa.rel_cut = rel_cut;
  qa.excl = excluded;
  qa.w = wk;

  const void* prep = x64 ? reinterpret_cast<const void*>(lupp_prep<double>)
                         : reinterpret_cast<const void*>(lupp_prep<float>);
  const size_t max_lds = static_cast<size_t>(steps + kLC) * kPW * sizeof(double);
  if (max_lds > 64 * 1024)
    ICUR_HIP(hipFuncSetAttribute(prep, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(max_lds)));
  const void* panel = reinterpret_cast<const void*>(kShape[sh].fn);
  for (int t0 = 0; t0 < steps; t0 += kPW) {
    pa.t0 = t0;
    qa.t0 = t0;
    const int extra = t0 > 0 ? std::max(0, (steps - t0 + kPW - 1) / kPW - 1) : 0;
    const size_t lds = t0 > 0 ? static_cast<size_t>(t0 + kLC) * kPW * sizeof(double) : 0;
    void* pparams[] = {&pa};
    ICUR_HIP(hipLaunchKernel(prep, dim3(pa.ncand + extra), dim3(kPT), pparams, lds, st));
    void* qparams[] = {&qa};
    ICUR_HIP(hipLaunchKernel(panel, dim3(groups), dim3(kShape[sh].LT), qparams, 0, st));
  }
  return ICUR_OK;
}

}  // namespace icur
