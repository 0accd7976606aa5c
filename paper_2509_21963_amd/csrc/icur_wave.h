// Wave- and workgroup-wide argmax on gfx950 (DPP moves and ballots), shared by the
// selection kernels and the small Gauss-Jordan inverse.
#pragma once

#include <climits>

#include <hip/hip_runtime.h>

namespace icur {

// Argmax keys: the bit pattern of |value|, which orders non-negative doubles like their
// values; key 0 stands for "no candidate with a nonzero value".
__device__ __forceinline__ unsigned long long cand_key(double v) {
  return v > 0.0 ? static_cast<unsigned long long>(__double_as_longlong(v)) : 0ull;
}

template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long x) {
  const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(x & 0xffffffffull), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(x >> 32), CTRL, 0xF, 0xF, false);
  return (static_cast<unsigned long long>(static_cast<unsigned>(hi)) << 32) | static_cast<unsigned>(lo);
}

__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long x, int lane) {
  const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(x & 0xffffffffull), lane));
  const unsigned hi = static_cast<unsigned>(__builtin_amdgcn_readlane(static_cast<int>(x >> 32), lane));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}

// Wave-wide argmax (every lane of the wave must be active): the largest key, the lowest
// index among the lanes holding it and that lane's tag w.  The maximum is taken with DPP
// moves inside each row of 16 lanes (quad permutations, then row rotations by 4 and 8)
// and across the four rows with lane reads; the winning lane comes from a ballot.
__device__ __forceinline__ void wave_argmax(unsigned long long k, int i, int w, unsigned long long* wk,
                                            int* wi, int* ww) {
  unsigned long long m = k, o;
  o = dpp_u64<0xB1>(m);   // quad_perm [1,0,3,2]
  m = o > m ? o : m;
  o = dpp_u64<0x4E>(m);   // quad_perm [2,3,0,1]
  m = o > m ? o : m;
  o = dpp_u64<0x124>(m);  // row_ror 4
  m = o > m ? o : m;
  o = dpp_u64<0x128>(m);  // row_ror 8
  m = o > m ? o : m;
  unsigned long long best = readlane_u64(m, 0);
#pragma unroll
  for (int row = 1; row < 4; ++row) {
    const unsigned long long r = readlane_u64(m, 16 * row);
    best = r > best ? r : best;
  }
  *wk = best;
  *wi = INT_MAX;
  *ww = -1;
  if (best == 0ull) return;
  unsigned long long lanes = __ballot(k == best);
  int lane = __builtin_ctzll(lanes);
  int bi = __builtin_amdgcn_readlane(i, lane);
  int bw = __builtin_amdgcn_readlane(w, lane);
  lanes &= lanes - 1;
  while (lanes) {  // equal keys in several lanes (rare): lowest index
    lane = __builtin_ctzll(lanes);
    const int i2 = __builtin_amdgcn_readlane(i, lane);
    if (i2 < bi) {
      bi = i2;
      bw = __builtin_amdgcn_readlane(w, lane);
    }
    lanes &= lanes - 1;
  }
  *wi = bi;
  *ww = bw;
}

struct Red {
  unsigned long long k;
  int i, w;
};

// Workgroup-wide argmax over (key, index, tag), ties to the lowest index; every thread gets
// the result.  red holds LT / 64 entries; one __syncthreads.
template <int LT>
__device__ __forceinline__ void block_argmax(unsigned long long k, int i, int w, Red* red,
                                             unsigned long long* gk, int* gi, int* gw) {
  unsigned long long wk;
  int wi, ww;
  wave_argmax(k, i, w, &wk, &wi, &ww);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = Red{wk, wi, ww};
  __syncthreads();
  Red b = red[0];
#pragma unroll
  for (int q = 1; q < LT / 64; ++q) {
    const Red c = red[q];
    if (c.k > b.k || (c.k == b.k && c.i < b.i)) b = c;
  }
  *gk = b.k;
  *gi = b.i;
  *gw = b.w;
}

}  // namespace icur
