// icur_lupp_noalloc: the LUPP selection of icur_lupp for callers that cannot allocate
// device memory (code under stream capture, tight serving loops).  Its workspace (the
// multipliers, the current panel, the extended pivot rows, the chosen flags, the
// exchange slots and the control words) lives in one file-scope device array, so a call
// makes no allocation of any kind.
//
// The array exists once per device.  Its device address is looked up once per device,
// with that device current, and kept; kernels only ever receive that address.  Calls
// on one device share the array: two calls that overlap on one device race.  Every
// word a call reads was written earlier in the same call (the first prep launch clears
// the control words and the chosen flags), so nothing has to be cleared between calls.
#include <map>
#include <mutex>

#include "icur_internal.h"

namespace icur {
namespace {

// Large enough for b = 100 pivots over the 40000 columns of a 40000 x 40000 sketch
// (about 37.3 MB); the limit is stated in icur.h.
constexpr size_t kScratchBytes = size_t(48) << 20;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> address of that device's copy

// The device address of the current device's copy of `scratch` (looked up once).
int scratch_address(void** out) {
  int dev = 0;
  ICUR_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      return ICUR_ERR_HIP;
    }
    // warm the cached device properties the launcher reads, so a later call does no
    // first-time set-up
    DeviceInfo di;
    ICUR_TRY(device_info(&di));
    it = g_scratch_ptr.emplace(dev, p).first;
  }
  *out = it->second;
  return ICUR_OK;
}

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

}  // namespace icur

using namespace icur;

extern "C" {

int icur_init_noalloc(void) {
  set_error("");
  void* p = nullptr;
  return scratch_address(&p);
}

int icur_lupp_noalloc(const float* X, int64_t K, int64_t N, int64_t ldx, int32_t steps,
                      const uint8_t* excluded, int64_t* piv, int32_t* npiv, void* stream) {
  set_error("");
  if (!X || !piv || !npiv) return arg_error("null pointer");
  if (K < 1 || N < 1 || ldx < N) return arg_error("invalid shape");
  if (steps < 1 || steps > K) return arg_error("need 1 <= steps <= K");
  if (K > 4096) return arg_error("K above 4096 is not supported");
  if (steps > 256) return arg_error("icur_lupp_noalloc: steps above 256 are not supported");
  if (N > 0x7fffffffLL) return arg_error("N must be below 2^31");
  const size_t need = lupp_workspace_bytes(steps, N);
  if (need > kScratchBytes)
    return arg_error("icur_lupp_noalloc: the workspace for " + std::to_string(steps) + " steps over " +
                     std::to_string(N) + " candidates needs " + std::to_string(need) +
                     " bytes, above the fixed " + std::to_string(kScratchBytes) + "-byte scratch area");
  void* base = nullptr;
  ICUR_TRY(scratch_address(&base));
  hipStream_t st = as_stream(stream);
  LuppWork lw;
  lupp_bind_workspace(base, steps, N, &lw);
  ICUR_TRY(lupp_launch(X, false, K, N, ldx, steps, excluded, piv, lw, st));
  // the pivot count and the fault flag: a copy into this frame, then the stream's end
  int words[2] = {0, 0};
  ICUR_HIP(hipMemcpyAsync(words, lw.status, sizeof(words), hipMemcpyDeviceToHost, st));
  ICUR_HIP(hipStreamSynchronize(st));
  if (words[1]) {
    set_error("selection kernel: grid barrier did not complete");
    return ICUR_ERR_HIP;
  }
  *npiv = words[0];
  return ICUR_OK;
}

}  // extern "C"
