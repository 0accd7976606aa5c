// The C-ABI of libicur: argument checking, the per-device workspace cache and the host
// driver of Alg. 1 (IterativeCUR).  Every step of the loop runs in the kernels of the
// other translation units; the host only orders launches, reads back three scalars per
// iteration (two pivot counts and the residual norm) and decides when to stop.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "icur_batched.h"
#include "icur_internal.h"
#include "icur_wide_kernel.h"

namespace icur {

// ----------------------------------------------------------------- errors and info
namespace {
thread_local std::string t_error;
thread_local icur_info t_info;
}  // namespace

void set_error(const std::string& msg) { t_error = msg; }
const char* last_error() { return t_error.c_str(); }

int device_info(DeviceInfo* out) {
  static std::mutex mu;
  static std::map<int, int> cus;
  int dev = 0;
  ICUR_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(mu);
  auto it = cus.find(dev);
  if (it == cus.end()) {
    int n = 0;
    ICUR_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
    it = cus.emplace(dev, n).first;
  }
  out->device = dev;
  out->num_cus = it->second;
  return ICUR_OK;
}

// ----------------------------------------------------------------- workspace cache
namespace {

enum Slot {
  kG, kRowsPat, kSignsPat, kX0, kS, kSrow, kCt, kR, kU, kY, kA12, kA21, kA22, kYt, kX0J, kW64,
  kWp, kColMask, kRowMask, kJk, kIk, kJall, kIall, kLupp, kGemmWs, kNormPart, kScal, kCoreWs,
  kStepA, kStepB, kCsc, kQrcp, kUrk64, kCoreRef, kNumSlots
};

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

// One workspace per (device, slot).  Slot 0 serves the single-matrix calls; the batched
// call gives each of its concurrent workers a slot of its own, with its own stream.
struct DeviceCache {
  std::mutex mu;
  int device = 0;
  Buf buf[kNumSlots];
  // pinned staging area: scalars (byte 0), status words (byte 256) and, from
  // kStageOffset on, the results of a call (infos, I, J and U when they fit)
  void* host_pinned = nullptr;
  void* host_pinned_dev = nullptr;  // its device address (read-backs are kernel stores)
  unsigned flag_seq = 0;            // last value published in the read-back flag
  std::vector<hipEvent_t> events;
  hipEvent_t sync_event = nullptr;  // marks the end of the work a read-back waits for
  bool spin = true;                 // wait for read-backs by polling (single calls)
  hipStream_t stream = nullptr;     // worker stream of a batched slot (default priority)
  ~DeviceCache() {}
};

constexpr size_t kFlagOffset = 1024;  // read-back completion flag in the pinned area
constexpr size_t kStageOffset = 4096;
constexpr size_t kStageBytes = size_t(2) << 20;
constexpr size_t kPinnedBytes = kStageOffset + kStageBytes;

std::mutex g_cache_mu;
std::map<std::pair<int, int>, std::unique_ptr<DeviceCache>> g_cache;

DeviceCache& cache_for(int dev, int slot) {
  std::lock_guard<std::mutex> g(g_cache_mu);
  auto& p = g_cache[{dev, slot}];
  if (!p) {
    p.reset(new DeviceCache());
    p->device = dev;
    p->spin = slot == 0;
  }
  return *p;
}

int ensure(DeviceCache& dc, int slot, size_t bytes, void** out) {
  Buf& b = dc.buf[slot];
  if (bytes == 0) bytes = 256;
  if (b.bytes < bytes) {
    if (b.p) ICUR_HIP(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
    const size_t want = (bytes + 4095) & ~size_t(4095);
    if (hipMalloc(&b.p, want) != hipSuccess) {
      (void)hipGetLastError();
      b.p = nullptr;
      set_error("device allocation of " + std::to_string(want) + " bytes failed");
      return ICUR_ERR_NOMEM;
    }
    b.bytes = want;
  }
  *out = b.p;
  return ICUR_OK;
}

// Grow a slot, keeping a 2D region: rows x row_bytes from (old, old_ld_bytes) to
// (new, new_ld_bytes).
int grow_keep(DeviceCache& dc, int slot, size_t bytes, int64_t rows, size_t row_bytes,
              size_t old_ld_bytes, size_t new_ld_bytes, hipStream_t st, void** out) {
  Buf& b = dc.buf[slot];
  const bool keep = rows > 0 && row_bytes > 0;
  if (b.bytes >= bytes && (!keep || old_ld_bytes == new_ld_bytes)) {
    *out = b.p;
    return ICUR_OK;
  }
  void* np = nullptr;
  const size_t want = (bytes + 4095) & ~size_t(4095);
  if (hipMalloc(&np, want) != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation of " + std::to_string(want) + " bytes failed");
    return ICUR_ERR_NOMEM;
  }
  if (b.p && keep)
    ICUR_HIP(hipMemcpy2DAsync(np, new_ld_bytes, b.p, old_ld_bytes, row_bytes, rows,
                              hipMemcpyDeviceToDevice, st));
  ICUR_HIP(hipStreamSynchronize(st));
  if (b.p) ICUR_HIP(hipFree(b.p));
  b.p = np;
  b.bytes = want;
  *out = np;
  return ICUR_OK;
}

// Device scalars read back once per iteration.
struct Scal {
  double normsq_x0;
  double normsq_s;
  double norms[2];
  int info;
  int pad;
  double normsq_a;  // ||A||_F^2 (the ||A||_F denominator only)
};

// Device-event timing of the phases (icur_info).  When off (the batched workers), every
// call is a no-op and every duration reads 0.  Durations are read once, after the call's
// last wait (add, then flush), so no timing call sits between a read-back and the next
// launch.
struct Timer {
  DeviceCache* dc;
  hipStream_t st;
  bool on = true;
  size_t used = 0;
  struct Span {
    size_t a, b;
    double* acc;
  };
  std::vector<Span> spans;
  void add(size_t a, size_t b, double* acc) {
    if (on) spans.push_back(Span{a, b, acc});
  }
  void flush() {
    for (const Span& sp : spans) *sp.acc += ms(sp.a, sp.b);
    spans.clear();
  }
  // An event slot that the caller records itself (or that mark() records now).
  int reserve(size_t* idx) {
    if (!on) {
      *idx = 0;
      return ICUR_OK;
    }
    if (used == dc->events.size()) {
      hipEvent_t e;
      ICUR_HIP(hipEventCreate(&e));
      dc->events.push_back(e);
    }
    *idx = used++;
    return ICUR_OK;
  }
  int mark(size_t* idx) {
    ICUR_TRY(reserve(idx));
    return record(*idx);
  }
  int record(size_t idx) {
    if (on) ICUR_HIP(hipEventRecord(dc->events[idx], st));
    return ICUR_OK;
  }
  hipEvent_t event(size_t idx) const { return on ? dc->events[idx] : nullptr; }
  float ms(size_t a, size_t b) {
    if (!on) return 0.f;
    float v = 0.f;
    if (hipEventElapsedTime(&v, dc->events[a], dc->events[b]) != hipSuccess) {
      (void)hipGetLastError();
      v = 0.f;
    }
    return v;
  }
};

// Waits for the work queued on st.  A single call polls an event: the blocking wait of
// the runtime wakes up tens of microseconds after the work ends, and a call makes a few
// read-backs per iteration.  The batched workers, which share the host cores, block.
int sync_stream(DeviceCache& dc, hipStream_t st) {
  if (!dc.spin) {
    ICUR_HIP(hipStreamSynchronize(st));
    return ICUR_OK;
  }
  if (!dc.sync_event) ICUR_HIP(hipEventCreateWithFlags(&dc.sync_event, hipEventDisableTiming));
  ICUR_HIP(hipEventRecord(dc.sync_event, st));
  for (;;) {
    const hipError_t e = hipEventQuery(dc.sync_event);
    if (e == hipSuccess) break;
    if (e != hipErrorNotReady) ICUR_HIP(e);
    __builtin_ia32_pause();
  }
  return ICUR_OK;
}

// Polls the read-back flag until the kernel has published seq; every 1024 polls the
// stream is queried, so a failed or drained stream ends the wait.
int wait_flag(DeviceCache& dc, unsigned seq, hipStream_t st) {
  volatile unsigned* f = reinterpret_cast<volatile unsigned*>(static_cast<char*>(dc.host_pinned) + kFlagOffset);
  for (uint64_t polls = 1;; ++polls) {
    if (*f == seq) break;
    if ((polls & 1023u) == 0) {
      const hipError_t e = hipStreamQuery(st);
      if (e == hipSuccess) {
        if (*f == seq) break;
        set_error("read-back: the completion flag was not seen after the stream drained");
        return ICUR_ERR_HIP;
      }
      if (e != hipErrorNotReady) ICUR_HIP(e);
    }
    __builtin_ia32_pause();
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return ICUR_OK;
}

// Device segments into the pinned staging area, then one wait.  Small read-backs of a
// single call are kernel stores into the host-mapped buffer followed by a flag the host
// polls; the results at the end of a call use a multi-workgroup copy and a stream wait;
// without a device address for the buffer, copies.
int read_back(DeviceCache& dc, const HostSegs& segs, hipStream_t st, bool small = true) {
  if (dc.host_pinned_dev && dc.spin && small) {
    const unsigned seq = ++dc.flag_seq;
    ICUR_TRY(launch_to_host_flag(segs, dc.host_pinned_dev,
                                 reinterpret_cast<unsigned*>(static_cast<char*>(dc.host_pinned_dev) + kFlagOffset), seq,
                                 st));
    return wait_flag(dc, seq, st);
  }
  if (dc.host_pinned_dev) {
    ICUR_TRY(launch_to_host(segs, dc.host_pinned_dev, st));
  } else {
    for (int i = 0; i < segs.n; ++i)
      ICUR_HIP(hipMemcpyAsync(static_cast<char*>(dc.host_pinned) + segs.seg[i].dst_off, segs.seg[i].src,
                              static_cast<size_t>(segs.seg[i].bytes), hipMemcpyDeviceToHost, st));
  }
  return sync_stream(dc, st);
}

int read_scal(DeviceCache& dc, const Scal* dev, Scal* host, hipStream_t st) {
  Scal* pin = static_cast<Scal*>(dc.host_pinned);
  HostSegs h{};
  h.seg[0] = HostSeg{dev, static_cast<int64_t>(sizeof(Scal)), 0};
  h.n = 1;
  ICUR_TRY(read_back(dc, h, st));
  *host = *pin;
  return ICUR_OK;
}

int read_int(DeviceCache& dc, const int* dev, int* host, int count, hipStream_t st) {
  int* pin = reinterpret_cast<int*>(static_cast<char*>(dc.host_pinned) + 256);
  HostSegs h{};
  h.seg[0] = HostSeg{dev, static_cast<int64_t>(sizeof(int)) * count, 256};
  h.n = 1;
  ICUR_TRY(read_back(dc, h, st));
  std::memcpy(host, pin, sizeof(int) * count);
  return ICUR_OK;
}

// Status words and the scalars in one synchronisation.
int read_int_scal(DeviceCache& dc, const int* dev, int* host, int count, const Scal* dscal, Scal* hscal,
                  hipStream_t st) {
  Scal* spin = static_cast<Scal*>(dc.host_pinned);
  int* pin = reinterpret_cast<int*>(static_cast<char*>(dc.host_pinned) + 256);
  HostSegs h{};
  h.seg[0] = HostSeg{dev, static_cast<int64_t>(sizeof(int)) * count, 256};
  h.seg[1] = HostSeg{dscal, static_cast<int64_t>(sizeof(Scal)), 0};
  h.n = 2;
  ICUR_TRY(read_back(dc, h, st));
  std::memcpy(host, pin, sizeof(int) * count);
  *hscal = *spin;
  return ICUR_OK;
}

int prepare_device(DeviceCache** out, int slot = 0) {
  DeviceInfo dev;
  ICUR_TRY(device_info(&dev));
  DeviceCache& dc = cache_for(dev.device, slot);
  if (!dc.host_pinned) {
    ICUR_HIP(hipHostMalloc(&dc.host_pinned, kPinnedBytes, hipHostMallocDefault));
    std::memset(dc.host_pinned, 0, kStageOffset);
    dc.flag_seq = 0;
    void* d = nullptr;
    if (hipHostGetDevicePointer(&d, dc.host_pinned, 0) == hipSuccess) {
      dc.host_pinned_dev = d;
    } else {
      (void)hipGetLastError();  // not mapped: read-backs use copies
      dc.host_pinned_dev = nullptr;
    }
  }
  *out = &dc;
  return ICUR_OK;
}

// Row selection ends at a pivot below this fraction of its first pivot: the Schur
// complement is then rounding noise of the factors' precision (a block straddling the
// exact rank of A), and inverting that noise in N_k would wreck the residual recurrence.
// What is dropped is at most this fraction of the block's largest residual entry.
constexpr double kRowCutFp64 = 0x1.0p-40;
// FP64 residual products at least this tall, and this deep, go to the library GEMM
// (measured: faster for blocks of 128 rows at depth >= 256, slower for blocks of 32; on
// rows of 16384 or more columns also from depth 64: 47 against 60-90 us for the two
// 110 x 100 x 40000 products of an iteration).
constexpr int64_t kLibraryGemmMinK = 256;
constexpr int64_t kLibraryGemmMinKWide = 64;
constexpr int64_t kLibraryGemmWideN = 16384;
constexpr int64_t kLibraryGemmMinM = 96;
constexpr double kRowCutFp32 = 0x1.0p-16;

double risk_factor(double alpha, double delta, int64_t c, int* status) {
  *status = ICUR_OK;
  if (alpha == 0.0) return 1.0;
  if (!(alpha > 0.0 && alpha < 1.0) || !(delta >= 0.0) || !std::isfinite(delta)) {
    *status = arg_error("risk-aware stopping needs 0 < alpha < 1 and delta >= 0");
    return 1.0;
  }
  if (!(static_cast<double>(c) > -4.0 * std::log(alpha))) {
    *status = arg_error("risk-aware stopping needs c > -4 ln(alpha)");
    return 1.0;
  }
  return (1.0 + delta) * std::sqrt(1.0 - 2.0 * std::sqrt(-std::log(alpha) / static_cast<double>(c)));
}

// --------------------------------------------------------------------- the driver
// The matrix the loop reads: dense FP32 (A, lda), or CSR with its CSC copy.  Only the
// sketch and the three gathers (columns A(:,J_k), rows A(I_k,:), the cross A(I,J))
// depend on it; every other step works on dense gathered operands.
struct Source {
  const float* A = nullptr;
  int64_t lda = 0;
  const CsrMatrix* csr = nullptr;  // checked and copied to CSC by run_impl
};

// Every argument check of a run, before any device work: shape, tolerance, block, sketch
// kind and options.  On success *o holds the options with defaults applied.
int check_run_args(bool sparse, const float* A, int64_t m, int64_t n, int64_t lda, double tol, int32_t block,
                   int32_t kind, const icur_opts* opts, icur_opts* o) {
  if (!A && !sparse) return arg_error("A is null");
  if (m < 1 || n < 1) return arg_error("need m >= 1 and n >= 1");
  if (!sparse && lda < n) return arg_error("need lda >= n");
  if (!(tol > 0.0) || !std::isfinite(tol)) return arg_error("tol must be finite and > 0");
  if (block < 1 || block > std::min(m, n)) return arg_error("need 1 <= block <= min(m, n)");
  if (kind != ICUR_SKETCH_GAUSSIAN && kind != ICUR_SKETCH_SPARSE_SIGN && kind != ICUR_SKETCH_SRTT)
    return arg_error("unknown sketch kind");
  if (m > 0x7fffffffLL || n > 0x7fffffffLL) return arg_error("m and n must be below 2^31");
  std::memset(o, 0, sizeof(*o));
  if (opts) *o = *opts;
  const int64_t b = block;
  const int64_t c = (11 * b) / 10;
  if (c > 4096) return arg_error("sketch rows c = floor(1.1 b) above 4096 are not supported");
  // the pivot blocks N_k (b x b) are inverted by one workgroup, up to 512 rows
  if (b > 512) return arg_error("block above 512 is not supported");
  if (kind == ICUR_SKETCH_SPARSE_SIGN && c > 255) return arg_error("sparse-sign sketch needs c <= 255");
  if (sparse && c > 256) return arg_error("the CSR sketch needs c = floor(1.1 b) <= 256");
  if (sparse && kind == ICUR_SKETCH_SRTT) return arg_error("the CSR path takes the Gaussian or sparse-sign sketch");
  if (kind == ICUR_SKETCH_SRTT && c > m) return arg_error("the SRTT sketch needs c = floor(1.1 b) <= m");
  if (o->zeta < 0 || o->zeta > 8) return arg_error("zeta must be at most 8");
  if (o->precision != ICUR_FP32 && o->precision != ICUR_BF16_SPLIT) return arg_error("unknown precision");
  if (o->split_terms < 0 || o->split_terms > 3) return arg_error("split_terms must be 0..3");
  if (o->residual_fp64 < -1 || o->residual_fp64 > 1) return arg_error("residual_fp64 must be -1, 0 or 1");
  if (o->max_rank < 0) return arg_error("max_rank must be >= 0");
  if (o->batch_workers < 0 || o->batch_workers > 16) return arg_error("batch_workers must be 0..16");
  if (o->denominator != ICUR_DENOM_GA && o->denominator != ICUR_DENOM_A) return arg_error("unknown denominator");
  if (o->selection != ICUR_SELECT_LUPP && o->selection != ICUR_SELECT_QRCP) return arg_error("unknown selection");
  if (o->device_outputs != 0 && o->device_outputs != 1) return arg_error("device_outputs must be 0 or 1");
  // the Corollary of §3.3 is stated for a Gaussian G
  if (o->alpha != 0.0 && kind != ICUR_SKETCH_GAUSSIAN)
    return arg_error("risk-aware stopping needs the Gaussian sketch (the §3.3 Corollary's hypothesis)");
  int st_risk = ICUR_OK;
  (void)risk_factor(o->alpha, o->delta, c, &st_risk);
  return st_risk;
}

}  // namespace

// BF16 pieces per FP32 operand for a tolerance.  One piece rounds with relative error
// up to 2^-8, two with 2^-16, three reproduce FP32.  The sketched residual's noise
// floor is this error amplified by the interpolation coefficients of the cross, so the
// count leaves a wide margin: one piece only for very loose tolerances.
int terms_for_tol(double tol) {
  if (tol >= 1e-1) return 1;
  if (tol >= 5e-4) return 2;
  return 3;
}

// BF16 pieces per operand of the precision form's residual products (see run_impl).
int residual_terms_for_tol(double tol) { return tol >= 1e-1 ? 2 : 3; }

// The precision form runs FP32 factors from this tolerance up (see run_impl).
constexpr double kSplitResidualMinTol = 1e-4;

// G (c x m BF16, leading dimension ldg) drawn from (kind, seed, zeta), X0 = G A into S
// (c x n FP64) and ||X0||_F^2 into *normsq_dev: the sketch kernel when the shape allows
// (A split into `terms` BF16 pieces), else the general product.  ev_begin / ev_end (may
// be null) bracket the product kernel.
size_t sketch_G_bytes(int kind, int64_t c, int64_t m, int64_t ldg) {
  if (kind == ICUR_SKETCH_SRTT)
    return ((static_cast<size_t>(c) * ldg * 4 + 255) & ~size_t(255)) + static_cast<size_t>(c) * 8 + static_cast<size_t>(m) + 256;
  return static_cast<size_t>(c) * ldg * 2;
}

int form_sketch(int kind, uint64_t seed, int64_t c, int64_t m, int64_t n, const float* A, int64_t lda, int zeta,
                int terms, bool precise, uint16_t* G, int64_t ldg, double* S, double* partials, void* ws,
                size_t ws_bytes, double* normsq_dev, hipStream_t st, hipEvent_t ev_begin, hipEvent_t ev_end,
                bool* used_kernel) {
  if (used_kernel) *used_kernel = false;
  const bool srtt = (kind == ICUR_SKETCH_SRTT);
  if (kind == ICUR_SKETCH_GAUSSIAN) {
    ICUR_TRY(launch_gaussian_G(seed, c, m, G, ldg, st));
  } else if (kind == ICUR_SKETCH_SPARSE_SIGN) {
    ICUR_TRY(launch_sparse_sign(seed, c, m, zeta, nullptr, nullptr, G, ldg, st));
  } else {
    // the SRTT operator is not BF16-exact: FP32 G on the FP32 matrix cores
    char* gp = reinterpret_cast<char*>(G);
    const size_t gbytes = (static_cast<size_t>(c) * ldg * 4 + 255) & ~size_t(255);
    ICUR_TRY(launch_srtt(seed, c, m, reinterpret_cast<float*>(gp), ldg, reinterpret_cast<int64_t*>(gp + gbytes),
                         reinterpret_cast<uint8_t*>(gp + gbytes + static_cast<size_t>(c) * 8), st));
    terms = 0;
  }
  int parts = 0;
  int sk = ICUR_ERR_UNSUPPORTED;
  if (terms > 0)
    sk = sketch_product(G, ldg, c, A, m, n, lda, terms, precise, S, n, partials, &parts, ws, ws_bytes, st, ev_begin,
                        ev_end);
  if (sk != ICUR_OK && sk != ICUR_ERR_UNSUPPORTED) return sk;
  if (used_kernel) *used_kernel = (sk == ICUR_OK);
  if (sk == ICUR_ERR_UNSUPPORTED) {
    if (ev_begin) ICUR_HIP(hipEventRecord(ev_begin, st));
    WideGemm g{};
    g.W = G;
    g.ldw = ldg;
    g.wterms = terms == 0 ? 0 : 1;
    g.w_bf16 = !srtt;
    g.B = A;
    g.ldb = lda;
    g.bterms = terms;
    g.M = c;
    g.K = m;
    g.N = n;
    g.subtract = false;
    g.out64 = true;
    g.OUT = S;
    g.ldo = n;
    g.norm_partials = partials;
    g.nparts = &parts;
    ICUR_TRY(wide_gemm(g, ws, ws_bytes, st));
    if (ev_end) ICUR_HIP(hipEventRecord(ev_end, st));
  }
  return launch_reduce_partials(partials, parts, normsq_dev, st);
}

namespace {

// OUT = X - W B (subtract) or W B in FP64 (W is M x K with leading dimension ldw, B is
// K x N, X and OUT M x N), routed as the loop routes its residual products: products of
// at least kLibraryGemmMinM rows at depth >= kLibraryGemmMinK (or >= kLibraryGemmMinKWide
// on rows of >= kLibraryGemmWideN columns), in place (X == OUT) or plain (X null), on the
// library FP64 GEMM, with the norm partials from a separate pass; all others on the
// short-M FP64 matrix-core kernel, which fuses the partials.  norm_partials may be null.
int product_f64(const double* W, int64_t ldw, int64_t M, int64_t K, const double* X, int64_t ldx, const double* B,
                int64_t ldb, int64_t N, bool subtract, double* OUT, int64_t ldo, double* norm_partials, int* parts,
                void* gemm_ws, size_t gemm_ws_bytes, hipStream_t st) {
  if (M >= kLibraryGemmMinM && (K >= kLibraryGemmMinK || (K >= kLibraryGemmMinKWide && N >= kLibraryGemmWideN)) &&
      ((X == OUT && subtract) || (X == nullptr && !subtract))) {
    ICUR_TRY(dgemm(M, N, K, subtract ? -1.0 : 1.0, W, ldw, 1, B, ldb, 1, subtract ? 1.0 : 0.0, OUT, ldo, st));
    if (norm_partials) {
      const int blocks = static_cast<int>(std::min<int64_t>((M * N + 255) / 256, 1024));
      ICUR_TRY(wide::launch_reduce_f64(nullptr, 0, M, N, OUT, ldo, 1, OUT, ldo, norm_partials, blocks, st));
      *parts = blocks;
    } else {
      *parts = 0;
    }
    return ICUR_OK;
  }
  WideGemm g{};
  g.X = X;
  g.ldx = ldx;
  g.W = W;
  g.ldw = ldw;
  g.wterms = -1;
  g.B = B;
  g.ldb = ldb;
  g.bterms = -1;
  g.M = M;
  g.K = K;
  g.N = N;
  g.subtract = subtract;
  g.out64 = true;
  g.OUT = OUT;
  g.ldo = ldo;
  g.norm_partials = norm_partials;
  g.nparts = parts;
  return wide_gemm(g, gemm_ws, gemm_ws_bytes, st);
}

// cache_slot: the workspace to use (0 for single calls); lupp_groups > 0 caps the
// workgroups of the selection grids (concurrent batched workers share the CUs); timing
// false skips the per-phase device events.
int run_impl(const Source& src, int64_t m, int64_t n, double tol, int32_t block, int32_t kind, uint64_t seed,
             const icur_opts* opts, int64_t* I_out, int64_t* J_out, double* U_out, int64_t* rank_out,
             double* est_out, std::chrono::steady_clock::time_point t_start, int cache_slot = 0,
             int lupp_groups = 0, bool timing = true) {
  const float* A = src.A;
  const int64_t lda = src.lda;
  const bool sparse = (src.csr != nullptr);
  // ---- arguments (before any device work)
  if (!I_out || !J_out || !U_out || !rank_out || !est_out) return arg_error("null output pointer");
  icur_opts o;
  ICUR_TRY(check_run_args(sparse, A, m, n, lda, tol, block, kind, opts, &o));
  const int64_t b = block;
  const int64_t c = (11 * b) / 10;
  const int zeta = o.zeta > 0 ? o.zeta : 8;
  const int64_t rmax = (o.max_rank == 0) ? std::min(m, n) : std::min(o.max_rank, std::min(m, n));
  int st_risk = ICUR_OK;
  const double xi = risk_factor(o.alpha, o.delta, c, &st_risk);
  if (st_risk != ICUR_OK) return st_risk;
  const double thr = xi * tol;
  const bool denom_a = (o.denominator == ICUR_DENOM_A);
  // s_G^2: E ||G x||^2 = s_G^2 ||x||^2 for the unscaled operators
  const double sg2 = kind == ICUR_SKETCH_GAUSSIAN ? static_cast<double>(c)
                     : kind == ICUR_SKETCH_SRTT   ? 1.0
                                                  : static_cast<double>(std::min<int64_t>(zeta, c));
  const bool split = (o.precision == ICUR_BF16_SPLIT);
  const int T = split ? (o.split_terms ? o.split_terms : terms_for_tol(tol)) : 0;
  // sketch pieces: the plain form forms every product exactly (three pieces of A times a
  // BF16-exact G) unless FP32 matrix cores are asked for
  const int sketch_terms = split ? T : (o.sketch_fp32 ? 0 : 3);
  // Residual factors.  Plain form: FP64 factors on the FP64 matrix cores.  Precision
  // form at tol >= 1e-4 (and residual_fp64 = -1): the factors LcT and Ur are stored in
  // FP32 and the two large products of every iteration, the row residual at the new
  // columns and the residual at the new rows, run on BF16 pieces of both operands (FP32
  // matrix cores in the plain form) with FP32 chunk sums added in FP64.  N_k^{-1}
  // S(I_k,:) stays FP64: N_k^{-1} grows like cond(N_k) while Ur_k stays O(1), so it must
  // not be rounded before it multiplies; the column update S -= S(:,J_k) Ur_k and its
  // norm use that FP64 Ur_k.  The residual form rebuilds A(I_k,:) from the factors and
  // subtracts, so FP32 factors (and FP32 sums) leave an absolute error near 2^-24 of the
  // entries of A in every residual; below tol 1e-4 that reaches the residual itself on
  // slowly decaying spectra (the estimate then undershoots the error), so the precision
  // form keeps FP64 factors there.  residual_fp64 = 1 forces FP64 factors in either form.
  const bool res64 = o.residual_fp64 == 1 || (o.residual_fp64 == 0 && !(split && tol >= kSplitResidualMinTol));
  const size_t fsz = res64 ? 8 : 4;
  // BF16 pieces of the FP32-factor products: their rounding enters the residual relative
  // to the scale of A, and the next factors amplify it by the conditioning of the pivot
  // blocks, so the residual needs more than the sketch: three pieces (FP32-exact
  // operands) below tol 1e-1, two above; none on the plain form's FP32 matrix cores
  const int Tres = split ? residual_terms_for_tol(tol) : 0;
  hipStream_t st = as_stream(o.stream);

  DeviceCache* dcp = nullptr;
  ICUR_TRY(prepare_device(&dcp, cache_slot));
  DeviceCache& dc = *dcp;
  std::lock_guard<std::mutex> lock(dc.mu);
  DeviceInfo dev;
  ICUR_TRY(device_info(&dev));
  Timer tm{&dc, st};
  tm.on = timing;
  CscCopy csc{};
  if (sparse) {
    // a canonical CSR is required: rowptr from 0 to nnz, columns in range, sorted and
    // unique within each row (checked on the device before anything else)
    const CsrMatrix& S0 = *src.csr;
    void* pc;
    ICUR_TRY(ensure(dc, kCsc, csc_workspace_bytes(S0.nnz, S0.n) + 256, &pc));
    unsigned* flag = reinterpret_cast<unsigned*>(static_cast<char*>(pc) + csc_workspace_bytes(S0.nnz, S0.n));
    ICUR_TRY(csr_validate(S0, flag, st));
    int hflag = 0;
    ICUR_TRY(read_int(dc, reinterpret_cast<const int*>(flag), &hflag, 1, st));
    if (hflag & 1) return arg_error("CSR: rowptr must start at 0, end at nnz and not decrease");
    if (hflag & 2) return arg_error("CSR: column index out of range [0, n)");
    if (hflag & 4) return arg_error("CSR: column indices must be strictly increasing within each row");
    ICUR_TRY(csc_build(S0, &csc, pc, csc_workspace_bytes(S0.nnz, S0.n), st));
  }

  // ---- fixed-size buffers
  void *pG, *pX0, *pSr, *pColMask, *pRowMask, *pJk, *pIk, *pLupp, *pGemm, *pNorm, *pScal, *pN;
  const int64_t ldg = (m + 7) / 8 * 8;  // 16-byte aligned rows of G for the sketch kernel
  ICUR_TRY(ensure(dc, kG, sparse ? csr_sketch_aux_bytes(m, c) : sketch_G_bytes(kind, c, m, ldg), &pG));
  ICUR_TRY(ensure(dc, kX0, static_cast<size_t>(c) * n * 8, &pX0));
  ICUR_TRY(ensure(dc, kSrow, static_cast<size_t>(b) * n * 8, &pSr));  // FP64 in both forms
  ICUR_TRY(ensure(dc, kColMask, static_cast<size_t>(n), &pColMask));
  ICUR_TRY(ensure(dc, kRowMask, static_cast<size_t>(m), &pRowMask));
  ICUR_TRY(ensure(dc, kJk, static_cast<size_t>(b) * 8, &pJk));
  ICUR_TRY(ensure(dc, kIk, static_cast<size_t>(b) * 8, &pIk));
  ICUR_TRY(ensure(dc, kA22, static_cast<size_t>(b) * b * 16 + small_inverse_work_bytes(b), &pN));
  ICUR_TRY(ensure(dc, kLupp, lupp_workspace_bytes(b, std::max(m, n)), &pLupp));
  const int64_t BIGK = int64_t(1) << 40;
  size_t gemm_ws = wide_gemm_workspace_bytes(c, m, n, dev.num_cus);
  gemm_ws = std::max(gemm_ws, wide_gemm_workspace_bytes(c, BIGK, n, dev.num_cus));
  gemm_ws = std::max(gemm_ws, wide_gemm_workspace_bytes(b, BIGK, m, dev.num_cus));
  gemm_ws = std::max(gemm_ws, wide_gemm_workspace_bytes(b, BIGK, n, dev.num_cus));
  gemm_ws = std::max(gemm_ws, sketch_workspace_bytes(c, m, n, dev.num_cus));
  ICUR_TRY(ensure(dc, kGemmWs, gemm_ws, &pGemm));
  const int nparts_cap = std::max(std::max(std::max(std::max(max_norm_partials(c, n), max_norm_partials(b, m)), kSumsqMaxParts),
                                           sketch_max_norm_partials(c, n)),
                                  csr_max_norm_partials(n));
  ICUR_TRY(ensure(dc, kNormPart, static_cast<size_t>(nparts_cap) * 8, &pNorm));
  ICUR_TRY(ensure(dc, kScal, sizeof(Scal), &pScal));
  void* pUrk64 = nullptr;  // FP64 Ur_k of the FP32-factor path
  if (!res64) ICUR_TRY(ensure(dc, kUrk64, static_cast<size_t>(b) * n * 8, &pUrk64));
  LuppWork lw;
  lupp_bind_workspace(pLupp, b, std::max(m, n), &lw);
  lw.max_groups = lupp_groups;
  const bool qrcp = (o.selection == ICUR_SELECT_QRCP);
  void* pQr = nullptr;
  if (qrcp)
    ICUR_TRY(ensure(dc, kQrcp, std::max(qrcp_workspace_bytes(c, n, 4 * dev.num_cus), qrcp_workspace_bytes(b, m, 4 * dev.num_cus)),
                    &pQr));
  // the selection of Alg. 1: LUPP (default) or QRCP, same status words
  auto select = [&](const void* X, bool x64, int64_t K, int64_t N, int64_t ldx, int steps, const uint8_t* excl,
                    int64_t* piv, double rel_cut) -> int {
    if (qrcp)
      return qrcp_launch(X, x64, K, N, ldx, steps, excl, piv, lw.status, pQr, dc.buf[kQrcp].bytes, st, rel_cut);
    return lupp_launch(X, x64, K, N, ldx, steps, excl, piv, lw, st, rel_cut);
  };
  Scal* dscal = static_cast<Scal*>(pScal);
  double* dnorm = static_cast<double*>(pNorm);
  double* Nblk = static_cast<double*>(pN);                 // b x b, then its inverse
  double* N1inv = Nblk + static_cast<size_t>(b) * b;       // N_1^{-1}, kept for the core
  double* Nwork = N1inv + static_cast<size_t>(b) * b;      // Gauss-Jordan work (b > 128)
  const int64_t bc = std::max(b, c);

  // ---- rank-sized buffers, grown geometrically: the residual-form factors
  //   LcT (r x m): column factors, row t = S^{(k-1)}(:, J_k[t])^T  (S^row of its block)
  //   Ur  (r x n): row factors, block k = N_k^{-1} S^{(k-1)}(I_k, :)
  // with A - C U R = A - sum_k Lc_k Ur_k (the residual-recurrence lemma of §4.2).
  int64_t rcap = 0;
  void *pLcT = nullptr, *pUr = nullptr, *pJall = nullptr, *pIall = nullptr, *pW64 = nullptr, *pWp = nullptr;
  auto grow_to = [&](int64_t need) -> int {
    if (need <= rcap) return ICUR_OK;
    int64_t nc = std::max<int64_t>(std::max<int64_t>(rcap * 2, need), std::min<int64_t>(rmax, std::max<int64_t>(4 * b, 512)));
    nc = std::min(nc, rmax);
    if (nc < need) nc = need;
    const int64_t keep = rcap;
    ICUR_TRY(grow_keep(dc, kCt, static_cast<size_t>(nc) * m * fsz, keep, static_cast<size_t>(m) * fsz,
                       static_cast<size_t>(m) * fsz, static_cast<size_t>(m) * fsz, st, &pLcT));
    ICUR_TRY(grow_keep(dc, kR, static_cast<size_t>(nc) * n * fsz, keep, static_cast<size_t>(n) * fsz,
                       static_cast<size_t>(n) * fsz, static_cast<size_t>(n) * fsz, st, &pUr));
    ICUR_TRY(grow_keep(dc, kJall, static_cast<size_t>(nc) * 8, 1, static_cast<size_t>(keep) * 8,
                       static_cast<size_t>(keep) * 8 + 8, static_cast<size_t>(nc) * 8 + 8, st, &pJall));
    ICUR_TRY(grow_keep(dc, kIall, static_cast<size_t>(nc) * 8, 1, static_cast<size_t>(keep) * 8,
                       static_cast<size_t>(keep) * 8 + 8, static_cast<size_t>(nc) * 8 + 8, st, &pIall));
    ICUR_TRY(ensure(dc, kW64, static_cast<size_t>(bc) * std::max(nc, b) * 8, &pW64));
    ICUR_TRY(ensure(dc, kWp, static_cast<size_t>(bc) * std::max(nc, b) * 6, &pWp));
    rcap = nc;
    return ICUR_OK;
  };
  // OUT = X - W B (subtract) or W B, W given in FP64 (rows x K, ld K) and split here;
  // X and OUT are FP64 when out64.
  auto product = [&](const double* W64, int64_t M, int64_t K, const void* X, int64_t ldx, const void* B,
                     int64_t ldb, int64_t N, bool subtract, void* OUT, int64_t ldo, bool norm, bool out64,
                     int* parts) -> int {
    // res64: W and B are FP64 and OUT is FP64 (FP64 matrix cores); else W is split into
    // BF16 pieces (or rounded to FP32) and B is FP32.
    if (res64)
      return product_f64(W64, K, M, K, static_cast<const double*>(X), ldx, static_cast<const double*>(B), ldb, N,
                         subtract, static_cast<double*>(OUT), ldo, norm ? dnorm : nullptr, parts, pGemm,
                         dc.buf[kGemmWs].bytes, st);
    if (K > 0) ICUR_TRY(launch_split_f64(W64, M, K, K, false, Tres, pWp, K, M * K, st));
    WideGemm g{};
    g.X = X;
    g.ldx = ldx;
    g.W = pWp;
    g.ldw = K;
    g.wterms = Tres;
    g.B = B;
    g.ldb = ldb;
    g.bterms = Tres;
    g.M = M;
    g.K = K;
    g.N = N;
    g.subtract = subtract;
    g.out64 = out64;
    g.OUT = OUT;
    g.ldo = ldo;
    g.norm_partials = norm ? dnorm : nullptr;
    g.nparts = parts;
    return wide_gemm(g, pGemm, dc.buf[kGemmWs].bytes, st);
  };

  // ---- sketch: G, X0 = G A, ||X0||_F^2
  size_t ev_s0, ev_s1, ev_p0, ev_p1;
  ICUR_TRY(tm.mark(&ev_s0));
  uint16_t* G = static_cast<uint16_t*>(pG);
  double* S = static_cast<double*>(pX0);  // X0, then the sketched column residual in place (FP64)
  if (sparse) {
    // G is drawn inside (as row masks or transposed Gaussian values); X0 from the CSC copy
    int parts = 0;
    ICUR_TRY(tm.mark(&ev_p0));
    ICUR_TRY(csr_sketch(csc, m, n, c, kind, seed, zeta, S, n, dnorm, &parts, pG, st));
    ICUR_TRY(tm.mark(&ev_p1));
    ICUR_TRY(launch_reduce_partials(dnorm, parts, &dscal->normsq_x0, st));
  } else {
    // ev_p0 / ev_p1 bracket the sketch kernel itself (the first 160-row slice of G when
    // c > 160), not its split-K reduce; the general product is bracketed whole
    ICUR_TRY(tm.reserve(&ev_p0));
    ICUR_TRY(tm.reserve(&ev_p1));
    bool used = false;
    ICUR_TRY(form_sketch(kind, seed, c, m, n, A, lda, zeta, sketch_terms, tol < kSketchChunkFlushBelow, G, ldg, S,
                         dnorm, pGemm, dc.buf[kGemmWs].bytes, &dscal->normsq_x0, st, tm.event(ev_p0),
                         tm.event(ev_p1), &used));
    t_info.sketch_kernel = used ? 1 : 0;
  }
  if (denom_a) {
    int parts = 0;
    if (sparse)
      ICUR_TRY(launch_sumsq_f32(src.csr->vals, 1, src.csr->nnz, std::max<int64_t>(src.csr->nnz, 1), dnorm, &parts, st));
    else
      ICUR_TRY(launch_sumsq_f32(A, m, n, lda, dnorm, &parts, st));
    ICUR_TRY(launch_reduce_partials(dnorm, parts, &dscal->normsq_a, st));
  }
  ICUR_TRY(launch_fill_u8(static_cast<uint8_t*>(pColMask), n, 0, st));
  ICUR_TRY(launch_fill_u8(static_cast<uint8_t*>(pRowMask), m, 0, st));
  ICUR_TRY(tm.mark(&ev_s1));
  tm.add(ev_s0, ev_s1, &t_info.ms_sketch);
  tm.add(ev_p0, ev_p1, &t_info.ms_sketch_product);
  t_info.threshold = thr;
  t_info.split_terms = T;
  t_info.residual_terms = res64 ? -1 : Tres;
  // ||G A||_F^2 is read back with the first selection's status (one synchronisation
  // less); the selection on a zero or non-finite sketch is harmless and discarded.
  // Returns 1 when the call ends here (rank 0, or an error in *err).
  Scal hs;
  double gnorm2 = -1.0;
  double denom2 = -1.0;  // the estimate's squared denominator: ||G A||_F^2 or s_G^2 ||A||_F^2
  int norm_err = ICUR_OK;
  auto take_norm = [&]() -> bool {
    gnorm2 = hs.normsq_x0;
    t_info.sketch_norm = std::sqrt(gnorm2);
    if (!std::isfinite(gnorm2)) {
      set_error("||G A||_F is not finite: A holds Inf or NaN");
      norm_err = ICUR_ERR_NONFINITE;
      return true;
    }
    denom2 = denom_a ? sg2 * hs.normsq_a : gnorm2;
    // with the ||A||_F denominator the empty approximation already has rho < 1, and may
    // meet the tolerance without any index
    const double rho0 = gnorm2 == 0.0 ? 0.0 : std::sqrt(gnorm2 / denom2);
    if (gnorm2 == 0.0 || (denom_a && rho0 <= thr)) {
      *rank_out = 0;
      *est_out = rho0;
      tm.flush();
      t_info.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
      return true;
    }
    return false;
  };

  // ---- the loop of Alg. 1, residual form
  int64_t r = 0;
  double rho = 1.0;
  int status = ICUR_OK;
  int64_t* Jk = static_cast<int64_t*>(pJk);
  int64_t* Ik = static_cast<int64_t*>(pIk);
  std::vector<int64_t> blocks;
  // factor element access: FP32 or FP64 storage
  auto fp = [&](void* base, int64_t elems) -> void* { return static_cast<char*>(base) + elems * fsz; };
  auto gather_w = [&](const void* src, int64_t lds, int64_t rk, const int64_t* cols, int64_t ck, bool trans,
                      double* dst, int64_t ldd) -> int {
    return res64 ? launch_gather_f64(static_cast<const double*>(src), lds, nullptr, rk, cols, ck, trans, dst, ldd, st)
                 : launch_gather_f64(static_cast<const float*>(src), lds, nullptr, rk, cols, ck, trans, dst, ldd, st);
  };
  size_t iter_start = ev_s1;
  while (rho > thr && r < rmax) {
    const int64_t s = std::min(b, rmax - r);
    ICUR_TRY(grow_to(r + s));
    void* LcT = pLcT;
    void* Ur = pUr;
    void* Sr = pSr;
    double* W64 = static_cast<double*>(pW64);
    // e0: the previous iteration's end (nothing is queued in between)
    size_t e0 = iter_start, e1, e2, e3, e4;
    int parts = 0;
    // column selection: LUPP on (S^col)^T
    ICUR_TRY(select(S, true, c, n, n, static_cast<int>(s), static_cast<const uint8_t*>(pColMask), Jk, 0.0));
    ICUR_TRY(tm.mark(&e1));
    int lst[2];
    if (gnorm2 < 0.0) {
      ICUR_TRY(read_int_scal(dc, lw.status, lst, 2, dscal, &hs, st));
      if (take_norm()) return norm_err;
    } else {
      ICUR_TRY(read_int(dc, lw.status, lst, 2, st));
    }
    if (lst[1]) {
      set_error("selection kernel: grid barrier did not complete");
      return ICUR_ERR_HIP;
    }
    const int64_t nJ = lst[0];
    if (nJ == 0) {
      status = ICUR_STALLED;
      break;
    }
    // row residual S^row = A(:,J_k) - C U R(:,J_k) = A(:,J_k) - Lc Ur(:,J_k), stored
    // transposed as the next rows of LcT
    void* Lk = fp(LcT, r * m);
    if (sparse) {
      if (res64)
        ICUR_TRY(csc_gather_cols_T(csc, m, Jk, nJ, static_cast<double*>(Lk), m, st));
      else
        ICUR_TRY(csc_gather_cols_T(csc, m, Jk, nJ, static_cast<float*>(Lk), m, st));
    } else if (res64) {
      ICUR_TRY(launch_gather_cols_T(A, m, n, lda, Jk, nJ, static_cast<double*>(Lk), m, st));
    } else {
      ICUR_TRY(launch_gather_cols_T(A, m, n, lda, Jk, nJ, static_cast<float*>(Lk), m, st));
    }
    if (r > 0) {
      ICUR_TRY(gather_w(Ur, n, r, Jk, nJ, true, W64, r));   // Ur(:,J_k)^T
      ICUR_TRY(product(W64, nJ, r, Lk, m, LcT, m, m, true, Lk, m, false, false, &parts));
    }
    ICUR_TRY(tm.mark(&e2));
    // row selection: LUPP on S^row
    ICUR_TRY(select(Lk, res64, nJ, m, m, static_cast<int>(nJ), static_cast<const uint8_t*>(pRowMask), Ik,
                    res64 ? kRowCutFp64 : kRowCutFp32));
    ICUR_TRY(tm.mark(&e3));
    ICUR_TRY(read_int(dc, lw.status, lst, 2, st));
    if (lst[1]) {
      set_error("selection kernel: grid barrier did not complete");
      return ICUR_ERR_HIP;
    }
    const int64_t nI = lst[0];
    if (nI == 0) {
      status = ICUR_STALLED;
      break;
    }
    // N_k = S^{(k-1)}(I_k, J_k) and its inverse (FP64), and the residual at the new rows
    // Sr = A(I_k,:) - Lc(I_k,:) Ur (FP64 in both forms).  With FP64 factors N_k is read
    // from the row residual S^row; with FP32 factors it is read from Sr, the FP64 product
    // that N_k^{-1} multiplies, so that Ur_k(:, J_k) is the identity to FP64 rounding (the
    // FP32-stored S^row differs from Sr by its rounding, which cond(N_k) would amplify)
    auto pivot_block = [&](const void* from_rows, bool from_sr) -> int {
      if (from_sr)
        ICUR_TRY(launch_gather_f64(static_cast<const double*>(from_rows), n, nullptr, nI, Jk, nI, false, Nblk, nI,
                                   st));
      else
        ICUR_TRY(gather_w(from_rows, m, nI, Ik, nI, true, Nblk, nI));
      ICUR_TRY(launch_inorder_inverse(Nblk, nI, Nwork, &dscal->info, st));
      // N_1 = A(I_1, J_1) exactly: its inverse is the core's first diagonal block inverse
      if (r == 0)
        ICUR_HIP(hipMemcpyAsync(N1inv, Nblk, static_cast<size_t>(nI) * nI * 8, hipMemcpyDeviceToDevice, st));
      return ICUR_OK;
    };
    if (res64) ICUR_TRY(pivot_block(Lk, false));
    if (sparse)
      ICUR_TRY(csr_gather_rows(*src.csr, Ik, nI, static_cast<double*>(Sr), n, st));
    else
      ICUR_TRY(launch_gather_rows(A, m, n, lda, Ik, nI, static_cast<double*>(Sr), n, st));
    if (r > 0) {
      ICUR_TRY(gather_w(LcT, m, r, Ik, nI, true, W64, r));  // Lc(I_k,:)
      ICUR_TRY(product(W64, nI, r, Sr, n, Ur, n, n, true, Sr, n, false, true, &parts));
    }
    if (!res64) ICUR_TRY(pivot_block(Sr, true));
    // new row factors Ur_k = N_k^{-1} Sr (FP64), then the column residual update
    // S^col <- S^col - S^col(:,J_k) Ur_k and its norm (FP64)
    void* Urk = fp(Ur, r * n);
    double* Urk64 = res64 ? static_cast<double*>(Urk) : static_cast<double*>(pUrk64);
    ICUR_TRY(product_f64(Nblk, nI, nI, nI, nullptr, n, static_cast<const double*>(Sr), n, n, false, Urk64, n, nullptr,
                         &parts, pGemm, dc.buf[kGemmWs].bytes, st));
    if (!res64) ICUR_TRY(convert_f64_f32_norm(Urk64, nI, n, static_cast<float*>(Urk), n, dnorm, nullptr, st));
    ICUR_TRY(launch_gather_f64(S, n, nullptr, c, Jk, nI, false, W64, nI, st));
    ICUR_TRY(product_f64(W64, nI, c, nI, S, n, Urk64, n, n, true, S, n, dnorm, &parts, pGemm, dc.buf[kGemmWs].bytes,
                         st));
    if (dc.host_pinned_dev) {
      // norm, commit and the scalar read-back in one launch
      const bool flag = dc.spin;
      const unsigned seq = flag ? ++dc.flag_seq : 0u;
      unsigned* flag_dev =
          flag ? reinterpret_cast<unsigned*>(static_cast<char*>(dc.host_pinned_dev) + kFlagOffset) : nullptr;
      ICUR_TRY(launch_iteration_end(dnorm, parts, &dscal->normsq_s, static_cast<uint8_t*>(pColMask),
                                    static_cast<uint8_t*>(pRowMask), Jk, Ik, nI, static_cast<int64_t*>(pJall) + r,
                                    static_cast<int64_t*>(pIall) + r, dscal, static_cast<int64_t>(sizeof(Scal)),
                                    dc.host_pinned_dev, flag_dev, seq, st));
      ICUR_TRY(tm.mark(&e4));
      if (flag)
        ICUR_TRY(wait_flag(dc, seq, st));
      else
        ICUR_TRY(sync_stream(dc, st));
      hs = *static_cast<const Scal*>(dc.host_pinned);
    } else {
      ICUR_TRY(launch_reduce_partials(dnorm, parts, &dscal->normsq_s, st));
      ICUR_TRY(launch_commit_block(static_cast<uint8_t*>(pColMask), static_cast<uint8_t*>(pRowMask), Jk, Ik, nI,
                                   static_cast<int64_t*>(pJall) + r, static_cast<int64_t*>(pIall) + r, st));
      ICUR_TRY(tm.mark(&e4));
      ICUR_TRY(read_scal(dc, dscal, &hs, st));
    }
    if (hs.info != 0) {
      set_error("the residual block N_k = S(I_k, J_k) is exactly singular");
      return ICUR_ERR_HIP;
    }
    r += nI;
    blocks.push_back(nI);
    rho = std::sqrt(hs.normsq_s / denom2);
    const int it = t_info.iterations++;
    if (it < 512) {
      t_info.rho[it] = rho;
      t_info.block_sizes[it] = static_cast<int32_t>(nI);
    }
    t_info.n_rho = std::min(t_info.iterations, 512);
    tm.add(e0, e1, &t_info.ms_select);
    tm.add(e2, e3, &t_info.ms_select);
    tm.add(e1, e2, &t_info.ms_residual);
    tm.add(e3, e4, &t_info.ms_residual);
    iter_start = e4;
  }
  if (gnorm2 < 0.0) {  // no iteration ran
    ICUR_TRY(read_scal(dc, dscal, &hs, st));
    if (take_norm()) return norm_err;
  }
  if (status == ICUR_OK && rho > thr) status = ICUR_MAXRANK;

  // ---- the core U = A(I,J)^{-1} in FP64 from the exact cross entries: block LU in the
  //      selection order (its diagonal blocks are the pivot blocks N_k of the row
  //      selections), block triangular solves on the identity, and one Newton step
  if (r > 0) {
    // the core starts where the last iteration ended, unless the loop stopped part-way
    size_t ec0 = iter_start, ec1;
    if (status == ICUR_STALLED) ICUR_TRY(tm.mark(&ec0));
    void *pU, *pM, *pCore;
    const int64_t nb = static_cast<int64_t>(blocks.size());
    ICUR_TRY(ensure(dc, kU, static_cast<size_t>(r) * r * 8, &pU));
    ICUR_TRY(ensure(dc, kY, static_cast<size_t>(r) * r * 8, &pM));
    ICUR_TRY(ensure(dc, kCoreWs, core_inverse_ws_doubles(r, b) * 8 + static_cast<size_t>(nb) * 4 + 256, &pCore));
    double* U = static_cast<double*>(pU);
    double* M = static_cast<double*>(pM);
    int* infos = reinterpret_cast<int*>(static_cast<double*>(pCore) + core_inverse_ws_doubles(r, b));
    if (sparse)
      ICUR_TRY(csr_gather_cross(*src.csr, static_cast<const int64_t*>(pIall), r, static_cast<const int64_t*>(pJall), r,
                                M, r, st));
    else
      ICUR_TRY(launch_gather_f64(A, lda, static_cast<const int64_t*>(pIall), r, static_cast<const int64_t*>(pJall), r,
                                 false, M, r, st));
    // with more than one block the cross is kept for the refinement of the block-LU
    // inverse (one block is the pivot block's in-order inverse: LU with partial pivoting)
    double* M0 = nullptr;
    if (nb > 1) {
      void* pRef;
      ICUR_TRY(ensure(dc, kCoreRef, (static_cast<size_t>(r) * r + core_refine_ws_doubles(r)) * 8, &pRef));
      M0 = static_cast<double*>(pRef);
      ICUR_TRY(dcopy2d(r, r, 1.0, M, r, M0, r, st));
    }
    ICUR_TRY(core_block_inverse(M, r, blocks.data(), nb, b, U, static_cast<double*>(pCore), infos, nullptr, st, N1inv));
    if (M0) ICUR_TRY(core_refine(M0, U, r, 1e-2 * tol, M0 + static_cast<size_t>(r) * r, st));
    ICUR_TRY(tm.mark(&ec1));
    // the pivot-block flags and the results: through the pinned staging area in one
    // synchronisation when they fit, else the flags first and the results directly
    const size_t info_bytes = (static_cast<size_t>(nb) * sizeof(int) + 7) & ~size_t(7);
    const size_t ij_bytes = static_cast<size_t>(r) * 8;
    const size_t u_bytes = static_cast<size_t>(r) * r * 8;
    char* stage = static_cast<char*>(dc.host_pinned) + kStageOffset;
    const bool dev_out = o.device_outputs != 0;
    const size_t out_bytes = dev_out ? 0 : 2 * ij_bytes + u_bytes;
    const bool staged = info_bytes + out_bytes <= kStageBytes;
    std::vector<int> hinfo(nb);
    if (staged) {
      HostSegs h{};
      const int64_t so = static_cast<int64_t>(kStageOffset);
      h.seg[0] = HostSeg{infos, static_cast<int64_t>(nb * sizeof(int)), so};
      h.n = 1;
      if (!dev_out) {
        h.seg[1] = HostSeg{pIall, static_cast<int64_t>(ij_bytes), so + static_cast<int64_t>(info_bytes)};
        h.seg[2] = HostSeg{pJall, static_cast<int64_t>(ij_bytes), so + static_cast<int64_t>(info_bytes + ij_bytes)};
        h.seg[3] = HostSeg{U, static_cast<int64_t>(u_bytes), so + static_cast<int64_t>(info_bytes + 2 * ij_bytes)};
        h.n = 4;
      }
      ICUR_TRY(read_back(dc, h, st, false));
      std::memcpy(hinfo.data(), stage, nb * sizeof(int));
    } else {
      ICUR_HIP(hipMemcpyAsync(hinfo.data(), infos, nb * sizeof(int), hipMemcpyDeviceToHost, st));
      ICUR_HIP(hipStreamSynchronize(st));
    }
    for (int v : hinfo)
      if (v != 0) {
        set_error("core assembly: a pivot block of A(I,J) is exactly singular");
        return ICUR_ERR_HIP;
      }
    tm.add(ec0, ec1, &t_info.ms_core);
    if (dev_out) {
      ICUR_HIP(hipMemcpyAsync(I_out, pIall, r * 8, hipMemcpyDeviceToDevice, st));
      ICUR_HIP(hipMemcpyAsync(J_out, pJall, r * 8, hipMemcpyDeviceToDevice, st));
      ICUR_HIP(hipMemcpyAsync(U_out, U, r * r * 8, hipMemcpyDeviceToDevice, st));
    } else if (staged) {
      std::memcpy(I_out, stage + info_bytes, ij_bytes);
      std::memcpy(J_out, stage + info_bytes + ij_bytes, ij_bytes);
      std::memcpy(U_out, stage + info_bytes + 2 * ij_bytes, u_bytes);
    } else {
      ICUR_HIP(hipMemcpyAsync(I_out, pIall, r * 8, hipMemcpyDeviceToHost, st));
      ICUR_HIP(hipMemcpyAsync(J_out, pJall, r * 8, hipMemcpyDeviceToHost, st));
      ICUR_HIP(hipMemcpyAsync(U_out, U, r * r * 8, hipMemcpyDeviceToHost, st));
    }
  }
  ICUR_HIP(hipStreamSynchronize(st));
  tm.flush();
  *rank_out = r;
  *est_out = rho;
  t_info.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  return status;
}

}  // namespace
}  // namespace icur

using namespace icur;

// =========================================================================== C-ABI
extern "C" {

int icur_run(const float* A, int64_t m, int64_t n, int64_t lda, double tol, int32_t block,
             int32_t sketch_kind, uint64_t seed, const icur_opts* opts, int64_t* I, int64_t* J,
             double* U, int64_t* rank, double* est_err) {
  const auto t0 = std::chrono::steady_clock::now();
  t_error.clear();
  std::memset(&t_info, 0, sizeof(t_info));
  Source src;
  src.A = A;
  src.lda = lda;
  return run_impl(src, m, n, tol, block, sketch_kind, seed, opts, I, J, U, rank, est_err, t0);
}

int icur_run_csr(const int64_t* rowptr, const int32_t* colind, const float* vals, int64_t m, int64_t n,
                 int64_t nnz, double tol, int32_t block, int32_t sketch_kind, uint64_t seed,
                 const icur_opts* opts, int64_t* I, int64_t* J, double* U, int64_t* rank, double* est_err) {
  const auto t0 = std::chrono::steady_clock::now();
  t_error.clear();
  std::memset(&t_info, 0, sizeof(t_info));
  if (!rowptr || (nnz > 0 && (!colind || !vals))) return arg_error("null CSR array");
  if (nnz < 0 || nnz > 0x7fffffffLL) return arg_error("need 0 <= nnz < 2^31");
  CsrMatrix csr{rowptr, colind, vals, m, n, nnz};
  Source src;
  src.csr = &csr;
  return run_impl(src, m, n, tol, block, sketch_kind, seed, opts, I, J, U, rank, est_err, t0);
}

int icur_run_batched(int32_t count, const float* const* A, const int64_t* m, const int64_t* n,
                     const int64_t* lda, const double* tol, int32_t block, int32_t sketch_kind,
                     const uint64_t* seed, const icur_opts* opts, int64_t* I_pool, int64_t* J_pool,
                     double* U_pool, const int64_t* cap_offsets, int64_t* rank, double* est_err,
                     int32_t* status) {
  const auto t0 = std::chrono::steady_clock::now();
  t_error.clear();
  std::memset(&t_info, 0, sizeof(t_info));
  if (count < 0) return arg_error("count must be >= 0");
  if (count == 0) return ICUR_OK;
  if (!A || !m || !n || !lda || !tol || !seed || !cap_offsets || !I_pool || !J_pool || !U_pool || !rank ||
      !est_err || !status)
    return arg_error("null array argument");
  // ---- every argument of every matrix, before any device work
  icur_opts o;
  std::vector<int64_t> uoff(static_cast<size_t>(count) + 1, 0);
  if (cap_offsets[0] != 0) return arg_error("cap_offsets[0] must be 0");
  for (int32_t i = 0; i < count; ++i) {
    const int e = check_run_args(false, A[i], m[i], n[i], lda[i], tol[i], block, sketch_kind, opts, &o);
    if (e != ICUR_OK) {
      set_error("matrix " + std::to_string(i) + ": " + t_error);
      return e;
    }
    const int64_t cap = cap_offsets[i + 1] - cap_offsets[i];
    const int64_t rmax = (o.max_rank == 0) ? std::min(m[i], n[i]) : std::min(o.max_rank, std::min(m[i], n[i]));
    if (cap < rmax)
      return arg_error("matrix " + std::to_string(i) + ": capacity " + std::to_string(cap) + " below its rank bound " +
                       std::to_string(rmax));
    uoff[i + 1] = uoff[i] + cap * cap;
  }
  DeviceInfo dev;
  ICUR_TRY(device_info(&dev));
  const hipStream_t caller = as_stream(o.stream);

  // ---- workers: batch_workers concurrent runs, each on its own slot and stream.  The
  // selection grids of concurrent runs share the CUs, so each is capped at its share;
  // a matrix too large for the share runs afterwards, alone.
  // on the uneven batch: 8 about 25% faster than 4, 16 about 6% faster than 8, 24 and 32
  // no faster than 16
  // ---- grouped form (default): every matrix that fits one selection workgroup and uses
  // FP64 residual factors advances together with the others, one launch per step
  std::vector<std::string> errs(static_cast<size_t>(count), "not run: no worker thread could select the device");
  std::vector<int> grouped, rest;
  BatchedCall gstat{};  // the grouped form's statistics, reported in icur_last_info
  const bool group_ok = o.batch_workers == 0 && block <= kGMaxSteps && o.residual_fp64 >= 0 &&
                        o.selection == ICUR_SELECT_LUPP;
  for (int32_t i = 0; i < count; ++i)
    (group_ok && std::max(m[i], n[i]) <= kGMaxN ? grouped : rest).push_back(i);
  int64_t total_iters = 0;
  if (!grouped.empty()) {
    int st_risk = ICUR_OK;
    BatchedCall bc{};
    bc.count = count;
    bc.A = A;
    bc.m = m;
    bc.n = n;
    bc.lda = lda;
    bc.tol = tol;
    bc.block = block;
    bc.kind = sketch_kind;
    bc.seed = seed;
    bc.opts = &o;
    bc.xi = risk_factor(o.alpha, o.delta, (11 * static_cast<int64_t>(block)) / 10, &st_risk);
    bc.row_cut = kRowCutFp64;
    bc.I_pool = I_pool;
    bc.J_pool = J_pool;
    bc.U_pool = U_pool;
    bc.cap_offsets = cap_offsets;
    bc.uoff = uoff.data();
    bc.rank = rank;
    bc.est = est_err;
    bc.status = status;
    bc.errs = errs.data();
    for (int i : grouped) status[i] = ICUR_ERR_HIP;
    const int gst = run_batched_grouped(grouped, bc, caller);
    if (gst < 0) {
      for (int i : grouped) {
        status[i] = gst;
        errs[i] = t_error;
      }
    }
    total_iters += bc.iterations;
    gstat = bc;
  }

  constexpr int kBatchWorkers = 16;
  const int S = std::max(1, std::min<int32_t>(static_cast<int32_t>(rest.size()),
                                              o.batch_workers > 0 ? o.batch_workers : kBatchWorkers));
  const int gcap = std::max(1, dev.num_cus / S);
  std::vector<int> small, large;
  for (int i : rest) (std::max(m[i], n[i]) <= lupp_max_candidates(gcap) ? small : large).push_back(i);
  auto by_size = [&](int x, int y) { return m[x] * n[x] > m[y] * n[y] || (m[x] * n[x] == m[y] * n[y] && x < y); };
  std::sort(small.begin(), small.end(), by_size);
  std::sort(large.begin(), large.end(), by_size);
  std::vector<hipStream_t> streams(S);
  for (int s = 0; s < S; ++s) {
    DeviceCache* dcp;
    ICUR_TRY(prepare_device(&dcp, 1 + s));
    std::lock_guard<std::mutex> lock(dcp->mu);
    if (!dcp->stream) ICUR_HIP(hipStreamCreateWithFlags(&dcp->stream, hipStreamNonBlocking));
    streams[s] = dcp->stream;
  }
  hipEvent_t ready;
  ICUR_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  ICUR_HIP(hipEventRecord(ready, caller));
  for (int s = 0; s < S; ++s) ICUR_HIP(hipStreamWaitEvent(streams[s], ready, 0));

  // a matrix stays marked as not run unless a worker reaches it
  for (int i : rest) status[i] = ICUR_ERR_HIP;
  std::mutex iters_mu;
  auto run_one = [&](int i, int s, int groups) {
    icur_opts oo = o;
    oo.stream = streams[s];
    t_error.clear();
    std::memset(&t_info, 0, sizeof(t_info));
    Source src;
    src.A = A[i];
    src.lda = lda[i];
    const int st = run_impl(src, m[i], n[i], tol[i], block, sketch_kind, seed[i], &oo, I_pool + cap_offsets[i],
                            J_pool + cap_offsets[i], U_pool + uoff[i], rank + i, est_err + i,
                            std::chrono::steady_clock::now(), 1 + s, groups, false);
    status[i] = st;
    if (st < 0) {
      errs[i] = t_error;
      rank[i] = 0;
      est_err[i] = 0.0;
    }
    std::lock_guard<std::mutex> g(iters_mu);
    total_iters += t_info.iterations;
  };
  std::atomic<size_t> next{0};
  auto worker = [&](int s) {
    if (hipSetDevice(dev.device) != hipSuccess) return;
    for (;;) {
      const size_t q = next.fetch_add(1);
      if (q >= small.size()) break;
      run_one(small[q], s, gcap);
    }
  };
  std::vector<std::thread> pool;
  try {
    for (int s = 1; s < S; ++s) pool.emplace_back(worker, s);
  } catch (...) {
    // fewer threads than asked for: the ones started and this thread share the queue
  }
  worker(0);  // the calling thread is worker 0 (its device is already current)
  for (auto& th : pool) th.join();
  for (int i : large) run_one(i, 0, 0);
  (void)hipEventDestroy(ready);
  int first_err = ICUR_OK;
  std::string msg;
  for (int32_t i = 0; i < count; ++i) {
    if (status[i] < 0 && first_err == ICUR_OK) {
      first_err = status[i];
      msg = "matrix " + std::to_string(i) + ": " + errs[i];
    }
  }
  std::memset(&t_info, 0, sizeof(t_info));
  t_info.ms_sketch = gstat.ms_sketch;
  t_info.ms_select = gstat.ms_select;
  t_info.ms_products = gstat.ms_products;
  t_info.product_bytes = gstat.product_bytes;
  t_info.product_launches = gstat.product_launches;
  t_info.group_iterations = gstat.iterations;
  t_info.ms_residual = gstat.ms_loop;
  t_info.ms_core = gstat.ms_final;
  t_info.ms_setup = gstat.ms_alloc;
  t_info.ms_results = gstat.ms_results;
  t_info.sketch_kernel = gstat.sketch_kernel;
  t_info.graph_iterations = gstat.graph_iterations;
  for (int q = 0; q < 5; ++q) t_info.ms_stage[q] = gstat.ms_stage[q];
  for (int q = 0; q < 5; ++q) t_info.stage_bytes[q] = gstat.stage_bytes[q];
  for (int q = 0; q < 4; ++q) t_info.tiles[q] = gstat.tiles[q];
  t_info.iterations = static_cast<int32_t>(std::min<int64_t>(total_iters, INT32_MAX));
  t_info.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (first_err != ICUR_OK) {
    set_error(msg);
    return first_err;
  }
  t_error.clear();
  return ICUR_OK;
}

int icur_last_info(icur_info* info) {
  if (!info) return ICUR_ERR_ARG;
  *info = t_info;
  return ICUR_OK;
}

const char* icur_last_error(void) { return last_error(); }

int icur_release(void) {
  std::lock_guard<std::mutex> g(g_cache_mu);
  int dev0 = 0;
  ICUR_HIP(hipGetDevice(&dev0));
  for (auto& kv : g_cache) {
    DeviceCache& dc = *kv.second;
    std::lock_guard<std::mutex> l(dc.mu);
    ICUR_HIP(hipSetDevice(dc.device));
    if (dc.stream) ICUR_HIP(hipStreamDestroy(dc.stream));
    dc.stream = nullptr;
    for (auto& b : dc.buf) {
      if (b.p) ICUR_HIP(hipFree(b.p));
      b.p = nullptr;
      b.bytes = 0;
    }
    if (dc.host_pinned) ICUR_HIP(hipHostFree(dc.host_pinned));
    dc.host_pinned = nullptr;
    dc.host_pinned_dev = nullptr;
    for (auto e : dc.events) (void)hipEventDestroy(e);
    dc.events.clear();
    if (dc.sync_event) (void)hipEventDestroy(dc.sync_event);
    dc.sync_event = nullptr;
  }
  g_cache.clear();
  release_blas_handles();
  release_batch_arenas();
  ICUR_HIP(hipSetDevice(dev0));
  return ICUR_OK;
}

int icur_make_sketch(uint64_t seed, int64_t c, int64_t m, int32_t sketch_kind, int32_t zeta,
                     uint16_t* G_bf16, uint8_t* rows, uint8_t* signs, void* stream) {
  t_error.clear();
  if (c < 1 || m < 1) return arg_error("need c >= 1 and m >= 1");
  hipStream_t st = as_stream(stream);
  if (sketch_kind == ICUR_SKETCH_GAUSSIAN) {
    if (!G_bf16) return arg_error("Gaussian sketch needs G_bf16");
    ICUR_TRY(launch_gaussian_G(seed, c, m, G_bf16, m, st));
  } else if (sketch_kind == ICUR_SKETCH_SPARSE_SIGN) {
    if (!G_bf16 && !rows && !signs) return arg_error("no output given");
    if (zeta < 0 || zeta > 8) return arg_error("zeta must be in 0..8");
    ICUR_TRY(launch_sparse_sign(seed, c, m, zeta > 0 ? zeta : 8, rows, signs, G_bf16, m, st));
  } else if (sketch_kind == ICUR_SKETCH_SRTT) {
    return arg_error("the SRTT operator is not BF16-valued: use icur_make_srtt");
  } else {
    return arg_error("unknown sketch kind");
  }
  ICUR_HIP(hipStreamSynchronize(st));
  return ICUR_OK;
}

int icur_make_srtt(uint64_t seed, int64_t c, int64_t m, float* G, int64_t* rows, void* stream) {
  t_error.clear();
  if (c < 1 || m < 1 || c > m) return arg_error("need 1 <= c <= m");
  if (!rows) return arg_error("rows is null");
  hipStream_t st = as_stream(stream);
  void* mark = nullptr;
  if (hipMalloc(&mark, static_cast<size_t>(m)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation failed");
    return ICUR_ERR_NOMEM;
  }
  const int e = launch_srtt(seed, c, m, G, m, rows, static_cast<uint8_t*>(mark), st);
  const hipError_t se = hipStreamSynchronize(st);
  (void)hipFree(mark);
  if (e != ICUR_OK) return e;
  ICUR_HIP(se);
  return ICUR_OK;
}

int icur_sketch(const uint16_t* G_bf16, int64_t c, const float* A, int64_t m, int64_t n,
                int64_t lda, int32_t terms, float* X0, double* normsq, void* stream) {
  t_error.clear();
  if (!G_bf16 || !A || !X0) return arg_error("null pointer");
  if (c < 1 || m < 1 || n < 1 || lda < n) return arg_error("invalid shape");
  if (c > 4096) return arg_error("c above 4096 is not supported");
  if (terms < 0 || terms > 3) return arg_error("terms must be 0..3");
  DeviceCache* dcp;
  ICUR_TRY(prepare_device(&dcp));
  DeviceCache& dc = *dcp;
  std::lock_guard<std::mutex> lock(dc.mu);
  DeviceInfo dev;
  ICUR_TRY(device_info(&dev));
  hipStream_t st = as_stream(stream);
  void *pGemm, *pNorm, *pScal, *p64;
  ICUR_TRY(ensure(dc, kGemmWs,
                  std::max(wide_gemm_workspace_bytes(c, m, n, dev.num_cus), sketch_workspace_bytes(c, m, n, dev.num_cus)),
                  &pGemm));
  ICUR_TRY(ensure(dc, kNormPart,
                  static_cast<size_t>(std::max(max_norm_partials(c, n), sketch_max_norm_partials(c, n))) * 8, &pNorm));
  ICUR_TRY(ensure(dc, kScal, sizeof(Scal), &pScal));
  int parts = 0;
  // the sketch kernel (FP64 result, then FP32 and its norm), as in icur_run; other
  // shapes and terms 0 take the general product
  int sk = ICUR_ERR_UNSUPPORTED;
  if (terms > 0) {
    ICUR_TRY(ensure(dc, kStepA, static_cast<size_t>(c) * n * 8, &p64));
    sk = sketch_product(G_bf16, m, c, A, m, n, lda, terms, false, static_cast<double*>(p64), n, nullptr, nullptr,
                        pGemm, dc.buf[kGemmWs].bytes, st, nullptr, nullptr);
    if (sk != ICUR_OK && sk != ICUR_ERR_UNSUPPORTED) return sk;
    if (sk == ICUR_OK)
      ICUR_TRY(convert_f64_f32_norm(static_cast<const double*>(p64), c, n, X0, n, static_cast<double*>(pNorm), &parts,
                                    st));
  }
  WideGemm g{};
  g.W = G_bf16;
  g.ldw = m;
  g.wterms = terms == 0 ? 0 : 1;
  g.w_bf16 = true;
  g.B = A;
  g.ldb = lda;
  g.bterms = terms;
  g.M = c;
  g.K = m;
  g.N = n;
  g.subtract = false;
  g.out64 = false;
  g.OUT = X0;
  g.ldo = n;
  g.norm_partials = static_cast<double*>(pNorm);
  g.nparts = &parts;
  if (sk == ICUR_ERR_UNSUPPORTED) ICUR_TRY(wide_gemm(g, pGemm, dc.buf[kGemmWs].bytes, st));
  Scal* ds = static_cast<Scal*>(pScal);
  ICUR_TRY(launch_reduce_partials(static_cast<double*>(pNorm), parts, &ds->normsq_x0, st));
  Scal hs;
  ICUR_TRY(read_scal(dc, ds, &hs, st));
  if (normsq) *normsq = hs.normsq_x0;
  return ICUR_OK;
}

int icur_lupp(const float* X, int64_t K, int64_t N, int64_t ldx, int32_t steps,
              const uint8_t* excluded, int64_t* piv, int32_t* npiv, void* stream) {
  t_error.clear();
  if (!X || !piv || !npiv) return arg_error("null pointer");
  if (K < 1 || N < 1 || ldx < N) return arg_error("invalid shape");
  if (steps < 1 || steps > K) return arg_error("need 1 <= steps <= K");
  if (K > 4096) return arg_error("K above 4096 is not supported");
  if (N > 0x7fffffffLL) return arg_error("N must be below 2^31");
  DeviceCache* dcp;
  ICUR_TRY(prepare_device(&dcp));
  DeviceCache& dc = *dcp;
  std::lock_guard<std::mutex> lock(dc.mu);
  hipStream_t st = as_stream(stream);
  void* pL;
  ICUR_TRY(ensure(dc, kStepA, lupp_workspace_bytes(steps, N), &pL));
  LuppWork lw;
  lupp_bind_workspace(pL, steps, N, &lw);
  ICUR_TRY(lupp_launch(X, false, K, N, ldx, steps, excluded, piv, lw, st));
  int lst[2];
  ICUR_TRY(read_int(dc, lw.status, lst, 2, st));
  if (lst[1]) {
    set_error("selection kernel: grid barrier did not complete");
    return ICUR_ERR_HIP;
  }
  *npiv = lst[0];
  return ICUR_OK;
}

int icur_qrcp(const float* X, int64_t K, int64_t N, int64_t ldx, int32_t steps, const uint8_t* excluded, int64_t* piv,
              int32_t* npiv, void* stream) {
  t_error.clear();
  if (!X || !piv || !npiv) return arg_error("null pointer");
  if (K < 1 || N < 1 || ldx < N) return arg_error("invalid shape");
  if (steps < 1 || steps > K) return arg_error("need 1 <= steps <= K");
  if (K > 4096) return arg_error("K above 4096 is not supported");
  if (N > 0x7fffffffLL) return arg_error("N must be below 2^31");
  DeviceCache* dcp;
  ICUR_TRY(prepare_device(&dcp));
  DeviceCache& dc = *dcp;
  std::lock_guard<std::mutex> lock(dc.mu);
  DeviceInfo dev;
  ICUR_TRY(device_info(&dev));
  hipStream_t st = as_stream(stream);
  void *pQ, *pS;
  ICUR_TRY(ensure(dc, kQrcp, qrcp_workspace_bytes(K, N, 4 * dev.num_cus), &pQ));
  ICUR_TRY(ensure(dc, kScal, 256, &pS));
  int* status = static_cast<int*>(pS);
  ICUR_TRY(qrcp_launch(X, false, K, N, ldx, steps, excluded, piv, status, pQ, dc.buf[kQrcp].bytes, st));
  int lst[1];
  ICUR_TRY(read_int(dc, status, lst, 1, st));
  *npiv = lst[0];
  return ICUR_OK;
}

int icur_residual(const float* X, int64_t ldx, const double* W, int64_t ldw, const float* B,
                  int64_t ldb, int64_t M, int64_t K, int64_t N, int32_t terms, float* OUT,
                  int64_t ldo, double* normsq, void* stream) {
  t_error.clear();
  if (!OUT || (K > 0 && (!W || !B))) return arg_error("null pointer");
  if (M < 1 || N < 1 || K < 0) return arg_error("invalid shape");
  if (M > 4096) return arg_error("M above 4096 is not supported");
  if (ldo < N || (X && ldx < N) || (K > 0 && (ldw < K || ldb < N))) return arg_error("invalid leading dimension");
  if (terms < 0 || terms > 3) return arg_error("terms must be 0..3");
  DeviceCache* dcp;
  ICUR_TRY(prepare_device(&dcp));
  DeviceCache& dc = *dcp;
  std::lock_guard<std::mutex> lock(dc.mu);
  DeviceInfo dev;
  ICUR_TRY(device_info(&dev));
  hipStream_t st = as_stream(stream);
  void *pWp, *pGemm, *pNorm, *pScal;
  const size_t wbytes = static_cast<size_t>(M) * std::max<int64_t>(K, 1) * (terms == 0 ? 4 : 2 * terms);
  ICUR_TRY(ensure(dc, kStepB, wbytes, &pWp));
  ICUR_TRY(ensure(dc, kGemmWs, wide_gemm_workspace_bytes(M, K, N, dev.num_cus), &pGemm));
  ICUR_TRY(ensure(dc, kNormPart, static_cast<size_t>(max_norm_partials(M, N)) * 8, &pNorm));
  ICUR_TRY(ensure(dc, kScal, sizeof(Scal), &pScal));
  if (K > 0) ICUR_TRY(launch_split_f64(W, M, K, ldw, false, terms, pWp, K, M * K, st));
  WideGemm g{};
  g.X = X;
  g.ldx = ldx;
  g.W = pWp;
  g.ldw = K;
  g.wterms = terms;
  g.B = B;
  g.ldb = ldb;
  g.bterms = terms;
  g.M = M;
  g.K = K;
  g.N = N;
  g.subtract = true;
  g.out64 = false;
  g.OUT = OUT;
  g.ldo = ldo;
  g.norm_partials = static_cast<double*>(pNorm);
  int parts = 0;
  g.nparts = &parts;
  ICUR_TRY(wide_gemm(g, pGemm, dc.buf[kGemmWs].bytes, st));
  Scal* ds = static_cast<Scal*>(pScal);
  ICUR_TRY(launch_reduce_partials(static_cast<double*>(pNorm), parts, &ds->normsq_s, st));
  Scal hs;
  ICUR_TRY(read_scal(dc, ds, &hs, st));
  if (normsq) *normsq = hs.normsq_s;
  return ICUR_OK;
}

int icur_residual_f64(const double* X, int64_t ldx, const double* W, int64_t ldw, const double* B, int64_t ldb,
                      int64_t M, int64_t K, int64_t N, double* OUT, int64_t ldo, double* normsq, void* stream) {
  t_error.clear();
  if (!OUT || (K > 0 && (!W || !B))) return arg_error("null pointer");
  if (M < 1 || N < 1 || K < 0) return arg_error("invalid shape");
  if (M > 4096) return arg_error("M above 4096 is not supported");
  if (ldo < N || (X && ldx < N) || (K > 0 && (ldw < K || ldb < N))) return arg_error("invalid leading dimension");
  DeviceCache* dcp;
  ICUR_TRY(prepare_device(&dcp));
  DeviceCache& dc = *dcp;
  std::lock_guard<std::mutex> lock(dc.mu);
  DeviceInfo dev;
  ICUR_TRY(device_info(&dev));
  hipStream_t st = as_stream(stream);
  void *pGemm, *pNorm, *pScal;
  ICUR_TRY(ensure(dc, kGemmWs, wide_gemm_workspace_bytes(M, K, N, dev.num_cus), &pGemm));
  ICUR_TRY(ensure(dc, kNormPart, static_cast<size_t>(std::max(max_norm_partials(M, N), 1024)) * 8, &pNorm));
  ICUR_TRY(ensure(dc, kScal, sizeof(Scal), &pScal));
  int parts = 0;
  // X == OUT or X null with K > 0 take the library route when the shape qualifies; a
  // separate X is subtracted by the short-M kernel
  const bool plain = (X == nullptr);
  ICUR_TRY(product_f64(W, ldw, M, K, X, ldx, B, ldb, N, !plain, OUT, ldo, static_cast<double*>(pNorm), &parts, pGemm,
                       dc.buf[kGemmWs].bytes, st));
  Scal* ds = static_cast<Scal*>(pScal);
  ICUR_TRY(launch_reduce_partials(static_cast<double*>(pNorm), parts, &ds->normsq_s, st));
  Scal hs;
  ICUR_TRY(read_scal(dc, ds, &hs, st));
  if (normsq) *normsq = hs.normsq_s;
  return ICUR_OK;
}

int icur_gather(const float* A, int64_t m, int64_t n, int64_t lda, const int64_t* cols,
                const int64_t* rows, int64_t k, float* Ct, int64_t ldct, float* Rout, int64_t ldr,
                void* stream) {
  t_error.clear();
  if (!A || m < 1 || n < 1 || lda < n || k < 0) return arg_error("invalid matrix");
  const bool c_given = cols && Ct, r_given = rows && Rout;
  if (c_given == r_given) return arg_error("give exactly one of (cols, Ct) and (rows, Rout)");
  hipStream_t st = as_stream(stream);
  if (c_given) {
    if (ldct < m) return arg_error("ldct < m");
    ICUR_TRY(launch_gather_cols_T(A, m, n, lda, cols, k, Ct, ldct, st));
  } else {
    if (ldr < n) return arg_error("ldr < n");
    ICUR_TRY(launch_gather_rows(A, m, n, lda, rows, k, Rout, ldr, st));
  }
  ICUR_HIP(hipStreamSynchronize(st));
  return ICUR_OK;
}

int icur_core_update(double* U, int64_t ldu, int64_t r, int64_t k, const double* Y,
                     const double* A21, const double* A22, double* rcond, void* stream) {
  t_error.clear();
  if (!U || !A22 || (r > 0 && (!Y || !A21))) return arg_error("null pointer");
  if (r < 0 || k < 1 || k > 512 || ldu < r + k) return arg_error("invalid shape");
  DeviceCache* dcp;
  ICUR_TRY(prepare_device(&dcp));
  DeviceCache& dc = *dcp;
  std::lock_guard<std::mutex> lock(dc.mu);
  hipStream_t st = as_stream(stream);
  void *pCore, *pScal;
  ICUR_TRY(ensure(dc, kStepA, core_update_ws_doubles(r, k) * 8, &pCore));
  ICUR_TRY(ensure(dc, kScal, sizeof(Scal), &pScal));
  Scal* ds = static_cast<Scal*>(pScal);
  ICUR_TRY(core_update(U, ldu, r, k, Y, k, A21, A22, static_cast<double*>(pCore), &ds->info, ds->norms, st));
  Scal hs;
  ICUR_TRY(read_scal(dc, ds, &hs, st));
  if (hs.info != 0) return arg_error("the Schur complement block is exactly singular");
  if (rcond) *rcond = (hs.norms[0] > 0 && hs.norms[1] > 0) ? 1.0 / (hs.norms[0] * hs.norms[1]) : 0.0;
  return ICUR_OK;
}

}  // extern "C"
