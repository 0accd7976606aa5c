// Host driver of the grouped batched form: many dense matrices of uneven sizes and
// tolerances advanced together through Alg. 1, one launch per step for all of them.
//
//   1. sketch: G and X0 = G A for every matrix (the single-matrix sketch kernels, spread
//      over a few streams), then one read-back of all ||G A||_F^2;
//   2. loop: one iteration of every unfinished matrix (launch_batch_iteration: the two
//      grouped selections, grouped gathers and FP64 products, the pivot-block inverses,
//      the bordered core and the stopping decision), then one read-back of a small record
//      per matrix (rank, state), from which the host only grows rank-sized buffers;
//   3. results: a matrix that stops has its core multiplied out at the end of that
//      iteration (one launch for all that stopped), and a copy thread moves its I, J
//      and core to the caller's pools while the others go on.
// The rank-sized buffers come from one device arena: at the full rank bound when that
// fits in free memory, else at a fraction of it, grown (first fit, stream ordered) when
// a matrix needs more.
// Each matrix follows Alg. 1 on its own: the grouping changes no arithmetic.
#include <dlfcn.h>

#include <algorithm>
#include <cstdio>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "icur_batched.h"

namespace icur {

int launch_batch_iteration(BatchMat* mats, int count, int c, int b, double row_cut, void* plan_ws, BatchRec* rec,
                           const GemmTiles& tiles, int grid, hipStream_t st, hipEvent_t* ev);
int launch_batch_final(BatchMat* mats, int count, int c, int b, void* plan_ws, const GemmTiles& tiles,
                       hipStream_t st);
size_t batch_plan_bytes(int count);
double* batch_plan_bytes_ptr(void* plan_ws, int count);
int batch_plan_stages();
int batch_plan_final_stage();
std::vector<int> batch_plan_product_stages();

namespace {

size_t al(size_t b) { return (b + 255) & ~size_t(255); }

// Rank-sized part of a matrix's state for capacity cap.
size_t rank_bytes(int64_t cap, int64_t m, int64_t n, int64_t b) {
  return al(cap * m * 8) + al(cap * n * 8) + 2 * al(cap * cap * 8) + 3 * al(b * cap * 8) + 2 * al(cap * 8);
}

void bind_rank(BatchMat& bm, char* p, int64_t cap, int64_t b) {
  const int64_t m = bm.m, n = bm.n;
  bm.LcT = reinterpret_cast<double*>(p);
  p += al(cap * m * 8);
  bm.Ur = reinterpret_cast<double*>(p);
  p += al(cap * n * 8);
  bm.QT = reinterpret_cast<double*>(p);
  p += al(cap * cap * 8);
  bm.Pi = reinterpret_cast<double*>(p);
  p += al(cap * cap * 8);
  double** three[3] = {&bm.Wa, &bm.Wl, &bm.Wp};
  for (double** q : three) {
    *q = reinterpret_cast<double*>(p);
    p += al(b * cap * 8);
  }
  bm.Jall = reinterpret_cast<int64_t*>(p);
  p += al(cap * 8);
  bm.Iall = reinterpret_cast<int64_t*>(p);
  bm.cap = static_cast<int>(cap);
}


struct DevBuf {
  void* p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  int alloc(size_t bytes) {
    if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      set_error("device allocation of " + std::to_string(bytes) + " bytes failed (batched)");
      return ICUR_ERR_NOMEM;
    }
    return ICUR_OK;
  }
};

// First-fit allocator over one device arena (offsets in 256-byte units of the arena).
// Regions are released in stream order: every use of a region is enqueued on the one
// stream of the loop, so a later allocation of the same bytes is used after them.
class Arena {
 public:
  char* base = nullptr;
  size_t size = 0;
  void reset(void* p, size_t bytes) {
    base = static_cast<char*>(p);
    size = bytes & ~size_t(255);
    free_.clear();
    if (size) free_[0] = size;
  }
  char* take(size_t bytes) {
    bytes = al(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > bytes) free_[off + bytes] = len - bytes;
      return base + off;
    }
    return nullptr;
  }
  void give(char* p, size_t bytes) {
    size_t off = static_cast<size_t>(p - base);
    bytes = al(bytes);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  bool owns(const char* p) const { return p >= base && p < base + size; }

 private:
  std::map<size_t, size_t> free_;
};

// The arena of the last grouped call on each device, kept for the next one (allocating
// and clearing a few hundred GB of device memory costs seconds); released by icur_release.
// A call takes it out for its duration, so concurrent calls never share one.
struct CachedArena {
  void* p = nullptr;
  size_t bytes = 0;
};
std::mutex g_arena_mu;
std::map<int, CachedArena> g_arenas;

CachedArena take_arena(int device) {
  std::lock_guard<std::mutex> g(g_arena_mu);
  CachedArena a = g_arenas[device];
  g_arenas[device] = CachedArena();
  return a;
}

void put_arena(int device, CachedArena a) {
  if (!a.p) return;
  std::lock_guard<std::mutex> g(g_arena_mu);
  CachedArena& slot = g_arenas[device];
  if (slot.p && slot.bytes >= a.bytes) {
    (void)hipFree(a.p);
    return;
  }
  if (slot.p) (void)hipFree(slot.p);
  slot = a;
}

// Owns a call's arena; gives it back to the cache at the end of the call.
struct ArenaHold {
  int device = 0;
  CachedArena a;
  ~ArenaHold() { put_arena(device, a); }
};

// A host thread that copies finished matrices' results to the caller's pools (pageable host
// memory, or device memory with device_outputs) on a stream of its own while the loop goes
// on.
class ResultCopier {
 public:
  struct Job {
    void* dst[3];
    const void* src[3];
    size_t bytes[3];
  };
  ResultCopier(int device, hipMemcpyKind kind) : kind_(kind), th_([this, device] { run(device); }) {}
  ~ResultCopier() { finish(); }
  void push(const Job& j) {
    {
      std::lock_guard<std::mutex> g(mu_);
      q_.push_back(j);
    }
    cv_.notify_one();
  }
  // Waits for every queued copy; returns the first failure's message ("" when none).
  std::string finish() {
    {
      std::lock_guard<std::mutex> g(mu_);
      done_ = true;
    }
    cv_.notify_one();
    if (th_.joinable()) th_.join();
    return err_;
  }

 private:
  void run(int device) {
    hipStream_t cs = nullptr;
    if (hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
      err_ = "copy thread: no stream";
      cs = nullptr;
    }
    for (;;) {
      Job j;
      {
        std::unique_lock<std::mutex> g(mu_);
        cv_.wait(g, [this] { return done_ || !q_.empty(); });
        if (q_.empty()) break;
        j = q_.front();
        q_.pop_front();
      }
      if (!cs || !err_.empty()) continue;
      hipError_t e = hipSuccess;
      for (int k = 0; k < 3 && e == hipSuccess; ++k)
        if (j.bytes[k]) e = hipMemcpyAsync(j.dst[k], j.src[k], j.bytes[k], kind_, cs);
      if (e == hipSuccess) e = hipStreamSynchronize(cs);
      if (e != hipSuccess) err_ = std::string("copy of the results: ") + hipGetErrorString(e);
    }
    if (cs) (void)hipStreamDestroy(cs);
  }
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Job> q_;
  bool done_ = false;
  std::string err_;
  const hipMemcpyKind kind_;
  std::thread th_;
};

}  // namespace

// ---- tile shapes of the grouped products
// Defaults: row tiles that hold a block (P1 - P3), 32 x 128 with two chunks in flight for
// the core products.  A tune
// file written by the package's autotuner (measured per stage on the device) overrides
// them for the block sizes it lists; ICUR_BATCH_TILES="p1,p2,p3,fin" overrides both (the
// autotuner's own runs use it).  The file is ICUR_TUNE_FILE, else tune_gfx950.json beside
// the library.
namespace {

std::mutex g_tune_mu;
bool g_tune_loaded = false;
std::string g_tune_text;

std::string library_dir() {
  Dl_info di;
  if (dladdr(reinterpret_cast<void*>(&release_batch_arenas), &di) == 0 || !di.dli_fname) return ".";
  std::string f = di.dli_fname;
  const size_t slash = f.rfind('/');
  return slash == std::string::npos ? "." : f.substr(0, slash);
}

const std::string& tune_text() {
  std::lock_guard<std::mutex> g(g_tune_mu);
  if (!g_tune_loaded) {
    g_tune_loaded = true;
    const char* env = std::getenv("ICUR_TUNE_FILE");
    const std::string path = env ? std::string(env) : library_dir() + "/tune_gfx950.json";
    if (FILE* f = std::fopen(path.c_str(), "rb")) {
      char buf[4096];
      size_t k;
      while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0 && g_tune_text.size() < (size_t(1) << 20))
        g_tune_text.append(buf, k);
      std::fclose(f);
    }
  }
  return g_tune_text;
}

// The integer after "key": within text[from, to), or -1.
int json_int(const std::string& text, size_t from, size_t to, const std::string& key) {
  const std::string k = "\"" + key + "\"";
  const size_t at = text.find(k, from);
  if (at == std::string::npos || at >= to) return -1;
  size_t p = text.find(':', at + k.size());
  if (p == std::string::npos || p >= to) return -1;
  ++p;
  while (p < to && (text[p] == ' ' || text[p] == '\t' || text[p] == '\n' || text[p] == '\r')) ++p;
  if (p >= to || text[p] < '0' || text[p] > '9') return -1;
  int v = 0;
  while (p < to && text[p] >= '0' && text[p] <= '9' && v < 1000000) v = 10 * v + (text[p++] - '0');
  return v;
}

}  // namespace

GemmTiles batch_tiles(int b) {
  GemmTiles t;
  // a block of up to 32 rows: 32 x 128 tiles with two chunks in flight; else the tile
  // that holds the block
  const int rows = b <= 16 ? 0 : b <= 32 ? 9 : b <= 48 ? 2 : 10;
  t.p1 = t.p2 = t.p3 = rows;
  t.fin = 9;
  // tune file: "batched_tiles": { "<b>": {"p1": .., "p2": .., "p3": .., "fin": ..}, ... }
  const std::string& txt = tune_text();
  const size_t sec = txt.find("\"batched_tiles\"");
  if (sec != std::string::npos) {
    const size_t at = txt.find("\"" + std::to_string(b) + "\"", sec);
    if (at != std::string::npos) {
      const size_t open = txt.find('{', at), close = txt.find('}', at);
      if (open != std::string::npos && close != std::string::npos && open < close) {
        int* f[4] = {&t.p1, &t.p2, &t.p3, &t.fin};
        const char* names[4] = {"p1", "p2", "p3", "fin"};
        for (int q = 0; q < 4; ++q) {
          const int v = json_int(txt, open, close, names[q]);
          if (v >= 0 && v < kGemmShapes) *f[q] = v;
        }
      }
    }
  }
  if (const char* env = std::getenv("ICUR_BATCH_TILES")) {
    int v[4];
    if (std::sscanf(env, "%d,%d,%d,%d", &v[0], &v[1], &v[2], &v[3]) == 4) {
      int* f[4] = {&t.p1, &t.p2, &t.p3, &t.fin};
      for (int q = 0; q < 4; ++q)
        if (v[q] >= 0 && v[q] < kGemmShapes) *f[q] = v[q];
    }
  }
  return t;
}

void release_batch_arenas() {
  std::lock_guard<std::mutex> g(g_arena_mu);
  int dev0 = 0;
  (void)hipGetDevice(&dev0);
  for (auto& kv : g_arenas) {
    if (!kv.second.p) continue;
    (void)hipSetDevice(kv.first);
    (void)hipFree(kv.second.p);
  }
  g_arenas.clear();
  (void)hipSetDevice(dev0);
}

namespace {

// The grouped call on its own stream st (see run_batched_grouped).
int run_grouped_on(const std::vector<int>& which, BatchedCall& a, hipStream_t st) {
  const int count = static_cast<int>(which.size());
  if (count == 0) return ICUR_OK;
  const icur_opts& o = *a.opts;
  const int64_t b = a.block;
  const int64_t c = (11 * b) / 10;
  const int zeta = o.zeta > 0 ? o.zeta : 8;
  const bool split = (o.precision == ICUR_BF16_SPLIT);
  DeviceInfo dev;
  ICUR_TRY(device_info(&dev));

  // ---- fixed per-matrix buffers in one allocation
  std::vector<BatchMat> hm(count);
  std::vector<size_t> off(count + 1, 0);
  for (int q = 0; q < count; ++q) {
    const int i = which[q];
    const int64_t m = a.m[i], n = a.n[i];
    const int64_t nparts = ((c + 31) / 32) * ((n + 127) / 128);
    off[q + 1] = off[q] + al(c * n * 8) + al(b * std::max(m, n) * 8) + al(b * n * 8) + al(c * b * 8) +
                 al(b * b * 8) + al(nparts * 8) + al(n) + al(m) + 2 * al(b * 8);
  }
  DevBuf fixed;
  ICUR_TRY(fixed.alloc(off[count]));
  for (int q = 0; q < count; ++q) {
    const int i = which[q];
    BatchMat& bm = hm[q];
    std::memset(&bm, 0, sizeof(bm));
    bm.A = a.A[i];
    bm.lda = a.lda[i];
    bm.m = static_cast<int>(a.m[i]);
    bm.n = static_cast<int>(a.n[i]);
    const int64_t m = bm.m, n = bm.n;
    const int64_t nparts = ((c + 31) / 32) * ((n + 127) / 128);
    char* p = static_cast<char*>(fixed.p) + off[q];
    bm.S = reinterpret_cast<double*>(p);
    p += al(c * n * 8);
    bm.Lsel = reinterpret_cast<double*>(p);
    p += al(b * std::max(m, n) * 8);
    bm.Sr = reinterpret_cast<double*>(p);
    p += al(b * n * 8);
    bm.Wc = reinterpret_cast<double*>(p);
    p += al(c * b * 8);
    bm.Nk = reinterpret_cast<double*>(p);
    p += al(b * b * 8);
    bm.normp = reinterpret_cast<double*>(p);
    p += al(nparts * 8);
    bm.colmask = reinterpret_cast<uint8_t*>(p);
    p += al(n);
    bm.rowmask = reinterpret_cast<uint8_t*>(p);
    p += al(m);
    bm.Jk = reinterpret_cast<int64_t*>(p);
    p += al(b * 8);
    bm.Ik = reinterpret_cast<int64_t*>(p);
    bm.rmax = static_cast<int>(o.max_rank == 0 ? std::min(m, n) : std::min<int64_t>(o.max_rank, std::min(m, n)));
  }
  ICUR_HIP(hipMemsetAsync(fixed.p, 0, off[count], st));

  // ---- sketch of every matrix: G, X0 = G A into S, ||G A||_F^2 (and ||A||_F^2)
  constexpr int kSketchStreams = 4;
  std::vector<hipStream_t> ss(kSketchStreams);
  hipEvent_t ready;
  ICUR_HIP(hipEventCreate(&ready));
  ICUR_HIP(hipEventRecord(ready, st));
  const auto t_sk0 = std::chrono::steady_clock::now();
  int64_t mmax = 0, nmax = 0;
  for (int q = 0; q < count; ++q) {
    mmax = std::max<int64_t>(mmax, hm[q].m);
    nmax = std::max<int64_t>(nmax, hm[q].n);
  }
  const int64_t ldg_max = (mmax + 7) / 8 * 8;
  size_t gemm_ws = std::max(sketch_workspace_bytes(c, mmax, nmax, dev.num_cus),
                            wide_gemm_workspace_bytes(c, mmax, nmax, dev.num_cus));
  const int nparts_cap = std::max(std::max(sketch_max_norm_partials(c, nmax), max_norm_partials(c, nmax)),
                                  kSumsqMaxParts);
  const size_t gbytes = al(sketch_G_bytes(a.kind, c, mmax, ldg_max));
  const size_t per_stream = gbytes + al(gemm_ws) + al(nparts_cap * 8);
  DevBuf sk;
  ICUR_TRY(sk.alloc(per_stream * kSketchStreams + al(static_cast<size_t>(count) * 16)));
  double* norms_dev = reinterpret_cast<double*>(static_cast<char*>(sk.p) + per_stream * kSketchStreams);
  int err = ICUR_OK;
  for (int s = 0; s < kSketchStreams; ++s) {
    ICUR_HIP(hipStreamCreateWithFlags(&ss[s], hipStreamNonBlocking));
    ICUR_HIP(hipStreamWaitEvent(ss[s], ready, 0));
  }
  const bool denom_a = (o.denominator == ICUR_DENOM_A);
  for (int q = 0; q < count && err == ICUR_OK; ++q) {
    const int i = which[q];
    const int sidx = q % kSketchStreams;
    hipStream_t s2 = ss[sidx];
    char* base = static_cast<char*>(sk.p) + per_stream * sidx;
    uint16_t* G = reinterpret_cast<uint16_t*>(base);
    void* ws = base + gbytes;
    double* parts = reinterpret_cast<double*>(base + gbytes + al(gemm_ws));
    BatchMat& bm = hm[q];
    const int64_t m = bm.m, n = bm.n, ldg = (m + 7) / 8 * 8;
    const int terms = split ? (o.split_terms ? o.split_terms : terms_for_tol(a.tol[i])) : (o.sketch_fp32 ? 0 : 3);
    bool used = false;
    err = form_sketch(a.kind, a.seed[i], c, m, n, bm.A, bm.lda, zeta, terms, a.tol[i] < kSketchChunkFlushBelow, G,
                      ldg, bm.S, parts, ws, gemm_ws, norms_dev + 2 * q, s2, nullptr, nullptr, &used);
    a.sketch_kernel += used ? 1 : 0;
    if (err == ICUR_OK && denom_a) {
      int np = 0;
      err = launch_sumsq_f32(bm.A, m, n, bm.lda, parts, &np, s2);
      if (err == ICUR_OK) err = launch_reduce_partials(parts, np, norms_dev + 2 * q + 1, s2);
    }
  }
  for (int s = 0; s < kSketchStreams; ++s) {
    if (err == ICUR_OK) {
      const hipError_t e = hipStreamSynchronize(ss[s]);
      if (e != hipSuccess) {
        set_error(std::string("batched sketch: ") + hipGetErrorString(e));
        err = ICUR_ERR_HIP;
      }
    }
    (void)hipStreamDestroy(ss[s]);
  }
  (void)hipEventDestroy(ready);
  if (err != ICUR_OK) return err;
  a.ms_sketch = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_sk0).count();
  std::vector<double> norms(2 * count);
  ICUR_HIP(hipMemcpy(norms.data(), norms_dev, norms.size() * 8, hipMemcpyDeviceToHost));

  // ---- loop state
  const auto t_al0 = std::chrono::steady_clock::now();
  const double sg2 = a.kind == ICUR_SKETCH_GAUSSIAN ? static_cast<double>(c)
                     : a.kind == ICUR_SKETCH_SRTT   ? 1.0
                                                    : static_cast<double>(std::min<int64_t>(zeta, c));
  std::vector<char> live(count, 0);
  for (int q = 0; q < count; ++q) {
    const int i = which[q];
    BatchMat& bm = hm[q];
    const double g2 = norms[2 * q];
    a.status[i] = ICUR_OK;
    a.rank[i] = 0;
    a.est[i] = 0.0;
    if (!std::isfinite(g2)) {
      a.status[i] = ICUR_ERR_NONFINITE;
      a.errs[i] = "||G A||_F is not finite: A holds Inf or NaN";
      continue;
    }
    bm.denom2 = denom_a ? sg2 * norms[2 * q + 1] : g2;
    bm.thr = a.xi * a.tol[i];
    const double rho0 = g2 == 0.0 ? 0.0 : std::sqrt(g2 / bm.denom2);
    bm.rho = rho0;
    a.est[i] = rho0;
    if (g2 == 0.0 || (denom_a && rho0 <= bm.thr)) continue;  // rank 0
    bm.s = static_cast<int>(std::min<int64_t>(b, bm.rmax));
    live[q] = 1;
  }
  for (int q = 0; q < count; ++q) {
    if (!live[q]) hm[q].fin = 1;  // nothing to multiply out
  }
  // rank-sized buffers: the whole rank bound of every matrix when that fits in the free
  // device memory (no growth), else the largest common fraction of it that fills 60% of
  // the arena, grown on demand
  ArenaHold hold;
  hold.device = dev.device;
  hold.a = take_arena(dev.device);
  size_t free_b = 0, total_b = 0;
  ICUR_HIP(hipMemGetInfo(&free_b, &total_b));
  free_b += hold.a.bytes;
  const size_t reserve = std::max<size_t>(size_t(2) << 30, total_b / 32) + batch_plan_bytes(count) +
                         sizeof(BatchMat) * count + (size_t(64) << 20);
  size_t budget = free_b > reserve ? free_b - reserve : 0;
  // ICUR_BATCH_MEMORY_LIMIT (bytes) lowers the budget, which exercises the growth path
  if (const char* lim = std::getenv("ICUR_BATCH_MEMORY_LIMIT")) {
    const unsigned long long v = std::strtoull(lim, nullptr, 10);
    if (v > 0) budget = std::min<size_t>(budget, static_cast<size_t>(v));
  }
  std::vector<int64_t> cap0(count, 0);
  auto total_for = [&](double f) {
    size_t t = 0;
    for (int q = 0; q < count; ++q) {
      if (!live[q]) continue;
      const BatchMat& bm = hm[q];
      const int64_t cq = std::min<int64_t>(bm.rmax, std::max<int64_t>(std::min<int64_t>(4 * b, bm.rmax),
                                                                      static_cast<int64_t>(std::ceil(f * bm.rmax))));
      cap0[q] = cq;
      t += al(rank_bytes(cq, bm.m, bm.n, b));
    }
    return t;
  };
  size_t need = total_for(1.0);
  size_t arena_bytes = need;
  if (need > budget) {
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 30; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (total_for(mid) <= budget * 6 / 10) lo = mid;
      else hi = mid;
    }
    need = total_for(lo);
    arena_bytes = std::max(need, budget);
  }
  if (need > 0 && hold.a.bytes < arena_bytes) {
    if (hold.a.p) ICUR_HIP(hipFree(hold.a.p));
    hold.a = CachedArena();
    void* p = nullptr;
    if (hipMalloc(&p, arena_bytes) != hipSuccess) {
      (void)hipGetLastError();
      arena_bytes = need;
      if (hipMalloc(&p, arena_bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_error("device allocation of " + std::to_string(arena_bytes) + " bytes failed (batched)");
        return ICUR_ERR_NOMEM;
      }
    }
    hold.a.p = p;
    hold.a.bytes = arena_bytes;
  }
  Arena arena;
  arena.reset(hold.a.p, need > 0 ? arena_bytes : 0);
  std::deque<DevBuf> extra;  // growth beyond the arena (a deque: elements never move)
  for (int q = 0; q < count; ++q) {
    if (!live[q]) continue;
    char* p = arena.take(rank_bytes(cap0[q], hm[q].m, hm[q].n, b));
    if (!p) return arg_error("batched: arena plan");  // cannot happen: sized from the same sums
    bind_rank(hm[q], p, cap0[q], b);
  }
  a.ms_alloc = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_al0).count();
  DevBuf mats, plan;
  ICUR_TRY(mats.alloc(sizeof(BatchMat) * count));
  ICUR_TRY(plan.alloc(batch_plan_bytes(count)));
  BatchMat* dmats = static_cast<BatchMat*>(mats.p);
  BatchRec* hrec = nullptr;
  ICUR_HIP(hipHostMalloc(reinterpret_cast<void**>(&hrec), sizeof(BatchRec) * count, hipHostMallocMapped));
  struct PinnedFree {
    void* p;
    ~PinnedFree() { (void)hipHostFree(p); }
  } pin_guard{hrec};
  BatchRec* drec = nullptr;
  ICUR_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&drec), hrec, 0));
  ICUR_HIP(hipMemcpyAsync(dmats, hm.data(), sizeof(BatchMat) * count, hipMemcpyHostToDevice, st));
  const int grid = 4 * dev.num_cus;
  const GemmTiles tiles = batch_tiles(static_cast<int>(b));
  a.tiles[0] = tiles.p1;
  a.tiles[1] = tiles.p2;
  a.tiles[2] = tiles.p3;
  a.tiles[3] = tiles.fin;
  for (double& v : a.ms_stage) v = 0.0;
  // device events around the selections, the product stages and the closing core
  // products of every iteration
  constexpr int kEv = 14;
  hipEvent_t ev[kEv];
  for (int e = 0; e < kEv; ++e) ICUR_HIP(hipEventCreate(&ev[e]));
  struct EvFree {
    hipEvent_t* e;
    ~EvFree() {
      for (int q = 0; q < kEv; ++q) (void)hipEventDestroy(e[q]);
    }
  } ev_guard{ev};
  ICUR_HIP(hipMemsetAsync(batch_plan_bytes_ptr(plan.p, count), 0, sizeof(double) * batch_plan_stages(), st));
  a.ms_select = a.ms_products = a.ms_final = 0.0;
  a.product_launches = 0;

  // a matrix that stops: its results to the copy thread (its core was multiplied out by
  // the same iteration's closing launch)
  ResultCopier copier(dev.device, a.opts->device_outputs ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost);
  auto settle = [&](int q) {
    const int i = which[q];
    const BatchMat& bm = hm[q];
    if (bm.status == ICUR_ERR_HIP || bm.info != 0) {
      a.status[i] = ICUR_ERR_HIP;
      a.errs[i] = "the residual block N_k = S(I_k, J_k) is exactly singular";
      a.rank[i] = 0;
      a.est[i] = 0.0;
      return;
    }
    const int64_t r = bm.r;
    a.rank[i] = r;
    a.est[i] = bm.rho;
    a.status[i] = bm.status;
    if (r == 0) return;
    ResultCopier::Job j;
    j.dst[0] = a.I_pool + a.cap_offsets[i];
    j.src[0] = bm.Iall;
    j.bytes[0] = r * 8;
    j.dst[1] = a.J_pool + a.cap_offsets[i];
    j.src[1] = bm.Jall;
    j.bytes[1] = r * 8;
    j.dst[2] = a.U_pool + a.uoff[i];
    j.src[2] = bm.LcT;
    j.bytes[2] = r * r * 8;
    copier.push(j);
  };

  bool any = false;
  for (const BatchMat& bm : hm) any |= bm.s != 0;
  int iters = 0;
  const auto t_loop0 = std::chrono::steady_clock::now();
  int err_loop = ICUR_OK;
  // One iteration's launches (the selections, plan, gathers, products, end kernel and
  // the core products of the matrices that stop), with device events for the timings.
  // With ICUR_BATCH_GRAPH=1 they run from the second iteration on as one captured graph
  // (the configuration of every launch depends only on the batch size and the device, and
  // all state lives in device memory).  Plain launches are the default: an iteration is
  // about ten milliseconds of device work against tens of microseconds of launches, so the
  // replay gains nothing, and the event nodes of a replayed graph do not time the stages.
  auto enqueue_iteration = [&]() -> int {
    ICUR_TRY(launch_batch_iteration(dmats, count, static_cast<int>(c), static_cast<int>(b), a.row_cut, plan.p, drec,
                                    tiles, grid, st, ev));
    ICUR_HIP(hipEventRecord(ev[12], st));
    ICUR_TRY(launch_batch_final(dmats, count, static_cast<int>(c), static_cast<int>(b), plan.p, tiles, st));
    ICUR_HIP(hipEventRecord(ev[13], st));
    return ICUR_OK;
  };
  const char* genv = std::getenv("ICUR_BATCH_GRAPH");
  const bool use_graph = genv && genv[0] == '1';
  struct GraphHold {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    ~GraphHold() {
      if (x) (void)hipGraphExecDestroy(x);
      if (g) (void)hipGraphDestroy(g);
    }
  } gh;
  a.graph_iterations = 0;
  while (any && err_loop == ICUR_OK) {
    if (gh.x) {
      const hipError_t le = hipGraphLaunch(gh.x, st);
      if (le != hipSuccess) {
        err_loop = hip_error(le, "batched: iteration graph launch");
        break;
      }
      ++a.graph_iterations;
    } else {
      err_loop = enqueue_iteration();
      if (err_loop != ICUR_OK) break;
    }
    const hipError_t se = hipStreamSynchronize(st);
    if (se != hipSuccess) {
      err_loop = hip_error(se, "batched loop");
      break;
    }
    ++iters;
    for (int e = 0; e < kEv; e += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[e], ev[e + 1]) != hipSuccess) {
        (void)hipGetLastError();
        ms = 0.f;
      }
      if (e < 4) {
        a.ms_select += ms;
      } else if (e < 12) {
        a.ms_products += ms;
        a.product_launches += 1;
      } else {
        a.ms_final += ms;
      }
      if (e >= 4) a.ms_stage[(e - 4) / 2] += ms;
    }
    any = false;
    bool grow = false;
    for (int q = 0; q < count && err_loop == ICUR_OK; ++q) {
      BatchMat& bm = hm[q];
      if (bm.s == 0) continue;
      const BatchRec& rc = hrec[q];
      bm.r = rc.r;
      bm.s = rc.s;
      bm.status = rc.status;
      bm.info = rc.info;
      bm.iters = rc.iters;
      bm.rho = rc.rho;
      if (bm.s == 0) {
        bm.fin = 1;  // as the device set it in this iteration's closing launch
        settle(q);
        continue;
      }
      any = true;
      if (bm.r + bm.s > bm.cap) {
        // grow the rank-sized buffers: keep LcT, Ur and the two inverses (rows 0..r, new
        // leading dimension) and the index lists
        const int64_t ncap = std::min<int64_t>(bm.rmax, std::max<int64_t>(2 * bm.cap, bm.r + bm.s));
        const size_t nbytes = rank_bytes(ncap, bm.m, bm.n, b);
        char* np = arena.take(nbytes);
        if (!np) {
          extra.emplace_back();
          err_loop = extra.back().alloc(nbytes);
          if (err_loop != ICUR_OK) break;
          np = static_cast<char*>(extra.back().p);
        }
        BatchMat nm = bm;
        bind_rank(nm, np, ncap, b);
        const size_t r = static_cast<size_t>(bm.r);
        hipError_t e = hipMemcpyAsync(nm.LcT, bm.LcT, r * bm.m * 8, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(nm.Ur, bm.Ur, r * bm.n * 8, hipMemcpyDeviceToDevice, st);
        if (r > 0) {
          // the r block rows of both inverses, their band beyond the old width zeroed
          const size_t oc = static_cast<size_t>(bm.cap);
          const size_t zc = std::min<size_t>(ncap, r + kBandCols);
          for (int f = 0; f < 2 && e == hipSuccess; ++f) {
            double* dst = f ? nm.Pi : nm.QT;
            const double* src = f ? bm.Pi : bm.QT;
            e = hipMemcpy2DAsync(dst, ncap * 8, src, oc * 8, oc * 8, r, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess && zc > oc) e = hipMemset2DAsync(dst + oc, ncap * 8, 0, (zc - oc) * 8, r, st);
          }
        }
        if (e == hipSuccess) e = hipMemcpyAsync(nm.Jall, bm.Jall, r * 8, hipMemcpyDeviceToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(nm.Iall, bm.Iall, r * 8, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) {
          err_loop = hip_error(e, "batched: growth copies");
          break;
        }
        // the old region is free for later allocations (stream ordered)
        char* old = reinterpret_cast<char*>(bm.LcT);
        if (arena.owns(old)) arena.give(old, rank_bytes(bm.cap, bm.m, bm.n, b));
        bm = nm;
        grow = true;
      }
    }
    if (grow && err_loop == ICUR_OK) {
      const hipError_t e = hipMemcpyAsync(dmats, hm.data(), sizeof(BatchMat) * count, hipMemcpyHostToDevice, st);
      if (e != hipSuccess) err_loop = hip_error(e, "batched: state upload");
    }
    if (use_graph && !gh.x && any && err_loop == ICUR_OK) {
      // capture the next iteration (every lazily initialised launch parameter is set by now)
      const hipError_t be = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
      if (be != hipSuccess) {
        err_loop = hip_error(be, "batched: begin capture");
        break;
      }
      const int qe = enqueue_iteration();
      hipGraph_t g = nullptr;
      const hipError_t ce = hipStreamEndCapture(st, &g);
      gh.g = g;
      if (qe != ICUR_OK) {
        err_loop = qe;
        break;
      }
      if (ce != hipSuccess || !g) {
        err_loop = hip_error(ce, "batched: iteration capture");
        break;
      }
      const hipError_t ie = hipGraphInstantiate(&gh.x, g, nullptr, nullptr, 0);
      if (ie != hipSuccess) {
        gh.x = nullptr;
        err_loop = hip_error(ie, "batched: iteration graph");
        break;
      }
    }
  }
  a.ms_loop = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_loop0).count();
  const auto t_res0 = std::chrono::steady_clock::now();
  const std::string cerr = copier.finish();
  if (err_loop != ICUR_OK) return err_loop;
  if (!cerr.empty()) {
    set_error(cerr);
    return ICUR_ERR_HIP;
  }
  double stage_bytes[8];
  if (batch_plan_stages() > 8) return arg_error("batched: plan stage count");
  ICUR_HIP(hipMemcpyAsync(stage_bytes, batch_plan_bytes_ptr(plan.p, count), sizeof(double) * batch_plan_stages(),
                          hipMemcpyDeviceToHost, st));
  ICUR_HIP(hipStreamSynchronize(st));
  a.iterations = iters;
  a.product_bytes = 0.0;
  for (int q = 0; q < batch_plan_stages(); ++q)
    if (q != batch_plan_final_stage()) a.product_bytes += stage_bytes[q];
  {
    int k = 0;
    for (int q : batch_plan_product_stages()) a.stage_bytes[k++] = stage_bytes[q];
  }
  a.ms_results = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_res0).count();
  return ICUR_OK;
}

}  // namespace

// Runs the matrices listed in `which` (all with max(m, n) <= kGMaxN, block <= kGMaxSteps)
// on a stream of its own (a graph cannot be captured on the legacy default stream), after
// the caller's stream; the caller's stream then waits for it.
int run_batched_grouped(const std::vector<int>& which, BatchedCall& a, hipStream_t caller) {
  hipStream_t ps = nullptr;
  ICUR_HIP(hipStreamCreateWithFlags(&ps, hipStreamNonBlocking));
  struct StreamFree {
    hipStream_t s;
    ~StreamFree() { (void)hipStreamDestroy(s); }
  } sf{ps};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ICUR_HIP(hipEventCreateWithFlags(&e0, hipEventDisableTiming));
  struct EventFree {
    hipEvent_t* e[2];
    ~EventFree() {
      for (hipEvent_t* q : e)
        if (*q) (void)hipEventDestroy(*q);
    }
  } ef{{&e0, &e1}};
  ICUR_HIP(hipEventCreateWithFlags(&e1, hipEventDisableTiming));
  ICUR_HIP(hipEventRecord(e0, caller));
  ICUR_HIP(hipStreamWaitEvent(ps, e0, 0));
  const int rc = run_grouped_on(which, a, ps);
  ICUR_HIP(hipEventRecord(e1, ps));
  ICUR_HIP(hipStreamWaitEvent(caller, e1, 0));
  return rc;
}

}  // namespace icur
