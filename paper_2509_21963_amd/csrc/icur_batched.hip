// Host driver of the grouped batched form: many dense matrices of uneven sizes and
// tolerances advanced together through Alg. 1, one launch per step for all of them.
//
//   1. sketch: G and X0 = G A for every matrix (the single-matrix sketch kernels, spread
//      over a few streams), then one read-back of all ||G A||_F^2;
//   2. loop: one iteration of every unfinished matrix (launch_batch_iteration: the two
//      grouped selections, grouped gathers and FP64 products, the pivot-block inverses,
//      the bordered core and the stopping decision), then one read-back of a small record
//      per matrix (rank, state), from which the host only grows rank-sized buffers;
//   3. results: I, J and the core U of each matrix copied to the caller's pools.
// Each matrix follows Alg. 1 on its own: the grouping changes no arithmetic.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "icur_batched.h"

namespace icur {

int launch_batch_iteration(BatchMat* mats, int count, int c, int b, double row_cut, void* plan_ws, BatchRec* rec,
                           int grid, hipStream_t st, hipEvent_t* ev);
size_t batch_plan_bytes(int count);
double* batch_plan_bytes_ptr(void* plan_ws, int count);

namespace {

size_t al(size_t b) { return (b + 255) & ~size_t(255); }

// Rank-sized part of a matrix's state for capacity cap.
size_t rank_bytes(int64_t cap, int64_t m, int64_t n, int64_t b) {
  return al(cap * m * 8) + al(cap * n * 8) + al(cap * cap * 8) + 6 * al(b * cap * 8) + 2 * al(cap * 8);
}

void bind_rank(BatchMat& bm, char* p, int64_t cap, int64_t b) {
  const int64_t m = bm.m, n = bm.n;
  bm.LcT = reinterpret_cast<double*>(p);
  p += al(cap * m * 8);
  bm.Ur = reinterpret_cast<double*>(p);
  p += al(cap * n * 8);
  bm.U = reinterpret_cast<double*>(p);
  p += al(cap * cap * 8);
  double** six[6] = {&bm.Wa, &bm.AIJk, &bm.AIkJ, &bm.Y, &bm.Z, &bm.V};
  for (double** q : six) {
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

}  // namespace

// Runs the matrices listed in `which` (all with max(m, n) <= kGMaxN, block <= kGMaxSteps).
int run_batched_grouped(const std::vector<int>& which, BatchedCall& a, hipStream_t st) {
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
    err = form_sketch(a.kind, a.seed[i], c, m, n, bm.A, bm.lda, zeta, terms, a.tol[i] < kSketchChunkFlushBelow, G,
                      ldg, bm.S, parts, ws, gemm_ws, norms_dev + 2 * q, s2, nullptr, nullptr);
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
  std::vector<DevBuf> rankbuf(count);
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
    // rank-sized buffers for the whole rank bound when they fit (no growth, no host
    // synchronisation inside the loop); else a quarter of it, grown on demand
    int64_t cap = bm.rmax;
    if (rankbuf[q].alloc(rank_bytes(cap, bm.m, bm.n, b)) != ICUR_OK) {
      set_error("");
      cap = std::min<int64_t>(bm.rmax, std::max<int64_t>(4 * b, bm.rmax / 4));
      ICUR_TRY(rankbuf[q].alloc(rank_bytes(cap, bm.m, bm.n, b)));
    }
    bind_rank(bm, static_cast<char*>(rankbuf[q].p), cap, b);
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
  // device events around the selections and the product stages of every iteration
  constexpr int kEv = 12;
  hipEvent_t ev[kEv];
  for (int e = 0; e < kEv; ++e) ICUR_HIP(hipEventCreate(&ev[e]));
  struct EvFree {
    hipEvent_t* e;
    ~EvFree() {
      for (int q = 0; q < kEv; ++q) (void)hipEventDestroy(e[q]);
    }
  } ev_guard{ev};
  ICUR_HIP(hipMemsetAsync(batch_plan_bytes_ptr(plan.p, count), 0, 8 * 8, st));
  a.ms_select = a.ms_products = 0.0;
  a.product_launches = 0;

  bool any = false;
  for (const BatchMat& bm : hm) any |= bm.s != 0;
  int iters = 0;
  const auto t_loop0 = std::chrono::steady_clock::now();
  while (any) {
    ICUR_TRY(launch_batch_iteration(dmats, count, static_cast<int>(c), static_cast<int>(b), a.row_cut, plan.p, drec,
                                    grid, st, ev));
    ICUR_HIP(hipStreamSynchronize(st));
    ++iters;
    for (int e = 0; e < kEv; e += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[e], ev[e + 1]) != hipSuccess) {
        (void)hipGetLastError();
        ms = 0.f;
      }
      if (e < 4) {
        a.ms_select += ms;
      } else {
        a.ms_products += ms;
        a.product_launches += 1;
      }
    }
    any = false;
    bool grow = false;
    for (int q = 0; q < count; ++q) {
      BatchMat& bm = hm[q];
      if (bm.s == 0) continue;
      const BatchRec& rc = hrec[q];
      bm.r = rc.r;
      bm.s = rc.s;
      bm.status = rc.status;
      bm.info = rc.info;
      bm.iters = rc.iters;
      bm.rho = rc.rho;
      if (bm.s == 0) continue;
      any = true;
      if (bm.r + bm.s > bm.cap) {
        // grow the rank-sized buffers: keep LcT, Ur (rows 0..r), U (r x r, new leading
        // dimension) and the index lists
        const int64_t ncap = std::min<int64_t>(bm.rmax, std::max<int64_t>(2 * bm.cap, bm.r + bm.s));
        DevBuf nb;
        ICUR_TRY(nb.alloc(rank_bytes(ncap, bm.m, bm.n, b)));
        BatchMat nm = bm;
        bind_rank(nm, static_cast<char*>(nb.p), ncap, b);
        const size_t r = static_cast<size_t>(bm.r);
        ICUR_HIP(hipMemcpyAsync(nm.LcT, bm.LcT, r * bm.m * 8, hipMemcpyDeviceToDevice, st));
        ICUR_HIP(hipMemcpyAsync(nm.Ur, bm.Ur, r * bm.n * 8, hipMemcpyDeviceToDevice, st));
        if (r > 0)
          ICUR_HIP(hipMemcpy2DAsync(nm.U, ncap * 8, bm.U, static_cast<size_t>(bm.cap) * 8, r * 8, r,
                                    hipMemcpyDeviceToDevice, st));
        ICUR_HIP(hipMemcpyAsync(nm.Jall, bm.Jall, r * 8, hipMemcpyDeviceToDevice, st));
        ICUR_HIP(hipMemcpyAsync(nm.Iall, bm.Iall, r * 8, hipMemcpyDeviceToDevice, st));
        ICUR_HIP(hipStreamSynchronize(st));
        std::swap(rankbuf[q].p, nb.p);
        bm = nm;
        grow = true;
      }
    }
    if (grow) ICUR_HIP(hipMemcpyAsync(dmats, hm.data(), sizeof(BatchMat) * count, hipMemcpyHostToDevice, st));
  }
  a.ms_loop = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_loop0).count();
  const auto t_res0 = std::chrono::steady_clock::now();
  // final state of every matrix (the host mirror holds r, status and rho of the last
  // iteration of each)
  ICUR_HIP(hipMemcpyAsync(hm.data(), dmats, sizeof(BatchMat) * count, hipMemcpyDeviceToHost, st));
  double stage_bytes[8];
  ICUR_HIP(hipMemcpyAsync(stage_bytes, batch_plan_bytes_ptr(plan.p, count), sizeof(stage_bytes), hipMemcpyDeviceToHost,
                          st));
  ICUR_HIP(hipStreamSynchronize(st));
  a.iterations = iters;
  a.product_bytes = 0.0;
  for (double v : stage_bytes) a.product_bytes += v;

  // ---- results
  for (int q = 0; q < count; ++q) {
    const int i = which[q];
    const BatchMat& bm = hm[q];
    if (a.status[i] < 0 && bm.cap == 0) continue;  // non-finite sketch
    if (bm.cap == 0) continue;                       // rank 0 (a zero matrix, or met at once)
    if (bm.status == ICUR_ERR_HIP || bm.info != 0) {
      a.status[i] = ICUR_ERR_HIP;
      a.errs[i] = "the residual block N_k = S(I_k, J_k) is exactly singular";
      a.rank[i] = 0;
      a.est[i] = 0.0;
      continue;
    }
    const int64_t r = bm.r;
    a.rank[i] = r;
    a.est[i] = bm.rho;
    a.status[i] = bm.status;
    if (r == 0) continue;
    ICUR_HIP(hipMemcpyAsync(a.I_pool + a.cap_offsets[i], bm.Iall, r * 8, hipMemcpyDeviceToHost, st));
    ICUR_HIP(hipMemcpyAsync(a.J_pool + a.cap_offsets[i], bm.Jall, r * 8, hipMemcpyDeviceToHost, st));
    ICUR_HIP(hipMemcpy2DAsync(a.U_pool + a.uoff[i], r * 8, bm.U, static_cast<size_t>(bm.cap) * 8, r * 8, r,
                              hipMemcpyDeviceToHost, st));
  }
  ICUR_HIP(hipStreamSynchronize(st));
  a.ms_results = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_res0).count();
  return ICUR_OK;
}

}  // namespace icur
