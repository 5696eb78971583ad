// C ABI: handles, device upload of the symbolic analysis, launch sequencing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/spchol.h"
#include "analyze.hpp"
#include "host_factor.hpp"
#include "order.hpp"
#include "device.hpp"

using namespace spchol;

namespace {

thread_local std::string g_err;

spchol_status fail(spchol_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? SPCHOL_ERR_OOM : SPCHOL_ERR_HIP,            \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                     \
  } while (0)

template <class T>
hipError_t upload(T** dst, const std::vector<T>& v) {
  *dst = nullptr;
  size_t bytes = v.size() * sizeof(T);
  if (bytes == 0) bytes = sizeof(T);
  hipError_t e = hipMalloc((void**)dst, bytes);
  if (e != hipSuccess) return e;
  if (!v.empty()) e = hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  return e;
}

}  // namespace

// Solve work vectors for callers that cannot allocate device memory
// (spchol_solve_noalloc): one array per GPU in static device memory, kept
// until the process ends, split into three fixed slices (permuted right-hand
// sides, forward result, split-panel accumulators).  Host code never passes
// `scratch` itself to a kernel: its device address comes from
// hipGetSymbolAddress, taken once per device.
constexpr int64_t kScratchSlice = int64_t(1) << 21;  // entries (n x nrhs) per slice
constexpr int kScratchMaxDevices = 64;
static __device__ __align__(256) double scratch[3 * kScratchSlice];  // 48 MiB

namespace {
std::mutex g_scratch_mu;
double* g_scratch_dev[kScratchMaxDevices] = {};

// Device address of `scratch` on the current device (set up on first use).
spchol_status scratch_address(double** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchMaxDevices) return fail(SPCHOL_ERR_ARG, "device ordinal out of range for the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(SPCHOL_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return SPCHOL_OK;
}
}  // namespace

struct spchol_sym_s {
  Symbolic S;
  int64_t ws_limit = 0;  // device bytes a numeric handle may hold (0: no limit)
  std::vector<int64_t> batch_off, batch_nzoff;  // block boundaries of a batch (empty: one matrix)
  const int64_t* dev_batch_off = nullptr;
  bool uploaded = false;
  int device = -1;
  DevSym dev{};
  const int64_t* si_yoff = nullptr;
  std::vector<void*> allocs;

  ~spchol_sym_s() {
    for (void* p : allocs) (void)hipFree(p);
  }

  template <class T>
  hipError_t up(const T** dst, const std::vector<T>& v) {
    T* p = nullptr;
    hipError_t e = upload(&p, v);
    if (p) allocs.push_back(p);
    *dst = p;
    return e;
  }

  // device bytes of the upload below (without uploading)
  int64_t device_bytes() const {
    int64_t b = 0;
    auto add = [&](size_t cnt, size_t sz) { b += (int64_t)((cnt > 0 ? cnt : 1) * sz); };
    const size_t ns = (size_t)S.ns;
    add(S.loff.size(), 8); add(ns, 4); add(ns, 4); add(ns, 4);
    add(S.rptr.size(), 8); add(S.rows.size(), 4); add(S.obase.size(), 8); add(S.opair.size(), 4);
    add(S.ocbase.size(), 8); add(S.pa0.size(), 4); add(S.relptr.size(), 8); add(S.tpos.size(), 4);
    add((size_t)S.n, 4); add(S.amap.size(), 8); add(S.perm.size(), 8); add(S.tasks.size(), sizeof(DevTask));
    add(S.a_rp.size(), 8); add(S.a_col.size(), 4); add(S.a_vidx.size(), 8); add(S.e_row.size(), 4);
    add(S.e_col.size(), 4); add(S.wbase.size(), 8); add(S.si_yoff.size(), 8);
    add(batch_off.empty() ? 2 : batch_off.size(), 8);
    return b;
  }

  spchol_status ensure_device() {
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (uploaded) {
      if (cur != device) return fail(SPCHOL_ERR_ARG, "symbolic handle is bound to another device");
      return SPCHOL_OK;
    }
    const int64_t ns = S.ns;
    std::vector<int32_t> sk(ns), sm(ns), sf(ns), pa0(S.pa0.size()), snode(S.n);
    for (int64_t J = 0; J < ns; ++J) {
      sk[J] = (int32_t)(S.sptr[J + 1] - S.sptr[J]);
      sm[J] = (int32_t)(S.rptr[J + 1] - S.rptr[J]);
      sf[J] = (int32_t)S.sptr[J];
    }
    for (size_t t = 0; t < S.pa0.size(); ++t) pa0[t] = (int32_t)S.pa0[t];
    for (int64_t j = 0; j < S.n; ++j) snode[j] = (int32_t)S.snode_of[j];
    std::vector<DevTask> tasks(S.tasks.size());
    for (size_t t = 0; t < S.tasks.size(); ++t) tasks[t] = {S.tasks[t].J, S.tasks[t].a, S.tasks[t].b, S.tasks[t].c};
    HIP_TRY(up(&dev.loff, S.loff));
    HIP_TRY(up(&dev.sk, sk));
    HIP_TRY(up(&dev.sm, sm));
    HIP_TRY(up(&dev.sfirst, sf));
    HIP_TRY(up(&dev.rptr, S.rptr));
    HIP_TRY(up(&dev.rows, S.rows));
    HIP_TRY(up(&dev.obase, S.obase));
    HIP_TRY(up(&dev.opair, S.opair));
    HIP_TRY(up(&dev.ocbase, S.ocbase));
    HIP_TRY(up(&dev.pa0, pa0));
    HIP_TRY(up(&dev.relptr, S.relptr));
    HIP_TRY(up(&dev.tpos, S.tpos));
    HIP_TRY(up(&dev.snode_of, snode));
    HIP_TRY(up(&dev.amap, S.amap));
    HIP_TRY(up(&dev.perm, S.perm));
    HIP_TRY(up(&dev.tasks, tasks));
    HIP_TRY(up(&dev.a_rp, S.a_rp));
    HIP_TRY(up(&dev.a_col, S.a_col));
    HIP_TRY(up(&dev.a_vidx, S.a_vidx));
    HIP_TRY(up(&dev.e_row, S.e_row));
    HIP_TRY(up(&dev.e_col, S.e_col));
    HIP_TRY(up(&dev.wbase, S.wbase));
    HIP_TRY(up(&si_yoff, S.si_yoff));
    {
      std::vector<int64_t> bo = batch_off;
      if (bo.empty()) bo = {0, S.n};
      HIP_TRY(up(&dev_batch_off, bo));
    }
    dev.n = S.n;
    dev.ns = ns;
    dev.nnzA = S.nnzA;
    dev.storage = S.loff[ns];
    dev.nb = S.nb;
    device = cur;
    uploaded = true;
    return SPCHOL_OK;
  }
};

// HIP events around launches, summed per kernel kind on request.
struct Profiler {
  struct Rec {
    int kind, level, side;
    hipEvent_t a, b;
    double flops, bytes;
  };
  bool on = false;
  bool serial = false;  // every launch alone: the far updates on the main stream
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Rec> recs;

  ~Profiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
  hipError_t take(hipEvent_t* e) {
    if (used == pool.size()) {
      hipEvent_t ne;
      hipError_t err = hipEventCreate(&ne);
      if (err != hipSuccess) return err;
      pool.push_back(ne);
    }
    *e = pool[used++];
    return hipSuccess;
  }
};

// Work vectors of a solve: the permuted right-hand sides y, the forward
// result x (solved in place by the backward sweep) and the backward sweep's
// per-column accumulators of split panels (zero between solves: the
// kernels leave them cleared).
struct SolveWork {
  double* y = nullptr;
  double* x = nullptr;
  double* acc = nullptr;
  int64_t cap = 0;  // entries of y, x and acc (n x nrhs)
  static int64_t bytes_for(int64_t n, int64_t nrhs) { return 3 * (n * nrhs > 0 ? n * nrhs : 1) * 8; }
  int64_t bytes() const { return cap > 0 ? 3 * cap * 8 : 0; }
  ~SolveWork() {
    for (double* p : {y, x, acc})
      if (p) (void)hipFreeAsync(p, nullptr);
  }
  // (Re)allocates stream-ordered on st and clears acc with a kernel: no
  // host synchronization, never inside a capture.  *moved is set when the
  // buffers were (re)allocated.
  hipError_t ensure(int64_t n, int64_t nrhs, hipStream_t st, bool* moved = nullptr) {
    if (moved) *moved = false;
    if (cap >= n * nrhs && acc) return hipSuccess;
    if (moved) *moved = true;
    for (double** p : {&y, &x, &acc}) {
      if (*p) {
        hipError_t e = hipFreeAsync(*p, st);
        if (e != hipSuccess) return e;
      }
      *p = nullptr;
    }
    cap = 0;
    const int64_t cnt = n * nrhs > 0 ? n * nrhs : 1;
    const size_t v = (size_t)cnt * sizeof(double);
    for (double** p : {&y, &x, &acc}) {
      hipError_t e = hipMallocAsync((void**)p, v, st);
      if (e != hipSuccess) return e;
    }
    hipError_t e = launch_fill(acc, cnt, 0.0, st);
    if (e != hipSuccess) return e;
    cap = cnt;
    return hipSuccess;
  }
};

// A launch sequence seen again with the same arguments is captured as a
// hipGraph and replayed from then on (one host launch instead of hundreds).
struct CachedGraph {
  int kind = 0;            // 0: factorization, 1: solve
  const void* ptr = nullptr;  // values / right-hand sides
  int64_t a = 0, b = 0;    // precision / (nrhs, ldb)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
};

struct spchol_num_s {
  spchol_sym_s* sym = nullptr;
  // second stream (default priority) for the external updates that run
  // beside the next level's panel chain, and the events that fork and join it
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev = nullptr;  // solves: the second stream's groups joined back
  std::vector<hipEvent_t> side_ev;  // per level
  std::vector<CachedGraph> gcache;  // most recent last
  bool gcache_on = true;
  double* L = nullptr;
  unsigned long long* status = nullptr;
  SolveWork sw;
  double* red = nullptr;  // logdet partials + result
  double* winv = nullptr;  // inverted diagonal blocks of all panels
  int32_t prec = 0;           // update precision of the last factorization
  double* rwork = nullptr;    // refinement residual / correction, n x nrhs
  int64_t rcap = 0;
  double* pwork = nullptr;    // conjugate gradients: z, p, q (n x nrhs each), then 3 nrhs scalars
  int64_t pcap = 0;
  unsigned long long* stats = nullptr;  // refinement norms (3 per RHS + 1)
  int64_t scap = 0;
  double* Z = nullptr;     // selected inverse, layout of L
  double* sibuf = nullptr; // Y blocks, inverses and T of one round
  double* lam = nullptr;   // adjoint solve, n x nrhs
  int64_t lcap = 0;
  int64_t zcap = 0, sicap = 0;  // elements of Z and sibuf
  Profiler prof;
  int64_t held = 0;  // device bytes counted against the analysis' workspace limit
  void drop_graphs(int kind) {  // kind < 0: all
    std::vector<CachedGraph> keep;
    for (CachedGraph& g : gcache) {
      if (kind < 0 || g.kind == kind) g.release();
      else keep.push_back(g);
    }
    gcache.swap(keep);
  }
  ~spchol_num_s() {
    drop_graphs(-1);
    for (hipEvent_t e : side_ev)
      if (e) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (join_ev) (void)hipEventDestroy(join_ev);
    if (side) (void)hipStreamDestroy(side);
    for (void* p : {(void*)Z, (void*)sibuf, (void*)lam, (void*)rwork, (void*)pwork, (void*)stats})
      if (p) (void)hipFreeAsync(p, nullptr);
    if (L) (void)hipFree(L);
    if (winv) (void)hipFree(winv);
    if (status) (void)hipFree(status);
    if (red) (void)hipFree(red);
  }
};

// Run `launch` (returning hipError_t), bracketed by events when profiling;
// level / side: the launch's level in the schedule (-1: outside it) and
// whether it runs on the second stream.
template <class F>
static hipError_t timed_at(spchol_num_s* N, int kind, int level, int side, double flops, double bytes,
                           hipStream_t st, F&& launch) {
  if (!N->prof.on) return launch();
  Profiler::Rec r{kind, level, side, nullptr, nullptr, flops, bytes};
  hipError_t e = N->prof.take(&r.a);
  if (e == hipSuccess) e = N->prof.take(&r.b);
  if (e == hipSuccess) e = hipEventRecord(r.a, st);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(r.b, st);
  if (e == hipSuccess) N->prof.recs.push_back(r);
  return e;
}

template <class F>
static hipError_t timed(spchol_num_s* N, int kind, double flops, double bytes, hipStream_t st, F&& launch) {
  return timed_at(N, kind, -1, 0, flops, bytes, st, launch);
}

// The workspace limit of the analysis: fail before allocating `extra` more
// bytes when the handle would then hold more than the limit.
static spchol_status ws_check(spchol_num_s* N, int64_t extra) {
  const int64_t lim = N->sym->ws_limit;
  if (lim > 0 && N->held + extra > lim)
    return fail(SPCHOL_ERR_OOM, "workspace limit of " + std::to_string(lim) + " bytes: the handle holds " +
                                    std::to_string(N->held) + " and needs " + std::to_string(extra) + " more");
  return SPCHOL_OK;
}

// Grow a device buffer of the handle to at least `want` elements,
// stream-ordered on st (no host synchronization; never inside a capture),
// after checking the workspace limit.  *moved is set when it was
// (re)allocated.
template <class T>
static spchol_status grow(spchol_num_s* N, T** buf, int64_t* cap, int64_t want, hipStream_t st,
                          bool* moved = nullptr) {
  if (moved) *moved = false;
  if (want < 1) want = 1;
  if (*buf && *cap >= want) return SPCHOL_OK;
  const int64_t oldb = *buf ? *cap * (int64_t)sizeof(T) : 0, newb = want * (int64_t)sizeof(T);
  spchol_status s = ws_check(N, newb - oldb);
  if (s) return s;
  if (*buf) HIP_TRY(hipFreeAsync(*buf, st));
  *buf = nullptr;
  *cap = 0;
  N->held -= oldb;
  HIP_TRY(hipMallocAsync((void**)buf, (size_t)newb, st));
  N->held += newb;
  *cap = want;
  if (moved) *moved = true;
  return SPCHOL_OK;
}

// Enqueue the whole numeric factorization on st (no host synchronization:
// also what a graph capture records).
static spchol_status enqueue_factor(spchol_num_s* N, const double* vals, hipStream_t st) {
  const Symbolic& S = N->sym->S;
  const int32_t prec = N->prec;
  const DevSym& D = N->sym->dev;
  HIP_TRY(timed(N, SPCHOL_KERNEL_FILL, 0.0, 8.0 * D.storage, st,
                [&] { return launch_fill(N->L, D.storage, 0.0, st); }));
  HIP_TRY(launch_status_init(N->status, st));
  HIP_TRY(timed(N, SPCHOL_KERNEL_SCATTER_A, 0.0, 24.0 * D.nnzA, st,
                [&] { return launch_scatter_values(D, vals, N->L, st); }));
  if (!N->side) {
    // created before any capture (stream and event creation is not captured)
    HIP_TRY(hipStreamCreateWithFlags(&N->side, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&N->fork_ev, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&N->join_ev, hipEventDisableTiming));
    N->side_ev.assign(S.nlevels + 1, nullptr);
    for (hipEvent_t& e : N->side_ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  std::vector<int64_t> outstanding;  // levels whose side launch is not joined yet
  bool forked = false;
  // profiling with every launch alone: the far updates run on st in plan
  // order (right after the near ones), so each record is one launch's own time
  const bool one_stream = N->prof.on && N->prof.serial;
  for (size_t li = 0; li < S.factor_plan.size(); ++li) {
    const Launch& l = S.factor_plan[li];
    if (l.side && !one_stream) {
      // fork: the side stream starts once everything before is done
      if (!forked) HIP_TRY(hipEventRecord(N->fork_ev, st));
      forked = false;
      HIP_TRY(hipStreamWaitEvent(N->side, N->fork_ev, 0));
      const int32_t uk = l.kind == K_UPD_RLB ? 4 : l.kind;
      HIP_TRY(timed_at(N, SPCHOL_KERNEL_UPDATE_EXT, l.level, 1, l.flops, l.bytes, N->side,
                       [&] { return launch_update(D, N->L, uk, l.off, l.ntasks, prec, N->side); }));
      HIP_TRY(hipEventRecord(N->side_ev[l.level], N->side));
      outstanding.push_back(l.level);
      continue;
    }
    // the far updates of a level fork before its near ones: both read the
    // level's finished panels and add into disjoint ancestors, so the far
    // tiles fill the CUs the near launch leaves idle
    if (!one_stream && (l.kind == K_UPD_EXT || l.kind == K_UPD_RLB) && li + 1 < S.factor_plan.size() &&
        S.factor_plan[li + 1].side && S.factor_plan[li + 1].level == l.level) {
      HIP_TRY(hipEventRecord(N->fork_ev, st));
      forked = true;
    }
    // join: a side launch of level v must be done before level v + 2
    while (!outstanding.empty() && l.level >= outstanding.front() + 2) {
      HIP_TRY(hipStreamWaitEvent(st, N->side_ev[outstanding.front()], 0));
      outstanding.erase(outstanding.begin());
    }
    if (l.kind == K_SMALL) {
      HIP_TRY(timed_at(N, SPCHOL_KERNEL_FACTOR, l.level, 0, l.flops, l.bytes, st, [&] {
        return launch_small(D, N->L, l.off, l.ntasks, N->status, N->winv, prec, st);
      }));
    } else if (l.kind == K_MEDIUM) {
      HIP_TRY(timed_at(N, SPCHOL_KERNEL_FACTOR, l.level, 0, l.flops, l.bytes, st, [&] {
        return launch_medium(D, N->L, l.off, l.nfirst, l.ntasks, N->status, N->winv, st);
      }));
    } else if (l.kind == K_FACTOR_LA) {
      HIP_TRY(timed_at(N, SPCHOL_KERNEL_FACTOR, l.level, 0, l.flops, l.bytes, st, [&] {
        return launch_factor_la(D, N->L, l.off, l.nfirst, l.ntrsm, l.ntasks, N->status, N->winv, prec, st);
      }));
    } else if (l.kind == K_FACTOR || l.kind == K_TRSM) {
      const bool diag = l.kind == K_FACTOR;
      HIP_TRY(timed_at(N, SPCHOL_KERNEL_FACTOR, l.level, 0, l.flops, l.bytes, st, [&] {
        return launch_factor_panel(D, N->L, l.off, l.ntasks, N->status, N->winv, diag, st);
      }));
    } else {
      // deterministic schedule: an external launch's supernodes have
      // disjoint row lists, so its tiles read-modify-write (update kind 3)
      const int32_t uk = l.kind == K_UPD_RLB ? 4 : (l.kind == K_UPD_EXT && S.deterministic) ? 3 : l.kind;
      HIP_TRY(timed_at(N, l.kind == K_UPD_INT ? SPCHOL_KERNEL_UPDATE_INT : SPCHOL_KERNEL_UPDATE_EXT, l.level, 0,
                       l.flops, l.bytes, st,
                       [&] { return launch_update(D, N->L, uk, l.off, l.ntasks, prec, st); }));
    }
  }
  for (int64_t v : outstanding) HIP_TRY(hipStreamWaitEvent(st, N->side_ev[v], 0));
  // failure injection for tests of the error paths: SPCHOL_DEBUG_FAIL_AT=c
  // (1-based permuted column) reports a failed pivot at column c as if the
  // factorization had met one (read when the launches are enqueued)
  if (const char* ev = std::getenv("SPCHOL_DEBUG_FAIL_AT")) {
    const long long c = std::atoll(ev);
    if (c >= 1 && c <= S.n) HIP_TRY(launch_status_min(N->status, (unsigned long long)(c - 1), st));
  }
  return SPCHOL_OK;
}

// Read the pivot status word (synchronizes st).
static spchol_status read_info(spchol_num_s* N, hipStream_t st, int64_t* info) {
  unsigned long long h = 0;
  HIP_TRY(hipMemcpyAsync(&h, N->status, sizeof(h), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  int64_t inf = (h == ~0ULL) ? 0 : (int64_t)h + 1;
  if (info) *info = inf;
  if (inf) return fail(SPCHOL_ERR_NOT_SPD, "matrix is not positive definite at permuted column " + std::to_string(inf));
  return SPCHOL_OK;
}

// Permute, forward and backward supernodal solves, permute back, with the
// work vectors wy, wx, wacc (n x nrhs each; wacc zero on entry, left zero).
static spchol_status enqueue_solve(spchol_num_s* num, double* wy, double* wx, double* wacc, double* B_dev,
                                   int64_t nrhs, int64_t ldb, hipStream_t st) {
  const Symbolic& S = num->sym->S;
  const DevSym& D = num->sym->dev;
  const double pbytes = 24.0 * double(S.n) * double(nrhs);
  HIP_TRY(timed(num, SPCHOL_KERNEL_PERM, 0.0, pbytes, st,
                [&] { return launch_perm_gather(D, B_dev, ldb, nrhs, wy, st); }));
  // The solve of columns [c0, c0 + nr) of the block on stream s: the
  // forward and backward rounds, right-hand sides four at a time.
  auto chain = [&](int64_t c0, int64_t nr, hipStream_t s) -> hipError_t {
    double *y = wy + c0 * S.n, *x = wx + c0 * S.n, *acc = wacc + c0 * S.n;
    auto step = [&](const Launch& l) {
      // solve flops/bytes were counted for one right-hand side; L is read once
      const double fl = l.flops * double(nr);
      const double by = l.bytes;
      const bool fwd = l.kind == K_FWD || l.kind == K_FWD2 || l.kind == K_FWD_SMALL;
      return timed_at(num, fwd ? SPCHOL_KERNEL_FWD : SPCHOL_KERNEL_BWD, l.level, s == st ? 0 : 1, fl, by, s, [&] {
        return launch_solve_step(D, num->L, num->winv, l.kind, l.off, l.nfirst, l.ntasks, y, x, acc, nr, s);
      });
    };
    for (const Launch& l : S.fwd_plan) {
      hipError_t e = step(l);
      if (e != hipSuccess) return e;
    }
    for (const Launch& l : S.bwd_plan) {
      hipError_t e = step(l);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  // The rounds are latency-bound chains: more than four right-hand sides
  // go as groups of four, alternately on this stream and on the second one
  // (idle once the factorization is done), so that two chains run at once.
  const int64_t groups = (nrhs + 3) / 4;
  if (groups <= 1) {
    HIP_TRY(chain(0, nrhs, st));
  } else {
    HIP_TRY(hipEventRecord(num->fork_ev, st));
    HIP_TRY(hipStreamWaitEvent(num->side, num->fork_ev, 0));
    for (int64_t g = 0; g < groups; ++g)
      HIP_TRY(chain(4 * g, std::min<int64_t>(4, nrhs - 4 * g), (g & 1) ? num->side : st));
    HIP_TRY(hipEventRecord(num->join_ev, num->side));
    HIP_TRY(hipStreamWaitEvent(st, num->join_ev, 0));
  }
  HIP_TRY(timed(num, SPCHOL_KERNEL_PERM, 0.0, pbytes, st,
                [&] { return launch_perm_scatter(D, wx, nrhs, B_dev, ldb, st); }));
  return SPCHOL_OK;
}

// Residual and statistics buffers of the refinement (n x nrhs, 3 nrhs + 1).
static spchol_status ensure_refine_work(spchol_num_s* num, int64_t nrhs, hipStream_t st) {
  const int64_t n = num->sym->S.n;
  spchol_status s = grow(num, &num->rwork, &num->rcap, n * nrhs, st);
  if (s) return s;
  return grow(num, &num->stats, &num->scap, 3 * nrhs + 1, st);
}

// rwork <- B - A X (fp64, original A) and the normwise backward error per
// column, eta = ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf); expects
// stats[3 nrhs] to hold ||A||_inf.  Synchronizes st.
static spchol_status residual_eta(spchol_num_s* num, const double* vals, const double* B, int64_t ldb,
                                  const double* X, int64_t ldx, int64_t nrhs, hipStream_t st, double* eta) {
  std::vector<unsigned long long> h(3 * nrhs + 1);
  HIP_TRY(launch_residual(num->sym->dev, vals, B, ldb, X, ldx, nrhs, num->rwork, num->stats, st));
  HIP_TRY(hipMemcpyAsync(h.data(), num->stats, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  double an;
  std::memcpy(&an, &h[3 * nrhs], sizeof(double));
  for (int64_t c = 0; c < nrhs; ++c) {
    double r, x, b;
    std::memcpy(&r, &h[3 * c], sizeof(double));
    std::memcpy(&x, &h[3 * c + 1], sizeof(double));
    std::memcpy(&b, &h[3 * c + 2], sizeof(double));
    const double den = an * x + b;
    eta[c] = den > 0 ? r / den : (r > 0 ? INFINITY : 0.0);
  }
  return SPCHOL_OK;
}

// Enqueue a launch sequence through the graph cache: the first call with a
// given key runs eagerly, the second captures the sequence into a hipGraph,
// later ones replay it.  Eager when profiling (per-launch events), on the
// legacy null stream, or while the stream is itself being captured.
constexpr size_t kGraphCacheSize = 8;

template <class F>
static spchol_status cached_run(spchol_num_s* N, int kind, const void* ptr, int64_t a, int64_t b, hipStream_t st,
                                F&& enqueue) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (!N->gcache_on || N->prof.on || !st || hipStreamIsCapturing(st, &cs) != hipSuccess ||
      cs != hipStreamCaptureStatusNone)
    return enqueue();
  for (size_t i = 0; i < N->gcache.size(); ++i) {
    CachedGraph g = N->gcache[i];
    if (g.kind != kind || g.ptr != ptr || g.a != a || g.b != b) continue;
    N->gcache.erase(N->gcache.begin() + i);  // move to the back (most recent)
    if (!g.exec) {
      // second call: capture
      hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) {
        N->gcache.push_back(g);
        return enqueue();
      }
      spchol_status s = enqueue();
      hipError_t e2 = hipStreamEndCapture(st, &g.graph);
      if (s) {
        g.release();
        return s;
      }
      if (e2 == hipSuccess) e2 = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
      if (e2 != hipSuccess) {
        g.release();
        (void)hipGetLastError();
        N->gcache.push_back(g);
        return enqueue();  // capture failed: run eagerly
      }
    }
    N->gcache.push_back(g);
    HIP_TRY(hipGraphLaunch(g.exec, st));
    return SPCHOL_OK;
  }
  if (N->gcache.size() >= kGraphCacheSize) {
    N->gcache.front().release();
    N->gcache.erase(N->gcache.begin());
  }
  CachedGraph g;
  g.kind = kind;
  g.ptr = ptr;
  g.a = a;
  g.b = b;
  N->gcache.push_back(g);
  return enqueue();
}

// SPCHOL_TRACE=1: the factorization runs with per-launch events and, once
// it is done, prints one JSON line to stderr with the time, launches and
// algorithmic flops of every level of the schedule.
static void trace_levels(spchol_num_s* N) {
  struct Lv { int64_t launches = 0; double ms = 0, flops = 0; };
  std::vector<Lv> lv(N->sym->S.nlevels + 1);
  double other = 0;
  for (const Profiler::Rec& r : N->prof.recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
    if (r.level < 0 || r.level >= (int)lv.size()) { other += ms; continue; }
    lv[r.level].launches += 1;
    lv[r.level].ms += ms;
    lv[r.level].flops += r.flops;
  }
  std::string o = "{\"spchol_trace\": \"factor\", \"deterministic\": " +
                  std::string(N->sym->S.deterministic ? "true" : "false") + ", \"other_ms\": " + std::to_string(other) +
                  ", \"levels\": [";
  for (size_t l = 0; l < lv.size(); ++l) {
    if (!lv[l].launches) continue;
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s{\"level\": %zu, \"launches\": %lld, \"ms\": %.4f, \"gflops\": %.2f}",
                  o.back() == '[' ? "" : ", ", l, (long long)lv[l].launches, lv[l].ms,
                  lv[l].ms > 0 ? lv[l].flops / lv[l].ms / 1e6 : 0.0);
    o += buf;
  }
  o += "]}";
  std::fprintf(stderr, "%s\n", o.c_str());
}

static spchol_status run_factor(spchol_num_s* N, const double* vals, hipStream_t st, int64_t* info) {
  const char* tv = std::getenv("SPCHOL_TRACE");
  const bool trace = tv && std::atoi(tv) != 0 && !N->prof.on;
  if (trace) {
    N->prof.on = true;
    N->prof.recs.clear();
    N->prof.used = 0;
  }
  spchol_status s = cached_run(N, 0, vals, N->prec, 0, st, [&] { return enqueue_factor(N, vals, st); });
  if (trace) {
    N->prof.on = false;
    if (!s) trace_levels(N);
    N->prof.recs.clear();
    N->prof.used = 0;
  }
  if (s) return s;
  return read_info(N, st, info);
}

extern "C" {

const char* spchol_last_error(void) { return g_err.c_str(); }

const char* spchol_version(void) { return "spchol-mi355x 0.1"; }

spchol_status spchol_default_options(spchol_options* opt) {
  if (!opt) return fail(SPCHOL_ERR_ARG, "null options");
  opt->snode_mode = SPCHOL_SNODE_FUNDAMENTAL;
  opt->amalg_max_zeros = 0;
  opt->panel_width = 64;
  opt->deterministic = 0;
  opt->workspace_limit = 0;
  opt->amalg_rule = SPCHOL_AMALG_ZEROS;
  opt->amalg_cap_percent = 25;
  opt->update_method = SPCHOL_UPDATE_RL;
  opt->partition_refinement = 0;
  return SPCHOL_OK;
}

spchol_status spchol_order_nd(int64_t n, const int64_t* colptr, const int64_t* rowind, int64_t leaf_size,
                              uint64_t seed, int64_t* perm_out) {
  std::string err;
  const int rc = order_nd(n, colptr, rowind, leaf_size, seed, perm_out, err);
  if (rc) return fail((spchol_status)rc, err);
  return SPCHOL_OK;
}

spchol_status spchol_analyze(int64_t n, const int64_t* colptr, const int64_t* rowind, const int64_t* perm,
                             const spchol_options* opt, spchol_sym* out) {
  if (!out) return fail(SPCHOL_ERR_ARG, "null output handle");
  *out = nullptr;
  spchol_options o;
  spchol_default_options(&o);
  if (opt) o = *opt;
  if (o.workspace_limit < 0) return fail(SPCHOL_ERR_ARG, "workspace_limit < 0");
  {
    const char* ev = std::getenv("SPCHOL_DETERMINISTIC");
    if (ev && std::atoi(ev) != 0) o.deterministic = 1;
  }
  spchol_sym_s* h = new (std::nothrow) spchol_sym_s();
  if (!h) return fail(SPCHOL_ERR_OOM, "out of host memory");
  std::string err;
  AnalyzeOptions ao;
  ao.snode_mode = o.snode_mode;
  ao.amalg_max_zeros = o.amalg_max_zeros;
  ao.panel_width = o.panel_width;
  ao.deterministic = o.deterministic;
  ao.amalg_rule = o.amalg_rule;
  ao.amalg_cap_percent = o.amalg_cap_percent;
  ao.update_method = o.update_method;
  ao.partition_refinement = o.partition_refinement;
  int rc = analyze(n, colptr, rowind, perm, ao, h->S, err);
  if (rc) {
    delete h;
    return fail((spchol_status)rc, err);
  }
  h->ws_limit = o.workspace_limit;
  *out = h;
  return SPCHOL_OK;
}

spchol_status spchol_batch_analyze(int32_t count, const int64_t* n, const int64_t* const* colptr,
                                   const int64_t* const* rowind, const int64_t* const* perm,
                                   const spchol_options* opt, spchol_sym* out) {
  if (!out) return fail(SPCHOL_ERR_ARG, "null output handle");
  *out = nullptr;
  if (count < 0 || (count > 0 && (!n || !colptr || !rowind))) return fail(SPCHOL_ERR_ARG, "bad batch arguments");
  try {
    std::vector<int64_t> off(count + 1, 0), nzoff(count + 1, 0);
    for (int32_t b = 0; b < count; ++b) {
      if (n[b] < 0 || !colptr[b] || (n[b] > 0 && !rowind[b]))
        return fail(SPCHOL_ERR_ARG, "bad matrix " + std::to_string(b) + " in batch");
      off[b + 1] = off[b] + n[b];
      nzoff[b + 1] = nzoff[b] + colptr[b][n[b]];
    }
    const int64_t N = off[count];
    std::vector<int64_t> cp(N + 1, 0), ri(nzoff[count]), pm(N);
    for (int32_t b = 0; b < count; ++b) {
      for (int64_t j = 0; j < n[b]; ++j) cp[off[b] + j + 1] = nzoff[b] + colptr[b][j + 1];
      for (int64_t p = 0; p < colptr[b][n[b]]; ++p) ri[nzoff[b] + p] = off[b] + rowind[b][p];
      for (int64_t k = 0; k < n[b]; ++k) {
        const int64_t o = (perm && perm[b]) ? perm[b][k] : k;
        if (o < 0 || o >= n[b]) return fail(SPCHOL_ERR_ARG, "bad permutation of matrix " + std::to_string(b));
        pm[off[b] + k] = off[b] + o;
      }
    }
    spchol_status s = spchol_analyze(N, cp.data(), ri.data(), pm.data(), opt, out);
    if (s) return s;
    (*out)->batch_off = off;
    (*out)->batch_nzoff = nzoff;
    return SPCHOL_OK;
  } catch (const std::bad_alloc&) {
    return fail(SPCHOL_ERR_OOM, "out of host memory");
  }
}

spchol_status spchol_batch_info(spchol_sym sym, int32_t* count, int64_t* col_off, int64_t* nz_off) {
  if (!sym || !count) return fail(SPCHOL_ERR_ARG, "null argument");
  const int32_t c = sym->batch_off.empty() ? 1 : (int32_t)sym->batch_off.size() - 1;
  *count = c;
  if (col_off) {
    if (sym->batch_off.empty()) { col_off[0] = 0; col_off[1] = sym->S.n; }
    else std::memcpy(col_off, sym->batch_off.data(), sym->batch_off.size() * sizeof(int64_t));
  }
  if (nz_off) {
    if (sym->batch_nzoff.empty()) { nz_off[0] = 0; nz_off[1] = sym->S.nnzA; }
    else std::memcpy(nz_off, sym->batch_nzoff.data(), sym->batch_nzoff.size() * sizeof(int64_t));
  }
  return SPCHOL_OK;
}

spchol_status spchol_sym_info(spchol_sym sym, spchol_sym_info_t* info) {
  if (!sym || !info) return fail(SPCHOL_ERR_ARG, "null argument");
  const Symbolic& S = sym->S;
  info->n = S.n;
  info->nnz_a = S.nnzA;
  int64_t nz = 0;
  for (int64_t c : S.count) nz += c;
  info->nnz_l = nz;
  info->storage = S.loff[S.ns];
  info->nsuper = S.ns;
  info->nrows_total = S.rptr[S.ns];
  info->npairs = (int64_t)S.pJ.size();
  info->nrelind = (int64_t)S.tpos.size();
  info->nlevels = S.nlevels;
  info->max_k = S.max_k;
  info->max_m = S.max_m;
  info->flops_alg = S.flops_alg;
  info->flops_exec = S.flops_exec;
  return SPCHOL_OK;
}

spchol_status spchol_sym_export(spchol_sym sym, int64_t* parent, int64_t* count, int64_t* super_ptr,
                                int64_t* sparent, int64_t* row_ptr, int64_t* row_idx, int64_t* pair_J,
                                int64_t* pair_P, int64_t* pair_a0, int64_t* relind_ptr, int32_t* relind,
                                int64_t* level) {
  if (!sym) return fail(SPCHOL_ERR_ARG, "null handle");
  const Symbolic& S = sym->S;
  auto cp = [](int64_t* dst, const std::vector<int64_t>& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(int64_t));
  };
  cp(parent, S.parent);
  cp(count, S.count);
  cp(super_ptr, S.sptr);
  cp(sparent, S.sparent);
  cp(row_ptr, S.rptr);
  if (row_idx)
    for (size_t i = 0; i < S.rows.size(); ++i) row_idx[i] = S.rows[i];
  cp(pair_J, S.pJ);
  cp(pair_P, S.pP);
  cp(pair_a0, S.pa0);
  cp(relind_ptr, S.relptr);
  if (relind) {
    // device form is the position from the top; export the distance from the bottom
    for (size_t t = 0; t + 1 < S.relptr.size(); ++t) {
      int64_t P = S.pP[t];
      int64_t mP = S.rptr[P + 1] - S.rptr[P];
      for (int64_t q = S.relptr[t]; q < S.relptr[t + 1]; ++q) relind[q] = (int32_t)(mP - 1 - S.tpos[q]);
    }
  }
  cp(level, S.level);
  return SPCHOL_OK;
}

spchol_status spchol_sym_perm(spchol_sym sym, int64_t* perm_out) {
  if (!sym || !perm_out) return fail(SPCHOL_ERR_ARG, "null argument");
  if (!sym->S.perm.empty()) std::memcpy(perm_out, sym->S.perm.data(), sym->S.perm.size() * sizeof(int64_t));
  return SPCHOL_OK;
}

spchol_status spchol_sym_storage(spchol_sym sym, int64_t* storage_off) {
  if (!sym || !storage_off) return fail(SPCHOL_ERR_ARG, "null argument");
  std::memcpy(storage_off, sym->S.loff.data(), sym->S.loff.size() * sizeof(int64_t));
  return SPCHOL_OK;
}

spchol_status spchol_factor(spchol_sym sym, const double* vals_dev, void* stream, spchol_num* out,
                            int64_t* info) {
  return spchol_factor_prec(sym, vals_dev, SPCHOL_UPD_F64, stream, out, info);
}

spchol_status spchol_factor_prec(spchol_sym sym, const double* vals_dev, int32_t update_precision, void* stream,
                                 spchol_num* out, int64_t* info) {
  if (!sym || !out) return fail(SPCHOL_ERR_ARG, "null argument");
  if (update_precision != SPCHOL_UPD_F64 && update_precision != SPCHOL_UPD_F32 && update_precision != SPCHOL_UPD_BF16)
    return fail(SPCHOL_ERR_ARG, "unsupported update precision");
  if (!vals_dev && sym->S.nnzA > 0) return fail(SPCHOL_ERR_ARG, "null values");
  *out = nullptr;
  if (info) *info = 0;
  const int64_t storage = sym->S.loff[sym->S.ns];
  // device bytes of the new handle: the factor, the inverted diagonal
  // blocks, status and logdet partials, and the analysis' device copy;
  // checked against the workspace limit before anything is allocated
  const int64_t need = 8 * std::max<int64_t>(storage, 1) + 8 * std::max<int64_t>(sym->S.wbase[sym->S.ns], 1) +
                       8 + 8 * (logdet_partials(sym->S.n) + 1) + sym->device_bytes();
  if (sym->ws_limit > 0 && need > sym->ws_limit)
    return fail(SPCHOL_ERR_OOM, "workspace limit of " + std::to_string(sym->ws_limit) + " bytes: the factor needs " +
                                    std::to_string(need));
  spchol_status s = sym->ensure_device();
  if (s) return s;
  spchol_num_s* N = new (std::nothrow) spchol_num_s();
  if (!N) return fail(SPCHOL_ERR_OOM, "out of host memory");
  N->sym = sym;
  N->held = need;
  hipError_t e = hipMalloc((void**)&N->L, (size_t)(storage > 0 ? storage : 1) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&N->status, sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMalloc((void**)&N->red, (size_t)(logdet_partials(sym->S.n) + 1) * sizeof(double));
  if (e == hipSuccess)
    e = hipMalloc((void**)&N->winv, (size_t)(sym->S.wbase[sym->S.ns] > 0 ? sym->S.wbase[sym->S.ns] : 1) * sizeof(double));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&N->side, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&N->fork_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&N->join_ev, hipEventDisableTiming);
  if (e == hipSuccess) {
    N->side_ev.assign(sym->S.nlevels + 1, nullptr);
    for (hipEvent_t& ev : N->side_ev)
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    delete N;
    return fail(e == hipErrorOutOfMemory ? SPCHOL_ERR_OOM : SPCHOL_ERR_HIP,
                std::string("device allocation: ") + hipGetErrorString(e));
  }
  N->prec = update_precision;
  *out = N;
  return run_factor(N, vals_dev, (hipStream_t)stream, info);
}

// ---------------------------------------------------------------------------
// Host-resident factorization (the paper's architecture, Sec. III): the
// factor lives in caller-owned host memory; supernodes with k m below the
// threshold are factored and applied on the host; each other supernode is
// copied to the device, factored there by its panel rounds (the same
// kernels), copied back, and its update matrix is computed on the device in
// column blocks that fit the device budget, each copied back and added into
// the ancestors by the host.  Device memory: one supernode, its inverted
// diagonal blocks, one update block and the task lists (plus the analysis'
// device copy).
// ---------------------------------------------------------------------------

// Task lists of one supernode's numeric step on the device: per panel a
// diagonal task, the row tiles of the triangular solve and the trailing
// internal update tiles; then the update matrix's tiles by column block.
static void stream_plan(const Symbolic& S, int64_t J, int64_t wc, std::vector<DevTask>& tasks,
                        std::vector<std::pair<int32_t, std::pair<int64_t, int32_t>>>& launches) {
  const int64_t nb = S.nb, k = S.sptr[J + 1] - S.sptr[J], m = S.rptr[J + 1] - S.rptr[J];
  auto open = [&](int32_t kind) { launches.push_back({kind, {(int64_t)tasks.size(), 0}}); };
  auto close = [&] {
    auto& l = launches.back();
    l.second.second = (int32_t)((int64_t)tasks.size() - l.second.first);
    if (l.second.second == 0) launches.pop_back();
  };
  for (int64_t p = 0; p * nb < k; ++p) {
    const int64_t kp = std::min<int64_t>(nb, k - p * nb);
    open(K_FACTOR);
    tasks.push_back({(int32_t)J, (int32_t)p, (int32_t)m, 0});
    close();
    open(K_TRSM);
    for (int64_t r0 = p * nb + kp; r0 < m; r0 += kTile) tasks.push_back({(int32_t)J, (int32_t)p, (int32_t)r0, 0});
    close();
    open(K_UPD_INT);
    for (int64_t c0 = (p + 1) * nb; c0 < k; c0 += kTile)
      for (int64_t r0 = c0; r0 < m; r0 += kTile) tasks.push_back({(int32_t)J, (int32_t)r0, (int32_t)c0, (int32_t)p});
    close();
  }
  for (int64_t cb = k; cb < m; cb += wc) {
    open(-1);  // dense update block
    for (int64_t c0 = cb; c0 < std::min<int64_t>(cb + wc, m); c0 += kTile)
      for (int64_t r0 = c0; r0 < m; r0 += kTile) tasks.push_back({(int32_t)J, (int32_t)r0, (int32_t)c0, (int32_t)cb});
    close();
  }
}

spchol_status spchol_refactor(spchol_num num, const double* vals_dev, void* stream, int64_t* info) {
  if (!num) return fail(SPCHOL_ERR_ARG, "null handle");
  return spchol_refactor_prec(num, vals_dev, num->prec, stream, info);
}

spchol_status spchol_refactor_prec(spchol_num num, const double* vals_dev, int32_t update_precision, void* stream,
                                   int64_t* info) {
  if (!num) return fail(SPCHOL_ERR_ARG, "null handle");
  if (update_precision != SPCHOL_UPD_F64 && update_precision != SPCHOL_UPD_F32 && update_precision != SPCHOL_UPD_BF16)
    return fail(SPCHOL_ERR_ARG, "unsupported update precision");
  num->prec = update_precision;
  if (!vals_dev && num->sym->S.nnzA > 0) return fail(SPCHOL_ERR_ARG, "null values");
  if (info) *info = 0;
  spchol_status s = num->sym->ensure_device();
  if (s) return s;
  return run_factor(num, vals_dev, (hipStream_t)stream, info);
}

spchol_status spchol_factor_streamed(spchol_sym sym, const double* vals_host, const spchol_stream_options* opt,
                                     void* stream, double* L_host, int64_t* info, spchol_stream_stats* stats) {
  if (!sym || !L_host || (!vals_host && sym->S.nnzA > 0)) return fail(SPCHOL_ERR_ARG, "null argument");
  spchol_stream_options o{};
  o.device_budget = int64_t(256) << 20;
  o.host_threshold = 600000;
  if (opt) o = *opt;
  if (o.device_budget <= 0) o.device_budget = int64_t(256) << 20;
  if (o.host_threshold < 0) return fail(SPCHOL_ERR_ARG, "host_threshold < 0");
  int threads = o.host_threads > 0 ? o.host_threads : (int)std::max(1u, std::thread::hardware_concurrency());
  const Symbolic& S = sym->S;
  const int64_t nb = S.nb;
  if (info) *info = 0;
  spchol_stream_stats st{};
  auto on_gpu = [&](int64_t J) {
    const int64_t k = S.sptr[J + 1] - S.sptr[J], m = S.rptr[J + 1] - S.rptr[J];
    return k * m >= o.host_threshold;
  };
  // device buffers: the largest GPU supernode, its inverse blocks, an
  // update block of at least 64 columns, status
  int64_t maxst = 0, maxw = 0, maxr = 0;
  for (int64_t J = 0; J < S.ns; ++J) {
    if (!on_gpu(J)) continue;
    const int64_t k = S.sptr[J + 1] - S.sptr[J], m = S.rptr[J + 1] - S.rptr[J];
    maxst = std::max(maxst, k * m);
    maxw = std::max(maxw, S.wbase[J + 1] - S.wbase[J]);
    maxr = std::max(maxr, m - k);
  }
  const bool any_gpu = maxst > 0;
  const int64_t fixed = 8 * (maxst + maxw) + 8;
  const int64_t ubytes = o.device_budget - fixed;
  if (any_gpu && (ubytes < 8 * maxr * std::min<int64_t>(kTile, std::max<int64_t>(maxr, 1))))
    return fail(SPCHOL_ERR_OOM, "device budget of " + std::to_string(o.device_budget) +
                                    " bytes holds no supernode with one update block (needs " +
                                    std::to_string(fixed + 8 * maxr * kTile) + ")");
  try {
    host_scatter_values(S, vals_host, L_host);
    int64_t fail_col = -1;
    hipStream_t hs = (hipStream_t)stream;
    // device buffers of the call, freed on every way out
    struct Bufs {
      double *L = nullptr, *W = nullptr, *U = nullptr;
      unsigned long long* status = nullptr;
      DevTask* tasks = nullptr;
      ~Bufs() {
        for (void* q : {(void*)L, (void*)W, (void*)U, (void*)status, (void*)tasks})
          if (q) (void)hipFree(q);
      }
    } bufs;
    double *&dL = bufs.L, *&dW = bufs.W, *&dU = bufs.U;
    unsigned long long*& dstatus = bufs.status;
    DevTask*& dtasks = bufs.tasks;
    spchol_status status = SPCHOL_OK;
    DevSym D{};
    std::vector<double> hU;
    if (any_gpu) {
      spchol_status s = sym->ensure_device();
      if (s) return s;
      D = sym->dev;
      // the update block: as many 64-column groups as the budget holds
      // for the tallest supernode
      const int64_t wc_all = std::max<int64_t>(kTile, (ubytes / 8 / std::max<int64_t>(maxr, 1)) / kTile * kTile);
      HIP_TRY(hipMalloc((void**)&dL, (size_t)maxst * 8));
      HIP_TRY(hipMalloc((void**)&dW, (size_t)std::max<int64_t>(maxw, 1) * 8));
      HIP_TRY(hipMalloc((void**)&dU, (size_t)std::max<int64_t>(maxr * std::min(wc_all, maxr), 1) * 8));
      HIP_TRY(hipMalloc((void**)&dstatus, sizeof(unsigned long long)));
      st.device_bytes = 8 * (maxst + std::max<int64_t>(maxw, 1) + maxr * std::min(wc_all, maxr)) + 8;
      HIP_TRY(launch_status_init(dstatus, hs));
      hU.resize((size_t)(maxr * std::min(wc_all, maxr)));
      std::vector<DevTask> tasks;
      std::vector<std::pair<int32_t, std::pair<int64_t, int32_t>>> launches;
      std::vector<int64_t> wcol(S.ns, kTile);  // update block width (columns) per supernode
      std::vector<std::vector<std::pair<int32_t, std::pair<int64_t, int32_t>>>> plan(S.ns);
      for (int64_t J = 0; J < S.ns; ++J) {
        if (!on_gpu(J)) continue;
        const int64_t k = S.sptr[J + 1] - S.sptr[J], m = S.rptr[J + 1] - S.rptr[J];
        const int64_t r = m - k;
        wcol[J] = std::max<int64_t>(kTile, r > 0 ? std::min(wc_all, (r + kTile - 1) / kTile * kTile) : kTile);
        stream_plan(S, J, wcol[J], tasks, plan[J]);
      }
      HIP_TRY(hipMalloc((void**)&dtasks, std::max<size_t>(tasks.size(), 1) * sizeof(DevTask)));
      HIP_TRY(hipMemcpy(dtasks, tasks.data(), tasks.size() * sizeof(DevTask), hipMemcpyHostToDevice));
      st.device_bytes += (int64_t)(std::max<size_t>(tasks.size(), 1) * sizeof(DevTask));
      D.tasks = dtasks;
      for (int64_t J = 0; J < S.ns; ++J) {
        const int64_t k = S.sptr[J + 1] - S.sptr[J], m = S.rptr[J + 1] - S.rptr[J];
        if (!on_gpu(J)) {
          const int64_t f = host_factor_supernode(S, J, L_host);
          if (f >= 0 && (fail_col < 0 || f < fail_col)) fail_col = f;
          host_update_supernode(S, J, L_host, threads);
          st.host_supernodes += 1;
          continue;
        }
        // the supernode to the device (its updates from descendants are in)
        double* base = dL - S.loff[J];  // kernels address L + loff[J] + ...
        double* wb = dW - S.wbase[J];
        HIP_TRY(hipMemcpyAsync(dL, L_host + S.loff[J], (size_t)(k * m) * 8, hipMemcpyHostToDevice, hs));
        st.h2d_bytes += 8 * k * m;
        for (const auto& l : plan[J]) {
          const int32_t kind = l.first;
          const int64_t off = l.second.first;
          const int32_t nt = l.second.second;
          if (kind == K_FACTOR || kind == K_TRSM) {
            HIP_TRY(launch_factor_panel(D, base, off, nt, dstatus, wb, kind == K_FACTOR, hs));
          } else if (kind == K_UPD_INT) {
            HIP_TRY(launch_update(D, base, 1, off, nt, 0, hs));
          } else {
            // an update column block: compute, copy back, add on the host
            const int64_t cb = tasks[off].c;
            const int64_t ce = std::min<int64_t>(m, cb + wcol[J]);
            const int64_t ldu = m - cb;
            HIP_TRY(launch_update_dense(D, base, off, nt, dU, hs));
            HIP_TRY(hipMemcpyAsync(hU.data(), dU, (size_t)(ldu * (ce - cb)) * 8, hipMemcpyDeviceToHost, hs));
            HIP_TRY(hipStreamSynchronize(hs));
            st.d2h_bytes += 8 * ldu * (ce - cb);
            host_assemble_block(S, J, cb, ce, hU.data(), L_host, threads);
            st.update_blocks += 1;
          }
        }
        // the factored supernode back to the host
        HIP_TRY(hipMemcpyAsync(L_host + S.loff[J], dL, (size_t)(k * m) * 8, hipMemcpyDeviceToHost, hs));
        HIP_TRY(hipStreamSynchronize(hs));
        st.d2h_bytes += 8 * k * m;
        st.gpu_supernodes += 1;
      }
      unsigned long long hstat = ~0ULL;
      HIP_TRY(hipMemcpy(&hstat, dstatus, sizeof(hstat), hipMemcpyDeviceToHost));
      if (hstat != ~0ULL && (fail_col < 0 || (int64_t)hstat < fail_col)) fail_col = (int64_t)hstat;
    } else {
      // every supernode below the threshold: no device work at all
      for (int64_t J = 0; J < S.ns; ++J) {
        const int64_t f = host_factor_supernode(S, J, L_host);
        if (f >= 0 && (fail_col < 0 || f < fail_col)) fail_col = f;
        host_update_supernode(S, J, L_host, threads);
        st.host_supernodes += 1;
      }
    }
    st.host_threads = threads;
    if (stats) *stats = st;
    if (fail_col >= 0) {
      if (info) *info = fail_col + 1;
      return fail(SPCHOL_ERR_NOT_SPD, "matrix is not positive definite at permuted column " + std::to_string(fail_col + 1));
    }
    (void)nb;
    (void)status;
    return SPCHOL_OK;
  } catch (const std::bad_alloc&) {
    return fail(SPCHOL_ERR_OOM, "out of host memory");
  }
}

spchol_status spchol_solve(spchol_num num, double* B_dev, int64_t nrhs, int64_t ldb, void* stream) {
  if (!num) return fail(SPCHOL_ERR_ARG, "null handle");
  const Symbolic& S = num->sym->S;
  if (nrhs < 0 || ldb < S.n || ldb < 1) return fail(SPCHOL_ERR_ARG, "bad nrhs or ldb");
  if (nrhs == 0 || S.n == 0) return SPCHOL_OK;
  if (!B_dev) return fail(SPCHOL_ERR_ARG, "null right-hand side");
  hipStream_t st = (hipStream_t)stream;
  bool moved = false;
  if (num->sw.cap < S.n * nrhs || !num->sw.acc) {
    const int64_t nb = SolveWork::bytes_for(S.n, nrhs), ob = num->sw.bytes();
    spchol_status s = ws_check(num, nb - ob);
    if (s) return s;
    HIP_TRY(num->sw.ensure(S.n, nrhs, st, &moved));
    num->held += nb - ob;
  }
  if (moved) num->drop_graphs(1);  // captured solves hold the old work vectors
  return cached_run(num, 1, B_dev, nrhs, ldb, st, [&] {
    return enqueue_solve(num, num->sw.y, num->sw.x, num->sw.acc, B_dev, nrhs, ldb, st);
  });
}

spchol_status spchol_solve_noalloc(spchol_num num, double* B_dev, int64_t nrhs, int64_t ldb, void* stream) {
  if (!num) return fail(SPCHOL_ERR_ARG, "null handle");
  const Symbolic& S = num->sym->S;
  if (nrhs < 0 || ldb < S.n || ldb < 1) return fail(SPCHOL_ERR_ARG, "bad nrhs or ldb");
  if (nrhs == 0 || S.n == 0) return SPCHOL_OK;
  if (!B_dev) return fail(SPCHOL_ERR_ARG, "null right-hand side");
  if (nrhs > kScratchSlice / S.n)
    return fail(SPCHOL_ERR_ARG, "n * nrhs = " + std::to_string(S.n) + " * " + std::to_string(nrhs) +
                                    " exceeds the static solve workspace (" + std::to_string(kScratchSlice) +
                                    " entries)");
  int cur = 0;
  HIP_TRY(hipGetDevice(&cur));
  if (!num->sym->uploaded || cur != num->sym->device)
    return fail(SPCHOL_ERR_ARG, "the factor lives on another device");
  double* base = nullptr;
  spchol_status s = scratch_address(&base);
  if (s) return s;
  double *y = base, *x = base + kScratchSlice, *acc = base + 2 * kScratchSlice;
  hipStream_t st = (hipStream_t)stream;
  // the array keeps whatever the last call left: clear the accumulators
  HIP_TRY(launch_fill(acc, S.n * nrhs, 0.0, st));
  // no per-launch events (creating them may allocate)
  const bool prof = num->prof.on;
  num->prof.on = false;
  s = enqueue_solve(num, y, x, acc, B_dev, nrhs, ldb, st);
  num->prof.on = prof;
  return s;
}

// Preconditioned conjugate gradients on A (fp64, original ordering) with
// M = L~ L~^T, the stored factor (symmetric positive definite whatever the
// update precision, once the factorization succeeded), from the current X,
// whose residual rwork holds; the path iterative refinement switches to when
// it stalls.  Per column: z = M^{-1} r, p = z, then alpha = r.z / p.Ap,
// x += alpha p, r = b - A x (recomputed, with eta), z = M^{-1} r,
// beta = r.z (new) / r.z (old), p = z + beta p.  A column whose r.z or p.Ap
// is zero or not finite keeps its iterate (its scalars are zero).  Runs
// until every eta <= tol or `budget` iterations; adds them to *it.
static spchol_status pcg(spchol_num_s* num, const double* vals, const double* B, int64_t ldb, double* X, int64_t ldx,
                         int64_t nrhs, double tol, int32_t budget, hipStream_t st, std::vector<double>& eta,
                         int32_t* it, bool* ok) {
  const int64_t n = num->sym->S.n, blk = n * nrhs;
  {
    spchol_status s0 = grow(num, &num->pwork, &num->pcap, 3 * blk + 3 * nrhs, st);
    if (s0) return s0;
  }
  double *z = num->pwork, *pv = z + blk, *q = pv + blk, *dots = q + blk, *scal = dots + nrhs;
  std::vector<double> rz(nrhs), h(nrhs), a(nrhs);
  auto precond = [&]() -> spchol_status {  // z = M^{-1} r, h = r.z
    HIP_TRY(launch_copy_cols(z, n, num->rwork, n, n, nrhs, st));
    spchol_status s = spchol_solve(num, z, nrhs, n, st);
    if (s) return s;
    HIP_TRY(launch_dot_cols(num->rwork, z, n, nrhs, dots, st));
    HIP_TRY(hipMemcpyAsync(h.data(), dots, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return SPCHOL_OK;
  };
  auto upload = [&](const std::vector<double>& v) -> spchol_status {
    HIP_TRY(hipMemcpyAsync(scal, v.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));  // v is pageable host memory
    return SPCHOL_OK;
  };
  auto usable = [](double v) { return std::isfinite(v) && v != 0.0; };
  spchol_status s = precond();
  if (s) return s;
  rz = h;
  HIP_TRY(launch_copy_cols(pv, n, z, n, n, nrhs, st));
  for (int32_t k = 0; k < budget; ++k) {
    // q = -A p, h = p.q = -p.Ap
    HIP_TRY(launch_residual(num->sym->dev, vals, nullptr, n, pv, n, nrhs, q, num->stats, st));
    HIP_TRY(launch_dot_cols(pv, q, n, nrhs, dots, st));
    HIP_TRY(hipMemcpyAsync(h.data(), dots, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int64_t c = 0; c < nrhs; ++c) a[c] = (usable(rz[c]) && usable(h[c])) ? -rz[c] / h[c] : 0.0;
    if ((s = upload(a))) return s;
    HIP_TRY(launch_axpy_cols(X, ldx, pv, n, nrhs, scal, st));
    ++*it;
    if ((s = residual_eta(num, vals, B, ldb, X, ldx, nrhs, st, eta.data()))) return s;
    *ok = true;
    for (int64_t c = 0; c < nrhs; ++c)
      if (!(eta[c] <= tol)) *ok = false;
    if (*ok || k + 1 == budget) break;
    if ((s = precond())) return s;
    for (int64_t c = 0; c < nrhs; ++c) {
      a[c] = (usable(rz[c]) && std::isfinite(h[c])) ? h[c] / rz[c] : 0.0;
      rz[c] = h[c];
    }
    if ((s = upload(a))) return s;
    HIP_TRY(launch_xpby_cols(pv, z, n, nrhs, scal, st));
  }
  return SPCHOL_OK;
}

spchol_status spchol_refine(spchol_num num, const double* vals_dev, const double* B_dev, double* X_dev,
                            int64_t nrhs, int64_t ldb, int64_t ldx, double tol, int32_t max_iter, void* stream,
                            double* berr_out, int32_t* iters_out, int32_t* path_out) {
  if (!num) return fail(SPCHOL_ERR_ARG, "null handle");
  const Symbolic& S = num->sym->S;
  if (nrhs < 0 || ldb < S.n || ldx < S.n || ldb < 1 || ldx < 1 || max_iter < 0)
    return fail(SPCHOL_ERR_ARG, "bad nrhs, leading dimension or max_iter");
  if (iters_out) *iters_out = 0;
  if (path_out) *path_out = 0;
  if (nrhs == 0 || S.n == 0) {
    for (int64_t c = 0; c < nrhs; ++c)
      if (berr_out) berr_out[c] = 0.0;
    return SPCHOL_OK;
  }
  if (!vals_dev || !B_dev || !X_dev) return fail(SPCHOL_ERR_ARG, "null device pointer");
  hipStream_t st = (hipStream_t)stream;
  const DevSym& D = num->sym->dev;
  {
    spchol_status s = ensure_refine_work(num, nrhs, st);
    if (s) return s;
  }
  unsigned long long* anorm = num->stats + 3 * nrhs;
  // x0 = A~^{-1} b
  HIP_TRY(launch_copy_cols(X_dev, ldx, B_dev, ldb, S.n, nrhs, st));
  if (ldx == S.n) {
    spchol_status s = spchol_solve(num, X_dev, nrhs, ldx, stream);
    if (s) return s;
  } else {
    HIP_TRY(launch_copy_cols(num->rwork, S.n, X_dev, ldx, S.n, nrhs, st));
    spchol_status s = spchol_solve(num, num->rwork, nrhs, S.n, stream);
    if (s) return s;
    HIP_TRY(launch_copy_cols(X_dev, ldx, num->rwork, S.n, S.n, nrhs, st));
  }
  HIP_TRY(launch_anorm(D, vals_dev, anorm, st));
  std::vector<double> eta(nrhs, 0.0), prev(nrhs, INFINITY);
  int32_t it = 0, path = 0;
  bool ok = false;
  for (;; ++it) {
    {
      spchol_status s = residual_eta(num, vals_dev, B_dev, ldb, X_dev, ldx, nrhs, st, eta.data());
      if (s) return s;
    }
    ok = true;
    bool stall = false;
    for (int64_t c = 0; c < nrhs; ++c) {
      if (!(eta[c] <= tol)) ok = false;
      // a correction that did not halve the backward error of a column
      // still above the tolerance (or made it worse, or not finite)
      if (it > 0 && !(eta[c] <= tol) && !(eta[c] <= 0.5 * prev[c])) stall = true;
    }
    if (ok || it >= max_iter) break;
    if (stall) {
      // the remaining corrections as preconditioned conjugate gradients
      path = 1;
      spchol_status s = pcg(num, vals_dev, B_dev, ldb, X_dev, ldx, nrhs, tol, max_iter - it, st, eta, &it, &ok);
      if (s) return s;
      break;
    }
    prev = eta;
    spchol_status s = spchol_solve(num, num->rwork, nrhs, S.n, stream);
    if (s) return s;
    HIP_TRY(launch_axpy(X_dev, ldx, num->rwork, S.n, nrhs, st));
  }
  if (berr_out)
    for (int64_t c = 0; c < nrhs; ++c) berr_out[c] = eta[c];
  if (iters_out) *iters_out = it;
  if (path_out) *path_out = path;
  if (!ok) return fail(SPCHOL_ERR_NOCONV, "iterative refinement did not reach the tolerance");
  return SPCHOL_OK;
}

spchol_status spchol_berr(spchol_num num, const double* vals_dev, const double* B_dev, const double* X_dev,
                          int64_t nrhs, int64_t ldb, int64_t ldx, void* stream, double* berr_out) {
  if (!num || !berr_out) return fail(SPCHOL_ERR_ARG, "null argument");
  const Symbolic& S = num->sym->S;
  if (nrhs < 0 || ldb < S.n || ldx < S.n || ldb < 1 || ldx < 1) return fail(SPCHOL_ERR_ARG, "bad nrhs or leading dimension");
  if (nrhs == 0 || S.n == 0) {
    for (int64_t c = 0; c < nrhs; ++c) berr_out[c] = 0.0;
    return SPCHOL_OK;
  }
  if (!vals_dev || !B_dev || !X_dev) return fail(SPCHOL_ERR_ARG, "null device pointer");
  hipStream_t st = (hipStream_t)stream;
  spchol_status s = ensure_refine_work(num, nrhs, st);
  if (s) return s;
  HIP_TRY(launch_anorm(num->sym->dev, vals_dev, num->stats + 3 * nrhs, st));
  return residual_eta(num, vals_dev, B_dev, ldb, X_dev, ldx, nrhs, st, berr_out);
}

static spchol_status run_selinv(spchol_num_s* N, hipStream_t st) {
  const Symbolic& S = N->sym->S;
  const DevSym& D = N->sym->dev;
  const int64_t storage = S.loff[S.ns];
  const int64_t blk = (int64_t)kMaxPanel * kMaxPanel;
  const int64_t ws = S.si_max_y + S.si_max_slots * blk;
  if (!N->Z || !N->sibuf) {
    spchol_status s = ws_check(N, 8 * (std::max<int64_t>(storage, 1) + std::max<int64_t>(ws, 1)));
    if (s) return s;
    if ((s = grow(N, &N->Z, &N->zcap, storage, st))) return s;
    if ((s = grow(N, &N->sibuf, &N->sicap, ws, st))) return s;
    // Z: zero once (the selected inversion writes the lower part of every
    // block; above the diagonal of the diagonal blocks stays zero, as in L).
    // Y blocks and T accumulators: zero here (kernels, stream-ordered), and
    // left zero by their readers
    HIP_TRY(launch_fill(N->Z, std::max<int64_t>(storage, 1), 0.0, st));
    HIP_TRY(launch_fill(N->sibuf, std::max<int64_t>(ws, 1), 0.0, st));
  }
  double* ybuf = N->sibuf;
  double* tbuf = ybuf + S.si_max_y;
  // the launch sequence (kernels only: the Y blocks and T accumulators are
  // left zero by their readers) goes through the graph cache like the
  // factorization and the solves
  return cached_run(N, 2, N->Z, 0, 0, st, [&]() -> spchol_status {
    for (const Launch& l : S.si_plan) {
      const int64_t* yoff = N->sym->si_yoff + l.slot_base;
      HIP_TRY(timed(N, SPCHOL_KERNEL_SELINV, 0.0, 0.0, st, [&] {
        return launch_si(D, l.kind, l.off, l.ntasks, N->L, N->winv, N->Z, yoff, ybuf, tbuf, l.seg, st);
      }));
    }
    return SPCHOL_OK;
  });
}

spchol_status spchol_backward(spchol_num num, const double* X_dev, const double* Xbar_dev, int64_t nrhs,
                              int64_t ld, double gbar_logdet, double* Abar_dev, double* Bbar_dev, void* stream) {
  if (!num || !Abar_dev) return fail(SPCHOL_ERR_ARG, "null argument");
  const Symbolic& S = num->sym->S;
  if (nrhs < 0 || (nrhs > 0 && (ld < S.n || ld < 1))) return fail(SPCHOL_ERR_ARG, "bad nrhs or leading dimension");
  if (nrhs > 0 && Xbar_dev && !X_dev) return fail(SPCHOL_ERR_ARG, "X is needed with Xbar");
  hipStream_t st = (hipStream_t)stream;
  const DevSym& D = num->sym->dev;
  const bool use_lam = nrhs > 0 && Xbar_dev != nullptr && S.n > 0;
  if (use_lam) {
    {
      spchol_status s0 = grow(num, &num->lam, &num->lcap, S.n * nrhs, st);
      if (s0) return s0;
    }
    HIP_TRY(launch_copy_cols(num->lam, S.n, Xbar_dev, ld, S.n, nrhs, st));
    spchol_status s = spchol_solve(num, num->lam, nrhs, S.n, stream);
    if (s) return s;
    if (Bbar_dev) HIP_TRY(launch_copy_cols(Bbar_dev, ld, num->lam, S.n, S.n, nrhs, st));
  }
  const bool use_z = gbar_logdet != 0.0 && S.n > 0;
  if (use_z) {
    spchol_status s = run_selinv(num, st);
    if (s) return s;
  }
  // X may have a leading dimension other than n: lam uses n, X uses ld;
  // k_abar indexes both with one leading dimension, so copy X when they differ
  const double* Xc = X_dev;
  if (use_lam && ld != S.n) {
    double* tmp = nullptr;
    HIP_TRY(hipMallocAsync((void**)&tmp, (size_t)(S.n * nrhs) * sizeof(double), st));
    HIP_TRY(launch_copy_cols(tmp, S.n, X_dev, ld, S.n, nrhs, st));
    HIP_TRY(launch_abar(D, use_z ? num->Z : nullptr, gbar_logdet, tmp, num->lam, S.n, nrhs, Abar_dev, st));
    HIP_TRY(hipFreeAsync(tmp, st));
  } else {
    HIP_TRY(launch_abar(D, use_z ? num->Z : nullptr, gbar_logdet, Xc, use_lam ? num->lam : nullptr, S.n,
                        use_lam ? nrhs : 0, Abar_dev, st));
  }
  return SPCHOL_OK;
}

spchol_status spchol_selinv_export(spchol_num num, double* dst_dev, void* stream) {
  if (!num || !dst_dev) return fail(SPCHOL_ERR_ARG, "null argument");
  hipStream_t st = (hipStream_t)stream;
  spchol_status s = run_selinv(num, st);
  if (s) return s;
  const int64_t storage = num->sym->S.loff[num->sym->S.ns];
  if (storage > 0)
    HIP_TRY(hipMemcpyAsync(dst_dev, num->Z, (size_t)storage * sizeof(double), hipMemcpyDeviceToDevice, st));
  return SPCHOL_OK;
}

spchol_status spchol_logdet(spchol_num num, double* out_host, void* stream) {
  if (!num || !out_host) return fail(SPCHOL_ERR_ARG, "null argument");
  hipStream_t st = (hipStream_t)stream;
  const DevSym& D = num->sym->dev;
  const int32_t np = logdet_partials(num->sym->S.n);
  HIP_TRY(timed(num, SPCHOL_KERNEL_LOGDET, 0.0, 8.0 * double(num->sym->S.n), st,
                [&] { return launch_logdet(D, num->L, num->red, np, num->red + np, st); }));
  HIP_TRY(hipMemcpyAsync(out_host, num->red + np, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return SPCHOL_OK;
}

spchol_status spchol_logdet_batch(spchol_num num, double* out_dev, void* stream) {
  if (!num || !out_dev) return fail(SPCHOL_ERR_ARG, "null argument");
  const int32_t count = num->sym->batch_off.empty() ? 1 : (int32_t)num->sym->batch_off.size() - 1;
  HIP_TRY(timed(num, SPCHOL_KERNEL_LOGDET, 0.0, 8.0 * double(num->sym->S.n), (hipStream_t)stream, [&] {
    return launch_logdet_segments(num->sym->dev, num->L, num->sym->dev_batch_off, count, out_dev,
                                  (hipStream_t)stream);
  }));
  return SPCHOL_OK;
}

spchol_status spchol_info(spchol_num num, int64_t* info, void* stream) {
  if (!num) return fail(SPCHOL_ERR_ARG, "null handle");
  int64_t v = 0;
  spchol_status s = read_info(num, (hipStream_t)stream, &v);
  if (info) *info = v;
  return s;
}

struct spchol_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  SolveWork sw;  // the captured solve's own work vectors
  ~spchol_graph_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

spchol_status spchol_graph_create(spchol_num num, const double* vals_dev, double* B_dev, int64_t nrhs, int64_t ldb,
                                  void* stream, spchol_graph* out) {
  if (!num || !out) return fail(SPCHOL_ERR_ARG, "null argument");
  *out = nullptr;
  const Symbolic& S = num->sym->S;
  if (nrhs < 0 || (nrhs > 0 && (!B_dev || ldb < S.n || ldb < 1))) return fail(SPCHOL_ERR_ARG, "bad right-hand side");
  if (!vals_dev && nrhs == 0) return fail(SPCHOL_ERR_ARG, "nothing to capture");
  hipStream_t st = (hipStream_t)stream;
  if (!st) return fail(SPCHOL_ERR_ARG, "graph capture needs a non-null stream");
  spchol_graph_s* G = new (std::nothrow) spchol_graph_s();
  if (!G) return fail(SPCHOL_ERR_OOM, "out of host memory");
  // buffers the captured work uses must exist before the capture; the graph
  // owns its solve vector so that later eager solves cannot move it
  if (nrhs > 0 && S.n > 0) {
    const int64_t nb = SolveWork::bytes_for(S.n, nrhs);
    spchol_status s0 = ws_check(num, nb);
    if (s0) {
      delete G;
      return s0;
    }
    hipError_t ea = G->sw.ensure(S.n, nrhs, st);
    // the graph may be replayed on any stream: its buffers must exist first
    if (ea == hipSuccess) ea = hipStreamSynchronize(st);
    if (ea != hipSuccess) {
      delete G;
      return fail(SPCHOL_ERR_OOM, std::string("graph work vectors: ") + hipGetErrorString(ea));
    }
  }
  const bool prof = num->prof.on;
  num->prof.on = false;
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  spchol_status s = SPCHOL_OK;
  if (e == hipSuccess) {
    if (vals_dev || S.nnzA == 0) s = enqueue_factor(num, vals_dev, st);
    if (!s && nrhs > 0 && S.n > 0) s = enqueue_solve(num, G->sw.y, G->sw.x, G->sw.acc, B_dev, nrhs, ldb, st);
    hipError_t e2 = hipStreamEndCapture(st, &G->graph);
    if (!s && e2 != hipSuccess) e = e2;
  }
  num->prof.on = prof;
  if (s) {
    delete G;
    return s;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    delete G;
    return fail(SPCHOL_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
  }
  *out = G;
  return SPCHOL_OK;
}

spchol_status spchol_graph_launch(spchol_graph graph, void* stream) {
  if (!graph) return fail(SPCHOL_ERR_ARG, "null graph");
  HIP_TRY(hipGraphLaunch(graph->exec, (hipStream_t)stream));
  return SPCHOL_OK;
}

void spchol_graph_destroy(spchol_graph graph) { delete graph; }

spchol_status spchol_num_export(spchol_num num, double* dst_dev, void* stream) {
  if (!num || !dst_dev) return fail(SPCHOL_ERR_ARG, "null argument");
  const int64_t storage = num->sym->S.loff[num->sym->S.ns];
  if (storage == 0) return SPCHOL_OK;
  HIP_TRY(hipMemcpyAsync(dst_dev, num->L, (size_t)storage * sizeof(double), hipMemcpyDeviceToDevice,
                         (hipStream_t)stream));
  return SPCHOL_OK;
}

spchol_status spchol_profile(spchol_num num, int32_t enable) {
  if (!num) return fail(SPCHOL_ERR_ARG, "null handle");
  if (enable < 0 || enable > 2) return fail(SPCHOL_ERR_ARG, "profile mode must be 0, 1 or 2");
  num->prof.on = enable != 0;
  num->prof.serial = enable == 2;
  if (num->prof.on) {
    num->prof.recs.clear();
    num->prof.used = 0;
  }
  return SPCHOL_OK;
}

spchol_status spchol_profile_read(spchol_num num, spchol_kernel_stat* out) {
  if (!num || !out) return fail(SPCHOL_ERR_ARG, "null argument");
  for (int k = 0; k < SPCHOL_KERNEL_KINDS; ++k) out[k] = spchol_kernel_stat{0, 0.0, 0.0, 0.0};
  for (const Profiler::Rec& r : num->prof.recs) {
    HIP_TRY(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    spchol_kernel_stat& s = out[r.kind];
    s.launches += 1;
    s.ms += ms;
    s.flops += r.flops;
    s.bytes += r.bytes;
  }
  num->prof.recs.clear();
  num->prof.used = 0;
  return SPCHOL_OK;
}

spchol_status spchol_profile_launches(spchol_num num, spchol_launch_record* out, int64_t cap, int64_t* count) {
  if (!num || !count || cap < 0) return fail(SPCHOL_ERR_ARG, "null argument or negative capacity");
  *count = (int64_t)num->prof.recs.size();
  if (!out) return SPCHOL_OK;
  const int64_t nout = std::min<int64_t>(cap, *count);
  for (int64_t q = 0; q < nout; ++q) {
    const Profiler::Rec& r = num->prof.recs[q];
    HIP_TRY(hipEventSynchronize(r.b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, r.a, r.b));
    out[q] = spchol_launch_record{r.kind, r.level, r.side, 0, ms, r.flops, r.bytes};
  }
  num->prof.recs.clear();
  num->prof.used = 0;
  return SPCHOL_OK;
}

void spchol_sym_destroy(spchol_sym sym) { delete sym; }
void spchol_num_destroy(spchol_num num) { delete num; }

}  // extern "C"
