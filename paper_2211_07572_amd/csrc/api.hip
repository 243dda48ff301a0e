// C ABI of the slab solver: argument checks, device memory of handles and
// batches, and the orchestration of Alg. 3 (factor) and Alg. 4 (solve) with
// FP64 iterative refinement around the working-precision solve.
//
// Every factorization and solve is planned for a group of problems (a single
// problem is a group of one): the planners record grouped launches, the plan's
// descriptor tables go to the device in one copy, and the launches are issued
// in order.  Batched solves can capture a refinement pass into a HIP graph and
// replay it.
#include "launch.h"

#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <vector>

namespace slab {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace slab

using namespace slab;

namespace {

// Caching device allocator.  Mapping fresh device memory costs far more than
// the factorization of a small problem (tens of GB for a large batch), so
// blocks released by a handle, a batch or a finished factorization are kept
// per device and handed out again for requests of about the same size.  A
// failed hipMalloc empties the cache and retries; slab_release_cache() empties
// it on request.  Blocks are released only after the work using them is
// finished (every entry point synchronizes before it releases).
class Pool {
 public:
  static Pool& get() {
    static Pool p;
    return p;
  }
  hipError_t alloc(void** p, size_t n) {
    n = round(n);
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto& fb = free_[dev];
      auto it = fb.lower_bound(n);
      if (it != fb.end() && it->first <= n + std::max<size_t>(n / 8, 2 << 20)) {
        *p = it->second;
        size_[*p] = it->first;
        cached_ -= it->first;
        fb.erase(it);
        return hipSuccess;
      }
    }
    hipError_t e = hipMalloc(p, n);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      trim(dev);
      e = hipMalloc(p, n);
    }
    if (e == hipSuccess) {
      std::lock_guard<std::mutex> lk(mu_);
      size_[*p] = n;
      dev_[*p] = dev;
    }
    return e;
  }
  void release(void* p) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = size_.find(p);
    if (it == size_.end()) return;
    const size_t n = it->second;
    size_.erase(it);
    free_[dev_[p]].insert({n, p});
    cached_ += n;
  }
  void trim(int dev) {
    std::lock_guard<std::mutex> lk(mu_);
    auto& fb = free_[dev];
    for (auto& kv : fb) {
      cached_ -= kv.first;
      dev_.erase(kv.second);
      (void)hipFree(kv.second);
    }
    fb.clear();
  }
  size_t cached(int dev) {
    std::lock_guard<std::mutex> lk(mu_);
    size_t t = 0;
    for (auto& kv : free_[dev]) t += kv.first;
    return t;
  }
  size_t size_of(void* p) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = size_.find(p);
    return it == size_.end() ? 0 : it->second;
  }

 private:
  static size_t round(size_t n) {
    const size_t g = n >= (64u << 20) ? (2u << 20) : 256;
    return (std::max<size_t>(n, 256) + g - 1) / g * g;
  }
  std::mutex mu_;
  std::map<int, std::multimap<size_t, void*>> free_;
  std::map<void*, size_t> size_;
  std::map<void*, int> dev_;
  size_t cached_ = 0;
};

// Device allocations owned by a handle or a batch.
struct Owner {
  std::vector<void*> owned;
  size_t bytes = 0;
  void* table = nullptr;   // uploaded plan tables
  size_t table_cap = 0;

  int alloc(void** p, size_t n) {
    *p = nullptr;
    const hipError_t e = Pool::get().alloc(p, n);
    if (e != hipSuccess) {
      set_error("device allocation of " + std::to_string(n) + " bytes failed: " +
                hipGetErrorString(e));
      *p = nullptr;
      return SLAB_E_NOMEM;
    }
    owned.push_back(*p);
    bytes += Pool::get().size_of(*p);
    return SLAB_OK;
  }
  void release(void* p) {
    if (!p) return;
    for (size_t i = 0; i < owned.size(); ++i)
      if (owned[i] == p) {
        bytes -= Pool::get().size_of(p);
        Pool::get().release(p);
        owned.erase(owned.begin() + i);
        return;
      }
  }
  void release_all() {
    for (void* p : owned) Pool::get().release(p);
    owned.clear();
    bytes = 0;
    table = nullptr;
    table_cap = 0;
  }
};

#define SLAB_TRY(expr)              \
  do {                              \
    int rc_ = (expr);               \
    if (rc_ != SLAB_OK) return rc_; \
  } while (0)

// Several buffers carved out of one device allocation (one hipMalloc for a
// whole batch instead of one per buffer and problem).
struct Layout {
  std::vector<std::pair<void**, size_t>> parts;
  size_t total = 0;
  template <class P>
  void add(P** p, size_t n) {
    parts.push_back({(void**)p, n});
    total += (std::max<size_t>(n, 1) + 255) & ~size_t(255);
  }
  // assign the parts consecutively from base (a block of at least total bytes)
  void place(void* base) {
    char* c = (char*)base;
    for (auto& pr : parts) {
      *pr.first = c;
      c += (std::max<size_t>(pr.second, 1) + 255) & ~size_t(255);
    }
  }
  int commit(Owner& o, void** block) {
    void* base = nullptr;
    SLAB_TRY(o.alloc(&base, total));
    place(base);
    if (block) *block = base;
    return SLAB_OK;
  }
};

// Upload the plan's tables into the owner's table buffer (grown as needed).
// The copy is ordered on the stream before the plan's launches.
int upload_plan(Owner& o, const Plan& plan, hipStream_t st, const char** dev) {
  if (plan.bytes() > o.table_cap) {
    if (o.table) {
      SLAB_HIP_CHECK(hipStreamSynchronize(st));
      o.release(o.table);
      o.table = nullptr;
    }
    const size_t cap = std::max<size_t>(plan.bytes() * 2, 1 << 16);
    SLAB_TRY(o.alloc(&o.table, cap));
    o.table_cap = cap;
  }
  if (plan.bytes())
    SLAB_HIP_CHECK(hipMemcpyAsync(o.table, plan.host(), plan.bytes(), hipMemcpyHostToDevice, st));
  *dev = (const char*)o.table;
  return SLAB_OK;
}

int run_plan(Owner& o, const Plan& plan, hipStream_t st) {
  const char* dev = nullptr;
  SLAB_TRY(upload_plan(o, plan, st, &dev));
  return plan.run(dev, st);
}

long long elapsed_us(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1;
  return (long long)(ms * 1000.0f);
}

}  // namespace

// The allocation holding the solve buffers of one or more handles (the items
// of a batch share one); returned to its owner when the last handle using it
// lets go.
struct WsBlock {
  Owner* owner = nullptr;
  void* p = nullptr;
  ~WsBlock() {
    if (owner) owner->release(p);
  }
};

struct Workspace {
  int nrhs = 0;
  std::shared_ptr<WsBlock> block;  // allocation holding the buffers below
  long long generation = 0;        // distinct for every allocation (graph keys)
  void* zbuf = nullptr;
  void* xb = nullptr;
  void* ft = nullptr;
  void* yt = nullptr;
  void* tt = nullptr;
  double* r = nullptr;
  double* norms = nullptr;
  double* partial = nullptr;
  // refined reduced solve (mixed precision): FP64 right-hand side, solution
  // and residual of the reduced system
  double* g64 = nullptr;
  double* u64 = nullptr;
  double* r64 = nullptr;
  void* bpart = nullptr;  // partial products of k-split block-vector products
};

struct slab_handle_s {
  int n1 = 0, n2 = 0, b = 0, m = 0, BP = 0;
  double h = 0.0;
  int precision = SLAB_FP64;
  double tol = 1e-10;
  int max_iter = 10;
  int flags = 0;
  int device = 0;
  int odd_even = 0;
  size_t esz = 8;   // slab factors / Schur pieces / slab sweeps
  size_t esz2 = 8;  // reduced system: T blocks, block factorization, Alg. 2
  double* kappa = nullptr;
  double* wh = nullptr;
  double* wv = nullptr;
  const double* shift_src = nullptr;  // caller's diagonal term (read at factor time)
  double* shift = nullptr;            // its copy, or one zero
  int* status = nullptr;
  void* Gl = nullptr;
  void* Linv = nullptr;
  void* Z = nullptr;
  void* Td = nullptr;  // odd-even order: U_e blocks (kept for the solve)
  void* J = nullptr;   // pivot signs of the signed block factorization (with a shift)
  double* T64 = nullptr;
  double* O64 = nullptr;
  double* S64 = nullptr;
  int tile = 0;    // forced FP32 product tile (0: size rule)
  long long phase_us[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  long long launches[LK_COUNT] = {0, 0, 0, 0, 0, 0, 0, 0};
  Owner mem;
  Workspace ws;
};

static void count_launches(slab_handle h, const Plan& p) {
  for (int k = 0; k < LK_COUNT; ++k) h->launches[k] += p.launches[k];
}

// Work captured as a HIP graph (all refinement passes of a batch solve, or a
// batch's factorization and solve), valid for one set of arguments.
struct GraphCache {
  std::vector<long long> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* tables = nullptr;   // descriptor tables the captured launches read
  void clear(Owner& o) {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (tables) o.release(tables);
    exec = nullptr;
    graph = nullptr;
    tables = nullptr;
    key.clear();
  }
};

struct slab_batch_s {
  std::vector<slab_handle> items;
  int precision = SLAB_FP64;
  int flags = 0;
  int device = 0;
  long long phase_us[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  Owner mem;            // plan tables of batched factorizations and solves
  GraphCache graphs[2]; // all passes of a batch solve (forward, adjoint)
  GraphCache run;       // factorization and solve (slab_batch_run)
  void* run_temps = nullptr;  // factorization temporaries of the run graph
  size_t run_temps_cap = 0;
  // device-side refinement state per problem (graphs): int live[n], iters[n],
  // factor status[4n]; double relres[n]
  void* conv = nullptr;
};

namespace {

int check_vec_args(slab_handle h, const void* in, const void* out, int32_t nrhs, int64_t ld) {
  if (!h) { set_error("null handle"); return SLAB_E_INVALID; }
  if (!in || !out) { set_error("null vector pointer"); return SLAB_E_INVALID; }
  if (nrhs <= 0) { set_error("nrhs must be >= 1"); return SLAB_E_INVALID; }
  const long long N = (long long)h->n1 * h->n2;
  if (ld < N) { set_error("ld must be >= n1*n2"); return SLAB_E_INVALID; }
  const char* a = (const char*)in;
  const char* b = (const char*)out;
  const long long span = ((long long)(nrhs - 1) * ld + N) * 8;
  if (a < b + span && b < a + span) { set_error("input and output overlap"); return SLAB_E_INVALID; }
  return SLAB_OK;
}

// Solve buffers of every job whose handle has none large enough, carved from
// one allocation of `mem` (the handle's own memory for a single problem, the
// batch's for a batch).
void workspace_layout(slab_handle h, int nrhs, Layout& L) {
  Workspace& w = h->ws;
  const size_t n = h->n2, m = h->m, e = h->esz, e2 = h->esz2;
  const size_t N = (size_t)h->n1 * h->n2;
  L.add(&w.zbuf, m * nrhs * n * h->BP * e);
  L.add(&w.xb, m * 2 * nrhs * n * e);
  L.add(&w.ft, m * nrhs * n * e2);
  L.add(&w.yt, m * nrhs * n * e2);
  L.add(&w.tt, nrhs * n * e2);
  L.add(&w.r, nrhs * N * sizeof(double));
  L.add(&w.norms, 2 * nrhs * sizeof(double));
  L.add(&w.partial, residual_partial_count(h->n1, h->n2, nrhs) * sizeof(double));
  L.add(&w.bpart, BMV_PART_SLOTS * bmv_part_elems(h->n2, nrhs) * e2);
  if (h->precision == SLAB_MIXED) {
    L.add(&w.g64, m * nrhs * n * sizeof(double));
    L.add(&w.u64, m * nrhs * n * sizeof(double));
    L.add(&w.r64, m * nrhs * n * sizeof(double));
  }
}

int ensure_workspaces(const std::vector<std::pair<slab_handle, int>>& need, Owner& mem) {
  static std::atomic<long long> generations{0};
  Layout L;
  std::vector<std::pair<slab_handle, int>> grow;
  for (const auto& q : need) {
    slab_handle h = q.first;
    if (h->ws.nrhs >= q.second) continue;
    h->ws = Workspace();  // the old block goes back once no handle uses it
    workspace_layout(h, q.second, L);
    grow.push_back(q);
  }
  if (grow.empty()) return SLAB_OK;
  void* base = nullptr;
  SLAB_TRY(L.commit(mem, &base));
  auto block = std::make_shared<WsBlock>();
  block->owner = &mem;
  block->p = base;
  const long long gen = ++generations;
  for (const auto& q : grow) {
    q.first->ws.nrhs = q.second;
    q.first->ws.block = block;
    q.first->ws.generation = gen;
  }
  return SLAB_OK;
}

int ensure_workspace(slab_handle h, int nrhs) {
  return ensure_workspaces({{h, nrhs}}, h->mem);
}

// ---------------------------------------------------------------------------
// Factorization of a group of handles of one precision and elimination order.
// ---------------------------------------------------------------------------
struct FactorTemps {
  void *Hsw = nullptr, *sig = nullptr, *PRR = nullptr, *PLL = nullptr, *PLR = nullptr,
       *PRL = nullptr, *Td = nullptr, *To = nullptr, *fchk = nullptr;
  int* fredo = nullptr;
};

// Segments of the slab recursion's chains (k_slab_factor): chains of n2 row
// steps are cut into round(n2 / L) equal segments, L = 512 + 5 (b - 31) (at
// least 384), the last taking the remainder, once there are at least two.  At 2048 x 4096, b = 31, with
// two-wave workgroups: 6.2 ms with four segments, 6.5 with three, 8.5 with
// two, 8.6 with five (four-wave workgroups: 9.7 ms unsegmented, 7.2 with
// three, 8.7 with four, 10.2 with segments of 256, 14.5 with 128): the
// redundant warm-up work, not the chain, bounds the shorter segments;
// each segment after the first warming up over `warm` = 6 (b+1) steps (the
// influence of the start shrinks by about exp(-2 pi/(b+1)) per step, so by
// ~4e-17 over the warm-up, far below the check's 1e-13; 7 (b+1): 6.25 ms,
// 6 (b+1): 6.0 ms at 2048 x 4096).  The environment variables SLAB_FACTOR_SEG
// (segment length, 0: no segments) and SLAB_FACTOR_WARM (warm-up steps)
// override both, for measurements and tests.
void slab_segments(int n2, int b, int* nseg, int* seg, int* warm) {
  const char* es = getenv("SLAB_FACTOR_SEG");
  const char* ew = getenv("SLAB_FACTOR_WARM");
  *warm = ew ? std::max(1, atoi(ew)) : 6 * (b + 1);
  if (es) {
    const int seg_len = atoi(es);
    *seg = seg_len > 0 ? seg_len : n2;
    *nseg = seg_len > 0 ? std::max(1, n2 / seg_len) : 1;
  } else {
    // (longer segments for wider slabs, whose warm-up is longer: at b = 49,
    // three of 667 measured faster than four of 500 at n2 = 2000, and two of
    // 500 faster than none at n2 = 1000)
    const double target = std::max(384.0, 512.0 + 5.0 * (b - 31));
    *nseg = std::max(1, (int)std::lround(n2 / target));
    *seg = n2 / *nseg;
  }
  if (*nseg < 2) {
    *nseg = 1;
    *seg = n2;
  }
}

// Memory a handle keeps after the factorization.
template <typename T, typename TR>
void persistent_layout(slab_handle h, Layout& L) {
  const size_t n = h->n2, m = h->m, e = sizeof(T), e2 = sizeof(TR), BP = h->BP;
  const size_t nsq = n * n;
  const size_t ncoef = (size_t)(h->n1 + 2) * (h->n2 + 2);
  L.add(&h->kappa, ncoef * sizeof(double));
  L.add(&h->wh, (size_t)(h->n1 + 1) * n * sizeof(double));
  L.add(&h->wv, (size_t)h->n1 * (n + 1) * sizeof(double));
  L.add(&h->shift, (h->shift_src ? (size_t)h->n1 * n : 1) * sizeof(double));
  L.add(&h->status, 4 * sizeof(int));
  L.add(&h->Gl, m * n * BP * BP * e);
  L.add(&h->Linv, m * nsq * e2);
  L.add(&h->Z, (m > 1 ? m - 1 : 1) * nsq * e2);
  if (h->odd_even) L.add(&h->Td, m * nsq * e2);
  // a diagonal term can make T indefinite: its pivot blocks are factored in
  // signed form L J L^T
  if (h->shift_src) L.add(&h->J, m * n * e2);
  // FP64 reduced blocks: exported on request, and always kept in mixed
  // precision, where the reduced solve is refined against them
  if ((h->flags & SLAB_KEEP_REDUCED) || h->precision == SLAB_MIXED) {
    L.add(&h->T64, m * nsq * sizeof(double));
    L.add(&h->O64, (m > 1 ? m - 1 : 1) * nsq * sizeof(double));
  }
  if (h->flags & SLAB_KEEP_REDUCED) L.add(&h->S64, m * nsq * sizeof(double));
}

// Memory a handle needs only while it is factored (Schur pieces, propagators,
// T blocks).
template <typename T, typename TR>
void temp_layout(slab_handle h, FactorTemps& t, Layout& L) {
  const size_t n = h->n2, m = h->m, e = sizeof(T), e2 = sizeof(TR), BP = h->BP;
  const size_t nsq = n * n;
  L.add(&t.Hsw, m * n * BP * BP * e);
  L.add(&t.sig, m * n * 2 * BP * e);
  int nseg, seg, warm;
  slab_segments(h->n2, h->b, &nseg, &seg, &warm);
  L.add(&t.fchk, nseg > 1 ? m * 2 * nseg * BP * BP * e : 0);
  L.add(&t.fredo, m * 2 * sizeof(int));
  L.add(&t.PRR, m * nsq * e);
  L.add(&t.PLL, m * nsq * e);
  L.add(&t.PLR, m * nsq * e);
  L.add(&t.PRL, m * nsq * e);
  L.add(&t.To, (m > 1 ? m - 1 : 1) * nsq * e2);
  if (!h->odd_even) L.add(&t.Td, m * nsq * e2);
}

// Problem descriptors of stage one for handles whose persistent buffers are
// in place; coefs[i] is the field read by the coefficient step.
std::vector<ProbDev> prob_descs(const std::vector<slab_handle>& hs,
                                const std::vector<const double*>& coefs) {
  std::vector<ProbDev> pd(hs.size());
  for (size_t i = 0; i < hs.size(); ++i) {
    slab_handle h = hs[i];
    ProbDev& d = pd[i];
    std::memset(&d, 0, sizeof(d));
    d.n1 = h->n1; d.n2 = h->n2; d.b = h->b; d.m = h->m; d.h = h->h;
    d.is_log = (h->flags & SLAB_COEF_LOG) ? 1 : 0;
    d.coef = coefs[i]; d.kappa = h->kappa; d.wh = h->wh; d.wv = h->wv;
    d.Gl = h->Gl; d.T64 = h->T64; d.O64 = h->O64; d.status = h->status;
    d.shift_src = h->shift_src; d.shift = h->shift; d.shift_stride = h->shift_src ? 1 : 0;
    slab_segments(h->n2, h->b, &d.fnseg, &d.fseg, &d.fwarm);
  }
  return pd;
}

// Consecutive chunks of handles whose factorization temporaries fit `budget`
// bytes together; every chunk is laid out from the start of one block of
// *block_bytes (the largest chunk).  tmp receives each handle's temporaries
// once a chunk's layout is placed.
struct Chunks {
  std::vector<FactorTemps> tmp;
  std::vector<std::pair<size_t, size_t>> ranges;
  std::vector<Layout> layouts;
  size_t block_bytes = 0;
};

template <typename T, typename TR>
void chunk_layouts(const std::vector<slab_handle>& hs, size_t budget, Chunks& ch) {
  const size_t cnt = hs.size();
  ch.tmp.assign(cnt, FactorTemps());
  for (size_t lo = 0; lo < cnt;) {
    size_t hi = lo;
    Layout L;
    while (hi < cnt) {
      Layout L1 = L;
      temp_layout<T, TR>(hs[hi], ch.tmp[hi], L1);
      if (hi > lo && L1.total > budget) break;
      L = L1;
      ++hi;
    }
    ch.ranges.push_back({lo, hi});
    ch.block_bytes = std::max(ch.block_bytes, L.total);
    ch.layouts.push_back(L);
    lo = hi;
  }
}

// Stage one and stage two of chunk ci, placed in `block`, recorded into p
// (ev: optional phase events of stage one).
template <typename T, typename TR>
void plan_chunk(Plan& p, const std::vector<slab_handle>& hs, const std::vector<ProbDev>& pd,
                Chunks& ch, size_t ci, void* block, const hipEvent_t* ev) {
  const size_t lo = ch.ranges[ci].first, hi = ch.ranges[ci].second;
  ch.layouts[ci].place(block);
  std::vector<ProbDev> cd;
  std::vector<Stage2Prob> s2;
  for (size_t i = lo; i < hi; ++i) {
    FactorTemps& t = ch.tmp[i];
    if (hs[i]->odd_even) t.Td = hs[i]->Td;
    ProbDev d = pd[i];
    d.Hsw = t.Hsw; d.sig = t.sig; d.PRR = t.PRR; d.PLL = t.PLL; d.PLR = t.PLR; d.PRL = t.PRL;
    d.Td = t.Td; d.To = t.To; d.fchk = t.fchk; d.fredo = t.fredo;
    cd.push_back(d);
    Stage2Prob q;
    q.n = hs[i]->n2; q.m = hs[i]->m; q.Td = t.Td; q.To = t.To; q.Linv = hs[i]->Linv;
    q.Z = hs[i]->Z; q.S64 = hs[i]->S64; q.status = hs[i]->status;
    q.J = hs[i]->J; q.indef = hs[i]->J ? 1 : 0;
    s2.push_back(q);
  }
  // one forced product tile for the chunk when its problems agree on it
  int tile = hs[lo]->tile;
  for (size_t i = lo; i < hi; ++i)
    if (hs[i]->tile != tile) tile = 0;
  plan_stage1<T, TR>(p, cd, ev);
  plan_stage2<TR>(p, s2, hs[lo]->odd_even != 0, tile);
}

// Temporaries of a factorization may take half of the memory that is free or
// cached, and at least 1 GiB.
int temp_budget(size_t* budget) {
  size_t free_b = 0, total_b = 0;
  SLAB_HIP_CHECK(hipMemGetInfo(&free_b, &total_b));
  int dev = 0;
  SLAB_HIP_CHECK(hipGetDevice(&dev));
  *budget = std::max<size_t>((free_b + Pool::get().cached(dev)) / 2, (size_t)1 << 30);
  return SLAB_OK;
}

// Factor every handle of hs (sizes set) from probs[i]->kappa.  Per problem,
// fail[i] receives 0 (ok), 1 (invalid kappa), 2 (slab breakdown) or 3 (block
// breakdown) and blk[i] the slab / interface index; ph the group's phase times.
// The problems are factored in consecutive chunks whose temporaries fit half of
// the free device memory; every chunk is one set of grouped launches.
template <typename T, typename TR>
int factor_group(const std::vector<slab_handle>& hs, const std::vector<const slab_problem*>& probs,
                 hipStream_t st, Owner& plan_mem, std::vector<int>& fail, std::vector<int>& blk,
                 long long* ph) {
  const size_t cnt = hs.size();
  fail.assign(cnt, 0);
  blk.assign(cnt, -1);
  for (int i = 0; i < 6; ++i) ph[i] = 0;
  {
    Layout L;
    for (size_t i = 0; i < cnt; ++i) persistent_layout<T, TR>(hs[i], L);
    SLAB_TRY(L.commit(plan_mem, nullptr));
  }
  std::vector<const double*> coefs;
  for (size_t i = 0; i < cnt; ++i) coefs.push_back(probs[i]->kappa);
  const std::vector<ProbDev> pd = prob_descs(hs, coefs);
  hipEvent_t ev[6];
  for (int i = 0; i < 6; ++i) SLAB_HIP_CHECK(hipEventCreate(&ev[i]));
  struct EvGuard {
    hipEvent_t* e;
    ~EvGuard() { for (int i = 0; i < 6; ++i) (void)hipEventDestroy(e[i]); }
  } guard{ev};
  std::vector<int> hs_status(4 * cnt, 0);
  auto read_status = [&](size_t lo, size_t hi) -> int {
    for (size_t i = lo; i < hi; ++i)
      SLAB_HIP_CHECK(hipMemcpyAsync(&hs_status[4 * i], hs[i]->status, 4 * sizeof(int),
                                    hipMemcpyDeviceToHost, st));
    SLAB_HIP_CHECK(hipStreamSynchronize(st));
    return SLAB_OK;
  };
  // coefficients first: an invalid field is reported before any factor work
  {
    Plan p;
    plan_coef_weights(p, pd);
    SLAB_TRY(run_plan(plan_mem, p, st));
  }
  SLAB_TRY(read_status(0, cnt));
  bool any_bad = false;
  for (size_t i = 0; i < cnt; ++i)
    if (hs_status[4 * i + 2] == 1) { fail[i] = 1; any_bad = true; }
  if (any_bad) return SLAB_E_INVALID;
  // chunks first; one block of the largest chunk's size serves them all (the
  // caching allocator then meets every later factorization of the same set)
  size_t budget = 0;
  SLAB_TRY(temp_budget(&budget));
  Chunks ch;
  chunk_layouts<T, TR>(hs, budget, ch);
  void* block = nullptr;
  SLAB_TRY(plan_mem.alloc(&block, ch.block_bytes));
  for (size_t ci = 0; ci < ch.ranges.size(); ++ci) {
    const size_t lo = ch.ranges[ci].first, hi = ch.ranges[ci].second;
    Plan p;
    p.timer = std::make_shared<Plan::Timer>();
    plan_chunk<T, TR>(p, hs, pd, ch, ci, block, ev + 1);
    for (size_t i = lo; i < hi; ++i) count_launches(hs[i], p);
    SLAB_HIP_CHECK(hipEventRecord(ev[0], st));
    SLAB_TRY(run_plan(plan_mem, p, st));
    SLAB_HIP_CHECK(hipEventRecord(ev[5], st));
    SLAB_TRY(read_status(lo, hi));
    // phases: slab factor, boundary columns, Schur propagation, assembly of T,
    // block factorization (summed over chunks); 5: the block products inside
    // the block factorization
    for (int i = 0; i < 5; ++i) ph[i] += elapsed_us(ev[i], ev[i + 1]);
    ph[5] += (long long)(p.timer->total_ms() * 1000.0);
    SLAB_HIP_CHECK(hipStreamSynchronize(st));
    for (size_t i = lo; i < hi; ++i) {
      if (hs_status[4 * i] != 0) {
        fail[i] = hs_status[4 * i];
        blk[i] = hs_status[4 * i + 1];
      }
    }
  }
  plan_mem.release(block);
  return SLAB_OK;
}

// The whole factorization of handles whose persistent buffers are in place,
// recorded into p with no host synchronization (for graph capture): status
// words cleared and coefficients from coefs on the device, then every chunk in
// order, all chunks in *block (allocated from mem on first use, or when too
// small).  Failures are left in the handles' status words.
template <typename T, typename TR>
int plan_factor_nosync(Plan& p, const std::vector<slab_handle>& hs,
                       const std::vector<const double*>& coefs, Owner& mem, void** block,
                       size_t* block_cap) {
  const std::vector<ProbDev> pd = prob_descs(hs, coefs);
  plan_coef_weights(p, pd);
  size_t budget = 0;
  SLAB_TRY(temp_budget(&budget));
  Chunks ch;
  chunk_layouts<T, TR>(hs, budget + *block_cap, ch);
  if (!*block || *block_cap < ch.block_bytes) {
    if (*block) mem.release(*block);
    *block = nullptr;
    *block_cap = 0;
    SLAB_TRY(mem.alloc(block, ch.block_bytes));
    *block_cap = ch.block_bytes;
  }
  for (size_t ci = 0; ci < ch.ranges.size(); ++ci) plan_chunk<T, TR>(p, hs, pd, ch, ci, *block, nullptr);
  for (slab_handle h : hs) count_launches(h, p);
  return SLAB_OK;
}

int factor_dispatch(int precision, const std::vector<slab_handle>& hs,
                    const std::vector<const slab_problem*>& probs, hipStream_t st, Owner& mem,
                    std::vector<int>& fail, std::vector<int>& blk, long long* ph) {
  if (precision == SLAB_FP32_REFINE)
    return factor_group<float, float>(hs, probs, st, mem, fail, blk, ph);
  if (precision == SLAB_MIXED)
    return factor_group<double, float>(hs, probs, st, mem, fail, blk, ph);
  return factor_group<double, double>(hs, probs, st, mem, fail, blk, ph);
}

std::string fail_message(int code, int blk) {
  if (code == 1)
    return "coefficient field has a value that is not positive and finite (or the diagonal "
           "term one that is not finite)";
  if (code == 2) return "slab factorization breakdown in slab " + std::to_string(blk);
  return "block factorization breakdown at interface " + std::to_string(blk);
}

slab_handle new_handle(const slab_problem* prob, const slab_options* opts, int device) {
  slab_handle h = new slab_handle_s();
  h->n1 = prob->n1; h->n2 = prob->n2; h->b = prob->b; h->m = prob->n1 / (prob->b + 1);
  h->BP = padded_block(prob->b); h->h = prob->h; h->shift_src = prob->shift;
  if (opts) { h->precision = opts->precision; h->tol = opts->tol; h->max_iter = opts->max_iter; h->flags = opts->flags; }
  h->odd_even = (h->flags & SLAB_ODD_EVEN) ? 1 : 0;
  h->tile = opts ? opts->tile : 0;
  h->esz = h->precision == SLAB_FP32_REFINE ? 4 : 8;
  h->esz2 = h->precision == SLAB_FP64 ? 8 : 4;
  h->device = device;
  return h;
}

void delete_handle(slab_handle h) {
  h->mem.release_all();
  delete h;
}

// ---------------------------------------------------------------------------
// Solves with FP64 refinement for a group of handles of one precision:
//   pass 1: u = solve(f); later passes: u += solve(r); r = f - A u after each.
// A problem leaves the group once its residual meets its tolerance.
// ---------------------------------------------------------------------------
struct SolveJob {
  slab_handle h;
  const double* f;
  double* u;
  int nrhs;
  long long ld;
  slab_solve_info* info;
};

// live (optional): the refinement flag of every job; the pass's work for a
// job whose flag is 0 is skipped on the device.
template <typename T, typename TR>
void plan_pass(Plan& p, const std::vector<SolveJob>& jobs, bool first, bool trans,
               const std::vector<const int*>* live) {
  std::vector<SolveDev> sd(jobs.size());
  std::vector<ReducedDev> red(jobs.size());
  for (size_t i = 0; i < jobs.size(); ++i) {
    const SolveJob& j = jobs[i];
    slab_handle h = j.h;
    SolveDev& d = sd[i];
    std::memset(&d, 0, sizeof(d));
    d.n1 = h->n1; d.n2 = h->n2; d.b = h->b; d.m = h->m; d.nrhs = j.nrhs;
    d.wh = h->wh; d.wv = h->wv; d.Gl = h->Gl;
    d.shift = h->shift; d.shift_stride = h->shift_src ? 1 : 0;
    d.zbuf = h->ws.zbuf; d.xb = h->ws.xb; d.ft = h->ws.ft;
    const long long N = (long long)h->n1 * h->n2;
    d.rhs = first ? j.f : h->ws.r;
    d.ld = first ? j.ld : N;
    d.out = j.u; d.ldo = j.ld; d.accumulate = first ? 0 : 1;
    d.f = j.f; d.u = j.u; d.r = h->ws.r; d.ldf = j.ld; d.norms = h->ws.norms;
    d.partial = h->ws.partial;
    d.live = live ? (*live)[i] : nullptr;
    ReducedDev& r = red[i];
    std::memset(&r, 0, sizeof(r));
    r.n = h->n2; r.m = h->m; r.nrhs = j.nrhs; r.Linv = h->Linv; r.Z = h->Z; r.Td = h->Td;
    r.ft = h->ws.ft; r.yt = h->ws.yt; r.tt = h->ws.tt; r.part = h->ws.bpart;
    r.J = h->J;
    r.live = d.live;
    if (h->precision == SLAB_MIXED) {
      r.T64 = h->T64; r.O64 = h->O64;
      r.g64 = h->ws.g64; r.u64 = h->ws.u64; r.r64 = h->ws.r64;
      d.g64 = h->ws.g64; d.uo64 = h->ws.u64;
    }
  }
  plan_solve_pass<T, TR>(p, sd, red, trans, jobs[0].h->odd_even != 0);
  // the transposed residual equals A^T u = A u (A is symmetric)
  plan_residual(p, sd);
}

void plan_pass_dispatch(int precision, Plan& p, const std::vector<SolveJob>& jobs, bool first,
                        bool trans, const std::vector<const int*>* live = nullptr) {
  if (precision == SLAB_FP32_REFINE) plan_pass<float, float>(p, jobs, first, trans, live);
  else if (precision == SLAB_MIXED) plan_pass<double, float>(p, jobs, first, trans, live);
  else plan_pass<double, double>(p, jobs, first, trans, live);
}

int read_relres(const std::vector<SolveJob>& jobs, hipStream_t st,
                std::vector<std::vector<double>>& rr) {
  std::vector<std::vector<double>> nrm(jobs.size());
  for (size_t i = 0; i < jobs.size(); ++i) {
    nrm[i].resize(2 * jobs[i].nrhs);
    SLAB_HIP_CHECK(hipMemcpyAsync(nrm[i].data(), jobs[i].h->ws.norms,
                                  2 * jobs[i].nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  SLAB_HIP_CHECK(hipStreamSynchronize(st));
  rr.resize(jobs.size());
  for (size_t i = 0; i < jobs.size(); ++i) {
    rr[i].resize(jobs[i].nrhs);
    for (int c = 0; c < jobs[i].nrhs; ++c) {
      const double fn = std::sqrt(nrm[i][2 * c + 1]);
      rr[i][c] = fn > 0 ? std::sqrt(nrm[i][2 * c]) / fn : std::sqrt(nrm[i][2 * c]);
    }
  }
  return SLAB_OK;
}

double worst_of(const std::vector<double>& v) {
  double w = 0.0;
  for (double x : v) {
    if (!std::isfinite(x)) return NAN;
    w = std::max(w, x);
  }
  return w;
}

// Device memory of a call that allocates nothing: the plan tables of every
// pass are copied to `tables` (the solve buffers were placed by the caller).
struct FixedTables {
  char* tables;
  size_t cap;
};

// One refinement pass of `jobs`, eagerly (plan tables in the owner's table
// buffer, or in fx's region).
int run_pass(Owner& mem, const std::vector<SolveJob>& jobs, int precision, bool first, bool trans,
             hipStream_t st, const FixedTables* fx) {
  Plan p;
  plan_pass_dispatch(precision, p, jobs, first, trans);
  for (const SolveJob& j : jobs) count_launches(j.h, p);
  if (fx) {
    if (p.bytes() > fx->cap) {
      set_error("plan tables of " + std::to_string(p.bytes()) + " bytes exceed the " +
                std::to_string(fx->cap) + " bytes reserved for them in the scratch array");
      return SLAB_E_INVALID;
    }
    // ordered on the stream after the previous pass's launches, which read
    // the same table region
    if (p.bytes())
      SLAB_HIP_CHECK(hipMemcpyAsync(fx->tables, p.host(), p.bytes(), hipMemcpyHostToDevice, st));
    return p.run(fx->tables, st);
  }
  return run_plan(mem, p, st);
}

// Pass counts and final residuals into the jobs' infos; SLAB_E_NOCONV (with
// a message naming the problem) if one missed its tolerance.
int finish_jobs(std::vector<SolveJob>& jobs, const std::vector<int>& it,
                const std::vector<double>& worst) {
  int rc = SLAB_OK;
  for (size_t i = 0; i < jobs.size(); ++i) {
    if (jobs[i].info) {
      jobs[i].info->iterations = it[i];
      jobs[i].info->max_relres = worst[i];
      jobs[i].info->failed_block = -1;
    }
    if (!(worst[i] <= jobs[i].h->tol) && rc == SLAB_OK) {
      char buf[96];
      std::snprintf(buf, sizeof buf, "%.3e after %d passes (tol %.3e)", worst[i], it[i],
                    jobs[i].h->tol);
      set_error(std::string("refinement stopped at relative residual ") + buf +
                (jobs.size() > 1 ? " in problem " + std::to_string(i) : std::string()));
      rc = SLAB_E_NOCONV;
    }
  }
  return rc;
}

// fx: the workspaces of the jobs' handles are already in place and the plan
// tables go to fx->tables (nothing is allocated); null: the usual path.
// Passes run one at a time; the host reads the residuals after each one and
// drops the problems that meet their tolerance.
int solve_group(std::vector<SolveJob>& jobs, int precision, bool trans, hipStream_t st,
                Owner& mem, const FixedTables* fx = nullptr) {
  if (!fx) {
    std::vector<std::pair<slab_handle, int>> need;
    for (SolveJob& j : jobs) need.push_back({j.h, j.nrhs});
    SLAB_TRY(ensure_workspaces(need, mem));
  }
  std::vector<int> it(jobs.size(), 0);
  std::vector<double> worst(jobs.size(), 0.0);
  std::vector<SolveJob> live = jobs;
  std::vector<size_t> idx(jobs.size());
  for (size_t i = 0; i < jobs.size(); ++i) idx[i] = i;
  bool first = true;
  while (!live.empty()) {
    SLAB_TRY(run_pass(mem, live, precision, first, trans, st, fx));
    std::vector<std::vector<double>> rr;
    SLAB_TRY(read_relres(live, st, rr));
    std::vector<SolveJob> next;
    std::vector<size_t> nidx;
    for (size_t k = 0; k < live.size(); ++k) {
      const size_t i = idx[k];
      ++it[i];
      const double prev = worst[i];
      worst[i] = worst_of(rr[k]);
      // a residual above the right-hand side that grew since the last pass:
      // the refinement diverges (the device-side test stops it the same way)
      const bool diverged = it[i] >= 2 && worst[i] > 1.0 && worst[i] > prev;
      const bool done = !(worst[i] > jobs[i].h->tol) || it[i] >= jobs[i].h->max_iter || diverged;
      if (!done) {
        next.push_back(live[k]);
        nidx.push_back(i);
      }
    }
    live.swap(next);
    idx.swap(nidx);
    first = false;
  }
  return finish_jobs(jobs, it, worst);
}

// Launch gc's graph if it was captured for `key`; otherwise record the work
// with build(p) (no host synchronization inside), upload its tables to a
// buffer that lives with the graph, capture, instantiate and launch.
int launch_graph(Owner& mem, GraphCache* gc, const std::vector<long long>& key,
                 const std::function<int(Plan&)>& build, hipStream_t st) {
  if (gc->exec && gc->key == key) {
    SLAB_HIP_CHECK(hipGraphLaunch(gc->exec, st));
    return SLAB_OK;
  }
  SLAB_HIP_CHECK(hipStreamSynchronize(st));
  gc->clear(mem);
  Plan p;
  SLAB_TRY(build(p));
  SLAB_TRY(mem.alloc(&gc->tables, std::max<size_t>(p.bytes(), 256)));
  SLAB_HIP_CHECK(hipMemcpyAsync(gc->tables, p.host(), p.bytes(), hipMemcpyHostToDevice, st));
  SLAB_HIP_CHECK(hipStreamSynchronize(st));
  SLAB_HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  const int rc = p.run((const char*)gc->tables, st);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  if (rc != SLAB_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) {
    set_error(std::string("graph capture failed: ") + hipGetErrorString(e));
    return SLAB_E_HIP;
  }
  gc->graph = g;
  SLAB_HIP_CHECK(hipGraphInstantiate(&gc->exec, g, nullptr, nullptr, 0));
  gc->key = key;
  SLAB_HIP_CHECK(hipGraphLaunch(gc->exec, st));
  return SLAB_OK;
}

// Device-side refinement state of a batch (see slab_batch_s::conv).
struct ConvPtrs {
  int* live;
  int* iters;
  int* fstat;
  double* relres;
};

int batch_conv(slab_batch bt, ConvPtrs* c) {
  const size_t n = bt->items.size();
  const size_t ib = (6 * n * sizeof(int) + 255) & ~size_t(255);
  if (!bt->conv) SLAB_TRY(bt->mem.alloc(&bt->conv, ib + n * sizeof(double)));
  c->live = (int*)bt->conv;
  c->iters = c->live + n;
  c->fstat = c->iters + n;
  c->relres = (double*)((char*)bt->conv + ib);
  return SLAB_OK;
}

// Every refinement pass of the jobs (as many as the largest max_iter), each
// followed by the device-side convergence test, recorded after what p holds.
// Passes after a problem has met its tolerance skip its work on the device.
// fstatus: copy the factorization status words too (batch runs).
void plan_all_passes(Plan& p, const std::vector<SolveJob>& jobs, int precision, bool trans,
                     const ConvPtrs& c, bool fstatus) {
  int maxit = 1;
  for (const SolveJob& j : jobs) maxit = std::max(maxit, j.h->max_iter);
  std::vector<ConvDev> conv(jobs.size());
  std::vector<const int*> live(jobs.size());
  for (size_t i = 0; i < jobs.size(); ++i) {
    slab_handle h = jobs[i].h;
    conv[i] = ConvDev{h->ws.norms, jobs[i].nrhs, h->max_iter, h->tol, c.live + i, c.iters + i,
                      c.relres + i, fstatus ? h->status : nullptr,
                      fstatus ? c.fstat + 4 * i : nullptr};
    live[i] = c.live + i;
  }
  for (int k = 0; k < maxit; ++k) {
    plan_pass_dispatch(precision, p, jobs, k == 0, trans, k == 0 ? nullptr : &live);
    plan_converge(p, conv, k == 0);
  }
}

// Key of a graph over jobs: the captured launches read the jobs' vectors and
// workspaces, so a new workspace (grown by any call on one of the handles)
// invalidates it.
std::vector<long long> jobs_key(const std::vector<SolveJob>& jobs, long long tag) {
  std::vector<long long> key{tag};
  for (const SolveJob& j : jobs) {
    key.push_back((long long)(uintptr_t)j.h);
    key.push_back((long long)(uintptr_t)j.f);
    key.push_back((long long)(uintptr_t)j.u);
    key.push_back(j.nrhs);
    key.push_back(j.ld);
    key.push_back(j.h->ws.generation);
  }
  return key;
}

// Read the pass counts, residuals and (optionally) factorization statuses of a
// batch after its graph (one copy, one synchronization).
int read_conv(slab_batch bt, hipStream_t st, std::vector<int>& it, std::vector<double>& worst,
              std::vector<int>* fstat) {
  const size_t n = bt->items.size();
  const size_t ib = (6 * n * sizeof(int) + 255) & ~size_t(255);
  std::vector<char> host(ib + n * sizeof(double));
  SLAB_HIP_CHECK(hipMemcpyAsync(host.data(), bt->conv, host.size(), hipMemcpyDeviceToHost, st));
  SLAB_HIP_CHECK(hipStreamSynchronize(st));
  const int* ip = (const int*)host.data();
  const double* dp = (const double*)(host.data() + ib);
  it.assign(ip + n, ip + 2 * n);
  worst.assign(dp, dp + n);
  if (fstat) fstat->assign(ip + 2 * n, ip + 6 * n);
  return SLAB_OK;
}

int plan_factor_nosync_dispatch(int precision, Plan& p, const std::vector<slab_handle>& hs,
                                const std::vector<const double*>& coefs, Owner& mem,
                                void** block, size_t* cap) {
  if (precision == SLAB_FP32_REFINE)
    return plan_factor_nosync<float, float>(p, hs, coefs, mem, block, cap);
  if (precision == SLAB_MIXED) return plan_factor_nosync<double, float>(p, hs, coefs, mem, block, cap);
  return plan_factor_nosync<double, double>(p, hs, coefs, mem, block, cap);
}

// All refinement passes of a batch solve as one graph launch (SLAB_GRAPH):
// the convergence test runs on the device and the host synchronizes once.
int solve_batch_graph(slab_batch bt, std::vector<SolveJob>& jobs, bool trans, hipStream_t st) {
  {
    std::vector<std::pair<slab_handle, int>> need;
    for (SolveJob& j : jobs) need.push_back({j.h, j.nrhs});
    SLAB_TRY(ensure_workspaces(need, bt->mem));
  }
  ConvPtrs c;
  SLAB_TRY(batch_conv(bt, &c));
  auto build = [&](Plan& p) {
    plan_all_passes(p, jobs, bt->precision, trans, c, false);
    for (const SolveJob& j : jobs) count_launches(j.h, p);
    return SLAB_OK;
  };
  SLAB_TRY(launch_graph(bt->mem, &bt->graphs[trans ? 1 : 0], jobs_key(jobs, trans ? 1 : 0),
                        build, st));
  std::vector<int> it;
  std::vector<double> worst;
  SLAB_TRY(read_conv(bt, st, it, worst, nullptr));
  return finish_jobs(jobs, it, worst);
}

int solve_one(slab_handle h, const double* f, double* u, int32_t nrhs, int64_t ld, void* stream,
              slab_solve_info* info, bool trans) {
  SLAB_TRY(check_vec_args(h, f, u, nrhs, ld));
  hipStream_t st = (hipStream_t)stream;
  SLAB_HIP_CHECK(hipSetDevice(h->device));
  std::vector<SolveJob> jobs{{h, f, u, nrhs, ld, info}};
  return solve_group(jobs, h->precision, trans, st, h->mem);
}

// ---------------------------------------------------------------------------
// Allocation-free solve.  The solve buffers and plan tables of one call live
// in a file-scope device array of fixed size; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device
// (the array's name is a host-side stand-in, not a device address).
// ---------------------------------------------------------------------------
constexpr size_t kScratchTableBytes = size_t(1) << 20;

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_addr;  // device -> address of `scratch` on it

}  // namespace

__device__ __align__(256) char scratch[SLAB_NOALLOC_SCRATCH_BYTES];

namespace {

// Address of the scratch array on the current device, looked up once per
// device (with that device current) and kept.
int scratch_address(char** out) {
  int dev = 0;
  SLAB_HIP_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it == g_scratch_addr.end()) {
    char* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error(std::string("hipGetSymbolAddress of the scratch array failed: ") +
                hipGetErrorString(e));
      return SLAB_E_HIP;
    }
    it = g_scratch_addr.emplace(dev, ptr).first;
  }
  *out = it->second;
  return SLAB_OK;
}

int solve_noalloc(slab_handle h, const double* f, double* u, int32_t nrhs, int64_t ld,
                  void* stream, slab_solve_info* info) {
  SLAB_TRY(check_vec_args(h, f, u, nrhs, ld));
  hipStream_t st = (hipStream_t)stream;
  SLAB_HIP_CHECK(hipSetDevice(h->device));
  char* base = nullptr;
  SLAB_TRY(scratch_address(&base));
  // the call's solve buffers, laid out as for the handle's own workspace but
  // placed in the scratch array after the table region; the handle's own
  // workspace is put back afterwards
  Workspace own = h->ws;
  h->ws = Workspace();
  Layout L;
  workspace_layout(h, nrhs, L);
  if (L.total > SLAB_NOALLOC_SCRATCH_BYTES - kScratchTableBytes) {
    h->ws = own;
    set_error("the allocation-free solve needs " + std::to_string(L.total) +
              " bytes of solve buffers for this problem and nrhs; its scratch array holds " +
              std::to_string(SLAB_NOALLOC_SCRATCH_BYTES - kScratchTableBytes));
    return SLAB_E_INVALID;
  }
  L.place(base + kScratchTableBytes);
  h->ws.nrhs = nrhs;
  h->ws.generation = -1;  // never equal to a batch graph's key
  const FixedTables fx{base, kScratchTableBytes};
  std::vector<SolveJob> jobs{{h, f, u, nrhs, ld, info}};
  const int rc = solve_group(jobs, h->precision, false, st, h->mem, &fx);
  h->ws = own;
  return rc;
}

// ---------------------------------------------------------------------------
// Autotuner: slab width b and the FP32 product tile of stage two.
// ---------------------------------------------------------------------------
const int kWidths[5] = {3, 7, 15, 31, 63};

// Predicted seconds for slab width b (Sec. 4, eq. (complexity_funcb): the slab
// work grows and the reduced-system work shrinks with b), at half of the
// nominal peaks, plus the row-by-row latency of the slab recursion.
double model_seconds(int n1, int n2, int b, int precision, bool odd_even) {
  const double m = n1 / (b + 1), n = n2;
  const double r1 = 0.5 * (precision == SLAB_FP32_REFINE ? 157.3e12 : 78.6e12);
  const double r2 = 0.5 * (precision == SLAB_FP64 ? 78.6e12 : 157.3e12);
  const double schur = m * 2.0 * n * n * (double)b * b / r1;
  const double reduced = m * (odd_even ? 6.67 : 2.67) * n * n * n / r2;
  const double latency = 0.5e-6 * n * b;
  return schur + reduced + latency;
}

std::mutex g_tune_mu;
std::map<std::vector<long long>, int> g_width_cache;
std::map<int, int> g_tile_cache;  // FP32 product tile measured fastest per block size

int cached_tile(int n) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tile_cache.find(n);
  return it == g_tile_cache.end() ? 0 : it->second;
}

// Time the two tile widths on `count` products of n x n FP32 blocks shaped
// like the odd-even update L^-1 C, and record the faster one.
int tune_tile(int n, int count, hipStream_t st) {
  if (cached_tile(n)) return SLAB_OK;
  Owner tmp;
  struct Free {
    Owner& o;
    ~Free() { o.release_all(); }
  } fr{tmp};
  const size_t bytes = (size_t)count * n * n * sizeof(float);
  void *A, *B, *C;
  SLAB_TRY(tmp.alloc(&A, bytes));
  SLAB_TRY(tmp.alloc(&B, bytes));
  SLAB_TRY(tmp.alloc(&C, bytes));
  SLAB_HIP_CHECK(hipMemsetAsync(A, 0, bytes, st));
  SLAB_HIP_CHECK(hipMemsetAsync(B, 0, bytes, st));
  std::vector<GemmItem> items;
  for (int q = 0; q < count; ++q) {
    GemmItem g;
    const size_t off = (size_t)q * n * n;
    g.A = (float*)A + off; g.B = (float*)B + off; g.C = (float*)C + off;
    g.M = g.N = g.K = n; g.lda = g.ldb = g.ldc = n;
    items.push_back(g);
  }
  hipEvent_t e0, e1;
  SLAB_HIP_CHECK(hipEventCreate(&e0));
  SLAB_HIP_CHECK(hipEventCreate(&e1));
  double best = 1e300;
  int best_tile = 64;
  for (int tile : {64, 128}) {
    Plan p;
    plan_gemm<float>(p, false, false, items, 1.f, 0.f, GEMM_A_LOWER, tile);
    const char* dev = nullptr;
    SLAB_TRY(upload_plan(tmp, p, st, &dev));
    SLAB_TRY(p.run(dev, st));  // warm-up
    SLAB_HIP_CHECK(hipEventRecord(e0, st));
    for (int r = 0; r < 3; ++r) SLAB_TRY(p.run(dev, st));
    SLAB_HIP_CHECK(hipEventRecord(e1, st));
    SLAB_HIP_CHECK(hipEventSynchronize(e1));
    float ms = 0.f;
    SLAB_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) { best = ms; best_tile = tile; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tile_cache[n] = best_tile;
  return SLAB_OK;
}

}  // namespace

extern "C" {

int slab_autotune(const slab_problem* prob, const slab_options* opts, int32_t nrhs,
                  void* hip_stream, int32_t* b_out, double* times) {
  if (!prob || !b_out || nrhs < 1) { set_error("bad arguments to slab_autotune"); return SLAB_E_INVALID; }
  slab_problem p = *prob;
  p.b = 0;
  SLAB_TRY(slab_check_problem(&p, opts));
  slab_options o = opts ? *opts : slab_options{SLAB_FP64, 1e-10, 10, 0, 0};
  o.flags &= ~(SLAB_KEEP_REDUCED | SLAB_GRAPH);
  const bool odd_even = (o.flags & SLAB_ODD_EVEN) != 0;
  const std::vector<long long> key{p.n1, p.n2, o.precision, o.flags, nrhs, o.tile};
  for (int k = 0; k < 5; ++k)
    if (times) times[k] = -1.0;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_width_cache.find(key);
    if (it != g_width_cache.end() && !times) {
      *b_out = it->second;
      return SLAB_OK;
    }
  }
  hipStream_t st = (hipStream_t)hip_stream;
  // candidates dividing n1, pruned by the model to within 3x of its best
  double mbest = 1e300;
  for (int b : kWidths)
    if (p.n1 % (b + 1) == 0) mbest = std::min(mbest, model_seconds(p.n1, p.n2, b, o.precision, odd_even));
  if (o.precision != SLAB_FP64 && odd_even && p.n2 >= 256 && o.tile == 0) {
    SLAB_TRY(tune_tile(p.n2, std::min(16, std::max(1, p.n1 / 64)), st));
    o.tile = cached_tile(p.n2);  // the candidates are timed with it
  }
  const long long N = (long long)p.n1 * p.n2;
  Owner tmp;
  struct Free {
    Owner& o;
    ~Free() { o.release_all(); }
  } fr{tmp};
  double *f = nullptr, *u = nullptr;
  SLAB_TRY(tmp.alloc((void**)&f, (size_t)N * nrhs * sizeof(double)));
  SLAB_TRY(tmp.alloc((void**)&u, (size_t)N * nrhs * sizeof(double)));
  {
    // right-hand sides uniform in [-1, 1) (a smooth load such as f = 1 would
    // put the FP64 residual's rounding floor near the tolerance on fine grids)
    std::vector<double> rhs((size_t)N * nrhs);
    std::mt19937_64 gen(12345);
    std::uniform_real_distribution<double> uni(-1.0, 1.0);
    for (double& v : rhs) v = uni(gen);
    SLAB_HIP_CHECK(hipMemcpy(f, rhs.data(), rhs.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  hipEvent_t e0, e1;
  SLAB_HIP_CHECK(hipEventCreate(&e0));
  SLAB_HIP_CHECK(hipEventCreate(&e1));
  double best = 1e300;
  int best_b = -1;
  for (int k = 0; k < 5; ++k) {
    const int b = kWidths[k];
    if (p.n1 % (b + 1) != 0) continue;
    if (model_seconds(p.n1, p.n2, b, o.precision, odd_even) > 3.0 * mbest) continue;
    p.b = b;
    slab_handle h = nullptr;
    SLAB_HIP_CHECK(hipEventRecord(e0, st));
    int rc = slab_factor(&p, &o, st, &h, nullptr);
    if (rc == SLAB_OK) {
      rc = slab_solve(h, f, u, nrhs, N, st, nullptr);
      SLAB_HIP_CHECK(hipEventRecord(e1, st));
      SLAB_HIP_CHECK(hipEventSynchronize(e1));
      slab_free(h);
    }
    if (rc != SLAB_OK && rc != SLAB_E_NOCONV) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return rc;
    }
    if (rc == SLAB_E_NOCONV) continue;  // a width that does not converge is not a choice
    float ms = 0.f;
    SLAB_HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
    if (times) times[k] = ms * 1e-3;
    if (ms < best) { best = ms; best_b = b; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_b < 0) { set_error("no slab width converged"); return SLAB_E_NOCONV; }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_width_cache[key] = best_b;
  }
  *b_out = best_b;
  return SLAB_OK;
}

const char* slab_last_error(void) { return g_last_error.c_str(); }

int slab_check_problem(const slab_problem* prob, const slab_options* opts) {
  if (!prob) { set_error("null problem"); return SLAB_E_INVALID; }
  if (prob->n2 < 1 || prob->n1 < 2 || prob->b < 0 || prob->b > 63) {
    set_error("need n2 >= 1, n1 >= 2, 0 <= b <= 63");
    return SLAB_E_INVALID;
  }
  if (prob->b == 0 && prob->n1 % 4 != 0) {
    set_error("b = 0 (autotuned) needs n1 to be a multiple of 4");
    return SLAB_E_INVALID;
  }
  if (prob->b > 0 && prob->n1 % (prob->b + 1) != 0) { set_error("n1 must be a multiple of b+1"); return SLAB_E_INVALID; }
  if (!(prob->h > 0.0) || !std::isfinite(prob->h)) { set_error("h must be positive and finite"); return SLAB_E_INVALID; }
  if (!prob->kappa) { set_error("null coefficient pointer"); return SLAB_E_INVALID; }
  if ((long long)prob->n1 * prob->n2 > (1LL << 40)) { set_error("grid too large"); return SLAB_E_INVALID; }
  if (opts) {
    if (opts->precision != SLAB_FP64 && opts->precision != SLAB_FP32_REFINE &&
        opts->precision != SLAB_MIXED) {
      set_error("unknown precision"); return SLAB_E_INVALID;
    }
    if (!(opts->tol > 0.0) || !std::isfinite(opts->tol)) { set_error("tol must be positive"); return SLAB_E_INVALID; }
    if (opts->max_iter < 1) { set_error("max_iter must be >= 1"); return SLAB_E_INVALID; }
    if (opts->flags & ~(SLAB_KEEP_REDUCED | SLAB_COEF_LOG | SLAB_ODD_EVEN | SLAB_GRAPH)) {
      set_error("unknown flag"); return SLAB_E_INVALID;
    }
    if (opts->tile != 0 && opts->tile != 64 && opts->tile != 128) {
      set_error("tile must be 0, 64 or 128"); return SLAB_E_INVALID;
    }
  }
  return SLAB_OK;
}

int slab_factor(const slab_problem* prob, const slab_options* opts, void* hip_stream,
                slab_handle* out, slab_solve_info* info) {
  if (info) { info->iterations = 0; info->max_relres = 0.0; info->failed_block = -1; }
  if (!out) { set_error("null output handle pointer"); return SLAB_E_INVALID; }
  *out = nullptr;
  int rc = slab_check_problem(prob, opts);
  if (rc) return rc;
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) { set_error("no HIP device"); return SLAB_E_HIP; }
  hipStream_t st = (hipStream_t)hip_stream;
  slab_problem tuned = *prob;
  const bool autotuned = tuned.b == 0;
  if (autotuned) {
    rc = slab_autotune(prob, opts, 1, hip_stream, &tuned.b, nullptr);
    if (rc) return rc;
    prob = &tuned;
  }
  slab_handle h = new_handle(prob, opts, device);
  if (autotuned && h->tile == 0 && h->precision != SLAB_FP64) h->tile = cached_tile(h->n2);
  std::vector<slab_handle> hs{h};
  std::vector<const slab_problem*> ps{prob};
  std::vector<int> fail, blk;
  rc = factor_dispatch(h->precision, hs, ps, st, h->mem, fail, blk, h->phase_us);
  if ((rc == SLAB_OK || rc == SLAB_E_INVALID) && !fail.empty() && fail[0] != 0) {
    if (info && fail[0] != 1) info->failed_block = blk[0];
    set_error(fail_message(fail[0], blk[0]));
    rc = fail[0] == 1 ? SLAB_E_INVALID : SLAB_E_BREAKDOWN;
  }
  if (rc != SLAB_OK) {
    (void)hipStreamSynchronize(st);
    delete_handle(h);
    return rc;
  }
  *out = h;
  return SLAB_OK;
}

int slab_solve(slab_handle h, const double* f, double* u, int32_t nrhs, int64_t ld,
               void* hip_stream, slab_solve_info* info) {
  return solve_one(h, f, u, nrhs, ld, hip_stream, info, false);
}

int slab_solve_adjoint(slab_handle h, const double* g, double* lam, int32_t nrhs, int64_t ld,
                       void* hip_stream, slab_solve_info* info) {
  return solve_one(h, g, lam, nrhs, ld, hip_stream, info, true);
}

int slab_solve_noalloc(slab_handle h, const double* f, double* u, int32_t nrhs, int64_t ld,
                       void* hip_stream, slab_solve_info* info) {
  return solve_noalloc(h, f, u, nrhs, ld, hip_stream, info);
}

int slab_free(slab_handle h) {
  if (!h) return SLAB_OK;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  delete_handle(h);
  return SLAB_OK;
}

// ---- batches ------------------------------------------------------------------

int slab_batch_free(slab_batch bt) {
  if (!bt) return SLAB_OK;
  (void)hipSetDevice(bt->device);
  (void)hipDeviceSynchronize();
  for (GraphCache& g : bt->graphs) g.clear(bt->mem);
  bt->run.clear(bt->mem);
  for (slab_handle h : bt->items) delete_handle(h);
  bt->mem.release_all();
  delete bt;
  return SLAB_OK;
}

int slab_factor_batch(const slab_problem* probs, int32_t count, const slab_options* opts,
                      void* hip_stream, slab_batch* out, slab_solve_info* infos) {
  if (!out) { set_error("null output batch pointer"); return SLAB_E_INVALID; }
  *out = nullptr;
  if (!probs || count < 1) { set_error("need count >= 1 problems"); return SLAB_E_INVALID; }
  for (int i = 0; i < count; ++i) {
    if (infos) { infos[i].iterations = 0; infos[i].max_relres = 0.0; infos[i].failed_block = -1; }
    const int rc = slab_check_problem(&probs[i], opts);
    if (rc) {
      set_error("problem " + std::to_string(i) + ": " + g_last_error);
      return rc;
    }
  }
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) { set_error("no HIP device"); return SLAB_E_HIP; }
  std::vector<slab_problem> tuned(probs, probs + count);
  std::vector<char> autotuned(count, 0);
  for (int i = 0; i < count; ++i) {
    if (tuned[i].b != 0) continue;
    const int rc = slab_autotune(&probs[i], opts, 1, hip_stream, &tuned[i].b, nullptr);
    if (rc) return rc;
    autotuned[i] = 1;
  }
  probs = tuned.data();
  slab_batch bt = new slab_batch_s();
  bt->device = device;
  bt->precision = opts ? opts->precision : SLAB_FP64;
  bt->flags = opts ? opts->flags : 0;
  std::vector<const slab_problem*> ps;
  for (int i = 0; i < count; ++i) {
    slab_handle h = new_handle(&probs[i], opts, device);
    if (autotuned[i] && h->tile == 0 && h->precision != SLAB_FP64) h->tile = cached_tile(h->n2);
    bt->items.push_back(h);
    ps.push_back(&probs[i]);
  }
  hipStream_t st = (hipStream_t)hip_stream;
  std::vector<int> fail, blk;
  int rc = factor_dispatch(bt->precision, bt->items, ps, st, bt->mem, fail, blk, bt->phase_us);
  if (rc == SLAB_OK || rc == SLAB_E_INVALID) {
    for (int i = 0; i < count && i < (int)fail.size(); ++i) {
      if (fail[i] == 0) continue;
      if (infos && fail[i] != 1) infos[i].failed_block = blk[i];
      set_error("problem " + std::to_string(i) + ": " + fail_message(fail[i], blk[i]));
      rc = fail[i] == 1 ? SLAB_E_INVALID : SLAB_E_BREAKDOWN;
      break;
    }
  }
  if (rc != SLAB_OK) {
    (void)hipStreamSynchronize(st);
    const std::string msg = g_last_error;
    slab_batch_free(bt);
    set_error(msg);
    return rc;
  }
  *out = bt;
  return SLAB_OK;
}

}  // extern "C"

namespace {

int solve_batch(slab_batch bt, const double* const* f, double* const* u, const int32_t* nrhs,
                const int64_t* ld, void* hip_stream, slab_solve_info* infos, bool trans) {
  if (!bt || !f || !u || !nrhs || !ld) { set_error("null argument"); return SLAB_E_INVALID; }
  std::vector<SolveJob> jobs;
  for (size_t i = 0; i < bt->items.size(); ++i) {
    const int rc = check_vec_args(bt->items[i], f[i], u[i], nrhs[i], ld[i]);
    if (rc) {
      set_error("problem " + std::to_string(i) + ": " + g_last_error);
      return rc;
    }
    jobs.push_back({bt->items[i], f[i], u[i], nrhs[i], (long long)ld[i],
                    infos ? &infos[i] : nullptr});
  }
  SLAB_HIP_CHECK(hipSetDevice(bt->device));
  hipStream_t st = (hipStream_t)hip_stream;
  if (!(bt->flags & SLAB_GRAPH)) return solve_group(jobs, bt->precision, trans, st, bt->mem);
  // stream capture needs a stream other than the legacy default stream
  // (work queued on the default stream, e.g. the inputs, is finished first)
  hipStream_t cs = st;
  if (!cs) {
    SLAB_HIP_CHECK(hipStreamSynchronize(st));
    SLAB_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  }
  const int rc = solve_batch_graph(bt, jobs, trans, cs);
  if (!st) {
    (void)hipStreamSynchronize(cs);
    (void)hipStreamDestroy(cs);
  }
  return rc;
}

}  // namespace

extern "C" {

int slab_solve_batch(slab_batch bt, const double* const* f, double* const* u, const int32_t* nrhs,
                     const int64_t* ld, void* hip_stream, slab_solve_info* infos) {
  return solve_batch(bt, f, u, nrhs, ld, hip_stream, infos, false);
}

int slab_solve_adjoint_batch(slab_batch bt, const double* const* g, double* const* lam,
                             const int32_t* nrhs, const int64_t* ld, void* hip_stream,
                             slab_solve_info* infos) {
  return solve_batch(bt, g, lam, nrhs, ld, hip_stream, infos, true);
}

int slab_batch_run(slab_batch bt, const double* const* kappa, const double* const* f,
                   double* const* u, const int32_t* nrhs, const int64_t* ld, void* hip_stream,
                   slab_solve_info* infos) {
  if (!bt || !kappa || !f || !u || !nrhs || !ld) { set_error("null argument"); return SLAB_E_INVALID; }
  std::vector<SolveJob> jobs;
  std::vector<const double*> coefs;
  for (size_t i = 0; i < bt->items.size(); ++i) {
    const int rc = check_vec_args(bt->items[i], f[i], u[i], nrhs[i], ld[i]);
    if (rc || !kappa[i]) {
      set_error("problem " + std::to_string(i) + ": " +
                (rc ? g_last_error : std::string("null coefficient pointer")));
      return SLAB_E_INVALID;
    }
    if (infos) { infos[i].iterations = 0; infos[i].max_relres = 0.0; infos[i].failed_block = -1; }
    jobs.push_back({bt->items[i], f[i], u[i], nrhs[i], (long long)ld[i],
                    infos ? &infos[i] : nullptr});
    coefs.push_back(kappa[i]);
  }
  SLAB_HIP_CHECK(hipSetDevice(bt->device));
  hipStream_t st = (hipStream_t)hip_stream;
  // stream capture needs a stream other than the legacy default stream
  hipStream_t cs = st;
  if (!cs) {
    SLAB_HIP_CHECK(hipStreamSynchronize(st));
    SLAB_HIP_CHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  }
  auto body = [&]() -> int {
    {
      std::vector<std::pair<slab_handle, int>> need;
      for (SolveJob& j : jobs) need.push_back({j.h, j.nrhs});
      SLAB_TRY(ensure_workspaces(need, bt->mem));
    }
    ConvPtrs c;
    SLAB_TRY(batch_conv(bt, &c));
    std::vector<long long> key = jobs_key(jobs, 2);
    for (const double* k : coefs) key.push_back((long long)(uintptr_t)k);
    auto build = [&](Plan& p) {
      SLAB_TRY(plan_factor_nosync_dispatch(bt->precision, p, bt->items, coefs, bt->mem,
                                           &bt->run_temps, &bt->run_temps_cap));
      plan_all_passes(p, jobs, bt->precision, false, c, true);
      for (const SolveJob& j : jobs) count_launches(j.h, p);
      return SLAB_OK;
    };
    SLAB_TRY(launch_graph(bt->mem, &bt->run, key, build, cs));
    std::vector<int> it, fstat;
    std::vector<double> worst;
    SLAB_TRY(read_conv(bt, cs, it, worst, &fstat));
    // an invalid field first (the factorization of such a field breaks down too)
    for (size_t i = 0; i < jobs.size(); ++i) {
      if (fstat[4 * i + 2] == 0) continue;
      set_error("problem " + std::to_string(i) + ": " + fail_message(1, -1));
      return SLAB_E_INVALID;
    }
    for (size_t i = 0; i < jobs.size(); ++i) {
      if (fstat[4 * i] == 0) continue;
      if (infos) infos[i].failed_block = fstat[4 * i + 1];
      set_error("problem " + std::to_string(i) + ": " + fail_message(fstat[4 * i], fstat[4 * i + 1]));
      return SLAB_E_BREAKDOWN;
    }
    return finish_jobs(jobs, it, worst);
  };
  const int rc = body();
  if (!st) {
    (void)hipStreamSynchronize(cs);
    (void)hipStreamDestroy(cs);
  }
  return rc;
}

int slab_kappa_grad_batch(slab_batch bt, const double* const* u, const double* const* lam,
                          const int32_t* nrhs, const int64_t* ld, int32_t mode,
                          double* const* grad, void* hip_stream) {
  if (!bt || !u || !lam || !nrhs || !ld || !grad || (mode != 0 && mode != 1)) {
    set_error("bad arguments to slab_kappa_grad_batch");
    return SLAB_E_INVALID;
  }
  for (size_t i = 0; i < bt->items.size(); ++i) {
    slab_handle h = bt->items[i];
    if (!u[i] || !lam[i] || !grad[i] || nrhs[i] <= 0 || ld[i] < (long long)h->n1 * h->n2) {
      set_error("bad arguments to slab_kappa_grad_batch in problem " + std::to_string(i));
      return SLAB_E_INVALID;
    }
  }
  hipStream_t st = (hipStream_t)hip_stream;
  SLAB_HIP_CHECK(hipSetDevice(bt->device));
  for (size_t i = 0; i < bt->items.size(); ++i) {
    slab_handle h = bt->items[i];
    SLAB_TRY(launch_kappa_grad(h->n1, h->n2, nrhs[i], ld[i], h->h, h->kappa, u[i], lam[i], mode,
                               grad[i], st));
  }
  SLAB_HIP_CHECK(hipStreamSynchronize(st));
  return SLAB_OK;
}

int slab_batch_handle(slab_batch bt, int32_t i, slab_handle* out) {
  if (!bt || !out || i < 0 || i >= (int)bt->items.size()) { set_error("bad batch index"); return SLAB_E_INVALID; }
  *out = bt->items[i];
  return SLAB_OK;
}

int slab_batch_query(slab_batch bt, int32_t what, int64_t* value) {
  if (!bt || !value) { set_error("null argument"); return SLAB_E_INVALID; }
  if (what == 0) { *value = (int64_t)bt->items.size(); return SLAB_OK; }
  if (what == 5) {
    int64_t tot = (int64_t)bt->mem.bytes;
    for (slab_handle h : bt->items) tot += (int64_t)h->mem.bytes;
    *value = tot;
    return SLAB_OK;
  }
  if (what >= 10 && what < 16) { *value = bt->phase_us[what - 10]; return SLAB_OK; }
  set_error("unknown query");
  return SLAB_E_INVALID;
}

// ---- auxiliary ----------------------------------------------------------------

int slab_release_cache(void) {
  int dev = 0;
  SLAB_HIP_CHECK(hipGetDevice(&dev));
  SLAB_HIP_CHECK(hipDeviceSynchronize());
  Pool::get().trim(dev);
  return SLAB_OK;
}

int slab_index_maps(int32_t n1, int32_t n2, int32_t b, int32_t* col_kind, int32_t* slab_of_col,
                    int32_t* local_of_col, int64_t* perm_even, int64_t* perm_odd,
                    void* hip_stream) {
  if (n2 < 1 || n1 < 2 || b < 1 || n1 % (b + 1) != 0) {
    set_error("bad grid for index maps");
    return SLAB_E_INVALID;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  SLAB_TRY(launch_maps(n1, n2, b, col_kind, slab_of_col, local_of_col, perm_even, perm_odd, st));
  SLAB_HIP_CHECK(hipStreamSynchronize(st));
  return SLAB_OK;
}

int slab_kappa_grad(slab_handle h, const double* u, const double* lam, int32_t nrhs, int64_t ld,
                    int32_t mode, double* grad, void* hip_stream) {
  if (!h || !u || !lam || !grad || nrhs <= 0 || ld < (long long)h->n1 * h->n2 ||
      (mode != 0 && mode != 1)) {
    set_error("bad arguments to slab_kappa_grad");
    return SLAB_E_INVALID;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  SLAB_HIP_CHECK(hipSetDevice(h->device));
  SLAB_TRY(launch_kappa_grad(h->n1, h->n2, nrhs, ld, h->h, h->kappa, u, lam, mode, grad, st));
  SLAB_HIP_CHECK(hipStreamSynchronize(st));
  return SLAB_OK;
}

int slab_dirichlet_load(slab_handle h, const double* g, double* f, int32_t nrhs, int64_t ld,
                        void* hip_stream) {
  if (!h || !g || !f || nrhs <= 0 || ld < (long long)h->n1 * h->n2) {
    set_error("bad arguments to slab_dirichlet_load");
    return SLAB_E_INVALID;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  SLAB_HIP_CHECK(hipSetDevice(h->device));
  SLAB_TRY(launch_dirichlet(h->n1, h->n2, nrhs, ld, h->wh, h->wv, g, f, st));
  return SLAB_OK;
}

int slab_residual(slab_handle h, const double* f, const double* u, int32_t nrhs, int64_t ld,
                  double* relres, void* hip_stream) {
  if (!relres) { set_error("null relres"); return SLAB_E_INVALID; }
  if (!h || !f || !u || nrhs <= 0 || ld < (long long)h->n1 * h->n2) {
    set_error("bad arguments to slab_residual");
    return SLAB_E_INVALID;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  SLAB_HIP_CHECK(hipSetDevice(h->device));
  SLAB_TRY(ensure_workspace(h, nrhs));
  SolveDev d;
  std::memset(&d, 0, sizeof(d));
  d.n1 = h->n1; d.n2 = h->n2; d.b = h->b; d.m = h->m; d.nrhs = nrhs;
  d.wh = h->wh; d.wv = h->wv; d.f = f; d.u = u; d.r = nullptr; d.ldf = ld;
  d.shift = h->shift; d.shift_stride = h->shift_src ? 1 : 0;
  d.norms = h->ws.norms; d.partial = h->ws.partial;
  Plan p;
  plan_residual(p, std::vector<SolveDev>{d});
  SLAB_TRY(run_plan(h->mem, p, st));
  std::vector<SolveJob> jobs{{h, f, nullptr, nrhs, ld, nullptr}};
  std::vector<std::vector<double>> rr;
  SLAB_TRY(read_relres(jobs, st, rr));
  for (int c = 0; c < nrhs; ++c) relres[c] = rr[0][c];
  return SLAB_OK;
}

int slab_apply_reduced(slab_handle h, const double* x, double* y, int32_t ncols,
                       void* hip_stream) {
  if (!h || !x || !y || ncols < 1) { set_error("bad arguments to slab_apply_reduced"); return SLAB_E_INVALID; }
  const long long span = (long long)h->m * ncols * h->n2 * 8;
  if ((const char*)x < (const char*)y + span && (const char*)y < (const char*)x + span) {
    set_error("x and y overlap");
    return SLAB_E_INVALID;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  SLAB_HIP_CHECK(hipSetDevice(h->device));
  SLAB_TRY(ensure_workspace(h, ncols));
  SolveDev d;
  std::memset(&d, 0, sizeof(d));
  const long long N = (long long)h->n1 * h->n2;
  d.n1 = h->n1; d.n2 = h->n2; d.b = h->b; d.m = h->m; d.nrhs = ncols;
  d.wh = h->wh; d.wv = h->wv; d.Gl = h->Gl;
  d.shift = h->shift; d.shift_stride = h->shift_src ? 1 : 0;
  d.zbuf = h->ws.zbuf; d.xb = h->ws.xb; d.ft = h->ws.ft;
  d.rhs = h->ws.r; d.ld = N; d.r = h->ws.r; d.u = x; d.g64 = y;
  Plan p;
  if (h->precision == SLAB_FP32_REFINE) plan_reduced_apply<float, float>(p, {d});
  else if (h->precision == SLAB_MIXED) plan_reduced_apply<double, float>(p, {d});
  else plan_reduced_apply<double, double>(p, {d});
  SLAB_TRY(run_plan(h->mem, p, st));
  SLAB_HIP_CHECK(hipStreamSynchronize(st));
  return SLAB_OK;
}

int slab_export_reduced(slab_handle h, int32_t which, int32_t j, double* out, void* hip_stream) {
  if (!h || !out) { set_error("null argument"); return SLAB_E_INVALID; }
  if (!(h->flags & SLAB_KEEP_REDUCED)) { set_error("factor without SLAB_KEEP_REDUCED"); return SLAB_E_INVALID; }
  const int limit = which == 1 ? h->m - 1 : h->m;
  if (which < 0 || which > 2 || j < 0 || j >= limit) { set_error("bad block index"); return SLAB_E_INVALID; }
  const size_t nsq = (size_t)h->n2 * h->n2;
  const double* src = which == 0 ? h->T64 : (which == 1 ? h->O64 : h->S64);
  hipStream_t st = (hipStream_t)hip_stream;
  SLAB_HIP_CHECK(hipMemcpyAsync(out, src + (size_t)j * nsq, nsq * sizeof(double),
                                hipMemcpyDeviceToDevice, st));
  SLAB_HIP_CHECK(hipStreamSynchronize(st));
  return SLAB_OK;
}

int slab_query(slab_handle h, int32_t what, int64_t* value) {
  if (!h || !value) { set_error("null argument"); return SLAB_E_INVALID; }
  switch (what) {
    case 0: *value = h->m; return SLAB_OK;
    case 1: *value = h->n1; return SLAB_OK;
    case 2: *value = h->n2; return SLAB_OK;
    case 3: *value = h->b; return SLAB_OK;
    case 4: *value = h->precision; return SLAB_OK;
    case 5: *value = (int64_t)h->mem.bytes; return SLAB_OK;
    case 6: *value = h->tile; return SLAB_OK;
    case 7: {  // negative pivots of the signed block factorization (0 without one)
      *value = 0;
      if (!h->J) return SLAB_OK;
      SLAB_HIP_CHECK(hipSetDevice(h->device));
      const size_t cnt = (size_t)h->m * h->n2;
      std::vector<char> sg(cnt * h->esz2);
      SLAB_HIP_CHECK(hipMemcpy(sg.data(), h->J, sg.size(), hipMemcpyDeviceToHost));
      int64_t neg = 0;
      for (size_t i = 0; i < cnt; ++i)
        neg += h->esz2 == 8 ? (((const double*)sg.data())[i] < 0) : (((const float*)sg.data())[i] < 0);
      *value = neg;
      return SLAB_OK;
    }
    case 8: *value = (int64_t)(intptr_t)h->Gl; return SLAB_OK;
    default:
      if (what >= 10 && what < 16) { *value = h->phase_us[what - 10]; return SLAB_OK; }
      if (what >= 20 && what < 20 + LK_COUNT) { *value = h->launches[what - 20]; return SLAB_OK; }
  }
  set_error("unknown query");
  return SLAB_E_INVALID;
}

}  // extern "C"
