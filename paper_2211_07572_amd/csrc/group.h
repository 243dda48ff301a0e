// Grouped launches and launch plans.
//
// A grouped launch covers several independent items (problems of a batch,
// pivot blocks of one elimination level, products of one update step) in one
// kernel: item i owns the workgroups [offs[i], offs[i+1]) of blockIdx.x, where
// offs and the item descriptors live in device memory.  A single problem is a
// group of one, so every factorization and solve runs through these kernels.
//
// A Plan collects the descriptor tables of a whole factorization or solve
// pass on the host, uploads them in one copy, and then issues the recorded
// launches in order; a recorded solve pass can be captured into a HIP graph
// and replayed.
#pragma once

#include "common.h"

#include <cstring>
#include <functional>
#include <memory>
#include <vector>

namespace slab {

// Item owning workgroup bx: the largest i with offs[i] <= bx.
__device__ __forceinline__ int group_item(const int* __restrict__ offs, int count, int bx) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= bx) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Workgroups are handed to the eight XCDs round-robin by blockIdx.x, and each
// XCD has an L2 of its own.  This renumbering gives XCD x the contiguous range
// [x*G/8, (x+1)*G/8) of virtual indices (G = gridDim.x; a tail of G % 8
// workgroups keeps its index), so that workgroups running side by side on one
// XCD take neighbouring tiles and share their operand panels in its L2.
__device__ __forceinline__ int xcd_linear(int bx, int G) {
  const int per = G >> 3;
  return bx < (per << 3) ? (bx & 7) * per + (bx >> 3) : bx;
}

// Refinement passes issued ahead of their convergence test (a graph of a fixed
// number of passes) carry a per-problem flag: once a problem's residual has
// met its tolerance (k_converge writes 0), every workgroup of its later
// passes returns at once.  A null flag means the work always runs.
__device__ __forceinline__ bool item_done(const int* live) {
  return live != nullptr && *live == 0;
}

// ---- descriptors ----------------------------------------------------------------

// One problem of stage one (edge weights, slab factors, Schur pieces, assembly).
struct ProbDev {
  int n1, n2, b, m;
  double h;
  int is_log;
  const double* coef;  // caller's field (kappa or theta), read once
  double* kappa;       // working copy
  double* wh;
  double* wv;
  // diagonal term c_p of the operator (the Helmholtz term of eq. (var_helm)):
  // shift_src is the caller's n1 x n2 field or null; shift the working copy
  // (n1 x n2 entries with shift_stride 1, or one zero with stride 0)
  const double* shift_src;
  double* shift;
  long long shift_stride;
  void* Gl;
  void* Hsw;
  void* sig;
  void* PRR;
  void* PLL;
  void* PLR;
  void* PRL;
  void* Td;            // T_jj (reduced precision)
  void* To;            // T_{j,j+1}
  double* T64;         // optional FP64 copies
  double* O64;
  int* status;
  // segmented slab recursion (k_slab_factor): the n2 row steps of a chain are
  // cut into fnseg segments of fseg steps; a segment after the first starts
  // fwarm steps early from a zero inverse and stores only its own rows, plus
  // its warm-up's last block into fchk ([slab][dir][segment][BP][BP]) for the
  // check against the previous segment; fredo[slab*2+dir] = 1 marks a chain
  // whose warm-up did not converge (recomputed in one piece)
  int fnseg, fseg, fwarm;
  void* fchk;
  int* fredo;
};

// One pivot block of the block factorization.
struct FactorItem {
  void* S;        // n x n, lower triangle; overwritten by L
  void* Li;       // n x n, receives L^-1 (L J L^T = S)
  double* S64;    // optional FP64 copy of S before the factorization
  void* J = nullptr;  // n entries: the signs of the pivots, J = diag(+-1)
  int* status;
  int n;
  int blk;        // interface index reported on breakdown
  int indef = 0;      // 1: negative pivots are allowed (S symmetric indefinite)
};

// One product C = beta C + alpha op(A) op(B) (row-major, leading dimensions).
struct GemmItem {
  const void* A;
  const void* B;
  void* C;
  int M, N, K;
  int lda, ldb, ldc;
  // optional: op(A)(i, k) is taken times kscale[k] (the signs J of an
  // L J L^T factorization between the two operands); all items of a launch
  // have one or none
  const void* kscale = nullptr;
};

// One block-vector product y = beta xin + alpha op(M) x over nrhs columns.
struct BmvItem {
  const void* M;
  const void* x;
  const void* xin;  // may be null or equal to y
  void* y;
  int n;
  int nrhs;
  // scratch for a product split over k (BMV_SPLIT_MAX partial results of
  // 16*ceil(nrhs/16) columns of n), or null: the product is not split
  void* part;
  const int* live;  // refinement flag of the problem (see item_done), or null
  // optional: x(k) is taken times xscale[k] (pivot signs J); all items of a
  // launch have one or none
  const void* xscale = nullptr;
};

// Most k-splits of a small block-vector launch; scratch per item in elements.
constexpr int BMV_SPLIT_MAX = 8;
// Items of one problem in one launch that get a scratch (more: not split).
constexpr int BMV_PART_SLOTS = 4;
inline long long bmv_part_elems(int n, int nrhs) {
  return (long long)BMV_SPLIT_MAX * 16 * ((nrhs + 15) / 16) * n;
}

// One problem of a solve pass (slab sweeps, reduced right-hand side,
// coupling, interface output, residual).
struct SolveDev {
  int n1, n2, b, m, nrhs;
  int accumulate;
  long long ld;    // rhs leading dimension
  long long ldo;   // out leading dimension
  const double* wh;
  const double* wv;
  const double* shift;       // diagonal term c_p (see ProbDev), index p * shift_stride
  long long shift_stride;
  const void* Gl;
  void* zbuf;
  void* xb;
  void* ft;
  const double* rhs;
  double* out;
  // residual r = f - A u and per-column norms
  const double* f;
  const double* u;
  double* r;
  long long ldf;   // f and u leading dimension
  double* norms;
  double* partial;
  // refined reduced solve (FP64 reduced right-hand side out, FP64 interface
  // values in); null when the reduced system is solved in one go
  double* g64;
  const double* uo64;
  const int* live;  // refinement flag of the problem (see item_done), or null
};

// Convergence test of one problem after a refinement pass (k_converge).
struct ConvDev {
  const double* norms;  // per column: sum r^2, sum f^2
  int nrhs;
  int max_iter;
  double tol;
  int* live;      // out: 1 while another pass is needed
  int* iters;     // passes done
  double* relres; // max over columns of ||r|| / ||f|| after the last pass
  const int* fstatus;  // optional: the problem's four factorization status
  int* fstatus_out;    // words, copied beside the counts on the first pass
};

// Reduced system of one problem in a solve pass (block factors from stage two
// and the reduced vectors, nrhs columns of n at [j][c][r]).
struct ReducedDev {
  int n, m, nrhs;
  const void* Linv;
  const void* Z;
  const void* Td;   // odd-even order: the U_e blocks
  void* ft;         // in: f~, out: the interface values
  void* yt;
  void* tt;         // nrhs x n temporary
  void* part;       // BMV_PART_SLOTS partial-product scratches (bmv_part_elems each)
  const void* J;    // pivot signs (m blocks of n), or null: all +1 (L L^T)
  // refinement against the FP64 reduced matrix (null T64: none): diagonal
  // blocks T64[j], couplings O64[j] = T_{j,j+1}; FP64 right-hand side g64,
  // solution u64 and residual r64, all [j][c][r]
  const double* T64;
  const double* O64;
  double* g64;
  double* u64;
  double* r64;
  const int* live;  // refinement flag of the problem (see item_done), or null
};

// Stage two of one problem (see plan_stage2).
struct Stage2Prob {
  int n, m;
  void* Td;
  void* To;
  void* Linv;
  void* Z;        // m-1 blocks: Z_j (Alg. 1) or V_e (odd-even)
  double* S64;
  void* J = nullptr;  // m blocks of n pivot signs
  int indef = 0;      // signed (L J L^T) factorization of every pivot block
  int* status;
};

// ---- host-side plan -----------------------------------------------------------

// Kinds of launches a plan counts (reported per handle by slab_query).
enum LaunchKind {
  LK_GEMM128 = 0,   // block products on 128-wide tiles
  LK_GEMM64 = 1,    // block products on 64-wide tiles
  LK_GEMM_CPRE = 2, // factorization updates with the C tile prefetched
  LK_BMV_SPLIT = 3, // block-vector products split over k (+ the partial-sum launch)
  LK_BMV = 4,       // block-vector products in one launch
  LK_COUNT = 8
};

class Plan {
 public:
  // Stage `bytes` of table data; returns its offset (256-byte aligned).
  size_t add(const void* data, size_t bytes) {
    const size_t off = (host_.size() + 255) & ~size_t(255);
    host_.resize(off + bytes);
    if (bytes) std::memcpy(host_.data() + off, data, bytes);
    return off;
  }
  template <class V>
  size_t add_vec(const std::vector<V>& v) { return add(v.data(), v.size() * sizeof(V)); }

  // Offsets table of a grouped launch from per-item workgroup counts.
  size_t add_offsets(const std::vector<int>& counts, long long* total) {
    std::vector<int> offs(counts.size() + 1, 0);
    long long t = 0;
    for (size_t i = 0; i < counts.size(); ++i) {
      offs[i] = (int)t;
      t += counts[i];
    }
    offs[counts.size()] = (int)t;
    *total = t;
    return add_vec(offs);
  }

  // A recorded launch: receives the device base of the uploaded tables.
  typedef std::function<int(const char* dev, hipStream_t st)> Step;
  void step(Step s) { steps_.push_back(std::move(s)); }

  // Optional timing of one class of launches (the block products of stage
  // two): when set, those launches record an event pair around themselves.
  struct Timer {
    std::vector<hipEvent_t> ev;
    ~Timer() {
      for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    // summed milliseconds of the recorded pairs (after a synchronization)
    double total_ms() const {
      double t = 0.0;
      for (size_t i = 0; i + 1 < ev.size(); i += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) == hipSuccess) t += ms;
      }
      return t;
    }
  };
  std::shared_ptr<Timer> timer;
  // launches recorded so far, by LaunchKind
  long long launches[LK_COUNT] = {0, 0, 0, 0, 0, 0, 0, 0};

  size_t bytes() const { return host_.size(); }
  const char* host() const { return host_.data(); }
  int run(const char* dev, hipStream_t st) const {
    for (const Step& s : steps_) {
      const int rc = s(dev, st);
      if (rc) return rc;
    }
    return 0;
  }

 private:
  std::vector<char> host_;
  std::vector<Step> steps_;
};

template <class V>
inline const V* dev_at(const char* dev, size_t off) { return (const V*)(dev + off); }

}  // namespace slab
