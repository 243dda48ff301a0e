// C ABI of the slab solver: argument checks, device memory of a handle, phase
// orchestration of Alg. 3 (factor) and Alg. 4 (solve) with FP64 iterative
// refinement around the working-precision solve.
#include "launch.h"

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

namespace slab {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

}  // namespace slab

using namespace slab;

struct Workspace {
  int nrhs = 0;
  void* zbuf = nullptr;
  void* xb = nullptr;
  void* ft = nullptr;
  void* yt = nullptr;
  void* tt = nullptr;
  double* r = nullptr;
  double* norms = nullptr;
  double* partial = nullptr;
};

struct slab_handle_s {
  int n1 = 0, n2 = 0, b = 0, m = 0, BP = 0;
  double h = 0.0;
  int precision = SLAB_FP64;
  double tol = 1e-10;
  int max_iter = 10;
  int flags = 0;
  int device = 0;
  size_t esz = 8;   // slab factors / Schur pieces / slab sweeps
  size_t esz2 = 8;  // reduced system: T blocks, block factorization, Alg. 2
  double* kappa = nullptr;
  double* wh = nullptr;
  double* wv = nullptr;
  int* status = nullptr;
  void* Gl = nullptr;
  void* Linv = nullptr;
  void* Z = nullptr;
  void* Td = nullptr;  // odd-even order: U_e blocks (kept for the solve)
  int odd_even = 0;
  double* T64 = nullptr;
  double* O64 = nullptr;
  double* S64 = nullptr;
  size_t bytes = 0;
  long long phase_us[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<void*> owned;
  Workspace ws;
};

namespace {

int dev_alloc(slab_handle h, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation of " + std::to_string(bytes) + " bytes failed: " +
              hipGetErrorString(e));
    *p = nullptr;
    return SLAB_E_NOMEM;
  }
  h->owned.push_back(*p);
  h->bytes += bytes;
  return SLAB_OK;
}

void dev_release(slab_handle h, void* p) {
  if (!p) return;
  for (size_t i = 0; i < h->owned.size(); ++i)
    if (h->owned[i] == p) {
      (void)hipFree(p);
      h->owned.erase(h->owned.begin() + i);
      return;
    }
}

void release_all(slab_handle h) {
  for (void* p : h->owned) (void)hipFree(p);
  h->owned.clear();
}

#define SLAB_TRY(expr)           \
  do {                           \
    int rc_ = (expr);            \
    if (rc_ != SLAB_OK) return rc_; \
  } while (0)

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

int ensure_workspace(slab_handle h, int nrhs, hipStream_t st) {
  Workspace& w = h->ws;
  if (w.nrhs >= nrhs) return SLAB_OK;
  void* ptrs[] = {w.zbuf, w.xb, w.ft, w.yt, w.tt, w.r, w.norms, w.partial};
  for (void* p : ptrs) dev_release(h, p);
  w = Workspace();
  const size_t n = h->n2, m = h->m, e = h->esz, e2 = h->esz2;
  const size_t N = (size_t)h->n1 * h->n2;
  SLAB_TRY(dev_alloc(h, &w.zbuf, m * nrhs * n * h->BP * e));
  SLAB_TRY(dev_alloc(h, &w.xb, m * 2 * nrhs * n * e));
  SLAB_TRY(dev_alloc(h, &w.ft, m * nrhs * n * e2));
  SLAB_TRY(dev_alloc(h, &w.yt, m * nrhs * n * e2));
  SLAB_TRY(dev_alloc(h, &w.tt, nrhs * n * e2));
  SLAB_TRY(dev_alloc(h, (void**)&w.r, nrhs * N * sizeof(double)));
  SLAB_TRY(dev_alloc(h, (void**)&w.norms, 2 * nrhs * sizeof(double)));
  SLAB_TRY(dev_alloc(h, (void**)&w.partial, residual_partial_count(h->n1, h->n2, nrhs) * sizeof(double)));
  w.nrhs = nrhs;
  return SLAB_OK;
}

SolveArgs solve_args(slab_handle h, int nrhs, int transpose) {
  SolveArgs a;
  a.n1 = h->n1; a.n2 = h->n2; a.b = h->b; a.m = h->m; a.nrhs = nrhs;
  a.wh = h->wh; a.wv = h->wv; a.Gl = h->Gl; a.Linv = h->Linv; a.Z = h->Z; a.Td = h->Td;
  a.zbuf = h->ws.zbuf; a.xb = h->ws.xb; a.ft = h->ws.ft; a.yt = h->ws.yt; a.tt = h->ws.tt;
  a.transpose = transpose;
  a.odd_even = h->odd_even;
  return a;
}

int solve_pass(slab_handle h, const SolveArgs& a, const double* rhs, long long ldr, double* out,
               long long ldo, int acc, hipStream_t st) {
  if (h->precision == SLAB_FP32_REFINE)
    return launch_solve_pass<float, float>(a, rhs, ldr, out, ldo, acc, st);
  if (h->precision == SLAB_MIXED)
    return launch_solve_pass<double, float>(a, rhs, ldr, out, ldo, acc, st);
  return launch_solve_pass<double, double>(a, rhs, ldr, out, ldo, acc, st);
}

int residual_host(slab_handle h, const double* f, const double* u, int nrhs, long long ld,
                  double* r, std::vector<double>& relres, hipStream_t st) {
  SLAB_TRY(launch_residual(h->n1, h->n2, nrhs, ld, h->wh, h->wv, f, u, r,
                           (long long)h->n1 * h->n2, h->ws.norms, h->ws.partial, st));
  std::vector<double> nrm(2 * nrhs);
  SLAB_HIP_CHECK(hipMemcpyAsync(nrm.data(), h->ws.norms, 2 * nrhs * sizeof(double),
                                hipMemcpyDeviceToHost, st));
  SLAB_HIP_CHECK(hipStreamSynchronize(st));
  relres.resize(nrhs);
  for (int c = 0; c < nrhs; ++c) {
    const double fn = std::sqrt(nrm[2 * c + 1]);
    relres[c] = fn > 0 ? std::sqrt(nrm[2 * c]) / fn : std::sqrt(nrm[2 * c]);
  }
  return SLAB_OK;
}

// Alg. 4 with FP64 refinement: u = 0, r = f; repeat { d = solve(r); u += d; r = f - A u }.
int solve_common(slab_handle h, const double* f, double* u, int32_t nrhs, int64_t ld,
                 void* stream, slab_solve_info* info, int transpose) {
  SLAB_TRY(check_vec_args(h, f, u, nrhs, ld));
  hipStream_t st = (hipStream_t)stream;
  SLAB_HIP_CHECK(hipSetDevice(h->device));
  SLAB_TRY(ensure_workspace(h, nrhs, st));
  const SolveArgs a = solve_args(h, nrhs, transpose);
  const long long N = (long long)h->n1 * h->n2;
  std::vector<double> rr;
  int it = 0;
  double worst = 0.0;
  SLAB_TRY(solve_pass(h, a, f, ld, u, ld, 0, st));
  ++it;
  while (true) {
    // the transposed residual equals A^T u = A u (A is symmetric)
    SLAB_TRY(residual_host(h, f, u, nrhs, ld, h->ws.r, rr, st));
    worst = 0.0;
    bool finite = true;
    for (double v : rr) {
      if (!std::isfinite(v)) finite = false;
      worst = std::max(worst, v);
    }
    if (!finite) worst = NAN;
    if (!finite || worst <= h->tol || it >= h->max_iter) break;
    SLAB_TRY(solve_pass(h, a, h->ws.r, N, u, ld, 1, st));
    ++it;
  }
  SLAB_HIP_CHECK(hipStreamSynchronize(st));
  if (info) {
    info->iterations = it;
    info->max_relres = worst;
    info->failed_block = -1;
  }
  if (!(worst <= h->tol)) {
    set_error("refinement stopped at relative residual " + std::to_string(worst) + " after " +
              std::to_string(it) + " passes (tol " + std::to_string(h->tol) + ")");
    return SLAB_E_NOCONV;
  }
  return SLAB_OK;
}

long long elapsed_us(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return -1;
  return (long long)(ms * 1000.0f);
}

template <typename T, typename TR>
int factor_impl(slab_handle h, const slab_problem* prob, hipStream_t st, slab_solve_info* info) {
  const size_t n = h->n2, m = h->m, e = sizeof(T), e2 = sizeof(TR), BP = h->BP;
  const size_t nsq = n * n;
  const size_t ncoef = (size_t)(h->n1 + 2) * (h->n2 + 2);
  SLAB_TRY(dev_alloc(h, (void**)&h->kappa, ncoef * sizeof(double)));
  SLAB_TRY(dev_alloc(h, (void**)&h->wh, (size_t)(h->n1 + 1) * n * sizeof(double)));
  SLAB_TRY(dev_alloc(h, (void**)&h->wv, (size_t)h->n1 * (n + 1) * sizeof(double)));
  SLAB_TRY(dev_alloc(h, (void**)&h->status, 4 * sizeof(int)));
  SLAB_TRY(dev_alloc(h, &h->Gl, m * n * BP * BP * e));
  void *Hsw, *sig, *PRR, *PLL, *PLR, *PRL, *Td, *To;
  SLAB_TRY(dev_alloc(h, &Hsw, m * n * BP * BP * e));
  SLAB_TRY(dev_alloc(h, &sig, m * n * 2 * BP * e));
  SLAB_TRY(dev_alloc(h, &PRR, m * nsq * e));
  SLAB_TRY(dev_alloc(h, &PLL, m * nsq * e));
  SLAB_TRY(dev_alloc(h, &PLR, m * nsq * e));
  SLAB_TRY(dev_alloc(h, &PRL, m * nsq * e));
  SLAB_TRY(dev_alloc(h, &Td, m * nsq * e2));
  SLAB_TRY(dev_alloc(h, &To, (m > 1 ? m - 1 : 1) * nsq * e2));
  SLAB_TRY(dev_alloc(h, &h->Linv, m * nsq * e2));
  SLAB_TRY(dev_alloc(h, &h->Z, (m > 1 ? m - 1 : 1) * nsq * e2));
  if (h->flags & SLAB_KEEP_REDUCED) {
    SLAB_TRY(dev_alloc(h, (void**)&h->T64, m * nsq * sizeof(double)));
    SLAB_TRY(dev_alloc(h, (void**)&h->O64, (m > 1 ? m - 1 : 1) * nsq * sizeof(double)));
    SLAB_TRY(dev_alloc(h, (void**)&h->S64, m * nsq * sizeof(double)));
  }
  hipEvent_t ev[6];
  for (int i = 0; i < 6; ++i) SLAB_HIP_CHECK(hipEventCreate(&ev[i]));
  SLAB_HIP_CHECK(hipMemsetAsync(h->status, 0, 4 * sizeof(int), st));
  SLAB_HIP_CHECK(hipEventRecord(ev[0], st));
  SLAB_TRY(launch_coef_weights(prob->kappa, (h->flags & SLAB_COEF_LOG) ? 1 : 0, h->n1, h->n2, h->h,
                               h->kappa, h->wh, h->wv, h->status, st));
  int hs[4] = {0, 0, 0, 0};
  SLAB_HIP_CHECK(hipMemcpyAsync(hs, h->status, sizeof(hs), hipMemcpyDeviceToHost, st));
  SLAB_HIP_CHECK(hipStreamSynchronize(st));
  if (hs[0] == 1) {
    set_error("coefficient field has a value that is not positive and finite");
    return SLAB_E_INVALID;
  }
  Stage1Args A;
  A.n1 = h->n1; A.n2 = h->n2; A.b = h->b; A.m = h->m;
  A.wh = h->wh; A.wv = h->wv; A.Gl = h->Gl; A.Hsw = Hsw; A.sig = sig;
  A.PRR = PRR; A.PLL = PLL; A.PLR = PLR; A.PRL = PRL; A.Tdiag = Td; A.Toff = To;
  A.Tdiag64 = h->T64; A.Toff64 = h->O64; A.status = h->status;
  A.ev[0] = ev[1]; A.ev[1] = ev[2]; A.ev[2] = ev[3]; A.ev[3] = ev[4];
  SLAB_TRY((launch_stage1<T, TR>(A, st)));
  Stage2Args B;
  B.n = h->n2; B.m = h->m; B.Tdiag = Td; B.Toff = To; B.Linv = h->Linv; B.Z = h->Z;
  B.S64 = h->S64; B.status = h->status; B.odd_even = h->odd_even;
  SLAB_TRY(launch_stage2<TR>(B, st));
  SLAB_HIP_CHECK(hipEventRecord(ev[5], st));
  SLAB_HIP_CHECK(hipMemcpyAsync(hs, h->status, sizeof(hs), hipMemcpyDeviceToHost, st));
  SLAB_HIP_CHECK(hipStreamSynchronize(st));
  // phases: weights + slab factor, boundary columns, Schur propagation (k_schur
  // alone), assembly of T, block factorization
  for (int i = 0; i < 5; ++i) h->phase_us[i] = elapsed_us(ev[i], ev[i + 1]);
  for (int i = 0; i < 6; ++i) (void)hipEventDestroy(ev[i]);
  void* tmp[] = {Hsw, sig, PRR, PLL, PLR, PRL, To};
  for (void* p : tmp) dev_release(h, p);
  if (h->odd_even) h->Td = Td;
  else dev_release(h, Td);
  if (hs[0] != 0) {
    if (info) info->failed_block = hs[1];
    set_error(hs[0] == 2 ? "slab factorization breakdown in slab " + std::to_string(hs[1])
                         : "block factorization breakdown at interface " + std::to_string(hs[1]));
    return SLAB_E_BREAKDOWN;
  }
  return SLAB_OK;
}

}  // namespace

extern "C" {

const char* slab_last_error(void) { return g_last_error.c_str(); }

int slab_check_problem(const slab_problem* prob, const slab_options* opts) {
  if (!prob) { set_error("null problem"); return SLAB_E_INVALID; }
  if (prob->n2 < 1 || prob->n1 < 2 || prob->b < 1 || prob->b > 63) {
    set_error("need n2 >= 1, n1 >= 2, 1 <= b <= 63");
    return SLAB_E_INVALID;
  }
  if (prob->n1 % (prob->b + 1) != 0) { set_error("n1 must be a multiple of b+1"); return SLAB_E_INVALID; }
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
    if (opts->flags & ~(SLAB_KEEP_REDUCED | SLAB_COEF_LOG | SLAB_ODD_EVEN)) { set_error("unknown flag"); return SLAB_E_INVALID; }
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
  slab_handle h = new slab_handle_s();
  h->n1 = prob->n1; h->n2 = prob->n2; h->b = prob->b; h->m = prob->n1 / (prob->b + 1);
  h->BP = padded_block(prob->b); h->h = prob->h;
  if (opts) { h->precision = opts->precision; h->tol = opts->tol; h->max_iter = opts->max_iter; h->flags = opts->flags; }
  h->odd_even = (h->flags & SLAB_ODD_EVEN) ? 1 : 0;
  h->esz = h->precision == SLAB_FP32_REFINE ? 4 : 8;
  h->esz2 = h->precision == SLAB_FP64 ? 8 : 4;
  if (hipGetDevice(&h->device) != hipSuccess) {
    set_error("no HIP device");
    delete h;
    return SLAB_E_HIP;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  if (h->precision == SLAB_FP32_REFINE) rc = factor_impl<float, float>(h, prob, st, info);
  else if (h->precision == SLAB_MIXED) rc = factor_impl<double, float>(h, prob, st, info);
  else rc = factor_impl<double, double>(h, prob, st, info);
  if (rc != SLAB_OK) {
    (void)hipStreamSynchronize(st);
    release_all(h);
    delete h;
    return rc;
  }
  *out = h;
  return SLAB_OK;
}

int slab_solve(slab_handle h, const double* f, double* u, int32_t nrhs, int64_t ld,
               void* hip_stream, slab_solve_info* info) {
  return solve_common(h, f, u, nrhs, ld, hip_stream, info, 0);
}

int slab_solve_adjoint(slab_handle h, const double* g, double* lam, int32_t nrhs, int64_t ld,
                       void* hip_stream, slab_solve_info* info) {
  return solve_common(h, g, lam, nrhs, ld, hip_stream, info, 1);
}

int slab_free(slab_handle h) {
  if (!h) return SLAB_OK;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  release_all(h);
  delete h;
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

int slab_residual(slab_handle h, const double* f, const double* u, int32_t nrhs, int64_t ld,
                  double* relres, void* hip_stream) {
  if (!relres) { set_error("null relres"); return SLAB_E_INVALID; }
  if (!h || !f || !u || nrhs <= 0 || ld < (long long)h->n1 * h->n2) {
    set_error("bad arguments to slab_residual");
    return SLAB_E_INVALID;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  SLAB_HIP_CHECK(hipSetDevice(h->device));
  SLAB_TRY(ensure_workspace(h, nrhs, st));
  std::vector<double> rr;
  SLAB_TRY(residual_host(h, f, u, nrhs, ld, nullptr, rr, st));
  for (int c = 0; c < nrhs; ++c) relres[c] = rr[c];
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
    case 5: *value = (int64_t)h->bytes; return SLAB_OK;
    default:
      if (what >= 10 && what < 15) { *value = h->phase_us[what - 10]; return SLAB_OK; }
  }
  set_error("unknown query");
  return SLAB_E_INVALID;
}

}  // extern "C"
