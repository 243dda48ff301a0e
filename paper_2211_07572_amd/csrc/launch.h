// Host-side launchers shared by the slab solver's HIP sources.
#pragma once

#include "common.h"
#include "slab.h"

#include <algorithm>

namespace slab {

// ---- stage one --------------------------------------------------------------
int launch_coef_weights(const double* coef, int is_log, int n1, int n2, double h, double* kappa,
                        double* wh, double* wv, int* status, hipStream_t st);
int launch_maps(int n1, int n2, int b, int32_t* ck, int32_t* sc, int32_t* lc, int64_t* pe,
                int64_t* po, hipStream_t st);

struct Stage1Args {
  int n1, n2, b, m;
  const double* wh;
  const double* wv;
  void* Gl;    // m * n2 * BP * BP, top-down inverses, row-major blocks
  void* Hsw;   // m * n2 * BP * BP, bottom-up propagators, fragment-major
  void* sig;   // m * n2 * 2 * BP, scaled boundary columns of the inverse blocks
  void* PRR;   // m * n2 * n2 each: lower-triangular Schur pieces per slab
  void* PLL;
  void* PLR;
  void* PRL;
  void* Tdiag; // m * n2 * n2, working precision
  void* Toff;  // (m-1) * n2 * n2, T_{j,j+1}
  double* Tdiag64;  // optional FP64 copies
  double* Toff64;
  int* status;
  void* ev[4];      // optional events after slab factor, boundary columns, Schur, assembly
};
// T: slab factors and Schur pieces; TO: the assembled T blocks (block factorization).
template <typename T, typename TO> int launch_stage1(const Stage1Args& a, hipStream_t st);

// ---- dense kernels ------------------------------------------------------------
enum { GEMM_LOWER_C = 1, GEMM_A_LOWER = 2, GEMM_B_LOWER = 4 };

// C = beta*C + alpha * op(A) op(B); A(i,k) = A[i*lda+k] (ak=false) or A[k*lda+i]
// (ak=true); B(k,j) = B[k*ldb+j] (bn=false) or B[j*ldb+k] (bn=true); batched over
// `batch` with element strides sa, sb, sc.
template <typename T>
int launch_gemm(bool ak, bool bn, int M, int N, int K, T alpha, const T* A, long long lda,
                long long sa, const T* B, long long ldb, long long sb, T beta, T* C,
                long long ldc, long long sc, int batch, int flags, hipStream_t st);

struct Stage2Args {
  int n, m;
  // Alg. 1:    Tdiag in T_jj, overwritten; Linv_j = L_j^-1 with L_j L_j^T = S_j;
  //            Z_j = L_j^-1 T_{j,j+1}; Toff unchanged.
  // odd-even:  Linv_e = L_e^-1 of the pivot block of interface e; Tdiag_e is
  //            overwritten by U_e = L_e^-1 C^T (coupling to the neighbour
  //            before e), Z_e = V_e = L_e^-1 C_e (to the neighbour after e);
  //            Toff holds the couplings of the last level that used them.
  void* Tdiag;   // m blocks of n x n
  void* Toff;    // m-1 blocks, T_{j,j+1} on entry
  void* Linv;    // m blocks
  void* Z;       // m-1 blocks
  double* S64;   // optional: FP64 copy of each pivot block before its factorization
  int* status;
  int odd_even;  // 0: Alg. 1 sweep; 1: odd-even elimination order
};
template <typename T> int launch_stage2(const Stage2Args& a, hipStream_t st);

// y_q = beta*xin_q + alpha * M_q x_q for q < batch (M_q = M + q*sM, likewise
// x, xin, y) over nrhs columns of length n (column c of a block vector at
// c*n); M(i,k) = M[i*n+k] (tr=false) or M[k*n+i] (tr=true); lower=true
// restricts M to its triangle (k <= i for tr=false, k >= i for tr=true).
// xin may be null (beta ignored) or equal to y.
template <typename T>
int launch_gemv(bool tr, bool lower, int n, int nrhs, T alpha, const T* M, long long sM,
                const T* x, long long sx, T beta, const T* xin, long long sxin, T* y, long long sy,
                int batch, hipStream_t st);

// ---- solve kernels -----------------------------------------------------------
struct SolveArgs {
  int n1, n2, b, m, nrhs;
  const double* wh;
  const double* wv;
  const void* Gl;
  const void* Linv;
  const void* Z;
  const void* Td;  // odd-even order: U_e blocks
  void* zbuf;      // m * nrhs * n2 * BP scratch (slab precision)
  void* xb;        // m * 2 * nrhs * n2 boundary values (slab precision)
  void* ft;        // m * nrhs * n2 reduced vectors (reduced-system precision)
  void* yt;        // m * nrhs * n2
  void* tt;        // nrhs * n2 temporary
  int transpose;   // 1: adjoint (A^T) sweeps
  int odd_even;    // reduced system factored in odd-even order
};
// One pass of Alg. 4: slab sweeps in T (the slab factors' type), the reduced
// system in TR (the block factorization's type); rhs (FP64) -> out (FP64);
// accumulate=0 writes out, 1 adds to out.
template <typename T, typename TR>
int launch_solve_pass(const SolveArgs& a, const double* rhs, long long ld_rhs, double* out,
                      long long ld_out, int accumulate, hipStream_t st);

// r = f - A u and per-column sums of r^2 and f^2 (FP64).
int launch_residual(int n1, int n2, int nrhs, long long ld, const double* wh, const double* wv,
                    const double* f, const double* u, double* r, long long ldr, double* norms,
                    double* partial, hipStream_t st);
size_t residual_partial_count(int n1, int n2, int nrhs);

int launch_kappa_grad(int n1, int n2, int nrhs, long long ld, double h, const double* kappa,
                      const double* u, const double* lam, int mode, double* grad, hipStream_t st);

int launch_cast_f64(const void* src, int src_is_float, double* dst, long long count,
                    hipStream_t st);

}  // namespace slab
