// Host-side planners shared by the slab solver's HIP sources.  Each planner
// records grouped launches (see group.h) into a Plan; nothing runs until the
// plan's tables are uploaded and its steps are issued.
#pragma once

#include "common.h"
#include "group.h"
#include "slab.h"

#include <algorithm>

namespace slab {

// Refinement steps of the mixed-precision reduced solve (FP64 residual of the
// reduced system, FP32 correction): three take the FP32 solve's relative error
// of about 1e-4..1e-3 below 1e-11 on the interface values.
constexpr int REDUCED_REFINE_STEPS = 3;

// ---- stage one --------------------------------------------------------------
// Status words cleared, coefficient copy (or exp of theta) with positivity
// check, then edge weights.
void plan_coef_weights(Plan& plan, const std::vector<ProbDev>& probs);
// Slab factors, boundary columns, Schur propagation and assembly of T for a
// group of problems (one launch per phase and padded block order).  T: slab
// factors and Schur pieces; TO: the assembled T blocks.  ev (optional, 4
// events) is recorded after each phase.
template <typename T, typename TO>
void plan_stage1(Plan& plan, const std::vector<ProbDev>& probs, const hipEvent_t* ev);
int launch_maps(int n1, int n2, int b, int32_t* ck, int32_t* sc, int32_t* lc, int64_t* pe,
                int64_t* po, hipStream_t st);

// ---- dense kernels ------------------------------------------------------------
enum { GEMM_LOWER_C = 1, GEMM_A_LOWER = 2, GEMM_B_LOWER = 4,
       // load the C tile before the k loop (short k, beta != 0): 64-wide tiles
       GEMM_C_PREFETCH = 8 };

// C = beta*C + alpha * op(A) op(B) for every item; op(A)(i,k) = A[i*lda+k]
// (ak=false) or A[k*lda+i] (ak=true); op(B)(k,j) = B[k*ldb+j] (bn=false) or
// B[j*ldb+k] (bn=true).
// force_tile (64 or 128, FP32 only) overrides the size rule's tile choice.
template <typename T>
void plan_gemm(Plan& plan, bool ak, bool bn, const std::vector<GemmItem>& items, T alpha, T beta,
               int flags, int force_tile = 0);

// Cholesky factorization with carried inverse of independent pivot blocks.
template <typename T>
void plan_factor_blocks(Plan& plan, std::vector<FactorItem> items);

// Stage two of a group of problems: Alg. 1 (odd_even = false) or the
// odd-even order.  Alg. 1: Td in T_jj (overwritten), Linv_j = L_j^-1 with
// L_j L_j^T = S_j, Z_j = L_j^-1 T_{j,j+1}.  Odd-even: Linv_e = L_e^-1 of the
// pivot block of interface e, Td_e = U_e = L_e^-1 C^T (coupling to the
// neighbour before e), Z_e = V_e = L_e^-1 C_e (to the neighbour after e);
// To holds the couplings of the last level that used them.  S64 (optional)
// receives every pivot block before its factorization.  tile (0, 64 or 128)
// is passed to the block products as their forced FP32 tile width.
template <typename T>
void plan_stage2(Plan& plan, const std::vector<Stage2Prob>& probs, bool odd_even, int tile);

// y = beta*xin + alpha * op(M) x for every item over nrhs columns of length n
// (column c of a block vector at c*n); op(M)(i,k) = M[i*n+k] (tr=false) or
// M[k*n+i] (tr=true); lower=true restricts M to its triangle (k <= i for
// tr=false, k >= i for tr=true).  xin may be null (beta ignored) or equal y.
template <typename T>
void plan_gemv(Plan& plan, bool tr, bool lower, const std::vector<BmvItem>& items, T alpha,
               T beta);

// ---- solve ----------------------------------------------------------------------
// One pass of Alg. 4 for every problem: slab sweeps in T (the slab factors'
// type), the reduced system in TR (the block factorization's type); rhs (FP64)
// -> out (FP64), written or added (SolveDev::accumulate).
// rhs_only: stop after the reduced right-hand side (step (i)).
template <typename T, typename TR>
void plan_solve_pass(Plan& plan, const std::vector<SolveDev>& probs,
                     const std::vector<ReducedDev>& red, bool trans, bool odd_even,
                     bool rhs_only = false);

// y = T x for nrhs interface vectors (matrix-free, through the slab sweeps):
// x in d.u and y in d.g64, both [j][c][r]; d.r receives the load built from x
// (nrhs x n1 n2, FP64), the solve workspace as for a pass.
template <typename T, typename TR>
void plan_reduced_apply(Plan& plan, const std::vector<SolveDev>& probs);

// r = f - A u and per-column sums of r^2 and f^2 (FP64) for every problem.
void plan_residual(Plan& plan, const std::vector<SolveDev>& probs);
size_t residual_partial_count(int n1, int n2, int nrhs);
// Device-side convergence test of every problem after a pass (see ConvDev);
// first: the first pass (resets the pass counts).
void plan_converge(Plan& plan, const std::vector<ConvDev>& conv, bool first);

int launch_kappa_grad(int n1, int n2, int nrhs, long long ld, double h, const double* kappa,
                      const double* u, const double* lam, int mode, double* grad, hipStream_t st);

// f += load of the Dirichlet data g on the ring (nrhs fields of (n1+2)(n2+2)).
int launch_dirichlet(int n1, int n2, int nrhs, long long ld, const double* wh, const double* wv,
                     const double* g, double* f, hipStream_t st);

// FP64 copy of a float or double array.
int launch_cast_f64(const void* src, int src_is_float, double* dst, long long count,
                    hipStream_t st);

}  // namespace slab
