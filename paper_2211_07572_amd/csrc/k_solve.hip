// Solve phase of the slab solver (Alg. 4): reduced right-hand side
// (eqs. (f1)-(f5)), the sweeping solve of Alg. 2 on the factored T, and the
// interior back substitution (eq. (usol_even)); plus the FP64 residual used
// by iterative refinement and the coefficient gradient of the adjoint method.
#include "launch.h"

namespace slab {

// ---------------------------------------------------------------------------
// Block forward/backward sweeps through one slab with the stored inverses
// Gl_r of the top-down block recursion (A_ee = L U, L_{r,r-1} = -W_r Gl_{r-1},
// U_rr = Gl_r^-1, U_{r-1,r} = -W_r):
//   A_ee x = y:   z_r = y_r + W_r Gl_{r-1} z_{r-1};   x_r = Gl_r (z_r + W_{r+1} x_{r+1})
//   A_ee^T x = y: z_r = Gl_r^T (y_r + W_r z_{r-1});  x_r = z_r + Gl_r^T W_{r+1} x_{r+1}
// MODE 0 (reduced right-hand side): y = f_e; emits w * x at the slab's first
//   and last column, xb[s][0|1][c][r].
// MODE 1 (interior): y = f_e + wL u_o(s-1) + wR u_o(s) (the coupling terms
//   precomputed by k_coupling into xb); writes (or adds) x into the
//   natural-order output (the interface values go through k_interface_out).
// One workgroup per (slab, group of 256/BP columns); thread = (row i, column).
// Software pipeline: while row step r is computed, the block inverse, edge
// weights and right-hand side of the next step are loaded into registers and
// then parked in the other half of double-buffered LDS, so each step costs one
// barrier and no exposed global-memory latency.
// ---------------------------------------------------------------------------
struct SweepArgs {
  int n1, n2, b, m, nrhs;
  long long ld;       // leading dimension of rhs
  long long ldo;      // leading dimension of out
  const double* wh;
  const double* wv;
  const void* Gl;
  void* zbuf;
  void* xb;
  const void* uo;     // interface values [j][c][r] (MODE 1)
  const double* rhs;  // natural order FP64
  double* out;        // natural order FP64 (MODE 1)
  int accumulate;
};

template <typename T, typename TU, int BP, bool TRANS, int MODE>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs a) {
  constexpr int NC = 256 / BP;            // columns per workgroup
  constexpr int GPT = BP * BP / 256;      // block-inverse elements loaded per thread
  constexpr int D = BP == 64 ? (sizeof(T) == 8 ? 2 : 4) : 8;  // prefetch depth (row steps)
  __shared__ T Gs[2][BP][BP + 1];
  __shared__ T Ws[2][BP];
  __shared__ T Ys[2][NC][BP + 1];
  __shared__ T Vs[2][NC][BP + 1];
  const int s = blockIdx.x;
  // kernel-argument fields copied to locals (the lambdas below must not take
  // the address of the argument block)
  const int n2 = a.n2, b = a.b, nrhs = a.nrhs;
  const long long ld = a.ld, ldo = a.ldo;
  const double* __restrict__ wh = a.wh;
  const double* __restrict__ wv = a.wv;
  const double* __restrict__ rhs = a.rhs;
  double* __restrict__ out_g = a.out;
  T* __restrict__ xbuf = (T*)a.xb;
  const int tid = threadIdx.x;
  const int i = tid % BP, cl = tid / BP;
  const int c = blockIdx.y * NC + cl;
  const bool valid = c < nrhs;
  const bool act = i < b;
  const long long c0 = (long long)s * (b + 1);
  const long long ci = c0 + (act ? i : 0);
  const T* Gl = (const T*)a.Gl + (size_t)s * n2 * BP * BP;
  T* zbuf = (T*)a.zbuf + (size_t)s * nrhs * n2 * BP;
  const bool acc_out = MODE == 1 && a.accumulate;

  // register ring: RAW loaded operands of the next D row steps (no arithmetic on
  // them until they are parked, so the loads stay in flight across steps)
  T rg[D][GPT];
  double rw[D], ry[D], ru[D], rbl[D], rbr[D];
  T rx[D], rz[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
#pragma unroll
    for (int e = 0; e < GPT; ++e) rg[d][e] = (T)0;
    rw[d] = ry[d] = ru[d] = rbl[d] = rbr[d] = 0.0;
    rx[d] = rz[d] = (T)0;
  }
  // MODE 1: the interface coupling w u_o was precomputed into xb (lane 0 reads
  // slot 0, lane b-1 slot 1; for b = 1 slot 0 carries both terms)
  const int xslot = (i == 0) ? 0 : ((i == b - 1) ? 1 : -1);
  auto load_w = [&](int r) __attribute__((always_inline)) -> double {
    return (tid < BP && act && r >= 1 && r <= n2 - 1) ? wv[ci * (n2 + 1) + r] : 0.0;
  };
  // forward step r: G = Gl_{r-1} (A x) or Gl_r (A^T x), w = W_r, y = y_r
  auto load_fwd = [&](int d, int r) __attribute__((always_inline)) {
    const int gr = TRANS ? r : r - 1;
    if (gr >= 0) {
      const T* G = Gl + (size_t)gr * BP * BP;
#pragma unroll
      for (int e = 0; e < GPT; ++e) rg[d][e] = G[tid + 256 * e];
    }
    rw[d] = load_w(r);
    ry[d] = (valid && act) ? rhs[(long long)c * ld + ci * n2 + r] : 0.0;
    if (MODE == 1)
      rx[d] = (valid && act && xslot >= 0)
                  ? xbuf[(((size_t)s * 2 + xslot) * nrhs + c) * n2 + r] : (T)0;
  };
  // backward step r: G = Gl_r, w = W_{r+1}, z = z_r (+ old outputs when accumulating)
  auto load_bwd = [&](int d, int r) __attribute__((always_inline)) {
    const T* G = Gl + (size_t)r * BP * BP;
#pragma unroll
    for (int e = 0; e < GPT; ++e) rg[d][e] = G[tid + 256 * e];
    rw[d] = load_w(r + 1);
    rz[d] = valid ? zbuf[((size_t)c * n2 + r) * BP + i] : (T)0;
    ru[d] = (MODE == 1 && valid && acc_out && act) ? out_g[(long long)c * ldo + ci * n2 + r] : 0.0;
    if (MODE == 0) {  // interface edge weights of the boundary outputs
      rbl[d] = (valid && i == 0) ? wh[c0 * n2 + r] : 0.0;
      rbr[d] = (valid && i == b - 1) ? wh[(c0 + b) * n2 + r] : 0.0;
    }
  };
  auto parkG = [&](int d, int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < GPT; ++e) {
      const int idx = tid + 256 * e;
      Gs[buf][idx / BP][idx % BP] = rg[d][e];
    }
    if (tid < BP) Ws[buf][tid] = (T)rw[d];
  };
  auto park_fwd = [&](int d, int buf) __attribute__((always_inline)) {
    parkG(d, buf);
    Ys[buf][cl][i] = (T)(ry[d] + (MODE == 1 ? (double)rx[d] : 0.0));
  };
  auto park_bwd = [&](int d, int buf) __attribute__((always_inline)) {
    parkG(d, buf);
    Ys[buf][cl][i] = rz[d];
  };

  // ---------------- forward sweep: z_r (stored in zbuf) ----------------
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (d < n2) load_fwd(d, d);
  Vs[0][cl][i] = (T)0;
  for (int r0 = 0; r0 < n2; r0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int r = r0 + d;
      if (r < n2) {  // uniform
      const int cur = r & 1;
      park_fwd(d, cur);
      if (r + D < n2) load_fwd(d, r + D);
      __syncthreads();
      // dot products over k in four independent partial sums (short FMA chains)
      T out;
      if (!TRANS) {
        T t[4] = {(T)0, (T)0, (T)0, (T)0};
        if (r > 0) {
#pragma unroll
          for (int k = 0; k < BP; ++k) t[k & 3] += Gs[cur][i][k] * Vs[cur][cl][k];
        }
        out = Ys[cur][cl][i] + Ws[cur][i] * ((t[0] + t[1]) + (t[2] + t[3]));
      } else {
        T t[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
        for (int k = 0; k < BP; ++k)
          t[k & 3] += Gs[cur][k][i] * (Ys[cur][cl][k] + Ws[cur][k] * Vs[cur][cl][k]);
        out = (t[0] + t[1]) + (t[2] + t[3]);
      }
      if (valid) zbuf[((size_t)c * n2 + r) * BP + i] = out;
      Vs[cur ^ 1][cl][i] = out;
      }
    }
  }
  __syncthreads();

  // ---------------- backward sweep: x_r ----------------
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (d < n2) load_bwd(d, n2 - 1 - d);
  Vs[0][cl][i] = (T)0;
  for (int t0 = 0; t0 < n2; t0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int it = t0 + d;
      if (it < n2) {  // uniform
      const int r = n2 - 1 - it;
      const int cur = it & 1;
      park_bwd(d, cur);
      const double uold = ru[d], wbl = rbl[d], wbr = rbr[d];
      if (it + D < n2) load_bwd(d, r - D);
      __syncthreads();
      T x;
      if (!TRANS) {
        T t[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
        for (int k = 0; k < BP; ++k)
          t[k & 3] += Gs[cur][i][k] * (Ys[cur][cl][k] + Ws[cur][k] * Vs[cur][cl][k]);
        x = (t[0] + t[1]) + (t[2] + t[3]);
      } else {
        T t[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
        for (int k = 0; k < BP; ++k) t[k & 3] += Gs[cur][k][i] * (Ws[cur][k] * Vs[cur][cl][k]);
        x = Ys[cur][cl][i] + ((t[0] + t[1]) + (t[2] + t[3]));
      }
      Vs[cur ^ 1][cl][i] = x;
      if (valid) {
        if (MODE == 0) {
          if (i == 0) xbuf[(((size_t)s * 2 + 0) * nrhs + c) * n2 + r] = (T)(wbl * (double)x);
          if (i == b - 1) xbuf[(((size_t)s * 2 + 1) * nrhs + c) * n2 + r] = (T)(wbr * (double)x);
        } else if (act) {
          out_g[(long long)c * ldo + ci * n2 + r] = acc_out ? uold + (double)x : (double)x;
        }
      }
      }
    }
  }
}

// Interface coupling of the interior solve (eq. (usol_even)): for slab s,
//   xb[s][0][c][r] = wL_r u_o(s-1)[c][r]   (+ wR_r u_o(s)[c][r] when b = 1)
//   xb[s][1][c][r] = wR_r u_o(s)[c][r]
// with wL, wR the edge weights between the slab and its two interfaces.
template <typename T, typename TR>
__global__ void k_coupling(int n2, int b, int m, int nrhs, const double* __restrict__ wh,
                           const TR* __restrict__ uo, T* __restrict__ xb) {
  const long long tot = (long long)m * nrhs * n2;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e % n2;
    const long long c = (e / n2) % nrhs;
    const long long s = e / ((long long)n2 * nrhs);
    const long long c0 = s * (b + 1);
    const double right = wh[(c0 + b) * n2 + r] * (double)uo[(s * nrhs + c) * n2 + r];
    double left = s > 0 ? wh[c0 * n2 + r] * (double)uo[((s - 1) * nrhs + c) * n2 + r] : 0.0;
    if (b == 1) left += right;
    xb[((s * 2 + 0) * nrhs + c) * n2 + r] = (T)left;
    xb[((s * 2 + 1) * nrhs + c) * n2 + r] = (T)right;
  }
}

// Interface values u_o(j) (reduced solution, [j][c][r]) into the natural-order
// output column j(b+1)+b, written or added.
template <typename TR>
__global__ void k_interface_out(int n2, int b, int m, int nrhs, long long ldo,
                                const TR* __restrict__ uo, double* __restrict__ out,
                                int accumulate) {
  const long long tot = (long long)m * nrhs * n2;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e % n2;
    const long long c = (e / n2) % nrhs;
    const long long j = e / ((long long)n2 * nrhs);
    double* o = out + c * ldo + (j * (b + 1) + b) * n2 + r;
    const double v = (double)uo[e];
    *o = accumulate ? *o + v : v;
  }
}

// f~_j = f_o(j) + xb[j][right] + xb[j+1][left]   (FP64 sum, stored in T)
template <typename T, typename TR>
__global__ void k_reduced_rhs(int n2, int b, int m, int nrhs, long long ld,
                              const double* __restrict__ rhs, const T* __restrict__ xb,
                              TR* __restrict__ ft) {
  const long long tot = (long long)m * nrhs * n2;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const long long r = e % n2;
    const long long c = (e / n2) % nrhs;
    const long long j = e / ((long long)n2 * nrhs);
    const long long cj = j * (b + 1) + b;
    double v = rhs[c * ld + cj * n2 + r];
    v += (double)xb[((j * 2 + 1) * nrhs + c) * n2 + r];
    if (j + 1 < m) v += (double)xb[(((j + 1) * 2 + 0) * nrhs + c) * n2 + r];
    ft[e] = (TR)v;
  }
}

template <typename T, typename TR, int BP>
static int sweeps_bp(const SolveArgs& A, const double* rhs, long long ld_rhs, double* out,
                     long long ld_out, int accumulate, hipStream_t st) {
  SweepArgs s;
  s.n1 = A.n1; s.n2 = A.n2; s.b = A.b; s.m = A.m; s.nrhs = A.nrhs; s.ld = ld_rhs; s.ldo = ld_out;
  s.wh = A.wh; s.wv = A.wv; s.Gl = A.Gl; s.zbuf = A.zbuf; s.xb = A.xb;
  s.uo = A.ft; s.rhs = rhs; s.out = out; s.accumulate = accumulate;
  const int n = A.n2, m = A.m, nrhs = A.nrhs;
  const long long nsq = (long long)n * n;
  dim3 grid(m, (nrhs + 256 / BP - 1) / (256 / BP));
  // (i) reduced right-hand side
  if (A.transpose) hipLaunchKernelGGL((k_sweep<T, TR, BP, true, 0>), grid, dim3(256), 0, st, s);
  else hipLaunchKernelGGL((k_sweep<T, TR, BP, false, 0>), grid, dim3(256), 0, st, s);
  SLAB_LAUNCH_CHECK();
  {
    long long tot = (long long)m * nrhs * n;
    unsigned g = (unsigned)std::min<long long>((tot + 255) / 256, 16384);
    hipLaunchKernelGGL((k_reduced_rhs<T, TR>), dim3(g), dim3(256), 0, st, n, A.b, m, nrhs, ld_rhs,
                       rhs, (const T*)A.xb, (TR*)A.ft);
    SLAB_LAUNCH_CHECK();
  }
  // (ii) the reduced system
  TR* ft = (TR*)A.ft;
  TR* yt = (TR*)A.yt;
  TR* tt = (TR*)A.tt;
  const TR* Li = (const TR*)A.Linv;
  const TR* Z = (const TR*)A.Z;
  const TR* U = (const TR*)A.Td;
  const long long vs = (long long)nrhs * n;
  if (!A.odd_even) {
    // Alg. 2 with the block Cholesky factors: T = R R^T, R_jj = L_j, R_{j+1,j} = Z_j^T
    for (int j = 0; j < m; ++j) {
      const TR* src = ft + j * vs;
      if (j > 0) {
        int rc = launch_gemv<TR>(true, false, n, nrhs, (TR)-1, Z + (j - 1) * nsq, 0,
                                 yt + (j - 1) * vs, 0, (TR)1, ft + j * vs, 0, tt, 0, 1, st);
        if (rc) return rc;
        src = tt;
      }
      int rc = launch_gemv<TR>(false, true, n, nrhs, (TR)1, Li + j * nsq, 0, src, 0, (TR)0,
                               nullptr, 0, yt + j * vs, 0, 1, st);
      if (rc) return rc;
    }
    for (int j = m - 1; j >= 0; --j) {
      const TR* src = yt + j * vs;
      if (j < m - 1) {
        int rc = launch_gemv<TR>(false, false, n, nrhs, (TR)-1, Z + j * nsq, 0, ft + (j + 1) * vs,
                                 0, (TR)1, yt + j * vs, 0, tt, 0, 1, st);
        if (rc) return rc;
        src = tt;
      }
      int rc = launch_gemv<TR>(true, true, n, nrhs, (TR)1, Li + j * nsq, 0, src, 0, (TR)0,
                               nullptr, 0, ft + j * vs, 0, 1, st);
      if (rc) return rc;
    }
  } else {
    // odd-even order (same levels as the factorization): reduce the
    // right-hand side level by level, y_e = L_e^-1 g_e, g_l -= U_e^T y_e,
    // g_r -= V_e^T y_e; then from the top level down
    // x_e = L_e^-T (y_e - U_e x_l - V_e x_r), x_e overwriting g_e.
    int nlev = 0;
    for (long long s = 1; m / s >= 1; s *= 2) ++nlev;
    for (int lev = 0; lev < nlev; ++lev) {
      const long long s = 1LL << lev;
      const int k = (int)(m / s), E = (k + 1) / 2, NR = k / 2;
      const long long e0 = s - 1, e1 = e0 + 2 * s, ms = 2 * s * nsq, v2 = 2 * s * vs;
      int rc = launch_gemv<TR>(false, true, n, nrhs, (TR)1, Li + e0 * nsq, ms, ft + e0 * vs, v2,
                               (TR)0, nullptr, 0, yt + e0 * vs, v2, E, st);
      if (rc) return rc;
      rc = launch_gemv<TR>(true, false, n, nrhs, (TR)-1, Z + e0 * nsq, ms, yt + e0 * vs, v2, (TR)1,
                           ft + (e0 + s) * vs, v2, ft + (e0 + s) * vs, v2, NR, st);
      if (rc) return rc;
      rc = launch_gemv<TR>(true, false, n, nrhs, (TR)-1, U + e1 * nsq, ms, yt + e1 * vs, v2, (TR)1,
                           ft + (e1 - s) * vs, v2, ft + (e1 - s) * vs, v2, E - 1, st);
      if (rc) return rc;
    }
    for (int lev = nlev - 1; lev >= 0; --lev) {
      const long long s = 1LL << lev;
      const int k = (int)(m / s), E = (k + 1) / 2, NR = k / 2;
      const long long e0 = s - 1, e1 = e0 + 2 * s, ms = 2 * s * nsq, v2 = 2 * s * vs;
      int rc = launch_gemv<TR>(false, false, n, nrhs, (TR)-1, Z + e0 * nsq, ms, ft + (e0 + s) * vs,
                               v2, (TR)1, yt + e0 * vs, v2, yt + e0 * vs, v2, NR, st);
      if (rc) return rc;
      rc = launch_gemv<TR>(false, false, n, nrhs, (TR)-1, U + e1 * nsq, ms, ft + (e1 - s) * vs, v2,
                           (TR)1, yt + e1 * vs, v2, yt + e1 * vs, v2, E - 1, st);
      if (rc) return rc;
      rc = launch_gemv<TR>(true, true, n, nrhs, (TR)1, Li + e0 * nsq, ms, yt + e0 * vs, v2, (TR)0,
                           nullptr, 0, ft + e0 * vs, v2, E, st);
      if (rc) return rc;
    }
  }
  // (iii) interior back substitution, and the interface values
  {
    long long tot = (long long)m * nrhs * n;
    unsigned g = (unsigned)std::min<long long>((tot + 255) / 256, 16384);
    hipLaunchKernelGGL((k_coupling<T, TR>), dim3(g), dim3(256), 0, st, n, A.b, m, nrhs, A.wh,
                       (const TR*)A.ft, (T*)A.xb);
    SLAB_LAUNCH_CHECK();
  }
  if (A.transpose) hipLaunchKernelGGL((k_sweep<T, TR, BP, true, 1>), grid, dim3(256), 0, st, s);
  else hipLaunchKernelGGL((k_sweep<T, TR, BP, false, 1>), grid, dim3(256), 0, st, s);
  SLAB_LAUNCH_CHECK();
  {
    long long tot = (long long)m * nrhs * n;
    unsigned g = (unsigned)std::min<long long>((tot + 255) / 256, 16384);
    hipLaunchKernelGGL((k_interface_out<TR>), dim3(g), dim3(256), 0, st, n, A.b, m, nrhs, ld_out,
                       (const TR*)A.ft, out, accumulate);
    SLAB_LAUNCH_CHECK();
  }
  return SLAB_OK;
}

template <typename T, typename TR>
int launch_solve_pass(const SolveArgs& a, const double* rhs, long long ld_rhs, double* out,
                      long long ld_out, int accumulate, hipStream_t st) {
  switch (padded_block(a.b)) {
    case 16: return sweeps_bp<T, TR, 16>(a, rhs, ld_rhs, out, ld_out, accumulate, st);
    case 32: return sweeps_bp<T, TR, 32>(a, rhs, ld_rhs, out, ld_out, accumulate, st);
    default: return sweeps_bp<T, TR, 64>(a, rhs, ld_rhs, out, ld_out, accumulate, st);
  }
}
template int launch_solve_pass<float, float>(const SolveArgs&, const double*, long long, double*,
                                             long long, int, hipStream_t);
template int launch_solve_pass<double, double>(const SolveArgs&, const double*, long long,
                                               double*, long long, int, hipStream_t);
template int launch_solve_pass<double, float>(const SolveArgs&, const double*, long long,
                                              double*, long long, int, hipStream_t);

// ---------------------------------------------------------------------------
// Residual r = f - A u (FP64) with per-column partial sums of r^2 and f^2.
// Grid: (chunks, nrhs); partial[(c*chunks + blk)*2 + {0,1}].
// ---------------------------------------------------------------------------
constexpr int RES_CHUNKS = 256;

size_t residual_partial_count(int n1, int n2, int nrhs) { return (size_t)nrhs * RES_CHUNKS * 2; }

__global__ __launch_bounds__(256) void k_residual(int n1, int n2, long long ld,
                                                  const double* __restrict__ wh,
                                                  const double* __restrict__ wv,
                                                  const double* __restrict__ f,
                                                  const double* __restrict__ u,
                                                  double* __restrict__ r, long long ldr,
                                                  double* __restrict__ partial) {
  __shared__ double red[2][256];
  const int c = blockIdx.y;
  const long long N = (long long)n1 * n2;
  const double* fc = f + c * ld;
  const double* uc = u + c * ld;
  double sr = 0.0, sf = 0.0;
  for (long long p = blockIdx.x * 256LL + threadIdx.x; p < N; p += (long long)gridDim.x * 256) {
    const long long col = p / n2, row = p % n2;
    const double w_l = wh[col * n2 + row], w_r = wh[(col + 1) * n2 + row];
    const double w_d = wv[col * (n2 + 1) + row], w_u = wv[col * (n2 + 1) + row + 1];
    const double up = uc[p];
    double au = (w_l + w_r + w_d + w_u) * up;
    if (col > 0) au -= w_l * uc[p - n2];
    if (col < n1 - 1) au -= w_r * uc[p + n2];
    if (row > 0) au -= w_d * uc[p - 1];
    if (row < n2 - 1) au -= w_u * uc[p + 1];
    const double fv = fc[p];
    const double rv = fv - au;
    if (r) r[c * ldr + p] = rv;
    sr += rv * rv;
    sf += fv * fv;
  }
  red[0][threadIdx.x] = sr;
  red[1][threadIdx.x] = sf;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      red[0][threadIdx.x] += red[0][threadIdx.x + off];
      red[1][threadIdx.x] += red[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[((long long)c * gridDim.x + blockIdx.x) * 2 + 0] = red[0][0];
    partial[((long long)c * gridDim.x + blockIdx.x) * 2 + 1] = red[1][0];
  }
}

__global__ void k_norms(int nrhs, int chunks, const double* __restrict__ partial,
                        double* __restrict__ norms) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  double sr = 0.0, sf = 0.0;
  for (int k = 0; k < chunks; ++k) {
    sr += partial[((long long)c * chunks + k) * 2 + 0];
    sf += partial[((long long)c * chunks + k) * 2 + 1];
  }
  norms[2 * c + 0] = sr;
  norms[2 * c + 1] = sf;
}

int launch_residual(int n1, int n2, int nrhs, long long ld, const double* wh, const double* wv,
                    const double* f, const double* u, double* r, long long ldr, double* norms,
                    double* partial, hipStream_t st) {
  const long long N = (long long)n1 * n2;
  const int chunks = (int)std::min<long long>(RES_CHUNKS, (N + 255) / 256);
  hipLaunchKernelGGL(k_residual, dim3(chunks, nrhs), dim3(256), 0, st, n1, n2, ld, wh, wv, f, u, r,
                     ldr, partial);
  SLAB_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_norms, dim3((nrhs + 63) / 64), dim3(64), 0, st, nrhs, chunks, partial,
                     norms);
  SLAB_LAUNCH_CHECK();
  return SLAB_OK;
}

// ---------------------------------------------------------------------------
// Coefficient gradient: for every node p of the ring-padded field,
//   dL/dkappa_p = sum over edges e = (p, q) of -(1/(2h^2)) sum_k (lam_p - lam_q)(u_p - u_q),
// ring values zero; mode 1 multiplies by kappa_p (theta = log kappa).
// ---------------------------------------------------------------------------
__global__ void k_kappa_grad(int n1, int n2, int nrhs, long long ld, double h,
                             const double* __restrict__ kappa, const double* __restrict__ u,
                             const double* __restrict__ lam, int mode,
                             double* __restrict__ grad) {
  const long long W = n2 + 2;
  const long long tot = (long long)(n1 + 2) * W;
  const double scale = 1.0 / (2.0 * h * h);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const long long ic = e / W, ir = e % W;   // padded coordinates
    const long long c = ic - 1, r = ir - 1;   // interior coordinates
    const bool inside = c >= 0 && c < n1 && r >= 0 && r < n2;
    double gsum = 0.0;
    const long long nbr[4][2] = {{c - 1, r}, {c + 1, r}, {c, r - 1}, {c, r + 1}};
    for (int k = 0; k < nrhs; ++k) {
      const double* uk = u + k * ld;
      const double* lk = lam + k * ld;
      const double up = inside ? uk[c * n2 + r] : 0.0;
      const double lp = inside ? lk[c * n2 + r] : 0.0;
      for (int q = 0; q < 4; ++q) {
        const long long cq = nbr[q][0], rq = nbr[q][1];
        // the edge exists when both ends lie in the padded field and one of them is interior
        if (cq < -1 || cq > n1 || rq < -1 || rq > n2) continue;
        const bool qin = cq >= 0 && cq < n1 && rq >= 0 && rq < n2;
        if (!inside && !qin) continue;
        if (!inside && !(q < 2 ? (r >= 0 && r < n2) : (c >= 0 && c < n1))) continue;
        const double uq = qin ? uk[cq * n2 + rq] : 0.0;
        const double lq = qin ? lk[cq * n2 + rq] : 0.0;
        gsum -= (lp - lq) * (up - uq);
      }
    }
    double g = gsum * scale;
    if (mode == 1) g *= kappa[e];
    grad[e] = g;
  }
}

int launch_kappa_grad(int n1, int n2, int nrhs, long long ld, double h, const double* kappa,
                      const double* u, const double* lam, int mode, double* grad, hipStream_t st) {
  const long long tot = (long long)(n1 + 2) * (n2 + 2);
  unsigned grid = (unsigned)std::min<long long>((tot + 255) / 256, 16384);
  hipLaunchKernelGGL(k_kappa_grad, dim3(grid), dim3(256), 0, st, n1, n2, nrhs, ld, h, kappa, u,
                     lam, mode, grad);
  SLAB_LAUNCH_CHECK();
  return SLAB_OK;
}

}  // namespace slab
