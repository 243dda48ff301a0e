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
//   A_ee^T x = y: z_r = Gl_r^T (y_r + W_r z_{r-1});  x_{r-1} = z_{r-1} + Gl_{r-1}^T W_r x_r
// MODE 0 (reduced right-hand side): y = f_e; emits w * x at the slab's first
//   and last column, xb[s][0|1][c][r].
// MODE 1 (interior): y = f_e + wL u_o(s-1) + wR u_o(s); writes (or adds) x and
//   the interface values u_o(s) into the natural-order output.
// One workgroup per (slab, group of NCG columns); thread = (row i, column slot).
// ---------------------------------------------------------------------------
constexpr int NCG = 16;

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

template <typename T, int BP, bool TRANS, int MODE>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs a) {
  constexpr int SLOTS = 256 / BP;
  constexpr int Q = (NCG + SLOTS - 1) / SLOTS;
  __shared__ T Gs[BP][BP + 1];
  __shared__ T Va[NCG][BP];
  __shared__ T Vb[NCG][BP];
  const int s = blockIdx.x;
  const int cbase = blockIdx.y * NCG;
  const int n2 = a.n2, b = a.b;
  const int tid = threadIdx.x;
  const int i = tid % BP, slot = tid / BP;
  const long long c0 = (long long)s * (b + 1);
  const long long ci = c0 + (i < b ? i : 0);
  const bool act = i < b;
  const T* Gl = (const T*)a.Gl + (size_t)s * n2 * BP * BP;
  T* zbuf = (T*)a.zbuf + (size_t)s * a.nrhs * n2 * BP;
  const T* uo = (const T*)a.uo;

  auto loadG = [&](int r) {
    const T* G = Gl + (size_t)r * BP * BP;
    for (int e = tid; e < BP * BP; e += 256) Gs[e / BP][e % BP] = G[e];
  };
  auto wv_at = [&](int r) -> T {  // edge between rows r-1 and r of column ci; 0 outside
    return (act && r >= 0 && r <= n2 - 1 + 1) ? (T)a.wv[ci * (n2 + 1) + r] : (T)0;
  };
  auto rhs_at = [&](int c, int r) -> T {
    if (!act) return (T)0;
    double v = a.rhs[(long long)c * a.ld + ci * n2 + r];
    if (MODE == 1) {
      if (i == 0 && s > 0)
        v += a.wh[c0 * n2 + r] * (double)uo[((size_t)(s - 1) * a.nrhs + c) * n2 + r];
      if (i == b - 1) v += a.wh[(c0 + b) * n2 + r] * (double)uo[((size_t)s * a.nrhs + c) * n2 + r];
    }
    return (T)v;
  };

  // ---------------- forward sweep: z_r, stored in zbuf ----------------
  for (int r = 0; r < n2; ++r) {
    __syncthreads();
    const T w = (r > 0) ? wv_at(r) : (T)0;
    if (!TRANS) {
      if (r > 0) loadG(r - 1);
      __syncthreads();
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int cl = slot + q * SLOTS;
        const int c = cbase + cl;
        if (cl < NCG && c < a.nrhs) {
          T t = (T)0;
          if (r > 0) {
#pragma unroll 8
            for (int k = 0; k < BP; ++k) t += Gs[i][k] * Va[cl][k];
          }
          const T z = rhs_at(c, r) + w * t;
          Vb[cl][i] = z;
          zbuf[((size_t)c * n2 + r) * BP + i] = z;
        }
      }
    } else {
      loadG(r);
#pragma unroll
      for (int q = 0; q < Q; ++q) {  // u = y_r + W_r z_{r-1}
        const int cl = slot + q * SLOTS;
        const int c = cbase + cl;
        if (cl < NCG && c < a.nrhs) Vb[cl][i] = rhs_at(c, r) + (r > 0 ? w * Va[cl][i] : (T)0);
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int cl = slot + q * SLOTS;
        const int c = cbase + cl;
        T z = (T)0;
        if (cl < NCG && c < a.nrhs) {
#pragma unroll 8
          for (int k = 0; k < BP; ++k) z += Gs[k][i] * Vb[cl][k];
          zbuf[((size_t)c * n2 + r) * BP + i] = z;
        }
        __syncthreads();
        if (cl < NCG && c < a.nrhs) Vb[cl][i] = z;
      }
    }
    __syncthreads();
    // Vb -> Va
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int cl = slot + q * SLOTS;
      if (cl < NCG) Va[cl][i] = Vb[cl][i];
    }
  }

  // ---------------- backward sweep ----------------
  for (int r = n2 - 1; r >= 0; --r) {
    __syncthreads();
    if (!TRANS) {
      // u = z_r + W_{r+1} x_{r+1};  x_r = Gl_r u
      loadG(r);
      const T w = (r + 1 <= n2 - 1) ? wv_at(r + 1) : (T)0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int cl = slot + q * SLOTS;
        const int c = cbase + cl;
        if (cl < NCG && c < a.nrhs) {
          const T z = zbuf[((size_t)c * n2 + r) * BP + i];
          Vb[cl][i] = z + (r < n2 - 1 ? w * Va[cl][i] : (T)0);
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int cl = slot + q * SLOTS;
        const int c = cbase + cl;
        T x = (T)0;
        if (cl < NCG && c < a.nrhs) {
#pragma unroll 8
          for (int k = 0; k < BP; ++k) x += Gs[i][k] * Vb[cl][k];
        }
        __syncthreads();
        if (cl < NCG && c < a.nrhs) Vb[cl][i] = x;
      }
    } else {
      // x_{n-1} = z_{n-1};  x_r = z_r + Gl_r^T W_{r+1} x_{r+1}
      if (r < n2 - 1) {
        loadG(r);
        const T w = wv_at(r + 1);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int cl = slot + q * SLOTS;
          if (cl < NCG) Vb[cl][i] = w * Va[cl][i];
        }
        __syncthreads();
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int cl = slot + q * SLOTS;
        const int c = cbase + cl;
        T x = (T)0;
        if (cl < NCG && c < a.nrhs) {
          x = zbuf[((size_t)c * n2 + r) * BP + i];
          if (r < n2 - 1) {
#pragma unroll 8
            for (int k = 0; k < BP; ++k) x += Gs[k][i] * Vb[cl][k];
          }
        }
        __syncthreads();
        if (cl < NCG && c < a.nrhs) Vb[cl][i] = x;
      }
    }
    __syncthreads();
    // outputs of row r, then Vb -> Va
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int cl = slot + q * SLOTS;
      const int c = cbase + cl;
      if (cl < NCG && c < a.nrhs) {
        const T x = Vb[cl][i];
        if (MODE == 0) {
          T* xb = (T*)a.xb;
          if (i == 0)
            xb[(((size_t)s * 2 + 0) * a.nrhs + c) * n2 + r] = (T)(a.wh[c0 * n2 + r] * (double)x);
          if (i == b - 1)
            xb[(((size_t)s * 2 + 1) * a.nrhs + c) * n2 + r] =
                (T)(a.wh[(c0 + b) * n2 + r] * (double)x);
        } else {
          if (act) {
            double* o = a.out + (long long)c * a.ldo + ci * n2 + r;
            *o = a.accumulate ? *o + (double)x : (double)x;
          }
          if (i == 0) {
            double* o = a.out + (long long)c * a.ldo + (c0 + b) * n2 + r;
            const double v = (double)uo[((size_t)s * a.nrhs + c) * n2 + r];
            *o = a.accumulate ? *o + v : v;
          }
        }
      }
      if (cl < NCG) Va[cl][i] = Vb[cl][i];
    }
  }
}

// f~_j = f_o(j) + xb[j][right] + xb[j+1][left]   (FP64 sum, stored in T)
template <typename T>
__global__ void k_reduced_rhs(int n2, int b, int m, int nrhs, long long ld,
                              const double* __restrict__ rhs, const T* __restrict__ xb,
                              T* __restrict__ ft) {
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
    ft[e] = (T)v;
  }
}

template <typename T, int BP>
static int sweeps_bp(const SolveArgs& A, const double* rhs, long long ld_rhs, double* out,
                     long long ld_out, int accumulate, hipStream_t st) {
  SweepArgs s;
  s.n1 = A.n1; s.n2 = A.n2; s.b = A.b; s.m = A.m; s.nrhs = A.nrhs; s.ld = ld_rhs; s.ldo = ld_out;
  s.wh = A.wh; s.wv = A.wv; s.Gl = A.Gl; s.zbuf = A.zbuf; s.xb = A.xb;
  s.uo = A.ft; s.rhs = rhs; s.out = out; s.accumulate = accumulate;
  const int n = A.n2, m = A.m, nrhs = A.nrhs;
  const long long nsq = (long long)n * n;
  dim3 grid(m, (nrhs + NCG - 1) / NCG);
  // (i) reduced right-hand side
  if (A.transpose) hipLaunchKernelGGL((k_sweep<T, BP, true, 0>), grid, dim3(256), 0, st, s);
  else hipLaunchKernelGGL((k_sweep<T, BP, false, 0>), grid, dim3(256), 0, st, s);
  SLAB_LAUNCH_CHECK();
  {
    long long tot = (long long)m * nrhs * n;
    unsigned g = (unsigned)std::min<long long>((tot + 255) / 256, 16384);
    hipLaunchKernelGGL((k_reduced_rhs<T>), dim3(g), dim3(256), 0, st, n, A.b, m, nrhs, ld_rhs, rhs,
                       (const T*)A.xb, (T*)A.ft);
    SLAB_LAUNCH_CHECK();
  }
  // (ii) Alg. 2 with the block Cholesky factors: T = R R^T, R_jj = L_j, R_{j+1,j} = Z_j^T
  T* ft = (T*)A.ft;
  T* yt = (T*)A.yt;
  T* tt = (T*)A.tt;
  const T* Li = (const T*)A.Linv;
  const T* Z = (const T*)A.Z;
  const long long vs = (long long)nrhs * n;
  for (int j = 0; j < m; ++j) {
    const T* src = ft + j * vs;
    if (j > 0) {
      int rc = launch_gemv<T>(true, false, n, nrhs, (T)-1, Z + (j - 1) * nsq, yt + (j - 1) * vs,
                              (T)1, ft + j * vs, tt, A.gemv_work, A.gemv_counters, st);
      if (rc) return rc;
      src = tt;
    }
    int rc = launch_gemv<T>(false, true, n, nrhs, (T)1, Li + j * nsq, src, (T)0, nullptr,
                            yt + j * vs, A.gemv_work, A.gemv_counters, st);
    if (rc) return rc;
  }
  for (int j = m - 1; j >= 0; --j) {
    const T* src = yt + j * vs;
    if (j < m - 1) {
      int rc = launch_gemv<T>(false, false, n, nrhs, (T)-1, Z + j * nsq, ft + (j + 1) * vs, (T)1,
                              yt + j * vs, tt, A.gemv_work, A.gemv_counters, st);
      if (rc) return rc;
      src = tt;
    }
    int rc = launch_gemv<T>(true, true, n, nrhs, (T)1, Li + j * nsq, src, (T)0, nullptr,
                            ft + j * vs, A.gemv_work, A.gemv_counters, st);
    if (rc) return rc;
  }
  // (iii) interior back substitution, interface values written alongside
  if (A.transpose) hipLaunchKernelGGL((k_sweep<T, BP, true, 1>), grid, dim3(256), 0, st, s);
  else hipLaunchKernelGGL((k_sweep<T, BP, false, 1>), grid, dim3(256), 0, st, s);
  SLAB_LAUNCH_CHECK();
  return SLAB_OK;
}

template <typename T>
int launch_solve_pass(const SolveArgs& a, const double* rhs, long long ld_rhs, double* out,
                      long long ld_out, int accumulate, hipStream_t st) {
  switch (padded_block(a.b)) {
    case 16: return sweeps_bp<T, 16>(a, rhs, ld_rhs, out, ld_out, accumulate, st);
    case 32: return sweeps_bp<T, 32>(a, rhs, ld_rhs, out, ld_out, accumulate, st);
    default: return sweeps_bp<T, 64>(a, rhs, ld_rhs, out, ld_out, accumulate, st);
  }
}
template int launch_solve_pass<float>(const SolveArgs&, const double*, long long, double*,
                                      long long, int, hipStream_t);
template int launch_solve_pass<double>(const SolveArgs&, const double*, long long, double*,
                                       long long, int, hipStream_t);

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
