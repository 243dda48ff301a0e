// Stage two of the slab solver: block factorization of the block-tridiagonal
// reduced matrix T (Alg. 1) and the dense kernels it is built from.
//
// T is symmetric positive definite for kappa > 0, so every S_j of Alg. 1 is
// too.  "Compute and store S_j^-1" is realised as S_j = L_j L_j^T with the
// explicit inverse L_j^-1 kept, and the next pivot block formed as
//   S_{j+1} = T_{j+1,j+1} - Z_j^T Z_j,   Z_j = L_j^-1 T_{j,j+1},
// which equals T_{j+1,j+1} - T_{j+1,j} S_j^-1 T_{j,j+1} since T_{j+1,j} = T_{j,j+1}^T.
// The factorization of each S_j is right-looking in 64-column panels; the
// identity carried along as extra columns turns into L_j^-1 (forward
// substitution with a matrix right-hand side).  All products run on
// 16x16x4 MFMA tiles in the working precision (FP32 or FP64).
#include "launch.h"

namespace slab {

// ---------------------------------------------------------------------------
// Tiled MFMA GEMM: C = beta*C + alpha * op(A) op(B).
// 64x64 output tile per workgroup, four waves of 32x32, k chunks of 16.
// ---------------------------------------------------------------------------
template <typename T, bool AK, bool BN>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, T alpha,
                                              const T* __restrict__ A, long long lda,
                                              long long sa, const T* __restrict__ B,
                                              long long ldb, long long sb, T beta, T* C,
                                              long long ldc, long long sc, int flags) {
  typedef typename acc4<T>::type V4;
  constexpr int TM = 64, TN = 64, TK = 16;
  __shared__ T As[TK][TM + 4];
  __shared__ T Bs[TK][TN + 4];
  int ti, tj;
  if (flags & GEMM_LOWER_C) {
    const long long t = blockIdx.x;
    int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((long long)(r + 1) * (r + 2) / 2 <= t) ++r;
    while ((long long)r * (r + 1) / 2 > t) --r;
    ti = r;
    tj = (int)(t - (long long)r * (r + 1) / 2);
  } else {
    ti = blockIdx.y;
    tj = blockIdx.x;
  }
  A += (long long)blockIdx.z * sa;
  B += (long long)blockIdx.z * sb;
  C += (long long)blockIdx.z * sc;
  const int i0 = ti * TM, j0 = tj * TN;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, nn = lane & 15;
  const int wm = wave >> 1, wn = wave & 1;
  int kmin = (flags & GEMM_B_LOWER) ? j0 : 0;
  int kmax = (flags & GEMM_A_LOWER) ? min(K, i0 + TM) : K;
  kmin = (kmin / TK) * TK;

  V4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = V4{0, 0, 0, 0};

  for (int k0 = kmin; k0 < kmax; k0 += TK) {
    if (!AK) {
      const int row = tid >> 2, kq = (tid & 3) * 4;
      const long long gi = i0 + row;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gk = k0 + kq + e;
        As[kq + e][row] = (gi < M && gk < kmax) ? A[gi * lda + gk] : (T)0;
      }
    } else {
      const int kk = tid >> 4, iq = (tid & 15) * 4;
      const long long gk = k0 + kk;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gi = i0 + iq + e;
        As[kk][iq + e] = (gi < M && gk < kmax) ? A[gk * lda + gi] : (T)0;
      }
    }
    if (!BN) {
      const int kk = tid >> 4, jq = (tid & 15) * 4;
      const long long gk = k0 + kk;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gj = j0 + jq + e;
        Bs[kk][jq + e] = (gj < N && gk < kmax) ? B[gk * ldb + gj] : (T)0;
      }
    } else {
      const int col = tid >> 2, kq = (tid & 3) * 4;
      const long long gj = j0 + col;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gk = k0 + kq + e;
        Bs[kq + e][col] = (gj < N && gk < kmax) ? B[gj * ldb + gk] : (T)0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      T av[2], bv[2];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt) av[mt] = As[4 * ks + g][wm * 32 + 16 * mt + nn];
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) bv[nt] = Bs[4 * ks + g][wn * 32 + 16 * nt + nn];
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = mfma16(av[mt], bv[nt], acc[mt][nt]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long long gi = i0 + wm * 32 + 16 * mt + acc_row<T>(g, i);
        const long long gj = j0 + wn * 32 + 16 * nt + nn;
        if (gi < M && gj < N) {
          T v = alpha * acc[mt][nt][i];
          if (beta != (T)0) v += beta * C[gi * ldc + gj];
          C[gi * ldc + gj] = v;
        }
      }
}

template <typename T>
int launch_gemm(bool ak, bool bn, int M, int N, int K, T alpha, const T* A, long long lda,
                long long sa, const T* B, long long ldb, long long sb, T beta, T* C,
                long long ldc, long long sc, int batch, int flags, hipStream_t st) {
  if (M <= 0 || N <= 0) return SLAB_OK;
  const int tm = (M + 63) / 64, tn = (N + 63) / 64;
  dim3 grid;
  if (flags & GEMM_LOWER_C) grid = dim3((unsigned)((long long)tm * (tm + 1) / 2), 1, batch);
  else grid = dim3(tn, tm, batch);
#define SLAB_GEMM_CASE(AKV, BNV)                                                          \
  hipLaunchKernelGGL((k_gemm<T, AKV, BNV>), grid, dim3(256), 0, st, M, N, K, alpha, A, lda, sa, \
                     B, ldb, sb, beta, C, ldc, sc, flags)
  if (!ak && !bn) SLAB_GEMM_CASE(false, false);
  else if (!ak && bn) SLAB_GEMM_CASE(false, true);
  else if (ak && !bn) SLAB_GEMM_CASE(true, false);
  else SLAB_GEMM_CASE(true, true);
#undef SLAB_GEMM_CASE
  SLAB_LAUNCH_CHECK();
  return SLAB_OK;
}
template int launch_gemm<float>(bool, bool, int, int, int, float, const float*, long long,
                                long long, const float*, long long, long long, float, float*,
                                long long, long long, int, int, hipStream_t);
template int launch_gemm<double>(bool, bool, int, int, int, double, const double*, long long,
                                 long long, const double*, long long, long long, double, double*,
                                 long long, long long, int, int, hipStream_t);

// ---------------------------------------------------------------------------
// Panel of the right-looking factorization of one pivot block S (n x n).
// Every workgroup first inverts the Cholesky factor of the 64x64 diagonal
// block [k0, k0+nb) in LDS: Gaussian elimination without pivoting on
// [S_kk | I], kept in one array (U on and above the diagonal, the unit lower
// L~^-1 below it), gives S_kk = L~ U with U = D L~^T, hence
// L_kk^-1 = D^-1/2 L~^-1.  Then, on 16x16x4 MFMA tiles, it either
//   * computes 64 rows of L below the block:       L_ik = S_ik L_kk^-T, or
//   * advances 64 columns of the carried inverse:  X_k = L_kk^-1 X_k.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_panel(T* __restrict__ S, T* __restrict__ Lv, int n,
                                               int k0, int nrow_wg, int* __restrict__ status,
                                               int blk) {
  typedef typename acc4<T>::type V4;
  __shared__ T E[64][65];   // elimination workspace, then L_kk^-1
  __shared__ T Bt[64][65];  // operand tile
  __shared__ T fcol[64];
  const int nb = min(64, n - k0);
  const int tid = threadIdx.x;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e >> 6, c = e & 63;
    T v = (i == c) ? (T)1 : (T)0;
    if (i < nb && c < nb) v = S[(long long)(k0 + max(i, c)) * n + k0 + min(i, c)];
    E[i][c] = v;
  }
  __syncthreads();
  for (int p = 0; p < nb; ++p) {
    if (tid < 64) fcol[tid] = (tid > p) ? E[tid][p] / E[p][p] : (T)0;
    __syncthreads();
    for (int e = tid; e < 64 * 64; e += 256) {
      const int i = e >> 6, c = e & 63;
      if (i > p) {
        if (c == p) E[i][c] = -fcol[i];
        else E[i][c] -= fcol[i] * E[p][c];
      }
    }
    __syncthreads();
  }
  if (tid < 64) {
    const T d = E[tid][tid];
    if (tid < nb && (!(d > (T)0) || !isfinite((double)d))) {
      status[0] = 3;
      status[1] = blk;
    }
    fcol[tid] = (T)1 / sqrt(d);
  }
  __syncthreads();
  for (int e = tid; e < 64 * 64; e += 256) {
    const int i = e >> 6, c = e & 63;
    E[i][c] = (c < i) ? E[i][c] * fcol[i] : ((c == i) ? fcol[i] : (T)0);
  }
  __syncthreads();

  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, nn = lane & 15;
  const int wm = wave >> 1, wn = wave & 1;
  V4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = V4{0, 0, 0, 0};
  const bool rows = (int)blockIdx.x < nrow_wg;
  const long long r0 = (long long)k0 + nb + (long long)blockIdx.x * 64;  // rows case
  const long long c0 = (long long)(blockIdx.x - nrow_wg) * 64;            // columns case
  const long long ncols = (long long)k0 + nb;
  if (rows) {
    for (int e = tid; e < 64 * 64; e += 256) {
      const int rr = e >> 6, t = e & 63;
      Bt[rr][t] = (r0 + rr < n && t < nb) ? S[(r0 + rr) * n + k0 + t] : (T)0;
    }
  } else {
    for (int e = tid; e < 64 * 64; e += 256) {
      const int t = e >> 6, cc = e & 63;
      Bt[t][cc] = (t < nb && c0 + cc < ncols) ? Lv[(long long)(k0 + t) * n + c0 + cc] : (T)0;
    }
  }
  __syncthreads();
#pragma unroll 4
  for (int ks = 0; ks < 16; ++ks) {
    const int k = 4 * ks + g;
    T av[2], bv[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const int row = wm * 32 + 16 * mt + nn;
      av[mt] = rows ? Bt[row][k] : E[row][k];
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int col = wn * 32 + 16 * nt + nn;
      bv[nt] = rows ? E[col][k] : Bt[k][col];
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = mfma16(av[mt], bv[nt], acc[mt][nt]);
  }
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = wm * 32 + 16 * mt + acc_row<T>(g, i);
        const int col = wn * 32 + 16 * nt + nn;
        if (rows) {
          if (r0 + row < n && col < nb) S[(r0 + row) * n + k0 + col] = acc[mt][nt][i];
        } else {
          if (row < nb && c0 + col < ncols) Lv[(long long)(k0 + row) * n + c0 + col] = acc[mt][nt][i];
        }
      }
}

template <typename T>
__global__ void k_identity(T* __restrict__ X, int n) {
  const long long tot = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    X[e] = (e / n == e % n) ? (T)1 : (T)0;
  }
}

// FP64 copy of a symmetric block stored in its lower triangle.
template <typename T>
__global__ void k_sym_to_f64(const T* __restrict__ S, double* __restrict__ out, int n) {
  const long long tot = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const long long i = e / n, k = e % n;
    out[e] = (double)(k <= i ? S[e] : S[k * n + i]);
  }
}

template <typename T>
int launch_stage2(const Stage2Args& a, hipStream_t st) {
  const int n = a.n, m = a.m;
  const long long nsq = (long long)n * n;
  T* Tdiag = (T*)a.Tdiag;
  T* Toff = (T*)a.Toff;
  T* Linv = (T*)a.Linv;
  T* Z = (T*)a.Z;
  const unsigned fill_grid = (unsigned)std::min<long long>((nsq + 255) / 256, 16384);
  for (int j = 0; j < m; ++j) {
    T* S = Tdiag + (long long)j * nsq;
    T* Li = Linv + (long long)j * nsq;
    if (j > 0) {
      const T* Zp = Z + (long long)(j - 1) * nsq;
      int rc = launch_gemm<T>(true, false, n, n, n, (T)-1, Zp, n, 0, Zp, n, 0, (T)1, S, n, 0, 1,
                              GEMM_LOWER_C, st);
      if (rc) return rc;
    }
    if (a.S64) {
      hipLaunchKernelGGL((k_sym_to_f64<T>), dim3(fill_grid), dim3(256), 0, st, S,
                         a.S64 + (long long)j * nsq, n);
      SLAB_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL((k_identity<T>), dim3(fill_grid), dim3(256), 0, st, Li, n);
    SLAB_LAUNCH_CHECK();
    for (int k0 = 0; k0 < n; k0 += 64) {
      const int nb = std::min(64, n - k0);
      const int nrow = n - k0 - nb;
      const int nrow_wg = (nrow + 63) / 64;
      const int ncol_wg = (k0 + nb + 63) / 64;
      hipLaunchKernelGGL((k_panel<T>), dim3(nrow_wg + ncol_wg), dim3(256), 0, st, S, Li, n, k0,
                         nrow_wg, a.status, j);
      SLAB_LAUNCH_CHECK();
      if (nrow > 0) {
        const T* P = S + (long long)(k0 + nb) * n + k0;  // rows below, panel columns
        int rc = launch_gemm<T>(false, true, nrow, nrow, nb, (T)-1, P, n, 0, P, n, 0, (T)1,
                                S + (long long)(k0 + nb) * n + (k0 + nb), n, 0, 1, GEMM_LOWER_C,
                                st);
        if (rc) return rc;
        rc = launch_gemm<T>(false, false, nrow, k0 + nb, nb, (T)-1, P, n, 0,
                            Li + (long long)k0 * n, n, 0, (T)1, Li + (long long)(k0 + nb) * n, n,
                            0, 1, 0, st);
        if (rc) return rc;
      }
    }
    if (j < m - 1) {
      int rc = launch_gemm<T>(false, false, n, n, n, (T)1, Li, n, 0, Toff + (long long)j * nsq, n,
                              0, (T)0, Z + (long long)j * nsq, n, 0, 1, GEMM_A_LOWER, st);
      if (rc) return rc;
    }
  }
  return SLAB_OK;
}
template int launch_stage2<float>(const Stage2Args&, hipStream_t);
template int launch_stage2<double>(const Stage2Args&, hipStream_t);

// ---------------------------------------------------------------------------
// Block-vector product for the sweeping solve (Alg. 2):
//   y = beta * xin + alpha * M x,  x and y hold nrhs columns of length n.
// Grid: 64-row tiles x k-splits; each k-split writes a partial sum, and the
// last workgroup of a row tile (atomic ticket) adds the partials in fixed
// order, so the result is deterministic.
// ---------------------------------------------------------------------------
constexpr int GEMV_MAXC = 32;

static int gemv_splits(int n) {
  const int tiles = (n + 63) / 64;
  int nks = std::max(1, 512 / tiles);
  return std::min(nks, tiles);
}
size_t gemv_work_bytes(int n, int nrhs, int elem) {
  return (size_t)gemv_splits(n) * nrhs * n * elem;
}
int gemv_counter_count(int n) { return (n + 63) / 64; }

template <typename T, bool TR, bool LOWER>
__global__ __launch_bounds__(256) void k_gemv(int n, int nrhs, T alpha, const T* __restrict__ M,
                                              const T* __restrict__ x, T beta,
                                              const T* __restrict__ xin, T* __restrict__ y,
                                              T* __restrict__ work, int* __restrict__ counters,
                                              int nks) {
  __shared__ T Ms[64][65];
  __shared__ T xs[GEMV_MAXC][64];
  __shared__ int last;
  const int tile = blockIdx.x, ks = blockIdx.y;
  const int i0 = tile * 64;
  const int tid = threadIdx.x;
  const int ii = tid & 63, cg = tid >> 6;
  const int ktiles = (n + 63) / 64;
  const int per = (ktiles + nks - 1) / nks;
  int kt0 = ks * per, kt1 = std::min(ktiles, kt0 + per);
  if (LOWER) {
    if (!TR) kt1 = std::min(kt1, tile + 1);   // k <= i
    else kt0 = std::max(kt0, tile);           // k >= i
  }
  T acc[GEMV_MAXC / 4];
#pragma unroll
  for (int q = 0; q < GEMV_MAXC / 4; ++q) acc[q] = (T)0;
  for (int kt = kt0; kt < kt1; ++kt) {
    const int k0 = kt * 64;
    for (int e = tid; e < 64 * 64; e += 256) {
      const int a = e >> 6, bq = e & 63;  // a slow, bq fast (coalesced)
      T v;
      if (!TR) {  // M(i0+a, k0+bq) = M[(i0+a)*n + k0+bq]
        v = (i0 + a < n && k0 + bq < n) ? M[(long long)(i0 + a) * n + k0 + bq] : (T)0;
        Ms[a][bq] = v;
      } else {    // M(i0+bq, k0+a) = M[(k0+a)*n + i0+bq]
        v = (i0 + bq < n && k0 + a < n) ? M[(long long)(k0 + a) * n + i0 + bq] : (T)0;
        Ms[bq][a] = v;
      }
    }
    for (int e = tid; e < nrhs * 64; e += 256) {
      const int c = e >> 6, kk = e & 63;
      xs[c][kk] = (k0 + kk < n) ? x[(long long)c * n + k0 + kk] : (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < GEMV_MAXC / 4; ++q) {
      const int c = cg + 4 * q;
      if (c < nrhs) {
        T s = acc[q];
#pragma unroll 16
        for (int kk = 0; kk < 64; ++kk) s += Ms[ii][kk] * xs[c][kk];
        acc[q] = s;
      }
    }
    __syncthreads();
  }
  const int i = i0 + ii;
  if (nks == 1) {
#pragma unroll
    for (int q = 0; q < GEMV_MAXC / 4; ++q) {
      const int c = cg + 4 * q;
      if (c < nrhs && i < n) {
        T v = alpha * acc[q];
        if (xin) v += beta * xin[(long long)c * n + i];
        y[(long long)c * n + i] = v;
      }
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < GEMV_MAXC / 4; ++q) {
    const int c = cg + 4 * q;
    if (c < nrhs && i < n) work[((long long)ks * nrhs + c) * n + i] = acc[q];
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) last = (atomicAdd(&counters[tile], 1) == nks - 1);
  __syncthreads();
  if (!last) return;
  __threadfence();
#pragma unroll
  for (int q = 0; q < GEMV_MAXC / 4; ++q) {
    const int c = cg + 4 * q;
    if (c < nrhs && i < n) {
      T s = (T)0;
      for (int k = 0; k < nks; ++k) s += work[((long long)k * nrhs + c) * n + i];
      T v = alpha * s;
      if (xin) v += beta * xin[(long long)c * n + i];
      y[(long long)c * n + i] = v;
    }
  }
  if (tid == 0) counters[tile] = 0;
}

template <typename T>
int launch_gemv(bool tr, bool lower, int n, int nrhs, T alpha, const T* M, const T* x, T beta,
                const T* xin, T* y, void* work, int* counters, hipStream_t st) {
  const int nks = gemv_splits(n);
  for (int c0 = 0; c0 < nrhs; c0 += GEMV_MAXC) {
    const int nc = std::min(GEMV_MAXC, nrhs - c0);
    const long long off = (long long)c0 * n;
    dim3 grid((n + 63) / 64, nks);
#define SLAB_GEMV_CASE(TRV, LOV)                                                                \
  hipLaunchKernelGGL((k_gemv<T, TRV, LOV>), grid, dim3(256), 0, st, n, nc, alpha, M, x + off,  \
                     beta, xin ? xin + off : nullptr, y + off, (T*)work, counters, nks)
    if (!tr && !lower) SLAB_GEMV_CASE(false, false);
    else if (!tr && lower) SLAB_GEMV_CASE(false, true);
    else if (tr && !lower) SLAB_GEMV_CASE(true, false);
    else SLAB_GEMV_CASE(true, true);
#undef SLAB_GEMV_CASE
    SLAB_LAUNCH_CHECK();
  }
  return SLAB_OK;
}
template int launch_gemv<float>(bool, bool, int, int, float, const float*, const float*, float,
                                const float*, float*, void*, int*, hipStream_t);
template int launch_gemv<double>(bool, bool, int, int, double, const double*, const double*,
                                 double, const double*, double*, void*, int*, hipStream_t);

// ---------------------------------------------------------------------------
__global__ void k_cast_f64(const void* __restrict__ src, int is_float, double* __restrict__ dst,
                           long long count) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < count;
       e += (long long)gridDim.x * blockDim.x)
    dst[e] = is_float ? (double)((const float*)src)[e] : ((const double*)src)[e];
}

int launch_cast_f64(const void* src, int src_is_float, double* dst, long long count,
                    hipStream_t st) {
  unsigned grid = (unsigned)std::min<long long>((count + 255) / 256, 16384);
  hipLaunchKernelGGL(k_cast_f64, dim3(grid), dim3(256), 0, st, src, src_is_float, dst, count);
  SLAB_LAUNCH_CHECK();
  return SLAB_OK;
}

}  // namespace slab
