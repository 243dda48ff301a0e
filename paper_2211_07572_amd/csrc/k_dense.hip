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
// Tiled MFMA GEMM: C = beta*C + alpha * op(A) op(B) for gridDim.z independent
// products (operands sa, sb, sc elements apart).
// TILE x TILE output tile per workgroup, four waves of (TILE/2)^2, k chunks of
// TK.  The next chunk is loaded into registers (16-byte vector loads when the
// leading dimensions allow) while the current one is multiplied out of LDS;
// one barrier per chunk (double-buffered LDS).
//   op(A)(i,k) = A[i*lda+k] (AK=false) or A[k*lda+i] (AK=true)
//   op(B)(k,j) = B[k*ldb+j] (BN=false) or B[j*ldb+k] (BN=true)
// flags: GEMM_LOWER_C computes only tiles on or below the diagonal (a linear
// tile index over the lower triangle); GEMM_A_LOWER / GEMM_B_LOWER skip the
// k ranges where op(A) / op(B) is known to be zero (lower-triangular factors).
// ---------------------------------------------------------------------------
template <typename T, int TILE, int TK, bool AK, bool BN, bool VECOK>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, T alpha,
                                              const T* __restrict__ A, long long lda,
                                              long long sa, const T* __restrict__ B,
                                              long long ldb, long long sb, T beta, T* C,
                                              long long ldc, long long sc, int flags) {
  typedef typename acc4<T>::type V4;
  constexpr int TM = TILE, TN = TILE;
  constexpr int FM = TILE / 32, FN = TILE / 32;  // 16x16 MFMA tiles per wave and direction
  constexpr int VEC = 16 / sizeof(T);
  constexpr int NV = TM * TK / 256 / VEC;  // vectors per thread per operand and chunk
  static_assert(NV >= 1 && TM * TK == NV * VEC * 256, "tile shape");
  typedef T vt __attribute__((ext_vector_type(VEC)));
  __shared__ T As[2][TK][TM + 4];
  __shared__ T Bs[2][TK][TN + 4];
  int ti, tj;
  if (flags & GEMM_LOWER_C) {
    const long long t = blockIdx.x;
    int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((long long)(r + 1) * (r + 2) / 2 <= t) ++r;
    while ((long long)r * (r + 1) / 2 > t) --r;
    ti = r;
    tj = (int)(t - (long long)r * (r + 1) / 2);
  } else {
    // with A lower triangular the last tile rows carry the longest k ranges:
    // hand them out first
    ti = (flags & GEMM_A_LOWER) ? (int)(gridDim.y - 1 - blockIdx.y) : (int)blockIdx.y;
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
  const int kmax = (flags & GEMM_A_LOWER) ? min(K, i0 + TM) : K;
  kmin = (kmin / TK) * TK;

  vt ra[NV], rb[NV];
  auto load = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int v = tid + 256 * q;
      int row, kk;
      if (!AK) { row = v / (TK / VEC); kk = (v % (TK / VEC)) * VEC; }
      else { kk = v / (TM / VEC); row = (v % (TM / VEC)) * VEC; }
      const long long gi = i0 + row, gk = k0 + kk;
      if (VECOK) {
        const bool in = gi < M && gk < kmax;
        ra[q] = in ? *(const vt*)(!AK ? A + gi * lda + gk : A + gk * lda + gi) : vt(0);
        if (in) {  // partial vectors at the edges
#pragma unroll
          for (int e = 0; e < VEC; ++e)
            if (!AK ? (gk + e >= kmax) : (gi + e >= M)) ra[q][e] = (T)0;
        }
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const long long ii = !AK ? gi : gi + e, kq = !AK ? gk + e : gk;
          ra[q][e] = (ii < M && kq < kmax) ? A[!AK ? ii * lda + kq : kq * lda + ii] : (T)0;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int v = tid + 256 * q;
      int col, kk;
      if (!BN) { kk = v / (TN / VEC); col = (v % (TN / VEC)) * VEC; }
      else { col = v / (TK / VEC); kk = (v % (TK / VEC)) * VEC; }
      const long long gj = j0 + col, gk = k0 + kk;
      if (VECOK) {
        const bool in = gj < N && gk < kmax;
        rb[q] = in ? *(const vt*)(!BN ? B + gk * ldb + gj : B + gj * ldb + gk) : vt(0);
        if (in) {
#pragma unroll
          for (int e = 0; e < VEC; ++e)
            if (!BN ? (gj + e >= N) : (gk + e >= kmax)) rb[q][e] = (T)0;
        }
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const long long jj = !BN ? gj + e : gj, kq = !BN ? gk : gk + e;
          rb[q][e] = (jj < N && kq < kmax) ? B[!BN ? kq * ldb + jj : jj * ldb + kq] : (T)0;
        }
      }
    }
  };
  auto park = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int v = tid + 256 * q;
      if (!AK) {
        const int row = v / (TK / VEC), kk = (v % (TK / VEC)) * VEC;
#pragma unroll
        for (int e = 0; e < VEC; ++e) As[buf][kk + e][row] = ra[q][e];
      } else {
        const int kk = v / (TM / VEC), row = (v % (TM / VEC)) * VEC;
#pragma unroll
        for (int e = 0; e < VEC; ++e) As[buf][kk][row + e] = ra[q][e];
      }
      if (!BN) {
        const int kk = v / (TN / VEC), col = (v % (TN / VEC)) * VEC;
#pragma unroll
        for (int e = 0; e < VEC; ++e) Bs[buf][kk][col + e] = rb[q][e];
      } else {
        const int col = v / (TK / VEC), kk = (v % (TK / VEC)) * VEC;
#pragma unroll
        for (int e = 0; e < VEC; ++e) Bs[buf][kk + e][col] = rb[q][e];
      }
    }
  };

  V4 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = V4{0, 0, 0, 0};

  if (kmin < kmax) {
    load(kmin);
    park(0);
    __syncthreads();
    int it = 0;
    for (int k0 = kmin; k0 < kmax; k0 += TK, ++it) {
      const int cur = it & 1;
      const bool more = k0 + TK < kmax;
      if (more) load(k0 + TK);
#pragma unroll
      for (int ks = 0; ks < TK / 4; ++ks) {
        T av[FM], bv[FN];
#pragma unroll
        for (int mt = 0; mt < FM; ++mt) av[mt] = As[cur][4 * ks + g][wm * (TM / 2) + 16 * mt + nn];
#pragma unroll
        for (int nt = 0; nt < FN; ++nt) bv[nt] = Bs[cur][4 * ks + g][wn * (TN / 2) + 16 * nt + nn];
#pragma unroll
        for (int mt = 0; mt < FM; ++mt)
#pragma unroll
          for (int nt = 0; nt < FN; ++nt) acc[mt][nt] = mfma16(av[mt], bv[nt], acc[mt][nt]);
      }
      if (more) park(cur ^ 1);
      __syncthreads();
    }
  }
#pragma unroll
  for (int mt = 0; mt < FM; ++mt)
#pragma unroll
    for (int nt = 0; nt < FN; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long long gi = i0 + wm * (TM / 2) + 16 * mt + acc_row<T>(g, i);
        const long long gj = j0 + wn * (TN / 2) + 16 * nt + nn;
        if (gi < M && gj < N) {
          T v = alpha * acc[mt][nt][i];
          if (beta != (T)0) v += beta * C[gi * ldc + gj];
          C[gi * ldc + gj] = v;
        }
      }
}

template <typename T, int TILE, int TK>
static void gemm_tile(bool ak, bool bn, bool vecok, dim3 grid, int M, int N, int K, T alpha,
                      const T* A, long long lda, long long sa, const T* B, long long ldb,
                      long long sb, T beta, T* C, long long ldc, long long sc, int flags,
                      hipStream_t st) {
#define SLAB_GEMM_CASE(AKV, BNV)                                                                 \
  do {                                                                                           \
    if (vecok)                                                                                   \
      hipLaunchKernelGGL((k_gemm<T, TILE, TK, AKV, BNV, true>), grid, dim3(256), 0, st, M, N, K, \
                         alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, flags);                \
    else                                                                                         \
      hipLaunchKernelGGL((k_gemm<T, TILE, TK, AKV, BNV, false>), grid, dim3(256), 0, st, M, N,   \
                         K, alpha, A, lda, sa, B, ldb, sb, beta, C, ldc, sc, flags);             \
  } while (0)
  if (!ak && !bn) SLAB_GEMM_CASE(false, false);
  else if (!ak && bn) SLAB_GEMM_CASE(false, true);
  else if (ak && !bn) SLAB_GEMM_CASE(true, false);
  else SLAB_GEMM_CASE(true, true);
#undef SLAB_GEMM_CASE
}

template <typename T>
int launch_gemm(bool ak, bool bn, int M, int N, int K, T alpha, const T* A, long long lda,
                long long sa, const T* B, long long ldb, long long sb, T beta, T* C,
                long long ldc, long long sc, int batch, int flags, hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return SLAB_OK;
  // 128-wide tiles once there are enough of them for four per compute unit
  const int tile = (sizeof(T) == 4 && (long long)M * N * batch >= 1024LL * 128 * 128) ? 128 : 64;
  const int tm = (M + tile - 1) / tile, tn = (N + tile - 1) / tile;
  dim3 grid;
  if (flags & GEMM_LOWER_C) grid = dim3((unsigned)((long long)tm * (tm + 1) / 2), 1, batch);
  else grid = dim3(tn, tm, batch);
  // 16-byte vector loads need 16-byte aligned bases, strides and batch strides
  const long long vec = 16 / (long long)sizeof(T);
  const bool vecok = lda % vec == 0 && ldb % vec == 0 && sa % vec == 0 && sb % vec == 0 &&
                     ((uintptr_t)A & 15) == 0 && ((uintptr_t)B & 15) == 0;
  if (tile == 128)
    gemm_tile<T, 128, 16>(ak, bn, vecok, grid, M, N, K, alpha, A, lda, sa, B, ldb, sb, beta, C,
                          ldc, sc, flags, st);
  else
    gemm_tile<T, 64, 32>(ak, bn, vecok, grid, M, N, K, alpha, A, lda, sa, B, ldb, sb, beta, C,
                         ldc, sc, flags, st);
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
// Panel of the right-looking factorization of a pivot block S (n x n), for
// gridDim.y independent blocks at once.
// Every workgroup first inverts the Cholesky factor of the 64x64 diagonal
// block [k0, k0+nb): Gaussian elimination without pivoting on [S_kk | I],
// kept in one array (U on and above the diagonal, the unit lower L~^-1 below
// it), gives S_kk = L~ U with U = D L~^T, hence L_kk^-1 = D^-1/2 L~^-1.  The
// working matrix lives in registers (thread = row x 16-column quarter); each
// elimination step exchanges only the pivot row and column through LDS, with
// one barrier per step.  Then, on 16x16x4 MFMA tiles, it either
//   * computes 64 rows of L below the block:       L_ik = S_ik L_kk^-T, or
//   * advances 64 columns of the carried inverse:  X_k = L_kk^-1 X_k.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_panel(T* __restrict__ S, T* __restrict__ Lv, int n,
                                               int k0, int nrow_wg, int* __restrict__ status,
                                               int blk, long long bs, int blk_step) {
  typedef typename acc4<T>::type V4;
  // blockIdx.y selects one of several independent pivot blocks, bs elements apart
  S += (long long)blockIdx.y * bs;
  Lv += (long long)blockIdx.y * bs;
  blk += (int)blockIdx.y * blk_step;
  __shared__ T E[64][65];   // L_kk^-1 after the elimination
  __shared__ T Bt[64][65];  // operand tile
  __shared__ T rowbuf[2][64];
  __shared__ T colbuf[2][64];
  const int nb = min(64, n - k0);
  const int tid = threadIdx.x;
  // thread (row i, column quarter q) keeps 16 entries of the working matrix in registers
  const int i = tid & 63, q = tid >> 6;
  T a[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int col = 16 * q + c;
    T v = (i == col) ? (T)1 : (T)0;
    if (i < nb && col < nb) v = S[(long long)(k0 + max(i, col)) * n + k0 + min(i, col)];
    a[c] = v;
  }
  if (i == 0) {
#pragma unroll
    for (int c = 0; c < 16; ++c) rowbuf[0][16 * q + c] = a[c];
  }
  if (q == 0) colbuf[0][i] = a[0];
  __syncthreads();
  // pivot p = 16 pb + pp: the register index pp is a compile-time constant and
  // the owner of column p is the wave q == pb (uniform branches only)
  for (int pb = 0; pb < 4; ++pb) {
#pragma unroll
    for (int pp = 0; pp < 16; ++pp) {
      const int p = 16 * pb + pp;
      if (p >= nb) break;
      const int buf = p & 1;
      const T ipiv = (T)1 / rowbuf[buf][p];
      T rp[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) rp[c] = rowbuf[buf][16 * q + c];
      const T f = (i > p) ? colbuf[buf][i] * ipiv : (T)0;  // f = 0 keeps rows <= p
#pragma unroll
      for (int c = 0; c < 16; ++c) a[c] -= f * rp[c];
      if (q == pb && i > p) a[pp] = -f;
      if (p + 1 < nb) {  // publish the next pivot row and pivot column
        if (i == p + 1) {
#pragma unroll
          for (int c = 0; c < 16; ++c) rowbuf[buf ^ 1][16 * q + c] = a[c];
        }
        if (pp < 15) {
          if (q == pb) colbuf[buf ^ 1][i] = a[(pp + 1) & 15];
        } else {
          if (q == pb + 1) colbuf[buf ^ 1][i] = a[0];
        }
      }
      __syncthreads();
    }
  }
  // diagonal of U is D; L_kk^-1 = D^-1/2 L~^-1
  if (q == (i >> 4)) {
    T d = (T)1;
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (c == (i & 15)) d = a[c];
    if (i < nb && (!(d > (T)0) || !isfinite((double)d))) {
      status[0] = 3;
      status[1] = blk;
    }
    colbuf[0][i] = (T)1 / sqrt(d);
  }
  __syncthreads();
  {
    const T rs = colbuf[0][i];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int col = 16 * q + c;
      E[i][col] = (col < i) ? a[c] * rs : ((col == i) ? rs : (T)0);
    }
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

// ---------------------------------------------------------------------------
// Update after panel [k0, k0+nb) of the factorization of one pivot block:
//   trailing  S_ij -= L_i L_j^T     (lower 64x64 tiles of rows/cols >= k0+nb)
//   carried   X_ic -= L_i X_k,c     (rows >= k0+nb, columns < k0+nb)
// with L_i = S[i, k0:k0+nb] (just computed by the panel) and X_k the panel's
// rows of the carried inverse.  One launch covers both tile kinds; every
// workgroup issues all its loads (A, B and the C tile) before the first MFMA.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_rank64(T* __restrict__ S, T* __restrict__ Lv, int n,
                                                int k0, int nb, int ntrail, long long bs) {
  typedef typename acc4<T>::type V4;
  S += (long long)blockIdx.y * bs;
  Lv += (long long)blockIdx.y * bs;
  __shared__ T As[64][65];  // As[row][k]
  __shared__ T Bs[64][65];  // Bs[col][k]
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, nn = lane & 15;
  const int wm = wave >> 1, wn = wave & 1;
  const long long base = (long long)k0 + nb;
  long long r0, c0;
  T* C;
  bool trail = (int)blockIdx.x < ntrail;
  if (trail) {
    const long long t = blockIdx.x;
    int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((long long)(r + 1) * (r + 2) / 2 <= t) ++r;
    while ((long long)r * (r + 1) / 2 > t) --r;
    r0 = base + 64LL * r;
    c0 = base + 64LL * (t - (long long)r * (r + 1) / 2);
    C = S;
  } else {
    const long long t = blockIdx.x - ntrail;
    const long long ncb = (base + 63) / 64;
    r0 = base + 64LL * (t / ncb);
    c0 = 64LL * (t % ncb);
    C = Lv;
  }
  const long long cmax = trail ? n : base;
  // A: L rows r0.., panel columns
  for (int e = tid; e < 64 * 64; e += 256) {
    const int rr = e >> 6, k = e & 63;
    As[rr][k] = (r0 + rr < n && k < nb) ? S[(r0 + rr) * n + k0 + k] : (T)0;
  }
  // B: trailing -> L rows c0.. (B(k, j) = L[j][k]); carried -> X_k rows (B(k, c) = X[k0+k][c])
  if (trail) {
    for (int e = tid; e < 64 * 64; e += 256) {
      const int cc = e >> 6, k = e & 63;
      Bs[cc][k] = (c0 + cc < n && k < nb) ? S[(c0 + cc) * n + k0 + k] : (T)0;
    }
  } else {
    for (int e = tid; e < 64 * 64; e += 256) {
      const int k = e >> 6, cc = e & 63;
      Bs[cc][k] = (k < nb && c0 + cc < cmax) ? Lv[(long long)(k0 + k) * n + c0 + cc] : (T)0;
    }
  }
  // C is loaded up front; the 64 products are summed first and subtracted once
  // (adding them one by one into the larger C would lose accuracy in FP32)
  T cin[2][2][4];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long long row = r0 + wm * 32 + 16 * mt + acc_row<T>(g, i);
        const long long col = c0 + wn * 32 + 16 * nt + nn;
        cin[mt][nt][i] = (row < n && col < cmax) ? C[row * n + col] : (T)0;
      }
  V4 acc[2][2];
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = V4{0, 0, 0, 0};
  __syncthreads();
#pragma unroll 4
  for (int ks = 0; ks < 16; ++ks) {
    const int k = 4 * ks + g;
    T av[2], bv[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) av[mt] = As[wm * 32 + 16 * mt + nn][k];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) bv[nt] = Bs[wn * 32 + 16 * nt + nn][k];
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
        const long long row = r0 + wm * 32 + 16 * mt + acc_row<T>(g, i);
        const long long col = c0 + wn * 32 + 16 * nt + nn;
        if (row < n && col < cmax) C[row * n + col] = cin[mt][nt][i] - acc[mt][nt][i];
      }
}

template <typename T>
__global__ void k_identity(T* __restrict__ X, int n, long long bs) {
  X += (long long)blockIdx.y * bs;
  const long long tot = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    X[e] = (e / n == e % n) ? (T)1 : (T)0;
  }
}

// FP64 copy of a symmetric block stored in its lower triangle.
template <typename T>
__global__ void k_sym_to_f64(const T* __restrict__ S, double* __restrict__ out, int n,
                             long long bs) {
  S += (long long)blockIdx.y * bs;
  out += (long long)blockIdx.y * bs;
  const long long tot = (long long)n * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const long long i = e / n, k = e % n;
    out[e] = (double)(k <= i ? S[e] : S[k * n + i]);
  }
}

// Cholesky factorization with carried inverse of `count` pivot blocks S_q =
// S + q*bs (n x n, lower triangles), L_q^-1 into Li + q*bs; breakdown of block
// q is reported as blk0 + q*blk_step.
template <typename T>
static int factor_blocks(T* S, T* Li, int n, int count, long long bs, int blk0, int blk_step,
                         double* S64, int* status, hipStream_t st) {
  if (count <= 0) return SLAB_OK;
  const long long nsq = (long long)n * n;
  const unsigned fill_grid = (unsigned)std::min<long long>((nsq + 255) / 256, 4096);
  if (S64) {
    hipLaunchKernelGGL((k_sym_to_f64<T>), dim3(fill_grid, count), dim3(256), 0, st, S, S64, n, bs);
    SLAB_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL((k_identity<T>), dim3(fill_grid, count), dim3(256), 0, st, Li, n, bs);
  SLAB_LAUNCH_CHECK();
  for (int k0 = 0; k0 < n; k0 += 64) {
    const int nb = std::min(64, n - k0);
    const int nrow = n - k0 - nb;
    const int nrow_wg = (nrow + 63) / 64;
    const int ncol_wg = (k0 + nb + 63) / 64;
    hipLaunchKernelGGL((k_panel<T>), dim3(nrow_wg + ncol_wg, count), dim3(256), 0, st, S, Li, n,
                       k0, nrow_wg, status, blk0, bs, blk_step);
    SLAB_LAUNCH_CHECK();
    if (nrow > 0) {
      const long long tr = (nrow + 63) / 64;
      const int ntrail = (int)(tr * (tr + 1) / 2);
      const int naug = (int)(tr * ((k0 + nb + 63) / 64));
      hipLaunchKernelGGL((k_rank64<T>), dim3(ntrail + naug, count), dim3(256), 0, st, S, Li, n,
                         k0, nb, ntrail, bs);
      SLAB_LAUNCH_CHECK();
    }
  }
  return SLAB_OK;
}

template <typename T>
int launch_stage2(const Stage2Args& a, hipStream_t st) {
  const int n = a.n, m = a.m;
  const long long nsq = (long long)n * n;
  T* Tdiag = (T*)a.Tdiag;
  T* Toff = (T*)a.Toff;
  T* Linv = (T*)a.Linv;
  T* Z = (T*)a.Z;
  if (!a.odd_even) {
    // Alg. 1 in block Cholesky form: S_j = T_jj - Z_{j-1}^T Z_{j-1}, S_j = L_j L_j^T,
    // Z_j = L_j^-1 T_{j,j+1}
    for (int j = 0; j < m; ++j) {
      T* S = Tdiag + (long long)j * nsq;
      T* Li = Linv + (long long)j * nsq;
      if (j > 0) {
        const T* Zp = Z + (long long)(j - 1) * nsq;
        int rc = launch_gemm<T>(true, false, n, n, n, (T)-1, Zp, n, 0, Zp, n, 0, (T)1, S, n, 0, 1,
                                GEMM_LOWER_C, st);
        if (rc) return rc;
      }
      int rc = factor_blocks<T>(S, Li, n, 1, 0, j, 0, a.S64 ? a.S64 + (long long)j * nsq : nullptr,
                                a.status, st);
      if (rc) return rc;
      if (j < m - 1) {
        rc = launch_gemm<T>(false, false, n, n, n, (T)1, Li, n, 0, Toff + (long long)j * nsq, n,
                            0, (T)0, Z + (long long)j * nsq, n, 0, 1, GEMM_A_LOWER, st);
        if (rc) return rc;
      }
    }
    return SLAB_OK;
  }
  // Odd-even order.  At level l (stride s = 2^l) the interfaces still present
  // are a_p = (p+1)s - 1, p < k = floor(m/s); those at even positions,
  // e_q = (2q+1)s - 1, q < E = ceil(k/2), are eliminated together.  e_q has a
  // kept neighbour l = e_q - s when q >= 1 and r = e_q + s when q < floor(k/2).
  // With D_e = L L^T:  U_e = L^-1 C_l^T (stored over D_e), V_e = L^-1 C_e (in Z),
  //   D_l -= U_e^T U_e,  D_r -= V_e^T V_e,  C_l = -U_e^T V_e,
  // where C_x (in Toff) is the coupling of x to the next interface present.
  for (long long s = 1; m / s >= 1; s *= 2) {
    const int k = (int)(m / s);
    const int E = (k + 1) / 2, NR = k / 2;
    const long long e0 = s - 1, es = 2 * s * nsq;
    int rc = factor_blocks<T>(Tdiag + e0 * nsq, Linv + e0 * nsq, n, E, es, (int)e0, (int)(2 * s),
                              a.S64 ? a.S64 + e0 * nsq : nullptr, a.status, st);
    if (rc) return rc;
    const long long e1 = e0 + 2 * s;  // first eliminated interface with a left neighbour
    if (E > 1) {  // U_e = L_e^-1 C_{e-s}^T
      rc = launch_gemm<T>(false, true, n, n, n, (T)1, Linv + e1 * nsq, n, es,
                          Toff + (e1 - s) * nsq, n, es, (T)0, Tdiag + e1 * nsq, n, es, E - 1,
                          GEMM_A_LOWER, st);
      if (rc) return rc;
    }
    if (NR > 0) {  // V_e = L_e^-1 C_e
      rc = launch_gemm<T>(false, false, n, n, n, (T)1, Linv + e0 * nsq, n, es, Toff + e0 * nsq, n,
                          es, (T)0, Z + e0 * nsq, n, es, NR, GEMM_A_LOWER, st);
      if (rc) return rc;
    }
    if (E > 1) {  // D_l -= U_e^T U_e
      rc = launch_gemm<T>(true, false, n, n, n, (T)-1, Tdiag + e1 * nsq, n, es, Tdiag + e1 * nsq,
                          n, es, (T)1, Tdiag + (e1 - s) * nsq, n, es, E - 1, GEMM_LOWER_C, st);
      if (rc) return rc;
    }
    if (NR > 0) {  // D_r -= V_e^T V_e
      rc = launch_gemm<T>(true, false, n, n, n, (T)-1, Z + e0 * nsq, n, es, Z + e0 * nsq, n, es,
                          (T)1, Tdiag + (e0 + s) * nsq, n, es, NR, GEMM_LOWER_C, st);
      if (rc) return rc;
    }
    if (NR > 1) {  // C_l = -U_e^T V_e for the interfaces with both neighbours
      rc = launch_gemm<T>(true, false, n, n, n, (T)-1, Tdiag + e1 * nsq, n, es, Z + e1 * nsq, n,
                          es, (T)0, Toff + (e1 - s) * nsq, n, es, NR - 1, 0, st);
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
// 16 columns at a time on 16x16x4 MFMA tiles.  A workgroup owns 16 rows; its
// sixteen waves split k and are reduced through LDS, so no result crosses a
// workgroup (a device-scope fence would write back every L2 of the chip).
// Each lane loads 16 contiguous bytes of M and of x per step, which feed
// VEC consecutive MFMA k-steps (k permuted consistently in A and B).
// ---------------------------------------------------------------------------
constexpr int BMV_WAVES = 16;



template <typename T, bool TR, bool LOWER>
__global__ __launch_bounds__(1024) void k_bmv(int n, int nrhs, T alpha, const T* __restrict__ M,
                                             long long sM, const T* __restrict__ x, long long sx,
                                             T beta, const T* xin, long long sxin, T* y,
                                             long long sy) {
  // blockIdx.z: independent product q (operands sM, sx, sxin, sy elements
  // apart); blockIdx.y: group of 16 columns.  xin may alias y.
  M += (long long)blockIdx.z * sM;
  {
    const long long c0 = (long long)blockIdx.y * 16 * n;
    x += (long long)blockIdx.z * sx + c0;
    if (xin) xin += (long long)blockIdx.z * sxin + c0;
    y += (long long)blockIdx.z * sy + c0;
  }
  const int nc = min(16, nrhs - 16 * (int)blockIdx.y);
  typedef typename acc4<T>::type V4;
  constexpr int VEC = 16 / sizeof(T);   // elements per 16-byte load
  constexpr int KS = 4 * VEC;           // k covered by one load per lane
  __shared__ T red[BMV_WAVES][16][17];
  const int row0 = blockIdx.x * 16;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, nn = lane & 15;
  int klo = 0, khi = n;
  if (LOWER) {
    if (!TR) khi = min(n, row0 + 16);      // M(i,k) = 0 for k > i
    else klo = row0;                       // M(i,k) = 0 for k < i
  }
  // split [klo, khi) over the waves in whole KS chunks
  const int nch = (khi - klo + KS - 1) / KS;
  const int per = (nch + BMV_WAVES - 1) / BMV_WAVES;
  const int c_begin = wave * per, c_end = min(nch, c_begin + per);
  const int row = row0 + nn;
  const bool rowok = row < n;
  const bool colok = nn < nc;
  V4 acc = V4{0, 0, 0, 0};
#pragma unroll 8
  for (int ch = c_begin; ch < c_end; ++ch) {
    const int kb = klo + ch * KS + VEC * g;   // this lane's first k of the chunk
    T av[VEC], bv[VEC];
    if (!TR && rowok && kb + VEC <= n && ((((size_t)row * n + kb) * sizeof(T)) & 15) == 0) {
      typedef T vt __attribute__((ext_vector_type(VEC)));
      const vt v = *(const vt*)(M + (size_t)row * n + kb);
#pragma unroll
      for (int t = 0; t < VEC; ++t) av[t] = v[t];
    } else {
#pragma unroll
      for (int t = 0; t < VEC; ++t) {
        const int k = kb + t;
        av[t] = (rowok && k < n) ? (TR ? M[(size_t)k * n + row] : M[(size_t)row * n + k]) : (T)0;
      }
    }
#pragma unroll
    for (int t = 0; t < VEC; ++t) {
      const int k = kb + t;
      bv[t] = (colok && k < n) ? x[(size_t)nn * n + k] : (T)0;
    }
#pragma unroll
    for (int t = 0; t < VEC; ++t) acc = mfma16(av[t], bv[t], acc);
  }
  // acc[i]: row 16 blockIdx + acc_row(g, i), column nn; reduce the waves
#pragma unroll
  for (int i = 0; i < 4; ++i) red[wave][acc_row<T>(g, i)][nn] = acc[i];
  __syncthreads();
  if (tid < 256) {
    const int rr = tid >> 4, c = tid & 15;
    const int r = row0 + rr;
    if (r < n && c < nc) {
      T sum = (T)0;
#pragma unroll
      for (int w = 0; w < BMV_WAVES; ++w) sum += red[w][rr][c];
      T v = alpha * sum;
      if (xin) v += beta * xin[(size_t)c * n + r];
      y[(size_t)c * n + r] = v;
    }
  }
}

template <typename T>
int launch_gemv(bool tr, bool lower, int n, int nrhs, T alpha, const T* M, long long sM,
                const T* x, long long sx, T beta, const T* xin, long long sxin, T* y, long long sy,
                int batch, hipStream_t st) {
  if (batch <= 0 || nrhs <= 0 || n <= 0) return SLAB_OK;
  dim3 grid((n + 15) / 16, (nrhs + 15) / 16, batch);
#define SLAB_BMV_CASE(TRV, LOV)                                                                   \
  hipLaunchKernelGGL((k_bmv<T, TRV, LOV>), grid, dim3(64 * BMV_WAVES), 0, st, n, nrhs, alpha, M, \
                     sM, x, sx, beta, xin, sxin, y, sy)
  if (!tr && !lower) SLAB_BMV_CASE(false, false);
  else if (!tr && lower) SLAB_BMV_CASE(false, true);
  else if (tr && !lower) SLAB_BMV_CASE(true, false);
  else SLAB_BMV_CASE(true, true);
#undef SLAB_BMV_CASE
  SLAB_LAUNCH_CHECK();
  return SLAB_OK;
}
template int launch_gemv<float>(bool, bool, int, int, float, const float*, long long,
                                const float*, long long, float, const float*, long long, float*,
                                long long, int, hipStream_t);
template int launch_gemv<double>(bool, bool, int, int, double, const double*, long long,
                                 const double*, long long, double, const double*, long long,
                                 double*, long long, int, hipStream_t);

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
