// Stage two of the slab solver: block factorization of the block-tridiagonal
// reduced matrix T (Alg. 1) and the dense kernels it is built from.
//
// T is symmetric positive definite for kappa > 0, so every S_j of Alg. 1 is
// too.  Alg. 1 keeps the inverse of each S_j; here it is held as the Cholesky
// factor S_j = L_j L_j^T with its explicit inverse L_j^-1, and the next pivot
// block is formed as
//   S_{j+1} = T_{j+1,j+1} - Z_j^T Z_j,   Z_j = L_j^-1 T_{j,j+1},
// which equals T_{j+1,j+1} - T_{j+1,j} S_j^-1 T_{j,j+1} since T_{j+1,j} = T_{j,j+1}^T.
// A Helmholtz term (eq. (var_helm)) can make T indefinite while the slab
// interiors stay definite; the pivot blocks are then factored in signed form
// S_j = L_j J_j L_j^T, J_j = diag(+-1) (the signs of the pivots of the
// elimination without pivoting), S_j^-1 = L_j^-T J_j L_j^-1, and every product
// that passes through S_j^-1 carries J_j between its two factors:
//   S_{j+1} = T_{j+1,j+1} - Z_j^T J_j Z_j.
// The factorization of each S_j is right-looking in 64-column panels; the
// identity carried along as extra columns turns into L_j^-1 (forward
// substitution with a matrix right-hand side).  All products run on
// 16x16x4 MFMA tiles in the working precision (FP32 or FP64).
#include "launch.h"

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>

namespace slab {

// ---------------------------------------------------------------------------
// Tiled MFMA GEMM: C = beta*C + alpha * op(A) op(B) for a group of independent
// products (one GemmItem each, grouped launch).
// Tiles are numbered per XCD (xcd_linear) and, inside a product, in bands of
// eight tile rows walked column by column, so that the workgroups resident on
// one XCD at a time cover a near-square block of C and read each A and B panel
// once into that XCD's L2.
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
#ifndef SLAB_GEMM_WAVES
#define SLAB_GEMM_WAVES 1   // minimum waves per SIMD asked of the register allocator
                                   // (4 fits the 128 tile in 126 registers: no faster)
#endif
// KS: op(A)(i, k) is taken times items[].kscale[k] (pivot signs J).
template <typename T, int TILE, int TK, bool AK, bool BN, bool VECOK, bool CPRE = false,
          int WNF = 1, bool KS = false>
__global__ __launch_bounds__(256, SLAB_GEMM_WAVES) void k_gemm(const GemmItem* __restrict__ items,
                                              const int* __restrict__ offs, int count, T alpha,
                                              T beta, int flags) {
  typedef typename acc4<T>::type V4;
  // WNF = 2: TILE x 2 TILE output tiles, each wave TILE/2 x TILE (twice the
  // MFMAs per fragment read; full-output products only)
  constexpr int TM = TILE, TN = TILE * WNF;
  constexpr int FM = TM / 32, FN = TN / 32;  // 16x16 MFMA tiles per wave and direction
  constexpr int VEC = 16 / sizeof(T);
  constexpr int NV = TM * TK / 256 / VEC;  // vectors of op(A) per thread and chunk
  constexpr int NVB = TN * TK / 256 / VEC;  // vectors of op(B)
  static_assert(NV >= 1 && TM * TK == NV * VEC * 256 && NVB * VEC * 256 == TN * TK, "tile shape");
  typedef T vt __attribute__((ext_vector_type(VEC)));
  __shared__ T As[2][TK][TM + 4];
  __shared__ T Bs[2][TK][TN + 4];
  // (products with a lower-triangular A keep the row order inside an XCD range)
  const int vb = xcd_linear(blockIdx.x, gridDim.x);
  const int itm = group_item(offs, count, vb);
  const long long bx = vb - offs[itm];
  const g_t<const T>* __restrict__ A = gp((const T*)items[itm].A);
  const g_t<const T>* __restrict__ B = gp((const T*)items[itm].B);
  g_t<T>* C = gp((T*)items[itm].C);
  const g_t<const T>* __restrict__ ksc = gp((const T*)items[itm].kscale);
  const int M = items[itm].M, N = items[itm].N, K = items[itm].K;
  const long long lda = items[itm].lda, ldb = items[itm].ldb, ldc = items[itm].ldc;
  int ti, tj;
  if (flags & GEMM_LOWER_C) {
    const long long t = bx;
    int r = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((long long)(r + 1) * (r + 2) / 2 <= t) ++r;
    while ((long long)r * (r + 1) / 2 > t) --r;
    ti = r;
    tj = (int)(t - (long long)r * (r + 1) / 2);
  } else {
    const int tm = (M + TM - 1) / TM, tn = (N + TN - 1) / TN;
    if (flags & GEMM_A_LOWER) {
      // the last tile rows carry the longest k ranges: hand them out first
      ti = tm - 1 - (int)(bx / tn);
      tj = (int)(bx % tn);
    } else {
      constexpr int BAND = 8;
      const int band = (int)(bx / (BAND * tn));
      const int pos = (int)(bx - (long long)band * BAND * tn);
      const int rows = min(BAND, tm - band * BAND);
      ti = band * BAND + pos % rows;
      tj = pos / rows;
    }
  }
  const int i0 = ti * TM, j0 = tj * TN;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, nn = lane & 15;
  const int wm = wave >> 1, wn = wave & 1;
  int kmin = (flags & GEMM_B_LOWER) ? j0 : 0;
  const int kmax = (flags & GEMM_A_LOWER) ? min(K, i0 + TM) : K;
  kmin = (kmin / TK) * TK;

  vt ra[NV], rb[NVB];
  // KS: the scales of the k indices of ra (clamped loads, used in park())
  T rk[KS ? NV : 1][KS && !AK ? VEC : 1];
  auto load = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int v = tid + 256 * q;
      int row, kk;
      if (!AK) { row = v / (TK / VEC); kk = (v % (TK / VEC)) * VEC; }
      else { kk = v / (TM / VEC); row = (v % (TM / VEC)) * VEC; }
      const long long gi = i0 + row, gk = k0 + kk;
      if (KS) {
#pragma unroll
        for (int e = 0; e < (AK ? 1 : VEC); ++e)
          rk[KS ? q : 0][KS && !AK ? e : 0] = ksc[min(gk + e, (long long)K - 1)];
      }
      if (VECOK) {
        // nothing here may touch the loaded value (that would wait for the
        // load): elements outside the operand are zeroed in park()
        if (gi < M && gk < kmax)
          ra[q] = *(const g_t<const vt>*)(!AK ? A + gi * lda + gk : A + gk * lda + gi);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const long long ii = !AK ? gi : gi + e, kq = !AK ? gk + e : gk;
          ra[q][e] = (ii < M && kq < kmax) ? A[!AK ? ii * lda + kq : kq * lda + ii] : (T)0;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NVB; ++q) {
      const int v = tid + 256 * q;
      int col, kk;
      if (!BN) { kk = v / (TN / VEC); col = (v % (TN / VEC)) * VEC; }
      else { col = v / (TK / VEC); kk = (v % (TK / VEC)) * VEC; }
      const long long gj = j0 + col, gk = k0 + kk;
      if (VECOK) {
        if (gj < N && gk < kmax)
          rb[q] = *(const g_t<const vt>*)(!BN ? B + gk * ldb + gj : B + gj * ldb + gk);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const long long jj = !BN ? gj + e : gj, kq = !BN ? gk : gk + e;
          rb[q][e] = (jj < N && kq < kmax) ? B[!BN ? kq * ldb + jj : jj * ldb + kq] : (T)0;
        }
      }
    }
  };
  // store the chunk loaded for k0 into LDS buffer buf; with vector loads the
  // elements outside op(A) / op(B) (also those of a skipped load) become zero
  auto park = [&](int buf, int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int v = tid + 256 * q;
      if (!AK) {
        const int row = v / (TK / VEC), kk = (v % (TK / VEC)) * VEC;
        const bool rin = i0 + row < M;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const T w = KS ? ra[q][e] * rk[KS ? q : 0][KS ? e : 0] : ra[q][e];
          As[buf][kk + e][row] = (!VECOK || (rin && k0 + kk + e < kmax)) ? w : (T)0;
        }
      } else {
        const int kk = v / (TM / VEC), row = (v % (TM / VEC)) * VEC;
        const bool kin = k0 + kk < kmax;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const T w = KS ? ra[q][e] * rk[KS ? q : 0][0] : ra[q][e];
          As[buf][kk][row + e] = (!VECOK || (kin && i0 + row + e < M)) ? w : (T)0;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NVB; ++q) {
      const int v = tid + 256 * q;
      if (!BN) {
        const int kk = v / (TN / VEC), col = (v % (TN / VEC)) * VEC;
        const bool kin = k0 + kk < kmax;
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          Bs[buf][kk][col + e] = (!VECOK || (kin && j0 + col + e < N)) ? rb[q][e] : (T)0;
      } else {
        const int col = v / (TK / VEC), kk = (v % (TK / VEC)) * VEC;
        const bool cin = j0 + col < N;
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          Bs[buf][kk + e][col] = (!VECOK || (cin && k0 + kk + e < kmax)) ? rb[q][e] : (T)0;
      }
    }
  };

  V4 acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = V4{0, 0, 0, 0};

  // the fragments of k-step ks+1 are read from LDS while the MFMAs of ks run
  auto multiply = [&](int cur) __attribute__((always_inline)) {
    T av[2][FM], bv[2][FN];
    auto frag = [&](int ks, int f) __attribute__((always_inline)) {
#pragma unroll
      for (int mt = 0; mt < FM; ++mt) av[f][mt] = As[cur][4 * ks + g][wm * (TM / 2) + 16 * mt + nn];
#pragma unroll
      for (int nt = 0; nt < FN; ++nt) bv[f][nt] = Bs[cur][4 * ks + g][wn * (TN / 2) + 16 * nt + nn];
    };
    frag(0, 0);
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      if (ks + 1 < TK / 4) frag(ks + 1, (ks + 1) & 1);
#pragma unroll
      for (int mt = 0; mt < FM; ++mt)
#pragma unroll
        for (int nt = 0; nt < FN; ++nt)
          acc[mt][nt] = mfma16(av[ks & 1][mt], bv[ks & 1][nt], acc[mt][nt]);
    }
    // schedule: reads of step 0, then the next step's reads in the middle of
    // each step's MFMAs (while half of them are still to issue)
    __builtin_amdgcn_sched_group_barrier(0x100, (FM + FN) / 2, 0);
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      __builtin_amdgcn_sched_group_barrier(0x008, FM * FN / 2, 0);
      if (ks + 1 < TK / 4) __builtin_amdgcn_sched_group_barrier(0x100, (FM + FN) / 2, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, FM * FN / 2, 0);
    }
  };
  // CPRE: the C tile (beta != 0) is loaded now, from clamped indices, so that
  // its latency hides behind the k loop instead of following it
  T cpre[CPRE ? FM : 1][CPRE ? FN : 1][4];
  if (CPRE) {
#pragma unroll
    for (int mt = 0; mt < FM; ++mt)
#pragma unroll
      for (int nt = 0; nt < FN; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const long long gi = min((long long)i0 + wm * (TM / 2) + 16 * mt + acc_row<T>(g, i), (long long)M - 1);
          const long long gj = min((long long)j0 + wn * (TN / 2) + 16 * nt + nn, (long long)N - 1);
          cpre[mt][nt][i] = C[gi * ldc + gj];
        }
  }
  if (kmin < kmax) {
    load(kmin);
    park(0, kmin);
    __syncthreads();
    // the last chunk is peeled off, so that every pass through the loop
    // stores what it loaded and no load is outstanding at the loop head
    int cur = 0, k0 = kmin;
    for (; k0 + TK < kmax; k0 += TK, cur ^= 1) {
      load(k0 + TK);
      multiply(cur);
      park(cur ^ 1, k0 + TK);
      __syncthreads();
    }
    multiply(cur);
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
          if (CPRE) v += beta * cpre[CPRE ? mt : 0][CPRE ? nt : 0][i];
          else if (beta != (T)0) v += beta * C[gi * ldc + gj];
          C[gi * ldc + gj] = v;
        }
      }
}

#ifndef SLAB_GEMM128_TK
#define SLAB_GEMM128_TK 16   // k per chunk of the 128-wide tiles
#endif
#ifndef SLAB_GEMM_F64_TILE
#define SLAB_GEMM_F64_TILE 64   // FP64 block-product tile (64 or 128)
#endif
#ifndef SLAB_GEMM_F64_TK
#define SLAB_GEMM_F64_TK 16     // k per chunk of the 64-wide FP64 tiles (32 and 8: slower)
#endif
#ifndef SLAB_GEMM_CPRE_F64_TK
#define SLAB_GEMM_CPRE_F64_TK 16  // k per chunk of the FP64 factorization updates (32: slower)
#endif
#ifndef SLAB_GEMM_CPRE_TILE
#define SLAB_GEMM_CPRE_TILE 64    // tile of the factorization updates (C prefetched)
#endif
#ifndef SLAB_GEMM_F32_TK
#define SLAB_GEMM_F32_TK 32       // k per chunk of the 64-wide FP32 tiles
#endif
#ifndef SLAB_GEMM_CPRE_F32_TK
#define SLAB_GEMM_CPRE_F32_TK 32  // k per chunk of the FP32 factorization updates
#endif
#ifndef SLAB_GEMM_WIDE
#define SLAB_GEMM_WIDE 0   // 128 x 256 tiles for full-output FP32 products (measured
                                   // slower: 265 registers, one wave per SIMD)
#endif
// ks (scaled k of op(A)) exists for the two operand forms that use it: the
// updates op(A) = U^T (ak, !bn) and the factorization's trailing update
// (!ak, bn); plan_gemm checks the form.
template <typename T, int TILE, int TK, bool CPRE = false, int WNF = 1>
static void gemm_tile(bool ak, bool bn, bool vecok, bool ks, unsigned grid, const GemmItem* items,
                      const int* offs, int count, T alpha, T beta, int flags, hipStream_t st) {
#define SLAB_GEMM_CASE(AKV, BNV, KSV)                                                              \
  do {                                                                                             \
    if (vecok)                                                                                     \
      hipLaunchKernelGGL((k_gemm<T, TILE, TK, AKV, BNV, true, CPRE, WNF, KSV>), dim3(grid),       \
                         dim3(256), 0, st, items, offs, count, alpha, beta, flags);                \
    else                                                                                           \
      hipLaunchKernelGGL((k_gemm<T, TILE, TK, AKV, BNV, false, CPRE, WNF, KSV>), dim3(grid),      \
                         dim3(256), 0, st, items, offs, count, alpha, beta, flags);                \
  } while (0)
  if (ks) {
    if (ak && !bn) SLAB_GEMM_CASE(true, false, true);
    else SLAB_GEMM_CASE(false, true, true);
  } else if (!ak && !bn) SLAB_GEMM_CASE(false, false, false);
  else if (!ak && bn) SLAB_GEMM_CASE(false, true, false);
  else if (ak && !bn) SLAB_GEMM_CASE(true, false, false);
  else SLAB_GEMM_CASE(true, true, false);
#undef SLAB_GEMM_CASE
}

template <typename T>
void plan_gemm(Plan& plan, bool ak, bool bn, const std::vector<GemmItem>& items, T alpha, T beta,
               int flags, int force_tile) {
  if (items.empty()) return;
  // items with scaled k and items without go to launches of their own
  const bool ks = items[0].kscale != nullptr;
  for (const GemmItem& g : items)
    if ((g.kscale != nullptr) != ks) {
      std::vector<GemmItem> with, without;
      for (const GemmItem& h : items) (h.kscale ? with : without).push_back(h);
      plan_gemm<T>(plan, ak, bn, with, alpha, beta, flags, force_tile);
      plan_gemm<T>(plan, ak, bn, without, alpha, beta, flags, force_tile);
      return;
    }
  if (ks && !((ak && !bn) || (!ak && bn))) {  // a planner's mistake, not an input's
    std::fprintf(stderr, "slab: plan_gemm: scaled k only for op(A) = A^T with B, or A with B^T\n");
    std::abort();
  }
  // 128-wide tiles once there are enough of them for four per compute unit,
  // unless the caller forces a width (FP32 only)
  long long area = 0;
  bool vecok = true;
  const uintptr_t vec = 16;
  for (const GemmItem& g : items) {
    area += (long long)g.M * g.N;
    vecok = vecok && g.lda % (vec / sizeof(T)) == 0 && g.ldb % (vec / sizeof(T)) == 0 &&
            ((uintptr_t)g.A % vec) == 0 && ((uintptr_t)g.B % vec) == 0;
  }
  if (flags & GEMM_LOWER_C) area /= 2;
  int tile = (sizeof(T) == 4 && area >= 1024LL * 128 * 128) ? 128 : 64;
  const bool cpre = (flags & GEMM_C_PREFETCH) != 0;
  if (sizeof(T) == 4 && (force_tile == 64 || force_tile == 128)) tile = force_tile;
  if (sizeof(T) == 8) tile = SLAB_GEMM_F64_TILE;
  if (cpre) tile = sizeof(T) == 4 ? SLAB_GEMM_CPRE_TILE : 64;
  ++plan.launches[cpre ? LK_GEMM_CPRE : (tile == 128 ? LK_GEMM128 : LK_GEMM64)];
  // full-output products on 128-wide tiles take 128 x 256 tiles
  const int wnf = (SLAB_GEMM_WIDE && tile == 128 && !cpre && !(flags & GEMM_LOWER_C)) ? 2 : 1;
  std::vector<int> c;
  for (const GemmItem& g : items) {
    const long long tm = (g.M + tile - 1) / tile, tn = (g.N + tile * wnf - 1) / (tile * wnf);
    c.push_back((int)((flags & GEMM_LOWER_C) ? tm * (tm + 1) / 2 : tm * tn));
  }
  long long tot;
  const size_t oi = plan.add_vec(items), oo = plan.add_offsets(c, &tot);
  const int count = (int)items.size();
  const std::shared_ptr<Plan::Timer> tm = plan.timer;
  plan.step([=](const char* dev, hipStream_t st) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (tm) {
      SLAB_HIP_CHECK(hipEventCreate(&e0));
      SLAB_HIP_CHECK(hipEventCreate(&e1));
      tm->ev.push_back(e0);
      tm->ev.push_back(e1);
      SLAB_HIP_CHECK(hipEventRecord(e0, st));
    }
    if (cpre && tile == 128)
      gemm_tile<T, 128, SLAB_GEMM128_TK, true>(ak, bn, vecok, ks, (unsigned)tot,
                                               dev_at<GemmItem>(dev, oi), dev_at<int>(dev, oo),
                                               count, alpha, beta, flags, st);
    else if (cpre)
      gemm_tile<T, 64, (sizeof(T) == 8 ? SLAB_GEMM_CPRE_F64_TK : SLAB_GEMM_CPRE_F32_TK), true>(
          ak, bn, vecok, ks, (unsigned)tot, dev_at<GemmItem>(dev, oi), dev_at<int>(dev, oo), count,
          alpha, beta, flags, st);
    else if (tile == 128 && wnf == 2)
      gemm_tile<T, 128, SLAB_GEMM128_TK, false, 2>(ak, bn, vecok, ks, (unsigned)tot,
                                                  dev_at<GemmItem>(dev, oi), dev_at<int>(dev, oo),
                                                  count, alpha, beta, flags, st);
    else if (tile == 128)
      gemm_tile<T, 128, SLAB_GEMM128_TK>(ak, bn, vecok, ks, (unsigned)tot,
                                         dev_at<GemmItem>(dev, oi), dev_at<int>(dev, oo), count,
                                         alpha, beta, flags, st);
    else
      gemm_tile<T, 64, (sizeof(T) == 8 ? SLAB_GEMM_F64_TK : SLAB_GEMM_F32_TK)>(
          ak, bn, vecok, ks, (unsigned)tot, dev_at<GemmItem>(dev, oi), dev_at<int>(dev, oo), count,
          alpha, beta, flags, st);
    SLAB_LAUNCH_CHECK();
    if (tm) SLAB_HIP_CHECK(hipEventRecord(e1, st));
    return SLAB_OK;
  });
}
template void plan_gemm<float>(Plan&, bool, bool, const std::vector<GemmItem>&, float, float,
                              int, int);
template void plan_gemm<double>(Plan&, bool, bool, const std::vector<GemmItem>&, double, double,
                               int, int);

// ---------------------------------------------------------------------------
// Panel of the right-looking factorization of a pivot block S (n x n), grouped
// over independent pivot blocks (items), in two launches.
// k_panel_diag (one workgroup per item) inverts the Cholesky factor of the
// 64x64 diagonal block [k0, k0+nb): Gaussian elimination without pivoting on
// [S_kk | I], kept in one array (U on and above the diagonal, the unit lower
// L~^-1 below it), gives S_kk = L~ U with U = D L~^T, hence
// L_kk^-1 = D^-1/2 L~^-1.  Signed items (indef) take L_kk^-1 = |D|^-1/2 L~^-1
// and J_k = sign(D), so that S_kk = L_kk J_k L_kk^T.  The working matrix lives in registers (thread = row
// x 16-column quarter); each step eliminates two pivots and exchanges only the
// two pivot rows and columns through LDS, with one barrier per step.  L_kk^-1 overwrites the lower
// triangle of S_kk (L_kk itself is never needed again).
// k_panel then, on 16x16x4 MFMA tiles, either
//   * computes 64 rows of L below the block:       L_ik = S_ik L_kk^-T J_k, or
//   * advances 64 columns of the carried inverse:  X_k = L_kk^-1 X_k.
// ---------------------------------------------------------------------------
#ifndef PANEL_DIAG_THREADS
#define PANEL_DIAG_THREADS 512
#endif
template <typename T, int NT = PANEL_DIAG_THREADS>
__global__ __launch_bounds__(NT) void k_panel_diag(const FactorItem* __restrict__ items,
                                                    int count, int k0) {
  const int itm = blockIdx.x;
  g_t<T>* __restrict__ S = gp((T*)items[itm].S);
  g_t<int>* __restrict__ status = gp(items[itm].status);
  const int n = items[itm].n, blk = items[itm].blk, indef = items[itm].indef;
  if (k0 >= n) return;  // uniform: this item has no panel at k0
  __shared__ T rowbuf[2][2][64];  // the two pivot rows of a step
  __shared__ T colbuf[2][2][64];  // the two pivot columns of a step
  const int nb = min(64, n - k0);
  const int tid = threadIdx.x;
  // thread (row i, column group q) keeps CQ entries of the working matrix in
  // registers; rows and columns beyond nb are the identity (their pivots are
  // eliminated as no-ops)
  constexpr int NQ = NT / 64, CQ = 64 / NQ;  // column groups, columns per group
  const int i = tid & 63, q = tid >> 6;
  T a[CQ];
#pragma unroll
  for (int c = 0; c < CQ; ++c) {
    const int col = CQ * q + c;
    T v = (i == col) ? (T)1 : (T)0;
    if (i < nb && col < nb) v = S[(long long)(k0 + max(i, col)) * n + k0 + min(i, col)];
    a[c] = v;
  }
  if (i < 2) {
#pragma unroll
    for (int c = 0; c < CQ; ++c) rowbuf[0][i][CQ * q + c] = a[c];
  }
  if (q == 0) {
    colbuf[0][0][i] = a[0];
    colbuf[0][1][i] = a[1];
  }
  __syncthreads();
  // two pivots p, p+1 per step (one barrier): with the pivot block
  // M = [d0 e; e2 d11] (rows p, p+1 at columns p, p+1), a row i > p+1 takes
  // (h0, h1) = (a_ip, a_i,p+1) M^-1, i.e. both eliminations at once:
  //   a_i -= h0 a_p + h1 a_p+1,  a_ip = -h0,  a_i,p+1 = -h1;
  // row p+1 takes the first elimination only (g = e2 / d0):
  //   a_p+1 -= g a_p,  a_p+1,p = -g.
  // p = CQ pb + pp: the register index pp is a compile-time constant and the
  // owner of columns p, p+1 is the wave q == pb (uniform branches only)
  for (int pb = 0; pb < NQ; ++pb) {
#pragma unroll
    for (int pp = 0; pp < CQ; pp += 2) {
      const int p = CQ * pb + pp;
      if (p >= nb) break;
      const int buf = (p >> 1) & 1;
      const T d0 = rowbuf[buf][0][p], e = rowbuf[buf][0][p + 1];
      const T e2 = rowbuf[buf][1][p], d11 = rowbuf[buf][1][p + 1];
      const T ai0 = colbuf[buf][0][i], ai1 = colbuf[buf][1][i];
      T r0[CQ], r1[CQ];
#pragma unroll
      for (int c = 0; c < CQ; ++c) {
        r0[c] = rowbuf[buf][0][CQ * q + c];
        r1[c] = rowbuf[buf][1][CQ * q + c];
      }
      const T rdet = fast_recip(fma(d0, d11, -(e * e2)));
      const T h0 = fma(ai0, d11, -(ai1 * e2)) * rdet;
      const T h1 = fma(ai1, d0, -(ai0 * e)) * rdet;
      const T gg = e2 * fast_recip(d0);
      const bool below = i > p + 1, next = i == p + 1;
      const T t0 = below ? h0 : (next ? gg : (T)0);
      const T t1 = below ? h1 : (T)0;
#pragma unroll
      for (int c = 0; c < CQ; ++c) a[c] = fma(-t0, r0[c], fma(-t1, r1[c], a[c]));
      if (q == pb) {
        if (below) {
          a[pp] = -h0;
          a[pp + 1] = -h1;
        } else if (next) {
          a[pp] = -gg;
        }
      }
      if (p + 2 < nb) {  // publish the next two pivot rows and columns
        const int nr = i - (p + 2);
        if (nr >= 0 && nr < 2) {
#pragma unroll
          for (int c = 0; c < CQ; ++c) rowbuf[buf ^ 1][nr][CQ * q + c] = a[c];
        }
        if (pp < CQ - 2) {
          if (q == pb) {
            colbuf[buf ^ 1][0][i] = a[(pp + 2) % CQ];
            colbuf[buf ^ 1][1][i] = a[(pp + 3) % CQ];
          }
        } else {
          if (q == pb + 1) {
            colbuf[buf ^ 1][0][i] = a[0];
            colbuf[buf ^ 1][1][i] = a[1];
          }
        }
      }
      __syncthreads();
    }
  }
  // diagonal of U is D; L_kk^-1 = |D|^-1/2 L~^-1 (a signed item keeps the
  // signs of D in J, an unsigned one needs D > 0)
  if (q == i / CQ) {
    T d = (T)1;
#pragma unroll
    for (int c = 0; c < CQ; ++c)
      if (c == i % CQ) d = a[c];
    const bool bad = indef ? !(d != (T)0) : !(d > (T)0);
    if (i < nb && (bad || !isfinite((double)d))) {
      status[0] = 3;
      status[1] = blk;
    }
    colbuf[0][0][i] = (T)1 / sqrt(indef ? fabs(d) : d);
    if (indef && i < nb) gp((T*)items[itm].J)[k0 + i] = d < (T)0 ? (T)-1 : (T)1;
  }
  __syncthreads();
  if (i < nb) {
    const T rs = colbuf[0][0][i];
    g_t<T>* row = S + (long long)(k0 + i) * n + k0;
#pragma unroll
    for (int c = 0; c < CQ; ++c) {
      const int col = CQ * q + c;
      if (col <= i) row[col] = (col < i) ? a[c] * rs : rs;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_panel(const FactorItem* __restrict__ items,
                                               const int* __restrict__ offs, int count, int k0) {
  typedef typename acc4<T>::type V4;
  const int itm = group_item(offs, count, blockIdx.x);
  const int bx = blockIdx.x - offs[itm];
  g_t<T>* __restrict__ S = gp((T*)items[itm].S);
  g_t<T>* __restrict__ Lv = gp((T*)items[itm].Li);
  const int n = items[itm].n;
  const int nrow_wg = (n - k0 - min(64, n - k0) + 63) / 64;
  __shared__ T E[64][65];   // L_kk^-1 (from the lower triangle of S_kk)
  __shared__ T Bt[64][65];  // operand tile
  const int nb = min(64, n - k0);
  const int tid = threadIdx.x;
  const bool rows = bx < nrow_wg;
  const long long r0 = (long long)k0 + nb + (long long)bx * 64;  // rows case
  const long long c0 = (long long)(bx - nrow_wg) * 64;            // columns case
  const long long ncols = (long long)k0 + nb;
  // every load is issued before the first LDS store (unconditional, from
  // clamped indices; values outside the operands are zeroed when stored)
  T te[16], tb[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = tid + 256 * u, hi = e >> 6, lo = e & 63;
    te[u] = S[(long long)(k0 + min(hi, nb - 1)) * n + k0 + min(lo, nb - 1)];
    if (rows) tb[u] = S[min(r0 + hi, (long long)n - 1) * n + k0 + min(lo, nb - 1)];
    else tb[u] = Lv[(long long)(k0 + min(hi, nb - 1)) * n + min(c0 + lo, ncols - 1)];
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = tid + 256 * u, hi = e >> 6, lo = e & 63;
    E[hi][lo] = (hi < nb && lo <= hi) ? te[u] : (T)0;
    // rows case Bt[rr][t], columns case Bt[t][cc]; zero outside the operand
    const bool in = rows ? (r0 + hi < n && lo < nb) : (hi < nb && c0 + lo < ncols);
    Bt[hi][lo] = in ? tb[u] : (T)0;
  }
  __syncthreads();

  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, nn = lane & 15;
  const int wm = wave >> 1, wn = wave & 1;
  // signed item, rows case: L_ik = (S_ik L_kk^-T) J_k, column col times J[k0+col]
  T js[2] = {(T)1, (T)1};
  if (rows && items[itm].indef) {
    const g_t<const T>* J = gp((const T*)items[itm].J);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) js[nt] = J[k0 + min(wn * 32 + 16 * nt + nn, nb - 1)];
  }
  V4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = V4{0, 0, 0, 0};
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
          if (r0 + row < n && col < nb) S[(r0 + row) * n + k0 + col] = acc[mt][nt][i] * js[nt];
        } else {
          if (row < nb && c0 + col < ncols) Lv[(long long)(k0 + row) * n + c0 + col] = acc[mt][nt][i];
        }
      }
}

// ---------------------------------------------------------------------------
// The factorization advances in 128-column panels made of two 64-column
// sub-panels.  After the first sub-panel [k0, k0+64) this kernel applies its
// update to what the second sub-panel [k0+64, k0+128) needs:
//   trailing  S_ij -= L_i J_k L_j^T (rows i >= k0+64, columns j in [k0+64, k0+128);
//                                    J_k = I for an unsigned item)
//   carried   X_ic -= L_i X_k,c     (rows i in [k0+64, k0+128), columns c < k0+64)
// with L_i = S[i, k0:k0+64] (just computed by the panel) and X_k the panel's
// rows of the carried inverse.  The rest of both updates, for both sub-panels
// at once, is two 128-deep GEMMs (see plan_factor_blocks).  One launch covers
// both tile kinds; every workgroup issues all its loads (A, B and the C tile)
// before the first MFMA.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_rank64(const FactorItem* __restrict__ items,
                                                const int* __restrict__ offs, int count, int k0) {
  typedef typename acc4<T>::type V4;
  const int itm = group_item(offs, count, blockIdx.x);
  const int bx = blockIdx.x - offs[itm];
  g_t<T>* __restrict__ S = gp((T*)items[itm].S);
  g_t<T>* __restrict__ Lv = gp((T*)items[itm].Li);
  const int n = items[itm].n;
  const int nb = min(64, n - k0);
  const int ntrail = (n - k0 - nb + 63) / 64;  // row tiles of the one column tile
  __shared__ T As[64][65];  // As[row][k]
  __shared__ T Bs[64][65];  // Bs[col][k]
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, nn = lane & 15;
  const int wm = wave >> 1, wn = wave & 1;
  const long long base = (long long)k0 + nb;
  long long r0, c0;
  g_t<T>* C;
  bool trail = bx < ntrail;
  if (trail) {
    r0 = base + 64LL * bx;
    c0 = base;
    C = S;
  } else {
    r0 = base;
    c0 = 64LL * (bx - ntrail);
    C = Lv;
  }
  const long long cmax = trail ? n : base;
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
  // all operand loads are issued before the first LDS store, so that their
  // latencies overlap
  // A: L rows r0.., panel columns
  // B: trailing -> L rows c0.. (B(k, j) = L[j][k]); carried -> X_k rows (B(k, c) = X[k0+k][c])
  T ta[16], tb[16];
  // signed item, trailing tiles: A(row, k) times J[k0+k]; k = tid & 63 for
  // every element this thread stores
  T jk = (T)1;
  if (trail && items[itm].indef) jk = gp((const T*)items[itm].J)[k0 + min(tid & 63, nb - 1)];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = tid + 256 * u, hi = e >> 6, lo = e & 63;
    ta[u] = (r0 + hi < n && lo < nb) ? S[(r0 + hi) * n + k0 + lo] : (T)0;
    if (trail) tb[u] = (c0 + hi < n && lo < nb) ? S[(c0 + hi) * n + k0 + lo] : (T)0;
    else tb[u] = (hi < nb && c0 + lo < cmax) ? Lv[(long long)(k0 + hi) * n + c0 + lo] : (T)0;
  }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = tid + 256 * u, hi = e >> 6, lo = e & 63;
    As[hi][lo] = ta[u] * jk;
    if (trail) Bs[hi][lo] = tb[u];
    else Bs[lo][hi] = tb[u];
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
__global__ void k_identity(const FactorItem* __restrict__ items, const int* __restrict__ offs,
                           int count) {
  const int itm = group_item(offs, count, blockIdx.x);
  const long long nwg = offs[itm + 1] - offs[itm];
  g_t<T>* __restrict__ X = gp((T*)items[itm].Li);
  const int n = items[itm].n;
  const long long tot = (long long)n * n;
  for (long long e = (blockIdx.x - offs[itm]) * (long long)blockDim.x + threadIdx.x; e < tot;
       e += nwg * blockDim.x) {
    X[e] = (e / n == e % n) ? (T)1 : (T)0;
  }
}

// FP64 copy of a symmetric block stored in its lower triangle.
template <typename T>
__global__ void k_sym_to_f64(const FactorItem* __restrict__ items, const int* __restrict__ offs,
                             int count) {
  const int itm = group_item(offs, count, blockIdx.x);
  const long long nwg = offs[itm + 1] - offs[itm];
  const g_t<const T>* __restrict__ S = gp((const T*)items[itm].S);
  g_t<double>* __restrict__ out = gp(items[itm].S64);
  const int n = items[itm].n;
  const long long tot = (long long)n * n;
  for (long long e = (blockIdx.x - offs[itm]) * (long long)blockDim.x + threadIdx.x; e < tot;
       e += nwg * blockDim.x) {
    const long long i = e / n, k = e % n;
    out[e] = (double)(k <= i ? S[e] : S[k * n + i]);
  }
}

// Cholesky factorization with carried inverse of independent pivot blocks
// (items, any sizes): L^-1 into item.Li, breakdown of an item reported as
// status = {3, item.blk}.  Signed items (indef) factor S = L J L^T with the
// pivot signs J into item.J; their breakdown is a zero (or non-finite) pivot.
template <typename T>
void plan_factor_blocks(Plan& plan, std::vector<FactorItem> items) {
  if (items.empty()) return;
  std::sort(items.begin(), items.end(),
            [](const FactorItem& a, const FactorItem& b) { return a.n > b.n; });
  const size_t oi = plan.add_vec(items);
  const int count = (int)items.size();
  std::vector<int> c;
  long long tot;
  // FP64 copies (items without one get no workgroups), then identities
  for (const FactorItem& f : items)
    c.push_back(f.S64 ? (int)std::min<long long>(((long long)f.n * f.n + 255) / 256, 1024) : 0);
  const size_t oc = plan.add_offsets(c, &tot);
  if (tot > 0) {
    const long long t = tot;
    plan.step([=](const char* dev, hipStream_t st) {
      hipLaunchKernelGGL((k_sym_to_f64<T>), dim3((unsigned)t), dim3(256), 0, st,
                         dev_at<FactorItem>(dev, oi), dev_at<int>(dev, oc), count);
      SLAB_LAUNCH_CHECK();
      return SLAB_OK;
    });
  }
  c.clear();
  for (const FactorItem& f : items)
    c.push_back((int)std::min<long long>(((long long)f.n * f.n + 255) / 256, 1024));
  const size_t od = plan.add_offsets(c, &tot);
  {
    const long long t = tot;
    plan.step([=](const char* dev, hipStream_t st) {
      hipLaunchKernelGGL((k_identity<T>), dim3((unsigned)t), dim3(256), 0, st,
                         dev_at<FactorItem>(dev, oi), dev_at<int>(dev, od), count);
      SLAB_LAUNCH_CHECK();
      return SLAB_OK;
    });
  }
  // 128-column panels; at each step the items with n beyond the step form a
  // prefix (items are sorted by n).  The update GEMMs are not block products
  // of the elimination: they stay out of the plan's product timer.
  const std::shared_ptr<Plan::Timer> timer = plan.timer;
  plan.timer.reset();
  auto live_beyond = [&](int k) {
    int l = 0;
    while (l < count && items[l].n > k) ++l;
    return l;
  };
  auto panel = [&](int k0, int live) {
    std::vector<int> cp;
    for (int i = 0; i < live; ++i) {
      const int n = items[i].n, nb = std::min(64, n - k0), nrow = n - k0 - nb;
      cp.push_back((nrow + 63) / 64 + (k0 + nb + 63) / 64);
    }
    long long tp;
    const size_t op = plan.add_offsets(cp, &tp);
    plan.step([=](const char* dev, hipStream_t st) {
      hipLaunchKernelGGL((k_panel_diag<T>), dim3((unsigned)live), dim3(PANEL_DIAG_THREADS), 0, st,
                         dev_at<FactorItem>(dev, oi), live, k0);
      SLAB_LAUNCH_CHECK();
      hipLaunchKernelGGL((k_panel<T>), dim3((unsigned)tp), dim3(256), 0, st,
                         dev_at<FactorItem>(dev, oi), dev_at<int>(dev, op), live, k0);
      SLAB_LAUNCH_CHECK();
      return SLAB_OK;
    });
  };
  for (int K0 = 0; K0 < items[0].n; K0 += 128) {
    panel(K0, live_beyond(K0));
    const int live2 = live_beyond(K0 + 64);
    if (live2 == 0) continue;
    {
      std::vector<int> cr;
      for (int i = 0; i < live2; ++i) {
        const int n = items[i].n, base = K0 + 64;
        cr.push_back((n - base + 63) / 64 + (base + 63) / 64);
      }
      long long trk;
      const size_t orr = plan.add_offsets(cr, &trk);
      plan.step([=](const char* dev, hipStream_t st) {
        hipLaunchKernelGGL((k_rank64<T>), dim3((unsigned)trk), dim3(256), 0, st,
                           dev_at<FactorItem>(dev, oi), dev_at<int>(dev, orr), live2, K0);
        SLAB_LAUNCH_CHECK();
        return SLAB_OK;
      });
    }
    panel(K0 + 64, live2);
    // both sub-panels' updates of everything beyond the panel, 128 deep:
    //   S_22 -= L_21 L_21^T (lower tiles),  X_2c -= L_21 X_1c  (c < K0+128)
    const int live3 = live_beyond(K0 + 128);
    std::vector<GemmItem> tr, ca;
    for (int i = 0; i < live3; ++i) {
      const FactorItem& f = items[i];
      const long long n = f.n, K2 = K0 + 128;
      T* S = (T*)f.S;
      T* X = (T*)f.Li;
      GemmItem a;
      a.A = S + K2 * n + K0; a.B = S + K2 * n + K0; a.C = S + K2 * n + K2;
      a.M = a.N = (int)(n - K2); a.K = 128; a.lda = a.ldb = a.ldc = (int)n;
      a.kscale = f.indef ? (const T*)f.J + K0 : nullptr;   // S_22 -= L_21 J L_21^T
      tr.push_back(a);
      GemmItem c;
      c.A = S + K2 * n + K0; c.B = X + (long long)K0 * n; c.C = X + K2 * n;
      c.M = (int)(n - K2); c.N = (int)K2; c.K = 128; c.lda = c.ldb = c.ldc = (int)n;
      c.kscale = nullptr;
      ca.push_back(c);
    }
    plan_gemm<T>(plan, false, true, tr, (T)-1, (T)1, GEMM_LOWER_C | GEMM_C_PREFETCH);
    plan_gemm<T>(plan, false, false, ca, (T)-1, (T)1, GEMM_C_PREFETCH);
  }
  plan.timer = timer;
}

template <typename T>
void plan_stage2(Plan& plan, const std::vector<Stage2Prob>& probs, bool odd_even, int tile) {
  auto blk = [](const Stage2Prob& p, void* base, long long j) {
    return (void*)((T*)base + j * (long long)p.n * p.n);
  };
  auto sq = [](const void* A, const void* B, void* C, int n, const void* ks = nullptr) {
    GemmItem g;
    g.A = A; g.B = B; g.C = C; g.M = g.N = g.K = n; g.lda = g.ldb = g.ldc = n;
    g.kscale = ks;
    return g;
  };
  // pivot signs of block j (signed problems), or null
  auto sg = [](const Stage2Prob& p, long long j) -> const void* {
    return p.indef ? (const void*)((const T*)p.J + j * p.n) : nullptr;
  };
  int mmax = 0;
  for (const Stage2Prob& p : probs) mmax = std::max(mmax, p.m);
  if (!odd_even) {
    // Alg. 1 in block Cholesky form, all problems in lockstep over j:
    // S_j = T_jj - Z_{j-1}^T J_{j-1} Z_{j-1}, S_j = L_j J_j L_j^T, Z_j = L_j^-1 T_{j,j+1}
    // (J = I for an unsigned problem)
    for (int j = 0; j < mmax; ++j) {
      std::vector<GemmItem> upd, zi;
      std::vector<FactorItem> fi;
      for (const Stage2Prob& p : probs) {
        if (j >= p.m) continue;
        if (j > 0)
          upd.push_back(sq(blk(p, p.Z, j - 1), blk(p, p.Z, j - 1), blk(p, p.Td, j), p.n,
                           sg(p, j - 1)));
        FactorItem f;
        f.S = blk(p, p.Td, j); f.Li = blk(p, p.Linv, j);
        f.S64 = p.S64 ? p.S64 + (long long)j * p.n * p.n : nullptr;
        f.J = p.indef ? (void*)((T*)p.J + (long long)j * p.n) : nullptr;
        f.indef = p.indef;
        f.status = p.status; f.n = p.n; f.blk = j;
        fi.push_back(f);
        if (j < p.m - 1) zi.push_back(sq(blk(p, p.Linv, j), blk(p, p.To, j), blk(p, p.Z, j), p.n));
      }
      plan_gemm<T>(plan, true, false, upd, (T)-1, (T)1, GEMM_LOWER_C, tile);
      plan_factor_blocks<T>(plan, fi);
      plan_gemm<T>(plan, false, false, zi, (T)1, (T)0, GEMM_A_LOWER, tile);
    }
    return;
  }
  // Odd-even order.  At level l (stride s = 2^l) the interfaces still present
  // are a_p = (p+1)s - 1, p < k = floor(m/s); those at even positions,
  // e_q = (2q+1)s - 1, q < E = ceil(k/2), are eliminated together.  e_q has a
  // kept neighbour l = e_q - s when q >= 1 and r = e_q + s when q < floor(k/2).
  // With D_e = L J L^T:  U_e = L^-1 C_l^T (stored over D_e), V_e = L^-1 C_e (in Z),
  //   D_l -= U_e^T J U_e,  D_r -= V_e^T J V_e,  C_l = -U_e^T J V_e,
  // where C_x (in To) is the coupling of x to the next interface present
  // (J = I for an unsigned problem).
  for (long long s = 1; s <= mmax; s *= 2) {
    std::vector<FactorItem> fi;
    std::vector<GemmItem> gu, gv, gdl, gdr, gc;
    for (const Stage2Prob& p : probs) {
      const int k = (int)(p.m / s);
      if (k < 1) continue;
      const int E = (k + 1) / 2, NR = k / 2;
      for (int q = 0; q < E; ++q) {
        const long long e = (2 * q + 1) * s - 1;
        FactorItem f;
        f.S = blk(p, p.Td, e); f.Li = blk(p, p.Linv, e);
        f.S64 = p.S64 ? p.S64 + e * p.n * p.n : nullptr;
        f.J = p.indef ? (void*)((T*)p.J + e * p.n) : nullptr;
        f.indef = p.indef;
        f.status = p.status; f.n = p.n; f.blk = (int)e;
        fi.push_back(f);
        if (q >= 1) {
          gu.push_back(sq(blk(p, p.Linv, e), blk(p, p.To, e - s), blk(p, p.Td, e), p.n));
          gdl.push_back(sq(blk(p, p.Td, e), blk(p, p.Td, e), blk(p, p.Td, e - s), p.n, sg(p, e)));
        }
        if (q < NR) {
          gv.push_back(sq(blk(p, p.Linv, e), blk(p, p.To, e), blk(p, p.Z, e), p.n));
          gdr.push_back(sq(blk(p, p.Z, e), blk(p, p.Z, e), blk(p, p.Td, e + s), p.n, sg(p, e)));
        }
        if (q >= 1 && q < NR)
          gc.push_back(sq(blk(p, p.Td, e), blk(p, p.Z, e), blk(p, p.To, e - s), p.n, sg(p, e)));
      }
    }
    plan_factor_blocks<T>(plan, fi);
    plan_gemm<T>(plan, false, true, gu, (T)1, (T)0, GEMM_A_LOWER, tile);    // U_e = L^-1 C_l^T
    plan_gemm<T>(plan, false, false, gv, (T)1, (T)0, GEMM_A_LOWER, tile);   // V_e = L^-1 C_e
    plan_gemm<T>(plan, true, false, gdl, (T)-1, (T)1, GEMM_LOWER_C, tile);  // D_l -= U^T J U
    plan_gemm<T>(plan, true, false, gdr, (T)-1, (T)1, GEMM_LOWER_C, tile);  // D_r -= V^T J V
    plan_gemm<T>(plan, true, false, gc, (T)-1, (T)0, 0, tile);              // C_l = -U^T J V
  }
}
template void plan_stage2<float>(Plan&, const std::vector<Stage2Prob>&, bool, int);
template void plan_stage2<double>(Plan&, const std::vector<Stage2Prob>&, bool, int);

// ---------------------------------------------------------------------------
// Block-vector product for the sweeping solve (Alg. 2):
//   y = beta * xin + alpha * M x,  x and y hold nrhs columns of length n.
// 16 columns at a time on 16x16x4 MFMA tiles.  A workgroup owns 16 rows; its
// sixteen waves split k and are reduced through LDS, so no result crosses a
// workgroup (a device-scope fence would write back every L2 of the chip).
// Each lane loads 16 contiguous bytes of M and of x per step, which feed
// VEC consecutive MFMA k-steps (k permuted consistently in A and B).
// ---------------------------------------------------------------------------
// Block-vector products y = beta xin + alpha op(M) x (nrhs <= 16 columns per
// workgroup column group) of the reduced solve.  These stream n x n blocks
// from HBM once per product, so the kernel is laid out for bandwidth: a
// workgroup owns 64 output rows and walks k in chunks; each chunk of op(M)
// (64 rows x TK) is fetched with 16-byte loads along the block's contiguous
// dimension (k for M, i for M^T: 256-byte runs), parked in LDS, and consumed
// by 16x16x4 MFMA tiles (one per wave) while the next chunk is in flight.
// XS: x(k) is taken times items[].xscale[k] (pivot signs J of a signed
// factorization), loaded with the x chunk.
// ---------------------------------------------------------------------------
template <typename T, bool TR, bool LOWER, bool VECOK, bool XS = false>
__global__ __launch_bounds__(256) void k_bmv(const BmvItem* __restrict__ items,
                                            const int* __restrict__ offs, int count, T alpha,
                                            T beta, int nsplit) {
  typedef typename acc4<T>::type V4;
  constexpr int VEC = 16 / sizeof(T);
  constexpr int TM = 64;                      // output rows per workgroup
  constexpr int TK = 256 / sizeof(T);         // k per chunk: 64 (FP32), 32 (FP64)
  constexpr int NVA = TM * TK / VEC / 256;    // vectors of op(M) per thread and chunk
  static_assert(NVA * VEC * 256 == TM * TK && 16 * TK == VEC * 256, "bmv tile");
  typedef T vt __attribute__((ext_vector_type(VEC)));
  // op(M) chunk in LDS: [k][row] for M^T (loaded along rows), [row][k] for M
  // (loaded along k), so that both are parked with 16-byte stores; the MFMA A
  // fragments read either layout without bank conflicts
  constexpr int AS0 = TR ? TK : TM, AS1 = TR ? TM + 4 : TK + 4;
  __shared__ __attribute__((aligned(16))) T As[2][AS0][AS1];
  __shared__ T Bs[2][TK][16 + 4];
  const int itm = group_item(offs, count, blockIdx.x);
  if (item_done(items[itm].live)) return;
  const int bx = blockIdx.x - offs[itm];
  const int n = items[itm].n, nrhs = items[itm].nrhs;
  const int nrt = (n + TM - 1) / TM, ncg = (nrhs + 15) / 16;
  // a triangular op(M) pairs row tile p with row tile nrt-1-p in one
  // workgroup, so every workgroup walks nrt+1 chunks and the launch keeps its
  // concurrency to the end
  const int nrw = LOWER ? (nrt + 1) / 2 : nrt;
  const int rp = bx % nrw, cg = (bx / nrw) % ncg, sk = bx / (nrw * ncg);
  const g_t<const T>* __restrict__ M = gp((const T*)items[itm].M);
  const g_t<const T>* __restrict__ x = gp((const T*)items[itm].x) + (long long)cg * 16 * n;
  const g_t<const T>* __restrict__ xsc = gp((const T*)items[itm].xscale);
  const g_t<const T>* xin = gp((const T*)items[itm].xin);
  if (xin) xin += (long long)cg * 16 * n;
  g_t<T>* y = gp((T*)items[itm].y) + (long long)cg * 16 * n;
  const int nc = min(16, nrhs - 16 * cg);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, nn = lane & 15;
  for (int pass = 0; pass < (LOWER ? 2 : 1); ++pass) {
  const int rt = pass == 0 ? rp : nrt - 1 - rp;
  if (pass == 1) {
    if (rt == rp) break;  // the middle tile of an odd count (uniform)
    __syncthreads();      // the LDS buffers of the first tile are free again
  }
  const int row0 = rt * TM;
  // op(M)(i, k) is zero for k > i (M lower) or k < i (M^T of a lower M)
  int klo = 0, khi = n;
  if (LOWER) {
    if (!TR) khi = min(n, row0 + TM);
    else klo = (row0 / TK) * TK;
  }
  if (nsplit > 1) {  // this workgroup's share of the chunks of [klo, khi)
    const int per = ((khi - klo + TK - 1) / TK + nsplit - 1) / nsplit;
    const int lo2 = klo + sk * per * TK;
    khi = min(khi, lo2 + per * TK);
    klo = lo2;
  }
  // Chunks of op(M) and x are loaded D chunks ahead into a register ring.
  // Every load is unconditional, from indices clamped into the arrays (a load
  // skipped on some path would make the compiler wait for all outstanding
  // loads); values outside the operands are zeroed when parked in LDS, and the
  // chunk loop runs to a multiple of D (extra chunks are all zero).
  // (triangular operands: many row tiles walk only a few chunks, so the ring
  // is shallower; measured faster)
  constexpr int D = VECOK ? (LOWER ? 2 : 3) : 1;
  vt ra[D][NVA], rb[D], rs[XS ? D : 1];
  auto load = [&](int d, int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < NVA; ++q) {
      const int v = tid + 256 * q;
      int row, kk;
      if (!TR) { row = v / (TK / VEC); kk = (v % (TK / VEC)) * VEC; }
      else { kk = v / (TM / VEC); row = (v % (TM / VEC)) * VEC; }
      if (VECOK) {
        // n % VEC == 0 here: the clamped vector stays inside its row
        const long long gi = !TR ? min(row0 + row, n - 1) : min(row0 + row, n - VEC);
        const long long gk = !TR ? min(k0 + kk, n - VEC) : min(k0 + kk, n - 1);
        ra[d][q] = *(const g_t<const vt>*)(!TR ? M + gi * n + gk : M + gk * n + gi);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const long long ii = !TR ? row0 + row : row0 + row + e, kq = !TR ? k0 + kk + e : k0 + kk;
          ra[d][q][e] = (ii < n && kq < khi) ? M[!TR ? ii * n + kq : kq * n + ii] : (T)0;
        }
      }
    }
    {
      const int c = tid / (TK / VEC), kk = (tid % (TK / VEC)) * VEC;
      if (VECOK) {
        rb[d] = *(const g_t<const vt>*)(x + (long long)min(c, nc - 1) * n + min(k0 + kk, n - VEC));
        if (XS) rs[XS ? d : 0] = *(const g_t<const vt>*)(xsc + min(k0 + kk, n - VEC));
      } else {
        const long long gk = k0 + kk;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          rb[d][e] = (c < nc && gk + e < khi) ? x[(long long)c * n + gk + e] : (T)0;
          if (XS) rs[XS ? d : 0][e] = xsc[min(gk + e, (long long)n - 1)];
        }
      }
    }
  };
  auto park = [&](int d, int buf, int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < NVA; ++q) {
      const int v = tid + 256 * q;
      if (!TR) {
        const int row = v / (TK / VEC), kk = (v % (TK / VEC)) * VEC;
        const bool rin = row0 + row < n;
        vt w;
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          w[e] = VECOK ? keep_if(rin && k0 + kk + e < khi, ra[d][q][e]) : ra[d][q][e];
        *(vt*)&As[buf][row][kk] = w;
      } else {
        const int kk = v / (TM / VEC), row = (v % (TM / VEC)) * VEC;
        const bool kin = k0 + kk < khi;
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          As[buf][kk][row + e] = VECOK ? keep_if(kin && row0 + row + e < n, ra[d][q][e]) : ra[d][q][e];
      }
    }
    const int c = tid / (TK / VEC), kk = (tid % (TK / VEC)) * VEC;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const T xv = XS ? rb[d][e] * rs[XS ? d : 0][e] : rb[d][e];
      Bs[buf][kk + e][c] = VECOK ? keep_if(c < nc && k0 + kk + e < khi, xv) : xv;
    }
  };
  // two accumulators: the chunk's MFMAs form two interleaved dependency chains
  V4 acc2[2] = {V4{0, 0, 0, 0}, V4{0, 0, 0, 0}};
  if (klo < khi) {
    const int nsteps = ((khi - klo + TK - 1) / TK + D - 1) / D * D;
#pragma unroll
    for (int d = 0; d < D; ++d) load(d, klo + d * TK);
    // nothing from before the loop in flight at its head, so the compiler's
    // wait counts inside follow the loop's own load order
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    for (int c0 = 0; c0 < nsteps; c0 += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int ch = c0 + d, cur = ch & 1;
        park(d, cur, klo + ch * TK);
        load(d, klo + (ch + D) * TK);
        __syncthreads();
        // (chunks past the end are zero: their products add nothing)
#pragma unroll
        for (int ks = 0; ks < TK / 4; ++ks)
          acc2[ks & 1] = mfma16(TR ? As[cur][4 * ks + g][16 * wave + nn]
                                   : As[cur][16 * wave + nn][4 * ks + g],
                                Bs[cur][4 * ks + g][nn],
                                acc2[ks & 1]);
      }
    }
  }
  V4 acc;
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = acc2[0][i] + acc2[1][i];
  if (nsplit > 1) {  // partial result; k_bmv_sum adds the splits up
    g_t<T>* part = gp((T*)items[itm].part) + ((long long)sk * 16 * ncg + 16 * cg) * n;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = row0 + 16 * wave + acc_row<T>(g, i);
      if (r < n && nn < nc) part[(long long)nn * n + r] = alpha * acc[i];
    }
    continue;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = row0 + 16 * wave + acc_row<T>(g, i);
    if (r < n && nn < nc) {
      T v = alpha * acc[i];
      if (xin) v += beta * xin[(long long)nn * n + r];
      y[(long long)nn * n + r] = v;
    }
  }
  }
}

// y = beta xin + (sum of the nsplit partial products), column c of n at c*n.
template <typename T>
__global__ void k_bmv_sum(const BmvItem* __restrict__ items, const int* __restrict__ offs,
                          int count, T beta, int nsplit) {
  const int itm = group_item(offs, count, blockIdx.x);
  if (item_done(items[itm].live)) return;
  const long long nwg = offs[itm + 1] - offs[itm];
  const int n = items[itm].n, nrhs = items[itm].nrhs, ncg = (nrhs + 15) / 16;
  const g_t<const T>* __restrict__ part = gp((const T*)items[itm].part);
  const g_t<const T>* xin = gp((const T*)items[itm].xin);
  g_t<T>* y = gp((T*)items[itm].y);
  const long long tot = (long long)nrhs * n, stride = (long long)16 * ncg * n;
  for (long long e = (blockIdx.x - offs[itm]) * (long long)blockDim.x + threadIdx.x; e < tot;
       e += nwg * blockDim.x) {
    T v = xin ? beta * xin[e] : (T)0;
    for (int k = 0; k < nsplit; ++k) v += part[k * stride + e];
    y[e] = v;
  }
}

template <typename T>
void plan_gemv(Plan& plan, bool tr, bool lower, const std::vector<BmvItem>& items, T alpha,
               T beta) {
  if (items.empty()) return;
  // items with scaled x and items without go to launches of their own
  const bool xs = items[0].xscale != nullptr;
  for (const BmvItem& b : items)
    if ((b.xscale != nullptr) != xs) {
      std::vector<BmvItem> with, without;
      for (const BmvItem& c : items) (c.xscale ? with : without).push_back(c);
      plan_gemv<T>(plan, tr, lower, with, alpha, beta);
      plan_gemv<T>(plan, tr, lower, without, alpha, beta);
      return;
    }
  if (xs && !tr) {  // a planner's mistake, not an input's
    std::fprintf(stderr, "slab: plan_gemv: scaled x only for products with M^T\n");
    std::abort();
  }
  bool vecok = true, can_split = true;
  const uintptr_t al = 16;
  long long base = 0;
  // (a triangular operand pairs two row tiles per workgroup, see k_bmv)
  auto row_wgs = [&](int n) { return lower ? ((n + 63) / 64 + 1) / 2 : (n + 63) / 64; };
  for (const BmvItem& b : items) {
    base += row_wgs(b.n) * ((b.nrhs + 15) / 16);
    vecok = vecok && b.n % (int)(16 / sizeof(T)) == 0 && ((uintptr_t)b.M % al) == 0 &&
            ((uintptr_t)b.x % al) == 0 && ((uintptr_t)b.xscale % al) == 0;
    can_split = can_split && b.part != nullptr && b.n >= 512;
  }
  // a launch of few workgroups is bound by one workgroup's walk over k: split
  // k so that the chip holds about 512 workgroups, then add the partial sums
  int nsplit = 1;
  if (can_split)
    while (nsplit < BMV_SPLIT_MAX && base * nsplit * 2 <= 512) nsplit *= 2;
  ++plan.launches[nsplit > 1 ? LK_BMV_SPLIT : LK_BMV];
  std::vector<int> c;
  for (const BmvItem& b : items) c.push_back(row_wgs(b.n) * ((b.nrhs + 15) / 16) * nsplit);
  long long tot;
  const size_t oi = plan.add_vec(items), oo = plan.add_offsets(c, &tot);
  const int count = (int)items.size();
  size_t os = 0;
  long long ts = 0;
  if (nsplit > 1) {
    std::vector<int> cs;
    for (const BmvItem& b : items)
      cs.push_back((int)std::min<long long>(((long long)b.nrhs * b.n + 255) / 256, 256));
    os = plan.add_offsets(cs, &ts);
  }
  plan.step([=](const char* dev, hipStream_t st) {
    const BmvItem* it = dev_at<BmvItem>(dev, oi);
    const int* of = dev_at<int>(dev, oo);
#define SLAB_BMV_CASE(TRV, LOV, XSV)                                                            \
  do {                                                                                          \
    if (vecok)                                                                                  \
      hipLaunchKernelGGL((k_bmv<T, TRV, LOV, true, XSV>), dim3((unsigned)tot), dim3(256), 0,    \
                         st, it, of, count, alpha, beta, nsplit);                               \
    else                                                                                        \
      hipLaunchKernelGGL((k_bmv<T, TRV, LOV, false, XSV>), dim3((unsigned)tot), dim3(256), 0,   \
                         st, it, of, count, alpha, beta, nsplit);                               \
  } while (0)
    if (xs) {
      if (lower) SLAB_BMV_CASE(true, true, true);
      else SLAB_BMV_CASE(true, false, true);
    } else if (!tr && !lower) SLAB_BMV_CASE(false, false, false);
    else if (!tr && lower) SLAB_BMV_CASE(false, true, false);
    else if (tr && !lower) SLAB_BMV_CASE(true, false, false);
    else SLAB_BMV_CASE(true, true, false);
#undef SLAB_BMV_CASE
    SLAB_LAUNCH_CHECK();
    if (nsplit > 1) {
      hipLaunchKernelGGL((k_bmv_sum<T>), dim3((unsigned)ts), dim3(256), 0, st, it,
                         dev_at<int>(dev, os), count, beta, nsplit);
      SLAB_LAUNCH_CHECK();
    }
    return SLAB_OK;
  });
}

template void plan_gemv<float>(Plan&, bool, bool, const std::vector<BmvItem>&, float, float);
template void plan_gemv<double>(Plan&, bool, bool, const std::vector<BmvItem>&, double, double);

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
