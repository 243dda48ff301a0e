// Stage one of the slab solver: edge weights, index maps, slab factorizations
// (two-sided block recursion), the boundary columns of each slab inverse, the
// Schur-complement propagation on MFMA, and assembly of the reduced blocks T.
//
// Paper: Sec. 2 (discretization, clustering), Sec. 3.1 (Schur complements,
// eqs. (dell1)-(T35)), Alg. 3 (first loop: factor every slab interior).
#include "launch.h"

namespace slab {

// The four status words of every problem cleared (a kernel rather than a
// memset, so that a captured graph holds no memset node).
__global__ void k_status_clear(const ProbDev* __restrict__ P, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 4 * count) gp(P[i >> 2].status)[i & 3] = 0;
}

// ---------------------------------------------------------------------------
// Coefficient field: copy (or exponentiate theta) and check positivity.
// status[2] is set to 1 when some kappa is not > 0 or not finite (status[0..1]
// record a breakdown of the factorization).
// Grouped: each problem owns a fixed number of workgroups and strides over
// its (n1+2)(n2+2) nodes with them.
// ---------------------------------------------------------------------------
__global__ void k_coef(const ProbDev* __restrict__ P, const int* __restrict__ offs, int count) {
  const int it = group_item(offs, count, blockIdx.x);
  const ProbDev& d = P[it];
  const long long nwg = offs[it + 1] - offs[it];
  const long long tot = (long long)(d.n1 + 2) * (d.n2 + 2);
  const g_t<const double>* coef = gp(d.coef);
  g_t<double>* kappa = gp(d.kappa);
  bool bad = false;
  for (long long i = (blockIdx.x - offs[it]) * (long long)blockDim.x + threadIdx.x; i < tot;
       i += nwg * blockDim.x) {
    const double v = coef[i];
    const double k = d.is_log ? exp(v) : v;
    if (!(k > 0.0) || !isfinite(k)) bad = true;
    kappa[i] = k;
  }
  if (bad) gp(d.status)[2] = 1;
}

// Diagonal term of the operator: the caller's field copied (status[2] = 1 for
// a value that is not finite), or the single zero a problem without one
// points at.
__global__ void k_shift(const ProbDev* __restrict__ P, const int* __restrict__ offs, int count) {
  const int it = group_item(offs, count, blockIdx.x);
  const ProbDev& d = P[it];
  const long long nwg = offs[it + 1] - offs[it];
  const long long tot = d.shift_src ? (long long)d.n1 * d.n2 : 1;
  g_t<double>* sh = gp(d.shift);
  bool bad = false;
  for (long long i = (blockIdx.x - offs[it]) * (long long)blockDim.x + threadIdx.x; i < tot;
       i += nwg * blockDim.x) {
    const double v = d.shift_src ? gp(d.shift_src)[i] : 0.0;
    if (!isfinite(v)) bad = true;
    sh[i] = v;
  }
  if (bad) gp(d.status)[2] = 1;
}

// Edge weights w = (kappa_p + kappa_q) / (2 h^2) of the 5-point stencil.
// wh[c*n2 + r], c = 0..n1: edge (c-1, r)-(c, r); wv[c*(n2+1) + r], r = 0..n2:
// edge (c, r-1)-(c, r).  Columns/rows -1 and n1/n2 are the Dirichlet ring.
__global__ void k_weights(const ProbDev* __restrict__ P, const int* __restrict__ offs, int count) {
  const int it = group_item(offs, count, blockIdx.x);
  const ProbDev& d = P[it];
  const long long nwg = offs[it + 1] - offs[it];
  const int n1 = d.n1, n2 = d.n2;
  const long long nh = (long long)(n1 + 1) * n2;
  const long long nv = (long long)n1 * (n2 + 1);
  const long long ld = n2 + 2;
  const double hh = d.h * d.h;
  const g_t<const double>* kappa = gp((const double*)d.kappa);
  g_t<double>* wh = gp(d.wh);
  g_t<double>* wv = gp(d.wv);
  for (long long i = (blockIdx.x - offs[it]) * (long long)blockDim.x + threadIdx.x; i < nh + nv;
       i += nwg * blockDim.x) {
    if (i < nh) {
      long long c = i / n2, r = i % n2;  // edge between ring-padded columns c and c+1
      wh[i] = 0.5 * (kappa[c * ld + r + 1] + kappa[(c + 1) * ld + r + 1]) / hh;
    } else {
      long long j = i - nh;
      long long c = j / (n2 + 1), r = j % (n2 + 1);
      wv[j] = 0.5 * (kappa[(c + 1) * ld + r] + kappa[(c + 1) * ld + r + 1]) / hh;
    }
  }
}

// ---------------------------------------------------------------------------
// Index maps of the clustering (Sec. 2.2).
// ---------------------------------------------------------------------------
__global__ void k_maps(int n1, int n2, int b, int32_t* col_kind, int32_t* slab_of_col,
                       int32_t* local_of_col, int64_t* perm_even, int64_t* perm_odd) {
  const int m = n1 / (b + 1);
  const long long ne = (long long)m * n2 * b;
  const long long no = (long long)m * n2;
  const long long tot = n1 + ne + no;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < tot;
       i += (long long)gridDim.x * blockDim.x) {
    if (i < n1) {
      int c = (int)i;
      if (col_kind) col_kind[c] = (c % (b + 1) == b) ? 1 : 0;
      if (slab_of_col) slab_of_col[c] = c / (b + 1);
      if (local_of_col) local_of_col[c] = c % (b + 1);
    } else if (i < n1 + ne) {
      long long e = i - n1;
      long long s = e / ((long long)n2 * b);
      long long rem = e % ((long long)n2 * b);
      long long r = rem / b, k = rem % b;
      if (perm_even) perm_even[e] = (s * (b + 1) + k) * n2 + r;
    } else {
      long long o = i - n1 - ne;
      long long j = o / n2, r = o % n2;
      if (perm_odd) perm_odd[o] = (j * (b + 1) + b) * n2 + r;
    }
  }
}

int launch_maps(int n1, int n2, int b, int32_t* ck, int32_t* sc, int32_t* lc, int64_t* pe,
                int64_t* po, hipStream_t st) {
  const int m = n1 / (b + 1);
  long long tot = n1 + (long long)m * n2 * b + (long long)m * n2;
  unsigned grid = (unsigned)std::min<long long>((tot + 255) / 256, 65536);
  hipLaunchKernelGGL(k_maps, dim3(grid), dim3(256), 0, st, n1, n2, b, ck, sc, lc, pe, po);
  SLAB_LAUNCH_CHECK();
  return SLAB_OK;
}

// ---------------------------------------------------------------------------
// Row `lane` of the slab block D_r (b x b, tridiagonal: one grid row of a slab
// interior, b-fastest local order), padded to BP with identity rows.
// ---------------------------------------------------------------------------
template <typename T, int BP>
__device__ __forceinline__ void build_D_row(T (&a)[BP], const g_t<const double>* __restrict__ wh,
                                            const g_t<const double>* __restrict__ wv,
                                            const g_t<const double>* __restrict__ sh,
                                            long long ss, int n2, int b, int c0, int r, int lane) {
  const bool act = lane < b;
  double d = 1.0, wl = 0.0, wr = 0.0;
  if (act) {
    const long long c = c0 + lane;
    d = wh[c * n2 + r] + wh[(c + 1) * n2 + r] + wv[c * (n2 + 1) + r] + wv[c * (n2 + 1) + r + 1] +
        sh[(c * n2 + r) * ss];
    if (lane > 0) wl = wh[c * n2 + r];
    if (lane < b - 1) wr = wh[(c + 1) * n2 + r];
  }
#pragma unroll
  for (int k = 0; k < BP; ++k) {
    double v = (k == lane) ? d : ((k == lane - 1) ? -wl : ((k == lane + 1) ? -wr : 0.0));
    a[k] = (T)v;
  }
}

// ---------------------------------------------------------------------------
// Slab factorization (Alg. 3 first loop), block-tridiagonal form of the banded
// slab matrix A_{2s,2s}: diagonal blocks D_r, couplings A_{r,r-1} = -W_r with
// W_r = diag of the vertical edge weights between grid rows r-1 and r.
//   top-down  (dir 0):  Dl_0 = D_0,        Dl_r = D_r - W_r Gl_{r-1} W_r,    Gl_r = Dl_r^-1
//   bottom-up (dir 1):  Dr_{n-1} = D_{n-1}, Dr_r = D_r - W_{r+1} Gr_{r+1} W_{r+1}
// Stored: Gl_r row-major (block solves), Hr_r = Gr_r W_r in fragment-major
// order (Schur propagation).  One four-wave workgroup per (slab, direction):
// thread = (row i, column group q) holds BP/R entries of row i, R = 256/BP
// threads per row.  Each block is inverted in place by the symmetric sweep
// operator taken two pivots at a time: the 2x2 pivot block is inverted in
// registers by every thread (adjugate over the determinant), and since the
// swept matrix stays symmetric, the pivot columns every row needs are the
// pivot rows published through LDS: one barrier per pivot pair, the same
// instructions for the pivot rows and the others (selects pick the scaled
// pivot rows).  Every thread loads the edge weights of its own row and columns
// one row step ahead, so no load latency sits on the row-to-row chain.
// ---------------------------------------------------------------------------
//
// Segments.  The recursion forgets where it started: a change of Gl_{r-1}
// reaches Gl_r through Gl_r W_r (.) W_r Gl_r, which shrinks it by about
// exp(-2 pi / (b+1)) per row for this operator (the decay of the slowest
// mode across a strip of b+1 columns).  So the n2 row steps of a chain are
// cut into segments that run in parallel: a segment after the first starts
// fwarm steps before its first row from a zero inverse (the recursion of a
// slab cut off there), and stores only its own rows.  Its warm-up's last
// block goes to fchk; k_factor_check compares it with the block the previous
// segment stored for that row, and a chain whose warm-up has not converged
// there is recomputed in one piece by the redo launch (redo = 1: one
// workgroup per chain, only for marked chains).
// ---------------------------------------------------------------------------
// Threads per slab-recursion workgroup: 256 by default; 128 (two waves) for
// blocks of up to 32 rows when a launch has at least four workgroups per
// compute unit to interleave (measured faster there: 6.2 against 7.1 ms at
// 2048 x 4096, b = 31, and slower with fewer workgroups); 64-row blocks keep
// 256 (fewer would spill).
#define SLAB_FACTOR_THREADS 256
constexpr int SLAB_FACTOR_MANY = 1024;   // workgroups of a launch that take 128 threads
#ifndef SLAB_FACTOR_PB
#define SLAB_FACTOR_PB 2
#endif
template <typename T, int BP, int NT = SLAB_FACTOR_THREADS, int PB = SLAB_FACTOR_PB>
__global__ __launch_bounds__(NT) void k_slab_factor(const ProbDev* __restrict__ P,
                                                    const int* __restrict__ offs, int count,
                                                    int redo) {
  constexpr int R = NT / BP;   // lanes per row
  constexpr int C = BP / R;    // columns per lane
  constexpr int D = 1;         // weight prefetch depth (row steps): one row step
                               // (an elimination) outlasts a memory latency
  const int it = group_item(offs, count, blockIdx.x);
  const int bx = blockIdx.x - offs[it];
  const g_t<const double>* __restrict__ wh = gp((const double*)P[it].wh);
  const g_t<const double>* __restrict__ wv = gp((const double*)P[it].wv);
  const int n2 = P[it].n2, b = P[it].b;
  g_t<T>* __restrict__ Gl = gp((T*)P[it].Gl);
  g_t<T>* __restrict__ Hsw = gp((T*)P[it].Hsw);
  g_t<int>* __restrict__ status = gp(P[it].status);
  const int nseg = redo ? 1 : P[it].fnseg;
  const int seg = bx % nseg, sd = bx / nseg;
  const int s = sd >> 1, dir = sd & 1;
  g_t<int>* __restrict__ fredo = gp(P[it].fredo);
  if (redo && fredo[sd] == 0) return;   // uniform: this chain's segments agreed
  if (!redo && seg == 0 && threadIdx.x == 0) fredo[sd] = 0;
  // steps [t_lo, t_hi) are stored; the chain starts at t_start
  const int t_lo = seg * P[it].fseg;
  const int t_hi = seg == nseg - 1 ? n2 : t_lo + P[it].fseg;
  const int t_start = seg == 0 ? 0 : max(0, t_lo - P[it].fwarm);
  g_t<T>* __restrict__ fchk =
      seg > 0 ? gp((T*)P[it].fchk) + ((size_t)sd * nseg + seg) * BP * BP : nullptr;
  const int lane = threadIdx.x;
  const int i = lane % BP, q = lane / BP;
  const int k0 = q * C;                    // first column of this lane
  const bool act = i < b;
  const long long c = (long long)s * (b + 1) + (act ? i : 0);
  static_assert((BP / PB) % 2 == 0 && BP % PB == 0, "an even number of pivot blocks");
  // rows of the current pivot block; double-buffered, and with an even number
  // of blocks per row step the next step's first block never overwrites a
  // buffer still being read
  __shared__ T colbuf[2][PB][BP];
  T g[C], a[C];
#pragma unroll
  for (int j = 0; j < C; ++j) g[j] = (T)0;
  // raw edge weights of row r: wh left/right of the node, wv below/above; and
  // wv below/above the nodes of this lane's columns k0 .. k0+C-1
  double rl[D], rr[D], rd[D], ru[D], rs[D], cd[D][C], cu[D][C];
  const g_t<const double>* __restrict__ sh = gp((const double*)P[it].shift);
  const long long ss = P[it].shift_stride;
  // with a diagonal term the slab blocks may be indefinite: nonzero pivots
  // of either sign are taken (no pivoting), else they must be positive
  const bool signed_piv = ss != 0;
  // unconditional loads from clamped rows (a load skipped on some path makes
  // the compiler wait for every outstanding load); masked where used
  auto load = [&](int d, int t) __attribute__((always_inline)) {
    const int tc = min(t, n2 - 1);
    const int r = dir == 0 ? tc : n2 - 1 - tc;
    rl[d] = wh[c * n2 + r];
    rr[d] = wh[(c + 1) * n2 + r];
    rd[d] = wv[c * (n2 + 1) + r];
    ru[d] = wv[c * (n2 + 1) + r + 1];
    rs[d] = sh[(c * n2 + r) * ss];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const long long ck = (long long)s * (b + 1) + min(k0 + j, b - 1);
      cd[d][j] = wv[ck * (n2 + 1) + r];
      cu[d][j] = wv[ck * (n2 + 1) + r + 1];
    }
  };
#pragma unroll
  for (int d = 0; d < D; ++d) load(d, t_start + d);
  bool ok = true;
  for (int t0 = t_start; t0 < t_hi; t0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int t = t0 + d;
      if (t < t_hi) {  // uniform
        const int r = dir == 0 ? t : n2 - 1 - t;
        const double whl = rl[d], whr = rr[d], wvd = rd[d], wvu = ru[d], csh = rs[d];
        // W of the coupling to the previous row step and W_r, at this lane's columns
        T wk[C], wup[C];
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const bool ak = k0 + j < b;
          wk[j] = (ak && t > 0) ? (T)(dir == 0 ? cd[d][j] : cu[d][j]) : (T)0;
          wup[j] = ak ? (T)cd[d][j] : (T)0;
        }
        load(d, t + D);
        const T dd = act ? (T)(whl + whr + wvd + wvu + csh) : (T)1;
        const T wl = (act && i > 0) ? (T)whl : (T)0;
        const T wr = (act && i < b - 1) ? (T)whr : (T)0;
        const T wc = (act && t > 0) ? (T)(dir == 0 ? wvd : wvu) : (T)0;
        // row i of D_r - W G W (columns k0 .. k0+C-1)
#pragma unroll
        for (int j = 0; j < C; ++j) {
          const int k = k0 + j;
          const T dk = (k == i) ? dd : ((k == i - 1) ? -wl : ((k == i + 1) ? -wr : (T)0));
          a[j] = dk - wc * g[j] * wk[j];
        }
        if (i < PB) {
#pragma unroll
          for (int j = 0; j < C; ++j) colbuf[0][i][k0 + j] = a[j];
        }
        group_sync<NT>();
        // block sweeps over pivots p0 .. p0+PB-1 (rows published in colbuf)
#pragma unroll
        for (int p0 = 0; p0 < BP; p0 += PB) {
          const int buf = (p0 / PB) & 1;
          // all LDS reads first, unconditionally (no read inside a divergent branch)
          T h[PB][PB], mpk[PB][C], mip[PB];
#pragma unroll
          for (int u = 0; u < PB; ++u) {
#pragma unroll
            for (int v = 0; v < PB; ++v) h[u][v] = colbuf[buf][u][p0 + v];
#pragma unroll
            for (int j = 0; j < C; ++j) mpk[u][j] = colbuf[buf][u][k0 + j];
            mip[u] = colbuf[buf][u][i];  // = entry (i, p0+u) by symmetry
          }
          // h := -(pivot block)^{-1}: the sweep over its own PB pivots, in
          // registers (2 x 2: adjugate over the determinant; the leading
          // entry and the determinant positive <=> both pivots positive)
          if constexpr (PB == 2) {
            const T h00 = h[0][0], h01 = h[0][1], h11 = h[1][1];
            const T det = fma(h00, h11, -(h01 * h01));
            ok = ok && (signed_piv ? det != (T)0 : (h00 > (T)0) && (det > (T)0)) &&
                 isfinite((double)det);
            const T ninv = -fast_recip(det);
            h[0][0] = h11 * ninv;
            h[1][1] = h00 * ninv;
            h[0][1] = h[1][0] = -h01 * ninv;
          } else {
#pragma unroll
          for (int pp = 0; pp < PB; ++pp) {
            const T dp = h[pp][pp];
            ok = ok && (signed_piv ? dp != (T)0 : dp > (T)0) && isfinite((double)dp);
            const T inv = fast_recip(dp);
#pragma unroll
            for (int u = 0; u < PB; ++u) {
              if (u == pp) continue;
              const T f = h[u][pp] * inv;
#pragma unroll
              for (int v = 0; v < PB; ++v)
                if (v != pp) h[u][v] = fma(-f, h[pp][v], h[u][v]);
              h[u][pp] = f;
            }
#pragma unroll
            for (int v = 0; v < PB; ++v)
              if (v != pp) h[pp][v] *= inv;
            h[pp][pp] = -inv;
          }
          }
          // row multipliers: other rows -c = (row i, pivot columns) * h; a pivot
          // row pr takes row pr of h, and keeps nothing of its old values.  In
          // both cases the new entries in the pivot columns are -t.
          const int pr = i - p0;
          const bool piv = pr >= 0 && pr < PB;
          T tv[PB];
#pragma unroll
          for (int v = 0; v < PB; ++v) {
            T cv = (T)0;
#pragma unroll
            for (int u = 0; u < PB; ++u) cv = fma(mip[u], h[u][v], cv);
            T hv = h[0][v];
#pragma unroll
            for (int u = 1; u < PB; ++u) hv = (pr == u) ? h[u][v] : hv;
            tv[v] = piv ? -hv : cv;
          }
          const T keep = piv ? (T)0 : (T)1;
#pragma unroll
          for (int j = 0; j < C; ++j) {
            T acc = a[j] * keep;
#pragma unroll
            for (int v = 0; v < PB; ++v) acc = fma(tv[v], mpk[v][j], acc);
            a[j] = acc;
          }
#pragma unroll
          for (int v = 0; v < PB; ++v)
            if (q == (p0 + v) / C) a[(p0 + v) % C] = -tv[v];
          if (p0 + PB < BP) {
            const int nr = i - (p0 + PB);
            if (nr >= 0 && nr < PB) {
#pragma unroll
              for (int j = 0; j < C; ++j) colbuf[buf ^ 1][nr][k0 + j] = a[j];
            }
            group_sync<NT>();
          }
        }
#pragma unroll
        for (int j = 0; j < C; ++j) g[j] = -a[j];
        // own rows go to Gl / Hsw; the warm-up's last row to the check block
        if (t >= t_lo || t == t_lo - 1) {  // uniform
          const bool own = t >= t_lo;
          if (dir == 0) {
            g_t<T>* dst = own ? Gl + (((size_t)s * n2 + r) * BP + i) * BP + k0
                              : fchk + (size_t)i * BP + k0;
#pragma unroll
            for (int j = 0; j < C; ++j) dst[j] = g[j];
          } else {
            g_t<T>* dst = own ? Hsw + ((size_t)s * n2 + r) * BP * BP : fchk;
#pragma unroll
            for (int j = 0; j < C; ++j) dst[swz_index<T>(i, k0 + j, BP)] = g[j] * wup[j];
          }
        }
      }
    }
  }
  if (!ok && lane == 0) { status[0] = 2; status[1] = s; }
}

// Warm-up check of the segmented slab recursion: for every segment after the
// first, the block its warm-up reached at the row before its first one is
// compared with the block the previous segment stored for that row; a
// relative difference above tol (or a non-finite one) marks the chain for the
// redo launch.  One workgroup per (slab, direction, segment > 0).
template <typename T, int BP>
__global__ __launch_bounds__(256) void k_factor_check(const ProbDev* __restrict__ P,
                                                      const int* __restrict__ offs, int count,
                                                      double tol) {
  __shared__ double red[2][256];
  const int it = group_item(offs, count, blockIdx.x);
  const int bx = blockIdx.x - offs[it];
  const int nseg = P[it].fnseg, n2 = P[it].n2;
  const int seg = 1 + bx % (nseg - 1), sd = bx / (nseg - 1);
  const int s = sd >> 1, dir = sd & 1;
  const int t = seg * P[it].fseg - 1;
  const int r = dir == 0 ? t : n2 - 1 - t;
  const g_t<const T>* ref = dir == 0 ? gp((const T*)P[it].Gl) + ((size_t)s * n2 + r) * BP * BP
                                     : gp((const T*)P[it].Hsw) + ((size_t)s * n2 + r) * BP * BP;
  const g_t<const T>* chk = gp((const T*)P[it].fchk) + ((size_t)sd * nseg + seg) * BP * BP;
  double dmax = 0.0, rmax = 0.0;
  for (int e = threadIdx.x; e < BP * BP; e += 256) {
    const double a = (double)ref[e], c = (double)chk[e];
    const double d = fabs(a - c);
    dmax = (d > dmax || d != d) ? d : dmax;   // a NaN difference is kept
    rmax = fmax(rmax, fabs(a));
  }
  red[0][threadIdx.x] = dmax;
  red[1][threadIdx.x] = rmax;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double x = red[0][threadIdx.x + off];
      red[0][threadIdx.x] = (x > red[0][threadIdx.x] || x != x) ? x : red[0][threadIdx.x];
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && !(red[0][0] <= tol * red[1][0])) gp(P[it].fredo)[sd] = 1;
}

// ---------------------------------------------------------------------------
// Boundary columns of the diagonal block of each slab inverse:
//   Sigma_rho = (D_rho - W_rho Gl_{rho-1} W_rho - W_{rho+1} Gr_{rho+1} W_{rho+1})^-1,
// columns k = 0 (left, next to interface s-1) and k = b-1 (right, next to
// interface s), pre-scaled by the interface edge weights:
//   sig[s][rho][0] = wL_rho Sigma_rho[:, 0],  sig[s][rho][1] = wR_rho Sigma_rho[:, b-1].
// These start the downward propagation (Sec. 3.1, eq. (T11_detailed)).
// BP lanes per (slab, rho), lane = row; Gauss-Jordan elimination of the matrix
// augmented with the two unit columns, touching at pivot p only the columns
// right of p and the two right-hand sides (the inverse itself is not formed).
// The pivot row goes through LDS with wave-level ordering only: the problems
// of a wave never wait for another wave.
// ---------------------------------------------------------------------------
template <typename T, int BP>
__global__ __launch_bounds__(256) void k_sigma(const ProbDev* __restrict__ P,
                                               const int* __restrict__ offs, int count) {
  constexpr int PPW = 64 / BP;  // problems per wave
  constexpr int RW = BP + 3;    // published pivot row: columns, pivot, two right-hand sides
  const int it = group_item(offs, count, blockIdx.x);
  const int bx = blockIdx.x - offs[it];
  const g_t<const double>* __restrict__ wh = gp((const double*)P[it].wh);
  const g_t<const double>* __restrict__ wv = gp((const double*)P[it].wv);
  const int n2 = P[it].n2, b = P[it].b, m = P[it].m;
  const g_t<const T>* __restrict__ Gl = gp((const T*)P[it].Gl);
  const g_t<const T>* __restrict__ Hsw = gp((const T*)P[it].Hsw);
  g_t<T>* __restrict__ sig = gp((T*)P[it].sig);
  g_t<int>* __restrict__ status = gp(P[it].status);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int h = lane / BP, i = lane % BP;
  const long long idx = ((long long)bx * 4 + wave) * PPW + h;
  const bool valid = idx < (long long)m * n2;
  const int s = valid ? (int)(idx / n2) : 0;
  const int rho = valid ? (int)(idx % n2) : 0;
  const int c0 = s * (b + 1);
  const long long c = c0 + (i < b ? i : 0);
  __shared__ T pivrow[4][PPW][2][RW];
  __shared__ T wsh[4][PPW][BP];
  T a[BP];
  build_D_row<T, BP>(a, wh, wv, gp((const double*)P[it].shift), P[it].shift_stride, n2, b, c0,
                     rho, i);
  // top coupling W_rho Gl_{rho-1} W_rho (column weights through LDS), bottom
  // coupling W_{rho+1} Hr_{rho+1} (Hr already carries the column scaling);
  // loads from clamped rows, masked by the weights
  const T wt = (rho > 0 && i < b) ? (T)wv[c * (n2 + 1) + rho] : (T)0;
  const T wb = (rho < n2 - 1 && i < b) ? (T)wv[c * (n2 + 1) + rho + 1] : (T)0;
  wsh[wave][h][i] = wt;
  wave_lds_sync();
  {
    const g_t<const T>* G = Gl + (((size_t)s * n2 + max(rho - 1, 0)) * BP + i) * BP;
    const g_t<const T>* H = Hsw + ((size_t)s * n2 + min(rho + 1, n2 - 1)) * BP * BP;
#pragma unroll
    for (int k = 0; k < BP; ++k) a[k] -= wt * G[k] * wsh[wave][h][k] + wb * H[swz_index<T>(i, k, BP)];
  }
  T rl = (i == 0) ? (T)1 : (T)0, rr = (i == b - 1) ? (T)1 : (T)0;
  const bool signed_piv = P[it].shift_stride != 0;   // as in k_slab_factor
  bool ok = true;
#pragma unroll
  for (int p = 0; p < BP; ++p) {
    T* pr = pivrow[wave][h][p & 1];
    if (i == p) {
#pragma unroll
      for (int k = p; k < BP; ++k) pr[k] = a[k];
      pr[BP + 1] = rl;
      pr[BP + 2] = rr;
    }
    wave_lds_sync();
    const T d = pr[p];
    ok = ok && (signed_piv ? d != (T)0 : d > (T)0) && isfinite((double)d);
    const T inv = fast_recip(d);
    const bool piv = i == p;
    // other rows: x -= f x_p with f = a[p] / d; the pivot row is scaled (no
    // cancellation): x = inv x_p
    const T t = piv ? inv : -(a[p] * inv);
    const T keep = piv ? (T)0 : (T)1;
#pragma unroll
    for (int k = p + 1; k < BP; ++k) a[k] = fma(t, pr[k], a[k] * keep);
    rl = fma(t, pr[BP + 1], rl * keep);
    rr = fma(t, pr[BP + 2], rr * keep);
  }
  if (valid) {
    const double wL = wh[(long long)c0 * n2 + rho];
    const double wR = wh[(long long)(c0 + b) * n2 + rho];
    g_t<T>* dst = sig + ((size_t)s * n2 + rho) * 2 * BP;
    dst[i] = (T)(wL * (double)rl);
    dst[BP + i] = (T)(wR * (double)rr);
  }
  if (valid && !ok && i == 0) { status[0] = 2; status[1] = s; }
}

// ---------------------------------------------------------------------------
// Schur propagation.  For slab s the 2n x 2n block A_oe A_ee^-1 A_eo needs the
// entries of A_ee^-1 at the slab's first and last column only.  Column rho of
// the inverse below its diagonal block follows
//   (A_ee^-1)_{r,rho} = Hr_r (A_ee^-1)_{r-1,rho},  r > rho,
// so each chain starts from sig[s][rho] and is propagated down the slab.  A
// workgroup carries 64 consecutive rho (128 chains: left and right) as the
// N dimension of 16x16x4 MFMA tiles whose results stay in registers between
// steps (the fragment-major propagator order makes the output layout equal the
// next B operand).  Row 0 of a chain sits in lane group 0, element 0 for both
// precisions.  Outputs, lower triangles (r >= rho) only, per slab:
//   PLL[s][r][rho] = wL_r (A_ee^-1)[(r,0),(rho,0)] wL_rho     (-> T_{s-1,s-1})
//   PRR[s][r][rho] = wR_r (A_ee^-1)[(r,b-1),(rho,b-1)] wR_rho (-> T_{s,s})
//   PLR[s][r][rho] = wL_r (A_ee^-1)[(r,0),(rho,b-1)] wR_rho   (-> T_{s-1,s})
//   PRL[s][r][rho] = wR_r (A_ee^-1)[(r,b-1),(rho,0)] wL_rho   (-> T_{s,s-1})
// ---------------------------------------------------------------------------
#ifndef SLAB_SCHUR_LDS
#define SLAB_SCHUR_LDS 1
#endif
#ifndef SLAB_SCHUR_ROWS
#define SLAB_SCHUR_ROWS 1   // propagator rows per barrier (2 measured slower)
#endif
template <typename T, int BP>
__global__ __launch_bounds__(256) void k_schur(const ProbDev* __restrict__ P,
                                               const int* __restrict__ offs, int count) {
  typedef typename acc4<T>::type V4;
  constexpr int NM = BP / 16, NK = BP / 4;
  // (generic pointers on purpose: with global-space pointers the compiler
  // interleaves per-load waits with the MFMA chain and the kernel is slower)
  const int it = group_item(offs, count, blockIdx.x);
  const int bx = blockIdx.x - offs[it];
  const double* __restrict__ wh = P[it].wh;
  const int n2 = P[it].n2, b = P[it].b, m = P[it].m;
  const T* __restrict__ Hsw = (const T*)P[it].Hsw;
  const T* __restrict__ sig = (const T*)P[it].sig;
  T* __restrict__ PRR = (T*)P[it].PRR;
  T* __restrict__ PLL = (T*)P[it].PLL;
  T* __restrict__ PLR = (T*)P[it].PLR;
  T* __restrict__ PRL = (T*)P[it].PRL;
  const int q = bx / m, s = bx % m;
  const int rho0 = q * 64;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane >> 4, nn = lane & 15;
  const int Y = wave >> 1;                 // 0: left chains, 1: right chains
  const int rb = rho0 + (wave & 1) * 32;  // first rho of this wave
  const int c0 = s * (b + 1);
  const size_t nsq = (size_t)n2 * n2;
  const int RB = b - 1;
  const int mtR = RB >> 4, gR = acc_group<T>(RB & 15), iR = acc_elem<T>(RB & 15);
  T* outL = (Y == 0) ? PLL : PLR;
  T* outR = (Y == 0) ? PRL : PRR;
  const bool wL_ok = s > 0;
  const bool wR_ok = (Y == 1) || (s > 0);

  V4 acc[2][NM];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt)
#pragma unroll
    for (int mt = 0; mt < NM; ++mt) acc[nt][mt] = V4{0, 0, 0, 0};

#if SLAB_SCHUR_LDS
  // The four waves of a workgroup multiply by the same propagator Hr_r: it is
  // loaded once per workgroup (each thread a quarter) and parked in LDS
  // instead of being fetched from L2 by every wave.  Rows go in groups of G
  // (one barrier per group): while a group is multiplied, the next group's
  // propagators are in flight in registers; a ring of 2G slots holds them
  // (row r in slot (r - rho0 - 1) % 2G).
  constexpr int HE = BP * BP / 256;   // elements per thread and row
  constexpr int G = (BP == 64 && sizeof(T) == 8) ? 1 : SLAB_SCHUR_ROWS;
  __shared__ T Hs[2 * G][BP * BP];
  T hreg[G][HE];
#pragma unroll
  for (int q2 = 0; q2 < G; ++q2) {
    const T* H = Hsw + ((size_t)s * n2 + min(rho0 + 1 + q2, n2 - 1)) * BP * BP;
#pragma unroll
    for (int e = 0; e < HE; ++e) Hs[q2][threadIdx.x + 256 * e] = H[threadIdx.x + 256 * e];
  }
  __syncthreads();
#endif

  for (int r = rho0; r < n2; ++r) {
    if (r > rho0) {
      T afr[NM][NK];
#if SLAB_SCHUR_LDS
      const int ph = (r - rho0 - 1) % G;     // position in the group (uniform)
      const int slot = (r - rho0 - 1) % (2 * G);
      if (ph == 0) {
        // the next group's propagators (clamped rows past the end are not used)
#pragma unroll
        for (int q2 = 0; q2 < G; ++q2) {
          const T* Hn = Hsw + ((size_t)s * n2 + min(r + G + q2, n2 - 1)) * BP * BP;
#pragma unroll
          for (int e = 0; e < HE; ++e) hreg[q2][e] = Hn[threadIdx.x + 256 * e];
        }
      }
      const T* Hc = Hs[slot];
#pragma unroll
      for (int mt = 0; mt < NM; ++mt)
#pragma unroll
        for (int ks = 0; ks < NK; ++ks) afr[mt][ks] = Hc[(mt * NK + ks) * 64 + lane];
#else
      const T* H = Hsw + ((size_t)s * n2 + r) * BP * BP;
#pragma unroll
      for (int mt = 0; mt < NM; ++mt)
#pragma unroll
        for (int ks = 0; ks < NK; ++ks) afr[mt][ks] = H[(mt * NK + ks) * 64 + lane];
#endif
      V4 nacc[2][NM];
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int mt = 0; mt < NM; ++mt) {
          V4 d = V4{0, 0, 0, 0};
#pragma unroll
          for (int mt2 = 0; mt2 < NM; ++mt2)
#pragma unroll
            for (int i = 0; i < 4; ++i) d = mfma16(afr[mt][4 * mt2 + i], acc[nt][mt2][i], d);
          nacc[nt][mt] = d;
        }
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int mt = 0; mt < NM; ++mt) acc[nt][mt] = nacc[nt][mt];
#if SLAB_SCHUR_LDS
      if (ph == G - 1) {
        const int nslot = (slot + 1) % (2 * G);   // first slot of the next group
#pragma unroll
        for (int q2 = 0; q2 < G; ++q2)
#pragma unroll
          for (int e = 0; e < HE; ++e) Hs[(nslot + q2) % (2 * G)][threadIdx.x + 256 * e] = hreg[q2][e];
        __syncthreads();
      }
#endif
    }
    // start the chains of rho = r
    const int jr = r - rb;
    if (jr >= 0 && jr < 32 && nn == (jr & 15)) {
      const T* sv = sig + (((size_t)s * n2 + r) * 2 + Y) * BP;
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
        if (nt == (jr >> 4)) {
#pragma unroll
          for (int mt = 0; mt < NM; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[nt][mt][i] = sv[16 * mt + acc_row<T>(g, i)];
        }
    }
    // emit rows (r, left) and (r, right) of the chains started so far
    const double wLr = wh[(size_t)c0 * n2 + r];
    const double wRr = wh[(size_t)(c0 + b) * n2 + r];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int rho = rb + 16 * nt + nn;
      if (rho <= r) {
        const size_t off = (size_t)s * nsq + (size_t)r * n2 + rho;
        if (g == 0 && wL_ok) outL[off] = (T)(wLr * (double)acc[nt][0][0]);
        if (g == gR && wR_ok) {
          T v = (T)0;
#pragma unroll
          for (int mt = 0; mt < NM; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if (mt == mtR && i == iR) v = acc[nt][mt][i];
          outR[off] = (T)(wRr * (double)v);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Assembly of the reduced blocks (eqs. (T11)-(T35)), sums in FP64:
//   T_jj     = A_oo(j) - PRR[j] - PLL[j+1]      (symmetric; full block written)
//   T_{j,j+1} = -PLR[j+1] (lower part), -PRL[j+1]^T (upper part)
// A_oo(j): diagonal of the interface column, -w on the vertical edges.
// 64x64 tiles, 16 entries per thread.  The pieces hold lower triangles only:
// a tile at or below the diagonal reads its own entries, a tile at or above it
// reads the mirrored source tile and transposes it through LDS.  Every load is
// unconditional, from clamped indices, and masked where it is used (a skipped
// load makes the compiler wait for all outstanding ones); the A_oo entries of
// the tile's rows go through LDS.  Outputs in the precision TO of the block
// factorization, and in FP64 when the T64 pointers are given.
// ---------------------------------------------------------------------------
template <typename T, typename TO, bool OFF>
__device__ __forceinline__ void assemble_tile(const ProbDev& pd, int j, int ti, int tj,
                                              double (*tile)[65], double* aoo_d,
                                              double* aoo_s) {
  const g_t<const double>* __restrict__ wh = gp((const double*)pd.wh);
  const g_t<const double>* __restrict__ wv = gp((const double*)pd.wv);
  const int n2 = pd.n2, b = pd.b, m = pd.m;
  const g_t<const T>* __restrict__ PRR = gp((const T*)pd.PRR);
  const g_t<const T>* __restrict__ PLL = gp((const T*)pd.PLL);
  const g_t<const T>* __restrict__ PLR = gp((const T*)pd.PLR);
  const g_t<const T>* __restrict__ PRL = gp((const T*)pd.PRL);
  g_t<TO>* __restrict__ Tout = gp((TO*)(OFF ? pd.To : pd.Td));
  g_t<double>* __restrict__ Tout64 = gp(OFF ? pd.O64 : pd.T64);
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const size_t nsq = (size_t)n2 * n2;
  const bool lastj = j + 1 >= m;
  // T_jj: -PRR[j] - PLL[j+1] (+ A_oo);  T_{j,j+1}: -PLR[j+1] (lower), -PRL[j+1]^T (upper)
  const g_t<const T>* __restrict__ src0 = OFF ? PLR + (size_t)(j + 1) * nsq : PRR + (size_t)j * nsq;
  const g_t<const T>* __restrict__ src0m = OFF ? PRL + (size_t)(j + 1) * nsq : src0;
  const g_t<const T>* __restrict__ src1 = PLL + (size_t)min(j + 1, m - 1) * nsq;
  const bool direct = ti >= tj, mirrored = ti <= tj;  // uniform
  // A_oo entries of rows ti*64 + tx (diagonal tiles and the tiles just below
  // them), and A_oo(rho, rho-1) of this thread's column (the superdiagonal of
  // the mirrored part)
  double aoo_c = 0.0;
  if (!OFF) {
    const long long cj = (long long)j * (b + 1) + b;
    const int R = min(ti * 64 + tx, n2 - 1), C = min(tj * 64 + tx, n2 - 1);
    aoo_d[tx] = wh[cj * n2 + R] + wh[(cj + 1) * n2 + R] + wv[cj * (n2 + 1) + R] +
                wv[cj * (n2 + 1) + R + 1] + gp((const double*)pd.shift)[(cj * n2 + R) * pd.shift_stride];
    aoo_s[tx] = -wv[cj * (n2 + 1) + R];
    aoo_c = -wv[cj * (n2 + 1) + C];
  }
  T q0[16], q1[16];
  if (mirrored) {  // source tile (tj, ti), transposed through LDS
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int R = min(tj * 64 + ty + 4 * k, n2 - 1), Pc = min(ti * 64 + tx, n2 - 1);
      const size_t o = (size_t)R * n2 + Pc;
      q0[k] = src0m[o];
      if (!OFF) q1[k] = src1[o];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int R = tj * 64 + ty + 4 * k, Pc = ti * 64 + tx;
      double v = -(double)q0[k];
      if (!OFF) v -= lastj ? 0.0 : (double)q1[k];
      tile[ty + 4 * k][tx] = (R < n2 && Pc < n2 && R >= Pc) ? v : 0.0;
    }
  }
  T d0[16], d1[16];
  if (direct) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int r = min(ti * 64 + ty + 4 * k, n2 - 1), rho = min(tj * 64 + tx, n2 - 1);
      const size_t o = (size_t)r * n2 + rho;
      d0[k] = src0[o];
      if (!OFF) d1[k] = src1[o];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int yy = ty + 4 * k;
    const int r = ti * 64 + yy, rho = tj * 64 + tx;
    double v = 0.0;
    if (r >= rho) {
      if (direct) {
        v = -(double)d0[k];
        if (!OFF) {
          v -= lastj ? 0.0 : (double)d1[k];
          if (r == rho) v += aoo_d[yy];
          if (r == rho + 1) v += aoo_s[yy];
        }
      }
    } else if (mirrored) {
      v = tile[tx][yy];  // source (rho, r)
      if (!OFF && rho == r + 1) v += aoo_c;
    }
    if (r < n2 && rho < n2) {
      const size_t o = (size_t)j * nsq + (size_t)r * n2 + rho;
      Tout[o] = (TO)v;
      if (Tout64) Tout64[o] = v;
    }
  }
}

template <typename T, typename TO>
__global__ __launch_bounds__(256) void k_assemble(const ProbDev* __restrict__ P,
                                                  const int* __restrict__ offs, int count) {
  __shared__ double tile[64][65];
  __shared__ double aoo_d[64], aoo_s[64];  // A_oo(r, r) and A_oo(r, r-1) of the tile's rows
  const int it = group_item(offs, count, blockIdx.x);
  const int bx = blockIdx.x - offs[it];
  const int n2 = P[it].n2, m = P[it].m;
  // workgroup bx: tile (ti, tj) of block j, kind off (0: T_jj, 1: T_{j,j+1})
  const int ntl = (n2 + 63) / 64;
  const int per = ntl * ntl;
  const int j = (bx / per) % m;
  const bool off = bx / (per * m) == 1;
  const int ti = (bx % per) / ntl, tj = (bx % per) % ntl;
  if (off) {
    if (j >= m - 1) return;  // uniform
    assemble_tile<T, TO, true>(P[it], j, ti, tj, tile, aoo_d, aoo_s);
  } else {
    assemble_tile<T, TO, false>(P[it], j, ti, tj, tile, aoo_d, aoo_s);
  }
}

// ---------------------------------------------------------------------------
// Launchers: record stage one of a group of problems into a plan.
// ---------------------------------------------------------------------------
static long long fill_wgs(long long elems) { return std::min<long long>((elems + 255) / 256, 1024); }

void plan_coef_weights(Plan& plan, const std::vector<ProbDev>& probs) {
  const size_t pd = plan.add_vec(probs);
  std::vector<int> cc, cw;
  for (const ProbDev& d : probs) {
    cc.push_back((int)fill_wgs((long long)(d.n1 + 2) * (d.n2 + 2)));
    cw.push_back((int)fill_wgs((long long)(d.n1 + 1) * d.n2 + (long long)d.n1 * (d.n2 + 1)));
  }
  std::vector<int> cs;
  for (const ProbDev& d : probs)
    cs.push_back((int)fill_wgs(d.shift_src ? (long long)d.n1 * d.n2 : 1));
  long long tc, tw, ts;
  const size_t oc = plan.add_offsets(cc, &tc), ow = plan.add_offsets(cw, &tw),
               os = plan.add_offsets(cs, &ts);
  const int count = (int)probs.size();
  plan.step([=](const char* dev, hipStream_t st) {
    hipLaunchKernelGGL(k_status_clear, dim3((unsigned)((4 * count + 255) / 256)), dim3(256), 0,
                       st, dev_at<ProbDev>(dev, pd), count);
    SLAB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_coef, dim3((unsigned)tc), dim3(256), 0, st, dev_at<ProbDev>(dev, pd),
                       dev_at<int>(dev, oc), count);
    SLAB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_shift, dim3((unsigned)ts), dim3(256), 0, st, dev_at<ProbDev>(dev, pd),
                       dev_at<int>(dev, os), count);
    SLAB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_weights, dim3((unsigned)tw), dim3(256), 0, st, dev_at<ProbDev>(dev, pd),
                       dev_at<int>(dev, ow), count);
    SLAB_LAUNCH_CHECK();
    return SLAB_OK;
  });
}

template <typename T, typename TO, int BP>
static void plan_stage1_bp(Plan& plan, const std::vector<ProbDev>& probs, int phase,
                           hipEvent_t ev) {
  const size_t pd = plan.add_vec(probs);
  const int count = (int)probs.size();
  std::vector<int> c;
  long long tot = 0;
  size_t off = 0;
  auto counts = [&](auto f) {
    c.clear();
    for (const ProbDev& d : probs) c.push_back((int)f(d));
    off = plan.add_offsets(c, &tot);
  };
  if (phase == 0) {
    // segments of every chain, then the warm-up check and the redo of the
    // chains it marks (its workgroups of unmarked chains return at once)
    counts([](const ProbDev& d) { return 2LL * d.m * d.fnseg; });
    const size_t o_seg = off;
    const long long t_seg = tot;
    counts([](const ProbDev& d) { return 2LL * d.m * (d.fnseg - 1); });
    const size_t o_chk = off;
    const long long t_chk = tot;
    counts([](const ProbDev& d) { return 2LL * d.m; });
    const size_t o_redo = off;
    const long long t_redo = tot;
    // a converged warm-up differs from the full chain by rounding only
    const double tol = sizeof(T) == 8 ? 1e-13 : 1e-5;
    const bool narrow = BP <= 32 && t_seg >= SLAB_FACTOR_MANY;
    plan.step([=](const char* dev, hipStream_t st) {
      if (narrow)
        hipLaunchKernelGGL((k_slab_factor<T, BP, (BP <= 32 ? 128 : SLAB_FACTOR_THREADS)>),
                           dim3((unsigned)t_seg), dim3(BP <= 32 ? 128 : SLAB_FACTOR_THREADS), 0,
                           st, dev_at<ProbDev>(dev, pd), dev_at<int>(dev, o_seg), count, 0);
      else
        hipLaunchKernelGGL((k_slab_factor<T, BP>), dim3((unsigned)t_seg), dim3(SLAB_FACTOR_THREADS),
                           0, st, dev_at<ProbDev>(dev, pd), dev_at<int>(dev, o_seg), count, 0);
      SLAB_LAUNCH_CHECK();
      if (t_chk > 0) {
        hipLaunchKernelGGL((k_factor_check<T, BP>), dim3((unsigned)t_chk), dim3(256), 0, st,
                           dev_at<ProbDev>(dev, pd), dev_at<int>(dev, o_chk), count, tol);
        SLAB_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_slab_factor<T, BP>), dim3((unsigned)t_redo), dim3(SLAB_FACTOR_THREADS), 0, st,
                           dev_at<ProbDev>(dev, pd), dev_at<int>(dev, o_redo), count, 1);
        SLAB_LAUNCH_CHECK();
      }
      if (ev) SLAB_HIP_CHECK(hipEventRecord(ev, st));
      return SLAB_OK;
    });
  } else if (phase == 1) {
    counts([](const ProbDev& d) { return ceil_div((long long)d.m * d.n2, 4LL * (64 / BP)); });
    plan.step([=](const char* dev, hipStream_t st) {
      hipLaunchKernelGGL((k_sigma<T, BP>), dim3((unsigned)tot), dim3(256), 0, st,
                         dev_at<ProbDev>(dev, pd), dev_at<int>(dev, off), count);
      SLAB_LAUNCH_CHECK();
      if (ev) SLAB_HIP_CHECK(hipEventRecord(ev, st));
      return SLAB_OK;
    });
  } else if (phase == 2) {
    counts([](const ProbDev& d) { return (long long)((d.n2 + 63) / 64) * d.m; });
    plan.step([=](const char* dev, hipStream_t st) {
      hipLaunchKernelGGL((k_schur<T, BP>), dim3((unsigned)tot), dim3(256), 0, st,
                         dev_at<ProbDev>(dev, pd), dev_at<int>(dev, off), count);
      SLAB_LAUNCH_CHECK();
      if (ev) SLAB_HIP_CHECK(hipEventRecord(ev, st));
      return SLAB_OK;
    });
  } else {
    counts([](const ProbDev& d) {
      const long long ntl = (d.n2 + 63) / 64;
      return ntl * ntl * d.m * 2;
    });
    plan.step([=](const char* dev, hipStream_t st) {
      hipLaunchKernelGGL((k_assemble<T, TO>), dim3((unsigned)tot), dim3(256), 0, st,
                         dev_at<ProbDev>(dev, pd), dev_at<int>(dev, off), count);
      SLAB_LAUNCH_CHECK();
      if (ev) SLAB_HIP_CHECK(hipEventRecord(ev, st));
      return SLAB_OK;
    });
  }
}

template <typename T, typename TO>
void plan_stage1(Plan& plan, const std::vector<ProbDev>& probs, const hipEvent_t* ev) {
  // one launch per phase and padded block order; the event of a phase is
  // recorded after its last launch
  std::vector<ProbDev> cls[3];
  for (const ProbDev& d : probs) {
    const int bp = padded_block(d.b);
    cls[bp == 16 ? 0 : (bp == 32 ? 1 : 2)].push_back(d);
  }
  for (int phase = 0; phase < 4; ++phase) {
    int last = -1;
    for (int k = 0; k < 3; ++k)
      if (!cls[k].empty()) last = k;
    for (int k = 0; k < 3; ++k) {
      if (cls[k].empty()) continue;
      const hipEvent_t e = (ev && k == last) ? ev[phase] : nullptr;
      if (k == 0) plan_stage1_bp<T, TO, 16>(plan, cls[k], phase, e);
      else if (k == 1) plan_stage1_bp<T, TO, 32>(plan, cls[k], phase, e);
      else plan_stage1_bp<T, TO, 64>(plan, cls[k], phase, e);
    }
  }
}
template void plan_stage1<float, float>(Plan&, const std::vector<ProbDev>&, const hipEvent_t*);
template void plan_stage1<double, double>(Plan&, const std::vector<ProbDev>&, const hipEvent_t*);
template void plan_stage1<double, float>(Plan&, const std::vector<ProbDev>&, const hipEvent_t*);

}  // namespace slab
