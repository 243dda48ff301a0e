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
// One workgroup per (problem, slab, group of SLAB_SWEEP_THREADS/BP columns);
// thread = (row i, column).
// Software pipeline: while row step r is computed, the block inverses and
// edge weights of the next D steps are in flight in a register ring and
// parked in the other half of double-buffered LDS when their step comes (one
// barrier per step).  The natural-order vectors are touched one ring pass at
// a time: each thread loads its right-hand sides of the next D rows together
// and stores its outputs of the last D rows together (consecutive rows of one
// column share cache lines).  The vector a step multiplies is formed by the
// thread that owns each entry, so a step reads only the block inverse and
// that vector from LDS.
// ---------------------------------------------------------------------------
#ifndef SLAB_SWEEP_VEC
#define SLAB_SWEEP_VEC 1   // 16-byte LDS reads in the sweep products (0: 8-byte, measured slower)
#endif
#ifndef SLAB_SWEEP_THREADS
#define SLAB_SWEEP_THREADS 256   // threads per sweep workgroup (64, 128 or 256)
#endif
// t[k mod 4] += g[k] v[k] over k < BP; VEC: 16-byte LDS reads (g and v
// 16-byte aligned)
template <typename T, int BP, bool VEC>
__device__ __forceinline__ void dot_row(const T* g, const T* v, T (&t)[4]) {
  if constexpr (VEC) {
    constexpr int W = 16 / sizeof(T);
    typedef T vt __attribute__((ext_vector_type(W)));
#pragma unroll
    for (int k = 0; k < BP; k += W) {
      const vt gg = *(const vt*)(g + k), vv = *(const vt*)(v + k);
#pragma unroll
      for (int e = 0; e < W; ++e) t[(k + e) & 3] += gg[e] * vv[e];
    }
  } else {
#pragma unroll
    for (int k = 0; k < BP; ++k) t[k & 3] += g[k] * v[k];
  }
}

template <typename T, typename TU, int BP, bool TRANS, int MODE>
__global__ __launch_bounds__(SLAB_SWEEP_THREADS) void k_sweep(const SolveDev* __restrict__ P,
                                                              const int* __restrict__ offs,
                                                              int count) {
  constexpr int NT = SLAB_SWEEP_THREADS;
  constexpr int NC = NT / BP;             // columns per workgroup
  constexpr int GPT = BP * BP / NT;       // block-inverse elements loaded per thread
  static_assert(NC >= 1 && GPT * NT == BP * BP, "sweep workgroup shape");
  // prefetch depth (row steps), scaled with the elements each thread loads
#ifdef SLAB_SWEEP_D0
  constexpr int D0 = SLAB_SWEEP_D0;
#else
  // (16 for 16- and 32-row blocks: measured faster than 8 and 4; 32 spills)
  constexpr int D0 = BP == 64 ? (sizeof(T) == 8 ? 2 : 4) : 16;
#endif
  constexpr int D = D0 * NT / 256 > 0 ? D0 * NT / 256 : 1;
  // SLAB_SWEEP_VEC: rows padded to 16 bytes and read as 16-byte vectors in the
  // products with Gl (not transposed)
  constexpr int GPAD = SLAB_SWEEP_VEC ? 16 / (int)sizeof(T) : 1;
  __shared__ __attribute__((aligned(16))) T Gs[2][BP][BP + GPAD];
  __shared__ __attribute__((aligned(16))) T Vs[2][NC][BP + GPAD];
  const int itm = group_item(offs, count, blockIdx.x);
  if (item_done(P[itm].live)) return;
  const int bx = blockIdx.x - offs[itm];
  const int m = P[itm].m;
  const int s = bx % m;
  // descriptor fields copied to locals (the lambdas below capture locals only)
  const int n2 = P[itm].n2, b = P[itm].b, nrhs = P[itm].nrhs;
  const long long ld = P[itm].ld, ldo = P[itm].ldo;
  const g_t<const double>* __restrict__ wh = gp(P[itm].wh);
  const g_t<const double>* __restrict__ wv = gp(P[itm].wv);
  const g_t<const double>* __restrict__ rhs = gp(P[itm].rhs);
  g_t<double>* __restrict__ out_g = gp(P[itm].out);
  g_t<T>* __restrict__ xbuf = gp((T*)P[itm].xb);
  const int tid = threadIdx.x;
  const int i = tid % BP, cl = tid / BP;
  const int c = (bx / m) * NC + cl;
  const bool valid = c < nrhs;
  const bool act = i < b;
  const long long c0 = (long long)s * (b + 1);
  const long long ci = c0 + (act ? i : 0);
  const g_t<const T>* Gl = gp((const T*)P[itm].Gl) + (size_t)s * n2 * BP * BP;
  g_t<T>* zbuf = gp((T*)P[itm].zbuf) + (size_t)s * nrhs * n2 * BP;
  const bool acc_out = MODE == 1 && P[itm].accumulate;

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
    return (act && r >= 1 && r <= n2 - 1) ? wv[ci * (n2 + 1) + r] : 0.0;
  };
  // forward step r: G = Gl_{r-1} (A x) or Gl_r (A^T x), w = W_r, y = y_r
  auto load_fwd = [&](int d, int r) __attribute__((always_inline)) {
    const int gr = TRANS ? r : r - 1;
    if (gr >= 0) {
      const g_t<const T>* G = Gl + (size_t)gr * BP * BP;
#pragma unroll
      for (int e = 0; e < GPT; ++e) rg[d][e] = G[tid + NT * e];
    }
    rw[d] = load_w(r);
  };
  // right-hand side of row r (natural order) into y slot d
  auto load_y = [&](double (&yy)[D], T (&xx)[D], int d, int r) __attribute__((always_inline)) {
    yy[d] = (valid && act && r < n2) ? rhs[(long long)c * ld + ci * n2 + r] : 0.0;
    if (MODE == 1)
      xx[d] = (valid && act && xslot >= 0 && r < n2)
                  ? xbuf[(((size_t)s * 2 + xslot) * nrhs + c) * n2 + r] : (T)0;
  };
  // backward step r: G = Gl_r, w = W_{r+1}, z = z_r (+ old outputs when accumulating)
  auto load_bwd = [&](int d, int r) __attribute__((always_inline)) {
    const g_t<const T>* G = Gl + (size_t)r * BP * BP;
#pragma unroll
    for (int e = 0; e < GPT; ++e) rg[d][e] = G[tid + NT * e];
    rw[d] = load_w(r + 1);
    rz[d] = valid ? zbuf[((size_t)c * n2 + r) * BP + i] : (T)0;
    ru[d] = (MODE == 1 && valid && acc_out && act) ? out_g[(long long)c * ldo + ci * n2 + r] : 0.0;
    if (MODE == 0) {  // interface edge weights of the boundary outputs
      rbl[d] = (valid && i == 0) ? wh[c0 * n2 + r] : 0.0;
      rbr[d] = (valid && i == b - 1) ? wh[(c0 + b) * n2 + r] : 0.0;
    }
  };
  // (A^T x: the block is parked transposed, so that every product reads a row)
  auto parkG = [&](int d, int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < GPT; ++e) {
      const int idx = tid + NT * e;
      if (TRANS) Gs[buf][idx % BP][idx / BP] = rg[d][e];
      else Gs[buf][idx / BP][idx % BP] = rg[d][e];
    }
  };
  // right-hand side of ring slot d (forward steps)
  auto yval = [&](int d) __attribute__((always_inline)) -> T {
    return (T)(ry[d] + (MODE == 1 ? (double)rx[d] : 0.0));
  };

  // ---------------- forward sweep: z_r (stored in zbuf) ----------------
  // Vs holds the vector the step's block inverse multiplies; the thread that
  // owns entry (i, column) forms it for the next step from its own values:
  //   A x:    forward v = z_{r-1};                backward v = z_r + W_{r+1} x_{r+1}
  //   A^T x:  forward v = y_r + W_r z_{r-1};      backward v = W_{r+1} x_{r+1}
  // so a step reads only the block inverse and v from LDS.
  // the right-hand sides of a ring pass are loaded together one pass ahead
  // (consecutive rows of one natural-order column: each cache line is read
  // at once instead of over D row steps)
  double ryn[D];
  T rxn[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    ryn[d] = 0.0;
    rxn[d] = (T)0;
  }
#pragma unroll
  for (int d = 0; d < D; ++d) load_y(ry, rx, d, d);
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (d < n2) load_fwd(d, d);
  Vs[0][cl][i] = TRANS ? yval(0) : (T)0;
  for (int r0 = 0; r0 < n2; r0 += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) load_y(ryn, rxn, d, r0 + D + d);
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int r = r0 + d;
      if (r < n2) {  // uniform
      const int cur = r & 1;
      parkG(d, cur);
      const T y = yval(d), w = (T)rw[d];
      if (r + D < n2) load_fwd(d, r + D);
      __syncthreads();
      // dot products over k in four independent partial sums (short FMA chains)
      T out, vn;
      if (!TRANS) {
        T t[4] = {(T)0, (T)0, (T)0, (T)0};
        if (r > 0) dot_row<T, BP, SLAB_SWEEP_VEC>(&Gs[cur][i][0], &Vs[cur][cl][0], t);
        out = y + w * ((t[0] + t[1]) + (t[2] + t[3]));
        vn = out;
      } else {
        T t[4] = {(T)0, (T)0, (T)0, (T)0};
        dot_row<T, BP, SLAB_SWEEP_VEC>(&Gs[cur][i][0], &Vs[cur][cl][0], t);
        out = (t[0] + t[1]) + (t[2] + t[3]);
        const int dn = (d + 1) % D;  // ring slot of the next step
        // (the next pass's first right-hand side is still in the batch buffer)
        const T yn = d + 1 < D ? yval(dn) : (T)(ryn[0] + (MODE == 1 ? (double)rxn[0] : 0.0));
        vn = yn + (T)rw[dn] * out;
      }
      if (valid) zbuf[((size_t)c * n2 + r) * BP + i] = out;
      Vs[cur ^ 1][cl][i] = vn;
      }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      ry[d] = ryn[d];
      rx[d] = rxn[d];
    }
  }
  __syncthreads();

  // ---------------- backward sweep: x_r ----------------
#pragma unroll
  for (int d = 0; d < D; ++d)
    if (d < n2) load_bwd(d, n2 - 1 - d);
  Vs[0][cl][i] = TRANS ? (T)0 : rz[0];
  for (int t0 = 0; t0 < n2; t0 += D) {
    // MODE 1: this thread's outputs of the D steps, stored together after them
    // (consecutive rows of one natural-order column: each cache line is
    // written at once instead of over D row steps)
    T xs[D];
    double us[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int it = t0 + d;
      if (it < n2) {  // uniform
      const int r = n2 - 1 - it;
      const int cur = it & 1;
      parkG(d, cur);
      const double uold = ru[d], wbl = rbl[d], wbr = rbr[d];
      const T z = rz[d];
      if (it + D < n2) load_bwd(d, r - D);
      __syncthreads();
      T x;
      const int dn = (d + 1) % D;  // ring slot of the next step (row r - 1)
      if (!TRANS) {
        T t[4] = {(T)0, (T)0, (T)0, (T)0};
        dot_row<T, BP, SLAB_SWEEP_VEC>(&Gs[cur][i][0], &Vs[cur][cl][0], t);
        x = (t[0] + t[1]) + (t[2] + t[3]);
        Vs[cur ^ 1][cl][i] = rz[dn] + (T)rw[dn] * x;
      } else {
        T t[4] = {(T)0, (T)0, (T)0, (T)0};
        dot_row<T, BP, SLAB_SWEEP_VEC>(&Gs[cur][i][0], &Vs[cur][cl][0], t);
        x = z + ((t[0] + t[1]) + (t[2] + t[3]));
        Vs[cur ^ 1][cl][i] = (T)rw[dn] * x;
      }
      if (MODE == 0 && valid) {
        if (i == 0) xbuf[(((size_t)s * 2 + 0) * nrhs + c) * n2 + r] = (T)(wbl * (double)x);
        if (i == b - 1) xbuf[(((size_t)s * 2 + 1) * nrhs + c) * n2 + r] = (T)(wbr * (double)x);
      }
      xs[d] = x;
      us[d] = uold;
      }
    }
    if (MODE == 1 && valid && act) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int it = t0 + d;
        if (it < n2)
          out_g[(long long)c * ldo + ci * n2 + (n2 - 1 - it)] =
              acc_out ? us[d] + (double)xs[d] : (double)xs[d];
      }
    }
  }
}

// Interface coupling of the interior solve (eq. (usol_even)): for slab s,
//   xb[s][0][c][r] = wL_r u_o(s-1)[c][r]   (+ wR_r u_o(s)[c][r] when b = 1)
//   xb[s][1][c][r] = wR_r u_o(s)[c][r]
// with wL, wR the edge weights between the slab and its two interfaces.
// Grid-stride loop over m * nrhs * n2 entries of a problem with its own
// workgroups of a grouped launch.
#define SLAB_ITEM_LOOP(e, tot)                                                        \
  const int itm = group_item(offs, count, blockIdx.x);                                \
  const long long nwg_ = offs[itm + 1] - offs[itm];                                   \
  const SolveDev& d = P[itm];                                                         \
  if (item_done(d.live)) return;                                                      \
  const int n2 = d.n2, b = d.b, m = d.m, nrhs = d.nrhs;                               \
  const long long tot = (long long)m * nrhs * n2;                                     \
  for (long long e = (blockIdx.x - offs[itm]) * (long long)blockDim.x + threadIdx.x; \
       e < tot; e += nwg_ * blockDim.x)

template <typename T, typename TR>
__global__ void k_coupling(const SolveDev* __restrict__ P, const int* __restrict__ offs,
                           int count) {
  SLAB_ITEM_LOOP(e, tot) {
    const g_t<const double>* __restrict__ wh = gp(d.wh);
    const g_t<const TR>* __restrict__ uo = gp((const TR*)d.ft);
    const g_t<const double>* __restrict__ u64 = gp(d.uo64);
    auto uval = [&](long long i) -> double { return u64 ? u64[i] : (double)uo[i]; };
    g_t<T>* __restrict__ xb = gp((T*)d.xb);
    const long long r = e % n2;
    const long long c = (e / n2) % nrhs;
    const long long s = e / ((long long)n2 * nrhs);
    const long long c0 = s * (b + 1);
    const double right = wh[(c0 + b) * n2 + r] * uval((s * nrhs + c) * n2 + r);
    double left = s > 0 ? wh[c0 * n2 + r] * uval(((s - 1) * nrhs + c) * n2 + r) : 0.0;
    if (b == 1) left += right;
    xb[((s * 2 + 0) * nrhs + c) * n2 + r] = (T)left;
    xb[((s * 2 + 1) * nrhs + c) * n2 + r] = (T)right;
  }
}

// Interface values u_o(j) (reduced solution, [j][c][r]) into the natural-order
// output column j(b+1)+b, written or added.
template <typename TR>
__global__ void k_interface_out(const SolveDev* __restrict__ P, const int* __restrict__ offs,
                                int count) {
  SLAB_ITEM_LOOP(e, tot) {
    const long long r = e % n2;
    const long long c = (e / n2) % nrhs;
    const long long j = e / ((long long)n2 * nrhs);
    g_t<double>* o = gp(d.out) + c * d.ldo + (j * (b + 1) + b) * n2 + r;
    const double v = d.uo64 ? gp(d.uo64)[e] : (double)gp((const TR*)d.ft)[e];
    *o = d.accumulate ? *o + v : v;
  }
}

// f~_j = f_o(j) + xb[j][right] + xb[j+1][left]   (FP64 sum, stored in TR, and
// in FP64 too when the reduced solve is refined)
template <typename T, typename TR>
__global__ void k_reduced_rhs(const SolveDev* __restrict__ P, const int* __restrict__ offs,
                              int count) {
  SLAB_ITEM_LOOP(e, tot) {
    const g_t<const T>* __restrict__ xb = gp((const T*)d.xb);
    const long long r = e % n2;
    const long long c = (e / n2) % nrhs;
    const long long j = e / ((long long)n2 * nrhs);
    const long long cj = j * (b + 1) + b;
    double v = gp(d.rhs)[c * d.ld + cj * n2 + r];
    v += (double)xb[((j * 2 + 1) * nrhs + c) * n2 + r];
    if (j + 1 < m) v += (double)xb[(((j + 1) * 2 + 0) * nrhs + c) * n2 + r];
    gp((TR*)d.ft)[e] = (TR)v;
    if (d.g64) gp(d.g64)[e] = v;
  }
}
#undef SLAB_ITEM_LOOP

static long long item_wgs(long long elems) { return std::min<long long>((elems + 255) / 256, 1024); }

// Reduced system T x = f~ of every problem (in place in ft): Alg. 2 with the
// block Cholesky factors, or the odd-even order, as factored.
template <typename TR>
static void plan_reduced(Plan& plan, const std::vector<ReducedDev>& R, bool odd_even) {
  auto at = [](const void* base, long long j, long long stride) {
    return (void*)((TR*)base + j * stride);
  };
  // every product of a problem carries its refinement flag
  const int* live_flag = nullptr;
  auto item = [&live_flag](const void* M, const void* x, const void* xin, void* y, int n,
                           int nrhs, void* part = nullptr, const void* xs = nullptr) {
    BmvItem b;
    b.M = M; b.x = x; b.xin = xin; b.y = y; b.n = n; b.nrhs = nrhs; b.part = part;
    b.live = live_flag;
    b.xscale = xs;
    return b;
  };
  // pivot signs J_j of a signed factorization, or null
  auto sg = [](const ReducedDev& r, long long j) -> const void* {
    return r.J ? (const void*)((const TR*)r.J + j * r.n) : nullptr;
  };
  // scratch slot s of a problem for a product split over k (see plan_gemv)
  auto part = [](const ReducedDev& r, int s) -> void* {
    if (!r.part || s >= BMV_PART_SLOTS) return nullptr;
    return (TR*)r.part + s * bmv_part_elems(r.n, r.nrhs);
  };
  int mmax = 0;
  for (const ReducedDev& r : R) mmax = std::max(mmax, r.m);
  if (!odd_even) {
    // T = R J R^T with R_jj = L_j, R_{j+1,j} = Z_j^T J_j (J = I unless signed):
    // forward y_j = L_j^-1 (f~_j - Z_{j-1}^T J_{j-1} y_{j-1}),
    // backward x_j = L_j^-T J_j (y_j - Z_j x_{j+1}), x overwriting f~
    for (int j = 0; j < mmax; ++j) {
      std::vector<BmvItem> a, bb;
      for (const ReducedDev& r : R) {
        if (j >= r.m) continue;
        live_flag = r.live;
        const long long nsq = (long long)r.n * r.n, vs = (long long)r.nrhs * r.n;
        const void* src = at(r.ft, j, vs);
        if (j > 0) {
          a.push_back(item(at(r.Z, j - 1, nsq), at(r.yt, j - 1, vs), at(r.ft, j, vs), r.tt, r.n,
                           r.nrhs, part(r, 0), sg(r, j - 1)));
          src = r.tt;
        }
        bb.push_back(item(at(r.Linv, j, nsq), src, nullptr, at(r.yt, j, vs), r.n, r.nrhs,
                          part(r, 1)));
      }
      plan_gemv<TR>(plan, true, false, a, (TR)-1, (TR)1);
      plan_gemv<TR>(plan, false, true, bb, (TR)1, (TR)0);
    }
    for (int j = mmax - 1; j >= 0; --j) {
      std::vector<BmvItem> a, bb;
      for (const ReducedDev& r : R) {
        if (j >= r.m) continue;
        live_flag = r.live;
        const long long nsq = (long long)r.n * r.n, vs = (long long)r.nrhs * r.n;
        const void* src = at(r.yt, j, vs);
        if (j < r.m - 1) {
          a.push_back(item(at(r.Z, j, nsq), at(r.ft, j + 1, vs), at(r.yt, j, vs), r.tt, r.n,
                           r.nrhs, part(r, 0)));
          src = r.tt;
        }
        bb.push_back(item(at(r.Linv, j, nsq), src, nullptr, at(r.ft, j, vs), r.n, r.nrhs,
                          part(r, 1), sg(r, j)));
      }
      plan_gemv<TR>(plan, false, false, a, (TR)-1, (TR)1);
      plan_gemv<TR>(plan, true, true, bb, (TR)1, (TR)0);
    }
    return;
  }
  // odd-even order (levels as in the factorization): reduce the right-hand
  // side level by level, y_e = L_e^-1 g_e, g_l -= U_e^T J_e y_e, g_r -= V_e^T J_e y_e;
  // then from the top level down x_e = L_e^-T J_e (y_e - U_e x_l - V_e x_r),
  // x_e overwriting g_e (J_e = I unless signed).
  std::vector<long long> strides;
  for (long long s = 1; s <= mmax; s *= 2) strides.push_back(s);
  for (int pass = 0; pass < 2; ++pass) {
    for (size_t li = 0; li < strides.size(); ++li) {
      const long long s = pass == 0 ? strides[li] : strides[strides.size() - 1 - li];
      std::vector<BmvItem> a, bb, cc;
      for (const ReducedDev& r : R) {
        const int k = (int)(r.m / s);
        if (k < 1) continue;
        live_flag = r.live;
        const int E = (k + 1) / 2, NR = k / 2;
        const long long nsq = (long long)r.n * r.n, vs = (long long)r.nrhs * r.n;
        for (int q = 0; q < E; ++q) {
          const long long e = (2 * q + 1) * s - 1;
          if (pass == 0) {
            a.push_back(item(at(r.Linv, e, nsq), at(r.ft, e, vs), nullptr, at(r.yt, e, vs), r.n,
                             r.nrhs, part(r, q)));
            if (q < NR)
              bb.push_back(item(at(r.Z, e, nsq), at(r.yt, e, vs), at(r.ft, e + s, vs),
                                at(r.ft, e + s, vs), r.n, r.nrhs, part(r, q), sg(r, e)));
            if (q >= 1)
              cc.push_back(item(at(r.Td, e, nsq), at(r.yt, e, vs), at(r.ft, e - s, vs),
                                at(r.ft, e - s, vs), r.n, r.nrhs, part(r, q - 1), sg(r, e)));
          } else {
            if (q < NR)
              a.push_back(item(at(r.Z, e, nsq), at(r.ft, e + s, vs), at(r.yt, e, vs),
                               at(r.yt, e, vs), r.n, r.nrhs, part(r, q)));
            if (q >= 1)
              bb.push_back(item(at(r.Td, e, nsq), at(r.ft, e - s, vs), at(r.yt, e, vs),
                                at(r.yt, e, vs), r.n, r.nrhs, part(r, q - 1)));
            cc.push_back(item(at(r.Linv, e, nsq), at(r.yt, e, vs), nullptr, at(r.ft, e, vs), r.n,
                              r.nrhs, part(r, q), sg(r, e)));
          }
        }
      }
      if (pass == 0) {
        plan_gemv<TR>(plan, false, true, a, (TR)1, (TR)0);    // y_e = L^-1 g_e
        plan_gemv<TR>(plan, true, false, bb, (TR)-1, (TR)1);  // g_r -= V^T J y_e
        plan_gemv<TR>(plan, true, false, cc, (TR)-1, (TR)1);  // g_l -= U^T J y_e
      } else {
        plan_gemv<TR>(plan, false, false, a, (TR)-1, (TR)1);  // y_e -= V x_r
        plan_gemv<TR>(plan, false, false, bb, (TR)-1, (TR)1); // y_e -= U x_l
        plan_gemv<TR>(plan, true, true, cc, (TR)1, (TR)0);    // x_e = L^-T J y_e
      }
    }
  }
}

template <typename T, typename TR, int BP>
static void plan_sweep(Plan& plan, const std::vector<SolveDev>& probs, size_t pd, bool trans,
                       int mode) {
  constexpr int NC = SLAB_SWEEP_THREADS / BP;
  std::vector<int> c;
  for (const SolveDev& d : probs) c.push_back(d.m * ((d.nrhs + NC - 1) / NC));
  long long tot;
  const size_t oo = plan.add_offsets(c, &tot);
  const int count = (int)probs.size();
  plan.step([=](const char* dev, hipStream_t st) {
    const SolveDev* P = dev_at<SolveDev>(dev, pd);
    const int* of = dev_at<int>(dev, oo);
    if (mode == 0) {
      if (trans) hipLaunchKernelGGL((k_sweep<T, TR, BP, true, 0>), dim3((unsigned)tot), dim3(SLAB_SWEEP_THREADS), 0, st, P, of, count);
      else hipLaunchKernelGGL((k_sweep<T, TR, BP, false, 0>), dim3((unsigned)tot), dim3(SLAB_SWEEP_THREADS), 0, st, P, of, count);
    } else {
      if (trans) hipLaunchKernelGGL((k_sweep<T, TR, BP, true, 1>), dim3((unsigned)tot), dim3(SLAB_SWEEP_THREADS), 0, st, P, of, count);
      else hipLaunchKernelGGL((k_sweep<T, TR, BP, false, 1>), dim3((unsigned)tot), dim3(SLAB_SWEEP_THREADS), 0, st, P, of, count);
    }
    SLAB_LAUNCH_CHECK();
    return SLAB_OK;
  });
}

// Elementwise steps of the refined reduced solve, m * nrhs * n entries per
// problem in its own workgroups of a grouped launch:
//   MODE 0: u64 = x      MODE 1: u64 += x      (x = the TR solve in ft)
//   MODE 2: ft = (TR) r64
template <typename TR, int MODE>
__global__ void k_red_step(const ReducedDev* __restrict__ R, const int* __restrict__ offs,
                           int count) {
  const int itm = group_item(offs, count, blockIdx.x);
  const long long nwg = offs[itm + 1] - offs[itm];
  const ReducedDev& d = R[itm];
  if (item_done(d.live)) return;
  const long long tot = (long long)d.m * d.nrhs * d.n;
  g_t<TR>* __restrict__ ft = gp((TR*)d.ft);
  g_t<double>* __restrict__ u64 = gp(d.u64);
  const g_t<const double>* __restrict__ r64 = gp((const double*)d.r64);
  for (long long e = (blockIdx.x - offs[itm]) * (long long)blockDim.x + threadIdx.x; e < tot;
       e += nwg * blockDim.x) {
    if (MODE == 0) u64[e] = (double)ft[e];
    else if (MODE == 1) u64[e] += (double)ft[e];
    else ft[e] = (TR)r64[e];
  }
}

// Reduced solve refined against the FP64 reduced matrix (mixed precision):
// u = T~^-1 f~ with the TR factorization, then `steps` times
//   r = f~ - T u  (FP64, T block tridiagonal from T64 / O64),  u += T~^-1 r.
// Each step multiplies the error by about the relative accuracy of the TR
// factorization, so the interface values reach FP64 accuracy without
// repeating the slab sweeps.  The result is left in u64.
template <typename TR>
static void plan_reduced_refined(Plan& plan, const std::vector<ReducedDev>& R, bool odd_even,
                                 int steps) {
  std::vector<int> cw;
  for (const ReducedDev& r : R) cw.push_back((int)item_wgs((long long)r.m * r.nrhs * r.n));
  long long tw;
  const size_t ow = plan.add_offsets(cw, &tw), orr = plan.add_vec(R);
  const int count = (int)R.size();
  auto elementwise = [&](int mode) {
    plan.step([=](const char* dev, hipStream_t st) {
      const ReducedDev* P = dev_at<ReducedDev>(dev, orr);
      const int* of = dev_at<int>(dev, ow);
      if (mode == 0) hipLaunchKernelGGL((k_red_step<TR, 0>), dim3((unsigned)tw), dim3(256), 0, st, P, of, count);
      else if (mode == 1) hipLaunchKernelGGL((k_red_step<TR, 1>), dim3((unsigned)tw), dim3(256), 0, st, P, of, count);
      else hipLaunchKernelGGL((k_red_step<TR, 2>), dim3((unsigned)tw), dim3(256), 0, st, P, of, count);
      SLAB_LAUNCH_CHECK();
      return SLAB_OK;
    });
  };
  const int* live_flag = nullptr;
  auto item = [&live_flag](const void* M, const void* x, const void* xin, void* y, int n,
                           int nrhs) {
    BmvItem b;
    b.M = M; b.x = x; b.xin = xin; b.y = y; b.n = n; b.nrhs = nrhs; b.part = nullptr;
    b.live = live_flag;
    return b;
  };
  plan_reduced<TR>(plan, R, odd_even);
  elementwise(0);
  for (int it = 0; it < steps; ++it) {
    // r_j = g_j - T_jj u_j - T_{j,j+1} u_{j+1} - T_{j-1,j}^T u_{j-1}
    std::vector<BmvItem> dg, up, lo;
    for (const ReducedDev& r : R) {
      const long long nsq = (long long)r.n * r.n, vs = (long long)r.nrhs * r.n;
      live_flag = r.live;
      for (int j = 0; j < r.m; ++j) {
        dg.push_back(item(r.T64 + j * nsq, r.u64 + j * vs, r.g64 + j * vs, r.r64 + j * vs, r.n,
                          r.nrhs));
        if (j + 1 < r.m)
          up.push_back(item(r.O64 + j * nsq, r.u64 + (j + 1) * vs, r.r64 + j * vs,
                            r.r64 + j * vs, r.n, r.nrhs));
        if (j >= 1)
          lo.push_back(item(r.O64 + (j - 1) * nsq, r.u64 + (j - 1) * vs, r.r64 + j * vs,
                            r.r64 + j * vs, r.n, r.nrhs));
      }
    }
    // T_jj is stored in full and exactly symmetric (its upper part is written
    // from the lower one), so it is read as T_jj^T: the transposed product
    // streams the block along its rows and measured faster
    plan_gemv<double>(plan, true, false, dg, -1.0, 1.0);
    plan_gemv<double>(plan, false, false, up, -1.0, 1.0);
    plan_gemv<double>(plan, true, false, lo, -1.0, 1.0);
    elementwise(2);
    plan_reduced<TR>(plan, R, odd_even);
    elementwise(1);
  }
}

template <typename T, typename TR>
void plan_solve_pass(Plan& plan, const std::vector<SolveDev>& probs,
                     const std::vector<ReducedDev>& red, bool trans, bool odd_even,
                     bool rhs_only) {
  if (probs.empty()) return;
  // problems split by padded block order for the sweeps
  std::vector<SolveDev> cls[3];
  for (const SolveDev& d : probs) {
    const int bp = padded_block(d.b);
    cls[bp == 16 ? 0 : (bp == 32 ? 1 : 2)].push_back(d);
  }
  size_t pcls[3] = {0, 0, 0};
  for (int k = 0; k < 3; ++k)
    if (!cls[k].empty()) pcls[k] = plan.add_vec(cls[k]);
  const size_t pall = plan.add_vec(probs);
  const int count = (int)probs.size();
  std::vector<int> cw;
  for (const SolveDev& d : probs) cw.push_back((int)item_wgs((long long)d.m * d.nrhs * d.n2));
  long long tw;
  const size_t ow = plan.add_offsets(cw, &tw);
  auto sweeps = [&](int mode) {
    for (int k = 0; k < 3; ++k) {
      if (cls[k].empty()) continue;
      if (k == 0) plan_sweep<T, TR, 16>(plan, cls[k], pcls[k], trans, mode);
      else if (k == 1) plan_sweep<T, TR, 32>(plan, cls[k], pcls[k], trans, mode);
      else plan_sweep<T, TR, 64>(plan, cls[k], pcls[k], trans, mode);
    }
  };
  // (i) reduced right-hand side
  sweeps(0);
  plan.step([=](const char* dev, hipStream_t st) {
    hipLaunchKernelGGL((k_reduced_rhs<T, TR>), dim3((unsigned)tw), dim3(256), 0, st,
                       dev_at<SolveDev>(dev, pall), dev_at<int>(dev, ow), count);
    SLAB_LAUNCH_CHECK();
    return SLAB_OK;
  });
  if (rhs_only) return;
  // (ii) the reduced system (refined in FP64 when the FP64 blocks are given)
  if (!red.empty() && red[0].T64) plan_reduced_refined<TR>(plan, red, odd_even, REDUCED_REFINE_STEPS);
  else plan_reduced<TR>(plan, red, odd_even);
  // (iii) interior back substitution, and the interface values
  plan.step([=](const char* dev, hipStream_t st) {
    hipLaunchKernelGGL((k_coupling<T, TR>), dim3((unsigned)tw), dim3(256), 0, st,
                       dev_at<SolveDev>(dev, pall), dev_at<int>(dev, ow), count);
    SLAB_LAUNCH_CHECK();
    return SLAB_OK;
  });
  sweeps(1);
  plan.step([=](const char* dev, hipStream_t st) {
    hipLaunchKernelGGL((k_interface_out<TR>), dim3((unsigned)tw), dim3(256), 0, st,
                       dev_at<SolveDev>(dev, pall), dev_at<int>(dev, ow), count);
    SLAB_LAUNCH_CHECK();
    return SLAB_OK;
  });
}
template void plan_solve_pass<float, float>(Plan&, const std::vector<SolveDev>&,
                                            const std::vector<ReducedDev>&, bool, bool, bool);
template void plan_solve_pass<double, double>(Plan&, const std::vector<SolveDev>&,
                                              const std::vector<ReducedDev>&, bool, bool, bool);
template void plan_solve_pass<double, float>(Plan&, const std::vector<SolveDev>&,
                                             const std::vector<ReducedDev>&, bool, bool, bool);

// ---------------------------------------------------------------------------
// Matrix-free product with the reduced matrix, T x = A_oo x - A_oe A_ee^-1 A_eo x
// (eq. (T11_detailed); the operation the paper's randomized sketches of T are
// built from, Sec. 3.3), for nrhs interface vectors x ([j][c][r], the layout of
// the reduced vectors): k_apply_rhs writes the load f = (A_eo x on the slab
// nodes next to an interface, A_oo x on the interface nodes, zero elsewhere)
// in natural order into d.r; the reduced right-hand side of f (slab sweeps +
// k_reduced_rhs) is then f_o - A_oe A_ee^-1 f_e = T x, which k_reduced_rhs
// writes to d.g64 in FP64.
// ---------------------------------------------------------------------------
__global__ void k_apply_rhs(const SolveDev* __restrict__ P, const int* __restrict__ offs,
                            int count) {
  const int itm = group_item(offs, count, blockIdx.x);
  const long long nwg = offs[itm + 1] - offs[itm];
  const SolveDev& d = P[itm];
  const int n1 = d.n1, n2 = d.n2, b = d.b, m = d.m, nrhs = d.nrhs;
  const long long N = (long long)n1 * n2;
  const g_t<const double>* __restrict__ wh = gp(d.wh);
  const g_t<const double>* __restrict__ wv = gp(d.wv);
  const g_t<const double>* __restrict__ x = gp(d.u);
  g_t<double>* __restrict__ f = gp(d.r);
  auto xv = [&](long long j, long long c, long long r) -> double {
    return (j >= 0 && j < m) ? x[(j * nrhs + c) * n2 + r] : 0.0;
  };
  for (long long e = (blockIdx.x - offs[itm]) * (long long)blockDim.x + threadIdx.x;
       e < (long long)nrhs * N; e += nwg * blockDim.x) {
    const long long c = e / N, p = e % N;
    const long long col = p / n2, r = p % n2;
    const long long k = col % (b + 1), s = col / (b + 1);
    double v = 0.0;
    if (k == b) {
      // interface node of interface s: its row of A_oo (vertical edges within
      // the interface column; horizontal edges lead to slab nodes)
      const double wl = wh[col * n2 + r], wr = wh[(col + 1) * n2 + r];
      const double wd = wv[col * (n2 + 1) + r], wu = wv[col * (n2 + 1) + r + 1];
      v = (wl + wr + wd + wu + gp(d.shift)[p * d.shift_stride]) * xv(s, c, r);
      if (r > 0) v -= wd * xv(s, c, r - 1);
      if (r < n2 - 1) v -= wu * xv(s, c, r + 1);
    } else {
      // slab node: -w to the interface on its left (interface s-1) at k = 0
      // and on its right (interface s) at k = b-1
      if (k == 0) v -= wh[col * n2 + r] * xv(s - 1, c, r);
      if (k == b - 1) v -= wh[(col + 1) * n2 + r] * xv(s, c, r);
    }
    f[c * N + p] = v;
  }
}

template <typename T, typename TR>
void plan_reduced_apply(Plan& plan, const std::vector<SolveDev>& probs) {
  if (probs.empty()) return;
  std::vector<int> cw;
  for (const SolveDev& d : probs)
    cw.push_back((int)item_wgs((long long)d.nrhs * d.n1 * d.n2));
  long long tw;
  const size_t ow = plan.add_offsets(cw, &tw), pd = plan.add_vec(probs);
  const int count = (int)probs.size();
  plan.step([=](const char* dev, hipStream_t st) {
    hipLaunchKernelGGL(k_apply_rhs, dim3((unsigned)tw), dim3(256), 0, st,
                       dev_at<SolveDev>(dev, pd), dev_at<int>(dev, ow), count);
    SLAB_LAUNCH_CHECK();
    return SLAB_OK;
  });
  plan_solve_pass<T, TR>(plan, probs, {}, false, false, true);
}
template void plan_reduced_apply<float, float>(Plan&, const std::vector<SolveDev>&);
template void plan_reduced_apply<double, double>(Plan&, const std::vector<SolveDev>&);
template void plan_reduced_apply<double, float>(Plan&, const std::vector<SolveDev>&);

// ---------------------------------------------------------------------------
// Residual r = f - A u (FP64) with per-column partial sums of r^2 and f^2.
// Per problem: chunks x nrhs workgroups, partial[(c*chunks + blk)*2 + {0,1}],
// then norms[2c] = sum r^2, norms[2c+1] = sum f^2.
// ---------------------------------------------------------------------------
constexpr int RES_CHUNKS = 256;

size_t residual_partial_count(int n1, int n2, int nrhs) { return (size_t)nrhs * RES_CHUNKS * 2; }

__host__ __device__ inline int res_chunks(int n1, int n2) {
  const long long N = (long long)n1 * n2;
  const long long c = (N + 255) / 256;
  return (int)(c < RES_CHUNKS ? c : RES_CHUNKS);
}

__global__ __launch_bounds__(256) void k_residual(const SolveDev* __restrict__ P,
                                                  const int* __restrict__ offs, int count) {
  __shared__ double red[2][256];
  const int itm = group_item(offs, count, blockIdx.x);
  if (item_done(P[itm].live)) return;
  const int bx = blockIdx.x - offs[itm];
  const int n1 = P[itm].n1, n2 = P[itm].n2;
  const int chunks = res_chunks(n1, n2);
  const int c = bx / chunks, blk = bx % chunks;
  const long long ld = P[itm].ldf;
  const g_t<const double>* __restrict__ wh = gp(P[itm].wh);
  const g_t<const double>* __restrict__ wv = gp(P[itm].wv);
  const g_t<const double>* __restrict__ sh = gp(P[itm].shift);
  const long long ss = P[itm].shift_stride;
  const long long N = (long long)n1 * n2;
  const g_t<const double>* fc = gp(P[itm].f) + c * ld;
  const g_t<const double>* uc = gp(P[itm].u) + c * ld;
  g_t<double>* r = gp(P[itm].r);
  double sr = 0.0, sf = 0.0;
  for (long long p = blk * 256LL + threadIdx.x; p < N; p += (long long)chunks * 256) {
    const long long col = p / n2, row = p % n2;
    const double w_l = wh[col * n2 + row], w_r = wh[(col + 1) * n2 + row];
    const double w_d = wv[col * (n2 + 1) + row], w_u = wv[col * (n2 + 1) + row + 1];
    const double up = uc[p];
    double au = (w_l + w_r + w_d + w_u + sh[p * ss]) * up;
    if (col > 0) au -= w_l * uc[p - n2];
    if (col < n1 - 1) au -= w_r * uc[p + n2];
    if (row > 0) au -= w_d * uc[p - 1];
    if (row < n2 - 1) au -= w_u * uc[p + 1];
    const double fv = fc[p];
    const double rv = fv - au;
    if (r) r[c * N + p] = rv;
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
    g_t<double>* partial = gp(P[itm].partial);
    partial[((long long)c * chunks + blk) * 2 + 0] = red[0][0];
    partial[((long long)c * chunks + blk) * 2 + 1] = red[1][0];
  }
}

__global__ void k_norms(const SolveDev* __restrict__ P, const int* __restrict__ offs, int count) {
  const int itm = group_item(offs, count, blockIdx.x);
  const int c = (blockIdx.x - offs[itm]) * blockDim.x + threadIdx.x;
  const int nrhs = P[itm].nrhs;
  if (c >= nrhs || item_done(P[itm].live)) return;
  const int chunks = res_chunks(P[itm].n1, P[itm].n2);
  const g_t<const double>* __restrict__ partial = gp((const double*)P[itm].partial);
  double sr = 0.0, sf = 0.0;
  for (int k = 0; k < chunks; ++k) {
    sr += partial[((long long)c * chunks + k) * 2 + 0];
    sf += partial[((long long)c * chunks + k) * 2 + 1];
  }
  gp(P[itm].norms)[2 * c + 0] = sr;
  gp(P[itm].norms)[2 * c + 1] = sf;
}

// r = f - A u and the norms of every problem (r of problem i: nrhs x n1 n2,
// leading dimension n1 n2; r may be null).
void plan_residual(Plan& plan, const std::vector<SolveDev>& probs) {
  if (probs.empty()) return;
  std::vector<int> c1, c2;
  for (const SolveDev& d : probs) {
    c1.push_back(res_chunks(d.n1, d.n2) * d.nrhs);
    c2.push_back((d.nrhs + 63) / 64);
  }
  long long t1, t2;
  const size_t pd = plan.add_vec(probs);
  const size_t o1 = plan.add_offsets(c1, &t1), o2 = plan.add_offsets(c2, &t2);
  const int count = (int)probs.size();
  plan.step([=](const char* dev, hipStream_t st) {
    hipLaunchKernelGGL(k_residual, dim3((unsigned)t1), dim3(256), 0, st,
                       dev_at<SolveDev>(dev, pd), dev_at<int>(dev, o1), count);
    SLAB_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_norms, dim3((unsigned)t2), dim3(64), 0, st, dev_at<SolveDev>(dev, pd),
                       dev_at<int>(dev, o2), count);
    SLAB_LAUNCH_CHECK();
    return SLAB_OK;
  });
}

// ---------------------------------------------------------------------------
// Convergence test on the device, for passes issued without a host
// synchronization in between: after the residual norms of a pass, the pass
// count and the max-over-columns relative residual of every live problem are
// updated, and the problem stays live while relres > tol and passes remain
// (a non-finite residual, or one above 1 that grew, stops it, like the host
// test).  One thread per problem.
// ---------------------------------------------------------------------------
__global__ void k_converge(const ConvDev* __restrict__ C, int count, int first) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const ConvDev& c = C[i];
  if (first) {
    *c.iters = 0;
    if (c.fstatus)
      for (int k = 0; k < 4; ++k) c.fstatus_out[k] = c.fstatus[k];
  } else if (*c.live == 0) {
    return;
  }
  double worst = 0.0;
  bool finite = true;
  for (int k = 0; k < c.nrhs; ++k) {
    const double rn = sqrt(c.norms[2 * k]), fn = sqrt(c.norms[2 * k + 1]);
    const double v = fn > 0.0 ? rn / fn : rn;
    if (!isfinite(v)) finite = false;
    else worst = fmax(worst, v);
  }
  if (!finite) worst = NAN;
  const int it = *c.iters + 1;
  // a residual above the right-hand side that grew since the last pass: the
  // refinement diverges (stopped, like the host test)
  const bool diverged = it >= 2 && worst > 1.0 && worst > *c.relres;
  *c.iters = it;
  *c.relres = worst;
  *c.live = (worst > c.tol && it < c.max_iter && !diverged) ? 1 : 0;
}

void plan_converge(Plan& plan, const std::vector<ConvDev>& conv, bool first) {
  if (conv.empty()) return;
  const size_t pc = plan.add_vec(conv);
  const int count = (int)conv.size();
  plan.step([=](const char* dev, hipStream_t st) {
    hipLaunchKernelGGL(k_converge, dim3((unsigned)((count + 63) / 64)), dim3(64), 0, st,
                       dev_at<ConvDev>(dev, pc), count, first ? 1 : 0);
    SLAB_LAUNCH_CHECK();
    return SLAB_OK;
  });
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

// Load of Dirichlet data g on the ring (eq. (bvp)) into the right-hand side of
// eq. (Au=f): f_p += sum over the edges from p to a ring node q of w_e g_q.
// One thread per interior node next to the ring, each node once: the n2 nodes
// of the first and of the last column, then the nodes of the bottom and top
// rows of the columns between them.  The terms are added left, right, below,
// above, then to f.
__global__ void k_dirichlet(int n1, int n2, int nrhs, long long ld, const double* __restrict__ wh,
                            const double* __restrict__ wv, const double* __restrict__ g,
                            double* __restrict__ f) {
  const int nc = min(n1, 2), nr = min(n2, 2);
  const long long per = (long long)nc * n2 + (long long)max(n1 - 2, 0) * nr;
  const long long gs = (long long)(n1 + 2) * (n2 + 2);
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < per * nrhs;
       e += (long long)gridDim.x * blockDim.x) {
    const long long k = e / per, q = e % per;
    int c, r;
    if (q < (long long)nc * n2) {
      c = q < n2 ? 0 : n1 - 1;
      r = (int)(q % n2);
    } else {
      const long long q2 = q - (long long)nc * n2;
      c = 1 + (int)(q2 / nr);
      r = (q2 % nr == 0) ? 0 : n2 - 1;
    }
    const double* gk = g + k * gs;
    // every product and sum rounded on its own (no fused multiply-add), so the
    // load is the same to the bit whatever the compiler contracts
    double add = 0.0;
    if (c == 0) add = __dadd_rn(add, __dmul_rn(wh[r], gk[r + 1]));
    if (c == n1 - 1)
      add = __dadd_rn(add, __dmul_rn(wh[(long long)n1 * n2 + r],
                                     gk[(long long)(n1 + 1) * (n2 + 2) + r + 1]));
    if (r == 0)
      add = __dadd_rn(add, __dmul_rn(wv[(long long)c * (n2 + 1)], gk[(long long)(c + 1) * (n2 + 2)]));
    if (r == n2 - 1)
      add = __dadd_rn(add, __dmul_rn(wv[(long long)c * (n2 + 1) + n2],
                                     gk[(long long)(c + 1) * (n2 + 2) + n2 + 1]));
    double* fp = f + k * ld + (long long)c * n2 + r;
    *fp = __dadd_rn(*fp, add);
  }
}

int launch_dirichlet(int n1, int n2, int nrhs, long long ld, const double* wh, const double* wv,
                     const double* g, double* f, hipStream_t st) {
  const long long per = (long long)std::min(n1, 2) * n2 + (long long)std::max(n1 - 2, 0) * std::min(n2, 2);
  const unsigned grid = (unsigned)std::min<long long>((per * nrhs + 255) / 256, 4096);
  hipLaunchKernelGGL(k_dirichlet, dim3(grid), dim3(256), 0, st, n1, n2, nrhs, ld, wh, wv, g, f);
  SLAB_LAUNCH_CHECK();
  return SLAB_OK;
}

}  // namespace slab
