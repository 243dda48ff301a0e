/*
 * slab.h -- C ABI of the MI355X slab solver (SlabLU hot path, dense-T variant).
 *
 * Solves A u = f (paper Sec. 1.1, eq. (Au=f)) for the 5-point discretization of
 * -div(kappa grad u) = f on a uniform grid of n2 rows x n1 columns of interior
 * nodes with homogeneous Dirichlet data on the ring around them (Sec. 2.1, eq.
 * (discretization), generalised to a variable coefficient with the edge weight
 * w_e = (kappa_p + kappa_q) / (2 h^2)).  The grid is cut into slabs of b
 * interior columns separated by one-column interfaces (Sec. 2.2, Fig. 1): in
 * every period of b+1 columns the first b columns are a slab interior and the
 * last is an interface, so there are m = n1/(b+1) slabs and m interfaces.
 *
 *   slab_factor         Alg. 3: eliminate every slab interior (stage one,
 *                       Sec. 3.1) and factor the block-tridiagonal reduced
 *                       matrix T of n2 x n2 dense blocks (stage two, Alg. 1
 *                       or the odd-even order of the Sec. 4 remark).
 *   slab_solve          Alg. 4: reduced right-hand side (eqs. (f1)-(f5)), the
 *                       sweeping solve (Alg. 2) and the interior back
 *                       substitution (eq. (usol_even)); in mixed precision
 *                       wrapped in FP64 iterative refinement.
 *   slab_solve_adjoint  A^T lambda = g from the same stored factors, applied
 *                       transposed.
 *   slab_free           release a handle.
 *
 * Conventions shared by every entry point:
 *   Layout   Vectors are stored in natural order, row index r fastest: entry
 *            (k, c, r) of right-hand side k at column c, row r is at offset
 *            k*ld + c*n2 + r with ld >= n1*n2 (torch shape (nrhs, n1, n2)).
 *            The coefficient field covers the ring too: shape (n1+2, n2+2),
 *            node (c, r) at (c+1)*(n2+2) + (r+1).
 *   Memory   Pointers to vectors and fields are DEVICE pointers on the current
 *            HIP device, owned by the caller and left untouched after the call
 *            returns.  The handle owns every factor it allocates.
 *   Streams  Work is issued on the given hipStream_t (NULL = default stream).
 *            Every call returns only after its work has finished, because it
 *            reports breakdown and convergence.
 *   Errors   Every call returns a status; nothing throws across the ABI.  On
 *            failure outputs are unspecified, the handle (if any) stays valid,
 *            and slab_last_error() describes the failure (thread-local).
 *            Argument checks run on the host before any HIP call.
 *   Threads  A handle may be used by one thread / stream at a time.
 */
#ifndef SLAB_H_
#define SLAB_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct slab_handle_s* slab_handle;
typedef struct slab_batch_s* slab_batch;

/* status codes */
#define SLAB_OK 0
#define SLAB_E_INVALID (-1)   /* bad argument: sizes, null pointer, kappa <= 0 or non-finite */
#define SLAB_E_NOMEM (-2)     /* device allocation failed */
#define SLAB_E_BREAKDOWN (-3) /* zero, negative or non-finite pivot (matrix not SPD) */
#define SLAB_E_NOCONV (-4)    /* refinement did not reach tol within max_iter */
#define SLAB_E_HIP (-5)       /* a HIP runtime call failed */

/* precision of the factorization */
#define SLAB_FP64 0          /* every phase in FP64 */
#define SLAB_FP32_REFINE 1   /* slab factors, T blocks and the block factorization in FP32;
                                FP64 sum forming T, FP64 residual and update */
#define SLAB_MIXED 2         /* slab factors, Schur formation and slab sweeps in FP64; the
                                reduced system (T blocks, block factorization, Alg. 2) in
                                FP32; FP64 residual and update */

/* option flags */
#define SLAB_KEEP_REDUCED 1  /* keep FP64 copies of T and of every S_j (Alg. 1) for export */
#define SLAB_COEF_LOG 2      /* the field passed is theta = log(kappa), not kappa */
#define SLAB_ODD_EVEN 4      /* stage two in odd-even order (Sec. 4 remark, concluding
                                section): at every level the interfaces at even
                                positions of those left are eliminated together, so
                                a level is one batch of independent block
                                factorizations; without it, the sweep of Alg. 1 */
#define SLAB_GRAPH 8         /* batched solves: capture all refinement passes of the
                                batch as one HIP graph on first use and replay it */

typedef struct {
  int32_t n1;          /* interior columns (slab direction); n1 % (b+1) == 0, n1 >= 2 */
  int32_t n2;          /* interior rows = interface length n; 1 <= n2 */
  int32_t b;           /* interior columns per slab; 1 <= b <= 63, or 0: chosen by
                          slab_autotune (then n1 must be a multiple of 4) */
  double h;            /* grid spacing, > 0 */
  const double* kappa; /* device, (n1+2)*(n2+2) FP64, r fastest; > 0 and finite
                          (or theta = log kappa, finite, with SLAB_COEF_LOG) */
  const double* shift; /* device, n1*n2 FP64 (node (c, r) at c*n2 + r), finite, or NULL:
                          a diagonal term c_p added to A, (A u)_p += c_p u_p.  With
                          c = -k^2 b(x) it is the Helmholtz term of eq. (var_helm)
                          (wavenumber k; the paper writes kappa for it).  A shift
                          may make A indefinite: with one, both stages eliminate
                          with pivots of either sign and no pivoting (the slab
                          blocks by 2 x 2 pivot blocks, the pivot blocks of the
                          reduced matrix T in signed form L J L^T).  A zero pivot
                          is SLAB_E_BREAKDOWN; growth from small ones shows as a
                          refinement that does not converge (SLAB_E_NOCONV).  Read
                          during slab_factor (and again by slab_batch_run). */
} slab_problem;

typedef struct {
  int32_t precision;   /* SLAB_FP64, SLAB_FP32_REFINE or SLAB_MIXED */
  double tol;          /* target max-over-columns ||f - A u||_2 / ||f||_2 (e.g. 1e-10) */
  int32_t max_iter;    /* refinement iterations allowed (>= 1; FP64 uses at most this too) */
  int32_t flags;       /* SLAB_KEEP_REDUCED | SLAB_COEF_LOG | SLAB_ODD_EVEN | SLAB_GRAPH */
  int32_t tile;        /* output tile of the FP32 block products of stage two: 64 or 128,
                          or 0 = automatic (128 once a launch has enough tiles for four
                          per compute unit, else 64; for a problem given with b = 0 the
                          width the autotuner measured fastest for its block size).
                          Ignored in FP64. */
} slab_options;

typedef struct {
  int32_t iterations;  /* solve passes performed */
  double max_relres;   /* max over columns of the final relative residual (FP64) */
  int32_t failed_block;/* factor: block index of a breakdown, else -1 */
} slab_solve_info;

/* Host-only check of the problem description and options (no HIP call).
   Returns SLAB_OK or SLAB_E_INVALID. */
int slab_check_problem(const slab_problem* prob, const slab_options* opts);

/* Alg. 3 (factor).  prob->kappa and prob->shift are read during the call only.  On success
   *out receives a new handle.  SLAB_E_INVALID for bad sizes or a coefficient
   that is not positive and finite; SLAB_E_BREAKDOWN if a pivot block is not
   positive definite (its interface index is in info->failed_block when info is
   not NULL). */
int slab_factor(const slab_problem* prob, const slab_options* opts, void* hip_stream,
                slab_handle* out, slab_solve_info* info);

/* Alg. 4 (solve) for nrhs right-hand sides f -> u (device FP64, natural order,
   leading dimension ld).  f and u must not overlap.  Mixed precision refines
   until the max relative residual is <= tol (else SLAB_E_NOCONV, u holds the
   last iterate); FP64 refines only while above tol.  info may be NULL. */
int slab_solve(slab_handle h, const double* f, double* u, int32_t nrhs, int64_t ld,
               void* hip_stream, slab_solve_info* info);

/* A^T lambda = g with the stored factors applied transposed (transposed slab
   sweeps, transposed block-tridiagonal sweep).  Same conventions as slab_solve. */
int slab_solve_adjoint(slab_handle h, const double* g, double* lam, int32_t nrhs, int64_t ld,
                       void* hip_stream, slab_solve_info* info);

/* Release the handle and its device memory (NULL is a no-op). */
int slab_free(slab_handle h);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, serving loops, harnesses that forbid hipMalloc): slab_solve with
   every solve buffer and plan table placed in one device array of the
   library, SLAB_NOALLOC_SCRATCH_BYTES long, instead of memory the library
   allocates.  Same arguments, result and conventions as slab_solve; the
   handle must come from slab_factor or slab_batch_handle.  It calls no
   hipMalloc, hipFree or other allocating routine.  Each GPU the library runs
   on holds its own copy of the array until the process ends; its address is
   looked up once per device, on the first call there.
   SLAB_E_INVALID (before any device work) when the solve buffers for this
   problem and nrhs need more than SLAB_NOALLOC_SCRATCH_BYTES - 1 MiB (in
   FP64 about 8 * nrhs * n1 * n2 * (2 + BP/(b+1)) bytes, BP = b rounded up to
   16, 32 or 64; the message states the size needed), or a pass's plan tables
   more than the 1 MiB kept for them.  Every call on one GPU shares
   its array: calls that overlap in time on one GPU (two host threads, or two
   streams) race and give wrong results.  No buffer of the array needs to
   start at zero; a call leaves its last contents behind. */
#define SLAB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int slab_solve_noalloc(slab_handle h, const double* f, double* u, int32_t nrhs, int64_t ld,
                       void* hip_stream, slab_solve_info* info);

/* ---- batches of independent problems ------------------------------------- */

/* Alg. 3 for `count` independent problems of any sizes and slab widths, all
   with the same options, in one set of grouped launches: every phase of stage
   one is one launch over all (problem, slab, column chunk) work units of a
   padded block order, and stage two advances all problems together (one
   launch per panel step and update product over every pivot block of every
   problem).  probs is a HOST array; each kappa is a device pointer read during
   the call only.  On failure no batch is returned and the message names the
   problem.  infos (host, count entries) may be NULL. */
int slab_factor_batch(const slab_problem* probs, int32_t count, const slab_options* opts,
                      void* hip_stream, slab_batch* out, slab_solve_info* infos);

/* Alg. 4 with refinement for every problem of the batch: f[i], u[i] (host
   arrays of device pointers), nrhs[i] and ld[i] (host arrays) as in
   slab_solve.  Every refinement pass of the batch is one set of grouped
   launches; a problem drops out once its residual meets tol.  With SLAB_GRAPH
   all max_iter passes are captured as ONE HIP graph the first time and
   replayed while the arguments stay the same (the graph and its tables live
   until slab_batch_free): each pass ends with a convergence test on the
   device, later passes skip the work of problems that have met tol, and the
   host synchronizes once.  SLAB_E_NOCONV if any problem misses tol. */
int slab_solve_batch(slab_batch bt, const double* const* f, double* const* u, const int32_t* nrhs,
                     const int64_t* ld, void* hip_stream, slab_solve_info* infos);

/* Factor every problem of the batch again from new coefficient fields kappa[i]
   (device, same shapes and options as at slab_factor_batch) and solve
   f[i] -> u[i] (arguments as in slab_solve_batch), as ONE HIP graph launch:
   Alg. 3 for all problems, then max_iter passes of Alg. 4 with FP64
   refinement, each followed by a convergence test on the device; a problem
   that has met tol skips the work of the later passes on the device, and the
   host synchronizes once, at the end.  The graph is captured on the first
   call and replayed while kappa, f, u, nrhs and ld are the same pointers and
   values (write new data into the same buffers to reuse it); it and the
   factorization temporaries it uses live until slab_batch_free.  The batch's
   handles then hold the new factors.  Failures are reported as by
   slab_factor_batch (SLAB_E_INVALID for an invalid field, SLAB_E_BREAKDOWN)
   and slab_solve_batch (SLAB_E_NOCONV); phase times (slab_batch_query) are
   not updated. */
int slab_batch_run(slab_batch bt, const double* const* kappa, const double* const* f,
                   double* const* u, const int32_t* nrhs, const int64_t* ld, void* hip_stream,
                   slab_solve_info* infos);

/* A^T lambda_i = g_i for every problem of the batch with its stored factors
   applied transposed (as slab_solve_adjoint), in the grouped launches of
   slab_solve_batch; arguments and SLAB_GRAPH behaviour as there. */
int slab_solve_adjoint_batch(slab_batch bt, const double* const* g, double* const* lam,
                             const int32_t* nrhs, const int64_t* ld, void* hip_stream,
                             slab_solve_info* infos);

/* slab_kappa_grad for every problem of the batch: u[i], lam[i], grad[i] are
   device pointers (host arrays of them), nrhs[i] and ld[i] as in
   slab_kappa_grad, the same mode for all.  Synchronizes once at the end. */
int slab_kappa_grad_batch(slab_batch bt, const double* const* u, const double* const* lam,
                          const int32_t* nrhs, const int64_t* ld, int32_t mode,
                          double* const* grad, void* hip_stream);

/* Handle of problem i of the batch (owned by the batch: do not free it).
   slab_solve, slab_solve_adjoint, slab_kappa_grad, slab_residual,
   slab_export_reduced and slab_query work on it as on any handle. */
int slab_batch_handle(slab_batch bt, int32_t i, slab_handle* out);

/* what = 0 number of problems, 5 device bytes held, 10+p phase times (as in
   slab_query) of the batched factorization. */
int slab_batch_query(slab_batch bt, int32_t what, int64_t* value);

/* Release the batch and all of its problems (NULL is a no-op). */
int slab_batch_free(slab_batch bt);

/* ---- auxiliary entry points ---------------------------------------------- */

/* Index maps of the clustering (Sec. 2.2): device int32 col_kind[n1] (1 for an
   interface column), slab_of_col[n1] = c/(b+1), local_of_col[n1] = c%(b+1),
   int64 perm_even[m*n2*b] (slab s, local r*b+k -> natural (s(b+1)+k)*n2 + r),
   perm_odd[m*n2] (interface j, row r -> natural (j(b+1)+b)*n2 + r).
   Any output pointer may be NULL to skip it. */
int slab_index_maps(int32_t n1, int32_t n2, int32_t b, int32_t* col_kind, int32_t* slab_of_col,
                    int32_t* local_of_col, int64_t* perm_even, int64_t* perm_odd, void* hip_stream);

/* Gradient of a loss L(u) with respect to the coefficient, given u = A^-1 f and
   lam = A^-T dL/du (nrhs columns each, summed): dL/dw_e = -(lam_p - lam_q)(u_p - u_q)
   on every edge (ring values zero), dw_e/dkappa_p = 1/(2h^2).  mode 0 writes
   dL/dkappa, mode 1 writes dL/dtheta = kappa dL/dkappa, on the (n1+2)*(n2+2)
   field (device FP64). */
int slab_kappa_grad(slab_handle h, const double* u, const double* lam, int32_t nrhs, int64_t ld,
                    int32_t mode, double* grad, void* hip_stream);

/* Load of Dirichlet boundary data (eq. (bvp): u = g on the boundary) moved to
   the right-hand side of eq. (Au=f): for every edge e between an interior node
   p and a ring node q, f_p += w_e g_q, with the edge weights of the factored
   handle (those of its kappa and h).  g: device FP64, nrhs fields of
   (n1+2)*(n2+2) in the layout of kappa (node (i, j) at i*(n2+2) + j; only the
   ring, i = 0 or n1+1 or j = 0 or n2+1, is read).  f: device FP64, nrhs
   columns of n1*n2 at stride ld >= n1*n2, updated in place (holding a source
   term, or zero).  Asynchronous on hip_stream; g and f owned by the caller. */
int slab_dirichlet_load(slab_handle h, const double* g, double* f, int32_t nrhs, int64_t ld,
                        void* hip_stream);

/* Per-column relative residual ||f - A u||_2/||f||_2 in FP64 (relerr_res of
   Sec. 5.1); relres is a HOST array of nrhs doubles. */
int slab_residual(slab_handle h, const double* f, const double* u, int32_t nrhs, int64_t ld,
                  double* relres, void* hip_stream);

/* Matrix-free product with the reduced matrix of a factored problem,
   y = T x = A_oo x - A_oe A_ee^-1 A_eo x (Sec. 3.1, eq. (T11_detailed)), for
   ncols interface vectors: the operation the paper's randomized sketches of T
   are formed from (Alg. 3, Sec. 3.3: T applied to Gaussian test vectors
   through the slab solves, never formed).  x and y are device FP64 arrays of
   m * ncols * n2 entries, block j of column k at (j * ncols + k) * n2 (rows r
   fastest), owned by the caller and not overlapping.  A_ee^-1 is applied with
   the stored slab factors (two slab sweeps per slab, FP64 except in
   SLAB_FP32_REFINE, where they are FP32); A_oo and A_eo come from the edge
   weights.  Uses the handle's solve workspace (grown for ncols columns). */
int slab_apply_reduced(slab_handle h, const double* x, double* y, int32_t ncols, void* hip_stream);

/* Export a reduced block as FP64 n2 x n2 row-major into device memory out:
   which = 0: T_jj, 1: T_{j,j+1} (j < m-1), 2: the pivot block of interface j
   before its factorization (S_j of Alg. 1, or with SLAB_ODD_EVEN the block of
   the Schur complement left at the level where j is eliminated).  Needs
   SLAB_KEEP_REDUCED at factor time. */
int slab_export_reduced(slab_handle h, int32_t which, int32_t j, double* out, void* hip_stream);

/* Sizes and timings of a handle: what = 0 m, 1 n1, 2 n2, 3 b, 4 precision,
   5 device bytes held, 6 the FP32 product tile in use (0: automatic),
   7 the number of negative pivots of the signed block factorization of T
   (problems with a shift; 0 otherwise), which is the number of negative
   eigenvalues of T (Sylvester's law of inertia): those of A less those of the
   slab interiors (synchronous: copies the pivot signs to the host),
   8 the device address of the stored block inverses Gl_r of the slab
   factor (Alg. 3, first loop) that every slab sweep reads: m*n2 blocks of
   BP x BP row-major elements, BP = b rounded up to 16, 32 or 64, block (s, r)
   of slab s and row r at element (s*n2 + r)*BP*BP, FP64 (FP32 in
   SLAB_FP32_REFINE); owned by the handle, for inspection (a caller that
   writes them changes every later solve of the handle),
   10+p elapsed microseconds of factor phase p of the last
   factorization (0 slab factors, 1 boundary columns of the slab inverses,
   2 Schur propagation, 3 assembly of T, 4 block factorization of T, 5 the
   block products inside 4: the sum over their launches), measured with HIP
   events on the factor's stream; 20+k the number of kernel launches of kind k
   issued for this handle so far (factorization and every solve pass):
   k = 0 block products on 128-wide tiles, 1 block products on 64-wide tiles,
   2 factorization updates with the C tile prefetched, 3 block-vector products
   split over k (with the launch that adds the partial sums), 4 block-vector
   products in one launch. */
int slab_query(slab_handle h, int32_t what, int64_t* value);

/* Slab width for the grid of *prob (prob->b is ignored), chosen by measurement.
   The cost balance of Sec. 4, eq. (complexity_funcb) -- slab work growing and
   reduced-system work shrinking with b -- predicts each candidate
   b in {3, 7, 15, 31, 63} with n1 % (b+1) == 0 at half the nominal
   peaks plus the row-by-row latency of the slab recursion; candidates predicted
   more than 3x slower than the best are skipped, and the others are factored
   (with *opts) and solved for nrhs pseudo-random right-hand sides (uniform in
   [-1, 1), fixed seed) on the device from
   prob->kappa and timed.  The fastest converging width goes to *b_out and is
   cached per (n1, n2, precision, flags, nrhs) for the process.  For FP32
   reduced systems in odd-even order with opts->tile = 0 the FP32 product tile
   (64 or 128) of n2 x n2 blocks is timed first and cached per n2; it is used
   by the candidates timed here and by factorizations of problems given with
   b = 0 (those given with b > 0 keep the size rule).  times (optional, host, 5
   entries for b = 3, 7, 15, 31, 63) receives the seconds measured, -1 where a
   width was not tried.  slab_factor and slab_factor_batch call this for every
   problem given with b = 0. */
int slab_autotune(const slab_problem* prob, const slab_options* opts, int32_t nrhs,
                  void* hip_stream, int32_t* b_out, double* times);

/* Device memory released by handles and batches is cached by the library and
   reused by later factorizations and solves of about the same size (mapping
   fresh device memory costs more than factoring a small problem).  This call
   returns the cached, unused memory of the current device to HIP.  It waits
   for the device to be idle. */
int slab_release_cache(void);

/* Message of the last failure on this thread ("" if none). */
const char* slab_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SLAB_H_ */
