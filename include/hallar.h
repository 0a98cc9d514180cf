/*
 * hallar.h -- C ABI of the MI355X (gfx950) HALLaR hot path.
 *
 * The library solves the primal-dual SDP pair (P)/(D) of the cuHALLaR paper
 * (arXiv 2505.13719, Section 1):
 *
 *     min  C . X   s.t.  A_l . X = b_l (l = 1..m),  Tr X <= tau^2,  X PSD
 *
 * with the factorisation X = U U^T.  Each data matrix A_l (A_0 = C) is given
 * in the hybrid sparse / low-rank form of Section 3.2 (eq. HSLR-rep-body):
 * a sparse symmetric part listed by its upper-triangle entries plus low-rank
 * terms K D K^T; or, for complex phase retrieval (Section 5.4), the
 * coded-diffraction constraints applied on the fly with FFTs.
 *
 * Conventions shared by every call
 *   - Every call returns hallar_status; nothing throws or aborts across the
 *     ABI.  On failure hallar_last_error(h) (or hallar_last_error(NULL) for
 *     calls without a handle) returns a message owned by the library, valid
 *     until the next failing call on the same thread.
 *   - "device" pointers are HIP device allocations owned by the caller (for
 *     example torch tensors on cuda:0); "host" pointers are ordinary memory.
 *     The library never frees caller memory.  It copies what it keeps.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Operator calls are asynchronous on that stream unless a host scalar
 *     is returned.  A handle is not thread-safe; use one per thread.
 *   - Dense row-major layouts: element (i, c) of an n x r matrix with
 *     leading dimension ld is at [i * ld + c].
 *   - All allocation happens in hallar_create / hallar_pool_*; the operator
 *     and solve calls allocate nothing, except that a coded-diffraction
 *     instance makes the FFT plan for a column count it has not met before
 *     on first use (rocFFT may allocate then; its work buffer grows if that
 *     plan needs more) and hallar_get_solution stages its tile list.
 */
#ifndef HALLAR_H
#define HALLAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hallar_s *hallar_t;
typedef struct hallar_pool_s *hallar_pool_t;

typedef enum {
  HALLAR_OK = 0,
  HALLAR_E_INVALID = 1,        /* bad argument, shape or index (i > j, l > m, ...) */
  HALLAR_E_UNSUPPORTED = 2,    /* valid input outside what the library implements */
  HALLAR_E_OOM = 3,            /* device memory / pool budget exhausted */
  HALLAR_E_HIP = 4,            /* a HIP runtime call failed */
  HALLAR_E_NOT_CONVERGED = 5,  /* eigen solve stopped above its tolerance */
  HALLAR_E_ITER_LIMIT = 6,     /* an iteration cap of the solver was reached */
  HALLAR_E_TIME_LIMIT = 7,     /* the solve's wall-clock limit was reached */
  HALLAR_E_RANK_CAP = 8,       /* a Frank-Wolfe step needs more columns than opts.rank_cap */
  HALLAR_E_NUMERICAL = 9,      /* NaN/Inf, or the prox stepsize underflowed */
  HALLAR_E_BUSY = 10           /* pool: no free slot right now */
} hallar_status;

/* Arithmetic of the operator hot path.  FP64: everything in double.
 * FP32_MIXED: U, the sparse values and the SDDMM/SpMM/vector work in float;
 * every reduction, the multipliers, the Lanczos basis, Ritz values, the dual
 * objective, gap and infeasibility norms in double. */
typedef enum { HALLAR_FP64 = 0, HALLAR_FP32_MIXED = 1 } hallar_precision;

/* Problem descriptor (host memory, read during hallar_create only).
 * Sparse part: nnz entries (row[k], col[k], con[k], val[k]) with
 * 0 <= row[k] <= col[k] < n and 0 <= con[k] <= m, meaning
 * (A_con)_{row,col} = (A_con)_{col,row} = val (con = 0 is C).  Repeated
 * (row, col, con) triples are summed.  Low-rank part: n_lowrank terms; term t
 * adds K_t D_t K_t^T to A_{lr_con[t]}, K_t is n x lr_rank[t] row-major at
 * K + K_off[t], D_t is lr_rank[t] x lr_rank[t] row-major at D + D_off[t].
 * Supported: on the objective (lr_con = 0) at most one term of rank <= 2;
 * on the constraints any number of terms of any rank, at most 4096 columns
 * in all (the terms of one constraint are merged); others give
 * HALLAR_E_UNSUPPORTED.  A constraint with a low-rank part is summed per
 * constraint (the general mode of the index lists L_ij), and its low-rank
 * part enters A~(UU^T) as Tr(D (K^T U)(K^T U)^T) (Algorithm 3) and the
 * adjoint as K (D (K^T U)) (Algorithm 5), K^T U a dense contraction. */
typedef struct {
  int64_t n;             /* X is n x n, 1 <= n < 2^31 */
  int64_t m;             /* number of constraints A_1..A_m, 0 <= m < 2^31 */
  double trace_bound;    /* tau^2 > 0: Tr X <= tau^2, ||U||_F <= tau */
  int64_t nnz;
  const int32_t *row, *col, *con;
  const double *val;
  int32_t n_lowrank;
  const int32_t *lr_con, *lr_rank;
  const int64_t *K_off, *D_off;
  const double *K, *D;
  const double *b;       /* length m */
  /* Coded-diffraction constraints of complex phase retrieval (Section 5.4,
   * eq. phase retrieval SDP), applied on the fly with FFTs instead of being
   * stored.  cdp_patterns = L > 0 states the SDP on the real form of the
   * complex Hermitian variable: n = 2 n_c, a real column z of U stands for
   * u = z[0:n_c] + i z[n_c:n] (so Tr X = ||U||_F^2), and constraint
   * l n_c + k (0-based, l < L, k < n_c) is
   *   A_{l n_c + k} . UU^T = sum_c |(F (d_l * u_c))_k|^2,
   * F the unitary n_c-point DFT and d_l the l-th mask, complex, interleaved
   * (re, im) in cdp_masks[2 (l n_c + j) + {0, 1}] (host, L n_c pairs, read
   * during hallar_create only).  Then m = L n_c, and the problem may hold
   * only objective entries (con = 0) and no low-rank terms; otherwise
   * HALLAR_E_INVALID (shapes) or HALLAR_E_UNSUPPORTED (mixtures).
   * cdp_patterns = 0: no such constraints (cdp_masks ignored). */
  int32_t cdp_patterns;
  const double *cdp_masks;
} hallar_problem;

/* Solver constants.  hallar_default_options() fills the values the library
 * documents as its readings of the paper where the paper leaves them open. */
typedef struct {
  double eps;            /* relative tolerance of eq. termination2 (default 1e-5) */
  double beta1, beta_growth, beta_max, infeas_ratio, pinf_gate;
  double stall_ratio, stall_growth; /* ||r_t|| > stall_ratio ||r_{t-1}||: grow beta by stall_growth */
  double eps1, eps_floor, eps_decay;
  double sigma, chi, lam0;          /* ADAP-AIPP / ADAP-FISTA universal parameters */
  int32_t fista_max_iter, aipp_max_iter, hlr_max_iter, outer_max_iter;
  double eig_tol, eig_frac;         /* Lanczos: residual <= max(eig_frac eps_t / tau^2, eig_tol max(1,|lambda|)) */
  int32_t eig_kmax;                 /* Lanczos basis size before a thick restart (<= 64) */
  int32_t eig_max_iter;             /* Lanczos matvec cap per eigen solve */
  int32_t rank_cap;                 /* columns of U after a Frank-Wolfe step; 0 = none (then at most 63).
                                       A step that would exceed it first drops the directions with
                                       sigma^2 <= drop_tol sigma_max^2; if that is not enough the solve
                                       stops with HALLAR_E_RANK_CAP and returns the iterate before the
                                       step, unless rank_cap_truncate is set */
  double drop_tol;                  /* drop directions with sigma^2 <= drop_tol sigma_max^2 */
  double time_limit;                /* seconds per solve */
  uint64_t seed;                    /* Lanczos start vectors and default U0 */
  int32_t verbose;
  int32_t profile;                  /* 1: time every kernel class with HIP events (see hallar_profile);
                                       2: only the sparse classes (SDDMM, SpMM, fused trial, Lanczos
                                       SpMV), for less event overhead; 0: off */
  int32_t autotune;                 /* 1: hallar_create times candidate tile schedules on the instance and
                                       keeps the fastest (see hallar_schedule); 0: the default schedule.
                                       The schedule fixes the order of the partial sums, so results of
                                       differently tuned handles agree to rounding, not bit for bit. */
  int32_t lower_gather;             /* 1: the gradient SpMM always reads the lower half's pair values
                                       through the pair ids; 0 (default): where every strictly-lower
                                       pair is constrained with one shared coefficient and no sparse
                                       objective entry, it recomputes them from the factor rows and
                                       (p_l, b_l) kept in lower order.  Both give identical bits. */
  int32_t unfused_trial;            /* 1: a FISTA trial point runs the SDDMM and the gradient SpMM as two
                                       kernels; 0 (default): one kernel where the instance recomputes its
                                       lower half, has no low-rank objective term and narrow rows
                                       (r <= 8 in FP32-mixed, r <= 4 in FP64).  Both give identical bits. */
  int32_t obj_check;                /* 1 (default): besides the three relative errors of eq. termination2
                                       the solve stops only when |pval - dval| + |p^T (A(X) - b)| <=
                                       eps (1 + |pval|), an a-posteriori bound on the objective error (the
                                       relative gap divides by about twice the objective); 0: off */
  int32_t rank_cap_truncate;        /* 1: at the rank cap keep the cap's largest directions of Y Y^T and
                                       count each such truncation in n_truncations (X changes); 0
                                       (default): stop with HALLAR_E_RANK_CAP */
  int32_t graphs;                   /* 1: a round of kernel launches of one operation group that repeats
                                       one seen before (same operation, instances, buckets and tile
                                       ranges) is replayed as a captured HIP graph instead of being
                                       enqueued kernel by kernel; same kernels in the same order, so the
                                       same bits.  Rounds of several groups (batches, the serving pool)
                                       and rounds while opts.profile times kernel classes are enqueued
                                       directly.  0 (default): always enqueue directly */
  int32_t pad_;
} hallar_options;

void hallar_default_options(hallar_options *opts);

/* Result of a solve (all host scalars). */
typedef struct {
  int32_t status;        /* hallar_status of the solve: HALLAR_OK = converged */
  int32_t rank;          /* columns of the final U */
  int32_t outer_iters;
  int32_t pad_;
  double pval, dval;     /* C . U U^T and -b^T p - tau^2 theta */
  double theta;          /* max(-lambda, 0), lambda the smallest Ritz value of
                            C + A*(p) (an upper bound on lambda_min); once the
                            relative errors pass, rechecked by a cold-started
                            run whose Ritz value is taken if smaller */
  double pinf, gap, dinf;/* relative errors of eq. termination2 */
  double beta;           /* final penalty */
  double seconds;        /* wall-clock of the solve */
  int64_t n_sddmm, n_spmm, n_matvec, n_fista_trials, n_aipp_iters;
  int64_t n_hlr_iters, n_eig_calls, n_truncations, n_rounds;
  double obj_bound;      /* |pval - dval| + |p^T (A(X) - b)| at the last outer iteration: an
                            a-posteriori estimate of |pval - P*| (see opts.obj_check) */
  int64_t n_graph_rounds;/* rounds of n_rounds whose kernels ran as a replayed graph (opts.graphs) */
} hallar_result;

typedef struct {
  int32_t iters;         /* matrix-vector products */
  int32_t restarts;
  double residual;       /* ||G v - lambda v|| of the returned pair */
} hallar_eig_info;

/* Build a handle: dedups and sorts the entries, builds the union support S
 * (Section 4.1, eq. def: support S ell), the index lists L_ij (eq. index
 * list), the symmetric pattern S u S^T used by the adjoint (Alg. 4) and the
 * tile schedule, and copies everything to device memory (Section 3.1: the
 * problem data live on the device).  opts may be NULL (defaults).
 * Errors: E_INVALID (bad shape/index), E_UNSUPPORTED, E_OOM, E_HIP. */
hallar_status hallar_create(const hallar_problem *prob, hallar_precision prec,
                            const hallar_options *opts, void *stream, hallar_t *out);
/* The tile schedule of a handle: rows of a tile are contiguous, at least
 * *min_rows of them (more on large instances) and at most *ent_cap entries of
 * S u S^T; *ntiles tiles in all.  Segment-indexed kernels walk these tiles
 * (one workgroup per tile) and reduce their partial sums in tile order; with
 * opts.autotune the schedule is the fastest of the candidates timed on the
 * instance at create.  E_INVALID on a bad handle; NULL outputs are skipped. */
hallar_status hallar_schedule(hallar_t h, int32_t *min_rows, int32_t *ent_cap, int64_t *ntiles);

hallar_status hallar_destroy(hallar_t h);
const char *hallar_last_error(hallar_t h);

/* Sizes of the handle's structures: pairs |S|, symmetric nnz of S u S^T,
 * device bytes held. */
hallar_status hallar_describe(hallar_t h, int64_t *pairs, int64_t *sym_nnz, int64_t *device_bytes);

/* T = A~(U U^T) (Section 4, eq. A tilde operator; Algorithms 2 and 3):
 * T[0] = C . UU^T, T[l] = A_l . UU^T for l = 1..m.
 * U: device, n x r row-major with leading dimension ldu >= r, of the
 * handle's operator type (double for FP64, float for FP32_MIXED);
 * 1 <= r <= 64.  T: device double[m + 1].  Asynchronous on `stream`.
 * U is read in place when r is a column bucket of the handle (FP32: 4, 8,
 * 16, 32, 64; FP64: 2, 4, 8, ...), ldu = r and U is 16-byte aligned;
 * otherwise it is first copied into a zero-padded work buffer. */
hallar_status hallar_eval_AUUt(hallar_t h, const void *U, int32_t r, int64_t ldu, double *T, void *stream);

/* For callers that cannot allocate device memory at call time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same T = A~(U U^T) as hallar_eval_AUUt, same arguments, layouts and
 * bits, but everything the evaluation writes besides T (a copy of the
 * handle's descriptor and parameters, result scalars, per-tile partial
 * sums, the packed U when U is not used in place, low-rank products and, for
 * instances with multi-entry constraints, per-pair dot products and T, y'
 * staging) lives in one static device array of 64 MiB per GPU, held until
 * the process ends; the handle's own workspace is not touched.  The call
 * allocates nothing and returns E_INVALID if the instance needs more
 * scratch than that (about 8 bytes per partial-sum slot and tile, plus
 * n r_pad operator words when U is packed).  Every call on a GPU shares
 * that GPU's array, so calls that overlap on one GPU (different streams or
 * threads) race; calls ordered on one stream do not. */
hallar_status hallar_eval_AUUt_noalloc(hallar_t h, const void *U, int32_t r, int64_t ldu, double *T, void *stream);

/* W = A~*(1, p) U = (C + sum_l p_l A_l) U (Section 4.2, eq. Adjoint
 * calculation; Algorithms 4 and 5).  p: device double[m].  U as above; W:
 * device n x r, leading dimension ldw >= r, operator type.  Asynchronous.
 * With r a column bucket and ldu = ldw = r (16-byte aligned), U is read and
 * W written in place (no packing copy), unless the two overlap. */
hallar_status hallar_adjoint_spmm(hallar_t h, const double *p, const void *U, int32_t r, int64_t ldu,
                                  void *W, int64_t ldw, void *stream);

/* Minimum eigenpair of G = C + A*(p) by thick-restart Lanczos in FP64 with
 * full reorthogonalisation (the eigen step of Alg. 1, which the paper does not
 * specify).  p: device double[m].  v0: device double[n] start vector or NULL
 * (a seeded Gaussian).  Stops when ||G v - lambda v|| <= tol * max(1,|lambda|)
 * or after max_iter products.  lambda: host; v: device double[n], unit
 * norm.  Synchronises `stream`.  E_NOT_CONVERGED if the cap was reached
 * (lambda and v then hold the best Ritz pair). */
hallar_status hallar_min_eig(hallar_t h, const double *p, const double *v0, double tol, int32_t max_iter,
                             double *lambda, double *v, hallar_eig_info *info, void *stream);

/* Full HALLaR solve (Alg. 1 with ADAP-AIPP / ADAP-FISTA, Appendix A).
 * U0: device double n x r0 (row-major, ld = r0) or NULL (n x 1 standard
 * Gaussian from opts.seed, Section 5.1); it is projected onto ||U||_F <= tau.
 * p0: device double[m] or NULL (zeros).  Blocks until done; res: host.
 * res->status is the solve's outcome; the call itself returns HALLAR_OK
 * unless the inputs were invalid or the device failed. */
hallar_status hallar_solve(hallar_t h, const double *U0, int32_t r0, const double *p0, hallar_result *res);

/* Copy the last solve's U (device double n x rank, leading dimension
 * ldu >= rank) and p (device double[m]); either may be NULL. */
hallar_status hallar_get_solution(hallar_t h, double *U, int64_t ldu, double *p, void *stream);

/* One record per outer iteration t of the last solve on the handle (Alg. 1,
 * outer loop; the quantities of eq. termination2 after the multiplier update
 * of that iteration, and the penalty it ran with). */
typedef struct {
  int32_t t;             /* outer iteration, 1-based */
  int32_t rank;          /* columns of U after the iteration */
  double beta;           /* penalty used in the iteration */
  double pval, dval, theta;
  double pinf, gap, dinf;/* relative errors of eq. termination2 */
  double obj_bound;      /* |pval - dval| + |p^T (A(X) - b)| */
  double seconds;        /* since the solve started */
  int64_t n_fista_trials, n_matvec, n_hlr_iters; /* cumulative */
} hallar_outer_record;

/* Copy the last solve's outer-iteration records (a trace of the run) into
 * out[0 .. min(cap, total) - 1] (host); *total receives the number of
 * records (= res.outer_iters for a solve that ended inside the loop).
 * out may be NULL with cap = 0 to query the count.  Handles solved in a
 * batch keep their own records. */
hallar_status hallar_get_history(hallar_t h, hallar_outer_record *out, int32_t cap, int32_t *total);

/* Batched solve: `count` handles of the same precision solved together;
 * their operator work runs in shared, segment-indexed kernel launches (one
 * launch covers the tiles of every instance that needs that kernel).  U0s
 * may be NULL or hold per-instance device pointers (n_k x 1) or NULLs. */
hallar_status hallar_solve_batch(hallar_t *hs, int32_t count, const double *const *U0s,
                                 hallar_result *results);

/* Host-side structure of an instance (Section 4.1: the union support S and
 * the symmetric pattern S u S^T), computed without a GPU.  tile_row0, when
 * not NULL, receives the first row of each tile of the default schedule plus
 * n at the end (min(tiles + 1, cap) entries written); the schedule's tiles
 * hold at most 1024 rows and 2048 entries of S u S^T (a longer row is a tile
 * of its own), and a tile closed by the entry cap has a power-of-two row
 * count when it has 4 to 128 rows.  E_INVALID / E_UNSUPPORTED /
 * E_NUMERICAL as for hallar_create; NULL out gives E_INVALID. */
typedef struct {
  int64_t pairs;            /* |S|: upper-triangle pairs with an objective or constraint entry */
  int64_t lower;            /* strictly-lower entries of S u S^T */
  int64_t tiles;            /* tiles of the default schedule */
  int32_t direct;           /* every constraint has one pair, every pair at most one constraint */
  int32_t con_rule;         /* direct mode: 1 if exactly the off-diagonal pairs are constrained,
                               2 if exactly the diagonal ones are, 0 otherwise */
  int32_t lower_recompute;  /* every strictly-lower pair is constrained with one shared coefficient
                               and has no sparse objective entry (see opts.lower_gather) */
  int32_t pad_;
} hallar_structure;

hallar_status hallar_inspect(const hallar_problem *prob, hallar_structure *out, int64_t *tile_row0, int64_t cap);

/* ---- serving pool: continuous batching with HBM-footprint admission ---- */

/* Device bytes an instance would hold in a pool (problem data + solver
 * workspaces).  Deterministic: the pool admits by exactly this number.  Not
 * included: the FFT plans of a coded-diffraction instance and their work
 * buffer, which rocFFT sizes when the plans are made (allocated outside the
 * pool's budget, up to about the spectra of L x the column capacity). */
hallar_status hallar_footprint(const hallar_problem *prob, hallar_precision prec,
                               const hallar_options *opts, size_t *bytes);

/* A pool owns up to hbm_budget bytes of device memory and at most
 * max_active resident instances; all of them advance together, one batched
 * round per step. */
hallar_status hallar_pool_create(size_t hbm_budget, int32_t max_active, hallar_precision prec,
                                 const hallar_options *opts, void *stream, hallar_pool_t *out);
hallar_status hallar_pool_destroy(hallar_pool_t pool);

/* Try to admit one request now.  Copies the problem to the device and
 * starts its solve at the next step.  U0: host double n x 1 or NULL.
 * Returns E_OOM if its footprint does not fit in the free budget and E_BUSY
 * if max_active instances are resident; the caller retries later. */
hallar_status hallar_pool_admit(hallar_pool_t pool, const hallar_problem *prob, const double *U0,
                                int64_t ticket);

/* Advance every resident instance by up to `rounds` batched rounds (each
 * round: one host-device exchange of per-instance scalars).  Finished
 * instances release their memory at the end of the round that finishes
 * them.  n_active: host, resident instances after the step. */
hallar_status hallar_pool_step(hallar_pool_t pool, int32_t rounds, int32_t *n_active);

/* Collect up to cap finished solves (tickets and results, host arrays). */
hallar_status hallar_pool_poll(hallar_pool_t pool, int64_t *tickets, hallar_result *results, int32_t cap,
                               int32_t *n_done);

/* Bytes in use / budget of the pool. */
hallar_status hallar_pool_usage(hallar_pool_t pool, size_t *used, size_t *budget);

/* ---- profiling (opts.profile = 1) ---- */
/* Kernel classes timed with HIP events recorded on the library's stream
 * around each launch: 0 SDDMM (A~(UU^T) + AL epilogue), 1 SpMM
 * ((C + A*(y))U + epilogue), 2 Lanczos SpMV, 3 Lanczos reorthogonalisation,
 * 4 vector updates, 5 reductions, 6 other, 7 the fused FISTA trial kernel
 * (SDDMM and gradient SpMM in one row walk), 8 the coded-diffraction
 * operator (mask products, FFTs, |.|^2 sums, multiplier scaling and the
 * gather of the adjoint block; Section 5.4).  For each class: total
 * milliseconds, launches, and algorithmic bytes (every index, value and
 * constraint array read once, U read once, outputs written once).  Counters
 * accumulate since the handle/pool was created or last reset (reset != 0).
 * Arrays are host, length n_classes (<= 9). */
hallar_status hallar_profile(hallar_t h, double *ms, int64_t *launches, double *bytes, int32_t n_classes, int32_t reset);
hallar_status hallar_pool_profile(hallar_pool_t pool, double *ms, int64_t *launches, double *bytes, int32_t n_classes,
                                  int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* HALLAR_H */
