/*
 * mlmc.h -- C ABI of the MI355X (gfx950) library for multilevel Monte-Carlo
 * estimation of tr(A^{-1}) over an aggregation multigrid hierarchy.
 *
 * Method: Frommer, Nasr Khalil, Ramirez-Hidalgo, "A Multilevel Approach to
 * Variance Reduction in the Stochastic Estimation of the Trace of a Matrix"
 * (arXiv 2108.11281).  The operator A = A_1 is known only through products
 * (Sec. 3, opening paragraph); a hierarchy {A_l, P_l, R_l} with
 * A_{l+1} = R_l A_l P_l is built (Sec. 4.1); with orthonormal aggregation
 * (R_l = P_l^H, R_l P_l = I) the trace splits as in Remark 4.3:
 *   tr(A^{-1}) = sum_{l<L} [tr(A_l^{-1}) - tr(P_l A_{l+1}^{-1} R_l)] + tr(A_L^{-1}),
 * each bracket estimated from samples x^H A_l^{-1} x - (R_l x)^H A_{l+1}^{-1} (R_l x)
 * and the last term computed directly by inverting A_L (Remark 4.2).
 *
 * Conventions (all entry points):
 *  - Every function returns an int status: MLMC_OK (0) or a negative error
 *    code.  Nothing aborts and no C++ exception crosses the ABI.  After an
 *    error on a context, mlmc_last_error() describes it.
 *  - Levels are 1-based as in the paper: level 1 is the given operator.
 *  - Pointers named *_dev are device pointers on the context's device;
 *    everything else is host memory.  The caller owns every buffer it passes;
 *    the library copies what it keeps (operator data is copied at setup).
 *  - Complex vectors are interleaved (re, im) doubles; a block of nrhs vectors
 *    of length n is stored vector after vector ("RHS-major"):
 *    element i of vector k is at [k*n + i].
 *  - All work runs on the HIP stream given to mlmc_setup (NULL = default
 *    stream).  One context must not be used from two threads at once.
 *  - Sample k of level l for seed s is a pure function of (s, l, k): a
 *    Philox4x64-10 counter RNG gives the probe entries (Rademacher for real
 *    operators, Z4 for complex ones; Sec. 3, eqs. iid_components1/2).
 */
#ifndef MLMC_H
#define MLMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque context handle: the hierarchy, work buffers and solvers of one operator
 * (created by mlmc_setup, released by mlmc_destroy). */
typedef struct mlmc_ctx mlmc_ctx;

enum mlmc_status {
  MLMC_OK = 0,
  MLMC_EINVAL = -1,       /* invalid argument or descriptor */
  MLMC_ENOMEM = -2,       /* device or host allocation failed */
  MLMC_EDEVICE = -3,      /* HIP runtime error (no device, launch failure) */
  MLMC_ENOCONV = -4,      /* a solve or the estimator did not converge */
  MLMC_ESTATE = -5,       /* call not valid in the context's state */
  MLMC_EUNSUPPORTED = -6  /* combination not implemented */
};

enum mlmc_kind {
  MLMC_POISSON2D = 0,  /* A = diag*I - off*(4 grid neighbours), N x N, Dirichlet
                          (Example 4.1 with diag = 4, off = 1) */
  MLMC_WILSON2D = 1,   /* (m0+2) I - 1/2 sum_mu [(I - s_mu) U_mu(x) d_{x+mu}
                          + (I + s_mu) U_mu(x-mu)^* d_{x-mu}], 2 spins, N x N
                          periodic (Example 4.3 halved, m0 = m/2) */
  MLMC_VARCOEF3D = 2,  /* 7-point diffusion with face coefficients, N^3,
                          Dirichlet faces, plus shift*I */
  MLMC_CSR = 3,        /* a real symmetric positive definite matrix given in
                          compressed sparse row form (the algebraic operators
                          of Sec. 5, whose hierarchy an algebraic multigrid
                          method supplies): aggregates of the matrix graph
                          (given per level, or built by greedy aggregation),
                          orthonormal piecewise-constant P (entries 1/sqrt|J|),
                          Galerkin coarse operators (Sec. 4.1), multicolour
                          Gauss-Seidel smoothing over a first-fit colouring */
  MLMC_GAUGE2D = 4     /* gauge Laplacian (Example 4.2): (4 + m) I minus the
                          U(1)-linked nearest neighbours, one unknown per site,
                          N x N periodic; Hermitian; field = link phases
                          theta[2][N][N] as for WILSON2D, mass = m; hierarchy by
                          test-vector aggregation as for WILSON2D */
};

enum mlmc_precision {
  MLMC_FP64 = 0,       /* every solve in FP64 (plain FP64 MLMC) */
  MLMC_FP32_IR64 = 1   /* FP32 (complex64) Krylov + V-cycle inside FP64
                          iterative refinement; FP64 residual decides */
};

enum mlmc_alloc {
  MLMC_ALLOC_EQUAL = 0,   /* rho_l^2 = (eps tau)^2/(L-1)  (Sec. 5 default) */
  MLMC_ALLOC_WEIGHTS = 1, /* rho_l^2 = w_l (eps tau)^2, given w (Example 4.3) */
  MLMC_ALLOC_GILES = 2    /* optimal N_l ~ sqrt(V_l/C_l) (Sec. 2), V_l from the
                             samples so far, C_l = n_l + n_{l+1} */
};

/* Operator A = A_1.  Host data, copied at setup. */
typedef struct mlmc_operator {
  int kind;           /* enum mlmc_kind */
  int n_side;         /* grid / lattice side N (all directions) */
  double diag, off;   /* POISSON2D coefficients (Example 4.1: 4, 1) */
  double mass;        /* WILSON2D: m0; GAUGE2D: m */
  double shift;       /* VARCOEF3D: shift (>= 0) */
  const double* field;/* WILSON2D, GAUGE2D: link phases theta[2][N][N] (mu, y, x);
                         VARCOEF3D: face coefficients k[3][N][N][N+1]
                         (x-faces [z][y][f], y-faces [z][x][f], z-faces [y][x][f],
                          face f between cells f-1 and f); unused for POISSON2D */
  /* CSR: A (n x n) as row offsets row_ptr[0..n] (row_ptr[0] = 0), column
     indices col_idx[row_ptr[i]..row_ptr[i+1]-1] in [0, n) and their values.
     Columns may come in any order; repeated entries are summed; entries equal
     to zero are dropped.  Every row needs a positive diagonal entry; the
     matrix must be symmetric (pattern and values, to 1e-12 relative) and
     positive definite (not checked: a solve that fails to converge returns
     MLMC_ENOCONV).  n < 2^31, nnz < 2^31.  Unused by the other kinds. */
  int64_t n;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const double* vals;
} mlmc_operator;

/* A sparse matrix in compressed sparse row form (host memory): row_ptr[0..rows],
 * column indices in [0, cols) and values per entry. */
typedef struct mlmc_csr {
  int64_t rows, cols;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const double* vals;
} mlmc_csr;

/* Hierarchy description (Sec. 4.1; solver levels may exceed MLMC levels, Sec. 5). */
typedef struct mlmc_hierarchy {
  int levels_solver;  /* L_s: levels of the multigrid solver (>= 2) */
  int levels_mlmc;    /* L <= L_s: levels of the trace decomposition (>= 2) */
  int block;          /* WILSON2D: aggregate side in sites (4) */
  int n_vec;          /* WILSON2D: test vectors per aggregate (8); coarse dofs per
                         site = n_vec, or 2 n_vec with spin_split */
  int setup_sweeps;   /* WILSON2D: smoothing sweeps on A v = 0 per test vector */
  uint64_t setup_seed;/* WILSON2D: seed of the test-vector start vectors */
  /* CSR: NULL, or levels_solver - 1 host arrays: agg[l][i] = aggregate (the
     coarse unknown of level l+2) of unknown i of level l+1.  Aggregate numbers
     must cover 0..n_{l+2}-1 without gaps.  NULL builds every level by greedy
     aggregation of the matrix graph (j is a neighbour of i when a_ij != 0):
     pass 1 visits the unknowns in index order, and one whose neighbours are
     all unassigned founds an aggregate with them; pass 2 puts every unknown
     left over into the pass-1 aggregate of its neighbour with the largest
     |a_ij| (the smallest j among equal ones).  Aggregates are numbered in
     order of creation. */
  const int32_t* const* agg;
  /* WILSON2D: 1 = spin-structure-preserving aggregation (Example 4.3): on every
     level the test vectors are restricted separately to the unknowns of each
     spin (a site's first dof/2 unknowns carry spin 0) and orthonormalised per
     spin, so an aggregate has 2 n_vec coarse unknowns (the first n_vec on spin
     0) and every coarse operator keeps J A = A^* J.  2 n_vec must be one of
     the supported site sizes (2, 4, 8, 12, 16).  0 = n_vec coarse unknowns. */
  int spin_split;
  /* CSR: NULL, or levels_solver - 1 prolongations P_l (n_l x n_{l+1}, any
     sparse real matrices with full column rank, e.g. the bilinear
     interpolation of Example 4.1), copied at setup.  Then R_l = P_l^T,
     A_{l+1} = R_l A_l P_l, and the estimator uses the general decomposition of
     Sec. 4.1: the level-l sample is x^T Phat_l A_l^{-1} Rhat_l x -
     x^T Phat_{l+1} A_{l+1}^{-1} Rhat_{l+1} x with a probe x on the finest level
     (keyed by (seed, l, k) like every probe), and the coarsest term is
     tr(A_L^{-1} Rhat_L Phat_L) (Remark 4.2).  Excludes agg. */
  const mlmc_csr* P;
} mlmc_hierarchy;

typedef struct mlmc_options {
  int precision;      /* enum mlmc_precision */
  int nb;             /* maximum right-hand sides per launch (1..1024) */
  int nu_pre, nu_post;/* red-black Gauss-Seidel sweeps before/after the coarse
                         correction in the V-cycle */
  double omega;       /* coarse-correction scaling in the V-cycle (1 = none) */
  int alloc;          /* enum mlmc_alloc */
  const double* rho_weights; /* MLMC_ALLOC_WEIGHTS: L-1 weights (host) */
  double solve_tol;   /* per-column FP64 relative residual |b-Ay|/|b| target */
  double inner_tol;   /* MLMC_FP32_IR64: FP32 CG residual reduction after which
                         the iterate is refined in FP64 (y64 += x32, residual
                         recomputed in FP64; the search direction is kept);
                         for the complex operators the FGMRES cycle's residual
                         reduction.  0 = automatic: 1e-3 (real), 1e-2 (complex) */
  int max_iter;       /* Krylov iterations per solve (MLMC_FP32_IR64: times
                         max_refine) */
  int max_refine;     /* MLMC_FP32_IR64: iteration budget multiplier */
  int krylov_restart; /* FGMRES restart length (complex operators) */
  int min_samples;    /* minimum estimates per level difference (5) */
  int64_t max_samples;/* per-level cap; exceeding it returns MLMC_ENOCONV */
  double tau;         /* > 0: use this tau instead of the 5-sample pilot */
  int learned;        /* 1: learned smoother on the finest level (WILSON2D with
                         MLMC_FP32_IR64, lattice side a multiple of 16); it
                         takes effect once weights are set or trained.  0: plain */
  int graphs;         /* 1: the FP32 refined CG of the real operators replays the
                         two iterations between refinement checks (V-cycles,
                         direction update, x/r update, refinement test) from a
                         HIP graph captured once per (level, batch width), and
                         the FGMRES of the complex operators replays every
                         iteration (V-cycle, operator, Gram-Schmidt, Givens
                         step) from a graph captured once per (precision,
                         level, batch width, iteration, learned smoother on or
                         off); results are bitwise identical.  Bypassed while
                         per-kernel timing is on.  0: direct launches */
  int narrow_fp64;    /* MLMC_FP32_IR64, real operators: solves of batches of at
                         most this many columns run in plain FP64 CG (for a few
                         columns the refinement's extra launches cost more than
                         the FP32 bandwidth saves); FP64 work vectors of this
                         width are allocated.  0: every batch in FP32 + FP64
                         refinement */
  int top_cycles;     /* coarse-grid corrections on the top level of every
                         Krylov solve (CG for the real kinds, each FGMRES
                         preconditioner application for the complex ones):
                         1 = one V-cycle on
                         the next level (plain V-cycle), 2 = two V-cycles there
                         (the second on the residual of the first: a W-cycle on
                         the top level only, V-cycles below); the preconditioner
                         stays symmetric, and positive definite while the
                         level's V-cycle contracts in the energy norm, i.e.
                         while every eigenvalue of M A of the level's V-cycle
                         M is below 2 (with 2 and one sweep on each side at
                         omega 1.8 the 2D Poisson V-cycle exceeds it: about 2.4
                         at 512^2, and solves then miss solve_tol).  0 =
                         automatic: 2 for POISSON2D with nu_pre >= 2 and
                         nu_post >= 2 (fewer iterations, faster), 1 otherwise
                         and for the other kinds (measured: the 3D batch and the
                         bilinear hierarchy of Example 4.1 then miss their
                         tolerance, the graph Laplacian runs 8% slower; the
                         Wilson 256^2 trace takes 12% fewer FGMRES iterations
                         at the same time, the gauge Laplacian is unchanged) */
} mlmc_options;

#define MLMC_MAX_LEVELS 16

typedef struct mlmc_result {
  double trace[2];            /* estimate of tr(A^{-1}) (re, im) */
  double rmsd;                /* sqrt(sum_l V_l/N_l) */
  double tau;                 /* pilot value used for the target eps*tau */
  double coarse_trace[2];     /* tr(A_L^{-1}) */
  int levels;                 /* L */
  int64_t n_samples[MLMC_MAX_LEVELS];   /* N_l, l = 1..L-1 at [l-1] */
  double level_mean[MLMC_MAX_LEVELS][2];
  double level_var[MLMC_MAX_LEVELS];
  double level_cost[MLMC_MAX_LEVELS];   /* cost model C_l */
  double level_seconds[MLMC_MAX_LEVELS];/* wall time spent on level l's samples */
  int64_t solves;             /* right-hand sides solved, all levels */
  int64_t iterations;         /* Krylov iterations x RHS columns, all solves */
  double seconds;             /* wall time of the call */
  double max_stated_error;    /* largest stated FP64 error of any sample */
} mlmc_result;

/* Fill *opt with defaults: FP32_IR64, nb 128, 1+1 sweeps, omega 1.8, EQUAL,
 * solve_tol 1e-10, inner_tol 0 (automatic), max_iter 200, max_refine 8, restart 16,
 * min_samples 5, max_samples 2^22, tau 0, learned 0, graphs 0, narrow_fp64 0. */
int mlmc_default_options(mlmc_options* opt);

/* Build the hierarchy on the device: copies the operator data, forms the
 * aggregation P_l and Galerkin A_{l+1} = P_l^H A_l P_l (Sec. 4.1), and inverts
 * the coarsest operators in FP64 (the MLMC level L for the direct trace term of
 * Remark 4.2, the solver level L_s for the V-cycle).  hip_stream: a
 * hipStream_t or NULL.  On success *out owns device memory until
 * mlmc_destroy.  Errors: EINVAL for inconsistent sizes (a grid side that is not
 * divisible by the aggregate side at every level, L > L_s, nb out of range, a
 * coarsest operator with a zero pivot in its partially pivoted Gauss-Jordan
 * inverse), EDEVICE/ENOMEM from the runtime. */
int mlmc_setup(const mlmc_operator* A, const mlmc_hierarchy* h,
               const mlmc_options* opt, void* hip_stream, mlmc_ctx** out_ctx);

/* MLMC estimate of tr(A^{-1}) to relative accuracy tol (Sec. 5): tau from five
 * pilot Hutchinson estimates (or opt.tau), per-level RMSD targets rho_l with
 * sum rho_l^2 = (tol*tau)^2, at least min_samples per level difference,
 * batches of at most nb samples, coarsest term exact.  Fills *out. */
int mlmc_trace(mlmc_ctx* ctx, double tol, uint64_t seed, mlmc_result* out);

/* Plain Hutchinson estimate (eq. plain_tr_estimate) on level 1 with the same
 * tau rule and batch rule, for comparison.  Fills trace, rmsd, tau,
 * n_samples[0], solves, seconds. */
int mlmc_hutchinson(mlmc_ctx* ctx, double tol, uint64_t seed, mlmc_result* out);

/* Level-difference samples s_{l,k}, k = first .. first+nsamples-1:
 *   s = x^H A_l^{-1} x - (R_l x)^H A_{l+1}^{-1} (R_l x),  x = probe(seed, l, k),
 * 1 <= level < L (level L is not sampled: use mlmc_coarse_trace).
 * out: host, nsamples x 2 doubles (re, im).  out_err: host, nsamples doubles,
 * or NULL: the stated FP64 error of each sample (relative to |x^H y| +
 * |(Rx)^H z|) -- the contribution of the last refinement correction, or the
 * final relative residual in MLMC_FP64 mode.  Any nsamples >= 1 is accepted
 * (split into launches of at most nb).  MLMC_ENOCONV when a solve misses
 * solve_tol: out and out_err then hold every sample of the batches before the
 * failing one and that batch's converged samples, NaN for its failed ones, and
 * mlmc_last_error names the level whose solve failed, the first failed sample
 * index and its column in the batch; later batches are not run. */
int mlmc_sample_level(mlmc_ctx* ctx, int level, uint64_t seed, int64_t first,
                      int64_t nsamples, double* out, double* out_err);

/* tr(A_L^{-1}) computed at setup by inverting A_L (Remark 4.2). out: 2 doubles. */
int mlmc_coarse_trace(mlmc_ctx* ctx, double* out);

/* n_l, the number of unknowns of level l (1 <= l <= L_s). */
int mlmc_level_size(mlmc_ctx* ctx, int level, int64_t* n);

/* Y = A_l^{-1} B for nrhs <= nb vectors: the solver used by the samples
 * (precision and tolerance from the options).  b_dev, y_dev: FP64 (complex:
 * interleaved) RHS-major blocks of nrhs vectors of n_l.  relres: host, nrhs
 * doubles or NULL, final FP64 relative residuals.  ENOCONV if a column misses
 * solve_tol within max_refine x max_iter. */
int mlmc_solve(mlmc_ctx* ctx, int level, int nrhs, const double* b_dev,
               double* y_dev, double* relres);

/* Y = A_l X in FP64 (the FP64 operator of level l). */
int mlmc_apply(mlmc_ctx* ctx, int level, int nrhs, const double* x_dev, double* y_dev);

/* Flags of mlmc_smooth. */
enum mlmc_smooth_flags {
  MLMC_SMOOTH_REVERSE = 1,    /* odd colour first, as in post-smoothing */
  MLMC_SMOOTH_ZERO_START = 2, /* start from X = 0 (x_dev's input is not read) with
                                 the zero-start kernel forms that the V-cycle's
                                 pre-smoothing runs; forward sweeps only
                                 (with MLMC_SMOOTH_REVERSE: MLMC_EINVAL) */
  /* MLMC_CSR sweep schedule of this call instead of the level's autotuned one
   * (the results do not depend on it; other kinds ignore these flags; both
   * together: MLMC_EINVAL): */
  MLMC_SMOOTH_CLASS_LAUNCHES = 4, /* one launch per colour class */
  MLMC_SMOOTH_SHARED_TAIL = 8     /* the trailing colour classes of at most 16
                                     slices (1024 rows) each share launches */
};

/* X <- `sweeps` red-black Gauss-Seidel sweeps of A_l X = B (the V-cycle's
 * smoother, Section 4 multigrid setting; sites coloured by the parity of the sum
 * of their coordinates, first colour (even) first; flags: enum
 * mlmc_smooth_flags), run in the working precision by the V-cycle's own kernels
 * and sweep grouping (2D Poisson levels: passes of up to two fused sweeps, an
 * odd remainder first for forward sweeps, last for reverse ones; the Wilson
 * level: both colours of a sweep in one out-of-place pass).  With rc_dev
 * non-NULL (forward sweeps only) also Rc = R_l (B - A_l X) of the final X, as
 * the last pre-smoothing pass of the V-cycle writes it (fused into that pass
 * where the V-cycle fuses it).  b_dev, x_dev: FP64 (complex: interleaved)
 * RHS-major blocks of nrhs <= nb vectors of n_l; x_dev is read (unless
 * MLMC_SMOOTH_ZERO_START) and overwritten; rc_dev: nrhs vectors of n_{l+1}.
 * 1 <= l < L_s; sweeps >= 0.  The library allocates and frees
 * working-precision copies during the call (see mlmc_smooth_noalloc for the
 * allocation-free form).  For tests and inspection. */
int mlmc_smooth(mlmc_ctx* ctx, int level, int nrhs, int sweeps, int flags, const double* b_dev,
                double* x_dev, double* rc_dev);

/* Xc = R_l X = P_l^H X (restriction to level l+1), FP64, 1 <= l < L_s. */
int mlmc_restrict(mlmc_ctx* ctx, int level, int nrhs, const double* x_dev, double* xc_dev);

/* X = P_l Xc (prolongation from level l+1), FP64, 1 <= l < L_s. */
int mlmc_prolong(mlmc_ctx* ctx, int level, int nrhs, const double* xc_dev, double* x_dev);

/* Probe block: vectors k = first..first+nrhs-1 of level l, stream `stream`
 * (0 level probes, 1 pilot, 3 Hutchinson), written as FP64 (complex:
 * interleaved) to out_dev [nrhs][n_l]. */
int mlmc_probes(mlmc_ctx* ctx, int level, uint64_t seed, int stream, int64_t first,
                int nrhs, double* out_dev);

/* Copy the dense FP64 coarsest operator A_{L_s} (or A_L if which == 1) to host
 * memory, n x n row-major (complex: interleaved).  For inspection and tests. */
int mlmc_export_coarse(mlmc_ctx* ctx, int which, double* out);

/* WILSON2D: copy the aggregation basis of level l (1 <= l < L_s) to host memory
 * as n_l x n_vec complex values: row i holds the n_vec coefficients of unknown
 * i in the basis of its aggregate (Example 4.3 aggregation sketch). */
int mlmc_export_prolongation(mlmc_ctx* ctx, int level, double* out);

/* MLMC_CSR: level `level` (1..L_s) of the hierarchy as the library holds it
 * (Sec. 4.1: A_{l+1} = P_l^T A_l P_l).  *nnz receives its entry count; row_ptr
 * (n_l + 1), col_idx and vals (nnz each) the matrix in canonical form (columns
 * ascending, no repeated or zero entries); agg (n_l, levels below L_s) the
 * aggregate of every unknown; colour (n_l) its first-fit colour class, the
 * Gauss-Seidel order.  Host arrays, each may be NULL (not written).  Other
 * kinds: MLMC_EUNSUPPORTED. */
int mlmc_export_csr(mlmc_ctx* ctx, int level, int64_t* nnz, int64_t* row_ptr, int32_t* col_idx,
                    double* vals, int32_t* agg, int32_t* colour);

/* Any kind: level `level` of the hierarchy as the library holds it, as a sparse
 * matrix in canonical compressed-row form (columns ascending, repeated entries
 * summed, zero entries dropped).  which = 0: the operator A_l (1 <= l <= L_s,
 * n_l x n_l; Sec. 4.1, A_{l+1} = R_l A_l P_l); which = 1: the prolongation P_l
 * (1 <= l < L_s, n_l x n_{l+1}; R_l = P_l^H): orthonormal aggregation
 * (2D Poisson: entries 1/2 on the 2 x 2 aggregates, 3D: 1/sqrt(8) on 2 x 2 x 2,
 * matrix-given: 1/sqrt|J|), the test-vector bases of the lattice kinds (row i
 * holds unknown i's coefficients in its aggregate's basis), or the given P.
 * Outputs (host, each may be NULL = not written): rows, cols, nnz; row_ptr
 * (rows + 1), col_idx (nnz), vals (nnz doubles, or 2 nnz interleaved (re, im)
 * for the complex kinds).  Call once with NULL arrays for the sizes. */
int mlmc_export_level(mlmc_ctx* ctx, int level, int which, int64_t* rows, int64_t* cols,
                      int64_t* nnz, int64_t* row_ptr, int32_t* col_idx, double* vals);

/* Host-side estimator driver over a caller-supplied sampler (no device use).
 * sample(user, level, first, count, out): write count samples of level l as
 * (re, im) pairs; return 0 or a negative status.  pilot(user, count, out):
 * five (or count) plain Hutchinson samples for tau; may be NULL if opt->tau > 0.
 * coarse: tr(A_L^{-1}) (re, im).  cost: C_l for l = 1..L-1 (NULL = all 1).
 * Same control as mlmc_trace. */
typedef int (*mlmc_sample_fn)(void* user, int level, int64_t first, int64_t count,
                              double* out);
typedef int (*mlmc_pilot_fn)(void* user, int64_t count, double* out);
int mlmc_run_estimator(int levels, mlmc_sample_fn sample, mlmc_pilot_fn pilot,
                       void* user, const double* coarse, const double* cost,
                       const mlmc_options* opt, double tol, mlmc_result* out);

/* Device memory hooks (e.g. a framework's caching allocator).  Applies to
 * contexts created afterwards.  alloc returns NULL on failure.  Pass NULLs to
 * restore hipMalloc/hipFree. */
typedef void* (*mlmc_alloc_fn)(size_t bytes, void* user);
typedef void (*mlmc_free_fn)(void* ptr, void* user);
int mlmc_set_allocator(mlmc_alloc_fn alloc, mlmc_free_fn free_fn, void* user);

/* Batch of independent problems (Sec. 4.1 samples of each), run concurrently:
 * `workers` host threads each take the next problem, longest level first, and
 * draw samples first..first+nsamples-1 of level `level` with seeds[i] exactly
 * as mlmc_sample_level would.  Problems overlap on the GPU when their contexts
 * were set up on different HIP streams (contexts sharing a stream run one
 * after another, with the same results).  out: count x nsamples x 2 doubles
 * (re, im), problem-major; seconds (nullable): wall time per problem.  Every
 * context must be distinct; level must be sampleable on all of them.
 * Returns the first failing problem's status (its context holds the message). */
int mlmc_batch_sample(mlmc_ctx* const* ctxs, int count, int level, const uint64_t* seeds,
                      int64_t first, int64_t nsamples, int workers, double* out,
                      double* seconds);

/* Batch of independent problems (Sec. 4.1 samples of each) solved together on
 * one GPU: the samples first..first+nsamples-1 of level `level` of every
 * problem, identical to what mlmc_sample_level(ctxs[i], level, seeds[i], ...)
 * returns.  All problems' solves run in lockstep on the first context's
 * stream: each step of the refined CG is one launch over every problem still
 * iterating.  Each preconditioner application is, with mode 1, one persistent
 * launch over the whole V-cycle of every problem: a workgroup per (problem,
 * column pair) runs all levels and stages of its problem's V-cycle for its
 * two columns (larger problems first), with no synchronisation between
 * workgroups; with mode 2, one launch per V-cycle position and stage kernel
 * over the (problem, level, stage, tile) items of all problems at that
 * position.  Both give the same results.  Needs VARCOEF3D
 * contexts with MLMC_FP32_IR64, equal nb and iteration limits, nu_pre and
 * nu_post >= 1, one coarse-grid cycle (top_cycles 1), narrow_fp64 0, and the
 * fused sweep on every smoothed level (even sides up to 128); otherwise
 * MLMC_EUNSUPPORTED.  out: count x nsamples x 2 doubles (re, im),
 * problem-major; status (count ints, caller-owned): per problem MLMC_OK, or
 * the error of its first failing batch (the problem takes no further batches;
 * its context names the sample, and out holds its samples as
 * mlmc_sample_level leaves them).  Returns the first failing problem's status. */
int mlmc_batch_sample_grouped(mlmc_ctx* const* ctxs, int count, int level,
                              const uint64_t* seeds, int64_t first, int64_t nsamples, int mode,
                              double* out, int* status);

/* Counters of the last mlmc_trace / mlmc_sample_level / mlmc_solve call:
 * out[0] Krylov iterations (per batch), out[1] refinement steps,
 * out[2] V-cycles, out[3] batches.  n: entries to copy (<= 4). */
int mlmc_counters(mlmc_ctx* ctx, int64_t* out, int n);

/* Measurement mode.  mask: bit i set = launches of kernel id i (listed
 * below) are bracketed by HIP events on the context stream and record their
 * active columns, so that per-kernel launch counts, durations and algorithmic
 * bytes can be read back; mask = 0 stops it.  stride >= 1: about one launch in
 * stride of each timed kernel is bracketed (the others run
 * untouched; which launches is fixed by a hash of the launch index, so the
 * sample does not alias with the launch pattern of the V-cycle), which bounds
 * the cost of the two event records per timed launch.
 * Returns MLMC_EINVAL for stride < 1. */
int mlmc_set_timing(mlmc_ctx* ctx, int mask, int stride);

/* Kernel ids for mlmc_kernel_stats (algorithmic bytes per unknown and RHS for
 * element size e; each operator kind reports its own smoother, residual and
 * transfer kernels under the same ids): 0 red-black Gauss-Seidel sweep (2e from a zero start:
 * b in, x out; 3e with an input iterate; +0.25e with the folded coarse
 * correction), 1 fused residual + restriction (2.25e), 2 prolongation +
 * correction when there is no post-smoothing (2.25e), 3 Krylov direction update
 * fused with the operator apply and its dot (4e: z, p in; p, q out), 4 CG x/r
 * update with |r|^2 (6e), 5 learned-smoother network (counts FLOPs, not
 * bytes: 2 x 4032 per site and column), 6 FP64 refinement fold y += x32 with
 * its b^T x32 partial sums and x32 = 0 (32 bytes: FP64 y, b and FP32 x32 in; y
 * and x32 out; fp64 slot), 7 FP64 refinement residual (20 bytes: FP64 b and y
 * in, FP32 r out; fp64 slot).  fp64 = 0 selects the FP32/complex64
 * instantiation, 1 the FP64 one.  out: launches, total milliseconds, total
 * algorithmic bytes (active columns only). */
int mlmc_kernel_stats(mlmc_ctx* ctx, int kernel, int fp64, double* out);
/* The same restricted to the launches on one level (1 <= level <= L_s; 0 = all
 * levels, as mlmc_kernel_stats). */
int mlmc_kernel_stats_level(mlmc_ctx* ctx, int kernel, int fp64, int level, double* out);
int mlmc_reset_kernel_stats(mlmc_ctx* ctx);

/* Measurement of the sustained HBM rate (the practical peak beside the vendor
 * figure): copies `bytes` from src_dev to dst_dev (device pointers, 16-byte
 * aligned, bytes a multiple of 16, no overlap) with a streaming kernel of
 * 16-byte loads and stores on hip_stream (NULL: the default stream); the copy
 * moves 2 x bytes through HBM.  Asynchronous; MLMC_EINVAL on misaligned
 * arguments. */
int mlmc_stream_copy(const void* src_dev, void* dst_dev, size_t bytes, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Learned smoother (WILSON2D).  A 3-layer network of 3x3 periodic convolutions
 * without bias (8 -> 16 -> 16 -> 4 channels, ReLU after the first two) maps, per
 * lattice site, the residual scaled by its RMS s over the column (Re/Im of the
 * two spin components) and cos/sin of the two link phases at the site to a
 * correction s * (o0 + i o1, o2 + i o3) added to the iterate.  On the finest
 * level the V-cycle becomes: Gauss-Seidel sweep, network, coarse correction,
 * network, Gauss-Seidel sweep (two of the four plain sweeps replaced).  The
 * network runs in BF16 with FP32 accumulation on MFMA.  The FP64 residual of
 * the refinement loop stays the judge: a solve converges to solve_tol or fails
 * exactly as without the network, so the estimate is unchanged in
 * distribution.  If a refinement cycle with the network reduces some column's
 * FP64 residual norm by less than a factor 2, the rest of that solve uses the
 * plain smoother (a fallback, counted).
 *
 * Weights: MLMC_NN_WEIGHTS FP32 values, W1 [16][8][3][3], W2 [16][16][3][3],
 * W3 [4][16][3][3] ([out channel][in channel][row offset][column offset],
 * cross-correlation, offsets -1, 0, +1).
 * ------------------------------------------------------------------------- */
#define MLMC_NN_WEIGHTS 4032
#define MLMC_NN_CROP 22      /* training crop side (output 16 x 16) */

typedef struct mlmc_train_options {
  int n_batches;        /* plain-multigrid solves used: n_batches * nb */
  int crops_per_column; /* crops drawn per solved column and state (2 states) */
  int steps;            /* Adam steps */
  int batch;            /* crops per step (<= n_batches * nb * 2 * crops_per_column) */
  double lr;            /* Adam learning rate (betas 0.9, 0.999, eps 1e-8) */
  uint64_t seed;        /* probes (RNG stream 5) and crop positions */
  double pair_tol;      /* relative residual of the plain solves that give the
                           training targets (0: 1e-6; a target error of that size
                           is far below the network's BF16 rounding) */
} mlmc_train_options;

typedef struct mlmc_train_report {
  double loss_first;    /* mean squared error of the first step */
  double loss_last;     /* mean over the last min(10, steps) steps */
  int64_t solves;       /* plain solves that produced training pairs */
  int64_t crops;        /* crops in the training set */
  double gen_seconds;   /* pair generation (solves, states, crops) */
  double train_seconds; /* Adam steps */
} mlmc_train_report;

/* Train the network on pairs (r, e) from the method's own plain multigrid
 * solves: Z4 right-hand sides b (stream 5), y = A^-1 b by the plain solver,
 * and two states x per solve -- one Gauss-Seidel sweep from zero, and that plus
 * the coarse-grid correction -- with r = b - A x and e = y - x, both scaled by
 * the RMS of r, cut into crops of MLMC_NN_CROP^2 sites at positions drawn from
 * `seed`.  w_init: host MLMC_NN_WEIGHTS initial weights.  The trained weights
 * stay in ctx.  Errors: MLMC_EUNSUPPORTED for kinds other than WILSON2D or a
 * lattice side not a multiple of 16; MLMC_EINVAL for bad options. */
int mlmc_learned_train(mlmc_ctx* ctx, const float* w_init, const mlmc_train_options* opt,
                       mlmc_train_report* out);
/* Set / read the network weights (host arrays of MLMC_NN_WEIGHTS floats). */
int mlmc_learned_set_weights(mlmc_ctx* ctx, const float* w);
int mlmc_learned_get_weights(mlmc_ctx* ctx, float* w);
/* out[0] network applications (launches) and out[1] fallbacks to the plain
 * smoother since setup. */
int mlmc_learned_stats(mlmc_ctx* ctx, int64_t* out);
/* Building blocks for tests.  mlmc_nn_apply: e = correction of the network for
 * residuals r (device, nrhs x n_1 complex as interleaved FP64, level 1).
 * mlmc_nn_loss_grad: mean squared error and its gradient (host, FP32
 * MLMC_NN_WEIGHTS) over ncrops crops: in device FP32 [ncrops][22][22][8]
 * (rounded to BF16), target device FP32 [ncrops][16][16][4]. */
int mlmc_nn_apply(mlmc_ctx* ctx, int nrhs, const double* r, double* e);
int mlmc_nn_loss_grad(mlmc_ctx* ctx, int ncrops, const float* in, const float* target, double* loss,
                      float* grad);

/* mlmc_nn_crops: the training-pair builder of mlmc_learned_train on given data.
 * r, e: device, nrhs x n_1 complex as interleaved FP64 (residuals and errors,
 * level 1, nrhs <= nb); origin: host int32 [ncrops][3] = (column, y0, x0) of
 * each crop's input corner (0 <= y0, x0 < N; sites wrap periodically).  Writes
 * in: host FP32 [ncrops][22][22][8], the BF16 network inputs (r / s for the
 * column's RMS s = sqrt(|r|^2 / n_1), Re/Im of both spins, then cos/sin of the
 * two link phases), and target: host FP32 [ncrops][16][16][4], e / s on the
 * crop's interior (rows and columns 3..18).  1 <= ncrops <= 65536.
 * mlmc_nn_adam_step: one Adam update (Kingma and Ba; betas 0.9, 0.999, eps
 * 1e-8, bias-corrected with step count t >= 1) of the FP32 master weights with
 * the given gradient (host FP32, MLMC_NN_WEIGHTS); t == 1 first zeroes the
 * moments; the inference fragments are re-packed.  ESTATE without weights. */
int mlmc_nn_crops(mlmc_ctx* ctx, int nrhs, const double* r, const double* e, int ncrops,
                  const int32_t* origin, float* in, float* target);
int mlmc_nn_adam_step(mlmc_ctx* ctx, const float* grad, double lr, int t);

/* ---------------------------------------------------------------------------
 * Allocation-free entry point, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  mlmc_smooth_noalloc has the arguments, results and errors of
 * mlmc_smooth (same kernels, bit-identical output) but calls no hipMalloc,
 * hipFree or allocating routine: its working-precision copies (3 blocks of
 * nrhs x n_l, plus nrhs x n_{l+1} with rc_dev, each rounded up to 256 bytes;
 * 4 or 8 bytes per real unknown, twice that for complex ones) live in a fixed
 * device array of MLMC_NOALLOC_SCRATCH_BYTES that every GPU the library runs on
 * holds until the process ends (looked up at the first mlmc_setup on the
 * device).  Larger requests return MLMC_EINVAL and name the size.  It does not
 * synchronise the stream: the output is ready when the context's stream
 * reaches it.  All calls on one GPU share its array, so calls that overlap in
 * time on one GPU (contexts on different streams, or different threads) race
 * and must be serialised by the caller; calls queued on one stream are
 * ordered and safe.
 * ------------------------------------------------------------------------- */
#define MLMC_NOALLOC_SCRATCH_BYTES (64u << 20)
int mlmc_smooth_noalloc(mlmc_ctx* ctx, int level, int nrhs, int sweeps, int flags,
                        const double* b_dev, double* x_dev, double* rc_dev);

/* ---------------------------------------------------------------------------
 * Deflated Hutchinson: the comparison method of Sec. 5 (Sec. 4.2, eqs.
 * orth_proj and defl).  With Pi = U U^H for the n_defl eigenvectors of the
 * smallest eigenvalues of a Hermitian A, tr(A^{-1}) = tr(A^{-1}(I - Pi)) +
 * tr(A^{-1} Pi): the first trace is estimated from samples
 * x^H A^{-1} (x - U (U^H x)) with the plain Hutchinson probes (RNG stream 3, so
 * sample k shares its probe with mlmc_hutchinson's sample k), the second is
 * computed once as tr(U^H A^{-1} U) (sum 1/lambda_i for exact eigenvectors;
 * the split stays exact for approximate ones).  Real symmetric kinds (POISSON2D,
 * VARCOEF3D, CSR); others return MLMC_EUNSUPPORTED.
 * ------------------------------------------------------------------------- */
typedef struct mlmc_deflation_options {
  int n_defl;        /* deflated eigenpairs k (1..1024) */
  int oversample;    /* extra block vectors p of the subspace iteration (0: max(8, k/2)) */
  double eig_tol;    /* stop when every |A u_i - theta_i u_i| / theta_i <= eig_tol */
  int max_iter;      /* subspace iterations (each: k + p solves, Rayleigh-Ritz) */
  double solve_tol;  /* relative residual of the iteration's solves (0: 1e-8); the
                        direct term is solved to the context's solve_tol */
  uint64_t seed;     /* start block (Rademacher, RNG stream 6) */
} mlmc_deflation_options;

typedef struct mlmc_deflation_report {
  int iterations;        /* subspace iterations run */
  double seconds;        /* wall time of the setup (eigenpairs and direct term) */
  double max_residual;   /* largest relative Ritz residual of the k pairs */
  double direct_trace;   /* tr(U^H A^{-1} U) */
  double sum_inv_eig;    /* sum of 1/theta_i over the k Ritz values */
  int64_t solves;        /* right-hand sides solved by the setup */
} mlmc_deflation_report;

/* Compute the deflation space of level 1 (block subspace iteration with the
 * library's own solves: W = A^{-1} V, two passes of Cholesky QR, Rayleigh-Ritz
 * with a Jacobi eigensolver on the (k+p) x (k+p) projected matrix) and the
 * direct term.  Replaces an earlier deflation space.  ENOCONV if a solve fails;
 * the Ritz residuals reached are reported even when max_iter ran out. */
int mlmc_deflation_setup(mlmc_ctx* ctx, const mlmc_deflation_options* opt,
                         mlmc_deflation_report* report);
/* Deflated samples x_k^H A^{-1} (I - Pi) x_k, k = first..first+nsamples-1, as
 * (re, im) pairs in out (host, nsamples x 2); out_err (nullable): stated FP64
 * error per sample as for mlmc_sample_level.  ESTATE before mlmc_deflation_setup. */
int mlmc_deflated_sample(mlmc_ctx* ctx, uint64_t seed, int64_t first, int64_t nsamples,
                         double* out, double* out_err);
/* Deflated Hutchinson estimate to relative accuracy tol with the control of
 * Sec. 5 (tau from the five plain pilot estimates, samples until their RMSD is
 * at most tol * tau, batches of at most nb).  trace = sample mean + direct term;
 * coarse_trace holds the direct term; n_samples[0] the sample count. */
int mlmc_deflated_hutchinson(mlmc_ctx* ctx, double tol, uint64_t seed, mlmc_result* out);
/* Copy the deflation space: eigenvalues (host, k Ritz values ascending, or
 * NULL), vectors_dev (device, k x n_1 FP64 RHS-major, or NULL), direct (host,
 * 1 double, or NULL). */
int mlmc_deflation_export(mlmc_ctx* ctx, double* eigenvalues, double* vectors_dev, double* direct);

/* Description of the last error on ctx (or of the last failed mlmc_setup
 * when ctx is NULL).  Valid until the next call on ctx. */
const char* mlmc_last_error(const mlmc_ctx* ctx);

const char* mlmc_status_string(int status);

/* Free everything the context owns.  NULL is ignored. */
void mlmc_destroy(mlmc_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* MLMC_H */
