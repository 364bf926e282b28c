/*
 * libglasso -- pISTA for the graphical lasso on AMD Instinct MI355X (gfx950).
 *
 * Problem (Shalom, Treister & Yavneh, arXiv 2205.10027, Sec. 3.1, eqs. log_MLE
 * and sparse_obj):
 *
 *     minimise  F(A) = -log det A + tr(S A) + lambda * sum_{i,j} |A_ij|   over A > 0,
 *
 * the diagonal being penalised.  The solver is Algorithm 1 (pISTA) with the
 * initialisation, line search and stopping rule of Sec. 6.
 *
 * Conventions for every entry point below
 *  - Matrices are dense, FP64, n x n, row-major with leading dimension n, in
 *    DEVICE memory owned by the caller (e.g. a torch tensor's data_ptr()).
 *    Symmetric inputs are read through their lower triangle only.
 *  - `stream` is a hipStream_t (NULL = the null stream).  All work is enqueued
 *    on it; calls return after the work they need to inspect has completed.
 *  - Every call returns a glasso_err and never aborts the process.
 *  - A handle owns a cached device workspace (grown on demand, freed by
 *    glasso_destroy).  A handle is not thread-safe: use one per host thread.
 */
#ifndef GLASSO_H
#define GLASSO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct glasso_handle_s* glasso_handle;

typedef enum {
  GLASSO_OK = 0,
  GLASSO_ERR_INVALID_ARG = 1, /* bad size, lambda, tol, NULL pointer, non-finite S, S_ii + lambda <= 0 */
  GLASSO_ERR_NOT_PD = 2,      /* the warm start (or a Cholesky input) is not positive definite */
  GLASSO_ERR_OOM = 3,         /* device workspace allocation failed */
  GLASSO_ERR_HIP = 4,         /* a HIP runtime call or kernel launch failed */
  GLASSO_ERR_INTERNAL = 5
} glasso_err;

typedef enum {
  GLASSO_CONVERGED = 0, /* ||Z||_1 <= tol * ||A||_1 (stopping rule, Sec. 6) */
  GLASSO_MAX_ITER = 1,  /* max_iter accepted steps without meeting tol */
  GLASSO_LS_FAILED = 2  /* no step size down to t_min passed the line search's test */
} glasso_status;

typedef enum {
  GLASSO_FP64 = 0,        /* every step in FP64 */
  GLASSO_MIXED_FP32 = 1,  /* A Z A products in FP32 MFMA; factor, log det, PD test and KKT in FP64;
                             W as set by w_mixed */
  GLASSO_MIXED_BF16X3 = 2 /* A Z A with each operand split into two BF16 parts, x = hi + lo, and each
                             product formed as hi hi + hi lo + lo hi on BF16 MFMA with FP32
                             accumulation (about 2^-16 relative); factor, log det, PD test and
                             KKT in FP64; W as set by w_mixed */
} glasso_precision;

typedef struct {
  int precision;   /* glasso_precision; default GLASSO_FP64 */
  int max_iter;    /* accepted steps before GLASSO_MAX_ITER; default 500 */
  double t0;       /* first step size of every line search; default 1 (Alg. 1) */
  double shrink;   /* backtracking factor; default 0.5 (Sec. 4.3.2) */
  double t_floor;  /* below it, t = min(t, (0.9/cond A)^2) (Sec. 6); default 1e-4 */
  double t_min;    /* the line search fails below it; default 1e-12 */
  int warm_start;  /* nonzero: A holds the starting iterate (Alg. 1 takes A^(0)) */
  int tile_policy; /* FP64 GEMM launches (Cholesky updates, triangular inverse, LAUUM,
                      the FP64 A Z A) with fewer than this many 128x128 output tiles
                      run 64x64 tiles; GLASSO_TILES_AUTO (the default): the value the
                      autotuner measured for the padded size and batch count, tuned
                      on first use and kept for the process.  Results are bitwise
                      the same under every policy. */
  int graphs;      /* nonzero: each launch sequence of an iteration (inverse + gradient
                      pass, A Z A, trial point + Cholesky, accept) is captured once as
                      a HIP graph per workspace shape and replayed; results are bitwise
                      the same as eager launches.  time_ms[1] then holds [1] + [2], and
                      time_ms[5] the whole A Z A sequence.  Default 0. */
  int w_mixed;     /* W = A^{-1} from the FP64 factor with FP32 accuracy (triangular inverse
                      and V^T V, each product formed from exact three-part BF16 splits of
                      FP32 values, six BF16 MFMA products per pair) while a problem iterates;
                      before it stops (KKT <= tol or max_iter) W and the measures are
                      recomputed in FP64 and only those decide, after which the problem
                      keeps FP64 W.  Returned W and reported measures are always FP64.
                      -1 (default): on for the mixed precisions, off for FP64; 0 off; 1 on. */
  int ls_width;    /* step sizes of the backtracking sequence (t, t*shrink, ...) that one
                      line-search round factors per problem, at once; the first that
                      succeeds is taken, so the accepted steps, iterations and ls_trials
                      are the same for every width.  Each unit of width holds one more
                      trial point and factor (2 n^2 doubles) per problem.  0 (default):
                      4 for n <= 2048 (1 when that workspace does not fit in device
                      memory), 1 above; else 1 .. 16. */
  int dense_product; /* 0 (default): each iteration's A Z A is formed, per problem, by the
                        sampled sparse product when every row of the iterate has at most 16
                        nonzeros and every row of the free set at most 64 entries on or left
                        of the diagonal (only entries on the free set are needed, eq. d_sol),
                        in FP64 from the same Z; otherwise by the dense GEMM pair of
                        `precision`.  1: always the dense pair (the paper's dense design). */
  int screen;      /* 1: before iterating, split every problem into the connected components
                      of the graph {|S_ij| > lambda, i != j} (its solution is block diagonal over
                      them, each block the solution of its own problem) and solve the blocks:
                      those of n <= GLASSO_SMALL_MAX_N in one persistent launch (FP64), the
                      others batched in `precision`; A and W are assembled with zeros between
                      blocks.  Each block stops on its own measure, so the whole problem meets
                      ||Z||_1 <= tol ||A||_1; the status is CONVERGED whenever the assembled
                      A meets it (a block may stall a little below its own share), else the
                      worst status of the blocks.  Results equal the unscreened solve to the
                      tolerance, not bitwise.  0 (default): no screening. */
  double sigma;    /* sufficient-decrease fraction of the line search: a trial point is
                      accepted when F(At) - F(A) < sigma * (<g, At - A> + lambda (||At||_1 -
                      ||A||_1)), the decrease that the linear model of f plus the l1 term
                      predicts (an Armijo rule); 0 (default): strict decrease, the paper's
                      condition t_cond_min.  0 <= sigma < 1. */
  int method;      /* glasso_method; default GLASSO_PISTA.  GLASSO_GISTA solves the same problem
                      by proximal gradient descent (the H = I case of eq. proximal_gen, Sec. 3.2;
                      the paper's first-order comparison method, Sec. 6): trial point
                      ST(A - t (S - W), t lambda); accepted when positive definite with
                      f(At) <= f(A) + <g, At - A> + ||At - A||_F^2 / (2t), f = -log det + tr(S .),
                      evaluated in difference form; the first step of each iteration is the
                      Barzilai-Borwein step <dA, dA> / <dA, W_prev - W> of the last accepted step
                      dA (t0 in the first iteration), then t *= shrink down to t_min (t_floor and
                      sigma do not apply); a trial point equal to A (the step lost in rounding)
                      ends the search with GLASSO_LS_FAILED.  Same start, stopping rule,
                      precisions (no product: precision only sets the W ladder) and outputs as
                      pISTA.  glasso_solve_small and glasso_solve_small_static accept
                      GLASSO_PISTA only; with screen, every block goes to the batched engine. */
} glasso_options;

typedef enum {
  GLASSO_PISTA = 0, /* Alg. 1 (preconditioned ISTA) */
  GLASSO_GISTA = 1  /* proximal gradient (G-ISTA), see glasso_options.method */
} glasso_method;

#define GLASSO_TILES_AUTO (-1)

typedef struct {
  double objective; /* F(A) of the returned A */
  double kkt_rel1;  /* ||Z||_1 / ||A||_1, Z the minimum-norm subgradient (Sec. 4.3.1, Sec. 6) */
  double kkt_fro;   /* ||Z||_F (the measure the paper's tables report) */
  double kkt_max;   /* max |Z_ij| */
  int64_t nnz;      /* nonzeros of the returned A (full count, diagonal included) */
  int iterations;   /* accepted steps */
  int ls_trials;    /* trial points factored by the line search, over all iterations */
  int status;       /* glasso_status */
  int fallback_steps; /* line searches that reached t_floor and used the cond-based step */
  double time_ms[8];  /* [0] total, [1] W = A^-1, [2] gradient pass, [3] A Z A,
                        [4] line search, [5] the two A Z A GEMM launches alone,
                        [6] the line search's trial factorisations alone, [7] the
                        V^T V launches of the FP32-accurate W alone (both: eager
                        launches only; 0 with graphs) */
  int aza_gemm_products; /* A Z A products formed by the GEMM pair; the first product
                            of a diagonal start is D Z D, formed elementwise */
  int aza_sparse_products; /* A Z A products formed by the sampled sparse product
                              (see dense_product); time_ms[5] excludes them */
  int leaf_launches;  /* leaf steps of the blocked Cholesky timed one by one: those of the
                         first trial factorisation of the call in which every trial
                         point was positive definite (eager launches only; 0 if none) */
  double leaf_ms;     /* their summed launch times (HIP events around each launch) */
  double leaf_flops;  /* their algorithmic flops: per step at column k, nb = min(128, n - k),
                         nb^3/3 for the diagonal block and (n - k - nb) nb^2 for the panel */
  int components;         /* with screen: blocks the problem split into (1 otherwise) */
  int largest_component;  /* with screen: size of the largest block (n otherwise) */
} glasso_info;

/* Fill *opt with the defaults listed above. */
glasso_err glasso_default_options(glasso_options* opt);

/* Create a handle bound to the current HIP device.  opt may be NULL (defaults).
 * The options are copied.  Errors: INVALID_ARG for h == NULL or out-of-range options. */
glasso_err glasso_create(glasso_handle* h, const glasso_options* opt);

/* Release the handle and its device workspace.  NULL is accepted. */
glasso_err glasso_destroy(glasso_handle h);

/* Static description of an error code. */
const char* glasso_error_string(glasso_err e);

/* Device bytes of workspace a solve of size n needs with `precision` and the
 * default ls_width (for admission by HBM footprint).  Errors: INVALID_ARG for n < 1 or bytes == NULL. */
glasso_err glasso_workspace_size(int64_t n, int precision, size_t* bytes);

/* Many small problems (n <= GLASSO_SMALL_MAX_N each, sizes may differ) in ONE
 * persistent launch: each workgroup takes problems i, i + G, i + 2G, ... (G =
 * min(count, 512) workgroups) and runs the whole of Alg. 1 (Sec. 6 settings,
 * FP64 for every step whatever opt.precision says) for each on the device, with no
 * host round trip between iterations or trials.  Arguments, outputs and errors as
 * for glasso_solve_batched (A[i] is also the starting iterate with warm_start);
 * info[i].time_ms[0] is the wall time of the whole call.  Results meet the same
 * bar against the definition as glasso_solve but are not bitwise equal to it (the
 * reductions run in another order).  INVALID_ARG also for n[i] > GLASSO_SMALL_MAX_N. */
#define GLASSO_SMALL_MAX_N 64
glasso_err glasso_solve_small(glasso_handle h, int count, const double* const* S, const int64_t* n,
                              const double* lambda, double tol, double* const* A, double* const* W,
                              glasso_info* info, void* stream);

/* glasso_solve_small without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same persistent launch as glasso_solve_small, but its
 * scratch (per-workgroup matrix slots, problem descriptors, outputs, the
 * work-queue counter) lives in a fixed array of the library's device data,
 * GLASSO_SMALL_STATIC_BYTES (about 51 MB) on every GPU the library runs on, held
 * until the process ends, instead of in a handle's workspace; at most 256
 * workgroups (one per compute unit).  No handle: opt gives the options (NULL =
 * defaults); the host-side staging arrays are static as well.
 *   count  1 .. GLASSO_SMALL_STATIC_MAX_COUNT problems; INVALID_ARG beyond
 *   other arguments, outputs and errors as for glasso_solve_small; HIP when the
 *   array's device address cannot be obtained.
 * All calls on one GPU share that GPU's array, which keeps the last call's
 * contents (the kernel rewrites every part it reads first).  Calls overlapping
 * on one GPU would race on it: the library serialises the calls of a process
 * with a lock, so calls from several host threads wait for each other.  Results
 * are bitwise those of glasso_solve_small. */
#define GLASSO_SMALL_STATIC_MAX_COUNT 16384
#define GLASSO_SMALL_STATIC_BYTES 53084416u
glasso_err glasso_solve_small_static(const glasso_options* opt, int count, const double* const* S,
                                     const int64_t* n, const double* lambda, double tol, double* const* A,
                                     double* const* W, glasso_info* info, void* stream);

/* Tile autotuner: for problems of size n solved `count` at a time, time the
 * Cholesky, triangular inverse and LAUUM (and, with opt.precision FP64, the
 * A Z A product) of identity matrices under each candidate tile policy
 * {0, 64, 256, 1024, never} and record the fastest for this device, padded size
 * and count for the rest of the process (solves with GLASSO_TILES_AUTO use it).
 * *policy (host, may be NULL) receives the choice.  Allocates the workspace for
 * (n, count) like a solve; runs on `stream` and waits for it.
 * Errors: INVALID_ARG (n < 1, count < 1), OOM, HIP. */
glasso_err glasso_autotune(glasso_handle h, int64_t n, int count, int* policy, void* stream);

/* Solve the graphical lasso for one S (Alg. 1 of the paper, Sec. 6 settings).
 *   S      n x n empirical covariance (device, read-only, lower triangle read)
 *   lambda regularisation weight (alpha in the paper), > 0
 *   tol    stopping tolerance on ||Z||_1 / ||A||_1, > 0
 *   A      n x n output (device): the solution, full symmetric.  With
 *          opt.warm_start it is also the input iterate A^(0).
 *   W      n x n output (device, may be NULL): A^{-1}, full symmetric, FP64
 *   info   output (host, may be NULL)
 * Reaching max_iter or failing the line search is reported in info->status and
 * is not an error; the last accepted iterate is returned.
 * Errors: INVALID_ARG (n < 1, lambda <= 0, tol <= 0, NULL S/A, non-finite S,
 * S_ii + lambda <= 0), NOT_PD (warm start not PD), OOM, HIP. */
glasso_err glasso_solve(glasso_handle h, const double* S, int64_t n, double lambda, double tol,
                        double* A, double* W, glasso_info* info, void* stream);

/* Solve `count` independent problems (e.g. a regularisation path: one S, many
 * lambda) in batched launches: problems of equal n advance together, one pISTA
 * iteration per round of launches, each with its own lambda, iterate, line search
 * (its own step size, same backtracking as glasso_solve) and stopping test;
 * problems that stop are skipped by later launches.  Problems of different n run
 * group after group.
 *   S[i]   device pointer to problem i's S (n[i] x n[i]); entries may alias
 *   n[i], lambda[i]  size and regularisation weight of problem i
 *   A[i], W[i]       outputs as in glasso_solve (W may be NULL, or W[i] NULL);
 *                    with opt.warm_start A[i] also holds problem i's A^(0)
 *   info   host array of count entries (may be NULL)
 * Results are bitwise identical to solving each problem alone with glasso_solve
 * (every kernel treats the problems of a batch independently).
 * Errors: as glasso_solve, for any problem. */
glasso_err glasso_solve_batched(glasso_handle h, int count, const double* const* S, const int64_t* n,
                                const double* lambda, double tol, double* const* A, double* const* W,
                                glasso_info* info, void* stream);

/* ------------------------------------------------------------------------------
 * Step-level entry points: each runs one step of the per-iteration path on
 * caller buffers (device, n x n, row-major, ld n), so every step can be checked
 * on its own.  They use the handle's workspace and synchronise the stream.
 * -------------------------------------------------------------------------- */

/* Sample covariance, the solver's input (Sec. 3.1, eq. empirical_cov):
 * S = (1/m) sum_i (y_i - mu)(y_i - mu)^T over the m samples y_i, the rows of Y
 * (device, m x n, row-major, ld n), with mu = (1/m) sum_i y_i when center != 0
 * and mu = 0 otherwise (samples of known zero mean).  S (device, n x n, full
 * symmetric) is formed as the lower triangle of one FP64 MFMA product and
 * mirrored.  The handle keeps a workspace of (m + n) x n + n doubles (rounded up
 * to whole tiles) for the padded samples and product; it is freed with the handle.
 * Errors: INVALID_ARG for null pointers, m < 1 or n < 1; OOM. */
glasso_err glasso_covariance(glasso_handle h, const double* Y, int64_t m, int64_t n, int center, double* S,
                             void* stream);

/* Seeded synthetic workloads on the device (the experiments' setup, Sec. 6.1.1:
 * a sparse precision matrix, samples drawn from its Gaussian model, their
 * covariance), so that inputs need no host-side generation.  Random numbers come
 * from the counter-based generator Philox4x32-10 (Salmon et al., SC 2011) with
 * key = (seed mod 2^32, seed / 2^32); every value is a pure function of the seed
 * and its position.
 *   kind   GLASSO_GEN_RANDOM_SPARSE: each pair i < j is an edge with probability
 *          min(1, 10 / (n - 1)) (about ten off-diagonal nonzeros per row), value
 *          +-U(0.5, 1) with a random sign, A_ii = sum_j |A_ij| + 0.1;
 *          GLASSO_GEN_CHAIN: A_ii = 1.25, A_{i,i+1} = -0.5 (the seed is unused).
 *   n, m   variables and samples (m is ignored when only A_true is asked for)
 *   A_true n x n output (device, may be NULL): the precision matrix
 *   Y      m x n output (device, may be NULL): the samples as rows,
 *          x_r = L^{-T} z_r with A_true = L L^T and z_r standard normal
 *          (Box-Muller of 53-bit uniforms), so Cov(x) = A_true^{-1}
 *   S      n x n output (device, may be NULL): S = Y^T Y / m (known zero mean,
 *          eq. empirical_cov without centring), full symmetric
 *   lambda_max  host output (may be NULL): max_{i != j} |S_ij|
 * At least one output must be given.  The handle keeps a workspace of about
 * (2.3 n^2 + 2 m n) doubles (padded to whole tiles).
 * Errors: INVALID_ARG (bad kind, n < 1, m < 1 with sample outputs, no output),
 * NOT_PD (cannot happen for these diagonally dominant recipes), OOM, HIP. */
typedef enum { GLASSO_GEN_RANDOM_SPARSE = 0, GLASSO_GEN_CHAIN = 1 } glasso_gen_kind;
glasso_err glasso_generate(glasso_handle h, int kind, int64_t n, int64_t m, uint64_t seed, double* A_true, double* Y,
                           double* S, double* lambda_max, void* stream);

/* Lower Cholesky factor L of SPD A (the PD test of condition t_cond_pd,
 * Sec. 4.3.2): L (n x n, output) gets L in its lower triangle and zeros above.
 * *info = 0 on success, else the 1-based column of the first non-positive or
 * non-finite pivot.  *logdet (may be NULL) = 2 sum log L_ii (eq. log_MLE). */
glasso_err glasso_cholesky(glasso_handle h, const double* A, int64_t n, double* L, int64_t* info,
                           double* logdet, void* stream);

/* W = A^{-1} (full symmetric) from the Cholesky factor of A (eq. grad_hessian
 * needs it for g = S - W).  With opt.w_mixed == 1 the triangular inverse and the
 * product V^T V run with FP32 accuracy on BF16 MFMA, as in the mixed-W iterations
 * of glasso_solve.
 * Errors: NOT_PD when A is not PD. */
glasso_err glasso_inverse(glasso_handle h, const double* A, int64_t n, double* W, void* stream);

/* One gradient pass (eq. grad_hessian of Sec. 3.2; eqs. free_set, M of Sec. 4.1; eq. G+):
 * g = S - W, M = (A != 0) | (|g| > lambda), G = sign(A) where A != 0 else
 * -sign(g); outputs Z = (g + lambda G) (.) M (n x n, full symmetric) and
 * GM = G (.) M (n x n int8).  kkt (host, 4 doubles, may be NULL) receives
 * ||Z||_1, ||A||_1, ||Z||_F, max|Z|.  S, W, A are read through their lower triangles. */
glasso_err glasso_gradient_pass(glasso_handle h, const double* S, const double* W, const double* A,
                                int64_t n, double lambda, double* Z, int8_t* GM, double* kkt,
                                void* stream);

/* Preconditioned product P = A Z A (eq. b's first two terms:
 * A(g.M)A + lambda A(G.M)A = A Z A), lower triangle exact, full symmetric output.
 * precision selects the FP64, FP32 or BF16x3 product. */
glasso_err glasso_precond_product(glasso_handle h, const double* A, const double* Z, int64_t n,
                                  int precision, double* P, void* stream);

/* Trial point of the line search (eqs. c, b, d_sol; masked update of Alg. 1):
 * C_ij = lambda (A_ii A_jj + A_ij^2) (i != j), lambda A_ii^2 (i = j);
 * B = P - C (.) GM;  At = M (.) SoftThreshold(A - t B, t C), M = (GM != 0).
 * sums (host, 2 doubles, may be NULL) receive sum S (.) (At - A) and
 * sum (|At| - |A|).  At is n x n full symmetric. */
glasso_err glasso_trial_point(glasso_handle h, const double* A, const double* P, const double* S,
                              const int8_t* GM, int64_t n, double lambda, double t, double* At,
                              double* sums, void* stream);

/* Trial point of a G-ISTA step (eq. proximal_gen with H = I, Sec. 3.2):
 * g = S - W, At = SoftThreshold(A - t g, t lambda) on the free set M = (GM != 0)
 * (zero elsewhere, where the step gives exactly zero), n x n full symmetric.
 * sums (host, 4 doubles, may be NULL) receive sum S (.) (At - A), sum (|At| - |A|),
 * sum W (.) (At - A) and ||At - A||_F^2.  A, S, W (n x n, symmetric, lower
 * triangles read) and GM (n x n int8, from glasso_gradient_pass) are device
 * buffers; At is a device buffer the caller owns.
 * Errors: INVALID_ARG for a null handle or buffer, n < 1, lambda <= 0 or t <= 0. */
glasso_err glasso_gista_trial_point(glasso_handle h, const double* A, const double* S, const double* W,
                                    const int8_t* GM, int64_t n, double lambda, double t, double* At,
                                    double* sums, void* stream);

/* The preconditioned product as a solve forms it when dense_product is 0 (the
 * sampled sparse form; the paper's design forms A Z A densely, Sec. 4.3.3): P_ij =
 * (A Z A)_ij in FP64 for every (i, j) with GM_ij != 0 and P_ij = 0 elsewhere, n x n
 * full symmetric (the trial point, eq. d_sol, reads P only there).  The sparse
 * form serves the call when every row of A has at most 16 nonzeros and every row
 * of GM at most 64 nonzeros on or left of the diagonal; otherwise the FP64 GEMM
 * pair forms the same entries.  *used (host, may be NULL) = 1 when the sparse form
 * served the call, else 0.  A and Z (n x n, symmetric) and GM (n x n int8) are
 * device buffers read in full; P is a device buffer the caller owns.
 * Errors: INVALID_ARG for a null handle or buffer or n < 1. */
glasso_err glasso_sparse_product(glasso_handle h, const double* A, const double* Z, const int8_t* GM,
                                 int64_t n, double* P, int* used, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GLASSO_H */
