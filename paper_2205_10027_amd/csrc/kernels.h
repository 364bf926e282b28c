// Host-side launchers of the gfx950 kernels (internal to libglasso).
// All matrices are row-major with leading dimensions in elements; every launcher
// enqueues work on `stream` and returns 0 on success, -1 on a shape error and -2
// when the launch itself failed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace glasso {

// A batch of independent problems of equal padded size: problem z uses
// operands offset by z * stride (elements) and abort/skip flag [z].
struct ZBatch {
  int count = 1;
  int64_t sA = 0, sB = 0, sC = 0;
  // Optional zero-block skipping for the Cholesky updates C -= A B^T, where A and
  // B are rows of the factor's finished panels: nz[z * snz + s * nz_chunks + c]
  // says whether rows 64c..64c+63 of 128-column panel s hold a nonzero (bit 0 in
  // the panel's columns 0..63, bit 1 in 64..127; nonzero = either).  A tile
  // whose operand rows (global rows nz_row0 + m0.., nz_col0 + n0..) meet a zero
  // block in every panel of its K range (global columns nz_k0..) adds nothing and
  // leaves C untouched.  nz == nullptr: no skipping.
  const uint8_t* nz = nullptr;
  int64_t snz = 0;
  int nz_chunks = 0, nz_row0 = 0, nz_col0 = 0, nz_k0 = 0;
};

// ---------------------------------------------------------------- dense kernels
int gemm_f64(hipStream_t stream, int ta, int tb, int M, int N, int K, double alpha,
             const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
             int64_t ldc, int lower_out, int a_tri, int b_tri, const int* abort_flag,
             int batch = 1, int64_t sA = 0, int64_t sB = 0, int64_t sC = 0, int role = 0,
             const ZBatch& zb = ZBatch(), int in_place = 0);

// Launches of gemm_f64 with fewer than `tiles` 128x128 output tiles (over the
// whole grid, batch included) use 64x64 tiles instead.  Per calling thread (each
// handle sets its own before its launches); results do not depend on it.
void set_gemm_f64_small_tile_below(int tiles);
int get_gemm_f64_small_tile_below();

// C = A B^T on FP32 MFMA with FP32 accumulation (A: M x K, B: N x K, row-major
// FP32); C is float or (c_is_double) double; lower_out as in gemm_f64.
int gemm_f32_nt(hipStream_t stream, int M, int N, int K, const float* A, int64_t lda,
                const float* B, int64_t ldb, void* C, int64_t ldc, int c_is_double,
                int lower_out, const ZBatch& zb = ZBatch(), const int* skip = nullptr);
int f64_to_f32(hipStream_t stream, const double* src, float* dst, int64_t count);

// C = A B^T as three BF16 products with FP32 accumulation; A (M x K) and B (N x K)
// in the split layout of gemm_bf16x3.hip (4 bytes per element, row stride 4 ld
// bytes).  C is written in split layout, or (c_is_double) as FP64; lower_out as
// in gemm_f64 (FP64 output only).  ZBatch strides are in elements.
int gemm_bf16x3_nt(hipStream_t stream, int M, int N, int K, const void* A, int64_t lda, const void* B,
                   int64_t ldb, void* C, int64_t ldc, int c_is_double, int lower_out,
                   const ZBatch& zb = ZBatch(), const int* skip = nullptr);
// FP64 -> split layout (count a multiple of 8)
int split_bf16x2(hipStream_t stream, const double* src, void* dst, int64_t count, const int* skip = nullptr);

// V = inv(L) and V^T as three-part bf16 splits (6 bytes per element) by recursive
// doubling from the factor L (FP64, lower, intact) and its diagonal-block inverses
// Dinv; tmp needs np^2/4 split elements.  Strides: sL, sD elements; sT, sTt, sTmp
// bytes per problem.
// nz (may be null): the zero-block map of L's factorisation (FactorBatch::nz layout,
// snz bytes per problem); products over L's zero blocks are then skipped.
int trtri_bf16x6(hipStream_t stream, const double* L, const double* Dinv, int64_t np, void* T, void* Tt, void* tmp,
                 int count, int64_t sL, int64_t sD, int64_t sT, int64_t sTt, int64_t sTmp, const int* skip,
                 const uint8_t* nz = nullptr, int64_t snz = 0);
// C = tril(A B^T) in FP64 from three-part splits (six BF16 products, FP32 accuracy);
// N x N output, K inner; k_from_row starts tile row m0's K range at m0.  Strides of
// the batch: bytes for A and B, elements for C.
int gemm_bf16x6_lower(hipStream_t stream, int N, int K, const void* A, int64_t lda, const void* B, int64_t ldb,
                      double* C, int64_t ldc, int k_from_row, int count, int64_t zA_bytes, int64_t zB_bytes,
                      int64_t zC, const int* skip);

// Strides (elements) between the problems of a batched factorisation: the
// matrix, its diagonal vector and its diagonal-block inverses.
struct FactorBatch {
  int count = 1;
  int64_t sA = 0, sdL = 0, sDinv = 0;
  // optional per-problem map of the nonzero 64-row blocks of each finished
  // 128-column panel below its diagonal block (layout of ZBatch::nz); the
  // factorisation's updates skip the tiles it shows to be zero
  uint8_t* nz = nullptr;
  int64_t snz = 0;
  int nz_chunks = 0;
};

// In-place lower Cholesky of the n x n (n multiple of 128) matrix A.  Writes the
// diagonal of L to dL, the inverses of its 128x128 diagonal blocks to Dinv
// (n/128 blocks of 128x128, zeros above the diagonal) and, on a non-positive or
// non-finite pivot, info = global column + 1.  A problem whose info is nonzero
// on entry (or becomes nonzero) is skipped by every later kernel.  info has one
// entry per problem of the batch.  With finish == 0 the factor is left unfinished:
// the strict lower part of each 128x128 diagonal block of L sits transposed in the
// block's strict upper triangle (dL is final) until finish_factor runs; the line
// search only needs dL of its trial points.
// Optional timing of the leaf launches of one factorisation: events recorded
// around each leaf launch (two per launch, while used + 2 <= cap) and the
// launches' algorithmic flops (for `active` problems of actual size n: per step at
// column k, nb = min(128, n - k) gives nb^3/3 for the block and (n - k - nb) nb^2
// for the panel solve).
struct LeafTimer {
  hipEvent_t* ev = nullptr;
  int cap = 0, used = 0;
  int64_t n = 0;
  int active = 1;
  double flops = 0.0;
};
int potrf_lower(hipStream_t stream, double* A, int64_t lda, int n, double* dL, double* Dinv,
                int* info, const FactorBatch& fb = FactorBatch(), int finish = 1, LeafTimer* timer = nullptr);
// Places the diagonal blocks of a factor left by potrf_lower(finish = 0) and
// writes their inverses to Dinv, for the problems with skip == 0.  Idempotent as
// long as L has not been overwritten in between (trtri_lower does that).
int finish_factor(hipStream_t stream, double* A, int64_t lda, int n, const double* dL, double* Dinv,
                  const int* skip, const FactorBatch& fb = FactorBatch());

// In-place inverse of the lower-triangular n x n factor L given its diagonal-block
// inverses (from potrf_lower).  tmp needs n*n/4 doubles per problem (stride sTmp).
// abort_flag (per problem, may be null) skips problems.
int trtri_lower(hipStream_t stream, double* L, int64_t ld, int n, const double* Dinv, double* tmp,
                const int* abort_flag, const FactorBatch& fb = FactorBatch(), int64_t sTmp = 0);

// W (lower triangle) = V^T V for lower-triangular V (the LAUUM product).
int lauum_lower(hipStream_t stream, const double* V, int64_t ldv, double* W, int64_t ldw, int n,
                const int* abort_flag = nullptr, const FactorBatch& fb = FactorBatch(),
                int64_t sW = 0);

// ---------------------------------------------------------------- elementwise passes
int copy_in_padded(hipStream_t stream, const double* src, int64_t n, double* dst, int64_t np,
                   int64_t* bad_count_dev, double lam, int check);
// A^(0) = diag(1/(S_ii + lam)) (identity padding) with its factor L, diag(L) in dL,
// the diagonal-block inverses of L in Dinv and W = A^-1, all in closed form.
int init_diag(hipStream_t stream, const double* Sp, int64_t n, int64_t np, double lam, double* A,
              double* L, double* dL, double* Dinv, double* W);
// P = A Z A for diagonal A (elementwise, FP64), problems with skip == 0.
int diag_product(hipStream_t stream, const double* A, const double* Z, double* P, int64_t np, int count,
                 const int* skip);

// Sampled sparse form of the preconditioned product (sparse_product.hip).  Per
// problem: column lists of the iterate's rows (at most SPARSE_KA nonzeros) and of
// the free set's rows left of and on the diagonal (at most SPARSE_KM), their
// lengths, and the per-problem choice: dense[b] = 1 when some row is longer (the
// dense GEMM pair runs, with dskip[b] = 0), else 0 (dskip[b] = 1).  All arrays
// hold `rows` (>= np) rows per problem.
constexpr int SPARSE_KA = 16;
constexpr int SPARSE_KM = 64;
struct SparseRows {
  int* colA = nullptr;     // rows x SPARSE_KA
  double* valA = nullptr;  // rows x SPARSE_KA
  int* colM = nullptr;     // rows x SPARSE_KM
  int* cnt = nullptr;      // rows x 2: nonzeros of A's row, lower free entries of the row
  int* dense = nullptr;    // per problem
  int* dskip = nullptr;    // per problem: skip flag for the dense pair
  int64_t rows = 0;
};
// P_ij = (A Z A)_ij for (i, j) in the free set (GM != 0), j <= i < n, FP64, for
// the problems with skip == 0 whose rows are short enough; writes SC_DENSE_PRODUCT
// of each such problem's scalars.  Z: FP64 (z_split = 0) or the bf16 hi + lo split
// layout (z_split = 1); sZ = bytes between problems' Z.
int sparse_product(hipStream_t stream, const double* A, const int8_t* GM, const void* Z, int z_split, int64_t sZ,
                   int64_t n, int64_t np, int count, const int* skip, const SparseRows& r, double* scal, double* P);
// P_e = 0 where GM_e == 0, for `count` elements
int mask_free_set(hipStream_t stream, double* P, const int8_t* GM, int64_t count);
int pad_copy_f64(hipStream_t stream, const double* src, int64_t n, int64_t np, double* dst,
                 double* dst2, int pad_diag);
int pad_copy_i8(hipStream_t stream, const int8_t* src, int64_t n, int64_t np, int8_t* dst);
int unpad_copy_i8(hipStream_t stream, const int8_t* src, int64_t np, int8_t* dst, int64_t n);
int sum_log(hipStream_t stream, const double* d, int64_t n, double* out);
// nlog: number of diagonal entries of the factor that enter log det (n in the solver)
// Batch of problems for the elementwise passes (problem = grid.y): element
// strides of S (0 = one shared S) and of the other np x np buffers, of the
// diagonal vectors, and optional per-problem lambda, step size and skip flags
// (device arrays; null = the scalar argument / no skipping).
struct PassBatch {
  int count = 1;
  int64_t sS = 0, sM = 0, sV = 0;
  const double* lam = nullptr;
  const double* t = nullptr;
  const int* skip = nullptr;
  // trial passes: batch entry y is a trial slot of problem y / div; the problem's
  // inputs (A, P, S, GM, diag(L), lambda) are read at that index, the slot's own
  // step size, skip flag and outputs at y
  int div = 1;
};

// Z (FP64, may be null) and/or Zs, its two-part bf16 split (4 bytes per element,
// per-problem byte stride sZs; may be null).
// Aprev (may be null; per-problem stride pb.sM): the previous iterate, for
// SC_DW_NEW = sum W (.) (A - Aprev), the second half of the Barzilai-Borwein
// denominator of G-ISTA.
int pass_grad(hipStream_t stream, const double* S, const double* W, const double* A,
              const double* dL, int64_t n, int64_t nlog, int64_t np, double lam, double* Z,
              int8_t* GM, double* part, double* scal, const PassBatch& pb = PassBatch(),
              void* Zs = nullptr, int64_t sZs = 0, const double* Aprev = nullptr);
// info_reset[b] is set to 0 for the problems the pass handles and to -1 for the
// skipped ones, so that the Cholesky that follows skips them too.
// W (may be null): with it the pass also sums W (.) (At - A) for the predicted
// change of the sufficient-decrease test (finish_trial writes SC_PRED, SC_DW).
// gista != 0: the trial point is the G-ISTA step ST(A - t (S - W), t lam) instead
// of eq. d_sol (W required, P unread); finish_trial then writes SC_QB.
int pass_trial(hipStream_t stream, const double* A, const double* P, const double* S,
               const int8_t* GM, int64_t n, int64_t np, double lam, double t, double* At,
               double* Lt, double* part, int* info_reset, const PassBatch& pb = PassBatch(),
               const double* W = nullptr, int gista = 0);
// t: the step size when pb.t is null (for SC_QB)
int finish_trial(hipStream_t stream, const double* part, int nparts, const double* dL,
                 const double* dLt, const int* info, int64_t n, double lam, double* scal,
                 const PassBatch& pb = PassBatch(), double t = 1.0);
// for every problem b with accept[b] = j + 1 != 0 copy trial slot j's point, its
// (unfinished) factor and diagonal over problem b's current ones; the diagonal-block
// inverses are formed when the factor is finished
// (Aprev, may be null: receives problem b's replaced iterate first)
int accept_trials(hipStream_t stream, const int* accept, int count, double* A, const double* At,
                  double* L, const double* Lt, double* dL, const double* dLt, int64_t np,
                  double* Aprev = nullptr);
int sym_copy_out(hipStream_t stream, const double* src, int64_t np, double* dst, int64_t n,
                 int mode);
// sample covariance (eq. empirical_cov): column means of Y (m x n row-major) into mu;
// Yp (mp x np) = Y - 1 mu^T with zero padding (mu may be null: no centring)
int column_mean(hipStream_t stream, const double* Y, int64_t m, int64_t n, double* mu);
int center_pad(hipStream_t stream, const double* Y, int64_t m, int64_t n, const double* mu, double* Yp, int64_t mp,
               int64_t np);
// ---- seeded synthetic workloads (generate.hip)
constexpr int GEN_RANDOM_SPARSE = 0, GEN_CHAIN = 1;  // glasso_gen_kind
// lower triangle of the padded precision matrix of the recipe (zeros above, the
// identity in the padding)
int gen_precision_lower(hipStream_t stream, double* A, int64_t n, int64_t np, int kind, uint64_t seed);
// Z (mp x np, ld np): standard normals for r < m, c < n, zero padding
int gen_normals(hipStream_t stream, double* Z, int64_t m, int64_t n, int64_t mp, int64_t np, uint64_t seed);
int copy_rect(hipStream_t stream, const double* src, int64_t lds, double* dst, int64_t rows, int64_t cols);
// *out = max_{j < i < n} |S_ij| of the padded S; part: 256 doubles of scratch
int offdiag_absmax(hipStream_t stream, const double* S, int64_t n, int64_t np, double* part, double* out);

// ---- block-diagonal screening (screen.hip)
// One block (connected component of {|S_ij| > lambda}) of a problem: its k
// variables idx[0..k) (device, ascending) of the full matrices S, A, W (ld), and
// its packed k x k copies Sk, Ak, Wk; off = its first element in the packing.
struct ScreenBlock {
  const double* S;
  double* A;
  double* W;
  int64_t ld;
  const int* idx;
  int k;
  int64_t off;
  double *Sk, *Ak, *Wk;
};
// parent[i] = the smallest index of i's component (n x n S, ld lds); *err |= 1 if a
// union did not settle (never expected)
int screen_components(hipStream_t stream, const double* S, int64_t n, int64_t lds, double lam, int* parent,
                      int* err);
// which = 0: Sk <- S on the block; 1: Ak <- A (a warm start)
int gather_blocks(hipStream_t stream, const ScreenBlock* blk, int count, int64_t total, int which);
// A (and W) on the block <- Ak (Wk)
int scatter_blocks(hipStream_t stream, const ScreenBlock* blk, int count, int64_t total, int with_w);
// out[b] = sum |Ak| of block b
int block_abs_sums(hipStream_t stream, const ScreenBlock* blk, int count, double* out);
int zero_fill(hipStream_t stream, double* X, int64_t count);

// ---- persistent small-problem solver (n <= SMALL_MAX_N, one workgroup per problem)
constexpr int SMALL_MAX_N = 64;
constexpr int GLASSO_CONVERGED_DEV = 0, GLASSO_MAX_ITER_DEV = 1, GLASSO_LS_FAILED_DEV = 2;  // glasso_status
struct SmallProblem {
  const double* S;  // n x n (device), lower triangle read
  double* A;        // n x n out (in: the starting iterate with warm_start)
  double* W;        // n x n out, may be null
  int64_t n;
  double lam;
};
struct SmallOut {
  double objective, kkt_rel1, kkt_fro, kkt_max, nnz;
  int iterations, ls_trials, status, fallback_steps;
  int error;  // 0 ok, 1 warm start not PD, 2 invalid S, 3 initial iterate not PD
  int pad;
};
struct SmallParams {
  const SmallProblem* prob;
  SmallOut* out;
  int count;
  double* ws;  // per workgroup: 6 x 64 x 64 doubles (S, A, At, W, Z, P)
  int8_t* gm;  // per workgroup: 64 x 64
  int* next;   // work queue: the next problem index to take (set to the grid size by solve_small)
  double tol, t0, shrink, t_floor, t_min;
  double sigma;  // sufficient-decrease fraction (0: strict decrease)
  int max_iter, warm_start;
};
constexpr int64_t SMALL_WS_DOUBLES = 6 * 64 * 64;
constexpr int64_t SMALL_GM_BYTES = 64 * 64;
int solve_small(hipStream_t stream, const SmallParams& p, int grid);

// X_b = identity for count consecutive np x np matrices
int fill_identity(hipStream_t stream, double* X, int64_t np, int count);
int mirror_lower(hipStream_t stream, double* M, int64_t np);
int power_iteration(hipStream_t stream, const double* M, int64_t n, int64_t np, double* vec,
                    double* out, int iters);

// device scalar slots written by the passes
enum ScalarSlot {
  SC_SUM_ABS_Z = 0,
  SC_SUM_Z2,
  SC_MAX_ABS_Z,
  SC_SUM_ABS_A,
  SC_NNZ_A,
  SC_SUM_SA,
  SC_LOGDET,
  SC_OBJECTIVE,
  SC_KKT_REL1,
  SC_KKT_FRO,
  SC_DF,
  SC_DTR,
  SC_DL1,
  SC_DLOG,
  SC_TRIAL_INFO,
  SC_NNZ_AT,
  SC_POWER_A,
  SC_POWER_W,
  SC_DENSE_PRODUCT,  // 1: the last product used the dense GEMM pair, 0: the sparse product
  SC_PRED,           // predicted change <g, At - A> + lam (||At||_1 - ||A||_1) (with W given)
  SC_DW,             // sum W (.) (At - A) (with W given)
  SC_D2,             // ||At - A||_F^2
  SC_QB,             // G-ISTA: f(At) - f(A) - <g, At - A> - ||At - A||_F^2 / (2t) (with W given)
  SC_DW_NEW,         // gradient pass with the previous iterate: sum W (.) (A - A_prev)
  SC_COUNT = 24
};

constexpr int GRAD_PARTS = 7;   // per-workgroup partials of pass_grad
constexpr int TRIAL_PARTS = 5;  // per-workgroup partials of pass_trial

inline int64_t pass_tiles(int64_t np) {
  const int64_t T = np / 64;
  return T * (T + 1) / 2;
}

}  // namespace glasso
