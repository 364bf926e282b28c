// C ABI of libglasso: handle, workspace and the pISTA driver (Alg. 1 with the
// Sec. 6 initialisation, line search and stopping rule).  Every arithmetic step
// runs in the kernels of gemm_f64.hip, chol.hip and passes.hip; the host only
// sequences launches and reads back a few scalars (KKT, decrease, pivot status).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/glasso.h"
#include "common.h"
#include "kernels.h"

using namespace glasso;

namespace {

struct Workspace {
  int cap_count = 0;   // problems the buffers were laid out for
  int64_t cap_np = 0;  // padded size the buffers were laid out for
  int count = 0;       // problems of the current call
  int slots = 0;       // line-search trial slots of the current call (>= count)
  int64_t np = 0;      // padded size (leading dimension) of the current call
  void* base = nullptr;
  size_t bytes = 0;
  // per problem b: matrices at + b * np^2, diagonals at + b * np, block inverses at
  // + b * np * 128, pass partials at + b * tiles * 8, scalar slots at + b * SC_COUNT.
  // The trial point and factor (At, Lt, dLt), info, lsskip and t are per trial slot
  // j (slots of problem b: b * slots / count ...); trial scalars at scal_t + j * SC_COUNT.
  double *S = nullptr, *A = nullptr, *At = nullptr, *L = nullptr, *Lt = nullptr, *W = nullptr, *Z = nullptr,
         *X = nullptr, *P = nullptr;
  int8_t* GM = nullptr;
  double *dL = nullptr, *dLt = nullptr, *Dinv = nullptr, *Dinvt = nullptr;
  double* part = nullptr;
  double* scal = nullptr;
  double* scal_t = nullptr;
  int *info = nullptr, *skip = nullptr, *lsskip = nullptr, *accept = nullptr;
  int *skip32 = nullptr, *skip64 = nullptr;  // W with FP32 accuracy / in FP64 (the mixed-W ladder)
  double *lam = nullptr, *t = nullptr;
  int64_t* bad = nullptr;
  double* vec = nullptr;
  SparseRows sp;  // row lists of the sparse product
  uint8_t* nzmap = nullptr;  // zero-block maps of the factorisations (per trial slot)
  int64_t nn() const { return np * np; }
};

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Carve the workspace for `count` problems of padded size np out of one
// allocation (base may be null to only measure).
size_t layout(Workspace& w, int count, int slots, int64_t np, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  const size_t mat = (size_t)count * np * np * sizeof(double);
  const size_t mat_t = (size_t)slots * np * np * sizeof(double);
  w.S = (double*)take(mat);
  w.A = (double*)take(mat);
  w.At = (double*)take(mat_t);
  w.L = (double*)take(mat);
  w.Lt = (double*)take(mat_t);
  w.W = (double*)take(mat);
  w.Z = (double*)take(mat);
  w.X = (double*)take(mat);
  w.P = (double*)take(mat);
  w.GM = (int8_t*)take((size_t)count * np * np);
  w.dL = (double*)take((size_t)count * np * sizeof(double));
  w.dLt = (double*)take((size_t)slots * np * sizeof(double));
  w.Dinv = (double*)take((size_t)count * np * TILE * sizeof(double));
  w.Dinvt = (double*)take((size_t)count * np * TILE * sizeof(double));
  w.part = (double*)take((size_t)slots * pass_tiles(np) * 8 * sizeof(double));
  w.scal = (double*)take((size_t)(count + slots) * SC_COUNT * sizeof(double));
  w.scal_t = base ? w.scal + (size_t)count * SC_COUNT : nullptr;
  w.info = (int*)take(slots * sizeof(int));
  w.skip = (int*)take(count * sizeof(int));
  w.lsskip = (int*)take(slots * sizeof(int));
  w.accept = (int*)take(count * sizeof(int));
  w.skip32 = (int*)take(count * sizeof(int));
  w.skip64 = (int*)take(count * sizeof(int));
  w.lam = (double*)take(count * sizeof(double));
  w.t = (double*)take(slots * sizeof(double));
  w.bad = (int64_t*)take(sizeof(int64_t));
  w.vec = (double*)take(2 * np * sizeof(double));
  const size_t rows = (size_t)count * np;
  w.sp.rows = np;
  w.sp.colA = (int*)take(rows * SPARSE_KA * sizeof(int));
  w.sp.valA = (double*)take(rows * SPARSE_KA * sizeof(double));
  w.sp.colM = (int*)take(rows * SPARSE_KM * sizeof(int));
  w.sp.cnt = (int*)take(rows * 2 * sizeof(int));
  w.sp.dense = (int*)take(count * sizeof(int));
  w.sp.dskip = (int*)take(count * sizeof(int));
  w.nzmap = (uint8_t*)take((size_t)std::max(count, slots) * (np / TILE) * (np / 64));
  return off;
}

// pinned host mirrors of the per-problem device arrays
struct HostMirror {
  int cap = 0;        // problems
  int cap_slots = 0;  // trial slots
  int count = 0;      // problems of the current call (scal_t follows their scalars)
  double* scal = nullptr;
  int *info = nullptr, *skip = nullptr, *lsskip = nullptr, *accept = nullptr;
  int *skip32 = nullptr, *skip64 = nullptr;
  double *lam = nullptr, *t = nullptr;
  int64_t* bad = nullptr;
};

// Captured launch sequences of one engine iteration, valid for one workspace
// shape (the kernels' pointer, size and launch arguments are baked in).
struct GraphKey {
  const void* base = nullptr;
  const void* host = nullptr;
  int64_t np = 0, n = 0, sS = 0;
  int count = 0, slots = 0, precision = -1, tiles = -1;
  bool operator==(const GraphKey& o) const {
    return base == o.base && host == o.host && np == o.np && n == o.n && sS == o.sS && count == o.count &&
           slots == o.slots && precision == o.precision && tiles == o.tiles;
  }
};
struct Graphs {
  GraphKey key;
  hipGraphExec_t head = nullptr, prod = nullptr, trial = nullptr, acc = nullptr, rechk = nullptr;
};

}  // namespace

struct glasso_handle_s {
  glasso_options opt;
  int device = 0;
  Workspace ws;
  HostMirror hm;
  hipEvent_t ev[12] = {};
  std::vector<hipEvent_t> leaf_ev;  // around the leaf launches of one sampled factorisation per call
  hipStream_t cap = nullptr;  // capture stream (graphs option)
  Graphs graphs;
  void* small_base = nullptr;  // workspace of the persistent small-problem solver
  size_t small_bytes = 0;
  void* cov_base = nullptr;  // workspace of glasso_covariance (padded samples, padded S, means)
  size_t cov_bytes = 0;
  void* gen_base = nullptr;  // workspace of glasso_generate
  size_t gen_bytes = 0;
  void* scr_base = nullptr;  // workspace of the screening (labels, packed blocks, block table)
  size_t scr_bytes = 0;
};

namespace {

#define HIP_TRY(expr)                                  \
  do {                                                 \
    if ((expr) != hipSuccess) return GLASSO_ERR_HIP;   \
  } while (0)
#define K_TRY(expr)                                    \
  do {                                                 \
    int _rc = (expr);                                  \
    if (_rc == -1) return GLASSO_ERR_INTERNAL;         \
    if (_rc) return GLASSO_ERR_HIP;                    \
  } while (0)

void free_host(HostMirror& m) {
  if (m.scal) (void)hipHostFree(m.scal);
  m = HostMirror();
}

// host arrays: per problem (skip, accept, skip32, skip64, lam) or per trial slot
// (scalars after the problems' own, info, lsskip, t)
glasso_err ensure_host(glasso_handle h, int count, int slots) {
  HostMirror& m = h->hm;
  m.count = count;
  if (m.scal && m.cap >= count && m.cap_slots >= slots) return GLASSO_OK;
  const int c = std::max(count, m.cap), sl = std::max({slots, count, m.cap_slots});
  free_host(m);
  const size_t bytes = (size_t)(c + sl) * SC_COUNT * sizeof(double) + (size_t)(c + sl) * sizeof(double) +
                       (size_t)(5 * c + 2 * sl) * sizeof(int) + 64;
  char* p = nullptr;
  if (hipHostMalloc((void**)&p, bytes, hipHostMallocDefault) != hipSuccess) return GLASSO_ERR_HIP;
  m.cap = c;
  m.cap_slots = sl;
  m.count = count;
  m.scal = (double*)p;  // problems' scalars, then the trial slots' (placed at scal + count * SC_COUNT)
  m.lam = m.scal + (size_t)(c + sl) * SC_COUNT;
  m.t = m.lam + c;
  m.info = (int*)(m.t + sl);
  m.lsskip = m.info + sl;
  m.skip = m.lsskip + sl;
  m.accept = m.skip + c;
  m.skip32 = m.accept + c;
  m.skip64 = m.skip32 + c;
  m.bad = (int64_t*)(((uintptr_t)(m.skip64 + c) + 7) & ~uintptr_t(7));
  return GLASSO_OK;
}

// The zero fill of a new allocation is ordered on `st`, the stream of the call
// that uses the workspace: a plain hipMemset runs on the null stream, which is not
// ordered with non-blocking caller streams and could land after the first kernels.
glasso_err ensure_workspace(glasso_handle h, int count, int64_t np, hipStream_t st, int slots = 0) {
  Workspace& w = h->ws;
  slots = std::max(slots, count);
  glasso_err e = ensure_host(h, count, slots);
  if (e) return e;
  if (w.base && w.cap_count >= count && w.cap_np >= np &&
      (size_t)w.cap_count * w.cap_np * w.cap_np >= (size_t)count * np * np) {
    // re-carve the same allocation for this (count, slots, np): every buffer fits
    Workspace probe;
    if (layout(probe, count, slots, np, nullptr) <= w.bytes) {
      layout(w, count, slots, np, (char*)w.base);
      w.count = count;
      w.slots = slots;
      w.np = np;
      return GLASSO_OK;
    }
  }
  if (w.base) {
    (void)hipFree(w.base);
    w = Workspace();
  }
  Workspace probe;
  const size_t bytes = layout(probe, count, slots, np, nullptr);
  void* base = nullptr;
  if (hipMalloc(&base, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return GLASSO_ERR_OOM;
  }
  if (hipMemsetAsync(base, 0, bytes, st) != hipSuccess) {
    (void)hipFree(base);
    return GLASSO_ERR_HIP;
  }
  layout(w, count, slots, np, (char*)base);
  w.base = base;
  w.bytes = bytes;
  w.cap_count = count;
  w.cap_np = np;
  w.count = count;
  w.slots = slots;
  w.np = np;
  return GLASSO_OK;
}

FactorBatch factor_batch(const Workspace& w) {
  FactorBatch fb;
  fb.count = w.count;
  fb.sA = w.nn();
  fb.sdL = w.np;
  fb.sDinv = w.np * TILE;
  fb.nz = w.nzmap;
  fb.nz_chunks = (int)(w.np / 64);
  fb.snz = (w.np / TILE) * fb.nz_chunks;
  return fb;
}

// scalar slots and factor status of every problem -> pinned host memory
glasso_err fetch_async(glasso_handle h, hipStream_t st) {
  const Workspace& w = h->ws;
  HIP_TRY(hipMemcpyAsync(h->hm.scal, w.scal, (size_t)(w.count + w.slots) * SC_COUNT * sizeof(double),
                         hipMemcpyDeviceToHost, st));
  HIP_TRY(hipMemcpyAsync(h->hm.info, w.info, (size_t)w.slots * sizeof(int), hipMemcpyDeviceToHost, st));
  return GLASSO_OK;
}
// ... and wait for it
glasso_err fetch(glasso_handle h, hipStream_t st) {
  glasso_err e = fetch_async(h, st);
  if (e) return e;
  HIP_TRY(hipStreamSynchronize(st));
  return GLASSO_OK;
}

void drop_graphs(Graphs& g) {
  for (hipGraphExec_t* x : {&g.head, &g.prod, &g.trial, &g.acc, &g.rechk})
    if (*x) (void)hipGraphExecDestroy(*x);
  g = Graphs();
}

// Record what body(stream) enqueues on the handle's capture stream as a graph.
template <class F>
glasso_err capture_graph(glasso_handle h, hipGraphExec_t* out, F&& body) {
  HIP_TRY(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
  const glasso_err e = body(h->cap);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(h->cap, &g);
  if (e || ce != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return e ? e : GLASSO_ERR_HIP;
  }
  const hipError_t ie = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    *out = nullptr;
    return GLASSO_ERR_HIP;
  }
  return GLASSO_OK;
}
double hscal(glasso_handle h, int b, int slot) { return h->hm.scal[(size_t)b * SC_COUNT + slot]; }
// scalar of trial slot j
double hscal_t(glasso_handle h, int j, int slot) {
  return h->hm.scal[(size_t)(h->hm.count + j) * SC_COUNT + slot];
}

glasso_err push_ints(hipStream_t st, int* dev, const int* host, int count) {
  HIP_TRY(hipMemcpyAsync(dev, host, count * sizeof(int), hipMemcpyHostToDevice, st));
  return GLASSO_OK;
}
glasso_err push_doubles(hipStream_t st, double* dev, const double* host, int count) {
  HIP_TRY(hipMemcpyAsync(dev, host, count * sizeof(double), hipMemcpyHostToDevice, st));
  return GLASSO_OK;
}

bool valid_precision(int p) { return p == GLASSO_FP64 || p == GLASSO_MIXED_FP32 || p == GLASSO_MIXED_BF16X3; }

// Default line-search width: up to LS_WIDTH step sizes per round for padded sizes
// up to LS_WIDE_MAX_NP, where one trial (pass + factorisation) leaves most of the
// chip idle.
constexpr int LS_WIDTH = 4, LS_WIDTH_MAX = 16;
constexpr int64_t LS_WIDE_MAX_NP = 2048;
int ls_width(int64_t np) { return np <= LS_WIDE_MAX_NP ? LS_WIDTH : 1; }

glasso_err check_options(const glasso_options* o) {
  if (!valid_precision(o->precision)) return GLASSO_ERR_INVALID_ARG;
  if (o->max_iter < 0 || o->tile_policy < GLASSO_TILES_AUTO || o->w_mixed < -1 || o->w_mixed > 1)
    return GLASSO_ERR_INVALID_ARG;
  if (o->ls_width < 0 || o->ls_width > LS_WIDTH_MAX) return GLASSO_ERR_INVALID_ARG;
  if (o->dense_product < 0 || o->dense_product > 1) return GLASSO_ERR_INVALID_ARG;
  if (o->screen < 0 || o->screen > 1 || !(o->sigma >= 0.0 && o->sigma < 1.0)) return GLASSO_ERR_INVALID_ARG;
  if (o->method != GLASSO_PISTA && o->method != GLASSO_GISTA) return GLASSO_ERR_INVALID_ARG;
  if (!(o->t0 > 0.0) || !(o->shrink > 0.0 && o->shrink < 1.0) || !(o->t_floor >= 0.0) || !(o->t_min > 0.0))
    return GLASSO_ERR_INVALID_ARG;
  return GLASSO_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
    (void)hipGetLastError();
    return 0.f;
  }
  return ms;
}

// Factor every problem's w.L (lower, in place); info[b] = 0 on entry for all.
glasso_err factor_all(glasso_handle h, hipStream_t st) {
  Workspace& w = h->ws;
  for (int b = 0; b < w.count; ++b) h->hm.info[b] = 0;
  glasso_err e = push_ints(st, w.info, h->hm.info, w.count);
  if (e) return e;
  K_TRY(potrf_lower(st, w.L, w.np, (int)w.np, w.dL, w.Dinv, w.info, factor_batch(w)));
  return fetch(h, st);
}

// W (lower) = A^{-1} with FP32 accuracy for every problem with skip == 0, from its
// factor in w.L (left unchanged) and diagonal-block inverses.
// vev (optional): two events recorded around the V^T V launch alone
glasso_err inverse_f32(Workspace& w, hipStream_t st, const int* skip, hipEvent_t* vev = nullptr) {
  // W = A^-1 with FP32 accuracy on the BF16 matrix cores: V = inv(L) by recursive
  // doubling and W = V^T V, every operand an exact three-part bf16 split of an FP32
  // value (6 bytes per element), six products per element pair.  V split in X,
  // V^T split in P, the doubling's scratch (at most nn/4 elements) after it in P.
  const int64_t nn = w.nn();
  const int64_t zb = nn * (int64_t)sizeof(double);  // per-problem stride of X and P, bytes
  uint8_t* Vs = reinterpret_cast<uint8_t*>(w.X);
  uint8_t* Vts = reinterpret_cast<uint8_t*>(w.P);
  uint8_t* tmp = Vts + nn * 6;
  // one problem with one trial slot: the map holds the last factorisation, which is
  // L's (the accepted trial point, or the start's factor)
  const FactorBatch fb = factor_batch(w);
  const bool map = w.count == 1 && w.slots == 1;
  K_TRY(trtri_bf16x6(st, w.L, w.Dinv, w.np, Vs, Vts, tmp, w.count, nn, w.np * TILE, zb, zb, zb, skip,
                     map ? fb.nz : nullptr, fb.snz));
  if (vev) HIP_TRY(hipEventRecord(vev[0], st));
  K_TRY(gemm_bf16x6_lower(st, (int)w.np, (int)w.np, Vts, w.np, Vts, w.np, w.W, w.np, 1, w.count, zb, zb, nn, skip));
  if (vev) HIP_TRY(hipEventRecord(vev[1], st));
  return GLASSO_OK;
}

// W (lower) = A^{-1} in FP64 from the factor in w.L for every problem with skip ==
// 0: L <- inv(L) in place, W = inv(L)^T inv(L).  tmp: the X buffer.
glasso_err inverse_from_factor(Workspace& w, hipStream_t st, const int* skip) {
  const FactorBatch fb = factor_batch(w);
  K_TRY(trtri_lower(st, w.L, w.np, (int)w.np, w.Dinv, w.X, skip, fb, w.nn()));
  K_TRY(lauum_lower(st, w.L, w.np, w.W, w.np, (int)w.np, skip, fb, w.nn()));
  return GLASSO_OK;
}

// P (lower) = A Z A for every problem with skip == 0: X = A Z^T (Z symmetric),
// P = tril(X A^T) (A symmetric).  Mixed FP32: A and Z are rounded to FP32 (A32,
// Z32 in the X buffer), X32 = A32 Z32^T overwrites Z (no longer needed), and
// P = tril(X32 A32^T) is written in FP64.
// sparse: first try the sampled sparse product (sparse_product.hip); the problems
// it serves are then skipped by the dense pair, which serves the rest.
// gev (optional): two events recorded around the two GEMM launches only
glasso_err precond_product(Workspace& w, hipStream_t st, int precision, const int* skip, int64_t n, bool sparse,
                           hipEvent_t* gev = nullptr, bool z_split_ready = false) {
  const int np = (int)w.np;
  const int64_t nn = w.nn();
  if (sparse) {
    const bool zs = precision == GLASSO_MIXED_BF16X3 && z_split_ready;
    const void* Zsrc = zs ? static_cast<const void*>(reinterpret_cast<const uint8_t*>(w.X) + 4 * nn)
                          : static_cast<const void*>(w.Z);
    K_TRY(sparse_product(st, w.A, w.GM, Zsrc, zs ? 1 : 0, 8 * nn, n, w.np, w.count, skip, w.sp, w.scal, w.P));
    skip = w.sp.dskip;
  }
  ZBatch z;
  z.count = w.count;
  z.sA = z.sB = z.sC = nn;
  if (precision == GLASSO_FP64) {
    if (gev) HIP_TRY(hipEventRecord(gev[0], st));
    K_TRY(gemm_f64(st, 0, 0, np, np, np, 1.0, w.A, np, w.Z, np, 0.0, w.X, np, 0, 0, 0, skip, 1, 0, 0, 0, 1, z));
    K_TRY(gemm_f64(st, 0, 0, np, np, np, 1.0, w.X, np, w.A, np, 0.0, w.P, np, 1, 0, 0, skip, 1, 0, 0, 0, 1, z));
    if (gev) HIP_TRY(hipEventRecord(gev[1], st));
    return GLASSO_OK;
  }
  if (precision == GLASSO_MIXED_FP32) {
    // A32 and Z32 share the X buffer: A32 of problem b at b * 2nn floats, Z32 after it
    float* X32buf = reinterpret_cast<float*>(w.X);
    float* X32 = reinterpret_cast<float*>(w.Z);
    for (int b = 0; b < w.count; ++b) {
      K_TRY(f64_to_f32(st, w.A + b * nn, X32buf + 2 * b * nn, nn));
      K_TRY(f64_to_f32(st, w.Z + b * nn, X32buf + 2 * b * nn + nn, nn));
    }
    ZBatch z1;  // X32 = A32 Z32^T
    z1.count = w.count;
    z1.sA = 2 * nn;
    z1.sB = 2 * nn;
    z1.sC = 2 * nn;  // floats: X32 of problem b inside Z's doubles at b * nn doubles
    if (gev) HIP_TRY(hipEventRecord(gev[0], st));
    K_TRY(gemm_f32_nt(st, np, np, np, X32buf, np, X32buf + nn, np, X32, np, 0, 0, z1, skip));
    ZBatch z2;  // P = tril(X32 A32^T)
    z2.count = w.count;
    z2.sA = 2 * nn;
    z2.sB = 2 * nn;
    z2.sC = nn;
    K_TRY(gemm_f32_nt(st, np, np, np, X32, np, X32buf, np, w.P, np, 1, 1, z2, skip));
    if (gev) HIP_TRY(hipEventRecord(gev[1], st));
    return GLASSO_OK;
  }
  if (precision == GLASSO_MIXED_BF16X3) {
    // split A and Z (4 bytes per element) share the X buffer: A of problem b at
    // b * 2nn elements, Z after it (written there by the gradient pass when
    // z_split_ready); the split X = A Z is written over Z
    uint8_t* As = reinterpret_cast<uint8_t*>(w.X);
    uint8_t* Xs = reinterpret_cast<uint8_t*>(w.Z);
    for (int b = 0; b < w.count; ++b) {
      const int* sb = skip ? skip + b : nullptr;
      K_TRY(split_bf16x2(st, w.A + b * nn, As + 2 * b * nn * 4, nn, sb));
      if (!z_split_ready) K_TRY(split_bf16x2(st, w.Z + b * nn, As + (2 * b + 1) * nn * 4, nn, sb));
    }
    ZBatch z1;  // Xs = A Z^T (Z symmetric)
    z1.count = w.count;
    z1.sA = z1.sB = z1.sC = 2 * nn;
    if (gev) HIP_TRY(hipEventRecord(gev[0], st));
    K_TRY(gemm_bf16x3_nt(st, np, np, np, As, np, As + nn * 4, np, Xs, np, 0, 0, z1, skip));
    ZBatch z2;  // P = tril(X A^T)
    z2.count = w.count;
    z2.sA = z2.sB = 2 * nn;
    z2.sC = nn;
    K_TRY(gemm_bf16x3_nt(st, np, np, np, Xs, np, As, np, w.P, np, 1, 1, z2, skip));
    if (gev) HIP_TRY(hipEventRecord(gev[1], st));
    return GLASSO_OK;
  }
  return GLASSO_ERR_INVALID_ARG;
}

// cond(A_b) ~ lambda_max(A_b) lambda_max(A_b^{-1}) by power iteration; t = (0.9/cond)^2.
// Ritz values approach from below, so each estimate is inflated by 5%.
glasso_err cond_fallback_step(glasso_handle h, hipStream_t st, int b, int64_t n, double* t_out) {
  Workspace& w = h->ws;
  const int64_t nn = w.nn();
  double* scal = w.scal + (size_t)b * SC_COUNT;
  double* Xb = w.X + b * nn;
  K_TRY(power_iteration(st, w.A + b * nn, n, w.np, w.vec, scal + SC_POWER_A, 60));
  HIP_TRY(hipMemcpyAsync(Xb, w.W + b * nn, (size_t)nn * sizeof(double), hipMemcpyDeviceToDevice, st));
  K_TRY(mirror_lower(st, Xb, w.np));
  K_TRY(power_iteration(st, Xb, n, w.np, w.vec, scal + SC_POWER_W, 60));
  glasso_err e = fetch(h, st);
  if (e) return e;
  const double cond = (1.05 * hscal(h, b, SC_POWER_A)) * (1.05 * hscal(h, b, SC_POWER_W));
  *t_out = (0.9 / cond) * (0.9 / cond);
  return GLASSO_OK;
}

// ----------------------------------------------------------------- the engine
//
// Alg. 1 for `count` problems of equal size n at once (the single solve is
// count = 1).  Every phase is one batched launch sequence over the problems
// still iterating; per-problem flags skip the others.  The line search runs in
// rounds: each round evaluates one or more consecutive trial steps per searching
// problem, and each problem backtracks on its own t and takes the first step
// that succeeds, so every problem follows exactly the sequential line search of
// the paper.
// ------------------------------------------------------------------ tile autotuner
// The FP64 GEMMs run 64x64 tiles for launches with fewer than `threshold`
// 128x128 tiles.  The best threshold depends on the padded size and batch count
// (how many tiles the skinny launches of the factorisation have); it is measured
// once per (device, np, count) and kept for the process.  Results do not depend
// on it (both tile edges accumulate every output in the same order).
constexpr int TUNE_CANDIDATES[] = {0, 64, 256, 1024, 1 << 30};



std::mutex g_tune_mu;
std::map<std::tuple<int, int64_t, int>, int> g_tune;

// Times factor + inverse (+ the FP64 A Z A) of identity matrices in the handle's
// workspace under each candidate; the workspace contents are overwritten.  The
// factorisation runs without its zero-block map, so that every update tile does
// its whole K range (with the map, every tile of an identity returns at once and
// the timing would only rank launch overheads).
glasso_err tune_tiles(glasso_handle h, hipStream_t st, int precision, int* chosen) {
  Workspace& w = h->ws;
  FactorBatch dense = factor_batch(w);
  dense.nz = nullptr;
  float best = 0.f;
  int best_thr = TUNE_CANDIDATES[0];
  bool have = false;
  for (int thr : TUNE_CANDIDATES) {
    set_gemm_f64_small_tile_below(thr);
    float t_min = 0.f;
    for (int rep = 0; rep < 2; ++rep) {
      K_TRY(fill_identity(st, w.L, w.np, w.count));
      if (precision == GLASSO_FP64) {
        K_TRY(fill_identity(st, w.A, w.np, w.count));
        K_TRY(fill_identity(st, w.Z, w.np, w.count));
      }
      for (int b = 0; b < w.count; ++b) h->hm.info[b] = 0;
      glasso_err e = push_ints(st, w.info, h->hm.info, w.count);
      if (e) return e;
      HIP_TRY(hipEventRecord(h->ev[0], st));
      K_TRY(potrf_lower(st, w.L, w.np, (int)w.np, w.dL, w.Dinv, w.info, dense));
      e = inverse_from_factor(w, st, nullptr);
      if (e) return e;
      if (precision == GLASSO_FP64) {
        e = precond_product(w, st, precision, nullptr, w.np, false);
        if (e) return e;
      }
      HIP_TRY(hipEventRecord(h->ev[1], st));
      HIP_TRY(hipEventSynchronize(h->ev[1]));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
      if (rep == 0 || ms < t_min) t_min = ms;
    }
    if (!have || t_min < best) {
      best = t_min;
      best_thr = thr;
      have = true;
    }
  }
  *chosen = best_thr;
  return GLASSO_OK;
}

// Set this thread's GEMM tile threshold for the handle's workspace shape: the
// fixed policy of the options, else the tuned one (tuning now if unseen).
// Call right after ensure_workspace and before the workspace is filled.
glasso_err apply_tile_policy(glasso_handle h, hipStream_t st, int precision) {
  if (h->opt.tile_policy >= 0) {
    set_gemm_f64_small_tile_below(h->opt.tile_policy);
    return GLASSO_OK;
  }
  const auto key = std::make_tuple(h->device, h->ws.np, h->ws.count);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      set_gemm_f64_small_tile_below(it->second);
      return GLASSO_OK;
    }
  }
  int thr = 0;
  glasso_err e = tune_tiles(h, st, precision, &thr);
  if (e) return e;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[key] = thr;
  }
  set_gemm_f64_small_tile_below(thr);
  return GLASSO_OK;
}

glasso_err run_engine(glasso_handle h, hipStream_t st, int count, int64_t n, const double* const* S,
                      const double* lam, double tol, double* const* Aout, double* const* Wout, glasso_info* info) {
  const auto t_start = std::chrono::steady_clock::now();
  const glasso_options& o = h->opt;
  const int64_t np = pad_to_tile(n);
  // line-search width: trial slots per problem (several step sizes of the
  // backtracking sequence per round while one round is launch-latency bound)
  int K = o.ls_width > 0 ? o.ls_width : ls_width(np);
  glasso_err e = ensure_workspace(h, count, np, st, count * K);
  if (e == GLASSO_ERR_OOM && o.ls_width == 0 && K > 1) {
    // the automatic width falls back to one step size per round when the extra
    // trial slots do not fit in device memory
    K = 1;
    e = ensure_workspace(h, count, np, st, count);
  }
  if (e) return e;
  const int slots = count * K;
  e = apply_tile_policy(h, st, o.precision);
  if (e) return e;
  Workspace& w = h->ws;
  HostMirror& hm = h->hm;
  const int64_t nn = w.nn();
  const int tiles = (int)pass_tiles(np);

  // S into the padded layout (shared when every problem passes the same pointer);
  // reject non-finite entries and S_ii + lambda <= 0
  bool shared = true;
  double lam_min = lam[0];
  for (int b = 0; b < count; ++b) {
    if (S[b] != S[0]) shared = false;
    lam_min = std::min(lam_min, lam[b]);
  }
  HIP_TRY(hipMemsetAsync(w.bad, 0, sizeof(int64_t), st));
  for (int b = 0; b < (shared ? 1 : count); ++b)
    K_TRY(copy_in_padded(st, S[b], n, w.S + b * nn, np, w.bad, shared ? lam_min : lam[b], 1));
  HIP_TRY(hipMemcpyAsync(hm.bad, w.bad, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (*hm.bad) return GLASSO_ERR_INVALID_ARG;
  const int64_t sS = shared ? 0 : nn;

  for (int b = 0; b < count; ++b) hm.lam[b] = lam[b];
  e = push_doubles(st, w.lam, hm.lam, count);
  if (e) return e;

  // A^(0): warm start or diag(1/(S_ii + lambda)) (Sec. 6); its factor.  The
  // diagonal start comes with its factor and W = A^-1 in closed form.
  const bool diag_start = !o.warm_start;
  for (int b = 0; b < count; ++b) {
    if (o.warm_start)
      K_TRY(pad_copy_f64(st, Aout[b], n, np, w.A + b * nn, w.L + b * nn, 1));
    else
      K_TRY(init_diag(st, w.S + b * sS, n, np, lam[b], w.A + b * nn, w.L + b * nn, w.dL + b * np,
                      w.Dinv + b * np * TILE, w.W + b * nn));
  }
  if (diag_start) {
    for (int b = 0; b < count; ++b) hm.info[b] = 0;
    e = push_ints(st, w.info, hm.info, count);
    if (e) return e;
  } else {
    e = factor_all(h, st);
    if (e) return e;
    for (int b = 0; b < count; ++b)
      if (hm.info[b]) return GLASSO_ERR_NOT_PD;
  }

  std::vector<int> active(count, 1), status(count, GLASSO_MAX_ITER), it(count, 0), trials(count, 0),
      fallbacks(count, 0), ls(count, 0), fb_used(count, 0), gemm_products(count, 0), sparse_products(count, 0),
      prod_b(count, 0), ncand(count, 0),
      last_trials(count, 1), since(count, 0);
  std::vector<double> tb(count, o.t0);  // next step size of each problem's backtracking sequence
  // G-ISTA (eq. proximal_gen with H = I): no preconditioned product; the trial point
  // is ST(A - t g, t lam), accepted when PD with f below its quadratic model; the
  // first step of an iteration is the Barzilai-Borwein step of the last accepted
  // one (bb_num / (bb_dw - SC_DW_NEW), the gradient pass summing W (.) (A - A_prev)
  // against the replaced iterate, which the accept step leaves in P)
  const bool gista = o.method == GLASSO_GISTA;
  std::vector<double> t_next(count, o.t0), bb_num(count, 0.0), bb_dw(count, 0.0);
  std::vector<int> bb_have(count, 0);
  const bool sparse_on = o.dense_product == 0;
  // this iteration's product tries the sparse form (eager launches skip it when every
  // active problem has more than SPARSE_KA nonzeros per row on average, so some row
  // is surely too long; a captured graph always holds both forms)
  bool sparse_now = sparse_on;
  PassBatch pb;
  pb.count = count;
  pb.sS = sS;
  pb.sM = nn;
  pb.sV = np;
  pb.lam = w.lam;
  pb.skip = w.skip;
  pb.t = nullptr;
  PassBatch pt = pb;  // trial passes: slot y is candidate y % K of problem y / K
  pt.count = slots;
  pt.div = K;
  pt.skip = w.lsskip;
  pt.t = w.t;
  FactorBatch fbt = factor_batch(w);
  fbt.count = slots;
  fbt.sDinv = 0;

  // The four launch sequences of an iteration.  Each reads its host inputs from
  // the pinned mirrors when it runs and ends without waiting; `timed` adds the
  // phase events (eager runs only).
  // W precision ladder (mixed forms): W with FP32 accuracy (BF16x6) while a problem
  // iterates; once its KKT measure (or the iteration cap) says stop, W and the
  // measures are recomputed in FP64 from the same factor and only the FP64 values
  // decide; from then on that problem keeps FP64 W.  Every returned W and reported
  // measure is FP64.
  const bool w_mixed = (o.w_mixed < 0) ? (o.precision != GLASSO_FP64) : (o.w_mixed != 0);
  std::vector<int> wexact(count, w_mixed ? 0 : 1), wlast(count, 1);
  PassBatch pr = pb;  // FP64 re-check of the problems in skip64 == 0
  pr.skip = w.skip64;
  const FactorBatch fbw = factor_batch(w);
  // BF16x3 form: the gradient pass writes Z only as the split the product reads
  // (into the second half of each problem's X region, free once W is formed)
  double* const z_f64 = (o.precision == GLASSO_MIXED_BF16X3) ? nullptr : w.Z;
  void* const z_split = (o.precision == GLASSO_MIXED_BF16X3) ? (void*)(reinterpret_cast<uint8_t*>(w.X) + 4 * nn)
                                                             : nullptr;
  // the replaced iterate of the last accepted step (G-ISTA): the trial buffer that
  // held the old iterate after an exchange, else P, where the accept step saves it
  const bool swap_accept = !o.graphs && count == 1 && K == 1;
  auto a_prev = [&]() -> const double* { return gista ? (swap_accept ? w.At : w.P) : nullptr; };
  auto head = [&](hipStream_t s, bool timed) -> glasso_err {  // a1, a2
    glasso_err e2 = push_ints(s, w.skip, hm.skip, count);
    if (e2) return e2;
    e2 = push_ints(s, w.skip32, hm.skip32, count);
    if (e2) return e2;
    e2 = push_ints(s, w.skip64, hm.skip64, count);
    if (e2) return e2;
    if (timed) HIP_TRY(hipEventRecord(h->ev[0], s));
    // the accepted trial's factor: place and invert its diagonal blocks
    K_TRY(finish_factor(s, w.L, np, (int)np, w.dL, w.Dinv, w.skip, fbw));
    // FP64-W problems: V = inv(L) in place, W = V^T V; the others keep L intact
    // (their FP64 re-check starts from it).  Eager launches leave out the kernels
    // every problem would skip (a captured graph holds them all).
    bool any64 = o.graphs != 0, any32 = o.graphs != 0;
    for (int b = 0; b < count; ++b) {
      any64 = any64 || !hm.skip64[b];
      any32 = any32 || !hm.skip32[b];
    }
    if (any64) {
      K_TRY(trtri_lower(s, w.L, np, (int)np, w.Dinv, w.X, w.skip64, fbw, nn));
      K_TRY(lauum_lower(s, w.L, np, w.W, np, (int)np, w.skip64, fbw, nn));
    }
    if (w_mixed && any32) {
      e2 = inverse_f32(w, s, w.skip32, timed ? h->ev + 10 : nullptr);
      if (e2) return e2;
    } else if (w_mixed && timed) {
      HIP_TRY(hipEventRecord(h->ev[10], s));
      HIP_TRY(hipEventRecord(h->ev[11], s));
    }
    if (timed) HIP_TRY(hipEventRecord(h->ev[1], s));
    K_TRY(pass_grad(s, w.S, w.W, w.A, w.dL, n, n, np, 0.0, z_f64, w.GM, w.part, w.scal, pb, z_split, 8 * nn,
                    a_prev()));
    if (timed) HIP_TRY(hipEventRecord(h->ev[2], s));
    return fetch_async(h, s);
  };
  auto head_given_w = [&](hipStream_t s, bool timed) -> glasso_err {  // a2 with W already formed
    glasso_err e2 = push_ints(s, w.skip, hm.skip, count);
    if (e2) return e2;
    if (timed) {
      HIP_TRY(hipEventRecord(h->ev[0], s));
      HIP_TRY(hipEventRecord(h->ev[1], s));
    }
    K_TRY(pass_grad(s, w.S, w.W, w.A, w.dL, n, n, np, 0.0, w.Z, w.GM, w.part, w.scal, pb));
    if (timed) HIP_TRY(hipEventRecord(h->ev[2], s));
    return fetch_async(h, s);
  };
  auto recheck = [&](hipStream_t s, bool) -> glasso_err {  // a1, a2 in FP64 for skip64 == 0
    glasso_err e2 = push_ints(s, w.skip64, hm.skip64, count);
    if (e2) return e2;
    K_TRY(trtri_lower(s, w.L, np, (int)np, w.Dinv, w.X, w.skip64, fbw, nn));
    K_TRY(lauum_lower(s, w.L, np, w.W, np, (int)np, w.skip64, fbw, nn));
    K_TRY(pass_grad(s, w.S, w.W, w.A, w.dL, n, n, np, 0.0, z_f64, w.GM, w.part, w.scal, pr, z_split, 8 * nn,
                    a_prev()));
    return fetch_async(h, s);
  };
  auto prod = [&](hipStream_t s, bool timed) -> glasso_err {  // a3
    glasso_err e2 = push_ints(s, w.skip, hm.skip, count);
    if (e2) return e2;
    return precond_product(w, s, o.precision, w.skip, n, sparse_now, timed ? h->ev + 5 : nullptr, z_split != nullptr);
  };
  // the leaf launches of the first eagerly launched trial factorisation of the call
  // in which every trial point was positive definite (so that no launch returned
  // early after a failed pivot) are timed one by one, with events around each launch
  LeafTimer leaf;
  bool leaf_done = false;
  double leaf_ms = 0.0;
  {
    const int want = 2 * (int)std::min<int64_t>(np / TILE, 256);
    while ((int)h->leaf_ev.size() < want) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) break;
      h->leaf_ev.push_back(e);
    }
  }
  auto trial = [&](hipStream_t s, bool timed) -> glasso_err {  // a4, a5
    glasso_err e2 = push_ints(s, w.lsskip, hm.lsskip, slots);
    if (e2) return e2;
    e2 = push_doubles(s, w.t, hm.t, slots);
    if (e2) return e2;
    K_TRY(pass_trial(s, w.A, w.P, w.S, w.GM, n, np, 0.0, 0.0, w.At, w.Lt, w.part, w.info, pt,
                     (o.sigma > 0.0 || gista) ? w.W : nullptr, gista ? 1 : 0));
    // the trial's factor is finished (diagonal blocks placed and inverted) only if
    // it is accepted, at the next head
    if (timed) HIP_TRY(hipEventRecord(h->ev[8], s));
    LeafTimer* lt = nullptr;
    if (timed && !leaf_done && (int)h->leaf_ev.size() >= 2) {
      leaf.used = 0;
      leaf.flops = 0.0;
      leaf.ev = h->leaf_ev.data();
      leaf.cap = (int)h->leaf_ev.size();
      leaf.n = n;
      leaf.active = 0;
      for (int j = 0; j < slots; ++j) leaf.active += hm.lsskip[j] == 0;
      lt = &leaf;
    }
    K_TRY(potrf_lower(s, w.Lt, np, (int)np, w.dLt, nullptr, w.info, fbt, 0, lt));
    if (timed) HIP_TRY(hipEventRecord(h->ev[9], s));
    K_TRY(finish_trial(s, w.part, tiles, w.dL, w.dLt, w.info, n, 0.0, w.scal_t, pt));
    return fetch_async(h, s);
  };
  auto accept = [&](hipStream_t s, bool) -> glasso_err {  // a7
    glasso_err e2 = push_ints(s, w.accept, hm.accept, count);
    if (e2) return e2;
    K_TRY(accept_trials(s, w.accept, count, w.A, w.At, w.L, w.Lt, w.dL, w.dLt, np, gista ? w.P : nullptr));
    return GLASSO_OK;
  };
  const bool graphs = o.graphs != 0;
  // A single problem run with eager launches takes an accepted trial point by
  // exchanging the current and trial buffers (A, L, diag(L), the diagonal-block
  // inverses) instead of copying them.  The exchange is undone when the call
  // returns, so later calls (and graphs captured by them) see the usual layout.
  struct BufferSwap {
    Workspace& w;
    int parity;
    void flip() {
      std::swap(w.A, w.At);
      std::swap(w.L, w.Lt);
      std::swap(w.dL, w.dLt);
      std::swap(w.Dinv, w.Dinvt);
      parity ^= 1;
    }
    ~BufferSwap() {
      if (parity) flip();
    }
  } swapped{w, 0};
  if (graphs) {
    GraphKey key;
    key.base = w.base;
    key.host = hm.scal;
    key.np = np;
    key.n = n;
    key.sS = sS;
    key.count = count;
    key.slots = slots;
    key.precision = o.precision;
    key.tiles = get_gemm_f64_small_tile_below();
    if (!(h->graphs.key == key)) {
      drop_graphs(h->graphs);
      h->graphs.key = key;
    }
  }
  // eager: run the sequence on st; graphs: capture it once, then replay it on st
  auto run = [&](hipGraphExec_t* slot, auto& body) -> glasso_err {
    if (!graphs) return body(st, true);
    if (!*slot) {
      glasso_err e2 = capture_graph(h, slot, [&](hipStream_t cs) { return body(cs, false); });
      if (e2) return e2;
    }
    HIP_TRY(hipGraphLaunch(*slot, st));
    return GLASSO_OK;
  };

  double phase[8] = {0};
  // FP64 W and measures for the problems with mark[b] != 0 (skip64 = !mark)
  auto run_recheck = [&](const std::vector<int>& mark) -> glasso_err {
    for (int b = 0; b < count; ++b) hm.skip64[b] = !mark[b];
    glasso_err e2 = run(&h->graphs.rechk, recheck);
    if (e2) return e2;
    HIP_TRY(hipStreamSynchronize(st));
    for (int b = 0; b < count; ++b)
      if (mark[b]) wlast[b] = 1;
    return GLASSO_OK;
  };

  // the first W of a diagonal start is exact (formed with A^(0))
  bool w_given = diag_start;
  for (;;) {
    for (int b = 0; b < count; ++b) {
      hm.skip[b] = !active[b];
      hm.skip32[b] = !(active[b] && !wexact[b]);
      hm.skip64[b] = !(active[b] && wexact[b]);
      if (active[b]) wlast[b] = w_given ? 1 : wexact[b];
    }
    const bool exact_w = w_given;
    if (w_given) {
      e = head_given_w(st, true);
      w_given = false;
    } else {
      if (graphs) HIP_TRY(hipEventRecord(h->ev[0], st));
      e = run(&h->graphs.head, head);
      if (e) return e;
      if (graphs) {
        HIP_TRY(hipEventRecord(h->ev[1], st));
        HIP_TRY(hipEventRecord(h->ev[2], st));
      }
    }
    if (e) return e;
    HIP_TRY(hipStreamSynchronize(st));
    phase[1] += elapsed(h->ev[0], h->ev[1]);
    phase[2] += elapsed(h->ev[1], h->ev[2]);
    if (w_mixed && !exact_w && !graphs) phase[7] += elapsed(h->ev[10], h->ev[11]);
    // a problem that would stop on an FP32-accurate W is re-checked with FP64 W first
    std::vector<int> mark(count, 0);
    int nmark = 0;
    for (int b = 0; b < count; ++b)
      if (active[b] && !wexact[b] && !exact_w && (hscal(h, b, SC_KKT_REL1) <= tol || it[b] >= o.max_iter)) {
        mark[b] = 1;
        wexact[b] = 1;
        ++nmark;
      }
    if (nmark) {
      e = run_recheck(mark);
      if (e) return e;
    }
    if (gista)
      for (int b = 0; b < count; ++b) {
        if (!active[b] || !bb_have[b]) continue;
        const double den = bb_dw[b] - hscal(h, b, SC_DW_NEW);
        const double bb = bb_num[b] / den;
        if (den > 0.0 && bb_num[b] > 0.0 && std::isfinite(bb)) t_next[b] = bb;
        bb_have[b] = 0;
      }
    int nact = 0;
    for (int b = 0; b < count; ++b) {
      if (!active[b]) continue;
      if (hscal(h, b, SC_KKT_REL1) <= tol) {
        status[b] = GLASSO_CONVERGED;
        active[b] = 0;
      } else if (it[b] >= o.max_iter) {
        status[b] = GLASSO_MAX_ITER;
        active[b] = 0;
      } else {
        ++nact;
      }
    }
    if (!nact) break;
    for (int b = 0; b < count; ++b) hm.skip[b] = !active[b];
    // a3: P = A Z A; with A still the diagonal A^(0) it is D Z D, formed elementwise
    HIP_TRY(hipEventRecord(h->ev[2], st));
    if (gista) {
      // no preconditioned product
    } else if (exact_w) {
      HIP_TRY(hipEventRecord(h->ev[5], st));
      e = push_ints(st, w.skip, hm.skip, count);
      if (e) return e;
      K_TRY(diag_product(st, w.A, w.Z, w.P, np, count, w.skip));
      HIP_TRY(hipEventRecord(h->ev[6], st));
    } else {
      sparse_now = sparse_on;
      if (sparse_on && !graphs) {
        sparse_now = false;
        for (int b = 0; b < count && !sparse_now; ++b)
          sparse_now = active[b] && hscal(h, b, SC_NNZ_A) <= (double)SPARSE_KA * (double)n;
      }
      if (graphs) HIP_TRY(hipEventRecord(h->ev[5], st));
      e = run(&h->graphs.prod, prod);
      if (e) return e;
      if (graphs) HIP_TRY(hipEventRecord(h->ev[6], st));
      for (int b = 0; b < count; ++b) prod_b[b] = active[b];
    }
    HIP_TRY(hipEventRecord(h->ev[3], st));
    // a4-a6: trial points t = t0, t0*shrink, ... until PD with a strict decrease.
    // A round evaluates the next ncand[b] <= K step sizes of that sequence for each
    // searching problem (never past the point where the sequential search would
    // take the fallback step or give up) and takes the first that succeeds, so the
    // accepted step is the one the one-at-a-time search takes.  The first round of
    // an iteration evaluates as many as the last accepted step needed.
    for (int b = 0; b < count; ++b) {
      ls[b] = active[b];
      fb_used[b] = 0;
      tb[b] = gista ? t_next[b] : o.t0;
    }
    // acceptance: a strict decrease (sigma = 0, condition t_cond_min) or sigma times
    // the decrease the linear model predicts (the trial pass read W for it)
    auto decrease_target = [&](int j) { return o.sigma > 0.0 ? o.sigma * hscal_t(h, j, SC_PRED) : 0.0; };
    bool first_round = true;
    for (;;) {
      int nls = 0;
      for (int b = 0; b < count; ++b) {
        if (!ls[b]) continue;
        if (!gista && tb[b] < o.t_floor && !fb_used[b]) {
          double tf = 0.0;
          e = cond_fallback_step(h, st, b, n, &tf);
          if (e) return e;
          tb[b] = std::min(tb[b], tf);
          fb_used[b] = 1;
          ++fallbacks[b];
        }
        if (tb[b] < o.t_min) {
          ls[b] = 0;
          active[b] = 0;
          status[b] = GLASSO_LS_FAILED;
          continue;
        }
        ++nls;
      }
      if (!nls) break;
      for (int b = 0; b < count; ++b) {
        for (int i = 0; i < K; ++i) hm.lsskip[b * K + i] = 1;
        ncand[b] = 0;
        if (!ls[b]) continue;
        const int want = first_round ? std::min(K, std::max(1, last_trials[b])) : K;
        double c = tb[b];
        for (;;) {
          hm.t[b * K + ncand[b]] = c;
          hm.lsskip[b * K + ncand[b]] = 0;
          if (++ncand[b] == want) break;
          c *= o.shrink;
          if (c < o.t_min || (!gista && c < o.t_floor && !fb_used[b])) break;
        }
      }
      first_round = false;
      e = run(&h->graphs.trial, trial);
      if (e) return e;
      HIP_TRY(hipStreamSynchronize(st));
      if (!graphs) phase[6] += elapsed(h->ev[8], h->ev[9]);
      if (!leaf_done && leaf.used) {
        bool all_pd = true;
        for (int j = 0; j < slots; ++j) all_pd = all_pd && (hm.lsskip[j] || hm.info[j] == 0);
        if (all_pd) {
          for (int i = 0; i + 1 < leaf.used; i += 2) leaf_ms += elapsed(leaf.ev[i], leaf.ev[i + 1]);
          leaf_done = true;
        } else {
          leaf.used = 0;
          leaf.flops = 0.0;
        }
      }
      int nacc = 0;
      for (int b = 0; b < count; ++b) {
        hm.accept[b] = 0;
        if (!ls[b]) continue;
        int got = -1, stalled = -1;
        for (int i = 0; i < ncand[b] && got < 0 && stalled < 0; ++i) {
          const int j = b * K + i;
          if (gista) {
            // a trial point equal to A: the step is below the resolution of A
            if (hscal_t(h, j, SC_D2) == 0.0)
              stalled = i;
            else if (hm.info[j] == 0 && hscal_t(h, j, SC_QB) <= 0.0)
              got = i;
          } else if (hm.info[j] == 0 && hscal_t(h, j, SC_DF) < decrease_target(j)) {
            got = i;
          }
        }
        if (stalled >= 0) {
          trials[b] += stalled;
          ls[b] = 0;
          active[b] = 0;
          status[b] = GLASSO_LS_FAILED;
          continue;
        }
        if (got >= 0) {
          if (gista) {
            const int j = b * K + got;
            t_next[b] = hm.t[j];
            bb_num[b] = hscal_t(h, j, SC_D2);
            bb_dw[b] = hscal_t(h, j, SC_DW);
            bb_have[b] = 1;
          }
          trials[b] += got + 1;
          since[b] += got + 1;
          last_trials[b] = since[b];
          since[b] = 0;
          hm.accept[b] = b * K + got + 1;
          ls[b] = 0;
          ++it[b];
          ++nacc;
        } else {
          trials[b] += ncand[b];
          since[b] += ncand[b];
          tb[b] = hm.t[b * K + ncand[b] - 1] * o.shrink;
        }
      }
      if (nacc) {
        // a7: accept
        if (swap_accept) {
          swapped.flip();
        } else {
          e = run(&h->graphs.acc, accept);
          if (e) return e;
        }
      }
    }
    HIP_TRY(hipEventRecord(h->ev[4], st));
    HIP_TRY(hipEventSynchronize(h->ev[4]));
    phase[3] += elapsed(h->ev[2], h->ev[3]);
    phase[4] += elapsed(h->ev[3], h->ev[4]);
    // which form served each problem's product (the scalars were fetched with the
    // line search's last round); the GEMM time counts only when the pair ran
    bool pair_ran = false;
    for (int b = 0; b < count; ++b) {
      if (!prod_b[b]) continue;
      prod_b[b] = 0;
      const bool dense = !sparse_now || hscal(h, b, SC_DENSE_PRODUCT) != 0.0;
      (dense ? gemm_products[b] : sparse_products[b]) += 1;
      pair_ran = pair_ran || dense;
    }
    if (pair_ran) phase[5] += elapsed(h->ev[5], h->ev[6]);
  }

  {
    std::vector<int> mark(count, 0);
    int nmark = 0;
    for (int b = 0; b < count; ++b)
      if (!wlast[b]) {
        mark[b] = 1;
        ++nmark;
      }
    if (nmark) {
      e = run_recheck(mark);
      if (e) return e;
    }
  }
  for (int b = 0; b < count; ++b) {
    K_TRY(sym_copy_out(st, w.A + b * nn, np, Aout[b], n, 0));
    if (Wout && Wout[b]) K_TRY(sym_copy_out(st, w.W + b * nn, np, Wout[b], n, 1));
  }
  HIP_TRY(hipStreamSynchronize(st));
  if (!leaf_done) {
    leaf.used = 0;
    leaf.flops = 0.0;
  }
  if (info) {
    const double total =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    for (int b = 0; b < count; ++b) {
      glasso_info& in = info[b];
      memset(&in, 0, sizeof(in));
      in.objective = hscal(h, b, SC_OBJECTIVE);
      in.kkt_rel1 = hscal(h, b, SC_KKT_REL1);
      in.kkt_fro = hscal(h, b, SC_KKT_FRO);
      in.kkt_max = hscal(h, b, SC_MAX_ABS_Z);
      in.nnz = (int64_t)llround(hscal(h, b, SC_NNZ_A));
      in.iterations = it[b];
      in.ls_trials = trials[b];
      in.status = status[b];
      in.fallback_steps = fallbacks[b];
      in.aza_gemm_products = gemm_products[b];
      in.aza_sparse_products = sparse_products[b];
      in.components = 1;
      in.largest_component = (int)n;
      for (int i = 1; i < 8; ++i) in.time_ms[i] = phase[i];
      in.time_ms[0] = total;
      in.leaf_launches = leaf_done ? leaf.used / 2 : 0;
      in.leaf_ms = leaf_ms;
      in.leaf_flops = leaf.flops;
    }
  }
  return GLASSO_OK;
}

}  // namespace

extern "C" {

glasso_err glasso_default_options(glasso_options* opt) {
  if (!opt) return GLASSO_ERR_INVALID_ARG;
  memset(opt, 0, sizeof(*opt));
  opt->precision = GLASSO_FP64;
  opt->tile_policy = GLASSO_TILES_AUTO;
  opt->graphs = 0;
  opt->w_mixed = -1;
  opt->max_iter = 500;
  opt->t0 = 1.0;
  opt->shrink = 0.5;
  opt->t_floor = 1e-4;
  opt->t_min = 1e-12;
  opt->warm_start = 0;
  opt->method = GLASSO_PISTA;
  return GLASSO_OK;
}

glasso_err glasso_create(glasso_handle* h, const glasso_options* opt) {
  if (!h) return GLASSO_ERR_INVALID_ARG;
  *h = nullptr;
  glasso_options o;
  if (opt)
    o = *opt;
  else
    glasso_default_options(&o);
  if (check_options(&o)) return GLASSO_ERR_INVALID_ARG;
  glasso_handle_s* hh = new (std::nothrow) glasso_handle_s();
  if (!hh) return GLASSO_ERR_OOM;
  hh->opt = o;
  if (hipGetDevice(&hh->device) != hipSuccess) {
    delete hh;
    return GLASSO_ERR_HIP;
  }
  if (ensure_host(hh, 1, 1) != GLASSO_OK) {
    delete hh;
    return GLASSO_ERR_HIP;
  }
  for (auto& e : hh->ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      glasso_destroy(hh);
      return GLASSO_ERR_HIP;
    }
  }
  if (hipStreamCreateWithFlags(&hh->cap, hipStreamNonBlocking) != hipSuccess) {
    glasso_destroy(hh);
    return GLASSO_ERR_HIP;
  }
  *h = hh;
  return GLASSO_OK;
}

glasso_err glasso_destroy(glasso_handle h) {
  if (!h) return GLASSO_OK;
  drop_graphs(h->graphs);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  if (h->small_base) (void)hipFree(h->small_base);
  if (h->cov_base) (void)hipFree(h->cov_base);
  if (h->gen_base) (void)hipFree(h->gen_base);
  if (h->scr_base) (void)hipFree(h->scr_base);
  if (h->ws.base) (void)hipFree(h->ws.base);
  free_host(h->hm);
  for (auto& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : h->leaf_ev)
    if (e) (void)hipEventDestroy(e);
  delete h;
  return GLASSO_OK;
}

const char* glasso_error_string(glasso_err e) {
  switch (e) {
    case GLASSO_OK: return "success";
    case GLASSO_ERR_INVALID_ARG: return "invalid argument";
    case GLASSO_ERR_NOT_PD: return "matrix is not positive definite";
    case GLASSO_ERR_OOM: return "out of device memory";
    case GLASSO_ERR_HIP: return "HIP runtime error";
    case GLASSO_ERR_INTERNAL: return "internal error";
  }
  return "unknown error";
}

glasso_err glasso_workspace_size(int64_t n, int precision, size_t* bytes) {
  if (n < 1 || !bytes || !valid_precision(precision)) return GLASSO_ERR_INVALID_ARG;
  Workspace probe;
  const int64_t np = pad_to_tile(n);
  *bytes = layout(probe, 1, ls_width(np), np, nullptr);
  return GLASSO_OK;
}

namespace {

glasso_err small_with_handle(glasso_handle h, int count, const double* const* S, const int64_t* n,
                             const double* lambda, double tol, double* const* A, double* const* W, glasso_info* info,
                             hipStream_t st);

// Problems of equal padded size run together; groups run one after another.
glasso_err solve_batched_plain(glasso_handle h, hipStream_t st, int count, const double* const* S, const int64_t* n,
                               const double* lambda, double tol, double* const* A, double* const* W,
                               glasso_info* info) {
  std::vector<int> done(count, 0);
  for (int i = 0; i < count; ++i) {
    if (done[i]) continue;
    const int64_t np = pad_to_tile(n[i]);
    std::vector<int> idx;
    for (int j = i; j < count; ++j)
      if (!done[j] && pad_to_tile(n[j]) == np && n[j] == n[i]) idx.push_back(j);
    std::vector<const double*> Sg;
    std::vector<double> lg;
    std::vector<double*> Ag, Wg;
    std::vector<glasso_info> ig(idx.size());
    for (int j : idx) {
      Sg.push_back(S[j]);
      lg.push_back(lambda[j]);
      Ag.push_back(A[j]);
      Wg.push_back(W ? W[j] : nullptr);
      done[j] = 1;
    }
    glasso_err e = run_engine(h, st, (int)idx.size(), n[i], Sg.data(), lg.data(), tol, Ag.data(), Wg.data(),
                              ig.data());
    if (e) return e;
    if (info)
      for (size_t k = 0; k < idx.size(); ++k) info[idx[k]] = ig[k];
  }
  return GLASSO_OK;
}

glasso_err grow_scr(glasso_handle h, size_t bytes) {
  if (bytes <= h->scr_bytes) return GLASSO_OK;
  if (h->scr_base) (void)hipFree(h->scr_base);
  h->scr_base = nullptr;
  h->scr_bytes = 0;
  if (hipMalloc(&h->scr_base, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return GLASSO_ERR_OOM;
  }
  h->scr_bytes = bytes;
  return GLASSO_OK;
}

// Block-diagonal screening (screen.hip): every problem is split into the connected
// components of {|S_ij| > lambda}; a problem that stays in one piece is solved in
// place, the blocks of the others are gathered, solved (n <= GLASSO_SMALL_MAX_N in
// one persistent launch, the rest batched) and scattered back between zeros.
glasso_err run_screened(glasso_handle h, hipStream_t st, int count, const double* const* S, const int64_t* n,
                        const double* lambda, double tol, double* const* A, double* const* W, glasso_info* info) {
  const auto t_start = std::chrono::steady_clock::now();
  std::vector<int64_t> loff(count + 1, 0);
  for (int p = 0; p < count; ++p) loff[p + 1] = loff[p] + n[p];
  const size_t lab_bytes = align_up((size_t)(loff[count] + 64) * sizeof(int));
  glasso_err e = grow_scr(h, lab_bytes);
  if (e) return e;
  int* lab = static_cast<int*>(h->scr_base);
  int* err = lab + loff[count];
  HIP_TRY(hipMemsetAsync(err, 0, sizeof(int), st));
  for (int p = 0; p < count; ++p) K_TRY(screen_components(st, S[p], n[p], n[p], lambda[p], lab + loff[p], err));
  std::vector<int> hlab(loff[count] + 1);
  HIP_TRY(hipMemcpyAsync(hlab.data(), lab, (size_t)(loff[count] + 1) * sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (hlab[loff[count]]) return GLASSO_ERR_INTERNAL;

  // the blocks of every problem, variables ascending (a block is labelled by its
  // smallest variable)
  struct Blk {
    int p;
    std::vector<int> idx;
  };
  std::vector<Blk> blocks;
  std::vector<int> direct, ncomp(count, 0), largest(count, 0);
  for (int p = 0; p < count; ++p) {
    const int* lp = hlab.data() + loff[p];
    std::vector<int> id_of(n[p], -1);
    const size_t first = blocks.size();
    for (int64_t i = 0; i < n[p]; ++i) {
      const int r = lp[i];
      if (id_of[r] < 0) {
        id_of[r] = (int)blocks.size();
        blocks.push_back(Blk{p, {}});
      }
      blocks[id_of[r]].idx.push_back((int)i);
    }
    ncomp[p] = (int)(blocks.size() - first);
    for (size_t b = first; b < blocks.size(); ++b) largest[p] = std::max(largest[p], (int)blocks[b].idx.size());
    if (ncomp[p] == 1) {  // one piece: solved in place
      blocks.resize(first);
      direct.push_back(p);
    }
  }

  // packing of the gathered blocks: S_k, A_k, W_k (k^2 each), the variables, the table
  const int nb = (int)blocks.size();
  std::vector<ScreenBlock> tab(nb);
  int64_t total = 0, nidx = 0;
  for (int b = 0; b < nb; ++b) {
    tab[b].k = (int)blocks[b].idx.size();
    tab[b].off = total;
    total += (int64_t)tab[b].k * tab[b].k;
    nidx += tab[b].k;
  }
  const bool want_w = W != nullptr;
  if (nb) {
    const size_t pack = align_up((size_t)total * sizeof(double));
    const size_t bytes = lab_bytes + 3 * pack + align_up((size_t)nidx * sizeof(int)) +
                         align_up((size_t)nb * sizeof(ScreenBlock)) + align_up((size_t)nb * sizeof(double));
    e = grow_scr(h, bytes);
    if (e) return e;
    char* base = static_cast<char*>(h->scr_base) + lab_bytes;
    double* Sk = reinterpret_cast<double*>(base);
    double* Ak = reinterpret_cast<double*>(base + pack);
    double* Wk = reinterpret_cast<double*>(base + 2 * pack);
    int* didx = reinterpret_cast<int*>(base + 3 * pack);
    ScreenBlock* dtab = reinterpret_cast<ScreenBlock*>(base + 3 * pack + align_up((size_t)nidx * sizeof(int)));
    double* dsum = reinterpret_cast<double*>(reinterpret_cast<char*>(dtab) + align_up((size_t)nb * sizeof(ScreenBlock)));
    std::vector<int> hidx(nidx);
    int64_t io = 0;
    for (int b = 0; b < nb; ++b) {
      const int p = blocks[b].p;
      ScreenBlock& t = tab[b];
      t.S = S[p];
      t.A = A[p];
      t.W = want_w ? W[p] : nullptr;
      t.ld = n[p];
      t.idx = didx + io;
      t.Sk = Sk + t.off;
      t.Ak = Ak + t.off;
      t.Wk = Wk + t.off;
      std::copy(blocks[b].idx.begin(), blocks[b].idx.end(), hidx.begin() + io);
      io += t.k;
    }
    HIP_TRY(hipMemcpyAsync(didx, hidx.data(), (size_t)nidx * sizeof(int), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(dtab, tab.data(), (size_t)nb * sizeof(ScreenBlock), hipMemcpyHostToDevice, st));
    K_TRY(gather_blocks(st, dtab, nb, total, 0));
    if (h->opt.warm_start) K_TRY(gather_blocks(st, dtab, nb, total, 1));
    HIP_TRY(hipStreamSynchronize(st));  // the host staging arrays are released below

    // small blocks in one persistent launch, the others batched
    std::vector<const double*> sS, bS;
    std::vector<int64_t> sn, bn;
    std::vector<double> sl, bl;
    std::vector<double*> sA, sW, bA, bW;
    std::vector<int> sid, bid;
    for (int b = 0; b < nb; ++b) {
      // the persistent small solver runs pISTA only
      const bool small = tab[b].k <= GLASSO_SMALL_MAX_N && h->opt.method == GLASSO_PISTA;
      (small ? sS : bS).push_back(tab[b].Sk);
      (small ? sn : bn).push_back(tab[b].k);
      (small ? sl : bl).push_back(lambda[blocks[b].p]);
      (small ? sA : bA).push_back(tab[b].Ak);
      (small ? sW : bW).push_back(want_w ? tab[b].Wk : nullptr);
      (small ? sid : bid).push_back(b);
    }
    std::vector<glasso_info> binfo(nb);
    if (!sS.empty()) {
      std::vector<glasso_info> si(sS.size());
      e = small_with_handle(h, (int)sS.size(), sS.data(), sn.data(), sl.data(), tol, sA.data(), want_w ? sW.data() : nullptr,
                            si.data(), st);
      if (e) return e;
      for (size_t q = 0; q < si.size(); ++q) binfo[sid[q]] = si[q];
    }
    if (!bS.empty()) {
      std::vector<glasso_info> bi(bS.size());
      e = solve_batched_plain(h, st, (int)bS.size(), bS.data(), bn.data(), bl.data(), tol, bA.data(),
                              want_w ? bW.data() : nullptr, bi.data());
      if (e) return e;
      for (size_t q = 0; q < bi.size(); ++q) binfo[bid[q]] = bi[q];
    }
    // assemble: zeros between the blocks
    for (int p = 0; p < count; ++p) {
      if (ncomp[p] == 1) continue;
      K_TRY(zero_fill(st, A[p], n[p] * n[p]));
      if (want_w && W[p]) K_TRY(zero_fill(st, W[p], n[p] * n[p]));
    }
    K_TRY(scatter_blocks(st, dtab, nb, total, want_w ? 1 : 0));
    K_TRY(block_abs_sums(st, dtab, nb, dsum));
    std::vector<double> hsum(nb);
    HIP_TRY(hipMemcpyAsync(hsum.data(), dsum, (size_t)nb * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (info) {
      std::vector<double> z1(count, 0.0), a1(count, 0.0), fro2(count, 0.0);
      for (int p = 0; p < count; ++p) {
        if (ncomp[p] == 1) continue;
        memset(&info[p], 0, sizeof(glasso_info));
        info[p].status = GLASSO_CONVERGED;
      }
      for (int b = 0; b < nb; ++b) {
        glasso_info& in = info[blocks[b].p];
        const glasso_info& bi = binfo[b];
        in.objective += bi.objective;
        z1[blocks[b].p] += bi.kkt_rel1 * hsum[b];
        a1[blocks[b].p] += hsum[b];
        fro2[blocks[b].p] += bi.kkt_fro * bi.kkt_fro;
        in.kkt_max = std::max(in.kkt_max, bi.kkt_max);
        in.nnz += bi.nnz;
        in.iterations = std::max(in.iterations, bi.iterations);
        in.ls_trials += bi.ls_trials;
        in.status = std::max(in.status, bi.status);
        in.fallback_steps += bi.fallback_steps;
        in.aza_gemm_products += bi.aza_gemm_products;
        in.aza_sparse_products += bi.aza_sparse_products;
        for (int i = 1; i < 8; ++i) in.time_ms[i] += bi.time_ms[i];
      }
      for (int p = 0; p < count; ++p) {
        if (ncomp[p] == 1) continue;
        info[p].kkt_rel1 = a1[p] > 0.0 ? z1[p] / a1[p] : 0.0;
        info[p].kkt_fro = sqrt(fro2[p]);
        // the stopping rule is the whole problem's: met when the assembled A meets it,
        // even if a block stalled (status LS_FAILED) below its own share
        if (info[p].kkt_rel1 <= tol) info[p].status = GLASSO_CONVERGED;
      }
    }
  }
  if (!direct.empty()) {
    std::vector<const double*> dS;
    std::vector<int64_t> dn;
    std::vector<double> dl;
    std::vector<double*> dA, dW;
    for (int p : direct) {
      dS.push_back(S[p]);
      dn.push_back(n[p]);
      dl.push_back(lambda[p]);
      dA.push_back(A[p]);
      dW.push_back(want_w ? W[p] : nullptr);
    }
    std::vector<glasso_info> di(direct.size());
    e = solve_batched_plain(h, st, (int)direct.size(), dS.data(), dn.data(), dl.data(), tol, dA.data(),
                            want_w ? dW.data() : nullptr, di.data());
    if (e) return e;
    if (info)
      for (size_t q = 0; q < direct.size(); ++q) info[direct[q]] = di[q];
  }
  if (info) {
    const double total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    for (int p = 0; p < count; ++p) {
      info[p].components = ncomp[p];
      info[p].largest_component = largest[p];
      info[p].time_ms[0] = total_ms;
    }
  }
  return GLASSO_OK;
}

}  // namespace

glasso_err glasso_solve(glasso_handle h, const double* S, int64_t n, double lambda, double tol, double* A,
                        double* W, glasso_info* info, void* stream) {
  if (!h || !S || !A || n < 1 || !(lambda > 0.0) || !(tol > 0.0) || !isfinite(lambda) || n > (1 << 20))
    return GLASSO_ERR_INVALID_ARG;
  const double* Sp[1] = {S};
  double* Ap[1] = {A};
  double* Wp[1] = {W};
  if (h->opt.screen) return run_screened(h, (hipStream_t)stream, 1, Sp, &n, &lambda, tol, Ap, Wp, info);
  return run_engine(h, (hipStream_t)stream, 1, n, Sp, &lambda, tol, Ap, Wp, info);
}

glasso_err glasso_solve_batched(glasso_handle h, int count, const double* const* S, const int64_t* n,
                                const double* lambda, double tol, double* const* A, double* const* W,
                                glasso_info* info, void* stream) {
  if (!h || count < 1 || !S || !n || !lambda || !A || !(tol > 0.0)) return GLASSO_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i)
    if (!S[i] || !A[i] || n[i] < 1 || n[i] > (1 << 20) || !(lambda[i] > 0.0) || !isfinite(lambda[i]))
      return GLASSO_ERR_INVALID_ARG;
  if (h->opt.screen) return run_screened(h, (hipStream_t)stream, count, S, n, lambda, tol, A, W, info);
  return solve_batched_plain(h, (hipStream_t)stream, count, S, n, lambda, tol, A, W, info);
}

glasso_err glasso_autotune(glasso_handle h, int64_t n, int count, int* policy, void* stream) {
  if (!h || n < 1 || n > (1 << 20) || count < 1) return GLASSO_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  glasso_err e = ensure_workspace(h, count, pad_to_tile(n), st);
  if (e) return e;
  int thr = 0;
  e = tune_tiles(h, st, h->opt.precision, &thr);
  if (e) return e;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[std::make_tuple(h->device, h->ws.np, h->ws.count)] = thr;
  }
  if (policy) *policy = thr;
  return GLASSO_OK;
}

namespace {

bool small_args_ok(int count, const double* const* S, const int64_t* n, const double* lambda, double tol,
                   double* const* A) {
  if (count < 1 || !S || !n || !lambda || !A || !(tol > 0.0)) return false;
  for (int i = 0; i < count; ++i)
    if (!S[i] || !A[i] || n[i] < 1 || n[i] > GLASSO_SMALL_MAX_N || !(lambda[i] > 0.0) || !isfinite(lambda[i]))
      return false;
  return true;
}

// Carving of the persistent solver's scratch for `grid` workgroups and `count`
// problems: per-workgroup matrix slots, free-set signs, problem descriptors,
// outputs and the work-queue counter.
struct SmallLayout {
  size_t ws, gm, pr, out, total;
  SmallLayout(int grid, int count) {
    ws = (size_t)grid * SMALL_WS_DOUBLES * sizeof(double);
    gm = (size_t)grid * SMALL_GM_BYTES;
    pr = ((size_t)count * sizeof(SmallProblem) + 255) / 256 * 256;
    out = ((size_t)count * sizeof(SmallOut) + 255) / 256 * 256;
    total = ws + gm + pr + out + 256;
  }
};

// One persistent launch over `count` problems with its scratch at `base` (device)
// and the host staging arrays pr, out (count entries each).
glasso_err run_small(const glasso_options& o, int count, const double* const* S, const int64_t* n,
                     const double* lambda, double tol, double* const* A, double* const* W, glasso_info* info,
                     hipStream_t st, char* base, int grid, SmallProblem* pr, SmallOut* out) {
  const auto t_start = std::chrono::steady_clock::now();
  const SmallLayout lay(grid, count);
  for (int i = 0; i < count; ++i) {
    pr[i].S = S[i];
    pr[i].A = A[i];
    pr[i].W = W ? W[i] : nullptr;
    pr[i].n = n[i];
    pr[i].lam = lambda[i];
  }
  SmallParams p;
  p.ws = reinterpret_cast<double*>(base);
  p.gm = reinterpret_cast<int8_t*>(base + lay.ws);
  SmallProblem* dpr = reinterpret_cast<SmallProblem*>(base + lay.ws + lay.gm);
  SmallOut* dout = reinterpret_cast<SmallOut*>(base + lay.ws + lay.gm + lay.pr);
  p.prob = dpr;
  p.out = dout;
  p.next = reinterpret_cast<int*>(base + lay.ws + lay.gm + lay.pr + lay.out);
  p.count = count;
  p.tol = tol;
  p.t0 = o.t0;
  p.shrink = o.shrink;
  p.t_floor = o.t_floor;
  p.t_min = o.t_min;
  p.sigma = o.sigma;
  p.max_iter = o.max_iter;
  p.warm_start = o.warm_start;
  HIP_TRY(hipMemcpyAsync(dpr, pr, (size_t)count * sizeof(SmallProblem), hipMemcpyHostToDevice, st));
  K_TRY(solve_small(st, p, grid));
  HIP_TRY(hipMemcpyAsync(out, dout, (size_t)count * sizeof(SmallOut), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const double total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  glasso_err err = GLASSO_OK;
  for (int i = 0; i < count; ++i) {
    if (out[i].error == 2 && !err) err = GLASSO_ERR_INVALID_ARG;
    if (out[i].error == 1 && !err) err = GLASSO_ERR_NOT_PD;
    if (out[i].error == 3 && !err) err = GLASSO_ERR_INTERNAL;
    if (info) {
      glasso_info& in = info[i];
      memset(&in, 0, sizeof(in));
      in.objective = out[i].objective;
      in.kkt_rel1 = out[i].kkt_rel1;
      in.kkt_fro = out[i].kkt_fro;
      in.kkt_max = out[i].kkt_max;
      in.nnz = (int64_t)llround(out[i].nnz);
      in.iterations = out[i].iterations;
      in.ls_trials = out[i].ls_trials;
      in.status = (glasso_status)out[i].status;
      in.fallback_steps = out[i].fallback_steps;
      in.time_ms[0] = total;
      in.components = 1;
      in.largest_component = (int)n[i];
    }
  }
  return err;
}

}  // namespace

namespace {

// The persistent small-problem launch on the handle's own workspace (grown as needed).
glasso_err small_with_handle(glasso_handle h, int count, const double* const* S, const int64_t* n,
                             const double* lambda, double tol, double* const* A, double* const* W, glasso_info* info,
                             hipStream_t st) {
  const int grid = std::min(count, 512);
  const SmallLayout lay(grid, count);
  if (lay.total > h->small_bytes) {
    if (h->small_base) (void)hipFree(h->small_base);
    h->small_base = nullptr;
    h->small_bytes = 0;
    if (hipMalloc(&h->small_base, lay.total) != hipSuccess) {
      (void)hipGetLastError();
      return GLASSO_ERR_OOM;
    }
    h->small_bytes = lay.total;
  }
  std::vector<SmallProblem> pr(count);
  std::vector<SmallOut> out(count);
  return run_small(h->opt, count, S, n, lambda, tol, A, W, info, st, static_cast<char*>(h->small_base), grid,
                   pr.data(), out.data());
}

}  // namespace

glasso_err glasso_solve_small(glasso_handle h, int count, const double* const* S, const int64_t* n,
                              const double* lambda, double tol, double* const* A, double* const* W,
                              glasso_info* info, void* stream) {
  if (!h || !small_args_ok(count, S, n, lambda, tol, A) || h->opt.method != GLASSO_PISTA) return GLASSO_ERR_INVALID_ARG;
  return small_with_handle(h, count, S, n, lambda, tol, A, W, info, (hipStream_t)stream);
}

// ------------------------------------------------------------------ allocation-free small solves
//
// glasso_solve_small_static keeps the persistent solver's scratch in `scratch`, an
// array of this library's device data sized for SMALL_STATIC_GRID workgroups and
// GLASSO_SMALL_STATIC_MAX_COUNT problems.  Each GPU holds its own copy at its own
// address; host code must use that address (from hipGetSymbolAddress, taken once
// per device with the device current), never the array's name.  The host staging
// arrays are static too, and one lock serialises the calls of a process, which all
// share the arrays.
namespace {

constexpr int SMALL_STATIC_GRID = 256;  // one workgroup per compute unit
constexpr int SMALL_STATIC_MAX_DEVICES = 64;
constexpr size_t SMALL_STATIC_BYTES =
    (size_t)SMALL_STATIC_GRID * SMALL_WS_DOUBLES * sizeof(double) + (size_t)SMALL_STATIC_GRID * SMALL_GM_BYTES +
    ((size_t)GLASSO_SMALL_STATIC_MAX_COUNT * sizeof(SmallProblem) + 255) / 256 * 256 +
    ((size_t)GLASSO_SMALL_STATIC_MAX_COUNT * sizeof(SmallOut) + 255) / 256 * 256 + 256;
static_assert(SMALL_STATIC_BYTES == GLASSO_SMALL_STATIC_BYTES, "GLASSO_SMALL_STATIC_BYTES in glasso.h");

static __device__ __align__(256) unsigned char scratch[SMALL_STATIC_BYTES];

std::mutex g_static_mu;
void* g_static_ptr[SMALL_STATIC_MAX_DEVICES] = {};
SmallProblem g_static_pr[GLASSO_SMALL_STATIC_MAX_COUNT];
SmallOut g_static_out[GLASSO_SMALL_STATIC_MAX_COUNT];

}  // namespace

glasso_err glasso_solve_small_static(const glasso_options* opt, int count, const double* const* S,
                                     const int64_t* n, const double* lambda, double tol, double* const* A,
                                     double* const* W, glasso_info* info, void* stream) {
  if (count > GLASSO_SMALL_STATIC_MAX_COUNT || !small_args_ok(count, S, n, lambda, tol, A))
    return GLASSO_ERR_INVALID_ARG;
  glasso_options o;
  glasso_default_options(&o);
  if (opt) {
    if (check_options(opt) || opt->method != GLASSO_PISTA) return GLASSO_ERR_INVALID_ARG;
    o = *opt;
  }
  std::lock_guard<std::mutex> lock(g_static_mu);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= SMALL_STATIC_MAX_DEVICES) return GLASSO_ERR_INVALID_ARG;
  if (!g_static_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return GLASSO_ERR_HIP;
    }
    g_static_ptr[dev] = ptr;
  }
  const int grid = std::min(count, SMALL_STATIC_GRID);
  return run_small(o, count, S, n, lambda, tol, A, W, info, (hipStream_t)stream,
                   static_cast<char*>(g_static_ptr[dev]), grid, g_static_pr, g_static_out);
}

// ------------------------------------------------------------------ step-level entry points
glasso_err glasso_covariance(glasso_handle h, const double* Y, int64_t m, int64_t n, int center, double* S,
                             void* stream) {
  if (!h || !Y || !S || m < 1 || n < 1 || n > (1 << 20) || m > ((int64_t)1 << 31) - 16) return GLASSO_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = pad_to_tile(n);
  const int64_t mp = (m + 15) / 16 * 16;  // K of the product, padded with zero samples
  const size_t bytes = ((size_t)mp * np + (size_t)np * np + (size_t)np) * sizeof(double);
  if (bytes > h->cov_bytes) {
    if (h->cov_base) (void)hipFree(h->cov_base);
    h->cov_base = nullptr;
    h->cov_bytes = 0;
    if (hipMalloc(&h->cov_base, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return GLASSO_ERR_OOM;
    }
    h->cov_bytes = bytes;
  }
  double* Yp = static_cast<double*>(h->cov_base);
  double* Sp = Yp + mp * np;
  double* mu = Sp + np * np;
  if (center) K_TRY(column_mean(st, Y, m, n, mu));
  K_TRY(center_pad(st, Y, m, n, center ? mu : nullptr, Yp, mp, np));
  // lower triangle of (1/m) Yp^T Yp on FP64 MFMA, then mirrored into the n x n output
  // (op(A) = op(B) = the columns of Yp: both operands read transposed)
  K_TRY(gemm_f64(st, 1, 1, (int)np, (int)np, (int)mp, 1.0 / (double)m, Yp, np, Yp, np, 0.0, Sp, np, 1, 0, 0, nullptr));
  K_TRY(sym_copy_out(st, Sp, np, S, n, 1));
  HIP_TRY(hipStreamSynchronize(st));
  return GLASSO_OK;
}

glasso_err glasso_generate(glasso_handle h, int kind, int64_t n, int64_t m, uint64_t seed, double* A_true, double* Y,
                           double* S, double* lambda_max, void* stream) {
  if (!h || n < 1 || n > (1 << 20) || (kind != GLASSO_GEN_RANDOM_SPARSE && kind != GLASSO_GEN_CHAIN))
    return GLASSO_ERR_INVALID_ARG;
  const bool samples = Y || S || lambda_max;
  if (!A_true && !samples) return GLASSO_ERR_INVALID_ARG;
  if (samples && (m < 1 || m > ((int64_t)1 << 31) - TILE)) return GLASSO_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = pad_to_tile(n);
  const int64_t mp = samples ? pad_to_tile(m) : 0;
  // L (np^2: the precision's lower triangle, then its factor, then V = inv(L)),
  // the diagonal-block inverses and diag(L), the inverse's scratch (np^2/4), Z and
  // the padded samples (mp x np each), the padded S (np^2), 256 partial maxima, the
  // maximum and the factor status
  const size_t dbl = (size_t)np * np + (size_t)np * TILE + (size_t)np + (size_t)np * np / 4 + 2 * (size_t)mp * np +
                     (samples ? (size_t)np * np : 0) + 256 + 8;
  const size_t bytes = dbl * sizeof(double) + 256;
  if (bytes > h->gen_bytes) {
    if (h->gen_base) (void)hipFree(h->gen_base);
    h->gen_base = nullptr;
    h->gen_bytes = 0;
    if (hipMalloc(&h->gen_base, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return GLASSO_ERR_OOM;
    }
    h->gen_bytes = bytes;
  }
  double* L = static_cast<double*>(h->gen_base);
  double* Dinv = L + np * np;
  double* dL = Dinv + np * TILE;
  double* tmp = dL + np;
  double* Z = tmp + np * np / 4;
  double* Yp = Z + mp * np;
  double* Sp = Yp + mp * np;
  double* part = Sp + (samples ? np * np : 0);
  double* lmax = part + 256;
  int* info = reinterpret_cast<int*>(lmax + 4);
  K_TRY(gen_precision_lower(st, L, n, np, kind == GLASSO_GEN_CHAIN ? GEN_CHAIN : GEN_RANDOM_SPARSE, seed));
  if (A_true) K_TRY(sym_copy_out(st, L, np, A_true, n, 1));
  if (samples) {
    // x_r = L^{-T} z_r: the rows of Y = Z V with V = inv(L) lower triangular
    HIP_TRY(hipMemsetAsync(info, 0, sizeof(int), st));
    K_TRY(potrf_lower(st, L, np, (int)np, dL, Dinv, info));
    int hinfo = 0;
    HIP_TRY(hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (hinfo) return GLASSO_ERR_NOT_PD;
    K_TRY(trtri_lower(st, L, np, (int)np, Dinv, tmp, nullptr));
    K_TRY(gen_normals(st, Z, m, n, mp, np, seed));
    // op(A) = Z (rows), op(B) = V read as [k][n] (tb = 1), lower triangular (b_tri = 1)
    K_TRY(gemm_f64(st, 0, 1, (int)mp, (int)np, (int)np, 1.0, Z, np, L, np, 0.0, Yp, np, 0, 0, 1, nullptr));
    if (Y) K_TRY(copy_rect(st, Yp, np, Y, m, n));
    if (S || lambda_max) {
      // S = (1/m) Y^T Y, lower triangle on FP64 MFMA (zero rows pad the samples)
      K_TRY(gemm_f64(st, 1, 1, (int)np, (int)np, (int)mp, 1.0 / (double)m, Yp, np, Yp, np, 0.0, Sp, np, 1, 0, 0,
                     nullptr));
      if (S) K_TRY(sym_copy_out(st, Sp, np, S, n, 1));
      if (lambda_max) {
        K_TRY(offdiag_absmax(st, Sp, n, np, part, lmax));
        HIP_TRY(hipMemcpyAsync(lambda_max, lmax, sizeof(double), hipMemcpyDeviceToHost, st));
      }
    }
  }
  HIP_TRY(hipStreamSynchronize(st));
  return GLASSO_OK;
}

glasso_err glasso_cholesky(glasso_handle h, const double* A, int64_t n, double* L, int64_t* info, double* logdet,
                           void* stream) {
  if (!h || !A || !L || n < 1) return GLASSO_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = pad_to_tile(n);
  glasso_err e = ensure_workspace(h, 1, np, st);
  if (e) return e;
  e = apply_tile_policy(h, st, h->opt.precision);
  if (e) return e;
  Workspace& w = h->ws;
  K_TRY(pad_copy_f64(st, A, n, np, w.L, nullptr, 1));
  e = factor_all(h, st);
  if (e) return e;
  const int finfo = h->hm.info[0];
  if (info) *info = finfo;
  K_TRY(sym_copy_out(st, w.L, np, L, n, 2));
  if (logdet) {
    K_TRY(sum_log(st, w.dL, n, w.scal + SC_LOGDET));
    e = fetch(h, st);
    if (e) return e;
    *logdet = finfo ? NAN : hscal(h, 0, SC_LOGDET);
  }
  HIP_TRY(hipStreamSynchronize(st));
  return GLASSO_OK;
}

glasso_err glasso_inverse(glasso_handle h, const double* A, int64_t n, double* W, void* stream) {
  if (!h || !A || !W || n < 1) return GLASSO_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = pad_to_tile(n);
  glasso_err e = ensure_workspace(h, 1, np, st);
  if (e) return e;
  e = apply_tile_policy(h, st, h->opt.precision);
  if (e) return e;
  Workspace& w = h->ws;
  K_TRY(pad_copy_f64(st, A, n, np, w.L, nullptr, 1));
  e = factor_all(h, st);
  if (e) return e;
  if (h->hm.info[0]) return GLASSO_ERR_NOT_PD;
  if (h->opt.w_mixed == 1) {
    e = inverse_f32(w, st, nullptr);  // the mixed-W inverse of the ladder
  } else {
    e = inverse_from_factor(w, st, nullptr);
  }
  if (e) return e;
  K_TRY(sym_copy_out(st, w.W, np, W, n, 1));
  HIP_TRY(hipStreamSynchronize(st));
  return GLASSO_OK;
}

glasso_err glasso_gradient_pass(glasso_handle h, const double* S, const double* W, const double* A, int64_t n,
                                double lambda, double* Z, int8_t* GM, double* kkt, void* stream) {
  if (!h || !S || !W || !A || !Z || !GM || n < 1 || !(lambda > 0.0)) return GLASSO_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = pad_to_tile(n);
  glasso_err e = ensure_workspace(h, 1, np, st);
  if (e) return e;
  e = apply_tile_policy(h, st, h->opt.precision);
  if (e) return e;
  Workspace& w = h->ws;
  K_TRY(pad_copy_f64(st, S, n, np, w.S, nullptr, 0));
  K_TRY(pad_copy_f64(st, W, n, np, w.W, nullptr, 1));
  K_TRY(pad_copy_f64(st, A, n, np, w.A, nullptr, 1));
  // no factor is at hand here: the log-det term is left out (nlog = 0)
  K_TRY(pass_grad(st, w.S, w.W, w.A, w.dL, n, 0, np, lambda, w.Z, w.GM, w.part, w.scal));
  K_TRY(sym_copy_out(st, w.Z, np, Z, n, 0));
  K_TRY(unpad_copy_i8(st, w.GM, np, GM, n));
  e = fetch(h, st);
  if (e) return e;
  if (kkt) {
    kkt[0] = hscal(h, 0, SC_SUM_ABS_Z);
    kkt[1] = hscal(h, 0, SC_SUM_ABS_A);
    kkt[2] = hscal(h, 0, SC_KKT_FRO);
    kkt[3] = hscal(h, 0, SC_MAX_ABS_Z);
  }
  return GLASSO_OK;
}

glasso_err glasso_precond_product(glasso_handle h, const double* A, const double* Z, int64_t n, int precision,
                                  double* P, void* stream) {
  if (!h || !A || !Z || !P || n < 1) return GLASSO_ERR_INVALID_ARG;
  if (!valid_precision(precision)) return GLASSO_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = pad_to_tile(n);
  glasso_err e = ensure_workspace(h, 1, np, st);
  if (e) return e;
  e = apply_tile_policy(h, st, h->opt.precision);
  if (e) return e;
  Workspace& w = h->ws;
  K_TRY(pad_copy_f64(st, A, n, np, w.A, nullptr, 1));
  K_TRY(pad_copy_f64(st, Z, n, np, w.Z, nullptr, 0));
  e = precond_product(w, st, precision, nullptr, n, false);
  if (e) return e;
  K_TRY(sym_copy_out(st, w.P, np, P, n, 1));
  HIP_TRY(hipStreamSynchronize(st));
  return GLASSO_OK;
}

glasso_err glasso_trial_point(glasso_handle h, const double* A, const double* P, const double* S, const int8_t* GM,
                              int64_t n, double lambda, double t, double* At, double* sums, void* stream) {
  if (!h || !A || !P || !S || !GM || !At || n < 1 || !(lambda > 0.0) || !(t > 0.0)) return GLASSO_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = pad_to_tile(n);
  glasso_err e = ensure_workspace(h, 1, np, st);
  if (e) return e;
  e = apply_tile_policy(h, st, h->opt.precision);
  if (e) return e;
  Workspace& w = h->ws;
  K_TRY(pad_copy_f64(st, A, n, np, w.A, nullptr, 1));
  K_TRY(pad_copy_f64(st, P, n, np, w.P, nullptr, 0));
  K_TRY(pad_copy_f64(st, S, n, np, w.S, nullptr, 0));
  K_TRY(pad_copy_i8(st, GM, n, np, w.GM));
  K_TRY(pass_trial(st, w.A, w.P, w.S, w.GM, n, np, lambda, t, w.At, w.Lt, w.part, w.info));
  // no factor: the log-ratio term reads the same diagonal twice and vanishes
  K_TRY(finish_trial(st, w.part, (int)pass_tiles(np), w.dL, w.dL, w.info, 0, lambda, w.scal));
  K_TRY(sym_copy_out(st, w.At, np, At, n, 0));
  e = fetch(h, st);
  if (e) return e;
  if (sums) {
    sums[0] = hscal(h, 0, SC_DTR);
    sums[1] = hscal(h, 0, SC_DL1);
  }
  return GLASSO_OK;
}

glasso_err glasso_gista_trial_point(glasso_handle h, const double* A, const double* S, const double* W,
                                    const int8_t* GM, int64_t n, double lambda, double t, double* At, double* sums,
                                    void* stream) {
  if (!h || !A || !S || !W || !GM || !At || n < 1 || !(lambda > 0.0) || !(t > 0.0)) return GLASSO_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = pad_to_tile(n);
  glasso_err e = ensure_workspace(h, 1, np, st);
  if (e) return e;
  Workspace& w = h->ws;
  K_TRY(pad_copy_f64(st, A, n, np, w.A, nullptr, 1));
  K_TRY(pad_copy_f64(st, S, n, np, w.S, nullptr, 0));
  K_TRY(pad_copy_f64(st, W, n, np, w.W, nullptr, 0));
  K_TRY(pad_copy_i8(st, GM, n, np, w.GM));
  K_TRY(pass_trial(st, w.A, w.P, w.S, w.GM, n, np, lambda, t, w.At, w.Lt, w.part, w.info, PassBatch(), w.W, 1));
  // no factor: the log-ratio term reads the same diagonal twice and vanishes
  K_TRY(finish_trial(st, w.part, (int)pass_tiles(np), w.dL, w.dL, w.info, 0, lambda, w.scal, PassBatch(), t));
  K_TRY(sym_copy_out(st, w.At, np, At, n, 0));
  e = fetch(h, st);
  if (e) return e;
  if (sums) {
    sums[0] = hscal(h, 0, SC_DTR);
    sums[1] = hscal(h, 0, SC_DL1);
    sums[2] = hscal(h, 0, SC_DW);
    sums[3] = hscal(h, 0, SC_D2);
  }
  return GLASSO_OK;
}

glasso_err glasso_sparse_product(glasso_handle h, const double* A, const double* Z, const int8_t* GM, int64_t n,
                                 double* P, int* used, void* stream) {
  if (!h || !A || !Z || !GM || !P || n < 1) return GLASSO_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t np = pad_to_tile(n);
  glasso_err e = ensure_workspace(h, 1, np, st);
  if (e) return e;
  e = apply_tile_policy(h, st, h->opt.precision);
  if (e) return e;
  Workspace& w = h->ws;
  K_TRY(pad_copy_f64(st, A, n, np, w.A, nullptr, 1));
  K_TRY(pad_copy_f64(st, Z, n, np, w.Z, nullptr, 0));
  K_TRY(pad_copy_i8(st, GM, n, np, w.GM));
  e = precond_product(w, st, GLASSO_FP64, nullptr, n, true);
  if (e) return e;
  // off the free set: zero (the dense pair, when it ran, filled the whole triangle)
  K_TRY(mask_free_set(st, w.P, w.GM, w.nn()));
  K_TRY(sym_copy_out(st, w.P, np, P, n, 1));
  e = fetch(h, st);
  if (e) return e;
  if (used) *used = hscal(h, 0, SC_DENSE_PRODUCT) == 0.0 ? 1 : 0;
  return GLASSO_OK;
}

}  // extern "C"
