// Block-diagonal screening of the graphical lasso: when |S_ij| <= lambda for every
// pair i, j in different parts of a partition of the variables, the minimiser is
// block diagonal over that partition and each block is the solution of its own
// problem (the screening rule of Witten, Friedman and Simon, 2011, and of Mazumder
// and Hastie, 2012; it follows from the optimality conditions: A = blockdiag(A_k)
// with each A_k optimal gives W = blockdiag(W_k), g_ij = S_ij off the blocks and
// |g_ij| <= lambda there).  The finest such partition is given by the connected
// components of the graph with an edge wherever |S_ij| > lambda.
//
// Components by a lock-free union-find over the edges (hooking the larger root
// under the smaller with compare-and-swap, path halving in the finds): each
// component ends up labelled by its smallest index, whatever the order in which
// the edges were processed.  Then gather / scatter between the full matrices and
// the packed blocks of the components.
#include "common.h"
#include "kernels.h"

namespace glasso {

namespace {

__device__ __forceinline__ int load_parent(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int uf_find(int* parent, int x) {
  int next = load_parent(parent + x);
  while (next != x) {
    const int up = load_parent(parent + next);
    // path halving: any ancestor is a valid parent, so the racing stores are benign
    if (up != next) __hip_atomic_store(parent + x, up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = next;
    next = up;
  }
  return x;
}

// the root of x without changing the forest (the final labelling must not race with
// path-halving stores, which may leave a node pointing at an ancestor below the root)
__device__ __forceinline__ int uf_root(const int* parent, int x) {
  int next = load_parent(parent + x);
  while (next != x) {
    x = next;
    next = load_parent(parent + x);
  }
  return x;
}

__global__ __launch_bounds__(256) void uf_init_kernel(int* parent, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) parent[i] = (int)i;
}

// one thread per entry of the strict lower triangle (grid-stride)
__global__ __launch_bounds__(256) void uf_edges_kernel(const double* S, int64_t n, int64_t lds, double lam,
                                                       int* parent, int* err) {
  const int64_t pairs = n * (n - 1) / 2;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < pairs; e += (int64_t)gridDim.x * 256) {
    // e -> (i, j), j < i, row-major over the strict lower triangle
    int64_t i = (int64_t)((1.0 + sqrt(1.0 + 8.0 * (double)e)) * 0.5);
    while (i * (i - 1) / 2 > e) --i;
    while ((i + 1) * i / 2 <= e) ++i;
    const int64_t j = e - i * (i - 1) / 2;
    if (!(fabs(S[i * lds + j]) > lam)) continue;
    int a = (int)i, b = (int)j;
    bool done = false;
    for (int tries = 0; tries < (1 << 20) && !done; ++tries) {
      a = uf_find(parent, a);
      b = uf_find(parent, b);
      if (a == b) {
        done = true;
        break;
      }
      if (a < b) {
        const int t = a;
        a = b;
        b = t;
      }
      // hook root a (the larger) under root b
      done = atomicCAS(parent + a, a, b) == a;
    }
    if (!done) atomicOr(err, 1);
  }
}

// labels: every node's root, found by read-only walks; the only stores are roots,
// so a walk that passes a relabelled node still ends at the same root
__global__ __launch_bounds__(256) void uf_flatten_kernel(int* parent, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) {
    const int r = uf_root(parent, (int)i);
    __hip_atomic_store(parent + i, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// the component holding packed element e: the last c with off[c] <= e
__device__ __forceinline__ int comp_of(const ScreenBlock* blk, int count, int64_t e) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (blk[mid].off <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void gather_blocks_kernel(const ScreenBlock* blk, int count, int64_t total,
                                                            int which) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const ScreenBlock& b = blk[comp_of(blk, count, e)];
    const int64_t q = e - b.off, r = q / b.k, c = q % b.k;
    const double* src = which ? b.A : b.S;
    double* dst = which ? b.Ak : b.Sk;
    dst[q] = src[(int64_t)b.idx[r] * b.ld + b.idx[c]];
  }
}

__global__ __launch_bounds__(256) void scatter_blocks_kernel(const ScreenBlock* blk, int count, int64_t total,
                                                             int with_w) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const ScreenBlock& b = blk[comp_of(blk, count, e)];
    const int64_t q = e - b.off, r = q / b.k, c = q % b.k;
    const int64_t at = (int64_t)b.idx[r] * b.ld + b.idx[c];
    b.A[at] = b.Ak[q];
    if (with_w && b.W) b.W[at] = b.Wk[q];
  }
}

// per block: sum |A_k| over its k x k entries, fixed order (one workgroup per block)
__global__ __launch_bounds__(256) void block_abs_sum_kernel(const ScreenBlock* blk, double* out) {
  const ScreenBlock& b = blk[blockIdx.x];
  const int64_t kk = (int64_t)b.k * b.k;
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < kk; q += 256) s += fabs(b.Ak[q]);
  __shared__ double sh[256];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void zero_fill_kernel(double* X, int64_t count) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < count; e += (int64_t)gridDim.x * 256) X[e] = 0.0;
}

unsigned grid_for(int64_t count) {
  const int64_t b = (count + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace

int screen_components(hipStream_t stream, const double* S, int64_t n, int64_t lds, double lam, int* parent,
                      int* err) {
  if (n < 1) return -1;
  hipLaunchKernelGGL(uf_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, parent, n);
  if (hipGetLastError() != hipSuccess) return -2;
  if (n > 1) {
    hipLaunchKernelGGL(uf_edges_kernel, dim3(grid_for(n * (n - 1) / 2)), dim3(256), 0, stream, S, n, lds, lam,
                       parent, err);
    if (hipGetLastError() != hipSuccess) return -2;
  }
  hipLaunchKernelGGL(uf_flatten_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, parent, n);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int gather_blocks(hipStream_t stream, const ScreenBlock* blk, int count, int64_t total, int which) {
  if (count < 1 || total < 1) return 0;
  hipLaunchKernelGGL(gather_blocks_kernel, dim3(grid_for(total)), dim3(256), 0, stream, blk, count, total, which);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int scatter_blocks(hipStream_t stream, const ScreenBlock* blk, int count, int64_t total, int with_w) {
  if (count < 1 || total < 1) return 0;
  hipLaunchKernelGGL(scatter_blocks_kernel, dim3(grid_for(total)), dim3(256), 0, stream, blk, count, total, with_w);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int block_abs_sums(hipStream_t stream, const ScreenBlock* blk, int count, double* out) {
  if (count < 1) return 0;
  hipLaunchKernelGGL(block_abs_sum_kernel, dim3(count), dim3(256), 0, stream, blk, out);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

int zero_fill(hipStream_t stream, double* X, int64_t count) {
  if (count < 1) return 0;
  hipLaunchKernelGGL(zero_fill_kernel, dim3(grid_for(count)), dim3(256), 0, stream, X, count);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace glasso
