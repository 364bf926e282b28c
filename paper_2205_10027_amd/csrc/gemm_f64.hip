// FP64 GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4_f64), LDS-staged tiles.
//
//   C = alpha * op(A) * op(B) + beta * C      (row-major C, ldc)
//
// op(A) is M x K: TA = 0 reads A[m*lda + k], TA = 1 reads A[k*lda + m].
// op(B) is K x N: TB = 0 reads B[n*ldb + k], TB = 1 reads B[k*ldb + n].
// M, N are multiples of 128 and K of 16 (callers pad every matrix).
//
// Structure flags serve the blocked Cholesky / triangular-inverse / LAUUM code:
//   lower_out : compute only tiles on or below the tile diagonal (M == N);
//               diagonal tiles are written in full, callers read their lower part.
//   a_tri     : 1 = op(A) lower triangular (zero for k > m), 2 = upper (k < m);
//               the K range of a tile is clipped and the straddling slices masked.
//   b_tri     : 1 = op(B) lower triangular (zero for k < n), 2 = upper (k > n).
//   abort_flag: when non-null and abort_flag[z] is nonzero at launch, problem z
//               of the batch is skipped (a failed pivot earlier in the same
//               factorisation, or a problem that is not being iterated).
//
// Batching: grid.y walks a first batch dimension (strides sA, sB, sC) and grid.z
// a second one (strides zA, zB, zC), e.g. the groups of one problem and the
// problems of a batch.
//
// Workgroup: 256 threads = 4 wave64s in a 2x2 arrangement.  Output tile 128x128
// (each wave 64x64 = 4x4 MFMA blocks, 64 FP64 accumulators per lane) or, for
// launches with too few tiles to fill the chip, 64x64 (each wave 2x2 blocks).
// BK=16 slices of op(A) and op(B) are double-buffered in LDS ([row][k], k
// contiguous).  Every output accumulates over k in the same order under both tile
// edges, so the choice never changes a result.
#include "common.h"
#include "kernels.h"

namespace glasso {

namespace {

constexpr int BK = 16;
constexpr int LDK = BK + 2;  // 144-byte rows keep 16-byte alignment and spread banks

// Tile edge T (128 or 64): 2x2 waves of (T/2)x(T/2); each thread stages R
// doubles of each operand per BK slice.
template <int T>
struct Tile {
  static constexpr int WT = T / 2;        // wave tile edge
  static constexpr int NBLK = WT / 16;    // 16x16 MFMA blocks per wave edge
  static constexpr int R = T * BK / 256;  // doubles per thread and operand slice
  static constexpr int TPR = BK / R;      // threads per LDS row for k-contiguous loads
};

struct GemmF64Params {
  int M, N, K;
  int tiles_m, tiles_n;
  int lower_out, a_tri, b_tri;
  double alpha, beta;
  const double* A;
  const double* B;
  double* C;
  int64_t lda, ldb, ldc;
  int64_t sA, sB, sC;  // grid.y batch strides (elements)
  int64_t zA, zB, zC;  // grid.z batch strides (elements)
  const int* abort_flag;
  const uint8_t* nz;  // zero-block map (ZBatch::nz), may be null
  int64_t snz;
  int nz_chunks, nz_row0, nz_col0, nz_k0;
};

// Stage one T x BK slice of op(X) (rows r0.., k from kt) into registers.
// TX = 0: X[row * ld + k] (k contiguous); TX = 1: X[k * ld + row] (one LDS row per
// thread: coalesced loads along the rows, 16-byte LDS stores).
template <int TX, int T>
__device__ __forceinline__ void load_slice(const double* X, int64_t ld, int r0, int kt, int tid,
                                           double (&r)[Tile<T>::R]) {
  constexpr int R = Tile<T>::R, TPR = Tile<T>::TPR;
  if (TX == 0) {
    const int row = tid / TPR, k0 = (tid % TPR) * R;
    const double2* src = reinterpret_cast<const double2*>(X + (int64_t)(r0 + row) * ld + kt + k0);
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      const double2 v = src[i];
      r[2 * i] = v.x;
      r[2 * i + 1] = v.y;
    }
  } else {
    const int row = tid % T, k0 = (tid / T) * R;
    const double* src = X + (int64_t)(kt + k0) * ld + r0 + row;
#pragma unroll
    for (int i = 0; i < R; ++i) r[i] = src[(int64_t)i * ld];
  }
}
// Triangular mask of a staged slice (rows r0.., k from kt), applied when the slice
// goes to LDS (so the loads need not have arrived before): tri 1 zeroes k > row,
// 2 zeroes k < row; for the B operand the caller passes the mirrored code.
template <int TX, int T>
__device__ __forceinline__ void mask_slice(int r0, int kt, int tid, int tri, double (&r)[Tile<T>::R]) {
  constexpr int R = Tile<T>::R, TPR = Tile<T>::TPR;
  if (!tri) return;
  const int row = TX == 0 ? tid / TPR : tid % T;
  const int k0 = TX == 0 ? (tid % TPR) * R : (tid / T) * R;
  const int m = r0 + row;
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int k = kt + k0 + i;
    if ((tri == 1 && k > m) || (tri == 2 && k < m)) r[i] = 0.0;
  }
}

template <int TX, int T>
__device__ __forceinline__ void store_slice(double (*S)[LDK], int tid, const double (&r)[Tile<T>::R]) {
  constexpr int R = Tile<T>::R, TPR = Tile<T>::TPR;
  const int row = TX == 0 ? tid / TPR : tid % T;
  const int k0 = TX == 0 ? (tid % TPR) * R : (tid / T) * R;
  double2* dst = reinterpret_cast<double2*>(&S[row][k0]);
#pragma unroll
  for (int i = 0; i < R / 2; ++i) dst[i] = make_double2(r[2 * i], r[2 * i + 1]);
}

// ROLE only separates instantiations in profiles: 0 = factorisation/inverse
// updates, 1 = the preconditioned product A Z A.
template <int TA, int TB, int ROLE, int T>
__global__ __launch_bounds__(256, T == 128 ? 2 : 4) void gemm_f64_kernel(GemmF64Params p) {
  if (p.abort_flag && p.abort_flag[blockIdx.z]) return;
  constexpr int WT = Tile<T>::WT, NBLK = Tile<T>::NBLK, R = Tile<T>::R;

  __shared__ __attribute__((aligned(16))) double As[2][T][LDK];
  __shared__ __attribute__((aligned(16))) double Bs[2][T][LDK];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // Contiguous tile ranges per XCD share operand panels in L2, but when the K
  // range depends on the tile (triangular operands) they would also give one XCD
  // all the long tiles; those launches keep the hardware's round-robin order and
  // enumerate the tiles longest K range first, so the short ones fill the tail.
  const int L = (p.a_tri || p.b_tri) ? (int)blockIdx.x : xcd_remap(blockIdx.x, gridDim.x);
  int ti, tj;
  if (p.lower_out) {
    lower_tile(L, p.tiles_m, ti, tj);  // bands from the top: longest first for LAUUM-type K >= row
  } else if (p.a_tri) {
    // K range grows with the tile row for a_tri = 1 (k <= m), shrinks for a_tri = 2
    const int q = L / p.tiles_n;
    tj = L - q * p.tiles_n;
    ti = (p.a_tri == 1) ? p.tiles_m - 1 - q : q;
  } else if (p.b_tri) {
    // K range shrinks with the tile column for b_tri = 1 (k >= n), grows for b_tri = 2
    const int q = L / p.tiles_m;
    ti = L - q * p.tiles_m;
    tj = (p.b_tri == 2) ? p.tiles_n - 1 - q : q;
  } else {
    grouped_tile(L, p.tiles_m, p.tiles_n, ti, tj);
  }
  const int m0 = ti * T, n0 = tj * T;
  // 128-wide K chunks the tile multiplies: all of them, or with a zero-block map
  // those panels of the K range that have a nonzero block in both the tile's A rows
  // and its B rows (the others add exact zeros).  No chunk: C stays as it is.
  uint64_t kmask = ~0ull;
  if (p.nz) {
    __shared__ unsigned long long kmask_sh;
    if (wave == 0) {
      // lane c looks at panel c of the K range (at most 64 panels)
      const uint8_t* f = p.nz + (int64_t)blockIdx.z * p.snz;
      const int ca = (p.nz_row0 + m0) >> 6, cb = (p.nz_col0 + n0) >> 6;
      int on = 0;
      if (lane < (p.K >> 7)) {
        const uint8_t* fs = f + (int64_t)((p.nz_k0 >> 7) + lane) * p.nz_chunks;
        int a = 0, b = 0;
#pragma unroll
        for (int c = 0; c < T / 64; ++c) {
          a |= fs[ca + c];
          b |= fs[cb + c];
        }
        on = a && b;
      }
      const unsigned long long bal = __ballot(on);
      if (lane == 0) kmask_sh = bal;
    }
    __syncthreads();
    kmask = kmask_sh;
    if (!kmask) return;
  }

  const double* A = p.A + (int64_t)blockIdx.y * p.sA + (int64_t)blockIdx.z * p.zA;
  const double* B = p.B + (int64_t)blockIdx.y * p.sB + (int64_t)blockIdx.z * p.zB;
  double* C = p.C + (int64_t)blockIdx.y * p.sC + (int64_t)blockIdx.z * p.zC;

  int kbeg = 0, kend = p.K;
  if (p.a_tri == 1) kend = min(kend, m0 + T);
  if (p.a_tri == 2) kbeg = max(kbeg, m0);
  if (p.b_tri == 1) kbeg = max(kbeg, n0);
  if (p.b_tri == 2) kend = min(kend, n0 + T);
  kbeg = max(kbeg, __builtin_ctzll(kmask) << 7);
  // the slice after kt: the next one of its chunk, else the first of the next chunk
  // in kmask (kend when there is none); without a map simply the next one (K may
  // exceed the 64 chunks a mask holds)
  auto next_k = [&](int kt) -> int {
    const int nk = kt + BK;
    if (!p.nz || (nk & 127)) return nk;
    const int c = kt >> 7;
    const uint64_t later = (c >= 63) ? 0ull : (kmask & (~0ull << (c + 1)));
    return later ? (int)(__builtin_ctzll(later) << 7) : kend;
  };
  // op(B) is indexed [k][n]: its "lower" (zero for k < n) is the staged row's k < row
  const int btri = p.b_tri == 1 ? 2 : (p.b_tri == 2 ? 1 : 0);

  v4d acc[NBLK][NBLK];
#pragma unroll
  for (int i = 0; i < NBLK; ++i)
#pragma unroll
    for (int j = 0; j < NBLK; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

  // With a zero-block map (sparse factors) a BK slice whose op(A) or op(B) part is
  // all zero adds exact zeros: its MFMAs are skipped, decided at the barrier that
  // publishes the slice.  Dense launches use plain barriers.
  const bool sparse = p.nz != nullptr;
  auto nonzero = [&](const double (&r)[R]) {
    bool any = false;
#pragma unroll
    for (int i = 0; i < R; ++i) any = any || r[i] != 0.0;
    return any;
  };
  // The slice in LDS buffer `cur` is multiplied while the next one is stored to the
  // other buffer from one of PD register sets, each holding a slice whose loads were
  // issued PD slices earlier.  PD > 1 for 64x64 tiles: a long K range on few tiles
  // (the updates of a sparse factorisation past a few dense rows) then waits on
  // global-load latency once per PD slices instead of once per slice.
  constexpr int PD = T == 64 ? 3 : 1;
  if (kbeg < kend) {
    double ra[PD][R], rb[PD][R];
    load_slice<TA, T>(A, p.lda, m0, kbeg, tid, ra[0]);
    load_slice<TB, T>(B, p.ldb, n0, kbeg, tid, rb[0]);
    mask_slice<TA, T>(m0, kbeg, tid, p.a_tri, ra[0]);
    mask_slice<TB, T>(n0, kbeg, tid, btri, rb[0]);
    store_slice<TA, T>(As[0], tid, ra[0]);
    store_slice<TB, T>(Bs[0], tid, rb[0]);
    // whether a stored slice has a nonzero in op(A) and in op(B): per wave a ballot
    // each, bit 0 and bit 1 of the wave's word, read by all after the one barrier
    // that publishes the slice (two words per wave used in turn: a wave can write
    // the next slice's word only after every wave has passed this barrier)
    __shared__ unsigned int zflags[2][4];
    int zpar = 0;
    auto publish = [&](const double (&xa)[R], const double (&xb)[R]) -> bool {
      if (!sparse) {
        __syncthreads();
        return true;
      }
      const uint64_t ba = __ballot(nonzero(xa)), bb = __ballot(nonzero(xb));
      if (lane == 0) zflags[zpar][wave] = (ba ? 1u : 0u) | (bb ? 2u : 0u);
      __syncthreads();
      const unsigned int f = zflags[zpar][0] | zflags[zpar][1] | zflags[zpar][2] | zflags[zpar][3];
      zpar ^= 1;
      return f == 3u;
    };
    bool live = publish(ra[0], rb[0]);  // the slice in As[cur], Bs[cur] has a nonzero product
    // kq[s]: the slice register set s holds (kend: none); klast: the last one issued.
    // Past the last slice a set is loaded with the last valid one and never used: the
    // loads stay unconditional, so the compiler waits for each only where it is used.
    int kq[PD];
    int klast = kbeg;
#pragma unroll
    for (int s = 0; s < PD; ++s) {
      klast = (klast < kend) ? next_k(klast) : kend;
      kq[s] = klast;
      const int kl = min(klast, kend - BK);
      load_slice<TA, T>(A, p.lda, m0, kl, tid, ra[s]);
      load_slice<TB, T>(B, p.ldb, n0, kl, tid, rb[s]);
    }
    // Straight-line groups of PD steps (no exit inside a group, every load, store and
    // barrier unconditional) let the compiler wait, before storing set s, only for
    // that set's loads.  `have` says whether LDS buffer `cur` holds a slice; past the
    // last one a group finishes with steps that multiply nothing.
    int cur = 0;
    bool have = true;
    do {
#pragma unroll
      for (int s = 0; s < PD; ++s) {
        if (have && live) {
#pragma unroll
          for (int kk = 0; kk < BK / 4; ++kk) {
            double af[NBLK], bf[NBLK];
            const int kc = kk * 4 + (lane >> 4);
#pragma unroll
            for (int i = 0; i < NBLK; ++i) af[i] = As[cur][wm * WT + i * 16 + (lane & 15)][kc];
#pragma unroll
            for (int j = 0; j < NBLK; ++j) bf[j] = Bs[cur][wn * WT + j * 16 + (lane & 15)][kc];
            // a 16x4 operand block that is zero in the whole wave adds exact zeros to
            // its row (or column) of output blocks: past a sparse factor's dense rows
            // most of a tile's rows are zero (launches with a zero-block map only)
            unsigned int la = (1u << NBLK) - 1u, lb = (1u << NBLK) - 1u;
            if (sparse) {
#pragma unroll
              for (int i = 0; i < NBLK; ++i) {
                const uint64_t b = __ballot(af[i] != 0.0);
                if (!b) la &= ~(1u << i);
              }
#pragma unroll
              for (int j = 0; j < NBLK; ++j) {
                const uint64_t b = __ballot(bf[j] != 0.0);
                if (!b) lb &= ~(1u << j);
              }
            }
#pragma unroll
            for (int i = 0; i < NBLK; ++i)
#pragma unroll
              for (int j = 0; j < NBLK; ++j)
                if (((la >> i) & 1u) && ((lb >> j) & 1u))
                  acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
          }
        }
        // the slices are consumed in k order: set s holds the next one (if any)
        have = have && kq[s] < kend;
        mask_slice<TA, T>(m0, kq[s], tid, p.a_tri, ra[s]);
        mask_slice<TB, T>(n0, kq[s], tid, btri, rb[s]);
        store_slice<TA, T>(As[cur ^ 1], tid, ra[s]);
        store_slice<TB, T>(Bs[cur ^ 1], tid, rb[s]);
        live = publish(ra[s], rb[s]);
        // refill set s with the slice PD places further on
        klast = (klast < kend) ? next_k(klast) : kend;
        kq[s] = klast;
        const int kl = min(klast, kend - BK);
        load_slice<TA, T>(A, p.lda, m0, kl, tid, ra[s]);
        load_slice<TB, T>(B, p.ldb, n0, kl, tid, rb[s]);
        cur ^= 1;
      }
    } while (have);
  }

  // D[r][c] of a 16x16 block sits in lane (c + 16*(r%4)), element r/4
  // (v_mfma_f64_16x16x4f64 output layout, checked on gfx950).
  // With beta != 0 every old value of the tile is loaded before the first store:
  // loads interleaved with stores to C, which the compiler must assume may alias,
  // would each wait for the one before.
  const double alpha = p.alpha, beta = p.beta;
  double* const Cw = C + (int64_t)(m0 + wm * WT + (lane >> 4)) * p.ldc + n0 + wn * WT + (lane & 15);
  double old[NBLK][NBLK][4];
#pragma unroll
  for (int i = 0; i < NBLK; ++i)
#pragma unroll
    for (int j = 0; j < NBLK; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) old[i][j][r] = 0.0;
  if (beta != 0.0) {
#pragma unroll
    for (int i = 0; i < NBLK; ++i)
#pragma unroll
      for (int j = 0; j < NBLK; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) old[i][j][r] = Cw[(int64_t)(i * 16 + 4 * r) * p.ldc + j * 16];
  }
#pragma unroll
  for (int i = 0; i < NBLK; ++i)
#pragma unroll
    for (int j = 0; j < NBLK; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double v = alpha * acc[i][j][r];
        if (beta != 0.0) v += beta * old[i][j][r];
        Cw[(int64_t)(i * 16 + 4 * r) * p.ldc + j * 16] = v;
      }
}

template <int T>
void launch(int ta, int tb, int role, dim3 grid, hipStream_t stream, const GemmF64Params& p) {
  dim3 block(256);
  if (role == 1 && ta == 0 && tb == 0)
    hipLaunchKernelGGL((gemm_f64_kernel<0, 0, 1, T>), grid, block, 0, stream, p);
  else if (ta == 0 && tb == 0)
    hipLaunchKernelGGL((gemm_f64_kernel<0, 0, 0, T>), grid, block, 0, stream, p);
  else if (ta == 0 && tb == 1)
    hipLaunchKernelGGL((gemm_f64_kernel<0, 1, 0, T>), grid, block, 0, stream, p);
  else if (ta == 1 && tb == 0)
    hipLaunchKernelGGL((gemm_f64_kernel<1, 0, 0, T>), grid, block, 0, stream, p);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<1, 1, 0, T>), grid, block, 0, stream, p);
}

}  // namespace

namespace {
thread_local int small_tile_below = 256;  // see set_gemm_f64_small_tile_below
}

void set_gemm_f64_small_tile_below(int tiles) { small_tile_below = tiles < 0 ? 0 : tiles; }
int get_gemm_f64_small_tile_below() { return small_tile_below; }

int gemm_f64(hipStream_t stream, int ta, int tb, int M, int N, int K, double alpha,
             const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
             int64_t ldc, int lower_out, int a_tri, int b_tri, const int* abort_flag, int batch,
             int64_t sA, int64_t sB, int64_t sC, int role, const ZBatch& zb, int in_place) {
  if (M <= 0 || N <= 0 || batch <= 0 || zb.count <= 0) return 0;
  if (M % 128 || N % 128 || K % BK || K < 0) return -1;
  if (lower_out && M != N) return -1;
  GemmF64Params p;
  p.M = M;
  p.N = N;
  p.K = K;
  p.lower_out = lower_out;
  p.a_tri = a_tri;
  p.b_tri = b_tri;
  p.alpha = alpha;
  p.beta = beta;
  p.A = A;
  p.B = B;
  p.C = C;
  p.lda = lda;
  p.ldb = ldb;
  p.ldc = ldc;
  p.sA = sA;
  p.sB = sB;
  p.sC = sC;
  p.zA = zb.sA;
  p.zB = zb.sB;
  p.zC = zb.sC;
  p.abort_flag = abort_flag;
  p.nz = zb.nz;
  p.snz = zb.snz;
  p.nz_chunks = zb.nz_chunks;
  p.nz_row0 = zb.nz_row0;
  p.nz_col0 = zb.nz_col0;
  p.nz_k0 = zb.nz_k0;
  if (zb.nz && (ta || tb || K % 128 || K > 64 * 128 || zb.nz_k0 % 128 || zb.nz_row0 % 64 || zb.nz_col0 % 64))
    return -1;
  // 128x128 tiles unless the launch has too few of them to fill the chip; both
  // tile edges accumulate every output in the same k order (bitwise equal results).
  // An in-place product (C aliases A, N = 128) keeps 128-wide tiles: one workgroup
  // must read a whole row block of A before it overwrites it.
  const int64_t t128 = (int64_t)(lower_out ? (M / 128) * (M / 128 + 1) / 2 : (M / 128) * (N / 128)) * batch * zb.count;
  if (in_place && N != 128) return -1;
  const int T = (!in_place && t128 < small_tile_below) ? 64 : 128;
  p.tiles_m = M / T;
  p.tiles_n = N / T;
  const int tiles = lower_out ? p.tiles_m * (p.tiles_m + 1) / 2 : p.tiles_m * p.tiles_n;
  dim3 grid(tiles, batch, zb.count);
  if (T == 64)
    launch<64>(ta, tb, role, grid, stream, p);
  else
    launch<128>(ta, tb, role, grid, stream, p);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace glasso
