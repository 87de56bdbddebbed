// Batched sweeps in step-synchronous form (FP64 storage, n <= 512).  Every problem of the batch
// runs the same sequence of block steps of Sec. 4.2's algorithms with 64-wide blocks, and each step
// is ONE grouped launch over all problems that have it:
//   factor   (chol_blocked, left-looking as Sec. 4.2 writes it):  for s = 0, 1, ...:
//              U   [D_s; C] -= [R; B] R^T over the columns left of block s   (64-row tiles)
//              F1  D_s <- chol_unblocked(D_s) and D_s^-1          (one wave per problem)
//              F2  C <- C D_s^-T                                   (64-row tiles)
//   GP loss  z = L^-1 y by block substitution inside the factor steps (F1 forms z_s = D_s^-1 t_s,
//            F2 subtracts L_rs z_s from the t of the rows below) and f at each problem's last
//            block; L-bar = diag(1/L_ii) - tril(w z^T), w = L^-T z, is never stored: the reverse
//            steps compute w block by block (b2_gp_w) and form L-bar's entries where they read them
//   reverse  (chol_blocked_rev in the left-looking order of the single-matrix sweep), problem p
//            at step t takes its block b = nblk_p - 1 - t, so every problem starts with its last
//            block:
//              R0  X = L-bar_C - 2 S_sym[k:, k:] L[k:, j:k]        (64-row tiles, in place)
//              R1  C-bar / 2 = X D^-1 / 2 with its mirrored store          (64-row tiles)
//              R2  D-bar = tril(L-bar_D) - tril(C-bar^T C)                  (one workgroup per problem)
//              R3  D-bar <- D^-T Phi(D^T D-bar) D^-1, symmetric part (eqn (symrev) on the
//                  block: the symbolic form of chol_unblocked_rev)   (one wave per problem)
// so the block products of the large problems spread over the whole GPU, and the diagonal-block
// routines (POTF2 with the single-wave cores of cg_diag.hpp, the reverse block as MFMA tiles) run
// four per compute unit with every wave busy.  Problems are ordered largest first; a plan (order, per-step tile counts
// and their prefix sums) is built on the device once per call, so the host needs only n_max.
// Every output element is computed by the same operations in the same order whatever the batch,
// so results are bitwise independent of the other problems.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cg_batched.hpp"
#include "cg_diag.hpp"

namespace cg {

constexpr int B2_NB = 64;                              // block width
constexpr int B2_MAXBLK = BATCH_NMAX / B2_NB;          // 8 blocks at n = 512
constexpr int B2_PACKED = B2_NB * (B2_NB + 1) / 2;     // 2080 doubles: a packed 64-block
constexpr int B2_BLK = B2_NB * B2_NB;                  // 4096 doubles: a square 64-block
// Prefix arrays of the plan: F2 tiles per step s, U tiles per step s, reverse-step tiles per
// step t, diagonal blocks per problem.
constexpr int B2_Q_F2 = 0, B2_Q_UP = B2_MAXBLK, B2_Q_RV = 2 * B2_MAXBLK, B2_Q_BLK = 3 * B2_MAXBLK;
constexpr int B2_NPREF = 3 * B2_MAXBLK + 1;

struct B2Args {
  int op;                   // BatchOp: FACTOR, REV, GP or FACTOR_REV
  int batch;                // positions: the problems this plan takes
  int nprob;                // problems in the caller's arrays
  int sel_mod, sel_rem;     // this plan takes the problems i < nprob with i % sel_mod == sel_rem
  int sbar_form;
  int n_max;
  const int64_t *n;
  double *const *A;         // factor ops: Sigma -> L;  REV: L-bar -> Sigma-bar
  const int64_t *lda;
  const double *const *L;   // REV: the factors
  const int64_t *ldl;
  const double *const *y;   // GP: right-hand sides
  double *const *G;         // GP: Sigma-bar out;  FACTOR_REV: L-bar -> Sigma-bar
  const int64_t *ldg;
  double *f;                // GP: losses
  int *info;                // factor ops
  // plan and scratch (workspace)
  int *order;               // ordered position -> problem index
  int *nv;                  // ordered position -> size (0 for a skipped problem)
  int *pref;                // B2_NPREF arrays of batch + 1 ints
  int *count;               // B2_MAXBLK: positions with more than s blocks
  double *dinv;             // per position: ceil(n_max / 64) inverses of 64-blocks
  double *vec;              // per position: z and w (2 n_max)
  int64_t dinv_stride, vec_stride;  // doubles per position
};

__device__ __forceinline__ int b2_nblk(int n) { return (n + B2_NB - 1) / B2_NB; }
__device__ __forceinline__ int b2_below(int n, int b) { return max(0, n - min(n, (b + 1) * B2_NB)); }
__device__ __forceinline__ int b2_cdiv(int a, int b) { return (a + b - 1) / b; }

// Tiles of prefix array q for a problem of size n.
__device__ __forceinline__ int b2_tiles(int q, int n) {
  const int nb = b2_nblk(n);
  if (q < B2_Q_UP) {
    const int s = q - B2_Q_F2;
    return nb > s ? b2_cdiv(b2_below(n, s), B2_NB) : 0;
  }
  if (q < B2_Q_RV) {
    const int s = q - B2_Q_UP;
    return (s > 0 && nb > s) ? b2_cdiv(n - s * B2_NB, B2_NB) : 0;
  }
  if (q < B2_Q_BLK) {
    const int t = q - B2_Q_RV;
    return nb > t ? b2_cdiv(b2_below(n, nb - 1 - t), B2_NB) : 0;
  }
  return nb;
}

__device__ __forceinline__ bool b2_factor_op(int op) {
  return op == BATCH_FACTOR || op == BATCH_GP || op == BATCH_FACTOR_REV;
}

// The problems' arrays in their storage type T (double, or float for FP32 storage: the kernels
// compute in FP64 and round every value they store): A, the factor of problem i (the factor ops
// overwrite A with it; REV reads L), the array the reverse sweep works in (REV: A; GP and
// FACTOR_REV: G), y and the losses.
// The pointers come out of pointer arrays in device memory, so the compiler cannot tell which
// memory they address, and accesses through them compile to flat loads and stores, which also
// count against the LDS wait counter: every LDS wait in the tile loops after a store would wait
// for the store as well.  Re-typed as a global-memory pointer, passed through an empty asm (else
// the compiler folds the two casts away and the pointer is generic again), they compile to global
// loads and stores.
template <typename T>
__device__ __forceinline__ T *as_global(T *p) {
  __attribute__((address_space(1))) T *q = (__attribute__((address_space(1))) T *)p;
  asm("" : "+v"(q));
  return (T *)q;
}
template <typename T>
__device__ __forceinline__ T *b2_A(const B2Args &a, int i) { return as_global(reinterpret_cast<T *>(a.A[i])); }
template <typename T>
__device__ __forceinline__ const T *b2_L(const B2Args &a, int i, int64_t &ld) {
  if (a.op == BATCH_REV) { ld = a.ldl[i]; return as_global(reinterpret_cast<const T *>(a.L[i])); }
  ld = a.lda[i];
  return as_global(reinterpret_cast<T *>(a.A[i]));
}
template <typename T>
__device__ __forceinline__ T *b2_G(const B2Args &a, int i, int64_t &ld) {
  if (a.op == BATCH_REV) { ld = a.lda[i]; return as_global(reinterpret_cast<T *>(a.A[i])); }
  ld = a.ldg[i];
  return as_global(reinterpret_cast<T *>(a.G[i]));
}
template <typename T>
__device__ __forceinline__ double b2_y(const B2Args &a, int i, int r) { return as_global(reinterpret_cast<const T *>(a.y[i]))[r]; }
template <typename T>
__device__ __forceinline__ void b2_set_f(const B2Args &a, int i, double v) { reinterpret_cast<T *>(a.f)[i] = (T)v; }

// Plan, part 1 (one workgroup of 1024 threads): over the problems the plan takes (every
// sel_mod-th from sel_rem), validate each (size in [0, n_max], leading dimensions >= size;
// otherwise it is skipped: size 0 in the plan, info -1), order them by decreasing size (counting
// sort), count the positions with more than s blocks, and initialise info (0) and, for n == 0, the
// loss (0).
template <typename T>
__global__ __launch_bounds__(1024) void b2_order_kernel(B2Args a) {
  __shared__ int cnt[BATCH_NMAX + 2];
  __shared__ int blk[B2_MAXBLK];
  const int tid = threadIdx.x;
  for (int i = tid; i < BATCH_NMAX + 2; i += blockDim.x) cnt[i] = 0;
  if (tid < B2_MAXBLK) blk[tid] = 0;
  __syncthreads();
  auto key_of = [&](int i) -> int {
    const int64_t v = a.n[i];
    bool ok = v >= 0 && v <= a.n_max && a.lda[i] >= v;
    if (a.op == BATCH_REV) ok = ok && a.ldl[i] >= v;
    if (a.op == BATCH_GP || a.op == BATCH_FACTOR_REV) ok = ok && a.ldg[i] >= v;
    return ok ? (int)v : -1;
  };
  const int step = blockDim.x * a.sel_mod;
  for (int i = a.sel_rem + tid * a.sel_mod; i < a.nprob; i += step) {
    const int key = max(0, key_of(i));
    atomicAdd(&cnt[BATCH_NMAX - key], 1);  // bin 0 holds the largest size
    const int nb = b2_nblk(key);
    for (int s = 0; s < nb; ++s) atomicAdd(&blk[s], 1);
  }
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int i = 0; i < BATCH_NMAX + 1; ++i) {
      const int c = cnt[i];
      cnt[i] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int i = a.sel_rem + tid * a.sel_mod; i < a.nprob; i += step) {
    const int key = key_of(i);
    const int pos = atomicAdd(&cnt[BATCH_NMAX - max(0, key)], 1);
    a.order[pos] = i;
    a.nv[pos] = max(0, key);
    if (b2_factor_op(a.op)) a.info[i] = key < 0 ? -1 : 0;
    if (a.op == BATCH_GP && key == 0) b2_set_f<T>(a, i, 0.0);
  }
  if (tid < B2_MAXBLK) a.count[tid] = blk[tid];
}

// Plan, part 2 (B2_NPREF workgroups of 1024 threads, one per prefix array): exclusive prefix sum
// over the ordered positions of the tiles each problem has in that launch; entry batch holds the
// total.
__global__ __launch_bounds__(1024) void b2_prefix_kernel(B2Args a) {
  __shared__ int sc[1024];
  __shared__ int carry;
  const int q = blockIdx.x, tid = threadIdx.x;
  int *pr = a.pref + (int64_t)q * (a.batch + 1);
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < a.batch; base += 1024) {
    const int p = base + tid;
    const int v = p < a.batch ? b2_tiles(q, a.nv[p]) : 0;
    sc[tid] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {  // inclusive Hillis-Steele scan
      const int add = tid >= o ? sc[tid - o] : 0;
      __syncthreads();
      sc[tid] += add;
      __syncthreads();
    }
    if (p < a.batch) pr[p] = carry + sc[tid] - v;
    __syncthreads();
    if (tid == 1023) carry += sc[1023];
    __syncthreads();
  }
  if (tid == 0) pr[a.batch] = carry;
}

// Position p of item `it` in prefix array pr (last p with pr[p] <= it; items of empty problems
// never match).
__device__ __forceinline__ int b2_find(const int *pr, int batch, int it) {
  int lo = 0, hi = batch;  // pr[lo] <= it < pr[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pr[mid] <= it) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------------------------
// 64 x 64 MFMA tile product by one 256-thread workgroup: four waves in a 2 x 2 arrangement, each
// owning a 32 x 32 quadrant as 2 x 2 v_mfma_f64_16x16x4_f64 accumulators; K staged through LDS 16
// deep, double-buffered from registers (one barrier per K-step), so ragged operands just return 0
// from their accessors.  acc[a][b][e] holds (row 32 wm + 16 a + 4 e + lane/16, column
// 32 wn + 16 b + lane % 16).  AK / BK: the operand is contiguous along k in memory (the load
// mapping follows it so that loads coalesce).
constexpr int T64_LD = B2_NB + 4;
constexpr int T64_BK = 16;                     // K depth of one LDS stage
constexpr int T64_LDS = 4 * T64_BK * T64_LD;  // doubles: two stages of A and B

__device__ __forceinline__ int t64_row(int a, int e) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  return 32 * (wave >> 1) + 16 * a + 4 * e + (lane >> 4);
}
__device__ __forceinline__ int t64_col(int b) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  return 32 * (wave & 1) + 16 * b + (lane & 15);
}

template <bool AK, bool BK, class FA, class FB>
__device__ __forceinline__ void t64_mma(dbl4 (&acc)[2][2], FA A, FB B, int K, double *lds) {
  double *const lb = (double *)(__attribute__((address_space(3))) double *)lds;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  auto As = [&](int st) { return lb + st * T64_BK * T64_LD; };
  auto Bs = [&](int st) { return lb + (2 + st) * T64_BK * T64_LD; };
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = dbl4{0, 0, 0, 0};
  constexpr int NL = T64_BK / 4;  // loads per thread per operand and stage
  // Prefetch registers in the operands' own storage types (the accessors' return types): values
  // are widened only when they go to LDS, so a float operand's loads stay in flight across the
  // K-step instead of being waited for by an early conversion.
  typedef decltype(A(0, 0)) TA;
  typedef decltype(B(0, 0)) TB;
  TA ra[NL];
  TB rb[NL];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = u * 256 + tid;
      const int i = AK ? (e / T64_BK) : (e & 63), k = AK ? (e % T64_BK) : (e >> 6);
      ra[u] = (k0 + k < K) ? A(i, k0 + k) : TA(0);
      const int j = BK ? (e / T64_BK) : (e & 63), kb = BK ? (e % T64_BK) : (e >> 6);
      rb[u] = (k0 + kb < K) ? B(k0 + kb, j) : TB(0);
    }
  };
  auto store = [&](int st) {
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int e = u * 256 + tid;
      const int i = AK ? (e / T64_BK) : (e & 63), k = AK ? (e % T64_BK) : (e >> 6);
      As(st)[k * T64_LD + i] = (double)ra[u];
      const int j = BK ? (e / T64_BK) : (e & 63), kb = BK ? (e % T64_BK) : (e >> 6);
      Bs(st)[kb * T64_LD + j] = (double)rb[u];
    }
  };
  const int nkt = (K + T64_BK - 1) / T64_BK;
  if (nkt > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  const int fk = lane >> 4, fi = lane & 15;
  for (int kt = 0; kt < nkt; ++kt) {
    const int st = kt & 1;
    if (kt + 1 < nkt) load((kt + 1) * T64_BK);
    const double *as = As(st), *bs = Bs(st);
#pragma unroll
    for (int kk = 0; kk < T64_BK; kk += 4) {
      double af[2], bf[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) af[t] = as[(kk + fk) * T64_LD + 32 * wm + 16 * t + fi];
#pragma unroll
      for (int t = 0; t < 2; ++t) bf[t] = bs[(kk + fk) * T64_LD + 32 * wn + 16 * t + fi];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[x], bf[y], acc[x][y], 0, 0, 0);
    }
    if (kt + 1 < nkt) store(st ^ 1);
    __syncthreads();
  }
}

// Elementwise epilogue over the tile: out(r, c, v) for every accumulator element.
template <class F>
__device__ __forceinline__ void t64_each(const dbl4 (&acc)[2][2], F out) {
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int e = 0; e < 4; ++e) out(t64_row(x, e), t64_col(y), acc[x][y][e]);
}

// Split-K SYRK partials of the single-matrix reverse sweep on 64 x 64 tiles:
//   P[z][x][y] = sum_{k in split z} Cb[k][x] L[k][y]   for the lower 64-tiles (x >= y) of a w x w
// output (w <= 256; K = m rows of the block column), workgroup blockIdx.x = u + ntiles * z with u
// the lower tile in row order.  Many small tiles fill the GPU with short K-splits and write less
// partial data than 128 x 128 tiles would; the splits are summed in order by the caller's reduction.
__global__ __launch_bounds__(256) void syrk_t64_kernel(int m, int w, const double *Cb, int64_t ldcb, const double *L,
                                                        int64_t ldl, int kchunk, double *P) {
  __shared__ double lds[T64_LDS];
  const int nt = (w + B2_NB - 1) / B2_NB, ntiles = nt * (nt + 1) / 2;
  const int u = blockIdx.x % ntiles, z = blockIdx.x / ntiles;
  int ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= u) ++ti;
  const int tj = u - ti * (ti + 1) / 2;
  const int k0 = z * kchunk, K = min(m, k0 + kchunk) - k0;
  const int x0 = ti * B2_NB, y0 = tj * B2_NB;
  dbl4 acc[2][2];
  t64_mma<false, false>(
      acc, [&](int x, int kk) { return (x0 + x < w) ? Cb[(int64_t)(k0 + kk) * ldcb + x0 + x] : 0.0; },
      [&](int kk, int y) { return (y0 + y < w) ? L[(int64_t)(k0 + kk) * ldl + y0 + y] : 0.0; }, K, lds);
  double *Pz = P + (int64_t)z * w * w;
  t64_each(acc, [&](int r, int c, double v) {
    if (x0 + r < w && y0 + c < w) Pz[(int64_t)(x0 + r) * w + y0 + c] = v;
  });
}

// ---------------------------------------------------------------------------------------------
// Diagonal blocks (w <= 64) one WAVE each: the Level-2 cores of cg_diag.hpp are single-wave
// already, so a wave can run a whole 64-block -- its two 32-column inner blocks, the products
// between them as 16 x 16 MFMA tiles, the inverse -- with only wave-level ordering of its LDS
// accesses, and the four waves of a workgroup take four different problems.  Each wave holds two
// packed 64-blocks (33 KB), so a compute unit runs four blocks at once with every wave busy.
constexpr int B2W_WAVES = 4;
constexpr int B2W_LDS = 2 * B2_PACKED;  // doubles per wave

// Packed lower triangle of a w x w block (1 <= w <= 64, row-major source) into Dp, by one wave,
// sixteen rows of loads in flight.  The loads are unconditional, their row and column clamped into
// the block's lower triangle: a load under a per-row condition gets its own branch, and in FP32
// storage the widening then follows it inside the branch with a wait, one row at a time.
template <typename T>
__device__ __forceinline__ void wave_load_lower(double *Dp, const T *src, int64_t ld, int w) {
  const int lane = threadIdx.x & 63;
  for (int r0 = 0; r0 < w; r0 += 16) {
    T v[16];  // in the source's type: widened as they go to LDS, after all sixteen are in flight
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int r = min(r0 + u, w - 1);
      v[u] = src[(int64_t)r * ld + min(lane, r)];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int r = r0 + u;
      if (r < w && lane <= r) Dp[pidx(r, lane)] = (double)v[u];
    }
  }
}

// D <- chol_unblocked(D) and Xp = D^-1 for the w x w block (w <= 64) packed in Dp, by one wave:
// inner block 0 with the rows below it (one pass of the Level-2 core), the update of inner block 1
// (three 16 x 16 MFMA tiles), inner block 1, then X00 and X11 in one pass and X10 = -X11 (D10 X00).  Returns the
// first column with a non-positive or NaN pivot, or -1.
__device__ int wave_potf2_64(double *Dp_, double *Xp_, int w) {
  lds_double *Dp = lds_view(Dp_), *Xp = lds_view(Xp_);
  const int ib0 = min(INNER, w), ib1 = w - ib0;
  int bad = panel_core32<false>(Dp_, 0, ib0, w, INNER, true);
  wave_sync();
  if (ib1 > 0) {
    // D11 <- D11 - D10 D10^T, lower 16 x 16 tiles, K = 32
    dbl4 acc[3];
    const int nt = (ib1 + 15) / 16;
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int ti = (u == 0) ? 0 : 1, tj = (u == 2) ? 1 : 0;
      acc[u] = dbl4{0, 0, 0, 0};
      if (ti < nt) {
        auto A = [&](int i, int k) { const int r = 16 * ti + i; return r < ib1 ? Dp[pidx(INNER + r, k)] : 0.0; };
        auto B = [&](int k, int j) { const int c = 16 * tj + j; return c < ib1 ? Dp[pidx(INNER + c, k)] : 0.0; };
        acc[u] = tile_mma(acc[u], A, B, INNER);
      }
    }
    wave_sync();
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int ti = (u == 0) ? 0 : 1, tj = (u == 2) ? 1 : 0;
      if (ti >= nt) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 16 * ti + tile_row(e), c = 16 * tj + tile_col();
        if (r < ib1 && c <= r) Dp[pidx(INNER + r, INNER + c)] -= acc[u][e];
      }
    }
    wave_sync();
    const int f = panel_core32<false>(Dp_, INNER, ib1, w, 2 * INNER, true);
    if (bad < 0 && f >= 0) bad = INNER + f;
    wave_sync();
  }
  wave_trinv32x2(Dp_, Xp_, ib0, ib1);
  if (ib1 > 0) {
    wave_sync();
    // Y = D10 X00 (ib1 x 32), then X10 = -X11 Y, each as up to 2 x 2 tiles held in registers
    const int nt = (ib1 + 15) / 16;
    dbl4 y[2][2], x[2][2];
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        y[ti][tj] = dbl4{0, 0, 0, 0};
        if (ti >= nt) continue;
        auto A = [&](int i, int k) { const int r = 16 * ti + i; return r < ib1 ? Dp[pidx(INNER + r, k)] : 0.0; };
        auto B = [&](int k, int j) { const int c = 16 * tj + j; return k >= c ? Xp[pidx(k, c)] : 0.0; };
        y[ti][tj] = tile_mma(y[ti][tj], A, B, INNER);
      }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        if (ti >= nt) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = 16 * ti + tile_row(e), c = 16 * tj + tile_col();
          if (r < ib1) Xp[pidx(INNER + r, c)] = y[ti][tj][e];
        }
      }
    wave_sync();
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        x[ti][tj] = dbl4{0, 0, 0, 0};
        if (ti >= nt) continue;
        auto A = [&](int i, int k) {
          const int r = 16 * ti + i;
          return (r < ib1 && k <= r) ? Xp[pidx(INNER + r, INNER + k)] : 0.0;
        };
        auto B = [&](int k, int j) { return k < ib1 ? Xp[pidx(INNER + k, 16 * tj + j)] : 0.0; };
        x[ti][tj] = tile_mma(x[ti][tj], A, B, min(ib1, 16 * ti + 16));
      }
    wave_sync();
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        if (ti >= nt) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = 16 * ti + tile_row(e), c = 16 * tj + tile_col();
          if (r < ib1) Xp[pidx(INNER + r, c)] = -x[ti][tj][e];
        }
      }
  }
  wave_sync();
  return bad;
}

// The symmetric gradient of a w x w diagonal block (w <= 64) from its symbolic form (eqn (symrev)
// on the block, as the single-matrix sweeps take by default), by one wave on 16 x 16 MFMA tiles
// with triangular K ranges:
//   P = tril(D)^T tril(D-bar)   (lower tiles);   Y = (Phi(P) + Phi(P)^T) / 2, written over D-bar;
//   then per 16-column block of R = Y D^-1 (four tiles, in registers) the lower tiles of
//   S = D^-T R, whose B operand is R's accumulator layout as it stands (element e of a tile holds
//   rows 4e + lane/16, the rows of K-slice e); S is symmetric and goes to both triangles of G.
// D packed in Dp, D-bar packed in Bp (both overwritten), Dinv row-major 64 x 64 with zeros outside
// w x w (staged into Dp once P is formed); G: the block's place in the output, leading dim ldg.
template <typename T>
__device__ void wave_diag_rev_sym64(double *Dp_, double *Bp_, const double *Dinv, int w, T *G, int64_t ldg) {
  lds_double *Dp = lds_view(Dp_), *Bp = lds_view(Bp_);
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  dbl4 P[10];
#pragma unroll
  for (int ti = 0, u = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj <= ti; ++tj, ++u) {
      dbl4 acc = dbl4{0, 0, 0, 0};
      const int ci = 16 * ti + li, cj = 16 * tj + li;
#pragma unroll
      for (int k0 = 16 * ti; k0 < B2_NB; k0 += 4) {
        const int k = k0 + lk;
        const double a = (k < w && k >= ci) ? Dp[pidx(k, ci)] : 0.0;  // D[k][i]
        const double b = (k < w && k >= cj) ? Bp[pidx(k, cj)] : 0.0;  // D-bar[k][j]
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
      }
      P[u] = acc;
    }
  wave_sync();
  wave_load_lower(Dp_, Dinv, B2_NB, w);
#pragma unroll
  for (int ti = 0, u = 0; ti < 4; ++ti)
#pragma unroll
    for (int tj = 0; tj <= ti; ++tj, ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 16 * ti + 4 * e + lk, c = 16 * tj + li;
        if (c <= r) Bp[pidx(r, c)] = 0.5 * P[u][e];
      }
  wave_sync();
  auto Y = [&](int r, int c) { return r >= c ? Bp[pidx(r, c)] : Bp[pidx(c, r)]; };
  auto X = [&](int r, int c) { return (r >= c && r < w) ? Dp[pidx(r, c)] : 0.0; };  // D^-1 (rows >= w: stale)
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) {
    if (16 * tj >= w) break;
    dbl4 R[4];
#pragma unroll
    for (int tk = 0; tk < 4; ++tk) {
      R[tk] = dbl4{0, 0, 0, 0};
#pragma unroll
      for (int k0 = 16 * tj; k0 < B2_NB; k0 += 4)
        R[tk] = __builtin_amdgcn_mfma_f64_16x16x4f64(Y(16 * tk + li, k0 + lk), X(k0 + lk, 16 * tj + li), R[tk], 0,
                                                      0, 0);
    }
#pragma unroll
    for (int ti = tj; ti < 4; ++ti) {
      dbl4 S = dbl4{0, 0, 0, 0};
#pragma unroll
      for (int k0 = 16 * ti; k0 < B2_NB; k0 += 4)
        S = __builtin_amdgcn_mfma_f64_16x16x4f64(X(k0 + lk, 16 * ti + li), R[k0 >> 4][(k0 & 15) >> 2], S, 0, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = 16 * ti + 4 * e + lk, c = 16 * tj + li;
        if (r < w && c <= r) {
          G[(int64_t)r * ldg + c] = (T)S[e];
          if (c < r) G[(int64_t)c * ldg + r] = (T)S[e];
        }
      }
    }
  }
}

// GP forward solve inside the factorisation, block s of problem p (Sec. 2's z = L^-1 y, block
// forward substitution): t_s = y_s - sum_{b<s} L_sb z_b has been accumulated in the w slot of the
// problem's vector by the panel solves of the earlier steps (b2_f2_kernel); z_s = D_s^-1 t_s with
// the inverse just formed in Xp, by the wave that factored the block.  At the problem's last block
// the wave also forms f = sum_i log L_ii + |z|^2 / 2 (per-lane partial sums over a fixed stride,
// then a fixed xor tree: reproducible), NaN when the factorisation failed.  Dp is free here (L has
// been stored); its first 64 entries stage t_s.
template <typename T>
__device__ void b2_gp_forward_block(const B2Args &a, int p, int n, int s, double *Dp_, const double *Xp_) {
  lds_double *Dp = lds_view(Dp_);
  const lds_double *Xp = lds_view(Xp_);
  const int lane = threadIdx.x & 63, i = a.order[p];
  const int j = s * B2_NB, w = min(B2_NB, n - j);
  double *zg = a.vec + p * a.vec_stride, *tg = zg + a.n_max;
  if (lane < w) Dp[lane] = s == 0 ? b2_y<T>(a, i, lane) : tg[j + lane];
  wave_sync();
  double z = 0.0;
  for (int c = 0; c < w; ++c)
    if (c <= lane) z = fma(Xp[pidx(lane, c)], Dp[c], z);
  if (lane < w) zg[j + lane] = z;
  if (j + w < n) return;
  // last block: f over the whole problem (earlier blocks' z were written by earlier launches)
  const T *L = b2_A<T>(a, i);
  const int64_t ldl = a.lda[i];
  double dv[B2_MAXBLK], zv[B2_MAXBLK];  // earlier blocks' entries, all loads in flight at once
#pragma unroll
  for (int u = 0; u < B2_MAXBLK; ++u) {
    const int ii = lane + B2_NB * u;
    dv[u] = ii < j ? L[(int64_t)ii * ldl + ii] : 1.0;
    zv[u] = ii < j ? zg[ii] : 0.0;
  }
  double part = lane < w ? log(L[(int64_t)(j + lane) * ldl + j + lane]) + 0.5 * z * z : 0.0;
#pragma unroll
  for (int u = 0; u < B2_MAXBLK; ++u) part += log(dv[u]) + 0.5 * zv[u] * zv[u];
  const double f = wave_sum(part);
  if (lane == 0) b2_set_f<T>(a, i, a.info[i] != 0 ? __builtin_nan("") : f);
  wave_sync();
}

// F1: POTF2 of block s of every problem with more than s blocks, and its inverse, one wave per
// problem.
template <typename T>
__global__ __launch_bounds__(256) void b2_potf2_kernel(B2Args a, int s) {
  __shared__ double lds[B2W_WAVES * B2W_LDS];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double *Dp = as_lds(lds + wave * B2W_LDS), *Xp = Dp + B2_PACKED;
  const int cnt = a.count[s];
  for (int p = blockIdx.x * B2W_WAVES + wave; p < cnt; p += gridDim.x * B2W_WAVES) {
    const int i = a.order[p], n = a.nv[p];
    const int j = s * B2_NB, w = min(B2_NB, n - j);
    T *Ad = b2_A<T>(a, i) + (int64_t)j * a.lda[i] + j;
    const int64_t lda = a.lda[i];
    wave_load_lower(Dp, Ad, lda, w);
    wave_sync();
    const int bad = wave_potf2_64(Dp, Xp, w);
    if (lane == 0 && bad >= 0 && a.info[i] == 0) a.info[i] = j + bad + 1;
    for (int r = 0; r < w; ++r)
      if (lane < w) Ad[(int64_t)r * lda + lane] = (T)(lane <= r ? Dp[pidx(r, lane)] : 0.0);
    double *X = a.dinv + p * a.dinv_stride + s * B2_BLK;
    for (int r = 0; r < B2_NB; ++r) X[r * B2_NB + lane] = (r < w && lane <= r) ? Xp[pidx(r, lane)] : 0.0;
    wave_sync();
    if (a.op == BATCH_GP) b2_gp_forward_block<T>(a, p, n, s, Dp, Xp);
  }
}

// Inverses of every diagonal block of L (REV, which is given L), one wave per block.
template <typename T>
__global__ __launch_bounds__(256) void b2_trinv_kernel(B2Args a) {
  __shared__ double lds[B2W_WAVES * B2W_LDS];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double *Dp = as_lds(lds + wave * B2W_LDS), *Xp = Dp + B2_PACKED;
  const int *pr = a.pref + (int64_t)B2_Q_BLK * (a.batch + 1);
  const int total = pr[a.batch];
  for (int it = blockIdx.x * B2W_WAVES + wave; it < total; it += gridDim.x * B2W_WAVES) {
    const int p = b2_find(pr, a.batch, it), b = it - pr[p];
    const int i = a.order[p], n = a.nv[p];
    const int j = b * B2_NB, w = min(B2_NB, n - j);
    int64_t ldl;
    const T *Li = b2_L<T>(a, i, ldl);
    wave_load_lower(Dp, Li + (int64_t)j * ldl + j, ldl, w);
    wave_sync();
    const int ib0 = min(INNER, w), ib1 = w - ib0;
    wave_trinv32x2(Dp, Xp, ib0, ib1);
    if (ib1 > 0) {
      wave_sync();
      const int nt = (ib1 + 15) / 16;
      dbl4 y[2][2];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
          y[ti][tj] = dbl4{0, 0, 0, 0};
          if (ti >= nt) continue;
          auto A = [&](int ii, int k) { const int r = 16 * ti + ii; return r < ib1 ? Dp[pidx(INNER + r, k)] : 0.0; };
          auto B = [&](int k, int jj) { const int c = 16 * tj + jj; return k >= c ? Xp[pidx(k, c)] : 0.0; };
          y[ti][tj] = tile_mma(y[ti][tj], A, B, INNER);
        }
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
          if (ti >= nt) continue;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int r = 16 * ti + tile_row(e), c = 16 * tj + tile_col();
            if (r < ib1) Xp[pidx(INNER + r, c)] = y[ti][tj][e];
          }
        }
      wave_sync();
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
          y[ti][tj] = dbl4{0, 0, 0, 0};
          if (ti >= nt) continue;
          auto A = [&](int ii, int k) {
            const int r = 16 * ti + ii;
            return (r < ib1 && k <= r) ? Xp[pidx(INNER + r, INNER + k)] : 0.0;
          };
          auto B = [&](int k, int jj) { return k < ib1 ? Xp[pidx(INNER + k, 16 * tj + jj)] : 0.0; };
          y[ti][tj] = tile_mma(y[ti][tj], A, B, min(ib1, 16 * ti + 16));
        }
      wave_sync();
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
          if (ti >= nt) continue;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int r = 16 * ti + tile_row(e), c = 16 * tj + tile_col();
            if (r < ib1) Xp[pidx(INNER + r, c)] = -y[ti][tj][e];
          }
        }
    }
    wave_sync();
    double *X = a.dinv + p * a.dinv_stride + b * B2_BLK;
    for (int r = 0; r < B2_NB; ++r) X[r * B2_NB + lane] = (r < w && lane <= r) ? Xp[pidx(r, lane)] : 0.0;
    wave_sync();
  }
}


// F2: rows below block s, C <- C D_s^-T, one 64-row tile per item (the tile spans all of the
// block's columns, so it is read before it is written); the mirrored positions above the
// diagonal are set to 0 (the factor's strict upper triangle).
template <typename T>
__global__ __launch_bounds__(256) void b2_f2_kernel(B2Args a, int s) {
  __shared__ double lds[T64_LDS];
  __shared__ double gpbuf[B2_NB + 4 * B2_NB];  // GP: z_s and the row partial sums
  const int *pr = a.pref + (int64_t)(B2_Q_F2 + s) * (a.batch + 1);
  const int total = pr[a.batch];
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int p = b2_find(pr, a.batch, it), ti = it - pr[p];
    const int i = a.order[p], n = a.nv[p];
    const int j = s * B2_NB, w = min(B2_NB, n - j), k = j + w;
    const int r0 = k + ti * B2_NB, R = min(B2_NB, n - r0);
    T *Ai = b2_A<T>(a, i);
    const int64_t lda = a.lda[i];
    const double *Di = a.dinv + p * a.dinv_stride + s * B2_BLK;
    dbl4 acc[2][2];
    t64_mma<true, true>(
        acc, [&](int r, int kk) { return (r < R && kk < w) ? Ai[(int64_t)(r0 + r) * lda + j + kk] : T(0); },
        [&](int kk, int c) { return (c < w && kk <= c) ? Di[c * B2_NB + kk] : 0.0; }, w, lds);
    t64_each(acc, [&](int r, int c, double v) {
      if (r < R && c < w) {
        Ai[(int64_t)(r0 + r) * lda + j + c] = (T)v;
        Ai[(int64_t)(j + c) * lda + r0 + r] = (T)0;
      }
    });
    if (a.op == BATCH_GP) {
      // GP forward solve: t_r -= L[r, block s] z_s for this tile's rows (t starts as y at step 0);
      // the tile and z_s go through LDS (free after the product), four threads per row take 16
      // columns each and the four partial sums are added in a fixed order
      __syncthreads();
      lds_double *Tl = lds_view(lds);
      lds_double *Z = lds_view(gpbuf), *Q = Z + B2_NB;
      const double *zg = a.vec + p * a.vec_stride;
      double *tg = (double *)zg + a.n_max;
      t64_each(acc, [&](int r, int c, double v) { Tl[r * (B2_NB + 1) + c] = v; });
      if ((int)threadIdx.x < B2_NB) Z[threadIdx.x] = (int)threadIdx.x < w ? zg[j + threadIdx.x] : 0.0;
      __syncthreads();
      {
        const int r = threadIdx.x >> 2, q = threadIdx.x & 3;
        double acc2 = 0.0;
#pragma unroll
        for (int c = 16 * q; c < 16 * q + 16; ++c) acc2 = fma(Tl[r * (B2_NB + 1) + c], Z[c], acc2);
        Q[threadIdx.x] = acc2;
      }
      __syncthreads();
      if ((int)threadIdx.x < R) {
        const int r = threadIdx.x;
        const double sum = (Q[4 * r] + Q[4 * r + 1]) + (Q[4 * r + 2] + Q[4 * r + 3]);
        tg[r0 + r] = (s == 0 ? b2_y<T>(a, i, r0 + r) : tg[r0 + r]) - sum;
      }
    }
    __syncthreads();
  }
}

// U: left-looking update of block column s, [D_s; C] -= [R; B] R^T over columns [0, 64 s), one
// 64-row tile of rows [64 s, n) per item (in place: it reads only columns left of the block).  The
// diagonal block's strict upper part is not needed (POTF2 reads the lower triangle).
template <typename T>
__global__ __launch_bounds__(256) void b2_up_kernel(B2Args a, int s) {
  __shared__ double lds[T64_LDS];
  const int *pr = a.pref + (int64_t)(B2_Q_UP + s) * (a.batch + 1);
  const int total = pr[a.batch];
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int p = b2_find(pr, a.batch, it), ti = it - pr[p];
    const int i = a.order[p], n = a.nv[p];
    const int j = s * B2_NB, w = min(B2_NB, n - j);
    const int r0 = j + ti * B2_NB, R = min(B2_NB, n - r0);
    T *Ai = b2_A<T>(a, i);
    const int64_t lda = a.lda[i];
    dbl4 acc[2][2];
    t64_mma<true, true>(
        acc, [&](int r, int kk) { return (r < R) ? Ai[(int64_t)(r0 + r) * lda + kk] : T(0); },
        [&](int kk, int c) { return (c < w) ? Ai[(int64_t)(j + c) * lda + kk] : T(0); }, j, lds);
    t64_each(acc, [&](int r, int c, double v) {
      if (r < R && c < w && (ti > 0 || c <= r)) {
        T *d = Ai + (int64_t)(r0 + r) * lda + j + c;
        *d = (T)((double)*d - v);
      }
    });
    __syncthreads();
  }
}


__device__ __forceinline__ bool b2_rev_skip(const B2Args &a, int i) {
  return (a.op == BATCH_GP || a.op == BATCH_FACTOR_REV) && a.info[i] != 0;
}

// GP mode: w_b = D_b^-T (z_b - L[k:, j:k]^T w[k:]) for block b = [j, k) by a whole workgroup
// (called by all its threads), once w[k:] is known -- the backward substitution of w = L^-T z, one
// block per reverse step.  Thread (h, r) = (wave, lane) walks rows k + h, k + h + 4, ... of column
// j + r (coalesced, sixteen loads in flight) and the four partial sums are added in a fixed order.
// tb and pt: B2_NB and 4 * B2_NB doubles of LDS.
template <typename T>
__device__ void b2_gp_w(const B2Args &a, int p, int n, int b, double *tb_, double *pt_) {
  lds_double *tb = lds_view(tb_), *pt = lds_view(pt_);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = a.order[p];
  const int j = b * B2_NB, k = min(n, j + B2_NB), w = k - j;
  const T *L = b2_A<T>(a, i);
  const int64_t ldl = a.lda[i];
  const double *zg = a.vec + p * a.vec_stride;
  double *wg = (double *)zg + a.n_max;
  double sv = 0.0;
  if (lane < w) {
    int ii = k + wave;
    for (; ii + 60 < n; ii += 64) {
      double lv[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) lv[u] = L[(int64_t)(ii + 4 * u) * ldl + j + lane];
#pragma unroll
      for (int u = 0; u < 16; ++u) sv = fma(lv[u], wg[ii + 4 * u], sv);
    }
    for (; ii < n; ii += 4) sv = fma(L[(int64_t)ii * ldl + j + lane], wg[ii], sv);
  }
  pt[wave * B2_NB + lane] = sv;
  __syncthreads();
  if (wave == 0 && lane < w)
    tb[lane] = zg[j + lane] - (((pt[lane] + pt[B2_NB + lane]) + pt[2 * B2_NB + lane]) + pt[3 * B2_NB + lane]);
  __syncthreads();
  const double *Di = a.dinv + p * a.dinv_stride + b * B2_BLK;
  double dv[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int q = lane + wave + 4 * u;
    dv[u] = (lane < w && q < w) ? Di[q * B2_NB + lane] : 0.0;
  }
  sv = 0.0;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int q = lane + wave + 4 * u;
    if (lane < w && q < w) sv = fma(dv[u], tb[q], sv);
  }
  pt[wave * B2_NB + lane] = sv;
  __syncthreads();
  if (wave == 0 && lane < w) wg[j + lane] = ((pt[lane] + pt[B2_NB + lane]) + pt[2 * B2_NB + lane]) + pt[3 * B2_NB + lane];
  __syncthreads();
}

// GP mode: entry (r, c), r >= c, of L-bar = diag(1 / L_ii) - tril(w z^T).
template <typename T>
__device__ __forceinline__ double b2_gp_lbar(const double *zg, const double *wg, const T *L, int64_t ldl,
                                             int r, int c) {
  const double v = -wg[r] * zg[c];
  return r == c ? 1.0 / (double)L[(int64_t)r * ldl + r] + v : v;
}

// R0: X = L-bar_C - 2 S_sym[k:, k:] L[k:, j:k] for the rows below block b = nblk - 1 - t, in place
// in the block column of G (one 64-row tile per item; it reads only columns >= k of G).
template <typename T>
__global__ __launch_bounds__(256) void b2_r0_kernel(B2Args a, int t) {
  __shared__ double lds[T64_LDS];
  const int *pr = a.pref + (int64_t)(B2_Q_RV + t) * (a.batch + 1);
  const int total = pr[a.batch];
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int p = b2_find(pr, a.batch, it), ti = it - pr[p];
    const int i = a.order[p], n = a.nv[p];
    if (b2_rev_skip(a, i)) continue;
    const int b = b2_nblk(n) - 1 - t;
    const int j = b * B2_NB, k = min(n, j + B2_NB), w = k - j, m = n - k;
    const int r0 = k + ti * B2_NB, R = min(B2_NB, n - r0);
    int64_t ldl, ldg;
    const T *Li = b2_L<T>(a, i, ldl);
    T *Gi = b2_G<T>(a, i, ldg);
    dbl4 acc[2][2];
    t64_mma<true, false>(
        acc, [&](int r, int kk) { return (r < R && kk < m) ? Gi[(int64_t)(r0 + r) * ldg + k + kk] : T(0); },
        [&](int kk, int c) { return (c < w && kk < m) ? Li[(int64_t)(k + kk) * ldl + j + c] : T(0); }, m, lds);
    const bool gp = a.op == BATCH_GP;
    const double *zg = a.vec + p * a.vec_stride, *wg = zg + a.n_max;
    t64_each(acc, [&](int r, int c, double v) {
      if (r < R && c < w) {
        T *d = Gi + (int64_t)(r0 + r) * ldg + j + c;
        const double lbar = gp ? -wg[r0 + r] * zg[j + c] : (double)*d;
        *d = (T)(lbar - 2.0 * v);
      }
    });
    __syncthreads();
  }
}

// R1: C-bar / 2 = X D_b^-1 / 2 for one 64-row tile (in place: the tile spans all of the block's
// columns, so it is read before it is written), mirrored to the upper triangle.
template <typename T>
__global__ __launch_bounds__(256) void b2_r1_kernel(B2Args a, int t) {
  __shared__ double lds[T64_LDS];
  const int *pr = a.pref + (int64_t)(B2_Q_RV + t) * (a.batch + 1);
  const int total = pr[a.batch];
  for (int it = blockIdx.x; it < total; it += gridDim.x) {
    const int p = b2_find(pr, a.batch, it), ti = it - pr[p];
    const int i = a.order[p], n = a.nv[p];
    if (b2_rev_skip(a, i)) continue;
    const int b = b2_nblk(n) - 1 - t;
    const int j = b * B2_NB, k = min(n, j + B2_NB), w = k - j;
    const int r0 = k + ti * B2_NB, R = min(B2_NB, n - r0);
    int64_t ldg;
    T *Gi = b2_G<T>(a, i, ldg);
    const double *Di = a.dinv + p * a.dinv_stride + b * B2_BLK;
    dbl4 acc[2][2];
    t64_mma<true, false>(
        acc, [&](int r, int kk) { return (r < R && kk < w) ? Gi[(int64_t)(r0 + r) * ldg + j + kk] : T(0); },
        [&](int kk, int c) { return (c < w && kk < w && kk >= c) ? Di[kk * B2_NB + c] : 0.0; }, w, lds);
    t64_each(acc, [&](int r, int c, double v) {
      if (r < R && c < w) {
        const double h = 0.5 * v;
        Gi[(int64_t)(r0 + r) * ldg + j + c] = (T)h;
        Gi[(int64_t)(j + c) * ldg + r0 + r] = (T)h;
      }
    });
    __syncthreads();
  }
}

// R2: D-bar = tril(L-bar_D) - tril(C-bar^T C) for block b = nblk - 1 - t, C-bar = 2 G[k:, j:k]
// (after R1) and C = L[k:, j:k], K = m; one workgroup per problem, written in place into the
// lower triangle of G's diagonal block.
template <typename T>
__global__ __launch_bounds__(256) void b2_r2_kernel(B2Args a, int t) {
  __shared__ double lds[T64_LDS];
  __shared__ double tb[B2_NB];
  __shared__ double pt[4 * B2_NB];
  const int cnt = a.count[t];
  const bool gp = a.op == BATCH_GP;
  for (int p = blockIdx.x; p < cnt; p += gridDim.x) {
    const int i = a.order[p], n = a.nv[p];
    if (b2_rev_skip(a, i)) continue;
    const int b = b2_nblk(n) - 1 - t;
    const int j = b * B2_NB, k = min(n, j + B2_NB), w = k - j, m = n - k;
    int64_t ldl, ldg;
    const T *Li = b2_L<T>(a, i, ldl);
    T *Gi = b2_G<T>(a, i, ldg);
    if (gp) b2_gp_w<T>(a, p, n, b, as_lds(tb), as_lds(pt));
    const double *zg = a.vec + p * a.vec_stride, *wg = zg + a.n_max;
    dbl4 acc[2][2];
    t64_mma<false, false>(
        acc, [&](int x, int kk) { return (x < w) ? Gi[(int64_t)(k + kk) * ldg + j + x] : T(0); },
        [&](int kk, int y) { return (y < w) ? Li[(int64_t)(k + kk) * ldl + j + y] : T(0); }, m, lds);
    t64_each(acc, [&](int x, int y, double v) {
      if (x < w && y <= x) {
        T *d = Gi + (int64_t)(j + x) * ldg + j + y;
        const double lbar = gp ? b2_gp_lbar<T>(zg, wg, Li, ldl, j + x, j + y) : (double)*d;
        *d = (T)(lbar - 2.0 * v);
      }
    });
    __syncthreads();
  }
}

// R3: the diagonal block's adjoint (eqn (symrev) on the block: D^-T Phi(D^T D-bar) D^-1, the
// symbolic form of Sec. 4.1's chol_unblocked_rev with its Phi halving) on the diagonal block
// b = nblk - 1 - t of every problem that has it, one wave per problem, from D = L's block and
// D-bar in the lower triangle of G's block; the symmetric gradient's block goes to both
// triangles of G.
template <typename T>
__global__ __launch_bounds__(256) void b2_r3_kernel(B2Args a, int t) {
  __shared__ double lds[B2W_WAVES * B2W_LDS];
  __shared__ double wv[B2W_WAVES * B2_NB];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double *Dp = as_lds(lds + wave * B2W_LDS), *Bp = Dp + B2_PACKED, *wl = as_lds(wv + wave * B2_NB);
  const int cnt = a.count[t];
  const bool gp0 = a.op == BATCH_GP && t == 0;
  for (int p = blockIdx.x * B2W_WAVES + wave; p < cnt; p += gridDim.x * B2W_WAVES) {
    const int i = a.order[p], n = a.nv[p];
    if (b2_rev_skip(a, i)) continue;
    const int b = b2_nblk(n) - 1 - t;
    const int j = b * B2_NB, w = min(B2_NB, n - j);
    int64_t ldl, ldg;
    const T *Ld = b2_L<T>(a, i, ldl) + (int64_t)j * ldl + j;
    T *Gd = b2_G<T>(a, i, ldg) + (int64_t)j * ldg + j;
    const double *Di = a.dinv + p * a.dinv_stride + b * B2_BLK;
    wave_load_lower(Dp, Ld, ldl, w);
    if (gp0) {
      // GP, last block: w_b = D_b^-T z_b (nothing below it), then D-bar = L-bar_D from w and z
      const double *zg = a.vec + p * a.vec_stride;
      double *wg = (double *)zg + a.n_max;
      double sv = 0.0;
      for (int q0 = 0; q0 < w; q0 += 16) {
        double dv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int q = q0 + u;
          dv[u] = (lane < w && q < w && q >= lane) ? Di[q * B2_NB + lane] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (q0 + u < w) sv = fma(dv[u], zg[j + q0 + u], sv);
      }
      if (lane < w) {
        wl[lane] = sv;
        wg[j + lane] = sv;
      }
      wave_sync();
      for (int r = 0; r < w; ++r)
        if (lane <= r) {
          const double v = -wl[r] * zg[j + lane];
          Bp[pidx(r, lane)] = lane == r ? 1.0 / (double)Ld[(int64_t)r * ldl + r] + v : v;
        }
    } else {
      wave_load_lower(Bp, Gd, ldg, w);
    }
    wave_sync();
    wave_diag_rev_sym64<T>(Dp, Bp, Di, w, Gd, ldg);
    wave_sync();
  }
}

// Paper's lower-triangular form T = Phi(S + S^T) from the symmetric gradient (strict lower doubled,
// strict upper 0), per problem.
template <typename T>
__global__ __launch_bounds__(256) void b2_form_kernel(B2Args a) {
  const int cnt = a.count[0];
  for (int p = blockIdx.x; p < cnt; p += gridDim.x) {
    const int i = a.order[p], n = a.nv[p];
    if (b2_rev_skip(a, i)) continue;
    int64_t ldg;
    T *Gi = b2_G<T>(a, i, ldg);
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int r = e / n, c = e - r * n;
      T *d = Gi + (int64_t)r * ldg + c;
      if (c > r) *d = (T)0;
      else if (c < r) *d = (T)(2.0 * (double)*d);
    }
  }
}

}  // namespace cg
