// Batched forward sweep: many independent problems (n <= 512) in ONE persistent launch.  Each
// 256-thread workgroup claims problems from a device work counter (largest first) and runs the
// blocked forward sweep of the single-matrix path (Sec. 4.2 chol_blocked_fwd, nb = 128) on each:
// the block inverses and diagonal blocks with the LDS routines of cg_diag.hpp, the block-column
// products as 128 x 128 MFMA tiles (gemm_tile), all inside the workgroup.  A problem with n <= 128
// is a single diagonal block and never leaves LDS between load and store.  The factor, reverse,
// factor + reverse and Gaussian-process calls take the step-synchronous path (cg_batched2.hpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cg_diag.hpp"
#include "cg_gemm.hpp"

namespace cg {

constexpr int BATCH_NB = 128;
constexpr int BATCH_NMAX = 512;
constexpr int BATCH_NBLK = BATCH_NMAX / BATCH_NB;
// LDS shared by all phases: two packed 128-blocks + a staged 32 x 32 inverse, or one tile product.
constexpr int BATCH_LDS = 2 * DIAG_PACKED + INNER * XLD;
static_assert(BATCH_LDS >= GEMM_LDS, "tile-product staging must fit in the shared LDS buffer");

enum BatchOp { BATCH_FACTOR = 0, BATCH_REV = 1, BATCH_FWD = 2, BATCH_GP = 3, BATCH_FACTOR_REV = 4 };

// Per-workgroup scratch of the persistent kernel in global memory (doubles).
constexpr int64_t SLOT_DINV = (int64_t)BATCH_NBLK * BATCH_NB * BATCH_NB;  // block inverses
constexpr int64_t SLOT_PANEL = (int64_t)BATCH_NMAX * BATCH_NB;            // one block column
constexpr int64_t SLOT_DOUBLES = SLOT_DINV + SLOT_PANEL;

// A batched call's arguments as the entry points fill them (every op; the step-synchronous path
// copies them into its own B2Args), then order .. stage_stride for the persistent kernel.
struct BatchArgs {
  int op;
  int batch;
  int sbar_form;
  const int64_t *n;
  double *const *A;         // factor (+rev), GP: Sigma -> L; rev: L-bar -> Sigma-bar; fwd: Sigma-dot -> L-dot
  const int64_t *lda;
  const double *const *L;   // rev / fwd
  const int64_t *ldl;
  const double *const *y;   // GP mode: right-hand sides
  double *const *G;         // GP mode: Sigma-bar output; factor+rev: L-bar -> Sigma-bar
  const int64_t *ldg;
  double *f;                // GP mode: losses
  int *info;                // factor / GP mode
  const int *order;         // persistent kernel: processing order (largest first)
  int *counter;             // work counter, zero at launch
  double *slots;            // gridDim.x * SLOT_DOUBLES
  int n_max;                // bound on every size (host value); larger problems are skipped
  int f32;                  // FP32 storage: the problems' arrays, vectors and losses are float
  double *stage;            // FP32 storage: gridDim.x * stage_stride doubles of FP64 staging
  int64_t stage_stride;
};

// Doubles of FP64 staging one workgroup of the persistent kernel needs for FP32 storage at sizes
// up to n_max: two n x n matrices (L and the tangent), rounded up to whole 256-byte lines.
__host__ __device__ constexpr int64_t stage_doubles(int64_t n_max) {
  return (2 * n_max * n_max + 31) / 32 * 32;
}

// Out-of-line entry points to the diagonal-block routines for the batched kernels (the single-
// matrix kernels inline them).
__device__ __noinline__ void nl_trinv_block(int w, const double *Ld, int64_t ldl, double *Dinv, int nb,
                                            double *Dp, double *Xp) {
  trinv_block(w, Ld, ldl, Dinv, nb, nb, 0, as_lds(Dp), as_lds(Xp));
}
__device__ __noinline__ void nl_diag_fwd_block(int w, const double *Ld, int64_t ldl, const double *Dinv, int nb,
                                               double *Ad, int64_t lda, double *Dp, double *Ap, double *Xi) {
  diag_fwd_block(w, Ld, ldl, Dinv, nb, Ad, lda, as_lds(Dp), as_lds(Ap), as_lds(Xi));
}
// C = alpha op(A) op(B) + beta Cin over all 128 x 128 output tiles, by the whole workgroup.
template <bool AT, bool BT>
__device__ __noinline__ void wg_gemm(int M, int N, int K, const double *A, int64_t lda, const double *B, int64_t ldb,
                        double alpha, const double *Cin, int64_t ldcin, double beta, double *C,
                        int64_t ldc, double *Cm, int64_t ldcm, double *lds) {
  GemmArgs p{};
  p.M = M; p.N = N; p.K = K;
  p.A = A; p.lda = lda; p.B = B; p.ldb = ldb;
  p.C = C; p.ldc = ldc; p.Cin = Cin; p.ldcin = ldcin; p.alpha = alpha; p.beta = beta;
  p.Cm = Cm; p.ldcm = ldcm; p.kchunk = K; p.split_stride = 0; p.lower_only = 0;
  for (int m0 = 0; m0 < M; m0 += GEMM_BM)
    for (int n0 = 0; n0 < N; n0 += GEMM_BN) gemm_tile<AT, BT>(p, m0, n0, 0, K, C, as_lds(lds));
}

// FP32 storage: the lower triangle of a float input is widened into a compact FP64 copy (leading
// dimension n, strict upper 0), the problem is computed exactly as in FP64, and each output is
// rounded to float once at the end.
__device__ void stage_in_lower(int n, const float *src, int64_t ld, double *dst) {
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int r = e / n, c = e - r * n;
    dst[e] = (c <= r) ? (double)src[(int64_t)r * ld + c] : 0.0;
  }
  __syncthreads();
}

__device__ void stage_out(int n, const double *src, float *dst, int64_t ld) {
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int r = e / n, c = e - r * n;
    dst[(int64_t)r * ld + c] = (float)src[e];
  }
  __syncthreads();
}

__device__ void wg_zero_upper(int n, double *A, int64_t lda) {
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int r = e / n, c = e - r * n;
    if (c > r) A[(int64_t)r * lda + c] = 0.0;
  }
  __syncthreads();
}

__device__ __noinline__ void batch_block_inverses(int n, const double *L, int64_t ldl, double *dinv, double *lds) {
  lds = as_lds(lds);
  const int nblk = (n + BATCH_NB - 1) / BATCH_NB;
  for (int b = 0; b < nblk; ++b) {
    const int j = b * BATCH_NB, w = min(BATCH_NB, n - j);
    nl_trinv_block(w, L + (int64_t)j * ldl + j, ldl, dinv + (int64_t)b * BATCH_NB * BATCH_NB, BATCH_NB, lds,
                lds + DIAG_PACKED);
  }
}

// Forward sweep (Sec. 4.2 chol_blocked_fwd) on one matrix; dinv must hold the block inverses of L.
__device__ __noinline__ void batch_fwd_one(int n, const double *L, int64_t ldl, double *A, int64_t lda, double *slot,
                              double *lds) {
  lds = as_lds(lds);
  double *dinv = slot, *panel = slot + SLOT_DINV;
  const int nblk = (n + BATCH_NB - 1) / BATCH_NB;
  for (int b = 0; b < nblk; ++b) {
    const int j = b * BATCH_NB, k = min(n, j + BATCH_NB), w = k - j, m = n - k;
    const double *Dinv = dinv + (int64_t)b * BATCH_NB * BATCH_NB;
    if (j > 0) {
      wg_gemm<false, true>(n - j, w, j, A + (int64_t)j * lda, lda, L + (int64_t)j * ldl, ldl, -1.0,
                           A + (int64_t)j * lda + j, lda, 1.0, A + (int64_t)j * lda + j, lda, nullptr, 0, lds);
      wg_gemm<false, true>(n - j, w, j, L + (int64_t)j * ldl, ldl, A + (int64_t)j * lda, lda, -1.0,
                           A + (int64_t)j * lda + j, lda, 1.0, A + (int64_t)j * lda + j, lda, nullptr, 0, lds);
    }
    nl_diag_fwd_block(w, L + (int64_t)j * ldl + j, ldl, Dinv, BATCH_NB, A + (int64_t)j * lda + j, lda, lds,
                   lds + DIAG_PACKED, lds + 2 * DIAG_PACKED);
    if (m > 0) {
      wg_gemm<false, true>(m, w, w, L + (int64_t)k * ldl + j, ldl, A + (int64_t)j * lda + j, lda, -1.0,
                           A + (int64_t)k * lda + j, lda, 1.0, panel, BATCH_NB, nullptr, 0, lds);
      wg_gemm<false, true>(m, w, w, panel, BATCH_NB, Dinv, BATCH_NB, 1.0, nullptr, 0, 0.0,
                           A + (int64_t)k * lda + j, lda, nullptr, 0, lds);
    }
  }
  wg_zero_upper(n, A, lda);
}

// Sum over a wave in a fixed xor-tree order (reproducible).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Counting sort of the problem indices by decreasing size (one workgroup): sizes outside
// [0, nmax] sort as size 0.
__global__ __launch_bounds__(256) void batch_order_kernel(int batch, const int64_t *n, int nmax, int *order,
                                                          int *counter) {
  __shared__ int cnt[BATCH_NMAX + 2];
  for (int i = threadIdx.x; i < BATCH_NMAX + 2; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < batch; i += blockDim.x) {
    int64_t v = n[i];
    const int key = (v < 0 || v > nmax) ? 0 : (int)v;
    atomicAdd(&cnt[BATCH_NMAX - key], 1);  // bin 0 holds the largest size
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < BATCH_NMAX + 1; ++i) {
      const int c = cnt[i];
      cnt[i] = run;
      run += c;
    }
    *counter = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < batch; i += blockDim.x) {
    int64_t v = n[i];
    const int key = (v < 0 || v > nmax) ? 0 : (int)v;
    order[atomicAdd(&cnt[BATCH_NMAX - key], 1)] = i;
  }
}

// The persistent kernel of chol_fwd_batched.  Every workgroup loops until the counter passes the
// batch, so all waves reach the same exit.  A problem with a size outside [0, n_max] or a leading
// dimension below its size is skipped; n_max <= BATCH_NMAX keeps every slot and staging access
// inside the workgroup's own region.
__global__ __launch_bounds__(DIAG_THREADS) void batch_fwd_kernel(BatchArgs a) {
  __shared__ double lds[BATCH_LDS];
  __shared__ int item;
  double *slot = a.slots + (int64_t)blockIdx.x * SLOT_DOUBLES;
  double *stage = a.f32 ? a.stage + (int64_t)blockIdx.x * a.stage_stride : nullptr;
  for (;;) {
    if (threadIdx.x == 0) item = atomicAdd(a.counter, 1);
    __syncthreads();
    const int it = item;
    __syncthreads();
    if (it >= a.batch) break;
    const int b = a.order[it];
    const int64_t n64 = a.n[b];
    if (n64 <= 0 || n64 > a.n_max || a.lda[b] < n64 || a.ldl[b] < n64) continue;
    const int n = (int)n64;
    // Working copies: the caller's arrays for FP64 storage, the staging area for FP32 storage.
    double *A = a.A[b];
    int64_t lda = a.lda[b];
    const double *L = a.L[b];
    int64_t ldl = a.ldl[b];
    if (a.f32) {
      double *const st2 = stage + (int64_t)n * n;
      stage_in_lower(n, reinterpret_cast<const float *>(a.A[b]), a.lda[b], stage);
      stage_in_lower(n, reinterpret_cast<const float *>(a.L[b]), a.ldl[b], st2);
      A = stage; lda = n;
      L = st2; ldl = n;
    }
    batch_block_inverses(n, L, ldl, slot, lds);
    batch_fwd_one(n, L, ldl, A, lda, slot, lds);
    if (a.f32) stage_out(n, stage, reinterpret_cast<float *>(a.A[b]), a.lda[b]);
  }
}

}  // namespace cg
