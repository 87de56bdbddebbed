// Batched sweeps: many independent matrices (n <= 512) in ONE persistent launch.  Each 256-thread
// workgroup claims matrices from a device work counter (largest first) and runs the same blocked
// algorithms as the single-matrix path (Sec. 4.2, nb = 128) on each: the diagonal blocks with the
// LDS routines of cg_diag.hpp, the block-column products as 128 x 128 MFMA tiles (gemm_tile), all
// inside the workgroup.  A matrix with n <= 128 is a single diagonal block and never leaves LDS
// between load and store.  A fused mode runs a Gaussian-process style loss per matrix:
//   L = chol(Sigma);  z = L^-1 y;  w = L^-T z;  f = sum_i log L_ii + |z|^2 / 2;
//   L-bar = diag(1 / L_ii) - tril(w z^T);  Sigma-bar = chol_rev(L, L-bar)  (the x -> Sigma -> L -> f
// chain of Sec. 2 with the reverse sweep closing it).
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

// Per-workgroup scratch in global memory (doubles).
constexpr int64_t SLOT_DINV = (int64_t)BATCH_NBLK * BATCH_NB * BATCH_NB;  // block inverses
constexpr int64_t SLOT_PANEL = (int64_t)BATCH_NMAX * BATCH_NB;            // one block column
constexpr int64_t SLOT_DBLK = (int64_t)BATCH_NB * BATCH_NB;               // one diagonal block
constexpr int64_t SLOT_VEC = 2 * BATCH_NMAX;                               // z and w
constexpr int64_t SLOT_DOUBLES = SLOT_DINV + SLOT_PANEL + SLOT_DBLK + SLOT_VEC;

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
  const int *order;         // processing order (largest first)
  int *counter;             // work counter, zero at launch
  double *slots;            // gridDim.x * SLOT_DOUBLES
  int n_max;                // bound on every size (host value); larger problems are skipped
  int f32;                  // FP32 storage: matrices, vectors and losses are float
  double *stage;            // FP32 storage: gridDim.x * stage_stride doubles of FP64 staging
  int64_t stage_stride;
};

// Doubles of FP64 staging one workgroup needs for FP32 storage at sizes up to n_max: two n x n
// matrices, one vector and the loss, rounded up to whole 256-byte lines.
__host__ __device__ constexpr int64_t stage_doubles(int64_t n_max) {
  return (2 * n_max * n_max + n_max + 1 + 31) / 32 * 32;
}

// Out-of-line entry points to the diagonal-block routines for the batched kernels (the single-
// matrix kernels inline them).
__device__ __noinline__ void nl_trinv_block(int w, const double *Ld, int64_t ldl, double *Dinv, int nb,
                                            double *Dp, double *Xp) {
  trinv_block(w, Ld, ldl, Dinv, nb, nb, 0, as_lds(Dp), as_lds(Xp));
}
__device__ __noinline__ void nl_diag_rev_block(int w, const double *Ld, int64_t ldl, const double *Dbar,
                                               int64_t ldd, const double *Dinv, int nb, double *Aout,
                                               int64_t lda, double *Dp, double *Bp, double *Xi) {
  diag_rev_block(w, Ld, ldl, Dbar, ldd, Dinv, nb, Aout, lda, as_lds(Dp), as_lds(Bp), as_lds(Xi));
}
__device__ __noinline__ void nl_diag_fwd_block(int w, const double *Ld, int64_t ldl, const double *Dinv, int nb,
                                               double *Ad, int64_t lda, double *Dp, double *Ap, double *Xi) {
  diag_fwd_block(w, Ld, ldl, Dinv, nb, Ad, lda, as_lds(Dp), as_lds(Ap), as_lds(Xi));
}
__device__ __noinline__ void nl_potf2_block(int w, double *Ad, int64_t lda, double *Dinv, int nb, int *info,
                                            int64_t col0, double *Dp, double *Xp, int &bad) {
  potf2_block(w, Ad, lda, Dinv, nb, nb, 0, info, col0, as_lds(Dp), bad);
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

// Sec. 4.2 chol_blocked on one matrix (n <= 512).  Block inverses are left in the slot.
__device__ __noinline__ void batch_factor_one(int n, double *A, int64_t lda, int *info, double *slot, double *lds,
                                 int &bad) {
  lds = as_lds(lds);
  double *dinv = slot;
  const int nblk = (n + BATCH_NB - 1) / BATCH_NB;
  double *Dp = lds, *Xp = lds + DIAG_PACKED;
  for (int b = 0; b < nblk; ++b) {
    const int j = b * BATCH_NB, k = min(n, j + BATCH_NB), w = k - j, m = n - k;
    if (j > 0)
      wg_gemm<false, true>(n - j, w, j, A + (int64_t)j * lda, lda, A + (int64_t)j * lda, lda, -1.0,
                           A + (int64_t)j * lda + j, lda, 1.0, A + (int64_t)j * lda + j, lda, nullptr, 0, lds);
    nl_potf2_block(w, A + (int64_t)j * lda + j, lda, dinv + (int64_t)b * BATCH_NB * BATCH_NB, BATCH_NB, info,
                j, Dp, Xp, bad);
    if (m > 0)
      wg_gemm<false, true>(m, w, w, A + (int64_t)k * lda + j, lda, dinv + (int64_t)b * BATCH_NB * BATCH_NB,
                           BATCH_NB, 1.0, nullptr, 0, 0.0, A + (int64_t)k * lda + j, lda, nullptr, 0, lds);
  }
  wg_zero_upper(n, A, lda);
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

// Reverse sweep (Sec. 4.2 chol_blocked_rev in the left-looking order of the single-matrix path)
// on one matrix; dinv must hold the block inverses of L.
__device__ __noinline__ void batch_rev_one(int n, const double *L, int64_t ldl, double *A, int64_t lda, int form,
                              double *slot, double *lds) {
  lds = as_lds(lds);
  double *dinv = slot, *panel = slot + SLOT_DINV, *dblk = panel + SLOT_PANEL;
  const int nblk = (n + BATCH_NB - 1) / BATCH_NB;
  for (int b = nblk - 1; b >= 0; --b) {
    const int j = b * BATCH_NB, k = min(n, j + BATCH_NB), w = k - j, m = n - k;
    const double *Dinv = dinv + (int64_t)b * BATCH_NB * BATCH_NB;
    if (m > 0) {
      // X = L-bar_C - 2 S_sym[k:, k:] L[k:, j:k];  C-bar = X D^-1 (stored halved, both triangles);
      // D-bar = tril(L-bar_D) - tril(C-bar^T C)
      wg_gemm<false, false>(m, w, m, A + (int64_t)k * lda + k, lda, L + (int64_t)k * ldl + j, ldl, -2.0,
                            A + (int64_t)k * lda + j, lda, 1.0, panel, BATCH_NB, nullptr, 0, lds);
      wg_gemm<false, false>(m, w, w, panel, BATCH_NB, Dinv, BATCH_NB, 0.5, nullptr, 0, 0.0,
                            A + (int64_t)k * lda + j, lda, A + (int64_t)j * lda + k, lda, lds);
      wg_gemm<true, false>(w, w, m, A + (int64_t)k * lda + j, lda, L + (int64_t)k * ldl + j, ldl, -2.0,
                           A + (int64_t)j * lda + j, lda, 1.0, dblk, BATCH_NB, nullptr, 0, lds);
    } else {
      for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
        const int r = e / w, c = e - r * w;
        if (c <= r) dblk[r * BATCH_NB + c] = A[(int64_t)(j + r) * lda + j + c];
      }
      __syncthreads();
    }
    nl_diag_rev_block(w, L + (int64_t)j * ldl + j, ldl, dblk, BATCH_NB, Dinv, BATCH_NB, A + (int64_t)j * lda + j,
                   lda, lds, lds + DIAG_PACKED, lds + 2 * DIAG_PACKED);
  }
  if (form == 1) {  // lower-triangular form T = Phi(S + S^T)
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int r = e / n, c = e - r * n;
      double *p = A + (int64_t)r * lda + c;
      if (c > r) *p = 0.0;
      else if (c < r) *p = 2.0 * *p;
    }
    __syncthreads();
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

// Gaussian-process style loss on one matrix, after batch_factor_one has replaced Sigma by L and
// left the block inverses in the slot: z = L^-1 y and w = L^-T z by block substitution with the
// block inverses, f = sum log L_ii + |z|^2 / 2, and L-bar = diag(1/L_ii) - tril(w z^T) into G.
__device__ __forceinline__ double wave_sum(double v) {  // fixed xor-tree order: reproducible
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __noinline__ void batch_gp_loss_one(int n, const double *L, int64_t ldl, const double *y, double *G,
                                  int64_t ldg, double *f_out, double *slot, double *lds) {
  lds = as_lds(lds);
  const double *dinv = slot;
  double *z = slot + SLOT_DINV + SLOT_PANEL + SLOT_DBLK, *wv = z + BATCH_NMAX;
  double *t = lds;                          // BATCH_NB doubles of staging
  double *zl = lds + BATCH_NB;              // z, staged in LDS as it is produced
  double *wl = zl + BATCH_NMAX;             // w, likewise
  double *pt = wl + BATCH_NMAX;             // 2 x BATCH_NB partial sums
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int NW = DIAG_THREADS / 64, RU = 4;
  const int nblk = (n + BATCH_NB - 1) / BATCH_NB;
  // forward: z_b = D_b^-1 (y_b - L_{b,<b} z_<b).  Rows of L are contiguous, so a wave takes RU
  // rows at a time with its lanes along them (coalesced loads) and reduces each with wave_sum.
  for (int b = 0; b < nblk; ++b) {
    const int j = b * BATCH_NB, w = min(BATCH_NB, n - j);
    for (int r0 = wave * RU; r0 < w; r0 += NW * RU) {
      double s[RU];
#pragma unroll
      for (int u = 0; u < RU; ++u) s[u] = 0.0;
      for (int l = lane; l < j; l += 64) {
        const double zv = zl[l];
#pragma unroll
        for (int u = 0; u < RU; ++u)
          if (r0 + u < w) s[u] = fma(L[(int64_t)(j + r0 + u) * ldl + l], zv, s[u]);
      }
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const double tot = wave_sum(s[u]);
        if (lane == 0 && r0 + u < w) t[r0 + u] = y[j + r0 + u] - tot;
      }
    }
    __syncthreads();
    const double *Di = dinv + (int64_t)b * BATCH_NB * BATCH_NB;
    for (int r0 = wave * RU; r0 < w; r0 += NW * RU) {
      double s[RU];
#pragma unroll
      for (int u = 0; u < RU; ++u) s[u] = 0.0;
      for (int q = lane; q < w; q += 64) {
        const double tv = t[q];
#pragma unroll
        for (int u = 0; u < RU; ++u)
          if (q <= r0 + u && r0 + u < w) s[u] = fma(Di[(r0 + u) * BATCH_NB + q], tv, s[u]);
      }
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const double tot = wave_sum(s[u]);
        if (lane == 0 && r0 + u < w) {
          z[j + r0 + u] = tot;
          zl[j + r0 + u] = tot;
        }
      }
    }
    __syncthreads();
  }
  // backward: w_b = D_b^-T (z_b - L_{>b,b}^T w_>b).  Columns of L are strided, so thread (h, r)
  // walks rows i = k + h, k + h + 2, ... of column j + r (loads coalesced over r) and the two
  // halves are added in a fixed order.
  const int r = threadIdx.x % BATCH_NB, h = threadIdx.x / BATCH_NB;
  for (int b = nblk - 1; b >= 0; --b) {
    const int j = b * BATCH_NB, k = min(n, j + BATCH_NB), w = k - j;
    double s = 0.0;
    if (r < w) {
      int i = k + h;
      for (; i + 6 < n; i += 8) {
        const double l0 = L[(int64_t)i * ldl + j + r], l1 = L[(int64_t)(i + 2) * ldl + j + r];
        const double l2 = L[(int64_t)(i + 4) * ldl + j + r], l3 = L[(int64_t)(i + 6) * ldl + j + r];
        s = fma(l0, wl[i], s);
        s = fma(l1, wl[i + 2], s);
        s = fma(l2, wl[i + 4], s);
        s = fma(l3, wl[i + 6], s);
      }
      for (; i < n; i += 2) s = fma(L[(int64_t)i * ldl + j + r], wl[i], s);
    }
    pt[h * BATCH_NB + r] = s;
    __syncthreads();
    if (h == 0 && r < w) t[r] = zl[j + r] - (pt[r] + pt[BATCH_NB + r]);
    __syncthreads();
    const double *Di = dinv + (int64_t)b * BATCH_NB * BATCH_NB;
    s = 0.0;
    if (r < w)
      for (int q = r + h; q < w; q += 2) s = fma(Di[q * BATCH_NB + r], t[q], s);
    pt[h * BATCH_NB + r] = s;
    __syncthreads();
    if (h == 0 && r < w) {
      const double v = pt[r] + pt[BATCH_NB + r];
      wv[j + r] = v;
      wl[j + r] = v;
    }
    __syncthreads();
  }
  // f: per-thread partial sums over a fixed stride, then a fixed-order tree in LDS
  double part = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) part += log(L[(int64_t)i * ldl + i]) + 0.5 * zl[i] * zl[i];
  double *red = pt;
  red[threadIdx.x] = part;
  __syncthreads();
  for (int hh = blockDim.x / 2; hh > 0; hh >>= 1) {
    if ((int)threadIdx.x < hh) red[threadIdx.x] += red[threadIdx.x + hh];
    __syncthreads();
  }
  if (threadIdx.x == 0) *f_out = red[0];
  // L-bar = diag(1 / L_ii) - tril(w z^T), one wave per row
  for (int rr = wave; rr < n; rr += NW)
    for (int c = lane; c < n; c += 64) {
      double v = 0.0;
      if (c <= rr) v = -wl[rr] * zl[c] + ((rr == c) ? 1.0 / L[(int64_t)rr * ldl + rr] : 0.0);
      G[(int64_t)rr * ldg + c] = v;
    }
  __syncthreads();
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

// The persistent kernel.  Every workgroup loops until the counter passes the batch, so all waves
// reach the same exit.  A problem with a size outside [0, n_max] or a leading dimension below its
// size is skipped (its info, when there is one, is set to -1); n_max <= BATCH_NMAX keeps every
// slot and staging access inside the workgroup's own region.
template <int OP>
__global__ __launch_bounds__(DIAG_THREADS) void batch_kernel(BatchArgs a) {
  __shared__ double lds[BATCH_LDS];
  __shared__ int item;
  __shared__ int bad;
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
    const bool has_info = (OP == BATCH_FACTOR || OP == BATCH_GP || OP == BATCH_FACTOR_REV);
    if (n64 < 0 || n64 > a.n_max || a.lda[b] < n64 ||
        ((OP == BATCH_REV || OP == BATCH_FWD) && a.ldl[b] < n64) ||
        ((OP == BATCH_GP || OP == BATCH_FACTOR_REV) && a.ldg[b] < n64)) {
      if (has_info && threadIdx.x == 0) a.info[b] = -1;
      continue;
    }
    const int n = (int)n64;
    if (n == 0) {
      if (has_info && threadIdx.x == 0) a.info[b] = 0;
      if (OP == BATCH_GP && threadIdx.x == 0) {
        if (a.f32) reinterpret_cast<float *>(a.f)[b] = 0.0f;
        else a.f[b] = 0.0;
      }
      continue;
    }
    // Working copies: the caller's arrays for FP64 storage, the staging area for FP32 storage.
    double *const st2 = a.f32 ? stage + (int64_t)n * n : nullptr;      // second matrix (L or G)
    double *const sty = a.f32 ? stage + 2 * (int64_t)n * n : nullptr;  // y
    double *const stf = a.f32 ? sty + n : nullptr;                      // loss
    double *A = a.A[b];
    int64_t lda = a.lda[b];
    if (a.f32) {
      stage_in_lower(n, reinterpret_cast<const float *>(a.A[b]), a.lda[b], stage);
      A = stage;
      lda = n;
    }
    if (OP == BATCH_FACTOR || OP == BATCH_GP || OP == BATCH_FACTOR_REV) {
      if (threadIdx.x == 0) a.info[b] = 0;
      __syncthreads();
      batch_factor_one(n, A, lda, &a.info[b], slot, lds, bad);
      if (OP == BATCH_FACTOR_REV) {  // the factor's block inverses are still in the slot
        const int inf = a.info[b];
        __syncthreads();
        if (inf == 0) {
          double *G = a.G[b];
          int64_t ldg = a.ldg[b];
          if (a.f32) {
            stage_in_lower(n, reinterpret_cast<const float *>(a.G[b]), a.ldg[b], st2);
            G = st2;
            ldg = n;
          }
          batch_rev_one(n, A, lda, G, ldg, a.sbar_form, slot, lds);
          if (a.f32) stage_out(n, st2, reinterpret_cast<float *>(a.G[b]), a.ldg[b]);
        }
      }
      if (OP == BATCH_GP) {
        const int inf = a.info[b];
        __syncthreads();
        if (inf != 0) {  // not positive definite: no loss or gradient
          if (threadIdx.x == 0) {
            if (a.f32) reinterpret_cast<float *>(a.f)[b] = __builtin_nanf("");
            else a.f[b] = __builtin_nan("");
          }
        } else {
          const double *y = a.y[b];
          double *G = a.G[b];
          int64_t ldg = a.ldg[b];
          double *fo = &a.f[b];
          if (a.f32) {
            const float *yf = reinterpret_cast<const float *>(a.y[b]);
            for (int i = threadIdx.x; i < n; i += blockDim.x) sty[i] = (double)yf[i];
            __syncthreads();
            y = sty; G = st2; ldg = n; fo = stf;
          }
          batch_gp_loss_one(n, A, lda, y, G, ldg, fo, slot, lds);
          batch_rev_one(n, A, lda, G, ldg, 0, slot, lds);
          if (a.f32) {
            stage_out(n, st2, reinterpret_cast<float *>(a.G[b]), a.ldg[b]);
            if (threadIdx.x == 0) reinterpret_cast<float *>(a.f)[b] = (float)*stf;
          }
        }
      }
    } else {
      const double *L = a.L[b];
      int64_t ldl = a.ldl[b];
      if (a.f32) {
        stage_in_lower(n, reinterpret_cast<const float *>(a.L[b]), a.ldl[b], st2);
        L = st2;
        ldl = n;
      }
      batch_block_inverses(n, L, ldl, slot, lds);
      if (OP == BATCH_REV) batch_rev_one(n, L, ldl, A, lda, a.sbar_form, slot, lds);
      else batch_fwd_one(n, L, ldl, A, lda, slot, lds);
    }
    if (a.f32) stage_out(n, stage, reinterpret_cast<float *>(a.A[b]), a.lda[b]);
  }
}

}  // namespace cg
