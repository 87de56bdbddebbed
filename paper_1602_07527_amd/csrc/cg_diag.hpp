// Diagonal-block kernels of the blocked sweeps (Sec. 4.2 of Murray 2016).  Each works on one
// w x w diagonal block (w <= 128) held entirely in LDS as packed lower triangles, one workgroup
// of 256 threads per block:
//   trinv_kernel    : D^-1 of every diagonal block of L (the TRSM steps then run as MFMA products)
//   diag_rev_kernel : D-bar <- chol_unblocked_rev(D, D-bar) (Sec. 4.1), organised as the blocked
//                     reverse sweep of Sec. 4.2 with 32-column inner blocks whose Level-2 adjoint
//                     runs in one wave64 out of registers (Phi's halving of the diagonal included).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cg {

constexpr int DIAG_MAX = 128;
constexpr int DIAG_PACKED = DIAG_MAX * (DIAG_MAX + 1) / 2;  // 8256 doubles
constexpr int DIAG_THREADS = 256;
constexpr int INNER = 32;

__device__ __forceinline__ int pidx(int r, int c) { return (r * (r + 1)) / 2 + c; }  // r >= c

// Uniform copy of lane `src`'s value (two 32-bit v_readlane).  src must be wave-uniform.
__device__ __forceinline__ double wave_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Packed-lower load of a w x w block (row-major source, leading dimension ld).
__device__ __forceinline__ void load_packed(double *dst, const double *src, int64_t ld, int w) {
  for (int e = threadIdx.x; e < w * w; e += blockDim.x) {
    const int r = e / w, c = e - r * w;
    if (c <= r) dst[pidx(r, c)] = src[(int64_t)r * ld + c];
  }
}

// ---------------------------------------------------------------------------------------------
// Inverse of each lower-triangular diagonal block: block b covers rows/cols [b*nb, min(n,(b+1)nb)).
// Row recurrence of D X = I:  X[i][c] = (delta_ic - sum_{c<=l<i} D[i][l] X[l][c]) / D[i][i].
// Output Dinv + b*nb*nb, row-major with leading dimension nb, zero above the diagonal and outside
// the w x w block.
__global__ __launch_bounds__(DIAG_THREADS) void trinv_kernel(int64_t n, int nb, const double *L,
                                                             int64_t ldl, double *Dinv) {
  __shared__ double Dp[DIAG_PACKED];
  __shared__ double Xp[DIAG_PACKED];
  const int64_t j = (int64_t)blockIdx.x * nb;
  const int w = (int)min<int64_t>(nb, n - j);
  load_packed(Dp, L + j * ldl + j, ldl, w);
  __syncthreads();
  for (int i = 0; i < w; ++i) {
    const double dii = Dp[pidx(i, i)];
    for (int c = threadIdx.x; c <= i; c += blockDim.x) {
      double s = (c == i) ? 1.0 : 0.0;
      for (int l = c; l < i; ++l) s -= Dp[pidx(i, l)] * Xp[pidx(l, c)];
      Xp[pidx(i, c)] = s / dii;
    }
    __syncthreads();
  }
  double *out = Dinv + (int64_t)blockIdx.x * nb * nb;
  for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
    const int r = e / nb, c = e - r * nb;
    out[e] = (r < w && c <= r) ? Xp[pidx(r, c)] : 0.0;
  }
}

// ---------------------------------------------------------------------------------------------
// Level-2 reverse sweep (Sec. 4.1 chol_unblocked_rev) on the ib x ib block at offset a of the
// packed matrices, by ONE wave: lane c < 32 owns column c of D and D-bar in registers.  For
// j = 31 .. 0:  d-bar <- d-bar - c^T c-bar / d;  [d-bar; c-bar] /= d;
// r-bar <- r-bar - [d-bar c-bar^T][r; B];  B-bar <- B-bar - c-bar r;  d-bar <- d-bar / 2.
// Lane j owns (d, c, d-bar, c-bar); the lanes l < j own the entries of r, B, r-bar, B-bar.
// A ragged block (ib < 32) is padded with D = I and D-bar = 0, which leaves the leading ib x ib
// result unchanged (the padded columns carry zero sensitivities and zero couplings), so every loop
// bound is a compile-time constant.
__device__ void level2_rev_wave(const double *Dp, double *Bp, int a, int ib) {
  const int c = threadIdx.x & 63;
  double Dc[INNER], Bc[INNER];
#pragma unroll
  for (int i = 0; i < INNER; ++i) {
    const bool ok = (c < ib) && (i < ib) && (i >= c);
    Dc[i] = ok ? Dp[pidx(a + i, a + c)] : (i == c ? 1.0 : 0.0);
    Bc[i] = ok ? Bp[pidx(a + i, a + c)] : 0.0;
  }
#pragma unroll
  for (int j = INNER - 1; j >= 0; --j) {
    double dot = 0.0;
#pragma unroll
    for (int i = j + 1; i < INNER; ++i) dot = fma(Dc[i], Bc[i], dot);
    const double inv_d = 1.0 / wave_bcast(Dc[j], j);
    const double dbar = wave_bcast((Bc[j] - dot * inv_d) * inv_d, j);
    const bool below = c < j, owner = c == j;
    const double r = Dc[j];  // D[j][c] on the lanes below
    double acc = dbar * r;
#pragma unroll
    for (int i = j + 1; i < INNER; ++i) {
      const double cbi = wave_bcast(Bc[i], j) * inv_d;
      acc = fma(cbi, Dc[i], acc);
      const double upd = fma(-cbi, r, Bc[i]);
      Bc[i] = owner ? cbi : (below ? upd : Bc[i]);
    }
    Bc[j] = owner ? 0.5 * dbar : (below ? Bc[j] - acc : Bc[j]);
  }
#pragma unroll
  for (int i = 0; i < INNER; ++i)
    if ((c < ib) && (i < ib) && (i >= c)) Bp[pidx(a + i, a + c)] = Bc[i];
}

// D-bar <- chol_unblocked_rev(D, D-bar) for one w x w diagonal block (w <= 128), run as the
// blocked reverse sweep of Sec. 4.2 over 32-column inner blocks [a, b) from the bottom-right:
//   C-bar <- C-bar D_i^-1;  B-bar <- B-bar - C-bar R;  D-bar_i <- D-bar_i - tril(C-bar^T C);
//   D-bar_i <- Level-2 adjoint (one wave);  R-bar <- R-bar - C-bar^T B - (D-bar_i + D-bar_i^T) R.
// In: L + (j, j) with ldl (only the block's lower triangle is read); Dbar (w x w, ld ldd, lower).
// Out: the block of the symmetric gradient, written to both triangles of A + (j, j):
//   A[r][c] = A[c][r] = T[r][c] / 2 (r > c),  A[r][r] = T[r][r],   T = final D-bar.
__global__ __launch_bounds__(DIAG_THREADS) void diag_rev_kernel(int w, const double *Ld, int64_t ldl,
                                                                const double *Dbar, int64_t ldd,
                                                                double *Aout, int64_t lda) {
  __shared__ double Dp[DIAG_PACKED];
  __shared__ double Bp[DIAG_PACKED];
  const int tid = threadIdx.x;
  load_packed(Dp, Ld, ldl, w);
  load_packed(Bp, Dbar, ldd, w);
  __syncthreads();

  for (int a = ((w - 1) / INNER) * INNER; a >= 0; a -= INNER) {
    const int b = min(w, a + INNER);
    const int ib = b - a;
    const int rest = w - b;  // rows below the inner block; when > 0, ib == INNER
    if (rest > 0) {
      // C-bar <- C-bar D_i^-1, one row per thread: x D_i = c-bar by back substitution in place.
      for (int r = b + tid; r < w; r += blockDim.x) {
        for (int q = INNER - 1; q >= 0; --q) {
          double s = Bp[pidx(r, a + q)];
          for (int p = q + 1; p < INNER; ++p) s = fma(-Bp[pidx(r, a + p)], Dp[pidx(a + p, a + q)], s);
          Bp[pidx(r, a + q)] = s / Dp[pidx(a + q, a + q)];
        }
      }
      __syncthreads();
      // B-bar <- B-bar - C-bar R   (rows [b, w), columns [0, a))
      for (int e = tid; e < rest * a; e += blockDim.x) {
        const int r = b + e / a, cc = e % a;
        double s = Bp[pidx(r, cc)];
#pragma unroll 8
        for (int q = 0; q < INNER; ++q) s = fma(-Bp[pidx(r, a + q)], Dp[pidx(a + q, cc)], s);
        Bp[pidx(r, cc)] = s;
      }
      // D-bar_i <- D-bar_i - tril(C-bar^T C)
      for (int e = tid; e < INNER * INNER; e += blockDim.x) {
        const int p = e / INNER, q = e % INNER;
        if (q <= p) {
          double s = 0.0;
          for (int r = b; r < w; ++r) s = fma(Bp[pidx(r, a + p)], Dp[pidx(r, a + q)], s);
          Bp[pidx(a + p, a + q)] -= s;
        }
      }
      __syncthreads();
    }
    if ((tid >> 6) == 0) level2_rev_wave(Dp, Bp, a, ib);
    __syncthreads();
    // R-bar <- R-bar - C-bar^T B - (D-bar_i + D-bar_i^T) R   (rows [a, b), columns [0, a))
    for (int e = tid; e < ib * a; e += blockDim.x) {
      const int p = e / a, cc = e % a;
      double s = 0.0;
      for (int r = b; r < w; ++r) s = fma(Bp[pidx(r, a + p)], Dp[pidx(r, cc)], s);
      for (int q = 0; q < ib; ++q) {
        const double dsym = (q < p) ? Bp[pidx(a + p, a + q)]
                          : (q > p) ? Bp[pidx(a + q, a + p)] : 2.0 * Bp[pidx(a + p, a + p)];
        s = fma(dsym, Dp[pidx(a + q, cc)], s);
      }
      Bp[pidx(a + p, cc)] -= s;
    }
    __syncthreads();
  }

  for (int e = tid; e < w * w; e += blockDim.x) {
    const int r = e / w, cc = e - r * w;
    const double v = (r > cc) ? 0.5 * Bp[pidx(r, cc)] : (r == cc ? Bp[pidx(r, r)] : 0.5 * Bp[pidx(cc, r)]);
    Aout[(int64_t)r * lda + cc] = v;
  }
}

// Level-2 forward sweep (Sec. 4.1 chol_unblocked_fwd) on the ib x ib block at offset a, by ONE
// wave: lane i < 32 owns row i of D and D-dot in registers.  For j = 0 .. 31 (eqns (dub1),(dub2)):
//   d-dot <- (d-dot/2 - r r-dot^T) / d;   c-dot <- (c-dot - B-dot r^T - B r-dot^T - c d-dot) / d.
// Lane j owns (r, d, r-dot, d-dot); lanes i > j own the rows of (B, c, B-dot, c-dot).  A ragged
// block is padded with D = I, D-dot = 0 (rows past ib never feed the leading rows).
__device__ void level2_fwd_wave(const double *Dp, double *Ap, int a, int ib) {
  const int i = threadIdx.x & 63;
  double Dr[INNER], Ar[INNER];
#pragma unroll
  for (int l = 0; l < INNER; ++l) {
    const bool ok = (i < ib) && (l <= i);
    Dr[l] = ok ? Dp[pidx(a + i, a + l)] : (l == i ? 1.0 : 0.0);
    Ar[l] = ok ? Ap[pidx(a + i, a + l)] : 0.0;
  }
#pragma unroll
  for (int j = 0; j < INNER; ++j) {
    double dot = 0.0;
#pragma unroll
    for (int l = 0; l < j; ++l) dot = fma(Dr[l], Ar[l], dot);
    const double d = wave_bcast(Dr[j], j);
    const double ddot = wave_bcast((0.5 * Ar[j] - dot) / Dr[j], j);
    double acc = Ar[j];
#pragma unroll
    for (int l = 0; l < j; ++l) {
      acc = fma(-Ar[l], wave_bcast(Dr[l], j), acc);
      acc = fma(-Dr[l], wave_bcast(Ar[l], j), acc);
    }
    acc = fma(-Dr[j], ddot, acc);
    Ar[j] = (i > j) ? acc / d : ((i == j) ? ddot : Ar[j]);
  }
#pragma unroll
  for (int l = 0; l < INNER; ++l)
    if ((i < ib) && (l <= i)) Ap[pidx(a + i, a + l)] = Ar[l];
}

// D-dot <- chol_unblocked_fwd(D, D-dot) for one w x w diagonal block (w <= 128), run as Sec. 4.2's
// blocked forward sweep over 32-column inner blocks [a, b), left to right:
//   D-dot_i <- D-dot_i - tril(R-dot R^T + R R-dot^T);  C-dot <- C-dot - B-dot R^T - B R-dot^T;
//   D-dot_i <- Level-2 forward (one wave);  C-dot <- (C-dot - C D-dot_i^T) D_i^-T.
// In: L + (j, j) (ldl), A + (j, j) holding tril of the updated Sigma-dot block.  Out: the block's
// L-dot in the lower triangle of A + (j, j); its strict upper triangle is set to 0.
__global__ __launch_bounds__(DIAG_THREADS) void diag_fwd_kernel(int w, const double *Ld, int64_t ldl,
                                                                double *Ad, int64_t lda) {
  __shared__ double Dp[DIAG_PACKED];
  __shared__ double Ap[DIAG_PACKED];
  const int tid = threadIdx.x;
  load_packed(Dp, Ld, ldl, w);
  load_packed(Ap, Ad, lda, w);
  __syncthreads();
  for (int a = 0; a < w; a += INNER) {
    const int b = min(w, a + INNER);
    const int ib = b - a;
    if (a > 0) {
      // D-dot_i -= tril(R-dot R^T + R R-dot^T)   (K = a)
      for (int e = tid; e < ib * ib; e += blockDim.x) {
        const int p = e / ib, q = e % ib;
        if (q <= p) {
          double s = 0.0;
          for (int l = 0; l < a; ++l)
            s = fma(Ap[pidx(a + p, l)], Dp[pidx(a + q, l)], fma(Dp[pidx(a + p, l)], Ap[pidx(a + q, l)], s));
          Ap[pidx(a + p, a + q)] -= s;
        }
      }
      // C-dot -= B-dot R^T + B R-dot^T   (rows [b, w), K = a)
      for (int e = tid; e < (w - b) * ib; e += blockDim.x) {
        const int r = b + e / ib, q = e % ib;
        double s = 0.0;
        for (int l = 0; l < a; ++l)
          s = fma(Ap[pidx(r, l)], Dp[pidx(a + q, l)], fma(Dp[pidx(r, l)], Ap[pidx(a + q, l)], s));
        Ap[pidx(r, a + q)] -= s;
      }
      __syncthreads();
    }
    if ((tid >> 6) == 0) level2_fwd_wave(Dp, Ap, a, ib);
    __syncthreads();
    // C-dot <- (C-dot - C D-dot_i^T) D_i^-T, one row per thread in place (ib == INNER whenever
    // b < w): first y = C-dot - C D-dot_i^T (right to left, so unread entries stay original),
    // then x D_i^T = y by forward substitution.
    for (int r = b + tid; r < w; r += blockDim.x) {
      for (int q = INNER - 1; q >= 0; --q) {
        double s = Ap[pidx(r, a + q)];
        for (int p = 0; p <= q; ++p) s = fma(-Dp[pidx(r, a + p)], Ap[pidx(a + q, a + p)], s);
        Ap[pidx(r, a + q)] = s;
      }
      for (int q = 0; q < INNER; ++q) {
        double s = Ap[pidx(r, a + q)];
        for (int p = 0; p < q; ++p) s = fma(-Ap[pidx(r, a + p)], Dp[pidx(a + q, a + p)], s);
        Ap[pidx(r, a + q)] = s / Dp[pidx(a + q, a + q)];
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < w * w; e += blockDim.x) {
    const int r = e / w, c = e - r * w;
    Ad[(int64_t)r * lda + c] = (c <= r) ? Ap[pidx(r, c)] : 0.0;
  }
}

// D <- chol_unblocked(D) (Sec. 4.1, DPOTF2) for one w x w diagonal block (w <= 128) in LDS,
// followed by the block's inverse for the panel solve.  Column j: d <- sqrt(d - r r^T) and
// c <- (c - B r^T) / d, applied right-looking.  The first non-positive (or NaN) pivot sets
// *info = col0 + j + 1 unless an earlier block already set it; the sweep then continues with
// NaN so that every kernel still exits normally.
// In/out: A + (j, j) (lower triangle in, factor out, strict upper set to 0).  Out: Dinv (w x w,
// ld nb, zero above the diagonal).
__global__ __launch_bounds__(DIAG_THREADS) void potf2_kernel(int w, double *Ad, int64_t lda,
                                                             double *Dinv, int nb, int *info,
                                                             int64_t col0) {
  __shared__ double Dp[DIAG_PACKED];
  __shared__ double Xp[DIAG_PACKED];
  __shared__ int bad;
  const int tid = threadIdx.x;
  load_packed(Dp, Ad, lda, w);
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    const double piv = Dp[pidx(j, j)];
    const double d = sqrt(piv);
    if (tid == 0) {
      if (!(piv > 0.0) && bad == 0) {
        bad = 1;
        if (*info == 0) *info = (int)(col0 + j + 1);
      }
    }
    for (int r = j + 1 + tid; r < w; r += blockDim.x) Dp[pidx(r, j)] /= d;
    __syncthreads();
    if (tid == 0) Dp[pidx(j, j)] = d;
    // trailing update of the lower triangle: D[r][c] -= D[r][j] D[c][j], j < c <= r
    const int t = w - j - 1;
    for (int e = tid; e < t * t; e += blockDim.x) {
      const int r = j + 1 + e / t, c = j + 1 + e % t;
      if (c <= r) Dp[pidx(r, c)] = fma(-Dp[pidx(r, j)], Dp[pidx(c, j)], Dp[pidx(r, c)]);
    }
    __syncthreads();
  }
  // inverse by the row recurrence of D X = I
  for (int i = 0; i < w; ++i) {
    const double dii = Dp[pidx(i, i)];
    for (int c = tid; c <= i; c += blockDim.x) {
      double s = (c == i) ? 1.0 : 0.0;
      for (int l = c; l < i; ++l) s -= Dp[pidx(i, l)] * Xp[pidx(l, c)];
      Xp[pidx(i, c)] = s / dii;
    }
    __syncthreads();
  }
  for (int e = tid; e < w * w; e += blockDim.x) {
    const int r = e / w, c = e - r * w;
    Ad[(int64_t)r * lda + c] = (c <= r) ? Dp[pidx(r, c)] : 0.0;
  }
  for (int e = tid; e < nb * nb; e += blockDim.x) {
    const int r = e / nb, c = e - r * nb;
    Dinv[e] = (r < w && c <= r) ? Xp[pidx(r, c)] : 0.0;
  }
}

// Zero the strict upper triangle of an n x n matrix.
__global__ __launch_bounds__(256) void zero_upper_kernel(int64_t n, double *A, int64_t lda) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n, c = e - r * n;
    if (c > r) A[r * lda + c] = 0.0;
  }
}

__global__ void set_int_kernel(int *p, int v) { *p = v; }

// Convert the symmetric gradient held in both triangles to the paper's lower-triangular form
// T = Phi(S + S^T) (eqn (symrevtril)): strict lower doubled, diagonal kept, strict upper zeroed.
__global__ __launch_bounds__(256) void sym_to_tril_kernel(int64_t n, double *A, int64_t lda) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n, c = e - r * n;
    double *p = A + r * lda + c;
    if (c > r) *p = 0.0;
    else if (c < r) *p = 2.0 * *p;
  }
}

}  // namespace cg
