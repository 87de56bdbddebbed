// Diagonal-block kernels of the blocked sweeps (Sec. 4.2 of Murray 2016).  Each works on one
// w x w diagonal block (w <= 128) held in LDS as packed lower triangles, one 256-thread workgroup
// (four wave64s) per block, organised exactly like the outer sweeps: 32-column inner blocks whose
// Level-2 step (Sec. 4.1) runs in ONE wave out of registers, with the Level-3 updates between them
// done as 16 x 16 v_mfma_f64_16x16x4_f64 tiles shared out over the four waves.
//   trinv_kernel    : D^-1 of every diagonal block of L (the panel solves are MFMA products)
//   diag_rev_kernel : D-bar <- chol_unblocked_rev(D, D-bar)     (Sec. 4.1, Phi halving included)
//   diag_fwd_kernel : D-dot <- chol_unblocked_fwd(D, D-dot)     (Sec. 4.1, eqns (dub1), (dub2))
//   potf2_kernel    : D <- chol_unblocked(D) (Sec. 4.1, DPOTF2) and D^-1
// and the symbolic diagonal-block forms (three tiled MFMA launches per block, one 16 x 16 output
// tile per workgroup) plus the tiled panel solves of both sweeps:
//   sym_rev_{p,q,s}_kernel : D-bar <- D^-T Phi(D^T D-bar) D^-1, symmetric part (eqn (symrev))
//   sym_fwd_{p,n,l}_kernel : D-dot <- D Phi(D^-1 D-dot D^-T)                  (eqn (symfwd))
//   rev_panel_solve_kernel : C-bar/2 = X D^-1 / 2 with its mirrored store
//   fwd_panel_solve_kernel : L-dot_C = C-dot D^-T + C (-Phi(Q))^T
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cg {

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int DIAG_MAX = 128;
constexpr int DIAG_PACKED = DIAG_MAX * (DIAG_MAX + 1) / 2;  // 8256 doubles
constexpr int DIAG_THREADS = 256;
constexpr int DIAG_WAVES = DIAG_THREADS / 64;
constexpr int INNER = 32;
constexpr int XLD = INNER + 1;  // leading dimension of a staged 32 x 32 inverse block

__device__ __forceinline__ int pidx(int r, int c) { return (r * (r + 1)) / 2 + c; }  // r >= c

// A pointer known to address LDS, re-typed so that the compiler sees it.  Out-of-line functions
// receive LDS arrays as plain pointers; without this their accesses compile to flat loads and
// stores (global-memory latency, counted with the vector-memory operations) instead of LDS ones.
__device__ __forceinline__ double *as_lds(double *p) {
  return (double *)(__attribute__((address_space(3))) double *)p;
}

// An LDS array seen through an LDS-typed pointer.  Indexing it compiles to ds_read / ds_write even
// inside a function the compiler keeps out of line, whose pointer parameters are generic (through
// those, LDS accesses become flat loads and stores, which wait on the vector-memory counter).
typedef __attribute__((address_space(3))) double lds_double;
__device__ __forceinline__ lds_double *lds_view(double *p) { return (lds_double *)p; }
__device__ __forceinline__ const lds_double *lds_view(const double *p) { return (const lds_double *)p; }

// Uniform copy of lane `src`'s value (two 32-bit v_readlane).  src must be wave-uniform.
__device__ __forceinline__ double wave_bcast(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Packed-lower load of a w x w block (w <= 128; row-major source, leading dimension ld).  The
// block is walked as a 128-wide grid so that row/column come from shifts, and each thread keeps
// 16 global loads in flight before it writes them to LDS.
__device__ __forceinline__ void load_packed(double *dst, const double *src, int64_t ld, int w) {
  constexpr int BATCH = 16;
  for (int e0 = 0; e0 < w * DIAG_MAX; e0 += BATCH * DIAG_THREADS) {
    double v[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int e = e0 + u * DIAG_THREADS + (int)threadIdx.x;
      const int r = e >> 7, c = e & (DIAG_MAX - 1);
      v[u] = (r < w && c <= r) ? src[(int64_t)r * ld + c] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int e = e0 + u * DIAG_THREADS + (int)threadIdx.x;
      const int r = e >> 7, c = e & (DIAG_MAX - 1);
      if (r < w && c <= r) dst[pidx(r, c)] = v[u];
    }
  }
}

typedef double dbl2d __attribute__((ext_vector_type(2)));

// 16-byte accesses to a row-major block need a 16-byte aligned base, an even leading dimension
// and an even width (so that a column pair never leaves the block).
__device__ __forceinline__ bool pairs_ok(const void *p, int64_t ld, int w) {
  return ((reinterpret_cast<uintptr_t>(p) & 15u) == 0) && ((ld & 1) == 0) && ((w & 1) == 0);
}

// Packed-lower load of two w x w blocks at once (src2 may be null), by column pairs with 16-byte
// loads when both sources allow it (16 loads of each in flight per thread); element loads
// otherwise.  A pair (c, c+1) with c <= r < w has c + 1 <= w - 1 for even w, so it stays inside
// the block even when c + 1 lies above the diagonal (that element is not stored).
__device__ __forceinline__ void load_packed2(double *dst, const double *src, int64_t ld, double *dst2,
                                             const double *src2, int64_t ld2, int w) {
  if (!pairs_ok(src, ld, w) || (src2 && !pairs_ok(src2, ld2, w))) {
    load_packed(dst, src, ld, w);
    if (src2) load_packed(dst2, src2, ld2, w);
    return;
  }
  constexpr int BATCH = 16;
  for (int e0 = 0; e0 < w * (DIAG_MAX / 2); e0 += BATCH * DIAG_THREADS) {
    dbl2d v[BATCH], v2[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int e = e0 + u * DIAG_THREADS + (int)threadIdx.x;
      const int r = e >> 6, c = (e & (DIAG_MAX / 2 - 1)) * 2;
      const bool ok = r < w && c <= r;
      v[u] = ok ? *(const dbl2d *)(src + (int64_t)r * ld + c) : dbl2d{0.0, 0.0};
      if (src2) v2[u] = ok ? *(const dbl2d *)(src2 + (int64_t)r * ld2 + c) : dbl2d{0.0, 0.0};
    }
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int e = e0 + u * DIAG_THREADS + (int)threadIdx.x;
      const int r = e >> 6, c = (e & (DIAG_MAX / 2 - 1)) * 2;
      if (r < w && c <= r) {
        dst[pidx(r, c)] = v[u][0];
        if (c + 1 <= r) dst[pidx(r, c + 1)] = v[u][1];
        if (src2) {
          dst2[pidx(r, c)] = v2[u][0];
          if (c + 1 <= r) dst2[pidx(r, c + 1)] = v2[u][1];
        }
      }
    }
  }
}

// dst[r * ld + c] = val(r, c) for r < rows, c < cols (cols <= 128), by column pairs with 16-byte
// stores when dst allows it, element stores otherwise.
template <typename F>
__device__ __forceinline__ void store_block(double *dst, int64_t ld, int rows, int cols, F val) {
  if (pairs_ok(dst, ld, cols)) {
#pragma unroll 4
    for (int e = threadIdx.x; e < rows * (DIAG_MAX / 2); e += blockDim.x) {
      const int r = e >> 6, c = (e & (DIAG_MAX / 2 - 1)) * 2;
      if (c < cols) *(dbl2d *)(dst + (int64_t)r * ld + c) = dbl2d{val(r, c), val(r, c + 1)};
    }
  } else {
#pragma unroll 4
    for (int e = threadIdx.x; e < rows * DIAG_MAX; e += blockDim.x) {
      const int r = e >> 7, c = e & (DIAG_MAX - 1);
      if (c < cols) dst[(int64_t)r * ld + c] = val(r, c);
    }
  }
}

// ---------------------------------------------------------------------------------------------
// One wave's 16 x 16 MFMA tile:  acc += sum_{k < K} A(i, k) B(k, j)  for i, j < 16.  A and B are
// accessors returning 0 outside their valid range; K need not be a multiple of 4.
// The accumulator layout is that of v_mfma_f64_16x16x4_f64: lane l, element e holds
// (row 4e + l/16, column l%16).
template <class FA, class FB>
__device__ __forceinline__ dbl4 tile_mma(dbl4 acc, FA A, FB B, int K) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, kq = lane >> 4;
  int k0 = 0;
  for (; k0 + 16 <= K; k0 += 16) {  // four k-steps per round: eight LDS reads in flight
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = A(i, k0 + 4 * u + kq);
      b[u] = B(k0 + 4 * u + kq, i);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
  }
  for (; k0 < K; k0 += 4) {
    const int k = k0 + kq;
    const double a = (k < K) ? A(i, k) : 0.0;
    const double b = (k < K) ? B(k, i) : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  return acc;
}

__device__ __forceinline__ int tile_row(int e) { return 4 * e + ((threadIdx.x & 63) >> 4); }
__device__ __forceinline__ int tile_col() { return threadIdx.x & 15; }

// ---------------------------------------------------------------------------------------------
// Per-wave 32 x 32 Level-2 cores.  A ragged inner block (ib < 32) is padded with the identity
// (and zero sensitivities), which leaves the leading ib x ib result unchanged, so all loop bounds
// are compile-time constants and every lane index is static.

// Sec. 4.1 chol_unblocked_rev on the block at offset a: lane c < 32 owns column c of D and D-bar.
// For j = 31 .. 0:  d-bar <- d-bar - c^T c-bar / d;  [d-bar; c-bar] /= d;
// r-bar <- r-bar - [d-bar c-bar^T][r; B];  B-bar <- B-bar - c-bar r;  d-bar <- d-bar / 2.
// Lane j owns (d, c, d-bar, c-bar); the lanes l < j own the entries of r, B, r-bar, B-bar and take
// lane j's column with v_readlane.  Lane j scales its column by 1/d before the broadcast, and a
// lane l > j holds D[j][l] = 0 (the zero-padded upper triangle), so every lane runs the same two
// FMAs per broadcast element with no per-element select.
__device__ void level2_rev_wave(const double *Dp_, double *Bp_, int a, int ib) {
  const lds_double *Dp = lds_view(Dp_);
  lds_double *Bp = lds_view(Bp_);
  const int c = threadIdx.x & 63;
  double Dc[INNER], Bc[INNER];
#pragma unroll
  for (int i = 0; i < INNER; ++i) {
    const bool ok = (c < ib) && (i < ib) && (i >= c);
    Dc[i] = ok ? Dp[pidx(a + i, a + c)] : (i == c ? 1.0 : 0.0);
    Bc[i] = ok ? Bp[pidx(a + i, a + c)] : 0.0;
  }
  double own = 1.0;
#pragma unroll
  for (int i = 0; i < INNER; ++i) own = (i == c) ? Dc[i] : own;
  const double inv_own = 1.0 / own;
#pragma unroll
  for (int j = INNER - 1; j >= 0; --j) {
    double p0 = 0.0, p1 = 0.0;
#pragma unroll
    for (int i = j + 1; i < INNER; ++i) {
      if ((i - j) & 1) p0 = fma(Dc[i], Bc[i], p0);
      else p1 = fma(Dc[i], Bc[i], p1);
    }
    const double inv_d = wave_bcast(inv_own, j);
    const double dbar = wave_bcast((Bc[j] - (p0 + p1) * inv_d) * inv_d, j);
    const bool owner = c == j;
    // c-bar <- c-bar / d on the owner (the other lanes multiply by exactly 1), so that it is
    // broadcast already scaled
    const double sc = owner ? inv_d : 1.0;
#pragma unroll
    for (int i = j + 1; i < INNER; ++i) Bc[i] *= sc;
    // D[j][c] on the lanes below; 0 on the owner (its column is final) and, from the zero-padded
    // upper triangle, on the lanes above
    const double r = owner ? 0.0 : Dc[j];
    double q0 = dbar * r, q1 = 0.0;
#pragma unroll
    for (int i = j + 1; i < INNER; ++i) {
      const double cbi = wave_bcast(Bc[i], j);
      if ((i - j) & 1) q1 = fma(cbi, Dc[i], q1);
      else q0 = fma(cbi, Dc[i], q0);
      Bc[i] = fma(-cbi, r, Bc[i]);
    }
    // lanes above change only their entry j, which lies above their diagonal and is never stored
    Bc[j] = owner ? 0.5 * dbar : Bc[j] - (q0 + q1);
  }
#pragma unroll
  for (int i = 0; i < INNER; ++i)
    if ((c < ib) && (i < ib) && (i >= c)) Bp[pidx(a + i, a + c)] = Bc[i];
}

// Sec. 4.1 chol_unblocked_fwd on the block at offset a: lane i < 32 owns row i of D and D-dot.
// For j = 0 .. 31:  d-dot <- (d-dot/2 - r r-dot^T) / d;
// c-dot <- (c-dot - B-dot r^T - B r-dot^T - c d-dot) / d.
__device__ void level2_fwd_wave(const double *Dp_, double *Ap_, int a, int ib) {
  const lds_double *Dp = lds_view(Dp_);
  lds_double *Ap = lds_view(Ap_);
  const int i = threadIdx.x & 63;
  double Dr[INNER], Ar[INNER];
#pragma unroll
  for (int l = 0; l < INNER; ++l) {
    const bool ok = (i < ib) && (l <= i);
    Dr[l] = ok ? Dp[pidx(a + i, a + l)] : (l == i ? 1.0 : 0.0);
    Ar[l] = ok ? Ap[pidx(a + i, a + l)] : 0.0;
  }
  // 1 / D[i][i], once per lane: the divisions of every column become multiplications
  double own = 1.0;
#pragma unroll
  for (int l = 0; l < INNER; ++l) own = (l == i) ? Dr[l] : own;
  const double inv_own = 1.0 / own;
#pragma unroll
  for (int j = 0; j < INNER; ++j) {
    double p0 = 0.0, p1 = 0.0;
#pragma unroll
    for (int l = 0; l < j; ++l) {
      if (l & 1) p1 = fma(Dr[l], Ar[l], p1);
      else p0 = fma(Dr[l], Ar[l], p0);
    }
    const double inv_d = wave_bcast(inv_own, j);
    const double ddot = wave_bcast((0.5 * Ar[j] - (p0 + p1)) * inv_own, j);
    double q0 = Ar[j], q1 = 0.0;
#pragma unroll
    for (int l = 0; l < j; ++l) {
      const double r = wave_bcast(Dr[l], j), rd = wave_bcast(Ar[l], j);
      if (l & 1) { q1 = fma(-Ar[l], r, q1); q1 = fma(-Dr[l], rd, q1); }
      else       { q0 = fma(-Ar[l], r, q0); q0 = fma(-Dr[l], rd, q0); }
    }
    const double num = fma(-Dr[j], ddot, q0 + q1);
    Ar[j] = (i > j) ? num * inv_d : ((i == j) ? ddot : Ar[j]);
  }
#pragma unroll
  for (int l = 0; l < INNER; ++l)
    if ((i < ib) && (l <= i)) Ap[pidx(a + i, a + l)] = Ar[l];
}

// Orders this wave's LDS writes before its later LDS reads (a wave's LDS accesses are processed in
// order; this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// d = sqrt(x) and rd = 1/sqrt(x) from v_rsq_f64 and two Goldschmidt steps (each about doubles the
// correct bits), with a last Newton correction of d; inputs below 2^-767 are scaled by 2^256 first
// so the steps stay in range.  A pivot column is then scaled by the multiplication with rd (as
// LAPACK's DPOTF2 scales by 1/L_jj).  x = 0, x < 0 and NaN give NaN in both.
__device__ __forceinline__ void sqrt_rsqrt(double x, double &d, double &rd) {
  const bool tiny = x < 0x1p-767;
  const double xs = tiny ? __builtin_ldexp(x, 256) : x;
  const double y = __builtin_amdgcn_rsq(xs);
  double g = xs * y, h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  g = fma(fma(-g, g, xs), h, g);
  d = tiny ? __builtin_ldexp(g, -128) : g;
  rd = tiny ? __builtin_ldexp(2.0 * h, 128) : 2.0 * h;
}

// Sec. 4.1 chol_unblocked (DPOTF2) on the 32 columns [a, a + ib) of the packed block, for the
// diagonal rows [a, a + ib) and up to 32 rows below them, by one wave: lane i < ib holds diagonal
// row a + i, lane 32 + t holds row rb + t (if rb + t < w).  Right-looking: at column j the pivot
// row's lane gives d = sqrt(D_jj), every lane scales its entry by 1/d, and each lane then
// subtracts its multiple of column j from its later entries, taking column j's entry of row k from
// lane k (v_readlane).  Rows below the diagonal block go through the same steps as the diagonal
// rows with i > j, so the panel below comes out solved (C <- C D^-T) in the same pass.  Several
// waves can share one diagonal block, each with its own rows below; every wave then holds the
// diagonal rows and only the one with diag_out writes them back.  WG: all threads of the
// workgroup call this (a barrier separates the loads from the stores); otherwise only the wave.
// Returns (uniformly) the first column < ib with a non-positive or NaN pivot, or -1.
template <bool WG>
__device__ int panel_core32(double *Dp_, int a, int ib, int w, int rb, bool diag_out) {
  lds_double *Dp = lds_view(Dp_);
  const int i = threadIdx.x & 63;
  const bool low = i >= INNER;
  const int row = low ? rb + (i - INNER) : a + i;
  const bool own = low ? row < w : i < ib;
  double Dr[INNER];
#pragma unroll
  for (int l = 0; l < INNER; ++l) Dr[l] = (own && l < ib && (low || l <= i)) ? Dp[pidx(row, a + l)] : 0.0;
  if (WG) __syncthreads();
  else wave_sync();
  int bad = -1;
#pragma unroll
  for (int j = 0; j < INNER; ++j) {
    const double piv = wave_bcast(Dr[j], j);
    if (bad < 0 && j < ib && !(piv > 0.0)) bad = j;
    double d, rd;
    sqrt_rsqrt(piv, d, rd);
    Dr[j] = (i == j) ? d : Dr[j] * rd;
#pragma unroll
    for (int k = j + 1; k < INNER; ++k) Dr[k] = fma(-Dr[j], wave_bcast(Dr[j], k), Dr[k]);
  }
#pragma unroll
  for (int l = 0; l < INNER; ++l)
    if (own && l < ib && (low || (diag_out && l <= i))) Dp[pidx(row, a + l)] = Dr[l];
  return bad;
}

// Inverse of the lower-triangular ib x ib block (ib <= 32) of Dp at offset a, by ONE wave (D X = I
// by forward substitution): lane c < ib builds column c of X, x_r = (delta_rc - sum_{l<r} D_rl x_l)
// / D_rr, reading row r of D with LDS loads whose address is the same in every lane (broadcasts);
// x_l = 0 for l < c comes out by itself.  Row r's loads wait (through an empty asm that takes
// x_{r-2}) until row r - 2 is done, which keeps the compiler from hoisting the whole triangle's
// loads into registers.  Writes the lower triangle of X into packed Xp at offset a.
__device__ void wave_trinv32(const double *Dp, double *Xp_, int a, int ib) {
  const lds_double *D = lds_view(Dp);
  lds_double *Xp = lds_view(Xp_);
  const int c = threadIdx.x & 63;
  const double inv_own = (c < ib) ? 1.0 / D[pidx(a + c, a + c)] : 0.0;
  double x[INNER];
#pragma unroll
  for (int r = 0; r < INNER; ++r) {
    x[r] = 0.0;
    if (r < ib) {
      int base = pidx(a + r, a);
      if (r >= 2) asm volatile("" : "+v"(base) : "v"(x[r - 2]));
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
      for (int l = 0; l < r; ++l) {
        const double dv = D[base + l];
        if ((l & 3) == 0) s0 = fma(dv, x[l], s0);
        else if ((l & 3) == 1) s1 = fma(dv, x[l], s1);
        else if ((l & 3) == 2) s2 = fma(dv, x[l], s2);
        else s3 = fma(dv, x[l], s3);
      }
      x[r] = (((r == c) ? 1.0 : 0.0) - ((s0 + s1) + (s2 + s3))) * wave_bcast(inv_own, r);
    }
  }
#pragma unroll
  for (int r = 0; r < INNER; ++r)
    if (c < ib && r < ib && r >= c) Xp[pidx(a + r, a + c)] = x[r];
}

// The inverses of the two 32 x 32 diagonal blocks of a packed 64-block in ONE pass of one wave:
// lanes 0..31 build the columns of the block at offset 0 (size ib0), lanes 32..63 those of the
// block at offset 32 (size ib1 >= 0), as wave_trinv32 does for one block (each half's LDS loads
// share one address per half).  Rows past a block's size compute values that are never stored.
__device__ void wave_trinv32x2(const double *Dp, double *Xp_, int ib0, int ib1) {
  const lds_double *D = lds_view(Dp);
  lds_double *Xp = lds_view(Xp_);
  const int lane = threadIdx.x & 63, h = lane >> 5, c = lane & 31, a = h * INNER;
  const int ib = h ? ib1 : ib0;
  const double inv_own = (c < ib) ? 1.0 / D[pidx(a + c, a + c)] : 0.0;
  double x[INNER];
#pragma unroll
  for (int r = 0; r < INNER; ++r) {
    int base = pidx(a + r, a);
    if (r >= 2) asm volatile("" : "+v"(base) : "v"(x[r - 2]));
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
    for (int l = 0; l < r; ++l) {
      const double dv = D[base + l];
      if ((l & 3) == 0) s0 = fma(dv, x[l], s0);
      else if ((l & 3) == 1) s1 = fma(dv, x[l], s1);
      else if ((l & 3) == 2) s2 = fma(dv, x[l], s2);
      else s3 = fma(dv, x[l], s3);
    }
    const double inv_r = h ? wave_bcast(inv_own, INNER + r) : wave_bcast(inv_own, r);
    x[r] = (((r == c) ? 1.0 : 0.0) - ((s0 + s1) + (s2 + s3))) * inv_r;
  }
#pragma unroll
  for (int r = 0; r < INNER; ++r)
    if (c < ib && r < ib && r >= c) Xp[pidx(a + r, a + c)] = x[r];
}

// X = D^-1 for the whole w x w block (packed; the workgroup cooperates).  The 32 x 32 diagonal
// blocks are inverted one per wave; block row p then follows from the rows above it:
//   X_pq = -X_pp (sum_{q <= l < p} D_pl X_lq)      (q < p),
// each product as MFMA tiles.  Ends with a barrier.
__device__ void block_inverse(const double *Dp_, double *Xp_, int w) {
  const lds_double *Dp = lds_view(Dp_);
  lds_double *Xp = lds_view(Xp_);
  const int wave = threadIdx.x >> 6;
  const int nI = (w + INNER - 1) / INNER;
  for (int p = wave; p < nI; p += DIAG_WAVES) {
    const int a = p * INNER;
    wave_trinv32(Dp_, Xp_, a, min(INNER, w - a));
  }
  __syncthreads();
  for (int p = 1; p < nI; ++p) {
    const int ap = p * INNER, bp = min(w, ap + INNER);
    // Y_pq = sum_l D_pl X_lq over columns [0, ap): 16 x 16 tiles of rows [ap, bp) x cols [0, ap)
    const int tr = (bp - ap + 15) / 16, tc = ap / 16;
    dbl4 acc[3];
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      const int t = wave + DIAG_WAVES * sl;
      if (t >= tr * tc) continue;
      const int r0 = ap + (t / tc) * 16, c0 = (t % tc) * 16;
      auto A = [&](int i, int k) { const int r = r0 + i, cc = c0 + k; return (r < w) ? Dp[pidx(r, cc)] : 0.0; };
      auto B = [&](int k, int j) { const int r = c0 + k, cc = c0 + j; return (r >= cc) ? Xp[pidx(r, cc)] : 0.0; };
      acc[sl] = tile_mma(dbl4{0, 0, 0, 0}, A, B, ap - c0);
    }
    __syncthreads();
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      const int t = wave + DIAG_WAVES * sl;
      if (t >= tr * tc) continue;
      const int r0 = ap + (t / tc) * 16, c0 = (t % tc) * 16;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = r0 + tile_row(e), cc = c0 + tile_col();
        if (r < w) Xp[pidx(r, cc)] = acc[sl][e];
      }
    }
    __syncthreads();
    // X_pq = -X_pp Y_pq   (Y_pq now held in the X_pq slots)
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      const int t = wave + DIAG_WAVES * sl;
      if (t >= tr * tc) continue;
      const int r0 = ap + (t / tc) * 16, c0 = (t % tc) * 16;
      auto A = [&](int i, int k) { const int r = r0 + i, cc = ap + k; return (r < w && r >= cc) ? Xp[pidx(r, cc)] : 0.0; };
      auto B = [&](int k, int j) { const int r = ap + k; return (r < w) ? Xp[pidx(r, c0 + j)] : 0.0; };
      acc[sl] = tile_mma(dbl4{0, 0, 0, 0}, A, B, bp - ap);
    }
    __syncthreads();
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      const int t = wave + DIAG_WAVES * sl;
      if (t >= tr * tc) continue;
      const int r0 = ap + (t / tc) * 16, c0 = (t % tc) * 16;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = r0 + tile_row(e), cc = c0 + tile_col();
        if (r < w) Xp[pidx(r, cc)] = -acc[sl][e];
      }
    }
    __syncthreads();
  }
}

// X = D^-1 for the whole w x w block IN PLACE (packed; the workgroup cooperates; whatever still
// needs D must have read it first).  The 32 x 32 diagonal blocks are inverted in place, one per
// wave (each wave reads its block whole before it writes); block column p of X then follows from
// the block columns right of it, right to left:
//   X_qp = -(sum_{p < r <= q} X_qr D_rp) X_pp      (q > p),
// the sum first written over D's own block column p below the diagonal (which it consumes) and
// then multiplied by X_pp, each product as MFMA tiles.  Half the LDS of block_inverse, which lets
// the POTF2 kernel share a compute unit with a contraction workgroup.  Ends with a barrier.
__device__ void block_inverse_inplace(double *Dp_, int w) {
  lds_double *Dp = lds_view(Dp_);
  const int wave = threadIdx.x >> 6;
  const int nI = (w + INNER - 1) / INNER;
  for (int p = wave; p < nI; p += DIAG_WAVES) {
    const int a = p * INNER;
    wave_trinv32(Dp_, Dp_, a, min(INNER, w - a));
  }
  __syncthreads();
  for (int p = nI - 2; p >= 0; --p) {
    const int ap = p * INNER, bp = ap + INNER;  // block p is full: only the last block can be short
    const int tr = (w - bp + 15) / 16, tc = INNER / 16;
    dbl4 acc[3];
    // Y = X[bp:w, bp:w] D[bp:w, ap:bp]   (tiles of rows [bp, w) x columns [ap, bp))
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      const int t = wave + DIAG_WAVES * sl;
      if (t >= tr * tc) continue;
      const int r0 = bp + (t / tc) * 16, c0 = ap + (t % tc) * 16;
      auto A = [&](int i, int k) { const int r = r0 + i, c = bp + k; return (r < w && c <= r) ? Dp[pidx(r, c)] : 0.0; };
      auto B = [&](int k, int j) { return Dp[pidx(bp + k, c0 + j)]; };
      acc[sl] = tile_mma(dbl4{0, 0, 0, 0}, A, B, min(w, r0 + 16) - bp);
    }
    __syncthreads();
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      const int t = wave + DIAG_WAVES * sl;
      if (t >= tr * tc) continue;
      const int r0 = bp + (t / tc) * 16, c0 = ap + (t % tc) * 16;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = r0 + tile_row(e);
        if (r < w) Dp[pidx(r, c0 + tile_col())] = acc[sl][e];
      }
    }
    __syncthreads();
    // X_qp = -Y X_pp
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      const int t = wave + DIAG_WAVES * sl;
      if (t >= tr * tc) continue;
      const int r0 = bp + (t / tc) * 16, c0 = ap + (t % tc) * 16;
      auto A = [&](int i, int k) { const int r = r0 + i; return (r < w) ? Dp[pidx(r, ap + k)] : 0.0; };
      auto B = [&](int k, int j) { const int c = c0 + j; return (ap + k >= c) ? Dp[pidx(ap + k, c)] : 0.0; };
      acc[sl] = tile_mma(dbl4{0, 0, 0, 0}, A, B, INNER);
    }
    __syncthreads();
#pragma unroll
    for (int sl = 0; sl < 3; ++sl) {
      const int t = wave + DIAG_WAVES * sl;
      if (t >= tr * tc) continue;
      const int r0 = bp + (t / tc) * 16, c0 = ap + (t % tc) * 16;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int r = r0 + tile_row(e);
        if (r < w) Dp[pidx(r, c0 + tile_col())] = -acc[sl][e];
      }
    }
    __syncthreads();
  }
}

// Write the packed lower triangle of a w x w block into the ext x ext region at dst (row-major,
// leading dimension ld, ext <= 128), zero elsewhere in the region, and zero `right` (<= 128) more
// columns to the right of the region in its rows (the part of a wider block's inverse above the
// next diagonal half).
__device__ __forceinline__ void store_lower_region(double *dst, int64_t ld, int ext, const double *Xp, int w,
                                                   int right) {
  store_block(dst, ld, ext, ext, [&](int r, int c) { return (r < w && c <= r) ? Xp[pidx(r, c)] : 0.0; });
  if (right > 0) store_block(dst + ext, ld, ext, right, [&](int, int) { return 0.0; });
}

// ---------------------------------------------------------------------------------------------
// Inverse of one lower-triangular w x w block (w <= 128) of L (ldl) into the ext x ext region at
// Dinv (leading dimension ld; see store_lower_region).
__device__ __forceinline__ void trinv_block(int w, const double *Ld, int64_t ldl, double *Dinv, int64_t ld,
                                            int ext, int right, double *Dp, double *Xp) {
  load_packed2(Dp, Ld, ldl, nullptr, nullptr, 0, w);
  __syncthreads();
  block_inverse(Dp, Xp, w);
  store_lower_region(Dinv, ld, ext, Xp, w, right);
  __syncthreads();
}

// Inverse of each lower-triangular diagonal block: block b covers rows/cols [b*nb, min(n,(b+1)nb)).
// Output Dinv + b*nb*nb, row-major with leading dimension nb, zero above the diagonal.
//   nb <= 128: workgroup b inverts block b whole (zero outside its w x w part as well).
//   128 < nb <= 256: workgroups 2b and 2b+1 invert the two halves of block b (widths 128 and
//   w - 128) into their diagonal positions; the first also zeroes the part above the second
//   half.  The part below the first half, -X11 L10 X00, comes from inv_offdiag_kernel.
__global__ __launch_bounds__(DIAG_THREADS) void trinv_kernel(int64_t n, int nb, const double *L,
                                                             int64_t ldl, double *Dinv) {
  __shared__ double Dp[DIAG_PACKED];
  __shared__ double Xp[DIAG_PACKED];
  if (nb <= DIAG_MAX) {
    const int64_t j = (int64_t)blockIdx.x * nb;
    const int w = (int)min<int64_t>(nb, n - j);
    trinv_block(w, L + j * ldl + j, ldl, Dinv + (int64_t)blockIdx.x * nb * nb, nb, nb, 0, Dp, Xp);
    return;
  }
  const int64_t b = blockIdx.x >> 1;
  const int h = blockIdx.x & 1;
  const int wb = (int)min<int64_t>(nb, n - b * nb);   // width of block b
  const int w = min(DIAG_MAX, wb - h * DIAG_MAX);      // width of this half
  if (w <= 0) return;                                   // workgroup-uniform
  const int64_t j = b * nb + h * DIAG_MAX;
  double *dst = Dinv + b * nb * nb + (int64_t)h * DIAG_MAX * nb + h * DIAG_MAX;
  trinv_block(w, L + j * ldl + j, ldl, dst, nb, w, h == 0 ? wb - w : 0, Dp, Xp);
}

// Stage the 32 x 32 diagonal sub-block [a, a+32)^2 of a block inverse (row-major, ld nb) in LDS.
__device__ __forceinline__ void stage_inverse32(double *Xi, const double *Dinv, int nb, int a) {
  for (int e = threadIdx.x; e < INNER * INNER; e += blockDim.x) {
    const int r = e / INNER, c = e % INNER;
    Xi[r * XLD + c] = Dinv[(int64_t)(a + r) * nb + a + c];
  }
}

// ---------------------------------------------------------------------------------------------
// D-bar <- chol_unblocked_rev(D, D-bar) for one w x w diagonal block (w <= 128), run as the
// blocked reverse sweep of Sec. 4.2 over 32-column inner blocks [a, b) from the bottom-right:
//   C-bar <- C-bar D_i^-1;  B-bar <- B-bar - C-bar R;  D-bar_i <- D-bar_i - tril(C-bar^T C);
//   D-bar_i <- Level-2 adjoint (one wave);  R-bar <- R-bar - C-bar^T B - (D-bar_i + D-bar_i^T) R.
// In: L + (j, j) with ldl (only the block's lower triangle is read); Dbar (w x w, ld ldd, lower);
// Dinv: this block's inverse (ld nb).
// Out: the block of the symmetric gradient, written to both triangles of A + (j, j):
//   A[r][c] = A[c][r] = T[r][c] / 2 (r > c),  A[r][r] = T[r][r],   T = final D-bar.
// The sweep itself, on D (packed in Dp) and D-bar (packed in Bp) already in LDS.
__device__ __forceinline__ void diag_rev_core(int w, const double *Dinv, int nb, double *Aout, int64_t lda,
                                              double *Dp, double *Bp, double *Xi) {
  const int tid = threadIdx.x, wave = tid >> 6;

  for (int a = ((w - 1) / INNER) * INNER; a >= 0; a -= INNER) {
    const int b = min(w, a + INNER);
    const int ib = b - a;
    const int rest = w - b;  // rows below the inner block; when > 0, ib == INNER
    const int trr = (rest + 15) / 16;
    if (rest > 0) {
      stage_inverse32(Xi, Dinv, nb, a);
      __syncthreads();
      // C-bar <- C-bar D_i^-1  (rows [b, w) x cols [a, b), K = 32)
      dbl4 acc[3];
#pragma unroll
      for (int sl = 0; sl < 3; ++sl) {
        const int t = wave + DIAG_WAVES * sl;
        if (t >= trr * 2) continue;
        const int r0 = b + (t >> 1) * 16, c0 = (t & 1) * 16;
        auto A = [&](int i, int k) { const int r = r0 + i; return (r < w) ? Bp[pidx(r, a + k)] : 0.0; };
        auto B = [&](int k, int j) { return Xi[k * XLD + c0 + j]; };
        acc[sl] = tile_mma(dbl4{0, 0, 0, 0}, A, B, INNER);
      }
      __syncthreads();
#pragma unroll
      for (int sl = 0; sl < 3; ++sl) {
        const int t = wave + DIAG_WAVES * sl;
        if (t >= trr * 2) continue;
        const int r0 = b + (t >> 1) * 16, c0 = (t & 1) * 16;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = r0 + tile_row(e);
          if (r < w) Bp[pidx(r, a + c0 + tile_col())] = acc[sl][e];
        }
      }
      __syncthreads();
      // B-bar -= C-bar R  (rows [b, w) x cols [0, a), K = 32)   and
      // D-bar_i -= tril(C-bar^T C)  (the three lower 16 x 16 tiles of the 32 x 32 block, K = rest)
      const int tca = a / 16;
      const int n2 = trr * tca;
      for (int t = wave; t < n2 + 3; t += DIAG_WAVES) {
        if (t < n2) {
          const int r0 = b + (t / tca) * 16, c0 = (t % tca) * 16;
          auto A = [&](int i, int k) { const int r = r0 + i; return (r < w) ? Bp[pidx(r, a + k)] : 0.0; };
          auto B = [&](int k, int j) { return Dp[pidx(a + k, c0 + j)]; };
          const dbl4 s = tile_mma(dbl4{0, 0, 0, 0}, A, B, INNER);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int r = r0 + tile_row(e);
            if (r < w) Bp[pidx(r, c0 + tile_col())] -= s[e];
          }
        } else {
          const int u = t - n2;  // 0: (0,0), 1: (1,0), 2: (1,1)
          const int r0 = (u == 0) ? 0 : 16, c0 = (u == 2) ? 16 : 0;
          auto A = [&](int i, int k) { return Bp[pidx(b + k, a + r0 + i)]; };
          auto B = [&](int k, int j) { return Dp[pidx(b + k, a + c0 + j)]; };
          const dbl4 s = tile_mma(dbl4{0, 0, 0, 0}, A, B, rest);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int r = r0 + tile_row(e), cc = c0 + tile_col();
            if (cc <= r) Bp[pidx(a + r, a + cc)] -= s[e];
          }
        }
      }
      __syncthreads();
    }
    if (wave == 0) level2_rev_wave(Dp, Bp, a, ib);
    __syncthreads();
    if (a > 0) {
      // R-bar -= C-bar^T B + (D-bar_i + D-bar_i^T) R   (rows [a, b) x cols [0, a))
      const int tri = (ib + 15) / 16, tca = a / 16;
      for (int t = wave; t < tri * tca; t += DIAG_WAVES) {
        const int r0 = (t / tca) * 16, c0 = (t % tca) * 16;
        dbl4 s = dbl4{0, 0, 0, 0};
        if (rest > 0) {
          auto A1 = [&](int i, int k) { return (r0 + i < ib) ? Bp[pidx(b + k, a + r0 + i)] : 0.0; };
          auto B1 = [&](int k, int j) { return Dp[pidx(b + k, c0 + j)]; };
          s = tile_mma(s, A1, B1, rest);
        }
        auto A2 = [&](int i, int k) {
          const int m = r0 + i;
          if (m >= ib || k >= ib) return 0.0;
          return (k < m) ? Bp[pidx(a + m, a + k)]
                         : (k > m) ? Bp[pidx(a + k, a + m)] : 2.0 * Bp[pidx(a + m, a + m)];
        };
        auto B2 = [&](int k, int j) { return (k < ib) ? Dp[pidx(a + k, c0 + j)] : 0.0; };
        s = tile_mma(s, A2, B2, ib);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int m = r0 + tile_row(e);
          if (m < ib) Bp[pidx(a + m, c0 + tile_col())] -= s[e];
        }
      }
      __syncthreads();
    }
  }

  store_block(Aout, lda, w, w, [&](int r, int cc) {
    return (r > cc) ? 0.5 * Bp[pidx(r, cc)] : (r == cc ? Bp[pidx(r, r)] : 0.5 * Bp[pidx(cc, r)]);
  });
  __syncthreads();
}

__device__ __forceinline__ void diag_rev_block(int w, const double *Ld, int64_t ldl, const double *Dbar, int64_t ldd,
                               const double *Dinv, int nb, double *Aout, int64_t lda, double *Dp,
                               double *Bp, double *Xi) {
  load_packed2(Dp, Ld, ldl, Bp, Dbar, ldd, w);
  __syncthreads();
  diag_rev_core(w, Dinv, nb, Aout, lda, Dp, Bp, Xi);
}

__global__ __launch_bounds__(DIAG_THREADS) void diag_rev_kernel(int w, const double *Ld, int64_t ldl,
                                                                const double *Dbar, int64_t ldd,
                                                                const double *Dinv, int nb,
                                                                double *Aout, int64_t lda) {
  __shared__ double Dp[DIAG_PACKED];
  __shared__ double Bp[DIAG_PACKED];
  __shared__ double Xi[INNER * XLD];
  diag_rev_block(w, Ld, ldl, Dbar, ldd, Dinv, nb, Aout, lda, Dp, Bp, Xi);
}

// ---------------------------------------------------------------------------------------------
// D-dot <- chol_unblocked_fwd(D, D-dot) for one w x w diagonal block (w <= 128), run as Sec. 4.2's
// blocked forward sweep over 32-column inner blocks [a, b), left to right:
//   [D-dot_i; C-dot] <- [D-dot_i; C-dot] - [R-dot; B-dot] R^T - [R; B] R-dot^T;
//   D-dot_i <- Level-2 forward (one wave);  C-dot <- (C-dot - C D-dot_i^T) D_i^-T.
// In: L + (j, j) (ldl), A + (j, j) holding tril of the updated Sigma-dot block, Dinv: this
// block's inverse (ld nb).  Out: the block's L-dot in the lower triangle of A + (j, j); its strict
// upper triangle is set to 0.
__device__ __forceinline__ void diag_fwd_block(int w, const double *Ld, int64_t ldl, const double *Dinv, int nb,
                               double *Ad, int64_t lda, double *Dp, double *Ap, double *Xi) {
  const int tid = threadIdx.x, wave = tid >> 6;
  load_packed2(Dp, Ld, ldl, Ap, Ad, lda, w);
  __syncthreads();
  for (int a = 0; a < w; a += INNER) {
    const int b = min(w, a + INNER);
    const int ib = b - a;
    const int rest = w - b;
    if (a > 0) {
      // rows [a, w) x cols [a, b): subtract [R-dot; B-dot] R^T + [R; B] R-dot^T  (K = a each);
      // tiles of the diagonal 32 x 32 block keep only their lower part.
      const int tr = (w - a + 15) / 16, tc = (ib + 15) / 16;
      for (int t = wave; t < tr * tc; t += DIAG_WAVES) {
        const int r0 = a + (t / tc) * 16, c0 = (t % tc) * 16;
        if (r0 - a + 15 < c0) continue;  // tile strictly above the diagonal
        auto A1 = [&](int i, int k) { const int r = r0 + i; return (r < w) ? Ap[pidx(r, k)] : 0.0; };
        auto B1 = [&](int k, int j) { return (c0 + j < ib) ? Dp[pidx(a + c0 + j, k)] : 0.0; };
        auto A2 = [&](int i, int k) { const int r = r0 + i; return (r < w) ? Dp[pidx(r, k)] : 0.0; };
        auto B2 = [&](int k, int j) { return (c0 + j < ib) ? Ap[pidx(a + c0 + j, k)] : 0.0; };
        dbl4 s = tile_mma(dbl4{0, 0, 0, 0}, A1, B1, a);
        s = tile_mma(s, A2, B2, a);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = r0 + tile_row(e), cc = a + c0 + tile_col();
          if (r < w && cc < b && cc <= r) Ap[pidx(r, cc)] -= s[e];
        }
      }
      __syncthreads();
    }
    if (wave == 0) level2_fwd_wave(Dp, Ap, a, ib);
    __syncthreads();
    if (rest > 0) {
      // Y = C-dot - C D-dot_i^T  (rows [b, w) x cols [a, b), K = 32), then C-dot = Y D_i^-T
      stage_inverse32(Xi, Dinv, nb, a);
      const int trr = (rest + 15) / 16;
      dbl4 acc[3];
#pragma unroll
      for (int sl = 0; sl < 3; ++sl) {
        const int t = wave + DIAG_WAVES * sl;
        if (t >= trr * 2) continue;
        const int r0 = b + (t >> 1) * 16, c0 = (t & 1) * 16;
        auto A = [&](int i, int k) { const int r = r0 + i; return (r < w) ? Dp[pidx(r, a + k)] : 0.0; };
        auto B = [&](int k, int j) { return (c0 + j >= k) ? Ap[pidx(a + c0 + j, a + k)] : 0.0; };
        acc[sl] = tile_mma(dbl4{0, 0, 0, 0}, A, B, INNER);
      }
      __syncthreads();
#pragma unroll
      for (int sl = 0; sl < 3; ++sl) {
        const int t = wave + DIAG_WAVES * sl;
        if (t >= trr * 2) continue;
        const int r0 = b + (t >> 1) * 16, c0 = (t & 1) * 16;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = r0 + tile_row(e);
          if (r < w) Ap[pidx(r, a + c0 + tile_col())] -= acc[sl][e];
        }
      }
      __syncthreads();
#pragma unroll
      for (int sl = 0; sl < 3; ++sl) {
        const int t = wave + DIAG_WAVES * sl;
        if (t >= trr * 2) continue;
        const int r0 = b + (t >> 1) * 16, c0 = (t & 1) * 16;
        auto A = [&](int i, int k) { const int r = r0 + i; return (r < w) ? Ap[pidx(r, a + k)] : 0.0; };
        auto B = [&](int k, int j) { return Xi[(c0 + j) * XLD + k]; };   // (D_i^-1)^T
        acc[sl] = tile_mma(dbl4{0, 0, 0, 0}, A, B, INNER);
      }
      __syncthreads();
#pragma unroll
      for (int sl = 0; sl < 3; ++sl) {
        const int t = wave + DIAG_WAVES * sl;
        if (t >= trr * 2) continue;
        const int r0 = b + (t >> 1) * 16, c0 = (t & 1) * 16;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = r0 + tile_row(e);
          if (r < w) Ap[pidx(r, a + c0 + tile_col())] = acc[sl][e];
        }
      }
      __syncthreads();
    }
  }
  store_block(Ad, lda, w, w, [&](int r, int c) { return (c <= r) ? Ap[pidx(r, c)] : 0.0; });
  __syncthreads();
}

__global__ __launch_bounds__(DIAG_THREADS) void diag_fwd_kernel(int w, const double *Ld, int64_t ldl,
                                                                const double *Dinv, int nb,
                                                                double *Ad, int64_t lda) {
  __shared__ double Dp[DIAG_PACKED];
  __shared__ double Ap[DIAG_PACKED];
  __shared__ double Xi[INNER * XLD];
  diag_fwd_block(w, Ld, ldl, Dinv, nb, Ad, lda, Dp, Ap, Xi);
}

// ---------------------------------------------------------------------------------------------
// D <- chol_unblocked(D) (Sec. 4.1, DPOTF2) for one w x w diagonal block (w <= 128), left-looking
// over 32-column inner blocks [a, b):  [D_i; C] -= [R; B] R^T (MFMA tiles);  then D_i <- its
// Level-2 factor and C <- C D_i^-T in one pass of panel_core32 (every wave holds D_i, the rows of
// C are split 32 per wave).  Then D^-1 for the panel solve, formed in place after L is stored.
// The first non-positive (or NaN) pivot sets *info = col0 + column + 1 unless an earlier block
// already set it; the sweep then continues with NaN so that every kernel still exits normally.
// In/out: A + (j, j) (lower triangle in, factor out, strict upper set to 0).  Out: Dinv (w x w
// inverse, ld nb, zero above the diagonal), only when inv is set (the last block of a
// factorisation has no rows below to solve).  Dp: packed LDS block (DIAG_PACKED doubles).
__device__ __forceinline__ void potf2_block(int w, double *Ad, int64_t lda, double *Dinv, int64_t ld, int ext,
                                            int right, int *info, int64_t col0, double *Dp, int &bad, int inv) {
  const int tid = threadIdx.x, wave = tid >> 6;
  load_packed2(Dp, Ad, lda, nullptr, nullptr, 0, w);
  if (tid == 0) bad = -1;
  __syncthreads();
  for (int a = 0; a < w; a += INNER) {
    const int b = min(w, a + INNER);
    const int ib = b - a;
    if (a > 0) {
      // rows [a, w) x cols [a, b) -= [R; B] R^T  (K = a)
      const int tr = (w - a + 15) / 16, tc = (ib + 15) / 16;
      for (int t = wave; t < tr * tc; t += DIAG_WAVES) {
        const int r0 = a + (t / tc) * 16, c0 = (t % tc) * 16;
        if (r0 - a + 15 < c0) continue;
        auto A = [&](int i, int k) { const int r = r0 + i; return (r < w) ? Dp[pidx(r, k)] : 0.0; };
        auto B = [&](int k, int j) { return (c0 + j < ib) ? Dp[pidx(a + c0 + j, k)] : 0.0; };
        const dbl4 s = tile_mma(dbl4{0, 0, 0, 0}, A, B, a);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = r0 + tile_row(e), cc = a + c0 + tile_col();
          if (r < w && cc < b && cc <= r) Dp[pidx(r, cc)] -= s[e];
        }
      }
      __syncthreads();
    }
    // the diagonal rows in every wave, the rows below split 32 per wave (w - b <= 96)
    const int f = panel_core32<true>(Dp, a, ib, w, b + INNER * wave, wave == 0);
    if (tid == 0 && f >= 0 && bad < 0) bad = a + f;
    __syncthreads();
  }
  if (tid == 0 && bad >= 0 && *info == 0) *info = (int)(col0 + bad + 1);
  // L out first (its stores drain while the inverse is formed in place over it)
  store_block(Ad, lda, w, w, [&](int r, int c) { return (c <= r) ? Dp[pidx(r, c)] : 0.0; });
  if (!inv) return;  // uniform over the workgroup
  __syncthreads();
  block_inverse_inplace(Dp, w);
  store_lower_region(Dinv, ld, ext, Dp, w, right);
  __syncthreads();
}

// POTF2 of one w x w block (w <= 128) with its inverse written to the ext x ext region at Dinv
// (leading dimension ld) and `right` zero columns beside it (see store_lower_region).  66 KB of
// LDS: it fits beside one 64 KB contraction workgroup on a compute unit.
__global__ __launch_bounds__(DIAG_THREADS) void potf2_kernel(int w, double *Ad, int64_t lda, double *Dinv,
                                                             int64_t ld, int ext, int right, int *info,
                                                             int64_t col0, int inv) {
  __shared__ double Dp[DIAG_PACKED];
  __shared__ int bad;
  potf2_block(w, Ad, lda, Dinv, ld, ext, right, info, col0, Dp, bad, inv);
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
// ---------------------------------------------------------------------------------------------
// Symbolic diagonal block (w x w, w <= DIAG_MAX): three small products per sweep step, each one
// launch with one 16 x 16 output tile per workgroup (grid = ceil(w / 16)^2, tile (blockIdx.x /
// nt, blockIdx.x % nt)).  The four waves of a workgroup take consecutive quarters of the tile's
// K range and their partial tiles are summed through LDS in wave order (deterministic), so each
// workgroup reads only its own strips of the operands.  The element-wise steps between the
// products (the triangle masks, Phi, the symmetric output) are folded into the operand accessors
// and the epilogues, and triangular operands start the K range where their nonzeros start.
constexpr int SYM_TILE = 16;

// Sum over k in [k0, k1) of A(i, k) B(k, j) for the workgroup's 16 x 16 tile; the result is
// valid in wave 0 only (tile_mma's layout).  `red` is 3 * 256 doubles of LDS.  Every thread of
// the workgroup must call it.
// tile_mma for K <= 32 with every operand load of the wave issued before the first MFMA (one
// memory latency instead of two).
template <class FA, class FB>
__device__ __forceinline__ dbl4 tile_mma_k32(dbl4 acc, FA A, FB B, int K) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, kq = lane >> 4;
  double a[8], b[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int k = 4 * u + kq;
    a[u] = (k < K) ? A(i, k) : 0.0;
    b[u] = (k < K) ? B(k, i) : 0.0;
  }
#pragma unroll
  for (int u = 0; u < 8; ++u)
    if (4 * u < K) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
  return acc;
}

template <class FA, class FB>
__device__ __forceinline__ dbl4 wg_tile16(FA A, FB B, int k0, int k1, double *red) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int span = (((k1 - k0) + 15) / 16) * 4;  // per wave, a multiple of 4
  const int ka = k0 + wave * span, kb = min(k1, ka + span);
  dbl4 acc{0, 0, 0, 0};
  auto As = [&](int i, int k) { return A(i, ka + k); };
  auto Bs = [&](int k, int j) { return B(ka + k, j); };
  if (kb - ka > 32) acc = tile_mma(acc, As, Bs, kb - ka);  // only the forward panel's two-term range
  else if (kb > ka) acc = tile_mma_k32(acc, As, Bs, kb - ka);
  double *r = as_lds(red);
  if (wave > 0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) r[(wave - 1) * 256 + e * 64 + lane] = acc[e];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] += r[q * 256 + e * 64 + lane];
  }
  return acc;
}

// Reverse (eqn (symrev) on the block), product 1:  P = tril(D)^T tril(Dbar), lower tiles only
// (the rest of P is never read).  D: the factor's diagonal block (ldd); Dbar: the block's
// sensitivities (ldb; lower triangle read); P: ldp.  tril(D)^T[r][k] = D[k][r] needs k >= r and
// tril(Dbar)[k][c] needs k >= c, so k starts at the tile's row offset.
__global__ __launch_bounds__(256) void sym_rev_p_kernel(int w, const double *D, int64_t ldd,
                                                        const double *Dbar, int64_t ldb, double *P,
                                                        int64_t ldp) {
  __shared__ double red[3 * 256];
  const int nt = (w + SYM_TILE - 1) / SYM_TILE;
  const int r0 = (blockIdx.x / nt) * SYM_TILE, c0 = (blockIdx.x % nt) * SYM_TILE;
  if (c0 > r0) return;  // strictly upper tile (workgroup-uniform)
  auto A = [&](int i, int k) {
    const int r = r0 + i;
    return (r < w && k < w && k >= r) ? D[(int64_t)k * ldd + r] : 0.0;
  };
  auto B = [&](int k, int j) {
    const int c = c0 + j;
    return (c < w && k < w && k >= c) ? Dbar[(int64_t)k * ldb + c] : 0.0;
  };
  const dbl4 acc = wg_tile16(A, B, r0, w, red);
  if (threadIdx.x >= 64) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = r0 + tile_row(e), c = c0 + tile_col();
    if (r < w && c <= r) P[(int64_t)r * ldp + c] = acc[e];
  }
}

// Reverse, product 2:  Q = D^-T Y with Y = (Phi(P) + Phi(P)^T) / 2, i.e. Y[k][c] =
// P[max(k,c)][min(k,c)] / 2 read from P's lower triangle.  D^-T[r][k] = Dinv[k][r] needs k >= r.
// Dinv: the block's inverse (ldi, lower); Q: ldq, all tiles.
__global__ __launch_bounds__(256) void sym_rev_q_kernel(int w, const double *P, int64_t ldp,
                                                        const double *Dinv, int64_t ldi, double *Q,
                                                        int64_t ldq) {
  __shared__ double red[3 * 256];
  const int nt = (w + SYM_TILE - 1) / SYM_TILE;
  const int r0 = (blockIdx.x / nt) * SYM_TILE, c0 = (blockIdx.x % nt) * SYM_TILE;
  auto A = [&](int i, int k) {
    const int r = r0 + i;
    return (r < w && k < w && k >= r) ? Dinv[(int64_t)k * ldi + r] : 0.0;
  };
  auto B = [&](int k, int j) {
    const int c = c0 + j;
    if (c >= w || k >= w) return 0.0;
    return 0.5 * P[k >= c ? (int64_t)k * ldp + c : (int64_t)c * ldp + k];
  };
  const dbl4 acc = wg_tile16(A, B, r0, w, red);
  if (threadIdx.x >= 64) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = r0 + tile_row(e), c = c0 + tile_col();
    if (r < w && c < w) Q[(int64_t)r * ldq + c] = acc[e];
  }
}

// Reverse, product 3:  S = Q D^-1 (D^-1[k][c] needs k >= c), lower tiles; each lower entry goes
// to both triangles of A (lda), so the block of the symmetric gradient is exactly symmetric.
__global__ __launch_bounds__(256) void sym_rev_s_kernel(int w, const double *Q, int64_t ldq,
                                                        const double *Dinv, int64_t ldi, double *A,
                                                        int64_t lda) {
  __shared__ double red[3 * 256];
  const int nt = (w + SYM_TILE - 1) / SYM_TILE;
  const int r0 = (blockIdx.x / nt) * SYM_TILE, c0 = (blockIdx.x % nt) * SYM_TILE;
  if (c0 > r0) return;
  auto Am = [&](int i, int k) {
    const int r = r0 + i;
    return (r < w && k < w) ? Q[(int64_t)r * ldq + k] : 0.0;
  };
  auto Bm = [&](int k, int j) {
    const int c = c0 + j;
    return (c < w && k < w && k >= c) ? Dinv[(int64_t)k * ldi + c] : 0.0;
  };
  const dbl4 acc = wg_tile16(Am, Bm, c0, w, red);
  if (threadIdx.x >= 64) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = r0 + tile_row(e), c = c0 + tile_col();
    if (r < w && c <= r) {
      A[(int64_t)r * lda + c] = acc[e];
      A[(int64_t)c * lda + r] = acc[e];
    }
  }
}

// Forward (eqn (symfwd) on the block), product 1:  P = D^-1 Ds, Ds the symmetric matrix with the
// lower triangle of Ad (lda).  D^-1[r][k] needs k <= r.  P: ldp, all tiles.
__global__ __launch_bounds__(256) void sym_fwd_p_kernel(int w, const double *Ad, int64_t lda,
                                                        const double *Dinv, int64_t ldi, double *P,
                                                        int64_t ldp) {
  __shared__ double red[3 * 256];
  const int nt = (w + SYM_TILE - 1) / SYM_TILE;
  const int r0 = (blockIdx.x / nt) * SYM_TILE, c0 = (blockIdx.x % nt) * SYM_TILE;
  auto Am = [&](int i, int k) {
    const int r = r0 + i;
    return (r < w && k <= r) ? Dinv[(int64_t)r * ldi + k] : 0.0;
  };
  auto Bm = [&](int k, int j) {
    const int c = c0 + j;
    if (c >= w || k >= w) return 0.0;
    return Ad[k >= c ? (int64_t)k * lda + c : (int64_t)c * lda + k];
  };
  const dbl4 acc = wg_tile16(Am, Bm, 0, min(w, r0 + SYM_TILE), red);
  if (threadIdx.x >= 64) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = r0 + tile_row(e), c = c0 + tile_col();
    if (r < w && c < w) P[(int64_t)r * ldp + c] = acc[e];
  }
}

// Forward, product 2:  Q = P D^-T (D^-T[k][c] = Dinv[c][k] needs k <= c) and N = -Phi(Q) in full
// (N: ldn): strict upper 0 (upper tiles write zeros without a product), diagonal -Q/2, strict
// lower -Q.
__global__ __launch_bounds__(256) void sym_fwd_n_kernel(int w, const double *P, int64_t ldp,
                                                        const double *Dinv, int64_t ldi, double *N,
                                                        int64_t ldn) {
  __shared__ double red[3 * 256];
  const int nt = (w + SYM_TILE - 1) / SYM_TILE;
  const int r0 = (blockIdx.x / nt) * SYM_TILE, c0 = (blockIdx.x % nt) * SYM_TILE;
  dbl4 acc{0, 0, 0, 0};
  if (c0 <= r0) {
    auto Am = [&](int i, int k) {
      const int r = r0 + i;
      return (r < w && k < w) ? P[(int64_t)r * ldp + k] : 0.0;
    };
    auto Bm = [&](int k, int j) {
      const int c = c0 + j;
      return (c < w && k <= c) ? Dinv[(int64_t)c * ldi + k] : 0.0;
    };
    acc = wg_tile16(Am, Bm, 0, min(w, c0 + SYM_TILE), red);
  }
  if (threadIdx.x >= 64) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = r0 + tile_row(e), c = c0 + tile_col();
    if (r < w && c < w) N[(int64_t)r * ldn + c] = c < r ? -acc[e] : (c == r ? -0.5 * acc[e] : 0.0);
  }
}

// Forward, product 3:  L-dot_D = tril(D) Phi(Q) = -(tril(D) N), lower tiles, lower entries written
// to Ad (lda); D: the factor's diagonal block (ldd).  tril(D)[r][k] needs k <= r and N[k][c]
// needs k >= c.  The strict upper triangle of the block in Ad is set to 0 (products that read
// the block as a dense operand rely on it).
__global__ __launch_bounds__(256) void sym_fwd_l_kernel(int w, const double *D, int64_t ldd,
                                                        const double *N, int64_t ldn, double *Ad,
                                                        int64_t lda) {
  __shared__ double red[3 * 256];
  const int nt = (w + SYM_TILE - 1) / SYM_TILE;
  const int r0 = (blockIdx.x / nt) * SYM_TILE, c0 = (blockIdx.x % nt) * SYM_TILE;
  if (c0 > r0) {  // strictly upper tile: zeros, no product (workgroup-uniform)
    const int r = r0 + (int)threadIdx.x / SYM_TILE, c = c0 + (int)threadIdx.x % SYM_TILE;
    if (r < w && c < w) Ad[(int64_t)r * lda + c] = 0.0;
    return;
  }
  auto Am = [&](int i, int k) {
    const int r = r0 + i;
    return (r < w && k <= r) ? D[(int64_t)r * ldd + k] : 0.0;
  };
  auto Bm = [&](int k, int j) {
    const int c = c0 + j;
    return (c < w && k < w) ? N[(int64_t)k * ldn + c] : 0.0;
  };
  const dbl4 acc = wg_tile16(Am, Bm, c0, min(w, r0 + SYM_TILE), red);
  if (threadIdx.x >= 64) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = r0 + tile_row(e), c = c0 + tile_col();
    if (r < w && c < w) Ad[(int64_t)r * lda + c] = c <= r ? -acc[e] : 0.0;
  }
}

// Reverse-sweep panel solve C-bar/2 = alpha X D^-1 (X: M x w panel, ldx; D^-1 lower, ldi, so
// k >= c), written to C (ldc) and mirrored to Cm (ldcm: Cm[c][r] = C[r][c]).  One 16 x 16 output
// tile per workgroup with the K range split over its waves, so there are no partial tiles to
// reduce.  The w/16 column tiles of one 16-row strip go to workgroups 8 apart in launch order
// (one XCD under round-robin dispatch), so each strip of the panel is fetched into one L2; grid =
// ceil(ceil(M/16) / 8) * 8 * ceil(w/16).
__global__ __launch_bounds__(256) void rev_panel_solve_kernel(int M, int w, const double *X, int64_t ldx,
                                                              const double *Dinv, int64_t ldi, double alpha,
                                                              double *C, int64_t ldc, double *Cm, int64_t ldcm) {
  __shared__ double red[3 * 256];
  const int nct = (w + SYM_TILE - 1) / SYM_TILE;
  const int g = blockIdx.x;
  const int r0 = ((g / (8 * nct)) * 8 + (g % 8)) * SYM_TILE, c0 = ((g / 8) % nct) * SYM_TILE;
  if (r0 >= M) return;  // padding of the last group of strips (workgroup-uniform)
  auto A = [&](int i, int k) {
    const int r = r0 + i;
    return (r < M && k < w) ? X[(int64_t)r * ldx + k] : 0.0;
  };
  auto B = [&](int k, int j) {
    const int c = c0 + j;
    return (c < w && k < w && k >= c) ? Dinv[(int64_t)k * ldi + c] : 0.0;
  };
  const dbl4 acc = wg_tile16(A, B, c0, w, red);
  if (threadIdx.x >= 64) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = r0 + tile_row(e), c = c0 + tile_col();
    if (r < M && c < w) {
      const double v = alpha * acc[e];
      C[(int64_t)r * ldc + c] = v;
      if (Cm) Cm[(int64_t)c * ldcm + r] = v;
    }
  }
}

// Forward-sweep panel solve with the symbolic diagonal block:  Out = Cd D^-T + Cl N^T  (M x w),
// N = -Phi(Q) and D^-1 both lower, so both terms run over k <= c; Cd (ldcd) is the updated
// C-dot, Cl (ldcl) the factor's panel C, Out (ldo) must not overlap Cd.  Same tiling and
// strip-to-XCD mapping as rev_panel_solve_kernel; the two terms form one K range of 2 kq.
__global__ __launch_bounds__(256) void fwd_panel_solve_kernel(int M, int w, const double *Cd, int64_t ldcd,
                                                              const double *Cl, int64_t ldcl,
                                                              const double *Dinv, int64_t ldi,
                                                              const double *N, int64_t ldn, double *Out,
                                                              int64_t ldo) {
  __shared__ double red[3 * 256];
  const int nct = (w + SYM_TILE - 1) / SYM_TILE;
  const int g = blockIdx.x;
  const int r0 = ((g / (8 * nct)) * 8 + (g % 8)) * SYM_TILE, c0 = ((g / 8) % nct) * SYM_TILE;
  if (r0 >= M) return;  // padding of the last group of strips (workgroup-uniform)
  const int kq = min(w, c0 + SYM_TILE);
  auto A = [&](int i, int k) {
    const int r = r0 + i;
    if (r >= M) return 0.0;
    return k < kq ? Cd[(int64_t)r * ldcd + k] : Cl[(int64_t)r * ldcl + (k - kq)];
  };
  auto B = [&](int k, int j) {
    const int c = c0 + j;
    if (c >= w) return 0.0;
    const int kk = k < kq ? k : k - kq;
    if (kk > c) return 0.0;
    return k < kq ? Dinv[(int64_t)c * ldi + kk] : N[(int64_t)c * ldn + kk];
  };
  const dbl4 acc = wg_tile16(A, B, 0, 2 * kq, red);
  if (threadIdx.x >= 64) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = r0 + tile_row(e), c = c0 + tile_col();
    if (r < M && c < w) Out[(int64_t)r * ldo + c] = acc[e];
  }
}

// Lower-left part of the inverse of a block of width 128 < w <= 256 whose two diagonal halves
// X00 = D00^-1 (128 wide) and X11 = D11^-1 (w - 128 wide) are already in place in Dinv (leading
// dimension nb):  X10 = -X11 (D10 X00), the block form of the triangular inverse.  Two launches
// over every such block of L (block b at (b nb, b nb); n bounds the last one):
//   phase 0: T_b = D10 X00 into T + b * 128 * 128 (ld 128);   phase 1: X10 = -X11 T_b.
// grid = nblocks * 64, one 16 x 16 tile of a 128 x 128 output per workgroup.
__global__ __launch_bounds__(256) void inv_offdiag_kernel(int phase, int64_t n, int nb, const double *L,
                                                          int64_t ldl, double *Dinv, double *T) {
  __shared__ double red[3 * 256];
  const int64_t b = blockIdx.x / 64;
  const int t = blockIdx.x % 64;
  const int wb = (int)min<int64_t>(nb, n - b * nb);
  const int h2 = wb - DIAG_MAX;
  const int r0 = (t / 8) * SYM_TILE, c0 = (t % 8) * SYM_TILE;
  if (h2 <= 0 || r0 >= h2) return;  // workgroup-uniform
  double *Xb = Dinv + b * nb * nb;
  double *Tb = T + b * DIAG_MAX * DIAG_MAX;
  const double *L10 = L + (b * nb + DIAG_MAX) * ldl + b * nb;
  dbl4 acc;
  if (phase == 0) {  // T[r][c] = sum_{k >= c} D10[r][k] X00[k][c]
    auto A = [&](int i, int k) {
      const int r = r0 + i;
      return (r < h2 && k < DIAG_MAX) ? L10[(int64_t)r * ldl + k] : 0.0;
    };
    auto B = [&](int k, int j) {
      const int c = c0 + j;
      return (k < DIAG_MAX && k >= c) ? Xb[(int64_t)k * nb + c] : 0.0;
    };
    acc = wg_tile16(A, B, c0, DIAG_MAX, red);
  } else {           // X10[r][c] = -sum_{k <= r} X11[r][k] T[k][c]
    auto A = [&](int i, int k) {
      const int r = r0 + i;
      return (r < h2 && k <= r) ? Xb[(int64_t)(DIAG_MAX + r) * nb + DIAG_MAX + k] : 0.0;
    };
    auto B = [&](int k, int j) { return (k < h2) ? Tb[(int64_t)k * DIAG_MAX + c0 + j] : 0.0; };
    acc = wg_tile16(A, B, 0, min(h2, r0 + SYM_TILE), red);
  }
  if (threadIdx.x >= 64) return;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int r = r0 + tile_row(e), c = c0 + tile_col();
    if (r < h2) {
      if (phase == 0) Tb[(int64_t)r * DIAG_MAX + c] = acc[e];
      else Xb[(int64_t)(DIAG_MAX + r) * nb + c] = -acc[e];
    }
  }
}

// Column-major (LAPACK) storage of an n x n matrix is the row-major storage of its transpose, so
// the column-major entry points convert with these two element-wise kernels.  Each element pair
// (r, c), (c, r) is read and written by one thread only, so both may work in place.
// dst[r][c] = src[c][r] for r >= c: the lower triangle of dst from the upper triangle of src.
__global__ __launch_bounds__(256) void lower_from_upper_kernel(int64_t n, const double *src, int64_t lds,
                                                               double *dst, int64_t ldd) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n, c = e - r * n;
    if (c <= r) dst[r * ldd + c] = src[c * lds + r];
  }
}

// A[c][r] = A[r][c] for r > c, then A[r][c] = 0: the strict lower triangle moved to the strict
// upper triangle (the diagonal stays).
__global__ __launch_bounds__(256) void lower_to_upper_kernel(int64_t n, double *A, int64_t lda) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n, c = e - r * n;
    if (c < r) {
      A[c * lda + r] = A[r * lda + c];
      A[r * lda + c] = 0.0;
    }
  }
}

// FP32 storage of the single-matrix calls: dst[r * ldd + c] = element (r, c) of the float matrix
// src for c <= r (src row-major with ld lds, or column-major when col is set), 0 above the
// diagonal (the lower triangle is the input).
__global__ __launch_bounds__(256) void widen_lower_kernel(int64_t n, const float *src, int64_t lds, int col,
                                                          double *dst, int64_t ldd) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n, c = e - r * n;
    dst[r * ldd + c] = c <= r ? (double)(col ? src[r + c * lds] : src[r * lds + c]) : 0.0;
  }
}

// Element (r, c) of the float matrix dst (layout as above) = src[r * lds + c] rounded to float, for
// every r, c < n.
__global__ __launch_bounds__(256) void narrow_kernel(int64_t n, const double *src, int64_t lds, float *dst,
                                                     int64_t ldd, int col) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / n, c = e - r * n;
    const float v = (float)src[r * lds + c];
    if (col) dst[r + c * ldd] = v;
    else dst[r * ldd + c] = v;
  }
}

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
