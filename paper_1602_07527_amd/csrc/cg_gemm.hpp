// MFMA contraction kernels for the Level-3 updates (Sec. 4.2 of Murray 2016: the GEMM-, SYRK- and
// TRSM-shaped steps of the blocked factorisation and its derivatives).  Operands and results are
// FP64 in memory; the products run on FP64 MFMA, or on FP32 MFMA or split-bfloat16 MFMA for the
// reduced-precision trailing updates (template parameter CP).
//
//   C[m, n] = alpha * sum_k A(m, k) B(k, n) + beta * Cin[m, n]        (m < M, n < N, k < K)
//
// With a second operand pair (A2, B2 non-null) the sum runs over both pairs,
//   C = alpha * (op(A) op(B) + op(A2) op(B2)) + beta * Cin,
// as one K range of length 2K whose second half reads the second pair (the SYR2K-shaped updates
// of the forward sweep: one launch and one pass over C instead of two).
//
// A(m, k) is read from A[m*lda + k] (AT = false) or A[k*lda + m] (AT = true); B(k, n) from
// B[k*ldb + n] (BT = false) or B[n*ldb + k] (BT = true).  All matrices are row-major doubles.
//
// Tiling for gfx950: a 256-thread workgroup (four wave64s in a 2 x 2 arrangement) owns a
// 128 x 128 output tile; each wave owns 64 x 64 as a 4 x 4 grid of 16 x 16 accumulators fed by
// v_mfma_f64_16x16x4_f64.  K is staged through LDS 16 deep, double-buffered, so one barrier per
// K-step.  Tall-skinny products are split over K (grid.z); each split writes a private partial
// tile and a separate kernel sums the partials in a fixed order, so results are bitwise
// reproducible (no floating-point atomics).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cg {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// Arithmetic of a contraction.  Operands and results are FP64 in memory either way.
//   CP_F64: v_mfma_f64_16x16x4_f64, FP64 accumulation.
//   CP_F32: operands rounded to FP32 as they leave LDS, v_mfma_f32_16x16x4_f32 with FP32
//           accumulation over the K range of one launch (one split); the epilogue (alpha, beta,
//           split sums) stays in FP64.
//   CP_BF16X3: each operand split into bfloat16 hi + lo parts (hi = bf16(fp32(x)),
//           lo = bf16(fp32(x) - hi), round to nearest even), the product taken as
//           hi*hi + hi*lo + lo*hi with v_mfma_f32_16x16x16_bf16 and FP32 accumulation within
//           one split; ~16 significant bits per operand.
//   CP_BF16X6: each operand split into three bfloat16 parts (hi = bf16(fp32(x)), mid =
//           bf16(fp32(x) - hi), lo = bf16(fp32(x) - hi - mid)) and the product taken as the six
//           terms hi*hi + hi*mid + mid*hi + hi*lo + lo*hi + mid*mid (the terms below 2^-24 of
//           the product dropped), FP32 accumulation within one split; ~24 significant bits per
//           operand, as FP32.
constexpr int CP_F64 = 0;
constexpr int CP_F32 = 1;
constexpr int CP_BF16X3 = 2;
constexpr int CP_BF16X6 = 3;
__host__ __device__ constexpr bool cp_split(int cp) { return cp == CP_BF16X3 || cp == CP_BF16X6; }

typedef short shrt4 __attribute__((ext_vector_type(4)));

// bfloat16 bits of a float, round to nearest even (finite inputs).
__device__ __forceinline__ unsigned bf16_rne(float f) {
  const unsigned u = __float_as_uint(f);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

// Split four doubles into their bf16 hi and lo parts.
__device__ __forceinline__ void bf16_split4(double x0, double x1, double x2, double x3, shrt4 &hi, shrt4 &lo) {
  const double x[4] = {x0, x1, x2, x3};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float f = (float)x[i];
    const unsigned h = bf16_rne(f);
    const float r = f - __uint_as_float(h << 16);
    hi[i] = (short)h;
    lo[i] = (short)bf16_rne(r);
  }
}

__device__ __forceinline__ flt4 mfma_bf16x3(const shrt4 &ah, const shrt4 &al, const shrt4 &bh, const shrt4 &bl,
                                             flt4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
}

// The parts of four operand values in one split mode: hi, mid (BF16X6 only) and lo.
struct Split4 {
  shrt4 h, m, l;
};

// Split four doubles into bfloat16 parts: two (hi, lo) for BF16X3, three (hi, mid, lo) for
// BF16X6, each the round-to-nearest-even bfloat16 of what the previous parts leave of fp32(x).
template <int CP>
__device__ __forceinline__ Split4 split4(double x0, double x1, double x2, double x3) {
  Split4 s;
  if constexpr (CP == CP_BF16X3) {
    bf16_split4(x0, x1, x2, x3, s.h, s.l);
  } else {
    const double x[4] = {x0, x1, x2, x3};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float f = (float)x[i];
      const unsigned h = bf16_rne(f);
      const float r1 = f - __uint_as_float(h << 16);
      const unsigned m = bf16_rne(r1);
      const float r2 = r1 - __uint_as_float(m << 16);
      s.h[i] = (short)h;
      s.m[i] = (short)m;
      s.l[i] = (short)bf16_rne(r2);
    }
  }
  return s;
}

// acc += a b over one 16-deep bfloat16 K-group in split mode CP, smallest terms first.
template <int CP>
__device__ __forceinline__ flt4 mfma_split(const Split4 &a, const Split4 &b, flt4 c) {
  if constexpr (CP == CP_BF16X3) {
    return mfma_bf16x3(a.h, a.l, b.h, b.l, c);
  } else {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.m, b.m, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.l, b.h, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.h, b.l, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.m, b.h, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.h, b.m, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a.h, b.h, c, 0, 0, 0);
  }
}

template <int CP> struct Mfma;
template <> struct Mfma<CP_F64> {
  typedef dbl4 acc_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // Output layout of the 16 x 16 block: lane l, element i holds row 4*i + l/16, column l%16.
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * i + (lane >> 4); }
};
template <> struct Mfma<CP_BF16X3> {  // accumulator and output layout of the FP32 MFMAs
  typedef flt4 acc_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0f, 0.0f, 0.0f, 0.0f}; }
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};
template <> struct Mfma<CP_BF16X6> : Mfma<CP_BF16X3> {};
template <> struct Mfma<CP_F32> {
  typedef flt4 acc_t;
  static __device__ __forceinline__ acc_t zero() { return acc_t{0.0f, 0.0f, 0.0f, 0.0f}; }
  static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32((float)a, (float)b, c, 0, 0, 0);
  }
  // Output layout: lane l, element i holds row 4*(l/16) + i, column l%16.
  static __device__ __forceinline__ int row(int lane, int i) { return 4 * (lane >> 4) + i; }
};

constexpr int GEMM_BM = 128;
constexpr int GEMM_BN = 128;
constexpr int GEMM_BK = 16;
constexpr int GEMM_PAD = 4;
constexpr int GEMM_THREADS = 256;

struct GemmArgs {
  int M, N, K;
  const double *A;
  int64_t lda;
  const double *B;
  int64_t ldb;
  double *C;            // output (or the partial buffer when splits > 1)
  int64_t ldc;
  const double *Cin;    // read when beta != 0 (may alias C)
  int64_t ldcin;
  double alpha, beta;
  double *Cm;           // optional transposed copy: Cm[n*ldcm + m] = C[m, n]
  int64_t ldcm;
  int kchunk;           // K extent of one split (multiple of GEMM_BK)
  int64_t split_stride; // elements between the partial tiles of consecutive splits
  int lower_only;       // skip output tiles lying strictly above the diagonal (m < n throughout)
  const double *A2;     // optional second pair, same shapes and transposition as (A, B)
  int64_t lda2;
  const double *B2;
  int64_t ldb2;
  // Stream-K schedule (fast kernel only; sk_wgs == 0 selects the uniform splits above): the
  // output's sk_tiles tiles (sk_tm along M, tile t at (t % sk_tm, t / sk_tm)) times their sk_kt
  // K-tiles form T units in tile-major order, and workgroup w takes units
  // [w T / sk_wgs, (w+1) T / sk_wgs).  Its piece of tile t goes to the 128 x 128 partial slot
  // w + t of C (row stride ldc = 128, slot stride split_stride).
  int sk_wgs = 0;
  int sk_kt = 0;
  int sk_tm = 0;
  int sk_tiles = 0;
};

// K extent of the combined range: K, or 2K with a second operand pair.
__device__ __forceinline__ int gemm_k_total(const GemmArgs &p) { return p.A2 ? 2 * p.K : p.K; }

constexpr int GEMM_LDS_A = GEMM_BK * (GEMM_BM + GEMM_PAD);   // doubles per A stage
constexpr int GEMM_LDS_B = GEMM_BK * (GEMM_BN + GEMM_PAD);   // doubles per B stage
constexpr int GEMM_LDS = 2 * (GEMM_LDS_A + GEMM_LDS_B);      // doubles of LDS for one tile product

// One 128 x 128 output tile (rows m0.., columns n0..) over K range [kbeg, kend), written to Cout
// with the epilogue of p (alpha, beta * Cin, optional transposed copy).  Called by a whole
// 256-thread workgroup; `lds` holds GEMM_LDS doubles.  Ends with a barrier, so the workgroup may
// reuse `lds` right after.
template <bool AT, bool BT, int CP = CP_F64>
__device__ void gemm_tile(const GemmArgs &p, int m0, int n0, int kbeg, int kend, double *Cout,
                          double *lds) {
  typedef Mfma<CP> MM;
  constexpr int BM = GEMM_BM, BN = GEMM_BN, BK = GEMM_BK, LDA_S = BM + GEMM_PAD,
                LDB_S = BN + GEMM_PAD;
  // lds addresses LDS; re-typed so that a caller that passes it as a plain pointer (an
  // out-of-line function) still gets LDS instructions rather than flat ones
  double *const lb = (double *)(__attribute__((address_space(3))) double *)lds;
  auto As = [&](int buf) { return lb + buf * GEMM_LDS_A; };
  auto Bs = [&](int buf) { return lb + 2 * GEMM_LDS_A + buf * GEMM_LDS_B; };

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  typename MM::acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = MM::zero();

  double ra[8], rb[8];
  // Global -> registers for the K-tile starting at k0.
  auto load_tile = [&](int k0) {
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int e = it * GEMM_THREADS + tid;
      int m, k;
      if (!AT) { m = e >> 4; k = e & 15; }      // contiguous along k
      else     { k = e >> 7; m = e & 127; }     // contiguous along m
      const int gm = m0 + m, gk = k0 + k;
      double v = 0.0;
      if (gm < p.M && gk < kend) {
        if (gk < p.K) v = AT ? p.A[(int64_t)gk * p.lda + gm] : p.A[(int64_t)gm * p.lda + gk];
        else v = AT ? p.A2[(int64_t)(gk - p.K) * p.lda2 + gm] : p.A2[(int64_t)gm * p.lda2 + (gk - p.K)];
      }
      ra[it] = v;
    }
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int e = it * GEMM_THREADS + tid;
      int n, k;
      if (!BT) { k = e >> 7; n = e & 127; }     // contiguous along n
      else     { n = e >> 4; k = e & 15; }      // contiguous along k
      const int gn = n0 + n, gk = k0 + k;
      double v = 0.0;
      if (gn < p.N && gk < kend) {
        if (gk < p.K) v = BT ? p.B[(int64_t)gn * p.ldb + gk] : p.B[(int64_t)gk * p.ldb + gn];
        else v = BT ? p.B2[(int64_t)gn * p.ldb2 + (gk - p.K)] : p.B2[(int64_t)(gk - p.K) * p.ldb2 + gn];
      }
      rb[it] = v;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int e = it * GEMM_THREADS + tid;
      int m, k;
      if (!AT) { m = e >> 4; k = e & 15; } else { k = e >> 7; m = e & 127; }
      As(buf)[k * LDA_S + m] = ra[it];
    }
#pragma unroll
    for (int it = 0; it < 8; ++it) {
      const int e = it * GEMM_THREADS + tid;
      int n, k;
      if (!BT) { k = e >> 7; n = e & 127; } else { n = e >> 4; k = e & 15; }
      Bs(buf)[k * LDB_S + n] = rb[it];
    }
  };

  const int nkt = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;
  if (nkt > 0) {
    load_tile(kbeg);
    store_tile(0);
  }
  __syncthreads();
  const int frag_k = lane >> 4, frag_i = lane & 15;
  for (int kt = 0; kt < nkt; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nkt) load_tile(kbeg + (kt + 1) * BK);
    const double *as = As(buf);
    const double *bs = Bs(buf);
    if constexpr (cp_split(CP)) {
      // one 16-deep bf16 K-group per K-tile: the lanes of slot frag_k take k = 4 frag_k .. + 3
      Split4 sa[4], sb[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double *pa = as + 4 * frag_k * LDA_S + wm * 64 + t * 16 + frag_i;
        sa[t] = split4<CP>(pa[0], pa[LDA_S], pa[2 * LDA_S], pa[3 * LDA_S]);
        const double *pb = bs + 4 * frag_k * LDB_S + wn * 64 + t * 16 + frag_i;
        sb[t] = split4<CP>(pb[0], pb[LDB_S], pb[2 * LDB_S], pb[3 * LDB_S]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = mfma_split<CP>(sa[a], sb[b], acc[a][b]);
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        double af[4], bf[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) af[t] = as[(kk + frag_k) * LDA_S + wm * 64 + t * 16 + frag_i];
#pragma unroll
        for (int t = 0; t < 4; ++t) bf[t] = bs[(kk + frag_k) * LDB_S + wn * 64 + t * 16 + frag_i];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            acc[a][b] = MM::step(af[a], bf[b], acc[a][b]);
      }
    }
    if (kt + 1 < nkt) store_tile(buf ^ 1);
    __syncthreads();
  }

  // Epilogue in FP64.
  const double alpha = p.alpha, beta = p.beta;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gm = m0 + wm * 64 + a * 16 + MM::row(lane, i);
        const int gn = n0 + wn * 64 + b * 16 + (lane & 15);
        if (gm < p.M && gn < p.N) {
          double v = alpha * (double)acc[a][b][i];
          if (beta != 0.0) v += beta * p.Cin[(int64_t)gm * p.ldcin + gn];
          Cout[(int64_t)gm * p.ldc + gn] = v;
          if (p.Cm) p.Cm[(int64_t)gn * p.ldcm + gm] = v;
        }
      }
  __syncthreads();
}

// TAG only separates kernel names for profiling (1: reverse-sweep panel contraction,
// 2: factor-sweep panel contraction, 3: forward-sweep panel contraction, 0: other products).
template <bool AT, bool BT, int TAG, int CP = CP_F64>
__global__ __launch_bounds__(GEMM_THREADS) void gemm_f64_kernel(GemmArgs p) {
  __shared__ double lds[GEMM_LDS];
  const int m0 = blockIdx.x * GEMM_BM;
  const int n0 = blockIdx.y * GEMM_BN;
  if (p.lower_only && m0 + GEMM_BM - 1 < n0) return;  // whole tile strictly above the diagonal
  const int z = blockIdx.z;
  const int kbeg = z * p.kchunk;
  const int kend = min(gemm_k_total(p), kbeg + p.kchunk);
  gemm_tile<AT, BT, CP>(p, m0, n0, kbeg, kend, p.C + (int64_t)z * p.split_stride, lds);
}

// ---------------------------------------------------------------------------------------------
// Fast path for tile-aligned products (M, N multiples of 128; every K-chunk a multiple of 16;
// leading dimensions even and A, B 16-byte aligned): eight wave64s (2 x 4, each 64 x 32 of the
// 128 x 128 tile) and gfx950's direct global->LDS loads (global_load_lds_dwordx4) into a two-stage
// ring of 16-deep K-tiles, so no registers stage the operands.  64 KB of LDS per workgroup lets two
// workgroups share a compute unit (four waves per SIMD).  Operands that are contiguous along K are
// stored with their 16-byte chunks XOR-swizzled by row, and each lane reads two consecutive k of
// such an operand with one 16-byte LDS read that feeds two consecutive MFMAs: the k of MFMA
// 2u + h for the lanes of slot s (= lane / 16) is 8u + 2s + h, which covers every k of the tile
// once and lets 8 lanes of a read pass hit 8 distinct 16-byte bank groups.
typedef __attribute__((address_space(3))) void lds_void;
typedef double dbl2v __attribute__((ext_vector_type(2)));
constexpr int DMA_BK = 16;
constexpr int DMA_THREADS = 512;

__host__ __device__ constexpr int waitcnt_vm(int n) {  // s_waitcnt immediate: vmcnt(n) only
  return (n & 15) | (((n >> 4) & 3) << 14) | (7 << 4) | (15 << 8);
}

// WIDE: 128 x 256 output tiles (each wave 64 x 64): the A strip of a K-tile is loaded once for
// both 128-column halves, 96 KB of LDS and up to 256 registers, one workgroup per compute unit.
template <bool AT, bool BT, int TAG, int CP = CP_F64, bool P2 = false, bool WIDE = false>
__global__ __launch_bounds__(DMA_THREADS, WIDE ? 2 : 4) void gemm_f64_dma_kernel(GemmArgs p) {
  typedef Mfma<CP> MM;
  constexpr int BM = GEMM_BM, BN = WIDE ? 2 * GEMM_BN : GEMM_BN, BK = DMA_BK;
  constexpr int TILE_A = BM * BK, TILE_B = BN * BK, STAGE = TILE_A + TILE_B;
  constexpr int WM = 2, WN = 4, NW = WM * WN;
  constexpr int NQA = TILE_A * 8 / 1024 / NW;  // 1 KB DMA instructions per wave per K-tile of A
  constexpr int NQB = TILE_B * 8 / 1024 / NW;  // ... and of B
  static_assert(NQA * NW * 1024 == TILE_A * 8 && NQB * NW * 1024 == TILE_B * 8,
                "tiles must split evenly over the waves");
  static_assert(BK % 8 == 0, "paired fragment reads take k in groups of 8");
  constexpr int CH = BK / 2;                   // 16-byte chunks in a K-contiguous row
  constexpr int RPI = 64 / CH;                 // K-contiguous rows per DMA instruction
  constexpr int NH = BN / GEMM_BN;             // 1 KB pieces of an N-contiguous row of B
  constexpr int TMW = BM / WM / 16, TNW = BN / WN / 16;
  __shared__ __attribute__((aligned(16))) double smem[2 * STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;
  // Work of this workgroup: one (tile, K-range) piece under uniform splits, or the pieces of its
  // stream-K unit range (at most two tiles, as the host keeps T / sk_wgs <= sk_kt).
  int m0 = 0, n0 = 0, kbeg = 0, nkt = 0, cm0 = 0, cn0 = 0;
  double *Cout = nullptr;
  int64_t su = 0, su1 = 0;
  if (p.sk_wgs) {
    const int64_t T = (int64_t)p.sk_kt * p.sk_tiles;
    su = (int64_t)blockIdx.x * T / p.sk_wgs;
    su1 = (int64_t)(blockIdx.x + 1) * T / p.sk_wgs;
  } else {
    m0 = blockIdx.x * BM;
    n0 = blockIdx.y * BN;
    if (p.lower_only && m0 + BM - 1 < n0) return;
    const int z = blockIdx.z;
    kbeg = z * p.kchunk;
    const int kend = min(P2 ? 2 * p.K : p.K, kbeg + p.kchunk);
    nkt = (kend > kbeg) ? (kend - kbeg) / BK : 0;
    Cout = p.C + (int64_t)z * p.split_stride;
  }

  // Loop-invariant per-lane byte offsets inside a tile (per operand pair); the tile bases are
  // wave-uniform.  K is a multiple of BK, so no K-tile straddles the two pairs.  P2 (a second
  // operand pair, in A2 and B2) is a template parameter so single products carry no pair logic.
  constexpr int NP = P2 ? 2 : 1;
  uint32_t offA[NP][NQA], offB[NP][NQB];
  int ldsA[NQA], ldsB[NQB];
#pragma unroll
  for (int h = 0; h < NP; ++h) {
    const int64_t la = h ? p.lda2 : p.lda, lb = h ? p.ldb2 : p.ldb;
#pragma unroll
    for (int q = 0; q < NQA; ++q) {
      const int i = wave * NQA + q;
      if (!AT) {
        const int r = i * RPI + lane / CH, c = (lane % CH) ^ (r % CH);
        offA[h][q] = (uint32_t)(r * la * 8 + c * 16);
        ldsA[q] = i * RPI * BK;
      } else {
        offA[h][q] = (uint32_t)(i * la * 8 + lane * 16);
        ldsA[q] = i * BM;
      }
    }
#pragma unroll
    for (int q = 0; q < NQB; ++q) {
      const int i = wave * NQB + q;
      if (!BT) {  // K-row i / NH, 128-column piece i % NH
        offB[h][q] = (uint32_t)((i / NH) * lb * 8 + (i % NH) * 1024 + lane * 16);
        ldsB[q] = (i / NH) * BN + (i % NH) * GEMM_BN;
      } else {
        const int r = i * RPI + lane / CH, c = (lane % CH) ^ (r % CH);
        offB[h][q] = (uint32_t)(r * lb * 8 + c * 16);
        ldsB[q] = i * RPI * BK;
      }
    }
  }

  auto issue = [&](int kt, int st) {
    const int kg = kbeg + kt * BK;                 // position in the combined K range
    const int h = (P2 && kg >= p.K) ? 1 : 0;       // operand pair (wave-uniform)
    const int kl = kg - h * p.K;
    const double *Ab = h ? p.A2 : p.A, *Bb = h ? p.B2 : p.B;
    const int64_t la = h ? p.lda2 : p.lda, lb = h ? p.ldb2 : p.ldb;
    const char *ga = (const char *)(AT ? Ab + (int64_t)kl * la + m0 : Ab + (int64_t)m0 * la + kl);
    const char *gb = (const char *)(BT ? Bb + (int64_t)n0 * lb + kl : Bb + (int64_t)kl * lb + n0);
    double *as = smem + st * STAGE;
    double *bs = as + TILE_A;
#pragma unroll
    for (int q = 0; q < NQA; ++q)
      __builtin_amdgcn_global_load_lds((const void *)(ga + offA[P2 ? h : 0][q]), (lds_void *)(as + ldsA[q]), 16, 0, 0);
#pragma unroll
    for (int q = 0; q < NQB; ++q)
      __builtin_amdgcn_global_load_lds((const void *)(gb + offB[P2 ? h : 0][q]), (lds_void *)(bs + ldsB[q]), 16, 0, 0);
  };

  const int fk = lane >> 4, fi = lane & 15;
  constexpr int W0 = waitcnt_vm(0);
  for (int seg = 0;; ++seg) {
  if (p.sk_wgs) {
    if (su >= su1) break;
    const int64_t t = su / p.sk_kt;
    const int64_t e = min(su1, (t + 1) * (int64_t)p.sk_kt);
    m0 = (int)(t % p.sk_tm) * BM;
    n0 = (int)(t / p.sk_tm) * BN;
    kbeg = (int)(su - t * p.sk_kt) * BK;
    nkt = (int)(e - su);
    cm0 = m0;
    cn0 = n0;
    Cout = p.C + ((int64_t)blockIdx.x + t) * p.split_stride;
    su = e;
    // every wave has finished reading the ring (and the previous piece's stores are queued)
    if (seg > 0) __syncthreads();
  } else if (seg > 0) {
    break;
  }
  typename MM::acc_t acc[TMW][TNW];
#pragma unroll
  for (int a = 0; a < TMW; ++a)
#pragma unroll
    for (int b = 0; b < TNW; ++b) acc[a][b] = MM::zero();

  if (nkt > 0) issue(0, 0);
  for (int kt = 0; kt < nkt; ++kt) {
    // This wave's loads of tile kt are done; the barrier makes every wave's part visible and
    // guarantees the other stage is no longer being read before it is refilled.
    __builtin_amdgcn_s_waitcnt(W0);
    __builtin_amdgcn_s_barrier();
    if (kt + 1 < nkt) issue(kt + 1, (kt + 1) & 1);
    const double *as = smem + (kt & 1) * STAGE;
    const double *bs = as + TILE_A;
    if constexpr (cp_split(CP)) {
      // one 16-deep bf16 K-group per K-tile: the lanes of slot fk take k = 4 fk .. 4 fk + 3,
      // i.e. 16-byte chunks 2 fk and 2 fk + 1 of a K-contiguous row
      static_assert(BK == 16, "the split-bf16 path takes one 16-deep K-tile per MFMA");
      Split4 sa[TMW], sb[TNW];
#pragma unroll
      for (int t = 0; t < TMW; ++t) {
        const int m = wm * (BM / WM) + t * 16 + fi;
        double x0, x1, x2, x3;
        if (AT) {
          x0 = as[(4 * fk) * BM + m]; x1 = as[(4 * fk + 1) * BM + m];
          x2 = as[(4 * fk + 2) * BM + m]; x3 = as[(4 * fk + 3) * BM + m];
        } else {
          const dbl2v p0 = *(const dbl2v *)&as[m * BK + (((2 * fk) ^ (m % CH)) << 1)];
          const dbl2v p1 = *(const dbl2v *)&as[m * BK + (((2 * fk + 1) ^ (m % CH)) << 1)];
          x0 = p0[0]; x1 = p0[1]; x2 = p1[0]; x3 = p1[1];
        }
        sa[t] = split4<CP>(x0, x1, x2, x3);
      }
#pragma unroll
      for (int t = 0; t < TNW; ++t) {
        const int n = wn * (BN / WN) + t * 16 + fi;
        double x0, x1, x2, x3;
        if (BT) {
          const dbl2v p0 = *(const dbl2v *)&bs[n * BK + (((2 * fk) ^ (n % CH)) << 1)];
          const dbl2v p1 = *(const dbl2v *)&bs[n * BK + (((2 * fk + 1) ^ (n % CH)) << 1)];
          x0 = p0[0]; x1 = p0[1]; x2 = p1[0]; x3 = p1[1];
        } else {
          x0 = bs[(4 * fk) * BN + n]; x1 = bs[(4 * fk + 1) * BN + n];
          x2 = bs[(4 * fk + 2) * BN + n]; x3 = bs[(4 * fk + 3) * BN + n];
        }
        sb[t] = split4<CP>(x0, x1, x2, x3);
      }
#pragma unroll
      for (int a = 0; a < TMW; ++a)
#pragma unroll
        for (int b = 0; b < TNW; ++b) acc[a][b] = mfma_split<CP>(sa[a], sb[b], acc[a][b]);
    } else {
#pragma unroll
      for (int u = 0; u < BK / 8; ++u) {
        const int g = 4 * u + fk;      // this lane's 16-byte chunk along k: k = 2g and 2g + 1
        const int k0 = 2 * g;
        dbl2v af[TMW], bf[TNW];
#pragma unroll
        for (int t = 0; t < TMW; ++t) {
          const int m = wm * (BM / WM) + t * 16 + fi;
          if (AT) af[t] = dbl2v{as[k0 * BM + m], as[(k0 + 1) * BM + m]};
          else af[t] = *(const dbl2v *)&as[m * BK + ((g ^ (m % CH)) << 1)];
        }
#pragma unroll
        for (int t = 0; t < TNW; ++t) {
          const int n = wn * (BN / WN) + t * 16 + fi;
          if (BT) bf[t] = *(const dbl2v *)&bs[n * BK + ((g ^ (n % CH)) << 1)];
          else bf[t] = dbl2v{bs[k0 * BN + n], bs[(k0 + 1) * BN + n]};
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int a = 0; a < TMW; ++a)
#pragma unroll
            for (int b = 0; b < TNW; ++b)
              acc[a][b] = MM::step(af[a][h], bf[b][h], acc[a][b]);
      }
    }
  }

  const double alpha = p.alpha, beta = p.beta;
#pragma unroll
  for (int a = 0; a < TMW; ++a)
#pragma unroll
    for (int b = 0; b < TNW; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gm = m0 + wm * (BM / WM) + a * 16 + MM::row(lane, i);
        const int gn = n0 + wn * (BN / WN) + b * 16 + (lane & 15);
        double v = alpha * (double)acc[a][b][i];
        if (beta != 0.0) v += beta * p.Cin[(int64_t)gm * p.ldcin + gn];
        Cout[(int64_t)(gm - cm0) * p.ldc + (gn - cn0)] = v;
        if (p.Cm) p.Cm[(int64_t)gn * p.ldcm + gm] = v;
      }
  }  // pieces
}

// The same sum for many splits of a small output: each element is shared by RG_GROUPS threads,
// thread g summing splits g, g + RG_GROUPS, g + 2 RG_GROUPS, ... in that order, and the group sums
// are then added in group order; the order is fixed, so the result is bitwise reproducible.
// Blocks of 256 threads cover 256 / RG_GROUPS consecutive elements.
constexpr int RG_GROUPS = 8;
constexpr int RG_ELEMS = 256 / RG_GROUPS;
__global__ __launch_bounds__(256) void reduce_splits_grouped_kernel(int M, int N, const double *P, int64_t ldp,
                                                                    int64_t sstride, int S, double alpha,
                                                                    const double *Cin, int64_t ldcin,
                                                                    double beta, double *C, int64_t ldc,
                                                                    double *Cm, int64_t ldcm, int lower_only) {
  __shared__ double red[RG_GROUPS][RG_ELEMS];
  const int el = threadIdx.x % RG_ELEMS, g = threadIdx.x / RG_ELEMS;
  const int64_t total = (int64_t)M * N;
  for (int64_t e0 = (int64_t)blockIdx.x * RG_ELEMS; e0 < total; e0 += (int64_t)gridDim.x * RG_ELEMS) {
    const int64_t e = e0 + el;
    double s = 0.0;
    if (e < total) {
      const int m = (int)(e / N), n = (int)(e % N);
      const double *src = P + (int64_t)m * ldp + n;
      int z = g;
      for (; z + 3 * RG_GROUPS < S; z += 4 * RG_GROUPS) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = src[(int64_t)(z + u * RG_GROUPS) * sstride];
#pragma unroll
        for (int u = 0; u < 4; ++u) s += v[u];
      }
      for (; z < S; z += RG_GROUPS) s += src[(int64_t)z * sstride];
    }
    red[g][el] = s;
    __syncthreads();
    if (g == 0 && e < total) {
      const int m = (int)(e / N), n = (int)(e % N);
      double t = red[0][el];
#pragma unroll
      for (int q = 1; q < RG_GROUPS; ++q) t += red[q][el];
      if (!(lower_only && n > m)) {
        double v = alpha * t;
        if (beta != 0.0) v += beta * Cin[(int64_t)m * ldcin + n];
        C[(int64_t)m * ldc + n] = v;
        if (Cm) Cm[(int64_t)n * ldcm + m] = v;
      }
    }
    __syncthreads();
  }
}

// C[m, n] = alpha * sum_{s < S} P[s*sstride + m*ldp + n] + beta * Cin[m, n], summed in split order;
// lower_only restricts the writes to n <= m.  Optional transposed copy Cm as in the GEMM.  Eight
// partial loads are kept in flight per thread; the additions stay in split order, so the result
// is bitwise reproducible.
__global__ __launch_bounds__(256) void reduce_splits_kernel(int M, int N, const double *P, int64_t ldp,
                                                            int64_t sstride, int S, double alpha,
                                                            const double *Cin, int64_t ldcin,
                                                            double beta, double *C, int64_t ldc,
                                                            double *Cm, int64_t ldcm, int lower_only) {
  const int64_t total = (int64_t)M * N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int m = (int)(e / N), n = (int)(e % N);
    if (lower_only && n > m) continue;
    const double *src = P + (int64_t)m * ldp + n;
    double s = 0.0;
    int z = 0;
    for (; z + 8 <= S; z += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = src[(int64_t)(z + u) * sstride];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; z < S; ++z) s += src[(int64_t)z * sstride];
    double v = alpha * s;
    if (beta != 0.0) v += beta * Cin[(int64_t)m * ldcin + n];
    C[(int64_t)m * ldc + n] = v;
    if (Cm) Cm[(int64_t)n * ldcm + m] = v;
  }
}

// Sum of the stream-K pieces: element (m, n) lies in tile t = m / 128 + (n / 128) tm, whose units
// [t KT, (t+1) KT) were taken by workgroups wf .. wl (w takes [w T / W, (w+1) T / W)); their partial
// slots w + t are added in workgroup order, so the result is bitwise reproducible.
__global__ __launch_bounds__(256) void reduce_streamk_kernel(int M, int N, int bn, const double *P,
                                                             int64_t sstride, int64_t W, int64_t KT, int tm,
                                                             double alpha, const double *Cin, int64_t ldcin,
                                                             double beta, double *C, int64_t ldc, double *Cm,
                                                             int64_t ldcm) {
  const int64_t total = (int64_t)M * N;
  const int64_t T = KT * tm * ((N + bn - 1) / bn);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int m = (int)(e / N), n = (int)(e % N);
    const int64_t t = m / GEMM_BM + (int64_t)(n / bn) * tm;
    // last workgroup whose range starts at or before unit x: floor(((x + 1) W - 1) / T)
    const int64_t wf = ((t * KT + 1) * W - 1) / T;
    const int64_t wl = (((t + 1) * KT) * W - 1) / T;
    const double *src = P + (wf + t) * sstride + (int64_t)(m % GEMM_BM) * bn + (n % bn);
    double s = 0.0;
    for (int64_t w = wf; w <= wl; ++w, src += sstride) s += *src;
    double v = alpha * s;
    if (beta != 0.0) v += beta * Cin[(int64_t)m * ldcin + n];
    C[(int64_t)m * ldc + n] = v;
    if (Cm) Cm[(int64_t)n * ldcm + m] = v;
  }
}

}  // namespace cg
