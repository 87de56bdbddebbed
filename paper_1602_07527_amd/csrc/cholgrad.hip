// libcholgrad: C ABI and host-side enqueuer for blocked Cholesky factorisation and blocked
// forward/reverse propagation of Cholesky derivatives on gfx950 (Murray 2016, Sec. 4.2).
//
// The host code only validates arguments, carves the caller's workspace and enqueues kernels on
// the caller's stream; every arithmetic step runs on the GPU.  Block columns are tile-aligned
// ([b*nb, min(n, (b+1)*nb))), so a short block, if any, is the last one in both sweeps; the
// column partition is arbitrary (Sec. 4.2), so this does not change the result beyond rounding.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>

#include <algorithm>
#include <cstddef>
#include <mutex>
#include <vector>

#include "cholgrad.h"
#include "cg_batched.hpp"
#include "cg_batched2.hpp"
#include "cg_diag.hpp"
#include "cg_gemm.hpp"

namespace {

constexpr size_t WS_ALIGN = 256;
constexpr int NOALLOC_DEFAULT_NB = 128;  // nb = 0 in chol_rev_noalloc
constexpr int FACTOR_ONE_STREAM_BLOCKS = 3;  // chol_factor sweeps this short skip the side stream
constexpr int TARGET_WGS = 512;  // two contraction workgroups per compute unit on 256 CUs
// Workgroups of a stream-K contraction in a sweep with a side stream: a little below the 512
// resident slots.  The diagonal block kernels of such a sweep run beside the contractions and
// hold most of a compute unit's LDS; with more workgroups than this, some of them wait for a slot
// until that kernel ends (measured on MI355X in the N = 16384 sweeps: 480 beats 448, 464, 496 and
// 504).  Short launches (under SK_SHORT_KTILES K-tiles per workgroup) lose the most to such a
// wait, and take SK_WGS_SHORT workgroups (chol_rev 64.9 -> 64.2 ms, chol_factor 39.6 -> 38.8 ms,
// same GPU).  A sweep whose products run alone on its stream (the symbolic diagonal block) takes
// all TARGET_WGS slots: N = 16384, nb = 256 chol_rev 53.3 -> 51.0 ms, nb = 128 chol_fwd 56.7 ->
// 54.6 ms, while chol_factor, with POTF2 beside, goes 35.5 -> 40.6 ms at 512.
constexpr int SK_WGS = 480;
constexpr int SK_WGS_SHORT = 448;
// 128 x 256-tile contractions hold one workgroup per compute unit.  Beside a side stream they take
// 248 workgroups, one compute unit per XCD left for the side stream's kernels (N = 16384 nb = 256
// chol_factor: 32.8 ms at 240, 32.2 at 248, 32.5 at 244, 37.7 at 252 and 37.6 at 256, where a
// stream-K workgroup waits for a compute unit held by POTF2).
constexpr int SK_WGS_WIDE = 248;
constexpr int64_t SK_SHORT_KTILES = 48;
constexpr int64_t PART_SLOTS = 2 * TARGET_WGS;  // 128 x 128 partial tiles per buffer
constexpr bool WIDE_TILES = true;               // 128 x 256 tiles for the 256-wide sweep contractions
constexpr int64_t TILE_ELEMS = (int64_t)cg::GEMM_BM * cg::GEMM_BN;

// A buffer of 128 x 128 partial tiles for split-K and stream-K products: base and capacity in
// tiles.  A null buffer forbids splitting.
struct PartBuf {
  double *p = nullptr;
  int64_t slots = 0;
  int sk_wgs = 0;  // stream-K workgroups when set (nothing else of the sweep runs beside)
  PartBuf() = default;
  PartBuf(std::nullptr_t) {}
  PartBuf(double *base, int64_t n) : p(base), slots(base ? n : 0) {}
};

// Benchmark instrumentation: event pairs around the panel contractions, per sweep (see
// chol_profile_begin).  Process-global and not thread-safe; off unless a benchmark enables it.
struct Profile {
  bool on = false;
  int cap = 0;
  std::vector<hipEvent_t> ev;   // 2 per launch
  std::vector<int> klass;
  std::vector<double> flops;
  std::vector<double> bytes;
  int used = 0;
};
Profile g_prof;

inline size_t align_up(size_t x) { return (x + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Workspace carving: the same function sizes (base == nullptr) and assigns.
struct Carver {
  char *base;
  size_t off = 0;
  explicit Carver(void *b) : base(static_cast<char *>(b)) {}
  double *take(size_t n_doubles) {
    const size_t o = off;
    off = align_up(off + n_doubles * sizeof(double));
    return base ? reinterpret_cast<double *>(base + o) : nullptr;
  }
};

struct SweepWs {
  double *dinv = nullptr;   // inverses of the diagonal blocks of L: nblk x nb x nb
  double *panel = nullptr;  // one block column: n x nb
  double *dblk = nullptr;   // one diagonal block: nb x nb
  PartBuf part;             // split-K partial tiles of the main stream
  PartBuf part2;            // split-K partial tiles of the side stream
  double *tmp = nullptr;    // two nb x nb blocks for the symbolic diagonal-block variants
};

// part_slots / part2_slots: capacity of the two partial-tile buffers (PART_SLOTS by default; the
// allocation-free entry point carves a smaller main buffer and no side buffer).
size_t carve(int64_t n, int nb, void *base, SweepWs *w, int64_t part_slots = PART_SLOTS,
             int64_t part2_slots = PART_SLOTS) {
  Carver c(base);
  const int64_t nblk = cdiv(n, nb);
  w->dinv = c.take((size_t)nblk * nb * nb);
  w->panel = c.take((size_t)n * nb);
  w->dblk = c.take((size_t)nb * nb);
  w->part = PartBuf(c.take((size_t)(part_slots * TILE_ELEMS)), part_slots);
  w->part2 = PartBuf(c.take((size_t)(part2_slots * TILE_ELEMS)), part2_slots);
  w->tmp = c.take((size_t)2 * nb * nb);
  return c.off;
}

// Side streams for look-ahead: the diagonal-block chain of one step runs there while the next
// step's bulk contraction runs on the caller's stream.  One side stream (default priority,
// non-blocking) and five events per (device, calling stream) pair, for up to SIDES_PER_DEVICE
// calling streams per device; further calling streams share those slots round-robin, which only
// costs overlap.  Created on first use and kept for the life of the process.  The mutex
// serialises whole enqueue sequences, and every event wait of a call refers to a record made
// earlier in the same call, so sharing a slot never mixes two calls' dependencies.
struct Side {
  hipStream_t s = nullptr;
  hipEvent_t start = nullptr, panel = nullptr, diag = nullptr, top = nullptr, low = nullptr;
};
constexpr int MAX_DEVICES = 64;
constexpr int SIDES_PER_DEVICE = 8;
struct SideSlot {
  bool used = false;
  hipStream_t caller = nullptr;
  Side side;
};
std::mutex g_side_mu;
SideSlot g_sides[MAX_DEVICES][SIDES_PER_DEVICE];
int g_side_next[MAX_DEVICES];

hipError_t side_for(hipStream_t caller, Side **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  SideSlot *slot = nullptr;
  for (int i = 0; i < SIDES_PER_DEVICE && !slot; ++i)
    if (g_sides[dev][i].used && g_sides[dev][i].caller == caller) slot = &g_sides[dev][i];
  for (int i = 0; i < SIDES_PER_DEVICE && !slot; ++i)
    if (!g_sides[dev][i].used) slot = &g_sides[dev][i];
  if (!slot) {  // every slot taken by other calling streams: share one
    slot = &g_sides[dev][g_side_next[dev]];
    g_side_next[dev] = (g_side_next[dev] + 1) % SIDES_PER_DEVICE;
  }
  Side &sd = slot->side;
  if (!sd.s) {
    if ((e = hipStreamCreateWithFlags(&sd.s, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&sd.start, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&sd.panel, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&sd.diag, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&sd.top, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&sd.low, hipEventDisableTiming)) != hipSuccess) return e;
  }
  if (!slot->used) {
    slot->used = true;
    slot->caller = caller;
  }
  *out = &sd;
  return hipSuccess;
}

// Precision modes of the single-matrix sweeps (FP64 storage): the trailing contractions run on
// FP64, FP32 or split-bfloat16 MFMA; diagonal blocks and panel solves are FP64 in all of them.
bool single_prec(int precision, int *cp) {
  if (precision == CHOL_PREC_F64) { *cp = cg::CP_F64; return true; }
  if (precision == CHOL_PREC_F64_TRAIL_F32) { *cp = cg::CP_F32; return true; }
  if (precision == CHOL_PREC_F64_TRAIL_BF16X3) { *cp = cg::CP_BF16X3; return true; }
  if (precision == CHOL_PREC_F64_TRAIL_BF16X6) { *cp = cg::CP_BF16X6; return true; }
  return false;
}

// Block widths: multiples of 16 up to 256.  Blocks wider than 128 (the widest diagonal block the
// LDS routines hold) factor and invert their diagonal block as two halves (potf2_any, trinv).
constexpr int NB_MAX = 2 * cg::DIAG_MAX;
bool nb_ok(int nb) { return nb == 0 || (nb >= 16 && nb <= NB_MAX && nb % 16 == 0); }

// The block width nb = 0 stands for, per sweep and size: the fastest of nb = 64, 128 and 256 in
// event timings of the three sweeps on squared-exponential matrices, n = 256 to 16384, on one
// MI355X.  chol_rev: 256 at every size (n = 4096: 2.00 ms against 2.66 at 128).  chol_fwd: 256 at
// every size (n = 12288: 23.6 ms against 25.7 at 128; n = 16384: 50.9 against 54.2).
// chol_factor: 128, except 256 for n in (256, 512] (two blocks on one stream: n = 512, 430 us
// against 496) and from n = 3072 up (n = 8192: 9.6 ms against 10.3).  chol_factor_fwd takes the
// factor's choice.  The Level-2 diagonal variant holds blocks of at most 128.  A workspace query
// with nb = 0 sizes for NB_MAX, which holds every one of these.
int auto_nb(int op, int64_t n, bool level2 = false) {
  int nb;
  if (op == CHOL_OP_REV) nb = NB_MAX;
  else if (op == CHOL_OP_FWD) nb = NB_MAX;
  else nb = ((n > 256 && n <= 512) || n >= 3072) ? NB_MAX : 128;
  return level2 ? std::min(nb, (int)cg::DIAG_MAX) : nb;
}
bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

template <int TAG, int CP>
void launch_gemm_tag(bool at, bool bt, bool fast, bool wide, dim3 grid, const cg::GemmArgs &p, hipStream_t s) {
  if constexpr (CP == cg::CP_F64 && (TAG == 0 || TAG == 3)) {
    if (fast && wide && p.A2 && !at && bt) {  // paired forward-sweep products on 128 x 256 tiles
      hipLaunchKernelGGL((cg::gemm_f64_dma_kernel<false, true, TAG, CP, true, true>), grid, dim3(cg::DMA_THREADS), 0, s, p);
      return;
    }
  }
  if constexpr (CP == cg::CP_F64 && (TAG == 1 || TAG == 2)) {
    if (fast && wide) {  // 128 x 256 output tiles (gemm() allows them only here, for A and B row-major or B^T)
      const dim3 block(cg::DMA_THREADS);
      if (!at && bt) hipLaunchKernelGGL((cg::gemm_f64_dma_kernel<false, true, TAG, CP, false, true>), grid, block, 0, s, p);
      else hipLaunchKernelGGL((cg::gemm_f64_dma_kernel<false, false, TAG, CP, false, true>), grid, block, 0, s, p);
      return;
    }
  }
  if (fast && p.A2) {  // paired products (the forward sweep's symmetric updates: B transposed)
    const dim3 block(cg::DMA_THREADS);
    if (!at && bt) hipLaunchKernelGGL((cg::gemm_f64_dma_kernel<false, true, TAG, CP, true>), grid, block, 0, s, p);
    else if (at && !bt) hipLaunchKernelGGL((cg::gemm_f64_dma_kernel<true, false, TAG, CP, true>), grid, block, 0, s, p);
    else if (!at && !bt) hipLaunchKernelGGL((cg::gemm_f64_dma_kernel<false, false, TAG, CP, true>), grid, block, 0, s, p);
    else hipLaunchKernelGGL((cg::gemm_f64_dma_kernel<true, true, TAG, CP, true>), grid, block, 0, s, p);
    return;
  }
  if (fast) {
    const dim3 block(cg::DMA_THREADS);
    if (at && !bt) hipLaunchKernelGGL((cg::gemm_f64_dma_kernel<true, false, TAG, CP>), grid, block, 0, s, p);
    else if (!at && bt) hipLaunchKernelGGL((cg::gemm_f64_dma_kernel<false, true, TAG, CP>), grid, block, 0, s, p);
    else if (!at && !bt) hipLaunchKernelGGL((cg::gemm_f64_dma_kernel<false, false, TAG, CP>), grid, block, 0, s, p);
    else hipLaunchKernelGGL((cg::gemm_f64_dma_kernel<true, true, TAG, CP>), grid, block, 0, s, p);
    return;
  }
  const dim3 block(cg::GEMM_THREADS);
  if (at && !bt) hipLaunchKernelGGL((cg::gemm_f64_kernel<true, false, TAG, CP>), grid, block, 0, s, p);
  else if (!at && bt) hipLaunchKernelGGL((cg::gemm_f64_kernel<false, true, TAG, CP>), grid, block, 0, s, p);
  else if (!at && !bt) hipLaunchKernelGGL((cg::gemm_f64_kernel<false, false, TAG, CP>), grid, block, 0, s, p);
  else hipLaunchKernelGGL((cg::gemm_f64_kernel<true, true, TAG, CP>), grid, block, 0, s, p);
}

template <int CP>
void launch_gemm_cp(bool at, bool bt, bool fast, bool wide, int tag, dim3 grid, const cg::GemmArgs &p,
                    hipStream_t s) {
  switch (tag) {
    case 1: launch_gemm_tag<1, CP>(at, bt, fast, wide, grid, p, s); break;
    case 2: launch_gemm_tag<2, CP>(at, bt, fast, wide, grid, p, s); break;
    case 3: launch_gemm_tag<3, CP>(at, bt, fast, wide, grid, p, s); break;
    default: launch_gemm_tag<0, CP>(at, bt, fast, wide, grid, p, s); break;
  }
}

void launch_gemm(bool at, bool bt, bool fast, bool wide, int tag, int cp, dim3 grid, const cg::GemmArgs &p,
                 hipStream_t s) {
  if (cp == cg::CP_F32) launch_gemm_cp<cg::CP_F32>(at, bt, fast, wide, tag, grid, p, s);
  else if (cp == cg::CP_BF16X3) launch_gemm_cp<cg::CP_BF16X3>(at, bt, fast, wide, tag, grid, p, s);
  else if (cp == cg::CP_BF16X6) launch_gemm_cp<cg::CP_BF16X6>(at, bt, fast, wide, tag, grid, p, s);
  else launch_gemm_cp<cg::CP_F64>(at, bt, fast, wide, tag, grid, p, s);
}

bool aligned16(const void *ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 15u) == 0; }

// C = alpha * op(A) op(B) + beta * Cin on the MFMA kernel; splits K when the output has too few
// tiles to fill the GPU, then sums the partial tiles in split order.  part == nullptr forbids
// splitting.
// Optional second operand pair of a contraction (same shapes and transposition as the first).
struct Pair2 {
  const double *A2 = nullptr;
  int64_t lda2 = 0;
  const double *B2 = nullptr;
  int64_t ldb2 = 0;
};

bool dma_ld_ok(int64_t ld) { return ld % 2 == 0 && ld < ((int64_t)1 << 21); }

hipError_t gemm(bool at, bool bt, int M, int N, int K, const double *A, int64_t lda,
                const double *B, int64_t ldb, double alpha, const double *Cin, int64_t ldcin,
                double beta, double *C, int64_t ldc, double *Cm, int64_t ldcm, int lower_only,
                PartBuf part, int min_kchunk, hipStream_t s, int tag = 0, int cp = cg::CP_F64,
                Pair2 q = Pair2()) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int Kt = q.A2 ? 2 * K : K;  // combined K range
  // The direct-to-LDS kernel needs whole 128 x 128 output tiles, whole 16-deep K-tiles in every
  // split (and in each operand pair), even leading dimensions below 2^21 (32-bit lane offsets)
  // and 16-byte aligned operands (its 16-byte loads never cross the matrix); everything else
  // takes the general kernel, which guards every access.
  const bool fast = (M % cg::GEMM_BM == 0) && (N % cg::GEMM_BN == 0) && (K > 0) && (K % cg::DMA_BK == 0) &&
                    dma_ld_ok(lda) && dma_ld_ok(ldb) && aligned16(A) && aligned16(B) &&
                    (!q.A2 || (dma_ld_ok(q.lda2) && dma_ld_ok(q.ldb2) && aligned16(q.A2) && aligned16(q.B2)));
  // 128 x 256 output tiles (one workgroup per compute unit) for the FP64 sweep contractions whose
  // output is one 256-wide column of tiles: each K-tile of the tall operand is loaded once for
  // both halves.  Paired products with B transposed take them in a sweep with no side stream (the
  // symbolic forward sweep): the two pairs run one after the other along K, so the tiles in LDS
  // are those of one product (N = 16384 chol_fwd at nb = 256: 56.6 -> 50.9 ms with its panel solve
  // below).  Beside a side stream (chol_factor_fwd) they were slower: 86.0 -> 88.5 ms.
  const bool wide = WIDE_TILES && fast && !lower_only && !at && N == 2 * cg::GEMM_BN && cp == cg::CP_F64 &&
                    ((!q.A2 && (tag == 1 || tag == 2)) || (q.A2 && bt && part.sk_wgs != 0));
  const int bn = wide ? 2 * cg::GEMM_BN : cg::GEMM_BN;
  const int tm = (int)cdiv(M, cg::GEMM_BM), tn = (int)cdiv(N, bn);
  int tiles = tm * tn;
  if (lower_only && tm == tn) tiles = (tm * (tm + 1)) / 2;
  const int64_t slots = part.slots / (bn / cg::GEMM_BN);  // partial tiles of this product's size
  const int kstep = fast ? cg::DMA_BK : cg::GEMM_BK;
  // Stream-K on the fast kernel when the output has too few tiles: SK_WGS (or SK_WGS_SHORT)
  // workgroups take equal shares of the (tile, K-tile) units, each piece deep enough
  // (>= min_kchunk) to be worth a partial tile; the pieces are then summed per tile in workgroup
  // order.
  int64_t skw = 0;
  if (part.p && fast && !lower_only && Kt > 0 && tiles >= 2) {
    const int64_t units = (int64_t)tiles * (Kt / cg::DMA_BK);
    skw = part.sk_wgs ? part.sk_wgs : (units < SK_SHORT_KTILES * SK_WGS ? SK_WGS_SHORT : SK_WGS);
    if (wide) skw = part.sk_wgs ? skw / 2 : SK_WGS_WIDE;  // one wide-tile workgroup per compute unit
    skw = std::min<int64_t>(skw, units * cg::DMA_BK / std::max(min_kchunk, cg::DMA_BK));
    skw = std::min<int64_t>(skw, slots - tiles + 1);
    if (skw <= tiles) skw = 0;
  }
  int S = 1;
  int kchunk = (int)(cdiv(Kt > 0 ? Kt : 1, kstep) * kstep);
  if (part.p && Kt > 0 && !skw) {
    int64_t s_want = (wide ? TARGET_WGS / 2 : TARGET_WGS) / tiles;
    s_want = std::min<int64_t>(s_want, cdiv(Kt, min_kchunk));
    s_want = std::min<int64_t>(s_want, part.slots * TILE_ELEMS / ((int64_t)M * N));
    if (s_want > 1) {
      kchunk = (int)(cdiv(cdiv(Kt, s_want), kstep) * kstep);
      S = (int)cdiv(Kt, kchunk);
    }
  }
  cg::GemmArgs p;
  p.M = M; p.N = N; p.K = K;
  p.A = A; p.lda = lda; p.B = B; p.ldb = ldb;
  p.A2 = q.A2; p.lda2 = q.A2 ? q.lda2 : 0; p.B2 = q.A2 ? q.B2 : nullptr; p.ldb2 = q.A2 ? q.ldb2 : 0;
  p.kchunk = kchunk;
  p.lower_only = lower_only;
  const dim3 grid = skw ? dim3((unsigned)skw, 1, 1) : dim3(tm, tn, S);
  if (skw) {
    p.C = part.p; p.ldc = bn; p.Cin = nullptr; p.ldcin = 0; p.alpha = 1.0; p.beta = 0.0;
    p.Cm = nullptr; p.ldcm = 0; p.split_stride = (int64_t)cg::GEMM_BM * bn;
    p.sk_wgs = (int)skw; p.sk_kt = Kt / cg::DMA_BK; p.sk_tm = tm; p.sk_tiles = tiles;
  } else if (S == 1) {
    p.C = C; p.ldc = ldc; p.Cin = Cin; p.ldcin = ldcin; p.alpha = alpha; p.beta = beta;
    p.Cm = Cm; p.ldcm = ldcm; p.split_stride = 0;
  } else {
    p.C = part.p; p.ldc = N; p.Cin = nullptr; p.ldcin = 0; p.alpha = 1.0; p.beta = 0.0;
    p.Cm = nullptr; p.ldcm = 0; p.split_stride = (int64_t)M * N;
  }
  const bool timed = g_prof.on && tag > 0 && g_prof.used < g_prof.cap;
  if (timed) {
    const int u = g_prof.used;
    if (hipEventRecord(g_prof.ev[2 * u], s) != hipSuccess) return hipErrorUnknown;
    g_prof.klass[u] = tag;
    g_prof.flops[u] = 2.0 * (double)M * (double)N * (double)Kt;
    // Algorithmic HBM bytes of the contraction: read op(A), op(B) and Cin once, write C (and
    // its mirror) once; split-K partials are not counted.
    const double mn = (double)M * (double)N * (lower_only ? 0.5 : 1.0);
    g_prof.bytes[u] = 8.0 * ((double)M * Kt + (double)Kt * N + mn * ((beta != 0.0 ? 2.0 : 1.0) + (Cm ? 1.0 : 0.0)));
  }
  launch_gemm(at, bt, fast, wide, tag, cp, grid, p, s);
  if (timed) {
    if (hipEventRecord(g_prof.ev[2 * g_prof.used + 1], s) != hipSuccess) return hipErrorUnknown;
    ++g_prof.used;
  }
  hipError_t e = hipGetLastError();
  const int64_t total = (int64_t)M * N;
  if (e == hipSuccess && skw) {
    const int blocks = (int)std::min<int64_t>(cdiv(total, 256), 4096);
    hipLaunchKernelGGL(cg::reduce_streamk_kernel, dim3(blocks), dim3(256), 0, s, M, N, bn, (const double *)part.p,
                       (int64_t)cg::GEMM_BM * bn, skw, (int64_t)(Kt / cg::DMA_BK), tm, alpha,
                       Cin, ldcin, beta, C, ldc, Cm, ldcm);
    return hipGetLastError();
  }
  if (e != hipSuccess || S == 1) return e;
  if (S >= 4 * cg::RG_GROUPS && total <= (int64_t)64 * 1024) {  // many splits of a small output
    const int blocks = (int)std::min<int64_t>(cdiv(total, cg::RG_ELEMS), 4096);
    hipLaunchKernelGGL(cg::reduce_splits_grouped_kernel, dim3(blocks), dim3(256), 0, s, M, N, (const double *)part.p,
                       (int64_t)N, (int64_t)M * N, S, alpha, Cin, ldcin, beta, C, ldc, Cm, ldcm,
                       lower_only);
    return hipGetLastError();
  }
  const int blocks = (int)std::min<int64_t>(cdiv(total, 256), 4096);
  hipLaunchKernelGGL(cg::reduce_splits_kernel, dim3(blocks), dim3(256), 0, s, M, N, (const double *)part.p, (int64_t)N,
                     (int64_t)M * N, S, alpha, Cin, ldcin, beta, C, ldc, Cm, ldcm, lower_only);
  return hipGetLastError();
}

// dst[0:M, 0:N] = beta * src (lower triangle only when lower_only), as a split-free reduce.
hipError_t copy_scaled(int M, int N, const double *src, int64_t lds, double beta, double *dst,
                       int64_t ldd, int lower_only, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(cdiv((int64_t)M * N, 256), 2048);
  hipLaunchKernelGGL(cg::reduce_splits_kernel, dim3(blocks), dim3(256), 0, s, M, N,
                     (const double *)nullptr, (int64_t)0, (int64_t)0, 0, 0.0, src, lds, beta, dst,
                     ldd, (double *)nullptr, (int64_t)0, lower_only);
  return hipGetLastError();
}


// Inverses of all diagonal blocks of L into dinv (nblk blocks of nb x nb, ld nb), on stream s.  For
// nb > 128 each block's two halves are inverted separately and the lower-left part follows from
// them (inv_offdiag_kernel), with T (>= ceil(n / nb) * 128 * 128 doubles) as scratch.
hipError_t block_inverses(int64_t n, int nb, const double *L, int64_t ldl, double *dinv, double *T,
                          hipStream_t s) {
  const int64_t nblk = cdiv(n, nb);
  const bool halves = nb > cg::DIAG_MAX;
  hipLaunchKernelGGL(cg::trinv_kernel, dim3((unsigned)(halves ? 2 * nblk : nblk)), dim3(cg::DIAG_THREADS), 0, s, n,
                     nb, L, ldl, dinv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !halves) return e;
  for (int phase = 0; phase < 2; ++phase) {
    hipLaunchKernelGGL(cg::inv_offdiag_kernel, dim3((unsigned)(nblk * 64)), dim3(256), 0, s, phase, n, nb, L, ldl,
                       dinv, T);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// D <- chol_unblocked(D) (POTF2) for the w x w diagonal block at Ad, in place, and D^-1 into dinv
// (ld nb), on stream s.  w <= 128: one potf2_kernel.  128 < w <= 256: the block factored as two
// halves, as Sec. 4.2's blocked algorithm with a smaller block (the paper suggests a recursive
// routine in place of the unblocked one for large blocks): POTF2 of the first half, the panel
// solve D10 <- D10 X00^T and the update D11 <- D11 - D10 D10^T as MFMA products, POTF2 of the
// second half, then the lower-left part of the inverse (T: 128 * 128 doubles of scratch).  With
// need_inv false (the last block of chol_factor, which has no rows below to solve) D^-1 is not
// formed, except the first half's, which the second half's panel solve takes (N = 256, nb = 128:
// the 128-block inverse is about 20 us of each POTF2).
hipError_t potf2_any(int w, double *Ad, int64_t lda, double *dinv, int nb, int *info, int64_t col0, double *T,
                     PartBuf part, hipStream_t s, bool need_inv = true) {
  const int h1 = std::min(w, cg::DIAG_MAX);
  hipLaunchKernelGGL(cg::potf2_kernel, dim3(1), dim3(cg::DIAG_THREADS), 0, s, h1, Ad, lda, dinv, (int64_t)nb,
                     std::min(nb, cg::DIAG_MAX), w - h1, info, col0, (need_inv || w > h1) ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || w <= cg::DIAG_MAX) return e;
  const int h2 = w - h1;
  double *A10 = Ad + (int64_t)h1 * lda, *A11 = A10 + h1;
  // D10 <- D10 X00^T (in place: the output is one 128-wide tile column)
  if ((e = gemm(false, true, h2, h1, h1, A10, lda, dinv, nb, 1.0, nullptr, 0, 0.0, A10, lda, nullptr, 0, 0, part,
                32, s)) != hipSuccess)
    return e;
  // D11 <- D11 - D10 D10^T
  if ((e = gemm(false, true, h2, h2, h1, A10, lda, A10, lda, -1.0, A11, lda, 1.0, A11, lda, nullptr, 0, 0, part, 32,
                s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(cg::potf2_kernel, dim3(1), dim3(cg::DIAG_THREADS), 0, s, h2, A11, lda,
                     dinv + (int64_t)h1 * nb + h1, (int64_t)nb, h2, 0, info, col0 + h1, need_inv ? 1 : 0);
  if ((e = hipGetLastError()) != hipSuccess || !need_inv) return e;
  for (int phase = 0; phase < 2; ++phase) {
    hipLaunchKernelGGL(cg::inv_offdiag_kernel, dim3(64), dim3(256), 0, s, phase, (int64_t)w, nb,
                       (const double *)Ad, lda, dinv, T);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// C <- C D^-T for the M x w panel C (ldc) with D^-1 in dinv (ld nb): in place when w <= 128 (each
// output tile spans every column, so its workgroup reads its rows before writing them), through
// the buffer `tmp` (M x w, ld nb) otherwise (measured faster than two in-place launches over the
// column halves: N = 16384, nb = 256 chol_factor 33.1 against 34.3 ms).
hipError_t panel_solve_t(int M, int w, double *C, int64_t ldc, const double *dinv, int nb, double *tmp,
                         PartBuf part, int min_kchunk, hipStream_t s) {
  if (M <= 0) return hipSuccess;
  if (w <= cg::GEMM_BN)
    return gemm(false, true, M, w, w, C, ldc, dinv, nb, 1.0, nullptr, 0, 0.0, C, ldc, nullptr, 0, 0, part,
                min_kchunk, s);
  hipError_t e = gemm(false, true, M, w, w, C, ldc, dinv, nb, 1.0, nullptr, 0, 0.0, tmp, nb, nullptr, 0, 0, part,
                      min_kchunk, s);
  if (e != hipSuccess) return e;
  return copy_scaled(M, w, tmp, nb, 1.0, C, ldc, 0, s);
}

// The reverse sweep's D-bar <- tril(L-bar_D) - tril(C-bar^T C) (w x w output, K = m), with C-bar/2
// in Cb: FP64 blocks wider than 128 take the 64 x 64-tile split-K kernel (10 lower tiles at w = 256,
// about SYRK_WGS workgroups, K-splits at least 64 deep) and the grouped fixed-order split sum; the
// 128 x 128-tile product left them with too few workgroups or too much partial data (measured at
// w = 256 on MI355X: 22.5 us per step on average against 29.1, 36.7 us at m = 16128 against 50;
// N = 16384 chol_rev 50.4 -> 49.8 ms); everything else the general product.
constexpr int SYRK_WGS = 480;  // workgroups of the 64-tile SYRK (measured: 960 and 1920 slower)

hipError_t rev_syrk(int w, int m, const double *Cb, int64_t ldcb, const double *Lc, int64_t ldl, const double *Ld,
                    int64_t ldd, double *dblk, int nb, PartBuf part, hipStream_t s, int cp) {
  const int nt = (int)cdiv(w, cg::B2_NB), ntiles = nt * (nt + 1) / 2;
  if (w > cg::GEMM_BN && cp == cg::CP_F64 && part.p) {
    int S = std::max(1, std::min<int>(SYRK_WGS / ntiles, (int)cdiv(m, 64)));
    S = (int)std::min<int64_t>(S, part.slots * TILE_ELEMS / ((int64_t)w * w));
    const int kchunk = (int)cdiv(m, S);
    S = (int)cdiv(m, kchunk);
    hipLaunchKernelGGL(cg::syrk_t64_kernel, dim3((unsigned)(ntiles * S)), dim3(256), 0, s, m, w, Cb, ldcb, Lc, ldl,
                       kchunk, part.p);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int blocks = (int)std::min<int64_t>(cdiv((int64_t)w * w, cg::RG_ELEMS), 4096);
    hipLaunchKernelGGL(cg::reduce_splits_grouped_kernel, dim3(blocks), dim3(256), 0, s, w, w, (const double *)part.p,
                       (int64_t)w, (int64_t)w * w, S, -2.0, Ld, ldd, 1.0, dblk, (int64_t)nb, nullptr, (int64_t)0, 1);
    return hipGetLastError();
  }
  // K-split depth of the general product: deeper splits over long K
  const int kc = w <= cg::GEMM_BN ? 64 : m <= 2048 ? 32 : m <= 4096 ? 64 : m <= 12288 ? 128 : 256;
  return gemm(true, false, w, w, m, Cb, ldcb, Lc, ldl, -2.0, Ld, ldd, 1.0, dblk, nb, nullptr, 0, 1, part, kc, s, 0, cp);
}

#define CG_TRY(expr)                          \
  do {                                        \
    hipError_t _e = (expr);                   \
    if (_e != hipSuccess) return CHOL_ERR_HIP; \
  } while (0)

// ---------------------------------------------------------------------------------------------
// Batched forward sweep: one persistent launch of cg::batch_fwd_kernel with BATCH_WGS workgroups.
constexpr int BATCH_WGS = 256;  // one 140 KB-LDS workgroup per compute unit of an MI355X

struct BatchWs {
  int *order = nullptr;
  int *counter = nullptr;
  double *slots = nullptr;
  double *stage = nullptr;
};

// Workspace of the persistent kernel: processing order, work counter, one slot per workgroup and,
// for FP32 storage, one FP64 staging area per workgroup.
size_t carve_batch(int batch, int64_t n_max, bool f32, void *base, BatchWs *w) {
  Carver c(base);
  w->order = reinterpret_cast<int *>(c.take((size_t)cdiv(batch, 2)));
  w->counter = reinterpret_cast<int *>(c.take(1));
  w->slots = c.take((size_t)std::min(batch, BATCH_WGS) * cg::SLOT_DOUBLES);  // one per workgroup
  w->stage = f32 ? c.take((size_t)std::min(batch, BATCH_WGS) * cg::stage_doubles(n_max)) : nullptr;
  return c.off;
}

// Workspace of the step-synchronous batched path (cg_batched2.hpp): the plan
// (order, sizes, B2_NPREF prefix arrays, step counts) and per problem ceil(n_max / 64) block
// inverses and the two GP vectors.
struct Batch2Ws {
  int *order = nullptr, *nv = nullptr, *pref = nullptr, *count = nullptr;
  double *dinv = nullptr, *vec = nullptr;
  int64_t dinv_stride = 0, vec_stride = 0;
};

size_t carve_batch2(int batch, int64_t n_max, void *base, Batch2Ws *w) {
  Carver c(base);
  const int64_t nblk = std::max<int64_t>(1, cdiv(n_max, cg::B2_NB));
  w->dinv_stride = nblk * cg::B2_BLK;
  w->vec_stride = 2 * std::max<int64_t>(1, n_max);
  w->order = reinterpret_cast<int *>(c.take((size_t)cdiv(batch, 2)));
  w->nv = reinterpret_cast<int *>(c.take((size_t)cdiv(batch, 2)));
  w->pref = reinterpret_cast<int *>(c.take((size_t)cdiv((int64_t)cg::B2_NPREF * (batch + 1), 2)));
  w->count = reinterpret_cast<int *>(c.take((size_t)cg::B2_MAXBLK));
  w->dinv = c.take((size_t)(batch * w->dinv_stride));
  w->vec = c.take((size_t)(batch * w->vec_stride));
  return c.off;
}

// Workspace of a batched call: enough for either path (the step-synchronous path of the factor,
// reverse, GP and factor + reverse calls, or the persistent kernel of the forward call, which
// with FP32 storage also needs its FP64 staging).
// Batches of at least B2_SPLIT_MIN problems run the step-synchronous path as two plans, the even-
// and the odd-indexed problems, one on the caller's stream and one on its side stream: each
// plan's latency-bound launches fill the gaps between the other's (2048-matrix GP launch: 3.47 ->
// 3.2 ms measured with two calls on two streams; three or four plans were slower, 4.5 ms).  Each
// plan has a workspace region of its own.
constexpr int B2_SPLIT_MIN = 1024;

size_t batch2_half_bytes(int batch, int64_t n_max) {
  Batch2Ws w2;
  return align_up(carve_batch2((int)cdiv(batch, 2), n_max, nullptr, &w2));
}

size_t batched_ws_bytes(int batch, int64_t n_max, bool f32) {
  BatchWs w;
  const size_t v1 = carve_batch(batch, n_max, f32, nullptr, &w);
  Batch2Ws w2;
  const size_t v2 = batch >= B2_SPLIT_MIN ? 2 * batch2_half_bytes(batch, n_max) : carve_batch2(batch, n_max, nullptr, &w2);
  return std::max(v1, v2);
}

// Factor, reverse, GP and factor + reverse batches take the step-synchronous path: a plan,
// then per 64-wide block step one grouped launch of each kind over every problem that has the
// step (cg_batched2.hpp), all on stream s.
constexpr int B2_GRID_DIAG = 256;    // diagonal blocks, one per wave: 133 KB of LDS, one per compute unit
constexpr int B2_GRID_TILE = 1024;   // 64 x 64 tile products: 35 KB of LDS, four per compute unit

bool batch2_op(const cg::BatchArgs &a) {
  return a.op == cg::BATCH_FACTOR || a.op == cg::BATCH_REV || a.op == cg::BATCH_GP || a.op == cg::BATCH_FACTOR_REV;
}

// T: the problems' storage type (double, or float for FP32 storage).
// sel_mod, sel_rem: the plan takes the problems i with i % sel_mod == sel_rem (1, 0: all).
template <typename T>
int run_batched2(const cg::BatchArgs &a, int64_t n_max, int sel_mod, int sel_rem, void *workspace, hipStream_t s) {
  const int npos = a.batch > sel_rem ? (int)cdiv(a.batch - sel_rem, sel_mod) : 0;
  if (npos == 0) return CHOL_SUCCESS;
  Batch2Ws ws;
  carve_batch2(npos, n_max, workspace, &ws);
  cg::B2Args b{};
  b.op = a.op; b.batch = npos; b.nprob = a.batch; b.sel_mod = sel_mod; b.sel_rem = sel_rem;
  b.sbar_form = a.sbar_form; b.n_max = (int)n_max;
  b.n = a.n; b.A = a.A; b.lda = a.lda; b.L = a.L; b.ldl = a.ldl; b.y = a.y; b.G = a.G; b.ldg = a.ldg;
  b.f = a.f; b.info = a.info;
  b.order = ws.order; b.nv = ws.nv; b.pref = ws.pref; b.count = ws.count;
  b.dinv = ws.dinv; b.vec = ws.vec;
  b.dinv_stride = ws.dinv_stride; b.vec_stride = ws.vec_stride;
  const int nsteps = (int)cdiv(std::max<int64_t>(n_max, 1), cg::B2_NB);
  hipLaunchKernelGGL(cg::b2_order_kernel<T>, dim3(1), dim3(1024), 0, s, b);
  CG_TRY(hipGetLastError());
  hipLaunchKernelGGL(cg::b2_prefix_kernel, dim3(cg::B2_NPREF), dim3(1024), 0, s, b);
  CG_TRY(hipGetLastError());
  const bool factor = a.op != cg::BATCH_REV;
  const unsigned gd = (unsigned)std::min<int64_t>(cdiv(npos, cg::B2W_WAVES), B2_GRID_DIAG);
  const unsigned gl = (unsigned)std::min(npos, 1024);  // one workgroup per problem (R2, form)
  if (factor) {
    for (int st = 0; st < nsteps; ++st) {
      if (st > 0) {
        hipLaunchKernelGGL(cg::b2_up_kernel<T>, dim3(B2_GRID_TILE), dim3(256), 0, s, b, st);
        CG_TRY(hipGetLastError());
      }
      hipLaunchKernelGGL(cg::b2_potf2_kernel<T>, dim3(gd), dim3(256), 0, s, b, st);
      CG_TRY(hipGetLastError());
      if (st + 1 < nsteps) {
        hipLaunchKernelGGL(cg::b2_f2_kernel<T>, dim3(B2_GRID_TILE), dim3(256), 0, s, b, st);
        CG_TRY(hipGetLastError());
      }
    }
  } else {
    hipLaunchKernelGGL(cg::b2_trinv_kernel<T>, dim3(B2_GRID_DIAG), dim3(256), 0, s, b);
    CG_TRY(hipGetLastError());
  }
  if (a.op == cg::BATCH_FACTOR) return CHOL_SUCCESS;
  for (int t = 0; t < nsteps; ++t) {
    if (t > 0) {
      hipLaunchKernelGGL(cg::b2_r0_kernel<T>, dim3(B2_GRID_TILE), dim3(256), 0, s, b, t);
      CG_TRY(hipGetLastError());
      hipLaunchKernelGGL(cg::b2_r1_kernel<T>, dim3(B2_GRID_TILE), dim3(256), 0, s, b, t);
      CG_TRY(hipGetLastError());
      hipLaunchKernelGGL(cg::b2_r2_kernel<T>, dim3(gl), dim3(256), 0, s, b, t);
      CG_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(cg::b2_r3_kernel<T>, dim3(gd), dim3(256), 0, s, b, t);
    CG_TRY(hipGetLastError());
  }
  if (a.sbar_form == CHOL_SBAR_TRIL) {
    hipLaunchKernelGGL(cg::b2_form_kernel<T>, dim3(gl), dim3(256), 0, s, b);
    CG_TRY(hipGetLastError());
  }
  return CHOL_SUCCESS;
}

int run_batched(cg::BatchArgs a, int64_t n_max, void *workspace, size_t workspace_bytes, hipStream_t s) {
  BatchWs ws;
  const size_t need = batched_ws_bytes(a.batch, n_max, a.f32 != 0);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % WS_ALIGN) != 0 || workspace_bytes < need)
    return CHOL_ERR_WORKSPACE;
  if (batch2_op(a)) {
    auto plan = [&](int mod, int rem, void *w, hipStream_t st) {
      return a.f32 ? run_batched2<float>(a, n_max, mod, rem, w, st) : run_batched2<double>(a, n_max, mod, rem, w, st);
    };
    if (a.batch < B2_SPLIT_MIN) return plan(1, 0, workspace, s);
    std::lock_guard<std::mutex> lock(g_side_mu);
    Side *side = nullptr;
    CG_TRY(side_for(s, &side));
    CG_TRY(hipEventRecord(side->start, s));
    CG_TRY(hipStreamWaitEvent(side->s, side->start, 0));
    int rc = plan(2, 0, workspace, s);
    if (rc == CHOL_SUCCESS)
      rc = plan(2, 1, static_cast<char *>(workspace) + batch2_half_bytes(a.batch, n_max), side->s);
    CG_TRY(hipEventRecord(side->panel, side->s));  // the caller's stream waits for both plans
    CG_TRY(hipStreamWaitEvent(s, side->panel, 0));
    return rc;
  }
  carve_batch(a.batch, n_max, a.f32 != 0, workspace, &ws);
  a.order = ws.order;
  a.counter = ws.counter;
  a.slots = ws.slots;
  a.n_max = (int)n_max;
  a.stage = ws.stage;
  a.stage_stride = cg::stage_doubles(n_max);
  hipLaunchKernelGGL(cg::batch_order_kernel, dim3(1), dim3(256), 0, s, a.batch, a.n, (int)n_max, ws.order,
                     ws.counter);
  CG_TRY(hipGetLastError());
  if (a.op != cg::BATCH_FWD) return CHOL_ERR_UNSUPPORTED;  // every other op is step-synchronous
  const dim3 grid(std::min(a.batch, BATCH_WGS)), block(cg::DIAG_THREADS);
  hipLaunchKernelGGL(cg::batch_fwd_kernel, grid, block, 0, s, a);
  CG_TRY(hipGetLastError());
  return CHOL_SUCCESS;
}


// FP32 storage of the single-matrix calls (defined at the end of this file).
bool f32_storage(int precision) {
  return precision == CHOL_PREC_F32 || precision == CHOL_PREC_F32_TRAIL_BF16X3;
}
int f32_factor(int precision, int64_t n, void *A, int64_t lda, int nb, int layout, int *info, void *ws,
               size_t wsb, void *stream);
int f32_rev(int precision, int64_t n, const void *L, int64_t ldl, void *A, int64_t lda, int sbar_form, int nb,
            int diag, int layout, void *ws, size_t wsb, void *stream);
int f32_fwd(int precision, int64_t n, const void *L, int64_t ldl, void *A, int64_t lda, int nb, int diag,
            int layout, void *ws, size_t wsb, void *stream);
int f32_factor_fwd(int precision, int64_t n, void *A, int64_t lda, void *D, int64_t ldd, int nb, int *info,
                   void *ws, size_t wsb, void *stream);

}  // namespace

extern "C" {

int chol_version(void) { return CHOLGRAD_VERSION; }

int chol_profile_begin(int max_launches) {
  if (g_prof.on) return -1;
  if (max_launches <= 0 || max_launches > (1 << 20)) return -1;
  g_prof.ev.assign(2 * (size_t)max_launches, nullptr);
  for (auto &e : g_prof.ev)
    if (hipEventCreate(&e) != hipSuccess) return CHOL_ERR_HIP;
  g_prof.klass.assign(max_launches, 0);
  g_prof.flops.assign(max_launches, 0.0);
  g_prof.bytes.assign(max_launches, 0.0);
  g_prof.cap = max_launches;
  g_prof.used = 0;
  g_prof.on = true;
  return CHOL_SUCCESS;
}

int chol_profile_end(double *ms, double *flops, double *bytes, int64_t *launches) {
  if (!g_prof.on) return -1;
  if (!ms || !flops || !bytes || !launches) return -1;
  int rc = CHOL_SUCCESS;
  for (int c = 0; c < 3; ++c) { ms[c] = 0.0; flops[c] = 0.0; bytes[c] = 0.0; launches[c] = 0; }
  for (int u = 0; u < g_prof.used; ++u) {
    float t = 0.0f;
    if (hipEventSynchronize(g_prof.ev[2 * u + 1]) != hipSuccess ||
        hipEventElapsedTime(&t, g_prof.ev[2 * u], g_prof.ev[2 * u + 1]) != hipSuccess) {
      rc = CHOL_ERR_HIP;
      continue;
    }
    const int c = g_prof.klass[u] - 1;
    if (c < 0 || c > 2) continue;
    ms[c] += t;
    flops[c] += g_prof.flops[u];
    bytes[c] += g_prof.bytes[u];
    launches[c] += 1;
  }
  for (auto &e : g_prof.ev)
    if (e) (void)hipEventDestroy(e);
  g_prof = Profile();
  return rc;
}

const char *chol_status_string(int status) {
  switch (status) {
    case CHOL_SUCCESS: return "success";
    case CHOL_ERR_HIP: return "a HIP runtime call or kernel launch failed";
    case CHOL_ERR_WORKSPACE: return "workspace missing, too small or not 256-byte aligned";
    case CHOL_ERR_UNSUPPORTED: return "unsupported precision, form or size";
    case CHOL_ERR_TOO_LARGE: return "problem larger than the allocation-free entry point's static scratch allows";
    default: break;
  }
  if (status < 0 && status > -32) return "invalid argument (status -i names argument i)";
  return "unknown status";
}

size_t chol_workspace_bytes(int op, int precision, int64_t n, int nb) {
  if (f32_storage(precision)) {  // FP64 copies of the matrices, then the FP64-storage sweep's own
    const int inner = precision == CHOL_PREC_F32 ? CHOL_PREC_F64 : CHOL_PREC_F64_TRAIL_BF16X3;
    const size_t base = chol_workspace_bytes(op, inner, n, nb);
    return base ? base + (op == CHOL_OP_FACTOR ? 1 : 2) * align_up((size_t)n * n * sizeof(double)) : 0;
  }
  int cp = cg::CP_F64;
  if (n <= 0 || !single_prec(precision, &cp) || !nb_ok(nb)) return 0;
  if (op != CHOL_OP_FACTOR && op != CHOL_OP_REV && op != CHOL_OP_FWD) return 0;
  if (nb == 0) nb = NB_MAX;  // holds whatever width nb = 0 selects in the call
  SweepWs w;
  return carve(n, nb, nullptr, &w);
}

// Diagonal-block variant of both sweeps (Sec. 4.2 leaves it open; the listing uses the symbolic
// form).  CHOL_DIAG_AUTO takes the symbolic form: on MI355X (same GPU, alternating builds) it is
// faster at every size measured, n = 256 to 16384 with nb = 32, 64 and 128.  With it each sweep is
// one stream of launches, so the trailing rows of a step need no split around the diagonal block,
// and its cost per block is three small MFMA products against the Level-2 routine's nb dependent
// column steps in one workgroup.
bool diag_ok(int diag) { return diag == CHOL_DIAG_AUTO || diag == CHOL_DIAG_SYMBOLIC || diag == CHOL_DIAG_LEVEL2; }
bool diag_symbolic(int diag) { return diag != CHOL_DIAG_LEVEL2; }

static int rev_impl(int precision, int64_t n, const void *Lv, int64_t ldl, void *Av, int64_t lda,
                    int sbar_form, int nb, int diag, void *workspace, size_t workspace_bytes, void *stream,
                    int64_t part_slots = PART_SLOTS, int64_t part2_slots = PART_SLOTS) {
  if (precision == CHOL_PREC_F32) return CHOL_ERR_UNSUPPORTED;
  int cp = cg::CP_F64;
  if (!single_prec(precision, &cp)) return -1;
  if (n < 0 || n > (int64_t)1 << 30) return -2;
  if (n == 0) return CHOL_SUCCESS;
  if (!Lv || !aligned8(Lv)) return -3;
  if (ldl < n) return -4;
  if (!Av || !aligned8(Av)) return -5;
  if (lda < n) return -6;
  if (sbar_form != CHOL_SBAR_SYM && sbar_form != CHOL_SBAR_TRIL) return -7;
  if (!nb_ok(nb)) return -8;
  if (!diag_ok(diag)) return -9;
  if (nb == 0) nb = auto_nb(CHOL_OP_REV, n, !diag_symbolic(diag));
  if (!diag_symbolic(diag) && nb > cg::DIAG_MAX) return CHOL_ERR_UNSUPPORTED;  // Level-2 cores hold <= 128
  SweepWs ws;
  const size_t need = carve(n, nb, nullptr, &ws, part_slots, part2_slots);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % WS_ALIGN) != 0 || workspace_bytes < need)
    return CHOL_ERR_WORKSPACE;
  carve(n, nb, workspace, &ws, part_slots, part2_slots);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const double *L = static_cast<const double *>(Lv);
  double *A = static_cast<double *>(Av);
  const int64_t nblk = cdiv(n, nb);

  // Diagonal-block adjoint.  Symbolic: D-bar <- D^-T Phi(D^T D-bar) D^-1 (symmetric part) as three
  // small MFMA products with the block inverse on the caller's stream, so the whole sweep is one
  // stream.  Level-2: Sec. 4.1's unblocked sweep in one workgroup on the side stream, overlapped
  // with the next step's bulk product.
  const bool sym = diag_symbolic(diag);
  std::lock_guard<std::mutex> lock(g_side_mu);
  Side *side = nullptr;
  hipStream_t s2 = nullptr;
  const bool any_level2 = !sym;
  if (any_level2) {
    CG_TRY(side_for(s, &side));
    s2 = side->s;
  } else {
    ws.part.sk_wgs = TARGET_WGS;
  }

  CG_TRY(block_inverses(n, nb, L, ldl, ws.dinv, ws.panel, s));  // the panel is free until the sweep
  if (any_level2) {
    CG_TRY(hipEventRecord(side->start, s));
    CG_TRY(hipStreamWaitEvent(s2, side->start, 0));
  }
  bool prev_level2 = false;  // the previous step (block b+1) left its diagonal adjoint on s2

  // Reverse sweep over block columns, right to left, in left-looking ("lazy") order: when block
  // [j, k) is reached, everything right of it is final and is stored as the symmetric gradient
  // S_sym in both triangles of A[k:, k:].  The accumulated knock-on terms of Sec. 4.2's
  // B-bar / R-bar updates then collapse to one product:
  //   C-bar = L-bar_C - (T + T^T)[k:, k:] L[k:, j:k] = L-bar_C - 2 S_sym[k:, k:] L[k:, j:k].
  // Look-ahead (Level-2 variant): the rows of that product below block b+1 need only block b+1's
  // panel, so they run on the caller's stream while block b+1's diagonal adjoint runs on the side
  // stream; only block b+1's own rows wait for its diagonal block.
  for (int64_t b = nblk - 1; b >= 0; --b) {
    const int64_t j = b * nb, k = std::min<int64_t>(n, j + nb);
    const int w = (int)(k - j);
    const int m = (int)(n - k);
    if (m > 0) {
      const int m1 = std::min(m, nb);  // rows of block b+1
      const int m2 = m - m1;           // rows below block b+1
      // X = L-bar_C - 2 S_sym[k:, k:] L[k:, j:k]   -> panel (m x w), rows below block b+1 first
      // After a symbolic diagonal adjoint (caller's stream) all of S_sym[k:, k:] is final: one
      // product over all m rows.  After a Level-2 one, the rows below block b+1 go first.
      const int mb = prev_level2 ? m2 : 0;
      if (mb > 0)
        CG_TRY(gemm(false, false, mb, w, m, A + (k + m1) * lda + k, lda, L + k * ldl + j, ldl, -2.0,
                    A + (k + m1) * lda + j, lda, 1.0, ws.panel + (int64_t)m1 * nb, nb, nullptr, 0, 0,
                    ws.part, 256, s, 1, cp));
      if (prev_level2) CG_TRY(hipStreamWaitEvent(s, side->diag, 0));
      // From here to the next diagonal adjoint every product is on the sweep's critical path and
      // has a single 128-wide tile column: fine K-splits spread it over many compute units.
      CG_TRY(gemm(false, false, m - mb, w, m, A + k * lda + k, lda, L + k * ldl + j, ldl, -2.0,
                  A + k * lda + j, lda, 1.0, ws.panel, nb, nullptr, 0, 0, ws.part, 64, s, 1, cp));
      // C-bar = X D^-1 (Sec. 4.2: C-bar <- C-bar D^-1); store C-bar/2 = S_sym entries in both
      // triangles.  Blocks wider than 128 below at least 8192 rows: one unsplit MFMA product on
      // 128 x 128 tiles with the mirrored store (each X row strip is read once per 128 output
      // columns instead of once per 16; measured at n = 16384, nb = 256: 46 us against the tiled
      // kernel's 95 us at m = 16128, but a fixed ~45 us of K-tile latency at small m, where the
      // tiled kernel takes 6 to 40 us); otherwise the tiled kernel.
      if (w > cg::GEMM_BN && m >= 8192) {
        CG_TRY(gemm(false, false, m, w, w, ws.panel, nb, ws.dinv + b * nb * nb, nb, 0.5, nullptr, 0, 0.0,
                    A + k * lda + j, lda, A + j * lda + k, lda, 0, nullptr, 64, s));
      } else {
        const int64_t nct = cdiv(w, cg::SYM_TILE);
        const unsigned grid = (unsigned)(cdiv(cdiv(m, cg::SYM_TILE), 8) * 8 * nct);
        hipLaunchKernelGGL(cg::rev_panel_solve_kernel, dim3(grid), dim3(256), 0, s, m, w, (const double *)ws.panel,
                           (int64_t)nb, (const double *)(ws.dinv + b * nb * nb), (int64_t)nb, 0.5,
                           A + k * lda + j, lda, A + j * lda + k, lda);
        CG_TRY(hipGetLastError());
      }
      // D-bar = tril(L-bar_D) - tril(C-bar^T C), C-bar = 2 * A[k:, j:k]   -> dblk (w x w).  On the
      // caller's stream, before the next step's bulk product is queued: a small split-K product
      // that runs fastest with the whole GPU to itself, and the diagonal adjoint released after
      // it then finds a free compute unit while that bulk product runs.
      CG_TRY(rev_syrk(w, m, A + k * lda + j, lda, L + k * ldl + j, ldl, A + j * lda + j, lda, ws.dblk, nb, ws.part,
                      s, cp));
    } else {
      CG_TRY(copy_scaled(w, w, A + j * lda + j, lda, 1.0, ws.dblk, nb, 1, s));
    }
    prev_level2 = !sym;
    if (!prev_level2) {
      // Symbolic diagonal adjoint with D = L[j:k, j:k] and its inverse from trinv, three tiled
      // launches:  P = tril(D)^T tril(D-bar);  Q = D^-T Y with Y = (Phi(P) + Phi(P)^T) / 2;
      // S_sym = Q D^-1, whose lower triangle is written to both triangles of A's diagonal block
      // (so the block is exactly symmetric).
      double *tP = ws.tmp, *tQ = ws.tmp + (int64_t)nb * nb;
      const double *dinv_b = ws.dinv + b * nb * nb;
      const unsigned tiles = (unsigned)(cdiv(w, cg::SYM_TILE) * cdiv(w, cg::SYM_TILE));
      hipLaunchKernelGGL(cg::sym_rev_p_kernel, dim3(tiles), dim3(256), 0, s, w, L + j * ldl + j, ldl,
                         (const double *)ws.dblk, (int64_t)nb, tP, (int64_t)nb);
      CG_TRY(hipGetLastError());
      hipLaunchKernelGGL(cg::sym_rev_q_kernel, dim3(tiles), dim3(256), 0, s, w, (const double *)tP,
                         (int64_t)nb, dinv_b, (int64_t)nb, tQ, (int64_t)nb);
      CG_TRY(hipGetLastError());
      hipLaunchKernelGGL(cg::sym_rev_s_kernel, dim3(tiles), dim3(256), 0, s, w, (const double *)tQ,
                         (int64_t)nb, dinv_b, (int64_t)nb, A + j * lda + j, lda);
      CG_TRY(hipGetLastError());
    } else {
      CG_TRY(hipEventRecord(side->panel, s));
      CG_TRY(hipStreamWaitEvent(s2, side->panel, 0));
      hipLaunchKernelGGL(cg::diag_rev_kernel, dim3(1), dim3(cg::DIAG_THREADS), 0, s2, w,
                         L + j * ldl + j, ldl, (const double *)ws.dblk, (int64_t)nb,
                         (const double *)(ws.dinv + b * nb * nb), nb, A + j * lda + j, lda);
      CG_TRY(hipGetLastError());
      CG_TRY(hipEventRecord(side->diag, s2));
    }
  }
  if (prev_level2) CG_TRY(hipStreamWaitEvent(s, side->diag, 0));
  if (sbar_form == CHOL_SBAR_TRIL) {
    const int blocks = (int)std::min<int64_t>(cdiv(n * n, 256), 4096);
    hipLaunchKernelGGL(cg::sym_to_tril_kernel, dim3(blocks), dim3(256), 0, s, n, A, lda);
    CG_TRY(hipGetLastError());
  }
  return CHOL_SUCCESS;
}

int chol_rev(int precision, int64_t n, const void *Lv, int64_t ldl, void *Av, int64_t lda,
             int sbar_form, int nb, void *workspace, size_t workspace_bytes, void *stream) {
  if (f32_storage(precision))
    return f32_rev(precision, n, Lv, ldl, Av, lda, sbar_form, nb, CHOL_DIAG_AUTO, CHOL_LAYOUT_ROW_MAJOR, workspace,
                   workspace_bytes, stream);
  return rev_impl(precision, n, Lv, ldl, Av, lda, sbar_form, nb, CHOL_DIAG_AUTO, workspace, workspace_bytes,
                  stream);
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// chol_rev_noalloc: chol_rev with its workspace in a file-scope device array instead of the
// caller's buffer.  The array's name is a host-side stand-in in host code; the device address
// comes from hipGetSymbolAddress, once per device (each device holds its own copy), with that
// device current.  Layout of the array: carve(n, nb) with a partial-tile buffer of
// NOALLOC_PART_SLOTS tiles and no side-stream buffer; at n = 4096, nb = 128 that is 4 MiB of block
// inverses + 4 MiB of panel + 0.4 MiB of small blocks + 36 MiB of partial tiles = 44.4 MiB.
namespace {
constexpr int64_t NOALLOC_N_MAX = 4096;
constexpr int NOALLOC_NB_MAX = 128;
constexpr int64_t NOALLOC_PART_SLOTS = 288;  // stream-K over up to ~258 workgroups at n = 4096
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)45 << 20;

__device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES];

// Device address of `scratch` on the current device (looked up on the first call per device).
hipError_t scratch_ptr(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

extern "C" {

int chol_rev_noalloc(int precision, int64_t n, const void *Lv, int64_t ldl, void *Av, int64_t lda,
                     int sbar_form, int nb, void *stream) {
  if (nb == 0) nb = NOALLOC_DEFAULT_NB;
  // Arguments first (a dry call without workspace), before the device is touched.
  const int chk = rev_impl(precision, n, Lv, ldl, Av, lda, sbar_form, nb, CHOL_DIAG_SYMBOLIC, nullptr, 0, stream,
                           NOALLOC_PART_SLOTS, 0);
  if (chk != CHOL_ERR_WORKSPACE) return chk;  // CHOL_SUCCESS for n == 0, or an argument error
  if (n > NOALLOC_N_MAX) return CHOL_ERR_TOO_LARGE;
  if (nb > NOALLOC_NB_MAX) return -8;
  SweepWs w;
  if (carve(n, nb, nullptr, &w, NOALLOC_PART_SLOTS, 0) > NOALLOC_SCRATCH_BYTES)
    return CHOL_ERR_TOO_LARGE;
  void *ws = nullptr;
  CG_TRY(scratch_ptr(&ws));
  return rev_impl(precision, n, Lv, ldl, Av, lda, sbar_form, nb, CHOL_DIAG_SYMBOLIC, ws, NOALLOC_SCRATCH_BYTES,
                  stream, NOALLOC_PART_SLOTS, 0);
}

int chol_factor(int precision, int64_t n, void *Av, int64_t lda, int nb, int *info,
                void *workspace, size_t workspace_bytes, void *stream) {
  if (f32_storage(precision)) {
    if (n > 0 && !info) return -6;
    return f32_factor(precision, n, Av, lda, nb, CHOL_LAYOUT_ROW_MAJOR, info, workspace, workspace_bytes, stream);
  }
  int cp = cg::CP_F64;
  if (!single_prec(precision, &cp)) return -1;
  if (n < 0 || n > (int64_t)1 << 30) return -2;
  if (n == 0) return CHOL_SUCCESS;
  if (!Av || !aligned8(Av)) return -3;
  if (lda < n) return -4;
  if (!nb_ok(nb)) return -5;
  if (!info) return -6;
  if (nb == 0) nb = auto_nb(CHOL_OP_FACTOR, n);
  SweepWs ws;
  const size_t need = carve(n, nb, nullptr, &ws);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % WS_ALIGN) != 0 || workspace_bytes < need)
    return CHOL_ERR_WORKSPACE;
  carve(n, nb, workspace, &ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *A = static_cast<double *>(Av);
  const int64_t nblk = cdiv(n, nb);
  // A sweep of at most FACTOR_ONE_STREAM_BLOCKS blocks has at most one update over older columns
  // (block 2's over block 0) to run beside its chain, so it stays on the caller's stream: the
  // side-stream hand-overs cost more than that overlap wins (N = 256, nb = 128: 255 -> 197 us;
  // with four blocks, N = 512 at nb = 128, the side stream is faster again).
  const bool one = nblk <= FACTOR_ONE_STREAM_BLOCKS;
  std::lock_guard<std::mutex> lock(g_side_mu);
  Side *side = nullptr;
  hipStream_t s2 = s;
  if (!one) {
    CG_TRY(side_for(s, &side));
    s2 = side->s;
  }
  auto record = [&](hipEvent_t Side::*e, hipStream_t st) { return one ? hipSuccess : hipEventRecord(side->*e, st); };
  auto wait = [&](hipStream_t st, hipEvent_t Side::*e) {
    return one ? hipSuccess : hipStreamWaitEvent(st, side->*e, 0);
  };
  hipLaunchKernelGGL(cg::set_int_kernel, dim3(1), dim3(1), 0, s, info, 0);
  CG_TRY(hipGetLastError());
  CG_TRY(record(&Side::start, s));
  CG_TRY(wait(s2, &Side::start));
  // Sec. 4.2 chol_blocked, left to right, with look-ahead.  Block b's diagonal factor needs only
  // block b's own rows updated, and those need only the rows of block b-1's panel solve that lie
  // in block b; so the chain from one diagonal factor to the next is: panel solve of the next
  // block's rows (side stream) -> update of those rows over block b-1's columns (caller's stream)
  // -> POTF2.  Everything else -- the update over older columns, the rows below, their panel
  // solve -- runs beside it.  Events: diag (own rows updated), low (rows below updated), top (own
  // rows of the next block solved), panel (whole panel solved).
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t j = b * nb, k = std::min<int64_t>(n, j + nb);
    const int w = (int)(k - j);
    const int m = (int)(n - k);
    if (b > 0) {
      const int64_t jp = j - nb;  // block b-1 is [jp, j)
      // [D; C] <- [D; C] - [R; B] R^T over the columns left of block b-1 (all rows below j)
      if (jp > 0)
        CG_TRY(gemm(false, true, (int)(n - j), w, (int)jp, A + j * lda, lda, A + j * lda, lda, -1.0,
                    A + j * lda + j, lda, 1.0, A + j * lda + j, lda, nullptr, 0, 0, ws.part, 256, s, 2, cp));
      // D <- D - D_{b,b-1} D_{b,b-1}^T   (chain: fine K-splits)
      CG_TRY(wait(s, &Side::top));
      CG_TRY(gemm(false, true, w, w, nb, A + j * lda + jp, lda, A + j * lda + jp, lda, -1.0, A + j * lda + j,
                  lda, 1.0, A + j * lda + j, lda, nullptr, 0, 0, ws.part, 32, s, 2, cp));
      CG_TRY(record(&Side::diag, s));
      CG_TRY(wait(s2, &Side::diag));
      // C <- C - B_{b-1} D_{b,b-1}^T   (rows below block b)
      if (m > 0) {
        CG_TRY(wait(s, &Side::panel));
        CG_TRY(gemm(false, true, m, w, nb, A + k * lda + jp, lda, A + j * lda + jp, lda, -1.0, A + k * lda + j,
                    lda, 1.0, A + k * lda + j, lda, nullptr, 0, 0, ws.part, 64, s, 2, cp));
        CG_TRY(record(&Side::low, s));
      }
    }
    // D <- chol_unblocked(D); D^-1 for the panel solve
    CG_TRY(potf2_any(w, A + j * lda + j, lda, ws.dblk, nb, info, j, ws.tmp, ws.part2, s2, m > 0));
    // C <- C tril(D)^-T, the next block's rows first
    if (m > 0) {
      const int m1 = std::min(m, nb);
      if (b > 0) CG_TRY(wait(s2, &Side::low));
      CG_TRY(panel_solve_t(m1, w, A + k * lda + j, lda, ws.dblk, nb, ws.panel, ws.part2, 32, s2));
      CG_TRY(record(&Side::top, s2));
      if (m > m1)
        CG_TRY(panel_solve_t(m - m1, w, A + (k + m1) * lda + j, lda, ws.dblk, nb, ws.panel + (int64_t)m1 * nb,
                             nullptr, 128, s2));
    }
    CG_TRY(record(&Side::panel, s2));
  }
  CG_TRY(wait(s, &Side::panel));
  const int blocks = (int)std::min<int64_t>(cdiv(n * n, 256), 4096);
  hipLaunchKernelGGL(cg::zero_upper_kernel, dim3(blocks), dim3(256), 0, s, n, A, lda);
  CG_TRY(hipGetLastError());
  return CHOL_SUCCESS;
}

static int fwd_impl(int precision, int64_t n, const void *Lv, int64_t ldl, void *Av, int64_t lda, int nb,
                    int diag, void *workspace, size_t workspace_bytes, void *stream) {
  if (precision == CHOL_PREC_F32) return CHOL_ERR_UNSUPPORTED;
  int cp = cg::CP_F64;
  if (!single_prec(precision, &cp)) return -1;
  if (n < 0 || n > (int64_t)1 << 30) return -2;
  if (n == 0) return CHOL_SUCCESS;
  if (!Lv || !aligned8(Lv)) return -3;
  if (ldl < n) return -4;
  if (!Av || !aligned8(Av)) return -5;
  if (lda < n) return -6;
  if (!nb_ok(nb)) return -7;
  if (!diag_ok(diag)) return -8;
  if (nb == 0) nb = auto_nb(CHOL_OP_FWD, n, !diag_symbolic(diag));
  if (!diag_symbolic(diag) && nb > cg::DIAG_MAX) return CHOL_ERR_UNSUPPORTED;  // Level-2 cores hold <= 128
  SweepWs ws;
  const size_t need = carve(n, nb, nullptr, &ws);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % WS_ALIGN) != 0 || workspace_bytes < need)
    return CHOL_ERR_WORKSPACE;
  carve(n, nb, workspace, &ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const double *L = static_cast<const double *>(Lv);
  double *A = static_cast<double *>(Av);
  const int64_t nblk = cdiv(n, nb);
  // Steps [0, b0) take the Level-2 diagonal block on the side stream with look-ahead, steps
  // [b0, nblk) the symbolic one on the caller's stream: all steps one way or the other.
  const int64_t b0 = diag_symbolic(diag) ? 0 : nblk;
  std::lock_guard<std::mutex> lock(g_side_mu);
  Side *side = nullptr;
  hipStream_t s2 = nullptr;
  if (b0 > 0) {
    CG_TRY(side_for(s, &side));
    s2 = side->s;
  } else {
    ws.part.sk_wgs = TARGET_WGS;
  }
  CG_TRY(block_inverses(n, nb, L, ldl, ws.dinv, ws.panel, s));  // the panel is free until the sweep
  if (b0 > 0) {
    CG_TRY(hipEventRecord(side->start, s));
    CG_TRY(hipStreamWaitEvent(s2, side->start, 0));
  }
  // Sec. 4.2 chol_blocked_fwd, left to right, with the same look-ahead as chol_factor: the chain
  // is panel step of the next block's rows -> update of those rows over block b-1's columns ->
  // diagonal block, everything else beside it.
  for (int64_t b = 0; b < b0; ++b) {
    const int64_t j = b * nb, k = std::min<int64_t>(n, j + nb);
    const int w = (int)(k - j);
    const int m = (int)(n - k);
    if (b > 0) {
      const int64_t jp = j - nb;
      // [D-dot; C-dot] -= [R-dot; B-dot] R^T + [R; B] R-dot^T   over columns [0, jp)
      // (one launch: the two products share the output as one combined K range)
      if (jp > 0)
        CG_TRY(gemm(false, true, (int)(n - j), w, (int)jp, A + j * lda, lda, L + j * ldl, ldl, -1.0,
                    A + j * lda + j, lda, 1.0, A + j * lda + j, lda, nullptr, 0, 0, ws.part, 256, s, 3, cp,
                    Pair2{L + j * ldl, ldl, A + j * lda, lda}));
      // block b's own rows over columns [jp, j)   (chain: fine K-splits)
      CG_TRY(hipStreamWaitEvent(s, side->top, 0));
      CG_TRY(gemm(false, true, w, w, nb, A + j * lda + jp, lda, L + j * ldl + jp, ldl, -1.0, A + j * lda + j,
                  lda, 1.0, A + j * lda + j, lda, nullptr, 0, 0, ws.part, 32, s, 3, cp,
                  Pair2{L + j * ldl + jp, ldl, A + j * lda + jp, lda}));
      CG_TRY(hipEventRecord(side->diag, s));
      CG_TRY(hipStreamWaitEvent(s2, side->diag, 0));
      // rows below block b over columns [jp, j)
      if (m > 0) {
        CG_TRY(hipStreamWaitEvent(s, side->panel, 0));
        CG_TRY(gemm(false, true, m, w, nb, A + k * lda + jp, lda, L + j * ldl + jp, ldl, -1.0, A + k * lda + j,
                    lda, 1.0, A + k * lda + j, lda, nullptr, 0, 0, ws.part, 64, s, 3, cp,
                    Pair2{L + k * ldl + jp, ldl, A + j * lda + jp, lda}));
        CG_TRY(hipEventRecord(side->low, s));
      }
    }
    // D-dot <- chol_unblocked_fwd(D, D-dot)   (strict upper triangle of the block set to 0)
    hipLaunchKernelGGL(cg::diag_fwd_kernel, dim3(1), dim3(cg::DIAG_THREADS), 0, s2, w, L + j * ldl + j,
                       ldl, (const double *)(ws.dinv + b * nb * nb), nb, A + j * lda + j, lda);
    CG_TRY(hipGetLastError());
    if (m > 0) {
      // C-dot <- (C-dot - C D-dot^T) D^-T, the next block's rows first
      const int m1 = std::min(m, nb);
      if (b > 0) CG_TRY(hipStreamWaitEvent(s2, side->low, 0));
      CG_TRY(gemm(false, true, m1, w, w, L + k * ldl + j, ldl, A + j * lda + j, lda, -1.0,
                  A + k * lda + j, lda, 1.0, ws.panel, nb, nullptr, 0, 0, ws.part2, 32, s2));
      CG_TRY(gemm(false, true, m1, w, w, ws.panel, nb, ws.dinv + b * nb * nb, nb, 1.0, nullptr, 0, 0.0,
                  A + k * lda + j, lda, nullptr, 0, 0, ws.part2, 32, s2));
      CG_TRY(hipEventRecord(side->top, s2));
      if (m > m1) {
        CG_TRY(gemm(false, true, m - m1, w, w, L + (k + m1) * ldl + j, ldl, A + j * lda + j, lda, -1.0,
                    A + (k + m1) * lda + j, lda, 1.0, ws.panel + (int64_t)m1 * nb, nb, nullptr, 0, 0, nullptr,
                    128, s2));
        CG_TRY(gemm(false, true, m - m1, w, w, ws.panel + (int64_t)m1 * nb, nb, ws.dinv + b * nb * nb, nb, 1.0,
                    nullptr, 0, 0.0, A + (k + m1) * lda + j, lda, nullptr, 0, 0, nullptr, 128, s2));
      }
    }
    CG_TRY(hipEventRecord(side->panel, s2));
  }
  if (b0 > 0) CG_TRY(hipStreamWaitEvent(s, side->panel, 0));
  // Symbolic steps, on the caller's stream only (after block b0-1's panel where Level-2 steps came
  // first): per step the update of block b's column (its own rows and every row below, one
  // contraction) over all older columns, then
  //   Ds = sym(D-dot);  P = D^-1 Ds;  Q = P D^-T;  L-dot_D = tril(D) Phi(Q),
  // then the panel solve C-dot <- (C-dot - C L-dot_D^T) D^-T of every row below.  Since
  // D^-1 L-dot_D = Phi(Q), that solve is the single paired product
  //   L-dot_C = C-dot D^-T + C (-Phi(Q))^T.
  double *tN = ws.tmp, *tP = ws.tmp + (int64_t)nb * nb;  // tN = -Phi(Q)
  for (int64_t b = b0; b < nblk; ++b) {
    const int64_t j = b * nb, k = std::min<int64_t>(n, j + nb);
    const int w = (int)(k - j);
    const int m = (int)(n - k);
    const double *dinv_b = ws.dinv + b * nb * nb;
    // Panel solve for nb < 128: the tiled kernel, which reads C-dot from the workspace panel
    // (ld nb) and writes L-dot_C to A, so the update puts the block column [D-dot; C-dot] there.
    // For nb = 128 the paired product on 128 x 128 tiles is faster (it reuses each operand strip
    // across all columns): the update and the solve then work in place in A.
    const bool tiled = nb != cg::GEMM_BN;
    double *const col = tiled ? ws.panel : A + j * lda + j;
    const int64_t ldcol = tiled ? (int64_t)nb : lda;
    if (j > 0) {
      // [D-dot; C-dot] = Sigma-dot's block column - [R-dot; B-dot] R^T - [R; B] R-dot^T over [0, j)
      CG_TRY(gemm(false, true, (int)(n - j), w, (int)j, A + j * lda, lda, L + j * ldl, ldl, -1.0,
                  A + j * lda + j, lda, 1.0, col, ldcol, nullptr, 0, 0, ws.part, 32, s, 3, cp,
                  Pair2{L + j * ldl, ldl, A + j * lda, lda}));
    } else if (tiled) {
      CG_TRY(copy_scaled((int)n, w, A, lda, 1.0, col, ldcol, 0, s));  // first column: no update
    }
    // Three tiled launches: tP = D^-1 Ds;  tN = -Phi(tP D^-T);  L-dot_D = -(tril(D) tN) into A's
    // diagonal block.
    const unsigned tiles = (unsigned)(cdiv(w, cg::SYM_TILE) * cdiv(w, cg::SYM_TILE));
    hipLaunchKernelGGL(cg::sym_fwd_p_kernel, dim3(tiles), dim3(256), 0, s, w, (const double *)col, ldcol, dinv_b,
                       (int64_t)nb, tP, (int64_t)nb);
    CG_TRY(hipGetLastError());
    hipLaunchKernelGGL(cg::sym_fwd_n_kernel, dim3(tiles), dim3(256), 0, s, w, (const double *)tP, (int64_t)nb,
                       dinv_b, (int64_t)nb, tN, (int64_t)nb);
    CG_TRY(hipGetLastError());
    hipLaunchKernelGGL(cg::sym_fwd_l_kernel, dim3(tiles), dim3(256), 0, s, w, L + j * ldl + j, ldl,
                       (const double *)tN, (int64_t)nb, A + j * lda + j, lda);
    CG_TRY(hipGetLastError());
    if (m > 0 && tiled && w > cg::GEMM_BN) {
      // blocks wider than 128: L-dot_C = C-dot D^-T - L_C tN^T as one paired product from the
      // workspace panel into A (out of place, so any tiling is safe), on 128 x 256 tiles when the
      // shapes allow them
      CG_TRY(gemm(false, true, m, w, w, col + w * ldcol, ldcol, dinv_b, nb, 1.0, nullptr, 0, 0.0,
                  A + k * lda + j, lda, nullptr, 0, 0, ws.part, 32, s, 0, cg::CP_F64,
                  Pair2{L + k * ldl + j, ldl, tN, nb}));
    } else if (m > 0 && tiled) {
      const int64_t nct = cdiv(w, cg::SYM_TILE);
      const unsigned grid = (unsigned)(cdiv(cdiv(m, cg::SYM_TILE), 8) * 8 * nct);
      hipLaunchKernelGGL(cg::fwd_panel_solve_kernel, dim3(grid), dim3(256), 0, s, m, w,
                         (const double *)(col + w * ldcol), ldcol, L + k * ldl + j, ldl, dinv_b, (int64_t)nb,
                         (const double *)tN, (int64_t)nb, A + k * lda + j, lda);
      CG_TRY(hipGetLastError());
    } else if (m > 0) {
      // in place: each 128-row tile's workgroup reads its rows of C-dot before it writes them
      CG_TRY(gemm(false, true, m, w, w, A + k * lda + j, lda, dinv_b, nb, 1.0, nullptr, 0, 0.0,
                  A + k * lda + j, lda, nullptr, 0, 0, ws.part, 32, s, 0, cg::CP_F64,
                  Pair2{L + k * ldl + j, ldl, tN, nb}));
    }
  }
  const int blocks = (int)std::min<int64_t>(cdiv(n * n, 256), 4096);
  hipLaunchKernelGGL(cg::zero_upper_kernel, dim3(blocks), dim3(256), 0, s, n, A, lda);
  CG_TRY(hipGetLastError());
  return CHOL_SUCCESS;
}


static bool batched_prec_ok(int precision) {
  return precision == CHOL_PREC_F64 || precision == CHOL_PREC_F32;
}

int chol_factor_fwd(int precision, int64_t n, void *Av, int64_t lda, void *Dv, int64_t ldd, int nb, int *info,
                    void *workspace, size_t workspace_bytes, void *stream) {
  if (f32_storage(precision))
    return f32_factor_fwd(precision, n, Av, lda, Dv, ldd, nb, info, workspace, workspace_bytes, stream);
  int cp = cg::CP_F64;
  if (!single_prec(precision, &cp)) return -1;
  if (n < 0 || n > (int64_t)1 << 30) return -2;
  if (n == 0) return CHOL_SUCCESS;
  if (!Av || !aligned8(Av)) return -3;
  if (lda < n) return -4;
  if (!Dv || !aligned8(Dv)) return -5;
  if (ldd < n) return -6;
  if (!nb_ok(nb)) return -7;
  if (!info) return -8;
  if (nb == 0) nb = auto_nb(CHOL_OP_FACTOR, n);
  SweepWs ws;
  const size_t need = carve(n, nb, nullptr, &ws);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % WS_ALIGN) != 0 || workspace_bytes < need)
    return CHOL_ERR_WORKSPACE;
  carve(n, nb, workspace, &ws);
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *A = static_cast<double *>(Av);   // Sigma -> L
  double *D = static_cast<double *>(Dv);   // Sigma-dot -> L-dot
  const int64_t nblk = cdiv(n, nb);
  std::lock_guard<std::mutex> lock(g_side_mu);
  Side *side = nullptr;
  CG_TRY(side_for(s, &side));
  hipStream_t s2 = side->s;
  hipLaunchKernelGGL(cg::set_int_kernel, dim3(1), dim3(1), 0, s, info, 0);
  CG_TRY(hipGetLastError());
  CG_TRY(hipEventRecord(side->start, s));
  CG_TRY(hipStreamWaitEvent(s2, side->start, 0));
  // One left-to-right sweep carrying both Sec. 4.2 chol_blocked and chol_blocked_fwd: when block
  // column b is reached, every column left of it holds its final L and L-dot, which is all both
  // updates need.  The chain and the look-ahead are those of chol_factor, with the forward
  // diagonal block (which reuses POTF2's block inverse) and the forward panel step following
  // the factor's on the side stream.
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t j = b * nb, k = std::min<int64_t>(n, j + nb);
    const int w = (int)(k - j);
    const int m = (int)(n - k);
    if (b > 0) {
      const int64_t jp = j - nb;
      if (jp > 0) {
        CG_TRY(gemm(false, true, (int)(n - j), w, (int)jp, A + j * lda, lda, A + j * lda, lda, -1.0,
                    A + j * lda + j, lda, 1.0, A + j * lda + j, lda, nullptr, 0, 0, ws.part, 256, s, 2, cp));
        CG_TRY(gemm(false, true, (int)(n - j), w, (int)jp, D + j * ldd, ldd, A + j * lda, lda, -1.0,
                    D + j * ldd + j, ldd, 1.0, D + j * ldd + j, ldd, nullptr, 0, 0, ws.part, 256, s, 3, cp,
                    Pair2{A + j * lda, lda, D + j * ldd, ldd}));
      }
      // block b's own rows over columns [jp, j)   (chain)
      CG_TRY(hipStreamWaitEvent(s, side->top, 0));
      CG_TRY(gemm(false, true, w, w, nb, A + j * lda + jp, lda, A + j * lda + jp, lda, -1.0, A + j * lda + j,
                  lda, 1.0, A + j * lda + j, lda, nullptr, 0, 0, ws.part, 32, s, 2, cp));
      CG_TRY(gemm(false, true, w, w, nb, D + j * ldd + jp, ldd, A + j * lda + jp, lda, -1.0, D + j * ldd + j,
                  ldd, 1.0, D + j * ldd + j, ldd, nullptr, 0, 0, ws.part, 32, s, 3, cp,
                  Pair2{A + j * lda + jp, lda, D + j * ldd + jp, ldd}));
      CG_TRY(hipEventRecord(side->diag, s));
      CG_TRY(hipStreamWaitEvent(s2, side->diag, 0));
      // rows below block b over columns [jp, j)
      if (m > 0) {
        CG_TRY(hipStreamWaitEvent(s, side->panel, 0));
        CG_TRY(gemm(false, true, m, w, nb, A + k * lda + jp, lda, A + j * lda + jp, lda, -1.0, A + k * lda + j,
                    lda, 1.0, A + k * lda + j, lda, nullptr, 0, 0, ws.part, 64, s, 2, cp));
        CG_TRY(gemm(false, true, m, w, nb, D + k * ldd + jp, ldd, A + j * lda + jp, lda, -1.0, D + k * ldd + j,
                    ldd, 1.0, D + k * ldd + j, ldd, nullptr, 0, 0, ws.part, 64, s, 3, cp,
                    Pair2{A + k * lda + jp, lda, D + j * ldd + jp, ldd}));
        CG_TRY(hipEventRecord(side->low, s));
      }
    }
    // L_bb = chol_unblocked(D_bb) and its inverse; then L-dot_bb from D-dot_bb: the Level-2
    // chol_unblocked_fwd for blocks up to 128 wide, the block's symbolic form
    // L-dot_bb = L_bb Phi(L_bb^-1 D-dot_bb L_bb^-T) (three tiled products) for wider ones
    CG_TRY(potf2_any(w, A + j * lda + j, lda, ws.dblk, nb, info, j, ws.tmp, ws.part2, s2));
    if (w <= cg::DIAG_MAX) {
      hipLaunchKernelGGL(cg::diag_fwd_kernel, dim3(1), dim3(cg::DIAG_THREADS), 0, s2, w,
                         (const double *)(A + j * lda + j), lda, (const double *)ws.dblk, nb, D + j * ldd + j, ldd);
      CG_TRY(hipGetLastError());
    } else {
      double *tN = ws.tmp, *tP = ws.tmp + (int64_t)nb * nb;
      const unsigned tiles = (unsigned)(cdiv(w, cg::SYM_TILE) * cdiv(w, cg::SYM_TILE));
      hipLaunchKernelGGL(cg::sym_fwd_p_kernel, dim3(tiles), dim3(256), 0, s2, w, (const double *)(D + j * ldd + j),
                         ldd, (const double *)ws.dblk, (int64_t)nb, tP, (int64_t)nb);
      CG_TRY(hipGetLastError());
      hipLaunchKernelGGL(cg::sym_fwd_n_kernel, dim3(tiles), dim3(256), 0, s2, w, (const double *)tP, (int64_t)nb,
                         (const double *)ws.dblk, (int64_t)nb, tN, (int64_t)nb);
      CG_TRY(hipGetLastError());
      hipLaunchKernelGGL(cg::sym_fwd_l_kernel, dim3(tiles), dim3(256), 0, s2, w, (const double *)(A + j * lda + j),
                         lda, (const double *)tN, (int64_t)nb, D + j * ldd + j, ldd);
      CG_TRY(hipGetLastError());
    }
    if (m > 0) {
      // C <- C tril(L_bb)^-T;  C-dot <- (C-dot - C L-dot_bb^T) L_bb^-T   -- the next block's rows first
      const int m1 = std::min(m, nb);
      if (b > 0) CG_TRY(hipStreamWaitEvent(s2, side->low, 0));
      CG_TRY(panel_solve_t(m1, w, A + k * lda + j, lda, ws.dblk, nb, ws.panel, ws.part2, 32, s2));
      CG_TRY(gemm(false, true, m1, w, w, A + k * lda + j, lda, D + j * ldd + j, ldd, -1.0,
                  D + k * ldd + j, ldd, 1.0, ws.panel, nb, nullptr, 0, 0, ws.part2, 32, s2));
      CG_TRY(gemm(false, true, m1, w, w, ws.panel, nb, ws.dblk, nb, 1.0, nullptr, 0, 0.0,
                  D + k * ldd + j, ldd, nullptr, 0, 0, ws.part2, 32, s2));
      CG_TRY(hipEventRecord(side->top, s2));
      if (m > m1) {
        const int64_t kl = k + m1;
        CG_TRY(panel_solve_t(m - m1, w, A + kl * lda + j, lda, ws.dblk, nb, ws.panel + (int64_t)m1 * nb, nullptr,
                             128, s2));
        CG_TRY(gemm(false, true, m - m1, w, w, A + kl * lda + j, lda, D + j * ldd + j, ldd, -1.0,
                    D + kl * ldd + j, ldd, 1.0, ws.panel + (int64_t)m1 * nb, nb, nullptr, 0, 0, nullptr, 128, s2));
        CG_TRY(gemm(false, true, m - m1, w, w, ws.panel + (int64_t)m1 * nb, nb, ws.dblk, nb, 1.0, nullptr, 0,
                    0.0, D + kl * ldd + j, ldd, nullptr, 0, 0, nullptr, 128, s2));
      }
    }
    CG_TRY(hipEventRecord(side->panel, s2));
  }
  CG_TRY(hipStreamWaitEvent(s, side->panel, 0));
  const int blocks = (int)std::min<int64_t>(cdiv(n * n, 256), 4096);
  hipLaunchKernelGGL(cg::zero_upper_kernel, dim3(blocks), dim3(256), 0, s, n, A, lda);
  CG_TRY(hipGetLastError());
  hipLaunchKernelGGL(cg::zero_upper_kernel, dim3(blocks), dim3(256), 0, s, n, D, ldd);
  CG_TRY(hipGetLastError());
  return CHOL_SUCCESS;
}

size_t chol_batched_workspace_bytes(int precision, int batch, int64_t n_max) {
  if (!batched_prec_ok(precision) || batch <= 0 || n_max < 0 || n_max > cg::BATCH_NMAX) return 0;
  return batched_ws_bytes(batch, n_max, precision == CHOL_PREC_F32);
}

static int batched_common_checks(int precision, int batch, int64_t n_max) {
  if (precision == CHOL_PREC_F64_TRAIL_F32 || precision == CHOL_PREC_F64_TRAIL_BF16X3 ||
      precision == CHOL_PREC_F64_TRAIL_BF16X6 || precision == CHOL_PREC_F32_TRAIL_BF16X3)
    return CHOL_ERR_UNSUPPORTED;
  if (!batched_prec_ok(precision)) return -1;
  if (batch < 0) return -2;
  if (n_max < 0 || n_max > cg::BATCH_NMAX) return CHOL_ERR_UNSUPPORTED;
  return CHOL_SUCCESS;
}

int chol_factor_batched(int precision, int batch, const int64_t *n, void *const *A, const int64_t *lda,
                        int64_t n_max, int *info, void *workspace, size_t workspace_bytes, void *stream) {
  int rc = batched_common_checks(precision, batch, n_max);
  if (rc != CHOL_SUCCESS) return rc;
  if (batch == 0) return CHOL_SUCCESS;
  if (!n) return -3;
  if (!A) return -4;
  if (!lda) return -5;
  if (!info) return -7;
  cg::BatchArgs a{};
  a.op = cg::BATCH_FACTOR; a.batch = batch; a.f32 = precision == CHOL_PREC_F32; a.n = n; a.A = reinterpret_cast<double *const *>(A); a.lda = lda;
  a.info = info;
  return run_batched(a, n_max, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

int chol_rev_batched(int precision, int batch, const int64_t *n, const void *const *L, const int64_t *ldl,
                     void *const *A, const int64_t *lda, int64_t n_max, int sbar_form, void *workspace,
                     size_t workspace_bytes, void *stream) {
  int rc = batched_common_checks(precision, batch, n_max);
  if (rc != CHOL_SUCCESS) return rc;
  if (batch == 0) return CHOL_SUCCESS;
  if (!n) return -3;
  if (!L) return -4;
  if (!ldl) return -5;
  if (!A) return -6;
  if (!lda) return -7;
  if (sbar_form != CHOL_SBAR_SYM && sbar_form != CHOL_SBAR_TRIL) return -9;
  cg::BatchArgs a{};
  a.op = cg::BATCH_REV; a.batch = batch; a.f32 = precision == CHOL_PREC_F32; a.n = n; a.L = reinterpret_cast<const double *const *>(L);
  a.ldl = ldl; a.A = reinterpret_cast<double *const *>(A); a.lda = lda; a.sbar_form = sbar_form;
  return run_batched(a, n_max, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

int chol_fwd(int precision, int64_t n, const void *Lv, int64_t ldl, void *Av, int64_t lda, int nb,
             void *workspace, size_t workspace_bytes, void *stream) {
  if (f32_storage(precision))
    return f32_fwd(precision, n, Lv, ldl, Av, lda, nb, CHOL_DIAG_AUTO, CHOL_LAYOUT_ROW_MAJOR, workspace,
                   workspace_bytes, stream);
  return fwd_impl(precision, n, Lv, ldl, Av, lda, nb, CHOL_DIAG_AUTO, workspace, workspace_bytes, stream);
}

// ---------------------------------------------------------------------------------------------
// Entry points with a caller-chosen diagonal-block variant and storage layout.  Column-major
// storage of a matrix is row-major storage of its transpose: the input lower triangles are
// mirrored in place into the row-major lower triangle (and L, which the call may not modify, is
// copied that way into the workspace), the row-major sweep runs, and each lower-triangular output
// is moved back to the column-major lower triangle.

static size_t transposed_l_bytes(int64_t n) { return align_up((size_t)n * n * sizeof(double)); }

static hipError_t launch_lower_from_upper(int64_t n, const double *src, int64_t lds, double *dst, int64_t ldd,
                                          hipStream_t s) {
  const int blocks = (int)std::min<int64_t>(cdiv(n * n, 256), 4096);
  hipLaunchKernelGGL(cg::lower_from_upper_kernel, dim3(blocks), dim3(256), 0, s, n, src, lds, dst, ldd);
  return hipGetLastError();
}

static hipError_t launch_lower_to_upper(int64_t n, double *A, int64_t lda, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>(cdiv(n * n, 256), 4096);
  hipLaunchKernelGGL(cg::lower_to_upper_kernel, dim3(blocks), dim3(256), 0, s, n, A, lda);
  return hipGetLastError();
}

size_t chol_workspace_bytes_ex(int op, int precision, int64_t n, int nb, int layout) {
  if (layout != CHOL_LAYOUT_ROW_MAJOR && layout != CHOL_LAYOUT_COL_MAJOR) return 0;
  if (f32_storage(precision)) return chol_workspace_bytes(op, precision, n, nb);  // copies take the layout
  const size_t base = chol_workspace_bytes(op, precision, n, nb);
  if (base == 0 || layout == CHOL_LAYOUT_ROW_MAJOR || op == CHOL_OP_FACTOR) return base;
  return transposed_l_bytes(n) + base;
}

int chol_factor_ex(int precision, int64_t n, void *Av, int64_t lda, int nb, int layout, int *info,
                   void *workspace, size_t workspace_bytes, void *stream) {
  if (f32_storage(precision)) return f32_factor(precision, n, Av, lda, nb, layout, info, workspace, workspace_bytes, stream);
  if (layout != CHOL_LAYOUT_ROW_MAJOR && layout != CHOL_LAYOUT_COL_MAJOR) return -6;
  if (n > 0 && !info) return -7;
  if (layout == CHOL_LAYOUT_ROW_MAJOR || n <= 0)
    return chol_factor(precision, n, Av, lda, nb, info, workspace, workspace_bytes, stream);
  // A dry call (no workspace) validates every argument before anything is enqueued.
  const int chk = chol_factor(precision, n, Av, lda, nb, info, nullptr, 0, stream);
  if (chk != CHOL_ERR_WORKSPACE) return chk;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % WS_ALIGN) != 0 ||
      workspace_bytes < chol_workspace_bytes_ex(CHOL_OP_FACTOR, precision, n, nb, layout))
    return CHOL_ERR_WORKSPACE;  // before anything is enqueued
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *A = static_cast<double *>(Av);
  CG_TRY(launch_lower_from_upper(n, A, lda, A, lda, s));
  const int rc = chol_factor(precision, n, Av, lda, nb, info, workspace, workspace_bytes, stream);
  if (rc != CHOL_SUCCESS) return rc;
  CG_TRY(launch_lower_to_upper(n, A, lda, s));
  return CHOL_SUCCESS;
}

int chol_rev_ex(int precision, int64_t n, const void *Lv, int64_t ldl, void *Av, int64_t lda, int sbar_form,
                int nb, int diag, int layout, void *workspace, size_t workspace_bytes, void *stream) {
  if (f32_storage(precision))
    return f32_rev(precision, n, Lv, ldl, Av, lda, sbar_form, nb, diag, layout, workspace, workspace_bytes, stream);
  if (layout != CHOL_LAYOUT_ROW_MAJOR && layout != CHOL_LAYOUT_COL_MAJOR) return -10;
  if (layout == CHOL_LAYOUT_ROW_MAJOR || n <= 0)
    return rev_impl(precision, n, Lv, ldl, Av, lda, sbar_form, nb, diag, workspace, workspace_bytes, stream);
  const int chk = rev_impl(precision, n, Lv, ldl, Av, lda, sbar_form, nb, diag, nullptr, 0, stream);
  if (chk != CHOL_ERR_WORKSPACE) return chk;
  const size_t lt = transposed_l_bytes(n);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % WS_ALIGN) != 0 ||
      workspace_bytes < chol_workspace_bytes_ex(CHOL_OP_REV, precision, n, nb, layout))
    return CHOL_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *Lt = static_cast<double *>(workspace), *A = static_cast<double *>(Av);
  CG_TRY(launch_lower_from_upper(n, static_cast<const double *>(Lv), ldl, Lt, n, s));
  CG_TRY(launch_lower_from_upper(n, A, lda, A, lda, s));
  const int rc = rev_impl(precision, n, Lt, n, Av, lda, sbar_form, nb, diag, static_cast<char *>(workspace) + lt,
                          workspace_bytes - lt, stream);
  if (rc != CHOL_SUCCESS) return rc;
  if (sbar_form == CHOL_SBAR_TRIL) CG_TRY(launch_lower_to_upper(n, A, lda, s));  // the sym form is symmetric
  return CHOL_SUCCESS;
}

int chol_fwd_ex(int precision, int64_t n, const void *Lv, int64_t ldl, void *Av, int64_t lda, int nb, int diag,
                int layout, void *workspace, size_t workspace_bytes, void *stream) {
  if (f32_storage(precision))
    return f32_fwd(precision, n, Lv, ldl, Av, lda, nb, diag, layout, workspace, workspace_bytes, stream);
  if (layout != CHOL_LAYOUT_ROW_MAJOR && layout != CHOL_LAYOUT_COL_MAJOR) return -9;
  if (layout == CHOL_LAYOUT_ROW_MAJOR || n <= 0)
    return fwd_impl(precision, n, Lv, ldl, Av, lda, nb, diag, workspace, workspace_bytes, stream);
  const int chk = fwd_impl(precision, n, Lv, ldl, Av, lda, nb, diag, nullptr, 0, stream);
  if (chk != CHOL_ERR_WORKSPACE) return chk;
  const size_t lt = transposed_l_bytes(n);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % WS_ALIGN) != 0 ||
      workspace_bytes < chol_workspace_bytes_ex(CHOL_OP_FWD, precision, n, nb, layout))
    return CHOL_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *Lt = static_cast<double *>(workspace), *A = static_cast<double *>(Av);
  CG_TRY(launch_lower_from_upper(n, static_cast<const double *>(Lv), ldl, Lt, n, s));
  CG_TRY(launch_lower_from_upper(n, A, lda, A, lda, s));
  const int rc = fwd_impl(precision, n, Lt, n, Av, lda, nb, diag, static_cast<char *>(workspace) + lt,
                          workspace_bytes - lt, stream);
  if (rc != CHOL_SUCCESS) return rc;
  CG_TRY(launch_lower_to_upper(n, A, lda, s));
  return CHOL_SUCCESS;
}

int chol_fwd_batched(int precision, int batch, const int64_t *n, const void *const *L, const int64_t *ldl,
                     void *const *A, const int64_t *lda, int64_t n_max, void *workspace,
                     size_t workspace_bytes, void *stream) {
  int rc = batched_common_checks(precision, batch, n_max);
  if (rc != CHOL_SUCCESS) return rc;
  if (batch == 0) return CHOL_SUCCESS;
  if (!n) return -3;
  if (!L) return -4;
  if (!ldl) return -5;
  if (!A) return -6;
  if (!lda) return -7;
  cg::BatchArgs a{};
  a.op = cg::BATCH_FWD; a.batch = batch; a.f32 = precision == CHOL_PREC_F32; a.n = n; a.L = reinterpret_cast<const double *const *>(L);
  a.ldl = ldl; a.A = reinterpret_cast<double *const *>(A); a.lda = lda;
  return run_batched(a, n_max, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

int chol_factor_rev_batched(int precision, int batch, const int64_t *n, void *const *A, const int64_t *lda,
                            void *const *G, const int64_t *ldg, int64_t n_max, int sbar_form, int *info,
                            void *workspace, size_t workspace_bytes, void *stream) {
  int rc = batched_common_checks(precision, batch, n_max);
  if (rc != CHOL_SUCCESS) return rc;
  if (batch == 0) return CHOL_SUCCESS;
  if (!n) return -3;
  if (!A) return -4;
  if (!lda) return -5;
  if (!G) return -6;
  if (!ldg) return -7;
  if (sbar_form != CHOL_SBAR_SYM && sbar_form != CHOL_SBAR_TRIL) return -9;
  if (!info) return -10;
  cg::BatchArgs a{};
  a.op = cg::BATCH_FACTOR_REV; a.batch = batch; a.f32 = precision == CHOL_PREC_F32; a.n = n;
  a.A = reinterpret_cast<double *const *>(A); a.lda = lda; a.G = reinterpret_cast<double *const *>(G);
  a.ldg = ldg; a.sbar_form = sbar_form; a.info = info;
  return run_batched(a, n_max, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

int chol_gp_nll_batched(int precision, int batch, const int64_t *n, void *const *A, const int64_t *lda,
                        const void *const *y, void *const *G, const int64_t *ldg, void *f, int64_t n_max,
                        int *info, void *workspace, size_t workspace_bytes, void *stream) {
  int rc = batched_common_checks(precision, batch, n_max);
  if (rc != CHOL_SUCCESS) return rc;
  if (batch == 0) return CHOL_SUCCESS;
  if (!n) return -3;
  if (!A) return -4;
  if (!lda) return -5;
  if (!y) return -6;
  if (!G) return -7;
  if (!ldg) return -8;
  if (!f) return -9;
  if (!info) return -11;
  cg::BatchArgs a{};
  a.op = cg::BATCH_GP; a.batch = batch; a.f32 = precision == CHOL_PREC_F32; a.n = n; a.A = reinterpret_cast<double *const *>(A); a.lda = lda;
  a.y = reinterpret_cast<const double *const *>(y); a.G = reinterpret_cast<double *const *>(G); a.ldg = ldg;
  a.f = static_cast<double *>(f); a.info = info;
  return run_batched(a, n_max, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

}  // extern "C"

// ---------------------------------------------------------------------------------------------
// FP32 storage for the single-matrix calls (CHOL_PREC_F32, CHOL_PREC_F32_TRAIL_BF16X3): the float
// inputs are widened into FP64 row-major copies at the front of the workspace (from either
// layout), the FP64-storage sweep runs on the copies (in CHOL_PREC_F64 or
// CHOL_PREC_F64_TRAIL_BF16X3) with the rest of the workspace, and each output is rounded to float
// once into the caller's array, in its layout.  Arguments are validated (a dry call of the FP64
// sweep on the copies) before anything is enqueued.
namespace {

int f64_inner(int precision) { return precision == CHOL_PREC_F32 ? CHOL_PREC_F64 : CHOL_PREC_F64_TRAIL_BF16X3; }
size_t copy_bytes(int64_t n) { return align_up((size_t)n * n * sizeof(double)); }
bool aligned4(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }
bool layout_ok(int layout) { return layout == CHOL_LAYOUT_ROW_MAJOR || layout == CHOL_LAYOUT_COL_MAJOR; }
unsigned elem_blocks(int64_t n) { return (unsigned)std::min<int64_t>(cdiv(n * n, 256), 4096); }

hipError_t widen(int64_t n, const void *src, int64_t lds, int layout, double *dst, hipStream_t s) {
  hipLaunchKernelGGL(cg::widen_lower_kernel, dim3(elem_blocks(n)), dim3(256), 0, s, n, static_cast<const float *>(src),
                     lds, layout == CHOL_LAYOUT_COL_MAJOR ? 1 : 0, dst, n);
  return hipGetLastError();
}

hipError_t narrow(int64_t n, const double *src, void *dst, int64_t ldd, int layout, hipStream_t s) {
  hipLaunchKernelGGL(cg::narrow_kernel, dim3(elem_blocks(n)), dim3(256), 0, s, n, src, n, static_cast<float *>(dst),
                     ldd, layout == CHOL_LAYOUT_COL_MAJOR ? 1 : 0);
  return hipGetLastError();
}

bool ws_ok(void *ws, size_t wsb, size_t need) {
  return ws && (reinterpret_cast<uintptr_t>(ws) % WS_ALIGN) == 0 && wsb >= need;
}

int f32_factor(int precision, int64_t n, void *A, int64_t lda, int nb, int layout, int *info, void *ws,
               size_t wsb, void *stream) {
  if (n < 0 || n > (int64_t)1 << 30) return -2;
  if (n == 0) return CHOL_SUCCESS;
  if (!A || !aligned4(A)) return -3;
  if (lda < n) return -4;
  if (!nb_ok(nb)) return -5;
  if (!layout_ok(layout)) return -6;
  if (!info) return -7;
  if (!ws_ok(ws, wsb, chol_workspace_bytes(CHOL_OP_FACTOR, precision, n, nb))) return CHOL_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *W = static_cast<double *>(ws);
  const size_t cb = copy_bytes(n);
  CG_TRY(widen(n, A, lda, layout, W, s));
  const int rc = chol_factor(f64_inner(precision), n, W, n, nb, info, static_cast<char *>(ws) + cb, wsb - cb, stream);
  if (rc != CHOL_SUCCESS) return rc;
  CG_TRY(narrow(n, W, A, lda, layout, s));
  return CHOL_SUCCESS;
}

int f32_rev(int precision, int64_t n, const void *L, int64_t ldl, void *A, int64_t lda, int sbar_form, int nb,
            int diag, int layout, void *ws, size_t wsb, void *stream) {
  if (n < 0 || n > (int64_t)1 << 30) return -2;
  if (n == 0) return CHOL_SUCCESS;
  if (!L || !aligned4(L)) return -3;
  if (ldl < n) return -4;
  if (!A || !aligned4(A)) return -5;
  if (lda < n) return -6;
  if (!layout_ok(layout)) return -10;
  const size_t cb = copy_bytes(n);
  double *Wl = static_cast<double *>(ws), *Wa = reinterpret_cast<double *>(static_cast<char *>(ws) + cb);
  const int inner = f64_inner(precision);
  double *const fake = reinterpret_cast<double *>((uintptr_t)WS_ALIGN);  // validation only: never touched
  const int chk = rev_impl(inner, n, fake, n, fake, n, sbar_form, nb, diag, nullptr, 0, stream);
  if (chk != CHOL_ERR_WORKSPACE) return chk;
  if (!ws_ok(ws, wsb, chol_workspace_bytes(CHOL_OP_REV, precision, n, nb))) return CHOL_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  CG_TRY(widen(n, L, ldl, layout, Wl, s));
  CG_TRY(widen(n, A, lda, layout, Wa, s));
  const int rc = rev_impl(inner, n, Wl, n, Wa, n, sbar_form, nb, diag, static_cast<char *>(ws) + 2 * cb,
                          wsb - 2 * cb, stream);
  if (rc != CHOL_SUCCESS) return rc;
  CG_TRY(narrow(n, Wa, A, lda, layout, s));
  return CHOL_SUCCESS;
}

int f32_fwd(int precision, int64_t n, const void *L, int64_t ldl, void *A, int64_t lda, int nb, int diag,
            int layout, void *ws, size_t wsb, void *stream) {
  if (n < 0 || n > (int64_t)1 << 30) return -2;
  if (n == 0) return CHOL_SUCCESS;
  if (!L || !aligned4(L)) return -3;
  if (ldl < n) return -4;
  if (!A || !aligned4(A)) return -5;
  if (lda < n) return -6;
  if (!layout_ok(layout)) return -9;
  const size_t cb = copy_bytes(n);
  double *Wl = static_cast<double *>(ws), *Wa = reinterpret_cast<double *>(static_cast<char *>(ws) + cb);
  const int inner = f64_inner(precision);
  double *const fake = reinterpret_cast<double *>((uintptr_t)WS_ALIGN);
  const int chk = fwd_impl(inner, n, fake, n, fake, n, nb, diag, nullptr, 0, stream);
  if (chk != CHOL_ERR_WORKSPACE) return chk;
  if (!ws_ok(ws, wsb, chol_workspace_bytes(CHOL_OP_FWD, precision, n, nb))) return CHOL_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  CG_TRY(widen(n, L, ldl, layout, Wl, s));
  CG_TRY(widen(n, A, lda, layout, Wa, s));
  const int rc = fwd_impl(inner, n, Wl, n, Wa, n, nb, diag, static_cast<char *>(ws) + 2 * cb, wsb - 2 * cb, stream);
  if (rc != CHOL_SUCCESS) return rc;
  CG_TRY(narrow(n, Wa, A, lda, layout, s));
  return CHOL_SUCCESS;
}

int f32_factor_fwd(int precision, int64_t n, void *A, int64_t lda, void *D, int64_t ldd, int nb, int *info,
                   void *ws, size_t wsb, void *stream) {
  if (n < 0 || n > (int64_t)1 << 30) return -2;
  if (n == 0) return CHOL_SUCCESS;
  if (!A || !aligned4(A)) return -3;
  if (lda < n) return -4;
  if (!D || !aligned4(D)) return -5;
  if (ldd < n) return -6;
  if (!nb_ok(nb)) return -7;
  if (!info) return -8;
  if (!ws_ok(ws, wsb, chol_workspace_bytes(CHOL_OP_FWD, precision, n, nb))) return CHOL_ERR_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t cb = copy_bytes(n);
  double *Wa = static_cast<double *>(ws), *Wd = reinterpret_cast<double *>(static_cast<char *>(ws) + cb);
  CG_TRY(widen(n, A, lda, CHOL_LAYOUT_ROW_MAJOR, Wa, s));
  CG_TRY(widen(n, D, ldd, CHOL_LAYOUT_ROW_MAJOR, Wd, s));
  const int rc = chol_factor_fwd(f64_inner(precision), n, Wa, n, Wd, n, nb, info, static_cast<char *>(ws) + 2 * cb,
                                 wsb - 2 * cb, stream);
  if (rc != CHOL_SUCCESS) return rc;
  CG_TRY(narrow(n, Wa, A, lda, CHOL_LAYOUT_ROW_MAJOR, s));
  CG_TRY(narrow(n, Wd, D, ldd, CHOL_LAYOUT_ROW_MAJOR, s));
  return CHOL_SUCCESS;
}

}  // namespace
