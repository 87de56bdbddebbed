/*
 * cholgrad.h -- C ABI of libcholgrad: blocked Cholesky factorisation and blocked forward- and
 * reverse-mode propagation of Cholesky derivatives on an AMD Instinct MI355X (gfx950).
 *
 * Method: I. Murray, "Differentiation of the Cholesky decomposition", arXiv:1602.07527 (2016).
 * The computation chain is x -> Sigma -> L -> f (Sec. 2, eqn (computation)):
 *   chol_factor : Sigma -> L          lower-triangular L, positive diagonal, L L^T = Sigma (Sec. 1)
 *   chol_fwd    : (L, Sigma-dot) -> L-dot      forward propagator (Sec. 2; eqn (symfwd))
 *   chol_rev    : (L, L-bar)     -> Sigma-bar  reverse propagator (Sec. 2; eqns (symrev), (symrevtril))
 * computed with Level-3 block algorithms derived from the blocked factorisation (Sec. 4.2).
 *
 * Conventions for every entry point
 *   - Matrices are DEVICE pointers, row-major: element (i, j) of an n x n matrix lives at
 *     A[i * ld + j], with ld >= max(1, n).  Storage type is double for the CHOL_PREC_F64* modes
 *     and float for CHOL_PREC_F32.
 *   - Only the lower triangle (i >= j) of each input matrix is read (Sec. 4.1: the algorithms only
 *     inspect the lower triangle).  Sigma-dot is symmetric; its lower triangle defines it (Sec. 3).
 *   - Outputs overwrite the array in place, as the paper's algorithms do.  The strict upper
 *     triangle of an output is written as documented per call (never left as garbage).
 *   - The caller owns all memory, including the workspace (size from chol_workspace_bytes, base
 *     aligned to 256 bytes).  The library never allocates, frees or synchronises inside these calls;
 *     all work is enqueued on `stream` (a hipStream_t; NULL means the default stream) in order.
 *     Calls on distinct (stream, workspace) pairs may run concurrently.  The device of `stream`
 *     must be the current device.  The single-matrix calls additionally run their diagonal-block
 *     chain on an auxiliary stream (default priority) ordered against `stream` with events: one
 *     auxiliary stream and three events per (device, calling stream) pair for up to 8 calling
 *     streams per device (further calling streams share them), created on first use and kept for
 *     the process.  Host-side enqueueing of these calls is serialised by a library mutex.
 *   - Return value: CHOL_SUCCESS (0), or a negative status checked synchronously on the host
 *     before anything is enqueued:  -i  means argument i (1-based) is invalid;  CHOL_ERR_* below.
 *     Numerical breakdown of chol_factor is reported asynchronously through `info`.
 *   - n == 0 is a no-op that returns CHOL_SUCCESS.
 *   - nb is the block size of the Level-3 sweep (Sec. 4.2, N_b): 0 selects a width measured per
 *     sweep and size on MI355X -- chol_rev and chol_fwd 256; chol_factor and chol_factor_fwd
 *     256 for 256 < n <= 512 and n >= 3072, 128 otherwise; at
 *     most 128 with CHOL_DIAG_LEVEL2 -- and chol_workspace_bytes with nb = 0 returns the size for
 *     nb = 256, which holds any of them; otherwise 16 <= nb <= 256 and nb % 16 == 0
 *     (chol_rev_noalloc: nb <= 128, 0 selects 128).  The result does not depend on nb beyond
 *     rounding (the column partition is arbitrary, Sec. 4.2).  Blocks wider than 128 factor and
 *     invert their diagonal block as two halves (Sec. 4.2's remark that the unblocked routine may
 *     be replaced by a recursive one for large blocks); the Level-2 diagonal-block variant
 *     (CHOL_DIAG_LEVEL2) is limited to nb <= 128 and returns CHOL_ERR_UNSUPPORTED above.
 */
#ifndef CHOLGRAD_H
#define CHOLGRAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHOLGRAD_VERSION 100

/* Status codes (negative small integers -i name the invalid argument instead). */
#define CHOL_SUCCESS 0
#define CHOL_ERR_HIP (-101)          /* a HIP runtime call or kernel launch failed           */
#define CHOL_ERR_WORKSPACE (-102)    /* workspace NULL, too small, or not 256-byte aligned    */
#define CHOL_ERR_UNSUPPORTED (-103)  /* precision / form / size combination not implemented */
#define CHOL_ERR_TOO_LARGE (-104)    /* beyond the static scratch of chol_rev_noalloc        */

/* Precision of the call.
 *   CHOL_PREC_F64 : double storage; every step in FP64 (FP64 MFMA for the contractions).
 *   CHOL_PREC_F32 : float storage (matrices, vectors and losses).  Single-matrix calls and
 *                   chol_fwd_batched: each input's lower triangle is widened to FP64 (single-
 *                   matrix calls: n*n doubles of the workspace per matrix argument, included by
 *                   chol_workspace_bytes), computed exactly as in CHOL_PREC_F64 and rounded to
 *                   float once on output, so the result is the FP64 result for the float input to
 *                   within float rounding.  The other batched calls compute in FP64 within each
 *                   64-wide block step and round every value they store to float (the problems'
 *                   arrays are updated in place between steps): against the FP64 result for the
 *                   float inputs, relative Frobenius errors <= 3e-7 for L, <= 7e-6 for Sigma-bar
 *                   and <= 6e-7 for f on well-conditioned problems (kappa <= ~40; measured
 *                   3.4e-8, 6.8e-7, 5.6e-8).
 *   CHOL_PREC_F64_TRAIL_F32 : double storage, single-matrix calls only (batched calls return
 *                   CHOL_ERR_UNSUPPORTED, as for the next mode).  The trailing contractions -- the block-column
 *                   updates of chol_factor and chol_fwd and the panel contraction and SYRK of
 *                   chol_rev -- round their operands to FP32 and run on FP32 MFMA with FP32
 *                   accumulation within one launch's K range; diagonal blocks, block inverses,
 *                   panel solves, split-K sums and every stored value stay FP64.  An
 *                   approximation of the FP64 result: on the N = 16384 squared-exponential
 *                   workload (condition number ~1e5) the stated relative Frobenius errors are
 *                   <= 3e-4 for L, <= 1e-4 for Sigma-bar and <= 3e-5 for L-dot (chol_rev and
 *                   chol_fwd given the exact L; measured on MI355X 7.6e-5, 7.1e-6, 2.6e-6).
 *                   Factor and chol_rev both in this mode, each on its own L, on squared-
 *                   exponential kernels in 2-D with n <= 4096 and condition numbers up to ~2e6:
 *                   <= 6e-4 for L and <= 2e-2 for Sigma-bar per problem (measured max 2.7e-4
 *                   and 9.2e-3; the error grows with the condition number).
 *   CHOL_PREC_F64_TRAIL_BF16X3 : as CHOL_PREC_F64_TRAIL_F32, but the trailing contractions split
 *                   each operand into bfloat16 hi + lo parts (hi = bf16(fp32(x)),
 *                   lo = bf16(fp32(x) - hi)) and take hi*hi + hi*lo + lo*hi on bfloat16 MFMA
 *                   with FP32 accumulation (~16 significant bits per operand).  Stated relative
 *                   errors on the same N = 16384 workload: <= 1e-3 for L, <= 3e-4 for Sigma-bar
 *                   and L-dot (measured 3.0e-4, 2.3e-5, 2.1e-5).
 *   CHOL_PREC_F64_TRAIL_BF16X6 : as CHOL_PREC_F64_TRAIL_BF16X3 with three bfloat16 parts per operand
 *                   (hi, mid = bf16(fp32(x) - hi), lo = bf16(fp32(x) - hi - mid)) and the six
 *                   products hi*hi + hi*mid + mid*hi + hi*lo + lo*hi + mid*mid (~24 significant
 *                   bits per operand, as FP32, on the bfloat16 matrix units).  Single-matrix calls.
 *                   Stated relative errors on the N = 16384 workload: <= 5e-4 for L, <= 2e-4 for
 *                   Sigma-bar, <= 3e-5 for L-dot (measured 4.6e-5, 2.0e-5, 1.9e-6).
 *   CHOL_PREC_F32_TRAIL_BF16X3 : float storage as CHOL_PREC_F32, computed as
 *                   CHOL_PREC_F64_TRAIL_BF16X3 on the widened copies (errors as that mode's, plus
 *                   the final rounding to float).  Single-matrix calls. */
#define CHOL_PREC_F64 0
#define CHOL_PREC_F32 1
#define CHOL_PREC_F64_TRAIL_F32 2
#define CHOL_PREC_F64_TRAIL_BF16X3 3
#define CHOL_PREC_F64_TRAIL_BF16X6 4
#define CHOL_PREC_F32_TRAIL_BF16X3 5

/* Which reverse-mode output (Sec. 3, eqns (symrev) and (symrevtril); S = L^-T Phi(L^T Lbar) L^-1):
 *   CHOL_SBAR_SYM  : (S + S^T)/2 in both triangles -- the symmetric gradient, for which
 *                    Tr(Lbar^T Ldot) = sum_ij Sbar_ij Sdot_ij holds for any symmetric Sigma-dot.
 *   CHOL_SBAR_TRIL : T = Phi(S + S^T), the paper's lower-triangular in-place output; the strict
 *                    upper triangle is set to 0.  T + T^T - diag(T) is eqn (symrev)'s form.     */
#define CHOL_SBAR_SYM 0
#define CHOL_SBAR_TRIL 1

/* Diagonal-block variant of chol_rev_ex and chol_fwd_ex (Sec. 4.2 leaves the routine for the
 * diagonal block open; both variants give the same result up to rounding):
 *   CHOL_DIAG_SYMBOLIC : the block's own symbolic form from its inverse D^-1 -- reverse
 *                        D-bar <- D^-T Phi(D^T D-bar) D^-1 (eqn (symrev) on the block), forward
 *                        D-dot <- D Phi(D^-1 D-dot D^-T) (eqn (symfwd)) -- as small MFMA products;
 *                        every launch of the sweep on the caller's stream.
 *   CHOL_DIAG_LEVEL2   : Sec. 4.1's unblocked chol_unblocked_rev / chol_unblocked_fwd (with the Phi
 *                        halving of the diagonal) in one workgroup per block, on a side stream
 *                        overlapped with the next step's trailing products.
 *   CHOL_DIAG_AUTO     : the library's choice; currently the symbolic form for every n and nb,
 *                        the faster of the two on MI355X at n = 256 to 16384, nb = 32 to 128
 *                        (the Level-2 variant holds blocks of at most 128: nb > 128 with
 *                        CHOL_DIAG_LEVEL2 returns CHOL_ERR_UNSUPPORTED). */
#define CHOL_DIAG_AUTO 0
#define CHOL_DIAG_SYMBOLIC 1
#define CHOL_DIAG_LEVEL2 2

/* Storage layout of the n x n matrices of chol_factor_ex, chol_rev_ex and chol_fwd_ex (the other
 * entry points are row-major):
 *   CHOL_LAYOUT_ROW_MAJOR : element (i, j) at A[i*ld + j];
 *   CHOL_LAYOUT_COL_MAJOR : element (i, j) at A[i + j*ld], LAPACK's layout (equivalently: the
 *                           upper-triangular factor U = L^T in row-major storage).
 * In both layouts the lower triangle of each input is read and every output has the same meaning
 * (L and L-dot lower triangular with a zero strict upper triangle; Sigma-bar in the chosen form).
 * The column-major calls convert in place with element-wise kernels (a few extra passes over each
 * n x n array); chol_rev_ex and chol_fwd_ex also copy L, transposed, into the workspace (n*n more
 * doubles, included by chol_workspace_bytes_ex). */
#define CHOL_LAYOUT_ROW_MAJOR 0
#define CHOL_LAYOUT_COL_MAJOR 1

/* Operation codes for chol_workspace_bytes. */
#define CHOL_OP_FACTOR 0
#define CHOL_OP_REV 1
#define CHOL_OP_FWD 2

/* Bytes of device workspace that a call with these parameters needs (0 for n == 0).  Returns 0
 * as well for invalid parameters; the call itself then reports the error. */
size_t chol_workspace_bytes(int op, int precision, int64_t n, int nb);

/* The same for a storage layout (CHOL_LAYOUT_*); 0 for an unknown layout.  Row-major: equal to
 * chol_workspace_bytes. */
size_t chol_workspace_bytes_ex(int op, int precision, int64_t n, int nb, int layout);

/*
 * chol_factor -- blocked Cholesky factorisation, Sec. 4.2 chol_blocked (left-looking DPOTRF):
 *   per block column: D <- D - tril(R R^T);  D <- chol_unblocked(D);  C <- C - B R^T;
 *   C <- C tril(D)^-T.
 *   A     in : tril(A) = tril(Sigma), Sigma symmetric positive definite (n x n, lda).
 *        out : tril(A) = L; the strict upper triangle is set to 0.
 *   info  device pointer to one int, written by the call: 0 on success, or k > 0 when the leading
 *         minor of order k is not positive definite (first non-positive pivot, 1-based, as
 *         LAPACK); L is then undefined from column k on.  May not be NULL.
 *   Arguments: 1 precision, 2 n, 3 A, 4 lda, 5 nb, 6 info, 7 workspace, 8 workspace_bytes, 9 stream.
 */
int chol_factor(int precision, int64_t n, void *A, int64_t lda, int nb, int *info,
                void *workspace, size_t workspace_bytes, void *stream);

/* chol_factor with the storage layout of A chosen by the caller (CHOL_LAYOUT_*, argument 6; any
 * other value returns -6; info is argument 7, -7 when NULL).  chol_factor(...) is
 * chol_factor_ex(..., CHOL_LAYOUT_ROW_MAJOR, ...). */
int chol_factor_ex(int precision, int64_t n, void *A, int64_t lda, int nb, int layout, int *info,
                   void *workspace, size_t workspace_bytes, void *stream);

/*
 * chol_rev -- reverse-mode propagation Sigma-bar(L, L-bar), Sec. 4.2 chol_blocked_rev, right to
 * left: per block C-bar <- C-bar D^-1 (panel solve), D-bar <- D-bar - tril(C-bar^T C), the
 * diagonal block's adjoint (CHOL_DIAG_AUTO's variant), and the knock-on updates of everything to
 * the left, gathered into one product per step.
 *   L     in : lower-triangular factor with positive diagonal (n x n, ldl); not modified.
 *   A     in : tril(A) = L-bar.   out: Sigma-bar in the form selected by sbar_form.
 *   L and A must not overlap.  A non-positive diagonal in L gives Inf/NaN, never a hang.
 *   Arguments: 1 precision, 2 n, 3 L, 4 ldl, 5 A, 6 lda, 7 sbar_form, 8 nb, 9 workspace,
 *              10 workspace_bytes, 11 stream.
 */
int chol_rev(int precision, int64_t n, const void *L, int64_t ldl, void *A, int64_t lda,
             int sbar_form, int nb, void *workspace, size_t workspace_bytes, void *stream);

/* chol_rev with the diagonal-block variant (CHOL_DIAG_*, argument 9; any other value returns -9)
 * and the storage layout of L and A (CHOL_LAYOUT_*, argument 10; any other value returns -10)
 * chosen by the caller; the remaining arguments as chol_rev's, shifted by two from workspace on
 * (workspace sized by chol_workspace_bytes_ex).  chol_rev(...) is
 * chol_rev_ex(..., CHOL_DIAG_AUTO, CHOL_LAYOUT_ROW_MAJOR, ...). */
int chol_rev_ex(int precision, int64_t n, const void *L, int64_t ldl, void *A, int64_t lda,
                int sbar_form, int nb, int diag, int layout, void *workspace, size_t workspace_bytes,
                void *stream);

/*
 * chol_rev_noalloc -- chol_rev for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same sweep, with the
 * symbolic diagonal-block variant, but its workspace is a static device array of the library
 * (45 MiB, held on each device the call runs on until the process ends) instead of a caller's
 * buffer.  The call allocates nothing, frees nothing and creates no stream or event; the device
 * address of the array is looked up once per device, on the first call with that device current.
 *   n  <= 4096 (CHOL_ERR_TOO_LARGE above), nb <= 128 (0 selects 128; -8 otherwise).
 *   Every call on a device shares that device's array: calls that overlap in time on one device
 *   (on different streams, or from different host threads) race and give wrong results; calls
 *   ordered on one stream are safe.  The array keeps the last call's contents; nothing in it needs
 *   to start at zero.
 *   Other arguments, results and errors as chol_rev (row-major storage).
 *   Arguments: 1 precision, 2 n, 3 L, 4 ldl, 5 A, 6 lda, 7 sbar_form, 8 nb, 9 stream.
 */
int chol_rev_noalloc(int precision, int64_t n, const void *L, int64_t ldl, void *A, int64_t lda,
                     int sbar_form, int nb, void *stream);

/*
 * chol_fwd -- forward-mode propagation L-dot(L, Sigma-dot), Sec. 4.2 chol_blocked_fwd, left to
 * right, with the diagonal block's tangent in CHOL_DIAG_AUTO's variant:
 *   D-dot <- D-dot - tril(R-dot R^T + R R-dot^T); D-dot <- chol_unblocked_fwd(D, D-dot);
 *   C-dot <- C-dot - B-dot R^T - B R-dot^T;  C-dot <- (C-dot - C D-dot^T) D^-T.
 *   L     in : lower-triangular factor with positive diagonal (n x n, ldl); not modified.
 *   A     in : tril(A) = tril(Sigma-dot).  out: tril(A) = L-dot; strict upper triangle set to 0.
 *   L and A must not overlap.
 *   Arguments: 1 precision, 2 n, 3 L, 4 ldl, 5 A, 6 lda, 7 nb, 8 workspace, 9 workspace_bytes,
 *              10 stream.
 */
int chol_fwd(int precision, int64_t n, const void *L, int64_t ldl, void *A, int64_t lda, int nb,
             void *workspace, size_t workspace_bytes, void *stream);

/* chol_fwd with the diagonal-block variant (CHOL_DIAG_*, argument 8; else -8) and the storage
 * layout of L and A (CHOL_LAYOUT_*, argument 9; else -9) chosen by the caller; workspace sized by
 * chol_workspace_bytes_ex.  chol_fwd(...) is chol_fwd_ex(..., CHOL_DIAG_AUTO, CHOL_LAYOUT_ROW_MAJOR, ...). */
int chol_fwd_ex(int precision, int64_t n, const void *L, int64_t ldl, void *A, int64_t lda, int nb,
                int diag, int layout, void *workspace, size_t workspace_bytes, void *stream);

/*
 * chol_factor_fwd -- chol_factor and chol_fwd in ONE left-to-right sweep (Sec. 4.2: the forward
 * updates of chol_blocked_fwd accumulated during the factorisation, as the paper remarks they can
 * be): at block column b every column to its left already holds its final L and L-dot, which is
 * all both updates need, so L is read once and POTF2's block inverse serves the forward step.
 *   A     in : tril(A) = tril(Sigma).      out: tril(A) = L; strict upper triangle set to 0.
 *   D     in : tril(D) = tril(Sigma-dot).  out: tril(D) = L-dot; strict upper triangle set to 0.
 *   info  as chol_factor (L-dot is undefined when info != 0).  A and D must not overlap.
 *   Workspace: chol_workspace_bytes(CHOL_OP_FWD, ...).
 *   Arguments: 1 precision, 2 n, 3 A, 4 lda, 5 D, 6 ldd, 7 nb, 8 info, 9 workspace,
 *              10 workspace_bytes, 11 stream.
 */
int chol_factor_fwd(int precision, int64_t n, void *A, int64_t lda, void *D, int64_t ldd, int nb, int *info,
                    void *workspace, size_t workspace_bytes, void *stream);

/*
 * Batched forms: many independent problems per call, Sec. 4.2's blocked algorithms applied per
 * problem.  chol_factor_batched, chol_rev_batched, chol_factor_rev_batched and
 * chol_gp_nll_batched run step-synchronous on 64-wide blocks, in FP64 or FP32 storage: a plan
 * built on the device orders the problems largest first, then each block step is one grouped
 * launch per kind over every problem that has that step (block-column updates and panel products
 * as 64 x 64 MFMA tiles, diagonal blocks one wave each); a batch of 1024 problems or more runs as
 * two such plans, the even- and the odd-indexed problems, one on `stream` and one on a side stream
 * of the library that `stream` then waits for (the call stays ordered on `stream` like every
 * other).  chol_fwd_batched runs one persistent launch (one workgroup per problem at a time,
 * nb = 128).  All per-problem arguments are DEVICE arrays
 * with `batch` entries: n[b] is the size of problem b, A[b] (and L[b], y[b], G[b]) are device
 * pointers to its row-major data with leading dimensions lda[b] (ldl[b], ldg[b]) >= n[b].  n_max
 * (host value, <= 512) bounds every n[b]; n_max above 512 returns CHOL_ERR_UNSUPPORTED.  A problem
 * whose size is outside [0, n_max] or whose leading dimension is smaller than its size is skipped
 * (its info entry, where there is one, becomes -1).  Each problem's result does not depend on the
 * batch it is in.  Workspace: chol_batched_workspace_bytes(precision, batch, n_max) bytes, 256-byte
 * aligned: the larger of the two paths' needs -- the step-synchronous path's plan, the inverses
 * of every problem's 64-blocks and two vectors per problem (about 528 * n_max bytes per problem:
 * 554 MB for 2048 problems at n_max = 512) and the persistent kernel's scratch (1.05 MB per
 * workgroup, one workgroup per problem up to 256: 268 MB), which for CHOL_PREC_F32 adds
 * 16 * n_max^2 bytes of FP64 staging per workgroup (1.34 GB in all for 256 or more problems at
 * n_max = 512).
 * Semantics per problem are those of the single-matrix calls above.
 */
size_t chol_batched_workspace_bytes(int precision, int batch, int64_t n_max);

/* Arguments: 1 precision, 2 batch, 3 n, 4 A, 5 lda, 6 n_max, 7 info (device, batch ints),
 *            8 workspace, 9 workspace_bytes, 10 stream. */
int chol_factor_batched(int precision, int batch, const int64_t *n, void *const *A, const int64_t *lda,
                        int64_t n_max, int *info, void *workspace, size_t workspace_bytes, void *stream);

/* Arguments: 1 precision, 2 batch, 3 n, 4 L, 5 ldl, 6 A, 7 lda, 8 n_max, 9 sbar_form, 10 workspace,
 *            11 workspace_bytes, 12 stream. */
int chol_rev_batched(int precision, int batch, const int64_t *n, const void *const *L, const int64_t *ldl,
                     void *const *A, const int64_t *lda, int64_t n_max, int sbar_form, void *workspace,
                     size_t workspace_bytes, void *stream);

/* Arguments: 1 precision, 2 batch, 3 n, 4 L, 5 ldl, 6 A, 7 lda, 8 n_max, 9 workspace,
 *            10 workspace_bytes, 11 stream. */
int chol_fwd_batched(int precision, int batch, const int64_t *n, const void *const *L, const int64_t *ldl,
                     void *const *A, const int64_t *lda, int64_t n_max, void *workspace,
                     size_t workspace_bytes, void *stream);

/*
 * chol_factor_rev_batched -- a factorisation followed by the reverse sweep on its own factor, per
 * problem, in one launch (the Sigma -> L forward pass and the L-bar -> Sigma-bar backward pass of
 * Sec. 2 with L kept on the device between them):
 *   A[b]   in: tril = Sigma_b.  out: L_b (strict upper set to 0), left in place for later use.
 *   G[b]   in: tril = L-bar_b.  out: Sigma-bar_b in the form selected by sbar_form (untouched when
 *          info[b] != 0).
 *   info   out: device array of batch ints (LAPACK convention; -1 for a skipped problem).
 *   Arguments: 1 precision, 2 batch, 3 n, 4 A, 5 lda, 6 G, 7 ldg, 8 n_max, 9 sbar_form, 10 info,
 *              11 workspace, 12 workspace_bytes, 13 stream.
 */
int chol_factor_rev_batched(int precision, int batch, const int64_t *n, void *const *A, const int64_t *lda,
                            void *const *G, const int64_t *ldg, int64_t n_max, int sbar_form, int *info,
                            void *workspace, size_t workspace_bytes, void *stream);

/*
 * chol_gp_nll_batched -- the whole x -> Sigma -> L -> f -> Sigma-bar chain of Sec. 2 per problem, in
 * one launch, for the Gaussian-process style loss
 *     f_b = sum_i log L_ii + (1/2) |L^-1 y_b|^2      (= (1/2) log det Sigma + (1/2) y^T Sigma^-1 y)
 * whose reverse-mode input is L-bar = diag(1/L_ii) - tril(w z^T), z = L^-1 y, w = L^-T z:
 *   A[b]   in: tril = Sigma_b.  out: L_b (strict upper set to 0).
 *   y[b]   in: n[b] values (double, or float for CHOL_PREC_F32).
 *   G[b]   out: Sigma-bar_b = df_b/dSigma_b, the symmetric gradient in both triangles
 *          (= (Sigma^-1 - a a^T)/2 with a = Sigma^-1 y).
 *   f      out: device array of batch values (double, or float for CHOL_PREC_F32).
 *   info   out: device array of batch ints (LAPACK convention; f = NaN and G untouched when > 0).
 *   Arguments: 1 precision, 2 batch, 3 n, 4 A, 5 lda, 6 y, 7 G, 8 ldg, 9 f, 10 n_max, 11 info,
 *              12 workspace, 13 workspace_bytes, 14 stream.
 */
int chol_gp_nll_batched(int precision, int batch, const int64_t *n, void *const *A, const int64_t *lda,
                        const void *const *y, void *const *G, const int64_t *ldg, void *f, int64_t n_max,
                        int *info, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Benchmark instrumentation (creates HIP events, so not for allocation-free paths).
 * chol_profile_begin: until chol_profile_end, each launch of a sweep's panel contraction -- the
 *   kernel that carries nearly all of a sweep's flops -- is bracketed by a pair of hipEvents on the
 *   call's stream, for at most max_launches launches in total.  Returns 0, or -1 when already
 *   active or max_launches is not in [1, 2^20].
 * chol_profile_end: waits for the recorded events and returns, per sweep (index 0 chol_rev,
 *   1 chol_factor, 2 chol_fwd), the summed kernel time in ms, the summed flops of the
 *   contractions (2*M*N*K per launch), their summed algorithmic HBM bytes (8 bytes for each
 *   element of op(A) and op(B) read once, of the accumulated-into C read once when it is read,
 *   and of C, and of its mirrored copy when one is written, written once; split-K partial sums
 *   are not counted) and the number of launches; then releases the events.  ms, flops, bytes
 *   and launches must each point to 3 elements.  Returns 0, -1 (not active / NULL
 *   argument) or CHOL_ERR_HIP.  Process-global; not thread-safe.
 */
int chol_profile_begin(int max_launches);
int chol_profile_end(double *ms, double *flops, double *bytes, int64_t *launches);

/* Human-readable text for a status code (static storage; never NULL). */
const char *chol_status_string(int status);

/* CHOLGRAD_VERSION of the built library. */
int chol_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CHOLGRAD_H */
