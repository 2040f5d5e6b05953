/*
 * lrinv.h - C ABI of the MI355X randomized low-rank covariance inverse.
 *
 * Method (Banerjee, Vogelstein, Dunson, "Parallel inversion of huge covariance
 * matrices"): for points x_1..x_n and a stationary kernel k, with
 * K_f[i,j] = k(x_i, x_j) and K = K_f + sigma2 I,
 *   1. sketch   Y = (K_f + nu I) Omega, Omega n x d random (Sec. 3.1) or the
 *               structured c R H P with H the Walsh-Hadamard matrix (Def. 1,
 *               Sec. 3.2); K is evaluated on the fly and never stored;
 *   2. tsqr     Y = Q R by leaf Householder QR of row blocks and a binary tree
 *               of QRs of stacked R factors (Sec. 3.3, Eq. 1-4);
 *   3. solve    the Woodbury-form approximation
 *               K~ = sigma2 I + Q (C - nu I) Q^T,  C = sym(F^{-1} R^T),
 *               F = Omega^T Q, applied to A: K~^{-1} A = (A - Q Z)/sigma2 +
 *               Q S^{-1} Z with Z = Q^T A, S = C + (sigma2 - nu) I = L L^T,
 *               and log|K~| = (n - d) log sigma2 + 2 sum log L_jj. (The paper
 *               states the target K^{-1} A, Sec. 1, and the column-space
 *               projection, Sec. 3.1 and the proof of Thm 5, but not this
 *               formula; this is the projected-process reading of it.)
 *   4. backward gradients of the approximate Gaussian log-likelihood, or of
 *               <Abar, K~^{-1} A>, with respect to (log ell, log s, log sigma2).
 *
 * Conventions for every entry point:
 *   - Matrices are row-major and contiguous unless a leading dimension is given.
 *   - "device" pointers are HIP device memory; "host" pointers are host memory.
 *   - The caller owns all memory. The library never allocates or frees; scratch
 *     space comes from the caller's workspace, sized by lr_*_workspace_bytes.
 *     The workspace pointer must be 256-byte aligned.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream). Argument errors are detected on the host BEFORE anything is
 *     launched and nothing is written then. Numerical breakdown is reported in
 *     a device int32 `info` (see lr_lowrank_solve).
 *   - Precision `prec`: LR_PREC_F64 (all float64), LR_PREC_F32 (float32 kernel
 *     tiles, sketch and leaf QR; float64 tree, d x d core and solves),
 *     LR_PREC_BF16 (as F32, but the dense-Omega sketch rounds K tiles to
 *     bfloat16 and runs on bf16 matrix cores with float32 accumulation;
 *     n <= 2^25, else LR_ERR_UNSUPPORTED), LR_PREC_BF16X2 (as BF16, but each
 *     kernel entry k is split into k_hi = bf16(k) and k_lo = bf16(k - k_hi),
 *     and both products with the bf16 Omega run on the matrix cores: K is
 *     carried to about 16 bits instead of 8; dense Omega with D <= 3 only).
 *     "real" below means double for F64 and float otherwise.
 *   - Points X are float32 n x D (1 <= D <= 15) in every precision.
 *   - Sizes: n >= 1, 1 <= d <= 1024, d <= n, 0 <= m <= 64.
 */
#ifndef LRINV_H
#define LRINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LR_OK = 0,
  LR_ERR_ARG = 1,         /* NaN/inf/out-of-range scalar, NULL pointer, unknown enum */
  LR_ERR_SHAPE = 2,       /* inconsistent or out-of-range sizes */
  LR_ERR_NOT_POW2 = 3,    /* SRHT Omega with n not a power of two */
  LR_ERR_WORKSPACE = 4,   /* workspace smaller than required or misaligned */
  LR_ERR_HIP = 5,         /* a HIP runtime call or kernel launch failed */
  LR_ERR_UNSUPPORTED = 6, /* valid but unsupported combination */
  LR_ERR_SCRATCH_LIMIT = 7 /* larger than the static scratch of lr_sketch_noalloc */
} lr_status;

typedef enum { LR_KERNEL_SE = 0, LR_KERNEL_MATERN32 = 1 } lr_kernel;
typedef enum { LR_OMEGA_SRHT = 0, LR_OMEGA_GAUSS = 1 } lr_omega_kind;
typedef enum { LR_PREC_F64 = 0, LR_PREC_F32 = 1, LR_PREC_BF16 = 2, LR_PREC_BF16X2 = 3 } lr_prec;

/* Stationary kernel (Sec. 5.1 forms):
 *   LR_KERNEL_SE       k(r) = s^2 exp(-r^2 / (2 ell^2))
 *   LR_KERNEL_MATERN32 k(r) = s^2 (1 + u) exp(-u),  u = sqrt(3) r / ell
 * with r = |x_i - x_j| in difference form. Requires ell > 0, s >= 0, finite. */
typedef struct {
  int32_t kernel;   /* lr_kernel */
  int32_t reserved; /* must be 0 */
  double ell;
  double s;
} lr_hyper;

/* Random matrix Omega (n x d).
 *   LR_OMEGA_SRHT  (Def. 1 with T = Walsh-Hadamard, Sec. 3.2):
 *       Omega[j,k] = n^{-1/2} signs[j] (-1)^popcount(j & cols[k]).
 *       signs: device int8[n] (negative = -1, otherwise +1);
 *       cols:  device int32[d], distinct, in [0, n) (see lr_check_srht_cols).
 *       n must be a power of two.
 *   LR_OMEGA_GAUSS (any dense Omega: i.i.d. N(0, 1/d), Sec. 3.1, or a structured
 *       transform written out by lr_structured_omega):
 *       dense_t: device, Omega TRANSPOSED, d rows of length >= n with leading
 *       dimension ld (elements, ld >= n, ld % 8 == 0, 16-byte aligned base),
 *       element type double (F64), float (F32) or bfloat16 bits (BF16, BF16X2). */
typedef struct {
  int32_t kind;        /* lr_omega_kind */
  int32_t d;
  int64_t n;
  int64_t ld;          /* GAUSS only */
  const int8_t *signs; /* SRHT only */
  const int32_t *cols; /* SRHT only */
  const void *dense_t; /* GAUSS only */
} lr_omega;

/* ---------------------------------------------------------------- structured Omega, written out
 * Omega[j,k] = signs[j] T[j, cols[k]] for a fast orthogonal transform T
 * (Def. 1 of Sec. 3.2; the paper's experiments use the cosine and Hartley
 * forms, Sec. 5 and Table 3), written as the dense TRANSPOSED Omega of
 * LR_OMEGA_GAUSS so that every entry point takes it as a dense Omega:
 *   LR_TRANSFORM_DCT  orthonormal DCT-II: T[j,p] = a_p cos(pi (2j+1) p / (2n)),
 *                     a_0 = n^{-1/2}, a_p = (2/n)^{1/2}; any n.
 *   LR_TRANSFORM_DHT  discrete Hartley: T[j,p] = n^{-1/2} (cos + sin)(2 pi j p / n); any n.
 *   LR_TRANSFORM_WHT  Walsh-Hadamard: T[j,p] = n^{-1/2} (-1)^popcount(j & p); n a power of two.
 * T is orthogonal, so the columns of Omega are orthonormal.
 *   signs    device int8[n] (negative = -1, otherwise +1).
 *   cols     device int32[d], distinct, in [0, n) (see lr_check_srht_cols); any
 *            value is memory-safe (it only enters the formula, reduced mod n).
 *   prec     element type written: double (F64), float (F32), bfloat16 bits
 *            (BF16, BF16X2). Each entry is evaluated in float64 with the angle
 *            reduced exactly in integers, then rounded to nearest even.
 *   omega_t  device output, d rows of leading dimension ld (elements; ld >= n,
 *            ld % 8 == 0, 16-byte aligned base); columns n .. ld-1 are zeroed.
 * Errors: LR_ERR_ARG (transform, prec, NULL pointer), LR_ERR_SHAPE (n, d, ld),
 * LR_ERR_NOT_POW2 (WHT with n not a power of two). No workspace. */
typedef enum { LR_TRANSFORM_DCT = 0, LR_TRANSFORM_DHT = 1, LR_TRANSFORM_WHT = 2 } lr_transform;
lr_status lr_structured_omega(void *stream, int32_t transform, int64_t n, int32_t d, const int8_t *signs,
                              const int32_t *cols, int32_t prec, void *omega_t, int64_t ld);

/* Host-side check of SRHT column indices (host pointer): LR_OK when the d entries
 * are distinct and in [0, n), LR_ERR_ARG otherwise. Device kernels are memory-safe
 * for any index values, but the method needs distinct columns. */
lr_status lr_check_srht_cols(const int32_t *cols_host, int32_t d, int64_t n);

/* ---------------------------------------------------------------- sketch
 * Y = (K_f + nu I) Omega (Sec. 3.1-3.2), K_f evaluated tile by tile from X and
 * never written to memory.
 *   X       device float32 n x D points.
 *   hyp     host pointer to the kernel description.
 *   omega   host pointer to the Omega description (omega->n == n).
 *   nu      shift of the sketched matrix (0 sketches K_f).
 *   Y       device real n x d output (may be NULL when only Yprime is wanted).
 *   Yprime  device real n x d output of (dK_f / dlog ell) Omega, or NULL. With
 *           SRHT and F32 both outputs come from one fused pass.
 * Unsupported: BF16 and BF16X2 with SRHT; BF16X2 with D > 3.
 * Workspace: the prescaled points ((n + 128) rows) and, for BF16 with D <= 3, a
 * copy of the Gaussian Omega in matrix-core operand order (about 2 n d bytes). */
size_t lr_sketch_workspace_bytes(int64_t n, int32_t D, int32_t d, int32_t prec);
lr_status lr_sketch(void *stream, int64_t n, int32_t D, const float *X, const lr_hyper *hyp,
                    const lr_omega *omega, double nu, int32_t prec, void *Y, void *Yprime,
                    void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------- sketch, no allocation
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lr_sketch
 * with its workspace (the prescaled points) in a static device array of
 * LR_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until the
 * process ends. Nothing is allocated or freed: the caller passes X, Y and
 * Yprime as for lr_sketch.
 *   Returns LR_ERR_SCRATCH_LIMIT when lr_sketch_workspace_bytes(n, D, d, prec)
 *   exceeds the array (about (n + 128) x 16 bytes for D <= 3 in float32:
 *   n <= 2,097,024; half that in float64), and LR_ERR_UNSUPPORTED for the bf16
 *   Gaussian sketch with D <= 3, whose operand copy of Omega (2 n d bytes) does
 *   not fit a static array. Every call on one GPU uses that GPU's array and
 *   leaves its contents behind; calls that overlap on one GPU (two streams,
 *   two threads) race on it and must be serialised by the caller. */
#define LR_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
lr_status lr_sketch_noalloc(void *stream, int64_t n, int32_t D, const float *X, const lr_hyper *hyp,
                            const lr_omega *omega, double nu, int32_t prec, void *Y, void *Yprime);

/* ---------------------------------------------------------------- hyperparameter grid
 * Sketches for a batch of ntheta kernels that share the points, the kernel
 * kind and Omega and differ in ell and s (the grids over the range parameter
 * of Sec. 5.2): Y_g = (K_f(theta_g) + nu I) Omega for g < ntheta, written to
 * Y + g n d. With an SRHT Omega one pass serves two kernels: each point load
 * and squared distance is shared, and each kernel runs its own transform. A
 * dense Omega runs the single-kernel sketch once per g.
 *   hyps    host array of ntheta lr_hyper, all with the same kernel kind
 *           (LR_ERR_ARG otherwise); 1 <= ntheta <= 4096.
 *   Y       device real ntheta x n x d (row-major per g).
 * Precisions as lr_sketch; no derivative output (lr_backward recomputes it).
 * Workspace: lr_sketch_grid_workspace_bytes, the same as lr_sketch's. */
size_t lr_sketch_grid_workspace_bytes(int64_t n, int32_t D, int32_t d, int32_t prec);
lr_status lr_sketch_grid(void *stream, int64_t n, int32_t D, const float *X, int32_t ntheta, const lr_hyper *hyps,
                         const lr_omega *omega, double nu, int32_t prec, void *Y, void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------- tsqr
 * Binary-tree blocked QR of the n x d matrix Y (Sec. 3.3, Eq. 1-4).
 *   Rows are split into leaves of leaf_rows rows (the last leaf may be shorter
 *   but needs >= d rows; d <= leaf_rows <= 8192). Each leaf is factored by
 *   blocked Householder QR in "real" precision; the leaf R factors are merged
 *   pairwise (left to right, an unpaired last one is carried up) in float64.
 *   Y   device real n x d input (not modified).
 *   Q   device real n x d output with Q^T Q = I.
 *   R   device double d x d output, upper triangular with diag(R) >= 0 (zeros
 *       are written below the diagonal); Y = Q R. */
size_t lr_tsqr_workspace_bytes(int64_t n, int32_t d, int32_t leaf_rows, int32_t prec);
lr_status lr_tsqr(void *stream, int64_t n, int32_t d, int32_t leaf_rows, int32_t prec,
                  const void *Y, void *Q, double *R, void *ws, size_t ws_bytes);

/* Tree shapes of the blocked QR and R without Q (Sec. 3.3). With group = 1
 * this is lr_tsqr's binary tree (Eq. 2-4). With group = g > 1 the leaves are
 * taken in groups of g consecutive blocks and each group runs the sequential
 * scheme of Eq. (5): the first block's QR, then the QR of the previous R
 * stacked on the next block, [R_{t-1}; K_t], in the working precision; the
 * groups' R factors then meet in the float64 binary tree. group = number of
 * blocks is the fully sequential scheme, and 1 < group < blocks the hybrids
 * between the two. Q may be NULL: only R is computed and Q is never formed
 * (all a caller needing R^{-1} alone requires, Sec. 3.3).
 *   group > 1 needs n % leaf_rows == 0, (n / leaf_rows) % group == 0 and
 *   d + leaf_rows <= 8192 (LR_ERR_SHAPE otherwise).
 * Outputs, precisions and errors otherwise as lr_tsqr; R (diag >= 0) and Q are
 * those of lr_tsqr up to rounding. Workspace: lr_tsqr_tree_workspace_bytes. */
size_t lr_tsqr_tree_workspace_bytes(int64_t n, int32_t d, int32_t leaf_rows, int32_t group, int32_t prec);
lr_status lr_tsqr_tree(void *stream, int64_t n, int32_t d, int32_t leaf_rows, int32_t group, int32_t prec,
                       const void *Y, void *Q, double *R, void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------- lowrank_solve
 * X = K~^{-1} A and log|K~| from the sketch factors (see the header comment).
 *   Q, R        outputs of lr_tsqr for the same Omega and nu.
 *   A, X        device real n x m (X may not alias A); m = 0 computes only the
 *               factors and log-determinant. Z = Q^T A is summed in float64 from
 *               exact products and X = A/sigma2 + Q (S^{-1} Z - Z/sigma2) is
 *               formed in float64 and rounded once to "real".
 *   C           device double d x d: sym(F^{-1} R^T).
 *   L           device double d x d: lower Cholesky factor of S (upper part 0).
 *   Flu, piv    device double d x d LU factors of F (unit lower L and U packed,
 *               LAPACK getrf layout, row-major) and int32[d] pivot rows.
 *   logdet      device double[1].
 *   info        device int32[1]: 0 = success; k > 0: the k-th leading minor
 *               of S is not positive (X is then not written, logdet is NaN);
 *               k < 0: F has a zero pivot at step -k. logdet is NaN then.
 *   sigma2 > 0; nu >= 0. */
size_t lr_lowrank_solve_workspace_bytes(int64_t n, int32_t d, int32_t m, int32_t prec);
lr_status lr_lowrank_solve(void *stream, int64_t n, int32_t d, int32_t m, const lr_omega *omega,
                           int32_t prec, const void *Q, const double *R, double sigma2, double nu,
                           const void *A, void *X, double *C, double *L, double *Flu,
                           int32_t *piv, double *logdet, int32_t *info, void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------- projection variant
 * The symmetric projection K~_f = Q (Q^T K_f Q) Q^T of the signal covariance
 * onto the sketch's basis (the object QQ^T K that Sec. 3.1 bounds, Thm 5,
 * with the further products Sec. 3.3 expects after the QR), with the nugget
 * added back by Woodbury as in lr_lowrank_solve:
 *   B = Q^T K_f Q   a second pass of K_f, Q in place of Omega, tiles never
 *                   stored (float64 for F64, float32 otherwise), the n-length
 *                   sums exact in float64, then exactly symmetric;
 *   clip = 1        B <- its positive semidefinite part V max(Lambda, 0) V^T
 *                   (the eig-clip core; rounding can leave B slightly
 *                   indefinite), by a Newton-Schulz sign iteration on float64
 *                   matrix cores;
 *   S = B + sigma2 I = L L^T, log|K~| = (n - d) log sigma2 + log|S|,
 *   X = sigma2^{-1} (A - Q Z) + Q S^{-1} Z,  Z = Q^T A  (when m > 0).
 * No Omega and no R enter, and no shift: B is positive semidefinite in exact
 * arithmetic for any sketch.
 *   X       device float32 n x D points; hyp as lr_sketch.
 *   Q       device real n x d, orthonormal columns (lr_tsqr's output).
 *   B, L    device float64 d x d outputs (the core used, its Cholesky factor).
 *   logdet, info  device outputs as lr_lowrank_solve (info > 0: S not PD).
 *   A, Xout device real n x m (m <= 64; m = 0 computes the factors only).
 * Workspace: lr_projection_solve_workspace_bytes (points, Q^T, K_f Q, d x d
 * blocks). Forward only: no adjoint for this variant. */
size_t lr_projection_solve_workspace_bytes(int64_t n, int32_t D, int32_t d, int32_t m, int32_t prec);
lr_status lr_projection_solve(void *stream, int64_t n, int32_t D, int32_t d, const float *X, const lr_hyper *hyp,
                              int32_t prec, const void *Q, double sigma2, int32_t clip, int32_t m, const void *A,
                              void *Xout, double *B, double *L, double *logdet, int32_t *info, void *ws,
                              size_t ws_bytes);

/* The positive semidefinite part of a symmetric float64 d x d matrix B
 * (device, row-major; d <= 1024): Bplus = V max(Lambda, 0) V^T for B = V Lambda
 * V^T, the eig-clip of the projection core. B is read only (Bplus must not
 * alias it). Workspace: lr_psd_part_workspace_bytes(d) (3 d^2 doubles). */
size_t lr_psd_part_workspace_bytes(int32_t d);
lr_status lr_psd_part(void *stream, int32_t d, const double *B, double *Bplus, void *ws, size_t ws_bytes);

/* ---------------------------------------------------------------- log-likelihood
 * out[0] = -1/2 y^T alpha - 1/2 logdet[0] (the approximate Gaussian
 * log-likelihood without the -n/2 log(2 pi) constant; Sec. 1 names Gaussian
 * likelihoods as the target use). y, alpha: device real[n]; logdet, out:
 * device double[1]. Writes NaN when info[0] != 0 (info may be NULL). */
lr_status lr_loglik(void *stream, int64_t n, int32_t prec, const void *y, const void *alpha,
                    const double *logdet, const int32_t *info, double *out);

/* ---------------------------------------------------------------- backward
 * Gradient with respect to theta = (log ell, log s, log sigma2) for the
 * forward's shift nu (a fixed parameter). (Not in the paper: the adjoint of
 * steps 1-3 above.) For a symmetric G, the derivative of the objective with
 * respect to K~, d/dtheta = tr(G dK~/dtheta) with, for Phi = F^{-1} and
 * Y' = (dK_f/dlog ell) Omega,
 *   d/dlog ell    = 2 <G Q Phi, Y'> - <Phi^T (Q^T G Q) Phi, Omega^T Y'>,
 *   d/dlog s      = 2 tr(Q^T G Q C),   d/dlog sigma2 = sigma2 tr G,
 * and for nu > 0 (K~ = sigma2 I + Y W^{-1} Y^T - nu Q Q^T) the terms of the
 * projector's derivative, -2 nu <(G Q - Q Q^T G Q) R^{-T}, Y''> for each
 * derivative sketch Y'' (Y' for log ell, 2 (Y - nu Omega) for log s), plus the
 * -2 nu Omega part of the log s sketch in the first two terms.
 *   mode 0 (log-likelihood -1/2 y^T K~^{-1} y - 1/2 log|K~|): G = (alpha alpha^T
 *          - K~^{-1})/2. A = y, the forward's right-hand side (device real
 *          n x 1, m must be 1); V and dA unused.
 *   mode 1 (solve, cotangent Abar of X = K~^{-1} A): G = -(X B^T + B X^T)/2 with
 *          B = K~^{-1} Abar. A = the forward's right-hand side (device real
 *          n x m), V = Abar (n x m); dA (device real n x m, or NULL) receives B.
 *   The solves alpha, X and B are recomputed here from A (and Abar) in float64
 *   (Q^T A summed in float64 from exact products, S^{-1} by the Cholesky
 *   factor), and their Q-basis projections are taken as S^{-1} Q^T A, so the
 *   result does not depend on how closely a float32 Q satisfies Q^T Q = I.
 *   Q, R, C, L, Flu, piv   forward factors from lr_tsqr / lr_lowrank_solve (R,
 *           device double d x d upper triangular, is read only when nu > 0
 *           and may be NULL otherwise).
 *   sigma2 > 0, nu >= 0: the forward's nugget and shift.
 *   Yprime  device real n x d (dK_f/dlog ell) Omega from lr_sketch, or NULL to
 *           recompute it here (K tiles are recomputed, never stored).
 *   dtheta  device double[3]. */
size_t lr_backward_workspace_bytes(int64_t n, int32_t D, int32_t d, int32_t m, int32_t prec);
lr_status lr_backward(void *stream, int64_t n, int32_t D, const float *X, const lr_hyper *hyp,
                      const lr_omega *omega, int32_t prec, const void *Q, const double *R,
                      const double *C, const double *L, const double *Flu, const int32_t *piv,
                      double sigma2, double nu, int32_t mode, int32_t m, const void *A,
                      const void *V, const void *Yprime, double *dtheta, void *dA, void *ws,
                      size_t ws_bytes);

/* Human-readable status name (static string). */
const char *lr_status_string(int32_t status);

/* ABI version: (major << 16) | minor. 2.0: lr_backward takes the forward's
 * right-hand side A instead of its solution, and R and the shift nu.
 * 2.1: lr_structured_omega, lr_sketch_grid, lr_projection_solve, lr_psd_part,
 * lr_tsqr_tree. */
int32_t lr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LRINV_H */
