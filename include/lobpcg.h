/*
 * lobpcg.h -- C ABI of the MI355X (gfx950) LOBPCG hot path.
 *
 * The library finds the lowest eigenpairs of a large sparse symmetric matrix
 * H, given by its upper triangle, with the block method of Maris, Yang,
 * Oryspayev & Cook (arXiv:2109.00485), Algorithm 1: block locally optimal
 * preconditioned conjugate gradients, one Rayleigh-Ritz step per iteration,
 * H X and H P carried by the recurrences eqs. upd1-upd2 so that H W is the
 * only sparse product per iteration.
 *
 * Conventions shared by every entry point
 *  - Blocks of k vectors are n x k, ROW-MAJOR (row i of all k vectors is
 *    contiguous; paper Section 3.3), device-resident, in the context dtype.
 *  - Every pointer argument is caller-owned; the library never frees it.
 *    "device" means memory the HIP runtime can address from gfx950 kernels
 *    (hipMalloc / torch CUDA tensors); "host" means ordinary CPU memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    spmm_sym, precond_apply and gram are asynchronous on that stream;
 *    create and solve are synchronous with respect to it.
 *  - Errors are returned as status codes (never thrown across the ABI).
 *    Scalar and shape checks run on the host before anything is enqueued,
 *    so they are testable without a GPU.  lobpcg_last_error() returns a
 *    human-readable message for the last failing call on a context.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef LOBPCG_MI355X_H
#define LOBPCG_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define LOBPCG_OK            0
#define LOBPCG_EINVAL       -1   /* bad argument or malformed matrix            */
#define LOBPCG_ENOMEM       -2   /* device allocation failed                    */
#define LOBPCG_EHIP         -3   /* HIP runtime error                           */
#define LOBPCG_ENOTSPD      -4   /* Cholesky QR / Rayleigh-Ritz lost definiteness */
#define LOBPCG_ENOCONV      -5   /* maxiter reached; best iterate still returned */
#define LOBPCG_ENONFINITE   -6   /* NaN/Inf in matrix values or iterates        */
#define LOBPCG_EUNSUPPORTED -7   /* valid request the build does not support    */

/* ---- enumerations ---- */
#define LOBPCG_F32 1             /* FP32 values, blocks and sparse arithmetic   */
#define LOBPCG_F64 2             /* FP64 everywhere                             */

#define LOBPCG_GRAM_AUTO   0     /* FP64 MFMA (on the FP32 values for F32 contexts) */
#define LOBPCG_GRAM_F64    1     /* inputs upcast to FP64, FP64 MFMA            */
#define LOBPCG_GRAM_F32    2     /* FP32 MFMA, FP64 reduction across workgroups */
#define LOBPCG_GRAM_BF16X3 3     /* split-BF16 (a0b0 + a0b1 + a1b0) MFMA, FP32 inputs */
#define LOBPCG_GRAM_BF16X6 4     /* three-term split-BF16, the six products with i + j <= 2;
                                    FP32 sums per 16 rows, FP64 across them; FP32 inputs */

#define LOBPCG_PRECOND_NONE 0    /* K = I                                       */
#define LOBPCG_PRECOND_DIAG 1    /* W_ij = R_ij / s(d_i - sigma_j), sigma_j = theta_j by default */
#define LOBPCG_PRECOND_MLP  2    /* learned scaling from an attached MLP        */
#define LOBPCG_PRECOND_FOM  3    /* shifted 64 x 64 diagonal tiles of H, FOM     */

#define LOBPCG_FORMAT_AUTO  0    /* tiled when tiles are dense enough, else CSR */
#define LOBPCG_FORMAT_CSR   1    /* row-split CSR of the strict upper triangle  */
#define LOBPCG_FORMAT_TILED 2    /* tile-row ordered sparse tiles               */

typedef struct lobpcg_ctx lobpcg_ctx;
typedef struct lobpcg_mlp lobpcg_mlp;

typedef struct {
    int dtype;        /* LOBPCG_F32 (default) or LOBPCG_F64                          */
    int gram;         /* LOBPCG_GRAM_*                                               */
    int format;       /* LOBPCG_FORMAT_*                                             */
    int tile;         /* tile edge of the tiled format; 64 is the only value built   */
    int kmax;         /* largest block size this context will be used with (<= 16)   */
    double tau_rel;   /* convergence floor tau = tau_rel * gamma (default 1e-3)      */
    double eps_rel;   /* preconditioner guard eps = eps_rel * gamma (default 1e-5)   */
} lobpcg_opts;

typedef struct {
    int iters;            /* LOBPCG iterations performed                        */
    int n_spmm;           /* sparse products performed (incl. confirmations)    */
    int p_dropped;        /* iterations whose Rayleigh-Ritz dropped P           */
    int cholqr_retries;   /* Cholesky QR retries after re-projection            */
    int confirmations;    /* explicit H X recomputations on apparent convergence */
    int refreshes;        /* periodic explicit recomputations of H X and H P     */
    int status;           /* same value the call returned                       */
    double gamma;         /* Gershgorin bound max_i sum_j |H_ij|                 */
    /* optional, caller-owned host arrays of maxiter*k doubles (NULL to skip):
       Ritz values and relative residual norms after every iteration          */
    double *theta_hist;
    double *rel_hist;
    /* optional per-phase device time in seconds (filled when timing != 0)      */
    int timing;
    double t_spmm, t_precond_update, t_gram, t_rr, t_orth, t_total;
    /* optional training-sample harvest (struct lobpcg_harvest below), NULL = off */
    struct lobpcg_harvest_s *harvest;
    int cholqr_shifted;       /* iterations whose Cholesky QR needed the diagonal shift */
    long long mlp_fallbacks;  /* entries where the learned factor was not finite and
                                 the diagonal step was used alone                     */
    int locked_max;           /* most columns soft-locked at once (lobpcg_set_soft_lock) */
} lobpcg_info;

/* Fill *o with the defaults: F32, GRAM_AUTO, FORMAT_AUTO, tile 64, kmax 16,
 * tau_rel 1e-3, eps_rel 1e-5. */
void lobpcg_opts_default(lobpcg_opts *o);

/*
 * lobpcg_create -- validate H, build the library's own device copy of it, and
 * allocate every workspace once (the paper creates its solver handles and
 * workspaces outside the iteration loop, Section 4.4).
 *
 *   n        matrix dimension, 1 <= n < 2^31
 *   row_ptr  device, int64[n+1], CSR row offsets of the UPPER triangle of H,
 *            diagonal included (the paper stores half of the symmetric H,
 *            Section 3.1)
 *   col      device, int32[nnz], nnz = row_ptr[n]; within each row strictly
 *            ascending, col >= row, and the first entry of row i is (i, i)
 *   val      device, nnz values in opts->dtype
 *   opts     host, may be NULL for defaults
 * The caller may free its arrays once create returns.  Malformed CSR content
 * is detected by a device validation pass and returns LOBPCG_EINVAL;
 * non-finite values return LOBPCG_ENONFINITE.  *out is NULL on failure.
 */
int lobpcg_create(lobpcg_ctx **out, int64_t n, const int64_t *row_ptr, const int32_t *col,
                  const void *val, const lobpcg_opts *opts, void *stream);

/*
 * lobpcg_create_rp32 -- lobpcg_create with int32 row offsets (row_ptr
 * device, int32[n+1]; so nnz < 2^31).  The offsets are widened into a
 * temporary int64 device array (8(n+1) bytes, freed before return), then
 * lobpcg_create runs on it; same validation, results and errors, plus
 * LOBPCG_ENOMEM when the temporary cannot be allocated.  A negative or
 * decreasing offset is caught by the validation pass (LOBPCG_EINVAL).
 */
int lobpcg_create_rp32(lobpcg_ctx **out, int64_t n, const int32_t *row_ptr, const int32_t *col,
                       const void *val, const lobpcg_opts *opts, void *stream);

void lobpcg_destroy(lobpcg_ctx *ctx);

/*
 * lobpcg_spmm_sym -- Y = H X from the stored upper triangle: each stored
 * off-diagonal h_ij (i < j) contributes h_ij X_j to Y_i and h_ij X_i to Y_j
 * (Algorithm 2, applied to the stored part and its transpose, Section 3.2).
 *   X  device, n x k row-major, read-only
 *   Y  device, n x k row-major, overwritten; must not alias X
 *   1 <= k <= kmax
 */
int lobpcg_spmm_sym(lobpcg_ctx *ctx, const void *X, void *Y, int k, void *stream);

/*
 * lobpcg_precond_apply -- W = K^{-1} R, the preconditioning step of
 * Algorithm 1.  With LOBPCG_PRECOND_DIAG, K is the diagonal of H shifted per
 * column (the 1x1-tile case of the block-diagonal preconditioner of Section
 * 3.4, whose shift lies near an approximate wanted eigenvalue):
 * W_ij = R_ij / s(d_i - sigma_j), sigma_j = theta_j - c (max theta - min theta)
 * with c the context's offset (lobpcg_set_precond_offset; default 0, i.e. the
 * shift is the Ritz value theta_j itself), s(x) = x if |x| >= eps else +-eps
 * (sign of x, + for 0), eps = eps_rel * gamma.  With LOBPCG_PRECOND_MLP the
 * attached network supplies a factor on that step (lobpcg_set_mlp).  With
 * LOBPCG_PRECOND_FOM, K is block diagonal, its blocks the 64 x 64 diagonal
 * tiles of H shifted by the same sigma_j, each system solved by m FOM steps
 * (lobpcg_set_fom_steps).
 *   R      device, n x k row-major
 *   theta  device, double[k]
 *   W      device, n x k row-major, written (may alias R)
 */
int lobpcg_precond_apply(lobpcg_ctx *ctx, const void *R, const double *theta, void *W, int k,
                         int kind, void *stream);

/*
 * lobpcg_set_test_faults -- force the failure branches of the solver at one
 * iteration of the following lobpcg_solve calls, for tests of the error paths
 * (the kernels then take the branch as if the factorisation had failed; no
 * kernel is made to fault).  iteration 0 is the first Rayleigh-Ritz step (on
 * X0), 1 the first LOBPCG iteration.  mask (0 turns it off) is an OR of
 *   LOBPCG_FAULT_CHOLQR_SHIFT   the unshifted Cholesky of W^T W fails: the
 *                               shifted factorisation (Section 3.5) is used
 *   LOBPCG_FAULT_CHOLQR_ONCE    both fail on the first attempt: W is projected
 *                               again and the retry proceeds
 *   LOBPCG_FAULT_CHOLQR_ALWAYS  both fail on every attempt: LOBPCG_ENOTSPD
 *   LOBPCG_FAULT_RR_DROP_P      the Rayleigh-Ritz Cholesky of O fails with P:
 *                               P is dropped for that iteration
 *   LOBPCG_FAULT_RR             it fails with and without P: LOBPCG_ENOTSPD
 * Returns LOBPCG_EINVAL for unknown bits or a negative iteration.  Host-only.
 */
#define LOBPCG_FAULT_CHOLQR_SHIFT  1
#define LOBPCG_FAULT_CHOLQR_ONCE   2
#define LOBPCG_FAULT_CHOLQR_ALWAYS 4
#define LOBPCG_FAULT_RR_DROP_P     8
#define LOBPCG_FAULT_RR            16
int lobpcg_set_test_faults(lobpcg_ctx *ctx, int mask, int iteration);

/*
 * lobpcg_set_cholqr_passes -- Cholesky QR passes per orthonormalisation of W
 * in lobpcg_solve: 1 (default; Section 3.5) or 2 (CholeskyQR2, Fukaya et al.
 * 2014: the second pass, on the already orthonormalised W, brings its
 * orthogonality error from about eps cond(W)^2 to about eps; each pass keeps
 * the shifted factorisation as its fallback).  Returns LOBPCG_EINVAL for
 * other values.  Host-only; applies to the following solves.
 */
int lobpcg_set_cholqr_passes(lobpcg_ctx *ctx, int passes);

/*
 * lobpcg_set_soft_lock -- soft locking in lobpcg_solve (on = 1; default 0): a
 * column whose relative residual was at or below tol at the last check is
 * locked, i.e. its residual direction W_j and its P_j are left out of the
 * Rayleigh-Ritz basis while X_j stays in it; a locked column is released
 * when its residual rises above tol again.  Converged columns then stop
 * feeding rounding noise into W and P (the FP32 recurrences of eqs.
 * upd1-upd2 drift).  The blocks keep their width: the Cholesky QR treats a
 * locked column as absent and the Rayleigh-Ritz step drops it from the
 * pencil.  lobpcg_info.locked_max reports the most columns locked at once.
 * Returns LOBPCG_EINVAL unless on is 0 or 1.
 */
int lobpcg_set_soft_lock(lobpcg_ctx *ctx, int on);

/*
 * lobpcg_cholqr -- Cholesky QR of a block in place (Section 3.5):
 * B = W^T W (FP64 Gram), B = R^T R, W <- W R^{-1}; passes = 2 repeats it on the
 * result (CholeskyQR2).  Each pass falls back to the shifted factorisation of
 * the unit-diagonal-scaled Gram (shift 1e-12 in FP64, 1e-6 in FP32 contexts)
 * when the plain one fails; *shifted (may be NULL) counts those passes.
 *   W   device, n x k row-major in the context dtype, overwritten
 * Returns LOBPCG_ENOTSPD when a pass fails even shifted (W then holds the
 * last completed pass), LOBPCG_EINVAL for k outside [1, kmax] or passes not
 * 1 or 2.  Synchronises the stream.
 */
int lobpcg_cholqr(lobpcg_ctx *ctx, void *W, int k, int passes, int *shifted, void *stream);

/*
 * lobpcg_orthonormalize -- the orthogonalisation step of lobpcg_solve on a
 * caller's blocks (Section 3.5; Algorithm 1 before the product H W):
 * W <- W - X (X^T W), then one Cholesky QR of the result, W <- W R^{-1}.
 * It takes one read of X and W: the Gram of [X W] gives C = X^T W, X^T X and
 * W^T W, the projected block's Gram is W^T W - C^T C - C^T C + C^T (X^T X) C
 * (exact for any X), and one pass writes W R^{-1} - X (C R^{-1}).  The
 * plain factorisation falls back to the shifted one as in lobpcg_cholqr;
 * *shifted (may be NULL) is set to 1 when it did.
 *   X   device, n x k row-major in the context dtype (read only; need not be
 *       orthonormal, the projection is the formula above)
 *   W   device, n x k row-major, overwritten; must not alias X
 * Returns LOBPCG_ENOTSPD when the projected Gram is not positive definite even
 * shifted (W is then unchanged), LOBPCG_EINVAL for null pointers or k outside
 * [1, kmax].  Synchronises the stream.
 */
int lobpcg_orthonormalize(lobpcg_ctx *ctx, const void *X, void *W, int k, int *shifted, void *stream);

/*
 * lobpcg_set_fom_steps -- FOM steps of LOBPCG_PRECOND_FOM, 1 <= m <= 8
 * (default 4; the paper uses three to five).  That preconditioner is the
 * block-diagonal K of Section 3.4: K_t = H_tt - sigma_j I, H_tt the t-th
 * 64 x 64 diagonal tile of H (rows t*64 .. t*64+63; the last tile is ragged),
 * sigma_j the diagonal step's shift of column j (lobpcg_set_precond_offset);
 * each (tile, column) system K_t w = r is solved by m steps of the full
 * orthogonalisation method (Arnoldi with modified Gram-Schmidt, w = V_m y,
 * H_m y = ||r|| e_1, stopping early on an invariant Krylov space), in FP64 for
 * either context precision; where H_m is singular to 1e-12 of its largest
 * entry, that column of that tile gets the guarded diagonal step.  The dense
 * tiles (n * 64 values) are built at create.  Returns LOBPCG_EINVAL outside
 * [1, 8].  Host-only; takes effect on the next launch.
 */
int lobpcg_set_fom_steps(lobpcg_ctx *ctx, int m);

/*
 * lobpcg_set_precond_offset -- place the diagonal preconditioner's shift c
 * Ritz-value spreads below each Ritz value: sigma_j = theta_j - c (max theta -
 * min theta) over the k values of the block (Section 3.4 puts the shift near
 * an approximate wanted eigenvalue).  Applies to lobpcg_precond_apply, to the
 * preconditioner inside lobpcg_solve, to the diagonal step the learned
 * preconditioner scales, and to harvested training samples.  c = 0 (the
 * default) is the shift at theta_j.  Returns LOBPCG_EINVAL unless
 * 0 <= c <= 1e6.  Host-only; takes effect on the next launch.
 */
int lobpcg_set_precond_offset(lobpcg_ctx *ctx, double c);

/*
 * lobpcg_gram -- G = A^T B for tall-skinny blocks (the products that form the
 * projected matrices of eqs. go / Glower and the Cholesky QR Gram W^T W,
 * Section 3.5), reduced across the whole column in FP64.
 *   A  device, n x ka row-major;  B device, n x kb row-major (may alias A)
 *   G  device, double[ka*kb], row-major ka x kb, overwritten
 *   1 <= ka, kb <= 48; prec is a LOBPCG_GRAM_* value (BF16X3 and BF16X6 need an F32 context)
 */
int lobpcg_gram(lobpcg_ctx *ctx, const void *A, int ka, const void *B, int kb, double *G,
                int prec, void *stream);

/*
 * lobpcg_gram_noalloc -- the product of lobpcg_gram without a context and
 * without allocating anything, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, allocation-free
 * harnesses): G = A^T B for two tall-skinny blocks.
 *   A      device, n x ka row-major;  B device, n x kb row-major (may alias A)
 *   n      rows, >= 1;  dtype LOBPCG_F32 or LOBPCG_F64 (of A and B)
 *   G      device, double[ka*kb], row-major ka x kb, overwritten
 *   prec   a LOBPCG_GRAM_* value; AUTO means FP64 (BF16X3, BF16X6 and F32 need F32 data)
 * The partial sums live in one library-owned device array per GPU (4.8 MB,
 * held until the process ends), so 1 <= ka, kb <= 48 (LOBPCG_EUNSUPPORTED
 * beyond) and calls that overlap on one GPU race: serialise them (one stream,
 * or events).  Asynchronous on `stream`; LOBPCG_EINVAL on a bad argument.
 */
int lobpcg_gram_noalloc(const void *A, int ka, const void *B, int kb, int64_t n, int dtype, double *G, int prec,
                        void *stream);

/*
 * lobpcg_solve -- lowest nev eigenpairs by Algorithm 1.
 *   k        block size, nev <= k <= kmax, 3k <= n
 *   X        device, n x k row-major: the starting block X0 on entry, the Ritz
 *            vectors (ascending Ritz values) on return
 *   evals    host, double[k]: Ritz values, ascending
 *   rel      host, double[k] or NULL: relative residual norms
 *            ||r_j|| / (max(|theta_j|, tau) ||x_j||)
 *   tol      > 0, convergence threshold on rel_j for j < nev
 *   maxiter  >= 0
 *   precond  LOBPCG_PRECOND_*
 *   info     host, may be NULL
 * The run ends when the nev wanted columns meet tol and an explicit product
 * H X confirms it (the recurrences eqs. upd1-upd2 drift in finite precision).
 * F32 contexts also recompute H X and H P explicitly every 20 iterations.
 * Returns LOBPCG_ENOCONV when maxiter is reached (X and evals still written).
 */
int lobpcg_solve(lobpcg_ctx *ctx, int k, int nev, void *X, double *evals, double *rel, double tol,
                 int maxiter, int precond, lobpcg_info *info, void *stream);

/* ======================================================================
 * Learned preconditioner.
 *
 * The paper's preconditioner (Section 3.4) is a shifted diagonal solve; its
 * 1 x 1-tile form is W_ij = R_ij / s(d_i - sigma_j) (sigma_j = theta_j unless the
 * context's offset moves it, lobpcg_set_precond_offset).  The learned variant
 * keeps that form and multiplies it by exp(2 tanh(o_ij / 2)) (a factor in
 * [e^-2, e^2]), where o_ij is the output of a
 * 4 -> 64 -> 64 -> 1 ReLU network of the standardised per-entry features
 *     f_ij = (d_i, theta_j, rho_i, t_i),  z = (f - mu) / sigma,
 * rho_i = sum_{j != i} |h_ij| over the full symmetric row and t_i the mean |h|
 * over the off-diagonal nonzeros of the 64-row tile holding row i.  A network
 * with zero output reproduces the diagonal preconditioner; any entry whose
 * scale is not finite falls back to the diagonal one.
 *
 * Arithmetic: W1, W2, w3 are used rounded to BF16 (round to nearest even);
 * the first hidden layer's activations are rounded to BF16 before the second
 * layer, which runs on BF16 matrix cores with FP32 accumulation; everything
 * else is FP32.  Training keeps FP32 master weights (Adam).
 *
 * Parameter blob (host float[LOBPCG_MLP_NBLOB]), row-major blocks in order:
 *   W1[64][4], b1[64], W2[64][64] (W2[v][u]: hidden-1 unit u -> hidden-2
 *   unit v), b2[64], w3[64], b3, mu[4], sigma[4].
 * Gradients use the first LOBPCG_MLP_NPARAM entries of the same layout.
 * ====================================================================== */
#define LOBPCG_MLP_NIN    4
#define LOBPCG_MLP_HID    64
#define LOBPCG_MLP_NPARAM 4545   /* trainable: 256 + 64 + 4096 + 64 + 64 + 1   */
#define LOBPCG_MLP_NBLOB  4553   /* + mu[4] + sigma[4]                          */

/* Create a network on the current device from a host parameter blob (sigma
 * entries must be > 0).  Adam state starts at zero. */
int lobpcg_mlp_create(lobpcg_mlp **out, const float *blob);
void lobpcg_mlp_destroy(lobpcg_mlp *m);
int lobpcg_mlp_set_params(lobpcg_mlp *m, const float *blob);  /* also resets Adam */
int lobpcg_mlp_get_params(lobpcg_mlp *m, float *blob);        /* host out        */
const char *lobpcg_mlp_last_error(const lobpcg_mlp *m);

/* Attach m to ctx for LOBPCG_PRECOND_MLP (NULL detaches).  The context does
 * not own the network; it must outlive its use by the context. */
int lobpcg_set_mlp(lobpcg_ctx *ctx, lobpcg_mlp *m);

/* Per-row feature columns of ctx (device float[n] each, NULL to skip): the
 * full-row off-diagonal 1-norm rho and the tile mean |h| t. */
int lobpcg_get_features(lobpcg_ctx *ctx, float *rownorm, float *tilemean, void *stream);

/* o[s] = network output for raw features feat[s][0..3] (device float N x 4 in,
 * device float N out), on the same matrix-core kernel the preconditioner
 * uses.  N >= 0. */
int lobpcg_mlp_forward(lobpcg_mlp *m, const float *feat, int64_t N, float *o, void *stream);

/* Set mu, sigma to the mean and standard deviation (sigma floored at 1e-12)
 * of N >= 2 raw feature rows (device float N x 4). */
int lobpcg_mlp_fit_standardizer(lobpcg_mlp *m, const float *feat, int64_t N, void *stream);

/* A training batch: samples grouped by (run, iteration, column j); the rows
 * of one group are contiguous.  Per sample s of group g:
 *   feat  raw features (d_i, theta_j, rho_i, t_i)
 *   U     the diagonal step R_ij / s(d_i - sigma_j) of the harvesting context
 *   T     the exact correction of column j at row i (its error outside span X)
 *   w     importance weight of the sampled row
 *   Xrow  row i of the block X (k values)
 * Loss of a group, u = exp(2 tanh(o / 2)) U, a = sum w Xrow u, u' = u - Xrow . a:
 *   L_g = 1 - (sum w u' T)^2 / ((sum w u'^2)(sum w T^2)),
 * 0 (with zero gradient) when either sum of squares is 0; the batch loss is
 * the mean over groups.  All arrays are device memory owned by the caller. */
typedef struct {
    int64_t nsamples;
    int ngroups;
    int k;                       /* 1..16 */
    const float *feat;           /* nsamples x 4 */
    const float *U, *T, *w;      /* nsamples each */
    const float *Xrow;           /* nsamples x k */
    const int64_t *group_off;    /* ngroups + 1, group_off[0] = 0, nondecreasing */
} lobpcg_mlp_batch;

/* Loss and its gradient (host double *loss, host float grad[NPARAM], either
 * may be NULL) at the current parameters; synchronous. */
int lobpcg_mlp_loss_grad(lobpcg_mlp *m, const lobpcg_mlp_batch *b, double *loss, float *grad, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the batch's gradient;
 * *loss (host, may be NULL) receives the loss before the step.  Synchronous. */
int lobpcg_mlp_train_step(lobpcg_mlp *m, const lobpcg_mlp_batch *b, float lr, double *loss, void *stream);

/* Harvest of training samples from a running solve (set info->harvest).
 * At every iteration it with it % every == 0, for each column j < nev, the
 * exact correction E_j = x*_j - X (X^T x*_j) is formed from converged
 * eigenvectors x* of the same matrix, and row i is kept with probability
 *   p_i = min(1, rows (1/(2n) + |E_ij| / (2 sum_l |E_lj|)))
 * (uniform draw: SplitMix64 of (seed, group, i), see the implementation),
 * weight w = 1/p_i.  Each (iteration, column) becomes one group appended to
 * the output arrays.  When the next group might not fit (capacity below
 * nsamples + n or groups exhausted) harvesting stops and `full` is set. */
typedef struct lobpcg_harvest_s {
    int every;                   /* >= 1 */
    int rows;                    /* >= 1, expected rows per group */
    int nev;                     /* columns harvested, 1..k */
    const void *xstar;           /* device, n x nev row-major, context dtype */
    uint64_t seed;
    int64_t capacity;            /* samples the arrays below hold */
    int capacity_groups;
    float *feat, *U, *T, *w;     /* device outputs (capacity x 4, capacity, ...) */
    float *Xrow;                 /* device, capacity x k */
    int32_t *row;                /* device, capacity, row index i (NULL to skip) */
    int64_t *group_off;          /* device, capacity_groups + 1 */
    int64_t nsamples;            /* in: samples already held; out: total */
    int ngroups;                 /* in: groups already held; out: total */
    int full;                    /* out */
} lobpcg_harvest;

/* One harvest step on a caller-supplied block: X, HX device n x k (context
 * dtype), theta device double[k]; appends h->nev groups to *h (as the solve
 * does every h->every iterations).  Synchronous. */
int lobpcg_harvest_block(lobpcg_ctx *ctx, const void *X, const void *HX, const double *theta, int k,
                         lobpcg_harvest *h, void *stream);

/* Matrix facts computed at create: n, stored nnz (incl. diagonal), format in
 * use, dtype, and the Gershgorin bound gamma.  Any output pointer may be NULL. */
int lobpcg_query(const lobpcg_ctx *ctx, int64_t *n, int64_t *nnz, int *format, int *dtype,
                 double *gamma);

/* Device copy of the diagonal d (n values, context dtype) into `d`. */
int lobpcg_get_diag(lobpcg_ctx *ctx, void *d, void *stream);

/* Streaming probes of the memory system (not part of the method): a plain
 * kernel that reads `bytes` from a (op LOBPCG_PROBE_READ; b receives at most
 * one float and must hold 4 bytes), writes `bytes` to b (LOBPCG_PROBE_WRITE;
 * a unused), or copies a to b (LOBPCG_PROBE_COPY; a and b must not overlap).
 * bytes > 0 and a multiple of 16; pointers device, 16-byte aligned,
 * caller-owned.  Asynchronous on `stream`.  Used for the achievable-bandwidth
 * reference of the sparse product and to scale hardware traffic counters by
 * a transfer of known size; LOBPCG_EINVAL on a bad argument. */
#define LOBPCG_PROBE_READ  0
#define LOBPCG_PROBE_WRITE 1
#define LOBPCG_PROBE_COPY  2
int lobpcg_stream_probe(int op, const void *a, void *b, int64_t bytes, void *stream);

const char *lobpcg_strerror(int status);
const char *lobpcg_last_error(const lobpcg_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* LOBPCG_MI355X_H */
