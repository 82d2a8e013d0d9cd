// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "lobpcg.h"

#define LOBPCG_WAVE 64
#define HEAVY_ROW 1024

// Spread max_j theta_j - min_j theta_j of the k Ritz values: the diagonal
// preconditioner's shift is sigma_j = theta_j - precond_offset * spread.
__device__ inline double ritz_spread(const double *theta, int k) {
    double lo = theta[0], hi = theta[0];
    for (int j = 1; j < k; ++j) {
        lo = fmin(lo, theta[j]);
        hi = fmax(hi, theta[j]);
    }
    return hi - lo;
}

// Device-side error flags raised by validation and by the dense kernels.
enum : int {
    FLAG_BAD_ROWPTR = 1,
    FLAG_BAD_COL = 2,
    FLAG_NO_DIAG = 4,
    FLAG_UNSORTED = 8,
    FLAG_NONFINITE = 16,
    FLAG_CHOLQR_FAIL = 32,   // Cholesky of W^T W failed; later kernels of the iteration skip
    FLAG_RR_FAIL = 64,       // Rayleigh-Ritz failed even without P
    FLAG_RR_PDROP = 128,     // Rayleigh-Ritz dropped P this iteration
    FLAG_CHOLQR_SHIFT = 256, // Cholesky QR needed the diagonal shift
};

// flags[2]: failure branches forced from the host for one attempt of one
// iteration (lobpcg_set_test_faults); the kernels take the branch as if the
// factorisation had failed, so every kernel still runs to its normal end.
enum : int {
    FORCE_CHOLQR_UNSHIFTED = 1,   // the unshifted Cholesky of W^T W "fails": the shifted one runs
    FORCE_CHOLQR = 2,             // both Cholesky factorisations of W^T W "fail"
    FORCE_RR_WITH_P = 4,          // the Rayleigh-Ritz Cholesky of O with P "fails": P is dropped
    FORCE_RR = 8,                 // the Rayleigh-Ritz Cholesky "fails" with and without P
};

// Per-iteration report copied to the host (doubles, padded to kmax).
struct Report {
    double theta[16];
    double rnorm2[16];
    double xnorm2[16];
    double flags;     // device flags as a double (exact for small ints)
    double nblk_used; // blocks used by the last Rayleigh-Ritz
    double pad[6];
};

// Tiled format: per 64-row tile-row a stream of windows over its row view and
// then its column view; a window covers up to `ws` consecutive 64-wide blocks
// ("slots") of X and holds, contiguously in `data`, a table of per-row chunk
// offsets, 16-bit codes (slot within the window << 6 | local index) and the
// values, each row padded to whole 4-entry chunks (see spmm_tiled.hip).
struct TiledFormat {
    int64_t ntilerows = 0, nwin = 0, nbytes = 0, nslots = 0, nent = 0;
    int ws = 0;                    // slots per window, at most
    int emax = 0;                  // chunk-padded entries of the largest window
    char *data = nullptr;          // window blocks
    int64_t *woff = nullptr;       // nwin + 1 byte offsets into data
    int2 *wdesc = nullptr;         // per window: first slot in `list`, slot count
    int32_t *wbeg = nullptr;       // ntilerows + 1: first window of each tile-row
    int32_t *list = nullptr;       // per slot: the 64-wide block of X it stages
};

// Learned preconditioner: FP32 master parameters (the host blob layout) and
// training state, all on the device the network was created on.
struct lobpcg_mlp {
    int device = 0;
    float *params = nullptr;        // LOBPCG_MLP_NBLOB
    float *adam_m = nullptr, *adam_v = nullptr;  // LOBPCG_MLP_NPARAM each
    int adam_t = 0;
    float *grad = nullptr;          // LOBPCG_MLP_NPARAM
    float *grad_partial = nullptr;  // [grad_max_parts][LOBPCG_MLP_NPARAM]
    int grad_max_parts = 0;
    float *so = nullptr;            // per-sample network output, then dL/do
    int64_t so_cap = 0;
    double *gloss = nullptr;        // per-group loss
    int gloss_cap = 0;
    double *loss = nullptr;         // 1
    std::string err;
};
int set_mlp_err(lobpcg_mlp *m, int code, const char *fmt, ...);

struct lobpcg_ctx {
    int64_t n = 0, nnz = 0, nnz_off = 0;
    int dtype = LOBPCG_F32, format = LOBPCG_FORMAT_CSR, format_request = LOBPCG_FORMAT_AUTO, tile = 64, kmax = 16, gram = LOBPCG_GRAM_AUTO;
    size_t esz = 4;
    double tau_rel = 1e-3, eps_rel = 1e-5, gamma = 0.0;
    // diagonal preconditioner shift sigma_j = theta_j - precond_offset * (max theta - min theta)
    double precond_offset = 0.0;
    int refresh_every = 0;  // explicit H X, H P recomputation period (0 = only on apparent convergence)
    // failure branches forced at one iteration (tests of the error paths)
    int test_fault_mask = 0, test_fault_iter = -1;
    // Cholesky QR passes per orthonormalisation of W (2: CholeskyQR2) and soft locking
    int cholqr_passes = 1;
    int soft_lock = 0;
    unsigned long long *mlp_fallback_count = nullptr;   // device counter of per-entry MLP fallbacks
    // block-diagonal preconditioner: dense symmetric 64 x 64 diagonal tiles of H
    // (context dtype, [tile][64][64], unit diagonal past n) and its FOM step count
    void *diag_tiles = nullptr;
    int fom_steps = 4;
    int device = 0;
    // strict upper triangle in CSR + diagonal
    int64_t *rp = nullptr;
    int32_t *ci = nullptr;
    void *val = nullptr;
    void *diag = nullptr;
    // the same strict upper triangle in column order (CSC): the transposed traversal
    int64_t *cp = nullptr;
    int32_t *cri = nullptr;
    void *cval = nullptr;
    TiledFormat tiled;
    // MLP features (float): full-row off-diagonal 1-norm and 64-row tile mean |h|
    float *feat_rownorm = nullptr, *feat_tilemean = nullptr;
    // LOBPCG blocks (n x kmax each)
    void *X = nullptr, *W = nullptr, *P = nullptr, *HX = nullptr, *HW = nullptr, *HP = nullptr;
    // Gram scratch
    double *gram_partial = nullptr;  // [gram_max_wg + gram_max_wg/64 + 1][48*96]: partials, then stage-1 rows
    int gram_max_wg = 0;
    double *gram_out = nullptr;      // up to 48 x 96
    double *gram_out2 = nullptr;     // a second k x k result (Cholesky QR)
    // small dense FP64 state
    double *rr_C = nullptr;          // 48 x 16
    double *rr_theta = nullptr;      // 16
    double *orth_rinv = nullptr;     // 16 x 16 R^{-1}, then 16 x 16 for -(X^T W) R^{-1}
    double *norm_partial = nullptr;  // [norm_max_wg][3*16]
    int norm_max_wg = 0;
    Report *report_dev = nullptr;
    Report *report_host = nullptr;   // pinned
    int *dflags = nullptr;
    lobpcg_mlp *mlp = nullptr;
    unsigned long long *harvest_counter = nullptr;
    // CSR rows whose two segments together exceed HEAVY_ROW entries: each gets a
    // whole workgroup in a second kernel (power-law rows would otherwise hold
    // one 8-lane group for their whole length)
    int32_t *heavy_rows = nullptr;
    int64_t n_heavy = 0;
    hipEvent_t ev[8] = {};
    std::string err;
};

// error helpers -------------------------------------------------------------
int set_err(lobpcg_ctx *ctx, int code, const char *fmt, ...);

#define HIP_TRY(ctx, expr)                                                               \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return set_err((ctx), LOBPCG_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

static inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// launchers implemented across the .hip files --------------------------------
int launch_spmm(lobpcg_ctx *ctx, const void *X, void *Y, int k, hipStream_t s);
// tiled format from host copies of both views of the strict upper triangle
// (CSR rp/ci/val and CSC cp/ri/cv); leaves the CSR format in place when the
// automatic choice finds the tiles too sparse
int build_tiled_format(lobpcg_ctx *ctx, const int64_t *rp, const int32_t *ci, const void *val, const int64_t *cp,
                       const int32_t *ri, const void *cv, hipStream_t s);
int spmm_tiled(lobpcg_ctx *ctx, const void *X, void *Y, int k, hipStream_t s);
int launch_fill_zero(void *p, size_t bytes, hipStream_t s);

// Gram: G = A^T B with A = [a_0 .. a_{na-1}] (each n x wa), B = [b_0 ..] (each n x wb).
struct GramArgs {
    const void *a[3];
    const void *b[6];
    int na, nb, wa, wb;
};
int launch_gram(lobpcg_ctx *ctx, const GramArgs &g, int prec, double *out, hipStream_t s);
// the Rayleigh-Ritz Gram of [X W P] for k = 8 with only eq. Glower's blocks computed
int launch_gram_rr8(lobpcg_ctx *ctx, const void *X, const void *W, const void *P, const void *HX,
                    const void *HW, const void *HP, int prec, double *out, hipStream_t s);

// out = sum_b in_b * M_b  (M_b k x k FP64 row-major; NULL = identity; coef_b scales)
int launch_combine(lobpcg_ctx *ctx, int k, int nin, const void *const *in, const double *const *mats,
                   const double *coef, void *out, hipStream_t s);

// flags[3] holds the soft-lock mask (bit j: column j of W and P left out);
// cholinv treats those columns as absent (identity), Rayleigh-Ritz drops them
int launch_set_flags(lobpcg_ctx *ctx, int f0, int f1, hipStream_t s, int force = 0, int lock = 0);
int launch_cholinv(lobpcg_ctx *ctx, int k, const double *B, double *rinv, hipStream_t s);
// the same for the projection of W against X: B2 is the 2k x 2k Gram of [X W];
// writes R^{-1} of W - X (X^T W) and m2 = -(X^T W) R^{-1}
int launch_cholinv_projected(lobpcg_ctx *ctx, int k, const double *B2, double *rinv, double *m2, hipStream_t s);
int launch_rr(lobpcg_ctx *ctx, int k, int nblk, hipStream_t s);
int launch_update(lobpcg_ctx *ctx, int k, int nblk, int precond, int write_w, hipStream_t s);
int launch_residual(lobpcg_ctx *ctx, int k, int precond, const double *theta, int write_w, hipStream_t s);
int launch_rayleigh_quotients(lobpcg_ctx *ctx, int k, hipStream_t s);
int launch_precond(lobpcg_ctx *ctx, const void *R, const double *theta, void *W, int k, int kind,
                   hipStream_t s);
int mlp_precond_ready(lobpcg_ctx *ctx);
// block-diagonal FOM preconditioner (in_solve: skip after a failed Cholesky QR / Rayleigh-Ritz)
int launch_fom_precond(lobpcg_ctx *ctx, const void *R, const double *theta, void *W, int k, hipStream_t s,
                       bool in_solve = false);
// in_solve: skip after a failed Cholesky QR / Rayleigh-Ritz and count fallbacks
int launch_mlp_precond(lobpcg_ctx *ctx, const void *R, const double *theta, void *W, int k, hipStream_t s,
                       bool in_solve = false);
// one harvest snapshot after iteration `it` of a solve (X, HX, rr_theta current)
int harvest_snapshot(lobpcg_ctx *ctx, int k, lobpcg_harvest *h, hipStream_t s);
// gamma and the per-row network features from both views of the strict upper triangle
int build_row_stats(lobpcg_ctx *ctx, hipStream_t s);
