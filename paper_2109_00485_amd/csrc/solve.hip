// The LOBPCG driver (Algorithm 1).  Every step runs on the device; the host
// only reads a small per-iteration report (Ritz values, residual and column
// norms, flags: about 3k doubles) to take the convergence decision.
//
// One iteration:
//   W <- W - X (X^T W); Cholesky QR of W           (Section 3.5)
//   HW = H W                                        (the only sparse product)
//   G, O from the lower blocks of [X W P]^T [X W P HX HW HP]   (eq. Glower)
//   Rayleigh-Ritz on (G, O) -> C, Theta             (eq. rreig)
//   X, HX, P, HP <- [X W P] C, [HX HW HP] C, ...    (eqs. xupd, pupd, upd1-upd2)
//   R = HX - X Theta, column norms, W = K^{-1} R    (Algorithm 1: residual, preconditioner)
// Convergence: rel_j = ||r_j|| / (max(|theta_j|, tau) ||x_j||) <= tol for the
// nev wanted columns; then H X is recomputed explicitly, theta_j becomes the
// Rayleigh quotient x_j^T H x_j / x_j^T x_j, and the test is repeated.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "internal.hpp"


namespace {

struct Timer {
    lobpcg_ctx *ctx;
    hipStream_t s;
    bool on;
    void mark(int i) {
        if (on) (void)hipEventRecord(ctx->ev[i], s);
    }
    double span(int a, int b) {
        if (!on) return 0.0;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ctx->ev[a], ctx->ev[b]);
        return ms * 1e-3;
    }
};

int read_report(lobpcg_ctx *ctx, hipStream_t s) {
    HIP_TRY(ctx, hipMemcpyAsync(ctx->report_host, ctx->report_dev, sizeof(Report), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return LOBPCG_OK;
}

void rel_from_report(const lobpcg_ctx *ctx, int k, double tau, double *rel, bool *finite) {
    const Report &r = *ctx->report_host;
    *finite = true;
    for (int j = 0; j < k; ++j) {
        double rn = std::sqrt(r.rnorm2[j]), xn = std::sqrt(r.xnorm2[j]);
        rel[j] = rn / (std::max(std::fabs(r.theta[j]), tau) * xn);
        if (!std::isfinite(rel[j]) || !std::isfinite(r.theta[j])) *finite = false;
    }
}

// W <- W - X (X^T W), then one Cholesky QR of the result (Section 3.5), from
// one Gram launch over [X W]: C = X^T W, X^T X and W^T W give the projected
// block's Gram, and one combine writes W R^{-1} - X (C R^{-1}).  Sets the
// device flags as the Cholesky QR does; the combine leaves W as it was when the
// factorisation failed.
int project_cholqr(lobpcg_ctx *ctx, const void *X, void *W, int k, hipStream_t s) {
    GramArgs g{};
    g.a[0] = g.b[0] = X;
    g.a[1] = g.b[1] = W;
    g.na = g.nb = 2;
    g.wa = g.wb = k;
    int rc = launch_gram(ctx, g, ctx->gram, ctx->gram_out2, s);
    if (rc != LOBPCG_OK) return rc;
    double *m2 = ctx->orth_rinv + 16 * 16;
    if ((rc = launch_cholinv_projected(ctx, k, ctx->gram_out2, ctx->orth_rinv, m2, s)) != LOBPCG_OK) return rc;
    const void *in[2] = {W, X};
    const double *mats[2] = {ctx->orth_rinv, m2};
    const double coef[2] = {1.0, 1.0};
    return launch_combine(ctx, k, 2, in, mats, coef, W, s);
}

}  // namespace

extern "C" int lobpcg_solve(lobpcg_ctx *ctx, int k, int nev, void *Xuser, double *evals, double *rel_out, double tol,
                            int maxiter, int precond, lobpcg_info *info, void *stream) {
    if (!ctx) return LOBPCG_EINVAL;
    if (!Xuser || !evals) return set_err(ctx, LOBPCG_EINVAL, "solve: null pointer");
    if (k < 1 || k > ctx->kmax) return set_err(ctx, LOBPCG_EINVAL, "solve: k=%d outside [1,%d]", k, ctx->kmax);
    if (nev < 1 || nev > k) return set_err(ctx, LOBPCG_EINVAL, "solve: need 1 <= nev <= k");
    if ((int64_t)3 * k > ctx->n) return set_err(ctx, LOBPCG_EINVAL, "solve: need 3k <= n");
    if (!(tol > 0)) return set_err(ctx, LOBPCG_EINVAL, "solve: tol must be > 0");
    if (maxiter < 0) return set_err(ctx, LOBPCG_EINVAL, "solve: maxiter must be >= 0");
    if (precond != LOBPCG_PRECOND_NONE && precond != LOBPCG_PRECOND_DIAG && precond != LOBPCG_PRECOND_MLP &&
        precond != LOBPCG_PRECOND_FOM)
        return set_err(ctx, LOBPCG_EINVAL, "solve: bad preconditioner %d", precond);
    if (precond == LOBPCG_PRECOND_MLP) {
        int rc = mlp_precond_ready(ctx);
        if (rc != LOBPCG_OK) return rc;
    }
    hipStream_t s = (hipStream_t)stream;
    const size_t blk = (size_t)ctx->n * k * ctx->esz;
    const double tau = ctx->tau_rel * ctx->gamma;
    const bool timing = info && info->timing;
    Timer tm{ctx, s, timing};
    double t_spmm = 0, t_upd = 0, t_gram = 0, t_rr = 0, t_orth = 0;
    int n_spmm = 0, p_dropped = 0, retries = 0, confirmations = 0, refreshes = 0, shifted = 0, locked_max = 0;
    // failure branches forced from the host (lobpcg_set_test_faults): device bits
    // for attempt `attempt` of iteration `iter` (iteration 0: the initial Rayleigh-Ritz)
    auto forced = [&](int iter, int attempt) -> int {
        const int m = ctx->test_fault_mask;
        if (!m || iter != ctx->test_fault_iter) return 0;
        int f = 0;
        if (attempt == 0 && (m & LOBPCG_FAULT_CHOLQR_SHIFT)) f |= FORCE_CHOLQR_UNSHIFTED;
        if ((attempt == 0 && (m & LOBPCG_FAULT_CHOLQR_ONCE)) || (m & LOBPCG_FAULT_CHOLQR_ALWAYS)) f |= FORCE_CHOLQR;
        if (m & LOBPCG_FAULT_RR_DROP_P) f |= FORCE_RR_WITH_P;
        if (m & LOBPCG_FAULT_RR) f |= FORCE_RR;
        return f;
    };
    // the learned and the block-diagonal preconditioners act on W = R after the update
    const int upd_precond = precond == LOBPCG_PRECOND_DIAG ? LOBPCG_PRECOND_DIAG : LOBPCG_PRECOND_NONE;
    auto apply_after_update = [&]() -> int {
        if (precond == LOBPCG_PRECOND_MLP) return launch_mlp_precond(ctx, ctx->W, ctx->rr_theta, ctx->W, k, s, true);
        if (precond == LOBPCG_PRECOND_FOM) return launch_fom_precond(ctx, ctx->W, ctx->rr_theta, ctx->W, k, s, true);
        return LOBPCG_OK;
    };
    auto gram_rr_input = [&](int nb) -> int {
        if (k == 8 && nb == 3)
            return launch_gram_rr8(ctx, ctx->X, ctx->W, ctx->P, ctx->HX, ctx->HW, ctx->HP, ctx->gram, ctx->gram_out, s);
        GramArgs g{};
        void *S[3] = {ctx->X, ctx->W, ctx->P};
        void *HS[3] = {ctx->HX, ctx->HW, ctx->HP};
        g.na = nb;
        g.nb = 2 * nb;
        g.wa = g.wb = k;
        for (int b = 0; b < nb; ++b) {
            g.a[b] = S[b];
            g.b[b] = S[b];
            g.b[nb + b] = HS[b];
        }
        return launch_gram(ctx, g, ctx->gram, ctx->gram_out, s);
    };
    int rc;
#define TRY(expr)                             \
    do {                                      \
        rc = (expr);                          \
        if (rc != LOBPCG_OK) return rc;       \
    } while (0)

    HIP_TRY(ctx, hipMemcpyAsync(ctx->X, Xuser, blk, hipMemcpyDeviceToDevice, s));
    TRY(launch_fill_zero(ctx->mlp_fallback_count, sizeof(unsigned long long), s));
    TRY(launch_set_flags(ctx, 0, 0, s, forced(0, 0)));
    tm.mark(0);
    // Algorithm 1, start: Rayleigh-Ritz on X0
    TRY(launch_spmm(ctx, ctx->X, ctx->HX, k, s));
    ++n_spmm;
    tm.mark(1);
    TRY(gram_rr_input(1));
    tm.mark(2);
    TRY(launch_rr(ctx, k, 1, s));
    tm.mark(3);
    TRY(launch_update(ctx, k, 1, upd_precond, 1, s));
    TRY(apply_after_update());
    tm.mark(4);
    TRY(read_report(ctx, s));
    t_spmm += tm.span(0, 1); t_gram += tm.span(1, 2); t_rr += tm.span(2, 3); t_upd += tm.span(3, 4);
    if ((int)ctx->report_host->flags & FLAG_RR_FAIL) return set_err(ctx, LOBPCG_ENOTSPD, "initial Rayleigh-Ritz failed");

    std::vector<double> rel(k);
    bool finite = true;
    // optional progress trace on stderr: LOBPCG_TRACE=<every n iterations>
    const char *tr = getenv("LOBPCG_TRACE");
    const int trace_every = tr ? std::max(1, atoi(tr)) : 0;
    bool have_p = false;
    int it = 0;
    int status = LOBPCG_ENOCONV;
    for (;;) {
        rel_from_report(ctx, k, tau, rel.data(), &finite);
        if (!finite) { status = set_err(ctx, LOBPCG_ENONFINITE, "non-finite residual at iteration %d", it); break; }
        bool conv = true;
        for (int j = 0; j < nev; ++j) conv = conv && rel[j] <= tol;
        if (conv) {
            // confirm with an explicit product (the recurrences drift)
            ++confirmations;
            tm.mark(0);
            TRY(launch_spmm(ctx, ctx->X, ctx->HX, k, s));
            ++n_spmm;
            tm.mark(1);
            GramArgs g{};
            g.a[0] = ctx->X;
            g.b[0] = ctx->X;
            g.b[1] = ctx->HX;
            g.na = 1; g.nb = 2; g.wa = g.wb = k;
            // the reported Ritz values: Rayleigh quotients with FP64 accumulation
            TRY(launch_gram(ctx, g, LOBPCG_GRAM_F64, ctx->gram_out, s));
            TRY(launch_rayleigh_quotients(ctx, k, s));
            tm.mark(2);
            TRY(launch_update(ctx, k, 0, upd_precond, 1, s));
            TRY(apply_after_update());
            tm.mark(3);
            TRY(read_report(ctx, s));
            t_spmm += tm.span(0, 1); t_gram += tm.span(1, 2); t_upd += tm.span(2, 3);
            rel_from_report(ctx, k, tau, rel.data(), &finite);
            if (!finite) { status = set_err(ctx, LOBPCG_ENONFINITE, "non-finite residual at iteration %d", it); break; }
            conv = true;
            for (int j = 0; j < nev; ++j) conv = conv && rel[j] <= tol;
            if (conv) { status = LOBPCG_OK; break; }
        }
        if (it >= maxiter) break;
        ++it;
        // soft locking: the columns converged at this check leave W and P
        int lock = 0;
        if (ctx->soft_lock)
            for (int j = 0; j < k; ++j)
                if (rel[j] <= tol) lock |= 1 << j;
        if (lock == (1 << k) - 1) lock = 0;   // (cannot happen: every column converged ends the solve)
        locked_max = std::max(locked_max, __builtin_popcount(lock));
        bool done_iter = false, rr_failed = false;
        for (int attempt = 0; attempt < 2 && !done_iter && !rr_failed; ++attempt) {
            TRY(launch_set_flags(ctx, 0, 0, s, forced(it, attempt), lock));
            tm.mark(0);
            // W <- W - X (X^T W), then Cholesky QR
            {
                GramArgs g{};
                const void *in1[1] = {ctx->W};
                const double *mats1[1] = {ctx->orth_rinv};
                const double coef1[1] = {1.0};
                if (attempt == 0) {
                    TRY(project_cholqr(ctx, ctx->X, ctx->W, k, s));
                } else {
                    // the retry after a failed factorisation (W left as it was):
                    // project twice, then Cholesky QR of the stored block
                    g.a[0] = ctx->X; g.b[0] = ctx->W; g.na = g.nb = 1; g.wa = g.wb = k;
                    const void *in[2] = {ctx->W, ctx->X};
                    const double *mats[2] = {nullptr, ctx->gram_out2};
                    const double coef[2] = {1.0, -1.0};
                    for (int pass = 0; pass < 2; ++pass) {
                        TRY(launch_gram(ctx, g, ctx->gram, ctx->gram_out2, s));
                        TRY(launch_combine(ctx, k, 2, in, mats, coef, ctx->W, s));
                    }
                    g.a[0] = ctx->W;
                    TRY(launch_gram(ctx, g, ctx->gram, ctx->gram_out2, s));
                    TRY(launch_cholinv(ctx, k, ctx->gram_out2, ctx->orth_rinv, s));
                    TRY(launch_combine(ctx, k, 1, in1, mats1, coef1, ctx->W, s));
                }
                g = GramArgs{};
                g.a[0] = g.b[0] = ctx->W; g.na = g.nb = 1; g.wa = g.wb = k;
                if (ctx->cholqr_passes == 2) {
                    // CholeskyQR2: a second Cholesky QR of the orthonormalised W
                    TRY(launch_gram(ctx, g, ctx->gram, ctx->gram_out2, s));
                    TRY(launch_cholinv(ctx, k, ctx->gram_out2, ctx->orth_rinv, s));
                    TRY(launch_combine(ctx, k, 1, in1, mats1, coef1, ctx->W, s));
                }
            }
            tm.mark(1);
            TRY(launch_spmm(ctx, ctx->W, ctx->HW, k, s));
            tm.mark(2);
            const int nb = have_p ? 3 : 2;
            TRY(gram_rr_input(nb));
            tm.mark(3);
            TRY(launch_rr(ctx, k, nb, s));
            tm.mark(4);
            TRY(launch_update(ctx, k, nb, upd_precond, 1, s));
            TRY(apply_after_update());
            tm.mark(5);
            TRY(read_report(ctx, s));
            const int fl = (int)ctx->report_host->flags;
            if (fl & FLAG_CHOLQR_FAIL) {
                ++retries;
                continue;  // W was only projected; project again and retry once
            }
            ++n_spmm;
            t_orth += tm.span(0, 1); t_spmm += tm.span(1, 2); t_gram += tm.span(2, 3);
            t_rr += tm.span(3, 4); t_upd += tm.span(4, 5);
            if (fl & FLAG_RR_FAIL) {
                // X, HX and P are untouched by the skipped update: the last iterate is returned
                rr_failed = true;
                break;
            }
            if (fl & FLAG_RR_PDROP) ++p_dropped;
            if (fl & FLAG_CHOLQR_SHIFT) ++shifted;
            have_p = true;
            done_iter = true;
        }
        if (rr_failed) { status = set_err(ctx, LOBPCG_ENOTSPD, "Rayleigh-Ritz failed at iteration %d", it); break; }
        if (!done_iter) { status = set_err(ctx, LOBPCG_ENOTSPD, "Cholesky QR failed twice at iteration %d", it); break; }
        if (ctx->refresh_every && it % ctx->refresh_every == 0) {
            // the recurrences eqs. upd1-upd2 drift in FP32: recompute H X and H P
            tm.mark(0);
            TRY(launch_spmm(ctx, ctx->X, ctx->HX, k, s));
            TRY(launch_spmm(ctx, ctx->P, ctx->HP, k, s));
            n_spmm += 2;
            ++refreshes;
            tm.mark(1);
            TRY(launch_update(ctx, k, 0, upd_precond, 1, s));
            TRY(apply_after_update());
            tm.mark(2);
            TRY(read_report(ctx, s));
            t_spmm += tm.span(0, 1); t_upd += tm.span(1, 2);
        }
        if (info && info->harvest && it % std::max(1, info->harvest->every) == 0 && !info->harvest->full) {
            // training samples for the learned preconditioner from this iterate
            TRY(harvest_snapshot(ctx, k, info->harvest, s));
        }
        if (trace_every && it % trace_every == 0) {
            rel_from_report(ctx, k, tau, rel.data(), &finite);
            fprintf(stderr, "[lobpcg] it %5d flags 0x%03x nblk %d theta", it, (int)ctx->report_host->flags,
                    (int)ctx->report_host->nblk_used);
            for (int j = 0; j < nev; ++j) fprintf(stderr, " %.9g", ctx->report_host->theta[j]);
            fprintf(stderr, " rel");
            for (int j = 0; j < k; ++j) fprintf(stderr, " %.2e", rel[j]);
            fprintf(stderr, "\n");
        }
        if (info && info->theta_hist && info->rel_hist) {
            rel_from_report(ctx, k, tau, rel.data(), &finite);
            for (int j = 0; j < k; ++j) {
                info->theta_hist[(size_t)(it - 1) * k + j] = ctx->report_host->theta[j];
                info->rel_hist[(size_t)(it - 1) * k + j] = rel[j];
            }
        }
    }
#undef TRY
    HIP_TRY(ctx, hipMemcpyAsync(Xuser, ctx->X, blk, hipMemcpyDeviceToDevice, s));
    unsigned long long fallbacks = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&fallbacks, ctx->mlp_fallback_count, sizeof fallbacks, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    rel_from_report(ctx, k, tau, rel.data(), &finite);
    for (int j = 0; j < k; ++j) {
        evals[j] = ctx->report_host->theta[j];
        if (rel_out) rel_out[j] = rel[j];
    }
    if (info) {
        info->iters = it;
        info->n_spmm = n_spmm;
        info->p_dropped = p_dropped;
        info->cholqr_retries = retries;
        info->confirmations = confirmations;
        info->refreshes = refreshes;
        info->cholqr_shifted = shifted;
        info->locked_max = locked_max;
        info->mlp_fallbacks = (long long)fallbacks;
        info->status = status;
        info->gamma = ctx->gamma;
        info->t_spmm = t_spmm;
        info->t_precond_update = t_upd;
        info->t_gram = t_gram;
        info->t_rr = t_rr;
        info->t_orth = t_orth;
        info->t_total = t_spmm + t_upd + t_gram + t_rr + t_orth;
    }
    if (status == LOBPCG_ENOCONV) set_err(ctx, status, "not converged after %d iterations", it);
    return status;
}

// Cholesky QR of a caller's block in place (Section 3.5): B = W^T W, B = R^T R,
// W <- W R^{-1}, once or twice; the shifted factorisation is the fallback of
// each pass, as in the solve.
extern "C" int lobpcg_cholqr(lobpcg_ctx *ctx, void *W, int k, int passes, int *shifted, void *stream) {
    if (!ctx) return LOBPCG_EINVAL;
    if (!W) return set_err(ctx, LOBPCG_EINVAL, "cholqr: null pointer");
    if (k < 1 || k > ctx->kmax) return set_err(ctx, LOBPCG_EINVAL, "cholqr: k=%d outside [1,%d]", k, ctx->kmax);
    if (passes != 1 && passes != 2) return set_err(ctx, LOBPCG_EINVAL, "cholqr: passes %d not 1 or 2", passes);
    hipStream_t s = (hipStream_t)stream;
    int nshift = 0;
    for (int pass = 0; pass < passes; ++pass) {
        int rc = launch_set_flags(ctx, 0, 0, s, 0, 0);
        if (rc != LOBPCG_OK) return rc;
        GramArgs g{};
        g.a[0] = W; g.b[0] = W; g.na = g.nb = 1; g.wa = g.wb = k;
        if ((rc = launch_gram(ctx, g, ctx->gram, ctx->gram_out2, s)) != LOBPCG_OK) return rc;
        if ((rc = launch_cholinv(ctx, k, ctx->gram_out2, ctx->orth_rinv, s)) != LOBPCG_OK) return rc;
        const void *in1[1] = {W};
        const double *mats1[1] = {ctx->orth_rinv};
        const double coef1[1] = {1.0};
        if ((rc = launch_combine(ctx, k, 1, in1, mats1, coef1, W, s)) != LOBPCG_OK) return rc;
        int fl = 0;
        HIP_TRY(ctx, hipMemcpyAsync(&fl, ctx->dflags, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        if (fl & FLAG_CHOLQR_FAIL) return set_err(ctx, LOBPCG_ENOTSPD, "cholqr: W^T W not positive definite (pass %d)", pass + 1);
        if (fl & FLAG_CHOLQR_SHIFT) ++nshift;
    }
    if (shifted) *shifted = nshift;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_err(ctx, LOBPCG_EHIP, "cholqr launch: %s", hipGetErrorString(e));
    return LOBPCG_OK;
}

// The orthogonalisation step of lobpcg_solve on a caller's blocks.
extern "C" int lobpcg_orthonormalize(lobpcg_ctx *ctx, const void *X, void *W, int k, int *shifted, void *stream) {
    if (!ctx) return LOBPCG_EINVAL;
    if (!X || !W) return set_err(ctx, LOBPCG_EINVAL, "orthonormalize: null pointer");
    if (k < 1 || k > ctx->kmax) return set_err(ctx, LOBPCG_EINVAL, "orthonormalize: k=%d outside [1,%d]", k, ctx->kmax);
    hipStream_t s = (hipStream_t)stream;
    int rc = launch_set_flags(ctx, 0, 0, s, 0, 0);
    if (rc == LOBPCG_OK) rc = project_cholqr(ctx, X, W, k, s);
    if (rc != LOBPCG_OK) return rc;
    int fl = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&fl, ctx->dflags, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (shifted) *shifted = (fl & FLAG_CHOLQR_SHIFT) ? 1 : 0;
    if (fl & FLAG_CHOLQR_FAIL) return set_err(ctx, LOBPCG_ENOTSPD, "orthonormalize: projected Gram not positive definite");
    return LOBPCG_OK;
}
