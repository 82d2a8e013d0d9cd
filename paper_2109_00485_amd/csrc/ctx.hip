// Context lifecycle: CSR validation, the library's own copy of H (strict upper
// triangle + diagonal), the Gershgorin bound, the per-row features of the
// learned preconditioner, and every workspace allocated once up front.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>

#include "internal.hpp"

int set_err(lobpcg_ctx *ctx, int code, const char *fmt, ...) {
    // the status carries a runtime failure: clear it so the caller's next HIP call
    // does not report it again
    if (code == LOBPCG_EHIP || code == LOBPCG_ENOMEM) (void)hipGetLastError();
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

namespace {

template <typename T>
__device__ inline bool finite_val(T v) { return isfinite((double)v); }

// One thread per row.  Every index is checked against [0, nnz) before it is
// dereferenced, so a malformed row_ptr cannot cause an out-of-bounds read.
template <typename T>
__global__ void validate_rows(int64_t n, int64_t nnz, const int64_t *__restrict__ rp,
                              const int32_t *__restrict__ col, const T *__restrict__ val,
                              int *__restrict__ flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t b = rp[i], e = rp[i + 1];
    int f = 0;
    if (i == 0 && b != 0) f |= FLAG_BAD_ROWPTR;
    if (b < 0 || e < b || e > nnz) {
        atomicOr(flags, f | FLAG_BAD_ROWPTR);
        return;
    }
    if (e == b || col[b] != (int32_t)i) f |= FLAG_NO_DIAG;
    int32_t prev = -1;
    for (int64_t q = b; q < e; ++q) {
        int32_t c = col[q];
        if (c < (int32_t)i || (int64_t)c >= n) f |= FLAG_BAD_COL;
        if (q > b && c <= prev) f |= FLAG_UNSORTED;
        if (!finite_val(val[q])) f |= FLAG_NONFINITE;
        prev = c;
    }
    if (f) atomicOr(flags, f);
}

__global__ void strict_rowptr(int64_t n, const int64_t *__restrict__ rp, int64_t *__restrict__ rps) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i <= n) rps[i] = rp[i] - i;
}

// One wavefront per row: split the row into its diagonal and strict part.
template <typename T>
__global__ void split_rows(int64_t n, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                           const T *__restrict__ val, int32_t *__restrict__ ci, T *__restrict__ vs,
                           T *__restrict__ diag) {
    int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LOBPCG_WAVE;
    int lane = threadIdx.x % LOBPCG_WAVE;
    if (i >= n) return;
    int64_t b = rp[i], e = rp[i + 1];
    for (int64_t q = b + 1 + lane; q < e; q += LOBPCG_WAVE) {
        int64_t dst = q - i - 1;
        ci[dst] = col[q];
        vs[dst] = val[q];
    }
    if (lane == 0) diag[i] = val[b];
}

// |h| statistics of the full symmetric rows from the two views of the strict
// upper triangle (row view rp/val, column view cp/cval): one wavefront per row,
// lane-strided sums combined by a fixed shuffle tree, so the results are the
// same in every run.  gamma = max_i (|d_i| + sum_{j != i} |h_ij|) (a maximum:
// any order gives the same value).
template <typename T>
__global__ void full_row_stats(int64_t n, const int64_t *__restrict__ rp, const T *__restrict__ val,
                               const int64_t *__restrict__ cp, const T *__restrict__ cval, const T *__restrict__ diag,
                               double *__restrict__ absrow, float *__restrict__ rownorm,
                               unsigned long long *__restrict__ gmax) {
    int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LOBPCG_WAVE;
    int lane = threadIdx.x % LOBPCG_WAVE;
    if (i >= n) return;
    double s = 0.0;
    for (int64_t q = rp[i] + lane; q < rp[i + 1]; q += LOBPCG_WAVE) s += fabs((double)val[q]);
    for (int64_t q = cp[i] + lane; q < cp[i + 1]; q += LOBPCG_WAVE) s += fabs((double)cval[q]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) {
        absrow[i] = s;
        rownorm[i] = (float)s;
        const double g = s + fabs((double)diag[i]);
        // non-negative doubles order like their bit patterns
        atomicMax(gmax, (unsigned long long)__double_as_longlong(g));
    }
}

// Mean |h| over the off-diagonal nonzeros of each 64-row tile-row: one
// wavefront per tile-row, fixed shuffle tree.
__global__ void tile_stats(int64_t n, const int64_t *__restrict__ rp, const int64_t *__restrict__ cp,
                           const double *__restrict__ absrow, float *__restrict__ tm) {
    const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LOBPCG_WAVE;
    const int lane = threadIdx.x % LOBPCG_WAVE;
    const int64_t i = t * 64 + lane;
    if (t * 64 >= n) return;
    double a = 0.0;
    int64_t c = 0;
    if (i < n) {
        a = absrow[i];
        c = (rp[i + 1] - rp[i]) + (cp[i + 1] - cp[i]);
    }
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        c += __shfl_xor(c, off);
    }
    if (i < n) tm[i] = c > 0 ? (float)(a / (double)c) : 0.0f;
}

template <typename T>
int build_csr(lobpcg_ctx *ctx, const int64_t *rp, const int32_t *col, const void *valv, hipStream_t s) {
    const T *val = (const T *)valv;
    const int64_t n = ctx->n;
    strict_rowptr<<<ceil_div(n + 1, 256), 256, 0, s>>>(n, rp, ctx->rp);
    split_rows<T><<<ceil_div(n * LOBPCG_WAVE, 256), 256, 0, s>>>(n, rp, col, val, ctx->ci, (T *)ctx->val,
                                                                 (T *)ctx->diag);
    HIP_TRY(ctx, hipGetLastError());
    return LOBPCG_OK;
}

}  // namespace

// gamma and the per-row network features, once both views of the strict upper
// triangle exist (called by the column-view build)
int build_row_stats(lobpcg_ctx *ctx, hipStream_t s) {
    const int64_t n = ctx->n;
    double *absrow = nullptr;
    unsigned long long *gmax = nullptr;
    HIP_TRY(ctx, hipMallocAsync((void **)&absrow, n * sizeof(double), s));
    HIP_TRY(ctx, hipMallocAsync((void **)&gmax, sizeof(unsigned long long), s));
    HIP_TRY(ctx, hipMemsetAsync(gmax, 0, sizeof(unsigned long long), s));
    const int grid = ceil_div(n * LOBPCG_WAVE, 256);
    if (ctx->dtype == LOBPCG_F32)
        full_row_stats<float><<<grid, 256, 0, s>>>(n, ctx->rp, (const float *)ctx->val, ctx->cp,
                                                   (const float *)ctx->cval, (const float *)ctx->diag, absrow,
                                                   ctx->feat_rownorm, gmax);
    else
        full_row_stats<double><<<grid, 256, 0, s>>>(n, ctx->rp, (const double *)ctx->val, ctx->cp,
                                                    (const double *)ctx->cval, (const double *)ctx->diag, absrow,
                                                    ctx->feat_rownorm, gmax);
    tile_stats<<<ceil_div(((n + 63) / 64) * LOBPCG_WAVE, 256), 256, 0, s>>>(n, ctx->rp, ctx->cp, absrow,
                                                                             ctx->feat_tilemean);
    unsigned long long g = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&g, gmax, sizeof g, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    HIP_TRY(ctx, hipGetLastError());
    double gd;
    memcpy(&gd, &g, sizeof gd);
    ctx->gamma = gd;
    (void)hipFreeAsync(absrow, s);
    (void)hipFreeAsync(gmax, s);
    return LOBPCG_OK;
}

namespace {

void free_ctx(lobpcg_ctx *c) {
    if (!c) return;
    void *ptrs[] = {c->rp, c->ci, c->val, c->diag, c->cp, c->cri, c->cval, c->feat_rownorm, c->feat_tilemean, c->X, c->W, c->P,
                    c->HX, c->HW, c->HP, c->gram_partial, c->gram_out, c->gram_out2, c->rr_C, c->rr_theta,
                    c->orth_rinv, c->norm_partial, c->report_dev, c->dflags, c->tiled.data, c->tiled.woff,
                    c->tiled.wdesc, c->tiled.wbeg, c->tiled.list, c->harvest_counter, c->mlp_fallback_count, c->diag_tiles,
                    c->heavy_rows};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (c->report_host) (void)hipHostFree(c->report_host);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

}  // namespace

int build_column_view(lobpcg_ctx *ctx, hipStream_t s);  // spmm.hip

extern "C" void lobpcg_opts_default(lobpcg_opts *o) {
    if (!o) return;
    o->dtype = LOBPCG_F32;
    o->gram = LOBPCG_GRAM_AUTO;
    o->format = LOBPCG_FORMAT_AUTO;
    o->tile = 64;
    o->kmax = 16;
    o->tau_rel = 1e-3;
    o->eps_rel = 1e-5;
}

extern "C" const char *lobpcg_strerror(int status) {
    switch (status) {
        case LOBPCG_OK: return "ok";
        case LOBPCG_EINVAL: return "invalid argument or malformed matrix";
        case LOBPCG_ENOMEM: return "device allocation failed";
        case LOBPCG_EHIP: return "HIP runtime error";
        case LOBPCG_ENOTSPD: return "Cholesky QR / Rayleigh-Ritz lost positive definiteness";
        case LOBPCG_ENOCONV: return "not converged within maxiter";
        case LOBPCG_ENONFINITE: return "non-finite values";
        case LOBPCG_EUNSUPPORTED: return "unsupported request";
        default: return "unknown status";
    }
}

extern "C" const char *lobpcg_last_error(const lobpcg_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" int lobpcg_set_test_faults(lobpcg_ctx *ctx, int mask, int iteration) {
    if (!ctx) return LOBPCG_EINVAL;
    const int all = LOBPCG_FAULT_CHOLQR_SHIFT | LOBPCG_FAULT_CHOLQR_ONCE | LOBPCG_FAULT_CHOLQR_ALWAYS |
                    LOBPCG_FAULT_RR_DROP_P | LOBPCG_FAULT_RR;
    if ((mask & ~all) || iteration < 0) return set_err(ctx, LOBPCG_EINVAL, "test faults: bad mask 0x%x or iteration %d", mask, iteration);
    ctx->test_fault_mask = mask;
    ctx->test_fault_iter = iteration;
    return LOBPCG_OK;
}

extern "C" int lobpcg_set_cholqr_passes(lobpcg_ctx *ctx, int passes) {
    if (!ctx) return LOBPCG_EINVAL;
    if (passes != 1 && passes != 2) return set_err(ctx, LOBPCG_EINVAL, "Cholesky QR passes %d not 1 or 2", passes);
    ctx->cholqr_passes = passes;
    return LOBPCG_OK;
}

extern "C" int lobpcg_set_soft_lock(lobpcg_ctx *ctx, int on) {
    if (!ctx) return LOBPCG_EINVAL;
    if (on != 0 && on != 1) return set_err(ctx, LOBPCG_EINVAL, "soft lock %d not 0 or 1", on);
    ctx->soft_lock = on;
    return LOBPCG_OK;
}

extern "C" int lobpcg_set_precond_offset(lobpcg_ctx *ctx, double c) {
    if (!ctx) return LOBPCG_EINVAL;
    if (!(c >= 0.0) || !(c <= 1e6)) return set_err(ctx, LOBPCG_EINVAL, "precond offset %g outside [0, 1e6]", c);
    ctx->precond_offset = c;
    return LOBPCG_OK;
}

extern "C" int lobpcg_create(lobpcg_ctx **out, int64_t n, const int64_t *row_ptr, const int32_t *col,
                             const void *val, const lobpcg_opts *opts_in, void *stream) {
    if (!out) return LOBPCG_EINVAL;
    *out = nullptr;
    lobpcg_opts o;
    lobpcg_opts_default(&o);
    if (opts_in) o = *opts_in;
    if (n < 1 || n >= (int64_t)1 << 31) return LOBPCG_EINVAL;
    if (!row_ptr || !col || !val) return LOBPCG_EINVAL;
    if (o.dtype != LOBPCG_F32 && o.dtype != LOBPCG_F64) return LOBPCG_EINVAL;
    if (o.kmax < 1 || o.kmax > 16) return LOBPCG_EINVAL;
    if (o.gram < LOBPCG_GRAM_AUTO || o.gram > LOBPCG_GRAM_BF16X6) return LOBPCG_EINVAL;
    if ((o.gram == LOBPCG_GRAM_BF16X3 || o.gram == LOBPCG_GRAM_BF16X6) && o.dtype != LOBPCG_F32) return LOBPCG_EINVAL;
    if (o.format < LOBPCG_FORMAT_AUTO || o.format > LOBPCG_FORMAT_TILED) return LOBPCG_EINVAL;
    if (o.tile != 64) return LOBPCG_EUNSUPPORTED;
    if (!(o.tau_rel > 0) || !(o.eps_rel > 0)) return LOBPCG_EINVAL;
    hipStream_t s = (hipStream_t)stream;

    lobpcg_ctx *ctx = new (std::nothrow) lobpcg_ctx();
    if (!ctx) return LOBPCG_ENOMEM;
    ctx->n = n;
    ctx->dtype = o.dtype;
    ctx->esz = o.dtype == LOBPCG_F32 ? 4 : 8;
    ctx->kmax = o.kmax;
    // FP32 blocks: FP64 accumulation of the exact FP32 products by default (an FP32
    // accumulation leaves the residual floor of the solve above 1e-6)
    ctx->gram = o.gram == LOBPCG_GRAM_AUTO ? LOBPCG_GRAM_F64 : o.gram;
    ctx->refresh_every = o.dtype == LOBPCG_F32 ? 20 : 0;
    ctx->tile = o.tile;
    ctx->tau_rel = o.tau_rel;
    ctx->eps_rel = o.eps_rel;
    (void)hipGetDevice(&ctx->device);

    auto fail = [&](int code) {
        free_ctx(ctx);
        // the status carries the failure: leave no runtime error behind for the
        // caller's next HIP call (a failed hipMalloc is otherwise reported again)
        (void)hipGetLastError();
        return code;
    };
    int64_t nnz = 0;
    if (hipMemcpyAsync(&nnz, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(LOBPCG_EHIP);
    if (nnz < n) return fail(LOBPCG_EINVAL);
    ctx->nnz = nnz;
    ctx->nnz_off = nnz - n;

    if (hipMalloc((void **)&ctx->dflags, sizeof(int) * 4) != hipSuccess) return fail(LOBPCG_ENOMEM);
    if (hipMemsetAsync(ctx->dflags, 0, sizeof(int) * 4, s) != hipSuccess) return fail(LOBPCG_EHIP);
    if (o.dtype == LOBPCG_F32)
        validate_rows<float><<<ceil_div(n, 256), 256, 0, s>>>(n, nnz, row_ptr, col, (const float *)val, ctx->dflags);
    else
        validate_rows<double><<<ceil_div(n, 256), 256, 0, s>>>(n, nnz, row_ptr, col, (const double *)val,
                                                               ctx->dflags);
    int hflags = 0;
    if (hipMemcpyAsync(&hflags, ctx->dflags, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(LOBPCG_EHIP);
    if (hflags & (FLAG_BAD_ROWPTR | FLAG_BAD_COL | FLAG_NO_DIAG | FLAG_UNSORTED)) {
        lobpcg_ctx tmp;
        set_err(&tmp, 0, "malformed CSR (flags 0x%x: rowptr=%d col=%d diag=%d sorted=%d)", hflags,
                !!(hflags & FLAG_BAD_ROWPTR), !!(hflags & FLAG_BAD_COL), !!(hflags & FLAG_NO_DIAG),
                !!(hflags & FLAG_UNSORTED));
        fprintf(stderr, "lobpcg_create: %s\n", tmp.err.c_str());
        return fail(LOBPCG_EINVAL);
    }
    if (hflags & FLAG_NONFINITE) return fail(LOBPCG_ENONFINITE);

    const size_t esz = ctx->esz;
    const size_t blk = (size_t)n * o.kmax * esz;
    bool ok = hipMalloc((void **)&ctx->rp, (n + 1) * sizeof(int64_t)) == hipSuccess &&
              hipMalloc((void **)&ctx->ci, (ctx->nnz_off ? ctx->nnz_off : 1) * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&ctx->val, (ctx->nnz_off ? ctx->nnz_off : 1) * esz) == hipSuccess &&
              hipMalloc(&ctx->diag, n * esz) == hipSuccess &&
              hipMalloc((void **)&ctx->feat_rownorm, n * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&ctx->feat_tilemean, n * sizeof(float)) == hipSuccess &&
              hipMalloc(&ctx->X, blk) == hipSuccess && hipMalloc(&ctx->W, blk) == hipSuccess &&
              hipMalloc(&ctx->P, blk) == hipSuccess && hipMalloc(&ctx->HX, blk) == hipSuccess &&
              hipMalloc(&ctx->HW, blk) == hipSuccess && hipMalloc(&ctx->HP, blk) == hipSuccess;
    ctx->gram_max_wg = 1024;
    ctx->norm_max_wg = 2048;
    ok = ok && hipMalloc((void **)&ctx->gram_partial, ((size_t)ctx->gram_max_wg + ctx->gram_max_wg / 64 + 1) * 48 * 96 * sizeof(double)) == hipSuccess &&
         hipMalloc((void **)&ctx->gram_out, 48 * 96 * sizeof(double)) == hipSuccess &&
         hipMalloc((void **)&ctx->gram_out2, 48 * 96 * sizeof(double)) == hipSuccess &&
         hipMalloc((void **)&ctx->rr_C, 48 * 16 * sizeof(double)) == hipSuccess &&
         hipMalloc((void **)&ctx->rr_theta, 16 * sizeof(double)) == hipSuccess &&
         hipMalloc((void **)&ctx->orth_rinv, 2 * 16 * 16 * sizeof(double)) == hipSuccess &&
         hipMalloc((void **)&ctx->norm_partial, (size_t)ctx->norm_max_wg * 3 * 16 * sizeof(double)) == hipSuccess &&
         hipMalloc((void **)&ctx->report_dev, sizeof(Report)) == hipSuccess &&
         hipMalloc((void **)&ctx->mlp_fallback_count, sizeof(unsigned long long)) == hipSuccess &&
         hipHostMalloc((void **)&ctx->report_host, sizeof(Report), hipHostMallocDefault) == hipSuccess;
    for (auto &e : ctx->ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    if (!ok) return fail(LOBPCG_ENOMEM);

    int rc = o.dtype == LOBPCG_F32 ? build_csr<float>(ctx, row_ptr, col, val, s)
                                   : build_csr<double>(ctx, row_ptr, col, val, s);
    if (rc != LOBPCG_OK) return fail(rc);
    ctx->format = LOBPCG_FORMAT_CSR;
    ctx->format_request = o.format;
    rc = build_column_view(ctx, s);
    if (rc != LOBPCG_OK) return fail(rc);
    if (hipStreamSynchronize(s) != hipSuccess) return fail(LOBPCG_EHIP);
    *out = ctx;
    return LOBPCG_OK;
}

namespace {
__global__ void widen_offsets_kernel(int64_t m, const int32_t *__restrict__ in, int64_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] = in[i];
}
}  // namespace

extern "C" int lobpcg_create_rp32(lobpcg_ctx **out, int64_t n, const int32_t *row_ptr, const int32_t *col,
                                  const void *val, const lobpcg_opts *opts, void *stream) {
    if (!out) return LOBPCG_EINVAL;
    *out = nullptr;
    if (n < 1 || n >= (int64_t)1 << 31 || !row_ptr) return LOBPCG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int64_t *rp64 = nullptr;
    if (hipMalloc((void **)&rp64, (n + 1) * sizeof(int64_t)) != hipSuccess) {
        (void)hipGetLastError();
        return LOBPCG_ENOMEM;
    }
    widen_offsets_kernel<<<ceil_div(n + 1, 256), 256, 0, s>>>(n + 1, row_ptr, rp64);
    int rc = hipGetLastError() == hipSuccess ? lobpcg_create(out, n, rp64, col, val, opts, stream) : LOBPCG_EHIP;
    (void)hipStreamSynchronize(s);
    (void)hipFree(rp64);
    return rc;
}

extern "C" void lobpcg_destroy(lobpcg_ctx *ctx) {
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    free_ctx(ctx);
}

extern "C" int lobpcg_query(const lobpcg_ctx *ctx, int64_t *n, int64_t *nnz, int *format, int *dtype,
                            double *gamma) {
    if (!ctx) return LOBPCG_EINVAL;
    if (n) *n = ctx->n;
    if (nnz) *nnz = ctx->nnz;
    if (format) *format = ctx->format;
    if (dtype) *dtype = ctx->dtype;
    if (gamma) *gamma = ctx->gamma;
    return LOBPCG_OK;
}

extern "C" int lobpcg_get_diag(lobpcg_ctx *ctx, void *d, void *stream) {
    if (!ctx || !d) return LOBPCG_EINVAL;
    HIP_TRY(ctx, hipMemcpyAsync(d, ctx->diag, ctx->n * ctx->esz, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return LOBPCG_OK;
}
