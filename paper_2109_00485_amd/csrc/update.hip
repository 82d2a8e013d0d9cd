// Row-parallel block kernels: the fused LOBPCG update (eqs. xupd, pupd and the
// recurrences eqs. upd1-upd2), the residual R = H X - X Theta with its column
// norms (Algorithm 1 line 10), the diagonal preconditioner (line 6), and the
// generic "out = sum_b in_b M_b" combination used by Cholesky QR.
//
// One thread owns one row of every block (row-major n x k, so a wavefront
// touches 64 consecutive rows: contiguous, coalesced traffic).  The small
// coefficient matrices are staged once per workgroup in LDS.
#include "internal.hpp"


namespace {

constexpr int UPD_THREADS = 256;
constexpr int KM = 16;

template <typename T>
__device__ inline T guard_div(T r, double dm, double eps) {
    // s(x) = x if |x| >= eps else sign+(x) eps
    double s = fabs(dm) >= eps ? dm : (dm < 0 ? -eps : eps);
    return (T)((double)r / s);
}

// Block reduction of 2*k per-thread FP64 sums into one partial per workgroup
// (fully unrolled so the per-thread sums stay in registers).
__device__ inline void block_reduce_store(const double (&vals)[2][KM], int k, double *__restrict__ out) {
    __shared__ double red[UPD_THREADS / LOBPCG_WAVE][2][KM];
    const int lane = threadIdx.x % LOBPCG_WAVE, wave = threadIdx.x / LOBPCG_WAVE;
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int q = 0; q < KM; ++q) {
            if (q < k) {
                double v = vals[s][q];
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
                if (lane == 0) red[wave][s][q] = v;
            }
        }
    __syncthreads();
    if (threadIdx.x < 2 * k) {
        int s = threadIdx.x / k, q = threadIdx.x % k;
        double acc = 0.0;
        for (int w = 0; w < UPD_THREADS / LOBPCG_WAVE; ++w) acc += red[w][s][q];
        out[(size_t)blockIdx.x * 3 * KM + s * KM + q] = acc;
    }
}

// mode: nblk in {1,2,3} = combine with C from Rayleigh-Ritz; 0 = no combine
// (X, HX used as they are, theta given).  nblk is read from flags[1] when
// nblk_dev != 0 (the Rayleigh-Ritz kernel may have dropped P).
template <typename T>
__global__ __launch_bounds__(UPD_THREADS) void update_kernel(
    int64_t n, int k, int nblk_host, int nblk_dev, const double *__restrict__ Cg, const double *__restrict__ theta_g,
    T *__restrict__ X, T *__restrict__ W, T *__restrict__ P, T *__restrict__ HX, T *__restrict__ HW,
    T *__restrict__ HP, const T *__restrict__ d, int precond, double eps, int write_w,
    double *__restrict__ partial, const int *__restrict__ flags) {
    if (flags[0] & (FLAG_CHOLQR_FAIL | FLAG_RR_FAIL)) return;
    const int nblk = nblk_dev ? flags[1] : nblk_host;
    __shared__ T Cs[3 * KM * KM];
    __shared__ double th[KM];
    const int N = nblk * k;
    for (int e = threadIdx.x; e < N * k; e += UPD_THREADS) Cs[e] = (T)Cg[e];
    if (threadIdx.x < k) th[threadIdx.x] = theta_g[threadIdx.x];
    __syncthreads();
    double sums[2][KM];
#pragma unroll
    for (int q = 0; q < KM; ++q) sums[0][q] = sums[1][q] = 0.0;

    for (int64_t i = (int64_t)blockIdx.x * UPD_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * UPD_THREADS) {
        T xn[KM], hn[KM], pn[KM], hpn[KM];
        const int64_t o = i * k;
        if (nblk == 0) {
#pragma unroll
            for (int q = 0; q < KM; ++q)
                if (q < k) { xn[q] = X[o + q]; hn[q] = HX[o + q]; }
        } else {
#pragma unroll
            for (int q = 0; q < KM; ++q) xn[q] = hn[q] = pn[q] = hpn[q] = T(0);
            // X and HX block rows
#pragma unroll
            for (int m = 0; m < KM; ++m) {
                if (m < k) {
                    T xv = X[o + m], hv = HX[o + m];
#pragma unroll
                    for (int q = 0; q < KM; ++q)
                        if (q < k) { xn[q] += xv * Cs[m * k + q]; hn[q] += hv * Cs[m * k + q]; }
                }
            }
            if (nblk >= 2) {
#pragma unroll
                for (int m = 0; m < KM; ++m) {
                    if (m < k) {
                        T wv = W[o + m], hv = HW[o + m];
#pragma unroll
                        for (int q = 0; q < KM; ++q)
                            if (q < k) { T c = Cs[(k + m) * k + q]; pn[q] += wv * c; hpn[q] += hv * c; }
                    }
                }
            }
            if (nblk >= 3) {
#pragma unroll
                for (int m = 0; m < KM; ++m) {
                    if (m < k) {
                        T pv = P[o + m], hv = HP[o + m];
#pragma unroll
                        for (int q = 0; q < KM; ++q)
                            if (q < k) { T c = Cs[(2 * k + m) * k + q]; pn[q] += pv * c; hpn[q] += hv * c; }
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < KM; ++q)
                if (q < k) { xn[q] += pn[q]; hn[q] += hpn[q]; }
        }
        const double di = precond == LOBPCG_PRECOND_DIAG ? (double)d[i] : 0.0;
        T wv[KM];
#pragma unroll
        for (int q = 0; q < KM; ++q) {
            if (q < k) {
                T r = hn[q] - xn[q] * (T)th[q];
                sums[0][q] += (double)r * (double)r;
                sums[1][q] += (double)xn[q] * (double)xn[q];
                wv[q] = precond == LOBPCG_PRECOND_DIAG ? guard_div<T>(r, di - th[q], eps) : r;
            }
        }
#pragma unroll
        for (int q = 0; q < KM; ++q) {
            if (q < k) {
                if (nblk != 0) {
                    X[o + q] = xn[q];
                    HX[o + q] = hn[q];
                    if (nblk >= 2) { P[o + q] = pn[q]; HP[o + q] = hpn[q]; }
                }
                if (write_w) W[o + q] = wv[q];
            }
        }
    }
    block_reduce_store(sums, k, partial);
}

// report = {theta, sum r^2, sum x^2, flags, nblk}
__global__ void finalize_kernel(int k, int nparts, const double *__restrict__ partial,
                                const double *__restrict__ theta, const int *__restrict__ flags,
                                Report *__restrict__ rep) {
    const int t = threadIdx.x;
    if (t < 2 * k) {
        int s = t / k, q = t % k;
        double acc = 0.0;
        for (int p = 0; p < nparts; ++p) acc += partial[(size_t)p * 3 * KM + s * KM + q];
        if (s == 0) rep->rnorm2[q] = acc; else rep->xnorm2[q] = acc;
    }
    if (t < k) rep->theta[t] = theta[t];
    if (t == 0) {
        rep->flags = (double)flags[0];
        rep->nblk_used = (double)flags[1];
    }
}

// out_i = sum_b coef_b * in_b,i * M_b   (M_b = identity when null), in place allowed
template <typename T>
__global__ __launch_bounds__(UPD_THREADS) void combine_kernel(int64_t n, int k, int nin, const T *in0, const T *in1,
                                                              const T *in2, const double *m0, const double *m1,
                                                              const double *m2, double c0, double c1, double c2,
                                                              T *out, const int *__restrict__ flags) {
    if (flags && (flags[0] & (FLAG_CHOLQR_FAIL | FLAG_RR_FAIL))) return;
    __shared__ T Ms[3][KM * KM];
    const T *ins[3] = {in0, in1, in2};
    const double *ms[3] = {m0, m1, m2};
    const double cs[3] = {c0, c1, c2};
    for (int b = 0; b < nin; ++b)
        for (int e = threadIdx.x; e < k * k; e += UPD_THREADS)
            Ms[b][e] = (T)(cs[b] * (ms[b] ? ms[b][e] : ((e / k) == (e % k) ? 1.0 : 0.0)));
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * UPD_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * UPD_THREADS) {
        T acc[KM];
#pragma unroll
        for (int q = 0; q < KM; ++q) acc[q] = T(0);
        for (int b = 0; b < nin; ++b) {
            const T *src = ins[b] + i * k;
#pragma unroll
            for (int m = 0; m < KM; ++m) {
                if (m < k) {
                    T v = src[m];
#pragma unroll
                    for (int q = 0; q < KM; ++q)
                        if (q < k) acc[q] += v * Ms[b][m * k + q];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < KM; ++q)
            if (q < k) out[i * k + q] = acc[q];
    }
}

template <typename T>
__global__ __launch_bounds__(UPD_THREADS) void precond_kernel(int64_t n, int k, const T *__restrict__ R,
                                                              const double *__restrict__ theta,
                                                              const T *__restrict__ d, T *__restrict__ W,
                                                              int kind, double eps) {
    __shared__ double th[KM];
    if (threadIdx.x < k) th[threadIdx.x] = theta[threadIdx.x];
    __syncthreads();
    const int64_t total = n * k;
    for (int64_t e = (int64_t)blockIdx.x * UPD_THREADS + threadIdx.x; e < total; e += (int64_t)gridDim.x * UPD_THREADS) {
        const int64_t i = e / k;
        const int q = (int)(e - i * k);
        T r = R[e];
        W[e] = kind == LOBPCG_PRECOND_DIAG ? guard_div<T>(r, (double)d[i] - th[q], eps) : r;
    }
}

__global__ void set_flags_kernel(int *flags, int f0, int f1) {
    if (threadIdx.x == 0) { flags[0] = f0; flags[1] = f1; }
}

int grid_rows(int64_t n, int cap) { return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (n + UPD_THREADS - 1) / UPD_THREADS)); }

}  // namespace

int launch_set_flags(lobpcg_ctx *ctx, int f0, int f1, hipStream_t s) {
    set_flags_kernel<<<1, 64, 0, s>>>(ctx->dflags, f0, f1);
    return LOBPCG_OK;
}

// write_w: store the preconditioned residual into W.  nblk = 0 means "no
// combination" (theta given in ctx->rr_theta); nblk > 0 reads the block count
// chosen by the Rayleigh-Ritz kernel from the device flags.
int launch_update(lobpcg_ctx *ctx, int k, int nblk, int precond, int write_w, hipStream_t s) {
    const int grid = grid_rows(ctx->n, ctx->norm_max_wg);
    const double eps = ctx->eps_rel * ctx->gamma;
    const int pk = precond == LOBPCG_PRECOND_DIAG ? LOBPCG_PRECOND_DIAG : LOBPCG_PRECOND_NONE;
    if (ctx->dtype == LOBPCG_F32)
        update_kernel<float><<<grid, UPD_THREADS, 0, s>>>(ctx->n, k, nblk, nblk > 0, ctx->rr_C, ctx->rr_theta,
            (float *)ctx->X, (float *)ctx->W, (float *)ctx->P, (float *)ctx->HX, (float *)ctx->HW, (float *)ctx->HP,
            (const float *)ctx->diag, pk, eps, write_w, ctx->norm_partial, ctx->dflags);
    else
        update_kernel<double><<<grid, UPD_THREADS, 0, s>>>(ctx->n, k, nblk, nblk > 0, ctx->rr_C, ctx->rr_theta,
            (double *)ctx->X, (double *)ctx->W, (double *)ctx->P, (double *)ctx->HX, (double *)ctx->HW,
            (double *)ctx->HP, (const double *)ctx->diag, pk, eps, write_w, ctx->norm_partial, ctx->dflags);
    finalize_kernel<<<1, 64, 0, s>>>(k, grid, ctx->norm_partial, ctx->rr_theta, ctx->dflags, ctx->report_dev);
    return LOBPCG_OK;
}

int launch_combine(lobpcg_ctx *ctx, int k, int nin, const void *const *in, const double *const *mats,
                   const double *coef, void *out, hipStream_t s) {
    const int grid = grid_rows(ctx->n, 4096);
    const void *i0 = in[0], *i1 = nin > 1 ? in[1] : nullptr, *i2 = nin > 2 ? in[2] : nullptr;
    const double *m0 = mats[0], *m1 = nin > 1 ? mats[1] : nullptr, *m2 = nin > 2 ? mats[2] : nullptr;
    double c0 = coef[0], c1 = nin > 1 ? coef[1] : 0.0, c2 = nin > 2 ? coef[2] : 0.0;
    if (ctx->dtype == LOBPCG_F32)
        combine_kernel<float><<<grid, UPD_THREADS, 0, s>>>(ctx->n, k, nin, (const float *)i0, (const float *)i1,
            (const float *)i2, m0, m1, m2, c0, c1, c2, (float *)out, ctx->dflags);
    else
        combine_kernel<double><<<grid, UPD_THREADS, 0, s>>>(ctx->n, k, nin, (const double *)i0, (const double *)i1,
            (const double *)i2, m0, m1, m2, c0, c1, c2, (double *)out, ctx->dflags);
    return LOBPCG_OK;
}

int launch_precond(lobpcg_ctx *ctx, const void *R, const double *theta, void *W, int k, int kind, hipStream_t s) {
    const int grid = grid_rows(ctx->n * k, 8192);
    const double eps = ctx->eps_rel * ctx->gamma;
    if (ctx->dtype == LOBPCG_F32)
        precond_kernel<float><<<grid, UPD_THREADS, 0, s>>>(ctx->n, k, (const float *)R, theta,
                                                           (const float *)ctx->diag, (float *)W, kind, eps);
    else
        precond_kernel<double><<<grid, UPD_THREADS, 0, s>>>(ctx->n, k, (const double *)R, theta,
                                                            (const double *)ctx->diag, (double *)W, kind, eps);
    return LOBPCG_OK;
}

extern "C" int lobpcg_precond_apply(lobpcg_ctx *ctx, const void *R, const double *theta, void *W, int k, int kind,
                                    void *stream) {
    if (!ctx) return LOBPCG_EINVAL;
    if (!R || !theta || !W) return set_err(ctx, LOBPCG_EINVAL, "precond_apply: null pointer");
    if (k < 1 || k > ctx->kmax) return set_err(ctx, LOBPCG_EINVAL, "precond_apply: k=%d outside [1,%d]", k, ctx->kmax);
    if (kind != LOBPCG_PRECOND_NONE && kind != LOBPCG_PRECOND_DIAG && kind != LOBPCG_PRECOND_MLP)
        return set_err(ctx, LOBPCG_EINVAL, "precond_apply: bad kind %d", kind);
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if (kind == LOBPCG_PRECOND_MLP) {
        rc = mlp_precond_ready(ctx);
        if (rc != LOBPCG_OK) return rc;
        rc = launch_mlp_precond(ctx, R, theta, W, k, s);
    } else {
        rc = launch_precond(ctx, R, theta, W, k, kind, s);
    }
    if (rc != LOBPCG_OK) return rc;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_err(ctx, LOBPCG_EHIP, "precond_apply launch: %s", hipGetErrorString(e));
    return LOBPCG_OK;
}
