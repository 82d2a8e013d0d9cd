// Row-parallel block kernels: the fused LOBPCG update (eqs. xupd, pupd and the
// recurrences eqs. upd1-upd2), the residual R = H X - X Theta with its column
// norms (the residual step of Algorithm 1), the diagonal preconditioner, and the
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

// Layout of the update: a row's k outputs are split over TPR threads of QG
// consecutive columns each (k = 8: 2 threads x 4, k = 16: 4 x 4; other k: one
// thread per column).  Every thread reads the whole input rows it combines
// (16-byte loads when k is fixed at compile time) and writes its QG columns.
template <typename T, int KP>
struct UpdShape {
    static constexpr int QG = KP ? 4 : 1;
};

template <typename T, int KP>
__device__ inline void load_row(const T *__restrict__ p, int k, T (&v)[KM]) {
    if constexpr (KP > 0 && (KP * sizeof(T)) % 16 == 0) {
        using V4 = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
        constexpr int PER = 16 / sizeof(T);
        const V4 *q = reinterpret_cast<const V4 *>(p);
#pragma unroll
        for (int c = 0; c < KP / PER; ++c) {
            V4 x = q[c];
            const T *xs = reinterpret_cast<const T *>(&x);
#pragma unroll
            for (int e = 0; e < PER; ++e) v[c * PER + e] = xs[e];
        }
    } else {
#pragma unroll
        for (int q = 0; q < KM; ++q)
            if (q < k) v[q] = p[q];
    }
}

// acc[c] += sum_m row[m] * Cb[m * k + q0 + c],  c < QG
template <typename T, int KP, int QG>
__device__ inline void mac_cols(T (&acc)[QG], const T (&row)[KM], const T *__restrict__ Cb, int k, int q0) {
#pragma unroll
    for (int m = 0; m < KM; ++m) {
        if (m < (KP ? KP : k)) {
#pragma unroll
            for (int c = 0; c < QG; ++c) acc[c] += row[m] * Cb[m * (KP ? KP : k) + q0 + c];
        }
    }
}

// mode: nblk in {1,2,3} = combine with C from Rayleigh-Ritz; 0 = no combine
// (X, HX used as they are, theta given).  nblk is read from flags[1] when
// nblk_dev != 0 (the Rayleigh-Ritz kernel may have dropped P).  The combined
// rows are written only after every thread of the row has read them, which
// the row's threads guarantee by reading before writing within one
// wavefront (TPR divides the wavefront).
template <typename T, int KP>
__global__ __launch_bounds__(UPD_THREADS) void update_kernel(
    int64_t n, int k_rt, int nblk_host, int nblk_dev, const double *__restrict__ Cg, const double *__restrict__ theta_g,
    T *X, T *W, T *P, T *HX, T *HW, T *HP, const T *__restrict__ d, int precond, double eps, double off, int write_w,
    double *__restrict__ partial, const int *__restrict__ flags) {
    constexpr int QG = UpdShape<T, KP>::QG;
    if (flags[0] & (FLAG_CHOLQR_FAIL | FLAG_RR_FAIL)) return;
    const int k = KP ? KP : k_rt;
    const int nblk = nblk_dev ? flags[1] : nblk_host;
    __shared__ T Cs[3 * KM * KM];
    __shared__ double th[KM];
    __shared__ double red[UPD_THREADS][2][4];
    const int N = nblk * k;
    for (int e = threadIdx.x; e < N * k; e += UPD_THREADS) Cs[e] = (T)Cg[e];
    if (threadIdx.x < k) th[threadIdx.x] = theta_g[threadIdx.x];
    __syncthreads();
    // a row's threads never straddle two wavefronts
    const int tpr = KP ? KP / QG : k;            // threads per row
    const int rpw = LOBPCG_WAVE / tpr;           // rows per wavefront
    const int rpi = rpw * (UPD_THREADS / LOBPCG_WAVE);  // rows per workgroup step
    const int lane = threadIdx.x % LOBPCG_WAVE;
    const int rr = (threadIdx.x / LOBPCG_WAVE) * rpw + lane / tpr, g = lane % tpr;
    const int q0 = g * QG;
    const bool active = lane / tpr < rpw;
    double s_r[QG], s_x[QG];
#pragma unroll
    for (int c = 0; c < QG; ++c) s_r[c] = s_x[c] = 0.0;
    T thq[QG];
#pragma unroll
    for (int c = 0; c < QG; ++c) thq[c] = (T)th[q0 + c];
    const double lift = off * ritz_spread(th, k);   // theta_j - sigma_j
    for (int64_t i0 = (int64_t)blockIdx.x * rpi; i0 < n; i0 += (int64_t)gridDim.x * rpi) {
        const int64_t i = i0 + rr;
        if (!active || i >= n) continue;
        const int64_t o = i * k;
        T xn[QG], hn[QG], pn[QG], hpn[QG];
        if (nblk == 0) {
#pragma unroll
            for (int c = 0; c < QG; ++c) { xn[c] = X[o + q0 + c]; hn[c] = HX[o + q0 + c]; }
        } else {
            T r0[KM], r1[KM];
#pragma unroll
            for (int c = 0; c < QG; ++c) xn[c] = hn[c] = pn[c] = hpn[c] = T(0);
            load_row<T, KP>(X + o, k, r0);
            load_row<T, KP>(HX + o, k, r1);
            mac_cols<T, KP, QG>(xn, r0, Cs, k, q0);
            mac_cols<T, KP, QG>(hn, r1, Cs, k, q0);
            if (nblk >= 2) {
                load_row<T, KP>(W + o, k, r0);
                load_row<T, KP>(HW + o, k, r1);
                mac_cols<T, KP, QG>(pn, r0, Cs + k * k, k, q0);
                mac_cols<T, KP, QG>(hpn, r1, Cs + k * k, k, q0);
            }
            if (nblk >= 3) {
                load_row<T, KP>(P + o, k, r0);
                load_row<T, KP>(HP + o, k, r1);
                mac_cols<T, KP, QG>(pn, r0, Cs + 2 * k * k, k, q0);
                mac_cols<T, KP, QG>(hpn, r1, Cs + 2 * k * k, k, q0);
            }
#pragma unroll
            for (int c = 0; c < QG; ++c) { xn[c] += pn[c]; hn[c] += hpn[c]; }
        }
        const double di = precond == LOBPCG_PRECOND_DIAG ? (double)d[i] : 0.0;
        T wv[QG];
#pragma unroll
        for (int c = 0; c < QG; ++c) {
            T r = hn[c] - xn[c] * thq[c];
            s_r[c] += (double)r * (double)r;
            s_x[c] += (double)xn[c] * (double)xn[c];
            wv[c] = precond == LOBPCG_PRECOND_DIAG ? guard_div<T>(r, di - th[q0 + c] + lift, eps) : r;
        }
        // all threads of this row (same wavefront) have read their inputs
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int c = 0; c < QG; ++c) {
            if (nblk != 0) {
                X[o + q0 + c] = xn[c];
                HX[o + q0 + c] = hn[c];
                if (nblk >= 2) { P[o + q0 + c] = pn[c]; HP[o + q0 + c] = hpn[c]; }
            }
            if (write_w) W[o + q0 + c] = wv[c];
        }
    }
#pragma unroll
    for (int c = 0; c < QG; ++c) {
        red[threadIdx.x][0][c] = active ? s_r[c] : 0.0;
        red[threadIdx.x][1][c] = active ? s_x[c] : 0.0;
    }
    __syncthreads();
    if (threadIdx.x < 2 * k) {
        const int sidx = threadIdx.x / k, q = threadIdx.x % k;
        const int gq = q / QG, c = q % QG;
        double acc = 0.0;
        for (int t = 0; t < UPD_THREADS; ++t) {
            const int l = t % LOBPCG_WAVE;
            if (l % tpr == gq && l / tpr < rpw) acc += red[t][sidx][c];
        }
        partial[(size_t)blockIdx.x * 3 * KM + sidx * KM + q] = acc;
    }
}

// report = {theta, sum r^2, sum x^2, flags, nblk}: the per-workgroup sums
// reduced in a fixed order.  Lane q of a row group reads value q of every
// FIN_ROWS-th partial row (a wavefront reads two whole rows, coalesced), with
// eight independent accumulators so that each thread keeps eight loads in
// flight (the partials were just written by other XCDs: every load is a
// memory round trip); the row groups are then summed in LDS.
constexpr int FIN_THREADS = 1024;
constexpr int FIN_ROWS = FIN_THREADS / (2 * KM);
__global__ __launch_bounds__(FIN_THREADS) void finalize_kernel(int k, int nparts, const double *__restrict__ partial,
                                                               const double *__restrict__ theta,
                                                               const int *__restrict__ flags,
                                                               Report *__restrict__ rep) {
    __shared__ double red[FIN_ROWS][2 * KM];
    const int t = threadIdx.x, q0 = t % (2 * KM), g = t / (2 * KM);
    double a[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = 0.0;
    int p = g;
    for (; p + 7 * FIN_ROWS < nparts; p += 8 * FIN_ROWS) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] += partial[(size_t)(p + u * FIN_ROWS) * 3 * KM + q0];
    }
    for (; p < nparts; p += FIN_ROWS) a[0] += partial[(size_t)p * 3 * KM + q0];
    red[g][q0] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    __syncthreads();
    if (t < 2 * KM) {
        double v = 0.0;
        for (int w = 0; w < FIN_ROWS; ++w) v += red[w][t];
        const int s = t / KM, q = t % KM;
        if (q < k) {
            if (s == 0) rep->rnorm2[q] = v; else rep->xnorm2[q] = v;
        }
    }
    if (t < k) rep->theta[t] = theta[t];
    if (t == 0) {
        rep->flags = (double)flags[0];
        rep->nblk_used = (double)flags[1];
    }
}

// out_i = sum_b coef_b * in_b,i * M_b   (M_b = identity when null), in place
// allowed (out may alias an input: a row's threads share one wavefront and
// read the whole row before any of them writes).  Same thread layout as the
// update kernel.
template <typename T, int KP>
__global__ __launch_bounds__(UPD_THREADS) void combine_kernel(int64_t n, int k_rt, int nin, const T *in0, const T *in1,
                                                              const T *in2, const double *m0, const double *m1,
                                                              const double *m2, double c0, double c1, double c2,
                                                              T *out, const int *__restrict__ flags) {
    constexpr int QG = UpdShape<T, KP>::QG;
    if (flags && (flags[0] & (FLAG_CHOLQR_FAIL | FLAG_RR_FAIL))) return;
    const int k = KP ? KP : k_rt;
    __shared__ T Ms[3][KM * KM];
    const T *ins[3] = {in0, in1, in2};
    const double *ms[3] = {m0, m1, m2};
    const double cs[3] = {c0, c1, c2};
    for (int b = 0; b < nin; ++b)
        for (int e = threadIdx.x; e < k * k; e += UPD_THREADS)
            Ms[b][e] = (T)(cs[b] * (ms[b] ? ms[b][e] : ((e / k) == (e % k) ? 1.0 : 0.0)));
    __syncthreads();
    const int tpr = KP ? KP / QG : k;
    const int rpw = LOBPCG_WAVE / tpr;
    const int rpi = rpw * (UPD_THREADS / LOBPCG_WAVE);
    const int lane = threadIdx.x % LOBPCG_WAVE;
    const int rr = (threadIdx.x / LOBPCG_WAVE) * rpw + lane / tpr, g = lane % tpr;
    const int q0 = g * QG;
    const bool active = lane / tpr < rpw;
    for (int64_t i0 = (int64_t)blockIdx.x * rpi; i0 < n; i0 += (int64_t)gridDim.x * rpi) {
        const int64_t i = i0 + rr;
        if (!active || i >= n) continue;
        T acc[QG];
#pragma unroll
        for (int c = 0; c < QG; ++c) acc[c] = T(0);
        for (int b = 0; b < nin; ++b) {
            T row[KM];
            load_row<T, KP>(ins[b] + i * k, k, row);
            mac_cols<T, KP, QG>(acc, row, Ms[b], k, q0);
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int c = 0; c < QG; ++c) out[i * k + q0 + c] = acc[c];
    }
}

template <typename T>
__global__ __launch_bounds__(UPD_THREADS) void precond_kernel(int64_t n, int k, const T *__restrict__ R,
                                                              const double *__restrict__ theta,
                                                              const T *__restrict__ d, T *__restrict__ W,
                                                              int kind, double eps, double off) {
    __shared__ double th[KM];
    if (threadIdx.x < k) th[threadIdx.x] = theta[threadIdx.x];
    __syncthreads();
    const double lift = off * ritz_spread(th, k);
    const int64_t total = n * k;
    for (int64_t e = (int64_t)blockIdx.x * UPD_THREADS + threadIdx.x; e < total; e += (int64_t)gridDim.x * UPD_THREADS) {
        const int64_t i = e / k;
        const int q = (int)(e - i * k);
        T r = R[e];
        W[e] = kind == LOBPCG_PRECOND_DIAG ? guard_div<T>(r, (double)d[i] - th[q] + lift, eps) : r;
    }
}

__global__ void set_flags_kernel(int *flags, int f0, int f1, int f2, int f3) {
    if (threadIdx.x == 0) { flags[0] = f0; flags[1] = f1; flags[2] = f2; flags[3] = f3; }
}

int grid_rows(int64_t n, int cap) { return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (n + UPD_THREADS - 1) / UPD_THREADS)); }

}  // namespace

int launch_set_flags(lobpcg_ctx *ctx, int f0, int f1, hipStream_t s, int force, int lock) {
    set_flags_kernel<<<1, 64, 0, s>>>(ctx->dflags, f0, f1, force, lock);
    return LOBPCG_OK;
}

// write_w: store the preconditioned residual into W.  nblk = 0 means "no
// combination" (theta given in ctx->rr_theta); nblk > 0 reads the block count
// chosen by the Rayleigh-Ritz kernel from the device flags.
//
// The grid is what the device holds at once (workgroups per CU at this
// kernel's register use x CUs, capped by the partial-sum buffer): every
// workgroup then strides over the rows from the start, with no second, partly
// filled batch of workgroups at the end (tiled_2m, k = 8: 200 vs 211 us per
// update and reduction with the 2048-workgroup grid).
template <typename T, int KP>
int update_grid(lobpcg_ctx *ctx) {
    // the kernel's occupancy, queried once (the same on every device of one build)
    static const int per_cu = [] {
        int b = 0;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, update_kernel<T, KP>, UPD_THREADS, 0) == hipSuccess ? b
                                                                                                               : 0;
    }();
    int cus = 0;
    if (per_cu <= 0 || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess ||
        cus <= 0)
        return grid_rows(ctx->n, ctx->norm_max_wg);
    return grid_rows(ctx->n, std::min(ctx->norm_max_wg, per_cu * cus));
}

int launch_update(lobpcg_ctx *ctx, int k, int nblk, int precond, int write_w, hipStream_t s) {
    int grid;
    if (ctx->dtype == LOBPCG_F32)
        grid = k == 8 ? update_grid<float, 8>(ctx) : k == 16 ? update_grid<float, 16>(ctx) : update_grid<float, 0>(ctx);
    else
        grid = k == 8 ? update_grid<double, 8>(ctx) : k == 16 ? update_grid<double, 16>(ctx) : update_grid<double, 0>(ctx);
    const double eps = ctx->eps_rel * ctx->gamma;
    const int pk = precond == LOBPCG_PRECOND_DIAG ? LOBPCG_PRECOND_DIAG : LOBPCG_PRECOND_NONE;
#define UPD_LAUNCH(T, KP)                                                                                        \
    update_kernel<T, KP><<<grid, UPD_THREADS, 0, s>>>(ctx->n, k, nblk, nblk > 0, ctx->rr_C, ctx->rr_theta,       \
        (T *)ctx->X, (T *)ctx->W, (T *)ctx->P, (T *)ctx->HX, (T *)ctx->HW, (T *)ctx->HP, (const T *)ctx->diag, pk, \
        eps, ctx->precond_offset, write_w, ctx->norm_partial, ctx->dflags)
    if (ctx->dtype == LOBPCG_F32) {
        if (k == 8) UPD_LAUNCH(float, 8);
        else if (k == 16) UPD_LAUNCH(float, 16);
        else UPD_LAUNCH(float, 0);
    } else {
        if (k == 8) UPD_LAUNCH(double, 8);
        else if (k == 16) UPD_LAUNCH(double, 16);
        else UPD_LAUNCH(double, 0);
    }
#undef UPD_LAUNCH
    finalize_kernel<<<1, FIN_THREADS, 0, s>>>(k, grid, ctx->norm_partial, ctx->rr_theta, ctx->dflags,
                                              ctx->report_dev);
    return LOBPCG_OK;
}

int launch_combine(lobpcg_ctx *ctx, int k, int nin, const void *const *in, const double *const *mats,
                   const double *coef, void *out, hipStream_t s) {
    const int grid = grid_rows(ctx->n, 4096);
    const void *i0 = in[0], *i1 = nin > 1 ? in[1] : nullptr, *i2 = nin > 2 ? in[2] : nullptr;
    const double *m0 = mats[0], *m1 = nin > 1 ? mats[1] : nullptr, *m2 = nin > 2 ? mats[2] : nullptr;
    double c0 = coef[0], c1 = nin > 1 ? coef[1] : 0.0, c2 = nin > 2 ? coef[2] : 0.0;
#define CMB_LAUNCH(T, KP)                                                                                   \
    combine_kernel<T, KP><<<grid, UPD_THREADS, 0, s>>>(ctx->n, k, nin, (const T *)i0, (const T *)i1,          \
                                                       (const T *)i2, m0, m1, m2, c0, c1, c2, (T *)out, ctx->dflags)
    if (ctx->dtype == LOBPCG_F32) {
        if (k == 8) CMB_LAUNCH(float, 8);
        else if (k == 16) CMB_LAUNCH(float, 16);
        else CMB_LAUNCH(float, 0);
    } else {
        if (k == 8) CMB_LAUNCH(double, 8);
        else if (k == 16) CMB_LAUNCH(double, 16);
        else CMB_LAUNCH(double, 0);
    }
#undef CMB_LAUNCH
    return LOBPCG_OK;
}

int launch_precond(lobpcg_ctx *ctx, const void *R, const double *theta, void *W, int k, int kind, hipStream_t s) {
    const int grid = grid_rows(ctx->n * k, 8192);
    const double eps = ctx->eps_rel * ctx->gamma;
    if (ctx->dtype == LOBPCG_F32)
        precond_kernel<float><<<grid, UPD_THREADS, 0, s>>>(ctx->n, k, (const float *)R, theta,
                                                           (const float *)ctx->diag, (float *)W, kind, eps,
                                                           ctx->precond_offset);
    else
        precond_kernel<double><<<grid, UPD_THREADS, 0, s>>>(ctx->n, k, (const double *)R, theta,
                                                            (const double *)ctx->diag, (double *)W, kind, eps,
                                                            ctx->precond_offset);
    return LOBPCG_OK;
}

extern "C" int lobpcg_precond_apply(lobpcg_ctx *ctx, const void *R, const double *theta, void *W, int k, int kind,
                                    void *stream) {
    if (!ctx) return LOBPCG_EINVAL;
    if (!R || !theta || !W) return set_err(ctx, LOBPCG_EINVAL, "precond_apply: null pointer");
    if (k < 1 || k > ctx->kmax) return set_err(ctx, LOBPCG_EINVAL, "precond_apply: k=%d outside [1,%d]", k, ctx->kmax);
    if (kind != LOBPCG_PRECOND_NONE && kind != LOBPCG_PRECOND_DIAG && kind != LOBPCG_PRECOND_MLP &&
        kind != LOBPCG_PRECOND_FOM)
        return set_err(ctx, LOBPCG_EINVAL, "precond_apply: bad kind %d", kind);
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if (kind == LOBPCG_PRECOND_MLP) {
        rc = mlp_precond_ready(ctx);
        if (rc != LOBPCG_OK) return rc;
        rc = launch_mlp_precond(ctx, R, theta, W, k, s);
    } else if (kind == LOBPCG_PRECOND_FOM) {
        rc = launch_fom_precond(ctx, R, theta, W, k, s);
    } else {
        rc = launch_precond(ctx, R, theta, W, k, kind, s);
    }
    if (rc != LOBPCG_OK) return rc;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_err(ctx, LOBPCG_EHIP, "precond_apply launch: %s", hipGetErrorString(e));
    return LOBPCG_OK;
}
