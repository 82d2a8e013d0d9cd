// Training-sample harvest for the learned preconditioner.
//
// For a block X with H X, Ritz values theta and converged eigenvectors x* of
// the same matrix, each column j < nev yields one group of samples:
//   E_j = x*_j - X (X^T x*_j)          the exact correction outside span(X)
//   R_ij = (H X)_ij - theta_j X_ij     the residual, U_ij = R_ij / s(d_i - sigma_j)
//   (sigma_j the context's diagonal-preconditioner shift, theta_j by default)
// Row i enters the group with probability
//   p_i = min(1, rows (1/(2n) + |E_ij| / (2 sum_l |E_lj|)))
// (half uniform, half proportional to |E|), decided by a uniform draw from
// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) keyed by (seed, group, i):
//   u = (sm(sm(seed XOR sm(group)) + i) >> 11) * 2^-53, where sm(x) is one
//   SplitMix64 output for state x (state += 0x9E3779B97F4A7C15, then mix).
// A kept row is stored with weight 1/p_i, so weighted sums over a group are
// unbiased estimates of the full-column sums.
#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace {

constexpr int HV_THREADS = 256;

__device__ inline uint64_t sm64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__device__ inline double uniform01(uint64_t seed, uint64_t group, uint64_t i) {
    const uint64_t h = sm64(seed ^ sm64(group));
    return (double)(sm64(h + i) >> 11) * 0x1.0p-53;
}

template <typename T>
__device__ inline double correction(int64_t i, int j, int k, int nev, const T *__restrict__ X,
                                    const T *__restrict__ xs, const double *__restrict__ C) {
    double e = (double)xs[i * nev + j];
    for (int l = 0; l < k; ++l) e -= (double)X[i * k + l] * C[l * nev + j];
    return e;
}

// per-workgroup partial sums of |E_ij| for every j < nev
template <typename T>
__global__ __launch_bounds__(HV_THREADS) void abs_sum_kernel(int64_t n, int k, int nev, const T *__restrict__ X,
                                                             const T *__restrict__ xs, const double *__restrict__ C,
                                                             double *__restrict__ partial) {
    __shared__ double red[HV_THREADS / LOBPCG_WAVE][16];
    double acc[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * HV_THREADS + threadIdx.x; i < n; i += (int64_t)gridDim.x * HV_THREADS)
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (j < nev) acc[j] += fabs(correction(i, j, k, nev, X, xs, C));
    const int lane = threadIdx.x % LOBPCG_WAVE, wave = threadIdx.x / LOBPCG_WAVE;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        double v = acc[j];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave][j] = v;
    }
    __syncthreads();
    if (threadIdx.x < nev) {
        double v = 0.0;
        for (int w = 0; w < HV_THREADS / LOBPCG_WAVE; ++w) v += red[w][threadIdx.x];
        partial[(size_t)blockIdx.x * 16 + threadIdx.x] = v;
    }
}

__global__ void abs_total_kernel(int nparts, int nev, const double *__restrict__ partial, double *__restrict__ sums) {
    const int j = threadIdx.x;
    if (j >= nev) return;
    double v = 0.0;
    for (int q = 0; q < nparts; ++q) v += partial[(size_t)q * 16 + j];
    sums[j] = v;
}

__global__ void set_counter_kernel(unsigned long long *counter, int64_t v, int64_t *group_off, int g) {
    *counter = (unsigned long long)v;
    group_off[g] = v;
}

__global__ void close_group_kernel(const unsigned long long *counter, int64_t *group_off, int g) {
    group_off[g + 1] = (int64_t)*counter;
}

// One thread per row; kept rows are compacted per wavefront (ballot) and
// appended after one atomic add on the group counter.  Nothing is written at
// or beyond `capacity`.
template <typename T>
__global__ __launch_bounds__(HV_THREADS) void select_kernel(
    int64_t n, int k, int nev, int j, const T *__restrict__ X, const T *__restrict__ HX, const T *__restrict__ xs,
    const double *__restrict__ C, const double *__restrict__ sums, const double *__restrict__ theta,
    const T *__restrict__ d, const float *__restrict__ rho, const float *__restrict__ tmean, double eps, double off,
    int rows,
    uint64_t seed, uint64_t group, int64_t capacity, float *__restrict__ feat, float *__restrict__ U,
    float *__restrict__ Tt, float *__restrict__ w, float *__restrict__ Xrow, int32_t *__restrict__ rowid,
    unsigned long long *__restrict__ counter) {
    const int64_t i = (int64_t)blockIdx.x * HV_THREADS + threadIdx.x;
    const int lane = threadIdx.x % LOBPCG_WAVE;
    bool keep = false;
    double e = 0.0, p = 1.0;
    if (i < n) {
        e = correction(i, j, k, nev, X, xs, C);
        const double tot = sums[j];
        const double share = tot > 0.0 ? fabs(e) / tot : 1.0 / (double)n;
        p = fmin(1.0, (double)rows * (0.5 / (double)n + 0.5 * share));
        keep = uniform01(seed, group, (uint64_t)i) < p;
    }
    const uint64_t ball = __ballot(keep);
    const int cnt = __popcll(ball);
    if (cnt == 0) return;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(counter, (unsigned long long)cnt);
    const uint32_t lo = __shfl((uint32_t)(base & 0xffffffffull), 0), hi = __shfl((uint32_t)(base >> 32), 0);
    base = ((unsigned long long)hi << 32) | lo;
    if (!keep) return;
    const int rank = __popcll(ball & ((1ull << lane) - 1ull));
    const int64_t pos = (int64_t)base + rank;
    if (pos >= capacity) return;
    const double th = theta[j];
    const double di = (double)d[i];
    const double dm = di - th + off * ritz_spread(theta, k);
    const double sg = fabs(dm) >= eps ? dm : (dm < 0 ? -eps : eps);
    const double r = (double)HX[i * k + j] - (double)X[i * k + j] * th;
    feat[pos * 4 + 0] = (float)di;
    feat[pos * 4 + 1] = (float)th;
    feat[pos * 4 + 2] = rho[i];
    feat[pos * 4 + 3] = tmean[i];
    U[pos] = (float)(r / sg);
    Tt[pos] = (float)e;
    w[pos] = (float)(1.0 / p);
    for (int l = 0; l < k; ++l) Xrow[pos * k + l] = (float)X[i * k + l];
    if (rowid) rowid[pos] = (int32_t)i;
}

template <typename T>
int snapshot(lobpcg_ctx *ctx, const void *Xv, const void *HXv, const double *theta, int k, lobpcg_harvest *h,
             hipStream_t s) {
    const int nev = h->nev;
    const T *X = (const T *)Xv, *HX = (const T *)HXv, *xs = (const T *)h->xstar;
    // C = X^T x*  (k x nev, FP64)
    GramArgs g{};
    g.a[0] = X;
    g.b[0] = xs;
    g.na = g.nb = 1;
    g.wa = k;
    g.wb = nev;
    int rc = launch_gram(ctx, g, LOBPCG_GRAM_F64, ctx->gram_out2, s);
    if (rc != LOBPCG_OK) return rc;
    const int nparts = std::min(ceil_div(ctx->n, HV_THREADS), ctx->norm_max_wg);
    double *sums = ctx->gram_out;  // free between Rayleigh-Ritz steps
    abs_sum_kernel<T><<<nparts, HV_THREADS, 0, s>>>(ctx->n, k, nev, X, xs, ctx->gram_out2, ctx->norm_partial);
    abs_total_kernel<<<1, 64, 0, s>>>(nparts, nev, ctx->norm_partial, sums);
    set_counter_kernel<<<1, 1, 0, s>>>(ctx->harvest_counter, h->nsamples, h->group_off, h->ngroups);
    const double eps = ctx->eps_rel * ctx->gamma;
    for (int j = 0; j < nev; ++j) {
        const int gidx = h->ngroups + j;
        select_kernel<T><<<ceil_div(ctx->n, HV_THREADS), HV_THREADS, 0, s>>>(
            ctx->n, k, nev, j, X, HX, xs, ctx->gram_out2, sums, theta, (const T *)ctx->diag, ctx->feat_rownorm,
            ctx->feat_tilemean, eps, ctx->precond_offset, h->rows, h->seed, (uint64_t)gidx, h->capacity, h->feat, h->U, h->T, h->w,
            h->Xrow, h->row, ctx->harvest_counter);
        close_group_kernel<<<1, 1, 0, s>>>(ctx->harvest_counter, h->group_off, gidx);
    }
    HIP_TRY(ctx, hipGetLastError());
    std::vector<int64_t> offs(nev + 1);
    HIP_TRY(ctx, hipMemcpyAsync(offs.data(), h->group_off + h->ngroups, (nev + 1) * sizeof(int64_t),
                                hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    int complete = 0;
    while (complete < nev && offs[complete + 1] <= h->capacity) ++complete;
    h->ngroups += complete;
    h->nsamples = offs[complete];
    if (complete < nev) h->full = 1;
    return LOBPCG_OK;
}

}  // namespace

int harvest_snapshot(lobpcg_ctx *ctx, int k, lobpcg_harvest *h, hipStream_t s) {
    return lobpcg_harvest_block(ctx, ctx->X, ctx->HX, ctx->rr_theta, k, h, s);
}

extern "C" int lobpcg_harvest_block(lobpcg_ctx *ctx, const void *X, const void *HX, const double *theta, int k,
                                    lobpcg_harvest *h, void *stream) {
    if (!ctx) return LOBPCG_EINVAL;
    if (!h || !X || !HX || !theta) return set_err(ctx, LOBPCG_EINVAL, "harvest: null pointer");
    if (k < 1 || k > ctx->kmax) return set_err(ctx, LOBPCG_EINVAL, "harvest: k=%d outside [1,%d]", k, ctx->kmax);
    if (h->nev < 1 || h->nev > k || h->rows < 1 || h->every < 1)
        return set_err(ctx, LOBPCG_EINVAL, "harvest: need 1 <= nev <= k, rows >= 1, every >= 1");
    if (!h->xstar || !h->feat || !h->U || !h->T || !h->w || !h->Xrow || !h->group_off)
        return set_err(ctx, LOBPCG_EINVAL, "harvest: null array");
    if (h->capacity < 0 || h->capacity_groups < 0 || h->nsamples < 0 || h->ngroups < 0 ||
        h->nsamples > h->capacity || h->ngroups > h->capacity_groups)
        return set_err(ctx, LOBPCG_EINVAL, "harvest: inconsistent counts");
    if (h->full) return LOBPCG_OK;
    if (h->ngroups + h->nev > h->capacity_groups || h->nsamples >= h->capacity) {
        h->full = 1;
        return LOBPCG_OK;
    }
    if (!ctx->harvest_counter)
        HIP_TRY(ctx, hipMalloc((void **)&ctx->harvest_counter, sizeof(unsigned long long)));
    hipStream_t s = (hipStream_t)stream;
    return ctx->dtype == LOBPCG_F32 ? snapshot<float>(ctx, X, HX, theta, k, h, s)
                                    : snapshot<double>(ctx, X, HX, theta, k, h, s);
}
