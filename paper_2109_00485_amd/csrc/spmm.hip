// Symmetric sparse x block-of-vectors product Y = H X from the stored upper
// triangle U.  Each stored off-diagonal h_ij (i < j) contributes h_ij X_j to
// Y_i and h_ij X_i to Y_j (Algorithm 2 applied to the stored part and to its
// transpose).
//
// As in the paper's CPU code (Section 3.2), the product with the stored part
// and the product with its transpose are separate traversals of the stored
// triangle, each written as a race-free pull over output rows:
//     Y_i = d_i X_i + sum_{j > i} u_ij X_j   (row view: CSR of U, row i)
//                   + sum_{j < i} u_ji X_j   (column view: CSC of U, column i)
// so Y is written once with plain stores: no atomics and no zero fill (on
// gfx950, coalesced atomic adds of whole 2 KB blocks ran at ~1.3 TB/s against
// ~6.5 TB/s for plain stores of the same pattern).  The column view holds the
// same entries in column order; it is built once at create.  For row i the two
// views together hold the full symmetric row, so the upper triangle's
// front-heavy rows and back-heavy columns even out.
//
// Mapping (CSR kernel): a group of 8 lanes owns one output row; the lanes take
// every 8th entry of the row's two segments, each lane gathers the full
// k-vector X_j with 16-byte loads and accumulates k partial sums in registers;
// the 8 partials are combined with lane shuffles at the end.  Matrices whose
// entries fall into dense-enough 64 x 64 tiles use the tiled format and kernel
// of spmm_tiled.hip instead.
#include <algorithm>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace {

template <typename T>
__global__ void fill_zero_kernel(T *__restrict__ p, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = T(0);
}

constexpr int GROUP = 8;          // lanes per output row
constexpr int SPMM_THREADS = 256;

template <typename T, int KP>
__device__ inline void axpy_row(T (&acc)[KP], T v, const T *__restrict__ x, int k) {
    if (k == KP) {
        if constexpr (sizeof(T) == 4) {
            const float4 *x4 = reinterpret_cast<const float4 *>(x);
#pragma unroll
            for (int q = 0; q < KP / 4; ++q) {
                float4 t = x4[q];
                acc[4 * q + 0] += v * t.x;
                acc[4 * q + 1] += v * t.y;
                acc[4 * q + 2] += v * t.z;
                acc[4 * q + 3] += v * t.w;
            }
        } else {
            const double2 *x2 = reinterpret_cast<const double2 *>(x);
#pragma unroll
            for (int q = 0; q < KP / 2; ++q) {
                double2 t = x2[q];
                acc[2 * q + 0] += v * t.x;
                acc[2 * q + 1] += v * t.y;
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < KP; ++q)
            if (q < k) acc[q] += v * x[q];
    }
}

// Each lane keeps U entries of its row in flight: the U index and value loads
// are issued together, then the U gathers of X rows, then the FMAs, so every
// lane has U independent memory chains outstanding (a single dependent chain
// per lane left the kernel latency-bound).  Padding slots load value 0 and
// gather the row's own X, so they add nothing.
#ifndef LOBPCG_SPMM_UNROLL
#define LOBPCG_SPMM_UNROLL 4
#endif
constexpr int UNROLL = LOBPCG_SPMM_UNROLL;

template <typename T, int KP>
__device__ inline void pull_segment(T (&acc)[KP], int64_t e0, int64_t e1, int sl, int64_t self,
                                    const int32_t *__restrict__ ix, const T *__restrict__ vals,
                                    const T *__restrict__ X, int k) {
    for (int64_t base = e0; base < e1; base += GROUP * UNROLL) {
        T v[UNROLL];
        int64_t j[UNROLL];
#pragma unroll
        for (int t = 0; t < UNROLL; ++t) {
            const int64_t e = base + t * GROUP + sl;
            const bool ok = e < e1;
            v[t] = ok ? vals[e] : T(0);
            j[t] = ok ? ix[e] : self;
        }
#pragma unroll
        for (int t = 0; t < UNROLL; ++t) axpy_row<T, KP>(acc, v[t], X + j[t] * k, k);
    }
}

template <typename T, int KP>
__global__ __launch_bounds__(SPMM_THREADS) void spmm_pull_kernel(
    int64_t n, int k, const int64_t *__restrict__ rp, const int32_t *__restrict__ rix, const T *__restrict__ rv,
    const int64_t *__restrict__ cp, const int32_t *__restrict__ cix, const T *__restrict__ cv,
    const T *__restrict__ diag, const T *__restrict__ X, T *__restrict__ Y) {
    constexpr int ROWS_PER_BLOCK = SPMM_THREADS / GROUP;
    const int64_t i = (int64_t)blockIdx.x * ROWS_PER_BLOCK + threadIdx.x / GROUP;
    const int sl = threadIdx.x % GROUP;
    if (i >= n) return;  // whole groups leave together; no barrier follows
    // long rows belong to spmm_heavy_kernel (the same predicate decides there)
    if ((rp[i + 1] - rp[i]) + (cp[i + 1] - cp[i]) > HEAVY_ROW) return;
    T acc[KP];
#pragma unroll
    for (int q = 0; q < KP; ++q) acc[q] = T(0);
    pull_segment<T, KP>(acc, rp[i], rp[i + 1], sl, i, rix, rv, X, k);
    pull_segment<T, KP>(acc, cp[i], cp[i + 1], sl, i, cix, cv, X, k);
#pragma unroll
    for (int q = 0; q < KP; ++q) {
        T v = acc[q];
        v += __shfl_xor(v, 4, GROUP);
        v += __shfl_xor(v, 2, GROUP);
        v += __shfl_xor(v, 1, GROUP);
        acc[q] = v;
    }
    const T di = diag[i];
    const T *xi = X + i * k;
    T *yi = Y + i * k;
#pragma unroll
    for (int q = 0; q < KP; ++q)
        if (q < k && (q % GROUP) == sl) yi[q] = acc[q] + di * xi[q];
}

// One workgroup per long CSR row (both segments longer than HEAVY_ROW in
// total): the threads stride over the row's entries, each keeps k partial
// sums, and a fixed-order block reduction writes Y_i.
constexpr int HEAVY_THREADS = 256;
template <typename T, int KP>
__global__ __launch_bounds__(HEAVY_THREADS) void spmm_heavy_kernel(
    int k, const int32_t *__restrict__ rows, const int64_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const T *__restrict__ rv, const int64_t *__restrict__ cp, const int32_t *__restrict__ cri,
    const T *__restrict__ cv, const T *__restrict__ diag, const T *__restrict__ X, T *__restrict__ Y) {
    __shared__ T red[HEAVY_THREADS / LOBPCG_WAVE][KP];
    const int64_t i = rows[blockIdx.x];
    T acc[KP];
#pragma unroll
    for (int q = 0; q < KP; ++q) acc[q] = T(0);
    for (int64_t e = rp[i] + threadIdx.x; e < rp[i + 1]; e += HEAVY_THREADS)
        axpy_row<T, KP>(acc, rv[e], X + (int64_t)ci[e] * k, k);
    for (int64_t e = cp[i] + threadIdx.x; e < cp[i + 1]; e += HEAVY_THREADS)
        axpy_row<T, KP>(acc, cv[e], X + (int64_t)cri[e] * k, k);
    const int lane = threadIdx.x % LOBPCG_WAVE, wave = threadIdx.x / LOBPCG_WAVE;
#pragma unroll
    for (int q = 0; q < KP; ++q) {
        T v = acc[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < k) {
        const int q = threadIdx.x;
        T v = red[0][q];
        for (int w = 1; w < HEAVY_THREADS / LOBPCG_WAVE; ++w) v += red[w][q];
        Y[i * k + q] = v + diag[i] * X[i * k + q];
    }
}

template <typename T>
void spmm_pull_launch(lobpcg_ctx *ctx, const T *X, T *Y, int k, hipStream_t s) {
    const int64_t n = ctx->n;
    const int grid = ceil_div(n * GROUP, SPMM_THREADS);
    const T *rv = (const T *)ctx->val, *cv = (const T *)ctx->cval, *diag = (const T *)ctx->diag;
#define SPMM_ARGS n, k, ctx->rp, ctx->ci, rv, ctx->cp, ctx->cri, cv, diag, X, Y
    if (k <= 4)
        spmm_pull_kernel<T, 4><<<grid, SPMM_THREADS, 0, s>>>(SPMM_ARGS);
    else if (k <= 8)
        spmm_pull_kernel<T, 8><<<grid, SPMM_THREADS, 0, s>>>(SPMM_ARGS);
    else
        spmm_pull_kernel<T, 16><<<grid, SPMM_THREADS, 0, s>>>(SPMM_ARGS);
#undef SPMM_ARGS
    if (ctx->n_heavy > 0) {
        const int hg = (int)ctx->n_heavy;
#define HEAVY_ARGS k, ctx->heavy_rows, ctx->rp, ctx->ci, rv, ctx->cp, ctx->cri, cv, diag, X, Y
        if (k <= 4)
            spmm_heavy_kernel<T, 4><<<hg, HEAVY_THREADS, 0, s>>>(HEAVY_ARGS);
        else if (k <= 8)
            spmm_heavy_kernel<T, 8><<<hg, HEAVY_THREADS, 0, s>>>(HEAVY_ARGS);
        else
            spmm_heavy_kernel<T, 16><<<hg, HEAVY_THREADS, 0, s>>>(HEAVY_ARGS);
#undef HEAVY_ARGS
    }
}

// Column view (CSC of the strict upper triangle) by a parallel, stable counting
// sort on the host: entries keep ascending row order within each column, so
// the result does not depend on the thread count.
template <typename T>
int build_csc(lobpcg_ctx *ctx, hipStream_t s) {
    const int64_t n = ctx->n, m = ctx->nnz_off;
    std::vector<int64_t> rp(n + 1);
    std::vector<int32_t> ci(m);
    std::vector<T> val(m);
    HIP_TRY(ctx, hipMemcpyAsync(rp.data(), ctx->rp, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (m) {
        HIP_TRY(ctx, hipMemcpyAsync(ci.data(), ctx->ci, m * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipMemcpyAsync(val.data(), ctx->val, m * sizeof(T), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(ctx, hipStreamSynchronize(s));
    unsigned hw = std::thread::hardware_concurrency();
    int nth = (int)std::max(1u, std::min(16u, hw ? hw : 1u));
    if (m < (1 << 20)) nth = 1;
    // contiguous row ranges with about equal entry counts
    std::vector<int64_t> rlo(nth + 1);
    for (int t = 0; t <= nth; ++t) {
        int64_t target = m * t / nth;
        rlo[t] = std::lower_bound(rp.begin(), rp.end(), target) - rp.begin();
        if (rlo[t] > n) rlo[t] = n;
    }
    rlo[0] = 0;
    rlo[nth] = n;
    std::vector<std::vector<int64_t>> cnt(nth, std::vector<int64_t>(n + 1, 0));
    auto run = [&](auto &&fn) {
        std::vector<std::thread> th;
        for (int t = 0; t < nth; ++t) th.emplace_back(fn, t);
        for (auto &x : th) x.join();
    };
    run([&](int t) {
        for (int64_t i = rlo[t]; i < rlo[t + 1]; ++i)
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) cnt[t][ci[e]]++;
    });
    std::vector<int64_t> cp(n + 1);
    int64_t acc = 0;
    for (int64_t j = 0; j < n; ++j) {
        cp[j] = acc;
        for (int t = 0; t < nth; ++t) {
            int64_t c = cnt[t][j];
            cnt[t][j] = acc;  // first slot of thread t in column j
            acc += c;
        }
    }
    cp[n] = acc;
    std::vector<int32_t> ri(m);
    std::vector<T> cv(m);
    run([&](int t) {
        for (int64_t i = rlo[t]; i < rlo[t + 1]; ++i)
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                int64_t p = cnt[t][ci[e]]++;
                ri[p] = (int32_t)i;
                cv[p] = val[e];
            }
    });
    HIP_TRY(ctx, hipMalloc((void **)&ctx->cp, (n + 1) * sizeof(int64_t)));
    HIP_TRY(ctx, hipMalloc((void **)&ctx->cri, (m ? m : 1) * sizeof(int32_t)));
    HIP_TRY(ctx, hipMalloc(&ctx->cval, (m ? m : 1) * sizeof(T)));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->cp, cp.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    if (m) {
        HIP_TRY(ctx, hipMemcpyAsync(ctx->cri, ri.data(), m * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipMemcpyAsync(ctx->cval, cv.data(), m * sizeof(T), hipMemcpyHostToDevice, s));
    }
    {
        const int rc = build_row_stats(ctx, s);   // while both views are on the device
        if (rc != LOBPCG_OK) return rc;
    }
    // long rows for spmm_heavy_kernel
    std::vector<int32_t> heavy;
    for (int64_t i = 0; i < n; ++i)
        if ((rp[i + 1] - rp[i]) + (cp[i + 1] - cp[i]) > HEAVY_ROW) heavy.push_back((int32_t)i);
    ctx->n_heavy = (int64_t)heavy.size();
    if (!heavy.empty()) {
        HIP_TRY(ctx, hipMalloc((void **)&ctx->heavy_rows, heavy.size() * sizeof(int32_t)));
        HIP_TRY(ctx, hipMemcpyAsync(ctx->heavy_rows, heavy.data(), heavy.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice, s));
    }
    HIP_TRY(ctx, hipStreamSynchronize(s));
    {
        // dense symmetric 64 x 64 diagonal tiles for the block-diagonal preconditioner
        const int64_t NT = (n + 63) / 64;
        std::vector<T> d(n);
        HIP_TRY(ctx, hipMemcpy(d.data(), ctx->diag, n * sizeof(T), hipMemcpyDeviceToHost));
        std::vector<T> tiles((size_t)NT * 64 * 64, T(0));
        for (int64_t i = 0; i < NT * 64; ++i) {
            T *tl = &tiles[(size_t)(i / 64) * 4096];
            const int a = (int)(i % 64);
            tl[a * 64 + a] = i < n ? d[i] : T(1);
            if (i >= n) continue;
            for (int64_t e = rp[i]; e < rp[i + 1] && ci[e] / 64 == i / 64; ++e) {
                const int b = ci[e] % 64;
                tl[a * 64 + b] = val[e];
                tl[b * 64 + a] = val[e];
            }
        }
        HIP_TRY(ctx, hipMalloc(&ctx->diag_tiles, tiles.size() * sizeof(T)));
        HIP_TRY(ctx, hipMemcpy(ctx->diag_tiles, tiles.data(), tiles.size() * sizeof(T), hipMemcpyHostToDevice));
    }
    if (ctx->format_request == LOBPCG_FORMAT_CSR) return LOBPCG_OK;

    // tiled format (window stream of both views); the 32-bit-index arrays are
    // then no longer needed on the device
    int rc = build_tiled_format(ctx, rp.data(), ci.data(), val.data(), cp.data(), ri.data(), cv.data(), s);
    if (rc != LOBPCG_OK) return rc;
    if (ctx->format == LOBPCG_FORMAT_TILED) {
        void **arrays[] = {(void **)&ctx->rp, (void **)&ctx->ci, &ctx->val, (void **)&ctx->cp, (void **)&ctx->cri,
                           &ctx->cval, (void **)&ctx->heavy_rows};
        for (void **p : arrays) {
            if (*p) (void)hipFree(*p);
            *p = nullptr;
        }
        ctx->n_heavy = 0;
    }
    return LOBPCG_OK;
}

}  // namespace

int launch_fill_zero(void *p, size_t bytes, hipStream_t s) {
    int64_t count = (int64_t)(bytes / 4);
    int zb = (int)std::min<int64_t>((count + 255) / 256, 65536);
    if (count > 0) fill_zero_kernel<float><<<zb, 256, 0, s>>>((float *)p, count);
    return LOBPCG_OK;
}

int build_column_view(lobpcg_ctx *ctx, hipStream_t s) {
    return ctx->dtype == LOBPCG_F32 ? build_csc<float>(ctx, s) : build_csc<double>(ctx, s);
}

int launch_spmm(lobpcg_ctx *ctx, const void *X, void *Y, int k, hipStream_t s) {
    if (ctx->format == LOBPCG_FORMAT_TILED) return spmm_tiled(ctx, X, Y, k, s);
    if (ctx->dtype == LOBPCG_F32) spmm_pull_launch<float>(ctx, (const float *)X, (float *)Y, k, s);
    else spmm_pull_launch<double>(ctx, (const double *)X, (double *)Y, k, s);
    return LOBPCG_OK;
}

extern "C" int lobpcg_spmm_sym(lobpcg_ctx *ctx, const void *X, void *Y, int k, void *stream) {
    if (!ctx) return LOBPCG_EINVAL;
    if (!X || !Y) return set_err(ctx, LOBPCG_EINVAL, "spmm_sym: null block");
    if (X == Y) return set_err(ctx, LOBPCG_EINVAL, "spmm_sym: Y must not alias X");
    if (k < 1 || k > ctx->kmax) return set_err(ctx, LOBPCG_EINVAL, "spmm_sym: k=%d outside [1,%d]", k, ctx->kmax);
    int rc = launch_spmm(ctx, X, Y, k, (hipStream_t)stream);
    if (rc != LOBPCG_OK) return rc;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_err(ctx, LOBPCG_EHIP, "spmm_sym launch: %s", hipGetErrorString(e));
    return LOBPCG_OK;
}
