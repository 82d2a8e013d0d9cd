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
// Mapping: a group of 8 lanes owns one output row; the lanes take every 8th
// entry of the row's two segments (8 consecutive entries per group and step),
// each lane gathers the full k-vector X_j with 16-byte loads and accumulates k
// partial sums in registers; the 8 partials are combined with lane shuffles at
// the end.
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

// Index decoding of the two storage formats.  CSR: int32 global indices.
// TILED: 16-bit (slot << 6 | local) pairs; slot indexes the list of 64-wide
// tile columns (row view) or tile rows (column view) touched by the 64-row
// tile-row that owns the output row, staged in LDS by the workgroup.
constexpr int TILE_SLOTS = 1023;

// Each lane keeps U entries of its row in flight: the U index and value loads
// are issued together, then the U gathers of X rows, then the FMAs, so every
// lane has U independent memory chains outstanding (a single dependent chain
// per lane left the kernel latency-bound).  Padding slots load value 0 and
// gather the row's own X, so they add nothing.
#ifndef LOBPCG_SPMM_UNROLL
#define LOBPCG_SPMM_UNROLL 4
#endif
constexpr int UNROLL = LOBPCG_SPMM_UNROLL;

template <bool TILED>
__device__ inline int64_t decode_index(const void *ix, int64_t e, const int32_t *s_list) {
    if constexpr (TILED) {
        const unsigned u = ((const uint16_t *)ix)[e];
        return (int64_t)s_list[u >> 6] * 64 + (u & 63);
    } else {
        return ((const int32_t *)ix)[e];
    }
}

template <typename T, int KP, bool TILED>
__device__ inline void pull_segment(T (&acc)[KP], int64_t e0, int64_t e1, int sl, int64_t self, const void *ix,
                                    const T *__restrict__ vals, const int32_t *s_list, const T *__restrict__ X,
                                    int k) {
    for (int64_t base = e0; base < e1; base += GROUP * UNROLL) {
        T v[UNROLL];
        int64_t j[UNROLL];
#pragma unroll
        for (int t = 0; t < UNROLL; ++t) {
            const int64_t e = base + t * GROUP + sl;
            const bool ok = e < e1;
            v[t] = ok ? vals[e] : T(0);
            j[t] = ok ? decode_index<TILED>(ix, e, s_list) : self;
        }
#pragma unroll
        for (int t = 0; t < UNROLL; ++t) axpy_row<T, KP>(acc, v[t], X + j[t] * k, k);
    }
}

template <typename T, int KP, bool TILED>
__global__ __launch_bounds__(SPMM_THREADS) void spmm_pull_kernel(
    int64_t n, int k, const int64_t *__restrict__ rp, const void *__restrict__ rix, const T *__restrict__ rv,
    const int64_t *__restrict__ cp, const void *__restrict__ cix, const T *__restrict__ cv,
    const int32_t *__restrict__ rlist_off, const int32_t *__restrict__ rlist,
    const int32_t *__restrict__ clist_off, const int32_t *__restrict__ clist,
    const T *__restrict__ diag, const T *__restrict__ X, T *__restrict__ Y) {
    constexpr int ROWS_PER_BLOCK = SPMM_THREADS / GROUP;   // 32: half of a 64-row tile-row
    __shared__ int32_t s_rl[TILED ? TILE_SLOTS : 1];
    __shared__ int32_t s_cl[TILED ? TILE_SLOTS : 1];
    if constexpr (TILED) {
        const int64_t I = ((int64_t)blockIdx.x * ROWS_PER_BLOCK) / 64;
        const int r0 = rlist_off[I], r1 = rlist_off[I + 1], c0 = clist_off[I], c1 = clist_off[I + 1];
        for (int t = threadIdx.x; t < r1 - r0; t += SPMM_THREADS) s_rl[t] = rlist[r0 + t];
        for (int t = threadIdx.x; t < c1 - c0; t += SPMM_THREADS) s_cl[t] = clist[c0 + t];
        __syncthreads();
    }
    const int64_t i = (int64_t)blockIdx.x * ROWS_PER_BLOCK + threadIdx.x / GROUP;
    const int sl = threadIdx.x % GROUP;
    if (i >= n) return;  // whole groups leave together; no barrier follows
    T acc[KP];
#pragma unroll
    for (int q = 0; q < KP; ++q) acc[q] = T(0);
    pull_segment<T, KP, TILED>(acc, rp[i], rp[i + 1], sl, i, rix, rv, s_rl, X, k);
    pull_segment<T, KP, TILED>(acc, cp[i], cp[i + 1], sl, i, cix, cv, s_cl, X, k);
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

// Tiled format: one 512-thread workgroup per 64-row tile-row (8 lanes per
// row).  Both traversals walk the tile-row's slot lists in windows of WT slots:
// the workgroup stages the 64-row blocks of X that the window's slots refer to
// into LDS with coalesced 16-byte loads (each X block is fetched once per
// tile-row, not once per entry), then each lane consumes its entries whose
// slot falls in the window, BATCH at a time: the batch's index and value
// loads are issued together and the entries past the window are read again
// (from cache) in the next window.  Within a lane the entries are sorted by
// slot, so the consumed entries of a batch are always a prefix.
constexpr int TW_THREADS = 512;
constexpr int BATCH = 8;

template <typename T, int KP>
struct TwShape {
    static constexpr int PAD = 16 / (int)sizeof(T);   // 16-byte pad: keeps row alignment, spreads banks
    static constexpr int STRIDE = KP + PAD;
    static constexpr int SLOT = 64 * STRIDE;           // elements per staged 64-row block
    static constexpr int WT = (32768 / (SLOT * (int)sizeof(T))) < 2 ? 2 : (32768 / (SLOT * (int)sizeof(T)));
};

template <typename T, int KP>
__global__ __launch_bounds__(TW_THREADS) void spmm_tiled_kernel(
    int64_t n, int k, const int64_t *__restrict__ rp, const uint16_t *__restrict__ rix, const T *__restrict__ rv,
    const int64_t *__restrict__ cp, const uint16_t *__restrict__ cix, const T *__restrict__ cv,
    const int32_t *__restrict__ rlist_off, const int32_t *__restrict__ rlist,
    const int32_t *__restrict__ clist_off, const int32_t *__restrict__ clist,
    const T *__restrict__ diag, const T *__restrict__ X, T *__restrict__ Y) {
    using S = TwShape<T, KP>;
    constexpr int VEC = 16 / (int)sizeof(T);           // elements per 16-byte load
    __shared__ int32_t s_list[TILE_SLOTS];
    __shared__ __align__(16) T Xs[S::WT * S::SLOT];
    const int64_t I = blockIdx.x;
    const int r = threadIdx.x / GROUP, sl = threadIdx.x % GROUP;
    const int64_t i = I * 64 + r;
    const bool valid = i < n;
    const bool vec = (k % VEC) == 0;
    T acc[KP];
#pragma unroll
    for (int q = 0; q < KP; ++q) acc[q] = T(0);
    for (int view = 0; view < 2; ++view) {
        const int32_t *loff = view == 0 ? rlist_off : clist_off;
        const int32_t *list = view == 0 ? rlist : clist;
        const uint16_t *ix = view == 0 ? rix : cix;
        const T *vals = view == 0 ? rv : cv;
        const int64_t *ptr = view == 0 ? rp : cp;
        const int l0 = loff[I], nslots = loff[I + 1] - l0;
        __syncthreads();  // the previous view is done with s_list and Xs
        for (int t = threadIdx.x; t < nslots; t += TW_THREADS) s_list[t] = list[l0 + t];
        int64_t e = 0, e_end = 0;
        if (valid) {
            e = ptr[i] + sl;
            e_end = ptr[i + 1];
        }
        for (int s0 = 0; s0 < nslots; s0 += S::WT) {
            const int s1 = min(s0 + S::WT, nslots);
            __syncthreads();  // s_list visible; the previous window is consumed
            if (vec) {
                const int per = 64 * k / VEC;   // 16-byte units per block
                for (int idx = threadIdx.x; idx < (s1 - s0) * per; idx += TW_THREADS) {
                    const int s = idx / per, rem = idx - s * per;
                    const int rr = rem / (k / VEC), q = (rem - rr * (k / VEC)) * VEC;
                    const int64_t grow = (int64_t)s_list[s0 + s] * 64 + rr;
                    T *dst = &Xs[s * S::SLOT + rr * S::STRIDE + q];
                    if constexpr (sizeof(T) == 4) {
                        float4 val = grow < n ? *reinterpret_cast<const float4 *>(X + grow * k + q) : float4{0, 0, 0, 0};
                        *reinterpret_cast<float4 *>(dst) = val;
                    } else {
                        double2 val = grow < n ? *reinterpret_cast<const double2 *>(X + grow * k + q) : double2{0, 0};
                        *reinterpret_cast<double2 *>(dst) = val;
                    }
                }
            } else {
                const int per = 64 * k;
                for (int idx = threadIdx.x; idx < (s1 - s0) * per; idx += TW_THREADS) {
                    const int s = idx / per, rem = idx - s * per, rr = rem / k, q = rem - rr * k;
                    const int64_t grow = (int64_t)s_list[s0 + s] * 64 + rr;
                    Xs[s * S::SLOT + rr * S::STRIDE + q] = grow < n ? X[grow * k + q] : T(0);
                }
            }
            __syncthreads();
            bool more = e < e_end;
            while (more) {
                unsigned u[BATCH];
                T v[BATCH];
#pragma unroll
                for (int t = 0; t < BATCH; ++t) {
                    const int64_t ee = e + (int64_t)t * GROUP;
                    const bool ok = ee < e_end;
                    u[t] = ok ? (unsigned)ix[ee] : 0xFFFFu;   // slot 1023: never inside a window
                    v[t] = ok ? vals[ee] : T(0);
                }
                int consumed = 0;
#pragma unroll
                for (int t = 0; t < BATCH; ++t) {
                    const int slot = (int)(u[t] >> 6);
                    if (slot < s1) {
                        axpy_row<T, KP>(acc, v[t], &Xs[(slot - s0) * S::SLOT + (u[t] & 63) * S::STRIDE], k);
                        ++consumed;
                    }
                }
                e += (int64_t)consumed * GROUP;
                more = consumed == BATCH && e < e_end;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < KP; ++q) {
        T v = acc[q];
        v += __shfl_xor(v, 4, GROUP);
        v += __shfl_xor(v, 2, GROUP);
        v += __shfl_xor(v, 1, GROUP);
        acc[q] = v;
    }
    if (!valid) return;
    const T di = diag[i];
    const T *xi = X + i * k;
    T *yi = Y + i * k;
#pragma unroll
    for (int q = 0; q < KP; ++q)
        if (q < k && (q % GROUP) == sl) yi[q] = acc[q] + di * xi[q];
}

template <typename T, bool TILED>
void spmm_pull_launch(lobpcg_ctx *ctx, const T *X, T *Y, int k, hipStream_t s) {
    const int64_t n = ctx->n;
    const int grid = ceil_div(n * GROUP, SPMM_THREADS);
    const T *rv = (const T *)ctx->val, *cv = (const T *)ctx->cval, *diag = (const T *)ctx->diag;
    const void *rix = TILED ? (const void *)ctx->tiled.rix : (const void *)ctx->ci;
    const void *cix = TILED ? (const void *)ctx->tiled.cix : (const void *)ctx->cri;
#define SPMM_ARGS n, k, ctx->rp, rix, rv, ctx->cp, cix, cv, ctx->tiled.rlist_off, ctx->tiled.rlist, \
                  ctx->tiled.clist_off, ctx->tiled.clist, diag, X, Y
    if (k <= 4)
        spmm_pull_kernel<T, 4, TILED><<<grid, SPMM_THREADS, 0, s>>>(SPMM_ARGS);
    else if (k <= 8)
        spmm_pull_kernel<T, 8, TILED><<<grid, SPMM_THREADS, 0, s>>>(SPMM_ARGS);
    else
        spmm_pull_kernel<T, 16, TILED><<<grid, SPMM_THREADS, 0, s>>>(SPMM_ARGS);
#undef SPMM_ARGS
}

template <typename T>
int spmm_pull(lobpcg_ctx *ctx, const T *X, T *Y, int k, hipStream_t s) {
    if (ctx->format == LOBPCG_FORMAT_TILED) {
        const int grid = (int)ctx->tiled.ntilerows;
        const TiledFormat &tf = ctx->tiled;
        const T *rv = (const T *)ctx->val, *cv = (const T *)ctx->cval, *diag = (const T *)ctx->diag;
#define TW_ARGS ctx->n, k, ctx->rp, tf.rix, rv, ctx->cp, tf.cix, cv, tf.rlist_off, tf.rlist, tf.clist_off, tf.clist, \
                diag, X, Y
        if (k <= 4)
            spmm_tiled_kernel<T, 4><<<grid, TW_THREADS, 0, s>>>(TW_ARGS);
        else if (k <= 8)
            spmm_tiled_kernel<T, 8><<<grid, TW_THREADS, 0, s>>>(TW_ARGS);
        else
            spmm_tiled_kernel<T, 16><<<grid, TW_THREADS, 0, s>>>(TW_ARGS);
#undef TW_ARGS
    } else {
        spmm_pull_launch<T, false>(ctx, X, Y, k, s);
    }
    return LOBPCG_OK;
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
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (ctx->format_request == LOBPCG_FORMAT_CSR) return LOBPCG_OK;

    // 16-bit (tile slot, local index) encoding of both views, per 64-row tile-row
    const int64_t NT = (n + 63) / 64;
    std::vector<std::vector<int32_t>> rl(NT), cl(NT);
    std::vector<uint16_t> rix(m), cix(m);
    std::vector<char> bad(nth, 0);
    auto tiles_of = [&](int64_t lo, int64_t hi, const std::vector<int64_t> &ptr, const std::vector<int32_t> &idx,
                        std::vector<int32_t> &list, std::vector<uint16_t> &out) -> bool {
        list.clear();
        for (int64_t i = lo; i < hi; ++i)
            for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) list.push_back(idx[e] >> 6);
        std::sort(list.begin(), list.end());
        list.erase(std::unique(list.begin(), list.end()), list.end());
        if ((int64_t)list.size() > TILE_SLOTS) return false;
        for (int64_t i = lo; i < hi; ++i)
            for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
                int32_t t = idx[e] >> 6;
                int slot = (int)(std::lower_bound(list.begin(), list.end(), t) - list.begin());
                out[e] = (uint16_t)((slot << 6) | (idx[e] & 63));
            }
        return true;
    };
    {
        std::vector<std::thread> th;
        for (int t = 0; t < nth; ++t)
            th.emplace_back([&, t]() {
                for (int64_t I = t; I < NT; I += nth) {
                    int64_t lo = I * 64, hi = std::min<int64_t>(n, lo + 64);
                    if (!tiles_of(lo, hi, rp, ci, rl[I], rix) || !tiles_of(lo, hi, cp, ri, cl[I], cix)) {
                        bad[t] = 1;
                        return;
                    }
                }
            });
        for (auto &x : th) x.join();
    }
    bool ok = true;
    for (char b : bad) ok = ok && !b;
    if (!ok) {
        if (ctx->format_request == LOBPCG_FORMAT_TILED)
            return set_err(ctx, LOBPCG_EUNSUPPORTED, "tiled format: a tile-row touches more than %d tiles", TILE_SLOTS);
        return LOBPCG_OK;  // automatic choice: keep 32-bit indices
    }
    std::vector<int32_t> roff(NT + 1), coff(NT + 1), rflat, cflat;
    roff[0] = coff[0] = 0;
    for (int64_t I = 0; I < NT; ++I) {
        roff[I + 1] = roff[I] + (int32_t)rl[I].size();
        coff[I + 1] = coff[I] + (int32_t)cl[I].size();
        rflat.insert(rflat.end(), rl[I].begin(), rl[I].end());
        cflat.insert(cflat.end(), cl[I].begin(), cl[I].end());
    }
    TiledFormat &tf = ctx->tiled;
    HIP_TRY(ctx, hipMalloc((void **)&tf.rix, (m ? m : 1) * sizeof(uint16_t)));
    HIP_TRY(ctx, hipMalloc((void **)&tf.cix, (m ? m : 1) * sizeof(uint16_t)));
    HIP_TRY(ctx, hipMalloc((void **)&tf.rlist_off, (NT + 1) * sizeof(int32_t)));
    HIP_TRY(ctx, hipMalloc((void **)&tf.clist_off, (NT + 1) * sizeof(int32_t)));
    HIP_TRY(ctx, hipMalloc((void **)&tf.rlist, std::max<size_t>(1, rflat.size()) * sizeof(int32_t)));
    HIP_TRY(ctx, hipMalloc((void **)&tf.clist, std::max<size_t>(1, cflat.size()) * sizeof(int32_t)));
    if (m) {
        HIP_TRY(ctx, hipMemcpyAsync(tf.rix, rix.data(), m * sizeof(uint16_t), hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, hipMemcpyAsync(tf.cix, cix.data(), m * sizeof(uint16_t), hipMemcpyHostToDevice, s));
    }
    HIP_TRY(ctx, hipMemcpyAsync(tf.rlist_off, roff.data(), (NT + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(tf.clist_off, coff.data(), (NT + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (!rflat.empty())
        HIP_TRY(ctx, hipMemcpyAsync(tf.rlist, rflat.data(), rflat.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (!cflat.empty())
        HIP_TRY(ctx, hipMemcpyAsync(tf.clist, cflat.data(), cflat.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    tf.ntilerows = NT;
    tf.nslots_row = (int64_t)rflat.size();
    tf.nslots_col = (int64_t)cflat.size();
    // the 32-bit index arrays are not needed by the tiled kernels
    (void)hipFree(ctx->ci);
    (void)hipFree(ctx->cri);
    ctx->ci = nullptr;
    ctx->cri = nullptr;
    ctx->format = LOBPCG_FORMAT_TILED;
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
    if (ctx->dtype == LOBPCG_F32) return spmm_pull<float>(ctx, (const float *)X, (float *)Y, k, s);
    return spmm_pull<double>(ctx, (const double *)X, (double *)Y, k, s);
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
