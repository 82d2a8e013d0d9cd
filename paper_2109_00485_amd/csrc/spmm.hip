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
// the 8 partials are combined with lane shuffles at the end.  The tiled kernel
// (below) keeps the 8 lanes per row but takes 4-entry chunks of the padded
// segments and reads X from blocks staged in LDS.
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
    if constexpr (!TILED) {
        // long rows belong to spmm_heavy_kernel (the same predicate decides there)
        if ((rp[i + 1] - rp[i]) + (cp[i + 1] - cp[i]) > HEAVY_ROW) return;
    }
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

#ifndef LOBPCG_TW_LDS
#define LOBPCG_TW_LDS 0         // bytes of LDS for staged X blocks per workgroup (0: by block width)
#endif
#ifndef LOBPCG_TW_DB
#define LOBPCG_TW_DB 0          // double-buffer the X windows
#endif
#ifndef LOBPCG_TW_GROUP
#define LOBPCG_TW_GROUP 0       // lanes per output row in the tiled kernel (0: 8)
#endif
#ifndef LOBPCG_TW_CHUNK
#define LOBPCG_TW_CHUNK 4       // entries a lane takes per step (4 or 8)
#endif
#ifndef LOBPCG_TW_PF
#define LOBPCG_TW_PF 1          // prefetch the next chunk of each lane (full-width path)
#endif
#ifndef LOBPCG_TW_MINWAVES
#define LOBPCG_TW_MINWAVES 6    // ask the register allocator for this many waves per SIMD (0: its choice)
#endif
#if LOBPCG_TW_MINWAVES > 0
#define TW_WAVES_ATTR __attribute__((amdgpu_waves_per_eu(LOBPCG_TW_MINWAVES)))
#else
#define TW_WAVES_ATTR
#endif
#ifndef LOBPCG_TW_PAD
#define LOBPCG_TW_PAD -1        // pad staged X rows by 16 bytes (-1: by block width)
#endif
constexpr int NBUF = LOBPCG_TW_DB ? 2 : 1;

template <typename T, int KP>
struct TwShape {
    // 8 lanes per output row taking 4-entry chunks; rows of up to 32 bytes are
    // staged unpadded, wider rows with a 16-byte pad (measured best on gfx950)
    static constexpr bool NARROW = KP * (int)sizeof(T) <= 32;
    static constexpr int TG = LOBPCG_TW_GROUP ? LOBPCG_TW_GROUP : 8;
    static constexpr int THREADS = 64 * TG;
    // entries per chunk (segments are padded to 8, so 8 or 4)
    static constexpr int CH = LOBPCG_TW_CHUNK;
    // keep the lane's next chunk in flight while it works on the current one
    static constexpr bool PF = LOBPCG_TW_PF;
    static constexpr int PAD = (LOBPCG_TW_PAD < 0 ? !NARROW : LOBPCG_TW_PAD) ? 16 / (int)sizeof(T) : 0;
    static constexpr int STRIDE = KP + PAD;
    static constexpr int SLOT = 64 * STRIDE;           // elements per staged 64-row block
    // staged X: 40 KB (20 slots of 32-byte rows) for rows of up to 32 bytes, so
    // three workgroups share a CU; 64 KB for wider rows (measured best on gfx950)
    static constexpr int LDS_BYTES = LOBPCG_TW_LDS ? LOBPCG_TW_LDS : (KP * (int)sizeof(T) > 32 ? 65536 : 40960);
    static constexpr int WT0 = LDS_BYTES / NBUF / (SLOT * (int)sizeof(T));
    static constexpr int WT = WT0 < 2 ? 2 : WT0;       // slots per window
    static constexpr int VEC = 16 / (int)sizeof(T);    // elements per 16-byte load
    static constexpr int MAXV = (WT * 64 * KP / VEC + THREADS - 1) / THREADS;  // 16-byte loads per thread
};

// one 16-byte unit of a staged window (vector path, k == KP): slot s, block row rr, column q
template <typename T, int KP>
__device__ inline void tw_unit(int idx, int &s, int &rr, int &q) {
    constexpr int VEC = TwShape<T, KP>::VEC;
    constexpr int UPR = KP / VEC;        // 16-byte units per row (power of two)
    constexpr int PER = 64 * UPR;        // units per 64-row block
    s = idx / PER;
    const int rem = idx - s * PER;
    rr = rem / UPR;
    q = (rem - rr * UPR) * VEC;
}

// Tiled format: one 512-thread workgroup per 64-row tile-row (8 lanes per
// row).  Both traversals walk the tile-row's slot lists in windows of WT slots:
// the workgroup stages the 64-row blocks of X that the window's slots refer to
// into LDS with coalesced 16-byte loads (each X block is fetched once per
// tile-row, not once per entry), then each lane consumes its entries whose
// slot falls in the window.  Row segments are padded to whole 8-entry chunks;
// chunk m (CH entries) of a segment belongs to lane m % 8, which reads its
// codes and values with one load each; a chunk that straddles a window
// boundary is consumed in two windows.  Entries are sorted by slot, so what a
// lane consumes of a chunk is always a contiguous run.
// FULL: k equals the compiled width KP (a whole number of 16-byte units), so
// staging is vectorised and each entry's update has no per-column branches,
// and each lane keeps its next chunk's loads in flight while it works on the
// current one.
template <typename T, int KP, bool FULL>
__global__ __launch_bounds__((TwShape<T, KP>::THREADS)) TW_WAVES_ATTR void spmm_tiled_kernel(
    int64_t n, int k, const int64_t *__restrict__ rp, const uint16_t *__restrict__ rix, const T *__restrict__ rv,
    const int64_t *__restrict__ cp, const uint16_t *__restrict__ cix, const T *__restrict__ cv,
    const int32_t *__restrict__ rlist_off, const int32_t *__restrict__ rlist,
    const int32_t *__restrict__ clist_off, const int32_t *__restrict__ clist,
    const T *__restrict__ diag, const T *__restrict__ X, T *__restrict__ Y) {
    using S = TwShape<T, KP>;
    constexpr int TG = S::TG;
    constexpr int VEC = S::VEC;
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    __shared__ int32_t s_list[TILE_SLOTS];
    __shared__ __align__(16) T Xs[NBUF * S::WT * S::SLOT];
    const int64_t I = blockIdx.x;
    const int r = threadIdx.x / TG, sl = threadIdx.x % TG;
    const int64_t i = I * 64 + r;
    const bool valid = i < n;
    constexpr bool vec = FULL;
    T acc[KP];
#pragma unroll
    for (int q = 0; q < KP; ++q) acc[q] = T(0);
    // stage window [s0, s1) into buffer b (scalar path for k not a multiple of the vector width)
    auto stage_scalar = [&](int s0, int s1, int b) {
        const int per = 64 * k;
        for (int idx = threadIdx.x; idx < (s1 - s0) * per; idx += S::THREADS) {
            const int s = idx / per, rem = idx - s * per, rr = rem / k, q = rem - rr * k;
            const int64_t grow = (int64_t)s_list[s0 + s] * 64 + rr;
            Xs[(b * S::WT + s) * S::SLOT + rr * S::STRIDE + q] = grow < n ? X[grow * k + q] : T(0);
        }
    };
    // one lane's chunk of CH entries in registers: CH 16-bit codes and CH values
    constexpr int CH = S::CH;
    using CodeT = typename std::conditional<CH == 8, uint4, uint2>::type;
    struct Chunk {
        CodeT c;
        V a[CH * (int)sizeof(T) / 16];
    };
    auto load_chunk = [&](const uint16_t *ix, const T *vals, int64_t p) {
        Chunk ck;
        ck.c = *reinterpret_cast<const CodeT *>(ix + p);
#pragma unroll
        for (int h = 0; h < CH * (int)sizeof(T) / 16; ++h) ck.a[h] = *reinterpret_cast<const V *>(vals + p + h * VEC);
        return ck;
    };
    auto pick_chunk = [&](bool first, const Chunk &a, const Chunk &b) {   // element-wise select
        Chunk ck;
        ck.c.x = first ? a.c.x : b.c.x;
        ck.c.y = first ? a.c.y : b.c.y;
        if constexpr (CH == 8) {
            ck.c.z = first ? a.c.z : b.c.z;
            ck.c.w = first ? a.c.w : b.c.w;
        }
#pragma unroll
        for (int h = 0; h < CH * (int)sizeof(T) / 16; ++h) {
            ck.a[h].x = first ? a.a[h].x : b.a[h].x;
            ck.a[h].y = first ? a.a[h].y : b.a[h].y;
            if constexpr (sizeof(T) == 4) {
                ck.a[h].z = first ? a.a[h].z : b.a[h].z;
                ck.a[h].w = first ? a.a[h].w : b.a[h].w;
            }
        }
        return ck;
    };
    V pre[S::MAXV];
    auto fetch = [&](int s0, int s1) {   // global loads of a window into registers
#pragma unroll
        for (int u = 0; u < S::MAXV; ++u) {
            const int idx = threadIdx.x + u * S::THREADS;
            if (idx < (s1 - s0) * (64 * KP / VEC)) {
                int s, rr, q;
                tw_unit<T, KP>(idx, s, rr, q);
                const int64_t grow = (int64_t)s_list[s0 + s] * 64 + rr;
                pre[u] = grow < n ? *reinterpret_cast<const V *>(X + grow * KP + q) : V{};
            }
        }
    };
    auto deposit = [&](int s0, int s1, int b) {   // registers into LDS buffer b
#pragma unroll
        for (int u = 0; u < S::MAXV; ++u) {
            const int idx = threadIdx.x + u * S::THREADS;
            if (idx < (s1 - s0) * (64 * KP / VEC)) {
                int s, rr, q;
                tw_unit<T, KP>(idx, s, rr, q);
                *reinterpret_cast<V *>(&Xs[(b * S::WT + s) * S::SLOT + rr * S::STRIDE + q]) = pre[u];
            }
        }
    };
    for (int view = 0; view < 2; ++view) {
        const int32_t *loff = view == 0 ? rlist_off : clist_off;
        const int32_t *list = view == 0 ? rlist : clist;
        const uint16_t *ix = view == 0 ? rix : cix;
        const T *vals = view == 0 ? rv : cv;
        const int64_t *ptr = view == 0 ? rp : cp;
        const int l0 = loff[I], nslots = loff[I + 1] - l0;
        __syncthreads();  // the previous view is done with s_list and Xs
        for (int t = threadIdx.x; t < nslots; t += S::THREADS) s_list[t] = list[l0 + t];
        // this lane's chunks of its row segment: chunk m (CH entries) belongs to lane m % TG
        int64_t pos = 0, seg_end = 0;
        int off = 0;   // entries of the current chunk already consumed
        if (valid) {
            pos = ptr[i] + S::CH * sl;
            seg_end = ptr[i + 1];
        }
        // with prefetch, cur holds the chunk at pos and nxt the lane's following one
        // (segments are padded to 8 entries, so a chunk that starts inside one ends inside it)
        constexpr bool PF = FULL && S::PF;
        Chunk cur{}, nxt{};
        if constexpr (PF) {
            if (pos < seg_end) {
                cur = load_chunk(ix, vals, pos);
                // past the segment's end the load is redirected to its last chunk (never used)
                nxt = load_chunk(ix, vals, min(pos + CH * TG, seg_end - CH));
            }
        }
        __syncthreads();
        if (nslots > 0) {
            if (vec) {
                fetch(0, min(S::WT, nslots));
                deposit(0, min(S::WT, nslots), 0);
            } else {
                stage_scalar(0, min(S::WT, nslots), 0);
            }
        }
        int w = 0;
        for (int s0 = 0; s0 < nslots; s0 += S::WT, ++w) {
            const int s1 = min(s0 + S::WT, nslots);
            const int b = NBUF == 2 ? (w & 1) : 0;
            const int n0 = s1, n1 = min(s1 + S::WT, nslots);
            __syncthreads();  // buffer b holds window [s0, s1)
            if (NBUF == 2 && vec && n0 < n1) fetch(n0, n1);   // next window in flight during this one
            bool more = pos < seg_end;
            while (more) {
                Chunk ck;
                if constexpr (PF) ck = cur;
                else ck = load_chunk(ix, vals, pos);
                unsigned u[CH];
                if constexpr (CH == 8) {
                    const unsigned w4[4] = {ck.c.x, ck.c.y, ck.c.z, ck.c.w};
#pragma unroll
                    for (int h = 0; h < 4; ++h) { u[2 * h] = w4[h] & 0xFFFFu; u[2 * h + 1] = w4[h] >> 16; }
                } else {
                    u[0] = ck.c.x & 0xFFFFu; u[1] = ck.c.x >> 16; u[2] = ck.c.y & 0xFFFFu; u[3] = ck.c.y >> 16;
                }
                T v[CH];
                if constexpr (sizeof(T) == 4) {
#pragma unroll
                    for (int h = 0; h < CH / 4; ++h) {
                        v[4 * h] = ck.a[h].x; v[4 * h + 1] = ck.a[h].y; v[4 * h + 2] = ck.a[h].z; v[4 * h + 3] = ck.a[h].w;
                    }
                } else {
#pragma unroll
                    for (int h = 0; h < CH / 2; ++h) {
                        v[2 * h] = ck.a[h].x;
                        v[2 * h + 1] = ck.a[h].y;
                    }
                }
                // the code slot*64 + c is the staged row index; rows of this window
                // start at s0*64, and padding (0xFFFF) never falls below lim
                const unsigned lim = (unsigned)s1 * 64u, base = (unsigned)s0 * 64u;
                const T *xb = &Xs[b * S::WT * S::SLOT];
                int nb = 0;
#pragma unroll
                for (int t = 0; t < CH; ++t) nb += u[t] < lim ? 1 : 0;
                // FULL: the width is a compile-time constant, so each entry is one
                // straight run of 16-byte LDS reads and FMAs
#pragma unroll
                for (int t = 0; t < CH; ++t)
                    if (t >= off && t < nb) axpy_row<T, KP>(acc, v[t], xb + (u[t] - base) * S::STRIDE, FULL ? KP : k);
                off = nb;   // slots are sorted within the chunk: [old off, nb) was just consumed
                if constexpr (PF) {
                    // every active lane reloads nxt (no load under a branch, so the loaded
                    // registers need no copy and the load stays in flight through the next
                    // chunk): the chunk after the next one when this chunk is done, else
                    // the next one again
                    const bool adv = off == CH;
                    const int64_t npos = pos + CH * TG;
                    const int64_t want = adv ? npos + CH * TG : npos;
                    cur = pick_chunk(adv, nxt, cur);
                    nxt = load_chunk(ix, vals, min(want, seg_end - CH));
                    if (adv) {
                        pos = npos;
                        off = 0;
                        more = pos < seg_end;
                    } else {
                        more = false;
                    }
                } else if (off == CH) {
                    pos += CH * TG;
                    off = 0;
                    more = pos < seg_end;
                } else {
                    more = false;
                }
            }
            if (n0 < n1) {
                if (NBUF == 2 && vec) {
                    deposit(n0, n1, b ^ 1);   // the other buffer was last read before the barrier above
                } else {
                    __syncthreads();          // single buffer: everyone is done reading window [s0, s1)
                    if (vec) {
                        fetch(n0, n1);
                        deposit(n0, n1, 0);
                    } else {
                        stage_scalar(n0, n1, NBUF == 2 ? (b ^ 1) : 0);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < KP; ++q) {
        T v = acc[q];
#pragma unroll
        for (int m = TG / 2; m > 0; m >>= 1) v += __shfl_xor(v, m, TG);
        acc[q] = v;
    }
    if (!valid) return;
    const T di = diag[i];
    const T *xi = X + i * k;
    T *yi = Y + i * k;
#pragma unroll
    for (int q = 0; q < KP; ++q)
        if (q < k && (q % TG) == sl) yi[q] = acc[q] + di * xi[q];
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
    if (!TILED && ctx->n_heavy > 0) {
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

template <typename T>
int spmm_pull(lobpcg_ctx *ctx, const T *X, T *Y, int k, hipStream_t s) {
    if (ctx->format == LOBPCG_FORMAT_TILED) {
        const int grid = (int)ctx->tiled.ntilerows;
        const TiledFormat &tf = ctx->tiled;
        const T *rv = (const T *)ctx->val, *cv = (const T *)ctx->cval, *diag = (const T *)ctx->diag;
#define TW_ARGS ctx->n, k, ctx->rp, tf.rix, rv, ctx->cp, tf.cix, cv, tf.rlist_off, tf.rlist, tf.clist_off, tf.clist, \
                diag, X, Y
#define TW_LAUNCH(KP)                                                                        \
    do {                                                                                     \
        if (k == (KP) && (KP) % TwShape<T, KP>::VEC == 0)                                    \
            spmm_tiled_kernel<T, KP, true><<<grid, TwShape<T, KP>::THREADS, 0, s>>>(TW_ARGS);  \
        else                                                                                 \
            spmm_tiled_kernel<T, KP, false><<<grid, TwShape<T, KP>::THREADS, 0, s>>>(TW_ARGS); \
    } while (0)
        if (k <= 4)
            TW_LAUNCH(4);
        else if (k <= 8)
            TW_LAUNCH(8);
        else
            TW_LAUNCH(16);
#undef TW_LAUNCH
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
    {
        const int rc = build_row_stats(ctx, s);   // before the tiled format pads the value arrays
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
    // pad every row segment of both views to a multiple of 8 entries (index
    // 0xFFFF = slot 1023, never inside a window; value 0) so that each lane
    // reads whole 8-entry chunks with 16-byte loads
    auto pad8 = [&](const std::vector<int64_t> &ptr, const std::vector<uint16_t> &ix, const std::vector<T> &vv,
                    std::vector<int64_t> &ptr8, std::vector<uint16_t> &ix8, std::vector<T> &v8) {
        ptr8.assign(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) ptr8[i + 1] = ptr8[i] + ((ptr[i + 1] - ptr[i] + 7) / 8) * 8;
        ix8.assign(ptr8[n], (uint16_t)0xFFFF);
        v8.assign(ptr8[n], T(0));
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) {
                ix8[ptr8[i] + (e - ptr[i])] = ix[e];
                v8[ptr8[i] + (e - ptr[i])] = vv[e];
            }
    };
    std::vector<int64_t> rp8, cp8;
    std::vector<uint16_t> rix8, cix8;
    std::vector<T> rv8, cv8;
    {
        std::thread t1([&]() { pad8(rp, rix, val, rp8, rix8, rv8); });
        pad8(cp, cix, cv, cp8, cix8, cv8);
        t1.join();
    }
    const int64_t mr = rp8[n], mc = cp8[n];
    // the padded views replace the 32-bit-index arrays on the device
    (void)hipFree(ctx->ci);
    (void)hipFree(ctx->cri);
    (void)hipFree(ctx->val);
    (void)hipFree(ctx->cval);
    ctx->ci = nullptr;
    ctx->cri = nullptr;
    ctx->val = nullptr;
    ctx->cval = nullptr;
    HIP_TRY(ctx, hipMalloc(&ctx->val, std::max<int64_t>(1, mr) * sizeof(T)));
    HIP_TRY(ctx, hipMalloc(&ctx->cval, std::max<int64_t>(1, mc) * sizeof(T)));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->rp, rp8.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->cp, cp8.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    if (mr) HIP_TRY(ctx, hipMemcpyAsync(ctx->val, rv8.data(), mr * sizeof(T), hipMemcpyHostToDevice, s));
    if (mc) HIP_TRY(ctx, hipMemcpyAsync(ctx->cval, cv8.data(), mc * sizeof(T), hipMemcpyHostToDevice, s));
    TiledFormat &tf = ctx->tiled;
    tf.nent_row = mr;
    tf.nent_col = mc;
    HIP_TRY(ctx, hipMalloc((void **)&tf.rix, std::max<int64_t>(1, mr) * sizeof(uint16_t)));
    HIP_TRY(ctx, hipMalloc((void **)&tf.cix, std::max<int64_t>(1, mc) * sizeof(uint16_t)));
    HIP_TRY(ctx, hipMalloc((void **)&tf.rlist_off, (NT + 1) * sizeof(int32_t)));
    HIP_TRY(ctx, hipMalloc((void **)&tf.clist_off, (NT + 1) * sizeof(int32_t)));
    HIP_TRY(ctx, hipMalloc((void **)&tf.rlist, std::max<size_t>(1, rflat.size()) * sizeof(int32_t)));
    HIP_TRY(ctx, hipMalloc((void **)&tf.clist, std::max<size_t>(1, cflat.size()) * sizeof(int32_t)));
    if (mr) HIP_TRY(ctx, hipMemcpyAsync(tf.rix, rix8.data(), mr * sizeof(uint16_t), hipMemcpyHostToDevice, s));
    if (mc) HIP_TRY(ctx, hipMemcpyAsync(tf.cix, cix8.data(), mc * sizeof(uint16_t), hipMemcpyHostToDevice, s));
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
