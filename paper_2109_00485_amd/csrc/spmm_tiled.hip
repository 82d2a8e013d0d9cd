// Tiled symmetric product Y = H X for matrices whose stored upper triangle
// falls into dense-enough 64 x 64 tiles (the block structure of the paper's
// CI matrices, Section 3.2).
//
// Both halves of the product are pulls over output rows, as in the paper's
// CPU code (Section 3.2): the row view holds the stored entries u_ij (j > i)
// of row i, the column view the stored entries u_ji (j < i) of column i, so
//     Y_i = d_i X_i + sum_{row view} u_ij X_j + sum_{column view} u_ji X_j
// and Y is written once, with no atomics.  (Pushing the transposed half from
// the stored tile instead needs a 2 KB block of partial sums per tile, more
// bytes than reading the tile's 6-byte entries a second time.)
//
// Layout: one workgroup per 64-row tile-row.  Its work is a stream of
// windows, first over the row view, then over the column view; a window
// covers up to `ws` consecutive tiles ("slots") of one view and holds
//     tab[65]   uint16 chunk offsets, one per row of the tile-row (+ end)
//     codes     4 uint16 per chunk: (slot - first slot) * 64 + local index
//     values    4 per chunk
// with each row's entries padded to whole 4-entry chunks (padding points at a
// zero row).  Window blocks are contiguous in memory, so a window's matrix
// bytes and the 64-row blocks of X its slots refer to are copied into LDS by
// direct global-to-LDS loads (global_load_lds_dwordx4): every byte the product
// reads from HBM is a wide, fully coalesced request, issued for the next
// window as soon as the workgroup is done with the current one.  The compute
// then only reads LDS: a group of TG lanes per row walks the row's chunks,
// each entry one row of staged X times its value.
#include <algorithm>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace {

typedef __attribute__((address_space(3))) void *lds_ptr;

constexpr int TAB_BYTES = 144;   // 65 uint16 chunk offsets, padded to 16 bytes
constexpr int CH = 4;            // entries per chunk
constexpr int CPOL_NT = 2;       // cache-policy operand of global_load_lds: non-temporal
#ifndef LOBPCG_TILE_TG
#define LOBPCG_TILE_TG 4         // lanes per output row
#endif
#ifndef LOBPCG_TILE_WS
#define LOBPCG_TILE_WS 8         // 64-wide blocks of X per window (FP32; half as many in FP64)
#endif
#ifndef LOBPCG_TILE_ECAP
#define LOBPCG_TILE_ECAP 320     // chunk-padded entries per window, per block it may hold
#endif
constexpr int TG = LOBPCG_TILE_TG;
constexpr int THREADS = 64 * TG;
constexpr int NWAVE = THREADS / LOBPCG_WAVE;
constexpr int MAXJ = 8;          // X wave-loads per wave and window (ws * row bytes / 16 <= MAXJ * NWAVE)

// Register budget: the FP32 k = 8 instantiation is held to five waves per SIMD
// (its LDS allows four to five workgroups per CU; measured 2% faster than the
// allocator's own choice of four waves); the others keep the allocator's.
template <typename T, int KP>
struct TileWaves {
    static constexpr int value = (sizeof(T) == 4 && KP == 8) ? 5 : 1;
};

__host__ __device__ inline int round16(int64_t b) { return (int)((b + 15) & ~(int64_t)15); }

// LDS bytes of the staged X rows: ws*64 rows + one zero row, KP elements each
__host__ __device__ inline int x_bytes(int ws, int kp, int esz) { return round16((int64_t)(ws * 64 + 1) * kp * esz); }
__host__ __device__ inline int m_bytes(int emax, int esz) { return TAB_BYTES + round16((int64_t)emax * 2) + emax * esz; }

// FULL: k == KP and rows are whole 16-byte units, so X blocks are staged by
// direct global-to-LDS loads; otherwise the workgroup stages them through
// registers with the columns beyond k set to zero.  LDS rows are always KP
// wide, so the compute loop never branches on k.
template <typename T, int KP, bool FULL>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(TileWaves<T, KP>::value))) void spmm_window_kernel(
    int64_t n, int k, int ws, int emax, const char *__restrict__ data, const int64_t *__restrict__ woff,
    const int2 *__restrict__ wdesc, const int32_t *__restrict__ wbeg, const int32_t *__restrict__ list,
    const T *__restrict__ diag, const T *__restrict__ X, T *__restrict__ Y) {
    extern __shared__ __align__(16) char lds[];
    constexpr int ESZ = (int)sizeof(T);
    constexpr int U = KP * ESZ / 16;                  // 16-byte units per X row (FULL)
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    constexpr int VE = 16 / ESZ;                      // elements per 16-byte vector
    const int xb = x_bytes(ws, KP, ESZ);
    T *Xs = reinterpret_cast<T *>(lds);
    char *mb = lds + xb;
    const int64_t I = blockIdx.x;
    const int r = threadIdx.x / TG, sl = threadIdx.x % TG;
    const int wave = threadIdx.x / LOBPCG_WAVE, lane = threadIdx.x % LOBPCG_WAVE;
    const int64_t i = I * 64 + r;
    if (threadIdx.x < KP) Xs[ws * 64 * KP + threadIdx.x] = T(0);   // the zero row padding codes point at
    T acc[KP];
#pragma unroll
    for (int q = 0; q < KP; ++q) acc[q] = T(0);

    // descriptor of the next window to stage (wave-uniform) and, for FULL, the
    // X block index of each of this wave's wave-loads
    int64_t nb0 = 0, nnb = 0;
    int nslot0 = 0, nns = 0;
    int tix[FULL ? MAXJ : 1];
    auto load_desc = [&](int w) {
        nb0 = woff[w];
        nnb = woff[w + 1] - nb0;
        const int2 d = wdesc[w];
        nslot0 = d.x;
        nns = d.y;
        if constexpr (FULL) {
#pragma unroll
            for (int m = 0; m < MAXJ; ++m) {
                const int j = wave + m * NWAVE;
                if (j < nns * U) tix[m] = list[nslot0 + j / U];
            }
        }
    };
    auto stage = [&]() {
        // matrix bytes of the window: 1 KB per wave-load, lanes past the end idle;
        // read once per product, so marked non-temporal (cache policy NT) to
        // leave the caches to the X blocks, which other windows read again
        const int nwl = (int)((nnb + 1023) >> 10);
        for (int j = wave; j < nwl; j += NWAVE)
            if ((int64_t)j * 1024 + lane * 16 < nnb)
                __builtin_amdgcn_global_load_lds((const void *)(data + nb0 + (int64_t)j * 1024 + lane * 16),
                                                 (lds_ptr)(mb + j * 1024), 16, 0, CPOL_NT);
        if constexpr (FULL) {
            // X blocks: U wave-loads of 64 lanes x 16 bytes per 64-row block
#pragma unroll
            for (int m = 0; m < MAXJ; ++m) {
                const int j = wave + m * NWAVE;
                if (j < nns * U) {
                    const int s = j / U, p = j % U;
                    const int u = p * 64 + lane, rr = u / U, q = u % U;
                    int64_t g = (int64_t)tix[m] * 64 + rr;
                    g = g < n ? g : n - 1;   // rows past n are never referenced by a code
                    __builtin_amdgcn_global_load_lds((const void *)(X + g * KP + q * VE),
                                                     (lds_ptr)(lds + (s * 64 * KP) * ESZ + p * 1024), 16, 0, 0);
                }
            }
        } else {
            for (int e = threadIdx.x; e < nns * 64 * KP; e += THREADS) {
                const int s = e / (64 * KP), rem = e - s * 64 * KP, rr = rem / KP, q = rem - rr * KP;
                const int64_t g = (int64_t)list[nslot0 + s] * 64 + rr;
                Xs[e] = (q < k && g < n) ? X[g * k + q] : T(0);
            }
        }
    };

    const int w0 = wbeg[I], w1 = wbeg[I + 1];
    if (w0 < w1) {
        load_desc(w0);
        __syncthreads();   // the zero row is written
        stage();
        if (w0 + 1 < w1) load_desc(w0 + 1);
    }
    for (int w = w0; w < w1; ++w) {
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's direct-to-LDS loads have landed
        __syncthreads();                      // ... and every other wave's
        const uint16_t *tab = reinterpret_cast<const uint16_t *>(mb);
        const int nchunk = tab[64];
        const uint2 *codes = reinterpret_cast<const uint2 *>(mb + TAB_BYTES);
        const V *vals = reinterpret_cast<const V *>(mb + TAB_BYTES + round16((int64_t)nchunk * 8));
        const int c1 = i < n ? tab[r + 1] : 0;
        for (int c = (i < n ? tab[r] : 0) + sl; c < c1; c += TG) {
            const uint2 cw = codes[c];
            T v[CH];
#pragma unroll
            for (int h = 0; h < CH / VE; ++h) {
                const V t = vals[c * (CH / VE) + h];
                if constexpr (sizeof(T) == 4) {
                    v[4 * h] = t.x; v[4 * h + 1] = t.y; v[4 * h + 2] = t.z; v[4 * h + 3] = t.w;
                } else {
                    v[2 * h] = t.x; v[2 * h + 1] = t.y;
                }
            }
            const unsigned u[CH] = {cw.x & 0xFFFFu, cw.x >> 16, cw.y & 0xFFFFu, cw.y >> 16};
#pragma unroll
            for (int t = 0; t < CH; ++t) {
                const V *xr = reinterpret_cast<const V *>(Xs + u[t] * KP);
#pragma unroll
                for (int h = 0; h < KP / VE; ++h) {
                    const V x = xr[h];
                    if constexpr (sizeof(T) == 4) {
                        acc[4 * h] += v[t] * x.x; acc[4 * h + 1] += v[t] * x.y;
                        acc[4 * h + 2] += v[t] * x.z; acc[4 * h + 3] += v[t] * x.w;
                    } else {
                        acc[2 * h] += v[t] * x.x; acc[2 * h + 1] += v[t] * x.y;
                    }
                }
            }
        }
        if (w + 1 < w1) {
            __syncthreads();   // everyone is done with this window's LDS
            stage();
            if (w + 2 < w1) load_desc(w + 2);
        }
    }
#pragma unroll
    for (int q = 0; q < KP; ++q) {
        T v = acc[q];
#pragma unroll
        for (int m = TG / 2; m > 0; m >>= 1) v += __shfl_xor(v, m, TG);
        acc[q] = v;
    }
    if (i >= n) return;
    const T di = diag[i];
#pragma unroll
    for (int q = 0; q < KP; ++q)
        if (q < k && q % TG == sl) Y[i * k + q] = acc[q] + di * X[i * k + q];
}

// Per tile-row and view: the sorted list of 64-wide blocks ("slots") the
// entries touch, the number of entries of every row in each slot, and the
// windows (consecutive slot ranges) they are cut into.
struct ViewPlan {
    std::vector<int32_t> slots;
    std::vector<uint8_t> cnt;          // [64][nslots]; a row has at most 64 entries in a slot
    struct Win { int s0, ns, chunks; };
    std::vector<Win> wins;
};

// Entries of rows [rlo, rhi) in one view: indices idx[ptr[r]..ptr[r+1]) ascending.
void plan_view(int64_t rlo, int64_t rhi, const int64_t *ptr, const int32_t *idx, int ws, int64_t ecap,
               ViewPlan &pl) {
    pl.slots.clear();
    pl.wins.clear();
    for (int64_t r = rlo; r < rhi; ++r)
        for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) pl.slots.push_back(idx[e] >> 6);
    std::sort(pl.slots.begin(), pl.slots.end());
    pl.slots.erase(std::unique(pl.slots.begin(), pl.slots.end()), pl.slots.end());
    const int ns = (int)pl.slots.size();
    pl.cnt.assign((size_t)64 * ns, 0);
    for (int64_t r = rlo; r < rhi; ++r) {
        int s = 0;
        for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
            const int32_t b = idx[e] >> 6;
            while (pl.slots[s] != b) ++s;   // entries and slots are both ascending
            pl.cnt[(size_t)(r - rlo) * ns + s]++;
        }
    }
    // windows: consecutive slots, at most ws of them and (beyond the first) at
    // most ecap chunk-padded entries
    int s0 = 0;
    std::vector<int> run(64);
    while (s0 < ns) {
        std::fill(run.begin(), run.end(), 0);
        int s1 = s0;
        int64_t chunks = 0;
        while (s1 < ns && s1 - s0 < ws) {
            int64_t c2 = 0;
            for (int r = 0; r < 64; ++r) c2 += (run[r] + pl.cnt[(size_t)r * ns + s1] + CH - 1) / CH;
            if (s1 > s0 && c2 * CH > ecap) break;
            for (int r = 0; r < 64; ++r) run[r] += pl.cnt[(size_t)r * ns + s1];
            chunks = c2;
            ++s1;
        }
        pl.wins.push_back({s0, s1 - s0, (int)chunks});
        s0 = s1;
    }
}

int64_t win_bytes(int chunks, int esz) { return TAB_BYTES + round16((int64_t)chunks * 8) + (int64_t)chunks * CH * esz; }

// Write the window blocks of one view of one tile-row at dst.
template <typename T>
void write_view(int64_t rlo, int64_t rhi, const int64_t *ptr, const int32_t *idx, const T *val, int ws,
                const ViewPlan &pl, char *dst) {
    const int ns = (int)pl.slots.size();
    std::vector<int64_t> e(64, 0);
    for (int64_t r = rlo; r < rhi; ++r) e[r - rlo] = ptr[r];
    for (const auto &w : pl.wins) {
        const int64_t cb = round16((int64_t)w.chunks * 8);
        uint16_t *tab = reinterpret_cast<uint16_t *>(dst);
        uint16_t *code = reinterpret_cast<uint16_t *>(dst + TAB_BYTES);
        T *v = reinterpret_cast<T *>(dst + TAB_BYTES + cb);
        std::fill(dst, dst + win_bytes(w.chunks, sizeof(T)), 0);
        int64_t pos = 0;
        for (int r = 0; r < 64; ++r) {
            tab[r] = (uint16_t)(pos / CH);
            if (rlo + r < rhi) {
                for (int s = w.s0; s < w.s0 + w.ns; ++s) {
                    for (int c = 0; c < pl.cnt[(size_t)r * ns + s]; ++c) {
                        const int64_t x = e[r]++;
                        code[pos] = (uint16_t)(((s - w.s0) << 6) | (idx[x] & 63));
                        v[pos] = val[x];
                        ++pos;
                    }
                }
            }
            while (pos % CH) {
                code[pos] = (uint16_t)(ws * 64);   // the zero row
                v[pos] = T(0);
                ++pos;
            }
        }
        tab[64] = (uint16_t)(pos / CH);
        dst += win_bytes(w.chunks, sizeof(T));
    }
}

template <typename T>
int build_windows(lobpcg_ctx *ctx, const int64_t *rp, const int32_t *ci, const T *val, const int64_t *cp,
                  const int32_t *ri, const T *cv, hipStream_t s) {
    const int64_t n = ctx->n, NT = (n + 63) / 64;
    const int esz = (int)sizeof(T);
    // window size: 8 blocks of X (16 KB at k = 8 in FP32) for FP32, 4 for FP64,
    // and about 320 chunk-padded entries per slot
    const int ws = esz == 4 ? LOBPCG_TILE_WS : std::max(1, LOBPCG_TILE_WS / 2);
    const int64_t ecap = (int64_t)ws * LOBPCG_TILE_ECAP;
    unsigned hw = std::thread::hardware_concurrency();
    const int nth = (int)std::max(1u, std::min(16u, hw ? hw : 1u));
    auto parallel = [&](auto &&fn) {
        std::vector<std::thread> th;
        for (int t = 0; t < nth; ++t) th.emplace_back(fn, t);
        for (auto &x : th) x.join();
    };
    const int64_t *ptrs[2] = {rp, cp};
    const int32_t *idxs[2] = {ci, ri};
    const T *vals[2] = {val, cv};

    if (ctx->format_request == LOBPCG_FORMAT_AUTO) {
        // tiles only pay when each staged block serves enough entries: decide on
        // an evenly spaced sample of tile-rows (mean entries per touched tile >= 64;
        // measured: random_sym 20k, 20 per touched tile, CSR 31 us and tiled 107 us
        // per product; random_sym 1k, 358, 13 us and 16 us, both latency; tiled_2m's
        // recipe at n = 1.28e5, 267, 546 us and 112 us)
        const int64_t step = std::max<int64_t>(1, NT / 512);
        std::vector<int64_t> ent(nth, 0), sl(nth, 0);
        parallel([&](int t) {
            ViewPlan pl;
            for (int64_t I = t * step; I < NT; I += step * nth)
                for (int v = 0; v < 2; ++v) {
                    const int64_t lo = I * 64, hi = std::min<int64_t>(n, lo + 64);
                    pl.slots.clear();
                    for (int64_t r = lo; r < hi; ++r)
                        for (int64_t e = ptrs[v][r]; e < ptrs[v][r + 1]; ++e) pl.slots.push_back(idxs[v][e] >> 6);
                    ent[t] += (int64_t)pl.slots.size();
                    std::sort(pl.slots.begin(), pl.slots.end());
                    sl[t] += std::unique(pl.slots.begin(), pl.slots.end()) - pl.slots.begin();
                }
        });
        int64_t te = 0, ts = 0;
        for (int t = 0; t < nth; ++t) { te += ent[t]; ts += sl[t]; }
        if (ts == 0 || te < 64 * ts) return LOBPCG_OK;   // keep the CSR format
    }

    // pass 1: sizes of every tile-row and view (slots, windows, bytes)
    struct Size { int64_t bytes = 0, ent = 0; int32_t slots = 0, wins = 0, emax = 0; };
    std::vector<Size> sz((size_t)NT * 2);
    parallel([&](int t) {
        ViewPlan pl;
        for (int64_t I = t; I < NT; I += nth)
            for (int v = 0; v < 2; ++v) {
                const int64_t lo = I * 64, hi = std::min<int64_t>(n, lo + 64);
                plan_view(lo, hi, ptrs[v], idxs[v], ws, ecap, pl);
                Size &z = sz[(size_t)I * 2 + v];
                z.slots = (int32_t)pl.slots.size();
                z.wins = (int32_t)pl.wins.size();
                for (const auto &w : pl.wins) {
                    z.bytes += win_bytes(w.chunks, esz);
                    z.ent += (int64_t)w.chunks * CH;
                    z.emax = std::max(z.emax, w.chunks * CH);
                }
            }
    });
    std::vector<int64_t> boff((size_t)NT * 2 + 1, 0);   // byte offset of each (tile-row, view)
    std::vector<int32_t> wbeg(NT + 1, 0), soff((size_t)NT * 2 + 1, 0);
    int emax = CH;
    int64_t nent = 0;
    for (int64_t I = 0; I < NT; ++I) {
        wbeg[I + 1] = wbeg[I];
        for (int v = 0; v < 2; ++v) {
            const size_t q = (size_t)I * 2 + v;
            boff[q + 1] = boff[q] + sz[q].bytes;
            soff[q + 1] = soff[q] + sz[q].slots;
            wbeg[I + 1] += sz[q].wins;
            emax = std::max(emax, (int)sz[q].emax);
            nent += sz[q].ent;
        }
    }
    sz.clear();
    sz.shrink_to_fit();
    if (emax > 65535 * CH) return set_err(ctx, LOBPCG_EUNSUPPORTED, "tiled format: window too large");
    const int64_t nwin = wbeg[NT], nbytes = boff[(size_t)NT * 2], nslots = soff[(size_t)NT * 2];
    // pass 2: the same plans again, written out as window blocks, descriptors and slot lists
    std::vector<char> data(std::max<int64_t>(nbytes, 16));
    std::vector<int64_t> woff(nwin + 1);
    std::vector<int2> wdesc(std::max<int64_t>(nwin, 1));
    std::vector<int32_t> list(std::max<int64_t>(nslots, 1));
    parallel([&](int t) {
        ViewPlan pl;
        for (int64_t I = t; I < NT; I += nth) {
            int64_t w = wbeg[I];
            for (int v = 0; v < 2; ++v) {
                const size_t q = (size_t)I * 2 + v;
                const int64_t lo = I * 64, hi = std::min<int64_t>(n, lo + 64);
                plan_view(lo, hi, ptrs[v], idxs[v], ws, ecap, pl);
                std::copy(pl.slots.begin(), pl.slots.end(), list.begin() + soff[q]);
                int64_t b = boff[q];
                for (const auto &win : pl.wins) {
                    woff[w] = b;
                    wdesc[w] = make_int2(soff[q] + win.s0, win.ns);
                    b += win_bytes(win.chunks, esz);
                    ++w;
                }
                write_view<T>(lo, hi, ptrs[v], idxs[v], vals[v], ws, pl, data.data() + boff[q]);
            }
        }
    });
    woff[nwin] = nbytes;

    TiledFormat &tf = ctx->tiled;
    HIP_TRY(ctx, hipMalloc((void **)&tf.data, data.size()));
    HIP_TRY(ctx, hipMalloc((void **)&tf.woff, woff.size() * sizeof(int64_t)));
    HIP_TRY(ctx, hipMalloc((void **)&tf.wdesc, wdesc.size() * sizeof(int2)));
    HIP_TRY(ctx, hipMalloc((void **)&tf.wbeg, wbeg.size() * sizeof(int32_t)));
    HIP_TRY(ctx, hipMalloc((void **)&tf.list, list.size() * sizeof(int32_t)));
    HIP_TRY(ctx, hipMemcpyAsync(tf.data, data.data(), data.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(tf.woff, woff.data(), woff.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(tf.wdesc, wdesc.data(), wdesc.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(tf.wbeg, wbeg.data(), wbeg.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipMemcpyAsync(tf.list, list.data(), list.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    tf.ntilerows = NT;
    tf.nwin = nwin;
    tf.nbytes = nbytes;
    tf.nslots = nslots;
    tf.nent = nent;
    tf.ws = ws;
    tf.emax = emax;
    ctx->format = LOBPCG_FORMAT_TILED;
    return LOBPCG_OK;
}

template <typename T, int KP, bool FULL>
int launch_window(lobpcg_ctx *ctx, const T *X, T *Y, int k, hipStream_t s) {
    const TiledFormat &tf = ctx->tiled;
    const int esz = (int)sizeof(T);
    if (FULL && tf.ws * (KP * esz / 16) > MAXJ * NWAVE)
        return set_err(ctx, LOBPCG_EUNSUPPORTED, "tiled product: window of %d blocks too wide", tf.ws);
    const int lds = x_bytes(tf.ws, KP, esz) + m_bytes(tf.emax, esz);
    if (lds > 160 * 1024) return set_err(ctx, LOBPCG_EUNSUPPORTED, "tiled product: %d bytes of LDS", lds);
    static bool attr = false;   // one per instantiation
    if (!attr) {
        HIP_TRY(ctx, hipFuncSetAttribute((const void *)spmm_window_kernel<T, KP, FULL>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        attr = true;
    }
    spmm_window_kernel<T, KP, FULL><<<(int)tf.ntilerows, THREADS, lds, s>>>(
        ctx->n, k, tf.ws, tf.emax, tf.data, tf.woff, tf.wdesc, tf.wbeg, tf.list, (const T *)ctx->diag, X, Y);
    return LOBPCG_OK;
}

template <typename T, int KP>
int launch_width(lobpcg_ctx *ctx, const T *X, T *Y, int k, hipStream_t s) {
    if (k == KP) return launch_window<T, KP, true>(ctx, X, Y, k, s);
    return launch_window<T, KP, false>(ctx, X, Y, k, s);
}

template <typename T>
int spmm_tiled_t(lobpcg_ctx *ctx, const T *X, T *Y, int k, hipStream_t s) {
    if (k <= 4) return launch_width<T, 4>(ctx, X, Y, k, s);
    if (k <= 8) return launch_width<T, 8>(ctx, X, Y, k, s);
    return launch_width<T, 16>(ctx, X, Y, k, s);
}

}  // namespace

int build_tiled_format(lobpcg_ctx *ctx, const int64_t *rp, const int32_t *ci, const void *val, const int64_t *cp,
                       const int32_t *ri, const void *cv, hipStream_t s) {
    if (ctx->dtype == LOBPCG_F32)
        return build_windows<float>(ctx, rp, ci, (const float *)val, cp, ri, (const float *)cv, s);
    return build_windows<double>(ctx, rp, ci, (const double *)val, cp, ri, (const double *)cv, s);
}

int spmm_tiled(lobpcg_ctx *ctx, const void *X, void *Y, int k, hipStream_t s) {
    if (ctx->dtype == LOBPCG_F32) return spmm_tiled_t<float>(ctx, (const float *)X, (float *)Y, k, s);
    return spmm_tiled_t<double>(ctx, (const double *)X, (double *)Y, k, s);
}
