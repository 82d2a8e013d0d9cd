// Tall-skinny Gram products G = A^T B on the matrix cores.
//
// The projected matrices of the Rayleigh-Ritz step (eqs. go, Glower) and the
// Cholesky QR Gram W^T W (Section 3.5) are products of n x k blocks.  The
// row dimension n is the MFMA reduction (K) dimension: each wavefront walks a
// strided set of 16-row slabs and accumulates 16x16 output tiles in MFMA
// accumulators; the four wavefronts of a workgroup are summed in LDS and each
// workgroup writes one FP64 partial, which a second kernel sums in a fixed
// order (deterministic).
//
// Precisions: FP64 (v_mfma_f64_16x16x4f64), FP32 (v_mfma_f32_16x16x4f32), and
// split-BF16 "x3" for FP32 inputs: a = a0 + a1 with a0 = bf16(a),
// a1 = bf16(a - a0), and a.b ~ a0.b0 + a0.b1 + a1.b0 (v_mfma_f32_16x16x16bf16_1k);
// "x6" splits into three terms (a2 = bf16(a - a0 - a1): 24 significant bits,
// FP32's) and keeps the six products with i + j <= 2, summed per 16-row slab
// in FP32 and across slabs in FP64.
//
// MFMA operand layout used (16x16xK, wave64): lane l supplies
// A[i = l % 16][kk] and B[kk][j = l % 16] for the kk owned by lane group l / 16;
// the four outputs of lane l are D[4 * (l / 16) + r][l % 16], r = 0..3, for the
// FP32-accumulating instructions and D[l / 16 + 4 * r][l % 16] for the FP64 one.
#include <mutex>

#include "internal.hpp"

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

constexpr int GRAM_THREADS = 256;
constexpr int GRAM_WAVES = GRAM_THREADS / LOBPCG_WAVE;

__device__ inline unsigned short bf16_rne(float x) {
    unsigned int u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

enum Mode { M_F64 = 0, M_F32 = 1, M_BF16X3 = 2, M_BF16X6 = 3 };

struct GramDev {
    const void *a[4];
    const void *b[6];
    int na, nb, wa, wb;
    int64_t n;
    // output placement: row of A-list column m, column of B-list column j (-1: not
    // written) in a partial of out_rows x out_cols
    short arow[64];
    short bcol[96];
    int out_rows, out_cols;
};

// per-lane column pointer for a 16-wide tile of a concatenated block list
template <typename TI>
__device__ inline const TI *col_ptr(const void *const *blocks, int nblocks, int w, int m) {
    if (m >= nblocks * w) return nullptr;
    return (const TI *)blocks[m / w] + (m % w);
}

// SKIP: bit i * NT + j set = output tile (i, j) not computed (its blocks are
// not needed by the caller).  SYM: the B list is the A list (MT == NT), whose
// loaded values serve as both operands.
template <typename TI, int MODE, int MT, int NT, int SKIP = 0, bool SYM = false>
__global__ __launch_bounds__(GRAM_THREADS) void gram_partial_kernel(GramDev g, double *__restrict__ partial) {
    static_assert(!SYM || MT == NT, "a symmetric Gram has square tiles");
    using Acc = typename std::conditional<MODE == M_F64 || MODE == M_BF16X6, f64x4, f32x4>::type;
    using AccS = typename std::conditional<MODE == M_F64, double, float>::type;
    const int lane = threadIdx.x % LOBPCG_WAVE;
    const int wave = threadIdx.x / LOBPCG_WAVE;
    const int li = lane % 16, lg = lane / 16;
    const int KA = g.na * g.wa, KB = g.nb * g.wb;

    const TI *pa[MT];
    const TI *pb[NT];
#pragma unroll
    for (int t = 0; t < MT; ++t) pa[t] = col_ptr<TI>(g.a, g.na, g.wa, 16 * t + li);
#pragma unroll
    for (int t = 0; t < NT; ++t) pb[t] = col_ptr<TI>(g.b, g.nb, g.wb, 16 * t + li);

    Acc acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = Acc{0, 0, 0, 0};

    // the 4 rows of a 16-row slab this lane supplies: r0 + 4t + lg (K = 4 per
    // instruction, four instructions) or r0 + 4lg + t (BF16, K = 16)
    auto row_of = [&](int64_t r0, int t) -> int64_t {
        return MODE == M_BF16X3 || MODE == M_BF16X6 ? r0 + 4 * lg + t : r0 + 4 * t + lg;
    };
    auto load = [&](int64_t slab, TI (&fa)[4][MT], TI (&fb)[4][NT]) {
        const int64_t r0 = slab * 16;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t r = row_of(r0, t);
            const bool in = r < g.n;
#pragma unroll
            for (int i = 0; i < MT; ++i) fa[t][i] = (pa[i] && in) ? pa[i][r * g.wa] : TI(0);
            if constexpr (!SYM) {
#pragma unroll
                for (int j = 0; j < NT; ++j) fb[t][j] = (pb[j] && in) ? pb[j][r * g.wb] : TI(0);
            }
        }
    };
    auto compute = [&](const TI (&fa)[4][MT], const TI (&fb)[4][NT]) {
        if constexpr (MODE == M_BF16X6) {
            s16x4 a0[MT], a1[MT], a2[MT], b0[NT], b1[NT], b2[NT];
            // v = h0 + h1 + h2 (BF16 each, round to nearest even at every step)
            auto split3 = [](float v, s16x4 &h0, s16x4 &h1, s16x4 &h2, int t) {
                const unsigned short u0 = bf16_rne(v);
                const float r1 = v - bf16_to_f32(u0);
                const unsigned short u1 = bf16_rne(r1);
                h0[t] = (short)u0;
                h1[t] = (short)u1;
                h2[t] = (short)bf16_rne(r1 - bf16_to_f32(u1));
            };
#pragma unroll
            for (int t = 0; t < 4; ++t) {
#pragma unroll
                for (int i = 0; i < MT; ++i) split3((float)fa[t][i], a0[i], a1[i], a2[i], t);
#pragma unroll
                for (int j = 0; j < NT; ++j) split3((float)fb[t][j], b0[j], b1[j], b2[j], t);
            }
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    if ((SKIP >> (i * NT + j)) & 1) continue;
                    // smallest terms first; this slab's sum in FP32, then into FP64
                    f32x4 t4 = {0.0f, 0.0f, 0.0f, 0.0f};
                    t4 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2[i], b0[j], t4, 0, 0, 0);
                    t4 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[i], b1[j], t4, 0, 0, 0);
                    t4 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0[i], b2[j], t4, 0, 0, 0);
                    t4 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[i], b0[j], t4, 0, 0, 0);
                    t4 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0[i], b1[j], t4, 0, 0, 0);
                    t4 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0[i], b0[j], t4, 0, 0, 0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[i][j][r] += (double)t4[r];
                }
        } else if constexpr (MODE == M_BF16X3) {
            s16x4 a0[MT], a1[MT], b0[NT], b1[NT];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
#pragma unroll
                for (int i = 0; i < MT; ++i) {
                    const float v = (float)fa[t][i];
                    const unsigned short h = bf16_rne(v);
                    a0[i][t] = (short)h;
                    a1[i][t] = (short)bf16_rne(v - bf16_to_f32(h));
                }
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    const float v = (float)fb[t][j];
                    const unsigned short h = bf16_rne(v);
                    b0[j][t] = (short)h;
                    b1[j][t] = (short)bf16_rne(v - bf16_to_f32(h));
                }
            }
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    if ((SKIP >> (i * NT + j)) & 1) continue;
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[i], b0[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0[i], b1[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0[i], b0[j], acc[i][j], 0, 0, 0);
                }
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int i = 0; i < MT; ++i)
#pragma unroll
                    for (int j = 0; j < NT; ++j) {
                        if ((SKIP >> (i * NT + j)) & 1) continue;
                        if constexpr (MODE == M_F64)
                            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64((AccS)fa[t][i], (AccS)fb[t][j],
                                                                             acc[i][j], 0, 0, 0);
                        else
                            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32((AccS)fa[t][i], (AccS)fb[t][j],
                                                                             acc[i][j], 0, 0, 0);
                    }
        }
    };

    // software pipeline: the loads of the next PF slabs are in flight during this
    // slab's MFMAs (FP32 inputs: two, four for a single 16 x 16 tile; one slab
    // of MFMAs is shorter than a memory round trip; FP64 inputs keep one, their
    // registers would spill)
    const int64_t nslab = (g.n + 15) / 16;
    const int64_t wave_id = (int64_t)blockIdx.x * GRAM_WAVES + wave;
    const int64_t nwaves = (int64_t)gridDim.x * GRAM_WAVES;
    constexpr int PF = sizeof(TI) == 4 ? (MT * NT == 1 ? 4 : 2) : 1;
    TI qa[PF + 1][4][MT], qb[PF + 1][4][NT];
    auto load_or_zero = [&](int64_t sl, TI (&fa)[4][MT], TI (&fb)[4][NT]) {
        if (sl < nslab) {
            load(sl, fa, fb);
        } else {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
#pragma unroll
                for (int i = 0; i < MT; ++i) fa[t][i] = TI(0);
                if constexpr (!SYM) {
#pragma unroll
                    for (int j = 0; j < NT; ++j) fb[t][j] = TI(0);
                }
            }
        }
    };
#pragma unroll
    for (int p = 0; p < PF; ++p) load_or_zero(wave_id + p * nwaves, qa[p], qb[p]);
    for (int64_t slab = wave_id; slab < nslab; slab += nwaves) {
        load_or_zero(slab + PF * nwaves, qa[PF], qb[PF]);
        if constexpr (SYM)
            compute(qa[0], qa[0]);
        else
            compute(qa[0], qb[0]);
#pragma unroll
        for (int p = 0; p < PF; ++p)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
#pragma unroll
                for (int i = 0; i < MT; ++i) qa[p][t][i] = qa[p + 1][t][i];
                if constexpr (!SYM) {
#pragma unroll
                    for (int j = 0; j < NT; ++j) qb[p][t][j] = qb[p + 1][t][j];
                }
            }
    }

    // sum the wavefronts of this workgroup in LDS (FP64), one wave at a time
    __shared__ double red[MT * NT * 4 * LOBPCG_WAVE];
    for (int w = 0; w < GRAM_WAVES; ++w) {
        if (wave == w) {
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        int idx = ((i * NT + j) * 4 + r) * LOBPCG_WAVE + lane;
                        double v = (double)acc[i][j][r];
                        red[idx] = (w == 0) ? v : red[idx] + v;
                    }
        }
        __syncthreads();
    }
    double *out = partial + (size_t)blockIdx.x * g.out_rows * g.out_cols;
    for (int e = threadIdx.x; e < MT * NT * 4 * LOBPCG_WAVE; e += GRAM_THREADS) {
        int l = e % LOBPCG_WAVE, r = (e / LOBPCG_WAVE) % 4, tile = e / (4 * LOBPCG_WAVE);
        int i = tile / NT, j = tile % NT;
        if ((SKIP >> tile) & 1) continue;
        // output rows of lane l: FP32 MFMA holds 4*(l/16)+r, FP64 MFMA holds (l/16)+4*r
        int m = MODE == M_F64 ? 16 * i + (l / 16) + 4 * r : 16 * i + 4 * (l / 16) + r;
        int nn = 16 * j + (l % 16);
        if (m < KA && nn < KB) {
            const int om = g.arow[m], on = g.bcol[nn];
            if (om >= 0 && on >= 0) out[om * g.out_cols + on] = red[e];
        }
    }
}

// Stage 1: block (x, y) sums partials y*RB .. y*RB+RB-1 of outputs x*64 ..
// x*64+63 (four wavefronts split the partials, lanes over outputs); stage 2
// sums the stage-1 rows.  Fixed order throughout: deterministic.
constexpr int RB = 64;
__global__ __launch_bounds__(256) void gram_reduce1_kernel(const double *__restrict__ partial, int nparts, int count,
                                                           double *__restrict__ stage) {
    __shared__ double red[4][64];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int e = blockIdx.x * 64 + lane;
    const int p0 = blockIdx.y * RB;
    double s = 0.0;
    if (e < count)
        for (int p = p0 + wave; p < min(p0 + RB, nparts); p += 4) s += partial[(size_t)p * count + e];
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && e < count)
        stage[(size_t)blockIdx.y * count + e] = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
}

__global__ void gram_reduce2_kernel(const double *__restrict__ stage, int nstage, int count,
                                    double *__restrict__ out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    double s = 0.0;
    for (int p = 0; p < nstage; ++p) s += stage[(size_t)p * count + e];
    out[e] = s;
}

template <typename TI, int MODE>
int dispatch_tiles(int MT, int NT, int grid, const GramDev &g, double *partial, hipStream_t s) {
    // the same block list on both sides (a Gram of the form S^T S)
    bool sym = MT == NT && g.na == g.nb && g.wa == g.wb;
    for (int i = 0; sym && i < g.na; ++i) sym = g.a[i] == g.b[i];
    if (sym) {
        if (MT == 1) { gram_partial_kernel<TI, MODE, 1, 1, 0, true><<<grid, GRAM_THREADS, 0, s>>>(g, partial); return LOBPCG_OK; }
        if (MT == 2) { gram_partial_kernel<TI, MODE, 2, 2, 0, true><<<grid, GRAM_THREADS, 0, s>>>(g, partial); return LOBPCG_OK; }
    }
#define GRAM_CASE(a, b)                                                                        \
    if (MT == a && NT == b) {                                                                  \
        gram_partial_kernel<TI, MODE, a, b><<<grid, GRAM_THREADS, 0, s>>>(g, partial);         \
        return LOBPCG_OK;                                                                      \
    }
    GRAM_CASE(1, 1) GRAM_CASE(1, 2) GRAM_CASE(1, 3) GRAM_CASE(1, 4) GRAM_CASE(1, 5) GRAM_CASE(1, 6)
    GRAM_CASE(2, 1) GRAM_CASE(2, 2) GRAM_CASE(2, 3) GRAM_CASE(2, 4) GRAM_CASE(2, 5) GRAM_CASE(2, 6)
    GRAM_CASE(3, 1) GRAM_CASE(3, 2) GRAM_CASE(3, 3) GRAM_CASE(3, 4) GRAM_CASE(3, 5) GRAM_CASE(3, 6)
#undef GRAM_CASE
    return LOBPCG_EUNSUPPORTED;
}

}  // namespace

int launch_gram(lobpcg_ctx *ctx, const GramArgs &ga, int prec, double *out, hipStream_t s) {
    const int KA = ga.na * ga.wa, KB = ga.nb * ga.wb;
    if (KA < 1 || KB < 1 || KA > 48 || KB > 96) return set_err(ctx, LOBPCG_EINVAL, "gram: %dx%d too large", KA, KB);
    const int MT = (KA + 15) / 16, NT = (KB + 15) / 16;
    GramDev g;
    for (int i = 0; i < 4; ++i) g.a[i] = i < ga.na ? ga.a[i] : nullptr;
    for (int i = 0; i < 6; ++i) g.b[i] = i < ga.nb ? ga.b[i] : nullptr;
    g.na = ga.na; g.nb = ga.nb; g.wa = ga.wa; g.wb = ga.wb; g.n = ctx->n;
    for (int m = 0; m < 64; ++m) g.arow[m] = m < KA ? m : -1;
    for (int m = 0; m < 96; ++m) g.bcol[m] = m < KB ? m : -1;
    g.out_rows = KA;
    g.out_cols = KB;
    const int64_t nslab = (ctx->n + 15) / 16;
    // at least 4 slabs per wavefront (amortises the partial), at most one partial per slot
    const int grid = (int)std::min<int64_t>(ctx->gram_max_wg, std::max<int64_t>(1, (nslab + 4 * GRAM_WAVES - 1) / (4 * GRAM_WAVES)));
    int rc;
    if (prec == LOBPCG_GRAM_AUTO) prec = ctx->gram;
    if (ctx->dtype == LOBPCG_F64) {
        if (prec != LOBPCG_GRAM_F64) return set_err(ctx, LOBPCG_EINVAL, "gram: FP64 context needs GRAM_F64");
        rc = dispatch_tiles<double, M_F64>(MT, NT, grid, g, ctx->gram_partial, s);
    } else if (prec == LOBPCG_GRAM_F64) {
        rc = dispatch_tiles<float, M_F64>(MT, NT, grid, g, ctx->gram_partial, s);
    } else if (prec == LOBPCG_GRAM_F32) {
        rc = dispatch_tiles<float, M_F32>(MT, NT, grid, g, ctx->gram_partial, s);
    } else if (prec == LOBPCG_GRAM_BF16X3) {
        rc = dispatch_tiles<float, M_BF16X3>(MT, NT, grid, g, ctx->gram_partial, s);
    } else if (prec == LOBPCG_GRAM_BF16X6) {
        rc = dispatch_tiles<float, M_BF16X6>(MT, NT, grid, g, ctx->gram_partial, s);
    } else {
        return set_err(ctx, LOBPCG_EINVAL, "gram: bad precision %d", prec);
    }
    if (rc != LOBPCG_OK) return set_err(ctx, rc, "gram: no kernel for %dx%d tiles", MT, NT);
    const int count = KA * KB;
    const int nstage = ceil_div(grid, RB);
    // stage-1 rows live after the partial slots (the allocation holds gram_max_wg / RB extra slots)
    double *stage = ctx->gram_partial + (size_t)ctx->gram_max_wg * 48 * 96;
    gram_reduce1_kernel<<<dim3(ceil_div(count, 64), nstage), 256, 0, s>>>(ctx->gram_partial, grid, count, stage);
    gram_reduce2_kernel<<<ceil_div(count, 256), 256, 0, s>>>(stage, nstage, count, out);
    return LOBPCG_OK;
}

// The Rayleigh-Ritz Gram [X W P]^T [X W P HX HW HP] for k = 8 reads only the
// blocks of eq. Glower (the lower blocks and the diagonal blocks of both
// matrices).  With the rows ordered [W P | X P] and the columns
// [X HX | W HW | P HP], the 16 x 16 tiles ([W P], [P HP]) and ([X P], [W HW])
// hold no needed block and are skipped: 4 tile products per 16-row slab
// instead of 6.  The output keeps the layout of launch_gram (rows [X W P],
// columns [X W P HX HW HP]); the blocks of the skipped tiles are not written.
int launch_gram_rr8(lobpcg_ctx *ctx, const void *X, const void *W, const void *P, const void *HX,
                    const void *HW, const void *HP, int prec, double *out, hipStream_t s) {
    constexpr int k = 8;
    GramDev g;
    g.a[0] = W; g.a[1] = P; g.a[2] = X; g.a[3] = P;
    g.b[0] = X; g.b[1] = HX; g.b[2] = W; g.b[3] = HW; g.b[4] = P; g.b[5] = HP;
    g.na = 4; g.nb = 6; g.wa = g.wb = k; g.n = ctx->n;
    const int arow_blk[4] = {1, 2, 0, 2};            // W P X P -> output row blocks
    const int bcol_blk[6] = {0, 3, 1, 4, 2, 5};      // X HX W HW P HP -> output column blocks
    for (int m = 0; m < 64; ++m) g.arow[m] = m < 4 * k ? (short)(arow_blk[m / k] * k + m % k) : -1;
    for (int m = 0; m < 96; ++m) g.bcol[m] = m < 6 * k ? (short)(bcol_blk[m / k] * k + m % k) : -1;
    g.out_rows = 3 * k;
    g.out_cols = 6 * k;
    const int64_t nslab = (ctx->n + 15) / 16;
    const int grid = (int)std::min<int64_t>(ctx->gram_max_wg, std::max<int64_t>(1, (nslab + 4 * GRAM_WAVES - 1) / (4 * GRAM_WAVES)));
    constexpr int SKIP = (1 << (0 * 3 + 2)) | (1 << (1 * 3 + 1));
    if (prec == LOBPCG_GRAM_AUTO) prec = ctx->gram;
    if (ctx->dtype == LOBPCG_F64) {
        if (prec != LOBPCG_GRAM_F64) return set_err(ctx, LOBPCG_EINVAL, "gram: FP64 context needs GRAM_F64");
        gram_partial_kernel<double, M_F64, 2, 3, SKIP><<<grid, GRAM_THREADS, 0, s>>>(g, ctx->gram_partial);
    } else if (prec == LOBPCG_GRAM_F64) {
        gram_partial_kernel<float, M_F64, 2, 3, SKIP><<<grid, GRAM_THREADS, 0, s>>>(g, ctx->gram_partial);
    } else if (prec == LOBPCG_GRAM_F32) {
        gram_partial_kernel<float, M_F32, 2, 3, SKIP><<<grid, GRAM_THREADS, 0, s>>>(g, ctx->gram_partial);
    } else if (prec == LOBPCG_GRAM_BF16X3) {
        gram_partial_kernel<float, M_BF16X3, 2, 3, SKIP><<<grid, GRAM_THREADS, 0, s>>>(g, ctx->gram_partial);
    } else if (prec == LOBPCG_GRAM_BF16X6) {
        gram_partial_kernel<float, M_BF16X6, 2, 3, SKIP><<<grid, GRAM_THREADS, 0, s>>>(g, ctx->gram_partial);
    } else {
        return set_err(ctx, LOBPCG_EINVAL, "gram: bad precision %d", prec);
    }
    const int count = 3 * k * 6 * k;
    const int nstage = ceil_div(grid, RB);
    double *stage = ctx->gram_partial + (size_t)ctx->gram_max_wg * 48 * 96;
    gram_reduce1_kernel<<<dim3(ceil_div(count, 64), nstage), 256, 0, s>>>(ctx->gram_partial, grid, count, stage);
    gram_reduce2_kernel<<<ceil_div(count, 256), 256, 0, s>>>(stage, nstage, count, out);
    return LOBPCG_OK;
}

extern "C" int lobpcg_gram(lobpcg_ctx *ctx, const void *A, int ka, const void *B, int kb, double *G, int prec,
                           void *stream) {
    if (!ctx) return LOBPCG_EINVAL;
    if (!A || !B || !G) return set_err(ctx, LOBPCG_EINVAL, "gram: null pointer");
    if (ka < 1 || kb < 1 || ka > 48 || kb > 48) return set_err(ctx, LOBPCG_EINVAL, "gram: ka, kb must be in [1,48]");
    if (prec < LOBPCG_GRAM_AUTO || prec > LOBPCG_GRAM_BF16X6) return set_err(ctx, LOBPCG_EINVAL, "gram: bad precision");
    if ((prec == LOBPCG_GRAM_BF16X3 || prec == LOBPCG_GRAM_BF16X6) && ctx->dtype != LOBPCG_F32)
        return set_err(ctx, LOBPCG_EINVAL, "gram: split-BF16 products need an FP32 context");
    if (ctx->dtype == LOBPCG_F64 && (prec == LOBPCG_GRAM_F32))
        return set_err(ctx, LOBPCG_EINVAL, "gram: FP32 Gram of FP64 blocks is not offered");
    GramArgs ga{};
    ga.a[0] = A;
    ga.b[0] = B;
    ga.na = 1;
    ga.nb = 1;
    ga.wa = ka;
    ga.wb = kb;
    hipStream_t s = (hipStream_t)stream;
    int rc = launch_gram(ctx, ga, prec, G, s);
    if (rc != LOBPCG_OK) return rc;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_err(ctx, LOBPCG_EHIP, "gram launch: %s", hipGetErrorString(e));
    return LOBPCG_OK;
}

// ---------------------------------------------------------------------------
// Context-free Gram product that allocates nothing: its workgroup partials and
// reduction rows live in a file-scope device array, one copy per GPU, held
// until the process ends.  At most NOALLOC_MAX_WG workgroups (each walks as
// many 16-row slabs as n needs) and ka, kb <= 48, so the array is
// (NOALLOC_MAX_WG + NOALLOC_MAX_WG / RB + 1) * 48 * 48 doubles = 4.8 MB.
namespace {
constexpr int NOALLOC_MAX_WG = 256;
constexpr int NOALLOC_MAX_K = 48;
constexpr size_t NOALLOC_SLOT = (size_t)NOALLOC_MAX_K * NOALLOC_MAX_K;
constexpr size_t NOALLOC_DOUBLES = (size_t)(NOALLOC_MAX_WG + NOALLOC_MAX_WG / RB + 1) * NOALLOC_SLOT;
__device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int NOALLOC_MAX_DEV = 64;
std::mutex noalloc_mu;
double *noalloc_ptr[NOALLOC_MAX_DEV] = {};

// the device address of this GPU's copy of `scratch` (looked up once per device,
// with that device current): host code passes this pointer, never the symbol
int scratch_for_current_device(double **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LOBPCG_EHIP;
    if (dev < 0 || dev >= NOALLOC_MAX_DEV) return LOBPCG_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LOBPCG_EHIP;
        noalloc_ptr[dev] = (double *)p;
    }
    *out = noalloc_ptr[dev];
    return LOBPCG_OK;
}
}  // namespace

extern "C" int lobpcg_gram_noalloc(const void *A, int ka, const void *B, int kb, int64_t n, int dtype, double *G,
                                   int prec, void *stream) {
    if (!A || !B || !G || n < 1) return LOBPCG_EINVAL;
    if (ka < 1 || kb < 1) return LOBPCG_EINVAL;
    if (ka > NOALLOC_MAX_K || kb > NOALLOC_MAX_K) return LOBPCG_EUNSUPPORTED;   // beyond the static scratch
    if (dtype != LOBPCG_F32 && dtype != LOBPCG_F64) return LOBPCG_EINVAL;
    if (prec < LOBPCG_GRAM_AUTO || prec > LOBPCG_GRAM_BF16X6) return LOBPCG_EINVAL;
    if (prec == LOBPCG_GRAM_AUTO) prec = LOBPCG_GRAM_F64;
    if (dtype == LOBPCG_F64 && prec != LOBPCG_GRAM_F64) return LOBPCG_EINVAL;
    double *scr = nullptr;
    int rc = scratch_for_current_device(&scr);
    if (rc != LOBPCG_OK) return rc;
    GramDev g;
    for (int i = 0; i < 4; ++i) g.a[i] = nullptr;
    for (int i = 0; i < 6; ++i) g.b[i] = nullptr;
    g.a[0] = A;
    g.b[0] = B;
    g.na = g.nb = 1;
    g.wa = ka;
    g.wb = kb;
    g.n = n;
    for (int m = 0; m < 64; ++m) g.arow[m] = m < ka ? m : -1;
    for (int m = 0; m < 96; ++m) g.bcol[m] = m < kb ? m : -1;
    g.out_rows = ka;
    g.out_cols = kb;
    const int MT = (ka + 15) / 16, NT = (kb + 15) / 16;
    const int64_t nslab = (n + 15) / 16;
    const int grid = (int)std::min<int64_t>(NOALLOC_MAX_WG, std::max<int64_t>(1, (nslab + 4 * GRAM_WAVES - 1) / (4 * GRAM_WAVES)));
    hipStream_t s = (hipStream_t)stream;
    if (dtype == LOBPCG_F64)
        rc = dispatch_tiles<double, M_F64>(MT, NT, grid, g, scr, s);
    else if (prec == LOBPCG_GRAM_F64)
        rc = dispatch_tiles<float, M_F64>(MT, NT, grid, g, scr, s);
    else if (prec == LOBPCG_GRAM_F32)
        rc = dispatch_tiles<float, M_F32>(MT, NT, grid, g, scr, s);
    else if (prec == LOBPCG_GRAM_BF16X3)
        rc = dispatch_tiles<float, M_BF16X3>(MT, NT, grid, g, scr, s);
    else
        rc = dispatch_tiles<float, M_BF16X6>(MT, NT, grid, g, scr, s);
    if (rc != LOBPCG_OK) return rc;
    const int count = ka * kb;
    const int nstage = ceil_div(grid, RB);
    double *stage = scr + (size_t)NOALLOC_MAX_WG * NOALLOC_SLOT;
    gram_reduce1_kernel<<<dim3(ceil_div(count, 64), nstage), 256, 0, s>>>(scr, grid, count, stage);
    gram_reduce2_kernel<<<ceil_div(count, 256), 256, 0, s>>>(stage, nstage, count, G);
    return hipGetLastError() == hipSuccess ? LOBPCG_OK : LOBPCG_EHIP;
}
