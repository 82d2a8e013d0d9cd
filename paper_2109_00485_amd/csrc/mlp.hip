// Learned preconditioner network 4 -> 64 -> 64 -> 1 (the preconditioner
// scale is exp(2 tanh(o / 2)) / s(d - sigma), sigma the diagonal step's shift).
//
// Inference (the preconditioner apply and lobpcg_mlp_forward) runs on the
// matrix cores, 16 samples per wavefront step, with both hidden layers
// computed transposed so that no data leaves the registers:
//   layer 1  a1^T (64 x 16) = W1 (64 x 4) z^T (4 x 16)   FP32 MFMA 16x16x4,
//            four 16-unit blocks, bias preloaded in the accumulator; lane l
//            ends up holding units 16nb + 4(l/16) + r of sample l%16;
//   layer 2  a2^T (64 x 16) = W2 (64 x 64) bf16(relu(a1))^T   BF16 MFMA
//            16x16x32 with FP32 accumulation; the K order of the contraction
//            is permuted (identically in both operands) so that the layer-1
//            output registers are the B operand as they are;
//   layer 3  o = w3 . relu(a2) + b3: 16 FMAs per lane and a reduction over
//            the four 16-lane groups.
// Training (loss, gradient, Adam) runs in FP32 on the vector units with the
// same roundings: forward and backward per sample, weight gradients as
// sample-batched outer products staged through LDS, FP64 reduction across
// workgroups.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <vector>

#include "internal.hpp"

int set_mlp_err(lobpcg_mlp *m, int code, const char *fmt, ...) {
    if (m) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        m->err = buf;
    }
    return code;
}

namespace {

constexpr int HID = LOBPCG_MLP_HID;
constexpr int NPARAM = LOBPCG_MLP_NPARAM;
constexpr int OFF_W1 = 0, OFF_B1 = 256, OFF_W2 = 320, OFF_B2 = 4416, OFF_W3 = 4480, OFF_B3 = 4544,
              OFF_MU = 4545, OFF_SIG = 4549;
static_assert(OFF_B3 + 1 == LOBPCG_MLP_NPARAM, "parameter blob layout");
static_assert(OFF_SIG + 4 == LOBPCG_MLP_NBLOB, "parameter blob layout");

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// round to the nearest BF16 (ties to even), returned as FP32
__device__ inline float bf16r(float x) { return (float)(__bf16)x; }

// ---------------------------------------------------------------------------
// matrix-core inference
// ---------------------------------------------------------------------------
constexpr int INF_THREADS = 256;

// The weights one lane holds for the whole kernel (c = lane % 16, g = lane / 16).
struct LaneWeights {
    float w1[4];       // W1[16nb + c][g]
    bf8 w2[4][2];      // W2[16vb + c][u(kb, g, t)]
    float b3;
    double mu, isg;    // standardisation of feature g
};

// The weights shared by the 16 lanes of a lane group, staged once per
// workgroup in LDS and read there on every step (in registers they would take
// 48 more per lane, one wave per SIMD less): [block][g].
struct GroupWeights {
    f4 b1[4][4];       // b1[16nb + 4g + r]
    f4 b2[4][4];       // b2[16vb + 4g + r]
    f4 w3[4][4];       // w3[16vb + 4g + r]
};

// hidden-1 unit paired with element t of lane group g in K block kb
__device__ inline int unit_of(int kb, int g, int t) { return 16 * (2 * kb + t / 4) + 4 * g + (t & 3); }

__device__ inline void load_lane_weights(LaneWeights &L, const float *__restrict__ P, int c, int g) {
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        L.w1[nb] = bf16r(P[OFF_W1 + (16 * nb + c) * 4 + g]);
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int t = 0; t < 8; ++t) L.w2[nb][kb][t] = (__bf16)P[OFF_W2 + (16 * nb + c) * HID + unit_of(kb, g, t)];
    }
    L.b3 = P[OFF_B3];
    L.mu = (double)P[OFF_MU + g];
    L.isg = 1.0 / (double)P[OFF_SIG + g];
}

// all threads of the workgroup call this (it ends with a barrier)
__device__ inline void stage_group_weights(GroupWeights &S, const float *__restrict__ P) {
    if (threadIdx.x < 64) {
        const int blk = threadIdx.x / 16, g = (threadIdx.x / 4) % 4, r = threadIdx.x % 4, u = 16 * blk + 4 * g + r;
        S.b1[blk][g][r] = P[OFF_B1 + u];
        S.b2[blk][g][r] = P[OFF_B2 + u];
        S.w3[blk][g][r] = bf16r(P[OFF_W3 + u]);
    }
    __syncthreads();
}

// relu as one integer max on the bit pattern: negative floats (sign bit set)
// compare below 0 (IEEE-mode fmaxf costs a NaN-quieting max as well)
__device__ inline float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));

// Network output for the 16 samples of one step; z is feature g of sample c.
// Every lane returns o of its sample c.  All 64 lanes must be active.  g is
// this lane's group, passed through an empty asm statement on every step by
// the callers so that the reads of S stay in the loop.
__device__ inline float mlp_step(const LaneWeights &L, const GroupWeights &S, int g, float z) {
    f4 a1[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) a1[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(L.w1[nb], z, S.b1[nb][g], 0, 0, 0);
    bf8 h[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
        // round pairs to BF16, then relu on the bit patterns, two per instruction:
        // rounding keeps the sign, so this equals rounding relu(a1) (a negative
        // value, -0 included, has its sign bit set and compares below 0 as an integer)
        const bf2 q0 = __builtin_convertvector(a1[2 * kb].xy, bf2), q1 = __builtin_convertvector(a1[2 * kb].zw, bf2);
        const bf2 q2 = __builtin_convertvector(a1[2 * kb + 1].xy, bf2), q3 = __builtin_convertvector(a1[2 * kb + 1].zw, bf2);
        const bf8 hp = {q0.x, q0.y, q1.x, q1.y, q2.x, q2.y, q3.x, q3.y};
        h[kb] = __builtin_bit_cast(bf8, __builtin_elementwise_max(__builtin_bit_cast(s16x8, hp), s16x8{}));
    }
    float p = 0.0f;
#pragma unroll
    for (int vb = 0; vb < 4; ++vb) {
        f4 a2 = S.b2[vb][g];
        a2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(L.w2[vb][0], h[0], a2, 0, 0, 0);
        a2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(L.w2[vb][1], h[1], a2, 0, 0, 0);
        const f4 w3 = S.w3[vb][g];
#pragma unroll
        for (int r = 0; r < 4; ++r) p = fmaf(w3[r], relu(a2[r]), p);
    }
    p += __shfl_xor(p, 16);
    p += __shfl_xor(p, 32);
    return p + L.b3;
}

// Log-scale applied by the preconditioner: b(o) = C tanh(o / C), C = 2, so a
// trained network reweights the diagonal step by a factor in [e^-2, e^2].
constexpr float OUT_BOUND = 2.0f;

// exp(2 tanh(o / 2)) from two hardware exponentials: with u = exp(-|o|),
// tanh(|o| / 2) = (1 - u) / (1 + u).  Relative error a few 1e-7 (the
// cancellation in 1 - u is absolute, and exp(2 tanh) ~ 1 + 2 tanh there).
__device__ inline float bounded_scale_fast(float o) {
    const float u = __expf(-fabsf(o));
    const float th = (1.0f - u) * __builtin_amdgcn_rcpf(1.0f + u);
    return __expf(OUT_BOUND * copysignf(th, o));
}

// W = m o R with m_ij = exp(b(o_ij)) / s(d_i - sigma_j), sigma_j the diagonal
// preconditioner's shift of column j; R may alias W.  An entry whose learned
// factor is not finite gets the diagonal step alone (counted in *fallbacks
// when that is given).  Inside a solve, flags stops the kernel when the
// iteration's Cholesky QR or Rayleigh-Ritz failed (W then still holds the
// block the retry starts from).
// KP > 0 fixes k at compile time (the sample -> (row, column) split is a shift).
// The next step's inputs are loaded before this step's matrix-core work, so
// every wave keeps one step of loads in flight.
// Five waves per SIMD (94 registers, no spills): 390 us per apply on n = 2e6,
// k = 8, against 400 us at four and 514 us before the group weights moved to
// LDS (three waves).
template <typename T, int KP>
__global__ __launch_bounds__(INF_THREADS) __attribute__((amdgpu_waves_per_eu(5, 8))) void mlp_precond_kernel(int64_t n, int k_rt, const float *__restrict__ P,
                                                                  const T *__restrict__ d,
                                                                  const float *__restrict__ rho,
                                                                  const float *__restrict__ tmean,
                                                                  const double *__restrict__ theta, const T *R, T *W,
                                                                  double eps, double off, const int *__restrict__ flags,
                                                                  unsigned long long *__restrict__ fallbacks) {
    if (flags && (flags[0] & (FLAG_CHOLQR_FAIL | FLAG_RR_FAIL))) return;
    const int lane = threadIdx.x % LOBPCG_WAVE, c = lane % 16, g = lane / 16;
    unsigned nfb = 0;
    const int k = KP ? KP : k_rt;
    LaneWeights L;
    load_lane_weights(L, P, c, g);
    __shared__ GroupWeights S;
    stage_group_weights(S, P);
    const double lift = off * ritz_spread(theta, k);   // theta_j - sigma_j of the diagonal step
    const int64_t total = n * k, nsteps = (total + 15) / 16;
    const int64_t wave = ((int64_t)blockIdx.x * INF_THREADS + threadIdx.x) / LOBPCG_WAVE;
    const int64_t nwaves = (int64_t)gridDim.x * (INF_THREADS / LOBPCG_WAVE);
    // the per-row feature array of lane group g (g = 1 reads theta instead),
    // chosen once by selects: as a chained conditional expression the compiler
    // turned it into a table in private memory, read on every step
    uintptr_t fbits = (uintptr_t)d;
    if (g == 2) fbits = (uintptr_t)rho;
    if (g == 3) fbits = (uintptr_t)tmean;
    const float *frow = (const float *)fbits;
    // inputs of one step: this lane's feature; for lane group 0 also theta_j and R_ij
    struct In {
        double f, th;
        T r;
    };
    auto load = [&](int64_t st, In &x) {
        const int64_t sidx = st * 16 + c;
        const bool valid = sidx < total;
        const int64_t i = valid ? sidx / k : 0;
        const int j = valid ? (int)(sidx - i * k) : 0;
        if constexpr (sizeof(T) == 4) {
            // the three per-row features are float arrays: one load through this lane's pointer
            x.f = g == 1 ? theta[j] : (double)frow[i];
        } else {
            if (g == 0) x.f = (double)d[i];
            else if (g == 1) x.f = theta[j];
            else if (g == 2) x.f = (double)rho[i];
            else x.f = (double)tmean[i];
        }
        if (g == 0) {
            x.th = theta[j];
            x.r = valid ? R[sidx] : T(0);
        }
    };
    In cur{}, nxt{};
    if (wave < nsteps) load(wave, cur);
    for (int64_t st = wave; st < nsteps; st += nwaves) {
        if (st + nwaves < nsteps) load(st + nwaves, nxt);
        int gs = g;
        asm volatile("" : "+v"(gs));
        const float o = mlp_step(L, S, gs, (float)((cur.f - L.mu) * L.isg));
        const int64_t sidx = st * 16 + c;
        if (g == 0 && sidx < total) {
            const double dm = cur.f - cur.th + lift;
            const double sg = fabs(dm) >= eps ? dm : (dm < 0 ? -eps : eps);
            if constexpr (sizeof(T) == 4) {
                // FP32 blocks: the scale in FP32 from hardware exponentials and
                // reciprocal (a few ulp; the guard decision stays in FP64)
                const float rs = __builtin_amdgcn_rcpf((float)sg);
                float m = bounded_scale_fast(o) * rs;
                if (!isfinite(m)) {
                    m = rs;
                    ++nfb;
                }
                W[sidx] = cur.r * m;
            } else {
                const float e = expf(OUT_BOUND * tanhf(o / OUT_BOUND));
                double m = (double)e / sg;
                if (!isfinite(m)) {
                    m = 1.0 / sg;
                    ++nfb;
                }
                W[sidx] = cur.r * m;
            }
        }
        cur = nxt;
    }
    if (fallbacks) {
        // one integer atomic per wave (a count: the order does not matter)
        for (int off2 = 32; off2 > 0; off2 >>= 1) nfb += __shfl_xor(nfb, off2);
        if (lane == 0 && nfb) atomicAdd(fallbacks, (unsigned long long)nfb);
    }
}

__global__ __launch_bounds__(INF_THREADS) void mlp_forward_kernel(int64_t N, const float *__restrict__ P,
                                                                  const float *__restrict__ feat,
                                                                  float *__restrict__ out) {
    const int lane = threadIdx.x % LOBPCG_WAVE, c = lane % 16, g = lane / 16;
    LaneWeights L;
    load_lane_weights(L, P, c, g);
    __shared__ GroupWeights S;
    stage_group_weights(S, P);
    const int64_t nsteps = (N + 15) / 16;
    const int64_t wave = ((int64_t)blockIdx.x * INF_THREADS + threadIdx.x) / LOBPCG_WAVE;
    const int64_t nwaves = (int64_t)gridDim.x * (INF_THREADS / LOBPCG_WAVE);
    auto load = [&](int64_t st) -> double {
        const int64_t sidx = st * 16 + c;
        return sidx < N ? (double)feat[sidx * 4 + g] : 0.0;
    };
    double cur = wave < nsteps ? load(wave) : 0.0;
    for (int64_t st = wave; st < nsteps; st += nwaves) {
        const double nxt = st + nwaves < nsteps ? load(st + nwaves) : 0.0;   // in flight during this step
        int gs = g;
        asm volatile("" : "+v"(gs));
        const float o = mlp_step(L, S, gs, (float)((cur - L.mu) * L.isg));
        const int64_t sidx = st * 16 + c;
        if (g == 0 && sidx < N) out[sidx] = o;
        cur = nxt;
    }
}

int inference_grid(int64_t nsamples) {
    const int64_t steps = (nsamples + 15) / 16;
    const int64_t blocks = (steps + INF_THREADS / LOBPCG_WAVE - 1) / (INF_THREADS / LOBPCG_WAVE);
    return (int)std::max<int64_t>(1, std::min<int64_t>(blocks, 2048));
}

// ---------------------------------------------------------------------------
// FP32 training kernels
// ---------------------------------------------------------------------------
constexpr int FWD_THREADS = 256;
constexpr int GRP_THREADS = 256;
constexpr int BWD_WAVES = 2, BWD_THREADS = BWD_WAVES * LOBPCG_WAVE, TS = LOBPCG_WAVE, LDP = HID + 1;
constexpr int MAX_PARTS = 1024;  // backward partial gradients (2 per workgroup)

struct TrainWeights {
    float W2[HID][HID];
    float W1[HID][4];
    float b1[HID], b2[HID], w3[HID];
    double mu[4], isg[4];
    float b3;
};

__device__ inline void load_train_weights(TrainWeights &S, const float *__restrict__ P) {
    for (int q = threadIdx.x; q < HID * HID; q += blockDim.x) S.W2[q / HID][q % HID] = bf16r(P[OFF_W2 + q]);
    for (int q = threadIdx.x; q < HID * 4; q += blockDim.x) S.W1[q / 4][q % 4] = bf16r(P[OFF_W1 + q]);
    for (int q = threadIdx.x; q < HID; q += blockDim.x) {
        S.b1[q] = P[OFF_B1 + q];
        S.b2[q] = P[OFF_B2 + q];
        S.w3[q] = bf16r(P[OFF_W3 + q]);
    }
    if (threadIdx.x < 4) {
        S.mu[threadIdx.x] = (double)P[OFF_MU + threadIdx.x];
        S.isg[threadIdx.x] = 1.0 / (double)P[OFF_SIG + threadIdx.x];
    }
    if (threadIdx.x == 0) S.b3 = P[OFF_B3];
    __syncthreads();
}

__device__ inline void standardise(const TrainWeights &S, const float *__restrict__ f, float (&z)[4]) {
#pragma unroll
    for (int c = 0; c < 4; ++c) z[c] = (float)(((double)f[c] - S.mu[c]) * S.isg[c]);
}

// h = bf16(relu(W1 z + b1)); bit u of *pos set when the pre-activation is > 0
__device__ inline void layer1(const TrainWeights &S, const float (&z)[4], float (&h)[HID], uint64_t *pos) {
    uint64_t m = 0;
#pragma unroll
    for (int u = 0; u < HID; ++u) {
        float a = S.b1[u];
#pragma unroll
        for (int c = 0; c < 4; ++c) a = fmaf(S.W1[u][c], z[c], a);
        h[u] = bf16r(fmaxf(a, 0.0f));
        m |= (uint64_t)(a > 0.0f) << u;
    }
    *pos = m;
}

__device__ inline float dot_row(const float *__restrict__ w, const float (&h)[HID], float a) {
#pragma unroll
    for (int u = 0; u < HID; ++u) a = fmaf(w[u], h[u], a);
    return a;
}

// o per sample (one thread per sample)
__global__ __launch_bounds__(FWD_THREADS) void train_forward_kernel(int64_t N, const float *__restrict__ P,
                                                                    const float *__restrict__ feat,
                                                                    float *__restrict__ o) {
    __shared__ TrainWeights S;
    load_train_weights(S, P);
    for (int64_t s = (int64_t)blockIdx.x * FWD_THREADS + threadIdx.x; s < N; s += (int64_t)gridDim.x * FWD_THREADS) {
        float z[4], h[HID];
        uint64_t pos;
        standardise(S, feat + s * 4, z);
        layer1(S, z, h, &pos);
        float out = 0.0f;
        for (int v = 0; v < HID; ++v) out = fmaf(S.w3[v], fmaxf(dot_row(S.W2[v], h, S.b2[v]), 0.0f), out);
        o[s] = out + S.b3;
    }
}

// Block-wide FP64 sum of NV values per thread; every thread gets the totals.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double (*red)[NV]) {
    const int lane = threadIdx.x % LOBPCG_WAVE, wave = threadIdx.x / LOBPCG_WAVE;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
        if (lane == 0) red[wave][q] = x;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = 0.0;
        for (int w = 0; w < GRP_THREADS / LOBPCG_WAVE; ++w) x += red[w][q];
        v[q] = x;
    }
    __syncthreads();
}

// One workgroup per group: the group loss and dL/do per sample (in place of o).
__global__ __launch_bounds__(GRP_THREADS) void group_loss_kernel(int ngroups, int k, const int64_t *__restrict__ off,
                                                                 float *so, const float *__restrict__ U,
                                                                 const float *__restrict__ T,
                                                                 const float *__restrict__ w,
                                                                 const float *__restrict__ X,
                                                                 double *__restrict__ gloss) {
    __shared__ double red16[GRP_THREADS / LOBPCG_WAVE][16];
    __shared__ double red3[GRP_THREADS / LOBPCG_WAVE][3];
    const int gi = blockIdx.x;
    const int64_t b = off[gi], e = off[gi + 1];
    double a[16];
#pragma unroll
    for (int l = 0; l < 16; ++l) a[l] = 0.0;
    // a = sum w u x
    auto lscale = [&](int64_t s) { return (double)OUT_BOUND * tanh((double)so[s] / (double)OUT_BOUND); };
    for (int64_t s = b + threadIdx.x; s < e; s += GRP_THREADS) {
        const double wu = (double)w[s] * exp(lscale(s)) * (double)U[s];
#pragma unroll
        for (int l = 0; l < 16; ++l)
            if (l < k) a[l] += wu * (double)X[s * k + l];
    }
    block_sum<16>(a, red16);
    auto uprime = [&](int64_t s, double *u_out, double *e_out) {
        const double ex = exp(lscale(s));
        const double u = ex * (double)U[s];
        double xa = 0.0;
#pragma unroll
        for (int l = 0; l < 16; ++l)
            if (l < k) xa += (double)X[s * k + l] * a[l];
        *u_out = u;
        *e_out = ex;
        return u - xa;
    };
    double S[3] = {0.0, 0.0, 0.0};
    for (int64_t s = b + threadIdx.x; s < e; s += GRP_THREADS) {
        double u, ex;
        const double up = uprime(s, &u, &ex);
        const double ws = w[s], ts = T[s];
        S[0] += ws * up * ts;
        S[1] += ws * up * up;
        S[2] += ws * ts * ts;
    }
    block_sum<3>(S, red3);
    const double SuT = S[0], Suu = S[1], STT = S[2];
    const bool valid = Suu > 0.0 && STT > 0.0;
    if (threadIdx.x == 0) gloss[gi] = valid ? 1.0 - SuT * SuT / (Suu * STT) : 0.0;
    const double coef = 1.0 / ngroups;
    const double den = valid ? Suu * Suu * STT : 1.0;
    double gx[16];
#pragma unroll
    for (int l = 0; l < 16; ++l) gx[l] = 0.0;
    for (int64_t s = b + threadIdx.x; s < e; s += GRP_THREADS) {
        double u, ex;
        const double up = uprime(s, &u, &ex);
        const double gup = valid ? -2.0 * w[s] * (SuT * T[s] * Suu - SuT * SuT * up) / den * coef : 0.0;
#pragma unroll
        for (int l = 0; l < 16; ++l)
            if (l < k) gx[l] += gup * (double)X[s * k + l];
    }
    block_sum<16>(gx, red16);
    for (int64_t s = b + threadIdx.x; s < e; s += GRP_THREADS) {
        double u, ex;
        const double up = uprime(s, &u, &ex);
        const double gup = valid ? -2.0 * w[s] * (SuT * T[s] * Suu - SuT * SuT * up) / den * coef : 0.0;
        double xg = 0.0;
#pragma unroll
        for (int l = 0; l < 16; ++l)
            if (l < k) xg += (double)X[s * k + l] * gx[l];
        const double gu = gup - (double)w[s] * xg;
        const double t = lscale(s) / (double)OUT_BOUND;
        so[s] = (float)(gu * (double)U[s] * ex * (1.0 - t * t));   // db/do = 1 - tanh^2
    }
}

struct BwdTile {
    float h1[TS][LDP];   // bf16(relu(a1)) per sample
    float g2[TS][LDP];   // dL/da2
    float q[TS][LDP];    // relu(a2) dL/do
    float g1[TS][LDP];   // dL/da1
    float z[TS][4];
    float go[TS];
};

// Per wavefront a 64-sample tile: per-sample forward and backward (one lane
// per sample), then lane t accumulates the gradient rows of hidden unit t
// over the tile.  One partial gradient per wavefront.
__global__ __launch_bounds__(BWD_THREADS) void train_backward_kernel(int64_t N, const float *__restrict__ P,
                                                                     const float *__restrict__ feat,
                                                                     const float *__restrict__ go_in,
                                                                     float *__restrict__ partial) {
    __shared__ TrainWeights S;
    __shared__ BwdTile tiles[BWD_WAVES];
    load_train_weights(S, P);
    const int lane = threadIdx.x % LOBPCG_WAVE, wv = threadIdx.x / LOBPCG_WAVE;
    BwdTile &tl = tiles[wv];
    float accW2[HID], accW1[4];
#pragma unroll
    for (int u = 0; u < HID; ++u) accW2[u] = 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) accW1[c] = 0.0f;
    float accb1 = 0.0f, accb2 = 0.0f, accw3 = 0.0f, accb3 = 0.0f;
    for (int64_t base = (int64_t)blockIdx.x * BWD_THREADS; base < N; base += (int64_t)gridDim.x * BWD_THREADS) {
        const int64_t s = base + threadIdx.x;
        const bool valid = s < N;
        {
            float z[4] = {0.0f, 0.0f, 0.0f, 0.0f}, h[HID], gh[HID];
            uint64_t pos;
            if (valid) standardise(S, feat + s * 4, z);
            const float go = valid ? go_in[s] : 0.0f;
            layer1(S, z, h, &pos);
#pragma unroll
            for (int u = 0; u < HID; ++u) {
                tl.h1[lane][u] = h[u];
                gh[u] = 0.0f;
            }
            for (int v = 0; v < HID; ++v) {
                const float a2 = dot_row(S.W2[v], h, S.b2[v]);
                const float ga2 = a2 > 0.0f ? go * S.w3[v] : 0.0f;
                tl.q[lane][v] = fmaxf(a2, 0.0f) * go;
                tl.g2[lane][v] = ga2;
#pragma unroll
                for (int u = 0; u < HID; ++u) gh[u] = fmaf(S.W2[v][u], ga2, gh[u]);
            }
#pragma unroll
            for (int u = 0; u < HID; ++u) tl.g1[lane][u] = ((pos >> u) & 1) ? gh[u] : 0.0f;
#pragma unroll
            for (int c = 0; c < 4; ++c) tl.z[lane][c] = z[c];
            tl.go[lane] = go;
        }
        __syncthreads();
        const int t = lane;
        for (int q = 0; q < TS; ++q) {
            const float g2 = tl.g2[q][t], g1 = tl.g1[q][t];
#pragma unroll
            for (int u = 0; u < HID; ++u) accW2[u] = fmaf(g2, tl.h1[q][u], accW2[u]);
            accb2 += g2;
            accw3 += tl.q[q][t];
#pragma unroll
            for (int c = 0; c < 4; ++c) accW1[c] = fmaf(g1, tl.z[q][c], accW1[c]);
            accb1 += g1;
            accb3 += tl.go[q];
        }
        __syncthreads();
    }
    float *out = partial + ((size_t)blockIdx.x * BWD_WAVES + wv) * NPARAM;
    const int t = lane;
#pragma unroll
    for (int c = 0; c < 4; ++c) out[OFF_W1 + t * 4 + c] = accW1[c];
    out[OFF_B1 + t] = accb1;
#pragma unroll
    for (int u = 0; u < HID; ++u) out[OFF_W2 + t * HID + u] = accW2[u];
    out[OFF_B2 + t] = accb2;
    out[OFF_W3 + t] = accw3;
    if (t == 0) out[OFF_B3] = accb3;
}

// Sum of the partial gradients (fixed order, FP64) and, when t > 0, one Adam
// step (Kingma & Ba 2015) on the FP32 master parameters.
__global__ void reduce_adam_kernel(int nparts, const float *__restrict__ partial, float *__restrict__ grad,
                                   float *__restrict__ P, float *__restrict__ m, float *__restrict__ v, int t,
                                   float lr) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NPARAM) return;
    double acc = 0.0;
    for (int q = 0; q < nparts; ++q) acc += (double)partial[(size_t)q * NPARAM + p];
    const float gq = (float)acc;
    grad[p] = gq;
    if (t > 0) {
        const double mm = 0.9 * (double)m[p] + 0.1 * (double)gq;
        const double vv = 0.999 * (double)v[p] + 0.001 * (double)gq * (double)gq;
        m[p] = (float)mm;
        v[p] = (float)vv;
        const double mh = mm / (1.0 - pow(0.9, t)), vh = vv / (1.0 - pow(0.999, t));
        P[p] = (float)((double)P[p] - (double)lr * mh / (sqrt(vh) + 1e-8));
    }
}

__global__ void mean_loss_kernel(int ngroups, const double *__restrict__ gloss, double *__restrict__ loss) {
    __shared__ double red[GRP_THREADS / LOBPCG_WAVE][1];
    double v[1] = {0.0};
    for (int g = threadIdx.x; g < ngroups; g += GRP_THREADS) v[0] += gloss[g];
    block_sum<1>(v, red);
    if (threadIdx.x == 0) *loss = ngroups > 0 ? v[0] / ngroups : 0.0;
}

// group_off[0] == 0, nondecreasing, group_off[ngroups] == N
__global__ void check_offsets_kernel(int ngroups, int64_t N, const int64_t *__restrict__ off, int *__restrict__ bad) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g > ngroups) return;
    const int64_t x = off[g];
    bool ok = x >= 0 && x <= N;
    if (g == 0) ok = ok && x == 0;
    if (g == ngroups) ok = ok && x == N;
    if (g > 0) ok = ok && off[g - 1] <= x;
    if (!ok) atomicOr(bad, 1);
}

// mu, sigma of the raw features (two passes, FP64)
__global__ void standardizer_kernel(int64_t N, const float *__restrict__ feat, float *__restrict__ P) {
    __shared__ double red[GRP_THREADS / LOBPCG_WAVE][4];
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t s = threadIdx.x; s < N; s += GRP_THREADS)
#pragma unroll
        for (int c = 0; c < 4; ++c) m[c] += (double)feat[s * 4 + c];
    block_sum<4>(m, red);
#pragma unroll
    for (int c = 0; c < 4; ++c) m[c] /= (double)N;
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t s = threadIdx.x; s < N; s += GRP_THREADS)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double x = (double)feat[s * 4 + c] - m[c];
            q[c] += x * x;
        }
    block_sum<4>(q, red);
    if (threadIdx.x < 4) {
        const int c = threadIdx.x;
        P[OFF_MU + c] = (float)m[c];
        P[OFF_SIG + c] = (float)fmax(sqrt(q[c] / (double)N), 1e-12);
    }
}

bool blob_ok(const float *blob) {
    for (int q = 0; q < LOBPCG_MLP_NBLOB; ++q)
        if (!std::isfinite(blob[q])) return false;
    for (int c = 0; c < 4; ++c)
        if (!(blob[OFF_SIG + c] > 0.0f)) return false;
    return true;
}

void free_mlp(lobpcg_mlp *m) {
    void *ptrs[] = {m->params, m->adam_m, m->adam_v, m->grad, m->grad_partial, m->so, m->gloss, m->loss};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete m;
}

#define MLP_HIP(m, expr)                                                                         \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return set_mlp_err((m), LOBPCG_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int check_batch(lobpcg_mlp *m, const lobpcg_mlp_batch *b) {
    if (!b) return set_mlp_err(m, LOBPCG_EINVAL, "null batch");
    if (b->nsamples < 0 || b->ngroups < 1 || b->k < 1 || b->k > 16)
        return set_mlp_err(m, LOBPCG_EINVAL, "batch: need nsamples >= 0, ngroups >= 1, 1 <= k <= 16");
    if (b->nsamples > 0 && (!b->feat || !b->U || !b->T || !b->w || !b->Xrow))
        return set_mlp_err(m, LOBPCG_EINVAL, "batch: null array");
    if (!b->group_off) return set_mlp_err(m, LOBPCG_EINVAL, "batch: null group_off");
    return LOBPCG_OK;
}

// loss and gradient at the current parameters; Adam step when step > 0
int loss_grad_impl(lobpcg_mlp *m, const lobpcg_mlp_batch *b, double *loss, float *grad_host, int step, float lr,
                   hipStream_t s) {
    int rc = check_batch(m, b);
    if (rc != LOBPCG_OK) return rc;
    MLP_HIP(m, hipSetDevice(m->device));
    const int64_t N = b->nsamples;
    const int G = b->ngroups;
    // buffers sized to the batch
    if (N > m->so_cap) {
        if (m->so) MLP_HIP(m, hipFree(m->so));
        m->so = nullptr;
        m->so_cap = 0;
        if (hipMalloc((void **)&m->so, (size_t)N * sizeof(float)) != hipSuccess)
            return set_mlp_err(m, LOBPCG_ENOMEM, "batch buffer of %lld samples", (long long)N);
        m->so_cap = N;
    }
    if (G > m->gloss_cap) {
        if (m->gloss) MLP_HIP(m, hipFree(m->gloss));
        m->gloss = nullptr;
        m->gloss_cap = 0;
        if (hipMalloc((void **)&m->gloss, ((size_t)G + 1) * sizeof(double)) != hipSuccess)
            return set_mlp_err(m, LOBPCG_ENOMEM, "group buffer of %d groups", G);
        m->gloss_cap = G;
    }
    // offsets are checked before any kernel indexes with them
    int *bad = (int *)(m->gloss + G);
    MLP_HIP(m, hipMemsetAsync(bad, 0, sizeof(int), s));
    check_offsets_kernel<<<ceil_div((int64_t)G + 1, 256), 256, 0, s>>>(G, N, b->group_off, bad);
    int hbad = 0;
    MLP_HIP(m, hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    MLP_HIP(m, hipStreamSynchronize(s));
    if (hbad) return set_mlp_err(m, LOBPCG_EINVAL, "batch: group_off must start at 0, not decrease and end at nsamples");
    int nparts = 0;
    if (N > 0) {
        train_forward_kernel<<<(int)std::min<int64_t>(ceil_div(N, FWD_THREADS), 4096), FWD_THREADS, 0, s>>>(
            N, m->params, b->feat, m->so);
        group_loss_kernel<<<G, GRP_THREADS, 0, s>>>(G, b->k, b->group_off, m->so, b->U, b->T, b->w, b->Xrow, m->gloss);
        const int nblk = (int)std::min<int64_t>(ceil_div(N, BWD_THREADS), MAX_PARTS / BWD_WAVES);
        train_backward_kernel<<<nblk, BWD_THREADS, 0, s>>>(N, m->params, b->feat, m->so, m->grad_partial);
        nparts = nblk * BWD_WAVES;
    } else {
        MLP_HIP(m, hipMemsetAsync(m->gloss, 0, (size_t)G * sizeof(double), s));
    }
    mean_loss_kernel<<<1, GRP_THREADS, 0, s>>>(G, m->gloss, m->loss);
    int t = 0;
    if (step) t = m->adam_t + 1;
    reduce_adam_kernel<<<ceil_div(NPARAM, 256), 256, 0, s>>>(nparts, m->grad_partial, m->grad, m->params, m->adam_m,
                                                            m->adam_v, t, lr);
    MLP_HIP(m, hipGetLastError());
    double hl = 0.0;
    MLP_HIP(m, hipMemcpyAsync(&hl, m->loss, sizeof(double), hipMemcpyDeviceToHost, s));
    if (grad_host) MLP_HIP(m, hipMemcpyAsync(grad_host, m->grad, NPARAM * sizeof(float), hipMemcpyDeviceToHost, s));
    MLP_HIP(m, hipStreamSynchronize(s));
    if (step) m->adam_t = t;
    if (loss) *loss = hl;
    return LOBPCG_OK;
}

}  // namespace

int mlp_precond_ready(lobpcg_ctx *ctx) {
    if (!ctx->mlp) return set_err(ctx, LOBPCG_EINVAL, "no MLP attached to this context");
    return LOBPCG_OK;
}

int launch_mlp_precond(lobpcg_ctx *ctx, const void *R, const double *theta, void *W, int k, hipStream_t s,
                       bool in_solve) {
    const int *flags = in_solve ? ctx->dflags : nullptr;
    unsigned long long *fb = in_solve ? ctx->mlp_fallback_count : nullptr;
    const double eps = ctx->eps_rel * ctx->gamma;
    const int grid = inference_grid(ctx->n * k);
#define MLP_LAUNCH(T, KP)                                                                                 \
    mlp_precond_kernel<T, KP><<<grid, INF_THREADS, 0, s>>>(ctx->n, k, ctx->mlp->params, (const T *)ctx->diag, \
                                                           ctx->feat_rownorm, ctx->feat_tilemean, theta,     \
                                                           (const T *)R, (T *)W, eps,  \
                                                           ctx->precond_offset, flags, fb)
    if (ctx->dtype == LOBPCG_F32) {
        if (k == 8) MLP_LAUNCH(float, 8);
        else if (k == 16) MLP_LAUNCH(float, 16);
        else MLP_LAUNCH(float, 0);
    } else {
        if (k == 8) MLP_LAUNCH(double, 8);
        else if (k == 16) MLP_LAUNCH(double, 16);
        else MLP_LAUNCH(double, 0);
    }
#undef MLP_LAUNCH
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_err(ctx, LOBPCG_EHIP, "MLP preconditioner launch: %s", hipGetErrorString(e));
    return LOBPCG_OK;
}

extern "C" {

int lobpcg_mlp_create(lobpcg_mlp **out, const float *blob) {
    if (!out) return LOBPCG_EINVAL;
    *out = nullptr;
    if (!blob || !blob_ok(blob)) return LOBPCG_EINVAL;
    lobpcg_mlp *m = new (std::nothrow) lobpcg_mlp();
    if (!m) return LOBPCG_ENOMEM;
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        return LOBPCG_EHIP;
    }
    m->grad_max_parts = MAX_PARTS;
    bool ok = hipMalloc((void **)&m->params, LOBPCG_MLP_NBLOB * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&m->adam_m, NPARAM * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&m->adam_v, NPARAM * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&m->grad, NPARAM * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&m->grad_partial, (size_t)MAX_PARTS * NPARAM * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&m->loss, sizeof(double)) == hipSuccess;
    if (!ok) {
        free_mlp(m);
        return LOBPCG_ENOMEM;
    }
    int rc = lobpcg_mlp_set_params(m, blob);
    if (rc != LOBPCG_OK) {
        free_mlp(m);
        return rc;
    }
    *out = m;
    return LOBPCG_OK;
}

void lobpcg_mlp_destroy(lobpcg_mlp *m) {
    if (!m) return;
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    free_mlp(m);
}

int lobpcg_mlp_set_params(lobpcg_mlp *m, const float *blob) {
    if (!m) return LOBPCG_EINVAL;
    if (!blob || !blob_ok(blob)) return set_mlp_err(m, LOBPCG_EINVAL, "parameters must be finite with sigma > 0");
    MLP_HIP(m, hipSetDevice(m->device));
    MLP_HIP(m, hipMemcpy(m->params, blob, LOBPCG_MLP_NBLOB * sizeof(float), hipMemcpyHostToDevice));
    MLP_HIP(m, hipMemset(m->adam_m, 0, NPARAM * sizeof(float)));
    MLP_HIP(m, hipMemset(m->adam_v, 0, NPARAM * sizeof(float)));
    m->adam_t = 0;
    return LOBPCG_OK;
}

int lobpcg_mlp_get_params(lobpcg_mlp *m, float *blob) {
    if (!m) return LOBPCG_EINVAL;
    if (!blob) return set_mlp_err(m, LOBPCG_EINVAL, "null output");
    MLP_HIP(m, hipSetDevice(m->device));
    MLP_HIP(m, hipDeviceSynchronize());
    MLP_HIP(m, hipMemcpy(blob, m->params, LOBPCG_MLP_NBLOB * sizeof(float), hipMemcpyDeviceToHost));
    return LOBPCG_OK;
}

const char *lobpcg_mlp_last_error(const lobpcg_mlp *m) { return m ? m->err.c_str() : "null network"; }

int lobpcg_set_mlp(lobpcg_ctx *ctx, lobpcg_mlp *m) {
    if (!ctx) return LOBPCG_EINVAL;
    if (m && m->device != ctx->device)
        return set_err(ctx, LOBPCG_EINVAL, "network on device %d, context on device %d", m->device, ctx->device);
    ctx->mlp = m;
    return LOBPCG_OK;
}

int lobpcg_get_features(lobpcg_ctx *ctx, float *rownorm, float *tilemean, void *stream) {
    if (!ctx) return LOBPCG_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)ctx->n * sizeof(float);
    if (rownorm) HIP_TRY(ctx, hipMemcpyAsync(rownorm, ctx->feat_rownorm, bytes, hipMemcpyDeviceToDevice, s));
    if (tilemean) HIP_TRY(ctx, hipMemcpyAsync(tilemean, ctx->feat_tilemean, bytes, hipMemcpyDeviceToDevice, s));
    return LOBPCG_OK;
}

int lobpcg_mlp_forward(lobpcg_mlp *m, const float *feat, int64_t N, float *o, void *stream) {
    if (!m) return LOBPCG_EINVAL;
    if (N < 0) return set_mlp_err(m, LOBPCG_EINVAL, "forward: N < 0");
    if (N == 0) return LOBPCG_OK;
    if (!feat || !o) return set_mlp_err(m, LOBPCG_EINVAL, "forward: null pointer");
    MLP_HIP(m, hipSetDevice(m->device));
    hipStream_t s = (hipStream_t)stream;
    mlp_forward_kernel<<<inference_grid(N), INF_THREADS, 0, s>>>(N, m->params, feat, o);
    MLP_HIP(m, hipGetLastError());
    return LOBPCG_OK;
}

int lobpcg_mlp_fit_standardizer(lobpcg_mlp *m, const float *feat, int64_t N, void *stream) {
    if (!m) return LOBPCG_EINVAL;
    if (N < 2 || !feat) return set_mlp_err(m, LOBPCG_EINVAL, "fit_standardizer: need N >= 2 rows");
    MLP_HIP(m, hipSetDevice(m->device));
    hipStream_t s = (hipStream_t)stream;
    standardizer_kernel<<<1, GRP_THREADS, 0, s>>>(N, feat, m->params);
    MLP_HIP(m, hipGetLastError());
    return LOBPCG_OK;
}

int lobpcg_mlp_loss_grad(lobpcg_mlp *m, const lobpcg_mlp_batch *b, double *loss, float *grad, void *stream) {
    if (!m) return LOBPCG_EINVAL;
    return loss_grad_impl(m, b, loss, grad, 0, 0.0f, (hipStream_t)stream);
}

int lobpcg_mlp_train_step(lobpcg_mlp *m, const lobpcg_mlp_batch *b, float lr, double *loss, void *stream) {
    if (!m) return LOBPCG_EINVAL;
    if (!(lr > 0.0f) || !std::isfinite(lr)) return set_mlp_err(m, LOBPCG_EINVAL, "train_step: lr must be > 0");
    return loss_grad_impl(m, b, loss, nullptr, 1, lr, (hipStream_t)stream);
}

}  // extern "C"
