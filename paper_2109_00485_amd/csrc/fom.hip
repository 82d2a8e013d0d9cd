// Block-diagonal preconditioner of Section 3.4: K = diag(K_1, ..., K_b) with
// K_t the t-th 64 x 64 diagonal tile of H shifted by sigma_j, and each system
// (H_tt - sigma_j I) w = r_j solved approximately by m steps of the full
// orthogonalisation method (FOM; the paper uses three to five): an Arnoldi
// process with modified Gram-Schmidt builds an orthonormal basis V_m of the
// Krylov space of r_j and the Hessenberg matrix H_m, and w = V_m y with
// H_m y = ||r_j|| e_1.  Every column of the block is its own right-hand side
// with its own shift (multiple Krylov spaces, as in the paper).  Each new
// Arnoldi vector is orthogonalised twice: on a tile dominated by a constant
// diagonal (|H_tt - sigma I - c I| << c) every product is nearly parallel to
// its input and one Gram-Schmidt pass loses the orthogonality of V_m.
//
// Mapping: one workgroup of eight waves per tile; the dense symmetric tile
// (built at create) is staged once in LDS in FP64 (rows padded to 66 values
// so that each lane's 16-byte reads of its own row are conflict-free) and
// shared by the waves; wave w runs the Arnoldi processes of columns w, w + 8,
// ... alone: lane r holds row r of every basis vector in registers, the
// product with the tile reads row r (= column r) of the tile and the current
// basis vector broadcast from LDS, and inner products are DPP wave
// reductions.  Each new vector is orthogonalised twice, by two classical
// Gram-Schmidt passes whose inner products are reduced together (the
// oracle's two modified Gram-Schmidt passes give the same basis up to
// rounding).  The small Hessenberg system is solved by the wave itself: lane
// j holds column j of H_m, the Givens rotations (uniform) update all columns
// at once, and back substitution reads the columns with readlane; nothing
// leaves registers.  No barrier after the tile is staged, so columns whose
// Arnoldi process ends early (an invariant Krylov space) do not hold the
// others back.  The arithmetic is FP64 for both context precisions (the tile
// and the block are read in the context precision).  A system whose H_m is
// singular to 1e-12 of its largest entry has no FOM iterate; that column of
// that tile gets the guarded diagonal step.
#include "internal.hpp"

namespace {

constexpr int FOM_WAVES = 8;
constexpr int FOM_THREADS = FOM_WAVES * LOBPCG_WAVE;
constexpr int LDA = 66;                 // padded LDS row of the tile (doubles)
constexpr int MMAX = 8;                 // FOM steps, at most
constexpr double BREAKDOWN = 1e-12;     // h_{j+1,j} <= this * ||A v_j||: invariant Krylov space
constexpr double SINGULAR = 1e-12;      // min |R_ii| <= this * max |h_ij|: no FOM iterate

// one DPP move of a double (both halves), rows outside ROW_MASK read 0
template <int CTRL, int ROW_MASK = 0xF>
__device__ inline double dpp(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ inline double readlane(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// the first N entries of v replaced by their sums over the wave (uniform);
// the N reductions are interleaved step by step, in a fixed order
template <int N>
__device__ inline void wave_sums(double (&v)[N], int count) {
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (i < count) v[i] += dpp<0xB1>(v[i]);     // quad_perm [1,0,3,2]
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (i < count) v[i] += dpp<0x4E>(v[i]);     // quad_perm [2,3,0,1]
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (i < count) v[i] += dpp<0x141>(v[i]);    // row_half_mirror: 8-lane sums
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (i < count) v[i] += dpp<0x140>(v[i]);    // row_mirror: 16-lane sums
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (i < count) v[i] += dpp<0x142, 0xA>(v[i]);   // row_bcast15 into rows 1, 3
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (i < count) v[i] += dpp<0x143, 0xC>(v[i]);   // row_bcast31 into rows 2, 3
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (i < count) v[i] = readlane(v[i], LOBPCG_WAVE - 1);
}

__device__ inline void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

// M: the FOM steps (the step count is a template argument so that every
// per-step array is indexed statically and stays in registers)
template <typename T, int M>
__global__ __launch_bounds__(FOM_THREADS) void fom_precond_kernel(int64_t n, int k, const T *__restrict__ tiles,
                                                                  const T *R, const double *__restrict__ theta, T *W,
                                                                  double eps, double off, const int *__restrict__ flags) {
    if (flags && (flags[0] & (FLAG_CHOLQR_FAIL | FLAG_RR_FAIL))) return;
    __shared__ __align__(16) double A[64 * LDA];
    __shared__ __align__(16) double vbuf[FOM_WAVES][64];
    const int64_t t = blockIdx.x;
    const int wave = threadIdx.x / LOBPCG_WAVE, r = threadIdx.x % LOBPCG_WAVE;
    {
        const T *src = tiles + t * 64 * 64;
        for (int e = threadIdx.x; e < 64 * 64; e += FOM_THREADS) A[(e / 64) * LDA + e % 64] = (double)src[e];
    }
    const double spread = ritz_spread(theta, k);
    __syncthreads();   // the only barrier: the tile is shared, everything else is per wave
    const int64_t row = t * 64 + r;
    const bool live = row < n;
    const double dr = A[r * LDA + r];
    const double *Ar = &A[r * LDA];
    double *vb = vbuf[wave];
    for (int c = wave; c < k; c += FOM_WAVES) {
        const double sigma = theta[c] - off * spread;
        const double b = live ? (double)R[row * k + c] : 0.0;
        double nb[1] = {b * b};
        wave_sums(nb, 1);
        const double beta = sqrt(nb[0]);
        double x = 0.0;
        if (beta > 0.0) {
            double V[M + 1], Hc[M + 1];   // lane j: column j of the Hessenberg matrix
#pragma unroll
            for (int i = 0; i <= M; ++i) V[i] = Hc[i] = 0.0;
            V[0] = b / beta;
            int steps = M;
            double hmax = 0.0;   // largest |h_ij| of the (steps + 1) x steps Hessenberg
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if (j >= steps) break;
                // w = (A - sigma I) v_j: row r of the symmetric tile times v_j
                vb[r] = V[j];
                wave_fence();
                double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
                for (int q = 0; q < 64; q += 4) {
                    const double2 x0 = *(const double2 *)&Ar[q], x1 = *(const double2 *)&Ar[q + 2];
                    const double2 v0 = *(const double2 *)&vb[q], v1 = *(const double2 *)&vb[q + 2];
                    a0 = fma(x0.x, v0.x, a0);
                    a1 = fma(x0.y, v0.y, a1);
                    a2 = fma(x1.x, v1.x, a2);
                    a3 = fma(x1.y, v1.y, a3);
                }
                double w = ((a0 + a1) + (a2 + a3)) - sigma * V[j];
                wave_fence();   // every lane has read v_j before the next step overwrites it
                // first pass: ||w||^2 and <w, v_i>, i <= j, reduced together
                double d[M + 1];
                d[0] = w * w;
#pragma unroll
                for (int i = 0; i < M; ++i)
                    if (i <= j) d[i + 1] = w * V[i];
                wave_sums(d, j + 2);
                const double wn = sqrt(d[0]);
                double h[M];
#pragma unroll
                for (int i = 0; i < M; ++i)
                    if (i <= j) {
                        h[i] = d[i + 1];
                        w -= h[i] * V[i];
                    }
                // second pass
                double e[M];
#pragma unroll
                for (int i = 0; i < M; ++i)
                    if (i <= j) e[i] = w * V[i];
                wave_sums(e, j + 1);
#pragma unroll
                for (int i = 0; i < M; ++i)
                    if (i <= j) {
                        w -= e[i] * V[i];
                        h[i] += e[i];
                    }
                double hn[1] = {w * w};
                wave_sums(hn, 1);
                const double hj = sqrt(hn[0]);
#pragma unroll
                for (int i = 0; i < M; ++i)
                    if (i <= j) {
                        Hc[i] = r == j ? h[i] : Hc[i];
                        hmax = fmax(hmax, fabs(h[i]));
                    }
                Hc[j + 1] = r == j ? hj : Hc[j + 1];
                hmax = fmax(hmax, hj);
                if (hj <= BREAKDOWN * wn) {
                    steps = j + 1;   // invariant Krylov space: the FOM iterate is exact
                    break;
                }
                V[j + 1] = w / hj;
            }
            // H_s y = beta e_1 by Givens rotations on the square Hessenberg H_s
            double g[M];
#pragma unroll
            for (int i = 0; i < M; ++i) g[i] = i == 0 ? beta : 0.0;
#pragma unroll
            for (int i = 0; i + 1 < M; ++i) {
                if (i + 1 >= steps) break;
                const double a = readlane(Hc[i], i), bb = readlane(Hc[i + 1], i);
                const double rr = sqrt(a * a + bb * bb);
                const double cs = rr > 0.0 ? a / rr : 1.0, sn = rr > 0.0 ? bb / rr : 0.0;
                if (r >= i) {
                    const double u = Hc[i], v = Hc[i + 1];
                    Hc[i] = cs * u + sn * v;
                    Hc[i + 1] = -sn * u + cs * v;
                }
                const double gu = g[i], gv = g[i + 1];
                g[i] = cs * gu + sn * gv;
                g[i + 1] = -sn * gu + cs * gv;
            }
            double rdiag[M];
            double rmin = 0.0;
#pragma unroll
            for (int i = 0; i < M; ++i)
                if (i < steps) {
                    rdiag[i] = readlane(Hc[i], i);
                    rmin = i == 0 ? fabs(rdiag[i]) : fmin(rmin, fabs(rdiag[i]));
                }
            if (rmin > SINGULAR * hmax) {
                // back substitution by columns: y_i = g_i / R_ii, then g_l -= R_li y_i (l < i)
#pragma unroll
                for (int i = M - 1; i >= 0; --i) {
                    if (i >= steps) continue;
                    const double yi = g[i] / rdiag[i];
                    x += V[i] * yi;
#pragma unroll
                    for (int l = 0; l < M; ++l)
                        if (l < i) g[l] -= readlane(Hc[l], i) * yi;
                }
            } else {
                // no FOM iterate: the diagonal step with its guard
                const double dm = dr - sigma;
                x = b / (fabs(dm) >= eps ? dm : (dm < 0 ? -eps : eps));
            }
        }
        if (live) W[row * k + c] = (T)x;
    }
}

template <typename T, int M>
void launch_fom_steps(lobpcg_ctx *ctx, const void *R, const double *theta, void *W, int k, hipStream_t s,
                      const int *flags, double eps) {
    const int grid = (int)((ctx->n + 63) / 64);
    fom_precond_kernel<T, M><<<grid, FOM_THREADS, 0, s>>>(ctx->n, k, (const T *)ctx->diag_tiles, (const T *)R, theta,
                                                          (T *)W, eps, ctx->precond_offset, flags);
}

template <typename T>
void launch_fom_typed(lobpcg_ctx *ctx, const void *R, const double *theta, void *W, int k, hipStream_t s,
                      const int *flags, double eps) {
    switch (ctx->fom_steps) {
    case 1: launch_fom_steps<T, 1>(ctx, R, theta, W, k, s, flags, eps); break;
    case 2: launch_fom_steps<T, 2>(ctx, R, theta, W, k, s, flags, eps); break;
    case 3: launch_fom_steps<T, 3>(ctx, R, theta, W, k, s, flags, eps); break;
    case 4: launch_fom_steps<T, 4>(ctx, R, theta, W, k, s, flags, eps); break;
    case 5: launch_fom_steps<T, 5>(ctx, R, theta, W, k, s, flags, eps); break;
    case 6: launch_fom_steps<T, 6>(ctx, R, theta, W, k, s, flags, eps); break;
    case 7: launch_fom_steps<T, 7>(ctx, R, theta, W, k, s, flags, eps); break;
    default: launch_fom_steps<T, 8>(ctx, R, theta, W, k, s, flags, eps); break;
    }
}

}  // namespace

int launch_fom_precond(lobpcg_ctx *ctx, const void *R, const double *theta, void *W, int k, hipStream_t s,
                       bool in_solve) {
    if (!ctx->diag_tiles) return set_err(ctx, LOBPCG_EUNSUPPORTED, "FOM preconditioner: no diagonal tiles");
    const double eps = ctx->eps_rel * ctx->gamma;
    const int *flags = in_solve ? ctx->dflags : nullptr;
    if (ctx->dtype == LOBPCG_F32)
        launch_fom_typed<float>(ctx, R, theta, W, k, s, flags, eps);
    else
        launch_fom_typed<double>(ctx, R, theta, W, k, s, flags, eps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_err(ctx, LOBPCG_EHIP, "FOM preconditioner launch: %s", hipGetErrorString(e));
    return LOBPCG_OK;
}

extern "C" int lobpcg_set_fom_steps(lobpcg_ctx *ctx, int m) {
    if (!ctx) return LOBPCG_EINVAL;
    if (m < 1 || m > MMAX) return set_err(ctx, LOBPCG_EINVAL, "FOM steps %d outside [1, %d]", m, MMAX);
    ctx->fom_steps = m;
    return LOBPCG_OK;
}
