// Small dense FP64 steps, each one workgroup of a single wavefront (the
// matrices are at most 48 x 48, so the work is latency-bound):
//  * Cholesky factor and triangular inverse for Cholesky QR (Section 3.5):
//    B = W^T W = R^T R, then R^{-1} is applied to W by the combine kernel;
//  * Rayleigh-Ritz (eq. rreig): assemble G = S^T H S and O = S^T S from the
//    lower blocks of eq. Glower, scale both by diag(O)^{-1/2} (equivalent to
//    normalising the columns of S), Cholesky O = L L^T, A = L^{-1} G L^{-T},
//    cyclic Jacobi with a round-robin pairing (all N/2 rotations of a round
//    are disjoint and applied at once), sort ascending, C = diag(O)^{-1/2}
//    L^{-T} V[:, :k].  If O is not positive definite with P, P is dropped
//    and the step repeated with S = [X, W].
#include <cfloat>

#include "internal.hpp"

namespace {

constexpr int NMAX = 48;
constexpr int LD = NMAX + 1;
constexpr int QMAX = (NMAX * NMAX + LOBPCG_WAVE - 1) / LOBPCG_WAVE;

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// In-place lower Cholesky of the N x N matrix a (row-major, leading dim LD).
// Returns false if a pivot falls below tol.  Single wavefront.
__device__ bool chol_lower(double *a, int N, double tol) {
    const int t = threadIdx.x;
    __shared__ int bad;
    if (t == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < N; ++j) {
        if (t == 0) {
            double d = a[j * LD + j];
            for (int p = 0; p < j; ++p) d -= a[j * LD + p] * a[j * LD + p];
            if (!(d > tol)) bad = 1;
            a[j * LD + j] = d > 0 ? sqrt(d) : 1.0;
        }
        __syncthreads();
        const double piv = a[j * LD + j];
        for (int i = j + 1 + t; i < N; i += LOBPCG_WAVE) {
            double v = a[i * LD + j];
            for (int p = 0; p < j; ++p) v -= a[i * LD + p] * a[j * LD + p];
            a[i * LD + j] = v / piv;
        }
        __syncthreads();
    }
    return bad == 0;
}

__global__ __launch_bounds__(64) void cholinv_kernel(int k, const double *__restrict__ B, double *__restrict__ rinv,
                                                     int *__restrict__ flags, double tol, double shift) {
    __shared__ double a[NMAX * LD];
    __shared__ double sc[NMAX];
    const int t = threadIdx.x;
    if (flags[0] & (FLAG_CHOLQR_FAIL | FLAG_RR_FAIL)) return;
    for (int e = t; e < k * k; e += LOBPCG_WAVE) {
        int i = e / k, j = e % k;
        a[i * LD + j] = 0.5 * (B[i * k + j] + B[j * k + i]);
    }
    __syncthreads();
    if (t < k) {
        double d = a[t * LD + t];
        sc[t] = d > 0 ? 1.0 / sqrt(d) : 0.0;
    }
    __syncthreads();
    bool posdiag = true;
    for (int i = 0; i < k; ++i) posdiag = posdiag && sc[i] > 0;
    for (int e = t; e < k * k; e += LOBPCG_WAVE) {
        int i = e / k, j = e % k;
        a[i * LD + j] *= sc[i] * sc[j];
    }
    __syncthreads();
    bool ok = posdiag && chol_lower(a, k, tol);
    if (posdiag && !ok) {
        // shifted Cholesky QR: factor B' + shift I (B' has unit diagonal)
        for (int e = t; e < k * k; e += LOBPCG_WAVE) {
            int i = e / k, j = e % k;
            a[i * LD + j] = 0.5 * (B[i * k + j] + B[j * k + i]) * sc[i] * sc[j] + (i == j ? shift : 0.0);
        }
        __syncthreads();
        ok = chol_lower(a, k, tol);
        if (ok && t == 0) atomicOr(&flags[0], FLAG_CHOLQR_SHIFT);
    }
    if (!ok) {
        if (t == 0) atomicOr(&flags[0], FLAG_CHOLQR_FAIL);
        return;
    }
    // R' = L^T (upper); Rinv' = R'^{-1} by back substitution per column c,
    // Rinv = diag(sc) Rinv' so that W diag(sc) R'^{-1} has orthonormal columns.
    if (t < k) {
        const int c = t;
        double y[NMAX];
        for (int i = k - 1; i >= 0; --i) {
            double v = (i == c) ? 1.0 : 0.0;
            for (int p = i + 1; p < k; ++p) v -= a[p * LD + i] * y[p];   // R'[i][p] = L[p][i]
            y[i] = v / a[i * LD + i];
        }
        for (int i = 0; i < k; ++i) rinv[i * k + c] = sc[i] * y[i];
    }
}

// Rayleigh-Ritz.  M is the Gram output [X W P]^T [X W P HX HW HP] for nblk_in
// blocks (KA = nblk_in*k rows, KB = 2*KA columns).
__global__ __launch_bounds__(64) void rr_kernel(int k, int nblk_in, const double *__restrict__ M,
                                                double *__restrict__ Cout, double *__restrict__ theta,
                                                int *__restrict__ flags, double tol) {
    __shared__ double O[NMAX * LD];
    __shared__ double A[NMAX * LD];
    __shared__ double V[NMAX * LD];
    __shared__ double sc[NMAX];
    __shared__ int idx[NMAX];
    __shared__ double rot_c[NMAX], rot_s[NMAX];
    __shared__ int partner[NMAX];
    __shared__ int isp[NMAX];
    const int t = threadIdx.x;
    if (flags[0] & (FLAG_CHOLQR_FAIL | FLAG_RR_FAIL)) return;
    const int KA = nblk_in * k, KB = 2 * KA;
    int nblk = nblk_in;
    for (;;) {
        const int N = nblk * k;
        // pencil from lower blocks; diagonal blocks symmetrised
        for (int e = t; e < N * N; e += LOBPCG_WAVE) {
            int a = e / N, b = e % N, ba = a / k, bb = b / k;
            double o, g;
            if (ba > bb) {
                o = M[a * KB + b];
                g = M[a * KB + KA + b];
            } else if (ba < bb) {
                o = M[b * KB + a];
                g = M[b * KB + KA + a];
            } else {
                o = 0.5 * (M[a * KB + b] + M[b * KB + a]);
                g = 0.5 * (M[a * KB + KA + b] + M[b * KB + KA + a]);
            }
            O[a * LD + b] = o;
            A[a * LD + b] = g;
        }
        __syncthreads();
        if (t < N) {
            double d = O[t * LD + t];
            sc[t] = d > 0 ? 1.0 / sqrt(d) : 0.0;
        }
        __syncthreads();
        bool posdiag = true;
        for (int i = 0; i < N; ++i) posdiag = posdiag && sc[i] > 0;
        for (int e = t; e < N * N; e += LOBPCG_WAVE) {
            int a = e / N, b = e % N;
            O[a * LD + b] *= sc[a] * sc[b];
            A[a * LD + b] *= sc[a] * sc[b];
        }
        __syncthreads();
        bool ok = posdiag && chol_lower(O, N, tol);
        if (!ok) {
            if (nblk == 3) {
                nblk = 2;
                if (t == 0) atomicOr(&flags[0], FLAG_RR_PDROP);
                __syncthreads();
                continue;
            }
            if (t == 0) atomicOr(&flags[0], FLAG_RR_FAIL);
            return;
        }
        // Z = L^{-1} G (column c per thread), stored in V
        for (int c = t; c < N; c += LOBPCG_WAVE) {
            for (int i = 0; i < N; ++i) {
                double v = A[i * LD + c];
                for (int p = 0; p < i; ++p) v -= O[i * LD + p] * V[p * LD + c];
                V[i * LD + c] = v / O[i * LD + i];
            }
        }
        __syncthreads();
        // A = L^{-1} Z^T  (= L^{-1} G L^{-T} since G is symmetric)
        for (int c = t; c < N; c += LOBPCG_WAVE) {
            for (int i = 0; i < N; ++i) {
                double v = V[c * LD + i];
                for (int p = 0; p < i; ++p) v -= O[i * LD + p] * A[p * LD + c];
                A[i * LD + c] = v / O[i * LD + i];
            }
        }
        __syncthreads();
        // symmetrise, V = I
        double regs[QMAX];
        double vv[QMAX];
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
            int e = t + LOBPCG_WAVE * q;
            if (e < N * N) {
                int a = e / N, b = e % N;
                regs[q] = 0.5 * (A[a * LD + b] + A[b * LD + a]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < QMAX; ++q) {
            int e = t + LOBPCG_WAVE * q;
            if (e < N * N) {
                int a = e / N, b = e % N;
                A[a * LD + b] = regs[q];
                V[a * LD + b] = (a == b) ? 1.0 : 0.0;
            }
        }
        __syncthreads();
        // cyclic Jacobi, round-robin pairing over Ne = N rounded up to even
        const int Ne = N + (N & 1);
        for (int sweep = 0; sweep < 30; ++sweep) {
            double off = 0.0, tot = 0.0;
            for (int e = t; e < N * N; e += LOBPCG_WAVE) {
                int a = e / N, b = e % N;
                double v = A[a * LD + b];
                tot += v * v;
                if (a != b) off += v * v;
            }
            off = wave_sum(off);
            tot = wave_sum(tot);
            if (off <= 1e-30 * tot || off == 0.0) break;
            for (int r = 0; r < Ne - 1; ++r) {
                if (t < Ne / 2) {
                    int pos_p = t, pos_q = Ne - 1 - t;
                    int p = pos_p == 0 ? 0 : 1 + (pos_p - 1 + r) % (Ne - 1);
                    int q = 1 + (pos_q - 1 + r) % (Ne - 1);
                    if (p > q) { int tmp = p; p = q; q = tmp; }
                    double c = 1.0, s = 0.0;
                    if (q < N) {
                        double apq = A[p * LD + q];
                        if (apq != 0.0) {
                            double tau = (A[q * LD + q] - A[p * LD + p]) / (2.0 * apq);
                            double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                            c = 1.0 / sqrt(1.0 + tt * tt);
                            s = tt * c;
                        }
                        partner[p] = q; partner[q] = p;
                        isp[p] = 1; isp[q] = 0;
                        rot_c[p] = c; rot_s[p] = s;
                        rot_c[q] = c; rot_s[q] = s;
                    } else if (p < N) {
                        partner[p] = -1;
                    }
                }
                __syncthreads();
                // A <- J^T A J and V <- V J, all rotations of the round at once
#pragma unroll
                for (int q = 0; q < QMAX; ++q) {
                    int e = t + LOBPCG_WAVE * q;
                    if (e < N * N) {
                        int i = e / N, j = e % N;
                        int pi = partner[i], pj = partner[j];
                        // row factors (J^T)[i][i], (J^T)[i][pi]; column factors J[j][j], J[pj][j]
                        double ri = 1.0, rpi = 0.0, cj = 1.0, cpj = 0.0;
                        if (pi >= 0) {
                            ri = rot_c[i];
                            rpi = isp[i] ? -rot_s[i] : rot_s[i];
                        }
                        if (pj >= 0) {
                            cj = rot_c[j];
                            cpj = isp[j] ? -rot_s[j] : rot_s[j];
                        }
                        double v = ri * cj * A[i * LD + j];
                        if (pj >= 0) v += ri * cpj * A[i * LD + pj];
                        if (pi >= 0) {
                            v += rpi * cj * A[pi * LD + j];
                            if (pj >= 0) v += rpi * cpj * A[pi * LD + pj];
                        }
                        regs[q] = v;
                        double w = cj * V[i * LD + j];
                        if (pj >= 0) w += cpj * V[i * LD + pj];
                        vv[q] = w;
                    }
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < QMAX; ++q) {
                    int e = t + LOBPCG_WAVE * q;
                    if (e < N * N) {
                        int i = e / N, j = e % N;
                        A[i * LD + j] = regs[q];
                        V[i * LD + j] = vv[q];
                    }
                }
                __syncthreads();
            }
        }
        // ascending order (ties by index)
        if (t < N) {
            double li = A[t * LD + t];
            int rank = 0;
            for (int j = 0; j < N; ++j) {
                double lj = A[j * LD + j];
                rank += (lj < li) || (lj == li && j < t);
            }
            idx[rank] = t;
        }
        __syncthreads();
        // C = diag(sc) L^{-T} V[:, idx[0..k)]
        if (t < k) {
            const int col = idx[t];
            double y[NMAX];
            for (int i = N - 1; i >= 0; --i) {
                double v = V[i * LD + col];
                for (int p = i + 1; p < N; ++p) v -= O[p * LD + i] * y[p];
                y[i] = v / O[i * LD + i];
            }
            for (int i = 0; i < N; ++i) Cout[i * k + t] = sc[i] * y[i];
            theta[t] = A[col * LD + col];
        }
        if (t == 0) flags[1] = nblk;
        return;
    }
}

// theta_j = (X^T H X)_jj / (X^T X)_jj from a k x 2k Gram [X]^T [X, HX]
__global__ void rayleigh_quotient_kernel(int k, const double *__restrict__ M, double *__restrict__ theta) {
    int j = threadIdx.x;
    if (j < k) theta[j] = M[j * 2 * k + k + j] / M[j * 2 * k + j];
}

}  // namespace

int launch_cholinv(lobpcg_ctx *ctx, int k, const double *B, double *rinv, hipStream_t s) {
    const double shift = ctx->dtype == LOBPCG_F64 ? 1e-12 : 1e-6;
    cholinv_kernel<<<1, 64, 0, s>>>(k, B, rinv, ctx->dflags, 1e-14, shift);
    return LOBPCG_OK;
}

int launch_rr(lobpcg_ctx *ctx, int k, int nblk, hipStream_t s) {
    if (nblk * k > NMAX) return set_err(ctx, LOBPCG_EUNSUPPORTED, "rr: %d x %d pencil too large", nblk * k, nblk * k);
    double tol = ctx->dtype == LOBPCG_F64 ? 1e-13 : 1e-8;
    rr_kernel<<<1, 64, 0, s>>>(k, nblk, ctx->gram_out, ctx->rr_C, ctx->rr_theta, ctx->dflags, tol);
    return LOBPCG_OK;
}

int launch_rayleigh_quotients(lobpcg_ctx *ctx, int k, hipStream_t s) {
    rayleigh_quotient_kernel<<<1, 64, 0, s>>>(k, ctx->gram_out, ctx->rr_theta);
    return LOBPCG_OK;
}
