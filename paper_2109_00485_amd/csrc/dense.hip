// Small dense FP64 steps, each one workgroup (the matrices are at most
// 48 x 48, so the work is latency-bound):
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
constexpr int KM_CHOL = 16;   // Cholesky QR block width bound (kmax)

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// In-place lower Cholesky of the N x N matrix a (row-major, leading dim LD).
// Returns false if a pivot falls below tol.  Any workgroup size.
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
        for (int i = j + 1 + t; i < N; i += blockDim.x) {
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
    __shared__ double y[KM_CHOL * LD];
    if (t < k) {
        const int c = t;
        for (int i = k - 1; i >= 0; --i) {
            double v = (i == c) ? 1.0 : 0.0;
            for (int p = i + 1; p < k; ++p) v -= a[p * LD + i] * y[p * KM_CHOL + c];   // R'[i][p] = L[p][i]
            y[i * KM_CHOL + c] = v / a[i * LD + i];
        }
        for (int i = 0; i < k; ++i) rinv[i * k + c] = sc[i] * y[i * KM_CHOL + c];
    }
}

// Rayleigh-Ritz.  M is the Gram output [X W P]^T [X W P HX HW HP] for nblk_in
// blocks (KA = nblk_in*k rows, KB = 2*KA columns).  One workgroup of
// RR_THREADS threads; every thread owns a fixed set of matrix entries for the
// Jacobi rounds.
constexpr int RR_THREADS = 256;
constexpr int RQ = (NMAX * NMAX + RR_THREADS - 1) / RR_THREADS;

__device__ inline double block_total(double v, double *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x % LOBPCG_WAVE, wave = threadIdx.x / LOBPCG_WAVE;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < RR_THREADS / LOBPCG_WAVE; ++w) t += sh[w];
    return t;
}

__global__ __launch_bounds__(RR_THREADS) void rr_kernel(int k, int nblk_in, const double *__restrict__ M,
                                                        double *__restrict__ Cout, double *__restrict__ theta,
                                                        int *__restrict__ flags, double tol) {
    __shared__ double O[NMAX * LD];
    __shared__ double Abuf[2][NMAX * LD];   // Jacobi rounds alternate between two copies
    __shared__ double Vbuf[2][NMAX * LD];
    __shared__ double sc[NMAX];
    __shared__ int idx[NMAX];
    __shared__ double rot_c[NMAX], rot_s[NMAX];
    __shared__ int partner[NMAX];
    __shared__ double sh[RR_THREADS / LOBPCG_WAVE];
    __shared__ double Ys[NMAX * KM_CHOL];
    double *A = Abuf[0], *V = Vbuf[0];
    const int t = threadIdx.x;
    if (flags[0] & (FLAG_CHOLQR_FAIL | FLAG_RR_FAIL)) return;
    const int KA = nblk_in * k, KB = 2 * KA;
    int nblk = nblk_in;
    for (;;) {
        const int N = nblk * k;
        // pencil from lower blocks; diagonal blocks symmetrised
        for (int e = t; e < N * N; e += RR_THREADS) {
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
        for (int e = t; e < N * N; e += RR_THREADS) {
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
        for (int c = t; c < N; c += RR_THREADS) {
            for (int i = 0; i < N; ++i) {
                double v = A[i * LD + c];
                for (int p = 0; p < i; ++p) v -= O[i * LD + p] * V[p * LD + c];
                V[i * LD + c] = v / O[i * LD + i];
            }
        }
        __syncthreads();
        // A = L^{-1} Z^T  (= L^{-1} G L^{-T} since G is symmetric)
        for (int c = t; c < N; c += RR_THREADS) {
            for (int i = 0; i < N; ++i) {
                double v = V[c * LD + i];
                for (int p = 0; p < i; ++p) v -= O[i * LD + p] * A[p * LD + c];
                A[i * LD + c] = v / O[i * LD + i];
            }
        }
        __syncthreads();
        // this thread's entries (fixed for the whole Jacobi iteration)
        int ei[RQ], ej[RQ];
#pragma unroll
        for (int q = 0; q < RQ; ++q) {
            const int e = t + RR_THREADS * q;
            ei[q] = e < N * N ? e / N : -1;
            ej[q] = e < N * N ? e % N : 0;
        }
        // symmetrise, V = I
        double ra[RQ];
#pragma unroll
        for (int q = 0; q < RQ; ++q)
            if (ei[q] >= 0) ra[q] = 0.5 * (A[ei[q] * LD + ej[q]] + A[ej[q] * LD + ei[q]]);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RQ; ++q)
            if (ei[q] >= 0) {
                A[ei[q] * LD + ej[q]] = ra[q];
                V[ei[q] * LD + ej[q]] = ei[q] == ej[q] ? 1.0 : 0.0;
            }
        __syncthreads();
        // cyclic Jacobi, round-robin pairing over Ne = N rounded up to even:
        // all Ne/2 rotations of a round are disjoint and applied at once as
        // A <- J^T A J, V <- V J, with J acting on index i as
        // (new)_i = c_i (old)_i + s_i (old)_partner(i)
        const int Ne = N + (N & 1);
        for (int sweep = 0; sweep < 30; ++sweep) {
            double off = 0.0, tot = 0.0;
#pragma unroll
            for (int q = 0; q < RQ; ++q)
                if (ei[q] >= 0) {
                    const double v = A[ei[q] * LD + ej[q]];
                    tot += v * v;
                    if (ei[q] != ej[q]) off += v * v;
                }
            off = block_total(off, sh);
            tot = block_total(tot, sh);
            // stop at an off-diagonal norm of 1e-13 of the matrix norm: below that the
            // rounding of the two-sided updates keeps it from shrinking further
            if (off <= 1e-26 * tot || off == 0.0) break;
            for (int r = 0; r < Ne - 1; ++r) {
                if (t < Ne / 2) {
                    const int pos_p = t, pos_q = Ne - 1 - t;
                    int p = pos_p == 0 ? 0 : 1 + (pos_p - 1 + r) % (Ne - 1);
                    int q = 1 + (pos_q - 1 + r) % (Ne - 1);
                    if (p > q) { int tmp = p; p = q; q = tmp; }
                    if (q < N) {
                        double c = 1.0, sn = 0.0;
                        const double apq = A[p * LD + q];
                        if (apq != 0.0) {
                            const double tau = (A[q * LD + q] - A[p * LD + p]) / (2.0 * apq);
                            const double tt = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                            c = 1.0 / sqrt(1.0 + tt * tt);
                            sn = tt * c;
                        }
                        partner[p] = q; partner[q] = p;
                        rot_c[p] = c; rot_s[p] = -sn;
                        rot_c[q] = c; rot_s[q] = sn;
                    } else if (p < N) {
                        partner[p] = p; rot_c[p] = 1.0; rot_s[p] = 0.0;
                    }
                }
                __syncthreads();
                // read the current copies, write the other ones (no write-back pass)
                double *An = (A == Abuf[0]) ? Abuf[1] : Abuf[0];
                double *Vn = (V == Vbuf[0]) ? Vbuf[1] : Vbuf[0];
#pragma unroll
                for (int q = 0; q < RQ; ++q) {
                    if (ei[q] >= 0) {
                        const int i = ei[q], j = ej[q];
                        const int pi = partner[i], pj = partner[j];
                        const double ci = rot_c[i], si = rot_s[i], cj = rot_c[j], sj = rot_s[j];
                        An[i * LD + j] = ci * (cj * A[i * LD + j] + sj * A[i * LD + pj]) +
                                         si * (cj * A[pi * LD + j] + sj * A[pi * LD + pj]);
                        Vn[i * LD + j] = cj * V[i * LD + j] + sj * V[i * LD + pj];
                    }
                }
                A = An;
                V = Vn;
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
            double *y = Ys + t;   // column t of Ys, stride KM_CHOL
            for (int i = N - 1; i >= 0; --i) {
                double v = V[i * LD + col];
                for (int p = i + 1; p < N; ++p) v -= O[p * LD + i] * y[p * KM_CHOL];
                y[i * KM_CHOL] = v / O[i * LD + i];
            }
            for (int i = 0; i < N; ++i) Cout[i * k + t] = sc[i] * y[i * KM_CHOL];
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
    rr_kernel<<<1, RR_THREADS, 0, s>>>(k, nblk, ctx->gram_out, ctx->rr_C, ctx->rr_theta, ctx->dflags, tol);
    return LOBPCG_OK;
}

int launch_rayleigh_quotients(lobpcg_ctx *ctx, int k, hipStream_t s) {
    rayleigh_quotient_kernel<<<1, 64, 0, s>>>(k, ctx->gram_out, ctx->rr_theta);
    return LOBPCG_OK;
}
