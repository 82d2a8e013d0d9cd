// Small dense FP64 steps, each one workgroup (the matrices are at most
// 48 x 48, so the work is latency-bound):
//  * Cholesky factor and triangular inverse for Cholesky QR (Section 3.5):
//    B = W^T W = R^T R, then R^{-1} is applied to W by the combine kernel;
//  * Rayleigh-Ritz (eq. rreig): assemble G = S^T H S and O = S^T S from the
//    lower blocks of eq. Glower, scale both by diag(O)^{-1/2} (equivalent to
//    normalising the columns of S), Cholesky O = L L^T, A = L^{-1} G L^{-T},
//    cyclic Jacobi with a round-robin pairing (all N/2 rotations of a round
//    are disjoint and applied at once, in place, by 2 x 2 blocks), sort ascending, C = diag(O)^{-1/2}
//    L^{-T} V[:, :k].  If O is not positive definite with P, P is dropped
//    and the step repeated with S = [X, W].
#include <cfloat>

#include "internal.hpp"

namespace {

constexpr int NMAX = 48;
constexpr int LD = NMAX + 1;
constexpr int KM_CHOL = 16;   // Cholesky QR block width bound (kmax)

// 1/x and 1/sqrt(x) for positive normal x: the hardware estimates refined by
// two Newton steps (each doubles the correct bits; a few ulp at the end).  A
// Jacobi rotation needs c^2 + s^2 = 1 to rounding, not correctly rounded
// quotients, and this chain is on the critical path of every round.
__device__ inline double recip_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}

__device__ inline double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// In-place lower Cholesky of the N x N matrix a (row-major, leading dim LD).
// Returns false if a pivot falls below tol.  Any workgroup size.  Right-looking:
// after column j is scaled, every thread subtracts its share of the rank-1
// update from the trailing lower triangle, so no thread runs a long dependent
// dot product; each entry still receives its updates in the order p = 0, 1, ...
__device__ bool chol_lower(double *a, int N, double tol) {
    const int t = threadIdx.x;
    __shared__ int bad;
    if (t == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < N; ++j) {
        if (t == 0) {
            const double d = a[j * LD + j];
            if (!(d > tol)) bad = 1;
            a[j * LD + j] = d > 0 ? sqrt(d) : 1.0;
        }
        __syncthreads();
        const double piv = a[j * LD + j];
        for (int i = j + 1 + t; i < N; i += blockDim.x) a[i * LD + j] /= piv;
        __syncthreads();
        // trailing lower triangle over a 16-column thread grid (no integer division)
        const int tr = t / 16, tc = t % 16, TR = blockDim.x / 16;
        for (int i = j + 1 + tr; i < N; i += TR) {
            const double aij = a[i * LD + j];
            for (int l = j + 1 + tc; l <= i; l += 16) a[i * LD + l] -= aij * a[l * LD + j];
        }
        __syncthreads();
    }
    return bad == 0;
}

// Cholesky QR factor R^{-1} of a block W (Section 3.5).
//   FUSED = false: B is W^T W (k x k).
//   FUSED = true:  B is the 2k x 2k Gram of [X W] and W is first projected,
//     W' = W - X C with C = X^T W; the Gram of W' follows from B without
//     another pass over the rows: W'^T W' = W^T W - C^T C - C^T C + C^T (X^T X) C
//     (exact for any X).  The kernel also writes m2 = -C R^{-1}, so that one
//     combine pass W <- W R^{-1} + X m2 gives the orthonormalised projection.
// One wavefront.
template <bool FUSED>
__global__ __launch_bounds__(64) void cholinv_kernel(int k, const double *__restrict__ B, double *__restrict__ rinv,
                                                     double *__restrict__ m2, int *__restrict__ flags, double tol,
                                                     double shift) {
    __shared__ double a[NMAX * LD];
    __shared__ double sc[NMAX];
    __shared__ double cs[FUSED ? KM_CHOL * KM_CHOL : 1], ts[FUSED ? KM_CHOL * KM_CHOL : 1];
    __shared__ double bp[FUSED ? KM_CHOL * KM_CHOL : 1];
    const int t = threadIdx.x;
    if (flags[0] & (FLAG_CHOLQR_FAIL | FLAG_RR_FAIL)) return;
    const int k2 = 2 * k;
    if constexpr (FUSED) {
        for (int e = t; e < k2 * k2; e += LOBPCG_WAVE) a[(e / k2) * LD + e % k2] = B[e];
        __syncthreads();
        // C = X^T W (both off-diagonal blocks averaged), then T = (X^T X) C
        for (int e = t; e < k * k; e += LOBPCG_WAVE) {
            const int i = e / k, j = e % k;
            cs[i * KM_CHOL + j] = 0.5 * (a[i * LD + k + j] + a[(k + j) * LD + i]);
        }
        __syncthreads();
        for (int e = t; e < k * k; e += LOBPCG_WAVE) {
            const int i = e / k, j = e % k;
            double v = 0.0;
            for (int p = 0; p < k; ++p) v += 0.5 * (a[i * LD + p] + a[p * LD + i]) * cs[p * KM_CHOL + j];
            ts[i * KM_CHOL + j] = v;
        }
        __syncthreads();
        // projected Gram: W^T W + sum_p C[p][i] (T[p][j] - 2 C[p][j])
        for (int e = t; e < k * k; e += LOBPCG_WAVE) {
            const int i = e / k, j = e % k;
            double v = a[(k + i) * LD + k + j];
            for (int p = 0; p < k; ++p) v += cs[p * KM_CHOL + i] * (ts[p * KM_CHOL + j] - 2.0 * cs[p * KM_CHOL + j]);
            bp[i * KM_CHOL + j] = v;
        }
        __syncthreads();
    }
    // soft-locked columns are absent: identity rows and columns (R^{-1} leaves them alone)
    const int lock = flags[3];
    auto entry = [&](int i, int j) -> double {
        if (((lock >> i) | (lock >> j)) & 1) return i == j ? 1.0 : 0.0;
        if constexpr (FUSED) return 0.5 * (bp[i * KM_CHOL + j] + bp[j * KM_CHOL + i]);
        return 0.5 * (B[i * k + j] + B[j * k + i]);
    };
    for (int e = t; e < k * k; e += LOBPCG_WAVE) {
        int i = e / k, j = e % k;
        a[i * LD + j] = entry(i, j);
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
    const int force = flags[2];
    bool ok = posdiag && chol_lower(a, k, tol) && !(force & (FORCE_CHOLQR_UNSHIFTED | FORCE_CHOLQR));
    if (posdiag && !ok) {
        // shifted Cholesky QR: factor B' + shift I (B' has unit diagonal)
        for (int e = t; e < k * k; e += LOBPCG_WAVE) {
            int i = e / k, j = e % k;
            const bool locked = ((lock >> i) | (lock >> j)) & 1;
            a[i * LD + j] = entry(i, j) * sc[i] * sc[j] + (i == j && !locked ? shift : 0.0);
        }
        __syncthreads();
        ok = chol_lower(a, k, tol) && !(force & FORCE_CHOLQR);
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
        for (int i = 0; i < k; ++i) {
            y[i * KM_CHOL + c] *= sc[i];
            rinv[i * k + c] = y[i * KM_CHOL + c];
        }
    }
    if constexpr (FUSED) {
        __syncthreads();
        // m2 = -C R^{-1}
        for (int e = t; e < k * k; e += LOBPCG_WAVE) {
            const int i = e / k, c = e % k;
            double v = 0.0;
            for (int p = 0; p < k; ++p) v += cs[i * KM_CHOL + p] * y[p * KM_CHOL + c];
            m2[i * k + c] = -v;
        }
    }
}

// Rayleigh-Ritz.  M is the Gram output [X W P]^T [X W P HX HW HP] for nblk_in
// blocks (KA = nblk_in*k rows, KB = 2*KA columns).  One workgroup of
// RR_THREADS threads.
//
// Jacobi rounds update in place by 2 x 2 blocks: a round pairs the indices
// into disjoint pairs (p_a, q_a); the entries of A with rows in pair a and
// columns in pair b depend only on each other (A' = J_a^T A[a, b] J_b), so
// one thread reads, rotates and writes one block and its mirror (a <= b only,
// which keeps A exactly symmetric), and one thread rotates one row of V for
// one pair (V' = V J).  Every thread derives the pairs of a round from the
// round number, so its loads of A, V and of the rotations are independent.
constexpr int RR_THREADS = 256;
constexpr int NPAIR = NMAX / 2;
// Jacobi units per thread: A blocks (a <= b) and V blocks of a pencil of up to
// 2 np indices; the kernel is compiled for 1 (up to 24 indices, the k = 8
// pencils), 2 (32) and 4 (48) units per thread
__host__ __device__ constexpr int rr_units(int np) { return (np * (np + 1) / 2 + np * np + RR_THREADS - 1) / RR_THREADS; }
static_assert(rr_units(12) == 1 && rr_units(16) == 2 && rr_units(NPAIR) == 4, "Jacobi units per thread");

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

// Pair a of round r of the round-robin ordering over Ne (even) indices:
// position 0 stays, the others rotate; returns p < q (q = Ne - 1 may be a
// dummy index when the order is odd).
__device__ inline void rr_pair(int a, int r, int Ne, int &p, int &q) {
    int x = 0;
    if (a > 0) {
        x = a - 1 + r;
        if (x >= Ne - 1) x -= Ne - 1;
        x += 1;
    }
    int y = Ne - 2 - a + r;
    if (y >= Ne - 1) y -= Ne - 1;
    y += 1;
    p = x < y ? x : y;
    q = x < y ? y : x;
}

template <int RR_UNITS>
__global__ __launch_bounds__(RR_THREADS) void rr_kernel(int k, int nblk_in, const double *__restrict__ M,
                                                        double *__restrict__ Cout, double *__restrict__ theta,
                                                        int *__restrict__ flags, double tol) {
    __shared__ double O[NMAX * LD];
    __shared__ double A[NMAX * LD];
    __shared__ double V[NMAX * LD];
    __shared__ double sc[NMAX];
    __shared__ int idx[NMAX];
    __shared__ double pr_c[NPAIR], pr_s[NPAIR];
    __shared__ short2 ptab[NMAX - 1][NPAIR];
    __shared__ int act[NMAX];
    __shared__ int nact;
    __shared__ double sh[RR_THREADS / LOBPCG_WAVE];
    __shared__ double Ys[NMAX * KM_CHOL];
    const int t = threadIdx.x;
    if (flags[0] & (FLAG_CHOLQR_FAIL | FLAG_RR_FAIL)) return;
    const int KA = nblk_in * k, KB = 2 * KA;
    int nblk = nblk_in;
    // a 16-column thread grid for the entry-wise loops (no integer division)
    const int tr = t / 16, tc = t % 16, TR = RR_THREADS / 16;
    // soft-locked columns of W and P (bit j of flags[3]) are left out of the pencil
    const int lock = flags[3];
    for (;;) {
        const int Nfull = nblk * k;
        if (t == 0) {
            int m = 0;
            for (int i = 0; i < Nfull; ++i) {
                const int col = i - k * ((i >= k) + (i >= 2 * k));
                if (i < k || !((lock >> col) & 1)) act[m++] = i;
            }
            nact = m;
        }
        __syncthreads();
        const int N = nact;
        // pencil from lower blocks; diagonal blocks symmetrised
        for (int a = tr; a < N; a += TR)
            for (int b = tc; b < N; b += 16) {
                const int ia = act[a], ib = act[b];
                const int ba = (ia >= k) + (ia >= 2 * k), bb = (ib >= k) + (ib >= 2 * k);
                double o, g;
                if (ba > bb) {
                    o = M[ia * KB + ib];
                    g = M[ia * KB + KA + ib];
                } else if (ba < bb) {
                    o = M[ib * KB + ia];
                    g = M[ib * KB + KA + ia];
                } else {
                    o = 0.5 * (M[ia * KB + ib] + M[ib * KB + ia]);
                    g = 0.5 * (M[ia * KB + KA + ib] + M[ib * KB + KA + ia]);
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
        for (int a = tr; a < N; a += TR)
            for (int b = tc; b < N; b += 16) {
                O[a * LD + b] *= sc[a] * sc[b];
                A[a * LD + b] *= sc[a] * sc[b];
            }
        __syncthreads();
        const int force = flags[2];
        bool ok = posdiag && chol_lower(O, N, tol) && !(force & FORCE_RR) && !(nblk == 3 && (force & FORCE_RR_WITH_P));
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
        // Z = L^{-1} G, then A = L^{-1} Z^T (= L^{-1} G L^{-T}, G symmetric), both by
        // right-looking forward substitution over a 16-column thread grid: at step p
        // row p is divided by L_pp, then every later row subtracts L_ip times it, so
        // each entry receives its updates in the order p = 0, 1, ... and no thread
        // runs a long dependent chain
        {
            auto forward = [&](double *Z) {
                for (int p = 0; p < N; ++p) {
                    for (int c = t; c < N; c += RR_THREADS) Z[p * LD + c] /= O[p * LD + p];
                    __syncthreads();
                    for (int i = p + 1 + tr; i < N; i += TR) {
                        const double lip = O[i * LD + p];
                        for (int c = tc; c < N; c += 16) Z[i * LD + c] -= lip * Z[p * LD + c];
                    }
                    __syncthreads();
                }
            };
            for (int i = tr; i < N; i += TR)
                for (int c = tc; c < N; c += 16) V[i * LD + c] = A[i * LD + c];
            __syncthreads();
            forward(V);
            for (int i = tr; i < N; i += TR)
                for (int c = tc; c < N; c += 16) A[i * LD + c] = V[c * LD + i];
            __syncthreads();
            forward(A);
        }
        // symmetrise (both triangles from their average), V = I
        for (int i = tr; i < N; i += TR)
            for (int j = tc; j < N; j += 16) {
                V[i * LD + j] = i == j ? 1.0 : 0.0;
                if (i > j) {
                    const double v = 0.5 * (A[i * LD + j] + A[j * LD + i]);
                    A[i * LD + j] = v;
                    A[j * LD + i] = v;
                }
            }
        __syncthreads();
        // cyclic Jacobi, round-robin pairing over Ne = N rounded up to even
        // (index N, if present, is a dummy whose rotation is the identity).  The
        // pairs of every round are tabulated once; a round's work is a list of
        // units, each one 2 x 2 block of A (pairs a <= b) or of V (row pair a,
        // column pair b), at most two per thread, so a thread's instructions per
        // round are few and the same for all rounds.
        const int Ne = N + (N & 1), NP = Ne / 2, NB = NP * (NP + 1) / 2, NU = NB + NP * NP;
        for (int e = t; e < (Ne - 1) * NP; e += RR_THREADS) {
            const int r = e / NP, a = e % NP;
            int p, q;
            rr_pair(a, r, Ne, p, q);
            ptab[r][a] = make_short2((short)p, (short)q);
        }
        // this thread's units (u < NB: A block (a, b), a <= b; else V block), fixed for all rounds
        int ua[RR_UNITS], ub[RR_UNITS];
        bool uv[RR_UNITS];
#pragma unroll
        for (int m = 0; m < RR_UNITS; ++m) {
            const int u = t + RR_THREADS * m;
            int a = -1, b = 0;
            if (u < NB) {
                int rem = u;
                a = 0;
                while (rem >= NP - a) {
                    rem -= NP - a;
                    ++a;
                }
                b = a + rem;
            } else if (u < NU) {
                a = (u - NB) / NP;
                b = (u - NB) % NP;
            }
            ua[m] = a;
            ub[m] = b;
            uv[m] = u >= NB;
        }
        __syncthreads();
        for (int sweep = 0; sweep < 30; ++sweep) {
            double off = 0.0, tot = 0.0;
            for (int i = tr; i < N; i += TR)
                for (int j = tc; j < N; j += 16) {
                    const double v = A[i * LD + j];
                    tot += v * v;
                    if (i != j) off += v * v;
                }
            off = block_total(off, sh);
            tot = block_total(tot, sh);
            // stop at an off-diagonal norm of 1e-13 of the matrix norm: below that the
            // rounding of the two-sided updates keeps it from shrinking further
            if (off <= 1e-26 * tot || off == 0.0) break;
            for (int r = 0; r < Ne - 1; ++r) {
                if (t < NP) {
                    const short2 pq = ptab[r][t];
                    const int p = pq.x, q = pq.y;
                    // tan of the angle that annihilates a_pq: the root of smaller
                    // magnitude of t^2 + 2 t (a_qq - a_pp) / (2 a_pq) - 1 = 0
                    double c = 1.0, sn = 0.0;
                    if (q < N) {
                        const double g2 = 2.0 * A[p * LD + q];
                        const double h = A[q * LD + q] - A[p * LD + p];
                        const double r2 = h * h + g2 * g2;
                        if (g2 != 0.0 && r2 >= DBL_MIN) {   // below: both negligible, no rotation
                            const double rad = r2 * rsqrt_nr(r2);
                            const double tt = (h >= 0 ? g2 : -g2) * recip_nr(fabs(h) + rad);
                            c = rsqrt_nr(fma(tt, tt, 1.0));
                            sn = tt * c;
                        }
                    }
                    pr_c[t] = c;
                    pr_s[t] = sn;
                }
                __syncthreads();
#pragma unroll
                for (int m = 0; m < RR_UNITS; ++m) {
                    if (ua[m] < 0) continue;
                    const short2 pa = ptab[r][ua[m]], pb = ptab[r][ub[m]];
                    const int p1 = pa.x, q1 = pa.y, p2 = pb.x, q2 = pb.y;
                    const bool v1 = q1 < N, v2 = q2 < N;
                    const double c2 = pr_c[ub[m]], s2 = pr_s[ub[m]];
                    if (uv[m]) {
                        // V <- V J on rows p1, q1 and the column pair (p2, q2)
                        if (!v2) continue;   // a dummy column pair: the identity
                        const double x11 = V[p1 * LD + p2], x12 = V[p1 * LD + q2];
                        const double x21 = v1 ? V[q1 * LD + p2] : 0.0, x22 = v1 ? V[q1 * LD + q2] : 0.0;
                        V[p1 * LD + p2] = c2 * x11 - s2 * x12;
                        V[p1 * LD + q2] = s2 * x11 + c2 * x12;
                        if (v1) {
                            V[q1 * LD + p2] = c2 * x21 - s2 * x22;
                            V[q1 * LD + q2] = s2 * x21 + c2 * x22;
                        }
                        continue;
                    }
                    // A <- J^T A J on the block: new column p = c p - s q, new column q = s p + c q
                    const double c1 = pr_c[ua[m]], s1 = pr_s[ua[m]];
                    const double x11 = A[p1 * LD + p2];
                    const double x12 = v2 ? A[p1 * LD + q2] : 0.0;
                    const double x21 = v1 ? A[q1 * LD + p2] : 0.0;
                    const double x22 = v1 && v2 ? A[q1 * LD + q2] : 0.0;
                    const double y11 = c2 * x11 - s2 * x12, y12 = s2 * x11 + c2 * x12;
                    const double y21 = c2 * x21 - s2 * x22, y22 = s2 * x21 + c2 * x22;
                    const double z11 = c1 * y11 - s1 * y21, z21 = s1 * y11 + c1 * y21;
                    const double z12 = c1 * y12 - s1 * y22, z22 = s1 * y12 + c1 * y22;
                    if (ua[m] == ub[m]) {
                        // the rotated pair: its off-diagonal entry is annihilated
                        A[p1 * LD + p1] = z11;
                        if (v1) {
                            A[q1 * LD + q1] = z22;
                            A[p1 * LD + q1] = 0.0;
                            A[q1 * LD + p1] = 0.0;
                        }
                    } else {
                        A[p1 * LD + p2] = z11;
                        A[p2 * LD + p1] = z11;
                        if (v2) {
                            A[p1 * LD + q2] = z12;
                            A[q2 * LD + p1] = z12;
                        }
                        if (v1) {
                            A[q1 * LD + p2] = z21;
                            A[p2 * LD + q1] = z21;
                        }
                        if (v1 && v2) {
                            A[q1 * LD + q2] = z22;
                            A[q2 * LD + q1] = z22;
                        }
                    }
                }
                __syncthreads();
            }
        }
        // ascending order (ties by index)
        for (int i0 = t; i0 < N; i0 += RR_THREADS) {
            double li = A[i0 * LD + i0];
            int rank = 0;
            for (int j = 0; j < N; ++j) {
                double lj = A[j * LD + j];
                rank += (lj < li) || (lj == li && j < i0);
            }
            idx[rank] = i0;
        }
        __syncthreads();
        // C = diag(sc) L^{-T} V[:, idx[0..k)]: right-looking back substitution over
        // a 16-column thread grid (row i is divided by L_ii, then every earlier row
        // subtracts L_ip times it)
        {
            for (int i = tr; i < N; i += TR)
                for (int c = tc; c < k; c += 16) Ys[i * KM_CHOL + c] = V[i * LD + idx[c]];
            __syncthreads();
            for (int i = N - 1; i >= 0; --i) {
                for (int c = t; c < k; c += RR_THREADS) Ys[i * KM_CHOL + c] /= O[i * LD + i];
                __syncthreads();
                for (int p = tr; p < i; p += TR) {
                    const double lip = O[i * LD + p];
                    for (int c = tc; c < k; c += 16) Ys[p * KM_CHOL + c] -= lip * Ys[i * KM_CHOL + c];
                }
                __syncthreads();
            }
            for (int i = tr; i < N; i += TR)
                for (int c = tc; c < k; c += 16) Cout[act[i] * k + c] = sc[i] * Ys[i * KM_CHOL + c];
            // left-out columns take no part in the update
            if (N < Nfull)
                for (int i = tr; i < Nfull; i += TR) {
                    const int col = i - k * ((i >= k) + (i >= 2 * k));
                    if (i >= k && ((lock >> col) & 1))
                        for (int c = tc; c < k; c += 16) Cout[i * k + c] = 0.0;
                }
            if (t < k) theta[t] = A[idx[t] * LD + idx[t]];
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
    cholinv_kernel<false><<<1, 64, 0, s>>>(k, B, rinv, nullptr, ctx->dflags, 1e-14, shift);
    return LOBPCG_OK;
}

int launch_cholinv_projected(lobpcg_ctx *ctx, int k, const double *B2, double *rinv, double *m2, hipStream_t s) {
    if (k > KM_CHOL) return set_err(ctx, LOBPCG_EUNSUPPORTED, "cholqr: k=%d above %d", k, KM_CHOL);
    const double shift = ctx->dtype == LOBPCG_F64 ? 1e-12 : 1e-6;
    cholinv_kernel<true><<<1, 64, 0, s>>>(k, B2, rinv, m2, ctx->dflags, 1e-14, shift);
    return LOBPCG_OK;
}

int launch_rr(lobpcg_ctx *ctx, int k, int nblk, hipStream_t s) {
    if (nblk * k > NMAX) return set_err(ctx, LOBPCG_EUNSUPPORTED, "rr: %d x %d pencil too large", nblk * k, nblk * k);
    // smallest squared pivot accepted in the Cholesky of the unit-diagonal O: below
    // it the basis has nearly lost a direction and the reduced pencil can yield
    // Ritz values outside the spectrum (measured on a nearly diagonal matrix with
    // the shift at theta_j: pivots of 1e-14 and, from some starts, 1e-9 were
    // followed by Ritz values below the lowest eigenvalue), so P is dropped
    // instead.  FP32 blocks keep 1e-8: at 1e-7 their rounding alone trips the test
    // there and the iteration, without P, stalls
    const double tol = ctx->dtype == LOBPCG_F64 ? 1e-7 : 1e-8;
    const int N = nblk * k, np = (N + 1) / 2;
    if (np <= 12)
        rr_kernel<1><<<1, RR_THREADS, 0, s>>>(k, nblk, ctx->gram_out, ctx->rr_C, ctx->rr_theta, ctx->dflags, tol);
    else if (np <= 16)
        rr_kernel<2><<<1, RR_THREADS, 0, s>>>(k, nblk, ctx->gram_out, ctx->rr_C, ctx->rr_theta, ctx->dflags, tol);
    else
        rr_kernel<rr_units(NPAIR)><<<1, RR_THREADS, 0, s>>>(k, nblk, ctx->gram_out, ctx->rr_C, ctx->rr_theta, ctx->dflags, tol);
    return LOBPCG_OK;
}

int launch_rayleigh_quotients(lobpcg_ctx *ctx, int k, hipStream_t s) {
    rayleigh_quotient_kernel<<<1, 64, 0, s>>>(k, ctx->gram_out, ctx->rr_theta);
    return LOBPCG_OK;
}
