// Symmetric sparse x block-of-vectors product Y = H X from the stored upper
// triangle (Algorithm 2 applied to the stored part and its transpose,
// Section 3.2): each stored off-diagonal h_ij, i < j, adds h_ij X_j to Y_i
// (row part) and h_ij X_i to Y_j (transposed part); the diagonal adds d_i X_i.
//
// CSR path: a group of L lanes (L = next power of two >= k) owns one row;
// lane q of the group holds component q.  The row part accumulates in a
// register; the transposed part is scattered with hardware float atomics
// (the paper's OpenACC kernels also rely on atomics, which are cheap when
// conflicts are rare, Section 4.2).  Adjacent rows have similar stored
// lengths in these matrices, so rows of one wavefront finish together.
#include "internal.hpp"

namespace {

template <typename T>
__global__ void fill_zero_kernel(T *__restrict__ p, int64_t count) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < count; i += stride) p[i] = T(0);
}

template <typename T, int L>
__global__ __launch_bounds__(256) void spmm_csr_rows(int64_t n, int k, const int64_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     const T *__restrict__ val, const T *__restrict__ diag,
                                                     const T *__restrict__ X, T *__restrict__ Y) {
    const int q = threadIdx.x % L;
    const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / L;
    if (i >= n || q >= k) return;
    const T xi = X[i * k + q];
    T acc = diag[i] * xi;
    const int64_t b = rp[i], e = rp[i + 1];
    for (int64_t p = b; p < e; ++p) {
        const int64_t j = ci[p];
        const T v = val[p];
        acc += v * X[j * k + q];
        unsafeAtomicAdd(&Y[j * k + q], v * xi);
    }
    unsafeAtomicAdd(&Y[i * k + q], acc);
}

template <typename T>
int spmm_csr(lobpcg_ctx *ctx, const T *X, T *Y, int k, hipStream_t s) {
    const int64_t n = ctx->n;
    const int64_t count = n * k;
    int zb = (int)std::min<int64_t>((count + 255) / 256, 65536);
    fill_zero_kernel<T><<<zb, 256, 0, s>>>(Y, count);
    const T *val = (const T *)ctx->val, *diag = (const T *)ctx->diag;
    if (k <= 4) {
        spmm_csr_rows<T, 4><<<ceil_div(n * 4, 256), 256, 0, s>>>(n, k, ctx->rp, ctx->ci, val, diag, X, Y);
    } else if (k <= 8) {
        spmm_csr_rows<T, 8><<<ceil_div(n * 8, 256), 256, 0, s>>>(n, k, ctx->rp, ctx->ci, val, diag, X, Y);
    } else {
        spmm_csr_rows<T, 16><<<ceil_div(n * 16, 256), 256, 0, s>>>(n, k, ctx->rp, ctx->ci, val, diag, X, Y);
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

int tiled_format_worthwhile(lobpcg_ctx *ctx, hipStream_t s, int *yes) {
    (void)ctx;
    (void)s;
    *yes = 0;
    return LOBPCG_OK;
}

int build_tiled_format(lobpcg_ctx *ctx, hipStream_t s) {
    (void)s;
    return set_err(ctx, LOBPCG_EUNSUPPORTED, "tiled format not built yet");
}

int launch_spmm(lobpcg_ctx *ctx, const void *X, void *Y, int k, hipStream_t s) {
    if (ctx->dtype == LOBPCG_F32) return spmm_csr<float>(ctx, (const float *)X, (float *)Y, k, s);
    return spmm_csr<double>(ctx, (const double *)X, (double *)Y, k, s);
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
