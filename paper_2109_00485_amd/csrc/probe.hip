// Streaming probes of the memory system: plain read, write and copy kernels of
// a known byte count.  They give the achievable HBM bandwidth the sparse
// product is compared with, and the known-size reference that scales the
// hardware traffic counters (FETCH_SIZE, WRITE_SIZE) read for the product.
#include "internal.hpp"

namespace {

constexpr int PROBE_THREADS = 256;
constexpr int PROBE_BLOCKS = 8192;   // 32 workgroups per CU, grid-stride

__global__ __launch_bounds__(PROBE_THREADS) void stream_read_kernel(const float4 *__restrict__ a, int64_t n4,
                                                                     float *__restrict__ sink) {
    float4 s = {0.f, 0.f, 0.f, 0.f};
    for (int64_t i = (int64_t)blockIdx.x * PROBE_THREADS + threadIdx.x; i < n4; i += (int64_t)gridDim.x * PROBE_THREADS) {
        const float4 t = a[i];
        s.x += t.x; s.y += t.y; s.z += t.z; s.w += t.w;
    }
    // the loads stay live through a store the data never triggers in practice
    const float tot = s.x + s.y + s.z + s.w;
    if (tot == -1.2345e30f) sink[0] = tot;
}

__global__ __launch_bounds__(PROBE_THREADS) void stream_write_kernel(float4 *__restrict__ b, int64_t n4) {
    for (int64_t i = (int64_t)blockIdx.x * PROBE_THREADS + threadIdx.x; i < n4; i += (int64_t)gridDim.x * PROBE_THREADS)
        b[i] = make_float4(1.f, 2.f, 3.f, 4.f);
}

__global__ __launch_bounds__(PROBE_THREADS) void stream_copy_kernel(const float4 *__restrict__ a, float4 *__restrict__ b,
                                                                     int64_t n4) {
    for (int64_t i = (int64_t)blockIdx.x * PROBE_THREADS + threadIdx.x; i < n4; i += (int64_t)gridDim.x * PROBE_THREADS)
        b[i] = a[i];
}

}  // namespace

extern "C" int lobpcg_stream_probe(int op, const void *a, void *b, int64_t bytes, void *stream) {
    if (bytes <= 0 || bytes % 16 != 0) return LOBPCG_EINVAL;
    if (((uintptr_t)a | (uintptr_t)b) % 16 != 0) return LOBPCG_EINVAL;
    const int64_t n4 = bytes / 16;
    hipStream_t s = (hipStream_t)stream;
    switch (op) {
        case LOBPCG_PROBE_READ:
            if (!a || !b) return LOBPCG_EINVAL;
            stream_read_kernel<<<PROBE_BLOCKS, PROBE_THREADS, 0, s>>>((const float4 *)a, n4, (float *)b);
            break;
        case LOBPCG_PROBE_WRITE:
            if (!b) return LOBPCG_EINVAL;
            stream_write_kernel<<<PROBE_BLOCKS, PROBE_THREADS, 0, s>>>((float4 *)b, n4);
            break;
        case LOBPCG_PROBE_COPY:
            if (!a || !b || a == b) return LOBPCG_EINVAL;
            stream_copy_kernel<<<PROBE_BLOCKS, PROBE_THREADS, 0, s>>>((const float4 *)a, (float4 *)b, n4);
            break;
        default:
            return LOBPCG_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? LOBPCG_OK : LOBPCG_EHIP;
}
