// diag.hip -- HBM streaming read for the bandwidth record of the benchmark
// (libbem_diag.so, not part of the solver library).  Each workgroup streams
// one contiguous panel of the buffer with 16-byte non-temporal loads, the
// access pattern that reads HBM fastest on this GPU; the measured rate is the
// practical read ceiling the product kernels are compared with.
#include <hip/hip_runtime.h>

namespace {

typedef double dv2 __attribute__((ext_vector_type(2)));

// Sum the panel [b0, b1) of 16-byte elements; the store never happens for a
// buffer of ones (its sums are integers), it only keeps the loads alive.
template <int U>
__global__ __launch_bounds__(256) void k_stream_read(const dv2* __restrict__ a, size_t n, size_t per_block,
                                                     double* __restrict__ sink)
{
    const size_t b0 = (size_t)blockIdx.x * per_block;
    const size_t b1 = b0 + per_block < n ? b0 + per_block : n;
    double s = 0.0;
    size_t i = b0 + threadIdx.x;
    for (; i + (U - 1) * 256 < b1; i += U * 256) {
        dv2 v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = __builtin_nontemporal_load(a + i + k * 256);
#pragma unroll
        for (int k = 0; k < U; ++k) s += v[k].x + v[k].y;
    }
    for (; i < b1; i += 256) s += a[i].x + a[i].y;
    if (s == 0.5) sink[blockIdx.x] = s;
}

}  // namespace

extern "C" {

// Read `bytes` (a multiple of 16) from the device buffer `buf` with `grid`
// workgroups of 256 threads, `unroll` (4 or 8) loads in flight per thread.
// `sink` is device memory of at least `grid` doubles (never written for a
// buffer of ones).  Enqueued on `stream`; returns the hipError_t of the launch.
int bem_diag_stream_read(const void* buf, size_t bytes, int grid, int unroll, double* sink, hipStream_t stream)
{
    if (!buf || !sink || grid < 1 || bytes % 16 != 0 || (unroll != 4 && unroll != 8))
        return (int)hipErrorInvalidValue;
    const size_t n = bytes / 16;
    const size_t per = (n + grid - 1) / grid;
    const dv2* a = static_cast<const dv2*>(buf);
    if (unroll == 8)
        hipLaunchKernelGGL((k_stream_read<8>), dim3(grid), dim3(256), 0, stream, a, n, per, sink);
    else
        hipLaunchKernelGGL((k_stream_read<4>), dim3(grid), dim3(256), 0, stream, a, n, per, sink);
    return (int)hipGetLastError();
}

}  // extern "C"
