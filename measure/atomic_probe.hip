// Measurement probe for profiling (not part of the method or of the library's ABI): reps passes
// of one global float atomic add of 1.0 (no return value) to each of y[i * stride], i < n.
// Distinct addresses; stride 1 = consecutive (many lanes per L2 request), stride 32 = one
// 128-byte line per lane, like the scattered window flushes of the J^T scatter.  The L2 atomic
// request rate of the J^T J v kernel is compared with this probe's under rocprofv3.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_atomic_probe(float* __restrict__ y, int64_t n, int reps, int stride) {
    for (int r = 0; r < reps; ++r)
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
            unsafeAtomicAdd(y + i * stride, 1.0f);
}

}  // namespace

extern "C" {

// 0 on success, -1 for bad arguments, -3 if the launch failed.  d_y [n * stride] is
// caller-owned device memory; asynchronous on stream (a hipStream_t, NULL = default stream).
int32_t probe_atomic_add(float* d_y, int64_t n, int32_t reps, int32_t stride, void* stream) {
    if (n < 0 || reps < 0 || stride < 1 || (n > 0 && !d_y) || (n > 0 && (n - 1) > ((int64_t)1 << 40))) return -1;
    if (n == 0 || reps == 0) return 0;
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_atomic_probe, dim3((unsigned)g), dim3(kBlock), 0, (hipStream_t)stream, d_y, n, reps, stride);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
