// Bandwidth probe: a plain streaming copy in 16-byte vectors, the ceiling the
// memory-bound stencil kernels are measured against.
#include "launch.hpp"

namespace stl {

__global__ __launch_bounds__(256) void k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                long long n) {
    const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
    for (long long q = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; q < n; q += stride)
        dst[q] = src[q];
}

hipError_t launch_probe_copy(const void *src, void *dst, long long nbytes, hipStream_t st) {
    const long long n = nbytes / 16;
    if (n == 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;  // 64 workgroups per CU, grid-stride beyond
    hipLaunchKernelGGL(k_copy16, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                       static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n);
    return hipGetLastError();
}

}  // namespace stl
