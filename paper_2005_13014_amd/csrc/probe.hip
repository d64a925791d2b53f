// Bandwidth probes: the measured HBM ceilings the memory-bound stencil kernels
// are compared with, and the calibration of the traffic counters.  Each lane
// moves four 16-byte vectors per trip, all loads issued before any store, so
// every wave keeps 4 KiB in flight.
#include "launch.hpp"

namespace stl {

constexpr int PROBE_UNROLL = 4, PROBE_BLOCK = 256;

__global__ __launch_bounds__(PROBE_BLOCK) void k_copy16(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                        long long n) {
    const long long stride = static_cast<long long>(gridDim.x) * PROBE_BLOCK * PROBE_UNROLL;
    for (long long base = static_cast<long long>(blockIdx.x) * PROBE_BLOCK * PROBE_UNROLL + threadIdx.x;
         base < n; base += stride) {
        uint4 v[PROBE_UNROLL];
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) {
            const long long q = base + static_cast<long long>(u) * PROBE_BLOCK;
            if (q < n) v[u] = src[q];
        }
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) {
            const long long q = base + static_cast<long long>(u) * PROBE_BLOCK;
            if (q < n) dst[q] = v[u];
        }
    }
}

// Reads n vectors; the XOR of everything read is stored only if it equals a
// value the caller passes (so the loads cannot be dropped, and in practice
// nothing is written).
__global__ __launch_bounds__(PROBE_BLOCK) void k_read16(const uint4 *__restrict__ src, long long n,
                                                        unsigned key, unsigned *__restrict__ sink) {
    const long long stride = static_cast<long long>(gridDim.x) * PROBE_BLOCK * PROBE_UNROLL;
    unsigned acc = 0;
    for (long long base = static_cast<long long>(blockIdx.x) * PROBE_BLOCK * PROBE_UNROLL + threadIdx.x;
         base < n; base += stride) {
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) {
            const long long q = base + static_cast<long long>(u) * PROBE_BLOCK;
            if (q < n) {
                const uint4 v = src[q];
                acc ^= v.x ^ v.y ^ v.z ^ v.w;
            }
        }
    }
    if (acc == key) sink[0] = acc;
}

// Multi-stream probe: nsrc arrays read and one written, 16 bytes per lane
// per array (the traffic mix of the fused kernel: six field streams in, one
// out, the output stored non-temporally as the fused kernel stores it).
constexpr int PROBE_MAX_STREAMS = 8;
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
struct StreamArgs {
    const uint4 *src[PROBE_MAX_STREAMS];
    uint4 *dst;
    int nsrc;
    long long n;  // 16-byte vectors per stream
};

__global__ __launch_bounds__(PROBE_BLOCK) void k_streams(StreamArgs a) {
    const long long stride = static_cast<long long>(gridDim.x) * PROBE_BLOCK * PROBE_UNROLL;
    for (long long base = static_cast<long long>(blockIdx.x) * PROBE_BLOCK * PROBE_UNROLL + threadIdx.x;
         base < a.n; base += stride) {
        uint4 acc[PROBE_UNROLL] = {};
        for (int f = 0; f < a.nsrc; ++f) {
            uint4 v[PROBE_UNROLL];
#pragma unroll
            for (int u = 0; u < PROBE_UNROLL; ++u) {
                const long long q = base + static_cast<long long>(u) * PROBE_BLOCK;
                v[u] = q < a.n ? a.src[f][q] : uint4{};
            }
#pragma unroll
            for (int u = 0; u < PROBE_UNROLL; ++u) {
                acc[u].x ^= v[u].x;
                acc[u].y ^= v[u].y;
                acc[u].z ^= v[u].z;
                acc[u].w ^= v[u].w;
            }
        }
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u) {
            const long long q = base + static_cast<long long>(u) * PROBE_BLOCK;
            if (q < a.n) {
                const u32x4 w = {acc[u].x, acc[u].y, acc[u].z, acc[u].w};
                __builtin_nontemporal_store(w, reinterpret_cast<u32x4 *>(a.dst + q));
            }
        }
    }
}

static unsigned probe_blocks(long long n, long long cap) {
    long long blocks = (n + PROBE_BLOCK * PROBE_UNROLL - 1) / (PROBE_BLOCK * PROBE_UNROLL);
    return static_cast<unsigned>(blocks < cap ? blocks : cap);
}

hipError_t launch_probe_copy(const void *src, void *dst, long long nbytes, hipStream_t st) {
    const long long n = nbytes / 16;
    if (n == 0) return hipSuccess;
    // 64 workgroups per CU (the best measured grid), grid-stride beyond.
    hipLaunchKernelGGL(k_copy16, dim3(probe_blocks(n, 256 * 64)), dim3(PROBE_BLOCK), 0, st,
                       static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n);
    return hipGetLastError();
}

hipError_t launch_probe_read(const void *src, long long nbytes, unsigned key, void *sink, hipStream_t st) {
    const long long n = nbytes / 16;
    if (n == 0) return hipSuccess;
    // 8 workgroups per CU (the best measured grid for reads), grid-stride beyond.
    hipLaunchKernelGGL(k_read16, dim3(probe_blocks(n, 256 * 8)), dim3(PROBE_BLOCK), 0, st,
                       static_cast<const uint4 *>(src), n, key, static_cast<unsigned *>(sink));
    return hipGetLastError();
}

hipError_t launch_probe_streams(const void *const *src, int nsrc, void *dst, long long nbytes, hipStream_t st) {
    if (nsrc < 1 || nsrc > PROBE_MAX_STREAMS) return hipErrorInvalidValue;
    StreamArgs a{};
    for (int f = 0; f < nsrc; ++f) a.src[f] = static_cast<const uint4 *>(src[f]);
    a.dst = static_cast<uint4 *>(dst);
    a.nsrc = nsrc;
    a.n = nbytes / 16;
    if (a.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_streams, dim3(probe_blocks(a.n, 256 * 16)), dim3(PROBE_BLOCK), 0, st, a);
    return hipGetLastError();
}

}  // namespace stl
