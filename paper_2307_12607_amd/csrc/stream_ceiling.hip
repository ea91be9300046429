// Plain HBM streams for gfx950: the measured ceiling the warp kernels are
// compared with. A copy (read + write), a read-only sweep and a write-only
// sweep, 16 bytes per lane, one pass with no grid-stride loop (one
// workgroup per 4 KB of a copy, per 16 KB of a sweep). These were the
// fastest forms measured on MI355X among grid-stride loops of 1024..8192
// workgroups and one-pass unrolled variants (1, 4 and 8 vectors per lane,
// with and without non-temporal hints).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "exwarp.h"
#include "launch.h"

namespace exw {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kThreads = 256;
constexpr int kSweepUnroll = 4;

__global__ __launch_bounds__(kThreads) void stream_copy_kernel(const f32x4 *src, f32x4 *dst,
                                                               int64_t n) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// Reads every vector; the sum feeds a store that only a sum equal to `never`
// makes (the caller passes a NaN, which no sum compares equal to), so the
// loads cannot be dropped and nothing is written.
__global__ __launch_bounds__(kThreads) void stream_read_kernel(const f32x4 *src, int64_t n,
                                                               float never, float *sink) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kThreads * kSweepUnroll + threadIdx.x;
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < kSweepUnroll; ++j) {
        const int64_t i = base + static_cast<int64_t>(j) * kThreads;
        if (i < n) {
            const f32x4 v = src[i];
            s += (v.x + v.y) + (v.z + v.w);
        }
    }
    if (s == never) sink[0] = s;
}

__global__ __launch_bounds__(kThreads) void stream_write_kernel(f32x4 *dst, int64_t n,
                                                                float value) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kThreads * kSweepUnroll + threadIdx.x;
    const f32x4 v = {value, value, value, value};
#pragma unroll
    for (int j = 0; j < kSweepUnroll; ++j) {
        const int64_t i = base + static_cast<int64_t>(j) * kThreads;
        if (i < n) dst[i] = v;
    }
}

unsigned blocks_for(int64_t n, int per_thread) {
    const int64_t per_block = static_cast<int64_t>(kThreads) * per_thread;
    return static_cast<unsigned>((n + per_block - 1) / per_block);
}

}  // namespace

hipError_t launch_stream(int kind, const void *src, void *dst, int64_t bytes, float *sink,
                         hipStream_t stream) {
    const int64_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    switch (kind) {
    case 0:
        hipLaunchKernelGGL(stream_copy_kernel, dim3(blocks_for(n, 1)), dim3(kThreads), 0, stream,
                           static_cast<const f32x4 *>(src), static_cast<f32x4 *>(dst), n);
        break;
    case 1:
        hipLaunchKernelGGL(stream_read_kernel, dim3(blocks_for(n, kSweepUnroll)), dim3(kThreads),
                           0, stream, static_cast<const f32x4 *>(src), n, __builtin_nanf(""),
                           sink);
        break;
    default:
        hipLaunchKernelGGL(stream_write_kernel, dim3(blocks_for(n, kSweepUnroll)),
                           dim3(kThreads), 0, stream, static_cast<f32x4 *>(dst), n, 0.0f);
        break;
    }
    return hipGetLastError();
}

}  // namespace exw
