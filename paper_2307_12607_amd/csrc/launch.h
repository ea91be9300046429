// Internal interface between the C-ABI layer (api.cpp) and the HIP kernels
// (warp_kernels.hip). Arguments arrive here already validated.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace exw {

struct WarpShape {
    int n, c, h, w, k;
    float phases[4];
};

hipError_t launch_forward(int dtype, const void *src, const float *mv, const WarpShape &s,
                          void *out, uint8_t *mask, uint32_t *count, hipStream_t stream);

// accum: float32 [N,C,H,W] image-gradient accumulator (grad_src itself for
// float32 storage, else the workspace), or NULL. cast_to: storage-dtype
// grad_src to round the accumulator into, or NULL (float32, or no grad_src).
hipError_t launch_backward(int dtype, const void *src, const float *mv, const WarpShape &s,
                           const void *grad_out, float *accum, void *cast_to, float *grad_mv,
                           hipStream_t stream);

hipError_t launch_zero_u32(uint32_t *p, int64_t count, hipStream_t stream);

}  // namespace exw
