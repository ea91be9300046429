// Device helpers shared by the forward and adjoint warp kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace exw {

constexpr int kNumXcd = 8;     // MI355X: 8 XCDs, each with its own L2
constexpr int kSegW = 64;      // one wavefront = 64 consecutive pixels of a row

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(_Float16 v) { return static_cast<float>(v); }
__device__ __forceinline__ float to_f32(__bf16 v) { return static_cast<float>(v); }

// Round-to-nearest-even into the storage type (gfx950 converts float32 ->
// bfloat16 in hardware).
template <typename T>
__device__ __forceinline__ T from_f32(float v) { return static_cast<T>(v); }

// Workgroups are dispatched to the XCDs round-robin (workgroup b runs on XCD
// b % 8). Renumber them so that each XCD receives one contiguous run of
// tiles: neighbouring tiles, which share source rows through the bilinear
// halo, then sit in the same L2.
__device__ __forceinline__ int xcd_tile_index(int b, int nblocks) {
    const int xcd = b % kNumXcd;
    const int local = b / kNumXcd;
    const int per = nblocks / kNumXcd;
    const int extra = nblocks % kNumXcd;
    return xcd * per + min(xcd, extra) + local;
}

// One axis of the sample point p - d, for integer pixel p and float32
// displacement d:
//   ok  <=> 0 <= p - d <= size-1, evaluated as p-(size-1) <= d <= p on float32
//           values, which is exact (p and size-1 are integers below 2^24);
//   i0  = floor(p - d) = p - ceil(d) (exact), i1 = min(i0 + 1, size - 1);
//   f   = (p - d) - i0 = ceil(d) - d, the weight of i1 (float32; exact except
//         when d lies in (0, 1) and 1 - d rounds).
// The absolute position p - d is never formed in float32: at p ~ 4000 that
// would lose up to 2^-12 px. When ok is false the fields are those of d = 0
// (i0 = p, f = 0): finite, but not a tap of the warp.
struct Axis {
    int i0, i1;
    float f;
    bool ok;
};

__device__ __forceinline__ Axis split_axis(float d, int p, int size) {
    Axis a;
    a.ok = (d <= static_cast<float>(p)) && (d >= static_cast<float>(p - (size - 1)));
    // Lanes that are not ok get the split of d = 0, so every field stays
    // finite (weights of invalid lanes are multiplied by zero gradients).
    const float dc = a.ok ? d : 0.0f;
    const float c = ceilf(dc);
    a.i0 = p - static_cast<int>(c);
    a.f = c - dc;
    a.i1 = min(a.i0 + 1, size - 1);
    return a;
}

// Element `i` of a plane whose base pointer is uniform across the wavefront:
// the byte offset is formed in 32 bits (the C-ABI caps a plane at 2^30
// pixels, 4 GB of float32), so the access can use a scalar base register plus
// a 32-bit vector offset instead of 64-bit vector address arithmetic.
template <typename T>
__device__ __forceinline__ const T *at(const T *base, uint32_t i) {
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) +
                                       i * static_cast<uint32_t>(sizeof(T)));
}
template <typename T>
__device__ __forceinline__ T *at(T *base, uint32_t i) {
    return reinterpret_cast<T *>(reinterpret_cast<char *>(base) +
                                 i * static_cast<uint32_t>(sizeof(T)));
}

// Two horizontally adjacent stored values p[0], p[1] in one load. The address
// is only element-aligned; gfx950 serves unaligned global loads.
typedef float f32x2_u __attribute__((ext_vector_type(2), aligned(4)));
typedef uint32_t u32_u __attribute__((aligned(2)));

__device__ __forceinline__ void load_pair(const float *p, float &a, float &b) {
    const f32x2_u v = *reinterpret_cast<const f32x2_u *>(p);
    a = v.x;
    b = v.y;
}

__device__ __forceinline__ float half_bits_to_f32(uint32_t bits, _Float16 *) {
    _Float16 h;
    const uint16_t b16 = static_cast<uint16_t>(bits);
    __builtin_memcpy(&h, &b16, 2);
    return static_cast<float>(h);
}

__device__ __forceinline__ float half_bits_to_f32(uint32_t bits, __bf16 *) {
    return __uint_as_float((bits & 0xffffu) << 16);
}

template <typename T>
__device__ __forceinline__ void load_pair(const T *p, float &a, float &b) {
    const uint32_t v = *reinterpret_cast<const u32_u *>(p);
    a = half_bits_to_f32(v, static_cast<T *>(nullptr));
    b = half_bits_to_f32(v >> 16, static_cast<T *>(nullptr));
}

// Wavefront-wide min / max over all 64 lanes (DPP + readlane, result in every
// lane; every lane must be active).
__device__ __forceinline__ int wave_min(int v) { return __ockl_wfred_min_i32(v); }
__device__ __forceinline__ int wave_max(int v) { return __ockl_wfred_max_i32(v); }

}  // namespace exw
