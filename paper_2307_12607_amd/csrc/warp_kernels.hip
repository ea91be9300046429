// HIP kernels of the motion-vector backward warp for CDNA4 (gfx950).
//
// Forward (paper §II-B image warping; §IV-B the predicted frames at
// t + i/4 all come from F_t; §III-B invalid pixels): every lane owns one
// output pixel, reads its motion vector once and produces all K phases, so
// the motion stream is read once per launch and the K gathers of one pixel
// hit the same neighbourhood of the source frame. Output, mask and motion
// accesses are coalesced across the 64 lanes of a wavefront (one wavefront =
// 64 consecutive pixels of a row); the bilinear taps of neighbouring lanes
// fall on neighbouring addresses whenever the motion is locally smooth.
//
// The gather is HBM-bound, not a contraction, so there is no MFMA here.
//
// Coordinates: the displacement d = s*u is one float32 multiply (the build
// turns off FMA contraction, so it is rounded once). The validity test
// 0 <= x - d <= W-1 is evaluated as x-(W-1) <= d <= x on float32 values,
// which is exact because x and W-1 are small integers; the absolute sample
// position x - d is never formed in float32 (it would lose up to 2^-11 px at
// x ~ 4000). The tap index and the fractional weight come from floor(d).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.h"

namespace exw {
namespace {

constexpr int kTileW = 64;  // one wavefront per tile row
constexpr int kTileH = 4;   // four wavefronts per workgroup
constexpr int kThreads = kTileW * kTileH;
constexpr int kNumXcd = 8;  // MI355X: 8 XCDs, each with its own L2

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(_Float16 v) { return static_cast<float>(v); }
__device__ __forceinline__ float to_f32(__bf16 v) { return static_cast<float>(v); }

// Round-to-nearest-even conversion into the storage type (gfx950 converts
// float32 -> bfloat16 in hardware).
template <typename T>
__device__ __forceinline__ T from_f32(float v) { return static_cast<T>(v); }

// Workgroups are dispatched to the XCDs round-robin (workgroup b runs on XCD
// b % 8). Renumber them so that each XCD receives one contiguous run of
// tiles: vertically adjacent tiles, which share source rows through the
// bilinear halo, then sit in the same L2.
__device__ __forceinline__ int xcd_tile_index(int b, int nblocks) {
    const int xcd = b % kNumXcd;
    const int local = b / kNumXcd;
    const int per = nblocks / kNumXcd;
    const int extra = nblocks % kNumXcd;
    return xcd * per + min(xcd, extra) + local;
}

struct Axis {
    int i0, i1;  // tap indices along this axis
    float f;     // weight of i1 (fraction of the sample point past i0)
    bool ok;     // 0 <= p - d <= size - 1
};

// One axis of the sample point p - d, for integer p and float32 d.
__device__ __forceinline__ Axis split_axis(float d, int p, int size) {
    Axis a;
    a.ok = (d <= static_cast<float>(p)) && (d >= static_cast<float>(p - (size - 1)));
    const float dc = a.ok ? d : 0.0f;  // keeps the integer conversion in range
    const float di = floorf(dc);
    const float df = dc - di;          // in [0, 1); > 0 exactly when d is not an integer
    const int base = p - static_cast<int>(di);
    const bool frac = df > 0.0f;
    a.i0 = frac ? base - 1 : base;
    a.f = frac ? 1.0f - df : 0.0f;
    a.i1 = min(a.i0 + 1, size - 1);
    return a;
}

template <typename T>
struct FwdArgs {
    const T *src;
    const float *mv;
    T *out;
    uint8_t *mask;
    uint32_t *count;
    int n, c, h, w, k;
    int tiles_x, tiles_y;
    float s[4];
};

// CT: channel count known at compile time, or 0 for a runtime loop.
template <typename T, int CT>
__global__ __launch_bounds__(kThreads) void warp_forward_kernel(FwdArgs<T> a) {
    const int C = CT > 0 ? CT : a.c;
    const int b = xcd_tile_index(blockIdx.x, gridDim.x);
    const int tx = b % a.tiles_x;
    const int rest = b / a.tiles_x;
    const int ty = rest % a.tiles_y;
    const int in = rest / a.tiles_y;
    const int x = tx * kTileW + threadIdx.x;
    const int y = ty * kTileH + threadIdx.y;
    const int w = a.w, h = a.h;
    const bool inside = (x < w) && (y < h);
    const int64_t hw = static_cast<int64_t>(h) * w;
    const int64_t p = static_cast<int64_t>(y) * w + x;

    float u = 0.0f, v = 0.0f;
    if (inside) {
        u = a.mv[(2 * static_cast<int64_t>(in)) * hw + p];
        v = a.mv[(2 * static_cast<int64_t>(in) + 1) * hw + p];
    }
    const T *img = a.src + static_cast<int64_t>(in) * C * hw;

    for (int j = 0; j < a.k; ++j) {
        const float s = a.s[j];
        const Axis ax = split_axis(s * u, x, w);
        const Axis ay = split_axis(s * v, y, h);
        const bool valid = inside && ax.ok && ay.ok;
        const int64_t plane = static_cast<int64_t>(in) * a.k + j;
        if (inside) {
            T *o = a.out + plane * C * hw + p;
            if (valid) {
                const float w00 = (1.0f - ax.f) * (1.0f - ay.f);
                const float w01 = ax.f * (1.0f - ay.f);
                const float w10 = (1.0f - ax.f) * ay.f;
                const float w11 = ax.f * ay.f;
                const int64_t r0 = static_cast<int64_t>(ay.i0) * w;
                const int64_t r1 = static_cast<int64_t>(ay.i1) * w;
#pragma unroll
                for (int ch = 0; ch < C; ++ch) {
                    const T *pl = img + ch * hw;
                    float acc = w00 * to_f32(pl[r0 + ax.i0]);
                    acc = fmaf(w01, to_f32(pl[r0 + ax.i1]), acc);
                    acc = fmaf(w10, to_f32(pl[r1 + ax.i0]), acc);
                    acc = fmaf(w11, to_f32(pl[r1 + ax.i1]), acc);
                    o[ch * hw] = from_f32<T>(acc);
                }
            } else {
#pragma unroll
                for (int ch = 0; ch < C; ++ch) o[ch * hw] = from_f32<T>(0.0f);
            }
            if (a.mask) a.mask[plane * hw + p] = valid ? 1 : 0;
        }
        if (a.count) {
            // One atomic per wavefront that saw invalid pixels.
            const unsigned long long bal = __ballot(inside && !valid);
            if (bal != 0ull && __lane_id() == 0)
                atomicAdd(a.count + plane, static_cast<uint32_t>(__popcll(bal)));
        }
    }
}

template <typename T>
struct BwdArgs {
    const T *src;
    const float *mv;
    const T *gout;
    float *accum;
    float *gmv;
    int n, c, h, w, k;
    int tiles_x, tiles_y;
    float s[4];
};

// Adjoint: each valid output pixel sends weight * grad to its four taps
// (float32 atomics into the accumulator) and forms its own motion gradient
// from the same taps, summed over the K phases.
template <typename T, int CT>
__global__ __launch_bounds__(kThreads) void warp_backward_kernel(BwdArgs<T> a) {
    const int C = CT > 0 ? CT : a.c;
    const int b = xcd_tile_index(blockIdx.x, gridDim.x);
    const int tx = b % a.tiles_x;
    const int rest = b / a.tiles_x;
    const int ty = rest % a.tiles_y;
    const int in = rest / a.tiles_y;
    const int x = tx * kTileW + threadIdx.x;
    const int y = ty * kTileH + threadIdx.y;
    const int w = a.w, h = a.h;
    if (x >= w || y >= h) return;
    const int64_t hw = static_cast<int64_t>(h) * w;
    const int64_t p = static_cast<int64_t>(y) * w + x;
    const float u = a.mv[(2 * static_cast<int64_t>(in)) * hw + p];
    const float v = a.mv[(2 * static_cast<int64_t>(in) + 1) * hw + p];
    const T *img = a.src ? a.src + static_cast<int64_t>(in) * C * hw : nullptr;
    float *acc = a.accum ? a.accum + static_cast<int64_t>(in) * C * hw : nullptr;

    float gu = 0.0f, gv = 0.0f;
    for (int j = 0; j < a.k; ++j) {
        const float s = a.s[j];
        const Axis ax = split_axis(s * u, x, w);
        const Axis ay = split_axis(s * v, y, h);
        if (!(ax.ok && ay.ok)) continue;
        const float w00 = (1.0f - ax.f) * (1.0f - ay.f);
        const float w01 = ax.f * (1.0f - ay.f);
        const float w10 = (1.0f - ax.f) * ay.f;
        const float w11 = ax.f * ay.f;
        const int64_t r0 = static_cast<int64_t>(ay.i0) * w;
        const int64_t r1 = static_cast<int64_t>(ay.i1) * w;
        const T *g = a.gout + (static_cast<int64_t>(in) * a.k + j) * C * hw + p;
        float su = 0.0f, sv = 0.0f;
#pragma unroll
        for (int ch = 0; ch < C; ++ch) {
            const float gc = to_f32(g[ch * hw]);
            if (acc) {
                float *pl = acc + ch * hw;
                if (w00 != 0.0f) atomicAdd(pl + r0 + ax.i0, w00 * gc);
                if (w01 != 0.0f) atomicAdd(pl + r0 + ax.i1, w01 * gc);
                if (w10 != 0.0f) atomicAdd(pl + r1 + ax.i0, w10 * gc);
                if (w11 != 0.0f) atomicAdd(pl + r1 + ax.i1, w11 * gc);
            }
            if (a.gmv) {
                const T *pl = img + ch * hw;
                const float i00 = to_f32(pl[r0 + ax.i0]);
                const float i01 = to_f32(pl[r0 + ax.i1]);
                const float i10 = to_f32(pl[r1 + ax.i0]);
                const float i11 = to_f32(pl[r1 + ax.i1]);
                // d out / d sx and d out / d sy of the bilinear blend
                const float dsx = fmaf(ay.f, i11 - i10, (1.0f - ay.f) * (i01 - i00));
                const float dsy = fmaf(ax.f, i11 - i01, (1.0f - ax.f) * (i10 - i00));
                su = fmaf(gc, dsx, su);
                sv = fmaf(gc, dsy, sv);
            }
        }
        // sx = x - s*u, so d sx / d u = -s (and likewise for v)
        gu = fmaf(-s, su, gu);
        gv = fmaf(-s, sv, gv);
    }
    if (a.gmv) {
        a.gmv[(2 * static_cast<int64_t>(in)) * hw + p] = gu;
        a.gmv[(2 * static_cast<int64_t>(in) + 1) * hw + p] = gv;
    }
}

// Plain fills and the accumulator cast: grid-stride, 16-byte accesses when
// the pointer allows.
__global__ void zero_f32_kernel(float *p, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
        float4 *q = reinterpret_cast<float4 *>(p);
        const int64_t n4 = n / 4;
        for (int64_t t = i; t < n4; t += stride) q[t] = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int64_t t = n4 * 4 + i; t < n; t += stride) p[t] = 0.0f;
    } else {
        for (int64_t t = i; t < n; t += stride) p[t] = 0.0f;
    }
}

__global__ void zero_u32_kernel(uint32_t *p, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
         t += stride)
        p[t] = 0u;
}

template <typename T>
__global__ void cast_f32_kernel(const float *src, T *dst, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
         t += stride)
        dst[t] = from_f32<T>(src[t]);
}

int stream_grid(int64_t n, int per_thread) {
    int64_t blocks = (n + 256LL * per_thread - 1) / (256LL * per_thread);
    if (blocks < 1) blocks = 1;
    if (blocks > 65536) blocks = 65536;
    return static_cast<int>(blocks);
}

template <typename T, int CT>
hipError_t fwd_launch(const void *src, const float *mv, const WarpShape &s, void *out,
                      uint8_t *mask, uint32_t *count, hipStream_t st) {
    FwdArgs<T> a;
    a.src = static_cast<const T *>(src);
    a.mv = mv;
    a.out = static_cast<T *>(out);
    a.mask = mask;
    a.count = count;
    a.n = s.n; a.c = s.c; a.h = s.h; a.w = s.w; a.k = s.k;
    a.tiles_x = (s.w + kTileW - 1) / kTileW;
    a.tiles_y = (s.h + kTileH - 1) / kTileH;
    for (int j = 0; j < 4; ++j) a.s[j] = s.phases[j];
    const int64_t blocks = static_cast<int64_t>(a.tiles_x) * a.tiles_y * s.n;
    hipLaunchKernelGGL((warp_forward_kernel<T, CT>), dim3(static_cast<unsigned>(blocks)),
                       dim3(kTileW, kTileH), 0, st, a);
    return hipGetLastError();
}

template <typename T, int CT>
hipError_t bwd_launch(const void *src, const float *mv, const WarpShape &s, const void *gout,
                      float *accum, float *gmv, hipStream_t st) {
    BwdArgs<T> a;
    a.src = static_cast<const T *>(src);
    a.mv = mv;
    a.gout = static_cast<const T *>(gout);
    a.accum = accum;
    a.gmv = gmv;
    a.n = s.n; a.c = s.c; a.h = s.h; a.w = s.w; a.k = s.k;
    a.tiles_x = (s.w + kTileW - 1) / kTileW;
    a.tiles_y = (s.h + kTileH - 1) / kTileH;
    for (int j = 0; j < 4; ++j) a.s[j] = s.phases[j];
    const int64_t blocks = static_cast<int64_t>(a.tiles_x) * a.tiles_y * s.n;
    hipLaunchKernelGGL((warp_backward_kernel<T, CT>), dim3(static_cast<unsigned>(blocks)),
                       dim3(kTileW, kTileH), 0, st, a);
    return hipGetLastError();
}

template <typename T>
hipError_t fwd_by_channels(const void *src, const float *mv, const WarpShape &s, void *out,
                           uint8_t *mask, uint32_t *count, hipStream_t st) {
    switch (s.c) {
    case 1: return fwd_launch<T, 1>(src, mv, s, out, mask, count, st);
    case 3: return fwd_launch<T, 3>(src, mv, s, out, mask, count, st);
    case 4: return fwd_launch<T, 4>(src, mv, s, out, mask, count, st);
    case 12: return fwd_launch<T, 12>(src, mv, s, out, mask, count, st);
    default: return fwd_launch<T, 0>(src, mv, s, out, mask, count, st);
    }
}

template <typename T>
hipError_t bwd_by_channels(const void *src, const float *mv, const WarpShape &s,
                           const void *gout, float *accum, float *gmv, hipStream_t st) {
    switch (s.c) {
    case 1: return bwd_launch<T, 1>(src, mv, s, gout, accum, gmv, st);
    case 3: return bwd_launch<T, 3>(src, mv, s, gout, accum, gmv, st);
    case 4: return bwd_launch<T, 4>(src, mv, s, gout, accum, gmv, st);
    case 12: return bwd_launch<T, 12>(src, mv, s, gout, accum, gmv, st);
    default: return bwd_launch<T, 0>(src, mv, s, gout, accum, gmv, st);
    }
}

}  // namespace

hipError_t launch_zero_u32(uint32_t *p, int64_t count, hipStream_t stream) {
    hipLaunchKernelGGL(zero_u32_kernel, dim3(stream_grid(count, 1)), dim3(256), 0, stream, p,
                       count);
    return hipGetLastError();
}

hipError_t launch_forward(int dtype, const void *src, const float *mv, const WarpShape &s,
                          void *out, uint8_t *mask, uint32_t *count, hipStream_t stream) {
    if (count) {
        hipError_t e = launch_zero_u32(count, static_cast<int64_t>(s.n) * s.k, stream);
        if (e != hipSuccess) return e;
    }
    switch (dtype) {
    case 0: return fwd_by_channels<float>(src, mv, s, out, mask, count, stream);
    case 1: return fwd_by_channels<_Float16>(src, mv, s, out, mask, count, stream);
    default: return fwd_by_channels<__bf16>(src, mv, s, out, mask, count, stream);
    }
}

hipError_t launch_backward(int dtype, const void *src, const float *mv, const WarpShape &s,
                           const void *grad_out, float *accum, void *cast_to, float *grad_mv,
                           hipStream_t stream) {
    const int64_t img_elems = static_cast<int64_t>(s.n) * s.c * s.h * s.w;
    if (accum) {
        hipLaunchKernelGGL(zero_f32_kernel, dim3(stream_grid(img_elems, 4)), dim3(256), 0,
                           stream, accum, img_elems);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipError_t e;
    switch (dtype) {
    case 0: e = bwd_by_channels<float>(src, mv, s, grad_out, accum, grad_mv, stream); break;
    case 1: e = bwd_by_channels<_Float16>(src, mv, s, grad_out, accum, grad_mv, stream); break;
    default: e = bwd_by_channels<__bf16>(src, mv, s, grad_out, accum, grad_mv, stream); break;
    }
    if (e != hipSuccess || !cast_to) return e;
    if (dtype == 1)
        hipLaunchKernelGGL(cast_f32_kernel<_Float16>, dim3(stream_grid(img_elems, 4)), dim3(256),
                           0, stream, accum, static_cast<_Float16 *>(cast_to), img_elems);
    else
        hipLaunchKernelGGL(cast_f32_kernel<__bf16>, dim3(stream_grid(img_elems, 4)), dim3(256),
                           0, stream, accum, static_cast<__bf16 *>(cast_to), img_elems);
    return hipGetLastError();
}

}  // namespace exw
