// Forward motion-vector warp for CDNA4 (gfx950).
//
// What is computed (paper §II-B image warping; §IV-B: the predicted frames
// P_1..P_3 shown at t + i/4 all come from F_t; §III-B: warped pixels without
// a source in the frame are invalid): each output pixel reads its motion
// vector once, forms all K phase displacements, gathers the four bilinear
// taps of every channel, and writes K output pixels, K mask bytes and the
// per-(frame, phase) invalid counts.
//
// Two layouts of the work. Frames whose rows are 4-element aligned use the
// staged kernel: a workgroup covers a 64 x 16 tile (a wavefront per 4 rows),
// and per phase it copies the bounding box of its taps into LDS with aligned
// 16-byte loads, then reads the taps there. Other frames use the direct
// kernel: a wavefront per 64 pixels of a row, taps gathered from global
// memory, the two horizontal taps of a row in one unaligned load, and all
// gathers of all phases issued before any store. In both, motion, output and
// mask accesses are coalesced, tiles are renumbered per XCD, and the motion
// vector is read once for all K phases. No MFMA: this is a gather.
#include <climits>

#include "launch.h"
#include "warp_common.h"

namespace exw {
namespace {

constexpr int kTileW = 64;
constexpr int kTileH = 4;
constexpr int kThreads = kTileW * kTileH;

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

struct PixelPos {
    int in, x, y;
    bool inside;
};

__device__ __forceinline__ PixelPos decode_pixel(int tiles_x, int tiles_y, int w, int h) {
    const int b = xcd_tile_index(blockIdx.x, gridDim.x);
    const int tx = b % tiles_x;
    const int rest = b / tiles_x;
    PixelPos q;
    q.in = rest / tiles_y;
    q.x = tx * kTileW + threadIdx.x;
    q.y = (rest % tiles_y) * kTileH + threadIdx.y;
    q.inside = (q.x < w) && (q.y < h);
    return q;
}

__device__ __forceinline__ void count_invalid(uint32_t *count, int64_t plane, bool inside,
                                              bool valid) {
    // One atomic per wavefront that saw invalid pixels (frame borders only).
    const unsigned long long bal = __ballot(inside && !valid);
    if (bal != 0ull && __lane_id() == 0)
        atomicAdd(count + plane, static_cast<uint32_t>(__popcll(bal)));
}

// Channel count CT and phase count KT known at compile time; requires W >= 2
// (paired horizontal loads).
template <typename T, int CT, int KT>
__global__ __launch_bounds__(kThreads) void warp_forward_kernel(FwdArgs<T> a) {
    const int w = a.w, h = a.h;
    const PixelPos q = decode_pixel(a.tiles_x, a.tiles_y, w, h);
    const int64_t hw = static_cast<int64_t>(h) * w;
    const int64_t p = static_cast<int64_t>(q.y) * w + q.x;

    float u = 0.0f, v = 0.0f;
    if (q.inside) {
        u = a.mv[(2 * static_cast<int64_t>(q.in)) * hw + p];
        v = a.mv[(2 * static_cast<int64_t>(q.in) + 1) * hw + p];
    }
    const T *img = a.src + static_cast<int64_t>(q.in) * CT * hw;

    Axis ax[KT], ay[KT];
    bool valid[KT];
    float i00[KT][CT], i01[KT][CT], i10[KT][CT], i11[KT][CT];
#pragma unroll
    for (int j = 0; j < KT; ++j) {
        ax[j] = split_axis(a.s[j] * u, q.x, w);
        ay[j] = split_axis(a.s[j] * v, q.y, h);
        valid[j] = q.inside && ax[j].ok && ay[j].ok;
        // The pair (xl, xl + 1) must stay in the row: at the last column the
        // pair starts one to the left and the tap takes its second element.
        const int xl = min(ax[j].i0, w - 2);
        const bool last = ax[j].i0 == w - 1;
        const T *r0 = img + static_cast<int64_t>(ay[j].i0) * w + xl;
        const T *r1 = img + static_cast<int64_t>(ay[j].i1) * w + xl;
#pragma unroll
        for (int ch = 0; ch < CT; ++ch) {
            float a0 = 0.f, b0 = 0.f, a1 = 0.f, b1 = 0.f;
            if (valid[j]) {
                load_pair(r0 + ch * hw, a0, b0);
                load_pair(r1 + ch * hw, a1, b1);
            }
            i00[j][ch] = last ? b0 : a0;
            i01[j][ch] = b0;
            i10[j][ch] = last ? b1 : a1;
            i11[j][ch] = b1;
        }
    }
#pragma unroll
    for (int j = 0; j < KT; ++j) {
        const int64_t plane = static_cast<int64_t>(q.in) * KT + j;
        if (q.inside) {
            const float fx = ax[j].f, fy = ay[j].f;
            const float w00 = (1.0f - fx) * (1.0f - fy);
            const float w01 = fx * (1.0f - fy);
            const float w10 = (1.0f - fx) * fy;
            const float w11 = fx * fy;
            T *o = a.out + plane * CT * hw + p;
#pragma unroll
            for (int ch = 0; ch < CT; ++ch) {
                float acc = w00 * i00[j][ch];
                acc = fmaf(w01, i01[j][ch], acc);
                acc = fmaf(w10, i10[j][ch], acc);
                acc = fmaf(w11, i11[j][ch], acc);
                o[ch * hw] = from_f32<T>(valid[j] ? acc : 0.0f);
            }
            if (a.mask) a.mask[plane * hw + p] = valid[j] ? 1 : 0;
        }
        if (a.count) count_invalid(a.count, plane, q.inside, valid[j]);
    }
}


// ------------------------------------------------------------ staged path
//
// Gathering the taps straight from global memory keeps the texture/L1 path
// busy with unaligned 8-byte loads that span several cache lines, and that
// path is shared with the (memory-bound) output stores, so the two do not
// overlap. When frames are 4-element aligned (W % 4 == 0) the forward kernel
// instead stages, per phase, the bounding box of the workgroup's taps into
// LDS with aligned 16-byte loads and reads the taps from LDS. A box that does
// not fit the LDS budget (strongly diverging motion) falls back to global
// gathers for that phase.

constexpr int kStTileW = 64;                  // tile width (one lane per column)
constexpr int kStRows = 4;                    // rows per wavefront
constexpr int kStTileH = 4 * kStRows;         // 16 rows per 4-wavefront workgroup
constexpr int kStLdsFloats = 6 * 1024;        // 24 KB of staged float32 source

template <typename T>
struct Vec4T;
template <>
struct Vec4T<float> {
    using type = float4;
};
template <>
struct Vec4T<_Float16> {
    using type = uint2;
};
template <>
struct Vec4T<__bf16> {
    using type = uint2;
};

__device__ __forceinline__ void unpack4(const float4 &v, float *o) {
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
template <typename T>
__device__ __forceinline__ void unpack4(const uint2 &v, float *o) {
    o[0] = half_bits_to_f32(v.x, static_cast<T *>(nullptr));
    o[1] = half_bits_to_f32(v.x >> 16, static_cast<T *>(nullptr));
    o[2] = half_bits_to_f32(v.y, static_cast<T *>(nullptr));
    o[3] = half_bits_to_f32(v.y >> 16, static_cast<T *>(nullptr));
}

template <typename T, int CT, int KT>
__global__ __launch_bounds__(kThreads) void warp_forward_staged_kernel(FwdArgs<T> a) {
    __shared__ float4 stage4[kStLdsFloats / 4];
    __shared__ int box_slot[4][4];
    float *stage = reinterpret_cast<float *>(stage4);
    const int w = a.w, h = a.h;
    const int lane = threadIdx.x % kSegW, wave = threadIdx.x / kSegW;
    const int b = xcd_tile_index(blockIdx.x, gridDim.x);
    const int tx = b % a.tiles_x;
    const int rest = b / a.tiles_x;
    const int in = rest / a.tiles_y;
    const int x = tx * kStTileW + lane;
    const int yb = (rest % a.tiles_y) * kStTileH + wave * kStRows;
    const int64_t hw = static_cast<int64_t>(h) * w;
    const T *img = a.src + static_cast<int64_t>(in) * CT * hw;

    float u[kStRows], v[kStRows];
    bool inside[kStRows];
#pragma unroll
    for (int r = 0; r < kStRows; ++r) {
        inside[r] = x < w && yb + r < h;
        const int64_t p = static_cast<int64_t>(yb + r) * w + x;
        u[r] = inside[r] ? a.mv[(2 * static_cast<int64_t>(in)) * hw + p] : 0.0f;
        v[r] = inside[r] ? a.mv[(2 * static_cast<int64_t>(in) + 1) * hw + p] : 0.0f;
    }

#pragma unroll 1
    for (int j = 0; j < KT; ++j) {
        // phase j without dynamic indexing of the argument array
        const float sj = j == 0 ? a.s[0] : (j == 1 ? a.s[1] : (j == 2 ? a.s[2] : a.s[3]));
        Axis ax[kStRows], ay[kStRows];
        bool valid[kStRows];
        int xl = INT_MAX, xh = INT_MIN, yl = INT_MAX, yh = INT_MIN;
#pragma unroll
        for (int r = 0; r < kStRows; ++r) {
            ax[r] = split_axis(sj * u[r], x, w);
            ay[r] = split_axis(sj * v[r], yb + r, h);
            valid[r] = inside[r] && ax[r].ok && ay[r].ok;
            if (valid[r]) {
                xl = min(xl, ax[r].i0);
                xh = max(xh, ax[r].i1);
                yl = min(yl, ay[r].i0);
                yh = max(yh, ay[r].i1);
            }
        }
        // Box of all taps of the workgroup for this phase.
        xl = wave_min(xl);
        xh = wave_max(xh);
        yl = wave_min(yl);
        yh = wave_max(yh);
        if (lane == 0) {
            box_slot[wave][0] = xl;
            box_slot[wave][1] = xh;
            box_slot[wave][2] = yl;
            box_slot[wave][3] = yh;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            xl = min(xl, box_slot[q][0]);
            xh = max(xh, box_slot[q][1]);
            yl = min(yl, box_slot[q][2]);
            yh = max(yh, box_slot[q][3]);
        }
        __syncthreads();  // box_slot is reused by the next phase
        const bool empty = xl > xh;
        const int xa = empty ? 0 : (xl & ~3);            // 16-byte aligned start column
        const int fw = empty ? 0 : ((xh - xa + 4) & ~3); // staged width, multiple of 4
        const int fh = empty ? 0 : (yh - yl + 1);
        const int plane = fw * fh;
        const int cg = plane > 0 ? min(CT, kStLdsFloats / plane) : CT;  // channels per pass
        const int64_t oplane = static_cast<int64_t>(in) * KT + j;
        T *obase = a.out + oplane * CT * hw;

        float fx[kStRows], fy[kStRows];
#pragma unroll
        for (int r = 0; r < kStRows; ++r) {
            fx[r] = ax[r].f;
            fy[r] = ay[r].f;
        }
        if (cg >= 1 && !empty) {
            for (int c0 = 0; c0 < CT; c0 += cg) {
                const int nc = min(cg, CT - c0);
                // Stage channels [c0, c0 + nc): rows yl..yh, columns xa..xa+fw-1.
                const int quads = nc * plane / 4;
                for (int qd = threadIdx.x; qd < quads; qd += kThreads) {
                    const int e = qd * 4;
                    const int cc = e / plane;
                    const int rem = e % plane;
                    const int ry = rem / fw, rx = rem % fw;
                    const T *gp = img + static_cast<int64_t>(c0 + cc) * hw +
                                  static_cast<int64_t>(yl + ry) * w + xa + rx;
                    float f4[4];
                    if constexpr (sizeof(T) == 4)
                        unpack4(*reinterpret_cast<const float4 *>(gp), f4);
                    else
                        unpack4<T>(*reinterpret_cast<const uint2 *>(gp), f4);
                    stage4[qd] = make_float4(f4[0], f4[1], f4[2], f4[3]);
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < kStRows; ++r) {
                    if (!inside[r]) continue;
                    const int64_t p = static_cast<int64_t>(yb + r) * w + x;
                    const float w00 = (1.0f - fx[r]) * (1.0f - fy[r]);
                    const float w01 = fx[r] * (1.0f - fy[r]);
                    const float w10 = (1.0f - fx[r]) * fy[r];
                    const float w11 = fx[r] * fy[r];
                    const bool last = ax[r].i0 == w - 1;
                    const int lx = (last ? ax[r].i0 - 1 : ax[r].i0) - xa;
                    const int l0 = (ay[r].i0 - yl) * fw + lx;
                    const int l1 = (ay[r].i1 - yl) * fw + lx;
                    for (int cc = 0; cc < nc; ++cc) {
                        float acc = 0.0f;
                        if (valid[r]) {
                            const float *sp = stage + cc * plane;
                            const float a0 = sp[l0], b0 = sp[l0 + 1];
                            const float a1 = sp[l1], b1 = sp[l1 + 1];
                            acc = w00 * (last ? b0 : a0);
                            acc = fmaf(w01, b0, acc);
                            acc = fmaf(w10, last ? b1 : a1, acc);
                            acc = fmaf(w11, b1, acc);
                        }
                        obase[static_cast<int64_t>(c0 + cc) * hw + p] = from_f32<T>(acc);
                    }
                }
                __syncthreads();  // the next pass overwrites the stage
            }
        } else {
            // Box too large for LDS (or no valid tap): gather from global memory.
#pragma unroll
            for (int r = 0; r < kStRows; ++r) {
                if (!inside[r]) continue;
                const int64_t p = static_cast<int64_t>(yb + r) * w + x;
                const float w00 = (1.0f - fx[r]) * (1.0f - fy[r]);
                const float w01 = fx[r] * (1.0f - fy[r]);
                const float w10 = (1.0f - fx[r]) * fy[r];
                const float w11 = fx[r] * fy[r];
                const int xl2 = min(ax[r].i0, w - 2);
                const bool last = ax[r].i0 == w - 1;
                const T *r0 = img + static_cast<int64_t>(ay[r].i0) * w + xl2;
                const T *r1 = img + static_cast<int64_t>(ay[r].i1) * w + xl2;
#pragma unroll 1
                for (int ch = 0; ch < CT; ++ch) {
                    float acc = 0.0f;
                    if (valid[r]) {
                        float a0, b0, a1, b1;
                        load_pair(r0 + ch * hw, a0, b0);
                        load_pair(r1 + ch * hw, a1, b1);
                        acc = w00 * (last ? b0 : a0);
                        acc = fmaf(w01, b0, acc);
                        acc = fmaf(w10, last ? b1 : a1, acc);
                        acc = fmaf(w11, b1, acc);
                    }
                    obase[static_cast<int64_t>(ch) * hw + p] = from_f32<T>(acc);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < kStRows; ++r) {
            const int64_t p = static_cast<int64_t>(yb + r) * w + x;
            if (a.mask && inside[r]) a.mask[oplane * hw + p] = valid[r] ? 1 : 0;
            if (a.count) count_invalid(a.count, oplane, inside[r], valid[r]);
        }
    }
}

// Any channel count, any phase count, any width (including W == 1): one
// channel at a time, scalar taps.
template <typename T>
__global__ __launch_bounds__(kThreads) void warp_forward_generic_kernel(FwdArgs<T> a) {
    const int C = a.c, w = a.w, h = a.h;
    const PixelPos q = decode_pixel(a.tiles_x, a.tiles_y, w, h);
    const int64_t hw = static_cast<int64_t>(h) * w;
    const int64_t p = static_cast<int64_t>(q.y) * w + q.x;
    float u = 0.0f, v = 0.0f;
    if (q.inside) {
        u = a.mv[(2 * static_cast<int64_t>(q.in)) * hw + p];
        v = a.mv[(2 * static_cast<int64_t>(q.in) + 1) * hw + p];
    }
    const T *img = a.src + static_cast<int64_t>(q.in) * C * hw;
    for (int j = 0; j < a.k; ++j) {
        const Axis ax = split_axis(a.s[j] * u, q.x, w);
        const Axis ay = split_axis(a.s[j] * v, q.y, h);
        const bool valid = q.inside && ax.ok && ay.ok;
        const int64_t plane = static_cast<int64_t>(q.in) * a.k + j;
        if (q.inside) {
            T *o = a.out + plane * C * hw + p;
            const float w00 = (1.0f - ax.f) * (1.0f - ay.f);
            const float w01 = ax.f * (1.0f - ay.f);
            const float w10 = (1.0f - ax.f) * ay.f;
            const float w11 = ax.f * ay.f;
            const int64_t r0 = static_cast<int64_t>(ay.i0) * w;
            const int64_t r1 = static_cast<int64_t>(ay.i1) * w;
            for (int ch = 0; ch < C; ++ch) {
                float acc = 0.0f;
                if (valid) {
                    const T *pl = img + ch * hw;
                    acc = w00 * to_f32(pl[r0 + ax.i0]);
                    acc = fmaf(w01, to_f32(pl[r0 + ax.i1]), acc);
                    acc = fmaf(w10, to_f32(pl[r1 + ax.i0]), acc);
                    acc = fmaf(w11, to_f32(pl[r1 + ax.i1]), acc);
                }
                o[ch * hw] = from_f32<T>(acc);
            }
            if (a.mask) a.mask[plane * hw + p] = valid ? 1 : 0;
        }
        if (a.count) count_invalid(a.count, plane, q.inside, valid);
    }
}

__global__ void zero_u32_kernel(uint32_t *p, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
         t += stride)
        p[t] = 0u;
}

template <typename T>
FwdArgs<T> make_args(const void *src, const float *mv, const WarpShape &s, void *out,
                     uint8_t *mask, uint32_t *count) {
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
    return a;
}

template <typename T, int CT, int KT>
hipError_t launch_staged(FwdArgs<T> a, hipStream_t st) {
    a.tiles_x = (a.w + kStTileW - 1) / kStTileW;
    a.tiles_y = (a.h + kStTileH - 1) / kStTileH;
    const dim3 grid(static_cast<unsigned>(static_cast<int64_t>(a.tiles_x) * a.tiles_y * a.n));
    hipLaunchKernelGGL((warp_forward_staged_kernel<T, CT, KT>), grid, dim3(kThreads), 0, st, a);
    return hipGetLastError();
}

template <typename T, int CT>
hipError_t launch_ck(const FwdArgs<T> &a, dim3 grid, hipStream_t st) {
    // Staged path: rows must start on 4-element boundaries that are also
    // 16-byte (float32) or 8-byte (16-bit) aligned in memory.
    const bool aligned4 = (reinterpret_cast<uintptr_t>(a.src) % (4 * sizeof(T))) == 0;
    if (a.w % 4 == 0 && aligned4) {
        switch (a.k) {
        case 1: return launch_staged<T, CT, 1>(a, st);
        case 2: return launch_staged<T, CT, 2>(a, st);
        case 3: return launch_staged<T, CT, 3>(a, st);
        default: return launch_staged<T, CT, 4>(a, st);
        }
    }
    switch (a.k) {
    case 1: hipLaunchKernelGGL((warp_forward_kernel<T, CT, 1>), grid, dim3(kTileW, kTileH), 0, st, a); break;
    case 2: hipLaunchKernelGGL((warp_forward_kernel<T, CT, 2>), grid, dim3(kTileW, kTileH), 0, st, a); break;
    case 3: hipLaunchKernelGGL((warp_forward_kernel<T, CT, 3>), grid, dim3(kTileW, kTileH), 0, st, a); break;
    default: hipLaunchKernelGGL((warp_forward_kernel<T, CT, 4>), grid, dim3(kTileW, kTileH), 0, st, a); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_typed(const void *src, const float *mv, const WarpShape &s, void *out,
                        uint8_t *mask, uint32_t *count, hipStream_t st) {
    const FwdArgs<T> a = make_args<T>(src, mv, s, out, mask, count);
    const dim3 grid(static_cast<unsigned>(static_cast<int64_t>(a.tiles_x) * a.tiles_y * s.n));
    if (s.w >= 2) {
        switch (s.c) {
        case 1: return launch_ck<T, 1>(a, grid, st);
        case 3: return launch_ck<T, 3>(a, grid, st);
        case 4: return launch_ck<T, 4>(a, grid, st);
        case 12: return launch_ck<T, 12>(a, grid, st);
        default: break;
        }
    }
    hipLaunchKernelGGL(warp_forward_generic_kernel<T>, grid, dim3(kTileW, kTileH), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_zero_u32(uint32_t *p, int64_t count, hipStream_t stream) {
    int64_t blocks = (count + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       p, count);
    return hipGetLastError();
}

hipError_t launch_forward(int dtype, const void *src, const float *mv, const WarpShape &s,
                          void *out, uint8_t *mask, uint32_t *count, hipStream_t stream) {
    if (count) {
        hipError_t e = launch_zero_u32(count, static_cast<int64_t>(s.n) * s.k, stream);
        if (e != hipSuccess) return e;
    }
    switch (dtype) {
    case 0: return launch_typed<float>(src, mv, s, out, mask, count, stream);
    case 1: return launch_typed<_Float16>(src, mv, s, out, mask, count, stream);
    default: return launch_typed<__bf16>(src, mv, s, out, mask, count, stream);
    }
}

}  // namespace exw
