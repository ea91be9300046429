// Footprint of the warp's taps per 64-pixel output row segment: what the
// adjoint's tile pass needs to know, before it replays a segment, about where
// that segment's bilinear taps land (paper §II-B: each output pixel reads the
// four source pixels around x - s*u). Written by the adjoint's footprint pass,
// or by the forward warp when the caller asks it to record them for a later
// adjoint of the same motion and phases; both use segment_footprint below, so
// the two records are identical.
#pragma once

#include <climits>

#include "warp_common.h"

namespace exw {

constexpr int kFar = 128;  // segments whose box lies further away use the atomic fallback

struct Box {
    int x_lo, x_hi, y_lo, y_hi;  // inclusive; x_lo > x_hi when the segment has no valid tap
};

// Integer tap offsets of a "uniform" segment: every lane is valid in every
// phase and all 64 lanes share ceil(s_k * u) and ceil(s_k * v), packed per
// phase k as (cx & 0xffff) | (cy << 16). Other segments hold kNotUniform in
// word 0 (offsets of uniform segments lie in [-32767, 32767]).
struct SegOffsets {
    uint32_t k[4];
};
constexpr uint32_t kNotUniform = 0x80008000u;

struct FrameInfo {
    int reach;    // largest distance (px) between a near segment and its box
    int has_far;  // 1 if a segment of this frame reaches further than kFar
};

__device__ __forceinline__ int box_reach(const Box &b, int sx0, int row) {
    const int r = max(max(sx0 - b.x_lo, b.x_hi - (sx0 + kSegW - 1)),
                      max(row - b.y_lo, b.y_hi - row));
    return max(r, 0);
}

// Box of first taps -> box of all taps, or the empty box.
__device__ __forceinline__ void finish_box(int (&b)[4], int y, int w, int h) {
    if (b[0] > b[1] || y >= h) {
        b[0] = 1; b[1] = 0; b[2] = 1; b[3] = 0;  // no valid tap
    } else {
        // the second tap is x0 + 1 clamped to the frame, applied to the maximum
        b[1] = min(b[1] + 1, w - 1);
        b[3] = min(b[3] + 1, h - 1);
    }
}

// Footprint of the segment of row y whose first pixel is sx0, from this
// lane's pixel x = sx0 + lane and its motion (u, v); in_r: the pixel lies in
// the frame. Results are wave-uniform: the box of the first taps over all
// valid pixels and phases, widened by one for the second taps (clamped to the
// frame), or {1, 0, 1, 0} when no tap is valid or y is past the frame; rec =
// the packed offsets when the segment is uniform, else kNotUniform in word 0.
// Every lane of the wavefront must take part.
template <int KT>
__device__ __forceinline__ void segment_footprint(float u, float v, int x, int y, int sx0, int w,
                                                  int h, bool in_r, const float (&s)[4],
                                                  int (&b)[4], uint32_t (&rec)[KT]) {
    bool uniform = true;  // wave-uniform
    uint32_t packed[KT];
    bool okj[KT];
    int cxj[KT], cyj[KT];
    int cx_lo = INT_MAX, cx_hi = INT_MIN, cy_lo = INT_MAX, cy_hi = INT_MIN;
#pragma unroll
    for (int j = 0; j < KT; ++j) {
        const float dx = s[j] * u, dy = s[j] * v;
        // the validity test of the warp: x - (w-1) <= dx <= x, likewise for y
        okj[j] = in_r && dx <= static_cast<float>(x) && dx >= static_cast<float>(x - (w - 1)) &&
                 dy <= static_cast<float>(y) && dy >= static_cast<float>(y - (h - 1));
        cxj[j] = static_cast<int>(ceilf(okj[j] ? dx : 0.0f));
        cyj[j] = static_cast<int>(ceilf(okj[j] ? dy : 0.0f));
        const int rcx = __builtin_amdgcn_readfirstlane(cxj[j]);
        const int rcy = __builtin_amdgcn_readfirstlane(cyj[j]);
        uniform = uniform && __ballot(okj[j] && cxj[j] == rcx && cyj[j] == rcy) == ~0ull &&
                  static_cast<unsigned>(rcx + 32767) <= 65534u &&
                  static_cast<unsigned>(rcy + 32767) <= 65534u;
        packed[j] = (static_cast<uint32_t>(rcx) & 0xffffu) | (static_cast<uint32_t>(rcy) << 16);
        cx_lo = min(cx_lo, rcx); cx_hi = max(cx_hi, rcx);
        cy_lo = min(cy_lo, rcy); cy_hi = max(cy_hi, rcy);
    }
    // first taps x0 = x - ceil(dx) (the exact floor of x - dx), y0 likewise
    if (uniform) {
        b[0] = sx0 - cx_hi; b[1] = sx0 + kSegW - 1 - cx_lo;
        b[2] = y - cy_hi;   b[3] = y - cy_lo;
    } else {  // branch-free per lane: invalid phases leave the box as is
        int xl = INT_MAX, xh = INT_MIN, yl = INT_MAX, yh = INT_MIN;
#pragma unroll
        for (int j = 0; j < KT; ++j) {
            xl = min(xl, okj[j] ? x - cxj[j] : INT_MAX);
            xh = max(xh, okj[j] ? x - cxj[j] : INT_MIN);
            yl = min(yl, okj[j] ? y - cyj[j] : INT_MAX);
            yh = max(yh, okj[j] ? y - cyj[j] : INT_MIN);
        }
        b[0] = __builtin_amdgcn_readfirstlane(wave_min(xl));
        b[1] = __builtin_amdgcn_readfirstlane(wave_max(xh));
        b[2] = __builtin_amdgcn_readfirstlane(wave_min(yl));
        b[3] = __builtin_amdgcn_readfirstlane(wave_max(yh));
    }
    finish_box(b, y, w, h);
#pragma unroll
    for (int j = 0; j < KT; ++j) rec[j] = uniform ? packed[j] : (j == 0 ? kNotUniform : 0u);
}

// The box of a segment whose pixels are all valid with the integer offsets
// (rx[k], ry[k]) = (ceil(s_k u), ceil(s_k v)) in every phase (wave-uniform
// values): what segment_footprint returns for such a segment, from the
// offsets alone.
template <int KT>
__device__ __forceinline__ void uniform_footprint(const int (&rx)[KT], const int (&ry)[KT], int y,
                                                  int sx0, int w, int h, int (&b)[4],
                                                  uint32_t (&rec)[KT]) {
    int cx_lo = INT_MAX, cx_hi = INT_MIN, cy_lo = INT_MAX, cy_hi = INT_MIN;
    bool fits = true;
#pragma unroll
    for (int j = 0; j < KT; ++j) {
        cx_lo = min(cx_lo, rx[j]); cx_hi = max(cx_hi, rx[j]);
        cy_lo = min(cy_lo, ry[j]); cy_hi = max(cy_hi, ry[j]);
        fits = fits && static_cast<unsigned>(rx[j] + 32767) <= 65534u &&
               static_cast<unsigned>(ry[j] + 32767) <= 65534u;
    }
    b[0] = sx0 - cx_hi; b[1] = sx0 + kSegW - 1 - cx_lo;
    b[2] = y - cy_hi;   b[3] = y - cy_lo;
    finish_box(b, y, w, h);
#pragma unroll
    for (int j = 0; j < KT; ++j)
        rec[j] = fits ? (static_cast<uint32_t>(rx[j]) & 0xffffu) | (static_cast<uint32_t>(ry[j]) << 16)
                      : (j == 0 ? kNotUniform : 0u);
}

// Folds a segment's box into the wavefront's per-frame figures: the largest
// reach among near segments, and whether any segment is far.
__device__ __forceinline__ void note_reach(const int (&b)[4], int sx0, int y, int &reach_max,
                                           int &far) {
    if (b[0] > b[1]) return;  // no valid tap
    const int rr = box_reach(Box{b[0], b[1], b[2], b[3]}, sx0, y);
    if (rr > kFar) far = 1; else reach_max = max(reach_max, rr);
}

// One lane's update of a frame's FrameInfo (zeroed before the pass).
__device__ __forceinline__ void publish_reach(FrameInfo *fi, int reach_max, int far) {
    if (far) atomicMax(&fi->has_far, 1);
    if (reach_max > __hip_atomic_load(&fi->reach, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMax(&fi->reach, reach_max);  // rare: the value only grows
}

}  // namespace exw
