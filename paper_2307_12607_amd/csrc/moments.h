// Float64 (count, mean, sum of squared deviations) of a set of values and
// their pairwise combination (Chan, Golub and LeVeque), used by the motion
// statistics (paper §IV-C, Eq. 1: Var_x(F_mv), Var_y(F_mv) of E_t): by the
// statistics pass and by the recording forward, which folds the motion it
// reads anyway. Every fold is in a fixed order, so results are reproducible.
// Sums of squares are formed only about a shift inside a small group of
// values (one thread's, or one 128 x 4 tile's), which bounds their
// cancellation by the group's size; everything above a group is combined
// two-pass or pairwise, never as E[x^2] - E[x]^2 over the frame, which
// cancels when the mean is large against the spread.
#pragma once

#include <hip/hip_runtime.h>

namespace exw {

struct Moments {
    double n, mean, m2;
};

__device__ __forceinline__ Moments fold(const Moments &a, const Moments &b) {
    if (b.n == 0.0) return a;
    if (a.n == 0.0) return b;
    const double n = a.n + b.n;
    const double d = b.mean - a.mean;
    const double fb = b.n / n;
    return Moments{n, a.mean + d * fb, a.m2 + b.m2 + d * d * a.n * fb};
}

__device__ __forceinline__ Moments shfl_xor(const Moments &m, int mask) {
    return Moments{__shfl_xor(m.n, mask), __shfl_xor(m.mean, mask), __shfl_xor(m.m2, mask)};
}

extern "C" __device__ double __ockl_wfred_add_f64(double);

// Sum over the 64 lanes of a wavefront, in every lane (DPP; every lane must be
// active; a fixed order, so the result is reproducible).
__device__ __forceinline__ double wave_sum(double v) { return __ockl_wfred_add_f64(v); }

// Fold over the 64 lanes of a wavefront (butterfly: every lane ends with the
// same value, built in the same order).
__device__ __forceinline__ Moments wave_fold(Moments m) {
#pragma unroll
    for (int mask = 1; mask < 64; mask <<= 1) {
        const Moments o = shfl_xor(m, mask);
        // lower lane of each pair first, so both lanes compute the same fold
        m = (__lane_id() & mask) ? fold(o, m) : fold(m, o);
    }
    return m;
}

// The recording forward's partials, one per 128 x 4 tile (thousands per
// frame), folded inside the launch that reduces the footprint records:
// kTileFoldParts workgroups per frame and component each fold a contiguous
// share with the two-pass combination (the share's mean mu = sum n_i mean_i /
// n, then M2 = sum (M2_i + n_i (mean_i - mu)^2), every term non-negative) into
// a slot; the last of them to finish (a counter per frame and component, which
// the recording forward zeroes) folds the slots in order and writes (mean,
// variance). Every order is fixed, so results are reproducible.
constexpr int kTileFoldParts = 8;
constexpr int kTileFoldThreads = 256;
constexpr int kTileFoldBatch = 8;  // partials per thread loaded together

struct TileFold {
    const Moments *parts;  // [N][2][tiles]
    int tiles;
    Moments *slots;        // [N][2][kTileFoldParts]
    unsigned *counters;    // [N][2], zero on entry
    double *stats;         // [N][4]: mean_x, var_x, mean_y, var_y
};

// Sum over the workgroup (kTileFoldThreads threads): every thread gets the
// same value, added in a fixed order.
__device__ __forceinline__ double tile_fold_sum(double v, double *lds) {
    v = wave_sum(v);
    __syncthreads();  // earlier readers of lds are done
    if (__lane_id() == 0) lds[threadIdx.x / 64] = v;
    __syncthreads();
    double t = lds[0];
#pragma unroll
    for (int k = 1; k < kTileFoldThreads / 64; ++k) t += lds[k];
    return t;
}

__device__ __forceinline__ Moments tile_share_moments(const Moments *p, int lo, int hi,
                                                      double *lds) {
    constexpr int kSpan = kTileFoldThreads * kTileFoldBatch;
    double n = 0.0, s = 0.0;
    for (int i0 = lo + static_cast<int>(threadIdx.x); i0 < hi; i0 += kSpan) {
        Moments m[kTileFoldBatch];
#pragma unroll
        for (int j = 0; j < kTileFoldBatch; ++j) {
            const int i = i0 + j * kTileFoldThreads;
            m[j] = i < hi ? p[i] : Moments{0.0, 0.0, 0.0};
        }
#pragma unroll
        for (int j = 0; j < kTileFoldBatch; ++j) {
            n += m[j].n;
            s += m[j].n * m[j].mean;
        }
    }
    n = tile_fold_sum(n, lds);
    s = tile_fold_sum(s, lds);
    if (n == 0.0) return Moments{0.0, 0.0, 0.0};  // (uniform: an empty share)
    const double mean = s / n;
    double m2 = 0.0;
    for (int i0 = lo + static_cast<int>(threadIdx.x); i0 < hi; i0 += kSpan) {
        Moments m[kTileFoldBatch];
#pragma unroll
        for (int j = 0; j < kTileFoldBatch; ++j) {
            const int i = i0 + j * kTileFoldThreads;
            m[j] = i < hi ? p[i] : Moments{0.0, 0.0, 0.0};
        }
#pragma unroll
        for (int j = 0; j < kTileFoldBatch; ++j) {
            // (an empty partial adds 0 * d * d: nothing while the mean is finite)
            const double d = m[j].mean - mean;
            m2 += m[j].m2 + m[j].n * d * d;
        }
    }
    m2 = tile_fold_sum(m2, lds);
    return Moments{n, mean, m2};
}

// Job (frame * 2 + comp) * kTileFoldParts + part; a workgroup of
// kTileFoldThreads threads, all of which call this.
__device__ __forceinline__ void fold_tile_share(const TileFold &f, int job) {
    __shared__ double lds[kTileFoldThreads / 64];
    const int fc = job / kTileFoldParts, part = job - fc * kTileFoldParts;
    const Moments *p = f.parts + static_cast<int64_t>(fc) * f.tiles;
    const int lo = static_cast<int>(static_cast<int64_t>(f.tiles) * part / kTileFoldParts);
    const int hi = static_cast<int>(static_cast<int64_t>(f.tiles) * (part + 1) / kTileFoldParts);
    const Moments m = tile_share_moments(p, lo, hi, lds);
    if (threadIdx.x != 0) return;
    f.slots[job] = m;
    __threadfence();  // the slot is visible before the count says so
    if (atomicAdd(&f.counters[fc], 1u) == kTileFoldParts - 1) {
        __threadfence();  // the other workgroups' slots, after their counts
        const Moments *sl = f.slots + static_cast<int64_t>(fc) * kTileFoldParts;
        Moments t = sl[0];
        for (int k = 1; k < kTileFoldParts; ++k) t = fold(t, sl[k]);
        const int frame = fc / 2, comp = fc - 2 * frame;
        f.stats[frame * 4 + 2 * comp] = t.mean;
        f.stats[frame * 4 + 2 * comp + 1] = t.m2 / t.n;
    }
}

// Partials of N frames, two components each: [N][2][parts] Moments, folded per
// frame and component by launch_motion_stats_fold into (mean_x, var_x,
// mean_y, var_y).
hipError_t launch_motion_stats_fold(const Moments *partial, int n, int parts, double *stats,
                                    hipStream_t stream);

// The statistics pass's partials of mv [N,2,H,W] into `partial` (its own
// number of parts per frame, motion_stats_parts(h, w)).
int motion_stats_parts(int h, int w);
hipError_t launch_motion_moments(const float *mv, int n, int h, int w, Moments *partial,
                                 hipStream_t stream);

}  // namespace exw
