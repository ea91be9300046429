// Per-frame motion statistics for CDNA4 (gfx950): mean and population
// variance of the horizontal and the vertical motion component of every frame
// (paper §IV-C, Eq. 1: the environment vector E_t holds Var_x(F_mv) and Var_y(F_mv);
// Table IV: the motion variance is the feature that reveals dynamic objects).
//
// The motion planes are streamed once (8 bytes per pixel, HBM bound). Each
// thread loads kChunk values per component with coalesced loads and sums, in
// float64, the differences of its values from its first one and their
// squares (differences and squares of float32 values are exact in float64):
// additions only, no division in the loop. At the end each thread forms its
// (count, mean, M2); the lanes of a wavefront are combined two-pass (the
// wavefront's mean first, then M2 = sum (M2_i + n_i (mean_i - mean)^2), every
// term non-negative), and wavefronts and then the partials of all workgroups
// of a frame with the pairwise update for (count, mean, M2) (Chan, Golub and
// LeVeque). Every fold is in a fixed order, so results are reproducible, and
// no step forms E[x^2] - E[x]^2 over more than one thread's values, so a mean
// that is large against the spread does not cancel.
#include <mutex>

#include "launch.h"
#include "moments.h"

namespace exw {
namespace {

constexpr int kStatThreads = 256;
constexpr int kChunk = 8;                          // values per thread, per component
constexpr int kSpan = kStatThreads * kChunk;       // pixels per workgroup pass
constexpr int kMaxParts = 256;                     // workgroups per frame, at most

// The lanes' (count, mean, M2) combined two-pass; the result in every lane.
__device__ __forceinline__ Moments wave_combine(double n, double mean, double m2, double total) {
    if (total == 0.0) return Moments{0.0, 0.0, 0.0};  // (wave-uniform)
    const double mu = wave_sum(n * mean) / total;
    const double d = mean - mu;
    // (a lane without values adds 0 * d * d: nothing while the mean is finite)
    return Moments{total, mu, wave_sum(m2 + n * d * d)};
}

// grid = n * parts workgroups; workgroup (frame, part) covers passes part,
// part + parts, ... of kSpan pixels and writes one partial per component.
__global__ __launch_bounds__(kStatThreads) void motion_moments_kernel(const float *mv, int64_t hw,
                                                                     int parts, Moments *partial) {
    __shared__ Moments lds[2][kStatThreads / 64];
    const int frame = blockIdx.x / parts;
    const int part = blockIdx.x % parts;
    const float *pu = mv + 2 * static_cast<int64_t>(frame) * hw;
    const float *pv = pu + hw;
    const int64_t stride = static_cast<int64_t>(parts) * kSpan;
    // The next chunk is loaded while the current one is summed.
    float xu[kChunk], xv[kChunk];
    auto load = [&](int64_t base, float (&u)[kChunk], float (&v)[kChunk]) {
#pragma unroll
        for (int j = 0; j < kChunk; ++j) {
            const int64_t i = base + j * kStatThreads + threadIdx.x;  // coalesced
            const bool in = i < hw;
            u[j] = in ? pu[i] : 0.0f;
            v[j] = in ? pv[i] : 0.0f;
        }
    };
    int64_t base = static_cast<int64_t>(part) * kSpan;
    if (base < hw) load(base, xu, xv);
    // the shift: the thread's first value (unused when it has none)
    const double ku = xu[0], kv = xv[0];
    double s1u = 0.0, s2u = 0.0, s1v = 0.0, s2v = 0.0;
    int count = 0;
    for (; base < hw; base += stride) {
        float nu[kChunk], nv[kChunk];
        if (base + stride < hw) load(base + stride, nu, nv);
        // in-range values are a prefix of the chunk (j increases with i)
        const int64_t left = (hw - base - threadIdx.x + kStatThreads - 1) / kStatThreads;
        const int c = static_cast<int>(left < kChunk ? left : kChunk);
#pragma unroll
        for (int j = 0; j < kChunk; ++j) {
            const double du = j < c ? static_cast<double>(xu[j]) - ku : 0.0;
            const double dv = j < c ? static_cast<double>(xv[j]) - kv : 0.0;
            s1u += du;
            s2u = fma(du, du, s2u);
            s1v += dv;
            s2v = fma(dv, dv, s2v);
        }
        count += c;
#pragma unroll
        for (int j = 0; j < kChunk; ++j) {
            xu[j] = nu[j];
            xv[j] = nv[j];
        }
    }
    const double n = count;
    double mean_u = 0.0, m2_u = 0.0, mean_v = 0.0, m2_v = 0.0;
    if (count > 0) {
        mean_u = ku + s1u / n;
        m2_u = s2u - s1u * s1u / n;
        mean_v = kv + s1v / n;
        m2_v = s2v - s1v * s1v / n;
    }
    const double total = wave_sum(n);
    const Moments mu = wave_combine(n, mean_u, m2_u, total);
    const Moments mvv = wave_combine(n, mean_v, m2_v, total);
    const int wave = threadIdx.x / 64;
    if (__lane_id() == 0) {
        lds[0][wave] = mu;
        lds[1][wave] = mvv;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        Moments m = lds[threadIdx.x][0];
        for (int k = 1; k < kStatThreads / 64; ++k) m = fold(m, lds[threadIdx.x][k]);
        partial[(static_cast<int64_t>(frame) * 2 + threadIdx.x) * parts + part] = m;
    }
}

// One wavefront per frame and component folds the workgroup partials.
__global__ __launch_bounds__(64) void motion_stats_final_kernel(const Moments *partial, int parts,
                                                                double *stats) {
    const int frame = blockIdx.x / 2, comp = blockIdx.x % 2;
    const Moments *p = partial + (static_cast<int64_t>(frame) * 2 + comp) * parts;
    Moments m{0.0, 0.0, 0.0};
    for (int i = __lane_id(); i < parts; i += 64) m = fold(m, p[i]);
    m = wave_fold(m);
    if (__lane_id() == 0) {
        stats[frame * 4 + 2 * comp] = m.mean;
        stats[frame * 4 + 2 * comp + 1] = m.m2 / m.n;
    }
}

int parts_for(int64_t hw) {
    const int64_t passes = (hw + kSpan - 1) / kSpan;
    return static_cast<int>(passes < kMaxParts ? passes : kMaxParts);
}

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// Scratch of the call that allocates nothing: the workgroup partials live in
// a file-scope device array instead of a caller's workspace. Each device holds
// its own copy at its own address; host code reaches it only through the
// address hipGetSymbolAddress returns for that device (the array's name is a
// host-side stand-in that no kernel may be given).
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

hipError_t no_alloc_scratch(void **ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        // once per device, with that device current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

size_t motion_stats_workspace_bytes(int n, int h, int w) {
    return sizeof(Moments) * 2 * static_cast<size_t>(n) *
           parts_for(static_cast<int64_t>(h) * w);
}

int motion_stats_parts(int h, int w) { return parts_for(static_cast<int64_t>(h) * w); }

hipError_t launch_motion_moments(const float *mv, int n, int h, int w, Moments *partial,
                                 hipStream_t stream) {
    const int64_t hw = static_cast<int64_t>(h) * w;
    const int parts = parts_for(hw);
    hipLaunchKernelGGL(motion_moments_kernel, dim3(static_cast<unsigned>(n) * parts),
                       dim3(kStatThreads), 0, stream, mv, hw, parts, partial);
    return hipGetLastError();
}

hipError_t launch_motion_stats_fold(const Moments *partial, int n, int parts, double *stats,
                                    hipStream_t stream) {
    hipLaunchKernelGGL(motion_stats_final_kernel, dim3(static_cast<unsigned>(n) * 2), dim3(64), 0,
                       stream, partial, parts, stats);
    return hipGetLastError();
}

hipError_t launch_motion_stats(const float *mv, int n, int h, int w, double *stats,
                               void *workspace, hipStream_t stream) {
    Moments *partial = static_cast<Moments *>(workspace);
    hipError_t e = launch_motion_moments(mv, n, h, w, partial, stream);
    if (e != hipSuccess) return e;
    return launch_motion_stats_fold(partial, n, parts_for(static_cast<int64_t>(h) * w), stats,
                                    stream);
}

}  // namespace exw
