// EMD features of the state vector on CDNA4 (gfx950): per frame and channel,
// the Earth Mover's Distance between the value distribution of a buffer of
// F_t and that of F_{t-1} (paper §III-D: the change of the world-normal and
// world-position buffers between frames is measured with the EMD; Table IV:
// EMD_{W_N}, EMD_{W_P}; §IV-C, Eq. 1: both are entries of E_t).
//
// Each channel's values are histogrammed over `bins` uniform bins on
// [lo, hi] (bin = floor((v - lo) * scale) in float64, clamped to the end
// bins; scale = bins / (hi - lo) from the host), and the one-dimensional EMD
// of the two unit-mass histograms is the L1 distance of their cumulative
// histograms times the bin width.
//
// Pass 1: workgroups own a contiguous run of one plane of both buffers,
// count into LDS histograms (integer LDS atomics; both buffers' counts side
// by side) and add their non-zero bins to the plane's global counters with
// one integer atomic each. Smooth buffers put many lanes of a wavefront in
// one bin, and atomics on one address serialise: the workgroup keeps up to
// four copies of its histograms, lane l counting into copy l mod copies (the
// copies one word apart, so one bin of different copies falls in different
// banks), and adds the copies up at the end. Pass 2: one workgroup per plane scans the count
// differences in 64-bit integers and sums their magnitudes exactly; the
// result is that exact sum / (H*W) * width in float64. Integer counts make
// every result independent of the order of the atomics.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.h"
#include "warp_common.h"

namespace exw {
namespace {

constexpr int kEmdThreads = 256;
constexpr int kEmdUnroll = 4;                          // loads in flight per thread and buffer
constexpr int64_t kEmdRun = 16384;                     // values of a plane per workgroup, at least
constexpr int kEmdMaxParts = 128;                      // workgroups per plane, at most

constexpr int kEmdLdsWords = 8200;                     // LDS words for the copies, at most (~32 KB)

struct EmdArgs {
    const void *cur, *prev;
    int64_t hw;
    int parts;
    int64_t run;       // values per workgroup (the last one may hold fewer)
    double lo, scale;  // bin = floor((v - lo) * scale), clamped
    int bins;
    int copies;        // LDS copies of the two histograms (1, 2 or 4)
    int stride;        // words from one copy to the next: 2 * bins + 1
    uint32_t *counts;  // [planes][2][bins]
};

__device__ __forceinline__ int bin_of(float v, double lo, double scale, int bins) {
    const double t = floor((static_cast<double>(v) - lo) * scale);
    // fmax / fmin return the non-NaN operand: NaN lands in bin 0
    return static_cast<int>(fmin(fmax(t, 0.0), static_cast<double>(bins - 1)));
}

template <typename T>
__global__ __launch_bounds__(kEmdThreads) void emd_hist_kernel(EmdArgs a) {
    extern __shared__ uint32_t lds[];  // [copies][stride]: [2][bins] and a pad word each
    const int plane = static_cast<int>(blockIdx.x) / a.parts;
    const int part = static_cast<int>(blockIdx.x) - plane * a.parts;
    for (int i = threadIdx.x; i < a.copies * a.stride; i += kEmdThreads) lds[i] = 0u;
    __syncthreads();
    uint32_t *hist = lds + (static_cast<int>(threadIdx.x) & (a.copies - 1)) * a.stride;
    const T *pa = static_cast<const T *>(a.cur) + static_cast<int64_t>(plane) * a.hw;
    const T *pb = static_cast<const T *>(a.prev) + static_cast<int64_t>(plane) * a.hw;
    const int64_t begin = static_cast<int64_t>(part) * a.run;
    const int64_t end = min(a.hw, begin + a.run);
    for (int64_t i0 = begin + threadIdx.x; i0 < end; i0 += kEmdThreads * kEmdUnroll) {
        // Coalesced loads, all in flight: past the run's end a thread reads
        // its last value again (counted nowhere) rather than skip the load,
        // so that no load, and no 16-bit conversion, sits in a branch (one
        // there is waited for before the next load issues).
        T ra[kEmdUnroll], rb[kEmdUnroll];
#pragma unroll
        for (int j = 0; j < kEmdUnroll; ++j) {
            const int64_t i = min(i0 + static_cast<int64_t>(j) * kEmdThreads, end - 1);
            ra[j] = pa[i];
            rb[j] = pb[i];
        }
#pragma unroll
        for (int j = 0; j < kEmdUnroll; ++j) {
            if (i0 + static_cast<int64_t>(j) * kEmdThreads < end) {
                atomicAdd(&hist[bin_of(to_f32(ra[j]), a.lo, a.scale, a.bins)], 1u);
                atomicAdd(&hist[a.bins + bin_of(to_f32(rb[j]), a.lo, a.scale, a.bins)], 1u);
            }
        }
    }
    __syncthreads();
    uint32_t *g = a.counts + static_cast<int64_t>(plane) * 2 * a.bins;
    for (int i = threadIdx.x; i < 2 * a.bins; i += kEmdThreads) {
        uint32_t t = lds[i];
        for (int k = 1; k < a.copies; ++k) t += lds[k * a.stride + i];
        if (t != 0u) atomicAdd(&g[i], t);
    }
}

// One workgroup per plane: S = sum_i |CA_i - CB_i| over the cumulative counts,
// in 64-bit integers (exact), then S / (H*W) * width.
__global__ __launch_bounds__(kEmdThreads) void emd_final_kernel(const uint32_t *counts, int bins,
                                                                int64_t hw, double width,
                                                                double *emd) {
    __shared__ long long part[kEmdThreads];
    const int plane = blockIdx.x;
    const uint32_t *ca = counts + static_cast<int64_t>(plane) * 2 * bins;
    const uint32_t *cb = ca + bins;
    const int per = (bins + kEmdThreads - 1) / kEmdThreads;
    const int b0 = min(bins, static_cast<int>(threadIdx.x) * per);
    const int b1 = min(bins, b0 + per);
    long long run = 0;
    for (int i = b0; i < b1; ++i) run += static_cast<long long>(ca[i]) - cb[i];
    // exclusive scan of the threads' totals (Hillis-Steele over LDS)
    part[threadIdx.x] = run;
    __syncthreads();
    for (int d = 1; d < kEmdThreads; d <<= 1) {
        const long long v = threadIdx.x >= static_cast<unsigned>(d) ? part[threadIdx.x - d] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    long long cum = part[threadIdx.x] - run;  // differences of the bins before b0
    long long s = 0;
    for (int i = b0; i < b1; ++i) {
        cum += static_cast<long long>(ca[i]) - cb[i];
        s += cum < 0 ? -cum : cum;
    }
    __syncthreads();
    part[threadIdx.x] = s;
    __syncthreads();
    for (int d = kEmdThreads / 2; d > 0; d >>= 1) {
        if (threadIdx.x < static_cast<unsigned>(d)) part[threadIdx.x] += part[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        emd[plane] = static_cast<double>(part[0]) / static_cast<double>(hw) * width;
}

}  // namespace

size_t buffer_emd_workspace_bytes(int n, int c, int bins) {
    return sizeof(uint32_t) * 2 * static_cast<size_t>(n) * c * bins;
}

hipError_t launch_buffer_emd(int dtype, const void *cur, const void *prev, int n, int c, int h,
                             int w, double lo, double hi, int bins, double *emd, void *workspace,
                             hipStream_t stream) {
    const int64_t planes = static_cast<int64_t>(n) * c;
    uint32_t *counts = static_cast<uint32_t *>(workspace);
    hipError_t e = launch_zero_u32(counts, planes * 2 * bins, stream);
    if (e != hipSuccess) return e;
    EmdArgs a;
    a.cur = cur;
    a.prev = prev;
    a.hw = static_cast<int64_t>(h) * w;
    const int64_t want = (a.hw + kEmdRun - 1) / kEmdRun;
    a.parts = static_cast<int>(want < kEmdMaxParts ? want : kEmdMaxParts);
    a.run = (a.hw + a.parts - 1) / a.parts;
    a.lo = lo;
    a.scale = static_cast<double>(bins) / (hi - lo);
    a.bins = bins;
    a.stride = 2 * bins + 1;
    a.copies = 4;
    while (a.copies > 1 && a.copies * a.stride > kEmdLdsWords) a.copies /= 2;
    a.counts = counts;
    const dim3 grid(static_cast<unsigned>(planes * a.parts));
    const size_t lds = sizeof(uint32_t) * a.copies * a.stride;
    switch (dtype) {
    case 0: hipLaunchKernelGGL(emd_hist_kernel<float>, grid, dim3(kEmdThreads), lds, stream, a); break;
    case 1: hipLaunchKernelGGL(emd_hist_kernel<_Float16>, grid, dim3(kEmdThreads), lds, stream, a); break;
    default: hipLaunchKernelGGL(emd_hist_kernel<__bf16>, grid, dim3(kEmdThreads), lds, stream, a); break;
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const double width = (hi - lo) / static_cast<double>(bins);
    hipLaunchKernelGGL(emd_final_kernel, dim3(static_cast<unsigned>(planes)), dim3(kEmdThreads), 0,
                       stream, counts, bins, a.hw, width, emd);
    return hipGetLastError();
}

}  // namespace exw
