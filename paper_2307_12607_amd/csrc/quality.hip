// Frame quality on CDNA4 (gfx950): per-frame MSE, PSNR and SSIM of a
// predicted frame against the ground truth (paper §IV-C1: the decision
// predictor's reward is the gain in PSNR = 10 log10(peak^2 / MSE) and in
// SSIM of the chosen action's frame over the other action's frame).
//
// SSIM is the Gaussian-window index (11 x 11 window, standard deviation 1.5,
// C1 = (0.01 peak)^2, C2 = (0.03 peak)^2) evaluated where the window lies
// inside the frame and averaged over those positions and the channels. The
// window is separable, so one wavefront owns a strip of 64 output columns x
// kStripRows output rows of one channel: each input row of the strip (plus
// the 10-pixel halo) is staged once in LDS, filtered horizontally in
// registers (window sums of x, y, x^2, y^2, xy), and added into the eleven
// output rows it contributes to, which live in registers as a ring indexed
// at compile time (the row loop is unrolled by 11). All filtering is float64:
// on this hardware float64 FMAs issue at the same rate as unpacked float32
// ones, and the local variances E[x^2] - E[x]^2 would otherwise lose their
// low digits. The squared differences for the MSE are summed in the same
// pass over each input pixel the strip owns. Partials are folded per frame
// in a fixed order, so the results are reproducible bit for bit.
#include <cmath>

#include "launch.h"
#include "warp_common.h"

namespace exw {
namespace {

constexpr int kWin = 11;
constexpr int kHalo = kWin - 1;
constexpr int kStripW = 64;     // output columns of a strip (one per lane)
constexpr int kStripRows = 66;  // output rows of a strip (a multiple of 11)

struct QualityArgs {
    const void *pred, *truth;
    int c, h, w;
    int strips_x, strips_y;
    double g[kWin];  // normalised 1-D Gaussian weights
    double c1, c2;
    double *partial;  // [B][C][strips_y][strips_x][2] = (ssim sum, squared-error sum)
};

template <typename T>
__device__ __forceinline__ float load_f32(const T *p, int64_t i) {
    return to_f32(p[i]);
}

template <typename T>
__global__ __launch_bounds__(64) void ssim_strip_kernel(QualityArgs a) {
    __shared__ float lx[kStripW + kHalo], ly[kStripW + kHalo];
    const int lane = threadIdx.x;
    int blk = blockIdx.x;
    const int sx = blk % a.strips_x;
    blk /= a.strips_x;
    const int sy = blk % a.strips_y;
    blk /= a.strips_y;
    const int ch = blk % a.c;
    const int frame = blk / a.c;
    const int w = a.w, h = a.h;
    const int64_t hw = static_cast<int64_t>(h) * w;
    const int64_t plane = (static_cast<int64_t>(frame) * a.c + ch) * hw;
    const T *px = static_cast<const T *>(a.pred) + plane;
    const T *py = static_cast<const T *>(a.truth) + plane;
    const int j0 = sx * kStripW, i0 = sy * kStripRows;
    const int out_w = w - kHalo, out_h = h - kHalo;
    const bool last_x = sx == a.strips_x - 1, last_y = sy == a.strips_y - 1;
    // Input rows this strip reads, and the rows whose squared errors it owns.
    const int rows_in = min(kStripRows, out_h - i0) + kHalo;
    const int own_rows = last_y ? h - i0 : kStripRows;
    const bool out_col = j0 + lane < out_w;

    double acc[kWin][5];
#pragma unroll
    for (int s = 0; s < kWin; ++s)
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[s][q] = 0.0;
    double ssim_sum = 0.0, sq_sum = 0.0;

    // The next input row is loaded while the current one is filtered.
    const int ca = min(j0 + lane, w - 1);
    const int cb = min(j0 + kStripW + lane, w - 1);
    float nxa, nya, nxb = 0.0f, nyb = 0.0f;
    nxa = load_f32(px, static_cast<int64_t>(i0) * w + ca);
    nya = load_f32(py, static_cast<int64_t>(i0) * w + ca);
    if (lane < kHalo) {
        nxb = load_f32(px, static_cast<int64_t>(i0) * w + cb);
        nyb = load_f32(py, static_cast<int64_t>(i0) * w + cb);
    }
    for (int base = 0; base < rows_in; base += kWin) {
#pragma unroll
        for (int s = 0; s < kWin; ++s) {
            const int r = base + s;  // input row of the strip (wave-uniform)
            if (r < rows_in) {
                const float xa = nxa, ya = nya, xb = nxb, yb = nyb;
                if (r + 1 < rows_in) {
                    const int64_t next = static_cast<int64_t>(i0 + r + 1) * w;
                    nxa = load_f32(px, next + ca);
                    nya = load_f32(py, next + ca);
                    if (lane < kHalo) {
                        nxb = load_f32(px, next + cb);
                        nyb = load_f32(py, next + cb);
                    }
                }
                __syncthreads();  // previous row's taps have been read
                lx[lane] = xa;
                ly[lane] = ya;
                if (lane < kHalo) {
                    lx[kStripW + lane] = xb;
                    ly[kStripW + lane] = yb;
                }
                __syncthreads();
                // squared errors of the input pixels this strip owns
                if (r < own_rows) {
                    if (j0 + lane < w && (last_x || lane < kStripW)) {
                        const double d = static_cast<double>(xa) - ya;
                        sq_sum = fma(d, d, sq_sum);
                    }
                    if (last_x && lane < kHalo && j0 + kStripW + lane < w) {
                        const double d = static_cast<double>(xb) - yb;
                        sq_sum = fma(d, d, sq_sum);
                    }
                }
                // horizontal window sums at output column j0 + lane
                double hx = 0.0, hy = 0.0, hxx = 0.0, hyy = 0.0, hxy = 0.0;
#pragma unroll
                for (int b = 0; b < kWin; ++b) {
                    const double xv = lx[lane + b], yv = ly[lane + b];
                    const double tx = a.g[b] * xv, ty = a.g[b] * yv;
                    hx += tx;
                    hy += ty;
                    hxx = fma(tx, xv, hxx);
                    hyy = fma(ty, yv, hyy);
                    hxy = fma(tx, yv, hxy);
                }
                // input row r feeds output rows r - t, t = 0..10, kept in ring
                // slot (r - t) mod 11 = (s - t) mod 11 (static)
#pragma unroll
                for (int t = 0; t < kWin; ++t) {
                    const int slot = (s - t + kWin) % kWin;
                    acc[slot][0] = fma(a.g[t], hx, acc[slot][0]);
                    acc[slot][1] = fma(a.g[t], hy, acc[slot][1]);
                    acc[slot][2] = fma(a.g[t], hxx, acc[slot][2]);
                    acc[slot][3] = fma(a.g[t], hyy, acc[slot][3]);
                    acc[slot][4] = fma(a.g[t], hxy, acc[slot][4]);
                }
                // output row r - 10 is complete (slot (s + 1) mod 11)
                const int slot = (s + 1) % kWin;
                if (r >= kHalo) {
                    const double mx = acc[slot][0], my = acc[slot][1];
                    const double vx = acc[slot][2] - mx * mx;
                    const double vy = acc[slot][3] - my * my;
                    const double cxy = acc[slot][4] - mx * my;
                    const double num = (2.0 * mx * my + a.c1) * (2.0 * cxy + a.c2);
                    const double den = (mx * mx + my * my + a.c1) * (vx + vy + a.c2);
                    if (out_col) ssim_sum += num / den;
                }
#pragma unroll
                for (int q = 0; q < 5; ++q) acc[slot][q] = 0.0;
            }
        }
    }
    // wavefront sums (butterfly; addition is commutative, so every lane agrees)
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        ssim_sum += __shfl_xor(ssim_sum, m);
        sq_sum += __shfl_xor(sq_sum, m);
    }
    if (lane == 0) {
        const int64_t idx =
            ((static_cast<int64_t>(frame) * a.c + ch) * a.strips_y + sy) * a.strips_x + sx;
        a.partial[2 * idx] = ssim_sum;
        a.partial[2 * idx + 1] = sq_sum;
    }
}

// One wavefront per frame folds its partials in a fixed order.
__global__ __launch_bounds__(64) void quality_final_kernel(const double *partial, int per_frame,
                                                           double n_px, double n_pos,
                                                           double peak, double *quality) {
    const int frame = blockIdx.x;
    const double *p = partial + 2 * static_cast<int64_t>(frame) * per_frame;
    double s = 0.0, q = 0.0;
    for (int i = threadIdx.x; i < per_frame; i += 64) {
        s += p[2 * i];
        q += p[2 * i + 1];
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        s += __shfl_xor(s, m);
        q += __shfl_xor(q, m);
    }
    if (threadIdx.x == 0) {
        const double mse = q / n_px;
        quality[3 * frame] = mse;
        quality[3 * frame + 1] = 10.0 * log10(peak * peak / mse);
        quality[3 * frame + 2] = s / n_pos;
    }
}

void strips(int h, int w, int &sx, int &sy) {
    sx = (w - kHalo + kStripW - 1) / kStripW;
    sy = (h - kHalo + kStripRows - 1) / kStripRows;
}

}  // namespace

size_t quality_workspace_bytes(int b, int c, int h, int w) {
    int sx, sy;
    strips(h, w, sx, sy);
    return sizeof(double) * 2 * static_cast<size_t>(b) * c * sx * sy;
}

hipError_t launch_quality(int dtype, const void *pred, const void *truth, int b, int c, int h,
                          int w, double peak, double *quality, void *workspace,
                          hipStream_t stream) {
    QualityArgs a;
    a.pred = pred;
    a.truth = truth;
    a.c = c;
    a.h = h;
    a.w = w;
    strips(h, w, a.strips_x, a.strips_y);
    double e[kWin], sum = 0.0;
    for (int i = 0; i < kWin; ++i) {
        const double r = i - (kWin - 1) / 2;
        e[i] = std::exp(-(r * r) / (2.0 * 1.5 * 1.5));
        sum += e[i];
    }
    for (int i = 0; i < kWin; ++i) a.g[i] = e[i] / sum;
    a.c1 = (0.01 * peak) * (0.01 * peak);
    a.c2 = (0.03 * peak) * (0.03 * peak);
    a.partial = static_cast<double *>(workspace);
    const int per_frame = c * a.strips_x * a.strips_y;
    const dim3 grid(static_cast<unsigned>(static_cast<int64_t>(b) * per_frame));
    switch (dtype) {
    case 0: hipLaunchKernelGGL(ssim_strip_kernel<float>, grid, dim3(64), 0, stream, a); break;
    case 1: hipLaunchKernelGGL(ssim_strip_kernel<_Float16>, grid, dim3(64), 0, stream, a); break;
    default: hipLaunchKernelGGL(ssim_strip_kernel<__bf16>, grid, dim3(64), 0, stream, a); break;
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const double n_px = static_cast<double>(c) * h * w;
    const double n_pos = static_cast<double>(c) * (h - kHalo) * (w - kHalo);
    hipLaunchKernelGGL(quality_final_kernel, dim3(static_cast<unsigned>(b)), dim3(64), 0, stream,
                       a.partial, per_frame, n_px, n_pos, peak, quality);
    return hipGetLastError();
}

}  // namespace exw
