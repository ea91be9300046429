/*
 * Float64 scalar-loop oracle of the motion-vector backward warp.
 * TEST INFRASTRUCTURE ONLY: linked by the test suite and timed as the CPU
 * baseline of the benchmark, never by the product path. Built with gcc, no HIP.
 *
 * Definition (paper §II-B image warping; §IV-B frames P_i at t + i/4 made from
 * F_t alone; §III-B invalid pixels of a warped frame; §III-D per-pixel motion):
 * output pixel (x, y) of frame n at phase s samples F_n bilinearly at
 * (x - s*u, y - s*v), (u, v) = mv[n, :, y, x]. The displacement d = s*u is
 * either exact (exact != 0: the float64 product of the float32 phase and
 * motion, which is exact since two 24-bit significands fit in 53 bits) or
 * rounded once to float32 (exact == 0: the motion field's precision, the one
 * a float32 implementation decides validity in); all later steps are float64.
 * Valid iff 0 <= sx <= W-1 and 0 <= sy <= H-1 (tested exactly on d); invalid
 * pixels are 0, mask 0, and are counted. Taps (x0, y0), (x1, y0), (x0, y1), (x1, y1) with
 * x0 = floor(sx), x1 = min(x0 + 1, W - 1), weights from the fractions.
 * Backward: the transpose of the gather for the image and the derivative of
 * the blend for the motion (d sx / d u = -s), summed over phases.
 *
 * Layouts: src [N,C,H,W] f64, mv [N,2,H,W] f32, phases [K] f32,
 * out [N,K,C,H,W] f64, mask [N,K,H,W] u8, invalid_count [N,K] i64,
 * grad_out [N,K,C,H,W] f64, grad_src [N,C,H,W] f64, grad_mv [N,2,H,W] f64.
 * All arrays are dense and owned by the caller. Returns 0, or -1 on bad sizes.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int valid;
    int64_t x0, x1, y0, y1;
    double fx, fy;
} taps_t;

static taps_t make_taps(float u, float v, float s, int64_t x, int64_t y, int64_t h, int64_t w,
                        int exact)
{
    taps_t t;
    double dx = (double)s * (double)u;
    double dy = (double)s * (double)v;
    if (!exact) {
        dx = (double)(float)dx;
        dy = (double)(float)dy;
    }
    memset(&t, 0, sizeof t);
    /* 0 <= x - d <= W-1 on d against integer bounds (exact even when |d| is
     * below half an ulp of x). */
    t.valid = (dx <= (double)x) && (dx >= (double)(x - (w - 1))) && (dy <= (double)y)
           && (dy >= (double)(y - (h - 1)));
    if (!t.valid)
        return t;
    /* floor(x - d) = x - ceil(d); fraction ceil(d) - d. */
    double cx = ceil(dx), cy = ceil(dy);
    t.x0 = x - (int64_t)cx;
    t.y0 = y - (int64_t)cy;
    t.fx = cx - dx;
    t.fy = cy - dy;
    t.x1 = t.x0 + 1 < w ? t.x0 + 1 : w - 1;
    t.y1 = t.y0 + 1 < h ? t.y0 + 1 : h - 1;
    return t;
}

int warp_ref_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void warp_ref_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int warp_ref_forward(const double *src, const float *mv, int64_t n, int64_t c, int64_t h,
                     int64_t w, const float *phases, int64_t k, double *out, uint8_t *mask,
                     int64_t *invalid_count, int exact)
{
    if (n < 0 || c < 1 || h < 1 || w < 1 || k < 1)
        return -1;
    const int64_t hw = h * w;
    for (int64_t i = 0; i < n * k; ++i)
        invalid_count[i] = 0;
#pragma omp parallel for collapse(3) schedule(static)
    for (int64_t in = 0; in < n; ++in)
        for (int64_t ik = 0; ik < k; ++ik)
            for (int64_t y = 0; y < h; ++y) {
                const double *img = src + in * c * hw;
                const float *u = mv + (in * 2 + 0) * hw;
                const float *v = mv + (in * 2 + 1) * hw;
                int64_t row_invalid = 0;
                for (int64_t x = 0; x < w; ++x) {
                    const int64_t p = y * w + x;
                    taps_t t = make_taps(u[p], v[p], phases[ik], x, y, h, w, exact);
                    mask[(in * k + ik) * hw + p] = (uint8_t)t.valid;
                    row_invalid += !t.valid;
                    for (int64_t ch = 0; ch < c; ++ch) {
                        double val = 0.0;
                        if (t.valid) {
                            const double *pl = img + ch * hw;
                            val = (1.0 - t.fx) * (1.0 - t.fy) * pl[t.y0 * w + t.x0]
                                + t.fx * (1.0 - t.fy) * pl[t.y0 * w + t.x1]
                                + (1.0 - t.fx) * t.fy * pl[t.y1 * w + t.x0]
                                + t.fx * t.fy * pl[t.y1 * w + t.x1];
                        }
                        out[((in * k + ik) * c + ch) * hw + p] = val;
                    }
                }
#pragma omp atomic
                invalid_count[in * k + ik] += row_invalid;
            }
    return 0;
}

int warp_ref_backward(const double *src, const float *mv, int64_t n, int64_t c, int64_t h,
                      int64_t w, const float *phases, int64_t k, const double *grad_out,
                      double *grad_src, double *grad_mv, int exact)
{
    if (n < 0 || c < 1 || h < 1 || w < 1 || k < 1)
        return -1;
    const int64_t hw = h * w;
    /* Motion gradient: one pixel at a time, summed over phases. */
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t in = 0; in < n; ++in)
        for (int64_t y = 0; y < h; ++y) {
            const double *img = src + in * c * hw;
            const float *u = mv + (in * 2 + 0) * hw;
            const float *v = mv + (in * 2 + 1) * hw;
            for (int64_t x = 0; x < w; ++x) {
                const int64_t p = y * w + x;
                double gu = 0.0, gv = 0.0;
                for (int64_t ik = 0; ik < k; ++ik) {
                    taps_t t = make_taps(u[p], v[p], phases[ik], x, y, h, w, exact);
                    if (!t.valid)
                        continue;
                    double su = 0.0, sv = 0.0;
                    for (int64_t ch = 0; ch < c; ++ch) {
                        const double *pl = img + ch * hw;
                        double i00 = pl[t.y0 * w + t.x0], i01 = pl[t.y0 * w + t.x1];
                        double i10 = pl[t.y1 * w + t.x0], i11 = pl[t.y1 * w + t.x1];
                        double g = grad_out[((in * k + ik) * c + ch) * hw + p];
                        su += g * ((1.0 - t.fy) * (i01 - i00) + t.fy * (i11 - i10));
                        sv += g * ((1.0 - t.fx) * (i10 - i00) + t.fx * (i11 - i01));
                    }
                    gu += -(double)phases[ik] * su;
                    gv += -(double)phases[ik] * sv;
                }
                grad_mv[(in * 2 + 0) * hw + p] = gu;
                grad_mv[(in * 2 + 1) * hw + p] = gv;
            }
        }
    /* Image gradient: transpose of the gather. Each (frame, channel) plane is
     * owned by one thread, so the scatter needs no synchronisation. */
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int64_t in = 0; in < n; ++in)
        for (int64_t ch = 0; ch < c; ++ch) {
            double *gs = grad_src + (in * c + ch) * hw;
            const float *u = mv + (in * 2 + 0) * hw;
            const float *v = mv + (in * 2 + 1) * hw;
            for (int64_t p = 0; p < hw; ++p)
                gs[p] = 0.0;
            for (int64_t ik = 0; ik < k; ++ik)
                for (int64_t y = 0; y < h; ++y)
                    for (int64_t x = 0; x < w; ++x) {
                        const int64_t p = y * w + x;
                        taps_t t = make_taps(u[p], v[p], phases[ik], x, y, h, w, exact);
                        if (!t.valid)
                            continue;
                        double g = grad_out[((in * k + ik) * c + ch) * hw + p];
                        gs[t.y0 * w + t.x0] += (1.0 - t.fx) * (1.0 - t.fy) * g;
                        gs[t.y0 * w + t.x1] += t.fx * (1.0 - t.fy) * g;
                        gs[t.y1 * w + t.x0] += (1.0 - t.fx) * t.fy * g;
                        gs[t.y1 * w + t.x1] += t.fx * t.fy * g;
                    }
        }
    return 0;
}
