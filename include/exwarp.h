/*
 * exwarp — motion-vector frame warping on AMD Instinct MI355X (gfx950).
 *
 * The fast branch of ExWarp predicts the frames shown between two rendered
 * frames by warping the last rendered frame F_t (paper §II-B: warping maps
 * every location of one image to a location in another) with its per-pixel
 * motion vectors (§III-D), for the display instants t + i/4, i = 1..3
 * (§IV-B, problem formulation: P_i is made from F_t alone, without F_t+1).
 * Warped pixels whose source lies outside the frame are marked invalid
 * (§III-B). The adjoint gives the gradients needed to train a learned
 * extrapolator through the warp.
 *
 * Definition of one output pixel (x, y) of frame n at phase s:
 *   (u, v) = mv[n, 0:2, y, x]           motion of the content over one
 *                                       rendered-frame interval, in pixels,
 *                                       +x right, +y down
 *   d = (s*u, s*v) rounded to float32   displacement
 *   (sx, sy) = (x - d.x, y - d.y)       sample point in F_n, pixel-index units
 *   valid  <=>  0 <= sx <= W-1  and  0 <= sy <= H-1   (NaN/Inf -> invalid)
 *   out[c] = bilinear sample of F_n[c] at (sx, sy), taps (x0, y0)..(x0+1, y0+1),
 *            x0 = floor(sx), second index clamped to W-1 / H-1 (its weight is 0
 *            there); out = 0 in every channel and mask = 0 where invalid.
 * Coordinates, weights and blending are float32; frames may be stored as
 * float32, float16 or bfloat16 (results are rounded to nearest-even into the
 * storage type); motion vectors are always float32.
 *
 * Layouts (all dense, row-major, no padding):
 *   src       [N, C, H, W]     storage dtype          (the frames F_t)
 *   mv        [N, 2, H, W]     float32                (u plane, then v plane)
 *   out       [N, K, C, H, W]  storage dtype          (P for each phase)
 *   mask      [N, K, H, W]     uint8, 1 = valid
 *   invalid_count [N, K]       uint32
 *   grad_out  [N, K, C, H, W]  storage dtype
 *   grad_src  [N, C, H, W]     storage dtype
 *   grad_mv   [N, 2, H, W]     float32
 *
 * Conventions for every call:
 *   - Device pointers are HIP device memory on the current device; `phases`
 *     is a HOST array of K floats read before the call returns.
 *   - The caller owns all memory. The library allocates nothing and keeps no
 *     pointer after a call returns.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream)
 *     and the call returns without synchronising. Faults inside kernels
 *     surface at the caller's next synchronisation.
 *   - Outputs are overwritten, never accumulated into.
 *   - Arguments are fully validated before any HIP call; a rejected call
 *     enqueues nothing and returns EXW_ERROR_INVALID_VALUE or
 *     EXW_ERROR_UNSUPPORTED with a message in exw_last_error().
 *   - Outputs may not overlap inputs or each other (no in-place warping).
 *   - A batch with N = 0, H = 0 or W = 0 is valid and does no work beyond
 *     zeroing invalid_count (if given).
 *   - Thread-safe: the only state is the calling thread's last error string.
 */
#ifndef EXWARP_H
#define EXWARP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EXW_ABI_VERSION 2
#define EXW_MAX_PHASES 4   /* K, phases fused into one launch */
#define EXW_MAX_CHANNELS 64

typedef enum exw_dtype {
    EXW_F32 = 0,   /* IEEE binary32 */
    EXW_F16 = 1,   /* IEEE binary16 */
    EXW_BF16 = 2   /* bfloat16: the upper 16 bits of a binary32 */
} exw_dtype;

typedef enum exw_status {
    EXW_SUCCESS = 0,
    EXW_ERROR_INVALID_VALUE = 1, /* bad pointer, size, alignment, overlap, phase */
    EXW_ERROR_UNSUPPORTED = 2,   /* valid request beyond what this library handles */
    EXW_ERROR_LAUNCH = 3         /* a HIP call or kernel launch failed */
} exw_status;

/* Returns EXW_ABI_VERSION of the built library. */
int exw_abi_version(void);

/* Static, never-NULL name of a status code ("EXW_SUCCESS", ...). */
const char *exw_status_string(int status);

/* Detail of the calling thread's last failed call ("" after a success).
 * Valid until the thread's next exwarp call. */
const char *exw_last_error(void);

/*
 * Forward warp of N frames at K phases in one launch (paper §IV-B: the three
 * predicted frames P_1..P_3 at t + 1/4, 2/4, 3/4 come from the same F_t, so
 * the motion field and source frame are read once for all K).
 *   src, mv, out: required device pointers (layouts above).
 *   phases: host array of k finite floats (s = i/4 in the method; any finite
 *           value is accepted, 0 gives the identity).
 *   k: 1..EXW_MAX_PHASES.   n >= 0, 1 <= c <= EXW_MAX_CHANNELS, h, w >= 0,
 *   h*w <= 2^30. Larger batches than the launch grids hold (below 2^31
 *   tiles of 64 x 4 pixels; for twelve 16-bit channels also below 2^31 row
 *   segments of 128 pixels, counting rows in fours) are EXW_ERROR_UNSUPPORTED.
 *   mask: optional [N,K,H,W] uint8 output, or NULL.
 *   invalid_count: optional [N,K] uint32 output (number of invalid pixels
 *           per frame and phase, paper §III-C holes statistic restricted to
 *           out-of-frame sources), or NULL.
 */
exw_status exw_warp_forward_batched(const void *src, exw_dtype dtype, int32_t n, int32_t c,
                                    int32_t h, int32_t w, const float *mv, const float *phases,
                                    int32_t k, void *out, uint8_t *mask,
                                    uint32_t *invalid_count, void *stream);

/* One frame [C,H,W] at one phase; same as the batched call with N = K = 1
 * (out [C,H,W], mask [H,W] or NULL). */
exw_status exw_warp_forward(const void *src, exw_dtype dtype, int32_t c, int32_t h, int32_t w,
                            const float *mv, float phase, void *out, uint8_t *mask,
                            void *stream);

/* Bytes of device workspace exw_warp_backward_batched (and the training pair)
 * needs when grad_src is requested: per row segment (64 output pixels of a
 * row) a 16-byte tap box and 16 bytes of tap offsets, 8 bytes per frame, the
 * recording forward's motion statistics (48 bytes per 128 x 4 tile of each
 * frame, at least one per 2048 pixels and at most 256 per frame, plus 392
 * bytes per frame for their fold), and for EXW_F16/EXW_BF16 a float32
 * image-gradient accumulator of 4*N*C*H*W bytes. Returns 0 for an invalid
 * dtype or an empty batch. */
size_t exw_warp_backward_workspace_bytes(exw_dtype dtype, int32_t n, int32_t c, int32_t h,
                                         int32_t w);

/*
 * Adjoint of exw_warp_forward_batched: given grad_out = dL/d out, writes
 *   grad_src = dL/d src  = sum over k of the transpose of the bilinear gather
 *              (each valid output pixel sends weight * grad_out to its four
 *              taps), accumulated in float32 and rounded once into dtype;
 *   grad_mv  = dL/d mv   = -s * sum_c grad_out[c] * d out[c]/d(sx, sy),
 *              summed over k, 0 at invalid pixels; at a floor kink the
 *              derivative is the one-sided one of the cell the pixel samples.
 * The derivative treats the displacement as s*u exactly (its float32
 * rounding is not differentiated). The phase and the mask get no gradient.
 *   src: required if grad_mv is requested, else may be NULL.
 *   grad_src: optional (NULL = not computed). grad_mv: optional.
 *   workspace: required when grad_src is requested: device memory of at least
 *           exw_warp_backward_workspace_bytes(...) bytes, 256-byte aligned;
 *           its contents are scratch. May be NULL when grad_src is NULL.
 * The image gradient is formed by gathering, per tile of the image, the
 * contributions of the output pixels whose taps land there (LDS
 * accumulation, plain stores); output segments whose taps lie more than 128
 * px away fall back to float32 atomics. The summation order is fixed except
 * where atomics are used (taps at motion boundaries of frames with 1, 2, 4
 * or 12 channels are added with LDS atomics, far segments with global ones),
 * so the last bits of grad_src can differ from run to run.
 */
exw_status exw_warp_backward_batched(const void *src, exw_dtype dtype, int32_t n, int32_t c,
                                     int32_t h, int32_t w, const float *mv, const float *phases,
                                     int32_t k, const void *grad_out, void *grad_src,
                                     float *grad_mv, void *workspace, size_t workspace_bytes,
                                     void *stream);

/* One frame at one phase; same as the batched call with N = K = 1. */
exw_status exw_warp_backward(const void *src, exw_dtype dtype, int32_t c, int32_t h, int32_t w,
                             const float *mv, float phase, const void *grad_out, void *grad_src,
                             float *grad_mv, void *workspace, size_t workspace_bytes,
                             void *stream);

/*
 * Training pair: the forward and its adjoint with the adjoint's first pass
 * (the footprint of every 64-pixel output row segment: the box its taps
 * cover and, under rigid motion, its integer tap offsets) done inside the
 * forward, which already forms every displacement and tap offset.
 *
 * exw_warp_forward_batched_record: exw_warp_forward_batched, plus the
 *   footprint of this motion and these phases written into `workspace`
 *   (device memory of at least exw_warp_backward_workspace_bytes(dtype, n, c,
 *   h, w) bytes, 256-byte aligned, disjoint from every input and output;
 *   required unless the batch is empty). The outputs equal those of
 *   exw_warp_forward_batched.
 *   motion_stats: optional [N, 4] float64 device output (8-byte aligned), or
 *   NULL: the per-frame motion statistics of exw_motion_stats (mean and
 *   population variance of each motion component, paper §IV-C, Eq. 1),
 *   formed from the motion the forward reads anyway: each 128 x 4 tile folds
 *   its values into a float64 (count, mean, M2) partial kept in the
 *   workspace, and the partials of a frame are folded in a fixed order, so
 *   the results are reproducible bit for bit (they may differ from
 *   exw_motion_stats in the last bits: another order of the same fold).
 *   With NULL the forward does none of this work. Requesting it for frames
 *   with H = 0 or W = 0 is EXW_ERROR_INVALID_VALUE.
 * exw_warp_backward_batched_recorded: exw_warp_backward_batched, taking the
 *   footprint from `workspace` instead of computing it. The caller guarantees
 *   that the workspace was last written by exw_warp_forward_batched_record
 *   with the same mv contents, phases, dtype and shape, on this stream or
 *   ordered before this call; anything else gives wrong image gradients
 *   (not detected). Validation and errors are those of
 *   exw_warp_backward_batched; the workspace is still the adjoint's scratch.
 */
exw_status exw_warp_forward_batched_record(const void *src, exw_dtype dtype, int32_t n, int32_t c,
                                           int32_t h, int32_t w, const float *mv,
                                           const float *phases, int32_t k, void *out,
                                           uint8_t *mask, uint32_t *invalid_count,
                                           double *motion_stats, void *workspace,
                                           size_t workspace_bytes, void *stream);

exw_status exw_warp_backward_batched_recorded(const void *src, exw_dtype dtype, int32_t n,
                                              int32_t c, int32_t h, int32_t w, const float *mv,
                                              const float *phases, int32_t k,
                                              const void *grad_out, void *grad_src,
                                              float *grad_mv, void *workspace,
                                              size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Scene-state statistics that accompany a warp.
 *
 * Paper §IV-C (Eq. 1): the state the warp/extrapolate decision is taken on includes the
 * variance of the motion-vector buffer, horizontally and vertically
 * (Var_x(F_mv), Var_y(F_mv) in the environment vector E_t; Table IV lists the
 * motion variance as the feature that reveals dynamic objects). Here it is
 * the population variance over all H*W per-pixel vectors of a frame.
 * ------------------------------------------------------------------------ */

/* Bytes of device workspace exw_motion_stats needs for N frames of H x W:
 * 48 bytes per workgroup partial, one partial per 2048 pixels of a frame and
 * at most 256 per frame. Returns 0 for an empty batch. */
size_t exw_motion_stats_workspace_bytes(int32_t n, int32_t h, int32_t w);

/*
 * Per-frame motion statistics:
 *   stats[n][0] = mean of mv[n, 0]   stats[n][1] = population variance of mv[n, 0]
 *   stats[n][2] = mean of mv[n, 1]   stats[n][3] = population variance of mv[n, 1]
 * in float64, over all H*W values of each plane.
 *   mv:        [N, 2, H, W] float32, device, 4-byte aligned.
 *   stats:     [N, 4] float64, device, 8-byte aligned; overwritten.
 *   workspace: device scratch of at least exw_motion_stats_workspace_bytes()
 *              bytes, 256-byte aligned.
 * Each frame is read once; per-thread chunks, lanes, wavefronts and
 * workgroups are combined with the pairwise (count, mean, sum of squared
 * deviations) update in float64, in a fixed order: the result is
 * reproducible bit for bit and does not cancel when the mean is large
 * against the spread. A non-finite value makes its component's mean and
 * variance non-finite. N = 0 does nothing; N > 0 with H = 0 or W = 0 is
 * EXW_ERROR_INVALID_VALUE (an empty frame has no variance); N >= 2^21 or
 * H*W > 2^30 is EXW_ERROR_UNSUPPORTED.
 */
exw_status exw_motion_stats(const float *mv, int32_t n, int32_t h, int32_t w, double *stats,
                            void *workspace, size_t workspace_bytes, void *stream);

/*
 * exw_motion_stats without a workspace and without any allocation, for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc. The workgroup
 * partials live in a file-scope device array of EXW_NO_ALLOC_SCRATCH_BYTES
 * bytes that the library holds on each GPU it runs on until the process
 * ends (its address is looked up once per device, on the first call with
 * that device current). Same arguments, results and errors as
 * exw_motion_stats minus the workspace; a batch whose partials need more
 * than EXW_NO_ALLOC_SCRATCH_BYTES (exw_motion_stats_workspace_bytes(n, h, w)
 * > EXW_NO_ALLOC_SCRATCH_BYTES: e.g. more than 85 frames of 1080p) is
 * EXW_ERROR_UNSUPPORTED. All calls on one GPU share that array: calls that
 * overlap in time on one GPU (other streams, other threads) race and give
 * wrong statistics; calls ordered on one stream are safe (each call writes
 * every partial it reads, so nothing needs clearing between calls).
 */
#define EXW_NO_ALLOC_SCRATCH_BYTES (1u << 20)
exw_status exw_motion_stats_no_alloc(const float *mv, int32_t n, int32_t h, int32_t w,
                                     double *stats, void *stream);

/* ------------------------------------------------------------------------
 * EMD features of the state.
 *
 * Paper §III-D (State Representation) and Table IV: the change of the world
 * normal and world position buffers from F_t-1 to F_t is measured with the
 * Earth Mover's Distance (EMD_{W_N}, EMD_{W_P}, entries of E_t in §IV-C,
 * Eq. 1). The paper names the metric, not how a buffer becomes a
 * distribution; here each channel's values over the frame form a histogram
 * of `bins` uniform bins on [lo, hi], and the EMD of the two unit-mass
 * histograms with ground distance |i - j| * width (width = (hi - lo) / bins)
 * is, in one dimension, sum_i |CA_i - CB_i| / (H*W) * width over the
 * cumulative counts CA, CB. A buffer's feature is the sum over its channels.
 * ------------------------------------------------------------------------ */

#define EXW_EMD_MAX_BINS 4096

/* Bytes of device workspace exw_buffer_emd needs: 2 * bins 32-bit counters
 * per frame and channel. Returns 0 for an empty batch or bins out of range. */
size_t exw_buffer_emd_workspace_bytes(int32_t n, int32_t c, int32_t bins);

/*
 * Per-frame, per-channel EMD between two buffers:
 *   emd[n][c] = EMD between the values of cur[n, c] and of prev[n, c].
 *   cur, prev: [N, C, H, W] in `dtype` (the buffer of F_t and of F_t-1),
 *              device, aligned to the element size.
 *   lo < hi:   finite float64 range of the bins; a value v falls in bin
 *              floor((v - lo) * (bins / (hi - lo))), computed in float64
 *              and clamped to [0, bins - 1] (values outside [lo, hi] join
 *              the end bins; NaN joins bin 0).
 *   bins:      1 .. EXW_EMD_MAX_BINS.
 *   emd:       [N, C] float64, device, 8-byte aligned; overwritten.
 *   workspace: device scratch of at least exw_buffer_emd_workspace_bytes()
 *              bytes, 256-byte aligned.
 * Counts are integers, so results do not depend on the order of the
 * atomics that build them. N = 0 does nothing; N > 0 with H = 0 or W = 0 is
 * EXW_ERROR_INVALID_VALUE (an empty frame has no distribution).
 */
exw_status exw_buffer_emd(const void *cur, const void *prev, exw_dtype dtype, int32_t n,
                          int32_t c, int32_t h, int32_t w, double lo, double hi, int32_t bins,
                          double *emd, void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * N_D, the number of dynamic objects (paper §III-D, State Representation:
 * the custom stencil buffer marks the pixels of dynamic objects, which are
 * found by clustering it; Table IV; §IV-C, Eq. 1: an entry of E_t). The
 * paper names no clustering method; here an object is a connected component
 * of the marked pixels (stencil value non-zero), two marked pixels being
 * joined when they share an edge (4-connectivity) or an edge or a corner
 * (8-connectivity). Objects that touch or overlap count once.
 * ------------------------------------------------------------------------ */

/* Bytes of device workspace exw_dynamic_objects needs: one int32 label per
 * pixel (4 * N * H * W). Returns 0 for an empty batch. */
size_t exw_dynamic_objects_workspace_bytes(int32_t n, int32_t h, int32_t w);

/*
 * count[n] = number of connected components of the marked pixels of frame n.
 *   stencil:      [N, H, W] uint8, device (marked = non-zero).
 *   connectivity: 4 or 8.
 *   count:        [N] uint32, device, 4-byte aligned; overwritten.
 *   workspace:    device scratch of at least exw_dynamic_objects_workspace_bytes()
 *                 bytes, 256-byte aligned.
 * The count is exact and does not depend on the order in which the GPU
 * joins pixels. N = 0 does nothing; frames with H = 0 or W = 0 have no
 * objects (count 0). H * W is at most 2^30.
 */
exw_status exw_dynamic_objects(const uint8_t *stencil, int32_t n, int32_t h, int32_t w,
                               int32_t connectivity, uint32_t *count, void *workspace,
                               size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Frame quality.
 *
 * Paper §IV-C1: the reward of the warp/extrapolate decision is the gain in PSNR
 * (10 log10(peak^2 / MSE)) and in SSIM of the frame an action produces over
 * the frame the other action would have produced, both against the ground
 * truth.
 * ------------------------------------------------------------------------ */

/* Bytes of device workspace exw_frame_quality needs: 16 bytes per strip of
 * 64 x 66 SSIM positions of each channel of each frame. Returns 0 for an
 * empty batch or frames below 11 x 11. */
size_t exw_frame_quality_workspace_bytes(int32_t b, int32_t c, int32_t h, int32_t w);

/*
 * Per-frame quality of B predicted frames against B ground-truth frames:
 *   quality[b][0] = MSE  = mean over C*H*W of (pred - truth)^2
 *   quality[b][1] = PSNR = 10 log10(peak^2 / MSE)  (+inf when MSE = 0)
 *   quality[b][2] = SSIM = mean over channels and over the (H-10)*(W-10)
 *                   positions where the window fits, of the index of Wang et
 *                   al. (2004): 11 x 11 Gaussian window, standard deviation
 *                   1.5, normalised; C1 = (0.01 peak)^2, C2 = (0.03 peak)^2.
 *   pred, truth: [B, C, H, W] in `dtype` (any leading batch shape flattened
 *                into B, e.g. the [N, K, C, H, W] output of a warp), device,
 *                aligned to the element size.
 *   quality:     [B, 3] float64, device, 8-byte aligned; overwritten.
 *   workspace:   device scratch of at least exw_frame_quality_workspace_bytes()
 *                bytes, 256-byte aligned.
 *   peak:        the value range of the frames (1.0 for unit-range frames;
 *                the paper's 255 for 8-bit frames), finite and > 0.
 * All window sums, the SSIM index and the sums are float64; the order of
 * every sum is fixed, so results are reproducible bit for bit. B = 0 does
 * nothing; H or W below 11 is EXW_ERROR_INVALID_VALUE.
 */
exw_status exw_frame_quality(const void *pred, const void *truth, exw_dtype dtype, int32_t b,
                             int32_t c, int32_t h, int32_t w, double peak, double *quality,
                             void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Decision paths (paper §IV-B, Table V).
 *
 * Between rendered frames F_t and F_t+1 the frames P_1, P_2, P_3 are shown
 * at t + 1/4, 2/4, 3/4. Decision d1 (at t) shows W(F_t) at t + 1/4, or F_t
 * again, after which the extrapolation E(F_t) is shown at t + 1/2. After
 * d1 = warp, d2 (at t + 1/4) shows W(P_1) or E(F_t) at t + 1/2. At t + 1/2
 * one more decision picks P_3: d3 (after d1 = extrapolate) between W(P_2) and
 * P_2 again; d4 (after d2 = warp) and d5 (after d2 = extrapolate) between
 * W(P_2) and E(P_1). The six paths are Table V's scenarios S1..S6.
 * A warp of a predicted frame, W(P_i), is the forward warp of P_i with the
 * motion of F_t at phase 1/4 (one display interval).
 * ------------------------------------------------------------------------ */

#define EXW_DECIDE_NONE (-1)
#define EXW_DECIDE_WARP 0
#define EXW_DECIDE_EXTRAPOLATE 1

#define EXW_SHOW_REPEAT 0       /* the previous frame again (no new frame) */
#define EXW_SHOW_WARP 1         /* W(source) */
#define EXW_SHOW_EXTRAPOLATE 2  /* E(source), made by an extrapolator */

#define EXW_FROM_RENDERED 0     /* F_t */
#define EXW_FROM_P1 1
#define EXW_FROM_P2 2

typedef struct {
    int32_t scenario;    /* 1..6: Table V's S1..S6 */
    int32_t kind[3];     /* P_1..P_3: EXW_SHOW_* */
    int32_t source[3];   /* P_1..P_3: EXW_FROM_* */
    int32_t node[3];     /* decision node taken at t, t + 1/4, t + 1/2 (1..5; 0 = none) */
    int32_t new_frames;  /* frames made between F_t and F_t+1; upsampling = new_frames + 1 */
} exw_display_plan;

/*
 * The frames shown for the decisions d1 (at t), d2 (at t + 1/4; ignored,
 * pass EXW_DECIDE_NONE, when d1 extrapolates) and d_last (at t + 1/2: node
 * d3, d4 or d5), each EXW_DECIDE_WARP or EXW_DECIDE_EXTRAPOLATE (at d3,
 * "extrapolate" means P_2 is shown again). Host-only; writes *plan.
 * Returns EXW_ERROR_INVALID_VALUE for a NULL plan or an invalid decision.
 */
exw_status exw_decision_plan(int32_t d1, int32_t d2, int32_t d_last, exw_display_plan *plan);

/*
 * A fixed policy for the three decisions of one frame (a stand-in for the
 * paper's learned predictor, §IV-C, which needs trained weights): warp at a
 * node when Var_x + Var_y of the frame's motion (motion_stats[1] +
 * motion_stats[3], the layout of exw_motion_stats) is at most max_variance
 * and the out-of-frame fraction of the warp that node would show is at most
 * max_invalid; else extrapolate. invalid_fraction[0..2] are those fractions
 * of W(F_t) at phases 1/4, 2/4, 3/4 (invalid_count / (H*W) of the forward
 * warp); node d1 looks at [0], d2 at [1], the node at t + 1/2 at [2].
 * Writes decisions[0..2] = (d1, d2 or EXW_DECIDE_NONE, d_last). Host-only;
 * all pointers are host memory.
 */
exw_status exw_threshold_policy(const double *motion_stats, const double *invalid_fraction,
                                double max_variance, double max_invalid, int32_t *decisions);

/*
 * Chained warps: out[0] = W(src, phase), out[i] = W(out[i-1], phase), each
 * with the same motion mv (the warps W(P_i) of the decision paths, phase
 * 1/4). Each step is the forward warp of exw_warp_forward_batched applied
 * to the previous step's stored output (rounded to dtype).
 *   src [N, C, H, W] dtype; mv [N, 2, H, W] float32;
 *   out [S, N, C, H, W] dtype (step-major, so each step is a contiguous batch);
 *   mask [S, N, H, W] uint8 or NULL; invalid_count [S, N] uint32 or NULL:
 *   each step's own out-of-frame test.
 *   steps S >= 1; phase finite. Same conventions and limits as the forward.
 */
exw_status exw_warp_chain(const void *src, exw_dtype dtype, int32_t n, int32_t c, int32_t h,
                          int32_t w, const float *mv, float phase, int32_t steps, void *out,
                          uint8_t *mask, uint32_t *invalid_count, void *stream);

/* ------------------------------------------------------------------------
 * Measurement: plain HBM streams.
 *
 * Not part of the method: the bandwidth ceiling the warp kernels are
 * measured against (a copy, a read-only and a write-only sweep of device
 * memory, 16 bytes per lane, one pass). The warp's algorithmic bytes per
 * second are reported as a fraction of the vendor peak and of these.
 *   bytes: a multiple of 16; pointers 16-byte aligned device memory.
 *   exw_stream_copy: dst[0, bytes) = src[0, bytes); the ranges may not overlap.
 *   exw_stream_read: reads src[0, bytes); `sink` (4 bytes of device memory,
 *                    4-byte aligned) is never written but must be valid.
 *   exw_stream_write: writes zeros to dst[0, bytes).
 * Same conventions as the warp calls (stream, validation, no allocation).
 * ------------------------------------------------------------------------ */
exw_status exw_stream_copy(const void *src, void *dst, size_t bytes, void *stream);
exw_status exw_stream_read(const void *src, size_t bytes, float *sink, void *stream);
exw_status exw_stream_write(void *dst, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* EXWARP_H */
