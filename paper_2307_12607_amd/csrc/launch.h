// Internal interface between the C-ABI layer (api.cpp) and the HIP kernels
// (warp_forward.hip, warp_backward.hip). Arguments arrive here validated.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "exwarp.h"

namespace exw {

// Record the calling thread's last error (or clear it on success) for host
// entry points outside api.cpp; returns st.
exw_status report(exw_status st, const char *msg);

struct WarpShape {
    int n, c, h, w, k;
    float phases[4];
};

struct Phases4 {
    float s[4];
};

// Device scratch of the adjoint, carved from the caller's workspace.
struct BwdWorkspace {
    void *boxes;     // per row segment: bounding box of its taps
    void *info;      // per frame: reach of the segments, far flag
    float *accum32;  // float32 image-gradient accumulator (16-bit storage only)
    bool recorded;   // boxes and info already hold the footprint of this motion and these phases
    void *stat_parts;  // motion-statistics partials of the recording forward (or NULL)
};

// Bytes of the recording forward's motion statistics for N frames of H x W:
// 48 bytes per 128 x 4 tile of each frame, the fold's 384 bytes of slots and
// 8 bytes of counters per frame.
size_t record_stats_bytes(int n, int h, int w);

size_t backward_box_bytes(int n, int h, int w);
size_t backward_info_bytes(int n);

// Whether the adjoint of C channels reads the footprint records (its tile path).
bool backward_uses_footprint(int c);

// The adjoint's footprint pass alone (records into ws.boxes, ws.info).
hipError_t launch_footprint(const float *mv, const WarpShape &s, const BwdWorkspace &ws,
                            hipStream_t stream);

// The per-frame figures of ws.info (reach of the near segments, far flag)
// from the boxes already in ws.boxes; ws.info must hold zeros.
// The per-frame figures of the footprint records; with `fold`, the same
// launch also folds the recording forward's motion-statistics partials.
struct TileFold;
hipError_t launch_frame_reach(const WarpShape &s, const BwdWorkspace &ws, const TileFold *fold,
                              hipStream_t stream);

hipError_t launch_zero_u32(uint32_t *p, int64_t count, hipStream_t stream);

hipError_t launch_forward(int dtype, const void *src, const float *mv, const WarpShape &s,
                          void *out, uint8_t *mask, uint32_t *count, hipStream_t stream);

// The forward, also recording the adjoint's footprint into ws (when the
// adjoint of this channel count reads it) and, when motion_stats is not NULL,
// the per-frame motion statistics [N][4] (partials in ws.stat_parts).
hipError_t launch_forward_record(int dtype, const void *src, const float *mv, const WarpShape &s,
                                 void *out, uint8_t *mask, uint32_t *count,
                                 const BwdWorkspace &ws, double *motion_stats,
                                 hipStream_t stream);

// grad_src / grad_mv may each be NULL (not requested). The workspace is used
// only when grad_src is requested.
hipError_t launch_backward(int dtype, const void *src, const float *mv, const WarpShape &s,
                           const void *grad_out, void *grad_src, float *grad_mv,
                           const BwdWorkspace &ws, hipStream_t stream);

// Per-frame mean and population variance of both motion components:
// stats[n][4] = (mean_x, var_x, mean_y, var_y) in float64.
size_t motion_stats_workspace_bytes(int n, int h, int w);
hipError_t launch_motion_stats(const float *mv, int n, int h, int w, double *stats,
                               void *workspace, hipStream_t stream);

// Size of the file-scope device scratch used by exw_motion_stats_no_alloc.
constexpr size_t kNoAllocScratchBytes = EXW_NO_ALLOC_SCRATCH_BYTES;

// That scratch's address on the current device (looked up once per device
// with hipGetSymbolAddress, then cached).
hipError_t no_alloc_scratch(void **ptr);

// Per-frame (MSE, PSNR, SSIM) of pred vs truth, both [B, C, H, W] in the
// storage dtype, H, W >= 11: quality[b][3] in float64.
size_t quality_workspace_bytes(int b, int c, int h, int w);
hipError_t launch_quality(int dtype, const void *pred, const void *truth, int b, int c, int h,
                          int w, double peak, double *quality, void *workspace,
                          hipStream_t stream);

// N_D: connected components of the marked pixels of stencil [N, H, W] (u8,
// marked = non-zero), 4- or 8-connectivity, into count [N]; the workspace
// holds one int32 label per pixel.
size_t dynamic_objects_workspace_bytes(int n, int h, int w);
hipError_t launch_dynamic_objects(const uint8_t *stencil, int n, int h, int w, int connectivity,
                                  uint32_t *count, void *workspace, hipStream_t stream);

// Per-frame, per-channel EMD between two buffers [N, C, H, W] (histograms of
// `bins` bins on [lo, hi]); emd[n][c] in float64.
size_t buffer_emd_workspace_bytes(int n, int c, int bins);
hipError_t launch_buffer_emd(int dtype, const void *cur, const void *prev, int n, int c, int h,
                             int w, double lo, double hi, int bins, double *emd, void *workspace,
                             hipStream_t stream);

// Plain HBM streams (kind 0 = copy src -> dst, 1 = read src, 2 = write dst),
// bytes a multiple of 16, 16-byte aligned pointers.
hipError_t launch_stream(int kind, const void *src, void *dst, int64_t bytes, float *sink,
                         hipStream_t stream);

}  // namespace exw
