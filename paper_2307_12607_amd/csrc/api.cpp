// C-ABI of libexwarp: argument validation, then dispatch to the HIP kernels.
// Every check runs before the first HIP call, so a rejected call touches
// neither the device nor the stream. See include/exwarp.h for the contract.
#include "exwarp.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "launch.h"

namespace {

thread_local std::string g_last_error;

exw_status fail(exw_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

exw_status succeed() {
    g_last_error.clear();
    return EXW_SUCCESS;
}

}  // namespace

namespace exw {

exw_status report(exw_status st, const char *msg) {
    if (st == EXW_SUCCESS) return succeed();
    return fail(st, "%s", msg);
}

}  // namespace exw

namespace {

size_t dtype_size(int dtype) {
    switch (dtype) {
    case EXW_F32: return 4;
    case EXW_F16: return 2;
    case EXW_BF16: return 2;
    default: return 0;
    }
}

struct Span {
    const char *name;
    uintptr_t lo, hi;  // [lo, hi)
};

Span span(const char *name, const void *p, uint64_t bytes) {
    const uintptr_t lo = reinterpret_cast<uintptr_t>(p);
    return Span{name, lo, p ? lo + bytes : lo};
}

bool overlaps(const Span &a, const Span &b) {
    return a.lo != a.hi && b.lo != b.hi && a.lo < b.hi && b.lo < a.hi;
}

// Largest element count of any buffer the library indexes: keeps every
// 64-bit offset far from overflow.
constexpr uint64_t kMaxElems = uint64_t(1) << 40;

struct Checked {
    exw::WarpShape shape;
    uint64_t hw = 0, img_elems = 0, out_elems = 0, mv_elems = 0;
    size_t esize = 0;
    bool empty = false;
};

exw_status check_common(exw_dtype dtype, int32_t n, int32_t c, int32_t h, int32_t w,
                        const float *phases, int32_t k, Checked *ck) {
    ck->esize = dtype_size(dtype);
    if (ck->esize == 0) return fail(EXW_ERROR_INVALID_VALUE, "unknown dtype %d", int(dtype));
    if (n < 0 || h < 0 || w < 0)
        return fail(EXW_ERROR_INVALID_VALUE, "negative size (n=%d, h=%d, w=%d)", n, h, w);
    if (c < 1) return fail(EXW_ERROR_INVALID_VALUE, "channel count %d < 1", c);
    if (c > EXW_MAX_CHANNELS)
        return fail(EXW_ERROR_UNSUPPORTED, "channel count %d > %d", c, EXW_MAX_CHANNELS);
    if (k < 1) return fail(EXW_ERROR_INVALID_VALUE, "phase count %d < 1", k);
    if (k > EXW_MAX_PHASES)
        return fail(EXW_ERROR_UNSUPPORTED, "phase count %d > %d", k, EXW_MAX_PHASES);
    if (!phases) return fail(EXW_ERROR_INVALID_VALUE, "phases is NULL");
    for (int j = 0; j < k; ++j)
        if (!std::isfinite(phases[j]))
            return fail(EXW_ERROR_INVALID_VALUE, "phase %d is not finite", j);
    // Frame coordinates must be exact in float32 and a plane index must fit int32.
    if (h >= (1 << 24) || w >= (1 << 24))
        return fail(EXW_ERROR_UNSUPPORTED, "frame side >= 2^24 (h=%d, w=%d)", h, w);
    // In-plane byte offsets are 32-bit in the kernels.
    ck->hw = uint64_t(h) * uint64_t(w);
    if (ck->hw > (uint64_t(1) << 30))
        return fail(EXW_ERROR_UNSUPPORTED, "h*w = %llu > 2^30", (unsigned long long)ck->hw);
    ck->img_elems = uint64_t(n) * uint64_t(c) * ck->hw;
    ck->out_elems = ck->img_elems * uint64_t(k);
    ck->mv_elems = uint64_t(n) * 2u * ck->hw;
    if (ck->out_elems > kMaxElems)
        return fail(EXW_ERROR_UNSUPPORTED, "batch too large (%llu output elements)",
                    (unsigned long long)ck->out_elems);
    // One workgroup per 64x4 tile must fit a 1-D grid.
    const uint64_t tiles = uint64_t(n) * ((uint64_t(w) + 63) / 64) * ((uint64_t(h) + 3) / 4);
    if (tiles >= (uint64_t(1) << 31))
        return fail(EXW_ERROR_UNSUPPORTED, "batch too large (%llu tiles)", (unsigned long long)tiles);
    // Twelve 16-bit channels run the forward with one workgroup per 128-pixel
    // row segment: that grid must fit as well.
    if (c == 12 && dtype != EXW_F32 && w >= 2) {
        const uint64_t segs = uint64_t(n) * ((uint64_t(w) + 127) / 128) * (((uint64_t(h) + 3) / 4) * 4);
        if (segs >= (uint64_t(1) << 31))
            return fail(EXW_ERROR_UNSUPPORTED, "batch too large (%llu row segments)",
                        (unsigned long long)segs);
    }
    ck->empty = (n == 0 || h == 0 || w == 0);
    ck->shape.n = n;
    ck->shape.c = c;
    ck->shape.h = h;
    ck->shape.w = w;
    ck->shape.k = k;
    for (int j = 0; j < 4; ++j) ck->shape.phases[j] = j < k ? phases[j] : 0.0f;
    return EXW_SUCCESS;
}

exw_status check_ptr(const char *name, const void *p, size_t align, bool required) {
    if (!p) {
        if (required) return fail(EXW_ERROR_INVALID_VALUE, "%s is NULL", name);
        return EXW_SUCCESS;
    }
    if (reinterpret_cast<uintptr_t>(p) % align != 0)
        return fail(EXW_ERROR_INVALID_VALUE, "%s is not %zu-byte aligned", name, align);
    return EXW_SUCCESS;
}

exw_status check_disjoint(const Span *outs, int n_out, const Span *ins, int n_in) {
    for (int i = 0; i < n_out; ++i) {
        for (int j = 0; j < n_in; ++j)
            if (overlaps(outs[i], ins[j]))
                return fail(EXW_ERROR_INVALID_VALUE, "%s overlaps input %s", outs[i].name,
                            ins[j].name);
        for (int j = i + 1; j < n_out; ++j)
            if (overlaps(outs[i], outs[j]))
                return fail(EXW_ERROR_INVALID_VALUE, "%s overlaps output %s", outs[i].name,
                            outs[j].name);
    }
    return EXW_SUCCESS;
}

exw_status launched(hipError_t e, const char *what) {
    if (e != hipSuccess)
        return fail(EXW_ERROR_LAUNCH, "%s: %s", what, hipGetErrorString(e));
    return succeed();
}

// Byte offsets of the adjoint's scratch inside the caller's workspace.
struct WsLayout {
    size_t boxes, info, stats, accum, total;
};

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

WsLayout workspace_layout(int dtype, int n, int c, int h, int w) {
    WsLayout l;
    l.boxes = 0;
    l.info = align_up(exw::backward_box_bytes(n, h, w));
    l.stats = align_up(l.info + exw::backward_info_bytes(n));
    l.accum = align_up(l.stats + exw::record_stats_bytes(n, h, w));
    const size_t accum_bytes =
        dtype == EXW_F32 ? 0 : size_t(n) * size_t(c) * size_t(h) * size_t(w) * sizeof(float);
    l.total = l.accum + accum_bytes;
    return l;
}

#define EXW_TRY(expr)                                  \
    do {                                               \
        exw_status st_ = (expr);                       \
        if (st_ != EXW_SUCCESS) return st_;            \
    } while (0)

// The forward; with `record`, it also leaves the adjoint's footprint of this
// motion and these phases in the caller's adjoint workspace.
exw_status forward_impl(const void *src, exw_dtype dtype, int32_t n, int32_t c, int32_t h,
                        int32_t w, const float *mv, const float *phases, int32_t k, void *out,
                        uint8_t *mask, uint32_t *invalid_count, double *motion_stats,
                        void *workspace, size_t workspace_bytes, bool record, void *stream) {
    Checked ck;
    EXW_TRY(check_common(dtype, n, c, h, w, phases, k, &ck));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint64_t nk = uint64_t(n) * uint64_t(k);
    EXW_TRY(check_ptr("invalid_count", invalid_count, 4, false));
    EXW_TRY(check_ptr("motion_stats", motion_stats, 8, false));
    if (motion_stats && n > 0 && (h == 0 || w == 0))
        return fail(EXW_ERROR_INVALID_VALUE,
                    "motion_stats of empty frames has no variance (h=%d, w=%d)", h, w);
    if (ck.empty) {
        if (invalid_count && nk > 0)
            return launched(exw::launch_zero_u32(invalid_count, int64_t(nk), st), "zero count");
        return succeed();
    }
    EXW_TRY(check_ptr("src", src, ck.esize, true));
    EXW_TRY(check_ptr("mv", mv, 4, true));
    EXW_TRY(check_ptr("out", out, ck.esize, true));
    EXW_TRY(check_ptr("mask", mask, 1, false));
    const WsLayout lay = workspace_layout(dtype, n, c, h, w);
    const uint64_t ws_need = record ? lay.total : 0;
    if (record) {
        EXW_TRY(check_ptr("workspace", workspace, 256, true));
        if (workspace_bytes < ws_need)
            return fail(EXW_ERROR_INVALID_VALUE, "workspace has %zu bytes, needs %llu",
                        workspace_bytes, (unsigned long long)ws_need);
    }
    const Span ins[] = {span("src", src, ck.img_elems * ck.esize),
                        span("mv", mv, ck.mv_elems * 4)};
    const Span outs[] = {span("out", out, ck.out_elems * ck.esize),
                         span("mask", mask, nk * ck.hw),
                         span("invalid_count", invalid_count, nk * 4),
                         span("workspace", record ? workspace : nullptr, ws_need),
                         span("motion_stats", motion_stats, uint64_t(n) * 4u * 8u)};
    EXW_TRY(check_disjoint(outs, 5, ins, 2));
    if (!record)
        return launched(exw::launch_forward(dtype, src, mv, ck.shape, out, mask, invalid_count, st),
                        "warp forward launch");
    char *base = static_cast<char *>(workspace);
    const exw::BwdWorkspace ws{base + lay.boxes, base + lay.info, nullptr, false,
                               base + lay.stats};
    return launched(exw::launch_forward_record(dtype, src, mv, ck.shape, out, mask, invalid_count,
                                               ws, motion_stats, st),
                    "warp forward launch");
}

// The adjoint; with `recorded`, the footprint in the workspace is taken as
// left there by the recording forward of the same motion and phases.
exw_status backward_impl(const void *src, exw_dtype dtype, int32_t n, int32_t c, int32_t h,
                         int32_t w, const float *mv, const float *phases, int32_t k,
                         const void *grad_out, void *grad_src, float *grad_mv, void *workspace,
                         size_t workspace_bytes, bool recorded, void *stream) {
    Checked ck;
    EXW_TRY(check_common(dtype, n, c, h, w, phases, k, &ck));
    if (ck.empty || (!grad_src && !grad_mv)) return succeed();
    EXW_TRY(check_ptr("src", src, ck.esize, grad_mv != nullptr));
    EXW_TRY(check_ptr("mv", mv, 4, true));
    EXW_TRY(check_ptr("grad_out", grad_out, ck.esize, true));
    EXW_TRY(check_ptr("grad_src", grad_src, ck.esize, false));
    EXW_TRY(check_ptr("grad_mv", grad_mv, 4, false));
    const bool needs_ws = grad_src != nullptr;
    const WsLayout lay = workspace_layout(dtype, n, c, h, w);
    const uint64_t ws_need = needs_ws ? lay.total : 0;
    if (needs_ws) {
        EXW_TRY(check_ptr("workspace", workspace, 256, true));
        if (workspace_bytes < ws_need)
            return fail(EXW_ERROR_INVALID_VALUE, "workspace has %zu bytes, needs %llu",
                        workspace_bytes, (unsigned long long)ws_need);
    }
    const Span ins[] = {span("src", src, ck.img_elems * ck.esize),
                        span("mv", mv, ck.mv_elems * 4),
                        span("grad_out", grad_out, ck.out_elems * ck.esize)};
    const Span outs[] = {span("grad_src", grad_src, ck.img_elems * ck.esize),
                         span("grad_mv", grad_mv, ck.mv_elems * 4),
                         span("workspace", needs_ws ? workspace : nullptr, ws_need)};
    EXW_TRY(check_disjoint(outs, 3, ins, 3));
    exw::BwdWorkspace ws{nullptr, nullptr, nullptr, recorded, nullptr};
    if (needs_ws) {
        char *base = static_cast<char *>(workspace);
        ws.boxes = base + lay.boxes;
        ws.info = base + lay.info;
        ws.accum32 = dtype == EXW_F32 ? nullptr : reinterpret_cast<float *>(base + lay.accum);
    }
    return launched(exw::launch_backward(dtype, grad_mv ? src : nullptr, mv, ck.shape, grad_out,
                                         grad_src, grad_mv, ws,
                                         static_cast<hipStream_t>(stream)),
                    "warp backward launch");
}

exw_status motion_stats_impl(const float *mv, int32_t n, int32_t h, int32_t w, double *stats,
                             void *workspace, size_t workspace_bytes, bool no_alloc,
                             void *stream);

}  // namespace

extern "C" {

int exw_abi_version(void) { return EXW_ABI_VERSION; }

const char *exw_status_string(int status) {
    switch (status) {
    case EXW_SUCCESS: return "EXW_SUCCESS";
    case EXW_ERROR_INVALID_VALUE: return "EXW_ERROR_INVALID_VALUE";
    case EXW_ERROR_UNSUPPORTED: return "EXW_ERROR_UNSUPPORTED";
    case EXW_ERROR_LAUNCH: return "EXW_ERROR_LAUNCH";
    default: return "EXW_UNKNOWN_STATUS";
    }
}

const char *exw_last_error(void) { return g_last_error.c_str(); }

exw_status exw_warp_forward_batched(const void *src, exw_dtype dtype, int32_t n, int32_t c,
                                    int32_t h, int32_t w, const float *mv, const float *phases,
                                    int32_t k, void *out, uint8_t *mask,
                                    uint32_t *invalid_count, void *stream) {
    return forward_impl(src, dtype, n, c, h, w, mv, phases, k, out, mask, invalid_count, nullptr,
                        nullptr, 0, false, stream);
}

exw_status exw_warp_forward_batched_record(const void *src, exw_dtype dtype, int32_t n, int32_t c,
                                           int32_t h, int32_t w, const float *mv,
                                           const float *phases, int32_t k, void *out,
                                           uint8_t *mask, uint32_t *invalid_count,
                                           double *motion_stats, void *workspace,
                                           size_t workspace_bytes, void *stream) {
    return forward_impl(src, dtype, n, c, h, w, mv, phases, k, out, mask, invalid_count,
                        motion_stats, workspace, workspace_bytes, true, stream);
}

exw_status exw_warp_forward(const void *src, exw_dtype dtype, int32_t c, int32_t h, int32_t w,
                            const float *mv, float phase, void *out, uint8_t *mask,
                            void *stream) {
    return exw_warp_forward_batched(src, dtype, 1, c, h, w, mv, &phase, 1, out, mask, nullptr,
                                    stream);
}

size_t exw_warp_backward_workspace_bytes(exw_dtype dtype, int32_t n, int32_t c, int32_t h,
                                         int32_t w) {
    if (dtype_size(dtype) == 0 || n <= 0 || c <= 0 || h <= 0 || w <= 0) return 0;
    return workspace_layout(dtype, n, c, h, w).total;
}

exw_status exw_warp_backward_batched(const void *src, exw_dtype dtype, int32_t n, int32_t c,
                                     int32_t h, int32_t w, const float *mv, const float *phases,
                                     int32_t k, const void *grad_out, void *grad_src,
                                     float *grad_mv, void *workspace, size_t workspace_bytes,
                                     void *stream) {
    return backward_impl(src, dtype, n, c, h, w, mv, phases, k, grad_out, grad_src, grad_mv,
                         workspace, workspace_bytes, false, stream);
}

exw_status exw_warp_backward_batched_recorded(const void *src, exw_dtype dtype, int32_t n,
                                              int32_t c, int32_t h, int32_t w, const float *mv,
                                              const float *phases, int32_t k,
                                              const void *grad_out, void *grad_src,
                                              float *grad_mv, void *workspace,
                                              size_t workspace_bytes, void *stream) {
    return backward_impl(src, dtype, n, c, h, w, mv, phases, k, grad_out, grad_src, grad_mv,
                         workspace, workspace_bytes, true, stream);
}

exw_status exw_warp_backward(const void *src, exw_dtype dtype, int32_t c, int32_t h, int32_t w,
                             const float *mv, float phase, const void *grad_out, void *grad_src,
                             float *grad_mv, void *workspace, size_t workspace_bytes,
                             void *stream) {
    return exw_warp_backward_batched(src, dtype, 1, c, h, w, mv, &phase, 1, grad_out, grad_src,
                                     grad_mv, workspace, workspace_bytes, stream);
}

size_t exw_motion_stats_workspace_bytes(int32_t n, int32_t h, int32_t w) {
    if (n <= 0 || h <= 0 || w <= 0) return 0;
    return exw::motion_stats_workspace_bytes(n, h, w);
}

exw_status exw_motion_stats(const float *mv, int32_t n, int32_t h, int32_t w, double *stats,
                            void *workspace, size_t workspace_bytes, void *stream) {
    return motion_stats_impl(mv, n, h, w, stats, workspace, workspace_bytes, false, stream);
}

exw_status exw_motion_stats_no_alloc(const float *mv, int32_t n, int32_t h, int32_t w,
                                     double *stats, void *stream) {
    return motion_stats_impl(mv, n, h, w, stats, nullptr, 0, true, stream);
}

}  // extern "C"

namespace {

exw_status motion_stats_impl(const float *mv, int32_t n, int32_t h, int32_t w, double *stats,
                             void *workspace, size_t workspace_bytes, bool no_alloc,
                             void *stream) {
    if (n < 0 || h < 0 || w < 0)
        return fail(EXW_ERROR_INVALID_VALUE, "negative size (n=%d, h=%d, w=%d)", n, h, w);
    if (n > 0 && (h == 0 || w == 0))
        return fail(EXW_ERROR_INVALID_VALUE, "empty frames have no statistics (h=%d, w=%d)", h,
                    w);
    if (n == 0) return succeed();
    if (h >= (1 << 24) || w >= (1 << 24))
        return fail(EXW_ERROR_UNSUPPORTED, "frame side >= 2^24 (h=%d, w=%d)", h, w);
    const uint64_t hw = uint64_t(h) * uint64_t(w);
    if (hw > (uint64_t(1) << 30))
        return fail(EXW_ERROR_UNSUPPORTED, "h*w = %llu > 2^30", (unsigned long long)hw);
    // the first pass runs at most 256 workgroups per frame in a 1-D grid
    if (n >= (1 << 21)) return fail(EXW_ERROR_UNSUPPORTED, "frame count %d >= 2^21", n);
    EXW_TRY(check_ptr("mv", mv, 4, true));
    EXW_TRY(check_ptr("stats", stats, 8, true));
    const size_t ws_need = exw::motion_stats_workspace_bytes(n, h, w);
    if (no_alloc) {
        if (ws_need > exw::kNoAllocScratchBytes)
            return fail(EXW_ERROR_UNSUPPORTED,
                        "batch needs %zu bytes of partials, more than the %zu-byte static "
                        "scratch of exw_motion_stats_no_alloc (use exw_motion_stats)",
                        ws_need, exw::kNoAllocScratchBytes);
    } else {
        EXW_TRY(check_ptr("workspace", workspace, 256, true));
        if (workspace_bytes < ws_need)
            return fail(EXW_ERROR_INVALID_VALUE, "workspace has %zu bytes, needs %zu",
                        workspace_bytes, ws_need);
    }
    const Span ins[] = {span("mv", mv, uint64_t(n) * 2u * hw * 4u)};
    const Span outs[] = {span("stats", stats, uint64_t(n) * 4u * 8u),
                         span("workspace", no_alloc ? nullptr : workspace, ws_need)};
    EXW_TRY(check_disjoint(outs, 2, ins, 1));
    if (no_alloc) {
        void *scratch = nullptr;
        const hipError_t e = exw::no_alloc_scratch(&scratch);
        if (e != hipSuccess) return launched(e, "static scratch lookup");
        workspace = scratch;
    }
    return launched(exw::launch_motion_stats(mv, n, h, w, stats, workspace,
                                             static_cast<hipStream_t>(stream)),
                    "motion statistics launch");
}

}  // namespace

extern "C" {

size_t exw_frame_quality_workspace_bytes(int32_t b, int32_t c, int32_t h, int32_t w) {
    if (b <= 0 || c <= 0 || h < 11 || w < 11) return 0;
    return exw::quality_workspace_bytes(b, c, h, w);
}

exw_status exw_frame_quality(const void *pred, const void *truth, exw_dtype dtype, int32_t b,
                             int32_t c, int32_t h, int32_t w, double peak, double *quality,
                             void *workspace, size_t workspace_bytes, void *stream) {
    const size_t esize = dtype_size(dtype);
    if (esize == 0) return fail(EXW_ERROR_INVALID_VALUE, "unknown dtype %d", int(dtype));
    if (b < 0 || c < 0 || h < 0 || w < 0)
        return fail(EXW_ERROR_INVALID_VALUE, "negative size (b=%d, c=%d, h=%d, w=%d)", b, c, h, w);
    if (!(std::isfinite(peak) && peak > 0.0))
        return fail(EXW_ERROR_INVALID_VALUE, "peak must be finite and > 0");
    if (b == 0) return succeed();
    if (c < 1) return fail(EXW_ERROR_INVALID_VALUE, "channel count %d < 1", c);
    if (h < 11 || w < 11)
        return fail(EXW_ERROR_INVALID_VALUE,
                    "frames smaller than the 11x11 SSIM window (h=%d, w=%d)", h, w);
    if (h >= (1 << 24) || w >= (1 << 24))
        return fail(EXW_ERROR_UNSUPPORTED, "frame side >= 2^24 (h=%d, w=%d)", h, w);
    const uint64_t hw = uint64_t(h) * uint64_t(w);
    const uint64_t elems = uint64_t(b) * uint64_t(c) * hw;
    if (elems > kMaxElems)
        return fail(EXW_ERROR_UNSUPPORTED, "batch too large (%llu elements)",
                    (unsigned long long)elems);
    const uint64_t strips = uint64_t(b) * uint64_t(c) * ((uint64_t(w) - 10 + 63) / 64) *
                            ((uint64_t(h) - 10 + 65) / 66);
    if (strips >= (uint64_t(1) << 31))
        return fail(EXW_ERROR_UNSUPPORTED, "batch too large (%llu strips)",
                    (unsigned long long)strips);
    EXW_TRY(check_ptr("pred", pred, esize, true));
    EXW_TRY(check_ptr("truth", truth, esize, true));
    EXW_TRY(check_ptr("quality", quality, 8, true));
    EXW_TRY(check_ptr("workspace", workspace, 256, true));
    const size_t ws_need = exw::quality_workspace_bytes(b, c, h, w);
    if (workspace_bytes < ws_need)
        return fail(EXW_ERROR_INVALID_VALUE, "workspace has %zu bytes, needs %zu",
                    workspace_bytes, ws_need);
    const Span ins[] = {span("pred", pred, elems * esize), span("truth", truth, elems * esize)};
    const Span outs[] = {span("quality", quality, uint64_t(b) * 3u * 8u),
                         span("workspace", workspace, ws_need)};
    EXW_TRY(check_disjoint(outs, 2, ins, 2));
    return launched(exw::launch_quality(dtype, pred, truth, b, c, h, w, peak, quality, workspace,
                                        static_cast<hipStream_t>(stream)),
                    "frame quality launch");
}

size_t exw_buffer_emd_workspace_bytes(int32_t n, int32_t c, int32_t bins) {
    if (n <= 0 || c <= 0 || bins < 1 || bins > EXW_EMD_MAX_BINS) return 0;
    return exw::buffer_emd_workspace_bytes(n, c, bins);
}

exw_status exw_buffer_emd(const void *cur, const void *prev, exw_dtype dtype, int32_t n,
                          int32_t c, int32_t h, int32_t w, double lo, double hi, int32_t bins,
                          double *emd, void *workspace, size_t workspace_bytes, void *stream) {
    const size_t esize = dtype_size(dtype);
    if (esize == 0) return fail(EXW_ERROR_INVALID_VALUE, "unknown dtype %d", int(dtype));
    if (n < 0 || h < 0 || w < 0)
        return fail(EXW_ERROR_INVALID_VALUE, "negative size (n=%d, h=%d, w=%d)", n, h, w);
    if (c < 1) return fail(EXW_ERROR_INVALID_VALUE, "channel count %d < 1", c);
    if (c > EXW_MAX_CHANNELS)
        return fail(EXW_ERROR_UNSUPPORTED, "channel count %d > %d", c, EXW_MAX_CHANNELS);
    if (!(std::isfinite(lo) && std::isfinite(hi) && lo < hi))
        return fail(EXW_ERROR_INVALID_VALUE, "the bin range needs finite lo < hi");
    if (bins < 1 || bins > EXW_EMD_MAX_BINS)
        return fail(EXW_ERROR_INVALID_VALUE, "bins %d outside 1..%d", bins, EXW_EMD_MAX_BINS);
    if (!std::isfinite(double(bins) / (hi - lo)))
        return fail(EXW_ERROR_INVALID_VALUE, "bin range too narrow for %d bins", bins);
    if (n > 0 && (h == 0 || w == 0))
        return fail(EXW_ERROR_INVALID_VALUE, "empty frames have no distribution (h=%d, w=%d)",
                    h, w);
    if (n == 0) return succeed();
    const uint64_t hw = uint64_t(h) * uint64_t(w);
    if (hw > (uint64_t(1) << 30))
        return fail(EXW_ERROR_UNSUPPORTED, "h*w = %llu > 2^30", (unsigned long long)hw);
    const uint64_t elems = uint64_t(n) * uint64_t(c) * hw;
    if (elems > kMaxElems)
        return fail(EXW_ERROR_UNSUPPORTED, "batch too large (%llu elements)",
                    (unsigned long long)elems);
    // at most 128 workgroups per plane in a 1-D grid
    if (uint64_t(n) * uint64_t(c) * 128u >= (uint64_t(1) << 31))
        return fail(EXW_ERROR_UNSUPPORTED, "too many planes (%llu)",
                    (unsigned long long)(uint64_t(n) * uint64_t(c)));
    EXW_TRY(check_ptr("cur", cur, esize, true));
    EXW_TRY(check_ptr("prev", prev, esize, true));
    EXW_TRY(check_ptr("emd", emd, 8, true));
    EXW_TRY(check_ptr("workspace", workspace, 256, true));
    const size_t ws_need = exw::buffer_emd_workspace_bytes(n, c, bins);
    if (workspace_bytes < ws_need)
        return fail(EXW_ERROR_INVALID_VALUE, "workspace has %zu bytes, needs %zu",
                    workspace_bytes, ws_need);
    const Span ins[] = {span("cur", cur, elems * esize), span("prev", prev, elems * esize)};
    const Span outs[] = {span("emd", emd, uint64_t(n) * uint64_t(c) * 8u),
                         span("workspace", workspace, ws_need)};
    EXW_TRY(check_disjoint(outs, 2, ins, 2));
    return launched(exw::launch_buffer_emd(dtype, cur, prev, n, c, h, w, lo, hi, bins, emd,
                                           workspace, static_cast<hipStream_t>(stream)),
                    "buffer EMD launch");
}

size_t exw_dynamic_objects_workspace_bytes(int32_t n, int32_t h, int32_t w) {
    if (n <= 0 || h <= 0 || w <= 0) return 0;
    return exw::dynamic_objects_workspace_bytes(n, h, w);
}

exw_status exw_dynamic_objects(const uint8_t *stencil, int32_t n, int32_t h, int32_t w,
                               int32_t connectivity, uint32_t *count, void *workspace,
                               size_t workspace_bytes, void *stream) {
    if (n < 0 || h < 0 || w < 0)
        return fail(EXW_ERROR_INVALID_VALUE, "negative size (n=%d, h=%d, w=%d)", n, h, w);
    if (connectivity != 4 && connectivity != 8)
        return fail(EXW_ERROR_INVALID_VALUE, "connectivity %d is not 4 or 8", connectivity);
    if (n == 0) return succeed();
    const uint64_t hw = uint64_t(h) * uint64_t(w);
    if (hw > (uint64_t(1) << 30))
        return fail(EXW_ERROR_UNSUPPORTED, "h*w = %llu > 2^30", (unsigned long long)hw);
    const uint64_t px = uint64_t(n) * hw;
    if (px > kMaxElems)
        return fail(EXW_ERROR_UNSUPPORTED, "batch too large (%llu pixels)",
                    (unsigned long long)px);
    EXW_TRY(check_ptr("count", count, 4, true));
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (hw == 0)  // no pixels, no objects
        return launched(exw::launch_zero_u32(count, n, st), "dynamic objects launch");
    const uint64_t tiles = uint64_t(n) * ((uint64_t(w) + 31) / 32) * ((uint64_t(h) + 31) / 32);
    if (tiles >= (uint64_t(1) << 31))
        return fail(EXW_ERROR_UNSUPPORTED, "too many 32 x 32 tiles (%llu)",
                    (unsigned long long)tiles);
    EXW_TRY(check_ptr("stencil", stencil, 1, true));
    EXW_TRY(check_ptr("workspace", workspace, 256, true));
    const size_t ws_need = exw::dynamic_objects_workspace_bytes(n, h, w);
    if (workspace_bytes < ws_need)
        return fail(EXW_ERROR_INVALID_VALUE, "workspace has %zu bytes, needs %zu",
                    workspace_bytes, ws_need);
    const Span ins[] = {span("stencil", stencil, px)};
    const Span outs[] = {span("count", count, uint64_t(n) * 4u),
                         span("workspace", workspace, ws_need)};
    EXW_TRY(check_disjoint(outs, 2, ins, 1));
    return launched(exw::launch_dynamic_objects(stencil, n, h, w, connectivity, count, workspace,
                                                st),
                    "dynamic objects launch");
}

exw_status exw_warp_chain(const void *src, exw_dtype dtype, int32_t n, int32_t c, int32_t h,
                          int32_t w, const float *mv, float phase, int32_t steps, void *out,
                          uint8_t *mask, uint32_t *invalid_count, void *stream) {
    if (steps < 1) return fail(EXW_ERROR_INVALID_VALUE, "steps %d < 1", steps);
    Checked ck;
    EXW_TRY(check_common(dtype, n, c, h, w, &phase, 1, &ck));
    const uint64_t step_out = ck.img_elems;  // one step: [N, C, H, W]
    if (step_out * uint64_t(steps) > kMaxElems)
        return fail(EXW_ERROR_UNSUPPORTED, "chain too large (%llu output elements)",
                    (unsigned long long)(step_out * uint64_t(steps)));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint64_t ns = uint64_t(n) * uint64_t(steps);
    EXW_TRY(check_ptr("invalid_count", invalid_count, 4, false));
    if (ck.empty) {
        if (invalid_count && ns > 0)
            return launched(exw::launch_zero_u32(invalid_count, int64_t(ns), st), "zero count");
        return succeed();
    }
    EXW_TRY(check_ptr("src", src, ck.esize, true));
    EXW_TRY(check_ptr("mv", mv, 4, true));
    EXW_TRY(check_ptr("out", out, ck.esize, true));
    EXW_TRY(check_ptr("mask", mask, 1, false));
    const Span ins[] = {span("src", src, ck.img_elems * ck.esize),
                        span("mv", mv, ck.mv_elems * 4)};
    const Span outs[] = {span("out", out, step_out * uint64_t(steps) * ck.esize),
                         span("mask", mask, ns * ck.hw),
                         span("invalid_count", invalid_count, ns * 4)};
    EXW_TRY(check_disjoint(outs, 3, ins, 2));
    char *o = static_cast<char *>(out);
    for (int i = 0; i < steps; ++i) {
        const void *in = i == 0 ? src : o + (i - 1) * step_out * ck.esize;
        hipError_t e = exw::launch_forward(
            dtype, in, mv, ck.shape, o + i * step_out * ck.esize,
            mask ? mask + uint64_t(i) * n * ck.hw : nullptr,
            invalid_count ? invalid_count + uint64_t(i) * n : nullptr, st);
        if (e != hipSuccess) return launched(e, "chained warp launch");
    }
    return succeed();
}

namespace {

exw_status stream_impl(int kind, const void *src, void *dst, size_t bytes, float *sink,
                       void *stream) {
    if (bytes % 16 != 0)
        return fail(EXW_ERROR_INVALID_VALUE, "bytes %zu is not a multiple of 16", bytes);
    if (bytes == 0) return succeed();
    if (kind != 2) EXW_TRY(check_ptr("src", src, 16, true));
    if (kind != 1) EXW_TRY(check_ptr("dst", dst, 16, true));
    if (kind == 1) EXW_TRY(check_ptr("sink", sink, 4, true));
    if (kind == 0) {
        const Span ins[] = {span("src", src, bytes)};
        const Span outs[] = {span("dst", dst, bytes)};
        EXW_TRY(check_disjoint(outs, 1, ins, 1));
    }
    return launched(exw::launch_stream(kind, src, dst, static_cast<int64_t>(bytes), sink,
                                       static_cast<hipStream_t>(stream)),
                    "stream launch");
}

}  // namespace

exw_status exw_stream_copy(const void *src, void *dst, size_t bytes, void *stream) {
    return stream_impl(0, src, dst, bytes, nullptr, stream);
}

exw_status exw_stream_read(const void *src, size_t bytes, float *sink, void *stream) {
    return stream_impl(1, src, nullptr, bytes, sink, stream);
}

exw_status exw_stream_write(void *dst, size_t bytes, void *stream) {
    return stream_impl(2, nullptr, dst, bytes, nullptr, stream);
}

}  // extern "C"
