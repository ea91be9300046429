// Adjoint of the motion-vector warp for CDNA4 (gfx950): gradients with
// respect to the source frames (transpose of the bilinear gather) and to the
// motion vectors (derivative of the bilinear blend), summed over phases.
//
// The image gradient is a scatter: each valid output pixel sends weight * g
// to its four taps. Float atomics on MI355X top out near 0.3 G lane-ops per
// ns even fully coalesced, and each one is a write to memory, so the scatter
// is turned into a gather instead:
//
//   pass 1 (footprint): for every 64-pixel row segment of the output, the
//     bounding box of all its taps over all phases, its integer tap offsets
//     when every lane shares them ("uniform" segments: rigid motion), plus
//     the per-frame largest distance between a segment and its box (one
//     wavefront per 16 rows of a 64-pixel column; reads the motion once).
//     In a training step the recording forward has already written these
//     records (footprint.h; the per-frame figures by frame_reach_kernel)
//     and this pass is skipped.
//   pass 2 (tiles): one wavefront owns a 128 x TH tile of the image gradient
//     in LDS. It walks the segments whose boxes reach the tile (only those
//     within the per-frame distance can), recomputes their taps, accumulates
//     weight * g for the taps inside the tile, and stores the finished tile
//     with plain coalesced stores: no global atomics, no zero fill. The tile
//     that contains a segment ("home") also computes that segment's motion
//     gradient, so every pixel's motion gradient is written exactly once.
//   pass 3 (far): segments whose box lies more than kFar pixels away are left
//     to a fallback that scatters with global atomics (frames without such
//     segments cost one check). For 16-bit storage such frames accumulate in a
//     float32 workspace and pass 4 rounds it into the output.
#include "footprint.h"
#include "launch.h"
#include "moments.h"
#include "warp_common.h"

namespace exw {
namespace {

constexpr int kTileW = 128;      // width of an image-gradient tile (pass 2)
constexpr int kThreads = 256;    // four wavefronts
constexpr int kFarBlocks = 1024; // grid of the fallback and cast passes

template <typename T>
struct BwdArgs {
    const T *src;
    const float *mv;
    const T *gout;
    T *gsrc;          // image gradient in the storage type, or NULL
    float *gmv;       // motion gradient, or NULL
    float *accum32;   // float32 accumulator for 16-bit frames with far segments
    Box *boxes;       // [N][H][segs]
    SegOffsets *offs; // [N][H][segs]
    FrameInfo *info;  // [N]
    int n, c, h, w, k;
    int segs;         // segments per row
    int tile_h, tiles_x, tiles_y;
    int frame_32bit;  // C * H * W * sizeof(T) < 2^32: frame-relative 32-bit offsets
    float s[4];
};

// ---------------------------------------------------------------- pass 1

// Rows handled by one wavefront of the footprint pass: 16 keeps 32 motion
// loads in flight per wavefront and amortises its scalar index work and its
// frame-info update (measured 84 us vs 110 us with 4 rows on workload 2; the
// standalone adjoint with 8 or 32 rows: 3-7 % slower on workload 2, 32 rows
// 2 % faster on workload 5).
constexpr int kFootRows = 16;

// One wavefront covers kFootRows rows of one 64-pixel column strip: all motion
// loads are issued first, then the per-row boxes are reduced across lanes.
template <int KT>
__global__ __launch_bounds__(kThreads) void footprint_kernel(const float *mv, Box *boxes,
                                                             SegOffsets *offs, FrameInfo *info,
                                                             int n, int h, int w, int segs,
                                                             Phases4 ph) {
    // The wavefront's unit index is made scalar so that its decoding runs on
    // the scalar unit; the unit count (one per 16 rows x 64 columns) is below
    // 2^31 (the C ABI bounds the count of 4 x 64 tiles of the same frames).
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kSegW);
    const int lane = threadIdx.x % kSegW;
    const int row_groups = (h + kFootRows - 1) / kFootRows;
    const int unit = static_cast<int>(blockIdx.x) * (kThreads / kSegW) + wave;
    if (unit >= n * row_groups * segs) return;  // whole wavefront leaves together
    const int sc = unit % segs;
    const int rg = unit / segs;
    const int y0 = (rg % row_groups) * kFootRows;
    const int in = rg / row_groups;
    const int sx0 = sc * kSegW;
    const int x = sx0 + lane;
    const int64_t hw = static_cast<int64_t>(h) * w;
    const float *mu = mv + (2 * static_cast<int64_t>(in)) * hw;
    const float *mvv = mu + hw;

    float u[kFootRows], v[kFootRows];
#pragma unroll
    for (int r = 0; r < kFootRows; ++r) {
        const bool in_r = x < w && y0 + r < h;
        const uint32_t p = static_cast<uint32_t>(y0 + r) * static_cast<uint32_t>(w) + x;
        u[r] = in_r ? *at(mu, p) : 0.0f;
        v[r] = in_r ? *at(mvv, p) : 0.0f;
    }
    // Row r's box and offsets are collected in lane r, which stores them.
    // A uniform row (every lane valid, one offset per phase) takes its box
    // from the offsets on the scalar unit; other rows reduce it across lanes.
    Box mine{1, 0, 1, 0};
    uint32_t rec[KT];
#pragma unroll
    for (int j = 0; j < KT; ++j) rec[j] = 0;
    int reach_max = -1, far = 0;  // wave-uniform
#pragma unroll
    for (int r = 0; r < kFootRows; ++r) {
        const int y = y0 + r;
        int b[4];
        uint32_t rr[KT];
        segment_footprint<KT>(u[r], v[r], x, y, sx0, w, h, x < w && y < h, ph.s, b, rr);
        note_reach(b, sx0, y, reach_max, far);
        if (lane == r) {
            mine = Box{b[0], b[1], b[2], b[3]};
#pragma unroll
            for (int j = 0; j < KT; ++j) rec[j] = rr[j];
        }
    }
    if (lane < kFootRows && y0 + lane < h) {
        const int64_t at_seg = (static_cast<int64_t>(in) * h + y0 + lane) * segs + sc;
        boxes[at_seg] = mine;
        SegOffsets o{{0u, 0u, 0u, 0u}};
#pragma unroll
        for (int j = 0; j < KT; ++j) o.k[j] = rec[j];
        offs[at_seg] = o;
    }
    if (lane == 0) publish_reach(&info[in], reach_max, far);
}

// Per-frame figures from recorded boxes: what the footprint pass accumulates
// as it goes, for boxes the forward recorded. Each frame gets
// blocks_per_frame consecutive blocks of a 1-D grid (frames can outnumber the
// 65535 blocks a second grid dimension allows); a block takes
// kReachPerThread segments per thread, all loads in flight at once, reduces
// through LDS and updates the frame once (updates of one address serialise:
// few of them, and no wavefront waits on more than one).
constexpr int kReachPerThread = 4;

// Workgroups past the reduction's (n * blocks_per_frame) fold the recording
// forward's motion-statistics partials.
static_assert(kThreads == kTileFoldThreads, "the statistics fold runs in these workgroups");
__global__ __launch_bounds__(kThreads) void frame_reach_kernel(const Box *boxes, FrameInfo *info,
                                                               int h, int segs,
                                                               int blocks_per_frame,
                                                               int reach_blocks, TileFold fold) {
    if (static_cast<int>(blockIdx.x) >= reach_blocks) {  // workgroup-uniform
        fold_tile_share(fold, static_cast<int>(blockIdx.x) - reach_blocks);
        return;
    }
    __shared__ int red[2][kThreads / kSegW];
    const int in = static_cast<int>(blockIdx.x) / blocks_per_frame;
    const int part = static_cast<int>(blockIdx.x) - in * blocks_per_frame;
    const int per_frame = h * segs;  // below 2^31: the C ABI bounds H * W
    const Box *fb = boxes + static_cast<int64_t>(in) * per_frame;
    const int i0 = part * (kThreads * kReachPerThread) + threadIdx.x;
    Box bx[kReachPerThread];
#pragma unroll
    for (int j = 0; j < kReachPerThread; ++j) {
        const int i = i0 + j * kThreads;
        bx[j] = i < per_frame ? fb[i] : Box{1, 0, 1, 0};
    }
    int reach_max = -1, far = 0;
#pragma unroll
    for (int j = 0; j < kReachPerThread; ++j) {
        const int i = i0 + j * kThreads;
        const int row = i / segs;
        const int b[4] = {bx[j].x_lo, bx[j].x_hi, bx[j].y_lo, bx[j].y_hi};
        note_reach(b, (i - row * segs) * kSegW, row, reach_max, far);
    }
    reach_max = wave_max(reach_max);
    far = wave_max(far);
    const int wave = threadIdx.x / kSegW;
    if (threadIdx.x % kSegW == 0) { red[0][wave] = reach_max; red[1][wave] = far; }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 1; q < kThreads / kSegW; ++q) {
            reach_max = max(reach_max, red[0][q]);
            far = max(far, red[1][q]);
        }
        publish_reach(info + in, reach_max, far);
    }
}

// ---------------------------------------------------------------- pass 2

// Per-pixel taps of one phase.
struct PTaps {
    Axis ax, ay;
    bool valid;
};

template <typename T, int CT>
__device__ __forceinline__ void motion_grad_phase(const T *const *iplane, int w, const PTaps &t,
                                                  const float *g, float s, float &gu, float &gv) {
    const int xl = min(t.ax.i0, w - 2);
    const bool last = t.ax.i0 == w - 1;
    const uint32_t o0 = static_cast<uint32_t>(t.ay.i0) * static_cast<uint32_t>(w) + xl;
    const uint32_t o1 = static_cast<uint32_t>(t.ay.i1) * static_cast<uint32_t>(w) + xl;
    const float fx = t.ax.f, fy = t.ay.f;
    float a0[CT], b0[CT], a1[CT], b1[CT];
    auto load_channel = [&](int ch) {
        if (w >= 2) {  // wave-uniform
            load_pair(at(iplane[ch], o0), a0[ch], b0[ch]);
            load_pair(at(iplane[ch], o1), a1[ch], b1[ch]);
        } else {  // single-column frame: both horizontal taps are column 0
            a0[ch] = b0[ch] = to_f32(*at(iplane[ch], static_cast<uint32_t>(t.ay.i0)));
            a1[ch] = b1[ch] = to_f32(*at(iplane[ch], static_cast<uint32_t>(t.ay.i1)));
        }
    };
    // Twelve 16-bit channels: every channel's samples are loaded, under one
    // column test, before any is used (4 x 1440p bf16: 940 -> 864 us; with
    // the column test repeated per channel the gain was lost). Elsewhere
    // each channel's loads come with its use: the batched form was 3-15 %
    // slower for four 16-bit channels and for twelve float32 ones.
    constexpr bool batch = CT == 12 && sizeof(T) == 2;
    if constexpr (batch) {
        if (w >= 2) {  // wave-uniform
#pragma unroll
            for (int ch = 0; ch < CT; ++ch) {
                load_pair(at(iplane[ch], o0), a0[ch], b0[ch]);
                load_pair(at(iplane[ch], o1), a1[ch], b1[ch]);
            }
        } else {
#pragma unroll
            for (int ch = 0; ch < CT; ++ch) load_channel(ch);
        }
    }
    float su = 0.0f, sv = 0.0f;
#pragma unroll
    for (int ch = 0; ch < CT; ++ch) {
        if constexpr (!batch) load_channel(ch);
        const float i00 = last ? b0[ch] : a0[ch], i01 = b0[ch];
        const float i10 = last ? b1[ch] : a1[ch], i11 = b1[ch];
        const float dsx = fmaf(fy, i11 - i10, (1.0f - fy) * (i01 - i00));
        const float dsy = fmaf(fx, i11 - i01, (1.0f - fx) * (i10 - i00));
        su = fmaf(g[ch], dsx, su);
        sv = fmaf(g[ch], dsy, sv);
    }
    // sx = x - s*u, so d sx / d u = -s (and likewise for v)
    gu = fmaf(-s, su, gu);
    gv = fmaf(-s, sv, gv);
}

// v from lane - 1 (0 into lane 0): a DPP wavefront shift whose out-of-range
// source reads as zero, so it folds into the consuming add.
__device__ __forceinline__ float shift_up1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}

// Channels of one LDS cell: padded to a multiple of four (one 16-byte LDS
// access per four channels) from three channels up.
template <int CT>
struct CellWidth {
    static constexpr int value = CT <= 2 ? CT : ((CT + 3) / 4) * 4;
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

template <int CP>
__device__ __forceinline__ void cell_read(const float *acc, int cell, float (&v)[CP]) {
    if constexpr (CP % 4 == 0) {
#pragma unroll
        for (int q = 0; q < CP / 4; ++q) {
            const f32x4 t = reinterpret_cast<const f32x4 *>(acc)[cell * (CP / 4) + q];
            v[4 * q] = t.x; v[4 * q + 1] = t.y; v[4 * q + 2] = t.z; v[4 * q + 3] = t.w;
        }
    } else if constexpr (CP == 2) {
        const f32x2 t = reinterpret_cast<const f32x2 *>(acc)[cell];
        v[0] = t.x; v[1] = t.y;
    } else {
        v[0] = acc[cell];
    }
}

template <int CP>
__device__ __forceinline__ void cell_write(float *acc, int cell, const float (&v)[CP]) {
    if constexpr (CP % 4 == 0) {
#pragma unroll
        for (int q = 0; q < CP / 4; ++q) {
            f32x4 t;
            t.x = v[4 * q]; t.y = v[4 * q + 1]; t.z = v[4 * q + 2]; t.w = v[4 * q + 3];
            reinterpret_cast<f32x4 *>(acc)[cell * (CP / 4) + q] = t;
        }
    } else if constexpr (CP == 2) {
        f32x2 t;
        t.x = v[0]; t.y = v[1];
        reinterpret_cast<f32x2 *>(acc)[cell] = t;
    } else {
        acc[cell] = v[0];
    }
}

// What one replayed segment needs from global memory, loaded one segment
// ahead of its use.
template <typename T, int CT, int KT>
struct SegLoad {
    float u, v;
    uint32_t off;      // word (lane & 3) of the segment's SegOffsets
    T g[KT][CT];
};

// One wavefront owns a kTileW x TH tile of the image gradient and keeps it in
// LDS as cells of CP consecutive channels. No other wavefront touches that
// LDS, so no barriers are needed.
//
// Work list: the segments whose boxes reach the tile (only rows and columns
// within the per-frame reach can), plus the tile's own segments ("home"),
// which are replayed even when their taps lie elsewhere because the home tile
// computes their motion gradient. Candidates are classified 64 at a time from
// their boxes; motion, upstream-gradient and tap-offset loads run one segment
// ahead.
//
// Accumulation: for one segment and phase, the lanes whose integer tap offset
// (x - x0, y - y0) equals that of the first lane with an in-tile tap
// ("uniform" lanes) hit pairwise distinct cells, and lane j's right-hand taps
// land on lane j+1's left-hand cells. Each lane therefore adds, without
// atomics, its own left taps plus its left neighbour's right taps to its cell
// of the uniform pattern (one read-add-write of the whole cell per row); lane
// 63 also adds its right taps one cell further. The pattern's row is the same
// for every lane, so a row outside the tile is skipped by the whole wavefront;
// lanes whose column lies outside the tile read a cell but do not write it.
// Lanes with another offset (motion boundaries, random motion) add their taps
// one at a time: where a cell has a spare word (three channels in four) by
// whole-cell read-add-writes that colliding lanes take in turns, otherwise by
// LDS atomics, one per channel, which serialise per lane on this hardware;
// the uniform path must carry the bulk of the work.
//
// Uniform segments (pass 1 found every lane valid with one offset per phase)
// skip the per-lane split, the pattern search and the atomics, and gather the
// samples of their motion gradient with aligned loads shared by the phases
// whose offsets agree. The vector-memory pipeline, not the ALUs, bounds this
// kernel on the pan-and-rectangle workloads, so load instructions are what
// these paths save.
template <typename T, int CT, int KT>
__global__ __launch_bounds__(kSegW) void adjoint_tiles_kernel(BwdArgs<T> a) {
    extern __shared__ __attribute__((aligned(16))) float acc[];  // [TH * kTileW][CP]
    constexpr int CP = CellWidth<CT>::value;
    const int TH = a.tile_h;
    const int w = a.w, h = a.h;
    const int lane = threadIdx.x;

    const int b = xcd_tile_index(blockIdx.x, gridDim.x);
    const int tx = b % a.tiles_x;
    const int rest = b / a.tiles_x;
    const int ty = rest % a.tiles_y;
    const int in = rest / a.tiles_y;
    const int tx0 = tx * kTileW, ty0 = ty * TH;
    const int64_t hw = static_cast<int64_t>(h) * w;
    const T *img = a.src ? a.src + static_cast<int64_t>(in) * CT * hw : nullptr;
    const float *mu = a.mv + (2 * static_cast<int64_t>(in)) * hw;
    const float *mvv = mu + hw;
    const T *gframe = a.gout + static_cast<int64_t>(in) * KT * CT * hw;
    const FrameInfo fi = a.info[in];
    const int reach = min(fi.reach, kFar);
    const int ncells = TH * kTileW;

    for (int i = lane; i < ncells * CP / 4; i += kSegW)
        reinterpret_cast<f32x4 *>(acc)[i] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    // Candidate segments: rows within `reach` of the tile, and columns whose
    // 64-pixel span lies within `reach` of it; the home segments are among them.
    const int r_lo = max(0, ty0 - reach);
    const int r_hi = min(h - 1, ty0 + TH - 1 + reach);
    const int ca = tx0 - (kSegW - 1) - reach;
    const int sc_lo = ca > 0 ? (ca + kSegW - 1) / kSegW : 0;
    const int sc_hi = min(a.segs - 1, (tx0 + kTileW - 1 + reach) / kSegW);
    // Candidate i is row r_lo + (i >> sh), column sc_lo + (i & cm): the columns
    // are padded to a power of two (at most 8 of them) so that no division is
    // needed; padding columns are never hits.
    const int nsc = sc_hi - sc_lo + 1;
    const int sh = nsc <= 1 ? 0 : 32 - __builtin_clz(static_cast<unsigned>(nsc - 1));
    const int cm = (1 << sh) - 1;
    const int total = (r_hi - r_lo + 1) << sh;
    const Box *fboxes = a.boxes + static_cast<int64_t>(in) * h * a.segs;

    auto box_of = [&](int i) -> Box {  // clamped: the load is always in bounds
        const int ic = min(i, total - 1);
        const int c = min(ic & cm, nsc - 1);
        return fboxes[static_cast<int64_t>(r_lo + (ic >> sh)) * a.segs + sc_lo + c];
    };
    // Bit 0: the segment is near (its taps are scattered here); bit 1: home.
    auto classify = [&](const Box &bx, int i) -> int {
        if (i >= total || (i & cm) >= nsc) return 0;
        const int r = r_lo + (i >> sh), sc = sc_lo + (i & cm);
        const bool home = a.gmv && (unsigned)(r - ty0) < (unsigned)TH && sc * kSegW / kTileW == tx;
        const bool near = bx.x_lo <= bx.x_hi && box_reach(bx, sc * kSegW, r) <= kFar &&
                          bx.x_hi >= tx0 && bx.x_lo < tx0 + kTileW && bx.y_hi >= ty0 &&
                          bx.y_lo < ty0 + TH;
        return (near ? 1 : 0) | (home ? 2 : 0);
    };

    int base = 0;
    unsigned long long m_hit = 0, m_near = 0;
    // Next segment to replay as (candidate << 1) | near, or -1 when done. A
    // batch's boxes are loaded when it is classified: holding the next batch's
    // boxes through the replays would cost four registers per lane all along.
    auto next_seg = [&]() -> int {
        while (m_hit == 0) {
            if (base >= total) return -1;
            const int cls = classify(box_of(base + lane), base + lane);
            m_hit = __ballot(cls != 0);
            m_near = __ballot(cls & 1);
            base += kSegW;
        }
        const int j = __builtin_ctzll(m_hit);
        m_hit &= m_hit - 1;
        return ((base - kSegW + j) << 1) | static_cast<int>((m_near >> j) & 1ull);
    };
    // Plane base pointers, loop-invariant and wave-uniform (scalar registers);
    // each load adds a 32-bit in-plane offset.
    const T *gplane[KT][CT];
    const T *iplane[CT];
#pragma unroll
    for (int k = 0; k < KT; ++k)
#pragma unroll
        for (int ch = 0; ch < CT; ++ch) gplane[k][ch] = gframe + (k * CT + ch) * hw;
#pragma unroll
    for (int ch = 0; ch < CT; ++ch) iplane[ch] = img ? img + ch * hw : nullptr;
    auto load_seg = [&](int code, SegLoad<T, CT, KT> &d) {
        const int i = code >> 1;
        const int y = r_lo + (i >> sh);
        const int x = (sc_lo + (i & cm)) * kSegW + lane;
        // lanes past the row end read its last pixel (always in bounds)
        const uint32_t pc = static_cast<uint32_t>(y) * static_cast<uint32_t>(w) + min(x, w - 1);
        d.u = *at(mu, pc);
        d.v = *at(mvv, pc);
        // A vector load (lane j reads word j & 3), not a scalar one: scalar
        // loads share their wait counter with LDS, and every LDS wait of the
        // current replay would also wait for this prefetch.
        const SegOffsets *so =
            a.offs + (static_cast<int64_t>(in) * h + y) * a.segs + (sc_lo + (i & cm));
        d.off = so->k[lane & 3];
#pragma unroll
        for (int k = 0; k < KT; ++k)
#pragma unroll
            for (int ch = 0; ch < CT; ++ch) d.g[k][ch] = *at(gplane[k][ch], pc);
    };

    // Uniform-pattern accumulation of one phase: lane j adds its left taps and
    // lane j-1's right taps to pattern cell (row uy0 / uy0 + 1, column ux);
    // uy0 is wave-uniform, ux = ux(lane 0) + lane.
    auto scatter_pattern = [&](int ux, int uy0, float fx, float fy, const float (&gg)[CT]) {
        const float w00 = (1.0f - fx) * (1.0f - fy), w01 = fx * (1.0f - fy);
        const float w10 = (1.0f - fx) * fy, w11 = fx * fy;
        // Lanes whose column lies outside the tile read some cell of the row
        // but do not write it back (the lane shift in the sums below needs
        // every lane active).
        const bool cx = (unsigned)ux < (unsigned)kTileW;
        const int col = cx ? ux : 0;
        auto add_row = [&](int r, float wl, float wr) {
            const int cell = r * kTileW + col;
            float c[CP], right[CT];
            cell_read<CP>(acc, cell, c);
#pragma unroll
            for (int ch = 0; ch < CT; ++ch) {
                right[ch] = wr * gg[ch];
                c[ch] = fmaf(wl, gg[ch], c[ch]) + shift_up1(right[ch]);
            }
            if (cx) cell_write<CP>(acc, cell, c);
            // lane 63's right-hand taps, one cell to the right
            if (lane == kSegW - 1 && (unsigned)(ux + 1) < (unsigned)kTileW) {
                const int c1 = r * kTileW + ux + 1;
                cell_read<CP>(acc, c1, c);
#pragma unroll
                for (int ch = 0; ch < CT; ++ch) c[ch] += right[ch];
                cell_write<CP>(acc, c1, c);
            }
        };
        if ((unsigned)uy0 < (unsigned)TH) add_row(uy0, w00, w01);
        if ((unsigned)(uy0 + 1) < (unsigned)TH) add_row(uy0 + 1, w10, w11);
    };

    // Replay of one segment (code from next_seg, loads from load_seg).
    auto process = [&](const int code, const SegLoad<T, CT, KT> &cur) {
        const int i = code >> 1;  // wave-uniform
        const bool near = code & 1;
        const int y = r_lo + (i >> sh);
        const int sx0 = (sc_lo + (i & cm)) * kSegW;
        const int x = sx0 + lane;
        const bool inx = x < w;
        // A uniform segment (every lane valid, one integer offset per phase,
        // from pass 1) needs no per-lane validity or pattern tests.
        const bool seg_uniform = __builtin_amdgcn_readlane(cur.off, 0) != kNotUniform;
        PTaps t[KT];
        int ox[KT], oy[KT];  // the offsets of a uniform segment (wave-uniform)
        float g[KT][CT];
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            const float dx = a.s[k] * cur.u, dy = a.s[k] * cur.v;
            if (seg_uniform) {
                const uint32_t o = __builtin_amdgcn_readlane(cur.off, k);
                ox[k] = static_cast<int16_t>(o & 0xffffu);
                oy[k] = static_cast<int>(o) >> 16;
                // the split of an ok lane: i0 = p - ceil(d), f = ceil(d) - d
                t[k].ax.i0 = x - ox[k];
                t[k].ax.i1 = min(t[k].ax.i0 + 1, w - 1);
                t[k].ax.f = static_cast<float>(ox[k]) - dx;
                t[k].ax.ok = true;
                t[k].ay.i0 = y - oy[k];
                t[k].ay.i1 = min(t[k].ay.i0 + 1, h - 1);
                t[k].ay.f = static_cast<float>(oy[k]) - dy;
                t[k].ay.ok = true;
                t[k].valid = true;
            } else {
                t[k].ax = split_axis(dx, x, w);
                t[k].ay = split_axis(dy, y, h);
                t[k].valid = inx && t[k].ax.ok && t[k].ay.ok;
            }
#pragma unroll
            for (int ch = 0; ch < CT; ++ch) g[k][ch] = to_f32(cur.g[k][ch]);
        }

        // Motion gradient of the home segments (every pixel written once).
        if (a.gmv && (unsigned)(y - ty0) < (unsigned)TH && sx0 / kTileW == tx) {
            float gu = 0.0f, gv = 0.0f;
            if (seg_uniform && a.frame_32bit) {
                // The taps of a uniform segment are contiguous across lanes,
                // so its samples are aligned, coalesced single-element loads.
                // When all phases share their offsets (rigid motion slower
                // than one pixel per phase step) they read the same pixels:
                // each channel is loaded once, the right taps come from the
                // neighbouring lane and the samples feed every phase.
                // Otherwise each phase loads its left and its right taps (the
                // second load touches the same cache lines).
                bool same = true;
#pragma unroll
                for (int k = 1; k < KT; ++k) same = same && ox[k] == ox[0] && oy[k] == oy[0];
                // frame-relative 32-bit element offsets from the frame's
                // wave-uniform base (the frame spans less than 4 GB)
                auto samples = [&](int k, int ch, float &a0, float &b0, float &a1, float &b1) {
                    const uint32_t pl = static_cast<uint32_t>(ch) * static_cast<uint32_t>(hw);
                    const uint32_t r0 =
                        pl + static_cast<uint32_t>(y - oy[k]) * static_cast<uint32_t>(w);
                    const uint32_t r1 =
                        pl + static_cast<uint32_t>(min(y - oy[k] + 1, h - 1)) * static_cast<uint32_t>(w);
                    const uint32_t xa = static_cast<uint32_t>(x - ox[k]);  // in the row
                    const uint32_t xb = static_cast<uint32_t>(min(x - ox[k] + 1, w - 1));
                    a0 = to_f32(*at(img, r0 + xa));
                    b0 = to_f32(*at(img, r0 + xb));
                    a1 = to_f32(*at(img, r1 + xa));
                    b1 = to_f32(*at(img, r1 + xb));
                };
                // per-phase sums over channels, in channel order as in
                // motion_grad_phase
                float su[KT], sv[KT];
#pragma unroll
                for (int k = 0; k < KT; ++k) su[k] = sv[k] = 0.0f;
                auto accumulate = [&](int k, int ch, float a0, float b0, float a1, float b1) {
                    const float fx = t[k].ax.f, fy = t[k].ay.f;
                    const float dsx = fmaf(fy, b1 - a1, (1.0f - fy) * (b0 - a0));
                    const float dsy = fmaf(fx, b1 - b0, (1.0f - fx) * (a1 - a0));
                    su[k] = fmaf(g[k][ch], dsx, su[k]);
                    sv[k] = fmaf(g[k][ch], dsy, sv[k]);
                };
                if (same) {  // wave-uniform
                    // Lane j's right taps are lane j+1's left taps (a DPP
                    // shift); lane 63's come from one load spread over lanes
                    // 0 .. 2C-1 (row r0 for lanes < C, r1 above).
                    const uint32_t r0 = static_cast<uint32_t>(y - oy[0]) * static_cast<uint32_t>(w);
                    const uint32_t r1 =
                        static_cast<uint32_t>(min(y - oy[0] + 1, h - 1)) * static_cast<uint32_t>(w);
                    const uint32_t xa = static_cast<uint32_t>(x - ox[0]);  // in the row
                    // Every lane loads (lanes from 2C up repeat lanes C .. 2C-1):
                    // without a branch the gather stays one block, which keeps
                    // its samples' live ranges short.
                    const uint32_t cq = static_cast<uint32_t>(lane % CT);
                    const uint32_t xe = static_cast<uint32_t>(min(sx0 + kSegW - ox[0], w - 1));
                    const float ex =
                        to_f32(*at(img, cq * static_cast<uint32_t>(hw) + (lane < CT ? r0 : r1) + xe));
#pragma unroll
                    for (int ch = 0; ch < CT; ++ch) {
                        const uint32_t pl = static_cast<uint32_t>(ch) * static_cast<uint32_t>(hw);
                        const float a0 = to_f32(*at(img, pl + r0 + xa));
                        const float a1 = to_f32(*at(img, pl + r1 + xa));
                        const int e0 = __builtin_amdgcn_readlane(__float_as_int(ex), ch);
                        const int e1 = __builtin_amdgcn_readlane(__float_as_int(ex), CT + ch);
                        // wave shift left by one; lane 63 keeps the old value
                        const float b0 = __int_as_float(
                            __builtin_amdgcn_update_dpp(e0, __float_as_int(a0), 0x130, 0xf, 0xf, false));
                        const float b1 = __int_as_float(
                            __builtin_amdgcn_update_dpp(e1, __float_as_int(a1), 0x130, 0xf, 0xf, false));
#pragma unroll
                        for (int k = 0; k < KT; ++k) accumulate(k, ch, a0, b0, a1, b1);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < KT; ++k) {
#pragma unroll
                        for (int ch = 0; ch < CT; ++ch) {
                            float a0, b0, a1, b1;
                            samples(k, ch, a0, b0, a1, b1);
                            accumulate(k, ch, a0, b0, a1, b1);
                        }
                        // one phase's samples in registers at a time
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                // sx = x - s*u, so d sx / d u = -s (and likewise for v)
#pragma unroll
                for (int k = 0; k < KT; ++k) {
                    gu = fmaf(-a.s[k], su[k], gu);
                    gv = fmaf(-a.s[k], sv[k], gv);
                }
            } else {
#pragma unroll
                for (int k = 0; k < KT; ++k)
                    if (t[k].valid) motion_grad_phase<T, CT>(iplane, w, t[k], g[k], a.s[k], gu, gv);
            }
            if (inx) {
                float *gm = a.gmv + 2 * static_cast<int64_t>(in) * hw;
                const uint32_t p = static_cast<uint32_t>(y) * static_cast<uint32_t>(w) + x;
                *at(gm, p) = gu;
                *at(gm + hw, p) = gv;
            }
        }

        if (!near) return;  // wave-uniform; far segments are scattered by pass 3
        if (seg_uniform) {
#pragma unroll
            for (int k = 0; k < KT; ++k) {
                // pattern column of lane 0 and pattern row (wave-uniform); the
                // taps span columns ux0 .. ux0 + 64 and rows uy0, uy0 + 1
                const int ux0 = sx0 - ox[k] - tx0, uy0 = y - oy[k] - ty0;
                if (ux0 < -kSegW || ux0 >= kTileW || uy0 < -1 || uy0 >= TH) continue;
                scatter_pattern(ux0 + lane, uy0, t[k].ax.f, t[k].ay.f, g[k]);
            }
            return;
        }
#pragma unroll
        for (int k = 0; k < KT; ++k) {
            // A tap lies in the tile iff the first tap is at most one column
            // (row) before it: the second is the first + 1, or the same at the
            // last column (row).
            const int lx0 = t[k].ax.i0 - tx0, ly0 = t[k].ay.i0 - ty0;
            const bool any = t[k].valid && (unsigned)(lx0 + 1) < (unsigned)(kTileW + 1) &&
                             (unsigned)(ly0 + 1) < (unsigned)(TH + 1);
            const unsigned long long any_m = __ballot(any);
            if (any_m == 0ull) continue;  // wave-uniform
            // Uniform offset: that of the first lane with an in-tile tap.
            const int offx = x - t[k].ax.i0, offy = y - t[k].ay.i0;
            const int src_lane = __builtin_ctzll(any_m);
            const int rx = __builtin_amdgcn_readlane(offx, src_lane);
            const int ry = __builtin_amdgcn_readlane(offy, src_lane);
            const bool uni = any && offx == rx && offy == ry;
            // (lanes off the pattern take part with g = 0: their cell of the
            // pattern still receives the left neighbour's taps)
            float gg[CT];
#pragma unroll
            for (int ch = 0; ch < CT; ++ch) gg[ch] = uni ? g[k][ch] : 0.0f;
            const float fx = t[k].ax.f, fy = t[k].ay.f;
            scatter_pattern(x - rx - tx0, y - ry - ty0, fx, fy, gg);
            // Lanes off the uniform pattern (motion boundaries, random motion).
            if constexpr (CP > CT) {
                // Cells have a spare word: whole-cell read-add-writes, one tap
                // position at a time. Lanes whose cells coincide take turns:
                // each writes its lane number into the cell's spare word and
                // the lane that reads its own number back adds its tap this
                // round (LDS accesses of one wavefront complete in order; every
                // round retires at least one lane per contested cell). One
                // read-add-write covers all channels, where atomics take one
                // per channel, and the order of the additions is fixed.
                const bool off = any && !uni;
                if (__ballot(off)) {
                    const float w00 = (1.0f - fx) * (1.0f - fy), w01 = fx * (1.0f - fy);
                    const float w10 = (1.0f - fx) * fy, w11 = fx * fy;
                    const int lx1 = t[k].ax.i1 - tx0, ly1 = t[k].ay.i1 - ty0;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int lx = (q & 1) ? lx1 : lx0, ly = (q & 2) ? ly1 : ly0;
                        const float wq = q == 0 ? w00 : (q == 1 ? w01 : (q == 2 ? w10 : w11));
                        bool pend = off && (unsigned)lx < (unsigned)kTileW &&
                                    (unsigned)ly < (unsigned)TH && wq != 0.0f;
                        const int cell = pend ? ly * kTileW + lx : 0;
                        // (atomic accesses: the read must not be served from
                        // this lane's own store)
                        int *own = reinterpret_cast<int *>(acc) + cell * CP + (CP - 1);
                        while (__ballot(pend)) {  // wave-uniform
                            if (pend)
                                __hip_atomic_store(own, lane, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
                            if (pend && __hip_atomic_load(own, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_WORKGROUP) == lane) {
                                float c[CP];
                                cell_read<CP>(acc, cell, c);
#pragma unroll
                                for (int ch = 0; ch < CT; ++ch) c[ch] = fmaf(wq, g[k][ch], c[ch]);
                                cell_write<CP>(acc, cell, c);
                                pend = false;
                            }
                        }
                    }
                }
            } else if (__ballot(any && !uni)) {  // LDS atomics
                if (any && !uni) {
                    const float w00 = (1.0f - fx) * (1.0f - fy), w01 = fx * (1.0f - fy);
                    const float w10 = (1.0f - fx) * fy, w11 = fx * fy;
                    const int lx1 = t[k].ax.i1 - tx0, ly1 = t[k].ay.i1 - ty0;
                    const bool inx0 = (unsigned)lx0 < (unsigned)kTileW;
                    const bool inx1 = (unsigned)lx1 < (unsigned)kTileW;
                    const bool iny0 = (unsigned)ly0 < (unsigned)TH;
                    const bool iny1 = (unsigned)ly1 < (unsigned)TH;
#pragma unroll
                    for (int ch = 0; ch < CT; ++ch) {
                        const float gk = g[k][ch];
                        if (inx0 && iny0 && w00 != 0.0f)
                            atomicAdd(acc + (ly0 * kTileW + lx0) * CP + ch, w00 * gk);
                        if (inx1 && iny0 && w01 != 0.0f)
                            atomicAdd(acc + (ly0 * kTileW + lx1) * CP + ch, w01 * gk);
                        if (inx0 && iny1 && w10 != 0.0f)
                            atomicAdd(acc + (ly1 * kTileW + lx0) * CP + ch, w10 * gk);
                        if (inx1 && iny1 && w11 != 0.0f)
                            atomicAdd(acc + (ly1 * kTileW + lx1) * CP + ch, w11 * gk);
                    }
                }
            }
        }
    };

    // The next segment's loads are in flight while the current one is
    // replayed. (Alternating two buffers without the copy needs more
    // registers and was measured slower for 16-bit frames.)
    SegLoad<T, CT, KT> cur, nxt;
    int code = next_seg();
    if (code >= 0) load_seg(code, cur);
    while (code >= 0) {
        const int ncode = next_seg();
        if (ncode >= 0) load_seg(ncode, nxt);
        process(code, cur);
        code = ncode;
        cur = nxt;
    }

    if (!a.gsrc) return;
    // Store the finished tile, one pixel (all channels) per lane and step. 16-bit
    // frames that also receive far-segment atomics go through the float32
    // accumulator instead.
    const bool to_accum = fi.has_far && a.accum32 != nullptr;
    for (int c = lane; c < ncells; c += kSegW) {
        const int X = tx0 + c % kTileW, Y = ty0 + c / kTileW;
        if (X >= w || Y >= h) continue;
        float v[CP];
        cell_read<CP>(acc, c, v);
        const uint32_t o = static_cast<uint32_t>(Y) * static_cast<uint32_t>(w) + X;
        const int64_t frame = static_cast<int64_t>(in) * CT * hw;
#pragma unroll
        for (int ch = 0; ch < CT; ++ch) {
            if (to_accum)
                *at(a.accum32 + frame + ch * hw, o) = v[ch];
            else
                *at(a.gsrc + frame + ch * hw, o) = from_f32<T>(v[ch]);
        }
    }
}

// ---------------------------------------------------------------- pass 3

// Far segments: scatter with global float32 atomics (their motion gradient is
// computed by their home tile in pass 2).
template <typename T, int CT, int KT>
__global__ __launch_bounds__(kThreads) void adjoint_far_kernel(BwdArgs<T> a, float *accum) {
    const int C = CT, w = a.w, h = a.h;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kSegW);  // scalar
    const int lane = threadIdx.x % kSegW;
    const int64_t hw = static_cast<int64_t>(h) * w;
    const int64_t per_frame = static_cast<int64_t>(h) * a.segs;
    // The frames' far flags, 64 at a time (one load and a ballot per 64
    // frames, not a chain of one load per frame); then the flagged frames.
    for (int f0 = 0; f0 < a.n; f0 += kSegW)
    for (unsigned long long fm = __ballot(f0 + lane < a.n && a.info[f0 + lane].has_far != 0); fm;
         fm &= fm - 1) {
        const int in = f0 + __builtin_ctzll(fm);  // uniform across the grid
        float *acc = accum + static_cast<int64_t>(in) * C * hw;
        for (int64_t sg = static_cast<int64_t>(blockIdx.x) * (kThreads / kSegW) + wave;
             sg < per_frame; sg += static_cast<int64_t>(gridDim.x) * (kThreads / kSegW)) {
            const int y = static_cast<int>(sg / a.segs);
            const int sx0 = static_cast<int>(sg % a.segs) * kSegW;
            const Box bx = a.boxes[static_cast<int64_t>(in) * per_frame + sg];
            if (bx.x_lo > bx.x_hi || box_reach(bx, sx0, y) <= kFar) continue;
            const int x = sx0 + lane;
            if (x >= w) continue;
            const int64_t p = static_cast<int64_t>(y) * w + x;
            const float u = a.mv[(2 * static_cast<int64_t>(in)) * hw + p];
            const float v = a.mv[(2 * static_cast<int64_t>(in) + 1) * hw + p];
#pragma unroll
            for (int k = 0; k < KT; ++k) {
                const Axis ax = split_axis(a.s[k] * u, x, w);
                const Axis ay = split_axis(a.s[k] * v, y, h);
                if (!(ax.ok && ay.ok)) continue;
                const T *gp = a.gout + (static_cast<int64_t>(in) * KT + k) * C * hw + p;
                const float fx = ax.f, fy = ay.f;
                const float w00 = (1.0f - fx) * (1.0f - fy), w01 = fx * (1.0f - fy);
                const float w10 = (1.0f - fx) * fy, w11 = fx * fy;
                const int64_t r0 = static_cast<int64_t>(ay.i0) * w;
                const int64_t r1 = static_cast<int64_t>(ay.i1) * w;
#pragma unroll
                for (int ch = 0; ch < CT; ++ch) {
                    const float g = to_f32(gp[ch * hw]);
                    float *pl = acc + ch * hw;
                    if (w00 != 0.0f) atomicAdd(pl + r0 + ax.i0, w00 * g);
                    if (w01 != 0.0f) atomicAdd(pl + r0 + ax.i1, w01 * g);
                    if (w10 != 0.0f) atomicAdd(pl + r1 + ax.i0, w10 * g);
                    if (w11 != 0.0f) atomicAdd(pl + r1 + ax.i1, w11 * g);
                }
            }
        }
    }
}

// ---------------------------------------------------------------- pass 4

template <typename T>
__global__ __launch_bounds__(kThreads) void cast_far_frames_kernel(const float *accum32, T *gsrc,
                                                                   const FrameInfo *info, int n,
                                                                   int64_t frame_elems) {
    const int lane = threadIdx.x % kSegW;
    for (int f0 = 0; f0 < n; f0 += kSegW)  // far flags 64 at a time, as in pass 3
    for (unsigned long long fm = __ballot(f0 + lane < n && info[f0 + lane].has_far != 0); fm;
         fm &= fm - 1) {
        const int in = f0 + __builtin_ctzll(fm);
        const float *s = accum32 + static_cast<int64_t>(in) * frame_elems;
        T *d = gsrc + static_cast<int64_t>(in) * frame_elems;
        for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
             i < frame_elems; i += static_cast<int64_t>(gridDim.x) * kThreads)
            d[i] = from_f32<T>(s[i]);
    }
}

// ---------------------------------------------------------------- motion only

// Motion gradient alone (no image gradient requested): per pixel, no atomics.
template <typename T, int CT, int KT>
__global__ __launch_bounds__(kThreads) void motion_grad_kernel(BwdArgs<T> a) {
    const int w = a.w, h = a.h;
    // wave-uniform (scalar) segment index
    const int64_t seg = static_cast<int64_t>(blockIdx.x) * (kThreads / kSegW) +
                        __builtin_amdgcn_readfirstlane(threadIdx.x / kSegW);
    const int64_t per_frame = static_cast<int64_t>(h) * a.segs;
    if (seg >= per_frame * a.n) return;
    const int in = static_cast<int>(seg / per_frame);
    const int64_t sg = seg % per_frame;
    const int y = static_cast<int>(sg / a.segs);
    const int x = static_cast<int>(sg % a.segs) * kSegW + static_cast<int>(threadIdx.x % kSegW);
    if (x >= w) return;
    const int64_t hw = static_cast<int64_t>(h) * w;
    const int64_t p = static_cast<int64_t>(y) * w + x;
    const T *img = a.src + static_cast<int64_t>(in) * CT * hw;
    const T *iplane[CT];
#pragma unroll
    for (int ch = 0; ch < CT; ++ch) iplane[ch] = img + ch * hw;
    const float u = a.mv[(2 * static_cast<int64_t>(in)) * hw + p];
    const float v = a.mv[(2 * static_cast<int64_t>(in) + 1) * hw + p];
    float gu = 0.0f, gv = 0.0f;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
        PTaps t;
        t.ax = split_axis(a.s[k] * u, x, w);
        t.ay = split_axis(a.s[k] * v, y, h);
        if (!(t.ax.ok && t.ay.ok)) continue;
        const T *gp = a.gout + (static_cast<int64_t>(in) * KT + k) * CT * hw + p;
        float g[CT];
#pragma unroll
        for (int ch = 0; ch < CT; ++ch) g[ch] = to_f32(gp[ch * hw]);
        motion_grad_phase<T, CT>(iplane, w, t, g, a.s[k], gu, gv);
    }
    a.gmv[(2 * static_cast<int64_t>(in)) * hw + p] = gu;
    a.gmv[(2 * static_cast<int64_t>(in) + 1) * hw + p] = gv;
}


// ---------------------------------------------------------------- any C

// Channel counts without a specialised path: scatter with global float32
// atomics into a zeroed accumulator, motion gradient per pixel.
template <typename T>
__global__ __launch_bounds__(kThreads) void adjoint_generic_kernel(BwdArgs<T> a, float *accum) {
    const int C = a.c, w = a.w, h = a.h;
    // wave-uniform (scalar) segment index
    const int64_t seg = static_cast<int64_t>(blockIdx.x) * (kThreads / kSegW) +
                        __builtin_amdgcn_readfirstlane(threadIdx.x / kSegW);
    const int64_t per_frame = static_cast<int64_t>(h) * a.segs;
    if (seg >= per_frame * a.n) return;
    const int in = static_cast<int>(seg / per_frame);
    const int64_t sg = seg % per_frame;
    const int y = static_cast<int>(sg / a.segs);
    const int x = static_cast<int>(sg % a.segs) * kSegW + static_cast<int>(threadIdx.x % kSegW);
    if (x >= w) return;
    const int64_t hw = static_cast<int64_t>(h) * w;
    const int64_t p = static_cast<int64_t>(y) * w + x;
    const T *img = a.src ? a.src + static_cast<int64_t>(in) * C * hw : nullptr;
    float *acc = accum ? accum + static_cast<int64_t>(in) * C * hw : nullptr;
    const float u = a.mv[(2 * static_cast<int64_t>(in)) * hw + p];
    const float v = a.mv[(2 * static_cast<int64_t>(in) + 1) * hw + p];
    float gu = 0.0f, gv = 0.0f;
    for (int k = 0; k < a.k; ++k) {
        const Axis ax = split_axis(a.s[k] * u, x, w);
        const Axis ay = split_axis(a.s[k] * v, y, h);
        if (!(ax.ok && ay.ok)) continue;
        const float fx = ax.f, fy = ay.f;
        const float w00 = (1.0f - fx) * (1.0f - fy), w01 = fx * (1.0f - fy);
        const float w10 = (1.0f - fx) * fy, w11 = fx * fy;
        const int64_t r0 = static_cast<int64_t>(ay.i0) * w;
        const int64_t r1 = static_cast<int64_t>(ay.i1) * w;
        const T *gp = a.gout + (static_cast<int64_t>(in) * a.k + k) * C * hw + p;
        float su = 0.0f, sv = 0.0f;
        for (int ch = 0; ch < C; ++ch) {
            const float g = to_f32(gp[ch * hw]);
            if (acc) {
                float *pl = acc + ch * hw;
                if (w00 != 0.0f) atomicAdd(pl + r0 + ax.i0, w00 * g);
                if (w01 != 0.0f) atomicAdd(pl + r0 + ax.i1, w01 * g);
                if (w10 != 0.0f) atomicAdd(pl + r1 + ax.i0, w10 * g);
                if (w11 != 0.0f) atomicAdd(pl + r1 + ax.i1, w11 * g);
            }
            if (a.gmv) {
                const T *pl = img + ch * hw;
                const float i00 = to_f32(pl[r0 + ax.i0]), i01 = to_f32(pl[r0 + ax.i1]);
                const float i10 = to_f32(pl[r1 + ax.i0]), i11 = to_f32(pl[r1 + ax.i1]);
                const float dsx = fmaf(fy, i11 - i10, (1.0f - fy) * (i01 - i00));
                const float dsy = fmaf(fx, i11 - i01, (1.0f - fx) * (i10 - i00));
                su = fmaf(g, dsx, su);
                sv = fmaf(g, dsy, sv);
            }
        }
        gu = fmaf(-a.s[k], su, gu);
        gv = fmaf(-a.s[k], sv, gv);
    }
    if (a.gmv) {
        a.gmv[(2 * static_cast<int64_t>(in)) * hw + p] = gu;
        a.gmv[(2 * static_cast<int64_t>(in) + 1) * hw + p] = gv;
    }
}

__global__ __launch_bounds__(kThreads) void zero_f32_kernel(float *p, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kThreads)
        p[i] = 0.0f;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void cast_all_kernel(const float *s, T *d, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kThreads)
        d[i] = from_f32<T>(s[i]);
}

template <typename T>
hipError_t run_generic(BwdArgs<T> a, const BwdWorkspace &ws, hipStream_t st) {
    const int64_t segs_total = static_cast<int64_t>(a.n) * a.h * a.segs;
    const unsigned seg_blocks =
        static_cast<unsigned>((segs_total + kThreads / kSegW - 1) / (kThreads / kSegW));
    const int64_t elems = static_cast<int64_t>(a.n) * a.c * a.h * a.w;
    float *accum = nullptr;
    if (a.gsrc) {
        accum = ws.accum32 ? ws.accum32 : reinterpret_cast<float *>(a.gsrc);
        hipLaunchKernelGGL(zero_f32_kernel, dim3(kFarBlocks * 4), dim3(kThreads), 0, st, accum,
                           elems);
    }
    hipLaunchKernelGGL(adjoint_generic_kernel<T>, dim3(seg_blocks), dim3(kThreads), 0, st, a,
                       accum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.gsrc || !ws.accum32) return e;
    hipLaunchKernelGGL(cast_all_kernel<T>, dim3(kFarBlocks * 4), dim3(kThreads), 0, st,
                       ws.accum32, a.gsrc, elems);
    return hipGetLastError();
}

// ---------------------------------------------------------------- launchers

// Pass 1 over N frames: zero the per-frame figures, then the footprint kernel.
template <int KT>
hipError_t footprint_pass(const float *mv, Box *boxes, SegOffsets *offs, FrameInfo *info, int n,
                          int h, int w, const float *s, hipStream_t st) {
    hipError_t e = launch_zero_u32(reinterpret_cast<uint32_t *>(info), static_cast<int64_t>(n) * 2, st);
    if (e != hipSuccess) return e;
    Phases4 ph;
    for (int j = 0; j < 4; ++j) ph.s[j] = s[j];
    const int segs = (w + kSegW - 1) / kSegW;
    const int64_t foot_units = static_cast<int64_t>(n) * ((h + kFootRows - 1) / kFootRows) * segs;
    const unsigned foot_blocks =
        static_cast<unsigned>((foot_units + kThreads / kSegW - 1) / (kThreads / kSegW));
    hipLaunchKernelGGL((footprint_kernel<KT>), dim3(foot_blocks), dim3(kThreads), 0, st, mv,
                       boxes, offs, info, n, h, w, segs, ph);
    return hipGetLastError();
}

int tile_rows_for(int c) {
    // One wavefront per 128 x TH tile of float32 accumulators (2 KB per
    // four-channel row). Taller tiles replay fewer segments (3.5 replays per
    // segment at TH = 2, 2.9 at TH = 3, 2.5 at TH = 4 on workload 2) but hold
    // more LDS per wavefront; measured on workload 2, TH = 3 is fastest for
    // float32 and 16-bit frames with up to four channels (TH = 2 and TH = 4
    // were slower in both), and on three-channel frames under i.i.d. motion
    // (8 x 1080p: 634-649 us against 780, 676 and 774 at TH = 2, 4, 6).
    return c <= 4 ? 3 : 2;
}

template <typename T, int CT, int KT>
hipError_t run(BwdArgs<T> a, const BwdWorkspace &ws, hipStream_t st) {
    const int64_t segs_total = static_cast<int64_t>(a.n) * a.h * a.segs;
    const unsigned seg_blocks =
        static_cast<unsigned>((segs_total + kThreads / kSegW - 1) / (kThreads / kSegW));
    if (!a.gsrc) {  // motion gradient only
        hipLaunchKernelGGL((motion_grad_kernel<T, CT, KT>), dim3(seg_blocks), dim3(kThreads), 0,
                           st, a);
        return hipGetLastError();
    }
    hipError_t e = hipSuccess;
    if (!ws.recorded &&  // else the forward left the footprint in the workspace
        (e = footprint_pass<KT>(a.mv, a.boxes, a.offs, a.info, a.n, a.h, a.w, a.s, st)) != hipSuccess)
        return e;

    const size_t lds = sizeof(float) * CellWidth<CT>::value * a.tile_h * kTileW;
    const int64_t tiles = static_cast<int64_t>(a.n) * a.tiles_x * a.tiles_y;
    hipLaunchKernelGGL((adjoint_tiles_kernel<T, CT, KT>), dim3(static_cast<unsigned>(tiles)),
                       dim3(kSegW), lds, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;

    float *far_accum = ws.accum32 ? ws.accum32 : reinterpret_cast<float *>(a.gsrc);
    hipLaunchKernelGGL((adjoint_far_kernel<T, CT, KT>), dim3(kFarBlocks), dim3(kThreads), 0, st,
                       a, far_accum);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ws.accum32) {
        hipLaunchKernelGGL(cast_far_frames_kernel<T>, dim3(kFarBlocks), dim3(kThreads), 0, st,
                           ws.accum32, a.gsrc, a.info, a.n,
                           static_cast<int64_t>(a.c) * a.h * a.w);
        e = hipGetLastError();
    }
    return e;
}

template <typename T, int CT>
hipError_t run_k(const BwdArgs<T> &a, const BwdWorkspace &ws, hipStream_t st) {
    switch (a.k) {
    case 1: return run<T, CT, 1>(a, ws, st);
    case 2: return run<T, CT, 2>(a, ws, st);
    case 3: return run<T, CT, 3>(a, ws, st);
    default: return run<T, CT, 4>(a, ws, st);
    }
}

template <typename T>
hipError_t run_typed(const void *src, const float *mv, const WarpShape &s, const void *gout,
                     void *gsrc, float *gmv, const BwdWorkspace &ws, hipStream_t st) {
    BwdArgs<T> a;
    a.src = static_cast<const T *>(src);
    a.mv = mv;
    a.gout = static_cast<const T *>(gout);
    a.gsrc = static_cast<T *>(gsrc);
    a.gmv = gmv;
    a.accum32 = ws.accum32;
    a.boxes = reinterpret_cast<Box *>(ws.boxes);
    a.offs = reinterpret_cast<SegOffsets *>(a.boxes + static_cast<size_t>(s.n) * s.h *
                                                          ((s.w + kSegW - 1) / kSegW));
    a.info = reinterpret_cast<FrameInfo *>(ws.info);
    a.n = s.n; a.c = s.c; a.h = s.h; a.w = s.w; a.k = s.k;
    a.segs = (s.w + kSegW - 1) / kSegW;
    a.tile_h = tile_rows_for(s.c);
    a.tiles_x = (s.w + kTileW - 1) / kTileW;
    a.tiles_y = (s.h + a.tile_h - 1) / a.tile_h;
    a.frame_32bit = static_cast<uint64_t>(s.c) * s.h * s.w * sizeof(T) < (uint64_t(1) << 32);
    for (int j = 0; j < 4; ++j) a.s[j] = s.phases[j];
    switch (s.c) {
    case 1: return run_k<T, 1>(a, ws, st);
    case 2: return run_k<T, 2>(a, ws, st);
    case 3: return run_k<T, 3>(a, ws, st);
    case 4: return run_k<T, 4>(a, ws, st);
    case 12: return run_k<T, 12>(a, ws, st);
    default: return run_generic<T>(a, ws, st);
    }
}

}  // namespace

size_t backward_box_bytes(int n, int h, int w) {
    return (sizeof(Box) + sizeof(SegOffsets)) * static_cast<size_t>(n) * h *
           ((w + kSegW - 1) / kSegW);
}

size_t backward_info_bytes(int n) { return sizeof(FrameInfo) * static_cast<size_t>(n); }

bool backward_uses_footprint(int c) { return c == 1 || c == 2 || c == 3 || c == 4 || c == 12; }

hipError_t launch_frame_reach(const WarpShape &s, const BwdWorkspace &ws, const TileFold *fold,
                              hipStream_t stream) {
    const int segs = (s.w + kSegW - 1) / kSegW;
    const int64_t per_frame = static_cast<int64_t>(s.h) * segs;
    const int bx = static_cast<int>((per_frame + kThreads * kReachPerThread - 1) /
                                    (kThreads * kReachPerThread));
    // n * bx < 2^31: the C ABI bounds the batch's 64 x 4 tiles below 2^31
    const int64_t reach_blocks = static_cast<int64_t>(s.n) * bx;
    const int64_t fold_blocks = fold ? static_cast<int64_t>(s.n) * 2 * kTileFoldParts : 0;
    const TileFold none{nullptr, 0, nullptr, nullptr, nullptr};
    hipLaunchKernelGGL(frame_reach_kernel, dim3(static_cast<unsigned>(reach_blocks + fold_blocks)),
                       dim3(kThreads), 0, stream, reinterpret_cast<const Box *>(ws.boxes),
                       reinterpret_cast<FrameInfo *>(ws.info), s.h, segs, bx,
                       static_cast<int>(reach_blocks), fold ? *fold : none);
    return hipGetLastError();
}

hipError_t launch_footprint(const float *mv, const WarpShape &s, const BwdWorkspace &ws,
                            hipStream_t stream) {
    Box *boxes = reinterpret_cast<Box *>(ws.boxes);
    SegOffsets *offs = reinterpret_cast<SegOffsets *>(
        boxes + static_cast<size_t>(s.n) * s.h * ((s.w + kSegW - 1) / kSegW));
    FrameInfo *info = reinterpret_cast<FrameInfo *>(ws.info);
    switch (s.k) {
    case 1: return footprint_pass<1>(mv, boxes, offs, info, s.n, s.h, s.w, s.phases, stream);
    case 2: return footprint_pass<2>(mv, boxes, offs, info, s.n, s.h, s.w, s.phases, stream);
    case 3: return footprint_pass<3>(mv, boxes, offs, info, s.n, s.h, s.w, s.phases, stream);
    default: return footprint_pass<4>(mv, boxes, offs, info, s.n, s.h, s.w, s.phases, stream);
    }
}

hipError_t launch_backward(int dtype, const void *src, const float *mv, const WarpShape &s,
                           const void *grad_out, void *grad_src, float *grad_mv,
                           const BwdWorkspace &ws, hipStream_t stream) {
    switch (dtype) {
    case 0: return run_typed<float>(src, mv, s, grad_out, grad_src, grad_mv, ws, stream);
    case 1: return run_typed<_Float16>(src, mv, s, grad_out, grad_src, grad_mv, ws, stream);
    default: return run_typed<__bf16>(src, mv, s, grad_out, grad_src, grad_mv, ws, stream);
    }
}

}  // namespace exw
