// Forward motion-vector warp for CDNA4 (gfx950).
//
// What is computed (paper §II-B image warping; §IV-B: the predicted frames
// P_1..P_3 shown at t + i/4 all come from F_t; §III-B: warped pixels without
// a source in the frame are invalid): each output pixel reads its motion
// vector once, forms all K phase displacements, gathers the four bilinear
// taps of every channel, and writes K output pixels, K mask bytes and the
// per-(frame, phase) invalid counts.
//
// Layout of the work: a wavefront per 128 consecutive pixels of a row, four
// wavefronts per 128 x 4 tile (a workgroup, or four consecutive workgroups of
// one wavefront for twelve 16-bit channels), tiles renumbered per XCD. The
// motion vector is read once for all K phases; motion, output and mask
// accesses are coalesced; the taps of neighbouring lanes fall on neighbouring addresses
// wherever the motion is locally smooth. A segment whose 128 pixels share one
// integer tap offset per phase takes two pixels per lane (two-element loads
// and stores plus a lane shift); otherwise each 64-pixel half runs the
// one-pixel paths: a wavefront whose lanes share one offset loads one aligned
// element per row and channel plus a lane shift, others load the two
// horizontal taps of a row in one (unaligned) 8-byte load. Measured HBM
// traffic equals the algorithmic bytes (the L2 serves the overlap between
// tiles), so the taps are gathered from global memory; an LDS-staged variant
// and four pixels per lane were both measured slower. No MFMA: this is a
// gather. The recording instantiation (REC) also writes the adjoint's
// footprint records of its two 64-pixel segments (footprint.h), so that the
// adjoint of a training step can skip its first pass.
#include "footprint.h"
#include "launch.h"
#include "moments.h"
#include "warp_common.h"

namespace exw {
namespace {

constexpr int kTileW = 64;     // pixels of a row per wavefront in the one-pixel paths
constexpr int kTileH = 4;
constexpr int kThreads = kTileW * kTileH;
constexpr int kSegPair = 2 * kTileW;  // pixels of a row per wavefront (two per lane)

template <typename T>
struct FwdArgs {
    const T *src;
    const float *mv;
    T *out;
    uint8_t *mask;
    uint32_t *count;
    int n, c, h, w, k;
    int tiles_x, tiles_y;
    int frame_32bit;  // C * H * W * sizeof(T) < 2^32: frame-relative 32-bit offsets
    float s[4];
    // The adjoint's footprint records, written when the caller asks for them
    // (the kernel's REC instantiation): [N][H][segs] boxes and offsets of
    // the 64-pixel row segments. The per-frame figures are reduced from the
    // boxes by a pass of their own (one update per wavefront here would hold
    // every wavefront for a memory round trip); this kernel zeroes them.
    Box *boxes;
    SegOffsets *offs;
    uint32_t *info_words;  // the per-frame figures (2 words per frame), zeroed by block 0
    int segs;
    // Motion-statistics partials ([N][2][tiles per frame], the STATS
    // instantiation): one per 128 x 4 tile and motion component; and the
    // fold's counters ([N][2]), zeroed by block 0 for the pass that follows.
    Moments *stat_parts;
    uint32_t *stat_counters;
};

struct PixelPos {
    int in, x, y;
    bool inside;
};


// v from lane + 1, and `last` (a value read back from another lane) into
// lane 63. Read-backs are taken outside divergent code: inside a branch of
// lane 63 alone, the compiler may sink the load they read there, and the
// lanes that were to load would not execute it.
__device__ __forceinline__ float shift_down1_or(int last, float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(last, __float_as_int(v), 0x130, 0xf, 0xf, false));
}

__device__ __forceinline__ void count_invalid(uint32_t *count, int64_t plane, bool inside,
                                              bool valid) {
    // One atomic per wavefront that saw invalid pixels (frame borders only).
    const unsigned long long bal = __ballot(inside && !valid);
    if (bal != 0ull && __lane_id() == 0)
        atomicAdd(count + plane, static_cast<uint32_t>(__popcll(bal)));
}

// The uniform gather of all K phases at once, if every lane of the wavefront
// is in the frame and every phase is uniform (see warp_forward_kernel);
// returns false, having done nothing, otherwise (all lanes must take part in
// the lane shifts: a shift from an inactive lane reads zero). Lanes 0 .. 2CK-1 fetch lane 63's right-hand taps of
// every phase, row and channel in one load instruction. Only the fractions
// stay in registers between the uniformity test and the blend; tap rows and
// columns are recomputed from the wave-uniform offsets.
template <typename T, int CT, int KT>
__device__ __forceinline__ bool all_phases_uniform(const FwdArgs<T> &a, const PixelPos &q, float u,
                                                   float v, const T *img, int64_t hw,
                                                   uint32_t p) {
    const int w = a.w, h = a.h;
    // Every access is the frame's wave-uniform base (scalar registers) plus a
    // 32-bit offset channel * H*W + pixel: the caller checks that a frame of
    // the source (and of one phase of the output) spans less than 4 GB.
    const T *fin = img;
    const uint32_t hw32 = static_cast<uint32_t>(hw);
    float fx[KT], fy[KT];
    int rx[KT], ry[KT];
    bool uni = true;
#pragma unroll
    for (int j = 0; j < KT; ++j) {
        const Axis ax = split_axis(a.s[j] * u, q.x, w);
        const Axis ay = split_axis(a.s[j] * v, q.y, h);
        const int offx = q.x - ax.i0, offy = q.y - ay.i0;
        rx[j] = __builtin_amdgcn_readfirstlane(offx);
        ry[j] = __builtin_amdgcn_readfirstlane(offy);
        // every lane in the frame: the lane shifts below read all 64 lanes
        uni = uni && q.inside && ax.ok && ay.ok && offx == rx[j] && offy == ry[j];
        fx[j] = ax.f;
        fy[j] = ay.f;
    }
    if (__ballot(uni) != ~0ull) return false;
    const int tx0 = q.x - static_cast<int>(threadIdx.x);
    // tap rows (wave-uniform) and columns of phase j
    auto row0 = [&](int j) { return static_cast<uint32_t>(q.y - ry[j]) * static_cast<uint32_t>(w); };
    auto row1 = [&](int j) {
        return static_cast<uint32_t>(min(q.y - ry[j] + 1, h - 1)) * static_cast<uint32_t>(w);
    };
    // Lane l < 2CK loads lane 63's right-hand tap of phase l / 2C, row
    // (l / C) % 2 and channel l % C; the other lanes repeat lane l % 2CK. No
    // branch around the load: converting a 16-bit value inside one made the
    // wavefront wait for it before issuing the gathers.
    T exr;
    {
        const int lq = static_cast<int>(threadIdx.x) % (2 * CT * KT);
        const int jq = lq / (2 * CT), rq = (lq / CT) % 2, cq = lq % CT;
        int ryq = ry[0], rxq = rx[0];
#pragma unroll
        for (int j = 1; j < KT; ++j)
            if (jq == j) { ryq = ry[j]; rxq = rx[j]; }
        const int rowq = rq ? min(q.y - ryq + 1, h - 1) : q.y - ryq;
        const uint32_t off = static_cast<uint32_t>(rowq) * static_cast<uint32_t>(w) +
                             static_cast<uint32_t>(min(tx0 + kTileW - rxq, w - 1));
        exr = *at(fin, off + static_cast<uint32_t>(cq) * hw32);
    }
    float a0[KT][CT], a1[KT][CT];
#pragma unroll
    for (int j = 0; j < KT; ++j) {
        if (j > 0 && rx[j] == rx[j - 1] && ry[j] == ry[j - 1]) {  // wave-uniform
            // same integer offsets as the previous phase: the same pixels
#pragma unroll
            for (int ch = 0; ch < CT; ++ch) {
                a0[j][ch] = a0[j - 1][ch];
                a1[j][ch] = a1[j - 1][ch];
            }
            continue;
        }
        const uint32_t xa = static_cast<uint32_t>(q.x - rx[j]);  // in the row: every lane is valid
        const uint32_t o0 = row0(j) + xa, o1 = row1(j) + xa;
#pragma unroll
        for (int ch = 0; ch < CT; ++ch) {
            a0[j][ch] = to_f32(*at(fin, o0 + ch * hw32));
            a1[j][ch] = to_f32(*at(fin, o1 + ch * hw32));
        }
    }
    const float ex = to_f32(exr);
#pragma unroll
    for (int j = 0; j < KT; ++j) {
        const float w00 = (1.0f - fx[j]) * (1.0f - fy[j]);
        const float w01 = fx[j] * (1.0f - fy[j]);
        const float w10 = (1.0f - fx[j]) * fy[j];
        const float w11 = fx[j] * fy[j];
        T *fout = a.out + (static_cast<int64_t>(q.in) * KT + j) * CT * hw;
#pragma unroll
        for (int ch = 0; ch < CT; ++ch) {
            const int e0 = __builtin_amdgcn_readlane(__float_as_int(ex), j * 2 * CT + ch);
            const int e1 = __builtin_amdgcn_readlane(__float_as_int(ex), j * 2 * CT + CT + ch);
            const float b0 = shift_down1_or(e0, a0[j][ch]), b1 = shift_down1_or(e1, a1[j][ch]);
            float acc = w00 * a0[j][ch];
            acc = fmaf(w01, b0, acc);
            acc = fmaf(w10, a1[j][ch], acc);
            acc = fmaf(w11, b1, acc);
            *at(fout, p + ch * hw32) = from_f32<T>(acc);
        }
        if (a.mask) *at(a.mask + (static_cast<int64_t>(q.in) * KT + j) * hw, p) = 1;  // all valid
    }
    return true;  // no invalid pixel: the zeroed counts stay as they are
}

// Channel count CT and phase count KT known at compile time; requires W >= 2
// (paired horizontal loads). Wavefronts that are uniform in every phase take
// all_phases_uniform; the others go one phase at a time: its gathers, then its
// stores. Addresses are 32-bit offsets inside a plane added to per-plane base
// pointers that are uniform across the wavefront (scalar registers), which
// keeps 64-bit address arithmetic off the vector ALU.
template <typename T, int CT, int KT>
__device__ __forceinline__ void forward_row(const FwdArgs<T> &a, const PixelPos q) {
    const int w = a.w, h = a.h;
    const int64_t hw = static_cast<int64_t>(h) * w;
    const uint32_t p = static_cast<uint32_t>(q.y) * static_cast<uint32_t>(w) +
                       static_cast<uint32_t>(q.x);
    const float *mu = a.mv + 2 * static_cast<int64_t>(q.in) * hw;
    float u = 0.0f, v = 0.0f;
    if (q.inside) {
        u = *at(mu, p);
        v = *at(mu + hw, p);
    }
    // Plane base pointers: loop-invariant and wave-uniform (scalar registers),
    // so every access is a scalar base plus a 32-bit vector offset.
    const T *img = a.src + static_cast<int64_t>(q.in) * CT * hw;
    const T *iplane[CT];
    T *oplane[KT][CT];
    uint8_t *mplane[KT];
#pragma unroll
    for (int ch = 0; ch < CT; ++ch) iplane[ch] = img + ch * hw;
#pragma unroll
    for (int j = 0; j < KT; ++j) {
        const int64_t plane = static_cast<int64_t>(q.in) * KT + j;
#pragma unroll
        for (int ch = 0; ch < CT; ++ch) oplane[j][ch] = a.out + (plane * CT + ch) * hw;
        mplane[j] = a.mask ? a.mask + plane * hw : nullptr;
    }
    // Every phase uniform and every lane in the frame (smooth motion: nearly
    // every wavefront): the gathers of all K phases are issued together, one
    // memory round trip instead of K.
    if constexpr (2 * CT * KT <= kTileW) {
        if (a.frame_32bit && all_phases_uniform<T, CT, KT>(a, q, u, v, img, hw, p)) return;
    }
#pragma unroll 1
    for (int j = 0; j < KT; ++j) {
        // phase j without dynamic indexing of the argument arrays
        const float sj = j == 0 ? a.s[0] : (j == 1 ? a.s[1] : (j == 2 ? a.s[2] : a.s[3]));
        const Axis ax = split_axis(sj * u, q.x, w);
        const Axis ay = split_axis(sj * v, q.y, h);
        const bool valid = q.inside && ax.ok && ay.ok;
        if (q.inside) {
            const float w00 = (1.0f - ax.f) * (1.0f - ay.f);
            const float w01 = ax.f * (1.0f - ay.f);
            const float w10 = (1.0f - ax.f) * ay.f;
            const float w11 = ax.f * ay.f;
            // The pair (xl, xl + 1) must stay in the row: at the last column the
            // pair starts one to the left and the tap takes its second element.
            const int xl = min(ax.i0, w - 2);
            const bool last = ax.i0 == w - 1;
            float vals[CT];
            // Uniform wavefront: every lane of the row is valid with the integer
            // tap offset of lane 0, so lane j's right-hand taps are lane j+1's
            // left-hand taps. One aligned element load per row and channel plus
            // a lane shift replaces the unaligned pair load; lane 63 fetches its
            // right-hand taps itself.
            const int offx = q.x - ax.i0, offy = q.y - ay.i0;
            const int rx = __builtin_amdgcn_readfirstlane(offx);
            const int ry = __builtin_amdgcn_readfirstlane(offy);
            // (inside this branch only lanes in the frame are active, so a
            // full ballot also means that all 64 lanes take part in the lane
            // shifts: a shift from an inactive lane would read zero)
            const bool uniform = __ballot(valid && offx == rx && offy == ry) == ~0ull;
            if (uniform) {
                const int tx0 = q.x - static_cast<int>(threadIdx.x);
                const uint32_t r0 = static_cast<uint32_t>(q.y - ry) * static_cast<uint32_t>(w);
                const uint32_t r1 = static_cast<uint32_t>(ay.i1) * static_cast<uint32_t>(w);
                // lanes past the row end read its last pixel (in bounds, unused)
                const uint32_t xa = static_cast<uint32_t>(min(q.x - rx, w - 1));
                const uint32_t xe = static_cast<uint32_t>(min(tx0 + kTileW - rx, w - 1));
                // Lane 63's right-hand taps (2 rows x C channels) are fetched by
                // lanes 0 .. 2C-1 in one load instruction and read back as
                // wave-uniform values; the other lanes repeat lane l % 2C, so
                // that no load sits in a branch of its own (a 16-bit value
                // converted there is waited for before the next loads issue),
                // and the read-backs follow the row loads.
                const int lq = static_cast<int>(threadIdx.x) % (2 * CT);
                const T *pl = iplane[0];
#pragma unroll
                for (int ch = 1; ch < CT; ++ch)
                    if (lq % CT == ch) pl = iplane[ch];
                const T exr = *at(pl, (lq < CT ? r0 : r1) + xe);
                T ra0[CT], ra1[CT];
#pragma unroll
                for (int ch = 0; ch < CT; ++ch) {
                    ra0[ch] = *at(iplane[ch], r0 + xa);
                    ra1[ch] = *at(iplane[ch], r1 + xa);
                }
                const float ex = to_f32(exr);
#pragma unroll
                for (int ch = 0; ch < CT; ++ch) {
                    const int e0 = __builtin_amdgcn_readlane(__float_as_int(ex), ch);
                    const int e1 = __builtin_amdgcn_readlane(__float_as_int(ex), CT + ch);
                    const float a0 = to_f32(ra0[ch]), a1 = to_f32(ra1[ch]);
                    const float b0 = shift_down1_or(e0, a0);
                    const float b1 = shift_down1_or(e1, a1);
                    float acc = w00 * a0;
                    acc = fmaf(w01, b0, acc);
                    acc = fmaf(w10, a1, acc);
                    acc = fmaf(w11, b1, acc);
                    vals[ch] = acc;
                }
            } else {
                const uint32_t o0 = static_cast<uint32_t>(ay.i0) * static_cast<uint32_t>(w) + xl;
                const uint32_t o1 = static_cast<uint32_t>(ay.i1) * static_cast<uint32_t>(w) + xl;
#pragma unroll
                for (int ch = 0; ch < CT; ++ch) {
                    float a0 = 0.f, b0 = 0.f, a1 = 0.f, b1 = 0.f;
                    if constexpr (sizeof(T) == 2) {
                        // 16-bit: invalid lanes read the plane's first pair
                        // (in bounds, unused) rather than skip the loads, so
                        // that no conversion sits in a branch (where it is
                        // waited for, channel after channel: 4 x 1440p bf16
                        // 241 -> 231 us, 4K f16 859 -> 830 us; float32 frames
                        // keep the branch, 1-2 % faster so)
                        load_pair(at(iplane[ch], valid ? o0 : 0u), a0, b0);
                        load_pair(at(iplane[ch], valid ? o1 : 0u), a1, b1);
                    } else if (valid) {
                        load_pair(at(iplane[ch], o0), a0, b0);
                        load_pair(at(iplane[ch], o1), a1, b1);
                    }
                    float acc = w00 * (last ? b0 : a0);
                    acc = fmaf(w01, b0, acc);
                    acc = fmaf(w10, last ? b1 : a1, acc);
                    acc = fmaf(w11, b1, acc);
                    vals[ch] = valid ? acc : 0.0f;
                }
            }
            T *const *op = oplane[0];
            uint8_t *mp = mplane[0];
#pragma unroll
            for (int jj = 1; jj < KT; ++jj)
                if (j == jj) { op = oplane[jj]; mp = mplane[jj]; }
#pragma unroll
            for (int ch = 0; ch < CT; ++ch) *at(op[ch], p) = from_f32<T>(vals[ch]);
            if (mp) *at(mp, p) = valid ? 1 : 0;
        }
        if (a.count) count_invalid(a.count, static_cast<int64_t>(q.in) * KT + j, q.inside, valid);
    }
}

// The wavefront's row, frame and 128-pixel segment; its first 64 pixels are
// lanes 0..63 of half 0, the next 64 those of half 1.
struct SegPos {
    int in, y, sx0;
};

// ONE: one wavefront per workgroup (the workgroup index counts wavefronts,
// the kTileH rows of a tile on consecutive indices, hence on one XCD);
// otherwise a workgroup of kTileH wavefronts per 128 x kTileH tile.
template <bool ONE>
__device__ __forceinline__ SegPos decode_segment(int tiles_x, int tiles_y) {
    const int bi = xcd_tile_index(blockIdx.x, gridDim.x);
    const int b = ONE ? bi / kTileH : bi;
    const int row = ONE ? bi % kTileH : static_cast<int>(threadIdx.y);
    const int tx = b % tiles_x;
    const int rest = b / tiles_x;
    // (the values are wave-uniform, and taking them from lane 0 keeps them,
    // and the frame bases, in scalar registers)
    SegPos g;
    g.in = __builtin_amdgcn_readfirstlane(rest / tiles_y);
    g.y = __builtin_amdgcn_readfirstlane((rest % tiles_y) * kTileH + row);
    g.sx0 = __builtin_amdgcn_readfirstlane(tx * kSegPair);
    return g;
}

// Workgroups of one wavefront for the kernels without statistics over
// twelve 16-bit channels: measured 8 % faster there (4 x 1440p bf16,
// 273 -> 250 us), and 1-11 % slower for three- and four-channel frames.
template <typename T, int CT, bool STATS>
constexpr bool one_wave_blocks() {
    return !STATS && CT == 12 && sizeof(T) == 2;
}

__device__ __forceinline__ PixelPos half_pixel(const SegPos &g, int half, int w, int h) {
    PixelPos q;
    q.in = g.in;
    q.x = g.sx0 + half * kTileW + threadIdx.x;
    q.y = g.y;
    q.inside = (q.x < w) && (q.y < h);
    return q;
}

// Two adjacent stored values written at once (element-aligned address).
typedef float f32x2_st __attribute__((ext_vector_type(2), aligned(4)));
typedef uint32_t u32_st __attribute__((aligned(2)));
typedef uint16_t u16_st __attribute__((aligned(1)));

__device__ __forceinline__ void store_pair(float *p, float a, float b) {
    f32x2_st v;
    v.x = a;
    v.y = b;
    *reinterpret_cast<f32x2_st *>(p) = v;
}

template <typename T>
__device__ __forceinline__ void store_pair(T *p, float a, float b) {
    const T ta = from_f32<T>(a), tb = from_f32<T>(b);
    uint16_t ba, bb;
    __builtin_memcpy(&ba, &ta, 2);
    __builtin_memcpy(&bb, &tb, 2);
    *reinterpret_cast<u32_st *>(p) = static_cast<uint32_t>(ba) | (static_cast<uint32_t>(bb) << 16);
}

// Two pixels per lane: lane j owns pixels 2j and 2j+1 of the wavefront's
// 128-pixel row segment. When every pixel is in the frame and each phase has
// one integer tap offset for the whole segment, the pair's taps in a row are
// columns c, c+1, c+2 (c = 2j minus the offset): one two-element load gives
// c and c+1, lane j+1's first element is c+2 (a DPP shift; lane 63's come
// from one load spread over lanes 0 .. 2C-1), and both outputs of a plane are
// stored at once - half the memory instructions per pixel of the one-pixel
// path. Phases with the offsets of the previous phase reuse its samples. The
// blend is that of the one-pixel path, term for term. (u0, v0), (u1, v1): the
// motion of the lane's two pixels; after_first_loads() runs once the first
// phase's gathers are issued. Returns false, having written nothing, when
// the segment is not uniform; else true, with the offsets (ceil(s_k u),
// ceil(s_k v)) of every phase in (orx, ory).
template <typename T, int CT, int KT, typename Hook>
__device__ __forceinline__ bool pair_uniform(const FwdArgs<T> &a, const SegPos &g, float u0,
                                             float u1, float v0, float v1, int (&orx)[KT],
                                             int (&ory)[KT], Hook &&after_first_loads) {
    const int w = a.w, h = a.h, y = g.y;
    const int64_t hw = static_cast<int64_t>(h) * w;
    const uint32_t hw32 = static_cast<uint32_t>(hw);  // the frame spans less than 4 GB
    const int x = g.sx0 + 2 * static_cast<int>(threadIdx.x);
    const uint32_t p = static_cast<uint32_t>(y) * static_cast<uint32_t>(w) + static_cast<uint32_t>(x);
    float fx0[KT], fx1[KT], fy0[KT], fy1[KT];
    int rx[KT], ry[KT];
    bool uni = true;
#pragma unroll
    for (int j = 0; j < KT; ++j) {
        const Axis ax0 = split_axis(a.s[j] * u0, x, w), ax1 = split_axis(a.s[j] * u1, x + 1, w);
        const Axis ay0 = split_axis(a.s[j] * v0, y, h), ay1 = split_axis(a.s[j] * v1, y, h);
        const int ox0 = x - ax0.i0, ox1 = x + 1 - ax1.i0;
        const int oy0 = y - ay0.i0, oy1 = y - ay1.i0;
        rx[j] = __builtin_amdgcn_readfirstlane(ox0);
        ry[j] = __builtin_amdgcn_readfirstlane(oy0);
        uni = uni && ax0.ok && ax1.ok && ay0.ok && ay1.ok && ox0 == rx[j] && ox1 == rx[j] &&
              oy0 == ry[j] && oy1 == ry[j];
        fx0[j] = ax0.f; fx1[j] = ax1.f;
        fy0[j] = ay0.f; fy1[j] = ay1.f;
    }
    if (__ballot(uni) != ~0ull) return false;
    const T *fin = a.src + static_cast<int64_t>(g.in) * CT * hw;
    float s0[CT], t0[CT], s1[CT], t1[CT];  // columns c, c+1 of rows r0 and r1
    float ex = 0.0f;                       // lane 63's column c+2, lanes 0 .. 2C-1
#pragma unroll
    for (int j = 0; j < KT; ++j) {
        if (j == 0 || rx[j] != rx[j - 1] || ry[j] != ry[j - 1]) {  // wave-uniform
            const uint32_t r0 = static_cast<uint32_t>(y - ry[j]) * static_cast<uint32_t>(w);
            const uint32_t r1 =
                static_cast<uint32_t>(min(y - ry[j] + 1, h - 1)) * static_cast<uint32_t>(w);
            const uint32_t c = static_cast<uint32_t>(x - rx[j]);  // in the row
            // every lane loads (lanes from 2C up repeat lanes C .. 2C-1): a
            // 16-bit value converted inside a branch would be waited for
            // before the gathers below are issued
            const uint32_t cq = threadIdx.x % CT;
            const uint32_t ce = static_cast<uint32_t>(min(g.sx0 + kSegPair - rx[j], w - 1));
            const T exr = *at(fin, cq * hw32 + (threadIdx.x < CT ? r0 : r1) + ce);
#pragma unroll
            for (int ch = 0; ch < CT; ++ch) {
                load_pair(at(fin, ch * hw32 + r0 + c), s0[ch], t0[ch]);
                load_pair(at(fin, ch * hw32 + r1 + c), s1[ch], t1[ch]);
            }
            ex = to_f32(exr);
        }
        if (j == 0) after_first_loads();  // work that overlaps the gathers in flight
        // pixel 2j: taps (s, t); pixel 2j+1: taps (t, next lane's s)
        const float a00 = (1.0f - fx0[j]) * (1.0f - fy0[j]), a01 = fx0[j] * (1.0f - fy0[j]);
        const float a10 = (1.0f - fx0[j]) * fy0[j], a11 = fx0[j] * fy0[j];
        const float b00 = (1.0f - fx1[j]) * (1.0f - fy1[j]), b01 = fx1[j] * (1.0f - fy1[j]);
        const float b10 = (1.0f - fx1[j]) * fy1[j], b11 = fx1[j] * fy1[j];
        T *fout = a.out + (static_cast<int64_t>(g.in) * KT + j) * CT * hw;
#pragma unroll
        for (int ch = 0; ch < CT; ++ch) {
            const int e0 = __builtin_amdgcn_readlane(__float_as_int(ex), ch);
            const int e1 = __builtin_amdgcn_readlane(__float_as_int(ex), CT + ch);
            const float n0 = shift_down1_or(e0, s0[ch]), n1 = shift_down1_or(e1, s1[ch]);
            float acc0 = a00 * s0[ch];
            acc0 = fmaf(a01, t0[ch], acc0);
            acc0 = fmaf(a10, s1[ch], acc0);
            acc0 = fmaf(a11, t1[ch], acc0);
            float acc1 = b00 * t0[ch];
            acc1 = fmaf(b01, n0, acc1);
            acc1 = fmaf(b10, t1[ch], acc1);
            acc1 = fmaf(b11, n1, acc1);
            store_pair(at(fout, p + ch * hw32), acc0, acc1);
        }
        if (a.mask)  // every pixel valid
            *reinterpret_cast<u16_st *>(a.mask + (static_cast<int64_t>(g.in) * KT + j) * hw + p) = 0x0101;
    }
#pragma unroll
    for (int j = 0; j < KT; ++j) { orx[j] = rx[j]; ory[j] = ry[j]; }
    return true;  // no invalid pixel: the zeroed counts stay as they are
}

// pair_uniform with the lane's motion loaded here (the kernels without
// statistics: the loads stay next to their first use).
template <typename T, int CT, int KT>
__device__ __forceinline__ bool pair_uniform_load(const FwdArgs<T> &a, const SegPos &g,
                                                  int (&orx)[KT], int (&ory)[KT]) {
    const int64_t hw = static_cast<int64_t>(a.h) * a.w;
    const float *mu = a.mv + 2 * static_cast<int64_t>(g.in) * hw;
    const uint32_t p = static_cast<uint32_t>(g.y) * static_cast<uint32_t>(a.w) +
                       static_cast<uint32_t>(g.sx0 + 2 * static_cast<int>(threadIdx.x));
    float u0, u1, v0, v1;
    load_pair(at(mu, p), u0, u1);
    load_pair(at(mu + hw, p), v0, v1);
    return pair_uniform<T, CT, KT>(a, g, u0, u1, v0, v1, orx, ory, [] {});
}

// Footprint records of the wavefront's two 64-pixel segments after the
// two-pixel path: every pixel valid with the offsets (rx, ry) in every phase,
// so the boxes follow from the offsets (what segment_footprint gives).
template <typename T, int KT>
__device__ __forceinline__ void record_pair(const FwdArgs<T> &a, const SegPos &g,
                                            const int (&rx)[KT], const int (&ry)[KT]) {
    int b0[4], b1[4];
    uint32_t rec[KT];
    uniform_footprint<KT>(rx, ry, g.y, g.sx0, a.w, a.h, b0, rec);
    uniform_footprint<KT>(rx, ry, g.y, g.sx0 + kSegW, a.w, a.h, b1, rec);
    const int lane = threadIdx.x;
    if (lane < 2) {  // lane i stores segment i of the pair
        const int64_t at = (static_cast<int64_t>(g.in) * a.h + g.y) * a.segs + g.sx0 / kSegW + lane;
        a.boxes[at] = lane ? Box{b1[0], b1[1], b1[2], b1[3]} : Box{b0[0], b0[1], b0[2], b0[3]};
        SegOffsets o{{0u, 0u, 0u, 0u}};
#pragma unroll
        for (int j = 0; j < KT; ++j) o.k[j] = rec[j];
        a.offs[at] = o;
    }
}

// Footprint records of the wavefront's segments (those inside the frame)
// after the one-pixel paths: the footprint pass's computation, row by row.
template <typename T, int KT>
__device__ __forceinline__ void record_rows(const FwdArgs<T> &a, const SegPos &g) {
    if (g.y >= a.h) return;  // wave-uniform
    const int64_t hw = static_cast<int64_t>(a.h) * a.w;
    const float *mu = a.mv + 2 * static_cast<int64_t>(g.in) * hw;
#pragma unroll 1
    for (int half = 0; half < 2; ++half) {
        const int sx0 = g.sx0 + half * kSegW;
        if (sx0 >= a.w) break;  // wave-uniform
        const int x = sx0 + static_cast<int>(threadIdx.x);
        const bool in_r = x < a.w;
        const int64_t p = static_cast<int64_t>(g.y) * a.w + x;
        const float u = in_r ? mu[p] : 0.0f, v = in_r ? mu[hw + p] : 0.0f;
        int b[4];
        uint32_t rec[KT];
        segment_footprint<KT>(u, v, x, g.y, sx0, a.w, a.h, in_r, a.s, b, rec);
        if (threadIdx.x == 0) {
            const int64_t at = (static_cast<int64_t>(g.in) * a.h + g.y) * a.segs + sx0 / kSegW;
            a.boxes[at] = Box{b[0], b[1], b[2], b[3]};
            SegOffsets o{{0u, 0u, 0u, 0u}};
#pragma unroll
            for (int j = 0; j < KT; ++j) o.k[j] = rec[j];
            a.offs[at] = o;
        }
    }
}

// Motion statistics of the block's tile (the recording forward, STATS). Every
// wavefront of the block takes the same shift (u_0, v_0), the motion of the
// tile's first pixel, and forms the float64 sums of its pixels' differences
// from it and of their squares (differences and squares of float32 values are
// exact in float64) from the motion it holds two pixels per lane for the
// two-pixel path. After the block's other work one lane adds the four
// wavefronts' sums in order and turns them into the tile's (count, mean, M2):
// mean = u_0 + S1 / n, M2 = S2 - S1^2 / n, which loses at most a factor of the
// tile's 512 pixels to cancellation against the two-pass value.
struct WaveSums {
    double n, s[4];  // count; S1(u), S2(u), S1(v), S2(v)
};

__device__ __forceinline__ WaveSums (&stat_slots())[kTileH] {
    __shared__ WaveSums slots[kTileH];
    return slots;
}

// v from another lane (DPP control CTRL on both halves); 0.0 where the
// source lane lies outside the row.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, static_cast<int>(b), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, static_cast<int>(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                static_cast<long long>(static_cast<unsigned>(lo)));
}

// The four sums over the wavefront, transposed: the first two exchange steps
// halve the values each lane carries (lane pairs, then quads), so the steps
// after them move one value instead of four. Afterwards lanes 12..15 of a row
// hold the sums of slots 0, 2, 1, 3 (a fixed order of additions).
__device__ __forceinline__ double wave_sums4(double a0, double a1, double a2, double a3) {
    const int lane = static_cast<int>(threadIdx.x);
    const bool odd = lane & 1, hb = (lane >> 1) & 1;
    // pairs (quad_perm 1,0,3,2): even lanes keep slots 0,1, odd lanes 2,3
    const double b0 = (odd ? a2 : a0) + dpp_f64<0xB1>(odd ? a0 : a2);
    const double b1 = (odd ? a3 : a1) + dpp_f64<0xB1>(odd ? a1 : a3);
    // quads (quad_perm 2,3,0,1): lane q of a quad keeps slot 0, 2, 1, 3
    double c = (hb ? b1 : b0) + dpp_f64<0x4E>(hb ? b0 : b1);
    // the four quads of a row into its lanes 12..15 (row_shr 4, row_shr 8)
    c += dpp_f64<0x114>(c);
    c += dpp_f64<0x118>(c);
    // the four rows
    c += __shfl_xor(c, 16);
    c += __shfl_xor(c, 32);
    return c;
}

__device__ __forceinline__ void wave_motion_sums(float su, float sv, float u0, float u1, float v0,
                                                 float v1, bool in0, bool in1) {
    const double n = static_cast<double>(__popcll(__ballot(in0)) + __popcll(__ballot(in1)));
    double s1u = 0.0, s2u = 0.0, s1v = 0.0, s2v = 0.0;
    if (in0) {
        const double du = static_cast<double>(u0) - su, dv = static_cast<double>(v0) - sv;
        s1u += du; s2u += du * du; s1v += dv; s2v += dv * dv;
    }
    if (in1) {
        const double du = static_cast<double>(u1) - su, dv = static_cast<double>(v1) - sv;
        s1u += du; s2u += du * du; s1v += dv; s2v += dv * dv;
    }
    const double t = wave_sums4(s1u, s2u, s1v, s2v);  // every lane is active here
    const int lane = static_cast<int>(threadIdx.x);
    if (lane >= 12 && lane < 16) {
        const int q = lane - 12;
        stat_slots()[threadIdx.y].s[(q & 1) * 2 + (q >> 1)] = t;
        if (q == 0) stat_slots()[threadIdx.y].n = n;
    }
}

// After the block's other work: every thread reaches the barrier.
template <typename T>
__device__ __forceinline__ void block_motion_partial(const FwdArgs<T> &a, const SegPos &g,
                                                     float su, float sv) {
    __syncthreads();
    if (threadIdx.y == 0 && threadIdx.x < 2) {
        const bool vc = threadIdx.x == 1;
        double n = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int wv = 0; wv < kTileH; ++wv) {
            const WaveSums &q = stat_slots()[wv];
            n += q.n;
            s1 += q.s[vc ? 2 : 0];
            s2 += q.s[vc ? 3 : 1];
        }
        const double shift = vc ? sv : su;
        // a block's tile always holds its first pixel: n >= 1
        const Moments m{n, shift + s1 / n, s2 - s1 * s1 / n};
        const int per_frame = a.tiles_x * a.tiles_y;
        const int tile = xcd_tile_index(blockIdx.x, gridDim.x) - g.in * per_frame;
        a.stat_parts[(static_cast<int64_t>(g.in) * 2 + threadIdx.x) * per_frame + tile] = m;
    }
}

// One 128-pixel row segment per wavefront: two pixels per lane when the whole
// segment is uniform in every phase, otherwise the one-pixel paths on each
// half. REC: also write the adjoint's footprint records of the two segments;
// STATS (with REC): also the tile's motion-statistics partial.
template <typename T, int CT, int KT, bool REC, bool STATS>
__global__ __launch_bounds__(kThreads) void warp_forward_kernel(FwdArgs<T> a) {
    if constexpr (REC) {  // ready for the reduction pass that follows (no launch of its own)
        if (blockIdx.x == 0 && threadIdx.y == 0) {
            for (int i = threadIdx.x; i < 2 * a.n; i += kTileW) a.info_words[i] = 0u;
            if constexpr (STATS)
                for (int i = threadIdx.x; i < 2 * a.n; i += kTileW) a.stat_counters[i] = 0u;
        }
    }
    const SegPos g = decode_segment<one_wave_blocks<T, CT, STATS>()>(a.tiles_x, a.tiles_y);
    if constexpr (STATS) {
        // the motion of the wavefront's pixels 2j, 2j+1 (lane j), for the
        // statistics and the two-pixel path alike
        const int x = g.sx0 + 2 * static_cast<int>(threadIdx.x);
        const bool in0 = g.y < a.h && x < a.w, in1 = g.y < a.h && x + 1 < a.w;
        const int64_t hw = static_cast<int64_t>(a.h) * a.w;
        const float *mu = a.mv + 2 * static_cast<int64_t>(g.in) * hw;
        const uint32_t p = static_cast<uint32_t>(g.y) * static_cast<uint32_t>(a.w) +
                           static_cast<uint32_t>(x);
        // the shift: the motion of the tile's first pixel (wave-uniform address)
        const int y0 = __builtin_amdgcn_readfirstlane(g.y - static_cast<int>(threadIdx.y));
        const uint32_t p0 = static_cast<uint32_t>(y0) * static_cast<uint32_t>(a.w) +
                            static_cast<uint32_t>(g.sx0);
        const float su = *at(mu, p0), sv = *at(mu + hw, p0);
        float u0 = 0.0f, u1 = 0.0f, v0 = 0.0f, v1 = 0.0f;
        if (g.y < a.h && g.sx0 + kSegPair <= a.w) {  // wave-uniform (see below)
            load_pair(at(mu, p), u0, u1);
            load_pair(at(mu + hw, p), v0, v1);
        } else {
            if (in0) { u0 = *at(mu, p); v0 = *at(mu + hw, p); }
            if (in1) { u1 = *at(mu, p + 1); v1 = *at(mu + hw, p + 1); }
        }
        auto sums = [&] { wave_motion_sums(su, sv, u0, u1, v0, v1, in0, in1); };
        bool done = false;
        if constexpr (2 * CT * KT <= kTileW) {
            int rx[KT], ry[KT];
            // (the sums are formed while the first gathers are in flight)
            if (a.frame_32bit && g.y < a.h && g.sx0 + kSegPair <= a.w &&
                pair_uniform<T, CT, KT>(a, g, u0, u1, v0, v1, rx, ry, sums)) {
                record_pair<T, KT>(a, g, rx, ry);
                done = true;
            }
        }
        if (!done) {
            sums();
#pragma unroll 1
            for (int half = 0; half < 2; ++half)
                forward_row<T, CT, KT>(a, half_pixel(g, half, a.w, a.h));
            record_rows<T, KT>(a, g);
        }
        block_motion_partial<T>(a, g, su, sv);
        return;
    } else if constexpr (2 * CT * KT <= kTileW) {
        int rx[KT], ry[KT];
        // (the condition stays in this form: a flag computed ahead of the
        // branch raised this kernel from 65 to 89 VGPRs, two waves per SIMD)
        if (a.frame_32bit && g.y < a.h && g.sx0 + kSegPair <= a.w &&  // wave-uniform
            pair_uniform_load<T, CT, KT>(a, g, rx, ry)) {
            if constexpr (REC) record_pair<T, KT>(a, g, rx, ry);
            return;
        }
    }
#pragma unroll 1
    for (int half = 0; half < 2; ++half) forward_row<T, CT, KT>(a, half_pixel(g, half, a.w, a.h));
    if constexpr (REC) record_rows<T, KT>(a, g);
}

// Any channel count, any phase count, any width (including W == 1): one
// channel at a time, scalar taps.
template <typename T>
__device__ __forceinline__ void generic_row(const FwdArgs<T> &a, const PixelPos q) {
    const int C = a.c, w = a.w, h = a.h;
    const int64_t hw = static_cast<int64_t>(h) * w;
    const int64_t p = static_cast<int64_t>(q.y) * w + q.x;
    float u = 0.0f, v = 0.0f;
    if (q.inside) {
        u = a.mv[(2 * static_cast<int64_t>(q.in)) * hw + p];
        v = a.mv[(2 * static_cast<int64_t>(q.in) + 1) * hw + p];
    }
    const T *img = a.src + static_cast<int64_t>(q.in) * C * hw;
    for (int j = 0; j < a.k; ++j) {
        const Axis ax = split_axis(a.s[j] * u, q.x, w);
        const Axis ay = split_axis(a.s[j] * v, q.y, h);
        const bool valid = q.inside && ax.ok && ay.ok;
        const int64_t plane = static_cast<int64_t>(q.in) * a.k + j;
        if (q.inside) {
            T *o = a.out + plane * C * hw + p;
            const float w00 = (1.0f - ax.f) * (1.0f - ay.f);
            const float w01 = ax.f * (1.0f - ay.f);
            const float w10 = (1.0f - ax.f) * ay.f;
            const float w11 = ax.f * ay.f;
            const int64_t r0 = static_cast<int64_t>(ay.i0) * w;
            const int64_t r1 = static_cast<int64_t>(ay.i1) * w;
            for (int ch = 0; ch < C; ++ch) {
                float acc = 0.0f;
                if (valid) {
                    const T *pl = img + ch * hw;
                    acc = w00 * to_f32(pl[r0 + ax.i0]);
                    acc = fmaf(w01, to_f32(pl[r0 + ax.i1]), acc);
                    acc = fmaf(w10, to_f32(pl[r1 + ax.i0]), acc);
                    acc = fmaf(w11, to_f32(pl[r1 + ax.i1]), acc);
                }
                o[ch * hw] = from_f32<T>(acc);
            }
            if (a.mask) a.mask[plane * hw + p] = valid ? 1 : 0;
        }
        if (a.count) count_invalid(a.count, plane, q.inside, valid);
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void warp_forward_generic_kernel(FwdArgs<T> a) {
    const SegPos g = decode_segment<false>(a.tiles_x, a.tiles_y);
#pragma unroll 1
    for (int half = 0; half < 2; ++half) generic_row<T>(a, half_pixel(g, half, a.w, a.h));
}

__global__ void zero_u32_kernel(uint32_t *p, int64_t n) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < n;
         t += stride)
        p[t] = 0u;
}

// The statistics region of the adjoint's workspace: the tile partials
// ([N][2][parts], parts = the larger of the tile count and the statistics
// pass's partial count, so either route fits), the fold's slots
// ([N][2][kTileFoldParts]) and its counters ([N][2]).
struct StatsRegion {
    Moments *parts, *slots;
    uint32_t *counters;
    int tiles;
    size_t bytes;
};

StatsRegion stats_region(void *base, int n, int h, int w) {
    StatsRegion r;
    r.tiles = ((w + kSegPair - 1) / kSegPair) * ((h + kTileH - 1) / kTileH);
    const int stat_parts = motion_stats_parts(h, w);
    const size_t parts = static_cast<size_t>(r.tiles > stat_parts ? r.tiles : stat_parts);
    const size_t parts_bytes = sizeof(Moments) * 2 * static_cast<size_t>(n) * parts;
    const size_t slot_bytes = sizeof(Moments) * 2 * static_cast<size_t>(n) * kTileFoldParts;
    const uintptr_t b = reinterpret_cast<uintptr_t>(base);
    r.parts = reinterpret_cast<Moments *>(b);
    r.slots = reinterpret_cast<Moments *>(b + parts_bytes);
    r.counters = reinterpret_cast<uint32_t *>(b + parts_bytes + slot_bytes);
    r.bytes = parts_bytes + slot_bytes + sizeof(uint32_t) * 2 * static_cast<size_t>(n);
    return r;
}

template <typename T>
FwdArgs<T> make_args(const void *src, const float *mv, const WarpShape &s, void *out,
                     uint8_t *mask, uint32_t *count) {
    FwdArgs<T> a;
    a.src = static_cast<const T *>(src);
    a.mv = mv;
    a.out = static_cast<T *>(out);
    a.mask = mask;
    a.count = count;
    a.n = s.n; a.c = s.c; a.h = s.h; a.w = s.w; a.k = s.k;
    a.tiles_x = (s.w + kSegPair - 1) / kSegPair;
    a.tiles_y = (s.h + kTileH - 1) / kTileH;
    a.frame_32bit = static_cast<uint64_t>(s.c) * s.h * s.w * sizeof(T) < (uint64_t(1) << 32);
    for (int j = 0; j < 4; ++j) a.s[j] = s.phases[j];
    a.boxes = nullptr;
    a.offs = nullptr;
    a.info_words = nullptr;
    a.segs = (s.w + kSegW - 1) / kSegW;
    a.stat_parts = nullptr;
    a.stat_counters = nullptr;
    return a;
}

template <typename T, int CT, bool REC, bool STATS>
hipError_t launch_ckr(const FwdArgs<T> &a, dim3 grid, hipStream_t st) {
    constexpr bool one = one_wave_blocks<T, CT, STATS>();
    const dim3 block(kTileW, one ? 1 : kTileH);
    if (one) {
        // (a batch of 2^29 tiles of twelve 16-bit channels would take some
        // 30 TB: never reached, but the block index must stay an int)
        if (grid.x >= (1u << 29)) return hipErrorInvalidValue;
        grid.x *= kTileH;
    }
    switch (a.k) {
    case 1: hipLaunchKernelGGL((warp_forward_kernel<T, CT, 1, REC, STATS>), grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL((warp_forward_kernel<T, CT, 2, REC, STATS>), grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL((warp_forward_kernel<T, CT, 3, REC, STATS>), grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL((warp_forward_kernel<T, CT, 4, REC, STATS>), grid, block, 0, st, a); break;
    }
    return hipGetLastError();
}

template <typename T, int CT>
hipError_t launch_ck(const FwdArgs<T> &a, dim3 grid, hipStream_t st) {
    if (!a.boxes) return launch_ckr<T, CT, false, false>(a, grid, st);
    return a.stat_parts ? launch_ckr<T, CT, true, true>(a, grid, st)
                        : launch_ckr<T, CT, true, false>(a, grid, st);
}

// Whether the specialised kernel (which can record the footprint) serves C.
bool specialised(int c, int w) { return w >= 2 && (c == 1 || c == 3 || c == 4 || c == 12); }

template <typename T>
hipError_t launch_typed(const void *src, const float *mv, const WarpShape &s, void *out,
                        uint8_t *mask, uint32_t *count, const BwdWorkspace *rec,
                        hipStream_t st) {
    FwdArgs<T> a = make_args<T>(src, mv, s, out, mask, count);
    if (rec) {
        a.boxes = reinterpret_cast<Box *>(rec->boxes);
        a.offs = reinterpret_cast<SegOffsets *>(a.boxes + static_cast<size_t>(s.n) * s.h * a.segs);
        a.info_words = reinterpret_cast<uint32_t *>(rec->info);
        if (rec->stat_parts) {
            const StatsRegion r = stats_region(rec->stat_parts, s.n, s.h, s.w);
            a.stat_parts = r.parts;
            a.stat_counters = r.counters;
        }
    }
    const dim3 grid(static_cast<unsigned>(static_cast<int64_t>(a.tiles_x) * a.tiles_y * s.n));
    if (specialised(s.c, s.w)) {
        switch (s.c) {
        case 1: return launch_ck<T, 1>(a, grid, st);
        case 3: return launch_ck<T, 3>(a, grid, st);
        case 4: return launch_ck<T, 4>(a, grid, st);
        case 12: return launch_ck<T, 12>(a, grid, st);
        default: break;
        }
    }
    hipLaunchKernelGGL(warp_forward_generic_kernel<T>, grid, dim3(kTileW, kTileH), 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_zero_u32(uint32_t *p, int64_t count, hipStream_t stream) {
    int64_t blocks = (count + 255) / 256;
    blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       p, count);
    return hipGetLastError();
}

hipError_t launch_forward(int dtype, const void *src, const float *mv, const WarpShape &s,
                          void *out, uint8_t *mask, uint32_t *count, hipStream_t stream) {
    if (count) {
        hipError_t e = launch_zero_u32(count, static_cast<int64_t>(s.n) * s.k, stream);
        if (e != hipSuccess) return e;
    }
    switch (dtype) {
    case 0: return launch_typed<float>(src, mv, s, out, mask, count, nullptr, stream);
    case 1: return launch_typed<_Float16>(src, mv, s, out, mask, count, nullptr, stream);
    default: return launch_typed<__bf16>(src, mv, s, out, mask, count, nullptr, stream);
    }
}

size_t record_stats_bytes(int n, int h, int w) {
    return stats_region(nullptr, n, h, w).bytes;
}

hipError_t launch_forward_record(int dtype, const void *src, const float *mv, const WarpShape &s,
                                 void *out, uint8_t *mask, uint32_t *count,
                                 const BwdWorkspace &ws, double *motion_stats,
                                 hipStream_t stream) {
    const StatsRegion r = stats_region(ws.stat_parts, s.n, s.h, s.w);
    if (!backward_uses_footprint(s.c) || !specialised(s.c, s.w)) {
        // the adjoint reads no records, or the kernel that serves this shape
        // does not write them: the plain forward, then the footprint pass
        // (and the statistics pass)
        hipError_t e = launch_forward(dtype, src, mv, s, out, mask, count, stream);
        if (e == hipSuccess && backward_uses_footprint(s.c)) e = launch_footprint(mv, s, ws, stream);
        if (e != hipSuccess || !motion_stats) return e;
        e = launch_motion_moments(mv, s.n, s.h, s.w, r.parts, stream);
        if (e != hipSuccess) return e;
        return launch_motion_stats_fold(r.parts, s.n, motion_stats_parts(s.h, s.w), motion_stats,
                                        stream);
    }
    hipError_t e = count ? launch_zero_u32(count, static_cast<int64_t>(s.n) * s.k, stream)
                         : hipSuccess;
    if (e != hipSuccess) return e;
    BwdWorkspace rec = ws;
    if (!motion_stats) rec.stat_parts = nullptr;  // the instantiation without statistics
    switch (dtype) {
    case 0: e = launch_typed<float>(src, mv, s, out, mask, count, &rec, stream); break;
    case 1: e = launch_typed<_Float16>(src, mv, s, out, mask, count, &rec, stream); break;
    default: e = launch_typed<__bf16>(src, mv, s, out, mask, count, &rec, stream); break;
    }
    if (e != hipSuccess) return e;
    if (!motion_stats) return launch_frame_reach(s, ws, nullptr, stream);
    // the tile partials are folded inside the reduction of the footprint records
    const TileFold fold{r.parts, r.tiles, r.slots, r.counters, motion_stats};
    return launch_frame_reach(s, ws, &fold, stream);
}

}  // namespace exw
