// N_D of the state vector on CDNA4 (gfx950): the number of dynamic objects
// in a frame, as the connected components of the pixels its custom stencil
// buffer marks (paper §III-D: the stencil buffer captures the dynamic
// objects, which are found by clustering it; Table IV: N_D; §IV-C, Eq. 1: an
// entry of E_t). A pixel is marked iff its stencil value is non-zero; two
// marked pixels are joined when they share an edge (4-connectivity) or an
// edge or a corner (8-connectivity).
//
// Pass 1, one workgroup per 32 x 32 tile: union-find over the tile in LDS.
// Each pixel starts labelled with the first pixel of its run of marked
// pixels in the row (a wavefront ballot), so only links between rows are
// made, once per stretch where two rows touch. Labels are in-tile indices;
// a union links the larger root under the smaller with an LDS atomicMin and
// retries from the old parent when another lane linked it first, so every
// label points to a smaller or equal index and every find ends. Each pixel then stores the frame-wide index of its
// tile root, and the tile adds its number of roots to the frame's count.
// Pass 2, one workgroup per tile: the tile's right column and bottom row are
// joined to their neighbours across the border with the same union-find in
// global memory (agent-scope atomics and loads), under the same rules for
// skipping implied links, and every link that joins two sets subtracts one
// from the count. The count is the number of sets
// left whatever the order of the links, so it is exact.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.h"

namespace exw {
namespace {

constexpr int kCcTile = 32;                     // tile edge (pixels)
constexpr int kCcThreads = 256;                 // pass 1: four pixels per thread
constexpr int kCcRows = kCcTile * kCcTile / kCcThreads;

__device__ __forceinline__ int lds_load(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int lds_find(const int *lab, int x) {
    for (int p = lds_load(lab + x); p != x; p = lds_load(lab + x)) x = p;
    return x;
}

__device__ __forceinline__ void lds_union(int *lab, int a, int b) {
    for (;;) {
        a = lds_find(lab, a);
        b = lds_find(lab, b);
        if (a == b) return;
        const int hi = a > b ? a : b, lo = a > b ? b : a;
        const int old = atomicMin(lab + hi, lo);
        if (old == hi) return;  // hi was a root: linked
        a = old;                // hi had been linked meanwhile: join its parent too
        b = lo;
    }
}

__device__ __forceinline__ int g_load(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int g_find(const int *lab, int x) {
    for (int p = g_load(lab + x); p != x; p = g_load(lab + x)) x = p;
    return x;
}

// Returns the number of links that joined two sets (0 or 1).
__device__ __forceinline__ int g_union(int *lab, int a, int b) {
    for (;;) {
        a = g_find(lab, a);
        b = g_find(lab, b);
        if (a == b) return 0;
        const int hi = a > b ? a : b, lo = a > b ? b : a;
        const int old = __hip_atomic_fetch_min(lab + hi, lo, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
        if (old == hi) return 1;
        a = old;
        b = lo;
    }
}

struct CcArgs {
    const uint8_t *stencil;  // [N][H][W]
    int *labels;             // [N][H][W] frame-wide indices, -1 where unmarked
    uint32_t *count;         // [N], zero on entry to pass 1
    int h, w, tiles_x, tiles_per_frame;
    int eight;               // 8-connectivity
};

__global__ __launch_bounds__(kCcThreads) void cc_tile_kernel(CcArgs a) {
    __shared__ int lab[kCcTile * kCcTile];
    __shared__ int roots[kCcThreads / 64];
    const int frame = static_cast<int>(blockIdx.x) / a.tiles_per_frame;
    const int tile = static_cast<int>(blockIdx.x) - frame * a.tiles_per_frame;
    const int x0 = (tile % a.tiles_x) * kCcTile, y0 = (tile / a.tiles_x) * kCcTile;
    const int64_t hw = static_cast<int64_t>(a.h) * a.w;
    const uint8_t *st = a.stencil + frame * hw;
    const int col = threadIdx.x % kCcTile;
    const int row0 = threadIdx.x / kCcTile;  // rows row0 + 8 j
    // The rows' stencil bytes are loaded first, all in flight (a pixel past
    // the frame's edge reads the edge pixel and is unmarked): a load inside
    // the bounds test would be waited for before the next one issues.
    bool mk[kCcRows];
    uint8_t sv[kCcRows];
#pragma unroll
    for (int j = 0; j < kCcRows; ++j) {
        const int r = row0 + j * (kCcThreads / kCcTile);
        const int x = min(x0 + col, a.w - 1), y = min(y0 + r, a.h - 1);
        sv[j] = st[static_cast<int64_t>(y) * a.w + x];
    }
#pragma unroll
    for (int j = 0; j < kCcRows; ++j) {
        const int r = row0 + j * (kCcThreads / kCcTile);
        const int x = x0 + col, y = y0 + r;
        mk[j] = x < a.w && y < a.h && sv[j] != 0;
        // A wavefront holds two whole tile rows (lanes 0..31, 32..63): each
        // marked pixel starts labelled with the first pixel of its run of
        // marked pixels in the row, so runs need no links of their own.
        const unsigned long long both = __ballot(mk[j]);
        const uint32_t bits = __lane_id() < kCcTile ? static_cast<uint32_t>(both)
                                                    : static_cast<uint32_t>(both >> kCcTile);
        const uint32_t gaps = ~bits & ((1u << col) - 1u);  // unmarked pixels left of this one
        const int start = gaps ? kCcTile - __clz(gaps) : 0;
        lab[r * kCcTile + col] = mk[j] ? r * kCcTile + start : -1;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kCcRows; ++j) {
        const int r = row0 + j * (kCcThreads / kCcTile);
        if (!mk[j] || r + 1 >= kCcTile) continue;
        const int i = r * kCcTile + col;
        // Links to the row below, made once per stretch where the two rows
        // touch: below at the stretch's first column (the pixel whose left
        // and lower-left neighbours are not both marked), a diagonal only
        // where neither the pixel beside nor the pixel below is marked. A
        // neighbour is marked iff its label is not -1 (labels stay >= 0).
        const bool lf = col > 0 && lds_load(lab + i - 1) >= 0;
        const bool rt = col + 1 < kCcTile && lds_load(lab + i + 1) >= 0;
        const bool dn = lds_load(lab + i + kCcTile) >= 0;
        const bool dl = col > 0 && lds_load(lab + i + kCcTile - 1) >= 0;
        const bool dr = col + 1 < kCcTile && lds_load(lab + i + kCcTile + 1) >= 0;
        if (dn && !(lf && dl)) lds_union(lab, i, i + kCcTile);
        if (a.eight) {
            if (dl && !dn && !lf) lds_union(lab, i, i + kCcTile - 1);
            if (dr && !dn && !rt) lds_union(lab, i, i + kCcTile + 1);
        }
    }
    __syncthreads();
    int mine = 0;
#pragma unroll
    for (int j = 0; j < kCcRows; ++j) {
        const int r = row0 + j * (kCcThreads / kCcTile);
        const int x = x0 + col, y = y0 + r;
        if (x >= a.w || y >= a.h) continue;
        int out = -1;
        if (mk[j]) {
            const int root = lds_find(lab, r * kCcTile + col);
            mine += root == r * kCcTile + col;
            out = (y0 + root / kCcTile) * a.w + x0 + root % kCcTile;  // <= this pixel's index
        }
        a.labels[frame * hw + static_cast<int64_t>(y) * a.w + x] = out;
    }
    // the tile's roots, one atomic per workgroup
    for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
    if (__lane_id() == 0) roots[threadIdx.x / 64] = mine;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int k = 0; k < kCcThreads / 64; ++k) t += roots[k];
        if (t) atomicAdd(a.count + frame, static_cast<uint32_t>(t));
    }
}

// 64 threads per tile: 0..31 its right column, 32..63 its bottom row.
__global__ __launch_bounds__(64) void cc_border_kernel(CcArgs a) {
    const int frame = static_cast<int>(blockIdx.x) / a.tiles_per_frame;
    const int tile = static_cast<int>(blockIdx.x) - frame * a.tiles_per_frame;
    const int x0 = (tile % a.tiles_x) * kCcTile, y0 = (tile / a.tiles_x) * kCcTile;
    const int64_t hw = static_cast<int64_t>(a.h) * a.w;
    int *lab = a.labels + frame * hw;
    const uint8_t *st = a.stencil + frame * hw;
    const int t = threadIdx.x;
    int x, y;
    if (t < kCcTile) { x = x0 + kCcTile - 1; y = y0 + t; }         // right column
    else { x = x0 + (t - kCcTile); y = y0 + kCcTile - 1; }          // bottom row
    // Whether a pixel is marked never changes: it is read from the stencil,
    // which the caches may serve (only the union-find needs coherent loads).
    // The six pixels a thread may test are loaded first, all in flight
    // (clamped to the frame; those outside it are unmarked): a load inside
    // the tests would be waited for before the next one issues. Right
    // column: (x, y), (x+1, y), (x, y-1), (x+1, y-1), (x, y+1), (x+1, y+1);
    // bottom row: (x, y), (x, y+1), (x-1, y), (x-1, y+1), (x+1, y),
    // (x+1, y+1).
    const bool rc = t < kCcTile;
    bool m[6];
    {
        uint8_t v[6];
        int mx[6], my[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const int side = k < 2 ? 0 : (k < 4 ? -1 : 1);
            const int dx = rc ? (k & 1) : side;
            const int dy = rc ? side : (k & 1);
            mx[k] = x + dx;
            my[k] = y + dy;
            v[k] = st[min(max(my[k], 0), a.h - 1) * a.w + min(max(mx[k], 0), a.w - 1)];
        }
#pragma unroll
        for (int k = 0; k < 6; ++k)
            m[k] = mx[k] >= 0 && mx[k] < a.w && my[k] >= 0 && my[k] < a.h && v[k] != 0;
    }
    int joined = 0;
    if (m[0]) {
        const int p = y * a.w + x;
        auto link = [&](int nx, int ny) { joined += g_union(lab, p, ny * a.w + nx); };
        // A link that the border's other links imply is skipped (the same
        // rules as inside the tiles, along the border).
        if (rc) {  // across the right border
            const bool rn = m[1], up = m[2], ru = m[3];
            if (rn && !(t > 0 && up && ru)) link(x + 1, y);
            if (a.eight) {
                if (ru && !rn && !up) link(x + 1, y - 1);
                if (!rn && !m[4] && m[5]) link(x + 1, y + 1);
            }
        } else {   // across the bottom border
            const bool dn = m[1], lf = m[2], dl = m[3];
            if (dn && !(t > kCcTile && lf && dl)) link(x, y + 1);
            if (a.eight) {
                if (dl && !dn && !lf) link(x - 1, y + 1);
                if (!dn && !m[4] && m[5]) link(x + 1, y + 1);
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) joined += __shfl_xor(joined, off);
    if (t == 0 && joined) atomicSub(a.count + frame, static_cast<uint32_t>(joined));
}

}  // namespace

size_t dynamic_objects_workspace_bytes(int n, int h, int w) {
    return sizeof(int) * static_cast<size_t>(n) * h * w;
}

hipError_t launch_dynamic_objects(const uint8_t *stencil, int n, int h, int w, int connectivity,
                                  uint32_t *count, void *workspace, hipStream_t stream) {
    hipError_t e = launch_zero_u32(count, n, stream);
    if (e != hipSuccess) return e;
    CcArgs a;
    a.stencil = stencil;
    a.labels = static_cast<int *>(workspace);
    a.count = count;
    a.h = h;
    a.w = w;
    a.tiles_x = (w + kCcTile - 1) / kCcTile;
    a.tiles_per_frame = a.tiles_x * ((h + kCcTile - 1) / kCcTile);
    a.eight = connectivity == 8;
    const dim3 grid(static_cast<unsigned>(static_cast<int64_t>(n) * a.tiles_per_frame));
    hipLaunchKernelGGL(cc_tile_kernel, grid, dim3(kCcThreads), 0, stream, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(cc_border_kernel, grid, dim3(64), 0, stream, a);
    return hipGetLastError();
}

}  // namespace exw
