// Uniform-grid build for one scene: bounding box -> cell keys -> counting sort
// -> cell-ordered SoA copy.  The grid only bounds which agents are examined as
// neighbour candidates (Sec. 1 and Sec. 3 use a grid spatial partition for
// the "nearby agents" query); the neighbour set itself is defined exactly
// and does not depend on the cell size.
#include "orca_internal.h"

#include <math.h>

namespace orca {

namespace {

constexpr int kBlock = 256;
// Crowds whose bounding box takes at most this many blocks of (1) form the
// grid geometry inside (3) (see k_cell_count).
constexpr int kFusedParts = 128;

// (1) partial bounding boxes; also clears the cell histogram for (3).
__global__ __launch_bounds__(kBlock) void k_bbox_partial(const float *__restrict__ px,
                                                         const float *__restrict__ py, int n,
                                                         float4 *__restrict__ partial,
                                                         uint32_t *__restrict__ count,
                                                         int count_len)
{
    float4 b = make_float4(INFINITY, INFINITY, -INFINITY, -INFINITY);
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const float x = px[i], y = py[i];
        b.x = fminf(b.x, x);
        b.y = fminf(b.y, y);
        b.z = fmaxf(b.z, x);
        b.w = fmaxf(b.w, y);
    }
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < count_len; c += stride) count[c] = 0u;
    b = block_bbox<kBlock>(b);
    if (threadIdx.x == 0) partial[blockIdx.x] = b;
}

// (2) one block: final bounding box and grid geometry (grid_geometry).
__global__ __launch_bounds__(kBlock) void k_grid_setup(const float4 *__restrict__ partial,
                                                       int n_partial, float rn, float cs_req,
                                                       int max_cells, int n,
                                                       const float *__restrict__ rn_dev,
                                                       GridMeta *__restrict__ meta)
{
    if (rn_dev) rn = *rn_dev;
    float4 b = make_float4(INFINITY, INFINITY, -INFINITY, -INFINITY);
    for (int k = threadIdx.x; k < n_partial; k += kBlock) {
        const float4 q = partial[k];
        b.x = fminf(b.x, q.x);
        b.y = fminf(b.y, q.y);
        b.z = fmaxf(b.z, q.z);
        b.w = fmaxf(b.w, q.w);
    }
    b = block_bbox<kBlock>(b);
    if (threadIdx.x != 0) return;
    GridMeta g;
    grid_geometry(b, rn, cs_req, max_cells, g);
    g.cell_base = 0;
    g.agent_base = 0;
    g.n = n;
    g.seg_end = (uint32_t)n;
    *meta = g;
}

// (3) cell key and rank inside the cell (atomic counting).  With `partial`
// (small crowds, at most kFusedParts boxes from (1)) every block also does
// (2) itself: it combines the boxes and forms the geometry (grid_geometry,
// the same bits in every block), and block 0 stores it for the kernels
// after this one; a crowd of 16,384 agents then saves the one-block launch.
// Without it (large crowds, whose (1) runs many more blocks than a block of
// (3) could combine cheaply) the geometry comes from (2) through `meta`.
__global__ __launch_bounds__(kBlock) void k_cell_count(const float *__restrict__ px,
                                                       const float *__restrict__ py, int n,
                                                       const float4 *__restrict__ partial,
                                                       int n_partial, float rn, float cs_req,
                                                       int max_cells,
                                                       const float *__restrict__ rn_dev,
                                                       GridMeta *__restrict__ meta,
                                                       uint32_t *__restrict__ cell,
                                                       uint32_t *__restrict__ rank,
                                                       uint32_t *__restrict__ count)
{
    GridMeta g;
    if (partial) {
        __shared__ GridMeta gs;
        float4 b = make_float4(INFINITY, INFINITY, -INFINITY, -INFINITY);
        for (int k = threadIdx.x; k < n_partial; k += kBlock) {
            const float4 q = partial[k];
            b.x = fminf(b.x, q.x);
            b.y = fminf(b.y, q.y);
            b.z = fmaxf(b.z, q.z);
            b.w = fmaxf(b.w, q.w);
        }
        b = block_bbox<kBlock>(b);
        if (threadIdx.x == 0) {
            GridMeta h;
            grid_geometry(b, rn_dev ? *rn_dev : rn, cs_req, max_cells, h);
            h.cell_base = 0;
            h.agent_base = 0;
            h.n = n;
            h.seg_end = (uint32_t)n;
            gs = h;
            if (blockIdx.x == 0) *meta = h;
        }
        __syncthreads();
        g = gs;
    } else {
        g = *meta;
    }
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int cx = cell_axis(px[i], g.x0, g.inv_cs, g.nx);
    const int cy = cell_axis(py[i], g.y0, g.inv_cs, g.ny);
    const uint32_t c = (uint32_t)(cx + g.nx * cy);
    cell[i] = c;
    rank[i] = atomicAdd(&count[c], 1u);
}

constexpr int kPer = kScanTile / kBlock;  // 8 cells per thread

// (4a) per-tile sums of the histogram.
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t *__restrict__ count,
                                                        const GridMeta *__restrict__ meta,
                                                        uint32_t *__restrict__ tiles)
{
    const int n_cells = meta->n_cells;
    const int base = blockIdx.x * kScanTile;
    if (base >= n_cells) return;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int c = base + threadIdx.x * kPer + k;
        if (c < n_cells) s += count[c];
    }
    uint32_t tot;
    block_excl_scan<kBlock>(s, &tot);
    if (threadIdx.x == 0) tiles[blockIdx.x] = tot;
}

// (4b) exclusive scan inside each tile, offset by the tile's prefix: the sum
// of the tile sums of (4a) before it, which every block adds up itself (at
// most a few thousand words from L2, in place of a one-block scan kernel
// between the two).
__global__ __launch_bounds__(kBlock) void k_scan_apply(const uint32_t *__restrict__ count,
                                                       const uint32_t *__restrict__ tiles,
                                                       const GridMeta *__restrict__ meta,
                                                       uint32_t *__restrict__ start)
{
    const GridMeta g = *meta;
    const int base = blockIdx.x * kScanTile;
    if (base >= g.n_cells) return;
    uint32_t before = 0;
    for (int t = threadIdx.x; t < (int)blockIdx.x; t += kBlock) before += tiles[t];
    uint32_t prefix;
    block_excl_scan<kBlock>(before, &prefix);
    uint32_t v[kPer];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int c = base + threadIdx.x * kPer + k;
        v[k] = c < g.n_cells ? count[c] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = prefix + block_excl_scan<kBlock>(s, &tot);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int c = base + threadIdx.x * kPer + k;
        if (c < g.n_cells) start[c] = run;
        run += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) start[g.n_cells] = (uint32_t)g.n;
}

// A velocity within the speed cap: (vx, vy) itself when |v| <= v_max (the
// test in double from the FP32 values, products exact), else scaled onto the
// cap and rounded to FP32, then moved toward zero one ulp at a time until the
// test holds.  The ORCA lines an agent takes no responsibility for (f = 0)
// all pass through its own velocity; a velocity the previous step left on
// the speed circle lies outside it by a few FP32 ulps half of the time, and
// the LP's feasible set around that apex would then be thinner than FP32
// resolves.  Inside the cap, the apex is a feasible point exactly.
__device__ __forceinline__ void cap_velocity(float &vx, float &vy, float vmax)
{
    const double vm2 = (double)vmax * (double)vmax;
    const double d = (double)vx * (double)vx + (double)vy * (double)vy;
    if (!(d > vm2)) return;
    const double s = (double)vmax / sqrt(d);
    float x = (float)((double)vx * s), y = (float)((double)vy * s);
    for (int it = 0; it < 16 && (double)x * (double)x + (double)y * (double)y > vm2; ++it) {
        if (fabsf(x) >= fabsf(y))
            x = nextafterf(x, 0.0f);
        else
            y = nextafterf(y, 0.0f);
    }
    vx = x;
    vy = y;
}

// (5) scatter into cell order: position = start[cell] + rank; velocities
// taken within the speed cap (cap_velocity).
__global__ __launch_bounds__(kBlock) void k_scatter(orca_agents_in in, int n,
                                                    const uint32_t *__restrict__ cell,
                                                    const uint32_t *__restrict__ rank,
                                                    const uint32_t *__restrict__ start,
                                                    float4 *__restrict__ s0,
                                                    float4 *__restrict__ s1)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t pos = start[cell[i]] + rank[i];
    if (pos >= (uint32_t)n) return;  // cannot happen for a consistent histogram
    s0[pos] = make_float4(in.px[i], in.py[i], __int_as_float(i), in.radius[i]);
    float vx = in.vx[i], vy = in.vy[i];
    cap_velocity(vx, vy, in.max_speed[i]);
    s1[pos] = make_float4(vx, vy, __int_as_float((int)in.cls[i]), 0.0f);
}

__global__ void k_fill_zero(uint4 *p, size_t n16)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n16; k += stride)
        p[k] = make_uint4(0, 0, 0, 0);
}

}  // namespace

hipError_t launch_grid_build(const orca_agents_in &in, int n, const orca_params &p,
                             const Layout &L, const Work &w, hipStream_t stream)
{
    return launch_grid_build_rn(in, n, p.neighbor_dist, p.cell_size, nullptr, L, w, stream);
}

hipError_t launch_grid_build_rn(const orca_agents_in &in, int n, float rn, float cell_size,
                                const float *rn_dev, const Layout &L, const Work &w,
                                hipStream_t stream)
{
    const int nb = (int)((n + kBlock - 1) / kBlock);
    const int nbb = nb < kBboxBlocks ? nb : kBboxBlocks;
    const int count_len = (int)L.max_cells;
    hipLaunchKernelGGL(k_bbox_partial, dim3(nbb), dim3(kBlock), 0, stream, in.px, in.py, n,
                       w.partial, w.count, count_len);
    const bool fused = nbb <= kFusedParts;
    if (!fused)
        hipLaunchKernelGGL(k_grid_setup, dim3(1), dim3(kBlock), 0, stream, w.partial, nbb, rn,
                           cell_size, count_len, n, rn_dev, w.meta);
    hipLaunchKernelGGL(k_cell_count, dim3(nb), dim3(kBlock), 0, stream, in.px, in.py, n,
                       fused ? w.partial : nullptr, nbb, rn, cell_size, count_len, rn_dev, w.meta,
                       w.cell, w.rank, w.count);
    return launch_scan_scatter(in, n, L, w, w.meta, stream);
}

hipError_t launch_scan_scatter(const orca_agents_in &in, int n, const Layout &L, const Work &w,
                               const GridMeta *scan_meta, hipStream_t stream)
{
    const int nb = (int)((n + kBlock - 1) / kBlock);
    const int nt = (int)L.n_tiles;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nt), dim3(kBlock), 0, stream, w.count, scan_meta,
                       w.tiles);
    hipLaunchKernelGGL(k_scan_apply, dim3(nt), dim3(kBlock), 0, stream, w.count, w.tiles,
                       scan_meta, w.start);
    hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kBlock), 0, stream, in, n, w.cell, w.rank,
                       w.start, w.s0, w.s1);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *ws, size_t bytes, hipStream_t stream)
{
    const size_t n16 = bytes / 16;
    if (n16) {
        size_t blocks = (n16 + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, stream, (uint4 *)ws,
                           n16);
    }
    return hipGetLastError();
}

}  // namespace orca
