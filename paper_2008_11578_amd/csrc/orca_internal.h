// Internal declarations shared by the HIP translation units of liborca.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/orca.h"

namespace orca {

constexpr int kWave = 64;
constexpr int kBboxBlocks = 1024;   // partial bounding boxes per scene (max)
constexpr int kBboxSplit = 8;      // blocks (partial boxes) per scene of a batch
constexpr int kScanTile = 2048;     // cells per scan tile (256 threads x 8)
constexpr int kAlign = 256;
constexpr int kScanPad = 16;        // float4 entries after the cell-ordered copy s0,
                                    // so candidate groups may read past its end

// Uniform grid of one scene, computed on the device from its bounding box.
struct GridMeta {
    float x0, y0;      // origin (bounding-box minimum)
    float cs;          // effective cell size (>= neighbour distance / m)
    float rn;          // neighbour distance
    int nx, ny;        // cells per axis
    int m;             // stencil radius in cells: in-range pairs are <= m cells apart
    int n_cells;       // nx * ny
    double cs_d;       // cs in double (the value inv_cs was derived from)
    double inv_cs;     // 1 / cs, for the FP64 cell coordinates
    double rn2;        // rn * rn in double (exact)
    int cell_base;     // first global cell id of this scene (batched form)
    int agent_base;    // first agent (caller order) of this scene
    int n;             // agents in this scene
    uint32_t seg_end;  // one past the scene's last cell-order position
};

// Byte offsets of the workspace regions (all 256-byte aligned).
struct Layout {
    size_t meta, partial, queue, cell, rank, count, start, tiles, s0, s1, guess, total;
    int64_t n, n_scenes, max_cells, n_tiles;
};

// Cells of the batched form: 2 per agent + 64 per scene.
__host__ __device__ inline int64_t batched_cells(int64_t n, int64_t n_scenes) { return 2 * n + 64 * n_scenes; }

// Cell coordinate along one axis, in FP64, clamped to [0, ncell - 1]
// (fmax/fmin also map NaN to 0).  Shared by the grid build and the
// neighbour query so that both see identical cells.
__device__ __forceinline__ int cell_axis(float v, float v0, double inv_cs, int ncell)
{
    double c = floor(((double)v - (double)v0) * inv_cs);
    c = fmin(fmax(c, 0.0), (double)(ncell - 1));
    return (int)c;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Remapping dispatch index b to a logical tile so that every XCD works
// on one contiguous range of tiles keeps neighbouring agents (which read each
// other's state) inside one L2.  Bijective on [0, nb).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int q = nb / kXcds, r = nb % kXcds;
    const int x = b % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}

// Inclusive prefix sum over the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x % kWave;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive block scan of one value per thread; returns the exclusive prefix
// and writes the block total to *total (all threads).
template <int BLOCK>
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wsum[BLOCK / kWave];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[wid] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < BLOCK / kWave; ++k) {
        if (k < wid) base += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

// Block-wide (min x, min y, max x, max y).  Result valid in thread 0.
template <int kBlock>
__device__ float4 block_bbox(float4 b)
{
    __shared__ float4 red[kBlock / kWave];
    b.x = wave_min(b.x);
    b.y = wave_min(b.y);
    b.z = wave_max(b.z);
    b.w = wave_max(b.w);
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) red[wid] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBlock / kWave; ++k) {
            b.x = fminf(b.x, red[k].x);
            b.y = fminf(b.y, red[k].y);
            b.z = fmaxf(b.z, red[k].z);
            b.w = fmaxf(b.w, red[k].w);
        }
    }
    return b;
}

// Grid geometry of one scene from its bounding box b = (min x, min y,
// max x, max y):
//   m  = stencil radius in cells, ceil(R_n / requested cell size)
//   cs = max(requested, R_n / m) * (1 + 1e-5), so that m * cs > R_n with a
//        margin far above the rounding of the FP64 cell coordinates
//   the cell size grows (and m is re-derived) until nx * ny <= max_cells;
//   non-finite boxes (NaN/Inf positions) collapse to a single cell.
// Fills every field except cell_base, agent_base, n and seg_end.
__device__ __forceinline__ void grid_geometry(float4 b, float rn, float cs_req, int max_cells,
                                              GridMeta &g)
{
    const bool finite = isfinite(b.x) && isfinite(b.y) && isfinite(b.z) && isfinite(b.w);
    const double w = finite ? (double)b.z - (double)b.x : 0.0;
    const double h = finite ? (double)b.w - (double)b.y : 0.0;
    double c0 = cs_req > 0.0f ? (double)cs_req : (double)rn;
    int m = 1;
    double cs = c0, fx = 0.0, fy = 0.0;
    for (int it = 0; it < 200; ++it) {
        m = (int)ceil((double)rn / c0 - 1e-6);
        if (m < 1) m = 1;
        cs = fmax(c0, (double)rn / m) * (1.0 + 1e-5);
        fx = floor(w / cs) + 1.0;
        fy = floor(h / cs) + 1.0;
        if (fx * fy <= (double)max_cells) break;
        c0 *= 1.25;
    }
    if (!(fx * fy <= (double)max_cells) || !(cs > 0.0)) {
        // only for extents beyond ~1e19 cells or non-positive sizes: one
        // cell holding everything is slow but still exact
        m = 1;
        fx = 1.0;
        fy = 1.0;
        cs = fmax(w, h) + fabs((double)rn) + 1.0;
    }
    g.x0 = finite ? b.x : 0.0f;
    g.y0 = finite ? b.y : 0.0f;
    g.cs = (float)cs;
    g.rn = rn;
    g.nx = (int)fx;
    g.ny = (int)fy;
    g.m = m;
    g.n_cells = g.nx * g.ny;
    g.cs_d = cs;
    g.inv_cs = 1.0 / cs;
    g.rn2 = (double)rn * (double)rn;
}

Layout make_layout(int64_t n, int64_t n_scenes, int64_t max_cells);

inline int64_t default_max_cells(int64_t n) { return n * 2 > 4096 ? n * 2 : 4096; }

// Device pointers into one workspace.
struct Work {
    GridMeta *meta;
    float4 *partial;
    uint32_t *queue;   // 8 tile counters (one per XCD) of the persistent kernel
    uint32_t *cell;
    uint32_t *rank;
    uint32_t *count;
    uint32_t *start;
    uint32_t *tiles;
    float4 *s0;   // cell order: (px, py, bits(caller index), radius)
    float4 *s1;   // cell order: (vx, vy, bits(class), 0)
    float *guess; // caller order: K-th neighbour distance of the last step (0: none)
};

Work bind(const Layout &L, void *ws);

// Grid build for one scene: bounding box, cell keys, counting sort, SoA
// gather into cell order.  Returns hipSuccess or the launch error.
hipError_t launch_grid_build(const orca_agents_in &in, int n, const orca_params &p,
                             const Layout &L, const Work &w, hipStream_t stream);

// The same with the neighbour distance read from device memory when rn_dev
// is not null (a query radius computed on the device).
hipError_t launch_grid_build_rn(const orca_agents_in &in, int n, float rn, float cell_size,
                                const float *rn_dev, const Layout &L, const Work &w,
                                hipStream_t stream);

// Histogram scan and scatter into cell order; scan_meta supplies the number
// of cells (n_cells) and of agents (n) of the whole cell space.
hipError_t launch_scan_scatter(const orca_agents_in &in, int n, const Layout &L, const Work &w,
                               const GridMeta *scan_meta, hipStream_t stream);

// Batched form: many independent scenes, scene s owning caller indices
// [off[s], off[s+1]) and cells [2 off[s] + 64 s, 2 off[s+1] + 64 (s + 1)).
hipError_t launch_batched(const orca_agents_in &in, const orca_agents_out &out, int n,
                          const int32_t *scene_off, int n_scenes, const orca_params *params,
                          int k_max, bool acc, int block, const Layout &L, const Work &w,
                          int32_t *error_flag, int mode, const orca_step_events *ev,
                          hipStream_t stream);

// Fused neighbour search + half-planes + LP + update for one scene; with
// nbr / cnt (nullable) also the neighbour lists the step used.
hipError_t launch_step(const orca_agents_in &in, const orca_agents_out &out, int n,
                       const orca_params &p, const Layout &L, const Work &w, int32_t *nbr,
                       int32_t *cnt, hipStream_t stream);

// Neighbour lists only (caller order), for orca_build_grid.
hipError_t launch_knn_export(const orca_agents_in &in, int n, const orca_params &p,
                             const Layout &L, const Work &w, int32_t *nbr, int32_t *cnt,
                             hipStream_t stream);

hipError_t launch_fill_zero(void *ws, size_t bytes, hipStream_t stream);

// Agent lifecycle (leaving at the goal, entering at clear spawn points).
size_t lifecycle_extra_bytes(int64_t n, int64_t n_cand);
hipError_t launch_remove_arrived(const orca_agents_in &in, const orca_agents_buf &out, int n,
                                 int32_t *n_alive, int32_t *old_to_new, void *extra,
                                 hipStream_t stream);
size_t overlap_extra_bytes(int64_t n);
hipError_t launch_overlap_stats(const orca_agents_in &in, int n, float reach, double *out,
                                const Layout &L, const Work &w, void *extra, hipStream_t stream);
hipError_t launch_spawn(const orca_agents_buf &state, int n, const orca_agents_in &cand,
                        int n_cand, float t_clear, int32_t *n_total, uint8_t *accepted,
                        const Layout &L, const Work &w, void *extra, hipStream_t stream);

// Extra workspace of the adjoint: per-agent tau contributions and the edge
// list (3 per agent) of contributions to neighbours with its transpose.
struct AdjointBufs {
    float *tau_part;     // n
    int32_t *e_tgt;      // 3n: target agent or -1
    float4 *e_val;       // 3n: (gp.x, gp.y, gv.x, gv.y) for the target
    uint32_t *e_rank;    // 3n
    uint32_t *e_list;    // 3n
    uint32_t *e_cnt;     // n
    uint32_t *e_start;   // n
    uint32_t *e_tiles;   // ceil(n / kScanTile) tile sums of the count scan
    double *tau_blocks;  // kTauBlocks partial sums of the tau contributions
};

constexpr int kTauBlocks = 256;

size_t adjoint_extra_bytes(int64_t n);
AdjointBufs bind_adjoint(int64_t n, void *base);

hipError_t launch_adjoint(const orca_agents_in &in, int n, const orca_params &prm,
                          const Layout &L, const Work &w, const AdjointBufs &b,
                          const float *gpx1, const float *gpy1, const float *gvx1,
                          const float *gvy1, float *gpx0, float *gpy0, float *gvx0, float *gvy0,
                          float *gprx, float *gpry, float *g_tau, const orca_step_events *ev,
                          hipStream_t stream);

}  // namespace orca
