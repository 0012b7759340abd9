// Internal declarations shared by the HIP translation units of liborca.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/orca.h"

namespace orca {

constexpr int kWave = 64;
constexpr int kBboxBlocks = 1024;   // partial bounding boxes per scene (max)
constexpr int kScanTile = 2048;     // cells per scan tile (256 threads x 8)
constexpr int kAlign = 256;

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
    size_t meta, partial, cell, rank, count, start, tiles, s0, s1, total;
    int64_t n, n_scenes, max_cells, n_tiles;
};

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

Layout make_layout(int64_t n, int64_t n_scenes, int64_t max_cells);

inline int64_t default_max_cells(int64_t n) { return n * 2 > 4096 ? n * 2 : 4096; }

// Device pointers into one workspace.
struct Work {
    GridMeta *meta;
    float4 *partial;
    uint32_t *cell;
    uint32_t *rank;
    uint32_t *count;
    uint32_t *start;
    uint32_t *tiles;
    float4 *s0;   // cell order: (px, py, bits(caller index), radius)
    float4 *s1;   // cell order: (vx, vy, bits(class), 0)
};

Work bind(const Layout &L, void *ws);

// Grid build for one scene: bounding box, cell keys, counting sort, SoA
// gather into cell order.  Returns hipSuccess or the launch error.
hipError_t launch_grid_build(const orca_agents_in &in, int n, const orca_params &p,
                             const Layout &L, const Work &w, hipStream_t stream);

// Fused neighbour search + half-planes + LP + update for one scene.
hipError_t launch_step(const orca_agents_in &in, const orca_agents_out &out, int n,
                       const orca_params &p, const Layout &L, const Work &w, hipStream_t stream);

// Neighbour lists only (caller order), for orca_build_grid.
hipError_t launch_knn_export(const orca_agents_in &in, int n, const orca_params &p,
                             const Layout &L, const Work &w, int32_t *nbr, int32_t *cnt,
                             hipStream_t stream);

hipError_t launch_fill_zero(void *ws, size_t bytes, hipStream_t stream);

}  // namespace orca
