// Batched ORCA step: many independent scenes of uneven sizes advanced by one
// set of launches per step (batched form; not in the paper, which simulates
// one scene).
//
// Scene s owns caller indices [off[s], off[s+1]) and the cells
// [2 off[s] + 64 s, 2 off[s+1] + 64 (s+1)) of one global cell space, so a
// single histogram, scan and scatter order every scene at once and each scene
// stays contiguous in cell order (its agents fill exactly the positions
// [off[s], off[s+1])).  Agents of different scenes never share a cell and so
// never see each other.
//
// The step kernel is persistent: a grid sized to the device's occupancy
// whose wavefronts pop 64-agent tiles from eight queues, one per XCD (each
// over a contiguous range of tiles, so neighbouring agents stay in one L2),
// and steal from the other queues once their own is drained.  Every queue is
// a monotone counter, so every wavefront exits.
#include "orca_device.h"

namespace orca {
namespace {

constexpr int kBlock = 256;
constexpr int kStepBlock = 128;
constexpr int kTile = 64;

// Scene of caller index i: the largest s with off[s] <= i (off ascending).
__device__ __forceinline__ int scene_of(const int32_t *__restrict__ off, int S, int i)
{
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= i)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int clamp_off(int v, int n) { return v < 0 ? 0 : (v > n ? n : v); }

// Scene of caller index i given the scene s0 of an index <= i (off
// ascending): a walk forward from s0, a step or two for the indices of one
// tile, instead of a binary search per index.
__device__ __forceinline__ int scene_from(const int32_t *__restrict__ off, int S, int s0, int i)
{
    int s = s0;
    while (s + 1 < S && off[s + 1] <= i) ++s;
    return s;
}

// (1) kBboxSplit blocks per scene: partial bounding boxes of its agents (a
// block per scene left the largest scenes to one block each).  All blocks
// also clear the histogram and block 0 the tile queues; scene offsets and
// parameters are checked and any violation is flagged (the kernels stay in
// bounds regardless: offsets are clamped to [0, n]).
__global__ __launch_bounds__(kBlock) void k_batch_bbox(const float *__restrict__ px,
                                                       const float *__restrict__ py, int n,
                                                       const int32_t *__restrict__ off, int S,
                                                       const orca_params *__restrict__ prm,
                                                       float4 *__restrict__ partial,
                                                       uint32_t *__restrict__ count, int count_len,
                                                       uint32_t *__restrict__ queue,
                                                       int32_t *__restrict__ error_flag,
                                                       int has_accel)
{
    const int s = blockIdx.x / kBboxSplit, part = blockIdx.x % kBboxSplit;
    const int a = clamp_off(off[s], n), b = clamp_off(off[s + 1], n);
    float4 bb = make_float4(INFINITY, INFINITY, -INFINITY, -INFINITY);
    for (int i = a + part * kBlock + threadIdx.x; i < b; i += kBlock * kBboxSplit) {
        const float x = px[i], y = py[i];
        bb.x = fminf(bb.x, x);
        bb.y = fminf(bb.y, y);
        bb.z = fmaxf(bb.z, x);
        bb.w = fmaxf(bb.w, y);
    }
    const int stride = gridDim.x * kBlock;
    for (int c = blockIdx.x * kBlock + threadIdx.x; c < count_len; c += stride) count[c] = 0u;
    if (s == 0 && threadIdx.x < kXcds) queue[threadIdx.x] = 0u;
    bb = block_bbox<kBlock>(bb);
    if (threadIdx.x == 0) {
        partial[blockIdx.x] = bb;
        if (error_flag && part == 0) {
            const orca_params p = prm[s];
            bool bad = off[s] > off[s + 1] || off[s] < 0 || off[s + 1] > n;
            if (s == 0) bad = bad || off[0] != 0;
            if (s == S - 1) bad = bad || off[S] != n;
            bad = bad || !(p.dt > 0.0f) || !(p.time_horizon > 0.0f) ||
                  !(p.neighbor_dist > 0.0f) || !(p.cell_size >= 0.0f) ||
                  p.max_neighbors < 1 || p.max_neighbors > ORCA_K_MAX ||
                  (p.pref_is_goal != 0 && p.pref_is_goal != 1) ||
                  !(p.accel[0] >= 0.0f) || !(p.accel[1] >= 0.0f) ||
                  !isfinite(p.accel[0]) || !isfinite(p.accel[1]) ||
                  !(p.turn[0] >= 0.0f) || !(p.turn[1] >= 0.0f) ||
                  !isfinite(p.turn[0]) || !isfinite(p.turn[1]) ||
                  (!has_accel && (p.accel[0] > 0.0f || p.accel[1] > 0.0f ||
                                  p.turn[0] > 0.0f || p.turn[1] > 0.0f));
            if (bad) atomicOr(error_flag, 1);
        }
    }
}

// (2) one thread per scene: grid geometry within the scene's cell budget.
// meta[S] describes the whole cell space for the scan.
__global__ __launch_bounds__(kBlock) void k_batch_setup(const float4 *__restrict__ partial,
                                                        const int32_t *__restrict__ off, int S,
                                                        int n, const orca_params *__restrict__ prm,
                                                        GridMeta *__restrict__ meta)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    if (s == 0) {
        GridMeta g{};
        g.n_cells = (int)batched_cells(n, S);
        g.n = n;
        g.seg_end = (uint32_t)n;
        meta[S] = g;
    }
    if (s >= S) return;
    const int a = clamp_off(off[s], n);
    const int b = max(clamp_off(off[s + 1], n), a);
    const int budget = 2 * (b - a) + 64;
    float4 bb = partial[s * kBboxSplit];
    for (int q = 1; q < kBboxSplit; ++q) {
        const float4 p = partial[s * kBboxSplit + q];
        bb = make_float4(fminf(bb.x, p.x), fminf(bb.y, p.y), fmaxf(bb.z, p.z), fmaxf(bb.w, p.w));
    }
    GridMeta g;
    grid_geometry(bb, prm[s].neighbor_dist, prm[s].cell_size, budget, g);
    // a budget is 2 cells per agent plus 64; the cell ranges of consecutive
    // scenes tile the global cell space when offsets are valid and stay
    // inside it otherwise
    g.cell_base = 2 * a + 64 * s;
    g.agent_base = a;
    g.n = b - a;
    g.seg_end = (uint32_t)b;
    meta[s] = g;
}

// (3) scene, cell and rank inside the cell.
__global__ __launch_bounds__(kBlock) void k_batch_count(const float *__restrict__ px,
                                                        const float *__restrict__ py, int n,
                                                        const int32_t *__restrict__ off, int S,
                                                        const GridMeta *__restrict__ meta,
                                                        uint32_t *__restrict__ cell,
                                                        uint32_t *__restrict__ rank,
                                                        uint32_t *__restrict__ count)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const GridMeta g = meta[scene_of(off, S, i)];
    const int cx = cell_axis(px[i], g.x0, g.inv_cs, g.nx);
    const int cy = cell_axis(py[i], g.y0, g.inv_cs, g.ny);
    const uint32_t c = (uint32_t)(g.cell_base + cx + g.nx * cy);
    cell[i] = c;
    rank[i] = atomicAdd(&count[c], 1u);
}

struct BatchArgs {
    orca_agents_in in;
    orca_agents_out out;
    const GridMeta *meta;
    const orca_params *prm;
    const int32_t *off;
    int S;
    int n;
    const uint32_t *start;
    const float4 *s0;
    const float4 *s1;
    uint32_t *queue;
    float *guess;  // per-agent K-th neighbour distance kept between steps
};

template <int K, int BLOCK, bool ACC>
__device__ __forceinline__ void batch_agent(const BatchArgs &a, int s, int first, float4 *lines,
                                            int tid)
{
    const int sc = scene_from(a.off, a.S, first, s);
    const GridMeta g = a.meta[sc];
    const dev::SceneP p = dev::scene_params(a.prm[sc]);
    // LP3's sub-problem boundaries cached in spare LDS columns: the batch's
    // scenes keep many lanes in LP3 (3.37 -> 3.25 ms per step on the
    // 512-scene batch, the same results bit for bit); on the dense crossing,
    // where LP3 is a small share, the plain kernel is faster without it
    dev::step_agent<K, BLOCK, ACC, false, true>(s, g, p, a.in, a.out, a.start, a.s0, a.s1, lines,
                                                tid, a.guess);
}


// Persistent step: wavefronts pop 64-agent tiles, first from their XCD's
// queue (a contiguous eighth of the tiles), then from the others.
template <int K, int BLOCK, bool ACC>
__global__ __launch_bounds__(BLOCK) void k_step_batched(BatchArgs a)
{
    __shared__ float4 lines[dev::KnnShape<K>::kSlots * BLOCK];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int n_tiles = (a.n + kTile - 1) / kTile;
    const int xcd = blockIdx.x % kXcds;
    for (int v = 0; v < kXcds; ++v) {
        const int x = (xcd + v) % kXcds;
        const int lo = (int)(((int64_t)n_tiles * x) / kXcds);
        const int hi = (int)(((int64_t)n_tiles * (x + 1)) / kXcds);
        for (;;) {
            int t = 0;
            if (lane == 0) t = (int)atomicAdd(&a.queue[x], 1u);
            t = __shfl(t, 0, kWave);
            if (t >= hi - lo) break;
            const int s = (lo + t) * kTile + lane;
            // the tile's first scene, searched once (a wavefront-uniform index)
            const int first = scene_of(a.off, a.S, (lo + t) * kTile);
            if (s < a.n) batch_agent<K, BLOCK, ACC>(a, s, first, lines, tid);
        }
    }
}

// Flat form of the same step: one tile per workgroup wave, XCD-aware order.
template <int K, int BLOCK, bool ACC>
__global__ __launch_bounds__(BLOCK) void k_step_batched_flat(BatchArgs a)
{
    __shared__ float4 lines[dev::KnnShape<K>::kSlots * BLOCK];
    const int tid = threadIdx.x;
    const int s0 = xcd_tile(blockIdx.x, gridDim.x) * BLOCK;
    const int s = s0 + tid;
    if (s < a.n) batch_agent<K, BLOCK, ACC>(a, s, scene_of(a.off, a.S, s0), lines, tid);
}

// Workgroups of k_step_batched that fit the device at once (cached per
// instantiation; multiple of the XCD count).
template <int K, int BLOCK, bool ACC>
int persistent_grid()
{
    static int cached = 0;
    if (cached) return cached;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_batched<K, BLOCK, ACC>, BLOCK,
                                                     0) !=
        hipSuccess)
        return 0;
    int g = cus * (per_cu > 0 ? per_cu : 1);
    g = (g + kXcds - 1) / kXcds * kXcds;
    cached = g;
    return g;
}

template <int K, int BLOCK, bool ACC>
hipError_t launch_step_batched_v(const BatchArgs &a, int mode, hipStream_t stream)
{
    if (mode == 1) {
        const int nb = (a.n + BLOCK - 1) / BLOCK;
        hipLaunchKernelGGL((k_step_batched_flat<K, BLOCK, ACC>), dim3(nb), dim3(BLOCK), 0, stream,
                           a);
        return hipGetLastError();
    }
    const int g = persistent_grid<K, BLOCK, ACC>();
    if (g <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_step_batched<K, BLOCK, ACC>), dim3(g), dim3(BLOCK), 0, stream, a);
    return hipGetLastError();
}

template <int K, int BLOCK>
hipError_t launch_step_batched_b(const BatchArgs &a, int mode, bool acc, hipStream_t stream)
{
    return acc ? launch_step_batched_v<K, BLOCK, true>(a, mode, stream)
               : launch_step_batched_v<K, BLOCK, false>(a, mode, stream);
}

// Workgroup size (one, two or four wavefronts; the LDS column per lane is
// the same, so occupancy differs only through the workgroup granularity).
template <int K>
hipError_t launch_step_batched_k(const BatchArgs &a, int mode, bool acc, int block,
                                 hipStream_t stream)
{
    if (block == 64) return launch_step_batched_b<K, 64>(a, mode, acc, stream);
    if (block == 256) return launch_step_batched_b<K, 256>(a, mode, acc, stream);
    return launch_step_batched_b<K, kStepBlock>(a, mode, acc, stream);
}

}  // namespace

hipError_t launch_batched(const orca_agents_in &in, const orca_agents_out &out, int n,
                          const int32_t *scene_off, int n_scenes, const orca_params *params,
                          int k_max, bool acc, int block, const Layout &L, const Work &w,
                          int32_t *error_flag, int mode, const orca_step_events *ev,
                          hipStream_t stream)
{
    const int S = n_scenes;
    const int nb = (n + kBlock - 1) / kBlock;
    if (ev && ev->grid_begin && hipEventRecord(ev->grid_begin, stream) != hipSuccess)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_bbox, dim3(S * kBboxSplit), dim3(kBlock), 0, stream, in.px, in.py,
                       n, scene_off,
                       S, params, w.partial, w.count, (int)L.max_cells, w.queue, error_flag,
                       acc ? 1 : 0);
    hipLaunchKernelGGL(k_batch_setup, dim3((S + kBlock - 1) / kBlock), dim3(kBlock), 0, stream,
                       w.partial, scene_off, S, n, params, w.meta);
    hipLaunchKernelGGL(k_batch_count, dim3(nb), dim3(kBlock), 0, stream, in.px, in.py, n,
                       scene_off, S, w.meta, w.cell, w.rank, w.count);
    hipError_t e = launch_scan_scatter(in, n, L, w, w.meta + S, stream);
    if (e != hipSuccess) return e;
    BatchArgs a;
    a.in = in;
    a.out = out;
    a.meta = w.meta;
    a.prm = params;
    a.off = scene_off;
    a.S = S;
    a.n = n;
    a.start = w.start;
    a.s0 = w.s0;
    a.s1 = w.s1;
    a.queue = w.queue;
    a.guess = w.guess;
    if (ev && ev->step_begin && hipEventRecord(ev->step_begin, stream) != hipSuccess)
        return hipErrorInvalidValue;
    if (k_max <= 4)
        e = launch_step_batched_k<4>(a, mode, acc, block, stream);
    else if (k_max <= 8)
        e = launch_step_batched_k<8>(a, mode, acc, block, stream);
    else if (k_max <= 10)
        e = launch_step_batched_k<10>(a, mode, acc, block, stream);
    else if (k_max <= 12)
        e = launch_step_batched_k<12>(a, mode, acc, block, stream);
    else if (k_max <= 16)
        e = launch_step_batched_k<16>(a, mode, acc, block, stream);
    else if (k_max <= 20)
        e = launch_step_batched_k<20>(a, mode, acc, block, stream);
    else if (k_max <= 24)
        e = launch_step_batched_k<24>(a, mode, acc, block, stream);
    else
        e = launch_step_batched_k<32>(a, mode, acc, block, stream);
    if (e != hipSuccess) return e;
    if (ev && ev->step_end && hipEventRecord(ev->step_end, stream) != hipSuccess)
        return hipErrorInvalidValue;
    return hipSuccess;
}

}  // namespace orca
