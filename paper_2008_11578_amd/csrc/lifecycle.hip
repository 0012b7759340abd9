// Agent lifecycle of the crossing experiments (Sec. 4, first experiment):
// agents leave once they reach their goal, and new agents enter at spawn
// points that keep clear of everyone for a time window.
//
//  - leaving: a stable compaction (per-block counts, one scan block, move),
//    with the arrival test evaluated in double without fused multiply-add so
//    that the decision is exactly reproducible;
//  - entering: candidates are checked against the current agents through a
//    uniform grid whose query radius is computed on the device from the
//    largest radii and speed caps, then against each other: every candidate
//    lists the earlier candidates it conflicts with, and one workgroup
//    settles the first-come decisions in rounds (a candidate enters once all
//    its earlier conflicts are rejected, and is rejected as soon as one of
//    them enters), which equals taking the candidates one by one in order.
#include "orca_device.h"

#include <math.h>

namespace orca {
namespace {

constexpr int kBlock = 256;
constexpr int kScanThreads = 1024;
constexpr int kConfCap = 16;  // earlier conflicts listed per candidate
constexpr uint8_t kUndecided = 0, kAccepted = 1, kRejected = 2;
constexpr int kBoundBlocksMax = 1024;

struct LifeBufs {
    uint32_t *block_count;  // leaving: survivors per block, then their offsets
    float4 *partial;        // entering: per-block maxima
    float *bounds;          // entering: max r, max s (agents), max r, max s (candidates), D_max
    uint8_t *blocked;       // entering: candidate blocked by a current agent
    int32_t *conf_count;    // entering: earlier conflicting candidates (may exceed the cap)
    int32_t *conf;          // entering: their indices, kConfCap per candidate
};

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

LifeBufs bind_life(int64_t n, int64_t n_cand, void *base)
{
    char *b = (char *)base;
    LifeBufs r;
    size_t o = 0;
    const int64_t nb = (n + kBlock - 1) / kBlock;
    r.block_count = (uint32_t *)(b + o);
    o += a256(sizeof(uint32_t) * (size_t)(nb + 1));
    r.partial = (float4 *)(b + o);
    o += a256(sizeof(float4) * kBoundBlocksMax);
    r.bounds = (float *)(b + o);
    o += a256(sizeof(float) * 8);
    r.blocked = (uint8_t *)(b + o);
    o += a256((size_t)n_cand);
    r.conf_count = (int32_t *)(b + o);
    o += a256(sizeof(int32_t) * (size_t)n_cand);
    r.conf = (int32_t *)(b + o);
    return r;
}

// Reaching the goal: |g - p|^2 <= r^2 in double, operations rounded
// separately (the same expression as the oracle's).
__device__ __forceinline__ bool arrived(float px, float py, float gx, float gy, float r)
{
#pragma clang fp contract(off)
    const double dx = (double)gx - (double)px;
    const double dy = (double)gy - (double)py;
    const double rr = (double)r;
    return dx * dx + dy * dy <= rr * rr;
}

// Two discs that could touch within t seconds at full speed.
__device__ __forceinline__ bool too_close(float ax, float ay, float ar, float as, float bx, float by,
                                          float br, float bs, double t)
{
#pragma clang fp contract(off)
    const double dx = (double)bx - (double)ax;
    const double dy = (double)by - (double)ay;
    const double d = ((double)ar + (double)br) + t * ((double)as + (double)bs);
    return dx * dx + dy * dy < d * d;
}

// (leaving 1) survivors per block
__global__ __launch_bounds__(kBlock) void k_arrive_count(orca_agents_in in, int n,
                                                          uint32_t *__restrict__ block_count)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    bool keep = false;
    if (i < n) keep = !arrived(in.px[i], in.py[i], in.pref_x[i], in.pref_y[i], in.radius[i]);
    const int c = __syncthreads_count(keep);
    if (threadIdx.x == 0) block_count[blockIdx.x] = (uint32_t)c;
}

// Exclusive scan of `count[0 .. m)` in place by one block; total to *sum.
__device__ void block_exclusive_scan(uint32_t *count, int m, uint32_t *sum)
{
    __shared__ uint32_t part[kScanThreads];
    const int tid = threadIdx.x;
    const int per = (m + kScanThreads - 1) / kScanThreads;
    const int a = tid * per, b = min(a + per, m);
    uint32_t s = 0;
    for (int k = a; k < b; ++k) s += count[k];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const uint32_t v = tid >= off ? part[tid - off] : 0u;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint32_t run = tid ? part[tid - 1] : 0u;
    for (int k = a; k < b; ++k) {
        const uint32_t c = count[k];
        count[k] = run;
        run += c;
    }
    if (tid == kScanThreads - 1) *sum = part[tid];
}

// (leaving 2) block offsets and the survivor count
__global__ __launch_bounds__(kScanThreads) void k_arrive_scan(uint32_t *__restrict__ block_count,
                                                              int nb, int32_t *__restrict__ n_alive)
{
    __shared__ uint32_t total;
    block_exclusive_scan(block_count, nb, &total);
    __syncthreads();
    if (threadIdx.x == 0) *n_alive = (int32_t)total;
}

// (leaving 3) move the survivors, keeping their order
__global__ __launch_bounds__(kBlock) void k_arrive_move(orca_agents_in in, orca_agents_buf out,
                                                         int n,
                                                         const uint32_t *__restrict__ block_off,
                                                         int32_t *__restrict__ old_to_new)
{
    __shared__ uint32_t wave_base[kBlock / kWave];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    bool keep = false;
    if (i < n) keep = !arrived(in.px[i], in.py[i], in.pref_x[i], in.pref_y[i], in.radius[i]);
    const uint64_t mask = __ballot(keep);
    if (lane == 0) wave_base[wid] = (uint32_t)__popcll(mask);
    __syncthreads();
    uint32_t base = block_off[blockIdx.x];
    for (int w = 0; w < wid; ++w) base += wave_base[w];
    const uint32_t rank = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    if (i >= n) return;
    if (keep) {
        out.px[rank] = in.px[i];
        out.py[rank] = in.py[i];
        out.vx[rank] = in.vx[i];
        out.vy[rank] = in.vy[i];
        out.pref_x[rank] = in.pref_x[i];
        out.pref_y[rank] = in.pref_y[i];
        out.radius[rank] = in.radius[i];
        out.max_speed[rank] = in.max_speed[i];
        out.cls[rank] = in.cls[i];
    }
    if (old_to_new) old_to_new[i] = keep ? (int32_t)rank : -1;
}

// (entering 1a) per-block largest radius and speed cap of the agents and of
// the candidates
__global__ __launch_bounds__(kBlock) void k_spawn_bounds(const float *__restrict__ r_a,
                                                          const float *__restrict__ s_a, int n,
                                                          const float *__restrict__ r_c,
                                                          const float *__restrict__ s_c, int nc,
                                                          float4 *__restrict__ partial)
{
    float4 m = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    const int stride = gridDim.x * kBlock;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        m.x = fmaxf(m.x, r_a[i]);
        m.y = fmaxf(m.y, s_a[i]);
    }
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < nc; i += stride) {
        m.z = fmaxf(m.z, r_c[i]);
        m.w = fmaxf(m.w, s_c[i]);
    }
    // the bounding-box reduction's (min, min, max, max) applied to (-x, -y, z, w)
    float4 q = block_bbox<kBlock>(make_float4(-m.x, -m.y, m.z, m.w));
    if (threadIdx.x == 0) partial[blockIdx.x] = make_float4(-q.x, -q.y, q.z, q.w);
}

// (entering 1b) the maxima, and the grid's query radius D_max (rounded up)
__global__ __launch_bounds__(kBlock) void k_spawn_dmax(const float4 *__restrict__ partial, int np,
                                                        float t_clear, float *__restrict__ bounds)
{
    float4 m = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int k = threadIdx.x; k < np; k += kBlock) {
        const float4 v = partial[k];
        m.x = fmaxf(m.x, v.x);
        m.y = fmaxf(m.y, v.y);
        m.z = fmaxf(m.z, v.z);
        m.w = fmaxf(m.w, v.w);
    }
    float4 q = block_bbox<kBlock>(make_float4(-m.x, -m.y, m.z, m.w));
    if (threadIdx.x != 0) return;
    bounds[0] = -q.x;
    bounds[1] = -q.y;
    bounds[2] = q.z;
    bounds[3] = q.w;
    const double d = ((double)bounds[2] + (double)bounds[0]) +
                     (double)t_clear * ((double)bounds[3] + (double)bounds[1]);
    // a positive radius for the grid even when everything is a point at rest
    bounds[4] = fmaxf(nextafterf((float)d, INFINITY) * (1.0f + 1e-6f), 1e-3f);
}

// (entering 2) candidates blocked by a current agent: each lane scans the
// grid disc of its own largest possible clearance.
__global__ __launch_bounds__(kBlock) void k_spawn_check(orca_agents_in cand, int nc,
                                                         const float *__restrict__ a_max_speed,
                                                         const GridMeta *__restrict__ meta,
                                                         const uint32_t *__restrict__ start,
                                                         const float4 *__restrict__ s0,
                                                         const float *__restrict__ bounds,
                                                         float t_clear, int n,
                                                         uint8_t *__restrict__ blocked,
                                                         int32_t *__restrict__ conf_count)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= nc) return;
    conf_count[c] = 0;
    const float cx = cand.px[c], cy = cand.py[c], cr = cand.radius[c], cs = cand.max_speed[c];
    const double t = (double)t_clear;
    bool hit = false;
    if (n > 0) {
        const GridMeta g = *meta;
        const double reach = ((double)cr + (double)bounds[0]) + t * ((double)cs + (double)bounds[1]);
        const double r2 = reach * reach * (1.0 + 1e-9);
        dev::scan_disc(g, start, s0, (double)cx, (double)cy, r2,
                       [&](const float4 &a, uint32_t, bool valid) {
                           if (valid && !hit) {
                               const int j = __float_as_int(a.z);
                               hit = too_close(cx, cy, cr, cs, a.x, a.y, a.w, a_max_speed[j], t);
                           }
                       });
    }
    blocked[c] = hit ? 1 : 0;
}

// (entering 3) each candidate's earlier conflicting candidates, found by
// tiles of candidates staged in LDS.  A candidate blocked by the agents is
// rejected whatever else happens, so lists are built for the unblocked ones
// and hold unblocked candidates only.  blockIdx.y splits the earlier
// candidates into chunks of kPairChunk tiles, so a list is filled through
// its atomic counter (zeroed by k_spawn_check); the decision rounds read a
// list as a set, and one that overflows sends its candidate to the
// exhaustive test, so the order of the entries does not matter.
constexpr int kPairChunk = 8;

__global__ __launch_bounds__(kBlock) void k_spawn_pairs(orca_agents_in cand, int nc, float t_clear,
                                                         const uint8_t *__restrict__ blocked,
                                                         int32_t *__restrict__ conf_count,
                                                         int32_t *__restrict__ conf)
{
    __shared__ float4 tile[kBlock];
    __shared__ uint8_t tile_blocked[kBlock];
    const int last = min((int)(blockIdx.x + 1) * kBlock, nc);  // candidates before the block's end
    const int b0 = (int)blockIdx.y * kPairChunk * kBlock;
    if (b0 >= last) return;  // the whole workgroup: no earlier candidates in this chunk
    const int b1 = min(b0 + kPairChunk * kBlock, last);
    const int c = blockIdx.x * kBlock + threadIdx.x;
    const bool live = c < nc && !blocked[c];
    float cx = 0.0f, cy = 0.0f, cr = 0.0f, cs = 0.0f;
    if (live) {
        cx = cand.px[c];
        cy = cand.py[c];
        cr = cand.radius[c];
        cs = cand.max_speed[c];
    }
    const double t = (double)t_clear;
    for (int base = b0; base < b1; base += kBlock) {
        const int e0 = base + threadIdx.x;
        __syncthreads();
        if (e0 < nc) {
            tile[threadIdx.x] = make_float4(cand.px[e0], cand.py[e0], cand.radius[e0],
                                            cand.max_speed[e0]);
            tile_blocked[threadIdx.x] = blocked[e0];
        }
        __syncthreads();
        if (!live) continue;
        const int m = min(kBlock, c - base);  // earlier candidates only
        for (int k = 0; k < m; ++k) {
            if (tile_blocked[k]) continue;
            const float4 e = tile[k];
            if (too_close(cx, cy, cr, cs, e.x, e.y, e.z, e.w, t)) {
                const int slot = atomicAdd(&conf_count[c], 1);
                if (slot < kConfCap) conf[(int64_t)c * kConfCap + slot] = base + k;
            }
        }
    }
}

// (entering 4) one workgroup: first-come decisions in rounds, then the
// accepted candidates are appended in order.
__global__ __launch_bounds__(kScanThreads) void k_spawn_resolve(
    orca_agents_in cand, int nc, float t_clear, const uint8_t *__restrict__ blocked,
    const int32_t *__restrict__ conf_count, const int32_t *__restrict__ conf,
    orca_agents_buf state, int n, int32_t *__restrict__ n_total, uint8_t *__restrict__ accepted)
{
    __shared__ uint8_t st[ORCA_SPAWN_MAX];
    __shared__ uint32_t part[kScanThreads];
    const int tid = threadIdx.x;
    const double t = (double)t_clear;
    for (int c = tid; c < nc; c += kScanThreads) st[c] = blocked[c] ? kRejected : kUndecided;
    __syncthreads();
    // every round decides at least the first undecided candidate, so at most
    // nc rounds; a decision never changes once taken
    for (int round = 0; round <= nc; ++round) {
        int open = 0;
        for (int c = tid; c < nc; c += kScanThreads) {
            if (st[c] != kUndecided) continue;
            bool any_acc = false, any_open = false;
            const int cnt = conf_count[c];
            if (cnt <= kConfCap) {
                for (int k = 0; k < cnt; ++k) {
                    const uint8_t s = st[conf[(int64_t)c * kConfCap + k]];
                    any_acc = any_acc || s == kAccepted;
                    any_open = any_open || s == kUndecided;
                }
            } else {
                // more conflicts than listed: test every earlier candidate
                const float cx = cand.px[c], cy = cand.py[c], cr = cand.radius[c],
                            cs = cand.max_speed[c];
                for (int e = 0; e < c; ++e) {
                    const uint8_t s = st[e];
                    if (s == kRejected) continue;
                    if (too_close(cx, cy, cr, cs, cand.px[e], cand.py[e], cand.radius[e],
                                  cand.max_speed[e], t)) {
                        any_acc = any_acc || s == kAccepted;
                        any_open = any_open || s == kUndecided;
                    }
                }
            }
            if (any_acc)
                st[c] = kRejected;
            else if (!any_open)
                st[c] = kAccepted;
            else
                open = 1;
        }
        if (!__syncthreads_or(open)) break;
    }
    // ranks of the accepted candidates (exclusive scan over thread chunks)
    const int per = (nc + kScanThreads - 1) / kScanThreads;
    const int a = tid * per, b = min(a + per, nc);
    uint32_t s = 0;
    for (int c = a; c < b; ++c) s += st[c] == kAccepted ? 1u : 0u;
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const uint32_t v = tid >= off ? part[tid - off] : 0u;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint32_t rank = (uint32_t)n + (tid ? part[tid - 1] : 0u);
    for (int c = a; c < b; ++c) {
        const bool ok = st[c] == kAccepted;
        if (accepted) accepted[c] = ok ? 1 : 0;
        if (!ok) continue;
        state.px[rank] = cand.px[c];
        state.py[rank] = cand.py[c];
        state.vx[rank] = cand.vx[c];
        state.vy[rank] = cand.vy[c];
        state.pref_x[rank] = cand.pref_x[c];
        state.pref_y[rank] = cand.pref_y[c];
        state.radius[rank] = cand.radius[c];
        state.max_speed[rank] = cand.max_speed[c];
        state.cls[rank] = cand.cls[c];
        ++rank;
    }
    if (tid == kScanThreads - 1) *n_total = (int32_t)((uint32_t)n + part[tid]);
}

// Overlap statistics, per block: pairs counted from both ends, agents in
// an overlap, and the smallest clearance over pairs closer than the grid's
// neighbour distance.  One lane per agent in cell order.
struct OverlapPart {
    double gap;
    uint32_t pairs2;  // overlapping pairs, each counted by both agents
    uint32_t agents;
};

__global__ __launch_bounds__(kBlock) void k_overlap(const GridMeta *__restrict__ meta,
                                                     const uint32_t *__restrict__ start,
                                                     const float4 *__restrict__ s0, int n,
                                                     OverlapPart *__restrict__ part)
{
    const int s = blockIdx.x * kBlock + threadIdx.x;
    uint32_t cnt = 0;
    double gap = INFINITY;
    if (s < n) {
        const GridMeta g = *meta;
        const float4 me = s0[s];
        const int self = __float_as_int(me.z);
        dev::scan_disc(g, start, s0, (double)me.x, (double)me.y, g.rn2,
                       [&](const float4 &a, uint32_t, bool valid) {
                           const double d2 = dev::nb_key(me.x, me.y, a.x, a.y);
                           if (valid && d2 < g.rn2 && __float_as_int(a.z) != self) {
                               const double rr = (double)me.w + (double)a.w;
                               cnt += d2 < rr * rr ? 1u : 0u;
                               gap = fmin(gap, sqrt(d2) - rr);
                           }
                       });
    }
    __shared__ double sg[kBlock / kWave];
    __shared__ uint32_t sp[kBlock / kWave], sa[kBlock / kWave];
    double wg = gap;
    uint32_t wp = cnt, wa = cnt > 0 ? 1u : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        wg = fmin(wg, __shfl_xor(wg, o, kWave));
        wp += __shfl_xor(wp, o, kWave);
        wa += __shfl_xor(wa, o, kWave);
    }
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    if (lane == 0) {
        sg[wid] = wg;
        sp[wid] = wp;
        sa[wid] = wa;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        OverlapPart r{INFINITY, 0u, 0u};
        for (int w = 0; w < kBlock / kWave; ++w) {
            r.gap = fmin(r.gap, sg[w]);
            r.pairs2 += sp[w];
            r.agents += sa[w];
        }
        part[blockIdx.x] = r;
    }
}

__global__ __launch_bounds__(kBlock) void k_overlap_final(const OverlapPart *__restrict__ part,
                                                           int np, double *__restrict__ out)
{
    __shared__ double sg[kBlock];
    __shared__ unsigned long long sp[kBlock], sa[kBlock];
    double g = INFINITY;
    unsigned long long p = 0, a = 0;
    for (int k = threadIdx.x; k < np; k += kBlock) {
        g = fmin(g, part[k].gap);
        p += part[k].pairs2;
        a += part[k].agents;
    }
    sg[threadIdx.x] = g;
    sp[threadIdx.x] = p;
    sa[threadIdx.x] = a;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sg[threadIdx.x] = fmin(sg[threadIdx.x], sg[threadIdx.x + o]);
            sp[threadIdx.x] += sp[threadIdx.x + o];
            sa[threadIdx.x] += sa[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = (double)(sp[0] / 2);
        out[1] = (double)sa[0];
        out[2] = sg[0];
    }
}

}  // namespace

size_t lifecycle_extra_bytes(int64_t n, int64_t n_cand)
{
    const int64_t nb = (n + kBlock - 1) / kBlock;
    return a256(sizeof(uint32_t) * (size_t)(nb + 1)) + a256(sizeof(float4) * kBoundBlocksMax) +
           a256(sizeof(float) * 8) +
           a256((size_t)n_cand) + a256(sizeof(int32_t) * (size_t)n_cand) +
           a256(sizeof(int32_t) * (size_t)kConfCap * (size_t)n_cand);
}

hipError_t launch_remove_arrived(const orca_agents_in &in, const orca_agents_buf &out, int n,
                                 int32_t *n_alive, int32_t *old_to_new, void *extra,
                                 hipStream_t stream)
{
    const LifeBufs b = bind_life(n, 0, extra);
    const int nb = (n + kBlock - 1) / kBlock;
    if (nb > 0)
        hipLaunchKernelGGL(k_arrive_count, dim3(nb), dim3(kBlock), 0, stream, in, n,
                           b.block_count);
    hipLaunchKernelGGL(k_arrive_scan, dim3(1), dim3(kScanThreads), 0, stream, b.block_count, nb,
                       n_alive);
    if (nb > 0)
        hipLaunchKernelGGL(k_arrive_move, dim3(nb), dim3(kBlock), 0, stream, in, out, n,
                           b.block_count, old_to_new);
    return hipGetLastError();
}

hipError_t launch_spawn(const orca_agents_buf &state, int n, const orca_agents_in &cand,
                        int n_cand, float t_clear, int32_t *n_total, uint8_t *accepted,
                        const Layout &L, const Work &w, void *extra, hipStream_t stream)
{
    const LifeBufs b = bind_life(n, n_cand, extra);
    const orca_agents_in cur{state.px,     state.py,        state.vx,
                             state.vy,     state.pref_x,    state.pref_y,
                             state.radius, state.max_speed, state.cls};
    const int m = n > n_cand ? n : n_cand;
    int nbb = (m + kBlock - 1) / kBlock;
    nbb = nbb < 1 ? 1 : (nbb > kBoundBlocksMax ? kBoundBlocksMax : nbb);
    hipLaunchKernelGGL(k_spawn_bounds, dim3(nbb), dim3(kBlock), 0, stream, state.radius,
                       state.max_speed, n, cand.radius, cand.max_speed, n_cand, b.partial);
    hipLaunchKernelGGL(k_spawn_dmax, dim3(1), dim3(kBlock), 0, stream, b.partial, nbb, t_clear,
                       b.bounds);
    if (n > 0) {
        // the grid's neighbour distance (and cell size) is D_max from the device
        const hipError_t e = launch_grid_build_rn(cur, n, 1.0f, 0.0f, b.bounds + 4, L, w, stream);
        if (e != hipSuccess) return e;
    }
    const int ncb = (n_cand + kBlock - 1) / kBlock;
    if (ncb > 0) {
        hipLaunchKernelGGL(k_spawn_check, dim3(ncb), dim3(kBlock), 0, stream, cand, n_cand,
                           (const float *)state.max_speed, w.meta, w.start, w.s0, b.bounds,
                           t_clear, n, b.blocked, b.conf_count);
        const int chunks = (ncb + kPairChunk - 1) / kPairChunk;
        hipLaunchKernelGGL(k_spawn_pairs, dim3(ncb, chunks), dim3(kBlock), 0, stream, cand,
                           n_cand, t_clear, b.blocked, b.conf_count, b.conf);
    }
    hipLaunchKernelGGL(k_spawn_resolve, dim3(1), dim3(kScanThreads), 0, stream, cand, n_cand,
                       t_clear, b.blocked, b.conf_count, b.conf, state, n, n_total, accepted);
    return hipGetLastError();
}

}  // namespace orca

namespace orca {

size_t overlap_extra_bytes(int64_t n)
{
    return a256(sizeof(OverlapPart) * (size_t)((n + kBlock - 1) / kBlock + 1));
}

hipError_t launch_overlap_stats(const orca_agents_in &in, int n, float reach, double *out,
                                const Layout &L, const Work &w, void *extra, hipStream_t stream)
{
    OverlapPart *part = (OverlapPart *)extra;
    const int nb = (n + kBlock - 1) / kBlock;
    if (n > 0) {
        const hipError_t e = launch_grid_build_rn(in, n, reach, 0.0f, nullptr, L, w, stream);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_overlap, dim3(nb), dim3(kBlock), 0, stream, w.meta, w.start, w.s0,
                           n, part);
    }
    hipLaunchKernelGGL(k_overlap_final, dim3(1), dim3(kBlock), 0, stream, part, nb, out);
    return hipGetLastError();
}

}  // namespace orca
