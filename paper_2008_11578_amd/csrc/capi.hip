// C ABI of liborca.so: argument validation, workspace layout and dispatch.
// Nothing here allocates or synchronises; every launch goes on the caller's
// stream.
#include "orca_internal.h"

#include <math.h>

#include <mutex>

namespace orca {

namespace {
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
}  // namespace

Layout make_layout(int64_t n, int64_t n_scenes, int64_t max_cells)
{
    Layout L{};
    if (n_scenes > 0)
        max_cells = batched_cells(n, n_scenes);
    else if (max_cells <= 0)
        max_cells = default_max_cells(n);
    const int64_t S = n_scenes > 0 ? n_scenes : 1;
    L.n = n;
    L.n_scenes = S;
    L.max_cells = max_cells;
    L.n_tiles = (max_cells + 1 + kScanTile - 1) / kScanTile;
    size_t o = 0;
    L.meta = o;
    o = align_up(o + sizeof(GridMeta) * (size_t)(S + 1));
    L.partial = o;
    const size_t n_partial = (size_t)S * kBboxSplit;
    o = align_up(o + sizeof(float4) * (n_partial > (size_t)kBboxBlocks ? n_partial
                                                                       : (size_t)kBboxBlocks));
    L.queue = o;
    o = align_up(o + sizeof(uint32_t) * kXcds);
    L.cell = o;
    o = align_up(o + sizeof(uint32_t) * (size_t)n);
    L.rank = o;
    o = align_up(o + sizeof(uint32_t) * (size_t)n);
    L.count = o;
    o = align_up(o + sizeof(uint32_t) * (size_t)(max_cells + 1));
    L.start = o;
    o = align_up(o + sizeof(uint32_t) * (size_t)(max_cells + 1));
    L.tiles = o;
    o = align_up(o + sizeof(uint32_t) * (size_t)(L.n_tiles + 1));
    L.s0 = o;
    o = align_up(o + sizeof(float4) * (size_t)(n + kScanPad));
    L.s1 = o;
    o = align_up(o + sizeof(float4) * (size_t)n);
    L.guess = o;
    o = align_up(o + sizeof(float) * (size_t)n);
    L.total = o;
    return L;
}

Work bind(const Layout &L, void *ws)
{
    char *b = (char *)ws;
    Work w;
    w.meta = (GridMeta *)(b + L.meta);
    w.partial = (float4 *)(b + L.partial);
    w.queue = (uint32_t *)(b + L.queue);
    w.cell = (uint32_t *)(b + L.cell);
    w.rank = (uint32_t *)(b + L.rank);
    w.count = (uint32_t *)(b + L.count);
    w.start = (uint32_t *)(b + L.start);
    w.tiles = (uint32_t *)(b + L.tiles);
    w.s0 = (float4 *)(b + L.s0);
    w.s1 = (float4 *)(b + L.s1);
    w.guess = (float *)(b + L.guess);
    return w;
}

size_t adjoint_extra_bytes(int64_t n)
{
    const size_t a = align_up(sizeof(float) * (size_t)n) + align_up(sizeof(int32_t) * 3 * (size_t)n) +
                     align_up(sizeof(float4) * 3 * (size_t)n) +
                     2 * align_up(sizeof(uint32_t) * 3 * (size_t)n) +
                     2 * align_up(sizeof(uint32_t) * (size_t)n) +
                     align_up(sizeof(uint32_t) * (size_t)((n + kScanTile - 1) / kScanTile + 1)) +
                     align_up(sizeof(double) * kTauBlocks);
    return a;
}

AdjointBufs bind_adjoint(int64_t n, void *base)
{
    char *b = (char *)base;
    AdjointBufs r;
    size_t o = 0;
    r.tau_part = (float *)(b + o);
    o += align_up(sizeof(float) * (size_t)n);
    r.e_tgt = (int32_t *)(b + o);
    o += align_up(sizeof(int32_t) * 3 * (size_t)n);
    r.e_val = (float4 *)(b + o);
    o += align_up(sizeof(float4) * 3 * (size_t)n);
    r.e_rank = (uint32_t *)(b + o);
    o += align_up(sizeof(uint32_t) * 3 * (size_t)n);
    r.e_list = (uint32_t *)(b + o);
    o += align_up(sizeof(uint32_t) * 3 * (size_t)n);
    r.e_cnt = (uint32_t *)(b + o);
    o += align_up(sizeof(uint32_t) * (size_t)n);
    r.e_start = (uint32_t *)(b + o);
    o += align_up(sizeof(uint32_t) * (size_t)n);
    r.e_tiles = (uint32_t *)(b + o);
    o += align_up(sizeof(uint32_t) * (size_t)((n + kScanTile - 1) / kScanTile + 1));
    r.tau_blocks = (double *)(b + o);
    return r;
}

namespace {

// The workspace size fixes max_cells for a given n: the largest cell count
// whose layout still fits, so the caller only has to pass the byte size.
int64_t max_cells_for(int64_t n, int64_t n_scenes, size_t ws_bytes)
{
    const Layout base = make_layout(n, n_scenes, 1);
    if (base.total > ws_bytes) return 0;
    int64_t lo = 1, hi = 1;
    while (make_layout(n, n_scenes, hi * 2).total <= ws_bytes && hi < (int64_t)1 << 30) hi *= 2;
    hi *= 2;
    while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (make_layout(n, n_scenes, mid).total <= ws_bytes)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

bool finite_pos(float v) { return isfinite(v) && v > 0.0f; }

int check_params(const orca_params *p)
{
    if (!p) return ORCA_EINVAL;
    if (p->max_neighbors < 1 || p->max_neighbors > ORCA_K_MAX) return ORCA_ERANGE;
    if (!finite_pos(p->dt) || !finite_pos(p->time_horizon) || !finite_pos(p->neighbor_dist))
        return ORCA_EINVAL;
    if (!(p->cell_size >= 0.0f) || !isfinite(p->cell_size)) return ORCA_EINVAL;
    if (!(p->par_eps >= 0.0f) || !isfinite(p->par_eps)) return ORCA_EINVAL;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            if (!isfinite(p->f[a][b])) return ORCA_EINVAL;
    if (p->pref_is_goal != 0 && p->pref_is_goal != 1) return ORCA_EINVAL;
    for (int c = 0; c < 2; ++c)
        if (!(p->accel[c] >= 0.0f) || !isfinite(p->accel[c])) return ORCA_EINVAL;
    for (int c = 0; c < 2; ++c)
        if (!(p->turn[c] >= 0.0f) || !isfinite(p->turn[c])) return ORCA_EINVAL;
    return ORCA_OK;
}

int check_in(const orca_agents_in *in)
{
    if (!in || !in->px || !in->py || !in->vx || !in->vy || !in->pref_x || !in->pref_y ||
        !in->radius || !in->max_speed || !in->cls)
        return ORCA_EINVAL;
    return ORCA_OK;
}

int check_out(const orca_agents_out *out)
{
    if (!out || !out->px || !out->py || !out->vx || !out->vy) return ORCA_EINVAL;
    return ORCA_OK;
}

int check_buf(const orca_agents_buf *b)
{
    if (!b || !b->px || !b->py || !b->vx || !b->vy || !b->pref_x || !b->pref_y || !b->radius ||
        !b->max_speed || !b->cls)
        return ORCA_EINVAL;
    return ORCA_OK;
}

// Workspace of the lifecycle entry points: the grid of n agents, then the
// lifecycle buffers.
Layout life_layout(int64_t n) { return make_layout(n > 0 ? n : 1, 0, 0); }

// Cell count that keeps the grid within what the 32-bit indices address.
constexpr int64_t kMaxCellsCap = (int64_t)1 << 30;

int prepare(int32_t n, const orca_params *params, void *ws, size_t ws_bytes, Layout &L)
{
    if (n < 0 || n > ORCA_N_MAX) return ORCA_EINVAL;
    const int rc = check_params(params);
    if (rc != ORCA_OK) return rc;
    if (n == 0) return ORCA_OK;
    if (!ws) return ORCA_EINVAL;
    int64_t mc = max_cells_for(n, 0, ws_bytes);
    if (mc <= 0) return ORCA_EWORKSPACE;
    if (mc > kMaxCellsCap) mc = kMaxCellsCap;
    L = make_layout(n, 0, mc);
    if (L.total > ws_bytes) return ORCA_EWORKSPACE;
    return ORCA_OK;
}

// Workspace of orca_step_noalloc: one array per GPU, in the library's own
// device memory.  Host code never passes `scratch` itself to a kernel (on
// the host that name is only a stand-in for the device array): it uses the
// device address looked up once per device below.
static __device__ __align__(256) unsigned char scratch[ORCA_NOALLOC_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// The current device's scratch address.  On the first call on a device:
// hipGetSymbolAddress with that device current, then one fill kernel on
// `stream` that clears the array before any use of it in stream order.
int noalloc_scratch(hipStream_t stream, void **ptr)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return ORCA_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return ORCA_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ORCA_EHIP;
        if (launch_fill_zero(p, ORCA_NOALLOC_BYTES, stream) != hipSuccess) return ORCA_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return ORCA_OK;
}

}  // namespace
}  // namespace orca

using namespace orca;

extern "C" {

size_t orca_workspace_bytes(int32_t n, int32_t n_scenes, int32_t max_cells)
{
    if (n < 0 || n_scenes < 0 || max_cells < 0) return 0;
    return make_layout(n, n_scenes, max_cells).total;
}

int orca_workspace_init(void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!ws && ws_bytes) return ORCA_EINVAL;
    if (launch_fill_zero(ws, ws_bytes, stream) != hipSuccess) return ORCA_EHIP;
    return ORCA_OK;
}

int orca_build_grid(const orca_agents_in *in, int32_t n, const orca_params *params, void *ws,
                    size_t ws_bytes, int32_t *nbr, int32_t *nbr_count, hipStream_t stream)
{
    Layout L{};
    int rc = prepare(n, params, ws, ws_bytes, L);
    if (rc != ORCA_OK || n == 0) return rc;
    rc = check_in(in);
    if (rc != ORCA_OK) return rc;
    const Work w = bind(L, ws);
    if (launch_grid_build(*in, n, *params, L, w, stream) != hipSuccess) return ORCA_EHIP;
    if (nbr || nbr_count) {
        if (launch_knn_export(*in, n, *params, L, w, nbr, nbr_count, stream) != hipSuccess)
            return ORCA_EHIP;
    }
    return ORCA_OK;
}

}  // extern "C"

namespace {

int step_impl(const orca_agents_in *in, const orca_agents_out *out, int32_t n,
              const orca_params *params, void *ws, size_t ws_bytes,
              const orca_step_events *events, int32_t *nbr, int32_t *nbr_count,
              hipStream_t stream)
{
    Layout L{};
    int rc = prepare(n, params, ws, ws_bytes, L);
    if (rc != ORCA_OK || n == 0) return rc;
    rc = check_in(in);
    if (rc != ORCA_OK) return rc;
    rc = check_out(out);
    if (rc != ORCA_OK) return rc;
    const Work w = bind(L, ws);
    if (events && events->grid_begin && hipEventRecord(events->grid_begin, stream) != hipSuccess)
        return ORCA_EHIP;
    if (launch_grid_build(*in, n, *params, L, w, stream) != hipSuccess) return ORCA_EHIP;
    if (events && events->step_begin && hipEventRecord(events->step_begin, stream) != hipSuccess)
        return ORCA_EHIP;
    if (launch_step(*in, *out, n, *params, L, w, nbr, nbr_count, stream) != hipSuccess)
        return ORCA_EHIP;
    if (events && events->step_end && hipEventRecord(events->step_end, stream) != hipSuccess)
        return ORCA_EHIP;
    return ORCA_OK;
}

}  // namespace

extern "C" {

int orca_step_ex(const orca_agents_in *in, const orca_agents_out *out, int32_t n,
                 const orca_params *params, void *ws, size_t ws_bytes,
                 const orca_step_events *events, hipStream_t stream)
{
    return step_impl(in, out, n, params, ws, ws_bytes, events, nullptr, nullptr, stream);
}

int orca_step(const orca_agents_in *in, const orca_agents_out *out, int32_t n,
              const orca_params *params, void *ws, size_t ws_bytes, hipStream_t stream)
{
    return step_impl(in, out, n, params, ws, ws_bytes, nullptr, nullptr, nullptr, stream);
}

int orca_step_nbr(const orca_agents_in *in, const orca_agents_out *out, int32_t n,
                  const orca_params *params, void *ws, size_t ws_bytes, int32_t *nbr,
                  int32_t *nbr_count, hipStream_t stream)
{
    return step_impl(in, out, n, params, ws, ws_bytes, nullptr, nbr, nbr_count, stream);
}

int orca_step_noalloc(const orca_agents_in *in, const orca_agents_out *out, int32_t n,
                      const orca_params *params, hipStream_t stream)
{
    // every argument is checked before the scratch set-up enqueues anything
    if (n < 0) return ORCA_EINVAL;
    if (n > ORCA_NOALLOC_N_MAX) return ORCA_ETOOBIG;
    int rc = check_params(params);
    if (rc != ORCA_OK || n == 0) return rc;
    rc = check_in(in);
    if (rc != ORCA_OK) return rc;
    rc = check_out(out);
    if (rc != ORCA_OK) return rc;
    const size_t bytes = make_layout(n, 0, 0).total;
    if (bytes > ORCA_NOALLOC_BYTES) return ORCA_ETOOBIG;
    void *ws = nullptr;
    rc = noalloc_scratch(stream, &ws);
    if (rc != ORCA_OK) return rc;
    return step_impl(in, out, n, params, ws, bytes, nullptr, nullptr, nullptr, stream);
}

int orca_step_batched(const orca_agents_in *in, const orca_agents_out *out, int32_t n,
                      const orca_batch *batch, void *ws, size_t ws_bytes, hipStream_t stream)
{
    return orca_step_batched_ex(in, out, n, batch, ws, ws_bytes, nullptr, stream);
}

int orca_step_batched_ex(const orca_agents_in *in, const orca_agents_out *out, int32_t n,
                         const orca_batch *batch, void *ws, size_t ws_bytes,
                         const orca_step_events *events, hipStream_t stream)
{
    if (n < 0 || n > ORCA_N_MAX || !batch) return ORCA_EINVAL;
    if (batch->n_scenes < 1 || !batch->scene_off || !batch->params) return ORCA_EINVAL;
    if (batch->max_neighbors < 1 || batch->max_neighbors > ORCA_K_MAX) return ORCA_ERANGE;
    if (batch->mode != 0 && batch->mode != 1) return ORCA_EINVAL;
    if (batch->has_accel != 0 && batch->has_accel != 1) return ORCA_EINVAL;
    if (batch->block != 0 && batch->block != 64 && batch->block != 128 && batch->block != 256)
        return ORCA_EINVAL;
    if (batch->k_tile != 0 && (batch->k_tile < batch->max_neighbors || batch->k_tile > ORCA_K_MAX))
        return ORCA_ERANGE;
    if (n == 0) return ORCA_OK;
    int rc = check_in(in);
    if (rc != ORCA_OK) return rc;
    rc = check_out(out);
    if (rc != ORCA_OK) return rc;
    if (!ws) return ORCA_EINVAL;
    if (batched_cells(n, batch->n_scenes) > kMaxCellsCap) return ORCA_EINVAL;
    const Layout L = make_layout(n, batch->n_scenes, 0);
    if (L.total > ws_bytes) return ORCA_EWORKSPACE;
    const Work w = bind(L, ws);
    if (launch_batched(*in, *out, n, batch->scene_off, batch->n_scenes, batch->params,
                       batch->k_tile ? batch->k_tile : batch->max_neighbors,
                       batch->has_accel != 0, batch->block ? batch->block : 128, L, w,
                       batch->error_flag, batch->mode, events, stream) != hipSuccess)
        return ORCA_EHIP;
    return ORCA_OK;
}

size_t orca_backward_workspace_bytes(int32_t n, int32_t max_cells)
{
    if (n < 0 || max_cells < 0) return 0;
    return make_layout(n, 0, max_cells).total + adjoint_extra_bytes(n);
}

int orca_step_backward(const orca_agents_in *in, int32_t n, const orca_params *params,
                       const orca_cotangents *g1, const orca_cotangents_out *g0, void *ws,
                       size_t ws_bytes, hipStream_t stream)
{
    return orca_step_backward_ex(in, n, params, g1, g0, ws, ws_bytes, nullptr, stream);
}

int orca_step_backward_ex(const orca_agents_in *in, int32_t n, const orca_params *params,
                          const orca_cotangents *g1, const orca_cotangents_out *g0, void *ws,
                          size_t ws_bytes, const orca_step_events *events, hipStream_t stream)
{
    if (n < 0 || n > ORCA_N_MAX) return ORCA_EINVAL;
    int rc = check_params(params);
    if (rc != ORCA_OK) return rc;
    if (n == 0) return ORCA_OK;
    rc = check_in(in);
    if (rc != ORCA_OK) return rc;
    if (!g1 || !g1->px || !g1->py || !g1->vx || !g1->vy) return ORCA_EINVAL;
    if (!g0 || !g0->px || !g0->py || !g0->vx || !g0->vy || !g0->pref_x || !g0->pref_y)
        return ORCA_EINVAL;
    if (!ws) return ORCA_EINVAL;
    const size_t extra = adjoint_extra_bytes(n);
    if (ws_bytes <= extra) return ORCA_EWORKSPACE;
    int64_t mc = max_cells_for(n, 0, ws_bytes - extra);
    if (mc <= 0) return ORCA_EWORKSPACE;
    if (mc > kMaxCellsCap) mc = kMaxCellsCap;
    const Layout L = make_layout(n, 0, mc);
    if (L.total + extra > ws_bytes) return ORCA_EWORKSPACE;
    const Work w = bind(L, ws);
    const AdjointBufs b = bind_adjoint(n, (char *)ws + L.total);
    if (events && events->grid_begin && hipEventRecord(events->grid_begin, stream) != hipSuccess)
        return ORCA_EHIP;
    if (launch_grid_build(*in, n, *params, L, w, stream) != hipSuccess) return ORCA_EHIP;
    if (launch_adjoint(*in, n, *params, L, w, b, g1->px, g1->py, g1->vx, g1->vy, g0->px, g0->py,
                       g0->vx, g0->vy, g0->pref_x, g0->pref_y, g0->tau, events,
                       stream) != hipSuccess)
        return ORCA_EHIP;
    return ORCA_OK;
}

size_t orca_lifecycle_workspace_bytes(int32_t n, int32_t n_cand)
{
    if (n < 0 || n_cand < 0) return 0;
    return align_up(life_layout(n).total) + lifecycle_extra_bytes(n, n_cand);
}

int orca_remove_arrived(const orca_agents_in *in, const orca_agents_buf *out, int32_t n,
                        int32_t *n_alive, int32_t *old_to_new, void *ws, size_t ws_bytes,
                        hipStream_t stream)
{
    if (n < 0 || !n_alive || !ws) return ORCA_EINVAL;
    if (n > 0 && (check_in(in) != ORCA_OK || check_buf(out) != ORCA_OK)) return ORCA_EINVAL;
    if (ws_bytes < orca_lifecycle_workspace_bytes(n, 0)) return ORCA_EWORKSPACE;
    void *extra = (char *)ws + align_up(life_layout(n).total);
    const orca_agents_in no_in{};
    const orca_agents_buf no_out{};
    if (launch_remove_arrived(n > 0 ? *in : no_in, n > 0 ? *out : no_out, n, n_alive, old_to_new,
                              extra, stream) != hipSuccess)
        return ORCA_EHIP;
    return ORCA_OK;
}

int orca_spawn(const orca_agents_buf *state, int32_t n, int32_t capacity,
               const orca_agents_in *cand, int32_t n_cand, float t_clear, int32_t *n_total,
               uint8_t *accepted, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (n < 0 || n_cand < 0 || n_cand > ORCA_SPAWN_MAX || !n_total || !ws) return ORCA_EINVAL;
    if ((int64_t)capacity < (int64_t)n + (int64_t)n_cand) return ORCA_EINVAL;
    if (!(t_clear >= 0.0f) || !isfinite(t_clear)) return ORCA_EINVAL;
    if (n + n_cand > 0 && check_buf(state) != ORCA_OK) return ORCA_EINVAL;
    if (n_cand > 0 && check_in(cand) != ORCA_OK) return ORCA_EINVAL;
    if (ws_bytes < orca_lifecycle_workspace_bytes(n, n_cand)) return ORCA_EWORKSPACE;
    const Layout L = life_layout(n);
    const Work w = bind(L, ws);
    void *extra = (char *)ws + align_up(L.total);
    const orca_agents_in no_cand{};
    const orca_agents_buf no_state{};
    if (launch_spawn(n + n_cand > 0 ? *state : no_state, n, n_cand > 0 ? *cand : no_cand, n_cand,
                     t_clear, n_total, accepted, L, w, extra, stream) != hipSuccess)
        return ORCA_EHIP;
    return ORCA_OK;
}

size_t orca_overlap_workspace_bytes(int32_t n)
{
    if (n < 0) return 0;
    return align_up(life_layout(n).total) + overlap_extra_bytes(n);
}

int orca_overlap_stats(const orca_agents_in *in, int32_t n, float reach, double *out, void *ws,
                       size_t ws_bytes, hipStream_t stream)
{
    if (n < 0 || !out || !ws || !finite_pos(reach)) return ORCA_EINVAL;
    if (n > 0 && check_in(in) != ORCA_OK) return ORCA_EINVAL;
    if (ws_bytes < orca_overlap_workspace_bytes(n)) return ORCA_EWORKSPACE;
    const Layout L = life_layout(n);
    const Work w = bind(L, ws);
    void *extra = (char *)ws + align_up(L.total);
    if (launch_overlap_stats(n > 0 ? *in : orca_agents_in{}, n, reach, out, L, w, extra, stream) !=
        hipSuccess)
        return ORCA_EHIP;
    return ORCA_OK;
}

const char *orca_status_string(int code)
{
    switch (code) {
    case ORCA_OK: return "ok";
    case ORCA_EINVAL: return "invalid argument";
    case ORCA_EWORKSPACE: return "workspace too small";
    case ORCA_EHIP: return "HIP launch error";
    case ORCA_ERANGE: return "max_neighbors outside 1..ORCA_K_MAX";
    case ORCA_ETOOBIG: return "more agents than the no-allocation scratch holds";
    default: return "unknown status";
    }
}

const char *orca_version(void) { return "orca-mi355x 0.1 (gfx950)"; }

}  // extern "C"
