// Fused ORCA step for one scene on gfx950: one lane per agent, agents taken in
// cell order so that the lanes of a wavefront share neighbour candidates; the
// per-agent work (exact kNN, half-planes, LP2, LP3, update) is
// dev::step_agent.  Also the neighbour-list export of orca_build_grid and of
// orca_step_nbr.
#include "orca_device.h"

namespace orca {
namespace {

constexpr int kStepBlock = 64;  // one wavefront: its LDS is free again as soon as it ends

struct StepArgs {
    orca_agents_in in;
    orca_agents_out out;
    const GridMeta *meta;
    const uint32_t *start;
    const float4 *s0;
    const float4 *s1;
    int n;
    int k;
    int32_t *nbr;   // knn export only
    int32_t *cnt;
    float *guess;   // per-agent K-th neighbour distance kept between steps
    orca_params prm;
};

using dev::buf_idx;
using dev::KnnShape;
using dev::knn_select;

// EXPORT: the same step, also writing the neighbour lists it used.
template <int K, int BLOCK, bool ACC, bool EXPORT>
__global__ __launch_bounds__(BLOCK) void k_step(StepArgs a, dev::SceneP p)
{
    __shared__ float4 lines[dev::KnnShape<K>::kSlots * BLOCK];
    const int tid = threadIdx.x;
    const int s = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + tid;
    if (s >= a.n) return;
    const GridMeta g = *a.meta;
    dev::step_agent<K, BLOCK, ACC, EXPORT>(s, g, p, a.in, a.out, a.start, a.s0, a.s1, lines, tid,
                                           a.guess, a.nbr, a.cnt, a.k);
}

template <int K, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_knn_export(StepArgs a)
{
    __shared__ float4 lds[KnnShape<K>::kSlots * BLOCK];
    const int tid = threadIdx.x;
    const int s = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + tid;
    if (s >= a.n) return;
    const GridMeta g = *a.meta;
    const float4 me0 = a.s0[s];
    const int i = __float_as_int(me0.z);
    uint64_t *buf = reinterpret_cast<uint64_t *>(lds);
    const int found =
        knn_select<K, BLOCK>(g, a.start, a.s0, me0.x, me0.y, i, (uint32_t)s, buf, tid, g.rn2);
    const int m = found < a.k ? found : a.k;
    if (a.nbr) {
        int32_t *row = a.nbr + (int64_t)i * a.k;
        for (int q = 0; q < a.k; ++q)
            row[q] = q < m ? __float_as_int(a.s0[dev::entry_pos(buf[buf_idx<BLOCK>(q, tid)])].z) : -1;
    }
    if (a.cnt) a.cnt[i] = m;
}

StepArgs make_args(const orca_agents_in &in, const orca_agents_out *out, int n,
                   const orca_params &p, const Work &w)
{
    StepArgs a;
    a.in = in;
    if (out)
        a.out = *out;
    else
        a.out = orca_agents_out{nullptr, nullptr, nullptr, nullptr, nullptr};
    a.meta = w.meta;
    a.start = w.start;
    a.s0 = w.s0;
    a.s1 = w.s1;
    a.n = n;
    a.k = p.max_neighbors;
    a.nbr = nullptr;
    a.cnt = nullptr;
    a.guess = w.guess;
    a.prm = p;
    return a;
}

template <int K>
void launch_step_k(const StepArgs &a, hipStream_t stream)
{
    const int nb = (a.n + kStepBlock - 1) / kStepBlock;
    // the variant with hard lines (acceleration, heading) only when a class
    // has a cap, the exporting variant only when lists are asked for
    const bool acc = a.prm.accel[0] > 0.0f || a.prm.accel[1] > 0.0f || a.prm.turn[0] > 0.0f ||
                     a.prm.turn[1] > 0.0f;
    const bool exp = a.nbr || a.cnt;
    const dev::SceneP p = dev::scene_params(a.prm);
    if (acc && exp)
        hipLaunchKernelGGL((k_step<K, kStepBlock, true, true>), dim3(nb), dim3(kStepBlock), 0,
                           stream, a, p);
    else if (acc)
        hipLaunchKernelGGL((k_step<K, kStepBlock, true, false>), dim3(nb), dim3(kStepBlock), 0,
                           stream, a, p);
    else if (exp)
        hipLaunchKernelGGL((k_step<K, kStepBlock, false, true>), dim3(nb), dim3(kStepBlock), 0,
                           stream, a, p);
    else
        hipLaunchKernelGGL((k_step<K, kStepBlock, false, false>), dim3(nb), dim3(kStepBlock), 0,
                           stream, a, p);
}

template <int K>
void launch_knn_k(const StepArgs &a, hipStream_t stream)
{
    const int nb = (a.n + kStepBlock - 1) / kStepBlock;
    hipLaunchKernelGGL((k_knn_export<K, kStepBlock>), dim3(nb), dim3(kStepBlock), 0, stream, a);
}

}  // namespace

// Register-list capacities compiled; k is rounded up to the next one (the k
// smallest of a set are the first k of its K smallest).
#define ORCA_DISPATCH_K(FN, k, a, stream)          \
    do {                                           \
        if ((k) <= 4)                              \
            FN<4>(a, stream);                      \
        else if ((k) <= 8)                         \
            FN<8>(a, stream);                      \
        else if ((k) <= 10)                        \
            FN<10>(a, stream);                     \
        else if ((k) <= 12)                        \
            FN<12>(a, stream);                     \
        else if ((k) <= 16)                        \
            FN<16>(a, stream);                     \
        else if ((k) <= 20)                        \
            FN<20>(a, stream);                     \
        else if ((k) <= 24)                        \
            FN<24>(a, stream);                     \
        else                                       \
            FN<32>(a, stream);                     \
    } while (0)

hipError_t launch_step(const orca_agents_in &in, const orca_agents_out &out, int n,
                       const orca_params &p, const Layout &L, const Work &w, int32_t *nbr,
                       int32_t *cnt, hipStream_t stream)
{
    (void)L;
    StepArgs a = make_args(in, &out, n, p, w);
    a.nbr = nbr;
    a.cnt = cnt;
    ORCA_DISPATCH_K(launch_step_k, p.max_neighbors, a, stream);
    return hipGetLastError();
}

hipError_t launch_knn_export(const orca_agents_in &in, int n, const orca_params &p,
                             const Layout &L, const Work &w, int32_t *nbr, int32_t *cnt,
                             hipStream_t stream)
{
    (void)L;
    StepArgs a = make_args(in, nullptr, n, p, w);
    a.nbr = nbr;
    a.cnt = cnt;
    ORCA_DISPATCH_K(launch_knn_k, p.max_neighbors, a, stream);
    return hipGetLastError();
}

}  // namespace orca
