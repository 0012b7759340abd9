// Per-agent device code of the ORCA step (gfx950), shared by the single-scene
// and the batched kernels.  One lane per agent:
//
//   kNN      exact k nearest (squared distance in FP64 without contraction,
//            ties by caller index) over the rows of the cell stencil, each row
//            one contiguous range of the cell-ordered copy
//   ORCA     one half-plane per neighbour (Fig. 1(b,c), Sec. 3.1), computed
//            without divergent branches: the arc, leg and overlap forms are
//            all evaluated and selected, so pedestrians and vehicles run the
//            same instructions (Sec. 3.1)
//   LP2      incremental closest-point LP over the half-planes and the speed
//            disc (Sec. 3)
//   LP3      least-penetration fallback when LP2 is infeasible (Sec. 3)
//   update   v' = LP result, p' = p + v' dt, written in caller order
//
// The half-planes of a lane live in LDS, one column per lane
// ([k][block] float4 = (q.x, q.y, d.x, d.y)), so the rolled LP loops index
// them dynamically without scratch memory.  Header-only: every translation
// unit instantiates the templates it launches.
#pragma once

#include "orca_internal.h"

#include <limits.h>
#include <math.h>

// Multiply-adds are fused within one expression only (C's FP_CONTRACT),
// never across statements: every instantiation of these templates (plain,
// batched, capped, adjoint recomputation) then rounds alike, which keeps
// their results equal bit for bit.
#pragma clang fp contract(on)

namespace orca {
namespace dev {

__device__ __forceinline__ float det2(float ax, float ay, float bx, float by)
{
    return ax * by - ay * bx;
}

__device__ __forceinline__ double det2(double ax, double ay, double bx, double by)
{
    return ax * by - ay * bx;
}

// The LP runs in float (LP2 over the agent's lines) or in double (LP3's
// sub-problems): these pick the operation of the scalar type.
__device__ __forceinline__ float lp_sqrt(float v) { return sqrtf(v); }
__device__ __forceinline__ double lp_sqrt(double v) { return sqrt(v); }
__device__ __forceinline__ float lp_abs(float v) { return fabsf(v); }
__device__ __forceinline__ double lp_abs(double v) { return fabs(v); }
__device__ __forceinline__ float lp_min(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double lp_min(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float lp_max(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double lp_max(double a, double b) { return fmax(a, b); }

template <class S>
struct LpVec;
template <>
struct LpVec<float> {
    using T = float4;
};
template <>
struct LpVec<double> {
    using T = double4;
};




// Squared distance in double from FP32 positions, each operation rounded
// separately (no fused multiply-add): the neighbour order is defined on it.
__device__ __forceinline__ double nb_key(float xi, float yi, float xj, float yj)
{
#pragma clang fp contract(off)
    const double dx = (double)xj - (double)xi;
    const double dy = (double)yj - (double)yi;
    return dx * dx + dy * dy;
}

// ---------------------------------------------------------------------------
// Exact k-nearest selection.
//
// Candidates are taken row by row from the cell stencil; each row is clipped
// to the chord of the neighbour circle at the row's nearest y (FP64, with a
// margin of 1e-6 cell on every bound, far above the rounding of the cell
// coordinates), so every agent with key < R_n^2 is visited.
//
// Pass 1 counts the in-range candidates of the lane in kBins bins of equal
// area (bin = floor(key * kBins / R_n^2), monotone in the key); a group of
// candidates adds to 4-bit fields of one 64-bit register, which are then
// widened into the 8-bit fields of two (even and odd bins).  The first bin
// b* at which the
// running count reaches k is the threshold: every candidate of a lower bin is
// among the k nearest and the rest of the k nearest lie in bin b*.
// Pass 2 visits only the circle that holds bins <= b* and appends their
// candidates to the lane's LDS column; a sorting network over registers then
// orders them.  Buffer entries are (float(key) bits << 32 | cell-order
// position): a strict order of the FP32-rounded keys implies the same order
// of the FP64 keys (rounding is monotone); equal FP32 keys among the entries
// that decide the result are resolved by an insertion pass that recomputes
// the FP64 keys and then compares the caller indices.
// A lane whose counts could overflow (> 255 in range) or whose candidates do
// not fit the buffer selects by repeated minimum instead (exact, slower).
// ---------------------------------------------------------------------------
constexpr int kBins = 16;

template <int K>
struct KnnShape {
    static constexpr int kSlots = K < 8 ? 8 : K;  // 16-byte LDS slots per lane
    static constexpr int kCap = 2 * kSlots;       // buffer entries per lane
};

// Widening of the kept K-th neighbour distance before the counting pass, in
// speed steps (v_max dt).  The result never depends on it (a circle holding
// fewer than K is rescanned whole); it trades rescans against candidates.
#ifndef ORCA_GUESS_SPEED_STEPS
#define ORCA_GUESS_SPEED_STEPS 2.0
#endif
constexpr double kGuessSpeedSteps = ORCA_GUESS_SPEED_STEPS;

// Hard lines of a vehicle's own motion limits: the acceleration octagon (see
// accel_line) and the two sides of the heading wedge (see turn_wedge).
constexpr int kAccLines = 8;
constexpr int kTurnLines = 2;

// Entry e of lane `tid` inside a [slot][BLOCK] float4 array viewed as u64.
// With several wavefronts per block, both entries of a 16-byte slot stay in
// the lane's own column tid: the buffer shares the LDS of the half-planes,
// and the wavefronts of a block run independently, so a lane that has
// reached its half-planes may only overwrite its own column (an
// [entry][BLOCK] layout would place a lane's entries in other lanes'
// columns, where a wavefront already writing half-planes corrupts one still
// selecting).  A block of one wavefront takes that [entry][BLOCK] layout
// (one address operation per entry instead of four): its lanes run in
// lockstep, so every lane has read its entries before any lane writes a
// half-plane, and lane_order() keeps the compiler from moving an LDS write
// across those phase boundaries.
template <int BLOCK>
__device__ __forceinline__ int buf_idx(int e, int tid)
{
    if (BLOCK == kWave) return e * BLOCK + tid;
    return (e >> 1) * (2 * BLOCK) + 2 * tid + (e & 1);
}

// Orders this lane's LDS accesses before and after it as seen by the other
// lanes of its wavefront (a compiler barrier; a one-wavefront block needs
// nothing more, its lanes execute together).
template <int BLOCK>
__device__ __forceinline__ void lane_order()
{
    if (BLOCK == kWave) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// Entry = (float(key) bits << 32) | (bin << 28) | cell-order position; the
// position needs 28 bits (at most 2^28 agents), the bin field is only read
// by the single-pass selection below.
constexpr uint32_t kPosBits = 28;
constexpr uint32_t kPosMask = (1u << kPosBits) - 1u;

__device__ __forceinline__ uint64_t pack_entry(double key, uint32_t t, uint32_t bin = 0u)
{
    return ((uint64_t)__float_as_uint((float)key) << 32) | (uint64_t)((bin << kPosBits) | t);
}

__device__ __forceinline__ uint32_t entry_pos(uint64_t e) { return (uint32_t)e & kPosMask; }
__device__ __forceinline__ uint32_t entry_bin(uint64_t e) { return (uint32_t)e >> kPosBits; }

// Strict (key, caller index) order of two buffer entries.
__device__ __forceinline__ bool entry_less(uint64_t ea, uint64_t eb, const float4 *__restrict__ s0,
                                           float xi, float yi)
{
    const uint32_t ha = (uint32_t)(ea >> 32), hb = (uint32_t)(eb >> 32);
    if (ha != hb) return ha < hb;
    const float4 ca = s0[entry_pos(ea)];
    const float4 cb = s0[entry_pos(eb)];
    const double ka = nb_key(xi, yi, ca.x, ca.y);
    const double kb = nb_key(xi, yi, cb.x, cb.y);
    if (ka != kb) return ka < kb;
    return __float_as_int(ca.z) < __float_as_int(cb.z);
}

// Candidates loaded per group by one lane.
#ifndef ORCA_SCAN_UNROLL
#define ORCA_SCAN_UNROLL 8
#endif
constexpr int kScanUnroll = ORCA_SCAN_UNROLL;
static_assert(kScanUnroll <= kScanPad, "candidate groups may read at most kScanPad past s0");

struct NoGroupEnd {
    __device__ __forceinline__ void operator()() const {}
};

// Grid rows that can hold an agent within sqrt(r2) of y (r2 <= R_n^2).
__device__ __forceinline__ void row_span(const GridMeta &g, double yd, double r2, int &ya, int &yb)
{
    const double r = sqrt(r2);
    const double ua = floor((yd - r - (double)g.y0) * g.inv_cs - 1e-6);
    const double ub = floor((yd + r - (double)g.y0) * g.inv_cs + 1e-6);
    ya = (int)fmin(fmax(ua, 0.0), (double)(g.ny - 1));
    yb = (int)fmin(fmax(ub, 0.0), (double)(g.ny - 1));
}

// Cell indices [xa, xb] of row yy's cells that meet the chord of the circle
// of squared radius r2 around (xd, yd) (FP64, with 1e-6-cell margins);
// false when the chord misses the row (xa = xb = the column of xd then).
// Returns the offsets of the two `start` entries that bound the row's range.
__device__ __forceinline__ bool row_cells(const GridMeta &g, double xd, double yd, double r2, int yy,
                                          int &ia, int &ib)
{
    const double ylo = (double)g.y0 + (double)yy * g.cs_d;
    const double dy = fmax(fmax(ylo - yd, yd - (ylo + g.cs_d)) - 1e-6 * g.cs_d, 0.0);
    const double h2 = r2 - dy * dy;
    const bool meets = h2 > 0.0;
    const double hw = meets ? sqrt(h2) : 0.0;
    const double ua = floor((xd - hw - (double)g.x0) * g.inv_cs - 1e-6);
    const double ub = floor((xd + hw - (double)g.x0) * g.inv_cs + 1e-6);
    const int xa = (int)fmin(fmax(ua, 0.0), (double)(g.nx - 1));
    const int xb = (int)fmin(fmax(ub, 0.0), (double)(g.nx - 1));
    const int row = g.cell_base + yy * g.nx;
    ia = row + xa;
    ib = row + xb + 1;
    return meets;
}

// Cell-order range of row yy clipped to the chord; false when empty.
__device__ __forceinline__ bool row_range(const GridMeta &g, const uint32_t *__restrict__ start,
                                          double xd, double yd, double r2, int yy, uint32_t &a,
                                          uint32_t &b)
{
    int ia, ib;
    if (!row_cells(g, xd, yd, r2, yy, ia, ib)) return false;
    a = start[ia];
    b = start[ib];
    if (b > g.seg_end) b = g.seg_end;  // defensive: stay inside the scene
    return a < b;
}

// Sorting network over N (a power of two) 64-bit keys held in registers,
// ascending; every index is a compile-time constant.
// Largest fixed-point sort key: 26 bits above the 6-bit buffer slot.
constexpr uint32_t kSortKeyMax = (1u << 26) - 1u;

template <int K>
struct SortNet {
    static constexpr int N = K <= 8 ? 16 : (K <= 24 ? 32 : 64);
};

template <int N>
__device__ __forceinline__ void cas(uint32_t (&e)[N], int i, int l)
{
    const uint32_t a = e[i], b = e[l];
    e[i] = a < b ? a : b;
    e[l] = a < b ? b : a;
}

// Batcher's odd-even merge sort (191 comparators for 32 keys against the
// bitonic network's 240); the loops run at compile time.
template <int N>
__device__ __forceinline__ void sort_network(uint32_t (&e)[N])
{
#pragma unroll
    for (int p = 1; p < N; p += p) {
#pragma unroll
        for (int k = p; k > 0; k /= 2) {
#pragma unroll
            for (int j = k % p; j + k < N; j += k + k) {
#pragma unroll
                for (int i = 0; i < k; ++i) {
                    if ((i + j) / (p + p) == (i + j + k) / (p + p)) cas<N>(e, i + j, i + j + k);
                }
            }
        }
    }
}

// Visits every candidate in the grid rows and chords of the circle of
// squared radius r2 around (xd, yd), row by row and in cell order within a
// row, in groups of kScanUnroll as group(c, t0, e): c[q] = s0[t0 + q], a
// member valid while t0 + q < e, the end of its row.  A group always loads
// all its members (the last one of a row reads up to kScanUnroll - 1
// entries past the row's end, inside s0 and its padding), so the visitor
// runs without a remainder loop and can stay branch-free.
//
// The loop runs over groups, not rows, with the memory one step ahead of
// the arithmetic: the next group -- the next one of the same row or the
// first one of the next row -- is loaded before the current one is visited,
// and a row's range is loaded from `start` one group before it is entered.
// Every lane issues both loads on every pass (a lane that stays in its row
// loads the same entries again), so the number of loads in flight is the
// same on every path and each wait covers only the data it needs.  In a
// dense crowd a row chord holds fewer candidates than one group, so a loop
// per row would wait for the memory at every row.  A row whose range turns
// out empty costs one group of invalid members.  Lanes step through their
// own rows, so a wave runs as many groups as its busiest lane.
template <class H>
__device__ __forceinline__ void scan_disc_groups(const GridMeta &g,
                                                 const uint32_t *__restrict__ start,
                                                 const float4 *__restrict__ s0, double xd,
                                                 double yd, double r2, H &&group)
{
    int yr, yb;
    row_span(g, yd, r2, yr, yb);
    // The range of row yr is loaded into one of two register pairs while the
    // other pair, loaded a pass earlier, is consumed (the two swap roles every
    // pass, so a load never lands in a register that is still being read);
    // rm: row yr's chord meets the row; (ia, ib): its `start` offsets.
    int ia, ib;
    bool rm = row_cells(g, xd, yd, r2, yr, ia, ib);
    uint32_t pa[2], pb[2];
    pa[0] = start[ia];
    pb[0] = start[ib];
    // the group after [t, t + kScanUnroll) of row [.., e): the next one of
    // the row, else the first one of row yr, whose range (pair P) is then
    // consumed and row yr + 1 requested; pair 1 - P is (re)loaded with the
    // range of the row requested now; false when no row is left
    auto next_group = [&](int P, uint32_t t, uint32_t e, uint32_t &tn, uint32_t &en) -> bool {
        const bool stay = t + kScanUnroll < e;
        bool live = true;
        if (stay) {
            tn = t + kScanUnroll;
            en = e;
        } else {
            live = yr <= yb;
            tn = pa[P];
            en = pb[P] < g.seg_end ? pb[P] : g.seg_end;  // defensive: stay inside the scene
            if (!rm || !(tn < en)) en = tn;              // an empty row: no valid member
            ++yr;
            if (yr <= yb) rm = row_cells(g, xd, yd, r2, yr, ia, ib);
        }
        pa[1 - P] = start[ia];
        pb[1 - P] = start[ib];
        return live;
    };
    // two register groups used in turn, so no group is copied; components a
    // visitor does not read are never loaded
    float4 c[kScanUnroll], d[kScanUnroll];
    uint32_t t0 = 0, e0 = 0;
    next_group(0, 0u, 0u, t0, e0);  // row yr exists: yr <= yb here
    {
        const float4 *pc = s0 + t0;
#pragma unroll
        for (int q = 0; q < kScanUnroll; ++q) c[q] = pc[q];
    }
    for (;;) {
        uint32_t t1, e1;
        const bool more1 = next_group(1, t0, e0, t1, e1);
        {
            const float4 *pd = s0 + (more1 ? t1 : t0);
#pragma unroll
            for (int q = 0; q < kScanUnroll; ++q) d[q] = pd[q];
        }
        // keep the loads ahead of the visit (the scheduler would otherwise
        // move them next to their use)
        __builtin_amdgcn_sched_barrier(0);
        group(c, t0, e0);
        if (!more1) break;
        const bool more2 = next_group(0, t1, e1, t0, e0);
        {
            const float4 *pc = s0 + (more2 ? t0 : t1);
#pragma unroll
            for (int q = 0; q < kScanUnroll; ++q) c[q] = pc[q];
        }
        __builtin_amdgcn_sched_barrier(0);
        group(d, t1, e1);
        if (!more2) break;
    }
    // the loads of the last pass are read on the way out too, so that the
    // compiler keeps each prefetch where it is written instead of moving it
    // behind the exit test, next to its use
#pragma unroll
    for (int q = 0; q < kScanUnroll; ++q)
        asm volatile("" ::"v"(c[q].x), "v"(c[q].y), "v"(d[q].x), "v"(d[q].y));
}

// The same scan with a visitor per candidate: visit(c, t, valid) for each
// member of a group, then group_end().
template <class F, class G = NoGroupEnd>
__device__ __forceinline__ void scan_disc(const GridMeta &g, const uint32_t *__restrict__ start,
                                          const float4 *__restrict__ s0, double xd, double yd,
                                          double r2, F &&visit, G &&group_end = G())
{
    scan_disc_groups(g, start, s0, xd, yd, r2,
                     [&](const float4 (&c)[kScanUnroll], uint32_t t0, uint32_t e) {
#pragma unroll
                         for (int q = 0; q < kScanUnroll; ++q) visit(c[q], t0 + q, t0 + q < e);
                         group_end();
                     });
}

// Selects the (at most K) nearest agents of the lane into entries [0, m) of
// its LDS buffer, ascending; returns m.  rg2 (<= R_n^2) is a guess of a
// squared radius that holds at least K candidates (from the previous step):
// the counting pass first covers only that circle and falls back to the
// whole neighbour circle when it holds fewer than K, so the result never
// depends on the guess.
template <int K, int BLOCK>
__device__ int knn_select(const GridMeta &g, const uint32_t *__restrict__ start,
                          const float4 *__restrict__ s0, float xi, float yi, int self,
                          uint32_t spos, uint64_t *buf, int tid, double rg2)
{
    constexpr int kCap = KnnShape<K>::kCap;
    const double xd = xi, yd = yi;
    lane_order<BLOCK>();  // other lanes' half-planes of a previous tile are read
    // pass 1: per-bin counts of the keys below r2c in kBins equal-area bins,
    // and the candidates themselves while they fit the buffer.  The lane's
    // own agent is counted (and stored) too -- it is always scanned, with
    // key 0, in bin 0 -- and taken out afterwards, which keeps the index
    // test out of this loop.
    double r2c = rg2 < g.rn2 ? rg2 : g.rn2;
    double bscale;
    // Counts per bin: 4-bit counters of one group of candidates in `nib`
    // (a group adds at most kScanUnroll <= 15 to a bin), widened after each
    // group into byte counters, even bins in `hev` (byte k: bin 2k) and odd
    // bins in `hod` (byte k: bin 2k + 1); bytes cannot overflow either, since
    // a lane with more than 255 candidates takes the exact fallback below.
    static_assert(kScanUnroll <= 15, "a group must fit the 4-bit counters");
    uint64_t hev, hod, nib;
    uint32_t total;
    for (;;) {
        bscale = (double)kBins / r2c;
        hev = 0;
        hod = 0;
        nib = 0;
        total = 0;
        scan_disc_groups(
            g, start, s0, xd, yd, r2c,
            [&](const float4 (&c)[kScanUnroll], uint32_t t0, uint32_t e) {
                // the keys of the whole group first (independent of one
                // another, so their FP64 chains interleave), then the
                // counters and the buffer in member order
                double key[kScanUnroll];
                int bin[kScanUnroll];
                bool in[kScanUnroll];
#pragma unroll
                for (int q = 0; q < kScanUnroll; ++q) {
                    key[q] = nb_key(xi, yi, c[q].x, c[q].y);
                    in[q] = t0 + q < e && key[q] < r2c;
                    // equals min((int)(key * bscale), kBins - 1) for every
                    // key, and is defined also for the far (or invalid)
                    // candidates it is not used for
                    bin[q] = (int)fmin(key[q] * bscale, (double)(kBins - 1));
                }
#pragma unroll
                for (int q = 0; q < kScanUnroll; ++q) {
                    nib += (uint64_t)(in[q] ? 1u : 0u) << (bin[q] * 4);
                    // branch-free, so that the candidates of a group form one
                    // block: every candidate is written at the next free slot
                    // and kept only when in range; once the buffer is full the
                    // writes land on its last slot, the only one they can
                    // overwrite
                    const int slot = total < (uint32_t)(kCap - 1) ? (int)total : kCap - 1;
                    buf[buf_idx<BLOCK>(slot, tid)] = pack_entry(key[q], t0 + q, (uint32_t)bin[q]);
                    total += in[q] ? 1u : 0u;
                }
                hev += nib & 0x0F0F0F0F0F0F0F0Full;
                hod += (nib >> 4) & 0x0F0F0F0F0F0F0F0Full;
                nib = 0;
            });
        hev -= 1ull;  // the lane's own entry, key 0, bin 0
        total -= 1u;
        if (total >= (uint32_t)K || !(r2c < g.rn2)) break;
        r2c = g.rn2;  // the guessed circle holds fewer than K: count them all
    }
    // every candidate of the circle (and the lane's own entry) is in the
    // buffer, below its last slot
    const bool captured = total + 1u <= (uint32_t)(kCap - 1);

    // threshold bin b*: the first bin at which the cumulative count reaches K
    uint32_t cum = 0, take = 0;
    int bstar = kBins - 1;
    bool found = false;
#pragma unroll
    for (int b = 0; b < kBins; ++b) {
        cum += (uint32_t)((((b & 1) ? hod : hev) >> ((b >> 1) * 8)) & 0xffull);
        if (!found && cum >= (uint32_t)K) {
            found = true;
            bstar = b;
            take = cum;
        }
    }
    if (!found) take = total;

    if (total <= 255u && take <= (uint32_t)kCap) {
        if (captured) {
            // the candidates of bins <= b* are already in the buffer: keep
            // them in place, dropping the lane's own entry.  Branch-free: each
            // entry is written at the next kept position, which never passes
            // the one being read, and the position advances only for kept
            // entries
            uint32_t w = 0;
            for (uint32_t e = 0; e <= total; ++e) {
                const uint64_t ent = buf[buf_idx<BLOCK>((int)e, tid)];
                buf[buf_idx<BLOCK>((int)w, tid)] = ent;
                w += (entry_pos(ent) != spos && (int)entry_bin(ent) <= bstar) ? 1u : 0u;
            }
        } else {
            // pass 2: collect the candidates of bins <= b*, in scan order.  For
            // b* below the last bin, bin <= b* is exactly key * bscale < b* + 1
            // (truncation of a non-negative value), so both passes count alike.
            // Every such key is below (b* + 1) R_n^2 / kBins, so only rows and
            // chords of that smaller circle are visited (with a relative margin
            // far above the rounding of key * bscale).
            const bool last = bstar + 1 >= kBins;
            const double bnext = last ? INFINITY : (double)(bstar + 1);
            const double r2 = last ? r2c : (double)(bstar + 1) * (r2c / (double)kBins) * (1.0 + 1e-9);
            uint32_t slot = 0;
            scan_disc(g, start, s0, xd, yd, r2, [&](const float4 &c, uint32_t t, bool valid) {
                const double key = nb_key(xi, yi, c.x, c.y);
                if (valid && key < r2c && key * bscale < bnext && __float_as_int(c.z) != self) {
                    if (slot < (uint32_t)kCap)  // always true: both passes count alike
                        buf[buf_idx<BLOCK>((int)slot, tid)] = pack_entry(key, t);
                    ++slot;
                }
            });
        }
        // order: a sorting network in registers when the entries fit it,
        // over 32-bit words (the FP32 key in 26-bit fixed point of r2c, above
        // the entry's buffer slot); the nearest K entries are then gathered
        // by slot.  The fixed-point key is non-decreasing in the FP32 key,
        // which is non-decreasing in the FP64 key, so distinct fixed-point
        // keys are in (FP64 key) order; a tie among the entries that decide
        // the result needs the (FP64 key, caller index) order of entry_less,
        // left to the insertion pass below (the buffer is then untouched).
        constexpr int N = SortNet<K>::N;
        static_assert(N <= 64, "buffer slots must fit six bits");
        bool sorted = false;
        if (take <= (uint32_t)N) {
            const float qscale = 67108864.0f / (float)r2c;  // 2^26 / r2c
            uint32_t e[N];
#pragma unroll
            for (int p = 0; p < N; ++p) {
                uint32_t w = ~0u;
                if (p < (int)take) {
                    const float fk = __uint_as_float(
                        (uint32_t)(buf[buf_idx<BLOCK>(p, tid)] >> 32));
                    // clamp in the integer domain: the FP32 product reaches
                    // 2^26 for keys within a few 1e-8 (relative) below r2c,
                    // and 2^26 - 1 has no FP32 value to clamp to
                    const uint32_t q = min((uint32_t)(fk * qscale), kSortKeyMax);
                    w = (q << 6) | (uint32_t)p;
                }
                e[p] = w;
            }
            sort_network<N>(e);
            bool tie = false;
#pragma unroll
            for (int p = 0; p + 1 < N; ++p)
                tie = tie || (p < K && p + 1 < (int)take && (e[p] >> 6) == (e[p + 1] >> 6));
            if (!tie) {
                uint64_t got[K];
#pragma unroll
                for (int p = 0; p < K; ++p)
                    if (p < (int)take) got[p] = buf[buf_idx<BLOCK>((int)(e[p] & 63u), tid)];
#pragma unroll
                for (int p = 0; p < K; ++p)
                    if (p < (int)take) buf[buf_idx<BLOCK>(p, tid)] = got[p];
                sorted = true;
            }
        }
        if (!sorted) {
            for (int p = 1; p < (int)take; ++p) {
                const uint64_t e = buf[buf_idx<BLOCK>(p, tid)];
                int q = p - 1;
                while (q >= 0) {
                    const uint64_t f = buf[buf_idx<BLOCK>(q, tid)];
                    if (!entry_less(e, f, s0, xi, yi)) break;
                    buf[buf_idx<BLOCK>(q + 1, tid)] = f;
                    --q;
                }
                buf[buf_idx<BLOCK>(q + 1, tid)] = e;
            }
        }
        return take < (uint32_t)K ? (int)take : K;
    }

    // fallback: repeated minimum over all candidates, strictly above the last pick
    int ya, yb;
    row_span(g, yd, g.rn2, ya, yb);
    double lk = -1.0;
    int lj = -1;
    int m = 0;
    for (; m < K; ++m) {
        double bk = INFINITY;
        int bj = INT_MAX;
        uint32_t bt = 0;
        for (int yy = ya; yy <= yb; ++yy) {
            uint32_t ra, rb;
            if (!row_range(g, start, xd, yd, g.rn2, yy, ra, rb)) continue;
            for (uint32_t t = ra; t < rb; ++t) {
                const float4 c = s0[t];
                const int j = __float_as_int(c.z);
                const double key = nb_key(xi, yi, c.x, c.y);
                const bool above = key > lk || (key == lk && j > lj);
                const bool below = key < bk || (key == bk && j < bj);
                if (key < g.rn2 && j != self && above && below) {
                    bk = key;
                    bj = j;
                    bt = t;
                }
            }
        }
        if (bj == INT_MAX) break;
        buf[buf_idx<BLOCK>(m, tid)] = pack_entry(bk, bt);
        lk = bk;
        lj = bj;
    }
    return m;
}

// |P|^2 - R^2 of two agents, in double from their FP32 positions and radii
// (the differences and the sum are exact there, the products nearly so): the
// contact test |P| > R and the length of the legs' tangent, sqrt(|P|^2 - R^2),
// which FP32 would form with a cancellation of its own rounding error when
// the two discs almost touch.
__device__ __forceinline__ double clearance2(float pax, float pay, float ra, float pbx, float pby,
                                             float rb)
{
    const double px = (double)pbx - (double)pax, py = (double)pby - (double)pay;
    const double r = (double)ra + (double)rb;
    return px * px + py * py - r * r;
}

// ORCA_{A|B} as (q.x, q.y, d.x, d.y); permitted side det(d, v - q) >= 0.
// P = p_B - p_A, V = v_A - v_B, R = r_A + r_B.
//  - not overlapping: w = V - P/tau; the cutoff arc is nearest when the angle
//    between w and -P is below arccos(R/|P|), else the left leg (det(P,w) > 0)
//    or the right leg; u is the shortest vector from V to the boundary and n
//    the outward normal there.
//  - overlapping (|P| <= R): the horizon becomes dt and only the disc is used;
//    w = 0 takes the normal (+1, 0) if A's caller index is the smaller one,
//    else (-1, 0).
//  - q = v_A + f u, d = (n.y, -n.x).  q is kept as this sum: with f = 0 all
//    of an agent's lines then pass exactly through v_A, so a feasible set that
//    has shrunk to that single point stays feasible in FP32.
__device__ __forceinline__ float4 halfplane(float pax, float pay, float vax, float vay, float ra,
                                            float pbx, float pby, float vbx, float vby, float rb,
                                            float f, float inv_tau, float inv_dt, bool a_first)
{
    const float Px = pbx - pax, Py = pby - pay;
    const float Vx = vax - vbx, Vy = vay - vby;
    const float R = ra + rb;
    const float dist2 = Px * Px + Py * Py;
    const float R2 = R * R;
    const double c2 = clearance2(pax, pay, ra, pbx, pby, rb);
    const bool overlap = !(c2 > 0.0);
    const float it = overlap ? inv_dt : inv_tau;
    const float wx = Vx - Px * it, wy = Vy - Py * it;
    const float w2 = wx * wx + wy * wy;
    const float wp = wx * Px + wy * Py;
    const bool arc = overlap || (wp < 0.0f && wp * wp > R2 * w2);
    // disc (cutoff arc / overlap) form
    const bool wz = !(w2 > 0.0f);
    const float wl = sqrtf(w2);
    const float iwl = wz ? 0.0f : 1.0f / wl;
    const float anx = wz ? (a_first ? 1.0f : -1.0f) : wx * iwl;
    const float any = wz ? 0.0f : wy * iwl;
    const float ul = R * it - wl;
    float nx = anx, ny = any, ux = ul * anx, uy = ul * any;
    // leg form, only where a lane of the wavefront needs it (in dense flows
    // most half-planes take the cutoff arc: relative velocities are small)
    if (__any(!arc)) {
        const float leg = sqrtf(fmaxf((float)c2, 0.0f));
        const float id2 = overlap ? 0.0f : 1.0f / dist2;
        const bool left = det2(Px, Py, wx, wy) > 0.0f;
        const float sR = left ? R : -R;
        const float ex = (Px * leg - Py * sR) * id2;
        const float ey = (Px * sR + Py * leg) * id2;
        const float lnx = left ? -ey : ey;
        const float lny = left ? ex : -ex;
        const float s = Vx * ex + Vy * ey;
        nx = arc ? nx : lnx;
        ny = arc ? ny : lny;
        ux = arc ? ux : s * ex - Vx;
        uy = arc ? uy : s * ey - Vy;
    }
    return make_float4(vax + f * ux, vay + f * uy, ny, -nx);
}

// Acceleration limit (Sec. 5: acceleration-limited vehicles add linear
// constraints of their own motion to the same LP).  Within one step the
// velocity may change by at most a dt: the new velocity must lie in the
// regular octagon inscribed in the disc of radius a dt about c, the current
// velocity scaled onto the speed circle when it lies outside it (so the
// octagon and the speed disc always meet).  Edge k has outward normal n_k at
// angle k pi/4 at distance h = a dt cos(pi/8) from c; as a line,
// q = c + h n_k, d = (-n_k.y, n_k.x).  The lines are hard constraints: they
// precede the ORCA lines in LP2 and LP3 never relaxes them.
__device__ __forceinline__ void accel_centre(float vx, float vy, float vmax, float &cx, float &cy)
{
    const float v2 = vx * vx + vy * vy;
    const float sc = v2 > vmax * vmax ? vmax / sqrtf(v2) : 1.0f;
    cx = vx * sc;
    cy = vy * sc;
}

// Distance of the octagon's edges from its centre, a dt cos(pi/8).
__device__ __forceinline__ float accel_half_width(float acc, float dt)
{
    return acc * dt * 0.92387953f;
}

// cos(k pi/4) for k in 0..7, exactly 0, +-1 or +-0.70710678f.
__device__ __forceinline__ float cos_quarter(int k)
{
    const int m = k & 7;
    const float mag = (m & 1) ? 0.70710678f : ((m & 2) ? 0.0f : 1.0f);
    return (m >= 3 && m <= 5) ? -mag : mag;
}

// Acceleration line k, generated where it is read (no LDS): q = c + h n_k
// with single-rounding fmaf, so every read of a line gives the same bits.
__device__ __forceinline__ float4 accel_line(int k, float cx, float cy, float h)
{
    const float nx = cos_quarter(k), ny = cos_quarter(k + 6);  // sin(x) = cos(x - pi/2)
    return make_float4(fmaf(h, nx, cx), fmaf(h, ny, cy), -ny, nx);
}

// Turn-rate limit (the non-holonomic half of the same Sec. 5 extension): a
// vehicle moves along its heading, the direction of its current velocity,
// and turns it by at most w dt per step, so the new velocity lies in the
// wedge of half-angle phi = min(w dt, pi/2) about the heading, apex at the
// origin.  Its sides are the lines through the origin with directions
// r_R = R(-phi) h and -r_L = -R(phi) h (permitted side on the left), hard
// constraints after any acceleration lines.  Returns false at rest (no
// heading, no wedge).  The heading is formed in double, so that a speed
// whose square underflows FP32 still has one.
// The heading h = v/|v| and the wedge's cos(phi), sin(phi); false at rest.
// `speed` is |v| (for the adjoint's Jacobian of h).
__device__ __forceinline__ bool turn_basis(float vx, float vy, float turn, float dt, float &hx,
                                           float &hy, float &cs, float &sn, float &speed)
{
    const double v2 = (double)vx * vx + (double)vy * vy;
    if (!(turn > 0.0f) || !(v2 > 0.0)) return false;
    const double sp = sqrt(v2);
    const double inv = 1.0 / sp;
    hx = (float)(vx * inv);
    hy = (float)(vy * inv);
    speed = (float)sp;
    const float phi = fminf(turn * dt, 1.57079633f);
    sincosf(phi, &sn, &cs);
    return true;
}

__device__ __forceinline__ bool turn_wedge(float vx, float vy, float turn, float dt, float &rx,
                                           float &ry, float &lx, float &ly)
{
    float hx, hy, cs, sn, speed;
    if (!turn_basis(vx, vy, turn, dt, hx, hy, cs, sn, speed)) return false;
    rx = hx * cs + hy * sn;
    ry = hy * cs - hx * sn;
    lx = -(hx * cs - hy * sn);
    ly = -(hy * cs + hx * sn);
    return true;
}

// The lines of this lane's LP: with ACC the first nh are hard -- nacc
// acceleration lines (generated from the centre (cx, cy) and half-width h),
// then the wedge sides (through the origin, directions (rx, ry), (lx, ly))
// -- followed by the half-planes, stored in LDS column `tid`.
template <int BLOCK, bool ACC = false>
struct LdsLines {
    const float4 *L;
    int tid;
    int nh = 0;
    float cx = 0.0f, cy = 0.0f, h = 0.0f;
    int nacc = kAccLines;
    float rx = 0.0f, ry = 0.0f, lx = 0.0f, ly = 0.0f;
    __device__ __forceinline__ float4 line(int j) const
    {
        if (!ACC) return L[j * BLOCK + tid];
        // a select, not a branch: the LP code around keeps the control flow
        // (and so the multiply-add fusion) of the kernel without caps, and an
        // agent without a cap gets the same bits from both kernels
        const float4 s = L[(j >= nh ? j - nh : 0) * BLOCK + tid];
        const float4 a = accel_line(j, cx, cy, h);
        const bool right = j == nacc;
        const float wx = right ? rx : lx, wy = right ? ry : ly;
        const bool hard = j < nh, oct = j < nacc;
        return make_float4(hard ? (oct ? a.x : 0.0f) : s.x, hard ? (oct ? a.y : 0.0f) : s.y,
                           hard ? (oct ? a.z : wx) : s.z, hard ? (oct ? a.w : wy) : s.w);
    }
    __device__ __forceinline__ bool get(int j, float4 &l) const
    {
        l = line(j);
        return true;
    }
};

// Boundaries of "delta_j(v) <= delta_i(v)" for j < i (least-penetration
// sub-problem), recomputed on demand from lines i and j.  Lines parallel to i
// and pointing the same way are not constraints (invalid).  With ACC the
// first nh lines are hard (acceleration lines) and are passed on unchanged.
// Since delta_j(v) - delta_i(v) = c - det(e, v) with e = d_j - d_i and
// c = det(d_j, q_j) - det(d_i, q_i), the boundary is det(e/|e|, v) = c/|e|;
// it is stored through its point nearest the origin, (c/|e|) (-e_y, e_x)/|e|.
// This is the same line as the one through the intersection of lines i and j
// (or the midpoint of q_i, q_j for antiparallel lines), but stays well
// scaled in FP32 when the two lines are nearly parallel and intersect far
// away from the speed disc.  Two lines with the same point q pass through it
// together, and so does their boundary: it keeps q itself as its point.
template <int BLOCK, bool ACC = false>
struct ProjLines {
    const LdsLines<BLOCK, ACC> &ls;
    float4 li;
    float ci;    // det(d_i, q_i)
    float eps;
    // Computes the boundary without a branch on the line; returns false when
    // it is not a constraint (its components are then meaningless).
    __device__ __forceinline__ bool get(int j, float4 &out) const
    {
        const float4 lj = ls.line(j);
        if (ACC && j < ls.nh) {
            out = lj;
            return true;
        }
        const float dij = det2(li.z, li.w, lj.z, lj.w);
        const bool same = fabsf(dij) <= eps && li.z * lj.z + li.w * lj.w > 0.0f;
        const float ex = lj.z - li.z, ey = lj.w - li.w;
        const float il = 1.0f / sqrtf(ex * ex + ey * ey);
        const float dx = ex * il, dy = ey * il;
        const float off = (det2(lj.z, lj.w, lj.x, lj.y) - ci) * il;
        // Lines through one point (the f = 0 lines of an agent all pass
        // exactly through its velocity) have their boundary through that same
        // point: it is kept exactly, so that an LP whose feasible region is a
        // cone with its apex there (or that apex alone) decides feasibility
        // at the apex exactly, as the oracle's intersection form does.
        const bool common = lj.x == li.x && lj.y == li.y;
        out = make_float4(common ? li.x : -dy * off, common ? li.y : dx * off, dx, dy);
        return !same;
    }
};


// The same boundaries in double, for a sub-problem that failed in FP32: the
// boundary passes through the intersection of lines i and j (the midpoint
// of q_i and q_j when they are antiparallel) with direction
// (d_j - d_i) / |d_j - d_i|.  Such a sub-problem always has a solution in
// exact arithmetic (the current point lies in its region), so its failure
// means a feasible set thinner than FP32 resolves: several lines through
// one vertex, the f = 0 lines that all meet at the agent's own velocity, an
// apex on the speed circle.  In double it is decided as the oracle decides.
template <int BLOCK, bool ACC = false>
struct ProjLinesD {
    const LdsLines<BLOCK, ACC> &ls;
    double4 li;
    double eps;
    // Computes the boundary without a branch on the line; returns false when
    // it is not a constraint (its components are then meaningless).
    __device__ __forceinline__ bool get(int j, double4 &out) const
    {
        const float4 l = ls.line(j);
        const double4 lj = make_double4(l.x, l.y, l.z, l.w);
        if (ACC && j < ls.nh) {
            out = lj;
            return true;
        }
        const double dij = det2(li.z, li.w, lj.z, lj.w);
        const bool par = fabs(dij) <= eps;
        const bool same = par && li.z * lj.z + li.w * lj.w > 0.0;
        const double t = det2(lj.z, lj.w, li.x - lj.x, li.y - lj.y) / dij;
        const double px = par ? 0.5 * (li.x + lj.x) : li.x + t * li.z;
        const double py = par ? 0.5 * (li.y + lj.y) : li.y + t * li.w;
        const double ex = lj.z - li.z, ey = lj.w - li.w;
        const double il = 1.0 / sqrt(ex * ex + ey * ey);
        out = make_double4(px, py, ex * il, ey * il);
        return !same;
    }
};

// The boundaries of one least-penetration sub-problem, cached in the LDS
// column of a lane of the same wavefront that runs no LP3 (its half-planes
// are not read again once its LP2 is done): lp3 computes the boundaries
// j < i of line i once, and the lp1 calls of the sub-problem read them
// instead of recomputing every one at each re-solve.  A cached boundary is
// the value ProjLines computes (multiply-adds are fused within an expression
// only, so it has the bits of one computed where it is used), so the result
// is the same bit for bit with or without a column; a lane without one (a
// wavefront with more lanes in LP3 than not) computes on demand.
template <int BLOCK, bool ACC>
struct CachedProj {
    const ProjLines<BLOCK, ACC> &pl;
    const float4 *L;  // the workgroup's [slot][BLOCK] array
    int col;          // cache column, or -1
    uint32_t valid;   // bit j: boundary j is a constraint
    __device__ __forceinline__ bool get(int j, float4 &out) const
    {
        if (col >= 0) {
            out = L[j * BLOCK + col];
            return (valid >> j) & 1u;
        }
        return pl.get(j, out);
    }
};

// The cache column of this lane for lp3 (CachedProj): the r-th lane of the
// wavefront that needs LP3 (in lane order) takes the column of the r-th lane
// that does not; -1 without one.  Every active lane of the wavefront calls
// it, after its LP2.  Only for callers whose lanes read none of their own
// half-planes after LP2: the step does not, the adjoint's recomputation does
// (its VJP reads the lines of the active set) and so takes no cache.
template <int BLOCK>
__device__ __forceinline__ int lp3_cache_column(bool need, int tid)
{
    const uint64_t needm = __ballot(need);
    uint64_t spare = __ballot(!need);
    const int lane = tid & (kWave - 1);
    int col = -1;
    if (need) {
        int r = __popcll(needm & ((1ull << lane) - 1ull));
        if (r < __popcll(spare)) {
            for (; r > 0; --r) spare &= spare - 1ull;
            col = (tid - lane) + __builtin_ctzll(spare);
        }
    }
    // the owners' last reads of those columns (their LP2) stay before the
    // cache writes of other lanes
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    return col;
}

// The constraints that define an LP result (its active set), recorded by
// the adjoint's recomputation of the step.  LP2 results: kFree (v = v_pref),
// kDisc (v_pref scaled onto the speed circle), kLine (projection of v_pref
// onto line a), kLineLine (intersection of lines a and b), kLineDisc (line a
// on the speed circle).  LP3 results, for the line i3 whose penetration was
// minimised last: kDir (v_max times i3's inward normal), kProjDisc (the
// equal-penetration boundary of a and i3 on the circle), kProjProj (the
// point of equal penetration of a, b and i3), kTie (v_pref projected onto
// the boundary of a and i3); with acceleration lines, a or b below their
// count stands for that hard line itself instead of a boundary.  kCentre:
// the acceleration octagon's centre (LP2 failed on a hard line).
enum ActiveKind {
    kFree = 0,
    kDisc,
    kLine,
    kLineLine,
    kLineDisc,
    kDir,
    kProjDisc,
    kProjProj,
    kTie,
    kCentre
};

struct ActiveSet {
    int kind;
    int i3;
    int a, b;
};

// What the LP's scalar type resolves in a velocity, relative to v_max (about
// 16 ulps): the slack of lp1's interval test and the least excess over
// LP3's level that makes a line be re-solved.
template <class S>
struct FeasSlack;
template <>
struct FeasSlack<float> {
    static constexpr float v = 0x1p-20f;
};
template <>
struct FeasSlack<double> {
    static constexpr double v = 0x1p-49;
};

// One-dimensional sub-problem on line li (index i): the parameter interval
// inside the speed disc and on the permitted side of every valid line j < i.
// mode 0: closest point to (ox, oy); mode 1: extreme along unit (ox, oy), or,
// when the line is orthogonal to it, the point closest to (tx, ty).
// `how` reports what fixed the result: 0 projection, 1 / 2 the lower / upper
// end of the interval (bounded by line `src`, or by the disc when src < 0),
// 3 the tie projection.
template <class S, class Src>
__device__ __forceinline__ bool lp1(const Src &src, int i, typename LpVec<S>::T li, S vmax,
                                    int mode, S ox, S oy, S tx, S ty, S eps, S &x, S &y, int &how,
                                    int &bound)
{
    using V4 = typename LpVec<S>::T;
    // The line meets the speed circle at t^2 + 2 dot t + c = 0, c = |q|^2 -
    // v_max^2.  c is formed in double (exact products), so its sign -- whether
    // q itself lies in the disc -- is exact; the root near q is taken as c
    // over the other root, which has no cancellation, so q stays inside the
    // interval exactly when it lies in the disc (the f = 0 lines of an agent
    // pass through its own velocity, which the grid build puts inside the
    // disc: that apex is then a feasible point, as it is exactly).
    const S dot = li.x * li.z + li.y * li.w;
    const double cd = (double)li.x * (double)li.x + (double)li.y * (double)li.y -
                      (double)vmax * (double)vmax;
    const S c = (S)cd;
    const S disc = dot * dot - c;
    if (disc < (S)0) return false;
    const S sq = lp_sqrt(disc);
    const S far = dot > (S)0 ? -dot - sq : -dot + sq;
    const S near = far != (S)0 ? c / far : (S)0;
    S tl = lp_min(far, near), tr = lp_max(far, near);
    int sl = -1, sr = -1;
    // Branch-free over j: the lanes of a wavefront meet different cases
    // (parallel, lower or upper bound) at the same j, so every case is a
    // select.  The interval only shrinks, so a failure at some j is a
    // failure at the end: it is recorded in `ok` instead of returning.
    // An interval empty by less than the scalar type resolves at this
    // velocity scale (FeasSlack v_max) counts as one point: a feasible set
    // that thin --
    // several lines through one vertex, an apex on the speed circle -- is
    // empty or not by rounding alone, and the point found then violates a
    // constraint by no more than that.
    const S slack = vmax * FeasSlack<S>::v;
    // Lines parallel within eps are one line when line i is offset to j's
    // forbidden side by no more than 2^-20 v_max (far below what the FP32
    // positions resolve), else disjoint; the same offset in either precision
    // and in the FP64 reference.
    const S pslack = vmax * (S)0x1p-20;
    bool ok = true;
    for (int j = 0; j < i; ++j) {
        V4 lj;
        const bool valid = src.get(j, lj);
        const S a = det2(lj.z, lj.w, li.z, li.w);
        const S b = det2(lj.z, lj.w, li.x - lj.x, li.y - lj.y);
        const bool par = lp_abs(a) <= eps;
        const S t = -b / a;
        const bool cut = valid && !par;
        const bool lo = cut && a > (S)0 && t > tl;
        const bool hi = cut && !(a > (S)0) && t < tr;
        tl = lo ? t : tl;
        sl = lo ? j : sl;
        tr = hi ? t : tr;
        sr = hi ? j : sr;
        ok = ok && !(valid && par && b < -pslack) && !(tl > tr + slack);
    }
    if (!ok) return false;
    S t;
    if (mode == 0) {
        t = li.z * (ox - li.x) + li.w * (oy - li.y);
        how = 0;
    } else {
        const S sd = ox * li.z + oy * li.w;
        if (lp_abs(sd) <= eps) {
            t = li.z * (tx - li.x) + li.w * (ty - li.y);
            how = 3;
        } else {
            t = sd > (S)0 ? tr : tl;
            how = sd > (S)0 ? 2 : 1;
        }
    }
    if (t < tl) {
        t = tl;
        how = 1;
    }
    if (t > tr) {
        t = tr;
        how = 2;
    }
    bound = how == 1 ? sl : (how == 2 ? sr : -1);
    x = li.x + t * li.z;
    y = li.y + t * li.w;
    return true;
}

// Incremental 2D LP over lines 0..m-1 of `src` and the disc |v| <= vmax.
// Returns the first infeasible line, or m; v keeps its pre-failure value.
// With REC the active set of the result is written to *rec.
template <bool REC, class S, class Src>
__device__ __forceinline__ int lp2(const Src &src, int m, S vmax, int mode, S ox, S oy, S tx,
                                   S ty, S eps, S &vx, S &vy, ActiveSet *rec)
{
    S x, y;
    if (mode == 1) {
        x = ox * vmax;
        y = oy * vmax;
        if (REC) rec->kind = kDir;
    } else {
        const S o2 = ox * ox + oy * oy;
        if (o2 > vmax * vmax) {
            const S sc = vmax / lp_sqrt(o2);
            x = ox * sc;
            y = oy * sc;
            if (REC) rec->kind = kDisc;
        } else {
            x = ox;
            y = oy;
            if (REC) rec->kind = kFree;
        }
    }
    for (int i = 0; i < m; ++i) {
        typename LpVec<S>::T li;
        const bool valid = src.get(i, li);
        if (valid && det2(li.z, li.w, li.x - x, li.y - y) > (S)0) {
            S nx = x, ny = y;
            int how, bound;
            if (!lp1<S>(src, i, li, vmax, mode, ox, oy, tx, ty, eps, nx, ny, how, bound)) {
                vx = x;
                vy = y;
                return i;
            }
            x = nx;
            y = ny;
            if (REC) {
                rec->a = i;
                rec->b = bound;
                if (mode == 0)
                    rec->kind = how == 0 ? kLine : (bound >= 0 ? kLineLine : kLineDisc);
                else
                    rec->kind = how == 3 ? kTie : (bound >= 0 ? kProjProj : kProjDisc);
            }
        }
    }
    vx = x;
    vy = y;
    return m;
}


// Least penetration (Sec. 3): from LP2's partial result at line `fail`, each
// later line i whose penetration exceeds the current level re-solves v in the
// region where no earlier line penetrates more than line i, as deep into line
// i's permitted side as possible.  With ACC the first nh lines are hard: never
// relaxed, they bound every re-solve as they are.
// `col`: a cache column for the sub-problems' boundaries (lp3_cache_column;
// only without hard lines), or -1.
template <bool REC, int BLOCK, bool ACC = false>
__device__ __forceinline__ void lp3(const LdsLines<BLOCK, ACC> &ls, int m, int fail, float vmax,
                                    float tx, float ty, float eps, float &vx, float &vy,
                                    ActiveSet *rec, int col = -1)
{
    static_assert(ORCA_K_MAX <= 32, "the cache's validity bits are one 32-bit word");
    float level = 0.0f;
    float x = vx, y = vy;
    const int nhard = ACC ? ls.nh : 0;
    // a line is re-solved only when it exceeds the level by more than FP32
    // resolves in a penetration (about 2^-20 v_max): at a point where several
    // lines are penetrated equally, FP32 rounding alone would otherwise
    // decide whether a later tied line triggers a re-solve, and the re-solve
    // then jumps to another vertex of the tie
    const float tol = vmax * FeasSlack<float>::v;
    // as in lp2: each lane steps on to its own next line above the level, and
    // the lanes re-solve together
    int i = fail > nhard ? fail : nhard;
    for (;;) {
        float4 li;
        for (; i < m; ++i) {
            li = ls.line(i);
            if (det2(li.z, li.w, li.x - x, li.y - y) > level + tol) break;
        }
        if (i >= m) break;
        ProjLines<BLOCK, ACC> src{ls, li, det2(li.z, li.w, li.x, li.y), eps};
        uint32_t valid = 0;
        if (!ACC && col >= 0) {
            float4 *C = const_cast<float4 *>(ls.L);
            for (int j = 0; j < i; ++j) {
                float4 b;
                valid |= (src.get(j, b) ? 1u : 0u) << j;
                C[j * BLOCK + col] = b;
            }
        }
        const CachedProj<BLOCK, ACC> cs{src, ls.L, ACC ? -1 : col, valid};
        float nx = x, ny = y;
        ActiveSet inner;
        bool solved = lp2<REC, float>(cs, i, vmax, 1, -li.w, li.z, tx, ty, eps, nx, ny,
                                      &inner) == i;
        if (!solved) {
            // failed in FP32 only: solve it again in double (ProjLinesD)
            const double4 lid = make_double4(li.x, li.y, li.z, li.w);
            ProjLinesD<BLOCK, ACC> srcd{ls, lid, (double)eps};
            double dx = x, dy = y;
            solved = lp2<REC, double>(srcd, i, (double)vmax, 1, -lid.w, lid.z, (double)tx,
                                      (double)ty, (double)eps, dx, dy, &inner) == i;
            nx = (float)dx;
            ny = (float)dy;
        }
        if (solved) {
            x = nx;
            y = ny;
            if (REC) {
                *rec = inner;
                rec->i3 = i;
            }
        }
        level = det2(li.z, li.w, li.x - x, li.y - y);
        ++i;
    }
    vx = x;
    vy = y;
}

// Scalar parameters of the scene an agent belongs to, in the form the
// per-agent step uses.
struct SceneP {
    float dt, inv_dt, inv_tau, eps;
    int k;
    int pref_is_goal;
    float f00, f01, f10, f11;
    float acc0, acc1;    // acceleration cap per class (0: none)
    float turn0, turn1;  // turn-rate cap per class (0: none)
};

__device__ __host__ __forceinline__ SceneP scene_params(const orca_params &p)
{
    SceneP s;
    s.dt = p.dt;
    s.inv_dt = 1.0f / p.dt;
    s.inv_tau = 1.0f / p.time_horizon;
    s.eps = p.par_eps;
    s.k = p.max_neighbors;
    s.pref_is_goal = p.pref_is_goal;
    s.f00 = p.f[0][0];
    s.f01 = p.f[0][1];
    s.f10 = p.f[1][0];
    s.f11 = p.f[1][1];
    s.acc0 = p.accel[0];
    s.acc1 = p.accel[1];
    s.turn0 = p.turn[0];
    s.turn1 = p.turn[1];
    return s;
}

// The half-planes of the agent's m neighbours into its LDS column.
// Neighbour states are loaded a group at a time without a branch (unused
// slots read position 0, a valid entry) so the loads of a group are in
// flight together; the half-planes of the group follow.
template <int K, int BLOCK>
__device__ __forceinline__ void build_halfplanes(const uint32_t (&pos)[K], int m,
                                                 const float4 *__restrict__ s0,
                                                 const float4 *__restrict__ s1, float xi,
                                                 float yi, float vxi, float vyi, float ri, int i,
                                                 int ci, const SceneP &p, float4 *lines, int tid)
{
    const float fa = ci ? p.f10 : p.f00;  // f[ci][0]
    const float fb = ci ? p.f11 : p.f01;  // f[ci][1]
    constexpr int kHpGroup = 4;
    lane_order<BLOCK>();  // every lane's selection entries are read
#pragma unroll
    for (int q0 = 0; q0 < K; q0 += kHpGroup) {
        float4 b0[kHpGroup], b1[kHpGroup];
#pragma unroll
        for (int u = 0; u < kHpGroup; ++u) {
            if (q0 + u < K) {
                b0[u] = s0[pos[q0 + u]];
                b1[u] = s1[pos[q0 + u]];
            }
        }
#pragma unroll
        for (int u = 0; u < kHpGroup; ++u) {
            const int q = q0 + u;
            if (q < K && q < m) {
                const float f = (__float_as_int(b1[u].z) & 1) ? fb : fa;
                lines[q * BLOCK + tid] =
                    halfplane(xi, yi, vxi, vyi, ri, b0[u].x, b0[u].y, b1[u].x, b1[u].y, b0[u].w,
                              f, p.inv_tau, p.inv_dt, i < __float_as_int(b0[u].z));
            }
        }
    }
}

// Goal mode: the pref input (the goal) becomes the desired velocity
// (g - p) min(v_max / |g - p|, 1/dt), zero at the goal.
__device__ __forceinline__ void desired_velocity(const SceneP &p, float xi, float yi, float vmax,
                                                 float &prx, float &pry)
{
    if (p.pref_is_goal) {
        const float gx = prx - xi, gy = pry - yi;
        const float d2 = gx * gx + gy * gy;
        const float sc = d2 > 0.0f ? fminf(vmax / sqrtf(d2), p.inv_dt) : 0.0f;
        prx = gx * sc;
        pry = gy * sc;
    }
}

// One whole ORCA step of the agent at cell-order position s: neighbours,
// half-planes (into the lane's LDS column), LP2, LP3 if needed, update.
// `lines` is a [KnnShape<K>::kSlots][BLOCK] float4 array; lane `tid` owns
// column tid.  `guess` (caller order, nullable) keeps each agent's K-th
// neighbour distance between steps (0: none); it only narrows the counting
// pass.  ACC compiles the acceleration lines in (used for agents whose class
// has a cap).  EXPORT also writes the neighbour list the step used (caller
// indices, ascending, -1 padded) to nbr[i * kout ..] and its length to
// cnt[i] (either nullable); the step itself is unchanged.  LP3CACHE lets
// LP3 cache its sub-problems' boundaries in spare LDS columns (CachedProj;
// without hard lines), which changes no result.
template <int K, int BLOCK, bool ACC = false, bool EXPORT = false, bool LP3CACHE = false>
__device__ __forceinline__ void step_agent(int s, const GridMeta &g, const SceneP &p,
                                           const orca_agents_in &in, const orca_agents_out &out,
                                           const uint32_t *__restrict__ start,
                                           const float4 *__restrict__ s0,
                                           const float4 *__restrict__ s1, float4 *lines, int tid,
                                           float *__restrict__ guess, int32_t *nbr = nullptr,
                                           int32_t *cnt = nullptr, int kout = 0)
{
    const float4 me0 = s0[s];
    const float4 me1 = s1[s];
    const int i = __float_as_int(me0.z);
    const float xi = me0.x, yi = me0.y, ri = me0.w, vxi = me1.x, vyi = me1.y;
    const int ci = __float_as_int(me1.z) & 1;
    const float vmax = in.max_speed[i];

    // the K nearest of the previous step, moved apart by at most their two
    // speeds times dt, stay within d_K + 2 v dt; a small slack covers the
    // faster neighbours the lane does not know of
    double rg2 = g.rn2;
    if (guess) {
        const float d = guess[i];
        if (d > 0.0f) {
            const double r = (double)d + kGuessSpeedSteps * (double)p.dt * (double)vmax +
                             0.005 * (double)g.rn;
            rg2 = fmin(r * r, g.rn2);
        }
    }

    uint64_t *buf = reinterpret_cast<uint64_t *>(lines);
    const int found = knn_select<K, BLOCK>(g, start, s0, xi, yi, i, (uint32_t)s, buf, tid, rg2);
    if (guess)
        guess[i] = found == K ? sqrtf(__uint_as_float((uint32_t)(buf[buf_idx<BLOCK>(K - 1, tid)] >> 32)))
                              : 0.0f;
    const int kk = p.k < K ? p.k : K;
    const int m = found < kk ? found : kk;
    uint32_t pos[K];
#pragma unroll
    for (int q = 0; q < K; ++q) pos[q] = q < m ? entry_pos(buf[buf_idx<BLOCK>(q, tid)]) : 0u;
    if (EXPORT) {
        if (nbr) {
            int32_t *row = nbr + (int64_t)i * kout;
            for (int q = 0; q < kout; ++q)
                row[q] = q < m ? __float_as_int(s0[entry_pos(buf[buf_idx<BLOCK>(q, tid)])].z) : -1;
        }
        if (cnt) cnt[i] = m;
    }

    float prx = in.pref_x[i], pry = in.pref_y[i];
    const float acc = ACC ? (ci ? p.acc1 : p.acc0) : 0.0f;
    const float turn = ACC ? (ci ? p.turn1 : p.turn0) : 0.0f;
    const int nacc = (ACC && acc > 0.0f) ? kAccLines : 0;
    float rx = 0.0f, ry = 0.0f, lx = 0.0f, ly = 0.0f;
    const int nh = nacc + ((ACC && turn_wedge(vxi, vyi, turn, p.dt, rx, ry, lx, ly))
                               ? kTurnLines : 0);
    build_halfplanes<K, BLOCK>(pos, m, s0, s1, xi, yi, vxi, vyi, ri, i, ci, p, lines, tid);
    float cx = 0.0f, cy = 0.0f;
    if (ACC && nh) accel_centre(vxi, vyi, vmax, cx, cy);
    desired_velocity(p, xi, yi, vmax, prx, pry);

    const LdsLines<BLOCK, ACC> src{lines, tid, nh, cx, cy,
                                   ACC && nacc ? accel_half_width(acc, p.dt) : 0.0f,
                                   nacc, rx, ry, lx, ly};
    const int mt = nh + m;
    float vx, vy;
    int fail = lp2<false, float>(src, mt, vmax, 0, prx, pry, 0.0f, 0.0f, p.eps, vx, vy, nullptr);
    uint8_t st = 0;
    if (ACC && fail < nh) {
        // the centre (the current velocity scaled into the speed disc) lies
        // in the octagon and on the wedge's axis, so only rounding can get
        // here: take the centre and let LP3 start from it
        vx = cx;
        vy = cy;
        fail = nh;
        st = 1;
    }
    const int col = (ACC || !LP3CACHE) ? -1 : lp3_cache_column<BLOCK>(fail < mt, tid);
    if (fail < mt) {
        lp3<false, BLOCK, ACC>(src, mt, fail, vmax, prx, pry, p.eps, vx, vy, nullptr, col);
        st = 1;
    }
    out.vx[i] = vx;
    out.vy[i] = vy;
    out.px[i] = xi + vx * p.dt;
    out.py[i] = yi + vy * p.dt;
    if (out.status) out.status[i] = st;
}

}  // namespace dev
}  // namespace orca
