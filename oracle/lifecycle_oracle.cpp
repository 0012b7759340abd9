/*
 * FP64 CPU oracle for the agent lifecycle of the crossing experiments
 * (Sec. 4, first experiment): agents leave the simulation once they reach
 * their goal, and new agents enter at spawn points chosen so that they
 * cannot overlap anyone for a while given sizes and speeds.
 *
 * TEST INFRASTRUCTURE ONLY: the plain definition the GPU library's
 * lifecycle entry points are checked against; shares no code with it.
 * Build with -ffp-contract=off.
 *
 * Readings (the paper states the rules, not their arithmetic):
 *  - reaching the goal: after the update the goal point lies inside or on
 *    the agent's disc, |g - p|^2 <= r^2.  dx = g.x - p.x etc. are formed in
 *    double from the FP32 values and every operation is rounded separately,
 *    so the decision is exactly reproducible.
 *  - leaving: the agents that stay keep their relative order.
 *  - entering: the caller proposes candidates (position, radius, speed cap;
 *    drawing them at random is the caller's part) and they are taken in the
 *    given order.  A candidate enters when, for every agent present (those
 *    already simulated and the candidates that entered before it),
 *        |p_c - p_j|^2 >= D^2,  D = (r_c + r_j) + T (s_c + s_j),
 *    i.e. the two discs cannot touch within T seconds even if both head
 *    straight for each other at full speed.  Both sides are in double from
 *    FP32 values, operations rounded separately in the order written.
 */
#include <cmath>
#include <cstdint>
#include <vector>

namespace {

double sq_dist(float ax, float ay, float bx, float by)
{
    const double dx = (double)bx - (double)ax;
    const double dy = (double)by - (double)ay;
    return dx * dx + dy * dy;
}

bool too_close(float ax, float ay, float ar, float as, float bx, float by, float br, float bs,
               double t)
{
    const double d = ((double)ar + (double)br) + t * ((double)as + (double)bs);
    return sq_dist(ax, ay, bx, by) < d * d;
}

}  // namespace

extern "C" {

/* arrived[i] = 1 when agent i's goal lies within its disc. */
int oracle_arrived(int n, const float *px, const float *py, const float *gx, const float *gy,
                   const float *radius, uint8_t *arrived)
{
    if (n < 0) return -1;
    for (int i = 0; i < n; ++i) {
        const double r = (double)radius[i];
        arrived[i] = sq_dist(px[i], py[i], gx[i], gy[i]) <= r * r ? 1 : 0;
    }
    return 0;
}

/* accepted[c] = 1 when candidate c enters; returns the number accepted. */
int oracle_spawn(int n, const float *px, const float *py, const float *radius,
                 const float *max_speed, int n_cand, const float *cx, const float *cy,
                 const float *cr, const float *cs, float t_clear, uint8_t *accepted)
{
    if (n < 0 || n_cand < 0) return -1;
    const double t = (double)t_clear;
    int count = 0;
    for (int c = 0; c < n_cand; ++c) {
        bool ok = true;
        for (int j = 0; j < n && ok; ++j)
            if (too_close(cx[c], cy[c], cr[c], cs[c], px[j], py[j], radius[j], max_speed[j], t))
                ok = false;
        for (int e = 0; e < c && ok; ++e)
            if (accepted[e] && too_close(cx[c], cy[c], cr[c], cs[c], cx[e], cy[e], cr[e], cs[e], t))
                ok = false;
        accepted[c] = ok ? 1 : 0;
        count += ok ? 1 : 0;
    }
    return count;
}

} /* extern "C" */

extern "C" {

/* Overlap statistics of a crowd (the collision measure of the crossing
 * experiments, Sec. 4) over the pairs i < j closer than `reach`
 * (|p_i - p_j|^2 < reach^2, double from FP32 values; reach >= 2 max r
 * covers every overlap): out[0] = pairs whose discs overlap,
 * |p_i - p_j|^2 < (r_i + r_j)^2; out[1] = agents in at least one of them;
 * out[2] = the smallest clearance |p_i - p_j| - (r_i + r_j) (+inf when no
 * pair is that close).  Brute force over all pairs. */
int oracle_overlap_stats(int n, const float *px, const float *py, const float *radius,
                         float reach, double *out)
{
    if (n < 0) return -1;
    const double q = (double)reach;
    int64_t pairs = 0, agents = 0;
    double gap = INFINITY;
    std::vector<uint8_t> hit((size_t)n, 0);
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double dx = (double)px[j] - (double)px[i];
            const double dy = (double)py[j] - (double)py[i];
            const double d2 = dx * dx + dy * dy;
            if (!(d2 < q * q)) continue;
            const double rr = (double)radius[i] + (double)radius[j];
            if (d2 < rr * rr) {
                ++pairs;
                hit[i] = hit[j] = 1;
            }
            const double g = std::sqrt(d2) - rr;
            if (g < gap) gap = g;
        }
    for (int i = 0; i < n; ++i) agents += hit[i];
    out[0] = (double)pairs;
    out[1] = (double)agents;
    out[2] = gap;
    return 0;
}

} /* extern "C" */
