// Adjoint of one ORCA step (the differentiable form; not in the paper).
//
// Given the cotangents (gp1, gv1) of the step's outputs p' = p + v' dt and v',
// the kernels below produce the cotangents of the step-t positions and
// velocities, accumulate those of the pref input (desired velocity, or goal in
// goal mode) and of the look-ahead tau:
//
//   k_adjoint       one lane per agent: recompute the agent's step exactly as
//                   the forward kernel does (same neighbours, half-planes, LP),
//                   recording the LP's active set; then differentiate:
//                     LP   implicit differentiation of the active equalities
//                          (a line, two lines, a line on the speed circle, or
//                          the equal-penetration boundaries of LP3),
//                     ORCA each involved half-plane through its branch (cutoff
//                          arc, leg, overlap) to P = p_B - p_A, V = v_A - v_B
//                          and 1/tau,
//                     caps an involved acceleration line (q = c + h n_k)
//                          through its centre c to the agent's own velocity
//                          (c = v, or v scaled onto the speed circle),
//                   writing the agent's own cotangents and up to three
//                   contributions to neighbours into an edge list;
//   k_edge_*,       counting sort of the edges by target (count, tiled scan,
//   k_escan_*       place), each target summing its edges in source order (no
//                   floating-point atomics, so results are bit-reproducible);
//   k_tau_*         the per-agent tau contributions summed in double in a
//                   fixed order (block sums, then one block).
// Neighbour sets and branches are held fixed (they are piecewise constant).
#include "orca_device.h"

namespace orca {
namespace {

constexpr int kAdjBlock = 64;
constexpr int kBlock = 256;
constexpr int kEdges = 3;  // at most three lines define an LP result

struct AdjArgs {
    orca_agents_in in;
    int n;
    const GridMeta *meta;
    const uint32_t *start;
    const float4 *s0;
    const float4 *s1;
    dev::SceneP p;
    const float *gpx1, *gpy1, *gvx1, *gvy1;
    float *gpx0, *gpy0, *gvx0, *gvy0, *gprx, *gpry;
    float *tau_part;
    int32_t *e_tgt;
    float4 *e_val;
    uint32_t *e_cnt;
};

// Cotangents of the (at most three) lines (q, n) that define the LP result:
// slot e holds line idx[e] (neighbour slot, -1 = unused).
struct LineBars {
    int idx[kEdges];
    float qx[kEdges], qy[kEdges], nx[kEdges], ny[kEdges];
};

__device__ __forceinline__ void add_line(LineBars &lb, int idx, float qx, float qy, float nx,
                                         float ny)
{
    // slot of line idx, or the first free one (static indices only, so the
    // arrays stay in registers)
    int slot = -1;
#pragma unroll
    for (int e = 0; e < kEdges; ++e)
        if (slot < 0 && lb.idx[e] == idx) slot = e;
#pragma unroll
    for (int e = 0; e < kEdges; ++e) {
        if (slot < 0 && lb.idx[e] < 0) {
            slot = e;
            lb.idx[e] = idx;
        }
    }
#pragma unroll
    for (int e = 0; e < kEdges; ++e) {
        if (e == slot) {
            lb.qx[e] += qx;
            lb.qy[e] += qy;
            lb.nx[e] += nx;
            lb.ny[e] += ny;
        }
    }
}

// VJP of ORCA_{A|B} (see dev::halfplane) given the cotangents of its point q
// and normal n.  Returns the cotangents of P = p_B - p_A, V = v_A - v_B, of
// the horizon's reciprocal (only when not overlapping), and q's direct
// dependence on v_A is left to the caller (q = v_A + f u).
__device__ __forceinline__ void halfplane_vjp(float pax, float pay, float vax, float vay, float ra,
                                              float pbx, float pby, float vbx, float vby, float rb,
                                              float f, float inv_tau, float inv_dt, bool a_first,
                                              float qbx, float qby, float nbx, float nby,
                                              float &Pbx, float &Pby, float &Vbx, float &Vby,
                                              float &itb, bool &uses_tau)
{
    const float Px = pbx - pax, Py = pby - pay;
    const float Vx = vax - vbx, Vy = vay - vby;
    const float R = ra + rb;
    const float dist2 = Px * Px + Py * Py;
    const float R2 = R * R;
    const double c2 = dev::clearance2(pax, pay, ra, pbx, pby, rb);
    const bool overlap = !(c2 > 0.0);
    const float it = overlap ? inv_dt : inv_tau;
    const float wx = Vx - Px * it, wy = Vy - Py * it;
    const float w2 = wx * wx + wy * wy;
    const float wp = wx * Px + wy * Py;
    const bool arc = overlap || (wp < 0.0f && wp * wp > R2 * w2);
    const float ubx = f * qbx, uby = f * qby;
    uses_tau = !overlap && arc;
    if (arc) {
        const bool wz = !(w2 > 0.0f);
        const float wl = sqrtf(w2);
        const float iwl = wz ? 0.0f : 1.0f / wl;
        const float nx = wz ? (a_first ? 1.0f : -1.0f) : wx * iwl;
        const float ny = wz ? 0.0f : wy * iwl;
        const float ul = R * it - wl;
        const float ulb = ubx * nx + uby * ny;
        const float tx = nbx + ul * ubx, ty = nby + ul * uby;
        const float nt = nx * tx + ny * ty;
        const float wbx = wz ? 0.0f : (tx - nx * nt) * iwl - ulb * nx;
        const float wby = wz ? 0.0f : (ty - ny * nt) * iwl - ulb * ny;
        itb = ulb * R - (wbx * Px + wby * Py);
        Vbx = wbx;
        Vby = wby;
        Pbx = -wbx * it;
        Pby = -wby * it;
        return;
    }
    // leg: e = (leg P + sigma R P_perp) / |P|^2, n = sigma (-e.y, e.x), u = (V.e) e - V
    const float leg = sqrtf(fmaxf((float)c2, 0.0f));
    const float id2 = 1.0f / dist2;
    const bool left = dev::det2(Px, Py, wx, wy) > 0.0f;
    const float sR = left ? R : -R;
    const float ex = (Px * leg - Py * sR) * id2;
    const float ey = (Px * sR + Py * leg) * id2;
    const float s = Vx * ex + Vy * ey;
    const float eu = ex * ubx + ey * uby;
    Vbx = ex * eu - ubx;
    Vby = ey * eu - uby;
    float ebx = s * ubx + eu * Vx;
    float eby = s * uby + eu * Vy;
    ebx += left ? nby : -nby;
    eby += left ? -nbx : nbx;
    const float abx = ebx * id2, aby = eby * id2;
    float Db = -(ebx * ex + eby * ey) * id2;
    Pbx = leg * abx + sR * aby;
    Pby = -sR * abx + leg * aby;
    const float legb = abx * Px + aby * Py;
    Db += leg > 0.0f ? legb / (2.0f * leg) : 0.0f;
    Pbx += 2.0f * Db * Px;
    Pby += 2.0f * Db * Py;
    itb = 0.0f;
}

// Solves mu_1 g1 + mu_2 g2 = w (2x2); zero when singular.
__device__ __forceinline__ void solve2(float g1x, float g1y, float g2x, float g2y, float wx,
                                       float wy, float &m1, float &m2)
{
    const float det = g1x * g2y - g1y * g2x;
    if (!(fabsf(det) > 1e-20f)) {
        m1 = 0.0f;
        m2 = 0.0f;
        return;
    }
    const float id = 1.0f / det;
    m1 = (wx * g2y - wy * g2x) * id;
    m2 = (g1x * wy - g1y * wx) * id;
}

template <int K, int BLOCK, bool ACC>
__device__ __forceinline__ void adjoint_agent(int s, const AdjArgs &a, const GridMeta &g,
                                              float4 *lines, int tid)
{
    const dev::SceneP &p = a.p;
    const float4 me0 = a.s0[s];
    const float4 me1 = a.s1[s];
    const int i = __float_as_int(me0.z);
    const float xi = me0.x, yi = me0.y, ri = me0.w, vxi = me1.x, vyi = me1.y;
    const int ci = __float_as_int(me1.z) & 1;

    // -- forward recomputation (identical to dev::step_agent) --
    uint64_t *buf = reinterpret_cast<uint64_t *>(lines);
    const int found = dev::knn_select<K, BLOCK>(g, a.start, a.s0, xi, yi, i, (uint32_t)s, buf, tid,
                                                g.rn2);
    const int kk = p.k < K ? p.k : K;
    const int m = found < kk ? found : kk;
    uint32_t pos[K];
#pragma unroll
    for (int q = 0; q < K; ++q)
        pos[q] = q < m ? dev::entry_pos(buf[dev::buf_idx<BLOCK>(q, tid)]) : 0u;
    const float vmax = a.in.max_speed[i];
    const float acc = ACC ? (ci ? p.acc1 : p.acc0) : 0.0f;
    const float turn = ACC ? (ci ? p.turn1 : p.turn0) : 0.0f;
    const int nacc = (ACC && acc > 0.0f) ? dev::kAccLines : 0;
    float rx = 0.0f, ry = 0.0f, lx = 0.0f, ly = 0.0f;
    const int nh = nacc + ((ACC && dev::turn_wedge(vxi, vyi, turn, p.dt, rx, ry, lx, ly))
                               ? dev::kTurnLines : 0);
    dev::build_halfplanes<K, BLOCK>(pos, m, a.s0, a.s1, xi, yi, vxi, vyi, ri, i, ci, p, lines,
                                    tid);
    float cx = 0.0f, cy = 0.0f;
    if (ACC && nh) dev::accel_centre(vxi, vyi, vmax, cx, cy);
    const float pin_x = a.in.pref_x[i], pin_y = a.in.pref_y[i];
    float prx = pin_x, pry = pin_y;
    dev::desired_velocity(p, xi, yi, vmax, prx, pry);
    // the goal-mode quantities the desired velocity was formed from
    float gxg = 0.0f, gyg = 0.0f, d2g = 0.0f;
    if (p.pref_is_goal) {
        gxg = pin_x - xi;
        gyg = pin_y - yi;
        d2g = gxg * gxg + gyg * gyg;
    }
    const dev::LdsLines<BLOCK, ACC> src{lines, tid, nh, cx, cy,
                                        ACC && nacc ? dev::accel_half_width(acc, p.dt) : 0.0f,
                                        nacc, rx, ry, lx, ly};
    float vx, vy;
    dev::ActiveSet rec{dev::kFree, -1, -1, -1};
    const int mt = nh + m;
    int fail = dev::lp2<true, float>(src, mt, vmax, 0, prx, pry, 0.0f, 0.0f, p.eps, vx, vy, &rec);
    if (ACC && fail < nh) {
        vx = cx;
        vy = cy;
        fail = nh;
        rec.kind = dev::kCentre;
    }
    if (fail < mt)
        dev::lp3<true, BLOCK, ACC>(src, mt, fail, vmax, prx, pry, p.eps, vx, vy, &rec);

    // -- cotangent of the new velocity: v' directly and through p' = p + v' dt --
    const float gpx = a.gpx1[i], gpy = a.gpy1[i];
    const float wx = a.gvx1[i] + gpx * p.dt, wy = a.gvy1[i] + gpy * p.dt;

    // -- LP: active-set VJP --
    LineBars lb;
#pragma unroll
    for (int e = 0; e < kEdges; ++e) {
        lb.idx[e] = -1;
        lb.qx[e] = lb.qy[e] = lb.nx[e] = lb.ny[e] = 0.0f;
    }
    float pbx = 0.0f, pby = 0.0f;  // cotangent of the desired velocity
    float cbx = 0.0f, cby = 0.0f;  // cotangent of the acceleration octagon's centre
    float hbx = 0.0f, hby = 0.0f;  // cotangent of the heading (turn wedge)
    auto Lq = [&](int idx) { return src.line(idx); };
    // Rows of an LP3 sub-problem: line j < nh is a hard line, g = n_j,
    // r = n_j . q_j; otherwise the equal-penetration boundary of j and i3,
    // g = n_i3 - n_j, r = n_i3 . q_i3 - n_j . q_j.  For v = G^-1 r the
    // cotangents are r-bar = mu, g-bar = -mu v with mu = G^-T w; row_bar
    // scatters them to the lines and returns the share that goes to i3.
    auto row_g = [&](int j, float nix, float niy, float &gx, float &gy) {
        const float4 lj = Lq(j);
        if (ACC && j < nh) {
            gx = -lj.w;
            gy = lj.z;
        } else {
            gx = nix - (-lj.w);
            gy = niy - lj.z;
        }
    };
    auto row_bar = [&](int j, float mu) -> float {
        const float4 lj = Lq(j);
        const float njx = -lj.w, njy = lj.z;
        if (ACC && j < nh) {
            add_line(lb, j, mu * njx, mu * njy, mu * (lj.x - vx), mu * (lj.y - vy));
            return 0.0f;
        }
        add_line(lb, j, -mu * njx, -mu * njy, -mu * (lj.x - vx), -mu * (lj.y - vy));
        return mu;
    };
    switch (rec.kind) {
    case dev::kFree:
        pbx = wx;
        pby = wy;
        break;
    case dev::kDisc: {
        const float ol = sqrtf(prx * prx + pry * pry);
        const float ux = prx / ol, uy = pry / ol;
        const float uw = ux * wx + uy * wy;
        pbx = vmax / ol * (wx - ux * uw);
        pby = vmax / ol * (wy - uy * uw);
        break;
    }
    case dev::kLine: {
        const float4 l = Lq(rec.a);
        const float rx = prx - l.x, ry = pry - l.y;
        const float t = rx * l.z + ry * l.w;
        const float c = wx * l.z + wy * l.w;
        pbx = c * l.z;
        pby = c * l.w;
        // d-bar = t w + c r; n = (-d.y, d.x) so n-bar = (-dbar.y, dbar.x)
        const float dbx = t * wx + c * rx, dby = t * wy + c * ry;
        add_line(lb, rec.a, wx - c * l.z, wy - c * l.w, -dby, dbx);
        break;
    }
    case dev::kLineLine: {
        const float4 la = Lq(rec.a), lc = Lq(rec.b);
        const float nax = -la.w, nay = la.z, ncx = -lc.w, ncy = lc.z;
        float ma, mc;
        solve2(nax, nay, ncx, ncy, wx, wy, ma, mc);
        add_line(lb, rec.a, ma * nax, ma * nay, -ma * (vx - la.x), -ma * (vy - la.y));
        add_line(lb, rec.b, mc * ncx, mc * ncy, -mc * (vx - lc.x), -mc * (vy - lc.y));
        break;
    }
    case dev::kLineDisc: {
        const float4 la = Lq(rec.a);
        const float nax = -la.w, nay = la.z;
        float m1, m2;
        solve2(nax, nay, vx, vy, wx, wy, m1, m2);
        add_line(lb, rec.a, m1 * nax, m1 * nay, -m1 * (vx - la.x), -m1 * (vy - la.y));
        break;
    }
    case dev::kDir:
        add_line(lb, rec.i3, 0.0f, 0.0f, vmax * wx, vmax * wy);
        break;
    case dev::kProjDisc: {
        const float4 li = Lq(rec.i3);
        const float nix = -li.w, niy = li.z;
        float gax, gay, m1, m2;
        row_g(rec.a, nix, niy, gax, gay);
        solve2(gax, gay, vx, vy, wx, wy, m1, m2);
        const float ms = row_bar(rec.a, m1);
        if (!ACC || ms != 0.0f)
            add_line(lb, rec.i3, ms * nix, ms * niy, ms * (li.x - vx), ms * (li.y - vy));
        break;
    }
    case dev::kProjProj: {
        const float4 li = Lq(rec.i3);
        const float nix = -li.w, niy = li.z;
        float gax, gay, gcx, gcy, ma, mc;
        row_g(rec.a, nix, niy, gax, gay);
        row_g(rec.b, nix, niy, gcx, gcy);
        solve2(gax, gay, gcx, gcy, wx, wy, ma, mc);
        const float msa = row_bar(rec.a, ma);
        const float ms = msa + row_bar(rec.b, mc);
        if (!ACC || ms != 0.0f)
            add_line(lb, rec.i3, ms * nix, ms * niy, ms * (li.x - vx), ms * (li.y - vy));
        break;
    }
    case dev::kTie: {
        const float4 li = Lq(rec.i3), la = Lq(rec.a);
        const float nix = -li.w, niy = li.z, nax = -la.w, nay = la.z;
        const bool hard = ACC && rec.a < nh;
        float gx, gy;
        row_g(rec.a, nix, niy, gx, gy);
        const float G = gx * gx + gy * gy;
        const float h = hard ? nax * la.x + nay * la.y
                             : nix * li.x + niy * li.y - (nax * la.x + nay * la.y);
        const float sv = (gx * prx + gy * pry - h) / G;
        const float c = wx * gx + wy * gy;
        pbx = wx - c / G * gx;
        pby = wy - c / G * gy;
        const float hb = c / G;
        const float gbx = -(c / G) * (prx - 2.0f * sv * gx) - sv * wx;
        const float gby = -(c / G) * (pry - 2.0f * sv * gy) - sv * wy;
        if (hard) {
            add_line(lb, rec.a, hb * nax, hb * nay, gbx + hb * la.x, gby + hb * la.y);
        } else {
            add_line(lb, rec.i3, hb * nix, hb * niy, gbx + hb * li.x, gby + hb * li.y);
            add_line(lb, rec.a, -hb * nax, -hb * nay, -gbx - hb * la.x, -gby - hb * la.y);
        }
        break;
    }
    case dev::kCentre:
        cbx = wx;
        cby = wy;
        break;
    default:
        break;
    }

    // -- ORCA half-planes of the involved lines --
    const float fa = ci ? p.f10 : p.f00;  // f[ci][0]
    const float fb = ci ? p.f11 : p.f01;  // f[ci][1]
    float spx = 0.0f, spy = 0.0f, svx = 0.0f, svy = 0.0f, taub = 0.0f;
#pragma unroll
    for (int e = 0; e < kEdges; ++e) {
        int32_t tgt = -1;
        float4 val = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (ACC && lb.idx[e] >= 0 && lb.idx[e] < nacc) {
            // acceleration line: q = c + h n_k with a constant normal
            cbx += lb.qx[e];
            cby += lb.qy[e];
        } else if (ACC && lb.idx[e] >= nacc && lb.idx[e] < nh) {
            // wedge side: q = 0, d = R(-phi) h (right) or -R(phi) h (left);
            // n = (-d.y, d.x), so d-bar = (n-bar.y, -n-bar.x), and h-bar =
            // R(phi) d-bar (right) or -R(-phi) d-bar (left)
            float hx, hy, cs, sn, speed;
            dev::turn_basis(vxi, vyi, turn, p.dt, hx, hy, cs, sn, speed);
            const float dbx = lb.ny[e], dby = -lb.nx[e];
            if (lb.idx[e] == nacc) {
                hbx += cs * dbx - sn * dby;
                hby += sn * dbx + cs * dby;
            } else {
                hbx -= cs * dbx + sn * dby;
                hby -= -sn * dbx + cs * dby;
            }
        } else if (lb.idx[e] >= 0) {
            uint32_t pj = 0u;
            const int qn = lb.idx[e] - nh;
#pragma unroll
            for (int q = 0; q < K; ++q)
                if (q == qn) pj = pos[q];
            const float4 b0 = a.s0[pj];
            const float4 b1 = a.s1[pj];
            const int j = __float_as_int(b0.z);
            const float f = (__float_as_int(b1.z) & 1) ? fb : fa;
            float Pbx, Pby, Vbx, Vby, itb;
            bool uses_tau;
            halfplane_vjp(xi, yi, vxi, vyi, ri, b0.x, b0.y, b1.x, b1.y, b0.w, f, p.inv_tau,
                          p.inv_dt, i < j, lb.qx[e], lb.qy[e], lb.nx[e], lb.ny[e], Pbx, Pby, Vbx,
                          Vby, itb, uses_tau);
            spx -= Pbx;
            spy -= Pby;
            svx += Vbx + lb.qx[e];
            svy += Vby + lb.qy[e];
            if (uses_tau) taub -= itb * p.inv_tau * p.inv_tau;
            tgt = j;
            val = make_float4(Pbx, Pby, -Vbx, -Vby);
        }
        a.e_tgt[(int64_t)kEdges * i + e] = tgt;
        a.e_val[(int64_t)kEdges * i + e] = val;
    }
    if (ACC && nh > nacc) {
        // h = v / |v|: Jacobian (I - h h^T) / |v|
        float hx, hy, cs, sn, speed;
        dev::turn_basis(vxi, vyi, turn, p.dt, hx, hy, cs, sn, speed);
        const float hh = hx * hbx + hy * hby;
        svx += (hbx - hx * hh) / speed;
        svy += (hby - hy * hh) / speed;
    }
    if (ACC && nh) {
        // c = v, or v (v_max / |v|) when |v| > v_max: Jacobian (v_max/|v|)(I - u u^T)
        const float v2 = vxi * vxi + vyi * vyi;
        if (v2 > vmax * vmax) {
            const float l = sqrtf(v2);
            const float ux = vxi / l, uy = vyi / l, sc = vmax / l;
            const float uc = ux * cbx + uy * cby;
            svx += sc * (cbx - ux * uc);
            svy += sc * (cby - uy * uc);
        } else {
            svx += cbx;
            svy += cby;
        }
    }

    // -- desired velocity: the pref input itself, or the goal --
    float grx = pbx, gry = pby;
    if (p.pref_is_goal) {
        grx = 0.0f;
        gry = 0.0f;
        if (d2g > 0.0f) {
            const float d = sqrtf(d2g);
            if (p.inv_dt < vmax / d) {
                grx = pbx * p.inv_dt;
                gry = pby * p.inv_dt;
            } else {
                const float ux = gxg / d, uy = gyg / d;
                const float up = ux * pbx + uy * pby;
                grx = vmax / d * (pbx - ux * up);
                gry = vmax / d * (pby - uy * up);
            }
        }
        spx -= grx;
        spy -= gry;
    }
    a.gprx[i] += grx;
    a.gpry[i] += gry;
    a.gpx0[i] = gpx + spx;
    a.gpy0[i] = gpy + spy;
    a.gvx0[i] = svx;
    a.gvy0[i] = svy;
    a.tau_part[i] = taub;
    a.e_cnt[i] = 0u;
}

template <int K, int BLOCK, bool ACC>
__global__ __launch_bounds__(BLOCK) void k_adjoint(AdjArgs a)
{
    __shared__ float4 lines[dev::KnnShape<K>::kSlots * BLOCK];
    const int tid = threadIdx.x;
    const int s = xcd_tile(blockIdx.x, gridDim.x) * BLOCK + tid;
    if (s >= a.n) return;
    const GridMeta g = *a.meta;
    adjoint_agent<K, BLOCK, ACC>(s, a, g, lines, tid);
}

// Edges by target: count and rank.
__global__ __launch_bounds__(kBlock) void k_edge_count(const int32_t *__restrict__ e_tgt, int ne,
                                                       int n, uint32_t *__restrict__ e_cnt,
                                                       uint32_t *__restrict__ e_rank)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= ne) return;
    const int t = e_tgt[e];
    if (t >= 0 && t < n) e_rank[e] = atomicAdd(&e_cnt[t], 1u);
}

// Exclusive scan of the per-target counts in tiles of kScanTile: the sum of
// each tile, then the scan inside each tile offset by its prefix, the sum of
// the tile sums before it (added up by each block itself).
constexpr int kPer = kScanTile / kBlock;

__global__ __launch_bounds__(kBlock) void k_escan_reduce(const uint32_t *__restrict__ cnt, int n,
                                                         uint32_t *__restrict__ tiles)
{
    const int base = blockIdx.x * kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int c = base + threadIdx.x * kPer + k;
        if (c < n) s += cnt[c];
    }
    uint32_t tot;
    block_excl_scan<kBlock>(s, &tot);
    if (threadIdx.x == 0) tiles[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_escan_apply(const uint32_t *__restrict__ cnt, int n,
                                                        const uint32_t *__restrict__ tiles,
                                                        uint32_t *__restrict__ start)
{
    const int base = blockIdx.x * kScanTile;
    uint32_t before = 0;
    for (int t = threadIdx.x; t < (int)blockIdx.x; t += kBlock) before += tiles[t];
    uint32_t prefix;
    block_excl_scan<kBlock>(before, &prefix);
    uint32_t v[kPer];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int c = base + threadIdx.x * kPer + k;
        v[k] = c < n ? cnt[c] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = prefix + block_excl_scan<kBlock>(s, &tot);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int c = base + threadIdx.x * kPer + k;
        if (c < n) start[c] = run;
        run += v[k];
    }
}

__global__ __launch_bounds__(kBlock) void k_edge_place(const int32_t *__restrict__ e_tgt, int ne,
                                                       int n, const uint32_t *__restrict__ e_rank,
                                                       const uint32_t *__restrict__ start,
                                                       uint32_t *__restrict__ list)
{
    const int e = blockIdx.x * kBlock + threadIdx.x;
    if (e >= ne) return;
    const int t = e_tgt[e];
    if (t >= 0 && t < n) list[start[t] + e_rank[e]] = (uint32_t)e;
}

// Each target sums its edges in increasing edge index (= source agent, slot).
__global__ __launch_bounds__(kBlock) void k_edge_gather(int n, const uint32_t *__restrict__ e_cnt,
                                                        const uint32_t *__restrict__ start,
                                                        uint32_t *__restrict__ list,
                                                        const float4 *__restrict__ e_val,
                                                        float *gpx0, float *gpy0, float *gvx0,
                                                        float *gvy0)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const uint32_t a = start[j], c = e_cnt[j];
    for (uint32_t p = 1; p < c; ++p) {
        const uint32_t v = list[a + p];
        int q = (int)p - 1;
        while (q >= 0 && list[a + q] > v) {
            list[a + q + 1] = list[a + q];
            --q;
        }
        list[a + q + 1] = v;
    }
    float sx = 0.0f, sy = 0.0f, tx = 0.0f, ty = 0.0f;
    for (uint32_t p = 0; p < c; ++p) {
        const float4 v = e_val[list[a + p]];
        sx += v.x;
        sy += v.y;
        tx += v.z;
        ty += v.w;
    }
    gpx0[j] += sx;
    gpy0[j] += sy;
    gvx0[j] += tx;
    gvy0[j] += ty;
}

// g_tau += sum of the per-agent contributions in double, in a fixed order:
// kTauBlocks blocks each reduce a contiguous share (threads strided, then a
// tree), and one block adds the block sums by a tree.
__global__ __launch_bounds__(kBlock) void k_tau_partial(const float *__restrict__ part, int n,
                                                        double *__restrict__ blocks)
{
    __shared__ double red[kBlock];
    const int per = (n + (int)gridDim.x - 1) / (int)gridDim.x;
    const int a = blockIdx.x * per, b = min(a + per, n);
    double s = 0.0;
    for (int k = a + threadIdx.x; k < b; k += kBlock) s += (double)part[k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) blocks[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(kTauBlocks) void k_tau_final(const double *__restrict__ blocks,
                                                          float *g_tau)
{
    __shared__ double red[kTauBlocks];
    red[threadIdx.x] = blocks[threadIdx.x];
    __syncthreads();
    for (int off = kTauBlocks / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *g_tau += (float)red[0];
}

template <int K>
void launch_adjoint_k(const AdjArgs &a, hipStream_t stream)
{
    const int nb = (a.n + kAdjBlock - 1) / kAdjBlock;
    if (a.p.acc0 > 0.0f || a.p.acc1 > 0.0f || a.p.turn0 > 0.0f || a.p.turn1 > 0.0f)
        hipLaunchKernelGGL((k_adjoint<K, kAdjBlock, true>), dim3(nb), dim3(kAdjBlock), 0, stream,
                           a);
    else
        hipLaunchKernelGGL((k_adjoint<K, kAdjBlock, false>), dim3(nb), dim3(kAdjBlock), 0, stream,
                           a);
}

}  // namespace

hipError_t launch_adjoint(const orca_agents_in &in, int n, const orca_params &prm,
                          const Layout &L, const Work &w, const AdjointBufs &b,
                          const float *gpx1, const float *gpy1, const float *gvx1,
                          const float *gvy1, float *gpx0, float *gpy0, float *gvx0, float *gvy0,
                          float *gprx, float *gpry, float *g_tau, const orca_step_events *ev,
                          hipStream_t stream)
{
    (void)L;
    AdjArgs a;
    a.in = in;
    a.n = n;
    a.meta = w.meta;
    a.start = w.start;
    a.s0 = w.s0;
    a.s1 = w.s1;
    a.p = dev::scene_params(prm);
    a.gpx1 = gpx1;
    a.gpy1 = gpy1;
    a.gvx1 = gvx1;
    a.gvy1 = gvy1;
    a.gpx0 = gpx0;
    a.gpy0 = gpy0;
    a.gvx0 = gvx0;
    a.gvy0 = gvy0;
    a.gprx = gprx;
    a.gpry = gpry;
    a.tau_part = b.tau_part;
    a.e_tgt = b.e_tgt;
    a.e_val = b.e_val;
    a.e_cnt = b.e_cnt;
    const int k = prm.max_neighbors;
    if (ev && ev->step_begin && hipEventRecord(ev->step_begin, stream) != hipSuccess)
        return hipErrorInvalidValue;
    if (k <= 4)
        launch_adjoint_k<4>(a, stream);
    else if (k <= 8)
        launch_adjoint_k<8>(a, stream);
    else if (k <= 10)
        launch_adjoint_k<10>(a, stream);
    else if (k <= 12)
        launch_adjoint_k<12>(a, stream);
    else if (k <= 16)
        launch_adjoint_k<16>(a, stream);
    else if (k <= 20)
        launch_adjoint_k<20>(a, stream);
    else if (k <= 24)
        launch_adjoint_k<24>(a, stream);
    else
        launch_adjoint_k<32>(a, stream);
    if (ev && ev->step_end && hipEventRecord(ev->step_end, stream) != hipSuccess)
        return hipErrorInvalidValue;
    const int ne = kEdges * n;
    const int nbe = (ne + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_edge_count, dim3(nbe), dim3(kBlock), 0, stream, b.e_tgt, ne, n, b.e_cnt,
                       b.e_rank);
    const int nt = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_escan_reduce, dim3(nt), dim3(kBlock), 0, stream, b.e_cnt, n, b.e_tiles);
    hipLaunchKernelGGL(k_escan_apply, dim3(nt), dim3(kBlock), 0, stream, b.e_cnt, n, b.e_tiles,
                       b.e_start);
    hipLaunchKernelGGL(k_edge_place, dim3(nbe), dim3(kBlock), 0, stream, b.e_tgt, ne, n, b.e_rank,
                       b.e_start, b.e_list);
    hipLaunchKernelGGL(k_edge_gather, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, stream, n,
                       b.e_cnt, b.e_start, b.e_list, b.e_val, gpx0, gpy0, gvx0, gvy0);
    if (g_tau) {
        hipLaunchKernelGGL(k_tau_partial, dim3(kTauBlocks), dim3(kBlock), 0, stream, b.tau_part,
                           n, b.tau_blocks);
        hipLaunchKernelGGL(k_tau_final, dim3(1), dim3(kTauBlocks), 0, stream, b.tau_blocks,
                           g_tau);
    }
    return hipGetLastError();
}

}  // namespace orca
