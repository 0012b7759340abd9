/*
 * FP64 CPU oracle for one ORCA step of pedestrians and vehicles
 * ("Simulating Crowds and Autonomous Vehicles", Charlton et al.), and for
 * the gradient of that step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * library path never calls it and shares no code with it.
 *
 * Every quantity is computed in IEEE double; FP32 caller state is widened
 * exactly.  Build with -ffp-contract=off so that the neighbour key below is
 * evaluated exactly as written.
 *
 * Notation: P = p_B - p_A, V = v_A - v_B (current velocities serve as the
 * "optimal" velocities), R = r_A + r_B, det(a,b) = a.x*b.y - a.y*b.x.
 * A half-plane is a point q and a unit direction d; its permitted side is
 * {v : det(d, v - q) >= 0}.  With the normal n = (-d.y, d.x) (equivalently
 * d = (n.y, -n.x)) this is n . (v - q) >= 0, and the penetration of v is
 * delta(v) = det(d, q - v) (positive = violated).
 *
 * What each function follows:
 *  - neighbour set: Sec. 3 (each agent observes the nearby agents; the
 *    conclusions note that considering fewer people trades memory for
 *    realism) -> exact k nearest within the neighbour distance, ties by index.
 *  - half-plane: Fig. 1(b,c) (truncated velocity obstacle, the vector u to
 *    its boundary) and Sec. 3.1 (ORCA_{A|B} = v_opt + f_{A|B} u, with the
 *    responsibility table person-person 1/2, car-car 1/2, person-car 1,
 *    car-person 0).
 *  - LP2: Sec. 3 (the permitted velocity closest to the desired one, solved
 *    incrementally, one constraint at a time, re-solving on the violated
 *    line), with the speed cap as a disc constraint.
 *  - LP3: Sec. 3 (when the half-planes leave no permitted velocity, pick the
 *    one that least penetrates them): incremental minimisation of the
 *    largest penetration.
 *  - desired velocity and update: Sec. 3 / Sec. 4 (velocity toward the goal
 *    scaled to the speed; all agents updated simultaneously, explicit Euler).
 *  - acceleration and turn-rate limits: Sec. 5 (vehicles whose own motion
 *    limits -- acceleration, non-holonomic motion -- add linear constraints
 *    to the same LP); see accel_lines and turn_lines.
 *
 * Gradient (not in the paper; the differentiable form of the step): every
 * function of one agent's update is a template over its scalar type.  With
 * T = double it is the step itself; with T = Dual<N> (a value and N partial
 * derivatives) the same instructions propagate derivatives forward, so the
 * result is the exact derivative of the piecewise-smooth map at the current
 * branch decisions (neighbour sets and every comparison held fixed).  Each
 * data-dependent branch outcome is also mixed into a per-agent trace hash, so
 * that finite-difference checks can tell when a perturbation crossed a kink.
 *
 * Readings where the paper is silent (overlap rule, tie rules, parallel
 * tolerance, f = 0 kept as a constraint, LP3 tie rule) are listed at the
 * functions that use them.
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

#include <omp.h>

#define ORACLE_K_MAX 64
#define ORACLE_ACC 8   /* acceleration lines of an acceleration-limited agent */
#define ORACLE_TURN 2  /* heading lines of a turn-rate-limited agent */
#define ORACLE_HARD (ORACLE_ACC + ORACLE_TURN)
#define ORACLE_NWORK 12

namespace {

/* ------------------------------------------------------------------------ */
/* Scalars: double, or a forward-mode dual number.                          */
/* ------------------------------------------------------------------------ */
template <int N>
struct Dual {
    double v;
    double g[N];
    Dual() : v(0.0) { std::fill(g, g + N, 0.0); }
    Dual(double x) : v(x) { std::fill(g, g + N, 0.0); }  // NOLINT: implicit on purpose
};

template <int N> Dual<N> operator+(const Dual<N> &a, const Dual<N> &b)
{
    Dual<N> r(a.v + b.v);
    for (int k = 0; k < N; ++k) r.g[k] = a.g[k] + b.g[k];
    return r;
}
template <int N> Dual<N> operator-(const Dual<N> &a, const Dual<N> &b)
{
    Dual<N> r(a.v - b.v);
    for (int k = 0; k < N; ++k) r.g[k] = a.g[k] - b.g[k];
    return r;
}
template <int N> Dual<N> operator-(const Dual<N> &a)
{
    Dual<N> r(-a.v);
    for (int k = 0; k < N; ++k) r.g[k] = -a.g[k];
    return r;
}
template <int N> Dual<N> operator*(const Dual<N> &a, const Dual<N> &b)
{
    Dual<N> r(a.v * b.v);
    for (int k = 0; k < N; ++k) r.g[k] = a.g[k] * b.v + a.v * b.g[k];
    return r;
}
template <int N> Dual<N> operator/(const Dual<N> &a, const Dual<N> &b)
{
    Dual<N> r(a.v / b.v);
    for (int k = 0; k < N; ++k) r.g[k] = (a.g[k] - r.v * b.g[k]) / b.v;
    return r;
}
template <int N> Dual<N> operator+(const Dual<N> &a, double b) { return a + Dual<N>(b); }
template <int N> Dual<N> operator+(double a, const Dual<N> &b) { return Dual<N>(a) + b; }
template <int N> Dual<N> operator-(const Dual<N> &a, double b) { return a - Dual<N>(b); }
template <int N> Dual<N> operator-(double a, const Dual<N> &b) { return Dual<N>(a) - b; }
template <int N> Dual<N> operator*(const Dual<N> &a, double b) { return a * Dual<N>(b); }
template <int N> Dual<N> operator*(double a, const Dual<N> &b) { return Dual<N>(a) * b; }
template <int N> Dual<N> operator/(const Dual<N> &a, double b) { return a / Dual<N>(b); }
template <int N> Dual<N> operator/(double a, const Dual<N> &b) { return Dual<N>(a) / b; }

inline double val(double x) { return x; }
template <int N> double val(const Dual<N> &x) { return x.v; }

inline double sqrt_(double x) { return sqrt(x); }
template <int N> Dual<N> sqrt_(const Dual<N> &x)
{
    Dual<N> r(sqrt(x.v));
    for (int k = 0; k < N; ++k) r.g[k] = x.g[k] / (2.0 * r.v);
    return r;
}

inline double abs_(double x) { return fabs(x); }
template <int N> Dual<N> abs_(const Dual<N> &x) { return x.v < 0.0 ? -x : x; }

/* Hash of branch outcomes (FNV-1a over small codes). */
struct Trace {
    uint64_t h = 1469598103934665603ull;
    void mix(uint64_t x)
    {
        h ^= x + 0x9e3779b97f4a7c15ull;
        h *= 1099511628211ull;
    }
};

template <class T> T det2(T ax, T ay, T bx, T by) { return ax * by - ay * bx; }

template <class T>
struct Line {
    T qx, qy; /* point on the boundary line */
    T dx, dy; /* unit direction; permitted side is to its left */
};

struct OParams {
    double dt, tau, rn;
    int32_t k;
    int32_t pref_is_goal;
    double f[2][2];
    double eps;
    double accel[2]; /* acceleration cap per class [m/s^2]; 0 = none */
    double turn[2];  /* turn-rate cap per class [rad/s]; 0 = none */
};

/* ------------------------------------------------------------------------ */
/* Half-plane ORCA_{A|B} (Fig. 1(b,c), Sec. 3.1).                           */
/*                                                                          */
/* The truncated velocity obstacle of B for A over horizon tau is the set   */
/* of relative velocities V with t*V inside Disc(P, R) for some t in        */
/* [0, tau]: the disc Disc(P/tau, R/tau) joined to the cone from the        */
/* origin tangent to it.  u is the shortest vector from V to its boundary;  */
/* n is the outward normal of the boundary at V + u.                        */
/*                                                                          */
/* Readings:                                                                */
/*  - v_opt is the current velocity.                                        */
/*  - boundary branch: cutoff arc when the angle between w = V - P/tau and  */
/*    -P is below arccos(R/|P|); otherwise the left leg when det(P,w) > 0,  */
/*    else the right leg (det = 0 goes right).                              */
/*  - already overlapping (|P| <= R): horizon replaced by the step dt and   */
/*    only the disc is used; if w = 0 the normal is (+1,0) when the own     */
/*    index is smaller than the neighbour's, else (-1,0).                   */
/*  - f = 0 keeps the constraint through v_A (same code path for all).      */
/* branch: 0 cutoff arc, 1 left leg, 2 right leg, 3 overlap.                */
/* out: qx, qy, dx, dy, ux, uy, nx, ny.                                     */
/* ------------------------------------------------------------------------ */
template <class T>
int halfplane(T pax, T pay, T vax, T vay, double ra, T pbx, T pby, T vbx, T vby, double rb,
              double f, T tau, double dt, int a_before_b, T *out, Trace &tr)
{
    const T Px = pbx - pax, Py = pby - pay;
    const T Vx = vax - vbx, Vy = vay - vby;
    const double R = ra + rb;
    const T dist2 = Px * Px + Py * Py;
    const double R2 = R * R;
    T ux, uy, nx, ny;
    int branch;
    if (val(dist2) > R2) {
        const T wx = Vx - Px / tau, wy = Vy - Py / tau;
        const T w2 = wx * wx + wy * wy;
        const T wp = wx * Px + wy * Py;
        if (val(wp) < 0.0 && val(wp * wp) > val(R2 * w2)) {
            const T wl = sqrt_(w2);
            nx = wx / wl;
            ny = wy / wl;
            const T ul = R / tau - wl;
            ux = ul * nx;
            uy = ul * ny;
            branch = 0;
        } else {
            const T leg = sqrt_(dist2 - R2);
            T ex, ey;
            if (val(det2(Px, Py, wx, wy)) > 0.0) {
                /* P rotated counter-clockwise by asin(R/|P|), unit length */
                ex = (Px * leg - Py * R) / dist2;
                ey = (Px * R + Py * leg) / dist2;
                nx = -ey;
                ny = ex;
                branch = 1;
            } else {
                /* P rotated clockwise by asin(R/|P|) */
                ex = (Px * leg + Py * R) / dist2;
                ey = (-Px * R + Py * leg) / dist2;
                nx = ey;
                ny = -ex;
                branch = 2;
            }
            const T s = Vx * ex + Vy * ey;
            ux = s * ex - Vx;
            uy = s * ey - Vy;
        }
    } else {
        const T wx = Vx - Px / dt, wy = Vy - Py / dt;
        const T wl = sqrt_(wx * wx + wy * wy);
        if (val(wl) > 0.0) {
            nx = wx / wl;
            ny = wy / wl;
        } else {
            nx = a_before_b ? 1.0 : -1.0;
            ny = 0.0;
        }
        const T ul = R / dt - wl;
        ux = ul * nx;
        uy = ul * ny;
        branch = 3;
    }
    tr.mix(10 + branch);
    out[0] = vax + f * ux;
    out[1] = vay + f * uy;
    out[2] = ny;
    out[3] = -nx;
    out[4] = ux;
    out[5] = uy;
    out[6] = nx;
    out[7] = ny;
    return branch;
}

/* ------------------------------------------------------------------------ */
/* One-dimensional sub-problem on line i of the incremental LP (Sec. 3: a   */
/* violated constraint moves the optimum onto its boundary line).           */
/* Feasible parameters t of q_i + t d_i: inside the speed disc and on the   */
/* permitted side of every line j < i.                                      */
/* mode 0: closest point to (ox, oy).                                       */
/* mode 1: extreme point along the unit direction (ox, oy); when the line   */
/*         is orthogonal to it (|d_i . o| <= eps) the point of the interval */
/*         closest to (tx, ty) is taken (proposed tie rule).                */
/* Lines with |det(d_j, d_i)| <= eps are treated as parallel: infeasible if */
/* line i lies outside line j, otherwise skipped.                           */
/* Returns 1 and writes v on success, 0 if the interval is empty.           */
/* *iters counts the j-loop iterations executed.                            */
/* ------------------------------------------------------------------------ */
template <class T>
int lp1(const Line<T> *L, int i, double vmax, T ox, T oy, int mode, T tx, T ty, double eps,
        T *vx, T *vy, int64_t *iters, Trace &tr)
{
    const Line<T> *li = &L[i];
    const T dot = li->qx * li->dx + li->qy * li->dy;
    const T disc = dot * dot + vmax * vmax - (li->qx * li->qx + li->qy * li->qy);
    if (val(disc) < 0.0) {
        tr.mix(20);
        return 0;
    }
    const T sq = sqrt_(disc);
    T tl = -dot - sq, tr_ = -dot + sq;
    int src_l = -1, src_r = -1; /* which constraint bounds each end (-1: disc) */
    for (int j = 0; j < i; ++j) {
        ++*iters;
        const Line<T> *lj = &L[j];
        const T a = det2(lj->dx, lj->dy, li->dx, li->dy);
        const T b = det2(lj->dx, lj->dy, li->qx - lj->qx, li->qy - lj->qy);
        if (fabs(val(a)) <= eps) {
            /* parallel within eps: line i lies wholly outside line j only
             * when it is offset to j's forbidden side by more than
             * 2^-20 v_max; closer than that the two are the same line */
            if (val(b) < -std::ldexp(vmax, -20)) {
                tr.mix(21);
                return 0;
            }
            continue;
        }
        const T t = -b / a;
        if (val(a) > 0.0) {
            if (val(t) > val(tl)) {
                tl = t;
                src_l = j;
            }
        } else {
            if (val(t) < val(tr_)) {
                tr_ = t;
                src_r = j;
            }
        }
        if (val(tl) > val(tr_)) {
            tr.mix(22);
            return 0;
        }
    }
    T t;
    int how;
    if (mode == 0) {
        t = li->dx * (ox - li->qx) + li->dy * (oy - li->qy);
        how = 0;
        if (val(t) < val(tl)) {
            t = tl;
            how = 1;
        }
        if (val(t) > val(tr_)) {
            t = tr_;
            how = 2;
        }
    } else {
        const T s = ox * li->dx + oy * li->dy;
        if (fabs(val(s)) <= eps) {
            t = li->dx * (tx - li->qx) + li->dy * (ty - li->qy);
            how = 3;
            if (val(t) < val(tl)) {
                t = tl;
                how = 1;
            }
            if (val(t) > val(tr_)) {
                t = tr_;
                how = 2;
            }
        } else {
            const bool right = val(s) > 0.0;
            t = right ? tr_ : tl;
            how = right ? 2 : 1;
        }
    }
    tr.mix(30 + how);
    tr.mix(100 + (how == 1 ? src_l : how == 2 ? src_r : -2) + 2);
    *vx = li->qx + t * li->dx;
    *vy = li->qy + t * li->dy;
    return 1;
}

/* Incremental 2D LP over lines 0..m-1 and the disc |v| <= vmax.
 * mode 0: v* = argmin |v - o| (start at o, or at vmax*o/|o| outside the disc).
 * mode 1: maximise v . o for unit o (start at vmax*o).
 * Returns the index of the first line whose sub-problem is infeasible, or m;
 * on failure v keeps the value it had before that line. */
template <class T>
int lp2_mode(const Line<T> *L, int m, double vmax, T ox, T oy, int mode, T tx, T ty, double eps,
             T *vx, T *vy, int64_t *n_check, int64_t *n_viol, int64_t *iters, Trace &tr)
{
    T x, y;
    if (mode == 1) {
        x = ox * vmax;
        y = oy * vmax;
    } else {
        const T o2 = ox * ox + oy * oy;
        if (val(o2) > vmax * vmax) {
            const T ol = sqrt_(o2);
            x = ox / ol * vmax;
            y = oy / ol * vmax;
            tr.mix(40);
        } else {
            x = ox;
            y = oy;
            tr.mix(41);
        }
    }
    for (int i = 0; i < m; ++i) {
        ++*n_check;
        if (val(det2(L[i].dx, L[i].dy, L[i].qx - x, L[i].qy - y)) > 0.0) {
            ++*n_viol;
            tr.mix(1000 + i);
            T nx2 = x, ny2 = y;
            if (!lp1(L, i, vmax, ox, oy, mode, tx, ty, eps, &nx2, &ny2, iters, tr)) {
                *vx = x;
                *vy = y;
                return i;
            }
            x = nx2;
            y = ny2;
        }
    }
    *vx = x;
    *vy = y;
    return m;
}

/* ------------------------------------------------------------------------ */
/* LP3: least penetration (Sec. 3, infeasible case).                        */
/* The plain objective is min over |v| <= vmax of max_j delta_j(v), with    */
/* delta_j(v) = det(d_j, q_j - v).  It is reached incrementally from LP2's  */
/* partial result: for each later line i whose penetration exceeds the      */
/* current level, v is re-solved in the region where no earlier line        */
/* penetrates more than line i does (boundaries of delta_j = delta_i),      */
/* pushing v as far as possible into line i's permitted side.               */
/* The first nh lines are hard (the agent's own motion limits): they are    */
/* never relaxed, i.e. they enter every re-solve unchanged and the max runs */
/* over lines nh..m-1 only.                                                 */
/* w: re-solved lines, boundary lines built, checked, re-solved, inner.     */
/* ------------------------------------------------------------------------ */
template <class T>
void lp3(const Line<T> *L, int m, int nh, int fail, double vmax, T tx, T ty, double eps, T *vx,
         T *vy, int64_t *w, Trace &tr)
{
    Line<T> proj[ORACLE_K_MAX + ORACLE_HARD]{};
    T level = 0.0;
    T x = *vx, y = *vy;
    for (int i = fail > nh ? fail : nh; i < m; ++i) {
        const Line<T> *li = &L[i];
        if (val(det2(li->dx, li->dy, li->qx - x, li->qy - y)) <= val(level)) continue;
        ++w[0];
        tr.mix(2000 + i);
        int np = 0;
        /* hard lines stay constraints as they are */
        for (int j = 0; j < nh; ++j) proj[np++] = L[j];
        for (int j = nh; j < i; ++j) {
            const Line<T> *lj = &L[j];
            const T dij = det2(li->dx, li->dy, lj->dx, lj->dy);
            T ptx, pty;
            if (fabs(val(dij)) <= eps) {
                if (val(li->dx * lj->dx + li->dy * lj->dy) > 0.0) continue; /* same direction */
                ptx = 0.5 * (li->qx + lj->qx);
                pty = 0.5 * (li->qy + lj->qy);
            } else {
                const T t = det2(lj->dx, lj->dy, li->qx - lj->qx, li->qy - lj->qy) / dij;
                ptx = li->qx + t * li->dx;
                pty = li->qy + t * li->dy;
            }
            T ddx = lj->dx - li->dx, ddy = lj->dy - li->dy;
            const T dl = sqrt_(ddx * ddx + ddy * ddy);
            proj[np].qx = ptx;
            proj[np].qy = pty;
            proj[np].dx = ddx / dl;
            proj[np].dy = ddy / dl;
            ++np;
        }
        w[1] += np;
        T nx = x, ny = y;
        /* objective direction: the inward normal of line i, (-d.y, d.x) */
        if (lp2_mode(proj, np, vmax, -li->dy, li->dx, 1, tx, ty, eps, &nx, &ny, &w[2], &w[3], &w[4],
                     tr) == np) {
            x = nx;
            y = ny;
            tr.mix(50);
        } else {
            tr.mix(51);
        }
        level = det2(li->dx, li->dy, li->qx - x, li->qy - y);
    }
    *vx = x;
    *vy = y;
}

/* ------------------------------------------------------------------------ */
/* One agent's velocity update from its own and its neighbours' state.      */
/* Desired velocity (goal mode): (g - p) * min(v_max/|g - p|, 1/dt), zero   */
/* when p = g; otherwise pref holds v_pref itself.                          */
/* ------------------------------------------------------------------------ */
template <class T>
struct AgentIn {
    T px, py, vx, vy, prx, pry, tau;
    T npx[ORACLE_K_MAX], npy[ORACLE_K_MAX], nvx[ORACLE_K_MAX], nvy[ORACLE_K_MAX];
};

/* ------------------------------------------------------------------------ */
/* Acceleration limit (Sec. 5 names acceleration-limited and non-holonomic  */
/* vehicles as an extension whose motion limits add linear constraints to  */
/* the same LP).  Reading: within one step the velocity can change by at    */
/* most a dt, so the new velocity must lie in the disc of radius a dt about */
/* the current velocity c -- taken scaled onto the speed circle when it lies */
/* outside it, so that the two regions always meet.  The disc is replaced   */
/* by the regular octagon inscribed in it (everything the octagon allows    */
/* respects the limit): edge k has outward unit normal n_k at angle k pi/4  */
/* and lies a dt cos(pi/8) from c, i.e. the constraint n_k . (v - c) <= h.  */
/* As a line: q = c + h n_k, d = (-n_k.y, n_k.x) (inward normal -n_k).      */
/* The eight lines are hard: they precede the ORCA lines in LP2 and LP3     */
/* never relaxes them.  Returns the number of lines written (0 or 8).       */
/* ------------------------------------------------------------------------ */
template <class T>
void accel_centre(T vx, T vy, double vmax, T *cx, T *cy)
{
    *cx = vx;
    *cy = vy;
    const T v2 = vx * vx + vy * vy;
    if (val(v2) > vmax * vmax) {
        const T s = vmax / sqrt_(v2);
        *cx = vx * s;
        *cy = vy * s;
    }
}

template <class T>
int accel_lines(T vx, T vy, double vmax, double accel, double dt, Line<T> *out)
{
    if (!(accel > 0.0)) return 0;
    T cx, cy;
    accel_centre<T>(vx, vy, vmax, &cx, &cy);
    const double h = accel * dt * std::cos(M_PI / 8.0);
    for (int k = 0; k < ORACLE_ACC; ++k) {
        const double nx = std::cos(k * M_PI / 4.0), ny = std::sin(k * M_PI / 4.0);
        out[k].qx = cx + h * nx;
        out[k].qy = cy + h * ny;
        out[k].dx = T(-ny);
        out[k].dy = T(nx);
    }
    return ORACLE_ACC;
}

/* ------------------------------------------------------------------------ */
/* Turn-rate limit: the non-holonomic half of the same Sec. 5 extension.    */
/* Reading: a vehicle moves along its heading, the direction of its current */
/* velocity, and can turn it by at most w dt within one step, so the new    */
/* velocity must lie in the wedge of half-angle phi = min(w dt, pi/2) about */
/* that heading, apex at the origin (braking to rest stays possible).  For  */
/* phi <= pi/2 the wedge is convex: with h = v/|v| and R(a) the rotation by */
/* a, its sides are the rays along r_R = R(-phi) h and r_L = R(phi) h, and  */
/* the constraints det(r_R, v) >= 0, det(v, r_L) >= 0 are the lines through */
/* the origin with directions r_R and -r_L (permitted side on the left).    */
/* At rest (v = 0) there is no heading and no wedge.  The lines are hard,   */
/* after any acceleration lines.  Returns the number written (0 or 2).      */
/* ------------------------------------------------------------------------ */
template <class T>
int turn_lines(T vx, T vy, double turn, double dt, Line<T> *out)
{
    if (!(turn > 0.0)) return 0;
    const T v2 = vx * vx + vy * vy;
    if (!(val(v2) > 0.0)) return 0;
    const T sp = sqrt_(v2);
    const T hx = vx / sp, hy = vy / sp;
    const double phi = std::min(turn * dt, M_PI / 2.0);
    const double c = std::cos(phi), s = std::sin(phi);
    out[0].qx = T(0.0);
    out[0].qy = T(0.0);
    out[0].dx = hx * c + hy * s; /* r_R */
    out[0].dy = hy * c - hx * s;
    out[1].qx = T(0.0);
    out[1].qy = T(0.0);
    out[1].dx = -(hx * c - hy * s); /* -r_L */
    out[1].dy = -(hy * c + hx * s);
    return ORACLE_TURN;
}

template <class T>
int agent_update(const AgentIn<T> &a, int self, double r, int cls, double vmax, int m,
                 const int32_t *nb, const double *radius, const uint8_t *klass, const OParams &prm,
                 T *vx_out, T *vy_out, int64_t *w, Trace &tr)
{
    Line<T> L[ORACLE_K_MAX + ORACLE_HARD];
    const int na = accel_lines<T>(a.vx, a.vy, vmax, prm.accel[cls & 1], prm.dt, L);
    const int nh = na + turn_lines<T>(a.vx, a.vy, prm.turn[cls & 1], prm.dt, L + na);
    if (nh) tr.mix(val(a.vx * a.vx + a.vy * a.vy) > vmax * vmax ? 71 : 70); /* centre clipped */
    T prx, pry;
    if (prm.pref_is_goal) {
        const T gx = a.prx - a.px, gy = a.pry - a.py;
        const T d2 = gx * gx + gy * gy;
        if (val(d2) > 0.0) {
            const T d = sqrt_(d2);
            T s = vmax / d;
            if (1.0 / prm.dt < val(s)) s = 1.0 / prm.dt;
            prx = gx * s;
            pry = gy * s;
        } else {
            prx = 0.0;
            pry = 0.0;
        }
    } else {
        prx = a.prx;
        pry = a.pry;
    }
    for (int s = 0; s < m; ++s) {
        const int j = nb[s];
        T hp[8];
        halfplane<T>(a.px, a.py, a.vx, a.vy, r, a.npx[s], a.npy[s], a.nvx[s], a.nvy[s], radius[j],
                     prm.f[cls & 1][klass[j] & 1], a.tau, prm.dt, self < j, hp, tr);
        L[nh + s].qx = hp[0];
        L[nh + s].qy = hp[1];
        L[nh + s].dx = hp[2];
        L[nh + s].dy = hp[3];
    }
    const int mt = nh + m;
    T nvx, nvy;
    int fail = lp2_mode<T>(L, mt, vmax, prx, pry, 0, T(0.0), T(0.0), prm.eps, &nvx, &nvy, &w[3],
                           &w[4], &w[5], tr);
    int st = 0;
    if (fail < nh) {
        /* the hard lines and the speed disc always meet (the centre, the
         * current velocity scaled into the disc, lies in the octagon and on
         * the heading wedge's axis), so this is rounding alone; the centre
         * itself is then taken and LP3 starts from it */
        accel_centre<T>(a.vx, a.vy, vmax, &nvx, &nvy);
        tr.mix(60);
        fail = nh;
        st = 1;
    }
    if (fail < mt) {
        lp3<T>(L, mt, nh, fail, vmax, prx, pry, prm.eps, &nvx, &nvy, &w[7], tr);
        st = 1;
        w[6] = 1;
    }
    tr.mix(3000 + fail);
    *vx_out = nvx;
    *vy_out = nvy;
    return st;
}

/* ------------------------------------------------------------------------ */
/* Neighbour search (Sec. 3: nearby agents; the neighbour cap k).           */
/* Definition: the k agents j != i with the smallest (key_ij, j) among      */
/* those with key_ij < R_n^2, in ascending (key, j) order, where            */
/*   dx = x_j - x_i, dy = y_j - y_i   (double, from the positions)          */
/*   key = dx*dx + dy*dy              (double, each operation rounded)      */
/*   R_n^2 = R_n * R_n                (double)                              */
/* (positions given in FP32 are widened exactly first).  A uniform grid of  */
/* cell size >= R_n only bounds which j are examined.                       */
/* ------------------------------------------------------------------------ */
struct Cand {
    double key;
    int32_t j;
};

bool cand_less(const Cand &x, const Cand &y)
{
    if (x.key < y.key) return true;
    if (x.key > y.key) return false;
    return x.j < y.j;
}

struct OGrid {
    double x0, y0, cs;
    int64_t nx, ny;
    std::vector<int32_t> start; /* nx*ny + 1 */
    std::vector<int32_t> order; /* agent indices sorted by (cell, index) */
};

int64_t cell_coord(double v, double v0, double cs, int64_t nmax)
{
    int64_t c = (int64_t)floor((v - v0) / cs);
    if (c < 0) c = 0;
    if (c >= nmax) c = nmax - 1;
    return c;
}

void ogrid_build(OGrid &g, int n, const double *px, const double *py, double rn)
{
    double x0 = px[0], y0 = py[0], x1 = px[0], y1 = py[0];
    for (int i = 1; i < n; ++i) {
        if (px[i] < x0) x0 = px[i];
        if (px[i] > x1) x1 = px[i];
        if (py[i] < y0) y0 = py[i];
        if (py[i] > y1) y1 = py[i];
    }
    /* slightly wider than R_n so that rounding of the cell coordinates can
     * never push an in-range pair more than one cell apart */
    double cs = (rn > 0.0 ? rn : 1.0) * (1.0 + 1e-6);
    for (;;) {
        g.nx = (int64_t)floor((x1 - x0) / cs) + 1;
        g.ny = (int64_t)floor((y1 - y0) / cs) + 1;
        if (g.nx * g.ny <= 4 * (int64_t)n + 1024) break;
        cs *= 2.0; /* a coarser grid still covers every in-range pair */
    }
    g.x0 = x0;
    g.y0 = y0;
    g.cs = cs;
    const int64_t nc = g.nx * g.ny;
    g.start.assign((size_t)nc + 1, 0);
    g.order.assign((size_t)n, 0);
    std::vector<int64_t> cell((size_t)n);
    for (int i = 0; i < n; ++i) {
        cell[i] = cell_coord(px[i], x0, cs, g.nx) + g.nx * cell_coord(py[i], y0, cs, g.ny);
        g.start[cell[i] + 1]++;
    }
    for (int64_t c = 0; c < nc; ++c) g.start[c + 1] += g.start[c];
    std::vector<int32_t> fill(g.start.begin(), g.start.end());
    for (int i = 0; i < n; ++i) g.order[fill[cell[i]]++] = i; /* stable: (cell, index) */
}

/* Exact k nearest of agent i; returns the number kept, writes the in-range
 * count and the number of candidates examined. */
int knn_one(const OGrid &g, int i, const double *px, const double *py, double rn2, int k,
            std::vector<Cand> &buf, int32_t *nbr, int64_t *n_inrange, int64_t *n_cand)
{
    const double xi = px[i], yi = py[i];
    const int64_t cx = cell_coord(xi, g.x0, g.cs, g.nx);
    const int64_t cy = cell_coord(yi, g.y0, g.cs, g.ny);
    buf.clear();
    for (int64_t yy = cy - 1; yy <= cy + 1; ++yy) {
        if (yy < 0 || yy >= g.ny) continue;
        for (int64_t xx = cx - 1; xx <= cx + 1; ++xx) {
            if (xx < 0 || xx >= g.nx) continue;
            const int64_t c = xx + g.nx * yy;
            for (int32_t s = g.start[c]; s < g.start[c + 1]; ++s) {
                const int32_t j = g.order[s];
                ++*n_cand;
                if (j == i) continue;
                const double dx = px[j] - xi;
                const double dy = py[j] - yi;
                const double key = dx * dx + dy * dy;
                if (!(key < rn2)) continue;
                buf.push_back(Cand{key, j});
            }
        }
    }
    *n_inrange = (int64_t)buf.size();
    std::sort(buf.begin(), buf.end(), cand_less);
    const int cnt = (int)buf.size();
    const int m = cnt < k ? cnt : k;
    for (int s = 0; s < m; ++s) nbr[s] = buf[s].j;
    for (int s = m; s < k; ++s) nbr[s] = -1;
    return m;
}

/* State of one scene in double (FP32 callers are widened exactly). */
struct DState {
    int n;
    const double *px, *py, *vx, *vy, *prx, *pry, *radius, *vmax;
    const uint8_t *cls;
};

AgentIn<double> agent_in(const DState &S, int i, const int32_t *nb, int m, double tau)
{
    AgentIn<double> a;
    a.px = S.px[i];
    a.py = S.py[i];
    a.vx = S.vx[i];
    a.vy = S.vy[i];
    a.prx = S.prx[i];
    a.pry = S.pry[i];
    a.tau = tau;
    for (int s = 0; s < m; ++s) {
        a.npx[s] = S.px[nb[s]];
        a.npy[s] = S.py[nb[s]];
        a.nvx[s] = S.vx[nb[s]];
        a.nvy[s] = S.vy[nb[s]];
    }
    return a;
}

bool params_ok(const OParams *prm)
{
    return prm && prm->k >= 1 && prm->k <= ORACLE_K_MAX && prm->dt > 0.0 && prm->tau > 0.0 &&
           prm->rn > 0.0 && prm->accel[0] >= 0.0 && prm->accel[1] >= 0.0 &&
           std::isfinite(prm->accel[0]) && std::isfinite(prm->accel[1]) &&
           prm->turn[0] >= 0.0 && prm->turn[1] >= 0.0 && std::isfinite(prm->turn[0]) &&
           std::isfinite(prm->turn[1]);
}

/* One synchronous step of every agent of one scene (double state). */
int step_impl(const DState &S, const OParams *prm, double *opx, double *opy, double *ovx,
              double *ovy, uint8_t *status, int32_t *nbr_out, int32_t *cnt_out, int64_t *work,
              double *lines_out, double *pref_out, uint64_t *trace)
{
    const int n = S.n;
    if (n < 0 || !params_ok(prm)) return -1;
    if (n == 0) return 0;
    OGrid g;
    ogrid_build(g, n, S.px, S.py, prm->rn);
    const double rn2 = prm->rn * prm->rn;
    const int k = prm->k;
#pragma omp parallel
    {
        std::vector<Cand> buf;
#pragma omp for schedule(static)
        for (int i = 0; i < n; ++i) {
            int32_t nb[ORACLE_K_MAX];
            int64_t w[ORACLE_NWORK] = {0};
            const int m = knn_one(g, i, S.px, S.py, rn2, k, buf, nb, &w[1], &w[0]);
            w[2] = m;
            const AgentIn<double> a = agent_in(S, i, nb, m, prm->tau);
            Trace tr;
            for (int s = 0; s < m; ++s) tr.mix(5000 + (uint64_t)nb[s]);
            double nvx, nvy;
            const int st = agent_update<double>(a, i, S.radius[i], S.cls[i], S.vmax[i], m, nb,
                                                S.radius, S.cls, *prm, &nvx, &nvy, w, tr);
            ovx[i] = nvx;
            ovy[i] = nvy;
            opx[i] = a.px + nvx * prm->dt;
            opy[i] = a.py + nvy * prm->dt;
            if (status) status[i] = (uint8_t)st;
            if (nbr_out) memcpy(nbr_out + (int64_t)i * k, nb, (size_t)k * sizeof(int32_t));
            if (cnt_out) cnt_out[i] = m;
            if (work) memcpy(work + (int64_t)i * ORACLE_NWORK, w, sizeof(w));
            if (trace) trace[i] = tr.h;
            if (lines_out || pref_out) {
                /* the half-planes and desired velocity of this agent, recomputed */
                Trace t2;
                double *lo = lines_out ? lines_out + (int64_t)i * k * 4 : nullptr;
                for (int s = 0; s < k; ++s) {
                    double hp[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                    if (s < m)
                        halfplane<double>(a.px, a.py, a.vx, a.vy, S.radius[i], a.npx[s], a.npy[s],
                                          a.nvx[s], a.nvy[s], S.radius[nb[s]],
                                          prm->f[S.cls[i] & 1][S.cls[nb[s]] & 1], a.tau, prm->dt,
                                          i < nb[s], hp, t2);
                    if (lo) memcpy(lo + 4 * s, hp, 4 * sizeof(double));
                }
                if (pref_out) {
                    double prx = a.prx, pry = a.pry;
                    if (prm->pref_is_goal) {
                        const double gx = a.prx - a.px, gy = a.pry - a.py;
                        const double d2 = gx * gx + gy * gy;
                        if (d2 > 0.0) {
                            double sc = S.vmax[i] / sqrt(d2);
                            if (1.0 / prm->dt < sc) sc = 1.0 / prm->dt;
                            prx = gx * sc;
                            pry = gy * sc;
                        } else {
                            prx = 0.0;
                            pry = 0.0;
                        }
                    }
                    pref_out[2 * i] = prx;
                    pref_out[2 * i + 1] = pry;
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Vector-Jacobian product of one step (double state).                      */
/* For agent i the inputs of its update are its own position, velocity,    */
/* pref input (goal or desired velocity), the shared tau, and its           */
/* neighbours' positions and velocities: 7 + 4m scalars.  Their partial     */
/* derivatives are propagated forward in chunks of 8 with Dual<8>.  Given   */
/* the cotangents gp1, gv1 of (p', v'), the cotangent of the new velocity is */
/* w = gv1 + gp1 dt (p' = p + v' dt), and                                   */
/*   gp0_i = gp1_i + sum over updates u of w_u . dv'_u/dp_i                 */
/*   gv0_i =         sum over updates u of w_u . dv'_u/dv_i                 */
/*   gpref_i += w_i . dv'_i/dpref_i,   gtau += sum_u w_u . dv'_u/dtau.       */
/* Contributions are added serially in agent order (deterministic).         */
/* ------------------------------------------------------------------------ */
constexpr int kChunk = 8;

int vjp_impl(const DState &S, const OParams *prm, const double *gpx1, const double *gpy1,
             const double *gvx1, const double *gvy1, double *gpx0, double *gpy0, double *gvx0,
             double *gvy0, double *gprx, double *gpry, double *gtau)
{
    const int n = S.n;
    if (n < 0 || !params_ok(prm)) return -1;
    if (n == 0) return 0;
    OGrid g;
    ogrid_build(g, n, S.px, S.py, prm->rn);
    const double rn2 = prm->rn * prm->rn;
    const int k = prm->k;
    const int ndir_max = 7 + 4 * k;
    std::vector<double> contrib((size_t)n * ndir_max, 0.0);
    std::vector<int32_t> nbrs((size_t)n * k, -1);
    std::vector<int32_t> cnts((size_t)n, 0);
#pragma omp parallel
    {
        std::vector<Cand> buf;
#pragma omp for schedule(static)
        for (int i = 0; i < n; ++i) {
            int32_t *nb = nbrs.data() + (size_t)i * k;
            int64_t w[ORACLE_NWORK] = {0};
            const int m = knn_one(g, i, S.px, S.py, rn2, k, buf, nb, &w[1], &w[0]);
            cnts[i] = m;
            const double wx = gvx1[i] + gpx1[i] * prm->dt;
            const double wy = gvy1[i] + gpy1[i] * prm->dt;
            const int ndir = 7 + 4 * m;
            double *out = contrib.data() + (size_t)i * ndir_max;
            for (int c0 = 0; c0 < ndir; c0 += kChunk) {
                AgentIn<Dual<kChunk>> a;
                const AgentIn<double> ad = agent_in(S, i, nb, m, prm->tau);
                a.px = ad.px;
                a.py = ad.py;
                a.vx = ad.vx;
                a.vy = ad.vy;
                a.prx = ad.prx;
                a.pry = ad.pry;
                a.tau = ad.tau;
                for (int s = 0; s < m; ++s) {
                    a.npx[s] = ad.npx[s];
                    a.npy[s] = ad.npy[s];
                    a.nvx[s] = ad.nvx[s];
                    a.nvy[s] = ad.nvy[s];
                }
                /* input order: px py vx vy prx pry tau, then per neighbour px py vx vy */
                Dual<kChunk> *slot[7] = {&a.px, &a.py, &a.vx, &a.vy, &a.prx, &a.pry, &a.tau};
                for (int d = c0; d < c0 + kChunk && d < ndir; ++d) {
                    Dual<kChunk> *x;
                    if (d < 7) {
                        x = slot[d];
                    } else {
                        const int s = (d - 7) / 4, f = (d - 7) % 4;
                        x = f == 0 ? &a.npx[s] : f == 1 ? &a.npy[s] : f == 2 ? &a.nvx[s] : &a.nvy[s];
                    }
                    x->g[d - c0] = 1.0;
                }
                Dual<kChunk> vx, vy;
                Trace tr;
                int64_t wd[ORACLE_NWORK] = {0};
                agent_update<Dual<kChunk>>(a, i, S.radius[i], S.cls[i], S.vmax[i], m, nb, S.radius,
                                           S.cls, *prm, &vx, &vy, wd, tr);
                for (int d = c0; d < c0 + kChunk && d < ndir; ++d)
                    out[d] = wx * vx.g[d - c0] + wy * vy.g[d - c0];
            }
        }
    }
    for (int i = 0; i < n; ++i) {
        gpx0[i] = gpx1[i];
        gpy0[i] = gpy1[i];
        gvx0[i] = 0.0;
        gvy0[i] = 0.0;
    }
    double tsum = 0.0;
    for (int i = 0; i < n; ++i) {
        const double *c = contrib.data() + (size_t)i * ndir_max;
        gpx0[i] += c[0];
        gpy0[i] += c[1];
        gvx0[i] += c[2];
        gvy0[i] += c[3];
        if (gprx) gprx[i] += c[4];
        if (gpry) gpry[i] += c[5];
        tsum += c[6];
        const int32_t *nb = nbrs.data() + (size_t)i * k;
        for (int s = 0; s < cnts[i]; ++s) {
            const int j = nb[s];
            gpx0[j] += c[7 + 4 * s];
            gpy0[j] += c[8 + 4 * s];
            gvx0[j] += c[9 + 4 * s];
            gvy0[j] += c[10 + 4 * s];
        }
    }
    if (gtau) *gtau += tsum;
    return 0;
}

/* FP32 caller arrays widened to double. */
struct Widened {
    std::vector<double> px, py, vx, vy, prx, pry, radius, vmax;
    DState s;
    Widened(int n, const float *px_, const float *py_, const float *vx_, const float *vy_,
            const float *prx_, const float *pry_, const float *r_, const float *vm_,
            const uint8_t *cls)
        : px(px_, px_ + n), py(py_, py_ + n), vx(vx_, vx_ + n), vy(vy_, vy_ + n),
          prx(prx_, prx_ + n), pry(pry_, pry_ + n), radius(r_, r_ + n), vmax(vm_, vm_ + n)
    {
        s = DState{n, px.data(), py.data(), vx.data(), vy.data(), prx.data(), pry.data(),
                   radius.data(), vmax.data(), cls};
    }
};

} /* namespace */

/* ======================================================================== */
/* C entry points (ctypes).                                                 */
/* ======================================================================== */
extern "C" {

typedef OParams oparams;

/* Sets the OpenMP thread count of later calls when t > 0; returns the count
 * now in effect. */
int oracle_set_threads(int t)
{
    if (t > 0) omp_set_num_threads(t);
    return omp_get_max_threads();
}

int oracle_halfplane(double pax, double pay, double vax, double vay, double ra, double pbx,
                     double pby, double vbx, double vby, double rb, double f, double tau,
                     double dt, int a_before_b, double *out /* qx,qy,dx,dy,ux,uy,nx,ny */)
{
    Trace tr;
    return halfplane<double>(pax, pay, vax, vay, ra, pbx, pby, vbx, vby, rb, f, tau, dt,
                             a_before_b, out, tr);
}

static void load_lines(int m, const double *lines, Line<double> *L)
{
    for (int i = 0; i < m; ++i) {
        L[i].qx = lines[4 * i + 0];
        L[i].qy = lines[4 * i + 1];
        L[i].dx = lines[4 * i + 2];
        L[i].dy = lines[4 * i + 3];
    }
}

/* Public LP entry points for the pin tests (lines as m x 4: qx,qy,dx,dy). */
int oracle_lp2(int m, const double *lines, double vmax, double ox, double oy, double eps,
               double *v)
{
    if (m < 0 || m > ORACLE_K_MAX) return -1;
    Line<double> L[ORACLE_K_MAX];
    load_lines(m, lines, L);
    int64_t a = 0, b = 0, c = 0;
    Trace tr;
    return lp2_mode<double>(L, m, vmax, ox, oy, 0, 0.0, 0.0, eps, &v[0], &v[1], &a, &b, &c, tr);
}

/* LP2 followed by LP3 when LP2 fails; returns the LP2 fail index (m = LP2
 * feasible, LP3 not run). */
int oracle_lp_full(int m, const double *lines, double vmax, double ox, double oy, double eps,
                   double *v)
{
    if (m < 0 || m > ORACLE_K_MAX) return -1;
    Line<double> L[ORACLE_K_MAX];
    load_lines(m, lines, L);
    int64_t a = 0, b = 0, c = 0, w[5] = {0};
    Trace tr;
    const int fail =
        lp2_mode<double>(L, m, vmax, ox, oy, 0, 0.0, 0.0, eps, &v[0], &v[1], &a, &b, &c, tr);
    if (fail < m) lp3<double>(L, m, 0, fail, vmax, ox, oy, eps, &v[0], &v[1], w, tr);
    return fail;
}

/* The same with the first nh lines hard (acceleration lines); a failure
 * among them takes v = hard_c (the octagon's centre).  Returns the LP2 fail
 * index. */
int oracle_lp_full_hard(int m, int nh, const double *lines, double vmax, double ox, double oy,
                        double eps, double cx, double cy, double *v)
{
    if (m < 0 || nh < 0 || nh > m || m > ORACLE_K_MAX + ORACLE_HARD) return -1;
    Line<double> L[ORACLE_K_MAX + ORACLE_HARD];
    load_lines(m, lines, L);
    int64_t a = 0, b = 0, c = 0, w[5] = {0};
    Trace tr;
    int fail =
        lp2_mode<double>(L, m, vmax, ox, oy, 0, 0.0, 0.0, eps, &v[0], &v[1], &a, &b, &c, tr);
    const int f0 = fail;
    if (fail < nh) {
        v[0] = cx;
        v[1] = cy;
        fail = nh;
    }
    if (fail < m) lp3<double>(L, m, nh, fail, vmax, ox, oy, eps, &v[0], &v[1], w, tr);
    return f0;
}

/* The eight acceleration lines of an agent with current velocity (vx, vy),
 * speed cap vmax, acceleration cap accel and step dt, as 8 x 4 (qx, qy, dx,
 * dy); returns the count (0 when accel <= 0). */
int oracle_accel_lines(double vx, double vy, double vmax, double accel, double dt, double *out)
{
    Line<double> L[ORACLE_ACC];
    const int nh = accel_lines<double>(vx, vy, vmax, accel, dt, L);
    for (int k = 0; k < nh; ++k) {
        out[4 * k + 0] = L[k].qx;
        out[4 * k + 1] = L[k].qy;
        out[4 * k + 2] = L[k].dx;
        out[4 * k + 3] = L[k].dy;
    }
    return nh;
}

/* The two heading lines of a turn-rate-limited agent with current velocity
 * (vx, vy), cap turn [rad/s] and step dt, as 2 x 4 (qx, qy, dx, dy);
 * returns the count (0 when turn <= 0 or v = 0). */
int oracle_turn_lines(double vx, double vy, double turn, double dt, double *out)
{
    Line<double> L[ORACLE_TURN];
    const int nh = turn_lines<double>(vx, vy, turn, dt, L);
    for (int k = 0; k < nh; ++k) {
        out[4 * k + 0] = L[k].qx;
        out[4 * k + 1] = L[k].qy;
        out[4 * k + 2] = L[k].dx;
        out[4 * k + 3] = L[k].dy;
    }
    return nh;
}

/* nbr: n x k (row-major, -1 padded), cnt: n.  Returns 0, or -1 on bad args. */
int oracle_knn(int n, const float *px, const float *py, float neighbor_dist, int k, int32_t *nbr,
               int32_t *cnt)
{
    if (n < 0 || k < 1 || k > ORACLE_K_MAX || !(neighbor_dist > 0.0f)) return -1;
    if (n == 0) return 0;
    std::vector<double> x(px, px + n), y(py, py + n);
    OGrid g;
    ogrid_build(g, n, x.data(), y.data(), (double)neighbor_dist);
    const double rn = (double)neighbor_dist;
    const double rn2 = rn * rn;
#pragma omp parallel
    {
        std::vector<Cand> buf;
#pragma omp for schedule(static)
        for (int i = 0; i < n; ++i) {
            int64_t a = 0, b = 0;
            cnt[i] = knn_one(g, i, x.data(), y.data(), rn2, k, buf, nbr + (int64_t)i * k, &a, &b);
        }
    }
    return 0;
}

/* One synchronous step of every agent of one scene from an FP32 state.
 * The LP result v' is the new velocity and p' = p + v' dt (explicit Euler),
 * all agents reading the step-t state.
 * work (nullable, n x 12): candidates examined, in-range count, neighbours
 * used; LP2 lines checked, lines re-solved, inner iterations; LP3 used,
 * LP3 lines re-solved, boundary lines built, boundary lines checked,
 * boundary lines re-solved, inner iterations.
 * lines_out (nullable, n x k x 4): each agent's half-planes (q, d), zero
 * past its neighbour count; pref_out (nullable, n x 2): desired velocity.
 * trace (nullable, n): hash of the agent's neighbour list and branch
 * outcomes. */
int oracle_step(int n, const float *px, const float *py, const float *vx, const float *vy,
                const float *pref_x, const float *pref_y, const float *radius,
                const float *max_speed, const uint8_t *cls, const oparams *prm, double *opx,
                double *opy, double *ovx, double *ovy, uint8_t *status, int32_t *nbr_out,
                int32_t *cnt_out, int64_t *work, double *lines_out, double *pref_out,
                uint64_t *trace)
{
    if (n < 0) return -1;
    if (n == 0) return params_ok(prm) ? 0 : -1;
    Widened W(n, px, py, vx, vy, pref_x, pref_y, radius, max_speed, cls);
    return step_impl(W.s, prm, opx, opy, ovx, ovy, status, nbr_out, cnt_out, work, lines_out,
                     pref_out, trace);
}

/* The same step from a double state (used by FP64 rollouts). */
int oracle_step_d(int n, const double *px, const double *py, const double *vx, const double *vy,
                  const double *pref_x, const double *pref_y, const double *radius,
                  const double *max_speed, const uint8_t *cls, const oparams *prm, double *opx,
                  double *opy, double *ovx, double *ovy, uint8_t *status, uint64_t *trace)
{
    DState S{n, px, py, vx, vy, pref_x, pref_y, radius, max_speed, cls};
    return step_impl(S, prm, opx, opy, ovx, ovy, status, nullptr, nullptr, nullptr, nullptr,
                     nullptr, trace);
}

/* Vector-Jacobian product of one step at a double state (see vjp_impl). */
int oracle_step_vjp_d(int n, const double *px, const double *py, const double *vx,
                      const double *vy, const double *pref_x, const double *pref_y,
                      const double *radius, const double *max_speed, const uint8_t *cls,
                      const oparams *prm, const double *gpx1, const double *gpy1,
                      const double *gvx1, const double *gvy1, double *gpx0, double *gpy0,
                      double *gvx0, double *gvy0, double *gprx, double *gpry, double *gtau)
{
    DState S{n, px, py, vx, vy, pref_x, pref_y, radius, max_speed, cls};
    return vjp_impl(S, prm, gpx1, gpy1, gvx1, gvy1, gpx0, gpy0, gvx0, gvy0, gprx, gpry, gtau);
}

/* Vector-Jacobian product of one step at an FP32 state. */
int oracle_step_vjp(int n, const float *px, const float *py, const float *vx, const float *vy,
                    const float *pref_x, const float *pref_y, const float *radius,
                    const float *max_speed, const uint8_t *cls, const oparams *prm,
                    const double *gpx1, const double *gpy1, const double *gvx1,
                    const double *gvy1, double *gpx0, double *gpy0, double *gvx0, double *gvy0,
                    double *gprx, double *gpry, double *gtau)
{
    if (n < 0) return -1;
    if (n == 0) return params_ok(prm) ? 0 : -1;
    Widened W(n, px, py, vx, vy, pref_x, pref_y, radius, max_speed, cls);
    return vjp_impl(W.s, prm, gpx1, gpy1, gvx1, gvy1, gpx0, gpy0, gvx0, gvy0, gprx, gpry, gtau);
}

/* Many independent scenes: scene s owns agents [off[s], off[s+1]) and uses
 * prm[s]; agents of different scenes never interact. */
int oracle_step_batched(int n_scenes, const int32_t *off, const float *px, const float *py,
                        const float *vx, const float *vy, const float *pref_x,
                        const float *pref_y, const float *radius, const float *max_speed,
                        const uint8_t *cls, const oparams *prm, double *opx, double *opy,
                        double *ovx, double *ovy, uint8_t *status, int64_t *work)
{
    if (n_scenes < 0) return -1;
    for (int s = 0; s < n_scenes; ++s) {
        const int a = off[s], n = off[s + 1] - off[s];
        if (n < 0) return -1;
        const int rc = oracle_step(n, px + a, py + a, vx + a, vy + a, pref_x + a, pref_y + a,
                                   radius + a, max_speed + a, cls + a, &prm[s], opx + a, opy + a,
                                   ovx + a, ovy + a, status ? status + a : nullptr, nullptr,
                                   nullptr, work ? work + (int64_t)a * ORACLE_NWORK : nullptr,
                                   nullptr, nullptr, nullptr);
        if (rc != 0) return rc;
    }
    return 0;
}

} /* extern "C" */
