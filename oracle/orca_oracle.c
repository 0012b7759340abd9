/*
 * FP64 CPU oracle for one ORCA step of pedestrians and vehicles
 * ("Simulating Crowds and Autonomous Vehicles", Charlton et al.).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * library path never calls it and shares no code with it.
 *
 * Every quantity is computed in IEEE double from the FP32 caller state
 * (upcast exactly).  Build with -ffp-contract=off so that the neighbour key
 * below is evaluated exactly as written.
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
 *
 * Readings where the paper is silent (overlap rule, tie rules, parallel
 * tolerance, f = 0 kept as a constraint, LP3 tie rule) are listed at the
 * functions that use them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_K_MAX 64
#define ORACLE_NWORK 12

typedef struct {
    double qx, qy; /* point on the boundary line */
    double dx, dy; /* unit direction; permitted side is to its left */
} oline;

typedef struct {
    double dt, tau, rn;
    int32_t k;
    int32_t pref_is_goal;
    double f[2][2];
    double eps;
} oparams;

static double det2(double ax, double ay, double bx, double by) { return ax * by - ay * bx; }

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
/* ------------------------------------------------------------------------ */
int oracle_halfplane(double pax, double pay, double vax, double vay, double ra,
                     double pbx, double pby, double vbx, double vby, double rb,
                     double f, double tau, double dt, int a_before_b,
                     double *out /* qx,qy,dx,dy,ux,uy,nx,ny */)
{
    const double Px = pbx - pax, Py = pby - pay;
    const double Vx = vax - vbx, Vy = vay - vby;
    const double R = ra + rb;
    const double dist2 = Px * Px + Py * Py;
    const double R2 = R * R;
    double ux, uy, nx, ny;
    int branch;
    if (dist2 > R2) {
        const double wx = Vx - Px / tau, wy = Vy - Py / tau;
        const double w2 = wx * wx + wy * wy;
        const double wp = wx * Px + wy * Py;
        if (wp < 0.0 && wp * wp > R2 * w2) {
            const double wl = sqrt(w2);
            nx = wx / wl;
            ny = wy / wl;
            const double ul = R / tau - wl;
            ux = ul * nx;
            uy = ul * ny;
            branch = 0;
        } else {
            const double leg = sqrt(dist2 - R2);
            double ex, ey;
            if (det2(Px, Py, wx, wy) > 0.0) {
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
            const double s = Vx * ex + Vy * ey;
            ux = s * ex - Vx;
            uy = s * ey - Vy;
        }
    } else {
        const double wx = Vx - Px / dt, wy = Vy - Py / dt;
        const double wl = sqrt(wx * wx + wy * wy);
        if (wl > 0.0) {
            nx = wx / wl;
            ny = wy / wl;
        } else {
            nx = a_before_b ? 1.0 : -1.0;
            ny = 0.0;
        }
        const double ul = R / dt - wl;
        ux = ul * nx;
        uy = ul * ny;
        branch = 3;
    }
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
static int lp1(const oline *L, int i, double vmax, double ox, double oy, int mode,
               double tx, double ty, double eps, double *vx, double *vy, int64_t *iters)
{
    const oline *li = &L[i];
    const double dot = li->qx * li->dx + li->qy * li->dy;
    const double disc = dot * dot + vmax * vmax - (li->qx * li->qx + li->qy * li->qy);
    if (disc < 0.0) return 0;
    const double sq = sqrt(disc);
    double tl = -dot - sq, tr = -dot + sq;
    for (int j = 0; j < i; ++j) {
        ++*iters;
        const oline *lj = &L[j];
        const double a = det2(lj->dx, lj->dy, li->dx, li->dy);
        const double b = det2(lj->dx, lj->dy, li->qx - lj->qx, li->qy - lj->qy);
        if (fabs(a) <= eps) {
            if (b < 0.0) return 0;
            continue;
        }
        const double t = -b / a;
        if (a > 0.0) {
            if (t > tl) tl = t;
        } else {
            if (t < tr) tr = t;
        }
        if (tl > tr) return 0;
    }
    double t;
    if (mode == 0) {
        t = li->dx * (ox - li->qx) + li->dy * (oy - li->qy);
        if (t < tl) t = tl;
        if (t > tr) t = tr;
    } else {
        const double s = ox * li->dx + oy * li->dy;
        if (fabs(s) <= eps) {
            t = li->dx * (tx - li->qx) + li->dy * (ty - li->qy);
            if (t < tl) t = tl;
            if (t > tr) t = tr;
        } else {
            t = s > 0.0 ? tr : tl;
        }
    }
    *vx = li->qx + t * li->dx;
    *vy = li->qy + t * li->dy;
    return 1;
}

/* Incremental 2D LP over lines 0..m-1 and the disc |v| <= vmax.
 * mode 0: v* = argmin |v - o| (start at o, or at vmax*o/|o| outside the disc).
 * mode 1: maximise v . o for unit o (start at vmax*o).
 * Returns the index of the first line whose sub-problem is infeasible, or m;
 * on failure v keeps the value it had before that line. */
static int lp2_mode(const oline *L, int m, double vmax, double ox, double oy, int mode,
                    double tx, double ty, double eps, double *vx, double *vy,
                    int64_t *n_check, int64_t *n_viol, int64_t *iters)
{
    double x, y;
    if (mode == 1) {
        x = ox * vmax;
        y = oy * vmax;
    } else {
        const double o2 = ox * ox + oy * oy;
        if (o2 > vmax * vmax) {
            const double ol = sqrt(o2);
            x = ox / ol * vmax;
            y = oy / ol * vmax;
        } else {
            x = ox;
            y = oy;
        }
    }
    for (int i = 0; i < m; ++i) {
        ++*n_check;
        if (det2(L[i].dx, L[i].dy, L[i].qx - x, L[i].qy - y) > 0.0) {
            ++*n_viol;
            double nx2 = x, ny2 = y;
            if (!lp1(L, i, vmax, ox, oy, mode, tx, ty, eps, &nx2, &ny2, iters)) {
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
/* ------------------------------------------------------------------------ */
static void lp3(const oline *L, int m, int fail, double vmax, double tx, double ty,
                double eps, double *vx, double *vy, int64_t *w)
{
    oline proj[ORACLE_K_MAX];
    double level = 0.0;
    double x = *vx, y = *vy;
    for (int i = fail; i < m; ++i) {
        const oline *li = &L[i];
        if (det2(li->dx, li->dy, li->qx - x, li->qy - y) <= level) continue;
        ++w[0];
        int np = 0;
        for (int j = 0; j < i; ++j) {
            const oline *lj = &L[j];
            const double dij = det2(li->dx, li->dy, lj->dx, lj->dy);
            double ptx, pty;
            if (fabs(dij) <= eps) {
                if (li->dx * lj->dx + li->dy * lj->dy > 0.0) continue; /* same direction */
                ptx = 0.5 * (li->qx + lj->qx);
                pty = 0.5 * (li->qy + lj->qy);
            } else {
                const double t = det2(lj->dx, lj->dy, li->qx - lj->qx, li->qy - lj->qy) / dij;
                ptx = li->qx + t * li->dx;
                pty = li->qy + t * li->dy;
            }
            double ddx = lj->dx - li->dx, ddy = lj->dy - li->dy;
            const double dl = sqrt(ddx * ddx + ddy * ddy);
            proj[np].qx = ptx;
            proj[np].qy = pty;
            proj[np].dx = ddx / dl;
            proj[np].dy = ddy / dl;
            ++np;
        }
        w[1] += np;
        double nx = x, ny = y;
        /* objective direction: the inward normal of line i, (-d.y, d.x) */
        if (lp2_mode(proj, np, vmax, -li->dy, li->dx, 1, tx, ty, eps, &nx, &ny, &w[2], &w[3],
                     &w[4]) == np) {
            x = nx;
            y = ny;
        }
        level = det2(li->dx, li->dy, li->qx - x, li->qy - y);
    }
    *vx = x;
    *vy = y;
}

/* Public LP entry points for the pin tests (lines as m x 4: qx,qy,dx,dy). */
int oracle_lp2(int m, const double *lines, double vmax, double ox, double oy, double eps,
               double *v)
{
    if (m < 0 || m > ORACLE_K_MAX) return -1;
    oline L[ORACLE_K_MAX];
    for (int i = 0; i < m; ++i) {
        L[i].qx = lines[4 * i + 0];
        L[i].qy = lines[4 * i + 1];
        L[i].dx = lines[4 * i + 2];
        L[i].dy = lines[4 * i + 3];
    }
    int64_t a = 0, b = 0, c = 0;
    return lp2_mode(L, m, vmax, ox, oy, 0, 0.0, 0.0, eps, &v[0], &v[1], &a, &b, &c);
}

/* LP2 followed by LP3 when LP2 fails; returns the LP2 fail index (m = LP2
 * feasible, LP3 not run). */
int oracle_lp_full(int m, const double *lines, double vmax, double ox, double oy, double eps,
                   double *v)
{
    if (m < 0 || m > ORACLE_K_MAX) return -1;
    oline L[ORACLE_K_MAX];
    for (int i = 0; i < m; ++i) {
        L[i].qx = lines[4 * i + 0];
        L[i].qy = lines[4 * i + 1];
        L[i].dx = lines[4 * i + 2];
        L[i].dy = lines[4 * i + 3];
    }
    int64_t a = 0, b = 0, c = 0, w[5] = {0};
    const int fail = lp2_mode(L, m, vmax, ox, oy, 0, 0.0, 0.0, eps, &v[0], &v[1], &a, &b, &c);
    if (fail < m) lp3(L, m, fail, vmax, ox, oy, eps, &v[0], &v[1], w);
    return fail;
}

/* ------------------------------------------------------------------------ */
/* Neighbour search (Sec. 3: nearby agents; the neighbour cap k).           */
/* Definition: the k agents j != i with the smallest (key_ij, j) among      */
/* those with key_ij < R_n^2, in ascending (key, j) order, where            */
/*   dx = x_j - x_i, dy = y_j - y_i   (double, from the FP32 positions)     */
/*   key = dx*dx + dy*dy              (double, each operation rounded)      */
/*   R_n^2 = R_n * R_n                (double, from the FP32 R_n)           */
/* A uniform grid of cell size >= R_n only bounds which j are examined.     */
/* ------------------------------------------------------------------------ */
typedef struct {
    double key;
    int32_t j;
} cand;

static int cand_cmp(const void *a, const void *b)
{
    const cand *x = (const cand *)a, *y = (const cand *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->j > y->j) - (x->j < y->j);
}

typedef struct {
    double x0, y0, cs;
    int64_t nx, ny;
    int32_t *start; /* nx*ny + 1 */
    int32_t *order; /* agent indices sorted by (cell, index) */
} ogrid;

static int64_t cell_coord(double v, double v0, double cs, int64_t nmax)
{
    int64_t c = (int64_t)floor((v - v0) / cs);
    if (c < 0) c = 0;
    if (c >= nmax) c = nmax - 1;
    return c;
}

static int ogrid_build(ogrid *g, int n, const float *px, const float *py, double rn)
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
        g->nx = (int64_t)floor((x1 - x0) / cs) + 1;
        g->ny = (int64_t)floor((y1 - y0) / cs) + 1;
        if (g->nx * g->ny <= 4 * (int64_t)n + 1024) break;
        cs *= 2.0; /* a coarser grid still covers every in-range pair */
    }
    g->x0 = x0;
    g->y0 = y0;
    g->cs = cs;
    const int64_t nc = g->nx * g->ny;
    g->start = (int32_t *)calloc((size_t)nc + 1, sizeof(int32_t));
    g->order = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int64_t *cell = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int32_t *fill = (int32_t *)malloc((size_t)(nc + 1) * sizeof(int32_t));
    if (!g->start || !g->order || !cell || !fill) {
        free(cell);
        free(fill);
        return -1;
    }
    for (int i = 0; i < n; ++i) {
        cell[i] = cell_coord(px[i], x0, cs, g->nx) + g->nx * cell_coord(py[i], y0, cs, g->ny);
        g->start[cell[i] + 1]++;
    }
    for (int64_t c = 0; c < nc; ++c) g->start[c + 1] += g->start[c];
    memcpy(fill, g->start, (size_t)(nc + 1) * sizeof(int32_t));
    for (int i = 0; i < n; ++i) g->order[fill[cell[i]]++] = i; /* stable: (cell, index) */
    free(cell);
    free(fill);
    return 0;
}

static void ogrid_free(ogrid *g)
{
    free(g->start);
    free(g->order);
}

/* Exact k nearest of agent i; returns the number kept, writes the in-range
 * count and the number of candidates examined. */
static int knn_one(const ogrid *g, int i, const float *px, const float *py, double rn2, int k,
                   cand **buf, int *cap, int32_t *nbr, int64_t *n_inrange, int64_t *n_cand)
{
    const double xi = px[i], yi = py[i];
    const int64_t cx = cell_coord(xi, g->x0, g->cs, g->nx);
    const int64_t cy = cell_coord(yi, g->y0, g->cs, g->ny);
    int cnt = 0;
    for (int64_t yy = cy - 1; yy <= cy + 1; ++yy) {
        if (yy < 0 || yy >= g->ny) continue;
        for (int64_t xx = cx - 1; xx <= cx + 1; ++xx) {
            if (xx < 0 || xx >= g->nx) continue;
            const int64_t c = xx + g->nx * yy;
            for (int32_t s = g->start[c]; s < g->start[c + 1]; ++s) {
                const int32_t j = g->order[s];
                ++*n_cand;
                if (j == i) continue;
                const double dx = (double)px[j] - xi;
                const double dy = (double)py[j] - yi;
                const double key = dx * dx + dy * dy;
                if (!(key < rn2)) continue;
                if (cnt == *cap) {
                    *cap = *cap ? 2 * *cap : 256;
                    *buf = (cand *)realloc(*buf, (size_t)*cap * sizeof(cand));
                }
                (*buf)[cnt].key = key;
                (*buf)[cnt].j = j;
                ++cnt;
            }
        }
    }
    *n_inrange = cnt;
    qsort(*buf, (size_t)cnt, sizeof(cand), cand_cmp);
    const int m = cnt < k ? cnt : k;
    for (int s = 0; s < m; ++s) nbr[s] = (*buf)[s].j;
    for (int s = m; s < k; ++s) nbr[s] = -1;
    return m;
}

/* nbr: n x k (row-major, -1 padded), cnt: n.  Returns 0, or -1 on bad args. */
int oracle_knn(int n, const float *px, const float *py, float neighbor_dist, int k,
               int32_t *nbr, int32_t *cnt)
{
    if (n < 0 || k < 1 || k > ORACLE_K_MAX || !(neighbor_dist > 0.0f)) return -1;
    if (n == 0) return 0;
    ogrid g;
    if (ogrid_build(&g, n, px, py, (double)neighbor_dist) != 0) return -2;
    const double rn = (double)neighbor_dist;
    const double rn2 = rn * rn;
#pragma omp parallel
    {
        cand *buf = NULL;
        int cap = 0;
#pragma omp for schedule(static)
        for (int i = 0; i < n; ++i) {
            int64_t a = 0, b = 0;
            cnt[i] = knn_one(&g, i, px, py, rn2, k, &buf, &cap, nbr + (int64_t)i * k, &a, &b);
        }
        free(buf);
    }
    ogrid_free(&g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One synchronous step of every agent of one scene.                        */
/* Desired velocity (goal mode): (g - p) * min(v_max/|g - p|, 1/dt), zero   */
/* when p = g; otherwise pref holds v_pref itself.  The LP result v' is the */
/* new velocity and p' = p + v' dt (explicit Euler), all agents reading the */
/* step-t state.                                                            */
/* work (nullable, n x 12): candidates examined, in-range count, neighbours */
/* used; LP2 lines checked, lines re-solved, inner iterations; LP3 used,    */
/* LP3 lines re-solved, boundary lines built, boundary lines checked,       */
/* boundary lines re-solved, inner iterations.                              */
/* lines_out (nullable, n x k x 4): each agent's half-planes (q, d), zero   */
/* past its neighbour count; pref_out (nullable, n x 2): desired velocity.  */
/* ------------------------------------------------------------------------ */
int oracle_step(int n, const float *px, const float *py, const float *vx, const float *vy,
                const float *pref_x, const float *pref_y, const float *radius,
                const float *max_speed, const uint8_t *cls, const oparams *prm,
                double *opx, double *opy, double *ovx, double *ovy, uint8_t *status,
                int32_t *nbr_out, int32_t *cnt_out, int64_t *work, double *lines_out,
                double *pref_out)
{
    if (n < 0 || !prm || prm->k < 1 || prm->k > ORACLE_K_MAX) return -1;
    if (!(prm->dt > 0.0) || !(prm->tau > 0.0) || !(prm->rn > 0.0)) return -1;
    if (n == 0) return 0;
    ogrid g;
    if (ogrid_build(&g, n, px, py, prm->rn) != 0) return -2;
    const double rn2 = prm->rn * prm->rn;
    const int k = prm->k;
#pragma omp parallel
    {
        cand *buf = NULL;
        int cap = 0;
#pragma omp for schedule(static)
        for (int i = 0; i < n; ++i) {
            int32_t nb[ORACLE_K_MAX];
            oline L[ORACLE_K_MAX];
            int64_t w[ORACLE_NWORK] = {0};
            const int m = knn_one(&g, i, px, py, rn2, k, &buf, &cap, nb, &w[1], &w[0]);
            w[2] = m;
            const double pix = px[i], piy = py[i], vix = vx[i], viy = vy[i];
            const double vmax = max_speed[i];
            double prx, pry;
            if (prm->pref_is_goal) {
                const double gx = (double)pref_x[i] - pix, gy = (double)pref_y[i] - piy;
                const double d2 = gx * gx + gy * gy;
                if (d2 > 0.0) {
                    const double d = sqrt(d2);
                    double s = vmax / d;
                    if (1.0 / prm->dt < s) s = 1.0 / prm->dt;
                    prx = gx * s;
                    pry = gy * s;
                } else {
                    prx = 0.0;
                    pry = 0.0;
                }
            } else {
                prx = pref_x[i];
                pry = pref_y[i];
            }
            for (int s = 0; s < m; ++s) {
                const int j = nb[s];
                double hp[8];
                oracle_halfplane(pix, piy, vix, viy, radius[i], px[j], py[j], vx[j], vy[j],
                                 radius[j], prm->f[cls[i] & 1][cls[j] & 1], prm->tau, prm->dt,
                                 i < j, hp);
                L[s].qx = hp[0];
                L[s].qy = hp[1];
                L[s].dx = hp[2];
                L[s].dy = hp[3];
            }
            double nvx, nvy;
            const int fail = lp2_mode(L, m, vmax, prx, pry, 0, 0.0, 0.0, prm->eps, &nvx, &nvy,
                                      &w[3], &w[4], &w[5]);
            uint8_t st = 0;
            if (fail < m) {
                lp3(L, m, fail, vmax, prx, pry, prm->eps, &nvx, &nvy, &w[7]);
                st = 1;
                w[6] = 1;
            }
            ovx[i] = nvx;
            ovy[i] = nvy;
            opx[i] = pix + nvx * prm->dt;
            opy[i] = piy + nvy * prm->dt;
            if (status) status[i] = st;
            if (nbr_out) memcpy(nbr_out + (int64_t)i * k, nb, (size_t)k * sizeof(int32_t));
            if (cnt_out) cnt_out[i] = m;
            if (work) memcpy(work + (int64_t)i * ORACLE_NWORK, w, sizeof(w));
            if (lines_out) {
                double *lo = lines_out + (int64_t)i * k * 4;
                for (int s = 0; s < k; ++s) {
                    const int ok = s < m;
                    lo[4 * s + 0] = ok ? L[s].qx : 0.0;
                    lo[4 * s + 1] = ok ? L[s].qy : 0.0;
                    lo[4 * s + 2] = ok ? L[s].dx : 0.0;
                    lo[4 * s + 3] = ok ? L[s].dy : 0.0;
                }
            }
            if (pref_out) {
                pref_out[2 * i] = prx;
                pref_out[2 * i + 1] = pry;
            }
        }
        free(buf);
    }
    ogrid_free(&g);
    return 0;
}

/* Many independent scenes: scene s owns agents [off[s], off[s+1]) and uses
 * prm[s]; agents of different scenes never interact.  Neighbour indices in
 * nbr_out are global (caller order). */
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
                                   radius + a, max_speed + a, cls + a, &prm[s], opx + a,
                                   opy + a, ovx + a, ovy + a, status ? status + a : NULL, NULL,
                                   NULL, work ? work + (int64_t)a * ORACLE_NWORK : NULL, NULL,
                                   NULL);
        if (rc != 0) return rc;
    }
    return 0;
}
