/*
 * FP64 reference renderer for differentiable motion-blur rasterization with
 * the fast barycentric coordinate solver (arXiv 2602.07860, Sec. 3 and App. B).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the benchmark's CPU-baseline leg load this library.  It shares no code,
 * header, table or helper with the GPU path.
 *
 * What it computes, per pixel p = (u, v) and per sub-frame k (plain loops,
 * double precision, faces culled only by a conservative bounding-box test):
 *
 *   keyframes    project M_s P0 for s = 0..S (App. I, eqs A33-A34)
 *   schedule     t_k = k/(K-1) (Sec. 3.2), split into S linear segments
 *                (Sec. 3.3); local time tau inside segment s
 *   positions    v(tau) = (1-tau) v(0) + tau v(1) per segment (eq 5)
 *   barycentric  naive: w = adj(F) p / det F per sub-frame (eqs 3, 7, A8-A10)
 *                fast:  w = (A1 t^2 + A2 t + A3)/(a1 t^2 + a2 t + a3) with the
 *                       closed-form coefficients of App. B (eqs 8, A11-A16)
 *   foreground   z-buffer winner (closest covering face), I = sum_i w_i c_i
 *                (eq 9)
 *   background   A_j = exp(-d/delta) (eq 10), d from the keyframe closest
 *                point (eqs 13-14, App. B edge projections), alpha =
 *                1 - prod_j (1 - A_j) (eq 15)
 *   average      I = (1/K) sum_k (rgb_k, alpha_k)
 *   gradient     exact derivative of the above with every discrete decision
 *                held fixed (Sec. 3.3 "Gradient Computation"), hand adjoint
 *
 * Readings of the paper taken where it is silent or ambiguous are listed in
 * the repository's design notes; each is marked "reading:" below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TAU_DET 1e-10      /* reading: |det F(tau)| <= this => face skipped */
/* Guard band: decisions that a float32 evaluation of the same quantities can
 * take either way.  The widths are multiples of the float32 unit roundoff
 * applied to the magnitudes that enter each decision (see orc_bg_band). */
#define ORC_EPS32 5.9604644775390625e-8   /* 2^-24, float32 unit roundoff */
#define ORC_GUARD_W 2e-5       /* |min_i w_i| below this: coverage may flip */
#define ORC_GUARD_DEPTH 1e-6   /* relative depth near-tie */
#define ORC_GUARD_ULPS 8.0     /* guard widths: this many times the float32 error estimate */
#define ORC_COND_MIN 1e-4      /* terms whose float32 relative error may exceed this get a bound */
#define ORC_MAX_AMBIG 8
#define ORC_ADJ_WMIN 1e-8      /* weight bound of the live-pair counter */

enum { CNT_BBOX, CNT_COV, CNT_FG, CNT_BG, CNT_BGPAIRS, CNT_SETUP, CNT_FLAGGED, CNT_SKIP,
       CNT_ALT_VALUE, CNT_ALT_GRAD, CNT_UNBOUNDED, CNT_BGLIVE, ORC_NCNT };

typedef struct {
    int V, F, C, S, K, W, H;
    const double *verts;     /* [V][3] rest positions (world)            */
    const int *faces;        /* [F][3]                                   */
    const double *attrs;     /* [V][C] per-vertex attributes             */
    const double *model;     /* [S+1][3][4] transforms at t_s = s/S      */
    const double *model_sub; /* [K][3][4] transforms at t_k (exact mode) */
    const double *view;      /* [3][4] world -> camera                   */
    double tan_half_fov;
    double delta;            /* softness of eq 10                        */
    double eps_cutoff;       /* A := 0 where A < eps (d > delta ln 1/eps); <= 0: no cut */
    int solver;              /* 0 naive per-sub-frame solve, 1 fast coefficients */
    int motion;              /* 0 segment-linear keyframes, 1 exact projection per sub-frame */
    int distance;            /* 0 keyframe closest point (eq 13), 1 closest point in F(tau) (eq 12) */
    int stop_grad_sigma;     /* variant: no gradient through the closest-point weights */
    double adj_wmin;         /* > 0: the adjoint leaves out background terms of weight
                                prod_{m != j}(1 - A_m) A_j below this, and whole (pixel,
                                sub-frame)s whose bound prod / min(min (1 - A), 1/2) on the
                                weights is; 0: exact */
    int nthreads;
    int row_begin, row_end, row_step;
} orc_scene;

typedef struct { int pk, face, edge, clamp; } orc_bg_rec;

typedef struct {
    int W, H, K;
    int *winner;             /* [H][W][K]; -1 background                  */
    int **row_start;         /* per row [W*K+1] offsets into row_list      */
    orc_bg_rec **row_list;   /* per row: contributing background faces     */
    int *row_n;
} orc_decisions;

/* ------------------------------------------------------------ helpers -- */

/* Sub-frame k of K: global time t_k = k/(K-1) (Sec. 3.2).  Reading: it falls
 * in segment s = min(floor(t_k S), S-1) with local time tau = t_k S - s, and
 * X = 0 iff tau <= 1/2 (eq 13).  Integer arithmetic keeps X exact. */
static void orc_schedule(int k, int K, int S, int *s, double *tau, int *X)
{
    if (K <= 1) { *s = 0; *tau = 0.0; *X = 0; return; }
    long num = (long)k * S;
    long seg = num / (K - 1);
    if (seg > S - 1) seg = S - 1;
    long rem = num - seg * (long)(K - 1);
    *s = (int)seg;
    *tau = (double)rem / (double)(K - 1);
    *X = (2 * rem <= (long)(K - 1)) ? 0 : 1;
}

/* Perspective projection of App. I: x_p = x/(z tan a), y_p = y/(z tan a);
 * camera depth z kept for the z-buffer. */
static void orc_project(const double *view, const double *m, double tanf,
                        const double *p, double out[3])
{
    double w[3], c[3];
    for (int r = 0; r < 3; ++r)
        w[r] = m[r * 4 + 0] * p[0] + m[r * 4 + 1] * p[1] + m[r * 4 + 2] * p[2] + m[r * 4 + 3];
    for (int r = 0; r < 3; ++r)
        c[r] = view[r * 4 + 0] * w[0] + view[r * 4 + 1] * w[1] + view[r * 4 + 2] * w[2] + view[r * 4 + 3];
    out[0] = c[0] / (c[2] * tanf);
    out[1] = c[1] / (c[2] * tanf);
    out[2] = c[2];
}

/* Barycentric coordinates by the linear solve of eq 3, written with the
 * determinant (eq A8) and adjugate (eq A9) of F = [x; y; 1]. */
static double orc_solve_naive(const double P[3][3], double u, double v, double w[3])
{
    double x0 = P[0][0], x1 = P[1][0], x2 = P[2][0];
    double y0 = P[0][1], y1 = P[1][1], y2 = P[2][1];
    double D = x0 * (y1 - y2) - x1 * (y0 - y2) + x2 * (y0 - y1);
    double r0 = (y1 - y2) * u + (x2 - x1) * v + (x1 * y2 - x2 * y1);
    double r1 = (y2 - y0) * u + (x0 - x2) * v + (x2 * y0 - x0 * y2);
    double r2 = (y0 - y1) * u + (x1 - x0) * v + (x0 * y1 - x1 * y0);
    w[0] = r0 / D; w[1] = r1 / D; w[2] = r2 / D;
    return D;
}

/* Fast-solver coefficients, App. B eqs A11-A16 (x_i(0) = xa[i], x_i(1) = xb[i]). */
void orc_fast_coeffs(const double *xa, const double *ya, const double *xb, const double *yb,
                     double u, double v, double *A1, double *A2, double *A3, double *a)
{
    double x00 = xa[0], x10 = xa[1], x20 = xa[2], y00 = ya[0], y10 = ya[1], y20 = ya[2];
    double x01 = xb[0], x11 = xb[1], x21 = xb[2], y01 = yb[0], y11 = yb[1], y21 = yb[2];
    A1[0] = -(x20 - x21) * (y10 - y11) + (x10 - x11) * (y20 - y21);
    A1[1] = (x20 - x21) * (y00 - y01) - (x00 - x01) * (y20 - y21);
    A1[2] = -((x10 - x11) * (y00 - y01)) + (x00 - x01) * (y10 - y11);

    A2[0] = u * (-y10 + y20 + y11 - y21) + v * (x10 - x20 - x11 + x21)
          + (y20 * x11 - y10 * x21 + x20 * (2 * y10 - y11) + x10 * (-2 * y20 + y21));
    A2[1] = u * (y00 - y20 - y01 + y21) + v * (-x00 + x20 + x01 - x21)
          + (-(y20 * x01) + y00 * x21 + x20 * (-2 * y00 + y01) + x00 * (2 * y20 - y21));
    A2[2] = u * (-y00 + y10 + y01 - y11) + v * (x00 - x10 - x01 + x11)
          + (y10 * x01 - y00 * x11 + x10 * (2 * y00 - y01) + x00 * (-2 * y10 + y11));

    A3[0] = u * (y10 - y20) + v * (-x10 + x20) + (-(x20 * y10) + x10 * y20);
    A3[1] = u * (-y00 + y20) + v * (x00 - x20) + (x20 * y00 - x00 * y20);
    A3[2] = u * (y00 - y10) + v * (-x00 + x10) + (-(x10 * y00) + x00 * y10);

    a[0] = -(y10 * x01) + y20 * x01 - y20 * x11 + y00 * (x11 - x21) + y10 * x21 - x11 * y01
         + x21 * y01 + x01 * y11 - x21 * y11 + x20 * (y00 - y10 - y01 + y11)
         + x10 * (-y00 + y20 + y01 - y21) - x01 * y21 + x11 * y21
         + x00 * (y10 - y20 - y11 + y21);
    a[1] = y10 * x01 - y20 * x01 + y20 * x11 - y10 * x21 + y00 * (-x11 + x21)
         + x20 * (-2 * y00 + 2 * y10 + y01 - y11) + x00 * (-2 * y10 + 2 * y20 + y11 - y21)
         + x10 * (2 * y00 - 2 * y20 - y01 + y21);
    a[2] = x20 * (y00 - y10) + x00 * (y10 - y20) + x10 * (-y00 + y20);
}

/* Fast solver (eq 8): evaluates the quadratic ratio at local time tau. */
static double orc_solve_fast(const double K0[3][3], const double K1[3][3], double tau,
                             double u, double v, double w[3])
{
    double xa[3], ya[3], xb[3], yb[3], A1[3], A2[3], A3[3], a[3];
    for (int i = 0; i < 3; ++i) { xa[i] = K0[i][0]; ya[i] = K0[i][1]; xb[i] = K1[i][0]; yb[i] = K1[i][1]; }
    orc_fast_coeffs(xa, ya, xb, yb, u, v, A1, A2, A3, a);
    double D = a[0] * tau * tau + a[1] * tau + a[2];
    for (int i = 0; i < 3; ++i) w[i] = (A1[i] * tau * tau + A2[i] * tau + A3[i]) / D;
    return D;
}

/* Closest point on a triangle (App. B, "Euclidean Distance Approximation"):
 * project q on the edges (0,1), (1,2), (2,0), clamp the edge parameter to
 * [0,1], keep the edge whose point is nearest (first one on exact ties).
 * Also reports the runner-up: the nearest other edge whose closest point
 * differs from the chosen one (for the parity guard band). */
typedef struct {
    int edge, clamp;       /* chosen edge; clamp state 0 (sigma < 0), 1 (inside), 2 (sigma > 1) */
    double sigma, sigma_raw, dist;
    int edge2, clamp2;     /* runner-up edge with a different closest point, -1 if none */
    double sigma2, dist2;
} orc_cp;

static void orc_closest_edge(const double T[3][2], double qx, double qy, orc_cp *cp)
{
    double t[3], tr[3], px[3], py[3], dist[3];
    int cl[3];
    for (int e = 0; e < 3; ++e) {
        int a = e, b = (e + 1) % 3;
        double ex = T[b][0] - T[a][0], ey = T[b][1] - T[a][1];
        double ee = ex * ex + ey * ey;
        tr[e] = ee > 0 ? ((qx - T[a][0]) * ex + (qy - T[a][1]) * ey) / ee : 0.0;
        t[e] = tr[e];
        cl[e] = 1;
        if (t[e] < 0) { t[e] = 0; cl[e] = 0; } else if (t[e] > 1) { t[e] = 1; cl[e] = 2; }
        if (ee <= 0) cl[e] = 0;
        px[e] = T[a][0] + t[e] * ex;
        py[e] = T[a][1] + t[e] * ey;
        dist[e] = (qx - px[e]) * (qx - px[e]) + (qy - py[e]) * (qy - py[e]);
    }
    int b = 0;
    for (int e = 1; e < 3; ++e) if (dist[e] < dist[b]) b = e;
    int r = -1;
    for (int e = 0; e < 3; ++e) {
        if (e == b || fabs(px[e] - px[b]) + fabs(py[e] - py[b]) <= 1e-12) continue;
        if (r < 0 || dist[e] < dist[r]) r = e;
    }
    cp->edge = b; cp->clamp = cl[b]; cp->sigma = t[b]; cp->sigma_raw = tr[b]; cp->dist = dist[b];
    cp->edge2 = r;
    cp->clamp2 = r >= 0 ? cl[r] : 0;
    cp->sigma2 = r >= 0 ? t[r] : 0.0;
    cp->dist2 = r >= 0 ? dist[r] : INFINITY;
}

void orc_closest_point(const double *tri /*[3][2]*/, double qx, double qy, double *wstar /*[3]*/)
{
    double T[3][2];
    orc_cp cp;
    for (int i = 0; i < 3; ++i) { T[i][0] = tri[2 * i]; T[i][1] = tri[2 * i + 1]; }
    orc_closest_edge(T, qx, qy, &cp);
    wstar[0] = wstar[1] = wstar[2] = 0.0;
    wstar[cp.edge] = 1.0 - cp.sigma;
    wstar[(cp.edge + 1) % 3] += cp.sigma;
}

/* --------------------------------------------------------- render core -- */

typedef struct {
    const orc_scene *sc;
    double *KF;        /* [S+1][V][3] keyframe screen positions            */
    double *SUB;       /* [K][V][3] exact positions (motion = exact)        */
    double halo;       /* sqrt(d_max), or +inf without cutoff               */
    double dmax;
    int *seg_k0, *seg_n;   /* sub-frames of each segment                    */
    double *swept;     /* [S][F][4] expanded bbox over the segment          */
} orc_ctx;

typedef struct {
    int f;
    double P[3][3];    /* x, y, z of the three vertices at the sub-frame    */
    double w[3], D, depth, mw;
    int skip, cover;
} orc_eval;

typedef struct {      /* one background face's forward quantities          */
    int f, j;          /* face; its index among the sub-frame's candidates  */
    int edge, clamp;
    double A, om, d, sigma, sigma_raw;
    double w[3];
    int nalt;          /* guard band: other (edge, clamp) decisions a float32 */
    int alt_edge[2], alt_clamp[2];   /* evaluation can take                  */
} orc_bgterm;

static void orc_face_pos(const orc_ctx *cx, int f, int k, int s, double tau, double P[3][3])
{
    const orc_scene *sc = cx->sc;
    for (int i = 0; i < 3; ++i) {
        int vi = sc->faces[f * 3 + i];
        if (sc->motion == 1) {
            const double *q = cx->SUB + ((size_t)k * sc->V + vi) * 3;
            P[i][0] = q[0]; P[i][1] = q[1]; P[i][2] = q[2];
        } else {
            const double *a = cx->KF + ((size_t)s * sc->V + vi) * 3;
            const double *b = cx->KF + ((size_t)(s + 1) * sc->V + vi) * 3;
            for (int c = 0; c < 3; ++c) P[i][c] = (1.0 - tau) * a[c] + tau * b[c];
        }
    }
}

static void orc_face_key(const orc_ctx *cx, int f, int s, double K[3][3])
{
    const orc_scene *sc = cx->sc;
    for (int i = 0; i < 3; ++i) {
        const double *a = cx->KF + ((size_t)s * sc->V + sc->faces[f * 3 + i]) * 3;
        K[i][0] = a[0]; K[i][1] = a[1]; K[i][2] = a[2];
    }
}

/* Barycentrics, depth and coverage of one face at one (pixel, sub-frame).
 * min w and depth are kept for skipped faces too (the guard band asks what
 * the face would do if a float32 evaluation did not skip it). */
static void orc_eval_face(const orc_ctx *cx, orc_eval *ev, int s, double tau, double u, double v)
{
    const orc_scene *sc = cx->sc;
    if (sc->solver == 1 && sc->motion == 0) {
        double K0[3][3], K1[3][3];
        orc_face_key(cx, ev->f, s, K0);
        orc_face_key(cx, ev->f, s + 1, K1);
        ev->D = orc_solve_fast(K0, K1, tau, u, v, ev->w);
    } else {
        ev->D = orc_solve_naive(ev->P, u, v, ev->w);
    }
    ev->skip = !(fabs(ev->D) > ORC_TAU_DET);
    ev->mw = fmin(ev->w[0], fmin(ev->w[1], ev->w[2]));
    ev->depth = ev->w[0] * ev->P[0][2] + ev->w[1] * ev->P[1][2] + ev->w[2] * ev->P[2][2];
    if (!isfinite(ev->mw)) ev->mw = -INFINITY;
    if (!isfinite(ev->depth)) ev->depth = INFINITY;
    ev->cover = !ev->skip && ev->mw >= 0.0;          /* reading: inclusive */
}

/* Float32 error model of the barycentrics w_i = N_i / det F, evaluated from
 * rounded coordinates:
 *  - each numerator N_i (a cross product of a pixel-to-vertex vector and an
 *    edge) carries an absolute error of about eps32 r e, with r the largest
 *    pixel-to-vertex distance and e the longest edge, so each w_i an
 *    independent absolute error of about eps32 r e / |det F| (orc_w_err);
 *  - det F carries a relative error of about eps32 (sum of squared edges) /
 *    |det F| (orc_det_rel), common to all three w_i. */
static double orc_w_err(const orc_eval *ev, double u, double v)
{
    double r = 0, e = 0;
    for (int i = 0; i < 3; ++i) {
        int j = (i + 1) % 3;
        double dx = ev->P[j][0] - ev->P[i][0], dy = ev->P[j][1] - ev->P[i][1];
        e = fmax(e, sqrt(dx * dx + dy * dy));
        r = fmax(r, sqrt((ev->P[i][0] - u) * (ev->P[i][0] - u) + (ev->P[i][1] - v) * (ev->P[i][1] - v)));
    }
    return fabs(ev->D) > 0 ? ORC_EPS32 * r * e / fabs(ev->D) : INFINITY;
}

static double orc_det_rel(const orc_eval *ev)
{
    double ee = 0;
    for (int i = 0; i < 3; ++i) {
        int j = (i + 1) % 3;
        double dx = ev->P[j][0] - ev->P[i][0], dy = ev->P[j][1] - ev->P[i][1];
        ee += dx * dx + dy * dy;
    }
    return fabs(ev->D) > 0 ? ORC_EPS32 * ee / fabs(ev->D) : INFINITY;
}

/* Half-width of the coverage guard band on min_i w_i. */
static double orc_w_band(const orc_eval *ev, double u, double v)
{
    return fmax(ORC_GUARD_W, ORC_GUARD_ULPS * orc_w_err(ev, u, v));
}

static double orc_hyp(double x, double y) { return sqrt(x * x + y * y); }

/* Background term of one face (eqs 10, 13, 14).  Returns 1 if it contributes.
 * Without a forced decision it also lists the closest-point decisions a
 * float32 evaluation could take instead: the clamp state when the edge
 * parameter is within rounding distance of 0 or 1, and the runner-up edge
 * when its (different) closest point is within rounding distance as near.
 * Rounding distance: ORC_GUARD_ULPS times the float32 error of q = F(X) w
 * (pixel and keyframe coordinates, the motion term, the error of w times
 * the vertices' motion) and of the edge projection. */
static int orc_bg_face(const orc_ctx *cx, const orc_eval *ev, int s, int X, double u, double v,
                       int forced_edge, int forced_clamp, orc_bgterm *bt)
{
    const orc_scene *sc = cx->sc;
    double T[3][2], qx, qy;
    if (sc->distance == 1) {           /* eq 12: closest point in F(tau) itself */
        for (int i = 0; i < 3; ++i) { T[i][0] = ev->P[i][0]; T[i][1] = ev->P[i][1]; }
        qx = u; qy = v;
    } else {                           /* eq 13: in keyframe F(X) */
        double KX[3][3];
        orc_face_key(cx, ev->f, s + X, KX);
        qx = qy = 0;
        for (int i = 0; i < 3; ++i) {
            T[i][0] = KX[i][0]; T[i][1] = KX[i][1];
            qx += ev->w[i] * KX[i][0];
            qy += ev->w[i] * KX[i][1];
        }
    }
    orc_cp cp;
    orc_closest_edge(T, qx, qy, &cp);
    int e = cp.edge, cl = cp.clamp;
    double sg = cp.sigma, sr = cp.sigma_raw;
    bt->nalt = 0;
    if (forced_edge >= 0) {            /* frozen-decision replay */
        int a = forced_edge, b = (forced_edge + 1) % 3;
        double ex = T[b][0] - T[a][0], ey = T[b][1] - T[a][1], ee = ex * ex + ey * ey;
        sr = ee > 0 ? ((qx - T[a][0]) * ex + (qy - T[a][1]) * ey) / ee : 0.0;
        e = forced_edge; cl = forced_clamp;
        sg = cl == 0 ? 0.0 : (cl == 2 ? 1.0 : sr);
    } else {
        /* float32 error of q = p + m, m = sum_i w_i (v_i(X) - v_i(tau)):
         * rounding of the pixel and keyframe coordinates and of m, and the
         * independent errors of the w_i times the vertices' motion (dq);
         * the relative error of det F, common to the w_i, scales m (rho) */
        double mx = 0, my = 0, wdv = 0;
        for (int i = 0; i < 3; ++i) {
            double dx = T[i][0] - ev->P[i][0], dy = T[i][1] - ev->P[i][1];
            mx += ev->w[i] * dx; my += ev->w[i] * dy;
            wdv += orc_hyp(dx, dy);
        }
        double mm = orc_hyp(mx, my), rho = orc_det_rel(ev);
        double dq = ORC_EPS32 * (orc_hyp(u - T[0][0], v - T[0][1]) + mm) + orc_w_err(ev, u, v) * wdv;
        int a = e, b = (e + 1) % 3;
        double len = orc_hyp(T[b][0] - T[a][0], T[b][1] - T[a][1]);
        double ra = orc_hyp(qx - T[a][0], qy - T[a][1]);
        if (len > 0) {
            /* det F's common relative error scales the motion term m, so it
             * moves the edge parameter by rho |m . e| / |e|^2 */
            double me = fabs(mx * (T[b][0] - T[a][0]) + my * (T[b][1] - T[a][1])) / (len * len);
            double band = ORC_GUARD_ULPS * ((dq + ORC_EPS32 * (ra + len)) / len + rho * me);
            if (fabs(sr) < band || fabs(sr - 1.0) < band) {
                bt->alt_edge[bt->nalt] = e;
                bt->alt_clamp[bt->nalt++] = cl != 1 ? 1 : (fabs(sr) < band ? 0 : 2);
            }
        }
        if (cp.edge2 >= 0) {
            int a2 = cp.edge2, b2 = (cp.edge2 + 1) % 3;
            double len2 = orc_hyp(T[b2][0] - T[a2][0], T[b2][1] - T[a2][1]);
            double ra2 = orc_hyp(qx - T[a2][0], qy - T[a2][1]);
            double tol = ORC_GUARD_ULPS * (dq + rho * mm + ORC_EPS32 * (ra + len + ra2 + len2));
            if (sqrt(cp.dist2) - sqrt(cp.dist) < tol) {
                bt->alt_edge[bt->nalt] = cp.edge2;
                bt->alt_clamp[bt->nalt++] = cp.clamp2;
            }
        }
    }
    int a = e, b = (e + 1) % 3;
    /* eq 14 (reading): p* = F(tau) w*, distance measured at the sub-frame */
    double px = (1.0 - sg) * ev->P[a][0] + sg * ev->P[b][0];
    double py = (1.0 - sg) * ev->P[a][1] + sg * ev->P[b][1];
    double d = (u - px) * (u - px) + (v - py) * (v - py);
    bt->f = ev->f; bt->edge = e; bt->clamp = cl; bt->sigma = sg; bt->sigma_raw = sr; bt->d = d;
    for (int i = 0; i < 3; ++i) bt->w[i] = ev->w[i];
    bt->A = exp(-d / sc->delta);
    bt->om = -expm1(-d / sc->delta);
    if (forced_edge < 0 && sc->eps_cutoff > 0 && d > cx->dmax) return 0;
    return 1;
}

/* Gradient buffers of one thread: dense accumulators, or (journal mode) a
 * list of (index, value) additions of one (pixel, sub-frame), used to
 * compare the gradient contributions of alternative decisions.  Index
 * space: keyframe gradient [S+1][V][2], then attributes [V][C]. */
typedef struct {
    double *gkf;
    double *gattr;
    int journal;
    size_t *ji; double *jv; int jn, jcap;
} orc_grad;

static void orc_gput(const orc_ctx *cx, orc_grad *g, size_t idx, double val)
{
    if (g->journal) {
        if (g->jn == g->jcap) {
            g->jcap = g->jcap ? 2 * g->jcap : 256;
            g->ji = (size_t *)realloc(g->ji, sizeof(size_t) * g->jcap);
            g->jv = (double *)realloc(g->jv, sizeof(double) * g->jcap);
        }
        g->ji[g->jn] = idx;
        g->jv[g->jn++] = val;
        return;
    }
    size_t nkf = (size_t)(cx->sc->S + 1) * cx->sc->V * 2;
    if (idx < nkf) g->gkf[idx] += val;
    else g->gattr[idx - nkf] += val;
}

static void orc_add_kf(const orc_ctx *cx, orc_grad *g, int f, int i, int s, double gx, double gy)
{
    int V = cx->sc->V;
    size_t p = ((size_t)s * V + cx->sc->faces[f * 3 + i]) * 2;
    orc_gput(cx, g, p, gx);
    orc_gput(cx, g, p + 1, gy);
}

static void orc_add_attr(const orc_ctx *cx, orc_grad *g, int vi, int c, double val)
{
    const orc_scene *sc = cx->sc;
    orc_gput(cx, g, (size_t)(sc->S + 1) * sc->V * 2 + (size_t)vi * sc->C + c, val);
}

/* d(w . gw)/d(vertex positions at tau): dw = -F^-1 dF w (static solve),
 * distributed to the segment's keyframes with weights (1-tau), tau (eq 5). */
static void orc_adj_bary(const orc_ctx *cx, orc_grad *g, const orc_eval *ev, const double w[3],
                         const double gw[3], int s, double tau)
{
    const double (*P)[3] = ev->P;
    double D = ev->D;
    double gxs = 0, gys = 0;
    for (int i = 0; i < 3; ++i) {
        int j = (i + 1) % 3, k = (i + 2) % 3;
        gxs += gw[i] * (P[j][1] - P[k][1]) / D;
        gys += gw[i] * (P[k][0] - P[j][0]) / D;
    }
    for (int i = 0; i < 3; ++i) {
        double gx = -w[i] * gxs, gy = -w[i] * gys;
        orc_add_kf(cx, g, ev->f, i, s, (1.0 - tau) * gx, (1.0 - tau) * gy);
        orc_add_kf(cx, g, ev->f, i, s + 1, tau * gx, tau * gy);
    }
}

/* Adjoint of one background term given dL/dd. */
static void orc_adj_bg(const orc_ctx *cx, orc_grad *g, const orc_eval *ev, const orc_bgterm *bt,
                       int s, double tau, int X, double u, double v, double gd)
{
    const orc_scene *sc = cx->sc;
    int a = bt->edge, b = (bt->edge + 1) % 3;
    double sg = bt->sigma;
    double px = (1.0 - sg) * ev->P[a][0] + sg * ev->P[b][0];
    double py = (1.0 - sg) * ev->P[a][1] + sg * ev->P[b][1];
    double gpx = 2.0 * gd * (px - u), gpy = 2.0 * gd * (py - v);
    /* p* = (1-sigma) v_a(tau) + sigma v_b(tau) */
    orc_add_kf(cx, g, ev->f, a, s, (1 - tau) * (1 - sg) * gpx, (1 - tau) * (1 - sg) * gpy);
    orc_add_kf(cx, g, ev->f, a, s + 1, tau * (1 - sg) * gpx, tau * (1 - sg) * gpy);
    orc_add_kf(cx, g, ev->f, b, s, (1 - tau) * sg * gpx, (1 - tau) * sg * gpy);
    orc_add_kf(cx, g, ev->f, b, s + 1, tau * sg * gpx, tau * sg * gpy);
    if (bt->clamp != 1 || sc->stop_grad_sigma) return;
    double gsig = gpx * (ev->P[b][0] - ev->P[a][0]) + gpy * (ev->P[b][1] - ev->P[a][1]);
    double KX[3][3];
    orc_face_key(cx, ev->f, s + X, KX);
    double qx = 0, qy = 0;
    for (int i = 0; i < 3; ++i) { qx += bt->w[i] * KX[i][0]; qy += bt->w[i] * KX[i][1]; }
    double ex = KX[b][0] - KX[a][0], ey = KX[b][1] - KX[a][1], ee = ex * ex + ey * ey;
    double rx = qx - KX[a][0], ry = qy - KX[a][1];
    double sr = bt->sigma_raw;
    /* sigma = (r . e)/(e . e) */
    double grx = gsig * ex / ee, gry = gsig * ey / ee;
    double gex = gsig * (rx - 2.0 * sr * ex) / ee, gey = gsig * (ry - 2.0 * sr * ey) / ee;
    orc_add_kf(cx, g, ev->f, a, s + X, -grx - gex, -gry - gey);
    orc_add_kf(cx, g, ev->f, b, s + X, gex, gey);
    /* q = sum_i w_i v_i(X) */
    double gw[3];
    for (int i = 0; i < 3; ++i) {
        orc_add_kf(cx, g, ev->f, i, s + X, bt->w[i] * grx, bt->w[i] * gry);
        gw[i] = grx * KX[i][0] + gry * KX[i][1];
    }
    orc_adj_bary(cx, g, ev, bt->w, gw, s, tau);
}

/* colour of one face at the pixel: sum_i w_i c_i (eq 9) */
static void orc_shade(const orc_scene *sc, const orc_eval *ev, double *rgb)
{
    for (int c = 0; c < sc->C; ++c) {
        rgb[c] = 0;
        for (int i = 0; i < 3; ++i) rgb[c] += ev->w[i] * sc->attrs[(size_t)sc->faces[ev->f * 3 + i] * sc->C + c];
    }
}

/* z-buffer over the faces with incl[j] set: closest covering face, ties to
 * the lowest face index (reading) */
static int orc_zbuffer(const orc_eval *ev, int n, const int *incl)
{
    int best = -1;
    for (int j = 0; j < n; ++j) {
        if (!incl[j]) continue;
        if (best < 0 || ev[j].depth < ev[best].depth ||
            (ev[j].depth == ev[best].depth && ev[j].f < ev[best].f)) best = j;
    }
    return best;
}

typedef struct {
    orc_eval *ev;     /* candidates of the current (pixel, sub-frame)      */
    orc_bgterm *bt;   /* its contributing background terms                 */
    orc_bgterm *bta;  /* guard band: background term of every candidate    */
    orc_bgterm *bt2;  /* guard band: terms of an alternative face set      */
    int *bta_ok, *skp;
    int *incl;
    int *cand;        /* row-segment candidates                            */
    int *pcand;       /* pixel-segment candidates                          */
    char *seen;       /* per pcand: bbox hit somewhere in the segment      */
    double *pre, *suf;
    orc_grad grad;
    /* guard band, gradient side: nominal journal, per-index scratch,
     * running max over alternatives, and the accumulated bound */
    size_t *j0i; double *j0v; int j0n, j0cap;
    double *dtmp, *dmx, *slack;
    size_t *mxl; int mxn, mxcap;
    double cnt[ORC_NCNT];
    orc_bg_rec *rl; int rl_n, rl_cap;
} orc_tls;

static void orc_push_rec(orc_tls *t, orc_bg_rec r)
{
    if (t->rl_n == t->rl_cap) {
        t->rl_cap = t->rl_cap ? 2 * t->rl_cap : 1024;
        t->rl = (orc_bg_rec *)realloc(t->rl, sizeof(orc_bg_rec) * t->rl_cap);
    }
    t->rl[t->rl_n++] = r;
}

/* background alpha of the current (pixel, sub-frame) over every non-skipped
 * candidate; fills t->bt; returns number of contributing faces */
static int orc_background(const orc_ctx *cx, orc_tls *t, int n, int s, int X, double u, double v,
                          double *alpha)
{
    int m = 0;
    double prod = 1.0;
    for (int j = 0; j < n; ++j) {
        if (t->ev[j].skip) continue;
        if (orc_bg_face(cx, &t->ev[j], s, X, u, v, -1, 0, &t->bt[m])) {
            t->bt[m].j = j;
            prod *= t->bt[m].om;
            ++m;
        }
    }
    *alpha = 1.0 - prod;
    return m;
}

/* Adjoint of the winner's shading (eq 9) and its barycentrics. */
static void orc_adj_fg(const orc_ctx *cx, orc_grad *g, const orc_eval *ev, const double *gI, int s, double tau)
{
    const orc_scene *sc = cx->sc;
    double gw[3];
    for (int i = 0; i < 3; ++i) {
        int vi = sc->faces[ev->f * 3 + i];
        gw[i] = 0;
        for (int c = 0; c < sc->C; ++c) {
            gw[i] += gI[c] * sc->attrs[(size_t)vi * sc->C + c];
            orc_add_attr(cx, g, vi, c, ev->w[i] * gI[c]);
        }
    }
    orc_adj_bary(cx, g, ev, ev->w, gw, s, tau);
}

/* Bound on the derivative weights prod_{m != j}(1 - A_m) A_j of a
 * background (pixel, sub-frame): 0 with two or more zero factors, infinite
 * with one, else prod_m (1 - A_m) / min(min_m (1 - A_m), 1/2). */
static double orc_weight_bound(const orc_bgterm *bt, int m)
{
    double P = 1.0, lo = 0.5;
    int nz = 0;
    for (int q = 0; q < m; ++q) {
        if (bt[q].om > 0) { P *= bt[q].om; lo = fmin(lo, bt[q].om); }
        else ++nz;
    }
    return nz >= 2 ? 0.0 : (nz == 1 ? INFINITY : P / lo);
}

/* Adjoint of alpha = 1 - prod_j (1 - A_j) over the terms bt[0..m):
 * d alpha / d A_j = prod_{m != j} (1 - A_m) by prefix/suffix products. */
static void orc_adj_bgset(const orc_ctx *cx, orc_grad *g, orc_tls *t, const orc_bgterm *bt, int m,
                          const double *gI, int s, double tau, int X, double u, double v)
{
    const orc_scene *sc = cx->sc;
    if (sc->adj_wmin > 0 && orc_weight_bound(bt, m) < sc->adj_wmin) return;
    t->pre[0] = 1.0;
    for (int q = 0; q < m; ++q) t->pre[q + 1] = t->pre[q] * bt[q].om;
    t->suf[m] = 1.0;
    for (int q = m - 1; q >= 0; --q) t->suf[q] = t->suf[q + 1] * bt[q].om;
    for (int q = 0; q < m; ++q) {
        if (sc->adj_wmin > 0 && t->pre[q] * t->suf[q + 1] * bt[q].A < sc->adj_wmin) continue;
        double dA = gI[sc->C] * t->pre[q] * t->suf[q + 1];
        orc_adj_bg(cx, g, &t->ev[bt[q].j], &bt[q], s, tau, X, u, v, dA * (-bt[q].A / sc->delta));
    }
}

static void orc_journal_begin(orc_grad *g) { g->journal = 1; g->jn = 0; }

/* keep the current journal as the nominal one */
static void orc_journal_keep(orc_tls *t)
{
    orc_grad *g = &t->grad;
    if (t->j0cap < g->jn) {
        t->j0cap = g->jn;
        t->j0i = (size_t *)realloc(t->j0i, sizeof(size_t) * t->j0cap);
        t->j0v = (double *)realloc(t->j0v, sizeof(double) * t->j0cap);
    }
    memcpy(t->j0i, g->ji, sizeof(size_t) * g->jn);
    memcpy(t->j0v, g->jv, sizeof(double) * g->jn);
    t->j0n = g->jn;
    g->journal = 0;
}

/* alternative (current journal) minus nominal, per index: into the running
 * max (to_max) or added in magnitude to the bound directly */
static void orc_journal_diff(orc_tls *t, int to_max)
{
    orc_grad *g = &t->grad;
    g->journal = 0;
    for (int e = 0; e < t->j0n; ++e) t->dtmp[t->j0i[e]] -= t->j0v[e];
    for (int e = 0; e < g->jn; ++e) t->dtmp[g->ji[e]] += g->jv[e];
    for (int pass = 0; pass < 2; ++pass) {
        const size_t *ix = pass ? g->ji : t->j0i;
        int ne = pass ? g->jn : t->j0n;
        for (int e = 0; e < ne; ++e) {
            size_t i = ix[e];
            double d = fabs(t->dtmp[i]);
            t->dtmp[i] = 0.0;
            if (!to_max) { t->slack[i] += d; continue; }
            if (d > t->dmx[i]) {
                if (t->dmx[i] == 0.0) {
                    if (t->mxn == t->mxcap) {
                        t->mxcap = t->mxcap ? 2 * t->mxcap : 256;
                        t->mxl = (size_t *)realloc(t->mxl, sizeof(size_t) * t->mxcap);
                    }
                    t->mxl[t->mxn++] = i;
                }
                t->dmx[i] = d;
            }
        }
    }
}

/* the current journal's magnitudes, times scale, added to the bound */
static void orc_journal_addabs(orc_tls *t, double scale)
{
    orc_grad *g = &t->grad;
    g->journal = 0;
    for (int e = 0; e < g->jn; ++e) t->slack[g->ji[e]] += scale * fabs(g->jv[e]);
}

/* Ill-conditioned terms: the gradient of a face whose det F is small against
 * its edges (a sliver, nearly edge-on at the sub-frame) goes through 1/det F
 * and a float32 evaluation has a relative error of about orc_det_rel there;
 * each such nominal term adds ORC_GUARD_ULPS times that share of itself to
 * the bound.  Call right after the nominal adjoint (uses t->pre, t->suf). */
static void orc_cond_bound(const orc_ctx *cx, orc_tls *t, int winner, int m, const double *gI,
                           int s, double tau, int X, double u, double v)
{
    const orc_scene *sc = cx->sc;
    if (winner >= 0) {
        double rho = ORC_GUARD_ULPS * orc_det_rel(&t->ev[winner]);
        if (!(rho > ORC_COND_MIN)) return;
        orc_journal_begin(&t->grad);
        orc_adj_fg(cx, &t->grad, &t->ev[winner], gI, s, tau);
        orc_journal_addabs(t, rho);
        return;
    }
    for (int q = 0; q < m; ++q) {
        const orc_bgterm *bq = &t->bt[q];
        const orc_eval *ev = &t->ev[bq->j];
        double rho = ORC_GUARD_ULPS * orc_det_rel(ev);
        if (!(rho > ORC_COND_MIN)) continue;
        double gd = gI[sc->C] * t->pre[q] * t->suf[q + 1] * (-bq->A / sc->delta);
        orc_journal_begin(&t->grad);
        orc_adj_bg(cx, &t->grad, ev, bq, s, tau, X, u, v, gd);
        orc_journal_addabs(t, rho);
    }
}

static void orc_max_flush(orc_tls *t)
{
    for (int e = 0; e < t->mxn; ++e) { t->slack[t->mxl[e]] += t->dmx[t->mxl[e]]; t->dmx[t->mxl[e]] = 0.0; }
    t->mxn = 0;
}

/*
 * Parity guard band of one (pixel, sub-frame): the decisions that sit within
 * rounding distance of flipping, and what the sub-frame would give under each
 * other choice.
 *  - coverage and skipping: every in/out choice of the faces whose min w is
 *    inside orc_w_band, or whose |det F| is within its float32 error (at
 *    least half the threshold) of the skip threshold, with the depth
 *    near-tie of each resulting z-buffer;
 *  - closest point (background): the other clamp state or edge of each term
 *    (orc_bg_face).
 * vlo/vhi receive the per-channel range of the sub-frame value over the
 * alternatives (nominal included).  With gI, t->slack receives a bound on
 * how far the gradient contribution of this (pixel, sub-frame) can move per
 * index: the max over the coverage alternatives plus the sum over the
 * closest-point alternatives of the change they make.
 * Returns bit 0 if an alternative moves the value by more than thr, bit 1 if
 * any alternative exists.
 */
static int orc_alternatives(const orc_ctx *cx, orc_tls *t, int n, int m, int s, double tau, int X,
                            double u, double v, int winner, const double *val, double thr,
                            const double *gI, double *vlo, double *vhi)
{
    const orc_scene *sc = cx->sc;
    const int C = sc->C;
    int amb[ORC_MAX_AMBIG], kind[ORC_MAX_AMBIG], na = 0;
    for (int c = 0; c <= C; ++c) vlo[c] = vhi[c] = val[c];
    for (int j = 0; j < n; ++j) {
        const orc_eval *ev = &t->ev[j];
        int k;
        if (fabs(fabs(ev->D) - ORC_TAU_DET) <= fmax(0.5 * ORC_TAU_DET, ORC_GUARD_ULPS * orc_det_rel(ev) * fabs(ev->D))) k = 1;
        else if (!ev->skip && fabs(ev->mw) < orc_w_band(ev, u, v)) k = 2;
        else continue;
        if (na == ORC_MAX_AMBIG) {
            /* too many: only the trivial range of a sub-frame value */
            t->cnt[CNT_UNBOUNDED] += 1;
            for (int c = 0; c < C; ++c) {
                double lo = 0, hi = 0;
                for (int vi = 0; vi < sc->V; ++vi) {
                    lo = fmin(lo, sc->attrs[(size_t)vi * C + c]);
                    hi = fmax(hi, sc->attrs[(size_t)vi * C + c]);
                }
                vlo[c] = fmin(vlo[c], lo); vhi[c] = fmax(vhi[c], hi);
            }
            vlo[C] = 0.0; vhi[C] = 1.0;
            return 3;
        }
        amb[na] = j; kind[na++] = k;
    }
    int bits = 0, have_j0 = 0, bta_ready = 0;
    double alt[16];
    for (int mask = 0; mask < (1 << na); ++mask) {
        int same_skip = 1;
        for (int j = 0; j < n; ++j) { t->skp[j] = t->ev[j].skip; t->incl[j] = t->ev[j].cover; }
        for (int a = 0; a < na; ++a) {
            if (!((mask >> a) & 1)) continue;
            int j = amb[a];
            if (kind[a] == 1) {
                t->skp[j] = !t->ev[j].skip;
                t->incl[j] = !t->skp[j] && t->ev[j].mw >= 0.0;
                same_skip = 0;
            } else {
                t->incl[j] = !t->incl[j];
            }
        }
        int w = orc_zbuffer(t->ev, n, t->incl);
        for (int pass = 0; pass < 2; ++pass) {
            int cand = w;
            if (pass == 1) {    /* runner-up within a relative depth near-tie */
                if (w < 0) break;
                int r = -1;
                for (int j = 0; j < n; ++j)
                    if (t->incl[j] && j != w && (r < 0 || t->ev[j].depth < t->ev[r].depth)) r = j;
                if (r < 0) break;
                double dz = fabs(t->ev[r].depth - t->ev[w].depth);
                if (dz > ORC_GUARD_DEPTH * fabs(t->ev[w].depth)) break;
                cand = r;
            }
            if (cand == winner && (cand >= 0 || same_skip)) continue;
            int m2 = 0;
            if (cand >= 0) {
                orc_shade(sc, &t->ev[cand], alt);
                alt[C] = 1.0;
            } else {
                if (!bta_ready) {
                    for (int j = 0; j < n; ++j) {
                        t->bta_ok[j] = orc_bg_face(cx, &t->ev[j], s, X, u, v, -1, 0, &t->bta[j]);
                        t->bta[j].j = j;
                    }
                    bta_ready = 1;
                }
                double prod = 1.0;
                for (int j = 0; j < n; ++j)
                    if (!t->skp[j] && t->bta_ok[j]) { prod *= t->bta[j].om; t->bt2[m2++] = t->bta[j]; }
                for (int c = 0; c < C; ++c) alt[c] = 0.0;
                alt[C] = 1.0 - prod;
            }
            for (int c = 0; c <= C; ++c) {
                vlo[c] = fmin(vlo[c], alt[c]);
                vhi[c] = fmax(vhi[c], alt[c]);
                if (fabs(alt[c] - val[c]) > thr) bits |= 1;
            }
            bits |= 2;
            if (!gI) continue;
            if (!have_j0) {
                orc_journal_begin(&t->grad);
                if (winner >= 0) orc_adj_fg(cx, &t->grad, &t->ev[winner], gI, s, tau);
                else orc_adj_bgset(cx, &t->grad, t, t->bt, m, gI, s, tau, X, u, v);
                orc_journal_keep(t);
                have_j0 = 1;
            }
            orc_journal_begin(&t->grad);
            if (cand >= 0) orc_adj_fg(cx, &t->grad, &t->ev[cand], gI, s, tau);
            else orc_adj_bgset(cx, &t->grad, t, t->bt2, m2, gI, s, tau, X, u, v);
            orc_journal_diff(t, 1);
        }
    }
    if (gI) orc_max_flush(t);
    if (winner >= 0 || m == 0) return bits;
    /* closest-point decisions of the background terms: each changes the
     * routing of its own term's gradient only (its value is continuous) */
    int any = 0;
    for (int q = 0; q < m; ++q) any |= t->bt[q].nalt > 0;
    if (!any) return bits;
    bits |= 2;
    if (!gI) return bits;
    t->pre[0] = 1.0;
    for (int q = 0; q < m; ++q) t->pre[q + 1] = t->pre[q] * t->bt[q].om;
    t->suf[m] = 1.0;
    for (int q = m - 1; q >= 0; --q) t->suf[q] = t->suf[q + 1] * t->bt[q].om;
    for (int q = 0; q < m; ++q) {
        const orc_bgterm *bq = &t->bt[q];
        if (!bq->nalt) continue;
        const orc_eval *ev = &t->ev[bq->j];
        double gd = gI[C] * t->pre[q] * t->suf[q + 1] * (-bq->A / sc->delta);
        orc_journal_begin(&t->grad);
        orc_adj_bg(cx, &t->grad, ev, bq, s, tau, X, u, v, gd);
        orc_journal_keep(t);
        for (int a = 0; a < bq->nalt; ++a) {
            orc_bgterm alt_t;
            orc_bg_face(cx, ev, s, X, u, v, bq->alt_edge[a], bq->alt_clamp[a], &alt_t);
            alt_t.j = bq->j;
            orc_journal_begin(&t->grad);
            orc_adj_bg(cx, &t->grad, ev, &alt_t, s, tau, X, u, v, gd);
            orc_journal_diff(t, 0);
        }
    }
    return bits;
}

static int orc_threads(const orc_scene *sc)
{
#ifdef _OPENMP
    return sc->nthreads > 0 ? sc->nthreads : omp_get_max_threads();
#else
    (void)sc;
    return 1;
#endif
}

static int orc_build(orc_ctx *cx, const orc_scene *sc)
{
    memset(cx, 0, sizeof(*cx));
    cx->sc = sc;
    int V = sc->V, S = sc->S, K = sc->K, F = sc->F;
    cx->KF = (double *)malloc(sizeof(double) * (size_t)(S + 1) * V * 3);
    if (!cx->KF) return -1;
#pragma omp parallel for schedule(static) num_threads(orc_threads(sc))
    for (int s = 0; s <= S; ++s)
        for (int v = 0; v < V; ++v)
            orc_project(sc->view, sc->model + s * 12, sc->tan_half_fov, sc->verts + v * 3,
                        cx->KF + ((size_t)s * V + v) * 3);
    if (sc->motion == 1) {
        cx->SUB = (double *)malloc(sizeof(double) * (size_t)K * V * 3);
        if (!cx->SUB) return -1;
        for (int k = 0; k < K; ++k)
            for (int v = 0; v < V; ++v)
                orc_project(sc->view, sc->model_sub + k * 12, sc->tan_half_fov, sc->verts + v * 3,
                            cx->SUB + ((size_t)k * V + v) * 3);
    }
    if (sc->eps_cutoff > 0) {
        cx->dmax = sc->delta * log(1.0 / sc->eps_cutoff);
        cx->halo = sqrt(cx->dmax) * (1.0 + 1e-9) + 1e-12;
    } else {
        cx->dmax = INFINITY;
        cx->halo = INFINITY;
    }
    cx->seg_k0 = (int *)calloc(S, sizeof(int));
    cx->seg_n = (int *)calloc(S, sizeof(int));
    for (int k = K - 1; k >= 0; --k) {
        int s, X; double tau;
        orc_schedule(k, K, S, &s, &tau, &X);
        cx->seg_k0[s] = k;
        cx->seg_n[s]++;
    }
    cx->swept = (double *)malloc(sizeof(double) * (size_t)S * F * 4);
    if (!cx->swept) return -1;
#pragma omp parallel for collapse(2) schedule(static) num_threads(orc_threads(sc))
    for (int s = 0; s < S; ++s) {
        for (int f = 0; f < F; ++f) {
            double *b = cx->swept + ((size_t)s * F + f) * 4;
            b[0] = b[2] = INFINITY; b[1] = b[3] = -INFINITY;
            for (int k = cx->seg_k0[s]; k < cx->seg_k0[s] + cx->seg_n[s]; ++k) {
                int ss, X; double tau; double P[3][3];
                orc_schedule(k, K, S, &ss, &tau, &X);
                orc_face_pos(cx, f, k, ss, tau, P);
                for (int i = 0; i < 3; ++i) {
                    b[0] = fmin(b[0], P[i][0]); b[1] = fmax(b[1], P[i][0]);
                    b[2] = fmin(b[2], P[i][1]); b[3] = fmax(b[3], P[i][1]);
                }
            }
            b[0] -= cx->halo; b[1] += cx->halo; b[2] -= cx->halo; b[3] += cx->halo;
        }
    }
    return 0;
}

static void orc_free_ctx(orc_ctx *cx)
{
    free(cx->KF); free(cx->SUB); free(cx->seg_k0); free(cx->seg_n); free(cx->swept);
}

/*
 * Render (and optionally differentiate).  image [C+1][H][W] receives the
 * averaged (rgb, alpha) for every rendered row (others untouched).  flags
 * [H][W] (optional, zeroed by the caller) ORs per pixel over its sub-frames:
 * bit 0 when a decision within rounding distance of flipping could move the
 * value beyond a quarter of the parity tolerance, bit 1 when such a decision
 * exists at all (it may change which vertices receive gradient).
 * counters[ORC_NCNT] (optional): bbox pairs, covering pairs, fg
 * pixel-subframes, bg pixel-subframes, contributing bg pairs, distinct
 * (pixel, face, segment) setups, pixel-subframes with bit 0, skipped
 * degenerate pairs, pixel-subframes whose value has alternatives,
 * pixel-subframes with any alternative, pixel-subframes with too many
 * ambiguous faces to enumerate, contributing bg pairs of (pixel,
 * sub-frame)s whose derivative weight bound is at least ORC_ADJ_WMIN.
 * With grad_image: grad_kf [S+1][V][2] (optional), grad_verts [V][3] and
 * grad_attrs [V][C] are overwritten with dL/d(...) for L = sum grad_image*I.
 * bounds (optional): the range of the image over the alternative decisions
 * of the guard band, and (with grad_image) per-component bounds on how far
 * those decisions can move the gradient.
 * rec: record decisions; rep: replay recorded decisions (frozen surrogate).
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
typedef struct {
    double *image_lo, *image_hi;   /* [C+1][H][W], rendered rows            */
    double *slack_kf;              /* [S+1][V][2] (optional)                */
    double *slack_verts;           /* [V][3]                                */
    double *slack_attrs;           /* [V][C]                                */
} orc_bounds;

int orc_render(const orc_scene *sc, double *image, int *flags, double *counters,
               const double *grad_image, double *grad_kf, double *grad_verts, double *grad_attrs,
               orc_decisions *rec, const orc_decisions *rep, orc_bounds *bd)
{
    if (!sc || sc->V <= 0 || sc->F <= 0 || sc->C <= 0 || sc->C > 14 || sc->S <= 0 || sc->K <= 0 ||
        sc->W <= 0 || sc->H <= 0 || !(sc->delta > 0) || !image)
        return -1;
    if (sc->motion == 1 && !sc->model_sub) return -1;
    if (grad_image && (sc->motion != 0 || sc->distance != 0)) return -1;
    if (rep && (rep->W != sc->W || rep->H != sc->H || rep->K != sc->K)) return -1;
    if (bd && rep) return -1;
    if (bd && (!bd->image_lo || !bd->image_hi)) return -1;
    const int V = sc->V, F = sc->F, C = sc->C, S = sc->S, K = sc->K, W = sc->W, H = sc->H;
    const size_t nkf = (size_t)(S + 1) * V * 2, ng = nkf + (size_t)V * C;
    const int guard = (flags || bd) && !rep;
    const int gslack = bd && grad_image;
    orc_ctx cx;
    if (orc_build(&cx, sc)) { orc_free_ctx(&cx); return -1; }
    int rb = sc->row_begin < 0 ? 0 : sc->row_begin;
    int re = (sc->row_end <= 0 || sc->row_end > H) ? H : sc->row_end;
    int rs = sc->row_step <= 0 ? 1 : sc->row_step;
    int nrows = re > rb ? (re - rb + rs - 1) / rs : 0;
    int nth = 1;
#ifdef _OPENMP
    nth = sc->nthreads > 0 ? sc->nthreads : omp_get_max_threads();
#endif
    if (rec) {
        rec->W = W; rec->H = H; rec->K = K;
        rec->winner = (int *)malloc(sizeof(int) * (size_t)H * W * K);
        rec->row_start = (int **)calloc(H, sizeof(int *));
        rec->row_list = (orc_bg_rec **)calloc(H, sizeof(orc_bg_rec *));
        rec->row_n = (int *)calloc(H, sizeof(int));
        for (size_t i = 0; i < (size_t)H * W * K; ++i) rec->winner[i] = -1;
    }
    orc_tls *tls = (orc_tls *)calloc(nth, sizeof(orc_tls));
    for (int i = 0; i < nth; ++i) {
        /* replay may add frozen faces that left the candidate set: 2F */
        tls[i].ev = (orc_eval *)malloc(sizeof(orc_eval) * 2 * F);
        tls[i].bt = (orc_bgterm *)malloc(sizeof(orc_bgterm) * 2 * F);
        tls[i].bta = (orc_bgterm *)malloc(sizeof(orc_bgterm) * F);
        tls[i].bt2 = (orc_bgterm *)malloc(sizeof(orc_bgterm) * F);
        tls[i].bta_ok = (int *)malloc(sizeof(int) * F);
        tls[i].skp = (int *)malloc(sizeof(int) * F);
        tls[i].incl = (int *)malloc(sizeof(int) * 2 * F);
        tls[i].cand = (int *)malloc(sizeof(int) * F);
        tls[i].pcand = (int *)malloc(sizeof(int) * F);
        tls[i].seen = (char *)malloc(F);
        tls[i].pre = (double *)malloc(sizeof(double) * (2 * F + 1));
        tls[i].suf = (double *)malloc(sizeof(double) * (2 * F + 1));
        if (grad_image) {
            tls[i].grad.gkf = (double *)calloc(nkf, sizeof(double));
            tls[i].grad.gattr = (double *)calloc((size_t)V * C, sizeof(double));
        }
        if (gslack) {
            tls[i].dtmp = (double *)calloc(ng, sizeof(double));
            tls[i].dmx = (double *)calloc(ng, sizeof(double));
            tls[i].slack = (double *)calloc(ng, sizeof(double));
        }
    }
    const double thr = 0.25e-5 * K;   /* flip that would move the pixel by > 1/4 of 1e-5 */

#pragma omp parallel for schedule(dynamic, 1) num_threads(nth)
    for (int ri = 0; ri < nrows; ++ri) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        orc_tls *t = &tls[tid];
        int r = rb + ri * rs;
        double v = (double)(H - 2 * r - 1) / (double)H;     /* reading: row 0 at the top */
        double *acc = (double *)calloc((size_t)W * (C + 1) * 3, sizeof(double));
        double *acc_lo = acc + (size_t)W * (C + 1), *acc_hi = acc_lo + (size_t)W * (C + 1);
        const int *rep_start = rep ? rep->row_start[r] : NULL;
        const orc_bg_rec *rep_list = rep ? rep->row_list[r] : NULL;
        int *rstart = NULL, *rend = NULL;
        t->rl_n = 0;
        if (rec) {
            rstart = (int *)malloc(sizeof(int) * ((size_t)W * K + 1));
            rend = (int *)malloc(sizeof(int) * ((size_t)W * K + 1));
        }
        for (int s = 0; s < S; ++s) {
            if (cx.seg_n[s] == 0) continue;
            int nc = 0;
            for (int f = 0; f < F; ++f) {
                const double *b = cx.swept + ((size_t)s * F + f) * 4;
                if (v >= b[2] && v <= b[3]) t->cand[nc++] = f;
            }
            for (int c = 0; c < W; ++c) {
                double u = (double)(2 * c + 1 - W) / (double)W;
                int np = 0;
                for (int j = 0; j < nc; ++j) {
                    const double *b = cx.swept + ((size_t)s * F + t->cand[j]) * 4;
                    if (u >= b[0] && u <= b[1]) { t->pcand[np] = t->cand[j]; t->seen[np] = 0; ++np; }
                }
                for (int k = cx.seg_k0[s]; k < cx.seg_k0[s] + cx.seg_n[s]; ++k) {
                    int ss, X; double tau;
                    orc_schedule(k, K, S, &ss, &tau, &X);
                    size_t pk = ((size_t)r * W + c) * K + k;
                    if (rec) rstart[(size_t)c * K + k] = t->rl_n;
                    /* candidates of this sub-frame: expanded bbox test */
                    int n = 0;
                    for (int j = 0; j < np; ++j) {
                        orc_eval *ev = &t->ev[n];
                        ev->f = t->pcand[j];
                        orc_face_pos(&cx, ev->f, k, ss, tau, ev->P);
                        double x0 = fmin(ev->P[0][0], fmin(ev->P[1][0], ev->P[2][0]));
                        double x1 = fmax(ev->P[0][0], fmax(ev->P[1][0], ev->P[2][0]));
                        double y0 = fmin(ev->P[0][1], fmin(ev->P[1][1], ev->P[2][1]));
                        double y1 = fmax(ev->P[0][1], fmax(ev->P[1][1], ev->P[2][1]));
                        if (u < x0 - cx.halo || u > x1 + cx.halo || v < y0 - cx.halo || v > y1 + cx.halo)
                            continue;
                        int inbox = u >= x0 && u <= x1 && v >= y0 && v <= y1;
                        if (inbox) {
                            t->cnt[CNT_BBOX] += 1;
                            if (!t->seen[j]) { t->seen[j] = 1; t->cnt[CNT_SETUP] += 1; }
                        }
                        orc_eval_face(&cx, ev, ss, tau, u, v);
                        if (ev->skip) t->cnt[CNT_SKIP] += 1;
                        if (ev->cover) t->cnt[CNT_COV] += 1;
                        ++n;
                    }
                    double val[16];
                    int winner;
                    if (rep) {
                        int wf = rep->winner[pk];
                        winner = -1;
                        for (int j = 0; j < n; ++j) if (t->ev[j].f == wf) winner = j;
                        if (wf >= 0 && winner < 0) {   /* frozen winner left the candidate set */
                            orc_eval *ev = &t->ev[n];
                            ev->f = wf;
                            orc_face_pos(&cx, wf, k, ss, tau, ev->P);
                            orc_eval_face(&cx, ev, ss, tau, u, v);
                            winner = n++;
                        }
                    } else {
                        for (int j = 0; j < n; ++j) t->incl[j] = t->ev[j].cover;
                        winner = orc_zbuffer(t->ev, n, t->incl);
                    }
                    int m = 0;
                    if (winner >= 0) {
                        orc_shade(sc, &t->ev[winner], val);
                        val[C] = 1.0;
                        t->cnt[CNT_FG] += 1;
                        if (rec) rec->winner[pk] = t->ev[winner].f;
                    } else if (rep) {
                        double prod = 1.0;
                        for (int e = rep_start[(size_t)c * K + k]; e < rep_start[(size_t)c * K + k + 1]; ++e) {
                            const orc_bg_rec *br = &rep_list[e];
                            int j = -1;
                            for (int q = 0; q < n; ++q) if (t->ev[q].f == br->face) j = q;
                            if (j < 0) {
                                orc_eval *ev = &t->ev[n];
                                ev->f = br->face;
                                orc_face_pos(&cx, br->face, k, ss, tau, ev->P);
                                orc_eval_face(&cx, ev, ss, tau, u, v);
                                j = n++;
                            }
                            orc_bg_face(&cx, &t->ev[j], ss, X, u, v, br->edge, br->clamp, &t->bt[m]);
                            t->bt[m].j = j;
                            prod *= t->bt[m].om;
                            ++m;
                        }
                        for (int c2 = 0; c2 < C; ++c2) val[c2] = 0.0;
                        val[C] = 1.0 - prod;
                    } else {
                        double alpha;
                        m = orc_background(&cx, t, n, ss, X, u, v, &alpha);
                        for (int c2 = 0; c2 < C; ++c2) val[c2] = 0.0;
                        val[C] = alpha;
                        t->cnt[CNT_BG] += 1;
                        t->cnt[CNT_BGPAIRS] += m;
                        if (!(orc_weight_bound(t->bt, m) < ORC_ADJ_WMIN)) t->cnt[CNT_BGLIVE] += m;
                        if (rec)
                            for (int q = 0; q < m; ++q) {
                                orc_bg_rec br = { (int)k, t->bt[q].f, t->bt[q].edge, t->bt[q].clamp };
                                orc_push_rec(t, br);
                            }
                    }
                    double gI[16];
                    if (grad_image)
                        for (int c2 = 0; c2 <= C; ++c2)
                            gI[c2] = grad_image[((size_t)c2 * H + r) * W + c] / (double)K;
                    double vlo[16], vhi[16];
                    for (int c2 = 0; c2 <= C; ++c2) vlo[c2] = vhi[c2] = val[c2];
                    if (guard) {
                        int fb = orc_alternatives(&cx, t, n, m, ss, tau, X, u, v, winner, val, thr,
                                                  gslack ? gI : NULL, vlo, vhi);
                        if (fb && flags) flags[(size_t)r * W + c] |= fb;
                        if (fb & 1) t->cnt[CNT_FLAGGED] += 1;
                        if (fb & 2) t->cnt[CNT_ALT_GRAD] += 1;
                        for (int c2 = 0; c2 <= C; ++c2)
                            if (vhi[c2] > vlo[c2]) { t->cnt[CNT_ALT_VALUE] += 1; break; }
                    }
                    if (rec) rend[(size_t)c * K + k] = t->rl_n;
                    for (int c2 = 0; c2 <= C; ++c2) {
                        acc[(size_t)c * (C + 1) + c2] += val[c2];
                        acc_lo[(size_t)c * (C + 1) + c2] += vlo[c2];
                        acc_hi[(size_t)c * (C + 1) + c2] += vhi[c2];
                    }

                    if (grad_image) {
                        if (winner >= 0) orc_adj_fg(&cx, &t->grad, &t->ev[winner], gI, ss, tau);
                        else if (m > 0) orc_adj_bgset(&cx, &t->grad, t, t->bt, m, gI, ss, tau, X, u, v);
                        if (gslack && (winner >= 0 || m > 0))
                            orc_cond_bound(&cx, t, winner, m, gI, ss, tau, X, u, v);
                    }
                }
            }
        }
        for (int c = 0; c < W; ++c)
            for (int c2 = 0; c2 <= C; ++c2) {
                size_t o = ((size_t)c2 * H + r) * W + c, a = (size_t)c * (C + 1) + c2;
                image[o] = acc[a] / (double)K;
                if (bd) { bd->image_lo[o] = acc_lo[a] / (double)K; bd->image_hi[o] = acc_hi[a] / (double)K; }
            }
        free(acc);
        if (rec) {
            /* sub-frames were visited segment by segment; store in (col, k) order */
            orc_bg_rec *lst = (orc_bg_rec *)malloc(sizeof(orc_bg_rec) * (t->rl_n + 1));
            int *st = (int *)malloc(sizeof(int) * ((size_t)W * K + 1));
            int pos = 0;
            for (size_t ck = 0; ck < (size_t)W * K; ++ck) {
                st[ck] = pos;
                for (int e = rstart[ck]; e < rend[ck]; ++e) lst[pos++] = t->rl[e];
            }
            st[(size_t)W * K] = pos;
            rec->row_start[r] = st;
            rec->row_list[r] = lst;
            rec->row_n[r] = pos;
            free(rstart);
            free(rend);
        }
    }

    if (counters) {
        for (int i = 0; i < ORC_NCNT; ++i) counters[i] = 0;
        for (int i = 0; i < nth; ++i)
            for (int j = 0; j < ORC_NCNT; ++j) counters[j] += tls[i].cnt[j];
    }
    if (grad_image) {
        double *gkf = (double *)calloc(nkf, sizeof(double));
        double *skf = gslack ? (double *)calloc(nkf, sizeof(double)) : NULL;
        if (grad_attrs) memset(grad_attrs, 0, sizeof(double) * (size_t)V * C);
        if (gslack && bd->slack_attrs) memset(bd->slack_attrs, 0, sizeof(double) * (size_t)V * C);
        for (int i = 0; i < nth; ++i) {
            for (size_t j = 0; j < nkf; ++j) gkf[j] += tls[i].grad.gkf[j];
            if (grad_attrs)
                for (size_t j = 0; j < (size_t)V * C; ++j) grad_attrs[j] += tls[i].grad.gattr[j];
            if (gslack) {
                for (size_t j = 0; j < nkf; ++j) skf[j] += tls[i].slack[j];
                if (bd->slack_attrs)
                    for (size_t j = 0; j < (size_t)V * C; ++j) bd->slack_attrs[j] += tls[i].slack[nkf + j];
            }
        }
        if (grad_kf) memcpy(grad_kf, gkf, sizeof(double) * nkf);
        if (gslack && bd->slack_kf) memcpy(bd->slack_kf, skf, sizeof(double) * nkf);
        if (grad_verts || (gslack && bd->slack_verts)) {
            /* keyframe -> rest position: chain through the projection (App. I)
             * and the rigid keyframe transform; the bound goes through the
             * magnitudes of the same linear map */
            for (int v = 0; v < V; ++v) {
                double g[3] = { 0, 0, 0 }, sl[3] = { 0, 0, 0 };
                for (int s = 0; s <= S; ++s) {
                    const double *m = sc->model + s * 12, *vw = sc->view, *p = sc->verts + v * 3;
                    double w[3], c[3];
                    for (int r = 0; r < 3; ++r)
                        w[r] = m[r * 4] * p[0] + m[r * 4 + 1] * p[1] + m[r * 4 + 2] * p[2] + m[r * 4 + 3];
                    for (int r = 0; r < 3; ++r)
                        c[r] = vw[r * 4] * w[0] + vw[r * 4 + 1] * w[1] + vw[r * 4 + 2] * w[2] + vw[r * 4 + 3];
                    double t = sc->tan_half_fov;
                    /* column i of the map (gx, gy) -> rest-position gradient */
                    double col[2][3];
                    for (int i = 0; i < 2; ++i) {
                        double gc[3] = { i == 0 ? 1.0 / (c[2] * t) : 0.0, i == 1 ? 1.0 / (c[2] * t) : 0.0,
                                         -c[i] / (c[2] * c[2] * t) };
                        double gw[3];
                        for (int j = 0; j < 3; ++j) gw[j] = vw[0 * 4 + j] * gc[0] + vw[1 * 4 + j] * gc[1] + vw[2 * 4 + j] * gc[2];
                        for (int j = 0; j < 3; ++j) col[i][j] = m[0 * 4 + j] * gw[0] + m[1 * 4 + j] * gw[1] + m[2 * 4 + j] * gw[2];
                    }
                    double gx = gkf[((size_t)s * V + v) * 2], gy = gkf[((size_t)s * V + v) * 2 + 1];
                    for (int j = 0; j < 3; ++j) g[j] += col[0][j] * gx + col[1][j] * gy;
                    if (skf) {
                        double sx = skf[((size_t)s * V + v) * 2], sy = skf[((size_t)s * V + v) * 2 + 1];
                        for (int j = 0; j < 3; ++j) sl[j] += fabs(col[0][j]) * sx + fabs(col[1][j]) * sy;
                    }
                }
                if (grad_verts) for (int j = 0; j < 3; ++j) grad_verts[v * 3 + j] = g[j];
                if (skf && bd->slack_verts) for (int j = 0; j < 3; ++j) bd->slack_verts[v * 3 + j] = sl[j];
            }
        }
        free(gkf);
        free(skf);
    }
    for (int i = 0; i < nth; ++i) {
        free(tls[i].ev); free(tls[i].bt); free(tls[i].bta); free(tls[i].bt2); free(tls[i].bta_ok);
        free(tls[i].skp); free(tls[i].incl); free(tls[i].cand); free(tls[i].pcand);
        free(tls[i].seen); free(tls[i].pre); free(tls[i].suf); free(tls[i].grad.gkf);
        free(tls[i].grad.gattr); free(tls[i].grad.ji); free(tls[i].grad.jv); free(tls[i].rl);
        free(tls[i].j0i); free(tls[i].j0v); free(tls[i].dtmp); free(tls[i].dmx); free(tls[i].slack);
        free(tls[i].mxl);
    }
    free(tls);
    orc_free_ctx(&cx);
    return 0;
}

orc_decisions *orc_decisions_new(void) { return (orc_decisions *)calloc(1, sizeof(orc_decisions)); }

void orc_decisions_free(orc_decisions *d)
{
    if (!d) return;
    if (d->row_start)
        for (int r = 0; r < d->H; ++r) { free(d->row_start[r]); free(d->row_list[r]); }
    free(d->row_start); free(d->row_list); free(d->row_n); free(d->winner);
    free(d);
}

/* keyframe screen positions [S+1][V][3] (x, y, camera depth) */
int orc_keyframes(const orc_scene *sc, double *out)
{
    for (int s = 0; s <= sc->S; ++s)
        for (int v = 0; v < sc->V; ++v)
            orc_project(sc->view, sc->model + s * 12, sc->tan_half_fov, sc->verts + v * 3,
                        out + ((size_t)s * sc->V + v) * 3);
    return 0;
}

void orc_schedule_export(int k, int K, int S, int *s, double *tau, int *X) { orc_schedule(k, K, S, s, tau, X); }

int orc_sizeof_scene(void) { return (int)sizeof(orc_scene); }
