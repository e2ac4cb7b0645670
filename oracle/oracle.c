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
#define ORC_GUARD_W 2e-5       /* guard band on min_i w_i for parity reporting */
#define ORC_GUARD_DEPTH 1e-6   /* relative depth near-tie */
#define ORC_GUARD_EDGE 1e-9    /* relative near-tie between edge distances */
#define ORC_GUARD_SIGMA 2e-5   /* edge parameter near a clamp bound (times max |w|) */
#define ORC_GUARD_EDGE_GRAD 1e-5 /* relative edge near-tie that may change the gradient */
#define ORC_MAX_AMBIG 6

enum { CNT_BBOX, CNT_COV, CNT_FG, CNT_BG, CNT_BGPAIRS, CNT_SETUP, CNT_FLAGGED, CNT_SKIP, ORC_NCNT };

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
 * Returns the squared distance; *gap receives the relative gap to the
 * runner-up edge whose point differs (for the parity guard band). */
static double orc_closest_edge(const double T[3][2], double qx, double qy,
                               int *edge, double *sigma, int *clamp, double *sigma_raw,
                               double *gap)
{
    double best = INFINITY, second = INFINITY;
    double bpx = 0, bpy = 0;
    for (int e = 0; e < 3; ++e) {
        int a = e, b = (e + 1) % 3;
        double ex = T[b][0] - T[a][0], ey = T[b][1] - T[a][1];
        double ee = ex * ex + ey * ey;
        double t = ee > 0 ? ((qx - T[a][0]) * ex + (qy - T[a][1]) * ey) / ee : 0.0;
        double traw = t;
        int cl = 1;
        if (t < 0) { t = 0; cl = 0; } else if (t > 1) { t = 1; cl = 2; }
        if (ee <= 0) cl = 0;
        double px = T[a][0] + t * ex, py = T[a][1] + t * ey;
        double dist = (qx - px) * (qx - px) + (qy - py) * (qy - py);
        if (dist < best) {
            if (fabs(px - bpx) + fabs(py - bpy) > 1e-12 || best == INFINITY) second = best;
            best = dist; *edge = e; *sigma = t; *clamp = cl; *sigma_raw = traw;
            bpx = px; bpy = py;
        } else if (dist < second && fabs(px - bpx) + fabs(py - bpy) > 1e-12) {
            second = dist;
        }
    }
    *gap = (second - best) / (fabs(best) + 1e-300);
    return best;
}

void orc_closest_point(const double *tri /*[3][2]*/, double qx, double qy, double *wstar /*[3]*/)
{
    double T[3][2];
    int e, cl; double sg, sr, gap;
    for (int i = 0; i < 3; ++i) { T[i][0] = tri[2 * i]; T[i][1] = tri[2 * i + 1]; }
    orc_closest_edge(T, qx, qy, &e, &sg, &cl, &sr, &gap);
    wstar[0] = wstar[1] = wstar[2] = 0.0;
    wstar[e] = 1.0 - sg;
    wstar[(e + 1) % 3] += sg;
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
    int f, edge, clamp;
    double A, om, d, sigma, sigma_raw;
    double w[3];
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

/* Barycentrics, depth and coverage of one face at one (pixel, sub-frame). */
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
    if (ev->skip) { ev->cover = 0; ev->mw = -INFINITY; ev->depth = INFINITY; return; }
    ev->mw = fmin(ev->w[0], fmin(ev->w[1], ev->w[2]));
    ev->cover = ev->mw >= 0.0;                       /* reading: inclusive */
    ev->depth = ev->w[0] * ev->P[0][2] + ev->w[1] * ev->P[1][2] + ev->w[2] * ev->P[2][2];
}

/* Background term of one face (eqs 10, 13, 14).  Returns 1 if it contributes. */
static int orc_bg_face(const orc_ctx *cx, const orc_eval *ev, int s, int X, double u, double v,
                       int forced_edge, int forced_clamp, orc_bgterm *bt, double *gap)
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
    int e, cl; double sg, sr;
    orc_closest_edge(T, qx, qy, &e, &sg, &cl, &sr, gap);
    if (forced_edge >= 0) {            /* frozen-decision replay */
        int a = forced_edge, b = (forced_edge + 1) % 3;
        double ex = T[b][0] - T[a][0], ey = T[b][1] - T[a][1], ee = ex * ex + ey * ey;
        sr = ee > 0 ? ((qx - T[a][0]) * ex + (qy - T[a][1]) * ey) / ee : 0.0;
        e = forced_edge; cl = forced_clamp;
        sg = cl == 0 ? 0.0 : (cl == 2 ? 1.0 : sr);
    }
    int a = e, b = (e + 1) % 3;
    /* eq 14 (reading): p* = F(tau) w*, distance measured at the sub-frame */
    double px = (1.0 - sg) * ev->P[a][0] + sg * ev->P[b][0];
    double py = (1.0 - sg) * ev->P[a][1] + sg * ev->P[b][1];
    double d = (u - px) * (u - px) + (v - py) * (v - py);
    bt->f = ev->f; bt->edge = e; bt->clamp = cl; bt->sigma = sg; bt->sigma_raw = sr; bt->d = d;
    for (int i = 0; i < 3; ++i) bt->w[i] = ev->w[i];
    if (forced_edge < 0 && sc->eps_cutoff > 0 && d > cx->dmax) return 0;
    bt->A = exp(-d / sc->delta);
    bt->om = -expm1(-d / sc->delta);
    return 1;
}

/* gradient buffers of one thread */
typedef struct { double *gkf; double *gattr; } orc_grad;

static void orc_add_kf(const orc_ctx *cx, orc_grad *g, int f, int i, int s, double gx, double gy)
{
    int V = cx->sc->V;
    int vi = cx->sc->faces[f * 3 + i];
    double *p = g->gkf + ((size_t)s * V + vi) * 2;
    p[0] += gx; p[1] += gy;
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

/* z-buffer: closest covering face, ties to the lowest face index (reading).
 * mode 0: nominal cover flags; mode 1: custom subset via incl[] */
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
    orc_bgterm *bt;
    int *incl;
    int *cand;        /* row-segment candidates                            */
    int *pcand;       /* pixel-segment candidates                          */
    char *seen;       /* per pcand: bbox hit somewhere in the segment      */
    double *pre, *suf;
    orc_grad grad;
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
                          double *alpha, int *edge_tie)
{
    int m = 0;
    double prod = 1.0;
    *edge_tie = 0;   /* bit 0: closest points of two edges tie; bit 1: edge parameter at a clamp bound */
    for (int j = 0; j < n; ++j) {
        if (t->ev[j].skip) continue;
        double gap;
        if (orc_bg_face(cx, &t->ev[j], s, X, u, v, -1, 0, &t->bt[m], &gap)) {
            /* two edges whose closest points differ are nearly as close: the
             * value is continuous across the switch, the frozen-decision
             * derivative (which vertices and whether the edge parameter
             * carries gradient) is not */
            if (gap < ORC_GUARD_EDGE) *edge_tie |= 3;
            else if (gap < ORC_GUARD_EDGE_GRAD) *edge_tie |= 2;
            /* the edge parameter within rounding distance of 0 or 1: the value
             * is continuous there but the frozen-decision derivative is not */
            const orc_bgterm *bq = &t->bt[m];
            double wm = fmax(1.0, fmax(fabs(bq->w[0]), fmax(fabs(bq->w[1]), fabs(bq->w[2]))));
            double gs = ORC_GUARD_SIGMA * wm;
            if (fabs(bq->sigma_raw) < gs || fabs(bq->sigma_raw - 1.0) < gs) *edge_tie |= 2;
            prod *= t->bt[m].om;
            ++m;
        }
    }
    *alpha = 1.0 - prod;
    return m;
}

/* Parity guard band of the foreground decision of one (pixel, sub-frame).
 * Enumerates every in/out choice of the faces whose min w is within
 * ORC_GUARD_W of 0, plus depth near-ties of each resulting z-buffer.
 * Returns bit 0 if a flip would move the sub-frame value by more than thr,
 * bit 1 if the z-buffer winner (whose vertices receive the gradient) could
 * change at all. */
static int orc_guard(const orc_ctx *cx, orc_tls *t, int n, int s, int X, double u, double v,
                     int nominal, const double *val, double thr)
{
    const orc_scene *sc = cx->sc;
    int amb[ORC_MAX_AMBIG], na = 0;
    for (int j = 0; j < n; ++j) {
        if (fabs(t->ev[j].D) >= 0.5 * ORC_TAU_DET && fabs(t->ev[j].D) <= 2.0 * ORC_TAU_DET) return 3;
        if (t->ev[j].skip) continue;
        if (fabs(t->ev[j].mw) < ORC_GUARD_W) {
            if (na == ORC_MAX_AMBIG) return 3;
            amb[na++] = j;
        }
    }
    double bgalpha = -1.0;
    double alt[16];
    int bits = 0;
    for (int mask = 0; mask < (1 << na); ++mask) {
        for (int j = 0; j < n; ++j) t->incl[j] = t->ev[j].cover;
        for (int a = 0; a < na; ++a) t->incl[amb[a]] = (mask >> a) & 1;
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
            if (cand == nominal) continue;
            bits |= 2;
            if (cand >= 0) {
                orc_shade(sc, &t->ev[cand], alt);
                alt[sc->C] = 1.0;
            } else {
                if (bgalpha < 0) { int tie; orc_background(cx, t, n, s, X, u, v, &bgalpha, &tie); }
                for (int c = 0; c < sc->C; ++c) alt[c] = 0.0;
                alt[sc->C] = bgalpha;
            }
            for (int c = 0; c <= sc->C; ++c)
                if (fabs(alt[c] - val[c]) > thr) return 3;
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
 * value beyond tolerance, bit 1 when such a decision could change which
 * vertices receive gradient (winner identity, clamp state of the closest
 * point).  counters[8]
 * (optional): bbox pairs, covering pairs, fg pixel-subframes, bg
 * pixel-subframes, contributing bg pairs, distinct (pixel, face, segment)
 * setups, guard-flagged pixel-subframes, skipped degenerate pairs.
 * With grad_image: grad_kf [S+1][V][2] (optional), grad_verts [V][3] and
 * grad_attrs [V][C] are overwritten with dL/d(...) for L = sum grad_image*I.
 * rec: record decisions; rep: replay recorded decisions (frozen surrogate).
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int orc_render(const orc_scene *sc, double *image, int *flags, double *counters,
               const double *grad_image, double *grad_kf, double *grad_verts, double *grad_attrs,
               orc_decisions *rec, const orc_decisions *rep)
{
    if (!sc || sc->V <= 0 || sc->F <= 0 || sc->C <= 0 || sc->C > 14 || sc->S <= 0 || sc->K <= 0 ||
        sc->W <= 0 || sc->H <= 0 || !(sc->delta > 0) || !image)
        return -1;
    if (sc->motion == 1 && !sc->model_sub) return -1;
    if (grad_image && (sc->motion != 0 || sc->distance != 0)) return -1;
    if (rep && (rep->W != sc->W || rep->H != sc->H || rep->K != sc->K)) return -1;
    const int V = sc->V, F = sc->F, C = sc->C, S = sc->S, K = sc->K, W = sc->W, H = sc->H;
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
        tls[i].ev = (orc_eval *)malloc(sizeof(orc_eval) * F);
        tls[i].bt = (orc_bgterm *)malloc(sizeof(orc_bgterm) * F);
        tls[i].incl = (int *)malloc(sizeof(int) * F);
        tls[i].cand = (int *)malloc(sizeof(int) * F);
        tls[i].pcand = (int *)malloc(sizeof(int) * F);
        tls[i].seen = (char *)malloc(F);
        tls[i].pre = (double *)malloc(sizeof(double) * (F + 1));
        tls[i].suf = (double *)malloc(sizeof(double) * (F + 1));
        if (grad_image) {
            tls[i].grad.gkf = (double *)calloc((size_t)(S + 1) * V * 2, sizeof(double));
            tls[i].grad.gattr = (double *)calloc((size_t)V * C, sizeof(double));
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
        double *acc = (double *)calloc((size_t)W * (C + 1), sizeof(double));
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
                    int m = 0, edge_tie = 0;
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
                            double gap;
                            orc_bg_face(&cx, &t->ev[j], ss, X, u, v, br->edge, br->clamp, &t->bt[m], &gap);
                            t->bt[m].A = exp(-t->bt[m].d / sc->delta);
                            t->bt[m].om = -expm1(-t->bt[m].d / sc->delta);
                            prod *= t->bt[m].om;
                            t->incl[m] = j;
                            ++m;
                        }
                        for (int c2 = 0; c2 < C; ++c2) val[c2] = 0.0;
                        val[C] = 1.0 - prod;
                    } else {
                        int tie;
                        double alpha;
                        m = orc_background(&cx, t, n, ss, X, u, v, &alpha, &tie);
                        for (int c2 = 0; c2 < C; ++c2) val[c2] = 0.0;
                        val[C] = alpha;
                        t->cnt[CNT_BG] += 1;
                        t->cnt[CNT_BGPAIRS] += m;
                        edge_tie = tie;
                        if (rec)
                            for (int q = 0; q < m; ++q) {
                                orc_bg_rec br = { (int)k, t->bt[q].f, t->bt[q].edge, t->bt[q].clamp };
                                orc_push_rec(t, br);
                            }
                    }
                    if (flags && !rep) {
                        int fb = edge_tie | orc_guard(&cx, t, n, ss, X, u, v, winner, val, thr);
                        if (fb) flags[(size_t)r * W + c] |= fb;
                        if (fb & 1) t->cnt[CNT_FLAGGED] += 1;
                    }
                    if (rec) rend[(size_t)c * K + k] = t->rl_n;
                    for (int c2 = 0; c2 <= C; ++c2) acc[(size_t)c * (C + 1) + c2] += val[c2];

                    if (grad_image) {
                        double gI[16];
                        for (int c2 = 0; c2 <= C; ++c2)
                            gI[c2] = grad_image[((size_t)c2 * H + r) * W + c] / (double)K;
                        if (winner >= 0) {
                            const orc_eval *ev = &t->ev[winner];
                            double gw[3];
                            for (int i = 0; i < 3; ++i) {
                                int vi = sc->faces[ev->f * 3 + i];
                                gw[i] = 0;
                                for (int c2 = 0; c2 < C; ++c2) {
                                    gw[i] += gI[c2] * sc->attrs[(size_t)vi * C + c2];
                                    t->grad.gattr[(size_t)vi * C + c2] += ev->w[i] * gI[c2];
                                }
                            }
                            orc_adj_bary(&cx, &t->grad, ev, ev->w, gw, ss, tau);
                        } else if (m > 0) {
                            /* d alpha / d A_j = prod_{m != j} (1 - A_m): prefix/suffix products */
                            t->pre[0] = 1.0;
                            for (int q = 0; q < m; ++q) t->pre[q + 1] = t->pre[q] * t->bt[q].om;
                            t->suf[m] = 1.0;
                            for (int q = m - 1; q >= 0; --q) t->suf[q] = t->suf[q + 1] * t->bt[q].om;
                            for (int q = 0; q < m; ++q) {
                                const orc_bgterm *bt = &t->bt[q];
                                const orc_eval *ev = NULL;
                                for (int j = 0; j < n; ++j) if (t->ev[j].f == bt->f) { ev = &t->ev[j]; break; }
                                double dA = gI[C] * t->pre[q] * t->suf[q + 1];
                                double gd = dA * (-bt->A / sc->delta);
                                orc_adj_bg(&cx, &t->grad, ev, bt, ss, tau, X, u, v, gd);
                            }
                        }
                    }
                }
            }
        }
        for (int c = 0; c < W; ++c)
            for (int c2 = 0; c2 <= C; ++c2)
                image[((size_t)c2 * H + r) * W + c] = acc[(size_t)c * (C + 1) + c2] / (double)K;
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
        double *gkf = (double *)calloc((size_t)(S + 1) * V * 2, sizeof(double));
        if (grad_attrs) memset(grad_attrs, 0, sizeof(double) * (size_t)V * C);
        for (int i = 0; i < nth; ++i) {
            for (size_t j = 0; j < (size_t)(S + 1) * V * 2; ++j) gkf[j] += tls[i].grad.gkf[j];
            if (grad_attrs)
                for (size_t j = 0; j < (size_t)V * C; ++j) grad_attrs[j] += tls[i].grad.gattr[j];
        }
        if (grad_kf) memcpy(grad_kf, gkf, sizeof(double) * (size_t)(S + 1) * V * 2);
        if (grad_verts) {
            /* keyframe -> rest position: chain through the projection (App. I)
             * and the rigid keyframe transform */
            for (int v = 0; v < V; ++v) {
                double g[3] = { 0, 0, 0 };
                for (int s = 0; s <= S; ++s) {
                    const double *m = sc->model + s * 12, *vw = sc->view, *p = sc->verts + v * 3;
                    double w[3], c[3];
                    for (int r = 0; r < 3; ++r)
                        w[r] = m[r * 4] * p[0] + m[r * 4 + 1] * p[1] + m[r * 4 + 2] * p[2] + m[r * 4 + 3];
                    for (int r = 0; r < 3; ++r)
                        c[r] = vw[r * 4] * w[0] + vw[r * 4 + 1] * w[1] + vw[r * 4 + 2] * w[2] + vw[r * 4 + 3];
                    double t = sc->tan_half_fov;
                    double gx = gkf[((size_t)s * V + v) * 2], gy = gkf[((size_t)s * V + v) * 2 + 1];
                    double gc[3] = { gx / (c[2] * t), gy / (c[2] * t),
                                     -(gx * c[0] + gy * c[1]) / (c[2] * c[2] * t) };
                    double gw[3];
                    for (int j = 0; j < 3; ++j) gw[j] = vw[0 * 4 + j] * gc[0] + vw[1 * 4 + j] * gc[1] + vw[2 * 4 + j] * gc[2];
                    for (int j = 0; j < 3; ++j) g[j] += m[0 * 4 + j] * gw[0] + m[1 * 4 + j] * gw[1] + m[2 * 4 + j] * gw[2];
                }
                grad_verts[v * 3 + 0] = g[0];
                grad_verts[v * 3 + 1] = g[1];
                grad_verts[v * 3 + 2] = g[2];
            }
        }
        free(gkf);
    }
    for (int i = 0; i < nth; ++i) {
        free(tls[i].ev); free(tls[i].bt); free(tls[i].incl); free(tls[i].cand); free(tls[i].pcand);
        free(tls[i].seen); free(tls[i].pre); free(tls[i].suf); free(tls[i].grad.gkf);
        free(tls[i].grad.gattr); free(tls[i].rl);
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
