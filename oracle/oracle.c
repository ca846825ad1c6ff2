/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of the indirect
 * single-layer collocation BEM of "Dielectric Breakdown Prediction with
 * GPU-Accelerated BEM" (arXiv 2003.12663), discretised with flat triangles,
 * piecewise-constant virtual charge sigma and centroid collocation, and (for
 * conductor bodies) the paper's own nodal piecewise-linear basis with vertex
 * collocation (the orc_p1_* functions).  It exists
 * only to check the GPU library: tests, the smoke check and the benchmark's
 * CPU-baseline leg may call it; the product path never does.  It shares no
 * source, header or table with the GPU library.
 *
 * Every step follows the paper in its own order:
 *   - single-layer potential and its field (Sec. 2, Eq. SL and the field
 *     formula that closes Sec. 2),
 *   - conductor, floating-conductor and dielectric rows (Eqs. Final1-Final4,
 *     with K' from Eq. ADL),
 *   - regular / near-singular / singular classification of a (point,
 *     triangle) pair by circumcentre distance D against eta * circumradius R
 *     (Sec. 4),
 *   - GMRES with a diagonal preconditioner (Sec. 5.2),
 *   - field lines and the streamer-inception integral (Sec. 1, Eq.
 *     Breakdowncrit).
 * Readings where the paper is silent are listed with each function.
 * No blocking, fusion or reordering beyond the definitions is done; OpenMP
 * only splits independent rows, points or lines across threads.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* threads of the parallel loops below (reported beside the timed CPU baseline) */
int orc_num_threads(void) { return omp_get_max_threads(); }

/* ORC_SHEET: a thin floating conductive sheet modelled by one (open) surface, Eq. sheets */
enum { ORC_DIRICHLET = 0, ORC_FLOATING = 1, ORC_INTERFACE = 2, ORC_SHEET = 3 };
static int is_floating_kind(int32_t kind) { return kind == ORC_FLOATING || kind == ORC_SHEET; }

typedef struct {
    int64_t n_vert;
    const double* vert;      /* [n_vert][3] */
    int64_t n_tri;
    const int32_t* tri;      /* [n_tri][3], CCW about the normal that points into eps+ */
    const int32_t* tri_body; /* [n_tri] */
    int32_t n_body;
    const int32_t* body_kind;
    const double* eps_plus;
    const double* eps_minus;
    double eta;              /* regular iff D > eta * R */
    int32_t constraint_form; /* 0: literal Eq. Final4, 1: net charge sum a_i sigma_i */
} orc_problem;

typedef struct {
    double h, e_min, start_offset;
    int32_t max_steps, direction;
    double alpha_a, alpha_e0, alpha_p, k_str;
} orc_trace_params;

/* ------------------------------------------------------------------ vectors */
static void sub3(const double a[3], const double b[3], double o[3]) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

/* ------------------------------------------------------------ panel geometry
 * Flat triangle (v1, v2, v3): area, unit normal (right-hand rule, pointing
 * into the eps+ side), centroid (the collocation point), circumcentre and
 * circumradius (precomputed for the Sec. 4 classification).
 */
void orc_panel_geometry(const double v1[3], const double v2[3], const double v3[3],
                        double cen[3], double nrm[3], double* area, double cc[3], double* R)
{
    double u[3], w[3], uxw[3];
    sub3(v2, v1, u);
    sub3(v3, v1, w);
    cross3(u, w, uxw);
    double len = norm3(uxw);
    *area = 0.5 * len;
    for (int k = 0; k < 3; ++k) {
        nrm[k] = uxw[k] / len;
        cen[k] = (v1[k] + v2[k] + v3[k]) / 3.0;
    }
    /* circumcentre: v1 + (|w|^2 (u x w) x u + |u|^2 w x (u x w)) / (2 |u x w|^2) */
    double t1[3], t2[3];
    cross3(uxw, u, t1);
    cross3(w, uxw, t2);
    double uu = dot3(u, u), ww = dot3(w, w), d = 2.0 * dot3(uxw, uxw);
    for (int k = 0; k < 3; ++k) cc[k] = v1[k] + (ww * t1[k] + uu * t2[k]) / d;
    double r[3];
    sub3(v1, cc, r);
    *R = norm3(r);
}

/* ------------------------------------------------------ 7-point Gauss rule
 * Degree-5 symmetric rule on the triangle (Radon 1948; Stroud T2:5-1):
 * the centroid with weight 9/40, and the orbits (a, a, 1-2a) for
 * a = (6 -+ sqrt 15)/21 with weights (155 -+ sqrt 15)/1200.  Weights sum to
 * one and multiply the area.
 */
void orc_quad7_rule(double bary[7][3], double wt[7])
{
    double s15 = sqrt(15.0);
    double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
    double w1 = (155.0 - s15) / 1200.0, w2 = (155.0 + s15) / 1200.0;
    double pts[7][3] = {
        {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0},
        {a1, a1, 1.0 - 2.0 * a1}, {a1, 1.0 - 2.0 * a1, a1}, {1.0 - 2.0 * a1, a1, a1},
        {a2, a2, 1.0 - 2.0 * a2}, {a2, 1.0 - 2.0 * a2, a2}, {1.0 - 2.0 * a2, a2, a2},
    };
    double ws[7] = {9.0 / 40.0, w1, w1, w1, w2, w2, w2};
    for (int q = 0; q < 7; ++q) {
        wt[q] = ws[q];
        for (int k = 0; k < 3; ++k) bary[q][k] = pts[q][k];
    }
}

/* Regular integration: S = sum_q w_q A / (4 pi |x - y_q|),
 * F = sum_q w_q A (x - y_q) / (4 pi |x - y_q|^3).  Unit density. */
void orc_tri_quad7(const double x[3], const double v1[3], const double v2[3], const double v3[3],
                   double* S, double F[3])
{
    double bary[7][3], wt[7];
    orc_quad7_rule(bary, wt);
    double cen[3], nrm[3], area, cc[3], R;
    orc_panel_geometry(v1, v2, v3, cen, nrm, &area, cc, &R);
    double s = 0.0, f[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < 7; ++q) {
        double y[3], d[3];
        for (int k = 0; k < 3; ++k) y[k] = bary[q][0] * v1[k] + bary[q][1] * v2[k] + bary[q][2] * v3[k];
        sub3(x, y, d);
        double r = norm3(d);
        double c = wt[q] * area / (4.0 * ORC_PI);
        s += c / r;
        for (int k = 0; k < 3; ++k) f[k] += c * d[k] / (r * r * r);
    }
    *S = s;
    for (int k = 0; k < 3; ++k) F[k] = f[k];
}

/* ------------------------------------------------ analytic flat-triangle integrals
 * Closed forms for a flat triangle of unit density (Wilton et al. 1984;
 * Graglia 1993).  With w = (x - v1).n, rho = x - w n and, per edge a -> b,
 * l = (b - a)/|b - a|, m = l x n (outward in-plane normal),
 * s- = (a - rho).l, s+ = (b - rho).l, t = (a - rho).m, R- = |x - a|,
 * R+ = |x - b|, R0^2 = t^2 + w^2:
 *   f_e    = ln((R+ + s+)/(R- + s-))     (or the equal ln((R- - s-)/(R+ - s+))
 *                                          when s+ + s- <= 0, and the equal
 *                                          ln((R+ + s+)(R- - s-)/R0^2) when
 *                                          s- < 0 < s+: (R + s)(R - s) = R0^2,
 *                                          so no form loses digits to R - |s|)
 *   beta_e = atan2(t s+, R0^2 + |w| R+) - atan2(t s-, R0^2 + |w| R-)
 *   int 1/R dS        = sum_e t f_e - |w| sum_e beta_e
 *   grad_x int 1/R dS = -sum_e m f_e - sign(w) n sum_e beta_e
 * so S = (1/4pi) int 1/R dS and F = -grad S.  on_plane forces w = 0 and
 * sign(w) = 0 (principal value, used when x is the triangle's own centroid).
 */
void orc_tri_analytic(const double x[3], const double v1[3], const double v2[3], const double v3[3],
                      int on_plane, double* S, double F[3])
{
    const double* v[3] = {v1, v2, v3};
    double e1[3], e2[3], cr[3], n[3];
    sub3(v2, v1, e1);
    sub3(v3, v1, e2);
    cross3(e1, e2, cr);
    double len = norm3(cr);
    for (int k = 0; k < 3; ++k) n[k] = cr[k] / len;
    double xv[3];
    sub3(x, v1, xv);
    double w = on_plane ? 0.0 : dot3(xv, n);
    double rho[3];
    for (int k = 0; k < 3; ++k) rho[k] = x[k] - w * n[k];
    double aw = fabs(w);
    double sum_tf = 0.0, sum_beta = 0.0, mf[3] = {0.0, 0.0, 0.0};
    for (int e = 0; e < 3; ++e) {
        const double* a = v[e];
        const double* b = v[(e + 1) % 3];
        double ab[3], l[3], m[3];
        sub3(b, a, ab);
        double lab = norm3(ab);
        for (int k = 0; k < 3; ++k) l[k] = ab[k] / lab;
        cross3(l, n, m);
        double ar[3], br[3], xa[3], xb[3];
        sub3(a, rho, ar);
        sub3(b, rho, br);
        double sm = dot3(ar, l), sp = dot3(br, l), t = dot3(ar, m);
        sub3(x, a, xa);
        sub3(x, b, xb);
        double Rm = norm3(xa), Rp = norm3(xb);
        double R02 = t * t + w * w;
        double f;
        if (sm < 0.0 && sp > 0.0)   /* foot within the edge's span: R- + s- = R0^2 / (R- - s-) */
            f = log((Rp + sp) * (Rm - sm) / R02);
        else if (sp + sm > 0.0)
            f = log((Rp + sp) / (Rm + sm));
        else
            f = log((Rm - sm) / (Rp - sp));
        double beta = atan2(t * sp, R02 + aw * Rp) - atan2(t * sm, R02 + aw * Rm);
        sum_tf += t * f;
        sum_beta += beta;
        for (int k = 0; k < 3; ++k) mf[k] += m[k] * f;
    }
    double sgn = (w > 0.0) ? 1.0 : ((w < 0.0) ? -1.0 : 0.0);
    *S = (sum_tf - aw * sum_beta) / (4.0 * ORC_PI);
    for (int k = 0; k < 3; ++k) F[k] = (mf[k] + sgn * n[k] * sum_beta) / (4.0 * ORC_PI);
}

/* ------------------------------------- near-singular rule of the paper (Sec. 4)
 * The paper integrates a near-singular (point, triangle) pair by finding the
 * point of the triangle closest to x, subdividing the triangle so that this
 * point is a corner of every piece, and applying the Duffy transformation on
 * each piece, which cancels the 1/r behaviour at the corner.  Written out:
 *   1. c = argmin over the closed triangle of |x - y|: the foot point of x in
 *      the plane when it lies inside, else the nearest point of the three
 *      edge segments.
 *   2. pieces (c, a, b) for the edges a -> b of the triangle; pieces of zero
 *      area (c on that edge) are dropped.  All pieces keep the triangle's
 *      orientation, so their areas add up to its area.
 *   3. Duffy map of a piece: y(u, v) = c + u ((1 - v)(a - c) + v (b - c)),
 *      u, v in [0, 1], dS = u |(a - c) x (b - c)| du dv.
 *   4. Gauss-Legendre in u and v.  The paper's rule is adaptive; the reading
 *      here: u is cut geometrically (doubling widths) towards the corner from a
 *      quarter of d / L (d = |x - c|, L the longest piece edge), and v towards
 *      the foot of the corner on the opposite edge from a quarter of that
 *      distance over the edge length (a piece whose corner lies close to its
 *      opposite edge is narrow, and its Duffy integrand peaks in v there);
 *      ORC_DUFFY_NU x ORC_DUFFY_NV nodes per cell.
 * Unit density; S = (1/4pi) int 1/|x - y| dS, F = (1/4pi) int (x - y)/|x - y|^3 dS.
 * For x on the triangle (d = 0, the singular pair) the Duffy integrand of S is
 * smooth and S is returned; F is then a principal value that the
 * transformation does not produce and is returned as NaN.
 */
#define ORC_DUFFY_NU 16
#define ORC_DUFFY_NV 16

/* n-point Gauss-Legendre nodes and weights on [0, 1] by Newton iteration on
 * the Legendre recurrence (Golub-Welsch would serve equally; n <= 64). */
static void orc_gauss_legendre01(int n, double* t, double* w)
{
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = cos(ORC_PI * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        double wi = 2.0 / ((1.0 - z * z) * dp * dp);
        t[i] = 0.5 * (1.0 - z);
        t[n - 1 - i] = 0.5 * (1.0 + z);
        w[i] = 0.5 * wi;
        w[n - 1 - i] = 0.5 * wi;
    }
}

/* closest point of the closed segment [a, b] to x */
static void orc_closest_on_segment(const double x[3], const double a[3], const double b[3], double c[3])
{
    double ab[3], ax[3];
    sub3(b, a, ab);
    sub3(x, a, ax);
    double t = dot3(ax, ab) / dot3(ab, ab);
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    for (int k = 0; k < 3; ++k) c[k] = a[k] + t * ab[k];
}

void orc_closest_point(const double x[3], const double v1[3], const double v2[3], const double v3[3], double c[3])
{
    double e1[3], e2[3], n[3], xv[3];
    sub3(v2, v1, e1);
    sub3(v3, v1, e2);
    cross3(e1, e2, n);
    double nn = dot3(n, n);
    sub3(x, v1, xv);
    double w = dot3(xv, n) / nn;
    double rho[3];
    for (int k = 0; k < 3; ++k) rho[k] = x[k] - w * n[k];
    /* barycentric coordinates of rho from signed sub-areas */
    const double* v[3] = {v1, v2, v3};
    int inside = 1;
    for (int e = 0; e < 3; ++e) {
        double pa[3], pb[3], cr[3];
        sub3(v[(e + 1) % 3], rho, pa);
        sub3(v[(e + 2) % 3], rho, pb);
        cross3(pa, pb, cr);
        if (dot3(cr, n) < 0.0) inside = 0;
    }
    if (inside) {
        for (int k = 0; k < 3; ++k) c[k] = rho[k];
        return;
    }
    double best = INFINITY;
    for (int e = 0; e < 3; ++e) {
        double ce[3], d[3];
        orc_closest_on_segment(x, v[e], v[(e + 1) % 3], ce);
        sub3(x, ce, d);
        double dd = dot3(d, d);
        if (dd < best) {
            best = dd;
            for (int k = 0; k < 3; ++k) c[k] = ce[k];
        }
    }
}

/* breakpoints of [0, 1] graded geometrically towards t0 in [0, 1] on the scale s (> 0): t0 and
 * t0 -+ (s/4) 2^k for k = 0, 1, ... up to the ends; returns their count (<= 256) */
static int orc_graded_breaks(double t0, double s, double* bp)
{
    double lo[128], hi[128];
    int nl = 0, nh = 0;
    for (double w = 0.25 * s; t0 - w > 0.0 && nl < 120; w *= 2.0) lo[nl++] = t0 - w;
    for (double w = 0.25 * s; t0 + w < 1.0 && nh < 120; w *= 2.0) hi[nh++] = t0 + w;
    int n = 0;
    bp[n++] = 0.0;
    for (int i = nl - 1; i >= 0; --i) bp[n++] = lo[i];
    if (t0 > 0.0 && t0 < 1.0) bp[n++] = t0;
    for (int i = 0; i < nh; ++i) bp[n++] = hi[i];
    bp[n++] = 1.0;
    return n;
}

void orc_tri_duffy(const double x[3], const double v1[3], const double v2[3], const double v3[3], double* S,
                   double F[3])
{
    double tu[ORC_DUFFY_NU], wu[ORC_DUFFY_NU], tv[ORC_DUFFY_NV], wv[ORC_DUFFY_NV];
    orc_gauss_legendre01(ORC_DUFFY_NU, tu, wu);
    orc_gauss_legendre01(ORC_DUFFY_NV, tv, wv);
    double c[3], xc[3];
    orc_closest_point(x, v1, v2, v3, c);
    sub3(x, c, xc);
    double d = norm3(xc);
    const double* v[3] = {v1, v2, v3};
    double e1[3], e2[3], tn[3];
    sub3(v2, v1, e1);
    sub3(v3, v1, e2);
    cross3(e1, e2, tn);
    double tarea2 = norm3(tn);
    /* x within rounding of the triangle (1e-14 of its size) is on it: the singular pair */
    if (d <= 1e-14 * sqrt(tarea2)) {
        d = 0.0;
        for (int k = 0; k < 3; ++k) c[k] = x[k];
    }
    double s = 0.0, f[3] = {0.0, 0.0, 0.0};
    double bu[260], bv[260];
    for (int e = 0; e < 3; ++e) {
        const double* a = v[e];
        const double* b = v[(e + 1) % 3];
        double pa[3], pb[3], cr[3], ab[3];
        sub3(a, c, pa);
        sub3(b, c, pb);
        sub3(b, a, ab);
        cross3(pa, pb, cr);
        double J = norm3(cr);
        if (J <= 1e-14 * tarea2) continue;   /* c on this edge: no piece */
        double L = norm3(pa), lab = norm3(ab);
        if (norm3(pb) > L) L = norm3(pb);
        if (lab > L) L = lab;
        /* u: towards the corner on the scale d / L (one interval when x is on the triangle) */
        int nu = 2;
        bu[0] = 0.0;
        bu[1] = 1.0;
        if (d > 0.0) nu = orc_graded_breaks(0.0, d / L, bu);
        /* v: towards the foot v* of the corner on the opposite edge, on the scale of the
         * corner's distance to it over the edge length (the factor 1/|dir(v)| of a narrow piece) */
        double vs = -dot3(pa, ab) / (lab * lab);
        if (vs < 0.0) vs = 0.0;
        if (vs > 1.0) vs = 1.0;
        double nv = orc_graded_breaks(vs, (J / lab) / lab, bv);
        for (int iu = 0; iu + 1 < nu; ++iu)
            for (int i = 0; i < ORC_DUFFY_NU; ++i) {
                double u = bu[iu] + (bu[iu + 1] - bu[iu]) * tu[i];
                double wuu = (bu[iu + 1] - bu[iu]) * wu[i];
                for (int iv = 0; iv + 1 < nv; ++iv)
                    for (int j = 0; j < ORC_DUFFY_NV; ++j) {
                        double vv = bv[iv] + (bv[iv + 1] - bv[iv]) * tv[j];
                        double wvv = (bv[iv + 1] - bv[iv]) * wv[j];
                        double y[3], r[3];
                        for (int k = 0; k < 3; ++k) y[k] = c[k] + u * ((1.0 - vv) * pa[k] + vv * pb[k]);
                        sub3(x, y, r);
                        double R = norm3(r);
                        double jw = u * J * wuu * wvv;
                        s += jw / R;
                        if (d > 0.0)
                            for (int k = 0; k < 3; ++k) f[k] += jw * r[k] / (R * R * R);
                    }
            }
    }
    *S = s / (4.0 * ORC_PI);
    for (int k = 0; k < 3; ++k) F[k] = (d > 0.0) ? f[k] / (4.0 * ORC_PI) : NAN;
}

/* ------------------------------------------- curved quadratic panels (Sec. 3, Sec. 4)
 * The paper's panels are curved triangles with a piecewise quadratic
 * parametrization (Sec. 3).  Reading: the image of the reference triangle
 * T = {(s, t): s, t >= 0, s + t <= 1} under the quadratic Lagrange map through
 * six nodes, the corners P1 = y(0,0), P2 = y(1,0), P3 = y(0,1) and the edge
 * nodes P4 = y(1/2,0), P5 = y(1/2,1/2), P6 = y(0,1/2):
 *   y(s,t) = sum_k N_k(s,t) P_k,  l1 = 1 - s - t, l2 = s, l3 = t,
 *   N1 = l1 (2 l1 - 1), N2 = l2 (2 l2 - 1), N3 = l3 (2 l3 - 1),
 *   N4 = 4 l1 l2, N5 = 4 l2 l3, N6 = 4 l3 l1,
 * with dS = |y_s x y_t| ds dt.  The near-singular rule of Sec. 4 on it, in the
 * paper's order, with every step taken in the parameter plane:
 *   1. the closest point: the parameter point c of T minimizing |x - y(s,t)|:
 *      the best of an interior minimum (Newton on the gradient of
 *      |x - y|^2 / 2 from the best of a 17 x 17 sampling, kept if it stays in
 *      T), the three edge minima (Newton along each edge from the best of 17
 *      samples, clipped to the edge) and the corners;
 *   2. pieces (c, a, b) of T for its edges a -> b, a piece of zero area
 *      (c on that edge) dropped;
 *   3. the Duffy map of a piece, (s, t) = c + u ((1 - v)(a - c) + v (b - c)),
 *      whose Jacobian u |det(a - c, b - c)| cancels the 1/r at the corner, times
 *      the surface Jacobian |y_s x y_t| at (s, t);
 *   4. the graded Gauss-Legendre rule of orc_tri_duffy, with the piece's
 *      edge vectors a - c, b - c, b - a taken through the tangent map
 *      (y_s, y_t) at c: near the corner the distance to x grows with the
 *      map's local metric there, not with the parameters (on a flat panel
 *      with mid-edge nodes at the edge midpoints the map is affine and this
 *      is orc_tri_duffy).
 * Unit density; S = (1/4pi) int 1/|x - y| dS, F = (1/4pi) int (x - y)/|x - y|^3 dS;
 * x on the panel (within 1e-14 of its size): S, and F = NaN. */
static void orc_quad_eval(const double P[6][3], double s, double t, double y[3], double ys[3], double yt[3],
                          double yss[3], double yst[3], double ytt[3])
{
    double l1 = 1.0 - s - t;
    /* N and its derivatives in s and t (dl1 = -ds - dt) */
    double N[6] = {l1 * (2.0 * l1 - 1.0), s * (2.0 * s - 1.0), t * (2.0 * t - 1.0), 4.0 * l1 * s, 4.0 * s * t,
                   4.0 * t * l1};
    double Ns[6] = {-(4.0 * l1 - 1.0), 4.0 * s - 1.0, 0.0, 4.0 * (l1 - s), 4.0 * t, -4.0 * t};
    double Nt[6] = {-(4.0 * l1 - 1.0), 0.0, 4.0 * t - 1.0, -4.0 * s, 4.0 * s, 4.0 * (l1 - t)};
    double Nss[6] = {4.0, 4.0, 0.0, -8.0, 0.0, 0.0};
    double Nst[6] = {4.0, 0.0, 0.0, -4.0, 4.0, -4.0};
    double Ntt[6] = {4.0, 0.0, 4.0, 0.0, 0.0, -8.0};
    for (int k = 0; k < 3; ++k) {
        y[k] = ys[k] = yt[k] = 0.0;
        if (yss) yss[k] = yst[k] = ytt[k] = 0.0;
        for (int m = 0; m < 6; ++m) {
            y[k] += N[m] * P[m][k];
            ys[k] += Ns[m] * P[m][k];
            yt[k] += Nt[m] * P[m][k];
            if (yss) {
                yss[k] += Nss[m] * P[m][k];
                yst[k] += Nst[m] * P[m][k];
                ytt[k] += Ntt[m] * P[m][k];
            }
        }
    }
}

static double orc_quad_dist2(const double P[6][3], const double x[3], double s, double t)
{
    double y[3], ys[3], yt[3], r[3];
    orc_quad_eval(P, s, t, y, ys, yt, NULL, NULL, NULL);
    sub3(y, x, r);
    return dot3(r, r);
}

void orc_quad_closest(const double P[6][3], const double x[3], double c[2])
{
    double best = INFINITY;
    /* corners */
    const double cs[3][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}};
    for (int k = 0; k < 3; ++k) {
        double d2 = orc_quad_dist2(P, x, cs[k][0], cs[k][1]);
        if (d2 < best) { best = d2; c[0] = cs[k][0]; c[1] = cs[k][1]; }
    }
    /* edges a -> b: (s, t) = a + tau (b - a) */
    for (int e = 0; e < 3; ++e) {
        const double* a = cs[e];
        const double* b = cs[(e + 1) % 3];
        double ds = b[0] - a[0], dt = b[1] - a[1], tau = 0.0, f0 = INFINITY;
        for (int i = 0; i <= 16; ++i) {
            double tt = i / 16.0, d2 = orc_quad_dist2(P, x, a[0] + tt * ds, a[1] + tt * dt);
            if (d2 < f0) { f0 = d2; tau = tt; }
        }
        for (int it = 0; it < 50; ++it) {
            double y[3], ys[3], yt[3], yss[3], yst[3], ytt[3], r[3], yd[3], ydd[3];
            orc_quad_eval(P, a[0] + tau * ds, a[1] + tau * dt, y, ys, yt, yss, yst, ytt);
            sub3(y, x, r);
            for (int k = 0; k < 3; ++k) {
                yd[k] = ys[k] * ds + yt[k] * dt;
                ydd[k] = yss[k] * ds * ds + 2.0 * yst[k] * ds * dt + ytt[k] * dt * dt;
            }
            double g = dot3(yd, r), h = dot3(yd, yd) + dot3(ydd, r);
            if (h <= 0.0) h = dot3(yd, yd);
            double nt = tau - g / h;
            if (nt < 0.0) nt = 0.0;
            if (nt > 1.0) nt = 1.0;
            double step = fabs(nt - tau);
            tau = nt;
            if (step <= 1e-16) break;
        }
        double d2 = orc_quad_dist2(P, x, a[0] + tau * ds, a[1] + tau * dt);
        if (d2 < best) { best = d2; c[0] = a[0] + tau * ds; c[1] = a[1] + tau * dt; }
    }
    /* interior: damped Newton on |x - y|^2 / 2 from the best sample, every step shortened to
     * stay in T and halved until the distance falls */
    double s = 0.0, t = 0.0, f0 = INFINITY;
    for (int i = 0; i <= 16; ++i)
        for (int j = 0; i + j <= 16; ++j) {
            double d2 = orc_quad_dist2(P, x, i / 16.0, j / 16.0);
            if (d2 < f0) { f0 = d2; s = i / 16.0; t = j / 16.0; }
        }
    for (int it = 0; it < 60; ++it) {
        double y[3], ys[3], yt[3], yss[3], yst[3], ytt[3], r[3];
        orc_quad_eval(P, s, t, y, ys, yt, yss, yst, ytt);
        sub3(y, x, r);
        double g0 = dot3(ys, r), g1 = dot3(yt, r);
        double h00 = dot3(ys, ys) + dot3(yss, r), h01 = dot3(ys, yt) + dot3(yst, r);
        double h11 = dot3(yt, yt) + dot3(ytt, r);
        double det = h00 * h11 - h01 * h01;
        if (!(h00 > 0.0 && det > 0.0)) {   /* Hessian not positive definite: Gauss-Newton */
            h00 = dot3(ys, ys);
            h01 = dot3(ys, yt);
            h11 = dot3(yt, yt);
            det = h00 * h11 - h01 * h01;
        }
        double d0 = -(h11 * g0 - h01 * g1) / det, d1 = -(h00 * g1 - h01 * g0) / det;
        /* the longest fraction of the step that stays in T */
        double a = 1.0;
        if (d0 < 0.0 && s + a * d0 < 0.0) a = -s / d0;
        if (d1 < 0.0 && t + a * d1 < 0.0) a = -t / d1;
        if (d0 + d1 > 0.0 && s + t + a * (d0 + d1) > 1.0) a = (1.0 - s - t) / (d0 + d1);
        double fn = INFINITY, sn = s, tn = t;
        for (int h = 0; h < 40; ++h, a *= 0.5) {
            sn = s + a * d0;
            tn = t + a * d1;
            if (sn < 0.0) sn = 0.0;
            if (tn < 0.0) tn = 0.0;
            if (sn + tn > 1.0) tn = 1.0 - sn;
            fn = orc_quad_dist2(P, x, sn, tn);
            if (fn <= f0) break;
        }
        if (!(fn <= f0)) break;   /* no decrease along the step: converged */
        double step = fabs(sn - s) + fabs(tn - t);
        s = sn;
        t = tn;
        f0 = fn;
        if (step <= 1e-16) break;
    }
    if (f0 < best) { best = f0; c[0] = s; c[1] = t; }
}

void orc_quad_duffy(const double x[3], const double* nodes /* [6][3] */, double* S, double F[3])
{
    double P[6][3];
    for (int m = 0; m < 6; ++m)
        for (int k = 0; k < 3; ++k) P[m][k] = nodes[3 * m + k];
    double tu[ORC_DUFFY_NU], wu[ORC_DUFFY_NU], tv[ORC_DUFFY_NV], wv[ORC_DUFFY_NV];
    orc_gauss_legendre01(ORC_DUFFY_NU, tu, wu);
    orc_gauss_legendre01(ORC_DUFFY_NV, tv, wv);
    double ch[2];
    orc_quad_closest(P, x, ch);
    double yc[3], ys[3], yt[3], yss[3], yst[3], ytt[3], xc[3];
    orc_quad_eval(P, ch[0], ch[1], yc, ys, yt, yss, yst, ytt);
    sub3(x, yc, xc);
    double d = norm3(xc);
    double size = 0.0;   /* the longest corner-to-corner chord */
    for (int k = 0; k < 3; ++k) {
        double e[3];
        sub3(P[(k + 1) % 3], P[k], e);
        if (norm3(e) > size) size = norm3(e);
    }
    if (d <= 1e-14 * size) d = 0.0;   /* on the panel: the singular pair */
    const double cs[3][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}};
    double s = 0.0, f[3] = {0.0, 0.0, 0.0};
    double bu[260], bv[260];
    for (int e = 0; e < 3; ++e) {
        const double* a = cs[e];
        const double* b = cs[(e + 1) % 3];
        double qa[2] = {a[0] - ch[0], a[1] - ch[1]}, qb[2] = {b[0] - ch[0], b[1] - ch[1]};
        double detp = qa[0] * qb[1] - qa[1] * qb[0];   /* > 0: T is counter-clockwise */
        if (detp <= 1e-14) continue;                   /* c on this edge: no piece */
        /* the piece's edge vectors through the tangent map at c: the scales of the grading */
        double pa[3], pb[3], ab[3], cr[3];
        for (int k = 0; k < 3; ++k) {
            pa[k] = ys[k] * qa[0] + yt[k] * qa[1];
            pb[k] = ys[k] * qb[0] + yt[k] * qb[1];
            ab[k] = pb[k] - pa[k];
        }
        cross3(pa, pb, cr);
        double Jc = norm3(cr), lab = norm3(ab), L = norm3(pa);
        if (norm3(pb) > L) L = norm3(pb);
        if (lab > L) L = lab;
        int nu = 2;
        bu[0] = 0.0;
        bu[1] = 1.0;
        if (d > 0.0) nu = orc_graded_breaks(0.0, d / L, bu);
        double vs = -dot3(pa, ab) / (lab * lab);
        if (vs < 0.0) vs = 0.0;
        if (vs > 1.0) vs = 1.0;
        int nv = orc_graded_breaks(vs, (Jc / lab) / lab, bv);
        for (int iu = 0; iu + 1 < nu; ++iu)
            for (int i = 0; i < ORC_DUFFY_NU; ++i) {
                double u = bu[iu] + (bu[iu + 1] - bu[iu]) * tu[i];
                double wuu = (bu[iu + 1] - bu[iu]) * wu[i];
                for (int iv = 0; iv + 1 < nv; ++iv)
                    for (int j = 0; j < ORC_DUFFY_NV; ++j) {
                        double vv = bv[iv] + (bv[iv + 1] - bv[iv]) * tv[j];
                        double wvv = (bv[iv + 1] - bv[iv]) * wv[j];
                        /* the node c + (ds, dt); y and its tangents there from c in exact
                         * Taylor form (the map is quadratic), so that x - y, short near the
                         * corner, is not the difference of two long vectors */
                        double dsn = u * ((1.0 - vv) * qa[0] + vv * qb[0]);
                        double dtn = u * ((1.0 - vv) * qa[1] + vv * qb[1]);
                        double dys[3], dyt[3], n[3], r[3];
                        for (int k = 0; k < 3; ++k) {
                            double dy = ys[k] * dsn + yt[k] * dtn +
                                        0.5 * (yss[k] * dsn * dsn + 2.0 * yst[k] * dsn * dtn + ytt[k] * dtn * dtn);
                            r[k] = xc[k] - dy;
                            dys[k] = ys[k] + yss[k] * dsn + yst[k] * dtn;
                            dyt[k] = yt[k] + yst[k] * dsn + ytt[k] * dtn;
                        }
                        cross3(dys, dyt, n);
                        double R = norm3(r);
                        double jw = u * detp * norm3(n) * wuu * wvv;
                        s += jw / R;
                        if (d > 0.0)
                            for (int k = 0; k < 3; ++k) f[k] += jw * r[k] / (R * R * R);
                    }
            }
    }
    *S = s / (4.0 * ORC_PI);
    for (int k = 0; k < 3; ++k) F[k] = (d > 0.0) ? f[k] / (4.0 * ORC_PI) : NAN;
}

/* ------------------------------------------------------------- problem geometry */
typedef struct {
    int64_t N;
    double* v;     /* [N][9] triangle vertices */
    double* cen;   /* [N][3] */
    double* nrm;   /* [N][3] */
    double* area;  /* [N] */
    double* cc;    /* [N][3] */
    double* R;     /* [N] */
    int32_t* fidx; /* [n_body] floating-body rank or -1 */
    int32_t n_float;
} orc_geom;

static void geom_build(const orc_problem* p, orc_geom* g)
{
    int64_t N = p->n_tri;
    g->N = N;
    g->v = (double*)malloc(sizeof(double) * 9 * N);
    g->cen = (double*)malloc(sizeof(double) * 3 * N);
    g->nrm = (double*)malloc(sizeof(double) * 3 * N);
    g->area = (double*)malloc(sizeof(double) * N);
    g->cc = (double*)malloc(sizeof(double) * 3 * N);
    g->R = (double*)malloc(sizeof(double) * N);
    for (int64_t j = 0; j < N; ++j) {
        for (int c = 0; c < 3; ++c)
            for (int k = 0; k < 3; ++k) g->v[9 * j + 3 * c + k] = p->vert[3 * (int64_t)p->tri[3 * j + c] + k];
        orc_panel_geometry(g->v + 9 * j, g->v + 9 * j + 3, g->v + 9 * j + 6, g->cen + 3 * j, g->nrm + 3 * j,
                           g->area + j, g->cc + 3 * j, g->R + j);
    }
    g->fidx = (int32_t*)malloc(sizeof(int32_t) * (p->n_body > 0 ? p->n_body : 1));
    g->n_float = 0;
    for (int32_t b = 0; b < p->n_body; ++b) g->fidx[b] = is_floating_kind(p->body_kind[b]) ? g->n_float++ : -1;
}

static void geom_free(orc_geom* g)
{
    free(g->v); free(g->cen); free(g->nrm); free(g->area); free(g->cc); free(g->R); free(g->fidx);
}

/* Sec. 4 classification: regular iff D > eta R with D the distance from x to
 * the circumcentre.  The triangle's own centroid (self) is always singular. */
static int pair_is_regular(const orc_problem* p, const orc_geom* g, const double x[3], int64_t j)
{
    double d[3];
    sub3(x, g->cc + 3 * j, d);
    return norm3(d) > p->eta * g->R[j];
}

/* Potential S and field F at x of triangle j with unit density.  self: x is
 * the centroid of j itself (principal value). */
static void pair_SF(const orc_problem* p, const orc_geom* g, const double x[3], int64_t j, int self,
                    double* S, double F[3])
{
    const double* v = g->v + 9 * j;
    if (!self && pair_is_regular(p, g, x, j))
        orc_tri_quad7(x, v, v + 3, v + 6, S, F);
    else
        orc_tri_analytic(x, v, v + 3, v + 6, self, S, F);
}

int64_t orc_n_unknowns(const orc_problem* p)
{
    int64_t n = p->n_tri;
    for (int32_t b = 0; b < p->n_body; ++b) n += is_floating_kind(p->body_kind[b]);
    return n;
}

/* Sec. 4 classification, exported for tests: 1 = regular, 0 = near or self. */
int orc_classify(const orc_problem* p, int64_t P, const double* pts, int32_t* regular)
{
    orc_geom g;
    geom_build(p, &g);
    for (int64_t i = 0; i < P; ++i)
        for (int64_t j = 0; j < p->n_tri; ++j) regular[i * p->n_tri + j] = pair_is_regular(p, &g, pts + 3 * i, j);
    geom_free(&g);
    return 0;
}

/* One row of the collocation system (Eqs. Final1-Final4), unknowns ordered
 * [sigma_1..sigma_N, V_1..V_Nfl], constraint rows last.
 *   conductor row i      : sum_j S_ij sigma_j                     (= V_body)
 *   floating row i in f  : sum_j S_ij sigma_j - V_f               (= 0)
 *   interface row i      : (eps+ + eps-)/2 sigma_i
 *                          + (eps+ - eps-) sum_{j != i} K'_ij sigma_j (= 0)
 *   constraint row of f  : sum_{i in f} a_i eps+ (sigma_i / 2 + sum_{j != i} K'_ij sigma_j)
 *                          scaled by 1/(eps+ sum_{i in f} a_i)    (= 0)
 *   constraint row of a sheet f (Eq. sheets):
 *                          sum_{i in f} a_i ((eps+ + eps-)/2 sigma_i
 *                                            + (eps+ - eps-) sum_{j != i} K'_ij sigma_j)
 *                          scaled by 1/((eps+ + eps-)/2 sum_{i in f} a_i)   (= 0)
 * with S_ij = S(x_i, tau_j) and K'_ij = n_i . F(x_i, tau_j).  The form
 * constraint_form = 1 replaces the constraint row of a closed floating body by
 * sum_{i in f} a_i sigma_i (same scaling), its value on a closed body by the
 * Gauss law; a sheet is not closed and always keeps Eq. sheets.
 */
static void assemble_row(const orc_problem* p, const orc_geom* g, int64_t row, double* out)
{
    int64_t N = p->n_tri, n = N + g->n_float;
    for (int64_t j = 0; j < n; ++j) out[j] = 0.0;
    if (row < N) {
        int64_t i = row;
        int32_t b = p->tri_body[i];
        int32_t kind = p->body_kind[b];
        const double* xi = g->cen + 3 * i;
        if (kind == ORC_DIRICHLET || is_floating_kind(kind)) {
            for (int64_t j = 0; j < N; ++j) {
                double S, F[3];
                pair_SF(p, g, xi, j, j == i, &S, F);
                out[j] = S;
            }
            if (is_floating_kind(kind)) out[N + g->fidx[b]] = -1.0;
        } else {
            double ep = p->eps_plus[b], em = p->eps_minus[b];
            for (int64_t j = 0; j < N; ++j) {
                if (j == i) {
                    out[j] = 0.5 * (ep + em);
                    continue;
                }
                double S, F[3];
                pair_SF(p, g, xi, j, 0, &S, F);
                out[j] = (ep - em) * dot3(g->nrm + 3 * i, F);
            }
        }
        return;
    }
    /* constraint row of floating body f */
    int32_t f = (int32_t)(row - N), fb = -1;
    for (int32_t b = 0; b < p->n_body; ++b)
        if (g->fidx[b] == f) fb = b;
    const int sheet = p->body_kind[fb] == ORC_SHEET;
    double ep = p->eps_plus[fb];
    /* coefficients of sigma_i and of (K' sigma)(x_i): eps+/2 and eps+ for a closed body (no
       field inside the metal), (eps+ + eps-)/2 and eps+ - eps- for a sheet */
    double c_self = sheet ? 0.5 * (ep + p->eps_minus[fb]) : 0.5 * ep;
    double c_kp = sheet ? ep - p->eps_minus[fb] : ep;
    double c_scale = sheet ? c_self : ep;
    double asum = 0.0;
    for (int64_t i = 0; i < N; ++i)
        if (p->tri_body[i] == fb) asum += g->area[i];
    double scale = 1.0 / (c_scale * asum);
    for (int64_t i = 0; i < N; ++i) {
        if (p->tri_body[i] != fb) continue;
        double ai = g->area[i];
        if (p->constraint_form == 1 && !sheet) {
            out[i] += scale * ep * ai;
            continue;
        }
        const double* xi = g->cen + 3 * i;
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) {
                out[j] += scale * ai * c_self;
                continue;
            }
            double S, F[3];
            pair_SF(p, g, xi, j, 0, &S, F);
            out[j] += scale * ai * c_kp * dot3(g->nrm + 3 * i, F);
        }
    }
}

/* Dense row-major system matrix, n x n with n = N + N_float. */
int orc_assemble(const orc_problem* p, double* A)
{
    orc_geom g;
    geom_build(p, &g);
    int64_t n = p->n_tri + g.n_float;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < n; ++r) assemble_row(p, &g, r, A + r * n);
    geom_free(&g);
    return 0;
}

/* Selected rows only (for checks at sizes where the full matrix is too big). */
int orc_assemble_rows(const orc_problem* p, int64_t n_rows, const int64_t* rows, double* out)
{
    orc_geom g;
    geom_build(p, &g);
    int64_t n = p->n_tri + g.n_float;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < n_rows; ++r) assemble_row(p, &g, rows[r], out + r * n);
    geom_free(&g);
    return 0;
}

/* Right-hand side: V of the body on conductor rows, 0 elsewhere. */
int orc_rhs(const orc_problem* p, const double* body_V, double* b)
{
    int64_t N = p->n_tri, n = orc_n_unknowns(p);
    for (int64_t r = 0; r < n; ++r) b[r] = 0.0;
    for (int64_t i = 0; i < N; ++i)
        if (p->body_kind[p->tri_body[i]] == ORC_DIRICHLET) b[i] = body_V[p->tri_body[i]];
    return 0;
}

/* ------------------------------------------------------------------ GMRES
 * Restarted GMRES(m) (Saad & Schultz 1986) with right diagonal (Jacobi)
 * preconditioning M = diag(A) (a zero diagonal entry is replaced by 1),
 * classical Gram-Schmidt applied twice, Givens rotations, zero initial guess,
 * stop when ||b - A x||_2 / ||b||_2 <= tol (checked on the true residual at
 * each restart, and on the Givens estimate inside a cycle).
 * Returns 0 on convergence, 1 otherwise; x holds the last iterate.
 */
static void matvec(int64_t n, const double* A, const double* x, double* y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        const double* a = A + i * n;
        for (int64_t j = 0; j < n; ++j) s += a[j] * x[j];
        y[i] = s;
    }
}

int orc_gmres(int64_t n, const double* A, const double* b, double tol, int32_t restart, int32_t max_iter,
              double* x, int32_t* iters_out, double* relres_out)
{
    int m = restart;
    double* d = (double*)malloc(sizeof(double) * n);
    double* V = (double*)malloc(sizeof(double) * n * (m + 1));
    double* H = (double*)calloc((size_t)(m + 1) * m, sizeof(double));
    double* cs = (double*)malloc(sizeof(double) * m);
    double* sn = (double*)malloc(sizeof(double) * m);
    double* g = (double*)malloc(sizeof(double) * (m + 1));
    double* y = (double*)malloc(sizeof(double) * (m + 1));
    double* z = (double*)malloc(sizeof(double) * n);
    double* w = (double*)malloc(sizeof(double) * n);
    double* h = (double*)malloc(sizeof(double) * (m + 1));
    for (int64_t i = 0; i < n; ++i) {
        d[i] = A[i * n + i];
        if (d[i] == 0.0) d[i] = 1.0;
        x[i] = 0.0;
    }
    double bnorm = 0.0;
    for (int64_t i = 0; i < n; ++i) bnorm += b[i] * b[i];
    bnorm = sqrt(bnorm);
    int iters = 0, converged = 0;
    double relres = 0.0;
    if (bnorm == 0.0) {
        converged = 1;
    } else {
        for (;;) {
            matvec(n, A, x, w);
            double beta = 0.0;
            for (int64_t i = 0; i < n; ++i) {
                w[i] = b[i] - w[i];
                beta += w[i] * w[i];
            }
            beta = sqrt(beta);
            relres = beta / bnorm;
            if (relres <= tol) { converged = 1; break; }
            if (iters >= max_iter) break;
            for (int64_t i = 0; i < n; ++i) V[i] = w[i] / beta;
            for (int k = 0; k <= m; ++k) g[k] = 0.0;
            g[0] = beta;
            memset(H, 0, sizeof(double) * (size_t)(m + 1) * m);
            int jend = 0;
            for (int j = 0; j < m; ++j) {
                for (int64_t i = 0; i < n; ++i) z[i] = V[j * n + i] / d[i];
                matvec(n, A, z, w);
                for (int pass = 0; pass < 2; ++pass) {
                    for (int k = 0; k <= j; ++k) {
                        double s = 0.0;
                        for (int64_t i = 0; i < n; ++i) s += V[k * n + i] * w[i];
                        h[k] = s;
                    }
                    for (int k = 0; k <= j; ++k) {
                        for (int64_t i = 0; i < n; ++i) w[i] -= h[k] * V[k * n + i];
                        H[k * m + j] += h[k];
                    }
                }
                double hn = 0.0;
                for (int64_t i = 0; i < n; ++i) hn += w[i] * w[i];
                hn = sqrt(hn);
                H[(j + 1) * m + j] = hn;
                if (hn > 0.0)
                    for (int64_t i = 0; i < n; ++i) V[(j + 1) * n + i] = w[i] / hn;
                for (int k = 0; k < j; ++k) {
                    double a = H[k * m + j], c = H[(k + 1) * m + j];
                    H[k * m + j] = cs[k] * a + sn[k] * c;
                    H[(k + 1) * m + j] = -sn[k] * a + cs[k] * c;
                }
                double a = H[j * m + j], c = H[(j + 1) * m + j];
                double r = sqrt(a * a + c * c);
                cs[j] = a / r;
                sn[j] = c / r;
                H[j * m + j] = r;
                H[(j + 1) * m + j] = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                ++iters;
                jend = j + 1;
                if (fabs(g[j + 1]) / bnorm <= tol || iters >= max_iter || hn == 0.0) break;
            }
            for (int k = jend - 1; k >= 0; --k) {
                double s = g[k];
                for (int q = k + 1; q < jend; ++q) s -= H[k * m + q] * y[q];
                y[k] = s / H[k * m + k];
            }
            for (int64_t i = 0; i < n; ++i) {
                double s = 0.0;
                for (int k = 0; k < jend; ++k) s += V[k * n + i] * y[k];
                x[i] += s / d[i];
            }
        }
    }
    *iters_out = iters;
    *relres_out = relres;
    free(d); free(V); free(H); free(cs); free(sn); free(g); free(y); free(z); free(w); free(h);
    return converged ? 0 : 1;
}

/* ------------------------------------------------------------- field evaluation
 * phi(x) = sum_j S_j(x) sigma_j and E(x) = sum_j F_j(x) sigma_j (field formula
 * closing Sec. 2).  on_panel[p] >= 0 marks x as the centroid of that panel:
 * the result is then the limit from the eps+ side, principal value plus
 * sigma_p n_p / 2 (the jump of the single-layer normal derivative, Eq. ADL).
 */
static void field_at(const orc_problem* p, const orc_geom* g, const double* sigma, const double x[3], int64_t op,
                     double* phi, double E[3])
{
    double ph = 0.0, e[3] = {0.0, 0.0, 0.0};
    for (int64_t j = 0; j < p->n_tri; ++j) {
        double S, F[3];
        pair_SF(p, g, x, j, j == op, &S, F);
        ph += S * sigma[j];
        for (int k = 0; k < 3; ++k) e[k] += F[k] * sigma[j];
    }
    if (op >= 0)
        for (int k = 0; k < 3; ++k) e[k] += 0.5 * sigma[op] * g->nrm[3 * op + k];
    *phi = ph;
    for (int k = 0; k < 3; ++k) E[k] = e[k];
}

int orc_eval(const orc_problem* p, const double* sigma, int64_t P, const double* pts, const int32_t* on_panel,
             double* phi, double* E)
{
    orc_geom g;
    geom_build(p, &g);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < P; ++i) {
        double ph, e[3];
        field_at(p, &g, sigma, pts + 3 * i, on_panel ? on_panel[i] : -1, &ph, e);
        if (phi) phi[i] = ph;
        for (int k = 0; k < 3; ++k) E[3 * i + k] = e[k];
    }
    geom_free(&g);
    return 0;
}

/* ------------------------------------------------ nodal linear basis (Sec. 3)
 * The paper's own discretisation: sigma_h = sum_k u_k psi_k with psi_k the
 * continuous piecewise-linear hat of vertex k (1 at x_k, 0 at every other
 * vertex, linear on each flat triangle), collocated at the vertices x_i.  The
 * entry of Eq. Matrix, v_ik = int psi_k(y) / (4 pi |x_i - y|) dS, collects over
 * the triangles tau that hold vertex k the integral of tau's barycentric
 * coordinate of k.
 *
 * Closed form of int_T lambda_k(y) / |x - y| dS on a flat triangle.  With rho
 * the projection of x on the plane, lambda_k is affine, so
 *   lambda_k(y) = lambda_k(rho) + g_k . (y - rho),
 *   g_k = n x (v_{k+2} - v_{k+1}) / (2 A)   (in-plane gradient of lambda_k),
 * and int lambda_k / R = lambda_k(rho) int 1/R + g_k . int (y - rho)/R.
 * int 1/R dS is the unit-density closed form above.  The in-plane gradient of
 * R = |x - y| is (y - rho)/R, so the divergence theorem in the plane gives
 *   int (y - rho)/R dS = sum_e m_e int_e R dl,
 *   int_e R dl = (s+ R+ - s- R- + R0^2 f_e) / 2     (edge notation as above).
 * on_plane (x is a vertex of T) forces w = 0 and rho = x; an edge that ends at
 * x then has t = R0 = 0, and its t f_e and R0^2 f_e terms vanish in the limit,
 * so they are dropped (f_e is infinite there).
 * out[k] = int lambda_k / (4 pi R) dS for the vertices in the order v1, v2, v3.
 */
void orc_tri_linear_analytic(const double x[3], const double v1[3], const double v2[3], const double v3[3],
                             int on_plane, double out[3])
{
    const double* v[3] = {v1, v2, v3};
    double e1[3], e2[3], cr[3], n[3];
    sub3(v2, v1, e1);
    sub3(v3, v1, e2);
    cross3(e1, e2, cr);
    double len = norm3(cr);   /* 2 A */
    for (int k = 0; k < 3; ++k) n[k] = cr[k] / len;
    double xv[3];
    sub3(x, v1, xv);
    double w = on_plane ? 0.0 : dot3(xv, n);
    double rho[3];
    for (int k = 0; k < 3; ++k) rho[k] = x[k] - w * n[k];
    double aw = fabs(w);
    double sum_tf = 0.0, sum_beta = 0.0, I1[3] = {0.0, 0.0, 0.0};
    for (int e = 0; e < 3; ++e) {
        const double* a = v[e];
        const double* b = v[(e + 1) % 3];
        double ab[3], l[3], m[3];
        sub3(b, a, ab);
        double lab = norm3(ab);
        for (int k = 0; k < 3; ++k) l[k] = ab[k] / lab;
        cross3(l, n, m);
        double ar[3], br[3], xa[3], xb[3];
        sub3(a, rho, ar);
        sub3(b, rho, br);
        double sm = dot3(ar, l), sp = dot3(br, l), t = dot3(ar, m);
        sub3(x, a, xa);
        sub3(x, b, xb);
        double Rm = norm3(xa), Rp = norm3(xb);
        double edge_R = 0.5 * (sp * Rp - sm * Rm);
        if (!(on_plane && (Rm == 0.0 || Rp == 0.0))) {
            double R02 = t * t + w * w;
            double f;
            if (sm < 0.0 && sp > 0.0)   /* foot within the edge's span: R- + s- = R0^2 / (R- - s-) */
                f = log((Rp + sp) * (Rm - sm) / R02);
            else if (sp + sm > 0.0)
                f = log((Rp + sp) / (Rm + sm));
            else
                f = log((Rm - sm) / (Rp - sp));
            double beta = atan2(t * sp, R02 + aw * Rp) - atan2(t * sm, R02 + aw * Rm);
            sum_tf += t * f;
            sum_beta += beta;
            edge_R += 0.5 * R02 * f;
        }
        for (int k = 0; k < 3; ++k) I1[k] += m[k] * edge_R;
    }
    double I0 = sum_tf - aw * sum_beta;
    for (int k = 0; k < 3; ++k) {
        const double* p1 = v[(k + 1) % 3];
        const double* p2 = v[(k + 2) % 3];
        double opp[3], g[3], r1[3], r2[3], c[3];
        sub3(p2, p1, opp);
        cross3(n, opp, g);
        sub3(p1, rho, r1);
        sub3(p2, rho, r2);
        cross3(r1, r2, c);
        double lam = dot3(c, n) / len;   /* barycentric coordinate of rho */
        out[k] = (lam * I0 + dot3(g, I1) / len) / (4.0 * ORC_PI);
    }
}

/* Field of the hats: out[k] = int lambda_k(y) (x - y) / (4 pi |x - y|^3) dS for
 * x off the triangle's plane or outside it (volume points).  With u = y - rho
 * (in-plane) and x - y = w n - u,
 *   int lambda_k (x - y)/R^3 = lambda_k(rho) F0 + w n (g_k . int u/R^3) - int (g_k . u) u/R^3,
 * F0 = int (x - y)/R^3 = sum_e m_e f_e + sign(w) n Omega (unit density, above), and
 * in-plane divergence identities with grad_u (1/R) = -u/R^3 and
 * grad_u ((g . u)/R) = g/R - (g . u) u/R^3:
 *   int u/R^3 dS = -sum_e m_e f_e,
 *   int (g . u) u/R^3 dS = g int 1/R dS - sum_e m_e int_e (g . u)/R dl,
 * where on edge e, u = t m_e + s l_e (s from s- to s+), so
 *   int_e (g . u)/R dl = t (g . m_e) f_e + (g . l_e)(R+ - R-).
 * (g_k is divided by 2A as in orc_tri_linear_analytic.) */
void orc_tri_linear_field(const double x[3], const double v1[3], const double v2[3], const double v3[3],
                          double out[3][3])
{
    const double* v[3] = {v1, v2, v3};
    double e1[3], e2[3], cr[3], n[3];
    sub3(v2, v1, e1);
    sub3(v3, v1, e2);
    cross3(e1, e2, cr);
    double len = norm3(cr);   /* 2 A */
    for (int k = 0; k < 3; ++k) n[k] = cr[k] / len;
    double xv[3];
    sub3(x, v1, xv);
    double w = dot3(xv, n);
    double rho[3];
    for (int k = 0; k < 3; ++k) rho[k] = x[k] - w * n[k];
    double aw = fabs(w);
    double sum_tf = 0.0, sum_beta = 0.0, mf[3] = {0.0, 0.0, 0.0};
    double f_e[3], t_e[3], dR_e[3], m_e[3][3], l_e[3][3];
    for (int e = 0; e < 3; ++e) {
        const double* a = v[e];
        const double* b = v[(e + 1) % 3];
        double ab[3], ar[3], br[3], xa[3], xb[3];
        sub3(b, a, ab);
        double lab = norm3(ab);
        for (int k = 0; k < 3; ++k) l_e[e][k] = ab[k] / lab;
        cross3(l_e[e], n, m_e[e]);
        sub3(a, rho, ar);
        sub3(b, rho, br);
        double sm = dot3(ar, l_e[e]), sp = dot3(br, l_e[e]), t = dot3(ar, m_e[e]);
        sub3(x, a, xa);
        sub3(x, b, xb);
        double Rm = norm3(xa), Rp = norm3(xb);
        double R02 = t * t + w * w;
        double f;
        if (sm < 0.0 && sp > 0.0)   /* foot within the edge's span: R- + s- = R0^2 / (R- - s-) */
            f = log((Rp + sp) * (Rm - sm) / R02);
        else if (sp + sm > 0.0)
            f = log((Rp + sp) / (Rm + sm));
        else
            f = log((Rm - sm) / (Rp - sp));
        double beta = atan2(t * sp, R02 + aw * Rp) - atan2(t * sm, R02 + aw * Rm);
        sum_tf += t * f;
        sum_beta += beta;
        for (int k = 0; k < 3; ++k) mf[k] += m_e[e][k] * f;
        f_e[e] = f;
        t_e[e] = t;
        dR_e[e] = Rp - Rm;
    }
    double sgn = (w > 0.0) ? 1.0 : ((w < 0.0) ? -1.0 : 0.0);
    double I0 = sum_tf - aw * sum_beta;
    double F0[3];
    for (int k = 0; k < 3; ++k) F0[k] = mf[k] + sgn * n[k] * sum_beta;
    for (int k = 0; k < 3; ++k) {
        const double* p1 = v[(k + 1) % 3];
        const double* p2 = v[(k + 2) % 3];
        double opp[3], g[3], r1[3], r2[3], c[3];
        sub3(p2, p1, opp);
        cross3(n, opp, g);
        for (int d = 0; d < 3; ++d) g[d] /= len;
        sub3(p1, rho, r1);
        sub3(p2, rho, r2);
        cross3(r1, r2, c);
        double lam = dot3(c, n) / len;
        double gu3 = -dot3(g, mf);                 /* g . int u/R^3 */
        double edge[3] = {0.0, 0.0, 0.0};          /* sum_e m_e int_e (g . u)/R dl */
        for (int e = 0; e < 3; ++e) {
            double ge = t_e[e] * dot3(g, m_e[e]) * f_e[e] + dot3(g, l_e[e]) * dR_e[e];
            for (int d = 0; d < 3; ++d) edge[d] += m_e[e][d] * ge;
        }
        for (int d = 0; d < 3; ++d)
            out[k][d] = (lam * F0[d] + w * n[d] * gu3 - (g[d] * I0 - edge[d])) / (4.0 * ORC_PI);
    }
}

/* Vertex -> body map of the nodal basis.  Returns 0, or -1 if a vertex is in
 * no triangle or in triangles of two bodies (the density of each body has its
 * own nodes; bodies that touch carry coincident vertices of their own). */
static int p1_vertex_body(const orc_problem* p, int32_t* vb)
{
    for (int64_t i = 0; i < p->n_vert; ++i) vb[i] = -1;
    for (int64_t j = 0; j < p->n_tri; ++j)
        for (int c = 0; c < 3; ++c) {
            int32_t k = p->tri[3 * j + c];
            if (vb[k] >= 0 && vb[k] != p->tri_body[j]) return -1;
            vb[k] = p->tri_body[j];
        }
    for (int64_t i = 0; i < p->n_vert; ++i)
        if (vb[i] < 0) return -1;
    return 0;
}

/* The three hat integrals of triangle j at x (Sec. 4 classification: the
 * 7-point rule with the rule's barycentric weights on regular pairs, the
 * closed form otherwise; a vertex of j is always singular). */
static void p1_pair(const orc_problem* p, const orc_geom* g, const double x[3], int64_t j, int is_vertex,
                    double c[3])
{
    const double* v = g->v + 9 * j;
    if (!is_vertex && pair_is_regular(p, g, x, j)) {
        double bary[7][3], wt[7];
        orc_quad7_rule(bary, wt);
        c[0] = c[1] = c[2] = 0.0;
        for (int q = 0; q < 7; ++q) {
            double y[3], d[3];
            for (int k = 0; k < 3; ++k) y[k] = bary[q][0] * v[k] + bary[q][1] * v[3 + k] + bary[q][2] * v[6 + k];
            sub3(x, y, d);
            double s = wt[q] * g->area[j] / (4.0 * ORC_PI) / norm3(d);
            for (int k = 0; k < 3; ++k) c[k] += s * bary[q][k];
        }
    } else {
        orc_tri_linear_analytic(x, v, v + 3, v + 6, is_vertex, c);
    }
}

/* The normal part at the centroid x_T of triangle T (normal n_T) of the field of
 * every hat, n_T . int lambda_k^j(y) (x_T - y) / (4 pi |x_T - y|^3) dS summed over the
 * triangles j != T, added with weight coef into row (the K' part, Eq. ADL, of a row
 * collocated at x_T).  T itself adds nothing: in its own plane the field of its
 * density has no normal component (principal value).  Regular pairs by the 7-point
 * rule with the hats at the nodes, the others by the closed form of the hat fields. */
static void p1_kp_centroid(const orc_problem* p, const orc_geom* g, int64_t T, double coef, double* row)
{
    const double* x = g->cen + 3 * T;
    const double* nT = g->nrm + 3 * T;
    double bary[7][3], wt[7];
    orc_quad7_rule(bary, wt);
    for (int64_t j = 0; j < p->n_tri; ++j) {
        if (j == T) continue;
        const int32_t* t = p->tri + 3 * j;
        const double* v = g->v + 9 * j;
        double Ek[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
        if (pair_is_regular(p, g, x, j)) {
            for (int q = 0; q < 7; ++q) {
                double y[3], d[3];
                for (int k = 0; k < 3; ++k) y[k] = bary[q][0] * v[k] + bary[q][1] * v[3 + k] + bary[q][2] * v[6 + k];
                sub3(x, y, d);
                double r = norm3(d);
                double s = wt[q] * g->area[j] / (4.0 * ORC_PI) / (r * r * r);
                for (int c = 0; c < 3; ++c)
                    for (int k = 0; k < 3; ++k) Ek[c][k] += s * bary[q][c] * d[k];
            }
        } else {
            orc_tri_linear_field(x, v, v + 3, v + 6, Ek);
        }
        for (int c = 0; c < 3; ++c) row[t[c]] += coef * dot3(nT, Ek[c]);
    }
}

/* Local corner of triangle j at vertex i: by index, or, for a vertex of another
 * body, by position (within 1e-13 of the triangle's longest edge); -1 if none. */
static int p1_corner(const orc_problem* p, const orc_geom* g, int64_t i, int64_t j)
{
    const int32_t* t = p->tri + 3 * j;
    for (int c = 0; c < 3; ++c)
        if (t[c] == i) return c;
    const double* v = g->v + 9 * j;
    const double* x = p->vert + 3 * i;
    double L = 0.0;
    for (int e = 0; e < 3; ++e) {
        double d[3];
        sub3(v + 3 * ((e + 1) % 3), v + 3 * e, d);
        if (norm3(d) > L) L = norm3(d);
    }
    for (int c = 0; c < 3; ++c) {
        double d[3];
        sub3(x, v + 3 * c, d);
        if (norm3(d) <= 1e-13 * L) return c;
    }
    return -1;
}

int64_t orc_p1_n_unknowns(const orc_problem* p)
{
    int32_t nf = 0;
    for (int32_t b = 0; b < p->n_body; ++b) nf += is_floating_kind(p->body_kind[b]);
    return p->n_vert + nf;
}

/* Dense row-major system of the nodal basis, n x n with n = n_vert + N_float,
 * unknowns [u_1..u_nvert, V_1..V_Nfl]:
 *   conductor vertex i     : sum_k v_ik u_k                 (= V_body)
 *   floating vertex i in f : sum_k v_ik u_k - V_f           (= 0)   (floating body or sheet)
 *   interface vertex i     : the hat-weighted mean over i's triangles T of the
 *       interface condition (Eq. nonconductors) at T's centroid x_T with T's normal,
 *       sum_T (a_T/3) [ (eps+ + eps-)/2 sigma_h(x_T) + (eps+ - eps-) (K' sigma_h)(x_T) ]
 *       / sum_T (a_T/3)                                     (= 0)
 *   row of floating body f : Eq. Final4 with the centroid rule over f's triangles,
 *       sum_T a_T [ c_self sigma_h(x_T) + c_kp (K' sigma_h)(x_T) ] / sum_T a_T (= 0),
 *       (c_self, c_kp) = (1/2, 1) (constraint_form 0, literal) or, for a sheet (Eq.
 *       sheets), (1, 2 (eps+ - eps-)/(eps+ + eps-)); constraint_form 1 for a closed
 *       floating body: its net charge sum_k u_k int_f psi_k / area_f.
 * sigma_h(x_T) = (u_a + u_b + u_c)/3.  A vertex has no normal on flat panels, so the
 * rows that need n . E (interface, Final4, sheets) take it at the centroids of the
 * triangles around the vertex or of the body; the potential rows stay at the vertex.
 * A vertex row meets the triangles of another body through a coincident vertex as
 * their vertex (the singular closed form, at that vertex's exact position). */
static void p1_row(const orc_problem* p, const orc_geom* g, const int32_t* vb, int64_t i, double* row)
{
    const int64_t nv = p->n_vert, n = orc_p1_n_unknowns(p);
    for (int64_t k = 0; k < n; ++k) row[k] = 0.0;
    if (i < nv) {
        const int32_t b = vb[i];
        const int32_t kind = p->body_kind[b];
        if (kind == ORC_INTERFACE) {
            const double ep = p->eps_plus[b], em = p->eps_minus[b];
            double W = 0.0;
            for (int64_t j = 0; j < p->n_tri; ++j) {
                const int32_t* t = p->tri + 3 * j;
                if (t[0] == i || t[1] == i || t[2] == i) W += g->area[j] / 3.0;
            }
            for (int64_t j = 0; j < p->n_tri; ++j) {
                const int32_t* t = p->tri + 3 * j;
                if (!(t[0] == i || t[1] == i || t[2] == i)) continue;
                const double wT = g->area[j] / 3.0 / W;
                for (int c = 0; c < 3; ++c) row[t[c]] += wT * 0.5 * (ep + em) / 3.0;
                p1_kp_centroid(p, g, j, wT * (ep - em), row);
            }
            return;
        }
        for (int64_t j = 0; j < p->n_tri; ++j) {
            const int32_t* t = p->tri + 3 * j;
            const int c0 = p1_corner(p, g, i, j);
            double c[3];
            /* at a coincident vertex of another body the closed form is taken at that vertex */
            p1_pair(p, g, c0 >= 0 ? g->v + 9 * j + 3 * c0 : p->vert + 3 * i, j, c0 >= 0, c);
            for (int k = 0; k < 3; ++k) row[t[k]] += c[k];
        }
        if (is_floating_kind(kind)) row[nv + g->fidx[b]] = -1.0;
        return;
    }
    int32_t b = 0;
    while (g->fidx[b] != i - nv) ++b;
    double asum = 0.0;
    for (int64_t j = 0; j < p->n_tri; ++j)
        if (p->tri_body[j] == b) asum += g->area[j];
    const int sheet = p->body_kind[b] == ORC_SHEET;
    if (!sheet && p->constraint_form == 1) {
        for (int64_t j = 0; j < p->n_tri; ++j)
            if (p->tri_body[j] == b)
                for (int k = 0; k < 3; ++k) row[p->tri[3 * j + k]] += g->area[j] / 3.0 / asum;
        return;
    }
    const double ep = p->eps_plus[b], em = p->eps_minus[b];
    const double c_self = sheet ? 1.0 : 0.5;
    const double c_kp = sheet ? 2.0 * (ep - em) / (ep + em) : 1.0;
    for (int64_t j = 0; j < p->n_tri; ++j) {
        if (p->tri_body[j] != b) continue;
        const double wT = g->area[j] / asum;
        for (int k = 0; k < 3; ++k) row[p->tri[3 * j + k]] += wT * c_self / 3.0;
        p1_kp_centroid(p, g, j, wT * c_kp, row);
    }
}

int orc_p1_assemble(const orc_problem* p, double* A)
{
    int32_t* vb = (int32_t*)malloc(sizeof(int32_t) * (p->n_vert > 0 ? p->n_vert : 1));
    int rc = p1_vertex_body(p, vb);
    if (rc != 0) {
        free(vb);
        return rc;
    }
    orc_geom g;
    geom_build(p, &g);
    const int64_t n = orc_p1_n_unknowns(p);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; ++i) p1_row(p, &g, vb, i, A + i * n);
    geom_free(&g);
    free(vb);
    return 0;
}

/* Selected rows of the nodal system (for checks at sizes where the full matrix is too big). */
int orc_p1_assemble_rows(const orc_problem* p, int64_t n_rows, const int64_t* rows, double* out)
{
    int32_t* vb = (int32_t*)malloc(sizeof(int32_t) * (p->n_vert > 0 ? p->n_vert : 1));
    int rc = p1_vertex_body(p, vb);
    if (rc != 0) {
        free(vb);
        return rc;
    }
    orc_geom g;
    geom_build(p, &g);
    const int64_t n = orc_p1_n_unknowns(p);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < n_rows; ++r) p1_row(p, &g, vb, rows[r], out + r * n);
    geom_free(&g);
    free(vb);
    return 0;
}

/* Right-hand side of the nodal system: V of the body on conductor vertex rows,
 * 0 elsewhere.  Returns as orc_p1_assemble. */
int orc_p1_rhs(const orc_problem* p, const double* body_V, double* b)
{
    int32_t* vb = (int32_t*)malloc(sizeof(int32_t) * (p->n_vert > 0 ? p->n_vert : 1));
    int rc = p1_vertex_body(p, vb);
    if (rc == 0) {
        const int64_t n = orc_p1_n_unknowns(p);
        for (int64_t i = 0; i < n; ++i) b[i] = 0.0;
        for (int64_t i = 0; i < p->n_vert; ++i)
            if (p->body_kind[vb[i]] == ORC_DIRICHLET) b[i] = body_V[vb[i]];
    }
    free(vb);
    return rc;
}

/* phi(x) = sum_k u_k int psi_k / (4 pi |x - y|) dS and E(x) = sum_k u_k
 * int psi_k (x - y) / (4 pi |x - y|^3) dS (the field formula closing Sec. 2) at
 * volume points (off the mesh), with the classification of the assembly:
 * regular pairs by the 7-point rule with the density at the nodes, the others
 * by the closed forms.  phi or E may be NULL. */
static void p1_field_at(const orc_problem* p, const orc_geom* g, const double* u, const double x[3], double* phi,
                        double E[3])
{
    double bary[7][3], wt[7];
    orc_quad7_rule(bary, wt);
    double s = 0.0, e[3] = {0.0, 0.0, 0.0};
    for (int64_t j = 0; j < p->n_tri; ++j) {
        const int32_t* t = p->tri + 3 * j;
        const double* v = g->v + 9 * j;
        if (pair_is_regular(p, g, x, j)) {
            for (int q = 0; q < 7; ++q) {
                double y[3], d[3];
                for (int k = 0; k < 3; ++k) y[k] = bary[q][0] * v[k] + bary[q][1] * v[3 + k] + bary[q][2] * v[6 + k];
                sub3(x, y, d);
                double r = norm3(d);
                double sig = bary[q][0] * u[t[0]] + bary[q][1] * u[t[1]] + bary[q][2] * u[t[2]];
                double c = wt[q] * g->area[j] / (4.0 * ORC_PI) * sig;
                s += c / r;
                for (int k = 0; k < 3; ++k) e[k] += c * d[k] / (r * r * r);
            }
        } else {
            double c[3], F[3][3];
            orc_tri_linear_analytic(x, v, v + 3, v + 6, 0, c);
            orc_tri_linear_field(x, v, v + 3, v + 6, F);
            for (int k = 0; k < 3; ++k) {
                s += c[k] * u[t[k]];
                for (int d = 0; d < 3; ++d) e[d] += F[k][d] * u[t[k]];
            }
        }
    }
    *phi = s;
    for (int k = 0; k < 3; ++k) E[k] = e[k];
}

int orc_p1_field(const orc_problem* p, const double* u, int64_t P, const double* pts, double* phi, double* E)
{
    orc_geom g;
    geom_build(p, &g);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < P; ++i) {
        double s, e[3];
        p1_field_at(p, &g, u, pts + 3 * i, &s, e);
        if (phi) phi[i] = s;
        if (E)
            for (int k = 0; k < 3; ++k) E[3 * i + k] = e[k];
    }
    geom_free(&g);
    return 0;
}

/* phi(x) = sum_k u_k int psi_k / (4 pi |x - y|) dS at points off the mesh
 * vertices (same classification as the assembly). */
int orc_p1_potential(const orc_problem* p, const double* u, int64_t P, const double* pts, double* phi)
{
    orc_geom g;
    geom_build(p, &g);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < P; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < p->n_tri; ++j) {
            const int32_t* t = p->tri + 3 * j;
            double c[3];
            p1_pair(p, &g, pts + 3 * i, j, 0, c);
            s += c[0] * u[t[0]] + c[1] * u[t[1]] + c[2] * u[t[2]];
        }
        phi[i] = s;
    }
    geom_free(&g);
    return 0;
}

/* ------------------------------------------------------------ segment hit test
 * Moeller-Trumbore (1997) ray/triangle test restricted to the closed segment
 * x0 -> x1 (t in [0,1]) and the closed triangle (u, v >= 0, u + v <= 1).  A
 * segment parallel to the triangle plane does not hit.  Among all hits the
 * smallest t wins, then the lowest panel index.  Returns the panel or -1.
 */
static int64_t segment_hit(const orc_problem* p, const orc_geom* g, const double x0[3], const double x1[3],
                           double* t_hit)
{
    double dir[3];
    sub3(x1, x0, dir);
    int64_t best = -1;
    double bt = 0.0;
    for (int64_t j = 0; j < p->n_tri; ++j) {
        const double* v = g->v + 9 * j;
        double e1[3], e2[3], pv[3], tv[3], qv[3];
        sub3(v + 3, v, e1);
        sub3(v + 6, v, e2);
        cross3(dir, e2, pv);
        double det = dot3(e1, pv);
        if (det == 0.0) continue;
        double inv = 1.0 / det;
        sub3(x0, v, tv);
        double u = dot3(tv, pv) * inv;
        if (u < 0.0 || u > 1.0) continue;
        cross3(tv, e1, qv);
        double vv = dot3(dir, qv) * inv;
        if (vv < 0.0 || u + vv > 1.0) continue;
        double t = dot3(e2, qv) * inv;
        if (t < 0.0 || t > 1.0) continue;
        if (best < 0 || t < bt) {
            best = j;
            bt = t;
        }
    }
    *t_hit = bt;
    return best;
}

int orc_segment_hit(const orc_problem* p, const double x0[3], const double x1[3], int64_t* panel, double* t)
{
    orc_geom g;
    geom_build(p, &g);
    *panel = segment_hit(p, &g, x0, x1, t);
    geom_free(&g);
    return 0;
}

/* --------------------------------------------------------- field lines + criterion
 * Field line dx/ds = dir E/|E| (Sec. 1: breakdown paths follow field lines),
 * classical RK4 with arc-length step h.  Before a step: |E(x_n)| < e_min stops
 * (code 4).  After a step: if the segment [x_n, x_{n+1}] hits a panel the step
 * is discarded and the line stops with that panel's kind (1 conductor,
 * 2 floating conductor, 3 dielectric interface).  max_steps accepted steps
 * stop with code 0; a non-finite field or position stops with code 5.
 * The streamer integral of Eq. Breakdowncrit, int alpha_eff(|E|) ds, is carried
 * as an extra RK4 state: I += h/6 (a1 + 2 a2 + 2 a3 + a4) with the alpha of the
 * four stage fields, alpha_eff(E) = alpha_a * max(E - alpha_e0, 0)^alpha_p.
 */
typedef void (*field_fn)(const void* ctx, const double x[3], double E[3]);
typedef int (*hit_fn)(const void* ctx, const double x0[3], const double x1[3]);

static double alpha_eff(const orc_trace_params* tp, double e)
{
    double d = e - tp->alpha_e0;
    if (d <= 0.0) return 0.0;
    return tp->alpha_a * pow(d, tp->alpha_p);
}

static void trace_one(const void* ctx, field_fn field, hit_fn hit, const orc_trace_params* tp, const double start[3],
                      int32_t* n_steps, int32_t* stop, double* integral, double* path)
{
    double x[3] = {start[0], start[1], start[2]};
    double I = 0.0, h = tp->h, dir = (tp->direction >= 0) ? 1.0 : -1.0;
    int32_t n = 0, code = 0;
    if (path)
        for (int k = 0; k < 3; ++k) path[k] = x[k];
    for (;;) {
        if (n >= tp->max_steps) { code = 0; break; }
        double E1[3], E2[3], E3[3], E4[3], k1[3], k2[3], k3[3], k4[3], y[3];
        field(ctx, x, E1);
        double m1 = norm3(E1);
        if (!isfinite(m1)) { code = 5; break; }
        if (m1 < tp->e_min) { code = 4; break; }
        for (int k = 0; k < 3; ++k) k1[k] = dir * E1[k] / m1;
        for (int k = 0; k < 3; ++k) y[k] = x[k] + 0.5 * h * k1[k];
        field(ctx, y, E2);
        double m2 = norm3(E2);
        for (int k = 0; k < 3; ++k) k2[k] = dir * E2[k] / m2;
        for (int k = 0; k < 3; ++k) y[k] = x[k] + 0.5 * h * k2[k];
        field(ctx, y, E3);
        double m3 = norm3(E3);
        for (int k = 0; k < 3; ++k) k3[k] = dir * E3[k] / m3;
        for (int k = 0; k < 3; ++k) y[k] = x[k] + h * k3[k];
        field(ctx, y, E4);
        double m4 = norm3(E4);
        for (int k = 0; k < 3; ++k) k4[k] = dir * E4[k] / m4;
        double xn[3];
        for (int k = 0; k < 3; ++k) xn[k] = x[k] + h / 6.0 * (k1[k] + 2.0 * k2[k] + 2.0 * k3[k] + k4[k]);
        if (!(isfinite(xn[0]) && isfinite(xn[1]) && isfinite(xn[2]))) { code = 5; break; }
        if (hit) {
            int c = hit(ctx, x, xn);
            if (c > 0) { code = c; break; }
        }
        I += h / 6.0 * (alpha_eff(tp, m1) + 2.0 * alpha_eff(tp, m2) + 2.0 * alpha_eff(tp, m3) + alpha_eff(tp, m4));
        for (int k = 0; k < 3; ++k) x[k] = xn[k];
        ++n;
        if (path)
            for (int k = 0; k < 3; ++k) path[3 * n + k] = x[k];
    }
    *n_steps = n;
    *stop = code;
    *integral = I;
}

typedef struct {
    const orc_problem* p;
    const orc_geom* g;
    const double* sigma;
} bem_field_ctx;

static void bem_field(const void* c, const double x[3], double E[3])
{
    const bem_field_ctx* b = (const bem_field_ctx*)c;
    double phi;
    field_at(b->p, b->g, b->sigma, x, -1, &phi, E);
}

static int bem_hit(const void* c, const double x0[3], const double x1[3])
{
    const bem_field_ctx* b = (const bem_field_ctx*)c;
    double t;
    int64_t j = segment_hit(b->p, b->g, x0, x1, &t);
    if (j < 0) return 0;
    int32_t kind = b->p->body_kind[b->p->tri_body[j]];
    return kind == ORC_DIRICHLET ? 1 : (is_floating_kind(kind) ? 2 : 3);
}

/* Field lines of the BEM field for sigma (first N entries of the solution). */
int orc_trace(const orc_problem* p, const double* sigma, int64_t L, const double* starts, const orc_trace_params* tp,
              int32_t* n_steps, int32_t* stop, double* integral, double* path)
{
    orc_geom g;
    geom_build(p, &g);
    bem_field_ctx c = {p, &g, sigma};
    int64_t stride = 3 * ((int64_t)tp->max_steps + 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t l = 0; l < L; ++l)
        trace_one(&c, bem_field, bem_hit, tp, starts + 3 * l, n_steps + l, stop + l, integral + l,
                  path ? path + l * stride : NULL);
    geom_free(&g);
    return 0;
}

/* Field lines of the nodal density u (Sec. 3 basis; the first n_vert entries of
 * the nodal solution): the same stepping, stops and integral as orc_trace, with
 * the field of orc_p1_field. */
static void p1_field_cb(const void* c, const double x[3], double E[3])
{
    const bem_field_ctx* b = (const bem_field_ctx*)c;
    double phi;
    p1_field_at(b->p, b->g, b->sigma, x, &phi, E);
}

int orc_p1_trace(const orc_problem* p, const double* u, int64_t L, const double* starts,
                 const orc_trace_params* tp, int32_t* n_steps, int32_t* stop, double* integral, double* path)
{
    orc_geom g;
    geom_build(p, &g);
    bem_field_ctx c = {p, &g, u};
    int64_t stride = 3 * ((int64_t)tp->max_steps + 1);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t l = 0; l < L; ++l)
        trace_one(&c, p1_field_cb, bem_hit, tp, starts + 3 * l, n_steps + l, stop + l, integral + l,
                  path ? path + l * stride : NULL);
    geom_free(&g);
    return 0;
}

/* Field lines of point charges E(x) = sum_k q_k (x - c_k)/|x - c_k|^3 with no
 * surfaces (a test harness for the RK4 stepping and the integral). */
typedef struct {
    int32_t n;
    const double* c;
    const double* q;
} charges_ctx;

static void charges_field(const void* cv, const double x[3], double E[3])
{
    const charges_ctx* c = (const charges_ctx*)cv;
    E[0] = E[1] = E[2] = 0.0;
    for (int32_t k = 0; k < c->n; ++k) {
        double d[3];
        sub3(x, c->c + 3 * k, d);
        double r = norm3(d);
        for (int i = 0; i < 3; ++i) E[i] += c->q[k] * d[i] / (r * r * r);
    }
}

int orc_trace_charges(int32_t n_charges, const double* centres, const double* charges, int64_t L,
                      const double* starts, const orc_trace_params* tp, int32_t* n_steps, int32_t* stop,
                      double* integral, double* path)
{
    charges_ctx c = {n_charges, centres, charges};
    int64_t stride = 3 * ((int64_t)tp->max_steps + 1);
    for (int64_t l = 0; l < L; ++l)
        trace_one(&c, charges_field, NULL, tp, starts + 3 * l, n_steps + l, stop + l, integral + l,
                  path ? path + l * stride : NULL);
    return 0;
}
