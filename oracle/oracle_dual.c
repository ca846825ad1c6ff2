/*
 * oracle_dual.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Directional derivative of the streamer integrals by forward-mode dual
 * numbers, for checking gradients of the GPU library.  A dual number
 * a + b eps (eps^2 = 0) carries a value and its derivative along one chosen
 * direction in parameter space: a perturbation dvert of every mesh vertex and
 * dbody_V of every body potential.  Every step of the method is redone here in
 * dual arithmetic, in the paper's order:
 *   - panel geometry (area, normal, centroid, quadrature nodes),
 *   - the collocation system of Eqs. Final1-Final4 with the 7-point rule for
 *     regular pairs and the flat-triangle closed forms for the others (Sec. 4),
 *   - the solve: A u = b gives u, and differentiating A u = b gives
 *     A du = db - dA u, solved with the same GMRES as the plain oracle,
 *   - RK4 field lines and the streamer integral of Eq. Breakdowncrit, with the
 *     line start moving with its panel: x0 = sum_k bary_k v_k + offset n.
 * The regular/near classification of every pair and each line's number of
 * accepted steps are held at their unperturbed values (the derivative of a
 * piecewise-smooth function on the piece that contains the point).  Nothing
 * here shares code with the GPU library, and nothing here is a reverse
 * (adjoint) sweep: it is an independent check of one.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ORC_SHEET: thin floating sheet, one (open) surface, constraint row of Eq. sheets */
enum { ORC_DIRICHLET = 0, ORC_FLOATING = 1, ORC_INTERFACE = 2, ORC_SHEET = 3 };
static int is_floating_kind(int32_t kind) { return kind == ORC_FLOATING || kind == ORC_SHEET; }

typedef struct {
    int64_t n_vert;
    const double* vert;
    int64_t n_tri;
    const int32_t* tri;
    const int32_t* tri_body;
    int32_t n_body;
    const int32_t* body_kind;
    const double* eps_plus;
    const double* eps_minus;
    double eta;
    int32_t constraint_form;
} orc_problem;

typedef struct {
    double h, e_min, start_offset;
    int32_t max_steps, direction;
    double alpha_a, alpha_e0, alpha_p, k_str;
} orc_trace_params;

/* plain-oracle routines reused as library steps */
void orc_panel_geometry(const double v1[3], const double v2[3], const double v3[3], double cen[3], double nrm[3],
                        double* area, double cc[3], double* R);
void orc_quad7_rule(double bary[7][3], double wt[7]);
int orc_gmres(int64_t n, const double* A, const double* b, double tol, int32_t restart, int32_t max_iter, double* x,
              int32_t* iters_out, double* relres_out);

/* ------------------------------------------------------------- dual numbers */
typedef struct {
    double v, d;
} dl;

static dl mk(double v, double d) { dl r = {v, d}; return r; }
static dl cst(double v) { return mk(v, 0.0); }
static dl add(dl a, dl b) { return mk(a.v + b.v, a.d + b.d); }
static dl sub(dl a, dl b) { return mk(a.v - b.v, a.d - b.d); }
static dl mul(dl a, dl b) { return mk(a.v * b.v, a.d * b.v + a.v * b.d); }
static dl scl(dl a, double s) { return mk(a.v * s, a.d * s); }
static dl dvd(dl a, dl b) { return mk(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
static dl dsqrt(dl a) { double s = sqrt(a.v); return mk(s, a.d / (2.0 * s)); }
static dl dlog(dl a) { return mk(log(a.v), a.d / a.v); }
static dl datan2(dl y, dl x) { return mk(atan2(y.v, x.v), (x.v * y.d - y.v * x.d) / (x.v * x.v + y.v * y.v)); }
static double sgn(double v) { return v > 0.0 ? 1.0 : (v < 0.0 ? -1.0 : 0.0); }
static dl dabs(dl a) { double s = sgn(a.v); return mk(s * a.v, s * a.d); }   /* slope 0 at 0 */

static void vsub(const dl a[3], const dl b[3], dl o[3]) { for (int k = 0; k < 3; ++k) o[k] = sub(a[k], b[k]); }
static dl vdot(const dl a[3], const dl b[3]) { return add(add(mul(a[0], b[0]), mul(a[1], b[1])), mul(a[2], b[2])); }
static void vcross(const dl a[3], const dl b[3], dl o[3])
{
    o[0] = sub(mul(a[1], b[2]), mul(a[2], b[1]));
    o[1] = sub(mul(a[2], b[0]), mul(a[0], b[2]));
    o[2] = sub(mul(a[0], b[1]), mul(a[1], b[0]));
}
static dl vnorm(const dl a[3]) { return dsqrt(vdot(a, a)); }

/* ------------------------------------------------------------ dual geometry
 * Per panel: dual vertices, centroid, unit normal and area; circumcentre and
 * circumradius only as values (they decide the frozen classification). */
typedef struct {
    int64_t N;
    dl* v;        /* [N][9] */
    dl* cen;      /* [N][3] */
    dl* nrm;      /* [N][3] */
    dl* area;     /* [N] */
    double* cc;   /* [N][3] values */
    double* R;    /* [N] values */
    int32_t* fidx;
    int32_t n_float;
} dgeom;

static void dgeom_build(const orc_problem* p, const double* dvert, dgeom* g)
{
    int64_t N = p->n_tri;
    g->N = N;
    g->v = (dl*)malloc(sizeof(dl) * 9 * N);
    g->cen = (dl*)malloc(sizeof(dl) * 3 * N);
    g->nrm = (dl*)malloc(sizeof(dl) * 3 * N);
    g->area = (dl*)malloc(sizeof(dl) * N);
    g->cc = (double*)malloc(sizeof(double) * 3 * N);
    g->R = (double*)malloc(sizeof(double) * N);
    for (int64_t j = 0; j < N; ++j) {
        dl* v = g->v + 9 * j;
        double vv[9];
        for (int c = 0; c < 3; ++c)
            for (int k = 0; k < 3; ++k) {
                int64_t idx = 3 * (int64_t)p->tri[3 * j + c] + k;
                v[3 * c + k] = mk(p->vert[idx], dvert ? dvert[idx] : 0.0);
                vv[3 * c + k] = p->vert[idx];
            }
        dl u[3], w[3], c[3];
        vsub(v + 3, v, u);
        vsub(v + 6, v, w);
        vcross(u, w, c);
        dl len = vnorm(c);
        g->area[j] = scl(len, 0.5);
        for (int k = 0; k < 3; ++k) {
            g->nrm[3 * j + k] = dvd(c[k], len);
            g->cen[3 * j + k] = scl(add(add(v[k], v[3 + k]), v[6 + k]), 1.0 / 3.0);
        }
        double cen[3], nrm[3], area;
        orc_panel_geometry(vv, vv + 3, vv + 6, cen, nrm, &area, g->cc + 3 * j, g->R + j);
    }
    g->fidx = (int32_t*)malloc(sizeof(int32_t) * (p->n_body > 0 ? p->n_body : 1));
    g->n_float = 0;
    for (int32_t b = 0; b < p->n_body; ++b) g->fidx[b] = is_floating_kind(p->body_kind[b]) ? g->n_float++ : -1;
}

static void dgeom_free(dgeom* g)
{
    free(g->v); free(g->cen); free(g->nrm); free(g->area); free(g->cc); free(g->R); free(g->fidx);
}

/* ------------------------------------------------------- dual pair integrals */
/* 7-point rule (regular pairs): S = sum_q w_q a / (4 pi r_q), F = sum_q w_q a d_q / (4 pi r_q^3). */
static void dquad7(const dl x[3], const dl* v, dl area, dl* S, dl F[3])
{
    double bary[7][3], wt[7];
    orc_quad7_rule(bary, wt);
    dl s = cst(0.0), f[3] = {cst(0.0), cst(0.0), cst(0.0)};
    for (int q = 0; q < 7; ++q) {
        dl y[3], d[3];
        for (int k = 0; k < 3; ++k)
            y[k] = add(add(scl(v[k], bary[q][0]), scl(v[3 + k], bary[q][1])), scl(v[6 + k], bary[q][2]));
        vsub(x, y, d);
        dl r = vnorm(d);
        dl c = scl(area, wt[q] / (4.0 * ORC_PI));
        s = add(s, dvd(c, r));
        dl r3 = mul(mul(r, r), r);
        for (int k = 0; k < 3; ++k) f[k] = add(f[k], dvd(mul(c, d[k]), r3));
    }
    *S = s;
    for (int k = 0; k < 3; ++k) F[k] = f[k];
}

/* Closed forms for a flat triangle of unit density (Wilton et al. 1984;
 * Graglia 1993), edge by edge: with w the height of x over the plane, rho its
 * foot point and, per edge a -> b, l the unit edge vector, m = l x n,
 * s-/s+ the abscissae of a/b, t the in-plane distance, R-/R+ the distances
 * from x to a/b:
 *   f_e = ln((R+ + s+)/(R- + s-))  (ln((R- - s-)/(R+ - s+)) if s+ + s- <= 0),
 *   beta_e = atan2(t s+, t^2 + w^2 + |w| R+) - atan2(t s-, t^2 + w^2 + |w| R-),
 *   4 pi S = sum t f_e - |w| sum beta_e,  4 pi F = sum m f_e + sign(w) n sum beta_e.
 * on_plane: x is the triangle's own centroid (principal value; w and sign(w)
 * are zero and stay zero when the triangle moves).  A point in the plane of the
 * triangle but outside it (coplanar panels) has w = 0 with a sum of angles that
 * vanishes like |w|: sign(w) sum beta and |w| sum beta are smooth in w there, and
 * their derivative is the one-sided one, taken by treating w as +0. */
static void danalytic(const dl x[3], const dl* v, int on_plane, dl* S, dl F[3])
{
    dl e1[3], e2[3], cr[3], n[3];
    vsub(v + 3, v, e1);
    vsub(v + 6, v, e2);
    vcross(e1, e2, cr);
    dl len = vnorm(cr);
    for (int k = 0; k < 3; ++k) n[k] = dvd(cr[k], len);
    dl xv[3];
    vsub(x, v, xv);
    dl w = on_plane ? cst(0.0) : vdot(xv, n);
    dl rho[3];
    for (int k = 0; k < 3; ++k) rho[k] = sub(x[k], mul(w, n[k]));
    dl aw = dabs(w);
    double s = sgn(w.v);
    if (!on_plane && w.v == 0.0) {
        aw = w;
        s = 1.0;
    }
    dl sum_tf = cst(0.0), sum_beta = cst(0.0), mf[3] = {cst(0.0), cst(0.0), cst(0.0)};
    for (int e = 0; e < 3; ++e) {
        const dl* a = v + 3 * e;
        const dl* b = v + 3 * ((e + 1) % 3);
        dl ab[3], l[3], m[3];
        vsub(b, a, ab);
        dl lab = vnorm(ab);
        for (int k = 0; k < 3; ++k) l[k] = dvd(ab[k], lab);
        vcross(l, n, m);
        dl ar[3], br[3], xa[3], xb[3];
        vsub(a, rho, ar);
        vsub(b, rho, br);
        dl sm = vdot(ar, l), sp = vdot(br, l), t = vdot(ar, m);
        vsub(x, a, xa);
        vsub(x, b, xb);
        dl Rm = vnorm(xa), Rp = vnorm(xb);
        dl R02 = add(mul(t, t), mul(w, w));
        dl f;
        if (sm.v < 0.0 && sp.v > 0.0)   /* foot within the edge's span: R- + s- = R0^2 / (R- - s-) */
            f = dlog(dvd(mul(add(Rp, sp), sub(Rm, sm)), R02));
        else if (sp.v + sm.v > 0.0)
            f = dlog(dvd(add(Rp, sp), add(Rm, sm)));
        else
            f = dlog(dvd(sub(Rm, sm), sub(Rp, sp)));
        dl beta = sub(datan2(mul(t, sp), add(R02, mul(aw, Rp))), datan2(mul(t, sm), add(R02, mul(aw, Rm))));
        sum_tf = add(sum_tf, mul(t, f));
        sum_beta = add(sum_beta, beta);
        for (int k = 0; k < 3; ++k) mf[k] = add(mf[k], mul(m[k], f));
    }
    *S = scl(sub(sum_tf, mul(aw, sum_beta)), 1.0 / (4.0 * ORC_PI));
    for (int k = 0; k < 3; ++k) F[k] = scl(add(mf[k], scl(mul(n[k], sum_beta), s)), 1.0 / (4.0 * ORC_PI));
}

/* Sec. 4 classification on the unperturbed values. */
static int dregular(const orc_problem* p, const dgeom* g, const dl x[3], int64_t j)
{
    double d0 = x[0].v - g->cc[3 * j], d1 = x[1].v - g->cc[3 * j + 1], d2 = x[2].v - g->cc[3 * j + 2];
    return sqrt(d0 * d0 + d1 * d1 + d2 * d2) > p->eta * g->R[j];
}

static void dpair(const orc_problem* p, const dgeom* g, const dl x[3], int64_t j, int self, dl* S, dl F[3])
{
    if (!self && dregular(p, g, x, j))
        dquad7(x, g->v + 9 * j, g->area[j], S, F);
    else
        danalytic(x, g->v + 9 * j, self, S, F);
}

/* ---------------------------------------------------------- dual system
 * Row r of Eqs. Final1-Final4 in dual arithmetic (values to Av, derivatives
 * to Ad), same rows and scaling as the plain oracle. */
static void dassemble_row(const orc_problem* p, const dgeom* g, int64_t row, double* Av, double* Ad)
{
    int64_t N = p->n_tri, n = N + g->n_float;
    for (int64_t j = 0; j < n; ++j) Av[j] = Ad[j] = 0.0;
    if (row < N) {
        int64_t i = row;
        int32_t b = p->tri_body[i];
        int32_t kind = p->body_kind[b];
        const dl* xi = g->cen + 3 * i;
        if (kind == ORC_DIRICHLET || is_floating_kind(kind)) {
            for (int64_t j = 0; j < N; ++j) {
                dl S, F[3];
                dpair(p, g, xi, j, j == i, &S, F);
                Av[j] = S.v;
                Ad[j] = S.d;
            }
            if (is_floating_kind(kind)) Av[N + g->fidx[b]] = -1.0;
        } else {
            double ep = p->eps_plus[b], em = p->eps_minus[b];
            for (int64_t j = 0; j < N; ++j) {
                if (j == i) {
                    Av[j] = 0.5 * (ep + em);
                    continue;
                }
                dl S, F[3];
                dpair(p, g, xi, j, 0, &S, F);
                dl v = scl(vdot(g->nrm + 3 * i, F), ep - em);
                Av[j] = v.v;
                Ad[j] = v.d;
            }
        }
        return;
    }
    int32_t f = (int32_t)(row - N), fb = -1;
    for (int32_t b = 0; b < p->n_body; ++b)
        if (g->fidx[b] == f) fb = b;
    /* (coefficient of sigma_i, of (K' sigma)_i) after the row scaling: a closed body's Eq. Final4
       over eps+ sum a gives (1/2, 1); a sheet's Eq. sheets over (eps+ + eps-)/2 sum a gives
       (1, 2 (eps+ - eps-) / (eps+ + eps-)), whatever constraint_form says */
    const int sheet = p->body_kind[fb] == ORC_SHEET;
    const double c_self = sheet ? 1.0 : 0.5;
    const double c_kp = sheet ? 2.0 * (p->eps_plus[fb] - p->eps_minus[fb]) / (p->eps_plus[fb] + p->eps_minus[fb]) : 1.0;
    dl asum = cst(0.0);
    for (int64_t i = 0; i < N; ++i)
        if (p->tri_body[i] == fb) asum = add(asum, g->area[i]);
    dl* acc = (dl*)malloc(sizeof(dl) * N);
    for (int64_t j = 0; j < N; ++j) acc[j] = cst(0.0);
    for (int64_t i = 0; i < N; ++i) {
        if (p->tri_body[i] != fb) continue;
        dl wi = dvd(g->area[i], asum);   /* a_i / sum a */
        if (p->constraint_form == 1 && !sheet) {
            acc[i] = add(acc[i], wi);
            continue;
        }
        const dl* xi = g->cen + 3 * i;
        for (int64_t j = 0; j < N; ++j) {
            if (j == i) {
                acc[j] = add(acc[j], scl(wi, c_self));
                continue;
            }
            dl S, F[3];
            dpair(p, g, xi, j, 0, &S, F);
            acc[j] = add(acc[j], scl(mul(wi, vdot(g->nrm + 3 * i, F)), c_kp));
        }
    }
    for (int64_t j = 0; j < N; ++j) {
        Av[j] = acc[j].v;
        Ad[j] = acc[j].d;
    }
    free(acc);
}

/* --------------------------------------------------------- dual field lines */
static void dfield(const orc_problem* p, const dgeom* g, const dl* sigma, const dl x[3], dl E[3])
{
    E[0] = E[1] = E[2] = cst(0.0);
    for (int64_t j = 0; j < p->n_tri; ++j) {
        dl S, F[3];
        dpair(p, g, x, j, 0, &S, F);
        for (int k = 0; k < 3; ++k) E[k] = add(E[k], mul(F[k], sigma[j]));
    }
}

static dl dalpha(const orc_trace_params* tp, dl e)
{
    double d = e.v - tp->alpha_e0;
    if (d <= 0.0) return cst(0.0);
    double v = tp->alpha_a * pow(d, tp->alpha_p);
    double dv = tp->alpha_a * tp->alpha_p * pow(d, tp->alpha_p - 1.0);
    return mk(v, dv * e.d);
}

/* ns accepted RK4 steps from x0 (Sec. 1; Eq. Breakdowncrit as an extra state). */
static dl dtrace_one(const orc_problem* p, const dgeom* g, const dl* sigma, const orc_trace_params* tp,
                     const dl x0[3], int32_t ns)
{
    dl x[3] = {x0[0], x0[1], x0[2]};
    dl I = cst(0.0);
    double h = tp->h, dir = (tp->direction >= 0) ? 1.0 : -1.0;
    for (int32_t n = 0; n < ns; ++n) {
        dl E[4][3], kk[4][3], m[4], y[3];
        double c[4] = {0.0, 0.5 * h, 0.5 * h, h};
        for (int s = 0; s < 4; ++s) {
            if (s == 0)
                for (int k = 0; k < 3; ++k) y[k] = x[k];
            else
                for (int k = 0; k < 3; ++k) y[k] = add(x[k], scl(kk[s - 1][k], c[s]));
            dfield(p, g, sigma, y, E[s]);
            m[s] = vnorm(E[s]);
            for (int k = 0; k < 3; ++k) kk[s][k] = scl(dvd(E[s][k], m[s]), dir);
        }
        for (int k = 0; k < 3; ++k)
            x[k] = add(x[k], scl(add(add(kk[0][k], scl(kk[1][k], 2.0)), add(scl(kk[2][k], 2.0), kk[3][k])),
                                 h / 6.0));
        dl a = add(add(dalpha(tp, m[0]), scl(dalpha(tp, m[1]), 2.0)),
                   add(scl(dalpha(tp, m[2]), 2.0), dalpha(tp, m[3])));
        I = add(I, scl(a, h / 6.0));
    }
    return I;
}

/* ------------------------------------------------------------ entry point
 * Streamer integrals I_l and their derivatives dI_l along the direction
 * (dvert [n_vert][3], dbody_V [n_body]).  The solution u solves A u = b(body_V)
 * and du solves A du = db - dA u (GMRES to tol).  Line l starts at
 * sum_k start_bary[l][k] v_k + start_offset n of panel start_panel[l] and takes
 * exactly n_steps[l] RK4 steps.  sigma_out / dsigma_out (n) may be NULL.
 * Returns 0, or 1 if a solve did not reach tol. */
int orc_dual_streamer(const orc_problem* p, const double* dvert, const double* body_V, const double* dbody_V,
                      int64_t L, const int32_t* start_panel, const double* start_bary, double start_offset,
                      const orc_trace_params* tp, const int32_t* n_steps, double tol, double* u_out, double* du_out,
                      double* I, double* dI)
{
    dgeom g;
    dgeom_build(p, dvert, &g);
    int64_t N = p->n_tri, n = N + g.n_float;
    double* Av = (double*)malloc(sizeof(double) * n * n);
    double* Ad = (double*)malloc(sizeof(double) * n * n);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < n; ++r) dassemble_row(p, &g, r, Av + r * n, Ad + r * n);
    double* b = (double*)calloc(n, sizeof(double));
    double* db = (double*)calloc(n, sizeof(double));
    for (int64_t i = 0; i < N; ++i)
        if (p->body_kind[p->tri_body[i]] == ORC_DIRICHLET) {
            b[i] = body_V[p->tri_body[i]];
            db[i] = dbody_V ? dbody_V[p->tri_body[i]] : 0.0;
        }
    double* u = (double*)malloc(sizeof(double) * n);
    double* du = (double*)malloc(sizeof(double) * n);
    int32_t it;
    double rr;
    int rc = orc_gmres(n, Av, b, tol, 100, 100000, u, &it, &rr);
    /* db - dA u */
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += Ad[i * n + j] * u[j];
        db[i] -= s;
    }
    int nz = 0;
    for (int64_t i = 0; i < n; ++i) nz |= (db[i] != 0.0);
    if (nz)
        rc |= orc_gmres(n, Av, db, tol, 100, 100000, du, &it, &rr);
    else
        for (int64_t i = 0; i < n; ++i) du[i] = 0.0;
    if (u_out) memcpy(u_out, u, sizeof(double) * n);
    if (du_out) memcpy(du_out, du, sizeof(double) * n);
    dl* sigma = (dl*)malloc(sizeof(dl) * N);
    for (int64_t j = 0; j < N; ++j) sigma[j] = mk(u[j], du[j]);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t l = 0; l < L; ++l) {
        const int64_t j = start_panel[l];
        const dl* v = g.v + 9 * j;
        dl x0[3];
        for (int k = 0; k < 3; ++k) {
            dl y = add(add(scl(v[k], start_bary[3 * l]), scl(v[3 + k], start_bary[3 * l + 1])),
                       scl(v[6 + k], start_bary[3 * l + 2]));
            x0[k] = add(y, scl(g.nrm[3 * j + k], start_offset));
        }
        dl r = dtrace_one(p, &g, sigma, tp, x0, n_steps[l]);
        I[l] = r.v;
        dI[l] = r.d;
    }
    free(sigma); free(u); free(du); free(b); free(db); free(Av); free(Ad);
    dgeom_free(&g);
    return rc;
}
