// The near-singular rule of Sec. 4 on the GPU: the point of the triangle
// closest to x is found, the triangle is cut into pieces that all have that
// point as a corner, and each piece is integrated after the Duffy
// transformation, which cancels the 1/r behaviour at the corner.
//   1. c = argmin over the closed triangle of |x - y|: the foot point of x in
//      the plane when it lies inside, else the nearest point of the edges.
//   2. pieces (c, a, b) for the edges a -> b; a piece of zero area (c on that
//      edge) is dropped.
//   3. y(u, v) = c + u ((1 - v)(a - c) + v (b - c)), dS = u |(a - c) x (b - c)| du dv.
//   4. tensor Gauss-Legendre (16 x 16 nodes per cell) on cells graded
//      geometrically: in u towards the corner from a quarter of d / L (d = |x - c|,
//      L the longest piece edge), in v towards the foot of the corner on the
//      opposite edge from a quarter of its distance to it over the edge length.
// The paper adapts its subdivision; the grading above is the fixed reading of
// that adaptivity this library uses (breakpoints t0 -+ (s/4) 2^k up to the ends).
// S = (1/4pi) int 1/|x - y| dS and F = (1/4pi) int (x - y)/|x - y|^3 dS for unit
// density.  A point on the triangle (within 1e-14 of its size) is the singular
// pair: the Duffy integrand of S is smooth there, while F is a principal value
// that the transformation does not produce (returned as NaN; a flat panel's own
// normal component is 0).
//
// k_duffy: one wave per (point, panel) pair; the wave walks the cells of a
// piece in step (cell bounds are wave-uniform, computed from their index) and
// each lane takes 4 of a cell's 256 nodes (its v node fixed, four u nodes), so
// no table is staged: a lane keeps its nodes in registers.  Lane sums are
// reduced over the wave at the end (fixed order).
// k_pair_closed: the closed forms of flat_tri_SF, one lane per pair.
#include <cmath>

#include "bem_device.h"

namespace bem {

namespace {

constexpr int DF_N = 16;          // Gauss-Legendre nodes per cell direction
constexpr int DF_MAXBRK = 120;    // graded breakpoints per side at most

struct GLRule {
    double t[DF_N], w[DF_N];   // nodes and weights on [0, 1]
};

// Graded breakpoints of [0, 1] towards t0 on the scale s: 0, t0 - (s/4) 2^k (descending k),
// t0 (if inside), t0 + (s/4) 2^k (ascending k), 1; at most DF_MAXBRK per side.
struct Graded {
    double t0, q;   // q = s / 4
    int nl, nh, mid, n;
    __device__ void init(double t0_, double s) {
        t0 = t0_;
        q = 0.25 * s;
        nl = 0;
        for (double w = q; t0 - w > 0.0 && nl < DF_MAXBRK; w *= 2.0) ++nl;
        nh = 0;
        for (double w = q; t0 + w < 1.0 && nh < DF_MAXBRK; w *= 2.0) ++nh;
        mid = (t0 > 0.0 && t0 < 1.0) ? 1 : 0;
        n = 2 + nl + mid + nh;
    }
    __device__ void unit() {
        t0 = 0.0;
        q = 0.0;
        nl = nh = mid = 0;
        n = 2;
    }
    // breakpoint m in 0 .. n - 1
    __device__ double at(int m) const {
        if (m == 0) return 0.0;
        if (m == n - 1) return 1.0;
        if (m <= nl) return t0 - ldexp(q, nl - m);
        if (mid && m == nl + 1) return t0;
        return t0 + ldexp(q, m - nl - 1 - mid);
    }
};

__device__ __forceinline__ void cross(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ double dot(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// point of the closed segment [a, b] closest to x
__device__ __forceinline__ void seg_closest(const double x[3], const double a[3], const double b[3], double c[3]) {
    const double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double ax[3] = {x[0] - a[0], x[1] - a[1], x[2] - a[2]};
    double t = dot(ax, ab) / dot(ab, ab);
    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
#pragma unroll
    for (int k = 0; k < 3; ++k) c[k] = a[k] + t * ab[k];
}

// point of the closed triangle v closest to x (step 1)
__device__ void tri_closest(const double x[3], const double v[3][3], double c[3]) {
    const double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
    const double e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
    double n[3];
    cross(e1, e2, n);
    const double xv[3] = {x[0] - v[0][0], x[1] - v[0][1], x[2] - v[0][2]};
    const double w = dot(xv, n) / dot(n, n);
    const double rho[3] = {x[0] - w * n[0], x[1] - w * n[1], x[2] - w * n[2]};
    bool inside = true;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const double* p = v[(e + 1) % 3];
        const double* q = v[(e + 2) % 3];
        const double pa[3] = {p[0] - rho[0], p[1] - rho[1], p[2] - rho[2]};
        const double pb[3] = {q[0] - rho[0], q[1] - rho[1], q[2] - rho[2]};
        double cr[3];
        cross(pa, pb, cr);
        if (dot(cr, n) < 0.0) inside = false;
    }
    if (inside) {
        c[0] = rho[0];
        c[1] = rho[1];
        c[2] = rho[2];
        return;
    }
    double best = INFINITY;
    for (int e = 0; e < 3; ++e) {
        double ce[3];
        seg_closest(x, v[e], v[(e + 1) % 3], ce);
        const double d[3] = {x[0] - ce[0], x[1] - ce[1], x[2] - ce[2]};
        const double dd = dot(d, d);
        if (dd < best) {
            best = dd;
            c[0] = ce[0];
            c[1] = ce[1];
            c[2] = ce[2];
        }
    }
}

// xrow: when not NULL, the point of pair p is the centroid of panel xrow[p] (pts unused)
__global__ __launch_bounds__(256) void k_duffy(int64_t P, const double* __restrict__ pts,
                                               const int32_t* __restrict__ xrow, const int32_t* __restrict__ panel,
                                               const double* __restrict__ tri64, GLRule gl, double* __restrict__ S,
                                               int64_t sstride, double* __restrict__ F, int64_t fstride) {
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= P) return;   // uniform over the wave
    const double* T = tri64 + (int64_t)TRI_REC * panel[p];
    double v[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) v[k][m] = T[TR_V + 3 * k + m];
    double x[3];
    if (xrow) {
        const double* Tx = tri64 + (int64_t)TRI_REC * xrow[p];
        x[0] = Tx[TR_C];
        x[1] = Tx[TR_C + 1];
        x[2] = Tx[TR_C + 2];
    } else {
        x[0] = pts[3 * p];
        x[1] = pts[3 * p + 1];
        x[2] = pts[3 * p + 2];
    }
    double c[3];
    tri_closest(x, v, c);
    double d = sqrt((x[0] - c[0]) * (x[0] - c[0]) + (x[1] - c[1]) * (x[1] - c[1]) + (x[2] - c[2]) * (x[2] - c[2]));
    const double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
    const double e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
    double tn[3];
    cross(e1, e2, tn);
    const double tarea2 = sqrt(dot(tn, tn));
    if (d <= 1e-14 * sqrt(tarea2)) {   // on the triangle: the singular pair
        d = 0.0;
        c[0] = x[0];
        c[1] = x[1];
        c[2] = x[2];
    }
    // this lane's nodes: v node j = lane % 16, u nodes i = lane / 16 + 4 k
    const int jn = lane & 15, in0 = lane >> 4;
    const double tvj = gl.t[jn], wvj = gl.w[jn];
    double tu[4], wu[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        tu[k] = gl.t[in0 + 4 * k];
        wu[k] = gl.w[in0 + 4 * k];
    }
    double s = 0.0, f0 = 0.0, f1 = 0.0, f2 = 0.0;
    for (int e = 0; e < 3; ++e) {
        const double* a = v[e];
        const double* b = v[(e + 1) % 3];
        const double pa[3] = {a[0] - c[0], a[1] - c[1], a[2] - c[2]};
        const double pb[3] = {b[0] - c[0], b[1] - c[1], b[2] - c[2]};
        const double ab[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double cr[3];
        cross(pa, pb, cr);
        const double J = sqrt(dot(cr, cr));
        if (J <= 1e-14 * tarea2) continue;   // c on this edge: no piece
        const double lab = sqrt(dot(ab, ab));
        double L = sqrt(dot(pa, pa));
        const double lb = sqrt(dot(pb, pb));
        if (lb > L) L = lb;
        if (lab > L) L = lab;
        Graded gu, gv;
        if (d > 0.0)
            gu.init(0.0, d / L);
        else
            gu.unit();
        double vs = -dot(pa, ab) / (lab * lab);
        vs = vs < 0.0 ? 0.0 : (vs > 1.0 ? 1.0 : vs);
        gv.init(vs, (J / lab) / lab);
        for (int iu = 0; iu + 1 < gu.n; ++iu) {
            const double u0 = gu.at(iu), du = gu.at(iu + 1) - u0;
            for (int iv = 0; iv + 1 < gv.n; ++iv) {
                const double v0 = gv.at(iv), dv = gv.at(iv + 1) - v0;
                const double vv = v0 + dv * tvj, wvv = dv * wvj;
                const double dir0 = (1.0 - vv) * pa[0] + vv * pb[0];
                const double dir1 = (1.0 - vv) * pa[1] + vv * pb[1];
                const double dir2 = (1.0 - vv) * pa[2] + vv * pb[2];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const double u = u0 + du * tu[k];
                    const double r0 = x[0] - (c[0] + u * dir0);
                    const double r1 = x[1] - (c[1] + u * dir1);
                    const double r2 = x[2] - (c[2] + u * dir2);
                    const double ir = rsqrt_pos(r0 * r0 + r1 * r1 + r2 * r2);
                    const double jw = u * J * (du * wu[k]) * wvv;
                    s += jw * ir;
                    const double t3 = jw * ir * ir * ir;
                    f0 += t3 * r0;
                    f1 += t3 * r1;
                    f2 += t3 * r2;
                }
            }
        }
    }
    s = wave_sum(s);
    f0 = wave_sum(f0);
    f1 = wave_sum(f1);
    f2 = wave_sum(f2);
    if (lane == 0) {
        S[p * sstride] = s * INV4PI;
        if (F) {
            const double nan = __builtin_nan("");
            F[p * fstride + 0] = d > 0.0 ? f0 * INV4PI : nan;
            F[p * fstride + 1] = d > 0.0 ? f1 * INV4PI : nan;
            F[p * fstride + 2] = d > 0.0 ? f2 * INV4PI : nan;
        }
    }
}

// closed forms, one lane per pair; a point on the triangle (within 1e-14 of its size of its
// plane and inside it) takes the principal value
__global__ __launch_bounds__(256) void k_pair_closed(int64_t P, const double* __restrict__ pts,
                                                     const int32_t* __restrict__ panel,
                                                     const double* __restrict__ tri64, double* __restrict__ S,
                                                     double* __restrict__ F, int64_t fstride) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const double* T = tri64 + (int64_t)TRI_REC * panel[p];
    double v[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int m = 0; m < 3; ++m) v[k][m] = T[TR_V + 3 * k + m];
    const double x[3] = {pts[3 * p], pts[3 * p + 1], pts[3 * p + 2]};
    double c[3];
    tri_closest(x, v, c);
    const double d = sqrt((x[0] - c[0]) * (x[0] - c[0]) + (x[1] - c[1]) * (x[1] - c[1]) + (x[2] - c[2]) * (x[2] - c[2]));
    const double on = d <= 1e-14 * sqrt(2.0 * T[TR_A]);
    double s, g0, g1, g2;
    flat_tri_SF<true, true>(T, x[0], x[1], x[2], on, s, g0, g1, g2);
    S[p] = s;
    if (F) {
        F[p * fstride + 0] = g0;
        F[p * fstride + 1] = g1;
        F[p * fstride + 2] = g2;
    }
}

// ---- curved quadratic panels (Sec. 3) ----------------------------------------
// A curved panel is the quadratic Lagrange map of the reference triangle
// {(s, t): s, t >= 0, s + t <= 1} through six nodes: corners P0 = y(0,0),
// P1 = y(1,0), P2 = y(0,1), edge nodes P3 = y(1/2,0), P4 = y(1/2,1/2), P5 = y(0,1/2).
// The rule of Sec. 4 runs in the parameter plane: the closest parameter point c
// (damped Newton on |x - y|^2 / 2 from the best of a 17 x 17 sampling, the three
// edge minima by Newton along each edge from 17 samples, the corners), pieces of
// the reference triangle with c as a corner, the Duffy map of each piece times
// the surface Jacobian |y_s x y_t|, and the graded cells of the flat rule with
// the piece's edge vectors taken through the tangent map at c.

struct QMap {
    double P[6][3];
    // y and its first (and, when ys2 != NULL, second) derivatives at (s, t)
    __device__ void eval(double s, double t, double y[3], double ys[3], double yt[3], double* ys2 = nullptr,
                         double* yst = nullptr, double* yt2 = nullptr) const {
        const double l1 = 1.0 - s - t;
        const double N[6] = {l1 * (2.0 * l1 - 1.0), s * (2.0 * s - 1.0), t * (2.0 * t - 1.0), 4.0 * l1 * s,
                             4.0 * s * t, 4.0 * t * l1};
        const double Ns[6] = {-(4.0 * l1 - 1.0), 4.0 * s - 1.0, 0.0, 4.0 * (l1 - s), 4.0 * t, -4.0 * t};
        const double Nt[6] = {-(4.0 * l1 - 1.0), 0.0, 4.0 * t - 1.0, -4.0 * s, 4.0 * s, 4.0 * (l1 - t)};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                a += N[m] * P[m][k];
                b += Ns[m] * P[m][k];
                c += Nt[m] * P[m][k];
            }
            y[k] = a;
            ys[k] = b;
            yt[k] = c;
            if (ys2) {   // constant second derivatives of the shape functions
                ys2[k] = 4.0 * P[0][k] + 4.0 * P[1][k] - 8.0 * P[3][k];
                yst[k] = 4.0 * P[0][k] - 4.0 * P[3][k] + 4.0 * P[4][k] - 4.0 * P[5][k];
                yt2[k] = 4.0 * P[0][k] + 4.0 * P[2][k] - 8.0 * P[5][k];
            }
        }
    }
    __device__ double dist2(const double x[3], double s, double t) const {
        double y[3], ys[3], yt[3];
        eval(s, t, y, ys, yt);
        const double r0 = y[0] - x[0], r1 = y[1] - x[1], r2 = y[2] - x[2];
        return r0 * r0 + r1 * r1 + r2 * r2;
    }
};

// closest parameter point of the panel to x (step 1); uniform over the wave
__device__ void quad_closest(const QMap& Q, const double x[3], double c[2]) {
    const double cs[3][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}};
    double best = INFINITY;
    for (int k = 0; k < 3; ++k) {
        const double d2 = Q.dist2(x, cs[k][0], cs[k][1]);
        if (d2 < best) {
            best = d2;
            c[0] = cs[k][0];
            c[1] = cs[k][1];
        }
    }
    for (int e = 0; e < 3; ++e) {   // edges a -> b
        const double a0 = cs[e][0], a1 = cs[e][1];
        const double ds = cs[(e + 1) % 3][0] - a0, dt = cs[(e + 1) % 3][1] - a1;
        double tau = 0.0, f0 = INFINITY;
        for (int i = 0; i <= 16; ++i) {
            const double tt = i / 16.0, d2 = Q.dist2(x, a0 + tt * ds, a1 + tt * dt);
            if (d2 < f0) {
                f0 = d2;
                tau = tt;
            }
        }
        for (int it = 0; it < 50; ++it) {
            double y[3], ys[3], yt[3], yss[3], yst[3], ytt[3];
            Q.eval(a0 + tau * ds, a1 + tau * dt, y, ys, yt, yss, yst, ytt);
            double g = 0.0, h1 = 0.0, h2 = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double r = y[k] - x[k];
                const double yd = ys[k] * ds + yt[k] * dt;
                const double ydd = yss[k] * ds * ds + 2.0 * yst[k] * ds * dt + ytt[k] * dt * dt;
                g += yd * r;
                h1 += yd * yd;
                h2 += ydd * r;
            }
            double h = h1 + h2;
            if (h <= 0.0) h = h1;
            double nt = tau - g / h;
            nt = nt < 0.0 ? 0.0 : (nt > 1.0 ? 1.0 : nt);
            const double step = fabs(nt - tau);
            tau = nt;
            if (step <= 1e-16) break;
        }
        const double d2 = Q.dist2(x, a0 + tau * ds, a1 + tau * dt);
        if (d2 < best) {
            best = d2;
            c[0] = a0 + tau * ds;
            c[1] = a1 + tau * dt;
        }
    }
    // interior: damped Newton from the best sample, steps kept in the triangle
    double s = 0.0, t = 0.0, f0 = INFINITY;
    for (int i = 0; i <= 16; ++i)
        for (int j = 0; i + j <= 16; ++j) {
            const double d2 = Q.dist2(x, i / 16.0, j / 16.0);
            if (d2 < f0) {
                f0 = d2;
                s = i / 16.0;
                t = j / 16.0;
            }
        }
    for (int it = 0; it < 60; ++it) {
        double y[3], ys[3], yt[3], yss[3], yst[3], ytt[3];
        Q.eval(s, t, y, ys, yt, yss, yst, ytt);
        double g0 = 0.0, g1 = 0.0, a00 = 0.0, a01 = 0.0, a11 = 0.0, b00 = 0.0, b01 = 0.0, b11 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double r = y[k] - x[k];
            g0 += ys[k] * r;
            g1 += yt[k] * r;
            a00 += ys[k] * ys[k];
            a01 += ys[k] * yt[k];
            a11 += yt[k] * yt[k];
            b00 += yss[k] * r;
            b01 += yst[k] * r;
            b11 += ytt[k] * r;
        }
        double h00 = a00 + b00, h01 = a01 + b01, h11 = a11 + b11;
        double det = h00 * h11 - h01 * h01;
        if (!(h00 > 0.0 && det > 0.0)) {   // not positive definite: Gauss-Newton
            h00 = a00;
            h01 = a01;
            h11 = a11;
            det = h00 * h11 - h01 * h01;
        }
        const double d0 = -(h11 * g0 - h01 * g1) / det, d1 = -(h00 * g1 - h01 * g0) / det;
        double al = 1.0;
        if (d0 < 0.0 && s + al * d0 < 0.0) al = -s / d0;
        if (d1 < 0.0 && t + al * d1 < 0.0) al = -t / d1;
        if (d0 + d1 > 0.0 && s + t + al * (d0 + d1) > 1.0) al = (1.0 - s - t) / (d0 + d1);
        double fn = INFINITY, sn = s, tn = t;
        for (int hh = 0; hh < 40; ++hh, al *= 0.5) {
            sn = s + al * d0;
            tn = t + al * d1;
            if (sn < 0.0) sn = 0.0;
            if (tn < 0.0) tn = 0.0;
            if (sn + tn > 1.0) tn = 1.0 - sn;
            fn = Q.dist2(x, sn, tn);
            if (fn <= f0) break;
        }
        if (!(fn <= f0)) break;
        const double step = fabs(sn - s) + fabs(tn - t);
        s = sn;
        t = tn;
        f0 = fn;
        if (step <= 1e-16) break;
    }
    if (f0 < best) {
        c[0] = s;
        c[1] = t;
    }
}

// one wave per (point, curved panel) pair; lanes take the cells' nodes as in k_duffy
__global__ __launch_bounds__(256) void k_quad_duffy(int64_t P, const double* __restrict__ pts,
                                                    const double* __restrict__ nodes, GLRule gl,
                                                    double* __restrict__ S, double* __restrict__ F) {
    const int lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= P) return;   // uniform over the wave
    QMap Q;
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
        for (int k = 0; k < 3; ++k) Q.P[m][k] = nodes[18 * p + 3 * m + k];
    const double x[3] = {pts[3 * p], pts[3 * p + 1], pts[3 * p + 2]};
    double ch[2];
    quad_closest(Q, x, ch);
    double yc[3], ys[3], yt[3], yss[3], yst[3], ytt[3];
    Q.eval(ch[0], ch[1], yc, ys, yt, yss, yst, ytt);
    const double xc[3] = {x[0] - yc[0], x[1] - yc[1], x[2] - yc[2]};
    double d = sqrt(dot(xc, xc));
    double size = 0.0;   // the longest corner-to-corner chord
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double e0 = Q.P[(k + 1) % 3][0] - Q.P[k][0], e1 = Q.P[(k + 1) % 3][1] - Q.P[k][1];
        const double e2 = Q.P[(k + 1) % 3][2] - Q.P[k][2];
        size = fmax(size, sqrt(e0 * e0 + e1 * e1 + e2 * e2));
    }
    if (d <= 1e-14 * size) d = 0.0;   // on the panel: the singular pair
    const int jn = lane & 15, in0 = lane >> 4;
    const double tvj = gl.t[jn], wvj = gl.w[jn];
    double tu[4], wu[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        tu[k] = gl.t[in0 + 4 * k];
        wu[k] = gl.w[in0 + 4 * k];
    }
    const double cs[3][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}};
    double sacc = 0.0, f0 = 0.0, f1 = 0.0, f2 = 0.0;
    for (int e = 0; e < 3; ++e) {
        const double qa0 = cs[e][0] - ch[0], qa1 = cs[e][1] - ch[1];
        const double qb0 = cs[(e + 1) % 3][0] - ch[0], qb1 = cs[(e + 1) % 3][1] - ch[1];
        const double detp = qa0 * qb1 - qa1 * qb0;   // > 0: counter-clockwise
        if (detp <= 1e-14) continue;                 // c on this edge: no piece
        double pa[3], pb[3], ab[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            pa[k] = ys[k] * qa0 + yt[k] * qa1;
            pb[k] = ys[k] * qb0 + yt[k] * qb1;
            ab[k] = pb[k] - pa[k];
        }
        double cr[3];
        cross(pa, pb, cr);
        const double Jc = sqrt(dot(cr, cr)), lab = sqrt(dot(ab, ab));
        double L = sqrt(dot(pa, pa));
        L = fmax(L, sqrt(dot(pb, pb)));
        L = fmax(L, lab);
        Graded gu, gv;
        if (d > 0.0)
            gu.init(0.0, d / L);
        else
            gu.unit();
        double vs = -dot(pa, ab) / (lab * lab);
        vs = vs < 0.0 ? 0.0 : (vs > 1.0 ? 1.0 : vs);
        gv.init(vs, (Jc / lab) / lab);
        for (int iu = 0; iu + 1 < gu.n; ++iu) {
            const double u0 = gu.at(iu), du = gu.at(iu + 1) - u0;
            for (int iv = 0; iv + 1 < gv.n; ++iv) {
                const double v0 = gv.at(iv), dv = gv.at(iv + 1) - v0;
                const double vv = v0 + dv * tvj, wvv = dv * wvj;
                const double dir0 = (1.0 - vv) * qa0 + vv * qb0, dir1 = (1.0 - vv) * qa1 + vv * qb1;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    // the node c + (ds, dt): x - y and the tangents there from c in exact Taylor
                    // form (the map is quadratic), so that x - y, short near the corner, is not
                    // the difference of two long vectors
                    const double u = u0 + du * tu[k];
                    const double dsn = u * dir0, dtn = u * dir1;
                    double r[3], dys[3], dyt[3], nv[3];
#pragma unroll
                    for (int m = 0; m < 3; ++m) {
                        const double dy = ys[m] * dsn + yt[m] * dtn +
                                          0.5 * (yss[m] * dsn * dsn + 2.0 * yst[m] * dsn * dtn + ytt[m] * dtn * dtn);
                        r[m] = xc[m] - dy;
                        dys[m] = ys[m] + yss[m] * dsn + yst[m] * dtn;
                        dyt[m] = yt[m] + yst[m] * dsn + ytt[m] * dtn;
                    }
                    cross(dys, dyt, nv);
                    const double r0 = r[0], r1 = r[1], r2 = r[2];
                    const double ir = rsqrt_pos(r0 * r0 + r1 * r1 + r2 * r2);
                    const double jw = u * detp * sqrt(dot(nv, nv)) * (du * wu[k]) * wvv;
                    sacc += jw * ir;
                    const double t3 = jw * ir * ir * ir;
                    f0 += t3 * r0;
                    f1 += t3 * r1;
                    f2 += t3 * r2;
                }
            }
        }
    }
    sacc = wave_sum(sacc);
    f0 = wave_sum(f0);
    f1 = wave_sum(f1);
    f2 = wave_sum(f2);
    if (lane == 0) {
        S[p] = sacc * INV4PI;
        if (F) {
            const double nan = __builtin_nan("");
            F[3 * p + 0] = d > 0.0 ? f0 * INV4PI : nan;
            F[3 * p + 1] = d > 0.0 ? f1 * INV4PI : nan;
            F[3 * p + 2] = d > 0.0 ? f2 * INV4PI : nan;
        }
    }
}

// n-point Gauss-Legendre rule on [0, 1]: the roots of P_n by Newton's method from the
// asymptotic guess cos(pi (i + 3/4) / (n + 1/2)), P_n and P_n' from the three-term recurrence;
// weight 1 / ((1 - z^2) P_n'(z)^2) on [0, 1].
GLRule make_gl16() {
    GLRule g;
    const int n = DF_N;
    for (int i = 0; i < n / 2; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 60; ++it) {
            double pm = 1.0, pc = z;   // P_0, P_1
            for (int k = 2; k <= n; ++k) {
                const double pn = ((2 * k - 1) * z * pc - (k - 1) * pm) / k;
                pm = pc;
                pc = pn;
            }
            dp = n * (pm - z * pc) / (1.0 - z * z);
            const double step = pc / dp;
            z -= step;
            if (std::fabs(step) <= 1e-17) break;
        }
        {
            double pm = 1.0, pc = z;
            for (int k = 2; k <= n; ++k) {
                const double pn = ((2 * k - 1) * z * pc - (k - 1) * pm) / k;
                pm = pc;
                pc = pn;
            }
            dp = n * (pm - z * pc) / (1.0 - z * z);
        }
        const double w = 1.0 / ((1.0 - z * z) * dp * dp);   // half of the [-1, 1] weight 2 / ...
        g.t[i] = 0.5 * (1.0 - z);
        g.t[n - 1 - i] = 0.5 * (1.0 + z);
        g.w[i] = w;
        g.w[n - 1 - i] = w;
    }
    return g;
}

}  // namespace

// S[p], F[p][0..3) (F row stride fstride; F may be NULL) of unit density on panel[p] at pts[p]:
// rule 0 closed forms, rule 1 the Sec. 4 near-singular rule.
void launch_pair_integrals(bem_ctx* c, int64_t P, const double* pts, const int32_t* panel, int rule, double* S,
                           double* F, int64_t fstride) {
    if (P == 0) return;
    KTimer t(c, rule ? "pair_duffy" : "pair_closed");
    if (rule == 0) {
        hipLaunchKernelGGL(k_pair_closed, dim3((unsigned)ceil_div(P, 256)), dim3(256), 0, c->stream, P, pts, panel,
                           c->tri64.as<double>(), S, F, fstride);
    } else {
        static const GLRule gl = make_gl16();
        hipLaunchKernelGGL(k_duffy, dim3((unsigned)ceil_div(P, 4)), dim3(256), 0, c->stream, P, pts,
                           (const int32_t*)nullptr, panel, c->tri64.as<double>(), gl, S, (int64_t)1, F, fstride);
    }
    BEM_CHECK_LAUNCH();
}

// S[p], F[p][0..3) (F may be NULL) of unit density on the curved quadratic panel nodes[p] (six
// nodes, [P][6][3]) at pts[p], by the Sec. 4 rule in the panel's parameter plane.
void launch_quad_pair_integrals(bem_ctx* c, int64_t P, const double* pts, const double* nodes, double* S,
                                double* F) {
    if (P == 0) return;
    KTimer t(c, "pair_quad");
    static const GLRule gl = make_gl16();
    hipLaunchKernelGGL(k_quad_duffy, dim3((unsigned)ceil_div(P, 4)), dim3(256), 0, c->stream, P, pts, nodes, gl, S,
                       F);
    BEM_CHECK_LAUNCH();
}

// The Sec. 4 rule for the assembly's near list: sf[4 k] = S and sf[4 k + 1 .. 4 k + 3] = F of
// panel col[k] at the centroid of panel row[k], k < nnz.
void launch_near_duffy(bem_ctx* c, int64_t nnz, const int32_t* row, const int32_t* col, double* sf) {
    if (nnz == 0) return;
    KTimer t(c, "near_duffy");
    static const GLRule gl = make_gl16();
    hipLaunchKernelGGL(k_duffy, dim3((unsigned)ceil_div(nnz, 4)), dim3(256), 0, c->stream, nnz,
                       (const double*)nullptr, row, col, c->tri64.as<double>(), gl, sf, (int64_t)4, sf + 1,
                       (int64_t)4);
    BEM_CHECK_LAUNCH();
}

}  // namespace bem
