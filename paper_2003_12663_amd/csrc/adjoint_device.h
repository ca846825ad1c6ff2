// Device building blocks of the gradient of the streamer integrals: dual
// numbers with three derivative directions and the closed-form potential and
// field of a flat triangle written over them, so that one evaluation gives the
// value and its derivatives along three coordinates (of the field point, or of
// one triangle vertex).  The formulas are those of flat_tri_SF (Wilton et al.
// 1984 edge terms, Van Oosterom & Strackee 1983 solid angle), with the solid
// angle carried signed so that the derivative is right for points in the plane
// of the triangle but outside it; the normal is recomputed from the (possibly
// perturbed) vertices.
#pragma once

#include "bem_device.h"

namespace bem {

struct D3 {
    double v, d0, d1, d2;
};

__device__ __forceinline__ D3 d3(double v) { return {v, 0.0, 0.0, 0.0}; }
// value v varying along direction k (0..2) with slope s
__device__ __forceinline__ D3 d3seed(double v, int k, double s) {
    return {v, k == 0 ? s : 0.0, k == 1 ? s : 0.0, k == 2 ? s : 0.0};
}
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return {a.v + b.v, a.d0 + b.d0, a.d1 + b.d1, a.d2 + b.d2}; }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return {a.v - b.v, a.d0 - b.d0, a.d1 - b.d1, a.d2 - b.d2}; }
__device__ __forceinline__ D3 operator-(D3 a) { return {-a.v, -a.d0, -a.d1, -a.d2}; }
__device__ __forceinline__ D3 operator*(D3 a, double s) { return {a.v * s, a.d0 * s, a.d1 * s, a.d2 * s}; }
__device__ __forceinline__ D3 operator*(D3 a, D3 b) {
    return {a.v * b.v, a.d0 * b.v + a.v * b.d0, a.d1 * b.v + a.v * b.d1, a.d2 * b.v + a.v * b.d2};
}
__device__ __forceinline__ D3 operator/(D3 a, D3 b) {
    const double iv = 1.0 / b.v, q = a.v * iv;
    return {q, (a.d0 - q * b.d0) * iv, (a.d1 - q * b.d1) * iv, (a.d2 - q * b.d2) * iv};
}
__device__ __forceinline__ D3 dsqrt(D3 a) {
    const double s = sqrt(a.v), h = 0.5 / s;
    return {s, a.d0 * h, a.d1 * h, a.d2 * h};
}
__device__ __forceinline__ D3 dlog(D3 a) {
    const double iv = 1.0 / a.v;
    return {log(a.v), a.d0 * iv, a.d1 * iv, a.d2 * iv};
}
__device__ __forceinline__ D3 datan2(D3 y, D3 x) {
    const double iv = 1.0 / (x.v * x.v + y.v * y.v);
    return {atan2(y.v, x.v), (x.v * y.d0 - y.v * x.d0) * iv, (x.v * y.d1 - y.v * x.d1) * iv,
            (x.v * y.d2 - y.v * x.d2) * iv};
}

// S and F = -grad_x S of a flat triangle (vertices V[k][c]) with unit density at X.
// inplane: X is the triangle's own centroid (principal value, w = 0, sign(w) = 0).
__device__ __forceinline__ void tri_SF_d3(const D3 (&V)[3][3], const D3 (&X)[3], bool inplane, D3& S, D3 (&F)[3]) {
    const D3 e10 = V[1][0] - V[0][0], e11 = V[1][1] - V[0][1], e12 = V[1][2] - V[0][2];
    const D3 e20 = V[2][0] - V[0][0], e21 = V[2][1] - V[0][1], e22 = V[2][2] - V[0][2];
    const D3 c0 = e11 * e22 - e12 * e21, c1 = e12 * e20 - e10 * e22, c2 = e10 * e21 - e11 * e20;
    const D3 clen = dsqrt(c0 * c0 + c1 * c1 + c2 * c2);
    const D3 n0 = c0 / clen, n1 = c1 / clen, n2 = c2 / clen;
    const D3 w = inplane ? d3(0.0) : (X[0] - V[0][0]) * n0 + (X[1] - V[0][1]) * n1 + (X[2] - V[0][2]) * n2;
    const D3 r0 = X[0] - w * n0, r1 = X[1] - w * n1, r2 = X[2] - w * n2;
    D3 P[3][3], Rv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        P[k][0] = V[k][0] - X[0];
        P[k][1] = V[k][1] - X[1];
        P[k][2] = V[k][2] - X[2];
        Rv[k] = dsqrt(P[k][0] * P[k][0] + P[k][1] * P[k][1] + P[k][2] * P[k][2]);
    }
    D3 st = d3(0.0), m0s = d3(0.0), m1s = d3(0.0), m2s = d3(0.0);
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int b = (e + 1) % 3;
        D3 l0 = V[b][0] - V[e][0], l1 = V[b][1] - V[e][1], l2 = V[b][2] - V[e][2];
        const D3 len = dsqrt(l0 * l0 + l1 * l1 + l2 * l2);
        l0 = l0 / len;
        l1 = l1 / len;
        l2 = l2 / len;
        const D3 m0 = l1 * n2 - l2 * n1, m1 = l2 * n0 - l0 * n2, m2 = l0 * n1 - l1 * n0;
        const D3 q0 = V[e][0] - r0, q1 = V[e][1] - r1, q2 = V[e][2] - r2;
        const D3 sm = q0 * l0 + q1 * l1 + q2 * l2;
        const D3 sp = sm + len;
        const D3 t = q0 * m0 + q1 * m1 + q2 * m2;
        D3 f;
        if (sm.v < 0.0 && sp.v > 0.0)   // foot within the edge's span (see flat_tri_SF)
            f = dlog((Rv[b] + sp) * (Rv[e] - sm) / (t * t + w * w));
        else if (sp.v + sm.v > 0.0)
            f = dlog((Rv[b] + sp) / (Rv[e] + sm));
        else
            f = dlog((Rv[e] - sm) / (Rv[b] - sp));
        st = st + t * f;
        m0s = m0s + m0 * f;
        m1s = m1s + m1 * f;
        m2s = m2s + m2 * f;
    }
    // signed solid angle Omega_s = sign(w) Omega = 2 atan2(-[r1 r2 r3], den): the triple product
    // equals -2 a w for a flat triangle, so this is smooth across the plane outside the triangle
    // (coplanar panels, w = 0) and sign(w) / |w| are not needed: |w| Omega = w Omega_s
    D3 omega_s = d3(0.0);
    if (!inplane) {
        const D3 x0 = P[1][1] * P[2][2] - P[1][2] * P[2][1];
        const D3 x1 = P[1][2] * P[2][0] - P[1][0] * P[2][2];
        const D3 x2 = P[1][0] * P[2][1] - P[1][1] * P[2][0];
        const D3 triple = P[0][0] * x0 + P[0][1] * x1 + P[0][2] * x2;
        const D3 d01 = P[0][0] * P[1][0] + P[0][1] * P[1][1] + P[0][2] * P[1][2];
        const D3 d02 = P[0][0] * P[2][0] + P[0][1] * P[2][1] + P[0][2] * P[2][2];
        const D3 d12 = P[1][0] * P[2][0] + P[1][1] * P[2][1] + P[1][2] * P[2][2];
        const D3 den = Rv[0] * Rv[1] * Rv[2] + d01 * Rv[2] + d02 * Rv[1] + d12 * Rv[0];
        omega_s = datan2(-triple, den) * 2.0;
    }
    S = (st - w * omega_s) * INV4PI;
    F[0] = (m0s + omega_s * n0) * INV4PI;
    F[1] = (m1s + omega_s * n1) * INV4PI;
    F[2] = (m2s + omega_s * n2) * INV4PI;
}

// Field F and its Jacobian dF/dx (Jac[a][b] = dF_a/dx_b) at the point x of the
// triangle with the exact-geometry record T (vertices held fixed).
__device__ __forceinline__ void tri_F_dx(const double* __restrict__ T, double x0, double x1, double x2,
                                         double (&Fv)[3], double (&Jac)[3][3]) {
    D3 V[3][3], X[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) V[k][c] = d3(T[TR_V + 3 * k + c]);
    X[0] = d3seed(x0, 0, 1.0);
    X[1] = d3seed(x1, 1, 1.0);
    X[2] = d3seed(x2, 2, 1.0);
    D3 S, F[3];
    tri_SF_d3(V, X, false, S, F);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        Fv[a] = F[a].v;
        Jac[a][0] = F[a].d0;
        Jac[a][1] = F[a].d1;
        Jac[a][2] = F[a].d2;
    }
}

}  // namespace bem
