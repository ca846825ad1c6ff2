// Closed form of the potential and field of a linear density on one flat
// triangle, used by the nodal-basis kernels (field evaluation and the near
// pairs of the field-line passes).
#pragma once

#include "bem_device.h"

namespace bem {

// Potential and field at a volume point x of the linear density on the flat
// triangle T with vertex values u0, u1, u2, added to phi and E.  With
// sigma(y) = sigma(rho) + G . (y - rho) (G the in-plane gradient of the
// density, sum_k u_k g_k) and x - y = w n - (y - rho):
//   4 pi phi = sigma(rho) int 1/R + G . int (y - rho)/R,
//   4 pi E   = sigma(rho) F0 - w n (G . sum_e m_e f_e)
//              - G int 1/R + sum_e m_e (t (G . m_e) f_e + (G . l_e)(R+ - R-)),
// F0 = sum_e m_e f_e + sign(w) n Omega the unit-density field; the last two
// terms are int (G . u) u / R^3 by the in-plane divergence identity
// grad_u ((G . u)/R) = G/R - (G . u) u/R^3, whose edge integrals are
// t (G . m) f_e + (G . l)(R+ - R-) for u = t m + s l.  Edge notation as in
// hat_edges; x must not lie on the triangle.
__device__ __forceinline__ void nodal_tri_phiE(const double* __restrict__ T, double x0, double x1, double x2,
                                               double u0, double u1, double u2, double& phi, double& E0, double& E1,
                                               double& E2) {
    const double n0 = T[TR_N + 0], n1 = T[TR_N + 1], n2 = T[TR_N + 2];
    const double two_area = 2.0 * T[TR_A];
    const double w = (x0 - T[0]) * n0 + (x1 - T[1]) * n1 + (x2 - T[2]) * n2;
    const double r0 = x0 - w * n0, r1 = x1 - w * n1, r2 = x2 - w * n2;
    const double aw = fabs(w);
    const double uk[3] = {u0, u1, u2};
    // sigma(rho) and G
    double srho = 0.0, G0 = 0.0, G1 = 0.0, G2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double* p = T + 3 * ((c + 1) % 3);
        const double* q = T + 3 * ((c + 2) % 3);
        const double a0 = p[0] - r0, a1 = p[1] - r1, a2 = p[2] - r2;
        const double b0 = q[0] - r0, b1 = q[1] - r1, b2 = q[2] - r2;
        srho += uk[c] * (n0 * (a1 * b2 - a2 * b1) + n1 * (a2 * b0 - a0 * b2) + n2 * (a0 * b1 - a1 * b0));
        const double e0 = q[0] - p[0], e1 = q[1] - p[1], e2 = q[2] - p[2];
        G0 += uk[c] * (n1 * e2 - n2 * e1);
        G1 += uk[c] * (n2 * e0 - n0 * e2);
        G2 += uk[c] * (n0 * e1 - n1 * e0);
    }
    srho /= two_area;
    G0 /= two_area; G1 /= two_area; G2 /= two_area;
    double V[3][3], Rv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        V[k][0] = T[3 * k] - x0;
        V[k][1] = T[3 * k + 1] - x1;
        V[k][2] = T[3 * k + 2] - x2;
        Rv[k] = sqrt(V[k][0] * V[k][0] + V[k][1] * V[k][1] + V[k][2] * V[k][2]);
    }
    double st = 0.0, mf0 = 0.0, mf1 = 0.0, mf2 = 0.0, J0 = 0.0, J1 = 0.0, J2 = 0.0, K0 = 0.0, K1 = 0.0, K2 = 0.0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int b = (e + 1) % 3;
        const double ax = T[3 * e], ay = T[3 * e + 1], az = T[3 * e + 2];
        double l0 = T[3 * b] - ax, l1 = T[3 * b + 1] - ay, l2 = T[3 * b + 2] - az;
        const double len = sqrt(l0 * l0 + l1 * l1 + l2 * l2);
        const double il = 1.0 / len;
        l0 *= il; l1 *= il; l2 *= il;
        const double m0 = l1 * n2 - l2 * n1, m1 = l2 * n0 - l0 * n2, m2 = l0 * n1 - l1 * n0;
        const double q0 = ax - r0, q1 = ay - r1, q2 = az - r2;
        const double sm = q0 * l0 + q1 * l1 + q2 * l2;
        const double sp = sm + len;
        const double t = q0 * m0 + q1 * m1 + q2 * m2;
        const double Rm = Rv[e], Rp = Rv[b];
        double f;
        if (sm < 0.0 && sp > 0.0)   // foot within the edge's span (see flat_tri_SF)
            f = log((Rp + sp) * (Rm - sm) / (t * t + w * w));
        else if (sp + sm > 0.0)
            f = log((Rp + sp) / (Rm + sm));
        else
            f = log((Rm - sm) / (Rp - sp));
        st += t * f;
        mf0 += m0 * f; mf1 += m1 * f; mf2 += m2 * f;
        const double er = 0.5 * (sp * Rp - sm * Rm + (t * t + w * w) * f);
        J0 += m0 * er; J1 += m1 * er; J2 += m2 * er;
        const double ge = t * (G0 * m0 + G1 * m1 + G2 * m2) * f + (G0 * l0 + G1 * l1 + G2 * l2) * (Rp - Rm);
        K0 += m0 * ge; K1 += m1 * ge; K2 += m2 * ge;
    }
    const double c0 = V[1][1] * V[2][2] - V[1][2] * V[2][1];
    const double c1 = V[1][2] * V[2][0] - V[1][0] * V[2][2];
    const double c2 = V[1][0] * V[2][1] - V[1][1] * V[2][0];
    const double triple = V[0][0] * c0 + V[0][1] * c1 + V[0][2] * c2;
    const double d01 = V[0][0] * V[1][0] + V[0][1] * V[1][1] + V[0][2] * V[1][2];
    const double d02 = V[0][0] * V[2][0] + V[0][1] * V[2][1] + V[0][2] * V[2][2];
    const double d12 = V[1][0] * V[2][0] + V[1][1] * V[2][1] + V[1][2] * V[2][2];
    const double den = Rv[0] * Rv[1] * Rv[2] + d01 * Rv[2] + d02 * Rv[1] + d12 * Rv[0];
    const double omega = 2.0 * atan2(fabs(triple), den);
    const double I0 = st - aw * omega;
    const double sg = (w > 0.0) ? omega : ((w < 0.0) ? -omega : 0.0);
    const double Gmf = G0 * mf0 + G1 * mf1 + G2 * mf2;
    phi += (srho * I0 + G0 * J0 + G1 * J1 + G2 * J2) * INV4PI;
    E0 += (srho * (mf0 + sg * n0) - w * n0 * Gmf - G0 * I0 + K0) * INV4PI;
    E1 += (srho * (mf1 + sg * n1) - w * n1 * Gmf - G1 * I0 + K1) * INV4PI;
    E2 += (srho * (mf2 + sg * n2) - w * n2 * Gmf - G2 * I0 + K2) * INV4PI;
}

// The normal part at x (unit normal nx) of the field of each hat of the flat
// triangle T, out[c] += nx . int lambda_c(y) (x - y) / (4 pi |x - y|^3) dS, for x off
// T (not on its closed surface).  Per hat c the density is lambda_c: sigma(rho) =
// lambda_c(rho), G = g_c, in the terms of nodal_tri_phiE, whose edge quantities the
// three hats share.
__device__ __forceinline__ void nodal_tri_hats_nE(const double* __restrict__ T, double x0, double x1, double x2,
                                                  double nx0, double nx1, double nx2, double (&out)[3]) {
    const double n0 = T[TR_N + 0], n1 = T[TR_N + 1], n2 = T[TR_N + 2];
    const double two_area = 2.0 * T[TR_A];
    const double w = (x0 - T[0]) * n0 + (x1 - T[1]) * n1 + (x2 - T[2]) * n2;
    const double r0 = x0 - w * n0, r1 = x1 - w * n1, r2 = x2 - w * n2;
    const double aw = fabs(w);
    double lam[3], g[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double* p = T + 3 * ((c + 1) % 3);
        const double* q = T + 3 * ((c + 2) % 3);
        const double a0 = p[0] - r0, a1 = p[1] - r1, a2 = p[2] - r2;
        const double b0 = q[0] - r0, b1 = q[1] - r1, b2 = q[2] - r2;
        lam[c] = (n0 * (a1 * b2 - a2 * b1) + n1 * (a2 * b0 - a0 * b2) + n2 * (a0 * b1 - a1 * b0)) / two_area;
        const double e0 = q[0] - p[0], e1 = q[1] - p[1], e2 = q[2] - p[2];
        g[c][0] = (n1 * e2 - n2 * e1) / two_area;
        g[c][1] = (n2 * e0 - n0 * e2) / two_area;
        g[c][2] = (n0 * e1 - n1 * e0) / two_area;
    }
    double V[3][3], Rv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        V[k][0] = T[3 * k] - x0;
        V[k][1] = T[3 * k + 1] - x1;
        V[k][2] = T[3 * k + 2] - x2;
        Rv[k] = sqrt(V[k][0] * V[k][0] + V[k][1] * V[k][1] + V[k][2] * V[k][2]);
    }
    // per edge: f_e, t_e, R+ - R-, and the unit vectors m_e, l_e
    double st = 0.0, mf0 = 0.0, mf1 = 0.0, mf2 = 0.0;
    double fe[3], te[3], dR[3], me[3][3], le[3][3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int b = (e + 1) % 3;
        const double ax = T[3 * e], ay = T[3 * e + 1], az = T[3 * e + 2];
        double l0 = T[3 * b] - ax, l1 = T[3 * b + 1] - ay, l2 = T[3 * b + 2] - az;
        const double len = sqrt(l0 * l0 + l1 * l1 + l2 * l2);
        const double il = 1.0 / len;
        l0 *= il; l1 *= il; l2 *= il;
        const double m0 = l1 * n2 - l2 * n1, m1 = l2 * n0 - l0 * n2, m2 = l0 * n1 - l1 * n0;
        const double q0 = ax - r0, q1 = ay - r1, q2 = az - r2;
        const double sm = q0 * l0 + q1 * l1 + q2 * l2;
        const double sp = sm + len;
        const double t = q0 * m0 + q1 * m1 + q2 * m2;
        const double Rm = Rv[e], Rp = Rv[b];
        double f;
        if (sm < 0.0 && sp > 0.0)   // foot within the edge's span (see flat_tri_SF)
            f = log((Rp + sp) * (Rm - sm) / (t * t + w * w));
        else if (sp + sm > 0.0)
            f = log((Rp + sp) / (Rm + sm));
        else
            f = log((Rm - sm) / (Rp - sp));
        st += t * f;
        mf0 += m0 * f; mf1 += m1 * f; mf2 += m2 * f;
        fe[e] = f;
        te[e] = t;
        dR[e] = Rp - Rm;
        me[e][0] = m0; me[e][1] = m1; me[e][2] = m2;
        le[e][0] = l0; le[e][1] = l1; le[e][2] = l2;
    }
    const double c0 = V[1][1] * V[2][2] - V[1][2] * V[2][1];
    const double c1 = V[1][2] * V[2][0] - V[1][0] * V[2][2];
    const double c2 = V[1][0] * V[2][1] - V[1][1] * V[2][0];
    const double triple = V[0][0] * c0 + V[0][1] * c1 + V[0][2] * c2;
    const double d01 = V[0][0] * V[1][0] + V[0][1] * V[1][1] + V[0][2] * V[1][2];
    const double d02 = V[0][0] * V[2][0] + V[0][1] * V[2][1] + V[0][2] * V[2][2];
    const double d12 = V[1][0] * V[2][0] + V[1][1] * V[2][1] + V[1][2] * V[2][2];
    const double den = Rv[0] * Rv[1] * Rv[2] + d01 * Rv[2] + d02 * Rv[1] + d12 * Rv[0];
    const double omega = 2.0 * atan2(fabs(triple), den);
    const double I0 = st - aw * omega;
    const double sg = (w > 0.0) ? omega : ((w < 0.0) ? -omega : 0.0);
    // nx . F0, nx . n and nx . m_e
    const double nF0 = nx0 * (mf0 + sg * n0) + nx1 * (mf1 + sg * n1) + nx2 * (mf2 + sg * n2);
    const double nn = nx0 * n0 + nx1 * n1 + nx2 * n2;
    double nme[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) nme[e] = nx0 * me[e][0] + nx1 * me[e][1] + nx2 * me[e][2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double G0 = g[c][0], G1 = g[c][1], G2 = g[c][2];
        const double Gmf = G0 * mf0 + G1 * mf1 + G2 * mf2;
        double nK = 0.0;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const double ge = te[e] * (G0 * me[e][0] + G1 * me[e][1] + G2 * me[e][2]) * fe[e] +
                              (G0 * le[e][0] + G1 * le[e][1] + G2 * le[e][2]) * dR[e];
            nK += nme[e] * ge;
        }
        const double nG = nx0 * G0 + nx1 * G1 + nx2 * G2;
        out[c] += (lam[c] * nF0 - w * nn * Gmf - nG * I0 + nK) * INV4PI;
    }
}

}  // namespace bem
