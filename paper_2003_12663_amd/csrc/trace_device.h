// Device helpers of the field-line kernels (Sec. 1, Eq. Breakdowncrit): the
// streamer coefficient alpha_eff, the far-field factor w / r^3 of the 7-point
// rule and the closed segment-triangle test that stops a line on a panel.
#pragma once

#include "bem_device.h"

namespace bem {

// Slot-indexed line state of the all-lines field-line layouts (one of two buffers): slots
// [0, count) hold the live lines of the two-kernel layout; the one-launch layout keeps a line in
// its slot and marks a stopped one with line -1.
struct LFState {
    double* x;      // [S][3] line point
    double* y;      // [S][3] query point of the pass to evaluate
    double* ks;     // [S][3] k1 + 2 k2 + 2 k3 + k4 so far
    double* asum;   // [S] alpha sum of the stages
    double* I;      // [S] integral
    int32_t* ns;    // [S] accepted steps
    int32_t* line;  // [S] line id
};

struct LBArgs {
    double h, e_min, dir, a, e0, p, k_str;
    int32_t max_steps;
};

static __device__ __noinline__ double lb_pow(double d, double p) { return pow(d, p); }

__device__ __forceinline__ double lb_alpha(const LBArgs& a, double e) {
    const double d = e - a.e0;
    if (!(d > 0.0)) return 0.0;
    return a.a * (a.p == 2.0 ? d * d : lb_pow(d, a.p));
}

// w / r^3 from r^2.  FP64: from the hardware estimate y of r^-1/2 (relative error about 2^-24),
// e = 1 - r^2 y^2 and r^-3 = y^3 (1 - e)^(-3/2) = y^3 (1 + 3/2 e + 15/8 e^2 + O(e^3)): seven
// operations, truncation error below 2^-68.  FP32: the hardware estimate is the answer.
// The series coefficients come in as k.c15 = 1.5 and k.c1875 = 1.875, held in registers by the
// caller (lb_series_consts): neither is an inline FP64 constant, and left as literals they are
// rebuilt inside the pair loop at every use.
struct LBSeries {
    double c15, c1875;
};
__device__ __forceinline__ LBSeries lb_series_consts() {
    LBSeries k{1.5, 1.875};
    asm volatile("" : "+v"(k.c15), "+v"(k.c1875));   // opaque: stays in a register
    return k;
}
__device__ __forceinline__ double lb_w_r3(double w, double r2, const LBSeries& k) {
    const double y = __builtin_amdgcn_rsq(r2);
    const double y2 = y * y;
    const double e = __fma_rn(-r2, y2, 1.0);
    const double wy3 = w * (y2 * y);
    return __fma_rn(wy3 * e, __fma_rn(e, k.c1875, k.c15), wy3);
}
__device__ __forceinline__ float lb_w_r3(float w, float r2, const LBSeries&) {
    const float ir = rsqrt_pos(r2);
    return w * ir * ir * ir;
}

// Moeller-Trumbore test of the closed segment q -> q + d against the closed
// triangle T; t in [0,1], or -1 when there is no hit.
__device__ __forceinline__ double lb_segment_tri(const double* __restrict__ T, double q0, double q1, double q2,
                                                 double d0, double d1, double d2) {
    const double a0 = T[3] - T[0], a1 = T[4] - T[1], a2 = T[5] - T[2];
    const double b0 = T[6] - T[0], b1 = T[7] - T[1], b2 = T[8] - T[2];
    const double pv0 = d1 * b2 - d2 * b1, pv1 = d2 * b0 - d0 * b2, pv2 = d0 * b1 - d1 * b0;
    const double det = a0 * pv0 + a1 * pv1 + a2 * pv2;
    if (det == 0.0) return -1.0;
    const double inv = 1.0 / det;
    const double t0 = q0 - T[0], t1 = q1 - T[1], t2 = q2 - T[2];
    const double u = (t0 * pv0 + t1 * pv1 + t2 * pv2) * inv;
    if (u < 0.0 || u > 1.0) return -1.0;
    const double qv0 = t1 * a2 - t2 * a1, qv1 = t2 * a0 - t0 * a2, qv2 = t0 * a1 - t1 * a0;
    const double v = (d0 * qv0 + d1 * qv1 + d2 * qv2) * inv;
    if (v < 0.0 || u + v > 1.0) return -1.0;
    const double t = (b0 * qv0 + b1 * qv1 + b2 * qv2) * inv;
    if (t < 0.0 || t > 1.0) return -1.0;
    return t;
}

// Field F = -grad S of a flat triangle with unit density at a point x off the
// triangle: the closed form of flat_tri_SF (field part), with the three edge
// terms taken one after another so that few registers stay live (the tracer
// evaluates it inside a kernel whose regular pass needs the registers).
__device__ __forceinline__ void flat_tri_F_seq(const double* __restrict__ T, double x0, double x1, double x2,
                                               double& F0, double& F1, double& F2) {
    const double n0 = T[TR_N + 0], n1 = T[TR_N + 1], n2 = T[TR_N + 2];
    const double w = (x0 - T[0]) * n0 + (x1 - T[1]) * n1 + (x2 - T[2]) * n2;
    const double r0 = x0 - w * n0, r1 = x1 - w * n1, r2 = x2 - w * n2;
    double m0s = 0.0, m1s = 0.0, m2s = 0.0;
#pragma unroll 1
    for (int e = 0; e < 3; ++e) {
        const int bv = (e == 2) ? 0 : e + 1;
        const double ax = T[3 * e], ay = T[3 * e + 1], az = T[3 * e + 2];
        const double bx = T[3 * bv], by = T[3 * bv + 1], bz = T[3 * bv + 2];
        double l0 = bx - ax, l1 = by - ay, l2 = bz - az;
        const double len = sqrt(l0 * l0 + l1 * l1 + l2 * l2);
        const double il = 1.0 / len;
        l0 *= il; l1 *= il; l2 *= il;
        const double m0 = l1 * n2 - l2 * n1, m1 = l2 * n0 - l0 * n2, m2 = l0 * n1 - l1 * n0;
        const double q0 = ax - r0, q1 = ay - r1, q2 = az - r2;
        const double sm = q0 * l0 + q1 * l1 + q2 * l2;
        const double sp = sm + len;
        const double t = q0 * m0 + q1 * m1 + q2 * m2;
        const double va0 = ax - x0, va1 = ay - x1, va2 = az - x2;
        const double vb0 = bx - x0, vb1 = by - x1, vb2 = bz - x2;
        const double Rm = sqrt(va0 * va0 + va1 * va1 + va2 * va2);
        const double Rp = sqrt(vb0 * vb0 + vb1 * vb1 + vb2 * vb2);
        // the quotient under the logarithm by case, picked before the one division and logarithm
        // (lanes of one wave that take different cases would otherwise run each case's in turn):
        // foot within the edge's span, R- + s- = R0^2 / (R- - s-) without cancellation; else the
        // side without cancellation
        const bool span = sm < 0.0 && sp > 0.0, fwd = sp + sm > 0.0;
        const double num = span ? (Rp + sp) * (Rm - sm) : (fwd ? Rp + sp : Rm - sm);
        const double den = span ? t * t + w * w : (fwd ? Rm + sm : Rp - sp);
        const double f = log(num / den);
        m0s += m0 * f;
        m1s += m1 * f;
        m2s += m2 * f;
    }
    // solid angle (Van Oosterom & Strackee)
    double V[3][3], Rv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        V[k][0] = T[3 * k] - x0;
        V[k][1] = T[3 * k + 1] - x1;
        V[k][2] = T[3 * k + 2] - x2;
        Rv[k] = sqrt(V[k][0] * V[k][0] + V[k][1] * V[k][1] + V[k][2] * V[k][2]);
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
    const double sg = (w > 0.0) ? omega : ((w < 0.0) ? -omega : 0.0);
    F0 = (m0s + sg * n0) * INV4PI;
    F1 = (m1s + sg * n1) * INV4PI;
    F2 = (m2s + sg * n2) * INV4PI;
}

// the one-launch-per-stage passes pass0 .. of the lines in slots [0, S) of buf0 (trace_fused.hip)
void fused_trace_loop(bem_ctx* c, const double* sol, int64_t L, const int32_t* line_rhs, const bem_trace_params* tp,
                      int32_t* n_steps, int32_t* stop_code, double* path, double* integral, uint8_t* exceeds,
                      LFState buf0, LFState buf1, int64_t S, int64_t pass0, unsigned long long* ncnt);

}  // namespace bem
