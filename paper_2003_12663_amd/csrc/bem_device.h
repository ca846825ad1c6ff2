// Device-side building blocks shared by the gfx950 kernels: the Sec. 4
// pair classification, the 7-point far-field sums and the closed-form
// potential/field of a flat triangle with unit charge density.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bem_internal.h"

namespace bem {

constexpr double INV4PI = 0.079577471545947667884;   // 1 / (4 pi)

// native clang vectors (usable with the nontemporal load builtin)
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

// Sec. 4 classification: the pair (x, panel) is regular iff the squared
// distance from x to the circumcentre exceeds (eta R)^2.  Written with
// explicit fma so that every kernel makes the identical decision.
__device__ __forceinline__ bool is_regular(double dx, double dy, double dz, double rr) {
    double d2 = __fma_rn(dx, dx, __fma_rn(dy, dy, dz * dz));
    return d2 > rr;
}

// Closed-form single-layer potential S and field F = -grad S of a flat
// triangle with unit density at x (Wilton et al. 1984; Graglia 1993).  With
// w the signed height of x over the plane, rho its foot point and, for each
// edge a -> b with in-plane outward normal m, the edge abscissae s-, s+, the
// in-plane distance t and the vertex distances R-, R+:
//   f_e = ln((R+ + s+)/(R- + s-))      (ln((R- - s-)/(R+ - s+)) if s+ + s- <= 0, and
//         ln((R+ + s+)(R- - s-)/R0^2) when s- < 0 < s+, R0^2 = t^2 + w^2: the same value
//         without the cancellation in R - |s| above an edge)
//   4 pi S = sum t f_e - |w| Omega,   4 pi F = sum m f_e + sign(w) n Omega,
// where Omega, the sum of the three edge angles of those papers, is the solid
// angle the triangle subtends at x, taken here in one step from the formula of
// Van Oosterom & Strackee (1983): tan(Omega/2) = |[r1 r2 r3]| /
// (R1 R2 R3 + (r1.r2) R3 + (r1.r3) R2 + (r2.r3) R1), r_k = v_k - x.
// inplane: x is the triangle's own centroid, so w = 0 and sign(w) = 0
// (principal value).  T is the 16-double exact-geometry record.
template <bool WANT_S, bool WANT_F>
__device__ __forceinline__ void flat_tri_SF(const double* __restrict__ T, double x0, double x1, double x2,
                                            bool inplane, double& S, double& F0, double& F1, double& F2) {
    const double n0 = T[TR_N + 0], n1 = T[TR_N + 1], n2 = T[TR_N + 2];
    double w = inplane ? 0.0 : (x0 - T[0]) * n0 + (x1 - T[1]) * n1 + (x2 - T[2]) * n2;
    const double r0 = x0 - w * n0, r1 = x1 - w * n1, r2 = x2 - w * n2;
    const double aw = fabs(w);
    // vectors and distances from x to the three vertices
    double V[3][3], Rv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        V[k][0] = T[3 * k] - x0;
        V[k][1] = T[3 * k + 1] - x1;
        V[k][2] = T[3 * k + 2] - x2;
        Rv[k] = sqrt(V[k][0] * V[k][0] + V[k][1] * V[k][1] + V[k][2] * V[k][2]);
    }
    double st = 0.0, m0s = 0.0, m1s = 0.0, m2s = 0.0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int b = (e + 1) % 3;
        const double ax = T[3 * e], ay = T[3 * e + 1], az = T[3 * e + 2];
        double l0 = T[3 * b] - ax, l1 = T[3 * b + 1] - ay, l2 = T[3 * b + 2] - az;
        const double len = sqrt(l0 * l0 + l1 * l1 + l2 * l2);
        const double il = 1.0 / len;
        l0 *= il; l1 *= il; l2 *= il;
        // m = l x n
        const double m0 = l1 * n2 - l2 * n1, m1 = l2 * n0 - l0 * n2, m2 = l0 * n1 - l1 * n0;
        const double q0 = ax - r0, q1 = ay - r1, q2 = az - r2;
        const double sm = q0 * l0 + q1 * l1 + q2 * l2;
        const double sp = sm + len;
        const double t = q0 * m0 + q1 * m1 + q2 * m2;
        const double Rm = Rv[e], Rp = Rv[b];
        // the quotient under the logarithm by case, picked before the one division and logarithm
        // (lanes of one wave that take different cases would otherwise run each case's in turn):
        // foot within the edge's span, R- + s- = R0^2 / (R- - s-) without cancellation; else the
        // side without cancellation
        const bool span = sm < 0.0 && sp > 0.0, fwd = sp + sm > 0.0;
        const double num = span ? (Rp + sp) * (Rm - sm) : (fwd ? Rp + sp : Rm - sm);
        const double den = span ? t * t + w * w : (fwd ? Rm + sm : Rp - sp);
        const double f = log(num / den);
        st += t * f;
        m0s += m0 * f;
        m1s += m1 * f;
        m2s += m2 * f;
    }
    double omega = 0.0;
    if (!inplane) {
        const double c0 = V[1][1] * V[2][2] - V[1][2] * V[2][1];
        const double c1 = V[1][2] * V[2][0] - V[1][0] * V[2][2];
        const double c2 = V[1][0] * V[2][1] - V[1][1] * V[2][0];
        const double triple = V[0][0] * c0 + V[0][1] * c1 + V[0][2] * c2;
        const double d01 = V[0][0] * V[1][0] + V[0][1] * V[1][1] + V[0][2] * V[1][2];
        const double d02 = V[0][0] * V[2][0] + V[0][1] * V[2][1] + V[0][2] * V[2][2];
        const double d12 = V[1][0] * V[2][0] + V[1][1] * V[2][1] + V[1][2] * V[2][2];
        const double den = Rv[0] * Rv[1] * Rv[2] + d01 * Rv[2] + d02 * Rv[1] + d12 * Rv[0];
        omega = 2.0 * atan2(fabs(triple), den);
    }
    if (WANT_S) S = (st - aw * omega) * INV4PI;
    if (WANT_F) {
        const double sg = (w > 0.0) ? omega : ((w < 0.0) ? -omega : 0.0);
        F0 = (m0s + sg * n0) * INV4PI;
        F1 = (m1s + sg * n1) * INV4PI;
        F2 = (m2s + sg * n2) * INV4PI;
    }
}

// 1/sqrt(x) for finite x > 0: the hardware estimate refined by one
// third-order step of y <- y (1 - e)^(-1/2) = y (1 + e/2 + 3 e^2/8 + ...),
// e = 1 - x y^2.  No special-value handling: callers mask x = 0 by select.
__device__ __forceinline__ double rsqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = __fma_rn(-x * y, y, 1.0);
    return __fma_rn(y * e, __fma_rn(e, 0.375, 0.5), y);
}
__device__ __forceinline__ float rsqrt_pos(float x) { return __builtin_amdgcn_rsqf(x); }

// ---- kernel-side launch timing (profiling mode 2) ----------------------------
// A timed launch owns KCLK_SUB pairs of device words: the earliest block start and the latest
// block end on the device's constant-rate wall clock, spread over sub-slots by block so that few
// atomics meet on one word.  Blocks are dispatched in order of their index, so only the first
// KCLK_SUB stamp their start; a block's end is stamped by its thread 0, whose wave finishes the
// block's reduction last in the kernels timed this way.  Stamps cost the kernel an atomic each
// (one per wave measured 6 % longer launches than rocprofv3), so they are kept this few.
// ts == nullptr: not timed.
constexpr int KCLK_SUB = 64;
__device__ __forceinline__ void kclock_start(unsigned long long* ts) {
    if (ts && blockIdx.x < KCLK_SUB && threadIdx.x == 0)
        atomicMin(ts + 2 * blockIdx.x, (unsigned long long)wall_clock64());
}
__device__ __forceinline__ void kclock_stop(unsigned long long* ts) {
    if (ts && threadIdx.x == 0)
        atomicMax(ts + 2 * (blockIdx.x % KCLK_SUB) + 1, (unsigned long long)wall_clock64());
}

// ---- wave / block reductions (wave64) --------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

}  // namespace bem
