// Nodal piecewise-linear basis with vertex collocation (Sec. 3; the matrix of
// Eq. Matrix).  sigma_h = sum_k u_k psi_k with psi_k the hat of vertex k;
// row i collocates at vertex x_i, so
//   v_ik = sum over the triangles tau holding k of int lambda_k^tau(y) / (4 pi |x_i - y|) dS,
// lambda_k^tau being tau's barycentric coordinate of k.  Conductor and
// floating-conductor bodies; a floating body's row is its net charge.
//
// Assembly keeps the collision-free ownership of Sec. 4 (each collocation
// point owns its row) at wave granularity: the 64 lanes of a wave are 64
// consecutive rows, while the column and the triangle are wave-uniform, so
// triangle records arrive through the scalar cache and every lane adds into
// its own row only.  A column is summed over the fan of its vertex (a CSR
// built at create), so each entry is written once, with no read-modify-write
// and no atomics; the price is that a regular (row, triangle) pair is
// integrated once per vertex of the triangle.  16 columns per wave are staged
// in LDS and leave as 128-byte row segments (64 bytes when the rows are stored
// in FP32, MIXED precision).  This pass takes the regular
// pairs only; the near-singular and singular ones (a small fraction, each a
// long closed form) follow in a second pass with one lane per row, which adds
// all three hats of a near triangle into its own row, so the first pass keeps
// few registers and many waves in flight.
#include <cmath>

#include "bem_device.h"
#include "nodal_device.h"

namespace bem {
namespace {

constexpr int NODAL_COLS = 16;   // columns per wave

// The rule's barycentric coordinate of local vertex c at node q (node order of
// the panel records: centroid, then the orbits (a, a, 1 - 2a) for a = a1, a2
// with the odd coordinate last, middle, first).
struct NodeBary {
    double b[7];
    __device__ NodeBary(int c) {
        const double s15 = sqrt(15.0);
        const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
        b[0] = 1.0 / 3.0;
#pragma unroll
        for (int q = 1; q <= 3; ++q) b[q] = (c == 3 - q) ? 1.0 - 2.0 * a1 : a1;
#pragma unroll
        for (int q = 4; q <= 6; ++q) b[q] = (c == 6 - q) ? 1.0 - 2.0 * a2 : a2;
    }
};

// Closed form of int lambda_c(y) / (4 pi |x - y|) dS over the flat triangle T
// (16-double exact-geometry record) for its local vertex c.  With rho the foot
// point of x on the plane and w the height,
//   lambda_c(y) = lambda_c(rho) + g_c . (y - rho),  g_c = n x (v_{c+2} - v_{c+1}) / (2A),
//   int 1/R dS = sum_e t f_e - |w| Omega                 (unit density),
//   int (y - rho)/R dS = sum_e m_e int_e R dl,  int_e R dl = (s+ R+ - s- R- + R0^2 f_e)/2,
// the second by the divergence theorem in the plane (the in-plane gradient of
// R is (y - rho)/R); edge notation and Omega as in flat_tri_SF.  vtx: x is a
// vertex of T, so w = 0 and rho = x; on the two edges that end at x, t = R0 = 0
// and their t f_e and R0^2 f_e terms vanish in the limit (f_e itself is
// infinite there), so they are skipped.
__device__ __forceinline__ void hat_edges(const double* __restrict__ T, double x0, double x1, double x2, bool vtx,
                                          double& I0, double& r0, double& r1, double& r2, double& J0, double& J1,
                                          double& J2) {
    const double n0 = T[TR_N + 0], n1 = T[TR_N + 1], n2 = T[TR_N + 2];
    const double w = vtx ? 0.0 : (x0 - T[0]) * n0 + (x1 - T[1]) * n1 + (x2 - T[2]) * n2;
    r0 = x0 - w * n0;
    r1 = x1 - w * n1;
    r2 = x2 - w * n2;
    const double aw = fabs(w);
    double V[3][3], Rv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        V[k][0] = T[3 * k] - x0;
        V[k][1] = T[3 * k + 1] - x1;
        V[k][2] = T[3 * k + 2] - x2;
        Rv[k] = sqrt(V[k][0] * V[k][0] + V[k][1] * V[k][1] + V[k][2] * V[k][2]);
    }
    double st = 0.0;
    J0 = J1 = J2 = 0.0;
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
        double er = 0.5 * (sp * Rp - sm * Rm);
        if (!(vtx && (Rm == 0.0 || Rp == 0.0))) {
            double f;
            if (sm < 0.0 && sp > 0.0)   // foot within the edge's span (see flat_tri_SF)
                f = log((Rp + sp) * (Rm - sm) / (t * t + w * w));
            else if (sp + sm > 0.0)
                f = log((Rp + sp) / (Rm + sm));
            else
                f = log((Rm - sm) / (Rp - sp));
            st += t * f;
            er += 0.5 * (t * t + w * w) * f;
        }
        J0 += m0 * er;
        J1 += m1 * er;
        J2 += m2 * er;
    }
    double omega = 0.0;
    if (!vtx) {
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
    I0 = st - aw * omega;
}

// Local corner of the triangle T at x, by position: within 1e-13 of T's longest edge; -1 if none
// (a vertex of another body that coincides with a corner of T)
__device__ __forceinline__ int coincident_corner(const double* __restrict__ T, double x0, double x1, double x2) {
    double L2 = 0.0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int b = (e + 1) % 3;
        const double d0 = T[3 * b] - T[3 * e], d1 = T[3 * b + 1] - T[3 * e + 1], d2 = T[3 * b + 2] - T[3 * e + 2];
        const double l2 = d0 * d0 + d1 * d1 + d2 * d2;
        L2 = l2 > L2 ? l2 : L2;
    }
    const double tol2 = 1e-26 * L2;
#pragma unroll
    for (int cv = 0; cv < 3; ++cv) {
        const double d0 = x0 - T[3 * cv], d1 = x1 - T[3 * cv + 1], d2 = x2 - T[3 * cv + 2];
        if (d0 * d0 + d1 * d1 + d2 * d2 <= tol2) return cv;
    }
    return -1;
}

// lambda_c(rho) I0 + g_c . J over 4 pi (see hat_edges)
__device__ __forceinline__ double hat_value(const double* __restrict__ T, int c, double I0, double r0, double r1,
                                           double r2, double J0, double J1, double J2) {
    const double n0 = T[TR_N + 0], n1 = T[TR_N + 1], n2 = T[TR_N + 2];
    const double* p = T + 3 * ((c + 1) % 3);
    const double* q = T + 3 * ((c + 2) % 3);
    const double a0 = p[0] - r0, a1 = p[1] - r1, a2 = p[2] - r2;
    const double b0 = q[0] - r0, b1 = q[1] - r1, b2 = q[2] - r2;
    const double two_area = 2.0 * T[TR_A];
    // barycentric coordinate of rho: signed area of (p, q, rho) over A
    const double lam = (n0 * (a1 * b2 - a2 * b1) + n1 * (a2 * b0 - a0 * b2) + n2 * (a0 * b1 - a1 * b0)) / two_area;
    // g = n x (q - p)
    const double e0 = q[0] - p[0], e1 = q[1] - p[1], e2 = q[2] - p[2];
    const double g0 = n1 * e2 - n2 * e1, g1 = n2 * e0 - n0 * e2, g2 = n0 * e1 - n1 * e0;
    return (lam * I0 + (g0 * J0 + g1 * J1 + g2 * J2) / two_area) * INV4PI;
}

// One wave: rows i0 + lane, columns j0 .. j0 + 15 (column group cg).  The wave walks the
// distinct triangles that hold a vertex of the group (ascending), evaluates the 7-point
// rule once per triangle and adds each hat whose vertex is in the group into that column's
// LDS slot, so a pair costs about two visits instead of one per vertex of the triangle.
// The four waves of a block take the same columns on four row tiles, so three of four
// record loads hit the scalar cache.  1-D grid of n_rt x n_cg blocks (row tiles of 256
// rows, n_cg a multiple of 8): blocks are dealt to the 8 XCDs in turn, so block b runs on
// XCD b % 8, and each XCD sweeps all row tiles of one column group before the next,
// keeping that group's records in its own L2.
template <class T>   // stored type: double (FP64) or float (MIXED)
__global__ __launch_bounds__(256) void k_nodal_assemble(int64_t nv, int64_t ld, int64_t n_rt,
                                                        const double* __restrict__ vert,
                                                        const int32_t* __restrict__ tri,
                                                        const int32_t* __restrict__ grp_ptr,
                                                        const int32_t* __restrict__ grp_tri,
                                                        const uint32_t* __restrict__ grp_loc,
                                                        const double* __restrict__ pan64, T* __restrict__ A) {
    __shared__ double tile[4][NODAL_COLS][65];   // padded: the row-segment reads stride 65
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t b = blockIdx.x, xcd = b & 7, slot = b >> 3;
    const int64_t cg = (slot / n_rt) * 8 + xcd, rt = slot % n_rt;
    const int64_t i0 = (rt * 4 + wv) * 64;
    const int64_t i = i0 + lane;
    const int64_t ic = i < nv ? i : nv - 1;
    const double x0 = vert[3 * ic], x1 = vert[3 * ic + 1], x2 = vert[3 * ic + 2];
    const int64_t j0 = cg * NODAL_COLS;
#pragma unroll
    for (int cc = 0; cc < NODAL_COLS; ++cc) tile[wv][cc][lane] = 0.0;
    if (j0 < nv) {
        const NodeBary nb0(0), nb1(1), nb2(2);
        const int32_t e1 = grp_ptr[cg + 1];
        for (int32_t e = grp_ptr[cg]; e < e1; ++e) {
            const int64_t t = grp_tri[e];
            const uint32_t loc = grp_loc[e];   // local column of corners 0, 1, 2 (0xff: not in the group)
            const double* P = pan64 + (int64_t)FAR_REC * t;
            const int32_t* tv = tri + 3 * t;
            const bool vtx = (tv[0] == i) || (tv[1] == i) || (tv[2] == i);
            // near and singular pairs are left to k_nodal_near (same predicate)
            if (!vtx && is_regular(x0 - P[FR_CC], x1 - P[FR_CC + 1], x2 - P[FR_CC + 2], P[FR_RR])) {
                double wr[7];
#pragma unroll
                for (int q = 0; q < 7; ++q) {
                    const double d0 = x0 - P[FR_X + q], d1 = x1 - P[FR_Y + q], d2 = x2 - P[FR_Z + q];
                    wr[q] = rsqrt_pos(d0 * d0 + d1 * d1 + d2 * d2);
                }
                const uint32_t l0 = loc & 0xffu, l1 = (loc >> 8) & 0xffu, l2 = (loc >> 16) & 0xffu;
                if (l0 != 0xffu) {
                    double s = 0.0;
#pragma unroll
                    for (int q = 0; q < 7; ++q) s += P[FR_W + q] * nb0.b[q] * wr[q];
                    tile[wv][l0][lane] += s;
                }
                if (l1 != 0xffu) {
                    double s = 0.0;
#pragma unroll
                    for (int q = 0; q < 7; ++q) s += P[FR_W + q] * nb1.b[q] * wr[q];
                    tile[wv][l1][lane] += s;
                }
                if (l2 != 0xffu) {
                    double s = 0.0;
#pragma unroll
                    for (int q = 0; q < 7; ++q) s += P[FR_W + q] * nb2.b[q] * wr[q];
                    tile[wv][l2][lane] += s;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll 4
    for (int s = 0; s < 16; ++s) {
        const int r = (lane >> 4) + 4 * s, cc = lane & 15;
        const int64_t ii = i0 + r, jj = j0 + cc;
        if (ii < nv && jj < nv) A[ii * ld + jj] = (T)tile[wv][cc][r];
    }
}

// Bound of each chunk of 64 consecutive triangles: a centre and a radius such
// that every point within eta R of a circumcentre of the chunk lies in the ball
// (radius = max |cc - centre| + eta R), so a ball of rows apart from it by more
// than the two radii makes only regular pairs with the chunk.
__global__ __launch_bounds__(256) void k_nodal_chunk_bounds(int64_t N, int64_t Np, const double* __restrict__ far64,
                                                            double* __restrict__ cb) {
    const int64_t ch = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t t0 = ch * 64;
    if (t0 >= N) return;
    const int64_t t1 = t0 + 64 < N ? t0 + 64 : N;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        m0 += far64[(int64_t)(FR_CC + 0) * Np + t];
        m1 += far64[(int64_t)(FR_CC + 1) * Np + t];
        m2 += far64[(int64_t)(FR_CC + 2) * Np + t];
    }
    const double inv = 1.0 / (double)(t1 - t0);
    m0 *= inv; m1 *= inv; m2 *= inv;
    double r = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        const double d0 = far64[(int64_t)(FR_CC + 0) * Np + t] - m0, d1 = far64[(int64_t)(FR_CC + 1) * Np + t] - m1;
        const double d2 = far64[(int64_t)(FR_CC + 2) * Np + t] - m2;
        const double e = sqrt(d0 * d0 + d1 * d1 + d2 * d2) + sqrt(far64[(int64_t)FR_RR * Np + t]);
        r = e > r ? e : r;
    }
    cb[4 * ch] = m0;
    cb[4 * ch + 1] = m1;
    cb[4 * ch + 2] = m2;
    cb[4 * ch + 3] = r;
}

__device__ __forceinline__ double lane_bcast(double v, int k) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, k), hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Near-singular and singular pairs of the vertex rows (one lane per row, 64 rows
// per block, the rows taken in a spatial (Morton) order of the vertices so that
// a block's rows are neighbours).  Chunks of 64 triangles whose bound is beyond
// reach of the rows' ball are skipped; in the others every triangle is classified with the
// predicate of the first pass, its circumcentre, (eta R)^2 and vertex indices
// loaded by the lanes together (component-major records) and broadcast from a
// lane register.  A near triangle adds its three hats into the lane's own row.
template <class T>
__global__ __launch_bounds__(64) void k_nodal_near(int64_t nv, int64_t ld, int64_t N, int64_t Np,
                                                   const int32_t* __restrict__ row_order,
                                                   const double* __restrict__ vert, const int32_t* __restrict__ tri,
                                                   const double* __restrict__ far64, const double* __restrict__ cb,
                                                   const double* __restrict__ tri64, T* __restrict__ A) {
    const int lane = threadIdx.x;
    const int64_t s = (int64_t)blockIdx.x * 64 + lane;
    const bool live = s < nv;
    const int64_t ic = row_order[live ? s : nv - 1];
    const int64_t i = live ? ic : -1;   // -1 matches no vertex
    const double x0 = vert[3 * ic], x1 = vert[3 * ic + 1], x2 = vert[3 * ic + 2];
    T* row = A + ic * ld;
    // ball of the 64 rows
    const double g0 = wave_sum(x0) / 64.0, g1 = wave_sum(x1) / 64.0, g2 = wave_sum(x2) / 64.0;
    double rg = sqrt((x0 - g0) * (x0 - g0) + (x1 - g1) * (x1 - g1) + (x2 - g2) * (x2 - g2));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double other = __shfl_xor(rg, o, 64);
        rg = other > rg ? other : rg;
    }
    for (int64_t t0 = 0; t0 < N; t0 += 64) {
        const double* B = cb + 4 * (t0 >> 6);
        const double e0 = B[0] - g0, e1 = B[1] - g1, e2 = B[2] - g2;
        const double reach = (rg + B[3]) * (1.0 + 1e-9) + 1e-300;
        if (e0 * e0 + e1 * e1 + e2 * e2 > reach * reach) continue;   // every pair regular
        const int64_t tl = t0 + lane < N ? t0 + lane : N - 1;
        const double c0 = far64[(int64_t)(FR_CC + 0) * Np + tl], c1 = far64[(int64_t)(FR_CC + 1) * Np + tl];
        const double c2 = far64[(int64_t)(FR_CC + 2) * Np + tl], rr = far64[(int64_t)FR_RR * Np + tl];
        const int32_t v0 = tri[3 * tl], v1 = tri[3 * tl + 1], v2 = tri[3 * tl + 2];
        const int kend = N - t0 < 64 ? (int)(N - t0) : 64;
        for (int k = 0; k < kend; ++k) {
            const double cc0 = lane_bcast(c0, k), cc1 = lane_bcast(c1, k), cc2 = lane_bcast(c2, k);
            const double crr = lane_bcast(rr, k);
            const int32_t a = __builtin_amdgcn_readlane(v0, k), b = __builtin_amdgcn_readlane(v1, k);
            const int32_t c = __builtin_amdgcn_readlane(v2, k);
            bool vtx = (a == i) || (b == i) || (c == i);
            const bool near = vtx || !is_regular(x0 - cc0, x1 - cc1, x2 - cc2, crr);
            if (near && live) {
                // the three entries are read first so that their latency overlaps the closed form;
                // the sum is formed in FP64 and rounded once to the stored type
                const double ya = (double)row[a], yb = (double)row[b], yc = (double)row[c];
                const double* Tr = tri64 + (int64_t)TRI_REC * (t0 + k);
                // a vertex of another body at x (bodies that touch): the singular closed form at
                // that vertex's own position
                double xs0 = x0, xs1 = x1, xs2 = x2;
                if (!vtx) {
                    const int cv = coincident_corner(Tr, x0, x1, x2);
                    if (cv >= 0) {
                        vtx = true;
                        xs0 = Tr[TR_V + 3 * cv];
                        xs1 = Tr[TR_V + 3 * cv + 1];
                        xs2 = Tr[TR_V + 3 * cv + 2];
                    }
                }
                double I0, r0, r1, r2, J0, J1, J2;
                hat_edges(Tr, xs0, xs1, xs2, vtx, I0, r0, r1, r2, J0, J1, J2);
                row[a] = (T)(ya + hat_value(Tr, 0, I0, r0, r1, r2, J0, J1, J2));
                row[b] = (T)(yb + hat_value(Tr, 1, I0, r0, r1, r2, J0, J1, J2));
                row[c] = (T)(yc + hat_value(Tr, 2, I0, r0, r1, r2, J0, J1, J2));
            }
        }
    }
}

// ---- rows that need n . E (interface vertices, literal Final4, sheets) ----------------
// A vertex of flat panels has no normal, so those rows take the normal field at the
// centroids x_T of triangles T (normal n_T): Kc[r][k] = n_T . (field of hat k over every
// triangle but T at x_T) for the centroid rows r (trow[r] = T), row stride ld.  T itself adds
// nothing (in its plane the field of its own density has no normal component).

// Regular pairs of the centroid rows: k_nodal_assemble's walk of column groups, with the
// kernel n_T . w (x - y)/|x - y|^3 in place of w/|x - y|.  Kc is FP64.
__global__ __launch_bounds__(256) void k_nodal_kp_assemble(int64_t nc, int64_t nv, int64_t ld, int64_t n_rt,
                                                           const int32_t* __restrict__ trow,
                                                           const int32_t* __restrict__ grp_ptr,
                                                           const int32_t* __restrict__ grp_tri,
                                                           const uint32_t* __restrict__ grp_loc,
                                                           const double* __restrict__ pan64,
                                                           const double* __restrict__ tri64, double* __restrict__ Kc) {
    __shared__ double tile[4][NODAL_COLS][65];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t b = blockIdx.x, xcd = b & 7, slot = b >> 3;
    const int64_t cg = (slot / n_rt) * 8 + xcd, rt = slot % n_rt;
    const int64_t r0 = (rt * 4 + wv) * 64;
    const int64_t r = r0 + lane;
    const int64_t T = trow[r < nc ? r : nc - 1];
    const double* Tr = tri64 + (int64_t)TRI_REC * T;
    const double x0 = Tr[TR_C], x1 = Tr[TR_C + 1], x2 = Tr[TR_C + 2];
    const double m0 = Tr[TR_N], m1 = Tr[TR_N + 1], m2 = Tr[TR_N + 2];
    const int64_t j0 = cg * NODAL_COLS;
#pragma unroll
    for (int cc = 0; cc < NODAL_COLS; ++cc) tile[wv][cc][lane] = 0.0;
    if (j0 < nv) {
        const NodeBary nb0(0), nb1(1), nb2(2);
        const int32_t e1 = grp_ptr[cg + 1];
        for (int32_t e = grp_ptr[cg]; e < e1; ++e) {
            const int64_t t = grp_tri[e];
            const uint32_t loc = grp_loc[e];
            const double* P = pan64 + (int64_t)FAR_REC * t;
            if (t != T && is_regular(x0 - P[FR_CC], x1 - P[FR_CC + 1], x2 - P[FR_CC + 2], P[FR_RR])) {
                double kq[7];
#pragma unroll
                for (int q = 0; q < 7; ++q) {
                    const double d0 = x0 - P[FR_X + q], d1 = x1 - P[FR_Y + q], d2 = x2 - P[FR_Z + q];
                    const double ir = rsqrt_pos(d0 * d0 + d1 * d1 + d2 * d2);
                    kq[q] = P[FR_W + q] * (d0 * m0 + d1 * m1 + d2 * m2) * (ir * ir * ir);
                }
                const uint32_t l0 = loc & 0xffu, l1 = (loc >> 8) & 0xffu, l2 = (loc >> 16) & 0xffu;
                if (l0 != 0xffu) {
                    double sacc = 0.0;
#pragma unroll
                    for (int q = 0; q < 7; ++q) sacc += kq[q] * nb0.b[q];
                    tile[wv][l0][lane] += sacc;
                }
                if (l1 != 0xffu) {
                    double sacc = 0.0;
#pragma unroll
                    for (int q = 0; q < 7; ++q) sacc += kq[q] * nb1.b[q];
                    tile[wv][l1][lane] += sacc;
                }
                if (l2 != 0xffu) {
                    double sacc = 0.0;
#pragma unroll
                    for (int q = 0; q < 7; ++q) sacc += kq[q] * nb2.b[q];
                    tile[wv][l2][lane] += sacc;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll 4
    for (int sgm = 0; sgm < 16; ++sgm) {
        const int rr = (lane >> 4) + 4 * sgm, cc = lane & 15;
        const int64_t ii = r0 + rr, jj = j0 + cc;
        if (ii < nc && jj < nv) Kc[ii * ld + jj] = tile[wv][cc][rr];
    }
}

// Near pairs of the centroid rows (one lane per row, chunks of 64 triangles beyond reach of the
// rows' ball skipped, as k_nodal_near): the closed form of the three hats' normal field.
__global__ __launch_bounds__(64) void k_nodal_kp_near(int64_t nc, int64_t ld, int64_t N, int64_t Np,
                                                      const int32_t* __restrict__ trow,
                                                      const int32_t* __restrict__ tri,
                                                      const double* __restrict__ far64, const double* __restrict__ cb,
                                                      const double* __restrict__ tri64, double* __restrict__ Kc) {
    const int lane = threadIdx.x;
    const int64_t r = (int64_t)blockIdx.x * 64 + lane;
    const bool live = r < nc;
    const int64_t rc = live ? r : nc - 1;
    const int64_t T = trow[rc];
    const double* Tx = tri64 + (int64_t)TRI_REC * T;
    const double x0 = Tx[TR_C], x1 = Tx[TR_C + 1], x2 = Tx[TR_C + 2];
    const double m0 = Tx[TR_N], m1 = Tx[TR_N + 1], m2 = Tx[TR_N + 2];
    double* row = Kc + rc * ld;
    const double g0 = wave_sum(x0) / 64.0, g1 = wave_sum(x1) / 64.0, g2 = wave_sum(x2) / 64.0;
    double rg = sqrt((x0 - g0) * (x0 - g0) + (x1 - g1) * (x1 - g1) + (x2 - g2) * (x2 - g2));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double other = __shfl_xor(rg, o, 64);
        rg = other > rg ? other : rg;
    }
    for (int64_t t0 = 0; t0 < N; t0 += 64) {
        const double* B = cb + 4 * (t0 >> 6);
        const double e0 = B[0] - g0, e1 = B[1] - g1, e2 = B[2] - g2;
        const double reach = (rg + B[3]) * (1.0 + 1e-9) + 1e-300;
        if (e0 * e0 + e1 * e1 + e2 * e2 > reach * reach) continue;   // every pair regular
        const int64_t tl = t0 + lane < N ? t0 + lane : N - 1;
        const double c0 = far64[(int64_t)(FR_CC + 0) * Np + tl], c1 = far64[(int64_t)(FR_CC + 1) * Np + tl];
        const double c2 = far64[(int64_t)(FR_CC + 2) * Np + tl], rr = far64[(int64_t)FR_RR * Np + tl];
        const int32_t v0 = tri[3 * tl], v1 = tri[3 * tl + 1], v2 = tri[3 * tl + 2];
        const int kend = N - t0 < 64 ? (int)(N - t0) : 64;
        for (int k = 0; k < kend; ++k) {
            const double cc0 = lane_bcast(c0, k), cc1 = lane_bcast(c1, k), cc2 = lane_bcast(c2, k);
            const double crr = lane_bcast(rr, k);
            const int32_t a = __builtin_amdgcn_readlane(v0, k), b = __builtin_amdgcn_readlane(v1, k);
            const int32_t c = __builtin_amdgcn_readlane(v2, k);
            const bool near = (t0 + k != T) && !is_regular(x0 - cc0, x1 - cc1, x2 - cc2, crr);
            if (near && live) {
                const double ya = row[a], yb = row[b], yc = row[c];
                double out[3] = {0.0, 0.0, 0.0};
                nodal_tri_hats_nE(tri64 + (int64_t)TRI_REC * (t0 + k), x0, x1, x2, m0, m1, m2, out);
                row[a] = ya + out[0];
                row[b] = yb + out[1];
                row[c] = yc + out[2];
            }
        }
    }
}

// Interface vertex rows (Eq. nonconductors at the vertex, taken as the hat-weighted mean over
// the vertex's triangles T of the condition at x_T): one block per interface vertex i,
//   A[i][k] = sum_{T in fan(i)} (a_T/3)/m_i [ (eps+ - eps-) Kc[crow(T)][k]
//                                             + (eps+ + eps-)/2 [k in T]/3 ],
// m_i = sum over the fan of a_T/3; fan order, so the sums are reproducible.  Columns k < nv.
template <class TT>
__global__ __launch_bounds__(256) void k_nodal_iface_rows(int64_t nv, int64_t ld, const int32_t* __restrict__ iface_v,
                                                          const int32_t* __restrict__ fan_ptr,
                                                          const int32_t* __restrict__ fan,
                                                          const int32_t* __restrict__ tri,
                                                          const int32_t* __restrict__ tri_crow,
                                                          const int32_t* __restrict__ vert_body,
                                                          const double* __restrict__ epsp,
                                                          const double* __restrict__ epsm,
                                                          const double* __restrict__ tri64,
                                                          const double* __restrict__ mass,
                                                          const double* __restrict__ Kc, TT* __restrict__ A) {
    const int64_t i = iface_v[blockIdx.x];
    const int32_t bd = vert_body[i];
    const double dk = epsp[bd] - epsm[bd], hs = 0.5 * (epsp[bd] + epsm[bd]) / 3.0;
    const double inv_m = 1.0 / mass[i];
    const int32_t f0 = fan_ptr[i], f1 = fan_ptr[i + 1];
    for (int64_t k = threadIdx.x; k < nv; k += 256) {
        double acc = 0.0;
        for (int32_t e = f0; e < f1; ++e) {
            const int64_t t = fan[e] >> 2;
            const double wT = tri64[(int64_t)TRI_REC * t + TR_A] / 3.0 * inv_m;
            const int32_t* tv = tri + 3 * t;
            const double self = (tv[0] == k || tv[1] == k || tv[2] == k) ? hs : 0.0;
            acc += wT * (dk * Kc[(int64_t)tri_crow[t] * ld + k] + self);
        }
        A[i * ld + k] = (TT)acc;
    }
}

// Rows of floating bodies with a normal-field term (literal Eq. Final4, sheets), the centroid
// rule over the body's triangles: row f (stored at row0 + f)
//   A[k] = sum_{T in f} (a_T/area_f) [ c_kp Kc[crow(T)][k] + c_self [k in T]/3 ]
//        = c_kp sum_T (a_T/area_f) Kc[crow(T)][k] + c_self m_k/area_f [k on f],
// over the body's contiguous centroid rows [cr0, cr1) in order; 0 in columns >= nv; Jacobi
// diagonal 1 (the entry is 0).  grid (column chunks, bodies in the list).
__global__ __launch_bounds__(256) void k_nodal_kp_body_rows(int64_t nv, int64_t ld, int64_t row0,
                                                            const int32_t* __restrict__ flist,
                                                            const int32_t* __restrict__ frange,
                                                            const double* __restrict__ fcoef,
                                                            const int32_t* __restrict__ trow,
                                                            const int32_t* __restrict__ vert_body,
                                                            const int32_t* __restrict__ fidx,
                                                            const double* __restrict__ tri64,
                                                            const double* __restrict__ mass,
                                                            const double* __restrict__ Af,
                                                            const double* __restrict__ Kc, double* __restrict__ A,
                                                            double* __restrict__ diag) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int32_t f = flist[blockIdx.y];
    if (k >= ld) return;
    const double inv_a = 1.0 / Af[f];
    const double cs = fcoef[2 * f], ck = fcoef[2 * f + 1];
    double acc = 0.0;
    if (k < nv) {
        double s = 0.0;
        for (int32_t r = frange[2 * f]; r < frange[2 * f + 1]; ++r)
            s += tri64[(int64_t)TRI_REC * trow[r] + TR_A] * Kc[(int64_t)r * ld + k];
        acc = ck * s * inv_a + (fidx[vert_body[k]] == f ? cs * mass[k] * inv_a : 0.0);
    }
    A[(row0 + f) * ld + k] = acc;
    if (k == 0) diag[nv + f] = 1.0;
}

// Jacobi diagonal of the vertex rows
template <class T>
__global__ __launch_bounds__(256) void k_nodal_diag(int64_t nv, int64_t ld, const T* __restrict__ A,
                                                    double* __restrict__ diag) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < nv) diag[i] = (double)A[i * ld + i];
}

// columns [nv, ld) of the vertex rows: -1 in the column of the row's floating body, else 0
template <class T>
__global__ __launch_bounds__(256) void k_nodal_tail(int64_t nv, int64_t ld, const int32_t* __restrict__ vert_body,
                                                    const int32_t* __restrict__ body_kind,
                                                    const int32_t* __restrict__ fidx, T* __restrict__ A) {
    const int64_t ncol = ld - nv;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= nv * ncol) return;
    const int64_t i = t / ncol, k = t % ncol;
    const int32_t b = vert_body[i];
    A[i * ld + nv + k] = (T)((body_kind[b] == BEM_FLOATING && fidx[b] == k) ? -1.0 : 0.0);
}

// m_k = int psi_k dS = sum over the fan of k of area / 3
__global__ __launch_bounds__(256) void k_nodal_mass(int64_t nv, const int32_t* __restrict__ fan_ptr,
                                                    const int32_t* __restrict__ fan, const double* __restrict__ tri64,
                                                    double* __restrict__ mass) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= nv) return;
    double s = 0.0;
    for (int32_t e = fan_ptr[k]; e < fan_ptr[k + 1]; ++e) s += tri64[(int64_t)TRI_REC * (fan[e] >> 2) + TR_A];
    mass[k] = s / 3.0;
}

// area of floating body f (one block each): sum of m_k over its vertices, fixed order
__global__ __launch_bounds__(256) void k_nodal_body_area(int64_t nv, const int32_t* __restrict__ vert_body,
                                                         const int32_t* __restrict__ fidx,
                                                         const double* __restrict__ mass, double* __restrict__ Af) {
    __shared__ double red[4];
    const int f = blockIdx.x;
    double s = 0.0;
    for (int64_t k = threadIdx.x; k < nv; k += 256)
        if (fidx[vert_body[k]] == f) s += mass[k];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) Af[f] = (red[0] + red[1]) + (red[2] + red[3]);
}

// row nv + f (stored at row0 + f): m_k / area_f on the vertices of floating body f, 0
// elsewhere (all ld columns); its Jacobi diagonal is 1 (the entry is 0)
__global__ __launch_bounds__(256) void k_nodal_constraint(int64_t nv, int64_t row0, int64_t ld, int32_t n_float,
                                                          const int32_t* __restrict__ vert_body,
                                                          const int32_t* __restrict__ fidx,
                                                          const double* __restrict__ mass,
                                                          const double* __restrict__ Af, double* __restrict__ A,
                                                          double* __restrict__ diag) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)n_float * ld) return;
    const int64_t f = t / ld, k = t % ld;
    A[(row0 + f) * ld + k] = (k < nv && fidx[vert_body[k]] == f) ? mass[k] / Af[f] : 0.0;
    if (k == 0) diag[nv + f] = 1.0;
}

// phi and E at volume points from vertex densities (the field formula closing
// Sec. 2): 64 points per block, the triangles split over the 4 waves, partial
// sums folded in LDS.  Regular pairs by the 7-point rule with the density at the
// nodes, the others by nodal_tri_phiE.  grid (point tiles, load cases); phi or E
// may be null.
__global__ __launch_bounds__(256) void k_nodal_field(int64_t P, const double* __restrict__ pts, int64_t N,
                                                     const int32_t* __restrict__ tri,
                                                     const double* __restrict__ pan64,
                                                     const double* __restrict__ tri64,
                                                     const double* __restrict__ sol, int64_t n,
                                                     double* __restrict__ phi, double* __restrict__ E) {
    __shared__ double part[4][4][64];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t p = (int64_t)blockIdx.x * 64 + lane;
    const int64_t pc = p < P ? p : P - 1;
    const double x0 = pts[3 * pc], x1 = pts[3 * pc + 1], x2 = pts[3 * pc + 2];
    const double* u = sol + (int64_t)blockIdx.y * n;
    const double s15 = sqrt(15.0);
    const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
    const double b1 = 1.0 - 2.0 * a1, b2 = 1.0 - 2.0 * a2;
    const int64_t per = (N + 3) / 4;
    const int64_t t0 = wv * per, t1 = t0 + per < N ? t0 + per : N;
    double ph = 0.0, e0 = 0.0, e1 = 0.0, e2 = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        const int32_t* tv = tri + 3 * t;
        const double u0 = u[tv[0]], u1 = u[tv[1]], u2 = u[tv[2]];
        const double* Pr = pan64 + (int64_t)FAR_REC * t;
        if (is_regular(x0 - Pr[FR_CC], x1 - Pr[FR_CC + 1], x2 - Pr[FR_CC + 2], Pr[FR_RR])) {
            // density at the nodes (same barycentrics as NodeBary)
            const double sq[7] = {(u0 + u1 + u2) / 3.0,
                                  a1 * u0 + a1 * u1 + b1 * u2, a1 * u0 + b1 * u1 + a1 * u2, b1 * u0 + a1 * u1 + a1 * u2,
                                  a2 * u0 + a2 * u1 + b2 * u2, a2 * u0 + b2 * u1 + a2 * u2, b2 * u0 + a2 * u1 + a2 * u2};
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                const double d0 = x0 - Pr[FR_X + q], d1 = x1 - Pr[FR_Y + q], d2 = x2 - Pr[FR_Z + q];
                const double ir = rsqrt_pos(d0 * d0 + d1 * d1 + d2 * d2);
                const double c = Pr[FR_W + q] * sq[q] * ir;
                const double c3 = c * ir * ir;
                ph += c;
                e0 += c3 * d0;
                e1 += c3 * d1;
                e2 += c3 * d2;
            }
        } else {
            nodal_tri_phiE(tri64 + (int64_t)TRI_REC * t, x0, x1, x2, u0, u1, u2, ph, e0, e1, e2);
        }
    }
    part[0][wv][lane] = ph;
    part[1][wv][lane] = e0;
    part[2][wv][lane] = e1;
    part[3][wv][lane] = e2;
    __syncthreads();
    if (wv == 0 && p < P) {
        const int64_t o = (int64_t)blockIdx.y * P + p;
        double r[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) r[c] = (part[c][0][lane] + part[c][1][lane]) + (part[c][2][lane] + part[c][3][lane]);
        if (phi) phi[o] = r[0];
        if (E) {
            E[3 * o] = r[1];
            E[3 * o + 1] = r[2];
            E[3 * o + 2] = r[3];
        }
    }
}

// Panel records of a nodal density for the field-line passes: the copy of each
// record (both layouts) with node weight q scaled by the density at node q,
// sum_c b_qc u_c, so that the constant-basis far kernels, run with a density of
// one per panel, sum the nodal density's far field.  Padding panels keep their
// zero weights.
__global__ __launch_bounds__(256) void k_nodal_records(int64_t N, int64_t Np, const int32_t* __restrict__ tri,
                                                       const double* __restrict__ pan64, const double* __restrict__ u,
                                                       double* __restrict__ npan, double* __restrict__ nfar,
                                                       double* __restrict__ ones) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= Np) return;
    double sq[7] = {1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0};
    if (j < N) {
        const double u0 = u[tri[3 * j]], u1 = u[tri[3 * j + 1]], u2 = u[tri[3 * j + 2]];
        const double s15 = sqrt(15.0);
        const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
        const double b1 = 1.0 - 2.0 * a1, b2 = 1.0 - 2.0 * a2;
        sq[0] = (u0 + u1 + u2) / 3.0;
        sq[1] = a1 * u0 + a1 * u1 + b1 * u2;
        sq[2] = a1 * u0 + b1 * u1 + a1 * u2;
        sq[3] = b1 * u0 + a1 * u1 + a1 * u2;
        sq[4] = a2 * u0 + a2 * u1 + b2 * u2;
        sq[5] = a2 * u0 + b2 * u1 + a2 * u2;
        sq[6] = b2 * u0 + a2 * u1 + a2 * u2;
    }
#pragma unroll
    for (int k = 0; k < FAR_REC; ++k) {
        double v = pan64[(int64_t)FAR_REC * j + k];
        if (k >= FR_W && k < FR_W + 7) v *= sq[k - FR_W];
        npan[(int64_t)FAR_REC * j + k] = v;
        nfar[(int64_t)k * Np + j] = v;
    }
    ones[j] = 1.0;
}

}  // namespace

void launch_nodal_records(bem_ctx* c, const double* u) {
    const int64_t Np = (int64_t)(c->far64.bytes / (sizeof(double) * FAR_REC));
    c->nod_pan64.alloc(sizeof(double) * FAR_REC * (size_t)Np);
    c->nod_far64.alloc(sizeof(double) * FAR_REC * (size_t)Np);
    c->nod_ones.alloc(sizeof(double) * (size_t)Np);
    hipLaunchKernelGGL(k_nodal_records, dim3((unsigned)ceil_div(Np, 256)), dim3(256), 0, c->stream, c->N, Np,
                       c->tri.as<int32_t>(), c->pan64.as<double>(), u, c->nod_pan64.as<double>(),
                       c->nod_far64.as<double>(), c->nod_ones.as<double>());
    BEM_CHECK_LAUNCH();
}

template <class T>
static void nodal_assemble_t(bem_ctx* c, T* A, double* Atail, int64_t tail_row0) {
    const int64_t nv = c->n_vert, ld = c->ld;
    hipStream_t s = c->stream;
    const int64_t n_rt = ceil_div(nv, 256), n_cg = ceil_div(ceil_div(nv, NODAL_COLS), 8) * 8;
    if (n_rt * n_cg > ((int64_t)1 << 31) - 1) throw Error(BEM_ERR_INVALID, "too many vertices for the LINEAR basis");
    hipLaunchKernelGGL(k_nodal_assemble<T>, dim3((unsigned)(n_rt * n_cg)), dim3(256), 0, s, nv, ld, n_rt,
                       c->vert.as<double>(), c->tri.as<int32_t>(), c->grp_ptr.as<int32_t>(), c->grp_tri.as<int32_t>(),
                       c->grp_loc.as<uint32_t>(), c->pan64.as<double>(), A);
    BEM_CHECK_LAUNCH();
    const int64_t Np = (int64_t)(c->far64.bytes / (sizeof(double) * FAR_REC));
    const int64_t nch = ceil_div(c->N, 64);
    c->nodal_bounds.alloc(sizeof(double) * 4 * (size_t)nch);
    hipLaunchKernelGGL(k_nodal_chunk_bounds, dim3((unsigned)ceil_div(nch, 256)), dim3(256), 0, s, c->N, Np,
                       c->far64.as<double>(), c->nodal_bounds.as<double>());
    BEM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_nodal_near<T>, dim3((unsigned)ceil_div(nv, 64)), dim3(64), 0, s, nv, ld, c->N, Np,
                       c->row_order.as<int32_t>(), c->vert.as<double>(), c->tri.as<int32_t>(), c->far64.as<double>(),
                       c->nodal_bounds.as<double>(), c->tri64.as<double>(), A);
    BEM_CHECK_LAUNCH();
    const int64_t nc = (int64_t)c->h_crow_tri.size(), niv = (int64_t)c->h_iface_v.size();
    const bool need_mass = c->n_float > 0 || niv > 0;
    double* mass = nullptr;
    if (need_mass) {
        c->nodal_mass.alloc(sizeof(double) * (size_t)(nv + c->n_float));
        mass = c->nodal_mass.as<double>();
        hipLaunchKernelGGL(k_nodal_mass, dim3((unsigned)ceil_div(nv, 256)), dim3(256), 0, s, nv,
                           c->fan_ptr.as<int32_t>(), c->fan.as<int32_t>(), c->tri64.as<double>(), mass);
        BEM_CHECK_LAUNCH();
    }
    if (nc > 0) {
        // normal-field rows at the centroids, then the interface vertex rows from them
        double* Kc = c->nod_Kc.as<double>();
        const int64_t n_rtc = ceil_div(nc, 256);
        if (n_rtc * n_cg > ((int64_t)1 << 31) - 1) throw Error(BEM_ERR_INVALID, "too many centroid rows");
        hipLaunchKernelGGL(k_nodal_kp_assemble, dim3((unsigned)(n_rtc * n_cg)), dim3(256), 0, s, nc, nv, ld, n_rtc,
                           c->nod_trow.as<int32_t>(), c->grp_ptr.as<int32_t>(), c->grp_tri.as<int32_t>(),
                           c->grp_loc.as<uint32_t>(), c->pan64.as<double>(), c->tri64.as<double>(), Kc);
        BEM_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_nodal_kp_near, dim3((unsigned)ceil_div(nc, 64)), dim3(64), 0, s, nc, ld, c->N, Np,
                           c->nod_trow.as<int32_t>(), c->tri.as<int32_t>(), c->far64.as<double>(),
                           c->nodal_bounds.as<double>(), c->tri64.as<double>(), Kc);
        BEM_CHECK_LAUNCH();
        if (niv > 0) {
            hipLaunchKernelGGL(k_nodal_iface_rows<T>, dim3((unsigned)niv), dim3(256), 0, s, nv, ld,
                               c->nod_iface_v.as<int32_t>(), c->fan_ptr.as<int32_t>(), c->fan.as<int32_t>(),
                               c->tri.as<int32_t>(), c->nod_tri_crow.as<int32_t>(), c->vert_body.as<int32_t>(),
                               c->body_epsp.as<double>(), c->body_epsm.as<double>(), c->tri64.as<double>(), mass, Kc,
                               A);
            BEM_CHECK_LAUNCH();
        }
    }
    hipLaunchKernelGGL(k_nodal_diag<T>, dim3((unsigned)ceil_div(nv, 256)), dim3(256), 0, s, nv, ld, A,
                       c->diag.as<double>());
    BEM_CHECK_LAUNCH();
    if (ld > nv) {
        hipLaunchKernelGGL(k_nodal_tail<T>, dim3((unsigned)ceil_div(nv * (ld - nv), 256)), dim3(256), 0, s, nv, ld,
                           c->vert_body.as<int32_t>(), c->body_kind.as<int32_t>(), c->body_fidx.as<int32_t>(), A);
        BEM_CHECK_LAUNCH();
    }
    if (c->n_float > 0) {
        double* Af = mass + nv;
        hipLaunchKernelGGL(k_nodal_body_area, dim3((unsigned)c->n_float), dim3(256), 0, s, nv,
                           c->vert_body.as<int32_t>(), c->body_fidx.as<int32_t>(), mass, Af);
        BEM_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_nodal_constraint, dim3((unsigned)ceil_div((int64_t)c->n_float * ld, 256)), dim3(256), 0,
                           s, nv, tail_row0, ld, c->n_float, c->vert_body.as<int32_t>(), c->body_fidx.as<int32_t>(),
                           mass, Af, Atail, c->diag.as<double>());
        BEM_CHECK_LAUNCH();
        if (!c->h_flt_kp.empty()) {   // rows with a K' term replace their net-charge rows
            hipLaunchKernelGGL(k_nodal_kp_body_rows, dim3((unsigned)ceil_div(ld, 256), (unsigned)c->h_flt_kp.size()),
                               dim3(256), 0, s, nv, ld, tail_row0, c->nod_flist.as<int32_t>(),
                               c->nod_frange.as<int32_t>(), c->flt_coef.as<double>(), c->nod_trow.as<int32_t>(),
                               c->vert_body.as<int32_t>(), c->body_fidx.as<int32_t>(), c->tri64.as<double>(), mass, Af,
                               c->nod_Kc.as<double>(), Atail, c->diag.as<double>());
            BEM_CHECK_LAUNCH();
        }
    }
}

void launch_nodal_assemble(bem_ctx* c) {
    KTimer kt(c, "nodal_assemble");
    if (c->opt.precision == BEM_MIXED)   // vertex rows FP32 in A32, constraint rows FP64 from row 0 of A64
        nodal_assemble_t<float>(c, c->A32.as<float>(), c->A64.as<double>(), 0);
    else
        nodal_assemble_t<double>(c, c->A64.as<double>(), c->A64.as<double>(), c->n_vert);
}

void launch_nodal_field(bem_ctx* c, int32_t nrhs, const double* sol, int64_t P, const double* pts, double* phi,
                        double* E) {
    KTimer kt(c, "nodal_field");
    if (P == 0) return;
    for (int32_t r0 = 0; r0 < nrhs; r0 += 65535) {   // load cases on grid.y
        const int32_t nr = nrhs - r0 < 65535 ? nrhs - r0 : 65535;
        hipLaunchKernelGGL(k_nodal_field, dim3((unsigned)ceil_div(P, 64), (unsigned)nr), dim3(256), 0, c->stream, P,
                           pts, c->N, c->tri.as<int32_t>(), c->pan64.as<double>(), c->tri64.as<double>(),
                           sol + (int64_t)r0 * c->n, c->n, phi ? phi + (int64_t)r0 * P : nullptr,
                           E ? E + (int64_t)r0 * P * 3 : nullptr);
        BEM_CHECK_LAUNCH();
    }
}

}  // namespace bem
