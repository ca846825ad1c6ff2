// Gradient of the streamer integrals with respect to the mesh vertices and the
// body potentials (reverse mode; the forward method is Secs. 1, 2 and 4).
//
// J = sum_l g_l I_l depends on the charges sigma (through the field on the
// lines), on the geometry directly (the field kernel of every panel, the line
// starts that sit on panels) and through sigma, which solves A u = b:
//   sigma_bar_j = sum over stage points X of ebar(X) . F_j(X)   (transposed field)
//   A^T lambda = [sigma_bar, 0]
//   dJ/dV_k     = sum of lambda_i over the conductor rows of body k
//   dJ/dgeom   += sum over (X, j) of sigma_j ebar(X) . dF_j(X)/dgeom
//               - lambda^T (dA/dgeom) u
// The pair terms are split by side.  Panel side (the three vertices of panel
// j): k_pan_far_adj for regular pairs by the 7-point rule, differentiated by
// hand (node positions and the area in the weights), k_pan_near_adj for the
// others with the closed forms in dual numbers.  Point side (collocation point
// x_i and normal n_i of row i): E and dE/dx at the centroids from
// adjoint_field.hip.  Per-panel adjoints of corners, area, normal and centroid
// are turned into vertex gradients at the end, each vertex summing its
// incident corners in a fixed order.  Every sum has a fixed order, so the
// gradient is bitwise reproducible.
#include <algorithm>
#include <cstring>
#include <vector>

#include "adjoint_device.h"

namespace bem {

void launch_reverse_sweep(bem_ctx* c, const double* sol, int64_t L, const int32_t* line_rhs, const int32_t* ns,
                          const double* path, int64_t pstride, const bem_trace_params* tp, const double* gI,
                          const int64_t* sbase, int32_t max_ns, double* SX, double* SE, double* x0bar);
void launch_rows_EH(bem_ctx* c, const double* sigma, int64_t P, const double* pts, double* out);
int gmres_solve_t(bem_ctx* c, const double* b, double* x, double tol, int max_iter, int* iters, double* relres);

namespace {

constexpr int PA_TILE = 64;    // points per LDS tile in k_pan_far_adj
constexpr int PA_ACC = 11;     // per-panel accumulators: T_far, T_near, 9 corner components

__device__ __forceinline__ void quad7_bary(int q, double& b0, double& b1, double& b2) {
    const double s15 = sqrt(15.0);
    const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
    if (q == 0) {
        b0 = b1 = b2 = 1.0 / 3.0;
        return;
    }
    const double a = q < 4 ? a1 : a2;
    const int r = (q - 1) % 3;   // position of 1 - 2a
    b0 = (r == 2) ? 1.0 - 2.0 * a : a;
    b1 = (r == 1) ? 1.0 - 2.0 * a : a;
    b2 = (r == 0) ? 1.0 - 2.0 * a : a;
}

// ---- panel-major near lists from (panel group, point) ballot masks --------------------
// mask[(j >> 6) * P + p] bit (j & 63) marks the pair (p, j) as not regular.
__global__ __launch_bounds__(64) void k_pm_count(const uint64_t* __restrict__ mask, int64_t P, int64_t N, int64_t chunk,
                                                 int32_t* __restrict__ cnt) {
    const int64_t g = blockIdx.x, pb = blockIdx.y;
    const int64_t j = g * 64 + threadIdx.x;
    const int64_t p0 = pb * chunk, p1 = std::min<int64_t>(P, p0 + chunk);
    int c = 0;
    for (int64_t p = p0; p < p1; ++p) c += (int)((mask[g * P + p] >> threadIdx.x) & 1ull);
    if (j < N) cnt[pb * N + j] = c;
}

// ptr[0] = 0, ptr[j + 1] = ptr[j] + sum_pb cnt[pb][j]; one block.
__global__ __launch_bounds__(1024) void k_pm_scan(const int32_t* __restrict__ cnt, int64_t N, int PB,
                                                  int64_t* __restrict__ ptr) {
    __shared__ int64_t part[1024];
    const int64_t per = (N + 1023) / 1024;
    const int64_t j0 = threadIdx.x * per, j1 = std::min<int64_t>(N, j0 + per);
    int64_t s = 0;
    for (int64_t j = j0; j < j1; ++j)
        for (int pb = 0; pb < PB; ++pb) s += cnt[(int64_t)pb * N + j];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int t = 0; t < 1024; ++t) {
            const int64_t v = part[t];
            part[t] = run;
            run += v;
        }
        ptr[0] = 0;
    }
    __syncthreads();
    int64_t run = part[threadIdx.x];
    for (int64_t j = j0; j < j1; ++j) {
        for (int pb = 0; pb < PB; ++pb) run += cnt[(int64_t)pb * N + j];
        ptr[j + 1] = run;
    }
}

__global__ __launch_bounds__(64) void k_pm_fill(const uint64_t* __restrict__ mask, int64_t P, int64_t N, int64_t chunk,
                                                const int32_t* __restrict__ cnt, const int64_t* __restrict__ ptr,
                                                int32_t* __restrict__ list) {
    const int64_t g = blockIdx.x, pb = blockIdx.y;
    const int64_t j = g * 64 + threadIdx.x;
    if (j >= N) return;
    int64_t pos = ptr[j];
    for (int64_t b = 0; b < pb; ++b) pos += cnt[b * N + j];
    const int64_t p0 = pb * chunk, p1 = std::min<int64_t>(P, p0 + chunk);
    for (int64_t p = p0; p < p1; ++p)
        if ((mask[g * P + p] >> threadIdx.x) & 1ull) list[pos++] = (int32_t)p;
}

// ---- panel side, regular pairs ------------------------------------------------------
// For panel j (one per lane) and the points of this block's range: with the pair value
// G = a_p S_j(x_p) + c_p . F_j(x_p) (7-point rule), accumulates T = sum G and the
// derivatives of sum G with respect to the three vertices at fixed area (node positions
// y_q = sum_k beta_qk v_k); the area part is added when folding (G is linear in the area).
__global__ __launch_bounds__(256) void k_pan_far_adj(const double* __restrict__ far64, int64_t Np, int64_t N,
                                                     int64_t P, int64_t span, const double* __restrict__ pts,
                                                     const double* __restrict__ aw, const double* __restrict__ cw,
                                                     int self_mode, int64_t p_off, double* __restrict__ part) {
    __shared__ double tp[PA_TILE][7];
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool valid = j < N;
    const int64_t jj = valid ? j : N - 1;
    double yq[7][3], wq[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        yq[q][0] = far64[(int64_t)(FR_X + q) * Np + jj];
        yq[q][1] = far64[(int64_t)(FR_Y + q) * Np + jj];
        yq[q][2] = far64[(int64_t)(FR_Z + q) * Np + jj];
        wq[q] = far64[(int64_t)(FR_W + q) * Np + jj];
    }
    const double cc0 = far64[(int64_t)(FR_CC + 0) * Np + jj], cc1 = far64[(int64_t)(FR_CC + 1) * Np + jj];
    const double cc2 = far64[(int64_t)(FR_CC + 2) * Np + jj], rr = far64[(int64_t)FR_RR * Np + jj];
    double T = 0.0, G[7][3];
#pragma unroll
    for (int q = 0; q < 7; ++q) G[q][0] = G[q][1] = G[q][2] = 0.0;
    const int64_t p_beg = (int64_t)blockIdx.y * span;
    const int64_t p_end = std::min<int64_t>(P, p_beg + span);
    for (int64_t t0 = p_beg; t0 < p_end; t0 += PA_TILE) {
        __syncthreads();
        for (int e = threadIdx.x; e < PA_TILE * 7; e += 256) {
            const int pi = e / 7, comp = e % 7;
            const int64_t p = t0 + pi;
            double v = 0.0;
            if (p < p_end) {
                if (comp < 3)
                    v = pts[3 * p + comp];
                else if (comp == 3)
                    v = aw ? aw[p] : 0.0;
                else
                    v = cw[3 * p + comp - 4];
            }
            tp[pi][comp] = v;
        }
        __syncthreads();
        const int cnt = (int)std::min<int64_t>(PA_TILE, p_end - t0);
        if (!valid) continue;
        for (int pi = 0; pi < cnt; ++pi) {
            const double x0 = tp[pi][0], x1 = tp[pi][1], x2 = tp[pi][2];
            if (self_mode && t0 + pi + p_off == j) continue;
            if (!is_regular(x0 - cc0, x1 - cc1, x2 - cc2, rr)) continue;
            const double a = tp[pi][3], c0 = tp[pi][4], c1 = tp[pi][5], c2 = tp[pi][6];
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                const double dx = x0 - yq[q][0], dy = x1 - yq[q][1], dz = x2 - yq[q][2];
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double ir = rsqrt_pos(r2);
                const double ir2 = ir * ir;
                const double t1 = wq[q] * ir;        // w / r
                const double t3 = t1 * ir2;          // w / r^3
                const double cd = c0 * dx + c1 * dy + c2 * dz;
                T += a * t1 + t3 * cd;
                // dG/dy_q = (a w / r^3 + 3 w (c.d) / r^5) d - (w / r^3) c
                const double coef = t3 * (a + 3.0 * cd * ir2);
                G[q][0] += coef * dx - t3 * c0;
                G[q][1] += coef * dy - t3 * c1;
                G[q][2] += coef * dz - t3 * c2;
            }
        }
    }
    if (!valid) return;
    double* o = part + ((int64_t)blockIdx.y * N + j) * 10;
    o[0] = T;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            double b[3];
            quad7_bary(q, b[0], b[1], b[2]);
            g0 += b[k] * G[q][0];
            g1 += b[k] * G[q][1];
            g2 += b[k] * G[q][2];
        }
        o[1 + 3 * k] = g0;
        o[2 + 3 * k] = g1;
        o[3 + 3 * k] = g2;
    }
}

// acc[j] (T_far, T_near, corners) = sum over the KS partials (fixed order)
__global__ __launch_bounds__(256) void k_pan_reduce(const double* __restrict__ part, int64_t KS, int64_t N,
                                                    double* __restrict__ acc) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    double s[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) s[c] = 0.0;
    for (int64_t k = 0; k < KS; ++k)
#pragma unroll
        for (int c = 0; c < 10; ++c) s[c] += part[(k * N + j) * 10 + c];
    double* a = acc + j * PA_ACC;
    a[0] += s[0];
#pragma unroll
    for (int c = 1; c < 10; ++c) a[1 + c] += s[c];
}

// ---- panel side, near pairs: one wave per panel over its near points -----------------
__global__ __launch_bounds__(256) void k_pan_near_adj(const int64_t* __restrict__ ptr, const int32_t* __restrict__ list,
                                                      int64_t N, const double* __restrict__ tri64,
                                                      const double* __restrict__ pts, const double* __restrict__ aw,
                                                      const double* __restrict__ cw, int self_mode, int64_t p_off,
                                                      double* __restrict__ acc) {
    const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= N) return;
    const double* Tj = tri64 + (int64_t)TRI_REC * j;
    double vv[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) vv[k][c] = Tj[TR_V + 3 * k + c];
    double T = 0.0, g[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) g[c] = 0.0;
    for (int64_t e = ptr[j] + lane; e < ptr[j + 1]; e += 64) {
        const int64_t p = list[e];
        const bool self = self_mode && p + p_off == j;
        const double a = aw ? aw[p] : 0.0;
        // the constant zero K'_ii of the own panel carries no derivative: no field term for self
        const double c0 = self ? 0.0 : cw[3 * p], c1 = self ? 0.0 : cw[3 * p + 1], c2 = self ? 0.0 : cw[3 * p + 2];
        for (int k = 0; k < 3; ++k) {
            D3 V[3][3], X[3];
#pragma unroll
            for (int kk = 0; kk < 3; ++kk)
#pragma unroll
                for (int c = 0; c < 3; ++c) V[kk][c] = (kk == k) ? d3seed(vv[kk][c], c, 1.0) : d3(vv[kk][c]);
#pragma unroll
            for (int c = 0; c < 3; ++c)
                X[c] = self ? d3seed(pts[3 * p + c], c, 1.0 / 3.0) : d3(pts[3 * p + c]);
            D3 S, F[3];
            tri_SF_d3(V, X, self, S, F);
            const D3 Gv = S * a + F[0] * c0 + F[1] * c1 + F[2] * c2;
            if (k == 0) T += Gv.v;
            g[3 * k] += Gv.d0;
            g[3 * k + 1] += Gv.d1;
            g[3 * k + 2] += Gv.d2;
        }
    }
    T = wave_sum(T);
#pragma unroll
    for (int c = 0; c < 9; ++c) g[c] = wave_sum(g[c]);
    if (lane == 0) {
        double* o = acc + j * PA_ACC;
        o[1] += T;
#pragma unroll
        for (int c = 0; c < 9; ++c) o[2 + c] += g[c];
    }
}

// GV[j][k] += sgn sigma_j (corner_k + (da/dv_k / a) T_far); sigbar[j] = T_far + T_near; acc cleared
__global__ __launch_bounds__(256) void k_pan_fold(double* __restrict__ acc, int64_t N, const double* __restrict__ tri64,
                                                  const double* __restrict__ sigma, double sgn,
                                                  double* __restrict__ GV, double* __restrict__ sigbar) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    double* a = acc + j * PA_ACC;
    const double* T = tri64 + (int64_t)TRI_REC * j;
    const double n0 = T[TR_N], n1 = T[TR_N + 1], n2 = T[TR_N + 2], area = T[TR_A];
    const double s = sgn * sigma[j];
    const double tf = a[0] / area;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        // da/dv_k = -(1/2) n x e_k with e_k = v_{k+1} - v_{k+2}
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        const double e0 = T[3 * k1] - T[3 * k2], e1 = T[3 * k1 + 1] - T[3 * k2 + 1], e2 = T[3 * k1 + 2] - T[3 * k2 + 2];
        const double da0 = -0.5 * (n1 * e2 - n2 * e1), da1 = -0.5 * (n2 * e0 - n0 * e2), da2 = -0.5 * (n0 * e1 - n1 * e0);
        GV[j * 9 + 3 * k] += s * (a[2 + 3 * k] + da0 * tf);
        GV[j * 9 + 3 * k + 1] += s * (a[3 + 3 * k] + da1 * tf);
        GV[j * 9 + 3 * k + 2] += s * (a[4 + 3 * k] + da2 * tf);
    }
    if (sigbar) sigbar[j] = a[0] + a[1];
#pragma unroll
    for (int c = 0; c < PA_ACC; ++c) a[c] = 0.0;
}

// ---- point side of the system rows ------------------------------------------------------
// Q_i of the constraint rows (floating panels): Q = c_self sigma_i + c_kp n_i . E_i with the
// body's coefficients coef[2f], coef[2f+1] (closed body literal (1/2, 1) or reduced (1, 0),
// thin sheet (1, 2 (eps+ - eps-) / (eps+ + eps-)), Eq. Final4 and Eq. sheets).
__global__ __launch_bounds__(256) void k_row_Q(int64_t N, const int32_t* __restrict__ tri_body,
                                               const int32_t* __restrict__ body_kind,
                                               const int32_t* __restrict__ fidx, const double* __restrict__ coef,
                                               const double* __restrict__ tri64, const double* __restrict__ sigma,
                                               const double* __restrict__ EH, double* __restrict__ Q) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const int32_t b = tri_body[i];
    if (body_kind[b] != BEM_FLOATING) {
        Q[i] = 0.0;
        return;
    }
    const int f = fidx[b];
    const double* T = tri64 + (int64_t)TRI_REC * i;
    const double* e = EH + i * 9;
    Q[i] = coef[2 * f] * sigma[i] + coef[2 * f + 1] * (T[TR_N] * e[0] + T[TR_N + 1] * e[1] + T[TR_N + 2] * e[2]);
}

// Per floating body f (one block each, panels rows_flt[s0[f] .. s0[f+1])): A_f = sum a_i and
// c_f = sum a_i Q_i / A_f, fixed-order block sums.
__global__ __launch_bounds__(256) void k_float_sums(const int32_t* __restrict__ rows_flt,
                                                    const int64_t* __restrict__ seg, const double* __restrict__ tri64,
                                                    const double* __restrict__ Q, double* __restrict__ Af,
                                                    double* __restrict__ cf) {
    __shared__ double red[2][4];
    const int f = blockIdx.x;
    double sa = 0.0, sq = 0.0;
    for (int64_t s = seg[f] + threadIdx.x; s < seg[f + 1]; s += 256) {
        const int64_t i = rows_flt[s];
        const double a = tri64[(int64_t)TRI_REC * i + TR_A];
        sa += a;
        sq += a * Q[i];
    }
    sa = wave_sum(sa);
    sq = wave_sum(sq);
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = sa;
        red[1][threadIdx.x >> 6] = sq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double A = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        const double S = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        Af[f] = A;
        cf[f] = S / A;
    }
}

// Row weights and the point-side terms of -lambda^T (dA) u for row i:
//   wS = lambda_i on conductor/floating rows, wK = lambda_i (eps+ - eps-) on interface rows,
//   plus lambda_f c_kp a_i / A_f on floating rows;
//   GX_i -= -wS E_i + wK H_i n_i,  GN_i -= wK E_i,  GA_i -= lambda_f (Q_i - c_f) / A_f.
__global__ __launch_bounds__(256) void k_row_adj(int64_t N, const int32_t* __restrict__ tri_body,
                                                 const int32_t* __restrict__ body_kind, const double* __restrict__ epsp,
                                                 const double* __restrict__ epsm, const int32_t* __restrict__ fidx,
                                                 const double* __restrict__ tri64, const double* __restrict__ lam,
                                                 const double* __restrict__ EH, const double* __restrict__ Q,
                                                 const double* __restrict__ Af, const double* __restrict__ cf,
                                                 const double* __restrict__ coef, double* __restrict__ aw,
                                                 double* __restrict__ cw,
                                                 double* __restrict__ GX, double* __restrict__ GN,
                                                 double* __restrict__ GA) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= N) return;
    const int32_t b = tri_body[i], kind = body_kind[b];
    const double* T = tri64 + (int64_t)TRI_REC * i;
    const double n0 = T[TR_N], n1 = T[TR_N + 1], n2 = T[TR_N + 2], area = T[TR_A];
    double wS = 0.0, wK = 0.0;
    if (kind == BEM_INTERFACE)
        wK = lam[i] * (epsp[b] - epsm[b]);
    else
        wS = lam[i];
    if (kind == BEM_FLOATING) {
        const int f = fidx[b];
        const double lf = lam[N + f];
        wK += lf * coef[2 * f + 1] * area / Af[f];
        GA[i] -= lf * (Q[i] - cf[f]) / Af[f];
    }
    const double* e = EH + i * 9;   // E (3), H xx yy zz xy xz yz
    const double hn0 = e[3] * n0 + e[6] * n1 + e[7] * n2;
    const double hn1 = e[6] * n0 + e[4] * n1 + e[8] * n2;
    const double hn2 = e[7] * n0 + e[8] * n1 + e[5] * n2;
    GX[3 * i] -= -wS * e[0] + wK * hn0;
    GX[3 * i + 1] -= -wS * e[1] + wK * hn1;
    GX[3 * i + 2] -= -wS * e[2] + wK * hn2;
    GN[3 * i] -= wK * e[0];
    GN[3 * i + 1] -= wK * e[1];
    GN[3 * i + 2] -= wK * e[2];
    aw[i] = wS;
    cw[3 * i] = wK * n0;
    cw[3 * i + 1] = wK * n1;
    cw[3 * i + 2] = wK * n2;
}

// dJ/dV[r][b] = sum of lambda_i over the conductor rows of body b (one block per body)
__global__ __launch_bounds__(256) void k_dV(int64_t N, const int32_t* __restrict__ tri_body,
                                            const int32_t* __restrict__ body_kind, const double* __restrict__ lam,
                                            double* __restrict__ out) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    double s = 0.0;
    if (body_kind[b] == BEM_DIRICHLET)
        for (int64_t i = threadIdx.x; i < N; i += 256)
            if (tri_body[i] == b) s += lam[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[b] = (red[0] + red[1]) + (red[2] + red[3]);
}

// line starts x0 = sum_k bary_k v_k + offset n of their panel: corner and normal adjoints
__global__ __launch_bounds__(256) void k_start_adj(int64_t N, int64_t L, const int32_t* __restrict__ start_panel,
                                                   const double* __restrict__ bary, const double* __restrict__ x0bar,
                                                   double offset, double* __restrict__ GV, double* __restrict__ GN) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    for (int64_t l = 0; l < L; ++l) {
        if (start_panel[l] != j) continue;
        const double x0 = x0bar[3 * l], x1 = x0bar[3 * l + 1], x2 = x0bar[3 * l + 2];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double b = bary[3 * l + k];
            GV[j * 9 + 3 * k] += b * x0;
            GV[j * 9 + 3 * k + 1] += b * x1;
            GV[j * 9 + 3 * k + 2] += b * x2;
        }
        GN[3 * j] += offset * x0;
        GN[3 * j + 1] += offset * x1;
        GN[3 * j + 2] += offset * x2;
    }
}

// corner adjoints: C[j][k] = GV[j][k] + GA_j da/dv_k + (dn/dv_k)^T GN_j + GX_j / 3
__global__ __launch_bounds__(256) void k_corners(int64_t N, const double* __restrict__ tri64,
                                                 const double* __restrict__ GV, const double* __restrict__ GX,
                                                 const double* __restrict__ GN, const double* __restrict__ GA,
                                                 double* __restrict__ C) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    const double* T = tri64 + (int64_t)TRI_REC * j;
    const double n0 = T[TR_N], n1 = T[TR_N + 1], n2 = T[TR_N + 2], area = T[TR_A];
    // p = (I - n n^T) GN / (2 a)
    const double g0 = GN[3 * j], g1 = GN[3 * j + 1], g2 = GN[3 * j + 2];
    const double gn = g0 * n0 + g1 * n1 + g2 * n2;
    const double i2a = 0.5 / area;
    const double p0 = (g0 - gn * n0) * i2a, p1 = (g1 - gn * n1) * i2a, p2 = (g2 - gn * n2) * i2a;
    const double ga = GA[j];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
        const double e0 = T[3 * k1] - T[3 * k2], e1 = T[3 * k1 + 1] - T[3 * k2 + 1], e2 = T[3 * k1 + 2] - T[3 * k2 + 2];
        // da/dv_k = -(1/2) n x e_k ; dn/dv_k^T GN = e_k x p
        const double da0 = -0.5 * (n1 * e2 - n2 * e1), da1 = -0.5 * (n2 * e0 - n0 * e2), da2 = -0.5 * (n0 * e1 - n1 * e0);
        const double q0 = e1 * p2 - e2 * p1, q1 = e2 * p0 - e0 * p2, q2 = e0 * p1 - e1 * p0;
        C[j * 9 + 3 * k] = GV[j * 9 + 3 * k] + ga * da0 + q0 + GX[3 * j] / 3.0;
        C[j * 9 + 3 * k + 1] = GV[j * 9 + 3 * k + 1] + ga * da1 + q1 + GX[3 * j + 1] / 3.0;
        C[j * 9 + 3 * k + 2] = GV[j * 9 + 3 * k + 2] + ga * da2 + q2 + GX[3 * j + 2] / 3.0;
    }
}

// dJ/dvert[v] = sum of the corner adjoints at v, in the order of the vertex's corner list
__global__ __launch_bounds__(256) void k_vertex_gather(int64_t n_vert, const int32_t* __restrict__ vptr,
                                                       const int32_t* __restrict__ vcorner,
                                                       const double* __restrict__ C, double* __restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n_vert) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int32_t e = vptr[v]; e < vptr[v + 1]; ++e) {
        const int64_t cidx = vcorner[e];
        s0 += C[3 * cidx];
        s1 += C[3 * cidx + 1];
        s2 += C[3 * cidx + 2];
    }
    out[3 * v] = s0;
    out[3 * v + 1] = s1;
    out[3 * v + 2] = s2;
}

__global__ __launch_bounds__(256) void k_zero(double* __restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

__global__ __launch_bounds__(256) void k_centroids(int64_t N, const double* __restrict__ tri64, double* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) out[3 * j + k] = tri64[(int64_t)TRI_REC * j + TR_C + k];
}

__global__ __launch_bounds__(256) void k_pad_rhs(const double* __restrict__ sigbar, int64_t N, int64_t n,
                                                 double* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = i < N ? sigbar[i] : 0.0;
}

void zero(bem_ctx* c, double* p, int64_t n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->stream, p, n);
    BEM_CHECK_LAUNCH();
}

// Panel-side pair terms over a point set: acc += (T_far, T_near, corner derivatives) of
// sum_p [a_p S_j(x_p) + c_p . F_j(x_p)] for every panel j.  self_mode: point p is the
// centroid of panel p (the point moves with its panel).  Points go in batches of grad_batch.
void panel_side(bem_ctx* c, int64_t P, const double* pts, const double* aw, const double* cw, bool self_mode,
                double* acc) {
    const int64_t N = c->N;
    const int64_t Np = (int64_t)(c->far64.bytes / (sizeof(double) * FAR_REC));
    const int64_t nblk = ceil_div(N, 64);
    const int64_t B = std::min<int64_t>(P, c->grad_batch);   // points per batch
    c->ad_mask.alloc(sizeof(uint64_t) * (size_t)nblk * B);
    const int PB = 32;
    c->ad_cnt.alloc(sizeof(int32_t) * (size_t)PB * N + sizeof(int64_t) * (N + 2));   // + alignment pad
    int32_t* cnt = c->ad_cnt.as<int32_t>();
    int64_t* ptr = reinterpret_cast<int64_t*>(cnt + (size_t)PB * N + (N & 1));
    c->ad_self.alloc(sizeof(int32_t) * (size_t)B);
    int32_t* host32 = c->host_stage.as<int32_t>();
    for (int64_t b0 = 0; b0 < P; b0 += B) {
        const int64_t nb = std::min<int64_t>(B, P - b0);
        const double* bp = pts + 3 * b0;
        const double* ba = aw ? aw + b0 : nullptr;
        const double* bc = cw + 3 * b0;
        // regular pairs
        {
            KTimer t(c, "grad_panel_far");
            const int64_t pb = ceil_div(N, 256);
            int64_t KS = std::max<int64_t>(1, 2048 / pb);
            KS = std::min<int64_t>(KS, ceil_div(nb, PA_TILE));
            const int64_t span = ceil_div(ceil_div(nb, KS), PA_TILE) * PA_TILE;
            KS = ceil_div(nb, span);
            c->ad_ppart.alloc(sizeof(double) * 10 * (size_t)KS * N);
            hipLaunchKernelGGL(k_pan_far_adj, dim3((unsigned)pb, (unsigned)KS), dim3(256), 0, c->stream,
                               c->far64.as<double>(), Np, N, nb, span, bp, ba, bc, (int)self_mode, b0,
                               c->ad_ppart.as<double>());
            BEM_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_pan_reduce, dim3((unsigned)pb), dim3(256), 0, c->stream, c->ad_ppart.as<double>(), KS,
                               N, acc);
            BEM_CHECK_LAUNCH();
        }
        // near pairs: masks -> panel-major lists -> closed forms in dual numbers
        {
            KTimer t(c, "grad_panel_near");
            const int32_t* op = nullptr;
            if (self_mode) {
                std::vector<int32_t> iota(nb);   // point i of the batch is the centroid of panel b0 + i
                for (int64_t i = 0; i < nb; ++i) iota[i] = (int32_t)(b0 + i);
                BEM_HIP(hipMemcpyAsync(c->ad_self.p, iota.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice,
                                       c->stream));
                BEM_HIP(hipStreamSynchronize(c->stream));
                op = c->ad_self.as<int32_t>();
            }
            launch_point_mask(c, nb, bp, op, c->ad_mask.as<uint64_t>());
            const int64_t chunk = ceil_div(nb, PB);
            hipLaunchKernelGGL(k_pm_count, dim3((unsigned)nblk, PB), dim3(64), 0, c->stream, c->ad_mask.as<uint64_t>(),
                               nb, N, chunk, cnt);
            BEM_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_pm_scan, dim3(1), dim3(1024), 0, c->stream, cnt, N, PB, ptr);
            BEM_CHECK_LAUNCH();
            int64_t nnz = 0;
            BEM_HIP(hipMemcpyAsync(host32, ptr + N, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
            BEM_HIP(hipStreamSynchronize(c->stream));
            std::memcpy(&nnz, host32, sizeof(int64_t));
            if (nnz >= ((int64_t)1 << 31)) throw Error(BEM_ERR_INVALID, "gradient near list exceeds 2^31 pairs");
            c->ad_list.alloc(sizeof(int32_t) * (size_t)std::max<int64_t>(nnz, 1));
            hipLaunchKernelGGL(k_pm_fill, dim3((unsigned)nblk, PB), dim3(64), 0, c->stream, c->ad_mask.as<uint64_t>(),
                               nb, N, chunk, cnt, ptr, c->ad_list.as<int32_t>());
            BEM_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_pan_near_adj, dim3((unsigned)ceil_div(N, 4)), dim3(256), 0, c->stream, ptr,
                               c->ad_list.as<int32_t>(), N, c->tri64.as<double>(), bp, ba, bc, (int)self_mode, b0, acc);
            BEM_CHECK_LAUNCH();
        }
    }
}

}  // namespace

// Gradient of J = sum_l gI[l] I_l.  See include/bem.h (bem_streamer_grad).
void streamer_grad(bem_ctx* c, int32_t nrhs, const double* sol, int64_t L, const int32_t* line_rhs,
                   const double* starts, const int32_t* start_panel, const double* start_bary,
                   const bem_trace_params* tp, const double* gI, double tol, double* dvert, double* dV,
                   double* dstart) {
    KTimer tall(c, "grad");
    const int64_t N = c->N, n = c->n, nv = c->n_vert;
    hipStream_t s = c->stream;
    // 1. forward run with paths (classification, step counts and stops of the forward method)
    const int64_t pstride = 3 * ((int64_t)tp->max_steps + 1);
    c->ad_path.alloc(sizeof(double) * (size_t)std::max<int64_t>(L, 1) * pstride + sizeof(int32_t) * 2 * (L + 16));
    double* path = c->ad_path.as<double>();
    int32_t* ns = reinterpret_cast<int32_t*>(path + (size_t)std::max<int64_t>(L, 1) * pstride);
    int32_t* stop = ns + L + 16;
    if (L > 0) launch_trace_batched(c, nrhs, sol, L, line_rhs, starts, tp, ns, stop, path, nullptr, nullptr, false);
    // 2. lines grouped by load case; stage-record offsets
    std::vector<int32_t> h_ns(L), h_rhs(L, 0);
    if (L > 0) {
        BEM_HIP(hipMemcpyAsync(h_ns.data(), ns, sizeof(int32_t) * L, hipMemcpyDeviceToHost, s));
        if (line_rhs) BEM_HIP(hipMemcpyAsync(h_rhs.data(), line_rhs, sizeof(int32_t) * L, hipMemcpyDeviceToHost, s));
        BEM_HIP(hipStreamSynchronize(s));
    }
    std::vector<int64_t> sbase(L), rbeg(nrhs + 1, 0);
    int32_t max_ns = 0;
    {
        int64_t off = 0;
        for (int32_t r = 0; r < nrhs; ++r) {
            rbeg[r] = off;
            for (int64_t l = 0; l < L; ++l)
                if (h_rhs[l] == r) {
                    sbase[l] = off;
                    off += 4 * (int64_t)h_ns[l];
                    max_ns = std::max(max_ns, h_ns[l]);
                }
        }
        rbeg[nrhs] = off;
    }
    const int64_t P = rbeg[nrhs];
    c->ad_stage.alloc(sizeof(double) * 6 * (size_t)std::max<int64_t>(P, 1) + sizeof(int64_t) * (L + 1) +
                      sizeof(double) * 3 * (L + 1));
    double* SX = c->ad_stage.as<double>();
    double* SE = SX + 3 * std::max<int64_t>(P, 1);
    int64_t* d_sbase = reinterpret_cast<int64_t*>(SE + 3 * std::max<int64_t>(P, 1));
    double* x0bar = reinterpret_cast<double*>(d_sbase + L + 1);
    if (L > 0) {
        BEM_HIP(hipMemcpyAsync(d_sbase, sbase.data(), sizeof(int64_t) * L, hipMemcpyHostToDevice, s));
        // 3. reverse sweep
        launch_reverse_sweep(c, sol, L, line_rhs, ns, path, pstride, tp, gI, d_sbase, max_ns, SX, SE, x0bar);
    }
    // 4. per-panel adjoint buffers
    const size_t accs = (size_t)N * PA_ACC;
    c->ad_geo.alloc(sizeof(double) * ((size_t)N * (9 + 3 + 3 + 1 + 9 + 9 + 3 + 1 + 3) + accs + 3 * n + 64));
    double* GV = c->ad_geo.as<double>();
    double* GX = GV + 9 * N;
    double* GN = GX + 3 * N;
    double* GA = GN + 3 * N;
    double* EH = GA + N;
    double* C = EH + 9 * N;
    double* cwb = C + 9 * N;
    double* awb = cwb + 3 * N;
    double* cen = awb + N;
    double* acc = cen + 3 * N;
    double* sigbar = acc + accs;   // [n]
    double* lam = sigbar + n;      // [n]
    double* Qb = lam + n;          // [n] (N used)
    double* Af = Qb + n;           // [64] floating sums
    zero(c, GV, (int64_t)N * (9 + 3 + 3 + 1));
    zero(c, acc, (int64_t)accs);
    hipLaunchKernelGGL(k_centroids, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, N, c->tri64.as<double>(), cen);
    BEM_CHECK_LAUNCH();
    // floating-body segments
    std::vector<int64_t> seg(c->n_float + 1, 0);
    {
        int64_t s0 = 0;
        for (int32_t f = 0; f < c->n_float; ++f) {
            int32_t fb = -1;
            for (int32_t b = 0; b < c->n_body; ++b)
                if (c->h_body_fidx[b] == f) fb = b;
            int64_t s1 = s0;
            while (s1 < (int64_t)c->h_rows_flt.size() && c->h_tri_body[c->h_rows_flt[s1]] == fb) ++s1;
            seg[f] = s0;
            s0 = s1;
        }
        seg[c->n_float] = s0;
    }
    if (c->n_float > 32) throw Error(BEM_ERR_INVALID, "gradient supports at most 32 floating bodies");
    c->ad_seg.alloc(sizeof(int64_t) * (seg.size() + 1));
    BEM_HIP(hipMemcpyAsync(c->ad_seg.p, seg.data(), sizeof(int64_t) * seg.size(), hipMemcpyHostToDevice, s));
    double* cf = Af + 32;
    for (int32_t r = 0; r < nrhs; ++r) {
        const double* sig_r = sol + (int64_t)r * n;
        // 5. trace terms: sigma_bar and panel-side geometry (ebar as the field weight)
        if (rbeg[r + 1] > rbeg[r])
            panel_side(c, rbeg[r + 1] - rbeg[r], SX + 3 * rbeg[r], nullptr, SE + 3 * rbeg[r], false, acc);
        hipLaunchKernelGGL(k_pan_fold, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, acc, N,
                           c->tri64.as<double>(), sig_r, 1.0, GV, sigbar);
        BEM_CHECK_LAUNCH();
        // 6. adjoint solve A^T lambda = [sigma_bar, 0]
        hipLaunchKernelGGL(k_pad_rhs, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, sigbar, N, n, sigbar);
        BEM_CHECK_LAUNCH();
        int it = 0;
        double rel = 0.0;
        const int rc = gmres_solve_t(c, sigbar, lam, tol, 20000, &it, &rel);
        if (rc != 0) throw Error(BEM_ERR_NOCONV, "adjoint GMRES did not converge");
        // 7. dJ/dV
        hipLaunchKernelGGL(k_dV, dim3((unsigned)c->n_body), dim3(256), 0, s, N, c->tri_body.as<int32_t>(),
                           c->body_kind.as<int32_t>(), lam, dV + (int64_t)r * c->n_body);
        BEM_CHECK_LAUNCH();
        // 8. matrix terms, point side: E and dE/dx at the centroids for sigma_r
        launch_rows_EH(c, sig_r, N, cen, EH);
        hipLaunchKernelGGL(k_row_Q, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, N, c->tri_body.as<int32_t>(),
                           c->body_kind.as<int32_t>(), c->body_fidx.as<int32_t>(), c->flt_coef.as<double>(),
                           c->tri64.as<double>(), sig_r, EH, Qb);
        BEM_CHECK_LAUNCH();
        if (c->n_float > 0) {
            hipLaunchKernelGGL(k_float_sums, dim3((unsigned)c->n_float), dim3(256), 0, s, c->rows_flt.as<int32_t>(),
                               c->ad_seg.as<int64_t>(), c->tri64.as<double>(), Qb, Af, cf);
            BEM_CHECK_LAUNCH();
        }
        hipLaunchKernelGGL(k_row_adj, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, N,
                           c->tri_body.as<int32_t>(), c->body_kind.as<int32_t>(), c->body_epsp.as<double>(),
                           c->body_epsm.as<double>(), c->body_fidx.as<int32_t>(), c->tri64.as<double>(), lam, EH, Qb,
                           Af, cf, c->flt_coef.as<double>(), awb, cwb, GX, GN, GA);
        BEM_CHECK_LAUNCH();
        // 9. matrix terms, panel side (row weights as point weights; self pairs move with the panel)
        panel_side(c, N, cen, awb, cwb, true, acc);
        hipLaunchKernelGGL(k_pan_fold, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, acc, N,
                           c->tri64.as<double>(), sig_r, -1.0, GV, (double*)nullptr);
        BEM_CHECK_LAUNCH();
    }
    // 10. line starts that move with their panels
    if (L > 0 && start_panel) {
        hipLaunchKernelGGL(k_start_adj, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, N, L, start_panel,
                           start_bary, x0bar, tp->start_offset, GV, GN);
        BEM_CHECK_LAUNCH();
    }
    if (dstart && L > 0)
        BEM_HIP(hipMemcpyAsync(dstart, x0bar, sizeof(double) * 3 * L, hipMemcpyDeviceToDevice, s));
    // 11. corners -> vertices
    hipLaunchKernelGGL(k_corners, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, N, c->tri64.as<double>(), GV, GX,
                       GN, GA, C);
    BEM_CHECK_LAUNCH();
    if (c->ad_vptr.bytes == 0) {
        std::vector<int32_t> vptr(nv + 1, 0), vc(3 * N);
        for (int64_t j = 0; j < N; ++j)
            for (int k = 0; k < 3; ++k) ++vptr[c->h_tri[3 * j + k] + 1];
        for (int64_t v = 0; v < nv; ++v) vptr[v + 1] += vptr[v];
        std::vector<int32_t> fill(vptr.begin(), vptr.end() - 1);
        for (int64_t j = 0; j < N; ++j)
            for (int k = 0; k < 3; ++k) vc[fill[c->h_tri[3 * j + k]]++] = (int32_t)(3 * j + k);
        c->ad_vptr.alloc(sizeof(int32_t) * (nv + 1));
        c->ad_vcorner.alloc(sizeof(int32_t) * 3 * N);
        BEM_HIP(hipMemcpyAsync(c->ad_vptr.p, vptr.data(), sizeof(int32_t) * (nv + 1), hipMemcpyHostToDevice, s));
        BEM_HIP(hipMemcpyAsync(c->ad_vcorner.p, vc.data(), sizeof(int32_t) * 3 * N, hipMemcpyHostToDevice, s));
        BEM_HIP(hipStreamSynchronize(s));
    }
    hipLaunchKernelGGL(k_vertex_gather, dim3((unsigned)ceil_div(nv, 256)), dim3(256), 0, s, nv,
                       c->ad_vptr.as<int32_t>(), c->ad_vcorner.as<int32_t>(), C, dvert);
    BEM_CHECK_LAUNCH();
}

}  // namespace bem
