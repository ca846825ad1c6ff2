// Reverse sweep of the field lines for the gradient of the streamer integrals
// (Sec. 1, Eq. Breakdowncrit), and field + field Jacobian at collocation points.
//
// The forward tracer (RK4 on dx/ds = dir E/|E| with the integral carried as an
// extra state) is differentiated step by step in reverse order.  Step n from
// x_n evaluates E at the stage points X_1..X_4; its reverse needs E and the
// Jacobian H = dE/dx at the same points, so each reverse step recomputes the
// four stages (four passes, all lines together, like the forward tracer) and
// then runs the adjoint of the step:
//   kbar_s  = h c_s xbar,           c = (1, 2, 2, 1) / 6
//   for s = 4..1:
//     ebar_s = dir (kbar_s - e_s (e_s . kbar_s)) / |E_s| + g h c_s alpha'(|E_s|) e_s
//     Xbar_s = H_s ebar_s;  xbar += Xbar_s;  kbar_{s-1} += (h, h/2, h/2)_s Xbar_s
// with e_s = E_s / |E_s| and g = dJ/dI of the line.  ebar_s is the sensitivity
// of J to the field value at X_s; the pairs (X_s, ebar_s) are written out for
// the charge and geometry terms.  Regular/near classification and the number
// of accepted steps are those of the forward run.
//
//  k_la_far  - (line tile x panel chunk) blocks, panel records read at
//              wave-uniform addresses: partial E and H of the regular pairs by
//              the 7-point rule, near pairs as bit masks, line-major partial
//              rows (as in the forward tracer).
//  k_la_step - one block per line: partial sums + near pairs by the closed
//              forms differentiated with dual numbers, then the stage machine.
//  k_rows_EH - one block per collocation point: E and H of all panels but the
//              point's own (the off-diagonal part of the interface and
//              constraint rows needs their derivative in x).
#include <algorithm>
#include <climits>

#include "adjoint_device.h"

namespace bem {
namespace {

constexpr int LA_T = 256;   // points per tile
constexpr int LA_C = 32;    // panels per chunk
constexpr int LA_NC = 9;    // E (3) + H (xx, yy, zz, xy, xz, yz)
constexpr int LA_Q = 512;   // near pairs per round in a point block

struct LAArgs {
    double h, dir, a, e0, p;
};

struct LAState {
    double* xn;     // [L][3] x_n of the step being reversed
    double* y;      // [L][3] query point of the pass
    double* Es;     // [L][4][3]
    double* Hs;     // [L][4][6]
    double* xb;     // [L][3] adjoint of the position
    int32_t* n;     // [L] step being reversed
};

__device__ __noinline__ double la_pow(double d, double p) { return pow(d, p); }

__global__ void k_fill_i32(int32_t* __restrict__ x, int n, int32_t v) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = v;
}

// alpha'(e) for alpha = a max(e - e0, 0)^p
__device__ __forceinline__ double la_dalpha(const LAArgs& a, double e) {
    const double d = e - a.e0;
    if (!(d > 0.0)) return 0.0;
    return a.a * a.p * (a.p == 2.0 ? d : la_pow(d, a.p - 1.0));
}

template <int SPLIT>
__global__ __launch_bounds__(SPLIT > 1 ? 64 * SPLIT : LA_T) void k_la_far(
    const double* __restrict__ pan64, int64_t N, const double* __restrict__ sol, int64_t n,
    const int32_t* __restrict__ line_rhs, int64_t L, const int32_t* __restrict__ act, const int32_t* __restrict__ count,
    int32_t* __restrict__ count_next, const double* __restrict__ ys, double* __restrict__ part,
    uint32_t* __restrict__ pmask, int32_t tiles, int64_t KS) {
    constexpr int TILE = SPLIT > 1 ? 64 : LA_T;
    constexpr int PER = LA_C / SPLIT;
    __shared__ double wred[SPLIT > 1 ? SPLIT : 1][64][LA_NC];
    __shared__ uint32_t wmask[SPLIT > 1 ? SPLIT : 1][64];

    // XCD x takes the contiguous chunk range [x CPX, (x + 1) CPX), all tiles of each (blocks are
    // dealt to the 8 XCDs round-robin by linear id): a chunk's tiles share one L2 and each
    // point's partials from one XCD are one contiguous run of its row
    const int64_t bid = blockIdx.x, xcd = bid & 7, m = bid >> 3;
    const int64_t CPX = (KS + 7) >> 3;
    const int64_t tile = m % tiles, chunk = xcd * CPX + m / tiles;
    if (count_next && bid == 0 && threadIdx.x == 0) count_next[0] = 0;
    if (chunk >= KS) return;   // padding of the chunk count to a multiple of 8
    const int32_t A = count ? count[0] : (int32_t)L;
    const int64_t tile0 = tile * TILE;
    if (tile0 >= A) return;
    const int64_t j0 = chunk * LA_C;
    const int nc = (int)((N - j0) < LA_C ? (N - j0) : LA_C);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t t = tile0 + (SPLIT > 1 ? lane : (int)threadIdx.x);
    const bool live = t < A;
    const int pj0 = SPLIT > 1 ? wv * PER : 0;
    const int pj1 = SPLIT > 1 ? (pj0 + PER < nc ? pj0 + PER : nc) : nc;
    double acc[LA_NC];
#pragma unroll
    for (int k = 0; k < LA_NC; ++k) acc[k] = 0.0;
    uint32_t nmask = 0;
    int64_t l = 0;
    if (live) {
        l = act ? act[t] : t;
        const double* sigma = sol + (line_rhs ? (int64_t)line_rhs[l] : 0) * n;
        const double p0 = ys[3 * l], p1 = ys[3 * l + 1], p2 = ys[3 * l + 2];
        for (int pj = pj0; pj < pj1; ++pj) {
            // the panel's record at a wave-uniform address: scalar registers, no LDS staging
            const double* cr = pan64 + FAR_REC * (j0 + pj);
            double qv[FR_CC];
#pragma unroll
            for (int k = 0; k < FR_CC; ++k) qv[k] = cr[k];
            if (!is_regular(p0 - cr[FR_CC], p1 - cr[FR_CC + 1], p2 - cr[FR_CC + 2], cr[FR_RR])) {
                nmask |= 1u << pj;
                continue;
            }
            double f0 = 0, f1 = 0, f2 = 0, s3 = 0, hxx = 0, hyy = 0, hzz = 0, hxy = 0, hxz = 0, hyz = 0;
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                const double dx = p0 - qv[FR_X + q], dy = p1 - qv[FR_Y + q], dz = p2 - qv[FR_Z + q];
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double ir = rsqrt_pos(r2);
                const double ir2 = ir * ir;
                const double t3 = qv[FR_W + q] * ir * ir2;   // w / r^3
                const double t5 = 3.0 * t3 * ir2;             // 3 w / r^5
                f0 += t3 * dx;
                f1 += t3 * dy;
                f2 += t3 * dz;
                s3 += t3;
                const double u0 = t5 * dx, u1 = t5 * dy, u2 = t5 * dz;
                hxx -= u0 * dx;
                hyy -= u1 * dy;
                hzz -= u2 * dz;
                hxy -= u0 * dy;
                hxz -= u0 * dz;
                hyz -= u1 * dz;
            }
            const double sg = sigma[j0 + pj];
            acc[0] = fma(sg, f0, acc[0]);
            acc[1] = fma(sg, f1, acc[1]);
            acc[2] = fma(sg, f2, acc[2]);
            acc[3] = fma(sg, hxx + s3, acc[3]);
            acc[4] = fma(sg, hyy + s3, acc[4]);
            acc[5] = fma(sg, hzz + s3, acc[5]);
            acc[6] = fma(sg, hxy, acc[6]);
            acc[7] = fma(sg, hxz, acc[7]);
            acc[8] = fma(sg, hyz, acc[8]);
        }
    }
    if (SPLIT > 1) {
#pragma unroll
        for (int k = 0; k < LA_NC; ++k) wred[wv][lane][k] = acc[k];
        wmask[wv][lane] = nmask;
        __syncthreads();
        if (wv != 0 || !live) return;
#pragma unroll
        for (int k = 0; k < LA_NC; ++k) acc[k] = wred[0][lane][k];
        nmask = wmask[0][lane];
        for (int w = 1; w < SPLIT; ++w) {
#pragma unroll
            for (int k = 0; k < LA_NC; ++k) acc[k] += wred[w][lane][k];
            nmask |= wmask[w][lane];
        }
    } else if (!live) {
        return;
    }
    double* o = part + (l * KS + chunk) * LA_NC;
#pragma unroll
    for (int k = 0; k < LA_NC; ++k) o[k] = acc[k];
    pmask[l * KS + chunk] = nmask;
}

// E and H at point p of line/point slot l, by the whole block: fixed-order sums of
// the chunk partials, the near pairs by dual-number closed forms (skipping panel
// `skip`).  The result is valid in thread 0 only.
__device__ void block_EH(int64_t L, int64_t KS, int64_t l, const double* __restrict__ part,
                         const uint32_t* __restrict__ pmask, const double* __restrict__ tri64,
                         const double* __restrict__ sigma, double p0, double p1, double p2, int64_t skip,
                         int32_t* list, int32_t* scan, double (*red)[LA_NC], double (&out)[LA_NC]) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double acc[LA_NC];
#pragma unroll
    for (int k = 0; k < LA_NC; ++k) acc[k] = 0.0;
    for (int64_t k = tid; k < KS; k += 256) {
        const double* o = part + (l * KS + k) * LA_NC;
#pragma unroll
        for (int c = 0; c < LA_NC; ++c) acc[c] += o[c];
    }
    int cnt = 0;
    for (int64_t k = tid; k < KS; k += 256) cnt += __popc(pmask[l * KS + k]);
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane == 63) scan[wv] = incl;
    __syncthreads();
    int wbase = 0;
    for (int w = 0; w < wv; ++w) wbase += scan[w];
    const int total = scan[0] + scan[1] + scan[2] + scan[3];
    const int off = wbase + incl - cnt;
    for (int base = 0; base < total; base += LA_Q) {
        __syncthreads();
        if (off + cnt > base && off < base + LA_Q) {
            int pos = off;
            for (int64_t k = tid; k < KS && pos < base + LA_Q; k += 256) {
                uint32_t m = pmask[l * KS + k];
                while (m) {
                    const int b = __builtin_ctz(m);
                    m &= m - 1;
                    if (pos >= base && pos < base + LA_Q) list[pos - base] = (int32_t)(k * LA_C + b);
                    ++pos;
                }
            }
        }
        __syncthreads();
        const int nq = (total - base) < LA_Q ? (total - base) : LA_Q;
        for (int q = tid; q < nq; q += 256) {
            const int j = list[q];
            if (j == skip) continue;
            double Fv[3], Jac[3][3];
            tri_F_dx(tri64 + (int64_t)TRI_REC * j, p0, p1, p2, Fv, Jac);
            const double sg = sigma[j];
            acc[0] = fma(sg, Fv[0], acc[0]);
            acc[1] = fma(sg, Fv[1], acc[1]);
            acc[2] = fma(sg, Fv[2], acc[2]);
            acc[3] = fma(sg, Jac[0][0], acc[3]);
            acc[4] = fma(sg, Jac[1][1], acc[4]);
            acc[5] = fma(sg, Jac[2][2], acc[5]);
            acc[6] = fma(sg, 0.5 * (Jac[0][1] + Jac[1][0]), acc[6]);
            acc[7] = fma(sg, 0.5 * (Jac[0][2] + Jac[2][0]), acc[7]);
            acc[8] = fma(sg, 0.5 * (Jac[1][2] + Jac[2][1]), acc[8]);
        }
    }
#pragma unroll
    for (int c = 0; c < LA_NC; ++c) acc[c] = wave_sum(acc[c]);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < LA_NC; ++c) red[wv][c] = acc[c];
    __syncthreads();
    if (tid == 0)
#pragma unroll
        for (int c = 0; c < LA_NC; ++c) out[c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

__global__ __launch_bounds__(256) void k_la_init(int64_t L, const int32_t* __restrict__ ns, const double* __restrict__ path,
                                                 int64_t pstride, LAState s, int32_t* __restrict__ act,
                                                 int32_t* __restrict__ count, double* __restrict__ x0bar) {
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (l >= L) return;
    const int32_t n = ns[l] - 1;
    s.n[l] = n;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        s.xb[3 * l + k] = 0.0;
        const double v = n >= 0 ? path[l * pstride + 3 * n + k] : 0.0;
        s.xn[3 * l + k] = v;
        s.y[3 * l + k] = v;
    }
    if (n < 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) x0bar[3 * l + k] = 0.0;
    } else {
        act[atomicAdd(count, 1)] = (int32_t)l;
    }
}

__global__ __launch_bounds__(256) void k_la_step(int64_t L, int64_t KS, const int32_t* __restrict__ act,
                                                 const int32_t* __restrict__ count, int32_t* __restrict__ act_next,
                                                 int32_t* __restrict__ count_next, const double* __restrict__ part,
                                                 const uint32_t* __restrict__ pmask, int phase, LAState s, LAArgs a,
                                                 const double* __restrict__ tri64, const double* __restrict__ sol,
                                                 int64_t n, const int32_t* __restrict__ line_rhs,
                                                 const double* __restrict__ path, int64_t pstride,
                                                 const double* __restrict__ gI, const int64_t* __restrict__ sbase,
                                                 double* __restrict__ SX, double* __restrict__ SE,
                                                 double* __restrict__ x0bar) {
    __shared__ int32_t list[LA_Q];
    __shared__ int32_t scan[4];
    __shared__ double red[4][LA_NC];
    const int32_t A = count[0];
    if ((int64_t)blockIdx.x >= A) return;
    const int64_t l = act[blockIdx.x];
    const double* sigma = sol + (line_rhs ? (int64_t)line_rhs[l] : 0) * n;
    const double p0 = s.y[3 * l], p1 = s.y[3 * l + 1], p2 = s.y[3 * l + 2];
    double EH[LA_NC];
    block_EH(L, KS, l, part, pmask, tri64, sigma, p0, p1, p2, -1, list, scan, red, EH);
    if (threadIdx.x != 0) return;
    const double h = a.h;
    double* Es = s.Es + 12 * l;
    double* Hs = s.Hs + 24 * l;
#pragma unroll
    for (int k = 0; k < 3; ++k) Es[3 * phase + k] = EH[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) Hs[6 * phase + k] = EH[3 + k];
    const double x0 = s.xn[3 * l], x1 = s.xn[3 * l + 1], x2 = s.xn[3 * l + 2];
    if (phase < 3) {
        const double m = sqrt(EH[0] * EH[0] + EH[1] * EH[1] + EH[2] * EH[2]);
        const double c = (phase == 2) ? h : 0.5 * h;
        s.y[3 * l] = x0 + c * a.dir * EH[0] / m;
        s.y[3 * l + 1] = x1 + c * a.dir * EH[1] / m;
        s.y[3 * l + 2] = x2 + c * a.dir * EH[2] / m;
        act_next[atomicAdd(count_next, 1)] = (int32_t)l;
        return;
    }
    // adjoint of step n
    const int32_t nstep = s.n[l];
    double kk[4][3], mm[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        const double e0 = Es[3 * st], e1 = Es[3 * st + 1], e2 = Es[3 * st + 2];
        mm[st] = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
        kk[st][0] = a.dir * e0 / mm[st];
        kk[st][1] = a.dir * e1 / mm[st];
        kk[st][2] = a.dir * e2 / mm[st];
    }
    const double cst[4] = {h / 6.0, h / 3.0, h / 3.0, h / 6.0};
    const double cback[4] = {0.0, 0.5 * h, 0.5 * h, h};   // X_s = x + cback[s] k_{s-1}
    double xb0 = s.xb[3 * l], xb1 = s.xb[3 * l + 1], xb2 = s.xb[3 * l + 2];
    double kb[4][3];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
        kb[st][0] = cst[st] * xb0;
        kb[st][1] = cst[st] * xb1;
        kb[st][2] = cst[st] * xb2;
    }
    const double g = gI[l];
    const int64_t rec0 = sbase[l] + 4 * (int64_t)nstep;
    for (int st = 3; st >= 0; --st) {
        const double im = 1.0 / mm[st];
        const double u0 = Es[3 * st] * im, u1 = Es[3 * st + 1] * im, u2 = Es[3 * st + 2] * im;
        const double uk = u0 * kb[st][0] + u1 * kb[st][1] + u2 * kb[st][2];
        const double ga = g * cst[st] * la_dalpha(a, mm[st]);
        const double eb0 = a.dir * (kb[st][0] - u0 * uk) * im + ga * u0;
        const double eb1 = a.dir * (kb[st][1] - u1 * uk) * im + ga * u1;
        const double eb2 = a.dir * (kb[st][2] - u2 * uk) * im + ga * u2;
        const double* H = Hs + 6 * st;   // xx yy zz xy xz yz
        const double X0 = H[0] * eb0 + H[3] * eb1 + H[4] * eb2;
        const double X1 = H[3] * eb0 + H[1] * eb1 + H[5] * eb2;
        const double X2 = H[4] * eb0 + H[5] * eb1 + H[2] * eb2;
        xb0 += X0;
        xb1 += X1;
        xb2 += X2;
        if (st > 0) {
            kb[st - 1][0] += cback[st] * X0;
            kb[st - 1][1] += cback[st] * X1;
            kb[st - 1][2] += cback[st] * X2;
        }
        // stage point and the field sensitivity there
        double q0 = x0, q1 = x1, q2 = x2;
        if (st > 0) {
            q0 += cback[st] * kk[st - 1][0];
            q1 += cback[st] * kk[st - 1][1];
            q2 += cback[st] * kk[st - 1][2];
        }
        const int64_t r = rec0 + st;
        SX[3 * r] = q0;
        SX[3 * r + 1] = q1;
        SX[3 * r + 2] = q2;
        SE[3 * r] = eb0;
        SE[3 * r + 1] = eb1;
        SE[3 * r + 2] = eb2;
    }
    s.xb[3 * l] = xb0;
    s.xb[3 * l + 1] = xb1;
    s.xb[3 * l + 2] = xb2;
    const int32_t nn = nstep - 1;
    s.n[l] = nn;
    if (nn < 0) {
        x0bar[3 * l] = xb0;
        x0bar[3 * l + 1] = xb1;
        x0bar[3 * l + 2] = xb2;
        return;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double v = path[l * pstride + 3 * nn + k];
        s.xn[3 * l + k] = v;
        s.y[3 * l + k] = v;
    }
    act_next[atomicAdd(count_next, 1)] = (int32_t)l;
}

// E and H (without the point's own panel) at the centroid of panel i, one block per point.
__global__ __launch_bounds__(256) void k_rows_EH(int64_t L, int64_t KS, int64_t row0, const double* __restrict__ part,
                                                 const uint32_t* __restrict__ pmask, const double* __restrict__ tri64,
                                                 const double* __restrict__ sigma, const double* __restrict__ pts,
                                                 double* __restrict__ out) {
    __shared__ int32_t list[LA_Q];
    __shared__ int32_t scan[4];
    __shared__ double red[4][LA_NC];
    const int64_t l = blockIdx.x;
    if (l >= L) return;
    double EH[LA_NC];
    block_EH(L, KS, l, part, pmask, tri64, sigma, pts[3 * l], pts[3 * l + 1], pts[3 * l + 2], row0 + l, list, scan,
             red, EH);
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < LA_NC; ++c) out[(row0 + l) * LA_NC + c] = EH[c];
}

}  // namespace

// Reverse sweep over L lines whose forward run left n_steps and path (stride pstride).
// Writes the stage records SX/SE at sbase[l] + 4 n + s and x0bar[l] (adjoint of the start).
void launch_reverse_sweep(bem_ctx* c, const double* sol, int64_t L, const int32_t* line_rhs, const int32_t* ns,
                          const double* path, int64_t pstride, const bem_trace_params* tp, const double* gI,
                          const int64_t* sbase, int32_t max_ns, double* SX, double* SE, double* x0bar) {
    if (L == 0) return;
    KTimer t(c, "grad_reverse");
    const int64_t N = c->N;
    const int64_t KS = ceil_div(N, LA_C);
    LAArgs a;
    a.h = tp->h;
    a.dir = tp->direction >= 0 ? 1.0 : -1.0;
    a.a = tp->alpha_a;
    a.e0 = tp->alpha_e0;
    a.p = tp->alpha_p;
    c->ad_state.alloc(sizeof(double) * (size_t)L * 46 + sizeof(int32_t) * ((size_t)L * 3 + 64));
    c->ad_part.alloc(sizeof(double) * LA_NC * (size_t)KS * L + sizeof(uint32_t) * (size_t)KS * L);
    double* base = c->ad_state.as<double>();
    LAState s;
    s.xn = base;
    s.y = base + 3 * L;
    s.Es = base + 6 * L;
    s.Hs = base + 18 * L;
    s.xb = base + 42 * L;
    int32_t* ib = reinterpret_cast<int32_t*>(base + 46 * L);
    s.n = ib;
    int32_t* act[2] = {ib + L, ib + 2 * L};
    int32_t* cnt[2] = {ib + 3 * L, ib + 3 * L + 16};
    double* part = c->ad_part.as<double>();
    uint32_t* pmask = reinterpret_cast<uint32_t*>(part + LA_NC * (size_t)KS * L);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, c->stream, cnt[0], 32, 0);
    BEM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_la_init, dim3((unsigned)ceil_div(L, 256)), dim3(256), 0, c->stream, L, ns, path, pstride, s,
                       act[0], cnt[0], x0bar);
    BEM_CHECK_LAUNCH();
    int32_t* host = c->host_stage.as<int32_t>();
    BEM_HIP(hipMemcpyAsync(host, cnt[0], sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    BEM_HIP(hipStreamSynchronize(c->stream));
    int64_t known_active = host[0];
    const int64_t max_pass = 4 * (int64_t)max_ns;
    int cur = 0;
    for (int64_t pass = 0; pass < max_pass && known_active > 0; ++pass) {
        const int phase = (int)(pass % 4);
        // up to 256 live lines: 64-line tiles with each chunk split over 8 waves (a 256-line tile
        // would leave lanes idle and give too few blocks to fill the GPU)
        const bool split = known_active <= 256;
        const int32_t ntile = (int32_t)ceil_div(known_active, split ? 64 : LA_T);
        dim3 g1((unsigned)(ntile * ceil_div(KS, 8) * 8));
        if (split)
            hipLaunchKernelGGL((k_la_far<8>), g1, dim3(512), 0, c->stream, c->pan64.as<double>(), N, sol, c->n,
                               line_rhs, L, act[cur], cnt[cur], cnt[cur ^ 1], s.y, part, pmask, ntile, KS);
        else
            hipLaunchKernelGGL((k_la_far<1>), g1, dim3(LA_T), 0, c->stream, c->pan64.as<double>(), N, sol, c->n,
                               line_rhs, L, act[cur], cnt[cur], cnt[cur ^ 1], s.y, part, pmask, ntile, KS);
        BEM_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_la_step, dim3((unsigned)known_active), dim3(256), 0, c->stream, L, KS, act[cur],
                           cnt[cur], act[cur ^ 1], cnt[cur ^ 1], part, pmask, phase, s, a, c->tri64.as<double>(), sol,
                           c->n, line_rhs, path, pstride, gI, sbase, SX, SE, x0bar);
        BEM_CHECK_LAUNCH();
        cur ^= 1;
        if ((pass & 31) == 31) {
            BEM_HIP(hipMemcpyAsync(host, cnt[cur], sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
            BEM_HIP(hipStreamSynchronize(c->stream));
            known_active = host[0];
        }
    }
}

// E and H (9 values per row, without the row's own panel) at the centroids pts of rows
// [0, P) of the collocation system, for charge sigma; out [P][9].
void launch_rows_EH(bem_ctx* c, const double* sigma, int64_t P, const double* pts, double* out) {
    if (P == 0) return;
    KTimer t(c, "grad_rows_EH");
    const int64_t N = c->N;
    const int64_t KS = ceil_div(N, LA_C);
    const int64_t B = std::min<int64_t>(P, std::min<int64_t>(8192, c->grad_batch));   // bounds the partial buffer
    c->ad_part.alloc(sizeof(double) * LA_NC * (size_t)KS * B + sizeof(uint32_t) * (size_t)KS * B);
    double* part = c->ad_part.as<double>();
    uint32_t* pmask = reinterpret_cast<uint32_t*>(part + LA_NC * (size_t)KS * B);
    for (int64_t p0 = 0; p0 < P; p0 += B) {
        const int64_t nb = std::min<int64_t>(B, P - p0);
        const int32_t ntile = (int32_t)ceil_div(nb, LA_T);
        dim3 g1((unsigned)(ntile * ceil_div(KS, 8) * 8));
        hipLaunchKernelGGL((k_la_far<1>), g1, dim3(LA_T), 0, c->stream, c->pan64.as<double>(), N, sigma, (int64_t)0,
                           (const int32_t*)nullptr, nb, (const int32_t*)nullptr, (const int32_t*)nullptr,
                           (int32_t*)nullptr, pts + 3 * p0, part, pmask, ntile, KS);
        BEM_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_rows_EH, dim3((unsigned)nb), dim3(256), 0, c->stream, nb, KS, p0, part, pmask,
                           c->tri64.as<double>(), sigma, pts + 3 * p0, out);
        BEM_CHECK_LAUNCH();
    }
}

}  // namespace bem
