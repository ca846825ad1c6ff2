// Matrix-free potential and field at arbitrary points (the field formula
// that closes Sec. 2; "E surface" of Sec. 5.2).
//
// k_eval_mask: Sec. 4 classification of (point, panel) pairs, panel-stationary
//   lanes, one 64-bit ballot per (point, 64-panel group).
// k_eval_far:  target-stationary: one lane per point, panel tiles staged in
//   LDS and read by broadcast; 7-point rule for regular pairs, near pairs
//   masked by select.  The panel range is split over blockIdx.y so that few
//   points still fill the GPU; each split writes its own partial sums.
// k_eval_finish: one wave per point: its lanes share the partials and the
//   point's near pairs (closed forms, FP64) from the CSR list, summed over the
//   wave in a fixed order, plus the exterior jump sigma n / 2 for on-surface
//   points.
#include "bem_device.h"

namespace bem {
namespace {

constexpr int EV_TILE = 64;
constexpr int EV_MASK_PTS = 64;

__global__ __launch_bounds__(256) void k_eval_mask(const double* __restrict__ far64, int64_t Np, int64_t N, int64_t P,
                                                   const double* __restrict__ pts, const int32_t* __restrict__ on_panel,
                                                   uint64_t* __restrict__ mask) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool valid = j < N;
    const bool wave_live = ((j & ~(int64_t)63) < N);
    const double ccx = far64[(int64_t)(FR_CC + 0) * Np + j];
    const double ccy = far64[(int64_t)(FR_CC + 1) * Np + j];
    const double ccz = far64[(int64_t)(FR_CC + 2) * Np + j];
    const double rr = far64[(int64_t)FR_RR * Np + j];
    const int64_t p0 = (int64_t)blockIdx.y * EV_MASK_PTS;
    const int64_t p1 = p0 + EV_MASK_PTS < P ? p0 + EV_MASK_PTS : P;
    for (int64_t p = p0; p < p1; ++p) {
        const double x0 = pts[3 * p], x1 = pts[3 * p + 1], x2 = pts[3 * p + 2];
        const int64_t op = on_panel ? on_panel[p] : -1;
        const bool reg = is_regular(x0 - ccx, x1 - ccy, x2 - ccz, rr) && (j != op);
        const uint64_t m = __ballot(valid && !reg);
        if (wave_live && (threadIdx.x & 63) == 0) mask[(j >> 6) * P + p] = m;
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_eval_far(const double* __restrict__ far64, const R* __restrict__ farR,
                                                  int64_t Np, int64_t N, int64_t span,
                                                  const double* __restrict__ sigma, int64_t P,
                                                  const double* __restrict__ pts, const int32_t* __restrict__ on_panel,
                                                  double* __restrict__ part) {
    __shared__ R tq[EV_TILE][4 * 7];      // node xyz + weight
    __shared__ double tc[EV_TILE][5];     // circumcentre, (eta R)^2, sigma
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool pv = p < P;
    const int64_t pc = pv ? p : P - 1;
    const double x0 = pts[3 * pc], x1 = pts[3 * pc + 1], x2 = pts[3 * pc + 2];
    const int64_t op = on_panel ? on_panel[pc] : -1;
    const R xr0 = (R)x0, xr1 = (R)x1, xr2 = (R)x2;
    double phi = 0.0, e0 = 0.0, e1 = 0.0, e2 = 0.0;
    const int64_t j_beg = (int64_t)blockIdx.y * span;
    const int64_t j_end = j_beg + span < N ? j_beg + span : N;
    for (int64_t t0 = j_beg; t0 < j_end; t0 += EV_TILE) {
        __syncthreads();
        // stage EV_TILE panels: 28 node values + 5 classification values each
        for (int e = threadIdx.x; e < EV_TILE * 33; e += 256) {
            const int pj = e % EV_TILE, comp = e / EV_TILE;
            const int64_t j = t0 + pj;   // < Np: span is a multiple of EV_TILE and Np >= N rounded up
            if (comp < 28)
                tq[pj][comp] = farR[(int64_t)comp * Np + j];
            else if (comp < 32)
                tc[pj][comp - 28] = far64[(int64_t)comp * Np + j];
            else
                tc[pj][4] = (j < N) ? sigma[j] : 0.0;
        }
        __syncthreads();
        const int cnt = (int)((j_end - t0) < EV_TILE ? (j_end - t0) : EV_TILE);
        for (int pj = 0; pj < cnt; ++pj) {
            const int64_t j = t0 + pj;
            const bool reg = is_regular(x0 - tc[pj][0], x1 - tc[pj][1], x2 - tc[pj][2], tc[pj][3]) && (j != op);
            R sp = 0, f0 = 0, f1 = 0, f2 = 0;
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                const R dx = xr0 - tq[pj][q], dy = xr1 - tq[pj][7 + q], dz = xr2 - tq[pj][14 + q];
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R ir = rsqrt_pos(r2);
                const R t = tq[pj][21 + q] * ir;
                sp += t;
                const R t3 = t * ir * ir;
                f0 += t3 * dx;
                f1 += t3 * dy;
                f2 += t3 * dz;
            }
            const double s = reg ? tc[pj][4] : 0.0;
            phi = fma(s, (double)(reg ? sp : (R)0), phi);
            e0 = fma(s, (double)(reg ? f0 : (R)0), e0);
            e1 = fma(s, (double)(reg ? f1 : (R)0), e1);
            e2 = fma(s, (double)(reg ? f2 : (R)0), e2);
        }
    }
    if (pv) {
        double* o = part + ((int64_t)blockIdx.y * P + p) * 4;
        o[0] = phi;
        o[1] = e0;
        o[2] = e1;
        o[3] = e2;
    }
}

__global__ __launch_bounds__(256) void k_eval_finish(const double* __restrict__ part, int KS, int64_t P,
                                                     const int64_t* __restrict__ nptr, const int32_t* __restrict__ ncol,
                                                     const double* __restrict__ tri64, const double* __restrict__ sigma,
                                                     const double* __restrict__ pts, const int32_t* __restrict__ on_panel,
                                                     double* __restrict__ phi_out, double* __restrict__ E_out) {
    const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);   // wave-uniform
    const int lane = threadIdx.x & 63;
    if (p >= P) return;
    double phi = 0.0, e0 = 0.0, e1 = 0.0, e2 = 0.0;
    for (int k = lane; k < KS; k += 64) {
        const double* o = part + ((int64_t)k * P + p) * 4;
        phi += o[0];
        e0 += o[1];
        e1 += o[2];
        e2 += o[3];
    }
    const double x0 = pts[3 * p], x1 = pts[3 * p + 1], x2 = pts[3 * p + 2];
    const int64_t op = on_panel ? on_panel[p] : -1;
    for (int64_t e = nptr[p] + lane; e < nptr[p + 1]; e += 64) {
        const int64_t j = ncol[e];
        double S, F0, F1, F2;
        flat_tri_SF<true, true>(tri64 + (int64_t)TRI_REC * j, x0, x1, x2, j == op, S, F0, F1, F2);
        const double s = sigma[j];
        phi = fma(s, S, phi);
        e0 = fma(s, F0, e0);
        e1 = fma(s, F1, e1);
        e2 = fma(s, F2, e2);
    }
    phi = wave_sum(phi);
    e0 = wave_sum(e0);
    e1 = wave_sum(e1);
    e2 = wave_sum(e2);
    if (lane != 0) return;
    if (op >= 0) {
        const double* T = tri64 + (int64_t)TRI_REC * op;
        const double hs = 0.5 * sigma[op];
        e0 += hs * T[TR_N + 0];
        e1 += hs * T[TR_N + 1];
        e2 += hs * T[TR_N + 2];
    }
    if (phi_out) phi_out[p] = phi;
    E_out[3 * p] = e0;
    E_out[3 * p + 1] = e1;
    E_out[3 * p + 2] = e2;
}

}  // namespace

void launch_point_mask(bem_ctx* c, int64_t P, const double* pts, const int32_t* on_panel, uint64_t* mask) {
    if (P == 0) return;
    const int64_t Np = (int64_t)(c->far64.bytes / (sizeof(double) * FAR_REC));
    dim3 grid((unsigned)(Np / 256), (unsigned)ceil_div(P, EV_MASK_PTS));
    hipLaunchKernelGGL(k_eval_mask, grid, dim3(256), 0, c->stream, c->far64.as<double>(), Np, c->N, P, pts, on_panel,
                       mask);
    BEM_CHECK_LAUNCH();
}

// K ranges of the panel split of the far pass for P points: about the tuned number of blocks
// (default 2048); span (panels per range) is a multiple of the LDS tile.
int64_t eval_split(const bem_ctx* c, int64_t P, int64_t* span) {
    const int64_t N = c->N;
    const int64_t pb = ceil_div(P, 256);
    int64_t KS = c->tune_eval_blocks / pb;
    if (KS < 1) KS = 1;
    if (KS > ceil_div(N, EV_TILE)) KS = ceil_div(N, EV_TILE);
    *span = ceil_div(ceil_div(N, KS), EV_TILE) * EV_TILE;
    return ceil_div(N, *span);
}

// far pass of the field evaluation into part[KS][P][4] (phi, E partial sums per panel range)
void launch_eval_far(bem_ctx* c, const double* sigma, int64_t P, const double* pts, const int32_t* on_panel,
                     double* part, int64_t KS, int64_t span) {
    const int64_t Np = (int64_t)(c->far64.bytes / (sizeof(double) * FAR_REC));
    dim3 grid((unsigned)ceil_div(P, 256), (unsigned)KS);
    if (c->opt.precision == BEM_FP64)
        hipLaunchKernelGGL((k_eval_far<double>), grid, dim3(256), 0, c->stream, c->far64.as<double>(),
                           c->far64.as<double>(), Np, c->N, span, sigma, P, pts, on_panel, part);
    else
        hipLaunchKernelGGL((k_eval_far<float>), grid, dim3(256), 0, c->stream, c->far64.as<double>(),
                           c->far32.as<float>(), Np, c->N, span, sigma, P, pts, on_panel, part);
    BEM_CHECK_LAUNCH();
}

void launch_eval(bem_ctx* c, const double* sigma, int64_t P, const double* pts, const int32_t* on_panel, double* phi,
                 double* E) {
    if (P == 0) return;
    const int64_t N = c->N;
    const int64_t nblk = ceil_div(N, 64);
    c->ev_mask.alloc(sizeof(uint64_t) * nblk * P);
    {
        KTimer t(c, "eval_mask");
        launch_point_mask(c, P, pts, on_panel, c->ev_mask.as<uint64_t>());
    }
    int64_t nnz = 0;
    launch_near_csr(c, c->ev_mask.as<uint64_t>(), P, c->ev_ptr, c->ev_row, c->ev_col, &nnz, "eval_near_csr");
    int64_t span = 0;
    const int64_t KS = eval_split(c, P, &span);
    c->ev_part.alloc(sizeof(double) * 4 * KS * P);
    {
        KTimer t(c, "eval_far");
        launch_eval_far(c, sigma, P, pts, on_panel, c->ev_part.as<double>(), KS, span);
    }
    {
        KTimer t(c, "eval_near");
        hipLaunchKernelGGL(k_eval_finish, dim3((unsigned)ceil_div(P, 4)), dim3(256), 0, c->stream,
                           c->ev_part.as<double>(), (int)KS, P, c->ev_ptr.as<int64_t>(), c->ev_col.as<int32_t>(),
                           c->tri64.as<double>(), sigma, pts, on_panel, phi, E);
        BEM_CHECK_LAUNCH();
    }
}

}  // namespace bem
