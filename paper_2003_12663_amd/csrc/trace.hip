// Field lines and the streamer-inception integral (Sec. 1, Eq. Breakdowncrit)
// in one persistent launch.
//
// Each workgroup takes lines from a global counter until none are left (so
// lines of uneven length balance across the GPU), and walks its line with
// classical RK4 on dx/ds = dir E/|E|.  Every field evaluation is one pass of
// the whole workgroup over all panels: lane k handles panels k, k + T, ...;
// regular pairs use the 7-point rule at once, near pairs are appended to a
// per-wave LDS queue (ballot + mbcnt, no atomics) and evaluated together by
// the wave with the closed forms when the queue fills and at the end of the
// pass -- the deferred near pass of Sec. 4 inside one evaluation.  Partial
// fields are reduced across the workgroup and every lane carries the same
// line state.  The segment hit test of a step is fused into the pass that
// evaluates the field at the step's end point: a panel the segment can reach
// lies within R + h of that point, so it is always in the near queue when
// h < (eta - 1) R_min (checked on the host).
#include <climits>

#include "bem_device.h"

namespace bem {
namespace {

struct TraceArgs {
    double h, e_min, dir, a, e0, p, k_str;
    int32_t max_steps;
};

constexpr int QW = 256;   // per-wave near-queue capacity

__device__ __noinline__ double alpha_pow(double d, double p) { return pow(d, p); }

__device__ __forceinline__ double alpha_eff(const TraceArgs& a, double e) {
    const double d = e - a.e0;
    if (!(d > 0.0)) return 0.0;
    return a.a * (a.p == 2.0 ? d * d : alpha_pow(d, a.p));
}

// sigma_j times the closed-form field of panel j, added to (e0, e1, e2); kept
// out of line so that the rare near pairs do not raise the register budget of
// the far-field loop
__device__ __noinline__ void add_near_field(const double* __restrict__ Tj, double p0, double p1, double p2, double sg,
                                            double* e) {
    double S, F0, F1, F2;
    flat_tri_SF<false, true>(Tj, p0, p1, p2, false, S, F0, F1, F2);
    e[0] = fma(sg, F0, e[0]);
    e[1] = fma(sg, F1, e[1]);
    e[2] = fma(sg, F2, e[2]);
}

// Moeller-Trumbore test of the closed segment q -> p against triangle T
// (closed); returns t in [0,1] or a negative value when there is no hit.
__device__ __forceinline__ double segment_tri(const double* __restrict__ T, double q0, double q1, double q2, double d0,
                                              double d1, double d2) {
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

template <int T>
struct Shared {
    int32_t q[T / 64][QW];
    double red[2][T / 64][4];
    int32_t redj[2][T / 64];
    int64_t line;
};

// E at p (FP64 sum of FP64 or FP32 pair terms).  HIT: also the first panel
// hit by the segment s -> p, or -1.
template <int T, typename R>
__device__ __forceinline__ void field_pass(const bool HIT, Shared<T>& sh, int& par, const double* __restrict__ far64,
                                           const R* __restrict__ farR, int64_t Np, int64_t N,
                                           const double* __restrict__ tri64, const double* __restrict__ sigma,
                                           double p0, double p1, double p2, double s0, double s1, double s2,
                                           double& E0, double& E1, double& E2, int& hitj) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int32_t* wq = sh.q[wv];
    double e0 = 0.0, e1 = 0.0, e2 = 0.0;
    double bt = 2.0;
    int bj = INT_MAX;
    const double sd0 = p0 - s0, sd1 = p1 - s1, sd2 = p2 - s2;
    const R pr0 = (R)p0, pr1 = (R)p1, pr2 = (R)p2;
    int qn = 0;
    auto drain = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int k = lane; k < qn; k += 64) {
            const int j = wq[k];
            const double* Tj = tri64 + (int64_t)TRI_REC * j;
            double ev[3] = {e0, e1, e2};
            add_near_field(Tj, p0, p1, p2, sigma[j], ev);
            e0 = ev[0];
            e1 = ev[1];
            e2 = ev[2];
            if (HIT) {
                const double t = segment_tri(Tj, s0, s1, s2, sd0, sd1, sd2);
                if (t >= 0.0 && (t < bt || (t == bt && j < bj))) {
                    bt = t;
                    bj = j;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    const double* __restrict__ cc0 = far64 + (int64_t)(FR_CC + 0) * Np;
    const double* __restrict__ cc1 = far64 + (int64_t)(FR_CC + 1) * Np;
    const double* __restrict__ cc2 = far64 + (int64_t)(FR_CC + 2) * Np;
    const double* __restrict__ crr = far64 + (int64_t)FR_RR * Np;
    const R* __restrict__ fx = farR + (int64_t)FR_X * Np;
    const R* __restrict__ fy = farR + (int64_t)FR_Y * Np;
    const R* __restrict__ fz = farR + (int64_t)FR_Z * Np;
    const R* __restrict__ fw = farR + (int64_t)FR_W * Np;
    const int32_t Ni = (int32_t)N, Npi = (int32_t)Np;
    for (int32_t j0 = 0; j0 < Ni; j0 += T) {
        const int32_t j = j0 + (int32_t)threadIdx.x;
        bool nearp = false;
        if (j < Ni) {
            if (is_regular(p0 - cc0[j], p1 - cc1[j], p2 - cc2[j], crr[j])) {
                R f0 = 0, f1 = 0, f2 = 0;
#pragma unroll
                for (int q = 0; q < 7; ++q) {
                    const R dx = pr0 - fx[q * Npi + j];
                    const R dy = pr1 - fy[q * Npi + j];
                    const R dz = pr2 - fz[q * Npi + j];
                    const R r2 = dx * dx + dy * dy + dz * dz;
                    const R ir = rsqrt_pos(r2);
                    const R t = fw[q * Npi + j] * ir * ir * ir;
                    f0 += t * dx;
                    f1 += t * dy;
                    f2 += t * dz;
                }
                const double sg = sigma[j];
                e0 = fma(sg, (double)f0, e0);
                e1 = fma(sg, (double)f1, e1);
                e2 = fma(sg, (double)f2, e2);
            } else {
                nearp = true;
            }
        }
        const uint64_t m = __ballot(nearp);
        if (m) {
            if (nearp) {
                const int pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
                wq[qn + pos] = (int32_t)j;
            }
            qn += __popcll(m);
            if (qn > QW - 64) {
                drain();
                qn = 0;
            }
        }
    }
    drain();
    // workgroup reduction (double-buffered slots: one barrier per pass)
    e0 = wave_sum(e0);
    e1 = wave_sum(e1);
    e2 = wave_sum(e2);
    if (HIT) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double t2 = __shfl_xor(bt, o, 64);
            const int j2 = __shfl_xor(bj, o, 64);
            if (t2 < bt || (t2 == bt && j2 < bj)) {
                bt = t2;
                bj = j2;
            }
        }
    }
    if (lane == 0) {
        sh.red[par][wv][0] = e0;
        sh.red[par][wv][1] = e1;
        sh.red[par][wv][2] = e2;
        sh.red[par][wv][3] = bt;
        sh.redj[par][wv] = bj;
    }
    __syncthreads();
    E0 = E1 = E2 = 0.0;
    double tb = 2.0;
    int jb = INT_MAX;
#pragma unroll 2
    for (int w = 0; w < T / 64; ++w) {
        E0 += sh.red[par][w][0];
        E1 += sh.red[par][w][1];
        E2 += sh.red[par][w][2];
        if (HIT) {
            const double t2 = sh.red[par][w][3];
            const int j2 = sh.redj[par][w];
            if (t2 < tb || (t2 == tb && j2 < jb)) {
                tb = t2;
                jb = j2;
            }
        }
    }
    hitj = (HIT && jb != INT_MAX) ? jb : -1;
    par ^= 1;
}

template <int T, typename R>
__global__ __launch_bounds__(T) void k_trace(const double* __restrict__ far64, const R* __restrict__ farR, int64_t Np,
                                             int64_t N, const double* __restrict__ tri64,
                                             const int32_t* __restrict__ tri_body,
                                             const int32_t* __restrict__ body_kind, const double* __restrict__ sol,
                                             int64_t n, int64_t L, const int32_t* __restrict__ line_rhs,
                                             const double* __restrict__ starts, TraceArgs a,
                                             int32_t* __restrict__ n_steps, int32_t* __restrict__ stop_code,
                                             double* __restrict__ path, double* __restrict__ integral,
                                             uint8_t* __restrict__ exceeds, int32_t* __restrict__ counter) {
    __shared__ Shared<T> sh;
    int par = 0;
    const int64_t pstride = 3 * ((int64_t)a.max_steps + 1);
    const double h = a.h;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) sh.line = atomicAdd(counter, 1);
        __syncthreads();
        const int64_t l = sh.line;
        if (l >= L) break;
        const int64_t rhs = line_rhs ? line_rhs[l] : 0;
        const double* sigma = sol + rhs * n;
        double x0 = starts[3 * l], x1 = starts[3 * l + 1], x2 = starts[3 * l + 2];
        if (path && threadIdx.x == 0) {
            path[l * pstride + 0] = x0;
            path[l * pstride + 1] = x1;
            path[l * pstride + 2] = x2;
        }
        double I = 0.0;
        int32_t ns = 0, code = 0;
        // One field evaluation per trip.  phase 0: E at the current point x;
        // phases 1-3: RK4 stages 2-4; phase 4: E at the step's end point fused
        // with the hit test of the step's segment.
        int phase = 0;
        double y0 = x0, y1 = x1, y2 = x2;           // query point
        double ks0 = 0, ks1 = 0, ks2 = 0, asum = 0.0; // k1 + 2 k2 + 2 k3 + k4 and the alpha sum
        for (;;) {
            double F0, F1, F2;
            int hit = -1;
            field_pass<T, R>(phase == 4, sh, par, far64, farR, Np, N, tri64, sigma, y0, y1, y2, x0, x1, x2, F0, F1,
                             F2, hit);
            if (phase == 4) {
                if (hit >= 0) {
                    const int32_t k = body_kind[tri_body[hit]];
                    code = (k == BEM_DIRICHLET) ? BEM_STOP_DIRICHLET
                                                : ((k == BEM_FLOATING) ? BEM_STOP_FLOATING : BEM_STOP_INTERFACE);
                    break;
                }
                I += h / 6.0 * asum;
                x0 = y0;
                x1 = y1;
                x2 = y2;
                ++ns;
                if (path && threadIdx.x == 0) {
                    path[l * pstride + 3 * ns + 0] = x0;
                    path[l * pstride + 3 * ns + 1] = x1;
                    path[l * pstride + 3 * ns + 2] = x2;
                }
                if (ns >= a.max_steps) {
                    code = BEM_STOP_MAXSTEPS;
                    break;
                }
            }
            const double m = sqrt(F0 * F0 + F1 * F1 + F2 * F2);
            const double k0 = a.dir * F0 / m, k1 = a.dir * F1 / m, k2 = a.dir * F2 / m;
            if (phase == 0 || phase == 4) {
                // stage 1 at x
                if (!isfinite(m)) {
                    code = BEM_STOP_NONFINITE;
                    break;
                }
                if (m < a.e_min) {
                    code = BEM_STOP_WEAK;
                    break;
                }
                ks0 = k0;
                ks1 = k1;
                ks2 = k2;
                asum = alpha_eff(a, m);
                y0 = x0 + 0.5 * h * k0;
                y1 = x1 + 0.5 * h * k1;
                y2 = x2 + 0.5 * h * k2;
                phase = 1;
            } else if (phase < 3) {
                // stages 2 and 3 (weight 2); next point x + h/2 k2 or x + h k3
                ks0 += 2.0 * k0;
                ks1 += 2.0 * k1;
                ks2 += 2.0 * k2;
                asum += 2.0 * alpha_eff(a, m);
                const double c = (phase == 1) ? 0.5 * h : h;
                y0 = x0 + c * k0;
                y1 = x1 + c * k1;
                y2 = x2 + c * k2;
                ++phase;
            } else {
                // stage 4 (weight 1): the step's end point
                ks0 += k0;
                ks1 += k1;
                ks2 += k2;
                asum += alpha_eff(a, m);
                y0 = x0 + h / 6.0 * ks0;
                y1 = x1 + h / 6.0 * ks1;
                y2 = x2 + h / 6.0 * ks2;
                if (!(isfinite(y0) && isfinite(y1) && isfinite(y2))) {
                    code = BEM_STOP_NONFINITE;
                    break;
                }
                phase = 4;
            }
        }
        if (threadIdx.x == 0) {
            n_steps[l] = ns;
            stop_code[l] = code;
            if (integral) integral[l] = I;
            if (exceeds) exceeds[l] = (I > a.k_str) ? 1 : 0;
        }
    }
}

__global__ void k_zero_counter(int32_t* c) { c[0] = 0; }

template <int T>
void launch_trace_T(bem_ctx* c, int64_t Np, const double* sol, int64_t L, const int32_t* line_rhs,
                    const double* starts, const TraceArgs& a, int32_t* n_steps, int32_t* stop_code, double* path,
                    double* integral, uint8_t* exceeds, int blocks) {
    if (c->opt.precision == BEM_FP64)
        hipLaunchKernelGGL((k_trace<T, double>), dim3(blocks), dim3(T), 0, c->stream, c->far64.as<double>(),
                           c->far64.as<double>(), Np, c->N, c->tri64.as<double>(), c->tri_body.as<int32_t>(),
                           c->body_kind.as<int32_t>(), sol, c->n, L, line_rhs, starts, a, n_steps, stop_code, path,
                           integral, exceeds, c->tr_queue.as<int32_t>());
    else
        hipLaunchKernelGGL((k_trace<T, float>), dim3(blocks), dim3(T), 0, c->stream, c->far64.as<double>(),
                           c->far32.as<float>(), Np, c->N, c->tri64.as<double>(), c->tri_body.as<int32_t>(),
                           c->body_kind.as<int32_t>(), sol, c->n, L, line_rhs, starts, a, n_steps, stop_code, path,
                           integral, exceeds, c->tr_queue.as<int32_t>());
    BEM_CHECK_LAUNCH();
}

}  // namespace

bool trace_fused_layout(const bem_ctx* c) { return c->trace_mode == 3; }
bool trace_fused_tail(const bem_ctx* c) {
    return c->trace_mode == 0 && c->tune_trace_tail > 0 && fused_trace_blocks(c->N, 4) > 0;
}

void launch_trace(bem_ctx* c, int32_t nrhs, const double* sol, int64_t L, const int32_t* line_rhs,
                  const double* starts, const bem_trace_params* tp, int32_t* n_steps, int32_t* stop_code, double* path,
                  double* integral, uint8_t* exceeds) {
    if (L == 0) return;
    int cus = 0;
    BEM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
    // default: all lines advance together (measured faster than one workgroup per line for
    // 4 to 4096 lines; the per-line layout is bound by per-CU load bandwidth), a far pass and a
    // step kernel per stage while many lines are live, one launch per stage for the last few
    // (measured on the 19,732-panel coax: 47 against 64 us a stage at 256 lines, 21.4 against
    // 17.1 us at 16, 16.1 against 12.4 us at 3)
    const int mode = c->trace_mode != 0 ? c->trace_mode : 1;
    if (mode == 1 || mode == 3) {
        if (c->opt.basis == BEM_BASIS_LINEAR && nrhs > 1 && line_rhs)
            launch_trace_nodal_cases(c, nrhs, sol, L, line_rhs, starts, tp, n_steps, stop_code, path, integral,
                                     exceeds);
        else if (trace_fused_layout(c))
            launch_trace_fused(c, nrhs, sol, L, line_rhs, starts, tp, n_steps, stop_code, path, integral, exceeds);
        else
            launch_trace_batched(c, nrhs, sol, L, line_rhs, starts, tp, n_steps, stop_code, path, integral, exceeds,
                                 trace_fused_tail(c));
        return;
    }
    KTimer t(c, "trace");
    const int64_t Np = (int64_t)(c->far64.bytes / (sizeof(double) * FAR_REC));
    TraceArgs a;
    a.h = tp->h;
    a.e_min = tp->e_min;
    a.dir = tp->direction >= 0 ? 1.0 : -1.0;
    a.a = tp->alpha_a;
    a.e0 = tp->alpha_e0;
    a.p = tp->alpha_p;
    a.k_str = tp->k_str;
    a.max_steps = tp->max_steps;
    c->tr_queue.alloc(sizeof(int32_t) * 64);
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, c->stream, c->tr_queue.as<int32_t>());
    BEM_CHECK_LAUNCH();
    // few lines: one wide workgroup per line; many lines: narrower workgroups, several per CU
    if (L <= (int64_t)cus) {
        launch_trace_T<512>(c, Np, sol, L, line_rhs, starts, a, n_steps, stop_code, path, integral, exceeds,
                            (int)L);
    } else {
        const int64_t blocks = L < (int64_t)cus * 4 ? L : (int64_t)cus * 4;
        launch_trace_T<256>(c, Np, sol, L, line_rhs, starts, a, n_steps, stop_code, path, integral, exceeds,
                            (int)blocks);
    }
}

}  // namespace bem
