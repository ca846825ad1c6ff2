// Field lines and the streamer integral with one launch per RK4 stage (Sec. 1,
// Eq. Breakdowncrit; RK4 on dx/ds = dir E/|E|): the default layout.
//
// All live lines advance by one stage per launch.  A launch is a grid of
// (panel block b, slot group o) blocks: slot group o holds LPB line slots and
// panel block b the panels [b P, (b + 1) P), P = 256 rnd.  Every block
//  1. finishes the previous stage of its group's lines: it sums the partial
//     records that the previous launch's blocks wrote for them (in the order of
//     b) and runs the RK4 stage machine (hit stop, step acceptance, streamer
//     integral, weak field, step limit).  The nb blocks of a group do this from
//     the same records in the same order, so they agree bit for bit; only the
//     block b = 0 writes the lines' state and results;
//  2. evaluates the field of its panels at the lines' new query points:
//     regular pairs by the 7-point rule, one panel per lane (Sec. 4); pairs
//     that fail the regularity test are marked in the regular pass and done
//     after it (Sec. 4's deferred near pass), queued in LDS and spread over the
//     block's threads, by the closed forms; on the stage that proposes a step's
//     end point, the step's segment is tested against those near panels;
//  3. writes one partial record per (line, panel block): field, first hit on
//     the segment, near pair count.
// A stage thus costs one launch instead of a far-field pass and a step kernel
// that waits for it; the price is the repeated reduction, nb records per line
// and block (nb ~ 20 at 20k panels).  Lines keep their slots; the host folds
// the live ones to the front when at most half remain.
// A panel that a step's segment can reach lies within R + h of the step's end
// point, hence in its near set when h < (eta - 1) R_min.
#include <algorithm>
#include <climits>

#include "bem_device.h"
#include "nodal_device.h"
#include "trace_device.h"

#include <hip/hip_ext.h>

namespace bem {
namespace {

constexpr int LF_REC = 6;        // partial record: E (3), hit parameter (2: none), hit panel, near pairs
constexpr int LF_RNDMAX = 4;     // 256-panel rounds per block at most
constexpr int LF_NBMAX = 128;    // panel blocks of a launch at most

// the RK4 phase of pass p: 0 the start point, then 1, 2, 3 (stage points) and 4 (a step's end point)
__host__ __device__ inline int lf_phase_of(int64_t pass) { return pass == 0 ? 0 : (int)((pass - 1) % 4) + 1; }


// What a stage launch, or the persistent loop, works on.
struct LFArgs {
    const double* far64;   // far-field records, component-major (FP64 part)
    const void* farR;      // the same in the pass precision R
    int64_t Np, N;
    const double* tri64;
    const int32_t* tri_body;
    const int32_t* body_kind;
    const double* fsol;    // densities of the far pass ([rhs][fn]; fn 0: one row)
    int64_t fn;
    const double* sol;     // solutions ([rhs][n]) for the near pairs
    int64_t n;
    const int32_t* line_rhs;
    const int32_t* ntri;   // nodal basis: vertices of each triangle
    // the phase of the pass whose records part_prev holds (0: start point, 1..3: stage points, 4:
    // a step's end point), -1 when there is none (the query points in cur are to be evaluated)
    int step_phase;
    int eval_phase;        // one-stage launch: the phase of the pass it evaluates
    int nb_prev, nb, rnd;
    int64_t S, pstride_part;
    LFState cur, nxt;
    const double* part_prev;
    double* part_cur;
    LBArgs a;
    int32_t* n_steps;
    int32_t* stop_code;
    double* integral;
    uint8_t* exceeds;
    double* path;
    int64_t pstride;
    unsigned long long* ncnt;
    int32_t* live;         // one-stage launch: live-line counters (three, used in turn)
    int pidx;
    // persistent loop: passes pass0 .., its three record buffers (lstride doubles apart, every
    // word the sentinel at the start), the error flag and the bound of every wait (polls)
    int64_t pass0, max_pass;
    double* lbuf;
    int64_t lstride;
    int32_t* err;
    uint32_t spin_limit;
    unsigned long long* kts;
};

// the near-pair closed forms as calls of their own: inlined into the persistent loop they raise
// the loop's register count past two blocks per CU
struct LFVec3 {
    double x, y, z;
};
__device__ __noinline__ LFVec3 flat_tri_F_call(const double* __restrict__ T, double x0, double x1, double x2) {
    LFVec3 F;
    flat_tri_F_seq(T, x0, x1, x2, F.x, F.y, F.z);
    return F;
}
__device__ __noinline__ LFVec3 nodal_tri_E_call(const double* __restrict__ T, double x0, double x1, double x2, double u0,
                                                double u1, double u2) {
    LFVec3 E{0.0, 0.0, 0.0};
    double ph = 0.0;
    nodal_tri_phiE(T, x0, x1, x2, u0, u1, u2, ph, E.x, E.y, E.z);
    return E;
}

// Coherent accesses for records that blocks of one launch exchange (agent scope: seen across
// the XCDs' L2 caches without writing back or invalidating them).
__device__ __forceinline__ double lf_load_coh(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lf_store_coh(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The persistent loop's "not written yet" word: a signalling NaN with its own payload.  Every
// record word is an arithmetic result (IEEE arithmetic returns quiet NaNs) or an integer
// converted to double, so no record ever holds it.
constexpr unsigned long long LF_SENT = 0x7FF4C0DE5EA1ED00ull;
__device__ __forceinline__ bool lf_is_sent(double v) {
    return (unsigned long long)__double_as_longlong(v) == LF_SENT;
}

__global__ __launch_bounds__(256) void k_lf_fill_sent(int64_t m, unsigned long long* __restrict__ v) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) v[i] = LF_SENT;
}

// One stage per launch (LOOP false) or every remaining stage in one launch (LOOP true), for the
// lines in slots [0, S).  Grid: (panel block b, slot group o) blocks, b fastest.
//
// LOOP: the blocks of slot group o keep the group's line state in LDS (each block its own copy,
// all computed alike) and loop over the passes.  The records themselves carry the signal: the
// loop's pass i (i = 0, 1, ...) writes buffer i mod 3 of lbuf, every word of which starts as
// the sentinel, and a block finishing pass i polls the records of pass i - 1 (coherent loads)
// until none of their words is the sentinel any more.  A buffer comes round again at pass
// i + 3; at pass i + 2 each block puts the sentinel back into its own records there (rows of
// live slots: pass i + 1's records of every block of the group are then in, and each block
// wrote them after reading those of pass i), and it waits for those stores to land before it
// stores its records of pass i + 2, which any later reader sees only after them.  Every wait is
// bounded (spin_limit polls); at the bound the block raises err and leaves, and so, at their
// own bounds, do the blocks waiting for it.  The grid must be resident at once (cooperative
// launch).
template <typename R, int LPB, bool NODAL, bool LOOP>
__device__ __forceinline__ void lf_run(const LFArgs& P) {
    const double* __restrict__ far64 = P.far64;
    const R* __restrict__ farR = static_cast<const R*>(P.farR);
    const int64_t Npa = P.Np, N = P.N, S = P.S, pstride_part = P.pstride_part;
    const double* __restrict__ tri64 = P.tri64;
    const double* __restrict__ sol = P.sol;
    const double* __restrict__ fsol = P.fsol;
    const int64_t fn = P.fn, n = P.n;
    const int32_t* __restrict__ ntri = P.ntri;
    const LBArgs& a = P.a;
    kclock_start(P.kts);
    constexpr int G = 256 / LPB;           // threads per slot in the near pass
    constexpr int GW = G < 64 ? G : 64;    // of them in one wave
    constexpr int NU = G / GW;             // waves per slot in the near pass
    constexpr int LS = LOOP ? LPB : 1;
    __shared__ double sy[LPB][3], sx[LPB][3];
    __shared__ int32_t sl[LPB], srhs[LPB];
    __shared__ double fred[4][LPB][3];
    __shared__ uint16_t nq[LPB][4][64 * LF_RNDMAX];
    __shared__ int32_t nqc[LPB][4];
    __shared__ double nred[LPB][NU][4];
    __shared__ int32_t nredj[LPB][NU];
    // LOOP: the rest of the slots' state (the line point and query point stay in sx, sy)
    __shared__ double lks[LS][3], lasum[LS], lI[LS];
    __shared__ int32_t lns[LS], lline[LS];
    __shared__ int32_t sabort;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nb = P.nb, rnd = P.rnd;
    const int64_t b = blockIdx.x % nb, o = blockIdx.x / nb;
    const int64_t s0 = o * LPB;
    const int64_t jbb = b * 256 * (int64_t)rnd;
    if (!LOOP && blockIdx.x == 0 && tid == 0) P.live[(P.pidx + 1) % 3] = 0;   // the next launch's counter

    // LOOP: the slots' state from cur, and pair counts of the slots this wave finishes
    unsigned long long nacc[2] = {0, 0}, facc[2] = {0, 0};
    if constexpr (LOOP) {
        if (tid < LPB) {
            const int64_t s = s0 + tid;
            const int32_t l = s < S ? P.cur.line[s] : -1;
            lline[tid] = l;
            sl[tid] = l;
            if (l >= 0) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    sx[tid][k] = P.cur.x[3 * s + k];
                    sy[tid][k] = P.cur.y[3 * s + k];
                    lks[tid][k] = P.cur.ks[3 * s + k];
                }
                lasum[tid] = P.cur.asum[s];
                lI[tid] = P.cur.I[s];
                lns[tid] = P.cur.ns[s];
                srhs[tid] = P.line_rhs ? P.line_rhs[l] : 0;
            }
        }
        if (tid == 0) sabort = 0;
        __syncthreads();
    }

    for (int64_t it = 0;; ++it) {
    // the block's first panel, opaque in the loop: otherwise the compiler computes the per-lane
    // record addresses of every round once, before the loop, and holds them in registers
    int64_t jb0 = jbb, Np = Npa;
    if (LOOP) asm volatile("" : "+s"(jb0), "+s"(Np));
    // the panel records of the first round do not depend on the step: requested first, so that
    // they arrive while the step waits for its own loads (index clamped to a real panel slot)
    R rx[7], ry[7], rz[7], rw[7];
    double rc0, rc1, rc2, rrr;
    {
        const int64_t j = (jb0 < N ? jb0 : 0) + tid;   // < Np
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            rx[k] = farR[(int64_t)(FR_X + k) * Np + j];
            ry[k] = farR[(int64_t)(FR_Y + k) * Np + j];
            rz[k] = farR[(int64_t)(FR_Z + k) * Np + j];
            rw[k] = farR[(int64_t)(FR_W + k) * Np + j];
        }
        rc0 = far64[(int64_t)(FR_CC + 0) * Np + j];
        rc1 = far64[(int64_t)(FR_CC + 1) * Np + j];
        rc2 = far64[(int64_t)(FR_CC + 2) * Np + j];
        rrr = far64[(int64_t)FR_RR * Np + j];
    }
    const int step_phase = LOOP ? (it == 0 ? P.step_phase : lf_phase_of(P.pass0 + it - 1)) : P.step_phase;
    const int eval_phase = LOOP ? lf_phase_of(P.pass0 + it) : P.eval_phase;
    // records of the pass to finish: part_prev (nb_prev blocks) first, then the loop's own
    const double* part_rd = (!LOOP || it == 0) ? P.part_prev : P.lbuf + ((it - 1) % 3) * P.lstride;
    const int nbr = (!LOOP || it == 0) ? P.nb_prev : nb;
    double* part_wr = !LOOP ? P.part_cur : P.lbuf + (it % 3) * P.lstride;

    // ---- 1. the previous stage of the group's lines: wave w takes slots w, w + 4 ----
    for (int q = wv; q < LPB; q += 4) {
        const int64_t s = s0 + q;
        // the one-stage launch reads the slot's state from cur: requested together with its line
        // id (slot clamped to [0, S)) rather than after it
        const int64_t sc = s < S ? s : S - 1;
        double cst[11];
        int32_t cns = 0, cl = -1;
        if constexpr (!LOOP) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                cst[k] = P.cur.y[3 * sc + k];
                cst[3 + k] = P.cur.x[3 * sc + k];
                cst[6 + k] = P.cur.ks[3 * sc + k];
            }
            cst[9] = P.cur.asum[sc];
            cst[10] = P.cur.I[sc];
            cns = P.cur.ns[sc];
            cl = P.cur.line[sc];
            asm volatile("" ::"v"(cst[0]), "v"(cst[5]), "v"(cst[8]), "v"(cst[9]), "v"(cns), "v"(cl));
        }
        const int32_t l = LOOP ? sl[q] : ((s < S) ? cl : -1);
        double Y0 = 0.0, Y1 = 0.0, Y2 = 0.0, X0 = 0.0, X1 = 0.0, X2 = 0.0;
        double K0 = 0.0, K1 = 0.0, K2 = 0.0, AS = 0.0, II = 0.0;   // LOOP: the slot's new state
        int32_t NS = 0;
        int32_t lo = -1;   // the line if it goes on
        if (l >= 0) {
            const double p0 = LOOP ? sy[q][0] : cst[0], p1 = LOOP ? sy[q][1] : cst[1], p2 = LOOP ? sy[q][2] : cst[2];
            const double q0 = LOOP ? sx[q][0] : cst[3], q1 = LOOP ? sx[q][1] : cst[4], q2 = LOOP ? sx[q][2] : cst[5];
            if (step_phase < 0) {   // nothing to finish: the query point is evaluated as it is
                Y0 = p0; Y1 = p1; Y2 = p2;
                X0 = q0; X1 = q1; X2 = q2;
                lo = l;
                if constexpr (LOOP) {
                    K0 = lks[q][0]; K1 = lks[q][1]; K2 = lks[q][2];
                    AS = lasum[q]; II = lI[q]; NS = lns[q];
                }
                if (!LOOP && b == 0 && lane == 0) {
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        P.nxt.x[3 * s + k] = P.cur.x[3 * s + k];
                        P.nxt.y[3 * s + k] = P.cur.y[3 * s + k];
                        P.nxt.ks[3 * s + k] = P.cur.ks[3 * s + k];
                    }
                    P.nxt.asum[s] = P.cur.asum[s];
                    P.nxt.I[s] = P.cur.I[s];
                    P.nxt.ns[s] = P.cur.ns[s];
                    P.nxt.line[s] = l;
                }
            } else {
                const int32_t ns0 = LOOP ? lns[q] : cns;
                const double asum0 = LOOP ? lasum[q] : cst[9], I0 = LOOP ? lI[q] : cst[10];
                const double ks0 = LOOP ? lks[q][0] : cst[6], ks1 = LOOP ? lks[q][1] : cst[7],
                             ks2 = LOOP ? lks[q][2] : cst[8];
                // field at the query point: the partial records in block order, lane k taking blocks k, k + 64
                double F0 = 0.0, F1 = 0.0, F2 = 0.0, nn = 0.0, tb = 2.0;
                int jb = INT_MAX;
                const double* prow = part_rd + s * pstride_part;
                // both records of the lane (blocks lane and lane + 64; nbr <= 128) requested at
                // once, indices clamped into the row and the clamped values dropped
                double rv[2][LF_REC];
                bool rec_ok = true;
                if (LOOP && it > 0) {
                    // the loop's own records: polled until the writers' words have replaced the
                    // sentinel, first word 0 of both records, then every word (the words of a
                    // record land in any order); a clamped index reads block 0's record, a real one
                    const double* r0 = prow + (int64_t)(lane < nbr ? lane : 0) * LF_REC;
                    const double* r1 = prow + (int64_t)(lane + 64 < nbr ? lane + 64 : 0) * LF_REC;
                    uint32_t polls = 0;
                    for (;;) {
                        rv[0][0] = lf_load_coh(r0);
                        rv[1][0] = lf_load_coh(r1);
                        const bool w = lf_is_sent(rv[0][0]) || lf_is_sent(rv[1][0]);
                        if (__ballot(w) == 0) break;   // uniform over the wave
                        if (++polls > P.spin_limit) {
                            rec_ok = false;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(8);
                    }
                    while (rec_ok) {
                        bool w = false;
#pragma unroll
                        for (int c = 0; c < LF_REC; ++c) {
                            rv[0][c] = lf_load_coh(r0 + c);
                            rv[1][c] = lf_load_coh(r1 + c);
                            w |= lf_is_sent(rv[0][c]) || lf_is_sent(rv[1][c]);
                        }
                        if (__ballot(w) == 0) break;
                        if (++polls > P.spin_limit) {
                            rec_ok = false;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(8);
                    }
                    if (!rec_ok && lane == 0) {   // the records are left unused and the loop ends
                        sabort = 1;
                        __hip_atomic_store(P.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                } else {
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int bb = lane + 64 * u;
                        const double* r = prow + (int64_t)(bb < nbr ? bb : 0) * LF_REC;
#pragma unroll
                        for (int c = 0; c < LF_REC; ++c) rv[u][c] = r[c];
                    }
                }
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    if (lane + 64 * u >= nbr || !rec_ok) continue;
                    F0 += rv[u][0];
                    F1 += rv[u][1];
                    F2 += rv[u][2];
                    const double t = rv[u][3];
                    const int j = (int)rv[u][4];
                    if (t < tb || (t == tb && j < jb)) {
                        tb = t;
                        jb = j;
                    }
                    nn += rv[u][5];
                }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {   // butterfly: every lane ends with the same sums
                    F0 += __shfl_xor(F0, off, 64);
                    F1 += __shfl_xor(F1, off, 64);
                    F2 += __shfl_xor(F2, off, 64);
                    nn += __shfl_xor(nn, off, 64);
                    const double t2 = __shfl_xor(tb, off, 64);
                    const int j2 = __shfl_xor(jb, off, 64);
                    if (t2 < tb || (t2 == tb && j2 < jb)) {
                        tb = t2;
                        jb = j2;
                    }
                }
                const bool own = (b == 0 && lane == 0);   // the writer of the group's lines
                if constexpr (LOOP) {   // counted here, written once at the end
                    nacc[q >> 2] += (unsigned long long)nn;
                    facc[q >> 2] += (unsigned long long)(N - (int64_t)nn);
                } else if (own) {   // added without waiting for them
                    atomicAdd(P.ncnt + 2 * l, (unsigned long long)nn);
                    atomicAdd(P.ncnt + 2 * l + 1, (unsigned long long)(N - (int64_t)nn));
                }
                const int phase = step_phase;
                const double h = a.h;
                double x0 = q0, x1 = q1, x2 = q2, I = I0;
                int32_t ns = ns0;
                int code = -1;   // -1: the line goes on
                if (phase == 4) {
                    if (jb != INT_MAX) {   // the step's segment hit a panel: the step is discarded
                        const int32_t k = P.body_kind[P.tri_body[jb]];
                        code = (k == BEM_DIRICHLET) ? BEM_STOP_DIRICHLET
                                                    : ((k == BEM_FLOATING) ? BEM_STOP_FLOATING : BEM_STOP_INTERFACE);
                    } else {   // accepted: its end point becomes the line's point
                        I = I0 + h / 6.0 * asum0;
                        x0 = p0;
                        x1 = p1;
                        x2 = p2;
                        ++ns;
                        if (P.path && own) {
                            P.path[l * P.pstride + 3 * ns + 0] = x0;
                            P.path[l * P.pstride + 3 * ns + 1] = x1;
                            P.path[l * P.pstride + 3 * ns + 2] = x2;
                        }
                        if (ns >= a.max_steps) code = BEM_STOP_MAXSTEPS;
                    }
                }
                double k0 = 0.0, k1 = 0.0, k2 = 0.0, asum = 0.0, y0 = 0.0, y1 = 0.0, y2 = 0.0;
                if (code < 0) {
                    const double m = sqrt(F0 * F0 + F1 * F1 + F2 * F2);
                    const double d0 = a.dir * F0 / m, d1 = a.dir * F1 / m, d2 = a.dir * F2 / m;
                    if (phase == 0 || phase == 4) {
                        if (!isfinite(m))
                            code = BEM_STOP_NONFINITE;
                        else if (m < a.e_min)
                            code = BEM_STOP_WEAK;
                        else {
                            k0 = d0;
                            k1 = d1;
                            k2 = d2;
                            asum = lb_alpha(a, m);
                            y0 = x0 + 0.5 * h * d0;
                            y1 = x1 + 0.5 * h * d1;
                            y2 = x2 + 0.5 * h * d2;
                        }
                    } else if (phase < 3) {
                        k0 = ks0 + 2.0 * d0;
                        k1 = ks1 + 2.0 * d1;
                        k2 = ks2 + 2.0 * d2;
                        asum = asum0 + 2.0 * lb_alpha(a, m);
                        const double cst = (phase == 1) ? 0.5 * h : h;
                        y0 = x0 + cst * d0;
                        y1 = x1 + cst * d1;
                        y2 = x2 + cst * d2;
                    } else {
                        k0 = ks0 + d0;
                        k1 = ks1 + d1;
                        k2 = ks2 + d2;
                        asum = asum0 + lb_alpha(a, m);
                        y0 = x0 + h / 6.0 * k0;
                        y1 = x1 + h / 6.0 * k1;
                        y2 = x2 + h / 6.0 * k2;
                        if (!(isfinite(y0) && isfinite(y1) && isfinite(y2))) code = BEM_STOP_NONFINITE;
                    }
                }
                if (own && code >= 0) {
                    P.n_steps[l] = ns;
                    P.stop_code[l] = code;
                    if (P.integral) P.integral[l] = I;
                    if (P.exceeds) P.exceeds[l] = (I > a.k_str) ? 1 : 0;
                }
                if (!LOOP && own) {
                    LFState nxt = P.nxt;
                    nxt.x[3 * s] = x0;
                    nxt.x[3 * s + 1] = x1;
                    nxt.x[3 * s + 2] = x2;
                    nxt.y[3 * s] = y0;
                    nxt.y[3 * s + 1] = y1;
                    nxt.y[3 * s + 2] = y2;
                    nxt.ks[3 * s] = k0;
                    nxt.ks[3 * s + 1] = k1;
                    nxt.ks[3 * s + 2] = k2;
                    nxt.asum[s] = asum;
                    nxt.I[s] = I;
                    nxt.ns[s] = ns;
                    nxt.line[s] = code < 0 ? l : -1;
                }
                if (code < 0) {
                    lo = l;
                    Y0 = y0; Y1 = y1; Y2 = y2;
                    X0 = x0; X1 = x1; X2 = x2;
                    K0 = k0; K1 = k1; K2 = k2;
                    AS = asum; II = I; NS = ns;
                }
            }
        } else if (!LOOP && s < S && b == 0 && lane == 0) {
            P.nxt.line[s] = -1;   // an empty slot stays empty in the other buffer
        }
        if (lane == 0) {
            sl[q] = lo;
            if (!LOOP) srhs[q] = (lo >= 0 && P.line_rhs) ? P.line_rhs[lo] : 0;
            sy[q][0] = Y0; sy[q][1] = Y1; sy[q][2] = Y2;
            sx[q][0] = X0; sx[q][1] = X1; sx[q][2] = X2;
            if constexpr (LOOP) {
                lks[q][0] = K0; lks[q][1] = K1; lks[q][2] = K2;
                lasum[q] = AS; lI[q] = II; lns[q] = NS;
            }
        }
    }
    __syncthreads();
    if (LOOP && sabort) break;   // uniform over the block
    if (!LOOP && b == 0 && tid == 0) {   // lines of the group still live after this step
        int nl = 0;
        for (int q = 0; q < LPB; ++q) nl += sl[q] >= 0 ? 1 : 0;
        if (nl > 0) atomicAdd(P.live + P.pidx, nl);
    }
    bool any = false;
    for (int q = 0; q < LPB; ++q) any |= sl[q] >= 0;
    if (!any) break;   // uniform over the block, and over the group's blocks
    if (LOOP && P.pass0 + it >= P.max_pass) break;   // not reached: the step limit stops every line first
    if (LOOP && it >= 2 && tid < LPB && s0 + tid < S) {   // the sentinel back into this block's records
        double* rr = P.lbuf + ((it + 1) % 3) * P.lstride + (s0 + tid) * pstride_part + b * LF_REC;
#pragma unroll
        for (int c = 0; c < LF_REC; ++c) lf_store_coh(rr + c, __longlong_as_double((long long)LF_SENT));
    }
    const bool hit_stage = (eval_phase == 4);   // the query points are proposed end points

    // ---- 2a. regular pairs, one panel per lane; near pairs queued per (slot, wave) ----
    double acc[LPB][3];
    int qc[LPB];
#pragma unroll
    for (int q = 0; q < LPB; ++q) {
        acc[q][0] = acc[q][1] = acc[q][2] = 0.0;
        qc[q] = 0;
    }
    const LBSeries kser = lb_series_consts();
    for (int r = 0; r < rnd; ++r) {
        const int64_t base = jb0 + (int64_t)r * 256;
        if (base >= N) break;   // uniform
        const int64_t j = base + tid;   // < Np: Np is a multiple of 256 above N
        const bool valid = j < N;
        if (r > 0) {
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                rx[k] = farR[(int64_t)(FR_X + k) * Np + j];
                ry[k] = farR[(int64_t)(FR_Y + k) * Np + j];
                rz[k] = farR[(int64_t)(FR_Z + k) * Np + j];
                rw[k] = farR[(int64_t)(FR_W + k) * Np + j];
            }
            rc0 = far64[(int64_t)(FR_CC + 0) * Np + j];
            rc1 = far64[(int64_t)(FR_CC + 1) * Np + j];
            rc2 = far64[(int64_t)(FR_CC + 2) * Np + j];
            rrr = far64[(int64_t)FR_RR * Np + j];
        }
        const R(&qx)[7] = rx;
        const R(&qy)[7] = ry;
        const R(&qz)[7] = rz;
        const R(&qw)[7] = rw;
        const double ccx = rc0, ccy = rc1, ccz = rc2, rr = rrr;
#pragma unroll
        for (int q = 0; q < LPB; ++q) {
            if (sl[q] < 0) continue;   // uniform
            const double p0 = sy[q][0], p1 = sy[q][1], p2 = sy[q][2];
            const bool reg = valid && is_regular(p0 - ccx, p1 - ccy, p2 - ccz, rr);
            const bool near = valid && !reg;
            const uint64_t nm = __ballot(near);
            if (nm) {
                const int pos = qc[q] + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(nm >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)nm, 0u));
                if (near) nq[q][wv][pos] = (uint16_t)(r * 256 + tid);
                qc[q] += __popcll(nm);
            }
            if (reg) {
                const R pr0 = (R)p0, pr1 = (R)p1, pr2 = (R)p2;
                R f0 = 0, f1 = 0, f2 = 0;
#pragma unroll
                for (int k = 0; k < 7; ++k) {
                    const R dx = pr0 - qx[k], dy = pr1 - qy[k], dz = pr2 - qz[k];
                    const R r2 = dx * dx + dy * dy + dz * dz;
                    const R tw = lb_w_r3(qw[k], r2, kser);
                    f0 += tw * dx;
                    f1 += tw * dy;
                    f2 += tw * dz;
                }
                const double sg = fsol[(int64_t)srhs[q] * fn + j];
                acc[q][0] = fma(sg, (double)f0, acc[q][0]);
                acc[q][1] = fma(sg, (double)f1, acc[q][1]);
                acc[q][2] = fma(sg, (double)f2, acc[q][2]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < LPB; ++q) {
        if (sl[q] < 0) continue;
        const double e0 = wave_sum(acc[q][0]), e1 = wave_sum(acc[q][1]), e2 = wave_sum(acc[q][2]);
        if (lane == 0) {
            fred[wv][q][0] = e0;
            fred[wv][q][1] = e1;
            fred[wv][q][2] = e2;
            nqc[q][wv] = qc[q];
        }
    }
    __syncthreads();

    // ---- 2b. near pairs: slot q's queue over its G threads (closed forms in FP64) ----
    {
        const int q = tid / G, k = tid % G;
        double n0 = 0.0, n1 = 0.0, n2 = 0.0, tb = 2.0;
        int jb = INT_MAX;
        if (sl[q] >= 0) {
            const int c0 = nqc[q][0], c1 = nqc[q][1], c2 = nqc[q][2], c3 = nqc[q][3];
            const int tot = c0 + c1 + c2 + c3;
            const double p0 = sy[q][0], p1 = sy[q][1], p2 = sy[q][2];
            const double x0 = sx[q][0], x1 = sx[q][1], x2 = sx[q][2];
            const double* sig = sol + (int64_t)srhs[q] * n;
            for (int e = k; e < tot; e += G) {
                int w = 0, i = e;
                if (i >= c0) {
                    i -= c0;
                    w = 1;
                    if (i >= c1) {
                        i -= c1;
                        w = 2;
                        if (i >= c2) {
                            i -= c2;
                            w = 3;
                        }
                    }
                }
                const int64_t j = jb0 + nq[q][w][i];
                const double* Tj = tri64 + (int64_t)TRI_REC * j;
                if constexpr (NODAL && LOOP) {
                    const LFVec3 E = nodal_tri_E_call(Tj, p0, p1, p2, sol[ntri[3 * j]], sol[ntri[3 * j + 1]],
                                                      sol[ntri[3 * j + 2]]);
                    n0 += E.x;
                    n1 += E.y;
                    n2 += E.z;
                } else if constexpr (NODAL) {
                    double ph = 0.0;
                    nodal_tri_phiE(Tj, p0, p1, p2, sol[ntri[3 * j]], sol[ntri[3 * j + 1]], sol[ntri[3 * j + 2]], ph,
                                   n0, n1, n2);
                } else {
                    double F0, F1, F2;
                    if constexpr (LOOP) {
                        const LFVec3 F = flat_tri_F_call(Tj, p0, p1, p2);
                        F0 = F.x;
                        F1 = F.y;
                        F2 = F.z;
                    } else {
                        flat_tri_F_seq(Tj, p0, p1, p2, F0, F1, F2);
                    }
                    const double sg = sig[j];
                    n0 = fma(sg, F0, n0);
                    n1 = fma(sg, F1, n1);
                    n2 = fma(sg, F2, n2);
                }
                if (hit_stage) {
                    const double th = lb_segment_tri(Tj, x0, x1, x2, p0 - x0, p1 - x1, p2 - x2);
                    if (th >= 0.0 && (th < tb || (th == tb && (int)j < jb))) {
                        tb = th;
                        jb = (int)j;
                    }
                }
            }
        }
        // fixed-order reduction over the slot's threads: within each wave, then over its waves
#pragma unroll
        for (int off = GW / 2; off > 0; off >>= 1) {
            n0 += __shfl_xor(n0, off, 64);
            n1 += __shfl_xor(n1, off, 64);
            n2 += __shfl_xor(n2, off, 64);
            const double t2 = __shfl_xor(tb, off, 64);
            const int j2 = __shfl_xor(jb, off, 64);
            if (t2 < tb || (t2 == tb && j2 < jb)) {
                tb = t2;
                jb = j2;
            }
        }
        if (k % GW == 0) {
            const int u = k / GW;
            nred[q][u][0] = n0;
            nred[q][u][1] = n1;
            nred[q][u][2] = n2;
            nred[q][u][3] = tb;
            nredj[q][u] = jb;
        }
    }
    __syncthreads();

    // ---- 3. one partial record per live slot ----
    if (tid < LPB && sl[tid] >= 0) {
        const int q = tid;
        double e[3], tb = 2.0;
        int jb = INT_MAX;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double v = (fred[0][q][c] + fred[1][q][c]) + (fred[2][q][c] + fred[3][q][c]);
            double nv = nred[q][0][c];
            for (int u = 1; u < NU; ++u) nv += nred[q][u][c];
            e[c] = v + nv;
        }
        for (int u = 0; u < NU; ++u)
            if (nred[q][u][3] < tb || (nred[q][u][3] == tb && nredj[q][u] < jb)) {
                tb = nred[q][u][3];
                jb = nredj[q][u];
            }
        double* rec = part_wr + (s0 + q) * pstride_part + b * LF_REC;
        const double rv[LF_REC] = {e[0], e[1], e[2], tb, (double)jb,
                                   (double)(nqc[q][0] + nqc[q][1] + nqc[q][2] + nqc[q][3])};
        // LOOP: the sentinel stores of this pass (same lanes) land before any record word
        if constexpr (LOOP) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
#pragma unroll
        for (int c = 0; c < LF_REC; ++c) {
            if constexpr (LOOP)
                lf_store_coh(rec + c, rv[c]);
            else
                rec[c] = rv[c];
        }
    }
    if constexpr (!LOOP) break;
    }   // passes
    if constexpr (LOOP) {   // the pair counts of the lines this wave finished
        for (int q = wv; q < LPB; q += 4) {
            const int32_t l = lline[q];
            if (b == 0 && lane == 0 && l >= 0) {
                P.ncnt[2 * l] += nacc[q >> 2];
                P.ncnt[2 * l + 1] += facc[q >> 2];
            }
        }
    }
    kclock_stop(P.kts);
}

template <typename R, int LPB, bool NODAL>
__global__ __launch_bounds__(256) void k_lf_pass(LFArgs P) {
    lf_run<R, LPB, NODAL, false>(P);
}

template <typename R, int LPB, bool NODAL>
__global__ __launch_bounds__(256) void k_lf_loop(LFArgs P) {
    lf_run<R, LPB, NODAL, true>(P);
}

__global__ void k_lf_zero_u32(int64_t m, uint32_t* __restrict__ v) {
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) v[i] = 0;
}

__global__ __launch_bounds__(256) void k_lf_init(int64_t L, const double* __restrict__ starts, LFState s,
                                                 double* __restrict__ path, int64_t pstride,
                                                 unsigned long long* __restrict__ ncnt) {
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (l >= L) return;
    ncnt[2 * l] = 0;
    ncnt[2 * l + 1] = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double v = starts[3 * l + k];
        s.x[3 * l + k] = v;
        s.y[3 * l + k] = v;
        s.ks[3 * l + k] = 0.0;
        if (path) path[l * pstride + k] = v;
    }
    s.asum[l] = 0.0;
    s.I[l] = 0.0;
    s.ns[l] = 0;
    s.line[l] = (int32_t)l;
}

__global__ void k_lf_zero3(int32_t* __restrict__ live) {
    if (threadIdx.x < 3) live[threadIdx.x] = 0;
}

// Fold of the live slots to the front, order kept: src_of[d] = the d-th live slot of [0, S), -1
// for d in [live, K).  One block.
__global__ __launch_bounds__(1024) void k_lf_fold_map(int64_t S, int64_t K, const int32_t* __restrict__ line,
                                                      int32_t* __restrict__ src_of) {
    __shared__ int32_t wsum[16];
    __shared__ int32_t carry;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) carry = 0;
    for (int64_t d = tid; d < K; d += 1024) src_of[d] = -1;
    __syncthreads();
    for (int64_t base = 0; base < S; base += 1024) {
        const int64_t s = base + tid;
        const int f = (s < S && line[s] >= 0) ? 1 : 0;
        int incl = f;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off, 64);
            if (lane >= off) incl += v;
        }
        if (lane == 63) wsum[wv] = incl;
        __syncthreads();
        int wb = carry;
        for (int w = 0; w < wv; ++w) wb += wsum[w];
        const int d = wb + incl - f;
        if (f && d < K) src_of[d] = (int32_t)s;
        __syncthreads();
        if (tid == 0) {
            int t = 0;
            for (int w = 0; w < 16; ++w) t += wsum[w];
            carry += t;
        }
        __syncthreads();
    }
}

// one block of 64 per destination slot d < K: the state and partial row of slot src_of[d] moved
// from (a, pa) to (b, pb); d without a source gets no line
__global__ __launch_bounds__(64) void k_lf_fold_move(int64_t K, const int32_t* __restrict__ src_of, LFState a,
                                                     LFState bs, const double* __restrict__ pa,
                                                     double* __restrict__ pb, int64_t pstride_part, int nrec) {
    const int64_t d = blockIdx.x;
    const int32_t s = src_of[d];
    const int t = threadIdx.x;
    if (s < 0) {
        if (t == 0) bs.line[d] = -1;
        return;
    }
    if (t < 3) {
        bs.x[3 * d + t] = a.x[3 * (int64_t)s + t];
        bs.y[3 * d + t] = a.y[3 * (int64_t)s + t];
        bs.ks[3 * d + t] = a.ks[3 * (int64_t)s + t];
    } else if (t == 3) {
        bs.asum[d] = a.asum[s];
        bs.I[d] = a.I[s];
        bs.ns[d] = a.ns[s];
        bs.line[d] = a.line[s];
    }
    for (int k = t; k < nrec * LF_REC; k += 64) pb[d * pstride_part + k] = pa[(int64_t)s * pstride_part + k];
}

// the lines' near and far pair counts added to the context's counters (one block, fixed order)
__global__ __launch_bounds__(256) void k_lf_count_sum(int64_t L, const unsigned long long* __restrict__ ncnt,
                                                      unsigned long long* __restrict__ counters) {
    __shared__ unsigned long long red[2][256];
    unsigned long long x = 0, y = 0;
    for (int64_t l = threadIdx.x; l < L; l += 256) {
        x += ncnt[2 * l];
        y += ncnt[2 * l + 1];
    }
    red[0][threadIdx.x] = x;
    red[1][threadIdx.x] = y;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long sx = 0, sy = 0;
        for (int k = 0; k < 256; ++k) {
            sx += red[0][k];
            sy += red[1][k];
        }
        counters[0] += sx;
        counters[1] += sy;
    }
}

// the persistent loop's kernel for a precision and a block shape
const void* lf_loop_kernel(bool nodal, bool fp64, int lpb) {
#define BEM_LK(R, ND)                                                                                    \
    (lpb == 1 ? reinterpret_cast<const void*>(&k_lf_loop<R, 1, ND>)                                      \
              : lpb == 2 ? reinterpret_cast<const void*>(&k_lf_loop<R, 2, ND>)                           \
                         : lpb == 4 ? reinterpret_cast<const void*>(&k_lf_loop<R, 4, ND>)                \
                                    : reinterpret_cast<const void*>(&k_lf_loop<R, 8, ND>))
    return nodal ? BEM_LK(double, true) : (fp64 ? BEM_LK(double, false) : BEM_LK(float, false));
#undef BEM_LK
}

// Every remaining pass of the slots [0, S) in one persistent launch (k_lf_loop): the fewest line
// slots per block whose grid the GPU holds at once, which a cooperative launch guarantees, and
// one 256-panel round per block where the panel count allows.  Waits for the launch and raises
// an error if one of its waits reached its bound.  Returns false, launching nothing, when no
// block shape fits.
template <typename MakeArgs>
bool fused_loop_launch(bem_ctx* c, bool nodal, bool fp64, int64_t S, int64_t N, MakeArgs&& args) {
    int cus = 0;
    BEM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
    // shapes by the pairs a thread evaluates per pass (slots x rounds), one round first (a second
    // round's records are loaded again every pass).  A grid of at most one block per CU first: a
    // CU holding two blocks takes twice as long over each pass, and every block waits for it
    // (measured on the 19,732-panel coax, us a stage: 4 slots 12.9 with one slot a block, 312
    // blocks, against 10.9 with two, 156 blocks; 3 slots 9.4 with one slot a block, 234 blocks)
    static const int shapes[][2] = {{1, 1}, {2, 1}, {1, 2}, {4, 1}, {2, 2}, {1, 4}, {8, 1}, {4, 2}, {2, 4},
                                    {8, 2}, {4, 4}, {8, 4}};
    for (int pass = 0; pass < 2; ++pass)
    for (const auto& sh : shapes) {
        const int lpb = sh[0], rnd = sh[1];
        if ((c->tune_trace_lpb > 0 && lpb != c->tune_trace_lpb) || (c->tune_trace_rnd > 0 && rnd != c->tune_trace_rnd))
            continue;
        const int nb = fused_trace_blocks(N, rnd);
        if (nb == 0) continue;
        const void* f = lf_loop_kernel(nodal, fp64, lpb);
        int per_cu = 0;
        BEM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 256, 0));
        const int64_t grid = ceil_div(S, lpb) * nb;
        if (grid > (int64_t)per_cu * cus || (pass == 0 && grid > cus)) continue;
        LFArgs P = args(lpb, rnd, nb);
        // the three record buffers, every word the sentinel, and the error flag cleared
        P.lstride = S * P.pstride_part;
        c->lf_loop.alloc(sizeof(double) * 3 * (size_t)P.lstride);
        P.lbuf = c->lf_loop.as<double>();
        const int64_t nw = 3 * P.lstride;
        hipLaunchKernelGGL(k_lf_fill_sent, dim3((unsigned)std::min<int64_t>(ceil_div(nw, 256), 1024)), dim3(256), 0,
                           c->stream, nw, reinterpret_cast<unsigned long long*>(P.lbuf));
        BEM_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_lf_zero_u32, dim3(1), dim3(256), 0, c->stream, (int64_t)1,
                           reinterpret_cast<uint32_t*>(P.err));
        BEM_CHECK_LAUNCH();
        hipEvent_t fa = nullptr, fb = nullptr;
        const bool timed = c->profiling == 1;
        if (timed) {
            timing_events(c, &fa, &fb);
            BEM_HIP(hipEventRecord(fa, c->stream));
        }
        void* kargs[] = {&P};
        const hipError_t le = hipLaunchCooperativeKernel(f, dim3((unsigned)grid), dim3(256), kargs, 0, c->stream);
        if (le != hipSuccess) {   // refused (nothing launched): the caller goes on one launch per stage
            (void)hipGetLastError();
            if (timed) {
                c->event_pool.push_back(fa);
                c->event_pool.push_back(fb);
            }
            return false;
        }
        if (timed) {
            BEM_HIP(hipEventRecord(fb, c->stream));
            push_timing(c, "trace_pass", fa, fb);
        }
        int32_t* host = c->host_stage.as<int32_t>() + 32;
        BEM_HIP(hipMemcpyAsync(host, P.err, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        BEM_HIP(hipStreamSynchronize(c->stream));
        if (*host != 0) throw Error(BEM_ERR_HIP, "field lines: a wait between the blocks of the persistent pass loop reached its bound");
        return true;
    }
    return false;
}

}  // namespace

// Panel blocks of the fused layout for N panels with rnd rounds of 256: 0 when N needs more
// than LF_NBMAX blocks (the caller then takes the two-kernel layout).
int fused_trace_blocks(int64_t N, int rnd) {
    const int64_t nb = ceil_div(N, 256 * (int64_t)rnd);
    return nb <= LF_NBMAX ? (int)nb : 0;
}

// Launches for passes pass0 .. max_pass - 1 of the lines in slots [0, S) of buf[rd] (x, y the
// line point and the query point of pass pass0; slots past the live lines hold line -1), each
// launch also finishing the previous pass; the launch after the last pass only finishes it.
void fused_trace_loop(bem_ctx* c, const double* sol, int64_t L, const int32_t* line_rhs, const bem_trace_params* tp,
                      int32_t* n_steps, int32_t* stop_code, double* path, double* integral, uint8_t* exceeds,
                      LFState buf0, LFState buf1, int64_t S, int64_t pass0, unsigned long long* ncnt) {
    if (S == 0) return;
    const int64_t Np = (int64_t)(c->far64.bytes / (sizeof(double) * FAR_REC));
    const int64_t N = c->N;
    const int64_t pstride = 3 * ((int64_t)tp->max_steps + 1);
    LBArgs a;
    a.h = tp->h;
    a.e_min = tp->e_min;
    a.dir = tp->direction >= 0 ? 1.0 : -1.0;
    a.a = tp->alpha_a;
    a.e0 = tp->alpha_e0;
    a.p = tp->alpha_p;
    a.k_str = tp->k_str;
    a.max_steps = tp->max_steps;
    // the block shape for a slot count: lines per block and 256-panel rounds per block
    // (measured on the 19,732-panel coax, us per stage: 3 lines 12.3 with 1 a block against 13.4
    // with 2; 8 lines 14.9 with 2 against 18.3 with 1; 16 lines 18.0 with 4 against 21.0 with 2,
    // all with one round; four rounds from 32 lines)
    auto shape = [&](int64_t s, int* lpb, int* rnd) {
        *lpb = c->tune_trace_lpb > 0 ? c->tune_trace_lpb : (s >= 128 ? 8 : (s >= 12 ? 4 : (s >= 4 ? 2 : 1)));
        *rnd = c->tune_trace_rnd > 0 ? c->tune_trace_rnd : (s >= 32 ? 4 : 1);
        while (*rnd < LF_RNDMAX && fused_trace_blocks(N, *rnd) == 0) *rnd *= 2;
    };
    const int64_t prs = (int64_t)LF_NBMAX * LF_REC;   // partial row stride per slot
    // two partial buffers, the fold map, three live counters and the persistent loop's error flag
    c->lf_part.alloc(sizeof(double) * 2 * (size_t)prs * (size_t)S + sizeof(int32_t) * ((size_t)S + 64));
    double* part[2] = {c->lf_part.as<double>(), c->lf_part.as<double>() + prs * S};
    int32_t* src_of = reinterpret_cast<int32_t*>(part[1] + prs * S);
    int32_t* live = src_of + S;
    int32_t* err = live + 32;
    hipLaunchKernelGGL(k_lf_zero3, dim3(1), dim3(64), 0, c->stream, live);
    BEM_CHECK_LAUNCH();
    if (c->coop_launch < 0) {
        int v = 0;
        BEM_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeCooperativeLaunch, c->device));
        c->coop_launch = v ? 1 : 0;
    }
    LFState buf[2] = {buf0, buf1};
    // nodal basis (one load case): records whose node weights carry the density, with a density
    // of one per panel, in FP64 in either precision; the near pairs read the vertex values
    const bool nodal = c->opt.basis == BEM_BASIS_LINEAR;
    const bool fp64 = c->opt.precision == BEM_FP64 || nodal;
    const double* F64 = nodal ? c->nod_far64.as<double>() : c->far64.as<double>();
    const double* fsol = nodal ? c->nod_ones.as<double>() : sol;
    const int64_t fn = nodal ? 0 : c->n;
    const int64_t max_pass = 4 * (int64_t)tp->max_steps + 1;
    // live counts come back asynchronously (a copy and an event every 16 launches); the host waits
    // only for the count of 64 launches back, so it never runs further ahead than that
    constexpr int NEV = 8;
    for (int k = 0; k < NEV; ++k)
        if (!c->lf_ev[k]) BEM_HIP(hipEventCreateWithFlags(&c->lf_ev[k], hipEventDisableTiming));
    c->host_stage.alloc(sizeof(int32_t) * 64);
    int32_t* host = c->host_stage.as<int32_t>();
    int64_t ev_launch[NEV];
    int head = 0, tail = 0;   // pending counts: [tail, head)
    int64_t known = S;
    int rd = 0, pw = 0;       // state buffer the next launch reads, partial buffer it writes
    int nb_prev = 0;
    for (int64_t p = 0; pass0 + p <= max_pass; ++p) {
        // counts that have arrived (waiting for those 64 or more launches old)
        while (tail < head) {
            const int k = tail % NEV;
            if (ev_launch[k] > p - 64) {
                const hipError_t e = hipEventQuery(c->lf_ev[k]);
                if (e == hipErrorNotReady) {
                    (void)hipGetLastError();   // not an error: leave no trace for the next launch check
                    break;
                }
                BEM_HIP(e);
            } else {
                BEM_HIP(hipEventSynchronize(c->lf_ev[k]));
            }
            known = std::min<int64_t>(known, host[k]);
            ++tail;
        }
        if (known == 0) break;
        if (known <= S / 2 && p > 0) {
            // fold the live slots to the front: state of buffer rd and partial rows of buffer pw ^ 1
            // (those of the last launch) into the other buffers, which become the current ones
            hipLaunchKernelGGL(k_lf_fold_map, dim3(1), dim3(1024), 0, c->stream, S, known, buf[rd].line, src_of);
            BEM_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_lf_fold_move, dim3((unsigned)known), dim3(64), 0, c->stream, known, src_of, buf[rd],
                               buf[rd ^ 1], part[pw ^ 1], part[pw], prs, nb_prev);
            BEM_CHECK_LAUNCH();
            rd ^= 1;
            pw ^= 1;
            S = known;
        }
        // the arguments of a launch that finishes pass pass0 + p - 1 and evaluates pass pass0 + p
        auto args = [&](int lpb, int rnd, int nb) {
            LFArgs P;
            P.far64 = F64;
            P.farR = fp64 ? static_cast<const void*>(F64) : static_cast<const void*>(c->far32.as<float>());
            P.Np = Np;
            P.N = N;
            P.tri64 = c->tri64.as<double>();
            P.tri_body = c->tri_body.as<int32_t>();
            P.body_kind = c->body_kind.as<int32_t>();
            P.fsol = fsol;
            P.fn = fn;
            P.sol = sol;
            P.n = c->n;
            P.line_rhs = line_rhs;
            P.ntri = c->tri.as<int32_t>();
            P.step_phase = p == 0 ? -1 : lf_phase_of(pass0 + p - 1);
            P.eval_phase = lf_phase_of(pass0 + p);
            P.nb_prev = nb_prev;
            P.nb = nb;
            P.rnd = rnd;
            P.S = S;
            P.pstride_part = prs;
            P.cur = buf[rd];
            P.nxt = buf[rd ^ 1];
            P.part_prev = part[pw ^ 1];
            P.part_cur = part[pw];
            P.a = a;
            P.n_steps = n_steps;
            P.stop_code = stop_code;
            P.integral = integral;
            P.exceeds = exceeds;
            P.path = path;
            P.pstride = pstride;
            P.ncnt = ncnt;
            P.live = live;
            P.pidx = (int)(p % 3);
            P.pass0 = pass0 + p;
            P.max_pass = max_pass;
            P.lbuf = nullptr;
            P.lstride = 0;
            P.err = err;
            P.spin_limit = (uint32_t)c->tune_trace_spin;
            P.kts = kclock_slot(c, "trace_pass");
            (void)lpb;
            return P;
        };
        // every remaining pass in one persistent launch, once the slots fit the GPU at once
        if (S <= c->tune_trace_loop && c->coop_launch > 0) {
            if (fused_loop_launch(c, nodal, fp64, S, N, args)) {
                ++c->trace_pass_launches;
                break;
            }
        }
        int lpb, rnd;
        shape(S, &lpb, &rnd);
        const int nb = fused_trace_blocks(N, rnd);
        const LFArgs P = args(lpb, rnd, nb);
        const dim3 grid((unsigned)(nb * ceil_div(S, lpb)));
        // timing: events carried in the dispatch (profiling mode 1) or the kernel's own clock (mode 2)
        hipEvent_t fa = nullptr, fb = nullptr;
        const bool timed = c->profiling == 1;
        if (timed) timing_events(c, &fa, &fb);
#define BEM_LF(R, LPB, ND) \
    hipExtLaunchKernelGGL((k_lf_pass<R, LPB, ND>), grid, dim3(256), 0, c->stream, fa, fb, 0, P)
#define BEM_LF_LPB(R, ND)    \
    if (lpb == 1)            \
        BEM_LF(R, 1, ND);    \
    else if (lpb == 2)       \
        BEM_LF(R, 2, ND);    \
    else if (lpb == 4)       \
        BEM_LF(R, 4, ND);    \
    else                     \
        BEM_LF(R, 8, ND)
        if (nodal) {
            BEM_LF_LPB(double, true);
        } else if (fp64) {
            BEM_LF_LPB(double, false);
        } else {
            BEM_LF_LPB(float, false);
        }
#undef BEM_LF_LPB
#undef BEM_LF
        BEM_CHECK_LAUNCH();
        if (timed) push_timing(c, "trace_pass", fa, fb);
        ++c->trace_pass_launches;
        rd ^= 1;
        pw ^= 1;
        nb_prev = nb;
        const int pidx = (int)(p % 3);
        if ((p & 15) == 15) {   // this launch's live count, read back without waiting
            if (head - tail == NEV) {   // ring full: take the oldest
                const int k = tail % NEV;
                BEM_HIP(hipEventSynchronize(c->lf_ev[k]));
                known = std::min<int64_t>(known, host[k]);
                ++tail;
            }
            const int k = head % NEV;
            BEM_HIP(hipMemcpyAsync(host + k, live + pidx, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
            BEM_HIP(hipEventRecord(c->lf_ev[k], c->stream));
            ev_launch[k] = p;
            ++head;
        }
    }
    // the pinned count buffer is shared: let the pending copies land before returning
    if (tail < head) BEM_HIP(hipEventSynchronize(c->lf_ev[(head - 1) % NEV]));
    (void)L;
}

void launch_trace_fused(bem_ctx* c, int32_t nrhs, const double* sol, int64_t L, const int32_t* line_rhs,
                        const double* starts, const bem_trace_params* tp, int32_t* n_steps, int32_t* stop_code,
                        double* path, double* integral, uint8_t* exceeds) {
    (void)nrhs;
    if (L == 0) return;
    KTimer t(c, "trace");
    const int64_t pstride = 3 * ((int64_t)tp->max_steps + 1);
    // two state buffers (x, y, ks: 3 doubles; asum, I: 1 double; ns, line: 1 int32 per slot) and
    // two pair counters per line
    c->lb_state.alloc(sizeof(double) * (size_t)L * 22 + sizeof(unsigned long long) * 2 * (size_t)L +
                      sizeof(int32_t) * (size_t)L * 4);
    double* dbase = c->lb_state.as<double>();
    unsigned long long* ncnt = reinterpret_cast<unsigned long long*>(dbase + (size_t)L * 22);
    int32_t* ibase = reinterpret_cast<int32_t*>(ncnt + 2 * (size_t)L);
    LFState buf[2];
    for (int k = 0; k < 2; ++k) {
        double* d = dbase + (size_t)L * 11 * k;
        int32_t* i = ibase + (size_t)L * 2 * k;
        buf[k] = {d, d + 3 * L, d + 6 * L, d + 9 * L, d + 10 * L, i, i + L};
    }
    hipLaunchKernelGGL(k_lf_init, dim3((unsigned)ceil_div(L, 256)), dim3(256), 0, c->stream, L, starts, buf[0], path,
                       pstride, ncnt);
    BEM_CHECK_LAUNCH();
    if (c->opt.basis == BEM_BASIS_LINEAR) launch_nodal_records(c, sol);
    kclock_begin(c, 4 * (int64_t)tp->max_steps + 3);
    fused_trace_loop(c, sol, L, line_rhs, tp, n_steps, stop_code, path, integral, exceeds, buf[0], buf[1], L, 0,
                     ncnt);
    kclock_end(c);
    hipLaunchKernelGGL(k_lf_count_sum, dim3(1), dim3(256), 0, c->stream, L, ncnt,
                       reinterpret_cast<unsigned long long*>(c->counters.p) + 2);
    BEM_CHECK_LAUNCH();
}

}  // namespace bem
