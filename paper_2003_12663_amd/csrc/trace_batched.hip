// Field lines and the streamer integral with all lines advancing together
// (Sec. 1, Eq. Breakdowncrit; RK4 on dx/ds = dir E/|E|).
//
// Every active line needs one field evaluation per RK4 stage, and a line's
// stages depend on each other, so one line alone cannot fill the GPU.  Here
// all active lines advance by one stage per pass, and a pass is one batched
// evaluation spread over the whole GPU, in two launches:
//  k_lb_far  - (line tile x panel chunk) blocks: a block walks a chunk of C
//              panels (each record read at a wave-uniform address into scalar
//              registers) and evaluates the regular pairs of its lines by the
//              7-point rule, one line per lane.
//              Near pairs are not evaluated here (Sec. 4: near-singular pairs
//              are marked and done after the regular ones); each lane records
//              them in a bit mask.  Output per (line, chunk): partial field and
//              near mask, line-major (a line's KS partials are contiguous, so
//              the step kernel reads them coalesced).
//  k_lb_step - one block per active line: sums the partials in a fixed order,
//              evaluates the line's near pairs with the closed forms (all 256
//              threads, fixed-order sums, so runs are bitwise reproducible),
//              tests them against the step's segment on end-of-step passes,
//              advances the RK4 stage machine, accumulates the streamer
//              integral, stops the line (hit, weak field, max steps,
//              non-finite) and appends survivors to the next active list.
// All lines start together, so every active line is in the same RK4 stage in
// a given pass.  A panel that a step's segment can reach lies within R + h of
// the step's end point, hence in its near set when h < (eta - 1) R_min.
#include <algorithm>
#include <climits>

#include "bem_device.h"
#include "nodal_device.h"
#include "trace_device.h"

#include <hip/hip_ext.h>

namespace bem {
namespace {

constexpr int LB_C = 32;         // panels per chunk



// slot-indexed line state: slots [0, count) of a buffer hold the live lines (trace_device.h);
// each pass moves every line that goes on to the slot it draws in the other buffer, so every
// kernel indexes by slot and nothing waits on an active-list lookup
using LBState = LFState;

// the same buffer seen from slot lo on (a line group's slot range)
inline LBState lb_shift(LBState s, int64_t lo) {
    return {s.x + 3 * lo, s.y + 3 * lo, s.ks + 3 * lo, s.asum + lo, s.I + lo, s.ns + lo, s.line + lo};
}

// Lines [g L / G, (g + 1) L / G) form group g, in slots [g L / G, (g + 1) L / G) of buffer 0
// at the start; its live count is count[32 g].
__global__ __launch_bounds__(256) void k_lb_init(int64_t L, int32_t G, const double* __restrict__ starts, LBState s,
                                                 int32_t* __restrict__ count, double* __restrict__ path,
                                                 int64_t pstride, unsigned long long* __restrict__ ncnt) {
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (l < G) count[32 * l] = (int32_t)((l + 1) * L / G - l * L / G);
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

// SPLIT = 1: TILE_LINES (64, 128 or 256) lines per block, one per lane, every lane
// walks the whole chunk.
// SPLIT > 1: 64 lines per block (SPLIT waves); wave w walks panels
// [w C/SPLIT, (w + 1) C/SPLIT) of the chunk and the partial fields are added
// in wave order (for few lines: 1/SPLIT of the serial work per lane).
// A wave walks its panels in step, so each panel's record (panel-major, pan64 /
// panR) is read at a wave-uniform address: it comes through the scalar cache
// into scalar registers, which the FP64 (or FP32) arithmetic takes as operands
// directly; nothing is staged in LDS and no lane reads a record of its own.
template <typename R, int SPLIT, int TILE_LINES>
__global__ __launch_bounds__(SPLIT > 1 ? 64 * SPLIT : TILE_LINES) void k_lb_far(const double* __restrict__ pan64, const R* __restrict__ panR,
                                                 int64_t N, const double* __restrict__ sol, int64_t n,
                                                 const int32_t* __restrict__ line_rhs,
                                                 const int32_t* __restrict__ line_of, int64_t cap,
                                                 const int32_t* __restrict__ count, int32_t* __restrict__ count_next,
                                                 const double* __restrict__ ys, double* __restrict__ part,
                                                 uint32_t* __restrict__ pmask, int32_t tiles, int64_t KS,
                                                 unsigned long long* __restrict__ kts) {
    constexpr int TILE = SPLIT > 1 ? 64 : TILE_LINES;         // lines per block
    kclock_start(kts);
    constexpr int PER = LB_C / SPLIT;
    __shared__ double wred[SPLIT > 1 ? SPLIT : 1][64][3];
    __shared__ uint32_t wmask[SPLIT > 1 ? SPLIT : 1][64];

    // XCD-aware order: blocks are dealt to the 8 XCDs round-robin by linear id; XCD x takes the
    // contiguous chunk range [x CPX, (x + 1) CPX) (CPX = ceil(KS / 8)), all tiles of each.  So the
    // tiles of one chunk share one XCD's L2 for the chunk's records, and each line's partials
    // from one XCD form one contiguous run of its line-major row (whole cache lines written back)
    const int64_t bid = blockIdx.x, xcd = bid & 7, m = bid >> 3;
    const int64_t CPX = (KS + 7) >> 3;
    const int64_t tile = m % tiles, chunk = xcd * CPX + m / tiles;
    const int64_t tile0 = tile * TILE;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int64_t t = tile0 + (SPLIT > 1 ? lane : (int)threadIdx.x);
    const int64_t j0 = chunk * LB_C;
    const int nc = (int)((N - j0) < LB_C ? (N - j0) : LB_C);
    const int pj0 = SPLIT > 1 ? wv * PER : 0;
    const int pj1 = SPLIT > 1 ? (pj0 + PER < nc ? pj0 + PER : nc) : nc;
    // Requested together and waited for once, before any exit: the live count, the slot's
    // query point (slot clamped into the group's cap slots; a slot past the count is never
    // used) and the wave's first panel record (index clamped to a real panel).  Left to
    // itself the compiler issues each of these after the branch that precedes its first use,
    // one round trip after another.
    const int64_t jf = (j0 + pj0 < N) ? j0 + pj0 : N - 1;
    R qf[FR_CC];
    double cf[4];
#pragma unroll
    for (int k = 0; k < FR_CC; ++k) qf[k] = panR[FAR_REC * jf + k];
#pragma unroll
    for (int k = 0; k < 4; ++k) cf[k] = pan64[FAR_REC * jf + FR_CC + k];
    const int64_t tc = t < cap ? t : cap - 1;
    const double p0 = ys[3 * tc], p1 = ys[3 * tc + 1], p2 = ys[3 * tc + 2];
    const int32_t A = count[0];
    asm volatile("" ::"s"(A), "v"(p0), "v"(p1), "v"(p2), "s"(qf[0]), "s"(qf[FR_CC - 1]), "s"(cf[0]), "s"(cf[3]));
    if (bid == 0 && threadIdx.x == 0) count_next[0] = 0;
    if (chunk >= KS) {   // padding of the chunk count to a multiple of 8
        kclock_stop(kts);
        return;
    }
    if (tile0 >= A) {    // uniform over the block
        kclock_stop(kts);
        return;
    }
    const bool live = t < A;
    double e0 = 0.0, e1 = 0.0, e2 = 0.0;
    uint32_t nmask = 0;
    if (live) {
        const double* sig = sol + (line_rhs ? (int64_t)line_rhs[line_of[t]] * n : 0);
        const R pr0 = (R)p0, pr1 = (R)p1, pr2 = (R)p2;
        const LBSeries ks = lb_series_consts();
        // one regular pair (the 7-point rule) or a near bit, for panel pj of the chunk
        auto pair = [&](int pj, const R (&qv)[FR_CC], const double (&cc)[4]) {
            if (!is_regular(p0 - cc[0], p1 - cc[1], p2 - cc[2], cc[3])) {
                nmask |= 1u << pj;
                return;
            }
            R f0 = 0, f1 = 0, f2 = 0;
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                const R dx = pr0 - qv[FR_X + q], dy = pr1 - qv[FR_Y + q], dz = pr2 - qv[FR_Z + q];
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R tw = lb_w_r3(qv[FR_W + q], r2, ks);
                f0 += tw * dx;
                f1 += tw * dy;
                f2 += tw * dz;
            }
            const double sg = sig[j0 + pj];
            e0 = fma(sg, (double)f0, e0);
            e1 = fma(sg, (double)f1, e1);
            e2 = fma(sg, (double)f2, e2);
        };
        if (pj0 < pj1) pair(pj0, qf, cf);
        for (int pj = pj0 + 1; pj < pj1; ++pj) {
            const int64_t j = j0 + pj;
            R qv[FR_CC];
            double cc[4];
#pragma unroll
            for (int k = 0; k < FR_CC; ++k) qv[k] = panR[FAR_REC * j + k];
#pragma unroll
            for (int k = 0; k < 4; ++k) cc[k] = pan64[FAR_REC * j + FR_CC + k];
            // the whole record is requested before the classification test and waited for once;
            // left to itself the compiler sinks the node loads below the test, two round trips per panel
            asm volatile("" ::"s"(qv[0]), "s"(qv[8]), "s"(qv[16]), "s"(qv[24]), "s"(qv[FR_CC - 1]), "s"(cc[0]),
                         "s"(cc[3]));
            pair(pj, qv, cc);
        }
    }
    if (SPLIT > 1) {
        wred[wv][lane][0] = e0;
        wred[wv][lane][1] = e1;
        wred[wv][lane][2] = e2;
        wmask[wv][lane] = nmask;
        __syncthreads();
        if (wv != 0 || !live) {
            kclock_stop(kts);
            return;
        }
        e0 = wred[0][lane][0];
        e1 = wred[0][lane][1];
        e2 = wred[0][lane][2];
        nmask = wmask[0][lane];
#pragma unroll
        for (int w = 1; w < SPLIT; ++w) {
            e0 += wred[w][lane][0];
            e1 += wred[w][lane][1];
            e2 += wred[w][lane][2];
            nmask |= wmask[w][lane];
        }
    } else if (!live) {
        kclock_stop(kts);
        return;
    }
    double* o = part + (t * KS + chunk) * 3;
    o[0] = e0;
    o[1] = e1;
    o[2] = e2;
    pmask[t * KS + chunk] = nmask;
    kclock_stop(kts);
}


// Few live lines (the tail of a run, when most lines have stopped): a
// panel-stationary pass.  One lane per panel (256 per block) loads its panel's
// record once and evaluates the regular pairs of all A <= LB_FEW lines; the
// per-line sums are reduced over the block (fixed order), so there are
// ceil(N/256) partial rows instead of one per 32-panel chunk, and the near bits
// come from ballots in the same (line, chunk) mask layout as k_lb_far.
constexpr int LB_FEW = 32;

template <typename R>
__global__ __launch_bounds__(256) void k_lb_far_few(const double* __restrict__ far64, const R* __restrict__ farR,
                                                    int64_t Np, int64_t N, const double* __restrict__ sol, int64_t n,
                                                    const int32_t* __restrict__ line_rhs,
                                                    const int32_t* __restrict__ line_of, int64_t cap,
                                                    const int32_t* __restrict__ count,
                                                    int32_t* __restrict__ count_next, const double* __restrict__ ys,
                                                    double* __restrict__ part, uint32_t* __restrict__ pmask, int64_t KS) {
    __shared__ double lp[LB_FEW][3];
    __shared__ int32_t lrhs[LB_FEW];
    __shared__ double wred[4][LB_FEW][3];
    if (blockIdx.x == 0 && threadIdx.x == 0) count_next[0] = 0;
    if (threadIdx.x < LB_FEW) {   // slot query points, read together with the live count
        const int64_t t = threadIdx.x < cap ? threadIdx.x : cap - 1;
        lp[threadIdx.x][0] = ys[3 * t];
        lp[threadIdx.x][1] = ys[3 * t + 1];
        lp[threadIdx.x][2] = ys[3 * t + 2];
    }
    const int32_t A = count[0] < LB_FEW ? count[0] : LB_FEW;   // the launcher guarantees count <= LB_FEW
    // a slot's line id is valid only below the live count
    if (threadIdx.x < A) lrhs[threadIdx.x] = line_rhs ? line_rhs[line_of[threadIdx.x]] : 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;   // < Np (grid covers N rounded up to 256)
    const bool valid = j < N;
    R qx[7], qy[7], qz[7], qw[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        qx[q] = farR[(int64_t)(FR_X + q) * Np + j];
        qy[q] = farR[(int64_t)(FR_Y + q) * Np + j];
        qz[q] = farR[(int64_t)(FR_Z + q) * Np + j];
        qw[q] = farR[(int64_t)(FR_W + q) * Np + j];
    }
    const double ccx = far64[(int64_t)(FR_CC + 0) * Np + j], ccy = far64[(int64_t)(FR_CC + 1) * Np + j];
    const double ccz = far64[(int64_t)(FR_CC + 2) * Np + j], rr = far64[(int64_t)FR_RR * Np + j];
    const LBSeries ks = lb_series_consts();
    for (int t = 0; t < A; ++t) {
        const double p0 = lp[t][0], p1 = lp[t][1], p2 = lp[t][2];
        const bool reg = valid && is_regular(p0 - ccx, p1 - ccy, p2 - ccz, rr);
        const uint64_t near = __ballot(valid && !reg);
        double e0 = 0.0, e1 = 0.0, e2 = 0.0;
        if (reg) {
            const R pr0 = (R)p0, pr1 = (R)p1, pr2 = (R)p2;
            R f0 = 0, f1 = 0, f2 = 0;
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                const R dx = pr0 - qx[q], dy = pr1 - qy[q], dz = pr2 - qz[q];
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R tw = lb_w_r3(qw[q], r2, ks);
                f0 += tw * dx;
                f1 += tw * dy;
                f2 += tw * dz;
            }
            const double sg = sol[(int64_t)lrhs[t] * n + j];
            e0 = sg * (double)f0;
            e1 = sg * (double)f1;
            e2 = sg * (double)f2;
        }
        // near bits: lanes 0..31 and 32..63 of the wave are two 32-panel chunks
        const int64_t c0 = (j - lane) / LB_C;
        if (lane == 0 && ((j - lane) < N)) pmask[t * KS + c0] = (uint32_t)near;
        if (lane == 32 && ((j - lane + 32) < N)) pmask[t * KS + c0 + 1] = (uint32_t)(near >> 32);
        e0 = wave_sum(e0);
        e1 = wave_sum(e1);
        e2 = wave_sum(e2);
        if (lane == 0) {   // one slot per (wave, line): no barrier inside the line loop
            wred[wv][t][0] = e0;
            wred[wv][t][1] = e1;
            wred[wv][t][2] = e2;
        }
    }
    __syncthreads();
    if (threadIdx.x < 3 * A) {
        const int t = threadIdx.x / 3, c = threadIdx.x % 3;
        part[((int64_t)t * KS + blockIdx.x) * 3 + c] = (wred[0][t][c] + wred[1][t][c]) + (wred[2][t][c] + wred[3][t][c]);
    }
}

constexpr int LB_Q = 1024;    // near pairs per round in k_lb_step
constexpr int LB_MREG = 8;    // near masks per thread held in registers by k_lb_step (KS <= 2048)

// One block per live slot: far partials + the line's near pairs (closed forms, and the
// segment test on end-of-step passes) + the RK4 stage machine.  Everything the block needs
// first (the live count, the slot's state, its partial row and masks) is indexed by the slot
// alone, so those loads go out together; a line that goes on is written whole to the slot it
// draws in the next buffer.
// NODAL: the density is the nodal one (vertex values nu, vertex indices ntri): near
// pairs take the linear-density closed form; otherwise sigma per panel.
template <bool NODAL>
__global__ __launch_bounds__(256) void k_lb_step(
    int64_t N, int64_t KS, int64_t KSP, const int32_t* __restrict__ count, int32_t* __restrict__ count_next,
    const double* __restrict__ part, const uint32_t* __restrict__ pmask, int phase, LBState cur, LBState nxt,
    LBArgs a, const double* __restrict__ tri64, const double* __restrict__ sol, int64_t n,
    const int32_t* __restrict__ line_rhs, const int32_t* __restrict__ tri_body, const int32_t* __restrict__ body_kind,
    int32_t* __restrict__ n_steps, int32_t* __restrict__ stop_code, double* __restrict__ integral,
    uint8_t* __restrict__ exceeds, double* __restrict__ path, int64_t pstride,
    unsigned long long* __restrict__ ncnt, const int32_t* __restrict__ ntri, const double* __restrict__ nu) {
    __shared__ int32_t list[LB_Q];
    __shared__ int32_t scan[4];
    __shared__ double red[4][4];
    __shared__ int32_t redj[4];
    // a latency chain that shares its CUs with the other line group's far pass: its waves issue
    // first, and the far pass's waves fill the cycles it spends waiting
    __builtin_amdgcn_s_setprio(3);
    const int64_t b = blockIdx.x;   // < the group's slot count (the grid is sized by an upper bound)
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    // slot state (a slot past the live count holds stale values that are never used)
    const int64_t l = cur.line[b];
    const double p0 = cur.y[3 * b], p1 = cur.y[3 * b + 1], p2 = cur.y[3 * b + 2];
    const double q0 = cur.x[3 * b], q1 = cur.x[3 * b + 1], q2 = cur.x[3 * b + 2];
    const int32_t ns0 = cur.ns[b];
    const double asum0 = cur.asum[b], I0 = cur.I[b];
    const double ks0 = cur.ks[3 * b], ks1 = cur.ks[3 * b + 1], ks2 = cur.ks[3 * b + 2];
    // far partials (fixed order per thread) and near masks in one sweep of the slot's contiguous
    // row; the first LB_MREG masks of each thread stay in registers for the list fill below
    const double* prow = part + b * KS * 3;
    const uint32_t* mrow = pmask + b * KS;
    double e0 = 0.0, e1 = 0.0, e2 = 0.0;
    uint32_t mreg[LB_MREG];
    int cnt = 0;
    // every load of the sweep is issued before any is used (indices clamped into the row, the
    // clamped values dropped below): left conditional, each would wait for the one before
    double pr[LB_MREG][3];
    const int32_t A = count[0];
#pragma unroll
    for (int t = 0; t < LB_MREG; ++t) {
        const int64_t k = tid + 256 * t;
        const int64_t kp = k < KSP ? k : KSP - 1, km = k < KS ? k : KS - 1;
        pr[t][0] = prow[3 * kp];
        pr[t][1] = prow[3 * kp + 1];
        pr[t][2] = prow[3 * kp + 2];
        mreg[t] = mrow[km];
    }
    // a stage-point pass (phase 1 or 2) never stops a line: its slot in the next pass is drawn
    // now, while the sweep's loads are in flight, rather than after the step
    const bool goes_on = (phase == 1 || phase == 2);
    int32_t sn_early = 0;
    if (goes_on && tid == 0 && b < A) sn_early = atomicAdd(count_next, 1);
#pragma unroll
    for (int t = 0; t < LB_MREG; ++t) {
        const int64_t k = tid + 256 * t;
        if (k < KSP) {
            e0 += pr[t][0];
            e1 += pr[t][1];
            e2 += pr[t][2];
        }
        if (k >= KS) mreg[t] = 0;
        cnt += __popc(mreg[t]);
    }
    for (int64_t k = tid + 256 * LB_MREG; k < KS || k < KSP; k += 256) {
        if (k < KSP) {
            e0 += prow[3 * k];
            e1 += prow[3 * k + 1];
            e2 += prow[3 * k + 2];
        }
        if (k < KS) cnt += __popc(mrow[k]);
    }
    if (b >= A) return;   // uniform over the block
    const double* sigma = sol + (line_rhs ? (int64_t)line_rhs[l] : 0) * n;
    const bool hit_pass = (phase == 4);
    // near pairs: exclusive scan of the per-thread counts over the block (wave scans + one barrier)
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
    if (tid == 0) {   // the line's own pair counters, added without waiting for them
        atomicAdd(ncnt + 2 * l, (unsigned long long)total);
        // every other panel of this line was a regular pair of the chunked far pass (k_lb_far);
        // the panel-stationary few-line pass (KSP != KS) is not counted
        if (KSP == KS) atomicAdd(ncnt + 2 * l + 1, (unsigned long long)(N - total));
    }
    double n0 = 0.0, n1 = 0.0, n2 = 0.0, bt = 2.0;
    int bj = INT_MAX;
    for (int base = 0; base < total; base += LB_Q) {
        __syncthreads();
        // this thread's pairs that fall in [base, base + LB_Q)
        if (off + cnt > base && off < base + LB_Q) {
            int pos = off;
#pragma unroll
            for (int t = 0; t < LB_MREG; ++t) {
                uint32_t m = mreg[t];
                const int64_t k = tid + 256 * t;
                while (m) {
                    const int bb = __builtin_ctz(m);
                    m &= m - 1;
                    if (pos >= base && pos < base + LB_Q) list[pos - base] = (int32_t)(k * LB_C + bb);
                    ++pos;
                }
            }
            for (int64_t k = tid + 256 * LB_MREG; k < KS && pos < base + LB_Q; k += 256) {
                uint32_t m = mrow[k];
                while (m) {
                    const int bb = __builtin_ctz(m);
                    m &= m - 1;
                    if (pos >= base && pos < base + LB_Q) list[pos - base] = (int32_t)(k * LB_C + bb);
                    ++pos;
                }
            }
        }
        __syncthreads();
        const int nq = (total - base) < LB_Q ? (total - base) : LB_Q;
        for (int q = tid; q < nq; q += 256) {
            const int j = list[q];
            const double* Tj = tri64 + (int64_t)TRI_REC * j;
            if constexpr (NODAL) {
                double ph = 0.0;
                nodal_tri_phiE(Tj, p0, p1, p2, nu[ntri[3 * (int64_t)j]], nu[ntri[3 * (int64_t)j + 1]],
                               nu[ntri[3 * (int64_t)j + 2]], ph, n0, n1, n2);
            } else {
                double S, F0, F1, F2;
                flat_tri_SF<false, true>(Tj, p0, p1, p2, false, S, F0, F1, F2);
                const double sg = sigma[j];
                n0 = fma(sg, F0, n0);
                n1 = fma(sg, F1, n1);
                n2 = fma(sg, F2, n2);
            }
            if (hit_pass) {
                const double th = lb_segment_tri(Tj, q0, q1, q2, p0 - q0, p1 - q1, p2 - q2);
                if (th >= 0.0 && (th < bt || (th == bt && j < bj))) {
                    bt = th;
                    bj = j;
                }
            }
        }
    }
    e0 = wave_sum(e0 + n0);
    e1 = wave_sum(e1 + n1);
    e2 = wave_sum(e2 + n2);
    if (hit_pass) {
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
        red[wv][0] = e0;
        red[wv][1] = e1;
        red[wv][2] = e2;
        red[wv][3] = bt;
        redj[wv] = bj;
    }
    __syncthreads();
    if (tid != 0) return;
    const double F0 = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
    const double F1 = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
    const double F2 = (red[0][2] + red[1][2]) + (red[2][2] + red[3][2]);
    int hit = -1;
    if (hit_pass) {
        double tb = 2.0;
        int jb = INT_MAX;
        for (int w = 0; w < 4; ++w)
            if (red[w][3] < tb || (red[w][3] == tb && redj[w] < jb)) {
                tb = red[w][3];
                jb = redj[w];
            }
        hit = (jb != INT_MAX) ? jb : -1;
    }
    const double h = a.h;
    double x0 = q0, x1 = q1, x2 = q2, I = I0;
    int32_t ns = ns0;
    int code = -1;   // -1: the line goes on
    if (hit_pass) {
        if (hit >= 0) {
            const int32_t k = body_kind[tri_body[hit]];
            code = (k == BEM_DIRICHLET) ? BEM_STOP_DIRICHLET
                                        : ((k == BEM_FLOATING) ? BEM_STOP_FLOATING : BEM_STOP_INTERFACE);
        } else {   // the step is accepted: its end point becomes the line's point
            I = I0 + h / 6.0 * asum0;
            x0 = p0;
            x1 = p1;
            x2 = p2;
            ++ns;
            if (path) {
                path[l * pstride + 3 * ns + 0] = x0;
                path[l * pstride + 3 * ns + 1] = x1;
                path[l * pstride + 3 * ns + 2] = x2;
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
            const double c = (phase == 1) ? 0.5 * h : h;
            y0 = x0 + c * d0;
            y1 = x1 + c * d1;
            y2 = x2 + c * d2;
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
    if (code >= 0) {
        n_steps[l] = ns;
        stop_code[l] = code;
        if (integral) integral[l] = I;
        if (exceeds) exceeds[l] = (I > a.k_str) ? 1 : 0;
    } else {
        const int32_t sn = goes_on ? sn_early : atomicAdd(count_next, 1);
        nxt.x[3 * sn] = x0;
        nxt.x[3 * sn + 1] = x1;
        nxt.x[3 * sn + 2] = x2;
        nxt.y[3 * sn] = y0;
        nxt.y[3 * sn + 1] = y1;
        nxt.y[3 * sn + 2] = y2;
        nxt.ks[3 * sn] = k0;
        nxt.ks[3 * sn + 1] = k1;
        nxt.ks[3 * sn + 2] = k2;
        nxt.asum[sn] = asum;
        nxt.I[sn] = I;
        nxt.ns[sn] = ns;
        nxt.line[sn] = (int32_t)l;
    }
}

}  // namespace

namespace {
// Folds group 1's live slots into group 0's (one block): group 0 keeps its n0 slots and takes
// group 1's n1 after them, whole states moved.  The launcher calls it only when n0 + n1 fits
// group 0's slot range [0, lo1), so the destination [n0, n0 + n1) lies below the source
// [lo1, lo1 + n1).
__global__ __launch_bounds__(256) void k_lb_merge(LBState s, int32_t* __restrict__ cnt0, int32_t* __restrict__ cnt1,
                                                  int64_t lo1) {
    const int32_t n0 = cnt0[0], n1 = cnt1[0];
    __syncthreads();   // every thread has read the counts before thread 0 rewrites them
    for (int32_t i = threadIdx.x; i < n1; i += 256) {
        const int64_t d = n0 + i, r = lo1 + i;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            s.x[3 * d + k] = s.x[3 * r + k];
            s.y[3 * d + k] = s.y[3 * r + k];
            s.ks[3 * d + k] = s.ks[3 * r + k];
        }
        s.asum[d] = s.asum[r];
        s.I[d] = s.I[r];
        s.ns[d] = s.ns[r];
        s.line[d] = s.line[r];
    }
    if (threadIdx.x == 0) {
        cnt0[0] = n0 + n1;
        cnt1[0] = 0;
    }
}

// slots [count, S) of a buffer hold no line (line -1)
__global__ __launch_bounds__(256) void k_lb_clear_slots(int32_t* __restrict__ line, const int32_t* __restrict__ count,
                                                        int64_t S) {
    for (int64_t s = (int64_t)count[0] + threadIdx.x; s < S; s += 256) line[s] = -1;
}

__global__ __launch_bounds__(256) void k_lb_zero_u64(int64_t m, unsigned long long* __restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < m) v[i] = 0;
}

__global__ void k_lb_set_count(int32_t* __restrict__ count, int32_t v) {
    if (threadIdx.x == 0) count[0] = v;
}

// the lines' near and far pair counts added to the context's counters (one block, fixed order)
__global__ __launch_bounds__(256) void k_lb_count_sum(int64_t L, const unsigned long long* __restrict__ ncnt,
                                                      unsigned long long* __restrict__ counters) {
    __shared__ unsigned long long red[2][256];
    unsigned long long a = 0, b = 0;
    for (int64_t l = threadIdx.x; l < L; l += 256) {
        a += ncnt[2 * l];
        b += ncnt[2 * l + 1];
    }
    red[0][threadIdx.x] = a;
    red[1][threadIdx.x] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long sa = 0, sb = 0;
        for (int k = 0; k < 256; ++k) {
            sa += red[0][k];
            sb += red[1][k];
        }
        counters[0] += sa;
        counters[1] += sb;
    }
}
}  // namespace

// Duration (ms, best of 3 after a warm-up) of one far-field pass over L lines at the points pts
// (FP64 or FP32 by the context's precision), split, or not with tile_lines lines per block
// (tile_lines = 0: the panel-stationary few-line pass); splitk waves per chunk when split:
// used by the autotuner.
double time_far_pass(bem_ctx* c, int64_t L, bool split, int tile_lines, int splitk, const double* pts,
                     const double* sol) {
    const int64_t Np = (int64_t)(c->far64.bytes / (sizeof(double) * FAR_REC));
    const int64_t N = c->N;
    const int64_t KS = ceil_div(N, LB_C);
    // the points are the query points of slots 0..L-1, all live
    c->lb_state.alloc(sizeof(double) * (size_t)L * 22 + sizeof(int32_t) * ((size_t)L * 4 + 32 * 4));
    c->lb_part.alloc(sizeof(double) * 3 * (size_t)KS * L + sizeof(uint32_t) * (size_t)KS * L);
    int32_t* cnt = reinterpret_cast<int32_t*>(c->lb_state.as<double>() + (size_t)L * 22) + (size_t)L * 4;
    double* part = c->lb_part.as<double>();
    uint32_t* pmask = reinterpret_cast<uint32_t*>(part + 3 * (size_t)KS * L);
    hipLaunchKernelGGL(k_lb_set_count, dim3(1), dim3(64), 0, c->stream, cnt, (int32_t)L);
    BEM_CHECK_LAUNCH();
    const bool fp64 = c->opt.precision == BEM_FP64;
    const int tile = split ? 64 : (tile_lines > 0 ? tile_lines : 256);
    const int32_t ntile = (int32_t)ceil_div(L, tile);
    dim3 g1((unsigned)(ntile * ceil_div(KS, 8) * 8));
    const bool few = !split && tile_lines == 0;
    if (few && L > LB_FEW) throw Error(BEM_ERR_INVALID, "few-line pass timed above its line limit");
    auto run = [&] {
        if (few) {
            if (fp64)
                hipLaunchKernelGGL((k_lb_far_few<double>), dim3((unsigned)(Np / 256)), dim3(256), 0, c->stream,
                                   c->far64.as<double>(), c->far64.as<double>(), Np, N, sol, c->n,
                                   (const int32_t*)nullptr, (const int32_t*)nullptr, L, cnt, cnt + 16, pts, part,
                                   pmask, KS);
            else
                hipLaunchKernelGGL((k_lb_far_few<float>), dim3((unsigned)(Np / 256)), dim3(256), 0, c->stream,
                                   c->far64.as<double>(), c->far32.as<float>(), Np, N, sol, c->n,
                                   (const int32_t*)nullptr, (const int32_t*)nullptr, L, cnt, cnt + 16, pts, part,
                                   pmask, KS);
            BEM_CHECK_LAUNCH();
            return;
        }
#define BEM_LB_FAR(R, SP, TL, FR)                                                                                 \
    hipLaunchKernelGGL((k_lb_far<R, SP, TL>), g1, dim3(SP > 1 ? 64 * SP : TL), 0, c->stream, c->pan64.as<double>(), \
                       FR, N, sol, c->n, (const int32_t*)nullptr, (const int32_t*)nullptr, L, cnt, cnt + 16, pts, \
                       part, pmask, ntile, KS, (unsigned long long*)nullptr)
#define BEM_LB_FAR_ALL(R, FR)                      \
    if (split && splitk == 2)                      \
        BEM_LB_FAR(R, 2, 64, FR);                  \
    else if (split && splitk == 4)                 \
        BEM_LB_FAR(R, 4, 64, FR);                  \
    else if (split)                                \
        BEM_LB_FAR(R, 8, 64, FR);                  \
    else if (tile == 64)                           \
        BEM_LB_FAR(R, 1, 64, FR);                  \
    else if (tile == 128)                          \
        BEM_LB_FAR(R, 1, 128, FR);                 \
    else                                           \
        BEM_LB_FAR(R, 1, 256, FR)
        if (fp64) {
            BEM_LB_FAR_ALL(double, c->pan64.as<double>());
        } else {
            BEM_LB_FAR_ALL(float, c->pan32.as<float>());
        }
#undef BEM_LB_FAR_ALL
#undef BEM_LB_FAR
        BEM_CHECK_LAUNCH();
    };
    hipEvent_t a, b;
    BEM_HIP(hipEventCreate(&a));
    BEM_HIP(hipEventCreate(&b));
    run();
    double best = 1e30;
    for (int rep = 0; rep < 3; ++rep) {
        BEM_HIP(hipEventRecord(a, c->stream));
        run();
        BEM_HIP(hipEventRecord(b, c->stream));
        BEM_HIP(hipEventSynchronize(b));
        float ms = 0.f;
        BEM_HIP(hipEventElapsedTime(&ms, a, b));
        best = std::min(best, (double)ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return best;
}

void launch_trace_batched(bem_ctx* c, int32_t nrhs, const double* sol, int64_t L, const int32_t* line_rhs,
                          const double* starts, const bem_trace_params* tp, int32_t* n_steps, int32_t* stop_code,
                          double* path, double* integral, uint8_t* exceeds, bool fused_tail) {
    if (L == 0) return;
    KTimer t(c, "trace");
    const int64_t Np = (int64_t)(c->far64.bytes / (sizeof(double) * FAR_REC));
    const int64_t N = c->N;
    const int64_t KS = ceil_div(N, LB_C);
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
    // Line groups: two contiguous slot ranges of lines, each with its own counters and its own
    // stream.  A group's pass is its own far launch and step launch, so while one group's step
    // kernel (a short chain of dependent loads over a few hundred blocks) runs, the other group's
    // far pass fills the rest of the GPU.  State, partials and masks are indexed by slot and a
    // group's slots stay in its range, so the groups share the buffers without overlap.  Once the
    // live lines fit one 64-line tile the groups are folded into one (two part-empty tiles would
    // cost twice the blocks of one).
    // (default: two groups from 128 lines, where one group's step kernel has the other's far
    // pass to overlap; measured 194 against 214 ms for 256 lines on the 19,732-panel coax)
    const int32_t G = (int32_t)std::min<int64_t>(c->tune_trace_groups > 0 ? c->tune_trace_groups : (L >= 128 ? 2 : 1), L);
    // two state buffers (x, y, ks: 3 doubles; asum, I: 1 double; ns, line: 1 int32 per slot), two
    // live counters per group, and two pair counters per line
    c->lb_state.alloc(sizeof(double) * (size_t)L * 22 + sizeof(int32_t) * ((size_t)L * 4 + 32 * 4) +
                      sizeof(unsigned long long) * 2 * (size_t)L);
    c->lb_part.alloc(sizeof(double) * 3 * (size_t)KS * L + sizeof(uint32_t) * (size_t)KS * L);
    double* dbase = c->lb_state.as<double>();
    int32_t* ibase = reinterpret_cast<int32_t*>(dbase + (size_t)L * 22);
    LBState buf[2];
    for (int k = 0; k < 2; ++k) {
        double* d = dbase + (size_t)L * 11 * k;
        int32_t* i = ibase + (size_t)L * 2 * k;
        buf[k] = {d, d + 3 * L, d + 6 * L, d + 9 * L, d + 10 * L, i, i + L};
    }
    int32_t* cnt0 = ibase + (size_t)L * 4;
    unsigned long long* ncnt = reinterpret_cast<unsigned long long*>(cnt0 + 32 * 4);
    double* part = c->lb_part.as<double>();
    uint32_t* pmask = reinterpret_cast<uint32_t*>(part + 3 * (size_t)KS * L);
    hipLaunchKernelGGL(k_lb_init, dim3((unsigned)ceil_div(L, 256)), dim3(256), 0, c->stream, L, G, starts, buf[0],
                       cnt0, path, pstride, ncnt);
    BEM_CHECK_LAUNCH();
    struct Group {
        int64_t lo, size, known;   // slot range [lo, lo + size); known: upper bound on the live count
        int32_t* cnt[2];
        hipStream_t st;
    };
    if (G > 1 && !c->aux_stream) {
        BEM_HIP(hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking));
        BEM_HIP(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
        BEM_HIP(hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming));
    }
    Group grp[2];
    for (int32_t g = 0; g < G; ++g) {
        Group& q = grp[g];
        q.lo = g * L / G;
        q.size = (g + 1) * L / G - q.lo;
        q.known = q.size;
        q.cnt[0] = cnt0 + 32 * g;
        q.cnt[1] = cnt0 + 32 * g + 16;
        q.st = (g & 1) ? c->aux_stream : c->stream;
    }
    if (G > 1) {   // the second stream starts after everything enqueued so far (init included)
        BEM_HIP(hipEventRecord(c->fork_ev, c->stream));
        BEM_HIP(hipStreamWaitEvent(c->aux_stream, c->fork_ev, 0));
    }
    // join on every exit (an error thrown by a launch included): later context-stream work sees
    // everything the second stream wrote
    struct Join {
        bem_ctx* c;
        bool on;
        ~Join() {
            if (on && hipEventRecord(c->join_ev, c->aux_stream) == hipSuccess)
                (void)hipStreamWaitEvent(c->stream, c->join_ev, 0);
        }
    } join{c, G > 1};
    // nodal basis (one load case): the far passes read records whose node weights carry the
    // density, with a density of one per panel; the step kernel's near pairs read the vertex values.
    // Those records exist in FP64 only, so nodal lines take the FP64 far passes in either
    // precision (the FP32 records and the few-line FP32 pass are laid out for the constant basis)
    const bool nodal = c->opt.basis == BEM_BASIS_LINEAR;
    const bool fp64 = c->opt.precision == BEM_FP64 || nodal;
    if (nodal) launch_nodal_records(c, sol);
    const double* P64 = nodal ? c->nod_pan64.as<double>() : c->pan64.as<double>();
    const double* F64 = nodal ? c->nod_far64.as<double>() : c->far64.as<double>();
    const double* fsol = nodal ? c->nod_ones.as<double>() : sol;
    const int64_t fn = nodal ? 0 : c->n;
    const int64_t max_pass = 4 * (int64_t)tp->max_steps + 1;
    kclock_begin(c, (max_pass + 2) * (G + 1));
    int cur = 0;
    int32_t* host = c->host_stage.as<int32_t>();
    // pending count copies: checkpoint parity x group (host slots 8 + 2 parity + group)
    for (int k = 0; k < 4; ++k)
        if (!c->lb_ev[k]) BEM_HIP(hipEventCreateWithFlags(&c->lb_ev[k], hipEventDisableTiming));
    bool pend[2][2] = {{false, false}, {false, false}};
    int ck = 0;
    // wait for the copies in flight and drop their counts; also on every exit, an error thrown
    // by a launch included (the staging slots are the context's: no copy may land after this call)
    auto settle = [&]() {
        for (int k = 0; k < 2; ++k)
            for (int g = 0; g < 2; ++g)
                if (pend[k][g]) {
                    BEM_HIP(hipEventSynchronize(c->lb_ev[2 * k + g]));
                    pend[k][g] = false;
                }
    };
    struct Settle {
        bem_ctx* c;
        bool (*pend)[2];
        ~Settle() {
            for (int k = 0; k < 2; ++k)
                for (int g = 0; g < 2; ++g)
                    if (pend[k][g]) (void)hipEventSynchronize(c->lb_ev[2 * k + g]);
        }
    } settle_on_exit{c, pend};
    for (int64_t pass = 0; pass < max_pass; ++pass) {
        const int phase = pass == 0 ? 0 : (int)((pass - 1) % 4) + 1;
        // Profiling: the far pass is timed at every launch by events carried in its dispatch
        // (hipExtLaunchKernelGGL), which add no work to the stream; the step kernel (profiling
        // mode 1) by event pairs around every 16th pass, which would otherwise cost more than the
        // short launches.  With two live groups a pass timed in mode 1 runs its launches one
        // after another, so the timed launches measure each kernel alone rather than its overlap
        // with the other group.
        const bool timed = (pass & 15) == 0;
        const bool serial = c->profiling == 1 && timed && G > 1 && grp[0].known > 0 && grp[1].known > 0;
        for (int32_t g = 0; g < G; ++g) {
            Group& q = grp[g];
            if (q.known == 0) continue;
            if (serial) {   // wait for everything enqueued on the other stream
                BEM_HIP(hipEventRecord(c->fork_ev, grp[g ^ 1].st));
                BEM_HIP(hipStreamWaitEvent(q.st, c->fork_ev, 0));
            }
            const LBState sc = lb_shift(buf[cur], q.lo), sn = lb_shift(buf[cur ^ 1], q.lo);
            double* gpart = part + 3 * q.lo * KS;
            uint32_t* gmask = pmask + q.lo * KS;
            const bool few = q.known <= std::min<int64_t>(c->tune_trace_few, LB_FEW);
            const bool split = q.known <= c->tune_trace_split;
            int64_t KSP = KS;   // partial rows the step kernel sums
            {
            // timing of a chunked far pass: events carried in its dispatch (profiling mode 1), or the
            // kernel's own clock stamps (mode 2; events would also count the wait for the other
            // line group's kernel)
            hipEvent_t fa = nullptr, fb = nullptr;
            const bool tfar = c->profiling == 1 && !few;
            if (tfar) timing_events(c, &fa, &fb);
            unsigned long long* kts = few ? nullptr : kclock_slot(c, "trace_far");
            // blocks of tiles past the live count would only launch and exit: size the grids by
            // the last known live count (an upper bound, the count only falls)
            const int tile = split ? 64 : c->tune_trace_tile;
            const int splitk = c->tune_trace_splitk;
            const int32_t ntile = (int32_t)ceil_div(q.known, tile);
            dim3 g1((unsigned)(ntile * ceil_div(KS, 8) * 8));
#define BEM_LB_FAR(R, SP, TL, FR)                                                                              \
    hipExtLaunchKernelGGL((k_lb_far<R, SP, TL>), g1, dim3(SP > 1 ? 64 * SP : TL), 0, q.st, fa, fb, 0, P64, FR, N, \
                          fsol, fn, line_rhs, sc.line, q.size, q.cnt[cur], q.cnt[cur ^ 1], sc.y, gpart, gmask,     \
                          ntile, KS, kts)
#define BEM_LB_FAR_ALL(R, FR)                      \
    if (split && splitk == 2)                      \
        BEM_LB_FAR(R, 2, 64, FR);                  \
    else if (split && splitk == 4)                 \
        BEM_LB_FAR(R, 4, 64, FR);                  \
    else if (split)                                \
        BEM_LB_FAR(R, 8, 64, FR);                  \
    else if (tile == 64)                           \
        BEM_LB_FAR(R, 1, 64, FR);                  \
    else if (tile == 128)                          \
        BEM_LB_FAR(R, 1, 128, FR);                 \
    else                                           \
        BEM_LB_FAR(R, 1, 256, FR)
            if (few) {
                KSP = Np / 256;
                if (fp64)
                    hipLaunchKernelGGL((k_lb_far_few<double>), dim3((unsigned)KSP), dim3(256), 0, q.st, F64, F64, Np,
                                       N, fsol, fn, line_rhs, sc.line, q.size, q.cnt[cur], q.cnt[cur ^ 1], sc.y,
                                       gpart, gmask, KS);
                else
                    hipLaunchKernelGGL((k_lb_far_few<float>), dim3((unsigned)KSP), dim3(256), 0, q.st,
                                       c->far64.as<double>(), c->far32.as<float>(), Np, N, sol, c->n, line_rhs,
                                       sc.line, q.size, q.cnt[cur], q.cnt[cur ^ 1], sc.y, gpart, gmask, KS);
            } else if (fp64) {
                BEM_LB_FAR_ALL(double, P64);
            } else {
                BEM_LB_FAR_ALL(float, c->pan32.as<float>());
            }
#undef BEM_LB_FAR_ALL
#undef BEM_LB_FAR
            BEM_CHECK_LAUNCH();
            if (tfar) push_timing(c, "trace_far", fa, fb);
            if (!few) ++c->trace_far_launches;
            }
            {
            KTimer ts(c, "trace_step", timed, q.st);
            if (nodal)
                hipLaunchKernelGGL(k_lb_step<true>, dim3((unsigned)q.known), dim3(256), 0, q.st, N, KS, KSP,
                                   q.cnt[cur], q.cnt[cur ^ 1], gpart, gmask, phase, sc, sn, a, c->tri64.as<double>(),
                                   sol, c->n, line_rhs, c->tri_body.as<int32_t>(), c->body_kind.as<int32_t>(), n_steps,
                                   stop_code, integral, exceeds, path, pstride, ncnt, c->tri.as<int32_t>(), sol);
            else
                hipLaunchKernelGGL(k_lb_step<false>, dim3((unsigned)q.known), dim3(256), 0, q.st, N, KS, KSP,
                                   q.cnt[cur], q.cnt[cur ^ 1], gpart, gmask, phase, sc, sn, a, c->tri64.as<double>(),
                                   sol, c->n, line_rhs, c->tri_body.as<int32_t>(), c->body_kind.as<int32_t>(), n_steps,
                                   stop_code, integral, exceeds, path, pstride, ncnt, (const int32_t*)nullptr,
                                   (const double*)nullptr);
            BEM_CHECK_LAUNCH();
            }
        }
        cur ^= 1;
        if ((pass & 31) == 31 || pass == max_pass - 1) {
            // Live counts every 32 passes.  Those of this checkpoint are copied without waiting, and
            // those of the checkpoint before (32 passes back, normally arrived) are taken, so the
            // GPU never waits for the host; a count only falls, so an older one is an upper bound,
            // and the kernels read the exact counts on the device.  The last pass reads its own.
            int64_t live = 0;
            const bool last = pass == max_pass - 1;
            if (last) {
                for (int32_t g = 0; g < G; ++g)
                    if (grp[g].known > 0)
                        BEM_HIP(hipMemcpyAsync(host + g, grp[g].cnt[cur], sizeof(int32_t), hipMemcpyDeviceToHost,
                                               grp[g].st));
                for (int32_t g = 0; g < G; ++g)
                    if (grp[g].known > 0) {
                        BEM_HIP(hipStreamSynchronize(grp[g].st));
                        grp[g].known = host[g];
                    }
            } else {
                for (int32_t g = 0; g < G; ++g)
                    if (grp[g].known > 0) {
                        BEM_HIP(hipMemcpyAsync(host + 8 + 2 * ck + g, grp[g].cnt[cur], sizeof(int32_t),
                                               hipMemcpyDeviceToHost, grp[g].st));
                        BEM_HIP(hipEventRecord(c->lb_ev[2 * ck + g], grp[g].st));
                        pend[ck][g] = true;
                    }
                ck ^= 1;
                for (int32_t g = 0; g < G; ++g)
                    if (pend[ck][g]) {
                        BEM_HIP(hipEventSynchronize(c->lb_ev[2 * ck + g]));
                        grp[g].known = std::min<int64_t>(grp[g].known, host[8 + 2 * ck + g]);
                        pend[ck][g] = false;
                    }
            }
            for (int32_t g = 0; g < G; ++g) live += grp[g].known;
            if (live == 0) break;
            // fold group 1 into group 0 once all live lines fit one tile and group 0's slot range
            // (the merge on group 0's stream after everything enqueued on group 1's; counts copied
            // before it no longer describe the groups)
            if (G > 1 && c->tune_trace_fold && grp[1].known > 0 && live <= std::min<int64_t>(64, grp[1].lo)) {
                BEM_HIP(hipEventRecord(c->fork_ev, grp[1].st));
                BEM_HIP(hipStreamWaitEvent(grp[0].st, c->fork_ev, 0));
                hipLaunchKernelGGL(k_lb_merge, dim3(1), dim3(256), 0, grp[0].st, buf[cur], grp[0].cnt[cur],
                                   grp[1].cnt[cur], grp[1].lo);
                BEM_CHECK_LAUNCH();
                grp[0].known = live;
                grp[1].known = 0;
                settle();
            }
            // the last few lines (all in group 0's slots [0, live)) go on one launch per stage,
            // from the next pass, with their own pair counters
            if (fused_tail && live <= c->tune_trace_tail && (G == 1 || grp[1].known == 0)) {
                settle();
                if (G > 1) {   // group 1's stream may still hold its last (empty) passes
                    BEM_HIP(hipEventRecord(c->fork_ev, grp[1].st));
                    BEM_HIP(hipStreamWaitEvent(c->stream, c->fork_ev, 0));
                }
                // live is an upper bound: slots from the device's live count on hold no line
                hipLaunchKernelGGL(k_lb_clear_slots, dim3(1), dim3(256), 0, c->stream, buf[cur].line, grp[0].cnt[cur],
                                   live);
                BEM_CHECK_LAUNCH();
                c->lf_cnt.alloc(sizeof(unsigned long long) * 2 * (size_t)L);
                unsigned long long* fcnt = c->lf_cnt.as<unsigned long long>();
                hipLaunchKernelGGL(k_lb_zero_u64, dim3((unsigned)ceil_div(2 * L, 256)), dim3(256), 0, c->stream,
                                   2 * L, fcnt);
                BEM_CHECK_LAUNCH();
                fused_trace_loop(c, sol, L, line_rhs, tp, n_steps, stop_code, path, integral, exceeds, buf[cur],
                                 buf[cur ^ 1], live, pass + 1, fcnt);
                hipLaunchKernelGGL(k_lb_count_sum, dim3(1), dim3(256), 0, c->stream, L, fcnt,
                                   reinterpret_cast<unsigned long long*>(c->counters.p) + 2);
                BEM_CHECK_LAUNCH();
                break;
            }
        }
    }
    settle();   // the staging slots are the context's: no copy may land after this call
    if (G > 1) {   // the counts below need both groups' step kernels
        BEM_HIP(hipEventRecord(c->join_ev, c->aux_stream));
        BEM_HIP(hipStreamWaitEvent(c->stream, c->join_ev, 0));
    }
    hipLaunchKernelGGL(k_lb_count_sum, dim3(1), dim3(256), 0, c->stream, L, ncnt,
                       reinterpret_cast<unsigned long long*>(c->counters.p));
    BEM_CHECK_LAUNCH();
    kclock_end(c);
}

namespace {
__global__ __launch_bounds__(256) void k_gather_starts(int64_t m, const int32_t* __restrict__ idx,
                                                       const double* __restrict__ starts, double* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= m) return;
    const int64_t l = idx[t];
    out[3 * t] = starts[3 * l];
    out[3 * t + 1] = starts[3 * l + 1];
    out[3 * t + 2] = starts[3 * l + 2];
}

// one lane per gathered line: its results back to the caller's slot l = idx[t]; a path copies
// only x_0 .. x_{n_steps}, so the caller's later slots stay untouched
__global__ __launch_bounds__(256) void k_scatter_lines(int64_t m, const int32_t* __restrict__ idx,
                                                       const int32_t* __restrict__ ns, const int32_t* __restrict__ st,
                                                       const double* __restrict__ I, const uint8_t* __restrict__ ex,
                                                       const double* __restrict__ tpath, int64_t pstride,
                                                       int32_t* __restrict__ n_steps, int32_t* __restrict__ stop_code,
                                                       double* __restrict__ integral, uint8_t* __restrict__ exceeds,
                                                       double* __restrict__ path) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= m) return;
    const int64_t l = idx[t];
    n_steps[l] = ns[t];
    stop_code[l] = st[t];
    if (integral) integral[l] = I[t];
    if (exceeds) exceeds[l] = ex[t];
    if (path)
        for (int64_t k = 0; k < 3 * ((int64_t)ns[t] + 1); ++k) path[l * pstride + k] = tpath[t * pstride + k];
}
}  // namespace

// Nodal basis with several load cases: the far passes read panel records built for one
// density, so the lines run case by case (gathered, traced as one load case, scattered back).
void launch_trace_nodal_cases(bem_ctx* c, int32_t nrhs, const double* sol, int64_t L, const int32_t* line_rhs,
                              const double* starts, const bem_trace_params* tp, int32_t* n_steps, int32_t* stop_code,
                              double* path, double* integral, uint8_t* exceeds) {
    std::vector<int32_t> h((size_t)L);
    BEM_HIP(hipMemcpyAsync(h.data(), line_rhs, sizeof(int32_t) * (size_t)L, hipMemcpyDeviceToHost, c->stream));
    BEM_HIP(hipStreamSynchronize(c->stream));
    const int64_t pstride = 3 * ((int64_t)tp->max_steps + 1);
    for (int32_t r = 0; r < nrhs; ++r) {
        std::vector<int32_t> idx;
        for (int64_t l = 0; l < L; ++l)
            if (h[l] == r) idx.push_back((int32_t)l);
        const int64_t m = (int64_t)idx.size();
        if (m == 0) continue;
        // staging: indices, starts, and the per-line outputs of this case
        const size_t bytes = sizeof(int32_t) * m + sizeof(double) * 3 * m + sizeof(int32_t) * 2 * m +
                             sizeof(double) * m + m + (path ? sizeof(double) * (size_t)(pstride * m) : 0) + 64;
        c->tr_cases.alloc(bytes);
        char* base = static_cast<char*>(c->tr_cases.p);
        double* tst = reinterpret_cast<double*>(base);
        double* tI = tst + 3 * m;
        double* tpath = tI + m;
        int32_t* didx = reinterpret_cast<int32_t*>(tpath + (path ? pstride * m : 0));
        int32_t* tns = didx + m;
        int32_t* tsc = tns + m;
        uint8_t* tex = reinterpret_cast<uint8_t*>(tsc + m);
        BEM_HIP(hipMemcpyAsync(didx, idx.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, c->stream));
        hipLaunchKernelGGL(k_gather_starts, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, c->stream, m, didx, starts,
                           tst);
        BEM_CHECK_LAUNCH();
        if (trace_fused_layout(c))
            launch_trace_fused(c, 1, sol + (int64_t)r * c->n, m, nullptr, tst, tp, tns, tsc, path ? tpath : nullptr,
                               integral ? tI : nullptr, exceeds ? tex : nullptr);
        else
            launch_trace_batched(c, 1, sol + (int64_t)r * c->n, m, nullptr, tst, tp, tns, tsc,
                                 path ? tpath : nullptr, integral ? tI : nullptr, exceeds ? tex : nullptr,
                                 trace_fused_tail(c));
        hipLaunchKernelGGL(k_scatter_lines, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, c->stream, m, didx, tns,
                           tsc, tI, tex, tpath, pstride, n_steps, stop_code, integral, exceeds, path);
        BEM_CHECK_LAUNCH();
        BEM_HIP(hipStreamSynchronize(c->stream));   // idx (host) and the staging buffer are reused
    }
}

}  // namespace bem
