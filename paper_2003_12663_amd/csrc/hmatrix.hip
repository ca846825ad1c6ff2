// Compression of the collocation operator (the outlook of Sec. 6: hierarchical
// matrices to escape the quadratic cost of assembly, storage and the Krylov
// products).  The panel-panel block A[0..N)[0..N) becomes a hierarchical matrix:
//   * a cluster tree of the panels by geometric bisection (the longer axis of the
//     centroids' bounding box, split at the median) down to leaves of <= leaf panels;
//   * a block tree of cluster pairs: a pair is admissible when the smaller of the two
//     boxes' diameters is at most eta_adm times the distance between the boxes (boxes of
//     the panels' vertices); admissible pairs are stored in low rank, U V^T, the other
//     pairs are split until both clusters are leaves and then stored dense;
//   * low-rank factors by adaptive cross approximation with partial pivoting: a row and a
//     column of the residual at a time, stopping once the newest cross is below eps times
//     the Frobenius estimate of the approximation and sampled rows and columns of the
//     residual agree (rows that vanish, as coplanar interface rows do, are skipped).
// Every entry comes from the assembly's own rule (Sec. 4 classification, the 7-point
// rule on regular pairs, the closed forms otherwise; interface rows scaled as in Eq.
// Final3), computed on demand: nothing of size N^2 is formed.  The floating bodies'
// potential columns (-1) and constraint rows (Eq. Final4 / sheets / net charge) stay
// dense.  FP64, CONSTANT basis.
//
// Kernels: k_hm_dense (dense leaf blocks, one lane per entry); k_hm_aca (one workgroup
// per admissible block; the residual row and column are spread over its 256 threads,
// pivots and norms by block reductions in a fixed order); k_hm_compact (the factors
// copied from the rank bound into their final, exact-rank storage); the product:
// k_hm_gather (x into cluster order), k_hm_vt (t_b = V_b^T x, one wave per rank index),
// k_hm_rows (one workgroup per leaf of rows: the dense blocks and U_b t_b of every block
// over the leaf, in block order, then the result scattered back), k_hm_constraint_rows.
#include <algorithm>
#include <cmath>
#include <memory>
#include <numeric>
#include <string>
#include <vector>

#include "bem_device.h"

namespace bem {

namespace {

constexpr int HM_KMAX = 64;   // rank bound of a low-rank block (a block that needs more is stored dense)

struct HmEntryArgs {
    const double* tri64;
    const double* pan64;
    const int32_t* perm;       // cluster order -> panel
    const int32_t* tri_body;
    const int32_t* body_kind;  // device kinds (sheets as floating)
    const double* epsp;
    const double* epsm;
};

// Entry (i, j) of the panel-panel block of the system (Eqs. Final1-Final3), i and j panels:
// potential rows S_ij, interface rows (eps+ - eps-) n_i . F_ij with 1/2 (eps+ + eps-) on the
// diagonal; regular pairs by the 7-point rule, the others by the closed forms (self: principal value).
__device__ double hm_entry(const HmEntryArgs& a, int64_t i, int64_t j) {
    const double* Ti = a.tri64 + (int64_t)TRI_REC * i;
    const double x0 = Ti[TR_C], x1 = Ti[TR_C + 1], x2 = Ti[TR_C + 2];
    const int32_t b = a.tri_body[i];
    const bool iface = a.body_kind[b] == BEM_INTERFACE;
    const double* P = a.pan64 + (int64_t)FAR_REC * j;
    const bool self = i == j;
    if (!self && is_regular(x0 - P[FR_CC], x1 - P[FR_CC + 1], x2 - P[FR_CC + 2], P[FR_RR])) {
        if (!iface) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                const double dx = x0 - P[FR_X + q], dy = x1 - P[FR_Y + q], dz = x2 - P[FR_Z + q];
                s += P[FR_W + q] * rsqrt_pos(dx * dx + dy * dy + dz * dz);
            }
            return s;
        }
        double f0 = 0.0, f1 = 0.0, f2 = 0.0;
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            const double dx = x0 - P[FR_X + q], dy = x1 - P[FR_Y + q], dz = x2 - P[FR_Z + q];
            const double ir = rsqrt_pos(dx * dx + dy * dy + dz * dz);
            const double t = P[FR_W + q] * ir * ir * ir;
            f0 += t * dx;
            f1 += t * dy;
            f2 += t * dz;
        }
        return (Ti[TR_N] * f0 + Ti[TR_N + 1] * f1 + Ti[TR_N + 2] * f2) * (a.epsp[b] - a.epsm[b]);
    }
    double S, F0, F1, F2;
    flat_tri_SF<true, true>(a.tri64 + (int64_t)TRI_REC * j, x0, x1, x2, self, S, F0, F1, F2);
    if (!iface) return S;
    if (self) return 0.5 * (a.epsp[b] + a.epsm[b]);
    return (a.epsp[b] - a.epsm[b]) * (Ti[TR_N] * F0 + Ti[TR_N + 1] * F1 + Ti[TR_N + 2] * F2);
}

// K'_ij = n_i . F_ij (the normal-derivative kernel of Eq. ADL) for a floating body's row i
__device__ double hm_kprime(const HmEntryArgs& a, int64_t i, int64_t j) {
    if (i == j) return 0.0;   // flat panel: no normal field of its own density at its centroid
    const double* Ti = a.tri64 + (int64_t)TRI_REC * i;
    const double x0 = Ti[TR_C], x1 = Ti[TR_C + 1], x2 = Ti[TR_C + 2];
    const double* P = a.pan64 + (int64_t)FAR_REC * j;
    if (is_regular(x0 - P[FR_CC], x1 - P[FR_CC + 1], x2 - P[FR_CC + 2], P[FR_RR])) {
        double f0 = 0.0, f1 = 0.0, f2 = 0.0;
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            const double dx = x0 - P[FR_X + q], dy = x1 - P[FR_Y + q], dz = x2 - P[FR_Z + q];
            const double ir = rsqrt_pos(dx * dx + dy * dy + dz * dz);
            const double t = P[FR_W + q] * ir * ir * ir;
            f0 += t * dx;
            f1 += t * dy;
            f2 += t * dz;
        }
        return Ti[TR_N] * f0 + Ti[TR_N + 1] * f1 + Ti[TR_N + 2] * f2;
    }
    double S, F0, F1, F2;
    flat_tri_SF<false, true>(a.tri64 + (int64_t)TRI_REC * j, x0, x1, x2, false, S, F0, F1, F2);
    return Ti[TR_N] * F0 + Ti[TR_N + 1] * F1 + Ti[TR_N + 2] * F2;
}

// Dense blocks, column-major D[j * m + i] (rows i < m of cluster-order range rs, columns j < nn
// from cs): one lane per entry; the blocks' entries are numbered consecutively (off = doff[b]).
__global__ __launch_bounds__(256) void k_hm_dense(HmEntryArgs a, int64_t total, int32_t nblk,
                                                  const int64_t* __restrict__ doff, const int32_t* __restrict__ rs,
                                                  const int32_t* __restrict__ m, const int32_t* __restrict__ cs,
                                                  const int32_t* __restrict__ nn, const int32_t* __restrict__ dlist,
                                                  double* __restrict__ D) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= total) return;
    // the dense block holding entry e: binary search of the offsets (dlist in offset order)
    int32_t lo = 0, hi = nblk - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (doff[dlist[mid]] <= e) lo = mid; else hi = mid - 1;
    }
    const int32_t b = dlist[lo];
    const int64_t k = e - doff[b];
    const int64_t i = k % m[b], j = k / m[b];
    D[e] = hm_entry(a, a.perm[rs[b] + i], a.perm[cs[b] + j]);
}

__device__ __forceinline__ double block_sum(double v, double* red) {   // 256 threads, fixed order
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// block argmax of |v| (ties: lowest index); returns the index, the value in *val
__device__ __forceinline__ int64_t block_argmax(double v, int64_t idx, double* redv, int64_t* redi, double* val) {
    double av = fabs(v);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(av, o, 64);
        const int64_t oi = __shfl_xor(idx, o, 64);
        const double vv = __shfl_xor(v, o, 64);
        if (ov > av || (ov == av && oi < idx)) {
            av = ov;
            idx = oi;
            v = vv;
        }
    }
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        redv[threadIdx.x >> 6] = av;
        redv[4 + (threadIdx.x >> 6)] = v;
        redi[threadIdx.x >> 6] = idx;
    }
    __syncthreads();
    double best = redv[0], bv = redv[4];
    int64_t bi = redi[0];
    for (int w = 1; w < 4; ++w)
        if (redv[w] > best || (redv[w] == best && redi[w] < bi)) {
            best = redv[w];
            bv = redv[4 + w];
            bi = redi[w];
        }
    *val = bv;
    return bi;
}

__device__ __forceinline__ double block_max(double v, double* red) {   // 256 threads
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Sample q < n of stratum s of a range of length len split into n strata, pass `round` (0: the
// strata's midpoints, later passes: hashed offsets inside each stratum).
__device__ __forceinline__ int64_t hm_sample(int64_t len, int n, int s, int round) {
    const int64_t w = len / n;
    if (round == 0) return s * w + w / 2;
    const uint32_t h = (uint32_t)round * 2654435761u + (uint32_t)s * 40503u;
    return s * w + (int64_t)(h % (uint32_t)w);
}

constexpr int HM_NCHK = 4;               // rows and columns sampled by each residual check
constexpr int HM_VISIT = 2 * HM_KMAX;    // rows a block may visit (pivots and vanishing rows)

// Adaptive cross approximation of low-rank block b (one workgroup): U (m x HM_KMAX, column k at
// U + k m) and V (nn x HM_KMAX) in the block's scratch; rank[b] = the rank reached, or -1 if the
// bound was reached first (the block is then stored dense).
//   Partial pivoting alone can stop early or anchor a cross on rounding noise when whole rows of
// a block vanish, as the interface rows of one flat face do against panels in the same plane
// (n . (x - y) = 0).  So: the first pivot row is the largest of a few sampled rows and columns,
// whose largest entry also sets the block's scale; a residual row below 1e-13 of that scale
// (or 0.01 eps of it) is skipped rather than taken as a pivot; and the usual stopping test
// (newest cross below eps times the Frobenius estimate) only ends the approximation once the
// residuals of HM_NCHK more sampled rows and columns, extrapolated to the block, pass it too;
// otherwise the worst of them supplies the next pivot row.
__global__ __launch_bounds__(256) void k_hm_aca(HmEntryArgs a, const int32_t* __restrict__ llist,
                                                const int32_t* __restrict__ rs, const int32_t* __restrict__ m,
                                                const int32_t* __restrict__ cs, const int32_t* __restrict__ nn,
                                                const int64_t* __restrict__ soff, double* __restrict__ scratch,
                                                double eps, int32_t* __restrict__ rank) {
    __shared__ double redv[8];
    __shared__ int64_t redi[4];
    __shared__ double red[4];
    __shared__ int32_t used[HM_VISIT];
    const int32_t b = llist[blockIdx.x];
    const int64_t M = m[b], Nn = nn[b], r0 = rs[b], c0 = cs[b];
    double* U = scratch + soff[b];
    double* V = U + (int64_t)HM_KMAX * M;
    const int tid = threadIdx.x;
    const int nr = (int)(M < HM_NCHK ? M : HM_NCHK), nc = (int)(Nn < HM_NCHK ? Nn : HM_NCHK);
    double dummy;

    // residual row i (local) at column j, residual column j at row i, with k crosses
    auto res_row = [&](int64_t i, int64_t pi, int64_t j, int k) {
        double v = hm_entry(a, pi, a.perm[c0 + j]);
        for (int q = 0; q < k; ++q) v -= U[(int64_t)q * M + i] * V[(int64_t)q * Nn + j];
        return v;
    };
    auto res_col = [&](int64_t j, int64_t pj, int64_t i, int k) {
        double u = hm_entry(a, a.perm[r0 + i], pj);
        for (int q = 0; q < k; ++q) u -= U[(int64_t)q * M + i] * V[(int64_t)q * Nn + j];
        return u;
    };
    // HM_NCHK sampled rows and columns of the residual: the extrapolated squared Frobenius norm
    // (the larger of the rows' and the columns' estimates), the largest entry, and the row to
    // pivot on next (the worst sampled row, or the largest entry's row of the worst column)
    auto check = [&](int k, int round, double* est, double* amx) {
        double er = 0.0, ec = 0.0, mx = 0.0, wr = -1.0, wc = -1.0;
        int64_t rowr = 0, rowc = 0;
        for (int s = 0; s < nr; ++s) {
            const int64_t i = hm_sample(M, nr, s, round), pi = a.perm[r0 + i];
            double ss = 0.0, sm = 0.0;
            for (int64_t j = tid; j < Nn; j += 256) {
                const double v = res_row(i, pi, j, k);
                ss += v * v;
                sm = fmax(sm, fabs(v));
            }
            ss = block_sum(ss, red);
            mx = fmax(mx, block_max(sm, red));
            er += ss;
            if (ss > wr) {
                wr = ss;
                rowr = i;
            }
        }
        for (int s = 0; s < nc; ++s) {
            const int64_t j = hm_sample(Nn, nc, s, round), pj = a.perm[c0 + j];
            double ss = 0.0, bu = -1.0, buv = 0.0;
            int64_t bi = 0;
            for (int64_t i = tid; i < M; i += 256) {
                const double u = res_col(j, pj, i, k);
                ss += u * u;
                if (fabs(u) > bu) {
                    bu = fabs(u);
                    buv = u;
                    bi = i;
                }
            }
            ss = block_sum(ss, red);
            double pv;
            const int64_t ib = block_argmax(bu >= 0.0 ? buv : 0.0, bu >= 0.0 ? bi : INT64_MAX, redv, redi, &pv);
            mx = fmax(mx, fabs(pv));
            ec += ss;
            if (ss > wc) {
                wc = ss;
                rowc = ib;
            }
        }
        *est = fmax(er * (double)M / nr, ec * (double)Nn / nc);
        *amx = mx;
        // compare per-entry means so that rows and columns of different lengths weigh alike
        return wr / (double)Nn >= wc / (double)M ? rowr : rowc;
    };

    double est, amax;
    int64_t ir = check(0, 0, &est, &amax);          // the block's scale and its first pivot row
    int round = 1;
    if (amax == 0.0) ir = check(0, round++, &est, &amax);
    const double zrel = fmin(1e-13, 0.01 * eps);
    double zthr = zrel * amax;
    double fro2 = 0.0;
    int k = 0, nvis = 0;
    int result = -1;
    if (amax == 0.0) result = 0;                    // every sampled entry is zero: nothing to capture
    while (result < 0 && k < HM_KMAX && nvis < HM_VISIT) {
        if (tid == 0) used[nvis] = (int32_t)ir;
        ++nvis;
        // residual row ir: V[:, k]
        double best = -1.0, bestv = 0.0;
        int64_t bj = 0;
        const int64_t pi = a.perm[r0 + ir];
        for (int64_t j = tid; j < Nn; j += 256) {
            const double v = res_row(ir, pi, j, k);
            V[(int64_t)k * Nn + j] = v;
            if (fabs(v) > best) {
                best = fabs(v);
                bestv = v;
                bj = j;
            }
        }
        double piv;
        const int64_t jr = block_argmax(best >= 0.0 ? bestv : 0.0, best >= 0.0 ? bj : INT64_MAX, redv, redi, &piv);
        bool test = true;
        if (fabs(piv) > zthr) {
            const double ip = 1.0 / piv;
            __syncthreads();   // every thread's V[:, k] written before the scaling reads them
            for (int64_t j = tid; j < Nn; j += 256) V[(int64_t)k * Nn + j] *= ip;
            // residual column jr: U[:, k]; the next pivot row: its largest unvisited entry
            const int64_t pj = a.perm[c0 + jr];
            double nu = 0.0, bu = -1.0, buv = 0.0;
            int64_t bi = 0;
            __syncthreads();
            for (int64_t i = tid; i < M; i += 256) {
                const double u = res_col(jr, pj, i, k);
                U[(int64_t)k * M + i] = u;
                nu += u * u;
                bool was = false;
                for (int q = 0; q < nvis; ++q) was = was || (used[q] == i);
                if (!was && fabs(u) > bu) {
                    bu = fabs(u);
                    buv = u;
                    bi = i;
                }
            }
            __syncthreads();
            // norms of the new cross and its products with the earlier ones (Frobenius estimate)
            nu = block_sum(nu, red);
            double nv = 0.0;
            for (int64_t j = tid; j < Nn; j += 256) nv += V[(int64_t)k * Nn + j] * V[(int64_t)k * Nn + j];
            nv = block_sum(nv, red);
            double cross = 0.0;
            for (int q = 0; q < k; ++q) {
                double du = 0.0, dv = 0.0;
                for (int64_t i = tid; i < M; i += 256) du += U[(int64_t)q * M + i] * U[(int64_t)k * M + i];
                for (int64_t j = tid; j < Nn; j += 256) dv += V[(int64_t)q * Nn + j] * V[(int64_t)k * Nn + j];
                du = block_sum(du, red);
                dv = block_sum(dv, red);
                cross += du * dv;
            }
            fro2 += nu * nv + 2.0 * cross;
            const int64_t inext = block_argmax(bu >= 0.0 ? buv : 0.0, bu >= 0.0 ? bi : INT64_MAX, redv, redi, &dummy);
            ++k;
            if (inext == INT64_MAX) {   // every row visited: the block is captured
                result = k;
                break;
            }
            amax = fmax(amax, fabs(piv));
            zthr = zrel * amax;
            test = nu * nv <= eps * eps * fro2;
            if (!test) ir = inext;
        }
        if (test) {   // the cross is small, or the row vanished: sample the residual
            double mx;
            const int64_t iw = check(k, round++, &est, &mx);
            if (mx <= zthr || est <= eps * eps * fro2) {
                result = k;
                break;
            }
            ir = iw;
        }
        __syncthreads();   // the visited list is read again after tid 0 appends to it
    }
    if (tid == 0) rank[b] = result;
}

// factors of block b from the rank bound into exact-rank storage: U (m x r), then V (nn x r)
__global__ __launch_bounds__(256) void k_hm_compact(const int32_t* __restrict__ llist, const int32_t* __restrict__ m,
                                                    const int32_t* __restrict__ nn, const int64_t* __restrict__ soff,
                                                    const double* __restrict__ scratch,
                                                    const int32_t* __restrict__ rank, const int64_t* __restrict__ foff,
                                                    double* __restrict__ F) {
    const int32_t b = llist[blockIdx.x];
    const int32_t r = rank[b];
    if (r <= 0) return;
    const int64_t M = m[b], Nn = nn[b];
    const double* U = scratch + soff[b];
    const double* V = U + (int64_t)HM_KMAX * M;
    double* Uf = F + foff[b];
    double* Vf = Uf + (int64_t)r * M;
    for (int64_t e = threadIdx.x; e < (int64_t)r * M; e += 256) Uf[e] = U[e];
    for (int64_t e = threadIdx.x; e < (int64_t)r * Nn; e += 256) Vf[e] = V[e];
}

__global__ __launch_bounds__(256) void k_hm_gather(int64_t N, const int32_t* __restrict__ perm,
                                                   const double* __restrict__ x, double* __restrict__ xp) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < N) xp[i] = x[perm[i]];
}

// t_b[q] = sum_j V_b[q][j] xp[cs + j] for q < rank_b: one workgroup per low-rank block, wave w takes
// q = w, w + 4, ...
__global__ __launch_bounds__(256) void k_hm_vt(const int32_t* __restrict__ llist, const int32_t* __restrict__ m,
                                               const int32_t* __restrict__ cs, const int32_t* __restrict__ nn,
                                               const int32_t* __restrict__ rank, const int64_t* __restrict__ foff,
                                               const int64_t* __restrict__ toff, const double* __restrict__ F,
                                               const double* __restrict__ xp, double* __restrict__ t) {
    const int32_t b = llist[blockIdx.x];
    const int32_t r = rank[b];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t M = m[b], Nn = nn[b], c0 = cs[b];
    const double* V = F + foff[b] + (int64_t)r * M;
    for (int q = wv; q < r; q += 4) {
        double s = 0.0;
        for (int64_t j = lane; j < Nn; j += 64) s += V[(int64_t)q * Nn + j] * xp[c0 + j];
        s = wave_sum(s);
        if (lane == 0) t[toff[b] + q] = s;
    }
}

// one workgroup per leaf of rows (<= 256 rows, one thread each): every block over the leaf in
// block order (dense: its rows' dot products with xp; low rank: U_b t_b), then y[perm[i]], with
// -x[N + f] for the rows of floating body f
__global__ __launch_bounds__(256) void k_hm_rows(const int32_t* __restrict__ leaf_rs, const int32_t* __restrict__ leaf_m,
                                                 const int32_t* __restrict__ lb_ptr, const int32_t* __restrict__ lb,
                                                 const int32_t* __restrict__ kind, const int32_t* __restrict__ rs,
                                                 const int32_t* __restrict__ m, const int32_t* __restrict__ cs,
                                                 const int32_t* __restrict__ nn, const int32_t* __restrict__ rank,
                                                 const int64_t* __restrict__ doff, const int64_t* __restrict__ foff,
                                                 const int64_t* __restrict__ toff, const double* __restrict__ D,
                                                 const double* __restrict__ F, const double* __restrict__ t,
                                                 const double* __restrict__ xp, const int32_t* __restrict__ perm,
                                                 const int32_t* __restrict__ tri_body,
                                                 const int32_t* __restrict__ body_kind,
                                                 const int32_t* __restrict__ fidx, const double* __restrict__ x,
                                                 int64_t N, double* __restrict__ y) {
    const int32_t L = blockIdx.x;
    const int64_t i = leaf_rs[L] + threadIdx.x;   // cluster-order row
    if (threadIdx.x >= leaf_m[L]) return;
    double acc = 0.0;
    for (int32_t e = lb_ptr[L]; e < lb_ptr[L + 1]; ++e) {
        const int32_t b = lb[e];
        const int64_t ii = i - rs[b], M = m[b];
        if (kind[b] == 0) {
            const double* Db = D + doff[b];
            const int64_t c0 = cs[b], Nn = nn[b];
            double s = 0.0;
            for (int64_t j = 0; j < Nn; ++j) s += Db[j * M + ii] * xp[c0 + j];
            acc += s;
        } else {
            const int32_t r = rank[b];
            const double* U = F + foff[b];
            const double* tb = t + toff[b];
            double s = 0.0;
            for (int q = 0; q < r; ++q) s += U[(int64_t)q * M + ii] * tb[q];
            acc += s;
        }
    }
    const int64_t p = perm[i];
    const int32_t bd = tri_body[p];
    if (body_kind[bd] == BEM_FLOATING) acc -= x[N + fidx[bd]];
    y[p] = acc;
}

// constraint row f of the system (Eq. Final4 / sheets / net charge), dense over the N panels in
// their own order: C[f][j] = sum_{i in f} a_i (c_self delta_ij + c_kp K'_ij) / sum_{i in f} a_i,
// the body's rows taken in ascending order (one thread per column)
__global__ __launch_bounds__(256) void k_hm_constraint_rows(HmEntryArgs a, int64_t N, const int32_t* __restrict__ rows,
                                                            int64_t s0, int64_t s1, double c_self, double c_kp,
                                                            double* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    double acc = 0.0, asum = 0.0;
    for (int64_t s = s0; s < s1; ++s) {
        const int64_t i = rows[s];
        const double ai = a.tri64[(int64_t)TRI_REC * i + TR_A];
        const double kp = c_kp != 0.0 ? hm_kprime(a, i, j) : 0.0;
        acc += ai * (c_kp * kp + (i == j ? c_self : 0.0));
        asum += ai;
    }
    out[j] = acc / asum;
}

// y[N + f] = C[f] . x[0..N) (one workgroup per floating body, fixed-order reduction)
__global__ __launch_bounds__(256) void k_hm_constraint_apply(int64_t N, const double* __restrict__ C,
                                                             const double* __restrict__ x, double* __restrict__ y) {
    __shared__ double red[4];
    const int f = blockIdx.x;
    double s = 0.0;
    for (int64_t j = threadIdx.x; j < N; j += 256) s += C[(int64_t)f * N + j] * x[j];
    s = block_sum(s, red);
    if (threadIdx.x == 0) y[N + f] = s;
}

// Jacobi diagonal: the entries (i, i) (1 where one vanishes) and 1 for the constraint rows
__global__ __launch_bounds__(256) void k_hm_diag(HmEntryArgs a, int64_t N, int64_t n, double* __restrict__ diag) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    if (i >= N) {
        diag[i] = 1.0;
        return;
    }
    const double v = hm_entry(a, i, i);
    diag[i] = v != 0.0 ? v : 1.0;
}

// ---- host: cluster tree and block tree -----------------------------------------------------
struct Cluster {
    int32_t start, size, child0, child1;
    double lo[3], hi[3];   // box of the cluster's panels (their vertices)
};

struct Builder {
    const std::vector<double>& rec;   // TRI_REC doubles per panel (host copy of tri64)
    std::vector<int32_t> perm;
    std::vector<Cluster> cl;
    int leaf;
    explicit Builder(const std::vector<double>& r, int64_t N, int lf) : rec(r), perm(N), leaf(lf) {
        std::iota(perm.begin(), perm.end(), 0);
    }
    double cen(int32_t p, int k) const { return rec[(size_t)TRI_REC * p + TR_C + k]; }
    int32_t build(int32_t s, int32_t e) {
        Cluster c{s, e - s, -1, -1, {INFINITY, INFINITY, INFINITY}, {-INFINITY, -INFINITY, -INFINITY}};
        double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int32_t q = s; q < e; ++q) {
            const int32_t p = perm[q];
            for (int k = 0; k < 3; ++k) {
                for (int v = 0; v < 3; ++v) {
                    const double x = rec[(size_t)TRI_REC * p + TR_V + 3 * v + k];
                    c.lo[k] = std::min(c.lo[k], x);
                    c.hi[k] = std::max(c.hi[k], x);
                }
                clo[k] = std::min(clo[k], cen(p, k));
                chi[k] = std::max(chi[k], cen(p, k));
            }
        }
        const int32_t id = (int32_t)cl.size();
        cl.push_back(c);
        if (e - s > leaf) {
            int ax = 0;
            for (int k = 1; k < 3; ++k)
                if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
            const int32_t mid = s + (e - s) / 2;
            // median split along the axis; ties by panel index, so the order is reproducible
            std::nth_element(perm.begin() + s, perm.begin() + mid, perm.begin() + e, [&](int32_t u, int32_t v) {
                const double cu = cen(u, ax), cv = cen(v, ax);
                return cu < cv || (cu == cv && u < v);
            });
            const int32_t c0 = build(s, mid);
            const int32_t c1 = build(mid, e);
            cl[id].child0 = c0;
            cl[id].child1 = c1;
        }
        return id;
    }
};

double box_diam(const Cluster& c) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) s += (c.hi[k] - c.lo[k]) * (c.hi[k] - c.lo[k]);
    return std::sqrt(s);
}
double box_dist(const Cluster& a, const Cluster& b) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double d = std::max(0.0, std::max(a.lo[k] - b.hi[k], b.lo[k] - a.hi[k]));
        s += d * d;
    }
    return std::sqrt(s);
}

}  // namespace

struct HMatrix {
    int64_t N = 0;
    std::vector<int32_t> perm;
    std::vector<Cluster> cl;
    // blocks: row cluster range (rs, m), column range (cs, nn), kind 0 dense / 1 low rank
    std::vector<int32_t> rs, m, cs, nn, kind, rank;
    std::vector<int64_t> doff, foff, toff;
    int64_t dense_entries = 0, factor_entries = 0, rank_entries = 0;
    std::vector<int32_t> leaf_rs, leaf_m, lb_ptr, lb;
    DBuf d_perm, d_rs, d_m, d_cs, d_nn, d_kind, d_rank, d_doff, d_foff, d_toff, d_leaf_rs, d_leaf_m, d_lb_ptr, d_lb;
    DBuf D, F, t, xp, C, d_llist;
    int32_t n_llist = 0;   // low-rank blocks (d_llist)
    double eps = 0.0, eta = 0.0;
    int leaf = 0;

    void blocks(int32_t a, int32_t b) {
        const Cluster& A = cl[a];
        const Cluster& B = cl[b];
        const double dist = box_dist(A, B);
        if (dist > 0.0 && std::min(box_diam(A), box_diam(B)) <= eta * dist) {
            add(A, B, 1);
            return;
        }
        const bool la = A.child0 < 0, lbf = B.child0 < 0;
        if (la && lbf) {
            add(A, B, 0);
            return;
        }
        if (la) {
            blocks(a, B.child0);
            blocks(a, B.child1);
        } else if (lbf) {
            blocks(A.child0, b);
            blocks(A.child1, b);
        } else {
            blocks(A.child0, B.child0);
            blocks(A.child0, B.child1);
            blocks(A.child1, B.child0);
            blocks(A.child1, B.child1);
        }
    }
    void add(const Cluster& A, const Cluster& B, int k) {
        rs.push_back(A.start);
        m.push_back(A.size);
        cs.push_back(B.start);
        nn.push_back(B.size);
        kind.push_back(k);
    }
};

void hmatrix_release(bem_ctx* c) {
    delete c->hm;
    c->hm = nullptr;
}

static HmEntryArgs entry_args(bem_ctx* c, const int32_t* perm) {
    return {c->tri64.as<double>(), c->pan64.as<double>(), perm, c->tri_body.as<int32_t>(), c->body_kind.as<int32_t>(),
            c->body_epsp.as<double>(), c->body_epsm.as<double>()};
}

template <class T>
static void up(DBuf& d, const std::vector<T>& h, hipStream_t s) {
    d.alloc(sizeof(T) * std::max<size_t>(h.size(), 1));
    if (!h.empty()) BEM_HIP(hipMemcpyAsync(d.p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice, s));
}

void hmatrix_build(bem_ctx* c, double eps, double eta, int leaf, HmStats* st) {
    const int64_t N = c->N, n = c->n;
    hipStream_t s = c->stream;
    std::unique_ptr<HMatrix> h(new HMatrix());
    h->N = N;
    h->eps = eps;
    h->eta = eta;
    h->leaf = leaf;
    // host copy of the panel records
    std::vector<double> rec((size_t)TRI_REC * N);
    BEM_HIP(hipMemcpyAsync(rec.data(), c->tri64.p, sizeof(double) * rec.size(), hipMemcpyDeviceToHost, s));
    BEM_HIP(hipStreamSynchronize(s));
    Builder bld(rec, N, leaf);
    bld.build(0, (int32_t)N);
    h->perm = std::move(bld.perm);
    h->cl = std::move(bld.cl);
    h->blocks(0, 0);
    const int32_t nb = (int32_t)h->rs.size();
    // leaves in cluster order and, for each, the blocks over it (block order)
    std::vector<int32_t> leaf_of((size_t)N, -1);
    for (const Cluster& q : h->cl)
        if (q.child0 < 0) {
            for (int32_t i = q.start; i < q.start + q.size; ++i) leaf_of[i] = (int32_t)h->leaf_rs.size();
            h->leaf_rs.push_back(q.start);
            h->leaf_m.push_back(q.size);
        }
    // leaves were appended in tree order (depth first, left to right): cluster order
    const int32_t nl = (int32_t)h->leaf_rs.size();
    std::vector<std::vector<int32_t>> per(nl);
    for (int32_t b = 0; b < nb; ++b) {
        const int32_t l0 = leaf_of[h->rs[b]], l1 = leaf_of[h->rs[b] + h->m[b] - 1];
        for (int32_t l = l0; l <= l1; ++l) per[l].push_back(b);
    }
    h->lb_ptr.assign(nl + 1, 0);
    for (int32_t l = 0; l < nl; ++l) h->lb_ptr[l + 1] = h->lb_ptr[l] + (int32_t)per[l].size();
    for (int32_t l = 0; l < nl; ++l) h->lb.insert(h->lb.end(), per[l].begin(), per[l].end());
    for (int32_t l = 0; l < nl; ++l)
        if (h->leaf_m[l] > 256) throw Error(BEM_ERR_INVALID, "leaf size above 256");
    // scratch of the low-rank blocks at the rank bound, and their list
    std::vector<int32_t> llist;
    std::vector<int64_t> soff((size_t)nb, 0);
    int64_t scratch = 0;
    for (int32_t b = 0; b < nb; ++b)
        if (h->kind[b] == 1) {
            llist.push_back(b);
            soff[b] = scratch;
            scratch += (int64_t)HM_KMAX * (h->m[b] + h->nn[b]);
        }
    // memory check before any allocation
    size_t free_b = 0, total_b = 0;
    BEM_HIP(hipMemGetInfo(&free_b, &total_b));
    int64_t dense0 = 0;
    for (int32_t b = 0; b < nb; ++b)
        if (h->kind[b] == 0) dense0 += (int64_t)h->m[b] * h->nn[b];
    const size_t need = sizeof(double) * ((size_t)scratch + (size_t)dense0 + (size_t)c->n_float * N + 2 * (size_t)N);
    if (need > free_b) throw Error(BEM_ERR_OOM, "compression needs " + std::to_string(need >> 20) + " MiB");
    h->rank.assign(nb, 0);
    up(h->d_perm, h->perm, s);
    up(h->d_rs, h->rs, s);
    up(h->d_m, h->m, s);
    up(h->d_cs, h->cs, s);
    up(h->d_nn, h->nn, s);
    up(h->d_kind, h->kind, s);
    const HmEntryArgs ea = entry_args(c, h->d_perm.as<int32_t>());
    // low-rank blocks by cross approximation
    DBuf d_scr, d_soff, d_llist;
    up(h->d_rank, h->rank, s);
    if (!llist.empty()) {
        d_scr.alloc(sizeof(double) * (size_t)scratch);
        up(d_soff, soff, s);
        up(d_llist, llist, s);
        hipLaunchKernelGGL(k_hm_aca, dim3((unsigned)llist.size()), dim3(256), 0, s, ea, d_llist.as<int32_t>(),
                           h->d_rs.as<int32_t>(), h->d_m.as<int32_t>(), h->d_cs.as<int32_t>(), h->d_nn.as<int32_t>(),
                           d_soff.as<int64_t>(), d_scr.as<double>(), eps, h->d_rank.as<int32_t>());
        BEM_CHECK_LAUNCH();
        BEM_HIP(hipMemcpyAsync(h->rank.data(), h->d_rank.p, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, s));
        BEM_HIP(hipStreamSynchronize(s));
    }
    // blocks whose cross approximation reached the rank bound are stored dense; a low-rank block
    // whose factors would hold more entries than the block is stored dense too
    std::vector<int32_t> final_lr;
    for (int32_t b : llist) {
        const int64_t r = h->rank[b];
        if (r < 0 || r * (h->m[b] + h->nn[b]) >= (int64_t)h->m[b] * h->nn[b])
            h->kind[b] = 0;
        else
            final_lr.push_back(b);
    }
    h->doff.assign(nb, 0);
    h->foff.assign(nb, 0);
    h->toff.assign(nb, 0);
    std::vector<int32_t> dlist;
    for (int32_t b = 0; b < nb; ++b)
        if (h->kind[b] == 0) {
            dlist.push_back(b);
            h->doff[b] = h->dense_entries;
            h->dense_entries += (int64_t)h->m[b] * h->nn[b];
        } else {
            h->foff[b] = h->factor_entries;
            h->factor_entries += (int64_t)h->rank[b] * (h->m[b] + h->nn[b]);
            h->toff[b] = h->rank_entries;
            h->rank_entries += h->rank[b];
        }
    up(h->d_kind, h->kind, s);
    up(h->d_rank, h->rank, s);
    up(h->d_doff, h->doff, s);
    up(h->d_foff, h->foff, s);
    up(h->d_toff, h->toff, s);
    h->F.alloc(sizeof(double) * (size_t)std::max<int64_t>(h->factor_entries, 1));
    up(h->d_llist, final_lr, s);
    h->n_llist = (int32_t)final_lr.size();
    if (!final_lr.empty()) {
        hipLaunchKernelGGL(k_hm_compact, dim3((unsigned)final_lr.size()), dim3(256), 0, s, h->d_llist.as<int32_t>(),
                           h->d_m.as<int32_t>(), h->d_nn.as<int32_t>(), d_soff.as<int64_t>(), d_scr.as<double>(),
                           h->d_rank.as<int32_t>(), h->d_foff.as<int64_t>(), h->F.as<double>());
        BEM_CHECK_LAUNCH();
        BEM_HIP(hipStreamSynchronize(s));   // the scratch and the list are released on return
    }
    d_scr.release();
    // dense blocks
    h->D.alloc(sizeof(double) * (size_t)std::max<int64_t>(h->dense_entries, 1));
    if (!dlist.empty()) {
        DBuf d_dlist;
        up(d_dlist, dlist, s);
        hipLaunchKernelGGL(k_hm_dense, dim3((unsigned)ceil_div(h->dense_entries, 256)), dim3(256), 0, s, ea,
                           h->dense_entries, (int32_t)dlist.size(), h->d_doff.as<int64_t>(), h->d_rs.as<int32_t>(),
                           h->d_m.as<int32_t>(), h->d_cs.as<int32_t>(), h->d_nn.as<int32_t>(), d_dlist.as<int32_t>(),
                           h->D.as<double>());
        BEM_CHECK_LAUNCH();
        BEM_HIP(hipStreamSynchronize(s));
    }
    up(h->d_leaf_rs, h->leaf_rs, s);
    up(h->d_leaf_m, h->leaf_m, s);
    up(h->d_lb_ptr, h->lb_ptr, s);
    up(h->d_lb, h->lb, s);
    h->t.alloc(sizeof(double) * (size_t)std::max<int64_t>(h->rank_entries, 1));
    h->xp.alloc(sizeof(double) * (size_t)N);
    // constraint rows of the floating bodies (panel order)
    h->C.alloc(sizeof(double) * (size_t)std::max<int64_t>((int64_t)c->n_float * N, 1));
    int64_t s0 = 0;
    const HmEntryArgs ea_id = entry_args(c, nullptr);
    for (int32_t f = 0; f < c->n_float; ++f) {
        int32_t fb = -1;
        for (int32_t b = 0; b < c->n_body; ++b)
            if (c->h_body_fidx[b] == f) fb = b;
        int64_t s1 = s0;
        while (s1 < (int64_t)c->h_rows_flt.size() && c->h_tri_body[c->h_rows_flt[s1]] == fb) ++s1;
        hipLaunchKernelGGL(k_hm_constraint_rows, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, ea_id, N,
                           c->rows_flt.as<int32_t>(), s0, s1, c->h_flt_coef[2 * f], c->h_flt_coef[2 * f + 1],
                           h->C.as<double>() + (int64_t)f * N);
        BEM_CHECK_LAUNCH();
        s0 = s1;
    }
    c->diag.alloc(sizeof(double) * (size_t)c->ld);
    hipLaunchKernelGGL(k_hm_diag, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, ea_id, N, n, c->diag.as<double>());
    BEM_CHECK_LAUNCH();
    BEM_HIP(hipStreamSynchronize(s));
    if (st) {
        st->blocks = nb;
        st->lowrank_blocks = (int64_t)final_lr.size();
        st->dense_entries = h->dense_entries;
        st->factor_entries = h->factor_entries;
        int64_t mx = 0;
        for (int32_t b : final_lr) mx = std::max<int64_t>(mx, h->rank[b]);
        st->max_rank = mx;
    }
    hmatrix_release(c);
    c->hm = h.release();
}

// y = A x with the compressed operator (x, y of length n, no overlap)
void hmatrix_matvec(bem_ctx* c, const double* x, double* y, hipStream_t s) {
    HMatrix* h = c->hm;
    const int64_t N = c->N;
    KTimer kt(c, "hm_matvec", true, s);
    hipLaunchKernelGGL(k_hm_gather, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, N, h->d_perm.as<int32_t>(), x,
                       h->xp.as<double>());
    BEM_CHECK_LAUNCH();
    if (h->n_llist > 0) {
        hipLaunchKernelGGL(k_hm_vt, dim3((unsigned)h->n_llist), dim3(256), 0, s, h->d_llist.as<int32_t>(),
                           h->d_m.as<int32_t>(), h->d_cs.as<int32_t>(), h->d_nn.as<int32_t>(), h->d_rank.as<int32_t>(),
                           h->d_foff.as<int64_t>(), h->d_toff.as<int64_t>(), h->F.as<double>(), h->xp.as<double>(),
                           h->t.as<double>());
        BEM_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_hm_rows, dim3((unsigned)h->leaf_rs.size()), dim3(256), 0, s, h->d_leaf_rs.as<int32_t>(),
                       h->d_leaf_m.as<int32_t>(), h->d_lb_ptr.as<int32_t>(), h->d_lb.as<int32_t>(),
                       h->d_kind.as<int32_t>(), h->d_rs.as<int32_t>(), h->d_m.as<int32_t>(), h->d_cs.as<int32_t>(),
                       h->d_nn.as<int32_t>(), h->d_rank.as<int32_t>(), h->d_doff.as<int64_t>(),
                       h->d_foff.as<int64_t>(), h->d_toff.as<int64_t>(), h->D.as<double>(), h->F.as<double>(),
                       h->t.as<double>(), h->xp.as<double>(), h->d_perm.as<int32_t>(), c->tri_body.as<int32_t>(),
                       c->body_kind.as<int32_t>(), c->body_fidx.as<int32_t>(), x, N, y);
    BEM_CHECK_LAUNCH();
    if (c->n_float > 0) {
        hipLaunchKernelGGL(k_hm_constraint_apply, dim3((unsigned)c->n_float), dim3(256), 0, s, N, h->C.as<double>(), x,
                           y);
        BEM_CHECK_LAUNCH();
    }
}

}  // namespace bem
