// Assembly of the collocation system (Eqs. Final1-Final4) on gfx950.
//
// Pass 1 (k_far): regular pairs by the 7-point rule.  Each lane owns one
// panel (column j), its nodes and weights live in registers, and the wave
// walks down a block of rows whose collocation points are wave-uniform
// (scalar loads).  Stores of a row are 64 consecutive doubles per wave.
// Near-singular and singular pairs are not integrated here: they are written
// as zero by a select (the 7-point rule has a node at the centroid, so the
// self pair would divide by zero) and recorded in a 64-bit ballot mask per
// (row, 64-panel group) -- the "not processed" marks of Sec. 4.
// Pass 2 compacts the masks into a CSR near list (count, scan, fill) and
// k_near evaluates every near pair with the closed forms, one lane per pair,
// so that the divergent work runs on its own (Sec. 4, deferred near pass).
// Pass 3 forms the constraint rows of floating bodies (Eq. Final4) and the
// -1 columns of their potentials (Eq. Final2).
#include <algorithm>

#include "bem_device.h"

namespace bem {
namespace {


// MODE 0: potential rows S_ij = sum_q w_q / |x_i - y_q|
// MODE 1: normal-derivative rows K'_ij = n_i . sum_q w_q (x_i - y_q) / |x_i - y_q|^3,
//         multiplied by row_scale[r]
template <int MODE, typename R>
__global__ __launch_bounds__(256) void k_far(const double* __restrict__ far64, const R* __restrict__ farR, int64_t Np,
                                             const double* __restrict__ tri64, int64_t N,
                                             const int32_t* __restrict__ rows, int64_t n_rows,
                                             const double* __restrict__ row_scale, R* __restrict__ out, int64_t ld,
                                             int out_by_slot, uint64_t* __restrict__ mask, int rows_per_block) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;   // < Np always
    const bool valid = j < N;
    const double ccx = far64[(int64_t)(FR_CC + 0) * Np + j];
    const double ccy = far64[(int64_t)(FR_CC + 1) * Np + j];
    const double ccz = far64[(int64_t)(FR_CC + 2) * Np + j];
    const double rr = far64[(int64_t)FR_RR * Np + j];
    R qx[7], qy[7], qz[7], qw[7];
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        qx[q] = farR[(int64_t)(FR_X + q) * Np + j];
        qy[q] = farR[(int64_t)(FR_Y + q) * Np + j];
        qz[q] = farR[(int64_t)(FR_Z + q) * Np + j];
        qw[q] = farR[(int64_t)(FR_W + q) * Np + j];
    }
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_block;
    const int64_t r1 = r0 + rows_per_block < n_rows ? r0 + rows_per_block : n_rows;
    const bool wave_live = ((j & ~(int64_t)63) < N);
    for (int64_t r = r0; r < r1; ++r) {
        const int64_t i = rows[r];
        const double* Ti = tri64 + (int64_t)TRI_REC * i;
        const double xi0 = Ti[TR_C + 0], xi1 = Ti[TR_C + 1], xi2 = Ti[TR_C + 2];
        const bool regular = is_regular(xi0 - ccx, xi1 - ccy, xi2 - ccz, rr) && (j != i);
        const R x0 = (R)xi0, x1 = (R)xi1, x2 = (R)xi2;
        R acc;
        if (MODE == 0) {
            R s = (R)0;
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                const R dx = x0 - qx[q], dy = x1 - qy[q], dz = x2 - qz[q];
                const R r2 = dx * dx + dy * dy + dz * dz;
                s += qw[q] * rsqrt_pos(r2);
            }
            acc = s;
        } else {
            R f0 = 0, f1 = 0, f2 = 0;
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                const R dx = x0 - qx[q], dy = x1 - qy[q], dz = x2 - qz[q];
                const R r2 = dx * dx + dy * dy + dz * dz;
                const R ir = rsqrt_pos(r2);
                const R t = qw[q] * ir * ir * ir;
                f0 += t * dx;
                f1 += t * dy;
                f2 += t * dz;
            }
            const R n0 = (R)Ti[TR_N + 0], n1 = (R)Ti[TR_N + 1], n2 = (R)Ti[TR_N + 2];
            acc = (n0 * f0 + n1 * f1 + n2 * f2) * (R)row_scale[r];
        }
        const R val = regular ? acc : (R)0;
        const int64_t orow = out_by_slot ? r : i;
        if (valid) out[orow * ld + j] = val;
        if (mask) {
            const uint64_t m = __ballot(valid && !regular);
            if (wave_live && (threadIdx.x & 63) == 0) mask[(j >> 6) * N + i] = m;
        }
    }
}

__global__ __launch_bounds__(256) void k_mask_count(const uint64_t* __restrict__ mask, int64_t nblk, int64_t T,
                                                    int64_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= T) return;
    int64_t c = 0;
    for (int64_t b = 0; b < nblk; ++b) c += __popcll(mask[b * T + i]);
    cnt[i] = c;
}

// exclusive scan of cnt[0..T) into ptr[0..T]; one block of 1024 threads
__global__ __launch_bounds__(1024) void k_scan(const int64_t* __restrict__ cnt, int64_t T, int64_t* __restrict__ ptr) {
    __shared__ int64_t s[1024];
    const int tid = threadIdx.x;
    const int64_t per = (T + 1023) / 1024;
    const int64_t beg = tid * per < T ? tid * per : T;
    const int64_t end = beg + per < T ? beg + per : T;
    int64_t local = 0;
    for (int64_t k = beg; k < end; ++k) local += cnt[k];
    s[tid] = local;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = tid >= d ? s[tid - d] : 0;
        __syncthreads();
        s[tid] += v;
        __syncthreads();
    }
    int64_t off = tid > 0 ? s[tid - 1] : 0;
    for (int64_t k = beg; k < end; ++k) {
        ptr[k] = off;
        off += cnt[k];
    }
    if (tid == 1023) ptr[T] = s[1023];
}

__global__ __launch_bounds__(256) void k_mask_fill(const uint64_t* __restrict__ mask, int64_t nblk, int64_t T,
                                                   const int64_t* __restrict__ ptr, int32_t* __restrict__ row,
                                                   int32_t* __restrict__ col) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= T) return;
    int64_t o = ptr[i];
    for (int64_t b = 0; b < nblk; ++b) {
        uint64_t m = mask[b * T + i];
        while (m) {
            const int bit = __builtin_ctzll(m);
            col[o] = (int32_t)(b * 64 + bit);
            row[o] = (int32_t)i;
            ++o;
            m &= m - 1;
        }
    }
}

// Deferred near pass: one lane per (row, panel) near pair, closed forms in FP64.
__global__ __launch_bounds__(256) void k_near(const double* __restrict__ tri64, const int32_t* __restrict__ tri_body,
                                              const int32_t* __restrict__ body_kind,
                                              const double* __restrict__ epsp, const double* __restrict__ epsm,
                                              const int32_t* __restrict__ row_slot, int64_t nnz,
                                              const int32_t* __restrict__ nrow, const int32_t* __restrict__ ncol,
                                              double* __restrict__ A64, float* __restrict__ A32, int64_t ld,
                                              double* __restrict__ nval, double* __restrict__ Kf, int64_t N,
                                              double* __restrict__ diag, const double* __restrict__ sf) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= nnz) return;
    const int64_t i = nrow[k], j = ncol[k];
    const double* Ti = tri64 + (int64_t)TRI_REC * i;
    const double* Tj = tri64 + (int64_t)TRI_REC * j;
    const int32_t b = tri_body[i];
    const int32_t kind = body_kind[b];
    const bool self = (i == j);
    double S, F0, F1, F2;
    if (sf) {   // S and F from the near-singular rule (Duffy); the self pair's F is not used
        S = sf[4 * k];
        F0 = sf[4 * k + 1];
        F1 = sf[4 * k + 2];
        F2 = sf[4 * k + 3];
    } else {
        flat_tri_SF<true, true>(Tj, Ti[TR_C + 0], Ti[TR_C + 1], Ti[TR_C + 2], self, S, F0, F1, F2);
    }
    const double kp = self ? 0.0 : (Ti[TR_N + 0] * F0 + Ti[TR_N + 1] * F1 + Ti[TR_N + 2] * F2);
    double v;
    if (kind == BEM_INTERFACE)
        v = self ? 0.5 * (epsp[b] + epsm[b]) : (epsp[b] - epsm[b]) * kp;
    else
        v = S;
    if (A64) A64[i * ld + j] = v;
    if (A32) {
        // mixed operator: FP32 head in the dense slot, exact FP64 remainder in the near list, so that
        // head + remainder == v exactly and a pure FP32 product sees every entry to FP32 accuracy
        const float hi = (float)v;
        A32[i * ld + j] = hi;
        nval[k] = v - (double)hi;
    }
    if (self) diag[i] = (v != 0.0) ? v : 1.0;
    if (Kf && kind == BEM_FLOATING) Kf[(int64_t)row_slot[i] * N + j] = kp;
}

// Constraint row of one floating body:
// row[j] = sum_{i in body} a_i (c_self delta_ij + c_kp K'_ij) / sum_{i in body} a_i
// with (c_self, c_kp) = (1/2, 1) for a closed body (Eq. Final4, eps+ (sigma/2 + K' sigma), scaled
// by 1/(eps+ sum a_i)) and (1, 2 (eps+ - eps-) / (eps+ + eps-)) for a thin sheet (Eq. sheets,
// (eps+ + eps-)/2 sigma + (eps+ - eps-) K' sigma, scaled by 2/((eps+ + eps-) sum a_i)).
// The body's rows s0..s1 are cut into slabs of `per` rows, one per grid row y, each summed in
// order into part[y][j] (and its area sum into apart[y]); k_constraint_sum adds the slabs in order.
__global__ __launch_bounds__(256) void k_constraint(const double* __restrict__ Kf, int64_t N,
                                                    const int32_t* __restrict__ rows_flt, int64_t s0, int64_t s1,
                                                    int64_t per, const double* __restrict__ tri64, double c_self,
                                                    double c_kp, double* __restrict__ part,
                                                    double* __restrict__ apart) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t y = blockIdx.y;
    const int64_t a0 = s0 + y * per, a1 = (a0 + per < s1) ? a0 + per : s1;
    double acc = 0.0, asum = 0.0;
    for (int64_t s = a0; s < a1; ++s) {
        const int64_t i = rows_flt[s];
        const double a = tri64[(int64_t)TRI_REC * i + TR_A];
        if (j < N) acc += a * (c_kp * Kf[s * N + j] + (i == j ? c_self : 0.0));
        asum += a;
    }
    if (j < N) part[y * N + j] = acc;
    if (blockIdx.x == 0 && threadIdx.x == 0) apart[y] = asum;
}

__global__ __launch_bounds__(256) void k_constraint_sum(int64_t N, int64_t slabs, const double* __restrict__ part,
                                                        const double* __restrict__ apart, double* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    double acc = 0.0, asum = 0.0;
    for (int64_t y = 0; y < slabs; ++y) {
        acc += part[y * N + j];
        asum += apart[y];
    }
    out[j] = acc / asum;
}

// Reduced constraint (net charge): row[j] = a_j / sum a_i for j in the body
__global__ __launch_bounds__(256) void k_constraint_reduced(int64_t N, const int32_t* __restrict__ rows_flt, int64_t s0,
                                                            int64_t s1, const double* __restrict__ tri64,
                                                            double* __restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    double asum = 0.0, aj = 0.0;
    for (int64_t s = s0; s < s1; ++s) {
        const int64_t i = rows_flt[s];
        const double a = tri64[(int64_t)TRI_REC * i + TR_A];
        asum += a;
        if (i == j) aj = a;
    }
    out[j] = aj / asum;
}

// Columns N..ld-1: -1 at the potential column of a floating row, 0 elsewhere.
template <typename R>
__global__ __launch_bounds__(256) void k_finalize_cols(R* __restrict__ A, int64_t rows, int64_t ld, int64_t N,
                                                       int64_t row_base, const int32_t* __restrict__ tri_body,
                                                       const int32_t* __restrict__ body_kind,
                                                       const int32_t* __restrict__ fidx) {
    const int64_t ncols = ld - N;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= rows * ncols) return;
    const int64_t r = t / ncols, c = N + t % ncols;
    const int64_t i = row_base + r;
    R v = (R)0;
    if (i < N) {
        const int32_t b = tri_body[i];
        if (body_kind[b] == BEM_FLOATING && c == N + fidx[b]) v = (R)-1;
    }
    A[r * ld + c] = v;
}

__global__ void k_fill_diag_tail(double* __restrict__ diag, int64_t N, int64_t n) {
    const int64_t i = N + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) diag[i] = 1.0;
}

__global__ __launch_bounds__(256) void k_copy_rows64(const double* __restrict__ A, int64_t ld, int64_t row0,
                                                     int64_t n_rows, int64_t n, double* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_rows * n) return;
    const int64_t r = t / n, c = t % n;
    out[t] = A[(row0 + r) * ld + c];
}

__global__ __launch_bounds__(256) void k_copy_rows32(const float* __restrict__ A, int64_t ld, int64_t row0,
                                                     int64_t n_rows, int64_t n, double* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= n_rows * n) return;
    const int64_t r = t / n, c = t % n;
    out[t] = (double)A[(row0 + r) * ld + c];
}

__global__ __launch_bounds__(256) void k_scatter_near_rows(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                                                           const double* __restrict__ val, int64_t row0,
                                                           int64_t n_rows, int64_t n, double* __restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n_rows) return;
    for (int64_t e = ptr[row0 + r]; e < ptr[row0 + r + 1]; ++e) out[r * n + col[e]] += val[e];
}

// rows [0, nb) carry a body (panels, or vertices of the nodal basis); the others are constraint rows
__global__ __launch_bounds__(256) void k_rhs(const int32_t* __restrict__ row_body, const int32_t* __restrict__ body_kind,
                                             int64_t nb, int64_t n, int32_t n_body, int32_t nrhs,
                                             const double* __restrict__ bodyV, double* __restrict__ b) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)nrhs * n) return;
    const int64_t r = t / n, i = t % n;
    double v = 0.0;
    if (i < nb) {
        const int32_t bd = row_body[i];
        if (body_kind[bd] == BEM_DIRICHLET) v = bodyV[r * n_body + bd];
    }
    b[t] = v;
}

}  // namespace

static int64_t padded_panels(const bem_ctx* c) { return (int64_t)(c->far64.bytes / (sizeof(double) * FAR_REC)); }

void launch_far_assemble(bem_ctx* c) {
    KTimer t(c, "far_assemble");
    const int64_t Np = padded_panels(c);
    const bool mixed = c->opt.precision == BEM_MIXED;
    uint64_t* mask = c->nearmask.as<uint64_t>();
    auto launch = [&](int mode, const bem::DBuf& rows, int64_t nr, const double* scale, bool by_slot, bool with_mask,
                      void* out, int64_t ld, bool fp32) {
        if (nr == 0) return;
        const int rpb = c->tune_far_rows;
        dim3 grid((unsigned)(Np / 256), (unsigned)ceil_div(nr, rpb));
        uint64_t* m = with_mask ? mask : nullptr;
        if (!fp32) {
            if (mode == 0)
                hipLaunchKernelGGL((k_far<0, double>), grid, dim3(256), 0, c->stream, c->far64.as<double>(),
                                   c->far64.as<double>(), Np, c->tri64.as<double>(), c->N, rows.as<int32_t>(), nr,
                                   scale, (double*)out, ld, (int)by_slot, m, rpb);
            else
                hipLaunchKernelGGL((k_far<1, double>), grid, dim3(256), 0, c->stream, c->far64.as<double>(),
                                   c->far64.as<double>(), Np, c->tri64.as<double>(), c->N, rows.as<int32_t>(), nr,
                                   scale, (double*)out, ld, (int)by_slot, m, rpb);
        } else {
            if (mode == 0)
                hipLaunchKernelGGL((k_far<0, float>), grid, dim3(256), 0, c->stream, c->far64.as<double>(),
                                   c->far32.as<float>(), Np, c->tri64.as<double>(), c->N, rows.as<int32_t>(), nr,
                                   scale, (float*)out, ld, (int)by_slot, m, rpb);
            else
                hipLaunchKernelGGL((k_far<1, float>), grid, dim3(256), 0, c->stream, c->far64.as<double>(),
                                   c->far32.as<float>(), Np, c->tri64.as<double>(), c->N, rows.as<int32_t>(), nr,
                                   scale, (float*)out, ld, (int)by_slot, m, rpb);
        }
        BEM_CHECK_LAUNCH();
    };
    const int64_t npot = (int64_t)c->h_rows_pot.size(), nint = (int64_t)c->h_rows_int.size();
    const int64_t nflt = (int64_t)c->h_rows_flt.size();
    double* scale_int = c->gm_misc.as<double>();            // (eps+ - eps-) per interface row
    double* scale_one = scale_int + (nint > 0 ? nint : 1);  // 1 per floating row
    void* A = mixed ? c->A32.p : c->A64.p;
    launch(0, c->rows_pot, npot, nullptr, false, true, A, c->ld, mixed);
    launch(1, c->rows_int, nint, scale_int, false, true, A, c->ld, mixed);
    // K' block of floating rows (FP64 in both modes) for the constraint rows
    if (nflt > 0 && (c->opt.constraint_form == 0 || c->has_sheet))
        launch(1, c->rows_flt, nflt, scale_one, true, false, c->Kf.p, c->N, false);
}

void launch_near_csr(bem_ctx* c, const uint64_t* mask, int64_t T, DBuf& ptr, DBuf& row, DBuf& col, int64_t* nnz,
                     const char* tname) {
    KTimer t(c, tname);
    const int64_t nblk = ceil_div(c->N, 64);   // waves that own at least one real panel
    ptr.alloc(sizeof(int64_t) * (T + 1) * 2);
    int64_t* cnt = ptr.as<int64_t>() + (T + 1);
    hipLaunchKernelGGL(k_mask_count, dim3((unsigned)ceil_div(T, 256)), dim3(256), 0, c->stream, mask, nblk, T, cnt);
    BEM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, c->stream, cnt, T, ptr.as<int64_t>());
    BEM_CHECK_LAUNCH();
    int64_t* hs = c->host_stage.as<int64_t>();
    BEM_HIP(hipMemcpyAsync(hs, ptr.as<int64_t>() + T, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
    BEM_HIP(hipStreamSynchronize(c->stream));
    *nnz = hs[0];
    if (*nnz >= ((int64_t)1 << 31)) throw Error(BEM_ERR_INVALID, "near list exceeds 2^31 pairs");
    row.alloc(sizeof(int32_t) * (*nnz > 0 ? *nnz : 1));
    col.alloc(sizeof(int32_t) * (*nnz > 0 ? *nnz : 1));
    hipLaunchKernelGGL(k_mask_fill, dim3((unsigned)ceil_div(T, 256)), dim3(256), 0, c->stream, mask, nblk, T,
                       ptr.as<int64_t>(), row.as<int32_t>(), col.as<int32_t>());
    BEM_CHECK_LAUNCH();
}

void launch_near_assemble(bem_ctx* c) {
    KTimer t(c, "near_assemble");
    const bool mixed = c->opt.precision == BEM_MIXED;
    if (c->near_nnz == 0) return;
    double* Kf = ((c->opt.constraint_form == 0 || c->has_sheet) && !c->h_rows_flt.empty()) ? c->Kf.as<double>()
                                                                                              : nullptr;
    const double* sf = nullptr;
    if (c->near_rule == 1) {   // the paper's near-singular rule instead of the closed forms
        c->near_sf.alloc(sizeof(double) * 4 * (size_t)c->near_nnz);
        launch_near_duffy(c, c->near_nnz, c->near_row.as<int32_t>(), c->near_col.as<int32_t>(),
                          c->near_sf.as<double>());
        sf = c->near_sf.as<double>();
    }
    hipLaunchKernelGGL(k_near, dim3((unsigned)ceil_div(c->near_nnz, 256)), dim3(256), 0, c->stream,
                       c->tri64.as<double>(), c->tri_body.as<int32_t>(), c->body_kind.as<int32_t>(),
                       c->body_epsp.as<double>(), c->body_epsm.as<double>(), c->row_slot.as<int32_t>(), c->near_nnz,
                       c->near_row.as<int32_t>(), c->near_col.as<int32_t>(), mixed ? nullptr : c->A64.as<double>(),
                       mixed ? c->A32.as<float>() : nullptr, c->ld, mixed ? c->near_val.as<double>() : nullptr, Kf,
                       c->N,
                       c->diag.as<double>(), sf);
    BEM_CHECK_LAUNCH();
}

void launch_finalize(bem_ctx* c) {
    KTimer t(c, "finalize");
    const bool mixed = c->opt.precision == BEM_MIXED;
    const int64_t N = c->N, ld = c->ld;
    double* tail = mixed ? c->A64.as<double>() : c->A64.as<double>() + N * ld;
    // constraint rows, one per floating body (slots of a body are contiguous)
    int64_t s0 = 0;
    for (int32_t f = 0; f < c->n_float; ++f) {
        int32_t fb = -1;
        for (int32_t b = 0; b < c->n_body; ++b)
            if (c->h_body_fidx[b] == f) fb = b;
        int64_t s1 = s0;
        while (s1 < (int64_t)c->h_rows_flt.size() && c->h_tri_body[c->h_rows_flt[s1]] == fb) ++s1;
        // Eq. sheets for a sheet whatever the constraint form; Eq. Final4 literal for a closed body
        if (c->h_body_kind[fb] == BEM_FLOATING_SHEET || c->opt.constraint_form == 0) {
            // rows in slabs over a second grid dimension, so that about 1024 blocks stream the
            // body's K' block (one block row alone used a third of the CUs)
            const int64_t cb = ceil_div(N, 256), rows = s1 - s0;
            const int64_t slabs = std::max<int64_t>(1, std::min<int64_t>(rows, 1024 / cb));
            const int64_t per = ceil_div(std::max<int64_t>(rows, 1), slabs);
            c->cons_part.alloc(sizeof(double) * (size_t)(slabs * N + slabs));
            double* part = c->cons_part.as<double>();
            hipLaunchKernelGGL(k_constraint, dim3((unsigned)cb, (unsigned)slabs), dim3(256), 0, c->stream,
                               c->Kf.as<double>(), N, c->rows_flt.as<int32_t>(), s0, s1, per, c->tri64.as<double>(),
                               c->h_flt_coef[2 * f], c->h_flt_coef[2 * f + 1], part, part + slabs * N);
            BEM_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_constraint_sum, dim3((unsigned)cb), dim3(256), 0, c->stream, N, slabs, part,
                               part + slabs * N, tail + (int64_t)f * ld);
        } else
            hipLaunchKernelGGL(k_constraint_reduced, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, c->stream, N,
                               c->rows_flt.as<int32_t>(), s0, s1, c->tri64.as<double>(), tail + (int64_t)f * ld);
        BEM_CHECK_LAUNCH();
        s0 = s1;
    }
    const int64_t ncols = ld - N;
    if (ncols > 0) {
        if (mixed) {
            hipLaunchKernelGGL((k_finalize_cols<float>), dim3((unsigned)ceil_div(N * ncols, 256)), dim3(256), 0,
                               c->stream, c->A32.as<float>(), N, ld, N, (int64_t)0, c->tri_body.as<int32_t>(),
                               c->body_kind.as<int32_t>(), c->body_fidx.as<int32_t>());
            BEM_CHECK_LAUNCH();
            if (c->n_float > 0) {
                hipLaunchKernelGGL((k_finalize_cols<double>), dim3((unsigned)ceil_div(c->n_float * ncols, 256)),
                                   dim3(256), 0, c->stream, tail, (int64_t)c->n_float, ld, N, N,
                                   c->tri_body.as<int32_t>(), c->body_kind.as<int32_t>(), c->body_fidx.as<int32_t>());
                BEM_CHECK_LAUNCH();
            }
        } else {
            hipLaunchKernelGGL((k_finalize_cols<double>), dim3((unsigned)ceil_div(c->n * ncols, 256)), dim3(256), 0,
                               c->stream, c->A64.as<double>(), c->n, ld, N, (int64_t)0, c->tri_body.as<int32_t>(),
                               c->body_kind.as<int32_t>(), c->body_fidx.as<int32_t>());
            BEM_CHECK_LAUNCH();
        }
    }
    if (c->n > N) {
        hipLaunchKernelGGL(k_fill_diag_tail, dim3((unsigned)ceil_div(c->n - N, 256)), dim3(256), 0, c->stream,
                           c->diag.as<double>(), N, c->n);
        BEM_CHECK_LAUNCH();
    }
}

void launch_copy_rows(bem_ctx* c, int64_t row0, int64_t n_rows, double* out) {
    const bool mixed = c->opt.precision == BEM_MIXED;
    const int64_t N = c->nb, n = c->n, ld = c->ld;
    if (!mixed) {
        hipLaunchKernelGGL(k_copy_rows64, dim3((unsigned)ceil_div(n_rows * n, 256)), dim3(256), 0, c->stream,
                           c->A64.as<double>(), ld, row0, n_rows, n, out);
        BEM_CHECK_LAUNCH();
        return;
    }
    const int64_t r_end = row0 + n_rows;
    const int64_t fa = row0, fb = r_end < N ? r_end : N;   // rows from the FP32 far part
    if (fb > fa) {
        hipLaunchKernelGGL(k_copy_rows32, dim3((unsigned)ceil_div((fb - fa) * n, 256)), dim3(256), 0, c->stream,
                           c->A32.as<float>(), ld, fa, fb - fa, n, out);
        BEM_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_scatter_near_rows, dim3((unsigned)ceil_div(fb - fa, 256)), dim3(256), 0, c->stream,
                           c->near_ptr.as<int64_t>(), c->near_col.as<int32_t>(), c->near_val.as<double>(), fa, fb - fa,
                           n, out);
        BEM_CHECK_LAUNCH();
    }
    const int64_t ta = row0 > N ? row0 : N;
    if (r_end > ta) {
        hipLaunchKernelGGL(k_copy_rows64, dim3((unsigned)ceil_div((r_end - ta) * n, 256)), dim3(256), 0, c->stream,
                           c->A64.as<double>(), ld, ta - N, r_end - ta, n, out + (ta - row0) * n);
        BEM_CHECK_LAUNCH();
    }
}

void launch_rhs(bem_ctx* c, int32_t nrhs, const double* d_bodyV, double* b) {
    const bool nodal = c->opt.basis == BEM_BASIS_LINEAR;
    hipLaunchKernelGGL(k_rhs, dim3((unsigned)ceil_div((int64_t)nrhs * c->n, 256)), dim3(256), 0, c->stream,
                       nodal ? c->vert_body.as<int32_t>() : c->tri_body.as<int32_t>(), c->body_kind.as<int32_t>(),
                       nodal ? c->n_vert : c->N, c->n, c->n_body, nrhs, d_bodyV, b);
    BEM_CHECK_LAUNCH();
}

}  // namespace bem
