// Many load cases at once: up to 64 independent GMRES(m) recurrences (the
// method of Sec. 5.2 for each right-hand side) whose matrix products are one
// multi-right-hand-side product per iteration (k_gemm_f32 / k_gemm_f64), so
// the matrix is read once per iteration for all load cases.
//
// FP64 mode: the product uses the FP64 matrix on the FP64 matrix cores.
// Mixed mode: the inner product is the FP32 matrix (far entries and the FP32
// heads of the near entries) on the FP32 matrix cores, FP32 operands and
// accumulation, plus the FP64 constraint rows (a K-split row product); an outer FP64 iterative
// refinement recomputes the residual with the exact FP64-accumulated product
// of the mixed operator (FP32 matrix widened + FP64 near remainders), so the
// FP32 rounding of the inner products does not limit the final residual.
//
// Each recurrence keeps its own basis, Hessenberg matrix and rotations
// (independent, not block, Krylov spaces: identical or proportional
// right-hand sides cannot break them down).  Orthogonalisation is CGS2 in
// FP64 on the device; the host reads one Hessenberg column per recurrence
// and iteration.
#include <cmath>
#include <vector>

#include "bem_device.h"

namespace bem {

void launch_gemm_f32(bem_ctx* c, const float* A, int64_t lda, int64_t M, int64_t K, const float* Zt, int64_t ldz,
                     int ncols, double* Y, int64_t ldy, bool accumulate);
void launch_gemm_f64(bem_ctx* c, const void* A, bool a_is_f32, int64_t lda, int64_t M, int64_t K, const double* Zt,
                     int64_t ldz, int ncols, double* Y, int64_t ldy, bool accumulate, double alpha);
void launch_gemm_rows(bem_ctx* c, const double* A, int64_t lda, int64_t M, int64_t K, const double* Zn, int ncols,
                      double* Y, int64_t ldy, bool accumulate, double alpha);

namespace {

constexpr int BR = 64;   // right-hand sides per batch

// Zt32/Zt64[r][i] and Zn64[i][r] from src[r * sstride + i] (divided by d[i] if given); zero padding
__global__ __launch_bounds__(256) void k_b_prep(const double* __restrict__ src, int64_t sstride, int nr, int64_t n,
                                                int64_t ld, const double* __restrict__ d, float* __restrict__ zt32,
                                                double* __restrict__ zt64, double* __restrict__ zn64) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= ld) return;
    double v = 0.0;
    if (r < nr && i < n) {
        v = src[(int64_t)r * sstride + i];
        if (d) v /= d[i];
    }
    if (zt32) zt32[(int64_t)r * ld + i] = (float)v;
    if (zt64) zt64[(int64_t)r * ld + i] = v;
    if (zn64) zn64[i * BR + r] = v;
}

// W[r][i] += sum_e val[e] * Zn[col[e]][r] for the near entries of row i < N (one wave per row)
__global__ __launch_bounds__(256) void k_b_near(const int64_t* __restrict__ nptr, const int32_t* __restrict__ ncol,
                                                const double* __restrict__ nval, int64_t N,
                                                const double* __restrict__ zn64, int nr, double* __restrict__ W,
                                                int64_t ld) {
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int r = threadIdx.x & 63;
    if (i >= N) return;
    double s = 0.0;
    for (int64_t e = nptr[i]; e < nptr[i + 1]; ++e) s = fma(nval[e], zn64[(int64_t)ncol[e] * BR + r], s);
    if (r < nr) W[(int64_t)r * ld + i] += s;
}

// part[(r * m1 + k) * G + b] = sum over block b's slice of V[(r * m1 + k) * ld + i] * W[r * ld + i]
__global__ __launch_bounds__(256) void k_b_dots(const double* __restrict__ V, int m1, int64_t ld, int64_t n,
                                                const double* __restrict__ W, double* __restrict__ part, int G) {
    const int k = blockIdx.y, r = blockIdx.z;
    const double* v = V + ((int64_t)r * m1 + k) * ld;
    const double* w = W + (int64_t)r * ld;
    double s = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += (int64_t)G * 256) s = fma(v[t], w[t], s);
    s = wave_sum(s);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[((int64_t)r * m1 + k) * G + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// h[r][k] = sum_b part; Hcol[r][k] (+)= h[r][k]; optional sqrt (norms)
__global__ void k_b_reduce(const double* __restrict__ part, int G, int m1, int kcount, int nr, double* __restrict__ h,
                           int hstride, double* __restrict__ Hcol, int accumulate, int take_sqrt) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kcount * nr) return;
    const int r = t / kcount, k = t % kcount;
    double s = 0.0;
    for (int b = 0; b < G; ++b) s += part[((int64_t)r * m1 + k) * G + b];
    if (take_sqrt) s = sqrt(s);
    h[r * hstride + k] = s;
    if (Hcol) Hcol[r * hstride + k] = accumulate ? Hcol[r * hstride + k] + s : s;
}

// W[r] -= sum_k h[r][k] V[r][k]
__global__ __launch_bounds__(256) void k_b_orth(const double* __restrict__ V, int m1, int64_t ld, int64_t n, int kcount,
                                                const double* __restrict__ h, int hstride, double* __restrict__ W) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= n) return;
    double s = W[(int64_t)r * ld + i];
    for (int k = 0; k < kcount; ++k) s -= h[r * hstride + k] * V[((int64_t)r * m1 + k) * ld + i];
    W[(int64_t)r * ld + i] = s;
}

// out[r] = W[r] / nrm[r * nstride] (untouched where the norm is zero)
__global__ __launch_bounds__(256) void k_b_scale(const double* __restrict__ W, int64_t wstride,
                                                 const double* __restrict__ nrm, int nstride, int64_t n,
                                                 double* __restrict__ out, int64_t ostride) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    const double v = nrm[r * nstride];
    if (i >= n || v == 0.0) return;
    out[(int64_t)r * ostride + i] = W[(int64_t)r * wstride + i] / v;
}

// R[r] = B[r] - W[r]
__global__ __launch_bounds__(256) void k_b_residual(const double* __restrict__ B, const double* W, int64_t ld,
                                                    int64_t n, double* R) {   // R may be W
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (i < n) R[(int64_t)r * ld + i] = B[(int64_t)r * ld + i] - W[(int64_t)r * ld + i];
}

// X[r] += (sum_{k < jend[r]} y[r][k] V[r][k]) / d
__global__ __launch_bounds__(256) void k_b_update_x(const double* __restrict__ V, int m1, int64_t ld, int64_t n,
                                                    const double* __restrict__ y, const int32_t* __restrict__ jend,
                                                    const double* __restrict__ d, double* __restrict__ X) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < jend[r]; ++k) s = fma(y[r * m1 + k], V[((int64_t)r * m1 + k) * ld + i], s);
    X[(int64_t)r * ld + i] += s / d[i];
}

__global__ __launch_bounds__(256) void k_b_fill(double* __restrict__ X, int64_t count, double v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) X[i] = v;
}

__global__ __launch_bounds__(256) void k_b_add(double* __restrict__ X, const double* __restrict__ D, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) X[i] += D[i];
}

struct BW {
    bem_ctx* c;
    int nr, m, m1, G;
    int64_t n, N, ld;
    hipStream_t s;
    double *V, *W, *part, *h, *Hcol, *y;
    int32_t* jend;
    float* zt32;
    double *zt64, *zn64;
    double* host;   // pinned
    dim3 gv() const { return dim3((unsigned)ceil_div(n, 256), (unsigned)nr); }
};

// W = A * (src / d) for the nr vectors (stride sstride), inner (mixed: FP32 cores) or exact
void apply(BW& w, const double* src, int64_t sstride, const double* d, bool exact) {
    bem_ctx* c = w.c;
    const bool mixed = c->opt.precision == BEM_MIXED;
    const bool f32 = mixed && !exact;
    hipLaunchKernelGGL(k_b_prep, dim3((unsigned)ceil_div(w.ld, 256), BR), dim3(256), 0, w.s, src, sstride, w.nr, w.n,
                       w.ld, d, f32 ? w.zt32 : nullptr, f32 ? nullptr : w.zt64, (mixed && !f32) ? w.zn64 : nullptr);
    BEM_CHECK_LAUNCH();
    if (!mixed) {
        launch_gemm_f64(c, c->A64.p, false, w.ld, w.n, w.ld, w.zt64, w.ld, w.nr, w.W, w.ld, false, 1.0);
        return;
    }
    if (f32) {
        launch_gemm_f32(c, c->A32.as<float>(), w.ld, w.N, w.ld, w.zt32, w.ld, w.nr, w.W, w.ld, false);
    } else {
        launch_gemm_f64(c, c->A32.p, true, w.ld, w.N, w.ld, w.zt64, w.ld, w.nr, w.W, w.ld, false, 1.0);
        // FP64 remainders of the near entries
        hipLaunchKernelGGL(k_b_near, dim3((unsigned)ceil_div(w.N, 4)), dim3(256), 0, w.s, c->near_ptr.as<int64_t>(),
                           c->near_col.as<int32_t>(), c->near_val.as<double>(), w.N, w.zn64, w.nr, w.W, w.ld);
        BEM_CHECK_LAUNCH();
    }
    if (w.n > w.N) {
        // constraint rows (FP64, a few) need the FP64 vectors, vector-interleaved for the K-split row product
        if (f32) {
            hipLaunchKernelGGL(k_b_prep, dim3((unsigned)ceil_div(w.ld, 256), BR), dim3(256), 0, w.s, src, sstride,
                               w.nr, w.n, w.ld, d, (float*)nullptr, (double*)nullptr, w.zn64);
            BEM_CHECK_LAUNCH();
        }
        launch_gemm_rows(c, c->A64.as<double>(), w.ld, w.n - w.N, w.ld, w.zn64, w.nr, w.W + w.N, w.ld, false, 1.0);
    }
}

// blocks per dot product: about 2048 blocks per launch in total, each at least a few waves of work
int dot_split(const BW& w, int ndots) {
    const int64_t g = 2048 / std::max(ndots, 1);
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, w.G));
}

// norms of the nr vectors v[r * ld] into dst[r * dstride] (device); with `out`, also to the host
void norms(BW& w, const double* v, double* dst, int dstride, std::vector<double>* out) {
    const int G = dot_split(w, w.nr);
    hipLaunchKernelGGL(k_b_dots, dim3(G, 1, w.nr), dim3(256), 0, w.s, v, 1, w.ld, w.n, v, w.part, G);
    BEM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_b_reduce, dim3((unsigned)ceil_div(w.nr, 64)), dim3(64), 0, w.s, w.part, G, 1, 1, w.nr, dst,
                       dstride, (double*)nullptr, 0, 1);
    BEM_CHECK_LAUNCH();
    if (out) {
        if (dst != w.h) throw Error(BEM_ERR_INVALID, "norms to host need the h block");
        BEM_HIP(hipMemcpyAsync(w.host, w.h, sizeof(double) * w.nr * dstride, hipMemcpyDeviceToHost, w.s));
        BEM_HIP(hipStreamSynchronize(w.s));
        out->resize(w.nr);
        for (int r = 0; r < w.nr; ++r) (*out)[r] = w.host[r * dstride];
    }
}

// Batched GMRES on A x_r = b_r (x updated in place; initial guess as given).
// Returns the number of iterations; rel[r] gets the final relative residual.
int bgmres(BW& w, const double* B, double* X, double tol, int max_iter, bool exact_apply, std::vector<double>& rel,
           std::vector<double>& bnorm) {
    bem_ctx* c = w.c;
    const int nr = w.nr, m = w.m, m1 = w.m1, hs = m + 2;
    const double* d = c->diag.as<double>();
    std::vector<double> H((size_t)nr * (m + 1) * m), cs((size_t)nr * m), sn((size_t)nr * m), g((size_t)nr * (m + 1)),
        yv((size_t)nr * m1);
    std::vector<int32_t> jend(nr), stopped(nr), done(nr);
    int iters = 0;
    std::vector<double> beta(nr);
    for (;;) {
        // W = B - A X, its norms, then V[r][0] = W[r] / beta[r]
        apply(w, X, w.ld, nullptr, exact_apply);
        hipLaunchKernelGGL(k_b_residual, w.gv(), dim3(256), 0, w.s, B, w.W, w.ld, w.n, w.W);
        BEM_CHECK_LAUNCH();
        norms(w, w.W, w.h, hs, &beta);
        bool all_done = true;
        for (int r = 0; r < nr; ++r) {
            rel[r] = bnorm[r] > 0.0 ? beta[r] / bnorm[r] : 0.0;
            done[r] = (bnorm[r] == 0.0 || rel[r] <= tol);
            if (!done[r]) all_done = false;
        }
        if (all_done || iters >= max_iter) break;
        hipLaunchKernelGGL(k_b_scale, w.gv(), dim3(256), 0, w.s, w.W, w.ld, w.h, hs, w.n, w.V, (int64_t)m1 * w.ld);
        BEM_CHECK_LAUNCH();
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        for (int r = 0; r < nr; ++r) {
            g[(size_t)r * (m + 1)] = beta[r];
            jend[r] = 0;
            stopped[r] = done[r];
        }
        for (int j = 0; j < m; ++j) {
            KTimer tj(c, "bgmres_iter");
            // W = A (V[:, j] / d)
            apply(w, w.V + (int64_t)j * w.ld, (int64_t)m1 * w.ld, d, exact_apply);
            const int G = dot_split(w, (j + 1) * nr);
            for (int pass = 0; pass < 2; ++pass) {
                hipLaunchKernelGGL(k_b_dots, dim3(G, j + 1, nr), dim3(256), 0, w.s, w.V, m1, w.ld, w.n, w.W, w.part,
                                   G);
                BEM_CHECK_LAUNCH();
                hipLaunchKernelGGL(k_b_reduce, dim3((unsigned)ceil_div((j + 1) * nr, 64)), dim3(64), 0, w.s, w.part,
                                   G, m1, j + 1, nr, w.h, hs, w.Hcol, pass, 0);
                BEM_CHECK_LAUNCH();
                hipLaunchKernelGGL(k_b_orth, w.gv(), dim3(256), 0, w.s, w.V, m1, w.ld, w.n, j + 1, w.h, hs, w.W);
                BEM_CHECK_LAUNCH();
            }
            norms(w, w.W, w.Hcol + j + 1, hs, nullptr);
            hipLaunchKernelGGL(k_b_scale, w.gv(), dim3(256), 0, w.s, w.W, w.ld, w.Hcol + j + 1, hs, w.n,
                               w.V + (int64_t)(j + 1) * w.ld, (int64_t)m1 * w.ld);
            BEM_CHECK_LAUNCH();
            BEM_HIP(hipMemcpyAsync(w.host, w.Hcol, sizeof(double) * nr * hs, hipMemcpyDeviceToHost, w.s));
            BEM_HIP(hipStreamSynchronize(w.s));
            ++iters;
            bool all_stopped = true;
            for (int r = 0; r < nr; ++r) {
                if (stopped[r]) continue;
                double* Hr = H.data() + (size_t)r * (m + 1) * m;
                double* cr = cs.data() + (size_t)r * m;
                double* sr = sn.data() + (size_t)r * m;
                double* gr = g.data() + (size_t)r * (m + 1);
                for (int k = 0; k <= j + 1; ++k) Hr[(size_t)k * m + j] = w.host[r * hs + k];
                const double hn = w.host[r * hs + j + 1];
                for (int k = 0; k < j; ++k) {
                    const double a = Hr[(size_t)k * m + j], b = Hr[(size_t)(k + 1) * m + j];
                    Hr[(size_t)k * m + j] = cr[k] * a + sr[k] * b;
                    Hr[(size_t)(k + 1) * m + j] = -sr[k] * a + cr[k] * b;
                }
                const double a = Hr[(size_t)j * m + j], b = Hr[(size_t)(j + 1) * m + j];
                const double rr = std::sqrt(a * a + b * b);
                cr[j] = a / rr;
                sr[j] = b / rr;
                Hr[(size_t)j * m + j] = rr;
                Hr[(size_t)(j + 1) * m + j] = 0.0;
                gr[j + 1] = -sr[j] * gr[j];
                gr[j] = cr[j] * gr[j];
                jend[r] = j + 1;
                if (std::fabs(gr[j + 1]) / bnorm[r] <= tol || hn == 0.0) stopped[r] = 1;
                if (!stopped[r]) all_stopped = false;
            }
            if (all_stopped || iters >= max_iter) break;
        }
        // y_r from the triangular systems, then X_r += V_r y_r / d
        for (int r = 0; r < nr; ++r) {
            const double* Hr = H.data() + (size_t)r * (m + 1) * m;
            const double* gr = g.data() + (size_t)r * (m + 1);
            double* yr = yv.data() + (size_t)r * m1;
            for (int k = jend[r] - 1; k >= 0; --k) {
                double sacc = gr[k];
                for (int q = k + 1; q < jend[r]; ++q) sacc -= Hr[(size_t)k * m + q] * yr[q];
                yr[k] = sacc / Hr[(size_t)k * m + k];
            }
        }
        std::copy(yv.begin(), yv.end(), w.host);
        BEM_HIP(hipMemcpyAsync(w.y, w.host, sizeof(double) * nr * m1, hipMemcpyHostToDevice, w.s));
        BEM_HIP(hipMemcpyAsync(w.jend, jend.data(), sizeof(int32_t) * nr, hipMemcpyHostToDevice, w.s));
        hipLaunchKernelGGL(k_b_update_x, w.gv(), dim3(256), 0, w.s, w.V, m1, w.ld, w.n, w.y, w.jend, d, X);
        BEM_CHECK_LAUNCH();
        BEM_HIP(hipStreamSynchronize(w.s));   // host staging and jend are reused
    }
    return iters;
}

}  // namespace

// Y[r * n + i] = (A X)[r][i] for nr <= 64 vectors X[r * n + i], exact FP64-accumulated product of the
// assembled operator on the matrix cores (the mixed operator's FP32 entries are widened exactly).
void batched_apply_exact(bem_ctx* c, int nr, const double* X, double* Y) {
    BW w;
    w.c = c;
    w.nr = nr;
    w.n = c->n;
    w.N = c->nb;
    w.ld = c->ld;
    w.s = c->stream;
    const size_t ld = (size_t)w.ld;
    c->bg_W.alloc(sizeof(double) * 64 * ld * 3);
    c->bg_z.alloc(sizeof(float) * BR * ld + sizeof(double) * BR * ld * 2);
    w.W = c->bg_W.as<double>();
    w.zt32 = c->bg_z.as<float>();
    w.zt64 = reinterpret_cast<double*>(w.zt32 + BR * ld);
    w.zn64 = w.zt64 + BR * ld;
    apply(w, X, w.n, nullptr, true);
    for (int r = 0; r < nr; ++r)
        BEM_HIP(hipMemcpyAsync(Y + (int64_t)r * w.n, w.W + (int64_t)r * w.ld, sizeof(double) * w.n,
                               hipMemcpyDeviceToDevice, w.s));
}

// Solve for nr <= 64 right-hand sides B[r * ld + i] (device); X[r * ld + i] receives the solutions.
int gmres_solve_batched(bem_ctx* c, int nr, const double* B, double* X, double tol, int max_iter, int* iters_out,
                        double* relres_out, int* refinements_out) {
    BW w;
    w.c = c;
    w.nr = nr;
    w.m = c->opt.restart;
    w.m1 = w.m + 1;
    w.n = c->n;
    w.N = c->nb;
    w.ld = c->ld;
    w.s = c->stream;
    w.G = (int)std::min<int64_t>(ceil_div(w.n, 256), 128);
    const size_t ld = (size_t)w.ld;
    c->bg_V.alloc(sizeof(double) * nr * w.m1 * ld);
    c->bg_W.alloc(sizeof(double) * nr * ld * 3);
    c->bg_part.alloc(sizeof(double) * nr * w.m1 * w.G);
    c->bg_small.alloc(sizeof(double) * (size_t)nr * (w.m + 2) * 3 + sizeof(int32_t) * 64);
    c->bg_z.alloc(sizeof(float) * BR * ld + sizeof(double) * BR * ld * 2);
    c->host_stage.alloc(sizeof(double) * std::max<size_t>(4096, (size_t)nr * (w.m + 2) + 64));
    w.V = c->bg_V.as<double>();
    w.W = c->bg_W.as<double>();
    double* R = w.W + nr * ld;
    double* D = R + nr * ld;
    w.part = c->bg_part.as<double>();
    w.h = c->bg_small.as<double>();
    w.Hcol = w.h + (size_t)nr * (w.m + 2);
    w.y = w.Hcol + (size_t)nr * (w.m + 2);
    w.jend = reinterpret_cast<int32_t*>(w.y + (size_t)nr * (w.m + 2));
    w.zt32 = c->bg_z.as<float>();
    w.zt64 = reinterpret_cast<double*>(w.zt32 + BR * ld);
    w.zn64 = w.zt64 + BR * ld;
    w.host = c->host_stage.as<double>();
    // zero the Z buffers once: rows >= nr stay zero
    hipLaunchKernelGGL(k_b_fill, dim3((unsigned)ceil_div((int64_t)BR * ld * 2, 256)), dim3(256), 0, w.s, w.zt64,
                       (int64_t)BR * ld * 2, 0.0);
    BEM_CHECK_LAUNCH();
    std::vector<double> bnorm(nr), rel(nr);
    norms(w, B, w.h, w.m + 2, &bnorm);
    const int64_t total = (int64_t)nr * w.ld;
    hipLaunchKernelGGL(k_b_fill, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, w.s, X, total, 0.0);
    BEM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_b_fill, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, w.s, D, total, 0.0);
    BEM_CHECK_LAUNCH();
    int iters = 0, refinements = 0;
    if (c->opt.precision == BEM_FP64) {
        iters = bgmres(w, B, X, tol, max_iter, true, rel, bnorm);
    } else {
        // FP64 iterative refinement around the FP32-core inner solves
        for (;;) {
            apply(w, X, w.ld, nullptr, true);
            hipLaunchKernelGGL(k_b_residual, w.gv(), dim3(256), 0, w.s, B, w.W, w.ld, w.n, R);
            BEM_CHECK_LAUNCH();
            std::vector<double> rn;
            norms(w, R, w.h, w.m + 2, &rn);
            double worst = 0.0;
            for (int r = 0; r < nr; ++r) {
                rel[r] = bnorm[r] > 0.0 ? rn[r] / bnorm[r] : 0.0;
                worst = std::max(worst, rel[r]);
            }
            if (worst <= tol || iters >= max_iter || refinements >= 20) break;
            // inner solve of A D = R on the FP32 cores to the digits still missing, but not below 1e-4:
            // FP32-accumulated products over ~10^4 terms carry ~1e-6..1e-5 relative noise, and an
            // inner target near that floor stalls GMRES
            std::vector<double> rr(nr);
            const double inner = std::min(0.1, std::max(1e-4, 0.3 * tol / std::max(worst, 1e-300)));
            iters += bgmres(w, R, D, inner, max_iter - iters, false, rr, rn);
            hipLaunchKernelGGL(k_b_add, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, w.s, X, D, total);
            BEM_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_b_fill, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, w.s, D, total, 0.0);
            BEM_CHECK_LAUNCH();
            ++refinements;
        }
    }
    double worst = 0.0;
    for (int r = 0; r < nr; ++r) worst = std::max(worst, rel[r]);
    *iters_out = iters;
    *relres_out = worst;
    *refinements_out = refinements;
    return worst <= tol ? 0 : 1;
}

}  // namespace bem
