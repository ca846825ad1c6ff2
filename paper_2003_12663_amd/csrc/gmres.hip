// Restarted GMRES(m) with right diagonal (Jacobi) preconditioning (Sec. 5.2:
// GMRES with a diagonal preconditioner), classical Gram-Schmidt applied
// twice, Givens rotations and a zero initial guess.  The Krylov basis,
// the dot products and the updates live on the device in FP64; the host
// keeps the (m+1) x m Hessenberg matrix and the rotations and reads one
// column (j + 2 doubles) per iteration.  The mixed mode wraps GMRES on the
// mixed operator in FP64 iterative refinement.
#include <cmath>
#include <vector>

#include "bem_device.h"

namespace bem {
namespace {

// part[k * G + b] = sum over block b's slice of V[k][i] * w[i]
__global__ __launch_bounds__(256) void k_dots(const double* __restrict__ V, int64_t vstride, int64_t n,
                                              const double* __restrict__ w, double* __restrict__ part, int G) {
    const int k = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double s = 0.0;
    for (int64_t t = i; t < n; t += (int64_t)G * 256) s = fma(V[k * vstride + t], w[t], s);
    s = wave_sum(s);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[(int64_t)k * G + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// h[k] = sum_b part[k * G + b];  H[k] (+)= h[k].  One wave per k: lane l sums b = l, l + 64, ...
// in order, then a fixed-order butterfly (a thread summing all G partials in turn was a chain of
// G dependent adds behind their loads).
__global__ __launch_bounds__(64) void k_reduce_parts(const double* __restrict__ part, int G, int kcount,
                                                     double* __restrict__ h, double* __restrict__ Hcol, int accumulate,
                                                     int take_sqrt) {
    const int k = blockIdx.x;
    if (k >= kcount) return;
    double s = 0.0;
    for (int b = threadIdx.x; b < G; b += 64) s += part[(int64_t)k * G + b];
    s = wave_sum(s);
    if (threadIdx.x != 0) return;
    if (take_sqrt) s = sqrt(s);
    h[k] = s;
    if (Hcol) Hcol[k] = accumulate ? Hcol[k] + s : s;
}

// w -= sum_k h[k] V[k]
__global__ __launch_bounds__(256) void k_orth_update(const double* __restrict__ V, int64_t vstride, int64_t n,
                                                     int kcount, const double* __restrict__ h, double* __restrict__ w) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = w[i];
    for (int k = 0; k < kcount; ++k) s -= h[k] * V[k * vstride + i];
    w[i] = s;
}

// the second orthogonalisation pass with the block partials of |w|^2 of its output: one element
// per thread and block b covering [256 b, 256 b + 256), the partition k_dots takes when its G
// blocks cover n at one element per thread, so the norm is the same to the bit
__global__ __launch_bounds__(256) void k_orth_update_norm(const double* __restrict__ V, int64_t vstride, int64_t n,
                                                          int kcount, const double* __restrict__ h,
                                                          double* __restrict__ w, double* __restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double s = 0.0;
    if (i < n) {
        s = w[i];
        for (int k = 0; k < kcount; ++k) s -= h[k] * V[k * vstride + i];
        w[i] = s;
    }
    double q = fma(s, s, 0.0);
    q = wave_sum(q);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// the next Krylov vector out = w / (*nrm) and the product's input z = out / d of the next
// iteration (both left untouched if the norm is zero)
__global__ __launch_bounds__(256) void k_scale_div(const double* __restrict__ w, const double* __restrict__ nrm,
                                                   const double* __restrict__ d, int64_t n, double* __restrict__ out,
                                                   double* __restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double v = *nrm;
    if (i >= n || v == 0.0) return;
    const double o = w[i] / v;
    out[i] = o;
    z[i] = o / d[i];
}

// out = w / (*nrm) (left untouched if the norm is zero)
__global__ __launch_bounds__(256) void k_scale_by_norm(const double* __restrict__ w, const double* __restrict__ nrm,
                                                       int64_t n, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double v = *nrm;
    if (i >= n || v == 0.0) return;
    out[i] = w[i] / v;
}

__global__ __launch_bounds__(256) void k_div_diag(const double* __restrict__ v, const double* __restrict__ d, int64_t n,
                                                  double* __restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) z[i] = v[i] / d[i];
}

// r = b - Ax
__global__ __launch_bounds__(256) void k_residual(const double* __restrict__ b, const double* __restrict__ Ax, int64_t n,
                                                  double* __restrict__ r) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) r[i] = b[i] - Ax[i];
}

// x += (sum_k y[k] V[k]) / d
__global__ __launch_bounds__(256) void k_update_x(const double* __restrict__ V, int64_t vstride, int64_t n, int kcount,
                                                  const double* __restrict__ y, const double* __restrict__ d,
                                                  double* __restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < kcount; ++k) s = fma(y[k], V[k * vstride + i], s);
    x[i] += s / d[i];
}

__global__ __launch_bounds__(256) void k_fill(double* __restrict__ x, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = v;
}

__global__ __launch_bounds__(256) void k_axpy(double* __restrict__ x, const double* __restrict__ d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] += d[i];
}

__global__ __launch_bounds__(256) void k_copy(const double* __restrict__ a, int64_t n, double* __restrict__ b) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) b[i] = a[i];
}

struct Work {
    bem_ctx* c;
    int64_t n, vs;   // length and padded stride of Krylov vectors
    int m, G;
    double *V, *w, *z, *h, *part, *Hcol, *misc;
    double* host;    // pinned host staging
    hipStream_t s;
    bool transpose = false;   // solve with A^T (same Jacobi diagonal)
    dim3 g1() const { return dim3((unsigned)ceil_div(n, 256)); }
};

// squared-norm -> sqrt into dst[0] (device); also returns it on the host if asked
void device_norm(Work& W, const double* v, double* dst) {
    hipLaunchKernelGGL(k_dots, dim3(W.G, 1), dim3(256), 0, W.s, v, (int64_t)0, W.n, v, W.part, W.G);
    BEM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(64), 0, W.s, W.part, W.G, 1, dst, (double*)nullptr, 0, 1);
    BEM_CHECK_LAUNCH();
}

double host_norm(Work& W, const double* v) {
    device_norm(W, v, W.misc);
    BEM_HIP(hipMemcpyAsync(W.host, W.misc, sizeof(double), hipMemcpyDeviceToHost, W.s));
    BEM_HIP(hipStreamSynchronize(W.s));
    return W.host[0];
}

// One GMRES solve of A x = b (x overwritten; zero initial guess unless keep_x).
int gmres_core(Work& W, const double* b, double* x, double tol, int max_iter, int* iters_out, double* relres_out,
               bool keep_x) {
    bem_ctx* c = W.c;
    const int64_t n = W.n;
    const int m = W.m;
    const double* d = c->diag.as<double>();
    if (!keep_x) {
        hipLaunchKernelGGL(k_fill, W.g1(), dim3(256), 0, W.s, x, n, 0.0);
        BEM_CHECK_LAUNCH();
    }
    const double bnorm = host_norm(W, b);
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m + 1);
    int iters = 0;
    double relres = 0.0;
    bool converged = false;
    if (bnorm == 0.0) {
        hipLaunchKernelGGL(k_fill, W.g1(), dim3(256), 0, W.s, x, n, 0.0);
        BEM_CHECK_LAUNCH();
        *iters_out = 0;
        *relres_out = 0.0;
        return 0;
    }
    for (;;) {
        // r = b - A x into V[0]
        if (W.transpose)
            launch_matvec_t(c, x, W.w, W.s);
        else
            launch_matvec(c, x, W.w, W.s);
        hipLaunchKernelGGL(k_residual, W.g1(), dim3(256), 0, W.s, b, W.w, n, W.V);
        BEM_CHECK_LAUNCH();
        const double beta = host_norm(W, W.V);
        relres = beta / bnorm;
        if (relres <= tol) {
            converged = true;
            break;
        }
        if (iters >= max_iter) break;
        hipLaunchKernelGGL(k_scale_by_norm, W.g1(), dim3(256), 0, W.s, W.V, W.misc, n, W.V);
        BEM_CHECK_LAUNCH();
        std::fill(g.begin(), g.end(), 0.0);
        std::fill(H.begin(), H.end(), 0.0);
        g[0] = beta;
        int jend = 0;
        // the norm's block partials from the second orthogonalisation pass and the next product's
        // input from the scaling, when the dot products' blocks cover w at one element per thread
        const bool fused = W.G == ceil_div(n, 256);
        for (int j = 0; j < m; ++j) {
            KTimer tj(c, "gmres_iter");
            double* Vj = W.V + (int64_t)j * W.vs;
            if (j == 0 || !fused) {   // else the scaling that made V[j] also wrote z
                hipLaunchKernelGGL(k_div_diag, W.g1(), dim3(256), 0, W.s, Vj, d, n, W.z);
                BEM_CHECK_LAUNCH();
            }
            if (W.transpose)
                launch_matvec_t(c, W.z, W.w, W.s);
            else
                launch_matvec(c, W.z, W.w, W.s);
            {
                KTimer to(c, "gmres_ortho");
                for (int pass = 0; pass < 2; ++pass) {
                    hipLaunchKernelGGL(k_dots, dim3(W.G, j + 1), dim3(256), 0, W.s, W.V, W.vs, n, W.w, W.part, W.G);
                    BEM_CHECK_LAUNCH();
                    hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)(j + 1)), dim3(64), 0, W.s, W.part,
                                       W.G, j + 1, W.h, W.Hcol, pass, 0);
                    BEM_CHECK_LAUNCH();
                    if (fused && pass == 1)
                        hipLaunchKernelGGL(k_orth_update_norm, W.g1(), dim3(256), 0, W.s, W.V, W.vs, n, j + 1, W.h,
                                           W.w, W.part);
                    else
                        hipLaunchKernelGGL(k_orth_update, W.g1(), dim3(256), 0, W.s, W.V, W.vs, n, j + 1, W.h, W.w);
                    BEM_CHECK_LAUNCH();
                }
                if (fused) {
                    hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(64), 0, W.s, W.part, W.G, 1, W.Hcol + j + 1,
                                       (double*)nullptr, 0, 1);
                    BEM_CHECK_LAUNCH();
                } else {
                    device_norm(W, W.w, W.Hcol + j + 1);
                }
                if (fused && j + 1 < m)
                    hipLaunchKernelGGL(k_scale_div, W.g1(), dim3(256), 0, W.s, W.w, W.Hcol + j + 1, d, n,
                                       W.V + (int64_t)(j + 1) * W.vs, W.z);
                else
                    hipLaunchKernelGGL(k_scale_by_norm, W.g1(), dim3(256), 0, W.s, W.w, W.Hcol + j + 1, n,
                                       W.V + (int64_t)(j + 1) * W.vs);
                BEM_CHECK_LAUNCH();
            }
            BEM_HIP(hipMemcpyAsync(W.host, W.Hcol, sizeof(double) * (j + 2), hipMemcpyDeviceToHost, W.s));
            BEM_HIP(hipStreamSynchronize(W.s));
            for (int k = 0; k <= j + 1; ++k) H[(size_t)k * m + j] = W.host[k];
            const double hn = W.host[j + 1];
            for (int k = 0; k < j; ++k) {
                const double a = H[(size_t)k * m + j], bb = H[(size_t)(k + 1) * m + j];
                H[(size_t)k * m + j] = cs[k] * a + sn[k] * bb;
                H[(size_t)(k + 1) * m + j] = -sn[k] * a + cs[k] * bb;
            }
            const double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
            const double r = std::sqrt(a * a + bb * bb);
            cs[j] = a / r;
            sn[j] = bb / r;
            H[(size_t)j * m + j] = r;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++iters;
            jend = j + 1;
            if (std::fabs(g[j + 1]) / bnorm <= tol || iters >= max_iter || hn == 0.0) break;
        }
        for (int k = jend - 1; k >= 0; --k) {
            double sacc = g[k];
            for (int q = k + 1; q < jend; ++q) sacc -= H[(size_t)k * m + q] * y[q];
            y[k] = sacc / H[(size_t)k * m + k];
        }
        for (int k = 0; k < jend; ++k) W.host[k] = y[k];
        BEM_HIP(hipMemcpyAsync(W.h, W.host, sizeof(double) * jend, hipMemcpyHostToDevice, W.s));
        hipLaunchKernelGGL(k_update_x, W.g1(), dim3(256), 0, W.s, W.V, W.vs, n, jend, W.h, d, x);
        BEM_CHECK_LAUNCH();
        // the pinned staging buffer is reused right away: wait for the copy
        BEM_HIP(hipStreamSynchronize(W.s));
    }
    *iters_out = iters;
    *relres_out = relres;
    return converged ? 0 : 1;
}

}  // namespace

static void setup_work(bem_ctx* c, Work& W) {
    W.c = c;
    W.n = c->n;
    W.vs = c->ld;
    W.m = c->opt.restart;
    W.G = (int)std::min<int64_t>(ceil_div(c->n, 256), 1024);
    W.s = c->stream;
    c->gm_V.alloc(sizeof(double) * (size_t)W.vs * (W.m + 1));
    c->gm_w.alloc(sizeof(double) * W.vs);
    c->gm_z.alloc(sizeof(double) * W.vs);
    c->gm_h.alloc(sizeof(double) * (W.m + 2) * 2);
    c->gm_part.alloc(sizeof(double) * (size_t)W.G * (W.m + 1));
    c->gm_r.alloc(sizeof(double) * W.vs * 3);
    W.V = c->gm_V.as<double>();
    W.w = c->gm_w.as<double>();
    W.z = c->gm_z.as<double>();
    W.h = c->gm_h.as<double>();
    W.Hcol = W.h + (W.m + 2);
    W.part = c->gm_part.as<double>();
    W.misc = c->gm_r.as<double>() + 2 * W.vs;
    W.host = c->host_stage.as<double>();
}

// A^T x = b (FP64 operator only): the adjoint solve of the gradient.
int gmres_solve_t(bem_ctx* c, const double* b, double* x, double tol, int max_iter, int* iters, double* relres) {
    if (c->opt.precision != BEM_FP64) throw Error(BEM_ERR_INVALID, "the adjoint solve needs precision FP64");
    Work W;
    setup_work(c, W);
    W.transpose = true;
    return gmres_core(W, b, x, tol, max_iter, iters, relres, false);
}

int gmres_solve(bem_ctx* c, const double* b, double* x, double tol, int max_iter, int* iters, double* relres,
                int* refinements_out) {
    *refinements_out = 0;
    Work W;
    setup_work(c, W);
    if (c->opt.precision == BEM_FP64) return gmres_core(W, b, x, tol, max_iter, iters, relres, false);

    // Mixed mode: FP64 iterative refinement around GMRES on the mixed operator.
    double* r = c->gm_r.as<double>();
    double* dx = r + W.vs;
    hipLaunchKernelGGL(k_fill, W.g1(), dim3(256), 0, W.s, x, W.n, 0.0);
    BEM_CHECK_LAUNCH();
    const double bnorm = host_norm(W, b);
    int total = 0, refinements = 0;
    double rel = 0.0;
    if (bnorm == 0.0) {
        *iters = 0;
        *relres = 0.0;
        return 0;
    }
    hipLaunchKernelGGL(k_copy, W.g1(), dim3(256), 0, W.s, b, W.n, r);
    BEM_CHECK_LAUNCH();
    for (;;) {
        rel = host_norm(W, r) / bnorm;
        if (rel <= tol || total >= max_iter || refinements >= 50) break;
        int it = 0;
        double rr = 0.0;
        const double inner = std::max(1e-4, 0.5 * tol / rel);
        gmres_core(W, r, dx, inner, max_iter - total, &it, &rr, false);
        total += it;
        ++refinements;
        hipLaunchKernelGGL(k_axpy, W.g1(), dim3(256), 0, W.s, x, dx, W.n);
        BEM_CHECK_LAUNCH();
        launch_matvec(c, x, W.w, W.s);
        hipLaunchKernelGGL(k_residual, W.g1(), dim3(256), 0, W.s, b, W.w, W.n, r);
        BEM_CHECK_LAUNCH();
    }
    *iters = total;
    *relres = rel;
    *refinements_out = refinements;
    return rel <= tol ? 0 : 1;
}

}  // namespace bem
