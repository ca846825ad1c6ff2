// Dense matrix-vector products of the Krylov solver (Sec. 3: Krylov methods
// need only products with the system matrix).  HBM-bound: every launch
// streams the whole row-major matrix once.
//
// k_gemv64: a 256-thread block owns RB consecutive rows; each thread reads
// 16-byte column pairs of all RB rows per step, so one x load feeds RB
// multiply-adds and each row segment read by the block is 4 KB contiguous.
// k_gemv32: the same for the FP32 matrix of the mixed mode (float4 loads,
// FP64 accumulation), with the FP64 remainders of the near entries (near list
// of the block's rows) added by the same block.
// k_gemvT64: y = A^T x, column pairs per thread over a slab of rows; slabs
// are summed by a second kernel in a fixed order (deterministic).
#include "bem_device.h"

#include <mutex>
#include <string>

namespace bem {
namespace {


template <int RB>
__device__ __forceinline__ void block_reduce_rows(double (&acc)[RB], double* __restrict__ y, int64_t row0,
                                                  int64_t n_rows) {
    __shared__ double red[4][RB];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const double s = wave_sum(acc[r]);
        if (lane == 0) red[wv][r] = s;
    }
    __syncthreads();
    if (threadIdx.x < RB && row0 + threadIdx.x < n_rows) {
        const int r = threadIdx.x;
        y[row0 + r] = (red[0][r] + red[1][r]) + (red[2][r] + red[3][r]);
    }
}

template <int RB>
__global__ __launch_bounds__(256) void k_gemv64(const double* __restrict__ A, int64_t ld, int64_t n_rows,
                                                int64_t n_cols, const double* __restrict__ x,
                                                double* __restrict__ y) {
    const int64_t row0 = (int64_t)blockIdx.x * RB;
    double acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] = 0.0;
    const double* Arow[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int64_t rr = row0 + r < n_rows ? row0 + r : n_rows - 1;
        Arow[r] = A + rr * ld;
    }
    const int64_t n2 = n_cols >> 1;
    int64_t c = threadIdx.x;
    for (; c + 256 < n2; c += 512) {
        const d2v x0 = reinterpret_cast<const d2v*>(x)[c];
        const d2v x1 = reinterpret_cast<const d2v*>(x)[c + 256];
        d2v a0[RB], a1[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            a0[r] = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(Arow[r]) + c);
            a1[r] = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(Arow[r]) + c + 256);
        }
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            acc[r] = fma(a0[r].x, x0.x, acc[r]);
            acc[r] = fma(a0[r].y, x0.y, acc[r]);
            acc[r] = fma(a1[r].x, x1.x, acc[r]);
            acc[r] = fma(a1[r].y, x1.y, acc[r]);
        }
    }
    for (; c < n2; c += 256) {
        const d2v x0 = reinterpret_cast<const d2v*>(x)[c];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const d2v a0 = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(Arow[r]) + c);
            acc[r] = fma(a0.x, x0.x, acc[r]);
            acc[r] = fma(a0.y, x0.y, acc[r]);
        }
    }
    if ((n_cols & 1) && threadIdx.x == 0) {
        const double xl = x[n_cols - 1];
#pragma unroll
        for (int r = 0; r < RB; ++r) acc[r] = fma(Arow[r][n_cols - 1], xl, acc[r]);
    }
    block_reduce_rows<RB>(acc, y, row0, n_rows);
}

// rows < N of the mixed operator: FP32 far part + FP64 near CSR
template <int RB>
__global__ __launch_bounds__(256) void k_gemv32(const float* __restrict__ A, int64_t ld, int64_t n_rows, int64_t n_cols,
                                                const double* __restrict__ x, const int64_t* __restrict__ nptr,
                                                const int32_t* __restrict__ ncol, const double* __restrict__ nval,
                                                double* __restrict__ y) {
    const int64_t row0 = (int64_t)blockIdx.x * RB;
    double acc[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] = 0.0;
    const float* Arow[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        const int64_t rr = row0 + r < n_rows ? row0 + r : n_rows - 1;
        Arow[r] = A + rr * ld;
    }
    const int64_t n4 = n_cols >> 2;
    for (int64_t c = threadIdx.x; c < n4; c += 256) {
        const d2v xa = reinterpret_cast<const d2v*>(x)[2 * c];
        const d2v xb = reinterpret_cast<const d2v*>(x)[2 * c + 1];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const f4v a = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(Arow[r]) + c);
            acc[r] = fma((double)a.x, xa.x, acc[r]);
            acc[r] = fma((double)a.y, xa.y, acc[r]);
            acc[r] = fma((double)a.z, xb.x, acc[r]);
            acc[r] = fma((double)a.w, xb.y, acc[r]);
        }
    }
    for (int64_t c = 4 * n4 + threadIdx.x; c < n_cols; c += 256) {
        const double xc = x[c];
#pragma unroll
        for (int r = 0; r < RB; ++r) acc[r] = fma((double)Arow[r][c], xc, acc[r]);
    }
    // near entries of this block's rows
    const int64_t rend = row0 + RB < n_rows ? row0 + RB : n_rows;
    const int64_t e0 = nptr[row0], e1 = nptr[rend];
#pragma unroll
    for (int r = 0; r < RB; ++r) {
        if (row0 + r >= rend) break;
        const int64_t b0 = nptr[row0 + r], b1 = nptr[row0 + r + 1];
        for (int64_t e = b0 + threadIdx.x; e < b1; e += 256) acc[r] = fma(nval[e], x[ncol[e]], acc[r]);
    }
    (void)e0;
    (void)e1;
    block_reduce_rows<RB>(acc, y, row0, n_rows);
}

constexpr int GT_SLABS = 64;

__global__ __launch_bounds__(256) void k_gemvT64_part(const double* __restrict__ A, int64_t ld, int64_t n_rows,
                                                      int64_t n_cols, const double* __restrict__ x,
                                                      double* __restrict__ part) {
    const int64_t c2 = (int64_t)blockIdx.x * 256 + threadIdx.x;   // column pair index
    const int64_t slab = blockIdx.y;
    const int64_t per = (n_rows + GT_SLABS - 1) / GT_SLABS;
    const int64_t r0 = slab * per, r1 = r0 + per < n_rows ? r0 + per : n_rows;
    const int64_t c = 2 * c2;
    if (c >= n_cols) return;
    double s0 = 0.0, s1 = 0.0;
    if (c + 1 < n_cols) {
        for (int64_t r = r0; r < r1; ++r) {
            const d2v a = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(A + r * ld) + c2);
            const double xr = x[r];
            s0 = fma(a.x, xr, s0);
            s1 = fma(a.y, xr, s1);
        }
        part[slab * n_cols + c] = s0;
        part[slab * n_cols + c + 1] = s1;
    } else {
        for (int64_t r = r0; r < r1; ++r) s0 = fma(A[r * ld + c], x[r], s0);
        part[slab * n_cols + c] = s0;
    }
}

__global__ __launch_bounds__(256) void k_sum_slabs(const double* __restrict__ part, int64_t n_cols, int slabs,
                                                   double* __restrict__ y) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n_cols) return;
    double s = 0.0;
    for (int k = 0; k < slabs; ++k) s += part[k * n_cols + c];
    y[c] = s;
}

}  // namespace

template <int RB>
void matvec_rb(bem_ctx* c, const double* x, double* y, hipStream_t s) {
    const int64_t n = c->n, N = c->nb, ld = c->ld;
    if (c->opt.precision == BEM_FP64) {
        hipLaunchKernelGGL((k_gemv64<RB>), dim3((unsigned)ceil_div(n, RB)), dim3(256), 0, s, c->A64.as<double>(), ld,
                           n, n, x, y);
        BEM_CHECK_LAUNCH();
        return;
    }
    hipLaunchKernelGGL((k_gemv32<RB>), dim3((unsigned)ceil_div(N, RB)), dim3(256), 0, s, c->A32.as<float>(), ld, N, n,
                       x, c->near_ptr.as<int64_t>(), c->near_col.as<int32_t>(), c->near_val.as<double>(), y);
    BEM_CHECK_LAUNCH();
    if (n > N) {
        hipLaunchKernelGGL((k_gemv64<RB>), dim3((unsigned)ceil_div(n - N, RB)), dim3(256), 0, s, c->A64.as<double>(),
                           ld, n - N, n, x, y + N);
        BEM_CHECK_LAUNCH();
    }
}

// y = A x for the assembled operator (FP64 or mixed); rows per block from the tuning
void launch_matvec(bem_ctx* c, const double* x, double* y, hipStream_t s) {
    if (c->hm) {
        hmatrix_matvec(c, x, y, s);
        return;
    }
    KTimer t(c, "gemv");
    switch (c->tune_gemv_rows) {
        case 2: matvec_rb<2>(c, x, y, s); break;
        case 8: matvec_rb<8>(c, x, y, s); break;
        case 16: matvec_rb<16>(c, x, y, s); break;
        default: matvec_rb<4>(c, x, y, s); break;
    }
}

// y = A^T x with the slab partials in part (GT_SLABS x n doubles, every entry written before it is
// read).  FP64 mode only: the mixed mode keeps no FP64 copy of the far entries.
void matvec_t_into(bem_ctx* c, const double* x, double* y, double* part, hipStream_t s) {
    const int64_t n = c->n;
    if (c->opt.precision != BEM_FP64) throw Error(BEM_ERR_INVALID, "transpose matvec needs precision FP64");
    dim3 grid((unsigned)ceil_div(ceil_div(n, 2), 256), GT_SLABS);
    hipLaunchKernelGGL(k_gemvT64_part, grid, dim3(256), 0, s, c->A64.as<double>(), c->ld, n, n, x, part);
    BEM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_sum_slabs, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, part, n, GT_SLABS, y);
    BEM_CHECK_LAUNCH();
}

void launch_matvec_t(bem_ctx* c, const double* x, double* y, hipStream_t s) {
    if (c->hm) throw Error(BEM_ERR_INVALID, "the compressed operator has no transpose product");
    KTimer t(c, "gemvT");
    if (c->opt.precision != BEM_FP64) throw Error(BEM_ERR_INVALID, "transpose matvec needs precision FP64");
    c->ev_tmp.alloc(sizeof(double) * GT_SLABS * c->n);
    matvec_t_into(c, x, y, c->ev_tmp.as<double>(), s);
}

// ---- the product without allocation ---------------------------------------------------------
// For callers that cannot allocate device memory (code under stream capture, serving loops): the
// staging of one vector pair and the transposed product's slab partials live in one file-scope
// device array, 66 x 65536 doubles (33 MiB), which every GPU the library runs on holds until the
// process ends.  Host code never passes the array's name (a host-side stand-in) to a kernel or a
// copy: it uses the device address that hipGetSymbolAddress returns for the current device, looked
// up once per device when a context is created.  Every call on one GPU shares that GPU's array,
// so calls that overlap on one GPU race.
constexpr int64_t NOALLOC_MAX_N = 65536;
constexpr int64_t NOALLOC_DOUBLES = (2 + GT_SLABS) * NOALLOC_MAX_N;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {
constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[NOALLOC_MAX_DEV] = {};
}  // namespace

// Looks up (once per device; the device must be current) the device address of this device's
// copy of the array.
void noalloc_scratch_init(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEV) throw Error(BEM_ERR_INVALID, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        throw Error(BEM_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<double*>(ptr);
}

// y[r] = A x[r] (transpose 0) or A^T x[r] (transpose 1) for r < nrhs, vector by vector through the
// staging in the device array; no allocation.  Same kernels as the allocating product of one vector.
void matvec_noalloc(bem_ctx* c, int32_t nrhs, const double* x, double* y, int transpose) {
    const int64_t n = c->n, ld = c->ld;
    if (n > NOALLOC_MAX_N || ld > NOALLOC_MAX_N)
        throw Error(BEM_ERR_INVALID, "bem_matvec_noalloc: at most 65536 unknowns (the fixed work array)");
    if (transpose && c->opt.precision != BEM_FP64)
        throw Error(BEM_ERR_INVALID, "transpose matvec needs precision FP64");
    if (!c->assembled) throw Error(BEM_ERR_STATE, "bem_assemble has not run");
    if (c->hm) throw Error(BEM_ERR_INVALID, "bem_matvec_noalloc needs the dense operator");
    double* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (c->device >= 0 && c->device < NOALLOC_MAX_DEV) base = g_scratch_ptr[c->device];
    }
    if (!base) throw Error(BEM_ERR_STATE, "bem_matvec_noalloc: work array of this device not set up");
    double* xa = base;
    double* ya = base + NOALLOC_MAX_N;
    double* part = base + 2 * NOALLOC_MAX_N;
    for (int32_t r = 0; r < nrhs; ++r) {
        BEM_HIP(hipMemcpyAsync(xa, x + (int64_t)r * n, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
        if (transpose) {
            matvec_t_into(c, xa, ya, part, c->stream);
        } else {
            switch (c->tune_gemv_rows) {
                case 2: matvec_rb<2>(c, xa, ya, c->stream); break;
                case 8: matvec_rb<8>(c, xa, ya, c->stream); break;
                case 16: matvec_rb<16>(c, xa, ya, c->stream); break;
                default: matvec_rb<4>(c, xa, ya, c->stream); break;
            }
        }
        BEM_HIP(hipMemcpyAsync(y + (int64_t)r * n, ya, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    }
}

}  // namespace bem
