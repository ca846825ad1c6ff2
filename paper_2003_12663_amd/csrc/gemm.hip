// Dense products with many right-hand sides: Y = A Z for up to 64 load cases
// at once (the matvec of a batched Krylov solve), on the MFMA matrix cores.
//
// A is the row-major system matrix (FP32 far matrix of the mixed mode, or the
// FP64 matrix); Z holds the 64 input vectors.  Each A row is streamed from
// HBM once per product and multiplied with all 64 vectors, so the product is
// bound by the matrix cores rather than by HBM (2 flop x 64 per A entry).
//
//  k_gemm_f32: v_mfma_f32_32x32x2f32, FP32 operands and FP32 accumulation
//     within a K range; A and Z tiles staged in LDS (see the kernel).
//  k_gemm_f64: v_mfma_f64_16x16x4f64, FP64 accumulation, A either FP64 or
//     FP32 widened exactly (FP32 values are FP64 numbers), so for the FP32
//     far matrix it is the exact FP64-accumulated product of the mixed
//     operator.  A block owns 64 rows x 64 columns over one of 8 K ranges,
//     the K range fixed per XCD (see the kernel).
//  k_rows_part: a few FP64 rows (constraint rows of floating bodies) times
//     the vectors, K split over hundreds of blocks.
// Operand k-order: lane (r, h) of a 32-lane half feeds A[row r][k0 + 16h + s]
// and Z[col][k0 + 16h + s] at step s; any order of k that is the same for both
// operands gives the same sum.
// Z layout: Zt[col][k] (vector-major), row stride ldz >= K, zero beyond the
// true length; K is a multiple of 32 (rows of A are padded with zeros).
#include <algorithm>

#include "bem_device.h"

namespace bem {
namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef double d4v __attribute__((ext_vector_type(4)));

// FP32 product, LDS-staged: a block owns 128 rows (32 per wave) x 64 columns over
// one K range (blockIdx.y); per step it stages a 128 x 32 tile of A and a
// 64 x 32 tile of Z in LDS with row-contiguous 16-byte loads (8 lanes cover a
// 128-byte row segment), prefetching the next step into registers, and each
// wave runs 32 MFMAs from LDS.  Partial tiles of the K ranges go to Ypart
// [ks][col][row] and k_gemm_f32_sum adds them in K-range order.
constexpr int G32_ROWS = 128, G32_KC = 32, G32_PAD = 36;

__global__ __launch_bounds__(256, 2) void k_gemm_f32(const float* __restrict__ A, int64_t lda, int64_t M, int64_t K,
                                                    const float* __restrict__ Zt, int64_t ldz, int64_t kb_per,
                                                    float* __restrict__ Ypart) {
    __shared__ __attribute__((aligned(16))) float As[G32_ROWS][G32_PAD];
    __shared__ __attribute__((aligned(16))) float Bs[64][G32_PAD];
    __shared__ float Ct[64][G32_ROWS + 1];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r = lane & 31, h = lane >> 5;
    const int64_t row0 = (int64_t)blockIdx.x * G32_ROWS;
    const int64_t kblocks = K / G32_KC;
    const int64_t kb0 = (int64_t)blockIdx.y * kb_per;
    const int64_t kb1 = kb0 + kb_per < kblocks ? kb0 + kb_per : kblocks;
    // this thread's staging slots: A rows (tid >> 3) + 32 i, Z column (tid >> 3) + 32 i, 16 bytes at 4 (tid & 7)
    const int sr = tid >> 3, sc = 4 * (tid & 7);
    const float* Ap[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int64_t rr = row0 + sr + 32 * i;
        if (rr >= M) rr = M - 1;   // rows past the end are read from the last row and never stored
        Ap[i] = A + rr * lda + sc;
    }
    const float* Zp0 = Zt + (int64_t)sr * ldz + sc;
    const float* Zp1 = Zt + (int64_t)(sr + 32) * ldz + sc;
    f16v acc0 = {0}, acc1 = {0};
    f4v ra[4], rz[2];
    if (kb0 < kb1) {
        const int64_t k = kb0 * G32_KC;
#pragma unroll
        for (int i = 0; i < 4; ++i) ra[i] = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(Ap[i] + k));
        rz[0] = *reinterpret_cast<const f4v*>(Zp0 + k);
        rz[1] = *reinterpret_cast<const f4v*>(Zp1 + k);
    }
    for (int64_t kb = kb0; kb < kb1; ++kb) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i) *reinterpret_cast<f4v*>(&As[sr + 32 * i][sc]) = ra[i];
        *reinterpret_cast<f4v*>(&Bs[sr][sc]) = rz[0];
        *reinterpret_cast<f4v*>(&Bs[sr + 32][sc]) = rz[1];
        __syncthreads();
        if (kb + 1 < kb1) {
            const int64_t k = (kb + 1) * G32_KC;
#pragma unroll
            for (int i = 0; i < 4; ++i) ra[i] = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(Ap[i] + k));
            rz[0] = *reinterpret_cast<const f4v*>(Zp0 + k);
            rz[1] = *reinterpret_cast<const f4v*>(Zp1 + k);
        }
        f4v a[4], b0[4], b1[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a[q] = *reinterpret_cast<const f4v*>(&As[32 * wv + r][16 * h + 4 * q]);
            b0[q] = *reinterpret_cast<const f4v*>(&Bs[r][16 * h + 4 * q]);
            b1[q] = *reinterpret_cast<const f4v*>(&Bs[32 + r][16 * h + 4 * q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q][e], b0[q][e], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a[q][e], b1[q][e], acc1, 0, 0, 0);
            }
        }
    }
    // accumulator element v of lane (r, h): row 8 (v / 4) + 4 h + v % 4 (+32 wv), column r (+32)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int row = 32 * wv + 8 * (v >> 2) + 4 * h + (v & 3);
        Ct[r][row] = acc0[v];
        Ct[32 + r][row] = acc1[v];
    }
    __syncthreads();
    float* out = Ypart + (int64_t)blockIdx.y * 64 * M;
    for (int e = tid; e < 64 * G32_ROWS; e += 256) {
        const int col = e / G32_ROWS, row = e % G32_ROWS;
        const int64_t i = row0 + row;
        if (i < M) out[(int64_t)col * M + i] = Ct[col][row];
    }
}

// Y[col][i] (+)= sum over the K ranges of Ypart[ks][col][i] (FP64 sum, fixed order)
__global__ __launch_bounds__(256) void k_gemm_f32_sum(const float* __restrict__ Ypart, int KS, int64_t M, int ncols,
                                                      double* __restrict__ Y, int64_t ldy, int accumulate) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int col = blockIdx.y;
    if (i >= M || col >= ncols) return;
    double s = 0.0;
    for (int k = 0; k < KS; ++k) s += (double)Ypart[((int64_t)k * 64 + col) * M + i];
    double* y = Y + (int64_t)col * ldy + i;
    *y = accumulate ? *y + s : s;
}

// FP64-accumulated product on v_mfma_f64_16x16x4f64.  A block owns 64 rows (16 per wave) x 64
// columns over one of GD_KS ranges of K.  Workgroups are dealt to the 8 XCDs round-robin, so with
// the K range taken as blockIdx % GD_KS every block of one XCD works one K range: that range's
// slice of Z (64 x K/8 doubles, 1.3 MB at 20k unknowns) stays in the XCD's L2 for all row blocks,
// while each A entry is read from HBM once.  Per 32-wide k step the block stages a 64 x 32 tile of
// A (FP32 entries widened) and a 64 x 32 tile of Z in LDS with row-contiguous loads (4 threads
// cover a 256-byte row segment), the next step's tiles prefetched into registers; each wave then
// runs 32 MFMAs with its operands read from LDS (a lane takes 4 consecutive k of its A row and of
// 4 Z columns per 16 k).  The 64 x 64 partial tile is transposed through the same LDS and leaves
// as column segments of 64 rows; k_gemm_f64_sum adds the K ranges in order.
constexpr int GD_ROWS = 64, GD_KS = 8, GD_KC = 32, GD_PAD = 34;

template <typename TA>
__global__ __launch_bounds__(256) void k_gemm_f64(const TA* __restrict__ A, int64_t lda, int64_t M, int64_t K,
                                                  const double* __restrict__ Zt, int64_t ldz, int64_t kb_per, int KS,
                                                  double* __restrict__ Ypart) {
    // A and Z tiles, reused after the loop for the 64 x 65 output tile (4160 <= 4352 doubles)
    __shared__ __attribute__((aligned(16))) double smem[2 * 64 * GD_PAD];
    double(*As)[GD_PAD] = reinterpret_cast<double(*)[GD_PAD]>(smem);
    double(*Bs)[GD_PAD] = reinterpret_cast<double(*)[GD_PAD]>(smem + 64 * GD_PAD);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int r = lane & 15, q4 = lane >> 4;   // row (A) / column (Z) within 16, k group 0..3
    const int64_t ks = blockIdx.x % KS, rb = blockIdx.x / KS;
    const int64_t row0 = rb * GD_ROWS;
    const int64_t kblocks = K / GD_KC;
    const int64_t kb0 = ks * kb_per, kb1 = kb0 + kb_per < kblocks ? kb0 + kb_per : kblocks;
    // this thread's staging slot: A row / Z column sr, 8 doubles from sc
    const int sr = tid >> 2, sc = 8 * (tid & 3);
    const int64_t ar = row0 + sr < M ? row0 + sr : M - 1;   // rows past M: read, never stored
    const TA* __restrict__ Ap = A + ar * lda + sc;
    const double* __restrict__ Zp = Zt + (int64_t)sr * ldz + sc;
    double ra[8], rz[8];
    auto load = [&](int64_t k) {
        if (sizeof(TA) == 4) {
            const f4v x0 = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(Ap + k));
            const f4v x1 = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(Ap + k) + 1);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                ra[e] = x0[e];
                ra[4 + e] = x1[e];
            }
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const d2v x = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(Ap + k) + e);
                ra[2 * e] = x[0];
                ra[2 * e + 1] = x[1];
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const d2v z = reinterpret_cast<const d2v*>(Zp + k)[e];
            rz[2 * e] = z[0];
            rz[2 * e + 1] = z[1];
        }
    };
    d4v acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = (d4v){0.0, 0.0, 0.0, 0.0};
    if (kb0 < kb1) load(kb0 * GD_KC);
    for (int64_t kb = kb0; kb < kb1; ++kb) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            *reinterpret_cast<d2v*>(&As[sr][sc + 2 * e]) = (d2v){ra[2 * e], ra[2 * e + 1]};
            *reinterpret_cast<d2v*>(&Bs[sr][sc + 2 * e]) = (d2v){rz[2 * e], rz[2 * e + 1]};
        }
        __syncthreads();
        if (kb + 1 < kb1) load((kb + 1) * GD_KC);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int kk = 16 * u + 4 * q4;
            const d2v a0 = *reinterpret_cast<const d2v*>(&As[16 * wv + r][kk]);
            const d2v a1 = *reinterpret_cast<const d2v*>(&As[16 * wv + r][kk + 2]);
            const double a[4] = {a0[0], a0[1], a1[0], a1[1]};
            double b[4][4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const d2v b0 = *reinterpret_cast<const d2v*>(&Bs[16 * c + r][kk]);
                const d2v b1 = *reinterpret_cast<const d2v*>(&Bs[16 * c + r][kk + 2]);
                b[c][0] = b0[0];
                b[c][1] = b0[1];
                b[c][2] = b1[0];
                b[c][3] = b1[1];
            }
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s4], b[c][s4], acc[c], 0, 0, 0);
        }
    }
    __syncthreads();   // every wave is done with the tiles before they are overwritten
    double(*tile)[GD_ROWS + 1] = reinterpret_cast<double(*)[GD_ROWS + 1]>(smem);
    // accumulator element v of lane (r, q4): row 4 v + q4 (+16 wv), column r (+16 c)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) tile[16 * c + r][16 * wv + 4 * v + q4] = acc[c][v];
    __syncthreads();
    double* out = Ypart + ks * 64 * M;
    for (int e = threadIdx.x; e < 64 * GD_ROWS; e += 256) {
        const int col = e / GD_ROWS, row = e % GD_ROWS;
        const int64_t i = row0 + row;
        if (i < M) out[(int64_t)col * M + i] = tile[col][row];
    }
}

// Y[col][i] (+)= alpha * sum over the K ranges of Ypart[ks][col][i], in K-range order
__global__ __launch_bounds__(256) void k_gemm_f64_sum(const double* __restrict__ Ypart, int KS, int64_t M, int ncols,
                                                      double* __restrict__ Y, int64_t ldy, int accumulate,
                                                      double alpha) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int col = blockIdx.y;
    if (i >= M || col >= ncols) return;
    double s = 0.0;
    for (int k = 0; k < KS; ++k) s += Ypart[((int64_t)k * 64 + col) * M + i];
    s *= alpha;
    double* y = Y + (int64_t)col * ldy + i;
    *y = accumulate ? *y + s : s;
}

// A few FP64 rows (the floating bodies' constraint rows) times up to 64 vectors, K split over
// many blocks: block b sums its K slice for every (row, column), Zn[k][col] vector-interleaved so
// a wave reads 64 consecutive doubles per k; the 4 waves take every 4th k and are added in a fixed
// order.  part[b][m][col].
__global__ __launch_bounds__(256) void k_rows_part(const double* __restrict__ A, int64_t lda, int M, int64_t K,
                                                   const double* __restrict__ Zn, int64_t kper,
                                                   double* __restrict__ part) {
    __shared__ double red[4][64];
    const int col = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int64_t k0 = (int64_t)blockIdx.x * kper;
    const int64_t k1 = k0 + kper < K ? k0 + kper : K;
    for (int m = 0; m < M; ++m) {
        const double* a = A + (int64_t)m * lda;
        double s = 0.0;
        for (int64_t k = k0 + q; k < k1; k += 4) s = fma(a[k], Zn[k * 64 + col], s);
        red[q][col] = s;
        __syncthreads();
        if (q == 0) part[((int64_t)blockIdx.x * M + m) * 64 + col] = (red[0][col] + red[1][col]) + (red[2][col] + red[3][col]);
        __syncthreads();
    }
}

// Y[col][m] (+)= alpha * sum_b part[b][m][col]: 16 lanes per column each sum every 16th block,
// then the 16 sums are added in lane order (a fixed order; one block per row)
__global__ __launch_bounds__(1024) void k_rows_sum(const double* __restrict__ part, int G, int M, int ncols,
                                                   double* __restrict__ Y, int64_t ldy, int accumulate,
                                                   double alpha) {
    __shared__ double red[16][64];
    const int col = threadIdx.x & 63, q = threadIdx.x >> 6, m = blockIdx.x;
    double s = 0.0;
    for (int b = q; b < G; b += 16) s += part[((int64_t)b * M + m) * 64 + col];
    red[q][col] = s;
    __syncthreads();
    if (q != 0 || col >= ncols) return;
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) t += red[k][col];
    t *= alpha;
    double* y = Y + (int64_t)col * ldy + m;
    *y = accumulate ? *y + t : t;
}

}  // namespace

// Y[c][0..M) (+)= A[0..M)[0..K) Zt[c][0..K) for c < ncols (<= 64); Zt has 64 rows.
void launch_gemm_f32(bem_ctx* c, const float* A, int64_t lda, int64_t M, int64_t K, const float* Zt, int64_t ldz,
                     int ncols, double* Y, int64_t ldy, bool accumulate) {
    if (M <= 0) return;
    if (K % G32_KC != 0 || ldz % 4 != 0 || lda % 4 != 0) throw Error(BEM_ERR_INVALID, "gemm_f32 shape not padded");
    KTimer t(c, "gemm_f32");
    const int64_t rb = ceil_div(M, G32_ROWS);
    const int64_t kblocks = K / G32_KC;
    // K ranges so that the grid has at least the tuned number of blocks (default 1024: 2 per CU)
    int64_t KS = std::max<int64_t>(1, std::min<int64_t>(ceil_div(c->tune_gemm_blocks, rb), kblocks));
    const int64_t kb_per = ceil_div(kblocks, KS);
    KS = ceil_div(kblocks, kb_per);
    c->gemm_part.alloc(sizeof(float) * (size_t)KS * 64 * M);
    hipLaunchKernelGGL(k_gemm_f32, dim3((unsigned)rb, (unsigned)KS), dim3(256), 0, c->stream, A, lda, M, K, Zt, ldz,
                       kb_per, c->gemm_part.as<float>());
    BEM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_gemm_f32_sum, dim3((unsigned)ceil_div(M, 256), (unsigned)ncols), dim3(256), 0, c->stream,
                       c->gemm_part.as<float>(), (int)KS, M, ncols, Y, ldy, (int)accumulate);
    BEM_CHECK_LAUNCH();
}

void launch_gemm_f64(bem_ctx* c, const void* A, bool a_is_f32, int64_t lda, int64_t M, int64_t K, const double* Zt,
                     int64_t ldz, int ncols, double* Y, int64_t ldy, bool accumulate, double alpha) {
    if (M <= 0) return;
    if (K % GD_KC != 0 || ldz % 2 != 0 || lda % 4 != 0) throw Error(BEM_ERR_INVALID, "gemm_f64 shape not padded");
    KTimer t(c, "gemm_f64");
    const int64_t rb = ceil_div(M, GD_ROWS);
    const int64_t kblocks = K / GD_KC;
    int64_t KS = std::min<int64_t>(GD_KS, kblocks);
    const int64_t kb_per = ceil_div(kblocks, KS);
    KS = ceil_div(kblocks, kb_per);
    if (rb * KS > ((int64_t)1 << 31) - 1) throw Error(BEM_ERR_INVALID, "gemm_f64 grid too large");
    c->gemm_part.alloc(sizeof(double) * (size_t)KS * 64 * M);
    double* part = c->gemm_part.as<double>();
    const dim3 grid((unsigned)(rb * KS));
    if (a_is_f32)
        hipLaunchKernelGGL((k_gemm_f64<float>), grid, dim3(256), 0, c->stream, (const float*)A, lda, M, K, Zt, ldz,
                           kb_per, (int)KS, part);
    else
        hipLaunchKernelGGL((k_gemm_f64<double>), grid, dim3(256), 0, c->stream, (const double*)A, lda, M, K, Zt, ldz,
                           kb_per, (int)KS, part);
    BEM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_gemm_f64_sum, dim3((unsigned)ceil_div(M, 256), (unsigned)ncols), dim3(256), 0, c->stream,
                       part, (int)KS, M, ncols, Y, ldy, (int)accumulate, alpha);
    BEM_CHECK_LAUNCH();
}

// Y[c][0..M) (+)= alpha A[0..M)[0..K) Zn[.][c] for a few FP64 rows, Zn[k][64] vector-interleaved (each
// row re-reads Zn, so this suits the handful of constraint rows, not a matrix).
void launch_gemm_rows(bem_ctx* c, const double* A, int64_t lda, int64_t M, int64_t K, const double* Zn, int ncols,
                      double* Y, int64_t ldy, bool accumulate, double alpha) {
    if (M <= 0) return;
    if (M > 65535) throw Error(BEM_ERR_INVALID, "gemm_rows: too many rows");
    KTimer t(c, "gemm_rows");
    // about 64 k per block and at most 512 blocks
    const int64_t G = std::max<int64_t>(1, std::min<int64_t>(512, ceil_div(K, 64)));
    const int64_t kper = ceil_div(K, G);
    const int64_t Gn = ceil_div(K, kper);
    c->rows_part.alloc(sizeof(double) * (size_t)Gn * M * 64);
    hipLaunchKernelGGL(k_rows_part, dim3((unsigned)Gn), dim3(256), 0, c->stream, A, lda, (int)M, K, Zn, kper,
                       c->rows_part.as<double>());
    BEM_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_rows_sum, dim3((unsigned)M), dim3(1024), 0, c->stream, c->rows_part.as<double>(), (int)Gn,
                       (int)M, ncols, Y, ldy, (int)accumulate, alpha);
    BEM_CHECK_LAUNCH();
}

}  // namespace bem
