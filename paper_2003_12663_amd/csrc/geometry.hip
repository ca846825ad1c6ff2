// Panel geometry (one thread per triangle): unit normal, area, centroid
// (the collocation point), circumcentre and circumradius (precomputed for
// the Sec. 4 pair classification) and the nodes and scaled weights of the
// degree-5, 7-point triangle rule used for regular pairs.
#include "bem_device.h"

namespace bem {
namespace {

__global__ __launch_bounds__(256) void k_geometry(const double* __restrict__ vert, const int32_t* __restrict__ tri,
                                                  int64_t N, int64_t Np, double eta, double* __restrict__ far64,
                                                  float* __restrict__ far32, double* __restrict__ tri64,
                                                  double* __restrict__ pan64, float* __restrict__ pan32) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= Np) return;
    if (j >= N) {
        // padding panels: far away, zero weight, never near
#pragma unroll
        for (int c = 0; c < FAR_REC; ++c) {
            double v = (c == FR_RR) ? -1.0 : ((c < FR_W || c >= FR_CC) ? 1.0e30 : 0.0);
            far64[(int64_t)c * Np + j] = v;
            far32[(int64_t)c * Np + j] = (float)((c == FR_RR) ? -1.0 : ((c < FR_W || c >= FR_CC) ? 1.0e30 : 0.0));
            pan64[FAR_REC * j + c] = v;
            pan32[FAR_REC * j + c] = far32[(int64_t)c * Np + j];
        }
        return;
    }
    double v[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t iv = tri[3 * j + a];
#pragma unroll
        for (int k = 0; k < 3; ++k) v[a][k] = vert[3 * iv + k];
    }
    const double e10 = v[1][0] - v[0][0], e11 = v[1][1] - v[0][1], e12 = v[1][2] - v[0][2];
    const double e20 = v[2][0] - v[0][0], e21 = v[2][1] - v[0][1], e22 = v[2][2] - v[0][2];
    const double c0 = e11 * e22 - e12 * e21, c1 = e12 * e20 - e10 * e22, c2 = e10 * e21 - e11 * e20;
    const double clen = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    const double area = 0.5 * clen;
    // circumcentre in barycentric form: weights a^2 (b^2 + c^2 - a^2) etc., with
    // a, b, c the side lengths opposite v1, v2, v3
    auto d2 = [&](int p, int q) {
        double x = v[p][0] - v[q][0], y = v[p][1] - v[q][1], z = v[p][2] - v[q][2];
        return x * x + y * y + z * z;
    };
    const double A2 = d2(1, 2), B2 = d2(2, 0), C2 = d2(0, 1);
    const double wa = A2 * (B2 + C2 - A2), wb = B2 * (C2 + A2 - B2), wc = C2 * (A2 + B2 - C2);
    const double ws = wa + wb + wc;
    double cc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) cc[k] = (wa * v[0][k] + wb * v[1][k] + wc * v[2][k]) / ws;
    const double Rx = v[0][0] - cc[0], Ry = v[0][1] - cc[1], Rz = v[0][2] - cc[2];
    const double R = sqrt(Rx * Rx + Ry * Ry + Rz * Rz);
    const double rr = (eta * R) * (eta * R);

    // 7-point rule: centroid (9/40) and two orbits (a, a, 1 - 2a)
    const double s15 = sqrt(15.0);
    const double a1 = (6.0 - s15) / 21.0, a2 = (6.0 + s15) / 21.0;
    const double wt1 = (155.0 - s15) / 1200.0, wt2 = (155.0 + s15) / 1200.0;
    double bw[7][4] = {
        {1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, 9.0 / 40.0},
        {a1, a1, 1.0 - 2.0 * a1, wt1}, {a1, 1.0 - 2.0 * a1, a1, wt1}, {1.0 - 2.0 * a1, a1, a1, wt1},
        {a2, a2, 1.0 - 2.0 * a2, wt2}, {a2, 1.0 - 2.0 * a2, a2, wt2}, {1.0 - 2.0 * a2, a2, a2, wt2},
    };
    const double wscale = area * INV4PI;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        double y[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) y[k] = bw[q][0] * v[0][k] + bw[q][1] * v[1][k] + bw[q][2] * v[2][k];
        const double wq = bw[q][3] * wscale;
        far64[(int64_t)(FR_X + q) * Np + j] = y[0];
        far64[(int64_t)(FR_Y + q) * Np + j] = y[1];
        far64[(int64_t)(FR_Z + q) * Np + j] = y[2];
        far64[(int64_t)(FR_W + q) * Np + j] = wq;
        far32[(int64_t)(FR_X + q) * Np + j] = (float)y[0];
        far32[(int64_t)(FR_Y + q) * Np + j] = (float)y[1];
        far32[(int64_t)(FR_Z + q) * Np + j] = (float)y[2];
        far32[(int64_t)(FR_W + q) * Np + j] = (float)wq;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        far64[(int64_t)(FR_CC + k) * Np + j] = cc[k];
        far32[(int64_t)(FR_CC + k) * Np + j] = (float)cc[k];
    }
    far64[(int64_t)FR_RR * Np + j] = rr;
    // the FP32 copy is never used to classify: kernels classify in FP64 or
    // with this value widened, so it only needs to be conservative
    far32[(int64_t)FR_RR * Np + j] = (float)rr;
    // the same records panel-major (one 32-value record per panel), for kernels that read a
    // panel's whole record at a wave-uniform address
#pragma unroll
    for (int c = 0; c < FAR_REC; ++c) {
        pan64[FAR_REC * j + c] = far64[(int64_t)c * Np + j];
        pan32[FAR_REC * j + c] = far32[(int64_t)c * Np + j];
    }

    double* T = tri64 + (int64_t)TRI_REC * j;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k = 0; k < 3; ++k) T[TR_V + 3 * a + k] = v[a][k];
    T[TR_N + 0] = c0 / clen;
    T[TR_N + 1] = c1 / clen;
    T[TR_N + 2] = c2 / clen;
#pragma unroll
    for (int k = 0; k < 3; ++k) T[TR_C + k] = (v[0][k] + v[1][k] + v[2][k]) / 3.0;
    T[TR_A] = area;
}

// One lane per point: the point of panel j = panel[l] with barycentric coordinates bary[l] (over
// the panel's vertices in their stored order), lifted by `offset` along the panel's unit normal.
__global__ __launch_bounds__(256) void k_panel_points(int64_t L, const int32_t* __restrict__ panel,
                                                      const double* __restrict__ bary, double offset,
                                                      const double* __restrict__ tri64, double* __restrict__ out) {
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (l >= L) return;
    const double* T = tri64 + (int64_t)TRI_REC * panel[l];
    const double b0 = bary[3 * l], b1 = bary[3 * l + 1], b2 = bary[3 * l + 2];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        out[3 * l + k] = b0 * T[TR_V + k] + b1 * T[TR_V + 3 + k] + b2 * T[TR_V + 6 + k] + offset * T[TR_N + k];
}

}  // namespace

void launch_panel_points(bem_ctx* c, int64_t L, const int32_t* panel, const double* bary, double offset,
                         double* out) {
    if (L == 0) return;
    hipLaunchKernelGGL(k_panel_points, dim3((unsigned)ceil_div(L, 256)), dim3(256), 0, c->stream, L, panel, bary,
                       offset, c->tri64.as<double>(), out);
    BEM_CHECK_LAUNCH();
}

void launch_geometry(bem_ctx* c) {
    KTimer t(c, "geometry");
    const int64_t Np = c->far64.bytes / (sizeof(double) * FAR_REC);
    dim3 grid((unsigned)ceil_div(Np, 256));
    hipLaunchKernelGGL(k_geometry, grid, dim3(256), 0, c->stream, c->vert.as<double>(), c->tri.as<int32_t>(), c->N, Np,
                       c->opt.eta, c->far64.as<double>(), c->far32.as<float>(), c->tri64.as<double>(),
                       c->pan64.as<double>(), c->pan32.as<float>());
    BEM_CHECK_LAUNCH();
}

}  // namespace bem
