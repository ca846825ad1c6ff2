// C ABI of the library: validation, context lifetime, device buffers and the
// order of the passes.  Nothing here computes the method itself; every
// numerical step runs in the kernels of the other translation units.
#include <algorithm>
#include <memory>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "bem_internal.h"

namespace {

thread_local std::string g_err;

bem_status fail(bem_status s, const std::string& m) {
    g_err = m;
    return s;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

#define API_TRY try {
#define API_CATCH                                                                  \
    }                                                                              \
    catch (const bem::Error& e) {                                                  \
        return fail(e.code, e.what());                                             \
    }                                                                              \
    catch (const std::bad_alloc&) {                                                \
        return fail(BEM_ERR_OOM, "host allocation failed");                        \
    }                                                                              \
    catch (const std::exception& e) {                                              \
        return fail(BEM_ERR_HIP, e.what());                                        \
    }

template <class T>
void upload(bem::DBuf& b, const T* h, size_t count, hipStream_t s) {
    b.alloc(sizeof(T) * (count > 0 ? count : 1));
    if (count) BEM_HIP(hipMemcpyAsync(b.p, h, sizeof(T) * count, hipMemcpyHostToDevice, s));
}

void check_assembled(const bem_ctx* c) {
    if (!c->assembled) throw bem::Error(BEM_ERR_STATE, "bem_assemble has not been called");
}

std::vector<double> fetch_f64(const bem_ctx* c, const double* d, size_t count) {
    std::vector<double> h(count);
    if (count) {
        BEM_HIP(hipMemcpyAsync(h.data(), d, sizeof(double) * count, hipMemcpyDeviceToHost, c->stream));
        BEM_HIP(hipStreamSynchronize(c->stream));
    }
    return h;
}

std::vector<int32_t> fetch_i32(const bem_ctx* c, const int32_t* d, size_t count) {
    std::vector<int32_t> h(count);
    if (count) {
        BEM_HIP(hipMemcpyAsync(h.data(), d, sizeof(int32_t) * count, hipMemcpyDeviceToHost, c->stream));
        BEM_HIP(hipStreamSynchronize(c->stream));
    }
    return h;
}

void check_points(const bem_ctx* c, int64_t P, const double* pts) {
    if (P < 0) throw bem::Error(BEM_ERR_INVALID, "negative point count");
    if (P > 0 && !pts) throw bem::Error(BEM_ERR_INVALID, "points pointer is NULL");
    auto h = fetch_f64(c, pts, (size_t)P * 3);
    for (double v : h)
        if (!std::isfinite(v)) throw bem::Error(BEM_ERR_INVALID, "non-finite point coordinate");
}

void check_trace(const bem_ctx* c, int32_t nrhs, const double* sol, int64_t L, const int32_t* line_rhs,
                 const double* starts, const bem_trace_params* tp) {
    if (c->opt.basis == BEM_BASIS_LINEAR && c->trace_mode == 2)
        throw bem::Error(BEM_ERR_INVALID, "field lines of the LINEAR basis need an all-lines layout (trace_mode 0, 1 or 3)");
    if (c->trace_mode == 3 && bem::fused_trace_blocks(c->N, 4) == 0)
        throw bem::Error(BEM_ERR_INVALID, "trace_mode 3 takes at most 131072 panels");
    if (!tp) throw bem::Error(BEM_ERR_INVALID, "trace parameters are NULL");
    if (nrhs < 1) throw bem::Error(BEM_ERR_INVALID, "nrhs must be >= 1");
    if (!sol) throw bem::Error(BEM_ERR_INVALID, "solution pointer is NULL");
    if (!(tp->h > 0.0) || !std::isfinite(tp->h)) throw bem::Error(BEM_ERR_INVALID, "step h must be finite and > 0");
    if (!(tp->h < (c->opt.eta - 1.0) * c->min_R * (1.0 - 1e-9)))
        throw bem::Error(BEM_ERR_INVALID,
                         "step h must be < (eta - 1) * smallest circumradius so that every panel a step can "
                         "reach is classified near");
    if (tp->max_steps < 1 || tp->max_steps > 1000000) throw bem::Error(BEM_ERR_INVALID, "max_steps out of 1..1e6");
    if (!(tp->e_min >= 0.0) || !std::isfinite(tp->e_min)) throw bem::Error(BEM_ERR_INVALID, "e_min must be >= 0");
    if (!std::isfinite(tp->alpha_a) || !std::isfinite(tp->alpha_e0) || !std::isfinite(tp->alpha_p) ||
        std::isnan(tp->k_str))
        throw bem::Error(BEM_ERR_INVALID, "non-finite ionisation parameters");
    if (L < 0 || L >= ((int64_t)1 << 31)) throw bem::Error(BEM_ERR_INVALID, "line count out of range");
    check_points(c, L, starts);
    if (line_rhs) {
        auto h = fetch_i32(c, line_rhs, (size_t)L);
        for (int32_t v : h)
            if (v < 0 || v >= nrhs) throw bem::Error(BEM_ERR_INVALID, "line_rhs entry out of range");
    }
}

}  // namespace

namespace bem {

void timing_events(bem_ctx* c, hipEvent_t* a, hipEvent_t* b) {
    hipEvent_t* out[2] = {a, b};
    for (hipEvent_t* e : out) {
        if (!c->event_pool.empty()) {
            *e = c->event_pool.back();
            c->event_pool.pop_back();
        } else {
            BEM_HIP(hipEventCreate(e));
        }
    }
}

void push_timing(bem_ctx* c, const char* name, hipEvent_t a, hipEvent_t b) {
    c->pending.push_back({name, {a, b}});
    if (c->pending.size() > 4096) resolve_ready(c);
}

KTimer::KTimer(bem_ctx* ctx, const char* nm, bool enabled, hipStream_t st)
    : c(ctx), name(nm), s(st ? st : ctx->stream) {
    if (c->profiling != 1 || !enabled) return;
    timing_events(c, &a, &b);
    BEM_HIP(hipEventRecord(a, s));
}

KTimer::~KTimer() {
    if (!a) return;
    if (hipEventRecord(b, s) != hipSuccess) return;
    push_timing(c, name, a, b);
}

namespace {
// add the pair's time to its statistic and return the events to the pool
void take(bem_ctx* c, const std::string& name, hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) == hipSuccess) {
        auto& s = c->stats[name];
        s.launches += 1;
        s.ms += ms;
    }
    c->event_pool.push_back(a);
    c->event_pool.push_back(b);
}
}  // namespace

void resolve_stats(bem_ctx* c) {
    for (auto& p : c->pending) {
        (void)hipEventSynchronize(p.second.second);
        take(c, p.first, p.second.first, p.second.second);
    }
    c->pending.clear();
}

// Resolves the pending pairs whose end event has completed, in order, without waiting, so that
// a long profiled run never blocks the host on the GPU to make room.
void resolve_ready(bem_ctx* c) {
    size_t k = 0;
    for (; k < c->pending.size(); ++k) {
        auto& p = c->pending[k];
        if (hipEventQuery(p.second.second) != hipSuccess) break;
        take(c, p.first, p.second.first, p.second.second);
    }
    c->pending.erase(c->pending.begin(), c->pending.begin() + (ptrdiff_t)k);
}

}  // namespace bem

extern "C" {

const char* bem_last_error(void) { return g_err.c_str(); }

bem_status bem_create(int64_t n_vert, const double* vert, int64_t n_tri, const int32_t* tri, const int32_t* tri_body,
                      int32_t n_body, const bem_body* bodies, const bem_options* opt, void* hip_stream,
                      bem_ctx** out) {
    if (!out) return fail(BEM_ERR_INVALID, "out pointer is NULL");
    *out = nullptr;
    if (!vert || !tri || !tri_body || !bodies) return fail(BEM_ERR_INVALID, "NULL mesh array");
    if (n_vert < 3 || n_tri < 1 || n_body < 1)
        return fail(BEM_ERR_INVALID, "mesh needs >= 3 vertices, >= 1 triangle, >= 1 body");
    if (n_tri >= ((int64_t)1 << 31) || n_vert >= ((int64_t)1 << 31)) return fail(BEM_ERR_INVALID, "mesh too large");
    bem_options o = {BEM_FP64, 6.0, 100, 0, BEM_BASIS_CONSTANT};
    if (opt) o = *opt;
    if (o.precision != BEM_FP64 && o.precision != BEM_MIXED) return fail(BEM_ERR_INVALID, "unknown precision");
    if (!(o.eta >= 1.0) || !std::isfinite(o.eta)) return fail(BEM_ERR_INVALID, "eta must be finite and >= 1");
    if (o.restart < 1 || o.restart > 1000) return fail(BEM_ERR_INVALID, "restart out of 1..1000");
    if (o.constraint_form != 0 && o.constraint_form != 1) return fail(BEM_ERR_INVALID, "unknown constraint_form");
    if (o.basis != BEM_BASIS_CONSTANT && o.basis != BEM_BASIS_LINEAR) return fail(BEM_ERR_INVALID, "unknown basis");
    if (o.basis == BEM_BASIS_LINEAR) {
        if (n_tri >= ((int64_t)1 << 29)) return fail(BEM_ERR_INVALID, "mesh too large for the LINEAR basis");
    }
    for (int64_t k = 0; k < 3 * n_vert; ++k)
        if (!std::isfinite(vert[k])) return fail(BEM_ERR_INVALID, "non-finite vertex coordinate");
    for (int32_t b = 0; b < n_body; ++b) {
        const bem_body& bd = bodies[b];
        if (bd.kind < BEM_DIRICHLET || bd.kind > BEM_FLOATING_SHEET) return fail(BEM_ERR_INVALID, "unknown body kind");
        if (!(bd.eps_plus > 0.0) || !std::isfinite(bd.eps_plus)) return fail(BEM_ERR_INVALID, "eps_plus must be > 0");
        if (bd.kind == BEM_INTERFACE && (!(bd.eps_minus > 0.0) || !std::isfinite(bd.eps_minus)))
            return fail(BEM_ERR_INVALID, "eps_minus must be > 0 on an interface");
    }
    double min_R = INFINITY;
    std::vector<int64_t> per_body(n_body, 0);
    for (int64_t j = 0; j < n_tri; ++j) {
        const int32_t* t = tri + 3 * j;
        for (int k = 0; k < 3; ++k)
            if (t[k] < 0 || t[k] >= n_vert) return fail(BEM_ERR_INVALID, "triangle vertex index out of range");
        if (tri_body[j] < 0 || tri_body[j] >= n_body) return fail(BEM_ERR_INVALID, "triangle body index out of range");
        per_body[tri_body[j]]++;
        const double* a = vert + 3 * (int64_t)t[0];
        const double* b = vert + 3 * (int64_t)t[1];
        const double* c = vert + 3 * (int64_t)t[2];
        double u[3], w[3], e[3];
        for (int k = 0; k < 3; ++k) {
            u[k] = b[k] - a[k];
            w[k] = c[k] - a[k];
            e[k] = c[k] - b[k];
        }
        const double cr0 = u[1] * w[2] - u[2] * w[1], cr1 = u[2] * w[0] - u[0] * w[2], cr2 = u[0] * w[1] - u[1] * w[0];
        const double area = 0.5 * std::sqrt(cr0 * cr0 + cr1 * cr1 + cr2 * cr2);
        const double lu = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        const double lw = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        const double le = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        const double lmax = std::max(lu, std::max(lw, le));
        if (!(area > 1e-14 * lmax * lmax)) return fail(BEM_ERR_DEGENERATE, "degenerate triangle " + std::to_string(j));
        min_R = std::min(min_R, lu * lw * le / (4.0 * area));
    }
    for (int32_t b = 0; b < n_body; ++b)
        if ((bodies[b].kind == BEM_FLOATING || bodies[b].kind == BEM_FLOATING_SHEET) && per_body[b] == 0)
            return fail(BEM_ERR_INVALID, "floating body without panels");
    // LINEAR basis: every vertex in a triangle, and all triangles at a vertex of one body
    std::vector<int32_t> vert_body;
    if (o.basis == BEM_BASIS_LINEAR) {
        vert_body.assign(n_vert, -1);
        for (int64_t j = 0; j < n_tri; ++j)
            for (int k = 0; k < 3; ++k) {
                int32_t& vb = vert_body[tri[3 * j + k]];
                if (vb >= 0 && vb != tri_body[j])
                    return fail(BEM_ERR_INVALID, "LINEAR basis: a vertex is shared by triangles of two bodies");
                vb = tri_body[j];
            }
        for (int64_t i = 0; i < n_vert; ++i)
            if (vert_body[i] < 0) return fail(BEM_ERR_INVALID, "LINEAR basis: a vertex is in no triangle");
    }

    API_TRY
    int dev = 0;
    BEM_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    BEM_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        throw bem::Error(BEM_ERR_HIP, std::string("this library is built for gfx950, device is ") + prop.gcnArchName);
    bem::noalloc_scratch_init(dev);   // bem_matvec_noalloc's work array on this device
    std::unique_ptr<bem_ctx> c(new bem_ctx());
    c->device = dev;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->opt = o;
    c->N = n_tri;
    c->n_vert = n_vert;
    c->n_body = n_body;
    c->min_R = min_R;
    c->h_tri.assign(tri, tri + 3 * n_tri);
    c->h_tri_body.assign(tri_body, tri_body + n_tri);
    c->h_body_kind.resize(n_body);
    c->h_epsp.resize(n_body);
    c->h_epsm.resize(n_body);
    c->h_body_fidx.assign(n_body, -1);
    for (int32_t b = 0; b < n_body; ++b) {
        c->h_body_kind[b] = bodies[b].kind;
        c->h_epsp[b] = bodies[b].eps_plus;
        c->h_epsm[b] = bodies[b].eps_minus;
        if (bodies[b].kind == BEM_FLOATING || bodies[b].kind == BEM_FLOATING_SHEET) c->h_body_fidx[b] = c->n_float++;
        if (bodies[b].kind == BEM_FLOATING_SHEET) c->has_sheet = true;
    }
    c->n = c->N + c->n_float;
    c->nb = c->N;
    // the FP32 matvec reads an FP64 x per FP32 entry: 8 rows per block halve that L2 traffic
    // (measured 9-10 % faster than 4 at 67k and 233k unknowns); FP64 keeps 4
    if (o.precision == BEM_MIXED) c->tune_gemv_rows = 8;
    std::vector<int32_t> fan_ptr, fan, row_order, grp_ptr, grp_tri;
    std::vector<uint32_t> grp_loc;
    if (o.basis == BEM_BASIS_LINEAR) {
        // vertex -> body (checked above) and the vertex fans
        c->h_vert_body = vert_body;
        fan_ptr.assign(n_vert + 1, 0);
        for (int64_t j = 0; j < n_tri; ++j)
            for (int k = 0; k < 3; ++k) ++fan_ptr[tri[3 * j + k] + 1];
        for (int64_t i = 0; i < n_vert; ++i) fan_ptr[i + 1] += fan_ptr[i];
        fan.resize(3 * (size_t)n_tri);
        std::vector<int32_t> fill(fan_ptr.begin(), fan_ptr.end() - 1);
        for (int64_t j = 0; j < n_tri; ++j)   // triangles ascending within each fan
            for (int k = 0; k < 3; ++k) fan[fill[tri[3 * j + k]]++] = (int32_t)((j << 2) | k);
        // column groups of 16 vertices: each triangle once per group that holds one of its
        // corners, triangles ascending, with the local column of every corner
        const int64_t ng = (n_vert + 15) / 16;
        grp_ptr.assign(ng + 1, 0);
        for (int64_t j = 0; j < n_tri; ++j) {
            const int64_t g0 = tri[3 * j] / 16, g1 = tri[3 * j + 1] / 16, g2 = tri[3 * j + 2] / 16;
            ++grp_ptr[g0 + 1];
            if (g1 != g0) ++grp_ptr[g1 + 1];
            if (g2 != g0 && g2 != g1) ++grp_ptr[g2 + 1];
        }
        for (int64_t g = 0; g < ng; ++g) grp_ptr[g + 1] += grp_ptr[g];
        grp_tri.resize((size_t)grp_ptr[ng]);
        grp_loc.resize((size_t)grp_ptr[ng]);
        std::vector<int32_t> gfill(grp_ptr.begin(), grp_ptr.end() - 1);
        for (int64_t j = 0; j < n_tri; ++j) {
            int64_t gs[3];
            int ngs = 0;
            for (int k = 0; k < 3; ++k) {
                const int64_t g = tri[3 * j + k] / 16;
                bool seen = false;
                for (int m = 0; m < ngs; ++m) seen = seen || gs[m] == g;
                if (!seen) gs[ngs++] = g;
            }
            for (int m = 0; m < ngs; ++m) {
                uint32_t loc = 0;
                for (int k = 0; k < 3; ++k) {
                    const int64_t v = tri[3 * j + k];
                    const uint32_t l = (v / 16 == gs[m]) ? (uint32_t)(v % 16) : 0xffu;
                    loc |= l << (8 * k);
                }
                const int32_t pos = gfill[gs[m]]++;
                grp_tri[pos] = (int32_t)j;
                grp_loc[pos] = loc;
            }
        }
        c->n = n_vert + c->n_float;
        c->nb = n_vert;
        // vertices in Morton (Z-curve) order of their positions in the bounding box, 21 bits
        // per axis: the near-pair pass takes its rows in this order so that a wave's rows are
        // neighbours
        double lo[3] = {vert[0], vert[1], vert[2]}, hi[3] = {vert[0], vert[1], vert[2]};
        for (int64_t i = 0; i < n_vert; ++i)
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], vert[3 * i + k]);
                hi[k] = std::max(hi[k], vert[3 * i + k]);
            }
        auto spread = [](uint64_t v) {   // 21 bits -> every third bit of 63
            v &= 0x1fffff;
            v = (v | v << 32) & 0x1f00000000ffffULL;
            v = (v | v << 16) & 0x1f0000ff0000ffULL;
            v = (v | v << 8) & 0x100f00f00f00f00fULL;
            v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
            v = (v | v << 2) & 0x1249249249249249ULL;
            return v;
        };
        std::vector<std::pair<uint64_t, int32_t>> key(n_vert);
        for (int64_t i = 0; i < n_vert; ++i) {
            uint64_t m = 0;
            for (int k = 0; k < 3; ++k) {
                const double ext = hi[k] - lo[k];
                const double f = ext > 0.0 ? (vert[3 * i + k] - lo[k]) / ext : 0.0;
                m |= spread((uint64_t)std::min(f * 2097151.0, 2097151.0)) << k;
            }
            key[i] = {m, (int32_t)i};
        }
        std::sort(key.begin(), key.end());
        row_order.resize(n_vert);
        for (int64_t i = 0; i < n_vert; ++i) row_order[i] = key[i].second;
    }
    c->ld = (c->n + 31) / 32 * 32;
    c->h_flt_coef.assign(2 * (size_t)std::max(c->n_float, 1), 0.0);
    for (int32_t b = 0; b < n_body; ++b) {
        const int32_t f = c->h_body_fidx[b];
        if (f < 0) continue;
        double cs = 0.5, ck = 1.0;   // Eq. Final4 over eps+ sum a
        if (bodies[b].kind == BEM_FLOATING_SHEET) {   // Eq. sheets over (eps+ + eps-) / 2 sum a
            cs = 1.0;
            ck = 2.0 * (bodies[b].eps_plus - bodies[b].eps_minus) / (bodies[b].eps_plus + bodies[b].eps_minus);
        } else if (o.constraint_form == 1) {   // net charge
            cs = 1.0;
            ck = 0.0;
        }
        c->h_flt_coef[2 * f] = cs;
        c->h_flt_coef[2 * f + 1] = ck;
    }
    if (o.basis == BEM_BASIS_LINEAR) {
        // centroid rows of the rows that need n . E: interface bodies, then floating bodies whose
        // row has a K' term (literal Eq. Final4, sheets), each body's triangles ascending
        std::vector<int32_t>& crow = c->h_crow_tri;
        c->h_flt_crange.assign(2 * (size_t)std::max(c->n_float, 1), 0);
        for (int32_t b = 0; b < n_body; ++b) {
            const int32_t f = c->h_body_fidx[b];
            const bool kp = bodies[b].kind == BEM_INTERFACE || (f >= 0 && c->h_flt_coef[2 * f + 1] != 0.0);
            if (!kp) continue;
            const int32_t r0 = (int32_t)crow.size();
            for (int64_t j = 0; j < n_tri; ++j)
                if (tri_body[j] == b) crow.push_back((int32_t)j);
            if (f >= 0) {
                c->h_flt_crange[2 * f] = r0;
                c->h_flt_crange[2 * f + 1] = (int32_t)crow.size();
                c->h_flt_kp.push_back(f);
            }
        }
        for (int64_t i = 0; i < n_vert; ++i)
            if (bodies[c->h_vert_body[i]].kind == BEM_INTERFACE) c->h_iface_v.push_back((int32_t)i);
    }
    // row segments by kind (Sec. 4: rows grouped by type); floating rows sorted by
    // (body, panel) so that each body's rows are contiguous
    std::vector<int32_t> slot(n_tri, -1);
    for (int64_t i = 0; i < n_tri; ++i) {
        if (c->h_body_kind[tri_body[i]] == BEM_INTERFACE)
            c->h_rows_int.push_back((int32_t)i);
        else
            c->h_rows_pot.push_back((int32_t)i);
    }
    for (int32_t f = 0; f < c->n_float; ++f)
        for (int64_t i = 0; i < n_tri; ++i)
            if (c->h_body_fidx[tri_body[i]] == f) {
                slot[i] = (int32_t)c->h_rows_flt.size();
                c->h_rows_flt.push_back((int32_t)i);
            }
    const int64_t Np = (c->N + 255) / 256 * 256;
    hipStream_t s = c->stream;
    c->host_stage.alloc(sizeof(double) * 4096);
    upload(c->vert, vert, (size_t)(3 * n_vert), s);
    upload(c->tri, tri, (size_t)(3 * n_tri), s);
    upload(c->tri_body, tri_body, (size_t)n_tri, s);
    // on the device a sheet is a floating body (its rows, columns and stop code); only the
    // constraint row, built on the host's kind list, differs
    std::vector<int32_t> dkind(c->h_body_kind);
    for (int32_t& k : dkind)
        if (k == BEM_FLOATING_SHEET) k = BEM_FLOATING;
    upload(c->body_kind, dkind.data(), (size_t)n_body, s);
    upload(c->body_epsp, c->h_epsp.data(), (size_t)n_body, s);
    upload(c->body_epsm, c->h_epsm.data(), (size_t)n_body, s);
    upload(c->body_fidx, c->h_body_fidx.data(), (size_t)n_body, s);
    upload(c->flt_coef, c->h_flt_coef.data(), c->h_flt_coef.size(), s);
    if (o.basis == BEM_BASIS_LINEAR) {
        upload(c->vert_body, c->h_vert_body.data(), c->h_vert_body.size(), s);
        upload(c->fan_ptr, fan_ptr.data(), fan_ptr.size(), s);
        upload(c->fan, fan.data(), fan.size(), s);
        upload(c->row_order, row_order.data(), row_order.size(), s);
        upload(c->grp_ptr, grp_ptr.data(), grp_ptr.size(), s);
        upload(c->grp_tri, grp_tri.data(), grp_tri.size(), s);
        upload(c->grp_loc, grp_loc.data(), grp_loc.size(), s);
        if (!c->h_crow_tri.empty()) {
            std::vector<int32_t> tri_crow((size_t)n_tri, -1);
            for (size_t r = 0; r < c->h_crow_tri.size(); ++r) tri_crow[c->h_crow_tri[r]] = (int32_t)r;
            upload(c->nod_trow, c->h_crow_tri.data(), c->h_crow_tri.size(), s);
            upload(c->nod_tri_crow, tri_crow.data(), tri_crow.size(), s);
            upload(c->nod_iface_v, c->h_iface_v.data(), c->h_iface_v.size(), s);
            upload(c->nod_frange, c->h_flt_crange.data(), c->h_flt_crange.size(), s);
            upload(c->nod_flist, c->h_flt_kp.data(), c->h_flt_kp.size(), s);
        }
    }
    upload(c->rows_pot, c->h_rows_pot.data(), c->h_rows_pot.size(), s);
    upload(c->rows_int, c->h_rows_int.data(), c->h_rows_int.size(), s);
    upload(c->rows_flt, c->h_rows_flt.data(), c->h_rows_flt.size(), s);
    upload(c->row_slot, slot.data(), slot.size(), s);
    // interface-row scales (eps+ - eps-) followed by ones for the K' rows of floating bodies
    std::vector<double> scales;
    for (int32_t i : c->h_rows_int) scales.push_back(c->h_epsp[tri_body[i]] - c->h_epsm[tri_body[i]]);
    if (scales.empty()) scales.push_back(0.0);
    for (size_t k = 0; k < c->h_rows_flt.size(); ++k) scales.push_back(1.0);
    upload(c->gm_misc, scales.data(), scales.size(), s);
    c->far64.alloc(sizeof(double) * bem::FAR_REC * Np);
    c->far32.alloc(sizeof(float) * bem::FAR_REC * Np);
    c->pan64.alloc(sizeof(double) * bem::FAR_REC * Np);
    c->pan32.alloc(sizeof(float) * bem::FAR_REC * Np);
    c->tri64.alloc(sizeof(double) * bem::TRI_REC * c->N);
    c->counters.alloc(sizeof(uint64_t) * 8);
    BEM_HIP(hipMemsetAsync(c->counters.p, 0, sizeof(uint64_t) * 8, s));
    bem::launch_geometry(c.get());
    BEM_HIP(hipStreamSynchronize(s));   // host-side sources of the uploads are temporaries
    *out = c.release();
    return BEM_OK;
    API_CATCH
}

void bem_destroy(bem_ctx* c) {
    if (!c) return;
    DeviceGuard g(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->aux_stream) (void)hipStreamSynchronize(c->aux_stream);
    bem::hmatrix_release(c);
    delete c;
}

int64_t bem_n_unknowns(const bem_ctx* c) { return c ? c->n : -1; }

int64_t bem_near_pairs(const bem_ctx* c) { return c ? c->near_nnz : -1; }

bem_status bem_assemble(bem_ctx* c) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    bem::hmatrix_release(c);   // the dense operator replaces a compressed one
    if (c->opt.basis == BEM_BASIS_LINEAR) {
        // FP64: one n x ld matrix.  MIXED: the vertex rows in FP32 (nb x ld) and the constraint
        // rows in FP64 (n_float x ld), with an empty list of FP64 near remainders
        const bool mixed = c->opt.precision == BEM_MIXED;
        const size_t nfl = (size_t)(c->n_float > 0 ? c->n_float : 1);
        const size_t kc = sizeof(double) * c->h_crow_tri.size() * (size_t)c->ld;   // normal-field rows
        const size_t need = (mixed ? sizeof(float) * (size_t)c->nb * c->ld + sizeof(double) * nfl * c->ld
                                   : sizeof(double) * (size_t)c->n * c->ld) + kc;
        size_t free_b = 0, total_b = 0;
        BEM_HIP(hipMemGetInfo(&free_b, &total_b));
        const size_t have = free_b + c->A64.bytes + c->A32.bytes + c->nod_Kc.bytes;
        if (need > have)
            throw bem::Error(BEM_ERR_OOM, "assembly needs " + std::to_string(need >> 20) + " MiB, " +
                                              std::to_string(have >> 20) + " MiB free");
        c->assembled = false;
        if (mixed) {
            c->A64.release();
            c->A32.alloc(sizeof(float) * (size_t)c->nb * c->ld);
            c->A64.alloc(sizeof(double) * nfl * c->ld);
            c->near_ptr.alloc(sizeof(int64_t) * (size_t)(c->nb + 1));
            BEM_HIP(hipMemsetAsync(c->near_ptr.p, 0, sizeof(int64_t) * (size_t)(c->nb + 1), c->stream));
            c->near_col.alloc(sizeof(int32_t));
            c->near_val.alloc(sizeof(double));
            c->near_nnz = 0;
        } else {
            c->A32.release();
            c->A64.alloc(need - kc);
        }
        if (kc) c->nod_Kc.alloc(kc);
        c->diag.alloc(sizeof(double) * c->ld);
        bem::launch_nodal_assemble(c);
        BEM_HIP(hipStreamSynchronize(c->stream));
        c->assembled = true;
        return BEM_OK;
    }
    const bool mixed = c->opt.precision == BEM_MIXED;
    const int64_t N = c->N, n = c->n, ld = c->ld;
    const int64_t nblk = bem::ceil_div(N, 64);
    const size_t nflt = c->h_rows_flt.size();
    // device memory needed, checked before allocating anything large
    size_t need = 0;
    need += mixed ? sizeof(float) * (size_t)N * ld + sizeof(double) * (size_t)c->n_float * ld
                  : sizeof(double) * (size_t)n * ld;
    need += sizeof(uint64_t) * (size_t)nblk * N;                 // near masks
    need += (size_t)N * 160 * (mixed ? 16 : 8);                   // near list, ~90-160 pairs per row
    if (c->opt.constraint_form == 0 || c->has_sheet) need += sizeof(double) * nflt * N;
    size_t free_b = 0, total_b = 0;
    BEM_HIP(hipMemGetInfo(&free_b, &total_b));
    const size_t have = free_b + c->A64.bytes + c->A32.bytes + c->Kf.bytes + c->near_col.bytes + c->near_row.bytes +
                        c->near_val.bytes;
    if (need > have) throw bem::Error(BEM_ERR_OOM, "assembly needs " + std::to_string(need >> 20) + " MiB, " +
                                                       std::to_string(have >> 20) + " MiB free");
    c->assembled = false;
    if (mixed) {
        c->A64.release();
        c->A32.alloc(sizeof(float) * (size_t)N * ld);
        c->A64.alloc(sizeof(double) * (size_t)(c->n_float > 0 ? c->n_float : 1) * ld);
    } else {
        c->A32.release();
        c->A64.alloc(sizeof(double) * (size_t)n * ld);
    }
    if ((c->opt.constraint_form == 0 || c->has_sheet) && nflt > 0) c->Kf.alloc(sizeof(double) * nflt * N);
    c->nearmask.alloc(sizeof(uint64_t) * nblk * N);
    c->diag.alloc(sizeof(double) * ld);
    bem::launch_far_assemble(c);
    bem::launch_near_csr(c, c->nearmask.as<uint64_t>(), N, c->near_ptr, c->near_row, c->near_col, &c->near_nnz,
                         "near_mask_csr");
    if (mixed) c->near_val.alloc(sizeof(double) * (c->near_nnz > 0 ? c->near_nnz : 1));
    bem::launch_near_assemble(c);
    bem::launch_finalize(c);
    c->nearmask.release();
    if (c->opt.constraint_form == 0 || c->has_sheet) c->Kf.release();
    BEM_HIP(hipStreamSynchronize(c->stream));
    c->assembled = true;
    return BEM_OK;
    API_CATCH
}

bem_status bem_copy_rows(bem_ctx* c, int64_t row0, int64_t n_rows, double* out) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    check_assembled(c);
    if (c->hm) throw bem::Error(BEM_ERR_INVALID, "the compressed operator keeps no dense rows");
    if (row0 < 0 || n_rows < 0 || row0 + n_rows > c->n) throw bem::Error(BEM_ERR_INVALID, "row range out of bounds");
    if (n_rows == 0) return BEM_OK;
    if (!out) throw bem::Error(BEM_ERR_INVALID, "out pointer is NULL");
    bem::launch_copy_rows(c, row0, n_rows, out);
    return BEM_OK;
    API_CATCH
}

bem_status bem_rhs(bem_ctx* c, int32_t nrhs, const double* body_V, double* b) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    if (nrhs < 1 || !body_V || !b) throw bem::Error(BEM_ERR_INVALID, "nrhs >= 1 and non-NULL arrays required");
    for (int64_t k = 0; k < (int64_t)nrhs * c->n_body; ++k)
        if (!std::isfinite(body_V[k])) throw bem::Error(BEM_ERR_INVALID, "non-finite body potential");
    upload(c->gm_b, body_V, (size_t)nrhs * c->n_body, c->stream);
    bem::launch_rhs(c, nrhs, c->gm_b.as<double>(), b);
    BEM_HIP(hipStreamSynchronize(c->stream));   // body_V staging buffer is reused
    return BEM_OK;
    API_CATCH
}

bem_status bem_matvec(bem_ctx* c, int32_t nrhs, const double* x, double* y, int32_t transpose) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    check_assembled(c);
    if (nrhs < 1 || !x || !y) throw bem::Error(BEM_ERR_INVALID, "nrhs >= 1 and non-NULL vectors required");
    if (transpose != 0 && transpose != 1) throw bem::Error(BEM_ERR_INVALID, "transpose must be 0 or 1");
    if (transpose && c->hm) throw bem::Error(BEM_ERR_INVALID, "the compressed operator has no transpose product");
    if (nrhs >= 2 && !transpose && c->batched_solve && !c->hm) {
        for (int32_t r0 = 0; r0 < nrhs; r0 += 64)
            bem::batched_apply_exact(c, (int)std::min<int32_t>(64, nrhs - r0), x + (int64_t)r0 * c->n,
                                     y + (int64_t)r0 * c->n);
        return BEM_OK;
    }
    c->gm_x.alloc(sizeof(double) * c->ld * 2);
    double* xa = c->gm_x.as<double>();
    double* ya = xa + c->ld;
    for (int32_t r = 0; r < nrhs; ++r) {
        BEM_HIP(hipMemcpyAsync(xa, x + (int64_t)r * c->n, sizeof(double) * c->n, hipMemcpyDeviceToDevice, c->stream));
        if (transpose)
            bem::launch_matvec_t(c, xa, ya, c->stream);
        else
            bem::launch_matvec(c, xa, ya, c->stream);
        BEM_HIP(hipMemcpyAsync(y + (int64_t)r * c->n, ya, sizeof(double) * c->n, hipMemcpyDeviceToDevice, c->stream));
    }
    return BEM_OK;
    API_CATCH
}

bem_status bem_matvec_noalloc(bem_ctx* c, int32_t nrhs, const double* x, double* y, int32_t transpose) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    if (nrhs < 1 || !x || !y) throw bem::Error(BEM_ERR_INVALID, "nrhs >= 1 and non-NULL vectors required");
    if (transpose != 0 && transpose != 1) throw bem::Error(BEM_ERR_INVALID, "transpose must be 0 or 1");
    bem::matvec_noalloc(c, nrhs, x, y, transpose);
    return BEM_OK;
    API_CATCH
}

bem_status bem_solve_gmres(bem_ctx* c, int32_t nrhs, const double* body_V, double tol, int32_t max_iter, double* sol,
                           bem_solve_info* info) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    check_assembled(c);
    if (nrhs < 1 || !body_V || !sol) throw bem::Error(BEM_ERR_INVALID, "nrhs >= 1 and non-NULL arrays required");
    if (!(tol > 0.0) || !std::isfinite(tol)) throw bem::Error(BEM_ERR_INVALID, "tol must be finite and > 0");
    if (max_iter < 1) throw bem::Error(BEM_ERR_INVALID, "max_iter must be >= 1");
    for (int64_t k = 0; k < (int64_t)nrhs * c->n_body; ++k)
        if (!std::isfinite(body_V[k])) throw bem::Error(BEM_ERR_INVALID, "non-finite body potential");
    const int64_t n = c->n, ld = c->ld;
    c->gm_b.alloc(sizeof(double) * (ld * 2 + (size_t)nrhs * c->n_body));
    double* bvec = c->gm_b.as<double>();
    double* xvec = bvec + ld;
    double* dV = xvec + ld;
    BEM_HIP(hipMemcpyAsync(dV, body_V, sizeof(double) * nrhs * c->n_body, hipMemcpyHostToDevice, c->stream));
    int total_it = 0, total_ref = 0;
    double worst = 0.0;
    bool all_conv = true;
    if (nrhs >= 2 && c->batched_solve && !c->hm) {
        // groups of up to 64 load cases, one shared matrix product per iteration
        for (int32_t r0 = 0; r0 < nrhs; r0 += 64) {
            const int nr = (int)std::min<int32_t>(64, nrhs - r0);
            c->bg_B.alloc(sizeof(double) * 64 * ld);
            c->bg_X.alloc(sizeof(double) * 64 * ld);
            double* B = c->bg_B.as<double>();
            double* X = c->bg_X.as<double>();
            for (int r = 0; r < nr; ++r)
                bem::launch_rhs(c, 1, dV + (int64_t)(r0 + r) * c->n_body, B + (int64_t)r * ld);
            int it = 0, ref = 0;
            double rr = 0.0;
            const int rc = bem::gmres_solve_batched(c, nr, B, X, tol, max_iter, &it, &rr, &ref);
            for (int r = 0; r < nr; ++r)
                BEM_HIP(hipMemcpyAsync(sol + (int64_t)(r0 + r) * n, X + (int64_t)r * ld, sizeof(double) * n,
                                       hipMemcpyDeviceToDevice, c->stream));
            total_it += it;
            total_ref += ref;
            worst = std::max(worst, rr);
            if (rc != 0) all_conv = false;
        }
    } else {
        for (int32_t r = 0; r < nrhs; ++r) {
            bem::launch_rhs(c, 1, dV + (int64_t)r * c->n_body, bvec);
            int it = 0, ref = 0;
            double rr = 0.0;
            const int rc = bem::gmres_solve(c, bvec, xvec, tol, max_iter, &it, &rr, &ref);
            BEM_HIP(hipMemcpyAsync(sol + (int64_t)r * n, xvec, sizeof(double) * n, hipMemcpyDeviceToDevice,
                                   c->stream));
            total_it += it;
            total_ref += ref;
            worst = std::max(worst, rr);
            if (rc != 0) all_conv = false;
        }
    }
    BEM_HIP(hipStreamSynchronize(c->stream));
    if (info) {
        info->iters = total_it;
        info->rel_residual = worst;
        info->refinements = total_ref;
    }
    if (!all_conv)
        return fail(BEM_ERR_NOCONV, "GMRES stopped at relative residual " + std::to_string(worst) + " after " +
                                        std::to_string(total_it) + " iterations");
    return BEM_OK;
    API_CATCH
}

bem_status bem_eval_field(bem_ctx* c, int32_t nrhs, const double* sol, int64_t P, const double* pts,
                          const int32_t* on_panel, double* phi, double* E) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    if (c->opt.basis == BEM_BASIS_LINEAR) {
        if (nrhs < 1 || !sol || (P > 0 && !phi && !E))
            throw bem::Error(BEM_ERR_INVALID, "nrhs >= 1, non-NULL sol and phi or E required");
        if (on_panel) throw bem::Error(BEM_ERR_INVALID, "the LINEAR basis evaluates at volume points (on_panel NULL)");
        check_points(c, P, pts);
        bem::launch_nodal_field(c, nrhs, sol, P, pts, phi, E);
        return BEM_OK;
    }
    if (nrhs < 1 || !sol || (P > 0 && !E)) throw bem::Error(BEM_ERR_INVALID, "nrhs >= 1 and non-NULL sol, E required");
    check_points(c, P, pts);
    if (on_panel) {
        auto h = fetch_i32(c, on_panel, (size_t)P);
        for (int32_t v : h)
            if (v < -1 || v >= c->N) throw bem::Error(BEM_ERR_INVALID, "on_panel entry out of range");
    }
    for (int32_t r = 0; r < nrhs; ++r)
        bem::launch_eval(c, sol + (int64_t)r * c->n, P, pts, on_panel, phi ? phi + (int64_t)r * P : nullptr,
                         E + (int64_t)r * P * 3);
    return BEM_OK;
    API_CATCH
}

bem_status bem_trace_lines(bem_ctx* c, int32_t nrhs, const double* sol, int64_t L, const int32_t* line_rhs,
                           const double* starts, const bem_trace_params* tp, int32_t* n_steps, int32_t* stop_code,
                           double* path) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    check_trace(c, nrhs, sol, L, line_rhs, starts, tp);
    if (L > 0 && (!n_steps || !stop_code)) throw bem::Error(BEM_ERR_INVALID, "n_steps and stop_code are required");
    bem::launch_trace(c, nrhs, sol, L, line_rhs, starts, tp, n_steps, stop_code, path, nullptr, nullptr);
    return BEM_OK;
    API_CATCH
}

bem_status bem_streamer_integral(bem_ctx* c, int32_t nrhs, const double* sol, int64_t L, const int32_t* line_rhs,
                                 const double* starts, const bem_trace_params* tp, double* integral, int32_t* n_steps,
                                 int32_t* stop_code, uint8_t* exceeds) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    check_trace(c, nrhs, sol, L, line_rhs, starts, tp);
    if (L > 0 && (!integral || !n_steps || !stop_code))
        throw bem::Error(BEM_ERR_INVALID, "integral, n_steps and stop_code are required");
    bem::launch_trace(c, nrhs, sol, L, line_rhs, starts, tp, n_steps, stop_code, nullptr, integral, exceeds);
    return BEM_OK;
    API_CATCH
}

bem_status bem_streamer_grad(bem_ctx* c, int32_t nrhs, const double* sol, int64_t L, const int32_t* line_rhs,
                             const double* starts, const int32_t* start_panel, const double* start_bary,
                             const bem_trace_params* tp, const double* dJ_dI, double tol, double* dJ_dvert,
                             double* dJ_dV, double* dJ_dstart) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    if (!c->assembled) throw bem::Error(BEM_ERR_STATE, "assemble the system first");
    if (c->opt.precision != BEM_FP64) throw bem::Error(BEM_ERR_INVALID, "the gradient needs precision FP64");
    if (c->opt.basis != BEM_BASIS_CONSTANT) throw bem::Error(BEM_ERR_INVALID, "the gradient needs the CONSTANT basis");
    check_trace(c, nrhs, sol, L, line_rhs, starts, tp);
    if (!(tp->alpha_p >= 1.0)) throw bem::Error(BEM_ERR_INVALID, "the gradient needs alpha_p >= 1");
    if (!(tol > 0.0) || !(tol < 1.0)) throw bem::Error(BEM_ERR_INVALID, "tol must be in (0, 1)");
    if (!dJ_dvert || !dJ_dV) throw bem::Error(BEM_ERR_INVALID, "dJ_dvert and dJ_dV are required");
    if (L > 0 && !dJ_dI) throw bem::Error(BEM_ERR_INVALID, "dJ_dI is required");
    if (start_panel) {
        if (L > 0 && !start_bary) throw bem::Error(BEM_ERR_INVALID, "start_bary is required with start_panel");
        auto h = fetch_i32(c, start_panel, (size_t)L);
        for (int32_t v : h)
            if (v < 0 || v >= c->N) throw bem::Error(BEM_ERR_INVALID, "start_panel entry out of range");
    }
    bem::streamer_grad(c, nrhs, sol, L, line_rhs, starts, start_panel, start_bary, tp, dJ_dI, tol, dJ_dvert, dJ_dV,
                       dJ_dstart);
    return BEM_OK;
    API_CATCH
}

bem_status bem_panel_points(bem_ctx* c, int64_t L, const int32_t* panel, const double* bary, double offset,
                            double* out) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    if (L < 0 || L >= ((int64_t)1 << 31)) throw bem::Error(BEM_ERR_INVALID, "point count out of range");
    if (L > 0 && (!panel || !bary || !out)) throw bem::Error(BEM_ERR_INVALID, "panel, bary and out are required");
    if (!std::isfinite(offset)) throw bem::Error(BEM_ERR_INVALID, "offset must be finite");
    auto hp = fetch_i32(c, panel, (size_t)L);
    for (int32_t v : hp)
        if (v < 0 || v >= c->N) throw bem::Error(BEM_ERR_INVALID, "panel entry out of range");
    auto hb = fetch_f64(c, bary, (size_t)L * 3);
    for (double v : hb)
        if (!std::isfinite(v)) throw bem::Error(BEM_ERR_INVALID, "non-finite barycentric coordinate");
    bem::launch_panel_points(c, L, panel, bary, offset, out);
    return BEM_OK;
    API_CATCH
}

bem_status bem_compress(bem_ctx* c, double eps, double eta_adm, int32_t leaf, bem_compress_info* info) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    if (c->opt.basis != BEM_BASIS_CONSTANT || c->opt.precision != BEM_FP64)
        throw bem::Error(BEM_ERR_INVALID, "compression needs the CONSTANT basis in FP64");
    if (!(eps > 0.0 && eps < 1.0)) throw bem::Error(BEM_ERR_INVALID, "eps must lie in (0, 1)");
    if (!(eta_adm > 0.0) || !std::isfinite(eta_adm)) throw bem::Error(BEM_ERR_INVALID, "eta_adm must be finite and > 0");
    if (leaf < 8 || leaf > 256) throw bem::Error(BEM_ERR_INVALID, "leaf must lie in 8..256");
    // the dense operator is released first: the compressed one is built in its place
    c->assembled = false;
    c->A64.release();
    c->A32.release();
    c->Kf.release();
    c->nearmask.release();
    bem::HmStats st{};
    bem::hmatrix_build(c, eps, eta_adm, leaf, &st);
    c->near_nnz = 0;
    c->assembled = true;
    if (info) {
        info->blocks = st.blocks;
        info->lowrank_blocks = st.lowrank_blocks;
        info->dense_entries = st.dense_entries;
        info->factor_entries = st.factor_entries;
        info->max_rank = st.max_rank;
    }
    return BEM_OK;
    API_CATCH
}

bem_status bem_pair_integrals(bem_ctx* c, int64_t P, const double* pts, const int32_t* panel, int32_t rule,
                              double* S, double* F) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    if (P < 0 || P >= ((int64_t)1 << 31)) throw bem::Error(BEM_ERR_INVALID, "pair count out of range");
    if (rule != 0 && rule != 1) throw bem::Error(BEM_ERR_INVALID, "rule must be 0 (closed forms) or 1 (Duffy)");
    if (P > 0 && (!pts || !panel || !S)) throw bem::Error(BEM_ERR_INVALID, "pts, panel and S are required");
    auto hp = fetch_i32(c, panel, (size_t)P);
    for (int32_t v : hp)
        if (v < 0 || v >= c->N) throw bem::Error(BEM_ERR_INVALID, "panel entry out of range");
    auto hx = fetch_f64(c, pts, (size_t)P * 3);
    for (double v : hx)
        if (!std::isfinite(v)) throw bem::Error(BEM_ERR_INVALID, "non-finite point coordinate");
    bem::launch_pair_integrals(c, P, pts, panel, rule, S, F, 3);
    return BEM_OK;
    API_CATCH
}

bem_status bem_quad_pair_integrals(bem_ctx* c, int64_t P, const double* pts, const double* nodes, double* S,
                                   double* F) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    if (P < 0 || P >= ((int64_t)1 << 31)) throw bem::Error(BEM_ERR_INVALID, "pair count out of range");
    if (P > 0 && (!pts || !nodes || !S)) throw bem::Error(BEM_ERR_INVALID, "pts, nodes and S are required");
    if (P == 0) return BEM_OK;
    auto hx = fetch_f64(c, pts, (size_t)P * 3);
    for (double v : hx)
        if (!std::isfinite(v)) throw bem::Error(BEM_ERR_INVALID, "non-finite point coordinate");
    auto hn = fetch_f64(c, nodes, (size_t)P * 18);
    for (int64_t p = 0; p < P; ++p) {
        const double* q = hn.data() + 18 * p;
        for (int k = 0; k < 18; ++k)
            if (!std::isfinite(q[k])) throw bem::Error(BEM_ERR_INVALID, "non-finite panel node");
        double e1[3], e2[3], cr[3], l1 = 0.0, l2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            e1[k] = q[3 + k] - q[k];
            e2[k] = q[6 + k] - q[k];
            l1 += e1[k] * e1[k];
            l2 += e2[k] * e2[k];
        }
        cr[0] = e1[1] * e2[2] - e1[2] * e2[1];
        cr[1] = e1[2] * e2[0] - e1[0] * e2[2];
        cr[2] = e1[0] * e2[1] - e1[1] * e2[0];
        const double a2 = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        if (!(a2 > 1e-14 * std::max(l1, l2))) throw bem::Error(BEM_ERR_INVALID, "curved panel without area");
    }
    bem::launch_quad_pair_integrals(c, P, pts, nodes, S, F);
    return BEM_OK;
    API_CATCH
}

bem_status bem_set_tuning(bem_ctx* c, const char* key, int64_t value) {
    if (!c || !key) return fail(BEM_ERR_INVALID, "NULL argument");
    if (std::strcmp(key, "trace_mode") == 0) {
        if (value < 0 || value > 3) return fail(BEM_ERR_INVALID, "trace_mode must be 0, 1, 2 or 3");
        c->trace_mode = (int32_t)value;
        return BEM_OK;
    }
    if (std::strcmp(key, "batched_solve") == 0) {
        if (value < 0 || value > 1) return fail(BEM_ERR_INVALID, "batched_solve must be 0 or 1");
        c->batched_solve = (int32_t)value;
        return BEM_OK;
    }
    if (std::strcmp(key, "near_rule") == 0) {
        if (value < 0 || value > 1) return fail(BEM_ERR_INVALID, "near_rule must be 0 or 1");
        if (value == 1 && c->opt.basis != BEM_BASIS_CONSTANT)
            return fail(BEM_ERR_INVALID, "near_rule 1 applies to the CONSTANT basis");
        c->near_rule = (int32_t)value;
        return BEM_OK;
    }
    struct Knob {
        const char* name;
        int32_t bem_ctx::*field;
        int64_t lo, hi;
        bool pow2_choice;
    };
    static const Knob knobs[] = {
        {"far_rows", &bem_ctx::tune_far_rows, 32, 128, true},     {"gemv_rows", &bem_ctx::tune_gemv_rows, 2, 16, true},
        {"gemm_blocks", &bem_ctx::tune_gemm_blocks, 64, 65536, false},
        {"eval_blocks", &bem_ctx::tune_eval_blocks, 64, 65536, false},
        {"trace_split", &bem_ctx::tune_trace_split, 0, 4096, false},
        {"trace_tile", &bem_ctx::tune_trace_tile, 64, 256, true},
        {"trace_few", &bem_ctx::tune_trace_few, 0, 16, false},
        {"trace_splitk", &bem_ctx::tune_trace_splitk, 2, 8, true},
        {"trace_groups", &bem_ctx::tune_trace_groups, 0, 2, false},
        {"trace_fold", &bem_ctx::tune_trace_fold, 0, 1, false},
        {"trace_lpb", &bem_ctx::tune_trace_lpb, 0, 8, true},
        {"trace_rnd", &bem_ctx::tune_trace_rnd, 0, 4, true},
        {"trace_tail", &bem_ctx::tune_trace_tail, 0, 4096, false},
        {"trace_loop", &bem_ctx::tune_trace_loop, 0, 4096, false},
        {"trace_spin", &bem_ctx::tune_trace_spin, 0, 1 << 30, false},
        {"grad_batch", &bem_ctx::grad_batch, 64, 1 << 24, false},
    };
    for (const Knob& k : knobs)
        if (std::strcmp(key, k.name) == 0) {
            const bool ok = value >= k.lo && value <= k.hi && (!k.pow2_choice || (value & (value - 1)) == 0);
            if (!ok) return fail(BEM_ERR_INVALID, std::string("value out of range for ") + key);
            c->*(k.field) = (int32_t)value;
            return BEM_OK;
        }
    return fail(BEM_ERR_INVALID, std::string("unknown tuning key ") + key);
}

bem_status bem_get_tuning(const bem_ctx* c, const char* key, int64_t* value) {
    if (!c || !key || !value) return fail(BEM_ERR_INVALID, "NULL argument");
    if (std::strcmp(key, "trace_mode") == 0) *value = c->trace_mode;
    else if (std::strcmp(key, "batched_solve") == 0) *value = c->batched_solve;
    else if (std::strcmp(key, "near_rule") == 0) *value = c->near_rule;
    else if (std::strcmp(key, "far_rows") == 0) *value = c->tune_far_rows;
    else if (std::strcmp(key, "gemv_rows") == 0) *value = c->tune_gemv_rows;
    else if (std::strcmp(key, "gemm_blocks") == 0) *value = c->tune_gemm_blocks;
    else if (std::strcmp(key, "eval_blocks") == 0) *value = c->tune_eval_blocks;
    else if (std::strcmp(key, "trace_split") == 0) *value = c->tune_trace_split;
    else if (std::strcmp(key, "grad_batch") == 0) *value = c->grad_batch;
    else if (std::strcmp(key, "trace_tile") == 0) *value = c->tune_trace_tile;
    else if (std::strcmp(key, "trace_few") == 0) *value = c->tune_trace_few;
    else if (std::strcmp(key, "trace_splitk") == 0) *value = c->tune_trace_splitk;
    else if (std::strcmp(key, "trace_groups") == 0) *value = c->tune_trace_groups;
    else if (std::strcmp(key, "trace_fold") == 0) *value = c->tune_trace_fold;
    else if (std::strcmp(key, "trace_lpb") == 0) *value = c->tune_trace_lpb;
    else if (std::strcmp(key, "trace_rnd") == 0) *value = c->tune_trace_rnd;
    else if (std::strcmp(key, "trace_tail") == 0) *value = c->tune_trace_tail;
    else if (std::strcmp(key, "trace_loop") == 0) *value = c->tune_trace_loop;
    else if (std::strcmp(key, "trace_spin") == 0) *value = c->tune_trace_spin;
    else return fail(BEM_ERR_INVALID, std::string("unknown tuning key ") + key);
    return BEM_OK;
}

bem_status bem_autotune(bem_ctx* c, const char* cache_path, int32_t* from_cache) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    if (c->opt.basis != BEM_BASIS_CONSTANT) throw bem::Error(BEM_ERR_INVALID, "the autotuner needs the CONSTANT basis");
    const int r = bem::autotune(c, cache_path);
    if (from_cache) *from_cache = r;
    return BEM_OK;
    API_CATCH
}

bem_status bem_set_profiling(bem_ctx* c, int32_t enable) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    if (enable < 0 || enable > 2) return fail(BEM_ERR_INVALID, "profiling mode must be 0, 1 or 2");
    c->profiling = enable;
    return BEM_OK;
}

bem_status bem_kernel_stats(bem_ctx* c, const char* name, int64_t* launches, double* total_ms) {
    if (!c || !name || !launches || !total_ms) return fail(BEM_ERR_INVALID, "NULL argument");
    DeviceGuard g(c->device);
    API_TRY
    bem::resolve_stats(c);
    auto it = c->stats.find(name);
    *launches = it == c->stats.end() ? 0 : it->second.launches;
    *total_ms = it == c->stats.end() ? 0.0 : it->second.ms;
    return BEM_OK;
    API_CATCH
}

bem_status bem_reset_stats(bem_ctx* c) {
    if (!c) return fail(BEM_ERR_INVALID, "NULL context");
    DeviceGuard g(c->device);
    API_TRY
    bem::resolve_stats(c);
    c->stats.clear();
    c->trace_far_launches = 0;
    c->trace_pass_launches = 0;
    BEM_HIP(hipMemsetAsync(c->counters.p, 0, sizeof(uint64_t) * 8, c->stream));
    BEM_HIP(hipStreamSynchronize(c->stream));
    return BEM_OK;
    API_CATCH
}

bem_status bem_get_counter(bem_ctx* c, const char* name, int64_t* value) {
    if (!c || !name || !value) return fail(BEM_ERR_INVALID, "NULL argument");
    DeviceGuard g(c->device);
    API_TRY
    if (std::strcmp(name, "trace_far_launches") == 0) {
        *value = c->trace_far_launches;
        return BEM_OK;
    }
    if (std::strcmp(name, "trace_pass_launches") == 0) {
        *value = c->trace_pass_launches;
        return BEM_OK;
    }
    int idx = -1;
    if (std::strcmp(name, "trace_near_pairs") == 0) idx = 0;
    if (std::strcmp(name, "trace_far_pairs") == 0) idx = 1;
    if (std::strcmp(name, "trace_pass_near_pairs") == 0) idx = 2;
    if (std::strcmp(name, "trace_pass_pairs") == 0) idx = 3;
    if (idx < 0) throw bem::Error(BEM_ERR_INVALID, std::string("unknown counter ") + name);
    uint64_t v = 0;
    BEM_HIP(hipMemcpyAsync(&v, c->counters.as<uint64_t>() + idx, sizeof(v), hipMemcpyDeviceToHost, c->stream));
    BEM_HIP(hipStreamSynchronize(c->stream));
    *value = (int64_t)v;
    return BEM_OK;
    API_CATCH
}

}  // extern "C"
