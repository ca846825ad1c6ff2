// Autotuner: picks the tile shapes of the hot kernels by timing candidates on
// the context's own assembled problem, and keeps the choice in a JSON cache.
//
// Knobs (none changes a result beyond summation order):
//   far_rows     collocation rows per block of the far-field assembly   {32, 64, 128}
//   gemv_rows    matrix rows per block of the GMRES matvec             {2, 4, 8}
//   gemm_blocks  minimum blocks of the FP32 multi-vector product       {512, 1024, 2048} (MIXED)
//   eval_blocks  target blocks of the field evaluation                 {1024, 2048, 4096}
//   trace_tile   lines per block of an unsplit field-line pass            {64, 128, 256} (at 256 lines)
//   trace_splitk waves splitting each panel chunk in a split field-line pass {2, 4, 8} (at 256 lines)
//   trace_split  live-line count at or below which a field-line pass splits each panel chunk over
//                eight waves; the largest of {0, 32, 64, 128, 256} at which the split pass is faster
//   trace_few    live-line count at or below which the panel-stationary pass is used: the largest
//                of {0, 2, 4, 8, 16} at which its far part beats the other far passes
// Each candidate runs once to warm up and is then timed three times with HIP
// events on the context stream (best of three); a candidate replaces the
// default only when it is more than 3 % faster.  Cache: a JSON object keyed by "<arch> N=<panels> n=<unknowns>
// precision=<0|1> eta=<eta>", one entry per line, read and rewritten whole.
#include <algorithm>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "bem_device.h"

extern "C" bem_status bem_assemble(bem_ctx* ctx);

namespace bem {

void launch_gemm_f32(bem_ctx* c, const float* A, int64_t lda, int64_t M, int64_t K, const float* Zt, int64_t ldz,
                     int ncols, double* Y, int64_t ldy, bool accumulate);
double time_far_pass(bem_ctx* c, int64_t L, bool split, int tile_lines, int splitk, const double* pts,
                     const double* sol);

namespace {

__global__ void k_tune_fill(double* __restrict__ x, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = v;
}
__global__ void k_tune_fill_f(float* __restrict__ x, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) x[i] = v;
}
// points just off the panels: centroid + 1e-3 R n (valid field points near the surface)
__global__ void k_tune_points(const double* __restrict__ tri64, int64_t P, double* __restrict__ pts) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= P) return;
    const double* T = tri64 + (int64_t)TRI_REC * i;
    const double s = 1e-3 * sqrt(T[TR_A]);
#pragma unroll
    for (int k = 0; k < 3; ++k) pts[3 * i + k] = T[TR_C + k] + s * T[TR_N + k];
}

template <typename F>
double time_ms(bem_ctx* c, F&& f) {
    hipEvent_t a, b;
    BEM_HIP(hipEventCreate(&a));
    BEM_HIP(hipEventCreate(&b));
    f();   // warm-up
    double best = 1e30;
    for (int rep = 0; rep < 3; ++rep) {
        BEM_HIP(hipEventRecord(a, c->stream));
        f();
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

// A candidate replaces the default only when it is faster by more than 3 %, so that timing
// noise does not flip the choice between runs.
constexpr double HYST = 0.97;

int choose(const std::vector<int>& cand, const std::vector<double>& t, int dflt) {
    double td = 1e30;
    for (size_t i = 0; i < cand.size(); ++i)
        if (cand[i] == dflt) td = t[i];
    int best = dflt;
    double tb = td;
    for (size_t i = 0; i < cand.size(); ++i)
        if (t[i] < HYST * td && t[i] < tb) {
            tb = t[i];
            best = cand[i];
        }
    return best;
}

template <typename Set>
int pick(bem_ctx* c, const std::vector<int>& cand, int dflt, Set&& set_and_run) {
    std::vector<double> t;
    for (int v : cand) t.push_back(time_ms(c, [&] { set_and_run(v); }));
    return choose(cand, t, dflt);
}

constexpr int NKNOB = 8;
const char* KNOBS[NKNOB] = {"far_rows",   "gemv_rows",    "gemm_blocks", "eval_blocks",
                            "trace_tile", "trace_splitk", "trace_split", "trace_few"};

int32_t* knob(bem_ctx* c, int k) {
    switch (k) {
        case 0: return &c->tune_far_rows;
        case 1: return &c->tune_gemv_rows;
        case 2: return &c->tune_gemm_blocks;
        case 3: return &c->tune_eval_blocks;
        case 4: return &c->tune_trace_tile;
        case 5: return &c->tune_trace_splitk;
        case 6: return &c->tune_trace_split;
        default: return &c->tune_trace_few;
    }
}

std::string cache_key(bem_ctx* c) {
    hipDeviceProp_t prop;
    BEM_HIP(hipGetDeviceProperties(&prop, c->device));
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s N=%lld n=%lld precision=%d eta=%.6g", arch.c_str(), (long long)c->N,
                  (long long)c->n, (int)c->opt.precision, c->opt.eta);
    return buf;
}

// lines of the cache file: `"<key>": {"far_rows": 64, ...},`
bool parse_line(const std::string& line, std::string& key, int (&vals)[NKNOB]) {
    const size_t q0 = line.find('"');
    if (q0 == std::string::npos) return false;
    const size_t q1 = line.find('"', q0 + 1);
    if (q1 == std::string::npos || line.find('{', q1) == std::string::npos) return false;
    key = line.substr(q0 + 1, q1 - q0 - 1);
    for (int k = 0; k < NKNOB; ++k) {
        const std::string pat = std::string("\"") + KNOBS[k] + "\":";
        const size_t p = line.find(pat, q1);
        if (p == std::string::npos) return false;
        vals[k] = std::atoi(line.c_str() + p + pat.size());
    }
    return true;
}

bool valid_value(int k, int v) {
    switch (k) {
        case 0: return v == 32 || v == 64 || v == 128;
        case 1: return v == 2 || v == 4 || v == 8;
        case 2: return v >= 64 && v <= 65536;
        case 3: return v >= 64 && v <= 65536;
        case 4: return v == 64 || v == 128 || v == 256;
        case 5: return v == 2 || v == 4 || v == 8;
        case 6: return v >= 0 && v <= 4096;
        default: return v >= 0 && v <= 16;
    }
}

}  // namespace

// Returns 1 if the choice came from the cache, 0 if it was timed now.
int autotune(bem_ctx* c, const char* cache_path) {
    if (!c->assembled) throw Error(BEM_ERR_STATE, "assemble the system before tuning");
    const std::string key = cache_key(c);
    std::vector<std::pair<std::string, std::vector<int>>> entries;
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            std::string k;
            int v[NKNOB];
            if (parse_line(line, k, v)) entries.push_back({k, std::vector<int>(v, v + NKNOB)});
        }
        for (auto& e : entries)
            if (e.first == key) {
                bool ok = true;
                for (int k = 0; k < NKNOB; ++k) ok = ok && valid_value(k, e.second[k]);
                if (!ok) throw Error(BEM_ERR_INVALID, std::string("invalid tuning cache entry in ") + cache_path);
                for (int k = 0; k < NKNOB; ++k) *knob(c, k) = e.second[k];
                return 1;
            }
    }
    const int64_t N = c->N, ld = c->ld;
    const bool mixed = c->opt.precision == BEM_MIXED;
    hipStream_t s = c->stream;
    DBuf x, y, z, pts;
    x.alloc(sizeof(double) * 64 * ld);
    y.alloc(sizeof(double) * 64 * ld);
    auto fill = [&](double* p, int64_t cnt, double v) {
        hipLaunchKernelGGL(k_tune_fill, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, s, p, cnt, v);
        BEM_CHECK_LAUNCH();
    };
    fill(x.as<double>(), 64 * ld, 1.0);
    // far-field assembly (needs the near masks and the floating K' block, released after assembly)
    {
        const int64_t nblk = ceil_div(N, 64);
        c->nearmask.alloc(sizeof(uint64_t) * nblk * N);
        if ((c->opt.constraint_form == 0 || c->has_sheet) && !c->h_rows_flt.empty())
            c->Kf.alloc(sizeof(double) * c->h_rows_flt.size() * N);
        c->tune_far_rows = pick(c, {32, 64, 128}, 64, [&](int v) {
            c->tune_far_rows = v;
            launch_far_assemble(c);
        });
    }
    // matvec
    c->tune_gemv_rows = pick(c, {2, 4, 8}, 4, [&](int v) {
        c->tune_gemv_rows = v;
        launch_matvec(c, x.as<double>(), y.as<double>(), s);
    });
    // FP32 multi-vector product (mixed mode)
    if (mixed) {
        z.alloc(sizeof(float) * 64 * ld);
        hipLaunchKernelGGL(k_tune_fill_f, dim3((unsigned)ceil_div(64 * ld, 256)), dim3(256), 0, s, z.as<float>(),
                           64 * ld, 1.0f);
        BEM_CHECK_LAUNCH();
        c->tune_gemm_blocks = pick(c, {512, 1024, 2048}, 1024, [&](int v) {
            c->tune_gemm_blocks = v;
            launch_gemm_f32(c, c->A32.as<float>(), ld, N, ld, z.as<float>(), ld, 64, y.as<double>(), ld, false);
        });
    }
    // field evaluation at N points just off the panels
    pts.alloc(sizeof(double) * 3 * N);
    hipLaunchKernelGGL(k_tune_points, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, s, c->tri64.as<double>(), N,
                       pts.as<double>());
    BEM_CHECK_LAUNCH();
    c->tune_eval_blocks = pick(c, {1024, 2048, 4096}, 2048, [&](int v) {
        c->tune_eval_blocks = v;
        launch_eval(c, x.as<double>(), N, pts.as<double>(), nullptr, nullptr, y.as<double>());
    });
    // field-line pass: lines per block at 256 live lines, then split or not at 32..256 live lines
    {
        const int64_t Lt = std::min<int64_t>(N, 256);
        std::vector<double> tt;
        for (int tile : {64, 128, 256}) tt.push_back(time_far_pass(c, Lt, false, tile, 8, pts.as<double>(), x.as<double>()));
        const int best_tile = choose({64, 128, 256}, tt, 256);
        c->tune_trace_tile = best_tile;
        tt.clear();
        for (int k : {2, 4, 8}) tt.push_back(time_far_pass(c, Lt, true, 64, k, pts.as<double>(), x.as<double>()));
        const int best_k = choose({2, 4, 8}, tt, 8);
        c->tune_trace_splitk = best_k;
        int thr = 0;
        for (int64_t L : {32, 64, 128, 256}) {
            if (L > N) break;
            const double t_split = time_far_pass(c, L, true, 64, best_k, pts.as<double>(), x.as<double>());
            const double t_full = time_far_pass(c, L, false, best_tile, best_k, pts.as<double>(), x.as<double>());
            if (t_split < t_full) thr = (int)L;
        }
        c->tune_trace_split = thr;
        int few = 0;
        for (int64_t L : {2, 4, 8, 16}) {
            if (L > N) break;
            const double t_few = time_far_pass(c, L, false, 0, best_k, pts.as<double>(), x.as<double>());
            const bool use_split = L <= thr;
            const double t_other =
                time_far_pass(c, L, use_split, best_tile, best_k, pts.as<double>(), x.as<double>());
            if (t_few < t_other) few = (int)L;
        }
        c->tune_trace_few = few;
    }
    BEM_HIP(hipStreamSynchronize(s));
    // the far-assembly candidates overwrote the matrix without its near entries: assemble again
    const bem_status rs = bem_assemble(c);
    if (rs != BEM_OK) throw Error(rs, "re-assembly after tuning failed");
    if (cache_path) {
        std::vector<int> mine(NKNOB);
        for (int k = 0; k < NKNOB; ++k) mine[k] = *knob(c, k);
        bool found = false;
        for (auto& e : entries)
            if (e.first == key) {
                e.second = mine;
                found = true;
            }
        if (!found) entries.push_back({key, mine});
        std::ostringstream os;
        os << "{\n";
        for (size_t i = 0; i < entries.size(); ++i) {
            os << "\"" << entries[i].first << "\": {";
            for (int k = 0; k < NKNOB; ++k)
                os << (k ? ", " : "") << "\"" << KNOBS[k] << "\": " << entries[i].second[k];
            os << "}" << (i + 1 < entries.size() ? "," : "") << "\n";
        }
        os << "}\n";
        const std::string tmp = std::string(cache_path) + ".tmp";
        {
            std::ofstream out(tmp, std::ios::trunc);
            if (!out) throw Error(BEM_ERR_INVALID, std::string("cannot write tuning cache ") + tmp);
            out << os.str();
        }
        if (std::rename(tmp.c_str(), cache_path) != 0)
            throw Error(BEM_ERR_INVALID, std::string("cannot replace tuning cache ") + cache_path);
    }
    return 0;
}

}  // namespace bem
