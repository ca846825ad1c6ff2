// Internal declarations of the gfx950 BEM library: context layout, device
// buffers and the host-side launchers of every kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "../../include/bem.h"

namespace bem {

// ---- error plumbing -------------------------------------------------------
struct Error : std::runtime_error {
    bem_status code;
    Error(bem_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define BEM_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            throw ::bem::Error(BEM_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define BEM_CHECK_LAUNCH() BEM_HIP(hipGetLastError())

// ---- device buffer with ownership -----------------------------------------
struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t b) {
        if (b <= bytes && p) return;
        release();
        if (b == 0) return;
        BEM_HIP(hipMalloc(&p, b));
        bytes = b;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// ---- pinned host buffer (staging of small device-to-host reads) ----------
struct HBuf {
    void* p = nullptr;
    size_t bytes = 0;
    HBuf() = default;
    HBuf(const HBuf&) = delete;
    HBuf& operator=(const HBuf&) = delete;
    ~HBuf() { release(); }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        bytes = 0;
    }
    void alloc(size_t b) {
        if (b <= bytes && p) return;
        release();
        BEM_HIP(hipHostMalloc(&p, b, hipHostMallocDefault));
        bytes = b;
    }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// ---- layout constants ----------------------------------------------------
// Far-field record of one panel (FP64 or FP32), 32 values:
//   [0..6] node x, [7..13] node y, [14..20] node z, [21..27] weight * area / (4 pi),
//   [28..30] circumcentre, [31] (eta * R)^2.
// Held component-major (far64/far32: value c of panel j at c * Np + j, for coalesced
// one-panel-per-lane reads) and panel-major (pan64/pan32: at FAR_REC * j + c, for reads of a
// whole record at a wave-uniform address through the scalar cache).
constexpr int FAR_REC = 32;
constexpr int FR_X = 0, FR_Y = 7, FR_Z = 14, FR_W = 21, FR_CC = 28, FR_RR = 31;
// Exact-geometry record of one panel (FP64), 16 values:
//   [0..8] v1 v2 v3, [9..11] unit normal, [12..14] centroid, [15] area.
constexpr int TRI_REC = 16;
constexpr int TR_V = 0, TR_N = 9, TR_C = 12, TR_A = 15;

struct KStat {
    int64_t launches = 0;
    double ms = 0.0;
};

}  // namespace bem

namespace bem {
struct HMatrix;   // compressed operator (hmatrix.hip)
struct HmStats {
    int64_t blocks, lowrank_blocks, dense_entries, factor_entries, max_rank;
};
}  // namespace bem

struct bem_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // second stream of the field-line tracer (line groups advance on both streams) and the
    // events that order it after / before the context stream; created on first use
    hipStream_t aux_stream = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    hipEvent_t lf_ev[8] = {};   // live-count read-backs of the one-launch-per-stage tracer
    hipEvent_t lb_ev[4] = {};   // live-count read-backs of the two-kernel tracer (2 checkpoints x 2 groups)
    bem_options opt{};
    int64_t N = 0, n = 0, ld = 0, n_vert = 0;
    // rows that carry a body's density: N panels, or n_vert vertices for the LINEAR basis; in
    // MIXED mode they are the FP32 block and the constraint rows after them stay FP64
    int64_t nb = 0;
    int32_t n_body = 0, n_float = 0;
    double shift[3] = {0, 0, 0};   // mesh translated by -shift on the device (FP32 accuracy)
    double min_R = 0.0;

    std::vector<int32_t> h_tri, h_tri_body, h_body_kind, h_body_fidx;   // h_body_kind: as given (sheets kept)
    bool has_sheet = false;   // some floating body is a thin sheet (its constraint row needs the K' block)
    std::vector<double> h_epsp, h_epsm;
    // per floating body f (index fidx): the constraint row after its scaling is
    // sum_i a_i (c_self sigma_i + c_kp (K' sigma)_i) / sum_i a_i, with (c_self, c_kp) at [2f], [2f+1]:
    // closed body (1/2, 1) literal or (1, 0) reduced, sheet (1, 2 (eps+ - eps-) / (eps+ + eps-))
    std::vector<double> h_flt_coef;
    // nodal basis (opt.basis == BEM_BASIS_LINEAR): body of each vertex and the fan of each
    // vertex, fan[fan_ptr[k] .. fan_ptr[k+1]) = (triangle << 2) | local index, triangles ascending
    std::vector<int32_t> h_vert_body;
    std::vector<int32_t> h_rows_pot, h_rows_int, h_rows_flt;   // row segments by kind (Sec. 4)

    bem::DBuf vert, tri, tri_body, body_kind, body_epsp, body_epsm, body_fidx, flt_coef;
    bem::DBuf vert_body, fan_ptr, fan, nodal_mass, nodal_bounds, row_order;   // nodal basis only
    // per group of 16 consecutive vertex columns: the triangles holding one of its vertices
    // (ascending) and the local column of each corner (8 bits each, 0xff outside the group)
    bem::DBuf grp_ptr, grp_tri, grp_loc;
    bem::DBuf nod_pan64, nod_far64, nod_ones;   // nodal density folded into the panel records (field lines)
    // nodal rows that need n . E, taken at triangle centroids: the centroid rows (triangles of
    // interface bodies, then of floating bodies whose row has a K' term, grouped by body), the
    // triangle -> centroid row map (-1), the interface vertices, each floating body's centroid-row
    // range and the list of floating bodies with a K' term; Kc is their normal-field matrix
    std::vector<int32_t> h_crow_tri, h_iface_v, h_flt_crange, h_flt_kp;
    bem::DBuf nod_trow, nod_tri_crow, nod_iface_v, nod_frange, nod_flist, nod_Kc;
    bem::DBuf tr_cases;                          // staging of the nodal basis's per-load-case line runs
    bem::DBuf far64, far32, tri64;
    bem::DBuf pan64, pan32;                 // far64 / far32 panel-major: [Np][FAR_REC]
    bem::DBuf rows_pot, rows_int, rows_flt, row_slot;
    bem::DBuf A64, A32, Kf;                 // dense operator (FP64 or FP32) and the K' block of floating rows
    bem::DBuf cons_part;                    // slab sums of a floating body's constraint row
    bem::DBuf nearmask, near_ptr, near_row, near_col, near_val;
    bem::DBuf diag;
    int64_t near_nnz = 0;
    bool assembled = false;

    // scratch
    bem::DBuf gm_V, gm_w, gm_z, gm_h, gm_part, gm_x, gm_r, gm_b, gm_misc;
    bem::HBuf host_stage;
    bem::DBuf ev_part, ev_mask, ev_ptr, ev_col, ev_row, ev_tmp, tr_queue, lb_state, lb_part, lf_part, lf_loop, lf_cnt;

    bem::DBuf bg_V, bg_W, bg_part, bg_small, bg_z, bg_B, bg_X, gemm_part, rows_part;   // batched GMRES
    bem::DBuf near_sf;   // S, F of the near list by the near-singular rule (near_rule 1)
    bem::HMatrix* hm = nullptr;   // compressed operator in use (bem_compress), else the dense matrix

    // gradient of the streamer integrals
    bem::DBuf ad_state, ad_part, ad_mask, ad_cnt, ad_self, ad_ppart, ad_list, ad_path, ad_stage, ad_geo, ad_seg,
        ad_vptr, ad_vcorner;

    // kernel-side launch timing (profiling mode 2): KCLK_SUB word pairs per launch slot, the
    // statistic each used slot feeds, the device's wall-clock rate (kHz)
    bem::DBuf kclk, kclk_dur;
    int64_t kclk_cap = 0;
    std::vector<std::string> kclk_names;
    int kclk_khz = 0;

    // device counters (bem_get_counter): near [0] and regular [1] pairs of the two-kernel field-line
    // passes, near [2] and regular [3] pairs of the one-launch passes
    bem::DBuf counters;
    int64_t trace_far_launches = 0;   // host-side count of two-kernel field-line far passes (bem_get_counter)
    int64_t trace_pass_launches = 0;  // host-side count of one-launch field-line stages (bem_get_counter)

    // tuning knobs (bem_set_tuning)
    // field-line layout: 1 all lines together, a far pass and a step kernel per stage; 2 persistent
    // per-line workgroups; 3 all lines together, one launch per stage; 0 (default) 1 until at most
    // tune_trace_tail lines are live, then 3 (1 throughout when the panel count exceeds what 3 takes)
    int32_t trace_mode = 0;
    int32_t near_rule = 0;       // near pairs of the assembly: 0 closed forms, 1 the Sec. 4 rule (closest point + Duffy)
    int32_t batched_solve = 1;   // several right-hand sides: 1 one batched solve (shared matrix products), 0 one by one
    // tile shapes (bem_set_tuning / bem_autotune); none changes a result beyond summation order
    int32_t tune_far_rows = 64;       // collocation rows per block of the far-field assembly
    int32_t tune_gemv_rows = 4;       // matrix rows per block of the GMRES matvec (2, 4, 8)
    int32_t tune_gemm_blocks = 1024;  // minimum blocks of the FP32 multi-vector product (K ranges)
    int32_t tune_eval_blocks = 2048;  // target blocks of the field evaluation (panel-range split)
    int32_t tune_trace_split = 64;    // live-line count at or below which field-line passes split chunks
    int32_t tune_trace_tile = 256;    // lines per block of an unsplit field-line pass (64, 128, 256)
    int32_t tune_trace_splitk = 8;    // waves that split a panel chunk in a split field-line pass (2, 4, 8)
    int32_t tune_trace_few = 8;       // live-line count at or below which the panel-stationary pass is used (<= 16)
    int32_t tune_trace_groups = 0;    // line groups of a field-line run, each on its own stream (1 or 2; 0: 2 from 128 lines)
    int32_t tune_trace_fold = 1;      // fold the second line group into the first once all live lines fit one tile
    int32_t tune_trace_lpb = 0;       // one-launch layout: line slots per block (1, 2, 4, 8; 0: by the live count)
    int32_t tune_trace_rnd = 0;       // one-launch layout: 256-panel rounds per block (1, 2, 4; 0: by the live count)
    int32_t tune_trace_tail = 16;     // trace_mode 0: live lines at or below which the one-launch layout takes over
    int32_t tune_trace_loop = 4;      // one-launch layout: line slots at or below which one persistent launch runs the rest
    int32_t tune_trace_spin = 1 << 22;   // persistent launch: polls of one wait between its blocks at most
    int32_t coop_launch = -1;         // the device takes cooperative launches (1) or not (0); -1: not asked yet
    int32_t grad_batch = 131072;      // points per batch of the gradient's pair passes (bounds scratch memory)

    // profiling: 0 off; 1 every kernel (event pairs around each launch, the field-line far pass
    // by events carried in its dispatch); 2 only the field-line far pass, by events carried in its
    // dispatch, so that the rest of the work runs as it does unprofiled
    int32_t profiling = 0;
    std::map<std::string, bem::KStat> stats;
    std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> event_pool;

    ~bem_ctx() {
        for (auto& p : pending) {
            (void)hipEventDestroy(p.second.first);
            (void)hipEventDestroy(p.second.second);
        }
        for (auto e : event_pool) (void)hipEventDestroy(e);
        if (fork_ev) (void)hipEventDestroy(fork_ev);
        if (join_ev) (void)hipEventDestroy(join_ev);
        if (aux_stream) (void)hipStreamDestroy(aux_stream);
        for (hipEvent_t e : lf_ev)
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : lb_ev)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace bem {

// RAII timer: records a pair of events on the context stream around a launch.
// enabled = false skips this launch (used to time a fixed sample of very frequent launches).
struct KTimer {
    bem_ctx* c;
    const char* name;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    // records on stream st (nullptr: the context stream)
    KTimer(bem_ctx* ctx, const char* nm, bool enabled = true, hipStream_t st = nullptr);
    ~KTimer();
};
// Kernel-side launch timing (profiling mode 2): kclock_begin readies max_launches slots,
// kclock_slot hands out the next one (nullptr when not timing or when the slots are used up),
// kclock_end adds each used slot's duration to its statistic (it waits for the stream).
void kclock_begin(bem_ctx* c, int64_t max_launches);
unsigned long long* kclock_slot(bem_ctx* c, const char* name);
void kclock_end(bem_ctx* c);
// resolve_stats waits for every pending event; resolve_ready takes only the completed prefix
void resolve_stats(bem_ctx* c);
void resolve_ready(bem_ctx* c);
// a pair of timing events from the context's pool, and their hand-over to the named statistic
void timing_events(bem_ctx* c, hipEvent_t* a, hipEvent_t* b);
void push_timing(bem_ctx* c, const char* name, hipEvent_t a, hipEvent_t b);

// ---- launchers (one translation unit each) --------------------------------
void launch_geometry(bem_ctx* c);                                  // geometry.hip
// S, F of unit density on panel[p] at pts[p]: rule 0 closed forms, 1 the Sec. 4 rule (duffy.hip)
void launch_pair_integrals(bem_ctx* c, int64_t P, const double* pts, const int32_t* panel, int rule, double* S,
                           double* F, int64_t fstride);
// S, F of unit density on curved quadratic panels (six nodes each) by the Sec. 4 rule (duffy.hip)
void launch_quad_pair_integrals(bem_ctx* c, int64_t P, const double* pts, const double* nodes, double* S,
                                double* F);
// the Sec. 4 rule for the assembly's near list into sf[4 k .. 4 k + 3] (duffy.hip)
void launch_near_duffy(bem_ctx* c, int64_t nnz, const int32_t* row, const int32_t* col, double* sf);
void launch_panel_points(bem_ctx* c, int64_t L, const int32_t* panel, const double* bary, double offset,
                         double* out);                                // geometry.hip
void launch_far_assemble(bem_ctx* c);                              // assemble.hip
void launch_near_csr(bem_ctx* c, const uint64_t* mask, int64_t n_targets, DBuf& ptr, DBuf& row, DBuf& col,
                     int64_t* nnz, const char* tname);             // assemble.hip
void launch_near_assemble(bem_ctx* c);                             // assemble.hip
void launch_finalize(bem_ctx* c);                                  // assemble.hip
void launch_copy_rows(bem_ctx* c, int64_t row0, int64_t n_rows, double* out);
void launch_rhs(bem_ctx* c, int32_t nrhs, const double* d_bodyV, double* b);
void launch_nodal_assemble(bem_ctx* c);                                          // nodal.hip
void launch_nodal_records(bem_ctx* c, const double* u);                          // nodal.hip
void launch_nodal_field(bem_ctx* c, int32_t nrhs, const double* sol, int64_t P, const double* pts, double* phi,
                        double* E);                                                  // nodal.hip
void launch_matvec(bem_ctx* c, const double* x, double* y, hipStream_t s);      // gemv.hip
// compressed operator (hmatrix.hip): build (replacing any earlier one), product, release
void hmatrix_build(bem_ctx* c, double eps, double eta, int leaf, HmStats* st);
void hmatrix_matvec(bem_ctx* c, const double* x, double* y, hipStream_t s);
void hmatrix_release(bem_ctx* c);
void launch_matvec_t(bem_ctx* c, const double* x, double* y, hipStream_t s);    // gemv.hip
// the product without allocation: its work array's device address for the current device (looked
// up once per device), and the product through that array (gemv.hip)
void noalloc_scratch_init(int device);
void matvec_noalloc(bem_ctx* c, int32_t nrhs, const double* x, double* y, int transpose);
int gmres_solve(bem_ctx* c, const double* b, double* x, double tol, int max_iter, int* iters, double* relres,
                int* refinements);
int gmres_solve_batched(bem_ctx* c, int nr, const double* B, double* X, double tol, int max_iter, int* iters,
                        double* relres, int* refinements);   // gmres_batched.hip: nr <= 64, rows of stride ld
void batched_apply_exact(bem_ctx* c, int nr, const double* X, double* Y);   // rows of stride n
void launch_eval(bem_ctx* c, const double* sigma, int64_t P, const double* pts, const int32_t* on_panel,
                 double* phi, double* E);                          // eval.hip
// Sec. 4 classification of (point, panel) pairs as ballot masks mask[(j >> 6) * P + p] (bit j & 63 set:
// not regular, or j == on_panel[p]); ceil(N / 64) * P words.
void launch_point_mask(bem_ctx* c, int64_t P, const double* pts, const int32_t* on_panel, uint64_t* mask);
// panel-range split of the field evaluation's far pass for P points (K ranges; span panels each)
int64_t eval_split(const bem_ctx* c, int64_t P, int64_t* span);   // eval.hip
void launch_eval_far(bem_ctx* c, const double* sigma, int64_t P, const double* pts, const int32_t* on_panel,
                     double* part, int64_t KS, int64_t span);    // eval.hip: part[KS][P][4]
void launch_trace(bem_ctx* c, int32_t nrhs, const double* sol, int64_t L, const int32_t* line_rhs,
                  const double* starts, const bem_trace_params* tp, int32_t* n_steps, int32_t* stop_code,
                  double* path, double* integral, uint8_t* exceeds);   // trace.hip
void launch_trace_nodal_cases(bem_ctx* c, int32_t nrhs, const double* sol, int64_t L, const int32_t* line_rhs,
                              const double* starts, const bem_trace_params* tp, int32_t* n_steps, int32_t* stop_code,
                              double* path, double* integral, uint8_t* exceeds);   // trace_batched.hip
// fused_tail: hand the last tune_trace_tail live lines to the one-launch layout
void launch_trace_batched(bem_ctx* c, int32_t nrhs, const double* sol, int64_t L, const int32_t* line_rhs,
                          const double* starts, const bem_trace_params* tp, int32_t* n_steps, int32_t* stop_code,
                          double* path, double* integral, uint8_t* exceeds, bool fused_tail);   // trace_batched.hip
// one launch per RK4 stage (trace_fused.hip); fused_trace_blocks: its panel blocks of 256 rnd
// panels, 0 when N needs more than it allows
void launch_trace_fused(bem_ctx* c, int32_t nrhs, const double* sol, int64_t L, const int32_t* line_rhs,
                        const double* starts, const bem_trace_params* tp, int32_t* n_steps, int32_t* stop_code,
                        double* path, double* integral, uint8_t* exceeds);
int fused_trace_blocks(int64_t N, int rnd);
// trace_mode 3 (one launch per stage throughout), and trace_mode 0 (two kernels, then one launch
// per stage for the last lines) where the panel count allows the one-launch layout
bool trace_fused_layout(const bem_ctx* c);
bool trace_fused_tail(const bem_ctx* c);

int autotune(bem_ctx* c, const char* cache_path);   // autotune.hip; 1 = loaded from the cache
void streamer_grad(bem_ctx* c, int32_t nrhs, const double* sol, int64_t L, const int32_t* line_rhs,
                   const double* starts, const int32_t* start_panel, const double* start_bary,
                   const bem_trace_params* tp, const double* gI, double tol, double* dvert, double* dV,
                   double* dstart);   // adjoint_panel.hip

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace bem
