/*
 * bem.h -- C ABI of the MI355X (gfx950) boundary-element library for the
 * indirect single-layer collocation method of "Dielectric Breakdown
 * Prediction with GPU-Accelerated BEM" (arXiv 2003.12663).
 *
 * Discretisation: flat triangles tau_j, piecewise-constant virtual charge
 * sigma_j, collocation at the centroids x_i.  Unknowns are ordered
 * [sigma_1..sigma_N, V_1..V_Nfl] (one potential per floating body, in body
 * order); constraint rows come last.
 *
 * Conventions shared by every call:
 *  - "host" pointers are CPU memory; "dev" pointers are device memory of the
 *    context's GPU (e.g. a torch tensor's data_ptr()).  The caller owns every
 *    array; no call keeps a caller pointer after it returns.
 *  - All device work is ordered on the stream given to bem_create.  Calls
 *    that return host-side results (bem_solve_gmres's info, counts) wait for
 *    that stream.  The batched field-line tracer also runs kernels on a second
 *    stream of its own, ordered after the work already on the context stream
 *    and joined back into it before the call returns.
 *  - Every call returns a bem_status; on failure bem_last_error() gives a
 *    thread-local message.  Inputs are validated before any kernel launch.
 *  - One context per host thread at a time; contexts are independent.
 *  - The library never falls back to the CPU: without a usable gfx950 GPU,
 *    bem_create fails with BEM_ERR_HIP.
 */
#ifndef BEM_H
#define BEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bem_ctx bem_ctx;

typedef enum {
    BEM_OK = 0,
    BEM_ERR_INVALID = 1,    /* bad argument (index range, non-finite value, size, state of options) */
    BEM_ERR_DEGENERATE = 2, /* a triangle with (numerically) zero area */
    BEM_ERR_OOM = 3,        /* device memory would not suffice; detected before any allocation */
    BEM_ERR_HIP = 4,        /* a HIP runtime call failed */
    BEM_ERR_NOCONV = 5,     /* GMRES did not reach the tolerance; best iterate written, info filled */
    BEM_ERR_STATE = 6       /* call order violated (e.g. solve before assemble) */
} bem_status;

/* Body kinds (paper Sec. 2, Fig. 2: conductor on a prescribed potential,
 * floating conductor, insulator). */
typedef enum {
    BEM_DIRICHLET = 0, /* rows of Eq. Final1: sum_j S_ij sigma_j = V_body */
    BEM_FLOATING = 1,  /* rows of Eq. Final2 (S sigma - V_f = 0) plus one row of Eq. Final4 per body */
    BEM_INTERFACE = 2, /* rows of Eq. Final3 / Eq. nonconductors, using K' of Eq. ADL */
    BEM_FLOATING_SHEET = 3 /* thin floating conductive sheet modelled by one (open) surface: rows of
                              Eq. Final2 plus one row of Eq. sheets per body, the net charge over both
                              sides, sum_i a_i ((eps+ + eps-)/2 sigma_i + (eps+ - eps-) (K' sigma)_i)
                              = 0, whatever constraint_form says; eps_plus / eps_minus are the
                              permittivities on the normal side and the other side.  bem_streamer_grad
                              covers sheets (the row of Eq. sheets is differentiated like Final4). */
} bem_kind;

typedef enum { BEM_FP64 = 0, BEM_MIXED = 1 } bem_precision;

/* Discretisation of the virtual charge (Sec. 3).
 *  CONSTANT: one value per flat triangle, collocated at the centroids (n = N + N_float).
 *  LINEAR:   the paper's own nodal basis: continuous piecewise-linear hats of the vertices,
 *            collocated at the vertices (Eq. Matrix; n = n_vert + N_float, unknowns
 *            [u_1..u_nvert, V_1..V_Nfl]).  Every body kind: conductor and floating vertex
 *            rows are potentials at the vertex; rows that need the normal field n . E (an
 *            interface vertex, Eq. nonconductors; a floating body's literal row, Eq. Final4,
 *            constraint_form 0; a sheet, Eq. sheets), which a vertex of flat panels lacks,
 *            are the hat-weighted mean of the condition over the centroids of the triangles
 *            around the vertex (or of the body), each with its triangle's normal;
 *            constraint_form 1 makes a closed floating body's row its net charge.  Bodies
 *            that touch carry coincident vertices of their own (a vertex in triangles of
 *            two bodies is refused); a vertex row meets the other body's triangles through
 *            the coincident vertex as their vertex.  FP64, or MIXED with the vertex rows stored in FP32
 *            (each entry formed in FP64 and rounded once, as the paper stores its matrix in
 *            single precision) and the constraint rows in FP64, solved inside FP64 iterative
 *            refinement; every vertex in at least one triangle and
 *            all triangles at a vertex of one body.  Supported calls: bem_assemble,
 *            bem_copy_rows, bem_rhs, bem_matvec, bem_solve_gmres, bem_eval_field at volume
 *            points (on_panel NULL; phi or E may be NULL), and bem_trace_lines /
 *            bem_streamer_integral in the all-lines layouts (trace_mode 0, 1 or 3; lines of several
 *            load cases run case by case; the line passes read FP64 panel records carrying
 *            the nodal density, in MIXED contexts too); the gradient and the autotuner need
 *            CONSTANT (INVALID otherwise). */
typedef enum { BEM_BASIS_CONSTANT = 0, BEM_BASIS_LINEAR = 1 } bem_basis;

/* One body.  Triangle normals (right-hand rule of the vertex order) point
 * into the eps_plus side. */
typedef struct {
    int32_t kind;      /* bem_kind */
    double eps_plus;   /* permittivity on the normal side */
    double eps_minus;  /* permittivity on the other side (INTERFACE and FLOATING_SHEET) */
} bem_body;

typedef struct {
    int32_t precision;       /* bem_precision.  FP64: dense FP64 matrix.  MIXED: far entries in a
                                dense FP32 matrix; each near entry v is stored as its FP32 head
                                h = fl32(v) in the dense slot plus the exact FP64 remainder v - h in
                                a near CSR list, so the operator is FP32 far + FP64 near; FP64
                                Krylov vectors and iterative refinement. */
    double eta;              /* Sec. 4 classification: (point, triangle) regular iff D > eta*R with
                                D the distance to the circumcentre, R the circumradius.  >= 1.
                                Regular pairs use the 7-point rule, the others closed forms. */
    int32_t restart;         /* GMRES restart length m, 1..1000 */
    int32_t constraint_form; /* 0: Eq. Final4 as printed (literal); 1: net charge sum a_i sigma_i = 0 */
    int32_t basis;           /* bem_basis */
} bem_options;

typedef struct {
    int32_t iters;        /* Krylov iterations (summed over right-hand sides and refinements) */
    double rel_residual;  /* max over right-hand sides of ||b - A x|| / ||b|| at exit */
    int32_t refinements;  /* outer iterative-refinement steps (MIXED), else 0 */
} bem_solve_info;

/* Field-line parameters (paper Sec. 1: breakdown paths follow field lines;
 * Eq. Breakdowncrit). */
typedef struct {
    double h;             /* RK4 arc-length step; must be < (eta - 1) * min circumradius */
    double e_min;         /* stop (code 4) when |E| < e_min at the start of a step */
    double start_offset;  /* offset of line starts along the panel normal; used by bem_streamer_grad
                             when starts move with their panels, informational elsewhere */
    int32_t max_steps;    /* stop (code 0) after this many accepted steps, 1..1e6 */
    int32_t direction;    /* +1: follow E, -1: follow -E */
    double alpha_a, alpha_e0, alpha_p; /* alpha_eff(E) = alpha_a * max(E - alpha_e0, 0)^alpha_p */
    double k_str;         /* streamer constant: exceeds[l] = integral[l] > k_str */
} bem_trace_params;

/* Stop codes written by bem_trace_lines / bem_streamer_integral. */
enum {
    BEM_STOP_MAXSTEPS = 0,
    BEM_STOP_DIRICHLET = 1, /* the step's segment hit a conductor panel; the step is discarded */
    BEM_STOP_FLOATING = 2,  /* ... a floating-conductor panel */
    BEM_STOP_INTERFACE = 3, /* ... a dielectric-interface panel */
    BEM_STOP_WEAK = 4,      /* |E| < e_min */
    BEM_STOP_NONFINITE = 5
};

/* Create a context: copies the mesh to the device and computes panel
 * geometry (centroid, normal, area, circumcentre/radius, 7-point nodes).
 *  vert      host [n_vert][3]
 *  tri       host [n_tri][3] vertex indices, CCW about the eps+ normal
 *  tri_body  host [n_tri] body index of each triangle
 *  bodies    host [n_body]
 *  opt       host; NULL = {FP64, eta 6, restart 100, literal constraint, CONSTANT basis}
 *  hip_stream  a hipStream_t (NULL = default stream) of the current device
 * Errors: INVALID (indices, non-finite coordinates, kinds, options),
 * DEGENERATE (area <= 1e-14 * longest edge^2), HIP. */
bem_status bem_create(int64_t n_vert, const double* vert, int64_t n_tri, const int32_t* tri,
                      const int32_t* tri_body, int32_t n_body, const bem_body* bodies,
                      const bem_options* opt, void* hip_stream, bem_ctx** out);
void bem_destroy(bem_ctx* ctx);
const char* bem_last_error(void);

/* Number of unknowns n (N + N_float, or n_vert + N_float for the LINEAR basis). */
int64_t bem_n_unknowns(const bem_ctx* ctx);

/* Assemble the collocation system of Eqs. Final1-Final4 (Sec. 4 quadrature:
 * regular pairs by the 7-point rule, near-singular and singular pairs by the
 * closed forms for flat triangles, done in a second pass over a compacted
 * near list).  Errors: OOM (checked before allocating), HIP. */
bem_status bem_assemble(bem_ctx* ctx);

/* Copy rows [row0, row0 + n_rows) of the assembled operator as FP64 into
 * out (dev [n_rows][n]).  In MIXED mode this is the operator actually used:
 * FP32 far entries widened, plus the FP64 near entries. */
bem_status bem_copy_rows(bem_ctx* ctx, int64_t row0, int64_t n_rows, double* out);

/* Number of near-singular and singular (row, panel) pairs of the assembly (CONSTANT
 * basis; 0 for LINEAR, whose near pass keeps no list). */
int64_t bem_near_pairs(const bem_ctx* ctx);

/* Right-hand sides for body potentials: b (dev [nrhs][n]); body_V host [nrhs][n_body]
 * (entries of non-DIRICHLET bodies are ignored). */
bem_status bem_rhs(bem_ctx* ctx, int32_t nrhs, const double* body_V, double* b);

/* y = A x (transpose = 0) or y = A^T x (transpose = 1) for nrhs vectors,
 * x, y dev [nrhs][n], FP64 (the Krylov matvec of Sec. 3).  With nrhs >= 2
 * and "batched_solve" on, A x is one product of up to 64 vectors on the
 * matrix cores with FP64 accumulation (MIXED: the FP32 far entries widened). */
bem_status bem_matvec(bem_ctx* ctx, int32_t nrhs, const double* x, double* y, int32_t transpose);

/* The product of bem_matvec without any device allocation, for callers that cannot allocate
 * (code under stream capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments and results: each vector goes through the one-vector kernels of bem_matvec (the
 * batched matrix-core product is not used, so with nrhs >= 2 and "batched_solve" on the sums
 * differ from bem_matvec's by rounding only).  Its work memory is a fixed device array of
 * 66 x 65536 doubles (33 MiB) that the library holds on every GPU it runs on until the process
 * ends: n (bem_n_unknowns) must be <= 65536, else INVALID.  Every call on one GPU uses that GPU's
 * array, so calls that overlap on one GPU (on different streams or host threads) race.  Enqueued
 * on the context stream; x and y must not overlap.  Errors: INVALID (sizes, NULL vectors,
 * transpose in MIXED precision), STATE (not assembled), HIP. */
bem_status bem_matvec_noalloc(bem_ctx* ctx, int32_t nrhs, const double* x, double* y, int32_t transpose);

/* Sizes of a compressed operator (bem_compress). */
typedef struct {
    int64_t blocks;          /* blocks of the block tree */
    int64_t lowrank_blocks;  /* of them stored as U V^T */
    int64_t dense_entries;   /* doubles in the dense blocks */
    int64_t factor_entries;  /* doubles in the low-rank factors */
    int64_t max_rank;        /* largest rank of a low-rank block */
} bem_compress_info;

/* Compress the collocation operator (the outlook of Sec. 6: hierarchical matrices in place of
 * the dense N x N matrix) and use it for the products of bem_matvec and bem_solve_gmres.
 * The panel-panel block becomes a hierarchical matrix: a cluster tree of the panels by
 * geometric bisection down to leaves of at most `leaf` panels (8..256); cluster pairs whose
 * bounding boxes are admissible, min(diam) <= eta_adm * dist (eta_adm > 0), are stored in low
 * rank by adaptive cross approximation with partial pivoting to the relative tolerance eps
 * (0 < eps < 1; rank at most 64, else the block is stored dense), the others dense at leaf
 * level.  Every entry is the assembly's own (Sec. 4 classification, 7-point rule, closed
 * forms, the row scaling of Eqs. Final1-Final3), evaluated on demand: no N x N array is
 * formed.  The floating bodies' potential columns and constraint rows (Eq. Final4, sheets,
 * net charge) are kept exactly.  Replaces the dense operator (its memory is released);
 * bem_assemble restores the dense one.  CONSTANT basis, FP64.  While it is in use: no
 * transpose product (bem_matvec transpose, bem_streamer_grad), no bem_copy_rows, no
 * bem_matvec_noalloc (INVALID), and several right-hand sides are solved one after another.
 * info may be NULL.  Errors: INVALID (options, basis, precision), OOM (checked before the
 * factors are allocated), HIP. */
bem_status bem_compress(bem_ctx* ctx, double eps, double eta_adm, int32_t leaf, bem_compress_info* info);

/* Single-layer potential S = (1/4pi) int 1/|x - y| dS and field F = -grad S =
 * (1/4pi) int (x - y)/|x - y|^3 dS of unit density on panel[p] at pts[p], p < P (Sec. 4 and
 * the field formula closing Sec. 2).  rule 0: the closed forms of the flat triangle
 * (Wilton et al. / Graglia); a point on the panel (within 1e-14 of its size) gets the
 * principal value (its normal component 0).  rule 1: the paper's near-singular rule of
 * Sec. 4: the point of the panel closest to x, the panel cut into pieces with that point as
 * a corner, the Duffy transformation of each piece and tensor Gauss-Legendre (16 x 16 nodes
 * per cell) on cells graded geometrically towards the corner and towards its foot on the
 * opposite edge; a point on the panel gets S, and F = NaN (the principal value is not formed
 * by this rule).  pts dev [P][3], panel dev int32 [P] (0 <= panel < N), S dev [P], F dev
 * [P][3] or NULL.  With tuning key "near_rule" = 1 the assembly uses rule 1 for its near and
 * self pairs (CONSTANT basis).  Errors: INVALID (P, rule, indices, non-finite points), HIP. */
bem_status bem_pair_integrals(bem_ctx* ctx, int64_t P, const double* pts, const int32_t* panel, int32_t rule,
                              double* S, double* F);

/* The near-singular rule of Sec. 4 on curved panels: S = (1/4pi) int 1/|x - y| dS and
 * F = (1/4pi) int (x - y)/|x - y|^3 dS of unit density on the curved quadratic panel p at
 * pts[p], p < P.  A curved panel (Sec. 3: piecewise quadratic parametrization of curved
 * triangles) is the quadratic Lagrange map of the reference triangle {(s, t): s, t >= 0,
 * s + t <= 1} through its six nodes, nodes[p][0..2] the corners y(0,0), y(1,0), y(0,1) and
 * nodes[p][3..5] the edge nodes y(1/2,0), y(1/2,1/2), y(0,1/2).  The rule runs in the
 * parameter plane: the closest parameter point c (Newton's method, with the edges and
 * corners), the reference triangle cut into pieces with c as a corner, the Duffy map of
 * each piece times the surface Jacobian |y_s x y_t|, and tensor Gauss-Legendre (16 x 16 nodes
 * per cell) on cells graded geometrically towards c and towards its foot on the opposite
 * edge, scaled by the piece's edges through the tangent map at c.  A point on the panel
 * (within 1e-14 of its size) gets S, and F = NaN.  The context supplies the device and the
 * stream only; the panels need not belong to its mesh.
 *  pts dev [P][3]; nodes dev [P][6][3]; S dev [P] (written); F dev [P][3] (written) or NULL.
 * Errors: INVALID (P < 0 or >= 2^31, NULL arrays, non-finite input, a panel whose corner
 * triangle has no area), HIP. */
bem_status bem_quad_pair_integrals(bem_ctx* ctx, int64_t P, const double* pts, const double* nodes, double* S,
                                   double* F);

/* Solve A sol = b(body_V) for nrhs load cases by restarted GMRES with the
 * diagonal (Jacobi) preconditioner applied on the right (Sec. 5.2), CGS2
 * orthogonalisation, zero initial guess, stopping at ||b - A x|| <= tol ||b||
 * for every load case.  MIXED: GMRES on the mixed operator inside FP64
 * iterative refinement.  Several load cases: see "batched_solve" below.
 *  body_V host [nrhs][n_body]; sol dev [nrhs][n]; info host (may be NULL).
 * Errors: STATE (not assembled), INVALID, NOCONV (best iterate written). */
bem_status bem_solve_gmres(bem_ctx* ctx, int32_t nrhs, const double* body_V, double tol,
                           int32_t max_iter, double* sol, bem_solve_info* info);

/* Potential and field at P points (the field formula closing Sec. 2):
 * phi(x) = sum_j S_j(x) sigma_j, E(x) = sum_j F_j(x) sigma_j.
 *  sol      dev [nrhs][n] (only the sigma part is read)
 *  pts      dev [P][3]
 *  on_panel dev [P] or NULL: >= 0 marks the point as that panel's centroid and
 *           returns the limit from the eps+ side (principal value + sigma n / 2);
 *           -1 = volume point (must not lie on a panel edge).
 *  phi      dev [nrhs][P] or NULL;  E dev [nrhs][P][3] (may be NULL for the LINEAR basis). */
bem_status bem_eval_field(bem_ctx* ctx, int32_t nrhs, const double* sol, int64_t P, const double* pts,
                          const int32_t* on_panel, double* phi, double* E);

/* Field lines dx/ds = direction * E/|E| by classical RK4 with step h, all
 * lines in one call ("trace_mode" picks the layout).  A step whose segment [x_n, x_{n+1}]
 * intersects a panel is discarded and the line stops with that panel's kind
 * (smallest segment parameter wins, then the lowest panel index).
 *  line_rhs dev [L] or NULL (all lines use load case 0): which sol row drives line l
 *  starts   dev [L][3]
 *  n_steps, stop_code  dev [L]
 *  path     dev [L][max_steps+1][3] or NULL: x_0..x_{n_steps}; later slots untouched. */
bem_status bem_trace_lines(bem_ctx* ctx, int32_t nrhs, const double* sol, int64_t L, const int32_t* line_rhs,
                           const double* starts, const bem_trace_params* tp, int32_t* n_steps,
                           int32_t* stop_code, double* path);

/* Streamer-inception integral of Eq. Breakdowncrit along each field line,
 * integral[l] = int alpha_eff(|E|) ds, carried as an extra RK4 state
 * (h/6 (a1 + 2 a2 + 2 a3 + a4) per accepted step from the stage fields).
 *  integral dev [L]; exceeds dev [L] (uint8, integral > k_str) or NULL. */
bem_status bem_streamer_integral(bem_ctx* ctx, int32_t nrhs, const double* sol, int64_t L,
                                 const int32_t* line_rhs, const double* starts, const bem_trace_params* tp,
                                 double* integral, int32_t* n_steps, int32_t* stop_code, uint8_t* exceeds);

/* Gradient of J = sum_l dJ_dI[l] * integral[l] (the streamer integrals above) with
 * respect to the mesh vertices and the body potentials, by reverse mode through
 * the whole method: the field lines (adjoint RK4 with the field Jacobian at every
 * stage point), the field of every panel (quadrature nodes and weights for regular
 * pairs, the closed forms for the others), the solve (one adjoint GMRES with A^T
 * per load case) and the collocation system of Eqs. Final1-Final4 (collocation
 * points, normals, areas of the constraint rows).  The regular/near classification
 * of Sec. 4 and each line's step count and stop reason are held at their values
 * for the given state (the derivative of the piecewise-smooth map on its piece).
 *  sol          dev [nrhs][n]: the solution for body_V (as from bem_solve_gmres; the
 *               gradient assumes it solves the assembled system)
 *  line_rhs, starts: as for bem_streamer_integral (the forward run is redone inside)
 *  start_panel  dev [L] or NULL: line l starts on that panel and moves with it,
 *               starts[l] = sum_k start_bary[l][k] v_k + start_offset n (vertices in
 *               the panel's own order); NULL = starts fixed in space
 *  start_bary   dev [L][3] (required with start_panel)
 *  dJ_dI        dev [L]
 *  tol          relative residual of the adjoint solves
 *  dJ_dvert     dev [n_vert][3] (written)
 *  dJ_dV        dev [nrhs][n_body] (written; 0 for non-conductor bodies)
 *  dJ_dstart    dev [L][3] or NULL: dJ/d starts[l] at fixed mesh
 * FP64 precision only; alpha_p >= 1.  Errors: STATE (not assembled), INVALID,
 * NOCONV (an adjoint solve missed tol), OOM, HIP. */
bem_status bem_streamer_grad(bem_ctx* ctx, int32_t nrhs, const double* sol, int64_t L,
                             const int32_t* line_rhs, const double* starts, const int32_t* start_panel,
                             const double* start_bary, const bem_trace_params* tp, const double* dJ_dI,
                             double tol, double* dJ_dvert, double* dJ_dV, double* dJ_dstart);

/* Points on panels, as field-line starts that sit on an electrode (Sec. 1: breakdown paths
 * start at the electrode surface):
 *   out[l] = sum_k bary[l][k] v_k + offset * n   for panel j = panel[l],
 * v_k the panel's vertices in their stored order, n its unit normal (into eps+).  This is
 * the placement bem_streamer_grad assumes when its starts move with their panels.
 *  panel dev [L] int32 in [0, N); bary dev [L][3]; out dev [L][3] (written).
 * Errors: INVALID (index range, non-finite input). */
bem_status bem_panel_points(bem_ctx* ctx, int64_t L, const int32_t* panel, const double* bary, double offset,
                            double* out);

/* Tuning knobs (no effect on results beyond summation order).
 *  "trace_mode": how field lines advance.  1 = all lines together, each RK4 stage one
 *                far-field pass spread over the GPU and one step kernel (one block per
 *                line); 3 = all lines together, each stage one launch whose blocks first
 *                finish the previous stage of their lines from the partial fields the
 *                previous launch wrote, then evaluate the new stage (at most 131072 panels);
 *                2 = one persistent launch, one workgroup per line; 0 (default) = 1 while
 *                more than "trace_tail" lines are live, then 3 (1 throughout above 131072
 *                panels).  Layout 3 (and the tail of 0) runs all its remaining stages in one
 *                persistent launch once at most "trace_loop" line slots remain and their grid
 *                fits the GPU at once (cooperative launch): blocks of a line group then exchange
 *                their partial fields through device memory and wait for each other between
 *                stages instead of ending the launch.
 *  "batched_solve": 1 (default) = bem_solve_gmres with nrhs >= 2 runs up to 64
 *                independent GMRES recurrences together, one multi-right-hand-
 *                side matrix product per iteration on the matrix cores (FP64:
 *                FP64 cores; MIXED: FP32 cores inside FP64 iterative
 *                refinement); 0 = one right-hand side after another.
 *  "near_rule":  0 (default) = near and self pairs of the assembly by the closed forms of
 *                the flat triangle; 1 = by the paper's near-singular rule (closest point,
 *                subdivision, Duffy; see bem_pair_integrals), CONSTANT basis only.  Takes
 *                effect at the next bem_assemble; one wave per pair, so far slower than 0.
 *  Tile shapes (set by bem_autotune, or by hand):
 *  "far_rows":    collocation rows per block of the far-field assembly (32, 64, 128; default 64)
 *  "gemv_rows":   matrix rows per block of the GMRES matvec (2, 4, 8, 16; default 4 for FP64, 8 for MIXED)
 *  "gemm_blocks": minimum blocks of the FP32 multi-vector product, by K ranges (64..65536; 1024)
 *  "eval_blocks": target blocks of the field evaluation, by panel ranges (64..65536; 2048)
 *  "trace_tile":  lines per block of an unsplit field-line pass (64, 128, 256; default 256)
 *  "trace_splitk": waves splitting each panel chunk in a split field-line pass (2, 4, 8; default 8)
 *  "trace_few":   live-line count at or below which a field-line pass is panel-stationary (one
 *                 lane per panel, all live lines per lane; 0..16; default 8)
 *  "trace_split": live-line count at or below which a field-line pass splits each panel chunk
 *                 over eight waves (0..4096; default 64)
 *  "trace_groups": line groups of a batched field-line run (1 or 2; 0, the default: 2 from 128
 *                 lines, else 1): lines are cut
 *                 into two contiguous halves that advance on two streams (the context stream
 *                 and a second one the library owns), so that one group's step kernel overlaps
 *                 the other group's far-field pass; the groups are folded into one once the live
 *                 lines fit one 64-line tile.  Each group picks its pass layout
 *                 ("trace_few", "trace_split") by its own live count, which can change the
 *                 summation order of a line's far field; with the layout fixed (trace_few 0,
 *                 trace_split 0 or above the line count) results do not depend on the grouping
 *  "trace_fold":  1 (default) = with two line groups, fold the second into the first once all
 *                 live lines fit one 64-line tile; 0 = keep both groups to the end
 *  "trace_tail":  trace_mode 0: live-line count at or below which the run goes on in the
 *                 one-launch layout (0..4096; default 16; 0 = never); checked every 32 passes
 *  "trace_loop":  one-launch layout: line-slot count at or below which the remaining stages
 *                 run in one persistent launch (0..4096; default 4; 0 = never)
 *  "trace_spin":  persistent launch: polls of one wait between its blocks before the launch
 *                 gives up and the call fails with BEM_ERR_HIP (0..2^30; default 2^22, seconds;
 *                 a safety bound, not reached in normal runs)
 *  "trace_lpb":   one-launch layout: line slots per block (1, 2, 4, 8; 0, the default: by the
 *                 live count)
 *  "trace_rnd":   one-launch layout: 256-panel rounds per block (1, 2, 4; 0, the default: by
 *                 the live count)
 *  "grad_batch":  points per batch of the pair passes of bem_streamer_grad (64..2^24; default
 *                 131072; bounds scratch memory)
 * Errors: INVALID for an unknown key or value. */
bem_status bem_set_tuning(bem_ctx* ctx, const char* key, int64_t value);

/* Current value of a tuning knob (keys as for bem_set_tuning).  Errors: INVALID. */
bem_status bem_get_tuning(const bem_ctx* ctx, const char* key, int64_t* value);

/* Autotuner for the tile shapes above: times each candidate on this context's
 * assembled problem (HIP events, best of three after a warm-up) and sets the
 * fastest; a candidate replaces the default only when it is more than 3 %
 * faster, so that timing noise does not flip the choice between runs.  cache_path (host string, or NULL for
 * no cache): a JSON file keyed by device architecture, panel and unknown
 * counts, precision and eta; an entry for this key is used without timing,
 * otherwise the new choice is added and the file rewritten.  Tuning re-runs
 * the assembly (the timed candidates overwrite the matrix); results change at
 * most in summation order.  from_cache (host, may be NULL): 1 if the cache
 * supplied the choice.  Errors: STATE (not assembled), INVALID (unreadable or
 * invalid cache entry, unwritable file), HIP, OOM. */
bem_status bem_autotune(bem_ctx* ctx, const char* cache_path, int32_t* from_cache);

/* Per-kernel timing with HIP events, on the stream of the launch (the context stream, or the
 * tracer's second stream for its line groups).
 *  enable 0: off.
 *  enable 1: every kernel, by an event pair recorded around each launch.  Names: "geometry",
 *            "far_assemble", "near_mask_csr", "near_assemble", "finalize", "gemv", "gmres_ortho",
 *            "gmres_iter", "eval_mask", "eval_near_csr", "eval_far", "eval_near", "trace" (a
 *            whole field-line call), "trace_step" (the step kernel of a batched pass; every
 *            16th pass is timed, so its launch count is a sample and total_ms covers that
 *            sample), "gemm_f32", "gemm_f64", "gemm_rows", "bgmres_iter", "grad",
 *            "grad_reverse", "grad_rows_EH", "grad_panel_far", "grad_panel_near", "gemvT".
 *  enable 1: also "trace_far", every chunked far pass of the two-kernel field-line layout, and
 *            "trace_pass", every launch of the one-launch layout, timed by events carried in
 *            their own dispatches (hipExtLaunchKernelGGL), nothing added to the stream.
 *  enable 2: only "trace_far" and "trace_pass", so that all other work runs as it does
 *            unprofiled, each launch timed by the kernel itself: the earliest block start to
 *            the latest wave end on the device's constant-rate wall clock (with two line
 *            groups on two streams, an event interval also counts the wait for the other
 *            group's kernel to free the compute units).  A field-line call then waits for its
 *            stream at the end to collect the stamps.
 * Errors: INVALID for another value. */
bem_status bem_set_profiling(bem_ctx* ctx, int32_t enable);
bem_status bem_kernel_stats(bem_ctx* ctx, const char* name, int64_t* launches, double* total_ms);
bem_status bem_reset_stats(bem_ctx* ctx);   /* also zeroes the counters below */

/* Work counters since creation or the last bem_reset_stats:
 * "trace_near_pairs"   = (point, panel) pairs of field-line evaluations that
 *                        took the closed-form (near) path in the two-kernel layout;
 * "trace_far_pairs"    = regular (7-point rule) pairs evaluated by the chunked
 *                        far-field passes (k_lb_far) of the two-kernel layout;
 * "trace_far_launches" = launches of those chunked passes (each timed as
 *                        "trace_far" when profiling); the panel-stationary
 *                        few-line passes are in neither;
 * "trace_pass_near_pairs", "trace_pass_pairs", "trace_pass_launches" = the
 *                        same for the one-launch layout (k_lf_pass, timed as
 *                        "trace_pass"; every launch counted). */
bem_status bem_get_counter(bem_ctx* ctx, const char* name, int64_t* value);

#ifdef __cplusplus
}
#endif
#endif /* BEM_H */
