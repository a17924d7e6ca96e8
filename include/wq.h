/*
 * wq.h -- C ABI of the MI355X (gfx950) weighted-quadrature library (libwq.so).
 *
 * Weighted quadrature (WQ) on unstructured bicubic splines: each test function N_i
 * gets its own quadrature rule Q_i(g) = sum_q w_iq g(x_q) over points placed in the
 * physical domain (Section 4.1, Eqs. (8)-(10)); the weights solve underdetermined
 * exactness systems by truncated SVD (Section 4.3, Eqs. (19)-(22)); Galerkin matrices
 * are then formed row by row (Eqs. (9), (11), (12), (36)).
 *
 * Conventions for every entry point:
 *  - Returns wq_status; WQ_OK == 0. No exceptions cross the ABI. On error, outputs are
 *    left untouched and wq_last_error() returns a thread-local message.
 *  - "host" pointers are read during the call only (the caller keeps ownership).
 *    "device" pointers are HIP device memory owned by the caller; they must stay valid
 *    until the work queued on `stream` has completed.
 *  - Handles (wq_mesh, wq_points, wq_weights) own their device memory and are released
 *    by the matching *_destroy call. A handle is used on the device that was current
 *    when it was created.
 *  - build_points and solve_weights synchronise their stream (they return counts);
 *    assemble_* calls are asynchronous on `stream` (0 = the null stream).
 *  - Indices are 0-based. Floating point is IEEE FP64 unless stated.
 */
#ifndef WQ_H
#define WQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wq_mesh wq_mesh;
typedef struct wq_points wq_points;
typedef struct wq_weights wq_weights;
typedef void* wq_stream; /* a hipStream_t */

typedef enum {
  WQ_OK = 0,
  WQ_EINVAL = -1,      /* bad argument, inconsistent sizes, unsupported option       */
  WQ_ENOMEM = -2,      /* device allocation failed                                   */
  WQ_EILLPOSED = -3,   /* some row has fewer points than constraints (r_i < n_i)     */
  WQ_ESVD = -4,        /* a Jacobi SVD did not converge within its sweep limit       */
  WQ_ENOCONV = -5,     /* an iterative solve did not converge                        */
  WQ_EDEVICE = -6      /* a HIP runtime call failed                                  */
} wq_status;

/* Weight families (bit mask): exactness for N_j, dN_j/dx, dN_j/dy, Lap N_j
 * (Eq. (9), the two planar terms of Eq. (11), Eq. (12)). */
typedef enum { WQ_FAM_MASS = 1, WQ_FAM_DX = 2, WQ_FAM_DY = 4, WQ_FAM_LAP = 8, WQ_FAM_DZ = 16 } wq_family;

/* Arithmetic of the row contraction. FP64 everywhere else, always. */
typedef enum { WQ_FP64 = 0, WQ_SPLIT_FP16 = 1, WQ_SPLIT_BF16 = 2, WQ_SLICED_FP16 = 3 } wq_precision;

/* ------------------------------------------------------------------ input mesh
 * Control mesh and Bezier extraction of the spline space (Section 3). All arrays are
 * host arrays, copied to the device by wq_mesh_create.
 *   face_vtx  [nf*4]  counter-clockwise vertex ids of each quad face
 *   split     [nf]    1: the face is split 2x2 into Bezier sub-elements (irregular)
 *   ext_ptr   [nf+1]  offsets into ext_fn; face f carries m_f = ext_ptr[f+1]-ext_ptr[f]
 *   ext_fn    [.]     global ids of the functions on each face, ascending
 *   coef_ptr  [nf+1]  offsets (in doubles) into coef
 *   coef      [.]     per face nsub x m_f x 16 Bernstein coefficients, index k + 4 l
 *                     (k along corner0->corner1); nsub = 4 if split (sub-element
 *                     sx + 2 sy covers [sx/2,(sx+1)/2] x [sy/2,(sy+1)/2]), else 1
 *   ctrl      [n_fn*dim] control points; the geometry map is x = sum_j ctrl_j N_j
 *   dim       2: a planar domain; 3: a 2-manifold in 3-D (Section 4.1): gradients are
 *             surface gradients with a third component (family WQ_FAM_DZ), the
 *             Laplacian is the Laplace-Beltrami operator and det J is sqrt(det g).
 *             0 is read as 2.
 * Faces touching the boundary are passive (zero parametric area) and carry m_f = 0. */
typedef struct {
  int32_t nv, nf, n_fn;
  const int32_t* face_vtx;
  const uint8_t* split;
  const int64_t* ext_ptr;
  const int32_t* ext_fn;
  const int64_t* coef_ptr;
  const double* coef;
  const double* ctrl;
  int32_t dim;
} wq_mesh_desc;

wq_status wq_mesh_create(const wq_mesh_desc* desc, wq_mesh** out);
void wq_mesh_destroy(wq_mesh* mesh);

/* ------------------------------------------------------------------ build_points
 * Classifies elements (Section 3 definitions) and chooses s_e x s_e points per element
 * from Table 2 (non-enriched transition: 3x3, 4x4 next to EPs of valence >= 7 or EPs
 * of two different irregular neighbourhoods), checks the well-posedness r_i >= n_i of
 * Section 4.2 and, where it fails, applies the min-max allocation of Eq. (18).
 * Then builds, on the device:
 *  - the points: s x s per element at ((2a+1)/(2s), (2b+1)/(2s)) of its parametric
 *    square, numbered Bezier cell by cell (split elements contribute 4 cells), inside a
 *    cell by (b, a) row-major; basis values N, dN/dx, dN/dy (and Lap N if
 *    want_laplacian) of every cell function at every point, x, and det J;
 *  - the CSR pattern of Eq. (10): row i holds S_i (functions nonzero on some cell of
 *    supp N_i), columns ascending;
 *  - the point sets Q_i: the point ranges of the cells of supp N_i, cells ascending.
 * Outputs the sizes (host scalars). Synchronises `stream`. */
wq_status build_points(wq_mesh* mesh, int want_laplacian, wq_stream stream, wq_points** out,
                       int64_t* n_rows, int64_t* nnz, int64_t* n_points);
void wq_points_destroy(wq_points* pts);

/* As build_points, but starting from the caller's points per direction s[nf] (host,
 * uint8, 0 for passive faces) instead of Table 2; the well-posedness check and the
 * min-max allocation of Eq. (18) still apply. For studies of point allocations. */
wq_status build_points_with_s(wq_mesh* mesh, const uint8_t* s_host, int want_laplacian, wq_stream stream,
                              wq_points** out, int64_t* n_rows, int64_t* nnz, int64_t* n_points);

/* Copies of the device arrays built above into caller device buffers (for checks and
 * for users that need the pattern). `what` selects the array and its element type:
 *   WQ_ARR_ROW_PTR  int64[n+1]   WQ_ARR_COL   int32[nnz]
 *   WQ_ARR_QPTR     int64[n+1]   WQ_ARR_QIDX  int32[sum r_i]
 *   WQ_ARR_ETYPE    uint8[nf]  (0 passive, 1 regular, 2 boundary, 3 irregular, 4 transition)
 *   WQ_ARR_S        uint8[nf]    points per direction (0: passive)
 *   WQ_ARR_X        double[dim*np] WQ_ARR_DETJ double[np] (sqrt(det g) on a surface)
 * wq_points_size() returns the element count of each array. */
typedef enum {
  WQ_ARR_ROW_PTR = 0, WQ_ARR_COL = 1, WQ_ARR_QPTR = 2, WQ_ARR_QIDX = 3,
  WQ_ARR_ETYPE = 4, WQ_ARR_S = 5, WQ_ARR_X = 6, WQ_ARR_DETJ = 7
} wq_array;
int64_t wq_points_size(const wq_points* pts, wq_array what);

/* Scalar sizes of the built structures (host): 0 max n_i, 1 max r_i, 2 Bezier cells,
 * 3 assembly tiles (8 consecutive rows each), 4 tile entries, 5 largest tile nnz, 6 largest tile
 * entry count, 7 largest tile member count, 8 (row, cell) pairs, 9 largest points x
 * functions of a cell entry, 10 largest member rows x points of a cell entry.
 * -1 if unknown. */
int64_t wq_points_info(const wq_points* pts, int what);
wq_status wq_points_get(const wq_points* pts, wq_array what, void* dst_device, wq_stream stream);

/* ------------------------------------------------------------------ solve_weights
 * For every row i and every family in fam_mask: the right-hand side b (the exact
 * integrals, computed ahead of the weights as Section 2 prescribes) by 4x4 Gauss
 * quadrature on every Bezier cell (Section 4.2), then the truncated-SVD weights of
 * Eqs. (20)-(22):
 *   A = U S V^T, keep sigma_k > tsvd_rel_cutoff * sigma_1,
 *   w = Z^2 V_t (V_t^T Z^2 V_t)^{-1} S_t^{-1} U_t^T b,  Z = diag(N_i(x_q)),
 * with the inverse applied through a QR factorisation of Z V_t (as Eq. (7) does for
 * A Z^2 A^T). The SVD in FP64: Householder QR of A^T with column pivoting, one-sided
 * Jacobi on the n x n triangular factor (left singular vectors directly), V_t formed as
 * A^T U_t S_t^{-1}. Where the pivoted QR alone proves how many singular values the
 * cutoff keeps (sigma_{k+1} <= ||R22|| below cutoff * R_00 / 10, sigma_k >=
 * 1 / ||R11^-1||_F - ||R22|| above 100 * cutoff * ||A||_F), the same solution is taken
 * from the k pivot rows of A directly (Z A_k^T = Q R, w = Z Q R^-T b_k) without the SVD.
 * Weights are stored aligned with Q_i.
 * report (host, nullable): per family counts and worst cases, see wq_solve_report; for
 * the systems solved without the SVD its ratios are the certified bounds.
 * Synchronises `stream`. Returns WQ_ESVD if a Jacobi SVD hit its sweep limit. */
typedef struct {
  int64_t systems;          /* number of (row, family) systems solved                 */
  int64_t truncated;        /* systems with t < n_i                                   */
  int32_t max_sweeps;       /* largest number of Jacobi sweeps used                   */
  double min_kept_ratio;    /* smallest sigma_t / sigma_1 kept                        */
  double max_dropped_ratio; /* largest sigma_{t+1} / sigma_1 dropped                  */
  int64_t certified;        /* systems whose kept count the pivoted QR proved (no SVD) */
} wq_solve_report;

wq_status solve_weights(wq_mesh* mesh, wq_points* pts, unsigned fam_mask, double tsvd_rel_cutoff,
                        wq_stream stream, wq_weights** out, wq_solve_report* report);
void wq_weights_destroy(wq_weights* w);

/* Device copies of the weights of one family (double[sum r_i], aligned with QIDX) and of
 * the Gauss right-hand sides of one family (double[nnz], aligned with COL). */
wq_status wq_weights_get(const wq_weights* w, wq_family fam, double* dst_device, wq_stream stream);
wq_status wq_rhs_get(const wq_weights* w, wq_family fam, double* dst_device, wq_stream stream);

/* ------------------------------------------------------------------ assembly
 * Row-wise WQ formation on the fixed pattern (Section 6.1: formed row by row).
 *   assemble_mass:       M_ij = sum_{q in Q_i} w^0_iq c(x_q) N_j(x_q)            (Eq. 9)
 *   assemble_stiffness:  K_ij = sum_q k(x_q) (w^x_iq dN_j/dx + w^y_iq dN_j/dy)   (Eq. 11)
 *   assemble_biharmonic: B_ij = sum_q d(x_q) w^L_iq Lap N_j(x_q)                 (Eq. 12)
 *   assemble_mass_stiffness: both M and K in one pass over the weights.
 * coef_at_points: device double[n_points] or NULL (coefficient 1).
 * vals: device output aligned with COL, double[nnz] for WQ_FP64, float[nnz] for the
 * low-precision contractions, which run the per-cell product (member rows x points) x
 * (points x functions) on MFMA with FP32 accumulation; cells are summed in FP64:
 *   WQ_SPLIT_FP16: each operand as two FP16 terms (22 bits; weights x coefficient scaled
 *     per row and cell by a power of two, basis data per family), three MFMA products;
 *   WQ_SPLIT_BF16: three BF16 terms (24 bits, no scaling), six MFMA products;
 *   WQ_SLICED_FP16: four 10-bit slices per operand on a grid shared along the summed
 *     index (row exponent for the weights, column exponent for the basis), so every
 *     MFMA sum is exact; ten MFMA products, about 40 bits.
 * The two split forms carry FP32 rounding relative to the sum of |terms|: where a
 * contraction cancels (stiffness rows: oscillating derivative-family weights) their
 * normwise error grows by that cancellation factor; the sliced form does not.
 * Asynchronous on `stream`. The first low-precision call on a handle converts the basis
 * data (allocates and synchronises). */
wq_status assemble_mass(const wq_points* pts, const wq_weights* w, const double* coef_at_points,
                        void* vals, wq_precision prec, wq_stream stream);
wq_status assemble_stiffness(const wq_points* pts, const wq_weights* w, const double* coef_at_points,
                             void* vals, wq_precision prec, wq_stream stream);
wq_status assemble_biharmonic(const wq_points* pts, const wq_weights* w, const double* coef_at_points,
                              void* vals, wq_precision prec, wq_stream stream);
wq_status assemble_mass_stiffness(const wq_points* pts, const wq_weights* w, const double* c_at_points,
                                  const double* k_at_points, void* mass_vals, void* stiff_vals,
                                  wq_precision prec, wq_stream stream);

/* ------------------------------------------------------------------ Gauss comparison
 * Element-wise Gauss quadrature, the system WQ is compared against (Section 1: the
 * standard loop over elements with 4 x 4 Gauss points per Bezier cell; Section 6.1 times
 * it against row-wise WQ with the basis at the quadrature points computed ahead and
 * excluded), on the same CSR pattern as the WQ matrices.
 * gauss_setup: the basis at the 16 Gauss points of every cell (values, physical
 *   gradients, Laplacians when want_laplacian, which needs build_points(want_laplacian=1)),
 *   the weights w_g |det J| and the physical points; synchronises `stream`.
 * wq_gauss_size: the number of Gauss points (16 per cell); wq_gauss_get_x copies their
 *   coordinates (device double[dim * size], the mesh's dim coordinates per point,
 *   cell-major, 4 x 4 points per cell with the first cell coordinate fastest).
 *   On a surface (dim 3) the stiffness sums the three surface-gradient components and
 *   the biharmonic kind uses the Laplace-Beltrami operator.
 * assemble_gauss: vals (device double[nnz], aligned with COL) :=
 *   WQ_GQ_MASS:       sum_cells sum_g w_g |det J| c_g N_i N_j
 *   WQ_GQ_STIFFNESS:  sum_cells sum_g w_g |det J| c_g grad N_i . grad N_j
 *   WQ_GQ_BIHARMONIC: sum_cells sum_g w_g |det J| c_g Lap N_i Lap N_j
 *   with coef_at_gauss (device double[size] in the order of wq_gauss_get_x, or NULL for
 *   1). Each cell's local matrix on FP64 MFMA, added into vals by FP64 atomics: the
 *   order of the additions, and so the last bits, can differ between runs. Asynchronous
 *   on `stream`; the handle must outlive the work queued on it. */
typedef struct wq_gauss wq_gauss;
typedef enum { WQ_GQ_MASS = 0, WQ_GQ_STIFFNESS = 1, WQ_GQ_BIHARMONIC = 2 } wq_gauss_kind;
wq_status gauss_setup(wq_mesh* mesh, wq_points* pts, int want_laplacian, wq_stream stream, wq_gauss** out);
void wq_gauss_destroy(wq_gauss* g);
int64_t wq_gauss_size(const wq_gauss* g);
wq_status wq_gauss_get_x(const wq_gauss* g, double* dst_device, wq_stream stream);
wq_status assemble_gauss(const wq_gauss* g, wq_gauss_kind kind, const double* coef_at_gauss, double* vals,
                         wq_stream stream);

/* ------------------------------------------------------------------ nonlinear heat
 * Section 5: Tdot N_A + k(T) grad T . grad N_A - f N_A = 0 (weak residual), time by the
 * generalised trapezoidal rule, Newton with the symmetric tangent of Eq. (35).
 * Thermal conductivity k(u): kind 0 a + b u, 1 a + b u^2, 2 a exp(b u), 3 a sin(b u)
 * (Section 6.3 uses k = 1, e^{-T}, sin(pi T) and 200 - 0.05 T). */
typedef enum { WQ_K_LINEAR = 0, WQ_K_QUADRATIC = 1, WQ_K_EXP = 2, WQ_K_SIN = 3 } wq_k_kind;
typedef struct {
  int32_t kind; /* wq_k_kind */
  double a, b;
} wq_conductivity;

/* assemble_tangent: for the spline fields T, Tdot (device double[n_rows], coefficients
 * of N_j), with T_q = T(x_q), grad T(x_q), Tdot(x_q) at every WQ point and k_q = k(T_q):
 *   S_ij = sum_{q in Q_i} [inv_theta_dt w^0_iq N_j(x_q)
 *                          + k_q (w^x_iq dN_j/dx(x_q) + w^y_iq dN_j/dy(x_q))]   (Eq. 36)
 *   R_i  = sum_{q in Q_i} [w^0_iq (Tdot(x_q) - f_q) + k_q (w^x_iq dT/dx + w^y_iq dT/dy)]
 * i.e. R = M Tdot + K[k_q] T - F with F_i = sum_q w^0_iq f_q (the WQ load vector).
 * Needs the MASS, DX and DY weights. f_at_pts: device double[n_points] or NULL (f = 0).
 * S_vals: device double[nnz] aligned with COL; R: device double[n_rows]. Only WQ_FP64.
 * Asynchronous on `stream`; uses scratch owned by `pts` (allocated on the first call),
 * so calls on the same handle must not overlap. */
wq_status assemble_tangent(const wq_points* pts, const wq_weights* w, const double* T, const double* Tdot,
                           double inv_theta_dt, wq_conductivity k, const double* f_at_pts, void* S_vals,
                           double* R, wq_precision prec, wq_stream stream);

/* assemble_tangent_exact: as assemble_tangent, with the exact Newton tangent of Eq. (34):
 * S also carries the non-symmetric term that Eq. (35) drops, read as the derivative of R
 * (the printed term is garbled):
 *   S_ij += sum_{q in Q_i} k'(T_q) N_j(x_q) (w^x_iq dT/dx(x_q) + w^y_iq dT/dy(x_q)).
 * Newton then converges quadratically. Same arguments, residual and asynchrony as
 * assemble_tangent; its scratch in `pts` holds 6 doubles per point (allocated on the
 * first call). */
wq_status assemble_tangent_exact(const wq_points* pts, const wq_weights* w, const double* T, const double* Tdot,
                                 double inv_theta_dt, wq_conductivity k, const double* f_at_pts, void* S_vals,
                                 double* R, wq_precision prec, wq_stream stream);

/* assemble_tangent_noalloc: assemble_tangent for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same arguments, kernels and results (bit for bit) as assemble_tangent; the
 * point fields live in a fixed array of the library, one per GPU (16 MiB: 4 doubles per
 * point for at most 524288 points), instead of scratch owned by `pts`. It calls no
 * hipMalloc, hipFree or other allocating routine. Errors: WQ_EINVAL if the handle has more
 * than 524288 points, or if its device is not the current device. All calls on one GPU
 * share the array and it keeps the last call's contents (each call overwrites all of the
 * part it reads): calls that overlap on one GPU (other streams or threads) race, and the
 * caller must serialise them. Asynchronous on `stream`. */
wq_status assemble_tangent_noalloc(const wq_points* pts, const wq_weights* w, const double* T, const double* Tdot,
                                   double inv_theta_dt, wq_conductivity k, const double* f_at_pts, void* S_vals,
                                   double* R, wq_precision prec, wq_stream stream);

/* wq_heat_step: one time step t_n -> t_{n+1} (Section 5.2). Predictor
 * T = T_n + (1 - theta) dt Tdot_n with T = g on prescribed DOFs; corrector iterations:
 * Tdot = (T - T_n - (1 - theta) dt Tdot_n) / (theta dt), S and R by assemble_tangent,
 * stop when ||R over free DOFs||_2 <= tol, else solve -S_ff dT_f = R_f (Eq. 33) by
 * Jacobi-preconditioned BiCGStab on the device (with a variable conductivity the WQ
 * tangent is not symmetric: each row is integrated with its own weights) and T_f += dT_f.
 * Prescribed DOFs keep g (their rows and columns are eliminated).
 *   dirichlet: device uint8[n_rows], 1 = prescribed; g_next: device double[n_rows] or
 *   NULL (prescribed values 0); f_at_pts: device double[n_points] (f at t_{n+1}) or NULL;
 *   T, Tdot: device double[n_rows], in: T_n, Tdot_n; out: T_{n+1}, Tdot_{n+1};
 *   S_vals: device double[nnz], receives the last tangent.
 * hp->tangent: WQ_TANGENT_SYMMETRIC (Eq. (35), as the paper) or WQ_TANGENT_EXACT (Eq. (34),
 * assemble_tangent_exact: quadratic convergence).
 * Synchronises `stream` (convergence tests read norms on the host). Returns
 * WQ_ENOCONV if Newton or BiCGStab hit their caps (T, Tdot then hold the last iterate).
 * Uses scratch owned by `pts`: calls on the same handle must not overlap. */
typedef enum { WQ_TANGENT_SYMMETRIC = 0, WQ_TANGENT_EXACT = 1 } wq_tangent;
typedef struct {
  double dt, theta;     /* time step, trapezoidal parameter in (0, 1]                 */
  wq_conductivity k;
  double tol;           /* Newton stop: ||R_free||_2 <= tol (absolute)                */
  int32_t max_newton;   /* Newton iteration cap                                       */
  double cg_rtol;       /* Krylov stop: ||r||_2 <= max(cg_rtol ||R_free||_2, tol/10) */
  int32_t max_cg;       /* Krylov iteration cap per solve                             */
  int32_t tangent;      /* wq_tangent                                                 */
} wq_heat_params;
typedef struct {
  int32_t newton_iters; /* corrector solves taken                                     */
  int32_t cg_iters;     /* BiCGStab iterations, all solves                            */
  double residual0;     /* ||R_free||_2 after the predictor                           */
  double residual;      /* final ||R_free||_2                                         */
} wq_heat_report;
wq_status wq_heat_step(const wq_points* pts, const wq_weights* w, const wq_heat_params* hp,
                       const uint8_t* dirichlet, const double* g_next, const double* f_at_pts, double* T,
                       double* Tdot, double* S_vals, wq_heat_report* rep, wq_stream stream);

/* ------------------------------------------------------------------ serving
 * A request loop for the nonlinear heat problem of Section 5 on meshes that arrive over
 * time (the paper's setting of repeated assembly on fixed domains, many domains).
 * A request carries a mesh, its prescribed DOFs (value 0), heat parameters and a number
 * of time steps from T = Tdot = 0; the server builds the points and the MASS/DX/DY
 * weights, runs the steps with wq_heat_step (source: none, or the manufactured
 * f = d(T*)/dt - div(k(T*) grad T*) for T* = (1 - e^{-lambda t}) sin(pi x) sin(pi y)) and
 * copies the final T to the caller's host buffer.
 * Admission: requests start in arrival order as soon as a slot is free and their HBM
 * estimate (from the mesh sizes) fits in the budget next to the running ones; each slot
 * is a host thread with its own non-blocking stream of default priority, so admitted
 * requests overlap on the device. Results do not depend on what else runs (the kernels
 * use fixed summation orders).
 *   wq_server_start: budget in bytes, 1..16 slots; the current device is used.
 *   wq_server_submit: copies the request's host arrays; T_out (host double[n_fn]) must
 *     stay valid until the request completes. WQ_ENOMEM if the estimate alone exceeds
 *     the budget. Returns a ticket.
 *   wq_server_poll: 1 = done (result copied to *out, ticket released), 0 = pending
 *     (wait = 0), negative = bad ticket. wait != 0 blocks until done.
 *   wq_server_stop: finishes queued and running requests, then frees the server.
 * Times are seconds since wq_server_start.
 * Setups are kept: after a request completes, its domain's mesh, points and weights (the
 * part computed once per fixed domain, Section 2) stay on the device, still charged to
 * the budget at the request's estimate. A later request whose mesh arrays are identical
 * takes an idle one over (one request at a time) and skips that work; a request that
 * needs room releases idle setups, least recently used first. Requests with
 * reuse_setup = 0 neither take over nor leave a setup. */
typedef struct wq_server wq_server;
typedef enum { WQ_SOURCE_NONE = 0, WQ_SOURCE_MANUFACTURED = 1 } wq_source;
typedef struct {
  wq_mesh_desc mesh;          /* host arrays, copied at submit                           */
  const uint8_t* dirichlet;   /* host uint8[n_fn], 1 = prescribed (value 0)              */
  wq_heat_params heat;
  int32_t n_steps;
  int32_t source;             /* wq_source                                               */
  double lambda;              /* manufactured source rate                                */
  int32_t reuse_setup;        /* 1: may take over a held setup of an identical domain and
                                 leave its own setup held; 0: set up from scratch and
                                 release it at completion                                */
} wq_request;
typedef struct {
  int32_t status;             /* wq_status of the whole request                          */
  int32_t newton_iters;       /* corrector solves, all steps                             */
  int32_t cg_iters;           /* BiCGStab iterations, all steps                          */
  int64_t n_rows, nnz;
  double residual;            /* final ||R_free||_2 of the last step                     */
  double submitted, started, finished;
  size_t hbm_estimate;        /* bytes charged against the budget while running, and
                                 while the server holds the request's setup afterwards   */
  int32_t setup_reused;       /* 1 if a held setup of the same domain was taken over     */
  int32_t joined;             /* meshes in the union the request ran in (1: alone)       */
} wq_result;
wq_status wq_server_start(size_t hbm_budget_bytes, int32_t slots, wq_server** out);
wq_status wq_server_submit(wq_server* server, const wq_request* req, double* T_out, int64_t* ticket);
int wq_server_poll(wq_server* server, int64_t ticket, int wait, wq_result* out);
void wq_server_stop(wq_server* server);

/* wq_server_set_join: joining of requests that are queued together (off by default,
 * max_meshes = 1). When a slot admits the oldest request and it has no held setup to take
 * over, later queued requests with the same heat parameters, step count and source (and
 * lambda) that have no idle held setup of their own domain and fit in the budget next to
 * it, up to max_meshes requests and max_rows rows (functions) in all, run with it as one: their meshes are joined into
 * one disjoint union (as wq_batch_create), the points and weights are built once over it,
 * and each time step is one heat step over the union with one segment per mesh, so that
 * setup and every Newton and Krylov step of all of them share launches. The union's tangent
 * is block diagonal; each segment is solved as if alone (its reductions sum its own rows in
 * the order they take alone, its scalars and its Newton and Krylov stops are its own), so a
 * joined request's temperature, iteration counts, residual and status are bit for bit those
 * it gets alone (wq_result.joined > 1 reports the union's size). A failed member does not
 * stop the others. No setup of a joined request is held afterwards. Joining pays where launches and host
 * round trips, not the device's throughput, bound a request (small meshes); max_rows keeps
 * larger ones apart (a request above it runs alone). Applies to admissions after the call;
 * max_meshes in 1..4096 and max_rows >= 0, else WQ_EINVAL. */
wq_status wq_server_set_join(wq_server* server, int32_t max_meshes, int64_t max_rows);

/* ------------------------------------------------------------------ batching
 * Many independent meshes through one set of launches: wq_batch_create joins them into
 * one disjoint union (vertex, face and function ids offset mesh by mesh, in the given
 * order) on the device; wq_batch_build runs build_points and solve_weights once over the
 * union, so the weight systems of all meshes are binned together by size and every
 * mesh's rows, points, weights and matrix values equal those it gets alone (the method
 * is local to each function's support). Mesh k owns rows [row0, row0 + n_rows), CSR
 * entries [nnz0, nnz0 + nnz) (columns are union ids, i.e. offset by row0) and points
 * [pt0, pt0 + n_points) of the union (wq_batch_info). wq_batch_points/weights return
 * the union handles (owned by the batch) for the assemble_* calls and array queries.
 * wq_batch_graph_assemble: mass + stiffness of all meshes as a HIP graph; the first call
 * (or a call with other pointers, precision or stream) runs once eagerly, captures the
 * launch and instantiates it; later calls replay it. The captured pointers are used as
 * they are: update the coefficient buffers' contents in place between replays. The
 * stream must be a created stream (capture is not possible on the null stream).
 * wq_batch_build and the first graph call synchronise `stream`. */
typedef struct wq_batch wq_batch;
wq_status wq_batch_create(const wq_mesh_desc* meshes, int32_t n_meshes, wq_batch** out);
wq_status wq_batch_build(wq_batch* batch, unsigned fam_mask, double tsvd_rel_cutoff, wq_stream stream,
                         wq_solve_report* report);
wq_status wq_batch_info(const wq_batch* batch, int32_t mesh, int64_t* row0, int64_t* n_rows, int64_t* nnz0,
                        int64_t* nnz, int64_t* pt0, int64_t* n_points);
wq_points* wq_batch_points(wq_batch* batch);
wq_weights* wq_batch_weights(wq_batch* batch);
wq_status wq_batch_graph_assemble(wq_batch* batch, const double* c_at_points, const double* k_at_points,
                                  void* mass_vals, void* stiff_vals, wq_precision prec, wq_stream stream);
void wq_batch_destroy(wq_batch* batch);

/* wq_autotune_assembly: times the FP64 mass + stiffness assembly on `pts` for each
 * candidate length of the runs of consecutive row tiles that one XCD takes in turn
 * (powers of two from 4 to 1024 below ceil(n_tiles / 8), then ceil(n_tiles / 8): one
 * contiguous band of tiles per XCD), keeps the fastest in the handle (later assembly
 * calls on it use it) and returns it with its median time in ms. Synchronises `stream`. */
wq_status wq_autotune_assembly(wq_points* pts, const wq_weights* w, wq_stream stream, int32_t* chosen_chunk,
                               double* best_ms);

/* wq_autotune_tiles: the tile shape of the same assembly, tuned with the run length. The
 * cell-major tiles (runs of at most 16 consecutive rows and 416 CSR entries, one wave each)
 * are also capped by their summed row steps (a row's step count: the blocks of four points
 * of its support cells), so that tiles next to extraordinary points do not take several
 * times the average tile's time. For each candidate cap (64, 96, 128, 192, 256, none) the
 * tiles of `pts` are rebuilt and the run length tuned as above; the fastest pair is kept in
 * the handle and returned with its median time in ms (the default cap is 128). Values are
 * unchanged: a row's sums do not depend on its tile. A batch's captured assembly graph is
 * captured again at its next call. Calls on `pts` must not overlap this one; synchronises
 * `stream`. */
wq_status wq_autotune_tiles(wq_points* pts, const wq_weights* w, wq_stream stream, int32_t* chosen_stepcap,
                            int32_t* chosen_chunk, double* best_ms);

/* ------------------------------------------------------------------ kernel timing
 * Measurement aid. While enabled (per process), the library records a pair of HIP
 * events on the launch stream around each of its main kernels (basis evaluation,
 * Gauss basis, Gauss rows, TSVD per size bucket, assembly). wq_timings() waits for the
 * recorded events, copies up to `cap` records into `out` (host) and clears the list;
 * it returns the number of records written. `name` is the kernel (TSVD: its template
 * instance). `work` is the launch's algorithmic work: for TSVD the FLOPs
 * sum(9 r n^2 - n^3) over its systems, for assembly the bytes 8 * (every basis value
 * and weight read once + coefficients + outputs), otherwise the unit count (points,
 * rows). */
typedef struct {
  char name[40];
  double ms;
  int64_t work;
} wq_timing;
void wq_timing_enable(int on);

/* wq_set_side_streams: streams for the independent launches within one call (the size
 * buckets of solve_weights and their second launches): n non-blocking streams of default
 * priority, created per call, forked from the caller's stream and joined back into it by
 * events, so the call stays ordered on `stream` as before. Small and partial launches then
 * fill CUs the large ones leave idle. 4 by default; n = 1 keeps every launch on the
 * caller's stream (then a timing record is the kernel's own time: with several, records
 * of concurrent kernels overlap). Results do not depend on it. n in 1..8, else WQ_EINVAL;
 * applies to calls that start after it. */
wq_status wq_set_side_streams(int32_t n);
int wq_timings(wq_timing* out, int cap);

/* ------------------------------------------------------------------ errors */
const char* wq_strerror(wq_status s);
const char* wq_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* WQ_H */
