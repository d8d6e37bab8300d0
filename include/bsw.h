/*
 * bsw.h -- C ABI of the MI355X (gfx950) library for the regularised-Bingham
 * shallow-water discontinuous Galerkin method of Fernandez, Lopez-Ordonez and
 * Gonzalez-Andrade (arXiv 2301.11238).
 *
 * The library evaluates the DG spatial operator of the paper's backward-Euler
 * step (Sec. 5.1, Eq. WeakForm7), its element-block Jacobian (Appendix A,
 * Eq. Newton) and the stage update, and drives whole solves.  All arrays named
 * `void*` below are DEVICE pointers owned by the caller (for example
 * torch.Tensor.data_ptr()); their element type is the discretisation's
 * precision (double for BSW_FP64, float for BSW_FP32).  `double*` arguments
 * named *_out or host_* are HOST pointers.  Handles are owned by the library
 * and released by the matching *_destroy call.
 *
 * State layout ("SoA", elements fastest): W[f][i][e] with f the field, i the
 * basis function, e the element.  Fields: 1-D (h, u, E11); 2-D
 * (h, u1, u2, E11, E21, E12, E22) with E_ab = d u_b / d x_a, the velocity
 * gradient of Sec. 3 (Eq. gradientVel).  Modal coefficients in the orthonormal
 * basis: normalised Legendre on [-1, 1] (Sec. 5) and the orthonormal Dubiner
 * basis on the unit triangle, modes ordered by total degree then by the
 * second index.  b_old and the first 1+d fields of R use the same layout.
 *
 * Every call returns an int status: BSW_OK (0), a negative error, or a
 * positive warning.  Nothing throws across this boundary.  bsw_last_error()
 * returns the context's last message.  Device work is enqueued on the
 * context's HIP stream and is asynchronous unless a host output is requested
 * (norms, diagnostics, solve statistics), in which case the call synchronises
 * that stream.
 */
#ifndef BSW_H
#define BSW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  BSW_OK = 0,
  BSW_E_ARG = -1,         /* invalid argument (sizes, null pointers, unsupported order) */
  BSW_E_OOM = -2,         /* device allocation failed */
  BSW_E_HIP = -3,         /* a HIP runtime call failed */
  BSW_E_STATE = -4,       /* call out of order (e.g. Jacobian apply before linearize) */
  BSW_E_MESH = -5,        /* degenerate or non-manifold mesh */
  BSW_W_NOT_CONVERGED = 1 /* warning: some Newton step hit its iteration cap */
};

enum { BSW_FP64 = 0, BSW_FP32 = 1 };
enum { BSW_REG1 = 1, BSW_REG2 = 2, BSW_REG3 = 3 };
enum { BSW_BC_WALL = 1, BSW_BC_NEUMANN = 2, BSW_BC_DIRICHLET = 3 };
enum {
  BSW_IC_CONST = 0, BSW_IC_STEP_X = 1, BSW_IC_MOUND = 2, BSW_IC_DISK = 3,
  BSW_IC_SINE_U = 4, BSW_IC_LINEAR_X = 5, BSW_IC_SHEAR_Y = 6, BSW_IC_VORTEX = 7,
  BSW_IC_SURFACE = 8
};
enum { BSW_BED_FLAT = 0, BSW_BED_COS = 1, BSW_BED_GAUSS = 2 };

typedef struct bsw_ctx_s* bsw_ctx;
typedef struct bsw_mesh_s* bsw_mesh;
typedef struct bsw_disc_s* bsw_disc;

/* Physical and regularisation parameters (Sec. 3: g, rho, alpha; Sec. 4: eta,
 * sigma0, gamma, beta and the regularisation k = reg in {1, 2, 3}).
 * bc applies to every boundary face without a code of its own
 * (bsw_mesh_set_boundary): wall (mirror state: h+ = h-, u+ = R u-,
 * E+ = R E- R with R = I - 2 n n^T), homogeneous Neumann (V+ = V-, E+ = E-,
 * Sec. 5.2) or Dirichlet (exterior state = dirichlet[0..n_f-1], Sec. 5.2;
 * faces with tag t = 1..3 take dirichlet_tag[t-1] instead).
 * Regularisations 1 and 2 need sigma0 = 0 or sigma0 >= 1 / (2 beta). */
typedef struct {
  double g, rho, alpha, eta, sigma0, gamma, beta;
  int32_t reg;
  int32_t bc;
  double dirichlet[7];
  int32_t jac_frozen;  /* Jacobian only: 0 exact (the HLL wave speeds S_L, S_R
                          differentiated), 1 the paper's Appendix A form with
                          S_L, S_R held fixed.  The residual is the same. */
  double dirichlet_tag[3][7]; /* exterior states of Dirichlet faces tagged 1..3 */
} bsw_params;

/* Analytic initial condition, L2-projected with the element rule; E = 0.
 * Where the projected depth falls below a tenth of the element mean at a
 * volume or face point (a discontinuous depth cut by the element), the higher
 * depth modes are scaled so that the minimum is a tenth of the mean.
 * kinds: CONST h=a,u=(b,c); STEP_X h = x<x0 ? a : b; MOUND h = a+b exp(-|x-x0,y0|^2/d);
 * DISK h = |x-(x0,y0)|<r ? a : b; SINE_U h=a,u1=b sin(pi x/L); LINEAR_X h=a+b x;
 * SHEAR_Y h=a,u1=b cos(pi y/L); VORTEX h=a, u=b(sin(pi x/L)cos(pi y/L), -cos(pi x/L)sin(pi y/L));
 * SURFACE h = a + b x1 - H with H the discretisation's bed (bsw_disc_set_bed;
 * zero when flat), u = 0: the linear free surface is projected exactly and the
 * bed coefficients subtracted, so h + H equals it mode by mode and h is as
 * continuous across faces as H (Sec. 6.1 and 6.2 initial states); no
 * positivity scaling. */
typedef struct {
  int32_t kind;
  double a, b, c, d, x0, y0, r, L;
} bsw_ic;

/* Analytic bed height H of the momentum source -g_c h dH/dx (Eq. Sterm):
 * FLAT H = 0; COS H = a cos(kx x1) cos(ky x2) (1-D: a cos(kx x1));
 * GAUSS H = a exp(-|x - (x0, y0)|^2 / d).  order = m0, the polynomial order of
 * the bed (Sec. 5: H is projected at order m0; 1 <= m0 <= P, 0 selects P). */
typedef struct {
  int32_t kind, order;
  double a, kx, ky, x0, y0, d;
} bsw_bed;

/* Whole-solve controls (Sec. 5.1 and Sec. 6: at most max_newton = 10 Newton
 * iterations per step).  dt > 0 fixes the step; otherwise
 * dt = cfl * h_min / max(|u| + sqrt(g h)) over the initial state's volume
 * points, and the last step is clipped to land on t_end. */
/* With BSW_FP32 the tolerances are floored at newton_tol 2e-6 and gmres_rtol
 * 1e-6 (float rounding of the state). */
typedef struct {
  int32_t max_newton;      /* Newton iterations per time step */
  int32_t gmres_m;         /* GMRES restart length (<= 64) */
  int32_t gmres_max_iters; /* total GMRES iterations per Newton system */
  double newton_tol;       /* stop when ||dW||_inf <= newton_tol (1 + ||W||_inf) */
  double gmres_rtol;       /* tightest relative residual asked of GMRES; each Newton
                              system uses an Eisenstat-Walker forcing term in
                              [gmres_rtol, forcing_max] */
  double cfl, t_end, dt;
  int32_t max_steps;       /* < 0: all steps */
  int32_t timing;          /* nonzero: time the Jacobian applies of every fourth Arnoldi step
                            * with HIP events (events on every apply would slow the solve) */
  double forcing_max;      /* largest GMRES relative tolerance of a Newton system (the
                              forcing term's ceiling); <= 0 selects 3e-2 */
  int32_t cont_steps;      /* continuation on gamma (Sec. 6.3): n >= 2 Newton solves per
                              time step at gamma_i = cont_gamma0 + (i-1)(gamma -
                              cont_gamma0)/(n-1), each starting from the last; beta and
                              the other parameters stay.  < 2: one solve at gamma */
  double cont_gamma0;      /* first gamma of the continuation (> 0 when cont_steps >= 2) */
  int32_t precond_lag;     /* 0: rebuild the block-Jacobi preconditioner every Newton
                              iteration; 1: build it at the first iteration of each
                              Newton solve and keep it while GMRES converges within
                              1.5x (+10) the iterations it took right after the build
                              (the Jacobian products always use the current state) */
  double res_tol;          /* Newton also stops when ||R||_2 <= res_tol ||b_old||_2,
                              checked on the initial and every accepted residual;
                              0 selects 1e-13, a negative value turns it off */
} bsw_solve_opts;

typedef struct {
  int32_t steps, newton_total, gmres_total, newton_max, capped, status;
  double dt, mass0, mass_end, max_mass_drift, active_pct, t_end, seconds;
  double operator_applies, jacobian_applies; /* counts of whole-mesh applies */
  double jac_apply_seconds;  /* summed HIP-event time of the Jacobian-apply launches (timing != 0) */
  double jac_apply_launches; /* launches that were timed */
  double queue_seconds;      /* served solves: submit to admission (seconds is admission to completion) */
  double host_issue_seconds; /* timing != 0: host time spent issuing the pipelined Arnoldi steps
                                (all launches of a step) ... */
  double host_wait_seconds;  /* ... and blocked waiting for a step's results */
  double arnoldi_steps;      /* timing != 0: Arnoldi steps issued and read */
} bsw_solve_stats;

/* ---------------------------------------------------------------- context */
/* Binds a device and a HIP stream (NULL: the null stream; the caller may pass
 * torch's current stream).  The stream must outlive the context.  The first
 * context on a device also looks up that device's copy of the library's
 * fixed scratch array (used by bsw_stage_update_noalloc). */
int bsw_ctx_create(int device, void* hip_stream, bsw_ctx* out);
int bsw_ctx_destroy(bsw_ctx ctx);
const char* bsw_last_error(bsw_ctx ctx);

/* ---------------------------------------------------------------- mesh (Sec. 5: Omega^h = U Omega_e^h) */
/* Host inputs: xy[n_vert * dim] vertex coordinates; el2vert[n_el * (dim+1)]
 * counter-clockwise triangles (2-D) or increasing segments (1-D).  The library
 * builds face->neighbour maps, outward normals, face lengths and the affine
 * metrics on the host and copies them to the device; the host arrays may be
 * freed on return.  Returns BSW_E_MESH for non-positive Jacobians or faces
 * shared by more than two elements. */
int bsw_mesh_upload(bsw_ctx ctx, int dim, int64_t n_vert, const double* xy, int64_t n_el,
                    const int32_t* el2vert, bsw_mesh* out);
int bsw_mesh_destroy(bsw_mesh mesh);
/* Boundary condition of each boundary face (Sec. 5.2; the examples of
 * Sec. 6.1 and 6.2 mix Dirichlet data of two depths, or a Neumann and a
 * no-flow end).  face_bc (host, n_el * faces per element, index
 * e * faces + local face; 1-D: face 0 at the element's first vertex, face 1
 * at its second; triangles: face f from vertex f to f+1) holds
 * code = kind | tag << 2: kind BSW_BC_WALL, BSW_BC_NEUMANN or
 * BSW_BC_DIRICHLET, or 0 for the parameters' bc; a Dirichlet face takes the
 * state of its tag (0: params.dirichlet, 1..3: params.dirichlet_tag[tag-1]).
 * Interior faces' entries are ignored; NULL gives every boundary face code 0.
 * The codes apply to every discretisation of the mesh; BSW_E_ARG for codes
 * outside 0..15. */
int bsw_mesh_set_boundary(bsw_mesh mesh, const int8_t* face_bc);

/* ---------------------------------------------------------------- discretisation */
/* Order P (1-D: 0..4; triangles: 1..3 with 3/7/12-point volume rules and P+1
 * Gauss points per edge) and precision (BSW_FP64 or BSW_FP32).  Builds the
 * reference tables (basis and gradients at the volume points, basis at the
 * face points, weights) in FP64 on the host and stages them in constant
 * memory.  The mesh must outlive the discretisation. */
int bsw_disc_create(bsw_mesh mesh, int P, int precision, bsw_disc* out);
int bsw_disc_destroy(bsw_disc disc);
/* info[8] = {dim, P, n_p, n_q, n_fq, n_faces_per_element, n_f, n_el} */
int bsw_disc_info(bsw_disc disc, int64_t* info);
/* n_f * n_p * n_el: the number of reals in W */
int64_t bsw_state_len(bsw_disc disc);

/* L2 projection of an analytic initial condition into W (device). */
int bsw_project_ic(bsw_disc disc, const bsw_ic* ic, void* W);

/* ---------------------------------------------------------------- variable bed (Eq. Sterm, Sec. 5, Sec. 6.1) */
/* Writes the order-m0 interpolant of bed into H (device, n_p * n_el reals of
 * the discretisation's precision, layout [i][e] like one field of W).  The
 * nodes are shared by neighbouring elements: Gauss-Lobatto points in 1-D; on
 * triangles the vertices, the interior Gauss-Lobatto points of each edge and,
 * for m0 = 3, the centroid.  The interpolant's face traces therefore agree,
 * which the lake at rest needs (the HLL flux damps depth jumps).  Modes of
 * degree above m0 are zero.  BSW_E_ARG for m0 outside 1..P (1-D: P <= 4,
 * triangles: P <= 3) or a bad kind. */
int bsw_bed_interpolate(bsw_disc disc, const bsw_bed* bed, void* H);
/* Sets the bed of the momentum source: H (device, layout as above) is kept by
 * reference and must stay valid and unchanged while the discretisation uses
 * it; NULL returns to the flat bed.  The next operator, linearize and solve
 * calls use it; a Jacobian linearized before the call must be linearized
 * again (BSW_E_STATE until then). */
int bsw_disc_set_bed(bsw_disc disc, const void* H);

/* ---------------------------------------------------------------- mixed orders (Sec. 5: m1, m2, m3) */
/* Orders of h, u and E, each in 0..P (P, the discretisation's order, is the
 * storage order and sets the quadrature rules; default m1 = m2 = m3 = P).
 * With the degree-ordered bases, a field of order m keeps its first N(m)
 * modes (N(m) = m + 1 in 1-D, (m + 1)(m + 2)/2 on triangles) and is tested
 * with them.  The higher modes stay in W and carry the trivial equations
 * W = 0: their residual rows equal the coefficient, their Jacobian rows are
 * identity rows (in the diagonal blocks of bsw_jacobian_blocks and the
 * preconditioner their columns are unit columns too, so solves keep them
 * exactly zero), and bsw_project_ic zeroes them (the L2 projection onto the
 * field's space, taken before the positivity scaling; for IC kind SURFACE
 * after subtracting the bed).  A bed may have any order m0 <= P, above m1
 * too (then the lake at rest is not exact, Sec. 6.1).  The Jacobian must be
 * linearized again after a change (BSW_E_STATE until then).  BSW_E_ARG for
 * orders outside 0..P. */
int bsw_disc_set_orders(bsw_disc disc, int m1, int m2, int m3);

/* ---------------------------------------------------------------- the operator */
/* b_old[f][i][e] = (1/dt) <phi_i, U_f(W_old)>_e for f < 1+d: the old-time part
 * of the first term of Eq. WeakForm7 (U = (h, h u), Eq. Uterm). */
int bsw_step_begin(bsw_disc disc, const bsw_params* prm, double dt, const void* W_old,
                   void* b_old);

/* R = the element residuals of Eq. WeakForm7 at W given b_old: volume fluxes
 * F (Eq. Fterm), the regularised Bingham stress term Q (Eq. Qterm, Sec. 4),
 * the source S (Eq. Sterm, with the bed set by bsw_disc_set_bed), the auxiliary
 * equation for E (Eq. Gterm),
 * HLL face fluxes for F (Eq. HLLSolver) and central ones for Q and G (Sec. 5).
 * Layout of R as W.  W, b_old and R must not alias. */
int bsw_operator_apply(bsw_disc disc, const bsw_params* prm, double dt, const void* W,
                       const void* b_old, void* R);

/* ---------------------------------------------------------------- element-block Jacobian (Appendix A) */
/* Records W (device pointer, kept by reference: the caller must not change or
 * free it until the next linearize), the parameters and dt; assembles the
 * diagonal blocks dR_e/dW_e of Eq. Newton and factors them for the
 * block-Jacobi preconditioner through the Schur complement of the stress block
 * (whose own block is the diagonal element mass matrix): the inverse of the
 * depth-velocity Schur complement (Gauss-Jordan with partial pivoting) and
 * the velocity rows' stress couplings, kept in FP32 (in 1-D also the stress
 * rows' velocity couplings and the diagonal; on triangles those come from
 * the geometry).  On triangles only the block parts the factors read are
 * assembled here; bsw_jacobian_blocks assembles whole blocks. */
int bsw_jacobian_linearize(bsw_disc disc, const bsw_params* prm, double dt, const void* W);
/* y = (dR/dW)(W) x, the directional derivative including the face coupling to
 * neighbours (matrix-free): exact, HLL wave speeds included, or with them held
 * fixed when prm->jac_frozen was set at linearize.  BSW_E_STATE before the
 * first linearize. */
int bsw_jacobian_apply(bsw_disc disc, const void* x, void* y);
/* y = blockdiag(dR_e/dW_e)^{-1} x from the factors of the last linearize
 * (FP32 factors, FP64 arithmetic). */
int bsw_precond_apply(bsw_disc disc, const void* x, void* y);
/* Writes the unfactored diagonal blocks of the last linearize to blocks
 * (device, [n_el][bs][bs] row-major, bs = n_f n_p, row/column index f*n_p+i);
 * on triangles they are assembled by this call from the linearisation state
 * (which must still be as recorded), into the library's block storage. */
int bsw_jacobian_blocks(bsw_disc disc, void* blocks);

/* ---------------------------------------------------------------- stage update and reductions */
/* W += alpha dW (Eq. Newton update).  norms_out (host, may be NULL) receives
 * FP64 {max|alpha dW|, max|W|, mass, active%} after the update, where
 * mass = sum_e sum_q w_q h(x_q) and active% = 100/|Omega| sum w_q H(s - sigma0/gamma)
 * (Sec. 6) with s the shear rate of the 2-D reading (|E| in 1-D). */
int bsw_stage_update(bsw_disc disc, const bsw_params* prm, void* W, const void* dW,
                     double alpha, double* norms_out);
/* bsw_stage_update without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): same arguments, same results as bsw_stage_update, but its
 * reduction partials and final values live in a fixed per-device array of the
 * library (4096 partial sums and 64 results, 33 KB per device, held until the
 * process ends) instead of memory bsw_stage_update allocates on first use.
 * No hipMalloc, hipFree or allocating library routine is called.  Every
 * workgroup writes its own partial before the final pass reads it, so nothing
 * needs clearing between calls.  All calls on one device share the array:
 * calls that overlap on one GPU (other streams or threads) race, so the
 * caller serialises them.  BSW_E_ARG if the reduction would need more partial
 * sums than the array holds (the workgroup counts are capped at 1024, so no
 * valid discretisation does); BSW_E_STATE for a context without the array. */
int bsw_stage_update_noalloc(bsw_disc disc, const bsw_params* prm, void* W, const void* dW,
                             double alpha, double* norms_out);
/* out4 (host) = {mass, active%, max(|u| + sqrt(g h)), min h} over volume points. */
int bsw_diagnostics(bsw_disc disc, const bsw_params* prm, const void* W, double* out4);
/* *out (host) = sqrt(sum x^2) accumulated in FP64. */
int bsw_norm2(bsw_disc disc, const void* x, double* out);
/* *dt_out (host) = cfl * h_min / max(|u| + sqrt(g h)) over W's volume points,
 * h_min the smallest element altitude (2-D) or length (1-D): the fixed time
 * step a whole solve takes from its initial state. */
int bsw_cfl_dt(bsw_disc disc, const bsw_params* prm, const void* W, double cfl, double* dt_out);

/* ---------------------------------------------------------------- whole solve */
/* Backward-Euler time loop from the state in W (device, updated in place) to
 * opts->t_end: per step b_old, then inexact Newton (residual, linearize,
 * block-Jacobi GMRES for Eq. Newton, backtracking on ||R||, update) until
 * ||dW||_inf <= newton_tol (1 + ||W||_inf) or max_newton iterations (per
 * continuation stage when cont_steps >= 2).  A step counts as capped when its
 * last Newton solve (at the target gamma) hit the cap.
 * Returns BSW_W_NOT_CONVERGED if any step hit the cap. */
int bsw_solve(bsw_disc disc, const bsw_params* prm, const bsw_solve_opts* opts, void* W,
              bsw_solve_stats* stats_out);

/* ---------------------------------------------------------------- element-tile autotuner */
/* The element pass of batched and whole solves (bsw_solve and the server)
 * runs in one of three variants.  On triangles: a workgroup of 4 waves on a
 * tile of 64 elements (one lane per element), compiled for at least 1, 2 or
 * 3 resident waves per SIMD (register budgets of 512, 256 and 168 per lane).
 * In 1-D: workgroups of 128, 256 or 512 lanes, each taking as many elements
 * as it has lanes per (volume + face) point set.  All variants give the same
 * bits.  Per (dimension, order, precision, residual or Jacobian pass, size
 * class floor(log2 of the launch's element count)) the library times the
 * first launches of every variant (HIP events, read without blocking) and
 * keeps the fastest for the process.  The single-call entry points
 * (bsw_operator_apply, bsw_jacobian_apply) use the variant the policy
 * forces, else variant 1.
 * bsw_tile_policy: -1 autotune (default), 0/1/2 force a variant;
 * *previous (may be NULL) receives the old policy.  Process-wide. */
int bsw_tile_policy(int policy, int* previous);
/* Up to max_rows rows of 10 doubles (host): {dim, P, bytes per real, pass
 * (0 residual, 1 Jacobian), size class, chosen variant (-1 while measuring),
 * best microseconds of variants 0, 1, 2 (-1 if not yet timed), timed
 * launches}; *n_rows receives the number of table entries. */
int bsw_tile_table(double* rows, int max_rows, int* n_rows);

/* ---------------------------------------------------------------- solve server (batched, continuous) */
/* A server owns a worker thread, its own HIP stream on the context's device
 * and a device-memory budget.  Submitted requests wait in a FIFO queue; between
 * time steps the worker admits the queue head while its footprint
 * (bsw_request_footprint) fits the remaining budget and fewer than max_slots
 * solves are resident, and retires finished solves (state copied to host
 * memory, device memory released).  Resident solves of the same order,
 * precision and restart length form one batch: every stage of their time
 * steps (b_old, residual, Jacobian blocks and their factors, block-Jacobi and
 * matrix-free Jacobian applies, Krylov vector updates, reductions) is one
 * kernel launch over all of them, while Newton, backtracking and GMRES
 * decisions stay per solve.  Reductions are per solve with a fixed shape, so
 * a solve's result does not depend on what else is resident.  Served solves
 * are 2-D with P in 1..3; at most 128 per (order, precision, restart) batch.
 * The algorithm per solve is that of bsw_solve. */
typedef struct bsw_server_s* bsw_server;

enum { BSW_REQ_QUEUED = 0, BSW_REQ_RUNNING = 1, BSW_REQ_DONE = 2, BSW_REQ_FAILED = 3, BSW_REQ_CANCELLED = 4 };

/* One solve.  All pointers are HOST memory and are copied by
 * bsw_solve_submit, so the caller may free them on return.  Mesh as for
 * bsw_mesh_upload (dim = 2): xy[2 n_vert], el2vert[3 n_el].  W0 (optional)
 * is an initial state of n_f n_p n_el reals of the request's precision in the
 * SoA layout; when NULL the initial condition ic is projected.  bed (kind
 * BSW_BED_FLAT when zero-initialised) is interpolated as by bsw_bed_interpolate
 * into memory of the request and set before ic is projected; so are the
 * orders m1, m2, m3 when mixed_orders is nonzero. */
typedef struct {
  int64_t n_vert;
  const double* xy;
  int64_t n_el;
  const int32_t* el2vert;
  int32_t P;
  int32_t precision;
  bsw_params params;
  bsw_ic ic;
  const void* W0;
  bsw_solve_opts opts;
  bsw_bed bed;
  int32_t mixed_orders;    /* nonzero: the orders below apply (bsw_disc_set_orders) */
  int32_t m1, m2, m3;
  const int8_t* face_bc;   /* optional per-face boundary codes (bsw_mesh_set_boundary) */
} bsw_solve_request;

/* Device bytes a request occupies while resident: state and 11 + gmres_m
 * work vectors, the diagonal Jacobian blocks and their FP32 factors, reduction
 * partials, mesh arrays and the bed coefficients (counted for every request).
 * -1 for an invalid request. */
int64_t bsw_request_footprint(const bsw_solve_request* req);
int bsw_server_create(bsw_ctx ctx, size_t hbm_budget_bytes, int max_slots, bsw_server* out);
/* Stops the worker after its current step; unfinished requests are dropped. */
int bsw_server_destroy(bsw_server server);
/* Validates and copies the request; BSW_E_ARG if it is invalid or its
 * footprint exceeds the whole budget.  *ticket identifies it from then on. */
int bsw_solve_submit(bsw_server server, const bsw_solve_request* req, uint64_t* ticket);
/* *state = one of BSW_REQ_*. */
int bsw_solve_poll(bsw_server server, uint64_t ticket, int* state);
/* Blocks until the request is done, failed or cancelled, or timeout_s passes. */
int bsw_solve_wait(bsw_server server, uint64_t ticket, double timeout_s, int* state);
/* For a finished request: copies the final state to host_W (may be NULL) and
 * the statistics, releases the ticket and returns the solve's status
 * (BSW_OK or BSW_W_NOT_CONVERGED).  A failed or cancelled request returns its
 * error and is released too.  BSW_E_STATE while queued or running. */
int bsw_solve_fetch(bsw_server server, uint64_t ticket, void* host_W, bsw_solve_stats* stats);
/* Queued: dropped before admission.  Running: detached at the next step
 * boundary.  The ticket stays valid until fetched. */
int bsw_solve_cancel(bsw_server server, uint64_t ticket);
/* out8 = {queued, resident, device bytes in use, budget, batched time steps
 * taken, kernel launches, completed requests, peak resident}. */
int bsw_server_info(bsw_server server, double* out8);

#ifdef __cplusplus
}
#endif
#endif /* BSW_H */
