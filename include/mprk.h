/*
 * mprk.h -- C ABI of the MI355X (gfx950) mixed-precision Runge--Kutta library.
 *
 * What it computes.  du/dt = K u for a 3-D finite-difference operator K on the
 * unit cube (the semi-discrete form of Section "Problem setting and solver
 * design" of arXiv 2412.16638), advanced by a diagonally implicit Runge--Kutta
 * method given by a Butcher tableau (eq. RKstep, Table Butchertab) whose matrix is
 * split A = A^(h) + A^(eps) (Section "Method stability in the context of mixed
 * precision").  Each implicit stage is the linear system
 *     (I - tau a_ii K) y_i = rhs_i,   rhs_i = u_n + tau sum_{j<i} (a^h_ij k_j + a^eps_ij k^eps_j)
 * (eq. corelinear, sign convention y = rhs + sigma K y), solved by a preconditioned
 * Krylov method (CG for SPD heat systems, GMRES for advection) in LOW precision
 * (FP32, or FP16 storage with FP32 arithmetic); the explicit evaluations k_i = K y_i,
 * the stage right-hand sides, the step combination u_{n+1} = u_n + tau sum b_i k_i
 * and an outer residual check stay in FP64 on the GPU (Section "Implementation of
 * the Mixed-precision Runge--Kutta methods": explicit parts and stage vectors in
 * double, implicit solves converted to float).  k^eps_j, the low-precision slope of
 * an implicit stage j, is (y_j - rhs_j)/(tau a_jj).
 *
 * Conventions.
 *   - All device pointers are HIP device addresses on the current device.  The
 *     library never allocates device memory: the state u and one workspace blob
 *     are caller-owned (e.g. torch tensors) and handed over with mprk_bind.
 *   - Vectors are lexicographic, x fastest: x_{ijk} = x[i + nx j + nx ny k]
 *     (the ordering stated with the tensor kernels T_L/T_M/T_R of the paper).
 *   - Every call returns an int32 status: MPRK_OK (0) or a negative error code;
 *     mprk_last_error() returns a thread-local message for the last failure.
 *   - Work is enqueued on the hip stream given at creation.  One handle per
 *     stream; a handle is not thread-safe.
 */
#ifndef MPRK_H
#define MPRK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPRK_MAX_STAGES 8
#define MPRK_MAX_RESTART 32
/* Size of the library's static device scratch (mprk_bind_static): 64 MiB per device. */
#define MPRK_STATIC_SCRATCH_BYTES (64LL << 20)

enum mprk_status {
  MPRK_OK = 0,
  MPRK_EINVAL = -1,        /* invalid argument, shape or tableau */
  MPRK_ENOMEM = -2,        /* host allocation failed or workspace too small */
  MPRK_EDEVICE = -3,       /* a HIP runtime call failed */
  MPRK_ENONFINITE = -4,    /* a residual became Inf/NaN; u is left at the last completed step */
  MPRK_ENOTCONV = -5,      /* a stage missed its tolerance (only with precisions.strict != 0) */
  MPRK_EUNSUPPORTED = -6,  /* valid but not implemented combination */
  MPRK_ESTATE = -7         /* call out of order (e.g. step before bind) */
};

enum { MPRK_BC_DIRICHLET0 = 0, MPRK_BC_PERIODIC = 1 };
enum { MPRK_OP_HEAT = 0, MPRK_OP_ADVDIFF = 1, MPRK_OP_CENTRAL = 2 };
enum { MPRK_FMT_STENCIL = 0, MPRK_FMT_CSR = 1 };
enum { MPRK_FP64 = 0, MPRK_FP32 = 1, MPRK_FP16 = 2 };
enum { MPRK_CG = 0, MPRK_GMRES = 1 };
enum { MPRK_PRECOND_NONE = 0, MPRK_PRECOND_BJ = 1, MPRK_PRECOND_FDM = 2 };
enum { MPRK_GMFORM_AUTO = 0, MPRK_GMFORM_GATHER = 1, MPRK_GMFORM_ZSPLIT = 2, MPRK_GMFORM_FOLDED = 3 };
enum {
  MPRK_START_AUTO = 0, MPRK_START_RHS = 1, MPRK_START_SLOPE = 2, MPRK_START_SLOPE_EVAL = 3,
  MPRK_START_EXTRAP = 4
};
enum { MPRK_STOP_AUTO = 0, MPRK_STOP_OUTER = 1, MPRK_STOP_RTOL = 2 };
enum { MPRK_TAB_SDIRK2 = 0, MPRK_TAB_SDIRK3 = 1, MPRK_TAB_MID = 2,
       MPRK_TAB_4S3PA = 3, MPRK_TAB_4S3PB = 4, MPRK_TAB_4S3PC = 5 };
enum { MPRK_APPLY_K64 = 0,     /* y = K x, FP64 in/out */
       MPRK_APPLY_M_LP = 1,    /* y = (I - sigma_stage K) x in the LP storage type, compute type arithmetic */
       MPRK_APPLY_BJ_LP = 2,   /* y = blockdiag(M)^{-1} x, LP storage type */
       MPRK_APPLY_M64 = 3,     /* y = (I - sigma_stage K) x, FP64 */
       MPRK_APPLY_FDM_LP = 4 }; /* y = P^{-1} x, fast-diagonalisation preconditioner, LP storage type */

/* Grid: nx*ny*nz unknowns on the unit cube.  bc = MPRK_BC_DIRICHLET0: zero
 * Dirichlet, n interior nodes per axis, h = 1/(n+1).  bc = MPRK_BC_PERIODIC:
 * h = 1/n.  (The paper's h = 1/(n-1) counts boundary nodes; Section "Heat equation".) */
typedef struct { int32_t nx, ny, nz, bc; } mprk_grid;

/* Operator K.  kind = MPRK_OP_HEAT: K = diff * Lap_h (7-point, second-order central;
 * Section "Test cases").  kind = MPRK_OP_ADVDIFF: K = diff * Lap_h - sum_d b[d] D_d, D_d the
 * first-order upwind difference (backward for b[d] >= 0, forward for b[d] < 0).
 * kind = MPRK_OP_CENTRAL: the same with D_d the second-order central difference
 * (u_{i+1} - u_{i-1}) / (2h), the discretisation of the paper's advection test (Section
 * "Advection equation"); nonsymmetric, so GMRES only.
 * format: MPRK_FMT_STENCIL (matrix-free) or MPRK_FMT_CSR (int32 row pointers and
 * column indices; FP64 values for the explicit parts, LP values for the solve). */
typedef struct { int32_t kind, format; double diff; double b[3]; } mprk_operator;

/* Split Butcher tableau: s stages, s*s row-major lower-triangular a_hi (A^(h)) and a_lo
 * (A^(eps)), weights b (high precision); c is not needed (autonomous f).  Stage i is
 * implicit iff a_hi[i*s+i] + a_lo[i*s+i] != 0. */
typedef struct {
  int32_t s;
  double a_hi[MPRK_MAX_STAGES * MPRK_MAX_STAGES];
  double a_lo[MPRK_MAX_STAGES * MPRK_MAX_STAGES];
  double b[MPRK_MAX_STAGES];
} mprk_tableau;

/* Solver precisions and parameters of the implicit stage solves.
 *  storage: MPRK_FP64 | MPRK_FP32 | MPRK_FP16 -- storage of Krylov vectors, LP matrix values
 *           and block-Jacobi inverses.  compute: MPRK_FP32 (with FP32 / FP16 storage) |
 *           MPRK_FP64: with FP64 storage the all-FP64 solve; with FP32 / FP16 storage the
 *           compressed-basis variant (every Krylov vector, the GMRES basis and the LP operator
 *           values stored in the low precision, all arithmetic in FP64; the Ginkgo-style
 *           alternative cited in the Introduction).
 *  krylov: MPRK_CG (SPD only) | MPRK_GMRES (right preconditioned, restart = cycle length m).
 *  precond: MPRK_PRECOND_NONE | MPRK_PRECOND_BJ with block in {1,2,4,8}: consecutive blocks of
 *           `block` rows in lexicographic order, inverses computed in FP64 per block |
 *           MPRK_PRECOND_FDM: the fast-diagonalisation preconditioner of eqs. preconbasic and
 *           Pinvform (Section "Problem setting and solver design"), P = I (x) I (x) A +
 *           I (x) B (x) I + C (x) I (x) I with A = I - sigma Kx, B = -sigma Ky, C = -sigma Kz, its
 *           inverse applied through the one-axis contractions of eq. TensorDecomp in the compute
 *           type.  P is the stage matrix itself for the operators implemented: the heat
 *           operator (zero Dirichlet or periodic ends; real orthogonal bases) and the advection
 *           operators with periodic ends (circulant factors; the complex unitary DFT basis), with
 *           CG or GMRES (the preconditioner applied by separate launches).  With the DFT
 *           basis only the x frequencies 0 .. nx/2 (rounded up to 4; all when nx < 4) pass
 *           through the y and z transforms, since the vectors are real and the diagonal factor
 *           conjugate-symmetric.  Advection with Dirichlet ends returns MPRK_EUNSUPPORTED; so
 *           does the batched form.
 *  rtol/atol/maxit: inner Krylov stop ||r|| <= max(rtol ||b||, atol) or maxit iterations per
 *           outer pass (the paper stops on the absolute or the relative residual with at most 40
 *           iterations; Section "Linear solvers and setup of the numerical experiments").
 *  refine_max/outer_tol: the FP64 outer residual loop.  Each pass computes the FP64 residual
 *           res = rhs - (I - sigma K) y, solves the scaled correction system in LP and adds it
 *           to y.  The stage stops when ||res|| <= outer_tol ||rhs|| or after refine_max passes.
 *           inner_stop = MPRK_STOP_OUTER: an inner solve also stops once its residual shows
 *           that the update meets half of outer_tol (rtol stays the bound on its iterations);
 *           MPRK_STOP_RTOL: each pass solves to rtol; MPRK_STOP_AUTO (0): OUTER with LP
 *           storage, RTOL with FP64 storage (whose inner tolerance is the accuracy asked for).
 *           refine_max = 0 is the paper's one-shot mode: exactly one LP solve (for GMRES one
 *           cycle) on the converted right-hand side, no residual check (inner_stop unused).
 *  strict: make a stage that misses its tolerance an error: outer_tol after refine_max passes,
 *           or, with refine_max = 0, the LP solve's own tolerance within maxit.  The step of
 *           that stage is not combined and the call's later steps are skipped, so u is left at
 *           the last step whose stages all met it; mprk_step returns MPRK_ENOTCONV.  Without
 *           strict such stages are counted in mprk_stats.missed and stepping continues (as the
 *           paper's experiments keep stepping after a solve that hit its iteration cap).
 *  reorth: 0 = GMRES orthogonalises each new Arnoldi vector by one classical Gram-Schmidt
 *           pass (CGS1); 1 = by two (CGS2: the once-orthogonalised vector is stored and
 *           orthogonalised again, the Hessenberg column is the sum of both passes'
 *           coefficients; one extra launch per Arnoldi step).  Ignored by CG.
 *  gm_form: kernel form of the GMRES Arnoldi step (same arithmetic, different memory traffic):
 *           MPRK_GMFORM_GATHER = product and update kernels, each stencil point gathered from
 *           memory; MPRK_GMFORM_ZSPLIT = the product on z-marching tiles (whole x-rows of a run
 *           of planes, the plane tile staged in LDS, the z neighbours in registers) and the
 *           update kernel; MPRK_GMFORM_FOLDED = one launch per step on z-marching tiles that
 *           forms the orthogonalised vector of the previous step from the stored product and
 *           applies block-Jacobi and the stencil to it (one read of the basis from memory per
 *           step instead of two; CGS1 and block-Jacobi or no preconditioner only).
 *           MPRK_GMFORM_AUTO (0) = the library's choice for the grid (the autotuner may time
 *           the eligible forms).  The tiled forms need the stencil format and whole groups of
 *           values per x-row (nx a multiple of 8 for FP16 storage, else of 4, and at most 128
 *           groups of them per row);
 *           a form the problem does not allow returns MPRK_EUNSUPPORTED from mprk_create.
 *  bj_adapt_tol: 0 = block-Jacobi inverses stored in the storage type (default); > 0 =
 *           adaptive precision (the Ginkgo preconditioner cited in the Introduction): each
 *           block's inverse may be stored in FP8 (E4M3), FP16, FP32 or FP64, the lowest whose
 *           unit roundoff u satisfies u * cond_1(D_b) <= bj_adapt_tol (for FP8 plus
 *           bs * 2^-10 * ||D_b||_1, its flush of entries below 2^-9) and whose range holds the
 *           inverse's entries; blocks are grouped in chunks of 64 lane groups (the rows one
 *           wave reads) stored in the widest type their blocks need.  The apply computes in the
 *           compute type.  Needs bj_shared = 0; not in the batched form.
 *  bj_shared: 0 = one stored inverse per block-Jacobi block (default); 1 = store each distinct
 *           diagonal block's inverse once plus a per-block index (a single shared inverse when
 *           all blocks coincide, e.g. constant coefficients with block | nx).  Both modes give
 *           bitwise-identical inverses; mode 1 removes the inverse stream from the apply.
 *  stage_start: start value of an implicit stage's solve y_i = rhs_i + sigma k_i (the paper
 *           leaves it open), i.e. a guess of the stage slope k_i: MPRK_START_RHS = none
 *           (y = rhs_i); MPRK_START_SLOPE = the previous stage's slope k_{i-1} for the stages
 *           after the step's first; MPRK_START_SLOPE_EVAL = as SLOPE, and the first implicit
 *           stage from f(u), evaluated in FP64 at the step's start (one more operator
 *           evaluation per step); MPRK_START_EXTRAP = the slopes of the two latest stages
 *           extrapolated linearly in c to c_i (f(u), evaluated at the step's start, taken as the
 *           slope at c = 0; the first stage from rhs).  A step thus depends on u alone, never on
 *           an earlier call.  MPRK_START_AUTO (0) = with the FP64 outer loop: GMRES -> SLOPE
 *           (SLOPE_EVAL under the FDM preconditioner), CG -> EXTRAP (RHS under FDM); RHS in the
 *           one-solve mode (refine_max = 0), whose result depends on the start value.  Every
 *           start value is iterated to the same tolerances; it changes iteration and pass
 *           counts (mprk_launch_info_get reports the one in use). */
typedef struct {
  int32_t storage, compute;
  int32_t krylov, restart;
  int32_t precond, block;
  double rtol, atol;
  int32_t maxit;
  int32_t refine_max;
  double outer_tol;
  int32_t strict;
  int32_t reorth;
  int32_t bj_shared;
  int32_t gm_form;
  double bj_adapt_tol;
  int32_t stage_start;
  int32_t inner_stop;
} mprk_precisions;

/* Statistics.  Per-stage entries describe the most recent step. */
typedef struct {
  int64_t steps;                    /* steps completed on this handle (see mprk_set_state) */
  double t;                         /* simulated time */
  int32_t stages;                   /* s */
  int32_t iters[MPRK_MAX_STAGES];   /* Krylov iterations summed over the outer passes */
  int32_t passes[MPRK_MAX_STAGES];  /* LP solves (outer passes) */
  double resid[MPRK_MAX_STAGES];    /* final FP64 ||res|| / ||rhs|| */
  int32_t converged[MPRK_MAX_STAGES]; /* 1 if resid <= outer_tol; with refine_max = 0, 1 if the
                                         one LP solve stopped on its own tolerance */
  int64_t total_iters;              /* cumulative over all steps */
  int64_t total_passes;
  int32_t nonfinite;                /* 1 if the last step hit a non-finite residual */
  int32_t missed;                   /* stages, over every step since the previous statistics
                                       read (mprk_step or mprk_stats_sync), that finished
                                       without reaching their tolerance: resid > outer_tol
                                       after the last allowed pass, or, with refine_max = 0,
                                       an LP solve stopped by maxit, the GMRES cycle length or
                                       a breakdown */
  int32_t graph_steps;              /* steps of the last mprk_step call replayed from the step
                                       graph (mprk_set_step_graph); 0 when steered */
} mprk_stats;

typedef struct { int32_t iters, passes, converged; double resid; } mprk_solve_info;

typedef struct mprk_handle mprk_handle;

/* Builtin tableaus.  id = MPRK_TAB_SDIRK2 (Alexander, gamma = 1 - 1/sqrt 2), MPRK_TAB_SDIRK3
 * (Alexander, L-stable order 3), MPRK_TAB_MID (implicit midpoint with `param` corrector steps,
 * Figure fig_Aq_rat and Appendix A; param in [0, 7]), MPRK_TAB_4S3PA / 4S3PB / 4S3PC
 * (Tables ButchertabA/B/C; 4s3pB with a42^(eps) = -3/2 - a42, the printed value breaking
 * order 2).  The SDIRKs put the diagonal in A^(eps) and the rest in A^(h).
 * Returns MPRK_EINVAL for an unknown id or param. */
int32_t mprk_tableau_builtin(int32_t id, int32_t param, mprk_tableau *out);

/* Fill *out with the library defaults for a storage precision and Krylov method. */
int32_t mprk_precisions_default(int32_t storage, int32_t krylov, mprk_precisions *out);

/* Validate the problem and create a handle (host memory; with a device present also the
 * handle's pinned status records and events).  dt is the time step tau; hip_stream is a
 * hipStream_t (NULL = the null stream).  FP16 storage needs no range check here: the stencil
 * coefficients stay in the compute type, CSR values are stored scaled by a power of two into
 * [-1, 1], right-hand sides are scaled to unit RMS (the rescaling Section "Method stability in
 * the context of mixed precision" gives as the remedy for FP16's range); a value that still
 * overflows shows up as a non-finite residual (MPRK_ENONFINITE from mprk_step).  Errors:
 * MPRK_EINVAL (bad shape, non-lower-triangular tableau, CG on a nonsymmetric operator, index
 * range beyond int32 for CSR), MPRK_EUNSUPPORTED, MPRK_EDEVICE. */
int32_t mprk_create(const mprk_grid *grid, const mprk_operator *op, const mprk_tableau *tab,
                    const mprk_precisions *prec, double dt, void *hip_stream, mprk_handle **out);

/* Exact number of bytes of device workspace the handle needs (<0 on error): the FP64 stage
 * vectors of eq. RKstep (rhs, y and k_i per stage, k^eps_i for split tableaus), the LP Krylov
 * vectors of the stage solve of eq. corelinear, the preconditioner's data and the reduction
 * and control records.  Serving admission sizes jobs by it. */
int64_t mprk_workspace_bytes(const mprk_handle *h);

/* Attach caller-owned device memory and run the setup on the handle's stream: CSR assembly,
 * block-Jacobi inverses of the stage matrices I - tau a_ii K of eq. corelinear (one set per
 * distinct a_ii, computed in FP64, stored in the LP type), the fast-diagonalisation bases of
 * eq. Pinvform.  u_dev: N doubles, the state, updated in place by
 * mprk_step.  workspace_dev: >= mprk_workspace_bytes bytes, 256-byte aligned.  The
 * library keeps both pointers until mprk_destroy or the next bind; it never frees them.
 * Synchronises the stream before returning.  Errors: MPRK_EINVAL, MPRK_ENOMEM (bytes too
 * small), MPRK_EDEVICE. */
int32_t mprk_bind(mprk_handle *h, double *u_dev, void *workspace_dev, int64_t bytes);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops
 * or harnesses that forbid hipMalloc): mprk_bind with the library's static device scratch as
 * the workspace instead of caller memory.  The caller still owns u_dev (N doubles, 32-byte
 * aligned, the state).  The call allocates no device or pinned host memory and calls no
 * hipMalloc/hipFree; the handle's pinned status records are made by mprk_create when a device
 * is present.  The scratch is one array of MPRK_STATIC_SCRATCH_BYTES per device, held from the
 * library's load on that device until the process ends; it is shared by every handle bound to
 * it on that device and keeps the last bind's contents (the bind re-initialises everything it
 * reads).  Binding another handle to it invalidates the previous one: later calls on that
 * handle return MPRK_ESTATE.  Calls of two handles that overlap in time on one device race.
 * Errors: MPRK_EINVAL, MPRK_ENOMEM (mprk_workspace_bytes > MPRK_STATIC_SCRATCH_BYTES),
 * MPRK_ESTATE (handle created without a device), MPRK_EDEVICE. */
int32_t mprk_bind_static(mprk_handle *h, double *u_dev);

/* Constant forcing: from the next step on, integrate du/dt = K u + g instead of du/dt = K u
 * (the paper's heat test has g = sin(pi x) sin(pi y) sin(pi z), Section "Heat equation").
 * g_dev: N doubles of caller-owned device memory, read by the FP64 explicit parts (k_i =
 * K y_i + g, so the stage systems solve (I - dt a_ii K) y = rhs + dt a_ii g); it must stay
 * valid and unchanged while steps or solves run.  NULL removes the forcing.  mprk_apply is
 * unaffected (it applies the operators alone).  Errors: MPRK_EINVAL (null handle). */
int32_t mprk_set_forcing(mprk_handle *h, const double *g_dev);

/* Step graph (eq. RKstep's time loop, Section "Implementation of the Mixed-precision
 * Runge--Kutta methods"): with enable != 0, mprk_step runs its steps by replaying one captured
 * hipGraph of a whole step on the bound stream, with no host wait between steps, once every
 * implicit stage has a solve history from an earlier steered step (the first call, or the
 * first steps after a change, run steered).  The graph enqueues, per stage, the passes and
 * Krylov iterations the stage's last steered solve needed (each plus the usual margin) and one
 * spare pass; a stage that needs more misses inside the graph, its step is not combined and the
 * call's remaining steps run steered from there (which also records new histories, and the
 * graph is captured again on a later call), so the results are those of steered stepping.
 * Launches are the same kernels; what the graph saves is the host's launch and polling cost,
 * which dominates on small grids.  The graph is captured on a stream the library creates and
 * is rebuilt after mprk_bind, mprk_set_forcing, mprk_set_reaction or mprk_autotune.  Not used
 * with refine_max = 0 (the one-solve mode steers every chunk) or while profiling is on.
 * enable = 0 releases the graph.  mprk_stats.graph_steps counts the replayed steps.
 * Errors: MPRK_EINVAL (null handle); capture failures surface from mprk_step as MPRK_EDEVICE. */
int32_t mprk_set_step_graph(mprk_handle *h, int32_t enable);

/* Pointwise cubic reaction: from the next step on, integrate the semi-linear
 * du/dt = K u + g + R(u), R(u) = r1 u + r2 u^2 + r3 u^3 applied to each grid value (non-linear
 * equations are the paper's first extension, Section "Summary and conclusions"; an implicit
 * stage then is the non-linear system y - dt a_ii f(y) = rhs of eq. RKstep, Section "Runge--Kutta
 * methods and mixed-precision").  The FP64 parts evaluate f with R (the outer residual and the
 * explicit slopes k_i = K y_i + g + R(y_i)); the LP solves keep the stage matrix I - dt a_ii K
 * and its preconditioner, so the outer defect-correction loop becomes a simplified Newton
 * iteration whose Jacobian is the linear part.  Each pass contracts the stage error by about
 * dt a_ii max|R'(y)| (on a dissipative K), so the stage needs about log(outer_tol) /
 * log(dt a_ii max|R'|) passes: more than the defaults of mprk_precisions_default allow for
 * linear problems (4 with FP64 CG), so raise refine_max with a reaction.  A stage that reaches
 * refine_max counts as not converged (mprk_stats.missed; MPRK_ENOTCONV under strict); with
 * dt a_ii max|R'| near or above 1 the iteration does not converge.  All three zero removes it.
 * mprk_solve and mprk_apply are unaffected (they treat the linear systems alone).
 * Errors: MPRK_EINVAL (null handle, non-finite coefficient), MPRK_EUNSUPPORTED (a non-zero
 * reaction with refine_max = 0: the one-solve mode makes a single linearised solve). */
int32_t mprk_set_reaction(mprk_handle *h, double r1, double r2, double r3);

/* Advance u by nsteps time steps of eq. RKstep: per implicit stage the right-hand side and
 * the FP64 residual, the LP solve of eq. corelinear, the FP64 update and explicit evaluation
 * k_i = K y_i, then u_{n+1} = u_n + tau sum b_i k_i (Section "Implementation of the
 * Mixed-precision Runge--Kutta methods").  The calling thread steers the Krylov loops by polling
 * small device-side status records; all arithmetic runs in the library's kernels on the
 * bound stream.  The call waits for the stream before it returns (it reads the device's step
 * and convergence counters) and fills stats_or_null if given.
 * Errors: MPRK_ESTATE (not bound), MPRK_ENONFINITE (u left at the last good step),
 * MPRK_ENOTCONV (strict only), MPRK_EDEVICE. */
int32_t mprk_step(mprk_handle *h, int32_t nsteps, mprk_stats *stats_or_null);

/* Solve one stage system (I - dt a_ii K) x = rhs of eq. corelinear with the handle's implicit
 * solver
 * (LP Krylov inside the FP64 outer loop), stage in [0, s) with a_ii != 0.  rhs_dev, x_dev:
 * N doubles each (may not alias u or the workspace).  Waits for completion; fills *info
 * if given.  Errors: MPRK_EINVAL (explicit stage), MPRK_ESTATE, MPRK_ENONFINITE, MPRK_EDEVICE. */
int32_t mprk_solve(mprk_handle *h, int32_t stage, const double *rhs_dev, double *x_dev,
                   mprk_solve_info *info);

/* Apply one component operator (kernel-level access for verification):
 * MPRK_APPLY_K64 / MPRK_APPLY_M64: x, y are N doubles; MPRK_APPLY_M_LP / MPRK_APPLY_BJ_LP /
 * MPRK_APPLY_FDM_LP: x, y are N values of the LP storage type (FP16 = IEEE binary16); BJ_LP
 * needs the block-Jacobi preconditioner and FDM_LP the fast-diagonalisation one (else
 * MPRK_EINVAL).  `stage` selects
 * sigma = dt a_ii (ignored for K64).  Enqueued on the stream; waits before returning. */
int32_t mprk_apply(mprk_handle *h, int32_t op, int32_t stage, const void *x_dev, void *y_dev);

/* Time and step counter (u itself lives in the bound buffer).  mprk_get_state waits for
 * the stream.  mprk_set_state resets the counters, e.g. after the caller restores u from a
 * checkpoint; it does not touch u. */
int32_t mprk_get_state(const mprk_handle *h, double *t, int64_t *step);
int32_t mprk_set_state(mprk_handle *h, double t, int64_t step);

/* Wait for the stream and return the statistics of the most recent step. */
int32_t mprk_stats_sync(mprk_handle *h, mprk_stats *out);

/* Autotuner: times candidate launch shapes (groups of unknowns per thread, hence workgroups
 * per launch, for the vector/stencil kernels and, with CSR, rows per thread) on the bound
 * workspace with the handle's own LP SpMV and FP64 operator kernels, keeps the fastest, and
 * caches the choice per (grid, operator, precision, format) for the life of the process.
 * Uses the workspace's Krylov vectors as scratch (state u is not touched).  Waits for the
 * stream.  *nit_vec / *nit_row (may be NULL) receive the chosen groups per thread. */
int32_t mprk_autotune(mprk_handle *h, int32_t *nit_vec, int32_t *nit_row);

/* Launch shapes in use (after mprk_create's defaults or mprk_autotune): groups of values per
 * thread of the streaming / reducing vector kernels (FP64 and LP) and CSR row kernels; planes
 * per z-marching tile of the FP64 residual (0 = gather kernel); the GMRES step form (an
 * MPRK_GMFORM value, 0 for CG) and its planes per tile (0 for the gather form); the storage
 * types of the adaptive block-Jacobi inverses; the stage start value.  Needs no device. */
typedef struct {
  int32_t nit_vec, nit_row, nit_vec_red, nit_row_red, nit_lp, nit_lp_red;
  int32_t residual_planes;
  int32_t gm_form, gm_planes;
  int64_t bj_chunks[4];  /* adaptive-precision block-Jacobi: chunks stored in FP8 (E4M3), FP16,
                            FP32, FP64 (summed over the distinct stage shifts; 0 without it) */
  int32_t stage_start;   /* the stage start value in use: an MPRK_START value other than AUTO */
} mprk_launch_info;
int32_t mprk_launch_info_get(const mprk_handle *h, mprk_launch_info *out);

/* Kernel classes for mprk_profile_read. */
enum { MPRK_KC_STAGE_RHS = 0, MPRK_KC_RESIDUAL, MPRK_KC_CG_BEGIN, MPRK_KC_CG_DIR, MPRK_KC_CG_UPD,
       MPRK_KC_PROMOTE, MPRK_KC_GM_BEGIN, MPRK_KC_GM_PREC, MPRK_KC_GM_MATVEC, MPRK_KC_GM_ORTH,
       MPRK_KC_GM_FINISH, MPRK_KC_KEPS, MPRK_KC_COMBINE, MPRK_KC_APPLY, MPRK_KC_CG_RZ,
       MPRK_KC_FDM, MPRK_KC_GM_REORTH, MPRK_KC_GM_STEP, MPRK_KC_GM_CLOSE, MPRK_KC_COUNT };

/* Per-kernel timing.  enable = 1 waits for the stream, clears the records and starts
 * recording a HIP event immediately before and after every kernel the handle launches (on its
 * stream); enable = 0 stops recording (records are kept for mprk_profile_read). */
int32_t mprk_profile(mprk_handle *h, int32_t enable);

/* Waits for the stream and returns, for kernel class `kclass` since the last mprk_profile(h, 1):
 * launches = kernels launched, worked = launches that did work (the rest returned at once
 * because their solve phase had finished), units = basis vectors touched summed over working
 * launches (GMRES kernels; = worked for the others), total_ms = summed event-to-event time. */
int32_t mprk_profile_read(mprk_handle *h, int32_t kclass, int64_t *launches, int64_t *worked,
                          int64_t *units, double *total_ms);

/* Thread-local description of the last error ("" if none). */
const char *mprk_last_error(void);

/* Release host resources.  Caller-owned device memory is untouched. */
void mprk_destroy(mprk_handle *h);

/* ---------------------------------------------------------------------------------------
 * Batched form: many independent problems (own grid, operator coefficients and dt; shared
 * tableau and precisions; stencil format; CG) advanced together.  Each stage is one
 * persistent kernel launch in which every problem owns a group of workgroups with its own
 * group barrier and reductions; a step is captured once as a hipGraph and replayed.
 * --------------------------------------------------------------------------------------- */
typedef struct { mprk_grid grid; mprk_operator op; double dt; } mprk_problem;
typedef struct mprk_batch mprk_batch;

/* Create a batch of `count` problems (count >= 1).  Errors as mprk_create; MPRK_EUNSUPPORTED
 * for GMRES, CSR or FP16/FP32 compute combinations the batched kernel does not implement.
 * stage_start as for one problem; AUTO = EXTRAP with the outer loop, RHS in the one-solve
 * mode. */
int32_t mprk_batch_create(int32_t count, const mprk_problem *problems, const mprk_tableau *tab,
                          const mprk_precisions *prec, void *hip_stream, mprk_batch **out);
/* CTA-group schedule: workgroups per problem.  By default they are planned in proportion to an
 * estimate of each problem's work (unknowns x sqrt of the stage matrix's condition number),
 * at least one each, within the device's co-resident capacity.  set_schedule (before sizing or
 * binding; NULL restores the plan) fixes them; get_schedule returns the plan in use. */
int32_t mprk_batch_set_schedule(mprk_batch *b, const int32_t *wg_per_problem);
int32_t mprk_batch_get_schedule(mprk_batch *b, int32_t *wg_per_problem);
/* Autotune a bound batch by replaying one step from the current states per candidate: first
 * the rows a thread handles together in the CG phases (1, 2 or 4: loads in flight vs
 * registers, hence co-resident workgroups), then the planned schedule's work model, unknowns x
 * (condition-number estimate)^e for e in {0, 1/4, 1/2, 3/4, 1}, and, when a step has run, the
 * measured work of the last step (unknowns x (CG iterations + 1.6 x outer passes) per problem).
 * The fastest choice is kept and written to *exponent_out (-1 for the measured model) /
 * *rows_out (either may be NULL).  States and statistics are restored; the call synchronises
 * the stream.  MPRK_ESTATE if unbound or if set_schedule fixed the schedule. */
int32_t mprk_batch_autotune(mprk_batch *b, double *exponent_out, int32_t *rows_out);
int64_t mprk_batch_workspace_bytes(const mprk_batch *b);
/* u_dev: array of `count` device pointers (problem p's state, N_p doubles each). */
int32_t mprk_batch_bind(mprk_batch *b, double *const *u_dev, void *workspace_dev, int64_t bytes);
/* Advance every problem by nsteps steps (graph replays); asynchronous on the stream. */
int32_t mprk_batch_step(mprk_batch *b, int32_t nsteps);
/* Wait and return problem idx's statistics of its most recent step. */
int32_t mprk_batch_stats_sync(mprk_batch *b, int32_t idx, mprk_stats *out);
void mprk_batch_destroy(mprk_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* MPRK_H */
