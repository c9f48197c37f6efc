/*
 * vts.h -- C ABI of libvts: the PBM method with multigrid-preconditioned
 * MINRES for the 3D variable thickness sheet (VTS) problem on one MI355X
 * (gfx950) GPU.
 *
 * Method: A. Brune, M. Kocvara, "On barrier and modified barrier multigrid
 * methods for 3d topology optimization" (arXiv 1904.06556).
 *   problem (1.1)        min 1/2 f^T u  s.t.  K(rho) u = f, sum rho = V,
 *                        rho_lo <= rho <= rho_hi,  K(rho) = sum_i rho_i K_i
 *   problem (2.1)        its dual, to which PBM is applied
 *   eq. (3.9)            augmented Lagrangian; eq. (3.10) its gradient
 *   eq. (3.12)-(3.14)    Schur complement S, reduced Newton system, Delta nu
 *   Algorithm 1 / 2      PBM outer loop / PBM Newton method
 *   Section 6            V-cycle multigrid preconditioned MINRES
 *
 * Conventions (apply to every entry point):
 *   - Grid: nx x ny x nz unit cubes of side h (finest level); nodes
 *     (nx+1)(ny+1)(nz+1) numbered i + (nx+1)(j + (ny+1)k), x fastest;
 *     displacement DOF c of node p is 3p + c ("all-DOF layout", length
 *     n_dof = 3 * nodes).  Elements numbered i + nx(j + ny k).
 *   - Fixed (Dirichlet) DOFs are held at zero; every vector this library
 *     writes is zero there and every vector it reads is masked on read.
 *   - "S-vector": length n_dof + 1, the all-DOF displacement part followed
 *     by the scalar alpha (the extra unknown of eq. (3.13)).
 *   - Pointers named *_dev are device pointers on the device that was
 *     current at vts_create; *_host are host pointers.  The caller owns
 *     every buffer it passes; no pointer is retained after a call returns.
 *   - All device work is issued on the stream given to vts_create, in
 *     stream order.  Calls that return host statistics synchronize it.
 *   - No call throws; failures return a vts_status and vts_last_error()
 *     gives a message.  A context is not thread-safe.
 */
#ifndef VTS_H
#define VTS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vts_ctx vts_ctx;

typedef enum {
    VTS_OK = 0,
    VTS_EINVAL = 1,       /* invalid argument or problem data (e.g. not strictly feasible) */
    VTS_ENOMEM = 2,       /* device allocation failed */
    VTS_EDEVICE = 3,      /* a HIP runtime call failed */
    VTS_ESTATE = 4,       /* call out of order (e.g. apply_S before newton_setup) */
    VTS_ENOTCONV = 5,     /* iteration limit reached, or the final Newton stalled */
    VTS_ENONDESCENT = 6,  /* Newton direction not a descent direction / line search stalled */
    VTS_ENONSPD = 7       /* preconditioner or coarse matrix not positive definite */
} vts_status;

typedef enum {
    VTS_FP64 = 0,         /* everything in FP64 */
    VTS_MIXED = 1         /* multigrid preconditioner in FP32, everything else FP64 */
} vts_precision;

/* Problem (1.1) on a structured grid.  Section 7: the design domain is a
 * coarse box refined levels-1 times, so nx, ny, nz must be divisible by
 * 2^(levels-1).  All pointers are host pointers, copied by vts_create.
 * rho_lo/rho_hi may be NULL, in which case the scalars are used for every
 * element.  Requirements (the assumptions after (1.1)): rho_hi > rho_lo,
 * sum rho_lo < V < sum rho_hi, at least one fixed DOF, and fixed DOFs
 * nested across levels (a fixed fine DOF interpolates from fixed coarse
 * DOFs only; holds for clamped faces and fixed corner nodes).  Violations
 * give VTS_EINVAL.
 *
 * Several load cases (nload = k in 2..4): the density minimises the sum of
 * the compliances 1/2 f_l^T u_l of the cases, K(rho) u_l = f_l.  This is
 * problem (1.1) for the stacked displacement U = (u_1, ..., u_k) with the
 * element matrices blockdiag(K_i, ..., K_i), so Sections 2-3 apply as
 * written: e_i sums the cases' element energies, res_1 and the Newton
 * system (3.12) take U, and the multigrid of Section 6 works on node blocks
 * of 3k unknowns (the rank-one element terms of (3.12) couple the cases).
 * f_host then holds k n_dof entries, case after case; every vector of the
 * context that has a displacement part (u, res_1, the Newton-system vectors
 * of vts_apply_S, vts_precondition, VTS_VEC_U, _RHS, _DY, _G1, the
 * checkpoint) holds k n_dof entries (case after case) before alpha.
 * Needs precision VTS_FP64.  vts_apply_K and vts_apply_K_rho apply K(rho)
 * to k vectors at once; the FP32 operators, the allocation-free S-apply,
 * DOC, the interior point method, server pools and group steps take one
 * load case only (VTS_EINVAL). */
typedef struct {
    int32_t nx, ny, nz, levels;
    double E, nu, h;
    const uint8_t* fixed_host;    /* n_dof entries, 1 = fixed */
    const double* f_host;         /* max(nload, 1) n_dof entries: the load case(s) */
    double V;
    const double* rho_lo_host;    /* m entries or NULL */
    const double* rho_hi_host;    /* m entries or NULL */
    double rho_lo_s, rho_hi_s;
    int32_t precision;            /* vts_precision */
    int32_t nload;                /* load cases; 0 or 1: one load */
} vts_problem;

/* Parameters of Algorithms 1 and 2 and of the MINRES rule of Section 6.2.
 * vts_default_options() fills the values used by this library: the paper's
 * beta = gamma = 0.3, eps_NWT = 1 and eps_MR rule; tighter eps_PBM = 1e-8,
 * eps_NWT_min = 1e-5, final eps_NWT = 5e-7 and a stationarity test so that
 * results meet a KKT residual of 1e-6; and floors of the penalties that are
 * relative to the problem's energy scale (p_min_relative = 1): p >= p_min
 * |alpha| with p_min = 1e-3 for the energy constraints and q >= q_min |alpha|
 * with the paper's q_min = 1e-8 for nu >= 0 (the volume multiplier alpha
 * equals the common element energy at the optimum).  The constraint values
 * scale with the square of the load, so the paper's absolute floors tie the
 * method's behaviour to that scale; the Schur weights grow like rho/p, and a
 * moderate relative p floor keeps the Newton systems within reach of the
 * Gauss-Seidel multigrid.  PBM converges for any positive floors. */
typedef struct {
    double beta, gamma, p_min, q_min;
    double eps_pbm, eps_nwt0, eps_nwt_min, eps_nwt_final;
    double eps_stat;              /* <= 0: outer loop stops on the gap test alone */
    double accept_stall;          /* final-Newton stall accepted if res_PBM below this */
    double eps_mr0;               /* <= 0: 1e-4 sqrt(n) (Section 6.2) */
    double eps_mr_min;            /* floor of the MINRES tolerance (1e-9) */
    double armijo_c1, armijo_min; /* Armijo constant and smallest step */
    int32_t max_outer, max_newton, max_minres;
    int32_t final_res4;           /* final Newton also requires the res_4 term */
    int32_t p_min_relative;       /* 1: floors p_min |alpha|, q_min |alpha|; 0: p_min, q_min */
    int32_t stall_steps;          /* a Newton call stops after this many steps without a new best
                                     criterion below 0.9 x the best (0: never).  A call before
                                     the final one that stalls is taken as the minimizer and the
                                     outer loop goes on; a stalled final call goes to the KKT
                                     check (kkt_tol) or the accept_stall rule (the paper accepts
                                     stalled near-optimal points, Section 7.2).  Also ends the outer loop
                                     once the gap test holds and the stationarity term, below
                                     10 x eps_stat, has gone this many outer iterations without a
                                     new value below 0.9 x its best; the final Newton call and
                                     kkt_tol then decide */
    int32_t use_graphs;           /* 1: replay each V-cycle from a captured HIP graph (the
                                     same kernels and arguments, bitwise equal results;
                                     recaptured after every multigrid setup; contexts built
                                     inside a server pool never do, so serving allocates
                                     nothing).  Default 0: measured no faster on MI355X,
                                     the V-cycle waits on dependent-kernel latency on the
                                     device, not on host launch cost */
    double kkt_tol;               /* > 0: vts_pbm_solve succeeds (VTS_OK) iff the KKT residual of
                                     the returned (rho, u, alpha) is at most this, whatever the
                                     final Newton call's own test gave; a final Newton that
                                     stalled (VTS_ENOTCONV, VTS_ENONDESCENT) then goes on to the
                                     rho update and state solve.  A check above kkt_tol (the
                                     final Newton call can move the stationarity term past it)
                                     resumes the outer loop from the returned state with half
                                     the stationarity target, at most 3 times and within
                                     max_outer (a "resume" line in the log).  <= 0: the
                                     accept_stall rule decides.  Default 1e-6 */
    double eps_state;             /* > 0: after the last update of rho, vts_pbm_solve solves the
                                     state equation K(rho) u = f for the returned rho (MINRES
                                     with one V-cycle of blockdiag(K(rho), 1), stopping at this
                                     relative residual in the preconditioner norm), so that the
                                     returned u is the state of the returned density; <= 0: u is
                                     the last Newton iterate.  Skipped when some lower bound
                                     rho_lo is 0: K(rho) may then be singular on a void region,
                                     where the state equation leaves u free, and the last Newton
                                     iterate (the dual solution of problem (2.2)) is the
                                     displacement that meets the optimality conditions.
                                     Default 1e-10 */
    const char* log_path;         /* NULL (default): no log.  Otherwise a file to which the
                                     context appends one JSON object per line: every Newton
                                     step of Algorithm 2 ("newton": outer index, step, res_PBM,
                                     res_4, Armijo step, slope, MINRES tolerance and count),
                                     every outer iteration of Algorithm 1 ("outer": gap ratio,
                                     stationarity, eps_NWT, sum of rho, Newton and MINRES
                                     counts, stop) and every vts_pbm_solve result ("result").
                                     The string is copied at vts_create; the file is opened on
                                     the first line and closed by vts_destroy.  A file that
                                     cannot be opened disables the log (the solve goes on). */
} vts_options;

typedef struct {
    int32_t iterations;
    double rel_residual;          /* phi_bar / beta_1 of preconditioned MINRES */
} vts_linstats;

typedef struct {
    double res_pbm;               /* eq. (3.15) at the new point */
    double res4;                  /* ||res_4|| / (||rho_lo|| + ||rho_hi||) */
    double kappa;                 /* accepted Armijo step */
    double slope;                 /* grad L^T Delta xi */
    double eps_mr;                /* MINRES tolerance used */
    int32_t minres_its;
} vts_newtonstats;

typedef struct {
    double gap, dual, ratio;      /* delta (2.6), dual objective of (2.1), |delta/d| */
    double stat;                  /* stationarity estimate of the candidate rho */
    double eps_nwt, sum_rho;
    int32_t newton_its, minres_its;
    int32_t converged;            /* 1 when Algorithm 1's stopping test holds */
} vts_pbmstats;

typedef struct {
    double compliance;            /* 1/2 f^T u at the returned state */
    double alpha, sum_rho;
    double res_pbm;
    int32_t outer, newton, minres;
    int32_t status;               /* vts_status of the run */
    /* KKT residual of the returned (rho, u) with multiplier lambda = alpha
     * (conditions of problem (1.1)): r_eq = ||K(rho)u - f|| / ||f||,
     * r_vol = |sum rho - V| / V, r_box = max bound violation / max rho_hi,
     * r_stat = max_i |rho_i - clip(rho_i + (e_i - lambda)/lambda)| / rho_hi_i;
     * kkt = the largest of the four (all 0 if the run ended before them) */
    double kkt, r_eq, r_vol, r_box, r_stat;
} vts_result;

/* Which internal vector vts_get_vector copies (device to device). */
typedef enum {
    VTS_VEC_U = 0,        /* displacement u, n_dof */
    VTS_VEC_RHO = 1,      /* element multipliers rho (densities), m */
    VTS_VEC_ENERGY = 2,   /* e_i = 1/2 u^T K_i u at the current state, m */
    VTS_VEC_RHS = 3,      /* reduced right-hand side of eq. (3.13), S-vector */
    VTS_VEC_DY = 4,       /* last Newton direction (Delta u, Delta alpha), S-vector */
    VTS_VEC_G1 = 5,       /* res_1 = K(rho')u - f, n_dof */
    VTS_VEC_DNU_LO = 6,   /* last Delta nu_lo, m */
    VTS_VEC_DNU_HI = 7,   /* last Delta nu_hi, m */
    VTS_VEC_RHO1 = 8,     /* rho' = rho phi'(s), m */
    VTS_VEC_W = 9         /* Schur weight w = (1/rho'' + 1/mu_lo'' + 1/mu_hi'')^-1, m */
} vts_vector;

/* Fills *opt with this library's defaults. */
void vts_default_options(vts_options* opt);

/* Creates a context holding all device state of one problem: the problem
 * data, the PBM state initialized as stated after Algorithm 1 (u = 0,
 * alpha = 1, nu = e, rho = V/m, mu = e, p = q = e), and the multigrid
 * hierarchy storage.  stream: a hipStream_t (NULL = default stream).
 * opt may be NULL (defaults).  On failure *out is NULL. */
vts_status vts_create(const vts_problem* pr, const vts_options* opt, void* stream,
                      vts_ctx** out);
void vts_destroy(vts_ctx* ctx);

/* Re-initializes the PBM state on the device to the initial point stated
 * after Algorithm 1 (as vts_create does) and resets the counters and
 * tolerances; the problem data stay resident. */
vts_status vts_reset(vts_ctx* ctx);

/* Device bytes vts_create would allocate for this problem (for admission):
 * an upper bound of vts_allocated_bytes, counted in 256-byte granules.
 * Returns 0 for an invalid problem and for a problem with several load
 * cases (those are not admitted to server pools; vts_allocated_bytes gives
 * a created context's size). */
size_t vts_footprint_bytes(const vts_problem* pr, const vts_options* opt);

/* Device bytes this context holds (256-byte granules). */
size_t vts_allocated_bytes(const vts_ctx* ctx);

/* Sizes of this context: n_dof, m, number of free DOFs n, levels. */
vts_status vts_sizes(const vts_ctx* ctx, int64_t* n_dof, int64_t* m, int64_t* n_free,
                     int32_t* levels);

/* Sets the element multipliers rho (= densities), m FP64 values on device. */
vts_status vts_set_rho(vts_ctx* ctx, const double* rho_dev);

/* y = K(rho) x with the current rho, problem (1.1): K(rho) = sum rho_i K_i,
 * K_i the Q1 element stiffness of Section 6.2 scattered to element i's DOFs.
 * x_dev, y_dev: n_dof FP64 (all-DOF layout); fixed DOFs masked on read and
 * written as 0.  x and y must not overlap. */
vts_status vts_apply_K(vts_ctx* ctx, const double* x_dev, double* y_dev);

/* The same operator in FP32 (the precision of the mixed-mode multigrid):
 * x_dev, y_dev n_dof floats; rho taken from the FP64 rho rounded to FP32. */
vts_status vts_apply_K_f32(vts_ctx* ctx, const float* x_dev, float* y_dev);

/* y = K(rho) x for a caller-supplied rho (problem (1.1)), leaving the
 * context's own rho untouched: rho_dev m FP64 values on the device, x_dev,
 * y_dev as for vts_apply_K (fixed DOFs masked on read, written as 0; x and y
 * must not overlap).  The _f32 form takes FP32 rho, x and y.  Reads x and
 * rho once and writes y once (the operator's compulsory traffic). */
vts_status vts_apply_K_rho(vts_ctx* ctx, const double* rho_dev, const double* x_dev,
                           double* y_dev);
vts_status vts_apply_K_rho_f32(vts_ctx* ctx, const float* rho_dev, const float* x_dev,
                               float* y_dev);

/* e_i = 1/2 u_e^T K_e u_e for all elements (the constraint of (2.1)).
 * u_dev: n_dof FP64; e_dev: m FP64. */
vts_status vts_element_energy(vts_ctx* ctx, const double* u_dev, double* e_dev);

/* Algorithm 2, step "compute matrix S and the right-hand side" at the
 * current state: element energies, the weights rho', rho'', mu', mu'' of
 * Section 3.2, the gradient (3.10) (res_3 with constant -rho_lo), the
 * reduced right-hand side of (3.13) and the multigrid hierarchy of S
 * (Galerkin coarse operators, Section 6.1). */
vts_status vts_newton_setup(vts_ctx* ctx);

/* y = S [x; beta] with S of eq. (3.12) at the state of the last
 * vts_newton_setup:  y_u = K(rho')x + sum_i w_i b_i (b_i^T x - beta),
 * y_alpha = -sum_i w_i (b_i^T x - beta), b_i = K_i u.  x_dev, y_dev:
 * S-vectors (FP64).  VTS_ESTATE before the first vts_newton_setup. */
vts_status vts_apply_S(vts_ctx* ctx, const double* x_dev, double* y_dev);

/* For callers that cannot allocate device memory at call time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same y = S [x; beta] as vts_apply_S, with its per-workgroup partial
 * sums of the alpha row kept in a static workspace of the library (65536
 * doubles per device, held until the process ends) instead of the context's
 * buffer.  Calls no hipMalloc, hipFree or allocating library routine.
 * Every partial sum is written before it is read, so nothing in the
 * workspace needs clearing; all calls on one device share the workspace, so
 * calls that overlap on one device (different streams or threads) race.
 * VTS_EINVAL if the grid needs more than 65536 partial sums (about 9e7
 * nodes) or the element is not the cube; VTS_ESTATE before the first
 * vts_newton_setup; VTS_EDEVICE if the workspace address cannot be found. */
vts_status vts_apply_S_noalloc(vts_ctx* ctx, const double* x_dev, double* y_dev);

/* z = M^{-1} r: one V-cycle (Section 6.1) on the hierarchy of the last
 * vts_newton_setup, in FP64 or FP32 per the problem's precision.
 * r_dev, z_dev: S-vectors (FP64); may not overlap. */
vts_status vts_precondition(vts_ctx* ctx, const double* r_dev, double* z_dev);

/* Solves S dy = rhs (3.13) by MINRES preconditioned with one V-cycle,
 * stopping when phi_bar <= eps_mr * beta_1 (eq. (6.2) in the
 * preconditioner norm) or after max_minres iterations.  The direction is
 * kept in the context (VTS_VEC_DY).  stats may be NULL. */
vts_status vts_solve_newton(vts_ctx* ctx, double eps_mr, vts_linstats* stats);

/* One iteration of Algorithm 2: setup (if not current), MINRES solve with
 * the context's eps_MR, Delta nu (3.14), Armijo backtracking on (3.9),
 * update of (u, alpha, nu), res_PBM (3.15) and the eps_MR rule of
 * Section 6.2.  Returns VTS_ENONDESCENT if no descent step was found. */
vts_status vts_newton_step(vts_ctx* ctx, vts_newtonstats* stats);

/* Runs Algorithm 2 to tolerance eps_nwt. */
vts_status vts_newton(vts_ctx* ctx, double eps_nwt, int32_t final_call,
                      vts_newtonstats* last);

/* One pass of the body of Algorithm 1: Newton to the current eps_NWT, the
 * gap (2.6) and dual objective, the stopping test; if not converged the
 * multiplier update with the beta safeguard, the penalty update and the
 * eps_NWT update. */
vts_status vts_pbm_iterate(vts_ctx* ctx, vts_pbmstats* stats);

/* Algorithm 1 to convergence, followed by the final Newton call, the last
 * update of rho, (eps_state > 0) the state solve K(rho) u = f for that rho
 * and the KKT residual of the result.  With kkt_tol > 0 the status is
 * VTS_OK iff that residual is at most kkt_tol (VTS_ENOTCONV otherwise);
 * with kkt_tol <= 0 a final Newton that stalls (VTS_ENOTCONV,
 * VTS_ENONDESCENT) with res_PBM below accept_stall is accepted.  Device,
 * argument and definiteness errors are always returned. */
vts_status vts_pbm_solve(vts_ctx* ctx, vts_result* result);

/* Copies an internal vector (see vts_vector) to dst_dev (device). */
vts_status vts_get_vector(const vts_ctx* ctx, int32_t which, double* dst_dev);

/* Kernel classes that vts_profile_start can time. */
typedef enum {
    VTS_PROF_NONE = 0,
    VTS_PROF_GS_FINE = 1,   /* Gauss-Seidel colour pass on the finest level */
    VTS_PROF_APPLY_K = 2,   /* K(rho) x (vts_apply_K) */
    VTS_PROF_APPLY_S = 3    /* S-apply (MINRES and vts_apply_S) */
} vts_prof_kernel;

/* Starts timing every launch of one kernel class with HIP events recorded
 * on the context's stream (a measurement aid).  Consecutive launches of the
 * class (the 8 colour passes of one Gauss-Seidel sweep) share one event
 * pair; single launches (K(rho)x, S-apply) get one pair each, which adds
 * the event overhead to their times.  Any previous profile is discarded. */
vts_status vts_profile_start(vts_ctx* ctx, int32_t kernel_class);

/* Stops profiling, synchronizes the stream and returns the summed kernel
 * time in ms, the number of kernel launches timed and their summed algorithmic
 * bytes (the compulsory traffic of each launch, as documented in the
 * kernels).  Any output pointer may be NULL. */
vts_status vts_profile_stop(vts_ctx* ctx, double* total_ms, int64_t* launches,
                            double* bytes);

/* Checkpoint of the PBM state to host memory, layout (FP64):
 *   header {5657683 (magic), 2 (layout version), n_dof, m},
 *   u[n_dof], alpha, nu_lo[m], nu_hi[m], rho[m], mu_lo[m], mu_hi[m],
 *   p[m], q_lo[m], q_hi[m], eps_nwt, eps_mr,
 *   outer iterations, Newton steps, MINRES iterations (the run's counters,
 *   so that a resumed run keeps its budgets and totals)
 * *bytes: in = capacity of host_buf (or 0 to query), out = size needed.
 * vts_set_state gives VTS_EINVAL for a wrong size, a header that does not
 * match the context, or counters that are not non-negative integers. */
vts_status vts_get_state(const vts_ctx* ctx, void* host_buf, size_t* bytes);
vts_status vts_set_state(vts_ctx* ctx, const void* host_buf, size_t bytes);

/* Message of the last failure on this context (static storage of ctx). */
const char* vts_last_error(const vts_ctx* ctx);

/* ---------------------------------------------------------------------
 * Damped optimality criteria (Section 5, Algorithm 4), the paper's
 * comparison method, on the same device data: the state equation
 * K(rho) u = f is solved by the same MINRES with one multigrid V-cycle
 * (the Schur operator with rho' = rho, no rank-one terms and a decoupled
 * alpha), followed by the bisection on alpha of Algorithm 4.  It overwrites
 * the PBM working data of the context (u, the operator, the hierarchy).
 * --------------------------------------------------------------------- */
typedef struct {
    double change;                /* ||rho+ - rho||_inf */
    double alpha;                 /* bisection midpoint defining rho+ */
    double compliance;            /* 1/2 f^T u at the iteration's rho */
    double volume;                /* sum rho+ */
    int32_t bisection_steps, minres_its;
    int32_t converged;            /* change <= eps_doc: rho kept, as Algorithm 4 stops */
    int32_t iterations;           /* DOC iterations taken (vts_doc_solve) */
} vts_docstats;

/* One iteration of Algorithm 4 at the context's rho with exponent q,
 * bisection tolerance tau (the paper: 0.1 eps_doc, bracket [0, 10000]) and
 * MINRES tolerance eps_mr.  If eps_doc > 0 and ||rho+ - rho||_inf <= eps_doc
 * the iteration reports convergence and keeps rho; otherwise rho becomes
 * rho+.  VTS_EINVAL for q <= 0 or tau <= 0. */
vts_status vts_doc_step(vts_ctx* ctx, double q, double tau, double eps_doc, double eps_mr,
                        vts_docstats* out);

/* Algorithm 4 from the context's rho until convergence (tau = 0.1 eps_doc)
 * or max_iter iterations (VTS_ENOTCONV). */
vts_status vts_doc_solve(vts_ctx* ctx, double q, double eps_doc, double eps_mr, int32_t max_iter,
                         vts_docstats* out);

/* ---------------------------------------------------------------------
 * Primal-dual interior point method (Section 4, Algorithm 3), the paper's
 * second comparison method, on the same device data.  Variables
 * (u, alpha, rho, nu_lo, nu_hi) live in the context's state vectors (it
 * overwrites the PBM state and working data); each iteration solves the
 * reduced system (eq. S_IP) by the same MINRES with one V-cycle: S_IP has
 * the structure of the PBM Schur operator with rho' = rho and the weights
 * W = ((rho - rho_lo)^-1 nu_lo + (rho_hi - rho)^-1 nu_hi)^-1.
 * Readings: the residual's nu_hi term belongs to res_5; the reduced
 * right-hand side and the increments are those of the Newton step of the
 * residual with the Jacobian (eq. gradres); in eq. (Delta_onu) the term
 * (N_lo - N_hi) rho is (N_lo - N_hi) Delta rho; alpha tends to minus the
 * volume multiplier, so the gap (2.6) is evaluated at (u, -alpha); the
 * multiplier step lengths are capped at 1; MINRES stops, keeping its
 * iterate, if the V-cycle loses definiteness in floating point.  Use FP64
 * contexts: with VTS_MIXED the FP32 V-cycle cannot resolve the late,
 * ill-conditioned IP systems (the 8x4x4 cantilever does not meet the
 * stopping test in 300 iterations).
 * --------------------------------------------------------------------- */
typedef struct {
    double eps_ip;                /* stopping tolerance (paper: 1e-5) */
    double sigma_r, sigma_s;      /* barrier reduction factors (0.2) */
    double r0, s0;                /* initial barrier parameters (1e-2) */
    double step_frac;             /* fraction of the step to the boundary (0.9) */
    double eps_mr0, eps_mr_min;   /* MINRES tolerance rule of Section 6.2 (1e-2, 1e-9) */
    int32_t max_iter;             /* iterations of Algorithm 3 (300) */
    int32_t max_minres;           /* MINRES iterations per system (3000) */
} vts_ip_options;

typedef struct {
    double gap_ratio;             /* delta(u, -alpha) / (1/2 f^T u) after the step */
    double res_ip;                /* feasibility measure eq. (ip_res) after the step */
    double compliance;            /* 1/2 f^T u after the step */
    double alpha;                 /* after the step (tends to minus the multiplier) */
    double r, s;                  /* barrier parameters of this iteration's system */
    double kappa_u, kappa_nu_lo, kappa_nu_hi;  /* step lengths taken */
    double eps_mr;                /* MINRES tolerance of this iteration's solve */
    int32_t minres_its;           /* this iteration (vts_ip_solve: all iterations) */
    int32_t converged;            /* the stopping test of Algorithm 3 holds */
    int32_t iterations;           /* iterations taken (vts_ip_solve) */
} vts_ipstats;

void vts_ip_default_options(vts_ip_options* o);

/* Sets the initial point stated before Algorithm 3 (u = 0, alpha = 1,
 * rho = V/m, nu_lo = nu_hi = e), the barrier parameters r0, s0 and their
 * first shifted update, and the MINRES tolerance.  opt NULL: defaults.
 * VTS_EINVAL for options out of range. */
vts_status vts_ip_init(vts_ctx* ctx, const vts_ip_options* opt);

/* One iteration of Algorithm 3 from the context's current point: reduced
 * system, MINRES, increments, barrier shift, step lengths, update, gap,
 * objective and res_IP, the next shifted barrier parameters and the MINRES
 * tolerance rule.  VTS_ESTATE before vts_ip_init; VTS_ENOTCONV if rounding
 * put a variable on its bound (the iterate is kept, the method cannot go on). */
vts_status vts_ip_step(vts_ctx* ctx, vts_ipstats* stats);

/* vts_ip_init followed by vts_ip_step until the stopping test holds
 * (VTS_OK) or max_iter iterations (VTS_ENOTCONV).  stats may be NULL. */
vts_status vts_ip_solve(vts_ctx* ctx, const vts_ip_options* opt, vts_ipstats* stats);

/* Advances each of the k (distinct) contexts by one outer iteration of
 * Algorithm 1 (as vts_pbm_iterate): one host thread per context for the
 * element-wise steps, and the Newton systems' preconditioned MINRES solves
 * (Section 6) of all k advanced together on one stream, step by step: the
 * launches of contexts with the same grid, levels and precision (V-cycle
 * smoother, transfer and coarse kernels, S-apply, vector updates and
 * reductions) go out as one launch per kernel over those contexts, with
 * one synchronization per MINRES step for all.  stats (NULL, or k entries)
 * receives each context's statistics.  Returns VTS_OK, or the status of the
 * first context (in index order) that failed; the others still complete
 * their iteration.  Each context's result is bitwise the same as with
 * vts_pbm_iterate alone (same kernel bodies, blocks and reduction orders). */
vts_status vts_group_step(vts_ctx** ctxs, int32_t k, vts_pbmstats* stats);

/* ---------------------------------------------------------------------
 * Serving: a request loop for streams of independent VTS problems (the
 * problem (1.1) of each request solved by Algorithm 1 to the options'
 * tolerances).  The server owns one device pool of hbm_bytes, allocated
 * once, and `slots` worker threads, each with its own non-blocking HIP
 * stream.  A pending request is admitted, in arrival order with first-fit
 * bypass, as soon as a slot is idle and a contiguous range of the pool
 * holds its vts_footprint_bytes; its context is built inside that range (no
 * hipMalloc or hipFree while serving), solved, and its range returned.
 * Admitted problems run concurrently on the device, each on its own stream.
 * With batching on (the default), the Newton-system MINRES solves of
 * admitted problems with the same grid, levels and precision join a group
 * runner for that shape (one thread and stream each, created on first use
 * with a small staging buffer): the solves in it advance step by step
 * together, and each kernel of a step is one launch over all of them
 * (problem = blockIdx.y), as in vts_group_step; solves join and leave
 * between steps.  Every problem's arithmetic is the same as in a context of
 * its own (same kernel bodies, blocks, fixed reduction orders, no
 * atomics), so results do not depend on the mix.
 * --------------------------------------------------------------------- */
typedef struct vts_server vts_server;

typedef struct {
    int64_t id;
    int32_t status;               /* vts_status of the solve */
    int32_t outer, newton, minres;
    double compliance, alpha, sum_rho;
    double t_submit, t_admit, t_done;   /* seconds on the server's clock */
    size_t footprint;             /* bytes of the pool the request held */
    int64_t n_dof, m;
} vts_request_info;

/* slots >= 1 workers; hbm_bytes of device memory on the current device.
 * VTS_ENOMEM if the pool cannot be allocated. */
vts_status vts_server_create(int32_t slots, size_t hbm_bytes, vts_server** out);

/* Copies the problem (host arrays) and options (NULL: defaults) into the
 * queue and returns its id.  VTS_EINVAL for an invalid problem, VTS_ENOMEM
 * if its footprint exceeds the whole pool.  Thread-safe. */
vts_status vts_server_submit(vts_server* srv, const vts_problem* pr, const vts_options* opt,
                             int64_t* id);

/* Moves up to max finished requests into out[] (oldest first), waiting up to
 * timeout_s seconds for the first one; returns how many were written. */
int32_t vts_server_poll(vts_server* srv, vts_request_info* out, int32_t max, double timeout_s);

/* Copies the final rho (m doubles) and u (n_dof doubles) of a finished
 * request to host memory (either pointer may be NULL) and forgets it.
 * VTS_EINVAL for an unknown id. */
vts_status vts_server_fetch(vts_server* srv, int64_t id, double* rho_host, double* u_host);

/* Seconds since the server was created (the clock of vts_request_info). */
double vts_server_clock(const vts_server* srv);

/* Numbers of requests waiting, running and finished-but-not-polled. */
void vts_server_counts(const vts_server* srv, int32_t* pending, int32_t* running,
                       int32_t* finished);

/* Batching of same-shape MINRES solves across requests: on (1, the
 * default) or off (0: each request's launches go out on its own stream).
 * Only before the first vts_server_submit: VTS_ESTATE afterwards. */
vts_status vts_server_batching(vts_server* srv, int32_t on);

/* Counters of the group runners, summed over shapes: out[0] synchronized
 * MINRES steps, out[1] solves completed, out[2] kernel launches the solves
 * asked for, out[3] launches issued for them (out[2] / out[3] is the mean
 * batch), out[4] the largest batch. */
void vts_server_group_stats(vts_server* srv, int64_t out[5]);

/* Finishes the running requests, drops the pending ones, frees the pool and
 * the group runners. */
void vts_server_destroy(vts_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* VTS_H */
