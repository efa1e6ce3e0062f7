/*
 * fe.h -- C-ABI of the MI355X (gfx950) matrix-free Newton-Krylov state solver
 * for density-based topology optimisation of heat sinks cooled by natural
 * convection (Alexandersen, Sigmund & Aage, arXiv:1508.04596).
 *
 * The library evaluates, on one GPU, the residual of the stabilised weak form of
 * the composite steady Navier-Stokes-Brinkman / Boussinesq / convection-diffusion
 * equations (Sec. "Governing equations", Eqs. BoussDimless-a..c), discretised
 * with trilinear equal-order hexahedra on a structured grid with element-
 * constant design (Sec. "Finite element formulation"), SUPG/PSPG stabilised with
 * the element parameter tau of Appendix "Stabilisation parameters"; its
 * consistent Jacobian-vector product (including the variation of tau), the
 * transposed product and the design derivative for adjoint sensitivities; the
 * damped Newton / flexible GMRES state solve of Sec. "Numerical implementation";
 * and a continuous-batching solve server.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid:    nx*ny*nz cubic elements of edge h.  Element e = i + nx*(j + ny*k);
 *          node n = i + (nx+1)*(j + (ny+1)*k).  All of nx, ny, nz >= 1.
 * State:   node-major interleaved, x[5*n + f] with f = 0..4 = (u, v, w, p, T).
 *          n_dof = 5*(nx+1)*(ny+1)*(nz+1).
 * Design:  gamma[e] (1 = fluid, 0 = solid), s_elem[e] heat source, FP64.
 * Mask:    dof_mask[5*n + f] = 1 marks a prescribed DOF whose value in x is the
 *          Dirichlet value.  Prescribed rows are eliminated symmetrically:
 *          R_d = 0, (J v)_d = v_d, (J^T w)_d = w_d, and directions are gathered
 *          with their prescribed entries set to 0 (J = [[J_ff, 0], [0, I]]).
 * Memory:  every array argument of fe_* / newton_solve is a DEVICE pointer owned
 *          by the caller; the library reads or writes it during the call (in
 *          stream order) and never keeps or frees it.  Outputs are overwritten,
 *          never accumulated.  Inputs are not modified.  The problem handle owns
 *          its workspace, released by fe_problem_destroy.
 * Streams: calls are ordered on the given stream (0 = the null stream).
 *          newton_solve and fe_adjoint_solve make host decisions and therefore
 *          synchronise that stream before they return.
 * Errors:  0 = FE_OK; > 0 non-fatal states; < 0 errors.  No exception crosses
 *          the ABI; fe_last_error() returns a thread-local message for the last
 *          failing call on the calling thread.
 * Threads: a problem handle must not be used by two threads at once.
 */
#ifndef FE_H
#define FE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    FE_OK = 0,
    FE_PENDING = 1,        /* serve_poll: request not finished yet */
    FE_NOT_CONVERGED = 2,  /* solver stopped at its iteration limit; report filled */
    FE_EINVAL = -1,        /* bad argument: null pointer, bad size, unknown ticket */
    FE_ENOMEM = -2,        /* device or host allocation failed */
    FE_EHIP = -3,          /* a HIP runtime call failed */
    FE_ENAN = -4,          /* NaN or Inf met in a residual or Krylov norm */
    FE_ESTATE = -5         /* handle in a state that does not allow the call */
};

typedef struct { int32_t nx, ny, nz; double h; } fe_grid;

/* Dimensionless parameters (Sec. "Governing equations" and Eqs. conducint,
 * alphaint): Prandtl and Grashof numbers, conductivity ratio C_k = k_f/k_s,
 * conductivity convexity q_f, maximum impermeability alpha_bar and its convexity
 * q_alpha, unit gravity direction e^g.  The buoyancy coefficient is Gr*Pr^2. */
typedef struct { double Pr, Gr, Ck, qf, alpha_max, q_alpha; double eg[3]; } fe_phys;

typedef enum { FE_FP64 = 0, FE_FP32 = 1 } fe_prec;

typedef struct fe_problem fe_problem;

/* Create a problem on the current device.  dof_mask: device uint8[n_dof] as
 * above, copied into the handle (NULL: nothing prescribed).  Returns FE_EINVAL
 * for non-positive sizes or h <= 0, FE_ENOMEM / FE_EHIP on device failures. */
int fe_problem_create(const fe_grid *grid, const fe_phys *phys, const uint8_t *dof_mask,
                      fe_problem **out);
int fe_problem_destroy(fe_problem *p);
/* Replace the physical parameters of an existing handle (e.g. Gr continuation). */
int fe_problem_set_phys(fe_problem *p, const fe_phys *phys);
int64_t fe_problem_ndof(const fe_problem *p);

/* R(x; gamma, s): residual of the stabilised weak form, prescribed rows 0.
 * x: FP64[n_dof]; gamma, s_elem: FP64[n_el]; r: FP64[n_dof]. */
int fe_residual(fe_problem *p, const double *x, const double *gamma, const double *s_elem,
                double *r, hipStream_t stream);

/* jv = J(x) v: the exact directional derivative of R (consistent Jacobian,
 * Sec. "Finite element formulation": the variation of tau with the element
 * velocity vector, Appendix "Stabilisation parameters", is included).
 * prec = FE_FP64: x, v, jv are double*.  prec = FE_FP32: x, v, jv are float*;
 * arithmetic and accumulation in FP32 (gamma and s_elem stay FP64 inputs). */
int fe_jvp(fe_problem *p, fe_prec prec, const void *x, const double *gamma, const double *s_elem,
           const void *v, void *jv, hipStream_t stream);

/* Batched J v over a table of problems (Sec. "Finite element formulation", as
 * fe_jvp).  fe_jvp_batch_create copies to device memory a table with, for
 * each of the n problems probs[i], its geometry, parameters and the device
 * pointers x[i], gamma[i], s_elem[i], v[i], jv[i] (host arrays of n pointers;
 * x, v, jv of precision prec, gamma and s_elem FP64), plus the workgroup
 * offsets of the problems' concatenated tile and node index spaces.
 * fe_jvp_batch_run then computes jv_i = J_i(x_i) v_i for all i with ONE launch
 * of the element pass and ONE of the shared-node pass.  Per problem the
 * arithmetic is fe_jvp's, so jv_i is bitwise what fe_jvp(probs[i], ...) gives.
 * The problems must be distinct (each owns its tile-face work buffer) and
 * outlive the batch; the vectors are read and written when run executes.
 * FE_EINVAL for n < 1, a NULL or repeated problem or a NULL pointer. */
typedef struct fe_batch fe_batch;
int fe_jvp_batch_create(int n, fe_problem *const *probs, fe_prec prec, const void *const *x,
                        const double *const *gamma, const double *const *s_elem,
                        const void *const *v, void *const *jv, fe_batch **out);
int fe_jvp_batch_run(fe_batch *b, hipStream_t stream);
int fe_jvp_batch_destroy(fe_batch *b);

/* Element-pass timer of fe_jvp (instrumentation; it changes no result).
 * fe_kernel_timer(p, 1) clears the record and starts timing: every later
 * fe_jvp on p records a pair of HIP events on its stream, right before and
 * right after its element-pass kernel (the tile kernel; the shared-node pass
 * that follows is not inside the pair).  fe_kernel_timer(p, 0) stops timing.
 * fe_kernel_timer_read waits for the last recorded pair, writes the summed
 * element-pass time in milliseconds and the number of timed launches, and
 * clears the record.  Events are created on first use and kept by the handle
 * (one pair per launch between reads).  FE_EINVAL for NULL arguments. */
int fe_kernel_timer(fe_problem *p, int enable);
int fe_kernel_timer_read(fe_problem *p, double *elem_ms, int64_t *launches);

/* jtw = J(x)^T w, the exact transpose of fe_jvp's operator, evaluated element by
 * element in reverse mode with every element quantity recomputed from x. */
int fe_adjoint_jtvp(fe_problem *p, fe_prec prec, const void *x, const double *gamma,
                    const double *s_elem, const void *w, void *jtw, hipStream_t stream);

/* g_elem[e] = lambda^T dR/dgamma_e (FP64[n_el]); the material interpolation of
 * Eqs. conducint / alphaint and the design derivative of tau enter through
 * alpha'(gamma_e) and K'(gamma_e).  Prescribed entries of lambda are ignored. */
int fe_dR_dgamma(fe_problem *p, const double *x, const double *gamma, const double *s_elem,
                 const double *lambda, double *g_elem, hipStream_t stream);

/* Thermal compliance f = integral over the source of s*T (Sec. "Optimisation
 * problem"), evaluated exactly for trilinear T: f = sum_e s_e h^3/8 sum_a T_a.
 * f_host: host double (may be NULL); dfdx: device FP64[n_dof] or NULL, receives
 * df/dx with prescribed entries 0.  Synchronises the stream when f_host != NULL. */
int fe_compliance(fe_problem *p, const double *x, const double *s_elem, double *f_host,
                  double *dfdx, hipStream_t stream);

typedef struct {
    double rtol_newton;     /* stop when |R|_2 <= rtol_newton |R(x0)|_2 (default 1e-8) */
    double rtol_lin;        /* FGMRES relative tolerance per Newton step (default 1e-5) */
    int max_newton;         /* default 50 */
    int restart;            /* FGMRES restart length m, 1..64 (default 60) */
    int max_lin;            /* Krylov iterations per linear solve (default 3000) */
    int n_refine;           /* mixed mode: iterative-refinement sweeps (default 3) */
    fe_prec krylov_op_prec; /* FE_FP64, or FE_FP32 for FP32 J v and preconditioner */
    double ls_lambda_min;   /* lower clamp of the line-search factor (default 0.05) */
    int verbose;            /* 0 silent, 1 one line per Newton step on stderr */
    int precond;            /* FE_PC_AUTO (default), FE_PC_BJACOBI or FE_PC_MULTIGRID */
    int mg_nu;              /* multigrid: smoothing sweeps before the coarse-grid correction
                               (default 2; the first is x = omega D^-1 b) */
    double mg_omega;        /* multigrid: block-Jacobi damping (default 0.6) */
    double atol_newton;     /* also stop when |R|_2 <= atol_newton (default 0; for warm starts) */
    int ramp_steps;         /* recovery when Newton fails from the given vector (Sec. "Solving the
                               non-linear system"): restart from it and solve ramp_steps problems
                               with the heat source scaled by k/ramp_steps, k = 1..ramp_steps, each
                               warm-started from the previous one; the last one is held to the
                               original tolerance.  0 (default) = off */
    int mg_assembled_nodes; /* multigrid: levels above the coarsest with at most this many nodes
                               apply their operator as an assembled 27-point block stencil (built
                               from element Jacobians once per Newton step) instead of the
                               matrix-free element pass; -1 (default) = 10000, 0 = none */
    int mg_nu_post;         /* multigrid: smoothing sweeps after the coarse-grid correction
                               (default 1; -1 = mg_nu) */
    fe_prec pc_prec;        /* preconditioner precision with the FP64 operator: FE_FP64
                               (default) or FE_FP32.  FE_FP32 applies the block-Jacobi or
                               multigrid preconditioner in FP32 (blocks, stencils and smoothing
                               from the FP32 state, as in mixed mode) while the Krylov operator,
                               basis and residuals stay FP64.  Flexible GMRES admits any
                               preconditioner (Sec. "Solving the linear systems"), so the
                               solution meets the same FP64 tolerance; only the iteration count
                               can change.  Ignored when krylov_op_prec = FE_FP32 (the
                               preconditioner is FP32 there already); also used by
                               fe_adjoint_solve and by the batched server's lockstep engine. */
    int mg_coarse_reuse;    /* preconditioner set-up kept from one Newton step to the next once
                               the previous step has cut |R| at least 100-fold (the state then
                               changes little; flexible GMRES admits the preconditioner formed at
                               the earlier state): 2 (default) keeps all of it (the nodal blocks
                               and assembled stencils of every level, the coarse levels' states
                               and the coarsest factorisation); 1 keeps the coarsest level's
                               factorisation only (no probing, host factorisation or inverse);
                               0 rebuilds everything every Newton step.  Every Newton solve (each
                               heat-source ramping stage included) and every adjoint solve builds
                               its set-up anew at its start. */
} fe_solve_opts;

/* Preconditioners of the Krylov solves: nodal 5x5 block-Jacobi, or a matrix-free
 * geometric multigrid V-cycle (Sec. "Solving the linear systems") whose levels
 * rediscretise the operator on grids with half the elements per direction,
 * with damped block-Jacobi smoothing and a direct solve on the coarsest level.
 * FE_PC_AUTO (the default) takes multigrid whenever the grid has at least two
 * levels: element counts are halved while they stay even (or, where an odd
 * count stops that early, rounded up with the coarse grid overhanging by half
 * an element) until the coarse problem is small enough for the direct solve;
 * grids with fewer than 4 elements along a direction before that (thin slabs)
 * get block-Jacobi. */
enum { FE_PC_AUTO = 0, FE_PC_BJACOBI = 1, FE_PC_MULTIGRID = 2 };

typedef struct {
    int newton_its, lin_its_total, status;  /* status: FE_OK / FE_NOT_CONVERGED / error */
    double res0, res_final, lambda_last;
    double t_total_s;                       /* wall time of the call */
    double t_jv_s, t_prec_s, t_orth_s, t_res_s, t_setup_s; /* stream time per phase */
    int lin_its[64];                        /* Krylov iterations of the first 64 Newton steps */
    double res_hist[65];                    /* |R| after each Newton step, [0] = |R(x0)| */
    int precond;                            /* preconditioner used (FE_PC_BJACOBI / FE_PC_MULTIGRID) */
    int mg_levels;                          /* multigrid levels (0 without multigrid) */
    int ramp_stages;                        /* heat-source ramping stages run (0: none needed) */
} fe_solve_report;

/* Fill opts with the defaults listed above. */
void fe_solve_opts_default(fe_solve_opts *opts);

/* Damped Newton (Sec. "Solving the non-linear system"): each step solves
 * J delta = -R with right-preconditioned flexible GMRES (Sec. "Solving the
 * linear systems") with the preconditioner opts->precond selects (FE_PC_AUTO by
 * default: the multigrid V-cycle, or nodal 5x5 block-Jacobi where the grid gives
 * no hierarchy), Gram-Schmidt, Hessenberg and Givens in FP64; then the damping
 * factor is the minimiser of a
 * quadratic fitted to |R|^2 at 0, 1/2 and 1 times the step.  x_inout: device
 * FP64[n_dof], the initial vector on entry (its prescribed entries hold the
 * Dirichlet values), the solution on exit.  With krylov_op_prec = FE_FP32 the
 * Krylov operator and preconditioner run in FP32 and the linear residual is
 * refined with FP64 J v.  Returns FE_OK, FE_NOT_CONVERGED (x_inout holds the
 * last iterate) or an error; report may be NULL. */
int newton_solve(fe_problem *p, const double *gamma, const double *s_elem, double *x_inout,
                 const fe_solve_opts *opts, fe_solve_report *report, hipStream_t stream);

/* Adjoint solve J(x)^T lambda = rhs with FGMRES on fe_adjoint_jtvp's operator,
 * preconditioned by the transpose of the state solve's preconditioner: with
 * FE_PC_AUTO (default) the transposed multigrid V-cycle (D^T smoothing, J^T on
 * every level, transposed coarse solve), else transposed block-Jacobi; rtol_lin
 * of opts applies.  All arrays device FP64. */
int fe_adjoint_solve(fe_problem *p, const double *x, const double *gamma, const double *s_elem,
                     const double *rhs, double *lambda, const fe_solve_opts *opts,
                     fe_solve_report *report, hipStream_t stream);

/* Nodal 5x5 diagonal blocks of J(x) (the block-Jacobi preconditioner of the
 * linear solves before inversion): D[25*n + 5*f + g] = dR_{n,f}/dx_{n,g}, with
 * the identity in place of prescribed rows and columns.  D: device FP64[25*n_nodes]. */
int fe_block_diagonal(fe_problem *p, const double *x, const double *gamma, const double *s_elem,
                      double *D, hipStream_t stream);
/* The same blocks evaluated in FP32 arithmetic from an FP32 state x (device
 * float[n_dof]) into D (device float[25*n_nodes]): the blocks that a
 * mixed-precision Newton step inverts in FP32 for its FP32 smoother (Sec.
 * "Solving the linear systems"; the preconditioner's precision does not enter
 * the FP64 residual that decides convergence). */
int fe_block_diagonal_fp32(fe_problem *p, const float *x, const double *gamma,
                           const double *s_elem, float *D, hipStream_t stream);

/* The assembled Jacobian J(x) of a small problem, dense and row-major:
 * J_host[i * n_dof + j] = dR_i/dx_j (host FP64[n_dof * n_dof], written in
 * full), with the identity in place of prescribed rows and columns: the matrix
 * whose product with a vector fe_jvp evaluates (Sec. "Finite element
 * formulation", consistent Jacobian).  Built on the device from the element
 * Jacobians by 135 colour-by-field probing products, then expanded on the
 * host; this is how the multigrid preconditioner obtains its coarsest-level
 * matrix.  FE_EINVAL for NULL arguments or n_dof > FE_DENSE_MAX_DOF; synchronises
 * the stream. */
#define FE_DENSE_MAX_DOF 20000
int fe_jacobian_dense(fe_problem *p, const double *x, const double *gamma, const double *s_elem,
                      double *J_host, hipStream_t stream);

/* Damping factor of the quadratic line search for scripted residual norms
 * phi(l) = |R(x + l delta)|^2 at l = 0, 1/2, 1 (host-only helper). */
double fe_line_search_lambda(double phi0, double phi_half, double phi1, double lambda_min);

/* Device bytes newton_solve allocates for a grid (for memory admission),
 * including the problem handle's own buffers; opts NULL = defaults. */
int64_t fe_solve_footprint_bytes(const fe_grid *grid, const fe_solve_opts *opts);

/* ---- continuous-batching server ------------------------------------------
 * Requests (grid, parameters, design, source, options) are copied in at
 * submit and queued.  serve_create allocates one device arena of
 * hbm_budget_bytes and starts max_active (1..64) worker threads, each with its
 * own HIP stream.  Workers admit queued requests in arrival order: the head
 * request is admitted as soon as the arena has a free contiguous block of its
 * footprint (fe_solve_footprint_bytes plus its design, source and state), and
 * its whole working set is carved from that block, so requests never compete
 * for memory while running and no device allocation happens after
 * serve_create.  Running requests' kernels overlap on the device; each request
 * runs the same kernels as a standalone newton_solve, so its result does not
 * depend on what else runs.  A finished request returns its block at once.
 * A request whose footprint exceeds the arena is refused at submit
 * (FE_ENOMEM).  Walls (u, v, w, T = 0 on every boundary node) and the pressure
 * pin at node 0 are applied to every request; the initial state is 0 unless
 * given (serve_submit_x0). */
typedef struct fe_server fe_server;
int serve_create(size_t hbm_budget_bytes, int max_active, fe_server **out);
/* flags = FE_SERVE_BATCHED: the same server, but the requests' linear solves
 * (one per Newton step: FGMRES with the multigrid V-cycle) run in lockstep on
 * engine threads -- each FGMRES step launches every kernel once over a device
 * table of the engine's running requests (concatenated element and DOF index
 * spaces, per-request segmented reductions) -- while the workers keep the
 * set-up and line search of their requests.  Requests go to one of four
 * engines by their DOF count (below 50,000 / 150,000 / 450,000 / above), each
 * with its own stream, so that requests batch with requests of similar size.
 * Requests that leave fe_solve_opts.mg_assembled_nodes at its default (-1)
 * get a limit of 1,000 nodes for assembled multigrid levels in this mode
 * (over a batch the element pass moves far fewer bytes than a stencil).  max_active may then be up to 256.
 * A request's result is the same alone and in any mix (its arithmetic does not
 * depend on the batch); it can differ from the default mode's in the last bits
 * (the batched reductions chunk the vectors differently).  Requests whose
 * grid has no multigrid hierarchy use their worker's one-problem FGMRES. */
#define FE_SERVE_BATCHED 1
int serve_create_ex(size_t hbm_budget_bytes, int max_active, int flags, fe_server **out);
/* Batched mode: lockstep steps run and batched launches issued so far (0 in
 * the default mode). */
int serve_engine_stats(fe_server *s, uint64_t *steps, uint64_t *launches);
/* gamma_host, s_host: host FP64[n_el]; copied.  Returns at once with a ticket. */
int serve_submit(fe_server *s, const fe_grid *grid, const fe_phys *phys, const double *gamma_host,
                 const double *s_host, const fe_solve_opts *opts, uint64_t *ticket);
/* As serve_submit, with an initial vector for Newton: x0_host, host
 * FP64[n_dof] (copied; NULL: zero), typically the solution of the previous
 * design of an optimisation (Sec. "Solving the non-linear system": the
 * previous design iteration's state is the initial vector).  Its prescribed
 * entries must hold the Dirichlet values (0 on the walls). */
int serve_submit_x0(fe_server *s, const fe_grid *grid, const fe_phys *phys,
                    const double *gamma_host, const double *s_host, const double *x0_host,
                    const fe_solve_opts *opts, uint64_t *ticket);
/* FE_PENDING while queued or running; otherwise the request's final status
 * (FE_OK, FE_NOT_CONVERGED or an error) with x_host_out (host FP64[n_dof], may
 * be NULL) and report filled.  A finished ticket can be polled again. */
int serve_poll(fe_server *s, uint64_t ticket, double *x_host_out, fe_solve_report *report);
/* Timestamps (seconds, server clock) of submit, admit and completion. */
int serve_times(fe_server *s, uint64_t ticket, double *t_submit, double *t_admit, double *t_done);
/* Error message of a finished request that failed ("" otherwise); the string
 * stays valid until serve_destroy. */
const char *serve_error(fe_server *s, uint64_t ticket);
int serve_destroy(fe_server *s);

/* ---- optimisation loop (Sec. "Optimisation problem", Sec. "Continuation scheme") ----
 *
 * PDE density filter.  -r^2 lap(psi) + psi = gamma on the box grid with zero
 * normal derivative, r = radius / (2 sqrt 3); psi trilinear on the nodes, the
 * element design value a constant load; the filtered element value is the mean
 * of psi over the element's nodes.  apply: out = F in; apply_transpose:
 * out = F^T in (element vectors, device FP64[n_el]; in and out may alias).
 * The nodal solve is conjugate gradients with Jacobi preconditioning to a
 * relative residual of 1e-12 (FE_NOT_CONVERGED after 5000 iterations). */
typedef struct fe_filter fe_filter;
int fe_filter_create(const fe_grid *grid, double radius, fe_filter **out);
int fe_filter_apply(fe_filter *f, const double *in, double *out, hipStream_t stream);
int fe_filter_apply_transpose(fe_filter *f, const double *in, double *out, hipStream_t stream);
int fe_filter_iterations(const fe_filter *f); /* CG iterations of the last call */
int fe_filter_destroy(fe_filter *f);

/* Method of moving asymptotes for min f0(x) s.t. f1(x) <= 0, xmin <= x <= xmax,
 * n variables, with a move limit (fraction of xmax - xmin).  update: one
 * iteration from x (device FP64[n], overwritten with the new iterate) given
 * the gradients df0, df1 (device FP64[n]) and the constraint value f1;
 * lambda_out (host, may be NULL) receives the subproblem's multiplier.  The
 * handle keeps the asymptotes and the last two iterates between calls. */
typedef struct fe_mma fe_mma;
int fe_mma_create(int64_t n, double xmin, double xmax, double move, fe_mma **out);
int fe_mma_update(fe_mma *m, double *x, const double *df0, double f1, const double *df1,
                  double *lambda_out, hipStream_t stream);
int fe_mma_destroy(fe_mma *m);

/* Design loop: minimise the thermal compliance subject to
 * mean over the design domain of (1 - gamma~) <= vf, gamma~ = filtered design
 * on the design domain and gamma_fixed elsewhere.  Each design iteration
 * filters, solves the state warm-started from the previous state (with
 * heat-source ramping on failure), evaluates the compliance, solves the
 * adjoint, forms the design sensitivities, takes them through the filter
 * transpose and updates the design by MMA (objective scaled by its first
 * value).  Continuation: n_steps steps of iters_per_step[k] iterations with
 * the material parameters (q_f, q_alpha, alpha_max)[k]. */
typedef struct {
    int n_steps;               /* 1..5 (default 5) */
    int iters_per_step[5];     /* default 100 each */
    double q_f[5], q_alpha[5], alpha_max[5]; /* default: the paper's five steps */
    double vf;                 /* volume fraction (default 0.05) */
    double filter_radius;      /* R in element sizes (default 2.5) */
    double move;               /* MMA move limit (default 0.2) */
    fe_solve_opts state;       /* state solves (default rtol_newton 1e-4, ramp_steps 4) */
    fe_solve_opts adjoint;     /* adjoint solves (default rtol_lin 1e-6) */
} fe_topopt_opts;
typedef struct {
    int iter, step;            /* design iteration, continuation step */
    double f, f_scaled, g;     /* compliance, compliance / first compliance, constraint */
    double change;             /* largest design change of the MMA update */
    double lambda_mma;         /* MMA subproblem multiplier */
    int newton_its, lin_its, adj_its, ramp_stages;
    double t_state_s, t_adjoint_s, t_total_s;
} fe_topopt_record;
typedef struct fe_topopt fe_topopt;
void fe_topopt_opts_default(fe_topopt_opts *opts);
/* p: the state problem (its mask and grid; its material parameters are set by
 * the continuation); design_mask: device uint8[n_el], 1 = design element;
 * gamma_fixed, s_elem: device FP64[n_el] (gamma off the design domain, heat
 * source), borrowed until fe_topopt_destroy. */
int fe_topopt_create(fe_problem *p, const uint8_t *design_mask, const double *gamma_fixed,
                     const double *s_elem, const fe_topopt_opts *opts, fe_topopt **out);
/* f, g and (if not NULL) their gradients with respect to the design values
 * rho (device FP64[n_el], entries off the design domain ignored; gradients 0
 * there) at rho; x: device FP64[n_dof], initial vector in, state out. */
int fe_topopt_evaluate(fe_topopt *t, const double *rho, double *x, double *f, double *g,
                       double *dfdrho, double *dgdrho, fe_topopt_record *rec, hipStream_t stream);
/* One design iteration: evaluate at rho, then rho <- MMA update (design entries). */
int fe_topopt_step(fe_topopt *t, double *rho, double *x, fe_topopt_record *rec, hipStream_t stream);
/* The whole continuation; hist (host, cap records, may be NULL), n_done: iterations run. */
int fe_topopt_run(fe_topopt *t, double *rho, double *x, fe_topopt_record *hist, int cap,
                  int *n_done, hipStream_t stream);
int fe_topopt_destroy(fe_topopt *t);

/* J v without device allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Computes exactly what fe_jvp computes on a problem
 * created with the same grid, phys and dof_mask (same kernels, bitwise the
 * same result), but takes the grid, parameters and mask directly instead of a
 * problem handle: its two work buffers (per-node mask bits and tile-face
 * partial sums) live in a static device array of FE_NOALLOC_SCRATCH_BYTES
 * that every GPU the library runs on holds until the process ends.
 *   dof_mask: device uint8[n_dof] (1 = prescribed; NULL = none), as for
 *   fe_problem_create; x, v, jv: device FP64 or FP32 [n_dof] per prec; gamma,
 *   s_elem: device FP64[n_el].  Stream-ordered, no synchronisation.
 * Grids whose scratch need (fe_jvp_noalloc_scratch_bytes) exceeds
 * FE_NOALLOC_SCRATCH_BYTES (64 MiB: FP64 grids up to about 4,000 8x8x4-element
 * tiles, e.g. 96^3) are refused with FE_EINVAL.  Every call on one GPU uses
 * the same array: calls that overlap on one GPU (different streams or host
 * threads without ordering between them) race and give wrong results. */
#define FE_NOALLOC_SCRATCH_BYTES (64ll << 20)
int64_t fe_jvp_noalloc_scratch_bytes(const fe_grid *grid, fe_prec prec);
int fe_jvp_noalloc(const fe_grid *grid, const fe_phys *phys, fe_prec prec, const uint8_t *dof_mask,
                   const void *x, const double *gamma, const double *s_elem, const void *v,
                   void *jv, hipStream_t stream);

const char *fe_last_error(void);
const char *fe_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FE_H */
